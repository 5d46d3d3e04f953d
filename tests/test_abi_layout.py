"""The ctypes binding matches include/mabd.h exactly (CPU only).

* Every struct the binding mirrors has the header's fields, in order, with
  matching types, and the same size and field offsets as gcc gives the
  header's own definition (a small C program prints them).
* Every function the binding declares has the header's parameter and return
  types.
A mismatch in either would corrupt arguments silently at run time.
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "mabd.h")

SCALAR = {"double": ctypes.c_double, "float": ctypes.c_float, "int32_t": ctypes.c_int32,
          "int64_t": ctypes.c_int64, "uint32_t": ctypes.c_uint32, "uint64_t": ctypes.c_uint64}
PAIRS = {"mabd_bodies": "Bodies", "mabd_joints": "Joints", "mabd_options": "Options",
         "mabd_step_stats": "StepStats"}


def header():
    with open(HDR) as f:
        return re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)


def defines(txt):
    return {k: int(v) for k, v in re.findall(r"#define\s+(\w+)\s+(\d+)", txt)}


def structs(txt):
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(mabd_\w+)\s*;", txt, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = " ".join(decl.split())
            if not decl:
                continue
            m = re.match(r"(?:const\s+)?(\w+)\s*(.*)", decl)
            base, rest = m.group(1), m.group(2)
            for d in rest.split(","):
                d = d.strip()
                ptr = d.startswith("*")
                am = re.match(r"(\w+)\s*(?:\[(\w+)\])?$", d.lstrip("*").strip())
                fields.append((am.group(1), base, ptr, am.group(2)))
        out[name] = fields
    return out


def ctype_of(base, ptr, arr, defs):
    if ptr:
        return ctypes.c_char_p if base == "char" else ctypes.c_void_p
    t = SCALAR[base]
    return t * int(defs.get(arr, arr)) if arr else t


def same_type(a, b):
    if isinstance(a, type) and issubclass(a, ctypes.Array):
        return issubclass(b, ctypes.Array) and a._type_ is b._type_ and a._length_ == b._length_
    return a is b


def c_offsets(tmp_path, S):
    """sizeof and offsetof of every field, as gcc lays out the header's structs."""
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mabd.h"', "int main(void) {"]
    for cname in PAIRS:
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f in S[cname]:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    return {(a, b): int(c) for a, b, c in (ln.split() for ln in out.splitlines())}


def test_structs_match_the_header(tmp_path):
    import paper_2603_08079_amd as pk

    txt = header()
    defs, S = defines(txt), structs(txt)
    assert set(PAIRS) <= set(S)
    off = c_offsets(tmp_path, S)
    for cname, pyname in PAIRS.items():
        cls = getattr(pk, pyname)
        py = cls._fields_
        assert [f[0] for f in py] == [f[0] for f in S[cname]], cname
        for (fname, t), (_, base, ptr, arr) in zip(py, S[cname]):
            assert same_type(t, ctype_of(base, ptr, arr, defs)), (cname, fname)
            assert getattr(cls, fname).offset == off[(cname, fname)], (cname, fname)
        assert ctypes.sizeof(cls) == off[(cname, "sizeof")], cname


def functions(txt):
    out = {}
    for ret, name, params in re.findall(r"([\w\s\*]+?)\b(mabd_\w+)\s*\(([^)]*)\)\s*;", txt):
        ret = " ".join(ret.split())
        ps = [] if params.strip() in ("", "void") else [" ".join(p.split()) for p in params.split(",")]
        out[name] = (ret, ps)
    return out


def param_type(p):
    p = re.sub(r"^const\s+", "", p)
    base = p.split()[0]
    if "*" in p:
        return ctypes.c_char_p if base == "char" else ctypes.c_void_p
    return SCALAR[base]


def return_type(r):
    r = re.sub(r"^const\s+", "", r)
    if r == "void":
        return None
    if r in ("mabd_status", "int32_t"):
        return ctypes.c_int32
    if r.startswith("char") and "*" in r:
        return ctypes.c_char_p
    return SCALAR[r]


def test_functions_match_the_header():
    import paper_2603_08079_amd as pk

    L = pk.lib()
    F = functions(header())
    assert set(pk.EXPORTED) <= set(F)
    for name in pk.EXPORTED:
        ret, ps = F[name]
        fn = getattr(L, name)
        if name == "mabd_options_default":
            assert fn.restype is None
        else:
            assert fn.restype is return_type(ret), name
        assert fn.argtypes is not None and len(fn.argtypes) == len(ps), name
        for a, p in zip(fn.argtypes, ps):
            assert a is param_type(p), (name, p)
