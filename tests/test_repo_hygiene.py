"""Structural guarantees of the repository, checked on the CPU.

* The product path (the package and its HIP/C++ sources) never imports,
  links or calls the oracle: parity claims rest on that independence.
* The oracle shares no source with the GPU library.
* Nothing that is part of the repository reads the untracked `_work/` folder.
* Every profile summary states the rocprofv3 command that produced it.
"""
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2603_08079_amd")
WORK = re.compile(r"(?<![A-Za-z0-9_])_work\b")  # the folder, not e.g. max_workers


def files(pattern):
    return sorted(glob.glob(os.path.join(ROOT, pattern), recursive=True))


def text(path):
    with open(path, encoding="utf-8", errors="replace") as f:
        return f.read()


def test_product_path_never_touches_the_oracle():
    srcs = files("paper_2603_08079_amd/**/*.py") + files("paper_2603_08079_amd/csrc/*")
    assert srcs
    for p in srcs:
        t = text(p)
        assert not re.search(r"^\s*(import|from)\s+oracle\b", t, re.M), p
        assert "mabd_oracle" not in t and "libmabd_oracle" not in t, p
        assert "ora_" not in re.sub(r"[A-Za-z0-9_]ora_", "", t), p


def test_oracle_shares_no_source_with_the_gpu_library():
    for p in files("oracle/*.c") + files("oracle/*.h") + files("oracle/*.py"):
        t = text(p)
        assert "csrc" not in t and "paper_2603_08079_amd" not in t, p
        assert not re.search(r'#include\s+"\.\./', t), p


def test_nothing_committed_reads_the_work_folder():
    srcs = (files("*.py") + files("paper_2603_08079_amd/**/*.py") + files("paper_2603_08079_amd/csrc/*")
            + files("oracle/*") + files("mabd_inputs/*.py") + files("tests/*.py") + files("include/*.h"))
    for p in srcs:
        if os.path.abspath(p) == os.path.abspath(__file__) or not os.path.isfile(p):
            continue
        if p.endswith(".so"):
            continue
        assert not WORK.search(text(p)), p


def test_profiles_state_their_commands():
    profs = files("profiles/*.md")
    assert profs
    for p in profs:
        t = text(p)
        assert "rocprofv3 " in t, p
        assert not WORK.search(t), p
