"""Planted mistakes in the oracle are caught by its pins.

Each case copies the oracle's C source, plants one mistake of the kind a
transcription of the paper's equations makes (a flipped sign, a dropped term,
a transposed index), compiles the copy with gcc into a temporary directory and
runs, against that copy, the pin that must catch it.  The reference network
of the learned warm start (numpy) is treated the same way: a mutated copy of
its source is loaded as a module of its own.  The oracle itself is never
modified; control cases run the same pins on unmodified copies.
"""
import importlib.util
import os
import subprocess

import pytest

import oracle
import test_gnn_ref as gnn_pins
import test_oracle_pins as pins
import test_oracle_verifier as vpins
import test_oracle_joint_pins as jpins
import test_oracle_polarfree_pins as ppins
import test_oracle_wrench_pins as wpins

ORACLE_DIR = os.path.dirname(os.path.abspath(oracle.__file__))
SRC = os.path.join(ORACLE_DIR, "mabd_oracle.c")
GNN_SRC = os.path.join(ORACLE_DIR, "gnn_ref.py")


def chain_lu():
    pins.test_solvers_match_dense_kkt_lu(*pins.small_assemblies()[0])


def tree_lu():
    pins.test_solvers_match_dense_kkt_lu(*pins.small_assemblies()[1])


def stretch_modes():
    pins.test_stretch_mode_is_implicit_euler_oscillator(0, 1e6, 0.0)
    pins.test_stretch_mode_is_implicit_euler_oscillator(1, 1e6, 0.3)


def hinge_pins():
    pins.test_hinge_blocks_off_axis_rotation()
    pins.test_pendulum_converges_to_elliptic_solution(True)
    pins.test_hinge_second_point_rows_are_normal_to_the_axis()


def verifier_pins():
    vpins.test_exact_solution_has_zero_residual()
    for sc in (0.0, 0.5, 2.0, -1.0):
        vpins.test_scaled_multipliers_give_closed_form_dual_residual(sc)
    vpins.test_perturbed_step_matches_brute_force_residual()
    vpins.test_primal_residual_is_relative_to_the_free_increment()
    vpins.test_post_step_constraints()


def wrench_pins():
    wpins.test_twist_of_rigid_spin()
    wpins.test_ball_joint_wrench_is_the_anchor_point_force()
    wpins.test_internal_joint_forces_cancel()
    wpins.test_hanging_box_carries_its_weight()


def joint_pins():
    jpins.test_universal_kinematics()
    jpins.test_prismatic_kinematics()
    for t in (1, 2, 3):
        jpins.test_gradient_away_from_rest(t)
    for name, asm in jpins.mixed_assemblies():
        jpins.test_mixed_joints_match_dense_kkt_lu(name, asm)
    jpins.test_vertical_slider_falls_freely()


def polar_free_pins():
    ppins.test_equals_polar_step_for_rotations()
    ppins.test_equals_polar_step_for_scaled_rotations()
    ppins.test_free_fall_closed_form()


# (name, text in the oracle, planted replacement, pin that must fail)
MUTANTS = [
    # Eq. variation_energy: gravity enters the force with its own sign
    ("gravity_sign", "m * s->gravity[r] : 0.0", "-m * s->gravity[r] : 0.0",
     pins.test_free_fall_closed_form),
    # implicit Euler: the momentum term M qdot_n / h dropped
    ("velocity_term_dropped", "f[a] = M * qdn[a] / h - M", "f[a] = 0.0 * qdn[a] / h - M",
     pins.test_free_fall_closed_form),
    # the elastic force is minus the energy gradient
    ("elastic_force_sign", "? -V * F[r * 3 + c] : 0.0", "? V * F[r * 3 + c] : 0.0", stretch_modes),
    # Eq. polar: (A^T A)^{-1/2}, not (A^T A)^{-1}
    ("polar_sqrt_dropped", "/ sqrt(w[k]);", "/ w[k];", pins.test_polar_against_svd),
    # Eq. abd_dof: J(p) = [p^T (x) I3, I3], not [I3 (x) p^T, I3]
    ("jacobian_transposed", "J[r * 12 + 3 * c + r] = p[c];", "J[r * 12 + 3 * r + c] = p[c];",
     pins.test_ball_constraints_exact_every_step),
    # footnote of Eq. kkt: the dual right-hand side carries the constraint value C
    ("dual_rhs_constraint_dropped", "r[i] = d->C[5 * k + i];", "r[i] = 0.0 * d->C[5 * k + i];",
     pins.test_ball_constraints_exact_every_step),
    # Eq. chain-btd, forward elimination: D_i - B^T D^{-1} B
    ("thomas_schur_sign", "Dh[25 * i + e] -= Y[e];", "Dh[25 * i + e] += Y[e];", chain_lu),
    # back-substitution with the coupling block transposed
    ("thomas_back_transposed", "x[a] -= Bm[25 * i + a * rk[i + 1] + c] * xn[c];",
     "x[a] -= Bm[25 * i + c * r0 + a] * xn[c];", chain_lu),
    # tree condensation: the child's G^T S^{-1} G update dropped
    ("tree_condensed_block_dropped", "Hh[144 * p + e] += U[e];", "Hh[144 * p + e] += 0.0 * U[e];",
     tree_lu),
    # tree condensation: the condensed right-hand side with the wrong sign
    ("tree_condensed_rhs_sign", "fh[12 * p + i] -= acc;", "fh[12 * p + i] += acc;", tree_lu),
    # PCG on the dual (closed loops): the recursive residual r - alpha S p
    ("pcg_residual_update_sign", "res[i] -= alpha * Ap[i];", "res[i] += alpha * Ap[i];",
     pins.test_pcg_matches_direct_on_small_lattice),
    # PCG: the iterate moves along +alpha p
    ("pcg_iterate_update_sign", "lam[i] += alpha * p[i];", "lam[i] -= alpha * p[i];",
     pins.test_pcg_matches_direct_on_small_lattice),
    # Sec. 4.3 hinge frame: the second-order Rodrigues term with the wrong sign
    ("hinge_frame_sign", "+ K2[i] / (1.0 + a[1]);", "- K2[i] / (1.0 + a[1]);", hinge_pins),
    # Eq. r_gradient, A-linearised: the rotation term with A's indices transposed
    ("hinge_rotation_term_transposed", "Ga[i * 12 + 3 * l + kk] += dRh[comp * 3 + l] * dm[kk];",
     "Ga[i * 12 + 3 * kk + l] += dRh[comp * 3 + l] * dm[kk];",
     vpins.test_hinge_gradient_along_rigid_motions_away_from_rest),
    # the verifier: a dual residual that reads zero
    ("verifier_rho_d_zeroed", "*rho_d = nr > 0.0 ? sqrt(nd / nr) : sqrt(nd);",
     "*rho_d = 0.0 * (nr > 0.0 ? sqrt(nd / nr) : sqrt(nd));", verifier_pins),
    # the verifier: a primal residual that reads zero
    ("verifier_rho_p_zeroed", "*rho_p = nf > 0.0 ? sqrt(np / nf) : sqrt(np);",
     "*rho_p = 0.0 * (nf > 0.0 ? sqrt(np / nf) : sqrt(np));", verifier_pins),
    # the verifier: C dropped from the dual residual G dq + C
    ("verifier_constraint_dropped", "for (int a = 0; a < rk; ++a) rd[a] = d->C[5 * k + a];",
     "for (int a = 0; a < rk; ++a) rd[a] = 0.0 * d->C[5 * k + a];", verifier_pins),
    # the verifier: r_p not mapped through H^{-1}
    ("verifier_rp_unscaled", "    chol_solve(12, d->L + 144 * b, rp);\n    memcpy(hf",
     "    memcpy(hf", verifier_pins),
    # the verifier: the ball joints' post-step value reads zero
    ("verifier_cball_zeroed", "if (s->jtype[k] == 0) { if (v > *cball) *cball = v; }",
     "if (s->jtype[k] == 0) { if (v > *cball) *cball = 0.0 * v; }", verifier_pins),
    # Eq. module1-G-twist: the factor 1/2 of the angular velocity dropped
    ("twist_half_dropped", "o[0] += 0.5 * (a[1] * ad[2] - a[2] * ad[1]);",
     "o[0] += (a[1] * ad[2] - a[2] * ad[1]);", wrench_pins),
    # Eq. module2-E: E(A)^T with the cross product reversed (E instead of -E)
    ("wrench_moment_sign", "o[1] += a[2] * fc[0] - a[0] * fc[2];", "o[1] -= a[2] * fc[0] - a[0] * fc[2];",
     wrench_pins),
    # Eq. universal: the fourth row on the wrong local component of the frame
    ("universal_row_component", "{1, 3, 2}, {0, 0, 2}},  /* universal */",
     "{2, 3, 2}, {0, 0, 2}},  /* universal */", joint_pins),
    # Eq. prismatic: the anti-twist point placed along the frame's x instead of z
    ("prismatic_third_point", "if (type == 3) memcpy(da3, dRh + 6, sizeof da3);",
     "if (type == 3) memcpy(da3, dRh + 0, sizeof da3);", joint_pins),
    # Eq. prismatic: the axis rows compare b's second point with a's first
    ("prismatic_axis_rows", "{0, 3, 2}, {2, 3, 2}, {0, 4, 2}}}; /* prismatic */",
     "{0, 3, 0}, {2, 3, 2}, {0, 4, 2}}}; /* prismatic */", joint_pins),
    # Alg. 1: the forces taken to the body frame by A instead of A^T
    ("polar_free_force_untransposed", "for (int k = 0; k < 4; ++k) lenpres(A, 1, w + 3 * k, phi + 3 * k);",
     "for (int k = 0; k < 4; ++k) lenpres(A, 0, w + 3 * k, phi + 3 * k);", polar_free_pins),
    # Eq. len_preserving: the rescaling to the original length dropped
    ("polar_free_length_dropped", "for (int r = 0; r < 3; ++r) y[r] *= lx / ly;",
     "for (int r = 0; r < 3; ++r) y[r] *= 1.0;", polar_free_pins),
    # the joint force taken as +G^T lambda instead of -G^T lambda
    ("wrench_force_sign", "f[12 * (size_t)b + c] -= G[i * 12 + c] * lam[off + i];",
     "f[12 * (size_t)b + c] += G[i * 12 + c] * lam[off + i];", wrench_pins),
]


def build_copy(tmp_path, old=None, new=None):
    src = open(SRC).read()
    if old is not None:
        assert src.count(old) == 1, f"mutation site not unique: {old!r}"
        src = src.replace(old, new)
    path = tmp_path / "mabd_oracle.c"
    path.write_text(src)
    lib = tmp_path / "libmabd_oracle_copy.so"
    subprocess.check_call(["gcc", "-O2", "-march=x86-64-v3", "-std=c99", "-fPIC", "-shared",
                           "-I", ORACLE_DIR, "-o", str(lib), str(path), "-lm"])
    return str(lib)


def use_library(monkeypatch, path):
    monkeypatch.setattr(oracle, "LIB_PATH", path)
    monkeypatch.setattr(oracle, "_lib", None)


def test_unmodified_copy_passes_every_pin(tmp_path, monkeypatch):
    use_library(monkeypatch, build_copy(tmp_path))
    for pin in {id(m[3]): m[3] for m in MUTANTS}.values():
        pin()


@pytest.mark.parametrize("name,old,new,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(name, old, new, pin, tmp_path, monkeypatch):
    use_library(monkeypatch, build_copy(tmp_path, old, new))
    with pytest.raises((AssertionError, oracle.OracleError)):
        pin()


def gnn_all_pins():
    gnn_pins.test_energy_identity()
    gnn_pins.test_permutation_equivariance()
    gnn_pins.test_two_joint_message_by_hand()


# (name, text in the reference network, planted replacement)
GNN_MUTANTS = [
    ("encoder_relu_dropped", "h = np.maximum(self.x @ We + ce, 0.0)", "h = self.x @ We + ce"),
    ("layer_relu_dropped", "h = np.maximum(np.concatenate([h, n], axis=1) @ Wl + cl, 0.0)",
     "h = np.concatenate([h, n], axis=1) @ Wl + cl"),
    ("degree_norm_one_side", "self.norm = 1.0 / np.maximum(1.0, dga + dgb)",
     "self.norm = 1.0 / np.maximum(1.0, dga)"),
    ("message_own_state", "n[k] += m[b]", "n[k] += h[k]"),
    ("loss_linear_term_sign", "return (0.5 * d @ (self.S @ d) - self.rb @ d) / self.eref",
     "return (0.5 * d @ (self.S @ d) + self.rb @ d) / self.eref"),
    ("base_residual_sign", "self.rb = self.r - S @ self.lb", "self.rb = self.r + S @ self.lb"),
]


def load_gnn_copy(tmp_path, old=None, new=None):
    src = open(GNN_SRC).read()
    if old is not None:
        assert src.count(old) == 1, f"mutation site not unique: {old!r}"
        src = src.replace(old, new)
    path = tmp_path / "gnn_ref_copy.py"
    path.write_text(src)
    spec = importlib.util.spec_from_file_location("gnn_ref_copy", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_unmodified_network_copy_passes_every_pin(tmp_path, monkeypatch):
    monkeypatch.setattr(gnn_pins, "G", load_gnn_copy(tmp_path))
    gnn_all_pins()


@pytest.mark.parametrize("name,old,new", GNN_MUTANTS, ids=[m[0] for m in GNN_MUTANTS])
def test_planted_network_mistake_is_caught(name, old, new, tmp_path, monkeypatch):
    monkeypatch.setattr(gnn_pins, "G", load_gnn_copy(tmp_path, old, new))
    with pytest.raises(AssertionError):
        gnn_all_pins()
