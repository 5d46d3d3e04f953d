// Device-side small linear algebra for libmabd (gfx950).
//
// Conventions: 3x3 matrices are row-major double[9]; q per body is
// [a1; a2; a3; t] with A(r, c) = q[3c + r] (Sec. 3.1, Eq. abd_dof).
//
// The per-shape table `Hinv` holds the structured inverse of the constant
// single-body matrix Hbar = M_A / h^2 + Kbar_A (Eq. abd_final) for a box whose
// rest frame sits at its centre of mass.  There M_A = diag(Mbar) (x) I3 and
// Kbar_A couples only (A00, A11, A22) among themselves and each off-diagonal
// pair (A_rc, A_cr), so Hbar^{-1} is one 3x3 block, three 2x2 blocks and a
// translation scalar (20 doubles, built once per shape and time step).
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

#define DEV __device__ __forceinline__

namespace mabd {

// layout of one Hinv entry
//   [0]       h^2 / m                      (translation block)
//   [1..6]    (A00,A11,A22) inverse, symmetric: 00 01 02 11 12 22
//   [7..15]   PD(r,c): diagonal inverse entry of off-diagonal element A_rc
//             (3x3 row-major, diagonal slots unused)
//   [16..18]  PX for pairs {A_01,A_10}, {A_02,A_20}, {A_12,A_21}
enum { HI_T = 0, HI_D = 1, HI_PD = 7, HI_PX = 16 };

DEV int pair_slot(int r, int c) {  // r != c
  int s = r + c;                   // (0,1)->1 (0,2)->2 (1,2)->3
  return s - 1;
}

DEV double sym3(const double *S6, int r, int c) {
  // S6 = 00 01 02 11 12 22
  int a = r < c ? r : c, b = r < c ? c : r;
  int idx = a == 0 ? b : (a == 1 ? 2 + b : 5);
  return S6[idx];
}

// y = Hbar^{-1} x for a 12-vector x (structured apply, ~40 flops), in the
// precision of x
template <typename real>
DEV void hinv_apply(const double *T, const real *x, real *y) {
  const real ht = real(T[HI_T]);
  y[9] = ht * x[9];
  y[10] = ht * x[10];
  y[11] = ht * x[11];
  const double *D = T + HI_D;
  const real x0 = x[0], x4 = x[4], x8 = x[8];
  y[0] = real(D[0]) * x0 + real(D[1]) * x4 + real(D[2]) * x8;
  y[4] = real(D[1]) * x0 + real(D[3]) * x4 + real(D[4]) * x8;
  y[8] = real(D[2]) * x0 + real(D[4]) * x4 + real(D[5]) * x8;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (r == c) continue;
      const int i1 = 3 * c + r, i2 = 3 * r + c;  // A_rc and its partner A_cr
      y[i1] = real(T[HI_PD + 3 * r + c]) * x[i1] + real(T[HI_PX + pair_slot(r, c)]) * x[i2];
    }
}

// W(p, p') = J(p) Hbar^{-1} J(p')^T  (3x3, row-major), J(p) = [p^T (x) I3, I3]
template <typename real>
DEV void wblock(const double *T, const real *p, const real *pp, real *W) {
  const double *D = T + HI_D;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      real v = p[r] * pp[s] * real(sym3(D, r, s));
      if (r == s) {
        v += real(T[HI_T]);
#pragma unroll
        for (int c = 0; c < 3; ++c)
          if (c != r) v += p[c] * pp[c] * real(T[HI_PD + 3 * r + c]);
      } else {
        v += p[s] * pp[r] * real(T[HI_PX + pair_slot(r, s)]);
      }
      W[3 * r + s] = v;
    }
}

// --------------------------------------------------------------- 3x3 algebra

template <typename real>
DEV real det3(const real *A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// cofactor matrix: C(r,c) = cofactor of A(r,c); A^{-1} = C^T / det
template <typename real>
DEV void cof3(const real *A, real *C) {
  C[0] = A[4] * A[8] - A[5] * A[7];
  C[1] = A[5] * A[6] - A[3] * A[8];
  C[2] = A[3] * A[7] - A[4] * A[6];
  C[3] = A[2] * A[7] - A[1] * A[8];
  C[4] = A[0] * A[8] - A[2] * A[6];
  C[5] = A[1] * A[6] - A[0] * A[7];
  C[6] = A[1] * A[5] - A[2] * A[4];
  C[7] = A[2] * A[3] - A[0] * A[5];
  C[8] = A[0] * A[4] - A[1] * A[3];
}

// Polar factor R = A (A^T A)^{-1/2} (Eq. polar).  A stiff body keeps A close
// to a rotation, and there the Newton-Schulz iteration X <- X (3I - X^T X)/2
// converges quadratically using only products (about 65 flops a step, no
// division): with E = X^T X - I each step maps |E| to about 1.5 |E|^2, so
// once |E|_F < 1e-8 (FP64; 1e-5 in FP32) the step just taken leaves an error
// below rounding and the iterate is final.  Farther from orthogonality
// (|E|_F >= 0.5, where Newton-Schulz may not converge) Newton's iteration
// X <- (zeta X + X^{-T} / zeta) / 2 with determinant scaling takes over
// (Higham, Functions of Matrices, Sec. 8.3).  Returns false if det A <= 0 or
// the input is not finite.
template <typename real>
DEV bool polar3(const real *A, real *R) {
  const real ns_stop = sizeof(real) == 8 ? real(1e-16) : real(1e-10);
  real X[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) X[i] = A[i];
  real d0 = det3(X);
  if (!(d0 > real(0)) || !isfinite(d0)) return false;
  bool done = false;
  for (int it = 0; it < 8 && !done; ++it) {
    // E = X^T X - I (symmetric)
    real E[6];
    E[0] = X[0] * X[0] + X[3] * X[3] + X[6] * X[6] - real(1);
    E[1] = X[0] * X[1] + X[3] * X[4] + X[6] * X[7];
    E[2] = X[0] * X[2] + X[3] * X[5] + X[6] * X[8];
    E[3] = X[1] * X[1] + X[4] * X[4] + X[7] * X[7] - real(1);
    E[4] = X[1] * X[2] + X[4] * X[5] + X[7] * X[8];
    E[5] = X[2] * X[2] + X[5] * X[5] + X[8] * X[8] - real(1);
    const real e2 = E[0] * E[0] + E[3] * E[3] + E[5] * E[5] +
                    real(2) * (E[1] * E[1] + E[2] * E[2] + E[4] * E[4]);
    if (!(e2 < real(0.25))) break;  // far from orthogonal: Newton below
    // X <- X (I - E / 2)
    const real N[9] = {real(1) - real(0.5) * E[0], -real(0.5) * E[1], -real(0.5) * E[2],
                       -real(0.5) * E[1], real(1) - real(0.5) * E[3], -real(0.5) * E[4],
                       -real(0.5) * E[2], -real(0.5) * E[4], real(1) - real(0.5) * E[5]};
    real Y[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        Y[3 * r + c] = X[3 * r] * N[c] + X[3 * r + 1] * N[3 + c] + X[3 * r + 2] * N[6 + c];
#pragma unroll
    for (int i = 0; i < 9; ++i) X[i] = Y[i];
    if (e2 < ns_stop) done = true;
  }
  const real stop = sizeof(real) == 8 ? real(1e-16) : real(1e-10);
  for (int it = 0; it < 40 && !done; ++it) {
    real C[9];
    cof3(X, C);
    real det = X[0] * C[0] + X[1] * C[1] + X[2] * C[2];
    if (!(det > real(0))) return false;
    real z = real(1), iz = real(1);
    real diff = real(0);
    // X^{-T} = C / det
    real inv = real(1) / det;
    real Y[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Y[i] = C[i] * inv;
    // scale only while the iterate is far from orthogonal
    real s0 = real(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) s0 += (X[i] - Y[i]) * (X[i] - Y[i]);
    if (s0 > real(1e-4)) {
      z = real(1) / cbrt(det);
      iz = cbrt(det);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      real xn = real(0.5) * (z * X[i] + Y[i] * iz);
      diff += (xn - X[i]) * (xn - X[i]);
      X[i] = xn;
    }
    // quadratic convergence: once the step is below 1e-8 (FP64) the next
    // error is below roundoff, so this iterate is final
    if (diff < stop) done = true;
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) R[i] = X[i];
  return done;
}

template <typename real>
DEV void mat3_mul(const real *A, const real *B, real *C) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}

// C = A B^T
template <typename real>
DEV void mat3_mul_bt(const real *A, const real *B, real *C) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      C[3 * r + c] = A[3 * r] * B[3 * c] + A[3 * r + 1] * B[3 * c + 1] + A[3 * r + 2] * B[3 * c + 2];
}

// C = A^T B
template <typename real>
DEV void mat3_mul_at(const real *A, const real *B, real *C) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      C[3 * r + c] = A[r] * B[c] + A[3 + r] * B[3 + c] + A[6 + r] * B[6 + c];
}

template <typename real>
DEV void mat3_vec(const real *A, const real *x, real *y) {
  y[0] = A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
  y[1] = A[3] * x[0] + A[4] * x[1] + A[5] * x[2];
  y[2] = A[6] * x[0] + A[7] * x[1] + A[8] * x[2];
}

template <typename real>
DEV void mat3t_vec(const real *A, const real *x, real *y) {
  y[0] = A[0] * x[0] + A[3] * x[1] + A[6] * x[2];
  y[1] = A[1] * x[0] + A[4] * x[1] + A[7] * x[2];
  y[2] = A[2] * x[0] + A[5] * x[1] + A[8] * x[2];
}

// R W R^T for symmetric or general W (full 3x3 out)
template <typename real>
DEV void rot_congr(const real *R, const real *W, real *out) {
  real T[9];
  mat3_mul(R, W, T);
  mat3_mul_bt(T, R, out);
}

// inverse of a symmetric positive definite 3x3 (returns false if not SPD)
DEV bool spd3_inv(const double *S, double *I) {
  double C[9];
  cof3(S, C);
  double det = S[0] * C[0] + S[1] * C[1] + S[2] * C[2];
  if (!(det > 0.0) || !(S[0] > 0.0)) return false;
  double inv = 1.0 / det;
#pragma unroll
  for (int i = 0; i < 9; ++i) I[i] = C[i] * inv;  // symmetric: C^T = C
  // symmetrise
  double a = 0.5 * (I[1] + I[3]), b = 0.5 * (I[2] + I[6]), c = 0.5 * (I[5] + I[7]);
  I[1] = I[3] = a;
  I[2] = I[6] = b;
  I[5] = I[7] = c;
  return true;
}

// y = Hbar x with Hbar = M_A / h^2 + Kbar_A (Eq. abd_final), Kbar_A =
// V (mu (I9 + P9) + lambda vec(I) vec(I)^T) on the nine A entries (P9: the
// transpose permutation), `sh` = {Mbar0, Mbar1, Mbar2, m, V, mu, lambda}
DEV void hbar_apply(const double *sh, double h, const double *x, double *y) {
  const double ih2 = 1.0 / (h * h);
  const double Vmu = sh[4] * sh[5], Vla = sh[4] * sh[6];
  const double tr = x[0] + x[4] + x[8];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int r = 0; r < 3; ++r)
      y[3 * c + r] = sh[c] * ih2 * x[3 * c + r] + Vmu * (x[3 * c + r] + x[3 * r + c]) +
                     (r == c ? Vla * tr : 0.0);
#pragma unroll
  for (int i = 9; i < 12; ++i) y[i] = sh[3] * ih2 * x[i];
}

// --------------------------------------------------------------- body force

// Local (rotated) right-hand side phi = diag4(R^T) f_A of one body, with
//   f_A = Mbar qd / h - Mbar (q - qn) / h^2 + [0; m g] + f_el + G(A)^T W
// (Eq. variation_energy; Eq. module1-wrench-map) and the co-rotated linear
// elastic force f_el = -V vec(R P(R^T A)) (Eq. reduced_K with dPsi/dA of
// Sec. 3.3), so that the rotated elastic part is simply -V P.  W = [tau; f]
// is the body's external wrench (world frame, about the COM; `wr` its 6
// values or null): G(A) maps qdot to the twist (omega = 1/2 sum_c q_c x
// qdot_c, v = tdot; Eq. module1-G-twist), so G(A)^T W adds 1/2 tau x q_c to
// column c of A and f to the translation.  `wr` is the SoA wrench array (six
// streams of stride `ws`) and `wb` this body's index in it, or wr is null.
// `sh` = {Mbar0, Mbar1, Mbar2, m, V, mu, lambda}.
template <typename real>
DEV void local_force(const double *sh, const real *R, const real *A, const real *q,
                     const real *qn, const real *qd, const double *g, double h, real *phi,
                     const double *wr = nullptr, int64_t ws = 0, int64_t wb = 0) {
  const real ih = real(1.0 / h), ih2 = real(1.0 / (h * h));
  real Sym[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      Sym[3 * r + c] = R[r] * A[c] + R[3 + r] * A[3 + c] + R[6 + r] * A[6 + c];
  const real mu = real(sh[5]), lam = real(sh[6]), V = real(sh[4]);
  const real tr = Sym[0] + Sym[4] + Sym[8] - real(3.0);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const real M = real(sh[c]);
    real w[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
      w[i] = M * qd[3 * c + i] * ih - M * (q[3 * c + i] - qn[3 * c + i]) * ih2;
    if (c == 3) {
#pragma unroll
      for (int i = 0; i < 3; ++i) w[i] += real(sh[3] * g[i]);
    }
    if (wr) {
      if (c < 3) {
        const real t0 = real(wr[wb]), t1 = real(wr[ws + wb]), t2 = real(wr[2 * ws + wb]);
        const real *qc = q + 3 * c;
        w[0] += real(0.5) * (t1 * qc[2] - t2 * qc[1]);
        w[1] += real(0.5) * (t2 * qc[0] - t0 * qc[2]);
        w[2] += real(0.5) * (t0 * qc[1] - t1 * qc[0]);
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) w[i] += real(wr[(3 + i) * ws + wb]);
      }
    }
    // R^T w
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      real v = R[r] * w[0] + R[3 + r] * w[1] + R[6 + r] * w[2];
      if (c < 3) {
        real P = mu * (Sym[3 * r + c] + Sym[3 * c + r] - real(2.0) * real(r == c)) +
                 lam * tr * real(r == c);
        v -= V * P;
      }
      phi[3 * c + r] = v;
    }
  }
}

// ------------------------------------------------ polar-free body solve
// Length-preserving stand-in for a rotation (Eq. len_preserving): y = M x
// (M^T x if transpose) scaled to |x|; x itself if M x vanishes.  M is a
// row-major 3x3 (the affine block A).
DEV void lenpres(const double *M, bool transpose, const double *x, double *y) {
  if (transpose) mat3t_vec(M, x, y);
  else mat3_vec(M, x, y);
  const double lx = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  const double ly = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
  if (ly > 0.0) {
    const double s = lx / ly;
    y[0] *= s; y[1] *= s; y[2] *= s;
  } else {
    y[0] = x[0]; y[1] = x[1]; y[2] = x[2];
  }
}

// Body-frame force of the polar-free solve (Alg. 1): the world forces of
// local_force (inertia, gravity, wrench) taken to the body frame block by
// block with A^T scaled to length instead of R^T, and the rotated elastic
// force -V P(R^T A) with the same stand-in for R^T A, column by column.
DEV void local_force_lp(const double *sh, const double *A, const double *q, const double *qn,
                        const double *qd, const double *g, double h, double *phi,
                        const double *wr, int64_t ws, int64_t wb) {
  const double ih = 1.0 / h, ih2 = 1.0 / (h * h);
  double Sh[9];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double col[3] = {A[c], A[3 + c], A[6 + c]};
    double x[3];
    lenpres(A, true, col, x);
#pragma unroll
    for (int r = 0; r < 3; ++r) Sh[3 * r + c] = x[r];
  }
  const double mu = sh[5], lam = sh[6], V = sh[4];
  const double tr = Sh[0] + Sh[4] + Sh[8] - 3.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double M = sh[c];
    double w[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) w[i] = M * qd[3 * c + i] * ih - M * (q[3 * c + i] - qn[3 * c + i]) * ih2;
    if (c == 3) {
#pragma unroll
      for (int i = 0; i < 3; ++i) w[i] += sh[3] * g[i];
    }
    if (wr) {
      if (c < 3) {
        const double t0 = wr[wb], t1 = wr[ws + wb], t2 = wr[2 * ws + wb];
        const double *qc = q + 3 * c;
        w[0] += 0.5 * (t1 * qc[2] - t2 * qc[1]);
        w[1] += 0.5 * (t2 * qc[0] - t0 * qc[2]);
        w[2] += 0.5 * (t0 * qc[1] - t1 * qc[0]);
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) w[i] += wr[(3 + i) * ws + wb];
      }
    }
    double v[3];
    lenpres(A, true, w, v);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      if (c < 3) {
        const double P = mu * (Sh[3 * r + c] + Sh[3 * c + r] - 2.0 * double(r == c)) + lam * tr * double(r == c);
        v[r] -= V * P;
      }
      phi[3 * c + r] = v[r];
    }
  }
}

}  // namespace mabd
