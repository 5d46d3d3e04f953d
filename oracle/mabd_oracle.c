/*
 * FP64 CPU oracle for one time step of M-ABD (arXiv 2603.08079).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares no
 * source with the GPU library.
 *
 * What is computed, in the paper's order:
 *   per body (Sec. 3.2-3.4): M_A = J^T M J (Eq. newton_abd), the rest stiffness
 *     K_A of linear elasticity (Sec. 3.3, dPsi/dA), Hbar = M_A/h^2 + K_A
 *     (Eq. abd_final), R = A (A^T A)^{-1/2} (Eq. polar) via a Jacobi eigen
 *     decomposition of A^T A, the co-rotated Hessian H = diag4(R) Hbar diag4(R^T)
 *     (Eq. reduced_newton), and the force f_A = -grad E at the current iterate
 *     (Eq. variation_energy with implicit Euler), elastic part evaluated in the
 *     rotated frame (Eq. reduced_K), plus external wrenches mapped by
 *     f_A,ext = G(A)^T W (Eqs. module1-G-twist, module1-wrench-map);
 *   per joint (Sec. 4): ball rows (Eq. ball) and 5-row hinge rows (Eq. hinge)
 *     with the gradient of Eqs. constraint_gradient, pcpq, pcpr, r_gradient
 *     (R approximated by A in the rotation term);
 *   globally (Sec. 5): the KKT system Eq. kkt with the -C right-hand side of its
 *     footnote, solved through the dual system Eq. dual by
 *       - block Thomas on chains (Sec. 5.2, Eq. chain-btd),
 *       - primal leaf-to-root condensation on trees (Sec. 5.3, Eq. module3-kkt),
 *       - dense Cholesky (Sec. 5.1 "any linear solver") or block-Jacobi PCG on
 *         graphs;
 *     then the primal back-projection Eq. primal / Eq. recover-dq-explicit.
 *
 * Dense 12x12 matrices are used everywhere on purpose; nothing is blocked,
 * fused or reordered beyond what the equations state.
 */
#include "mabd_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NQ 12
#define MAXC 5

/* ------------------------------------------------------------------ dense */

/* C(m x n) = A(m x k) B(k x n), row-major */
static void mm(int m, int k, int n, const double *A, const double *B, double *C) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s += A[i * k + l] * B[l * n + j];
      C[i * n + j] = s;
    }
}

/* C(m x n) = A(k x m)^T B(k x n) */
static void mtm(int m, int k, int n, const double *A, const double *B, double *C) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s += A[l * m + i] * B[l * n + j];
      C[i * n + j] = s;
    }
}

/* C(m x n) = A(m x k) B(n x k)^T */
static void mmt(int m, int k, int n, const double *A, const double *B, double *C) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s += A[i * k + l] * B[j * k + l];
      C[i * n + j] = s;
    }
}

/* in-place lower Cholesky of an n x n SPD matrix; returns 0 or -1 */
static int chol(int n, double *A) {
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0.0)) return -1;
    d = sqrt(d);
    A[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = s / d;
    }
    for (int i = 0; i < j; ++i) A[i * n + j] = 0.0;
  }
  return 0;
}

/* solve (L L^T) x = b in place, L from chol() */
static void chol_solve(int n, const double *L, double *b) {
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= L[i * n + k] * b[k];
    b[i] = s / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * b[k];
    b[i] = s / L[i * n + i];
  }
}

/* X(n x c) = M^{-1} B(n x c) for a Cholesky factor L of M, column by column */
static void chol_solve_cols(int n, int c, const double *L, const double *B, double *X) {
  double col[64];
  for (int j = 0; j < c; ++j) {
    for (int i = 0; i < n; ++i) col[i] = B[i * c + j];
    chol_solve(n, L, col);
    for (int i = 0; i < n; ++i) X[i * c + j] = col[i];
  }
}

/* ------------------------------------------------------------------ 3x3 */

/* A (row-major 3x3) from q: A(r,c) = q[3c + r] (column-stacked, Sec. 3.1) */
static void q_to_A(const double *q, double *A) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) A[r * 3 + c] = q[3 * c + r];
}

static double det3(const double *A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* cyclic Jacobi eigen decomposition of a symmetric 3x3: S = V diag(w) V^T */
static void jacobi_eig3(const double *S_in, double *V, double *w) {
  double S[9];
  memcpy(S, S_in, sizeof S);
  for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = S[1] * S[1] + S[2] * S[2] + S[5] * S[5];
    double dia = S[0] * S[0] + S[4] * S[4] + S[8] * S[8];
    if (off <= 1e-36 * dia || off == 0.0) break;
    for (int p = 0; p < 2; ++p)
      for (int qi = p + 1; qi < 3; ++qi) {
        double apq = S[p * 3 + qi];
        if (apq == 0.0) continue;
        double app = S[p * 3 + p], aqq = S[qi * 3 + qi];
        double tau = (aqq - app) / (2.0 * apq);
        double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        /* S <- G^T S G with G the rotation in the (p, qi) plane */
        for (int k = 0; k < 3; ++k) {
          double skp = S[k * 3 + p], skq = S[k * 3 + qi];
          S[k * 3 + p] = c * skp - s * skq;
          S[k * 3 + qi] = s * skp + c * skq;
        }
        for (int k = 0; k < 3; ++k) {
          double spk = S[p * 3 + k], sqk = S[qi * 3 + k];
          S[p * 3 + k] = c * spk - s * sqk;
          S[qi * 3 + k] = s * spk + c * sqk;
        }
        for (int k = 0; k < 3; ++k) {
          double vkp = V[k * 3 + p], vkq = V[k * 3 + qi];
          V[k * 3 + p] = c * vkp - s * vkq;
          V[k * 3 + qi] = s * vkp + c * vkq;
        }
      }
  }
  w[0] = S[0]; w[1] = S[4]; w[2] = S[8];
}

/* Eq. polar: R = A (A^T A)^{-1/2}; A, R row-major 3x3. */
static int polar_rm(const double *A, double *R) {
  for (int i = 0; i < 9; ++i)
    if (!isfinite(A[i])) return ORA_ENONFINITE;
  if (!(det3(A) > 0.0)) return ORA_ENONFINITE;
  double AtA[9], V[9], w[3], Sinv[9];
  mtm(3, 3, 3, A, A, AtA);
  jacobi_eig3(AtA, V, w);
  for (int i = 0; i < 3; ++i)
    if (!(w[i] > 0.0)) return ORA_ENONFINITE;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += V[i * 3 + k] * V[j * 3 + k] / sqrt(w[k]);
      Sinv[i * 3 + j] = s;
    }
  mm(3, 3, 3, A, Sinv, R);
  return ORA_OK;
}

/* exported: A and R in the column-stacked layout of q */
int32_t ora_polar(const double *Aq, double *Rq) {
  double A[9], R[9];
  q_to_A(Aq, A);
  int st = polar_rm(A, R);
  if (st) return st;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Rq[3 * c + r] = R[r * 3 + c];
  return ORA_OK;
}

/* ------------------------------------------------------------ body terms */

static void lame(const ora_system *s, int i, double *mu, double *lam) {
  double k = s->k_orth[i];
  if (s->material == 1) {
    double nu = s->poisson ? s->poisson[i] : 0.0;
    *mu = k / (2.0 * (1.0 + nu));
    *lam = k * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  } else {
    /* Eq. EA linearised at A = I: Hessian of k_A |A A^T - I|_F^2 is 4 k_A (I + P) */
    *mu = 4.0 * k;
    *lam = 0.0;
  }
}

/* generalised mass diagonal Mbar (M_A = Mbar (x) I3) of a box with its rest
   frame at the centre of mass: integral of rho xbar xbar^T and rho */
static void box_mass(const ora_system *s, int i, double *Mbar, double *V, double *m) {
  const double *d = s->dims + 3 * i;
  *V = d[0] * d[1] * d[2];
  *m = s->density[i] * (*V);
  for (int c = 0; c < 3; ++c) Mbar[c] = (*m) * d[c] * d[c] / 12.0;
  Mbar[3] = *m;
}

/* Hbar = M_A / h^2 + Kbar_A  (Eq. abd_final), dense 12x12 */
static void hbar(const ora_system *s, int i, double h, double *Hb) {
  double Mbar[4], V, m, mu, lam;
  box_mass(s, i, Mbar, &V, &m);
  lame(s, i, &mu, &lam);
  memset(Hb, 0, sizeof(double) * 144);
  for (int c = 0; c < 4; ++c)
    for (int r = 0; r < 3; ++r) Hb[(3 * c + r) * 12 + 3 * c + r] = Mbar[c] / (h * h);
  /* d/dA of mu (A + A^T - 2I) + lam tr(A - I) I, times V */
  for (int a = 0; a < 9; ++a) {
    int ai = a % 3, aj = a / 3; /* a = 3 aj + ai <-> A(ai, aj) */
    for (int b = 0; b < 9; ++b) {
      int bi = b % 3, bj = b / 3;
      double k = 0.0;
      if (a == b) k += mu;
      if (bi == aj && bj == ai) k += mu; /* transpose permutation */
      if (ai == aj && bi == bj) k += lam;
      Hb[a * 12 + b] += V * k;
    }
  }
}

/* diag4(R) as a dense 12x12 (R row-major) */
static void diag4(const double *R, double *D) {
  memset(D, 0, sizeof(double) * 144);
  for (int c = 0; c < 4; ++c)
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) D[(3 * c + r) * 12 + 3 * c + k] = R[r * 3 + k];
}

/* Per body: co-rotated H (Eq. reduced_newton) and f_A = -grad E at qi,
   E of Eq. variation_energy with xhat = x^n + h xdot^n + h^2 M^{-1} f_ext. */
static int body_terms_at(const ora_system *s, double h, const double *qi, const double *qn,
                         const double *qdn, int i, double *H, double *f, double *R) {
  double A[9], Hb[144], D4[144], T[144];
  double Mbar[4], V, m, mu, lam;
  q_to_A(qi, A);
  int st = polar_rm(A, R);
  if (st) return st;
  box_mass(s, i, Mbar, &V, &m);
  lame(s, i, &mu, &lam);
  hbar(s, i, h, Hb);
  diag4(R, D4);
  mm(12, 12, 12, D4, Hb, T);
  mmt(12, 12, 12, T, D4, H);
  /* elastic force in the rotated frame (Eq. reduced_K with dPsi/dA of Sec. 3.3) */
  double Sym[9], P[9], F[9];
  mtm(3, 3, 3, R, A, Sym);
  double tr = Sym[0] + Sym[4] + Sym[8] - 3.0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      P[r * 3 + c] = mu * (Sym[r * 3 + c] + Sym[c * 3 + r] - 2.0 * (r == c)) + lam * tr * (r == c);
  mm(3, 3, 3, R, P, F);
  /* external wrench W = [tau; f] at the current iterate: G(A) maps qdot to the
     twist [omega; v] with omega = 1/2 sum_c q_c x qdot_c and v = tdot (Eq.
     module1-G-twist), so G(A)^T W puts 1/2 [q_c]_x^T tau = 1/2 tau x q_c on
     column c of A and f on the translation */
  double gw[12];
  memset(gw, 0, sizeof gw);
  if (s->wrench) {
    const double *tau = s->wrench + 6 * i, *fw = tau + 3;
    for (int c = 0; c < 3; ++c) {
      const double *qc = qi + 3 * c;
      gw[3 * c + 0] = 0.5 * (tau[1] * qc[2] - tau[2] * qc[1]);
      gw[3 * c + 1] = 0.5 * (tau[2] * qc[0] - tau[0] * qc[2]);
      gw[3 * c + 2] = 0.5 * (tau[0] * qc[1] - tau[1] * qc[0]);
    }
    for (int r = 0; r < 3; ++r) gw[9 + r] = fw[r];
  }
  for (int a = 0; a < 12; ++a) {
    int c = a / 3, r = a % 3;
    double M = Mbar[c];
    double fel = (c < 3) ? -V * F[r * 3 + c] : 0.0;
    double fext = ((c == 3) ? m * s->gravity[r] : 0.0) + gw[a];
    f[a] = M * qdn[a] / h - M * (qi[a] - qn[a]) / (h * h) + fext + fel;
  }
  for (int a = 0; a < 144; ++a)
    if (!isfinite(H[a])) return ORA_ENONFINITE;
  for (int a = 0; a < 12; ++a)
    if (!isfinite(f[a])) return ORA_ENONFINITE;
  return ORA_OK;
}

static int is_dyn(const ora_system *s, int b) { return b >= 0 && !s->pinned[b]; }

int32_t ora_body_terms(const ora_system *s, double h, const double *q, const double *qd,
                       int32_t i, double *H, double *f, double *R) {
  if (i < 0 || i >= s->n) return ORA_EINVAL;
  double Rr[9];
  int st = body_terms_at(s, h, q + 12 * i, q + 12 * i, qd + 12 * i, i, H, f, Rr);
  if (R)
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) R[3 * c + r] = Rr[r * 3 + c];
  return st;
}

/* ----------------------------------------------------------- joint terms */

/* J(p) = [p^T (x) I3, I3] (Eq. abd_dof), 3x12 row-major */
static void jmat(const double *p, double *J) {
  memset(J, 0, sizeof(double) * 36);
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) J[r * 12 + 3 * c + r] = p[c];
    J[r * 12 + 9 + r] = 1.0;
  }
}

/* Rodrigues-type frame of Sec. 4.3: rows (r_x, a, r_z); maps the unit axis a to e_y */
static void hinge_frame(const double *a, double *Rh) {
  if (1.0 + a[1] < 1e-12) { /* a = -e_y: the formula is singular; rotate by pi about x */
    double D[9] = {1, 0, 0, 0, -1, 0, 0, 0, -1};
    memcpy(Rh, D, sizeof D);
    return;
  }
  /* v = a x e_y */
  double v[3] = {-a[2], 0.0, a[0]};
  double K[9] = {0, -v[2], v[1], v[2], 0, -v[0], -v[1], v[0], 0};
  double K2[9];
  mm(3, 3, 3, K, K, K2);
  for (int i = 0; i < 9; ++i) Rh[i] = (i % 4 == 0 ? 1.0 : 0.0) + K[i] + K2[i] / (1.0 + a[1]);
}

/* the side of a joint: translation t and matrix A (world: t = 0, A = I) */
static void side_pose(const ora_system *s, const double *q, int b, double *A, double *t) {
  if (b < 0) {
    for (int i = 0; i < 9; ++i) A[i] = (i % 4 == 0) ? 1.0 : 0.0;
    t[0] = t[1] = t[2] = 0.0;
  } else {
    const double *qb = s->pinned[b] ? s->q0 + 12 * b : q + 12 * b;
    q_to_A(qb, A);
    for (int r = 0; r < 3; ++r) t[r] = qb[9 + r];
  }
}

/* rotation of a side at creation (polar of A0; identity for the world) */
static int side_rot0(const ora_system *s, int b, double *R) {
  if (b < 0) {
    for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
    return ORA_OK;
  }
  double A[9];
  q_to_A(s->q0 + 12 * b, A);
  return polar_rm(A, R);
}

/* rows per joint: ball 3 (Eq. ball), hinge 5 (Eq. hinge), universal 4
   (Eq. universal), prismatic 5 (Eq. prismatic) */
static int jrows(const ora_system *s, int k) {
  static const int rows[4] = {3, 5, 4, 5};
  return rows[s->jtype[k]];
}

/* u = v / |v|; nonzero status if v is zero or not finite */
static int unit3(const double *v, double *u) {
  double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  if (!(n > 0.0) || !isfinite(n)) return ORA_EINVAL;
  for (int r = 0; r < 3; ++r) u[r] = v[r] / n;
  return ORA_OK;
}

/* difference of two attached points, translation difference first so that
   rounding stays at the scale of the bodies rather than the world position */
static void point_diff(const double *Aa, const double *ta, const double *pa, const double *Ab,
                       const double *tb, const double *pb, double *d) {
  double wa[3], wb[3];
  mm(3, 3, 1, Aa, pa, wa);
  mm(3, 3, 1, Ab, pb, wb);
  for (int r = 0; r < 3; ++r) d[r] = (ta[r] - tb[r]) + (wa[r] - wb[r]);
}

/* Constraint value C (rows) and gradients Ga, Gb (rows x 12, zero if that side
   is not dynamic).  Ball: Eq. ball.  Hinge: Eq. hinge with Eqs. pcpq and the
   A-linearised rotation term of Eq. r_gradient (alpha owns R_H = dR_H R_a^T). */
static int joint_terms(const ora_system *s, const double *q, int k, double *C, double *Ga,
                       double *Gb) {
  int a = s->ja[k], b = s->jb[k];
  double Aa[9], ta[3], Ab[9], tb[3];
  side_pose(s, q, a, Aa, ta);
  side_pose(s, q, b, Ab, tb);
  const double *pa = s->pa + 3 * k, *pb = s->pb + 3 * k;
  int rows = jrows(s, k);
  memset(Ga, 0, sizeof(double) * rows * 12);
  memset(Gb, 0, sizeof(double) * rows * 12);
  if (s->jtype[k] == 0) {
    point_diff(Aa, ta, pa, Ab, tb, pb, C);
    double J[36];
    if (is_dyn(s, a)) {
      jmat(pa, J);
      memcpy(Ga, J, sizeof J);
    }
    if (is_dyn(s, b)) {
      jmat(pb, J);
      for (int i = 0; i < 36; ++i) Gb[i] = -J[i];
    }
    return ORA_OK;
  }
  /* Joints expressed in a rotated frame (Secs. 4.3-4.5).  Body a owns the
     frame R_J = dR R_a^T, dR the joint's frame at rest (R_a the polar
     rotation of a, Eq. polar): hinge and prismatic use the Rodrigues frame of
     their axis (rows r_x, axis, r_z), the universal joint the rows
     (a1 x a2, a1, a2).  Control points (rest frames of their bodies): P1 of
     either side at the anchor; hinge: P2 = P1 + ell * axis on both sides;
     universal: b's P2 = P1 + ell * a2; prismatic: b's P2 = P1 + ell * axis and
     P3 = P1 + ell * n, n the frame's local z axis at rest.  A direction fixed
     in a's rest frame enters b's rest frame as the same world direction at
     creation.  Each row is one local component of R_J (y_X - y_Y):
       hinge      x, y, z of (P1a - P1b); x, z of (P2a - P2b)        (5 rows)
       universal  x, y, z of (P1a - P1b); y of (P2b - P1b)            (4 rows)
       prismatic  x, z of (P1a - P1b); x, z of (P2b - P1b); x of (P3b - P1b)
     Gradient (default hinge_grad): the frozen-frame part R_J J(p) on each
     point's body, plus on body a the rotation term of Eq. r_gradient with
     R_a ~ A_a (Eq. pcpr), d(rbar^T A_a^T d)/dvec(A_a). */
  const int type = s->jtype[k];
  double ax[3];
  if (unit3(s->axis + 3 * k, ax)) return ORA_EINVAL;
  double Ra0[9], Rb0[9];
  int st = side_rot0(s, a, Ra0);
  if (st) return st;
  st = side_rot0(s, b, Rb0);
  if (st) return st;
  double dRh[9];
  if (type == 2) {
    double a2[3];
    if (!s->axis2 || unit3(s->axis2 + 3 * k, a2)) return ORA_EINVAL;
    double dt = ax[0] * a2[0] + ax[1] * a2[1] + ax[2] * a2[2];
    for (int r = 0; r < 3; ++r) a2[r] -= dt * ax[r];
    if (unit3(a2, a2)) return ORA_EINVAL;
    double x[3] = {ax[1] * a2[2] - ax[2] * a2[1], ax[2] * a2[0] - ax[0] * a2[2],
                   ax[0] * a2[1] - ax[1] * a2[0]};
    for (int r = 0; r < 3; ++r) {
      dRh[r] = x[r];
      dRh[3 + r] = ax[r];
      dRh[6 + r] = a2[r];
    }
  } else {
    hinge_frame(ax, dRh);
  }
  double ell = s->cp_len[k];
  /* directions of b's second and third points, in a's rest frame, then in b's */
  double da2[3], da3[3] = {0.0, 0.0, 0.0}, wd[3], db2[3], db3[3];
  if (type == 2) memcpy(da2, dRh + 6, sizeof da2);
  else memcpy(da2, ax, sizeof da2);
  if (type == 3) memcpy(da3, dRh + 6, sizeof da3);
  mm(3, 3, 1, Ra0, da2, wd);
  mtm(3, 3, 1, Rb0, wd, db2);
  mm(3, 3, 1, Ra0, da3, wd);
  mtm(3, 3, 1, Rb0, wd, db3);
  /* points: 0 P1 of a, 1 P2 of a, 2 P1 of b, 3 P2 of b, 4 P3 of b */
  double P[5][3];
  for (int r = 0; r < 3; ++r) {
    P[0][r] = pa[r];
    P[1][r] = pa[r] + ell * ax[r];
    P[2][r] = pb[r];
    P[3][r] = pb[r] + ell * db2[r];
    P[4][r] = pb[r] + ell * db3[r];
  }
  const int pside[5] = {0, 0, 1, 1, 1};
  /* rows: local component, point X, point Y */
  static const int spec[4][5][3] = {
      {{0, 0, 2}, {1, 0, 2}, {2, 0, 2}, {0, 0, 2}, {0, 0, 2}},  /* (ball: unused) */
      {{0, 0, 2}, {1, 0, 2}, {2, 0, 2}, {0, 1, 3}, {2, 1, 3}},  /* hinge */
      {{0, 0, 2}, {1, 0, 2}, {2, 0, 2}, {1, 3, 2}, {0, 0, 2}},  /* universal */
      {{0, 0, 2}, {2, 0, 2}, {0, 3, 2}, {2, 3, 2}, {0, 4, 2}}}; /* prismatic */
  double Ra[9], Rh[9];
  if (a >= 0) {
    st = polar_rm(Aa, Ra);
    if (st) return st;
  } else {
    for (int i = 0; i < 9; ++i) Ra[i] = (i % 4 == 0) ? 1.0 : 0.0;
  }
  mmt(3, 3, 3, dRh, Ra, Rh); /* R_J = dR R_a^T */
  for (int i = 0; i < rows; ++i) {
    const int comp = spec[type][i][0], X = spec[type][i][1], Y = spec[type][i][2];
    /* y_X - y_Y: across the joint the translation difference first; on one
       body its affine block times the difference of the rest points */
    double dm[3];
    if (pside[X] != pside[Y]) {
      point_diff(Aa, ta, P[X], Ab, tb, P[Y], dm);
    } else {
      double dp[3] = {P[X][0] - P[Y][0], P[X][1] - P[Y][1], P[X][2] - P[Y][2]};
      mm(3, 3, 1, pside[X] ? Ab : Aa, dp, dm);
    }
    double e[3];
    mm(3, 3, 1, Rh, dm, e);
    C[i] = e[comp];
    for (int pt = 0; pt < 2; ++pt) {
      const int id = pt == 0 ? X : Y;
      const int body = pside[id] ? b : a;
      if (!is_dyn(s, body)) continue;
      double *G = pside[id] ? Gb : Ga;
      const double sg = pt == 0 ? 1.0 : -1.0;
      double Jm[36];
      jmat(P[id], Jm);
      for (int col = 0; col < 12; ++col) {
        double v = 0.0;
        for (int r = 0; r < 3; ++r) v += Rh[comp * 3 + r] * Jm[r * 12 + col];
        G[i * 12 + col] += sg * v;
      }
    }
    if (is_dyn(s, a) && s->hinge_grad == 0) {
      /* d(rbar_c^T A^T d_m)/dvec(A): entry 3l + kk is rbar_c[l] d_m[kk] */
      for (int l = 0; l < 3; ++l)
        for (int kk = 0; kk < 3; ++kk) Ga[i * 12 + 3 * l + kk] += dRh[comp * 3 + l] * dm[kk];
    }
  }
  return ORA_OK;
}

int32_t ora_joint_terms(const ora_system *s, const double *q, int32_t k, double *C, double *Ga,
                        double *Gb) {
  if (k < 0 || k >= s->m) return ORA_EINVAL;
  return joint_terms(s, q, k, C, Ga, Gb);
}

int32_t ora_rows(const ora_system *s) {
  int t = 0;
  for (int k = 0; k < s->m; ++k) t += jrows(s, k);
  return t;
}

/* --------------------------------------------------------------- topology */

static int uf_find(int *p, int x) {
  while (p[x] != x) x = p[x] = p[p[x]];
  return x;
}

static int validate(const ora_system *s) {
  if (s->n < 0 || s->m < 0) return ORA_EINVAL;
  for (int k = 0; k < s->m; ++k) {
    int a = s->ja[k], b = s->jb[k];
    if (a < -1 || a >= s->n || b < -1 || b >= s->n) return ORA_EINVAL;
    if (a == b) return ORA_EINVAL;
    if (!is_dyn(s, a) && !is_dyn(s, b)) return ORA_EINVAL;
    if (s->jtype[k] > 3) return ORA_EINVAL;
    if (s->jtype[k] >= 1 && !(s->cp_len[k] > 0.0)) return ORA_EINVAL;
    if (s->jtype[k] == 2 && !s->axis2) return ORA_EINVAL;
  }
  return ORA_OK;
}

/* 1 chain (every dual component a path), 2 tree (incidence graph acyclic), 3 graph */
int32_t ora_classify(const ora_system *s) {
  if (validate(s)) return ORA_EINVAL;
  int N = s->n + s->m;
  int *p = malloc(sizeof(int) * (N > 0 ? N : 1));
  int *deg = calloc(s->n > 0 ? s->n : 1, sizeof(int));
  for (int i = 0; i < N; ++i) p[i] = i;
  int cyc = 0;
  for (int k = 0; k < s->m; ++k) {
    int sides[2] = {s->ja[k], s->jb[k]};
    for (int t = 0; t < 2; ++t) {
      int b = sides[t];
      if (!is_dyn(s, b)) continue;
      deg[b]++;
      int x = uf_find(p, s->n + k), y = uf_find(p, b);
      if (x == y) cyc = 1;
      else p[x] = y;
    }
  }
  int maxdeg = 0;
  for (int i = 0; i < s->n; ++i)
    if (deg[i] > maxdeg) maxdeg = deg[i];
  free(p);
  free(deg);
  if (cyc) return 3;
  return maxdeg <= 2 ? 1 : 2;
}

/* body -> incident joints (CSR) */
typedef struct {
  int *off, *jt;
} incid_t;

static void build_incid(const ora_system *s, incid_t *I) {
  I->off = calloc(s->n + 1, sizeof(int));
  for (int k = 0; k < s->m; ++k) {
    if (is_dyn(s, s->ja[k])) I->off[s->ja[k] + 1]++;
    if (is_dyn(s, s->jb[k])) I->off[s->jb[k] + 1]++;
  }
  for (int i = 0; i < s->n; ++i) I->off[i + 1] += I->off[i];
  I->jt = malloc(sizeof(int) * (I->off[s->n] + 1));
  int *fill = calloc(s->n + 1, sizeof(int));
  for (int k = 0; k < s->m; ++k) {
    int sd[2] = {s->ja[k], s->jb[k]};
    for (int t = 0; t < 2; ++t)
      if (is_dyn(s, sd[t])) I->jt[I->off[sd[t]] + fill[sd[t]]++] = k;
  }
  free(fill);
}

static void free_incid(incid_t *I) {
  free(I->off);
  free(I->jt);
}

/* ------------------------------------------------------------ step state */

typedef struct {
  int nrow;
  int *roff;     /* row offset per joint */
  double *H, *L; /* per body 12x12 and its Cholesky factor */
  double *f;     /* per body 12 */
  double *C;     /* per joint 5 */
  double *Ga, *Gb;
  incid_t inc;
} stepdata;

static void free_sd(stepdata *d) {
  free(d->roff);
  free(d->H);
  free(d->L);
  free(d->f);
  free(d->C);
  free(d->Ga);
  free(d->Gb);
  free_incid(&d->inc);
}

static int build_sd(const ora_system *s, double h, const double *qi, const double *qn,
                    const double *qdn, stepdata *d) {
  memset(d, 0, sizeof *d);
  d->roff = malloc(sizeof(int) * (s->m + 1));
  d->roff[0] = 0;
  for (int k = 0; k < s->m; ++k) d->roff[k + 1] = d->roff[k] + jrows(s, k);
  d->nrow = d->roff[s->m];
  size_t n = s->n, m = s->m;
  d->H = malloc(sizeof(double) * 144 * (n ? n : 1));
  d->L = malloc(sizeof(double) * 144 * (n ? n : 1));
  d->f = calloc(12 * (n ? n : 1), sizeof(double));
  d->C = calloc(5 * (m ? m : 1), sizeof(double));
  d->Ga = calloc(60 * (m ? m : 1), sizeof(double));
  d->Gb = calloc(60 * (m ? m : 1), sizeof(double));
  build_incid(s, &d->inc);
  /* bodies and joints are independent of each other: with -fopenmp these
     loops run on all host cores (the result does not depend on it); the
     reported status is that of the first failing body, then joint */
  int *bst = calloc(n + 1, sizeof(int)), *jst = calloc(m + 1, sizeof(int));
#pragma omp parallel for schedule(static)
  for (int i = 0; i < s->n; ++i) {
    if (!is_dyn(s, i)) continue;
    double R[9];
    bst[i] = body_terms_at(s, h, qi + 12 * i, qn + 12 * i, qdn + 12 * i, i, d->H + 144 * i,
                           d->f + 12 * i, R);
    if (bst[i]) continue;
    memcpy(d->L + 144 * i, d->H + 144 * i, sizeof(double) * 144);
    if (chol(12, d->L + 144 * i)) bst[i] = ORA_ESINGULAR;
  }
  int st = ORA_OK;
  for (int i = 0; i < s->n && !st; ++i) st = bst[i];
  if (!st) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < s->m; ++k)
      jst[k] = joint_terms(s, qi, k, d->C + 5 * k, d->Ga + 60 * k, d->Gb + 60 * k);
    for (int k = 0; k < s->m && !st; ++k) st = jst[k];
  }
  free(bst);
  free(jst);
  return st;
}

/* gradient block of joint k on body b (NULL if b is not a dynamic side) */
static const double *gblk(const ora_system *s, const stepdata *d, int k, int b) {
  if (s->ja[k] == b && is_dyn(s, b)) return d->Ga + 60 * k;
  if (s->jb[k] == b && is_dyn(s, b)) return d->Gb + 60 * k;
  return NULL;
}

/* S block (rows k x rows l) contributed by body b: G_kb H_b^{-1} G_lb^T */
static void sblock(const stepdata *d, int b, const double *Gk, int rk, const double *Gl, int rl,
                   double *out) {
  double X[60];
  double GlT[60];
  for (int i = 0; i < 12; ++i)
    for (int j = 0; j < rl; ++j) GlT[i * rl + j] = Gl[j * 12 + i];
  chol_solve_cols(12, rl, d->L + 144 * b, GlT, X);
  mm(rk, 12, rl, Gk, X, out);
}

/* dual right-hand side of joint k: sum_b G_kb H_b^{-1} f_b + C_k (Eq. dual + footnote) */
static void dual_rhs(const ora_system *s, const stepdata *d, int k, double *r) {
  int rk = jrows(s, k);
  for (int i = 0; i < rk; ++i) r[i] = d->C[5 * k + i];
  int sd[2] = {s->ja[k], s->jb[k]};
  for (int t = 0; t < 2; ++t) {
    const double *G = gblk(s, d, k, sd[t]);
    if (!G) continue;
    double x[12];
    memcpy(x, d->f + 12 * sd[t], sizeof x);
    chol_solve(12, d->L + 144 * sd[t], x);
    for (int i = 0; i < rk; ++i)
      for (int c = 0; c < 12; ++c) r[i] += G[i * 12 + c] * x[c];
  }
}

/* ----------------------------------------------------------- chain solve */

/* block Thomas on every path of the dual graph (Eq. chain-btd) */
static int solve_chain(const ora_system *s, const stepdata *d, double *lam) {
  int m = s->m;
  int *done = calloc(m > 0 ? m : 1, sizeof(int));
  int *ord = malloc(sizeof(int) * (m > 0 ? m : 1));
  int st = ORA_OK;
  for (int start = 0; start < m && !st; ++start) {
    if (done[start]) continue;
    /* walk to one end of the path containing `start` */
    int prev = -1, cur = start;
    for (;;) {
      int nxt = -1;
      int sd[2] = {s->ja[cur], s->jb[cur]};
      for (int t = 0; t < 2 && nxt < 0; ++t) {
        int b = sd[t];
        if (!is_dyn(s, b)) continue;
        for (int e = d->inc.off[b]; e < d->inc.off[b + 1]; ++e) {
          int o = d->inc.jt[e];
          if (o != cur && o != prev) { nxt = o; break; }
        }
      }
      if (nxt < 0) break;
      prev = cur;
      cur = nxt;
      if (cur == start) break; /* cannot happen for a path */
    }
    /* collect the path from that end */
    int K = 0;
    prev = -1;
    for (;;) {
      ord[K++] = cur;
      done[cur] = 1;
      int nxt = -1;
      int sd[2] = {s->ja[cur], s->jb[cur]};
      for (int t = 0; t < 2 && nxt < 0; ++t) {
        int b = sd[t];
        if (!is_dyn(s, b)) continue;
        for (int e = d->inc.off[b]; e < d->inc.off[b + 1]; ++e) {
          int o = d->inc.jt[e];
          if (o != cur && o != prev && !done[o]) { nxt = o; break; }
        }
      }
      if (nxt < 0) break;
      prev = cur;
      cur = nxt;
    }
    /* blocks D_i, B_i, b_i (Eqs. chain-Schur-blocks, chain-b) */
    double *Dh = malloc(sizeof(double) * 25 * K);
    double *Bm = malloc(sizeof(double) * 25 * K);
    double *bh = malloc(sizeof(double) * 5 * K);
    int *rk = malloc(sizeof(int) * K);
    for (int i = 0; i < K; ++i) {
      int k = ord[i];
      rk[i] = jrows(s, k);
      memset(Dh + 25 * i, 0, sizeof(double) * 25);
      int sd[2] = {s->ja[k], s->jb[k]};
      for (int t = 0; t < 2; ++t) {
        const double *G = gblk(s, d, k, sd[t]);
        if (!G) continue;
        double blk[25];
        sblock(d, sd[t], G, rk[i], G, rk[i], blk);
        for (int e = 0; e < rk[i] * rk[i]; ++e) Dh[25 * i + e] += blk[e];
      }
      dual_rhs(s, d, k, bh + 5 * i);
      if (i + 1 < K) {
        int k2 = ord[i + 1], r2 = jrows(s, k2);
        int shared = -1;
        for (int t = 0; t < 2; ++t)
          if (is_dyn(s, sd[t]) && (s->ja[k2] == sd[t] || s->jb[k2] == sd[t])) shared = sd[t];
        sblock(d, shared, gblk(s, d, k, shared), rk[i], gblk(s, d, k2, shared), r2, Bm + 25 * i);
      }
    }
    /* forward elimination */
    for (int i = 1; i < K && !st; ++i) {
      int r0 = rk[i - 1], r1 = rk[i];
      double Lf[25], X[25], Y[25], z[5];
      memcpy(Lf, Dh + 25 * (i - 1), sizeof(double) * r0 * r0);
      if (chol(r0, Lf)) { st = ORA_ESINGULAR; break; }
      chol_solve_cols(r0, r1, Lf, Bm + 25 * (i - 1), X); /* Dhat^{-1} B */
      mtm(r1, r0, r1, Bm + 25 * (i - 1), X, Y);           /* B^T Dhat^{-1} B */
      for (int e = 0; e < r1 * r1; ++e) Dh[25 * i + e] -= Y[e];
      memcpy(z, bh + 5 * (i - 1), sizeof(double) * r0);
      chol_solve(r0, Lf, z);
      for (int a = 0; a < r1; ++a) {
        double acc = 0.0;
        for (int c = 0; c < r0; ++c) acc += Bm[25 * (i - 1) + c * r1 + a] * z[c];
        bh[5 * i + a] -= acc;
      }
    }
    /* back substitution */
    double xn[5];
    for (int i = K - 1; i >= 0 && !st; --i) {
      int r0 = rk[i];
      double Lf[25], x[5];
      memcpy(x, bh + 5 * i, sizeof(double) * r0);
      if (i + 1 < K)
        for (int a = 0; a < r0; ++a)
          for (int c = 0; c < rk[i + 1]; ++c) x[a] -= Bm[25 * i + a * rk[i + 1] + c] * xn[c];
      memcpy(Lf, Dh + 25 * i, sizeof(double) * r0 * r0);
      if (chol(r0, Lf)) { st = ORA_ESINGULAR; break; }
      chol_solve(r0, Lf, x);
      memcpy(lam + d->roff[ord[i]], x, sizeof(double) * r0);
      memcpy(xn, x, sizeof(double) * r0);
    }
    free(Dh); free(Bm); free(bh); free(rk);
  }
  free(done);
  free(ord);
  return st;
}

/* ------------------------------------------------------------ tree solve */

/* Local KKT of one body with its unary (world-side) rows U:
   [Hh Gu^T; Gu 0] [x; mu] = [rhs; -cu]   (Eq. module3-kkt restricted to U).
   Returns x and, if mu != NULL, the unary multipliers. */
static int local_solve(const double *Lh, int nu, const double *Gu, const double *cu,
                       const double *rhs, double *x, double *mu) {
  double y[12];
  memcpy(y, rhs, sizeof y);
  chol_solve(12, Lh, y);
  if (nu == 0) {
    memcpy(x, y, sizeof y);
    return ORA_OK;
  }
  double GuT[12 * 10], Y[12 * 10], M[100], t[10];
  for (int i = 0; i < 12; ++i)
    for (int j = 0; j < nu; ++j) GuT[i * nu + j] = Gu[j * 12 + i];
  chol_solve_cols(12, nu, Lh, GuT, Y);
  mm(nu, 12, nu, Gu, Y, M);
  if (chol(nu, M)) return ORA_ESINGULAR;
  for (int j = 0; j < nu; ++j) {
    double acc = cu ? cu[j] : 0.0;
    for (int c = 0; c < 12; ++c) acc += Gu[j * 12 + c] * y[c];
    t[j] = acc;
  }
  chol_solve(nu, M, t);
  for (int i = 0; i < 12; ++i) {
    double acc = y[i];
    for (int j = 0; j < nu; ++j) acc -= Y[i * nu + j] * t[j];
    x[i] = acc;
  }
  if (mu) memcpy(mu, t, sizeof(double) * nu);
  return ORA_OK;
}

/* Primal leaf-to-root condensation and root-to-leaf recovery on every tree
   of the body/joint incidence forest (Sec. 5.3, exact form of Eq. module3-kkt). */
static int solve_tree(const ora_system *s, const stepdata *d, double *lam) {
  int n = s->n, m = s->m;
  int st = ORA_OK;
  int *parent = malloc(sizeof(int) * (n + 1)), *pj = malloc(sizeof(int) * (n + 1));
  int *order = malloc(sizeof(int) * (n + 1)), *seen = calloc(n + 1, sizeof(int));
  double *Hh = malloc(sizeof(double) * 144 * (n + 1)), *fh = malloc(sizeof(double) * 12 * (n + 1));
  double *Lh = malloc(sizeof(double) * 144 * (n + 1));
  double *Sk = malloc(sizeof(double) * 25 * (m + 1)), *rho = malloc(sizeof(double) * 5 * (m + 1));
  double *dq = calloc(12 * (n + 1), sizeof(double));
  for (int i = 0; i < n; ++i) {
    if (!is_dyn(s, i)) continue;
    memcpy(Hh + 144 * i, d->H + 144 * i, sizeof(double) * 144);
    memcpy(fh + 12 * i, d->f + 12 * i, sizeof(double) * 12);
  }
  int no = 0;
  /* roots first prefer bodies carrying a unary joint */
  for (int pass = 0; pass < 2; ++pass)
    for (int r = 0; r < n; ++r) {
      if (!is_dyn(s, r) || seen[r]) continue;
      int has_unary = 0;
      for (int e = d->inc.off[r]; e < d->inc.off[r + 1]; ++e) {
        int k = d->inc.jt[e];
        if (!is_dyn(s, s->ja[k]) || !is_dyn(s, s->jb[k])) has_unary = 1;
      }
      if (pass == 0 && !has_unary) continue;
      int head = no;
      order[no++] = r;
      seen[r] = 1;
      parent[r] = -1;
      pj[r] = -1;
      while (head < no) {
        int b = order[head++];
        for (int e = d->inc.off[b]; e < d->inc.off[b + 1]; ++e) {
          int k = d->inc.jt[e];
          int o = s->ja[k] == b ? s->jb[k] : s->ja[k];
          if (!is_dyn(s, o) || seen[o]) continue;
          seen[o] = 1;
          parent[o] = b;
          pj[o] = k;
          order[no++] = o;
        }
      }
    }
  /* unary rows of body b */
  double Gu[10 * 12], cu[10];
#define GATHER_UNARY(b, nu)                                                        \
  do {                                                                             \
    nu = 0;                                                                        \
    for (int e = d->inc.off[b]; e < d->inc.off[b + 1]; ++e) {                      \
      int k = d->inc.jt[e];                                                        \
      if (is_dyn(s, s->ja[k]) && is_dyn(s, s->jb[k])) continue;                    \
      int rk = jrows(s, k);                                                        \
      if (nu + rk > 10) { st = ORA_ETOPO; break; }                                 \
      const double *G = gblk(s, d, k, b);                                          \
      memcpy(Gu + 12 * nu, G, sizeof(double) * 12 * rk);                          \
      memcpy(cu + nu, d->C + 5 * k, sizeof(double) * rk);                          \
      nu += rk;                                                                    \
    }                                                                              \
  } while (0)
  /* leaf to root */
  for (int t = no - 1; t >= 0 && !st; --t) {
    int j = order[t];
    memcpy(Lh + 144 * j, Hh + 144 * j, sizeof(double) * 144);
    if (chol(12, Lh + 144 * j)) { st = ORA_ESINGULAR; break; }
    if (parent[j] < 0) continue;
    int k = pj[j], p = parent[j], rk = jrows(s, k), nu;
    GATHER_UNARY(j, nu);
    if (st) break;
    const double *Gj = gblk(s, d, k, j), *Gp = gblk(s, d, k, p);
    /* S_k = G_kj K_j G_kj^T, rho_k = G_kj (K_j fh_j + o_j) + C_k */
    double X[12 * 5], col[12], xs[12], w[12];
    for (int c = 0; c < rk; ++c) {
      for (int i = 0; i < 12; ++i) col[i] = Gj[c * 12 + i];
      st = local_solve(Lh + 144 * j, nu, Gu, NULL, col, xs, NULL);
      if (st) break;
      for (int i = 0; i < 12; ++i) X[i * rk + c] = xs[i];
    }
    if (st) break;
    mm(rk, 12, rk, Gj, X, Sk + 25 * k);
    st = local_solve(Lh + 144 * j, nu, Gu, cu, fh + 12 * j, w, NULL);
    if (st) break;
    for (int a = 0; a < rk; ++a) {
      double acc = d->C[5 * k + a];
      for (int c = 0; c < 12; ++c) acc += Gj[a * 12 + c] * w[c];
      rho[5 * k + a] = acc;
    }
    /* Hh_p += G_kp^T S_k^{-1} G_kp ;  fh_p -= G_kp^T S_k^{-1} rho_k */
    double Ls[25], SG[5 * 12], z[5];
    memcpy(Ls, Sk + 25 * k, sizeof(double) * rk * rk);
    if (chol(rk, Ls)) { st = ORA_ESINGULAR; break; }
    chol_solve_cols(rk, 12, Ls, Gp, SG);
    double U[144];
    mtm(12, rk, 12, Gp, SG, U);
    for (int e = 0; e < 144; ++e) Hh[144 * p + e] += U[e];
    memcpy(z, rho + 5 * k, sizeof(double) * rk);
    chol_solve(rk, Ls, z);
    for (int i = 0; i < 12; ++i) {
      double acc = 0.0;
      for (int a = 0; a < rk; ++a) acc += Gp[a * 12 + i] * z[a];
      fh[12 * p + i] -= acc;
    }
  }
  /* root to leaf */
  for (int t = 0; t < no && !st; ++t) {
    int j = order[t], nu;
    GATHER_UNARY(j, nu);
    if (st) break;
    double rhs[12], mu[10];
    memcpy(rhs, fh + 12 * j, sizeof rhs);
    if (parent[j] >= 0) {
      int k = pj[j], p = parent[j], rk = jrows(s, k);
      const double *Gj = gblk(s, d, k, j), *Gp = gblk(s, d, k, p);
      double z[5], Ls[25];
      for (int a = 0; a < rk; ++a) {
        double acc = rho[5 * k + a];
        for (int c = 0; c < 12; ++c) acc += Gp[a * 12 + c] * dq[12 * p + c];
        z[a] = acc;
      }
      memcpy(Ls, Sk + 25 * k, sizeof(double) * rk * rk);
      if (chol(rk, Ls)) { st = ORA_ESINGULAR; break; }
      chol_solve(rk, Ls, z);
      memcpy(lam + d->roff[k], z, sizeof(double) * rk);
      for (int i = 0; i < 12; ++i)
        for (int a = 0; a < rk; ++a) rhs[i] -= Gj[a * 12 + i] * z[a];
    }
    st = local_solve(Lh + 144 * j, nu, Gu, cu, rhs, dq + 12 * j, mu);
    if (st) break;
    /* scatter unary multipliers in the same order they were gathered */
    int off = 0;
    for (int e = d->inc.off[j]; e < d->inc.off[j + 1] && nu; ++e) {
      int k = d->inc.jt[e];
      if (is_dyn(s, s->ja[k]) && is_dyn(s, s->jb[k])) continue;
      int rk = jrows(s, k);
      memcpy(lam + d->roff[k], mu + off, sizeof(double) * rk);
      off += rk;
    }
  }
#undef GATHER_UNARY
  free(parent); free(pj); free(order); free(seen); free(Hh); free(fh); free(Lh);
  free(Sk); free(rho); free(dq);
  return st;
}

/* ---------------------------------------------------------- dense / pcg */

/* dual matrix-vector product y = S x, S = sum_b G_b H_b^{-1} G_b^T (Eq. dual) */
static void dual_apply(const ora_system *s, const stepdata *d, const double *x, double *y) {
  memset(y, 0, sizeof(double) * d->nrow);
  for (int b = 0; b < s->n; ++b) {
    if (!is_dyn(s, b)) continue;
    double z[12] = {0};
    for (int e = d->inc.off[b]; e < d->inc.off[b + 1]; ++e) {
      int k = d->inc.jt[e];
      const double *G = gblk(s, d, k, b);
      for (int a = 0; a < jrows(s, k); ++a)
        for (int c = 0; c < 12; ++c) z[c] += G[a * 12 + c] * x[d->roff[k] + a];
    }
    chol_solve(12, d->L + 144 * b, z);
    for (int e = d->inc.off[b]; e < d->inc.off[b + 1]; ++e) {
      int k = d->inc.jt[e];
      const double *G = gblk(s, d, k, b);
      for (int a = 0; a < jrows(s, k); ++a) {
        double acc = 0.0;
        for (int c = 0; c < 12; ++c) acc += G[a * 12 + c] * z[c];
        y[d->roff[k] + a] += acc;
      }
    }
  }
}

static int solve_dense(const ora_system *s, const stepdata *d, double *lam) {
  int N = d->nrow;
  if (N == 0) return ORA_OK;
  double *S = calloc((size_t)N * N, sizeof(double));
  double *r = malloc(sizeof(double) * N);
  if (!S || !r) { free(S); free(r); return ORA_EINVAL; }
  for (int b = 0; b < s->n; ++b) {
    if (!is_dyn(s, b)) continue;
    for (int e = d->inc.off[b]; e < d->inc.off[b + 1]; ++e)
      for (int f = d->inc.off[b]; f < d->inc.off[b + 1]; ++f) {
        int k = d->inc.jt[e], l = d->inc.jt[f], rk = jrows(s, k), rl = jrows(s, l);
        double blk[25];
        sblock(d, b, gblk(s, d, k, b), rk, gblk(s, d, l, b), rl, blk);
        for (int i = 0; i < rk; ++i)
          for (int j = 0; j < rl; ++j) S[(size_t)(d->roff[k] + i) * N + d->roff[l] + j] += blk[i * rl + j];
      }
  }
  for (int k = 0; k < s->m; ++k) dual_rhs(s, d, k, r + d->roff[k]);
  int st = ORA_OK;
  if (chol(N, S)) st = ORA_ESINGULAR;
  else {
    chol_solve(N, S, r);
    memcpy(lam, r, sizeof(double) * N);
  }
  free(S);
  free(r);
  return st;
}

/* block-Jacobi preconditioned CG on the dual system, cold start, stop at
   |r - S lam| <= tol |r| */
static int solve_pcg(const ora_system *s, const stepdata *d, double tol, int maxit, double *lam,
                     int *iters) {
  int N = d->nrow;
  double *b = malloc(sizeof(double) * (N + 1)), *res = malloc(sizeof(double) * (N + 1));
  double *z = malloc(sizeof(double) * (N + 1)), *p = malloc(sizeof(double) * (N + 1));
  double *Ap = malloc(sizeof(double) * (N + 1)), *Pc = malloc(sizeof(double) * 25 * (s->m + 1));
  for (int k = 0; k < s->m; ++k) dual_rhs(s, d, k, b + d->roff[k]);
  int st = ORA_OK;
  for (int k = 0; k < s->m && !st; ++k) {
    int rk = jrows(s, k);
    double *D = Pc + 25 * k;
    memset(D, 0, sizeof(double) * 25);
    int sd[2] = {s->ja[k], s->jb[k]};
    for (int t = 0; t < 2; ++t) {
      const double *G = gblk(s, d, k, sd[t]);
      if (!G) continue;
      double blk[25];
      sblock(d, sd[t], G, rk, G, rk, blk);
      for (int e = 0; e < rk * rk; ++e) D[e] += blk[e];
    }
    if (chol(rk, D)) st = ORA_ESINGULAR;
  }
  double bn = 0.0;
  for (int i = 0; i < N; ++i) bn += b[i] * b[i];
  bn = sqrt(bn);
  memset(lam, 0, sizeof(double) * N);
  memcpy(res, b, sizeof(double) * N);
  int it = 0;
  double rz = 0.0;
  if (!st && bn > 0.0) {
    for (int k = 0; k < s->m; ++k) {
      memcpy(z + d->roff[k], res + d->roff[k], sizeof(double) * jrows(s, k));
      chol_solve(jrows(s, k), Pc + 25 * k, z + d->roff[k]);
    }
    memcpy(p, z, sizeof(double) * N);
    for (int i = 0; i < N; ++i) rz += res[i] * z[i];
    st = ORA_ENOTCONV;
    for (it = 0; it < maxit; ++it) {
      double rn = 0.0;
      for (int i = 0; i < N; ++i) rn += res[i] * res[i];
      if (sqrt(rn) <= tol * bn) { st = ORA_OK; break; }
      dual_apply(s, d, p, Ap);
      double pAp = 0.0;
      for (int i = 0; i < N; ++i) pAp += p[i] * Ap[i];
      double alpha = rz / pAp;
      for (int i = 0; i < N; ++i) {
        lam[i] += alpha * p[i];
        res[i] -= alpha * Ap[i];
      }
      for (int k = 0; k < s->m; ++k) {
        memcpy(z + d->roff[k], res + d->roff[k], sizeof(double) * jrows(s, k));
        chol_solve(jrows(s, k), Pc + 25 * k, z + d->roff[k]);
      }
      double rz2 = 0.0;
      for (int i = 0; i < N; ++i) rz2 += res[i] * z[i];
      double beta = rz2 / rz;
      rz = rz2;
      for (int i = 0; i < N; ++i) p[i] = z[i] + beta * p[i];
    }
    if (st == ORA_ENOTCONV) {
      double rn = 0.0;
      for (int i = 0; i < N; ++i) rn += res[i] * res[i];
      if (sqrt(rn) <= tol * bn) st = ORA_OK;
    }
  }
  if (iters) *iters = it;
  free(b); free(res); free(z); free(p); free(Ap); free(Pc);
  return st;
}

/* ----------------------------------------------- back-projection, residuals */

/* dq_b = H_b^{-1} (f_b - sum_k G_kb^T lam_k)  (Eq. primal) */
static void back_project(const ora_system *s, const stepdata *d, const double *lam, double *dq) {
#pragma omp parallel for schedule(static)
  for (int b = 0; b < s->n; ++b) {
    double *x = dq + 12 * b;
    memset(x, 0, sizeof(double) * 12);
    if (!is_dyn(s, b)) continue;
    memcpy(x, d->f + 12 * b, sizeof(double) * 12);
    for (int e = d->inc.off[b]; e < d->inc.off[b + 1]; ++e) {
      int k = d->inc.jt[e];
      const double *G = gblk(s, d, k, b);
      for (int a = 0; a < jrows(s, k); ++a)
        for (int c = 0; c < 12; ++c) x[c] -= G[a * 12 + c] * lam[d->roff[k] + a];
    }
    chol_solve(12, d->L + 144 * b, x);
  }
}

/* rho_p = |H^{-1} r_p| / |H^{-1} f|, rho_d = |G dq + C| / |G H^{-1} f + C| */
/* length-preserving stand-in for a rotation (Eq. len_preserving): M x scaled
   to the length of x; x itself if M x vanishes */
static void lenpres(const double *M, int transpose, const double *x, double *y) {
  if (transpose) mtm(3, 3, 1, M, x, y);
  else mm(3, 3, 1, M, x, y);
  double lx = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  double ly = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
  if (ly > 0.0)
    for (int r = 0; r < 3; ++r) y[r] *= lx / ly;
  else
    for (int r = 0; r < 3; ++r) y[r] = x[r];
}

/* a dynamic body that no joint touches */
static int unjointed(const ora_system *s, int b) {
  for (int k = 0; k < s->m; ++k)
    if (s->ja[k] == b || s->jb[k] == b) return 0;
  return 1;
}

/* The polar-free single-body solve of Alg. 1 for body i at the iterate qi:
   every rotation of a 3-block by R (Eq. polar) is replaced by the
   length-preserving action of A (Eq. len_preserving): R^T x by A^T x scaled to
   |x|, R y by A y scaled to |y|.  The forces of the Newton step (inertia,
   gravity, external wrench; Eq. variation_energy) are taken to the body frame
   so, the rotated elastic force -V P(R^T A) (Eq. reduced_K) uses the same
   stand-in for R^T A column by column, the constant Hbar (Eq. abd_final) is
   solved, and the increment is taken back to the world frame block by
   block. */
static int polar_free_dq(const ora_system *s, double h, const double *qi, const double *qn,
                         const double *qdn, int i, double *dq) {
  double A[9], Mbar[4], V, m, mu, lam, Hb[144];
  q_to_A(qi, A);
  box_mass(s, i, Mbar, &V, &m);
  lame(s, i, &mu, &lam);
  hbar(s, i, h, Hb);
  double w[12];
  for (int a = 0; a < 12; ++a) {
    int c = a / 3, r = a % 3;
    double M = Mbar[c];
    double fext = (c == 3) ? s->gravity[r] * m : 0.0;
    w[a] = M * qdn[a] / h - M * (qi[a] - qn[a]) / (h * h) + fext;
  }
  if (s->wrench) {
    const double *tau = s->wrench + 6 * i, *fw = tau + 3;
    for (int c = 0; c < 3; ++c) {
      const double *qc = qi + 3 * c;
      w[3 * c + 0] += 0.5 * (tau[1] * qc[2] - tau[2] * qc[1]);
      w[3 * c + 1] += 0.5 * (tau[2] * qc[0] - tau[0] * qc[2]);
      w[3 * c + 2] += 0.5 * (tau[0] * qc[1] - tau[1] * qc[0]);
    }
    for (int r = 0; r < 3; ++r) w[9 + r] += fw[r];
  }
  /* R^T A column by column, then P of Sec. 3.3 in the body frame */
  double Sh[9], P[9];
  for (int c = 0; c < 3; ++c) {
    double col[3] = {A[c], A[3 + c], A[6 + c]}, x[3];
    lenpres(A, 1, col, x);
    for (int r = 0; r < 3; ++r) Sh[r * 3 + c] = x[r];
  }
  double tr = Sh[0] + Sh[4] + Sh[8] - 3.0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      P[r * 3 + c] = mu * (Sh[r * 3 + c] + Sh[c * 3 + r] - 2.0 * (r == c)) + lam * tr * (r == c);
  double phi[12];
  for (int k = 0; k < 4; ++k) lenpres(A, 1, w + 3 * k, phi + 3 * k);
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < 3; ++r) phi[3 * c + r] -= V * P[r * 3 + c];
  double L[144], dp[12];
  memcpy(L, Hb, sizeof L);
  if (chol(12, L)) return ORA_ESINGULAR;
  memcpy(dp, phi, sizeof dp);
  chol_solve(12, L, dp);
  for (int k = 0; k < 4; ++k) lenpres(A, 0, dp + 3 * k, dq + 3 * k);
  for (int a = 0; a < 12; ++a)
    if (!isfinite(dq[a])) return ORA_ENONFINITE;
  return ORA_OK;
}

/* bodies that take the polar-free solve: unjointed dynamic bodies, when asked */
static int polar_free_body(const ora_system *s, int b) {
  return s->body_solve == 1 && is_dyn(s, b) && unjointed(s, b);
}

static void kkt_residual(const ora_system *s, const stepdata *d, const double *lam,
                         const double *dq, double *rho_p, double *rho_d) {
  double np = 0.0, nf = 0.0, nd = 0.0, nr = 0.0;
  for (int b = 0; b < s->n; ++b) {
    /* a polar-free body does not solve the co-rotated system of Eq. kkt */
    if (!is_dyn(s, b) || polar_free_body(s, b)) continue;
    double rp[12], hf[12];
    mm(12, 12, 1, d->H + 144 * b, dq + 12 * b, rp);
    for (int c = 0; c < 12; ++c) rp[c] -= d->f[12 * b + c];
    for (int e = d->inc.off[b]; e < d->inc.off[b + 1]; ++e) {
      int k = d->inc.jt[e];
      const double *G = gblk(s, d, k, b);
      for (int a = 0; a < jrows(s, k); ++a)
        for (int c = 0; c < 12; ++c) rp[c] += G[a * 12 + c] * lam[d->roff[k] + a];
    }
    chol_solve(12, d->L + 144 * b, rp);
    memcpy(hf, d->f + 12 * b, sizeof hf);
    chol_solve(12, d->L + 144 * b, hf);
    for (int c = 0; c < 12; ++c) {
      np += rp[c] * rp[c];
      nf += hf[c] * hf[c];
    }
  }
  for (int k = 0; k < s->m; ++k) {
    int rk = jrows(s, k);
    double rd[5], rr[5];
    for (int a = 0; a < rk; ++a) rd[a] = d->C[5 * k + a];
    int sd[2] = {s->ja[k], s->jb[k]};
    for (int t = 0; t < 2; ++t) {
      const double *G = gblk(s, d, k, sd[t]);
      if (!G) continue;
      for (int a = 0; a < rk; ++a)
        for (int c = 0; c < 12; ++c) rd[a] += G[a * 12 + c] * dq[12 * sd[t] + c];
    }
    dual_rhs(s, d, k, rr);
    for (int a = 0; a < rk; ++a) {
      nd += rd[a] * rd[a];
      nr += rr[a] * rr[a];
    }
  }
  *rho_p = nf > 0.0 ? sqrt(np / nf) : sqrt(np);
  *rho_d = nr > 0.0 ? sqrt(nd / nr) : sqrt(nd);
}

static void post_constraints(const ora_system *s, const double *q, double *cball, double *chinge) {
  *cball = 0.0;
  *chinge = 0.0;
  for (int k = 0; k < s->m; ++k) {
    double C[5], Ga[60], Gb[60];
    if (joint_terms(s, q, k, C, Ga, Gb)) continue;
    for (int a = 0; a < jrows(s, k); ++a) {
      double v = fabs(C[a]);
      if (s->jtype[k] == 0) { if (v > *cball) *cball = v; }
      else if (v > *chinge) *chinge = v;
    }
  }
}

/* ---------------------------------------------------------------- driver */

int32_t ora_step(const ora_system *s, double h, double *q, double *qd, int32_t solver,
                 double tol, int32_t max_iters, double *lam, double *diag) {
  if (!(h > 0.0)) return ORA_EINVAL;
  int st = validate(s);
  if (st) return st;
  int cls = ora_classify(s);
  if (solver == ORA_AUTO) solver = cls == 1 ? ORA_CHAIN : cls == 2 ? ORA_TREE : ORA_DENSE;
  if (solver == ORA_CHAIN && cls != 1) return ORA_ETOPO;
  if (solver == ORA_TREE && cls == 3) return ORA_ETOPO;
  int iters = s->newton_iters > 0 ? s->newton_iters : 1;
  size_t n = s->n;
  double *qn = malloc(sizeof(double) * 12 * (n + 1)), *qi = malloc(sizeof(double) * 12 * (n + 1));
  double *dq = malloc(sizeof(double) * 12 * (n + 1));
  double *dsum = calloc(12 * (n + 1), sizeof(double)); /* q^{n+1} - q^n, summed exactly */
  int nrow = ora_rows(s);
  double *lw = calloc(nrow + 1, sizeof(double));
  memcpy(qn, q, sizeof(double) * 12 * n);
  memcpy(qi, q, sizeof(double) * 12 * n);
  double rp = 0.0, rd = 0.0;
  int pcg_it = 0;
  for (int it = 0; it < iters && !st; ++it) {
    stepdata d;
    st = build_sd(s, h, qi, qn, qd, &d);
    if (!st) {
      if (solver == ORA_CHAIN) st = solve_chain(s, &d, lw);
      else if (solver == ORA_TREE) st = solve_tree(s, &d, lw);
      else if (solver == ORA_DENSE) st = solve_dense(s, &d, lw);
      else st = solve_pcg(s, &d, tol, max_iters, lw, &pcg_it);
    }
    if (!st || st == ORA_ENOTCONV) {
      back_project(s, &d, lw, dq);
      for (int b = 0; b < s->n && !st; ++b)
        if (polar_free_body(s, b))
          st = polar_free_dq(s, h, qi + 12 * b, qn + 12 * b, qd + 12 * b, b, dq + 12 * b);
      kkt_residual(s, &d, lw, dq, &rp, &rd);
      for (size_t a = 0; a < 12 * n; ++a) {
        qi[a] += dq[a];
        dsum[a] += dq[a];
      }
    }
    free_sd(&d);
  }
  int final_st = st;
  if (!st || st == ORA_ENOTCONV) {
    for (size_t a = 0; a < 12 * n; ++a)
      if (!isfinite(qi[a])) final_st = ORA_ENONFINITE;
  }
  if (final_st == ORA_OK || final_st == ORA_ENOTCONV) {
    for (size_t b = 0; b < n; ++b)
      for (int c = 0; c < 12; ++c) {
        if (s->pinned[b]) {
          qd[12 * b + c] = 0.0;
          continue;
        }
        /* implicit Euler velocity (q^{n+1} - q^n) / h, from the increments so
           that large coordinates do not cancel */
        qd[12 * b + c] = dsum[12 * b + c] / h;
        q[12 * b + c] = qi[12 * b + c];
      }
    if (lam) memcpy(lam, lw, sizeof(double) * nrow);
  }
  if (diag) {
    for (int i = 0; i < ORA_NDIAG; ++i) diag[i] = 0.0;
    diag[ORA_RHO_P] = rp;
    diag[ORA_RHO_D] = rd;
    diag[ORA_KKT] = rp > rd ? rp : rd;
    post_constraints(s, q, &diag[ORA_CBALL], &diag[ORA_CHINGE]);
    diag[ORA_ITERS] = pcg_it;
    diag[ORA_SOLVER] = solver;
  }
  free(qn); free(qi); free(dq); free(dsum); free(lw);
  return final_st;
}

/* dual system in coordinate form: blocks of S and the right-hand side r */
int64_t ora_dual_coo(const ora_system *s, double h, const double *q, const double *qd,
                     int64_t cap, int64_t *I, int64_t *J, double *V, double *r) {
  if (validate(s)) return ORA_EINVAL;
  stepdata d;
  int st = build_sd(s, h, q, q, qd, &d);
  if (st) { free_sd(&d); return st; }
  int64_t nnz = 0;
  for (int b = 0; b < s->n; ++b) {
    if (!is_dyn(s, b)) continue;
    for (int e = d.inc.off[b]; e < d.inc.off[b + 1]; ++e)
      for (int f = d.inc.off[b]; f < d.inc.off[b + 1]; ++f) {
        int k = d.inc.jt[e], l = d.inc.jt[f], rk = jrows(s, k), rl = jrows(s, l);
        double blk[25];
        sblock(&d, b, gblk(s, &d, k, b), rk, gblk(s, &d, l, b), rl, blk);
        for (int i = 0; i < rk; ++i)
          for (int j = 0; j < rl; ++j) {
            if (nnz < cap) {
              I[nnz] = d.roff[k] + i;
              J[nnz] = d.roff[l] + j;
              V[nnz] = blk[i * rl + j];
            }
            nnz++;
          }
      }
  }
  if (r)
    for (int k = 0; k < s->m; ++k) dual_rhs(s, &d, k, r + d.roff[k]);
  free_sd(&d);
  return nnz;
}

/* one Newton iteration's back-projection and diagnostics for given multipliers */
int32_t ora_finish(const ora_system *s, double h, const double *q, const double *qd,
                   const double *lam, double *q_out, double *qd_out, double *diag) {
  if (validate(s)) return ORA_EINVAL;
  stepdata d;
  int st = build_sd(s, h, q, q, qd, &d);
  if (st) { free_sd(&d); return st; }
  size_t n = s->n;
  double *dq = malloc(sizeof(double) * 12 * (n + 1));
  back_project(s, &d, lam, dq);
  for (int b = 0; b < s->n && !st; ++b)
    if (polar_free_body(s, b)) st = polar_free_dq(s, h, q + 12 * b, q + 12 * b, qd + 12 * b, b, dq + 12 * b);
  if (st) { free(dq); free_sd(&d); return st; }
  double rp, rd;
  kkt_residual(s, &d, lam, dq, &rp, &rd);
  for (size_t b = 0; b < n; ++b)
    for (int c = 0; c < 12; ++c) {
      q_out[12 * b + c] = q[12 * b + c] + (s->pinned[b] ? 0.0 : dq[12 * b + c]);
      qd_out[12 * b + c] = s->pinned[b] ? 0.0 : dq[12 * b + c] / h;
    }
  if (diag) {
    for (int i = 0; i < ORA_NDIAG; ++i) diag[i] = 0.0;
    diag[ORA_RHO_P] = rp;
    diag[ORA_RHO_D] = rd;
    diag[ORA_KKT] = rp > rd ? rp : rd;
    post_constraints(s, q_out, &diag[ORA_CBALL], &diag[ORA_CHINGE]);
  }
  free(dq);
  free_sd(&d);
  return ORA_OK;
}

/* The verifier: KKT residuals (oracle diagnostics, Eq. kkt) of a step given
   from outside as an increment dq and multipliers lam for the state (q, qd),
   one Newton iteration; post-step constraint values at q_new (at q + dq when
   q_new is NULL).  Nothing is solved here. */
int32_t ora_residual(const ora_system *s, double h, const double *q, const double *qd,
                     const double *dq, const double *lam, const double *q_new, double *diag) {
  if (validate(s)) return ORA_EINVAL;
  stepdata d;
  int st = build_sd(s, h, q, q, qd, &d);
  if (st) { free_sd(&d); return st; }
  size_t n = s->n;
  double *dqd = malloc(sizeof(double) * 12 * (n + 1));
  double *qe = malloc(sizeof(double) * 12 * (n + 1));
  for (size_t b = 0; b < n; ++b)
    for (int c = 0; c < 12; ++c) {
      dqd[12 * b + c] = is_dyn(s, (int)b) ? dq[12 * b + c] : 0.0;
      qe[12 * b + c] = q_new ? q_new[12 * b + c] : q[12 * b + c] + dqd[12 * b + c];
    }
  double rp, rd;
  kkt_residual(s, &d, lam, dqd, &rp, &rd);
  if (diag) {
    for (int i = 0; i < ORA_NDIAG; ++i) diag[i] = 0.0;
    diag[ORA_RHO_P] = rp;
    diag[ORA_RHO_D] = rd;
    diag[ORA_KKT] = rp > rd ? rp : rd;
    post_constraints(s, qe, &diag[ORA_CBALL], &diag[ORA_CHINGE]);
  }
  free(dqd);
  free(qe);
  free_sd(&d);
  return ORA_OK;
}

/* Spatial twist of every body (Eq. module1-G-twist): V = G(A) qdot with
   omega = 1/2 sum_c q_c x qdot_c (q_c the c-th column of A) and v = tdot;
   V holds n*6 values [omega; v], zero for pinned bodies. */
int32_t ora_twists(const ora_system *s, const double *q, const double *qd, double *V) {
  if (validate(s)) return ORA_EINVAL;
  for (int b = 0; b < s->n; ++b) {
    double *o = V + 6 * (size_t)b;
    for (int i = 0; i < 6; ++i) o[i] = 0.0;
    if (!is_dyn(s, b)) continue;
    for (int c = 0; c < 3; ++c) {
      const double *a = q + 12 * (size_t)b + 3 * c, *ad = qd + 12 * (size_t)b + 3 * c;
      o[0] += 0.5 * (a[1] * ad[2] - a[2] * ad[1]);
      o[1] += 0.5 * (a[2] * ad[0] - a[0] * ad[2]);
      o[2] += 0.5 * (a[0] * ad[1] - a[1] * ad[0]);
    }
    for (int i = 0; i < 3; ++i) o[3 + i] = qd[12 * (size_t)b + 9 + i];
  }
  return ORA_OK;
}

/* Joint wrench on every body: the spatial wrench (world frame, about the
   centre of mass) that does the same virtual work on rigid motions as the
   generalised joint force -sum_k G_kb^T lam_k of a step from q (the force
   term of the primal rows of Eq. kkt), W = E(A)^T f with the rigid-motion
   embedding E(A) of Eq. module2-E: W = [sum_c q_c x f_c; f_t].  G is taken
   at q; W holds n*6 values [tau; f], zero for pinned bodies. */
int32_t ora_joint_wrenches(const ora_system *s, const double *q, const double *lam, double *W) {
  if (validate(s)) return ORA_EINVAL;
  size_t n = s->n;
  double *f = calloc(12 * (n ? n : 1), sizeof(double));
  int off = 0;
  for (int k = 0; k < s->m; ++k) {
    double C[5], Ga[60], Gb[60];
    int rk = jrows(s, k);
    int st = joint_terms(s, q, k, C, Ga, Gb);
    if (st) { free(f); return st; }
    for (int side = 0; side < 2; ++side) {
      int b = side ? s->jb[k] : s->ja[k];
      if (!is_dyn(s, b)) continue;
      const double *G = side ? Gb : Ga;
      for (int c = 0; c < 12; ++c)
        for (int i = 0; i < rk; ++i) f[12 * (size_t)b + c] -= G[i * 12 + c] * lam[off + i];
    }
    off += rk;
  }
  for (size_t b = 0; b < n; ++b) {
    double *o = W + 6 * b;
    const double *fb = f + 12 * b, *qb = q + 12 * b;
    for (int i = 0; i < 6; ++i) o[i] = 0.0;
    if (!is_dyn(s, (int)b)) continue;
    for (int c = 0; c < 3; ++c) {
      const double *a = qb + 3 * c, *fc = fb + 3 * c;
      o[0] += a[1] * fc[2] - a[2] * fc[1];
      o[1] += a[2] * fc[0] - a[0] * fc[2];
      o[2] += a[0] * fc[1] - a[1] * fc[0];
    }
    for (int i = 0; i < 3; ++i) o[3 + i] = fb[9 + i];
  }
  free(f);
  return ORA_OK;
}
