// Generic-topology kernels of libmabd: per-shape factors, per-body co-rotated
// solve, per-joint rows, tree elimination, back-projection, state gather.
#include <algorithm>

#include "common.hpp"
#include "dmath.hpp"
#include "generic.hpp"

namespace mabd {

// -------------------------------------------------------------- a0: factors
// Hbar = M_A / h^2 + Kbar_A of a box (Eq. abd_final) inverted block by block.
__global__ void prefactor_kernel(const double *shape, int nshape, double h, double *hinv) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nshape) return;
  const double *sh = shape + (int64_t)SHAPE_STRIDE * s;
  double *T = hinv + (int64_t)HINV_STRIDE * s;
  const double ih2 = 1.0 / (h * h);
  const double m = sh[3], V = sh[4], mu = sh[5], lam = sh[6];
  const double M[3] = {sh[0] * ih2, sh[1] * ih2, sh[2] * ih2};
  T[HI_T] = 1.0 / (m * ih2);
  // (A00, A11, A22): diag(M_r + 2 V mu) + V lam 11^T, Sherman-Morrison
  double dinv[3], sum = 0.0;
  for (int r = 0; r < 3; ++r) {
    dinv[r] = 1.0 / (M[r] + 2.0 * V * mu);
    sum += dinv[r];
  }
  const double gam = V * lam / (1.0 + V * lam * sum);
  double Dm[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Dm[3 * r + c] = (r == c ? dinv[r] : 0.0) - gam * dinv[r] * dinv[c];
  T[HI_D + 0] = Dm[0]; T[HI_D + 1] = Dm[1]; T[HI_D + 2] = Dm[2];
  T[HI_D + 3] = Dm[4]; T[HI_D + 4] = Dm[5]; T[HI_D + 5] = Dm[8];
  // off-diagonal pairs (A_rc in column c, A_cr in column r):
  // [[M_c + V mu, V mu], [V mu, M_r + V mu]]
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      if (r == c) { T[HI_PD + 3 * r + c] = 0.0; continue; }
      const double e1 = M[c] + V * mu, e2 = M[r] + V * mu, o = V * mu;
      const double det = e1 * e2 - o * o;
      T[HI_PD + 3 * r + c] = e2 / det;  // inverse entry of A_rc
      if (r < c) T[HI_PX + pair_slot(r, c)] = -o / det;
    }
  T[19] = 0.0;
}

// ------------------------------------------------------- (a) generic bodies
// R and the local unconstrained increment u = Hbar^{-1} diag4(R^T) f_A for
// bodies [b0, b1) (Eqs. polar, abd_final).  q is the current iterate, qn/qdn
// the state at the start of the step.
// With pf_inc (the bodies' incidence offsets) given, bodies without joints
// take the polar-free solve of Alg. 1 instead: no polar decomposition, the
// length-preserving stand-ins of local_force_lp, R stored as the identity
// (unused: the back-projection applies the stand-in again).
// With fa.inc_off given, a body without joints also takes its back-projection
// here (it has no multipliers: dq = R u, or the stand-in of Alg. 1), exactly
// as gapply_kernel would, which then skips it: q_out = q + dq and
// qd_out = (fa.acc ? qd_out : 0) + dq / h, without the round trip of u.
struct FreeApply {
  const int32_t *inc_off;  // null: no body is applied here
  double *q_out, *qd_out, *dq_save;
  int acc;
};
DEV void free_apply(const FreeApply &fa, int64_t ns, int64_t b, const double *q, const double *dq, double h,
                    uint32_t *status, int step) {
  const double ih = 1.0 / h;
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    const int64_t o = (int64_t)i * ns + b;
    fa.q_out[o] = q[i] + dq[i];
    fa.qd_out[o] = (fa.acc ? fa.qd_out[o] : 0.0) + dq[i] * ih;
    if (fa.dq_save) fa.dq_save[o] = dq[i];
    if (!isfinite(dq[i])) raise_flag(status, FLAG_NONFINITE, step);
  }
}
__global__ __launch_bounds__(256) void gbody_kernel(int b0, int b1, const double *q, const double *qn, const double *qdn,
                             int64_t ns, const int32_t *shp, const double *hinv,
                             const double *shape, double g0, double g1, double g2, double h,
                             double *Rg, double *ug, uint32_t *status, int step, const double *wr,
                             const int32_t *pf_inc, int f32, FreeApply fa) {
  int64_t b = (int64_t)b0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= b1 || skip_step(status, step)) return;
  const bool fused = fa.inc_off && fa.inc_off[b] == fa.inc_off[b + 1];
  if (pf_inc && pf_inc[b] == pf_inc[b + 1]) {
    double qq[12], qnn[12], qd[12], A[9];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      qq[c] = q[c * ns + b];
      qnn[c] = qn[c * ns + b];
      qd[c] = qdn[c * ns + b];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) A[3 * i + c] = qq[3 * c + i];
    const int s = shp[b];
    const double g[3] = {g0, g1, g2};
    double phi[12], u[12];
    local_force_lp(shape + (int64_t)SHAPE_STRIDE * s, A, qq, qnn, qd, g, h, phi, wr, ns, b);
    hinv_apply(hinv + (int64_t)HINV_STRIDE * s, phi, u);
#pragma unroll
    for (int i = 0; i < 9; ++i) Rg[i * ns + b] = (i % 4 == 0) ? 1.0 : 0.0;
    if (fused) {
      double dq[12];
#pragma unroll
      for (int c = 0; c < 4; ++c) lenpres(A, false, u + 3 * c, dq + 3 * c);
      free_apply(fa, ns, b, qq, dq, h, status, step);
      return;
    }
#pragma unroll
    for (int i = 0; i < 12; ++i) ug[i * ns + b] = u[i];
    return;
  }
  double qq[12], qnn[12], qd[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    qq[c] = q[c * ns + b];
    qnn[c] = qn[c * ns + b];
    qd[c] = qdn[c * ns + b];
  }
  double A[9], R[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) A[3 * i + c] = qq[3 * c + i];
  if (!polar3(A, R)) {
    raise_flag(status, FLAG_NONFINITE, step);
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
  }
  const int s = shp[b];
  const double g[3] = {g0, g1, g2};
#pragma unroll
  for (int i = 0; i < 9; ++i) Rg[i * ns + b] = R[i];
  if (f32) {
    // precision form 1: the rotation stays FP64 (it defines the system the
    // FP64 refinement solves); force and local solve in FP32.  The force
    // is formed from the iterate's offset to the step's start, so that FP32
    // sees only the step's increments, not absolute positions.
    float Rf[9], Af[9], qf[12], qnf[12], qdf[12], phif[12], uf[12];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      Rf[i] = (float)R[i];
      Af[i] = (float)A[i];
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      qnf[c] = (float)qnn[c];
      qf[c] = qnf[c] + (float)(qq[c] - qnn[c]);
      qdf[c] = (float)qd[c];
    }
    local_force<float>(shape + (int64_t)SHAPE_STRIDE * s, Rf, Af, qf, qnf, qdf, g, h, phif, wr, ns, b);
    hinv_apply(hinv + (int64_t)HINV_STRIDE * s, phif, uf);
    if (fused) {
      double u[12], dq[12];
#pragma unroll
      for (int i = 0; i < 12; ++i) u[i] = (double)uf[i];
#pragma unroll
      for (int c = 0; c < 4; ++c) mat3_vec(R, u + 3 * c, dq + 3 * c);
      free_apply(fa, ns, b, qq, dq, h, status, step);
      return;
    }
#pragma unroll
    for (int i = 0; i < 12; ++i) ug[i * ns + b] = (double)uf[i];
    return;
  }
  double phi[12], u[12];
  local_force<double>(shape + (int64_t)SHAPE_STRIDE * s, R, A, qq, qnn, qd, g, h, phi, wr, ns, b);
  hinv_apply(hinv + (int64_t)HINV_STRIDE * s, phi, u);
  if (fused) {
    double dq[12];
#pragma unroll
    for (int c = 0; c < 4; ++c) mat3_vec(R, u + 3 * c, dq + 3 * c);
    free_apply(fa, ns, b, qq, dq, h, status, step);
    return;
  }
#pragma unroll
  for (int i = 0; i < 12; ++i) ug[i * ns + b] = u[i];
}

// ------------------------------------------------------- (b) generic joints
// Constraint value C and the local-frame gradients L = G diag4(R) of both
// sides (Eq. ball; Eqs. hinge, universal, prismatic with Eqs. pcpq, pcpr,
// r_gradient).  For a ball end L = s R J(p).  A rotated-frame joint's row is
// component comp of R_J (y_X - y_Y): on the frame owner a its frozen part is
// dR_comp J(p) for a's points, plus the A-linearised rotation term
// (dR_comp (x) R_a^T d) on the A columns; on side b it is (R_J R_b)_comp J(p)
// for b's points (with the signs of X and Y).
// Rows of a rotated-frame joint (hinge, universal, prismatic; Secs. 4.3-4.5)
// of type TYPE: row i is component comp of R_J (y_X - y_Y) with
// R_J = dR R_a^T.  The row loop is unrolled over the compile-time row table,
// so every point and component index is a constant (the joint record stays
// in registers).
template <int TYPE>
DEV void gjoint_rot_rows(const GJoint &j, const double *Aa, const double *ta, const double *Ab,
                         const double *tb, const double *Ra, const double *Rb, bool da, bool db,
                         int hinge_grad, double *out) {
  double RH[9];
  if (j.flags & GJ_FLAG_STATIC_OWNER) {
#pragma unroll
    for (int i = 0; i < 9; ++i) RH[i] = j.dR[i];
  } else {
    mat3_mul_bt(j.dR, Ra, RH);  // R_J = dR R_a^T
  }
  double Q[9];  // R_J R_b: rows of side b's local-frame gradient
  mat3_mul(RH, Rb, Q);
  const double *P[5] = {j.p1a, j.p2a, j.p1b, j.p2b, j.p3b};
  constexpr int ROWS = TYPE == 2 ? 4 : 5;
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const JointRow jr = joint_row(TYPE, i);
    // y_X - y_Y: across the joint translation difference first; on one body
    // its affine block times the difference of the rest points
    double d[3];
    if (point_side(jr.x) != point_side(jr.y)) {
      double wa[3], wb[3];
      mat3_vec(Aa, P[jr.x], wa);
      mat3_vec(Ab, P[jr.y], wb);
#pragma unroll
      for (int r = 0; r < 3; ++r) d[r] = (ta[r] - tb[r]) + (wa[r] - wb[r]);
    } else {
      const double dp[3] = {P[jr.x][0] - P[jr.y][0], P[jr.x][1] - P[jr.y][1], P[jr.x][2] - P[jr.y][2]};
      mat3_vec(point_side(jr.x) ? Ab : Aa, dp, d);
    }
    const double *rh = RH + 3 * jr.comp;
    out[GL_C + i] = rh[0] * d[0] + rh[1] * d[1] + rh[2] * d[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (side == 0 ? !da : !db) continue;
      // frozen frame: the rotated row times J(p) in the side's local frame
      // (dR row on side a, since J(p) diag4(R_a) = R_a J(p); (R_J R_b) row on b)
      const double *rr = side == 0 ? j.dR + 3 * jr.comp : Q + 3 * jr.comp;
      double L[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) L[c] = 0.0;
#pragma unroll
      for (int pt = 0; pt < 2; ++pt) {
        const int id = pt == 0 ? jr.x : jr.y;
        if (point_side(id) != side) continue;
        const double sg = pt == 0 ? 1.0 : -1.0;
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
#pragma unroll
          for (int c = 0; c < 3; ++c) L[3 * c + jj] += sg * rr[jj] * P[id][c];
          L[9 + jj] += sg * rr[jj];
        }
      }
      if (side == 0 && hinge_grad == 0) {
        // A-linearised rotation term of the frame owner (Eqs. pcpr,
        // r_gradient): dR_comp (x) R_a^T d on a's A columns
        double w[3];
        mat3t_vec(Ra, d, w);
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
          for (int kk = 0; kk < 3; ++kk) L[3 * l + kk] += rr[l] * w[kk];
      }
      double *Lo = out + (side == 0 ? GL_LA : GL_LB) + 12 * i;
#pragma unroll
      for (int c = 0; c < 12; ++c) Lo[c] = L[c];
    }
  }
}

__global__ __launch_bounds__(128) void gjoint_kernel(int m, const GJoint *J, const double *q, const double *Rg, int64_t ns,
                              int hinge_grad, double *gl) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const GJoint j = J[k];
  double *out = gl + (int64_t)GL_STRIDE * k;
  double Aa[9], ta[3], Ab[9], tb[3], Ra[9], Rb[9];
  const bool da = j.sa >= 0, db = j.sb >= 0;
  auto load_side = [&](int64_t b, double *A, double *t, double *R) {
    if (b >= 0) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int c = 0; c < 3; ++c) A[3 * i + c] = q[(3 * c + i) * ns + b];
        t[i] = q[(9 + i) * ns + b];
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) R[i] = Rg[i * ns + b];
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) { A[i] = (i % 4 == 0) ? 1.0 : 0.0; R[i] = A[i]; }
      t[0] = t[1] = t[2] = 0.0;
    }
  };
  load_side(j.sa, Aa, ta, Ra);
  load_side(j.sb, Ab, tb, Rb);
  if (j.type == 0) {
    double C[3], wa[3], wb[3];
    mat3_vec(Aa, j.p1a, wa);
    mat3_vec(Ab, j.p1b, wb);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      C[i] = (ta[i] - tb[i]) + (wa[i] - wb[i]);
      out[GL_C + i] = C[i];
    }
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (side == 0 ? !da : !db) continue;
      const double *R = side == 0 ? Ra : Rb;
      const double *p = side == 0 ? j.p1a : j.p1b;
      const double s = side == 0 ? 1.0 : -1.0;
      double *L = out + (side == 0 ? GL_LA : GL_LB);
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
#pragma unroll
          for (int c = 0; c < 3; ++c) L[12 * r + 3 * c + i] = s * R[3 * r + i] * p[c];
          L[12 * r + 9 + i] = s * R[3 * r + i];
        }
    }
    return;
  }
  if (j.type == 1)
    gjoint_rot_rows<1>(j, Aa, ta, Ab, tb, Ra, Rb, da, db, hinge_grad, out);
  else if (j.type == 2)
    gjoint_rot_rows<2>(j, Aa, ta, Ab, tb, Ra, Rb, da, db, hinge_grad, out);
  else
    gjoint_rot_rows<3>(j, Aa, ta, Ab, tb, Ra, Rb, da, db, hinge_grad, out);
}

// ------------------------------------------------------ (c2) tree solve
// Leaf-to-root block elimination of the dual system (Sec. 5.3; the exact tree
// KKT solution of Eq. module3-kkt).  In the dual graph the joints incident to
// one body form a clique (Fig. dual_mat).  Body j gathers the rows of its
// absorbed joints e (joints to its children, whose far side is already
// condensed into (Sigma, rho), and one-sided joints) and of its parent joint k:
//   K = [L_e; L_k] Hbar_j^{-1} [L_e; L_k]^T + diag(Sigma_e, 0),
//   y = [L_e; L_k] u_j + [rho_e or C_e; C_k],
// and factors the e-block by Cholesky: K_ee = Lc Lc^T, X = Lc^{-1} K_ek,
// z = Lc^{-1} y_e.  The Schur complement Sigma_k = K_kk - X^T X and
// rho_k = y_k - X^T z are the condensed far side of joint k seen from its
// parent.  Root to leaf, lambda_e = Lc^{-T} (z - X lambda_k).  This is block
// Cholesky of the SPD dual matrix in a perfect elimination order, so it keeps
// the backward stability of a dense Cholesky of S.
// A team of 16 lanes handles one body; cliques of up to TREE_KLDS rows are
// factored in LDS, larger ones in the body's global slot.
constexpr int TEAMS = 16;
constexpr int TREE_BLOCK = TEAMS * TEAM;


DEV void team_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Clique matrix of one body without its children's condensed far sides:
// K0 = L Hbar^{-1} L^T (lower triangle) and y0 = L u + C (C of one-sided and
// parent joints), written to the body's factor slot.  Independent of every
// other body, so all bodies of all components run in one parallel pre-pass;
// the level-ordered elimination then only adds the children's Sigma, rho and
// factors.
struct PrepLds {
  double L[TREE_KLDS * 12];
  double th[HINV_STRIDE];   // Hbar^{-1} of the body
  double uu[12];            // its local solve u
  int ek[24];               // clique entries: joint,
  int ei[24];               // first row << 8 | rows << 4 | unary << 1 | side
  uint8_t rowent[TREE_KMAX];  // clique row -> entry
};

__global__ __launch_bounds__(TREE_BLOCK) void tree_prep_kernel(TreeArgs a, const GJoint *J, int nslots) {
  __shared__ PrepLds team_lds[TEAMS];
  const int tm = threadIdx.x / TEAM, ln = threadIdx.x % TEAM;
  PrepLds &S = team_lds[tm];
  const StepGate gate = step_gate(a.status);  // tested with the slot's records
  const int slot = blockIdx.x * TEAMS + tm;
  if (slot >= nslots) return;  // whole teams only: team_sync is wave-local
  const int64_t b = a.tbody[slot];
  const int pk = a.tpk[slot];
  const int e0 = a.tabs_off[slot], e1 = a.tabs_off[slot + 1];
  const int ne = a.tne[slot];
  if (gate.skip()) return;
  const int kpar = pk >= 0 ? (pk >> 1) : -1;
  const int nabs = e1 - e0;
  const int nent = nabs + (kpar >= 0 ? 1 : 0);  // <= 21: cliques hold <= TREE_KMAX rows
  // 1) what depends only on the slot's records, fetched in one batch: the
  //    body's shape index and local solve u, its absorbed-joint entries (two
  //    per lane) and the parent joint's type; then Hbar^{-1}, which waits
  //    only for the shape index and lands while the entries are decoded
  const int shp = a.shp[b];
  const double u0 = ln < 12 ? a.u[(int64_t)ln * a.ns + b] : 0.0;
  const int ta = ln < nabs ? a.tabs[e0 + ln] : 0;
  const int tb = ln + TEAM < nabs ? a.tabs[e0 + ln + TEAM] : 0;
  const int prow = kpar >= 0 ? a.jrows[kpar] : 0;
  const double *Th = a.hinv + (int64_t)HINV_STRIDE * shp;
  const double t0 = Th[ln], t1 = ln + TEAM < HINV_STRIDE ? Th[ln + TEAM] : 0.0;
  //    clique entries (absorbed joints in list order, then the parent joint),
  //    their rows and the row -> entry map
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = ln + h * TEAM;
    if (e < nent) {
      int k, side, un;
      int rows;
      if (e < nabs) {
        const int t = h ? tb : ta;
        k = abs_joint(t);
        rows = abs_rows(t);
        side = (t >> 1) & 1;
        un = t & 1;
      } else {
        k = kpar;
        rows = prow;
        side = pk & 1;
        un = 1;  // parent rows take C_k only
      }
      S.ek[e] = k;
      S.ei[e] = (rows << 4) | (un << 1) | side;
    }
  }
  team_sync();
  if (nent <= TEAM) {
    // first rows by a prefix sum over the team; each lane maps its own rows
    const int c = ln < nent ? (S.ei[ln] >> 4) & 15 : 0;
    int x = c;
    for (int o = 1; o < TEAM; o <<= 1) {
      const int y = __shfl_up(x, o, TEAM);
      if (ln >= o) x += y;
    }
    const int r0 = x - c;
    if (ln < nent) {
      S.ei[ln] |= r0 << 8;
      for (int i = 0; i < c; ++i) S.rowent[r0 + i] = (uint8_t)ln;
    }
  } else if (ln == 0) {
    int r = 0;
    for (int e = 0; e < nent; ++e) {
      const int c = (S.ei[e] >> 4) & 15;
      S.ei[e] |= r << 8;
      for (int i = 0; i < c; ++i) S.rowent[r + i] = (uint8_t)e;
      r += c;
    }
  }
  team_sync();
  const int ck = kpar >= 0 ? (S.ei[nent - 1] >> 4) & 15 : 0;
  const int nr = ne + ck;
  if (nr == 0) return;
  const int LD = ne + 5;
  double *fac = a.fac + a.foff[slot];  // LD*LD K, LD y, then (big cliques) L, Y
  const bool big = nr > TREE_KLDS;
  double *Lm = big ? fac + LD * LD + LD : S.L;
  double *Ym = fac + LD * LD + LD + 12 * nr;  // large cliques only
  //    C of the unary rows this lane sums into y0 below, read with the rows
  double cv[TREE_KMAX / TEAM];
#pragma unroll
  for (int k = 0; k < TREE_KMAX / TEAM; ++k) {
    const int i = ln + k * TEAM;
    cv[k] = 0.0;
    if (i < nr) {
      const int e = S.rowent[i], ei = S.ei[e];
      if ((ei & 2) && !a.zero_c)
        cv[k] = a.cc ? a.cc[5 * (int64_t)S.ek[e] + (i - (ei >> 8))]
                     : a.gl[(int64_t)GL_STRIDE * S.ek[e] + GL_C + (i - (ei >> 8))];
    }
  }
  //    clique rows L (nr x 12), eight independent loads per lane in flight
  //    (one pass for cliques of up to 10 rows); lanes past the end read row 0
  for (int base = 0; base < nr * 12; base += 8 * TEAM) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * TEAM + ln;
      const int r = idx < nr * 12 ? idx / 12 : 0, sc = idx < nr * 12 ? idx % 12 : 0;
      const int e = S.rowent[r], ei = S.ei[e];
      v[u] = a.gl[(int64_t)GL_STRIDE * S.ek[e] + ((ei & 1) ? GL_LB : GL_LA) + 12 * (r - (ei >> 8)) + sc];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * TEAM + ln;
      if (idx < nr * 12) Lm[idx] = v[u];
    }
  }
  S.th[ln] = t0;
  if (ln + TEAM < HINV_STRIDE) S.th[ln + TEAM] = t1;
  if (ln < 12) S.uu[ln] = u0;
  team_sync();
  if (!big) {
    // 2-3) K0 = L Hbar^{-1} L^T (lower triangle): lane j holds
    //      y_j = Hbar^{-1} L_j^T in registers and forms column j
    if (ln < nr && a.f32) {
      float lf[12], yv[12];
#pragma unroll
      for (int s = 0; s < 12; ++s) lf[s] = (float)Lm[12 * ln + s];
      hinv_apply(S.th, lf, yv);
      for (int i = ln; i < nr; ++i) {
        float v = 0.0f;
#pragma unroll
        for (int s = 0; s < 12; ++s) v += (float)Lm[12 * i + s] * yv[s];
        fac[i * LD + ln] = (double)v;
      }
    } else if (ln < nr) {
      double yv[12];
      hinv_apply(S.th, Lm + 12 * ln, yv);
      for (int i = ln; i < nr; ++i) {
        double v = 0.0;
#pragma unroll
        for (int s = 0; s < 12; ++s) v += Lm[12 * i + s] * yv[s];
        fac[i * LD + ln] = v;
      }
    }
  } else {
    // 2) Y = Hbar^{-1} L^T, one clique row per lane
    for (int col = ln; col < nr; col += TEAM) {
      double yv[12];
      hinv_apply(S.th, Lm + 12 * col, yv);
      for (int s = 0; s < 12; ++s) Ym[s * nr + col] = yv[s];
    }
    team_sync();
    // 3) K0 = L Y (lower triangle)
    for (int idx = ln; idx < nr * (nr + 1) / 2; idx += TEAM) {
      // lower-triangle entry idx -> (i, jj), jj <= i (only the lower triangle is ever read)
      int i = (int)((sqrtf(8.0f * (float)idx + 1.0f) - 1.0f) * 0.5f);
      while (i * (i + 1) / 2 > idx) --i;
      while ((i + 1) * (i + 2) / 2 <= idx) ++i;
      const int jj = idx - i * (i + 1) / 2;
      if (a.f32) {
        float v = 0.0f;
        for (int s = 0; s < 12; ++s) v += (float)Lm[12 * i + s] * (float)Ym[s * nr + jj];
        fac[i * LD + jj] = (double)v;
      } else {
        double v = 0.0;
        for (int s = 0; s < 12; ++s) v += Lm[12 * i + s] * Ym[s * nr + jj];
        fac[i * LD + jj] = v;
      }
    }
  }
  //    y0 = L u + C of one-sided and parent rows
#pragma unroll
  for (int k = 0; k < TREE_KMAX / TEAM; ++k) {
    const int i = ln + k * TEAM;
    if (i < nr) {
      double v = 0.0;
#pragma unroll
      for (int s = 0; s < 12; ++s) v += Lm[12 * i + s] * S.uu[s];
      fac[LD * LD + i] = v + cv[k];
    }
  }
}

// Tree contraction (rake and compress rounds, planned on the host).  Every
// round's operations touch disjoint slots, so each round is one launch per
// kind and clique size.  The team kernels below (a 16-lane team per
// operation, matrices in the slots' global storage) take the compresses whose
// cliques exceed the LDS-staged kernels further down.

// add the condensed far sides (Sigma, rho) of v's child joints, entries
// [e0, e1) of its absorbed list
DEV void tc_add_children(const TreeArgs &a, const GJoint *J, int e0, int e1, double *K, double *y, int LD,
                         int ln) {
  int r0 = 0;
  for (int e = e0; e < e1; ++e) {
    const int k = abs_joint(a.tabs[e]);
    const int c = abs_rows(a.tabs[e]);
    if (!(a.tabs[e] & 1)) {
      const double *gtk = a.gt + (int64_t)GT_STRIDE * k;
      for (int idx = ln; idx < c * c; idx += TEAM) {
        const int i = idx / c, jj = idx % c;
        if (jj <= i) K[(r0 + i) * LD + r0 + jj] += gtk[GT_SIG + 5 * i + jj];
      }
      for (int i = ln; i < c; i += TEAM) y[r0 + i] += gtk[GT_RHO + i];
    }
    r0 += c;
  }
}

// partial Cholesky of the first np of nr rows (lower triangle, in place):
// K_pp = Lc Lc^T, X = Lc^{-1} K_pb, z = Lc^{-1} y_p; the trailing block
// becomes the Schur complement K_bb - X^T X, y_b - X^T z
DEV void tc_partial_cholesky(const TreeArgs &a, double *K, double *y, int LD, int nr, int np, int ln) {
  for (int p = 0; p < np; ++p) {
    if (ln == 0) {
      double d = K[p * LD + p];
      if (!(d > 0.0)) {
        raise_flag(a.status, FLAG_SINGULAR, a.step);
        d = 1.0;
      }
      d = sqrt(d);
      K[p * LD + p] = d;
      y[p] /= d;
    }
    team_sync();
    const double d = K[p * LD + p];
    for (int i = p + 1 + ln; i < nr; i += TEAM) K[i * LD + p] /= d;
    team_sync();
    for (int i = p + 1 + ln; i < nr; i += TEAM) {
      const double lip = K[i * LD + p];
      for (int jj = p + 1; jj <= i; ++jj) K[i * LD + jj] -= lip * K[jj * LD + p];
      y[i] -= lip * y[p];
    }
    team_sync();
  }
}

__global__ __launch_bounds__(TREE_BLOCK) void tc_compress_kernel(TreeArgs a, const GJoint *J, int op0, int op1) {
  __shared__ double scratch[TEAMS][160];
  const int tm = threadIdx.x / TEAM, ln = threadIdx.x % TEAM;
  if (skip_step(a.status, a.step)) return;
  const int i = op0 + blockIdx.x * TEAMS + tm;
  if (i >= op1) return;
  double *M = scratch[tm];  // boundary Schur complement of v, 10 x 10
  double *m = M + 100;      // its right-hand side
  double *Lp = M + 110;     // Cholesky factor of the pivot block of e, 5 x 5
  double *zp = M + 135;     // Lp^{-1} rhs_e
  const TcOp op = a.ops[i];
  const int v = op.v, cs = op.c, ce = op.ce, ck = op.ck;
  // 1) v: add condensed children except the live child (last entry), factor
  //    the private rows, boundary rows [e; kcur] remain
  const int av = a.tne[v], LDv = av + 5, pv = av - ce, nb = ce + ck;
  double *Kv = a.fac + a.foff[v];
  double *yv = Kv + LDv * LDv;
  tc_add_children(a, J, a.tabs_off[v], a.tabs_off[v + 1] - 1, Kv, yv, LDv, ln);
  team_sync();
  tc_partial_cholesky(a, Kv, yv, LDv, op.nv, pv, ln);
  for (int idx = ln; idx < nb * nb; idx += TEAM) {
    const int r = idx / nb, s = idx % nb;
    M[idx] = s <= r ? Kv[(pv + r) * LDv + pv + s] : Kv[(pv + s) * LDv + pv + r];
  }
  for (int r = ln; r < nb; r += TEAM) m[r] = yv[pv + r];
  team_sync();
  // 2) c: rows [absorbed (ac); e (ce)]; pivot P = K_c[e,e] + M[e,e]
  const int ac = a.tne[cs], LDc = ac + 5;
  double *Kc = a.fac + a.foff[cs];
  double *yc = Kc + LDc * LDc;
  double *rec = a.crec + op.rec;
  double *Xo = rec + 25, *Xk = rec + 25 + 5 * ac, *zr = Xk + 25;
  if (ln == 0) {
    double P[25], r[5];
    for (int p = 0; p < ce; ++p) {
      for (int q = 0; q <= p; ++q) P[5 * p + q] = Kc[(ac + p) * LDc + ac + q] + M[p * nb + q];
      r[p] = yc[ac + p] + m[p];
    }
    for (int p = 0; p < ce; ++p) {  // Cholesky, lower triangle
      double d = P[5 * p + p];
      for (int t = 0; t < p; ++t) d -= P[5 * p + t] * P[5 * p + t];
      if (!(d > 0.0)) {
        raise_flag(a.status, FLAG_SINGULAR, a.step);
        d = 1.0;
      }
      d = sqrt(d);
      P[5 * p + p] = d;
      for (int q = p + 1; q < ce; ++q) {
        double s = P[5 * q + p];
        for (int t = 0; t < p; ++t) s -= P[5 * q + t] * P[5 * p + t];
        P[5 * q + p] = s / d;
      }
    }
    for (int p = 0; p < ce; ++p) {  // z = Lp^{-1} rhs_e
      double s = r[p];
      for (int t = 0; t < p; ++t) s -= P[5 * p + t] * zp[t];
      zp[p] = s / P[5 * p + p];
    }
    for (int q = 0; q < 25; ++q) Lp[q] = (q / 5 < ce && q % 5 <= q / 5) ? P[q] : 0.0;
  }
  team_sync();
  // X_o = Lp^{-1} K_c[e, o] (ce x ac), X_k = Lp^{-1} M[e, k] (ce x ck)
  for (int col = ln; col < ac + ck; col += TEAM) {
    double x[5];
    for (int p = 0; p < ce; ++p) {
      double s = col < ac ? Kc[(ac + p) * LDc + col] : M[(ce + col - ac) * nb + p];
      for (int t = 0; t < p; ++t) s -= Lp[5 * p + t] * x[t];
      x[p] = s / Lp[5 * p + p];
    }
    for (int p = 0; p < ce; ++p) {
      if (col < ac) Xo[p * ac + col] = x[p];
      else Xk[p * 5 + (col - ac)] = x[p];
    }
  }
  team_sync();
  // K_c[o, o] -= X_o^T X_o ; rows of kcur replace the rows of e
  for (int idx = ln; idx < ac * ac; idx += TEAM) {
    const int r = idx / ac, s = idx % ac;
    if (s > r) continue;
    double t = 0.0;
    for (int p = 0; p < ce; ++p) t += Xo[p * ac + r] * Xo[p * ac + s];
    Kc[r * LDc + s] -= t;
  }
  for (int r = ln; r < ac; r += TEAM) {
    double t = 0.0;
    for (int p = 0; p < ce; ++p) t += Xo[p * ac + r] * zp[p];
    yc[r] -= t;
  }
  for (int idx = ln; idx < ck * (ac + ck); idx += TEAM) {
    const int r = idx / (ac + ck), s = idx % (ac + ck);
    double t = 0.0;
    if (s < ac) {
      for (int p = 0; p < ce; ++p) t -= Xk[p * 5 + r] * Xo[p * ac + s];
      Kc[(ac + r) * LDc + s] = t;
    } else if (s - ac <= r) {
      const int q = s - ac;
      t = M[(ce + r) * nb + ce + q];
      for (int p = 0; p < ce; ++p) t -= Xk[p * 5 + r] * Xk[p * 5 + q];
      Kc[(ac + r) * LDc + ac + q] = t;
    }
  }
  for (int r = ln; r < ck; r += TEAM) {
    double t = m[ce + r];
    for (int p = 0; p < ce; ++p) t -= Xk[p * 5 + r] * zp[p];
    yc[ac + r] = t;
  }
  for (int q = ln; q < 25; q += TEAM) rec[q] = Lp[q];
  for (int p = ln; p < 5; p += TEAM) zr[p] = p < ce ? zp[p] : 0.0;
}

// lambda of v's private rows: Lc^{-T} (z - X lambda_b), with lambda_b the
// multipliers of the boundary rows (nb values), and their write-out
DEV void tc_private_back(const TreeArgs &a, const GJoint *J, int v, int np, int nr, const double *lb,
                         int e_end) {
  const int LD = a.tne[v] + 5;
  const double *K = a.fac + a.foff[v];
  const double *y = K + LD * LD;
  const int nb = nr - np;
  double t[TREE_KMAX];
  for (int i = 0; i < np; ++i) {
    double s = y[i];
    for (int f = 0; f < nb; ++f) s -= K[(np + f) * LD + i] * lb[f];
    t[i] = s;
  }
  for (int i = np - 1; i >= 0; --i) {
    double s = t[i];
    for (int l = i + 1; l < np; ++l) s -= K[l * LD + i] * t[l];
    t[i] = s / K[i * LD + i];
  }
  int r0 = 0;
  for (int e = a.tabs_off[v]; e < e_end; ++e) {
    const int k = abs_joint(a.tabs[e]);
    const int c = abs_rows(a.tabs[e]);
    for (int i = 0; i < c; ++i) a.glam[5 * (int64_t)k + i] = t[r0 + i];
    for (int i = c; i < 5; ++i) a.glam[5 * (int64_t)k + i] = 0.0;
    r0 += c;
  }
}

__global__ __launch_bounds__(256) void tc_compress_back_kernel(TreeArgs a, const GJoint *J, int op0, int op1) {
  if (skip_step(a.status, a.step)) return;
  const int i = op0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= op1) return;
  const TcOp op = a.ops[i];
  const int ce = op.ce, ck = op.ck, cs = op.c;
  const int ac = a.tne[cs];
  const double *rec = a.crec + op.rec;
  const double *Lp = rec, *Xo = rec + 25, *Xk = rec + 25 + 5 * ac, *zr = Xk + 25;
  // lambda of c's absorbed joints (solved later in the forward order) and of kcur
  double lo[TREE_KMAX], lk[5] = {0, 0, 0, 0, 0};
  {
    int r0 = 0;
    for (int e = a.tabs_off[cs]; e < a.tabs_off[cs + 1]; ++e) {
      const int k = abs_joint(a.tabs[e]);
      const int c = abs_rows(a.tabs[e]);
      for (int r = 0; r < c; ++r) lo[r0 + r] = a.glam[5 * (int64_t)k + r];
      r0 += c;
    }
  }
  for (int r = 0; r < ck; ++r) lk[r] = a.glam[5 * (int64_t)op.kcur + r];
  // lambda_e = Lp^{-T} (z - X_o lambda_o - X_k lambda_k)
  double le[5];
  for (int p = 0; p < ce; ++p) {
    double s = zr[p];
    for (int q = 0; q < ac; ++q) s -= Xo[p * ac + q] * lo[q];
    for (int q = 0; q < ck; ++q) s -= Xk[p * 5 + q] * lk[q];
    le[p] = s;
  }
  for (int p = ce - 1; p >= 0; --p) {
    double s = le[p];
    for (int q = p + 1; q < ce; ++q) s -= Lp[5 * q + p] * le[q];
    le[p] = s / Lp[5 * p + p];
  }
  for (int r = 0; r < 5; ++r) a.glam[5 * (int64_t)op.e + r] = r < ce ? le[r] : 0.0;
  // v's private rows, boundary [e; kcur]
  double lb[10];
  for (int r = 0; r < ce; ++r) lb[r] = le[r];
  for (int r = 0; r < ck; ++r) lb[ce + r] = lk[r];
  tc_private_back(a, J, op.v, a.tne[op.v] - ce, op.nv, lb, a.tabs_off[op.v + 1] - 1);
}

// ------------------------------------------- team-per-operation contraction
// The rounds are bound by the latency of their slowest operations, not by
// bandwidth: a clique's partial Cholesky is a chain of dependent steps.  So
// each operation gets a team of TW lanes within one wave (TW = 16: four
// operations per wave, for cliques of up to 16 rows; TW = 64 for larger
// ones), its cliques are staged in LDS as packed lower triangles (row i at
// i (i + 1) / 2), every copy issues all of its loads before the first wait,
// and the rank-1 updates run column-parallel.  Clique sizes R = 16, 32 and
// 48 (compress) / 64 (rake); compresses with larger cliques use the team
// kernels above on the global slots.  Workgroups are one wave, so a team
// synchronises with a wave barrier.
constexpr int TCW = 64;  // lanes per workgroup

DEV int tri(int i) { return (i * (i + 1)) >> 1; }

template <int R>
struct TcwMat {
  double K[R * (R + 1) / 2];
  double y[R];
};
template <int R>
struct TcwComp {
  TcwMat<R> v, c;
  double Lp[25];  // Cholesky factor of the pivot block of e
  double zp[5];   // Lp^{-1} rhs_e
  double Xo[5 * R];
  double Xk[25];
};

template <int TW>
DEV int tlane() { return (int)threadIdx.x % TW; }

// lower triangle of rows [0, nr) of a global clique (leading dimension ls)
// into a packed LDS triangle; every lane issues U loads before the first
// wait (the factorisations stage with U = 16: half the round trips of
// batches of eight at no occupancy cost; the back-substitutions keep 8,
// where 16 would cost them occupancy)
template <int R, int TW, int U = 8>
DEV void tcw_load_lower(const double *src, int ls, double *dst, int nr) {
  const int n = nr * R;
  for (int base = 0; base < n; base += U * TW) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * TW + tlane<TW>();
      const int i = idx / R, j = idx - (idx / R) * R;
      v[u] = src[(idx < n && j <= i) ? i * ls + j : 0];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * TW + tlane<TW>();
      const int i = idx / R, j = idx - (idx / R) * R;
      if (idx < n && j <= i) dst[tri(i) + j] = v[u];
    }
  }
}

// packed LDS clique rows [0, nr), columns j <= i and j < ncol, back to global
template <int R, int TW>
DEV void tcw_store_lower(const double *src, double *dst, int ld, int nr, int ncol) {
  for (int idx = tlane<TW>(); idx < nr * R; idx += TW) {
    const int i = idx / R, j = idx - (idx / R) * R;
    if (j <= i && j < ncol) dst[i * ld + j] = src[tri(i) + j];
  }
}

// Entries [e0, e1) of an absorbed list, one per lane (e1 - e0 <= TW): joint,
// rows, first row in the clique, and whether the joint is one-sided.
struct TcwEnt {
  int k, c, r0, unary;
};
// the lane's entry word (issued early: nothing waits on it until used)
template <int TW>
DEV int tcw_tab(const TreeArgs &a, int e0, int e1) {
  const int ln = tlane<TW>();
  return ln < e1 - e0 ? a.tabs[e0 + ln] : 0;
}
template <int TW>
DEV TcwEnt tcw_entry_of(int tab, int nent) {
  TcwEnt t{0, 0, 0, 1};
  const int ln = tlane<TW>();
  if (ln < nent) {
    t.k = abs_joint(tab);
    t.unary = tab & 1;
    t.c = abs_rows(tab);
  }
  int x = t.c;  // inclusive prefix over the team
  for (int o = 1; o < TW; o <<= 1) {
    const int u = __shfl_up(x, o, TW);
    if (ln >= o) x += u;
  }
  t.r0 = x - t.c;
  return t;
}
template <int TW>
DEV TcwEnt tcw_entry(const TreeArgs &a, const GJoint *J, int e0, int e1) {
  return tcw_entry_of<TW>(tcw_tab<TW>(a, e0, e1), e1 - e0);
}

// add the condensed far sides of the list's non-unary joints; each lane
// adds its own entry's diagonal block (all loads in flight at once)
template <int R, int TW>
DEV void tcw_add_children(const TreeArgs &a, int tab, int nent, double *K, double *y) {
  const TcwEnt t = tcw_entry_of<TW>(tab, nent);
  if (tlane<TW>() < nent && !t.unary) {
    const double *g = a.gt + (int64_t)GT_STRIDE * t.k;
    double sg[25], rh[5];
#pragma unroll
    for (int q = 0; q < 25; ++q) sg[q] = g[GT_SIG + q];
#pragma unroll
    for (int q = 0; q < 5; ++q) rh[q] = g[GT_RHO + q];
#pragma unroll
    for (int r = 0; r < 5; ++r) {
      if (r < t.c) {
#pragma unroll
        for (int s = 0; s <= r; ++s) K[tri(t.r0 + r) + t.r0 + s] += sg[5 * r + s];
        y[t.r0 + r] += rh[r];
      }
    }
  }
}

// partial Cholesky of the first np of nr (<= R <= TW) rows of a packed LDS
// clique (the factorisation of tc_partial_cholesky, blocked): pivots are
// taken in panels of PB columns.  Within a panel lane r holds row r's panel
// entries and y_r in registers; a pivot's value, its right-hand side and
// the new column entries of the panel's later rows travel by wave shuffles
// (no LDS round trip or barrier per pivot); the panel then goes back to LDS and
// the trailing triangle gets one rank-PB update, lane i owning column
// p0 + PB + i, in batches of RB independent rows, and the lanes past the
// last column taking the lower halves of the longest columns.
template <int R, int TW>
DEV void tcw_partial_cholesky(const TreeArgs &a, double *K, double *y, int nr, int np) {
  static_assert(R <= TW, "a lane per clique row");
  constexpr int PB = R >= 32 ? 8 : 4;  // panel width
  constexpr int RB = 4;  // rows per batch of the trailing update
  const int ln = tlane<TW>();
  const bool mine = ln < nr;  // lane ln holds row ln
  double yr = mine ? y[ln] : 0.0;
  for (int p0 = 0; p0 < np; p0 += PB) {
    const int pe = p0 + PB < np ? p0 + PB : np;  // panel columns [p0, pe)
    double kp[PB];
#pragma unroll
    for (int q = 0; q < PB; ++q) kp[q] = mine && p0 + q < pe && p0 + q <= ln ? K[tri(ln) + p0 + q] : 0.0;
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int p = p0 + q;
      if (p >= pe) break;  // uniform
      double d = __shfl(kp[q], p, TW);  // the pivot, updated by the panel's earlier columns
      if (!(d > 0.0)) {
        if (ln == 0) raise_flag(a.status, FLAG_SINGULAR, a.step);
        d = 1.0;
      }
      const double sd = sqrt(d);
      double lip = 0.0;
      if (ln == p) {
        kp[q] = sd;
        yr /= sd;
      } else if (mine && ln > p) {
        lip = kp[q] / sd;
        kp[q] = lip;
      }
      const double yp = __shfl(yr, p, TW);
      if (mine && ln > p) yr -= lip * yp;
#pragma unroll
      for (int q2 = q + 1; q2 < PB; ++q2) {  // row ln, panel column j = p0 + q2 <= ln
        const double ljp = __shfl(kp[q], p0 + q2, TW);  // L[j][p], lane j's new entry
        if (mine && p0 + q2 < pe && p0 + q2 <= ln) kp[q2] -= lip * ljp;
      }
    }
#pragma unroll
    for (int q = 0; q < PB; ++q)
      if (mine && p0 + q < pe && p0 + q <= ln) K[tri(ln) + p0 + q] = kp[q];
    team_sync();
    // trailing column pe + c, rows [rb, re): lane c < ntr owns column c; the
    // lanes past the last column (nh of them) take the lower halves of the
    // nh longest columns, so the longest chain of rows is about halved
    const int ntr = nr - pe;
    const int nh = ntr < TW - ntr ? ntr : TW - ntr;
    const int c = ln < ntr ? ln : ln - ntr;
    const int j = pe + c;
    const int mid = j + ((nr - j + 1) >> 1);
    const int rb = ln < ntr ? j : (c < nh ? mid : nr);
    const int re = ln < ntr && c < nh ? mid : nr;
    if (pe < nr && rb < re) {
      double lj[PB];
#pragma unroll
      for (int q = 0; q < PB; ++q) lj[q] = p0 + q < pe ? K[tri(j) + p0 + q] : 0.0;
      for (int r = rb; r < re; r += RB) {
        double kv[RB], upd[RB];
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          const int rr = r + u < re ? r + u : re - 1;
          const double *row = K + tri(rr);
          kv[u] = row[j];
          double t = 0.0;
#pragma unroll
          for (int q = 0; q < PB; ++q) t += (p0 + q < pe ? row[p0 + q] : 0.0) * lj[q];
          upd[u] = t;
        }
#pragma unroll
        for (int u = 0; u < RB; ++u)
          if (r + u < re) K[tri(r + u) + j] = kv[u] - upd[u];
      }
    }
    team_sync();
  }
  if (mine) y[ln] = yr;
  team_sync();
}

template <int R, int TW>
DEV void tcw_rake_body(const TreeArgs &a, const GJoint *J, int op0, int op1, int blk, double *smem,
                       StepGate gate) {
  TcwMat<R> *team_sm = reinterpret_cast<TcwMat<R> *>(smem);
  const int ln = tlane<TW>(), tm = (int)threadIdx.x / TW;
  const int oi = op0 + blk * (TCW / TW) + tm;
  if (oi >= op1) return;
  TcwMat<R> &sm = team_sm[tm];
  const TcOp op = a.ops[oi];
  if (gate.skip()) return;  // tested with the operation record in flight
  if (op.nv > R) {  // the host sorts operations by clique size
    if (ln == 0) raise_flag(a.status, FLAG_GUARD, a.step);
    return;
  }
  const int ne = op.av, LDg = ne + 5, nr = op.nv;
  double *Kg = a.fac + op.fv;
  double *yg = Kg + LDg * LDg;
  const int tab = tcw_tab<TW>(a, op.ev0, op.ev1);
  tcw_load_lower<R, TW, 16>(Kg, LDg, sm.K, nr);
  for (int r = ln; r < nr; r += TW) sm.y[r] = yg[r];
  team_sync();
  tcw_add_children<R, TW>(a, tab, op.ev1 - op.ev0, sm.K, sm.y);
  team_sync();
  tcw_partial_cholesky<R, TW>(a, sm.K, sm.y, nr, ne);
  if (op.kcur >= 0) {
    double *gtk = a.gt + (int64_t)GT_STRIDE * op.kcur;
    for (int q = ln; q < 30; q += TW) {
      if (q < 25) {
        const int r = q / 5, s = q % 5;
        double val = 0.0;
        if (r < op.ck && s < op.ck) val = s <= r ? sm.K[tri(ne + r) + ne + s] : sm.K[tri(ne + s) + ne + r];
        gtk[GT_SIG + q] = val;
      } else {
        const int r = q - 25;
        gtk[GT_RHO + r] = r < op.ck ? sm.y[ne + r] : 0.0;
      }
    }
  }
  // factor columns and z of the private rows, for the back-substitution
  tcw_store_lower<R, TW>(sm.K, Kg, LDg, nr, ne);
  for (int r = ln; r < ne; r += TW) yg[r] = sm.y[r];
}

template <int R, int TW>
DEV void tcw_compress_body(const TreeArgs &a, const GJoint *J, int op0, int op1, int blk, double *smem,
                           StepGate gate) {
  TcwComp<R> *team_sm = reinterpret_cast<TcwComp<R> *>(smem);
  const int ln = tlane<TW>(), tm = (int)threadIdx.x / TW;
  const int oi = op0 + blk * (TCW / TW) + tm;
  if (oi >= op1) return;
  TcwComp<R> &sm = team_sm[tm];
  const TcOp op = a.ops[oi];
  if (gate.skip()) return;  // tested with the operation record in flight
  const int ce = op.ce, ck = op.ck;
  const int av = op.av, LDvg = av + 5, pv = av - ce, nv = op.nv;
  const int ac = op.ac, LDcg = ac + 5;
  if (nv > R || ac + (ce > ck ? ce : ck) > R) {  // the host sorts operations by clique size
    if (ln == 0) raise_flag(a.status, FLAG_GUARD, a.step);
    return;
  }
  double *Kvg = a.fac + op.fv;
  double *yvg = Kvg + LDvg * LDvg;
  double *Kcg = a.fac + op.fc;
  double *ycg = Kcg + LDcg * LDcg;
  double *Kv = sm.v.K, *yv = sm.v.y, *Kc = sm.c.K, *yc = sm.c.y;
  // boundary Schur complement of v on [e; kcur] (read in place, symmetric)
  auto Mv = [&](int r, int s) { return r >= s ? Kv[tri(pv + r) + pv + s] : Kv[tri(pv + s) + pv + r]; };
  // 1) v: condensed children except the live child (last entry), private
  //    rows factored; boundary rows [e; kcur] remain
  const int tab = tcw_tab<TW>(a, op.ev0, op.ev1 - 1);
  tcw_load_lower<R, TW, 16>(Kvg, LDvg, Kv, nv);
  tcw_load_lower<R, TW, 16>(Kcg, LDcg, Kc, ac + ce);
  for (int r = ln; r < nv; r += TW) yv[r] = yvg[r];
  for (int r = ln; r < ac + ce; r += TW) yc[r] = ycg[r];
  team_sync();
  tcw_add_children<R, TW>(a, tab, op.ev1 - 1 - op.ev0, Kv, yv);
  team_sync();
  tcw_partial_cholesky<R, TW>(a, Kv, yv, nv, pv);
  tcw_store_lower<R, TW>(Kv, Kvg, LDvg, nv, pv);
  for (int r = ln; r < pv; r += TW) yvg[r] = yv[r];
  // 2) c: rows [absorbed (ac); e (ce)]; pivot P = K_c[e,e] + M[e,e]
  if (ln == 0) {  // ce <= 5: fixed trip counts keep P, r, z in registers
    double P[25], r[5], z[5];
#pragma unroll
    for (int p = 0; p < 5; ++p) {
#pragma unroll
      for (int q = 0; q < 5; ++q)
        P[5 * p + q] = (p < ce && q <= p) ? Kc[tri(ac + p) + ac + q] + Mv(p, q) : 0.0;
      r[p] = p < ce ? yc[ac + p] + yv[pv + p] : 0.0;
    }
#pragma unroll
    for (int p = 0; p < 5; ++p) {  // Cholesky, lower triangle
      if (p < ce) {
        double d = P[5 * p + p];
#pragma unroll
        for (int t = 0; t < p; ++t) d -= P[5 * p + t] * P[5 * p + t];
        if (!(d > 0.0)) {
          raise_flag(a.status, FLAG_SINGULAR, a.step);
          d = 1.0;
        }
        d = sqrt(d);
        P[5 * p + p] = d;
#pragma unroll
        for (int q = p + 1; q < 5; ++q) {
          double s = P[5 * q + p];
#pragma unroll
          for (int t = 0; t < p; ++t) s -= P[5 * q + t] * P[5 * p + t];
          P[5 * q + p] = s / d;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < 5; ++p) {  // z = Lp^{-1} rhs_e
      double s = r[p];
#pragma unroll
      for (int t = 0; t < p; ++t) s -= P[5 * p + t] * z[t];
      z[p] = p < ce ? s / P[5 * p + p] : 0.0;
      sm.zp[p] = z[p];
    }
#pragma unroll
    for (int q = 0; q < 25; ++q) sm.Lp[q] = (q / 5 < ce && q % 5 <= q / 5) ? P[q] : 0.0;
  }
  team_sync();
  const double *Lp = sm.Lp, *zp = sm.zp;
  double *Xo = sm.Xo, *Xk = sm.Xk;
  // X_o = Lp^{-1} K_c[e, o] (ce x ac), X_k = Lp^{-1} M[e, k] (ce x ck)
  for (int col = ln; col < ac + ck; col += TW) {
    double x[5];
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      x[p] = 0.0;
      if (p < ce) {
        double s = col < ac ? Kc[tri(ac + p) + col] : Mv(ce + col - ac, p);
#pragma unroll
        for (int t = 0; t < p; ++t) s -= Lp[5 * p + t] * x[t];
        x[p] = s / Lp[5 * p + p];
      }
    }
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      if (p < ce) {
        if (col < ac) Xo[p * ac + col] = x[p];
        else Xk[p * 5 + (col - ac)] = x[p];
      }
    }
  }
  team_sync();
  // K_c[o, o] -= X_o^T X_o ; rows of kcur replace the rows of e (the e rows
  // were read into X_o before the barrier)
  for (int idx = ln; idx < ac * ac; idx += TW) {
    const int r = idx / ac, s = idx % ac;
    if (s > r) continue;
    double t = 0.0;
    for (int p = 0; p < ce; ++p) t += Xo[p * ac + r] * Xo[p * ac + s];
    Kc[tri(r) + s] -= t;
  }
  for (int r = ln; r < ac; r += TW) {
    double t = 0.0;
    for (int p = 0; p < ce; ++p) t += Xo[p * ac + r] * zp[p];
    yc[r] -= t;
  }
  for (int idx = ln; idx < ck * (ac + ck); idx += TW) {
    const int r = idx / (ac + ck), s = idx % (ac + ck);
    double t = 0.0;
    if (s < ac) {
      for (int p = 0; p < ce; ++p) t -= Xk[p * 5 + r] * Xo[p * ac + s];
      Kc[tri(ac + r) + s] = t;
    } else if (s - ac <= r) {
      const int q = s - ac;
      t = Mv(ce + r, ce + q);
      for (int p = 0; p < ce; ++p) t -= Xk[p * 5 + r] * Xk[p * 5 + q];
      Kc[tri(ac + r) + ac + q] = t;
    }
  }
  for (int r = ln; r < ck; r += TW) {
    double t = yv[pv + ce + r];
    for (int p = 0; p < ce; ++p) t -= Xk[p * 5 + r] * zp[p];
    yc[ac + r] = t;
  }
  // compress record: Lp 5x5, X_o (ce x ac), X_k 5x5, z 5
  double *rec = a.crec + op.rec;
  for (int q = ln; q < 25; q += TW) {
    rec[q] = Lp[q];
    rec[25 + 5 * ac + q] = (q / 5 < ce && q % 5 < ck) ? Xk[q] : 0.0;
  }
  if (ln < 5) rec[25 + 5 * ac + 25 + ln] = ln < ce ? zp[ln] : 0.0;
  for (int idx = ln; idx < ce * ac; idx += TW) rec[25 + idx] = Xo[idx];
  team_sync();
  // c's clique now has rows [absorbed; kcur]
  tcw_store_lower<R, TW>(Kc, Kcg, LDcg, ac + ck, ac + ck);
  for (int r = ln; r < ac + ck; r += TW) ycg[r] = yc[r];
}

// Back-substitution of one clique's private rows: lambda = Lc^{-T} (z - X
// lambda_b) (lambda_b: nb <= 10 boundary multipliers, the same in every
// lane), with lane i holding row i (np <= TW), then written to the absorbed
// joints.
template <int R, int TW>
DEV void tcw_private_back(const TreeArgs &a, const GJoint *J, const TcOp &op, int np, const double *lb,
                          int e_end, double *Ks) {
  const int ln = tlane<TW>();
  const int nr = op.nv, e_beg = op.ev0;
  const int LDg = op.av + 5;
  const double *Kg = a.fac + op.fv;
  const double *yg = Kg + LDg * LDg;
  const int nb = nr - np;
  const int tab = tcw_tab<TW>(a, e_beg, e_end);
  tcw_load_lower<R, TW>(Kg, LDg, Ks, nr);
  double t = 0.0;
  if (ln < np) t = yg[ln];
  team_sync();
  double dg = 1.0, rdg = 1.0;  // this lane's diagonal entry and its reciprocal
  if (ln < np) {
    dg = Ks[tri(ln) + ln];
    rdg = 1.0 / dg;  // formed before the substitution's dependent chain
#pragma unroll
    for (int f = 0; f < 10; ++f)
      if (f < nb) t -= Ks[tri(np + f) + ln] * lb[f];
  }
  for (int l = np - 1; l >= 0; --l) {
    if (ln == l) {
      // t / dg from the correctly rounded reciprocal with one remainder step
      // (Markstein's division): the correctly rounded quotient, so the same
      // value as the division, in three dependent operations
      const double q0 = t * rdg;
      t = fma(fma(-q0, dg, t), rdg, q0);
    }
    const double tl = __shfl(t, l, TW);
    if (ln < l) t -= Ks[tri(l) + ln] * tl;
  }
  // write-out: lane e owns absorbed entry e
  const TcwEnt en = tcw_entry_of<TW>(tab, e_end - e_beg);
  double w[5];
#pragma unroll
  for (int r = 0; r < 5; ++r) {
    const double tv = __shfl(t, en.r0 + r < TW ? en.r0 + r : 0, TW);
    w[r] = r < en.c ? tv : 0.0;
  }
  if (ln < e_end - e_beg) {
#pragma unroll
    for (int r = 0; r < 5; ++r) a.glam[5 * (int64_t)en.k + r] = w[r];
  }
}

template <int R, int TW>
DEV void tcw_rake_back_body(const TreeArgs &a, const GJoint *J, int op0, int op1, int blk, double *smem,
                            StepGate gate) {
  double(*team_ks)[R * (R + 1) / 2] = reinterpret_cast<double(*)[R * (R + 1) / 2]>(smem);
  const int tm = (int)threadIdx.x / TW;
  const int oi = op0 + blk * (TCW / TW) + tm;
  if (oi >= op1) return;
  const TcOp op = a.ops[oi];
  if (gate.skip()) return;  // tested with the operation record in flight
  if (op.nv > R) {
    if (tlane<TW>() == 0) raise_flag(a.status, FLAG_GUARD, a.step);
    return;
  }
  double lb[10];
#pragma unroll
  for (int r = 0; r < 10; ++r) lb[r] = (r < op.ck) ? a.glam[5 * (int64_t)op.kcur + (r < 5 ? r : 0)] : 0.0;
  tcw_private_back<R, TW>(a, J, op, op.av, lb, op.ev1, team_ks[tm]);
}

template <int R, int TW>
DEV void tcw_compress_back_body(const TreeArgs &a, const GJoint *J, int op0, int op1, int blk,
                                double *smem, StepGate gate) {
  double(*team_ks)[R * (R + 1) / 2] = reinterpret_cast<double(*)[R * (R + 1) / 2]>(smem);
  const int ln = tlane<TW>(), tm = (int)threadIdx.x / TW;
  const int oi = op0 + blk * (TCW / TW) + tm;
  if (oi >= op1) return;
  const TcOp op = a.ops[oi];
  if (gate.skip()) return;  // tested with the operation record in flight
  const int ce = op.ce, ck = op.ck;
  const int ac = op.ac;
  if (op.nv > R || ac > TW) {
    if (ln == 0) raise_flag(a.status, FLAG_GUARD, a.step);
    return;
  }
  const double *rec = a.crec + op.rec;
  const double *Lp = rec, *Xo = rec + 25, *Xk = rec + 25 + 5 * ac, *zr = Xk + 25;
  double lk[5];
#pragma unroll
  for (int r = 0; r < 5; ++r) lk[r] = r < ck ? a.glam[5 * (int64_t)op.kcur + r] : 0.0;
  // lambda_o of c's absorbed rows (solved later in the forward order): lane q
  // finds the entry that holds row q
  const TcwEnt en = tcw_entry<TW>(a, J, op.ec0, op.ec1);
  const int nent = op.ec1 - op.ec0;
  int myk = 0, myw = 0;
  for (int e = 0; e < nent; ++e) {
    const int r0 = __shfl(en.r0, e, TW), c = __shfl(en.c, e, TW), k = __shfl(en.k, e, TW);
    if (ln >= r0 && ln < r0 + c) {
      myk = k;
      myw = ln - r0;
    }
  }
  const double lo = ln < ac ? a.glam[5 * (int64_t)myk + myw] : 0.0;
  // lambda_e = Lp^{-T} (z - X_o lambda_o - X_k lambda_k)
  double le[5];
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    double s = (p < ce && ln < ac) ? Xo[p * ac + ln] * lo : 0.0;
    for (int o = TW / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, TW);
    double v = 0.0;
    if (p < ce) {
      v = zr[p] - s;
#pragma unroll
      for (int q = 0; q < 5; ++q)
        if (q < ck) v -= Xk[p * 5 + q] * lk[q];
    }
    le[p] = v;
  }
  double dp[5], rdp[5];  // Lp's diagonal and its reciprocals, before the chain
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    dp[p] = p < ce ? Lp[5 * p + p] : 1.0;
    rdp[p] = 1.0 / dp[p];
  }
#pragma unroll
  for (int p = 4; p >= 0; --p) {
    if (p < ce) {
      double s = le[p];
#pragma unroll
      for (int q = p + 1; q < 5; ++q)
        if (q < ce) s -= Lp[5 * q + p] * le[q];
      const double q0 = s * rdp[p];  // s / dp[p], correctly rounded (as in tcw_private_back)
      le[p] = fma(fma(-q0, dp[p], s), rdp[p], q0);
    }
  }
  if (ln < 5) a.glam[5 * (int64_t)op.e + ln] = ln < ce ? le[ln] : 0.0;
  // v's private rows, boundary [e; kcur]
  double lb[10];  // [lambda_e; lambda_kcur], e has 3, 4 or 5 rows
  if (ce == 3) {
#pragma unroll
    for (int r = 0; r < 10; ++r) lb[r] = r < 3 ? le[r] : (r < 8 ? lk[r - 3] : 0.0);
  } else if (ce == 4) {
#pragma unroll
    for (int r = 0; r < 10; ++r) lb[r] = r < 4 ? le[r] : (r < 9 ? lk[r - 4] : 0.0);
  } else {
#pragma unroll
    for (int r = 0; r < 10; ++r) lb[r] = r < 5 ? le[r] : lk[r - 5];
  }
  tcw_private_back<R, TW>(a, J, op, op.av - ce, lb, op.ev1 - 1, team_ks[tm]);
}

// One launch for several LDS-staged operation classes (rake or compress, by
// clique size) of a round.  A round's operations touch disjoint slots, and
// the planner keeps its rakes and compresses independent, so the classes
// need no ordering among themselves: launched together they cost the latency
// of the slowest operation instead of the sum over the classes.  Block b
// belongs to the last segment whose first block is <= b; the dynamic LDS is
// sized by the host for the largest class in the launch.
enum { TC_RAKE10, TC_RAKE16, TC_RAKE32, TC_RAKE64, TC_COMP10, TC_COMP16, TC_COMP32, TC_COMP48, TC_NCLASS };
static_assert(TC_NSEG == TC_NCLASS + 1, "one plan segment per class, then the large compresses");
struct TcwSeg {
  int32_t cls, op0, op1, blk0;
};
struct TcwLaunch {
  TcwSeg seg[TC_NCLASS];
  int32_t nseg;
};

// SMALL: the 10-row classes only, in a kernel of their own (compiled beside
// the other classes their code raised the register count of every class
// from 72 to 141 VGPRs)
template <bool BACK, bool SMALL>
__global__ __launch_bounds__(TCW) void tcw_round_kernel(TreeArgs a, const GJoint *J, TcwLaunch L) {
  extern __shared__ double tcw_smem[];
  const StepGate gate = step_gate(a.status);  // tested by each operation with its first read
  // fixed indices only (the launch record stays in kernel-argument memory)
  int cls = L.seg[0].cls, op0 = L.seg[0].op0, op1 = L.seg[0].op1, blk0 = L.seg[0].blk0;
#pragma unroll
  for (int k = 1; k < TC_NCLASS; ++k) {
    if (k < L.nseg && (int)blockIdx.x >= L.seg[k].blk0) {
      cls = L.seg[k].cls;
      op0 = L.seg[k].op0;
      op1 = L.seg[k].op1;
      blk0 = L.seg[k].blk0;
    }
  }
  const int blk = (int)blockIdx.x - blk0;
  if constexpr (SMALL) {
    if constexpr (!BACK) {
      if (cls == TC_RAKE10) tcw_rake_body<10, 16>(a, J, op0, op1, blk, tcw_smem, gate);
      else tcw_compress_body<10, 16>(a, J, op0, op1, blk, tcw_smem, gate);
    } else {
      if (cls == TC_RAKE10) tcw_rake_back_body<10, 16>(a, J, op0, op1, blk, tcw_smem, gate);
      else tcw_compress_back_body<10, 16>(a, J, op0, op1, blk, tcw_smem, gate);
    }
  } else if constexpr (!BACK) {
    switch (cls) {
      case TC_RAKE16: tcw_rake_body<16, 16>(a, J, op0, op1, blk, tcw_smem, gate); break;
      case TC_RAKE32: tcw_rake_body<32, 64>(a, J, op0, op1, blk, tcw_smem, gate); break;
      case TC_RAKE64: tcw_rake_body<64, 64>(a, J, op0, op1, blk, tcw_smem, gate); break;
      case TC_COMP16: tcw_compress_body<16, 16>(a, J, op0, op1, blk, tcw_smem, gate); break;
      case TC_COMP32: tcw_compress_body<32, 64>(a, J, op0, op1, blk, tcw_smem, gate); break;
      default: tcw_compress_body<48, 64>(a, J, op0, op1, blk, tcw_smem, gate); break;
    }
  } else {
    switch (cls) {
      case TC_RAKE16: tcw_rake_back_body<16, 16>(a, J, op0, op1, blk, tcw_smem, gate); break;
      case TC_RAKE32: tcw_rake_back_body<32, 64>(a, J, op0, op1, blk, tcw_smem, gate); break;
      case TC_RAKE64: tcw_rake_back_body<64, 64>(a, J, op0, op1, blk, tcw_smem, gate); break;
      case TC_COMP16: tcw_compress_back_body<16, 16>(a, J, op0, op1, blk, tcw_smem, gate); break;
      case TC_COMP32: tcw_compress_back_body<32, 64>(a, J, op0, op1, blk, tcw_smem, gate); break;
      default: tcw_compress_back_body<48, 64>(a, J, op0, op1, blk, tcw_smem, gate); break;
    }
  }
}

// ------------------------------------------------------ (d) back-projection
// dq = diag4(R) (u - Hbar^{-1} sum_k L_k^T lambda_k)  (Eq. primal), then
// q_out = q_cur + dq and qd_out = (accumulate ? qd_out : 0) + dq / h.
__global__ __launch_bounds__(256) void gapply_kernel(int b0, int b1, const int32_t *inc_off, const int32_t *inc,
                              const double *gl, const double *glam, const double *Rg,
                              const double *ug, int64_t ns, const int32_t *shp, const double *hinv,
                              const double *q_cur, double *q_out, double *qd_out, double h,
                              int accumulate, uint32_t *status, const uint8_t *jrows, int step,
                              double *dq_save, int polar_free, int skip_free) {
  int64_t b = (int64_t)b0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= b1 || skip_step(status, step)) return;
  if (skip_free && inc_off[b] == inc_off[b + 1]) return;  // applied by gbody_kernel
  if (polar_free && inc_off[b] == inc_off[b + 1]) {
    // polar-free solve (Alg. 1): dq = the length-preserving stand-in of R
    // applied to each block of u
    double A[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) A[3 * i + c] = q_cur[(3 * c + i) * ns + b];
    const double ih = 1.0 / h;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double dp[3], dq[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) dp[i] = ug[(3 * c + i) * ns + b];
      lenpres(A, false, dp, dq);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int64_t o = (int64_t)(3 * c + i) * ns + b;
        q_out[o] = q_cur[o] + dq[i];
        qd_out[o] = (accumulate ? qd_out[o] : 0.0) + dq[i] * ih;
        if (dq_save) dq_save[o] = dq[i];
        if (!isfinite(dq[i])) raise_flag(status, FLAG_NONFINITE, step);
      }
    }
    return;
  }
  double g12[12];
  for (int i = 0; i < 12; ++i) g12[i] = 0.0;
  for (int e = inc_off[b]; e < inc_off[b + 1]; ++e) {
    const int ent = inc[e];
    const int k = ent >> 1, side = ent & 1;
    const int c = jrows[k];
    const double *L = gl + (int64_t)GL_STRIDE * k + (side ? GL_LB : GL_LA);
    for (int r = 0; r < c; ++r) {
      const double lr = glam[5 * (int64_t)k + r];
      for (int s = 0; s < 12; ++s) g12[s] += L[12 * r + s] * lr;
    }
  }
  double hg[12], R[9];
  hinv_apply(hinv + (int64_t)HINV_STRIDE * shp[b], g12, hg);
  for (int i = 0; i < 9; ++i) R[i] = Rg[i * ns + b];
  const double ih = 1.0 / h;
  for (int c = 0; c < 4; ++c) {
    double dp[3], dq[3];
    for (int i = 0; i < 3; ++i) dp[i] = ug[(3 * c + i) * ns + b] - hg[3 * c + i];
    mat3_vec(R, dp, dq);
    for (int i = 0; i < 3; ++i) {
      const int64_t o = (int64_t)(3 * c + i) * ns + b;
      q_out[o] = q_cur[o] + dq[i];
      qd_out[o] = (accumulate ? qd_out[o] : 0.0) + dq[i] * ih;
      if (dq_save) dq_save[o] = dq[i];
      if (!isfinite(dq[i])) raise_flag(status, FLAG_NONFINITE, step);
    }
  }
}

// ------------------------------------------------------------ state copies
// solver-order SoA -> input-order AoS (n x 12) for dynamic bodies.  The
// state is buffer `cur` of (q0, qd0) / (q1, qd1), unless `status` is given
// and records a failed step: then it is the buffer that step read, index
// (cur0 + failing step) mod 2, cur0 the buffer current when the status word
// was cleared (steps after a failed one do nothing).
__global__ void gather_state_kernel(int nd, const int32_t *sol2in, const double *q0, const double *qd0,
                                    const double *q1, const double *qd1, int cur, int cur0,
                                    const uint32_t *status, int64_t ns, double *qo, double *qdo) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nd) return;
  int idx = cur;
  if (status && status[0] != 0u) idx = (int)((cur0 + status[1]) & 1u);
  const double *q = idx ? q1 : q0, *qd = idx ? qd1 : qd0;
  const int64_t o = sol2in[i];
  for (int c = 0; c < 12; ++c) {
    if (qo) qo[12 * o + c] = q[c * ns + i];
    if (qdo) qdo[12 * o + c] = qd[c * ns + i];
  }
}

// input-order AoS (n x 12) -> solver-order SoA for dynamic bodies
__global__ void scatter_state_kernel(int nd, const int32_t *sol2in, const double *qi, const double *qdi,
                                     double *q, double *qd, int64_t ns) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nd) return;
  const int64_t o = sol2in[i];
  for (int c = 0; c < 12; ++c) {
    q[c * ns + i] = qi[12 * o + c];
    qd[c * ns + i] = qdi[12 * o + c];
  }
}

// pinned bodies: q stays q0, qdot = 0
__global__ void write_pinned_kernel(int np, const int32_t *idx, const double *q0, double *qo,
                                    double *qdo) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int64_t o = idx[i];
  for (int c = 0; c < 12; ++c) {
    if (qo) qo[12 * o + c] = q0[12 * (int64_t)i + c];
    if (qdo) qdo[12 * o + c] = 0.0;
  }
}

__global__ void reset_status_kernel(uint32_t *st) {
  st[0] = 0u;
  st[1] = (uint32_t)NO_FAIL;
  st[2] = 0xffffffffu;  // the first begin_step makes it 0
}

__global__ void begin_step_kernel(uint32_t *st) { st[2] += 1u; }

// launchers ---------------------------------------------------------------
void launch_scatter_state(int nd, const int32_t *sol2in, const double *qi, const double *qdi,
                          double *q, double *qd, int64_t ns, hipStream_t s) {
  if (nd > 0)
    hipLaunchKernelGGL(scatter_state_kernel, dim3((nd + 255) / 256), dim3(256), 0, s, nd, sol2in, qi,
                       qdi, q, qd, ns);
}
void launch_write_pinned(int np, const int32_t *idx, const double *q0, double *qo, double *qdo,
                         hipStream_t s) {
  if (np > 0)
    hipLaunchKernelGGL(write_pinned_kernel, dim3((np + 255) / 256), dim3(256), 0, s, np, idx, q0, qo,
                       qdo);
}
void launch_reset_status(uint32_t *st, hipStream_t s) {
  hipLaunchKernelGGL(reset_status_kernel, dim3(1), dim3(1), 0, s, st);
}
void launch_begin_step(uint32_t *st, hipStream_t s) {
  hipLaunchKernelGGL(begin_step_kernel, dim3(1), dim3(1), 0, s, st);
}
void launch_prefactor(const double *shape, int nshape, double h, double *hinv, hipStream_t s) {
  if (nshape > 0)
    hipLaunchKernelGGL(prefactor_kernel, dim3((nshape + 255) / 256), dim3(256), 0, s, shape, nshape,
                       h, hinv);
}
void launch_gbody(int b0, int b1, const double *q, const double *qn, const double *qdn, int64_t ns,
                  const int32_t *shp, const double *hinv, const double *shape, const double *g,
                  double h, double *Rg, double *ug, uint32_t *status, int step, const double *wr,
                  const int32_t *pf_inc, int f32, const int32_t *free_inc, double *q_out, double *qd_out,
                  int acc, double *dq_save, hipStream_t s) {
  const FreeApply fa{free_inc, q_out, qd_out, dq_save, acc};
  if (b1 > b0)
    hipLaunchKernelGGL(gbody_kernel, dim3((b1 - b0 + 255) / 256), dim3(256), 0, s, b0, b1, q, qn, qdn,
                       ns, shp, hinv, shape, g[0], g[1], g[2], h, Rg, ug, status, step, wr, pf_inc, f32, fa);
}
// glam += dlam over n entries (refinement: the correction's multipliers)
__global__ void lam_add_kernel(int64_t n, double *glam, const double *dlam, const uint32_t *status) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n || skip_step(status, 0)) return;
  glam[i] += dlam[i];
}
void launch_lam_add(int64_t n, double *glam, const double *dlam, const uint32_t *status, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(lam_add_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, glam, dlam, status);
}
// raise a status flag for the current step from the host's decision
__global__ void raise_kernel(uint32_t *status, uint32_t flag) {
  if (threadIdx.x == 0 && !skip_step(status, 0)) raise_flag(status, flag, 0);
}
void launch_raise(uint32_t *status, uint32_t flag, hipStream_t s) {
  hipLaunchKernelGGL(raise_kernel, dim3(1), dim3(64), 0, s, status, flag);
}
void launch_gjoint(int m, const GJoint *J, const double *q, const double *Rg, int64_t ns, int hg,
                   double *gl, hipStream_t s) {
  if (m > 0)
    hipLaunchKernelGGL(gjoint_kernel, dim3((m + 127) / 128), dim3(128), 0, s, m, J, q, Rg, ns, hg, gl);
}
// operations of [o0, o1) with TW-lane teams, TCW / TW per workgroup

void launch_path(const TreeArgs &a, const PathPlan &P, hipStream_t s);

void launch_tree(const TreeArgs &a, const GJoint *J, int nslots, const int32_t *rounds, int nround,
                 int split_ops, int order, const PathPlan *path, hipStream_t s, int hook_round,
                 void (*hook)(void *), void *hook_arg) {
  // path components (no slots): their own solve
  if (path && path->nlevel > 0) launch_path(a, *path, s);
  if (nslots <= 0) {
    if (hook) hook(hook_arg);
    return;
  }
  hipLaunchKernelGGL(tree_prep_kernel, dim3((nslots + TEAMS - 1) / TEAMS), dim3(TREE_BLOCK), 0, s, a, J, nslots);
  // per round, TC_NSEG offsets of the operation list (o[TC_NSEG] starts the
  // next round): rakes with cliques of <= 10, 16, 32, 64 rows, then
  // compresses with cliques of <= 10, 16, 32, 48 rows and larger (team
  // kernels on the global slots).  The planner keeps a round's rakes and
  // compresses independent (a node with a child raked in the round is
  // compressed in a later one), so every LDS-staged class of a round shares
  // one launch, in both directions, except that the 10-row classes take a
  // kernel of their own and the 16-row classes a launch of their own when
  // they hold more than split_ops operations: those are throughput-bound,
  // and a launch is sized (LDS per workgroup, hence occupancy) by its
  // largest class.  Within a launch the
  // classes go largest first with order 0 (workgroups are dispatched in
  // index order, so the longest operations start first and the short ones
  // fill the tail), smallest first with order 1.  Both are schedule choices
  // only: every operation of a round is independent of the others.
  static const int tw[TC_NCLASS] = {16, 16, 64, 64, 16, 16, 64, 64};
  static const size_t lds_fwd[TC_NCLASS] = {4 * sizeof(TcwMat<10>),  4 * sizeof(TcwMat<16>),
                                            sizeof(TcwMat<32>),      sizeof(TcwMat<64>),
                                            4 * sizeof(TcwComp<10>), 4 * sizeof(TcwComp<16>),
                                            sizeof(TcwComp<32>),     sizeof(TcwComp<48>)};
  static const size_t lds_back[TC_NCLASS] = {4 * 55 * 8, 4 * 136 * 8, 528 * 8, 2080 * 8,
                                             4 * 55 * 8, 4 * 136 * 8, 528 * 8, 1176 * 8};
  static const int by_size[2][TC_NCLASS] = {
      {TC_RAKE64, TC_COMP48, TC_RAKE32, TC_COMP32, TC_RAKE16, TC_COMP16, TC_RAKE10, TC_COMP10},
      {TC_RAKE10, TC_COMP10, TC_RAKE16, TC_COMP16, TC_RAKE32, TC_RAKE64, TC_COMP32, TC_COMP48}};
  const int *all = by_size[order == 1 ? 1 : 0];
  auto launch_classes = [&](const int32_t *o, const int *cl, int ncl, bool back, bool small) {
    TcwLaunch L{};
    int nb = 0;
    size_t lds = 0;
    for (int i = 0; i < ncl; ++i) {
      const int c = cl[i], n = o[c + 1] - o[c];
      if (n <= 0) continue;
      const int per = TCW / tw[c];
      L.seg[L.nseg++] = TcwSeg{c, o[c], o[c + 1], nb};
      nb += (n + per - 1) / per;
      lds = std::max(lds, back ? lds_back[c] : lds_fwd[c]);
    }
    if (nb == 0) return;
    if (small) {
      if (back)
        hipLaunchKernelGGL((tcw_round_kernel<true, true>), dim3(nb), dim3(TCW), lds, s, a, J, L);
      else
        hipLaunchKernelGGL((tcw_round_kernel<false, true>), dim3(nb), dim3(TCW), lds, s, a, J, L);
    } else if (back) {
      hipLaunchKernelGGL((tcw_round_kernel<true, false>), dim3(nb), dim3(TCW), lds, s, a, J, L);
    } else {
      hipLaunchKernelGGL((tcw_round_kernel<false, false>), dim3(nb), dim3(TCW), lds, s, a, J, L);
    }
  };
  auto launch_round = [&](const int32_t *o, bool back) {
    // the 10-row classes are non-empty only where the planner kept them apart
    // from the 16-row ones (more operations than the 16-row kernel runs at
    // once): they always take their own kernel
    auto ops = [&](int c) { return o[c + 1] - o[c]; };
    const bool apart16 = ops(TC_RAKE16) + ops(TC_COMP16) > split_ops;
    int rest[TC_NCLASS], nrest = 0;
    for (int i = 0; i < TC_NCLASS; ++i) {
      const int c = all[i];
      const bool c10 = c == TC_RAKE10 || c == TC_COMP10, c16 = c == TC_RAKE16 || c == TC_COMP16;
      if (c10 || (c16 && apart16)) continue;
      rest[nrest++] = c;
    }
    static const int g10[2] = {TC_RAKE10, TC_COMP10}, g16[2] = {TC_RAKE16, TC_COMP16};
    launch_classes(o, g10, 2, back, true);
    if (apart16) launch_classes(o, g16, 2, back, false);
    launch_classes(o, rest, nrest, back, false);
  };
  // the hook (work launched elsewhere, e.g. on another stream) runs before
  // forward round hook_round, or after the last one
  bool hooked = false;
  for (int r = 0; r < nround; ++r) {
    const int32_t *o = rounds + TC_NSEG * r;
    if (hook && r == hook_round) {
      hook(hook_arg);
      hooked = true;
    }
    launch_round(o, false);
    if (o[TC_NSEG] > o[TC_NCLASS])
      hipLaunchKernelGGL(tc_compress_kernel, dim3((o[TC_NSEG] - o[TC_NCLASS] + TEAMS - 1) / TEAMS),
                         dim3(TREE_BLOCK), 0, s, a, J, o[TC_NCLASS], o[TC_NSEG]);
  }
  if (hook && !hooked) hook(hook_arg);
  for (int r = nround - 1; r >= 0; --r) {
    const int32_t *o = rounds + TC_NSEG * r;
    if (o[TC_NSEG] > o[TC_NCLASS])
      hipLaunchKernelGGL(tc_compress_back_kernel, dim3((o[TC_NSEG] - o[TC_NCLASS] + 255) / 256), dim3(256), 0, s,
                         a, J, o[TC_NCLASS], o[TC_NSEG]);
    launch_round(o, true);
  }
}
void launch_gapply(int b0, int b1, const int32_t *inc_off, const int32_t *inc, const double *gl,
                   const double *glam, const double *Rg, const double *ug, int64_t ns,
                   const int32_t *shp, const double *hinv, const double *q_cur, double *q_out,
                   double *qd_out, double h, int acc, uint32_t *status, const uint8_t *jrows,
                   int step, double *dq_save, int polar_free, int skip_free, hipStream_t s) {
  if (b1 > b0)
    hipLaunchKernelGGL(gapply_kernel, dim3((b1 - b0 + 255) / 256), dim3(256), 0, s, b0, b1, inc_off,
                       inc, gl, glam, Rg, ug, ns, shp, hinv, q_cur, q_out, qd_out, h, acc, status, jrows,
                       step, dq_save, polar_free, skip_free);
}
void launch_gather_state(int nd, const int32_t *sol2in, const double *const *q, const double *const *qd,
                         int cur, int cur0, const uint32_t *status, int64_t ns, double *qo, double *qdo,
                         hipStream_t s) {
  if (nd > 0)
    hipLaunchKernelGGL(gather_state_kernel, dim3((nd + 255) / 256), dim3(256), 0, s, nd, sol2in, q[0],
                       qd[0], q[1], qd[1], cur, cur0, status, ns, qo, qdo);
}

}  // namespace mabd
