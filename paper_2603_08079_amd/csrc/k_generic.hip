// Generic-topology kernels of libmabd: per-shape factors, per-body co-rotated
// solve, per-joint rows, tree elimination, back-projection, state gather.
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
__global__ void gbody_kernel(int b0, int b1, const double *q, const double *qn, const double *qdn,
                             int64_t ns, const int32_t *shp, const double *hinv,
                             const double *shape, double g0, double g1, double g2, double h,
                             double *Rg, double *ug, uint32_t *status, int step) {
  int64_t b = (int64_t)b0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= b1 || skip_step(status, step)) return;
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
  double phi[12], u[12];
  local_force<double>(shape + (int64_t)SHAPE_STRIDE * s, R, A, qq, qnn, qd, g, h, phi);
  hinv_apply(hinv + (int64_t)HINV_STRIDE * s, phi, u);
#pragma unroll
  for (int i = 0; i < 9; ++i) Rg[i * ns + b] = R[i];
#pragma unroll
  for (int i = 0; i < 12; ++i) ug[i * ns + b] = u[i];
}

// ------------------------------------------------------- (b) generic joints
// Constraint value C and the local-frame gradients L = G diag4(R) of both
// sides (Eq. ball; Eq. hinge with Eqs. pcpq, pcpr, r_gradient).  For a ball
// end L = s R J(p); for the hinge frame owner L = S_H diag2(dR_H)[J(p1); J(p2)]
// plus the A-linearised rotation term (rbar_c (x) R_a^T d_m) on the A columns;
// for the other side L = -S_H diag2(R_H R_b)[J(p1); J(p2)].
__global__ void gjoint_kernel(int m, const GJoint *J, const double *q, const double *Rg, int64_t ns,
                              int hinge_grad, double *gl) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const GJoint j = J[k];
  double *out = gl + (int64_t)GL_STRIDE * k;
  double Aa[9], ta[3], Ab[9], tb[3], Ra[9], Rb[9];
  const bool da = j.sa >= 0, db = j.sb >= 0;
  for (int side = 0; side < 2; ++side) {
    const int64_t b = side == 0 ? j.sa : j.sb;
    double *A = side == 0 ? Aa : Ab, *t = side == 0 ? ta : tb, *R = side == 0 ? Ra : Rb;
    if (b >= 0) {
      for (int i = 0; i < 3; ++i) {
        for (int c = 0; c < 3; ++c) A[3 * i + c] = q[(3 * c + i) * ns + b];
        t[i] = q[(9 + i) * ns + b];
      }
      for (int i = 0; i < 9; ++i) R[i] = Rg[i * ns + b];
    } else {
      for (int i = 0; i < 9; ++i) { A[i] = (i % 4 == 0) ? 1.0 : 0.0; R[i] = A[i]; }
      t[0] = t[1] = t[2] = 0.0;
    }
  }
  for (int i = 0; i < GL_STRIDE; ++i) out[i] = 0.0;
  auto point_diff = [&](const double *pa_, const double *pb_, double *d) {
    double wa[3], wb[3];
    mat3_vec(Aa, pa_, wa);
    mat3_vec(Ab, pb_, wb);
    for (int i = 0; i < 3; ++i) d[i] = (ta[i] - tb[i]) + (wa[i] - wb[i]);
  };
  if (j.type == 0) {
    double C[3];
    point_diff(j.p1a, j.p1b, C);
    for (int i = 0; i < 3; ++i) out[GL_C + i] = C[i];
    for (int side = 0; side < 2; ++side) {
      if (side == 0 ? !da : !db) continue;
      const double *R = side == 0 ? Ra : Rb;
      const double *p = side == 0 ? j.p1a : j.p1b;
      const double s = side == 0 ? 1.0 : -1.0;
      double *L = out + (side == 0 ? GL_LA : GL_LB);
      for (int r = 0; r < 3; ++r)
        for (int i = 0; i < 3; ++i) {
          for (int c = 0; c < 3; ++c) L[12 * r + 3 * c + i] = s * R[3 * r + i] * p[c];
          L[12 * r + 9 + i] = s * R[3 * r + i];
        }
    }
    return;
  }
  double d1[3], d2[3];
  point_diff(j.p1a, j.p1b, d1);
  point_diff(j.p2a, j.p2b, d2);
  double RH[9];
  if (j.flags & GJ_FLAG_STATIC_OWNER) {
    for (int i = 0; i < 9; ++i) RH[i] = j.dR[i];
  } else {
    mat3_mul_bt(j.dR, Ra, RH);  // R_H = dR_H R_a^T
  }
  double e1[3], e2[3];
  mat3_vec(RH, d1, e1);
  mat3_vec(RH, d2, e2);
  out[GL_C + 0] = e1[0]; out[GL_C + 1] = e1[1]; out[GL_C + 2] = e1[2];
  out[GL_C + 3] = e2[0]; out[GL_C + 4] = e2[2];
  const int cpi[5] = {0, 0, 0, 1, 1};
  const int comp[5] = {0, 1, 2, 0, 2};
  if (da) {
    // frozen part: dR_H rows times J(p_m)
    double *L = out + GL_LA;
    double Rtd[2][3];
    mat3t_vec(Ra, d1, Rtd[0]);
    mat3t_vec(Ra, d2, Rtd[1]);
    for (int i = 0; i < 5; ++i) {
      const double *p = cpi[i] == 0 ? j.p1a : j.p2a;
      const double *rr = j.dR + 3 * comp[i];
      for (int jj = 0; jj < 3; ++jj) {
        for (int c = 0; c < 3; ++c) L[12 * i + 3 * c + jj] = rr[jj] * p[c];
        L[12 * i + 9 + jj] = rr[jj];
      }
      if (hinge_grad == 0) {
        const double *w = Rtd[cpi[i]];
        for (int l = 0; l < 3; ++l)
          for (int kk = 0; kk < 3; ++kk) L[12 * i + 3 * l + kk] += rr[l] * w[kk];
      }
    }
  }
  if (db) {
    double Q[9];
    mat3_mul(RH, Rb, Q);
    double *L = out + GL_LB;
    for (int i = 0; i < 5; ++i) {
      const double *p = cpi[i] == 0 ? j.p1b : j.p2b;
      const double *rr = Q + 3 * comp[i];
      for (int jj = 0; jj < 3; ++jj) {
        for (int c = 0; c < 3; ++c) L[12 * i + 3 * c + jj] = -rr[jj] * p[c];
        L[12 * i + 9 + jj] = -rr[jj];
      }
    }
  }
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

struct TeamLds {
  double L[TREE_KLDS * 12];
  double Y[12 * TREE_KLDS];
  double K[TREE_KLDS * TREE_KLDS];
  double y[TREE_KLDS];
  int32_t rowk[TREE_KLDS];   // joint of each clique row
  int32_t rowi[TREE_KLDS];   // row index inside that joint
};

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
__global__ __launch_bounds__(TREE_BLOCK) void tree_prep_kernel(TreeArgs a, const GJoint *J, int nslots) {
  __shared__ TeamLds team_lds[TEAMS];
  const int tm = threadIdx.x / TEAM, ln = threadIdx.x % TEAM;
  TeamLds &S = team_lds[tm];
  if (skip_step(a.status, a.step)) return;
  const int slot = blockIdx.x * TEAMS + tm;
  if (slot >= nslots) return;  // whole teams only: team_sync is wave-local
  const int64_t b = a.tbody[slot];
  const double *Th = a.hinv + (int64_t)HINV_STRIDE * a.shp[b];
  const int pk = a.tpk[slot];
  const int kpar = pk >= 0 ? (pk >> 1) : -1;
  const int ck = kpar >= 0 ? (J[kpar].type ? 5 : 3) : 0;
  const int e0 = a.tabs_off[slot], e1 = a.tabs_off[slot + 1];
  const int ne = a.tne[slot];
  const int nr = ne + ck;
  if (nr == 0) return;
  double *fac = a.fac + a.foff[slot];  // nr*nr K, nr y, then (big cliques) L, Y
  const bool big = nr > TREE_KLDS;
  double *Lm = big ? fac + nr * nr + nr : S.L;
  double *Ym = big ? fac + nr * nr + nr + 12 * nr : S.Y;
  // 1) clique rows: absorbed joints in list order, then the parent joint
  {
    int r0 = 0;
    for (int e = e0; e <= e1; ++e) {
      int k, side;
      if (e < e1) {
        k = a.tabs[e] >> 2;
        side = (a.tabs[e] >> 1) & 1;
      } else {
        if (kpar < 0) break;
        k = kpar;
        side = pk & 1;
      }
      const int c = J[k].type ? 5 : 3;
      const double *Lsrc = a.gl + (int64_t)GL_STRIDE * k + (side ? GL_LB : GL_LA);
      for (int i = ln; i < c * 12; i += TEAM) Lm[r0 * 12 + i] = Lsrc[i];
      r0 += c;
    }
  }
  team_sync();
  // 2) Y = Hbar^{-1} L^T, one clique row per lane
  for (int col = ln; col < nr; col += TEAM) {
    double yv[12];
    hinv_apply(Th, Lm + 12 * col, yv);
    for (int s = 0; s < 12; ++s) Ym[s * nr + col] = yv[s];
  }
  team_sync();
  // 3) K0 = L Y (lower triangle), y0 = L u + C of one-sided and parent rows
  for (int idx = ln; idx < nr * nr; idx += TEAM) {
    const int i = idx / nr, jj = idx % nr;
    double v = 0.0;
    if (jj <= i)
      for (int s = 0; s < 12; ++s) v += Lm[12 * i + s] * Ym[s * nr + jj];
    fac[idx] = v;
  }
  for (int i = ln; i < nr; i += TEAM) {
    double v = 0.0;
    for (int s = 0; s < 12; ++s) v += Lm[12 * i + s] * a.u[s * a.ns + b];
    fac[nr * nr + i] = v;
  }
  team_sync();
  {
    int r0 = 0;
    for (int e = e0; e <= e1; ++e) {
      int k, unary;
      if (e < e1) {
        k = a.tabs[e] >> 2;
        unary = a.tabs[e] & 1;
      } else {
        if (kpar < 0) break;
        k = kpar;
        unary = 1;  // parent rows take C_k only
      }
      const int c = J[k].type ? 5 : 3;
      if (e == e1 || unary)
        for (int i = ln; i < c; i += TEAM) fac[nr * nr + r0 + i] += a.gl[(int64_t)GL_STRIDE * k + GL_C + i];
      r0 += c;
    }
  }
}

// Leaves first, per level: add the condensed far sides (Sigma, rho) of the
// child joints to K0, y0, factor the absorbed rows (partial Cholesky) and
// pass the Schur complement on the parent joint up.  One workgroup per
// component; a 16-lane team per body of the level.
__global__ __launch_bounds__(TREE_BLOCK) void tree_forward_kernel(TreeArgs a, const GJoint *J) {
  __shared__ TeamLds team_lds[TEAMS];
  const int tm = threadIdx.x / TEAM, ln = threadIdx.x % TEAM;
  TeamLds &S = team_lds[tm];
  if (skip_step(a.status, a.step)) return;
  const int l0 = a.comp_lvl[blockIdx.x], l1 = a.comp_lvl[blockIdx.x + 1];
  for (int lv = l0; lv < l1; ++lv) {
    const int s0 = a.lvl_off[lv], s1 = a.lvl_off[lv + 1];
    for (int slot = s0 + tm; slot < s1; slot += TEAMS) {
      const int pk = a.tpk[slot];
      const int kpar = pk >= 0 ? (pk >> 1) : -1;
      const int ck = kpar >= 0 ? (J[kpar].type ? 5 : 3) : 0;
      const int e0 = a.tabs_off[slot], e1 = a.tabs_off[slot + 1];
      const int ne = a.tne[slot];
      const int nr = ne + ck;
      if (nr == 0) continue;
      double *fac = a.fac + a.foff[slot];
      const bool big = nr > TREE_KLDS;
      double *Km = big ? fac : S.K;
      double *ym = big ? fac + nr * nr : S.y;
      if (!big) {
        for (int idx = ln; idx < nr * nr; idx += TEAM) Km[idx] = fac[idx];
        for (int i = ln; i < nr; i += TEAM) ym[i] = fac[nr * nr + i];
      }
      team_sync();
      // condensed far sides of the child joints
      {
        int r0 = 0;
        for (int e = e0; e < e1; ++e) {
          const int k = a.tabs[e] >> 2;
          const int c = J[k].type ? 5 : 3;
          if (!(a.tabs[e] & 1)) {
            const double *gtk = a.gt + (int64_t)GT_STRIDE * k;
            for (int idx = ln; idx < c * c; idx += TEAM) {
              const int i = idx / c, jj = idx % c;
              if (jj <= i) Km[(r0 + i) * nr + r0 + jj] += gtk[GT_SIG + 5 * i + jj];
            }
            for (int i = ln; i < c; i += TEAM) ym[r0 + i] += gtk[GT_RHO + i];
          }
          r0 += c;
        }
      }
      team_sync();
      // partial Cholesky over the ne absorbed rows (lower triangle, in place)
      for (int p = 0; p < ne; ++p) {
        if (ln == 0) {
          double d = Km[p * nr + p];
          if (!(d > 0.0)) {
            raise_flag(a.status, FLAG_SINGULAR, a.step);
            d = 1.0;
          }
          d = sqrt(d);
          Km[p * nr + p] = d;
          ym[p] /= d;
        }
        team_sync();
        const double d = Km[p * nr + p];
        for (int i = p + 1 + ln; i < nr; i += TEAM) Km[i * nr + p] /= d;
        team_sync();
        for (int i = p + 1 + ln; i < nr; i += TEAM) {
          const double lip = Km[i * nr + p];
          for (int jj = p + 1; jj <= i; ++jj) Km[i * nr + jj] -= lip * Km[jj * nr + p];
          ym[i] -= lip * ym[p];
        }
        team_sync();
      }
      // Schur complement on the parent joint; factor to the body's slot
      if (kpar >= 0) {
        double *gtk = a.gt + (int64_t)GT_STRIDE * kpar;
        for (int idx = ln; idx < 25; idx += TEAM) {
          const int i = idx / 5, jj = idx % 5;
          double v = 0.0;
          if (i < ck && jj < ck) v = jj <= i ? Km[(ne + i) * nr + ne + jj] : Km[(ne + jj) * nr + ne + i];
          gtk[GT_SIG + idx] = v;
        }
        if (ln < 5) gtk[GT_RHO + ln] = ln < ck ? ym[ne + ln] : 0.0;
      }
      if (!big) {
        for (int idx = ln; idx < nr * nr; idx += TEAM) fac[idx] = Km[idx];
        for (int i = ln; i < nr; i += TEAM) fac[nr * nr + i] = ym[i];
      }
      team_sync();
    }
    __syncthreads();
  }
}

// root to leaf: lambda_e = Lc^{-T} (z - X lambda_k), one thread per body
__global__ __launch_bounds__(256) void tree_backward_kernel(TreeArgs a, const GJoint *J) {
  if (skip_step(a.status, a.step)) return;
  const int l0 = a.comp_lvl[blockIdx.x], l1 = a.comp_lvl[blockIdx.x + 1];
  for (int lv = l1 - 1; lv >= l0; --lv) {
    const int s0 = a.lvl_off[lv], s1 = a.lvl_off[lv + 1];
    for (int slot = s0 + threadIdx.x; slot < s1; slot += blockDim.x) {
      const int pk = a.tpk[slot];
      const int kpar = pk >= 0 ? (pk >> 1) : -1;
      const int ck = kpar >= 0 ? (J[kpar].type ? 5 : 3) : 0;
      const int ne = a.tne[slot];
      const int nr = ne + ck;
      if (ne == 0) continue;
      const double *K = a.fac + a.foff[slot];
      const double *y = K + nr * nr;
      double lk[5] = {0, 0, 0, 0, 0};
      for (int i = 0; i < ck; ++i) lk[i] = a.glam[5 * (int64_t)kpar + i];
      // t = z - X lambda_k, X^T stored in rows ne.. of the factor
      double t[TREE_KMAX];
      for (int i = 0; i < ne; ++i) {
        double v = y[i];
        for (int f = 0; f < ck; ++f) v -= K[(ne + f) * nr + i] * lk[f];
        t[i] = v;
      }
      for (int i = ne - 1; i >= 0; --i) {
        double v = t[i];
        for (int l = i + 1; l < ne; ++l) v -= K[l * nr + i] * t[l];
        t[i] = v / K[i * nr + i];
      }
      int r0 = 0;
      for (int e = a.tabs_off[slot]; e < a.tabs_off[slot + 1]; ++e) {
        const int k = a.tabs[e] >> 2;
        const int c = J[k].type ? 5 : 3;
        for (int i = 0; i < c; ++i) a.glam[5 * (int64_t)k + i] = t[r0 + i];
        for (int i = c; i < 5; ++i) a.glam[5 * (int64_t)k + i] = 0.0;
        r0 += c;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------ (d) back-projection
// dq = diag4(R) (u - Hbar^{-1} sum_k L_k^T lambda_k)  (Eq. primal), then
// q_out = q_cur + dq and qd_out = (accumulate ? qd_out : 0) + dq / h.
__global__ void gapply_kernel(int b0, int b1, const int32_t *inc_off, const int32_t *inc,
                              const double *gl, const double *glam, const double *Rg,
                              const double *ug, int64_t ns, const int32_t *shp, const double *hinv,
                              const double *q_cur, double *q_out, double *qd_out, double h,
                              int accumulate, uint32_t *status, const GJoint *J, int step) {
  int64_t b = (int64_t)b0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= b1 || skip_step(status, step)) return;
  double g12[12];
  for (int i = 0; i < 12; ++i) g12[i] = 0.0;
  for (int e = inc_off[b]; e < inc_off[b + 1]; ++e) {
    const int ent = inc[e];
    const int k = ent >> 1, side = ent & 1;
    const int c = J[k].type ? 5 : 3;
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
      if (!isfinite(dq[i])) raise_flag(status, FLAG_NONFINITE, step);
    }
  }
}

// ------------------------------------------------------------ state copies
// solver-order SoA -> input-order AoS (n x 12) for dynamic bodies
__global__ void gather_state_kernel(int nd, const int32_t *sol2in, const double *q, const double *qd,
                                    int64_t ns, double *qo, double *qdo) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nd) return;
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
                  double h, double *Rg, double *ug, uint32_t *status, int step, hipStream_t s) {
  if (b1 > b0)
    hipLaunchKernelGGL(gbody_kernel, dim3((b1 - b0 + 255) / 256), dim3(256), 0, s, b0, b1, q, qn, qdn,
                       ns, shp, hinv, shape, g[0], g[1], g[2], h, Rg, ug, status, step);
}
void launch_gjoint(int m, const GJoint *J, const double *q, const double *Rg, int64_t ns, int hg,
                   double *gl, hipStream_t s) {
  if (m > 0)
    hipLaunchKernelGGL(gjoint_kernel, dim3((m + 127) / 128), dim3(128), 0, s, m, J, q, Rg, ns, hg, gl);
}
void launch_tree(const TreeArgs &a, const GJoint *J, int ncomp, int nslots, hipStream_t s) {
  if (ncomp > 0) {
    hipLaunchKernelGGL(tree_prep_kernel, dim3((nslots + TEAMS - 1) / TEAMS), dim3(TREE_BLOCK), 0, s, a, J,
                       nslots);
    hipLaunchKernelGGL(tree_forward_kernel, dim3(ncomp), dim3(TREE_BLOCK), 0, s, a, J);
    hipLaunchKernelGGL(tree_backward_kernel, dim3(ncomp), dim3(256), 0, s, a, J);
  }
}
void launch_gapply(int b0, int b1, const int32_t *inc_off, const int32_t *inc, const double *gl,
                   const double *glam, const double *Rg, const double *ug, int64_t ns,
                   const int32_t *shp, const double *hinv, const double *q_cur, double *q_out,
                   double *qd_out, double h, int acc, uint32_t *status, const GJoint *J,
                   int step, hipStream_t s) {
  if (b1 > b0)
    hipLaunchKernelGGL(gapply_kernel, dim3((b1 - b0 + 255) / 256), dim3(256), 0, s, b0, b1, inc_off,
                       inc, gl, glam, Rg, ug, ns, shp, hinv, q_cur, q_out, qd_out, h, acc, status, J,
                       step);
}
void launch_gather_state(int nd, const int32_t *sol2in, const double *q, const double *qd, int64_t ns,
                         double *qo, double *qdo, hipStream_t s) {
  if (nd > 0)
    hipLaunchKernelGGL(gather_state_kernel, dim3((nd + 255) / 256), dim3(256), 0, s, nd, sol2in, q, qd,
                       ns, qo, qdo);
}

}  // namespace mabd
