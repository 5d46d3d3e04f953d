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
// Leaf-to-root elimination in dual form.  Each body j keeps its condensed
// local inverse P (12x12, one row per lane of a 16-lane team) and free
// response w.  Absorbing a joint i whose far side is already condensed into
// (Sigma_i, rho_i) is the Woodbury update
//   M = L P L^T + Sigma,  a = M^{-1}(L w + rho),  w -= P L^T a,  P -= P L^T M^{-1} L P,
// the exact elimination of that joint's multipliers (Sec. 5.3, Eq. module3-kkt;
// one-sided joints have Sigma = 0).  For the parent joint k the body then
// reports Sigma_k = L_k P L_k^T and rho_k = L_k w + C_k.  Multipliers follow
// root to leaf as lambda_i = a_i - E_i lambda_k.
constexpr int TEAMS = 16;
constexpr int TREE_BLOCK = TEAMS * TEAM;
constexpr int MR = MAX_UNARY_ROWS;  // max rows absorbed at once

struct TeamLds {
  double L[MR * 12];
  double Lk[5 * 12];
  double Y[12 * MR];
  double w[12];
  double M[MR * MR];
  double Mi[MR * MR];
  double y[MR];
  double a[MR];
  double Tk[12 * 5];
  double Z[MR * 5];
};

DEV void team_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// in-place inverse of an SPD n x n (n <= MR) by Cholesky; false if not SPD
DEV bool spd_inverse(int n, const double *M, double *Mi) {
  double Lc[MR * MR];
  for (int i = 0; i < n * n; ++i) Lc[i] = M[i];
  for (int j = 0; j < n; ++j) {
    double d = Lc[j * n + j];
    for (int k = 0; k < j; ++k) d -= Lc[j * n + k] * Lc[j * n + k];
    if (!(d > 0.0)) return false;
    d = sqrt(d);
    Lc[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = Lc[i * n + j];
      for (int k = 0; k < j; ++k) s -= Lc[i * n + k] * Lc[j * n + k];
      Lc[i * n + j] = s / d;
    }
  }
  // inverse column by column
  for (int c = 0; c < n; ++c) {
    double x[MR];
    for (int i = 0; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= Lc[i * n + k] * x[k];
      x[i] = s / Lc[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = x[i];
      for (int k = i + 1; k < n; ++k) s -= Lc[k * n + i] * x[k];
      x[i] = s / Lc[i * n + i];
    }
    for (int i = 0; i < n; ++i) Mi[i * n + c] = x[i];
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double v = 0.5 * (Mi[i * n + j] + Mi[j * n + i]);
      Mi[i * n + j] = Mi[j * n + i] = v;
    }
  return true;
}




__global__ __launch_bounds__(TREE_BLOCK) void tree_forward_kernel(TreeArgs a, const GJoint *J) {
  __shared__ TeamLds team_lds[TEAMS];
  const int tm = threadIdx.x / TEAM, ln = threadIdx.x % TEAM;
  TeamLds &S = team_lds[tm];
  if (skip_step(a.status, a.step)) return;
  const int l0 = a.comp_lvl[blockIdx.x], l1 = a.comp_lvl[blockIdx.x + 1];
  for (int lv = l0; lv < l1; ++lv) {
    const int s0 = a.lvl_off[lv], s1 = a.lvl_off[lv + 1];
    for (int slot = s0 + tm; slot < s1; slot += TEAMS) {
      const int64_t b = a.tbody[slot];
      const double *Th = a.hinv + (int64_t)HINV_STRIDE * a.shp[b];
      double P[12];
      double wr = 0.0;
      if (ln < 12) {
        double e[12];
        for (int i = 0; i < 12; ++i) e[i] = (i == ln) ? 1.0 : 0.0;
        hinv_apply(Th, e, P);  // row ln of Hbar^{-1} (symmetric)
        wr = a.u[ln * a.ns + b];
        S.w[ln] = wr;
      }
      const int pk = a.tpk[slot];
      const int kpar = pk >= 0 ? (pk >> 1) : -1;
      const int ck = kpar >= 0 ? (J[kpar].type ? 5 : 3) : 0;
      if (kpar >= 0) {
        const double *Lsrc = a.gl + (int64_t)GL_STRIDE * kpar + ((pk & 1) ? GL_LB : GL_LA);
        for (int i = ln; i < ck * 12; i += TEAM) S.Lk[i] = Lsrc[i];
      }
      team_sync();
      const int e0 = a.tabs_off[slot], e1 = a.tabs_off[slot + 1];
      // children first, then the stacked one-sided rows
      for (int pass = 0; pass < 2; ++pass) {
        int nrow = 0;
        if (pass == 0) {
          // one child joint at a time
          for (int e = e0; e < e1; ++e) {
            const int ent = a.tabs[e];
            if (ent & 1) continue;
            const int k = ent >> 2, side = (ent >> 1) & 1;
            const int c = J[k].type ? 5 : 3;
            const double *Lsrc = a.gl + (int64_t)GL_STRIDE * k + (side ? GL_LB : GL_LA);
            const double *gtk = a.gt + (int64_t)GT_STRIDE * k;
            for (int i = ln; i < c * 12; i += TEAM) S.L[i] = Lsrc[i];
            for (int i = ln; i < c * c; i += TEAM) S.M[i] = gtk[GT_SIG + (i / c) * 5 + (i % c)];
            if (ln < c) S.y[ln] = gtk[GT_RHO + ln];
            team_sync();
            if (ln < 12)
              for (int cc = 0; cc < c; ++cc) {
                double v = 0.0;
                for (int s = 0; s < 12; ++s) v += P[s] * S.L[cc * 12 + s];
                S.Y[ln * MR + cc] = v;
              }
            team_sync();
            for (int i = ln; i < c * c; i += TEAM) {
              const int r = i / c, d = i % c;
              double v = S.M[i];
              for (int s = 0; s < 12; ++s) v += S.L[r * 12 + s] * S.Y[s * MR + d];
              S.M[i] = v;
            }
            if (ln < c) {
              double v = S.y[ln];
              for (int s = 0; s < 12; ++s) v += S.L[ln * 12 + s] * S.w[s];
              S.y[ln] = v;
            }
            team_sync();
            if (ln == 0) {
              if (!spd_inverse(c, S.M, S.Mi)) {
                raise_flag(a.status, FLAG_SINGULAR, a.step);
                for (int i = 0; i < c * c; ++i) S.Mi[i] = 0.0;
              }
              for (int r = 0; r < c; ++r) {
                double v = 0.0;
                for (int d = 0; d < c; ++d) v += S.Mi[r * c + d] * S.y[d];
                S.a[r] = v;
              }
            }
            team_sync();
            if (ln < 12) {
              double G[MR];
              double dw = 0.0;
              for (int d = 0; d < c; ++d) {
                double v = 0.0;
                for (int cc = 0; cc < c; ++cc) v += S.Y[ln * MR + cc] * S.Mi[cc * c + d];
                G[d] = v;
                dw += S.Y[ln * MR + d] * S.a[d];
              }
              wr -= dw;
              for (int s = 0; s < 12; ++s) {
                double v = 0.0;
                for (int d = 0; d < c; ++d) v += G[d] * S.Y[s * MR + d];
                P[s] -= v;
              }
            }
            team_sync();
            if (ln < 12) S.w[ln] = wr;
            team_sync();
          }
        } else {
          // stack the one-sided rows
          for (int e = e0; e < e1; ++e) {
            const int ent = a.tabs[e];
            if (!(ent & 1)) continue;
            const int k = ent >> 2, side = (ent >> 1) & 1;
            const int c = J[k].type ? 5 : 3;
            const double *Lsrc = a.gl + (int64_t)GL_STRIDE * k + (side ? GL_LB : GL_LA);
            for (int i = ln; i < c * 12; i += TEAM) S.L[nrow * 12 + i] = Lsrc[i];
            if (ln < c) S.y[nrow + ln] = a.gl[(int64_t)GL_STRIDE * k + GL_C + ln];
            nrow += c;
          }
          if (nrow == 0) break;
          const int c = nrow;
          for (int i = ln; i < c * c; i += TEAM) S.M[i] = 0.0;
          team_sync();
          if (ln < 12)
            for (int cc = 0; cc < c; ++cc) {
              double v = 0.0;
              for (int s = 0; s < 12; ++s) v += P[s] * S.L[cc * 12 + s];
              S.Y[ln * MR + cc] = v;
            }
          team_sync();
          for (int i = ln; i < c * c; i += TEAM) {
            const int r = i / c, d = i % c;
            double v = 0.0;
            for (int s = 0; s < 12; ++s) v += S.L[r * 12 + s] * S.Y[s * MR + d];
            S.M[i] = v;
          }
          if (ln < c) {
            double v = S.y[ln];
            for (int s = 0; s < 12; ++s) v += S.L[ln * 12 + s] * S.w[s];
            S.y[ln] = v;
          }
          // Z = Y^T L_k^T  (coupling of these rows to the parent joint)
          for (int i = ln; i < c * ck; i += TEAM) {
            const int r = i / ck, f = i % ck;
            double v = 0.0;
            for (int s = 0; s < 12; ++s) v += S.Y[s * MR + r] * S.Lk[f * 12 + s];
            S.Z[r * 5 + f] = v;
          }
          team_sync();
          if (ln == 0) {
            if (!spd_inverse(c, S.M, S.Mi)) {
              raise_flag(a.status, FLAG_SINGULAR, a.step);
              for (int i = 0; i < c * c; ++i) S.Mi[i] = 0.0;
            }
            for (int r = 0; r < c; ++r) {
              double v = 0.0;
              for (int d = 0; d < c; ++d) v += S.Mi[r * c + d] * S.y[d];
              S.a[r] = v;
            }
          }
          team_sync();
          // a_u, E_u = M^{-1} Z, scattered to the individual joints
          {
            int off = 0;
            for (int e = e0; e < e1; ++e) {
              const int ent = a.tabs[e];
              if (!(ent & 1)) continue;
              const int k = ent >> 2;
              const int cj = J[k].type ? 5 : 3;
              double *gtk = a.gt + (int64_t)GT_STRIDE * k;
              if (ln < cj) gtk[GT_A + ln] = S.a[off + ln];
              for (int i = ln; i < cj * 5; i += TEAM) {
                const int r = i / 5, f = i % 5;
                double v = 0.0;
                if (f < ck)
                  for (int d = 0; d < c; ++d) v += S.Mi[(off + r) * c + d] * S.Z[d * 5 + f];
                gtk[GT_E + i] = v;
              }
              off += cj;
            }
          }
          if (ln < 12) {
            double G[MR];
            double dw = 0.0;
            for (int d = 0; d < c; ++d) {
              double v = 0.0;
              for (int cc = 0; cc < c; ++cc) v += S.Y[ln * MR + cc] * S.Mi[cc * c + d];
              G[d] = v;
              dw += S.Y[ln * MR + d] * S.a[d];
            }
            wr -= dw;
            for (int s = 0; s < 12; ++s) {
              double v = 0.0;
              for (int d = 0; d < c; ++d) v += G[d] * S.Y[s * MR + d];
              P[s] -= v;
            }
          }
          team_sync();
          if (ln < 12) S.w[ln] = wr;
          team_sync();
        }
      }
      // parent joint: T_k = P L_k^T, Sigma_k = L_k T_k, rho_k = L_k w + C_k
      if (kpar >= 0) {
        if (ln < 12)
          for (int f = 0; f < ck; ++f) {
            double v = 0.0;
            for (int s = 0; s < 12; ++s) v += P[s] * S.Lk[f * 12 + s];
            S.Tk[ln * 5 + f] = v;
          }
        team_sync();
        double *gtk = a.gt + (int64_t)GT_STRIDE * kpar;
        for (int i = ln; i < ck * ck; i += TEAM) {
          const int r = i / ck, f = i % ck;
          double v = 0.0;
          for (int s = 0; s < 12; ++s) v += S.Lk[r * 12 + s] * S.Tk[s * 5 + f];
          gtk[GT_SIG + r * 5 + f] = v;
        }
        if (ln < ck) {
          double v = a.gl[(int64_t)GL_STRIDE * kpar + GL_C + ln];
          for (int s = 0; s < 12; ++s) v += S.Lk[ln * 12 + s] * S.w[s];
          gtk[GT_RHO + ln] = v;
        }
        team_sync();
      }
      // child joints: lambda_i = Sigma_i^{-1}(L_i dp_j + rho_i), dp_j = w - P L_k^T lambda_k
      for (int e = e0; e < e1; ++e) {
        const int ent = a.tabs[e];
        if (ent & 1) continue;
        const int k = ent >> 2, side = (ent >> 1) & 1;
        const int c = J[k].type ? 5 : 3;
        const double *Lsrc = a.gl + (int64_t)GL_STRIDE * k + (side ? GL_LB : GL_LA);
        double *gtk = a.gt + (int64_t)GT_STRIDE * k;
        for (int i = ln; i < c * 12; i += TEAM) S.L[i] = Lsrc[i];
        for (int i = ln; i < c * c; i += TEAM) S.M[i] = gtk[GT_SIG + (i / c) * 5 + (i % c)];
        team_sync();
        // y = L w + rho ; Z = L T_k
        if (ln < c) {
          double v = gtk[GT_RHO + ln];
          for (int s = 0; s < 12; ++s) v += S.L[ln * 12 + s] * S.w[s];
          S.y[ln] = v;
        }
        for (int i = ln; i < c * ck; i += TEAM) {
          const int r = i / ck, f = i % ck;
          double v = 0.0;
          for (int s = 0; s < 12; ++s) v += S.L[r * 12 + s] * S.Tk[s * 5 + f];
          S.Z[r * 5 + f] = v;
        }
        team_sync();
        if (ln == 0) {
          if (!spd_inverse(c, S.M, S.Mi)) {
            raise_flag(a.status, FLAG_SINGULAR, a.step);
            for (int i = 0; i < c * c; ++i) S.Mi[i] = 0.0;
          }
        }
        team_sync();
        if (ln < c) {
          double v = 0.0;
          for (int d = 0; d < c; ++d) v += S.Mi[ln * c + d] * S.y[d];
          gtk[GT_A + ln] = v;
        }
        for (int i = ln; i < c * 5; i += TEAM) {
          const int r = i / 5, f = i % 5;
          double v = 0.0;
          if (f < ck)
            for (int d = 0; d < c; ++d) v += S.Mi[r * c + d] * S.Z[d * 5 + f];
          gtk[GT_E + i] = v;
        }
        team_sync();
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void tree_backward_kernel(TreeArgs a, const GJoint *J) {
  if (skip_step(a.status, a.step)) return;
  const int l0 = a.comp_lvl[blockIdx.x], l1 = a.comp_lvl[blockIdx.x + 1];
  for (int lv = l1 - 1; lv >= l0; --lv) {
    const int s0 = a.lvl_off[lv], s1 = a.lvl_off[lv + 1];
    for (int slot = s0 + threadIdx.x; slot < s1; slot += blockDim.x) {
      const int pk = a.tpk[slot];
      const int kpar = pk >= 0 ? (pk >> 1) : -1;
      const int ck = kpar >= 0 ? (J[kpar].type ? 5 : 3) : 0;
      double lk[5] = {0, 0, 0, 0, 0};
      for (int i = 0; i < ck; ++i) lk[i] = a.glam[5 * (int64_t)kpar + i];
      for (int e = a.tabs_off[slot]; e < a.tabs_off[slot + 1]; ++e) {
        const int k = a.tabs[e] >> 2;
        const int c = J[k].type ? 5 : 3;
        const double *gtk = a.gt + (int64_t)GT_STRIDE * k;
        for (int r = 0; r < c; ++r) {
          double v = gtk[GT_A + r];
          for (int f = 0; f < ck; ++f) v -= gtk[GT_E + 5 * r + f] * lk[f];
          a.glam[5 * (int64_t)k + r] = v;
        }
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
}

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
void launch_tree(const TreeArgs &a, const GJoint *J, int ncomp, hipStream_t s) {
  if (ncomp > 0) {
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
