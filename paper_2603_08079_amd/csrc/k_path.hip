// Dual solve of path components (Sec. 5.3: a tree whose bodies each carry
// at most two joints).  The dual S = G H^{-1} G^T of a path is block
// tridiagonal over its joints in path order: the two diagonal contributions
// of a joint come from its two bodies, the coupling of consecutive joints
// from the body they share, each a block of that body's clique matrix
// K = L Hbar^{-1} L^T over the joint rows L on its side, with right-hand
// side L u (plus C once per joint).  A segment of consecutive units (joints)
// eliminates all but its last unit (the separator) by block Cholesky steps:
//   D_i = L_i L_i^T,  z_i = L_i^{-1} y_i,  W_i = L_i^{-1} E_i,  G_i = L_i^{-1} F_i^T,
//   D_{i+1} -= W_i^T W_i,  y_{i+1} -= W_i^T z_i,  F_{i+1} = -G_i^T W_i,
// where E_i couples unit i with unit i+1 and F_i carries the coupling of
// unit i with the left separator (the previous segment's last unit), whose
// block and right-hand side collect -G_i^T G_i and -G_i^T z_i.  The
// separators form the next level's block-tridiagonal system; a path left
// with one segment solves its separator at once.  Back-substitution:
//   lambda_i = L_i^{-T} (z_i - W_i lambda_{i+1} - G_i lambda_left).
// All blocks are 5x5 (units with fewer rows are padded with the identity).
// Level 0 runs a team of 16 lanes per segment, which forms each body's
// clique from the joint rows and shares the elimination step; the levels
// above (few separators) run one lane per segment on the stored blocks.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "dmath.hpp"
#include "generic.hpp"

namespace mabd {

namespace {

constexpr int PW = 64;      // threads per workgroup (one wave)
constexpr int PT = 16;      // lanes per level-0 team (one segment)
constexpr int PTEAMS = PW / PT;

DEV constexpr int px(int p, int q) { return p * (p + 1) / 2 + q; }
// packed lower index e < 15 -> (p, q)
DEV void unpack15(int e, int &p, int &q) {
  p = e < 1 ? 0 : (e < 3 ? 1 : (e < 6 ? 2 : (e < 10 ? 3 : 4)));
  q = e - p * (p + 1) / 2;
}

// D (packed lower) = L L^T in place, with the reciprocals of the pivots in
// place of L's diagonal (the solves below multiply by them); a non-positive
// pivot raises SINGULAR
DEV void chol5(double D[15], uint32_t *status) {
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    double d = D[px(p, p)];
#pragma unroll
    for (int k = 0; k < p; ++k) d -= D[px(p, k)] * D[px(p, k)];
    if (!(d > 0.0)) {
      raise_flag(status, FLAG_SINGULAR, 0);
      d = 1.0;
    }
    const double inv = 1.0 / sqrt(d);
    D[px(p, p)] = inv;
#pragma unroll
    for (int i = p + 1; i < 5; ++i) {
      double v = D[px(i, p)];
#pragma unroll
      for (int k = 0; k < p; ++k) v -= D[px(i, k)] * D[px(p, k)];
      D[px(i, p)] = v * inv;
    }
  }
}
// x = L^{-1} x (L as chol5 leaves it: reciprocal pivots on the diagonal)
DEV void fsub5(const double L[15], double x[5]) {
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    double v = x[p];
#pragma unroll
    for (int k = 0; k < p; ++k) v -= L[px(p, k)] * x[k];
    x[p] = v * L[px(p, p)];
  }
}
// x = L^{-T} x
DEV void bsub5(const double L[15], double x[5]) {
#pragma unroll
  for (int p = 4; p >= 0; --p) {
    double v = x[p];
#pragma unroll
    for (int k = p + 1; k < 5; ++k) v -= L[px(k, p)] * x[k];
    x[p] = v * L[px(p, p)];
  }
}

DEV void team_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// one level-0 team's shared state.  st holds a unit record (PU_* layout):
// the current unit's block and right-hand side, the coupling with the left
// separator, and what the left separator collects; the next unit's block
// and right-hand side alternate with the current one's (cur / nxt)
struct PathTeam {
  union {
    double L[10 * 12];      // clique rows of the current body (first joint, then second),
    double fr[PATH_FREC];   // dead once its K is formed: then the factors of the unit just
  };                        // eliminated, L, z, W, G (stored before the next body's rows)
  double th[HINV_STRIDE];   // its Hbar^{-1}
  double uu[12];            // its local solve u
  double K[55];             // its clique matrix (packed lower) ...
  double yl[10];            // ... and L u
  double st[PATH_UREC];     // D (15), y (5), F (25), dD (15), dy (5)
  double Db[15], yb[5];     // the other block buffer
  double E[25];             // coupling with the next unit
  PathUnitF rec[PATH_TMAX + 1];  // units u0 - 1 .. u0 + t - 1
  int32_t shb[PATH_TMAX + 1];    // shape of each unit's body after
  int32_t shp0;                  // shape of the first unit's body before
};

// what one body's clique needs from memory, held in registers while the
// previous unit is eliminated: its rows (eight per lane), u, Hbar^{-1}
struct CliqueLoad {
  double v[8], u, t0, t1;
};
struct CliqueDesc {
  int body, shp, gA, sA, rA, gB, sB, rB;
};

DEV CliqueLoad clique_issue(const TreeArgs &a, const CliqueDesc &d, int ln) {
  CliqueLoad c;
  const int nr = d.rA + d.rB;
  c.u = ln < 12 && d.body >= 0 ? a.u[(int64_t)ln * a.ns + d.body] : 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {  // up to 10 rows x 12
    const int idx = ln + k * PT;
    const int r = idx < nr * 12 ? idx / 12 : 0, col = idx % 12;
    const bool inA = r < d.rA;
    const int g = inA ? d.gA : d.gB, sd = inA ? d.sA : d.sB, rr = inA ? r : r - d.rA;
    c.v[k] = d.body >= 0 && idx < nr * 12 ? a.gl[(int64_t)GL_STRIDE * g + (sd ? GL_LB : GL_LA) + 12 * rr + col]
                                          : 0.0;
  }
  const double *Th = a.hinv + (int64_t)HINV_STRIDE * (d.body >= 0 ? d.shp : 0);
  c.t0 = Th[ln];
  c.t1 = ln + PT < HINV_STRIDE ? Th[ln + PT] : 0.0;
  return c;
}

// the clique of one body over joint A (rA rows, 0: none) then joint B (rB
// rows, 0: none), on its side of each: K and L u into the team's LDS
DEV void clique_form(const TreeArgs &a, PathTeam &S, const CliqueLoad &c, const CliqueDesc &d, int ln) {
  const int nr = d.rA + d.rB;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int idx = ln + k * PT;
    if (idx < nr * 12) S.L[idx] = c.v[k];
  }
  S.th[ln] = c.t0;
  if (ln + PT < HINV_STRIDE) S.th[ln + PT] = c.t1;
  if (ln < 12) S.uu[ln] = c.u;
  team_sync();
  // lane j forms column j of K (lower part) from Hbar^{-1} L_j^T in registers
  if (ln < nr) {
    if (a.f32) {
      float lf[12], yf[12];
#pragma unroll
      for (int s = 0; s < 12; ++s) lf[s] = (float)S.L[12 * ln + s];
      hinv_apply(S.th, lf, yf);
      for (int i = ln; i < nr; ++i) {
        float w = 0.0f;
#pragma unroll
        for (int s = 0; s < 12; ++s) w += (float)S.L[12 * i + s] * yf[s];
        S.K[px(i, ln)] = (double)w;
      }
    } else {
      double yv[12];
      hinv_apply(S.th, S.L + 12 * ln, yv);
      for (int i = ln; i < nr; ++i) {
        double w = 0.0;
#pragma unroll
        for (int s = 0; s < 12; ++s) w += S.L[12 * i + s] * yv[s];
        S.K[px(i, ln)] = w;
      }
    }
    double w = 0.0;
#pragma unroll
    for (int s = 0; s < 12; ++s) w += S.L[12 * ln + s] * S.uu[s];
    S.yl[ln] = w;
  }
}

// a unit's constraint value (Eq. kkt's -C right-hand side), or the
// refinement's or the loop-breaker's in its place
DEV double unit_c(const TreeArgs &a, int gj, int row) {
  if (a.zero_c) return 0.0;
  return a.cc ? a.cc[5 * (int64_t)gj + row] : a.gl[(int64_t)GL_STRIDE * gj + GL_C + row];
}

__global__ __launch_bounds__(PW) __attribute__((amdgpu_waves_per_eu(3))) void path_fwd0_kernel(TreeArgs a, PathPlan P) {
  __shared__ PathTeam team_lds[PTEAMS];
  const int tm = threadIdx.x / PT, ln = threadIdx.x % PT;
  PathTeam &S = team_lds[tm];
  const int nseg = P.seg_off[1] - P.seg_off[0];
  const int g = blockIdx.x * PTEAMS + tm;
  const StepGate gate = step_gate(a.status);
  if (g >= nseg) return;  // whole teams only: team_sync is wave-local
  const PathSeg sg = P.seg[g];
  if (gate.skip()) return;
  const bool left = sg.flags & 1, last = (sg.flags & 2) != 0, top = (sg.flags & 4) != 0;
  const int t = sg.t;  // <= PATH_TMAX (the planner's bound)
  double *fac = P.fac + P.fac_off[0] + (int64_t)g * (P.T0 - 1) * PATH_FREC;
  // the segment's unit records and the shapes of their bodies, once
  for (int j = ln; j <= t; j += PT) {
    const int u = sg.u0 - 1 + j;
    PathUnitF U{};
    if (u >= 0) U = P.uf[u];
    S.rec[j] = U;
    S.shb[j] = u >= 0 && U.ba >= 0 ? a.shp[U.ba] : 0;
    if (j == 1) S.shp0 = U.bb >= 0 ? a.shp[U.bb] : 0;
  }
  for (int e = ln; e < PATH_UREC; e += PT) S.st[e] = 0.0;
  team_sync();
  double *D = S.st + PU_D, *y = S.st + PU_Y, *Dn = S.Db, *yn = S.yb;
  double *F = S.st + PU_F, *dD = S.st + PU_DD, *dy = S.st + PU_DY;
  const PathUnitF U0 = S.rec[1];
  if (ln < 5) D[px(ln, ln)] = ln < U0.r ? 0.0 : 1.0;
  // step -1: the first unit's block from the body before it and (left
  // separator) the coupling with the previous unit
  CliqueDesc d{};
  d.body = U0.bb;
  d.shp = S.shp0;
  if (left) {
    d.gA = S.rec[0].gj;
    d.sA = S.rec[0].sa;
    d.rA = S.rec[0].r;
  }
  d.gB = U0.gj;
  d.sB = U0.sb;
  d.rB = U0.r;
  CliqueLoad c = clique_issue(a, d, ln);
  if (d.body >= 0) {
    clique_form(a, S, c, d, ln);
    team_sync();
    const int rA = d.rA;
    if (ln < 15) {
      int p, q;
      unpack15(ln, p, q);
      if (p < U0.r) D[ln] += S.K[px(rA + p, rA + q)];
    }
    if (ln < U0.r) y[ln] += S.yl[rA + ln];
    for (int e = ln; e < 25; e += PT) {  // F[p][q]: left rows p x our rows q
      const int p = e / 5, q = e % 5;
      if (p < rA && q < U0.r) F[e] = S.K[px(rA + q, p)];
    }
  }
  // step 0's clique
  auto desc = [&](int i) {  // the body after unit u0 + i, with that unit and the next
    CliqueDesc q{};
    const PathUnitF &U = S.rec[i + 1];
    q.body = U.ba;
    q.shp = S.shb[i + 1];
    q.gA = U.gj;
    q.sA = U.sa;
    q.rA = U.r;
    if (i + 1 < t) {
      const PathUnitF &Un = S.rec[i + 2];
      q.gB = Un.gj;
      q.sB = Un.sb;
      q.rB = Un.r;
    }
    return q;
  };
  d = desc(0);
  c = clique_issue(a, d, ln);
  team_sync();
  for (int i = 0; i < t; ++i) {
    const bool sep = i == t - 1;
    const PathUnitF U = S.rec[i + 1];
    const int rn = d.rB;
    const double cv = ln < U.r ? unit_c(a, U.gj, ln) : 0.0;
    if (d.body >= 0) clique_form(a, S, c, d, ln);
    // the next step's loads, in flight while this unit is eliminated
    CliqueDesc dn{};
    dn.body = -1;
    if (!sep) dn = desc(i + 1);
    const CliqueLoad cn = clique_issue(a, dn, ln);
    team_sync();
    // complete this unit's block from the body after it; the next unit's
    // block and the coupling from the same body
    const bool hb = d.body >= 0;
    if (ln < 15) {
      int p, q;
      unpack15(ln, p, q);
      if (hb && p < U.r) D[ln] += S.K[px(p, q)];
      double v = p == q ? (p < rn ? 0.0 : 1.0) : 0.0;
      if (hb && p < rn) v += S.K[px(U.r + p, U.r + q)];
      Dn[ln] = v;
    }
    if (ln < 5) {
      y[ln] += (hb && ln < U.r ? S.yl[ln] : 0.0) + cv;
      yn[ln] = hb && ln < rn ? S.yl[U.r + ln] : 0.0;
    }
    for (int e = ln; e < 25; e += PT) {  // E[p][q]: our rows p x the next unit's rows q
      const int p = e / 5, q = e % 5;
      S.E[e] = hb && p < U.r && q < rn ? S.K[px(U.r + q, p)] : 0.0;
    }
    team_sync();
    if (sep) break;
    // eliminate this unit: every lane factors the 5x5 block (cheap), lanes
    // 0-4 form the columns of G, 5-9 those of W, 10 z, 11 keeps L
    {
      double Lr[15];
#pragma unroll
      for (int k = 0; k < 15; ++k) Lr[k] = D[k];
      chol5(Lr, a.status);
      double col[5];
#pragma unroll
      for (int q = 0; q < 5; ++q)
        col[q] = ln < 5 ? F[5 * ln + q] : (ln < 10 ? S.E[5 * q + (ln - 5)] : y[q]);
      fsub5(Lr, col);
      if (ln < 5) {
#pragma unroll
        for (int q = 0; q < 5; ++q) S.fr[PF_G + 5 * q + ln] = col[q];
      } else if (ln < 10) {
#pragma unroll
        for (int q = 0; q < 5; ++q) S.fr[PF_W + 5 * q + (ln - 5)] = col[q];
      } else if (ln == 10) {
#pragma unroll
        for (int q = 0; q < 5; ++q) S.fr[PF_Z + q] = col[q];
      } else if (ln == 11) {
#pragma unroll
        for (int k = 0; k < 15; ++k) S.fr[PF_L + k] = Lr[k];
      }
    }
    team_sync();
    for (int e = ln; e < PATH_FREC; e += PT) fac[(int64_t)i * PATH_FREC + e] = S.fr[e];
    // updates, 65 outputs over the team: dD += G^T G, Dn -= W^T W,
    // F = -G^T W, yn -= W^T z, dy += G^T z
    const double *G = S.fr + PF_G, *W = S.fr + PF_W, *z = S.fr + PF_Z;
    for (int o = ln; o < 65; o += PT) {
      if (o < 30) {
        int p, q;
        unpack15(o < 15 ? o : o - 15, p, q);
        const double *X = o < 15 ? G : W;
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < 5; ++k) v += X[5 * k + p] * X[5 * k + q];
        if (o < 15) dD[o] += v;
        else Dn[o - 15] -= v;
      } else if (o < 55) {
        const int p = (o - 30) / 5, q = (o - 30) % 5;
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < 5; ++k) v += G[5 * k + p] * W[5 * k + q];
        F[o - 30] = -v;
      } else {
        const int p = o < 60 ? o - 55 : o - 60;
        const double *X = o < 60 ? W : G;
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < 5; ++k) v += X[5 * k + p] * z[k];
        if (o < 60) yn[p] -= v;
        else dy[p] += v;
      }
    }
    team_sync();
    // the next unit becomes the current one
    double *tD = D, *ty = y;
    D = Dn;
    y = yn;
    Dn = tD;
    yn = ty;
    d = dn;
    c = cn;
  }
  // the separator
  const int64_t kn = P.unit_off[1] + sg.k;
  if (top) {
    if (ln == 0) {
      double Lr[15], x[5];
#pragma unroll
      for (int k = 0; k < 15; ++k) Lr[k] = D[k];
#pragma unroll
      for (int k = 0; k < 5; ++k) x[k] = y[k];
      chol5(Lr, a.status);
      fsub5(Lr, x);
      bsub5(Lr, x);
#pragma unroll
      for (int k = 0; k < 5; ++k) P.lam[5 * kn + k] = x[k];
    }
    return;
  }
  double *Uk = P.unit + PATH_UREC * kn;
  for (int e = ln; e < 15; e += PT) Uk[PU_D + e] = D[e];
  if (ln < 5) Uk[PU_Y + ln] = y[ln];
  for (int e = ln; e < 25; e += PT) Uk[PU_F + e] = F[e];
  if (left)
    for (int e = PU_DD + ln; e < PATH_UREC; e += PT) Uk[e - PATH_UREC] = S.st[e];
  if (last)
    for (int e = PU_DD + ln; e < PATH_UREC; e += PT) Uk[e] = 0.0;
}

// levels >= 1: one lane per segment over the stored unit records
__global__ __launch_bounds__(PW) void path_fwd_kernel(TreeArgs a, PathPlan P, int lvl) {
  const int nseg = P.seg_off[lvl + 1] - P.seg_off[lvl];
  const int g = blockIdx.x * PW + threadIdx.x;
  const StepGate gate = step_gate(a.status);
  if (g >= nseg) return;
  const PathSeg S = P.seg[P.seg_off[lvl] + g];
  if (gate.skip()) return;
  const bool left = S.flags & 1, last = (S.flags & 2) != 0, top = (S.flags & 4) != 0;
  double *fac = P.fac + P.fac_off[lvl];
  const int64_t fstride = nseg;  // factor element e of step i: fac[(i * PATH_FREC + e) * nseg + g]
  double D[15], y[5], F[25], dD[15], dy[5];
#pragma unroll
  for (int i = 0; i < 15; ++i) dD[i] = 0.0;
#pragma unroll
  for (int i = 0; i < 5; ++i) dy[i] = 0.0;
  {
    const double *Ur = P.unit + PATH_UREC * (P.unit_off[lvl] + S.u0);
#pragma unroll
    for (int i = 0; i < 15; ++i) D[i] = Ur[PU_D + i] - Ur[PU_DD + i];
#pragma unroll
    for (int i = 0; i < 5; ++i) y[i] = Ur[PU_Y + i] - Ur[PU_DY + i];
#pragma unroll
    for (int i = 0; i < 25; ++i) F[i] = left ? Ur[PU_F + i] : 0.0;
  }
  for (int i = 0; i + 1 < S.t; ++i) {
    const int u = S.u0 + i;
    double E[25], Dn[15], yn[5];
    const double *Un = P.unit + PATH_UREC * (P.unit_off[lvl] + u + 1);
#pragma unroll
    for (int k = 0; k < 25; ++k) E[k] = Un[PU_F + k];
#pragma unroll
    for (int k = 0; k < 15; ++k) Dn[k] = Un[PU_D + k] - Un[PU_DD + k];
#pragma unroll
    for (int k = 0; k < 5; ++k) yn[k] = Un[PU_Y + k] - Un[PU_DY + k];
    chol5(D, a.status);
    fsub5(D, y);
    double G[25];
#pragma unroll
    for (int c = 0; c < 5; ++c) {  // G = L^{-1} F^T: column c is L^{-1} times row c of F
      double col[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) col[q] = F[5 * c + q];
      fsub5(D, col);
#pragma unroll
      for (int q = 0; q < 5; ++q) G[5 * q + c] = col[q];
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) {  // W = L^{-1} E, in place
      double col[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) col[q] = E[5 * q + c];
      fsub5(D, col);
#pragma unroll
      for (int q = 0; q < 5; ++q) E[5 * q + c] = col[q];
    }
    double *f = fac + (int64_t)i * PATH_FREC * fstride + g;
#pragma unroll
    for (int k = 0; k < 15; ++k) f[(PF_L + k) * fstride] = D[k];
#pragma unroll
    for (int k = 0; k < 5; ++k) f[(PF_Z + k) * fstride] = y[k];
#pragma unroll
    for (int k = 0; k < 25; ++k) f[(PF_W + k) * fstride] = E[k];
#pragma unroll
    for (int k = 0; k < 25; ++k) f[(PF_G + k) * fstride] = G[k];
#pragma unroll
    for (int p = 0; p < 5; ++p) {
#pragma unroll
      for (int q = 0; q <= p; ++q) {
        double sg = 0.0, sw = 0.0;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          sg += G[5 * k + p] * G[5 * k + q];
          sw += E[5 * k + p] * E[5 * k + q];
        }
        dD[px(p, q)] += sg;
        Dn[px(p, q)] -= sw;
      }
      double tg = 0.0, tw = 0.0;
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        tg += G[5 * k + p] * y[k];
        tw += E[5 * k + p] * y[k];
      }
      dy[p] += tg;
      yn[p] -= tw;
    }
#pragma unroll
    for (int p = 0; p < 5; ++p)
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < 5; ++k) v += G[5 * k + p] * E[5 * k + q];
        F[5 * p + q] = -v;
      }
#pragma unroll
    for (int k = 0; k < 15; ++k) D[k] = Dn[k];
#pragma unroll
    for (int k = 0; k < 5; ++k) y[k] = yn[k];
  }
  const int64_t kn = P.unit_off[lvl + 1] + S.k;
  if (top) {
    chol5(D, a.status);
    fsub5(D, y);
    bsub5(D, y);
    double *lam = P.lam + 5 * kn;
#pragma unroll
    for (int p = 0; p < 5; ++p) lam[p] = y[p];
    return;
  }
  double *Uk = P.unit + PATH_UREC * kn;
#pragma unroll
  for (int k = 0; k < 15; ++k) Uk[PU_D + k] = D[k];
#pragma unroll
  for (int k = 0; k < 5; ++k) Uk[PU_Y + k] = y[k];
#pragma unroll
  for (int k = 0; k < 25; ++k) Uk[PU_F + k] = F[k];
  if (left) {
    double *Ul = Uk - PATH_UREC;
#pragma unroll
    for (int k = 0; k < 15; ++k) Ul[PU_DD + k] = dD[k];
#pragma unroll
    for (int k = 0; k < 5; ++k) Ul[PU_DY + k] = dy[k];
  }
  if (last) {
#pragma unroll
    for (int k = 0; k < 15; ++k) Uk[PU_DD + k] = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) Uk[PU_DY + k] = 0.0;
  }
}

// back-substitution of level 0: a team per segment loads each record of
// factors (contiguous) into LDS, the next one in flight meanwhile, and every
// lane solves the 5x5 step
__global__ __launch_bounds__(PW) void path_back0_kernel(TreeArgs a, PathPlan P) {
  __shared__ double recs[PTEAMS][PATH_FREC];
  const int tm = threadIdx.x / PT, ln = threadIdx.x % PT;
  double *R = recs[tm];
  const int nseg = P.seg_off[1] - P.seg_off[0];
  const int g = blockIdx.x * PTEAMS + tm;
  const StepGate gate = step_gate(a.status);
  if (g >= nseg) return;  // whole teams only
  const PathSeg S = P.seg[g];
  if (gate.skip()) return;
  const bool left = S.flags & 1;
  const double *fac = P.fac + P.fac_off[0] + (int64_t)g * (P.T0 - 1) * PATH_FREC;
  const double *lnx = P.lam + 5 * (P.unit_off[1] + S.k);
  double x[5], xl[5];
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    x[p] = lnx[p];
    xl[p] = 0.0;
  }
  if (left) {
#pragma unroll
    for (int p = 0; p < 5; ++p) xl[p] = lnx[p - 5];
  }
  // lane p < rows writes multiplier row p of unit u
#define PATH_PUT(u, v)                                                  \
  {                                                                     \
    const PathUnitF U_ = P.uf[u];                                       \
    double w_ = v[0];                                                   \
    _Pragma("unroll") for (int p = 1; p < 5; ++p) w_ = ln == p ? v[p] : w_; \
    if (ln < U_.r) a.glam[5 * (int64_t)U_.gj + ln] = w_;                \
  }
  PATH_PUT(S.u0 + S.t - 1, x);
  double r0, r1, r2, r3, r4;  // the next record, five elements per lane
#define PATH_FETCH(i)                                                                      \
  {                                                                                        \
    const double *f_ = fac + (int64_t)(i) * PATH_FREC + ln;                                \
    const bool ok_ = (i) >= 0;                                                             \
    r0 = ok_ ? f_[0] : 0.0;                                                                \
    r1 = ok_ ? f_[PT] : 0.0;                                                               \
    r2 = ok_ ? f_[2 * PT] : 0.0;                                                           \
    r3 = ok_ ? f_[3 * PT] : 0.0;                                                           \
    r4 = ok_ && ln + 4 * PT < PATH_FREC ? f_[4 * PT] : 0.0;                                \
  }
  PATH_FETCH(S.t - 2);
  for (int i = S.t - 2; i >= 0; --i) {
    R[ln] = r0;
    R[ln + PT] = r1;
    R[ln + 2 * PT] = r2;
    R[ln + 3 * PT] = r3;
    if (ln + 4 * PT < PATH_FREC) R[ln + 4 * PT] = r4;
    team_sync();
    PATH_FETCH(i - 1);
    double L[15], v[5];
#pragma unroll
    for (int k = 0; k < 15; ++k) L[k] = R[PF_L + k];
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      double s = R[PF_Z + p];
#pragma unroll
      for (int q = 0; q < 5; ++q) s -= R[PF_W + 5 * p + q] * x[q] + R[PF_G + 5 * p + q] * xl[q];
      v[p] = s;
    }
    bsub5(L, v);
    PATH_PUT(S.u0 + i, v);
#pragma unroll
    for (int p = 0; p < 5; ++p) x[p] = v[p];
    team_sync();
  }
#undef PATH_PUT
#undef PATH_FETCH
}

// back-substitution of a level >= 1, one lane per segment (factors
// interleaved across the segments)
__global__ __launch_bounds__(PW) void path_back_kernel(TreeArgs a, PathPlan P, int lvl) {
  const int nseg = P.seg_off[lvl + 1] - P.seg_off[lvl];
  const int g = blockIdx.x * PW + threadIdx.x;
  const StepGate gate = step_gate(a.status);
  if (g >= nseg) return;
  const PathSeg S = P.seg[P.seg_off[lvl] + g];
  if (gate.skip()) return;
  const bool left = S.flags & 1;
  const double *fac = P.fac + P.fac_off[lvl] + g;
  const int64_t fe = nseg, fi = PATH_FREC * (int64_t)nseg;  // between a record's elements, records
  const double *lnx = P.lam + 5 * (P.unit_off[lvl + 1] + S.k);
  double x[5], xl[5];
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    x[p] = lnx[p];
    xl[p] = 0.0;
  }
  if (left) {
#pragma unroll
    for (int p = 0; p < 5; ++p) xl[p] = lnx[p - 5];
  }
  double *out = P.lam + 5 * (P.unit_off[lvl] + S.u0);
#pragma unroll
  for (int p = 0; p < 5; ++p) out[5 * (S.t - 1) + p] = x[p];
  for (int i = S.t - 2; i >= 0; --i) {
    const double *f = fac + i * fi;
    double L[15], v[5];
#pragma unroll
    for (int k = 0; k < 15; ++k) L[k] = f[(PF_L + k) * fe];
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      double s = f[(PF_Z + p) * fe];
#pragma unroll
      for (int q = 0; q < 5; ++q) s -= f[(PF_W + 5 * p + q) * fe] * x[q] + f[(PF_G + 5 * p + q) * fe] * xl[q];
      v[p] = s;
    }
    bsub5(L, v);
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      out[5 * i + p] = v[p];
      x[p] = v[p];
    }
  }
}

}  // namespace

void launch_path(const TreeArgs &a, const PathPlan &P, hipStream_t s) {
  for (int l = 0; l < P.nlevel; ++l) {
    const int n = P.seg_off[l + 1] - P.seg_off[l];
    if (n <= 0) continue;
    if (l == 0)
      hipLaunchKernelGGL(path_fwd0_kernel, dim3((n + PTEAMS - 1) / PTEAMS), dim3(PW), 0, s, a, P);
    else
      hipLaunchKernelGGL(path_fwd_kernel, dim3((n + PW - 1) / PW), dim3(PW), 0, s, a, P, l);
  }
  for (int l = P.nlevel - 1; l >= 0; --l) {
    const int n = P.seg_off[l + 1] - P.seg_off[l];
    if (n <= 0) continue;
    if (l == 0)
      hipLaunchKernelGGL(path_back0_kernel, dim3((n + PTEAMS - 1) / PTEAMS), dim3(PW), 0, s, a, P);
    else
      hipLaunchKernelGGL(path_back_kernel, dim3((n + PW - 1) / PW), dim3(PW), 0, s, a, P, l);
  }
}

}  // namespace mabd
