// Dual solve of path components (Sec. 5.3: a tree whose bodies each carry
// at most two joints).  The dual S = G H^{-1} G^T of a path is block
// tridiagonal over its joints in path order; its blocks are read from the
// clique matrices K0 = L Hbar^{-1} L^T and right-hand sides y0 = L u + C that
// the tree pre-pass forms per body (the two diagonal contributions of a
// joint come from its two bodies, the coupling of consecutive joints from the
// body they share).  One lane owns a segment of consecutive units and
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
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "generic.hpp"

namespace mabd {

namespace {

constexpr int PW = 64;  // threads per workgroup (one wave)

__device__ __forceinline__ constexpr int px(int p, int q) { return p * (p + 1) / 2 + q; }

// D (packed lower) = L L^T in place, with the reciprocals of the pivots in
// place of L's diagonal (the solves below multiply by them); a non-positive
// pivot raises SINGULAR
__device__ __forceinline__ void chol5(double D[15], uint32_t *status) {
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
__device__ __forceinline__ void fsub5(const double L[15], double x[5]) {
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    double v = x[p];
#pragma unroll
    for (int k = 0; k < p; ++k) v -= L[px(p, k)] * x[k];
    x[p] = v * L[px(p, p)];
  }
}
// x = L^{-T} x
__device__ __forceinline__ void bsub5(const double L[15], double x[5]) {
#pragma unroll
  for (int p = 4; p >= 0; --p) {
    double v = x[p];
#pragma unroll
    for (int k = p + 1; k < 5; ++k) v -= L[px(k, p)] * x[k];
    x[p] = v * L[px(p, p)];
  }
}

// D = identity on the rows past r, zero elsewhere
__device__ __forceinline__ void pad_init(double D[15], double y[5], int r) {
#pragma unroll
  for (int p = 0; p < 5; ++p) {
#pragma unroll
    for (int q = 0; q < p; ++q) D[px(p, q)] = 0.0;
    D[px(p, p)] = p < r ? 0.0 : 1.0;
    y[p] = 0.0;
  }
}
// add the diagonal block of rows [o, o + r) of a clique (lower triangle, ld)
// and its right-hand side
__device__ __forceinline__ void add_diag(const double *K, int ld, int o, int r, double D[15], double y[5]) {
  double v[15], w[5];
#pragma unroll
  for (int p = 0; p < 5; ++p) {
#pragma unroll
    for (int q = 0; q <= p; ++q) v[px(p, q)] = p < r ? K[(o + p) * ld + o + q] : 0.0;
    w[p] = p < r ? K[ld * ld + o + p] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < 15; ++i) D[i] += v[i];
#pragma unroll
  for (int p = 0; p < 5; ++p) y[p] += w[p];
}
// X[p][q] = clique entry (rows os + p, rows on + q), p < rs, q < rn; zero padding
__device__ __forceinline__ void load_cross(const double *K, int ld, int os, int rs, int on, int rn, double X[25]) {
#pragma unroll
  for (int p = 0; p < 5; ++p)
#pragma unroll
    for (int q = 0; q < 5; ++q)
      X[5 * p + q] = (p < rs && q < rn) ? (os > on ? K[(os + p) * ld + on + q] : K[(on + q) * ld + os + p]) : 0.0;
}

__device__ __forceinline__ int level_rows(const PathPlan &P, int lvl, int u) {
  return lvl == 0 ? P.u0[u].r : P.rows[P.unit_off[lvl] + u];
}

template <bool L0>
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
  int r = level_rows(P, lvl, S.u0);
#pragma unroll
  for (int i = 0; i < 15; ++i) dD[i] = 0.0;
#pragma unroll
  for (int i = 0; i < 5; ++i) dy[i] = 0.0;
  if (L0) {
    const PathUnit0 U = P.u0[S.u0];
    pad_init(D, y, r);
    if (U.fb >= 0) {
      const double *K = a.fac + U.fb;
      add_diag(K, U.ldb, U.ob, r, D, y);
    }
    if (left && U.fb >= 0 && U.obp >= 0) {
      const int rl = P.u0[S.u0 - 1].r;
      load_cross(a.fac + U.fb, U.ldb, U.obp, rl, U.ob, r, F);  // left rows x our rows
    } else {
#pragma unroll
      for (int i = 0; i < 25; ++i) F[i] = 0.0;
    }
  } else {
    const double *Ur = P.unit + PATH_UREC * (P.unit_off[lvl] + S.u0);
#pragma unroll
    for (int i = 0; i < 15; ++i) D[i] = Ur[PU_D + i] - Ur[PU_DD + i];
#pragma unroll
    for (int i = 0; i < 5; ++i) y[i] = Ur[PU_Y + i] - Ur[PU_DY + i];
#pragma unroll
    for (int i = 0; i < 25; ++i) F[i] = left ? Ur[PU_F + i] : 0.0;
  }
  for (int i = 0; i < S.t; ++i) {
    const int u = S.u0 + i;
    const bool sep = i == S.t - 1;
    double E[25], Dn[15], yn[5];
    int rn = 0;
    if (L0) {
      const PathUnit0 U = P.u0[u];
      if (U.fa >= 0) {
        const double *K = a.fac + U.fa;
        add_diag(K, U.lda, U.oa, r, D, y);
        if (!sep) {
          rn = P.u0[u + 1].r;
          load_cross(K, U.lda, U.oa, r, U.oan, rn, E);
          pad_init(Dn, yn, rn);
          add_diag(K, U.lda, U.oan, rn, Dn, yn);
        }
      }
    } else if (!sep) {
      const double *Un = P.unit + PATH_UREC * (P.unit_off[lvl] + u + 1);
      rn = P.rows[P.unit_off[lvl] + u + 1];
#pragma unroll
      for (int k = 0; k < 25; ++k) E[k] = Un[PU_F + k];
#pragma unroll
      for (int k = 0; k < 15; ++k) Dn[k] = Un[PU_D + k] - Un[PU_DD + k];
#pragma unroll
      for (int k = 0; k < 5; ++k) yn[k] = Un[PU_Y + k] - Un[PU_DY + k];
    }
    if (sep) break;
    // eliminate unit i
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
    // the left separator's block and right-hand side, the next unit's, and
    // the next unit's coupling with the left separator
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
    r = rn;
  }
  // the separator
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

template <bool L0>
__global__ __launch_bounds__(PW) void path_back_kernel(TreeArgs a, PathPlan P, int lvl) {
  const int nseg = P.seg_off[lvl + 1] - P.seg_off[lvl];
  const int g = blockIdx.x * PW + threadIdx.x;
  const StepGate gate = step_gate(a.status);
  if (g >= nseg) return;
  const PathSeg S = P.seg[P.seg_off[lvl] + g];
  if (gate.skip()) return;
  const bool left = S.flags & 1;
  const double *fac = P.fac + P.fac_off[lvl];
  const int64_t fstride = nseg;
  const double *ln = P.lam + 5 * (P.unit_off[lvl + 1] + S.k);
  double x[5], xl[5];
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    x[p] = ln[p];
    xl[p] = 0.0;
  }
  if (left) {
#pragma unroll
    for (int p = 0; p < 5; ++p) xl[p] = ln[p - 5];
  }
  auto put = [&](int u, const double *v) {
    if (L0) {
      const PathUnit0 U = P.u0[u];
      double *o = a.glam + 5 * (int64_t)U.gj;
#pragma unroll
      for (int p = 0; p < 5; ++p)
        if (p < U.r) o[p] = v[p];
    } else {
      double *o = P.lam + 5 * (P.unit_off[lvl] + u);
#pragma unroll
      for (int p = 0; p < 5; ++p) o[p] = v[p];
    }
  };
  put(S.u0 + S.t - 1, x);
  for (int i = S.t - 2; i >= 0; --i) {
    const double *f = fac + (int64_t)i * PATH_FREC * fstride + g;
    double L[15], v[5];
#pragma unroll
    for (int k = 0; k < 15; ++k) L[k] = f[(PF_L + k) * fstride];
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      double s = f[(PF_Z + p) * fstride];
#pragma unroll
      for (int q = 0; q < 5; ++q) s -= f[(PF_W + 5 * p + q) * fstride] * x[q] + f[(PF_G + 5 * p + q) * fstride] * xl[q];
      v[p] = s;
    }
    bsub5(L, v);
    put(S.u0 + i, v);
#pragma unroll
    for (int p = 0; p < 5; ++p) x[p] = v[p];
  }
}

}  // namespace

void launch_path(const TreeArgs &a, const PathPlan &P, hipStream_t s) {
  for (int l = 0; l < P.nlevel; ++l) {
    const int n = P.seg_off[l + 1] - P.seg_off[l];
    if (n <= 0) continue;
    if (l == 0)
      hipLaunchKernelGGL(path_fwd_kernel<true>, dim3((n + PW - 1) / PW), dim3(PW), 0, s, a, P, l);
    else
      hipLaunchKernelGGL(path_fwd_kernel<false>, dim3((n + PW - 1) / PW), dim3(PW), 0, s, a, P, l);
  }
  for (int l = P.nlevel - 1; l >= 0; --l) {
    const int n = P.seg_off[l + 1] - P.seg_off[l];
    if (n <= 0) continue;
    if (l == 0)
      hipLaunchKernelGGL(path_back_kernel<true>, dim3((n + PW - 1) / PW), dim3(PW), 0, s, a, P, l);
    else
      hipLaunchKernelGGL(path_back_kernel<false>, dim3((n + PW - 1) / PW), dim3(PW), 0, s, a, P, l);
  }
}

}  // namespace mabd
