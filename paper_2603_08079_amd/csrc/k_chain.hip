// Chain dual solve for ball-jointed chains (Sec. 5.2, Eq. chain-btd),
// fused with the per-body co-rotated solve (Sec. 3.4) and the primal
// back-projection (Eq. recover-dq-explicit).
//
// The dual system of a chain is block tridiagonal with 3x3 blocks.  Instead
// of the serial block Thomas sweep the rows are cut into tiles of T + 1 rows
// (T = workgroup size - 2, or PACK_T for packed tiles) that share their
// first/last (interface) rows with the neighbouring tiles.  One workgroup per
// tile
//   A) computes the polar rotation, force and local solve of its bodies
//      (one body per thread, coalesced SoA loads) and the rotated constant
//      blocks R W(p, p') R^T with W = J(p) Hbar^{-1} J(p')^T;
//   B) assembles its rows D, U, b (Eqs. chain-Schur-blocks, chain-b, with +C);
//   C) runs block cyclic reduction on the tile interior (log2 levels, one
//      row per thread, neighbours exchanged through LDS), which leaves the
//      Schur complement on the two interface rows.  Packed tiles run the
//      first two levels here and the rest in chain_pack_kernel, four tiles
//      to a wave.
// The interface rows form a block-tridiagonal system again, reduced in groups
// of 256 rows (chain_group_kernel) whose end rows form the top system (solved
// by the last group to finish, or by chain_global_kernel when it exceeds one
// workgroup).  The apply pass repeats A-C, back-substitutes the tile, and
// writes lambda and the new state.  Recomputing A-C costs one more read of
// q, qdot but moves no dense elimination factors through HBM (packed tiles
// read only the factors of the rows eliminated four tiles to a wave).
#include <cfloat>
#include <type_traits>

#include "common.hpp"
#include "dmath.hpp"

namespace mabd {



DEV void sym_from_full(const double *F, double *S6) {
  S6[0] = F[0];
  S6[1] = 0.5 * (F[1] + F[3]);
  S6[2] = 0.5 * (F[2] + F[6]);
  S6[3] = F[4];
  S6[4] = 0.5 * (F[5] + F[7]);
  S6[5] = F[8];
}

DEV void full_from_sym(const double *S6, double *F) {
  F[0] = S6[0]; F[1] = S6[1]; F[2] = S6[2];
  F[3] = S6[1]; F[4] = S6[3]; F[5] = S6[4];
  F[6] = S6[2]; F[7] = S6[4]; F[8] = S6[5];
}

// LDS layout (doubles): S_N arrays of CHAIN_THREADS entries
enum { S_WBB = 0, S_VB = 6, S_CB = 9, S_TB = 12, S_WAB = 15, S_N = 27 };
// cyclic reduction: what an eliminated row hands to its left neighbour
// (dD 6, db 3, new coupling 9) and to its right one (dD 6, db 3);
// back-substitution: x (3).  S_PL / S_PU / S_PB name the same slots for the
// two-row exchange of the top solve.
enum { S_DL = 0, S_BL = 6, S_UN = 9, S_DR = 18, S_BR = 24, S_X = 21 };
enum { S_PL = 0, S_PU = 9, S_PB = 18 };

// Block cyclic reduction of the rows 1..T-1 of a tile onto its interface
// rows 0 and T.  Row li (held by one thread, `row_active`) couples to its
// current left neighbour through L and to its right one through U; the
// system is symmetric, so a row's L is the transpose of its left
// neighbour's U.  At level d the rows li = d mod 2d are eliminated.  Each
// keeps (PL, PU, Pb) = D^{-1} (L, U, b) for the back-substitution and, since
// the left neighbour's coupling to it is L^T and the right one's is U^T,
// computes every Schur update itself:
//   left:  D -= L^T PL,  b -= L^T Pb,  U <- -L^T PU
//   right: D -= U^T PU,  b -= U^T Pb,  L <- (-L^T PU)^T
// The surviving rows then only add what their eliminated neighbours
// published, so the costly branch runs on one set of lanes per level.
// Levels d < dend run; dend must be the same in the whole workgroup (it
// brackets barriers), and a level with d >= T changes nothing, so rows of
// systems of different sizes can share one call.
template <int NT>
DEV void tile_cr_forward(double *lds, bool row_active, int li, int T, int dend, double *L,
                         double *D, double *U, double *b, double *PL, double *PU, double *Pb,
                         int &elim_d, uint32_t *status, int step) {
  for (int d = 1; d < dend; d *= 2) {  // d is a power of two: masks for mod and div
    const bool active = row_active && ((li & (d - 1)) == 0 || li == T);
    const bool elim = active && li < T && ((li & (2 * d - 1)) == d);
    if (elim) {
      double Df[9], Di[9];
      full_from_sym(D, Df);
      if (!spd3_inv(Df, Di)) {
        raise_flag(status, FLAG_SINGULAR, step);
#pragma unroll
        for (int i = 0; i < 9; ++i) Di[i] = 0.0;
      }
      mat3_mul(Di, L, PL);
      mat3_mul(Di, U, PU);
      mat3_vec(Di, b, Pb);
      elim_d = d;
      double M[9], v[3];
      // left neighbour
      mat3_mul_at(L, PL, M);
      lds[(S_DL + 0) * NT + li] = M[0];
      lds[(S_DL + 1) * NT + li] = 0.5 * (M[1] + M[3]);
      lds[(S_DL + 2) * NT + li] = 0.5 * (M[2] + M[6]);
      lds[(S_DL + 3) * NT + li] = M[4];
      lds[(S_DL + 4) * NT + li] = 0.5 * (M[5] + M[7]);
      lds[(S_DL + 5) * NT + li] = M[8];
      mat3t_vec(L, Pb, v);
#pragma unroll
      for (int i = 0; i < 3; ++i) lds[(S_BL + i) * NT + li] = v[i];
      mat3_mul_at(L, PU, M);
#pragma unroll
      for (int i = 0; i < 9; ++i) lds[(S_UN + i) * NT + li] = -M[i];
      // right neighbour
      mat3_mul_at(U, PU, M);
      lds[(S_DR + 0) * NT + li] = M[0];
      lds[(S_DR + 1) * NT + li] = 0.5 * (M[1] + M[3]);
      lds[(S_DR + 2) * NT + li] = 0.5 * (M[2] + M[6]);
      lds[(S_DR + 3) * NT + li] = M[4];
      lds[(S_DR + 4) * NT + li] = 0.5 * (M[5] + M[7]);
      lds[(S_DR + 5) * NT + li] = M[8];
      mat3t_vec(U, Pb, v);
#pragma unroll
      for (int i = 0; i < 3; ++i) lds[(S_BR + i) * NT + li] = v[i];
    }
    __syncthreads();
    if (active && !elim) {
      const int e = li + d;
      if (li != T && e < T) {
#pragma unroll
        for (int i = 0; i < 6; ++i) D[i] -= lds[(S_DL + i) * NT + e];
#pragma unroll
        for (int i = 0; i < 3; ++i) b[i] -= lds[(S_BL + i) * NT + e];
#pragma unroll
        for (int i = 0; i < 9; ++i) U[i] = lds[(S_UN + i) * NT + e];
      }
      const int lf = li == T ? ((T - 1) & ~(d - 1)) : li - d;
      if (li > 0 && lf > 0 && ((lf & (2 * d - 1)) == d)) {
#pragma unroll
        for (int i = 0; i < 6; ++i) D[i] -= lds[(S_DR + i) * NT + lf];
#pragma unroll
        for (int i = 0; i < 3; ++i) b[i] -= lds[(S_BR + i) * NT + lf];
#pragma unroll
        for (int r2 = 0; r2 < 3; ++r2)
#pragma unroll
          for (int c2 = 0; c2 < 3; ++c2) L[3 * r2 + c2] = lds[(S_UN + 3 * c2 + r2) * NT + lf];
      }
    }
    __syncthreads();
  }
}

// Back-substitution of tile_cr_forward: x of rows 0 and T must already be in
// LDS (S_X) and visible; on return every row's x is there.
template <int NT>
DEV void tile_cr_backward(double *lds, bool row_active, int li, int T, int elim_d,
                          const double *PL, const double *PU, const double *Pb) {
  int dmax = 0;
  for (int d = 1; d < T; d *= 2) dmax = d;
  for (int d = dmax; d >= 1; d /= 2) {
    if (row_active && elim_d == d) {
      const int lf = li - d;
      const int rt = li + d < T ? li + d : T;
      double xl[3], xr[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        xl[i] = lds[(S_X + i) * NT + lf];
        xr[i] = lds[(S_X + i) * NT + rt];
      }
      double t1[3], t2[3];
      mat3_vec(PL, xl, t1);
      mat3_vec(PU, xr, t2);
#pragma unroll
      for (int i = 0; i < 3; ++i) lds[(S_X + i) * NT + li] = Pb[i] - t1[i] - t2[i];
    }
    __syncthreads();
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Neighbouring tiles share a row and their body ranges straddle cache
// lines, so each XCD is given a contiguous range of tiles: the shared lines
// are then fetched once, into one L2.  Returns -1 for the padding blocks of
// the last range.
DEV int xcd_tile(int ntiles) {
  const int per = (ntiles + 7) / 8;
  const int ti = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  return ti < ntiles ? ti : -1;
}
inline unsigned xcd_grid(int ntiles) { return 8u * (unsigned)((ntiles + 7) / 8); }
// The same with ranges of a multiple of four tiles, so that the four tiles of
// a packed group share an XCD (and its L2).
DEV int xcd_tile4(int ntiles) {
  const int per = 4 * ((ntiles + 31) / 32);
  const int ti = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  return ti < ntiles ? ti : -1;
}
inline unsigned xcd_grid4(int ntiles) { return 32u * (unsigned)((ntiles + 31) / 32); }

// Packed tiles.  A tile of T <= PACK_T rows runs the first two levels of its
// cyclic reduction alone; its surviving rows are li = 4j (li < T) and li = T,
// at most 16, numbered j = 0..T' with T' = ceil(T/4).  Levels d = 4, 8, 16,
// 32 of the tile eliminate exactly the rows that levels 1, 2, 4, 8 of the
// survivors' own cyclic reduction (rows j, T') eliminate, with the same
// neighbours, so the survivors of four tiles are reduced as four 16-row
// systems side by side in one wave (chain_pack_kernel, launched after the
// tiles: handing the survivors over inside one launch would need device-scope
// cache maintenance per workgroup).  That wave writes the tiles' Schur
// records and the factors (PL, PU, Pb) of the rows it eliminated; the apply
// pass reads those factors instead of repeating the four sparse levels.
DEV void pack_reduce_group(const ChainArgs &a, int grp, double *lds, StepGate gate, double ir0) {
  const int t = threadIdx.x;
  const int q = t >> 4, j = t & 15;
  const int nq = min(4, a.ntiles - 4 * grp);
  const int tq = 4 * grp + q;
  // every slot of a present tile is read together with the tile size (slots
  // past the tile's survivors hold stale values and are discarded below)
  int Tp = 0;
  double L[9], D[6], U[9], b[3];
  if (q < nq) {
    const double *sv = a.psv + (int64_t)grp * (PACK_SV * 64) + t;
    Tp = (a.tiles[tq].T + 3) >> 2;
#pragma unroll
    for (int i = 0; i < 6; ++i) D[i] = sv[i * 64];
#pragma unroll
    for (int i = 0; i < 3; ++i) b[i] = sv[(6 + i) * 64];
#pragma unroll
    for (int i = 0; i < 9; ++i) U[i] = sv[(9 + i) * 64];
    // left coupling = (U of the previous survivor)^T
    const double *svl = sv - (j > 0 ? 1 : 0);
#pragma unroll
    for (int r2 = 0; r2 < 3; ++r2)
#pragma unroll
      for (int c2 = 0; c2 < 3; ++c2) L[3 * r2 + c2] = svl[(9 + 3 * c2 + r2) * 64];
  }
  if (gate.skip() || ir0 != 0.0) return;  // uniform, tested with the reads in flight
  const bool act = q < nq && j <= Tp;
  if (!act || j == 0) {
#pragma unroll
    for (int i = 0; i < 9; ++i) L[i] = 0.0;
  }
  if (!act) {
#pragma unroll
    for (int i = 0; i < 9; ++i) U[i] = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) D[i] = 0.0;
    b[0] = b[1] = b[2] = 0.0;
  }
  double PL[9], PU[9], Pb[3];
  int elim_d = 0;
  tile_cr_forward<64>(lds + 16 * q, act, j, Tp, 16, L, D, U, b, PL, PU, Pb, elim_d, a.status,
                      a.step);
  if (act && (j == 0 || j == Tp)) {
    double *rec = a.tilerec + (int64_t)TILE_REC * tq;
    if (j == 0) {
#pragma unroll
      for (int i = 0; i < 6; ++i) rec[i] = D[i];
#pragma unroll
      for (int i = 0; i < 3; ++i) rec[6 + i] = b[i];
#pragma unroll
      for (int i = 0; i < 9; ++i) rec[18 + i] = U[i];
    } else {
#pragma unroll
      for (int i = 0; i < 6; ++i) rec[9 + i] = D[i];
#pragma unroll
      for (int i = 0; i < 3; ++i) rec[15 + i] = b[i];
    }
  }
  if (elim_d > 0) {
    double *cf = a.pcf + (int64_t)grp * (PACK_CF * 64) + t;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      cf[i * 64] = PL[i];
      cf[(9 + i) * 64] = PU[i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) cf[(18 + i) * 64] = Pb[i];
  }
}

// MODE 0: plain FP64.  MODE 1 (precision form 1, first solve): phase A in
// FP32, the factor in FP64, the increment goes to dq.  MODE 2 (form 1
// correction): the right-hand side is the FP64 KKT residual (rp, rd) of the
// current iterate and the increment is added to dq and lam; skipped once the
// residual check has converged.  WR: the bodies carry external wrenches (a
// separate instantiation, so that the plain path holds none of that code).
// PACK: packed 64-thread tiles (pack_reduce_group).
template <int MODE, bool APPLY, int NT, bool WR, bool PACK>
#ifndef MABD_TILE_WAVES_REDUCE
#define MABD_TILE_WAVES_REDUCE 2
#endif
#ifndef MABD_TILE_WAVES_APPLY
#define MABD_TILE_WAVES_APPLY 2
#endif
__global__ __launch_bounds__(NT, APPLY ? MABD_TILE_WAVES_APPLY : MABD_TILE_WAVES_REDUCE) void chain_tile_kernel(
    ChainArgs a) {
  using breal = typename std::conditional<MODE == 0, double, float>::type;
  // packed apply pass: the packed factors and the interface x are staged
  // after the exchange slots (read with phase A's loads, used after phase C)
  constexpr int STG = S_N * NT, STG_X = STG + PACK_CF * 16;
  __shared__ double lds[S_N * NT + (PACK && APPLY ? PACK_CF * 16 + 6 : 0)];
  // the step gate is read first and tested once phase A's reads are in
  // flight (nothing before the test writes global memory or raises a flag);
  // a correction sweep's convergence flag is tested as soon as it arrives
  const StepGate gate = step_gate(a.status);
  const double ir0 = MODE == 2 ? a.ir[0] : 0.0;
  // a correction sweep after convergence ends before reading its tile: the
  // flag's round trip costs the sweep that runs less than phase A's reads
  // cost every sweep that is skipped
  if constexpr (MODE == 2) {
    if (ir0 != 0.0) return;
  }
  static_assert(!PACK || NT == 64, "packed tiles are 64-thread tiles");
  const int ti = PACK ? xcd_tile4(a.ntiles) : xcd_tile(a.ntiles);
  if (ti < 0) return;
  const TileDesc td = a.tiles[ti];
  const ChainDesc cd = a.chains[td.chain];
  const int t = threadIdx.x;
  const int T = td.T;
  const int r = td.r0 + t - 1;           // this thread's row (if 1 <= t <= T+1)
  const int p = r + 1 - cd.hl;           // body between rows r and r+1
  const bool in_tile = t <= T + 1;
  const bool has_body = in_tile && p >= 0 && p < cd.nb;
  const bool has_a = in_tile && r >= 0 && r < cd.K;
  const bool has_b = in_tile && r + 1 < cd.K;
  const int64_t gra = (int64_t)cd.row0 + r;
  const int64_t grb = gra + 1;
  const int64_t bg = (int64_t)cd.body0 + p;

  // ---------------------------------------------------------------- phase A
  breal R[9], u[12];
  double pa[3] = {0, 0, 0}, pb[3] = {0, 0, 0};
  double sa = 1.0, sb = 1.0;
  double Waa[6] = {0, 0, 0, 0, 0, 0}, Wab[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double va[3] = {0, 0, 0}, ca[3] = {0, 0, 0}, ta[3] = {0, 0, 0};
  double Wbb[6] = {0, 0, 0, 0, 0, 0}, vb[3] = {0, 0, 0}, cb[3] = {0, 0, 0}, tb[3] = {0, 0, 0};
  const double *T_h = nullptr, *shc = nullptr;
  double sh[7], hv[HINV_STRIDE];  // shape constants and Hbar^{-1}, read during the polar
  // Every independent read of phase A is issued before the first use, with
  // indices clamped in bounds for lanes without the row or the body: the
  // kernel is bound by memory latency, and reads issued under branches or
  // after the polar would each cost a round trip of their own.
  double q[12];    // kept for the state update of the apply pass
  double qd0[12];  // qdot (MODE 2: the FP64 primal residual)
  {
    const int64_t ia = has_a ? gra : 0, ib = has_b ? grb : 0, ibg = has_body ? bg : 0;
    const uint8_t fa = a.flag[ia], fb = a.flag[ib];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      pa[i] = a.pr[i * a.nrs + ia];
      pb[i] = a.pl[i * a.nrs + ib];
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) q[c] = a.q[c * a.ns + ibg];
    const double *src = MODE == 2 ? a.rp : a.qd;
#pragma unroll
    for (int c = 0; c < 12; ++c) qd0[c] = src[c * a.ns + ibg];
    const int s = a.shp[ibg];
    T_h = a.hinv + (int64_t)HINV_STRIDE * s;
    shc = a.shape + (int64_t)SHAPE_STRIDE * s;
    if constexpr (PACK && APPLY) {
      const int li = t - 1, j = li >> 2, Tp = (T + 3) >> 2;
      if (t >= 1 && t <= T + 1 && (li & 3) == 0 && j > 0 && j < Tp) {
        const double *cf = a.pcf + (int64_t)(ti >> 2) * (PACK_CF * 64) + 16 * (ti & 3) + j;
        double v[PACK_CF];
#pragma unroll
        for (int k = 0; k < PACK_CF; ++k) v[k] = cf[k * 64];
#pragma unroll
        for (int k = 0; k < PACK_CF; ++k) lds[STG + k * 16 + j] = v[k];
      }
      if (t == 1 || t == T + 1) {
        const int64_t gi = (int64_t)cd.grow0 + td.tidx + (t == T + 1 ? 1 : 0);
        double v[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) v[i] = a.xg[3 * gi + i];
#pragma unroll
        for (int i = 0; i < 3; ++i) lds[STG_X + (t == 1 ? 0 : 3) + i] = v[i];
      }
    }
    if (has_a) sa = (fa & 2) ? 1.0 : -1.0;
    else pa[0] = pa[1] = pa[2] = 0.0;
    if (has_b) sb = (fb & 1) ? 1.0 : -1.0;
    else pb[0] = pb[1] = pb[2] = 0.0;
  }
  if (gate.skip() || ir0 != 0.0) return;  // uniform: before any barrier
  if (has_body) {
    {
#pragma unroll
      for (int i = 0; i < 7; ++i) sh[i] = shc[i];
#pragma unroll
      for (int i = 0; i < HINV_STRIDE; ++i) hv[i] = T_h[i];
    }
    double A[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) A[3 * i + c] = q[3 * c + i];
    breal Ab[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Ab[i] = breal(A[i]);
    if (!polar3(Ab, R)) {
      raise_flag(a.status, FLAG_NONFINITE, a.step);
#pragma unroll
      for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? breal(1) : breal(0);
    }
    breal phi[12];
    if constexpr (MODE == 2) {
      // rotated FP64 primal residual of the current iterate
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        breal w[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) w[i] = breal(qd0[3 * c + i]);
        mat3t_vec(R, w, phi + 3 * c);
      }
    } else {
      breal qb[12], qdb[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        qb[c] = breal(q[c]);
        qdb[c] = breal(qd0[c]);
      }
      local_force<breal>(sh, R, Ab, qb, qb, qdb, a.g, a.h, phi, WR ? a.wr : nullptr, a.ns, bg);
    }
    hinv_apply(hv, phi, u);
    const breal paf[3] = {breal(pa[0]), breal(pa[1]), breal(pa[2])};
    const breal pbf[3] = {breal(pb[0]), breal(pb[1]), breal(pb[2])};
    if (has_a) {
      breal W[9], RW[9];
      wblock(hv, paf, paf, W);
      rot_congr(R, W, RW);
      double RWd[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) RWd[i] = double(RW[i]);
      sym_from_full(RWd, Waa);
      breal Ju[3], vv[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) Ju[i] = paf[0] * u[i] + paf[1] * u[3 + i] + paf[2] * u[6 + i] + u[9 + i];
      mat3_vec(R, Ju, vv);
#pragma unroll
      for (int i = 0; i < 3; ++i) va[i] = double(vv[i]) * sa;
      if constexpr (MODE != 2) {
        double Ap[3];
        mat3_vec(A, pa, Ap);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          ca[i] = sa * Ap[i];
          ta[i] = sa * q[9 + i];
        }
      }
    }
    if (has_b) {
      breal W[9], RW[9];
      wblock(hv, pbf, pbf, W);
      rot_congr(R, W, RW);
      double RWd[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) RWd[i] = double(RW[i]);
      sym_from_full(RWd, Wbb);
      breal Ju[3], vv[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) Ju[i] = pbf[0] * u[i] + pbf[1] * u[3 + i] + pbf[2] * u[6 + i] + u[9 + i];
      mat3_vec(R, Ju, vv);
#pragma unroll
      for (int i = 0; i < 3; ++i) vb[i] = double(vv[i]) * sb;
      if constexpr (MODE != 2) {
        double Ap[3];
        mat3_vec(A, pb, Ap);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          cb[i] = sb * Ap[i];
          tb[i] = sb * q[9 + i];
        }
      }
    }
    if (has_a && has_b) {
      breal W[9], RW[9];
      wblock(hv, paf, pbf, W);
      rot_congr(R, W, RW);
#pragma unroll
      for (int i = 0; i < 9; ++i) Wab[i] = double(RW[i]) * (sa * sb);
    }
  } else {
    // world end: only the constant point enters C
    if (has_a)
      for (int i = 0; i < 3; ++i) ca[i] = sa * pa[i];
    if (has_b)
      for (int i = 0; i < 3; ++i) cb[i] = sb * pb[i];
  }
  // publish the part that belongs to row r+1 (left end of that row)
#pragma unroll
  for (int i = 0; i < 6; ++i) lds[(S_WBB + i) * NT + t] = Wbb[i];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    lds[(S_VB + i) * NT + t] = vb[i];
    lds[(S_CB + i) * NT + t] = cb[i];
    lds[(S_TB + i) * NT + t] = tb[i];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) lds[(S_WAB + i) * NT + t] = Wab[i];
  __syncthreads();

  // ---------------------------------------------------------------- phase B
  const int li = t - 1;                  // local row index 0..T
  const bool row_active = t >= 1 && t <= T + 1;
  double L[9], D[6], U[9], b[3];
#pragma unroll
  for (int i = 0; i < 9; ++i) { L[i] = 0.0; U[i] = Wab[i]; }
  if (row_active) {
    const int tp = t - 1;
#pragma unroll
    for (int i = 0; i < 6; ++i) D[i] = Waa[i] + lds[(S_WBB + i) * NT + tp];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if constexpr (MODE == 2) {
        b[i] = va[i] + lds[(S_VB + i) * NT + tp] - a.rd[i * a.nrs + gra];
      } else {
        // C = (translation difference) + (rotated anchor difference)
        double C = (lds[(S_TB + i) * NT + tp] + ta[i]) +
                   (lds[(S_CB + i) * NT + tp] + ca[i]);
        b[i] = va[i] + lds[(S_VB + i) * NT + tp] + C;
      }
    }
    // left coupling = (U of the previous row)^T
    if (li >= 1) {
#pragma unroll
      for (int r2 = 0; r2 < 3; ++r2)
#pragma unroll
        for (int c2 = 0; c2 < 3; ++c2) L[3 * r2 + c2] = lds[(S_WAB + 3 * c2 + r2) * NT + tp];
    }
    if (li == T && r != cd.K - 1) {
      // interface row owned by the next tile: only Schur updates are summed here
#pragma unroll
      for (int i = 0; i < 6; ++i) D[i] = 0.0;
      b[0] = b[1] = b[2] = 0.0;
    }
    if (li == T) {
#pragma unroll
      for (int i = 0; i < 9; ++i) U[i] = 0.0;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 6; ++i) D[i] = 0.0;
    b[0] = b[1] = b[2] = 0.0;
  }
  __syncthreads();

  // ---------------------------------------------------------------- phase C
  double PL[9], PU[9], Pb[3];
  int elim_d = 0;
  tile_cr_forward<NT>(lds, row_active, li, T, PACK ? 4 : T, L, D, U, b, PL, PU, Pb, elim_d,
                      a.status, a.step);

  if constexpr (!APPLY && PACK) {
    // survivors to the group's slots (reduced by chain_pack_kernel)
    const int grp = ti >> 2, Tp = (T + 3) >> 2;
    if (row_active && (li == T || (li & 3) == 0)) {
      const int j = li == T ? Tp : li >> 2;
      double *sv = a.psv + (int64_t)grp * (PACK_SV * 64) + 16 * (ti & 3) + j;
#pragma unroll
      for (int i = 0; i < 6; ++i) sv[i * 64] = D[i];
#pragma unroll
      for (int i = 0; i < 3; ++i) sv[(6 + i) * 64] = b[i];
#pragma unroll
      for (int i = 0; i < 9; ++i) sv[(9 + i) * 64] = U[i];
    }
  } else if constexpr (!APPLY) {
    double *rec = a.tilerec + (int64_t)TILE_REC * ti;
    if (row_active && li == 0) {
#pragma unroll
      for (int i = 0; i < 6; ++i) rec[i] = D[i];
#pragma unroll
      for (int i = 0; i < 3; ++i) rec[6 + i] = b[i];
#pragma unroll
      for (int i = 0; i < 9; ++i) rec[18 + i] = U[i];
    }
    if (row_active && li == T) {
#pragma unroll
      for (int i = 0; i < 6; ++i) rec[9 + i] = D[i];
#pragma unroll
      for (int i = 0; i < 3; ++i) rec[15 + i] = b[i];
    }
  } else {
    // -------------------------------------------------- back-substitution
    if constexpr (PACK) {
      // rows eliminated in the packed levels take their factors from the
      // reduce pass
      const int j = li >> 2, Tp = (T + 3) >> 2;
      if (row_active && (li & 3) == 0 && j > 0 && j < Tp) {
        elim_d = 4 * (j & -j);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          PL[i] = lds[STG + i * 16 + j];
          PU[i] = lds[STG + (9 + i) * 16 + j];
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) Pb[i] = lds[STG + (18 + i) * 16 + j];
      }
    }
    if (row_active && (li == 0 || li == T)) {
      if constexpr (PACK) {
#pragma unroll
        for (int i = 0; i < 3; ++i) lds[(S_X + i) * NT + li] = lds[STG_X + (li == T ? 3 : 0) + i];
      } else {
        const int64_t gi = (int64_t)cd.grow0 + td.tidx + (li == T ? 1 : 0);
#pragma unroll
        for (int i = 0; i < 3; ++i) lds[(S_X + i) * NT + li] = a.xg[3 * gi + i];
      }
    }
    __syncthreads();
    tile_cr_backward<NT>(lds, row_active, li, T, elim_d, PL, PU, Pb);
    // multipliers of the tile's rows (interface row T is written by the next tile)
    const bool last_tile = td.tidx == cd.ntile - 1;
    if (row_active && (li < T || last_tile)) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        if constexpr (MODE == 2) a.lam[3 * gra + i] += lds[(S_X + i) * NT + li];
        else a.lam[3 * gra + i] = lds[(S_X + i) * NT + li];
      }
    }
    // -------------------------------------------------- body back-projection
    bool own = has_body && ((t >= 1 && t <= T) || (t == 0 && td.tidx == 0) ||
                            (t == T + 1 && last_tile));
    if (own) {
      breal g12[12];
#pragma unroll
      for (int i = 0; i < 12; ++i) g12[i] = breal(0);
      if (has_a) {  // row r is local row t-1
        breal lamv[3], w[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) lamv[i] = breal(lds[(S_X + i) * NT + (t - 1)]);
        mat3t_vec(R, lamv, w);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          w[i] *= breal(sa);
          g12[i] += breal(pa[0]) * w[i];
          g12[3 + i] += breal(pa[1]) * w[i];
          g12[6 + i] += breal(pa[2]) * w[i];
          g12[9 + i] += w[i];
        }
      }
      if (has_b) {  // row r+1 is local row t
        breal lamv[3], w[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) lamv[i] = breal(lds[(S_X + i) * NT + t]);
        mat3t_vec(R, lamv, w);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          w[i] *= breal(sb);
          g12[i] += breal(pb[0]) * w[i];
          g12[3 + i] += breal(pb[1]) * w[i];
          g12[6 + i] += breal(pb[2]) * w[i];
          g12[9 + i] += w[i];
        }
      }
      breal hg[12];
      hinv_apply(T_h, g12, hg);
      const double ih = 1.0 / a.h;
      bool finite = true;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        breal dp[3], dqv[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) dp[i] = u[3 * c + i] - hg[3 * c + i];
        mat3_vec(R, dp, dqv);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const int64_t o = (int64_t)(3 * c + i) * a.ns + bg;
          const double d = double(dqv[i]);
          if constexpr (MODE == 0) {
            a.q_out[o] = q[3 * c + i] + d;
            a.qd_out[o] = d * ih;
          } else if constexpr (MODE == 1) {
            a.dq[o] = d;
          } else {
            a.dq[o] += d;
          }
          finite = finite && isfinite(d);
        }
      }
      if (!finite) raise_flag(a.status, FLAG_NONFINITE, a.step);
    }
  }
}

// One wave per group of four packed tiles.  Groups are ordered like the tiles
// (xcd_tile4), so a group runs on the XCD whose L2 holds its survivors.
template <int MODE>
__global__ __launch_bounds__(64) void chain_pack_kernel(ChainArgs a) {
  __shared__ double lds[S_N * 64];
  const StepGate gate = step_gate(a.status);
  const double ir0 = MODE == 2 ? a.ir[0] : 0.0;
  if constexpr (MODE == 2) {
    if (ir0 != 0.0) return;  // converged: skip before the survivors' reads
  }
  const int ngrp = (a.ntiles + 3) / 4;
  const int per = (a.ntiles + 31) / 32;  // groups per XCD range
  const int grp = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (grp >= ngrp) return;
  pack_reduce_group(a, grp, lds, gate, ir0);
}

// Top system of a chain (rows that bound its groups), n = ngroup + 1 <= 256
// rows, one per thread: cyclic reduction onto rows 0 and n-1, a 6x6 Cholesky
// solve of those two, back-substitution.  Called by one whole workgroup.
DEV void top_solve(double *lds, const ChainDesc &cd, const double *grouprec, double *xtop,
                   uint32_t *status, int step) {
  const int n = cd.ngroup + 1;
  const int T = n - 1;
  const int li = threadIdx.x;
  const bool row_active = li < n;
  const double *TR = grouprec + (int64_t)TILE_REC * cd.group0;
  double L[9], D[6], U[9], b[3];
  for (int i = 0; i < 9; ++i) { L[i] = 0.0; U[i] = 0.0; }
  for (int i = 0; i < 6; ++i) D[i] = 0.0;
  b[0] = b[1] = b[2] = 0.0;
  if (row_active) {
    if (li < cd.ngroup) {
      for (int i = 0; i < 6; ++i) D[i] += TR[TILE_REC * li + i];
      for (int i = 0; i < 3; ++i) b[i] += TR[TILE_REC * li + 6 + i];
      for (int i = 0; i < 9; ++i) U[i] = TR[TILE_REC * li + 18 + i];
    }
    if (li > 0) {
      for (int i = 0; i < 6; ++i) D[i] += TR[TILE_REC * (li - 1) + 9 + i];
      for (int i = 0; i < 3; ++i) b[i] += TR[TILE_REC * (li - 1) + 15 + i];
      for (int r2 = 0; r2 < 3; ++r2)
        for (int c2 = 0; c2 < 3; ++c2) L[3 * r2 + c2] = TR[TILE_REC * (li - 1) + 18 + 3 * c2 + r2];
    }
  }
  double PL[9], PU[9], Pb[3];
  int elim_d = 0;
  tile_cr_forward<CHAIN_THREADS>(lds, row_active, li, T, T, L, D, U, b, PL, PU, Pb, elim_d, status, step);
  // rows 0 and T now form [D0 U0; U0^T DT] [x0; xT] = [b0; bT]
  if (li == 0) {
    for (int i = 0; i < 6; ++i) lds[(S_PL + i) * CHAIN_THREADS] = D[i];
    for (int i = 0; i < 9; ++i) lds[(S_PU + i) * CHAIN_THREADS] = U[i];
    for (int i = 0; i < 3; ++i) lds[(S_PB + i) * CHAIN_THREADS] = b[i];
  }
  if (li == T) {  // column 1 is free once the reduction has finished
    for (int i = 0; i < 6; ++i) lds[(S_PL + i) * CHAIN_THREADS + 1] = D[i];
    for (int i = 0; i < 3; ++i) lds[(S_PB + i) * CHAIN_THREADS + 1] = b[i];
  }
  __syncthreads();
  if (li == 0) {
    double M[36], r[6];
    double D0[9], DT[9];
    double s0[6], s1[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) { s0[i] = lds[(S_PL + i) * CHAIN_THREADS]; s1[i] = lds[(S_PL + i) * CHAIN_THREADS + 1]; }
    full_from_sym(s0, D0);
    full_from_sym(s1, DT);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double u = lds[(S_PU + 3 * i + j) * CHAIN_THREADS];
        M[6 * i + j] = D0[3 * i + j];
        M[6 * (i + 3) + j + 3] = DT[3 * i + j];
        M[6 * i + j + 3] = u;
        M[6 * (j + 3) + i] = u;
      }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      r[i] = lds[(S_PB + i) * CHAIN_THREADS];
      r[3 + i] = lds[(S_PB + i) * CHAIN_THREADS + 1];
    }
    // Cholesky 6x6, fully unrolled (constant indices keep M and r in
    // registers); a non-positive pivot is replaced by 1 and reported
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double d = M[6 * j + j];
#pragma unroll
      for (int k = 0; k < j; ++k) d -= M[6 * j + k] * M[6 * j + k];
      ok = ok && d > 0.0;
      d = d > 0.0 ? sqrt(d) : 1.0;
      M[6 * j + j] = d;
      const double id = 1.0 / d;
#pragma unroll
      for (int i = j + 1; i < 6; ++i) {
        double v = M[6 * i + j];
#pragma unroll
        for (int k = 0; k < j; ++k) v -= M[6 * i + k] * M[6 * j + k];
        M[6 * i + j] = v * id;
      }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      double v = r[i];
#pragma unroll
      for (int k = 0; k < i; ++k) v -= M[6 * i + k] * r[k];
      r[i] = v / M[6 * i + i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
      double v = r[i];
#pragma unroll
      for (int k = i + 1; k < 6; ++k) v -= M[6 * k + i] * r[k];
      r[i] = v / M[6 * i + i];
    }
    if (!ok) {
      raise_flag(status, FLAG_SINGULAR, step);
#pragma unroll
      for (int i = 0; i < 6; ++i) r[i] = 0.0;
    }
    for (int i = 0; i < 3; ++i) {
      lds[(S_X + i) * CHAIN_THREADS + 0] = r[i];
      lds[(S_X + i) * CHAIN_THREADS + T] = r[3 + i];
    }
  }
  __syncthreads();
  tile_cr_backward<CHAIN_THREADS>(lds, row_active, li, T, elim_d, PL, PU, Pb);
  if (row_active)
    for (int i = 0; i < 3; ++i) xtop[3 * ((int64_t)cd.gtop0 + li) + i] = lds[(S_X + i) * CHAIN_THREADS + li];
}

// Interface rows of one chain form again a block-tridiagonal system: row gi
// gathers D and b from the two tiles that share it and couples to row gi+1
// through the tile's Schur block U.  Groups of GROUP_T + 1 interface rows are
// reduced like tiles (reduce variant: Schur record of the group's two end
// rows) and back-substituted once the top system is solved (apply variant:
// x of every interface row).  The reduce variant keeps the factors
// (PL, PU, Pb) of the rows it eliminates in gfac ([PACK_CF][CHAIN_THREADS]
// per group); the apply variant reads them back instead of repeating the
// elimination (every interior row li is eliminated at level lowbit(li)).
template <bool APPLY>
__global__ __launch_bounds__(CHAIN_THREADS) void chain_group_kernel(
    const ChainDesc *chains, const GroupDesc *groups, const double *tilerec, double *grouprec,
    double *xtop, double *xg, double *gfac, int *counters, uint32_t *status, int step,
    const double *ir) {
  __shared__ double lds[S_N * CHAIN_THREADS];
  // step gate and convergence flag (form 1 corrections) read first, tested
  // once the group's reads are in flight (before any barrier or store)
  const StepGate gate = step_gate(status);
  const double ir0 = ir ? ir[0] : 0.0;
  const GroupDesc gd = groups[blockIdx.x];
  const ChainDesc cd = chains[gd.chain];
  const int li = threadIdx.x;
  const int T = gd.T;
  const int gi = gd.g0 + li;               // chain-local interface row
  const int n = cd.ntile + 1;
  const bool row_active = li <= T;
  double *fac = gfac + (int64_t)blockIdx.x * (PACK_CF * CHAIN_THREADS) + li;
  if constexpr (APPLY) {
    double PL[9], PU[9], Pb[3];
    int elim_d = 0;
    if (row_active && li > 0 && li < T) {
      elim_d = li & -li;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        PL[i] = fac[i * CHAIN_THREADS];
        PU[i] = fac[(9 + i) * CHAIN_THREADS];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) Pb[i] = fac[(18 + i) * CHAIN_THREADS];
    }
    if (gate.skip() || ir0 != 0.0) return;
    if (row_active && (li == 0 || li == T)) {
      const int64_t ti = (int64_t)cd.gtop0 + gd.gidx + (li == T ? 1 : 0);
      for (int i = 0; i < 3; ++i) lds[(S_X + i) * CHAIN_THREADS + li] = xtop[3 * ti + i];
    }
    __syncthreads();
    tile_cr_backward<CHAIN_THREADS>(lds, row_active, li, T, elim_d, PL, PU, Pb);
    const bool last = gd.gidx == cd.ngroup - 1;
    if (row_active && (li < T || last))
      for (int i = 0; i < 3; ++i) xg[3 * ((int64_t)cd.grow0 + gi) + i] = lds[(S_X + i) * CHAIN_THREADS + li];
    return;
  }
  const double *TR = tilerec + (int64_t)TILE_REC * cd.tile0;
  double L[9], D[6], U[9], b[3];
#pragma unroll
  for (int i = 0; i < 9; ++i) { L[i] = 0.0; U[i] = 0.0; }
#pragma unroll
  for (int i = 0; i < 6; ++i) D[i] = 0.0;
  b[0] = b[1] = b[2] = 0.0;
  if (row_active && !(li == T && gi != n - 1)) {
    if (gi < cd.ntile) {
      for (int i = 0; i < 6; ++i) D[i] += TR[TILE_REC * gi + i];
      for (int i = 0; i < 3; ++i) b[i] += TR[TILE_REC * gi + 6 + i];
    }
    if (gi > 0) {
      for (int i = 0; i < 6; ++i) D[i] += TR[TILE_REC * (gi - 1) + 9 + i];
      for (int i = 0; i < 3; ++i) b[i] += TR[TILE_REC * (gi - 1) + 15 + i];
    }
  }
  if (row_active && li < T)
    for (int i = 0; i < 9; ++i) U[i] = TR[TILE_REC * gi + 18 + i];
  if (row_active && li > 0)
    for (int r2 = 0; r2 < 3; ++r2)
      for (int c2 = 0; c2 < 3; ++c2) L[3 * r2 + c2] = TR[TILE_REC * (gi - 1) + 18 + 3 * c2 + r2];
  if (gate.skip() || ir0 != 0.0) return;
  double PL[9], PU[9], Pb[3];
  int elim_d = 0;
  tile_cr_forward<CHAIN_THREADS>(lds, row_active, li, T, T, L, D, U, b, PL, PU, Pb, elim_d, status, step);
  if (elim_d > 0) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      fac[i * CHAIN_THREADS] = PL[i];
      fac[(9 + i) * CHAIN_THREADS] = PU[i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) fac[(18 + i) * CHAIN_THREADS] = Pb[i];
  }
  {
    double *rec = grouprec + (int64_t)TILE_REC * (cd.group0 + gd.gidx);
    if (row_active && li == 0) {
      for (int i = 0; i < 6; ++i) rec[i] = D[i];
      for (int i = 0; i < 3; ++i) rec[6 + i] = b[i];
      for (int i = 0; i < 9; ++i) rec[18 + i] = U[i];
    }
    if (row_active && li == T) {
      for (int i = 0; i < 6; ++i) rec[9 + i] = D[i];
      for (int i = 0; i < 3; ++i) rec[15 + i] = b[i];
    }
    // The last group of the chain to finish solves the top system (its
    // ngroup + 1 rows fit one workgroup); longer chains use chain_global.
    if (!cd.top_global) {
      __shared__ int is_last;
      __syncthreads();
      if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int prev = atomicAdd(counters + gd.chain, 1);
        is_last = prev == cd.ngroup - 1;
      }
      __syncthreads();
      if (is_last) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        top_solve(lds, cd, grouprec, xtop, status, step);
        if (threadIdx.x == 0) counters[gd.chain] = 0;
      }
    }
  }
}

// Interface system of each chain: rows gi = 0..ntile, block tridiagonal,
// solved by block cyclic reduction in global scratch (one workgroup per chain).
__global__ __launch_bounds__(256) void chain_global_kernel(const ChainDesc *chains,
                                                           const double *tilerec, double *scr,
                                                           double *xg, uint32_t *status, int step,
                                                           const double *ir) {
  if (skip_step(status, step)) return;
  if (ir && ir[0] != 0.0) return;
  const ChainDesc cd = chains[blockIdx.x];
  if (!cd.top_global) return;  // solved by the last group workgroup
  // top system: the rows that bound the groups (records in tilerec = group records)
  const int n = cd.ngroup + 1;
  double *S = scr + (int64_t)GROW_REC * cd.gtop0;
  const double *TR = tilerec + (int64_t)TILE_REC * cd.group0;
  // record: L 0..8, D 9..17, U 18..26, b 27..29, PL 30..38, PU 39..47, Pb 48..50
  enum { GL = 0, GD = 9, GU = 18, GB = 27, GPL = 30, GPU = 39, GPB = 48 };
  for (int gi = threadIdx.x; gi < n; gi += blockDim.x) {
    double *row = S + (int64_t)GROW_REC * gi;
    double Ds[6] = {0, 0, 0, 0, 0, 0}, bb[3] = {0, 0, 0};
    if (gi < cd.ngroup) {
      for (int i = 0; i < 6; ++i) Ds[i] += TR[TILE_REC * gi + i];
      for (int i = 0; i < 3; ++i) bb[i] += TR[TILE_REC * gi + 6 + i];
    }
    if (gi > 0) {
      for (int i = 0; i < 6; ++i) Ds[i] += TR[TILE_REC * (gi - 1) + 9 + i];
      for (int i = 0; i < 3; ++i) bb[i] += TR[TILE_REC * (gi - 1) + 15 + i];
    }
    double Df[9];
    full_from_sym(Ds, Df);
    for (int i = 0; i < 9; ++i) row[GD + i] = Df[i];
    for (int i = 0; i < 3; ++i) row[GB + i] = bb[i];
    for (int i = 0; i < 9; ++i) {
      row[GU + i] = gi < cd.ngroup ? TR[TILE_REC * gi + 18 + i] : 0.0;
      int r2 = i / 3, c2 = i % 3;
      row[GL + i] = gi > 0 ? TR[TILE_REC * (gi - 1) + 18 + 3 * c2 + r2] : 0.0;
    }
  }
  __syncthreads();
  int dlast = 0;
  for (int d = 1; d < n; d *= 2) {
    dlast = d;
    for (int e = d + threadIdx.x * 2 * d; e < n; e += blockDim.x * 2 * d) {
      double *row = S + (int64_t)GROW_REC * e;
      double Di[9], Dm[9];
      for (int i = 0; i < 9; ++i) Dm[i] = row[GD + i];
      if (!spd3_inv(Dm, Di)) {
        raise_flag(status, FLAG_SINGULAR, step);
        for (int i = 0; i < 9; ++i) Di[i] = 0.0;
      }
      double X[9], Y[9], z[3], Lm[9], Um[9], bv[3];
      for (int i = 0; i < 9; ++i) { Lm[i] = row[GL + i]; Um[i] = row[GU + i]; }
      for (int i = 0; i < 3; ++i) bv[i] = row[GB + i];
      mat3_mul(Di, Lm, X);
      mat3_mul(Di, Um, Y);
      mat3_vec(Di, bv, z);
      for (int i = 0; i < 9; ++i) { row[GPL + i] = X[i]; row[GPU + i] = Y[i]; }
      for (int i = 0; i < 3; ++i) row[GPB + i] = z[i];
    }
    __syncthreads();
    for (int s = threadIdx.x * 2 * d; s < n; s += blockDim.x * 2 * d) {
      double *row = S + (int64_t)GROW_REC * s;
      double Dm[9], Lm[9], Um[9], bv[3];
      for (int i = 0; i < 9; ++i) { Dm[i] = row[GD + i]; Lm[i] = row[GL + i]; Um[i] = row[GU + i]; }
      for (int i = 0; i < 3; ++i) bv[i] = row[GB + i];
      if (s + d < n) {
        const double *er = S + (int64_t)GROW_REC * (s + d);
        double M[9], Xu[9], Xl[9], xb[3], v[3];
        for (int i = 0; i < 9; ++i) { Xl[i] = er[GPL + i]; Xu[i] = er[GPU + i]; }
        for (int i = 0; i < 3; ++i) xb[i] = er[GPB + i];
        mat3_mul(Um, Xl, M);
        for (int i = 0; i < 9; ++i) Dm[i] -= M[i];
        mat3_vec(Um, xb, v);
        for (int i = 0; i < 3; ++i) bv[i] -= v[i];
        mat3_mul(Um, Xu, M);
        for (int i = 0; i < 9; ++i) Um[i] = -M[i];
      } else {
        for (int i = 0; i < 9; ++i) Um[i] = 0.0;
      }
      if (s - d >= 0) {
        const double *er = S + (int64_t)GROW_REC * (s - d);
        double M[9], Xu[9], Xl[9], xb[3], v[3];
        for (int i = 0; i < 9; ++i) { Xl[i] = er[GPL + i]; Xu[i] = er[GPU + i]; }
        for (int i = 0; i < 3; ++i) xb[i] = er[GPB + i];
        mat3_mul(Lm, Xu, M);
        for (int i = 0; i < 9; ++i) Dm[i] -= M[i];
        mat3_vec(Lm, xb, v);
        for (int i = 0; i < 3; ++i) bv[i] -= v[i];
        mat3_mul(Lm, Xl, M);
        for (int i = 0; i < 9; ++i) Lm[i] = -M[i];
      }
      // symmetrise the pivot block
      double a01 = 0.5 * (Dm[1] + Dm[3]), a02 = 0.5 * (Dm[2] + Dm[6]), a12 = 0.5 * (Dm[5] + Dm[7]);
      Dm[1] = Dm[3] = a01; Dm[2] = Dm[6] = a02; Dm[5] = Dm[7] = a12;
      for (int i = 0; i < 9; ++i) { row[GD + i] = Dm[i]; row[GL + i] = Lm[i]; row[GU + i] = Um[i]; }
      for (int i = 0; i < 3; ++i) row[GB + i] = bv[i];
    }
    __syncthreads();
  }
  double *X = xg + 3 * (int64_t)cd.gtop0;
  if (threadIdx.x == 0) {
    double Dm[9], Di[9], bv[3], x[3];
    for (int i = 0; i < 9; ++i) Dm[i] = S[GD + i];
    for (int i = 0; i < 3; ++i) bv[i] = S[GB + i];
    if (!spd3_inv(Dm, Di)) {
      raise_flag(status, FLAG_SINGULAR, step);
      for (int i = 0; i < 9; ++i) Di[i] = 0.0;
    }
    mat3_vec(Di, bv, x);
    for (int i = 0; i < 3; ++i) X[i] = x[i];
  }
  __syncthreads();
  for (int d = dlast; d >= 1; d /= 2) {
    for (int e = d + threadIdx.x * 2 * d; e < n; e += blockDim.x * 2 * d) {
      const double *row = S + (int64_t)GROW_REC * e;
      double xl[3], xr[3] = {0, 0, 0}, x[3];
      for (int i = 0; i < 3; ++i) xl[i] = X[3 * (e - d) + i];
      if (e + d < n)
        for (int i = 0; i < 3; ++i) xr[i] = X[3 * (e + d) + i];
      for (int i = 0; i < 3; ++i) {
        x[i] = row[GPB + i];
        for (int j = 0; j < 3; ++j) x[i] -= row[GPL + 3 * i + j] * xl[j] + row[GPU + 3 * i + j] * xr[j];
      }
      for (int i = 0; i < 3; ++i) X[3 * e + i] = x[i];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ form 1
// FP64 KKT residual of the current iterate (q + dq, lam) on the chain rows and
// bodies: r_p = f_A - H dq - G^T lam per body (world frame) and
// r_d = -(C + G dq) per row, and per tile the sums behind
// rho_p = |H^{-1} r_p| / |H^{-1} f_A| and rho_d = |r_d| / |G H^{-1} f_A + C|
// (the KKT residual of Eq. kkt with the -C right-hand side).
//
// With a.diag set the kernel checks a finished step instead: q, qd are the
// state the step started from, dq = h qd_out its increment, nothing is
// stored but the tile partials (DIAG_PART per tile: the four sums, then the
// largest |C| of the rows at the new state q_out, then 0 for hinges).
template <int NT, bool WR>
__global__ __launch_bounds__(NT) void chain_resid_kernel(ChainArgs a) {
  enum { L_VB = 0, L_CB = 3, L_TB = 6, L_GB = 9, L_RED = 12, L_CN = 16, L_TN = 19, L_CM = 22, L_SE = 23 };
  __shared__ double lds[24 * NT];
  if (skip_step(a.status, a.step)) return;
  const bool diag = a.diag != 0;
  if (!diag && a.ir[0] != 0.0) return;
  const int ti = xcd_tile(a.ntiles);
  if (ti < 0) return;
  const TileDesc td = a.tiles[ti];
  const ChainDesc cd = a.chains[td.chain];
  const int t = threadIdx.x;
  const int T = td.T;
  const int r = td.r0 + t - 1;
  const int p = r + 1 - cd.hl;
  const bool in_tile = t <= T + 1;
  const bool has_body = in_tile && p >= 0 && p < cd.nb;
  const bool has_a = in_tile && r >= 0 && r < cd.K;
  const bool has_b = in_tile && r + 1 < cd.K;
  const int64_t gra = (int64_t)cd.row0 + r;
  const int64_t grb = gra + 1;
  const int64_t bg = (int64_t)cd.body0 + p;
  const bool last_tile = td.tidx == cd.ntile - 1;
  const bool own = has_body && ((t >= 1 && t <= T) || (t == 0 && td.tidx == 0) ||
                                (t == T + 1 && last_tile));
  double pa[3] = {0, 0, 0}, pb[3] = {0, 0, 0}, la[3] = {0, 0, 0}, lb[3] = {0, 0, 0};
  double sa = 1.0, sb = 1.0;
  double va[3] = {0, 0, 0}, ca[3] = {0, 0, 0}, ta[3] = {0, 0, 0}, ga[3] = {0, 0, 0};
  double vb[3] = {0, 0, 0}, cb[3] = {0, 0, 0}, tb[3] = {0, 0, 0}, gb[3] = {0, 0, 0};
  // diag: the joint values at the new state, split as in C
  double cna[3] = {0, 0, 0}, tna[3] = {0, 0, 0}, cnb[3] = {0, 0, 0}, tnb[3] = {0, 0, 0};
  // sums behind rho_p, rho_d; se: squared size of the summands of r_d (its
  // rounding floor); cmax: diagnostics
  double sp = 0.0, sf = 0.0, sr = 0.0, sd = 0.0, se = 0.0, cmax = 0.0;
  if (has_a) {
    for (int i = 0; i < 3; ++i) {
      pa[i] = a.pr[i * a.nrs + gra];
      la[i] = a.lam[3 * gra + i];
    }
    sa = (a.flag[gra] & 2) ? 1.0 : -1.0;
  }
  if (has_b) {
    for (int i = 0; i < 3; ++i) {
      pb[i] = a.pl[i * a.nrs + grb];
      lb[i] = a.lam[3 * grb + i];
    }
    sb = (a.flag[grb] & 1) ? 1.0 : -1.0;
  }
  if (has_body) {
    double q[12], qd[12], dq[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      q[c] = a.q[c * a.ns + bg];
      qd[c] = a.qd[c * a.ns + bg];
      dq[c] = diag ? a.h * a.qd_out[c * a.ns + bg] : a.dq[c * a.ns + bg];
    }
    if (diag) {
      double qn[12], An[9];
#pragma unroll
      for (int c = 0; c < 12; ++c) qn[c] = a.q_out[c * a.ns + bg];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) An[3 * i + c] = qn[3 * c + i];
      if (has_a) {
        mat3_vec(An, pa, cna);
#pragma unroll
        for (int i = 0; i < 3; ++i) { cna[i] *= sa; tna[i] = sa * qn[9 + i]; }
      }
      if (has_b) {
        mat3_vec(An, pb, cnb);
#pragma unroll
        for (int i = 0; i < 3; ++i) { cnb[i] *= sb; tnb[i] = sb * qn[9 + i]; }
      }
    }
    const int s = a.shp[bg];
    const double *T_h = a.hinv + (int64_t)HINV_STRIDE * s;
    const double *sh = a.shape + (int64_t)SHAPE_STRIDE * s;
    double A[9], R[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) A[3 * i + c] = q[3 * c + i];
    if (!polar3(A, R)) {
      raise_flag(a.status, FLAG_NONFINITE, a.step);
#pragma unroll
      for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
    }
    double phi[12], u[12];
    local_force<double>(sh, R, A, q, q, qd, a.g, a.h, phi, WR ? a.wr : nullptr, a.ns, bg);
    hinv_apply(T_h, phi, u);
    // r_p = diag4(R) (phi - Hbar diag4(R^T) dq) - G^T lam
    double dl[12], Hd[12], rw[12];
#pragma unroll
    for (int c = 0; c < 4; ++c) mat3t_vec(R, dq + 3 * c, dl + 3 * c);
    hbar_apply(sh, a.h, dl, Hd);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double e[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) e[i] = phi[3 * c + i] - Hd[3 * c + i];
      mat3_vec(R, e, rw + 3 * c);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double wa = has_a ? sa * la[i] : 0.0, wb = has_b ? sb * lb[i] : 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) rw[3 * c + i] -= pa[c] * wa + pb[c] * wb;
      rw[9 + i] -= wa + wb;
    }
    if (own) {
      if (!diag)
#pragma unroll
        for (int c = 0; c < 12; ++c) a.rp[c * a.ns + bg] = rw[c];
      double rl[12], y[12];
#pragma unroll
      for (int c = 0; c < 4; ++c) mat3t_vec(R, rw + 3 * c, rl + 3 * c);
      hinv_apply(T_h, rl, y);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        sp += y[k] * y[k];
        sf += u[k] * u[k];
      }
    }
    if (has_a) {
      double Ju[3], Ap[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) Ju[i] = pa[0] * u[i] + pa[1] * u[3 + i] + pa[2] * u[6 + i] + u[9 + i];
      mat3_vec(R, Ju, va);
      mat3_vec(A, pa, Ap);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        va[i] *= sa;
        ca[i] = sa * Ap[i];
        ta[i] = sa * q[9 + i];
        ga[i] = sa * (pa[0] * dq[i] + pa[1] * dq[3 + i] + pa[2] * dq[6 + i] + dq[9 + i]);
      }
    }
    if (has_b) {
      double Ju[3], Ap[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) Ju[i] = pb[0] * u[i] + pb[1] * u[3 + i] + pb[2] * u[6 + i] + u[9 + i];
      mat3_vec(R, Ju, vb);
      mat3_vec(A, pb, Ap);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        vb[i] *= sb;
        cb[i] = sb * Ap[i];
        tb[i] = sb * q[9 + i];
        gb[i] = sb * (pb[0] * dq[i] + pb[1] * dq[3 + i] + pb[2] * dq[6 + i] + dq[9 + i]);
      }
    }
  } else {
    // world end: only the constant point enters C
    if (has_a)
      for (int i = 0; i < 3; ++i) cna[i] = ca[i] = sa * pa[i];
    if (has_b)
      for (int i = 0; i < 3; ++i) cnb[i] = cb[i] = sb * pb[i];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    lds[(L_VB + i) * NT + t] = vb[i];
    lds[(L_CB + i) * NT + t] = cb[i];
    lds[(L_TB + i) * NT + t] = tb[i];
    lds[(L_GB + i) * NT + t] = gb[i];
    lds[(L_CN + i) * NT + t] = cnb[i];
    lds[(L_TN + i) * NT + t] = tnb[i];
  }
  __syncthreads();
  const int li = t - 1;
  if (t >= 1 && t <= T + 1 && (li < T || last_tile)) {
    const int tp = t - 1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double tt = lds[(L_TB + i) * NT + tp] + ta[i];
      const double cbl = lds[(L_CB + i) * NT + tp], gbl = lds[(L_GB + i) * NT + tp];
      const double C = tt + (cbl + ca[i]);
      const double rk = va[i] + lds[(L_VB + i) * NT + tp] + C;
      const double gdq = ga[i] + gbl;
      const double rdv = -(C + gdq);
      if (!diag) a.rd[i * a.nrs + gra] = rdv;
      sr += rk * rk;
      sd += rdv * rdv;
      // the summands r_d is formed from (the translation difference, both
      // anchor offsets, both ends' increments): its rounding floor
      se += tt * tt + cbl * cbl + ca[i] * ca[i] + ga[i] * ga[i] + gbl * gbl;
      if (diag) {
        const double Cn = (lds[(L_TN + i) * NT + tp] + tna[i]) + (lds[(L_CN + i) * NT + tp] + cna[i]);
        cmax = fmax(cmax, fabs(Cn));
      }
    }
  }
  lds[(L_RED + 0) * NT + t] = sp;
  lds[(L_RED + 1) * NT + t] = sf;
  lds[(L_RED + 2) * NT + t] = sr;
  lds[(L_RED + 3) * NT + t] = sd;
  lds[L_CM * NT + t] = cmax;
  lds[L_SE * NT + t] = se;
  __syncthreads();
  for (int w = NT / 2; w > 0; w /= 2) {
    if (t < w) {
#pragma unroll
      for (int k = 0; k < 4; ++k) lds[(L_RED + k) * NT + t] += lds[(L_RED + k) * NT + t + w];
      lds[L_SE * NT + t] += lds[L_SE * NT + t + w];
      lds[L_CM * NT + t] = fmax(lds[L_CM * NT + t], lds[L_CM * NT + t + w]);
    }
    __syncthreads();
  }
  if (diag) {
    double *o = a.part + DIAG_PART * (int64_t)ti;
    if (t < 4) o[t] = lds[(L_RED + t) * NT];
    if (t == 4) o[4] = lds[L_CM * NT];
    if (t == 5) o[5] = 0.0;
  } else if (t < 4) {
    a.part[IR_PART * (int64_t)ti + t] = lds[(L_RED + t) * NT];
  } else if (t == 4) {
    a.part[IR_PART * (int64_t)ti + 4] = lds[L_SE * NT];
  }
}

// Sums the tile partials in a fixed order and decides: converged (KKT
// residual <= tol: later corrections and checks of this step do nothing),
// stalled at the rounding floor within IR_STALL_FACTOR tol (likewise),
// stalled above it or, at the final check, still above tol (NOT_CONVERGED),
// or another correction sweep.
__global__ __launch_bounds__(256) void chain_ir_check_kernel(const double *part, int nblk, double tol,
                                                             int final_check, double *ir,
                                                             uint32_t *status) {
  __shared__ double red[IR_PART * 256];
  if (skip_step(status, 0)) return;
  if (ir[0] != 0.0) return;
  const int t = threadIdx.x;
  double s[IR_PART] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = t; b < nblk; b += 256)
    for (int k = 0; k < IR_PART; ++k) s[k] += part[IR_PART * (int64_t)b + k];
  for (int k = 0; k < IR_PART; ++k) red[k * 256 + t] = s[k];
  __syncthreads();
  for (int w = 128; w > 0; w /= 2) {
    if (t < w)
      for (int k = 0; k < IR_PART; ++k) red[k * 256 + t] += red[k * 256 + t + w];
    __syncthreads();
  }
  if (t == 0) {
    const double np = red[0], nf = red[256], nr = red[512], nd = red[768], ne = red[1024];
    const double rp = nf > 0.0 ? sqrt(np / nf) : sqrt(np);
    const double rdd = nr > 0.0 ? sqrt(nd / nr) : sqrt(nd);
    const double kkt = rp > rdd ? rp : rdd;
    ir[2] = rp;
    ir[3] = rdd;
    ir[4] = kkt;
    if (!isfinite(rp) || !isfinite(rdd)) raise_flag(status, FLAG_NONFINITE, 0);
    else if (kkt <= tol) ir[0] = 1.0;
    // a sweep that no longer halves the residual has reached the FP64
    // rounding floor of the residual itself: stop there, accepted when
    // within IR_STALL_FACTOR of the target, otherwise not converged
    else if (ir[1] > 0.0 && kkt > 0.5 * ir[5]) {
      // at the floor: within the factor of the target, or the primal part
      // is and the dual residual is at the rounding level of its own terms
      // (where the dual right-hand side all but vanishes, as for a freely
      // falling chain, rho_d is O(1) for every FP64 solution)
      const bool dual_at_rounding = sqrt(nd) <= IR_ROUND_FACTOR * DBL_EPSILON * sqrt(ne);
      if (kkt <= IR_STALL_FACTOR * tol || (rp <= IR_STALL_FACTOR * tol && dual_at_rounding)) {
        ir[0] = 2.0;
      } else {
        ir[0] = 3.0;
        raise_flag(status, FLAG_NOTCONV, 0);
      }
    }
    else if (final_check) raise_flag(status, FLAG_NOTCONV, 0);
    else ir[1] += 1.0;  // a correction sweep follows
    ir[5] = kkt;
  }
}

__global__ void chain_ir_reset_kernel(double *ir) {
  ir[0] = 0.0;
  ir[1] = 0.0;
}

// q_out = q + dq, qdot_out = dq / h for the chain bodies (form 1)
__global__ void chain_finish_kernel(const double *q, const double *dq, double *q_out, double *qd_out,
                                    int64_t ns, int nb, double h, uint32_t *status) {
  if (skip_step(status, 0)) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 12 * (int64_t)nb) return;
  const int64_t c = i / nb;
  const int64_t o = c * ns + (i - c * nb);
  const double d = dq[o];
  q_out[o] = q[o] + d;
  qd_out[o] = d * (1.0 / h);
  if (!isfinite(d)) raise_flag(status, FLAG_NONFINITE, 0);
}

// nt: 64, 128 or 256 threads per tile; pack: packed 64-thread tiles
template <int MODE, bool APPLY, bool WR>
static void launch_tiles(const ChainArgs &a, int ntiles, int nt, bool pack, hipStream_t s) {
  if (ntiles <= 0) return;
  if (pack) {
    hipLaunchKernelGGL((chain_tile_kernel<MODE, APPLY, 64, WR, true>), dim3(xcd_grid4(ntiles)),
                       dim3(64), 0, s, a);
    if (!APPLY)  // one workgroup per group of four tiles, XCD ranges as the tiles'
      hipLaunchKernelGGL((chain_pack_kernel<MODE>), dim3(8u * (unsigned)((ntiles + 31) / 32)),
                         dim3(64), 0, s, a);
    return;
  }
  const dim3 grid(xcd_grid(ntiles));
  if (nt == 64)
    hipLaunchKernelGGL((chain_tile_kernel<MODE, APPLY, 64, WR, false>), grid, dim3(64), 0, s, a);
  else if (nt == 128)
    hipLaunchKernelGGL((chain_tile_kernel<MODE, APPLY, 128, WR, false>), grid, dim3(128), 0, s, a);
  else
    hipLaunchKernelGGL((chain_tile_kernel<MODE, APPLY, 256, WR, false>), grid, dim3(256), 0, s, a);
}
template <bool APPLY>
static void launch_tiles_mode(const ChainArgs &a, int ntiles, int nt, bool pack, int mode,
                              hipStream_t s) {
  // the correction sweeps (mode 2) take the force from the FP64 residual
  if (mode == 0) {
    if (a.wr) launch_tiles<0, APPLY, true>(a, ntiles, nt, pack, s);
    else launch_tiles<0, APPLY, false>(a, ntiles, nt, pack, s);
  } else if (mode == 1) {
    if (a.wr) launch_tiles<1, APPLY, true>(a, ntiles, nt, pack, s);
    else launch_tiles<1, APPLY, false>(a, ntiles, nt, pack, s);
  } else {
    launch_tiles<2, APPLY, false>(a, ntiles, nt, pack, s);
  }
}
void launch_chain_reduce(const ChainArgs &a, int ntiles, int nt, bool pack, int mode,
                         hipStream_t s) {
  launch_tiles_mode<false>(a, ntiles, nt, pack, mode, s);
}
void launch_chain_apply(const ChainArgs &a, int ntiles, int nt, bool pack, int mode,
                        hipStream_t s) {
  launch_tiles_mode<true>(a, ntiles, nt, pack, mode, s);
}
void launch_chain_group(bool apply, const ChainDesc *chains, const GroupDesc *groups, int ngroups,
                        const double *tilerec, double *grouprec, double *xtop, double *xg,
                        double *gfac, int *counters, uint32_t *status, int step, const double *ir,
                        hipStream_t s) {
  if (ngroups <= 0) return;
  if (apply)
    hipLaunchKernelGGL(chain_group_kernel<true>, dim3(ngroups), dim3(CHAIN_THREADS), 0, s, chains,
                       groups, tilerec, grouprec, xtop, xg, gfac, counters, status, step, ir);
  else
    hipLaunchKernelGGL(chain_group_kernel<false>, dim3(ngroups), dim3(CHAIN_THREADS), 0, s, chains,
                       groups, tilerec, grouprec, xtop, xg, gfac, counters, status, step, ir);
}
void launch_chain_global(const ChainDesc *chains, int nchains, const double *tilerec, double *scr,
                         double *xg, uint32_t *status, int step, const double *ir, hipStream_t s) {
  if (nchains > 0)
    hipLaunchKernelGGL(chain_global_kernel, dim3(nchains), dim3(256), 0, s, chains, tilerec, scr,
                       xg, status, step, ir);
}
void launch_chain_resid(const ChainArgs &a, int ntiles, int nt, hipStream_t s) {
  if (ntiles <= 0) return;
  const dim3 grid(xcd_grid(ntiles));
  if (a.wr) {
    if (nt == 64)
      hipLaunchKernelGGL((chain_resid_kernel<64, true>), grid, dim3(64), 0, s, a);
    else if (nt == 128)
      hipLaunchKernelGGL((chain_resid_kernel<128, true>), grid, dim3(128), 0, s, a);
    else
      hipLaunchKernelGGL((chain_resid_kernel<256, true>), grid, dim3(256), 0, s, a);
  } else {
    if (nt == 64)
      hipLaunchKernelGGL((chain_resid_kernel<64, false>), grid, dim3(64), 0, s, a);
    else if (nt == 128)
      hipLaunchKernelGGL((chain_resid_kernel<128, false>), grid, dim3(128), 0, s, a);
    else
      hipLaunchKernelGGL((chain_resid_kernel<256, false>), grid, dim3(256), 0, s, a);
  }
}
void launch_chain_ir_check(const double *part, int nblk, double tol, int final_check, double *ir,
                           uint32_t *status, hipStream_t s) {
  hipLaunchKernelGGL(chain_ir_check_kernel, dim3(1), dim3(256), 0, s, part, nblk, tol, final_check,
                     ir, status);
}
void launch_chain_ir_reset(double *ir, hipStream_t s) {
  hipLaunchKernelGGL(chain_ir_reset_kernel, dim3(1), dim3(1), 0, s, ir);
}
void launch_chain_finish(const double *q, const double *dq, double *q_out, double *qd_out, int64_t ns,
                         int nb, double h, uint32_t *status, hipStream_t s) {
  if (nb <= 0) return;
  const int64_t n = 12 * (int64_t)nb;
  hipLaunchKernelGGL(chain_finish_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, q, dq,
                     q_out, qd_out, ns, nb, h, status);
}

}  // namespace mabd
