// Matrix-free dual operator of ball-jointed networks (Eq. ball, Eq. dual):
// the row block of a ball joint is s J(p) in world coordinates, so S v is a
// body pass followed by a joint pass.  Shared by the PCG and the learned
// warm start.
#pragma once
#include "common.hpp"
#include "dmath.hpp"
#include "generic.hpp"

namespace mabd {

// The body's own reads (incidence range, solver index, rotation, shape),
// which a caller may issue early, e.g. ahead of a reduction.
constexpr int BODY_ENT = 4;  // incidence entries read ahead (a lattice body has up to four joints)
struct BodyRefs {
  int e0, e1, shp;
  int64_t B;
  double R[9];
  int ent[BODY_ENT];
};
DEV BodyRefs body_refs(const PcgBallArgs &a, int i) {
  BodyRefs r;
  r.e0 = a.binc_off[i];
  r.e1 = a.binc_off[i + 1];
  r.B = a.bid[i];
#pragma unroll
  for (int k = 0; k < 9; ++k) r.R[k] = a.Rg[k * a.ns + r.B];
  r.shp = a.shp[r.B];
#pragma unroll
  for (int u = 0; u < BODY_ENT; ++u) r.ent[u] = r.e0 + u < r.e1 ? a.binc[r.e0 + u] : 0;
  return r;
}

// zw_i = diag4(R) Hbar^{-1} diag4(R^T) sum_k s J(p_k)^T (va_k + coef vb_k)
DEV void body_one(const PcgBallArgs &a, int i, const BodyRefs &br, const double *va, const double *vb,
                  double coef) {
  double g[12];
#pragma unroll
  for (int s = 0; s < 12; ++s) g[s] = 0.0;
  for (int e = br.e0; e < br.e1; ++e) {
    int ent = 0;
#pragma unroll
    for (int u = 0; u < BODY_ENT; ++u)
      if (e - br.e0 == u) ent = br.ent[u];
    if (e - br.e0 >= BODY_ENT) ent = a.binc[e];
    const int j = ent >> 1, side = ent & 1;
    const double sg = side ? -1.0 : 1.0;
    double v[3];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) {
      v[rr] = va[3 * (int64_t)j + rr];
      if (vb) v[rr] += coef * vb[3 * (int64_t)j + rr];
      v[rr] *= sg;
    }
    const double *pj = a.jp + 8 * (int64_t)j + 3 * side;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int rr = 0; rr < 3; ++rr) g[3 * c + rr] += pj[c] * v[rr];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) g[9 + rr] += v[rr];
  }
  const double *R = br.R;
  double gl_[12], zl[12];
#pragma unroll
  for (int c = 0; c < 4; ++c) mat3t_vec(R, g + 3 * c, gl_ + 3 * c);
  hinv_apply(a.hinv + (int64_t)HINV_STRIDE * br.shp, gl_, zl);
  double *zo = a.zw + 16 * (int64_t)i;
#pragma unroll
  for (int c = 0; c < 4; ++c) mat3_vec(R, zl + 3 * c, zo + 3 * c);
}

DEV void body_one(const PcgBallArgs &a, int i, const double *va, const double *vb, double coef) {
  body_one(a, i, body_refs(a, i), va, vb, coef);
}

// y = sum_sides s J(p) zw_b
DEV void joint_one(const PcgBallArgs &a, int j, double *y) {
  y[0] = y[1] = y[2] = 0.0;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int b = side ? a.jbb[j] : a.jba[j];
    if (b < 0) continue;
    const double sg = side ? -1.0 : 1.0;
    const double *pj = a.jp + 8 * (int64_t)j + 3 * side;
    const double *zb = a.zw + 16 * (int64_t)b;
#pragma unroll
    for (int rr = 0; rr < 3; ++rr)
      y[rr] += sg * (pj[0] * zb[rr] + pj[1] * zb[3 + rr] + pj[2] * zb[6 + rr] + zb[9 + rr]);
  }
}

DEV void precond(const double *Di, const double *rk, double *zk) {
  zk[0] = Di[0] * rk[0] + Di[1] * rk[1] + Di[2] * rk[2];
  zk[1] = Di[1] * rk[0] + Di[3] * rk[1] + Di[4] * rk[2];
  zk[2] = Di[2] * rk[0] + Di[4] * rk[1] + Di[5] * rk[2];
}

}  // namespace mabd
