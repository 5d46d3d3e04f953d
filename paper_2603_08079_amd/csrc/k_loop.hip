// Loop-breaker Schur complement of libmabd (Sec. 5, Case III, Eq. loop).
//
// A component with a few closed loops is split into a spanning tree of its
// joints (A) and the loop-closing joints (D).  Its dual system
//   [S_AA S_AD; S_DA S_DD] [l_A; l_D] = [r_A; r_D]
// is solved exactly through the small Schur complement
//   Sc = S_DD - S_DA S_AA^{-1} S_AD,   Sc l_D = r_D - S_DA S_AA^{-1} r_A,
//   l_A = S_AA^{-1} r_A - (S_AA^{-1} S_AD) l_D.
// S_AA^{-1} is applied by the tree contraction: once to r_A (the ordinary
// step), and once per loop row j to the column S_AD e_j, which is the dual
// right-hand side of the local increments u' = Hbar^{-1} L_D[j]^T at the two
// bodies of that loop row with zero constraint values (loop_inject_kernel
// prepares u', the tree solve runs with zero_c).  The rest is per component:
// loop_schur_kernel assembles and factors Sc (Cholesky, at most
// LOOP_MAX_ROWS rows) and loop_correct_kernel forms l_A.
#include "common.hpp"
#include "dmath.hpp"
#include "generic.hpp"

namespace mabd {

namespace {
constexpr int LNT = 64;

// local-frame row of joint k on side `side` (a: 0, b: 1), row r
__device__ inline const double *jrow(const double *gl, int k, int side, int r) {
  return gl + (int64_t)GL_STRIDE * k + (side ? GL_LB : GL_LA) + 12 * r;
}

// z_b = Hbar^{-1} sum over b's tree joints k of L_{k,b}^T w_k (body frame);
// jloop[k] == -2 marks the loop-closing joints, left out
__device__ void tree_force_solve(int64_t b, const int32_t *inc_off, const int32_t *inc, const GJoint *J,
                                 const double *gl, const int32_t *jloop, const double *w,
                                 const double *T, double *z) {
  double g[12];
  for (int i = 0; i < 12; ++i) g[i] = 0.0;
  for (int e = inc_off[b]; e < inc_off[b + 1]; ++e) {
    const int ent = inc[e];
    const int k = ent >> 1, side = ent & 1;
    if (jloop[k] == -2) continue;
    const int rows = joint_rows(J[k].type);
    for (int r = 0; r < rows; ++r) {
      const double l = w[5 * (int64_t)k + r];
      const double *L = jrow(gl, k, side, r);
      for (int i = 0; i < 12; ++i) g[i] += L[i] * l;
    }
  }
  hinv_apply(T, g, z);
}
}  // namespace

// u' of loop row j of every loop component (set = 1), or back to zero
// (set = 0), at the two bodies of that row's joint: Hbar^{-1} L^T of the row
__global__ __launch_bounds__(LNT) void loop_inject_kernel(int nloop, const int32_t *loff, const int32_t *lrow,
                                                          int j, const GJoint *J, const double *gl,
                                                          const int32_t *shp, const double *hinv, int64_t ns,
                                                          double *uloop, int set) {
  const int c = blockIdx.x * LNT + threadIdx.x;
  if (c >= nloop || j >= loff[c + 1] - loff[c]) return;
  const int32_t lr = lrow[loff[c] + j];
  const int k = lr >> 3, r = lr & 7;
  for (int side = 0; side < 2; ++side) {
    const int64_t b = side ? J[k].sb : J[k].sa;
    if (b < 0) continue;
    double z[12];
    if (set) {
      hinv_apply(hinv + (int64_t)HINV_STRIDE * shp[b], jrow(gl, k, side, r), z);
    } else {
      for (int i = 0; i < 12; ++i) z[i] = 0.0;
    }
    for (int i = 0; i < 12; ++i) uloop[i * ns + b] = z[i];
  }
}

// One workgroup per loop component: the Schur system of its loop rows from
// S_DD, S_DA W (W = S_AA^{-1} S_AD, column j in wcol + j * wstride) and
// r_D - S_DA l_A0 (l_A0 = S_AA^{-1} r_A in glam), its Cholesky solution l_D
// into lamD and glam.  A non-positive pivot raises FLAG_SINGULAR.
__global__ __launch_bounds__(LNT) void loop_schur_kernel(
    const int32_t *loff, const int32_t *lrow, const GJoint *J, const double *gl, const double *ug,
    const int32_t *shp, const double *hinv, int64_t ns, const int32_t *inc_off, const int32_t *inc,
    const int32_t *jloop, const double *wcol, int64_t wstride, double *glam, double *lamD,
    uint32_t *status) {
  __shared__ double Sc[LOOP_MAX_ROWS * LOOP_MAX_ROWS];
  __shared__ double rhs[LOOP_MAX_ROWS];
  if (skip_step(status, 0)) return;
  const int c = blockIdx.x, t = threadIdx.x;
  const int o = loff[c], nr = loff[c + 1] - o;
  // rows (i, j): S_DD, minus S_DA W; right-hand side column j = nr: r_D minus S_DA l_A0
  for (int idx = t; idx < nr * (nr + 1); idx += LNT) {
    const int i = idx / (nr + 1), jc = idx % (nr + 1);
    const int32_t li = lrow[o + i];
    const int ki = li >> 3, ri = li & 7;
    double v = 0.0;
    for (int side = 0; side < 2; ++side) {
      const int64_t b = side ? J[ki].sb : J[ki].sa;
      if (b < 0) continue;
      const double *T = hinv + (int64_t)HINV_STRIDE * shp[b];
      const double *Li = jrow(gl, ki, side, ri);
      double z[12];
      tree_force_solve(b, inc_off, inc, J, gl, jloop, jc < nr ? wcol + (int64_t)jc * wstride : glam, T, z);
      double sda = 0.0;
      for (int q = 0; q < 12; ++q) sda += Li[q] * z[q];
      v -= sda;
      if (jc < nr) {
        // S_DD entry through the bodies the two loop rows share
        const int32_t lj = lrow[o + jc];
        const int kj = lj >> 3, rj = lj & 7;
        for (int sj = 0; sj < 2; ++sj) {
          if ((sj ? J[kj].sb : J[kj].sa) != b) continue;
          double y[12];
          hinv_apply(T, jrow(gl, kj, sj, rj), y);
          for (int q = 0; q < 12; ++q) v += Li[q] * y[q];
        }
      } else {
        for (int q = 0; q < 12; ++q) v += Li[q] * ug[q * ns + b];
      }
    }
    if (jc < nr) Sc[i * LOOP_MAX_ROWS + jc] = v;
    else rhs[i] = v + gl[(int64_t)GL_STRIDE * ki + GL_C + ri];
  }
  __syncthreads();
  // Cholesky Sc = L L^T in place (lower triangle), then two triangular solves
  for (int p = 0; p < nr; ++p) {
    if (t == 0) {
      const double d = Sc[p * LOOP_MAX_ROWS + p];
      if (!(d > 0.0) || !isfinite(d)) raise_flag(status, FLAG_SINGULAR, 0);
      Sc[p * LOOP_MAX_ROWS + p] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const double piv = Sc[p * LOOP_MAX_ROWS + p];
    for (int i = p + 1 + t; i < nr; i += LNT) Sc[i * LOOP_MAX_ROWS + p] /= piv;
    __syncthreads();
    for (int idx = t; idx < (nr - p - 1) * (nr - p - 1); idx += LNT) {
      const int i = p + 1 + idx / (nr - p - 1), jj = p + 1 + idx % (nr - p - 1);
      if (jj <= i) Sc[i * LOOP_MAX_ROWS + jj] -= Sc[i * LOOP_MAX_ROWS + p] * Sc[jj * LOOP_MAX_ROWS + p];
    }
    __syncthreads();
  }
  if (t == 0) {
    double x[LOOP_MAX_ROWS];
    for (int i = 0; i < nr; ++i) {
      double s = rhs[i];
      for (int q = 0; q < i; ++q) s -= Sc[i * LOOP_MAX_ROWS + q] * x[q];
      x[i] = s / Sc[i * LOOP_MAX_ROWS + i];
    }
    for (int i = nr - 1; i >= 0; --i) {
      double s = x[i];
      for (int q = i + 1; q < nr; ++q) s -= Sc[q * LOOP_MAX_ROWS + i] * x[q];
      x[i] = s / Sc[i * LOOP_MAX_ROWS + i];
    }
    for (int i = 0; i < nr; ++i) {
      lamD[o + i] = x[i];
      const int32_t li = lrow[o + i];
      glam[5 * (int64_t)(li >> 3) + (li & 7)] = x[i];
    }
  }
}

// l_A = l_A0 - W l_D on the tree joints of the loop components (jloop[k] = c)
__global__ __launch_bounds__(256) void loop_correct_kernel(int mj, const int32_t *jloop, const int32_t *loff,
                                                           const double *wcol, int64_t wstride,
                                                           const double *lamD, double *glam,
                                                           const uint32_t *status) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= mj || skip_step(status, 0)) return;
  const int c = jloop[k];
  if (c < 0) return;
  const int o = loff[c], nr = loff[c + 1] - o;
  for (int r = 0; r < 5; ++r) {
    double v = glam[5 * (int64_t)k + r];
    for (int j = 0; j < nr; ++j) v -= wcol[(int64_t)j * wstride + 5 * (int64_t)k + r] * lamD[o + j];
    glam[5 * (int64_t)k + r] = v;
  }
}

void launch_loop_inject(int nloop, const int32_t *loff, const int32_t *lrow, int j, const GJoint *J,
                        const double *gl, const int32_t *shp, const double *hinv, int64_t ns, double *uloop,
                        int set, hipStream_t s) {
  if (nloop > 0)
    hipLaunchKernelGGL(loop_inject_kernel, dim3((nloop + LNT - 1) / LNT), dim3(LNT), 0, s, nloop, loff, lrow,
                       j, J, gl, shp, hinv, ns, uloop, set);
}

void launch_loop_schur(int nloop, const int32_t *loff, const int32_t *lrow, const GJoint *J, const double *gl,
                       const double *ug, const int32_t *shp, const double *hinv, int64_t ns,
                       const int32_t *inc_off, const int32_t *inc, const int32_t *jloop, const double *wcol,
                       int64_t wstride, double *glam, double *lamD, uint32_t *status, hipStream_t s) {
  if (nloop > 0)
    hipLaunchKernelGGL(loop_schur_kernel, dim3(nloop), dim3(LNT), 0, s, loff, lrow, J, gl, ug, shp, hinv, ns,
                       inc_off, inc, jloop, wcol, wstride, glam, lamD, status);
}

void launch_loop_correct(int mj, const int32_t *jloop, const int32_t *loff, const double *wcol, int64_t wstride,
                         const double *lamD, double *glam, const uint32_t *status, hipStream_t s) {
  if (mj > 0)
    hipLaunchKernelGGL(loop_correct_kernel, dim3((mj + 255) / 256), dim3(256), 0, s, mj, jloop, loff, wcol,
                       wstride, lamD, glam, status);
}

}  // namespace mabd
