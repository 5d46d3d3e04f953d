// Preconditioned conjugate gradients on the dual system S lambda = r of
// assemblies with closed loops (Secs. 5.4-5.5; Eq. dual with the -C of the
// footnote of Eq. kkt).  S is applied matrix-free,
//   S x = sum_b L_b Hbar_b^{-1} L_b^T x,
// as a body pass (z_b = Hbar^{-1} sum_k L_kb^T x_k) followed by a joint pass
// (y_k = sum_b L_kb z_b).  The preconditioner is block Jacobi with the exact
// diagonal blocks S_kk.  One persistent cooperative launch runs the whole
// solve: grid-wide barriers separate the passes, dot products are summed in
// a fixed order (block partials, then every block adds the partials in index
// order), so the iteration is deterministic and the convergence test
// |r| <= tol |b| is taken on the device by every block alike.
#include <hip/hip_cooperative_groups.h>

#include "common.hpp"
#include "dmath.hpp"
#include "generic.hpp"

namespace cg = cooperative_groups;

namespace mabd {



constexpr int PCG_THREADS = 256;

DEV int jrows(const GJoint *J, int k) { return joint_rows(J[k].type); }

// block-level sum of a per-thread value, result valid in thread 0
DEV double block_sum(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = PCG_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// x -> z_b = Hbar^{-1} sum_k L_kb^T x_k for bodies of graph components
DEV void body_pass(const PcgArgs &a, const double *x, int tid, int nth) {
  for (int i = tid; i < a.nb; i += nth) {
    const int64_t b = (int64_t)a.b0 + i;
    if (!a.bmask[b]) continue;
    double g[12];
    for (int s = 0; s < 12; ++s) g[s] = 0.0;
    for (int e = a.inc_off[b]; e < a.inc_off[b + 1]; ++e) {
      const int ent = a.inc[e];
      const int k = ent >> 1, side = ent & 1;
      const int c = jrows(a.J, k);
      const double *L = a.gl + (int64_t)GL_STRIDE * k + (side ? GL_LB : GL_LA);
      for (int rr = 0; rr < c; ++rr) {
        const double xv = x[5 * (int64_t)k + rr];
        for (int s = 0; s < 12; ++s) g[s] += L[12 * rr + s] * xv;
      }
    }
    double zz[12];
    hinv_apply(a.hinv + (int64_t)HINV_STRIDE * a.shp[b], g, zz);
    for (int s = 0; s < 12; ++s) a.zb[s * a.ns + b] = zz[s];
  }
}

// y_k = sum_b L_kb z_b
DEV void joint_pass_one(const PcgArgs &a, int k, double *y) {
  const GJoint &j = a.J[k];
  const int c = joint_rows(j.type);
  for (int rr = 0; rr < 5; ++rr) y[rr] = 0.0;
  for (int side = 0; side < 2; ++side) {
    const int64_t b = side ? j.sb : j.sa;
    if (b < 0) continue;
    const double *L = a.gl + (int64_t)GL_STRIDE * k + (side ? GL_LB : GL_LA);
    double zz[12];
    for (int s = 0; s < 12; ++s) zz[s] = a.zb[s * a.ns + b];
    for (int rr = 0; rr < c; ++rr) {
      double v = 0.0;
      for (int s = 0; s < 12; ++s) v += L[12 * rr + s] * zz[s];
      y[rr] += v;
    }
  }
}

DEV void precond(const PcgArgs &a, int k, const double *rk, double *zk) {
  const int c = jrows(a.J, k);
  const double *Di = a.dinv + 25 * (int64_t)k;
  for (int i = 0; i < 5; ++i) {
    double v = 0.0;
    if (i < c)
      for (int j = 0; j < c; ++j) v += Di[i * c + j] * rk[j];
    zk[i] = v;
  }
}

// fixed-order grid sum of the first `nv` partial slots
DEV void grid_sums(const PcgArgs &a, int nv, double *out) {
  for (int v = 0; v < nv; ++v) out[v] = 0.0;
  for (int blk = 0; blk < (int)gridDim.x; ++blk)
    for (int v = 0; v < nv; ++v) out[v] += a.partial[4 * blk + v];
}

__global__ __launch_bounds__(PCG_THREADS) void pcg_kernel(PcgArgs a) {
  __shared__ double sh[PCG_THREADS];
  cg::grid_group grid = cg::this_grid();
  if (skip_step(a.status, a.step)) return;  // uniform across the grid for this launch
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;

  // ---- setup: preconditioner blocks S_kk = sum_b L Hbar^{-1} L^T
  for (int k = tid; k < a.mj; k += nth) {
    if (!a.jmask[k]) continue;
    const GJoint &j = a.J[k];
    const int c = joint_rows(j.type);
    double D[25];
    for (int i = 0; i < 25; ++i) D[i] = 0.0;
    for (int side = 0; side < 2; ++side) {
      const int64_t b = side ? j.sb : j.sa;
      if (b < 0) continue;
      const double *L = a.gl + (int64_t)GL_STRIDE * k + (side ? GL_LB : GL_LA);
      const double *T = a.hinv + (int64_t)HINV_STRIDE * a.shp[b];
      for (int rr = 0; rr < c; ++rr) {
        double y[12];
        hinv_apply(T, L + 12 * rr, y);
        for (int q2 = 0; q2 < c; ++q2) {
          double v = 0.0;
          for (int s = 0; s < 12; ++s) v += L[12 * q2 + s] * y[s];
          D[q2 * c + rr] += v;
        }
      }
    }
    // invert by Cholesky
    double Lc[25];
    bool ok = true;
    for (int i = 0; i < c * c; ++i) Lc[i] = D[i];
    for (int jj = 0; jj < c && ok; ++jj) {
      double d = Lc[jj * c + jj];
      for (int kk = 0; kk < jj; ++kk) d -= Lc[jj * c + kk] * Lc[jj * c + kk];
      if (!(d > 0.0)) { ok = false; break; }
      d = sqrt(d);
      Lc[jj * c + jj] = d;
      for (int i = jj + 1; i < c; ++i) {
        double s = Lc[i * c + jj];
        for (int kk = 0; kk < jj; ++kk) s -= Lc[i * c + kk] * Lc[jj * c + kk];
        Lc[i * c + jj] = s / d;
      }
    }
    double *Di = a.dinv + 25 * (int64_t)k;
    if (!ok) {
      raise_flag(a.status, FLAG_SINGULAR, a.step);
      for (int i = 0; i < 25; ++i) Di[i] = 0.0;
    } else {
      for (int col = 0; col < c; ++col) {
        double x[5];
        for (int i = 0; i < c; ++i) {
          double s = (i == col) ? 1.0 : 0.0;
          for (int kk = 0; kk < i; ++kk) s -= Lc[i * c + kk] * x[kk];
          x[i] = s / Lc[i * c + i];
        }
        for (int i = c - 1; i >= 0; --i) {
          double s = x[i];
          for (int kk = i + 1; kk < c; ++kk) s -= Lc[kk * c + i] * x[kk];
          x[i] = s / Lc[i * c + i];
        }
        for (int i = 0; i < c; ++i) Di[i * c + col] = x[i];
      }
    }
  }
  // ---- right-hand side b = sum L u + C (kept in sp for now), and S lambda0
  for (int k = tid; k < a.mj; k += nth) {
    if (!a.jmask[k]) continue;
    const GJoint &j = a.J[k];
    const int c = joint_rows(j.type);
    double bk[5];
    for (int rr = 0; rr < c; ++rr) bk[rr] = a.gl[(int64_t)GL_STRIDE * k + GL_C + rr];
    for (int side = 0; side < 2; ++side) {
      const int64_t b = side ? j.sb : j.sa;
      if (b < 0) continue;
      const double *L = a.gl + (int64_t)GL_STRIDE * k + (side ? GL_LB : GL_LA);
      for (int rr = 0; rr < c; ++rr) {
        double v = 0.0;
        for (int s = 0; s < 12; ++s) v += L[12 * rr + s] * a.ug[s * a.ns + b];
        bk[rr] += v;
      }
    }
    for (int rr = 0; rr < 5; ++rr) {
      a.r[5 * (int64_t)k + rr] = rr < c ? bk[rr] : 0.0;
      a.bv[5 * (int64_t)k + rr] = rr < c ? bk[rr] : 0.0;
      if (!a.warm) a.lam[5 * (int64_t)k + rr] = 0.0;
    }
  }
  grid.sync();
  if (a.warm) body_pass(a, a.lam, tid, nth);
  grid.sync();
  // r = b - S lambda0 ; z = M^{-1} r ; p = z ; partials |b|^2, r.z, |r|^2
  double pb = 0.0, prz = 0.0, prr = 0.0;
  for (int k = tid; k < a.mj; k += nth) {
    if (!a.jmask[k]) continue;
    const int c = jrows(a.J, k);
    double y[5] = {0, 0, 0, 0, 0}, rk[5], zk[5];
    if (a.warm) joint_pass_one(a, k, y);
    for (int rr = 0; rr < 5; ++rr) {
      const double bv = a.r[5 * (int64_t)k + rr];
      pb += bv * bv;
      rk[rr] = bv - (rr < c ? y[rr] : 0.0);
    }
    precond(a, k, rk, zk);
    for (int rr = 0; rr < 5; ++rr) {
      a.r[5 * (int64_t)k + rr] = rk[rr];
      a.z[5 * (int64_t)k + rr] = zk[rr];
      a.p[5 * (int64_t)k + rr] = zk[rr];
      prz += rk[rr] * zk[rr];
      prr += rk[rr] * rk[rr];
    }
  }
  {
    double s0 = block_sum(pb, sh), s1 = block_sum(prz, sh), s2 = block_sum(prr, sh);
    if (threadIdx.x == 0) {
      a.partial[4 * blockIdx.x + 0] = s0;
      a.partial[4 * blockIdx.x + 1] = s1;
      a.partial[4 * blockIdx.x + 2] = s2;
    }
  }
  grid.sync();
  double tot[3];
  grid_sums(a, 3, tot);
  const double bnorm = sqrt(tot[0]);
  double rz = tot[1];
  double rnorm = sqrt(tot[2]);
  int it = 0;
  const double thresh = a.tol * bnorm;
  grid.sync();  // partials are rewritten below
  for (int restart = 0; restart < 4; ++restart) {
  while (rnorm > thresh && it < a.max_iters) {
    body_pass(a, a.p, tid, nth);
    grid.sync();
    double ppap = 0.0;
    for (int k = tid; k < a.mj; k += nth) {
      if (!a.jmask[k]) continue;
      double y[5];
      joint_pass_one(a, k, y);
      for (int rr = 0; rr < 5; ++rr) {
        a.sp[5 * (int64_t)k + rr] = y[rr];
        ppap += a.p[5 * (int64_t)k + rr] * y[rr];
      }
    }
    {
      double s0 = block_sum(ppap, sh);
      if (threadIdx.x == 0) a.partial[4 * blockIdx.x + 3] = s0;
    }
    grid.sync();
    double pap = 0.0;
    for (int blk = 0; blk < (int)gridDim.x; ++blk) pap += a.partial[4 * blk + 3];
    const double alpha = rz / pap;
    double prz2 = 0.0, prr2 = 0.0;
    for (int k = tid; k < a.mj; k += nth) {
      if (!a.jmask[k]) continue;
      double rk[5], zk[5];
      for (int rr = 0; rr < 5; ++rr) {
        a.lam[5 * (int64_t)k + rr] += alpha * a.p[5 * (int64_t)k + rr];
        rk[rr] = a.r[5 * (int64_t)k + rr] - alpha * a.sp[5 * (int64_t)k + rr];
        a.r[5 * (int64_t)k + rr] = rk[rr];
      }
      precond(a, k, rk, zk);
      for (int rr = 0; rr < 5; ++rr) {
        a.z[5 * (int64_t)k + rr] = zk[rr];
        prz2 += rk[rr] * zk[rr];
        prr2 += rk[rr] * rk[rr];
      }
    }
    {
      double s1 = block_sum(prz2, sh), s2 = block_sum(prr2, sh);
      if (threadIdx.x == 0) {
        a.partial[4 * blockIdx.x + 1] = s1;
        a.partial[4 * blockIdx.x + 2] = s2;
      }
    }
    grid.sync();
    double rz2 = 0.0, rr2 = 0.0;
    for (int blk = 0; blk < (int)gridDim.x; ++blk) {
      rz2 += a.partial[4 * blk + 1];
      rr2 += a.partial[4 * blk + 2];
    }
    const double beta = rz2 / rz;
    rz = rz2;
    rnorm = sqrt(rr2);
    for (int k = tid; k < a.mj; k += nth) {
      if (!a.jmask[k]) continue;
      for (int rr = 0; rr < 5; ++rr)
        a.p[5 * (int64_t)k + rr] = a.z[5 * (int64_t)k + rr] + beta * a.p[5 * (int64_t)k + rr];
    }
    ++it;
    grid.sync();
  }
  // The recursively updated residual drifts from b - S lambda; test the true
  // residual and, if it is above the tolerance, restart from it.
  if (it >= a.max_iters) break;
  body_pass(a, a.lam, tid, nth);
  grid.sync();
  double ptr = 0.0, ptz = 0.0;
  for (int k = tid; k < a.mj; k += nth) {
    if (!a.jmask[k]) continue;
    const int c = jrows(a.J, k);
    double y[5], rk[5], zk[5];
    joint_pass_one(a, k, y);
    for (int rr = 0; rr < 5; ++rr) rk[rr] = rr < c ? a.bv[5 * (int64_t)k + rr] - y[rr] : 0.0;
    precond(a, k, rk, zk);
    for (int rr = 0; rr < 5; ++rr) {
      a.r[5 * (int64_t)k + rr] = rk[rr];
      a.z[5 * (int64_t)k + rr] = zk[rr];
      a.p[5 * (int64_t)k + rr] = zk[rr];
      ptr += rk[rr] * rk[rr];
      ptz += rk[rr] * zk[rr];
    }
  }
  {
    double s1 = block_sum(ptz, sh), s2 = block_sum(ptr, sh);
    if (threadIdx.x == 0) {
      a.partial[4 * blockIdx.x + 1] = s1;
      a.partial[4 * blockIdx.x + 2] = s2;
    }
  }
  grid.sync();
  {
    double rz2 = 0.0, rr2 = 0.0;
    for (int blk = 0; blk < (int)gridDim.x; ++blk) {
      rz2 += a.partial[4 * blk + 1];
      rr2 += a.partial[4 * blk + 2];
    }
    rz = rz2;
    rnorm = sqrt(rr2);
  }
  grid.sync();
  if (rnorm <= thresh) break;
  }
  if (tid == 0) {
    *a.iters_out = it;
    *a.res_out = bnorm > 0.0 ? rnorm / bnorm : rnorm;
  }
  if (!(rnorm <= thresh) && tid == 0)
    raise_flag(a.status, isfinite(rnorm) ? FLAG_NOTCONV : FLAG_NONFINITE, a.step);
}

hipError_t launch_pcg(const PcgArgs &a, int nblocks, hipStream_t s) {
  void *args[] = {(void *)&a};
  return hipLaunchCooperativeKernel((const void *)pcg_kernel, dim3(nblocks), dim3(PCG_THREADS), args,
                                    0, s);
}

int pcg_max_blocks() {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)pcg_kernel, PCG_THREADS, 0) !=
      hipSuccess)
    return 0;
  return ncu * per;
}

}  // namespace mabd
