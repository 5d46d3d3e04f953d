// Preconditioned conjugate gradients on the dual system S lambda = r of
// ball-jointed networks (Secs. 5.4-5.5; Eq. dual with the -C of the footnote
// of Eq. kkt), as a sequence of ordinary launches.
//
// A ball row block of the dual is s J(p) in world coordinates (s = +1 for
// side a, -1 for side b, J(p) = [p^T (x) I3, I3], Eq. ball), so S v is a body
// pass zw_b = diag4(R_b) Hbar_b^{-1} diag4(R_b^T) sum_k s J(p_k)^T v_k followed
// by a joint pass (S v)_k = sum_b s J(p_k) zw_b.  The preconditioner is block
// Jacobi with the exact 3x3 diagonal blocks S_kk.
//
// One iteration is three launches (the launch boundary is the grid-wide
// barrier, far cheaper than a cooperative grid sync over many workgroups):
//   A: beta from the r.z partials of the previous C, convergence test, body
//      pass on p = z + beta p_prev;
//   B: p (stored), S p, partials of p.Sp;
//   C: alpha = r.z / p.Sp, x += alpha p, r -= alpha S p, z = M^{-1} r,
//      partials of r.z and r.r.
// Every workgroup sums the partials of the previous launch itself in a fixed
// order, so the iteration is deterministic.  The host launches iterations in
// chunks and reads the flags between chunks; once the recursive residual
// passes the test, the true residual b - S x is formed and the solve either
// ends or restarts from it (at most four restarts).
#include <algorithm>

#include "common.hpp"
#include "dmath.hpp"
#include "generic.hpp"
#include "ballop.hpp"

namespace mabd {

constexpr int PB_THREADS = 256;
// sc: [0] |b|, [1] tol |b|, [2..3] r.z of the last two iterations (by parity),
//     [4] r.r of the last test, [5] beta of the running iteration
enum { SC_BNORM = 0, SC_THRESH = 1, SC_RZ = 2, SC_RR = 4, SC_BETA = 5 };
// si: [0] done, [1] recursive residual below tol, [2] iterations,
//     [3] true residual below tol, [4] non-finite value met
enum { SI_DONE = 0, SI_CONV = 1, SI_ITERS = 2, SI_FINAL = 3, SI_BAD = 4 };

DEV double block_reduce(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = PB_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// fixed-order sum of one partial slot over all joint blocks (every thread
// gets the result); thread_partials is the per-thread part, so that its
// reads can be issued before a test that must precede the first barrier
DEV double thread_partials(const PcgBallArgs &a, int slot) {
  double v = 0.0;
  for (int b = threadIdx.x; b < a.nblk; b += PB_THREADS) v += a.partial[4 * (int64_t)b + slot];
  return v;
}
DEV double sum_partials(const PcgBallArgs &a, int slot, double *sh) {
  return block_reduce(thread_partials(a, slot), sh);
}

DEV void write_partial(const PcgBallArgs &a, int slot, double v, double *sh) {
  const double s = block_reduce(v, sh);
  if (threadIdx.x == 0) a.partial[4 * (int64_t)blockIdx.x + slot] = s;
}

// S_kk^{-1}, right-hand side b = sum s J(p) diag4(R) u + C, start value
__global__ __launch_bounds__(PB_THREADS) void pb_setup_kernel(PcgBallArgs a) {
  const int j = blockIdx.x * PB_THREADS + threadIdx.x;
  if (j >= a.nj || skip_step(a.status, a.step)) return;
  const int k = a.jid[j];
  double D[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, bk[3];
#pragma unroll
  for (int rr = 0; rr < 3; ++rr) bk[rr] = a.gl[(int64_t)GL_STRIDE * k + GL_C + rr];
  for (int side = 0; side < 2; ++side) {
    const int b = side ? a.jbb[j] : a.jba[j];
    if (b < 0) continue;
    const double sg = side ? -1.0 : 1.0;
    const int64_t B = a.bid[b];
    double R[9], pc[3], u[12];
#pragma unroll
    for (int q = 0; q < 9; ++q) R[q] = a.Rg[q * a.ns + B];
#pragma unroll
    for (int c = 0; c < 3; ++c) pc[c] = a.jp[8 * (int64_t)j + 3 * side + c];
#pragma unroll
    for (int q = 0; q < 12; ++q) u[q] = a.ug[q * a.ns + B];
    const double *T = a.hinv + (int64_t)HINV_STRIDE * a.shp[B];
    double W[9], RW[9];
    wblock(T, pc, pc, W);
    rot_congr(R, W, RW);
#pragma unroll
    for (int q = 0; q < 9; ++q) D[q] += RW[q];
    double Ju[3], v[3];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) Ju[rr] = pc[0] * u[rr] + pc[1] * u[3 + rr] + pc[2] * u[6 + rr] + u[9 + rr];
    mat3_vec(R, Ju, v);
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) bk[rr] += sg * v[rr];
  }
  D[1] = D[3] = 0.5 * (D[1] + D[3]);
  D[2] = D[6] = 0.5 * (D[2] + D[6]);
  D[5] = D[7] = 0.5 * (D[5] + D[7]);
  double Di[9];
  if (!spd3_inv(D, Di)) {
    raise_flag(a.status, FLAG_SINGULAR, a.step);
#pragma unroll
    for (int q = 0; q < 9; ++q) Di[q] = 0.0;
  }
  double *dj = a.dinv + 6 * (int64_t)j;
  dj[0] = Di[0]; dj[1] = Di[1]; dj[2] = Di[2]; dj[3] = Di[4]; dj[4] = Di[5]; dj[5] = Di[8];
#pragma unroll
  for (int rr = 0; rr < 3; ++rr) {
    a.bv[3 * (int64_t)j + rr] = bk[rr];
    a.x[3 * (int64_t)j + rr] = a.warm ? a.glam[5 * (int64_t)k + rr] : 0.0;
  }
}

// body pass on x (true residual, warm start)
__global__ __launch_bounds__(PB_THREADS) void pb_body_x_kernel(PcgBallArgs a) {
  const int i = blockIdx.x * PB_THREADS + threadIdx.x;
  if (i >= a.nbd || skip_step(a.status, a.step)) return;
  body_one(a, i, a.x, nullptr, 0.0);
}

// r = b - S x (use_x) or b, z = M^{-1} r, p_prev = 0; partials |b|^2, r.z, r.r
__global__ __launch_bounds__(PB_THREADS) void pb_init_kernel(PcgBallArgs a, int use_x) {
  __shared__ double sh[PB_THREADS];
  if (skip_step(a.status, a.step)) return;
  const int j = blockIdx.x * PB_THREADS + threadIdx.x;
  double pb = 0.0, prz = 0.0, prr = 0.0;
  if (j < a.nj) {
    double y[3] = {0.0, 0.0, 0.0}, rk[3], zk[3];
    if (use_x) joint_one(a, j, y);
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) {
      const double b = a.bv[3 * (int64_t)j + rr];
      pb += b * b;
      rk[rr] = b - y[rr];
    }
    precond(a.dinv + 6 * (int64_t)j, rk, zk);
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) {
      const int64_t o = 3 * (int64_t)j + rr;
      a.r[o] = rk[rr];
      a.z[o] = zk[rr];
      a.p0[o] = 0.0;
      a.p1[o] = 0.0;
      prz += rk[rr] * zk[rr];
      prr += rk[rr] * rk[rr];
    }
  }
  write_partial(a, 0, pb, sh);
  write_partial(a, 1, prz, sh);
  write_partial(a, 2, prr, sh);
}

// (re)start: norms and the test on the residual formed by pb_init (one block)
__global__ __launch_bounds__(PB_THREADS) void pb_start_kernel(PcgBallArgs a, int verify) {
  __shared__ double sh[PB_THREADS];
  if (skip_step(a.status, a.step)) return;
  const double bb = sum_partials(a, 0, sh), rz = sum_partials(a, 1, sh), rr = sum_partials(a, 2, sh);
  if (threadIdx.x != 0) return;
  if (!verify) {
    a.sc[SC_BNORM] = sqrt(bb);
    a.sc[SC_THRESH] = a.tol * sqrt(bb);
    a.si[SI_ITERS] = 0;
    a.si[SI_BAD] = 0;
  }
  a.sc[SC_RZ] = rz;
  a.sc[SC_RR] = rr;
  a.sc[SC_BETA] = 0.0;
  const double th = a.sc[SC_THRESH];
  const bool bad = !isfinite(rz) || !isfinite(rr);
  const bool conv = !bad && rr <= th * th;
  a.si[SI_CONV] = conv ? 1 : 0;
  a.si[SI_FINAL] = conv ? 1 : 0;
  a.si[SI_BAD] = bad ? 1 : 0;
  a.si[SI_DONE] = (conv || bad) ? 1 : 0;
}

// A: beta and the convergence test, then the body pass on p = z + beta p_prev
__global__ __launch_bounds__(PB_THREADS) void pb_iter_a_kernel(PcgBallArgs a, int par, int first) {
  __shared__ double sh[PB_THREADS];
  // the step gate, the done flag, the partials and the scalars go out
  // together; the flags are tested before the first barrier
  const StepGate gate = step_gate(a.status);
  const int done = a.si[SI_DONE];
  const double t1 = first ? 0.0 : thread_partials(a, 1), t2 = first ? 0.0 : thread_partials(a, 2);
  const double rzprev = a.sc[SC_RZ + (par ^ 1)], th = a.sc[SC_THRESH];
  const int i = blockIdx.x * PB_THREADS + threadIdx.x;
  BodyRefs br{};  // the body's own reads, independent of beta
  if (a.nbd > 0) br = body_refs(a, i < a.nbd ? i : 0);
  if (gate.skip() || done) return;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  double beta = 0.0;
  if (!first) {
    const double rz = block_reduce(t1, sh), rr = block_reduce(t2, sh);
    beta = rz / rzprev;
    const bool bad = !isfinite(rz) || !isfinite(rr) || !isfinite(beta);
    const bool conv = !bad && rr <= th * th;
    if (lead) {
      a.sc[SC_RZ + par] = rz;
      a.sc[SC_RR] = rr;
      a.sc[SC_BETA] = beta;
      if (conv) {
        a.si[SI_CONV] = 1;
        a.si[SI_DONE] = 1;
      } else if (bad) {
        a.si[SI_BAD] = 1;
        a.si[SI_DONE] = 1;
      } else if (a.si[SI_ITERS] >= a.max_iters) {
        a.si[SI_DONE] = 1;
      } else {
        a.si[SI_ITERS] += 1;
      }
    }
    if (conv || bad) return;
  } else if (lead) {
    a.sc[SC_BETA] = 0.0;
    if (a.si[SI_ITERS] >= a.max_iters) a.si[SI_DONE] = 1;
    else a.si[SI_ITERS] += 1;
  }
  if (i < a.nbd) body_one(a, i, br, a.z, par ? a.p1 : a.p0, beta);
}

// B: p = z + beta p_prev (stored), S p, partials of p.Sp
__global__ __launch_bounds__(PB_THREADS) void pb_iter_b_kernel(PcgBallArgs a, int par) {
  __shared__ double sh[PB_THREADS];
  // the step gate, flag and beta go out with the joint's own reads (end
  // bodies, anchors, z, p_prev); only the end bodies' zw wait for them
  const StepGate gate = step_gate(a.status);
  const int done = a.si[SI_DONE];
  const double beta = a.sc[SC_BETA];
  const double *pprev = par ? a.p1 : a.p0;
  double *pnext = par ? a.p0 : a.p1;
  const int j = blockIdx.x * PB_THREADS + threadIdx.x;
  const int64_t jc = j < a.nj ? j : 0;
  const int ba = a.jba[jc], bb = a.jbb[jc];
  double pj[6], zk[3], pk[3];
#pragma unroll
  for (int c = 0; c < 6; ++c) pj[c] = a.jp[8 * jc + c];
#pragma unroll
  for (int rr = 0; rr < 3; ++rr) {
    zk[rr] = a.z[3 * jc + rr];
    pk[rr] = pprev[3 * jc + rr];
  }
  if (gate.skip() || done) return;
  double ppap = 0.0;
  if (j < a.nj) {
    double y[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int b = side ? bb : ba;
      if (b < 0) continue;
      const double sg = side ? -1.0 : 1.0;
      const double *p = pj + 3 * side;
      const double *zb = a.zw + 16 * (int64_t)b;
#pragma unroll
      for (int rr = 0; rr < 3; ++rr)
        y[rr] += sg * (p[0] * zb[rr] + p[1] * zb[3 + rr] + p[2] * zb[6 + rr] + zb[9 + rr]);
    }
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) {
      const int64_t o = 3 * (int64_t)j + rr;
      const double pv = zk[rr] + beta * pk[rr];
      pnext[o] = pv;
      a.sp[o] = y[rr];
      ppap += pv * y[rr];
    }
  }
  write_partial(a, 3, ppap, sh);
}

// C: alpha, x and r updates, z = M^{-1} r, partials of r.z and r.r
__global__ __launch_bounds__(PB_THREADS) void pb_iter_c_kernel(PcgBallArgs a, int par) {
  __shared__ double sh[PB_THREADS];
  // the step gate, the done flag, the partials and this joint's vectors go
  // out together (none of them depends on alpha)
  const StepGate gate = step_gate(a.status);
  const int done = a.si[SI_DONE];
  const double rz = a.sc[SC_RZ + par], tp = thread_partials(a, 3);
  const double *pnext = par ? a.p0 : a.p1;
  const int j = blockIdx.x * PB_THREADS + threadIdx.x;
  const int64_t jc = j < a.nj ? j : 0;
  double pn[3], xo[3], ro[3], so[3], dv[6];
#pragma unroll
  for (int rr = 0; rr < 3; ++rr) {
    const int64_t o = 3 * jc + rr;
    pn[rr] = pnext[o];
    xo[rr] = a.x[o];
    ro[rr] = a.r[o];
    so[rr] = a.sp[o];
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) dv[q] = a.dinv[6 * jc + q];
  if (gate.skip() || done) return;
  const double alpha = rz / block_reduce(tp, sh);
  double prz = 0.0, prr = 0.0;
  if (j < a.nj) {
    double rk[3], zk[3];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) {
      const int64_t o = 3 * (int64_t)j + rr;
      a.x[o] = xo[rr] + alpha * pn[rr];
      rk[rr] = ro[rr] - alpha * so[rr];
      a.r[o] = rk[rr];
    }
    precond(dv, rk, zk);
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) {
      a.z[3 * (int64_t)j + rr] = zk[rr];
      prz += rk[rr] * zk[rr];
      prr += rk[rr] * rk[rr];
    }
  }
  write_partial(a, 1, prz, sh);
  write_partial(a, 2, prr, sh);
}

// multipliers out, iteration count, residual, failure flags
__global__ __launch_bounds__(PB_THREADS) void pb_finish_kernel(PcgBallArgs a) {
  if (skip_step(a.status, a.step)) return;
  const int j = blockIdx.x * PB_THREADS + threadIdx.x;
  if (j < a.nj) {
    const int k = a.jid[j];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) a.glam[5 * (int64_t)k + rr] = a.x[3 * (int64_t)j + rr];
    a.glam[5 * (int64_t)k + 3] = 0.0;
    a.glam[5 * (int64_t)k + 4] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double bn = a.sc[SC_BNORM], rn = sqrt(a.sc[SC_RR]);
    *a.iters_out = a.si[SI_ITERS];
    *a.res_out = bn > 0.0 ? rn / bn : rn;
    if (!a.si[SI_FINAL]) raise_flag(a.status, a.si[SI_BAD] ? FLAG_NONFINITE : FLAG_NOTCONV, a.step);
  }
}

static unsigned nblocks(int n) { return (unsigned)std::max(1, (n + PB_THREADS - 1) / PB_THREADS); }

void launch_pb_setup(const PcgBallArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(pb_setup_kernel, dim3(nblocks(a.nj)), dim3(PB_THREADS), 0, s, a);
}
void launch_pb_residual(const PcgBallArgs &a, int use_x, int verify, hipStream_t s) {
  if (use_x) hipLaunchKernelGGL(pb_body_x_kernel, dim3(nblocks(a.nbd)), dim3(PB_THREADS), 0, s, a);
  hipLaunchKernelGGL(pb_init_kernel, dim3(nblocks(a.nj)), dim3(PB_THREADS), 0, s, a, use_x);
  hipLaunchKernelGGL(pb_start_kernel, dim3(1), dim3(PB_THREADS), 0, s, a, verify);
}
void launch_pb_iters(const PcgBallArgs &a, int n, int first, hipStream_t s) {
  for (int i = 0; i < n; ++i) {
    const int par = i & 1;
    hipLaunchKernelGGL(pb_iter_a_kernel, dim3(nblocks(a.nbd)), dim3(PB_THREADS), 0, s, a, par,
                       (first && i == 0) ? 1 : 0);
    hipLaunchKernelGGL(pb_iter_b_kernel, dim3(nblocks(a.nj)), dim3(PB_THREADS), 0, s, a, par);
    hipLaunchKernelGGL(pb_iter_c_kernel, dim3(nblocks(a.nj)), dim3(PB_THREADS), 0, s, a, par);
  }
}
void launch_pb_finish(const PcgBallArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(pb_finish_kernel, dim3(nblocks(a.nj)), dim3(PB_THREADS), 0, s, a);
}

}  // namespace mabd
