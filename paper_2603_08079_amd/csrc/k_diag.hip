// Step diagnostics of libmabd: the FP64 KKT residual of a finished Newton
// iteration and the joint values at the state it produced.
//
// For the increment dq and multipliers lam of one iteration at the iterate q:
//   r_p = f_A - H dq - G^T lam    (primal rows of Eq. kkt),
//   r_d = G dq + C                (dual rows, with the -C of its footnote),
//   rho_p = |H^-1 r_p| / |H^-1 f_A|,  rho_d = |r_d| / |G H^-1 f_A + C|,
// and the largest |C| of the ball joints and of the hinges at q + dq.  Every
// block writes DIAG_PART partials (four sums, two maxima); diag_reduce_kernel
// combines them in a fixed order.  The chain rows' partials come from
// chain_resid_kernel in its diagnostics mode.
#include <mutex>

#include "common.hpp"
#include "dmath.hpp"
#include "generic.hpp"

namespace mabd {

namespace {
constexpr int DNT = 256;

// sums of v[0..3] and maxima of v[4..5] over the block, written by thread 0
__device__ void block_partials(const double v[DIAG_PART], double *out) {
  __shared__ double red[DIAG_PART][DNT];
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < DIAG_PART; ++k) red[k][t] = v[k];
  __syncthreads();
  for (int w = DNT / 2; w > 0; w /= 2) {
    if (t < w) {
#pragma unroll
      for (int k = 0; k < 4; ++k) red[k][t] += red[k][t + w];
      red[4][t] = fmax(red[4][t], red[4][t + w]);
      red[5][t] = fmax(red[5][t], red[5][t + w]);
    }
    __syncthreads();
  }
  if (t < DIAG_PART) out[t] = red[t][0];
}
}  // namespace

// Primal part, one generic body per thread.  q is the iterate the step's
// iteration started from, qn / qdn the state at the start of the step, and
// dq = dq_scale * dqv the iteration's increment (SoA, stride ns); Rg the
// iteration's rotations and gl / glam its joint rows and multipliers.
__global__ __launch_bounds__(DNT) void gdiag_body_kernel(
    int b0, int b1, const double *q, const double *qn, const double *qdn, const double *dqv,
    double dq_scale, int64_t ns, const int32_t *shp, const double *hinv, const double *shape,
    double g0, double g1, double g2, double h, const double *Rg, const int32_t *inc_off,
    const int32_t *inc, const GJoint *J, const double *gl, const double *glam, const double *wr,
    const uint32_t *status, double *part, int polar_free, double *ucorr) {
  const int64_t b = (int64_t)b0 + blockIdx.x * DNT + threadIdx.x;
  double v[DIAG_PART] = {0, 0, 0, 0, 0, 0};
  // refinement: a polar-free body takes no correction
  if (ucorr && b < b1 && polar_free && inc_off[b] == inc_off[b + 1] && !skip_step(status, 0))
    for (int i = 0; i < 12; ++i) ucorr[i * ns + b] = 0.0;
  // a body that took the polar-free solve does not solve the co-rotated
  // system of Eq. kkt: it is left out of rho_p
  const bool pf = b < b1 && polar_free && inc_off[b] == inc_off[b + 1];
  if (b < b1 && !pf && !skip_step(status, 0)) {
    double qq[12], qnn[12], qd[12], dq[12], A[9], R[9];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      qq[c] = q[c * ns + b];
      qnn[c] = qn[c * ns + b];
      qd[c] = qdn[c * ns + b];
      dq[c] = dq_scale * dqv[c * ns + b];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = Rg[i * ns + b];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) A[3 * i + c] = qq[3 * c + i];
    const int s = shp[b];
    const double *sh = shape + (int64_t)SHAPE_STRIDE * s;
    const double *T = hinv + (int64_t)HINV_STRIDE * s;
    const double g[3] = {g0, g1, g2};
    double phi[12], u[12], dl[12], Hd[12];
    local_force<double>(sh, R, A, qq, qnn, qd, g, h, phi, wr, ns, b);
    hinv_apply(T, phi, u);
    // body frame: r = phi - Hbar R^T dq - sum L^T lam
#pragma unroll
    for (int c = 0; c < 4; ++c) mat3t_vec(R, dq + 3 * c, dl + 3 * c);
    hbar_apply(sh, h, dl, Hd);
    double r[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) r[i] = phi[i] - Hd[i];
    for (int e = inc_off[b]; e < inc_off[b + 1]; ++e) {
      const int ent = inc[e];
      const int k = ent >> 1, side = ent & 1;
      const int rows = joint_rows(J[k].type);
      const double *L = gl + (int64_t)GL_STRIDE * k + (side ? GL_LB : GL_LA);
      for (int rr = 0; rr < rows; ++rr) {
        const double lr = glam[5 * (int64_t)k + rr];
        for (int i = 0; i < 12; ++i) r[i] -= L[12 * rr + i] * lr;
      }
    }
    double y[12];
    hinv_apply(T, r, y);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      v[0] += y[i] * y[i];
      v[1] += u[i] * u[i];
    }
    // refinement: the correction's local solve Hbar^{-1} R^T r_p (body frame),
    // the right-hand side in place of u
    if (ucorr)
#pragma unroll
      for (int i = 0; i < 12; ++i) ucorr[i * ns + b] = y[i];
  }
  block_partials(v, part + DIAG_PART * (int64_t)blockIdx.x);
}

// max |row value| of a rotated-frame joint of type TYPE at the new state
// (Eqs. hinge, universal, prismatic): row i is component comp of
// R_J (y_X - y_Y); the row loop is unrolled over the compile-time table.
template <int TYPE>
DEV double rot_joint_value(const GJoint &j, const double *Aa, const double *ta, const double *Ab,
                           const double *tb, const double *RH) {
  const double *P[5] = {j.p1a, j.p2a, j.p1b, j.p2b, j.p3b};
  constexpr int ROWS = TYPE == 2 ? 4 : 5;
  double v = 0.0;
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const JointRow jr = joint_row(TYPE, i);
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
    v = fmax(v, fabs(rh[0] * d[0] + rh[1] * d[1] + rh[2] * d[2]));
  }
  return v;
}

// Dual part and joint values, one generic joint per thread.  gl holds the
// iteration's rows L = G diag4(R) and C, ug its local increments
// u = Hbar^-1 diag4(R^T) f_A, Rg its rotations; dq as above; q_new the state
// the iteration produced.
__global__ __launch_bounds__(DNT) void gdiag_joint_kernel(
    int m, const GJoint *J, const double *gl, const double *Rg, const double *ug,
    const double *dqv, double dq_scale, const double *q_new, int64_t ns, const uint32_t *status,
    double *part, double *ccorr) {
  const int k = blockIdx.x * DNT + threadIdx.x;
  double v[DIAG_PART] = {0, 0, 0, 0, 0, 0};
  if (k < m && !skip_step(status, 0)) {
    const GJoint j = J[k];
    const int rows = joint_rows(j.type);
    const double *G = gl + (int64_t)GL_STRIDE * k;
    double rd[5], rr[5];
    for (int i = 0; i < rows; ++i) rd[i] = rr[i] = G[GL_C + i];
    double An[2][9], tn[2][3];
    for (int side = 0; side < 2; ++side) {
      const int64_t b = side == 0 ? j.sa : j.sb;
      if (b < 0) {
        for (int i = 0; i < 9; ++i) An[side][i] = (i % 4 == 0) ? 1.0 : 0.0;
        tn[side][0] = tn[side][1] = tn[side][2] = 0.0;
        continue;
      }
      double R[9], dq[12], dl[12], u[12];
      for (int i = 0; i < 9; ++i) R[i] = Rg[i * ns + b];
      for (int c = 0; c < 12; ++c) {
        dq[c] = dq_scale * dqv[c * ns + b];
        u[c] = ug[c * ns + b];
      }
      for (int c = 0; c < 4; ++c) mat3t_vec(R, dq + 3 * c, dl + 3 * c);
      const double *L = G + (side ? GL_LB : GL_LA);
      for (int i = 0; i < rows; ++i) {
        double sd = 0.0, su = 0.0;
        for (int c = 0; c < 12; ++c) {
          sd += L[12 * i + c] * dl[c];
          su += L[12 * i + c] * u[c];
        }
        rd[i] += sd;
        rr[i] += su;
      }
      for (int i = 0; i < 3; ++i) {
        for (int c = 0; c < 3; ++c) An[side][3 * i + c] = q_new[(3 * c + i) * ns + b];
        tn[side][i] = q_new[(9 + i) * ns + b];
      }
    }
    for (int i = 0; i < rows; ++i) {
      v[2] += rr[i] * rr[i];
      v[3] += rd[i] * rd[i];
    }
    // refinement: the correction solves G ddq = -r_d, i.e. the dual system
    // with r_d in place of C
    if (ccorr)
      for (int i = 0; i < 5; ++i) ccorr[5 * (int64_t)k + i] = i < rows ? rd[i] : 0.0;
    // joint values at the new state (Eq. ball; Eqs. hinge, universal,
    // prismatic with R_J from the polar rotation of side a's new affine block)
    auto point_diff = [&](const double *pa_, const double *pb_, double *d) {
      double wa[3], wb[3];
      mat3_vec(An[0], pa_, wa);
      mat3_vec(An[1], pb_, wb);
      for (int i = 0; i < 3; ++i) d[i] = (tn[0][i] - tn[1][i]) + (wa[i] - wb[i]);
    };
    if (j.type == 0) {
      double d1[3];
      point_diff(j.p1a, j.p1b, d1);
      v[4] = fmax(fabs(d1[0]), fmax(fabs(d1[1]), fabs(d1[2])));
    } else {
      double RH[9];
      if (j.flags & GJ_FLAG_STATIC_OWNER) {
        for (int i = 0; i < 9; ++i) RH[i] = j.dR[i];
      } else {
        double Ra[9];
        if (!polar3(An[0], Ra))
          for (int i = 0; i < 9; ++i) Ra[i] = (i % 4 == 0) ? 1.0 : 0.0;
        mat3_mul_bt(j.dR, Ra, RH);
      }
      v[5] = j.type == 1   ? rot_joint_value<1>(j, An[0], tn[0], An[1], tn[1], RH)
             : j.type == 2 ? rot_joint_value<2>(j, An[0], tn[0], An[1], tn[1], RH)
                           : rot_joint_value<3>(j, An[0], tn[0], An[1], tn[1], RH);
    }
  }
  block_partials(v, part + DIAG_PART * (int64_t)blockIdx.x);
}

// out = {rho_p, rho_d, max(rho_p, rho_d), max |C| ball, max |C| hinge} from
// nblk partial records, summed in a fixed order (deterministic)
__global__ __launch_bounds__(DNT) void diag_reduce_kernel(const double *part, int nblk, double *out,
                                                          const uint32_t *status) {
  if (skip_step(status, 0)) return;
  double v[DIAG_PART] = {0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblk; b += DNT) {
    const double *p = part + DIAG_PART * (int64_t)b;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += p[k];
    v[4] = fmax(v[4], p[4]);
    v[5] = fmax(v[5], p[5]);
  }
  __shared__ double tot[DIAG_PART];
  block_partials(v, tot);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double rp = tot[1] > 0.0 ? sqrt(tot[0] / tot[1]) : sqrt(tot[0]);
    const double rd = tot[2] > 0.0 ? sqrt(tot[3] / tot[2]) : sqrt(tot[3]);
    out[0] = rp;
    out[1] = rd;
    out[2] = rp > rd ? rp : rd;
    out[3] = tot[4];
    out[4] = tot[5];
  }
}

int diag_body_blocks(int nb) { return (nb + DNT - 1) / DNT; }

void launch_gdiag_body(int b0, int b1, const double *q, const double *qn, const double *qdn,
                       const double *dqv, double dq_scale, int64_t ns, const int32_t *shp,
                       const double *hinv, const double *shape, const double *g, double h,
                       const double *Rg, const int32_t *inc_off, const int32_t *inc, const GJoint *J,
                       const double *gl, const double *glam, const double *wr, const uint32_t *status,
                       double *part, int polar_free, double *ucorr, hipStream_t s) {
  if (b1 <= b0) return;
  hipLaunchKernelGGL(gdiag_body_kernel, dim3(diag_body_blocks(b1 - b0)), dim3(DNT), 0, s, b0, b1, q,
                     qn, qdn, dqv, dq_scale, ns, shp, hinv, shape, g[0], g[1], g[2], h, Rg, inc_off,
                     inc, J, gl, glam, wr, status, part, polar_free, ucorr);
}

void launch_gdiag_joint(int m, const GJoint *J, const double *gl, const double *Rg, const double *ug,
                        const double *dqv, double dq_scale, const double *q_new, int64_t ns,
                        const uint32_t *status, double *part, double *ccorr, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(gdiag_joint_kernel, dim3(diag_body_blocks(m)), dim3(DNT), 0, s, m, J, gl, Rg, ug,
                     dqv, dq_scale, q_new, ns, status, part, ccorr);
}

void launch_diag_reduce(const double *part, int nblk, double *out, const uint32_t *status,
                        hipStream_t s) {
  hipLaunchKernelGGL(diag_reduce_kernel, dim3(1), dim3(DNT), 0, s, part, nblk, out, status);
}


// ------------------------------------------------------------------
// Twist and joint-wrench diagnostics.  The twist of a body is
// V = G(A) qdot = [1/2 sum_c a_c x adot_c; tdot] (Eq. module1-G-twist).  The
// joint wrench is the spatial wrench about the centre of mass, world frame,
// that does the same virtual work on rigid motions as the body's generalised
// joint force f = -sum_k G_kb^T lambda_k of the last step, W = E(A)^T f =
// [sum_c a_c x f_c; f_t] with the rigid-motion embedding E(A) of Eq.
// module2-E, taken at the state the step started from (where G was
// evaluated).  Outputs are AoS n x 6 in input body order.

namespace {
__device__ void wrench_of(const double *q, int64_t ns, int64_t b, const double *f, double *w) {
  w[0] = w[1] = w[2] = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double a0 = q[(3 * c) * ns + b], a1 = q[(3 * c + 1) * ns + b], a2 = q[(3 * c + 2) * ns + b];
    w[0] += a1 * f[3 * c + 2] - a2 * f[3 * c + 1];
    w[1] += a2 * f[3 * c + 0] - a0 * f[3 * c + 2];
    w[2] += a0 * f[3 * c + 1] - a1 * f[3 * c + 0];
  }
  w[3] = f[9];
  w[4] = f[10];
  w[5] = f[11];
}
}  // namespace

__global__ __launch_bounds__(DNT) void twist_kernel(int nd, const int32_t *sol2in, const double *q,
                                                    const double *qd, int64_t ns, double *V) {
  const int64_t b = (int64_t)blockIdx.x * DNT + threadIdx.x;
  if (b >= nd) return;
  double w[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double a0 = q[(3 * c) * ns + b], a1 = q[(3 * c + 1) * ns + b], a2 = q[(3 * c + 2) * ns + b];
    const double d0 = qd[(3 * c) * ns + b], d1 = qd[(3 * c + 1) * ns + b], d2 = qd[(3 * c + 2) * ns + b];
    w[0] += 0.5 * (a1 * d2 - a2 * d1);
    w[1] += 0.5 * (a2 * d0 - a0 * d2);
    w[2] += 0.5 * (a0 * d1 - a1 * d0);
  }
  double *o = V + 6 * (int64_t)sol2in[b];
  o[0] = w[0];
  o[1] = w[1];
  o[2] = w[2];
  o[3] = qd[9 * ns + b];
  o[4] = qd[10 * ns + b];
  o[5] = qd[11 * ns + b];
}

// chain bodies: body p of a chain sits between rows p + hl - 1 (of which it
// is the right end) and p + hl (left end); a ball row's block on an end is
// s J(p) in world coordinates, s = +1 on the joint's side a
__global__ __launch_bounds__(DNT) void chain_wrench_kernel(const ChainDesc *chains, int nchains, int nb_total,
                                                           const double *q, int64_t ns, const double *pl,
                                                           const double *pr, const uint8_t *flag,
                                                           int64_t nrs, const double *lam,
                                                           const int32_t *sol2in, double *W) {
  const int b = blockIdx.x * DNT + threadIdx.x;
  if (b >= nb_total) return;
  int lo = 0, hi = nchains - 1;  // last chain with body0 <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (chains[mid].body0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const ChainDesc cd = chains[lo];
  const int p = b - cd.body0;
  double f[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) f[i] = 0.0;
  for (int e = 0; e < 2; ++e) {
    const int r = p + cd.hl - 1 + e;  // e = 0: the row on the left, 1: on the right
    if (r < 0 || r >= cd.K) continue;
    const int64_t gr = (int64_t)cd.row0 + r;
    const double *P = e == 0 ? pr : pl;
    const double s = (flag[gr] & (e == 0 ? 2 : 1)) ? 1.0 : -1.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double l = s * lam[3 * gr + i];
#pragma unroll
      for (int c = 0; c < 3; ++c) f[3 * c + i] -= P[c * nrs + gr] * l;
      f[9 + i] -= l;
    }
  }
  wrench_of(q, ns, b, f, W + 6 * (int64_t)sol2in[b]);
}

// generic bodies: f = -diag4(R) sum L^T lambda over the incident joints
__global__ __launch_bounds__(DNT) void gwrench_kernel(int b0, int b1, const double *q, int64_t ns,
                                                      const double *Rg, const int32_t *inc_off,
                                                      const int32_t *inc, const GJoint *J,
                                                      const double *gl, const double *glam,
                                                      const int32_t *sol2in, double *W) {
  const int64_t b = (int64_t)b0 + blockIdx.x * DNT + threadIdx.x;
  if (b >= b1) return;
  double g[12], f[12], R[9];
#pragma unroll
  for (int i = 0; i < 12; ++i) g[i] = 0.0;
  for (int e = inc_off[b]; e < inc_off[b + 1]; ++e) {
    const int ent = inc[e];
    const int k = ent >> 1, side = ent & 1;
    const int rows = joint_rows(J[k].type);
    const double *L = gl + (int64_t)GL_STRIDE * k + (side ? GL_LB : GL_LA);
    for (int r = 0; r < rows; ++r) {
      const double l = glam[5 * (int64_t)k + r];
      for (int i = 0; i < 12; ++i) g[i] += L[12 * r + i] * l;
    }
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) R[i] = Rg[i * ns + b];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double w[3];
    mat3_vec(R, g + 3 * c, w);
#pragma unroll
    for (int i = 0; i < 3; ++i) f[3 * c + i] = -w[i];
  }
  wrench_of(q, ns, b, f, W + 6 * (int64_t)sol2in[b]);
}

void launch_twists(int nd, const int32_t *sol2in, const double *q, const double *qd, int64_t ns,
                   double *V, hipStream_t s) {
  if (nd > 0)
    hipLaunchKernelGGL(twist_kernel, dim3(diag_body_blocks(nd)), dim3(DNT), 0, s, nd, sol2in, q, qd, ns,
                       V);
}

void launch_joint_wrenches(const ChainDesc *chains, int nchains, int nchain_bodies, const double *pl,
                           const double *pr, const uint8_t *flag, int64_t nrs, const double *clam,
                           int b0, int b1, const double *Rg, const int32_t *inc_off, const int32_t *inc,
                           const GJoint *J, const double *gl, const double *glam, const double *q,
                           int64_t ns, const int32_t *sol2in, double *W, hipStream_t s) {
  if (nchains > 0 && nchain_bodies > 0)
    hipLaunchKernelGGL(chain_wrench_kernel, dim3(diag_body_blocks(nchain_bodies)), dim3(DNT), 0, s,
                       chains, nchains, nchain_bodies, q, ns, pl, pr, flag, nrs, clam, sol2in, W);
  if (b1 > b0)
    hipLaunchKernelGGL(gwrench_kernel, dim3(diag_body_blocks(b1 - b0)), dim3(DNT), 0, s, b0, b1, q, ns,
                       Rg, inc_off, inc, J, gl, glam, sol2in, W);
}

// ---------------------------------------------------------------------------
// Fixed device scratch of mabd_residual_noalloc: RESID_STATIC_BLOCKS partial
// records of DIAG_PART doubles (3 MiB), one copy on every device the library
// runs on, held until the process ends.  In host code the name `scratch` is a
// host-side stand-in, not a device address: the address of a device's copy
// comes from hipGetSymbolAddress, looked up once per device with that device
// current (resid_scratch), and only that address is passed to kernels.
constexpr int RESID_STATIC_BLOCKS = 65536;
constexpr int RESID_MAX_DEVICES = 64;
static __device__ __align__(256) double scratch[(size_t)RESID_STATIC_BLOCKS * DIAG_PART];

int resid_static_blocks() { return RESID_STATIC_BLOCKS; }

// Device address of the current device's copy of `scratch` (device index
// `device`, which must be current).
hipError_t resid_scratch(int device, double **out) {
  static std::mutex mu;
  static double *ptr[RESID_MAX_DEVICES] = {};
  if (device < 0 || device >= RESID_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptr[device] = static_cast<double *>(p);
  }
  *out = ptr[device];
  return hipSuccess;
}

}  // namespace mabd
