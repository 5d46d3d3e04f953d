// Learned warm start of the ball-network PCG: forward pass, energy loss,
// backward pass and Adam, all on the GPU in FP32 (the network) and FP64 (the
// dual operator and the loss).  The network and the loss are described in
// gnn.hpp.  Every reduction (body sums, weight gradients, scalar sums) runs
// over CSR lists or per-block partials in a fixed order: no float atomics, so
// training is deterministic.
#include <algorithm>

#include "ballop.hpp"
#include "common.hpp"
#include "generic.hpp"
#include "gnn.hpp"

namespace mabd {

constexpr int GT = 256;  // threads of the elementwise kernels

DEV double gnn_block_sum(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = GT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

DEV int body_deg(const PcgBallArgs &a, int b) { return b < 0 ? 0 : a.binc_off[b + 1] - a.binc_off[b]; }
DEV float joint_norm(const PcgBallArgs &a, int j) {
  return 1.0f / (float)max(1, body_deg(a, a.jba[j]) + body_deg(a, a.jbb[j]));
}

// ---------------------------------------------------------------- features
// base start lambda_b (previous multipliers or zero) into g.lb and a.x, so
// that a body pass can form S lambda_b
__global__ __launch_bounds__(GT) void gnn_base_kernel(PcgBallArgs a, GnnBufs g, int have_prev) {
  const int j = blockIdx.x * GT + threadIdx.x;
  if (j >= a.nj) return;
  const int k = a.jid[j];
  for (int r = 0; r < 3; ++r) {
    const double v = have_prev ? a.glam[5 * (int64_t)k + r] : 0.0;
    g.lb[3 * (int64_t)j + r] = v;
    a.x[3 * (int64_t)j + r] = v;
  }
}

// r_b = b - S lambda_b (S lambda_b from the body pass on a.x when have_prev);
// partials of |D^{-1} r_b|^2, r_b^T D^{-1} r_b and |lambda_b|^2
__global__ __launch_bounds__(GT) void gnn_feat_a_kernel(PcgBallArgs a, GnnBufs g, int have_prev) {
  __shared__ double sh[GT];
  const int j = blockIdx.x * GT + threadIdx.x;
  double zz = 0.0, rz = 0.0, ll = 0.0;
  if (j < a.nj) {
    double y[3] = {0.0, 0.0, 0.0}, rb[3], z[3];
    if (have_prev) joint_one(a, j, y);
    for (int r = 0; r < 3; ++r) {
      rb[r] = a.bv[3 * (int64_t)j + r] - y[r];
      g.rb[3 * (int64_t)j + r] = rb[r];
      const double l = g.lb[3 * (int64_t)j + r];
      ll += l * l;
    }
    precond(a.dinv + 6 * (int64_t)j, rb, z);
    for (int r = 0; r < 3; ++r) {
      zz += z[r] * z[r];
      rz += rb[r] * z[r];
    }
  }
  const double s0 = gnn_block_sum(zz, sh), s1 = gnn_block_sum(rz, sh), s2 = gnn_block_sum(ll, sh);
  if (threadIdx.x == 0) {
    g.red[4 * (int64_t)blockIdx.x + 0] = s0;
    g.red[4 * (int64_t)blockIdx.x + 1] = s1;
    g.red[4 * (int64_t)blockIdx.x + 3] = s2;
  }
}

// one block: s, E_ref and s_l from the partials
__global__ __launch_bounds__(GT) void gnn_feat_reduce_kernel(int nj, int nblk, GnnBufs g) {
  __shared__ double sh[GT];
  double a0 = 0.0, a1 = 0.0, a3 = 0.0;
  for (int b = threadIdx.x; b < nblk; b += GT) {
    a0 += g.red[4 * (int64_t)b + 0];
    a1 += g.red[4 * (int64_t)b + 1];
    a3 += g.red[4 * (int64_t)b + 3];
  }
  const double zz = gnn_block_sum(a0, sh), rz = gnn_block_sum(a1, sh), ll = gnn_block_sum(a3, sh);
  if (threadIdx.x == 0) {
    const double s = sqrt(zz / (double)max(nj, 1)), sl = sqrt(ll / (double)max(nj, 1));
    g.sc[0] = s > 0.0 ? s : 1.0;
    g.sc[1] = fabs(rz) > 0.0 ? fabs(rz) : 1.0;
    g.sc[4] = sl > 0.0 ? sl : 1.0;
  }
}

__global__ __launch_bounds__(GT) void gnn_feat_b_kernel(PcgBallArgs a, GnnBufs g, int have_prev) {
  const int j = blockIdx.x * GT + threadIdx.x;
  if (j >= a.nj) return;
  const double is = 1.0 / g.sc[0], isl = 1.0 / g.sc[4];
  double rb[3], z[3];
  for (int r = 0; r < 3; ++r) rb[r] = g.rb[3 * (int64_t)j + r];
  precond(a.dinv + 6 * (int64_t)j, rb, z);
  float *x = g.x0 + (int64_t)GNN_FIN * j;
  for (int r = 0; r < 3; ++r) {
    x[r] = (float)(z[r] * is);
    x[3 + r] = (float)(g.lb[3 * (int64_t)j + r] * isl);
  }
  x[6] = 0.25f * (float)body_deg(a, a.jba[j]);
  x[7] = 0.25f * (float)body_deg(a, a.jbb[j]);
  x[8] = a.jba[j] < 0 ? 1.0f : 0.0f;
  x[9] = a.jbb[j] < 0 ? 1.0f : 0.0f;
  x[10] = have_prev ? 1.0f : 0.0f;
  for (int r = 11; r < GNN_FIN; ++r) x[r] = 0.0f;
}

// ----------------------------------------------------------- dense layers
// Y[N x NO] = X[N x K] W + c, then relu (RELU) or masked by M > 0 (MASK).
// W is [K][NO] row-major, or given as [NO][K] (TW: the transposed product).
// GR rows per workgroup, 16 outputs per thread, X and W staged in LDS (X rows
// padded to K + 1 floats against bank conflicts).
constexpr int GR = 32;
template <int K, int NO, bool RELU, bool TW, bool MASK>
__global__ __launch_bounds__(GR * NO / 16) void gnn_gemm_kernel(const float *X, const float *W, const float *c,
                                                               const float *M, float *Y, int N) {
  constexpr int G = NO / 16, NT = GR * G, KP = K + 1;
  __shared__ float Xs[GR * KP];
  __shared__ float Ws[K * NO];
  const int r0 = blockIdx.x * GR;
  for (int i = threadIdx.x; i < K * NO; i += NT) {
    const int k = i / NO, o = i % NO;
    Ws[i] = TW ? W[o * K + k] : W[i];
  }
  for (int i = threadIdx.x; i < GR * K; i += NT) {
    const int r = i / K, k = i % K;
    Xs[r * KP + k] = (r0 + r < N) ? X[(int64_t)(r0 + r) * K + k] : 0.0f;
  }
  __syncthreads();
  const int r = threadIdx.x / G, cg = threadIdx.x % G;
  float acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = c ? c[cg * 16 + q] : 0.0f;
  for (int k = 0; k < K; ++k) {
    const float xv = Xs[r * KP + k];
    const float *wr = Ws + k * NO + cg * 16;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] += xv * wr[q];
  }
  const int row = r0 + r;
  if (row >= N) return;
  float *yr = Y + (int64_t)row * NO + cg * 16;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    float v = acc[q];
    if (RELU) v = v > 0.0f ? v : 0.0f;
    if (MASK) v = M[(int64_t)row * NO + cg * 16 + q] > 0.0f ? v : 0.0f;
    yr[q] = v;
  }
}

// The same product on the matrix cores: v_mfma_f32_16x16x4_f32 takes a
// 16 x 4 block of A (lane l: row l mod 16, column l / 16), a 4 x 16 block of
// B (lane l: row l / 16, column l mod 16) and accumulates the 16 x 16 block
// of D in four registers (lane l, register j: row 4 (l / 16) + j, column
// l mod 16).  A workgroup of four waves takes 64 rows; each wave its 16 rows
// times all NO outputs (NO / 16 blocks), K / 4 steps of the contraction.
// X (rows padded to K + 1 floats) and W are staged in LDS.
typedef float gnn_v4f __attribute__((ext_vector_type(4)));
constexpr int MR = 64;  // rows per workgroup of the MFMA kernels
template <int K, int NO, bool RELU, bool TW, bool MASK>
__global__ __launch_bounds__(256) void gnn_mfma_gemm_kernel(const float *X, const float *W, const float *c,
                                                            const float *M, float *Y, int N) {
  static_assert(K % 4 == 0 && NO % 16 == 0, "MFMA blocks");
  constexpr int KP = K + 1, NB = NO / 16;
  __shared__ float Xs[MR * KP];
  __shared__ float Ws[K * NO];
  const int r0 = blockIdx.x * MR;
  for (int i = threadIdx.x; i < K * NO; i += 256) {
    const int k = i / NO, o = i % NO;
    Ws[i] = TW ? W[o * K + k] : W[i];
  }
  for (int i = threadIdx.x; i < MR * K; i += 256) {
    const int r = i / K, k = i % K;
    Xs[r * KP + k] = (r0 + r < N) ? X[(int64_t)(r0 + r) * K + k] : 0.0f;
  }
  __syncthreads();
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  const int ar = w * 16 + (l & 15), kq = l >> 4;
  gnn_v4f acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = gnn_v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 4
  for (int k0 = 0; k0 < K; k0 += 4) {
    const float a = Xs[ar * KP + k0 + kq];
#pragma unroll
    for (int b = 0; b < NB; ++b)
      acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, Ws[(k0 + kq) * NO + b * 16 + (l & 15)], acc[b], 0, 0, 0);
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int col = b * 16 + (l & 15);
    const float cv = c ? c[col] : 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = r0 + w * 16 + 4 * kq + j;
      if (row < N) {
        float v = acc[b][j] + cv;
        if (RELU) v = v > 0.0f ? v : 0.0f;
        if (MASK) v = M[(int64_t)row * NO + col] > 0.0f ? v : 0.0f;
        Y[(int64_t)row * NO + col] = v;
      }
    }
  }
}

// products whose contraction is a multiple of 4 run on the matrix cores; the
// decoder's transposed product (K = 3) stays on the FMA kernel
template <int K, int NO, bool RELU, bool TW, bool MASK>
static void gemm(const float *X, const float *W, const float *c, const float *M, float *Y, int N,
                 hipStream_t s) {
  if constexpr (K % 4 == 0 && NO % 16 == 0) {
    const unsigned nb = (unsigned)std::max(1, (N + MR - 1) / MR);
    hipLaunchKernelGGL((gnn_mfma_gemm_kernel<K, NO, RELU, TW, MASK>), dim3(nb), dim3(256), 0, s, X, W, c, M, Y,
                       N);
  } else {
    const unsigned nb = (unsigned)std::max(1, (N + GR - 1) / GR);
    hipLaunchKernelGGL((gnn_gemm_kernel<K, NO, RELU, TW, MASK>), dim3(nb), dim3(GR * NO / 16), 0, s, X, W, c, M,
                       Y, N);
  }
}

// decoder: y = h W_d + c_d (3 outputs), one joint per thread
__global__ __launch_bounds__(GT) void gnn_dec_kernel(const float *H, const float *W, const float *c, float *y,
                                                     int N) {
  const int j = blockIdx.x * GT + threadIdx.x;
  if (j >= N) return;
  float a0 = c[0], a1 = c[1], a2 = c[2];
  const float *h = H + (int64_t)GNN_W * j;
  for (int k = 0; k < GNN_W; ++k) {
    a0 += h[k] * W[3 * k];
    a1 += h[k] * W[3 * k + 1];
    a2 += h[k] * W[3 * k + 2];
  }
  y[3 * (int64_t)j] = a0;
  y[3 * (int64_t)j + 1] = a1;
  y[3 * (int64_t)j + 2] = a2;
}

// Per-block partials of the weight gradient [X, 1]^T dZ over a row range:
// (K + 1) x NO outputs (the last row is the bias gradient).
template <int K, int NO>
__global__ __launch_bounds__(GT) void gnn_wgrad_kernel(const float *X, const float *dZ, int N, int rows,
                                                       float *wpart) {
  constexpr int NOUT = (K + 1) * NO, PER = (NOUT + GT - 1) / GT, KP = K + 1;
  __shared__ float Xs[64 * KP];
  __shared__ float Zs[64 * NO];
  float acc[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) acc[p] = 0.0f;
  const int rb0 = blockIdx.x * rows, rb1 = min(N, rb0 + rows);
  for (int r0 = rb0; r0 < rb1; r0 += 64) {
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * KP; i += GT) {
      const int r = i / KP, k = i % KP;
      const bool in = r0 + r < rb1;
      Xs[i] = !in ? 0.0f : (k == K ? 1.0f : X[(int64_t)(r0 + r) * K + k]);
    }
    for (int i = threadIdx.x; i < 64 * NO; i += GT) {
      const int r = i / NO;
      Zs[i] = r0 + r < rb1 ? dZ[(int64_t)(r0 + r) * NO + (i % NO)] : 0.0f;
    }
    __syncthreads();
    // output o = tid + GT p has column (tid mod NO) when NO divides GT, so
    // one Z value per row serves all of a thread's outputs
    for (int r = 0; r < 64; ++r) {
      if constexpr (GT % NO == 0) {
        const float z = Zs[r * NO + threadIdx.x % NO];
#pragma unroll
        for (int p = 0; p < PER; ++p) {
          const int o = threadIdx.x + GT * p;
          if (o < NOUT) acc[p] += Xs[r * KP + o / NO] * z;
        }
      } else {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
          const int o = threadIdx.x + GT * p;
          if (o < NOUT) acc[p] += Xs[r * KP + o / NO] * Zs[r * NO + o % NO];
        }
      }
    }
  }
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int o = threadIdx.x + GT * p;
    if (o < NOUT) wpart[(int64_t)blockIdx.x * NOUT + o] = acc[p];
  }
}

// The weight gradient on the matrix cores: per block of `rows` rows, the
// (K + 1) x NO partial [X, 1]^T dZ as MFMA blocks (A = [X, 1]^T: lane l
// takes feature m0 + l mod 16 of row r + l / 16; B = dZ: row r + l / 16,
// output n0 + l mod 16), 64 rows staged in LDS at a time.  The (K + 1) rows
// of the output are padded to whole blocks of 16; the four waves split the
// output blocks between them.
template <int K, int NO>
__global__ __launch_bounds__(256) void gnn_mfma_wgrad_kernel(const float *X, const float *dZ, int N, int rows,
                                                             float *wpart) {
  static_assert(NO % 16 == 0, "MFMA blocks");
  constexpr int MP = (K + 1 + 15) / 16, NB = NO / 16, NBLK = MP * NB, PER = (NBLK + 3) / 4;
  constexpr int XP = MP * 16 + 1, NOUT = (K + 1) * NO;
  __shared__ float Xs[64 * XP];
  __shared__ float Zs[64 * NO];
  const int w = threadIdx.x / 64, l = threadIdx.x % 64, kq = l >> 4;
  gnn_v4f acc[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) acc[p] = gnn_v4f{0.0f, 0.0f, 0.0f, 0.0f};
  const int rb0 = blockIdx.x * rows, rb1 = min(N, rb0 + rows);
  for (int r0 = rb0; r0 < rb1; r0 += 64) {
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * MP * 16; i += 256) {
      const int r = i / (MP * 16), m = i % (MP * 16);
      const bool in = r0 + r < rb1;
      Xs[r * XP + m] = !in || m > K ? 0.0f : (m == K ? 1.0f : X[(int64_t)(r0 + r) * K + m]);
    }
    for (int i = threadIdx.x; i < 64 * NO; i += 256) {
      const int r = i / NO;
      Zs[i] = r0 + r < rb1 ? dZ[(int64_t)(r0 + r) * NO + (i % NO)] : 0.0f;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < 64; rr += 4) {
#pragma unroll
      for (int p = 0; p < PER; ++p) {
        const int blk = w + 4 * p;
        if (blk < NBLK) {
          const int mb = blk / NB, nb = blk % NB;
          const float a = Xs[(rr + kq) * XP + mb * 16 + (l & 15)];
          const float b = Zs[(rr + kq) * NO + nb * 16 + (l & 15)];
          acc[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[p], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int blk = w + 4 * p;
    if (blk < NBLK) {
      const int mb = blk / NB, nb = blk % NB;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = mb * 16 + 4 * kq + j, n = nb * 16 + (l & 15);
        if (m <= K) wpart[(int64_t)blockIdx.x * NOUT + m * NO + n] = acc[p][j];
      }
    }
  }
}

// sum of the partials over the blocks, in block order
__global__ __launch_bounds__(GT) void gnn_wgrad_reduce_kernel(const float *wpart, int nblk, int nout,
                                                              float *out) {
  const int o = blockIdx.x * GT + threadIdx.x;
  if (o >= nout) return;
  float s = 0.0f;
  for (int b = 0; b < nblk; ++b) s += wpart[(int64_t)b * nout + o];
  out[o] = s;
}

// ------------------------------------------------------------- aggregation
// m_b = sum over the joints of body b of H_j (forward), or of
// dX_j[64:] / norm_j (backward); one (body, channel) per thread
__global__ __launch_bounds__(GT) void gnn_agg_kernel(PcgBallArgs a, const float *src, int stride, int off,
                                                     int scaled, float *m) {
  const int64_t t = (int64_t)blockIdx.x * GT + threadIdx.x;
  if (t >= (int64_t)a.nbd * GNN_W) return;
  const int b = (int)(t / GNN_W), cc = (int)(t % GNN_W);
  float s = 0.0f;
  for (int e = a.binc_off[b]; e < a.binc_off[b + 1]; ++e) {
    const int j = a.binc[e] >> 1;
    const float v = src[(int64_t)j * stride + off + cc];
    s += scaled ? v * joint_norm(a, j) : v;
  }
  m[t] = s;
}

// X_l = [H_{l-1}, (m_a + m_b) / norm]
__global__ __launch_bounds__(GT) void gnn_concat_kernel(PcgBallArgs a, const float *Hp, const float *m,
                                                        float *X) {
  const int64_t t = (int64_t)blockIdx.x * GT + threadIdx.x;
  if (t >= (int64_t)a.nj * GNN_W) return;
  const int j = (int)(t / GNN_W), cc = (int)(t % GNN_W);
  const int ba = a.jba[j], bb = a.jbb[j];
  float n = 0.0f;
  if (ba >= 0) n += m[(int64_t)ba * GNN_W + cc];
  if (bb >= 0) n += m[(int64_t)bb * GNN_W + cc];
  X[(int64_t)j * 2 * GNN_W + cc] = Hp[t];
  X[(int64_t)j * 2 * GNN_W + GNN_W + cc] = n * joint_norm(a, j);
}

// dZ_{l-1} = (dX_l[:64] + dm_a + dm_b) masked by H_{l-1} > 0
__global__ __launch_bounds__(GT) void gnn_aggbwd_kernel(PcgBallArgs a, const float *dX, const float *dm,
                                                        const float *Hp, float *dZ) {
  const int64_t t = (int64_t)blockIdx.x * GT + threadIdx.x;
  if (t >= (int64_t)a.nj * GNN_W) return;
  const int j = (int)(t / GNN_W), cc = (int)(t % GNN_W);
  const int ba = a.jba[j], bb = a.jbb[j];
  float v = dX[(int64_t)j * 2 * GNN_W + cc];
  if (ba >= 0) v += dm[(int64_t)ba * GNN_W + cc];
  if (bb >= 0) v += dm[(int64_t)bb * GNN_W + cc];
  dZ[t] = Hp[t] > 0.0f ? v : 0.0f;
}

// ------------------------------------------------------------------- loss
// delta = s y (FP64, into a.x)
__global__ __launch_bounds__(GT) void gnn_lam_kernel(PcgBallArgs a, GnnBufs g) {
  const int j = blockIdx.x * GT + threadIdx.x;
  if (j >= a.nj) return;
  const double s = g.sc[0];
  for (int r = 0; r < 3; ++r) a.x[3 * (int64_t)j + r] = s * (double)g.y[3 * (int64_t)j + r];
}

// lambda0 = lambda_b + delta (a.x holds delta)
__global__ __launch_bounds__(GT) void gnn_add_base_kernel(PcgBallArgs a, GnnBufs g) {
  const int j = blockIdx.x * GT + threadIdx.x;
  if (j >= a.nj) return;
  for (int r = 0; r < 3; ++r) a.x[3 * (int64_t)j + r] += g.lb[3 * (int64_t)j + r];
}

__global__ __launch_bounds__(GT) void gnn_body_kernel(PcgBallArgs a) {
  const int i = blockIdx.x * GT + threadIdx.x;
  if (i < a.nbd) body_one(a, i, a.x, nullptr, 0.0);
}

// partials of the energy decrease 1/2 delta^T S delta - delta^T r_b and
// dL/dy = s (S delta - r_b) / E_ref (a.x holds delta, zw its body pass)
__global__ __launch_bounds__(GT) void gnn_loss_kernel(PcgBallArgs a, GnnBufs g) {
  __shared__ double sh[GT];
  const int j = blockIdx.x * GT + threadIdx.x;
  double e = 0.0;
  if (j < a.nj) {
    double y[3];
    joint_one(a, j, y);
    const double f = g.sc[0] / g.sc[1];
    for (int r = 0; r < 3; ++r) {
      const double d = a.x[3 * (int64_t)j + r], rb = g.rb[3 * (int64_t)j + r];
      e += 0.5 * d * y[r] - rb * d;
      g.dY[3 * (int64_t)j + r] = (float)(f * (y[r] - rb));
    }
  }
  const double s = gnn_block_sum(e, sh);
  if (threadIdx.x == 0) g.red[4 * (int64_t)blockIdx.x + 2] = s;
}

__global__ __launch_bounds__(GT) void gnn_loss_reduce_kernel(int nblk, GnnBufs g) {
  __shared__ double sh[GT];
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += GT) v += g.red[4 * (int64_t)b + 2];
  const double e = gnn_block_sum(v, sh);
  if (threadIdx.x == 0) {
    g.sc[3] = e;
    g.sc[2] = e / g.sc[1];
  }
}

// ------------------------------------------------------------------- Adam
__global__ __launch_bounds__(GT) void gnn_adam_kernel(GnnBufs g, int n, float lr, float b1, float b2,
                                                      float c1, float c2, float eps) {
  const int i = blockIdx.x * GT + threadIdx.x;
  if (i >= n) return;
  const float gr = g.grad[i];
  const float m = b1 * g.adam_m[i] + (1.0f - b1) * gr;
  const float v = b2 * g.adam_v[i] + (1.0f - b2) * gr * gr;
  g.adam_m[i] = m;
  g.adam_v[i] = v;
  g.params[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// -------------------------------------------------------------- launchers
static unsigned blocks_of(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + GT - 1) / GT); }
constexpr int WROWS = 1024;  // rows per weight-gradient block

int gnn_wgrad_blocks(int nj) { return std::max(1, (nj + WROWS - 1) / WROWS); }

// base start and residual, features, layers, decoder; delta = s y into a.x
void launch_gnn_forward(const PcgBallArgs &a, const GnnBufs &g, int have_prev, hipStream_t s) {
  const int nj = a.nj;
  const unsigned jb = blocks_of(nj);
  hipLaunchKernelGGL(gnn_base_kernel, dim3(jb), dim3(GT), 0, s, a, g, have_prev);
  if (have_prev) hipLaunchKernelGGL(gnn_body_kernel, dim3(blocks_of(a.nbd)), dim3(GT), 0, s, a);
  hipLaunchKernelGGL(gnn_feat_a_kernel, dim3(jb), dim3(GT), 0, s, a, g, have_prev);
  hipLaunchKernelGGL(gnn_feat_reduce_kernel, dim3(1), dim3(GT), 0, s, nj, (int)jb, g);
  hipLaunchKernelGGL(gnn_feat_b_kernel, dim3(jb), dim3(GT), 0, s, a, g, have_prev);
  gemm<GNN_FIN, GNN_W, true, false, false>(g.x0, g.params + GNN_P_WE, g.params + GNN_P_CE, nullptr, g.H[0],
                                           nj, s);
  for (int l = 0; l < GNN_L; ++l) {
    const float *W = g.params + GNN_P_L0 + l * GNN_P_LSTRIDE;
    hipLaunchKernelGGL(gnn_agg_kernel, dim3(blocks_of((int64_t)a.nbd * GNN_W)), dim3(GT), 0, s, a, g.H[l],
                       GNN_W, 0, 0, g.m);
    hipLaunchKernelGGL(gnn_concat_kernel, dim3(blocks_of((int64_t)nj * GNN_W)), dim3(GT), 0, s, a, g.H[l],
                       g.m, g.X[l]);
    gemm<2 * GNN_W, GNN_W, true, false, false>(g.X[l], W, W + 2 * GNN_W * GNN_W, nullptr, g.H[l + 1], nj, s);
  }
  hipLaunchKernelGGL(gnn_dec_kernel, dim3(jb), dim3(GT), 0, s, g.H[GNN_L], g.params + GNN_P_WD,
                     g.params + GNN_P_CD, g.y, nj);
  hipLaunchKernelGGL(gnn_lam_kernel, dim3(jb), dim3(GT), 0, s, a, g);
}

// energy decrease of delta = a.x (loss in g.sc[2], decrease in g.sc[3]) and dL/dy
void launch_gnn_loss(const PcgBallArgs &a, const GnnBufs &g, hipStream_t s) {
  const unsigned jb = blocks_of(a.nj);
  hipLaunchKernelGGL(gnn_body_kernel, dim3(blocks_of(a.nbd)), dim3(GT), 0, s, a);
  hipLaunchKernelGGL(gnn_loss_kernel, dim3(jb), dim3(GT), 0, s, a, g);
  hipLaunchKernelGGL(gnn_loss_reduce_kernel, dim3(1), dim3(GT), 0, s, (int)jb, g);
}

template <int K, int NO>
static void wgrad(const float *X, const float *dZ, int nj, float *wpart, float *out, hipStream_t s) {
  const int nb = gnn_wgrad_blocks(nj);
  if constexpr (NO % 16 == 0)
    hipLaunchKernelGGL((gnn_mfma_wgrad_kernel<K, NO>), dim3(nb), dim3(256), 0, s, X, dZ, nj, WROWS, wpart);
  else
    hipLaunchKernelGGL((gnn_wgrad_kernel<K, NO>), dim3(nb), dim3(GT), 0, s, X, dZ, nj, WROWS, wpart);
  hipLaunchKernelGGL(gnn_wgrad_reduce_kernel, dim3(blocks_of((K + 1) * NO)), dim3(GT), 0, s, wpart, nb,
                     (K + 1) * NO, out);
}

// gradient of the loss with respect to every parameter, into g.grad
void launch_gnn_backward(const PcgBallArgs &a, const GnnBufs &g, hipStream_t s) {
  const int nj = a.nj;
  // decoder
  wgrad<GNN_W, 3>(g.H[GNN_L], g.dY, nj, g.wpart, g.grad + GNN_P_WD, s);
  gemm<3, GNN_W, false, true, true>(g.dY, g.params + GNN_P_WD, nullptr, g.H[GNN_L], g.dZ, nj, s);
  for (int l = GNN_L - 1; l >= 0; --l) {
    const int off = GNN_P_L0 + l * GNN_P_LSTRIDE;
    wgrad<2 * GNN_W, GNN_W>(g.X[l], g.dZ, nj, g.wpart, g.grad + off, s);
    gemm<GNN_W, 2 * GNN_W, false, true, false>(g.dZ, g.params + off, nullptr, nullptr, g.dX, nj, s);
    hipLaunchKernelGGL(gnn_agg_kernel, dim3(blocks_of((int64_t)a.nbd * GNN_W)), dim3(GT), 0, s, a, g.dX,
                       2 * GNN_W, GNN_W, 1, g.m);
    hipLaunchKernelGGL(gnn_aggbwd_kernel, dim3(blocks_of((int64_t)nj * GNN_W)), dim3(GT), 0, s, a, g.dX,
                       g.m, g.H[l], g.dZ);
  }
  wgrad<GNN_FIN, GNN_W>(g.x0, g.dZ, nj, g.wpart, g.grad + GNN_P_WE, s);
}

void launch_gnn_add_base(const PcgBallArgs &a, const GnnBufs &g, hipStream_t s) {
  hipLaunchKernelGGL(gnn_add_base_kernel, dim3(blocks_of(a.nj)), dim3(GT), 0, s, a, g);
}

void launch_gnn_adam(const GnnBufs &g, float lr, int64_t t, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(gnn_adam_kernel, dim3(blocks_of(GNN_NPARAM)), dim3(GT), 0, s, g, GNN_NPARAM, lr, b1, b2,
                     c1, c2, 1e-8f);
}

}  // namespace mabd
