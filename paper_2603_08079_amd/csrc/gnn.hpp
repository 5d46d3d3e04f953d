// Learned warm start for the ball-network PCG (not part of the paper's
// method; it only supplies the start value of the dual solve).
//
// The network refines a base start lambda_b (the previous step's multipliers,
// or zero) by a correction delta = s y.  Nodes are the joints of the network;
// two joints exchange messages through every dynamic body they share.  Per
// joint j, with r_b = b - S lambda_b the base residual and D_j the diagonal
// block of the dual S:
//   x_j   = [D_j^{-1} r_bj / s, lambda_bj / s_l, deg_a / 4, deg_b / 4,
//            world_a, world_b, have_base, 0...]             (16 features)
//   h^0   = relu(x W_e + c_e)                               (width 64)
//   m_b   = sum of h^{l-1} over the joints of body b
//   n_j   = (m_a + m_b) / max(1, deg_a + deg_b)            (world side: 0)
//   h^l   = relu([h^{l-1}, n] W_l + c_l),  l = 1..3
//   y_j   = h^3 W_d + c_d,  lambda0_j = lambda_bj + s y_j
// s = sqrt(mean_j |D_j^{-1} r_bj|^2), s_l = sqrt(mean_j |lambda_bj|^2) (1 if
// zero).  The loss of one system is the decrease of the dual energy
// E(l) = 1/2 l^T S l - b^T l from the base start,
//   E(lambda0) - E(lambda_b) = 1/2 delta^T S delta - delta^T r_b,
// divided by E_ref = |r_b^T D^{-1} r_b|.  Since E(l) - E_min is half the
// squared S-norm error, the error that bounds conjugate gradients, a negative
// loss means the learned start is better than the base start.
#pragma once
#include <cstdint>

namespace mabd {

constexpr int GNN_W = 64;       // width
constexpr int GNN_FIN = 16;     // input features (11 used)
constexpr int GNN_L = 3;        // message-passing layers
// parameter layout (float32, weights row-major [in][out], each followed by
// its bias)
constexpr int GNN_P_WE = 0;
constexpr int GNN_P_CE = GNN_P_WE + GNN_FIN * GNN_W;
constexpr int GNN_P_L0 = GNN_P_CE + GNN_W;
constexpr int GNN_P_LSTRIDE = 2 * GNN_W * GNN_W + GNN_W;
constexpr int GNN_P_WD = GNN_P_L0 + GNN_L * GNN_P_LSTRIDE;
constexpr int GNN_P_CD = GNN_P_WD + GNN_W * 3;
constexpr int GNN_NPARAM = GNN_P_CD + 3;

struct GnnBufs {
  float *x0;                // nj x 16
  float *X[GNN_L];          // nj x 128: [h^{l-1}, n] inputs of layer l
  float *H[GNN_L + 1];      // nj x 64: h^0 .. h^3
  float *y;                 // nj x 3
  float *m;                 // nbd x 64 body sums
  float *dX;                // nj x 128
  float *dZ;                // nj x 64
  float *dY;                // nj x 3
  float *params, *grad, *adam_m, *adam_v;
  float *wpart;             // weight-gradient partials
  double *lb, *rb;          // 3 x nj: base start and its residual b - S lambda_b
  double *red;              // reduction partials (4 per joint block)
  double *sc;               // [0] s, [1] E_ref, [2] loss, [3] energy decrease, [4] s_l
};

}  // namespace mabd
