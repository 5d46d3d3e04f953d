// Learned warm start for the ball-network PCG (not part of the paper's
// method; it only supplies the start value of the dual solve).
//
// Nodes are the joints of the network; two joints exchange messages through
// every dynamic body they share.  Per joint j:
//   x_j   = [D_j^{-1} b_j / s, lambda_prev_j / s, deg_a / 4, deg_b / 4,
//            world_a, world_b, 0...]                       (16 features)
//   h^0   = relu(x W_e + c_e)                               (width 64)
//   m_b   = sum of h^{l-1} over the joints of body b
//   n_j   = (m_a + m_b) / max(1, deg_a + deg_b)            (world side: 0)
//   h^l   = relu([h^{l-1}, n] W_l + c_l),  l = 1..3
//   y_j   = h^3 W_d + c_d,  lambda0_j = s y_j
// with D_j the diagonal block of the dual S, b the dual right-hand side,
// s = sqrt(mean_j |D_j^{-1} b_j|^2).  The loss of one system is the energy of
// the dual quadratic, E(lambda0) = 1/2 lambda0^T S lambda0 - b^T lambda0,
// divided by E_ref = |b^T D^{-1} b|: its minimiser is the solution and
// E - E_min = 1/2 |lambda0 - lambda*|_S^2, the error that bounds conjugate
// gradients; E < 0 means the start is better than zero in that norm.
#pragma once
#include <cstdint>

namespace mabd {

constexpr int GNN_W = 64;       // width
constexpr int GNN_FIN = 16;     // input features (10 used)
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
  double *red;              // reduction partials (4 per joint block)
  double *sc;               // [0] s, [1] E_ref, [2] loss, [3] energy
};

}  // namespace mabd
