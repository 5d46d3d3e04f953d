"""Reference of the learned PCG warm start, for tests only.

Test infrastructure: plain numpy in FP64, written from the network's
definition (it is not part of the paper's method, which says nothing about
it; the method only fixes the dual system S lambda = r of Eq. dual, taken
here from the oracle's own assembly).  The GPU library must reproduce
`forward` and `loss` up to FP32 rounding, and its gradients must match
central differences of `loss`.

Network, per joint k of a ball-joint network (rows 3k..3k+2 of S), refining
a base start l_b (the previous multipliers, or zero) with residual
r_b = r - S l_b:
  x_k  = [D_k^{-1} r_bk / s, l_bk / s_l, deg_a / 4, deg_b / 4, world_a,
          world_b, have_base, 0 x 5],  D_k = S_kk,
  s = sqrt(mean_k |D_k^{-1} r_bk|^2),  s_l = sqrt(mean_k |l_bk|^2) (1 if 0)
  h0   = relu(x We + ce)
  m_b  = sum of h over the joints of dynamic body b
  n_k  = (m_a + m_b) / max(1, deg_a + deg_b)           (world side: 0)
  h_l  = relu([h_{l-1}, n] Wl + cl),  l = 1..3
  y    = h_3 Wd + cd,  delta = s y,  lam0 = l_b + delta
loss = (1/2 delta^T S delta - delta^T r_b) / |r_b^T D^{-1} r_b|, which is
(E(lam0) - E(l_b)) / E_ref for the dual energy E(l) = 1/2 l^T S l - r^T l.
Parameter layout: We (16x64), ce, then per layer W (128x64), c, then Wd
(64x3), cd; weights row-major [in][out].
"""
import numpy as np

FIN, W, L = 16, 64, 3
P_WE = 0
P_CE = P_WE + FIN * W
P_L0 = P_CE + W
P_LS = 2 * W * W + W
P_WD = P_L0 + L * P_LS
P_CD = P_WD + W * 3
NPARAM = P_CD + 3


def unpack(p):
    p = np.asarray(p, np.float64)
    assert p.shape == (NPARAM,)
    We = p[P_WE:P_CE].reshape(FIN, W)
    ce = p[P_CE:P_L0]
    layers = []
    for l in range(L):
        o = P_L0 + l * P_LS
        layers.append((p[o:o + 2 * W * W].reshape(2 * W, W), p[o + 2 * W * W:o + P_LS]))
    Wd = p[P_WD:P_CD].reshape(W, 3)
    cd = p[P_CD:]
    return We, ce, layers, Wd, cd


class Network:
    """Graph data of one ball-joint network: joint ends (-1 for the world or
    a pinned body) and the dual system of one state."""

    def __init__(self, asm, S, r, lam_prev=None):
        self.m = asm.m
        dyn = asm.pinned == 0
        ja = np.where((asm.ja >= 0) & dyn[np.maximum(asm.ja, 0)], asm.ja, -1)
        jb = np.where((asm.jb >= 0) & dyn[np.maximum(asm.jb, 0)], asm.jb, -1)
        self.ja, self.jb = ja, jb
        deg = np.zeros(asm.n)
        for k in range(self.m):
            for b in (ja[k], jb[k]):
                if b >= 0:
                    deg[b] += 1
        self.deg = deg
        S = S.toarray() if hasattr(S, "toarray") else np.asarray(S)
        self.S, self.r = S, np.asarray(r, np.float64)
        self.lb = np.zeros(3 * self.m) if lam_prev is None else np.asarray(lam_prev, np.float64).ravel()
        self.rb = self.r - S @ self.lb
        z = np.zeros((self.m, 3))
        for k in range(self.m):
            z[k] = np.linalg.solve(S[3 * k:3 * k + 3, 3 * k:3 * k + 3], self.rb[3 * k:3 * k + 3])
        self.s = np.sqrt(np.mean(np.sum(z * z, axis=1)))
        self.eref = abs(float(np.dot(self.rb, z.ravel())))
        sl = np.sqrt(np.mean(np.sum(self.lb.reshape(-1, 3) ** 2, axis=1)))
        self.sl = sl if sl > 0 else 1.0
        x = np.zeros((self.m, FIN))
        x[:, 0:3] = z / self.s
        x[:, 3:6] = self.lb.reshape(self.m, 3) / self.sl
        dga = np.where(ja >= 0, deg[np.maximum(ja, 0)], 0.0)
        dgb = np.where(jb >= 0, deg[np.maximum(jb, 0)], 0.0)
        x[:, 6] = dga / 4
        x[:, 7] = dgb / 4
        x[:, 8] = ja < 0
        x[:, 9] = jb < 0
        x[:, 10] = 0.0 if lam_prev is None else 1.0
        self.x = x
        self.norm = 1.0 / np.maximum(1.0, dga + dgb)
        self.nbody = asm.n

    def forward(self, p):
        We, ce, layers, Wd, cd = unpack(p)
        h = np.maximum(self.x @ We + ce, 0.0)
        for Wl, cl in layers:
            m = np.zeros((self.nbody, W))
            for k in range(self.m):
                for b in (self.ja[k], self.jb[k]):
                    if b >= 0:
                        m[b] += h[k]
            n = np.zeros_like(h)
            for k in range(self.m):
                for b in (self.ja[k], self.jb[k]):
                    if b >= 0:
                        n[k] += m[b]
            n *= self.norm[:, None]
            h = np.maximum(np.concatenate([h, n], axis=1) @ Wl + cl, 0.0)
        y = h @ Wd + cd
        return self.lb.reshape(self.m, 3) + self.s * y

    def loss(self, p):
        d = (self.forward(p) - self.lb.reshape(self.m, 3)).ravel()
        return (0.5 * d @ (self.S @ d) - self.rb @ d) / self.eref
