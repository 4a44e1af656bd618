"""FP64 oracle of the learned control variate (test infrastructure only).

The paper has no learned component; this follows the learned-control-variate form of the
TTCF estimator that the build adds beside the plain method:
  * start-state features x(Gamma): P_xy(0), Omega(0); for 20 slabs in y the sums over the
    slab's atoms of p_x, of p_x p_y (the kinetic shear stress) and of the pair virial
    x_ij F_y,ij (the configurational shear stress, each pair half to the slab of either
    atom); and the two parts of d(V P_xy)/dt at t = 0 that need no force derivative,
    sum_i (F_x,i p_y,i + p_x,i F_y,i) and sum_{i<j} (p_x,i - p_x,j) F_y,ij (reading: the 62
    "binned stress/momentum" features are these 60 slab sums and the two rates);
  * an MLP g(x) = W3 gelu(W2 gelu(W1 x + b1) + b2) + b3 that predicts B(t_k), k = 1..n_out;
  * the control variate of one daughter, h = Omega(0) int_0^t g(x, s) ds (trapezoid rule with
    g(x, 0) = B(0), the known start value), whose mean over equilibrium start states is
    estimated separately from many mother samples;
  * the CV estimate TTCF_cv(t) = mean_n [G_n(t) - H_n(t)] + mu_H(t), with G_n the plain
    per-start-state TTCF series and H_n the mapping average of h.
For any fixed g the estimate is unbiased (E[H] = mu_H); g = 0 gives the plain estimate.

GELU is the exact erf form. "bf16=True" rounds every GEMM operand to bfloat16 (round to
nearest even), as the GPU kernels do before their FP32-accumulating matrix instructions.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.special import erf

N_SLABS = 20
WCA_RC = 2.0 ** (1.0 / 6.0)


def bf16_round(a):
    """Round to bfloat16 (8-bit mantissa), nearest-even, returned as float64."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


# ----------------------------------------------------------------------------------------
# features
# ----------------------------------------------------------------------------------------

def pair_forces(r, box, rc=WCA_RC, c_attr=1.0):
    """Every pair i < j closer than rc in a periodic box without Lees-Edwards offset (a start
    state), by brute force: i, j, the minimum-image separation r_i - r_j (n_pairs, 3) and the
    force on i from j, 24 (2 r^-14 - c r^-8) (r_i - r_j) (Eq. LJ with c = c_attr)."""
    n = len(r) // 3
    x = np.asarray(r, np.float64).reshape(3, n).T
    L = np.asarray(box, np.float64)
    i, j = np.triu_indices(n, 1)
    d = x[i] - x[j]
    d -= L * np.rint(d / L)
    r2 = (d * d).sum(axis=1)
    keep = r2 < rc * rc
    i, j, d, r2 = i[keep], j[keep], d[keep], r2[keep]
    inv2 = 1.0 / r2
    inv6 = inv2 ** 3
    f = (24.0 * inv6 * (2.0 * inv6 - c_attr) * inv2)[:, None] * d
    return i, j, d, f


def features(r, p, box, vpxy0, gamma_dot, temperature, volume, rc=WCA_RC, c_attr=1.0):
    """64 features of one (mapped) start state, FP64: [P_xy(0), Omega(0), per slab (20 each):
    sum p_x, sum p_x p_y, sum of half the pair virials x_ij F_y,ij of the slab's atoms; then
    sum_i (F_x,i p_y,i + p_x,i F_y,i), sum_{i<j} (p_x,i - p_x,j) F_y,ij]. r, p: SoA (3n,).
    Slab k = floor(y * 20 / Ly), clamped."""
    n = len(r) // 3
    y = r[n:2 * n]
    px, py = p[:n], p[n:2 * n]
    k = np.minimum(np.floor(y * (N_SLABS / box[1])).astype(int), N_SLABS - 1)
    mom = np.zeros(N_SLABS)
    st = np.zeros(N_SLABS)
    vir = np.zeros(N_SLABS)
    np.add.at(mom, k, px)
    np.add.at(st, k, px * py)
    i, j, d, f = pair_forces(r, box, rc, c_attr)
    w = d[:, 0] * f[:, 1]
    np.add.at(vir, k[i], 0.5 * w)
    np.add.at(vir, k[j], 0.5 * w)
    F = np.zeros((n, 3))
    np.add.at(F, i, f)
    np.add.at(F, j, -f)
    d1 = np.sum(F[:, 0] * py + px * F[:, 1])
    d2 = np.sum((px[i] - px[j]) * f[:, 1])
    pxy0 = vpxy0 / volume
    om = -(volume / temperature) * gamma_dot * pxy0
    return np.concatenate([[pxy0, om], mom, st, vir, [d1, d2]])


# ----------------------------------------------------------------------------------------
# MLP
# ----------------------------------------------------------------------------------------

@dataclass
class MLP:
    W1: np.ndarray
    b1: np.ndarray
    W2: np.ndarray
    b2: np.ndarray
    W3: np.ndarray
    b3: np.ndarray

    def params(self):
        return [self.W1, self.b1, self.W2, self.b2, self.W3, self.b3]

    def flat(self):
        return np.concatenate([a.ravel() for a in self.params()])

    @staticmethod
    def from_flat(v, n_in, n_hid, n_out):
        v = np.asarray(v, np.float64)
        shapes = [(n_in, n_hid), (n_hid,), (n_hid, n_hid), (n_hid,), (n_hid, n_out), (n_out,)]
        out, o = [], 0
        for s in shapes:
            sz = int(np.prod(s))
            out.append(v[o:o + sz].reshape(s).copy())
            o += sz
        return MLP(*out)


def init_weights(n_in, n_hid, n_out, seed):
    """He-normal weights, zero biases (numpy PCG64, seeded)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return MLP(rng.standard_normal((n_in, n_hid)) * np.sqrt(2.0 / n_in), np.zeros(n_hid),
               rng.standard_normal((n_hid, n_hid)) * np.sqrt(2.0 / n_hid), np.zeros(n_hid),
               rng.standard_normal((n_hid, n_out)) * np.sqrt(1.0 / n_hid), np.zeros(n_out))


def _mm(a, b, bf16):
    return (bf16_round(a) @ bf16_round(b)) if bf16 else a @ b


def forward(net: MLP, x, bf16=False):
    """Returns (y, cache). x: (batch, n_in)."""
    z1 = _mm(x, net.W1, bf16) + net.b1
    a1 = gelu(z1)
    z2 = _mm(a1, net.W2, bf16) + net.b2
    a2 = gelu(z2)
    y = _mm(a2, net.W3, bf16) + net.b3
    return y, (x, z1, a1, z2, a2)


def mse_loss(y, t):
    return float(np.mean((y - t) ** 2))


def backward(net: MLP, cache, y, t, bf16=False):
    """Gradients of the mean squared error (mean over every element) w.r.t. the parameters."""
    x, z1, a1, z2, a2 = cache
    dy = 2.0 * (y - t) / y.size
    gW3 = _mm(a2.T, dy, bf16)
    gb3 = dy.sum(axis=0)
    da2 = _mm(dy, net.W3.T, bf16)
    dz2 = da2 * gelu_grad(z2)
    gW2 = _mm(a1.T, dz2, bf16)
    gb2 = dz2.sum(axis=0)
    da1 = _mm(dz2, net.W2.T, bf16)
    dz1 = da1 * gelu_grad(z1)
    gW1 = _mm(x.T, dz1, bf16)
    gb1 = dz1.sum(axis=0)
    return MLP(gW1, gb1, gW2, gb2, gW3, gb3)


@dataclass
class Adam:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: list = None
    v: list = None

    def step(self, net: MLP, grad: MLP):
        if self.m is None:
            self.m = [np.zeros_like(p) for p in net.params()]
            self.v = [np.zeros_like(p) for p in net.params()]
        self.t += 1
        c1 = 1.0 - self.beta1 ** self.t
        c2 = 1.0 - self.beta2 ** self.t
        for p, g, m, v in zip(net.params(), grad.params(), self.m, self.v):
            m *= self.beta1
            m += (1.0 - self.beta1) * g
            v *= self.beta2
            v += (1.0 - self.beta2) * g * g
            p -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)


# ----------------------------------------------------------------------------------------
# control variate
# ----------------------------------------------------------------------------------------

def cv_h(pred, b0, omega, dt):
    """h(t_k) = Omega(0) int_0^{t_k} g ds by the trapezoid rule on the step grid, with
    g(0) = B(0). pred: (n, n_out) predictions of B(t_1..t_nout); b0, omega: (n,).
    Returns (n, n_out + 1) with h(t_0) = 0."""
    g = np.concatenate([np.asarray(b0)[:, None], pred], axis=1)
    integ = np.zeros_like(g)
    integ[:, 1:] = np.cumsum(0.5 * dt * (g[:, :-1] + g[:, 1:]), axis=1)
    return np.asarray(omega)[:, None] * integ


def cv_estimate(g_series, h_daughters, mu_h, n_maps=4):
    """TTCF_cv(t) = mean_n [G_n(t) - H_n(t)] + mu_H(t), with H_n the mapping mean of h.
    Returns (mean, block SE, per-state residuals)."""
    nd, nt = h_daughters.shape
    hn = h_daughters.reshape(nd // n_maps, n_maps, nt).mean(axis=1)
    resid = g_series - hn
    ns = resid.shape[0]
    return resid.mean(axis=0) + mu_h, resid.std(axis=0, ddof=1) / np.sqrt(ns), resid
