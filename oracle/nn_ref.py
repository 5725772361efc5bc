"""FP64 CPU reference of the learned preconditioner network (test infrastructure only).

Not part of the paper's method: the network is the library's learned initial guess / right
preconditioner (documented in include/pb.h). This module restates its definition with plain
numpy (neighbours, features) and PyTorch CPU float64 ops (forward, and gradients by autograd),
independently of the GPU kernels. Where the GPU rounds to BF16 — layer inputs and weights —
this reference rounds at the same points, with a straight-through gradient.

Definition:
  * slots: each node's 16 nearest band nodes by projection distance (itself first), ties by
    index, squared distances as ((dx·dx + dy·dy) + dz·dz);
  * node features: φ/ε, n, H·ε with H = (2/m) Σ_{j≠i, |x_j−x_i|² ≥ 1e-12ε²} (n_j − n_i)·(x_j − x_i)/|x_j − x_i|²;
  * layer-1 slot features of neighbour j of node i: the node features of j, v1_j/s1, v2_j/s2,
    (x_j − x_i)/ε, zero-padded to 16 (s = per-half RMS of v, 1 when zero);
  * four layers Z = G·W + b over the 16 gathered slots, leaky ReLU (slope 0.01) after the
    first three, widths 16 → 64 → 64 → 64 → 16 (channels 0, 1 used);
  * M(v) = Λ⁻¹(v + s ⊙ O); loss Σ|O − T|²/Σ|T|² with T = (Λu − v)/s.
"""
from __future__ import annotations

import numpy as np
import torch

SLOTS = 16
CIN = (16, 64, 64, 64)
COUT = (64, 64, 64, 16)
SLOPE = 0.01


def layer_shapes():
    return [(SLOTS * c, o) for c, o in zip(CIN, COUT)]


def unpack(params: np.ndarray):
    """Flat parameters → list of (W[K][Cout], b[Cout]) float64 arrays."""
    out, off = [], 0
    for K, C in layer_shapes():
        W = params[off:off + K * C].reshape(K, C).astype(np.float64)
        off += K * C
        b = params[off:off + C].astype(np.float64)
        off += C
        out.append((W, b))
    assert off == params.size
    return out


def knn(xs: np.ndarray) -> np.ndarray:
    """16 nearest nodes by squared distance ((dx·dx + dy·dy) + dz·dz), ties by index."""
    n = len(xs)
    nbr = np.empty((n, SLOTS), dtype=np.int64)
    idx = np.arange(n)
    for i in range(n):
        d = xs[i] - xs
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        order = np.lexsort((idx, d2))
        nbr[i] = order[:SLOTS]
    return nbr


def features(nodes: np.ndarray, nbr: np.ndarray, eps: float) -> np.ndarray:
    """Node features (n × 5) in float64: φ/ε, n, H·ε."""
    x, nrm, phi = nodes[:, :3], nodes[:, 3:6], nodes[:, 6]
    n = len(nodes)
    H = np.zeros(n)
    for i in range(n):
        s, m = 0.0, 0
        for j in nbr[i]:
            d = x[j] - x[i]
            d2 = d @ d
            if j == i or d2 < 1e-12 * eps * eps:
                continue
            s += (nrm[j] - nrm[i]) @ d / d2
            m += 1
        H[i] = 2.0 * s / m if m else 0.0
    return np.column_stack([phi / eps, nrm, H * eps])


def bf16(t: torch.Tensor) -> torch.Tensor:
    """Round to BF16 (nearest even) in the forward pass, identity in the backward pass."""
    return t + (t.to(torch.bfloat16).to(torch.float64) - t).detach()


def forward(nodes, nbr, feat32, v, params, lam, eps, rounding=True):
    """Returns (O [n × 16], s) as torch float64 tensors; params: list of (W, b) tensors.
    rounding=False evaluates the same network exactly in FP64 (for finite-difference checks)."""
    rb = bf16 if rounding else (lambda t: t)
    r32 = (lambda t: t.to(torch.float32).to(torch.float64)) if rounding else (lambda t: t)
    n = len(nodes)
    v = torch.as_tensor(v, dtype=torch.float64)
    s1 = torch.sqrt(torch.mean(v[:n] ** 2))
    s2 = torch.sqrt(torch.mean(v[n:] ** 2))
    s1 = s1 if s1 > 0 else torch.tensor(1.0, dtype=torch.float64)
    s2 = s2 if s2 > 0 else torch.tensor(1.0, dtype=torch.float64)
    f = torch.as_tensor(feat32, dtype=torch.float64)
    x = torch.as_tensor(nodes[:, :3], dtype=torch.float64)
    nb = torch.as_tensor(nbr, dtype=torch.long)
    # layer-1 inputs per (node, slot): FP32 values rounded to BF16
    fj = f[nb]                                                    # n × 16 × 5
    vj = torch.stack([v[:n][nb] / s1, v[n:][nb] / s2], -1)       # n × 16 × 2
    rel = (x[nb] - x[:, None, :]) / eps                           # n × 16 × 3
    g = torch.cat([fj, r32(vj), r32(rel), torch.zeros(n, SLOTS, 6, dtype=torch.float64)], -1)
    h = rb(g.reshape(n, SLOTS * 16))
    for l, (W, b) in enumerate(params):
        if l > 0:
            h = rb(r32(h)[nb].reshape(n, -1))
        z = h @ rb(W) + b
        h = torch.where(z > 0, z, SLOPE * z) if l < 3 else z
    return h, (s1, s2)


def apply(nodes, nbr, feat32, v, params_flat, lam, eps):
    """M(v) = Λ⁻¹(v + s ⊙ O) as a numpy float64 array."""
    params = [(torch.as_tensor(W), torch.as_tensor(b)) for W, b in unpack(params_flat)]
    O, (s1, s2) = forward(nodes, nbr, feat32, v, params, lam, eps)
    n = len(nodes)
    v = np.asarray(v, dtype=np.float64)
    O = O.detach().numpy()
    return np.concatenate([(v[:n] + float(s1) * O[:, 0]) / lam[0], (v[n:] + float(s2) * O[:, 1]) / lam[1]])


def loss_and_grads(nodes, nbr, feat32, v, u, params_flat, lam, eps, rounding=True):
    """Loss Σ|O − T|²/Σ|T|² and its gradient w.r.t. the flat parameters (float64)."""
    n = len(nodes)
    params = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True))
              for W, b in unpack(np.asarray(params_flat, dtype=np.float64))]
    O, (s1, s2) = forward(nodes, nbr, feat32, v, params, lam, eps, rounding)
    v = torch.as_tensor(v, dtype=torch.float64)
    u = torch.as_tensor(u, dtype=torch.float64)
    r32 = (lambda t: t.to(torch.float32).to(torch.float64)) if rounding else (lambda t: t)
    T1 = r32((lam[0] * u[:n] - v[:n]) / s1)
    T2 = r32((lam[1] * u[n:] - v[n:]) / s2)
    den = torch.sum(T1 ** 2 + T2 ** 2)
    loss = torch.sum((O[:, 0] - T1) ** 2 + (O[:, 1] - T2) ** 2) / den
    loss.backward()
    flat = []
    for W, b in params:
        flat.append(W.grad.numpy().ravel())
        flat.append(b.grad.numpy().ravel())
    return float(loss.detach()), np.concatenate(flat)
