"""Gaussian parameters from a multiresolution hash grid and a small MLP, F(X|Theta)
of Sec. III-C (the model of Instant-NGP with four heads) -- test infrastructure
only, plain PyTorch CPU float64 with autograd for the gradients.

Encoding (per level l = 0..L-1): resolution N_l = floor(N_min * b^l) with
b = exp(ln(N_max / N_min) / (L - 1)); the position is normalised into [0, 1]^3 by
the scene box and clamped; p = x_n * N_l, cell = min(floor(p), N_l - 1), the 8
vertices of the cell are looked up in the level's table of T entries x F
features -- by dense index v0 + (N_l+1)(v1 + (N_l+1) v2) when (N_l+1)^3 <= T,
else by the spatial hash (v0 * 1) xor (v1 * 2654435761) xor (v2 * 805459861)
modulo T on 32-bit unsigned integers -- and blended trilinearly.
MLP: L*F -> H (ReLU) -> H (ReLU) -> 11, heads colour = sigmoid(o[0:3]),
opacity = sigmoid(o[3]), scale = s_max * sigmoid(o[4:7]) (every scale below the
voxel size, Sec. III-C), quaternion = o[7:11] + (1, 0, 0, 0).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

PRIMES = (1, 2654435761, 805459861)

__all__ = ["NgpConfig", "level_resolution", "dense_level", "vertex_index", "encode", "params",
           "params_and_grads", "init_model", "PRIMES"]


@dataclasses.dataclass
class NgpConfig:
    levels: int = 16
    feat: int = 2
    log2_table: int = 19
    n_min: int = 16
    n_max: int = 4096
    hidden: int = 64
    scale_max: float = 0.05


def level_resolution(cfg: NgpConfig, l: int) -> int:
    b = math.exp(math.log(cfg.n_max / cfg.n_min) / (cfg.levels - 1)) if cfg.levels > 1 else 1.0
    return int(math.floor(cfg.n_min * b ** l))


def dense_level(cfg: NgpConfig, l: int) -> bool:
    n = level_resolution(cfg, l) + 1
    return n * n * n <= (1 << cfg.log2_table)


def vertex_index(cfg: NgpConfig, l: int, v):
    """Table row of integer vertices v [..., 3] at level l (numpy uint64 arithmetic, exact)."""
    v = np.asarray(v, np.uint64)
    T = np.uint64(1 << cfg.log2_table)
    if dense_level(cfg, l):
        n = np.uint64(level_resolution(cfg, l) + 1)
        return (v[..., 0] + n * (v[..., 1] + n * v[..., 2])).astype(np.int64)
    m = np.uint64(0xFFFFFFFF)
    h = ((v[..., 0] * np.uint64(PRIMES[0])) & m) ^ ((v[..., 1] * np.uint64(PRIMES[1])) & m) ^ \
        ((v[..., 2] * np.uint64(PRIMES[2])) & m)
    return (h % T).astype(np.int64)


def _corners():
    return np.array([[(c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], np.int64)


def encode(cfg: NgpConfig, x, lo, hi, tables):
    """Encoding [G, L*F] (torch float64) of positions x [G,3]; tables is a torch tensor [L, T, F]."""
    import torch
    xn = (torch.as_tensor(np.asarray(x, np.float64)) - torch.as_tensor(lo, dtype=torch.float64)) / \
        (torch.as_tensor(hi, dtype=torch.float64) - torch.as_tensor(lo, dtype=torch.float64))
    xn = xn.clamp(0.0, 1.0)
    outs = []
    cs = _corners()
    for l in range(cfg.levels):
        N = level_resolution(cfg, l)
        p = xn * N
        cell = torch.clamp(torch.floor(p), max=N - 1).to(torch.int64)
        fr = p - cell.to(torch.float64)
        acc = 0.0
        for c in cs:
            v = cell.numpy() + c
            idx = torch.as_tensor(vertex_index(cfg, l, v))
            w = torch.ones(xn.shape[0], dtype=torch.float64)
            for d in range(3):
                w = w * (fr[:, d] if c[d] else (1.0 - fr[:, d]))
            acc = acc + w[:, None] * tables[l][idx]
        outs.append(acc)
    return torch.cat(outs, dim=1)


def init_model(cfg: NgpConfig, seed=0):
    """Tables U(-1e-4, 1e-4); weights uniform with bound sqrt(6 / fan_in), biases 0 (float32 numpy)."""
    rng = np.random.default_rng(seed)
    T = 1 << cfg.log2_table
    D, H = cfg.levels * cfg.feat, cfg.hidden
    m = dict(tables=rng.uniform(-1e-4, 1e-4, size=(cfg.levels, T, cfg.feat)).astype(np.float32))
    for name, (fo, fi) in (("w1", (H, D)), ("w2", (H, H)), ("w3", (11, H))):
        m[name] = rng.uniform(-1, 1, size=(fo, fi)).astype(np.float32) * np.float32(math.sqrt(6.0 / fi))
    m["b1"], m["b2"], m["b3"] = (np.zeros(H, np.float32), np.zeros(H, np.float32), np.zeros(11, np.float32))
    return m


def _forward(cfg, x, lo, hi, t):
    import torch
    enc = encode(cfg, x, lo, hi, t["tables"])
    h1 = torch.relu(enc @ t["w1"].T + t["b1"])
    h2 = torch.relu(h1 @ t["w2"].T + t["b2"])
    o = h2 @ t["w3"].T + t["b3"]
    color = torch.sigmoid(o[:, 0:3])
    opac = torch.sigmoid(o[:, 3])
    scale = cfg.scale_max * torch.sigmoid(o[:, 4:7])
    quat = o[:, 7:11] + torch.tensor([1.0, 0.0, 0.0, 0.0], dtype=torch.float64)
    return dict(quat=quat.T, scale=scale.T, opacity=opac, color=color.T)


def _tensors(model, grad=False):
    import torch
    return {k: torch.tensor(np.asarray(v, np.float64), requires_grad=grad) for k, v in model.items()}


def params(cfg: NgpConfig, x, lo, hi, model):
    """Gaussian parameters quat [4,G], scale [3,G], opacity [G], colour [3,G] (float64 numpy)."""
    out = _forward(cfg, x, lo, hi, _tensors(model))
    return {k: v.detach().numpy() for k, v in out.items()}


def params_and_grads(cfg: NgpConfig, x, lo, hi, model, dparams):
    """Parameters and the gradient of sum(dparams * params) with respect to every model tensor."""
    t = _tensors(model, grad=True)
    out = _forward(cfg, x, lo, hi, t)
    import torch
    s = sum((out[k] * torch.as_tensor(np.asarray(dparams[k], np.float64))).sum() for k in out)
    s.backward()
    return ({k: v.detach().numpy() for k, v in out.items()}, {k: v.grad.numpy() for k, v in t.items()})
