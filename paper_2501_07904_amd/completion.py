"""Masked tensor completion on TT cores, started from a TT-UTV decomposition.

The observed entries M[idx_s] (s = 1..N) of an order-d tensor are fitted by
gradient descent on the cores of f = 1/2 sum_s (A_TT[idx_s] - M[idx_s])^2.
Sampled values and core gradients come from the library's tt_sample and
tt_sample_backward kernels (left and right interface products recomputed per
sample); the step size is the exact minimiser of the linearised residual,
alpha = <e, J g> / ||J g||^2 with J g the sampled directional derivative
(d more sampling passes, one per core).  The initial cores are the TT-UTV
decomposition of the zero-filled observed tensor scaled by 1/(observed
fraction) (a spectral initialisation).
"""
import torch

from . import tt_sample, tt_sample_backward, tt_utv_decompose


def flat_index(idx, dims):
    """Flat (i_1 fastest) position of every row of idx (N x d)."""
    stride, flat = 1, torch.zeros(idx.shape[0], dtype=torch.int64, device=idx.device)
    for k, n in enumerate(dims):
        flat += idx[:, k] * stride
        stride *= int(n)
    return flat


def spectral_init(dims, idx, vals, ranks, q=1, oversample=8, seed=0):
    """TT-UTV (right-to-left TT-URV) of the zero-filled observed tensor / fraction."""
    total = 1
    for n in dims:
        total *= int(n)
    frac = idx.shape[0] / total
    Z = torch.zeros(total, dtype=torch.float64, device=vals.device)
    Z[flat_index(idx, dims)] = vals.to(torch.float64) / frac
    cores, rep = tt_utv_decompose(Z, dims, ranks=ranks, sweep="R2L", variant="URV", q=q, oversample=oversample,
                                  seed=seed)
    return [c.clone() for c in cores], rep


def completion_step(cores, idx, vals):
    """One gradient step; returns (new cores, f before the step, alpha)."""
    e = tt_sample(cores, idx) - vals.to(torch.float64)
    f = 0.5 * float(torch.dot(e, e))
    g = tt_sample_backward(cores, idx, e)
    jg = torch.zeros_like(e)
    for k in range(len(cores)):
        jg += tt_sample(cores[:k] + [g[k]] + cores[k + 1:], idx)
    den = float(torch.dot(jg, jg))
    alpha = float(torch.dot(e, jg)) / den if den > 0 else 0.0
    return [c - alpha * gk for c, gk in zip(cores, g)], f, alpha


def complete(dims, idx, vals, ranks, steps, cores=None, seed=0):
    """Spectral initialisation (unless cores are given) and `steps` gradient
    steps; returns (cores, list of f per step)."""
    if cores is None:
        cores, _ = spectral_init(dims, idx, vals, ranks, seed=seed)
    hist = []
    for _ in range(steps):
        cores, f, _ = completion_step(cores, idx, vals)
        hist.append(f)
    return cores, hist
