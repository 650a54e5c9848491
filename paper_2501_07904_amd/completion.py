"""Masked tensor completion on TT cores, started from a TT-UTV decomposition.

Two iterations are provided.  `completion_step`: gradient descent on the
cores (below).  `rgrad_step`: Riemannian gradient descent on the manifold of
trains of fixed ranks with TT-UTV as the retraction (Sec. 4.3): the sampled
Euclidean gradient is projected onto the tangent space at the current train
(core gradients at the mixed-canonical points from the tt_sample_backward_mixed
kernel, then a projection of each left unfolding), the step
X - alpha xi uses the exact minimiser alpha of f on that line, and the
retraction is a fixed-rank TT-ULV (left to right) of the full stepped tensor,
which also gives the left-orthogonal form for the next step; the
right-orthogonal form is a fixed-rank TT-URV (right to left) of the full
current tensor, which represents it exactly.


The observed entries M[idx_s] (s = 1..N) of an order-d tensor are fitted by
gradient descent on the cores of f = 1/2 sum_s (A_TT[idx_s] - M[idx_s])^2.
Sampled values and core gradients come from the library's tt_sample and
tt_sample_backward kernels (left and right interface products recomputed per
sample); the step size is the exact minimiser of the linearised residual,
alpha = <e, J g> / ||J g||^2 with J g the sampled directional derivative
(d more sampling passes, one per core).  The initial cores are the TT-UTV
decomposition of the zero-filled observed tensor scaled by 1/(observed
fraction) (a spectral initialisation).

Every arithmetic step of both iterations runs in the library's kernels: the
residual and f (tt_residual), the step size (tt_line_step), the core update
and the accumulation of directional derivatives (tt_axpy), the tangent
projection (tt_tangent_project) and the cores of the tangent vector and of
the stepped point (tt_tangent_train); f and alpha are read back once per step.
"""
import torch

from . import (_core_buffers, _core_view, tt_axpy, tt_line_step, tt_reconstruct, tt_residual, tt_sample,
               tt_sample_backward, tt_sample_backward_mixed, tt_tangent_project, tt_tangent_train,
               tt_utv_decompose)


# largest rank the sampling and reconstruction kernels take (TT_MAX_ELL)
TANGENT_TRAIN_MAX_RANK = 64


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
    """One gradient step; returns (new cores, f before the step, alpha).  The
    residual, the directional derivative's accumulation, the step size and the
    core update run in the library's kernels; f and alpha are read back once."""
    z, f = tt_residual(tt_sample(cores, idx), vals)
    g = tt_sample_backward(cores, idx, z)
    jg = tt_sample([g[0]] + cores[1:], idx)
    for k in range(1, len(cores)):
        tt_axpy(jg, tt_sample(cores[:k] + [g[k]] + cores[k + 1:], idx))
    st = tt_line_step(jg, z)
    new = []
    for c, gk in zip(cores, g):
        flat = _core_buffers([c])[0].clone()
        tt_axpy(flat, _core_buffers([gk])[0], a=-1.0, a_dev=st[0:1])
        new.append(_core_view(flat, *c.shape))
    return new, float(f[0]), float(st[0])


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


def rgrad_step(cores, idx, vals, q=1, oversample=8, seed=0, left_orthogonal=False):
    """One Riemannian gradient step (TT-UTV retraction) for
    f = 1/2 sum_s (X[idx_s] - m_s)^2 at the train `cores`.  With
    left_orthogonal the cores are already the left-orthogonal form (as
    returned by this function).  Returns (new left-orthogonal cores, f before
    the step, alpha)."""
    dims = [int(g.shape[1]) for g in cores]
    ranks = [int(g.shape[2]) for g in cores[:-1]]
    kw = dict(q=q, oversample=oversample, seed=seed)
    full = tt_reconstruct(cores)
    if left_orthogonal:
        U = [g.to(torch.float64) for g in cores]
    else:
        U, _ = tt_utv_decompose(full, dims, ranks=ranks, sweep="L2R", variant="ULV", **kw)
        U = [g.clone() for g in U]
    V, _ = tt_utv_decompose(full, dims, ranks=ranks, sweep="R2L", variant="URV", **kw)
    V = [g.clone() for g in V]
    del full
    z, f = tt_residual(tt_sample(U, idx), vals)
    G = tt_sample_backward_mixed(U, V, idx, z)
    dC = tt_tangent_project(U, G)
    if 2 * max(ranks) <= TANGENT_TRAIN_MAX_RANK:
        # the tangent vector and the stepped point as trains of ranks 2 r_k
        st = tt_line_step(tt_sample(tt_tangent_train(U, V, dC, 1.0), idx), z)
        xhat = tt_reconstruct(tt_tangent_train(U, V, dC, -1.0, t_dev=st[0:1], base=True))
    else:
        # ranks above half the sampling kernels' limit: xi term by term, each term
        # U_<k dC_k V_>k a train of the point's own ranks
        terms = [U[:k] + [dC[k]] + V[k + 1:] for k in range(len(dims))]
        pxi = tt_sample(terms[0], idx)
        for tk in terms[1:]:
            tt_axpy(pxi, tt_sample(tk, idx))
        st = tt_line_step(pxi, z)
        xhat = tt_reconstruct(U)
        for tk in terms:
            tt_axpy(xhat, tt_reconstruct(tk), a=-1.0, a_dev=st[0:1])
    new, _ = tt_utv_decompose(xhat, dims, ranks=ranks, sweep="L2R", variant="ULV", **kw)
    return [g.clone() for g in new], float(f[0]), float(st[0])


def complete_rgrad(dims, idx, vals, ranks, steps, cores=None, seed=0):
    """Spectral initialisation (unless cores are given) and `steps` Riemannian
    gradient steps; returns (left-orthogonal cores, list of f per step)."""
    if cores is None:
        cores, _ = spectral_init(dims, idx, vals, ranks, seed=seed)
    hist = []
    left = False
    for _ in range(steps):
        cores, f, _ = rgrad_step(cores, idx, vals, seed=seed, left_orthogonal=left)
        left = True
        hist.append(f)
    return cores, hist
