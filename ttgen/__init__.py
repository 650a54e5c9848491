"""Seeded synthetic inputs shared by the tests and the benchmark.

This module only draws random numbers and evaluates closed-form test
functions; it holds none of the TT-UTV arithmetic.  Every tensor is returned
flat in reverse lexicographic order (i1 fastest), the layout the library and
the oracle both take.

Workloads (stand-ins for the paper's experiments, whose data sets are not
available):
  gaussian_tt_tensor  -- Example 1 of the paper: Gaussian TT cores contracted,
                         plus i.i.d. Gaussian noise at a given relative
                         Frobenius norm.
  inverse_sum_tensor  -- smooth function 1/(1 + x_1 + ... + x_d) on a uniform
                         [0,1] grid (a function tensor like Example 2).
  sin_norm_tensor     -- Example 2: sin(sqrt(sum_k ((i_k-1)/(I-1))^2)).
  mri_like_volume     -- sum of random 3-D Gaussian ellipsoids plus Rician
                         noise (stand-in for the MRI volume).
  gaussian_tt_tensor_device -- the Example 1 recipe built on the GPU with
                         PyTorch (tensors of many GB: 40^6 FP32), split as
                         (left half-train) x (right half-train) + noise.
  sin_norm_tensor_device -- the Example 2 tensor built on the GPU.
"""
import numpy as np


def gaussian_cores(dims, ranks, seed):
    """Cores of shape (r_{k-1}, I_k, r_k) with i.i.d. N(0,1) entries."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((ranks[k], dims[k], ranks[k + 1])) for k in range(len(dims))]


def _contract_cores(cores):
    """Dense tensor of a train of cores by successive tensordot over the bond
    indices (numpy C-order logical array with axes i_1..i_d)."""
    t = cores[0][0]                                   # (I_1, r_1)
    for g in cores[1:]:
        t = np.tensordot(t, g, axes=([-1], [0]))      # (..., I_k, r_k)
    return t[..., 0]


def gaussian_tt_tensor(dims, ranks, noise_rel, seed, dtype=np.float64):
    """A = P + beta*N with P contracted from Gaussian cores of the given ranks
    and N i.i.d. N(0,1); beta makes ||beta N||_F = noise_rel * ||P||_F.
    Returns (flat tensor, cores of P)."""
    ranks = list(ranks)
    if len(ranks) == len(dims) - 1:
        ranks = [1] + ranks + [1]
    cores = gaussian_cores(dims, ranks, seed)
    P = _contract_cores(cores).reshape(-1, order="F")
    if noise_rel > 0:
        rng = np.random.default_rng(seed + 7919)
        N = rng.standard_normal(P.size)
        P = P + (noise_rel * np.linalg.norm(P) / np.linalg.norm(N)) * N
    return P.astype(dtype), cores


def inverse_sum_tensor(d, n, dtype=np.float32):
    """f(x) = 1/(1 + x_1 + ... + x_d) on x_j = j/(n-1), j = 0..n-1; evaluated
    in float64 and rounded once to `dtype`."""
    x = np.arange(n, dtype=np.float64) / (n - 1)
    s = np.zeros((n,) * d)
    for k in range(d):
        shape = [1] * d
        shape[k] = n
        s = s + x.reshape(shape)
    return (1.0 / (1.0 + s)).reshape(-1, order="F").astype(dtype)


def sin_norm_tensor(d, n):
    """B(i_1..i_d) = sin(sqrt(sum_k ((i_k-1)/(n-1))^2)), i_k = 1..n (float64).

    The squares are summed in index order k = 1..d; the slabs of the last
    index are filled on a thread pool (the ufuncs release the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    x2 = (np.arange(n, dtype=np.float64) / (n - 1)) ** 2
    head = np.zeros((n,) * (d - 1), order="F")
    for k in range(d - 1):
        shape = [1] * (d - 1)
        shape[k] = n
        head += x2.reshape(shape)
    out = np.empty((n,) * d, order="F")

    def slab(j):
        v = out[..., j]
        np.add(head, x2[j], out=v)
        np.sqrt(v, out=v)
        np.sin(v, out=v)

    with ThreadPoolExecutor(max_workers=min(8, n)) as pool:
        list(pool.map(slab, range(n)))
    return out.reshape(-1, order="F")


def random_indices(dims, count, seed):
    """count multi-indices (count x d, int64, 0-based), uniform over the grid."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, I, size=count) for I in dims], axis=1).astype(np.int64)


def mri_like_volume(shape=(256, 256, 160), n_ell=12, sigma=0.02, seed=0):
    """Sum of n_ell randomly rotated 3-D Gaussian ellipsoids with intensities
    U[0.2, 1], centres U[0.2, 0.8]*dim and semi-axes U[0.05, 0.25]*dim, plus
    Rician noise sqrt((s + sigma n1)^2 + (sigma n2)^2).  float32, shape order
    (x, y, z) flattened with x fastest."""
    rng = np.random.default_rng(seed)
    X, Y, Z = shape
    gx, gy, gz = np.meshgrid(np.arange(X), np.arange(Y), np.arange(Z), indexing="ij")
    pts = np.stack([gx, gy, gz], axis=-1).astype(np.float32)
    vol = np.zeros(shape, dtype=np.float32)
    dimv = np.array(shape, dtype=np.float64)
    for _ in range(n_ell):
        c = rng.uniform(0.2, 0.8, 3) * dimv
        ax = rng.uniform(0.05, 0.25, 3) * dimv
        q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        amp = rng.uniform(0.2, 1.0)
        m = (q / ax[None, :]).astype(np.float32)      # D^{-1} R^T applied as (x-c) @ (R D^{-1})
        u = (pts - c.astype(np.float32)) @ m
        vol += amp * np.exp(-0.5 * np.sum(u * u, axis=-1))
    n1 = rng.standard_normal(shape).astype(np.float32)
    n2 = rng.standard_normal(shape).astype(np.float32)
    vol = np.sqrt((vol + sigma * n1) ** 2 + (sigma * n2) ** 2)
    return vol.reshape(-1, order="F").astype(np.float32)


def gaussian_tt_tensor_device(dims, ranks, noise_rel, seed, dtype="float32", device="cuda"):
    """The gaussian_tt_tensor recipe built with PyTorch on `device` (for tensors
    of many GB, e.g. 40^6 in FP32): the same seeded Gaussian cores, contracted
    as P = L R with L the left half-train over modes 1..h (rows, i_1 fastest)
    and R the right half-train over modes h+1..d (columns, i_{h+1} fastest);
    N i.i.d. N(0,1) from a seeded generator on `device`; beta = noise_rel *
    ||P||_F / ||N||_F.  Returns the flat tensor (i_1 fastest) in `dtype`."""
    import torch

    dims = [int(x) for x in dims]
    d = len(dims)
    ranks = list(ranks)
    if len(ranks) == d - 1:
        ranks = [1] + ranks + [1]
    cores = [torch.from_numpy(c).to(device) for c in gaussian_cores(dims, ranks, seed)]
    h = max(1, d // 2)
    L = cores[0][0]                                               # (I_1, r_1)
    for g in cores[1:h]:
        # rows (i_prev, i_k) with i_prev fastest
        L = torch.einsum("pa,aib->ipb", L, g).reshape(-1, g.shape[2])
    R = cores[d - 1][:, :, 0]                                      # (r_{d-1}, I_d)
    for g in cores[h:d - 1][::-1]:
        # columns (i_k, rest) with i_k fastest
        R = torch.einsum("aib,br->ari", g, R).reshape(g.shape[0], -1)
    dt = getattr(torch, dtype)
    P = (R.transpose(0, 1).to(dt) @ L.transpose(0, 1).to(dt)).reshape(-1)   # flat index row_L + |L| col_R
    if noise_rel > 0:
        gen = torch.Generator(device=device)
        gen.manual_seed(seed + 7919)
        N = torch.randn(P.numel(), generator=gen, dtype=dt, device=device)
        beta = noise_rel * float(torch.linalg.vector_norm(P, dtype=torch.float64)) / \
            float(torch.linalg.vector_norm(N, dtype=torch.float64))
        P.add_(N, alpha=beta)
        del N
    return P


def sin_norm_tensor_device(d, n, device="cuda"):
    """sin_norm_tensor built with PyTorch on `device` (float64): the squares are
    summed in index order k = 1..d by broadcasting, then sqrt and sin in place.
    The device's sqrt and sin may round differently from the host's by an ulp."""
    import torch

    x2 = (torch.arange(n, dtype=torch.float64, device=device) / (n - 1)) ** 2
    s = x2
    for k in range(1, d):
        # s holds modes 1..k (mode 1 fastest); mode k+1 becomes the new slowest axis
        s = s.reshape((1,) + tuple(s.shape)) + x2.reshape((n,) + (1,) * s.dim())
    s = s.reshape(-1)
    s.sqrt_()
    s.sin_()
    return s
