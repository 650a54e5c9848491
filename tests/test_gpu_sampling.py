"""Sampled entries of a train and their backward (tt_sample,
tt_sample_backward(_mixed)) against the oracle's Eq. (TT) products and its
gradient (pinned on the CPU by central differences): every register width of
the one-sample-per-thread kernels (ranks <= 8, 16, 32), the wave-per-sample
kernels of wider trains, FP32 cores, cores too large for LDS, gradients
larger than one LDS range, several blocks of 2^20 samples, and bitwise
reproducibility of the backward on the completion shape."""
import numpy as np
import pytest
import torch

import oracle
import ttgen

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2501_07904_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(x, y):
    return float(np.max(np.abs(x - y)) / max(np.max(np.abs(y)), 1e-300))


CASES = [
    ([5, 7, 6, 4, 9], [1, 3, 6, 5, 2, 1], 5000),          # ranks <= 8
    ([16, 16, 16, 16, 16, 10], [1, 16, 16, 16, 16, 10, 1], 20000),   # the completion shape, ranks 16
    ([9, 11, 7, 13], [1, 9, 32, 11, 1], 7000),             # ranks <= 32, odd and even strides
    ([40, 40, 40], [1, 24, 24, 1], 20000),                 # cores beyond LDS, gradient beyond one LDS range
    ([37, 29], [1, 11, 1], 3000),                          # d = 2
    ([1, 6, 1, 5, 1], [1, 1, 4, 4, 2, 1], 500),            # unit extents and ranks
    ([8, 8, 8, 8], [1, 8, 40, 8, 1], 4000),                # a rank above 32: wave-per-sample kernels
]


@pytest.mark.parametrize("dims,ranks,N", CASES)
def test_sample_and_backward_match_oracle(dims, ranks, N):
    print(f"sampling dims={dims} ranks={ranks} N={N}", flush=True)
    cores_np = ttgen.gaussian_cores(dims, ranks, 300 + len(dims))
    cores = [_dev(c) for c in cores_np]
    idx = ttgen.random_indices(dims, N, 301)
    w = np.random.default_rng(302).standard_normal(N)
    vals = T.tt_sample(cores, _dev(idx)).cpu().numpy()
    assert _rel(vals, oracle.tt_sample(cores_np, idx)) <= 1e-12
    grads = T.tt_sample_backward(cores, _dev(idx), _dev(w))
    for k, (g, o) in enumerate(zip(grads, oracle.tt_sample_grad(cores_np, idx, w))):
        assert g.dtype == torch.float64 and tuple(g.shape) == o.shape
        assert _rel(g.cpu().numpy(), o) <= 1e-11, f"core {k + 1}: {_rel(g.cpu().numpy(), o):.3e}"


@pytest.mark.parametrize("dims,ranks,N", CASES[:4])
def test_mixed_point_backward_matches_oracle(dims, ranks, N):
    cores_np = ttgen.gaussian_cores(dims, ranks, 310)
    Lc = oracle.left_orthogonalize(cores_np)
    Rc = oracle.right_orthogonalize(cores_np)
    idx = ttgen.random_indices(dims, N, 311)
    w = np.random.default_rng(312).standard_normal(N)
    grads = T.tt_sample_backward_mixed([_dev(c) for c in Lc], [_dev(c) for c in Rc], _dev(idx), _dev(w))
    for k, (g, o) in enumerate(zip(grads, oracle.tt_sample_grad_mixed(Lc, Rc, idx, w))):
        assert _rel(g.cpu().numpy(), o) <= 1e-11, f"core {k + 1}"


def test_fp32_cores():
    """FP32 cores are read as they are and multiplied in FP64: the values equal
    the oracle's on the same (FP32-rounded) cores; gradients come back in FP32,
    the FP64 sums rounded once."""
    dims, ranks = [16, 16, 16, 16, 16, 10], [1, 16, 16, 16, 16, 10, 1]
    c64 = ttgen.gaussian_cores(dims, ranks, 320)
    c32 = [c.astype(np.float32) for c in c64]
    up = [c.astype(np.float64) for c in c32]
    idx = ttgen.random_indices(dims, 30000, 321)
    w = np.random.default_rng(322).standard_normal(30000)
    vals = T.tt_sample([_dev(c) for c in c32], _dev(idx)).cpu().numpy()
    assert _rel(vals, oracle.tt_sample(up, idx)) <= 1e-12
    grads = T.tt_sample_backward([_dev(c) for c in c32], _dev(idx), _dev(w))
    for g, o in zip(grads, oracle.tt_sample_grad(up, idx, w)):
        assert g.dtype == torch.float32
        np.testing.assert_allclose(g.cpu().numpy(), o.astype(np.float32), rtol=2e-7, atol=1e-6 * np.max(np.abs(o)))


def test_backward_over_several_sample_blocks():
    """More than 2^20 samples run as several blocks whose partial gradients
    carry over: the gradient is linear in gout, so it equals the sum of the
    gradients of the two halves (each one block)."""
    dims, ranks = [6, 5, 7, 4], [1, 3, 4, 2, 1]
    cores = [_dev(c) for c in ttgen.gaussian_cores(dims, ranks, 330)]
    N = (1 << 20) + 54321
    idx = _dev(ttgen.random_indices(dims, N, 331))
    w = _dev(np.random.default_rng(332).standard_normal(N))
    full = T.tt_sample_backward(cores, idx, w)
    cut = 1 << 20
    a = T.tt_sample_backward(cores, idx[:cut].contiguous(), w[:cut].contiguous())
    b = T.tt_sample_backward(cores, idx[cut:].contiguous(), w[cut:].contiguous())
    for f, x, y in zip(full, a, b):
        assert _rel(f.cpu().numpy(), (x + y).cpu().numpy()) <= 1e-12


def test_backward_bitwise_reproducible_on_the_completion_shape():
    dims, ranks = [16, 16, 16, 16, 16, 10], [1, 16, 16, 16, 16, 10, 1]
    cores = [_dev(c) for c in ttgen.gaussian_cores(dims, ranks, 340)]
    idx = _dev(ttgen.random_indices(dims, 3145728, 341))
    w = _dev(np.random.default_rng(342).standard_normal(3145728))
    g1 = T.tt_sample_backward(cores, idx, w)
    g2 = T.tt_sample_backward(cores, idx, w)
    for x, y in zip(g1, g2):
        assert torch.equal(x, y)
    # and the values against the oracle on a sample of the entries' samples:
    # the gradient of the first 50,000 samples
    sub = 50000
    gs = T.tt_sample_backward(cores, idx[:sub].contiguous(), w[:sub].contiguous())
    cn = [c.cpu().numpy() for c in cores]
    for g, o in zip(gs, oracle.tt_sample_grad(cn, idx[:sub].cpu().numpy(), w[:sub].cpu().numpy())):
        assert _rel(g.cpu().numpy(), o) <= 1e-11


def test_empty_sample_set():
    dims, ranks = [4, 5, 3], [1, 2, 3, 1]
    cores = [_dev(c) for c in ttgen.gaussian_cores(dims, ranks, 350)]
    idx = torch.zeros((0, 3), dtype=torch.int64, device="cuda")
    assert T.tt_sample(cores, idx).numel() == 0
    for g in T.tt_sample_backward(cores, idx, torch.zeros(0, dtype=torch.float64, device="cuda")):
        assert torch.count_nonzero(g) == 0
