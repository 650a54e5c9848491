"""Parity of the dense reconstruction's backward (tt_reconstruct_backward and
the TTReconstruct autograd function) with the oracle's gradient of
<gout, A_TT>, itself pinned on the CPU by central differences, Euler's
identity and the sampled-entry gradient."""
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


# shapes: the split of the train falls after core 1, in the middle and before
# the last core; d = 2; unit extents and unit ranks; extents and ranks off every
# 16/32/64 tile; the widest rank (64)
CASES = [
    ([5, 7, 6, 4, 9], [1, 3, 6, 5, 2, 1]),
    ([40, 3, 2, 2], [1, 5, 4, 3, 1]),
    ([2, 3, 2, 50], [1, 2, 4, 5, 1]),
    ([37, 29], [1, 11, 1]),
    ([3, 70], [1, 3, 1]),
    ([1, 6, 1, 5, 1], [1, 1, 4, 4, 2, 1]),
    ([17, 33, 9, 65], [1, 17, 33, 30, 1]),
    ([8, 8, 8, 8], [1, 8, 64, 8, 1]),
]


@pytest.mark.parametrize("dims,ranks", CASES)
@pytest.mark.parametrize("gdtype", [np.float64, np.float32])
def test_reconstruct_backward_matches_oracle(dims, ranks, gdtype):
    print(f"reconstruct backward dims={dims} ranks={ranks} gout={np.dtype(gdtype).name}", flush=True)
    cores_np = ttgen.gaussian_cores(dims, ranks, 200 + len(dims))
    gout = np.random.default_rng(201).standard_normal(int(np.prod(dims))).astype(gdtype)
    cores = [_dev(c) for c in cores_np]
    grads = T.tt_reconstruct_backward(cores, _dev(gout))
    torch.cuda.synchronize()
    want = oracle.tt_reconstruct_grad(cores_np, gout.astype(np.float64))
    for k, (g, w) in enumerate(zip(grads, want)):
        assert tuple(g.shape) == w.shape
        assert _rel(g.cpu().numpy(), w) <= 1e-12, f"core {k + 1}: {_rel(g.cpu().numpy(), w):.3e}"


def test_reconstruct_backward_bitwise_reproducible():
    dims, ranks = [16, 12, 10, 14, 8], [1, 9, 16, 12, 7, 1]
    cores = [_dev(c) for c in ttgen.gaussian_cores(dims, ranks, 210)]
    gout = _dev(np.random.default_rng(211).standard_normal(int(np.prod(dims))))
    g1 = T.tt_reconstruct_backward(cores, gout)
    g2 = T.tt_reconstruct_backward(cores, gout)
    for a, b in zip(g1, g2):
        assert torch.equal(a, b)


def test_reconstruct_autograd_function():
    """TTReconstruct: the loss 0.5 ||A_TT - M||^2 differentiated by autograd
    through the hand-written backward equals the oracle's gradient with
    gout = A_TT - M."""
    dims, ranks = [6, 5, 7, 4], [1, 3, 5, 2, 1]
    cores_np = ttgen.gaussian_cores(dims, ranks, 220)
    M = np.random.default_rng(221).standard_normal(int(np.prod(dims)))
    cores = [_dev(c).requires_grad_(True) for c in cores_np]
    full = T.TTReconstruct.apply(*cores)
    loss = 0.5 * ((full - _dev(M)) ** 2).sum()
    loss.backward()
    gout = oracle.tt_reconstruct(cores_np) - M
    want = oracle.tt_reconstruct_grad(cores_np, gout)
    for c, w in zip(cores, want):
        assert _rel(c.grad.cpu().numpy(), w) <= 1e-11


def test_reconstruct_backward_full_size_order5_32():
    """The 32^5 train of ranks 16 (33.5M entries, a 268 MB upstream gradient,
    split after core 3): every core gradient against the oracle's."""
    dims, ranks = [32] * 5, [1, 16, 16, 16, 16, 1]
    cores_np = ttgen.gaussian_cores(dims, ranks, 230)
    gout = np.random.default_rng(231).standard_normal(32 ** 5)
    cores = [_dev(c) for c in cores_np]
    grads = T.tt_reconstruct_backward(cores, _dev(gout))
    torch.cuda.synchronize()
    want = oracle.tt_reconstruct_grad(cores_np, gout)
    for k, (g, w) in enumerate(zip(grads, want)):
        assert _rel(g.cpu().numpy(), w) <= 1e-12, f"core {k + 1}"
