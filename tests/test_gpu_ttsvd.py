"""TT-SVD through the C ABI against the oracle's TT-SVD (LAPACK SVD of every
unfolding) on core sides above 64, where the library runs subspace iteration on
the leading 64 directions (30 power steps): the 32^5 FP64 workload at fixed rank
16 in both sweep directions, ragged shapes, a prescribed accuracy, and the
steps on either side of the switch (core sides 64 and 65).  Cores at
1e-10 where the singular values are well separated, the reconstruction and the
step errors always."""
import numpy as np
import pytest
import torch

import oracle
import ttgen

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2501_07904_amd")
TOL = 1e-10


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(cores):
    return [c.detach().cpu().numpy() for c in cores]


def _align(gpu, ora, sweep):
    gpu = [g.copy() for g in gpu]
    for k in range(len(gpu) - 1):
        if sweep == "L2R":
            s = np.sign(np.einsum("aib,aib->b", gpu[k], ora[k]))
        else:
            s = np.sign(np.einsum("aib,aib->a", gpu[k + 1], ora[k + 1]))
        s[s == 0] = 1
        gpu[k] = gpu[k] * s[None, None, :]
        gpu[k + 1] = gpu[k + 1] * s[:, None, None]
    return gpu


def _check(a, dims, cores, rep, oc, orep, sweep):
    assert rep["ranks"] == orep["ranks"]
    g = _align(_np(cores), oc, sweep)
    for k, (x, y) in enumerate(zip(g, oc)):
        assert x.shape == y.shape
        err = np.max(np.abs(x - y)) / max(np.max(np.abs(y)), 1e-300)
        assert err <= TOL, f"core {k + 1}: rel err {err:.3e}"
    rec = T.tt_reconstruct(cores).cpu().numpy()
    np.testing.assert_allclose(rec, oracle.tt_reconstruct(oc), rtol=0, atol=TOL * np.max(np.abs(a)))
    nA2 = orep["norm_A"] ** 2
    for x, y in zip(rep["delta"], orep["delta"]):
        assert abs(x * x - y * y) <= 1e-13 * nA2


@pytest.mark.parametrize("sweep", ["R2L", "L2R"])
def test_c2_order5_32_fixed_rank(sweep):
    """The 32^5 workload (Gaussian-TT ranks 16 + 1e-6 noise): the 32,768 x 512
    and 1,024 x 512 unfoldings take the iterative path."""
    dims = [32] * 5
    a, _ = ttgen.gaussian_tt_tensor(dims, [16] * 4, 1e-6, 0)
    print(f"TT-SVD 32^5 {sweep}", flush=True)
    cores, rep = T.tt_utv_decompose(_dev(a), dims, ranks=[16] * 4, sweep=sweep, variant="SVD")
    cores = [c.clone() for c in cores]
    oc, orep = oracle.tt_svd(a, dims, ranks=[16] * 4, sweep=sweep)
    _check(a, dims, cores, rep, oc, orep, sweep)


@pytest.mark.parametrize("sweep", ["R2L", "L2R"])
def test_ragged_and_prescribed_accuracy(sweep):
    """Core sides 70-300 off every tile, fixed ranks and eps = 1e-3 (ranks equal
    to the oracle's TT-SVD ranks, RSE within eps)."""
    dims = [10, 14, 9, 33]
    a, _ = ttgen.gaussian_tt_tensor(dims, [6, 20, 9], 1e-4, 7)
    print(f"TT-SVD ragged {sweep}", flush=True)
    A = _dev(a)
    cores, rep = T.tt_utv_decompose(A, dims, ranks=[6, 20, 9], sweep=sweep, variant="SVD")
    cores = [c.clone() for c in cores]
    oc, orep = oracle.tt_svd(a, dims, ranks=[6, 20, 9], sweep=sweep)
    _check(a, dims, cores, rep, oc, orep, sweep)
    cores, rep = T.tt_utv_decompose(A, dims, eps=1e-3, sweep=sweep, variant="SVD")
    oc, orep = oracle.tt_svd(a, dims, eps=1e-3, sweep=sweep)
    assert rep["ranks"] == orep["ranks"]
    rec = T.tt_reconstruct(cores).cpu().numpy()
    np.testing.assert_allclose(rec, oracle.tt_reconstruct(oc), rtol=0, atol=TOL * np.max(np.abs(a)))
    assert np.linalg.norm(rec - a) <= 1e-3 * np.linalg.norm(a)


@pytest.mark.parametrize("sweep", ["L2R", "R2L"])
def test_exact_and_subspace_steps_at_the_boundary(sweep):
    """Consecutive steps on either side of the switch: core side 64 (the exact
    step, l = n with G = I, in Gram mode) and 65 (subspace iteration on 64
    directions, m = 100 rows on the long side)."""
    dims, ranks = [8, 8, 13, 100], [8, 5, 10]
    if sweep == "R2L":
        dims, ranks = dims[::-1], ranks[::-1]
    print(f"tt-svd boundary {dims} {ranks} {sweep}", flush=True)
    a, _ = ttgen.gaussian_tt_tensor(dims, ranks, 1e-4, 9)
    cores, rep = T.tt_utv_decompose(_dev(a), dims, ranks=ranks, sweep=sweep, variant="SVD")
    torch.cuda.synchronize()
    oc, orep = oracle.tt_svd(a, dims, ranks=ranks, sweep=sweep)
    _check(a, dims, cores, rep, oc, orep, sweep)
    # the sketch widths per bond: n on the exact steps (8 and 64), 64 on the wide one
    assert rep["ell"] == ([8, 64, 64] if sweep == "L2R" else [64, 64, 8])
