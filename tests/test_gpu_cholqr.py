"""The CholeskyQR3 orthonormaliser of the intermediate power iterates
(opts.orth = TT_ORTH_CHOLQR) against the oracle's Householder-based sweep:
both orthonormalise the same span, and the Rayleigh-Ritz step that fixes the
cores does not depend on the basis, so the cores agree to FP64 parity (1e-10
relative, with the bond sign gauge aligned).  Shapes: the 16^4 workload with
q = 2 (two intermediate iterates), iterates too tall for one workgroup's
Householder QR (1,280 x 40 on the 40^3 x 32 sweep), the 32^5 workload
(512 x 24 iterates), the fused-mixed form,
Alg. 4, prescribed accuracy, and an exact-rank input whose sketch is
rank-deficient (the shift keeps the first Cholesky factor positive definite)."""
import numpy as np
import pytest
import torch

import oracle
import ttgen

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2501_07904_amd")
from test_gpu_parity import ALL, _compare, _dev  # noqa: E402


def _both(a, dims, sweep, variant, **kw):
    A = _dev(a)
    c1, r1 = T.tt_utv_decompose(A, dims, sweep=sweep, variant=variant, orth="cholqr", **kw)
    c0, r0 = T.tt_utv_decompose(A, dims, sweep=sweep, variant=variant, **kw)
    torch.cuda.synchronize()
    return c1, r1, c0, r0


@pytest.mark.parametrize("sweep,variant", ALL)
def test_cholqr_matches_oracle_q2(sweep, variant):
    print(f"cholqr 16^4 q=2 {sweep}/{variant}", flush=True)
    dims = [16] * 4
    a, _ = ttgen.gaussian_tt_tensor(dims, [4, 6, 4], 1e-8, 400)
    c1, r1, _, r0 = _both(a, dims, sweep, variant, ranks=[4, 6, 4], q=2, oversample=8)
    oc, orep = oracle.tt_utv(a, dims, ranks=[4, 6, 4], sweep=sweep, variant=variant, q=2, p=8, seed=0)
    assert r1["ranks"] == orep["ranks"]
    _compare(c1, oc, sweep)


@pytest.mark.parametrize("sweep,variant", [("R2L", "URV"), ("L2R", "ULV")])
def test_cholqr_tall_iterate(sweep, variant):
    """n = 40 x 32 = 1280 rows on the core side: the Householder path would
    take the block-QR tree; CholeskyQR runs its Gram passes on many workgroups."""
    dims, ranks = [40, 40, 40], [32, 32]
    if sweep == "L2R":
        dims, ranks = dims[::-1], ranks[::-1]
    a, _ = ttgen.gaussian_tt_tensor(dims, ranks, 1e-6, 401)
    c1, r1, _, _ = _both(a, dims, sweep, variant, ranks=ranks, q=1, oversample=8)
    oc, orep = oracle.tt_utv(a, dims, ranks=ranks, sweep=sweep, variant=variant, q=1, p=8, seed=0)
    assert r1["ranks"] == orep["ranks"]
    _compare(c1, oc, sweep)


def test_cholqr_c2_shape():
    """The 32^5 workload (ranks 16, q = 2): 512 x 24 intermediate iterates."""
    dims, ranks = [32] * 5, [16] * 4
    a, _ = ttgen.gaussian_tt_tensor(dims, ranks, 1e-6, 0)
    c1, r1, _, _ = _both(a, dims, "R2L", "URV", ranks=ranks, q=2, oversample=8)
    oc, orep = oracle.tt_utv(a, dims, ranks=ranks, sweep="R2L", variant="URV", q=2, p=8, seed=0)
    assert r1["ranks"] == orep["ranks"]
    _compare(c1, oc, "R2L")


def test_cholqr_prescribed_accuracy_and_mixed():
    dims = [12, 11, 10, 9, 8]
    a, _ = ttgen.gaussian_tt_tensor(dims, [4, 6, 6, 4], 1e-5, 402)
    c1, r1, c0, r0 = _both(a, dims, "R2L", "URV", eps=1e-3, q=2, oversample=8)
    assert r1["ranks"] == r0["ranks"]
    rec1 = T.tt_reconstruct(c1).cpu().numpy()
    rec0 = T.tt_reconstruct(c0).cpu().numpy()
    assert np.linalg.norm(rec1 - rec0) <= 1e-10 * np.linalg.norm(rec0)
    assert np.linalg.norm(rec1 - a) <= 1e-3 * np.linalg.norm(a)
    # mixed form: FP32 power products, CholeskyQR on the FP64 reduced iterate
    A32 = _dev(a.astype(np.float32))
    cm, rm = T.tt_utv_decompose(A32, dims, ranks=[4, 6, 6, 4], sweep="R2L", variant="URV", q=2, prec="mixed",
                                orth="cholqr", exact_delta=True)
    recm = T.tt_reconstruct(cm).cpu().numpy()
    assert np.linalg.norm(recm - a.astype(np.float32)) <= rm["err_bound"] * (1 + 1e-9)


def test_cholqr_exact_rank_rank_deficient_sketch():
    dims = [6, 70, 5, 8]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 4, 3], 0.0, 403)
    for sweep, variant in ALL:
        cores, rep = T.tt_utv_decompose(_dev(a), dims, ranks=[3, 4, 3], sweep=sweep, variant=variant, q=2,
                                        oversample=8, orth="cholqr")
        rec = T.tt_reconstruct(cores).cpu().numpy()
        assert np.linalg.norm(rec - a) / np.linalg.norm(a) < 1e-12, (sweep, variant)
