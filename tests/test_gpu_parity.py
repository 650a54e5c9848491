"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Every case runs the same seeded input and the same Gaussian test-matrix spec
on both sides.  Cores are compared after aligning the sign gauge of every TT
bond (the only freedom left once both sides canonicalise signs), the
reconstruction and the step errors directly.  FP64 tolerance: 1e-10 relative.
"""
import math

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
    """Flip the sign gauge of each bond of `gpu` to best match `ora`."""
    gpu = [g.copy() for g in gpu]
    d = len(gpu)
    for k in range(d - 1):
        if sweep == "L2R":      # bond k between core k (left-orthogonal, last index) and core k+1
            s = np.sign(np.einsum("aib,aib->b", gpu[k], ora[k]))
        else:                    # core k+1 is right-orthogonal (first index)
            s = np.sign(np.einsum("aib,aib->a", gpu[k + 1], ora[k + 1]))
        s[s == 0] = 1
        gpu[k] = gpu[k] * s[None, None, :]
        gpu[k + 1] = gpu[k + 1] * s[:, None, None]
    return gpu


def _compare(gpu_cores, ora_cores, sweep, tol=TOL):
    g = _align(_np(gpu_cores), ora_cores, sweep)
    assert [x.shape for x in g] == [x.shape for x in ora_cores]
    for k, (x, y) in enumerate(zip(g, ora_cores)):
        err = np.max(np.abs(x - y)) / max(np.max(np.abs(y)), 1e-300)
        assert err <= tol, f"core {k + 1}: rel err {err:.3e}"


def _compare_conditioned(gpu_cores, ora_cores, svals, sweep, tol=1e-8, floor=1e-4, gap=1e-3):
    """Orthogonal cores column by column, only for singular directions that
    are well determined in FP64: s_a >= floor * s_1 and relative gap to both
    neighbours >= gap.  Directions near s_1 * 1e-7 are fixed only to about
    u (s_1/s_a)^2 by any FP64 method that forms a Gram matrix."""
    g = _align(_np(gpu_cores), ora_cores, sweep)
    d = len(g)
    checked = 0
    for k in range(d - 1):
        s = np.asarray(svals[k])
        r = ora_cores[k].shape[2] if sweep == "L2R" else ora_cores[k + 1].shape[0]
        for a in range(r):
            if s[a] < floor * s[0]:
                continue
            lo = abs(s[a] - s[a + 1]) / s[0] if a + 1 < len(s) else 1.0
            hi = abs(s[a - 1] - s[a]) / s[0] if a > 0 else 1.0
            if min(lo, hi) < gap:
                continue
            x = g[k][:, :, a] if sweep == "L2R" else g[k + 1][a]
            y = ora_cores[k][:, :, a] if sweep == "L2R" else ora_cores[k + 1][a]
            err = np.max(np.abs(x - y))
            assert err <= tol, f"bond {k + 1} column {a}: {err:.3e}"
            checked += 1
    assert checked > 0


U64 = 2.0 ** -53


def _gram_floor_tol(orep, ranks, sweep):
    """Tolerance for comparing a prescribed-accuracy reconstruction with the
    oracle's, relative to ||A||_F.  The library takes the Rayleigh-Ritz
    factorisation of each step from the eigenvectors of the Gram matrix
    (AX)^T(AX), whose squared spectrum fixes the kept subspace only to about
    u s_1^2 / (s_r^2 - s_{r+1}^2) (Davis-Kahan with a Gram perturbation of
    u s_1^2); turning the subspace by that angle changes the rank-r part C V1
    V1^T by that angle times s_r.  Summed over the steps (the later steps see
    the perturbation linearly), with a factor 64 for the dimension-dependent
    constants of the rounding bounds, floored at the FP64 target 1e-10."""
    tol = 0.0
    nA = orep["norm_A"]
    d = len(ranks) - 1
    for k in range(d - 1):
        s = np.asarray(orep["s"][k], dtype=np.float64)
        r = ranks[k + 1] if sweep == "L2R" else ranks[k + 1]
        if r >= len(s):
            continue
        gap = s[r - 1] ** 2 - s[r] ** 2
        if gap <= 0:
            return float("inf")
        tol += U64 * s[0] ** 2 / gap * s[r - 1] / nA
    return max(1e-10, 64.0 * tol)


def _compare_reconstruction(cores, oc, orep, sweep):
    rec = T.tt_reconstruct(cores).cpu().numpy()
    orec = oracle.tt_reconstruct(oc)
    diff = np.linalg.norm(rec - orec) / orep["norm_A"]
    tol = _gram_floor_tol(orep, orep["ranks"], sweep)
    print(f"reconstruction vs oracle: {diff:.3e} (tolerance {tol:.3e})", flush=True)
    assert diff <= tol, (diff, tol)
    return rec


def _run(a, dims, sweep, variant, ranks=None, eps=None, q=1, p=8, seed=0, dtype=np.float64, **kw):
    A = _dev(a.astype(dtype))
    cores, rep = T.tt_utv_decompose(A, dims, ranks=ranks, eps=eps, sweep=sweep, variant=variant, q=q,
                                    oversample=p, seed=seed, **kw)
    torch.cuda.synchronize()
    oc, orep = oracle.tt_utv(a.astype(dtype).astype(np.float64), dims, ranks=ranks, eps=eps, sweep=sweep,
                             variant=variant, q=q, p=p, seed=seed)
    return cores, rep, oc, orep


COMBOS = [("R2L", "URV"), ("L2R", "ULV"), ("L2R", "URV")]
ALG4 = ("R2L", "ULV")           # appendix sweep: ULV factors, right-to-left
ALL = COMBOS + [ALG4]


# --------------------------------------------------------------------- generator
def test_sketch_matches_oracle_spec():
    """The device Gaussian test matrix equals the oracle's bit-for-bit up to
    libm rounding of log/cos (checked through a d = 2 sweep with q = 0 whose
    first product is A G: identical cores need identical G)."""
    dims = [40, 30]
    rng = np.random.default_rng(1)
    a = rng.standard_normal(40 * 30)
    for sweep, variant in ALL:
        cores, rep, oc, orep = _run(a, dims, sweep, variant, ranks=[5], q=0, p=3, seed=77)
        # a full-rank random matrix: the rank-5 subspace found by one sketch depends on G
        _compare(cores, oc, sweep, tol=1e-9)


# --------------------------------------------------------------------- fixed ranks
@pytest.mark.parametrize("sweep,variant", ALL)
def test_c1_order4_16(sweep, variant):
    """16^4 Gaussian-TT tensor, ranks (1,4,6,4,1), noise 1e-8, q = 1."""
    dims = [16] * 4
    a, _ = ttgen.gaussian_tt_tensor(dims, [4, 6, 4], 1e-8, 100)
    cores, rep, oc, orep = _run(a, dims, sweep, variant, ranks=[4, 6, 4], q=1, exact_delta=True)
    assert rep["ranks"] == orep["ranks"] == [1, 4, 6, 4, 1]
    _compare(cores, oc, sweep)
    rec = T.tt_reconstruct(cores).cpu().numpy()
    np.testing.assert_allclose(rec, oracle.tt_reconstruct(oc), rtol=0, atol=TOL * np.max(np.abs(a)))
    np.testing.assert_allclose(rep["delta"], orep["delta"], rtol=1e-6)
    assert rep["norm_A"] == pytest.approx(orep["norm_A"], rel=1e-13)
    assert rep["err_bound"] == pytest.approx(orep["err_bound"], rel=1e-6)
    # equality for the Pythagorean sweeps; the error itself is formed by cancellation
    assert np.linalg.norm(rec - a) <= rep["err_bound"] * (1 + 1e-6)
    # measured step errors make the reported bound a bound; the default run says it is an estimate
    assert rep["err_bound_measured"]
    _, rep0 = T.tt_utv_decompose(_dev(a), dims, ranks=[4, 6, 4], sweep=sweep, variant=variant, q=1)
    assert not rep0["err_bound_measured"]


@pytest.mark.parametrize("sweep,variant", ALL)
def test_gram_and_sketched_steps_at_the_switch(sweep, variant):
    """Consecutive steps with core sides 64 (the largest Gram-mode step: A^T A
    in one pass and the solve in one workgroup) and 65 (the smallest sketched
    step, l = 18)."""
    dims, ranks = [8, 8, 13, 100], [8, 5, 10]
    if sweep == "R2L":
        dims, ranks = dims[::-1], ranks[::-1]
    print(f"gram/sketch switch {dims} {ranks} {sweep}/{variant}", flush=True)
    a, _ = ttgen.gaussian_tt_tensor(dims, ranks, 1e-6, 110)
    cores, rep, oc, orep = _run(a, dims, sweep, variant, ranks=ranks, q=1, exact_delta=True)
    assert rep["ranks"] == orep["ranks"]
    assert rep["ell"] == [int(x) for x in orep["ell"]]
    _compare(cores, oc, sweep)
    rec = T.tt_reconstruct(cores).cpu().numpy()
    np.testing.assert_allclose(rec, oracle.tt_reconstruct(oc), rtol=0, atol=TOL * np.max(np.abs(a)))
    # the step whose rank equals its core side (8) truncates nothing: its error is rounding on both sides
    np.testing.assert_allclose(rep["delta"], orep["delta"], rtol=1e-6, atol=TOL * orep["norm_A"])


@pytest.mark.parametrize("sweep,variant", ALL)
def test_ragged_shapes(sweep, variant):
    """Extents and ranks that are not multiples of any tile; a step with n > 64
    (the sketched path) and one with m < n."""
    dims = [7, 13, 11, 9, 5]
    a, _ = ttgen.gaussian_tt_tensor(dims, [5, 9, 7, 4], 1e-6, 101)
    cores, rep, oc, orep = _run(a, dims, sweep, variant, ranks=[5, 9, 7, 4], q=2, p=5, exact_delta=True)
    assert rep["ranks"] == orep["ranks"]
    _compare(cores, oc, sweep)
    np.testing.assert_allclose(rep["delta"], orep["delta"], rtol=1e-6)


@pytest.mark.parametrize("sweep,variant", [("R2L", "URV"), ("L2R", "ULV")])
def test_partial_product_chunk_edges(sweep, variant):
    """More row tiles than the 512 row chunks a partial-product pass uses, with
    m not a multiple of a chunk's rows, so that the last chunks are short or
    empty and must add zero: the first step's Gram pass over 25,110 (R2L,
    column-major, vector loads) or 19,251 (L2R, row-major) rows, then power
    products and the Gram of A X over 930 rows."""
    dims = [30, 31, 27, 23]
    ranks = [6, 10, 8]
    a, _ = ttgen.gaussian_tt_tensor(dims, ranks, 1e-6, 202)
    cores, rep, oc, orep = _run(a, dims, sweep, variant, ranks=ranks, q=2, p=8, exact_delta=True)
    assert rep["ranks"] == orep["ranks"]
    _compare(cores, oc, sweep)
    np.testing.assert_allclose(rep["delta"], orep["delta"], rtol=1e-6)


@pytest.mark.parametrize("dims,ranks,p", [
    ([200, 30, 40], [8, 36], 8),      # ell = 16, n = 1080 > 1024 rows: two leaf blocks
    ([200, 30, 20], [16, 18], 8),     # ell = 24, n = 540 > 512
    ([300, 30, 20], [24, 18], 16),    # ell = 40, n = 540 > 256: three leaf blocks
    ([100, 30, 60], [24, 56], 16),    # ell = 40, n = 1680: seven leaf blocks whose stacked R is split again
    ([300, 30, 20], [56, 18], 8),     # ell = 64, the widest iterate, n = 540
])
@pytest.mark.parametrize("sweep,variant", [("R2L", "URV"), ("L2R", "ULV")])
def test_tall_iterate_tree_qr(dims, ranks, p, sweep, variant):
    """Core-side iterates taller than one register-resident QR block take the
    tree (TSQR) orthonormalisation: same cores as the oracle's Householder QR."""
    if sweep == "L2R":
        dims, ranks = dims[::-1], ranks[::-1]
    a, _ = ttgen.gaussian_tt_tensor(dims, ranks, 1e-6, 106)
    cores, rep, oc, orep = _run(a, dims, sweep, variant, ranks=ranks, q=1, p=p, exact_delta=True)
    assert rep["ranks"] == orep["ranks"]
    _compare(cores, oc, sweep)
    np.testing.assert_allclose(rep["delta"], orep["delta"], rtol=1e-6)


@pytest.mark.parametrize("dims,ranks,p", [
    ([37, 11, 40], [6, 9], 8),       # step 2: m = 37 (a partial row tile), n = 99, ell = 14 (one column tile)
    ([500, 12, 30], [20, 10], 8),    # m = 500, n = 120, ell = 28 (two column tiles)
    ([300, 16, 32], [19, 28], 8),    # n = 448, ell = 27: n ell = 12096 near the staged-X limit
])
@pytest.mark.parametrize("variant", ["URV", "ULV"])
@pytest.mark.parametrize("fuse", [True, False])
def test_one_pass_power_product(dims, ranks, p, variant, fuse):
    """Right-to-left power steps with A^T (A X) formed in one pass over A
    (fuse_ata) and in two (the default): both give the oracle's cores."""
    a, _ = ttgen.gaussian_tt_tensor(dims, ranks, 1e-6, 107)
    cores, rep, oc, orep = _run(a, dims, "R2L", variant, ranks=ranks, q=2, p=p, exact_delta=True, fuse_ata=fuse)
    assert rep["ranks"] == orep["ranks"]
    _compare(cores, oc, "R2L")
    np.testing.assert_allclose(rep["delta"], orep["delta"], rtol=1e-6)


@pytest.mark.parametrize("sweep,variant", COMBOS)
def test_truncation_below_true_rank(sweep, variant):
    """Ranks below the generating ranks: real truncation with well-separated spectra."""
    dims = [9, 10, 8, 11]
    a, _ = ttgen.gaussian_tt_tensor(dims, [6, 8, 6], 1e-3, 102)
    cores, rep, oc, orep = _run(a, dims, sweep, variant, ranks=[3, 4, 3], q=3, p=6, exact_delta=True)
    a_hat = T.tt_reconstruct(cores).cpu().numpy()
    o_hat = oracle.tt_reconstruct(oc)
    np.testing.assert_allclose(a_hat, o_hat, rtol=0, atol=1e-9 * np.max(np.abs(o_hat)))
    # Pythagoras equality of the step errors holds on the device result too
    err2 = np.sum((a_hat - a) ** 2)
    assert abs(err2 - rep["err_bound"] ** 2) <= 1e-8 * err2


@pytest.mark.parametrize("q", [0, 1, 3])
def test_alg4_truncation_sum_bound(q):
    """Appendix sweep (ULV, right-to-left) with real truncation: the carry is
    U_hat L11 without the U2 L21 term, so at q = 0 the result differs from
    TT-URV's (checked on the oracle side) and must match the oracle's Alg. 4;
    the error obeys the sum bound ||A - A_hat|| <= sum_k delta_k."""
    dims = [9, 10, 8, 11]
    a, _ = ttgen.gaussian_tt_tensor(dims, [6, 8, 6], 1e-3, 102)
    cores, rep, oc, orep = _run(a, dims, "R2L", "ULV", ranks=[3, 4, 3], q=q, p=6, exact_delta=True)
    a_hat = T.tt_reconstruct(cores).cpu().numpy()
    o_hat = oracle.tt_reconstruct(oc)
    np.testing.assert_allclose(a_hat, o_hat, rtol=0, atol=1e-9 * np.max(np.abs(o_hat)))
    np.testing.assert_allclose(rep["delta"], orep["delta"], rtol=1e-8)
    assert rep["err_bound"] == pytest.approx(sum(orep["delta"]), rel=1e-8)
    assert np.linalg.norm(a_hat - a) <= rep["err_bound"]
    if q == 0:
        ou, _ = oracle.tt_utv(a, dims, ranks=[3, 4, 3], sweep="R2L", variant="URV", q=0, p=6)
        assert np.linalg.norm(oracle.tt_reconstruct(ou) - o_hat) > 1e-6 * np.linalg.norm(a)


def test_exact_rank_no_noise_rank_deficient_sketch():
    """Exact TT-ranks and ell > rank: the sketch is rank-deficient; the
    Householder orthonormalisation keeps the basis orthonormal."""
    dims = [6, 70, 5, 8]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 4, 3], 0.0, 103)
    for sweep, variant in ALL:
        A = _dev(a)
        cores, rep = T.tt_utv_decompose(A, dims, ranks=[3, 4, 3], sweep=sweep, variant=variant, q=1, oversample=8)
        rec = T.tt_reconstruct(cores).cpu().numpy()
        assert np.linalg.norm(rec - a) / np.linalg.norm(a) < 1e-12


def test_tt_svd_variant_small_n():
    dims = [8, 6, 7, 5]
    a, _ = ttgen.gaussian_tt_tensor(dims, [4, 5, 4], 1e-2, 104)
    for sweep in ("L2R", "R2L"):
        A = _dev(a)
        cores, rep = T.tt_utv_decompose(A, dims, ranks=[3, 4, 3], sweep=sweep, variant="SVD")
        oc, orep = oracle.tt_svd(a, dims, ranks=[3, 4, 3], sweep=sweep)
        _compare(cores, oc, sweep)


def test_order2_matrix():
    rng = np.random.default_rng(5)
    a = rng.standard_normal(37 * 53)
    for sweep, variant in ALL:
        cores, rep, oc, orep = _run(a, [37, 53], sweep, variant, ranks=[6], q=2, p=4)
        _compare(cores, oc, sweep, tol=1e-9)


def test_unit_extents():
    dims = [1, 9, 1, 12, 1]
    a, _ = ttgen.gaussian_tt_tensor(dims, [1, 3, 3, 1], 1e-5, 105)
    for sweep, variant in ALL:
        cores, rep, oc, orep = _run(a, dims, sweep, variant, ranks=[1, 3, 3, 1], q=1)
        _compare(cores, oc, sweep)


def test_c2_full_size_order5_32():
    """32^5 (33.5M entries), ranks 16, noise 1e-6, q = 2: the full benchmark
    workload against the oracle, both recommended sweeps."""
    dims = [32] * 5
    a, _ = ttgen.gaussian_tt_tensor(dims, [16] * 4, 1e-6, 0)
    A = _dev(a)
    for sweep, variant in (("R2L", "URV"), ("L2R", "ULV")):
        cores, rep = T.tt_utv_decompose(A, dims, ranks=[16] * 4, sweep=sweep, variant=variant, q=2,
                                        oversample=8, seed=1, exact_delta=True)
        oc, orep = oracle.tt_utv(a, dims, ranks=[16] * 4, sweep=sweep, variant=variant, q=2, p=8, seed=1)
        _compare(cores, oc, sweep)
        # step errors measured directly (exact_delta) agree to their own rounding
        np.testing.assert_allclose(rep["delta"], orep["delta"], rtol=1e-7)
        assert rep["err_bound"] == pytest.approx(orep["err_bound"], rel=1e-7)
        # the default report takes delta^2 = ||C||^2 - ||carry||^2: its error is
        # about u * m * ||C||^2 / delta^2 relative, so only a loose check applies
        _, rep2 = T.tt_utv_decompose(A, dims, ranks=[16] * 4, sweep=sweep, variant=variant, q=2,
                                     oversample=8, seed=1)
        assert rep2["err_bound"] == pytest.approx(orep["err_bound"], rel=1e-2)


def test_jacobi_stops_at_the_rounding_floor():
    """32^5 with the one-pass power products, whose rounding once kept the
    threshold-only Jacobi rule rotating noise to its 30-sweep cap on the third
    unfolding: the solver now stops when sweeps no longer shrink the
    off-diagonal mass, with the oracle's cores."""
    dims = [32] * 5
    a, _ = ttgen.gaussian_tt_tensor(dims, [16] * 4, 1e-6, 0)
    cores, rep = T.tt_utv_decompose(_dev(a), dims, ranks=[16] * 4, sweep="R2L", variant="URV", q=2,
                                    oversample=8, seed=1, fuse_ata=True)
    assert max(rep["sweeps"]) <= 12, rep["sweeps"]
    oc, _ = oracle.tt_utv(a, dims, ranks=[16] * 4, sweep="R2L", variant="URV", q=2, p=8, seed=1)
    _compare(cores, oc, "R2L")


# --------------------------------------------------------------------- prescribed accuracy
@pytest.mark.parametrize("sweep,variant", ALL)
def test_eps_mode_function_tensor(sweep, variant):
    a = ttgen.inverse_sum_tensor(6, 8, dtype=np.float64)
    dims = [8] * 6
    for eps in (1e-3, 1e-6):
        cores, rep, oc, orep = _run(a, dims, sweep, variant, eps=eps, q=1, p=4, seed=2, exact_delta=True)
        assert rep["ranks"] == orep["ranks"]
        assert rep["rank_rule_met"]
        _compare_conditioned(cores, oc, orep["s"], sweep)
        rec = _compare_reconstruction(cores, oc, orep, sweep)
        assert np.linalg.norm(rec - a) / np.linalg.norm(a) <= eps
        np.testing.assert_allclose(rep["delta"], orep["delta"], rtol=1e-3, atol=1e-3 * eps * orep["norm_A"])


@pytest.mark.parametrize("sweep,variant", [("R2L", "URV"), ("L2R", "ULV")])
def test_eps_mode_retries_and_step_norms(sweep, variant):
    """Prescribed accuracy with a small oversampling, so that later steps widen
    their sketch and run their solve again (the same widths as the oracle's);
    each step's ||C|| is the previous carry's norm, summed from per-workgroup
    partials inside the next solve, and the step errors come from
    ||C||^2 - ||carry||^2: both against the oracle.  The noise makes the step
    norms differ by ~1e-6 relative, so a norm taken from the wrong step fails."""
    dims = [10, 12, 14, 12, 10]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 9, 12, 6], 3e-3, 303)
    cores, rep, oc, orep = _run(a, dims, sweep, variant, eps=3e-2, q=1, p=2, seed=4)
    assert rep["ranks"] == orep["ranks"] == [1, 3, 9, 12, 6, 1]
    assert rep["ell"] == orep["ell"]   # the oracle widens in the same steps (ell 5 -> 10 in L2R step 2)
    np.testing.assert_allclose(rep["normC"], orep["normC"], rtol=1e-12)
    np.testing.assert_allclose(rep["delta"], orep["delta"], rtol=1e-6)
    _compare_conditioned(cores, oc, orep["s"], sweep)
    _compare_reconstruction(cores, oc, orep, sweep)


def test_eps_mode_fp32_input_c3_shape():
    """8^8 FP32 function tensor at eps = 1e-6 through the plain FP64 path:
    the oracle sees the same FP32-rounded tensor in FP64."""
    a32 = ttgen.inverse_sum_tensor(8, 8, dtype=np.float32)
    dims = [8] * 8
    A = _dev(a32)
    cores, rep = T.tt_utv_decompose(A, dims, eps=1e-6, sweep="R2L", variant="URV", q=1, oversample=8, seed=3)
    oc, orep = oracle.tt_utv(a32.astype(np.float64), dims, eps=1e-6, sweep="R2L", variant="URV", q=1, p=8, seed=3)
    assert rep["ranks"] == orep["ranks"]
    _compare_conditioned(cores, oc, orep["s"], "R2L")
    rec = _compare_reconstruction(cores, oc, orep, "R2L")
    a = a32.astype(np.float64)
    assert np.linalg.norm(rec - a) / np.linalg.norm(a) <= 1e-6


def test_c5_shape_order5_40_fp32_eps():
    """The 40^6 workload's recipe one order down (40^5 FP32, 410 MB: Gaussian
    TT ranks 32 plus 1e-5 noise, eps = 1e-4, TT-URV right-to-left, q = 1,
    p = 8, rank cap 48), small enough for the oracle: the FP64 form against
    the oracle through the cores and the reconstruction; the mixed form within
    its stated bound, which stays below eps."""
    dims = [40] * 5
    a, _ = ttgen.gaussian_tt_tensor(dims, [32] * 4, 1e-5, 5)
    a32 = a.astype(np.float32)
    a = a32.astype(np.float64)
    A = _dev(a32)
    kw = dict(eps=1e-4, sweep="R2L", variant="URV", q=1, oversample=8, seed=5, max_rank=48)
    print("40^5 FP32: FP64 form", flush=True)
    cores, rep = T.tt_utv_decompose(A, dims, exact_delta=True, **kw)
    torch.cuda.synchronize()
    print("40^5 FP32: oracle", flush=True)
    oc, orep = oracle.tt_utv(a, dims, eps=1e-4, sweep="R2L", variant="URV", q=1, p=8, seed=5, max_rank=48)
    assert rep["ranks"] == orep["ranks"] == [1, 32, 32, 32, 32, 1]
    assert rep["ell"] == orep["ell"]
    _compare_conditioned(cores, oc, orep["s"], "R2L")
    rec = _compare_reconstruction(cores, oc, orep, "R2L")
    err = np.linalg.norm(rec - a)
    assert err <= rep["err_bound"] * (1 + 1e-9) <= 1e-4 * np.linalg.norm(a)
    del rec
    print("40^5 FP32: mixed form", flush=True)
    cmx, rmx = T.tt_utv_decompose(A, dims, exact_delta=True, prec="mixed", **kw)
    assert rmx["rank_rule_met"] and rmx["ranks"] == rep["ranks"]
    recmx = T.tt_reconstruct(cmx).cpu().numpy()
    errmx = np.linalg.norm(recmx - a)
    print(f"40^5 mixed: error {errmx / np.linalg.norm(a):.4e}, bound {rmx['err_bound'] / rmx['norm_A']:.4e}",
          flush=True)
    assert errmx <= rmx["err_bound"] * (1 + 1e-9) <= 1e-4 * rmx["norm_A"] * (1 + 1e-12)


def test_eps_rank_cap_reports_erank():
    a = ttgen.inverse_sum_tensor(5, 8, dtype=np.float64)
    A = _dev(a)
    cores, rep = T.tt_utv_decompose(A, [8] * 5, eps=1e-12, sweep="R2L", variant="URV", max_rank=2,
                                    allow_rank_miss=True)
    assert rep["status"] == T.TT_ERANK
    assert not rep["rank_rule_met"]
    assert max(rep["ranks"]) <= 2


# --------------------------------------------------------------------- reproducibility, errors
def test_bitwise_reproducible():
    dims = [12, 11, 10, 9]
    a, _ = ttgen.gaussian_tt_tensor(dims, [4, 5, 4], 1e-4, 106)
    A = _dev(a)
    c1, r1 = T.tt_utv_decompose(A, dims, ranks=[4, 5, 4], sweep="R2L", variant="URV", q=1)
    c2, r2 = T.tt_utv_decompose(A, dims, ranks=[4, 5, 4], sweep="R2L", variant="URV", q=1)
    for x, y in zip(c1, c2):
        assert torch.equal(x, y)
    assert r1["delta"] == r2["delta"]


def test_nonfinite_input_is_reported():
    dims = [6, 7, 8]
    a = np.ones(6 * 7 * 8)
    a[17] = np.nan
    with pytest.raises(T.TTError) as ei:
        T.tt_utv_decompose(_dev(a), dims, ranks=[2, 2], sweep="L2R", variant="ULV")
    assert ei.value.code == T.TT_ENONFINITE


# --------------------------------------------------------------------- train contractions
def test_reconstruct_sample_backward_parity():
    dims = [5, 7, 6, 4, 9]
    ranks = [1, 3, 6, 5, 2, 1]
    cores_np = ttgen.gaussian_cores(dims, ranks, 107)
    cores = [_dev(c) for c in cores_np]
    full = T.tt_reconstruct(cores).cpu().numpy()
    np.testing.assert_allclose(full, oracle.tt_reconstruct(cores_np), rtol=1e-13, atol=1e-12)
    full32 = T.tt_reconstruct(cores, dtype=torch.float32).cpu().numpy()
    np.testing.assert_array_equal(full32, full.astype(np.float32))
    idx = ttgen.random_indices(dims, 5000, 108)
    vals = T.tt_sample(cores, _dev(idx)).cpu().numpy()
    np.testing.assert_allclose(vals, oracle.tt_sample(cores_np, idx), rtol=1e-12, atol=1e-12)
    w = np.random.default_rng(109).standard_normal(5000)
    grads = T.tt_sample_backward(cores, _dev(idx), _dev(w))
    og = oracle.tt_sample_grad(cores_np, idx, w)
    for g, o in zip(grads, og):
        np.testing.assert_allclose(g.cpu().numpy(), o, rtol=1e-10, atol=1e-10 * np.max(np.abs(o)))


def test_autograd_function_matches_oracle_gradient():
    dims = [4, 5, 3, 6]
    ranks = [1, 2, 4, 3, 1]
    cores_np = ttgen.gaussian_cores(dims, ranks, 110)
    cores = [_dev(c).requires_grad_(True) for c in cores_np]
    idx = _dev(ttgen.random_indices(dims, 700, 111))
    w = np.random.default_rng(112).standard_normal(700)
    out = T.TTSample.apply(idx, *cores)
    (out * _dev(w)).sum().backward()
    og = oracle.tt_sample_grad(cores_np, idx.cpu().numpy(), w)
    for c, o in zip(cores, og):
        np.testing.assert_allclose(c.grad.cpu().numpy(), o, rtol=1e-10, atol=1e-12)


def test_sample_empty_and_large_index_range():
    dims = [3, 4]
    cores = [_dev(c) for c in ttgen.gaussian_cores(dims, [1, 2, 1], 113)]
    out = T.tt_sample(cores, torch.zeros((0, 2), dtype=torch.int64, device="cuda"))
    assert out.numel() == 0


# --------------------------------------------------------------------- mixed precision
@pytest.mark.parametrize("sweep,variant", ALL)
@pytest.mark.parametrize("prec", ["mixed", "mixed_bf16"])
def test_mixed_fixed_rank_bound_and_agreement(sweep, variant, prec):
    """FP32 carries with FP64 accumulation: the stated bound sqrt(sum delta^2) +
    sum rho holds, rho > 0 is measured, and the result stays within FP32
    storage accuracy of the FP64 form (oracle-pinned above)."""
    dims = [12, 11, 10, 9, 8]
    a, _ = ttgen.gaussian_tt_tensor(dims, [4, 6, 6, 4], 1e-3, 120)
    A = _dev(a.astype(np.float32))
    a32 = a.astype(np.float32).astype(np.float64)
    c64, r64 = T.tt_utv_decompose(A, dims, ranks=[4, 5, 5, 4], sweep=sweep, variant=variant, q=2, exact_delta=True)
    cmx, rmx = T.tt_utv_decompose(A, dims, ranks=[4, 5, 5, 4], sweep=sweep, variant=variant, q=2, exact_delta=True,
                                  prec=prec)
    assert rmx["ranks"] == r64["ranks"]
    # every carry but the last (which is written into an FP64 core) is rounded to FP32
    last = len(dims) - 2 if sweep == "L2R" else 0
    assert all((x > 0) == (k != last) for k, x in enumerate(rmx["rho"]))
    assert all(x == 0 for x in r64["rho"])
    rec64 = T.tt_reconstruct(c64).cpu().numpy()
    recmx = T.tt_reconstruct(cmx).cpu().numpy()
    err = np.linalg.norm(recmx - a32)
    assert err <= rmx["err_bound"] * (1 + 1e-9)
    if prec == "mixed":
        assert np.linalg.norm(recmx - rec64) <= 1e-5 * np.linalg.norm(a32)
    else:
        # BF16 power products: a coarser sketch, still within a few percent of the FP64 error
        assert err <= 1.05 * np.linalg.norm(rec64 - a32)


@pytest.mark.parametrize("sweep,variant", [("R2L", "URV"), ("L2R", "ULV")])
def test_mixed_tall_iterate(sweep, variant):
    """The mixed form where the sketched step takes the wide streaming kernels
    (m = 8192 rows, n = 540 core-side columns, ell = 40: FP32 matrix-core A*X
    and A^T Y, the FP64-accumulating Rayleigh-Ritz pass, the tree QR): same
    ranks as the FP64 form, the stated bound holds, and the result stays
    within FP32 storage accuracy of the FP64 form."""
    dims, ranks = [8192, 30, 20], [24, 18]
    if sweep == "L2R":
        dims, ranks = dims[::-1], ranks[::-1]
    a, _ = ttgen.gaussian_tt_tensor(dims, ranks, 1e-4, 121)
    A = _dev(a.astype(np.float32))
    a32 = a.astype(np.float32).astype(np.float64)
    c64, r64 = T.tt_utv_decompose(A, dims, ranks=ranks, sweep=sweep, variant=variant, q=1, oversample=16,
                                  exact_delta=True)
    cmx, rmx = T.tt_utv_decompose(A, dims, ranks=ranks, sweep=sweep, variant=variant, q=1, oversample=16,
                                  exact_delta=True, prec="mixed")
    assert rmx["ranks"] == r64["ranks"]
    rec64 = T.tt_reconstruct(c64).cpu().numpy()
    recmx = T.tt_reconstruct(cmx).cpu().numpy()
    assert np.linalg.norm(recmx - a32) <= rmx["err_bound"] * (1 + 1e-9)
    assert np.linalg.norm(recmx - rec64) <= 1e-5 * np.linalg.norm(a32)


def test_mixed_eps_1e6_function_tensor():
    """C3 shape: 8^8 FP32, eps = 1e-6 with FP32 carries meets RSE <= eps and
    stays within one rank of the FP64 form on every bond."""
    a32 = ttgen.inverse_sum_tensor(8, 8, dtype=np.float32)
    dims = [8] * 8
    A = _dev(a32)
    a = a32.astype(np.float64)
    # exact_delta: the bound uses measured step errors (sqrt(||C||^2 - ||carry||^2)
    # cancels at delta ~ 1e-6 ||C|| and is only an estimate there)
    c64, r64 = T.tt_utv_decompose(A, dims, eps=1e-6, sweep="R2L", variant="URV", q=1, oversample=8, seed=3,
                                  exact_delta=True)
    cmx, rmx = T.tt_utv_decompose(A, dims, eps=1e-6, sweep="R2L", variant="URV", q=1, oversample=8, seed=3,
                                  prec="mixed", exact_delta=True)
    for cores, rep in ((c64, r64), (cmx, rmx)):
        rec = T.tt_reconstruct(cores).cpu().numpy()
        rse = np.linalg.norm(rec - a) / np.linalg.norm(a)
        assert rse <= 1e-6
        assert np.linalg.norm(rec - a) <= rep["err_bound"] * (1 + 1e-6) + 1e-12
    assert max(abs(x - y) for x, y in zip(rmx["ranks"], r64["ranks"])) <= 1
    # measured step errors: the stated bound of the mixed form is within eps
    assert rmx["err_bound"] <= 1e-6 * rmx["norm_A"]
    # estimated step errors (the default): the same call meets its rank rule
    # (the estimates' rounding noise must not turn into TT_ERANK)
    cdf, rdf = T.tt_utv_decompose(A, dims, eps=1e-6, sweep="R2L", variant="URV", q=1, oversample=8, seed=3,
                                  prec="mixed")
    assert rdf["status"] == T.TT_OK and rdf["rank_rule_met"]
    assert rdf["ranks"] == rmx["ranks"]
