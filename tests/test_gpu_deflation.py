"""The deflation inner kernel (one core-side vector at a time, the USV-plus
reading of the paper's fastest TT-ULV variant, Sec. 3.3 / Sec. 4) through the
C ABI against the FP64 oracle: fixed ranks at 1e-10 on cores, reconstruction
and step errors, in Gram mode (core side n <= 64: A^T A in one pass, the search
in one workgroup) and in the streaming mode (one pass over A per power step)
for every form of its pass kernel (one wave per workgroup up to n = 128
column-major and 512 row-major, then four waves with 1, 2, 4, 8 or 16
register columns up to n = 4096), each at its width limits, both storage
orders, FP32 input, q = 1..3; prescribed accuracy with the oracle's ranks; the
32^5 workload in full."""
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


def _compare(gpu_cores, ora_cores, sweep, tol=TOL):
    g = _align(_np(gpu_cores), ora_cores, sweep)
    assert [x.shape for x in g] == [x.shape for x in ora_cores]
    for k, (x, y) in enumerate(zip(g, ora_cores)):
        err = np.max(np.abs(x - y)) / max(np.max(np.abs(y)), 1e-300)
        assert err <= tol, f"core {k + 1}: rel err {err:.3e}"


def _expected_passes(dims, r, sweep, q):
    """Streaming passes of a fixed-rank sweep: q per vector and one for the last
    vector's energy, on every step whose core side exceeds 64."""
    d = len(dims)
    total = 0
    steps = range(1, d) if sweep == "L2R" else range(d, 1, -1)
    for k in steps:
        n, rk = (r[k - 1] * dims[k - 1], r[k]) if sweep == "L2R" else (dims[k - 1] * r[k], r[k - 1])
        if n > 64:
            total += q * rk + 1
    return total


def _run(a, dims, sweep, variant, dtype=np.float64, q=1, seed=3, **kw):
    A = _dev(a.astype(dtype))
    cores, rep = T.tt_utv_decompose(A, dims, sweep=sweep, variant=variant, q=q, seed=seed, inner="deflation",
                                    profile=True, **kw)
    return [c.clone() for c in cores], rep


# (dims, generating ranks, fixed ranks, sweep): the core sides n of the steps are listed
CASES = [
    ([6, 10, 7, 40], [3, 9, 12], [3, 9, 12], "R2L"),     # n = 40 (Gram), 84, 90: streaming, one register column
    ([40, 12, 9, 10], [12, 20, 8], [12, 20, 8], "L2R"),  # n = 40 (Gram), 144, 180 (row-major streaming)
    ([50, 24, 40], [20, 30], [20, 30], "R2L"),           # n = 40, 720 (four register columns), m = 50 ragged
    ([40, 24, 50], [20, 30], [20, 30], "L2R"),           # n = 40, 480 (two), row-major
    ([7, 30, 60], [6, 30], [6, 30], "R2L"),              # n = 60, 900 with m = 7
    ([12, 120, 30], [10, 30], [10, 30], "R2L"),          # n = 3600: sixteen register columns
    ([30, 120, 12], [25, 10], [25, 10], "L2R"),          # n = 3000 row-major
    ([11, 13, 9, 5], [4, 7, 3], [4, 7, 3], "L2R"),       # every step in Gram mode
    # the pass kernel's forms at their width limits: column-major one-wave up to n = 128, then four-wave
    # with 1 (n <= 256), 2, 4, 8 (n <= 2048) register columns; row-major one-wave up to 512, then four-wave
    ([40, 8, 16], [12, 16], [12, 16], "R2L"),            # n = 128: the widest column-major one-wave pass
    ([40, 43, 9], [10, 3], [10, 3], "R2L"),              # n = 129: column-major four-wave, one register column
    ([40, 16, 20], [12, 16], [12, 16], "R2L"),           # n = 256: the same at its width limit
    ([30, 55, 20], [12, 20], [12, 20], "R2L"),           # n = 1100: eight register columns
    ([40, 32, 30], [16, 12], [16, 12], "L2R"),           # n = 512: the widest row-major one-wave pass
    ([30, 27, 25], [19, 10], [19, 10], "L2R"),           # n = 513: row-major four-wave, four register columns
    ([50, 55, 24], [20, 12], [20, 12], "L2R"),           # n = 1100 row-major: eight register columns
]


# every case in each sweep/variant pair with an orthonormal core side (Alg. 4, ULV right to left, has no
# deflation form)
FIXED = [(dims, gen, ranks, sweep, variant) for dims, gen, ranks, sweep in CASES
         for variant in (("ULV", "URV") if sweep == "L2R" else ("URV",))]


@pytest.mark.parametrize("dims,gen,ranks,sweep,variant", FIXED)
def test_fixed_ranks_match_oracle(dims, gen, ranks, sweep, variant):
    a, _ = ttgen.gaussian_tt_tensor(dims, gen, 1e-3, 17)
    print(f"deflation: dims {dims} ranks {ranks} {sweep}/{variant}", flush=True)
    cores, rep = _run(a, dims, sweep, variant, ranks=ranks)
    oc, orep = oracle.tt_utv(a, dims, ranks=ranks, sweep=sweep, variant=variant, q=1, seed=3, inner="deflation")
    assert rep["ranks"] == orep["ranks"]
    _compare(cores, oc, sweep)
    rec = T.tt_reconstruct(cores).cpu().numpy()
    np.testing.assert_allclose(rec, oracle.tt_reconstruct(oc), rtol=0, atol=TOL * np.max(np.abs(a)))
    # step errors sqrt(||C||^2 - ||carry||^2) hold delta^2 to about u ||C||^2
    for x, y in zip(rep["delta"], orep["delta"]):
        assert abs(x * x - y * y) <= 1e-13 * orep["norm_A"] ** 2
    assert rep["ell"] == [int(x) for x in orep["ell"]]
    assert rep["kstat"]["defl_pass"]["launches"] == _expected_passes(dims, rep["ranks"], sweep, 1)


@pytest.mark.parametrize("q", [2, 3])
def test_more_power_steps_and_fp32_input(q):
    dims = [6, 10, 7, 40]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 9, 12], 1e-3, 19)
    a = a.astype(np.float32)
    print(f"deflation: q = {q}, FP32 input", flush=True)
    for sweep in ("R2L", "L2R"):
        cores, rep = _run(a, dims, sweep, "URV", dtype=np.float32, q=q, ranks=[3, 9, 12])
        oc, orep = oracle.tt_utv(a.astype(np.float64), dims, ranks=[3, 9, 12], sweep=sweep, variant="URV", q=q,
                                 seed=3, inner="deflation")
        _compare(cores, oc, sweep)
        assert rep["kstat"]["defl_pass"]["launches"] == _expected_passes(dims, rep["ranks"], sweep, q)


@pytest.mark.parametrize("sweep,variant", [("R2L", "URV"), ("L2R", "ULV")])
def test_prescribed_accuracy_matches_oracle(sweep, variant):
    """eps mode: the search stops at the first vector meeting the rank rule;
    ranks equal the oracle's, the reconstruction matches it and meets eps."""
    dims = [10, 12, 9, 40]
    a, _ = ttgen.gaussian_tt_tensor(dims, [4, 20, 10], 1e-6, 8)
    print(f"deflation: eps mode {sweep}", flush=True)
    for eps in (1e-2, 1e-4):
        cores, rep = _run(a, dims, sweep, variant, q=2, eps=eps)
        oc, orep = oracle.tt_utv(a, dims, eps=eps, sweep=sweep, variant=variant, q=2, seed=3, inner="deflation")
        assert rep["ranks"] == orep["ranks"], (rep["ranks"], orep["ranks"])
        assert rep["rank_rule_met"] and orep["rank_rule_met"]
        rec = T.tt_reconstruct(cores).cpu().numpy()
        np.testing.assert_allclose(rec, oracle.tt_reconstruct(oc), rtol=0, atol=TOL * np.max(np.abs(a)))
        assert np.linalg.norm(rec - a) <= eps * np.linalg.norm(a) * (1 + 1e-9)


def test_prescribed_accuracy_rank_cap():
    """eps beyond reach under max_rank: the search ends at the cap, the rule is
    reported as missed (TT_ERANK, allowed here) and the ranks are the cap."""
    dims = [10, 12, 9, 40]
    # generating ranks above the cap: the five vectors kept at each bond lie in the
    # signal part of the spectrum (a vector in the noise tail, at sigma_j / sigma_1
    # near 1e-2, is fixed only to about u (sigma_1 / sigma_j)^2 by its power steps)
    a, _ = ttgen.gaussian_tt_tensor(dims, [6, 8, 6], 1e-2, 8)
    print("deflation: eps under a rank cap", flush=True)
    cores, rep = _run(a, dims, "R2L", "URV", q=1, eps=1e-6, max_rank=5, allow_rank_miss=True)
    oc, orep = oracle.tt_utv(a, dims, eps=1e-6, sweep="R2L", variant="URV", q=1, seed=3, max_rank=5,
                             inner="deflation")
    assert rep["ranks"] == orep["ranks"] and rep["ranks"][1:-1] == [5, 5, 5]
    assert not rep["rank_rule_met"] and not orep["rank_rule_met"]
    _compare(cores, oc, "R2L")


def test_full_size_order5_32():
    """The 32^5 FP64 workload (rank 16, right to left, q = 1): the 1,048,576 x 32
    first unfolding in Gram mode, the 32,768 x 512 ones streaming; cores and
    step errors against the oracle."""
    dims = [32] * 5
    a, _ = ttgen.gaussian_tt_tensor(dims, [16, 16, 16, 16], 1e-8, 5)
    print("deflation: 32^5 rank 16", flush=True)
    cores, rep = _run(a, dims, "R2L", "URV", q=1, ranks=[16] * 4)
    oc, orep = oracle.tt_utv(a, dims, ranks=[16] * 4, sweep="R2L", variant="URV", q=1, seed=3, inner="deflation")
    _compare(cores, oc, "R2L")
    for x, y in zip(rep["delta"], orep["delta"]):
        assert abs(x * x - y * y) <= 1e-13 * orep["norm_A"] ** 2


@pytest.mark.parametrize("sweep,variant", [("R2L", "URV"), ("L2R", "ULV")])
def test_fixed_rank_above_the_true_rank(sweep, variant):
    """Exact TT-ranks (3, 4, 3) asked for at ranks (5, 6, 5): after the true-rank
    vectors every power product is rounding noise, so the extra vectors are
    arbitrary unit directions orthogonal to the others (they differ from the
    oracle's); the reconstruction is exact on both sides and the cores stay
    orthonormal."""
    dims = [6, 7, 8, 9]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 4, 3], 0.0, 23)
    print(f"deflation: ranks above the true rank, {sweep}", flush=True)
    cores, rep = _run(a, dims, sweep, variant, ranks=[5, 6, 5])
    oc, orep = oracle.tt_utv(a, dims, ranks=[5, 6, 5], sweep=sweep, variant=variant, q=1, seed=3, inner="deflation")
    assert rep["ranks"] == orep["ranks"] == [1, 5, 6, 5, 1]
    rec = T.tt_reconstruct(cores).cpu().numpy()
    nrm = np.linalg.norm(a)
    assert np.linalg.norm(rec - a) <= 1e-12 * nrm
    assert np.linalg.norm(oracle.tt_reconstruct(oc) - a) <= 1e-12 * nrm
    g = _np(cores)
    for c in (g[:-1] if sweep == "L2R" else g[1:]):
        M = c.reshape(-1, c.shape[2], order="F") if sweep == "L2R" else c.reshape(c.shape[0], -1, order="F").T
        assert np.max(np.abs(M.T @ M - np.eye(M.shape[1]))) < 1e-13


def test_zero_tolerance_runs_to_the_cap():
    """eps = 0: the rule is met only by an exact fit, so on a noisy tensor every
    step keeps max_rank vectors; the search stops there and reports the miss."""
    dims = [8, 9, 10]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 4], 1e-2, 29)
    print("deflation: eps = 0", flush=True)
    cores, rep = _run(a, dims, "R2L", "URV", q=1, eps=0.0, max_rank=6, allow_rank_miss=True)
    oc, orep = oracle.tt_utv(a, dims, eps=0.0, sweep="R2L", variant="URV", q=1, seed=3, max_rank=6,
                             inner="deflation")
    assert rep["ranks"] == orep["ranks"] == [1, 6, 6, 1]
    assert not rep["rank_rule_met"]
    _compare(cores, oc, "R2L")


@pytest.mark.parametrize("dims,ranks,sweep", [
    ([1, 7, 1, 9], [1, 1, 1], "L2R"),      # unit extents: one-vector steps on a 1-wide core side
    ([13, 70], [9], "R2L"),                # d = 2, one column-major streaming step (n = 70)
    ([70, 13], [9], "L2R"),                # d = 2, one row-major streaming step (n = 70)
    ([13, 40], [9], "L2R"),                # d = 2, one Gram-mode step (n = 13)
])
def test_small_and_degenerate_shapes(dims, ranks, sweep):
    a, _ = ttgen.gaussian_tt_tensor(dims, ranks, 1e-3, 31)
    variant = "ULV" if sweep == "L2R" else "URV"
    print(f"deflation: dims {dims} ranks {ranks} {sweep}", flush=True)
    cores, rep = _run(a, dims, sweep, variant, q=2, ranks=ranks)
    oc, orep = oracle.tt_utv(a, dims, ranks=ranks, sweep=sweep, variant=variant, q=2, seed=3, inner="deflation")
    assert rep["ranks"] == orep["ranks"]
    _compare(cores, oc, sweep)
    rec = T.tt_reconstruct(cores).cpu().numpy()
    np.testing.assert_allclose(rec, oracle.tt_reconstruct(oc), rtol=0, atol=TOL * np.max(np.abs(a)))
