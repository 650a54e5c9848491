"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these retypes the oracle's formulas: each checks a property that a
dropped term, a wrong sign or index, or a transposed operand would break.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import ttutv_oracle as O
import ttgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
COMBOS = [("L2R", "ULV"), ("R2L", "URV"), ("L2R", "URV"), ("R2L", "ULV")]


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _rse(a, cores):
    return np.linalg.norm(oracle.tt_reconstruct(cores) - a) / np.linalg.norm(a)


# ---------------------------------------------------------------- generator
def test_splitmix64_published_outputs():
    want = [int(r[0]) for r in _read_golden("splitmix64_seed1234567.txt")]
    got = [int(x) for x in oracle.splitmix64(1234567, np.arange(1, 6, dtype=np.uint64))]
    assert got == want


def test_sketch_gaussian_distribution_and_ordering():
    g = oracle.sketch_gaussian(42, 3, 50, 40, 100, True)
    x = g.ravel()
    assert abs(x.mean()) < 5 / math.sqrt(x.size)
    assert abs(x.var() - 1) < 5 * math.sqrt(2 / x.size)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    # columns are uncorrelated
    c = np.corrcoef(g[:, :20].T)
    assert np.max(np.abs(c - np.eye(20))) < 6 / math.sqrt(g.shape[0])
    # the (i, beta) -> row map only permutes rows
    h = oracle.sketch_gaussian(42, 3, 50, 40, 100, False)
    i, b = 7, 11
    assert np.array_equal(g[i + 50 * b], h[b + 40 * i])
    # different modes and seeds give different matrices
    assert not np.allclose(g, oracle.sketch_gaussian(42, 4, 50, 40, 100, True))
    assert not np.allclose(g, oracle.sketch_gaussian(43, 3, 50, 40, 100, True))
    # extending ell keeps the leading columns
    assert np.array_equal(g[:, :30], oracle.sketch_gaussian(42, 3, 50, 40, 30, True))


# ---------------------------------------------------------------- Eq. (TT)
def test_reconstruct_closed_form_sum():
    """The rank-2 train [x1 1] [[1 0],[xk 1]] ... [1; xd] represents
    f(i) = sum_k x_k[i_k] (a textbook TT construction)."""
    rng = np.random.default_rng(0)
    dims = [3, 4, 5, 2]
    xs = [rng.standard_normal(I) for I in dims]
    d = len(dims)
    cores = []
    for k, x in enumerate(xs):
        if k == 0:
            g = np.zeros((1, dims[k], 2)); g[0, :, 0] = x; g[0, :, 1] = 1
        elif k == d - 1:
            g = np.zeros((2, dims[k], 1)); g[0, :, 0] = 1; g[1, :, 0] = x
        else:
            g = np.zeros((2, dims[k], 2)); g[0, :, 0] = 1; g[1, :, 0] = x; g[1, :, 1] = 1
        cores.append(g)
    want = np.zeros(dims)
    for k, x in enumerate(xs):
        shape = [1] * d; shape[k] = dims[k]
        want = want + x.reshape(shape)
    got = oracle.tt_reconstruct(cores)
    np.testing.assert_allclose(got, want.reshape(-1, order="F"), rtol=0, atol=1e-14)
    # entry i1 + I1*i2 + ... is (i1, i2, ...): check one off-diagonal entry
    i = (2, 1, 4, 1)
    flat = i[0] + dims[0] * (i[1] + dims[1] * (i[2] + dims[2] * i[3]))
    assert got[flat] == pytest.approx(sum(xs[k][i[k]] for k in range(d)), abs=1e-14)


def test_sample_equals_reconstruct_entries():
    dims = [4, 5, 3, 6]
    cores = ttgen.gaussian_cores(dims, [1, 3, 2, 4, 1], 1)
    full = oracle.tt_reconstruct(cores)
    idx = ttgen.random_indices(dims, 200, 2)
    flat = idx[:, 0] + dims[0] * (idx[:, 1] + dims[1] * (idx[:, 2] + dims[2] * idx[:, 3]))
    np.testing.assert_allclose(oracle.tt_sample(cores, idx), full[flat], rtol=1e-13, atol=1e-13)


def test_sample_grad_finite_differences():
    dims = [3, 4, 2, 3]
    cores = ttgen.gaussian_cores(dims, [1, 2, 3, 2, 1], 5)
    idx = ttgen.random_indices(dims, 40, 6)
    w = np.random.default_rng(7).standard_normal(40)
    grads = oracle.tt_sample_grad(cores, idx, w)
    h = 1e-6
    for k, g in enumerate(cores):
        fd = np.zeros_like(g)
        for pos in np.ndindex(g.shape):
            cp = [c.copy() for c in cores]; cp[k][pos] += h
            cm = [c.copy() for c in cores]; cm[k][pos] -= h
            fd[pos] = (w @ oracle.tt_sample(cp, idx) - w @ oracle.tt_sample(cm, idx)) / (2 * h)
        np.testing.assert_allclose(grads[k], fd, rtol=1e-6, atol=1e-7)


def test_reconstruct_grad_finite_differences():
    """<gout, A_TT> is linear in each core, so central differences of it are
    exact up to rounding: every entry of every core gradient is checked."""
    dims, ranks = [3, 4, 2, 5], [1, 2, 3, 2, 1]
    cores = ttgen.gaussian_cores(dims, ranks, 7)
    rng = np.random.default_rng(8)
    gout = rng.standard_normal(int(np.prod(dims)))
    grads = oracle.tt_reconstruct_grad(cores, gout)
    h = 1e-6
    for k in range(len(cores)):
        assert grads[k].shape == cores[k].shape
        fd = np.zeros_like(cores[k])
        for pos in np.ndindex(*cores[k].shape):
            cp = [c.copy() for c in cores]; cp[k][pos] += h
            cm = [c.copy() for c in cores]; cm[k][pos] -= h
            fd[pos] = (gout @ oracle.tt_reconstruct(cp) - gout @ oracle.tt_reconstruct(cm)) / (2 * h)
        np.testing.assert_allclose(grads[k], fd, rtol=1e-7, atol=1e-8)


def test_reconstruct_grad_euler_identity_and_sparse_gout():
    """A_TT is homogeneous of degree one in each core, so sum_k <dL/dG_k, G_k>
    = d <gout, A_TT> (Euler); with gout a weighted sum of unit tensors the dense
    gradient is the sampled-entry gradient (itself pinned by differences)."""
    dims, ranks = [4, 3, 5, 2, 3], [1, 3, 2, 4, 2, 1]
    cores = ttgen.gaussian_cores(dims, ranks, 17)
    rng = np.random.default_rng(18)
    gout = rng.standard_normal(int(np.prod(dims)))
    grads = oracle.tt_reconstruct_grad(cores, gout)
    lhs = sum(float(np.sum(g * c)) for g, c in zip(grads, cores))
    assert lhs == pytest.approx(len(dims) * float(gout @ oracle.tt_reconstruct(cores)), rel=1e-12)
    # sparse gout: 25 entries (some repeated) with weights
    idx = np.stack([rng.integers(0, I, 25) for I in dims], axis=1)
    w = rng.standard_normal(25)
    dense = np.zeros(int(np.prod(dims)))
    flat = np.ravel_multi_index(idx.T, dims, order="F")
    np.add.at(dense, flat, w)
    for g1, g2 in zip(oracle.tt_reconstruct_grad(cores, dense), oracle.tt_sample_grad(cores, idx, w)):
        np.testing.assert_allclose(g1, g2, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- sweeps
@pytest.mark.parametrize("sweep,variant", COMBOS + [("L2R", "SVD"), ("R2L", "SVD")])
def test_exact_tt_rank_reconstructs(sweep, variant):
    """Thm. 3.1/3.2 with eps_k = 0: a tensor of exact TT-ranks is recovered."""
    dims = [5, 6, 7, 5]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 4, 3], 0.0, 11)
    cores, rep = oracle.tt_utv(a, dims, ranks=[3, 4, 3], sweep=sweep, variant=variant, q=1, p=4, seed=3)
    assert _rse(a, cores) < 1e-12
    assert rep["ranks"] == [1, 3, 4, 3, 1]


@pytest.mark.parametrize("sweep,variant", [("L2R", "ULV"), ("R2L", "URV"), ("L2R", "URV")])
def test_pythagoras_equality(sweep, variant):
    """With carries equal to the exact projections (U1^T E = 0, resp. E V1 = 0)
    the proof of Thm. 3.1 holds with equality: ||A - A_TT||^2 = sum delta_k^2."""
    dims = [6, 7, 5, 6, 4]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 5, 5, 3], 1e-2, 21)
    cores, rep = oracle.tt_utv(a, dims, ranks=[3, 4, 4, 3], sweep=sweep, variant=variant, q=1, p=3, seed=9)
    err2 = np.sum((oracle.tt_reconstruct(cores) - a) ** 2)
    bound2 = np.sum(np.square(rep["delta"]))
    assert err2 > 0
    assert abs(err2 - bound2) <= 1e-9 * bound2


def test_alg4_sum_bound():
    """Prop. A.1: the ULV right-to-left sweep obeys ||A - A_TT|| <= sum delta_k."""
    dims = [6, 7, 5, 6, 4]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 5, 5, 3], 5e-2, 22)
    for q in (0, 1):
        cores, rep = oracle.tt_utv(a, dims, ranks=[3, 4, 4, 3], sweep="R2L", variant="ULV", q=q, p=2, seed=4)
        err = np.linalg.norm(oracle.tt_reconstruct(cores) - a)
        assert err <= np.sum(rep["delta"]) * (1 + 1e-12)
        assert rep["err_bound"] == pytest.approx(np.sum(rep["delta"]))


def test_alg4_step_is_a_ulv_with_range_side_orthogonality():
    """Alg. 4 (appendix): each step is a truncated ULV with the orthogonality on
    the range side, C = U1 S_r V1^T + E with U1^T E = 0, and its carry U1 S_r
    drops the part (I - U1 U1^T) C V1 = E V1 that TT-URV keeps (its carry is
    C V1, so E V1 = 0 there).  Checked on two successive unfoldings of a
    right-to-left sweep with ell < n, against the TT-URV step on the same
    matrices: a sign error or a swapped side in either step fails one of the
    conditions."""
    dims = [6, 7, 5, 6]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 5, 3], 5e-2, 23)
    C = a
    r_next = 1
    for k, r in ((4, 3), (3, 4)):
        n = dims[k - 1] * r_next
        Cm = C.reshape(-1, n, order="F")
        out = {}
        for kind in ("ulv_tall", "urv_tall"):
            U1, s_r, V1, _, ell, dk, _ = O._step(Cm, kind, r, None, 1, 1, 7, k, dims[k - 1], r_next, True,
                                                 k == 4, None, None, {"rank_rule_met": True})
            assert ell < n
            E = Cm - (U1 * s_r) @ V1.T
            out[kind] = (U1, s_r, V1, E)
            assert np.max(np.abs(U1.T @ U1 - np.eye(r))) < 1e-13
            assert np.max(np.abs(V1.T @ V1 - np.eye(r))) < 1e-13
            assert dk == pytest.approx(np.linalg.norm(E), rel=1e-12)
        U1, s_r, V1, E = out["ulv_tall"]
        nC = np.linalg.norm(Cm)
        assert np.linalg.norm(U1.T @ E) <= 1e-13 * nC                 # range side exact
        ev = np.linalg.norm(E @ V1)
        assert ev >= 1e-8 * nC                                         # the dropped U2 L21 term, far above rounding
        assert ev == pytest.approx(np.linalg.norm(Cm @ V1 - U1 @ (U1.T @ Cm @ V1)), rel=1e-10)
        U1u, s_ru, V1u, Eu = out["urv_tall"]
        assert np.linalg.norm(Eu @ V1u) <= 1e-13 * nC                  # TT-URV: core side exact
        # and the two carries differ by exactly the dropped term: C V1 - U1 S_r = E V1
        assert np.linalg.norm(Cm @ V1 - U1 * s_r) == pytest.approx(ev, rel=1e-10)
        C = (U1 * s_r).reshape(-1, order="F")                           # Alg. 4 carry U1 S_r
        r_next = r


@pytest.mark.parametrize("sweep,variant", COMBOS)
def test_core_orthogonality(sweep, variant):
    """Def. 2.2: L2R cores 1..d-1 are left-orthogonal, R2L cores 2..d right-orthogonal."""
    dims = [4, 6, 5, 7]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 4, 3], 1e-3, 31)
    cores, _ = oracle.tt_utv(a, dims, ranks=[3, 3, 2], sweep=sweep, variant=variant, q=1, p=3, seed=1)
    if sweep == "L2R":
        for g in cores[:-1]:
            G2 = g.reshape(g.shape[0] * g.shape[1], g.shape[2], order="F")
            assert np.max(np.abs(G2.T @ G2 - np.eye(g.shape[2]))) < 1e-13
    else:
        for g in cores[1:]:
            G1 = g.reshape(g.shape[0], g.shape[1] * g.shape[2], order="F")
            assert np.max(np.abs(G1 @ G1.T - np.eye(g.shape[0]))) < 1e-13


def test_matrix_case_is_eckart_young():
    """d = 2 with ell >= n: the sweep is one truncated SVD, whose error is
    sqrt(sum_{i>r} sigma_i^2) (LAPACK singular values as the library reference)."""
    rng = np.random.default_rng(3)
    U, _ = np.linalg.qr(rng.standard_normal((40, 30)))
    V, _ = np.linalg.qr(rng.standard_normal((25, 25)))
    s = 2.0 ** -np.arange(25)
    M = (U[:, :25] * s) @ V.T                   # 40 x 25, known spectrum
    a = M.reshape(-1, order="F")
    sig = np.linalg.svd(M, compute_uv=False)
    for sweep, variant in COMBOS + [("L2R", "SVD")]:
        for r in (1, 4, 9):
            cores, rep = oracle.tt_utv(a, [40, 25], ranks=[r], sweep=sweep, variant=variant, q=0, p=100, seed=0)
            err = np.linalg.norm(oracle.tt_reconstruct(cores) - a)
            assert err == pytest.approx(math.sqrt(np.sum(sig[r:] ** 2)), rel=1e-10)
    # with ell < n, q power steps still find the optimum on a strongly graded spectrum
    cores, _ = oracle.tt_utv(a, [40, 25], ranks=[4], sweep="R2L", variant="URV", q=2, p=4, seed=0)
    err = np.linalg.norm(oracle.tt_reconstruct(cores) - a)
    assert err == pytest.approx(math.sqrt(np.sum(sig[4:] ** 2)), rel=1e-6)


@pytest.mark.parametrize("sweep,variant", [("L2R", "ULV"), ("R2L", "URV"), ("R2L", "ULV")])
def test_full_sketch_equals_tt_svd(sweep, variant):
    """ell = n at every step (G = I) makes the UTV step an exact factorisation,
    so the cores equal TT-SVD's (distinct singular values, canonical signs)."""
    dims = [5, 6, 4, 5]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 4, 3], 1e-2, 41)
    c1, r1 = oracle.tt_utv(a, dims, ranks=[3, 4, 3], sweep=sweep, variant=variant, q=0, p=1000, seed=0)
    c2, r2 = oracle.tt_svd(a, dims, ranks=[3, 4, 3], sweep=sweep)
    for g1, g2 in zip(c1, c2):
        np.testing.assert_allclose(g1, g2, rtol=0, atol=1e-10 * np.max(np.abs(g2)))
    np.testing.assert_allclose(r1["delta"], r2["delta"], rtol=1e-8)


def test_reversed_urv_equals_ulv_left_to_right():
    """The index-reversal form of TT-URV (remark after Thm. 3.2) sees the same
    core-side test matrix as TT-ULV, so both give the same left-orthogonal cores."""
    dims = [6, 5, 7, 4]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 4, 3], 1e-4, 51)
    c1, _ = oracle.tt_utv(a, dims, ranks=[3, 4, 3], sweep="L2R", variant="ULV", q=1, p=3, seed=8)
    c2, _ = oracle.tt_utv(a, dims, ranks=[3, 4, 3], sweep="L2R", variant="URV", q=1, p=3, seed=8)
    for g1, g2 in zip(c1, c2):
        np.testing.assert_allclose(g1, g2, rtol=0, atol=1e-9 * np.max(np.abs(g2)))


@pytest.mark.parametrize("sweep,variant", COMBOS + [("L2R", "SVD")])
def test_prescribed_accuracy_meets_eps(sweep, variant):
    """Alg. 2 guarantee: RSE <= eps, with ranks found adaptively."""
    a = ttgen.inverse_sum_tensor(6, 8, dtype=np.float64)
    dims = [8] * 6
    for eps in (1e-2, 1e-4, 1e-6):
        cores, rep = oracle.tt_utv(a, dims, eps=eps, sweep=sweep, variant=variant, q=1, p=4, seed=2)
        assert rep["rank_rule_met"]
        assert _rse(a, cores) <= eps * (1 + 1e-9)


def test_prescribed_accuracy_recovers_generating_ranks():
    dims = [6, 7, 6, 5, 6]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 5, 4, 3], 1e-8, 61)
    for sweep, variant in COMBOS:
        cores, rep = oracle.tt_utv(a, dims, eps=1e-5, sweep=sweep, variant=variant, q=1, p=4, seed=5)
        assert rep["ranks"] == [1, 3, 5, 4, 3, 1], (sweep, variant)


def test_rank_rule_reads_frobenius_energy():
    """The rank rule is ||C||^2 - sum_{i<=r} s_i^2 <= eps_k^2, smallest r >= 1."""
    s = np.array([3.0, 2.0, 1.0, 0.5])
    n2 = float(np.sum(s * s))
    assert O._pick_rank(s, n2, math.sqrt(1.25) + 1e-12, None) == (2, True)
    assert O._pick_rank(s, n2, math.sqrt(1.25) - 1e-9, None) == (3, True)
    assert O._pick_rank(s, n2, 100.0, None) == (1, True)
    assert O._pick_rank(s, n2, 0.1, 2) == (2, False)


@pytest.mark.slow
def test_table_beps_ttsvd_ranks():
    """Example 2 (160^4): the TT-SVD ranks printed in Table "Beps"."""
    a = ttgen.sin_norm_tensor(4, 160)
    for row in _read_golden("table_beps_ttsvd_ranks.txt"):
        eps = float(row[0])
        want = [1] + [int(x) for x in row[1:]] + [1]
        _, rep = oracle.tt_svd(a, [160] * 4, eps=eps, sweep="L2R")
        assert rep["ranks"] == want, (eps, rep["ranks"])


# --------------------------------------------------------------------- masked completion
def test_completion_direction_is_the_directional_derivative():
    """J g (sum over k of the train with core k replaced by g_k) is the exact
    first-order term of A(G + h g): central differences agree to O(h^2)."""
    dims = [3, 4, 2, 5]
    cores = ttgen.gaussian_cores(dims, [1, 2, 3, 2, 1], 31)
    rng = np.random.default_rng(32)
    idx = np.stack([rng.integers(0, n, 40) for n in dims], axis=1)
    vals = rng.standard_normal(40)
    e = oracle.tt_sample(cores, idx) - vals
    g = oracle.tt_sample_grad(cores, idx, e)
    jg = sum(oracle.tt_sample(cores[:k] + [g[k]] + cores[k + 1:], idx) for k in range(len(cores)))
    h = 1e-5
    plus = oracle.tt_sample([c + h * gk for c, gk in zip(cores, g)], idx)
    minus = oracle.tt_sample([c - h * gk for c, gk in zip(cores, g)], idx)
    fd = (plus - minus) / (2 * h)
    np.testing.assert_allclose(jg, fd, rtol=1e-6, atol=1e-6 * np.max(np.abs(jg)))


def test_completion_step_size_minimises_the_linearised_residual():
    dims = [4, 3, 5]
    cores = ttgen.gaussian_cores(dims, [1, 2, 2, 1], 33)
    rng = np.random.default_rng(34)
    idx = np.stack([rng.integers(0, n, 30) for n in dims], axis=1)
    vals = rng.standard_normal(30)
    new, f, alpha = oracle.completion_step(cores, idx, vals)
    e = oracle.tt_sample(cores, idx) - vals
    assert f == pytest.approx(0.5 * float(e @ e), rel=1e-14)
    g = oracle.tt_sample_grad(cores, idx, e)
    jg = sum(oracle.tt_sample(cores[:k] + [g[k]] + cores[k + 1:], idx) for k in range(len(cores)))
    lin = lambda a: float(np.sum((e - a * jg) ** 2))
    assert lin(alpha) <= lin(alpha * 1.01) and lin(alpha) <= lin(alpha * 0.99)
    # the step is along -g with that size
    for c, n, gk in zip(cores, new, g):
        np.testing.assert_allclose(n, c - alpha * gk, rtol=1e-15, atol=1e-15)


def test_completion_descends_on_a_low_rank_tensor():
    """Observed entries of an exact TT of ranks (1,2,2,1): steps from a nearby
    start decrease f and bring the unobserved entries closer."""
    dims = [6, 5, 7]
    true = ttgen.gaussian_cores(dims, [1, 2, 2, 1], 35)
    full = oracle.tt_reconstruct(true)
    rng = np.random.default_rng(36)
    flat = rng.permutation(full.size)[: full.size // 2]
    idx = np.stack(np.unravel_index(flat, dims, order="F"), axis=1)
    cores = [c + 0.05 * rng.standard_normal(c.shape) for c in true]
    fs = []
    for _ in range(20):
        cores, f, _ = oracle.completion_step(cores, idx, full[flat])
        fs.append(f)
    assert fs[-1] < 0.1 * fs[0]
    rest = np.setdiff1d(np.arange(full.size), flat)
    err0 = np.linalg.norm(oracle.tt_reconstruct([c for c in true])[rest] - full[rest])
    assert err0 == 0.0
    err = np.linalg.norm(oracle.tt_reconstruct(cores)[rest] - full[rest]) / np.linalg.norm(full[rest])
    assert err < 0.05


# --------------------------------------------------------------------- Riemannian completion step
def _random_train(dims, ranks, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((ranks[k], dims[k], ranks[k + 1])) for k in range(len(dims))]


def _all_indices(dims):
    return np.array(np.unravel_index(np.arange(int(np.prod(dims))), dims, order="F")).T


def test_orthogonal_forms_keep_the_train():
    """Def. 2.2: the QR sweeps give left-orthogonal cores 1..d-1 (right-orthogonal
    cores 2..d) and represent the same tensor."""
    dims, ranks = [3, 4, 3, 2], [1, 2, 3, 2, 1]
    cores = _random_train(dims, ranks, 40)
    x = oracle.tt_reconstruct(cores)
    U, V = oracle.left_orthogonalize(cores), oracle.right_orthogonalize(cores)
    np.testing.assert_allclose(oracle.tt_reconstruct(U), x, atol=1e-13 * np.max(np.abs(x)))
    np.testing.assert_allclose(oracle.tt_reconstruct(V), x, atol=1e-13 * np.max(np.abs(x)))
    for k in range(len(dims) - 1):
        u = U[k].reshape(-1, ranks[k + 1], order="F")
        np.testing.assert_allclose(u.T @ u, np.eye(ranks[k + 1]), atol=1e-13)
    for k in range(1, len(dims)):
        v = V[k].reshape(ranks[k], -1, order="F")
        np.testing.assert_allclose(v @ v.T, np.eye(ranks[k]), atol=1e-13)


def test_mixed_gradient_is_the_linear_map_of_core_k():
    """L(C) = sum_s w_s (L_1..L_{k-1} C R_{k+1}..R_d)[idx_s] is linear in C, so
    <dL/dC_k, E> = L(E) for every E, evaluated by sampling the train with core
    k replaced; with equal left and right cores it is the plain gradient."""
    dims, ranks = [3, 4, 2, 5], [1, 2, 3, 2, 1]
    Lc, Rc = _random_train(dims, ranks, 41), _random_train(dims, ranks, 42)
    rng = np.random.default_rng(43)
    idx = np.stack([rng.integers(0, n, 50) for n in dims], axis=1)
    w = rng.standard_normal(50)
    g = oracle.tt_sample_grad_mixed(Lc, Rc, idx, w)
    for k in range(len(dims)):
        E = rng.standard_normal(Lc[k].shape)
        direct = float(w @ oracle.tt_sample(Lc[:k] + [E] + Rc[k + 1:], idx))
        assert float(np.sum(g[k] * E)) == pytest.approx(direct, rel=1e-12, abs=1e-12)
    for a, b in zip(oracle.tt_sample_grad_mixed(Lc, Lc, idx, w), oracle.tt_sample_grad(Lc, idx, w)):
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-13)


def test_riemannian_gradient_is_the_tangent_projection():
    """The projection onto the tangent space at X of a dense Z (all entries
    sampled): idempotent, self-adjoint, the residual orthogonal to the
    result, and X itself (a tangent vector of the manifold at X) left alone;
    the rank-2r train X + t xi reconstructs X + t xi."""
    dims, ranks = [3, 4, 3, 2], [1, 2, 3, 2, 1]
    cores = _random_train(dims, ranks, 44)
    idx = _all_indices(dims)
    x = oracle.tt_reconstruct(cores)

    def proj(z):
        U, V, dC = oracle.riemannian_gradient(cores, idx, z)
        return oracle.tt_reconstruct(oracle.tangent_train(U, V, dC))

    rng = np.random.default_rng(45)
    z1, z2 = rng.standard_normal(x.size), rng.standard_normal(x.size)
    p1 = proj(z1)
    scale = np.max(np.abs(p1))
    np.testing.assert_allclose(proj(p1), p1, atol=1e-12 * scale)
    np.testing.assert_allclose(proj(x), x, atol=1e-12 * np.max(np.abs(x)))
    assert float(p1 @ z2) == pytest.approx(float(z1 @ proj(z2)), rel=1e-11)
    assert abs(float((z1 - p1) @ p1)) <= 1e-11 * float(p1 @ p1)
    U, V, dC = oracle.riemannian_gradient(cores, idx, z1)
    np.testing.assert_allclose(oracle.tt_reconstruct(oracle.tangent_train(U, V, dC, t=-0.7, base=True)),
                               x - 0.7 * p1, atol=1e-12 * scale)


def test_rgrad_step_minimises_f_on_its_line_and_recovers_a_low_rank_train():
    """alpha is the exact minimiser of f(X - alpha xi) (before the retraction),
    the retraction keeps the ranks, and 40 steps recover an exact rank-(2,2,2)
    train from 60% of its entries (started 30% off)."""
    dims, r = [6, 5, 6, 5], [2, 2, 2]
    a, _ = ttgen.gaussian_tt_tensor(dims, r, 0.0, 11)
    rng = np.random.default_rng(46)
    obs = rng.permutation(a.size)[: int(0.6 * a.size)]
    idx = np.array(np.unravel_index(obs, dims, order="F")).T
    vals = a[obs]
    start, _ = oracle.tt_utv(a, dims, ranks=r, sweep="L2R", variant="ULV")
    cores = [c + 0.3 * np.std(c) * rng.standard_normal(c.shape) for c in start]
    z = oracle.tt_sample(cores, idx) - vals
    U, V, dC = oracle.riemannian_gradient(cores, idx, z)
    pxi = oracle.tt_sample(oracle.tangent_train(U, V, dC), idx)
    new, f0, alpha = oracle.rgrad_step(cores, idx, vals, r)
    assert f0 == pytest.approx(0.5 * float(z @ z))
    line = lambda t: 0.5 * float((z - t * pxi) @ (z - t * pxi))
    assert line(alpha) <= min(line(alpha * 0.99), line(alpha * 1.01))
    assert [c.shape[2] for c in new[:-1]] == r
    c = new
    for _ in range(39):
        c, _, _ = oracle.rgrad_step(c, idx, vals, r)
    assert np.linalg.norm(oracle.tt_reconstruct(c) - a) <= 1e-7 * np.linalg.norm(a)


# ---------------------------------------------------------------- deflation inner kernel
DEFL_COMBOS = [("L2R", "ULV"), ("R2L", "URV"), ("L2R", "URV")]


@pytest.mark.parametrize("sweep,variant", DEFL_COMBOS)
def test_deflation_exact_tt_rank_reconstructs(sweep, variant):
    """Thm. 3.1/3.2 with eps_k = 0 and the deflation inner kernel: after one
    power step every vector lies in the row space of the tall unfolding, so r
    orthonormal vectors span it and a tensor of exact TT-ranks is recovered."""
    dims = [5, 6, 7, 5]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 4, 3], 0.0, 11)
    cores, rep = oracle.tt_utv(a, dims, ranks=[3, 4, 3], sweep=sweep, variant=variant, q=1, seed=3,
                               inner="deflation")
    assert _rse(a, cores) < 1e-12
    assert rep["ranks"] == [1, 3, 4, 3, 1]


def test_deflation_converged_vectors_are_the_singular_vectors():
    """d = 2 on a matrix of known, well separated spectrum: with many power steps
    vector j converges to the j-th right singular vector and its energy to
    sigma_j^2 (LAPACK SVD as the library reference).  Without the projection of
    the earlier vectors every search would return the first one."""
    rng = np.random.default_rng(5)
    U, _ = np.linalg.qr(rng.standard_normal((60, 20)))
    V, _ = np.linalg.qr(rng.standard_normal((20, 20)))
    sig = 2.0 ** -np.arange(20)
    M = (U * sig) @ V.T                           # 60 x 20
    a = M.reshape(-1, order="F")
    for sweep, variant in DEFL_COMBOS:
        cores, rep = oracle.tt_utv(a, [60, 20], ranks=[6], sweep=sweep, variant=variant, q=80, seed=2,
                                   inner="deflation")
        s = rep["s"][0]
        np.testing.assert_allclose(s, sig[:6], rtol=1e-12)
        # the core side: the right singular vectors (R2L, n = 20) or the left ones (L2R, n = 60)
        side = V[:, :6] if sweep == "R2L" and variant == "URV" else U[:, :6]
        core = cores[1].reshape(6, 20).T if side.shape[0] == 20 else cores[0].reshape(60, 6)
        assert np.max(np.abs(np.abs(core.T @ side) - np.eye(6))) < 1e-10
        err = np.linalg.norm(oracle.tt_reconstruct(cores) - a)
        assert err == pytest.approx(math.sqrt(np.sum(sig[6:] ** 2)), rel=1e-10)


@pytest.mark.parametrize("sweep,variant", DEFL_COMBOS)
def test_deflation_pythagoras_equality(sweep, variant):
    """The deflation vectors are orthonormal and the carry is the exact
    projection, so ||A - A_TT||^2 = sum delta_k^2 holds with equality, in both
    rank modes; and the eps-mode error stays within eps."""
    dims = [6, 7, 5, 6, 4]
    a, _ = ttgen.gaussian_tt_tensor(dims, [3, 5, 5, 3], 1e-2, 21)
    for kw in (dict(ranks=[3, 4, 4, 3]), dict(eps=3e-2)):
        cores, rep = oracle.tt_utv(a, dims, sweep=sweep, variant=variant, q=1, seed=9, inner="deflation", **kw)
        err2 = np.sum((oracle.tt_reconstruct(cores) - a) ** 2)
        bound2 = np.sum(np.square(rep["delta"]))
        assert err2 > 0
        assert abs(err2 - bound2) <= 1e-9 * bound2
        if "eps" in kw:
            assert rep["rank_rule_met"]
            assert math.sqrt(err2) <= 3e-2 * np.linalg.norm(a) * (1 + 1e-12)
        # core-side orthogonality (Def. 2.2)
        for g in (cores[:-1] if sweep == "L2R" else cores[1:]):
            M = (g.reshape(-1, g.shape[2], order="F") if sweep == "L2R"
                 else g.reshape(g.shape[0], -1, order="F").T)
            assert np.max(np.abs(M.T @ M - np.eye(M.shape[1]))) < 1e-13


def test_deflation_converged_eps_ranks_are_tt_svd_ranks():
    """Prescribed accuracy on an Example-2 type tensor (smooth, 24^4): with
    converged vectors the kept energies are the leading sigma_i^2, so the rank
    rule picks the TT-SVD ranks at every tolerance (TT-SVD pinned above by
    Eckart-Young and Table "Beps")."""
    a = ttgen.sin_norm_tensor(4, 24)
    dims = [24] * 4
    for eps in (1e-2, 1e-3, 1e-4, 1e-6):
        _, rs = oracle.tt_svd(a, dims, eps=eps, sweep="L2R")
        for sweep, variant in (("L2R", "ULV"), ("R2L", "URV")):
            cores, rep = oracle.tt_utv(a, dims, eps=eps, sweep=sweep, variant=variant, q=40, seed=1,
                                       inner="deflation")
            _, rsv = oracle.tt_svd(a, dims, eps=eps, sweep=sweep)
            assert rep["ranks"] == rsv["ranks"], (eps, sweep, rep["ranks"], rsv["ranks"])
            assert _rse(a, cores) <= eps * (1 + 1e-9)


def test_deflation_rejects_alg4():
    a = np.zeros(4 * 5)
    with pytest.raises(ValueError):
        oracle.tt_utv(a, [4, 5], ranks=[1], sweep="R2L", variant="ULV", inner="deflation")
