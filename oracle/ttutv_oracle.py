"""FP64 CPU oracle of the TT-UTV sweep (Wang, Che & Wei, "Effective algorithms
for tensor-train decomposition via the UTV framework").

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the library.  Plain NumPy in float64;
LAPACK QR and SVD (through numpy.linalg, plus one batched QR through torch's
CPU build for very wide unfoldings) are used as library steps.  Nothing
here is blocked, fused or reordered beyond what the paper's algorithms state.

Data model (paper Sec. 2.1): a tensor is a flat vector in reverse
lexicographic order (i1 fastest, the `ivec` map), and every reshape is
column-major (NumPy order='F'), as MATLAB's reshape used by the paper.  A TT
core k is an array of shape (r_{k-1}, I_k, r_k); its flat layout in the C ABI
is the same array flattened in column-major order.

Inner low-rank kernel.  The paper leaves the truncated UTV to third-party
routines; this oracle uses a randomized power-iteration UTV: a Gaussian test
matrix G on the core side of the unfolding, q power steps with Householder
re-orthonormalisation after every product, then a triangular factorisation of
the projected matrix and an SVD of its ell x ell triangle to rank-reveal it
(the SVD is the UTV whose middle factor is diagonal, Sec. 2.2).

Deflation inner kernel (inner="deflation").  The paper's fastest variant,
TT-ULV with USV-plus (Sec. 3.3, Sec. 4), estimates singular vectors of the
unfolding one at a time by power iteration and stops once the latest estimate
is small enough.  The reading here: on the tall orientation A (m x n) of the
unfolding, vector j starts from column j of the same Gaussian test matrix
with the vectors already found projected out, takes q power steps
x <- P(A^T A x) / ||P(A^T A x)|| (P: projection onto the complement of the
earlier vectors, two Gram-Schmidt rounds), and its energy ||A v_j||^2 joins
the kept energy; the search stops at the fixed rank, or at the first j where
||C||^2 minus the kept energy is within eps_k^2 (the rank rule after
Alg. 2).  The vectors are orthonormal, so the step error is exactly
sqrt(||C||^2 - ||A V||^2), as for the sketched factorisation.

Function -> passage -> pin (see tests/test_oracle.py):
  splitmix64         SplitMix64 (Steele, Lea & Flood 2014)   published outputs
  sketch_gaussian    counter-based Gaussian test matrix         moments, KS test
  tt_utv ULV  L2R    Alg. 1 / Alg. 2                            exact-rank recon, Pythagoras, d=2 Eckart-Young
  tt_utv URV  R2L    Alg. 3 (+ its prescribed-accuracy form)    same
  tt_utv URV  L2R    index-reversal remark after Thm. 3.2       equals the reversed R2L sweep
  tt_utv ULV  R2L    Alg. 4 (appendix)                          Prop. A.1 sum bound
  tt_utv inner="deflation"  the USV-plus inner kernel of Sec. 3.3 / Sec. 4 (one vector at a time)
                                                                 exact-rank recon, converged = SVD, Pythagoras,
                                                                 converged eps ranks = TT-SVD ranks
  tt_svd             TT-SVD (Oseledets 2011)                     Table "Beps" ranks, Eckart-Young
  tt_reconstruct     Eq. (TT)                                    closed-form rank-2 TT of a sum
  tt_sample          Eq. (TT) at given multi-indices             equals reconstruct at those entries
  tt_sample_grad     gradient of a weighted sum of sampled entries   central finite differences
  tt_reconstruct_grad  gradient of <gout, A_TT> (dense gout)      central differences, Euler's identity,
                                                                 equals tt_sample_grad for a sparse gout
"""
import math

import numpy as np

_GAMMA = 0x9E3779B97F4A7C15
_MIX1 = 0xBF58476D1CE4E5B9
_MIX2 = 0x94D049BB133111EB


# --------------------------------------------------------------------------
# Random test matrices: one counter-based generator, defined here from its
# published description and independently in the library.
# --------------------------------------------------------------------------
def splitmix64(seed, t):
    """t-th output (t >= 1) of SplitMix64 started from state `seed`.

    SplitMix64 advances its state by the golden-ratio increment and outputs a
    two-round xor-shift-multiply finaliser of the new state; the t-th output is
    therefore a pure function of seed + t * increment (mod 2^64).
    """
    t = np.asarray(t, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + t * np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_MIX2)
        z = z ^ (z >> np.uint64(31))
    return z


def sketch_gaussian(seed, mode, n_mode, n_rank, ell, mode_fastest):
    """Gaussian test matrix G (n x ell), n = n_mode * n_rank, of the step that
    produces core `mode`.

    Entry (i, beta, j) -- mode index i, carried-rank index beta, column j --
    uses counter c = mode<<48 | j<<32 | beta<<16 | i and the SplitMix64 outputs
    2c+1 and 2c+2 as uniforms u1 in (0,1] and u2 in [0,1) (top 53 bits), turned
    into one N(0,1) value by the Box-Muller transform sqrt(-2 ln u1) cos(2 pi u2).
    The row of G is i + n_mode*beta if `mode_fastest`, else beta + n_rank*i,
    so the same (i, beta) pair gets the same row values in either ordering.
    """
    for v, lim in ((mode, 1 << 15), (n_mode, 1 << 16), (n_rank, 1 << 16), (ell, 1 << 16)):
        if not 0 <= v < lim:
            raise ValueError("sketch index out of the generator's range")
    i = np.arange(n_mode, dtype=np.uint64)[:, None, None]
    b = np.arange(n_rank, dtype=np.uint64)[None, :, None]
    j = np.arange(ell, dtype=np.uint64)[None, None, :]
    c = (np.uint64(mode) << np.uint64(48)) | (j << np.uint64(32)) | (b << np.uint64(16)) | i
    two_c = c * np.uint64(2)
    x1 = splitmix64(seed, two_c + np.uint64(1))
    x2 = splitmix64(seed, two_c + np.uint64(2))
    u1 = ((x1 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (x2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    g = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)   # (n_mode, n_rank, ell)
    if mode_fastest:
        return g.reshape(n_mode * n_rank, ell, order="F")
    return np.transpose(g, (1, 0, 2)).reshape(n_mode * n_rank, ell, order="F")


# --------------------------------------------------------------------------
# Small helpers
# --------------------------------------------------------------------------
def _orth(M):
    """Orthonormal basis of the columns of M by Householder QR (LAPACK)."""
    q, _ = np.linalg.qr(M, mode="reduced")
    return q


def canonical_signs(V):
    """Sign (+1/-1) per column of V that makes each column's largest-magnitude
    entry positive (lowest row index on ties).  The gauge of a TT core is not
    fixed by the paper; this fixes it so that two correct sweeps compare."""
    if V.shape[1] == 0:
        return np.ones(0)
    idx = np.argmax(np.abs(V), axis=0)
    s = np.sign(V[idx, np.arange(V.shape[1])])
    s[s == 0] = 1.0
    return s


def step_tall_view(n, m, sweep):
    """Shape bookkeeping shared by the tests: the unfolding C of one step is
    n x m in the L2R sweep (core side = rows, Alg. 1 step 3) and m x n in the
    R2L sweep (core side = columns, Alg. 3 step 3)."""
    return (n, m) if sweep == "L2R" else (m, n)


def _pick_rank(s, normC2, eps_k, max_rank):
    """Smallest r >= 1 with ||C||^2 - sum_{i<=r} s_i^2 <= eps_k^2 (the rank rule
    after Alg. 2).  Returns (r, satisfied)."""
    kept = np.cumsum(s * s)
    ok = np.nonzero(normC2 - kept <= eps_k * eps_k)[0]
    if ok.size == 0:
        r, sat = len(s), False
    else:
        r, sat = int(ok[0]) + 1, True
    if max_rank is not None and r > max_rank:
        r, sat = max_rank, False
    return max(r, 1), sat


def _ell_fixed(r, p, n, m):
    return min(r + p, n, m)


# --------------------------------------------------------------------------
# Randomized UTV factorisations of one unfolding
# --------------------------------------------------------------------------
def _rand_urv_tall(C, G, q):
    """Randomized URV of C (m x n): C = U R V^T + E with E V = 0.

    The right (core-side) basis V spans (C^T C)^(q+1) G: a range sketch C G,
    q power steps through C^T and C, and a last product with C^T, each product
    re-orthonormalised.  Then C V = U R (Householder QR, R upper triangular).
    G None means ell >= n: V is the identity and the factorisation is exact.
    """
    if G is None:
        V = np.eye(C.shape[1])
    else:
        Q = _orth(C @ G)
        for _ in range(q):
            W = _orth(C.T @ Q)
            Q = _orth(C @ W)
        V = _orth(C.T @ Q)
    U, R = np.linalg.qr(C @ V, mode="reduced")
    return U, R, V


def _rand_ulv_wide(C, G, q):
    """Randomized ULV of C (n x m): C = U L V^T + E with U^T E = 0.

    The left (core-side) basis U spans (C C^T)^(q+1) G: a sketch C^T G, q
    power steps through C and C^T, and a last product with C, each product
    re-orthonormalised.  Then U^T C = L V^T (an LQ factorisation computed as
    the QR of its transpose; L lower triangular).
    """
    if G is None:
        U = np.eye(C.shape[0])
    else:
        Z = _orth(C.T @ G)
        for _ in range(q):
            U = _orth(C @ Z)
            Z = _orth(C.T @ U)
        U = _orth(C @ Z)
    Vq, Rq = np.linalg.qr((U.T @ C).T, mode="reduced")
    return U, Rq.T, Vq


def _rand_ulv_tall(C, G, q):
    """Randomized ULV of C (m x n) with the orthogonality on the range side
    (the factorisation Alg. 4 asks for): U spans (C C^T)^q C G, then
    U^T C = L V^T (LQ).  G None means ell >= n (G = identity)."""
    if G is None:
        G = np.eye(C.shape[1])
    U = _orth(C @ G)
    for _ in range(q):
        W = _orth(C.T @ U)
        U = _orth(C @ W)
    Vq, Rq = np.linalg.qr((U.T @ C).T, mode="reduced")
    return U, Rq.T, Vq


# --------------------------------------------------------------------------
# The sweeps
# --------------------------------------------------------------------------
def _as_flat(a, dims):
    a = np.asarray(a, dtype=np.float64).reshape(-1, order="F")
    if a.size != int(np.prod(dims)):
        raise ValueError("tensor size does not match dims")
    return a


def _rank_targets(d, ranks, eps, normA, weights, sum_bound):
    """Per-step fixed ranks (list r_0..r_d) or per-step tolerances eps_k."""
    if ranks is not None:
        ranks = list(ranks)
        if len(ranks) == d - 1:
            ranks = [1] + ranks + [1]
        if len(ranks) != d + 1 or ranks[0] != 1 or ranks[-1] != 1 or min(ranks) < 1:
            raise ValueError("ranks must be r_0..r_d with r_0 = r_d = 1")
        return ranks, None
    if eps is None or eps < 0:
        raise ValueError("give ranks or eps >= 0")
    if weights is None:
        # Alg. 2 default: equal weights with sum w_k^2 = 1.  The appendix's
        # ULV right-to-left sweep only has the sum bound, so it splits eps
        # evenly: eps_k = eps ||A|| / (d-1).
        w = np.full(d - 1, 1.0 / (d - 1) if sum_bound else 1.0 / math.sqrt(d - 1))
    else:
        w = np.asarray(weights, dtype=np.float64)
        if w.shape != (d - 1,):
            raise ValueError("need d-1 weights")
    return None, w * eps * normA


def _truncate(U, T, V, r):
    """Rank-r truncation of U T V^T after rank-revealing the triangle T by its
    SVD T = W S Z^T: returns U1 = U W_r, S_r, V1 = V Z_r, all singular values."""
    W, s, Zt = np.linalg.svd(T)
    return U @ W[:, :r], s[:r], V @ Zt[:r, :].T, s


def tt_utv(a, dims, ranks=None, eps=None, sweep="L2R", variant="ULV", q=1, p=8,
           seed=0, weights=None, max_rank=None, inner="sketch", _labels=None):
    """TT-UTV of the tensor `a` (flat, i1 fastest) with dims I_1..I_d.

    sweep/variant: ("L2R","ULV") Alg. 1/2; ("R2L","URV") Alg. 3 and its
    prescribed-accuracy form; ("R2L","ULV") Alg. 4; ("L2R","URV") index
    reversal + Alg. 3; variant "SVD" is TT-SVD in the given direction.
    Fixed ranks: `ranks` = r_0..r_d (or r_1..r_{d-1}); prescribed accuracy:
    `eps` (relative), eps_k = w_k eps ||A||_F.
    inner: "sketch" (the randomized power-iteration factorisation) or
    "deflation" (one vector at a time, the USV-plus reading; ULV/URV sweeps
    that keep the core side orthonormal, not Alg. 4).
    Returns (cores, report).  cores[k-1] has shape (r_{k-1}, I_k, r_k).
    """
    dims = [int(x) for x in dims]
    d = len(dims)
    if d < 2:
        raise ValueError("need d >= 2")
    a = _as_flat(a, dims)
    if variant == "SVD":
        return tt_svd(a, dims, ranks=ranks, eps=eps, sweep=sweep, weights=weights, max_rank=max_rank)
    if inner not in ("sketch", "deflation"):
        raise ValueError("unknown inner factorisation")
    if inner == "deflation" and sweep == "R2L" and variant == "ULV":
        raise ValueError("the deflation inner kernel keeps the core side orthonormal; Alg. 4 does not")
    if sweep == "L2R" and variant == "URV":
        return _urv_l2r_by_reversal(a, dims, ranks, eps, q, p, seed, weights, max_rank, inner)
    labels = list(range(1, d + 1)) if _labels is None else list(_labels)
    normA = math.sqrt(float(a @ a))
    sum_bound = (sweep == "R2L" and variant == "ULV")
    fixed, eps_k = _rank_targets(d, ranks, eps, normA, weights, sum_bound)
    rep = {"ranks": [1] * (d + 1), "delta": [], "normC": [], "ell": [], "s": [],
           "norm_A": normA, "rank_rule_met": True}
    cores = [None] * d
    C = a
    if sweep == "L2R":
        if variant != "ULV":
            raise ValueError("unknown variant")
        r_prev = 1
        for k in range(1, d):                    # Alg. 1/2: k = 1..d-1
            n = r_prev * dims[k - 1]
            m = C.size // n
            Cm = C.reshape(n, m, order="F")      # reshape to [r_{k-1} I_k, rest]
            if inner == "deflation":
                U1, carry_t, s_all, dk, nC = _deflation_step(
                    Cm.T, q, seed, labels[k - 1], dims[k - 1], r_prev, False,
                    fixed[k] if fixed else None, eps_k[k - 1] if fixed is None else None, max_rank, rep)
                ell = U1.shape[1]
                C = carry_t.T.reshape(-1, order="F")                             # C = U1^T C_k = L11 V1^T
            else:
                U1, s_r, V1, s_all, ell, dk, nC = _step(
                    Cm, "ulv_wide", fixed[k] if fixed else None, eps_k[k - 1] if fixed is None else None,
                    q, p, seed, labels[k - 1], dims[k - 1], r_prev, False, k == 1,
                    rep["ranks"][k - 1] if k > 1 else None, max_rank, rep)
                C = (s_r[:, None] * V1.T).reshape(-1, order="F")                 # C = L11 V1^T
            r = U1.shape[1]
            cores[k - 1] = U1.reshape(r_prev, dims[k - 1], r, order="F")   # core from U1
            rep["ranks"][k] = r
            rep["delta"].append(dk); rep["normC"].append(nC); rep["ell"].append(ell); rep["s"].append(s_all)
            r_prev = r
        cores[d - 1] = C.reshape(r_prev, dims[d - 1], 1, order="F")
    elif sweep == "R2L":
        kind = "urv_tall" if variant == "URV" else "ulv_tall" if variant == "ULV" else None
        if kind is None:
            raise ValueError("unknown variant")
        r_next = 1
        for k in range(d, 1, -1):                # Alg. 3/4: k = d..2
            n = dims[k - 1] * r_next
            m = C.size // n
            Cm = C.reshape(m, n, order="F")      # reshape to [I_1..I_{k-1}, I_k r_k]
            if inner == "deflation":
                V1, carry, s_all, dk, nC = _deflation_step(
                    Cm, q, seed, labels[k - 1], dims[k - 1], r_next, True,
                    fixed[k - 1] if fixed else None, eps_k[k - 2] if fixed is None else None, max_rank, rep)
                ell = V1.shape[1]
                C = carry.reshape(-1, order="F")                                  # C = C_k V1 = U1 R11
            else:
                U1, s_r, V1, s_all, ell, dk, nC = _step(
                    Cm, kind, fixed[k - 1] if fixed else None, eps_k[k - 2] if fixed is None else None,
                    q, p, seed, labels[k - 1], dims[k - 1], r_next, True, k == d,
                    rep["ranks"][k] if k < d else None, max_rank, rep)
                C = (U1 * s_r[None, :]).reshape(-1, order="F")                    # C = U1 R11 (Alg. 4: U^ L11)
            r = V1.shape[1]
            cores[k - 1] = V1.T.reshape(r, dims[k - 1], r_next, order="F")  # core from V1^T
            rep["ranks"][k - 1] = r
            rep["delta"].insert(0, dk); rep["normC"].insert(0, nC); rep["ell"].insert(0, ell); rep["s"].insert(0, s_all)
            r_next = r
        cores[0] = C.reshape(1, dims[0], r_next, order="F")
    else:
        raise ValueError("unknown sweep")
    rep["err_bound"] = (float(np.sum(np.abs(rep["delta"]))) if sum_bound
                        else math.sqrt(float(np.sum(np.square(rep["delta"])))))
    return cores, rep


def _step(Cm, kind, r_fixed, eps_k, q, p, seed, label, n_mode, n_rank, mode_fastest,
          first, r_prev_step, max_rank, rep):
    """One truncated UTV of the unfolding Cm.  Returns U1 (the core side for
    ulv_wide; the range side otherwise), the kept singular values, V1,
    all singular values of the triangle, ell, the step error and ||C||_F."""
    if kind == "ulv_wide":
        n, m = Cm.shape
    else:
        m, n = Cm.shape
    normC2 = float(np.sum(Cm * Cm))
    if r_fixed is not None:
        r_want = min(r_fixed, n, m)
        ell = _ell_fixed(r_want, p, n, m)
    else:
        ell = min((2 * p) if first else (r_prev_step + p), n, m)
    while True:
        G = None if ell >= n else sketch_gaussian(seed, label, n_mode, n_rank, ell, mode_fastest)
        if kind == "ulv_wide":
            U, T, V = _rand_ulv_wide(Cm, G, q)
        elif kind == "urv_tall":
            U, T, V = _rand_urv_tall(Cm, G, q)
        else:
            U, T, V = _rand_ulv_tall(Cm, G, q)
        s_all = np.linalg.svd(T, compute_uv=False)
        if r_fixed is not None:
            r = min(r_want, T.shape[0])
            break
        r, sat = _pick_rank(s_all, normC2, eps_k, max_rank)
        r = min(r, T.shape[0])
        if sat or ell >= min(n, m) or (max_rank is not None and r >= max_rank):
            if not sat:
                rep["rank_rule_met"] = False
            break
        ell = min(2 * ell, n, m)
    U1, s_r, V1, _ = _truncate(U, T, V, r)
    core_side = U1 if kind == "ulv_wide" else V1
    sg = canonical_signs(core_side)
    U1 = U1 * sg[None, :]
    V1 = V1 * sg[None, :]
    if kind == "ulv_wide":
        approx = (U1 * s_r[None, :]) @ V1.T
    else:
        approx = (U1 * s_r[None, :]) @ V1.T
    dk = float(np.linalg.norm(Cm - approx))       # step error ||E||_F, measured directly
    return U1, s_r, V1, s_all, ell, dk, math.sqrt(normC2)


def _project_out(V, x):
    """x less its components along the orthonormal columns of V: two rounds of
    classical Gram-Schmidt (the second removes what rounding left after the
    first)."""
    for _ in range(2):
        x = x - V @ (V.T @ x)
    return x


def _deflation_basis(A, G, q, r_want, eps_k):
    """Core-side basis of the tall A (m x n), one vector at a time.

    Vector j starts from column j of G with the vectors found so far projected
    out, takes q power steps x <- P(A^T (A x)) normalised (a step whose product
    vanishes keeps x), and adds its energy ||A v_j||^2 to the kept energy.
    Stops after r_want vectors (fixed rank), or at the first j with
    ||A||^2 - kept <= eps_k^2, or when G's columns run out.
    Returns V (n x r, orthonormal columns), the energies, whether the rule was
    met, and ||A||_F^2."""
    n = A.shape[1]
    normC2 = float(np.sum(A * A))
    V = np.zeros((n, 0))
    e = []
    kept = 0.0
    sat = r_want is not None
    for j in range(G.shape[1]):
        x = _project_out(V, G[:, j])
        x = x / np.linalg.norm(x)
        for _ in range(q):
            z = _project_out(V, A.T @ (A @ x))
            nz = np.linalg.norm(z)
            if nz > 0.0:
                x = z / nz
        V = np.column_stack([V, x])
        y = A @ x
        e.append(float(y @ y))
        kept += e[-1]
        if r_want is not None:
            if V.shape[1] == r_want:
                break
        elif normC2 - kept <= eps_k * eps_k:
            sat = True
            break
    return V, np.array(e), sat, normC2


def _deflation_step(A, q, seed, label, n_mode, n_rank, mode_fastest, r_fixed, eps_k, max_rank, rep):
    """One step with the deflation inner kernel on the tall A (m x n): the basis
    V1 (n x r, signs canonical), the carry A V1 (m x r), the estimated singular
    values sqrt(energy), the step error ||A - A V1 V1^T||_F (measured directly)
    and ||A||_F."""
    m, n = A.shape
    if r_fixed is not None:
        r_want = min(r_fixed, n, m)
        cap = r_want
    else:
        r_want = None
        cap = min(n, m) if max_rank is None else min(n, m, max_rank)
    G = sketch_gaussian(seed, label, n_mode, n_rank, cap, mode_fastest)
    V, e, sat, normC2 = _deflation_basis(A, G, q, r_want, eps_k)
    if not sat:
        rep["rank_rule_met"] = False
    V1 = V * canonical_signs(V)[None, :]
    carry = A @ V1
    dk = float(np.linalg.norm(A - carry @ V1.T))
    return V1, carry, np.sqrt(e), dk, math.sqrt(normC2)


def _reverse_modes(a, dims):
    t = np.asarray(a).reshape(dims, order="F")
    return np.transpose(t, tuple(range(len(dims) - 1, -1, -1))).reshape(-1, order="F")


def _urv_l2r_by_reversal(a, dims, ranks, eps, q, p, seed, weights, max_rank, inner="sketch"):
    """TT-URV with left-orthogonal cores (remark after Thm. 3.2): reverse the
    index order, run the right-to-left URV sweep, reverse the cores back."""
    d = len(dims)
    rdims = dims[::-1]
    rranks = None
    if ranks is not None:
        rr = list(ranks)
        if len(rr) == d - 1:
            rr = [1] + rr + [1]
        rranks = rr[::-1]
    rw = None if weights is None else list(weights)[::-1]
    cores_b, rep = tt_utv(_reverse_modes(a, dims), rdims, ranks=rranks, eps=eps, sweep="R2L",
                          variant="URV", q=q, p=p, seed=seed, weights=rw, max_rank=max_rank,
                          inner=inner, _labels=list(range(d, 0, -1)))
    cores = [np.transpose(g, (2, 1, 0)) for g in cores_b[::-1]]
    rep["ranks"] = rep["ranks"][::-1]
    for key in ("delta", "normC", "ell", "s"):
        rep[key] = rep[key][::-1]
    return cores, rep


def _r_factor(T):
    """An upper-triangular R with T = Q R for a tall T (m x n, m >= n).

    Tree QR: the R of the stacked block triangles [R_1; R_2; ...] of row blocks
    T_i = Q_i R_i is an R of T (exact up to rounding and the signs of R's rows,
    which change no singular value or right singular vector).  The block QRs go
    to LAPACK as one batched call on torch's CPU build, which spreads them over
    the host threads; a single QR of a 4,096,000 x 160 matrix runs on one core
    for minutes."""
    m, n = T.shape
    if m <= 8 * n:
        return np.linalg.qr(T, mode="r")
    import torch                       # CPU LAPACK only; no device is touched
    b = max(2 * n, (1 << 19) // n)
    nb = m // b
    head = np.ascontiguousarray(T[: nb * b]).reshape(nb, b, n)
    Rs = torch.linalg.qr(torch.from_numpy(head), mode="r")[1].numpy().reshape(nb * n, n)
    if nb * b < m:
        Rs = np.vstack([Rs, np.linalg.qr(T[nb * b:], mode="r")])
    return _r_factor(Rs)


def _svd_rows(M):
    """Singular values s and left singular vectors U (n x min(n, m)) of M (n x m)
    by LAPACK.  A strongly wide M goes through its R factor first (M^T = Q R,
    so M = R^T Q^T and the left singular vectors of M are the right singular
    vectors of the small triangle R: the R-SVD), which is exact up to rounding."""
    n, m = M.shape
    if m >= 4 * n:
        _, s, Vt = np.linalg.svd(_r_factor(M.T), full_matrices=False)
        return Vt.T, s
    U, s, _ = np.linalg.svd(M, full_matrices=False)
    return U, s


def tt_svd(a, dims, ranks=None, eps=None, sweep="L2R", weights=None, max_rank=None):
    """TT-SVD (Oseledets 2011): the same sweeps with the exact truncated SVD of
    every unfolding (LAPACK, through _svd_rows); the rank rule is the one after
    Alg. 2.  The core takes the r leading singular vectors on the core side of
    the unfolding and the carry is the unfolding projected onto them, which is
    the product of the r leading singular values and vectors on the other
    side."""
    dims = [int(x) for x in dims]
    d = len(dims)
    a = _as_flat(a, dims)
    normA = math.sqrt(float(a @ a))
    fixed, eps_k = _rank_targets(d, ranks, eps, normA, weights, False)
    rep = {"ranks": [1] * (d + 1), "delta": [], "normC": [], "ell": [], "s": [],
           "norm_A": normA, "rank_rule_met": True}
    cores = [None] * d
    C = a
    steps = range(1, d) if sweep == "L2R" else range(d, 1, -1)
    r_carry = 1
    for k in steps:
        if sweep == "L2R":
            n = r_carry * dims[k - 1]
            Cm = C.reshape(n, C.size // n, order="F")
            core_vecs, s = _svd_rows(Cm)
            target = fixed[k] if fixed else None
            ek = None if fixed else eps_k[k - 1]
        else:
            n = dims[k - 1] * r_carry
            Cm = C.reshape(C.size // n, n, order="F")
            core_vecs, s = _svd_rows(Cm.T)
            target = fixed[k - 1] if fixed else None
            ek = None if fixed else eps_k[k - 2]
        normC2 = float(C @ C)
        if target is not None:
            r = min(target, len(s))
        else:
            r, sat = _pick_rank(s, normC2, ek, max_rank)
            r = min(r, len(s))
            if not sat:
                rep["rank_rule_met"] = False
        sg = canonical_signs(core_vecs[:, :r])
        cv = core_vecs[:, :r] * sg[None, :]
        dk = math.sqrt(max(float(np.sum(s[r:] ** 2)), 0.0))
        if sweep == "L2R":
            cores[k - 1] = cv.reshape(r_carry, dims[k - 1], r, order="F")
            C = (cv.T @ Cm).reshape(-1, order="F")
            rep["ranks"][k] = r
            rep["delta"].append(dk); rep["normC"].append(math.sqrt(normC2)); rep["s"].append(s)
        else:
            cores[k - 1] = cv.T.reshape(r, dims[k - 1], r_carry, order="F")
            C = (Cm @ cv).reshape(-1, order="F")
            rep["ranks"][k - 1] = r
            rep["delta"].insert(0, dk); rep["normC"].insert(0, math.sqrt(normC2)); rep["s"].insert(0, s)
        r_carry = r
    if sweep == "L2R":
        cores[d - 1] = C.reshape(r_carry, dims[d - 1], 1, order="F")
    else:
        cores[0] = C.reshape(1, dims[0], r_carry, order="F")
    rep["err_bound"] = math.sqrt(float(np.sum(np.square(rep["delta"]))))
    return cores, rep


# --------------------------------------------------------------------------
# Reconstruction, sampling and the sampled-entry gradient (Eq. (TT))
# --------------------------------------------------------------------------
def tt_reconstruct(cores):
    """Full tensor (flat, i1 fastest) from TT cores, Eq. (TT): contract the
    train left to right, T <- reshape(T G_k) with the mode index of each new
    core landing after all previous ones."""
    T = cores[0].reshape(cores[0].shape[1], cores[0].shape[2], order="F")   # (I_1, r_1)
    for g in cores[1:]:
        rk_1, Ik, rk = g.shape
        T = T @ g.reshape(rk_1, Ik * rk, order="F")                        # (P, I_k r_k)
        T = T.reshape(-1, rk, order="F")                                    # (P I_k, r_k)
    return T.reshape(-1, order="F")


def _left_interface(cores, k):
    """Product of cores 1..k-1 (0-based: cores[:k]) as a (I_1..I_{k-1}) x r_{k-1}
    matrix, rows in ivec order; the 1 x 1 identity for k = 0."""
    T = np.ones((1, 1))
    for g in cores[:k]:
        rk_1, Ik, rk = g.shape
        T = (T @ g.reshape(rk_1, Ik * rk, order="F")).reshape(-1, rk, order="F")
    return T


def _right_interface(cores, k):
    """Product of cores k+1..d (0-based: cores[k+1:]) as an r_k x (I_{k+1}..I_d)
    matrix, columns in ivec order; the 1 x 1 identity for k = d-1."""
    T = np.ones((1, 1))
    for g in reversed(cores[k + 1:]):
        rk_1, Ik, rk = g.shape
        T = (g.reshape(rk_1 * Ik, rk, order="F") @ T).reshape(rk_1, -1, order="F")
    return T


def tt_reconstruct_grad(cores, gout):
    """Gradients of L = <gout, A_TT> (gout a dense tensor, flat in ivec order)
    with respect to every core, from Eq. (TT): A_TT(p, i, q) = sum_{a,b}
    Left_k(p, a) G_k(a, i, b) Right_k(b, q) with p the modes before k and q
    the modes after it, so dL/dG_k(a, i, b) = sum_{p,q} Left_k(p, a) gout(p, i, q)
    Right_k(b, q)."""
    gout = np.asarray(gout, dtype=np.float64).reshape(-1, order="F")
    grads = []
    for k, g in enumerate(cores):
        Lk = _left_interface(cores, k)                   # (P, r_{k-1})
        Rk = _right_interface(cores, k)                  # (r_k, Q)
        G3 = gout.reshape(Lk.shape[0], g.shape[1], Rk.shape[1], order="F")   # (P, I_k, Q)
        grads.append(np.einsum("pa,piq,bq->aib", Lk, G3, Rk, optimize=True))
    return grads


def tt_sample(cores, idx):
    """Entries A_TT[i_1..i_d] for each row of idx (N x d, 0-based), Eq. (TT):
    the product G_1[:, i_1, :] G_2[:, i_2, :] ... G_d[:, i_d, :]."""
    idx = np.asarray(idx, dtype=np.int64)
    v = cores[0][0, idx[:, 0], :]                                           # (N, r_1)
    for k in range(1, len(cores)):
        v = np.einsum("na,anb->nb", v, cores[k][:, idx[:, k], :])
    return v[:, 0]


def tt_sample_grad(cores, idx, w):
    """Gradients of L = sum_s w_s A_TT[idx_s] with respect to every core.

    dL/dG_k[a, i, b] = sum over samples s with i_k(s) = i of
    w_s * l_s[a] * r_s[b], where l_s = G_1[i_1]...G_{k-1}[i_{k-1}] and
    r_s = G_{k+1}[i_{k+1}]...G_d[i_d] (products of core slices)."""
    idx = np.asarray(idx, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    d = len(cores)
    N = idx.shape[0]
    left = [np.ones((N, 1))]
    for k in range(d - 1):
        left.append(np.einsum("na,anb->nb", left[-1], cores[k][:, idx[:, k], :]))
    right = [np.ones((N, 1))]
    for k in range(d - 1, 0, -1):
        right.append(np.einsum("anb,nb->na", cores[k][:, idx[:, k], :], right[-1]))
    right = right[::-1]                          # right[k] = product of cores k+1..d-1 (0-based)
    grads = []
    for k in range(d):
        g = np.zeros_like(cores[k])
        contrib = w[:, None, None] * left[k][:, :, None] * right[k][:, None, :]   # (N, r_{k-1}, r_k)
        np.add.at(g, (slice(None), idx[:, k], slice(None)), np.transpose(contrib, (1, 0, 2)))
        grads.append(g)
    return grads


# --------------------------------------------------------------------------
# Masked completion (the differentiation extension): gradient descent on the
# cores of f = 1/2 sum over observed entries (A_TT[idx_s] - m_s)^2.
def completion_step(cores, idx, vals):
    """One gradient step with the linearised exact step size: with residual
    e = A_TT[idx] - m and core gradients g, the sampled directional derivative
    J g = sum_k (train with core k replaced by g_k)[idx]; alpha minimises
    ||e - alpha J g||^2, i.e. alpha = <e, J g> / ||J g||^2.  Returns (new
    cores, f before the step, alpha)."""
    e = tt_sample(cores, idx) - np.asarray(vals, dtype=np.float64)
    f = 0.5 * float(e @ e)
    g = tt_sample_grad(cores, idx, e)
    jg = np.zeros_like(e)
    for k in range(len(cores)):
        jg += tt_sample(cores[:k] + [g[k]] + cores[k + 1:], idx)
    den = float(jg @ jg)
    alpha = float(e @ jg) / den if den > 0 else 0.0
    return [c - alpha * gk for c, gk in zip(cores, g)], f, alpha


# --------------------------------------------------------------------------
# Riemannian gradient descent for completion (Sec. 4.3, "MRI data
# completion"): the gradient of f on the manifold of trains of fixed ranks
# (the Euclidean gradient projected onto the tangent space at the current
# train), a step along it with the exact minimiser of f on that line, and a
# fixed-rank TT-UTV of the stepped tensor as the retraction.
def _left_unfold(g):
    r0, n, r1 = g.shape
    return g.reshape(r0 * n, r1, order="F")


def left_orthogonalize(cores):
    """The same train with cores 1..d-1 left-orthogonal (Def. 2.2): QR of
    each left unfolding, left to right, the triangular factor pushed into
    the next core.  Ranks must satisfy r_k <= r_{k-1} I_k."""
    out = [np.array(c, dtype=np.float64) for c in cores]
    for k in range(len(out) - 1):
        r0, n, r1 = out[k].shape
        assert r1 <= r0 * n, "rank above what the left unfolding allows"
        Q, R = np.linalg.qr(_left_unfold(out[k]))
        out[k] = Q.reshape(r0, n, r1, order="F")
        out[k + 1] = np.einsum("ab,bjc->ajc", R, out[k + 1])
    return out


def right_orthogonalize(cores):
    """The same train with cores 2..d right-orthogonal (Def. 2.2): QR of the
    transposed right unfoldings, right to left."""
    out = [np.array(c, dtype=np.float64) for c in cores]
    for k in range(len(out) - 1, 0, -1):
        r0, n, r1 = out[k].shape
        assert r0 <= n * r1, "rank above what the right unfolding allows"
        Q, R = np.linalg.qr(out[k].reshape(r0, n * r1, order="F").T)     # G^T = Q R, G = R^T Q^T
        out[k] = Q.T.reshape(r0, n, r1, order="F")
        out[k - 1] = np.einsum("ajb,cb->ajc", out[k - 1], R)
    return out


def tt_sample_grad_mixed(left_cores, right_cores, idx, w):
    """dL/dC_k of L = sum_s w_s (L_1..L_{k-1} C_k R_{k+1}..R_d)[idx_s] for every
    k: the gradient of the sampled entries at the mixed-canonical point k,
    with the left interface products from left_cores and the right ones
    from right_cores (two forms of one train)."""
    idx = np.asarray(idx, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    d = len(left_cores)
    N = idx.shape[0]
    left = [np.ones((N, 1))]
    for k in range(d - 1):
        left.append(np.einsum("na,anb->nb", left[-1], left_cores[k][:, idx[:, k], :]))
    right = [np.ones((N, 1))]
    for k in range(d - 1, 0, -1):
        right.append(np.einsum("anb,nb->na", right_cores[k][:, idx[:, k], :], right[-1]))
    right = right[::-1]
    grads = []
    for k in range(d):
        g = np.zeros_like(left_cores[k])
        contrib = w[:, None, None] * left[k][:, :, None] * right[k][:, None, :]
        np.add.at(g, (slice(None), idx[:, k], slice(None)), np.transpose(contrib, (1, 0, 2)))
        grads.append(g)
    return grads


def riemannian_gradient(cores, idx, z):
    """Projection onto the tangent space at the train X of the (sampled)
    Euclidean gradient Z = sum_s z_s e_{idx_s}.  With left- and
    right-orthogonal forms U, V of X, the tangent vector is
    xi = sum_k U_1..U_{k-1} dC_k V_{k+1}..V_d, where dC_k = (I - U_k U_k^T) G_k
    on the left unfoldings for k < d, dC_d = G_d, and G_k is the gradient of
    <Z, .> at the mixed-canonical point k.  Returns (U, V, dC)."""
    U = left_orthogonalize(cores)
    V = right_orthogonalize(cores)
    G = tt_sample_grad_mixed(U, V, idx, z)
    dC = []
    for k in range(len(cores) - 1):
        u, g = _left_unfold(U[k]), _left_unfold(G[k])
        dC.append((g - u @ (u.T @ g)).reshape(G[k].shape, order="F"))
    dC.append(G[-1])
    return U, V, dC


def tangent_train(U, V, dC, t=1.0, base=False):
    """Cores (interior ranks 2 r_k) of t*xi, or of X + t*xi with base=True,
    where xi = sum_k U_<k dC_k V_>k and X = U_1 ... U_d: first core
    [t dC_1, U_1], interior cores [[V_k, 0], [t dC_k, U_k]], last core
    [[V_d], [t dC_d (+ U_d)]]."""
    d = len(U)
    W = []
    for k in range(d):
        if k == 0:
            W.append(np.concatenate([t * dC[0], U[0]], axis=2))
        elif k < d - 1:
            r0, n, r1 = U[k].shape
            blk = np.zeros((2 * r0, n, 2 * r1))
            blk[:r0, :, :r1] = V[k]
            blk[r0:, :, :r1] = t * dC[k]
            blk[r0:, :, r1:] = U[k]
            W.append(blk)
        else:
            last = t * dC[k] + (U[k] if base else 0.0)
            W.append(np.concatenate([V[k], last], axis=0))
    return W


def rgrad_step(cores, idx, vals, ranks, q=1, p=8, seed=0):
    """One Riemannian gradient step for f = 1/2 sum_s (X[idx_s] - m_s)^2:
    z = X[idx] - m, xi = the Riemannian gradient, alpha = <P xi, z> / ||P xi||^2
    (P: sampling at idx) the exact minimiser of f(X - alpha xi), then the
    retraction: TT-ULV left to right at the fixed ranks of the full tensor
    X - alpha xi.  Returns (new cores, f before the step, alpha)."""
    z = tt_sample(cores, idx) - np.asarray(vals, dtype=np.float64)
    f = 0.5 * float(z @ z)
    U, V, dC = riemannian_gradient(cores, idx, z)
    pxi = tt_sample(tangent_train(U, V, dC), idx)
    den = float(pxi @ pxi)
    alpha = float(pxi @ z) / den if den > 0 else 0.0
    xhat = tt_reconstruct(tangent_train(U, V, dC, t=-alpha, base=True))
    dims = [int(c.shape[1]) for c in cores]
    new, _ = tt_utv(xhat, dims, ranks=list(ranks), sweep="L2R", variant="ULV", q=q, p=p, seed=seed)
    return new, f, alpha
