"""The completion-step entry points (Sec. 4.3) through the C ABI against the
FP64 oracle and NumPy: residual and objective, line step, axpy with a device
scalar, tangent projection of mixed-point core gradients, and the cores of a
tangent vector and of the stepped point."""
import numpy as np
import pytest
import torch

import oracle
import ttgen

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2501_07904_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(cores):
    return [c.detach().cpu().numpy() for c in cores]


@pytest.mark.parametrize("n", [0, 1, 255, 1000003])
def test_residual_and_line_step(n):
    rng = np.random.default_rng(n + 1)
    pred, vals, p = rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n)
    print(f"residual / line step, N = {n}", flush=True)
    z, f = T.tt_residual(_dev(pred), _dev(vals))
    z = z.cpu().numpy()
    assert np.array_equal(z, pred - vals)
    want = 0.5 * float(np.dot(pred - vals, pred - vals))
    assert abs(float(f[0]) - want) <= 1e-13 * max(want, 1e-300)
    st = T.tt_line_step(_dev(p), _dev(z)).cpu().numpy()
    pz, pp = float(np.dot(p, z)), float(np.dot(p, p))
    assert abs(st[1] - pz) <= 1e-12 * max(abs(pz), np.sqrt(pp * 2 * want), 1e-300)
    assert abs(st[2] - pp) <= 1e-13 * max(pp, 1e-300)
    if n:
        assert abs(st[0] - pz / pp) <= 1e-11 * abs(pz / pp) + 1e-15
    else:
        assert st[0] == 0.0
    # a zero direction gives a zero step, not a division by zero
    if n:
        st0 = T.tt_line_step(torch.zeros(n, dtype=torch.float64, device="cuda"), _dev(z)).cpu().numpy()
        assert st0[0] == 0.0 and st0[2] == 0.0
    # bitwise reproducible
    z2, f2 = T.tt_residual(_dev(pred), _dev(vals))
    assert float(f2[0]) == float(f[0])


def test_axpy_with_host_and_device_scalars():
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(70001), rng.standard_normal(70001)
    yd = _dev(y.copy())
    T.tt_axpy(yd, _dev(x), a=-0.5)
    np.testing.assert_allclose(yd.cpu().numpy(), y - 0.5 * x, rtol=1e-15, atol=1e-15)
    s = torch.tensor([3.0, 99.0], dtype=torch.float64, device="cuda")
    yd = _dev(y.copy())
    T.tt_axpy(yd, _dev(x), a=-2.0, a_dev=s)
    np.testing.assert_allclose(yd.cpu().numpy(), y - 6.0 * x, rtol=1e-15, atol=1e-14)


CASES = [
    ([7, 9, 5, 6], [1, 5, 13, 4, 1]),       # ragged ranks, one row tile per core
    ([3, 70, 64], [1, 3, 64, 1]),           # rank 64, 210-row left unfolding (ragged 32-row tiles)
    ([16, 16, 16, 16, 16, 10], [1, 16, 16, 16, 16, 10, 1]),   # the completion shape
    ([11, 13], [1, 6, 1]),                  # d = 2
]


@pytest.mark.parametrize("dims,ranks", CASES)
def test_tangent_projection_and_tangent_train(dims, ranks):
    print(f"tangent projection / train: dims {dims} ranks {ranks}", flush=True)
    cores = ttgen.gaussian_cores(dims, ranks, 21)
    rng = np.random.default_rng(22)
    n = 4000
    idx = np.stack([rng.integers(0, I, size=n) for I in dims], axis=1).astype(np.int64)
    z = rng.standard_normal(n)
    U, V, dC = oracle.riemannian_gradient(cores, idx, z)
    G = oracle.tt_sample_grad_mixed(U, V, idx, z)
    Ud, Vd, Gd = ([_dev(c) for c in cs] for cs in (U, V, G))
    got = _np(T.tt_tangent_project(Ud, Gd))
    for k, (x, y) in enumerate(zip(got, dC)):
        # relative to the gradient: a square left unfolding (r_{k-1} I_k = r_k, as core 1 of the
        # second case) has dC_k = 0 up to rounding
        err = np.max(np.abs(x - y)) / max(np.max(np.abs(G[k])), 1e-300)
        assert err <= 1e-12, (k, err)
    dCd = [_dev(c) for c in dC]

    def same(got, want):
        # t dC_d + U_d may be formed with one rounding (a fused multiply-add)
        for x, y in zip(got, want):
            assert x.shape == y.shape
            assert np.max(np.abs(x - y)) <= 2.3e-16 * max(np.max(np.abs(y)), 1e-300), np.max(np.abs(x - y))

    for t, base in ((1.0, False), (-0.37, True), (2.5, False)):
        same(_np(T.tt_tangent_train(Ud, Vd, dCd, t, base=base)), oracle.tangent_train(U, V, dC, t=t, base=base))
    # the scale taken from a device scalar
    tdev = torch.tensor([0.25], dtype=torch.float64, device="cuda")
    same(_np(T.tt_tangent_train(Ud, Vd, dCd, -2.0, t_dev=tdev, base=True)),
         oracle.tangent_train(U, V, dC, t=-0.5, base=True))
