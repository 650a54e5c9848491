"""The C ABI without a GPU: the library loads, exports every entry point the
header declares, and rejects bad arguments on the host before enqueuing work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ttutv.h")

T = pytest.importorskip("paper_2501_07904_amd")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(T.LIB_PATH):
        pytest.skip("libttutv.so not built")
    return T.load_library()


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(tt_\w+)\s*\(", text, re.M)))


def test_header_declares_the_binding_names():
    assert _declared() == sorted(T.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def _ws(lib, dims, ranks=None, eps=-1.0, sweep=0, variant=0, dtype=0, opts=None):
    d = len(dims)
    o = opts or T.make_opts()[0]
    n = ctypes.c_size_t(0)
    rk = None if ranks is None else T._i64(ranks)
    rc = lib.tt_utv_workspace(d, T._i64(dims), rk, eps, sweep, variant, dtype, ctypes.byref(o), ctypes.byref(n))
    return rc, n.value


def test_workspace_query_and_argument_errors(lib):
    rc, n = _ws(lib, [16] * 4, [1, 4, 6, 4, 1])
    assert rc == T.TT_OK and n > 0
    assert _ws(lib, [16], [1, 1])[0] == T.TT_EINVAL                      # d < 2
    assert _ws(lib, [16, 0, 4], [1, 2, 2, 1])[0] == T.TT_EINVAL          # zero extent
    assert _ws(lib, [16] * 4, [2, 4, 6, 4, 1])[0] == T.TT_EINVAL         # r_0 != 1
    assert _ws(lib, [16] * 4, [1, 0, 6, 4, 1])[0] == T.TT_EINVAL         # zero rank
    assert _ws(lib, [16] * 4, [1, 4, 6, 4, 1], sweep=7)[0] == T.TT_EINVAL
    assert _ws(lib, [16] * 4, [1, 4, 6, 4, 1], variant=9)[0] == T.TT_EINVAL
    assert _ws(lib, [16] * 4, None, eps=float("nan"))[0] == T.TT_EINVAL
    assert _ws(lib, [32] * 5, [1, 100, 100, 100, 100, 1])[0] == T.TT_EUNSUPPORTED   # ell > 64
    o, keep = T.make_opts(weights=[0.5, 0.5, 0.5])
    assert _ws(lib, [8] * 4, None, eps=1e-3, opts=o)[0] == T.TT_EINVAL  # sum w^2 != 1
    assert "weights" in lib.tt_last_error().decode()
    o, keep = T.make_opts(weights=[0.6, 0.8])
    assert _ws(lib, [8] * 3, None, eps=1e-3, opts=o)[0] == T.TT_OK


def test_workspace_grows_with_the_problem(lib):
    small = _ws(lib, [16] * 4, [1, 4, 6, 4, 1])[1]
    big = _ws(lib, [32] * 5, [1, 16, 16, 16, 16, 1], sweep=1, variant=1)[1]
    assert big > small
    # eps mode sizes for the rank caps
    assert _ws(lib, [8] * 8, None, eps=1e-6, sweep=1, variant=1, dtype=1)[1] >= _ws(lib, [8] * 8, [1] + [8] * 7 + [1], sweep=1, variant=1, dtype=1)[1]


def test_one_pass_option_on_host(lib):
    """fuse_ata: off by default, 0 or 1 only, and when on the workspace holds
    one n x ell partial per workgroup of the one-pass kernel (256 for the
    32768 x 512 unfolding of 32^5, ell = 24)."""
    o = T.make_opts()[0]
    assert o.fuse_ata == 0
    off = _ws(lib, [32] * 5, [1, 16, 16, 16, 16, 1], sweep=1, variant=1, opts=o)[1]
    o1 = T.make_opts(fuse_ata=True)[0]
    rc, on = _ws(lib, [32] * 5, [1, 16, 16, 16, 16, 1], sweep=1, variant=1, opts=o1)
    # the partials grow from the two-pass kernel's 128 row chunks to 256 workgroups
    assert rc == T.TT_OK and on - off == (256 - 128) * 512 * 24 * 8
    o1.fuse_ata = 2
    assert _ws(lib, [32] * 5, [1, 16, 16, 16, 16, 1], sweep=1, variant=1, opts=o1)[0] == T.TT_EINVAL
    assert "fuse_ata" in lib.tt_last_error().decode()
    names = [lib.tt_kernel_class_name(c).decode() for c in range(T.TT_NKCLASS)]
    assert names[7] == "tall_ata" and lib.tt_kernel_class_name(T.TT_NKCLASS) is None


def test_decompose_rejects_on_host(lib):
    d = 4
    dims = T._i64([16] * 4)
    rk = T._i64([1, 4, 6, 4, 1])
    o = T.make_opts()[0]
    fake = ctypes.c_void_p(0x1000)
    cores = (ctypes.c_void_p * d)(*([0x2000] * d))
    rep = T.tt_report()
    # NULL input
    rc = lib.tt_utv_decompose(None, 0, d, dims, rk, -1.0, 0, 0, ctypes.byref(o), fake, 1 << 30, cores,
                              ctypes.byref(rep), None)
    assert rc == T.TT_EINVAL
    # workspace too small: detected before any device work
    rc = lib.tt_utv_decompose(fake, 0, d, dims, rk, -1.0, 0, 0, ctypes.byref(o), fake, 16, cores,
                              ctypes.byref(rep), None)
    assert rc == T.TT_ENOSPC
    assert "workspace" in lib.tt_last_error().decode()
    # NULL core pointer
    bad = (ctypes.c_void_p * d)(0x2000, 0, 0x2000, 0x2000)
    rc = lib.tt_utv_decompose(fake, 0, d, dims, rk, -1.0, 0, 0, ctypes.byref(o), fake, 1 << 30, bad,
                              ctypes.byref(rep), None)
    assert rc == T.TT_EINVAL


def test_core_capacity(lib):
    cap = (ctypes.c_int64 * 4)()
    o = T.make_opts()[0]
    assert lib.tt_utv_core_capacity(4, T._i64([16] * 4), T._i64([1, 4, 6, 4, 1]), -1.0, ctypes.byref(o), cap) == 0
    assert list(cap) == [1 * 16 * 4, 4 * 16 * 6, 6 * 16 * 4, 4 * 16 * 1]
    # ranks above what an unfolding allows are clamped: 3 x 5 -> r_1 <= 3
    cap = (ctypes.c_int64 * 2)()
    assert lib.tt_utv_core_capacity(2, T._i64([3, 5]), T._i64([1, 9, 1]), -1.0, ctypes.byref(o), cap) == 0
    assert list(cap) == [1 * 3 * 3, 3 * 5 * 1]


def test_reconstruct_and_sample_argument_errors(lib):
    n = ctypes.c_size_t(0)
    assert lib.tt_reconstruct_workspace(3, T._i64([4, 5, 6]), T._i64([1, 2, 3, 1]), ctypes.byref(n)) == 0
    assert n.value > 0
    assert lib.tt_reconstruct_workspace(3, T._i64([4, 5, 6]), T._i64([2, 2, 3, 1]), ctypes.byref(n)) == T.TT_EINVAL
    assert lib.tt_reconstruct_workspace(3, T._i64([4, 5, 6]), T._i64([1, 65, 3, 1]), ctypes.byref(n)) == T.TT_EUNSUPPORTED
    cores = (ctypes.c_void_p * 2)(0x1000, 0x1000)
    assert lib.tt_sample(2, T._i64([3, 4]), T._i64([1, 2, 1]), cores, 0, None, -1, None, None) == T.TT_EINVAL
    assert lib.tt_sample(2, T._i64([3, 4]), T._i64([1, 2, 1]), cores, 0, None, 5, None, None) == T.TT_EINVAL
    assert lib.tt_sample(2, T._i64([3, 4]), T._i64([1, 2, 1]), cores, 7, None, 0, None, None) == T.TT_EINVAL
    # FP32 cores need every rank <= 32 (wider trains take the FP64-only kernels)
    assert lib.tt_sample(2, T._i64([40, 40]), T._i64([1, 40, 1]), cores, 1, None, 0, None, None) == T.TT_EUNSUPPORTED
    assert lib.tt_sample(2, T._i64([40, 40]), T._i64([1, 40, 1]), cores, 0, None, 0, None, None) == T.TT_OK


def test_sample_backward_workspace(lib):
    """Workspace of the sampled-entry backward: the interface products of at
    most 2^20 samples (sum_k r_{k-1} + r_k doubles each) plus 256 partial
    gradients; none for trains with a rank above 32."""
    n = ctypes.c_size_t(0)
    dims, ranks = [16, 16, 16, 16, 16, 10], [1, 16, 16, 16, 16, 10, 1]
    total = sum(ranks[k] * dims[k] * ranks[k + 1] for k in range(6))
    per = sum(ranks[k] + ranks[k + 1] for k in range(6))
    assert lib.tt_sample_backward_workspace(6, T._i64(dims), T._i64(ranks), 3145728, ctypes.byref(n)) == 0
    assert n.value == ((1 << 20) * per + 256 * total) * 8 + 256
    assert lib.tt_sample_backward_workspace(6, T._i64(dims), T._i64(ranks), 1000, ctypes.byref(n)) == 0
    assert n.value == (1000 * per + 256 * total) * 8 + 256
    assert lib.tt_sample_backward_workspace(2, T._i64([40, 40]), T._i64([1, 40, 1]), 10, ctypes.byref(n)) == 0
    assert n.value == 0
    assert lib.tt_sample_backward_workspace(2, T._i64([40, 40]), T._i64([1, 4, 1]), -1, ctypes.byref(n)) == T.TT_EINVAL
    # too small a workspace is refused before any device work
    cores = (ctypes.c_void_p * 2)(0x1000, 0x1000)
    g = (ctypes.c_void_p * 2)(0x2000, 0x2000)
    rc = lib.tt_sample_backward(2, T._i64([4, 4]), T._i64([1, 2, 1]), cores, 0, ctypes.c_void_p(0x3000), 10,
                                ctypes.c_void_p(0x4000), g, ctypes.c_void_p(0x5000), 16, None)
    assert rc == T.TT_ENOSPC and "workspace" in lib.tt_last_error().decode()


def test_binding_rejects_bad_indices_and_gradients():
    """The sampling bindings validate idx and gout before any pointer reaches
    a kernel (the kernels use the indices as addresses)."""
    import torch

    dims = [3, 4, 5]
    good = torch.tensor([[0, 0, 0], [2, 3, 4]], dtype=torch.int64)
    assert T.check_indices(good, dims).dtype == torch.int64
    assert T.check_indices(good.to(torch.int32), dims).dtype == torch.int64
    assert T.check_indices(torch.zeros((0, 3), dtype=torch.int64), dims).shape == (0, 3)
    with pytest.raises(ValueError, match="outside"):
        T.check_indices(torch.tensor([[0, 4, 0]]), dims)            # i_2 = I_2
    with pytest.raises(ValueError, match="outside"):
        T.check_indices(torch.tensor([[0, 0, -1]]), dims)           # negative
    with pytest.raises(ValueError, match="shape"):
        T.check_indices(torch.zeros((2, 2), dtype=torch.int64), dims)
    with pytest.raises(ValueError, match="shape"):
        T.check_indices(torch.zeros(6, dtype=torch.int64), dims)
    with pytest.raises(ValueError, match="integers"):
        T.check_indices(torch.zeros((2, 3)), dims)
    # a host tensor is refused where a device is required
    with pytest.raises(ValueError, match="tensor on"):
        T.check_indices(good, dims, torch.device("cuda", 0))
    # a passed check is remembered per version and dims: an in-place change or
    # other dims are checked again
    idx = torch.tensor([[0, 0, 0], [2, 3, 4]], dtype=torch.int64)
    assert T.check_indices(idx, dims) is idx
    assert T.check_indices(idx, dims) is idx
    with pytest.raises(ValueError, match="outside"):
        T.check_indices(idx, [3, 3, 5])
    idx[1, 2] = 5
    with pytest.raises(ValueError, match="outside"):
        T.check_indices(idx, dims)
    idx[1].fill_(-1)
    with pytest.raises(ValueError, match="outside"):
        T.check_indices(idx, dims)
    assert T.check_gout(torch.ones(2), 2).dtype == torch.float64
    with pytest.raises(ValueError, match="elements"):
        T.check_gout(torch.ones(3), 2)
    with pytest.raises(ValueError, match="tensor on"):
        T.check_gout(torch.ones(2), 2, torch.device("cuda", 0))


def test_binding_rejects_a_tensor_of_the_wrong_size():
    import torch

    with pytest.raises(ValueError, match="elements"):
        T._check_tensor_size(torch.zeros(10), [3, 4])
    T._check_tensor_size(torch.zeros(12), [3, 4])
    with pytest.raises(ValueError, match="device tensor"):
        T.tt_utv_decompose(torch.zeros(12, dtype=torch.float64), [3, 4], ranks=[2])


def test_noalloc_entry_rejects_on_host(lib):
    """tt_utv_decompose_noalloc refuses, before any device work, a problem
    whose workspace exceeds its static scratch, and profiling (HIP events)."""
    d = 5
    dims = T._i64([32] * 5)
    rk = T._i64([1, 16, 16, 16, 16, 1])
    o = T.make_opts()[0]
    fake = ctypes.c_void_p(0x1000)
    cores = (ctypes.c_void_p * d)(*([0x2000] * d))
    rep = T.tt_report()
    need = _ws(lib, [32] * 5, [1, 16, 16, 16, 16, 1], sweep=1, variant=1)[1]
    assert need > T.TT_NOALLOC_SCRATCH_BYTES
    rc = lib.tt_utv_decompose_noalloc(fake, 0, d, dims, rk, -1.0, 1, 1, ctypes.byref(o), cores, ctypes.byref(rep),
                                      None)
    assert rc == T.TT_ENOSPC
    msg = lib.tt_last_error().decode()
    assert "static scratch" in msg and str(need) in msg
    # a problem that fits, with profiling asked for
    small = _ws(lib, [16] * 4, [1, 4, 6, 4, 1])[1]
    assert small <= T.TT_NOALLOC_SCRATCH_BYTES
    o.profile = T.TT_PROFILE_ALL
    cores4 = (ctypes.c_void_p * 4)(*([0x2000] * 4))
    rc = lib.tt_utv_decompose_noalloc(fake, 0, 4, T._i64([16] * 4), T._i64([1, 4, 6, 4, 1]), -1.0, 0, 0,
                                      ctypes.byref(o), cores4, ctypes.byref(rep), None)
    assert rc == T.TT_EINVAL and "profile" in lib.tt_last_error().decode()
    # argument errors of the decomposition itself come first
    o.profile = 0
    rc = lib.tt_utv_decompose_noalloc(fake, 0, 4, T._i64([16] * 4), T._i64([2, 4, 6, 4, 1]), -1.0, 0, 0,
                                      ctypes.byref(o), cores4, ctypes.byref(rep), None)
    assert rc == T.TT_EINVAL


def test_orth_option_on_host(lib):
    """opts.orth: Householder by default, CholeskyQR3 on request (its Gram,
    factor and inverse take more workspace), other values refused."""
    o = T.make_opts()[0]
    assert o.orth == 0
    base = _ws(lib, [40, 40, 40], [1, 32, 32, 1], sweep=1, variant=1, opts=o)[1]
    o1 = T.make_opts(orth="cholqr")[0]
    rc, n1 = _ws(lib, [40, 40, 40], [1, 32, 32, 1], sweep=1, variant=1, opts=o1)
    assert rc == T.TT_OK and n1 >= base
    o1.orth = 5
    assert _ws(lib, [40, 40, 40], [1, 32, 32, 1], sweep=1, variant=1, opts=o1)[0] == T.TT_EINVAL
    assert "orth" in lib.tt_last_error().decode()


def test_completion_step_entry_points_reject_bad_arguments_on_the_host(lib):
    """tt_residual / tt_line_step / tt_axpy / tt_tangent_project /
    tt_tangent_train: argument errors are reported before any work is
    enqueued (the pointers below are never dereferenced)."""
    fake = ctypes.c_void_p(0x1000)
    W = T.TT_REDUCE_WORK_BYTES
    assert lib.tt_residual(-1, fake, fake, fake, fake, fake, W, None) == T.TT_EINVAL
    assert lib.tt_residual(10, fake, fake, fake, fake, fake, W - 8, None) == T.TT_ENOSPC
    assert lib.tt_residual(10, fake, fake, fake, fake, None, W, None) == T.TT_ENOSPC
    assert lib.tt_residual(10, None, fake, fake, fake, fake, W, None) == T.TT_EINVAL
    assert lib.tt_residual(10, fake, fake, fake, None, fake, W, None) == T.TT_EINVAL
    assert lib.tt_line_step(-1, fake, fake, fake, fake, W, None) == T.TT_EINVAL
    assert lib.tt_line_step(10, fake, fake, None, fake, W, None) == T.TT_EINVAL
    assert lib.tt_line_step(10, fake, None, fake, fake, W, None) == T.TT_EINVAL
    assert lib.tt_line_step(10, fake, fake, fake, fake, 16, None) == T.TT_ENOSPC
    assert lib.tt_axpy(-1, 1.0, None, fake, fake, None) == T.TT_EINVAL
    assert lib.tt_axpy(10, 1.0, None, None, fake, None) == T.TT_EINVAL
    vp3 = (ctypes.c_void_p * 3)(fake, fake, fake)
    nul3 = (ctypes.c_void_p * 3)(fake, None, fake)
    dims = T._i64([4, 5, 6])
    assert lib.tt_tangent_project(3, dims, T._i64([1, 2, 3, 1]), vp3, vp3, nul3, None) == T.TT_EINVAL
    assert lib.tt_tangent_project(3, dims, T._i64([2, 2, 3, 1]), vp3, vp3, vp3, None) == T.TT_EINVAL
    assert lib.tt_tangent_project(3, dims, T._i64([1, 65, 3, 1]), vp3, vp3, vp3, None) == T.TT_EUNSUPPORTED
    assert lib.tt_tangent_project(1, dims, T._i64([1, 1]), vp3, vp3, vp3, None) == T.TT_EINVAL
    assert lib.tt_tangent_train(3, dims, T._i64([1, 2, 3, 1]), vp3, vp3, None, 1.0, None, 0, vp3,
                                None) == T.TT_EINVAL
    assert lib.tt_tangent_train(3, dims, T._i64([1, 2, 3, 1]), vp3, nul3, vp3, 1.0, None, 0, vp3,
                                None) == T.TT_EINVAL
    assert lib.tt_tangent_train(3, dims, T._i64([1, 2, 3, 2]), vp3, vp3, vp3, 1.0, None, 1, vp3,
                                None) == T.TT_EINVAL


def test_deflation_option_on_host(lib):
    """opts.inner: the sketch by default; the deflation inner kernel on request
    for the sweeps that keep the core side orthonormal, FP64 form, q >= 1, and
    core sides up to 4096 outside Gram mode; everything else refused."""
    o = T.make_opts()[0]
    assert o.inner == 0
    od = T.make_opts(inner="deflation")[0]
    assert od.inner == 1
    for sweep, variant in ((0, 0), (1, 1), (0, 1)):
        rc, nb = _ws(lib, [40, 40, 40], [1, 32, 32, 1], sweep=sweep, variant=variant, opts=od)
        assert rc == T.TT_OK and nb > 0, (sweep, variant, lib.tt_last_error())
    # Alg. 4 and TT-SVD
    for variant in (0, 2):
        rc, _ = _ws(lib, [40, 40, 40], [1, 32, 32, 1], sweep=1, variant=variant, opts=od)
        assert rc == T.TT_EINVAL and "deflation" in lib.tt_last_error().decode()
    od0 = T.make_opts(inner="deflation", q=0)[0]
    assert _ws(lib, [40, 40, 40], [1, 32, 32, 1], sweep=1, variant=1, opts=od0)[0] == T.TT_EINVAL
    assert "q >= 1" in lib.tt_last_error().decode()
    odm = T.make_opts(inner="deflation", prec="mixed")[0]
    assert _ws(lib, [40, 40, 40], [1, 32, 32, 1], sweep=1, variant=1, opts=odm)[0] == T.TT_EINVAL
    # a core side of 80 x 64 = 5120 > 4096 outside Gram mode
    rc, _ = _ws(lib, [80, 80, 80], [1, 64, 64, 1], sweep=1, variant=1, opts=od)
    assert rc == T.TT_EUNSUPPORTED and "4096" in lib.tt_last_error().decode()
    od.inner = 7
    assert _ws(lib, [40, 40, 40], [1, 32, 32, 1], sweep=1, variant=1, opts=od)[0] == T.TT_EINVAL
    assert "inner" in lib.tt_last_error().decode()
    assert lib.tt_kernel_class_name(8).decode() == "defl_pass"
    assert lib.tt_kernel_class_name(T.TT_NKCLASS) is None


def test_ttsvd_core_side_beyond_64_on_host(lib):
    """TT-SVD on core sides above 64 (subspace iteration on the leading 64
    directions): accepted up to rank 64, refused above (TT_EUNSUPPORTED)."""
    rc, nb = _ws(lib, [32] * 5, [1, 16, 16, 16, 16, 1], sweep=1, variant=2)
    assert rc == T.TT_OK and nb > 0
    rc, _ = _ws(lib, [32] * 5, [1, 16, 16, 16, 16, 1], sweep=0, variant=2)
    assert rc == T.TT_OK
    rc, _ = _ws(lib, [32] * 5, [1, 70, 70, 70, 70, 1], sweep=1, variant=2)
    assert rc == T.TT_EUNSUPPORTED and "rank" in lib.tt_last_error().decode()


def test_noalloc_without_report_needs_fixed_ranks():
    """The enqueue-only form (no report) exists for fixed ranks alone: a
    prescribed accuracy reads every step's rank back to the host."""
    with pytest.raises(ValueError, match="report=False needs fixed ranks"):
        T.tt_utv_decompose_noalloc(None, [2, 2], [], eps=0.1, report=False)
