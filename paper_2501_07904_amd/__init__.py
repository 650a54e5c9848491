"""TT-UTV on AMD MI355X: thin Python binding of libttutv.so.

Only argument marshalling happens here: every step of the decomposition,
reconstruction, sampling and sampled-entry backward runs in the HIP kernels
of libttutv.so.  PyTorch provides device memory and the current stream.  The
library must be built first (python -m paper_2501_07904_amd.build); importing
the binding without it raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libttutv.so")

TT_OK, TT_EINVAL, TT_ENOSPC, TT_ERANK, TT_ENONFINITE, TT_EHIP, TT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
TT_MAX_D = 32
TT_MAX_ELL = 64
TT_NOALLOC_SCRATCH_BYTES = 64 << 20
TT_REDUCE_WORK_BYTES = 4096
SWEEPS = {"L2R": 0, "R2L": 1}
VARIANTS = {"ULV": 0, "URV": 1, "SVD": 2}
DTYPES = {torch.float64: 0, torch.float32: 1}
EXPORTS = ["tt_default_opts", "tt_utv_workspace", "tt_utv_core_capacity", "tt_utv_decompose",
           "tt_utv_decompose_noalloc",
           "tt_reconstruct_workspace", "tt_reconstruct", "tt_reconstruct_backward_workspace",
           "tt_reconstruct_backward", "tt_sample", "tt_sample_backward_workspace", "tt_sample_backward",
           "tt_sample_backward_mixed", "tt_residual", "tt_line_step", "tt_axpy", "tt_tangent_project",
           "tt_tangent_train",
           "tt_last_error", "tt_kernel_class_name"]


class TTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libttutv error {code}: {msg}")
        self.code = code


class tt_opts(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("oversample", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("max_rank", ctypes.c_int32), ("exact_delta", ctypes.c_int32),
                ("weights", ctypes.POINTER(ctypes.c_double)), ("profile", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("fuse_ata", ctypes.c_int32), ("orth", ctypes.c_int32),
                ("separate_sketch", ctypes.c_int32), ("inner", ctypes.c_int32)]


TT_NKCLASS = 9
TT_PROFILE_ALL = (1 << TT_NKCLASS) - 1


class tt_kstat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("flops", ctypes.c_double)]


class tt_report(ctypes.Structure):
    _fields_ = [("ranks", ctypes.c_int64 * (TT_MAX_D + 1)), ("ell", ctypes.c_int64 * TT_MAX_D),
                ("delta", ctypes.c_double * TT_MAX_D), ("normC", ctypes.c_double * TT_MAX_D),
                ("norm_A", ctypes.c_double), ("err_bound", ctypes.c_double),
                ("rank_rule_met", ctypes.c_int32), ("d", ctypes.c_int32),
                ("kstat", tt_kstat * TT_NKCLASS), ("sweeps", ctypes.c_int32 * TT_MAX_D),
                ("rho", ctypes.c_double * TT_MAX_D), ("err_bound_measured", ctypes.c_int32)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libttutv.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2501_07904_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64p, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
    lib.tt_default_opts.argtypes = [ctypes.POINTER(tt_opts)]
    lib.tt_default_opts.restype = None
    lib.tt_last_error.restype = ctypes.c_char_p
    lib.tt_kernel_class_name.argtypes = [ctypes.c_int]
    lib.tt_kernel_class_name.restype = ctypes.c_char_p
    lib.tt_utv_workspace.argtypes = [ctypes.c_int, i64p, i64p, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.POINTER(tt_opts), ctypes.POINTER(ctypes.c_size_t)]
    lib.tt_utv_core_capacity.argtypes = [ctypes.c_int, i64p, i64p, ctypes.c_double, ctypes.POINTER(tt_opts), i64p]
    lib.tt_utv_decompose.argtypes = [vp, ctypes.c_int, ctypes.c_int, i64p, i64p, ctypes.c_double, ctypes.c_int,
                                     ctypes.c_int, ctypes.POINTER(tt_opts), vp, ctypes.c_size_t,
                                     ctypes.POINTER(vp), ctypes.POINTER(tt_report), vp]
    lib.tt_utv_decompose_noalloc.argtypes = [vp, ctypes.c_int, ctypes.c_int, i64p, i64p, ctypes.c_double,
                                             ctypes.c_int, ctypes.c_int, ctypes.POINTER(tt_opts), ctypes.POINTER(vp),
                                             ctypes.POINTER(tt_report), vp]
    lib.tt_reconstruct_workspace.argtypes = [ctypes.c_int, i64p, i64p, ctypes.POINTER(ctypes.c_size_t)]
    lib.tt_reconstruct.argtypes = [ctypes.c_int, i64p, i64p, ctypes.POINTER(vp), vp, ctypes.c_int, vp,
                                   ctypes.c_size_t, vp]
    lib.tt_reconstruct_backward_workspace.argtypes = [ctypes.c_int, i64p, i64p, ctypes.POINTER(ctypes.c_size_t)]
    lib.tt_reconstruct_backward.argtypes = [ctypes.c_int, i64p, i64p, ctypes.POINTER(vp), vp, ctypes.c_int,
                                            ctypes.POINTER(vp), vp, ctypes.c_size_t, vp]
    lib.tt_sample.argtypes = [ctypes.c_int, i64p, i64p, ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.c_int64, vp,
                              vp]
    lib.tt_sample_backward_workspace.argtypes = [ctypes.c_int, i64p, i64p, ctypes.c_int64,
                                                 ctypes.POINTER(ctypes.c_size_t)]
    lib.tt_sample_backward.argtypes = [ctypes.c_int, i64p, i64p, ctypes.POINTER(vp), ctypes.c_int, vp,
                                       ctypes.c_int64, vp, ctypes.POINTER(vp), vp, ctypes.c_size_t, vp]
    lib.tt_sample_backward_mixed.argtypes = [ctypes.c_int, i64p, i64p, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                             ctypes.c_int, vp, ctypes.c_int64, vp, ctypes.POINTER(vp), vp,
                                             ctypes.c_size_t, vp]
    lib.tt_residual.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.tt_line_step.argtypes = [ctypes.c_int64, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.tt_axpy.argtypes = [ctypes.c_int64, ctypes.c_double, vp, vp, vp, vp]
    lib.tt_tangent_project.argtypes = [ctypes.c_int, i64p, i64p, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                       ctypes.POINTER(vp), vp]
    lib.tt_tangent_train.argtypes = [ctypes.c_int, i64p, i64p, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                     ctypes.POINTER(vp), ctypes.c_double, vp, ctypes.c_int, ctypes.POINTER(vp), vp]
    for name in ("tt_utv_workspace", "tt_utv_core_capacity", "tt_utv_decompose", "tt_utv_decompose_noalloc",
                 "tt_reconstruct_workspace",
                 "tt_reconstruct", "tt_reconstruct_backward_workspace", "tt_reconstruct_backward", "tt_sample",
                 "tt_sample_backward_workspace", "tt_sample_backward", "tt_sample_backward_mixed", "tt_residual",
                 "tt_line_step", "tt_axpy", "tt_tangent_project", "tt_tangent_train"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc, allow=()):
    if rc != TT_OK and rc not in allow:
        raise TTError(rc, load_library().tt_last_error().decode())
    return rc


def _i64(vals):
    arr = (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])
    return arr


def _ptrs(tensors):
    return (ctypes.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _numel(dims):
    n = 1
    for x in dims:
        n *= int(x)
    return n


def _check_tensor_size(A, dims):
    if A.numel() != _numel(dims):
        raise ValueError(f"A has {A.numel()} elements, dims {list(dims)} need {_numel(dims)}")


def check_indices(idx, dims, device=None):
    """Validate sampling indices before they reach a kernel: an (N, d) int64
    tensor with 0 <= idx[:, k] < dims[k] (one min/max reduction per mode; the
    kernels use the indices as addresses), on `device` when given.  Returns
    the contiguous int64 tensor.  A tensor that passed is marked with its
    version counter and the dims, so the reductions are not repeated for the
    same unchanged indices (a completion loop samples the same mask every
    step); any in-place change bumps the version and forces a new check."""
    d = len(dims)
    if device is not None and (not idx.is_cuda or idx.device != device):
        raise ValueError(f"idx must be a tensor on {device}, got {idx.device}")
    if idx.dim() != 2 or idx.shape[1] != d:
        raise ValueError(f"idx must have shape (N, {d}), got {tuple(idx.shape)}")
    if idx.dtype.is_floating_point or idx.dtype.is_complex or idx.dtype == torch.bool:
        raise ValueError(f"idx must hold integers, got {idx.dtype}")
    idx = idx.contiguous().to(torch.int64)
    key = (idx._version, tuple(int(x) for x in dims))
    if getattr(idx, "_ttutv_checked", None) == key:
        return idx
    if idx.shape[0] > 0:
        lo = idx.amin(dim=0).tolist()
        hi = idx.amax(dim=0).tolist()
        for k in range(d):
            if lo[k] < 0 or hi[k] >= dims[k]:
                raise ValueError(f"idx[:, {k}] spans [{lo[k]}, {hi[k]}], outside [0, {dims[k] - 1}]")
    idx._ttutv_checked = key
    return idx


def check_gout(gout, n, device=None):
    """Validate the upstream gradient of N sampled entries (N values on `device`)."""
    if device is not None and (not gout.is_cuda or gout.device != device):
        raise ValueError(f"gout must be a tensor on {device}, got {gout.device}")
    if gout.numel() != n:
        raise ValueError(f"gout has {gout.numel()} elements for {n} sampled entries")
    return gout.contiguous().reshape(-1).to(torch.float64)


def _full_ranks(ranks, d):
    r = [int(x) for x in ranks]
    if len(r) == d - 1:
        r = [1] + r + [1]
    if len(r) != d + 1:
        raise ValueError("ranks must be r_0..r_d or r_1..r_{d-1}")
    return r


PRECS = {"fp64": 0, "mixed": 1, "mixed_bf16": 2}
ORTHS = {"householder": 0, "cholqr": 1}
INNERS = {"sketch": 0, "deflation": 1}


def make_opts(q=1, oversample=8, seed=0, max_rank=0, exact_delta=False, weights=None, profile=False,
              prec="fp64", fuse_ata=False, orth="householder", separate_sketch=False, inner="sketch"):
    o = tt_opts()
    load_library().tt_default_opts(ctypes.byref(o))
    o.q, o.oversample, o.seed, o.max_rank, o.exact_delta = q, oversample, seed, max_rank, int(bool(exact_delta))
    # profile: False/0 = off, True = every kernel class, an int = bit mask of classes
    o.profile = TT_PROFILE_ALL if profile is True else int(profile)
    o.prec = PRECS[prec]
    o.fuse_ata = int(bool(fuse_ata))
    o.orth = ORTHS[orth]
    o.separate_sketch = int(bool(separate_sketch))
    o.inner = INNERS[inner]
    keep = None
    if weights is not None:
        keep = (ctypes.c_double * len(weights))(*[float(w) for w in weights])
        o.weights = ctypes.cast(keep, ctypes.POINTER(ctypes.c_double))
    return o, keep


def _core_view(flat, r0, I, r1):
    """Logical (r_{k-1}, I_k, r_k) view of a column-major core buffer."""
    return flat[: r0 * I * r1].view(r1, I, r0).permute(2, 1, 0)


def tt_utv_workspace(dims, ranks=None, eps=None, sweep="L2R", variant="ULV", dtype=torch.float64, **kw):
    lib = load_library()
    d = len(dims)
    o, _keep = make_opts(**kw)
    nbytes = ctypes.c_size_t(0)
    rk = None if ranks is None else _i64(_full_ranks(ranks, d))
    _check(lib.tt_utv_workspace(d, _i64(dims), rk, -1.0 if eps is None else float(eps), SWEEPS[sweep],
                                VARIANTS[variant], DTYPES[dtype], ctypes.byref(o), ctypes.byref(nbytes)))
    return nbytes.value


def _decompose_args(A, dims, ranks, eps, q, oversample, seed, max_rank, exact_delta, weights, profile, prec,
                    fuse_ata, orth="householder", separate_sketch=False, inner="sketch"):
    if not (A.is_cuda and A.is_contiguous()):
        raise ValueError("A must be a contiguous device tensor")
    if A.dtype not in DTYPES:
        raise ValueError("A must be float64 or float32")
    dims = [int(x) for x in dims]
    _check_tensor_size(A, dims)
    if (ranks is None) == (eps is None):
        raise ValueError("give exactly one of ranks and eps")
    o, keep = make_opts(q, oversample, seed, max_rank, exact_delta, weights, profile, prec, fuse_ata, orth,
                        separate_sketch, inner)
    rk = None if ranks is None else _i64(_full_ranks(ranks, len(dims)))
    epsv = -1.0 if eps is None else float(eps)
    return dims, o, keep, rk, epsv


def _report_dict(lib, rep, d, rc, profile):
    report = {
        "ranks": [int(rep.ranks[k]) for k in range(d + 1)], "ell": [int(rep.ell[k]) for k in range(d - 1)],
        "delta": [float(rep.delta[k]) for k in range(d - 1)],
        "normC": [float(rep.normC[k]) for k in range(d - 1)],
        "norm_A": float(rep.norm_A), "err_bound": float(rep.err_bound),
        "rank_rule_met": bool(rep.rank_rule_met), "status": rc,
        "sweeps": [int(rep.sweeps[k]) for k in range(d - 1)],
        "rho": [float(rep.rho[k]) for k in range(d - 1)],
        "err_bound_measured": bool(rep.err_bound_measured),
    }
    if profile:
        report["kstat"] = {lib.tt_kernel_class_name(c).decode(): {
            "launches": int(rep.kstat[c].launches), "ms": float(rep.kstat[c].ms),
            "bytes": float(rep.kstat[c].bytes), "flops": float(rep.kstat[c].flops)} for c in range(TT_NKCLASS)}
    return report


def core_buffers_for(dims, ranks=None, eps=None, q=1, oversample=8, max_rank=0, device="cuda"):
    """Flat float64 device buffers large enough for every core the problem can
    produce (tt_utv_core_capacity), for callers that allocate them up front."""
    lib = load_library()
    dims = [int(x) for x in dims]
    d = len(dims)
    o, _keep = make_opts(q, oversample, 0, max_rank)
    rk = None if ranks is None else _i64(_full_ranks(ranks, d))
    cap = (ctypes.c_int64 * d)()
    _check(lib.tt_utv_core_capacity(d, _i64(dims), rk, -1.0 if eps is None else float(eps), ctypes.byref(o), cap))
    return [torch.empty(max(int(c), 1), dtype=torch.float64, device=device) for c in cap]


def tt_utv_decompose(A, dims, ranks=None, eps=None, sweep="L2R", variant="ULV", q=1, oversample=8, seed=0,
                     max_rank=0, exact_delta=False, weights=None, work=None, stream=None, allow_rank_miss=False,
                     profile=False, prec="fp64", fuse_ata=False, orth="householder", separate_sketch=False,
                     inner="sketch"):
    """TT-UTV of the device tensor A (float64/float32, flat in ivec order, i1
    fastest).  Returns (cores, report); cores[k] is a (r_{k-1}, I_k, r_k)
    float64 view of a column-major device buffer."""
    lib = load_library()
    dims, o, _keep, rk, epsv = _decompose_args(A, dims, ranks, eps, q, oversample, seed, max_rank, exact_delta,
                                               weights, profile, prec, fuse_ata, orth, separate_sketch, inner)
    d = len(dims)
    nbytes = ctypes.c_size_t(0)
    _check(lib.tt_utv_workspace(d, _i64(dims), rk, epsv, SWEEPS[sweep], VARIANTS[variant], DTYPES[A.dtype],
                                ctypes.byref(o), ctypes.byref(nbytes)))
    if work is None or work.numel() < nbytes.value:
        work = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=A.device)
    cap = (ctypes.c_int64 * d)()
    _check(lib.tt_utv_core_capacity(d, _i64(dims), rk, epsv, ctypes.byref(o), cap))
    flats = [torch.empty(max(int(c), 1), dtype=torch.float64, device=A.device) for c in cap]
    rep = tt_report()
    rc = lib.tt_utv_decompose(ctypes.c_void_p(A.data_ptr()), DTYPES[A.dtype], d, _i64(dims), rk, epsv,
                              SWEEPS[sweep], VARIANTS[variant], ctypes.byref(o), ctypes.c_void_p(work.data_ptr()),
                              nbytes.value, _ptrs(flats), ctypes.byref(rep), _stream(stream))
    _check(rc, allow=(TT_ERANK,) if allow_rank_miss else ())
    r = [int(rep.ranks[k]) for k in range(d + 1)]
    cores = [_core_view(flats[k], r[k], dims[k], r[k + 1]) for k in range(d)]
    return cores, _report_dict(lib, rep, d, rc, profile)


def tt_utv_decompose_noalloc(A, dims, core_flats, ranks=None, eps=None, sweep="L2R", variant="ULV", q=1,
                             oversample=8, seed=0, max_rank=0, exact_delta=False, weights=None, stream=None,
                             allow_rank_miss=False, prec="fp64", fuse_ata=False, orth="householder",
                             separate_sketch=False, inner="sketch", report=True):
    """tt_utv_decompose on the library's static device scratch (no workspace
    argument): for problems whose workspace fits TT_NOALLOC_SCRATCH_BYTES.
    core_flats: caller-allocated flat float64 device buffers, one per core, at
    least tt_utv_core_capacity long (core_buffers_for); the call allocates no
    device memory.  Returns (cores, report) with cores viewing core_flats.
    report=False (fixed ranks only) passes no report: the call then only
    enqueues kernels and never waits on the stream, so it can be recorded into
    a graph (after a first call on the device), and returns (cores, None), the
    ranks taken from the host-side capacity query."""
    lib = load_library()
    if not report and ranks is None:
        raise ValueError("report=False needs fixed ranks (a prescribed accuracy reads each step's rank back)")
    dims, o, _keep, rk, epsv = _decompose_args(A, dims, ranks, eps, q, oversample, seed, max_rank, exact_delta,
                                               weights, False, prec, fuse_ata, orth, separate_sketch, inner)
    d = len(dims)
    if len(core_flats) != d:
        raise ValueError(f"need {d} core buffers, got {len(core_flats)}")
    cap = (ctypes.c_int64 * d)()
    _check(lib.tt_utv_core_capacity(d, _i64(dims), rk, epsv, ctypes.byref(o), cap))
    for k, f in enumerate(core_flats):
        if not (f.is_cuda and f.dtype == torch.float64 and f.is_contiguous()) or f.numel() < int(cap[k]):
            raise ValueError(f"core buffer {k} must be a contiguous float64 device tensor of >= {int(cap[k])} entries")
    rep = tt_report() if report else None
    rc = lib.tt_utv_decompose_noalloc(ctypes.c_void_p(A.data_ptr()), DTYPES[A.dtype], d, _i64(dims), rk, epsv,
                                      SWEEPS[sweep], VARIANTS[variant], ctypes.byref(o), _ptrs(core_flats),
                                      ctypes.byref(rep) if report else None, _stream(stream))
    _check(rc, allow=(TT_ERANK,) if allow_rank_miss else ())
    if report:
        r = [int(rep.ranks[k]) for k in range(d + 1)]
    else:
        # with fixed ranks the capacity of core k is exactly r_{k-1} I_k r_k
        r = [1]
        for k in range(d):
            r.append(int(cap[k]) // (r[k] * dims[k]))
    cores = [_core_view(core_flats[k], r[k], dims[k], r[k + 1]) for k in range(d)]
    return cores, (_report_dict(lib, rep, d, rc, False) if report else None)


def _core_buffers(cores):
    """Column-major flat buffers of logical (r0, I, r1) cores."""
    out = []
    for g in cores:
        flat = g.permute(2, 1, 0).contiguous().reshape(-1)
        out.append(flat if flat.dtype == torch.float64 else flat.double())
    return out


def _train_shape(cores):
    dims = [int(g.shape[1]) for g in cores]
    ranks = [int(cores[0].shape[0])] + [int(g.shape[2]) for g in cores]
    return dims, ranks


def tt_reconstruct(cores, dtype=torch.float64, stream=None):
    """Dense tensor (flat, ivec order) of a train of (r0, I, r1) device cores."""
    lib = load_library()
    dims, ranks = _train_shape(cores)
    d = len(dims)
    bufs = _core_buffers(cores)
    nbytes = ctypes.c_size_t(0)
    _check(lib.tt_reconstruct_workspace(d, _i64(dims), _i64(ranks), ctypes.byref(nbytes)))
    dev = cores[0].device
    work = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=dev)
    total = 1
    for I in dims:
        total *= I
    out = torch.empty(total, dtype=dtype, device=dev)
    _check(lib.tt_reconstruct(d, _i64(dims), _i64(ranks), _ptrs(bufs), ctypes.c_void_p(out.data_ptr()),
                              DTYPES[dtype], ctypes.c_void_p(work.data_ptr()), nbytes.value, _stream(stream)))
    return out


def tt_reconstruct_backward(cores, gout, stream=None):
    """Core gradients of <gout, A_TT> for a dense upstream gradient gout (flat,
    ivec order, float64 or float32, on the device); list of (r0, I, r1)
    float64 tensors."""
    lib = load_library()
    dims, ranks = _train_shape(cores)
    d = len(dims)
    dev = cores[0].device
    if not gout.is_cuda or gout.device != dev:
        raise ValueError(f"gout must be a tensor on {dev}, got {gout.device}")
    if gout.dtype not in DTYPES:
        raise ValueError("gout must be float64 or float32")
    if gout.numel() != _numel(dims):
        raise ValueError(f"gout has {gout.numel()} elements, the train has {_numel(dims)}")
    gout = gout.contiguous()
    bufs = _core_buffers(cores)
    nbytes = ctypes.c_size_t(0)
    _check(lib.tt_reconstruct_backward_workspace(d, _i64(dims), _i64(ranks), ctypes.byref(nbytes)))
    work = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=dev)
    gflat = [torch.empty_like(b) for b in bufs]
    _check(lib.tt_reconstruct_backward(d, _i64(dims), _i64(ranks), _ptrs(bufs), ctypes.c_void_p(gout.data_ptr()),
                                       DTYPES[gout.dtype], _ptrs(gflat), ctypes.c_void_p(work.data_ptr()),
                                       nbytes.value, _stream(stream)))
    return [_core_view(gflat[k], ranks[k], dims[k], ranks[k + 1]) for k in range(d)]


def _sample_buffers(cores):
    """Column-major flat buffers of the cores for the sampling kernels: FP32
    when every core is float32 (the kernels take FP32 cores as they are),
    else FP64.  Returns (buffers, dtype code)."""
    if all(g.dtype == torch.float32 for g in cores):
        return [g.permute(2, 1, 0).contiguous().reshape(-1) for g in cores], DTYPES[torch.float32]
    return _core_buffers(cores), DTYPES[torch.float64]


def tt_sample(cores, idx, stream=None):
    """Train entries at the rows of idx (N x d int64, 0-based, on the device);
    float64 results for float64 or float32 cores."""
    lib = load_library()
    dims, ranks = _train_shape(cores)
    idx = check_indices(idx, dims, cores[0].device)
    N = idx.shape[0]
    bufs, dt = _sample_buffers(cores)
    out = torch.empty(N, dtype=torch.float64, device=cores[0].device)
    _check(lib.tt_sample(len(dims), _i64(dims), _i64(ranks), _ptrs(bufs), dt, ctypes.c_void_p(idx.data_ptr()), N,
                         ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def _sample_work(dims, ranks, N, device):
    lib = load_library()
    nbytes = ctypes.c_size_t(0)
    _check(lib.tt_sample_backward_workspace(len(dims), _i64(dims), _i64(ranks), N, ctypes.byref(nbytes)))
    return torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=device), nbytes.value


def tt_sample_backward(cores, idx, gout, stream=None):
    """Core gradients of sum_s gout[s] * A_TT[idx_s]; list of (r0, I, r1)
    tensors in the cores' precision (float32 for float32 cores)."""
    lib = load_library()
    dims, ranks = _train_shape(cores)
    idx = check_indices(idx, dims, cores[0].device)
    N = idx.shape[0]
    gout = check_gout(gout, N, cores[0].device)
    bufs, dt = _sample_buffers(cores)
    gflat = [torch.empty_like(b) for b in bufs]
    work, nbytes = _sample_work(dims, ranks, N, cores[0].device)
    _check(lib.tt_sample_backward(len(dims), _i64(dims), _i64(ranks), _ptrs(bufs), dt,
                                  ctypes.c_void_p(idx.data_ptr()), N, ctypes.c_void_p(gout.data_ptr()), _ptrs(gflat),
                                  ctypes.c_void_p(work.data_ptr()), nbytes, _stream(stream)))
    return [_core_view(gflat[k], ranks[k], dims[k], ranks[k + 1]) for k in range(len(dims))]


def tt_sample_backward_mixed(left_cores, right_cores, idx, gout, stream=None):
    """Core gradients of sum_s gout[s] * A_TT[idx_s] at the mixed-canonical
    points: the interfaces left of core k from left_cores, right of it from
    right_cores (two forms of one train with equal ranks)."""
    lib = load_library()
    dims, ranks = _train_shape(left_cores)
    if _train_shape(right_cores) != (dims, ranks):
        raise ValueError("left and right cores must describe trains of the same shape and ranks")
    idx = check_indices(idx, dims, left_cores[0].device)
    N = idx.shape[0]
    gout = check_gout(gout, N, left_cores[0].device)
    lb, dl = _sample_buffers(left_cores)
    rb, dr = _sample_buffers(right_cores)
    if dl != dr:
        lb, rb, dl = _core_buffers(left_cores), _core_buffers(right_cores), DTYPES[torch.float64]
    gflat = [torch.empty_like(b) for b in lb]
    work, nbytes = _sample_work(dims, ranks, N, left_cores[0].device)
    _check(lib.tt_sample_backward_mixed(len(dims), _i64(dims), _i64(ranks), _ptrs(lb), _ptrs(rb), dl,
                                        ctypes.c_void_p(idx.data_ptr()), N, ctypes.c_void_p(gout.data_ptr()),
                                        _ptrs(gflat), ctypes.c_void_p(work.data_ptr()), nbytes, _stream(stream)))
    return [_core_view(gflat[k], ranks[k], dims[k], ranks[k + 1]) for k in range(len(dims))]


def _vec64(x, n, device, name):
    if not x.is_cuda or x.device != device:
        raise ValueError(f"{name} must be a tensor on {device}, got {x.device}")
    if x.numel() != n:
        raise ValueError(f"{name} has {x.numel()} elements, expected {n}")
    return x.contiguous().reshape(-1).to(torch.float64)


def _reduce_work(device):
    return torch.empty(TT_REDUCE_WORK_BYTES, dtype=torch.uint8, device=device)


def tt_residual(pred, vals, stream=None):
    """(z, f): z = pred - vals (FP64, N) and f = sum z^2 / 2 as a one-element
    device tensor (Sec. 4.3: the completion objective at the sampled entries)."""
    lib = load_library()
    n = pred.numel()
    dev = pred.device
    pred = _vec64(pred, n, dev, "pred")
    vals = _vec64(vals, n, dev, "vals")
    z = torch.empty(n, dtype=torch.float64, device=dev)
    f = torch.empty(1, dtype=torch.float64, device=dev)
    work = _reduce_work(dev)
    _check(lib.tt_residual(n, ctypes.c_void_p(pred.data_ptr()), ctypes.c_void_p(vals.data_ptr()),
                           ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                           ctypes.c_void_p(work.data_ptr()), TT_REDUCE_WORK_BYTES, _stream(stream)))
    return z, f


def tt_line_step(p, z, stream=None):
    """Device tensor (alpha, <p, z>, <p, p>) with alpha = <p, z> / <p, p> (0 for
    p = 0): the exact minimiser of 1/2 ||z - alpha p||^2."""
    lib = load_library()
    n = z.numel()
    dev = z.device
    p = _vec64(p, n, dev, "p")
    z = _vec64(z, n, dev, "z")
    out = torch.empty(3, dtype=torch.float64, device=dev)
    work = _reduce_work(dev)
    _check(lib.tt_line_step(n, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(work.data_ptr()), TT_REDUCE_WORK_BYTES,
                            _stream(stream)))
    return out


def tt_axpy(y, x, a=1.0, a_dev=None, stream=None):
    """y += a * s * x in place (y and x contiguous FP64 device tensors of one
    size), s = a_dev[0] (a device scalar) when given, else 1.  Returns y."""
    lib = load_library()
    if y.dtype != torch.float64 or not y.is_contiguous() or not y.is_cuda:
        raise ValueError("y must be a contiguous float64 device tensor")
    x = _vec64(x, y.numel(), y.device, "x")
    ap = None
    if a_dev is not None:
        if not a_dev.is_cuda or a_dev.dtype != torch.float64 or a_dev.numel() < 1:
            raise ValueError("a_dev must be a float64 device tensor")
        ap = ctypes.c_void_p(a_dev.data_ptr())
    _check(lib.tt_axpy(y.numel(), float(a), ap, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                       _stream(stream)))
    return y


def _same_train(a, b, name):
    if len(a) != len(b) or any(tuple(x.shape) != tuple(y.shape) for x, y in zip(a, b)):
        raise ValueError(f"{name} must have the shapes of the first train")


def tt_tangent_project(U, G, stream=None):
    """dC_k = (I - U_k U_k^T) G_k on the left unfoldings for k < d, dC_d = G_d
    (U_1..U_{d-1} left-orthogonal; G the core gradients at the mixed-canonical
    points).  Returns the list of (r0, I, r1) float64 device cores."""
    lib = load_library()
    _same_train(U, G, "G")
    dims, ranks = _train_shape(U)
    ub, gb = _core_buffers(U), _core_buffers(G)
    out = [torch.empty_like(b) for b in ub]
    _check(lib.tt_tangent_project(len(dims), _i64(dims), _i64(ranks), _ptrs(ub), _ptrs(gb), _ptrs(out),
                                  _stream(stream)))
    return [_core_view(out[k], ranks[k], dims[k], ranks[k + 1]) for k in range(len(dims))]


def tt_tangent_train(U, V, dC, t=1.0, t_dev=None, base=False, stream=None):
    """Cores of t*xi (or X + t*xi with base) for the tangent vector
    xi = sum_k U_<k dC_k V_>k at X = U_1..U_d; t = t * t_dev[0] when t_dev (a
    device scalar) is given.  Ranks (1, 2 r_1, ..., 2 r_{d-1}, 1)."""
    lib = load_library()
    _same_train(U, V, "V")
    _same_train(U, dC, "dC")
    dims, ranks = _train_shape(U)
    d = len(dims)
    w = [1] + [2 * r for r in ranks[1:-1]] + [1]
    ub, vb, cb = _core_buffers(U), _core_buffers(V), _core_buffers(dC)
    out = [torch.empty(w[k] * dims[k] * w[k + 1], dtype=torch.float64, device=U[0].device) for k in range(d)]
    tp = None
    if t_dev is not None:
        if not t_dev.is_cuda or t_dev.dtype != torch.float64 or t_dev.numel() < 1:
            raise ValueError("t_dev must be a float64 device tensor")
        tp = ctypes.c_void_p(t_dev.data_ptr())
    _check(lib.tt_tangent_train(d, _i64(dims), _i64(ranks), _ptrs(ub), _ptrs(vb), _ptrs(cb), float(t), tp,
                                1 if base else 0, _ptrs(out), _stream(stream)))
    return [_core_view(out[k], w[k], dims[k], w[k + 1]) for k in range(d)]


class TTSample(torch.autograd.Function):
    """Sampled entries of a train as a differentiable function of its cores;
    the backward is the hand-written tt_sample_backward kernel."""

    @staticmethod
    def forward(ctx, idx, *cores):
        ctx.save_for_backward(idx, *cores)
        return tt_sample(list(cores), idx)

    @staticmethod
    def backward(ctx, gout):
        idx, *cores = ctx.saved_tensors
        grads = tt_sample_backward(list(cores), idx, gout)
        return (None, *[g.to(c.dtype) for g, c in zip(grads, cores)])


class TTReconstruct(torch.autograd.Function):
    """The dense tensor of a train (flat, ivec order) as a differentiable
    function of its cores; the backward is the hand-written
    tt_reconstruct_backward (partial products recomputed, not stored)."""

    @staticmethod
    def forward(ctx, *cores):
        ctx.save_for_backward(*cores)
        return tt_reconstruct(list(cores))

    @staticmethod
    def backward(ctx, gout):
        cores = ctx.saved_tensors
        grads = tt_reconstruct_backward(list(cores), gout)
        return tuple(g.to(c.dtype) for g, c in zip(grads, cores))


class Decomposer:
    """A planned TT-UTV decomposition for a fixed problem shape: workspace,
    core buffers and argument structs are allocated once; each call only runs
    tt_utv_decompose on the given device tensor (same shape and dtype)."""

    def __init__(self, dims, dtype=torch.float64, ranks=None, eps=None, sweep="L2R", variant="ULV", q=1,
                 oversample=8, seed=0, max_rank=0, exact_delta=False, weights=None, profile=False,
                 device="cuda", prec="fp64", fuse_ata=False, orth="householder", separate_sketch=False,
                 inner="sketch"):
        lib = load_library()
        self.lib = lib
        self.dims = [int(x) for x in dims]
        self.d = d = len(self.dims)
        if (ranks is None) == (eps is None):
            raise ValueError("give exactly one of ranks and eps")
        self.dtype = dtype
        self.profile = profile
        self.opts, self._keep = make_opts(q, oversample, seed, max_rank, exact_delta, weights, profile, prec,
                                          fuse_ata, orth, separate_sketch, inner)
        self._dims = _i64(self.dims)
        self._ranks = None if ranks is None else _i64(_full_ranks(ranks, d))
        self.eps = -1.0 if eps is None else float(eps)
        self.sweep, self.variant = SWEEPS[sweep], VARIANTS[variant]
        nbytes = ctypes.c_size_t(0)
        _check(lib.tt_utv_workspace(d, self._dims, self._ranks, self.eps, self.sweep, self.variant, DTYPES[dtype],
                                    ctypes.byref(self.opts), ctypes.byref(nbytes)))
        self.work_bytes = nbytes.value
        self.work = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=device)
        cap = (ctypes.c_int64 * d)()
        _check(lib.tt_utv_core_capacity(d, self._dims, self._ranks, self.eps, ctypes.byref(self.opts), cap))
        self.flats = [torch.empty(max(int(c), 1), dtype=torch.float64, device=device) for c in cap]
        self._cores = _ptrs(self.flats)
        self.rep = tt_report()

    def __call__(self, A, stream=None, allow_rank_miss=False):
        if A.dtype != self.dtype or not A.is_contiguous() or not A.is_cuda:
            raise ValueError("A must be a contiguous device tensor with the planned dtype")
        _check_tensor_size(A, self.dims)
        rc = self.lib.tt_utv_decompose(ctypes.c_void_p(A.data_ptr()), DTYPES[self.dtype], self.d, self._dims,
                                       self._ranks, self.eps, self.sweep, self.variant, ctypes.byref(self.opts),
                                       ctypes.c_void_p(self.work.data_ptr()), self.work_bytes, self._cores,
                                       ctypes.byref(self.rep), _stream(stream))
        _check(rc, allow=(TT_ERANK,) if allow_rank_miss else ())
        return rc

    def set_profile(self, profile):
        """Kernel classes timed with HIP events from the next call on: False/0
        none, True all, an int a bit mask of classes."""
        self.profile = profile
        self.opts.profile = TT_PROFILE_ALL if profile is True else int(profile)

    def cores(self):
        r = [int(self.rep.ranks[k]) for k in range(self.d + 1)]
        return [_core_view(self.flats[k], r[k], self.dims[k], r[k + 1]) for k in range(self.d)]

    def report(self):
        rep, d = self.rep, self.d
        out = {"ranks": [int(rep.ranks[k]) for k in range(d + 1)], "ell": [int(rep.ell[k]) for k in range(d - 1)],
               "delta": [float(rep.delta[k]) for k in range(d - 1)],
               "normC": [float(rep.normC[k]) for k in range(d - 1)], "norm_A": float(rep.norm_A),
               "err_bound": float(rep.err_bound), "rank_rule_met": bool(rep.rank_rule_met),
               "sweeps": [int(rep.sweeps[k]) for k in range(d - 1)],
               "rho": [float(rep.rho[k]) for k in range(d - 1)],
               "err_bound_measured": bool(rep.err_bound_measured)}
        if self.profile:
            out["kstat"] = {self.lib.tt_kernel_class_name(c).decode(): {
                "launches": int(rep.kstat[c].launches), "ms": float(rep.kstat[c].ms),
                "bytes": float(rep.kstat[c].bytes), "flops": float(rep.kstat[c].flops)} for c in range(TT_NKCLASS)}
        return out
