"""Benchmark of the TT-UTV sweep on one MI355X.

One step = one full TT-URV decomposition (right-to-left sweep, Alg. 3) at a
prescribed accuracy of the resident synthetic tensor: order 6, 40^6 FP32
(4.1e9 entries, 16.4 GB) built on the GPU from Gaussian TT cores of ranks 32
plus Gaussian noise at 1e-5 relative Frobenius norm; eps = 1e-4, q = 1 power
step, oversampling 8, ranks capped at 48, every product and carry in FP64
(the FP64 form).

Prints one JSON line: GB/s of tensor swept (tensor bytes / step time), the
roofline of the dominant kernel class (its launches timed with HIP events on
the launch stream during the timed steps), the FP64 oracle timed on the host
cores on a 40^5 instance of the same recipe (and on one thread on 40^4), the
mixed-precision form on the same tensor and on the 8^8 function tensor at
eps = 1e-6, the fixed-rank 32^5 FP64 decomposition, the train contractions,
and Examples 1 and 2 of the paper at 160^4 (SNR, rank and tolerance sweeps).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "TT-URV GB/s swept + roofline %, mixed vs FP64 GPU at 1e-6 rel. error"
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of a kernel class, from rocprofv3 FETCH_SIZE / WRITE_SIZE passes over each
# workload scaled by the copy-probe factors (profiles/); empty whenever the class's kernels changed
# after the counters were taken
MEASURED_TRAFFIC = {"order6_40_fp32_eps": {"tall_ax": 5208.95e6, "tall_atb": 8838.73e6},
                    "order5_32_fp64": {"tall_ax": 49.03e6, "tall_atb": 75.59e6},
                    "order4_160_fp64_defl": {"defl_pass": 1975.11e6}}
FP64_PEAK_TFLOPS = 78.6

WORKLOADS = {
    "order6_40_fp32_eps": dict(
        dims=[40] * 6, gen_ranks=[32] * 5, noise=1e-5, seed=5, eps=1e-4, max_rank=48, q=1, oversample=8,
        sweep="R2L", variant="URV", dtype="float32", device_built=True,
        desc="order-6 40^6 FP32 (4.1e9 entries, 16.4 GB) Gaussian-TT ranks 32 + 1e-5 relative noise; "
             "TT-URV right-to-left, eps=1e-4, q=1, p=8, rank cap 48, FP64 form"),
    "order5_32_fp64": dict(
        dims=[32] * 5, gen_ranks=[16] * 4, noise=1e-6, seed=0, ranks=[16] * 4, q=2, oversample=8,
        sweep="R2L", variant="URV", dtype="float64", device_built=False,
        desc="order-5 32^5 FP64 (33.5M entries) Gaussian-TT ranks 16 + 1e-6 relative noise; "
             "TT-URV right-to-left, fixed rank 16, q=2, p=8"),
    # Example 1 of Sec. 4.1 at 30 dB with the paper's "TT-ULV (USV-plus)" form: the deflation inner kernel
    "order4_160_fp64_defl": dict(
        dims=[160] * 4, gen_ranks=[20] * 3, noise=10.0 ** -1.5, seed=1, ranks=[20] * 3, q=2, oversample=8,
        sweep="L2R", variant="ULV", inner="deflation", dtype="float64", device_built=True,
        desc="order-4 160^4 FP64 (655M entries, 5.2 GB) Gaussian-TT ranks 20 + Gaussian noise at 30 dB SNR "
             "(Example 1); TT-ULV left-to-right with the deflation inner kernel (one vector at a time), fixed "
             "rank 20, q=2 power steps per vector"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stated_bound(T, dims, A, kw, dec):
    """Report of the timed decomposition with its error bound from measured
    step errors: the same (deterministic) decomposition rerun once with
    exact_delta, untimed -- the default step errors sqrt(||C||^2 - ||carry||^2)
    lose digits by cancellation when a step error is below ~1e-7 ||C||, so
    only the measured ones give a bound.  The cores are checked to be the same."""
    import torch

    chk = T.Decomposer(dims, A.dtype, exact_delta=True, **kw)
    chk(A)
    torch.cuda.synchronize()
    for x, y in zip(chk.cores(), dec.cores()):
        if not torch.equal(x, y):
            raise RuntimeError("exact_delta changed the decomposition")
    rep = chk.report()
    del chk
    return rep


def contractions(T, cores, reps=10):
    """The train contractions on the device: reconstruction of the decomposed
    32^5 train (268 MB of FP64 written, an HBM-write-bound pass), its backward
    for a dense upstream gradient (268 MB read twice), and sampling
    and its backward on a (16,16,16,16,16,10) train of ranks 16 and 10 at the
    3,145,728 entries of a 30% mask (the MRI-volume completion shape), each
    timed with events over `reps` calls after one untimed call.  Returns the
    JSON object for the bench line."""
    import numpy as np
    import torch

    import ttgen

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {}
    total = 1
    for g in cores:
        total *= int(g.shape[1])
    ms = timed(lambda: T.tt_reconstruct(cores))
    gbs = total * 8 / (ms * 1e-3) / 1e9
    out["reconstruct"] = {"workload": "32^5 train, ranks 16, to a dense FP64 tensor (268 MB written)",
                          "ms": round(ms, 4), "GB/s written": round(gbs, 1),
                          "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    log(f"bench: reconstruct 32^5 FP64: {ms:.4f} ms, {gbs:.1f} GB/s written ({gbs / HBM_PEAK_GBS:.1%} of HBM peak)")

    # the backward of the reconstruction: a dense FP64 upstream gradient of the
    # same 32^5 shape, read twice (one pass against each half of the train),
    # then the chain rule through the small partial products
    gdense = torch.randn(total, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(13))
    ms = timed(lambda: T.tt_reconstruct_backward(cores, gdense))
    gbs = 2 * total * 8 / (ms * 1e-3) / 1e9
    out["reconstruct_backward"] = {"workload": "32^5 train, ranks 16, dense FP64 upstream gradient (268 MB, read twice)",
                                   "ms": round(ms, 4), "GB/s read": round(gbs, 1),
                                   "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    log(f"bench: reconstruct backward 32^5 FP64: {ms:.4f} ms, {gbs:.1f} GB/s read ({gbs / HBM_PEAK_GBS:.1%} of HBM peak)")
    del gdense

    dims = [16, 16, 16, 16, 16, 10]
    ranks = [1, 16, 16, 16, 16, 10, 1]
    n_obs = 3145728
    c4 = [torch.from_numpy(g).cuda() for g in ttgen.gaussian_cores(dims, ranks, 11)]
    idx = torch.from_numpy(ttgen.random_indices(dims, n_obs, 12)).cuda()
    gout = torch.ones(n_obs, dtype=torch.float64, device="cuda")
    flops_fwd = 2.0 * sum(ranks[k] * ranks[k + 1] for k in range(len(dims)))   # the chain of mat-vecs
    for name, fn, fl in (("sample", lambda: T.tt_sample(c4, idx), flops_fwd),
                         ("sample_backward", lambda: T.tt_sample_backward(c4, idx, gout), 3.0 * flops_fwd)):
        ms = timed(fn)
        rate = n_obs / (ms * 1e-3)
        out[name] = {"workload": "(16,16,16,16,16,10) train, ranks 16/10, 3,145,728 sampled entries",
                     "ms": round(ms, 4), "Msamples/s": round(rate / 1e6, 2),
                     "GFLOP/s": round(rate * fl / 1e9, 1)}
        log(f"bench: {name} (16^5 x 10, 3.1M entries): {ms:.4f} ms, {rate / 1e6:.1f} M samples/s, {rate * fl / 1e9:.1f} GFLOP/s")
    return out


def mixed_vs_fp64(steps):
    """The two precision forms on the 1e-6 workload: 8^8 FP32 function tensor
    1/(1+x_1+...+x_8) on a uniform [0,1] grid, prescribed accuracy eps = 1e-6,
    TT-URV right-to-left, q = 1, p = 8.  Each form is timed over `steps`
    decompositions; the reported bound uses measured step errors."""
    import numpy as np
    import torch

    import paper_2501_07904_amd as T
    import ttgen

    dims = [8] * 8
    a32 = ttgen.inverse_sum_tensor(8, 8, dtype=np.float32)
    A = torch.from_numpy(a32).cuda()
    nbytes = A.numel() * A.element_size()
    res = {"workload": "order-8 8^8 FP32 function tensor 1/(1+sum x), eps=1e-6, TT-URV right-to-left, q=1, p=8"}
    for prec in ("fp64", "mixed"):
        dec = T.Decomposer(dims, A.dtype, eps=1e-6, sweep="R2L", variant="URV", q=1, oversample=8, seed=3,
                           prec=prec)
        dec(A)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            dec(A)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        rep = stated_bound(T, dims, A, dict(eps=1e-6, sweep="R2L", variant="URV", q=1, oversample=8, seed=3,
                                            prec=prec), dec)
        rec = T.tt_reconstruct(dec.cores())
        Ad = A.double()
        rse = float(torch.linalg.norm(rec - Ad) / torch.linalg.norm(Ad))
        res[prec] = {"ms": round(ms, 4), "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 2), "rse": rse,
                     "err_bound_rel": rep["err_bound"] / rep["norm_A"], "ranks": rep["ranks"]}
        log(f"bench: {prec:5s} eps=1e-6 8^8: {ms:.3f} ms, RSE {rse:.3e}, bound {res[prec]['err_bound_rel']:.3e}, "
            f"ranks {rep['ranks']}")
    res["speedup_mixed_over_fp64"] = round(res["fp64"]["ms"] / res["mixed"]["ms"], 3)
    res["note"] = ("every step of this workload has core side n <= 64 and forms A^T A in one FP64 pass: no "
                   "low-precision product runs, the mixed form differs only in the FP32 storage of the carries, "
                   "and both forms are bound by the same single-workgroup factorisations (ceiling 1.0x)")
    return res


# Sec. 4.1: Example 1 sweeps SNR 0..30 dB at TT-ranks (20,20,20) and the ranks (r,r,r), r = 2..20, at
# 30 dB; Example 2 takes the tolerances of Table "Beps", whose TT-SVD column is quoted here for comparison
EX1_SNR = (0, 5, 10, 15, 20, 25, 30)
EX1_RANKS = (2, 4, 6, 8, 10, 12, 14, 16, 18, 20)
BEPS_TTSVD_RANKS = {1e-2: [2, 2, 2], 1e-3: [3, 3, 3], 1e-4: [5, 5, 5], 1e-5: [7, 7, 6]}
EXAMPLE_FORMS = (("R2L", "URV"), ("L2R", "ULV"))
# TT-ULV with the deflation inner kernel (the paper's "TT-ULV (USV-plus)" rows): left to right, q = 2 power
# steps per vector; with a prescribed accuracy the rank cap 24 keeps every core side within the 4096 its
# streaming pass takes (24 x 160)
DEFL_KW = dict(sweep="L2R", variant="ULV", inner="deflation", q=2)
# TT-SVD, the paper's baseline, left to right (core sides above 64 by subspace iteration on 64 directions)
SVD_KW = dict(sweep="L2R", variant="SVD")
DEFL_EPS_MAX_RANK = 24


def paper_examples(T, reps):
    """Examples 1 and 2 of Sec. 4.1 at the paper's size on the GPU, each
    decomposition timed over `reps` calls after one untimed call, for TT-URV
    right to left (Alg. 3) and TT-ULV left to right (Alg. 1/2), q = 1, p = 8.
    Example 1: 160^4 FP64 (5.2 GB), A = P + beta N with P contracted from
    Gaussian cores of TT-ranks 20 and N Gaussian, beta set by the SNR
    10 log10(||P||^2 / ||beta N||^2); SNR sweep at ranks (20,20,20) and rank
    sweep at 30 dB.  Example 2: the 160^4 FP64 tensor sin(sqrt(sum x_k^2)) at
    the tolerances of Table "Beps"."""
    import torch

    import ttgen

    def run(A, dims, kw):
        dec = T.Decomposer(dims, A.dtype, **kw)
        dec(A)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            dec(A)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        rep = dec.report()
        rse = relative_error(T, dec.cores(), A)
        del dec
        torch.cuda.empty_cache()
        gbs = A.numel() * A.element_size() / (ms * 1e-3) / 1e9
        return {"ms": round(ms, 3), "GB/s": round(gbs, 1), "rse": rse, "ranks": rep["ranks"][1:-1],
                "err_bound_rel": rep["err_bound"] / rep["norm_A"]}

    dims = [160] * 4
    out = {"reps": reps}
    ex1 = {"workload": "160^4 FP64 (5.2 GB): Gaussian-TT cores of ranks 20 plus Gaussian noise at the given SNR "
                       "(Sec. 4.1, Example 1); fixed TT-ranks, q=1, p=8 (sketch), q=2 per vector (deflation)",
           "snr_sweep": [], "rank_sweep": []}
    for snr in EX1_SNR:
        noise = 10.0 ** (-snr / 20.0)
        A = ttgen.gaussian_tt_tensor_device(dims, [20] * 3, noise, 1, dtype="float64", device="cuda")
        row = {"snr_db": snr, "noise_rel_to_signal": noise}
        for sweep, variant in EXAMPLE_FORMS:
            row[f"{variant}_{sweep}"] = run(A, dims, dict(ranks=[20] * 3, sweep=sweep, variant=variant, q=1,
                                                          oversample=8, seed=1))
        row["ULV_L2R_deflation"] = run(A, dims, dict(ranks=[20] * 3, seed=1, **DEFL_KW))
        row["SVD_L2R"] = run(A, dims, dict(ranks=[20] * 3, seed=1, **SVD_KW))
        log(f"bench: example 1 SNR {snr:2d} dB, ranks 20: " + ", ".join(
            f"{k} {v['ms']:.2f} ms RSE {v['rse']:.4e}" for k, v in row.items() if isinstance(v, dict)))
        ex1["snr_sweep"].append(row)
        if snr == 30:
            for r in EX1_RANKS:
                rrow = {"rank": r}
                for sweep, variant in EXAMPLE_FORMS:
                    rrow[f"{variant}_{sweep}"] = run(A, dims, dict(ranks=[r] * 3, sweep=sweep, variant=variant,
                                                                   q=1, oversample=8, seed=1))
                rrow["ULV_L2R_deflation"] = run(A, dims, dict(ranks=[r] * 3, seed=1, **DEFL_KW))
                rrow["SVD_L2R"] = run(A, dims, dict(ranks=[r] * 3, seed=1, **SVD_KW))
                log(f"bench: example 1 SNR 30 dB, ranks {r:2d}: " + ", ".join(
                    f"{k} {v['ms']:.2f} ms RSE {v['rse']:.4e}" for k, v in rrow.items() if isinstance(v, dict)))
                ex1["rank_sweep"].append(rrow)
        del A
        torch.cuda.empty_cache()
    out["example1"] = ex1
    ex2 = {"workload": "160^4 FP64 (5.2 GB) sin(sqrt(sum_k ((i_k-1)/159)^2)) (Sec. 4.1, Example 2); prescribed "
                       "accuracy, q=1, p=8 (sketch), q=2 per vector and rank cap 24 (deflation); "
                       "ttsvd_ranks_paper is the TT-SVD column of Table \"Beps\"",
           "eps_sweep": []}
    B = ttgen.sin_norm_tensor_device(4, 160, device="cuda")
    for eps, svd_ranks in BEPS_TTSVD_RANKS.items():
        row = {"eps": eps, "ttsvd_ranks_paper": svd_ranks}
        for sweep, variant in EXAMPLE_FORMS:
            row[f"{variant}_{sweep}"] = run(B, dims, dict(eps=eps, sweep=sweep, variant=variant, q=1, oversample=8,
                                                          seed=2))
        row["ULV_L2R_deflation"] = run(B, dims, dict(eps=eps, seed=2, max_rank=DEFL_EPS_MAX_RANK, **DEFL_KW))
        row["SVD_L2R"] = run(B, dims, dict(eps=eps, seed=2, **SVD_KW))
        log(f"bench: example 2 eps {eps:g}: TT-SVD (paper) {svd_ranks}, " + ", ".join(
            f"{k} ranks {v['ranks']} {v['ms']:.2f} ms RSE {v['rse']:.3e}" for k, v in row.items()
            if isinstance(v, dict)))
        ex2["eps_sweep"].append(row)
    del B
    torch.cuda.empty_cache()
    out["example2"] = ex2
    return out


def decomposer_kw(W):
    kw = dict(sweep=W["sweep"], variant=W["variant"], q=W["q"], oversample=W["oversample"], seed=W["seed"],
              inner=W.get("inner", "sketch"))
    if "ranks" in W:
        kw["ranks"] = W["ranks"]
    else:
        kw["eps"] = W["eps"]
        kw["max_rank"] = W["max_rank"]
    return kw


def build_input(W):
    """The workload's tensor on the GPU (and on the host when it is built there)."""
    import numpy as np
    import torch

    import ttgen

    log(f"bench: generating {W['desc']}")
    if W["device_built"]:
        A = ttgen.gaussian_tt_tensor_device(W["dims"], W["gen_ranks"], W["noise"], W["seed"], dtype=W["dtype"],
                                            device="cuda")
        torch.cuda.synchronize()
        return A, None
    a, _ = ttgen.gaussian_tt_tensor(W["dims"], W["gen_ranks"], W["noise"], W["seed"], dtype=getattr(np, W["dtype"]))
    return torch.from_numpy(a).cuda(), a


def timed_decompositions(T, W, A, steps, warmup, prec="fp64"):
    """Warm-up, two calibration steps with every kernel class timed with events,
    then `steps` timed decompositions; the last one carries events on the
    launches of the dominant streaming class (an event pair idles the queue for
    a few microseconds, so the other timed steps run without them)."""
    import torch

    dec = T.Decomposer(W["dims"], A.dtype, prec=prec, **decomposer_kw(W))
    log(f"bench: [{prec}] warmup {warmup}")
    for _ in range(warmup):
        dec(A)
    torch.cuda.synchronize()
    dec.set_profile(True)
    cal = {}
    for _ in range(2):
        dec(A)
        for name, v in dec.report()["kstat"].items():
            acc = cal.setdefault(name, {"launches": 0, "ms": 0.0, "bytes": 0.0, "flops": 0.0})
            for key in acc:
                acc[key] += v[key] / 2
    streaming = {k: v for k, v in cal.items() if v["bytes"] > 0 and v["launches"] > 0}
    dom_name = max(streaming, key=lambda k: streaming[k]["ms"])
    names = [T.load_library().tt_kernel_class_name(c).decode() for c in range(T.TT_NKCLASS)]
    for name, v in sorted(cal.items(), key=lambda kv: -kv[1]["ms"]):
        if v["launches"]:
            gbs = v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] else 0.0
            log(f"bench: [{prec}] kernel {name:9s} launches/step {v['launches']:5.1f} ms/step {v['ms']:.4f}  "
                f"GB/s {gbs:8.1f}")
    log(f"bench: [{prec}] timing {steps} steps (events on the {dom_name} launches of the last one)")
    dec.set_profile(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        if i == steps - 1:
            dec.set_profile(1 << names.index(dom_name))
        dec(A)   # fixed ranks: one synchronisation at the end; eps: one per step
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kstat = dict(dec.report()["kstat"][dom_name])
    dec.set_profile(0)
    ms_per_step = (t1 - t0) * 1e3 / steps
    return dict(dec=dec, ms=ms_per_step, cal=cal, streaming=streaming, dom=dom_name, kstat=kstat)


def roofline(tm, traffic):
    """Roofline object of the dominant class: algorithmic bytes (or flops) per
    launch / average launch duration against the HBM (or FP64 matrix-core)
    peak, plus the whole-step figure over every streaming pass."""
    k = tm["kstat"]
    avg_ms = k["ms"] / k["launches"]
    bytes_per = k["bytes"] / k["launches"]
    flops_per = k["flops"] / k["launches"]
    intensity = flops_per / bytes_per if bytes_per else 0.0
    ridge = FP64_PEAK_TFLOPS * 1e3 / HBM_PEAK_GBS   # flop per byte where the HBM and FP64 peaks meet
    if intensity < ridge:
        achieved = bytes_per / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4)}
    else:
        achieved = flops_per / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4)}
    roof["traffic"] = traffic.get(tm["dom"])
    roof["kernel"] = tm["dom"]
    roof["launches_per_step"] = k["launches"]
    roof["avg_launch_ms"] = round(avg_ms, 5)
    roof["alg_bytes_per_launch"] = bytes_per
    roof["alg_flops_per_launch"] = flops_per
    roof["hbm_GBps_per_launch"] = round(bytes_per / (avg_ms * 1e-3) / 1e9, 1)
    roof["step_share"] = {n: round(v["ms"] / tm["ms"], 3) for n, v in tm["cal"].items() if v["launches"]}
    t_roof = sum(max(v["bytes"] / (HBM_PEAK_GBS * 1e9), v["flops"] / (FP64_PEAK_TFLOPS * 1e12))
                 for v in tm["streaming"].values()) * 1e3
    roof["step_t_roof_ms"] = round(t_roof, 5)
    roof["step_frac"] = round(t_roof / tm["ms"], 4)
    return roof


def relative_error(T, cores, A):
    """||A - A_TT||_F / ||A||_F with the train reconstructed in FP64 (an FP32
    reconstruction would add its own rounding), summed in slices."""
    import torch

    rec = T.tt_reconstruct(cores)
    err2 = nrm2 = 0.0
    step = 1 << 28
    for s0 in range(0, A.numel(), step):
        a = A[s0:s0 + step].double()
        err2 += float(torch.linalg.vector_norm(rec[s0:s0 + step] - a) ** 2)
        nrm2 += float(torch.linalg.vector_norm(a) ** 2)
    del rec
    return (err2 / nrm2) ** 0.5


def finish_form(T, W, A, tm, prec):
    """Cores, report, RSE and the stated bound (from measured step errors, the
    same decomposition rerun untimed with exact_delta) of a timed form; frees
    the timed decomposer first."""
    import torch

    dec = tm.pop("dec")
    cores = [c.clone() for c in dec.cores()]
    rep = dec.report()
    del dec
    torch.cuda.empty_cache()
    chk = T.Decomposer(W["dims"], A.dtype, prec=prec, exact_delta=True, **decomposer_kw(W))
    chk(A)
    torch.cuda.synchronize()
    for x, y in zip(chk.cores(), cores):
        if not torch.equal(x, y):
            raise RuntimeError("exact_delta changed the decomposition")
    brep = chk.report()
    del chk
    torch.cuda.empty_cache()
    rse = relative_error(T, cores, A)
    return cores, rep, rse, brep["err_bound"] / brep["norm_A"]


def cpu_baseline():
    """The FP64 oracle on the host on bounded samples of the headline recipe:
    40^5 FP32 (Gaussian-TT ranks 32 + 1e-5 noise, eps = 1e-4, q = 1, p = 8,
    rank cap 48, TT-URV right-to-left) on every BLAS thread, and 40^4 of the
    same recipe on one thread."""
    import numpy as np

    import oracle
    import ttgen
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores_used = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:  # threadpoolctl missing: numpy's BLAS default is all cores
        threadpool_limits = None
        cores_used = os.cpu_count()
    kw = dict(eps=1e-4, sweep="R2L", variant="URV", q=1, p=8, seed=5, max_rank=48)
    a5, _ = ttgen.gaussian_tt_tensor([40] * 5, [32] * 4, 1e-5, 5, dtype=np.float32)
    log(f"bench: timing the FP64 oracle on the host (40^5 FP32, {cores_used} threads, >= 10 s)")
    runs, t0 = 0, time.perf_counter()
    while runs == 0 or time.perf_counter() - t0 < 10.0:
        _, rep5 = oracle.tt_utv(a5, [40] * 5, **kw)
        runs += 1
    t5 = (time.perf_counter() - t0) / runs
    out = {"value": round(a5.nbytes / t5 / 1e9, 5), "unit": "GB/s", "cores": cores_used, "kind": "oracle",
           "sample": f"{runs} decompositions of a 40^5 FP32 instance of the same recipe ({a5.nbytes / 1e6:.0f} MB, "
                     f"ranks {rep5['ranks']}), {t5:.1f} s each"}
    del a5
    if threadpool_limits is not None:
        a4, _ = ttgen.gaussian_tt_tensor([40] * 4, [32] * 3, 1e-5, 5, dtype=np.float32)
        with threadpool_limits(limits=1):
            reps, t0 = 0, time.perf_counter()
            while reps == 0 or time.perf_counter() - t0 < 3.0:
                oracle.tt_utv(a4, [40] * 4, **kw)
                reps += 1
            t4 = (time.perf_counter() - t0) / reps
        out["single_thread"] = {"value": round(a4.nbytes / t4 / 1e9, 5), "unit": "GB/s", "cores": 1,
                                "sample": f"{reps} decompositions of a 40^4 FP32 instance ({a4.nbytes / 1e6:.1f} MB), "
                                          f"{t4:.2f} s each"}
    log(f"bench: oracle {out['value']} GB/s on {cores_used} threads"
        + (f", {out['single_thread']['value']} GB/s on one" if "single_thread" in out else ""))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="order6_40_fp32_eps", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision form")
    ap.add_argument("--mixed-steps", type=int, default=10)
    ap.add_argument("--no-c2", action="store_true", help="skip the fixed-rank 32^5 FP64 decomposition")
    ap.add_argument("--c2-steps", type=int, default=20)
    ap.add_argument("--no-examples", action="store_true",
                    help="skip Examples 1 and 2 of the paper at 160^4 (SNR, rank and tolerance sweeps)")
    ap.add_argument("--example-reps", type=int, default=3)
    ap.add_argument("--no-contractions", action="store_true",
                    help="skip the timing of reconstruction, sampling and its backward")
    ap.add_argument("--copy-probe", action="store_true",
                    help="allocate and fill a 4 GiB buffer before the timed steps and copy it once after them "
                         "(a kernel of known traffic on data the decompositions have evicted from every cache: "
                         "it calibrates the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2501_07904_amd as T

    W = WORKLOADS[args.workload]
    probe_src = None
    if args.copy_probe:
        probe_src = torch.empty(1 << 29, dtype=torch.float64, device="cuda").normal_()
    A, a_host = build_input(W)
    tensor_bytes = A.numel() * A.element_size()
    tm = timed_decompositions(T, W, A, args.steps, args.warmup)
    ms_per_step = tm["ms"]
    value = tensor_bytes / (ms_per_step * 1e-3) / 1e9
    roof = roofline(tm, MEASURED_TRAFFIC.get(args.workload, {}))
    if probe_src is not None:
        # an elementwise kernel (a device-to-device copy_ would go to the DMA engines, which the counters
        # do not see): reads and writes 4 GiB once
        dst = torch.empty_like(probe_src)
        torch.mul(probe_src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"bench: copy probe kernel read {probe_src.numel() * 8} bytes and wrote {probe_src.numel() * 8} bytes")
        del dst, probe_src
    cores, rep, rse, bound = finish_form(T, W, A, tm, "fp64")
    log(f"bench: {ms_per_step:.3f} ms/step, {value:.1f} GB/s swept, ranks {rep['ranks']}, RSE {rse:.3e}, "
        f"stated bound {bound:.3e}, Jacobi sweeps {rep['sweeps']}")
    log(f"bench: roofline {roof['kernel']}: {roof['achieved']} {roof['unit']} = {roof['frac']:.1%} of peak, "
        f"{roof['hbm_GBps_per_launch']} GB/s per launch, whole step {roof['step_frac']:.1%}")

    mixed = None
    if not args.no_mixed:
        mixed = {}
        if "eps" in W:
            tmm = timed_decompositions(T, W, A, args.mixed_steps, args.warmup, prec="mixed")
            mms = tmm["ms"]
            # what the roofline allows the mixed form to gain: algorithmic HBM bytes of the
            # streaming passes per decomposition, FP64 form over mixed form
            bytes64 = sum(v["bytes"] for v in tm["streaming"].values())
            bytesmx = sum(v["bytes"] for v in tmm["streaming"].values())
            _, mrep, mrse, mbound = finish_form(T, W, A, tmm, "mixed")
            mixed["c5"] = {"workload": W["desc"].replace("FP64 form", "mixed form"),
                           "fp64": {"ms": round(ms_per_step, 3), "GB/s": round(value, 1), "rse": rse,
                                    "err_bound_rel": bound, "ranks": rep["ranks"]},
                           "mixed": {"ms": round(mms, 3), "GB/s": round(tensor_bytes / (mms * 1e-3) / 1e9, 1),
                                     "rse": mrse, "err_bound_rel": mbound, "ranks": mrep["ranks"]},
                           "speedup_mixed_over_fp64": round(ms_per_step / mms, 3),
                           "alg_hbm_bytes_per_step": {"fp64": bytes64, "mixed": bytesmx},
                           "roofline_ceiling_speedup": round(bytes64 / bytesmx, 3),
                           "note": "the step-1 Gram pass over the FP32 input, the step-1 carry and the "
                                   "Rayleigh-Ritz pass decide the ranks and stay FP64-accurate in both forms; "
                                   "the mixed form halves the bytes of the FP64 step-2 carry and runs the power "
                                   "products on FP32 matrix cores, so its HBM-bound ceiling is the byte ratio"}
            log(f"bench: mixed {mms:.3f} ms/step ({ms_per_step / mms:.2f}x the FP64 form), RSE {mrse:.3e}, "
                f"stated bound {mbound:.3e}, ranks {mrep['ranks']}")
    del A
    torch.cuda.empty_cache()
    if not args.no_mixed:
        mixed["c3"] = mixed_vs_fp64(args.mixed_steps)

    c2 = None
    c2_cores = None
    if not args.no_c2 and args.workload != "order5_32_fp64":
        W2 = WORKLOADS["order5_32_fp64"]
        A2, _ = build_input(W2)
        tm2 = timed_decompositions(T, W2, A2, args.c2_steps, 3)
        roof2 = roofline(tm2, MEASURED_TRAFFIC.get("order5_32_fp64", {}))
        c2_cores = [c.clone() for c in tm2["dec"].cores()]
        c2_ranks = tm2["dec"].report()["ranks"]
        del tm2["dec"]
        rse2 = relative_error(T, c2_cores, A2)
        v2 = A2.numel() * A2.element_size() / (tm2["ms"] * 1e-3) / 1e9
        # the same decomposition with the CholeskyQR orthonormaliser for the intermediate iterates
        dq = T.Decomposer(W2["dims"], A2.dtype, orth="cholqr", **decomposer_kw(W2))
        for _ in range(3):
            dq(A2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.c2_steps):
            dq(A2)
        torch.cuda.synchronize()
        ms_q = (time.perf_counter() - t0) * 1e3 / args.c2_steps
        del dq
        # the same ranks with the deflation inner kernel (one vector at a time, q = 1 power step each)
        dd = T.Decomposer(W2["dims"], A2.dtype, **dict(decomposer_kw(W2), inner="deflation"))
        for _ in range(3):
            dd(A2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.c2_steps):
            dd(A2)
        torch.cuda.synchronize()
        ms_d = (time.perf_counter() - t0) * 1e3 / args.c2_steps
        rse_d = relative_error(T, dd.cores(), A2)
        dd.set_profile(True)   # one more call with HIP events on every launch, for the pass durations
        dd(A2)
        torch.cuda.synchronize()
        kd = dd.report()["kstat"]["defl_pass"]
        del dd
        defl = {"ms_per_step": round(ms_d, 5), "rse": rse_d,
                "defl_pass_launches": kd["launches"],
                "defl_pass_avg_us": round(kd["ms"] * 1e3 / max(kd["launches"], 1), 3),
                "defl_pass_GB/s": round(kd["bytes"] / max(kd["ms"], 1e-9) / 1e6, 1),
                "note": "pass figures from one extra call with HIP events on every launch"}
        log(f"bench: 32^5 deflation inner kernel: {ms_d:.4f} ms/step, RSE {rse_d:.3e}, {kd['launches']} passes at "
            f"{defl['defl_pass_avg_us']:.1f} us = {defl['defl_pass_GB/s']:.0f} GB/s")
        # the same tensor and ranks with TT-ULV left to right and with TT-SVD (the configuration's
        # "TT-SVD vs TT-URV vs TT-ULV", plain FP64 path)
        others = {}
        for key, kw in (("ttulv_l2r", dict(decomposer_kw(W2), sweep="L2R", variant="ULV")),
                        ("ttsvd_r2l", dict(decomposer_kw(W2), variant="SVD"))):
            do = T.Decomposer(W2["dims"], A2.dtype, **kw)
            for _ in range(3):
                do(A2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.c2_steps):
                do(A2)
            torch.cuda.synchronize()
            ms_o = (time.perf_counter() - t0) * 1e3 / args.c2_steps
            others[key] = {"ms_per_step": round(ms_o, 5), "rse": relative_error(T, do.cores(), A2),
                           "ranks": do.report()["ranks"]}
            del do
        log(f"bench: 32^5 TT-ULV L2R {others['ttulv_l2r']['ms_per_step']:.4f} ms/step (RSE "
            f"{others['ttulv_l2r']['rse']:.3e}), TT-SVD {others['ttsvd_r2l']['ms_per_step']:.4f} ms/step (RSE "
            f"{others['ttsvd_r2l']['rse']:.3e})")
        c2 = {"workload": W2["desc"], "value": round(v2, 2), "unit": "GB/s", "ms_per_step": round(tm2["ms"], 5),
              "steps": args.c2_steps, "ranks": c2_ranks, "rse": rse2, "roofline": roof2,
              "ms_per_step_orth_cholqr": round(ms_q, 5), "deflation": defl, **others,
              "ttsvd_note": "TT-SVD: the exact step (ell = n) where the core side is at most 64, else subspace "
                            "iteration on the leading 64 directions with 30 power steps"}
        log(f"bench: 32^5 FP64 fixed rank: {tm2['ms']:.4f} ms/step, {v2:.1f} GB/s swept, RSE {rse2:.3e}, "
            f"{roof2['kernel']} {roof2['frac']:.1%} of peak, whole step {roof2['step_frac']:.1%}")
        del A2
        torch.cuda.empty_cache()
    contr = None
    if not args.no_contractions:
        if c2_cores is None:
            W2 = WORKLOADS["order5_32_fp64"]
            A2, _ = build_input(W2)
            c2_cores, _ = T.tt_utv_decompose(A2, W2["dims"], **decomposer_kw(W2))
            del A2
        contr = contractions(T, c2_cores)

    examples = None if args.no_examples else paper_examples(T, args.example_reps)

    cpu = None if args.no_cpu_baseline else cpu_baseline()

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": W["desc"], "ranks": rep["ranks"], "rse": rse, "err_bound_rel": bound},
        "roofline": roof, "cpu_baseline": cpu, "mixed_vs_fp64": mixed, "c2_order5_32_fp64": c2,
        "contractions": contr, "paper_examples": examples,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
