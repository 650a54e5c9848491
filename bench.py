"""Benchmark of the TT-UTV sweep on one MI355X.

One step = one full TT-URV decomposition (right-to-left sweep, Alg. 3) of the
resident synthetic tensor: order 5, 32^5 FP64 (33.5M entries, 268 MB),
contracted from Gaussian TT cores of ranks 16 plus Gaussian noise at 1e-6
relative Frobenius norm, fixed rank 16, q = 2 power steps, oversampling 8.

Prints one JSON line: GB/s of tensor swept (tensor bytes / step time), the
roofline of the dominant kernel class (its launches timed with HIP events on
the launch stream during the timed steps), and the FP64 oracle timed on the
host cores for one decomposition of the same tensor.
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
# HBM bytes per launch of a kernel class, from rocprofv3 FETCH_SIZE / WRITE_SIZE passes over this
# workload scaled by the copy-probe factors (profiles/c2_order5_32_fp64_tturv_r2l.md); set to None
# whenever the class's kernels change after the counters were taken
MEASURED_TRAFFIC = {"tall_atb": 76.49e6, "tall_ax": 49.03e6}
FP64_PEAK_TFLOPS = 78.6

WORKLOADS = {
    "order5_32_fp64": dict(
        dims=[32] * 5, gen_ranks=[16] * 4, noise=1e-6, seed=0, ranks=[16] * 4, q=2, oversample=8,
        sweep="R2L", variant="URV",
        desc="order-5 32^5 FP64 (33.5M entries) Gaussian-TT ranks 16 + 1e-6 relative noise; "
             "TT-URV right-to-left, fixed rank 16, q=2, p=8"),
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
    32^5 train (268 MB of FP64 written, an HBM-write-bound pass), and sampling
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
    return res


def mixed_vs_fp64_c5(steps):
    """The large workload of the mixed-vs-FP64 comparison: order-6 40^6 FP32
    (4.1e9 entries, 16.4 GB) from Gaussian TT cores of ranks 32 plus 1e-5
    relative noise, built on the GPU; prescribed accuracy eps = 1e-4, TT-URV
    right-to-left, q = 1, p = 8, ranks capped at 48.  Each form is timed over
    `steps` decompositions; RSE from the reconstruction."""
    import torch

    import paper_2501_07904_amd as T
    import ttgen

    dims = [40] * 6
    log("bench: generating the 40^6 FP32 tensor on the GPU")
    A = ttgen.gaussian_tt_tensor_device(dims, [32] * 5, 1e-5, 5, dtype="float32", device="cuda")
    nbytes = A.numel() * A.element_size()
    normA = float(torch.linalg.vector_norm(A, dtype=torch.float64))
    res = {"workload": "order-6 40^6 FP32 (16.4 GB) Gaussian-TT ranks 32 + 1e-5 noise, eps=1e-4, "
                       "TT-URV right-to-left, q=1, p=8, rank cap 48"}
    for prec in ("fp64", "mixed"):
        dec = T.Decomposer(dims, A.dtype, eps=1e-4, sweep="R2L", variant="URV", q=1, oversample=8, seed=5,
                           max_rank=48, prec=prec)
        dec(A)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            dec(A)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        rep = stated_bound(T, dims, A, dict(eps=1e-4, sweep="R2L", variant="URV", q=1, oversample=8, seed=5,
                                            max_rank=48, prec=prec), dec)
        # FP64 reconstruction (32.8 GB): an FP32 one would add its own rounding to the error
        rec = T.tt_reconstruct(dec.cores())
        err2 = 0.0
        for s0 in range(0, A.numel(), 1 << 28):
            err2 += float(torch.linalg.vector_norm(rec[s0:s0 + (1 << 28)].double() - A[s0:s0 + (1 << 28)].double()) ** 2)
        del rec
        rse = err2 ** 0.5 / normA
        res[prec] = {"ms": round(ms, 3), "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1), "rse": rse,
                     "err_bound_rel": rep["err_bound"] / rep["norm_A"], "ranks": rep["ranks"]}
        log(f"bench: {prec:5s} eps=1e-4 40^6: {ms:.2f} ms, RSE {rse:.3e}, bound {res[prec]['err_bound_rel']:.3e}, "
            f"ranks {rep['ranks']}")
        del dec
        torch.cuda.empty_cache()
    res["speedup_mixed_over_fp64"] = round(res["fp64"]["ms"] / res["mixed"]["ms"], 3)
    del A
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="order5_32_fp64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-vs-FP64 comparison")
    ap.add_argument("--mixed-steps", type=int, default=10)
    ap.add_argument("--no-c5", action="store_true", help="skip the 40^6 (16.4 GB) mixed-vs-FP64 comparison")
    ap.add_argument("--c5-steps", type=int, default=3)
    ap.add_argument("--no-contractions", action="store_true",
                    help="skip the timing of reconstruction, sampling and its backward")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed steps, copy the input tensor once (a kernel of known "
                         "traffic: its bytes read and written) to calibrate HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2501_07904_amd as T
    import ttgen

    W = WORKLOADS[args.workload]
    log(f"bench: generating {W['desc']}")
    a, _ = ttgen.gaussian_tt_tensor(W["dims"], W["gen_ranks"], W["noise"], W["seed"])
    A = torch.from_numpy(a).cuda()
    tensor_bytes = A.numel() * A.element_size()
    dec = T.Decomposer(W["dims"], A.dtype, ranks=W["ranks"], sweep=W["sweep"], variant=W["variant"], q=W["q"],
                       oversample=W["oversample"])
    log(f"bench: warmup {args.warmup}")
    for _ in range(args.warmup):
        dec(A)
    torch.cuda.synchronize()

    # calibration, outside the timed region: every kernel class timed with events
    dec.set_profile(True)
    cal = {}
    for _ in range(2):
        dec(A)
        for name, v in dec.report()["kstat"].items():
            acc = cal.setdefault(name, {"launches": 0, "ms": 0.0, "bytes": 0.0, "flops": 0.0})
            for key in acc:
                acc[key] += v[key] / 2
    # the dominant streaming kernel: most launch time among the classes that read A
    streaming = {k: v for k, v in cal.items() if v["bytes"] > 0 and v["launches"] > 0}
    dom_name = max(streaming, key=lambda k: streaming[k]["ms"])
    names = [T.load_library().tt_kernel_class_name(c).decode() for c in range(T.TT_NKCLASS)]
    dom_class = names.index(dom_name)
    for name, v in sorted(cal.items(), key=lambda kv: -kv[1]["ms"]):
        if v["launches"]:
            gbs = v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] else 0.0
            log(f"bench: kernel {name:9s} launches/step {v['launches']:5.1f} ms/step {v['ms']:.4f}  GB/s {gbs:8.1f}")

    # timed region: the dominant class's launches of the last timed step carry
    # events (each event pair idles the queue for a few microseconds, so the
    # other steps run without them)
    kstat = {"launches": 0, "ms": 0.0, "bytes": 0.0, "flops": 0.0}
    log(f"bench: timing {args.steps} steps (events on the {dom_name} launches of the last one)")
    dec.set_profile(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        if i == args.steps - 1:
            dec.set_profile(1 << dom_class)
        dec(A)  # fixed ranks: the call synchronises once at the end to fill its report
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    v = dec.report()["kstat"][dom_name]
    for key in kstat:
        kstat[key] += v[key]
    dec.set_profile(0)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = tensor_bytes / (ms_per_step * 1e-3) / 1e9
    if args.copy_probe:
        # an elementwise kernel (a device-to-device copy_ would go to the DMA engines,
        # which the counters do not see): reads and writes the tensor once
        B = torch.empty_like(A)
        torch.mul(A, 1.0, out=B)
        torch.cuda.synchronize()
        log(f"bench: copy probe kernel read {tensor_bytes} bytes and wrote {tensor_bytes} bytes")
        del B
    rep = dec.report()
    cores = dec.cores()
    rec = T.tt_reconstruct(cores)
    rse = float(torch.linalg.norm(rec - A) / torch.linalg.norm(A))
    log(f"bench: {ms_per_step:.4f} ms/step, {value:.1f} GB/s swept, ranks {rep['ranks']}, RSE {rse:.3e}, "
        f"Jacobi sweeps {rep['sweeps']}")

    avg_ms = kstat["ms"] / kstat["launches"]
    bytes_per = kstat["bytes"] / kstat["launches"]
    flops_per = kstat["flops"] / kstat["launches"]
    intensity = flops_per / bytes_per if bytes_per else 0.0
    ridge = FP64_PEAK_TFLOPS * 1e3 / HBM_PEAK_GBS   # flop per byte where HBM and FP64 peaks meet
    if intensity < ridge:
        achieved = bytes_per / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None}
    else:
        achieved = flops_per / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": None}
    roof["traffic"] = MEASURED_TRAFFIC.get(dom_name) if W is WORKLOADS["order5_32_fp64"] else None
    roof["kernel"] = dom_name
    roof["launches_per_step"] = kstat["launches"]
    roof["avg_launch_ms"] = round(avg_ms, 5)
    roof["alg_bytes_per_launch"] = bytes_per
    roof["alg_flops_per_launch"] = flops_per
    # share of the step spent in each class (calibration steps), and the whole-step
    # roofline: algorithmic bytes and flops of every streaming pass at the HBM / FP64 peaks
    roof["step_share"] = {k: round(v["ms"] / ms_per_step, 3) for k, v in cal.items() if v["launches"]}
    t_roof = sum(max(v["bytes"] / (HBM_PEAK_GBS * 1e9), v["flops"] / (FP64_PEAK_TFLOPS * 1e12))
                 for v in streaming.values()) * 1e3
    roof["step_t_roof_ms"] = round(t_roof, 5)
    roof["step_frac"] = round(t_roof / ms_per_step, 4)

    del rec
    contr = None if args.no_contractions else contractions(T, cores)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        try:
            from threadpoolctl import threadpool_info
            cores_used = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
        except Exception:  # threadpoolctl missing: numpy's BLAS default is all cores
            cores_used = os.cpu_count()
        log("bench: timing the FP64 oracle on the host (full decompositions of the same tensor, >= 10 s)")
        runs = 0
        c0 = time.perf_counter()
        while runs == 0 or time.perf_counter() - c0 < 10.0:
            oracle.tt_utv(a, W["dims"], ranks=W["ranks"], sweep=W["sweep"], variant=W["variant"], q=W["q"],
                          p=W["oversample"], seed=0)
            runs += 1
        c1 = time.perf_counter()
        cpu = {"value": round(runs * tensor_bytes / (c1 - c0) / 1e9, 5), "unit": "GB/s", "cores": cores_used,
               "kind": "oracle", "sample": f"{runs} full decompositions of the same 32^5 FP64 tensor "
                                           f"({c1 - c0:.1f} s)"}

    mixed = None
    if not args.no_mixed:
        mixed = {"c3": mixed_vs_fp64(args.mixed_steps)}
        if not args.no_c5:
            mixed["c5"] = mixed_vs_fp64_c5(args.c5_steps)

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": W["desc"], "ranks": rep["ranks"], "rse": rse},
        "roofline": roof, "cpu_baseline": cpu, "mixed_vs_fp64": mixed, "contractions": contr,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
