"""Benchmark: TOD samples/s per PCG iteration of the map-making solve on one MI355X.

Workload (default): TQU polarisation, 4 detectors at 0/45/90/135 deg with a
2 Hz half-wave plate, 4 x 2^22 samples on a 256 x 256 raster, 2^20-sample
stationary intervals, 1/f noise (f_knee 0.2 Hz, alpha 1.7), correlation length
8192; float32 TOD and weights, mixed-precision PCG (float32 filtering and
scatter, float64 CG) to relative residual 1e-8.

One step = the whole hot path on inputs resident in HBM: plan (pixel sort,
observed compaction, filters, preconditioner), right-hand side, PCG iterations
to tolerance, map output.  value = samples x RHS x PCG iterations / step time.

Also reported: the per-iteration time, the dominant kernel's achieved HBM
bandwidth against the 8 TB/s peak (HIP events on its launch stream), the
float64-vs-mixed time to the same map error, and the CPU oracle timed on a
bounded sample.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ols_filter_c2_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_0906_1775_amd", "csrc", f) for f in ("k_filter.hip", "fft.hpp")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def make_plan(prob, tod_dev, precision, n_rhs):
    import torch
    from paper_0906_1775_amd import MapMaker
    dev = tod_dev.device
    return MapMaker(prob["pix"], prob["w"], prob["n_pix"], 3, prob["iv_start"], prob["iv_filter"],
                    filter_params=prob["filter_params"], f_samp=prob["f_samp"], n_c=prob["n_c"],
                    precision=precision, n_rhs=n_rhs)


def cpu_baseline(p, budget_s: float = 20.0):
    """The FP64 oracle's H application timed on the host on a bounded sample."""
    import numpy as np
    from oracle import Oracle
    # sample: the first detector's data (4 stationary intervals, 2^22 samples)
    n = int(p.det_start[1])
    nb = int(np.searchsorted(p.iv_start, n))
    orc = Oracle(p.pix[:n], p.w[:n], p.n_pix, 3, p.iv_start[:nb + 1], p.iv_filter[:nb],
                 p.filter_params, p.f_samp, p.n_c)
    x = np.random.default_rng(0).standard_normal(orc.n_unknowns)
    orc.apply_H(x)                          # warm-up
    reps, t0 = 0, time.perf_counter()
    while True:
        orc.apply_H(x)
        reps += 1
        if time.perf_counter() - t0 > budget_s / 2 or reps >= 40:
            break
    dt = (time.perf_counter() - t0) / reps
    return dict(value=n / dt, unit="TOD samples/s per PCG iteration", cores=os.cpu_count(),
                kind="oracle",
                sample=f"one H = P^T N^-1 P application of the FP64 oracle on detector 0 "
                       f"({n} samples, {nb} intervals), mean of {reps}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tts", action="store_true", help="skip the time-to-solution comparison")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see the sharding design); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth

    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    p = synth.make_problem("c2")
    print(f"[bench] generated c2 inputs in {time.perf_counter() - t_gen:.1f}s", file=sys.stderr, flush=True)
    prob = dict(pix=torch.from_numpy(p.pix).to(dev), w=torch.from_numpy(p.w).to(dev), n_pix=p.n_pix,
                iv_start=p.iv_start, iv_filter=p.iv_filter, filter_params=p.filter_params,
                f_samp=p.f_samp, n_c=p.n_c)
    tod = torch.from_numpy(p.tod).to(dev)
    n_t, R = p.n_samples, p.n_rhs
    torch.cuda.synchronize()

    def step():
        mm = make_plan(prob, tod, args.precision, R)
        m, info = mm.solve(tod, tol=args.tol, max_iter=1000, check_every=8)
        mm.close()
        return info

    for _ in range(args.warmup):
        info = step()
        print(f"[bench] warmup step: {info['iters']} iterations, status {info['status']}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    for _ in range(args.steps):
        info = step()
        iters += sum(info["iters"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    value = n_t * iters / elapsed
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.2f} ms/step, {iters / args.steps:.1f} iterations/step",
          file=sys.stderr, flush=True)

    # ---- per-iteration time and the dominant kernel, on a persistent plan
    mm = make_plan(prob, tod, args.precision, R)
    pinfo = mm.info()
    t_plan0 = time.perf_counter()
    mm2 = make_plan(prob, tod, args.precision, R)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t_plan0) * 1e3
    mm2.close()
    s = torch.cuda.current_stream()

    def timed_solve(k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        mm.solve(tod, fixed_iters=k, check_every=8)
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    timed_solve(8)
    t_a, t_b = timed_solve(8), timed_solve(40)
    t_iter_ms = (t_b - t_a) / 32.0

    # dominant kernel: the overlap-save N^-1 transform, launched alone by mm_weight on stream s
    y_in = tod if args.precision == "mixed" else tod.double()
    y_out = torch.empty_like(y_in)
    import ctypes
    from paper_0906_1775_amd import _lib as L
    lib = L.load()
    dt = L.MM_F32 if y_in.dtype == torch.float32 else L.MM_F64

    def launch():
        L.check(lib.mm_weight(mm._h, ctypes.c_void_p(y_in.data_ptr()), ctypes.c_void_p(y_out.data_ptr()),
                              dt, ctypes.c_void_p(s.cuda_stream)), lib)
    for _ in range(3):
        launch()
    n_launch = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(n_launch):
        launch()
    e1.record(s)
    torch.cuda.synchronize()
    ols_ms = e0.elapsed_time(e1) / n_launch
    # a plain device copy of the same TOD buffer, the reference for the HBM byte counters
    y_out.copy_(y_in)
    torch.cuda.synchronize()
    esz = 4 if args.precision == "mixed" else 8
    alg_bytes = n_t * R * 2 * esz          # read the TOD once, write the filtered TOD once
    achieved = alg_bytes / (ols_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_source_hash") == kernel_source_hash() and tr.get("precision") == args.precision:
            traffic = tr.get("bytes_per_launch")
    roofline = dict(kernel="k_ols (overlap-save N^-1, n_f=%d)" % pinfo["n_f"], bound="hbm",
                    achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    launch_ms=round(ols_ms, 4), algorithmic_bytes=alg_bytes)

    # ---- time to solution at fixed map error: plain FP64 vs mixed
    tts = None
    if not args.no_tts:
        ref_plan = make_plan(prob, tod, "fp64", R)
        ref, _ = ref_plan.solve(tod, tol=1e-11, max_iter=2000)

        def err(m):
            return float(torch.linalg.norm(m - ref) / torch.linalg.norm(ref))

        def tts_of(plan, tol):
            plan.solve(tod, tol=tol, max_iter=2000)      # warm (graph capture, lazy float64 path)
            torch.cuda.synchronize()
            t = time.perf_counter()
            m, inf = plan.solve(tod, tol=tol, max_iter=2000)
            torch.cuda.synchronize()
            return time.perf_counter() - t, err(m), inf["iters"][0]
        t64, e64, i64 = tts_of(ref_plan, args.tol)
        tmx, emx, imx = None, None, None
        for tol in (args.tol, args.tol / 3, args.tol / 10, args.tol / 30, args.tol / 100):
            tmx, emx, imx = tts_of(mm, tol)
            if emx <= e64:
                break
        tts = dict(target_map_error=e64, fp64_s=round(t64, 5), fp64_iters=i64, mixed_s=round(tmx, 5),
                   mixed_iters=imx, mixed_map_error=emx, speedup=round(t64 / tmx, 3) if tmx else None,
                   reached=bool(emx <= e64))
        ref_plan.close()
    mm.close()

    cpu = None if args.no_cpu_baseline else cpu_baseline(p)

    out = {
        "metric": "TOD samples/s per PCG iteration (% HBM roofline); time-to-solution at fixed error",
        "value": value,
        "unit": "TOD samples/s per PCG iteration",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "TQU 4 det x 2^22 samples, 256x256 px, HWP 2 Hz, n_c 8192, "
                               f"{args.precision} PCG to {args.tol:g}",
                   "n_samples": n_t, "n_rhs": R, "n_obs": pinfo["n_obs"], "n_f": pinfo["n_f"],
                   "n_c": p.n_c},
        "iters_per_step": iters / args.steps,
        "t_iter_ms": round(t_iter_ms, 4),
        "iter_samples_per_s": n_t * R / (t_iter_ms * 1e-3),
        "plan_ms": round(plan_ms, 2),
        "time_to_solution": tts,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
