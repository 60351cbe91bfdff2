"""Benchmark of the lattice-QCD hot path on one MI355X.

Workload (default): Wilson-clover on a 32^3x64 lattice, links U = exp(i eps H)
with eps = 0.25 (seed 2001), kappa = 0.124, c_sw = 1, antiperiodic in time,
one Gaussian source (seed 2002); mixed-precision GCR-DD (FP64 restarts, FP32
Krylov space, FP16 additive-Schwarz preconditioner on 8^4 Dirichlet blocks
with 8 MR steps) to ||b - M x|| <= 1e-10 ||b||.

One timed step is one pass over the whole path: a batch of Wilson dslash
launches (FP32, 12-real links; the headline kernel), one FP32 Schur matvec
batch, and one complete GCR-DD solve. `value` is the dslash bandwidth in
algorithmic bytes (input spinor 24 + output 24 + 8 links x 12 reals per
site, FP32) divided by the average kernel time measured with HIP events on
the launch stream. Time-to-solution of the GCR-DD solve is reported beside
plain FP64 CG (CGNE on the even-odd system, same stopping rule, same GPU),
and the CPU oracle (FP64, OpenMP) is timed on a bounded sample of the same
workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "dslash GB/s & % of HBM roofline; time-to-solution at 1e-10 residual vs FP64 CG"

WILSON_REALS = {18: 192, 12: 144, 8: 112}  # in 24 + out 24 + 8 links per output site
SCHUR_REALS = {18: 552, 12: 456, 8: 392}   # two fused kernels, per even site
PREC_BYTES = {0: 8, 1: 4, 2: 2, 3: 2}
PREC_NAME = {0: "f64", 1: "f32", 2: "f16", 3: "bf16"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dslash-launches", type=int, default=50)
    ap.add_argument("--dims", type=str, default="32,32,32,64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--kernels-only", action="store_true", help="time kernels only (for profiling runs)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_kernel(torch, fn, launches):
    """Average duration of `fn` (one kernel launch or a fixed sequence) with
    HIP events on the current stream."""
    fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(launches):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / 1e3 / launches


def device_copy(torch, nbytes=2 << 30, launches=20):
    """Bandwidth of a plain device-to-device copy kernel (read + write bytes /
    time), the practical ceiling next to the 8 TB/s specification. The same
    kernel, with known bytes, calibrates the HBM traffic counters."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    c = torch.empty_like(a)
    dt = time_kernel(torch, lambda: c.copy_(a), launches)
    del a, c
    return {"bytes_per_launch": 2 * nbytes, "us": round(dt * 1e6, 1), "GB/s": round(2 * nbytes / dt / 1e9, 1)}


def cpu_baseline(dims, U, b, kappa, csw):
    """The oracle's FP64 Wilson dslash (one parity) on the same fields, timed
    on the host cores; reported in the same unit (algorithmic GB/s, FP64
    18-real links: 1536 bytes per output site)."""
    import numpy as np
    import oracle
    oracle.lib()
    V = int(np.prod(dims))
    src = np.where(oracle.parity_mask(dims, 1)[..., None, None], b, 0)
    oracle.wilson_dslash(dims, U, src, bc_t=-1, out_parity=0)  # warm
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.wilson_dslash(dims, U, src, bc_t=-1, out_parity=0)
        reps += 1
        if time.perf_counter() - t0 > 10.0 or reps >= 5:
            break
    dt = (time.perf_counter() - t0) / reps
    gbs = (V // 2) * 1536 / dt / 1e9
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": "%d applications of the FP64 Wilson hopping term (one parity) on the full %s lattice, "
                      "%.2f s each" % (reps, "x".join(map(str, dims)), dt)}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the path runs on a single MI355X (--gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_1109_2935_amd import lqcd as L
    from paper_1109_2935_amd import ops

    dims = tuple(int(v) for v in args.dims.split(","))
    kappa, csw, eps, block, mr = 0.124, 1.0, 0.25, (8, 8, 8, 8), 8
    vh = int(np.prod(dims)) // 2
    log("generating fields", dims)
    t = time.time()
    U = synth.gauge_field(dims, eps, 2001)
    b = synth.gaussian_spinor(dims, 2002)
    log("fields ready %.1fs" % (time.time() - t))
    ctx = L.lqcd_context_create()
    Ud = torch.from_numpy(U).cuda()
    inst = {}
    for prec, recon in [(0, 18), (0, 12), (1, 18), (1, 12), (1, 8), (2, 18), (2, 12), (3, 12)]:
        inst[(prec, recon)] = ops.wilson_clover(ctx, U, dims, kappa, csw, prec, recon, tile=block, U_device=Ud)
    torch.cuda.synchronize()
    log("operators ready")

    # ---- kernel table: Wilson dslash and Schur matvec, every precision/recon
    kernels = {}
    head = None
    for (prec, recon), o in inst.items():
        inp = o.import_spinor(np.where(synth.parity_of_sites(dims)[..., None, None] == 1, b, 0), 1)
        out = o.spinor()
        dt = time_kernel(torch, lambda: L.lqcd_dslash(ctx, o.op, out, inp, 0, 0), args.dslash_launches)
        byts = vh * WILSON_REALS[recon] * PREC_BYTES[prec]
        kernels["dslash_%s_r%d" % (PREC_NAME[prec], recon)] = {
            "us": round(dt * 1e6, 2), "GB/s": round(byts / dt / 1e9, 1),
            "frac": round(byts / dt / 1e9 / HBM_PEAK_GBS, 4), "bytes": byts}
        if (prec, recon) == (1, 12):
            head = (dt, byts)
        ein = o.import_spinor(b, 0)
        eout = o.spinor()
        dts = time_kernel(torch, lambda: L.lqcd_schur_apply(ctx, o.op, eout, ein), max(5, args.dslash_launches // 4))
        sb = vh * SCHUR_REALS[recon] * PREC_BYTES[prec]
        kernels["schur_%s_r%d" % (PREC_NAME[prec], recon)] = {
            "us": round(dts * 1e6, 2), "GB/s": round(sb / dts / 1e9, 1),
            "frac": round(sb / dts / 1e9 / HBM_PEAK_GBS, 4), "bytes": sb}
        log("%-18s %8.1f us %7.1f GB/s | schur %8.1f us %7.1f GB/s" % (
            "%s r%d" % (PREC_NAME[prec], recon), dt * 1e6, byts / dt / 1e9, dts * 1e6, sb / dts / 1e9))
    copy = device_copy(torch)
    log("device copy %.1f GB/s" % copy["GB/s"])
    if args.kernels_only:
        print(json.dumps({"kernels": kernels, "device_copy": copy}))
        return

    o64, o32, o16 = inst[(0, 18)], inst[(1, 12)], inst[(2, 12)]
    bp = o64.import_spinor(b, -1)
    prm = ops.gcr_params(1e-10, k_max=16, delta=1e-3, max_iter=2000, precond=L.LQCD_PRECOND_SCHWARZ,
                         block=block, mr_steps=mr)
    inp = o32.import_spinor(np.where(synth.parity_of_sites(dims)[..., None, None] == 1, b, 0), 1)
    out = o32.spinor()
    ein, eout = o32.import_spinor(b, 0), o32.spinor()

    def step():
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(args.dslash_launches):
            L.lqcd_dslash(ctx, o32.op, out, inp, 0, 0)
        e.record()
        for _ in range(5):
            L.lqcd_schur_apply(ctx, o32.op, eout, ein)
        x = o64.spinor(full=True)
        st, info = L.lqcd_gcr_solve(ctx, o64.op, o32.op, o16.op, prm, x, bp)
        assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
        e.synchronize()
        return s.elapsed_time(e) / 1e3 / args.dslash_launches, info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dts, infos = [], []
    for _ in range(args.steps):
        dt, info = step()
        dts.append(dt)
        infos.append(info)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dt_avg = sum(dts) / len(dts)
    byts = head[1]
    gbs = byts / dt_avg / 1e9
    gcr = infos[-1]
    log("GCR-DD: %d steps, %d restarts, %.3f s, true residual %.2e" % (gcr.iters, gcr.restarts, gcr.seconds,
                                                                      gcr.true_residual))
    tts = {"gcr_dd_seconds": round(min(i.seconds for i in infos), 4), "gcr_dd_steps": gcr.iters,
           "gcr_dd_restarts": gcr.restarts, "gcr_dd_true_residual": gcr.true_residual,
           "precond_applies": gcr.precond_applies}
    if not args.no_cg:
        x = o64.spinor(full=True)
        st, cg = L.lqcd_cg_solve(ctx, o64.op, None, ops.cg_params(1e-10, max_iter=20000), x, bp)
        log("FP64 CGNE: %d iterations, %.3f s, true residual %.2e" % (cg.iters, cg.seconds, cg.true_residual))
        tts.update({"fp64_cg_seconds": round(cg.seconds, 4), "fp64_cg_iters": cg.iters,
                    "fp64_cg_true_residual": cg.true_residual,
                    "speedup_vs_fp64_cg": round(cg.seconds / tts["gcr_dd_seconds"], 2)})
    res = {
        "metric": METRIC, "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "wilson-clover %s, kappa %.3f, c_sw %.1f, eps %.2f, antiperiodic t; GCR-DD "
                               "FP64/FP32/FP16, Schwarz 8^4 blocks, %d MR steps" % (
                                   "x".join(map(str, dims)), kappa, csw, eps, mr),
                   "dims": list(dims), "kernel": "wilson dslash f32 recon12, one parity",
                   "dslash_launches_per_step": args.dslash_launches},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None},
        "time_to_solution": tts,
        "device_copy": copy,
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        res["cpu_baseline"] = cpu_baseline(dims, U, b, kappa, csw)
    torch.cuda.synchronize()
    L.lqcd_context_destroy(ctx)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
