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

# HBM traffic of the headline kernel per launch, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE scaled by the same counters on a 2 GiB device copy (summary under
# profiles/). Valid only for the kernel sources it was measured on: their hash
# is checked at run time and the traffic is reported as null when they differ.
PROFILED_TRAFFIC = {"sources_sha1": "d723e502af221fefc3ae477560ba39812b96399a", "bytes_per_launch": 662.6e6}


def kernel_sources_sha1():
    import hashlib
    h = hashlib.sha1()
    for f in ("wilson.hip", "lqcd_device.h"):
        with open(os.path.join(ROOT, "paper_1109_2935_amd", "csrc", f), "rb") as fh:
            h.update((hashlib.sha1(fh.read()).hexdigest() + "  " + os.path.join("paper_1109_2935_amd", "csrc", f) + "\n").encode())
    return h.hexdigest()
SCHUR_REALS = {18: 552, 12: 456, 8: 392}   # two fused kernels, per even site
PREC_BYTES = {0: 8, 1: 4, 2: 2, 3: 2, 4: 2}
# Link reals of the FP16 Schwarz operator: with the packed-half hops the
# block-resident K is bound by vector issue, and rebuilding the third link row
# costs more there than the 50% more link bytes of the full matrix (1.38 ms
# against 1.58 ms for 8 MR steps at 32^3x64)
K_RECON = 18
PREC_NAME = {0: "f64", 1: "f32", 2: "f16", 3: "bf16", 4: "half"}
# 16-bit fixed point adds an FP32 norm per site to every spinor and clover
# access: 2 spinor norms per dslash output site; 5 spinor and 2 clover norms
# per even site of the Schur operator
FIXED_NORM_BYTES = {"dslash": 8, "schur": 28}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dslash-launches", type=int, default=120,
                    help="launches per kernel timing (rotating over 3 buffer sets; median over groups)")
    ap.add_argument("--solves", type=int, default=5, help="timed solves per solver (after one warm-up): median")
    ap.add_argument("--dims", type=str, default="32,32,32,64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--kernels-only", action="store_true", help="time kernels only (for profiling runs)")
    ap.add_argument("--learned", default=os.path.join(ROOT, "paper_1109_2935_amd", "data", "ptc_16x4.npz"),
                    help="trained network weights; FGCR with it is timed when the file exists")
    ap.add_argument("--no-staggered", action="store_true", help="skip the 48^3x96 staggered workload")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched multi-RHS workload")
    ap.add_argument("--only", choices=("staggered", "batched", "learned", "solve", "blocks"), default=None,
                    help="run one secondary workload alone and print its JSON (for profiling runs); solve: one "
                         "warm-up and one timed GCR-DD solve of the default workload")
    ap.add_argument("--oracle-solve", choices=("8x4", "32x64"), default=None, help=argparse.SUPPRESS)
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stencil_tile(dims, block):
    """Tile of the stencil operators: the full x and y extents and 4 sites
    along z and t where they divide (of the tilings timed at 32^3x64 the
    fastest for the FP32 and FP64 hopping terms, 1-2% ahead of 8 sites along
    y, z and t); otherwise the full x extent and 8 sites along y, z and t
    where they divide, else the Schwarz block."""
    t = (dims[0], dims[1], 4, 4)
    if all(d % e == 0 for d, e in zip(dims, t)):
        return t
    t = (dims[0],) + tuple(8 if d % 8 == 0 else b for d, b in zip(dims[1:], block[1:]))
    return t if all(d % e == 0 and e % 2 == 0 for d, e in zip(dims, t)) else tuple(block)


def full_x_tile(dims):
    """The full x extent and, along y, z and t, the largest of 8, 6, 4, 2 that
    divides the extent (the batched lattices include 20^3x40)."""
    return (dims[0],) + tuple(next(e for e in (8, 6, 4, 2) if d % e == 0) for d in dims[1:])


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


def time_rotating(torch, fns, launches):
    """Median launch duration of a kernel over at least `launches` launches
    that rotate over len(fns) buffer sets (one callable per set, each set with
    its own inputs, outputs, links and clover fields, so that the 256 MB MALL
    cannot serve a launch from the previous one). Each group of len(fns)
    launches is bracketed by HIP events on the current stream; the result is the
    median over the groups of the group time divided by its launch count."""
    for f in fns:
        f()
    torch.cuda.synchronize()
    groups = max(1, -(-launches // len(fns)))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(groups + 1)]
    ev[0].record()
    for g in range(groups):
        for f in fns:
            f()
        ev[g + 1].record()
    ev[-1].synchronize()
    per = sorted(ev[g].elapsed_time(ev[g + 1]) / 1e3 / len(fns) for g in range(groups))
    return per[len(per) // 2]


def median_of(vals):
    v = sorted(vals)
    return v[len(v) // 2]


def device_copy(torch, L, ctx, nbytes=2 << 30, launches=20):
    """Bandwidth of the library's streaming copy kernel (read + write bytes /
    time), the practical ceiling of a read-once/write-once kernel next to the
    8 TB/s specification. The same kernel, with known bytes, calibrates the
    HBM traffic counters."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    c = torch.empty_like(a)
    dt = time_kernel(torch, lambda: L.lqcd_stream_copy(ctx, c, a, nbytes), launches)
    del a, c
    return {"kernel": "stream_copy_kernel", "bytes_per_launch": 2 * nbytes, "us": round(dt * 1e6, 1),
            "GB/s": round(2 * nbytes / dt / 1e9, 1)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_solve_timing(which):
    """The oracle's FP64 even-odd CGNE (bench.py --oracle-solve), run in a
    child process so that its thread count is set by the environment: the
    full 8^4 solve of the smallest workload to 1e-10 ("8x4"), or a bounded
    sample of the 32^3x64 solve: 2 CGNE iterations ("32x64")."""
    import numpy as np
    import oracle
    import synth
    from oracle import solvers
    oracle.lib()
    if which == "8x4":
        dims, kappa, su, sb, tol, maxit = (8, 8, 8, 8), 0.12, 1001, 1002, 1e-10, 100000
    else:
        dims, kappa, su, sb, tol, maxit = (32, 32, 32, 64), 0.124, 2001, 2002, 1e-10, 2
    U = synth.gauge_field(dims, 0.25, su)
    b = synth.gaussian_spinor(dims, sb)
    t0 = time.perf_counter()
    op = oracle.WilsonClover(dims, U, kappa, 1.0, bc_t=-1)
    bhat = op.schur_source(b)
    t1 = time.perf_counter()
    xe, it, _ = solvers.cgne(op.schur, lambda v: op.schur(v, dagger=True), bhat, tol=tol, maxiter=maxit)
    t2 = time.perf_counter()
    return {"setup_s": round(t1 - t0, 3), "solve_s": round(t2 - t1, 3), "iters": it}


def run_oracle_solve(which, threads):
    import subprocess
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = str(threads)
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-solve", which], env=env,
                         capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        raise RuntimeError(out.stderr[-2000:])
    return json.loads(out.stdout.strip().splitlines()[-1])


def cpu_baseline(dims, U, b, kappa, csw):
    """The oracle's FP64 Wilson dslash (one parity) on the same fields, timed
    on the host cores; reported in the same unit (algorithmic GB/s, FP64
    18-real links: 1536 bytes per output site). Beside it, the oracle's FP64
    even-odd CGNE: the whole 8^4 solve on one core and on all cores, and a
    2-iteration sample of the 32^3x64 solve on all cores."""
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
        # about 10 s of host work (bounded in count for slow hosts)
        if time.perf_counter() - t0 > 10.0 or reps >= 1000:
            break
    dt = (time.perf_counter() - t0) / reps
    gbs = (V // 2) * 1536 / dt / 1e9
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    solves = {}
    try:
        solves["cgne_8x4_1core"] = run_oracle_solve("8x4", 1)
        solves["cgne_8x4_all_cores"] = run_oracle_solve("8x4", cores)
        s = run_oracle_solve("32x64", cores)
        s["seconds_per_iteration"] = round(s["solve_s"] / max(1, s["iters"]), 3)
        solves["cgne_32x64_sample_all_cores"] = s
    except Exception as e:  # the dslash figure stands without them
        log("oracle solve timing failed: %s" % e)
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": "%d applications of the FP64 Wilson hopping term (one parity) on the full %s lattice, "
                      "%.2f s each" % (reps, "x".join(map(str, dims)), dt),
            "cpu_model": cpu_model(), "solves": solves}


def timed_solves(n, fn):
    """One warm-up solve, then n timed ones: (median seconds, all seconds, the
    info of the median run). fn() returns (status, info)."""
    fn()
    runs = []
    for _ in range(n):
        st, info = fn()
        runs.append((info.seconds, info))
    runs.sort(key=lambda r: r[0])
    return runs[len(runs) // 2][0], [round(r[0], 4) for r in runs], runs[len(runs) // 2][1]


def solve_record(med, allt, info):
    return {"seconds": round(med, 4), "seconds_runs": allt, "steps": info.iters, "restarts": info.restarts,
            "matvecs": info.matvecs, "true_residual": info.true_residual}


def learned_solves(args, L, ops, ctx, o64, o32, o32b, bp, net, prm):
    """FGCR with the network and GCR without a preconditioner (median of
    args.solves each, after a warm-up)."""
    import ctypes
    prm.learned = ctypes.pointer(net.net)

    def fgcr():
        x = o64.spinor(full=True)
        st, info = L.lqcd_gcr_solve(ctx, o64.op, o32.op, o32b.op, prm, x, bp)
        assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
        return st, info

    def plain():
        x = o64.spinor(full=True)
        st, info = L.lqcd_gcr_solve(ctx, o64.op, o32.op, None, ops.gcr_params(1e-10, 16, 1e-3, max_iter=5000), x, bp)
        assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
        return st, info

    med, allt, best = timed_solves(args.solves, fgcr)
    pmed, pall, pinfo = timed_solves(args.solves, plain)
    log("GCR without preconditioner: %d steps, %.3f s, true residual %.2e" % (pinfo.iters, pmed, pinfo.true_residual))
    log("FGCR(PTC): %d steps (%d Schwarz fallback), %.3f s, true residual %.2e" % (
        best.iters, best.fallback_applies, med, best.true_residual))
    r1, r2 = solve_record(pmed, pall, pinfo), solve_record(med, allt, best)
    r2["fallback_applies"] = best.fallback_applies
    return {"gcr_unpreconditioned": r1, "fgcr_learned": r2}


def learned_solve(args, torch, L, ops, ctx, o64, o32, o32b, bp, block, mr, dims):
    """Flexible GCR with the trained PTC network as preconditioner (Schwarz as
    fallback), FP64 restarts, FP32 Krylov; and the cost of one network
    application (BF16 matrix-core flops of its channel mixing). With
    --kernels-only, the application alone."""
    import numpy as np
    from paper_1109_2935_amd import ptc
    net = ptc.Network(ctx)
    net.load(args.learned)
    prm = ops.gcr_params(1e-10, 16, 1e-3, max_iter=2000, precond=L.LQCD_PRECOND_LEARNED, block=block, mr_steps=mr)
    res = {}
    if not args.kernels_only:
        res = learned_solves(args, L, ops, ctx, o64, o32, o32b, bp, net, prm)
    # one application in the layout the solver applies it in (the Schwarz block tiling)
    r = o32b.spinor()
    out = o32b.spinor()
    L.lqcd_spinor_convert(ctx, o32b.op, r, o64.op, bp, 0)
    dt = median_of([time_kernel(torch, lambda: net.apply(o32b, out, r), 1) for _ in range(7)])
    V = int(np.prod(dims))
    ch = net.channels
    # complex multiply-adds per site: cout*4 x cin*9*4 for each of 3 colours; both parities except the last layer
    macs = sum(co * 4 * ci * 36 * 3 * (V // 2 if k == len(ch) - 2 else V) for k, (ci, co) in enumerate(zip(ch[:-1], ch[1:])))
    log("PTC network: one application %.2f ms, %.1f TFLOP/s (BF16 channel mixing)" % (
        dt * 1e3, 8 * macs / dt / 1e12))
    res.update({"ptc_apply_ms": round(dt * 1e3, 3), "ptc_apply_tflops": round(8 * macs / dt / 1e12, 1)})
    return res


def staggered_workload(args, torch, L, ops, ctx):
    """48^3x96 improved staggered (m = 0.01, eps = 0.2): dslash bandwidth per
    precision and long-link format, reliable-update CG (FP32 / FP16 sloppy
    operator) against plain FP64 CG."""
    import numpy as np
    import synth
    dims, mass = (48, 48, 48, 96), 0.01
    t = time.time()
    U = synth.gauge_field(dims, 0.2, 3001)
    fat = synth.fat_links(dims, U, seed=3003)
    chi = synth.gaussian_spinor(dims, 3002, inner=(3,))
    log("staggered fields %.1fs" % (time.time() - t))
    Ud, Fd = torch.from_numpy(U).cuda(), torch.from_numpy(fat).cuda()
    vh = int(np.prod(dims)) // 2
    out = {"dims": list(dims), "kernels": {}}
    inst = {}
    odd_src = np.where(synth.parity_of_sites(dims)[..., None] == 1, chi, 0)
    for prec, recon in [(0, 18), (1, 18), (1, 12), (1, 8), (2, 12)]:
        o = ops.staggered(ctx, fat, U, dims, mass, prec, recon, U_device=Ud, fat_device=Fd)
        inst[(prec, recon)] = o
        sets = [(r, r.import_spinor(odd_src, 1), r.spinor()) for r in (o, o.replica(), o.replica())]
        dt = time_rotating(torch, [lambda r=r, i=i, q=q: L.lqcd_dslash(ctx, r.op, q, i, 0) for r, i, q in sets],
                           args.dslash_launches // 2)
        del sets
        byts = vh * (12 + 8 * 18 + 8 * recon) * PREC_BYTES[prec]
        out["kernels"]["stag_dslash_%s_r%d" % (PREC_NAME[prec], recon)] = {
            "us": round(dt * 1e6, 1), "GB/s": round(byts / dt / 1e9, 1), "frac": round(byts / dt / 1e9 / HBM_PEAK_GBS, 4)}
        log("staggered %s r%d: %.1f us %.1f GB/s" % (PREC_NAME[prec], recon, dt * 1e6, byts / dt / 1e9))
    del Ud, Fd
    if args.kernels_only:
        return out
    hi = inst[(0, 18)]
    b = hi.import_spinor(np.where(synth.parity_of_sites(dims)[..., None] == 0, chi, 0), 0)
    for name, lo in (("fp64", None), ("fp32_sloppy", inst[(1, 12)]), ("fp16_sloppy", inst[(2, 12)])):
        def solve(lo=lo):
            x = hi.spinor()
            st, info = L.lqcd_cg_solve(ctx, hi.op, lo.op if lo else None,
                                       ops.cg_params(1e-10, 20000, 0.1, L.LQCD_CG_STAG_NORMAL), x, b)
            assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
            return st, info
        med, allt, info = timed_solves(args.solves, solve)
        out["cg_" + name] = solve_record(med, allt, info)
        log("staggered CG %s: %d it, %.3f s, res %.2e" % (name, info.iters, med, info.true_residual))
    out["multishift"] = multishift_workload(L, ops, ctx, hi, inst[(1, 12)], b, mass)
    for name in ("fp32_sloppy", "fp16_sloppy"):
        out["speedup_%s_vs_fp64" % name] = round(out["cg_fp64"]["seconds"] / out["cg_" + name]["seconds"], 2)
    return out


def multishift_workload(L, ops, ctx, hi, lo, b, mass):
    """Eq. (4) for 8 shifts (sigma = 0 and 1e-4 .. 0.4 geometric) on 48^3x96:
    the multi-shift CG in FP32 then reliable-update refinement of each solution
    (Section VIII-B), against one mixed-precision CG per shift in sequence."""
    import math
    shifts = [0.0] + [1e-4 * 4 ** k for k in range(7)]
    xs = [hi.spinor() for _ in shifts]
    runs = []
    for _ in range(4):  # a warm-up, then the median of 3
        st, info = L.lqcd_multishift_cg_solve(ctx, hi.op, lo.op,
                                              ops.multishift_params(shifts, tol=1e-10, tol_sloppy=1e-8), xs, b)
        assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
        runs.append(info)
    info = sorted(runs[1:], key=lambda i: i.seconds)[1]
    ref_iters = [info.shift[i].iters for i in range(len(shifts))]
    worst = max(info.shift[i].true_residual for i in range(len(shifts)))
    # the same systems one at a time: mixed-precision CG at mass sqrt(m^2 + sigma)
    seq_seconds, seq_iters = 0.0, []
    for s_ in shifts:
        oh = L.lqcd_operator.from_buffer_copy(hi.op)
        ol = L.lqcd_operator.from_buffer_copy(lo.op)
        oh.mass = ol.mass = math.sqrt(mass * mass + s_)
        x = hi.spinor()
        st, ci = L.lqcd_cg_solve(ctx, oh, ol, ops.cg_params(1e-10, 20000, 0.1, L.LQCD_CG_STAG_NORMAL), x, b)
        assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
        seq_seconds += ci.seconds
        seq_iters.append(ci.iters)
    log("multi-shift (%d shifts): FP32 stage %d it %.3f s, refinements %s it, total %.3f s (worst residual %.2e); "
        "sequential mixed CG %.3f s (%s it)" % (len(shifts), info.ms_iters, info.ms_seconds, ref_iters, info.seconds,
                                               worst, seq_seconds, seq_iters))
    return {"shifts": shifts, "seconds": round(info.seconds, 4), "ms_iters": info.ms_iters,
            "ms_seconds": round(info.ms_seconds, 4), "refine_iters": ref_iters, "worst_true_residual": worst,
            "sequential_cg_seconds": round(seq_seconds, 4), "sequential_cg_iters": seq_iters,
            "speedup_vs_sequential": round(seq_seconds / info.seconds, 2)}


def batched_workload(args, torch, L, ops, ctx):
    """Multi-RHS Wilson hopping term: 12 point sources (spin x colour) on
    24^3x48, and one persistent launch over 16^3x32, 20^3x40 and 24^3x48 with
    4 Gaussian sources each (kappa 0.122), in full-x tiles. Bytes per site and right-hand side:
    spinor in + out (48 reals) plus the site's 8 links shared by its nrhs.
    16-bit operators are also timed with the link products on the matrix cores
    (LQCD_MRHS_MFMA=1)."""
    import numpy as np
    import synth
    out = {}

    def with_mfma(on, fn):
        old = os.environ.get("LQCD_MRHS_MFMA")
        os.environ["LQCD_MRHS_MFMA"] = "1" if on else "0"
        try:
            return fn()
        finally:
            if old is None:
                del os.environ["LQCD_MRHS_MFMA"]
            else:
                os.environ["LQCD_MRHS_MFMA"] = old

    for prec, recon in ((1, 12), (2, 12)):
        pb = PREC_BYTES[prec]
        variants = (False, True) if prec in (2, 3) else (False,)
        # 12 point sources on 24^3x48 (the origin is even: D_oe acts on them)
        dims = (24, 24, 24, 48)
        U = synth.gauge_field(dims, 0.25, 4001)
        # the layout tile: the fastest candidate for 12 sources (ops.tune_tile)
        tile, tile_us = ops.tune_tile(ctx, U, dims, 0.122, 1.0, prec, recon, nrhs=12)
        log("batched %s: layout tile %s (%s)" % (PREC_NAME[prec], tile, ", ".join(
            "%s %.1f us" % ("x".join(map(str, t)), u) for t, u in tile_us.items())))
        o = ops.wilson_clover(ctx, U, dims, 0.122, 1.0, prec, recon, tile=tile)
        srcs = np.stack([synth.point_source(dims, sc // 3, sc % 3) for sc in range(12)])
        reps = [o, o.replica(), o.replica()]
        sets = [(r, r.import_spinor(srcs, 0, nrhs=12), r.spinor(nrhs=12)) for r in reps]
        vh = int(np.prod(dims)) // 2
        byts = vh * (12 * 48 + 8 * recon) * pb
        singles = [(r, r.import_spinor(srcs[0], 0), r.spinor()) for r in reps]
        dt1 = time_rotating(torch, [lambda r=r, i=i, q=q: L.lqcd_dslash(ctx, r.op, q, i, 1) for r, i, q in singles],
                            args.dslash_launches // 2)
        for mf in variants:
            dt = with_mfma(mf, lambda: time_rotating(
                torch, [lambda r=r, i=i, q=q: L.lqcd_dslash(ctx, r.op, q, i, 1, nrhs=12) for r, i, q in sets],
                args.dslash_launches // 2))
            key = "point12_24x48_%s%s" % (PREC_NAME[prec], "_mfma" if mf else "")
            out[key] = {"us": round(dt * 1e6, 1), "GB/s": round(byts / dt / 1e9, 1), "bytes": byts,
                        "us_per_rhs": round(dt * 1e6 / 12, 2), "single_rhs_us": round(dt1 * 1e6, 1),
                        "speedup_vs_sequential": round(12 * dt1 / dt, 2), "tile": list(tile),
                        "tile_candidates_us": {"x".join(map(str, t)): round(u, 1) for t, u in tile_us.items()}}
            log("batched %s%s: 12 point sources %.1f us (%.1f GB/s, x%.2f vs 12 single-source launches)" % (
                PREC_NAME[prec], " mfma" if mf else "", dt * 1e6, byts / dt / 1e9, 12 * dt1 / dt))
        del sets, singles, reps
        # mixed batch, one persistent launch
        jobs, keep, tot_bytes, mixed_tiles = [], [], 0, []
        for k, dims in enumerate(((16, 16, 16, 32), (20, 20, 20, 40), (24, 24, 24, 48))):
            U = synth.gauge_field(dims, 0.25, 4011 + 10 * k)
            t_k, _ = ops.tune_tile(ctx, U, dims, 0.122, 1.0, prec, recon, nrhs=4)
            mixed_tiles.append(list(t_k))
            ok = ops.wilson_clover(ctx, U, dims, 0.122, 1.0, prec, recon, tile=t_k)
            srcs = np.stack([np.where(synth.parity_of_sites(dims)[..., None, None] == 1,
                                      synth.gaussian_spinor(dims, 4012 + 10 * k + r), 0) for r in range(4)])
            i_ = ok.import_spinor(srcs, 1, nrhs=4)
            o_ = ok.spinor(nrhs=4)
            jobs.append((ok.op, o_, i_, 0, 4))
            keep.append((ok, i_, o_))
            tot_bytes += int(np.prod(dims)) // 2 * (4 * 48 + 8 * recon) * pb
        # three buffer sets of the whole batch (links, inputs, outputs)
        jsets = [jobs]
        for _ in range(2):
            js = []
            for ok, i_, o_ in keep[:3]:
                rk = ok.replica()
                i2, o2 = i_.clone(), torch.empty_like(o_)
                js.append((rk.op, o2, i2, 0, 4))
                keep.append((rk, i2, o2))
            jsets.append(js)
        for mf in variants:
            def separate(js):  # the three launches in turn, as a caller without batching would run them
                for j in js:
                    L.lqcd_dslash(ctx, j[0], j[1], j[2], 0, nrhs=4)
            seq = with_mfma(mf, lambda: time_rotating(torch, [lambda js=js: separate(js) for js in jsets], 30))
            dtb = with_mfma(mf, lambda: time_rotating(
                torch, [lambda js=js: L.lqcd_dslash_batch(ctx, js) for js in jsets], args.dslash_launches // 2))
            key = "mixed3x4_%s%s" % (PREC_NAME[prec], "_mfma" if mf else "")
            out[key] = {"us": round(dtb * 1e6, 1), "GB/s": round(tot_bytes / dtb / 1e9, 1), "bytes": tot_bytes,
                        "separate_launches_us": round(seq * 1e6, 1), "tiles": mixed_tiles}
            log("batched %s%s: mixed batch %.1f us (%.1f GB/s; separate launches %.1f us)" % (
                PREC_NAME[prec], " mfma" if mf else "", dtb * 1e6, tot_bytes / dtb / 1e9, seq * 1e6))
        del jsets, jobs, keep
    out["solve_point12_24x48"] = batched_solve(args, torch, L, ops, ctx, tuple(out["point12_24x48_f32"]["tile"]))
    return out


def batched_solve(args, torch, L, ops, ctx, tile):
    """The batched workload's solve: even-odd CGNE for the 12 point sources on
    24^3x48 (kappa 0.122) with FP32 sloppy iterations and FP64 reliable
    updates, all sources in one multi-source solve (each operator application
    one launch over the 12 sources) against 12 single-source solves in
    sequence; a warm-up, then the median of 3 of each. The same with FP16
    sloppy iterations under "fp16_sloppy"."""
    import numpy as np
    import synth
    dims = (24, 24, 24, 48)
    U = synth.gauge_field(dims, 0.25, 4001)
    Ud = torch.from_numpy(U).cuda()
    t = tile  # the layout tile tuned for the FP32 hop with 12 sources
    hi = ops.wilson_clover(ctx, U, dims, 0.122, 1.0, 0, 18, tile=t, U_device=Ud)
    srcs = np.stack([synth.point_source(dims, sc // 3, sc % 3) for sc in range(12)])
    bp = hi.import_spinor(srcs, -1, nrhs=12)
    singles = [hi.import_spinor(srcs[j], -1) for j in range(12)]

    def run(sp):
        lo = ops.wilson_clover(ctx, U, dims, 0.122, 1.0, sp, 12, tile=t, U_device=Ud)

        def batch():
            x = hi.spinor(full=True, nrhs=12)
            prm = ops.cg_params(1e-10, 20000, 0.1, nrhs=12)
            st, info = L.lqcd_cg_solve(ctx, hi.op, lo.op, prm, x, bp)
            assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
            return st, info

        def sequential():
            tot, its, worst = 0.0, [], 0.0
            for bj in singles:
                x = hi.spinor(full=True)
                st, info = L.lqcd_cg_solve(ctx, hi.op, lo.op, ops.cg_params(1e-10, 20000, 0.1), x, bj)
                assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
                tot += info.seconds
                its.append(info.iters)
                worst = max(worst, info.true_residual)
            return tot, its, worst

        med, allt, info = timed_solves(3, batch)
        sequential()
        seq = sorted(sequential() for _ in range(3))[1]
        log("12 point sources on 24^3x48, CGNE %s/FP64: one multi-source solve %.3f s (%d iterations, worst "
            "residual %.2e); 12 single-source solves %.3f s" % (PREC_NAME[sp].upper(), med, info.iters,
                                                                info.true_residual, seq[0]))
        return {"batched_seconds": round(med, 4), "batched_seconds_runs": allt, "batched_iters": info.iters,
                "batched_updates": info.restarts, "batched_worst_true_residual": info.true_residual,
                "sequential_seconds": round(seq[0], 4), "sequential_iters": seq[1],
                "sequential_worst_true_residual": seq[2], "speedup_vs_sequential": round(seq[0] / med, 2)}

    out = run(1)  # FP32 sloppy iterations
    out["fp16_sloppy"] = run(2)
    return out


def main():
    args = parse()
    if args.oracle_solve:
        print(json.dumps(oracle_solve_timing(args.oracle_solve)))
        return
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
    if args.only in ("staggered", "batched"):
        ctx = L.lqcd_context_create()
        fn = staggered_workload if args.only == "staggered" else batched_workload
        res = {args.only: fn(args, torch, L, ops, ctx)}
        if args.kernels_only:
            res["device_copy"] = device_copy(torch, L, ctx)  # calibrates the profiler's byte counters
        print(json.dumps(res))
        L.lqcd_context_destroy(ctx)
        return
    vh = int(np.prod(dims)) // 2
    log("generating fields", dims)
    t = time.time()
    U = synth.gauge_field(dims, eps, 2001)
    b = synth.gaussian_spinor(dims, 2002)
    log("fields ready %.1fs" % (time.time() - t))
    ctx = L.lqcd_context_create()
    Ud = torch.from_numpy(U).cuda()
    if args.only == "learned":
        tile = stencil_tile(dims, block)
        o64 = ops.wilson_clover(ctx, U, dims, kappa, csw, 0, 18, tile=tile, U_device=Ud)
        o32 = ops.wilson_clover(ctx, U, dims, kappa, csw, 1, 12, tile=tile, U_device=Ud)
        o32b = ops.wilson_clover(ctx, U, dims, kappa, csw, 1, 12, tile=block, U_device=Ud)
        res = {"learned": learned_solve(args, torch, L, ops, ctx, o64, o32, o32b, o64.import_spinor(b, -1), block, mr,
                                        dims)}
        if args.kernels_only:
            res["device_copy"] = device_copy(torch, L, ctx)  # calibrates the profiler's byte counters
        print(json.dumps(res))
        L.lqcd_context_destroy(ctx)
        return
    if args.only == "blocks":
        print(json.dumps({"blocks": block_sweep(args, torch, L, ops, ctx, U, Ud, b, dims, kappa, csw, mr)}))
        L.lqcd_context_destroy(ctx)
        return
    if args.only == "solve":
        # the solve alone, for a kernel trace: one warm-up and one timed GCR-DD
        # solve (FP64 restarts, FP32 Krylov, FP16 Schwarz K on 8^4 blocks)
        tile = stencil_tile(dims, block)
        o64 = ops.wilson_clover(ctx, U, dims, kappa, csw, 0, 18, tile=tile, U_device=Ud)
        o32 = ops.wilson_clover(ctx, U, dims, kappa, csw, 1, 12, tile=tile, U_device=Ud)
        o16 = ops.wilson_clover(ctx, U, dims, kappa, csw, 2, K_RECON, tile=block, U_device=Ud)
        bp = o64.import_spinor(b, -1)
        prm = ops.gcr_params(1e-10, k_max=16, delta=1e-3, max_iter=2000, precond=L.LQCD_PRECOND_SCHWARZ,
                             block=block, mr_steps=mr)
        out = []
        for _ in range(2):
            x = o64.spinor(full=True)
            st, info = L.lqcd_gcr_solve(ctx, o64.op, o32.op, o16.op, prm, x, bp)
            assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
            out.append(solve_record(info.seconds, [round(info.seconds, 4)], info))
        print(json.dumps({"solve": out[-1], "warmup": out[0], "device_copy": device_copy(torch, L, ctx),
                          "tuned": L.lqcd_tuned_choices(ctx)}))
        L.lqcd_context_destroy(ctx)
        return
    # Stencil operators use tiles spanning the full x extent (the site order
    # with the least neighbour re-fetch from memory); the FP16 Schwarz operator
    # is tiled by its Dirichlet blocks, and the solver re-lays out K's input
    # and output.
    tile = stencil_tile(dims, block)
    inst = {}
    for prec, recon in [(0, 18), (0, 12), (1, 18), (1, 12), (1, 8), (2, 18), (2, 12), (3, 12), (4, 12)]:
        inst[(prec, recon)] = ops.wilson_clover(ctx, U, dims, kappa, csw, prec, recon, tile=tile, U_device=Ud)
    o16b = ops.wilson_clover(ctx, U, dims, kappa, csw, 2, K_RECON, tile=block, U_device=Ud)
    o16b12 = ops.wilson_clover(ctx, U, dims, kappa, csw, 2, 12, tile=block, U_device=Ud)
    ohb = ops.wilson_clover(ctx, U, dims, kappa, csw, 4, 12, tile=block, U_device=Ud)
    o32b = ops.wilson_clover(ctx, U, dims, kappa, csw, 1, 12, tile=block, U_device=Ud)
    torch.cuda.synchronize()
    log("operators ready (stencil tile %s, Schwarz tile %s)" % (tile, block))

    # ---- kernel table: Wilson dslash and Schur matvec, every precision/recon,
    # each the median over >= args.dslash_launches launches rotating over three
    # buffer sets (links, clover, input and output of their own)
    kernels = {}
    odd_b = np.where(synth.parity_of_sites(dims)[..., None, None] == 1, b, 0)
    for (prec, recon), o in inst.items():
        reps = [o, o.replica(), o.replica()]
        sets = [(r, r.import_spinor(odd_b, 1), r.spinor()) for r in reps]
        dt = time_rotating(torch, [lambda r=r, i=i, q=q: L.lqcd_dslash(ctx, r.op, q, i, 0, 0) for r, i, q in sets],
                           args.dslash_launches)
        byts = vh * (WILSON_REALS[recon] * PREC_BYTES[prec] + (FIXED_NORM_BYTES["dslash"] if prec == 4 else 0))
        kernels["dslash_%s_r%d" % (PREC_NAME[prec], recon)] = {
            "us": round(dt * 1e6, 2), "GB/s": round(byts / dt / 1e9, 1),
            "frac": round(byts / dt / 1e9 / HBM_PEAK_GBS, 4), "bytes": byts}
        esets = [(r, r.import_spinor(b, 0), r.spinor()) for r in reps]
        dts = time_rotating(torch, [lambda r=r, i=i, q=q: L.lqcd_schur_apply(ctx, r.op, q, i) for r, i, q in esets],
                            max(30, args.dslash_launches // 4))
        sb = vh * (SCHUR_REALS[recon] * PREC_BYTES[prec] + (FIXED_NORM_BYTES["schur"] if prec == 4 else 0))
        kernels["schur_%s_r%d" % (PREC_NAME[prec], recon)] = {
            "us": round(dts * 1e6, 2), "GB/s": round(sb / dts / 1e9, 1),
            "frac": round(sb / dts / 1e9 / HBM_PEAK_GBS, 4), "bytes": sb}
        log("%-18s %8.1f us %7.1f GB/s | schur %8.1f us %7.1f GB/s" % (
            "%s r%d" % (PREC_NAME[prec], recon), dt * 1e6, byts / dt / 1e9, dts * 1e6, sb / dts / 1e9))
        del reps, sets, esets
    if args.kernels_only:
        print(json.dumps({"kernels": kernels, "device_copy": device_copy(torch, L, ctx),
                          "tuned": L.lqcd_tuned_choices(ctx), "kernel_sources_sha1": kernel_sources_sha1()}))
        return
    # the same kernel in the Schwarz block tiling, for comparison
    reps = [o32b, o32b.replica(), o32b.replica()]
    sets = [(r, r.import_spinor(odd_b, 1), r.spinor()) for r in reps]
    dt = time_rotating(torch, [lambda r=r, i=i, q=q: L.lqcd_dslash(ctx, r.op, q, i, 0, 0) for r, i, q in sets],
                       args.dslash_launches)
    byts = vh * WILSON_REALS[12] * PREC_BYTES[1]
    kernels["dslash_f32_r12_block_tile"] = {"us": round(dt * 1e6, 2), "GB/s": round(byts / dt / 1e9, 1),
                                            "frac": round(byts / dt / 1e9 / HBM_PEAK_GBS, 4), "bytes": byts}
    log("f32 r12 in %s tiles %8.1f us %7.1f GB/s" % (block, dt * 1e6, byts / dt / 1e9))
    del reps, sets
    # the FP16 Schwarz preconditioner (8 MR steps on the 8^4 blocks) in each of
    # its forms: 0 separate launches per MR step, 1 and 2 one workgroup per
    # block with the block in LDS (x in memory / in registers), 3 and 4 the
    # same with 1024 threads of two sites each instead of 512 of four. Bytes: the
    # block form's algorithmic traffic per even site, r read once, then per MR
    # step the links of both half steps and both clover blocks, x written once
    # (x read and written each step in form 1 adds 96 bytes per step), for
    # 12 and 18 link reals.
    kprm = ops.schwarz_params(block, mr)
    for krec, ko in ((12, o16b12), (18, o16b if K_RECON == 18 else None)):
        if ko is None:
            ko = ops.wilson_clover(ctx, U, dims, kappa, csw, 2, krec, tile=block, U_device=Ud)
        reps = [ko, ko.replica(), ko.replica()]
        ksets = [(r, r.import_spinor(b, 0), r.spinor()) for r in reps]
        k_bytes = vh * (48 + mr * (2 * 8 * 2 * krec + 2 * 144) + 48)
        for form in (0, 1, 2, 3, 4):
            os.environ["LQCD_SCHWARZ_FORM"] = str(form)
            dk = time_rotating(torch, [lambda r=r, i=i, q=q: L.lqcd_schwarz_precond(ctx, r.op, kprm, q, i)
                                       for r, i, q in ksets], 30)
            kernels["schwarz_f16_r%d_form%d" % (krec, form)] = {
                "us": round(dk * 1e6, 2), "GB/s": round(k_bytes / dk / 1e9, 1),
                "frac": round(k_bytes / dk / 1e9 / HBM_PEAK_GBS, 4), "bytes": k_bytes}
            log("Schwarz K (FP16, %d link reals, %d MR steps) form %d: %8.1f us, %7.1f GB/s of the block form's "
                "bytes" % (krec, mr, form, dk * 1e6, k_bytes / dk / 1e9))
        del os.environ["LQCD_SCHWARZ_FORM"]
        del reps, ksets
    del o16b12
    copy = device_copy(torch, L, ctx)
    log("streaming copy %.1f GB/s" % copy["GB/s"])

    o64, o32, o16 = inst[(0, 18)], inst[(1, 12)], o16b
    bp = o64.import_spinor(b, -1)
    prm = ops.gcr_params(1e-10, k_max=16, delta=1e-3, max_iter=2000, precond=L.LQCD_PRECOND_SCHWARZ,
                         block=block, mr_steps=mr)
    hsets = [(r, r.import_spinor(odd_b, 1), r.spinor()) for r in (o32, o32.replica(), o32.replica())]
    esets = [(r, r.import_spinor(b, 0), r.spinor()) for r, _, _ in hsets]
    groups = max(1, -(-args.dslash_launches // 3))

    def step():
        """One pass over the path: the headline dslash (rotating over three
        buffer sets, each group of three launches timed with HIP events), a
        group of Schur matvecs, and one complete GCR-DD solve."""
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(groups + 1)]
        ev[0].record()
        for g in range(groups):
            for r, i, q in hsets:
                L.lqcd_dslash(ctx, r.op, q, i, 0, 0)
            ev[g + 1].record()
        for r, i, q in esets:
            L.lqcd_schur_apply(ctx, r.op, q, i)
        x = o64.spinor(full=True)
        st, info = L.lqcd_gcr_solve(ctx, o64.op, o32.op, o16.op, prm, x, bp)
        assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
        ev[-1].synchronize()
        return [ev[g].elapsed_time(ev[g + 1]) / 1e3 / 3 for g in range(groups)], info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per, infos = [], []
    for _ in range(args.steps):
        p, info = step()
        per += p
        infos.append(info)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dt_head = median_of(per)
    byts = vh * WILSON_REALS[12] * PREC_BYTES[1]
    gbs = byts / dt_head / 1e9
    log("headline dslash in the timed steps: median %.2f us over %d launches, %.1f GB/s" % (
        dt_head * 1e6, 3 * len(per), gbs))
    del hsets, esets

    # ---- time to solution: one warm-up, then the median of args.solves, per solver
    tts = {}

    def gcr(precond_op, p):
        def run():
            x = o64.spinor(full=True)
            st, info = L.lqcd_gcr_solve(ctx, o64.op, o32.op, precond_op, p, x, bp)
            assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
            run.x = x
            return st, info
        return run

    gold = load_oracle_solution()
    run = gcr(o16.op, prm)
    med, allt, info = timed_solves(args.solves, run)
    tts["gcr_dd"] = solve_record(med, allt, info)
    tts["gcr_dd"]["precond_applies"] = info.precond_applies
    if gold is not None:
        tts["gcr_dd"]["rel_error_vs_oracle"] = rel_error_sampled(o64, run.x, gold)
    log("GCR-DD: %d steps, %.3f s (median of %d), true residual %.2e, vs oracle %s" % (
        info.iters, med, args.solves, info.true_residual, tts["gcr_dd"].get("rel_error_vs_oracle")))
    # the same with re-orthogonalised classical Gram-Schmidt (CGS2)
    prm2 = ops.gcr_params(1e-10, k_max=16, delta=1e-3, max_iter=2000, precond=L.LQCD_PRECOND_SCHWARZ,
                          block=block, mr_steps=mr, orth_passes=2)
    med, allt, info = timed_solves(args.solves, gcr(o16.op, prm2))
    tts["gcr_dd_cgs2"] = solve_record(med, allt, info)
    log("GCR-DD with CGS2: %d steps, %.3f s" % (info.iters, med))
    if not args.no_cg:
        def cg():
            x = o64.spinor(full=True)
            st, info = L.lqcd_cg_solve(ctx, o64.op, None, ops.cg_params(1e-10, max_iter=20000), x, bp)
            assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
            cg.x = x
            return st, info
        med, allt, info = timed_solves(args.solves, cg)
        tts["fp64_cg"] = solve_record(med, allt, info)
        if gold is not None:
            tts["fp64_cg"]["rel_error_vs_oracle"] = rel_error_sampled(o64, cg.x, gold)
        log("FP64 CGNE: %d iterations, %.3f s, true residual %.2e" % (info.iters, med, info.true_residual))
        # CGNE with reliable updates: FP32 or FP16 sloppy iterations (recon 12), FP64 updates
        for sp in (1, 2):
            def cg_mixed(lo=inst[(sp, 12)]):
                x = o64.spinor(full=True)
                st, info = L.lqcd_cg_solve(ctx, o64.op, lo.op, ops.cg_params(1e-10, 20000, 0.1), x, bp)
                assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
                return st, info
            med, allt, info = timed_solves(args.solves, cg_mixed)
            tts["cgne_%s_sloppy" % PREC_NAME[sp]] = solve_record(med, allt, info)
            log("CGNE FP64/%s: %d iterations, %d reliable updates, %.3f s, true residual %.2e" % (
                PREC_NAME[sp].upper(), info.iters, info.restarts, med, info.true_residual))
    # GCR-DD with the multiplicative Schwarz K (two block colours), FP16, same blocks
    sap_mr, sap_cycles = 4, 3
    sprm = ops.gcr_params(1e-10, k_max=16, delta=1e-3, max_iter=2000, precond=L.LQCD_PRECOND_SCHWARZ,
                          block=block, mr_steps=sap_mr, cycles=sap_cycles)
    med, allt, info = timed_solves(args.solves, gcr(o16.op, sprm))
    tts["gcr_dd_sap"] = solve_record(med, allt, info)
    tts["gcr_dd_sap"].update({"mr_steps": sap_mr, "cycles": sap_cycles})
    log("GCR-DD with multiplicative Schwarz (%d MR steps, %d cycles): %d steps, %.3f s, true residual %.2e" % (
        sap_mr, sap_cycles, info.iters, med, info.true_residual))
    # the same two solvers with the Schwarz K in 16-bit fixed point (the paper's "half")
    for name, p in (("gcr_dd_half", prm), ("gcr_dd_sap_half", sprm)):
        med, allt, info = timed_solves(args.solves, gcr(ohb.op, p))
        tts[name] = solve_record(med, allt, info)
        log("%s: %d steps, %.3f s, true residual %.2e" % (name, info.iters, med, info.true_residual))
    # mixed-precision BiCGstab (FP64 reliable updates), the paper's baseline for GCR-DD
    for sp in (1, 2):
        def bicg(sp=sp):
            x = o64.spinor(full=True)
            st, info = L.lqcd_bicgstab_solve(ctx, o64.op, inst[(sp, 12)].op, ops.bicgstab_params(1e-10, 5000, 0.1),
                                             x, bp)
            assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
            return st, info
        med, allt, info = timed_solves(args.solves, bicg)
        name = "bicgstab_%s" % PREC_NAME[sp]
        tts[name] = solve_record(med, allt, info)
        log("BiCGstab FP64/%s: %d steps, %d reliable updates, %.3f s, true residual %.2e" % (
            PREC_NAME[sp].upper(), info.iters, info.restarts, med, info.true_residual))
    if os.path.exists(args.learned):
        tts.update(learned_solve(args, torch, L, ops, ctx, o64, o32, o32b, bp, block, mr, dims))
    if "fp64_cg" in tts:
        ref = tts["fp64_cg"]["seconds"]
        tts["speedup_vs_fp64_cg"] = {k: round(ref / v["seconds"], 2) for k, v in tts.items()
                                     if isinstance(v, dict) and "seconds" in v and k != "fp64_cg"}
    tts["smallest_8x4_fp64_cgne"] = smallest_workload(args, torch, L, ops, ctx)
    res = {
        "metric": METRIC, "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "wilson-clover %s, kappa %.3f, c_sw %.1f, eps %.2f, antiperiodic t; GCR-DD "
                               "FP64/FP32/FP16, Schwarz 8^4 blocks (FP16, %d link reals), %d MR steps" % (
                                   "x".join(map(str, dims)), kappa, csw, eps, K_RECON, mr),
                   "dims": list(dims), "tile": list(tile), "schwarz_tile": list(block),
                   "kernel": "wilson dslash f32 recon12, one parity",
                   "dslash_launches_per_step": 3 * groups, "buffer_sets": 3,
                   "timing": "median over groups of 3 launches (one per buffer set)"},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": (PROFILED_TRAFFIC["bytes_per_launch"]
                                 if kernel_sources_sha1() == PROFILED_TRAFFIC["sources_sha1"] else None),
                     "traffic_unit": "bytes per launch", "algorithmic_bytes_per_launch": byts,
                     "median_launch_us": round(dt_head * 1e6, 2),
                     "frac_of_streaming_copy": round(gbs / copy["GB/s"], 4)},
        "time_to_solution": tts,
        "device_copy": copy,
        "kernels": kernels,
    }
    if not args.no_staggered:
        res["staggered"] = staggered_workload(args, torch, L, ops, ctx)
    if not args.no_batched:
        res["batched"] = batched_workload(args, torch, L, ops, ctx)
    res["tuned"] = L.lqcd_tuned_choices(ctx)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        res["cpu_baseline"] = cpu_baseline(dims, U, b, kappa, csw)
    torch.cuda.synchronize()
    L.lqcd_context_destroy(ctx)
    print(json.dumps(res))


def block_sweep(args, torch, L, ops, ctx, U, Ud, b, dims, kappa, csw, mr):
    """GCR-DD with the additive FP16 Schwarz K on blocks from 4^4 (128 sites
    per parity) to 32x16^3 (65,536), 8 MR steps: one K application (median
    over rotated launches of one buffer set), GCR steps and time to solution
    (the median of 3 solves after the tuning ones), and the form of K the
    autotuner chose (2, 1: block in LDS; 0: separate launches)."""
    import numpy as np
    tile = stencil_tile(dims, (8, 8, 8, 8))
    o64 = ops.wilson_clover(ctx, U, dims, kappa, csw, 0, 18, tile=tile, U_device=Ud)
    o32 = ops.wilson_clover(ctx, U, dims, kappa, csw, 1, 12, tile=tile, U_device=Ud)
    bp = o64.import_spinor(b, -1)
    rows = []
    for block in [(4, 4, 4, 4), (8, 4, 4, 4), (8, 8, 4, 4), (8, 8, 8, 4), (8, 8, 8, 8), (16, 8, 8, 8),
                  (16, 16, 8, 8), (16, 16, 16, 16), (32, 16, 16, 16)]:
        if any(d % e for d, e in zip(dims, block)):
            continue
        ok = ops.wilson_clover(ctx, U, dims, kappa, csw, 2, 12, tile=block, U_device=Ud)
        inp, out = ok.import_spinor(b, 0), ok.spinor()
        kp = ops.schwarz_params(block, mr)
        dk = time_rotating(torch, [lambda: L.lqcd_schwarz_precond(ctx, ok.op, kp, out, inp)], 20)
        prm = ops.gcr_params(1e-10, k_max=16, delta=1e-3, max_iter=3000, precond=L.LQCD_PRECOND_SCHWARZ,
                             block=block, mr_steps=mr)

        def run():
            x = o64.spinor(full=True)
            st, info = L.lqcd_gcr_solve(ctx, o64.op, o32.op, ok.op, prm, x, bp)
            assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
            return st, info
        med, allt, info = timed_solves(3, run)
        form = [v for k, v in L.lqcd_tuned_choices(ctx).items()
                if k.startswith("schwarz") and "/%dx%dx%dx%d" % block in k]
        rows.append({"block": list(block), "sites_per_parity": int(np.prod(block)) // 2, "K_us": round(dk * 1e6, 1),
                     "steps": info.iters, "seconds": round(med, 4), "K_form": form[0] if form else 0})
        log("blocks %s: K %.1f us, %d steps, %.4f s" % (block, dk * 1e6, info.iters, med))
        del ok, inp, out
    return rows


def load_oracle_solution():
    """The oracle's FP64 solution of the default workload at 2048 sampled sites
    (written by tests/golden/make_wilson_solution_32x64.py), or None."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "wilson_solution_32x64_sites.npz")
    return np.load(path) if os.path.exists(path) else None


def rel_error_sampled(o64, x, gold):
    """||x - x_ora|| / ||x_ora|| over the sampled sites of the stored oracle solution."""
    import numpy as np
    xs = o64.export_spinor(x, -1).cpu().numpy().reshape(-1, 4, 3)[gold["sites"]]
    return float(np.linalg.norm(xs - gold["x"]) / np.linalg.norm(gold["x"]))


def smallest_workload(args, torch, L, ops, ctx):
    """8^4 Wilson-clover (kappa 0.12, c_sw 1, eps 0.25, seeds 1001/1002): FP64
    even-odd CGNE to 1e-10 on the GPU (a warm-up, then the median of
    args.solves). Latency-bound (2048 even sites), not a bandwidth datum."""
    import synth
    dims = (8, 8, 8, 8)
    U = synth.gauge_field(dims, 0.25, 1001)
    b = synth.gaussian_spinor(dims, 1002)
    o = ops.wilson_clover(ctx, U, dims, 0.12, 1.0, 0, 18)
    bp = o.import_spinor(b, -1)

    def run():
        x = o.spinor(full=True)
        st, info = L.lqcd_cg_solve(ctx, o.op, None, ops.cg_params(1e-10, 20000), x, bp)
        assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
        return st, info
    med, allt, info = timed_solves(args.solves, run)
    log("8^4 FP64 CGNE: %d iterations, %.4f s" % (info.iters, med))
    return solve_record(med, allt, info)


if __name__ == "__main__":
    main()
