"""Parity at the full workload sizes, in the launch configuration the
benchmark times: dslash outputs at sampled sites against the oracle computed
site by site, and complete solves whose FP64 residual the oracle recomputes on
the host over the whole lattice.

32^3x64 Wilson-clover (kappa 0.124, c_sw 1, eps 0.25, seeds 2001/2002) and
48^3x96 improved staggered (m 0.01, eps 0.2, seeds 3001/3002/3003)."""
import sys
import time

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import TOL, check, ctx, np_of  # noqa: F401

pytestmark = [pytest.mark.gpu, pytest.mark.fullsize]

L = pytest.importorskip("paper_1109_2935_amd.lqcd")
from paper_1109_2935_amd import ops  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


_W = {}


def wilson_fields():
    if "w" not in _W:
        dims = (32, 32, 32, 64)
        t = time.time()
        U = synth.gauge_field(dims, 0.25, 2001)
        b = synth.gaussian_spinor(dims, 2002)
        say("32^3x64 fields %.1fs" % (time.time() - t))
        _W["w"] = (dims, U, b, torch.from_numpy(U).cuda())
    return _W["w"]


def sample_sites(dims, parity, n, seed):
    rng = np.random.default_rng(seed)
    V = int(np.prod(dims))
    cand = rng.choice(V, size=4 * n, replace=False)
    x = cand % dims[0]
    y = (cand // dims[0]) % dims[1]
    z = (cand // (dims[0] * dims[1])) % dims[2]
    t = cand // (dims[0] * dims[1] * dims[2])
    keep = cand[((x + y + z + t) % 2) == parity]
    return np.sort(keep[:n])


# the benchmark's tilings: stencil operators span the full x and y extents
# (4 sites along z and t), the FP16 Schwarz operator is tiled by its 8^4
# Dirichlet blocks
STENCIL_TILE, BLOCK = (32, 32, 4, 4), (8, 8, 8, 8)


@pytest.mark.parametrize("prec,recon,tile", [(1, 12, STENCIL_TILE), (2, 12, STENCIL_TILE), (3, 12, STENCIL_TILE),
                                             (1, 8, STENCIL_TILE), (1, 18, STENCIL_TILE), (0, 18, STENCIL_TILE),
                                             (0, 12, STENCIL_TILE), (1, 12, BLOCK), (2, 12, BLOCK)])
def test_wilson_dslash_sampled_sites_32x64(ctx, prec, recon, tile):
    dims, U, b, Ud = wilson_fields()
    o = ops.wilson_clover(ctx, U, dims, 0.124, 1.0, prec, recon, tile=tile, U_device=Ud)
    src = np.where(oracle.parity_mask(dims, 1)[..., None, None], b, 0)
    out = o.spinor()
    L.lqcd_dslash(ctx, o.op, out, o.import_spinor(src, 1), 0)
    got = np_of(o.export_spinor(out, 0)).reshape(-1, 4, 3)
    sites = sample_sites(dims, 0, 256, 7)
    ref = oracle.wilson_dslash(dims, U, src, bc_t=-1, sites=sites)
    check(got[sites], ref, TOL[prec])


def neighbours(dims, sites):
    """The 8 nearest neighbours (natural index) of each site."""
    lx, ly, lz, lt = dims
    x, y, z, t = sites % lx, (sites // lx) % ly, (sites // (lx * ly)) % lz, sites // (lx * ly * lz)
    out = []
    for d in (1, -1):
        out += [(x + d) % lx + lx * (y + ly * (z + lz * t)), x + lx * ((y + d) % ly + ly * (z + lz * t)),
                x + lx * (y + ly * ((z + d) % lz + lz * t)), x + lx * (y + ly * (z + lz * ((t + d) % lt)))]
    return np.unique(np.concatenate(out))


@pytest.mark.parametrize("prec,recon", [(1, 12), (2, 12), (0, 18)])
def test_schur_sampled_sites_32x64(ctx, prec, recon):
    """Mhat x_e = A_ee x_e - kappa^2 D_eo A_oo^-1 D_oe x_e at sampled even
    sites, the two fused kernels the solvers use, in the stencil tiling. The
    oracle forms D_oe x_e only at the sampled sites' odd neighbours."""
    dims, U, b, Ud = wilson_fields()
    o = ops.wilson_clover(ctx, U, dims, 0.124, 1.0, prec, recon, tile=STENCIL_TILE, U_device=Ud)
    even = oracle.parity_mask(dims, 0)
    src = np.where(even[..., None, None], b, 0)
    out = o.spinor()
    L.lqcd_schur_apply(ctx, o.op, out, o.import_spinor(src, 0))
    got = np_of(o.export_spinor(out, 0)).reshape(-1, 4, 3)
    M = schur_oracle()
    sites = sample_sites(dims, 0, 128, 17)
    nb = neighbours(dims, sites)
    V = int(np.prod(dims))
    t = np.zeros((V, 4, 3), complex)
    t[nb] = oracle.wilson_dslash(dims, U, src, bc_t=-1, sites=nb)
    t = oracle.clover_apply(dims, M.Ainv, t.reshape(src.shape), parity=1)
    y = oracle.clover_apply(dims, M.A, src, parity=0).reshape(V, 4, 3)[sites]
    ref = y - 0.124 ** 2 * oracle.wilson_dslash(dims, U, t, bc_t=-1, sites=sites)
    check(got[sites], ref, TOL[prec])


def schur_oracle():
    if "M" not in _W:
        dims, U, _, _ = wilson_fields()
        _W["M"] = oracle.WilsonClover(dims, U, 0.124, 1.0, bc_t=-1)
    return _W["M"]


def schwarz_oracle_32x64():
    """The oracle's FP64 additive Schwarz K (8^4 blocks, 8 MR steps) of the
    benchmark's even source over the whole lattice."""
    if "K" not in _W:
        from oracle import solvers
        dims, U, b, _ = wilson_fields()
        src = np.where(oracle.parity_mask(dims, 0)[..., None, None], b, 0)
        t = time.time()
        _W["K"] = (src, solvers.schwarz(schur_oracle(), src, BLOCK, 8))
        say("oracle Schwarz K at 32^3x64 %.1fs" % (time.time() - t))
    return _W["K"]


@pytest.mark.parametrize("form", [0, 1, 2])
def test_schwarz_k_full_32x64(ctx, monkeypatch, form):
    """The FP16 Schwarz preconditioner of the benchmark's GCR-DD (8^4 blocks
    as the tiles, 8 MR steps) over the whole 32^3x64 even field, in each form
    (0 separate launches; 1, 2 one workgroup per block with the block in LDS),
    against the oracle's FP64 K, to the derived bound of the 16-bit K (5e-3,
    whole field and worst site)."""
    dims, U, b, Ud = wilson_fields()
    src, ref = schwarz_oracle_32x64()
    monkeypatch.setenv("LQCD_SCHWARZ_FORM", str(form))
    o = ops.wilson_clover(ctx, U, dims, 0.124, 1.0, 2, 12, tile=BLOCK, U_device=Ud)
    out = o.spinor()
    L.lqcd_schwarz_precond(ctx, o.op, ops.schwarz_params(BLOCK, 8), out, o.import_spinor(src, 0))
    check(np_of(o.export_spinor(out, 0)), ref, 5e-3, "form %d" % form)


def test_gcr_dd_exact_solution_32x64(ctx):
    """A system with a known solution: x* Gaussian (seed 2003), b = M x*
    formed by the oracle. The benchmark's GCR-DD (FP64 restarts, FP32 Krylov,
    FP16 Schwarz on 8^4 blocks, 8 MR steps) to 1e-10 must recover x* to
    ||x - x*|| / ||x*|| <= 1e-8."""
    dims, U, _, Ud = wilson_fields()
    M = schur_oracle()
    xstar = synth.gaussian_spinor(dims, 2003)
    b = M.M(xstar)
    o = {p: ops.wilson_clover(ctx, U, dims, 0.124, 1.0, p, r, tile=STENCIL_TILE if p < 2 else BLOCK, U_device=Ud)
         for p, r in ((0, 18), (1, 12), (2, 12))}
    x = o[0].spinor(full=True)
    prm = ops.gcr_params(1e-10, 16, 1e-3, max_iter=2000, precond=L.LQCD_PRECOND_SCHWARZ, block=BLOCK, mr_steps=8)
    st, info = L.lqcd_gcr_solve(ctx, o[0].op, o[1].op, o[2].op, prm, x, o[0].import_spinor(b, -1))
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    xs = np_of(o[0].export_spinor(x, -1))
    err = np.linalg.norm(xs - xstar) / np.linalg.norm(xstar)
    res = np.linalg.norm(b - M.M(xs)) / np.linalg.norm(b)
    say("exact-solution system: GCR-DD %d steps, ||x - x*||/||x*|| %.3e, oracle residual %.3e" % (info.iters, err, res))
    assert res <= 1.05e-10
    assert err <= 1e-8


def test_gcr_dd_against_oracle_solution_32x64(ctx):
    """The benchmark's GCR-DD solve of the Gaussian-source system against the
    oracle's FP64 CGNE solution to 1e-12 (stored at 2048 sampled sites by
    tests/golden/make_wilson_solution_32x64.py, which calls only the oracle):
    ||x - x_ora|| / ||x_ora|| over those sites <= 1e-8."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "wilson_solution_32x64_sites.npz")
    gold = np.load(path)
    dims, U, b, Ud = wilson_fields()
    o = {p: ops.wilson_clover(ctx, U, dims, 0.124, 1.0, p, r, tile=STENCIL_TILE if p < 2 else BLOCK, U_device=Ud)
         for p, r in ((0, 18), (1, 12), (2, 12))}
    x = o[0].spinor(full=True)
    prm = ops.gcr_params(1e-10, 16, 1e-3, max_iter=2000, precond=L.LQCD_PRECOND_SCHWARZ, block=BLOCK, mr_steps=8)
    st, info = L.lqcd_gcr_solve(ctx, o[0].op, o[1].op, o[2].op, prm, x, o[0].import_spinor(b, -1))
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    xs = np_of(o[0].export_spinor(x, -1)).reshape(-1, 4, 3)[gold["sites"]]
    err = np.linalg.norm(xs - gold["x"]) / np.linalg.norm(gold["x"])
    say("GCR-DD vs oracle CGNE solution (%d sites): %.3e" % (len(gold["sites"]), err))
    assert err <= 1e-8


def test_fgcr_shipped_network_32x64(ctx):
    """Flexible GCR with the shipped trained network as K (Schwarz fallback),
    FP64 restarts, FP32 Krylov, on the benchmark's system; the oracle
    recomputes ||b - M x|| / ||b|| <= 1e-10, and the network needs fewer
    steps than GCR without a preconditioner."""
    import os
    from paper_1109_2935_amd import ptc
    dims, U, b, Ud = wilson_fields()
    o64 = ops.wilson_clover(ctx, U, dims, 0.124, 1.0, 0, 18, tile=STENCIL_TILE, U_device=Ud)
    o32 = ops.wilson_clover(ctx, U, dims, 0.124, 1.0, 1, 12, tile=STENCIL_TILE, U_device=Ud)
    o32b = ops.wilson_clover(ctx, U, dims, 0.124, 1.0, 1, 12, tile=BLOCK, U_device=Ud)
    net = ptc.Network(ctx)
    net.load(os.path.join(os.path.dirname(ptc.__file__), "data", "ptc_16x4.npz"))
    import ctypes
    prm = ops.gcr_params(1e-10, 16, 1e-3, max_iter=2000, precond=L.LQCD_PRECOND_LEARNED, block=BLOCK, mr_steps=8)
    prm.learned = ctypes.pointer(net.net)
    bp = o64.import_spinor(b, -1)
    x = o64.spinor(full=True)
    st, info = L.lqcd_gcr_solve(ctx, o64.op, o32.op, o32b.op, prm, x, bp)
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    xs = np_of(o64.export_spinor(x, -1))
    res = np.linalg.norm(b - schur_oracle().M(xs)) / np.linalg.norm(b)
    x0 = o64.spinor(full=True)
    st0, i0 = L.lqcd_gcr_solve(ctx, o64.op, o32.op, None, ops.gcr_params(1e-10, 16, 1e-3, max_iter=5000), x0, bp)
    assert st0 == L.LQCD_OK
    say("FGCR(network) %d steps (%d fallback) %.3fs, oracle residual %.3e; GCR %d steps" % (
        info.iters, info.fallback_applies, info.seconds, res, i0.iters))
    assert res <= 1.05e-10
    assert info.iters < i0.iters


def test_staggered_dslash_sampled_sites_48x96(ctx):
    """Staggered hopping term (fat and 3-hop long links, FP32, long links in
    12 reals, the benchmark's configuration) at sampled sites."""
    dims = (48, 48, 48, 96)
    U, fat, chi, lng = staggered_fields()
    hi = ops.staggered(ctx, fat, U, dims, 0.01, 1, 12)
    src = np.where(oracle.parity_mask(dims, 1)[..., None], chi, 0)
    out = hi.spinor()
    L.lqcd_dslash(ctx, hi.op, out, hi.import_spinor(src, 1), 0)
    got = np_of(hi.export_spinor(out, 0)).reshape(-1, 3)
    sites = sample_sites(dims, 0, 256, 9)
    ref = oracle.stag_dslash(dims, fat, lng, src, bc_t=-1, sites=sites)
    check(got[sites], ref.reshape(-1, 3), TOL[1])


def staggered_fields():
    if "s" not in _W:
        dims = (48, 48, 48, 96)
        t = time.time()
        U = synth.gauge_field(dims, 0.2, 3001)
        fat = synth.fat_links(dims, U, seed=3003)
        chi = synth.gaussian_spinor(dims, 3002, inner=(3,))
        lng = oracle.long_links(dims, U)
        say("48^3x96 fields %.1fs" % (time.time() - t))
        _W["s"] = (U, fat, chi, lng)
    return _W["s"]


def full_x_tile(dims):
    return (dims[0],) + tuple(next(e for e in (8, 6, 4, 2) if d % e == 0) for d in dims[1:])


@pytest.mark.parametrize("prec", [1, 2])
def test_batched_full_size_in_bench_tiles(ctx, prec):
    """The benchmark's batched workloads in its full-x tiles: 12 point sources
    on 24^3x48 in one launch, and one persistent launch over 16^3x32, 20^3x40 and
    24^3x48 with 4 Gaussian sources each (kappa 0.122). Each equals the
    single-operator launch bit for bit, and sampled sites match the oracle."""
    dims = (24, 24, 24, 48)
    U = synth.gauge_field(dims, 0.25, 4001)
    o = ops.wilson_clover(ctx, U, dims, 0.122, 1.0, prec, 12, tile=full_x_tile(dims))
    srcs = np.stack([synth.point_source(dims, sc // 3, sc % 3) for sc in range(12)])
    out = o.spinor(nrhs=12)
    L.lqcd_dslash(ctx, o.op, out, o.import_spinor(srcs, 0, nrhs=12), 1, nrhs=12)
    got = np_of(o.export_spinor(out, 1, nrhs=12)).reshape(12, -1, 4, 3)
    # a point source at the origin reaches its 8 odd neighbours only
    nb = neighbours(dims, np.array([0]))
    for sc in (0, 5, 11):
        ref = oracle.wilson_dslash(dims, U, srcs[sc], bc_t=-1, sites=nb)
        check(got[sc][nb], ref, TOL[prec], "point source %d" % sc)
        assert np.abs(np.delete(got[sc], nb, axis=0)).max() == 0
    jobs, keep = [], []
    for k, d in enumerate(((16, 16, 16, 32), (20, 20, 20, 40), (24, 24, 24, 48))):
        Uk = synth.gauge_field(d, 0.25, 4011 + 10 * k)
        ok = ops.wilson_clover(ctx, Uk, d, 0.122, 1.0, prec, 12, tile=full_x_tile(d))
        odd = oracle.parity_mask(d, 1)
        sk = np.stack([np.where(odd[..., None, None], synth.gaussian_spinor(d, 4012 + 10 * k + r), 0)
                       for r in range(4)])
        i_ = ok.import_spinor(sk, 1, nrhs=4)
        o_ = ok.spinor(nrhs=4)
        single = ok.spinor(nrhs=4)
        L.lqcd_dslash(ctx, ok.op, single, i_, 0, nrhs=4)
        jobs.append((ok.op, o_, i_, 0, 4))
        keep.append((ok, o_, single, sk, Uk, d))
    L.lqcd_dslash_batch(ctx, jobs)
    torch.cuda.synchronize()
    for ok, o_, single, sk, Uk, d in keep:
        assert torch.equal(o_, single)
        g = np_of(ok.export_spinor(o_, 0, nrhs=4)).reshape(4, -1, 4, 3)
        sites = sample_sites(d, 0, 64, 5)
        for r in (0, 3):
            check(g[r][sites], oracle.wilson_dslash(d, Uk, sk[r], bc_t=-1, sites=sites), TOL[prec], "rhs %d" % r)


def test_multi_source_cg_point_sources_24x48(ctx):
    """The batched workload's solve: CGNE for the 12 point sources on 24^3x48
    (kappa 0.122) in one multi-source solve, FP32 sloppy iterations with FP64
    reliable updates; the oracle recomputes three sources' residuals."""
    dims = (24, 24, 24, 48)
    U = synth.gauge_field(dims, 0.25, 4001)
    Ud = torch.from_numpy(U).cuda()
    t = full_x_tile(dims)
    hi = ops.wilson_clover(ctx, U, dims, 0.122, 1.0, 0, 18, tile=t, U_device=Ud)
    lo = ops.wilson_clover(ctx, U, dims, 0.122, 1.0, 1, 12, tile=t, U_device=Ud)
    srcs = np.stack([synth.point_source(dims, sc // 3, sc % 3) for sc in range(12)])
    bp = hi.import_spinor(srcs, -1, nrhs=12)
    x = hi.spinor(full=True, nrhs=12)
    prm = ops.cg_params(1e-10, 20000, 0.1, nrhs=12)
    st, info = L.lqcd_cg_solve(ctx, hi.op, lo.op, prm, x, bp)
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    say("12-source CGNE: %d iterations, %d updates, %.3fs" % (info.iters, info.restarts, info.seconds))
    xs = np_of(hi.export_spinor(x, -1, nrhs=12))
    M = oracle.WilsonClover(dims, U, 0.122, 1.0, bc_t=-1)
    for sc in (0, 7, 11):
        res = np.linalg.norm(srcs[sc] - M.M(xs[sc])) / np.linalg.norm(srcs[sc])
        say("source %d: oracle residual %.3e" % (sc, res))
        assert res <= 1.05e-10


def test_gcr_dd_full_32x64(ctx):
    """The benchmark's solve: FP64 restarts, FP32 Krylov, FP16 Schwarz on 8^4
    blocks (its own tiling), 8 MR steps; the oracle recomputes ||b - M x|| / ||b||
    in FP64."""
    dims, U, b, Ud = wilson_fields()
    o = {p: ops.wilson_clover(ctx, U, dims, 0.124, 1.0, p, r, tile=STENCIL_TILE if p < 2 else BLOCK, U_device=Ud)
         for p, r in ((0, 18), (1, 12), (2, 12))}
    bp = o[0].import_spinor(b, -1)
    x = o[0].spinor(full=True)
    prm = ops.gcr_params(1e-10, 16, 1e-3, max_iter=2000, precond=L.LQCD_PRECOND_SCHWARZ, block=(8, 8, 8, 8), mr_steps=8)
    st, info = L.lqcd_gcr_solve(ctx, o[0].op, o[1].op, o[2].op, prm, x, bp)
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    say("GCR-DD %d steps %.3fs" % (info.iters, info.seconds))
    xs = np_of(o[0].export_spinor(x, -1))
    t = time.time()
    M = oracle.WilsonClover(dims, U, 0.124, 1.0, bc_t=-1)
    res = np.linalg.norm(b - M.M(xs)) / np.linalg.norm(b)
    say("oracle residual %.3e (%.1fs)" % (res, time.time() - t))
    assert res <= 1.05e-10


def test_gcr_dd_sap_full_32x64(ctx):
    """GCR-DD with the multiplicative Schwarz K (FP16, 8^4 blocks, one cycle
    over the two colours, 4 MR steps per visit); the oracle recomputes the
    residual."""
    dims, U, b, Ud = wilson_fields()
    o = {p: ops.wilson_clover(ctx, U, dims, 0.124, 1.0, p, r, tile=STENCIL_TILE if p < 2 else BLOCK, U_device=Ud)
         for p, r in ((0, 18), (1, 12), (2, 12))}
    x = o[0].spinor(full=True)
    prm = ops.gcr_params(1e-10, 16, 1e-3, max_iter=2000, precond=L.LQCD_PRECOND_SCHWARZ, block=BLOCK, mr_steps=4,
                         cycles=1)
    st, info = L.lqcd_gcr_solve(ctx, o[0].op, o[1].op, o[2].op, prm, x, o[0].import_spinor(b, -1))
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    say("GCR-DD (SAP) %d steps %.3fs" % (info.iters, info.seconds))
    xs = np_of(o[0].export_spinor(x, -1))
    M = oracle.WilsonClover(dims, U, 0.124, 1.0, bc_t=-1)
    res = np.linalg.norm(b - M.M(xs)) / np.linalg.norm(b)
    say("oracle residual %.3e" % res)
    assert res <= 1.05e-10


@pytest.mark.parametrize("sprec", [1, 2])
def test_bicgstab_full_32x64(ctx, sprec):
    """Mixed-precision BiCGstab on the same system: FP32 or FP16 sloppy
    iterations (recon 12, the stencil tiling), FP64 reliable updates; the
    oracle recomputes ||b - M x|| / ||b|| in FP64."""
    dims, U, b, Ud = wilson_fields()
    o = {p: ops.wilson_clover(ctx, U, dims, 0.124, 1.0, p, r, tile=STENCIL_TILE, U_device=Ud)
         for p, r in ((0, 18), (sprec, 12))}
    x = o[0].spinor(full=True)
    st, info = L.lqcd_bicgstab_solve(ctx, o[0].op, o[sprec].op, ops.bicgstab_params(1e-10, 5000, 0.1), x,
                                     o[0].import_spinor(b, -1))
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    say("BiCGstab sloppy %d: %d steps %d updates %.3fs" % (sprec, info.iters, info.restarts, info.seconds))
    xs = np_of(o[0].export_spinor(x, -1))
    M = oracle.WilsonClover(dims, U, 0.124, 1.0, bc_t=-1)
    res = np.linalg.norm(b - M.M(xs)) / np.linalg.norm(b)
    say("oracle residual %.3e" % res)
    assert res <= 1.05e-10


def test_staggered_cg_full_48x96(ctx):
    """Reliable-update CG on N_e = m^2 - D_eo D_oe/4, FP32 sloppy, FP64 updates,
    to 1e-10; the oracle recomputes the residual over all even sites."""
    dims, mass = (48, 48, 48, 96), 0.01
    t = time.time()
    U = synth.gauge_field(dims, 0.2, 3001)
    fat = synth.fat_links(dims, U, seed=3003)
    chi = synth.gaussian_spinor(dims, 3002, inner=(3,))
    say("48^3x96 fields %.1fs" % (time.time() - t))
    Ud, Fd = torch.from_numpy(U).cuda(), torch.from_numpy(fat).cuda()
    hi = ops.staggered(ctx, fat, U, dims, mass, 0, 18, U_device=Ud, fat_device=Fd)
    lo = ops.staggered(ctx, fat, U, dims, mass, 1, 12, U_device=Ud, fat_device=Fd)
    del Ud, Fd
    even = oracle.parity_mask(dims, 0)
    b = np.where(even[..., None], chi, 0)
    bp = hi.import_spinor(b, 0)
    x = hi.spinor()
    st, info = L.lqcd_cg_solve(ctx, hi.op, lo.op, ops.cg_params(1e-10, 20000, 0.1, L.LQCD_CG_STAG_NORMAL), x, bp)
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    say("staggered CG %d iterations %d updates %.3fs" % (info.iters, info.restarts, info.seconds))
    xs = np_of(hi.export_spinor(x, 0))
    t = time.time()
    lng = oracle.long_links(dims, U)
    op = oracle.Staggered(dims, fat, lng, mass)
    res = np.linalg.norm(b - op.normal_even(xs)) / np.linalg.norm(b)
    say("oracle residual %.3e (%.1fs)" % (res, time.time() - t))
    assert res <= 1.05e-10


def test_staggered_multishift_full_48x96(ctx):
    """Eq. (4) with three shifts at the benchmark's size: FP32 multi-shift
    stage, FP64-verified refinements; the oracle recomputes each shifted
    system's residual over all even sites."""
    dims, mass = (48, 48, 48, 96), 0.01
    U = synth.gauge_field(dims, 0.2, 3001)
    fat = synth.fat_links(dims, U, seed=3003)
    chi = synth.gaussian_spinor(dims, 3002, inner=(3,))
    Ud, Fd = torch.from_numpy(U).cuda(), torch.from_numpy(fat).cuda()
    hi = ops.staggered(ctx, fat, U, dims, mass, 0, 18, U_device=Ud, fat_device=Fd)
    lo = ops.staggered(ctx, fat, U, dims, mass, 1, 12, U_device=Ud, fat_device=Fd)
    del Ud, Fd
    even = oracle.parity_mask(dims, 0)
    b = np.where(even[..., None], chi, 0)
    bp = hi.import_spinor(b, 0)
    shifts = (0.0, 1e-3, 0.1)
    xs = [hi.spinor() for _ in shifts]
    st, info = L.lqcd_multishift_cg_solve(ctx, hi.op, lo.op, ops.multishift_params(shifts), xs, bp)
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    say("multi-shift %d it, refinements %s, %.3fs" % (info.ms_iters, [info.shift[i].iters for i in range(3)],
                                                       info.seconds))
    op = oracle.Staggered(dims, fat, oracle.long_links(dims, U), mass)
    bn = np.linalg.norm(b)
    for i, s in enumerate(shifts):
        x = np_of(hi.export_spinor(xs[i], 0))
        res = np.linalg.norm(b - op.normal_even(x) - s * np.where(even[..., None], x, 0)) / bn
        say("shift %g: oracle residual %.3e" % (s, res))
        assert res <= 1.05e-10
