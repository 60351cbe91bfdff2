"""Train the learned (PTC) preconditioner on residual -> error pairs that the
FP64 even-odd CGNE solver produces on a synthetic Wilson-clover field.

Defaults: 16^4 lattice, links exp(i eps H) with eps = 0.25 (seed 5001),
kappa = 0.124, c_sw = 1, Gaussian sources (seeds 5100 + j), every CGNE
iterate recorded up to 100 per source, sources added until 20,000 pairs,
streamed (each pair is generated on the GPU, used for one Adam step and
dropped). --objective residual trains on |Mhat N(r) - r|^2 / |r|^2, which
makes the network a much better preconditioner than the error objective
|N(r) - e|^2 / |e|^2 (the shipped weights use it).

    python -m paper_1109_2935_amd.train_ptc --out ptc_weights.npz
"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", default="16,16,16,16")
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--per-source", type=int, default=100)
    ap.add_argument("--every", type=int, default=1)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-end", type=float, default=2e-4, help="geometric decay of the step size to this value")
    ap.add_argument("--init", default=None, help="start from these weights (.npz written by Network.save)")
    ap.add_argument("--seed0", type=int, default=5100, help="seed of the first training source")
    ap.add_argument("--fields", type=int, default=1, help="number of gauge fields the sources are spread over")
    ap.add_argument("--objective", default="residual", choices=("error", "residual"),
                    help="error: |N r - e|^2/|e|^2; residual: |Mhat N r - r|^2/|r|^2")
    ap.add_argument("--kappa", type=float, default=0.124)
    ap.add_argument("--seed", type=int, default=5001)
    ap.add_argument("--out", default="ptc_weights.npz")
    a = ap.parse_args(argv)
    import numpy as np
    import torch

    import synth
    from paper_1109_2935_amd import lqcd as L
    from paper_1109_2935_amd import ops, ptc

    dims = tuple(int(v) for v in a.dims.split(","))
    ctx = L.lqcd_context_create()
    net = ptc.Network(ctx, ptc.CHANNELS, seed=a.seed + 1)
    if a.init:
        net.load(a.init)
    lr_end = a.lr if a.lr_end is None else a.lr_end
    t0 = time.time()
    losses = []
    # the pairs are split evenly over `fields` gauge fields (seeds seed, seed + 1,
    # ...); the step size decays over all of them
    for f in range(a.fields):
        n_f = a.pairs // a.fields + (1 if f < a.pairs % a.fields else 0)
        if n_f == 0:
            continue
        U = synth.gauge_field(dims, 0.25, a.seed + f)
        Ud = torch.from_numpy(U).cuda()
        op64 = ops.wilson_clover(ctx, U, dims, a.kappa, 1.0, L.LQCD_F64, 18, U_device=Ud)
        op32 = ops.wilson_clover(ctx, U, dims, a.kappa, 1.0, L.LQCD_F32, 12, U_device=Ud)
        done = len(losses)
        lr0 = a.lr * (lr_end / a.lr) ** (done / a.pairs)
        lr1 = a.lr * (lr_end / a.lr) ** ((done + n_f - 1) / a.pairs)
        losses += ptc.train(ctx, net, op64, op32, dims, None, every=a.every, pairs_per_source=a.per_source, lr=lr0,
                            seed0=a.seed0 + 1000 * f, log=lambda m: print("field %d: %s" % (f, m), flush=True),
                            lr_end=lr1, objective=a.objective, max_pairs=n_f)
        del op64, op32, Ud
    torch.cuda.synchronize()
    dt = time.time() - t0
    net.save(a.out)
    print("trained on %d pairs in %.1fs; loss first 100 %.4f, last 100 %.4f; saved %s" % (
        len(losses), dt, float(np.mean(losses[:100])), float(np.mean(losses[-100:])), a.out), flush=True)
    np.save(os.path.splitext(a.out)[0] + "_loss.npy", np.array(losses, dtype=np.float32))
    L.lqcd_context_destroy(ctx)


if __name__ == "__main__":
    main()
