"""Learned preconditioner across lattice sizes: one network, trained on the
24^4 field, preconditions the deflated main solves on fields of 12^4, 16^4,
20^4 and 24^4 (links eps = 0.4, kappa = 0.124).  The network's weights act on
(field, spin) along parallel-transport paths, so the same weights apply to
any volume.  Reported per lattice: inner GMRES iterations, MVPs and wall time
to a true relative residual of 1e-8, with and without the network, on the
same Z(4) right-hand sides and the same deflation set.  Last, the four
fields' Wilson applications (64 right-hand sides each) run as one batched
launch and as one launch per lattice, and their deflated solves run one
after another and in lockstep with one batched Wilson launch per inner
iteration (mpmc_solve_batch), plain and with the network.

    python -m paper_2402_00016_amd.netstudy --lattices 12,16,20,24 --rhs 16
    python -m paper_2402_00016_amd.netstudy --train-seeds 64 --train-rhs 16 --train-snaps 4 --train-restart 10
        (4096 training pairs from the solves of noise seeds 100-163)

Host bookkeeping only; every vector operation runs in libmpmc.so.
"""
import argparse
import json
import time

import numpy as np
import torch

from . import driver, inputs, mpmc


def timed(fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def train(dims, link_eps, kappa, seed, plan):
    ctx = mpmc.Context(dims, kappa, inputs.gauge_links(dims, link_eps, seed))
    def report(b, hist):
        if (b + 1) % 8 == 0 or b + 1 == plan.net_batches:
            print(json.dumps(dict(training_seeds_done=b + 1, adam_steps=len(hist),
                                  loss=float(hist[-1]) if hist else None)), flush=True)

    (net, hist), secs = timed(lambda: driver.train_net(ctx, plan, report))
    w = net.weights.copy()
    del net
    ctx.release_workspace()
    return w, hist, secs


def compare(dims, link_eps, kappa, seed, weights, nrhs, nev, restart, tol):
    ctx = mpmc.Context(dims, kappa, inputs.gauge_links(dims, link_eps, seed))
    plan = driver.Plan(degrees=[], nev=nev, seed=seed)
    defl, t_defl = timed(lambda: driver.build_deflation(ctx, plan))
    net = ctx.net(weights)
    b = ctx.noise(seed, 5, 0, nrhs, mpmc.FP64)
    out = dict(lattice=list(dims), deflated=int(defl.k) if defl is not None else 0, deflation_s=round(t_defl, 3))
    for name, nn in (("plain", None), ("learned", net)):
        ctx.solve(b, nrhs, defl=defl, restart=restart, tol=tol, inner_prec=mpmc.FP32, net=nn)   # warm-up
        mv0 = ctx.mvps
        (x, its, rel), secs = timed(lambda: ctx.solve(b, nrhs, defl=defl, restart=restart, tol=tol,
                                                      inner_prec=mpmc.FP32, net=nn))
        out[name] = dict(inner_iterations=int(its), mvps=int(ctx.mvps - mv0), seconds=round(secs, 4),
                         max_relres=float(np.max(rel)))
        del x
    out["speedup"] = round(out["plain"]["seconds"] / out["learned"]["seconds"], 3)
    out["iteration_ratio"] = round(out["plain"]["inner_iterations"] / max(out["learned"]["inner_iterations"], 1), 3)
    ctx.release_workspace()
    return out


def batch_solves(lattices, link_eps, kappa, seed, weights, nrhs, nev, restart, tol):
    """The lattices' deflated solves (nrhs right-hand sides each) one lattice
    after another and in lockstep with one batched Wilson launch per inner
    iteration (mpmc_solve_batch), plain and with the network; same iterates
    either way, so the same iteration counts."""
    ctxs = [mpmc.Context((L,) * 4, kappa, inputs.gauge_links((L,) * 4, link_eps, seed)) for L in lattices]
    defls = [driver.build_deflation(c, driver.Plan(degrees=[], nev=nev, seed=seed)) for c in ctxs]
    nets = [c.net(weights) for c in ctxs]
    bs = [c.noise(seed, 5, 0, nrhs, mpmc.FP64) for c in ctxs]
    out = dict(lattices=[[L] * 4 for L in lattices], nrhs=nrhs, deflated=[int(d.k) for d in defls])
    for name, nn in (("plain", None), ("learned", nets)):
        def sequential():
            return [c.solve(b, nrhs, defl=d, restart=restart, tol=tol, inner_prec=mpmc.FP32,
                            net=None if nn is None else nn[i])[1] for i, (c, b, d) in enumerate(zip(ctxs, bs, defls))]

        def batched():
            xs, its, rel = mpmc.Context.solve_batch(ctxs, bs, nrhs, defls=defls, nets=nn, restart=restart, tol=tol,
                                                    inner_prec=mpmc.FP32)
            assert float(np.max(rel)) <= tol
            return [int(v) for v in its]

        sequential()   # warm-up (workspace)
        its_s, t_s = timed(sequential)
        batched()
        its_b, t_b = timed(batched)
        out[name] = dict(inner_iterations=[int(v) for v in its_s], sequential_s=round(t_s, 4),
                         batched_s=round(t_b, 4), batched_iterations=its_b)
        for c in ctxs:
            c.release_workspace()
    out["learned_vs_plain_batched"] = round(out["plain"]["batched_s"] / out["learned"]["batched_s"], 3)
    return out


def batch_timing(lattices, link_eps, kappa, seed, nrhs=64, reps=10):
    """The uneven lattices' Wilson applications in one batched launch against
    one launch per lattice (FP32, same traversal, same results)."""
    ctxs = [mpmc.Context((L,) * 4, kappa, inputs.gauge_links((L,) * 4, link_eps, seed + i))
            for i, L in enumerate(lattices)]
    xs = [c.noise(seed, 7, 0, nrhs, mpmc.FP32) for c in ctxs]
    for c in ctxs:
        c.tune_set(nrhs, mpmc.FP32, 5)
    ys = [c.vector(nrhs, mpmc.FP32) for c in ctxs]

    def separate():
        for c, x, y in zip(ctxs, xs, ys):
            c.apply_M(x, nrhs, mpmc.FP32, out=y)

    def batched():
        mpmc.Context.apply_M_batch(ctxs, xs, nrhs, mpmc.FP32, outs=ys)

    out = {}
    for name, fn in (("separate", separate), ("batched", batched)):
        fn()
        _, secs = timed(lambda: [fn() for _ in range(reps)])
        out[name + "_ms"] = round(secs / reps * 1e3, 3)
    out.update(lattices=[[L] * 4 for L in lattices], nrhs=nrhs)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--lattices", default="12,16,20,24")
    ap.add_argument("--train-lattice", type=int, default=24)
    ap.add_argument("--eps", type=float, default=0.4, help="link generator spread")
    ap.add_argument("--kappa", type=float, default=0.124)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--rhs", type=int, default=16)
    ap.add_argument("--nev", type=int, default=20)
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--train-seeds", type=int, default=2,
                    help="training solves, Z(4) noise seeds 100, 101, ... (64: seeds 100-163)")
    ap.add_argument("--train-rhs", type=int, default=16, help="right-hand sides per training solve")
    ap.add_argument("--train-snaps", type=int, default=4, help="(r, e) batches recorded per training solve")
    ap.add_argument("--train-restart", type=int, default=20,
                    help="GMRES restart of the training solves (shorter: more outer cycles, more snapshots)")
    ap.add_argument("--batch-rhs", type=int, default=64,
                    help="right-hand sides per lattice of the lockstep solves (0: skip them)")
    ap.add_argument("--batch-restart", type=int, default=25)
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    Lt = a.train_lattice
    plan = driver.Plan(degrees=[], seed=a.seed, net_pairs=a.train_rhs, net_batches=a.train_seeds, net_steps=10,
                       net_source="solve", net_snaps=a.train_snaps, net_seed0=100, net_restart=a.train_restart)
    w, hist, t_train = train((Lt,) * 4, a.eps, a.kappa, a.seed, plan)
    # each recorded batch of right-hand sides is one minibatch of net_steps Adam steps
    pairs = len(hist) // plan.net_steps * plan.net_pairs
    print(json.dumps(dict(trained_on=[Lt] * 4, seconds=round(t_train, 3), loss_first=float(hist[0]),
                          loss_last=float(hist[-1]), adam_steps=len(hist), training_pairs=pairs,
                          noise_seeds=[100, 100 + a.train_seeds - 1])), flush=True)
    rows = []
    for L in (int(v) for v in a.lattices.split(",")):
        r = compare((L,) * 4, a.eps, a.kappa, a.seed, w, a.rhs, a.nev, a.restart, 1e-8)
        rows.append(r)
        print(json.dumps(r), flush=True)
        torch.cuda.empty_cache()
    print(json.dumps(dict(summary=rows)), flush=True)
    lat = [int(v) for v in a.lattices.split(",")]
    print(json.dumps(dict(batch=batch_timing(lat, a.eps, a.kappa, a.seed))), flush=True)
    if a.batch_rhs:
        print(json.dumps(dict(batch_solves=batch_solves(lat, a.eps, a.kappa, a.seed, w, a.batch_rhs, a.nev,
                                                          a.batch_restart, 1e-8))), flush=True)


if __name__ == "__main__":
    main()
