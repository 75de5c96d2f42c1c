"""Degree-versus-variance study of polynomial subtraction (Sec. 4).

For each lattice, configuration (link seed) and polynomial degree d, the
relative variance of the subtracted estimator is

    sigma_R^2 = var[eta^H Theta (M^-1 - p_d(M)) eta] / var[eta^H Theta M^-1 eta]   (eq. 3)

and over configurations both the plain average (eq. 3 with configuration-
averaged variances) and the base-10 log average (eq. 4) are reported.  All
samples come from mpmc_level_estimate (the no-subtraction samples are the
solve term with lower = 0).  Host bookkeeping only; every vector operation
runs in libmpmc.so.

    python -m paper_2402_00016_amd.sweep --lattice 8,8,8,8 --seeds 1,2,3 \
        --degrees 4,8,16,32,64 --kappa 0.14 --noises 32
"""
import argparse
import json
import math
import time

import numpy as np

from . import inputs, mpmc


def sample_var(X):
    X = np.asarray(X)
    return float(np.sum(np.abs(X - X.mean()) ** 2) / (len(X) - 1))


def sweep_config(dims, kappa, eps, seed, degrees, noises, theta=mpmc.THETA_I, solve_tol=1e-8, batch=0):
    """Variances for one configuration: {'ns': var, d: var, ...}."""
    ctx = mpmc.Context(dims, kappa, inputs.gauge_links(dims, eps, seed))
    out = {}
    X, _, _ = ctx.level(None, None, None, theta, seed, 0, 0, noises, prec=mpmc.FP64, max_batch=batch,
                        solve_tol=solve_tol, solve_inner_prec=mpmc.FP32)
    out["ns"] = sample_var(X)
    out["mean"] = [float(X.mean().real), float(X.mean().imag)]
    for j, d in enumerate(degrees):
        p = ctx.gmres_poly(seed, 0x100 + j, int(d) + 1)
        Xd, _, _ = ctx.level(None, p, None, theta, seed, 0, 0, noises, prec=mpmc.FP64, max_batch=batch,
                             solve_tol=solve_tol, solve_inner_prec=mpmc.FP32)
        out[int(d)] = sample_var(Xd)
    return out


def summarize(per_config, degrees):
    """Relative variance (eq. 3) and log-averaged relative variance (eq. 4)."""
    ns = np.array([c["ns"] for c in per_config])
    rows = []
    for d in degrees:
        v = np.array([c[int(d)] for c in per_config])
        rel = float(v.mean() / ns.mean())
        logrel = float(10 ** (np.mean(np.log10(v)) - np.mean(np.log10(ns))))
        rows.append(dict(degree=int(d), rel_var=rel, log_avg_rel_var=logrel))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--lattice", default="8,8,8,8")
    ap.add_argument("--seeds", default="1,2,3")
    ap.add_argument("--degrees", default="4,8,16,32,64")
    ap.add_argument("--kappa", type=float, default=0.14)
    ap.add_argument("--eps", type=float, default=0.5)
    ap.add_argument("--noises", type=int, default=32)
    ap.add_argument("--theta", choices=["I", "g5"], default="I")
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    dims = tuple(int(x) for x in a.lattice.split(","))
    degrees = [int(x) for x in a.degrees.split(",")]
    per = []
    t0 = time.perf_counter()
    for seed in (int(x) for x in a.seeds.split(",")):
        per.append(sweep_config(dims, a.kappa, a.eps, seed, degrees, a.noises, theta=mpmc.THETA[a.theta]))
        print(json.dumps(dict(seed=seed, **{str(k): v for k, v in per[-1].items()})), flush=True)
    print(json.dumps(dict(lattice=list(dims), kappa=a.kappa, eps=a.eps, noises=a.noises, configs=len(per),
                          theta=a.theta, seconds=round(time.perf_counter() - t0, 2),
                          relative_variance=summarize(per, degrees))), flush=True)


if __name__ == "__main__":
    main()
