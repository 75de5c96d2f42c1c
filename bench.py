#!/usr/bin/env python3
"""Benchmark of the Multipolynomial Monte Carlo hot path on one MI355X.

Default workload (one "step" = one complete trace estimate): 8^4 lattice
(n = 49152), SU(3) links U = exp(i 0.5 H) from seed 2, Wilson kappa = 0.120,
Theta = I; GMRES polynomials of degree 128, 32 and 8; the 20 lowest eigenpairs
of M asked from PP-Arnoldi (112 steps on M p_in(M), p_in of degree 8; the
pairs that pass the residual test are deflated); 128 Z(4) noise vectors per Monte Carlo term, each term's
noise processed as one multi-RHS batch; FP32 Wilson kernels with FP64
accumulation and FP64 defect correction of the main solves (relative residual
1e-8).  The step includes building the polynomials and the deflation set.

Printed metric: multi-RHS Dslash HBM GB/s = algorithmic bytes moved by all
Wilson-kernel launches of a step / wall time of the step.  The dominant
kernel's own rate (bytes / summed HIP-event kernel time) is the roofline
"achieved" figure.  Beside it, at the same noise seeds and counts (hence the
same standard error): the plain FP64 form of the estimate and the learned
form (the main solves preconditioned by the trained network; its training is
timed separately), for the time-to-fixed-standard-error comparison.  The FP64
CPU oracle is timed on the host as the baseline.

--workload 16x4 / 24x4 run the larger configurations (16^4 double polynomial
16x16 with 100 eigenpairs requested and 256 noises; 24^4 with four polynomials
16x16/128/32/8 and 64 noises per term) with the same report; the default line
is the 8^4 one.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--noises", type=int, default=None, help="noise vectors per term (default: the workload's)")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="8x4",
                    help="8x4 (default, the metric's configuration) or the larger parity configurations")
    ap.add_argument("--theta", choices=["I", "g5"], default="I")
    ap.add_argument("--solve-pp", action="store_true",
                    help="main solves of the mixed and plain forms as polynomial-preconditioned GMRES (p_in)")
    ap.add_argument("--net-source", choices=["random", "solve"], default="solve",
                    help="training pairs of the learned form: (M e, e) or snapshots of training solves")
    ap.add_argument("--no-plain", action="store_true", help="skip the FP64 comparison form")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device-to-device copy first (reference for hardware byte counters)")
    return ap.parse_args()


# Workloads: (lattice, link eps, seed, kappa, polynomial degrees ((din, dout) = double
# polynomial), noises per term, eigenpairs kept, right-hand sides per launch (0 = all),
# training pairs per minibatch of the learned form)
WORKLOADS = {
    "8x4": dict(dims=(8, 8, 8, 8), eps=0.5, seed=2, kappa=0.120, degrees=[128, 32, 8], noises=128, nev=20,
                max_batch=0, net_pairs=64),
    "16x4": dict(dims=(16, 16, 16, 16), eps=0.4, seed=3, kappa=0.124, degrees=[(15, 15)], noises=256, nev=100,
                 max_batch=0, net_pairs=16, solve_prec="fp16s"),
    "24x4": dict(dims=(24, 24, 24, 24), eps=0.4, seed=4, kappa=0.1245, degrees=[(15, 15), 128, 32, 8], noises=64,
                 nev=20, max_batch=0, net_pairs=16),
}

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_wilson_dot_fp32_8x4x128_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2402_00016_amd", "csrc", "wilson.hip")


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when the summary is missing or the kernel source changed
    since the counters were taken (the summary records the source's SHA-256)."""
    import hashlib
    try:
        txt = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        line = line.strip().strip("`")
        if ":" in line and line.split(":", 1)[0] in ("kernel_source_sha256", "traffic_bytes_per_launch"):
            k, v = line.split(":", 1)
            vals[k] = v.strip()
    if "traffic_bytes_per_launch" not in vals:
        return None
    if vals.get("kernel_source_sha256") != hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest():
        return None
    return float(vals["traffic_bytes_per_launch"])


def workload_name(key, W, noises, theta):
    L = W["dims"]
    degs = "/".join("%dx%d" % (d[0] + 1, d[1] + 1) if isinstance(d, tuple) else str(d) for d in W["degrees"])
    return ("%s^4 Wilson (kappa %g, eps %g links seed %d), GMRES polynomials of degree %s, %d deflated eigenpairs "
            "requested, %d Z(4) noises per term, Theta=%s, FP32 Dslash + FP64 refinement to 1e-8%s"
            % (L[0], W["kappa"], W["eps"], W["seed"], degs, W["nev"], noises, theta,
               ", FP16 Krylov basis in the solves" if W.get("solve_prec") == "fp16s" else ""))


def cpu_baseline(dims, kappa, links, seconds):
    """FP64 oracle Dslash on the host cores, on a bounded sample: repeated
    16-RHS applications on the same field for about `seconds` seconds."""
    import numpy as np

    from oracle.philox import z4_noise_batch
    from oracle.wilson import WilsonOp
    op = WilsonOp(dims, kappa, links)
    N = 16
    X = z4_noise_batch(2, 0, 0, N, op.n)
    op(X)
    t0 = time.perf_counter()
    reps = 0
    while time.perf_counter() - t0 < seconds:
        op(X)
        reps += 1
    dt = time.perf_counter() - t0
    V = op.V
    bytes_per_apply = V * (N * 384.0 + 576.0)      # FP64: 12 complex in + out per site per rhs, links once
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(bytes_per_apply * reps / dt / 1e9, 3), "unit": "GB/s", "cores": cores,
            "kind": "oracle",
            "sample": "FP64 oracle Wilson operator, %d^4 lattice, 16 Z(4) right-hand sides per call, "
                      "%d calls in %.1f s on %d host threads; same byte formula as the GPU figure"
                      % (dims[0], reps, dt, cores)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (the method's noise vectors "
              "shard across GPUs with one final all-reduce, which is not implemented); use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2402_00016_amd import driver, inputs, mpmc

    torch.cuda.set_device(0)
    W = WORKLOADS[a.workload]
    dims, eps, seed, kappa = W["dims"], W["eps"], W["seed"], W["kappa"]
    noises = a.noises or W["noises"]
    links = inputs.gauge_links(dims, eps, seed)
    ctx = mpmc.Context(dims, kappa, links)
    plan = driver.Plan(degrees=W["degrees"], noises=noises, seed=seed, nev=W["nev"],
                       defl_candidates=max(40, W["nev"] + 20), defl_m=112 if W["nev"] <= 40 else 136,
                       defl_pin_degree=8, theta=mpmc.THETA[a.theta], max_batch=W["max_batch"],
                       poly_prec=mpmc.FP32, solve_inner_prec=mpmc.PREC[W.get("solve_prec", "fp32")],
                       solve_tol=1e-8, solve_restart=50, net_pairs=W["net_pairs"], solve_pp=a.solve_pp)
    sync = torch.cuda.synchronize

    if a.calibrate_copy:
        src = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        sync()
        dst.copy_(src)
        sync()
        del src, dst
    for _ in range(a.warmup):
        driver.estimate(ctx, plan, sync)
    # the side contexts (setup work on other streams) exist after the warm-up;
    # their Wilson launches count in value as well
    sides = [c for c, _ in ctx._side.values()]
    for c in [ctx] + sides:
        mpmc.mpmc_timing_enable(c.handle, 1)
    sync()
    t0 = time.perf_counter()
    ests = [driver.estimate(ctx, plan, sync) for _ in range(a.steps)]
    sync()
    t1 = time.perf_counter()
    n32, ms32, by32 = mpmc.mpmc_timing_read(ctx.handle, mpmc.FP32)
    n64, ms64, by64 = mpmc.mpmc_timing_read(ctx.handle, mpmc.FP64)
    nd, msd, byd = mpmc.mpmc_timing_read(ctx.handle, mpmc.FP32 | mpmc.TIMING_FUSED)   # dominant kernel
    na, msa, bya = mpmc.mpmc_timing_read(ctx.handle, mpmc.FP32 | mpmc.TIMING_PLAIN)
    side_bytes = sum(mpmc.mpmc_timing_read(c.handle, p)[2] for c in sides for p in (mpmc.FP32, mpmc.FP64))
    for c in [ctx] + sides:
        mpmc.mpmc_timing_enable(c.handle, 0)
    step_s = (t1 - t0) / a.steps
    bytes_step = (by32 + by64 + side_bytes) / a.steps
    est = ests[-1]

    out = {
        "metric": "multi-RHS Dslash HBM GB/s; time to fixed trace std-error, learned vs plain",
        "value": round(bytes_step / step_s / 1e9, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": workload_name(a.workload, W, noises, a.theta), "lattice": list(dims),
                   "noises_per_term": noises, "rhs_per_launch": W["max_batch"] or noises,
                   "degrees": [list(d) if isinstance(d, tuple) else d for d in W["degrees"]], "theta": a.theta},
        "roofline": {"bound": "hbm", "achieved": round(byd / (msd * 1e-3) / 1e9, 1) if msd > 0 else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(byd / (msd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if msd > 0 else None,
                     "traffic": measured_traffic() if a.workload == "8x4" else None, "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, "
                                                                     "scaled by a 256 MiB copy)",
                     "algorithmic_bytes_per_launch": round(byd / max(nd, 1)),
                     "kernel": "k_wilson_dot<FP32> (fused polynomial level step: w' = w - c M w, eta^H Theta w')",
                     "launches": nd, "avg_launch_us": round(msd * 1e3 / max(nd, 1), 2),
                     "other_fp32_wilson": {"kernel": "k_wilson<FP32>", "launches": na,
                                           "avg_launch_us": round(msa * 1e3 / max(na, 1), 2),
                                           "GBs": round(bya / (msa * 1e-3) / 1e9, 1) if msa > 0 else None}},
        "trace": {"value": [est.value.real, est.value.imag], "stderr": est.stderr,
                  "levels": [{"name": L.name, "mean": [L.mean.real, L.mean.imag], "var": L.var, "n": L.n,
                              "corr": [L.corr.real, L.corr.imag], "mvps": L.mvps, "s": round(L.seconds, 4)}
                             for L in est.levels],
                  "deflated": est.defl_k, "setup_s": round(est.setup_seconds, 4), "mvps": est.mvps},
        "time_to_error_s": {"mixed_batched": round(step_s, 4)},
        "fp64_kernel_share": {"launches": n64, "multi_rhs_ms_per_step": round(ms64 / a.steps, 3),
                              "note": "single-vector launches are counted (bytes, launches) without events"},
    }
    def solve_term(e):
        L = e.levels[0]
        return {"s": round(L.seconds, 4), "mvps": L.mvps}

    out["solve_term"] = {"mixed_batched": solve_term(est)}
    if not a.no_learned:
        ctx.release_workspace()
        torch.cuda.empty_cache()
        # learned form: the network is trained once per gauge field (timed
        # separately) and then preconditions the main solves of the estimate
        lplan = driver.Plan(**{**plan.__dict__, "learned": True, "solve_inner_prec": mpmc.FP32,
                               "net_source": a.net_source,
                               "net_batches": 2 if a.net_source == "solve" else 8})
        sync()
        tl = time.perf_counter()
        net, hist = driver.train_net(ctx, lplan)
        sync()
        t_train = time.perf_counter() - tl
        driver.estimate(ctx, lplan, sync, net=net)
        sync()
        tl = time.perf_counter()
        el = driver.estimate(ctx, lplan, sync, net=net)
        sync()
        tl = time.perf_counter() - tl
        out["time_to_error_s"]["learned_batched"] = round(tl, 4)
        out["time_to_error_s"]["net_training"] = round(t_train, 4)
        out["time_to_error_s"]["learned_batched_incl_training"] = round(tl + t_train, 4)
        out["solve_term"]["learned_batched"] = solve_term(el)
        out["net"] = {"source": lplan.net_source, "minibatches": len(hist) // lplan.net_steps,
                      "pairs": len(hist) // lplan.net_steps * lplan.net_pairs, "adam_steps": len(hist),
                      "loss_first": float(hist[0]), "loss_last": float(hist[-1])}
        comb = float(np.hypot(el.stderr, est.stderr))
        out["trace"]["learned"] = {"value": [el.value.real, el.value.imag], "stderr": el.stderr,
                                   "diff_in_combined_sigma": abs(est.value - el.value) / comb}
    if not a.no_plain:
        ctx.release_workspace()
        torch.cuda.empty_cache()
        plain = driver.Plan(**{**plan.__dict__, "poly_prec": mpmc.FP64, "solve_inner_prec": mpmc.FP64})
        driver.estimate(ctx, plain, sync)
        sync()
        tp = time.perf_counter()
        e64 = driver.estimate(ctx, plain, sync)
        sync()
        tp = time.perf_counter() - tp
        out["time_to_error_s"]["plain_fp64"] = round(tp, 4)
        out["time_to_error_s"]["speedup_mixed_vs_plain"] = round(tp / step_s, 3)
        if "learned_batched" in out["time_to_error_s"]:
            out["time_to_error_s"]["speedup_learned_vs_plain"] = round(tp / out["time_to_error_s"]["learned_batched"], 3)
            out["time_to_error_s"]["speedup_learned_incl_training_vs_plain"] = round(
                tp / out["time_to_error_s"]["learned_batched_incl_training"], 3)
        out["solve_term"]["plain_fp64"] = solve_term(e64)
        comb = float(np.hypot(e64.stderr, est.stderr))
        out["trace"]["plain_fp64"] = {"value": [e64.value.real, e64.value.imag], "stderr": e64.stderr,
                                      "diff_in_combined_sigma": abs(est.value - e64.value) / comb}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(dims, kappa, links, a.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
