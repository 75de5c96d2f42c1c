#!/usr/bin/env python3
"""Benchmark of the Multipolynomial Monte Carlo hot path on one MI355X.

Default workload (one "step" = one complete trace estimate, setup included):
the 24^4 lattice (V = 331776, n = 3981312, the paper's lattice shape), SU(3)
links U = exp(i 0.4 H) from seed 4, Wilson kappa = 0.1245, Theta = I; four
polynomials: a 16x16 double polynomial (degree 255) and GMRES polynomials of
degree 128, 32 and 8; the 20 lowest eigenpairs of M asked from PP-Arnoldi
(p_in of degree 8, the pairs that pass the residual test are deflated); 64
Z(4) noise vectors per Monte Carlo term, each term's noise one multi-RHS
batch; FP32 Wilson kernels with FP64 sums, main solves deflated GMRES(50) with
FP32 inner cycles and FP64 defect correction to a true relative residual of
1e-8.

Printed metric: multi-RHS Dslash GB/s = algorithmic HBM bytes of every
multi-right-hand-side Wilson launch of the timed steps (spinor operands read
once, outputs written once, links once per site) / the summed HIP-event
durations of those launches.  The dominant kernel's own rate is the roofline
"achieved" figure.  Beside it, at the same noise seeds and counts (hence the
same standard error): the plain FP64 form of the estimate and the learned form
(the main solves preconditioned by the trained network, training timed too),
for the time-to-fixed-standard-error comparison; the per-term differences of
the mixed-precision means from the FP64 ones in units of the FP64 standard
errors; the FP64 CPU oracle timed on the host as the baseline.

--workload 16x4 runs the 16^4 configuration (the deflated 16x16 double
polynomial with 100 eigenpairs requested, 256 noises, FP16 Krylov basis in the
solves; the undeflated double polynomial's level variance is reported beside
it) and --workload 8x4 the 8^4 one (degrees 128/32/8, 128 noises).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--noises", type=int, default=None, help="noise vectors per term (default: the workload's)")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="24x4",
                    help="24x4 (default, the largest single-GPU configuration), 16x4 or 8x4")
    ap.add_argument("--compare-runs", type=int, default=0,
                    help="estimates of the learned and of the plain form timed (median reported); "
                         "0 = as many as --steps, at most 5")
    ap.add_argument("--theta", choices=["I", "g5"], default="I")
    ap.add_argument("--probe-last", action="store_true",
                    help="last term exactly by probing (distance colouring) in every form")
    ap.add_argument("--no-probe-report", action="store_true",
                    help="skip the extra estimate with the probed last term")
    ap.add_argument("--solve-prec", choices=["fp32", "fp16s"], default=None,
                    help="Krylov basis storage of the mixed form's main solves (default: the workload's)")
    ap.add_argument("--defl-m", type=int, default=0,
                    help="PP-Arnoldi steps of the deflation build (0: 2 x eigenpairs + 40, at least 112, at most 256)")
    ap.add_argument("--solve-pp", action="store_true",
                    help="main solves of the mixed and plain forms as polynomial-preconditioned GMRES (p_in)")
    ap.add_argument("--net-source", choices=["random", "solve"], default="solve",
                    help="training pairs of the learned form: (M e, e) or snapshots of training solves")
    ap.add_argument("--net-steps", type=int, default=5,
                    help="Adam steps per training minibatch of the learned form (24^4: 5 steps train in 0.69 s "
                         "against 0.94 s for 10, same solve term; 3 steps leave it 45%% slower)")
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
                 max_batch=0, net_pairs=16, solve_prec="fp16s", deflate_double=True),
    "24x4": dict(dims=(24, 24, 24, 24), eps=0.4, seed=4, kappa=0.1245, degrees=[(15, 15), 128, 32, 8], noises=64,
                 nev=20, max_batch=0, net_pairs=16, solve_prec="fp16s"),
}

TRAFFIC_FILES = {"8x4": os.path.join(ROOT, "profiles", "k_wilson_dot_fp32_8x4x128_traffic.md"),
                 "24x4": os.path.join(ROOT, "profiles", "wilson_fp32_24x4x64_traffic.md")}
KERNEL_SOURCE = os.path.join(ROOT, "paper_2402_00016_amd", "csrc", "wilson.hip")


def measured_traffic(workload, kernel, variant=None):
    """HBM bytes per launch of `kernel` ("fused" or "plain") from the committed
    counter summary of the workload, or None when the summary is missing or the
    kernel source changed since the counters were taken (the summary records
    the source's SHA-256).  variant: the traversal the run used (fused-step
    order or apply variant), when the summary lists it separately."""
    import hashlib
    try:
        txt = open(TRAFFIC_FILES[workload]).read()
    except (OSError, KeyError):
        return None
    key = "traffic_bytes_per_launch" if workload == "8x4" else "traffic_bytes_per_launch_" + kernel
    vals = {}
    for line in txt.splitlines():
        line = line.strip().strip("`")
        if ":" in line and line.split(":", 1)[0].startswith(("kernel_source_sha256", key)):
            k, v = line.split(":", 1)
            vals[k] = v.strip()
    if variant is not None and "%s_%s" % (key, variant) in vals:
        key = "%s_%s" % (key, variant)
    if key not in vals:
        return None
    if vals.get("kernel_source_sha256") != hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest():
        return None
    return float(vals[key])


def workload_name(key, W, noises, theta):
    L = W["dims"]
    degs = "/".join("%dx%d" % (d[0] + 1, d[1] + 1) if isinstance(d, tuple) else str(d) for d in W["degrees"])
    return ("%s^4 Wilson (kappa %g, eps %g links seed %d), GMRES polynomials of degree %s%s, %d deflated eigenpairs "
            "requested, %d Z(4) noises per term, Theta=%s, FP32 Dslash + FP64 refinement to 1e-8%s"
            % (L[0], W["kappa"], W["eps"], W["seed"], degs, " (deflated double)" if W.get("deflate_double") else "",
               W["nev"], noises, theta, ", FP16 Krylov basis in the solves" if W.get("solve_prec") == "fp16s" else ""))


def cpu_baseline(dims, kappa, links, seconds, step_mvps):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload: repeated 16-RHS operator applications on the same field for
    about `seconds` seconds on all threads, then a quarter of that on one
    thread, and one degree-8 polynomial application to one vector.  The
    oracle's time for a whole estimate is extrapolated from its per-MVP time
    and the estimate's MVP count (labelled as such)."""
    from oracle import krylov as OK
    from oracle import poly as OP
    from oracle.philox import z4_noise, z4_noise_batch
    from oracle.wilson import WilsonOp
    op = WilsonOp(dims, kappa, links)
    threads = WilsonOp.max_threads()
    N = 16
    X = z4_noise_batch(2, 0, 0, N, op.n)
    bytes_per_apply = op.V * (N * 384.0 + 576.0)     # FP64: 12 complex in + out per site per rhs, links once

    def rate(secs):
        op(X)
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < secs:
            op(X)
            reps += 1
        dt = time.perf_counter() - t0
        return bytes_per_apply * reps / dt / 1e9, dt / (reps * N), reps, dt

    gbs, s_per_mvp, reps, dt = rate(seconds)
    WilsonOp.set_threads(1)
    gbs1, s_per_mvp1, reps1, dt1 = rate(seconds / 4)
    WilsonOp.set_threads(threads)
    roots = OK.leja_order(np.array([1.0 + 0.05j * k for k in range(9)]))
    v = z4_noise(2, 1, 0, op.n)
    t0 = time.perf_counter()
    OP.apply_p(op, roots, v)
    t_poly8 = time.perf_counter() - t0
    # one GMRES(8) cycle (8 Arnoldi steps with CGS2) on one vector of this lattice
    t0 = time.perf_counter()
    OK.arnoldi(op, v, 8)
    t_arn8 = time.perf_counter() - t0
    # the whole plain-method estimate of the 4^4 configuration on the oracle:
    # GMRES(16) polynomial, 32 noises, solves to 1e-8, with and without subtraction
    from oracle import estimator as OES
    from paper_2402_00016_amd import inputs as _inputs
    d4, k4 = (4, 4, 4, 4), 0.115
    op4 = WilsonOp(d4, k4, _inputs.gauge_links(d4, 0.5, seed=1))
    t0 = time.perf_counter()
    P4, _, _ = OK.gmres_poly(op4, z4_noise(1, 0x100, 0, op4.n), 16)
    X0, _ = OES.level_samples(op4, None, None, None, "I", 1, 0, 0, 32, solve_tol=1e-8)
    X1, _ = OES.level_samples(op4, None, P4, None, "I", 1, 1, 0, 32, solve_tol=1e-8)
    X2, _ = OES.level_samples(op4, P4, None, None, "I", 1, 2, 0, 32)
    t_est4 = time.perf_counter() - t0
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": "FP64 oracle Wilson operator on the %s lattice, 16 Z(4) right-hand sides per call: "
                      "%d calls in %.1f s on %d threads, %d calls in %.1f s on 1 thread; one degree-8 polynomial "
                      "application to one vector; same byte formula as the GPU figure"
                      % ("x".join(map(str, dims)), reps, dt, threads, reps1, dt1),
            "one_core_GBs": round(gbs1, 3),
            "s_per_rhs_mvp": s_per_mvp, "s_per_rhs_mvp_one_core": s_per_mvp1,
            "degree8_poly_one_vector_s": round(t_poly8, 3),
            "gmres8_cycle_one_vector_s": round(t_arn8, 3),
            "estimate_4x4_plain_method_s": round(t_est4, 3),
            "estimate_4x4_note": "the 4^4 configuration's whole estimate on the oracle (GMRES(16) polynomial, "
                                 "32 noises, solves to 1e-8, with and without subtraction)",
            "estimate_s_extrapolated": round(s_per_mvp * step_mvps, 1),
            "estimate_note": "extrapolated: the oracle's per-MVP time x the MVPs of one GPU estimate "
                             "(Gram-Schmidt and dense work not included)"}


def level_report(est):
    return [{"name": L.name, "mean": [L.mean.real, L.mean.imag], "var": L.var, "n": L.n,
             "corr": [L.corr.real, L.corr.imag], "mvps": L.mvps, "s": round(L.seconds, 4)} for L in est.levels]


def progress(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def main():
    a = parse()
    if a.compare_runs <= 0:
        a.compare_runs = max(1, min(a.steps, 5))
    if a.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (the method's noise vectors "
              "shard across GPUs with one final all-reduce, which is not implemented); use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2402_00016_amd import driver, inputs, mpmc

    torch.cuda.set_device(0)
    W = dict(WORKLOADS[a.workload])
    if a.solve_prec:
        W["solve_prec"] = a.solve_prec
    dims, eps, seed, kappa = W["dims"], W["eps"], W["seed"], W["kappa"]
    noises = a.noises or W["noises"]
    links = inputs.gauge_links(dims, eps, seed)
    ctx = mpmc.Context(dims, kappa, links)
    plan = driver.Plan(degrees=W["degrees"], noises=noises, seed=seed, nev=W["nev"],
                       defl_candidates=max(40, W["nev"] + 20), defl_m=a.defl_m or min(256, max(112, 2 * W["nev"] + 40)),
                       defl_pin_degree=8, theta=mpmc.THETA[a.theta], max_batch=W["max_batch"],
                       poly_prec=mpmc.FP32, solve_inner_prec=mpmc.PREC[W.get("solve_prec", "fp32")],
                       solve_tol=1e-8, solve_restart=50, net_pairs=W["net_pairs"], solve_pp=a.solve_pp,
                       deflate_double=W.get("deflate_double", False), setup_prec=mpmc.FP32,
                       probe_last=a.probe_last)
    sync = torch.cuda.synchronize

    if a.calibrate_copy:
        src = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        sync()
        dst.copy_(src)
        sync()
        del src, dst
    for i in range(a.warmup):
        driver.estimate(ctx, plan, sync)
        progress("warm-up step %d done" % (i + 1))
    # the side contexts (setup work on other streams) exist after the warm-up
    sides = [c for c, _ in ctx._side.values()]
    for c in [ctx] + sides:
        mpmc.mpmc_timing_enable(c.handle, 1)
    sync()
    t0 = time.perf_counter()
    ests = [driver.estimate(ctx, plan, sync) for _ in range(a.steps)]
    sync()
    t1 = time.perf_counter()
    progress("%d timed steps done (%.3f s/step)" % (a.steps, (t1 - t0) / a.steps))

    def timing(prec):
        n = ms = by = 0.0
        for c in [ctx] + sides:
            cn, cms, cby = mpmc.mpmc_timing_read(c.handle, prec)
            n, ms, by = n + cn, ms + cms, by + cby
        return int(n), ms, by

    fused = timing(mpmc.FP32 | mpmc.TIMING_FUSED)
    plain32 = timing(mpmc.FP32 | mpmc.TIMING_PLAIN)
    fused64 = timing(mpmc.FP64 | mpmc.TIMING_FUSED)
    plain64 = timing(mpmc.FP64 | mpmc.TIMING_PLAIN)
    single = timing(mpmc.FP64 | mpmc.TIMING_SINGLE)
    single32 = timing(mpmc.FP32 | mpmc.TIMING_SINGLE)
    for c in [ctx] + sides:
        mpmc.mpmc_timing_enable(c.handle, 0)
    step_s = (t1 - t0) / a.steps
    multi = [fused, plain32, fused64, plain64]
    dslash_ms = sum(k[1] for k in multi)
    dslash_bytes = sum(k[2] for k in multi)
    est = ests[-1]

    def kern(name, k):
        n, ms, by = k
        return {"kernel": name, "launches": n, "avg_launch_us": round(ms * 1e3 / max(n, 1), 2),
                "algorithmic_bytes_per_launch": round(by / max(n, 1)),
                "GBs": round(by / (ms * 1e-3) / 1e9, 1) if ms > 0 else None, "ms_per_step": round(ms / a.steps, 2)}

    kf = kern("k_wilson_dot<FP32> (fused polynomial level step: w' = w - c M w, eta^H Theta w')", fused)
    kp = kern("k_wilson<FP32> (multi-RHS apply: solves, polynomial applications)", plain32)
    dom, dom_key = (kf, "fused") if fused[1] >= plain32[1] else (kp, "plain")
    tuned64 = getattr(ctx, "tuned", {}).get((noises if not W["max_batch"] else W["max_batch"], mpmc.FP32), {})
    dom_variant = ("order%s" % tuned64.get("level_order") if dom_key == "fused" else
                   "variant%s" % tuned64.get("variant")) if tuned64 else None
    out = {
        "metric": "multi-RHS Dslash HBM GB/s; time to fixed trace std-error, learned vs plain",
        "value": round(dslash_bytes / (dslash_ms * 1e-3) / 1e9, 3) if dslash_ms > 0 else None,
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
        "value_def": "algorithmic bytes of all multi-RHS Wilson launches of the timed steps / their summed "
                     "HIP-event durations (inputs resident in HBM)",
        "dslash": {"bytes_per_step": round(dslash_bytes / a.steps), "kernel_ms_per_step": round(dslash_ms / a.steps, 2),
                   "bytes_per_wall_s_GBs": round(dslash_bytes / a.steps / step_s / 1e9, 1),
                   "kernels": [kf, kp, kern("k_wilson_dot<FP64>", fused64), kern("k_wilson<FP64>", plain64)],
                   "single_vector_launches": {"fp64": single[0], "fp32": single32[0],
                                              "note": "nrhs = 1 (Arnoldi cycles): counted, not timed, not in value"}},
        "roofline": {"bound": "hbm", "achieved": dom["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(dom["GBs"] / HBM_PEAK_GBS, 4) if dom["GBs"] else None,
                     "traffic": measured_traffic(a.workload, dom_key, dom_variant),
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a 256 MiB copy)",
                     **{k: dom[k] for k in ("kernel", "launches", "avg_launch_us", "algorithmic_bytes_per_launch")}},
        "autotuned": {"%d_%s" % (k[0], {0: "fp64", 1: "fp32", 2: "fp16s"}[k[1]]): v
                      for k, v in getattr(ctx, "tuned", {}).items()},
        "trace": {"value": [est.value.real, est.value.imag], "stderr": est.stderr, "levels": level_report(est),
                  "deflated": est.defl_k, "eigenpairs_requested": W["nev"], "pp_arnoldi_steps": plan.defl_m,
                  "ritz_pairs_tested": plan.defl_candidates,
                  "setup_s": round(est.setup_seconds, 4), "mvps": est.mvps},
        "time_to_error_s": {"mixed_batched": round(step_s, 4)},
    }

    def solve_term(e):
        L = e.levels[0]
        return {"s": round(L.seconds, 4), "mvps": L.mvps}

    def timed_runs(fn, runs):
        ts, last = [], None
        for _ in range(max(1, runs)):
            sync()
            t = time.perf_counter()
            last = fn()
            sync()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts)), ts, last

    out["solve_term"] = {"mixed_batched": solve_term(est)}
    if not a.probe_last and not a.no_probe_report and est.polys:
        # probes x degree of the exact last term against the sampled estimate's MVPs: a
        # last polynomial whose distance colouring leaves (nearly) every site its own
        # colour (the 16^4 workload's degree-255 double polynomial) is not reported
        deg = est.polys[-1].info["degree"]
        nc = mpmc.mpmc_probe_colouring(dims, deg)[3]
        probe_cost = 12 * nc * deg
        if probe_cost > 20 * est.mvps:
            out["trace"]["probed_last"] = {"skipped": "the last polynomial (degree %d) needs %d probe vectors "
                                                      "(%d MVPs, %.0fx the sampled estimate's)"
                                                      % (deg, 12 * nc, probe_cost, probe_cost / max(est.mvps, 1))}
            progress("probed-last estimate skipped (%d probes)" % (12 * nc))
    if not a.probe_last and not a.no_probe_report and "probed_last" not in out["trace"]:
        # the same estimate with the last term exact by probing (Sec. 6)
        sync()
        tq = time.perf_counter()
        ep = driver.estimate(ctx, driver.Plan(**{**plan.__dict__, "probe_last": True}), sync)
        sync()
        tq = time.perf_counter() - tq
        Lq = ep.levels[-1]
        progress("probed-last estimate done")
        out["trace"]["probed_last"] = {"value": [ep.value.real, ep.value.imag], "stderr": ep.stderr,
                                       "s": round(tq, 4), "last_term": Lq.name, "last_term_s": round(Lq.seconds, 4),
                                       "last_term_mvps": Lq.mvps, "mvps": ep.mvps}
    if W.get("deflate_double"):
        # the same estimate with the undeflated double polynomial: its level variances beside the deflated ones
        und = driver.estimate(ctx, driver.Plan(**{**plan.__dict__, "deflate_double": False}), sync)
        out["trace"]["undeflated_double"] = {"value": [und.value.real, und.value.imag], "stderr": und.stderr,
                                             "levels": level_report(und)}
    if not a.no_learned:
        ctx.release_workspace()
        torch.cuda.empty_cache()
        # learned form: the network is trained once per gauge field (timed
        # separately) and then preconditions the main solves of the estimate
        # (FP32 inner cycles: with an FP16 basis each inner cycle ends at 1e-3 of
        # its start, and the network's restarts then cost more than they save:
        # 24^4 learned solve term 0.81 s with FP32, 1.01 s with FP16S)
        lplan = driver.Plan(**{**plan.__dict__, "learned": True, "solve_inner_prec": mpmc.FP32,
                               "net_source": a.net_source, "net_steps": a.net_steps,
                               "net_batches": 2 if a.net_source == "solve" else 8})
        sync()
        tl = time.perf_counter()
        net, hist = driver.train_net(ctx, lplan)
        sync()
        t_train = time.perf_counter() - tl
        progress("network trained (%.3f s)" % t_train)
        driver.estimate(ctx, lplan, sync, net=net)
        tl, tls, el = timed_runs(lambda: driver.estimate(ctx, lplan, sync, net=net), a.compare_runs)
        out["time_to_error_s"]["learned_batched"] = round(tl, 4)
        out["time_to_error_s"]["learned_runs"] = [round(t, 4) for t in tls]
        out["time_to_error_s"]["net_training"] = round(t_train, 4)
        out["time_to_error_s"]["learned_plus_separate_training"] = round(tl + t_train, 4)
        # from scratch: each estimate trains its own network inside its set-up
        # (side stream, overlapped with the deflation and polynomial builds)
        ctx.release_workspace()
        torch.cuda.empty_cache()
        driver.estimate(ctx, lplan, sync)
        ti, tis, ei = timed_runs(lambda: driver.estimate(ctx, lplan, sync), a.compare_runs)
        progress("learned estimates with in-setup training done (%.3f s)" % ti)
        out["time_to_error_s"]["learned_batched_incl_training"] = round(ti, 4)
        out["time_to_error_s"]["learned_incl_training_runs"] = [round(t, 4) for t in tis]
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
        plain = driver.Plan(**{**plan.__dict__, "poly_prec": mpmc.FP64, "solve_inner_prec": mpmc.FP64,
                               "setup_prec": mpmc.FP64})
        driver.estimate(ctx, plain, sync)
        tp, tps, e64 = timed_runs(lambda: driver.estimate(ctx, plain, sync), a.compare_runs)
        tt = out["time_to_error_s"]
        tt["plain_fp64"] = round(tp, 4)
        tt["plain_runs"] = [round(t, 4) for t in tps]
        tt["speedup_mixed_vs_plain"] = round(tp / step_s, 3)
        if "learned_batched" in tt:
            tt["speedup_learned_vs_plain"] = round(tp / tt["learned_batched"], 3)
            tt["speedup_learned_incl_training_vs_plain"] = round(tp / tt["learned_batched_incl_training"], 3)
        out["solve_term"]["plain_fp64"] = solve_term(e64)
        comb = float(np.hypot(e64.stderr, est.stderr))
        out["trace"]["plain_fp64"] = {"value": [e64.value.real, e64.value.imag], "stderr": e64.stderr,
                                      "diff_in_combined_sigma": abs(est.value - e64.value) / comb}
        # per term: (mixed mean - FP64 mean) / FP64 standard error of the mean, same noise
        # and against the FP64 estimate's total standard error (what the bias adds to the result)
        out["trace"]["fp32_bias_in_fp64_sigma"] = [
            {"name": Lm.name, "ratio": float(abs((Lm.mean + Lm.corr) - (Lp.mean + Lp.corr)) /
                                             max(np.sqrt(Lp.var / Lp.n), 1e-300)),
             "fp64_sigma": float(np.sqrt(Lp.var / Lp.n)),
             "ratio_to_total_sigma": float(abs((Lm.mean + Lm.corr) - (Lp.mean + Lp.corr)) / max(e64.stderr, 1e-300))}
            for Lm, Lp in zip(est.levels, e64.levels)]
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(dims, kappa, links, a.cpu_seconds, est.mvps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
