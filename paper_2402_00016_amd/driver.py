"""Host-side driver of Multipolynomial Monte Carlo (Sec. 6-8).

Only bookkeeping lives here; every vector operation is a libmpmc.so call.

    Tr(Theta M^-1) = Tr(Theta(M^-1 - p_1)) + sum_l Tr(Theta(p_l - p_{l+1})) + Tr(Theta p_K)

Each term is an independent Hutchinson Monte Carlo with its own noise stream
(stream l for term l).  The polynomial-difference terms are deflated (Sec. 7)
and carry the exact correction T_l = sum_i c_i u_i^H Theta z_i; the solve term
uses the deflation set inside its solves.  The total standard error is
sqrt(sum_l s_l^2 / N_l) with s_l^2 the complex sample variance.

Random streams: level l uses stream l, the GMRES start vector of polynomial j
uses stream 0x100 + j, the deflation start vector stream 0x200.

Learned form (not in the paper): a gauge-covariant linear network N is trained
on the device on residual/error pairs recorded by training solves of the method
(r_k = eta - M x_k and e_k = x - x_k at the start of each outer cycle, eta a
Z(4) vector of seed net_seed0, net_seed0 + 1, ..., stream 0), and then
preconditions the main solves (flexible GMRES).  The solves still stop on the same FP64 true
residual, so the estimate does not depend on N.
"""
import hashlib
import json
import math
import os
import threading
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import mpmc


@dataclass
class Plan:
    """One multipolynomial estimate.

    degrees: polynomial degrees d_1 > d_2 > ... (degree D uses GMRES(D+1));
    a degree given as (din, dout) is a double polynomial from GMRES(din+1)
    inner and GMRES(dout+1) outer cycles (degree (din+1)(dout+1) - 1).
    """
    degrees: list
    noises: int = 128                    # per level (fixed-count mode)
    theta: int = mpmc.THETA_I
    seed: int = 1
    nev: int = 20                        # eigenpairs kept for deflation (0: none)
    defl_candidates: int = 40            # Ritz pairs tested for acceptance
    defl_m: int = 112                    # PP-Arnoldi steps (Aberth sweeps up to 256; the QR fallback in LDS up to 137)
    defl_pin_degree: int = 8             # degree of p_in for PP-Arnoldi
    accept_tol: float = 1e-3
    real_tol: float = 2e-4
    poly_prec: int = mpmc.FP32           # precision of the polynomial levels
    solve_inner_prec: int = mpmc.FP32    # inner precision of the main solves
    solve_tol: float = 1e-8
    solve_restart: int = 50
    max_batch: int = 0                   # right-hand sides per launch (0: all noise of a level)
    deflate_levels: bool = True
    learned: bool = False                # precondition the main solves with a trained network
    net_batches: int = 2                 # training solves ("solve") or minibatches ("random"), one Z(4) seed each
    net_pairs: int = 64                  # (r, e) pairs per minibatch
    net_steps: int = 10                  # Adam steps per minibatch
    net_lr: float = 1e-2
    net_seed0: int = 100
    net_source: str = "solve"            # "solve": snapshots of training solves; "random": (M e, e), e Z(4)
    net_snaps: int = 4                   # outer cycles recorded per training solve ("solve" source)
    net_restart: int = 20                # GMRES restart of the training solves (their basis is the
                                         # training's memory: 21 vectors of net_pairs right-hand sides)
    overlap_setup: bool = True           # build polynomials (and train the net) on side streams
    solve_pp: bool = False               # precondition the main solves with p_in (Sec. 8's PP-GMRES)
    autotune: bool = True                # time the Wilson kernel variants for the level batches once per context
    batch_levels: bool = False           # polynomial terms in shared launches (mpmc_level_estimate_multi);
                                         # off: one term's operand pair stays in the 256 MB Infinity Cache
    overlap_levels: bool = False         # polynomial terms on a side stream while the solve term runs
                                         # (8^4: 56.5 vs 58.0 ms per estimate; both streams bandwidth-bound)
    deflate_double: bool = False         # double polynomials from a deflated outer cycle (Sec. 7); the
                                         # solve level is then deflated as well when p_1 is one of them
    setup_prec: int = mpmc.FP64          # Arnoldi vectors of the polynomial and deflation builds (scalars FP64)
    graphs: bool = False                 # fused polynomial recurrences replayed from captured hipGraphs
    probe_last: bool = False             # last term Tr(Theta p_K) exactly by probing (Sec. 6) instead of sampling
    probe_batch: int = 192               # probe vectors per batch


@dataclass
class LevelResult:
    name: str
    samples: np.ndarray
    corr: complex
    mvps: int
    seconds: float
    exact: bool = False                  # one exact value (probing), no sampling variance

    @property
    def n(self):
        return len(self.samples)

    @property
    def mean(self):
        return complex(np.mean(self.samples))

    @property
    def var(self):
        if self.exact:
            return 0.0
        X = self.samples
        return float(np.sum(np.abs(X - X.mean()) ** 2) / (len(X) - 1)) if len(X) > 1 else math.inf


@dataclass
class Estimate:
    value: complex
    stderr: float
    levels: List[LevelResult]
    setup_seconds: float
    total_seconds: float
    mvps: int
    polys: list = field(default_factory=list)
    defl_k: int = 0
    info: dict = field(default_factory=dict)

    def summary(self):
        return dict(
            trace=[self.value.real, self.value.imag], stderr=self.stderr, seconds=self.total_seconds,
            setup_seconds=self.setup_seconds, mvps=self.mvps, deflated=self.defl_k,
            levels=[dict(name=L.name, n=L.n, mean=[L.mean.real, L.mean.imag], var=L.var,
                         corr=[L.corr.real, L.corr.imag], mvps=L.mvps, seconds=L.seconds)
                    for L in self.levels],
            **self.info)


def build_polys(ctx, plan: Plan, defl=None, defer_deflated=False):
    """GMRES polynomials of the plan (highest degree first).  A double
    polynomial's outer cycle is the deflated one (Sec. 7) when
    plan.deflate_double and defl holds eigenpairs.  defer_deflated: such an
    outer cycle is not run; its entry is (j, p_in) for build_deferred."""
    polys = []
    for j, deg in enumerate(plan.degrees):
        if isinstance(deg, (tuple, list)):
            din, dout = deg
            pin = ctx.gmres_poly(plan.seed, 0x100 + j, din + 1)
            if plan.deflate_double and defer_deflated:
                p = (j, pin)
            else:
                d = defl if plan.deflate_double else None
                p = ctx.gmres_poly(plan.seed, 0x100 + j, dout + 1, inner=pin, defl=d)
        else:
            p = ctx.gmres_poly(plan.seed, 0x100 + j, int(deg) + 1)
        polys.append(p)
    return polys


def build_deferred(ctx, plan: Plan, polys, defl):
    """Outer cycles left by build_polys(defer_deflated=True), now on the
    deflation set (GMRES on Q phi_in(M) from Q b)."""
    out = []
    for p in polys:
        if isinstance(p, tuple):
            j, pin = p
            dout = plan.degrees[j][1]
            p = ctx.gmres_poly(plan.seed, 0x100 + j, dout + 1, inner=pin, defl=defl)
        out.append(p)
    return out


def build_deflation(ctx, plan: Plan):
    if plan.nev <= 0:
        return None
    pin = ctx.gmres_poly(plan.seed, 0x1FF, plan.defl_pin_degree + 1) if plan.defl_pin_degree > 0 else None
    D = ctx.deflate(pin, plan.seed, 0x200, plan.defl_m, max(plan.nev, plan.defl_candidates), plan.accept_tol,
                    plan.real_tol)
    D.keep(plan.nev)
    D.p_in = pin
    return D


NET_FIELDS = (1, 2, 2, 1)


def net_identity_weights():
    """Weights for which the network is the identity map: in every layer, path 0
    maps spin s of field 0 to spin s of field 0.  Order: layer, path p < 9,
    output channel o < 4 f_out, input channel i < 4 f_in, (Re, Im)."""
    out = []
    for l in range(3):
        fin, fout = NET_FIELDS[l], NET_FIELDS[l + 1]
        W = np.zeros((9, 4 * fout, 4 * fin, 2))
        for sp in range(4):
            W[0, sp, sp, 0] = 1.0
        out.append(W.ravel())
    return np.concatenate(out)


def train_net(ctx, plan: Plan, progress=None):
    """Network trained on residual/error pairs; initial weights: identity plus a
    small seeded perturbation (so that the second field receives gradient).

    net_source "random": pairs (r, e) = (M e, e) with e a Z(4) vector of seed
    net_seed0 + b (stream 0), one minibatch of net_pairs per b < net_batches.
    net_source "solve": for b < net_batches, solve M x = eta (eta Z(4) of seed
    net_seed0 + b, FP32 inner cycles) and train on the (r_k, e_k = x - x_k)
    batches recorded at the start of each outer cycle (mpmc_solve_pairs).
    progress(b, history) is called after each seed.  Returns (net, loss history)."""
    rng = np.random.default_rng(plan.seed)
    theta0 = net_identity_weights() + 0.01 * rng.standard_normal(mpmc.mpmc_net_n_params())
    net = ctx.net(theta0)
    hist = []
    P = plan.net_pairs
    for b in range(plan.net_batches):
        if plan.net_source == "solve":
            eta = ctx.noise(plan.net_seed0 + b, 0, 0, P, mpmc.FP64)
            x, R, E, ns, vb = ctx.solve_pairs(eta, P, plan.net_snaps, tol=plan.solve_tol,
                                              restart=plan.net_restart, inner_prec=mpmc.FP32)
            for k in range(ns):
                hist.extend(net.train(R[k * vb:(k + 1) * vb], E[k * vb:(k + 1) * vb], P, plan.net_steps,
                                      plan.net_lr))
        else:
            e = ctx.noise(plan.net_seed0 + b, 0, 0, P, mpmc.FP32)
            r = ctx.apply_M(e, P, mpmc.FP32)
            hist.extend(net.train(r, e, P, plan.net_steps, plan.net_lr))
        if progress is not None:
            progress(b, hist)
    return net, np.array(hist)


def rehome_poly(ctx, p, cache=None):
    """The same polynomial (roots, inner polynomial) as a handle of ctx."""
    cache = {} if cache is None else cache
    if id(p) not in cache:
        inner = rehome_poly(ctx, p.inner, cache) if p.inner is not None else None
        q = ctx.poly_from_roots(p.roots, inner=inner)
        q.d_eff, q.relres, q.deflated = p.d_eff, p.relres, p.deflated
        cache[id(p)] = q
    return cache[id(p)]


class _SideJob:
    """fn(side_context, *args) run by a host thread on a side context and its
    own stream; the library calls release the interpreter lock, so the GPU
    work of both threads overlaps."""

    def __init__(self, ctx, name, fn, *args):
        self.side, self.stream = ctx.side(name)
        self.result, self.error = None, None
        self.thread = threading.Thread(target=self._run, args=(fn, args), daemon=True)
        self.thread.start()

    def _run(self, fn, args):
        try:
            with self.side.torch.cuda.stream(self.stream):
                self.result = fn(self.side, *args)
                self.stream.synchronize()
        except BaseException as e:   # re-raised in join()
            self.error = e

    def join(self):
        self.thread.join()
        if self.error is not None:
            raise self.error
        return self.result


def autotune_levels(ctx, plan: Plan):
    """Autotune the Wilson kernel for the batch shapes of the levels (once per
    context and shape): the polynomial levels in plan.poly_prec (the operator
    and the fused level step), the solve level's inner precision and its FP64
    residuals.  The choices are kept in ctx.tuned[(nrhs, prec)]."""
    if not plan.autotune:
        return
    done = ctx.__dict__.setdefault("tuned", {})
    nb = plan.max_batch if plan.max_batch else plan.noises
    for prec in {plan.poly_prec, plan.solve_inner_prec, mpmc.FP64}:
        if (nb, prec) not in done:
            v = ctx.autotune(nb, prec)[0]
            lv = None
            if prec == plan.poly_prec and nb % 64 == 0 and (nb <= 256 or nb % 256 == 0):
                lv = ctx.autotune_level(nb, prec)[0]
            done[(nb, prec)] = {"variant": v, "level_order": lv}


def solve_preconditioner(ctx, plan: Plan, defl):
    """p_in of the deflation build (degree plan.defl_pin_degree), or a fresh GMRES
    polynomial of that degree, when the plan asks for PP-GMRES main solves."""
    if not plan.solve_pp:
        return None
    if defl is not None and getattr(defl, "p_in", None) is not None:
        return defl.p_in
    return ctx.gmres_poly(plan.seed, 0x1FF, max(plan.defl_pin_degree, 1) + 1)


def total_mvps(ctx):
    """Operator applications issued by ctx and its side contexts."""
    return ctx.mvps + sum(c.mvps for c, _ in ctx._side.values())


def build_setup(ctx, plan: Plan, train=False):
    """Deflation set, polynomials and (optionally) the trained network.  With
    plan.overlap_setup the polynomials and the training run on side streams
    while the deflation set is built on ctx's stream."""
    autotune_levels(ctx, plan)
    for c in [ctx] + [c for c, _ in ctx._side.values()] + ([ctx.side("polys")[0]] if plan.overlap_setup else []):
        c.set_setup_precision(plan.setup_prec)
    ctx.set_graph_recurrences(int(plan.graphs))
    if not plan.overlap_setup:
        defl = build_deflation(ctx, plan)
        polys = build_polys(ctx, plan, defl)
        net, hist = train_net(ctx, plan) if train else (None, None)
        return defl, polys, net, hist
    jp = _SideJob(ctx, "polys", build_polys, plan, None, True)
    jn = _SideJob(ctx, "net", train_net, plan) if train else None
    defl = build_deflation(ctx, plan)
    cache = {}
    polys = [(p[0], rehome_poly(ctx, p[1], cache)) if isinstance(p, tuple) else rehome_poly(ctx, p, cache)
             for p in jp.join()]
    polys = build_deferred(ctx, plan, polys, defl)
    net, hist = None, None
    if jn is not None:
        snet, hist = jn.join()
        net = ctx.net(snet.weights)
    return defl, polys, net, hist


def solve_level_deflated(polys, defl):
    """The solve level M^-1 - p_1 is deflated (c_i = 1/lambda_i - p_1(lambda_i))
    when p_1 comes from a deflated outer cycle: p_1 then does not approximate
    1/lambda on the deflated eigenvalues."""
    return int(bool(polys) and getattr(polys[0], "deflated", False) and defl is not None and defl.k > 0)


def combine(levels):
    est = sum((L.mean + L.corr for L in levels), 0j)
    var = sum(L.var / L.n for L in levels)
    return est, math.sqrt(var)


def run_levels(ctx, plan: Plan, polys, defl, noises=None, first=0, net=None, skip_solve=False):
    """Samples of every term of the multipolynomial formula (skip_solve: the
    polynomial terms only)."""
    noises = plan.noises if noises is None else noises
    names = ["M^-1 - p1"] + ["p%d - p%d" % (i + 1, i + 2) for i in range(len(polys) - 1)] + ["p%d" % len(polys)]
    uppers = [None] + polys
    lowers = polys + [None]
    if plan.batch_levels and not skip_solve and len(polys) > 0 and (not plan.max_batch or plan.max_batch >= noises):
        return _run_levels_batched(ctx, plan, polys, defl, noises, first, net, names, uppers, lowers)
    out = []
    for l, (up, lo) in enumerate(zip(uppers, lowers)):
        if skip_solve and up is None:
            continue
        if plan.probe_last and up is not None and lo is None:
            out.append(probe_term(ctx, plan, up, names[l]))
            continue
        d = defl if (up is not None and lo is not None and plan.deflate_levels) else (defl if up is None else None)
        t0 = time.perf_counter()
        X, T, mv = ctx.level(up, lo, d, plan.theta, plan.seed, l, first, noises, prec=plan.poly_prec,
                             max_batch=plan.max_batch, solve_tol=plan.solve_tol, solve_restart=plan.solve_restart,
                             solve_inner_prec=plan.solve_inner_prec, net=net if up is None else None)
        out.append(LevelResult(names[l], X, T, mv, time.perf_counter() - t0))
    return out


def probe_term(ctx, plan: Plan, p, name):
    """Tr(Theta p(M)) exactly by probing with the distance colouring (Sec. 6)."""
    t0 = time.perf_counter()
    tr, nprobe, mv = ctx.poly_trace_probe(p, theta=plan.theta, prec=plan.poly_prec, max_batch=plan.probe_batch)
    return LevelResult(name + " (probed, %d probes)" % nprobe, np.array([tr]), 0j, mv, time.perf_counter() - t0,
                       exact=True)


def run_levels_overlapped(ctx, plan: Plan, polys, defl, net=None):
    """run_levels with the polynomial terms on a side context (its own stream,
    the same polynomials and deflation set) while the solve term runs on ctx:
    the same samples, the two streams' kernels overlapping."""
    dvec = None
    if defl is not None and defl.k > 0 and plan.deflate_levels:
        dvec = ctx.defl_vectors(defl)    # exported on ctx's stream before the side thread starts
        ctx.torch.cuda.synchronize()

    def side_terms(side):
        cache = {}
        sp = [rehome_poly(side, p, cache) for p in polys]
        sd = side.defl_from_arrays(*dvec) if dvec is not None else None
        return run_levels(side, plan, sp, sd, skip_solve=True)

    job = _SideJob(ctx, "levels", side_terms)
    try:
        t0 = time.perf_counter()
        X, T, mv = ctx.level(None, polys[0], defl, plan.theta, plan.seed, 0, 0, plan.noises, prec=plan.poly_prec,
                             max_batch=plan.max_batch, solve_tol=plan.solve_tol, solve_restart=plan.solve_restart,
                             solve_inner_prec=plan.solve_inner_prec, net=net)
        first = LevelResult("M^-1 - p1", X, T, mv, time.perf_counter() - t0)
    finally:
        rest = job.join()
    return [first] + rest


def _run_levels_batched(ctx, plan, polys, defl, noises, first, net, names, uppers, lowers):
    """The solve term alone, the polynomial terms in shared launches (same
    samples as one term at a time).  The batch's time and MVPs are shared out
    over its terms in proportion to their recurrence lengths."""
    t0 = time.perf_counter()
    X, T, mv = ctx.level(None, lowers[0], defl, plan.theta, plan.seed, 0, first, noises, prec=plan.poly_prec,
                         solve_tol=plan.solve_tol, solve_restart=plan.solve_restart,
                         solve_inner_prec=plan.solve_inner_prec, net=net)
    out = [LevelResult(names[0], X, T, mv, time.perf_counter() - t0)]
    t0 = time.perf_counter()
    ups, los = uppers[1:], lowers[1:]
    Xs, Ts, mv = ctx.levels_multi(ups, los, defl if plan.deflate_levels else None, plan.theta, plan.seed,
                                  list(range(1, len(ups) + 1)), first, noises, prec=plan.poly_prec)
    secs = time.perf_counter() - t0
    work = [sum(p.info["matvecs"] for p in (u, l) if p is not None) for u, l in zip(ups, los)]
    tot = max(sum(work), 1)
    for l in range(len(ups)):
        share = work[l] / tot
        out.append(LevelResult(names[l + 1], Xs[l], complex(Ts[l]), int(round(mv * share)), secs * share))
    return out


def estimate(ctx, plan: Plan, sync=None, net=None) -> Estimate:
    """Full estimate: polynomials, deflation, (network training when the plan
    is learned and no trained net is given), all levels (fixed noise counts)."""
    sync = sync or (lambda: None)
    mv0 = total_mvps(ctx)
    t0 = time.perf_counter()
    defl, polys, tnet, hist = build_setup(ctx, plan, train=plan.learned and net is None)
    info = {}
    if tnet is not None:
        net = tnet
        info = dict(net_loss=[float(hist[0]), float(hist[-1])])
    sync()
    t1 = time.perf_counter()
    pp = solve_preconditioner(ctx, plan, defl) if not plan.learned else None
    ctx.set_level_solve_poly(pp)
    ctx.set_solve_level_deflation(solve_level_deflated(polys, defl))
    try:
        if plan.overlap_levels and plan.overlap_setup and len(polys) > 0:
            levels = run_levels_overlapped(ctx, plan, polys, defl, net=net if plan.learned else None)
        else:
            levels = run_levels(ctx, plan, polys, defl, net=net if plan.learned else None)
    finally:
        ctx.set_level_solve_poly(None)
        ctx.set_solve_level_deflation(0)
    sync()
    t2 = time.perf_counter()
    est, se = combine(levels)
    return Estimate(est, se, levels, t1 - t0, t2 - t0, total_mvps(ctx) - mv0, polys=polys,
                    defl_k=defl.k if defl is not None else 0, info=info)


# ------------------------------------------------------ checkpoint / resume --
# The state of an adaptive estimate is its set-up (polynomial roots, the
# deflation set, the network weights) and the samples of every term so far.
# Noise vector i of term l is regenerated from (seed, l, i), so a resumed run
# continues each term at its next index and reproduces the samples of an
# uninterrupted run.  Files: <dir>/setup.npz (written once) and <dir>/mc.npz
# (rewritten after every batch), each replaced atomically; both hold only
# numeric and string arrays (read with allow_pickle=False).

CHECKPOINT_VERSION = 1


def _links_digest(ctx):
    d = getattr(ctx, "_links_sha256", None)
    if d is None:
        a = ctx.links
        a = a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)
        d = hashlib.sha256(memoryview(np.ascontiguousarray(a).reshape(-1).view(np.uint8))).hexdigest()
        ctx._links_sha256 = d
    return d


def plan_identity(ctx, plan: Plan):
    """JSON text naming the lattice (extents, kappa, boundary, SHA-256 of the
    links) and every plan field: a checkpoint is only resumed under the
    identical configuration."""
    fields = {k: (list(v) if isinstance(v, tuple) else v) for k, v in sorted(plan.__dict__.items())}
    return json.dumps({"version": CHECKPOINT_VERSION, "dims": list(ctx.dims), "kappa": float(ctx.kappa),
                       "t_antiperiodic": bool(ctx.t_antiperiodic), "links_sha256": _links_digest(ctx),
                       "plan": fields}, sort_keys=True, default=lambda v: list(v) if isinstance(v, tuple) else str(v))


def _atomic_savez(path, arrays):
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        np.savez(f, **arrays)
    os.replace(tmp, path)


def _check_identity(z, ident, path):
    if str(z["identity"]) != ident:
        raise ValueError("checkpoint %s was written for another lattice or plan" % path)


def save_setup(path, ctx, plan: Plan, polys, defl, net=None):
    """Polynomials (roots, inner polynomials, d_eff, relres, deflated flag), the
    deflation set (eigenvalues, right and left vectors, p_in) and the network
    weights."""
    arrays = {"identity": np.array(plan_identity(ctx, plan))}
    handles, index = [], {}

    def reg(p):
        if p is None:
            return -1
        if id(p) not in index:
            inner = reg(p.inner)
            index[id(p)] = len(handles)
            handles.append((p, inner))
        return index[id(p)]

    top = [reg(p) for p in polys]
    pin = reg(getattr(defl, "p_in", None)) if defl is not None else -1
    meta = []
    for i, (p, inner) in enumerate(handles):
        arrays["poly%d_roots" % i] = np.asarray(p.roots, dtype=np.complex128)
        meta.append({"inner": inner, "d_eff": p.d_eff, "relres": p.relres, "deflated": bool(p.deflated)})
    arrays["polys"] = np.array(json.dumps({"handles": meta, "top": top, "defl_p_in": pin,
                                           "defl_k": -1 if defl is None else int(defl.k)}))
    if defl is not None and defl.k > 0:
        lam, Z, U = ctx.defl_vectors(defl)
        arrays["defl_lam"] = np.asarray(lam, dtype=np.complex128)[:defl.k]
        arrays["defl_Z"] = Z.cpu().numpy()
        arrays["defl_U"] = U.cpu().numpy()
    if net is not None:
        arrays["net_weights"] = np.asarray(net.weights, dtype=np.float64)
    _atomic_savez(path, arrays)


def load_setup(path, ctx, plan: Plan):
    """(polys, defl, net) of save_setup as handles of ctx."""
    with np.load(path, allow_pickle=False) as z:
        _check_identity(z, plan_identity(ctx, plan), path)
        info = json.loads(str(z["polys"]))
        handles = []
        for i, m in enumerate(info["handles"]):
            inner = handles[m["inner"]] if m["inner"] >= 0 else None
            q = ctx.poly_from_roots(z["poly%d_roots" % i], inner=inner)
            q.d_eff, q.relres, q.deflated = m["d_eff"], m["relres"], m["deflated"]
            handles.append(q)
        polys = [handles[i] for i in info["top"]]
        defl = None
        if info["defl_k"] >= 0:
            if info["defl_k"] > 0:
                t = ctx.torch
                defl = ctx.defl_from_arrays(z["defl_lam"], t.from_numpy(z["defl_Z"]).cuda(),
                                            t.from_numpy(z["defl_U"]).cuda())
            else:   # an empty set keeps the deflated code paths of the original run
                t = ctx.torch
                e = t.zeros((0, ctx.n), dtype=t.complex128, device="cuda")
                defl = ctx.defl_from_arrays(np.zeros(0, dtype=np.complex128), e, e)
            defl.p_in = handles[info["defl_p_in"]] if info["defl_p_in"] >= 0 else None
        net = ctx.net(z["net_weights"]) if "net_weights" in z else None
    return polys, defl, net


def save_mc(path, ctx, plan: Plan, terms):
    """terms: one record per term begun, in order: (LevelResult, done)."""
    arrays = {"identity": np.array(plan_identity(ctx, plan))}
    meta = []
    for l, (L, done) in enumerate(terms):
        arrays["term%d_samples" % l] = np.asarray(L.samples, dtype=np.complex128)
        meta.append({"name": L.name, "corr": [L.corr.real, L.corr.imag], "mvps": int(L.mvps),
                     "seconds": float(L.seconds), "exact": bool(L.exact), "done": bool(done)})
    arrays["terms"] = np.array(json.dumps(meta))
    _atomic_savez(path, arrays)


def load_mc(path, ctx, plan: Plan):
    with np.load(path, allow_pickle=False) as z:
        _check_identity(z, plan_identity(ctx, plan), path)
        out = []
        for l, m in enumerate(json.loads(str(z["terms"]))):
            L = LevelResult(m["name"], z["term%d_samples" % l].copy(), complex(*m["corr"]), m["mvps"], m["seconds"],
                            exact=m["exact"])
            out.append((L, m["done"]))
    return out


def estimate_to_error(ctx, plan: Plan, eps: float, min_counts=(2, 3, 6), check_every=3, max_noises=4096, net=None,
                      checkpoint=None, on_batch=None):
    """Adaptive stopping (Sec. 8): each Monte Carlo term stops once its standard
    error is below eps / sqrt(#terms), with minimum counts 2 (solve term),
    3 (first difference), 6 (later terms) and checks every `check_every` noises
    (an int, or one count per term).

    checkpoint: a directory; the set-up is saved there once and the samples
    after every batch, and a run given a directory that holds them resumes
    (same lattice and plan) instead of starting over.  on_batch(term, count) is
    called after each batch has been saved."""
    mv0 = total_mvps(ctx)
    t0 = time.perf_counter()
    setup_file = mc_file = None
    if checkpoint is not None:
        os.makedirs(checkpoint, exist_ok=True)
        setup_file, mc_file = os.path.join(checkpoint, "setup.npz"), os.path.join(checkpoint, "mc.npz")
    if setup_file is not None and os.path.exists(setup_file):
        polys, defl, tnet = load_setup(setup_file, ctx, plan)
        if plan.learned and net is None and tnet is None:
            raise ValueError("checkpoint %s holds no network for a learned plan" % setup_file)
    else:
        defl, polys, tnet, _ = build_setup(ctx, plan, train=plan.learned and net is None)
        if setup_file is not None:
            save_setup(setup_file, ctx, plan, polys, defl, tnet)
    net = tnet if tnet is not None else net
    t_setup = time.perf_counter() - t0
    resume = load_mc(mc_file, ctx, plan) if mc_file is not None and os.path.exists(mc_file) else []
    nterms = len(polys) + (0 if plan.probe_last and polys else 1)
    target = eps / math.sqrt(nterms)
    levels = []
    uppers = [None] + polys
    lowers = polys + [None]
    pp = solve_preconditioner(ctx, plan, defl) if not plan.learned else None
    ctx.set_level_solve_poly(pp)
    ctx.set_solve_level_deflation(solve_level_deflated(polys, defl))
    terms = []

    def saved(l, L, done):
        if l == len(terms):
            terms.append(None)
        terms[l] = (L, done)
        if mc_file is not None:
            save_mc(mc_file, ctx, plan, terms)
        if on_batch is not None:
            on_batch(l, L.n)

    try:
        _levels_to_error(ctx, plan, defl, uppers, lowers, net, target, min_counts, check_every, max_noises, levels,
                         resume, saved)
    finally:
        ctx.set_level_solve_poly(None)
        ctx.set_solve_level_deflation(0)
    est, se = combine(levels)
    return Estimate(est, se, levels, t_setup, time.perf_counter() - t0, total_mvps(ctx) - mv0, polys=polys,
                    defl_k=defl.k if defl is not None else 0)


def _levels_to_error(ctx, plan, defl, uppers, lowers, net, target, min_counts, check_every, max_noises, levels,
                     resume=(), saved=None):
    """resume: (LevelResult, done) per term begun by an earlier run; saved(l,
    LevelResult, done) after every batch."""
    saved = saved or (lambda l, L, done: None)
    for l, (up, lo) in enumerate(zip(uppers, lowers)):
        if l < len(resume) and resume[l][1]:
            levels.append(resume[l][0])
            saved(l, resume[l][0], True)
            continue
        if plan.probe_last and up is not None and lo is None:
            levels.append(probe_term(ctx, plan, up, "term %d" % l))
            saved(l, levels[-1], True)
            continue
        d = defl if (up is not None and lo is not None and plan.deflate_levels) else (defl if up is None else None)
        n0 = min_counts[min(l, len(min_counts) - 1)]
        step = check_every if isinstance(check_every, int) else check_every[min(l, len(check_every) - 1)]
        X = np.zeros(0, dtype=np.complex128)
        corr, mv, secs = 0j, 0, 0.0
        if l < len(resume):   # a term interrupted after some batches
            X, corr, mv, secs = resume[l][0].samples, resume[l][0].corr, resume[l][0].mvps, resume[l][0].seconds
        while True:
            want = n0 if len(X) == 0 else step
            ts = time.perf_counter()
            Xn, corr, m = ctx.level(up, lo, d, plan.theta, plan.seed, l, len(X), want, prec=plan.poly_prec,
                                    solve_tol=plan.solve_tol, solve_restart=plan.solve_restart,
                                    solve_inner_prec=plan.solve_inner_prec,
                                    net=net if (up is None and plan.learned) else None)
            secs += time.perf_counter() - ts
            mv += m
            X = np.concatenate([X, Xn])
            var = np.sum(np.abs(X - X.mean()) ** 2) / (len(X) - 1) if len(X) > 1 else math.inf
            done = math.sqrt(var / len(X)) <= target or len(X) >= max_noises
            saved(l, LevelResult("term %d" % l, X, corr, mv, secs), done)
            if done:
                break
        levels.append(LevelResult("term %d" % l, X, corr, mv, secs))


# ------------------------------------------------ level-cost optimisation --
# The paper leaves the optimisation of the cost function to future work,
# naming the multilevel Monte Carlo literature (Conclusions).  With per-noise
# variances V_l and costs C_l of the terms, the noise counts that minimise the
# total cost sum_l N_l C_l under the error constraint sum_l V_l / N_l <= eps^2
# follow from a Lagrange multiplier:
#     N_l = eps^-2 sqrt(V_l / C_l) sum_k sqrt(V_k C_k),   cost = eps^-2 (sum_k sqrt(V_k C_k))^2.

def optimal_noise_counts(variances, costs, eps, min_counts=(2, 3, 6)):
    """(noise counts per term (rounded up, at least the minimum counts),
    predicted total cost) for target standard error eps."""
    V = np.asarray(variances, dtype=float)
    C = np.asarray(costs, dtype=float)
    if V.shape != C.shape or np.any(V < 0) or np.any(C <= 0) or not eps > 0:
        raise ValueError("variances >= 0, costs > 0 of equal length and eps > 0 are required")
    S = float(np.sum(np.sqrt(V * C)))
    N = np.ceil(np.sqrt(V / C) * S / eps ** 2).astype(int)
    lo = np.array([min_counts[min(l, len(min_counts) - 1)] for l in range(len(V))])
    N = np.maximum(N, lo)
    return N, float(np.sum(N * C))


def estimate_optimized(ctx, plan: Plan, eps: float, pilot: int = 16, min_counts=(2, 3, 6), net=None,
                       rounds: int = 4):
    """Estimate with cost-optimal noise counts: `pilot` noises per term give
    the variances and the per-noise MVP costs, optimal_noise_counts turns them
    into counts for standard error eps, and each term is topped up to its
    count (noise indices continue).  The variances are re-estimated from all
    samples after each top-up and the counts recomputed, for at most `rounds`
    rounds.  Returns (Estimate, noise counts used, predicted MVPs of the Monte
    Carlo part)."""
    mv0 = total_mvps(ctx)
    t0 = time.perf_counter()
    defl, polys, tnet, _ = build_setup(ctx, plan, train=plan.learned and net is None)
    net = tnet if tnet is not None else net
    t_setup = time.perf_counter() - t0
    uppers = [None] + polys
    lowers = polys + [None]
    probed = plan.probe_last and len(polys) > 0   # the last term is then exact, outside the allocation
    terms = []
    for l, (up, lo) in enumerate(zip(uppers, lowers)):
        if probed and lo is None:
            continue
        d = defl if (up is not None and lo is not None and plan.deflate_levels) else (defl if up is None else None)
        terms.append((up, lo, d))
    pp = solve_preconditioner(ctx, plan, defl) if not plan.learned else None
    ctx.set_level_solve_poly(pp)
    ctx.set_solve_level_deflation(solve_level_deflated(polys, defl))

    def run(l, first, count):
        up, lo, d = terms[l]
        ts = time.perf_counter()
        X, corr, m = ctx.level(up, lo, d, plan.theta, plan.seed, l, first, count, prec=plan.poly_prec,
                               max_batch=plan.max_batch, solve_tol=plan.solve_tol,
                               solve_restart=plan.solve_restart, solve_inner_prec=plan.solve_inner_prec,
                               net=net if (up is None and plan.learned) else None)
        return X, corr, m, time.perf_counter() - ts

    try:
        st = [list(run(l, 0, max(pilot, 2))) for l in range(len(terms))]   # [X, corr, mvps, seconds]
        predicted = 0.0
        for _ in range(rounds):
            V = [float(np.sum(np.abs(X - X.mean()) ** 2) / (len(X) - 1)) for X, _, _, _ in st]
            C = [max(m / len(X), 1e-3) for X, _, m, _ in st]
            counts, predicted = optimal_noise_counts(V, C, eps, min_counts)
            grew = False
            for l in range(len(terms)):
                extra = int(counts[l]) - len(st[l][0])
                if extra > 0:
                    Xe, corr, me, se = run(l, len(st[l][0]), extra)
                    st[l] = [np.concatenate([st[l][0], Xe]), corr, st[l][2] + me, st[l][3] + se]
                    grew = True
            if not grew:
                break
        levels = [LevelResult("term %d" % l, X, corr, m, secs) for l, (X, corr, m, secs) in enumerate(st)]
        if probed:
            levels.append(probe_term(ctx, plan, polys[-1], "term %d" % len(polys)))
    finally:
        ctx.set_level_solve_poly(None)
        ctx.set_solve_level_deflation(0)
    est, se = combine(levels)
    return (Estimate(est, se, levels, t_setup, time.perf_counter() - t0, total_mvps(ctx) - mv0, polys=polys,
                     defl_k=defl.k if defl is not None else 0), [L.n for L in levels], predicted)
