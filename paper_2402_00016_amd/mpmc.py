"""ctypes binding of libmpmc.so (C ABI in include/mpmc.h).

Argument marshalling only: every function below forwards to the C entry point
of the same name; every compute step runs in the library's HIP kernels.
Device buffers are torch tensors on the current HIP device (passed as
``data_ptr()``), and the context runs on torch's current stream unless another
stream is given.  If the library is missing this module raises at import time:
there is no CPU fallback.

torch is imported before the library is opened, so that the process holds one
HIP runtime: torch's, already loaded, satisfies libmpmc.so's dependency.
Opening libmpmc.so first would load a second HIP/HSA runtime beside torch's,
and the one that comes second can find no device.
"""
import ctypes
import os

import numpy as np
import torch  # noqa: F401  (load order, see above)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MPMC_LIB", os.path.join(HERE, "libmpmc.so"))

OK, EINVAL, ENOMEM, EHIP, ENOCONV, ENUMERIC, ESTATE = 0, -1, -2, -3, -4, -5, -6
DENSE_ABERTH, DENSE_QR = 0, 1   # eigenvalue solvers of the small dense problems
FP64, FP32, FP16S = 0, 1, 2
THETA_I, THETA_G5 = 0, 1
TIMING_PLAIN, TIMING_FUSED, TIMING_SINGLE = 16, 32, 64   # or-ed into the precision of mpmc_timing_read
PREC = {"fp64": FP64, "fp32": FP32, "fp16s": FP16S}
THETA = {"I": THETA_I, "g5": THETA_G5}

if not os.path.exists(LIB_PATH):
    raise ImportError("libmpmc.so not found at %s: build it with `python -m paper_2402_00016_amd.build` "
                      "(there is no CPU fallback)" % LIB_PATH)

_L = ctypes.CDLL(LIB_PATH)
_vp, _i, _u32, _u64, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
_pi, _pd, _pu64, _psz = (ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_size_t))

_SIGS = {
    "mpmc_create": ([_pi, _d, _i, _vp, _vp, ctypes.POINTER(_vp)], _i),
    "mpmc_destroy": ([_vp], None),
    "mpmc_last_error": ([_vp], ctypes.c_char_p),
    "mpmc_set_stream": ([_vp, _vp], _i),
    "mpmc_vector_bytes": ([_vp, _i, _i, _psz], _i),
    "mpmc_mvp_count": ([_vp, _pu64], _i),
    "mpmc_mvp_reset": ([_vp], _i),
    "mpmc_timing_enable": ([_vp, _i], _i),
    "mpmc_timing_read": ([_vp, _i, _pu64, _pd, _pd], _i),
    "mpmc_pack": ([_vp, _vp, _vp, _i, _i], _i),
    "mpmc_unpack": ([_vp, _vp, _vp, _i, _i], _i),
    "mpmc_noise": ([_vp, _u64, _u32, _u64, _i, _i, _vp], _i),
    "mpmc_apply_M": ([_vp, _vp, _vp, _i, _i, _i, _i], _i),
    "mpmc_gmres_poly": ([_vp, _vp, _vp, _u64, _u32, _i, ctypes.POINTER(_vp), _pi, _pd], _i),
    "mpmc_poly_create": ([_vp, _vp, _i, _vp, ctypes.POINTER(_vp)], _i),
    "mpmc_poly_roots": ([_vp, _vp, _pi], _i),
    "mpmc_poly_info": ([_vp, _pi, _pi, _pi, _pi], _i),
    "mpmc_poly_eval": ([_vp, _vp, _vp, _i], _i),
    "mpmc_poly_destroy": ([_vp], None),
    "mpmc_poly_add_roots": ([_vp, _d, _d, _pi], _i),
    "mpmc_apply_poly": ([_vp, _vp, _vp, _vp, _i, _i], _i),
    "mpmc_apply_poly_noalloc": ([_vp, _vp, _vp, _vp, _i, _i], _i),
    "mpmc_poly_trace": ([_vp, _vp, _i, _pi, _i, _i, _vp, _pi, _pu64], _i),
    "mpmc_deflate": ([_vp, _vp, _u64, _u32, _i, _i, _d, _d, ctypes.POINTER(_vp), _pi], _i),
    "mpmc_defl_create": ([_vp, _vp, _vp, _vp, _i, ctypes.POINTER(_vp)], _i),
    "mpmc_defl_export": ([_vp, _vp, _vp, _vp, _pi], _i),
    "mpmc_defl_destroy": ([_vp], None),
    "mpmc_defl_keep": ([_vp, _i], _i),
    "mpmc_solve": ([_vp, _vp, _vp, _i, _vp, _vp, _i, _d, _i, _i, _pi, _vp], _i),
    "mpmc_autotune": ([_vp, _i, _i, _pi, _vp], _i),
    "mpmc_autotune_level": ([_vp, _i, _i, _pi, _vp], _i),
    "mpmc_wilson_variant_count": ([], _i),
    "mpmc_apply_M_batch": ([_vp, _vp, _vp, _i, _i, _i, _i, _i], _i),
    "mpmc_solve_batch": ([_vp, _i, _vp, _vp, _i, _vp, _vp, _i, _d, _i, _i, _vp, _vp], _i),
    "mpmc_release_workspace": ([_vp], _i),
    "mpmc_tune_set": ([_vp, _i, _i, _i], _i),
    "mpmc_net_n_params": ([], _i),
    "mpmc_net_create": ([_vp, _vp, ctypes.POINTER(_vp)], _i),
    "mpmc_net_destroy": ([_vp], None),
    "mpmc_net_set_weights": ([_vp, _vp], _i),
    "mpmc_net_get_weights": ([_vp, _vp], _i),
    "mpmc_net_apply": ([_vp, _vp, _vp, _i], _i),
    "mpmc_net_loss_grad": ([_vp, _vp, _vp, _i, _pd, _vp], _i),
    "mpmc_net_train": ([_vp, _vp, _vp, _i, _i, _d, _vp], _i),
    "mpmc_solve_pp": ([_vp, _vp, _vp, _i, _vp, _vp, _i, _d, _i, _i, _pi, _vp], _i),
    "mpmc_set_level_solve_poly": ([_vp, _vp], _i),
    "mpmc_set_dense_method": ([_vp, _i], _i),
    "mpmc_set_solve_level_deflation": ([_vp, _i], _i),
    "mpmc_set_site_order": ([_vp, _vp], _i),
    "mpmc_set_setup_precision": ([_vp, _i], _i),
    "mpmc_set_arnoldi_cgs2": ([_vp, _i], _i),
    "mpmc_set_solve_gs_passes": ([_vp, _i], _i),
    "mpmc_set_graph_recurrences": ([_vp, _i], _i),
    "mpmc_graph_replays": ([_vp, _pu64, _pi], _i),
    "mpmc_probe_colouring": ([_pi, _i, _pi, _pi, _pi, ctypes.POINTER(ctypes.c_long)], _i),
    "mpmc_poly_trace_probe": ([_vp, _vp, _i, _i, _i, _vp, ctypes.POINTER(ctypes.c_long), _pu64], _i),
    "mpmc_solve_pairs": ([_vp, _vp, _vp, _i, _vp, _i, _d, _i, _i, _vp, _vp, _i, _pi, _pi, _vp], _i),
    "mpmc_level_estimate": ([_vp, _vp, _vp, _vp, _i, _u64, _u32, _u64, _i, _i, _i, _d, _i, _i, _vp, _vp, _vp,
                             _pu64], _i),
    "mpmc_level_estimate_multi": ([_vp, _i, _vp, _vp, _vp, _i, _u64, _vp, _u64, _i, _i, _vp, _vp, _vp], _i),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_L, _name)
    _f.argtypes = _args
    _f.restype = _res


class MpmcError(RuntimeError):
    def __init__(self, rc, msg):
        super().__init__("mpmc error %d: %s" % (rc, msg))
        self.rc = rc


def _check(rc, ctx):
    if rc != OK:
        msg = _L.mpmc_last_error(ctx)
        raise MpmcError(rc, msg.decode() if msg else "")
    return rc


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _h(obj):
    return None if obj is None else obj.handle


# ------------------------------------------------------------- same-name calls

def mpmc_create(dims, kappa, t_antiperiodic, links_host, stream=None):
    links = np.ascontiguousarray(links_host, dtype=np.complex128)
    d = (ctypes.c_int * 4)(*[int(v) for v in dims])
    out = _vp()
    _check(_L.mpmc_create(d, float(kappa), int(t_antiperiodic), links.ctypes.data, stream, ctypes.byref(out)), None)
    return out


def mpmc_destroy(ctx):
    _L.mpmc_destroy(ctx)


def mpmc_last_error(ctx):
    m = _L.mpmc_last_error(ctx)
    return m.decode() if m else ""


def mpmc_vector_bytes(ctx, nrhs, prec):
    b = ctypes.c_size_t()
    _check(_L.mpmc_vector_bytes(ctx, int(nrhs), int(prec), ctypes.byref(b)), ctx)
    return b.value


def mpmc_mvp_count(ctx):
    v = ctypes.c_uint64()
    _check(_L.mpmc_mvp_count(ctx, ctypes.byref(v)), ctx)
    return v.value


def mpmc_mvp_reset(ctx):
    _check(_L.mpmc_mvp_reset(ctx), ctx)


def mpmc_timing_enable(ctx, on):
    _check(_L.mpmc_timing_enable(ctx, int(on)), ctx)


def mpmc_timing_read(ctx, prec):
    n, ms, by = ctypes.c_uint64(), ctypes.c_double(), ctypes.c_double()
    _check(_L.mpmc_timing_read(ctx, int(prec), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)), ctx)
    return n.value, ms.value, by.value


def mpmc_pack(ctx, canon, internal, nrhs, prec):
    _check(_L.mpmc_pack(ctx, _ptr(canon), _ptr(internal), int(nrhs), int(prec)), ctx)


def mpmc_unpack(ctx, internal, canon, nrhs, prec):
    _check(_L.mpmc_unpack(ctx, _ptr(internal), _ptr(canon), int(nrhs), int(prec)), ctx)


def mpmc_noise(ctx, seed, stream, first, nrhs, prec, internal):
    _check(_L.mpmc_noise(ctx, int(seed), int(stream), int(first), int(nrhs), int(prec), _ptr(internal)), ctx)


def mpmc_apply_M(ctx, x, y, nrhs, prec, dagger=0, theta=THETA_I):
    _check(_L.mpmc_apply_M(ctx, _ptr(x), _ptr(y), int(nrhs), int(prec), int(dagger), int(theta)), ctx)


def mpmc_gmres_poly(ctx, inner, defl, seed, stream, d):
    out, de, rr = _vp(), ctypes.c_int(), ctypes.c_double()
    _check(_L.mpmc_gmres_poly(ctx, _h(inner), _h(defl), int(seed), int(stream), int(d), ctypes.byref(out),
                              ctypes.byref(de), ctypes.byref(rr)), ctx)
    return out, de.value, rr.value


def mpmc_poly_create(ctx, roots, inner=None):
    r = np.ascontiguousarray(roots, dtype=np.complex128)
    out = _vp()
    _check(_L.mpmc_poly_create(ctx, r.ctypes.data, len(r), _h(inner), ctypes.byref(out)), ctx)
    return out


def mpmc_poly_roots(handle):
    d = ctypes.c_int(0)
    _check(_L.mpmc_poly_roots(handle, None, ctypes.byref(d)), None)
    r = np.zeros(d.value, dtype=np.complex128)
    _check(_L.mpmc_poly_roots(handle, r.ctypes.data, ctypes.byref(d)), None)
    return r


def mpmc_poly_info(handle):
    v = [ctypes.c_int() for _ in range(4)]
    _check(_L.mpmc_poly_info(handle, *[ctypes.byref(x) for x in v]), None)
    return dict(d=v[0].value, d_inner=v[1].value, degree=v[2].value, matvecs=v[3].value)


def mpmc_poly_eval(handle, lam):
    lam = np.ascontiguousarray(np.atleast_1d(lam), dtype=np.complex128)
    out = np.zeros_like(lam)
    _check(_L.mpmc_poly_eval(handle, lam.ctypes.data, out.ctypes.data, len(lam)), None)
    return out


def mpmc_poly_destroy(handle):
    _L.mpmc_poly_destroy(handle)


def mpmc_apply_poly(ctx, poly, x, y, nrhs, prec):
    _check(_L.mpmc_apply_poly(ctx, _h(poly), _ptr(x), _ptr(y), int(nrhs), int(prec)), ctx)


def mpmc_apply_poly_noalloc(ctx, poly, x, y, nrhs, prec):
    _check(_L.mpmc_apply_poly_noalloc(ctx, _h(poly), _ptr(x), _ptr(y), int(nrhs), int(prec)), ctx)


def mpmc_poly_trace(ctx, poly, theta, period, prec, max_batch=0):
    per = (ctypes.c_int * 4)(*[int(v) for v in period])
    tr = np.zeros(1, dtype=np.complex128)
    exact, mvps = ctypes.c_int(), ctypes.c_uint64()
    _check(_L.mpmc_poly_trace(ctx, _h(poly), int(theta), per, int(prec), int(max_batch), tr.ctypes.data,
                              ctypes.byref(exact), ctypes.byref(mvps)), ctx)
    return complex(tr[0]), bool(exact.value), mvps.value


def mpmc_probe_colouring(dims, distance):
    """(k, moduli[k], W[k][4], number of colours) of the distance colouring (host only)."""
    d = (ctypes.c_int * 4)(*[int(v) for v in dims])
    k, m, W, nc = ctypes.c_int(), (ctypes.c_int * 4)(), (ctypes.c_int * 16)(), ctypes.c_long()
    rc = _L.mpmc_probe_colouring(d, int(distance), ctypes.byref(k), m, W, ctypes.byref(nc))
    if rc != OK:
        raise MpmcError(rc, "mpmc_probe_colouring: bad argument")
    kk = k.value
    return kk, list(m)[:kk], [list(W)[4 * i:4 * i + 4] for i in range(kk)], nc.value


def mpmc_poly_trace_probe(ctx, poly, theta, prec, max_batch=0):
    tr = np.zeros(1, dtype=np.complex128)
    npr, mvps = ctypes.c_long(), ctypes.c_uint64()
    _check(_L.mpmc_poly_trace_probe(ctx, _h(poly), int(theta), int(prec), int(max_batch), tr.ctypes.data,
                                    ctypes.byref(npr), ctypes.byref(mvps)), ctx)
    return complex(tr[0]), npr.value, mvps.value


def mpmc_deflate(ctx, p_in, seed, stream, m, nev, accept_tol=1e-3, real_tol=2e-4):
    out, k = _vp(), ctypes.c_int()
    _check(_L.mpmc_deflate(ctx, _h(p_in), int(seed), int(stream), int(m), int(nev), float(accept_tol),
                           float(real_tol), ctypes.byref(out), ctypes.byref(k)), ctx)
    return out, k.value


def mpmc_defl_create(ctx, lam, Z, U):
    lam = np.ascontiguousarray(lam, dtype=np.complex128)
    out = _vp()
    _check(_L.mpmc_defl_create(ctx, lam.ctypes.data if len(lam) else None, _ptr(Z), _ptr(U), len(lam),
                               ctypes.byref(out)), ctx)
    return out


def mpmc_defl_export(handle, Z=None, U=None):
    k = ctypes.c_int()
    _check(_L.mpmc_defl_export(handle, None, None, None, ctypes.byref(k)), None)
    lam = np.zeros(k.value, dtype=np.complex128)
    _check(_L.mpmc_defl_export(handle, lam.ctypes.data if k.value else None, _ptr(Z), _ptr(U), ctypes.byref(k)), None)
    return lam


def mpmc_defl_keep(handle, k):
    _check(_L.mpmc_defl_keep(handle, int(k)), None)


def mpmc_defl_destroy(handle):
    _L.mpmc_defl_destroy(handle)


def mpmc_solve(ctx, b, x, nrhs, defl=None, net=None, restart=50, tol=1e-8, inner_prec=FP64, max_outer=100,
               raise_on_noconv=True):
    its = ctypes.c_int()
    rel = np.zeros(nrhs)
    rc = _L.mpmc_solve(ctx, _ptr(b), _ptr(x), int(nrhs), _h(defl), _h(net), int(restart), float(tol),
                       int(inner_prec), int(max_outer), ctypes.byref(its), rel.ctypes.data)
    if rc != ENOCONV or raise_on_noconv:
        _check(rc, ctx)
    return its.value, rel, rc


def mpmc_solve_pp(ctx, b, x, nrhs, defl, pp, restart=50, tol=1e-8, inner_prec=FP64, max_outer=100):
    its = ctypes.c_int()
    rel = np.zeros(nrhs)
    _check(_L.mpmc_solve_pp(ctx, _ptr(b), _ptr(x), int(nrhs), _h(defl), _h(pp), int(restart), float(tol),
                            int(inner_prec), int(max_outer), ctypes.byref(its), rel.ctypes.data), ctx)
    return its.value, rel


def mpmc_set_level_solve_poly(ctx, pp):
    _check(_L.mpmc_set_level_solve_poly(ctx, _h(pp)), ctx)


def mpmc_set_site_order(ctx, order):
    if order is None:
        _check(_L.mpmc_set_site_order(ctx, None), ctx)
        return
    o = np.ascontiguousarray(order, dtype=np.int32)
    _check(_L.mpmc_set_site_order(ctx, o.ctypes.data), ctx)


def mpmc_set_graph_recurrences(ctx, on):
    _check(_L.mpmc_set_graph_recurrences(ctx, int(on)), ctx)


def mpmc_graph_replays(ctx):
    r, g = ctypes.c_uint64(), ctypes.c_int()
    _check(_L.mpmc_graph_replays(ctx, ctypes.byref(r), ctypes.byref(g)), ctx)
    return r.value, g.value


def mpmc_set_setup_precision(ctx, prec):
    _check(_L.mpmc_set_setup_precision(ctx, int(prec)), ctx)


def mpmc_set_solve_level_deflation(ctx, on):
    _check(_L.mpmc_set_solve_level_deflation(ctx, int(on)), ctx)


def mpmc_set_dense_method(ctx, method):
    _check(_L.mpmc_set_dense_method(ctx, int(method)), ctx)


def mpmc_solve_pairs(ctx, b, x, nrhs, defl, restart, tol, inner_prec, max_outer, R, E, max_snap):
    its, ns = ctypes.c_int(), ctypes.c_int()
    rel = np.zeros(nrhs)
    _check(_L.mpmc_solve_pairs(ctx, _ptr(b), _ptr(x), int(nrhs), _h(defl), int(restart), float(tol), int(inner_prec),
                               int(max_outer), _ptr(R), _ptr(E), int(max_snap), ctypes.byref(ns), ctypes.byref(its),
                               rel.ctypes.data), ctx)
    return ns.value, its.value, rel


def mpmc_level_estimate_multi(ctx, uppers, lowers, defl, theta, seed, streams, first, nnoise, prec):
    """Polynomial terms (upper non-None) in shared launches: (samples [nterms, nnoise], corr [nterms], mvps)."""
    T = len(uppers)
    up = (ctypes.c_void_p * T)(*[_h(p) for p in uppers])
    lo = (ctypes.c_void_p * T)(*[_h(p) for p in lowers])
    st = (ctypes.c_uint32 * T)(*[int(x) for x in streams])
    samples = np.zeros((T, nnoise), dtype=np.complex128)
    corr = np.zeros(T, dtype=np.complex128)
    mvps = ctypes.c_uint64()
    _check(_L.mpmc_level_estimate_multi(ctx, T, up, lo, _h(defl), int(theta), int(seed), st, int(first), int(nnoise),
                                        int(prec), samples.ctypes.data, corr.ctypes.data, ctypes.byref(mvps)), ctx)
    return samples, corr, mvps.value


def mpmc_level_estimate(ctx, upper, lower, defl, theta, seed, stream, first, nnoise, prec, max_batch=0,
                        solve_tol=1e-8, solve_restart=50, solve_inner_prec=FP64, net=None):
    samples = np.zeros(nnoise, dtype=np.complex128)
    corr = np.zeros(1, dtype=np.complex128)
    mvps = ctypes.c_uint64()
    _check(_L.mpmc_level_estimate(ctx, _h(upper), _h(lower), _h(defl), int(theta), int(seed), int(stream),
                                  int(first), int(nnoise), int(prec), int(max_batch), float(solve_tol),
                                  int(solve_restart), int(solve_inner_prec), _h(net), samples.ctypes.data,
                                  corr.ctypes.data, ctypes.byref(mvps)), ctx)
    return samples, complex(corr[0]), mvps.value


WILSON_VARIANTS = _L.mpmc_wilson_variant_count()   # kernel variants of the multi-RHS Wilson kernel


def mpmc_autotune_level(ctx, nrhs, prec):
    """(chosen traversal order, microseconds per fused step for orders 0..7; 0 = not a candidate)."""
    o = ctypes.c_int()
    us = np.zeros(8)
    _check(_L.mpmc_autotune_level(ctx, int(nrhs), int(prec), ctypes.byref(o), us.ctypes.data), ctx)
    return o.value, us


def mpmc_autotune(ctx, nrhs, prec):
    v = ctypes.c_int()
    us = np.zeros(WILSON_VARIANTS)
    _check(_L.mpmc_autotune(ctx, int(nrhs), int(prec), ctypes.byref(v), us.ctypes.data), ctx)
    return v.value, us


def mpmc_apply_M_batch(ctxs, xs, ys, nrhs, prec, dagger=False, theta=THETA_I):
    n = len(ctxs)
    ch = (ctypes.c_void_p * n)(*[c for c in ctxs])
    xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
    yp = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ys])
    _check(_L.mpmc_apply_M_batch(ch, xp, yp, n, int(nrhs), int(prec), int(dagger), int(theta)), ctxs[0])


def mpmc_solve_batch(ctxs, bs, xs, nrhs, defls=None, nets=None, restart=50, tol=1e-8, inner_prec=FP32,
                     max_outer=100):
    """Lockstep solves of several contexts; returns (iterations per context, relres [count, nrhs])."""
    n = len(ctxs)
    vp = ctypes.c_void_p * n
    its = np.zeros(n, dtype=np.int32)
    rel = np.zeros((n, nrhs))
    dl = vp(*[_h(d) for d in defls]) if defls is not None else None
    nl = vp(*[_h(t) for t in nets]) if nets is not None else None
    rc = _L.mpmc_solve_batch(vp(*ctxs), n, vp(*[b.data_ptr() for b in bs]), vp(*[x.data_ptr() for x in xs]),
                             int(nrhs), dl, nl, int(restart), float(tol), int(inner_prec), int(max_outer),
                             its.ctypes.data, rel.ctypes.data)
    _check(rc, ctxs[0])
    return its, rel


def mpmc_tune_set(ctx, nrhs, prec, variant):
    _check(_L.mpmc_tune_set(ctx, int(nrhs), int(prec), int(variant)), ctx)


def mpmc_net_n_params():
    return _L.mpmc_net_n_params()


def mpmc_net_create(ctx, theta):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if th.size != mpmc_net_n_params():
        raise ValueError("network weights: %d values, expected %d" % (th.size, mpmc_net_n_params()))
    out = _vp()
    _check(_L.mpmc_net_create(ctx, th.ctypes.data, ctypes.byref(out)), ctx)
    return out


def mpmc_net_destroy(handle):
    _L.mpmc_net_destroy(handle)


def mpmc_net_set_weights(handle, theta):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if th.size != mpmc_net_n_params():
        raise ValueError("network weights: %d values, expected %d" % (th.size, mpmc_net_n_params()))
    _check(_L.mpmc_net_set_weights(handle, th.ctypes.data), None)


def mpmc_net_get_weights(handle):
    th = np.zeros(mpmc_net_n_params())
    _check(_L.mpmc_net_get_weights(handle, th.ctypes.data), None)
    return th


def mpmc_net_apply(handle, x, y, nrhs):
    _check(_L.mpmc_net_apply(handle, _ptr(x), _ptr(y), int(nrhs)), None)


def mpmc_net_loss_grad(handle, R, E, npairs):
    loss = ctypes.c_double()
    grad = np.zeros(mpmc_net_n_params())
    _check(_L.mpmc_net_loss_grad(handle, _ptr(R), _ptr(E), int(npairs), ctypes.byref(loss), grad.ctypes.data), None)
    return loss.value, grad


def mpmc_net_train(handle, R, E, npairs, steps, lr):
    hist = np.zeros(int(steps))
    _check(_L.mpmc_net_train(handle, _ptr(R), _ptr(E), int(npairs), int(steps), float(lr), hist.ctypes.data), None)
    return hist


# ---------------------------------------------------------- object wrappers

class _Handle:
    """Owns a library handle and frees it with the matching _destroy call."""

    _destroy = None

    def __init__(self, handle, owner):
        self.handle = handle
        self.owner = owner      # keeps the context (and inner polynomials) alive

    def close(self):
        if self.handle is not None and self.handle.value:
            type(self)._destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mpmc_poly_add_roots(handle, log10_threshold=4.0, digits=14.0):
    added = ctypes.c_int()
    _check(_L.mpmc_poly_add_roots(handle, float(log10_threshold), float(digits), ctypes.byref(added)), None)
    return added.value


class Poly(_Handle):
    _destroy = staticmethod(mpmc_poly_destroy)

    def add_roots(self, log10_threshold=4.0, digits=14.0):
        """Added-roots stabilisation (in place); returns the number of roots added."""
        return mpmc_poly_add_roots(self.handle, log10_threshold, digits)

    def __init__(self, handle, owner, inner=None, d_eff=None, relres=None):
        super().__init__(handle, owner)
        self.inner = inner
        self.d_eff = d_eff
        self.relres = relres
        self.deflated = False      # outer cycle built with a deflation set

    @property
    def roots(self):
        return mpmc_poly_roots(self.handle)

    @property
    def info(self):
        return mpmc_poly_info(self.handle)

    def eval(self, lam):
        return mpmc_poly_eval(self.handle, lam)


class Net(_Handle):
    """Learned right preconditioner (gauge-covariant linear network)."""
    _destroy = staticmethod(mpmc_net_destroy)

    @property
    def weights(self):
        return mpmc_net_get_weights(self.handle)

    @weights.setter
    def weights(self, theta):
        mpmc_net_set_weights(self.handle, theta)

    def apply(self, x, nrhs, out=None):
        """y = N(x) for FP32 internal-layout batches."""
        y = self.owner.vector(nrhs, FP32) if out is None else out
        mpmc_net_apply(self.handle, x, y, nrhs)
        return y

    def loss_grad(self, R, E, npairs):
        return mpmc_net_loss_grad(self.handle, R, E, npairs)

    def train(self, R, E, npairs, steps, lr):
        return mpmc_net_train(self.handle, R, E, npairs, steps, lr)


class Defl(_Handle):
    _destroy = staticmethod(mpmc_defl_destroy)

    def __init__(self, handle, owner, k):
        super().__init__(handle, owner)
        self.k = k

    @property
    def lam(self):
        return mpmc_defl_export(self.handle)

    def keep(self, k):
        mpmc_defl_keep(self.handle, k)
        self.k = min(self.k, int(k))


class Context:
    """One lattice on the current HIP device (torch tensors as device buffers)."""

    def __init__(self, dims, kappa, links, t_antiperiodic=True, stream=None):
        import torch
        self.torch = torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.n = 12 * self.V
        self.kappa = float(kappa)
        self.links = links
        self.t_antiperiodic = bool(t_antiperiodic)
        self.stream = stream
        self.handle = mpmc_create(self.dims, kappa, t_antiperiodic, links, ctypes.c_void_p(stream))
        self._side = {}

    def side(self, name):
        """A second context on the same lattice with its own HIP stream (default
        priority), for independent work that can overlap with this context's.
        Returns (context, torch stream); cached per name."""
        if name not in self._side:
            st = self.torch.cuda.Stream()
            self._side[name] = (Context(self.dims, self.kappa, self.links, self.t_antiperiodic, st.cuda_stream), st)
        return self._side[name]

    def close(self):
        for c, _ in getattr(self, "_side", {}).values():
            c.close()
        if getattr(self, "handle", None) is not None and self.handle.value:
            mpmc_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # buffers
    def vector(self, nrhs, prec=FP64):
        return self.torch.empty(mpmc_vector_bytes(self.handle, nrhs, prec), dtype=self.torch.uint8, device="cuda")

    def pack(self, canon, prec=FP64):
        """canon: complex128 tensor (nrhs, n) on the device -> internal buffer."""
        canon = canon.contiguous()
        nrhs = canon.shape[0]
        out = self.vector(nrhs, prec)
        mpmc_pack(self.handle, canon, out, nrhs, prec)
        return out

    def unpack(self, internal, nrhs, prec=FP64):
        out = self.torch.empty((nrhs, self.n), dtype=self.torch.complex128, device="cuda")
        mpmc_unpack(self.handle, internal, out, nrhs, prec)
        return out

    def noise(self, seed, stream, first, nrhs, prec=FP64):
        out = self.vector(nrhs, prec)
        mpmc_noise(self.handle, seed, stream, first, nrhs, prec, out)
        return out

    def apply_M(self, x, nrhs, prec=FP64, dagger=False, theta=THETA_I, out=None):
        y = self.vector(nrhs, prec) if out is None else out
        mpmc_apply_M(self.handle, x, y, nrhs, prec, int(dagger), theta)
        return y

    @staticmethod
    def apply_M_batch(ctxs, xs, nrhs, prec=FP32, dagger=False, theta=THETA_I, outs=None):
        """y[i] = M_i x[i] for several contexts (lattices) in one launch on the
        first context's stream."""
        ys = [c.vector(nrhs, prec) for c in ctxs] if outs is None else outs
        mpmc_apply_M_batch([c.handle for c in ctxs], xs, ys, nrhs, prec, dagger, theta)
        return ys

    @property
    def mvps(self):
        return mpmc_mvp_count(self.handle)

    # polynomials
    def gmres_poly(self, seed, stream, d, inner=None, defl=None):
        h, de, rr = mpmc_gmres_poly(self.handle, inner, defl, seed, stream, d)
        P = Poly(h, (self, inner, defl), inner=inner, d_eff=de, relres=rr)
        P.deflated = defl is not None and defl.k > 0
        return P

    def poly_from_roots(self, roots, inner=None):
        return Poly(mpmc_poly_create(self.handle, roots, inner), (self, inner), inner=inner)

    def apply_poly(self, poly, x, nrhs, prec=FP64, out=None):
        y = self.vector(nrhs, prec) if out is None else out
        mpmc_apply_poly(self.handle, poly, x, y, nrhs, prec)
        return y

    def poly_trace(self, poly, theta=THETA_I, period=None, prec=FP64, max_batch=0):
        """Exact Tr(Theta p(M)) by probing; period None = every site its own colour."""
        period = self.dims if period is None else period
        return mpmc_poly_trace(self.handle, poly, theta, period, prec, max_batch)

    # deflation
    def poly_trace_probe(self, poly, theta=THETA_I, prec=FP64, max_batch=0):
        """Exact Tr(Theta p(M)) with the distance-(deg p + 1) colouring:
        (trace, probe vectors, MVPs)."""
        return mpmc_poly_trace_probe(self.handle, poly, theta, prec, max_batch)

    def deflate(self, p_in, seed, stream, m, nev, accept_tol=1e-3, real_tol=2e-4):
        h, k = mpmc_deflate(self.handle, p_in, seed, stream, m, nev, accept_tol, real_tol)
        return Defl(h, (self, p_in), k)

    def defl_from_arrays(self, lam, Z, U):
        return Defl(mpmc_defl_create(self.handle, lam, Z, U), self, len(lam))

    def defl_vectors(self, defl):
        Z = self.torch.empty((max(defl.k, 1), self.n), dtype=self.torch.complex128, device="cuda")
        U = self.torch.empty_like(Z)
        lam = mpmc_defl_export(defl.handle, Z, U)
        return lam, Z[:defl.k], U[:defl.k]

    # solves and levels
    def release_workspace(self):
        """Free the library's cached device workspace of this context and its side contexts."""
        for c, _ in self._side.values():
            c.release_workspace()
        _check(_L.mpmc_release_workspace(self.handle), self.handle)

    def autotune(self, nrhs, prec=FP32):
        """Pick the fastest Wilson kernel variant for (nrhs, prec) -> (variant, us per variant)."""
        return mpmc_autotune(self.handle, nrhs, prec)

    def autotune_level(self, nrhs, prec=FP32):
        return mpmc_autotune_level(self.handle, nrhs, prec)

    def tune_set(self, nrhs, prec, variant):
        mpmc_tune_set(self.handle, nrhs, prec, variant)

    def net(self, theta):
        return Net(mpmc_net_create(self.handle, theta), self)

    def solve(self, b, nrhs, defl=None, restart=50, tol=1e-8, inner_prec=FP64, max_outer=100, x=None, net=None):
        x = self.vector(nrhs, FP64) if x is None else x
        its, rel, rc = mpmc_solve(self.handle, b, x, nrhs, defl, net, restart, tol, inner_prec, max_outer)
        return x, its, rel

    @staticmethod
    def solve_batch(ctxs, bs, nrhs, defls=None, nets=None, restart=50, tol=1e-8, inner_prec=FP32, max_outer=100):
        """Solves of several contexts in lockstep, one batched Wilson launch per
        inner iteration; returns (xs, iterations per context, relres)."""
        xs = [c.vector(nrhs, FP64) for c in ctxs]
        its, rel = mpmc_solve_batch([c.handle for c in ctxs], bs, xs, nrhs, defls, nets, restart, tol, inner_prec,
                                    max_outer)
        return xs, its, rel

    def solve_pp(self, b, nrhs, pp, defl=None, restart=50, tol=1e-8, inner_prec=FP64, max_outer=100, x=None):
        x = self.vector(nrhs, FP64) if x is None else x
        its, rel = mpmc_solve_pp(self.handle, b, x, nrhs, defl, pp, restart, tol, inner_prec, max_outer)
        return x, its, rel

    def set_dense_method(self, method):
        """Small eigenproblems: DENSE_ABERTH (default, QR fallback) or DENSE_QR."""
        mpmc_set_dense_method(self.handle, method)

    def set_site_order(self, order):
        """Traversal order of the blocked Wilson kernels (None: the default)."""
        mpmc_set_site_order(self.handle, order)

    def set_graph_recurrences(self, on):
        """Replay the fused polynomial recurrences from captured hipGraphs."""
        mpmc_set_graph_recurrences(self.handle, on)

    def set_arnoldi_cgs2(self, on):
        """1: plain CGS2 in the set-up Arnoldi cycles; 0: CGS2 with the second projection delayed;
        -1 (default): by lattice size."""
        _check(_L.mpmc_set_arnoldi_cgs2(self.handle, int(on)), self.handle)

    def set_solve_gs_passes(self, passes):
        """Projections per inner GMRES step of the solves: 1, 2, or 0 (default: 1 for FP32/FP16S
        inner cycles, 2 for FP64)."""
        _check(_L.mpmc_set_solve_gs_passes(self.handle, int(passes)), self.handle)

    def set_setup_precision(self, prec):
        """Storage of the Arnoldi vectors of gmres_poly and deflate (FP64 or FP32)."""
        mpmc_set_setup_precision(self.handle, prec)

    def set_solve_level_deflation(self, on):
        """Deflate the solve level M^-1 - p_1 of level estimates (for a deflated p_1)."""
        mpmc_set_solve_level_deflation(self.handle, on)

    def set_level_solve_poly(self, pp):
        """Polynomial preconditioner of the main solves inside level estimates (None: none)."""
        self._level_pp = pp          # keep the handle alive while the context uses it
        mpmc_set_level_solve_poly(self.handle, pp)

    def solve_pairs(self, b, nrhs, max_snap, defl=None, restart=50, tol=1e-8, inner_prec=FP32, max_outer=100):
        """Solve and return (x, R, E, nsnap): R/E hold nsnap batches of (residual, error) pairs."""
        x = self.vector(nrhs, FP64)
        vb = mpmc_vector_bytes(self.handle, nrhs, FP32)
        R = self.torch.empty(vb * max_snap, dtype=self.torch.uint8, device="cuda")
        E = self.torch.empty_like(R)
        ns, its, rel = mpmc_solve_pairs(self.handle, b, x, nrhs, defl, restart, tol, inner_prec, max_outer, R, E,
                                        max_snap)
        return x, R, E, ns, vb

    def levels_multi(self, uppers, lowers, defl, theta, seed, streams, first, nnoise, prec=FP64):
        return mpmc_level_estimate_multi(self.handle, uppers, lowers, defl, theta, seed, streams, first, nnoise, prec)

    def level(self, upper, lower, defl, theta, seed, stream, first, nnoise, prec=FP64, max_batch=0,
              solve_tol=1e-8, solve_restart=50, solve_inner_prec=FP64, net=None):
        return mpmc_level_estimate(self.handle, upper, lower, defl, theta, seed, stream, first, nnoise, prec,
                                   max_batch, solve_tol, solve_restart, solve_inner_prec, net)
