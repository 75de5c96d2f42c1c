// Main solves M x = b for a batch of right-hand sides (Sec. 1: the main
// expense of the method; Sec. 8: deflated GMRES).
//
// Mixed-precision defect correction: the outer loop keeps x and r = b - M x in
// FP64 and tests the TRUE residual; each inner restarted GMRES(m) cycle runs in
// the inner precision (FP64 or FP32 storage, FP64 dot products) on r and
// returns a correction e, x += e.  All right-hand sides advance together: one
// Wilson launch, one Gram-Schmidt dot launch and one update launch per inner
// iteration serve the whole batch, and the per-rhs Hessenberg/Givens state
// lives on the device.  With a learned preconditioner N the inner cycle is
// flexible GMRES (z_j = N v_j, Arnoldi on M z_j, correction sum_j y_j z_j).
// With a polynomial preconditioner p (the paper's PP-GMRES, Sec. 8) the inner
// cycle is right-preconditioned GMRES on M p(M) and the correction is p(M) V y.
// With a deflation set, x starts at Z Lambda^-1 U^H b and
// each restart adds Z Lambda^-1 U^H r (projection of the small eigen-components).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace {

// H column j (rows 0..j) += h2; h_{j+1,j} = sqrt(nrm2); scale = 1/h_{j+1,j}
__global__ void k_finalize_batch(double2 *Hcol, const double2 *h2, int j, int N, const double2 *nrm2,
                                 double2 *scale) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    for (int i = 0; i <= j; ++i) {
        Hcol[(long)i * N + r].x += h2[(long)i * N + r].x;
        Hcol[(long)i * N + r].y += h2[(long)i * N + r].y;
    }
    const double hn = sqrt(fmax(nrm2[r].x, 0.0));
    Hcol[(long)(j + 1) * N + r] = make_double2(hn, 0.0);
    scale[r] = make_double2(hn > 1e-290 ? 1.0 / hn : 0.0, 0.0);
}

__global__ void k_init_g(double2 *g, int m, int N, const double2 *rn2) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)(m + 1) * N) return;
    const int r = (int)(t % N);
    g[t] = t < N ? make_double2(sqrt(fmax(rn2[r].x, 0.0)), 0.0) : make_double2(0.0, 0.0);
}

}  // namespace

int solve_internal(mpmc_ctx *ctx, const void *b, void *x, int N, const mpmc_defl *defl, const mpmc_net *net,
                   int m, double tol, int inner_prec, int max_outer, int *iters_out, double *relres_host,
                   SolveSnap *snap, const mpmc_poly *pp) {
    if (pp && net) return set_err(ctx, MPMC_EINVAL, "mpmc_solve: polynomial and learned preconditioner are exclusive");
    if (pp && pp->ctx != ctx) return set_err(ctx, MPMC_ESTATE, "mpmc_solve: polynomial belongs to another context");
    if (net && net_context(net) != ctx) return set_err(ctx, MPMC_ESTATE, "mpmc_solve: network belongs to another context");
    if (net && inner_prec != MPMC_FP32)
        return set_err(ctx, MPMC_EINVAL, "mpmc_solve: the learned preconditioner runs with FP32 inner cycles only");
    if (inner_prec != MPMC_FP64 && inner_prec != MPMC_FP32 && inner_prec != MPMC_FP16S)
        return set_err(ctx, MPMC_EINVAL, "mpmc_solve: inner precision must be FP64, FP32 or FP16S");
    Scratch S(ctx);
    const long n = ctx->n;
    // basis vectors in pb (FP16S: half + per-(site, rhs) scale, storage only);
    // working vectors (w, e) and arithmetic in pw
    const int pb = inner_prec, pw = inner_prec == MPMC_FP64 ? MPMC_FP64 : MPMC_FP32;
    const bool half = pb == MPMC_FP16S;
    const size_t vb64 = vec_bytes(ctx, N, MPMC_FP64), vbi = vec_bytes(ctx, N, pw), vbb = vec_bytes(ctx, N, pb);
    const long vstride = n * N;   // complex elements between basis vectors (FP64/FP32 bases)
    double *r = (double *)S.get(vb64);
    void *V = S.get(vbb * (m + 1));
    void *Zb = net ? S.get(vbi * m) : nullptr;   // flexible GMRES: preconditioned basis z_j = N v_j
    void *w = S.get(vbi);
    void *e = S.get(vbi);
    void *tp = pp ? S.get(vbi) : nullptr;   // p(M) v_j (polynomial right preconditioning)
    void *tq = pp && half ? S.get(vbi) : nullptr;   // FP32 copy of an FP16S basis vector
    double *H = (double *)S.get(sizeof(double2) * (size_t)(m + 1) * (m + 1) * N);
    double *h2 = (double *)S.get(sizeof(double2) * (size_t)(m + 1) * N);
    double *cs = (double *)S.get(sizeof(double2) * (size_t)2 * m * N);
    double *g = (double *)S.get(sizeof(double2) * (size_t)(m + 1) * N);
    double *y = (double *)S.get(sizeof(double2) * (size_t)m * N);
    double *res = (double *)S.get(sizeof(double) * N);
    double *sc = (double *)S.get(sizeof(double2) * 4 * N);   // [0..N) norms, [N..2N) scales
    double *dc = defl && defl->k ? (double *)S.get(sizeof(double2) * (size_t)defl->k * N) : nullptr;
    void *xsnap = snap ? S.get(vb64 * (size_t)snap->max) : nullptr;   // FP64 iterates x_k of the record
    if (snap && !xsnap) return MPMC_ENOMEM;
    if (!r || !V || (net && !Zb) || (pp && !tp) || (pp && half && !tq) || !w || !e || !H || !h2 || !cs || !g || !y || !res || !sc || (defl && defl->k && !dc))
        return MPMC_ENOMEM;
    double *nrm = sc, *scale = sc + 2 * N;

    std::vector<double> bn2(2 * N), rn2(2 * N), resh(N);
    RET_IF(blas_norm2(ctx, b, N, MPMC_FP64, nrm));
    HIP_OR_RET(ctx, hipMemcpyAsync(bn2.data(), nrm, sizeof(double2) * N, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_RET(ctx, hipMemsetAsync(x, 0, vb64, ctx->stream));
    if (dc) {
        RET_IF(defl_coeffs(ctx, defl, b, N, dc, 1));
        RET_IF(defl_add(ctx, defl, dc, x, N, 1.0));
    }
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < N; ++i)
        if (!std::isfinite(bn2[2 * i])) return set_err(ctx, MPMC_ENUMERIC, "mpmc_solve: rhs %d is not finite", i);

    int total = 0;
    bool converged = false;
    std::vector<double> rel(N, 1.0);
    auto true_residual = [&]() -> int {
        RET_IF(wilson_launch_full(ctx, x, b, r, nullptr, N, MPMC_FP64, make_double2(1, 0), make_double2(-1, 0),
                                  make_double2(0, 0), 0, 0));
        RET_IF(blas_norm2(ctx, r, N, MPMC_FP64, nrm));
        HIP_OR_RET(ctx, hipMemcpyAsync(rn2.data(), nrm, sizeof(double2) * N, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
        bool all = true;
        for (int i = 0; i < N; ++i) {
            if (!std::isfinite(rn2[2 * i])) return set_err(ctx, MPMC_ENUMERIC, "mpmc_solve: residual %d is not finite", i);
            rel[i] = bn2[2 * i] > 0 ? std::sqrt(std::max(rn2[2 * i], 0.0) / bn2[2 * i]) : 0.0;
            if (rel[i] > tol) all = false;
        }
        converged = all;
        return MPMC_OK;
    };

    // The network is only a preconditioner: a cycle run with it that does not
    // cut some unconverged residual by 10% switches it off for the rest of the
    // solve, which then continues as plain (deflated) GMRES.
    bool use_net = net != nullptr;
    std::vector<double> rel_start;
    for (int outer = 0; outer < max_outer; ++outer) {
        RET_IF(true_residual());
        if (converged) break;
        if (use_net && !rel_start.empty())
            for (int i = 0; i < N; ++i)
                if (rel[i] > tol && rel[i] > 0.9 * rel_start[i]) use_net = false;
        if (dc) {
            RET_IF(defl_coeffs(ctx, defl, r, N, dc, 1));
            RET_IF(defl_add(ctx, defl, dc, x, N, 1.0));
            RET_IF(true_residual());
            if (converged) break;
        }
        rel_start = rel;
        const mpmc_net *cnet = use_net ? net : nullptr;
        if (snap && snap->count < snap->max) {   // r_k now; e_k = x* - x_k (FP64) at the end
            const size_t vb32 = vec_bytes(ctx, N, MPMC_FP32);
            RET_IF(blas_convert(ctx, r, MPMC_FP64, (char *)snap->R + (size_t)snap->count * vb32, MPMC_FP32, N));
            HIP_OR_RET(ctx, hipMemcpyAsync((char *)xsnap + (size_t)snap->count * vb64, x, vb64,
                                           hipMemcpyDeviceToDevice, ctx->stream));
            ++snap->count;
        }
        // inner targets: the final tolerance for an FP64 cycle; FP32 cycles
        // stop near single precision and the outer loop corrects the rest
        std::vector<double> target(N);
        for (int i = 0; i < N; ++i) {
            const double rn = std::sqrt(std::max(rn2[2 * i], 0.0)), bn = std::sqrt(std::max(bn2[2 * i], 0.0));
            double t = 0.5 * tol * bn;
            if (inner_prec == MPMC_FP32) t = std::max(t, 2e-6 * rn);
            if (half) t = std::max(t, 1e-3 * rn);   // FP16 basis: the Arnoldi relation holds to ~2^-11
            target[i] = t;
        }
        if (half) {
            RET_IF(blas_convert(ctx, r, MPMC_FP64, w, MPMC_FP32, N));
            RET_IF(blas_scale_rhs(ctx, w, w, N, MPMC_FP32, nrm, 1));
            RET_IF(blas_convert(ctx, w, MPMC_FP32, V, MPMC_FP16S, N));
        } else {
            RET_IF(blas_convert(ctx, r, MPMC_FP64, V, inner_prec, N));
            RET_IF(blas_scale_rhs(ctx, V, V, N, inner_prec, nrm, 1));
        }
        HIP_OR_RET(ctx, hipMemsetAsync(H, 0, sizeof(double2) * (size_t)(m + 1) * (m + 1) * N, ctx->stream));
        k_init_g<<<grid_for((long)(m + 1) * N, 256), 256, 0, ctx->stream>>>((double2 *)g, m, N, (const double2 *)nrm);
        HIP_OR_RET(ctx, hipGetLastError());
        const size_t es = inner_prec == MPMC_FP64 ? 16 : 8;
        int jdone = 0;
        for (int j = 0; j < m; ++j) {
            void *vj = half ? (void *)((char *)V + (size_t)j * vbb) : (char *)V + (size_t)j * vstride * es;
            void *vj1 = half ? (void *)((char *)V + (size_t)(j + 1) * vbb) : (char *)V + (size_t)(j + 1) * vstride * es;
            double *Hcol = H + 2 * (size_t)j * (m + 1) * N;
            const void *opin = vj;
            if (cnet) {
                void *zj = (char *)Zb + (size_t)j * vstride * es;
                RET_IF(net_apply_internal(ctx, cnet, vj, zj, N));
                opin = zj;
            }
            if (pp) {   // w = M p(M) v_j
                const void *src = vj;
                if (half) {
                    RET_IF(blas_convert(ctx, vj, MPMC_FP16S, tq, MPMC_FP32, N));
                    src = tq;
                }
                RET_IF(poly_apply_internal(ctx, pp, src, tp, N, pw));
                RET_IF(wilson_launch_full(ctx, tp, nullptr, w, nullptr, N, pw, make_double2(0, 0),
                                          make_double2(1, 0), make_double2(0, 0), 0, 0));
                if (half) {
                    RET_IF(blas_multi_dot_h(ctx, V, vbb, j + 1, w, N, Hcol, 0));
                    RET_IF(blas_multi_axpy_h(ctx, V, vbb, j + 1, w, N, Hcol, N, -1.0, nullptr));
                    RET_IF(blas_multi_dot_h(ctx, V, vbb, j + 1, w, N, h2, 0));
                    RET_IF(blas_multi_axpy_h(ctx, V, vbb, j + 1, w, N, h2, N, -1.0, nrm));
                } else {
                    RET_IF(blas_multi_dot(ctx, V, vstride, N, j + 1, w, N, pw, Hcol, 0, 0));
                    RET_IF(blas_multi_axpy_dot(ctx, V, vstride, j + 1, w, N, pw, Hcol, N, -1.0, h2));
                    RET_IF(blas_multi_axpy(ctx, V, vstride, N, j + 1, w, N, pw, h2, N, -1.0, nrm));
                }
            } else if (half) {
                RET_IF(wilson_apply_h2f(ctx, vj, w, N));
                RET_IF(blas_multi_dot_h(ctx, V, vbb, j + 1, w, N, Hcol, 0));
                RET_IF(blas_multi_axpy_h(ctx, V, vbb, j + 1, w, N, Hcol, N, -1.0, nullptr));
                RET_IF(blas_multi_dot_h(ctx, V, vbb, j + 1, w, N, h2, 0));
                RET_IF(blas_multi_axpy_h(ctx, V, vbb, j + 1, w, N, h2, N, -1.0, nrm));
            } else {
                RET_IF(wilson_launch_full(ctx, opin, nullptr, w, nullptr, N, inner_prec, make_double2(0, 0),
                                          make_double2(1, 0), make_double2(0, 0), 0, 0));
                RET_IF(blas_multi_dot(ctx, V, vstride, N, j + 1, w, N, inner_prec, Hcol, 0, 0));
                RET_IF(blas_multi_axpy_dot(ctx, V, vstride, j + 1, w, N, inner_prec, Hcol, N, -1.0, h2));
                RET_IF(blas_multi_axpy(ctx, V, vstride, N, j + 1, w, N, inner_prec, h2, N, -1.0, nrm));
            }
            k_finalize_batch<<<grid_for(N, 64), 64, 0, ctx->stream>>>((double2 *)Hcol, (const double2 *)h2, j, N,
                                                                      (const double2 *)nrm, (double2 *)scale);
            HIP_OR_RET(ctx, hipGetLastError());
            if (half) {
                RET_IF(blas_scale_rhs(ctx, w, w, N, MPMC_FP32, scale, 0));
                RET_IF(blas_convert(ctx, w, MPMC_FP32, vj1, MPMC_FP16S, N));
            } else {
                RET_IF(blas_scale_rhs(ctx, w, vj1, N, inner_prec, scale, 0));
            }
            RET_IF(dense_givens_step(ctx, H, m + 1, j, N, cs, g, res));
            jdone = j + 1;
            if ((j + 1) % 10 == 0 && j + 1 < m) {
                HIP_OR_RET(ctx, hipMemcpyAsync(resh.data(), res, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream));
                HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
                bool all = true;
                for (int i = 0; i < N; ++i) all = all && resh[i] <= target[i];
                if (all) break;
            }
        }
        RET_IF(dense_backsolve(ctx, H, m + 1, jdone, N, g, y));
        HIP_OR_RET(ctx, hipMemsetAsync(e, 0, vbi, ctx->stream));
        if (half)
            RET_IF(blas_multi_axpy_h(ctx, V, vbb, jdone, e, N, y, N, 1.0, nullptr));
        else
            RET_IF(blas_multi_axpy(ctx, cnet ? Zb : V, vstride, N, jdone, e, N, inner_prec, y, N, 1.0, nullptr));
        if (pp) {   // correction p(M) V y
            RET_IF(poly_apply_internal(ctx, pp, e, tp, N, pw));
            HIP_OR_RET(ctx, hipMemcpyAsync(e, tp, vbi, hipMemcpyDeviceToDevice, ctx->stream));
        }
        // x += e (in FP64)
        RET_IF(blas_convert(ctx, e, pw, r, MPMC_FP64, N));
        RET_IF(blas_axpby(ctx, r, x, N, MPMC_FP64, make_double2(1, 0), make_double2(1, 0)));
        total += jdone;
    }
    if (!converged) RET_IF(true_residual());
    if (snap && snap->count > 0) {
        const size_t vb32 = vec_bytes(ctx, N, MPMC_FP32);
        for (int k = 0; k < snap->count; ++k) {
            void *xk = (char *)xsnap + (size_t)k * vb64;
            RET_IF(blas_axpby(ctx, x, xk, N, MPMC_FP64, make_double2(1, 0), make_double2(-1, 0)));
            RET_IF(blas_convert(ctx, xk, MPMC_FP64, (char *)snap->E + (size_t)k * vb32, MPMC_FP32, N));
        }
    }
    if (iters_out) *iters_out = total;
    if (relres_host)
        for (int i = 0; i < N; ++i) relres_host[i] = rel[i];
    if (!converged) return set_err(ctx, MPMC_ENOCONV, "mpmc_solve: not converged after %d outer cycles", max_outer);
    return MPMC_OK;
}

MPMC_API int mpmc_solve_pairs(mpmc_ctx *ctx, const void *b, void *x, int nrhs, const mpmc_defl *defl, int restart,
                              double tol, int inner_prec, int max_outer, void *R_snap, void *E_snap, int max_snap,
                              int *nsnap_host, int *iters_host, double *relres_host) {
    if (!ctx) return MPMC_EINVAL;
    if (!b || !x || nrhs < 1 || restart < 1 || restart > 400 || !(tol > 0) || max_outer < 1 || !R_snap || !E_snap ||
        max_snap < 1 || !nsnap_host)
        return set_err(ctx, MPMC_EINVAL, "mpmc_solve_pairs: bad argument");
    if (b == x) return set_err(ctx, MPMC_EINVAL, "mpmc_solve_pairs: b and x must not alias");
    if (defl && defl->ctx != ctx) return set_err(ctx, MPMC_ESTATE, "deflation set belongs to another context");
    SolveSnap sn{R_snap, E_snap, max_snap, 0};
    const int rc = solve_internal(ctx, b, x, nrhs, defl, nullptr, restart, tol, inner_prec, max_outer, iters_host,
                                  relres_host, &sn, nullptr);
    *nsnap_host = sn.count;
    return rc;
}

MPMC_API int mpmc_solve(mpmc_ctx *ctx, const void *b, void *x, int nrhs, const mpmc_defl *defl, const mpmc_net *net,
                        int restart, double tol, int inner_prec, int max_outer, int *iters_host, double *relres_host) {
    if (!ctx) return MPMC_EINVAL;
    if (!b || !x || nrhs < 1 || restart < 1 || restart > 400 || !(tol > 0) || max_outer < 1)
        return set_err(ctx, MPMC_EINVAL, "mpmc_solve: bad argument");
    if (b == x) return set_err(ctx, MPMC_EINVAL, "mpmc_solve: b and x must not alias");
    if (defl && defl->ctx != ctx) return set_err(ctx, MPMC_ESTATE, "deflation set belongs to another context");
    return solve_internal(ctx, b, x, nrhs, defl, net, restart, tol, inner_prec, max_outer, iters_host, relres_host,
                          nullptr, nullptr);
}

MPMC_API int mpmc_solve_pp(mpmc_ctx *ctx, const void *b, void *x, int nrhs, const mpmc_defl *defl, const mpmc_poly *pp,
                           int restart, double tol, int inner_prec, int max_outer, int *iters_host,
                           double *relres_host) {
    if (!ctx) return MPMC_EINVAL;
    if (!b || !x || !pp || nrhs < 1 || restart < 1 || restart > 400 || !(tol > 0) || max_outer < 1)
        return set_err(ctx, MPMC_EINVAL, "mpmc_solve_pp: bad argument");
    if (b == x) return set_err(ctx, MPMC_EINVAL, "mpmc_solve_pp: b and x must not alias");
    if (defl && defl->ctx != ctx) return set_err(ctx, MPMC_ESTATE, "deflation set belongs to another context");
    return solve_internal(ctx, b, x, nrhs, defl, nullptr, restart, tol, inner_prec, max_outer, iters_host, relres_host,
                          nullptr, pp);
}

MPMC_API int mpmc_set_level_solve_poly(mpmc_ctx *ctx, const mpmc_poly *pp) {
    if (!ctx) return MPMC_EINVAL;
    if (pp && pp->ctx != ctx) return set_err(ctx, MPMC_ESTATE, "polynomial belongs to another context");
    ctx->level_pp = pp;
    return MPMC_OK;
}
