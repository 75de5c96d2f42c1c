// Monte Carlo level samples (Sec. 2 eq. 2, Sec. 6 multipolynomial formula,
// Sec. 7 deflated levels):
//   X_j = eta_j^H Theta (upper - lower) eta_j - sum_i c_i (eta_j^H Theta z_i)(u_i^H eta_j)
// with upper = M^-1 (a batched solve) or a polynomial, lower = 0 or a
// polynomial.  Noise is regenerated on the device from (seed, stream, index);
// every quadratic form is accumulated in FP64.
#include <algorithm>
#include <complex>
#include <vector>

#include "common.h"

namespace {

// acc[r] -= sum_i c_i conj(a[i][r]) b[i][r],  a = z^H Theta eta, b = u^H eta
__global__ void k_defl_term(double2 *acc, const double2 *a, const double2 *b, const double2 *c, int k, int N) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    double sx = 0, sy = 0;
    for (int i = 0; i < k; ++i) {
        const double2 av = a[(long)i * N + r], bv = b[(long)i * N + r], cv = c[i];
        // conj(a) * b
        const double px = av.x * bv.x + av.y * bv.y, py = av.x * bv.y - av.y * bv.x;
        sx += cv.x * px - cv.y * py;
        sy += cv.x * py + cv.y * px;
    }
    acc[r].x -= sx;
    acc[r].y -= sy;
}

// Deflated level (Sec. 7): coefficients c_i = upper(lambda_i) - lower(lambda_i)
// (upper == nullptr: M^-1, upper(lambda) = 1/lambda) on the device (dcf, k
// entries) and the exact correction corr = sum_i c_i u_i^H Theta z_i.
// Synchronises.
int defl_setup(mpmc_ctx *ctx, const mpmc_poly *upper, const mpmc_poly *lower, const mpmc_defl *defl, int th,
               double2 *dcf, double2 *uz, std::complex<double> &corr) {
    const int k = defl->k;
    std::vector<double> pu(2 * k), pl(2 * k), c(2 * k);
    if (upper) {
        poly_eval_host(upper, defl->lam.data(), pu.data(), k);
    } else {
        for (int i = 0; i < k; ++i) {
            const std::complex<double> v = 1.0 / std::complex<double>(defl->lam[2 * i], defl->lam[2 * i + 1]);
            pu[2 * i] = v.real();
            pu[2 * i + 1] = v.imag();
        }
    }
    poly_eval_host(lower, defl->lam.data(), pl.data(), k);
    for (int i = 0; i < 2 * k; ++i) c[i] = pu[i] - pl[i];
    HIP_OR_RET(ctx, hipMemcpyAsync(dcf, c.data(), sizeof(double2) * k, hipMemcpyHostToDevice, ctx->stream));
    for (int i = 0; i < k; ++i)
        RET_IF(blas_dot(ctx, defl->U + 2 * (size_t)i * ctx->n, defl->Z + 2 * (size_t)i * ctx->n, 1, MPMC_FP64, th,
                        (double *)(uz + i)));
    std::vector<double> uzh(2 * k);
    HIP_OR_RET(ctx, hipMemcpyAsync(uzh.data(), uz, sizeof(double2) * k, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    corr = 0;
    for (int i = 0; i < k; ++i)
        corr += std::complex<double>(c[2 * i], c[2 * i + 1]) * std::complex<double>(uzh[2 * i], uzh[2 * i + 1]);
    return MPMC_OK;
}

// acc[r] -= sum_i c_i (eta_r^H Theta z_i)(u_i^H eta_r) for the noise vectors
// first .. first+nb-1 of (seed, stream), regenerated in FP64 into eta64.
int defl_samples(mpmc_ctx *ctx, const mpmc_defl *defl, const double2 *dcf, uint64_t seed, uint32_t stream,
                 uint64_t first, int nb, int th, void *eta64, double2 *da, double2 *db, double2 *acc) {
    const int k = defl->k;
    RET_IF(launch_noise(ctx, seed, stream, first, nb, MPMC_FP64, eta64));
    RET_IF(blas_multi_dot(ctx, defl->Z, ctx->n, 1, k, eta64, nb, MPMC_FP64, (double *)da, 0, th));
    RET_IF(blas_multi_dot(ctx, defl->U, ctx->n, 1, k, eta64, nb, MPMC_FP64, (double *)db, 0, 0));
    k_defl_term<<<grid_for(nb, 64), 64, 0, ctx->stream>>>(acc, da, db, dcf, k, nb);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

}  // namespace

MPMC_API int mpmc_set_solve_level_deflation(mpmc_ctx *ctx, int on) {
    if (!ctx) return MPMC_EINVAL;
    if (on != 0 && on != 1) return set_err(ctx, MPMC_EINVAL, "mpmc_set_solve_level_deflation: on must be 0 or 1");
    ctx->solve_level_defl = on;
    return MPMC_OK;
}

MPMC_API int mpmc_level_estimate(mpmc_ctx *ctx, const mpmc_poly *upper, const mpmc_poly *lower,
                                 const mpmc_defl *defl, int theta, uint64_t seed, uint32_t stream, uint64_t first,
                                 int nnoise, int prec, int max_batch, double solve_tol, int solve_restart,
                                 int solve_inner_prec, const mpmc_net *net, double *samples_host, double *corr_host,
                                 uint64_t *mvps_host) {
    if (!ctx) return MPMC_EINVAL;
    if (nnoise < 1 || !samples_host || (prec != MPMC_FP64 && prec != MPMC_FP32) ||
        (theta != MPMC_THETA_I && theta != MPMC_THETA_G5) || first + (uint64_t)nnoise > 0x100000000ull)
        return set_err(ctx, MPMC_EINVAL, "mpmc_level_estimate: bad argument");
    if ((upper && upper->ctx != ctx) || (lower && lower->ctx != ctx) || (defl && defl->ctx != ctx))
        return set_err(ctx, MPMC_ESTATE, "mpmc_level_estimate: handle from another context");
    if (!upper && (!(solve_tol > 0) || solve_restart < 1))
        return set_err(ctx, MPMC_EINVAL, "mpmc_level_estimate: solve level needs solve_tol > 0 and restart >= 1");
    const uint64_t mvp0 = ctx->mvps;
    const int th = theta == MPMC_THETA_G5 ? 1 : 0;
    const int B = (max_batch > 0 && max_batch < nnoise) ? max_batch : nnoise;
    // polynomial-difference levels are deflated (Sec. 7); the solve level
    // M^-1 - p_1 too when the context asks for it (a deflated p_1)
    const bool use_defl = lower && defl && defl->k > 0 && (upper || ctx->solve_level_defl);
    const int k = use_defl ? defl->k : 0;

    Scratch S(ctx);
    const size_t vbp = vec_bytes(ctx, B, prec), vb64 = vec_bytes(ctx, B, MPMC_FP64);
    void *eta = S.get(std::max(vbp, vb64));
    void *yv = S.get(std::max(vbp, vb64));
    void *eta64 = (!upper || use_defl) ? S.get(vb64) : nullptr;
    double2 *acc = (double2 *)S.get(sizeof(double2) * B);
    double2 *tmp = (double2 *)S.get(sizeof(double2) * B);
    double2 *da = k ? (double2 *)S.get(sizeof(double2) * (size_t)k * B) : nullptr;
    double2 *db = k ? (double2 *)S.get(sizeof(double2) * (size_t)k * B) : nullptr;
    double2 *dcf = k ? (double2 *)S.get(sizeof(double2) * k) : nullptr;
    if (!eta || !yv || !acc || !tmp || ((!upper || use_defl) && !eta64) || (k && (!da || !db || !dcf)))
        return MPMC_ENOMEM;

    std::complex<double> corr(0, 0);
    if (use_defl) {
        double2 *uz = (double2 *)S.get(sizeof(double2) * k);
        if (!uz) return MPMC_ENOMEM;
        RET_IF(defl_setup(ctx, upper, lower, defl, th, dcf, uz, corr));
    }

    uint32_t *codes = (upper || lower) ? (uint32_t *)S.get(sizeof(uint32_t) * (size_t)ctx->V * B) : nullptr;
    if ((upper || lower) && !codes) return MPMC_ENOMEM;
    for (int b0 = 0; b0 < nnoise; b0 += B) {
        const int nb = std::min(B, nnoise - b0);
        const bool fused = poly_quad_fusable(nb);
        HIP_OR_RET(ctx, hipMemsetAsync(acc, 0, sizeof(double2) * nb, ctx->stream));
        if (upper || lower) {
            RET_IF(launch_noise(ctx, seed, stream, first + b0, nb, prec, eta));
            if (fused) RET_IF(wilson_noise_codes(ctx, seed, stream, first + b0, nb, codes));
        }
        if (!upper) {
            int its = 0;
            std::vector<double> rr(nb);
            RET_IF(launch_noise(ctx, seed, stream, first + b0, nb, MPMC_FP64, eta64));
            RET_IF(solve_internal(ctx, eta64, yv, nb, defl, net, solve_restart, solve_tol, solve_inner_prec, 400, &its,
                                  rr.data(), nullptr, net ? nullptr : ctx->level_pp));
            RET_IF(blas_dot(ctx, eta64, yv, nb, MPMC_FP64, th, (double *)acc));
        }
        const mpmc_poly *parts[2] = {upper, lower};
        const double signs[2] = {1.0, -1.0};
        for (int q = 0; q < 2; ++q) {
            const mpmc_poly *pq = parts[q];
            if (!pq) continue;
            if (fused) {
                RET_IF(poly_quad_fused(ctx, pq, eta, codes, nb, prec, th, (double *)acc, signs[q]));
            } else {
                RET_IF(poly_apply_internal(ctx, pq, eta, yv, nb, prec));
                RET_IF(blas_dot(ctx, eta, yv, nb, prec, th, (double *)tmp));
                RET_IF(blas_scale_acc(ctx, (double *)tmp, nb, make_double2(1, 0), signs[q], (double *)acc));
            }
        }
        if (use_defl) RET_IF(defl_samples(ctx, defl, dcf, seed, stream, first + b0, nb, th, eta64, da, db, acc));
        HIP_OR_RET(ctx, hipMemcpyAsync(samples_host + 2 * (size_t)b0, acc, sizeof(double2) * nb, hipMemcpyDeviceToHost,
                                       ctx->stream));
    }
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    if (corr_host) {
        corr_host[0] = corr.real();
        corr_host[1] = corr.imag();
    }
    if (mvps_host) *mvps_host = ctx->mvps - mvp0;
    return MPMC_OK;
}

// --------------------------------------------- several terms in one batch --
// The polynomial terms of the multipolynomial formula (Sec. 6) in shared
// launches: every single-polynomial recurrence (the upper and the lower
// polynomial of each term, both on that term's noise) takes its own run of
// 64-wide chunks on one right-hand-side axis, runs sorted by decreasing degree,
// so step k of the fused recurrence is one launch over the runs still active.
// Per (site, rhs) the arithmetic and the order of every sum are those of
// mpmc_level_estimate; terms with a double polynomial, or shapes without
// 64-wide chunks or the blocked traversal, go through mpmc_level_estimate.
MPMC_API int mpmc_level_estimate_multi(mpmc_ctx *ctx, int nterms, const mpmc_poly *const *upper,
                                       const mpmc_poly *const *lower, const mpmc_defl *defl, int theta,
                                       uint64_t seed, const uint32_t *streams, uint64_t first, int nnoise, int prec,
                                       double *samples_host, double *corr_host, uint64_t *mvps_host) {
    if (!ctx) return MPMC_EINVAL;
    if (nterms < 1 || nterms > 64 || !upper || !lower || !streams || nnoise < 1 || !samples_host ||
        (prec != MPMC_FP64 && prec != MPMC_FP32) || (theta != MPMC_THETA_I && theta != MPMC_THETA_G5) ||
        first + (uint64_t)nnoise > 0x100000000ull)
        return set_err(ctx, MPMC_EINVAL, "mpmc_level_estimate_multi: bad argument");
    for (int t = 0; t < nterms; ++t) {
        if (!upper[t]) return set_err(ctx, MPMC_EINVAL, "mpmc_level_estimate_multi: term %d has no polynomial", t);
        if (upper[t]->ctx != ctx || (lower[t] && lower[t]->ctx != ctx))
            return set_err(ctx, MPMC_ESTATE, "mpmc_level_estimate_multi: handle from another context");
    }
    if (defl && defl->ctx != ctx) return set_err(ctx, MPMC_ESTATE, "mpmc_level_estimate_multi: handle from another context");
    const uint64_t mvp0 = ctx->mvps;
    const int th = theta == MPMC_THETA_G5 ? 1 : 0;
    const int nb = nnoise;
    const bool chunks = ctx->V % 4 == 0 && nb % 64 == 0;

    struct Rec {
        int term;
        const mpmc_poly *p;
        double sign;
    };
    std::vector<Rec> recs;
    std::vector<int> batched(nterms, 0);
    for (int t = 0; t < nterms; ++t) {
        const bool single = !upper[t]->inner && (!lower[t] || !lower[t]->inner);
        if (chunks && single) {
            batched[t] = 1;
            recs.push_back({t, upper[t], 1.0});
            if (lower[t]) recs.push_back({t, lower[t], -1.0});
        } else {
            RET_IF(mpmc_level_estimate(ctx, upper[t], lower[t], defl, theta, seed, streams[t], first, nnoise, prec, 0,
                                       1e-8, 50, MPMC_FP64, nullptr, samples_host + 2 * (size_t)t * nb,
                                       corr_host ? corr_host + 2 * t : nullptr, nullptr));
        }
    }
    if (recs.empty()) {
        if (mvps_host) *mvps_host = ctx->mvps - mvp0;
        return MPMC_OK;
    }
    std::vector<int> order(recs.size());   // run j holds recs[order[j]]
    for (size_t j = 0; j < recs.size(); ++j) order[j] = (int)j;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return recs[a].p->d > recs[b].p->d; });
    std::vector<int> run_of(recs.size());
    for (size_t j = 0; j < order.size(); ++j) run_of[order[j]] = (int)j;
    const int R = (int)recs.size(), N = R * nb, nch = N / 64, cpr = nb / 64;
    const int dmax = recs[order[0]].p->d;
    int R2 = 0;   // runs with at least one fused step (degree >= 1 polynomial, d >= 2 roots)
    while (R2 < R && recs[order[R2]].p->d >= 2) ++R2;

    Scratch S(ctx);
    const size_t vb = vec_bytes(ctx, N, prec);
    void *eta = S.get(vb);
    void *wa = S.get(vb);
    void *wb = S.get(vb);
    uint32_t *codes = (uint32_t *)S.get(sizeof(uint32_t) * (size_t)ctx->V * N);
    double2 *first_dot = (double2 *)S.get(sizeof(double2) * N);
    double2 *fin = (double2 *)S.get(sizeof(double2) * N);
    double2 *acc = (double2 *)S.get(sizeof(double2) * (size_t)nterms * nb);
    double *part = (double *)S.get(sizeof(double2) * wilson_dot_partial_count(ctx, N));
    const size_t steps = dmax >= 2 ? (size_t)dmax - 1 : 0;
    double2 *coef = steps ? (double2 *)S.get(sizeof(double2) * 2 * nch * steps) : nullptr;
    const int k = defl ? defl->k : 0;
    void *eta64 = k ? S.get(vec_bytes(ctx, nb, MPMC_FP64)) : nullptr;
    double2 *da = k ? (double2 *)S.get(sizeof(double2) * (size_t)k * nb) : nullptr;
    double2 *db = k ? (double2 *)S.get(sizeof(double2) * (size_t)k * nb) : nullptr;
    double2 *dcf = k ? (double2 *)S.get(sizeof(double2) * k) : nullptr;
    double2 *uz = k ? (double2 *)S.get(sizeof(double2) * k) : nullptr;
    if (!eta || !wa || !wb || !codes || !first_dot || !fin || !acc || !part || (steps && !coef) ||
        (k && (!eta64 || !da || !db || !dcf || !uz)))
        return MPMC_ENOMEM;

    auto inv = [&](const mpmc_poly *p, int i) {
        const std::complex<double> v = 1.0 / std::complex<double>(p->roots[2 * i], p->roots[2 * i + 1]);
        return make_double2(v.real(), v.imag());
    };
    // noise and its codes, run by run
    for (int j = 0; j < R; ++j) {
        const uint32_t st = streams[recs[order[j]].term];
        RET_IF(launch_noise(ctx, seed, st, first, nb, prec, eta, N, j * nb));
        RET_IF(wilson_noise_codes(ctx, seed, st, first, nb, codes, N, j * nb));
    }
    RET_IF(blas_dot(ctx, eta, eta, N, prec, th, (double *)first_dot));   // eta^H Theta eta per right-hand side
    if (steps) {
        // coefficient table: step s, chunk q -> (1/theta_s, 1/theta_{s+1}) of the chunk's run
        std::vector<double2> tab(2 * nch * steps, make_double2(0, 0));
        for (size_t s = 0; s < steps; ++s)
            for (int q = 0; q < nch; ++q) {
                const mpmc_poly *p = recs[order[q / cpr]].p;
                if ((size_t)p->d >= s + 2) {
                    tab[2 * (s * nch + q)] = inv(p, (int)s);
                    tab[2 * (s * nch + q) + 1] = inv(p, (int)s + 1);
                }
            }
        HIP_OR_RET(ctx, hipMemcpyAsync(coef, tab.data(), sizeof(double2) * tab.size(), hipMemcpyHostToDevice,
                                       ctx->stream));
        const void *cur = eta;
        int active = R2;
        for (size_t s = 0; s < steps; ++s) {
            while (active > 0 && (size_t)recs[order[active - 1]].p->d < s + 2) --active;
            void *nxt = (cur == wa) ? wb : wa;
            RET_IF(wilson_dot_step_multi(ctx, cur, nxt, codes, N, active * nb, prec, (const double *)(coef + 2 * nch * s),
                                         th, part, s == 0));
            cur = nxt;
        }
        RET_IF(wilson_dot_finish_chunks(ctx, part, R2 * nb, (double *)fin));
        // the table is host memory read by the copy above: keep it until the stream has passed it
        HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    }
    // per term, in the order of mpmc_level_estimate: upper (first term, then the
    // recurrence), lower (the same), then the deflation correction
    for (int t = 0; t < nterms; ++t) {
        if (!batched[t]) continue;
        double2 *at = acc + (size_t)t * nb;
        HIP_OR_RET(ctx, hipMemsetAsync(at, 0, sizeof(double2) * nb, ctx->stream));
        for (int j = 0; j < R; ++j) {
            const Rec &rc = recs[j];   // recs are in term order, upper before lower
            if (rc.term != t) continue;
            const int run = run_of[j];
            RET_IF(blas_scale_acc(ctx, (const double *)(first_dot + (size_t)run * nb), nb, inv(rc.p, 0), rc.sign,
                                  (double *)at));
            if (rc.p->d >= 2)
                RET_IF(blas_scale_acc(ctx, (const double *)(fin + (size_t)run * nb), nb, make_double2(1, 0), rc.sign,
                                      (double *)at));
        }
        std::complex<double> corr(0, 0);
        if (lower[t] && k > 0) {
            RET_IF(defl_setup(ctx, upper[t], lower[t], defl, th, dcf, uz, corr));
            RET_IF(defl_samples(ctx, defl, dcf, seed, streams[t], first, nb, th, eta64, da, db, at));
        }
        HIP_OR_RET(ctx, hipMemcpyAsync(samples_host + 2 * (size_t)t * nb, at, sizeof(double2) * nb,
                                       hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
        if (corr_host) {
            corr_host[2 * t] = corr.real();
            corr_host[2 * t + 1] = corr.imag();
        }
    }
    if (mvps_host) *mvps_host = ctx->mvps - mvp0;
    return MPMC_OK;
}
