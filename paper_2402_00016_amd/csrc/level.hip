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

}  // namespace

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
    const bool use_defl = upper && lower && defl && defl->k > 0;
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
        std::vector<double> pu(2 * k), pl(2 * k), c(2 * k);
        poly_eval_host(upper, defl->lam.data(), pu.data(), k);
        poly_eval_host(lower, defl->lam.data(), pl.data(), k);
        for (int i = 0; i < 2 * k; ++i) c[i] = pu[i] - pl[i];
        HIP_OR_RET(ctx, hipMemcpyAsync(dcf, c.data(), sizeof(double2) * k, hipMemcpyHostToDevice, ctx->stream));
        // exact correction sum_i c_i u_i^H Theta z_i
        double2 *uz = (double2 *)S.get(sizeof(double2) * k);
        if (!uz) return MPMC_ENOMEM;
        for (int i = 0; i < k; ++i)
            RET_IF(blas_dot(ctx, defl->U + 2 * (size_t)i * ctx->n, defl->Z + 2 * (size_t)i * ctx->n, 1, MPMC_FP64, th,
                            (double *)(uz + i)));
        std::vector<double> uzh(2 * k);
        HIP_OR_RET(ctx, hipMemcpyAsync(uzh.data(), uz, sizeof(double2) * k, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
        for (int i = 0; i < k; ++i)
            corr += std::complex<double>(c[2 * i], c[2 * i + 1]) * std::complex<double>(uzh[2 * i], uzh[2 * i + 1]);
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
        if (use_defl) {
            RET_IF(launch_noise(ctx, seed, stream, first + b0, nb, MPMC_FP64, eta64));
            RET_IF(blas_multi_dot(ctx, defl->Z, ctx->n, 1, k, eta64, nb, MPMC_FP64, (double *)da, 0, th));
            RET_IF(blas_multi_dot(ctx, defl->U, ctx->n, 1, k, eta64, nb, MPMC_FP64, (double *)db, 0, 0));
            k_defl_term<<<grid_for(nb, 64), 64, 0, ctx->stream>>>(acc, da, db, dcf, k, nb);
            HIP_OR_RET(ctx, hipGetLastError());
        }
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
