// Eigen-deflation (Sec. 7, acceptance rule of Sec. 8).
//
// Eigenvectors are stored as k single vectors (FP64, [k][n]); the kernels
// that use them against a batch of right-hand sides read each z_i / u_i once
// per site and apply it to every right-hand side of the batch.
#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>

#include "common.h"

__global__ void k_div_lambda(double2 *c, int k, int N, const double2 *lam) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)k * N) return;
    const int i = (int)(t / N);
    const double2 l = lam[i], v = c[t];
    const double d = l.x * l.x + l.y * l.y;
    c[t] = d > 0 ? make_double2((v.x * l.x + v.y * l.y) / d, (v.y * l.x - v.x * l.y) / d) : make_double2(0, 0);
}

// y = coef * gamma5 x for one FP64 vector
__global__ void k_gamma5_scale(const double2 *x, double2 *y, long n, double2 coef) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int k = (int)(e % 12);
    double2 v = x[e];
    if (k >= 6) v = make_double2(-v.x, -v.y);
    y[e] = make_double2(coef.x * v.x - coef.y * v.y, coef.x * v.y + coef.y * v.x);
}

// Ritz vectors z_q = V y_q for q in [q0, q0 + QC) (q < ns), one thread per
// complex element: each basis vector is read once for QC Ritz vectors instead
// of once per vector.  Per z_q the arithmetic is that of forming it alone with
// the single-vector update from a zero start (same order, basis precision), so
// the vectors are the same bit for bit; they are written widened to FP64.
template <int PB, int QC>
__global__ __launch_bounds__(256) void k_ritz_vectors(const void *__restrict__ V, size_t vstep, int me,
                                                      const double2 *__restrict__ Y, int ns, int q0,
                                                      double2 *__restrict__ Z, long n) {
    using T = typename Store<PB>::real;
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    cpx<T> acc[QC];
#pragma unroll
    for (int q = 0; q < QC; ++q) acc[q] = mk(T(0), T(0));
    for (int j = 0; j < me; ++j) {
        const auto v0 = Store<PB>::ld((const char *)V + (size_t)j * vstep, nullptr, e, 0);
        const cpx<T> v = mk((T)v0.re, (T)v0.im);
#pragma unroll
        for (int q = 0; q < QC; ++q)
            if (q0 + q < ns) {
                const double2 y = Y[(size_t)(q0 + q) * me + j];
                acc[q] = acc[q] + mk((T)y.x, (T)y.y) * v;
            }
    }
#pragma unroll
    for (int q = 0; q < QC; ++q)
        if (q0 + q < ns) Z[(size_t)(q0 + q) * n + e] = make_double2((double)acc[q].re, (double)acc[q].im);
}

int defl_coeffs(mpmc_ctx *ctx, const mpmc_defl *d, const void *x, int nrhs, double *c_dev, int divide_by_lambda) {
    RET_IF(blas_multi_dot(ctx, d->U, ctx->n, 1, d->k, x, nrhs, MPMC_FP64, c_dev, 0, 0));
    if (divide_by_lambda) {
        k_div_lambda<<<grid_for((long)d->k * nrhs, 256), 256, 0, ctx->stream>>>((double2 *)c_dev, d->k, nrhs,
                                                                                (const double2 *)d->lam_dev);
        HIP_OR_RET(ctx, hipGetLastError());
    }
    return MPMC_OK;
}

int defl_add(mpmc_ctx *ctx, const mpmc_defl *d, const double *c_dev, void *x, int nrhs, double sign) {
    return blas_multi_axpy(ctx, d->Z, ctx->n, 1, d->k, x, nrhs, MPMC_FP64, c_dev, nrhs, sign, nullptr);
}

// Q x for one vector stored in prec (FP64 directly; FP32 through an FP64 copy).
int project_any(mpmc_ctx *ctx, const mpmc_defl *d, void *x, int prec) {
    if (prec == MPMC_FP64) return defl_project(ctx, d, x, 1);
    Scratch S(ctx);
    void *t = S.get(vec_bytes(ctx, 1, MPMC_FP64));
    if (!t) return MPMC_ENOMEM;
    RET_IF(blas_convert(ctx, x, prec, t, MPMC_FP64, 1));
    RET_IF(defl_project(ctx, d, t, 1));
    return blas_convert(ctx, t, MPMC_FP64, x, prec, 1);
}

int defl_project(mpmc_ctx *ctx, const mpmc_defl *d, void *x, int nrhs) {
    Scratch S(ctx);
    double *c = (double *)S.get(sizeof(double2) * (size_t)d->k * nrhs);
    if (!c) return MPMC_ENOMEM;
    RET_IF(defl_coeffs(ctx, d, x, nrhs, c, 0));
    return defl_add(ctx, d, c, x, nrhs, -1.0);
}

static mpmc_defl *defl_alloc(mpmc_ctx *ctx, int k) {
    mpmc_defl *d = new mpmc_defl();
    d->ctx = ctx;
    d->k = k;
    d->lam.assign(2 * (size_t)(k > 0 ? k : 0), 0.0);
    d->Z = d->U = d->lam_dev = nullptr;
    const size_t vb = sizeof(double2) * (size_t)ctx->n * (k > 0 ? k : 1);
    if (hipMalloc(&d->Z, vb) != hipSuccess || hipMalloc(&d->U, vb) != hipSuccess ||
        hipMalloc(&d->lam_dev, sizeof(double2) * (k > 0 ? k : 1)) != hipSuccess) {
        mpmc_defl_destroy(d);
        set_err(ctx, MPMC_ENOMEM, "deflation set: allocation of %zu bytes failed", 2 * vb);
        return nullptr;
    }
    return d;
}

MPMC_API void mpmc_defl_destroy(mpmc_defl *d) {
    if (!d) return;
    if (d->Z) hipFree(d->Z);
    if (d->U) hipFree(d->U);
    if (d->lam_dev) hipFree(d->lam_dev);
    delete d;
}

MPMC_API int mpmc_defl_keep(mpmc_defl *d, int k) {
    if (!d || k < 0) return MPMC_EINVAL;
    if (k < d->k) {
        d->k = k;
        d->lam.resize(2 * (size_t)k);
    }
    return MPMC_OK;
}

MPMC_API int mpmc_defl_create(mpmc_ctx *ctx, const double *lam_host, const void *Z, const void *U, int k,
                              mpmc_defl **out) {
    if (!ctx) return MPMC_EINVAL;
    if (!out || k < 0 || (k > 0 && (!lam_host || !Z || !U)))
        return set_err(ctx, MPMC_EINVAL, "mpmc_defl_create: bad argument");
    mpmc_defl *d = defl_alloc(ctx, k);
    if (!d) return MPMC_ENOMEM;
    if (k > 0) {
        const size_t vb = sizeof(double2) * (size_t)ctx->n * k;
        std::copy(lam_host, lam_host + 2 * k, d->lam.begin());
        HIP_OR_RET(ctx, hipMemcpyAsync(d->Z, Z, vb, hipMemcpyDeviceToDevice, ctx->stream));
        HIP_OR_RET(ctx, hipMemcpyAsync(d->U, U, vb, hipMemcpyDeviceToDevice, ctx->stream));
        HIP_OR_RET(ctx, hipMemcpyAsync(d->lam_dev, lam_host, sizeof(double2) * k, hipMemcpyHostToDevice, ctx->stream));
        HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    }
    *out = d;
    return MPMC_OK;
}

MPMC_API int mpmc_defl_export(const mpmc_defl *d, double *lam_host, void *Z, void *U, int *k) {
    if (!d || !k) return MPMC_EINVAL;
    mpmc_ctx *ctx = const_cast<mpmc_ctx *>(d->ctx);
    *k = d->k;
    if (d->k == 0) return MPMC_OK;
    if (lam_host) std::copy(d->lam.begin(), d->lam.end(), lam_host);
    const size_t vb = sizeof(double2) * (size_t)ctx->n * d->k;
    if (Z) HIP_OR_RET(ctx, hipMemcpyAsync(Z, d->Z, vb, hipMemcpyDeviceToDevice, ctx->stream));
    if (U) HIP_OR_RET(ctx, hipMemcpyAsync(U, d->U, vb, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    return MPMC_OK;
}

int arnoldi_run_ext(mpmc_ctx *ctx, const mpmc_poly *inner, void *V, double *H, int d, double *state, Scratch &S,
                    int prec);

MPMC_API int mpmc_deflate(mpmc_ctx *ctx, const mpmc_poly *p_in, uint64_t seed, uint32_t stream, int m, int nev,
                          double accept_tol, double real_tol, mpmc_defl **out, int *k_out) {
    if (!ctx) return MPMC_EINVAL;
    if (!out || m < 2 || m > 500 || nev < 1 || nev > m || !(accept_tol > 0) || !(real_tol >= 0))
        return set_err(ctx, MPMC_EINVAL, "mpmc_deflate: bad argument (m=%d nev=%d)", m, nev);
    if (p_in && (p_in->ctx != ctx || p_in->inner))
        return set_err(ctx, MPMC_EINVAL, "mpmc_deflate: p_in must be a single polynomial of this context");
    *out = nullptr;
    Scratch S(ctx);
    const long n = ctx->n;
    const size_t vb = sizeof(double2) * (size_t)n;
    const int bprec = ctx->setup_prec;   // storage of the Arnoldi basis; Ritz vectors are FP64
    void *V = S.get(vec_bytes(ctx, 1, bprec) * (size_t)(m + 1));
    double *H = (double *)S.get(sizeof(double2) * (size_t)(m + 1) * m);
    double *state = (double *)S.get(sizeof(double) * 8);
    double *mu = (double *)S.get(sizeof(double2) * (m + 2));
    double *info = (double *)S.get(sizeof(double) * 4);
    if (!V || !H || !state || !mu || !info) return MPMC_ENOMEM;
    RET_IF(launch_noise(ctx, seed, stream, 0, 1, bprec, V));
    RET_IF(arnoldi_run_ext(ctx, p_in, V, H, m, state, S, bprec));
    double hs[3];
    HIP_OR_RET(ctx, hipMemcpyAsync(hs, state, sizeof hs, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    const int me = hs[1] >= 0 ? (int)hs[1] : m;
    RET_IF(dense_hess_eigs(ctx, H, m + 1, me, mu, info));
    std::vector<double> muh(2 * me);
    double inf;
    HIP_OR_RET(ctx, hipMemcpyAsync(muh.data(), mu, sizeof(double) * 2 * me, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_RET(ctx, hipMemcpyAsync(&inf, info, sizeof inf, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    if (inf != 0) return set_err(ctx, MPMC_ENUMERIC, "mpmc_deflate: Hessenberg eigenproblem failed");

    // the nev Ritz values of smallest modulus (stable order)
    std::vector<int> idx(me);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        return std::hypot(muh[2 * a], muh[2 * a + 1]) < std::hypot(muh[2 * b], muh[2 * b + 1]);
    });
    const int ns = std::min(nev, me);
    std::vector<double> musel(2 * ns);
    for (int q = 0; q < ns; ++q) {
        musel[2 * q] = muh[2 * idx[q]];
        musel[2 * q + 1] = muh[2 * idx[q] + 1];
    }
    double *mus = (double *)S.get(sizeof(double2) * ns);
    double *Y = (double *)S.get(sizeof(double2) * (size_t)me * ns);
    double *Zc = (double *)S.get(vb * ns);
    double *MZ = (double *)S.get(vb * ns);
    double *tmp = (double *)S.get(vb);
    double *scal = (double *)S.get(sizeof(double2) * 8);
    if (!mus || !Y || !Zc || !MZ || !tmp || !scal) return MPMC_ENOMEM;
    HIP_OR_RET(ctx, hipMemcpyAsync(mus, musel.data(), sizeof(double2) * ns, hipMemcpyHostToDevice, ctx->stream));
    RET_IF(dense_inverse_iteration(ctx, H, m + 1, me, mus, ns, Y));

    // Ritz vectors z = V y in the basis precision (FP64 coefficients), widened
    // to FP64: all of them in passes over the basis (20 per pass from an FP32
    // basis, 8 from an FP64 one), then unit norm, M z, Rayleigh quotients
    {
        const unsigned grid = grid_for(n, 256);
        if (bprec == MPMC_FP64) {
            for (int q0 = 0; q0 < ns; q0 += 8)
                k_ritz_vectors<MPMC_FP64, 8><<<grid, 256, 0, ctx->stream>>>(V, (size_t)n * 16, me, (const double2 *)Y,
                                                                           ns, q0, (double2 *)Zc, n);
        } else {
            for (int q0 = 0; q0 < ns; q0 += 20)
                k_ritz_vectors<MPMC_FP32, 20><<<grid, 256, 0, ctx->stream>>>(V, (size_t)n * 8, me, (const double2 *)Y,
                                                                            ns, q0, (double2 *)Zc, n);
        }
        HIP_OR_RET(ctx, hipGetLastError());
    }
    std::vector<std::complex<double>> lam(ns);
    std::vector<double> rres(ns);
    for (int q = 0; q < ns; ++q) {
        double *z = Zc + 2 * (size_t)q * n, *mz = MZ + 2 * (size_t)q * n;
        RET_IF(blas_norm2(ctx, z, 1, MPMC_FP64, scal));
        RET_IF(blas_scale_rhs(ctx, z, z, 1, MPMC_FP64, scal, 1));
        RET_IF(wilson_launch_full(ctx, z, nullptr, mz, nullptr, 1, MPMC_FP64, make_double2(0, 0), make_double2(1, 0),
                                  make_double2(0, 0), 0, 0));
        RET_IF(blas_dot(ctx, z, mz, 1, MPMC_FP64, 0, scal + 2));
        double l[2];
        HIP_OR_RET(ctx, hipMemcpyAsync(l, scal + 2, sizeof l, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
        lam[q] = std::complex<double>(l[0], l[1]);
        // right residual ||M z - lambda z||
        HIP_OR_RET(ctx, hipMemcpyAsync(tmp, mz, vb, hipMemcpyDeviceToDevice, ctx->stream));
        RET_IF(blas_axpby(ctx, z, tmp, 1, MPMC_FP64, make_double2(-l[0], -l[1]), make_double2(1, 0)));
        RET_IF(blas_norm2(ctx, tmp, 1, MPMC_FP64, scal + 4));
        double r2[2];
        HIP_OR_RET(ctx, hipMemcpyAsync(r2, scal + 4, sizeof r2, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
        rres[q] = std::sqrt(std::max(r2[0], 0.0));
    }

    // left vectors from gamma5-hermiticity, biorthonormalised, and acceptance
    std::vector<int> accepted;
    std::vector<double> uscale_re(ns), uscale_im(ns);
    std::vector<int> partner(ns, -1);
    double *Uc = (double *)S.get(vb * ns);
    if (!Uc) return MPMC_ENOMEM;
    for (int q = 0; q < ns; ++q) {
        int j = q;
        if (std::fabs(lam[q].imag()) >= real_tol) {
            double best = INFINITY;
            j = -1;
            for (int t = 0; t < ns; ++t) {
                if (t == q) continue;
                const double dd = std::abs(lam[t] - std::conj(lam[q]));
                if (dd < best) { best = dd; j = t; }
            }
        }
        if (j < 0 || rres[q] >= accept_tol) continue;
        double *u = Uc + 2 * (size_t)q * n;
        k_gamma5_scale<<<grid_for(n, 256), 256, 0, ctx->stream>>>((const double2 *)(Zc + 2 * (size_t)j * n),
                                                                   (double2 *)u, n, make_double2(1, 0));
        HIP_OR_RET(ctx, hipGetLastError());
        RET_IF(blas_dot(ctx, u, Zc + 2 * (size_t)q * n, 1, MPMC_FP64, 0, scal));   // u^H z
        double ov[2];
        HIP_OR_RET(ctx, hipMemcpyAsync(ov, scal, sizeof ov, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
        const std::complex<double> o(ov[0], ov[1]);
        if (std::abs(o) < 1e-300) continue;
        // left residual with u normalised: ||M^H u - conj(lambda) u|| (u = g5 z_j has unit norm)
        RET_IF(wilson_launch_full(ctx, u, nullptr, tmp, nullptr, 1, MPMC_FP64, make_double2(0, 0), make_double2(1, 0),
                                  make_double2(0, 0), 1, 0));
        const std::complex<double> cl = std::conj(lam[q]);
        RET_IF(blas_axpby(ctx, u, tmp, 1, MPMC_FP64, make_double2(-cl.real(), -cl.imag()), make_double2(1, 0)));
        RET_IF(blas_norm2(ctx, tmp, 1, MPMC_FP64, scal + 2));
        double l2[2];
        HIP_OR_RET(ctx, hipMemcpyAsync(l2, scal + 2, sizeof l2, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
        if (std::sqrt(std::max(l2[0], 0.0)) >= accept_tol) continue;
        // scale u so that u^H z = 1: u <- u / conj(o)
        const std::complex<double> sc = 1.0 / std::conj(o);
        RET_IF(blas_axpby(ctx, u, u, 1, MPMC_FP64, make_double2(sc.real(), sc.imag()), make_double2(0, 0)));
        accepted.push_back(q);
        partner[q] = j;
    }
    std::stable_sort(accepted.begin(), accepted.end(),
                     [&](int a, int b) { return std::abs(lam[a]) < std::abs(lam[b]); });
    const int k = (int)accepted.size();
    mpmc_defl *d = defl_alloc(ctx, k);
    if (!d) return MPMC_ENOMEM;
    for (int i = 0; i < k; ++i) {
        const int q = accepted[i];
        d->lam[2 * i] = lam[q].real();
        d->lam[2 * i + 1] = lam[q].imag();
        hipMemcpyAsync(d->Z + 2 * (size_t)i * n, Zc + 2 * (size_t)q * n, vb, hipMemcpyDeviceToDevice, ctx->stream);
        hipMemcpyAsync(d->U + 2 * (size_t)i * n, Uc + 2 * (size_t)q * n, vb, hipMemcpyDeviceToDevice, ctx->stream);
    }
    if (k > 0)
        hipMemcpyAsync(d->lam_dev, d->lam.data(), sizeof(double2) * k, hipMemcpyHostToDevice, ctx->stream);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        mpmc_defl_destroy(d);
        return set_err(ctx, MPMC_EHIP, "mpmc_deflate: %s", hipGetErrorString(e));
    }
    *out = d;
    if (k_out) *k_out = k;
    return MPMC_OK;
}
