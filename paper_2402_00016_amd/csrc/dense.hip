// Small dense FP64 problems of the method, solved on the device:
//  * harmonic Ritz values of a GMRES(d) cycle, eig(H_d + |h|^2 H_d^-H e_d e_d^T)
//    (Sec. 3), with the GMRES least-squares residual,
//  * eigenvalues of an upper Hessenberg matrix by shifted QR with Givens
//    rotations (Wilkinson shift, exceptional shifts, bottom deflation),
//  * Leja ordering of the roots (Sec. 3),
//  * Ritz vectors by inverse iteration on H - mu I (deflation, Sec. 7),
//  * per-rhs Givens updates and back substitution of restarted GMRES solves.
// The matrices are at most a few hundred rows: one wavefront (64 lanes) works
// on one matrix; the matrix lives in global memory (L2 resident) because it
// does not fit in LDS for d > 90.  Every loop has a fixed iteration bound.
#include <cfloat>

#include "common.h"

typedef cpx<double> zd;

__device__ __forceinline__ double zabs(zd a) { return hypot(a.re, a.im); }
__device__ __forceinline__ zd zdiv(zd a, zd b) {   // Smith's algorithm
    if (fabs(b.re) >= fabs(b.im)) {
        if (b.re == 0.0 && b.im == 0.0) return mk(0.0, 0.0);
        const double r = b.im / b.re, den = b.re + b.im * r;
        return mk((a.re + a.im * r) / den, (a.im - a.re * r) / den);
    }
    const double r = b.re / b.im, den = b.re * r + b.im;
    return mk((a.re * r + a.im) / den, (a.im * r - a.re) / den);
}
__device__ __forceinline__ zd zsqrt(zd z) {
    const double r = zabs(z);
    if (r == 0.0) return mk(0.0, 0.0);
    const double t = sqrt(0.5 * (r + fabs(z.re)));
    if (z.re >= 0) return mk(t, z.im / (2 * t));
    return mk(fabs(z.im) / (2 * t), copysign(t, z.im));
}
__device__ __forceinline__ zd ld(const double2 *p, long i) { return mk(p[i].x, p[i].y); }
__device__ __forceinline__ void st(double2 *p, long i, zd v) { p[i] = make_double2(v.re, v.im); }

// --------------------------------------------------- Hessenberg QR eigs --
// A: n x n column-major (element (i, j) at A[i + j*lda]), upper Hessenberg,
// destroyed.  ev: n eigenvalues.  Returns 0 or -1 (no convergence / NaN).
// Called by all lanes of one workgroup.
__device__ int hess_eigvals(double2 *A, int lda, int n, double2 *ev) {
    const int tid = threadIdx.x, nt = blockDim.x;
    __shared__ double cs_c[512];
    __shared__ double2 cs_s[512];
    auto a = [&](int i, int j) -> double2 & { return A[i + (long)j * lda]; };
    int hi = n - 1, iter = 0, total = 0;
    const int max_total = 60 * n + 100;
    int status = 0;
    while (hi >= 0) {
        __syncthreads();
        if (hi == 0) {
            if (tid == 0) ev[0] = a(0, 0);
            break;
        }
        int l = hi;
        while (l > 0) {
            const double sub = zabs(ld(&a(l, l - 1), 0));
            const double dia = zabs(ld(&a(l - 1, l - 1), 0)) + zabs(ld(&a(l, l), 0));
            if (!(sub == sub)) { status = -1; break; }
            if (sub <= DBL_EPSILON * dia || sub < 1e-300) break;
            --l;
        }
        if (status) break;
        if (l == hi) {
            if (tid == 0) ev[hi] = a(hi, hi);
            --hi;
            iter = 0;
            continue;
        }
        if (l == hi - 1) {
            const zd p = ld(&a(hi - 1, hi - 1), 0), q = ld(&a(hi - 1, hi), 0), r = ld(&a(hi, hi - 1), 0),
                     s = ld(&a(hi, hi), 0);
            const zd half_tr = 0.5 * (p + s);
            const zd det = p * s - q * r;
            const zd disc = zsqrt(half_tr * half_tr - det);
            if (tid == 0) {
                st(ev, hi - 1, half_tr + disc);
                st(ev, hi, half_tr - disc);
            }
            hi -= 2;
            iter = 0;
            continue;
        }
        if (++total > max_total) { status = -1; break; }
        ++iter;
        // Wilkinson shift from the trailing 2x2 block
        const zd p = ld(&a(hi - 1, hi - 1), 0), q = ld(&a(hi - 1, hi), 0), r = ld(&a(hi, hi - 1), 0),
                 s = ld(&a(hi, hi), 0);
        const zd half_tr = 0.5 * (p + s), det = p * s - q * r;
        const zd disc = zsqrt(half_tr * half_tr - det);
        zd e1 = half_tr + disc, e2 = half_tr - disc;
        zd sigma = zabs(e1 - s) <= zabs(e2 - s) ? e1 : e2;
        if (iter % 11 == 10) {   // exceptional shift breaks cycles
            const double m = zabs(r) + zabs(ld(&a(hi - 1, hi - 2 >= l ? hi - 2 : hi - 1), 0));
            sigma = s + mk(0.75 * m, 0.4375 * m);
        }
        for (int i = l + tid; i <= hi; i += nt) st(&a(i, i), 0, ld(&a(i, i), 0) - sigma);
        __syncthreads();
        // QR: rotations G_k zero a(k+1, k)
        for (int k = l; k < hi; ++k) {
            const zd x = ld(&a(k, k), 0), y = ld(&a(k + 1, k), 0);
            const double ax = zabs(x), ay = zabs(y), rr = hypot(ax, ay);
            double c;
            zd sn;
            if (rr == 0.0) {
                c = 1.0;
                sn = mk(0.0, 0.0);
            } else if (ax == 0.0) {
                c = 0.0;
                sn = mk(y.re / ay, -y.im / ay);   // conj(y)/|y|
            } else {
                c = ax / rr;
                const zd ph = mk(x.re / ax, x.im / ax);
                sn = (1.0 / rr) * (ph * cconj(y));
            }
            for (int j = k + tid; j <= hi; j += nt) {
                const zd u = ld(&a(k, j), 0), v = ld(&a(k + 1, j), 0);
                st(&a(k, j), 0, c * u + sn * v);
                st(&a(k + 1, j), 0, c * v - cconj(sn) * u);
            }
            if (tid == 0) {
                cs_c[k - l] = c;
                cs_s[k - l] = make_double2(sn.re, sn.im);
            }
            __syncthreads();
        }
        // RQ: apply G_k^H on the right
        for (int k = l; k < hi; ++k) {
            const double c = cs_c[k - l];
            const zd sn = mk(cs_s[k - l].x, cs_s[k - l].y);
            for (int i = l + tid; i <= k + 1; i += nt) {
                const zd u = ld(&a(i, k), 0), v = ld(&a(i, k + 1), 0);
                st(&a(i, k), 0, c * u + cconj(sn) * v);
                st(&a(i, k + 1), 0, c * v - sn * u);
            }
            __syncthreads();
        }
        for (int i = l + tid; i <= hi; i += nt) st(&a(i, i), 0, ld(&a(i, i), 0) + sigma);
    }
    __syncthreads();
    return status;
}

// --------------------------------------------------------------- Leja --
// Orders ev[0..n) in place: candidates sorted by (Re, Im), first the largest
// modulus, then the maximiser of sum log|theta - chosen| (lowest index on ties).
__device__ void leja_order(double2 *ev, int n, double2 *tmp, double *S, int *taken) {
    const int tid = threadIdx.x, nt = blockDim.x;
    __syncthreads();
    if (tid == 0) {   // insertion sort by (Re, Im); n <= a few hundred
        for (int i = 1; i < n; ++i) {
            double2 v = ev[i];
            int j = i - 1;
            while (j >= 0 && (ev[j].x > v.x || (ev[j].x == v.x && ev[j].y > v.y))) {
                ev[j + 1] = ev[j];
                --j;
            }
            ev[j + 1] = v;
        }
    }
    __syncthreads();
    for (int j = tid; j < n; j += nt) {
        S[j] = 0.0;
        taken[j] = 0;
    }
    __syncthreads();
    __shared__ double bestv[64];
    __shared__ int besti[64];
    int last = -1;
    for (int step = 0; step < n; ++step) {
        double bv = -INFINITY;
        int bi = 0x7fffffff;
        for (int j = tid; j < n; j += nt) {
            if (taken[j]) continue;
            double v;
            if (step == 0) {
                v = hypot(ev[j].x, ev[j].y);
            } else {
                S[j] += log(hypot(ev[j].x - ev[last].x, ev[j].y - ev[last].y));
                v = S[j];
            }
            if (bi == 0x7fffffff || v > bv) {   // j increases: ties keep the lower index
                bv = v;
                bi = j;
            }
        }
        if (tid < 64) {
            bestv[tid] = bv;
            besti[tid] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            double b = -INFINITY;
            int bj = 0x7fffffff;
            for (int q = 0; q < (nt < 64 ? nt : 64); ++q) {
                if (besti[q] == 0x7fffffff) continue;
                if (bj == 0x7fffffff || bestv[q] > b || (bestv[q] == b && besti[q] < bj)) {
                    b = bestv[q];
                    bj = besti[q];
                }
            }
            besti[0] = bj;
        }
        __syncthreads();
        last = besti[0];
        if (tid == 0) {
            taken[last] = 1;
            tmp[step] = ev[last];
        }
        __syncthreads();
    }
    for (int j = tid; j < n; j += nt) ev[j] = tmp[j];
    __syncthreads();
}

// ------------------------------------------------ harmonic Ritz + Leja --
// H: (d+1) x d column-major with leading dimension ldh (Arnoldi matrix),
// beta = ||b||.  work: >= 2*d*d + 4*d + 8 complex doubles.
// out: roots[d] (Leja ordered), info[0] = relres, info[1] = status.
__global__ __launch_bounds__(64) void k_harmonic_leja(const double2 *H, int ldh, int d, double beta,
                                                      double2 *work, double2 *roots, double *info) {
    const int tid = threadIdx.x, nt = blockDim.x;
    double2 *A = work;                 // d x d, lda = d
    double2 *B = work + (long)d * d;   // d x d, H_d^H, then LU
    double2 *f = B + (long)d * d;      // d
    double2 *g = f + d;                // d+1 (least squares rhs)
    double2 *tmp = g + d + 1;          // d
    double *S = (double *)(tmp + d);   // d doubles
    int *taken = (int *)(S + d);       // d ints
    __shared__ int s_status;
    if (tid == 0) s_status = 0;
    for (long e = tid; e < (long)d * d; e += nt) {
        const int i = (int)(e % d), j = (int)(e / d);
        A[e] = H[i + (long)j * ldh];
        const double2 hji = H[j + (long)i * ldh];   // (H_d^H)(i, j) = conj(H_d(j, i))
        B[e] = make_double2(hji.x, -hji.y);
    }
    __syncthreads();

    // GMRES least-squares residual ||beta e1 - Hbar y|| by Givens on a copy of Hbar
    // (reuse tmp/f storage sequentially on lane 0; d is small).
    if (tid == 0) {
        // residual via rotations applied column by column to a scratch column
        zd gk = mk(beta, 0.0);
        double2 *cs = tmp;   // store (c, 0) and s in f
        for (int j = 0; j < d; ++j) {
            // column j of Hbar with previous rotations applied
            // (rows 0..j+1); keep only the two entries we need at each rotation
            zd col_j1 = ld(H, (j + 1) + (long)j * ldh);
            zd x = ld(H, 0 + (long)j * ldh);
            for (int i = 0; i < j; ++i) {
                const double c = cs[i].x;
                const zd sn = ld(f, i);
                const zd y = ld(H, (i + 1) + (long)j * ldh);
                // rotated entries of rows i, i+1: only row i+1 feeds the next rotation
                const zd xi = c * x + sn * y;
                const zd yi = c * y - cconj(sn) * x;
                (void)xi;
                x = yi;
            }
            const double ax = zabs(x), ay = zabs(col_j1), rr = hypot(ax, ay);
            double c;
            zd sn;
            if (rr == 0.0) { c = 1.0; sn = mk(0.0, 0.0); }
            else if (ax == 0.0) { c = 0.0; sn = mk(col_j1.re / ay, -col_j1.im / ay); }
            else { c = ax / rr; sn = (1.0 / rr) * (mk(x.re / ax, x.im / ax) * cconj(col_j1)); }
            cs[j] = make_double2(c, 0.0);
            st(f, j, sn);
            gk = mk(0.0, 0.0) - cconj(sn) * gk;   // g_{j+1} = -conj(s) g_j
        }
        info[0] = beta > 0 ? zabs(gk) / beta : 0.0;
    }
    __syncthreads();

    const zd h = ld(H, d + (long)(d - 1) * ldh);
    if (zabs(h) > 0.0) {
        // solve B f = e_d by Gaussian elimination with partial pivoting
        for (int i = tid; i < d; i += nt) f[i] = make_double2(i == d - 1 ? 1.0 : 0.0, 0.0);
        __syncthreads();
        for (int k = 0; k < d; ++k) {
            __shared__ int piv;
            if (tid == 0) {
                int p = k;
                double best = zabs(ld(B, k + (long)k * d));
                for (int i = k + 1; i < d; ++i) {
                    const double v = zabs(ld(B, i + (long)k * d));
                    if (v > best) { best = v; p = i; }
                }
                piv = p;
                if (best == 0.0) s_status = -2;
            }
            __syncthreads();
            const int p = piv;
            if (p != k) {
                for (int j = tid; j < d; j += nt) {
                    double2 t = B[k + (long)j * d];
                    B[k + (long)j * d] = B[p + (long)j * d];
                    B[p + (long)j * d] = t;
                }
                if (tid == 0) { double2 t = f[k]; f[k] = f[p]; f[p] = t; }
            }
            __syncthreads();
            const zd pk = ld(B, k + (long)k * d);
            // eliminate rows below k
            for (int i = k + 1 + tid; i < d; i += nt) {
                const zd l = zdiv(ld(B, i + (long)k * d), pk);
                for (int j = k + 1; j < d; ++j)
                    st(B, i + (long)j * d, ld(B, i + (long)j * d) - l * ld(B, k + (long)j * d));
                st(f, i, ld(f, i) - l * ld(f, k));
                B[i + (long)k * d] = make_double2(0, 0);
            }
            __syncthreads();
        }
        if (tid == 0) {   // back substitution
            for (int i = d - 1; i >= 0; --i) {
                zd acc = ld(f, i);
                for (int j = i + 1; j < d; ++j) acc = acc - ld(B, i + (long)j * d) * ld(f, j);
                st(f, i, zdiv(acc, ld(B, i + (long)i * d)));
            }
        }
        __syncthreads();
        const double h2 = h.re * h.re + h.im * h.im;
        for (int i = tid; i < d; i += nt) st(A, i + (long)(d - 1) * d, ld(A, i + (long)(d - 1) * d) + h2 * ld(f, i));
        __syncthreads();
    }
    int rc = hess_eigvals(A, d, d, roots);
    if (rc && tid == 0) s_status = -1;
    __syncthreads();
    leja_order(roots, d, tmp, S, taken);
    if (tid == 0) {
        for (int i = 0; i < d; ++i)
            if (!(roots[i].x == roots[i].x) || !(roots[i].y == roots[i].y) || (roots[i].x == 0 && roots[i].y == 0))
                s_status = -1;
        info[1] = (double)s_status;
    }
}

int dense_harmonic_leja(mpmc_ctx *ctx, const double *H_dev, int ldh, int d, double beta, double *roots_dev,
                        double *info_dev) {
    if (d < 1 || d > 500) return set_err(ctx, MPMC_EINVAL, "harmonic Ritz: d=%d out of range [1, 500]", d);
    double2 *work = (double2 *)ws_get(ctx, WS_DENSE, ((size_t)2 * d * d + 8 * d + 16) * sizeof(double2));
    if (!work) return MPMC_ENOMEM;
    k_harmonic_leja<<<1, 64, 0, ctx->stream>>>((const double2 *)H_dev, ldh, d, beta, work, (double2 *)roots_dev,
                                                info_dev);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// ------------------------------------------------- eigenvalues of H_m --
__global__ __launch_bounds__(64) void k_hess_eigs(const double2 *H, int ldh, int m, double2 *work, double2 *ev,
                                                  double *info) {
    for (long e = threadIdx.x; e < (long)m * m; e += blockDim.x) {
        const int i = (int)(e % m), j = (int)(e / m);
        work[e] = H[i + (long)j * ldh];
    }
    __syncthreads();
    int rc = hess_eigvals(work, m, m, ev);
    if (threadIdx.x == 0) info[0] = rc;
}

int dense_hess_eigs(mpmc_ctx *ctx, const double *H_dev, int ldh, int m, double *ev_dev, double *info_dev) {
    if (m < 1 || m > 500) return set_err(ctx, MPMC_EINVAL, "Hessenberg eigenproblem: m=%d out of range", m);
    double2 *work = (double2 *)ws_get(ctx, WS_DENSE, (size_t)m * m * sizeof(double2));
    if (!work) return MPMC_ENOMEM;
    k_hess_eigs<<<1, 64, 0, ctx->stream>>>((const double2 *)H_dev, ldh, m, work, (double2 *)ev_dev, info_dev);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// ------------------------------------------- inverse iteration vectors --
// One workgroup per eigenvalue mu_q: two solves of (H_m - mu I) y = rhs by
// Hessenberg LU with adjacent-row pivoting; y normalised.  Y: m x k column-major.
__global__ __launch_bounds__(64) void k_inverse_iteration(const double2 *H, int ldh, int m, const double2 *mu,
                                                          double2 *work, double2 *Y) {
    const int q = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    double2 *A = work + (size_t)q * ((size_t)m * m + m);
    double2 *y = A + (size_t)m * m;
    __shared__ double s_hn;
    if (tid == 0) {
        double mx = 0;
        for (long e = 0; e < (long)m * m; ++e) {
            const double2 v = H[(e % m) + (e / m) * (long)ldh];
            mx = fmax(mx, hypot(v.x, v.y));
        }
        s_hn = mx;
    }
    __syncthreads();
    const double hn = s_hn;
    const zd mq = ld(mu, q);
    for (int i = tid; i < m; i += nt) y[i] = make_double2(1.0, 0.0);
    for (int it = 0; it < 3; ++it) {
        __syncthreads();
        for (long e = tid; e < (long)m * m; e += nt) {
            const int i = (int)(e % m), j = (int)(e / m);
            zd v = ld(H, i + (long)j * ldh);
            if (i == j) v = v - mq;
            if (i > j + 1) v = mk(0.0, 0.0);
            st(A, e, v);
        }
        __syncthreads();
        if (tid == 0) {
            for (int k = 0; k < m; ++k) {
                if (k + 1 < m && zabs(ld(A, k + 1 + (long)k * m)) > zabs(ld(A, k + (long)k * m))) {
                    for (int j = k; j < m; ++j) {
                        double2 t = A[k + (long)j * m];
                        A[k + (long)j * m] = A[k + 1 + (long)j * m];
                        A[k + 1 + (long)j * m] = t;
                    }
                    double2 t = y[k];
                    y[k] = y[k + 1];
                    y[k + 1] = t;
                }
                zd pk = ld(A, k + (long)k * m);
                if (zabs(pk) < DBL_EPSILON * hn) {
                    pk = mk(DBL_EPSILON * (hn > 0 ? hn : 1.0), 0.0);
                    st(A, k + (long)k * m, pk);
                }
                if (k + 1 < m) {
                    const zd l = zdiv(ld(A, k + 1 + (long)k * m), pk);
                    for (int j = k + 1; j < m; ++j)
                        st(A, k + 1 + (long)j * m, ld(A, k + 1 + (long)j * m) - l * ld(A, k + (long)j * m));
                    st(y, k + 1, ld(y, k + 1) - l * ld(y, k));
                }
            }
            for (int i = m - 1; i >= 0; --i) {
                zd acc = ld(y, i);
                for (int j = i + 1; j < m; ++j) acc = acc - ld(A, i + (long)j * m) * ld(y, j);
                st(y, i, zdiv(acc, ld(A, i + (long)i * m)));
            }
            double nr = 0;
            for (int i = 0; i < m; ++i) nr += y[i].x * y[i].x + y[i].y * y[i].y;
            nr = sqrt(nr);
            const double inv = nr > 0 ? 1.0 / nr : 0.0;
            for (int i = 0; i < m; ++i) y[i] = make_double2(y[i].x * inv, y[i].y * inv);
        }
    }
    __syncthreads();
    for (int i = tid; i < m; i += nt) Y[i + (long)q * m] = y[i];
}

int dense_inverse_iteration(mpmc_ctx *ctx, const double *H_dev, int ldh, int m, const double *mu_dev, int k,
                            double *Y_dev) {
    if (k < 1) return MPMC_OK;
    double2 *work = (double2 *)ws_get(ctx, WS_DENSE, (size_t)k * ((size_t)m * m + m) * sizeof(double2));
    if (!work) return MPMC_ENOMEM;
    k_inverse_iteration<<<k, 64, 0, ctx->stream>>>((const double2 *)H_dev, ldh, m, (const double2 *)mu_dev, work,
                                                   (double2 *)Y_dev);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// ------------------------------------------ GMRES Givens (per rhs) --
// H layout for batched solves: column j, row i, rhs r at (j*ldc + i)*N + r.
// Applies the stored rotations to column j, forms the new rotation, updates
// g, writes res[r] = |g_{j+1}| (the GMRES residual norm estimate).
__global__ void k_givens_step(double2 *H, int ldc, int j, int N, double2 *cs, double2 *g, double *res) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    auto h = [&](int i) -> double2 & { return H[((long)j * ldc + i) * N + r]; };
    for (int i = 0; i < j; ++i) {
        const double c = cs[(long)i * 2 * N + r].x;
        const zd sn = ld(cs, (long)i * 2 * N + N + r);
        const zd x = ld(&h(i), 0), y = ld(&h(i + 1), 0);
        st(&h(i), 0, c * x + sn * y);
        st(&h(i + 1), 0, c * y - cconj(sn) * x);
    }
    const zd x = ld(&h(j), 0), y = ld(&h(j + 1), 0);
    const double ax = zabs(x), ay = zabs(y), rr = hypot(ax, ay);
    double c;
    zd sn;
    if (rr == 0.0) { c = 1.0; sn = mk(0.0, 0.0); }
    else if (ax == 0.0) { c = 0.0; sn = mk(y.re / ay, -y.im / ay); }
    else { c = ax / rr; sn = (1.0 / rr) * (mk(x.re / ax, x.im / ax) * cconj(y)); }
    st(&h(j), 0, c * x + sn * y);
    h(j + 1) = make_double2(0.0, 0.0);
    cs[(long)j * 2 * N + r] = make_double2(c, 0.0);
    st(cs, (long)j * 2 * N + N + r, sn);
    const zd gj = ld(g, (long)j * N + r);
    st(g, (long)j * N + r, c * gj);
    st(g, (long)(j + 1) * N + r, mk(0.0, 0.0) - cconj(sn) * gj);
    res[r] = zabs(ld(g, (long)(j + 1) * N + r));
}

int dense_givens_step(mpmc_ctx *ctx, double *H, int ldc, int j, int N, double *cs, double *g, double *res) {
    k_givens_step<<<grid_for(N, 64), 64, 0, ctx->stream>>>((double2 *)H, ldc, j, N, (double2 *)cs, (double2 *)g,
                                                          res);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// y = R^-1 g for the leading k x k triangle (rotated H), per rhs; y[i*N + r].
__global__ void k_backsolve(const double2 *H, int ldc, int k, int N, const double2 *g, double2 *y) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    for (int i = k - 1; i >= 0; --i) {
        zd acc = ld(g, (long)i * N + r);
        for (int j = i + 1; j < k; ++j) acc = acc - ld(H, ((long)j * ldc + i) * N + r) * ld(y, (long)j * N + r);
        const zd d = ld(H, ((long)i * ldc + i) * N + r);
        st(y, (long)i * N + r, (d.re == 0 && d.im == 0) ? mk(0.0, 0.0) : zdiv(acc, d));
    }
}

int dense_backsolve(mpmc_ctx *ctx, const double *H, int ldc, int k, int N, const double *g, double *y) {
    k_backsolve<<<grid_for(N, 64), 64, 0, ctx->stream>>>((const double2 *)H, ldc, k, N, (const double2 *)g,
                                                        (double2 *)y);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}
