// Small dense FP64 problems of the method, solved on the device:
//  * harmonic Ritz values of a GMRES(d) cycle, eig(H_d + |h|^2 H_d^-H e_d e_d^T)
//    (Sec. 3), with the GMRES least-squares residual,
//  * eigenvalues of an upper Hessenberg matrix by shifted QR with Givens
//    rotations (Wilkinson shift, exceptional shifts, bottom deflation),
//  * Leja ordering of the roots (Sec. 3),
//  * Ritz vectors by inverse iteration on H - mu I (deflation, Sec. 7),
//  * per-rhs Givens updates and back substitution of restarted GMRES solves.
// The matrices are at most a few hundred rows: one wavefront (64 lanes) works
// on one matrix, which lives in LDS (packed Hessenberg) up to 137 rows and in
// global memory (L2 resident) beyond.  Every loop has a fixed iteration bound.
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
// Matrix accessors: column-major in global memory, or packed upper Hessenberg
// in LDS (column j holds rows 0..min(j+1, n-1) at offset j(j+3)/2).
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) dvec2 lds_dvec2;
struct GlobalMat {
    double2 *A;
    int lda;
    __device__ __forceinline__ double2 &operator()(int i, int j) const { return A[i + (long)j * lda]; }
    __device__ __forceinline__ zd get(int i, int j) const {
        const double2 v = A[i + (long)j * lda];
        return mk(v.x, v.y);
    }
    __device__ __forceinline__ void set(int i, int j, zd v) const { A[i + (long)j * lda] = make_double2(v.re, v.im); }
};
struct PackedMat {
    double2 *A;
    __device__ __forceinline__ double2 &operator()(int i, int j) const { return A[j * (j + 3) / 2 + i]; }
    // direct LDS addressing: the low 32 bits of a flat LDS address are the LDS offset
    __device__ __forceinline__ lds_dvec2 *lds() const { return (lds_dvec2 *)(uintptr_t)(uint32_t)(uintptr_t)A; }
    __device__ __forceinline__ zd get(int i, int j) const {
        const dvec2 v = lds()[j * (j + 3) / 2 + i];
        return mk(v.x, v.y);
    }
    __device__ __forceinline__ void set(int i, int j, zd v) const {
        dvec2 w;
        w.x = v.re;
        w.y = v.im;
        lds()[j * (j + 3) / 2 + i] = w;
    }
};
__host__ __device__ inline long packed_hess_size(int n) { return (long)(n - 1) * (n + 2) / 2 + n; }

// Broadcast of lane `src` (wave-uniform) of a complex double register value.
__device__ __forceinline__ double rdlane(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, src), hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ zd rdlane(zd v, int src) { return mk(rdlane(v.re, src), rdlane(v.im, src)); }

// 1/sqrt(z) for z > 0: hardware estimate plus one Newton step.
__device__ __forceinline__ double rsqrt_nr(double z) {
    const double r = __builtin_amdgcn_rsq(z);
    const double e = fma(-z * r, r, 1.0);
    return fma(0.5 * r, e, r);
}

// Givens rotation G = [c s; -conj(s) c] with G [x; y] = [r; 0], c real >= 0:
// c = |x| / r, s = x conj(y) / (|x| r), r = sqrt(|x|^2 + |y|^2).
__device__ __forceinline__ void givens(zd x, zd y, double &c, zd &sn) {
    const double x2 = x.re * x.re + x.im * x.im, y2 = y.re * y.re + y.im * y.im;
    if (y2 == 0.0) {
        c = 1.0;
        sn = mk(0.0, 0.0);
    } else if (x2 == 0.0) {
        const double iy = rsqrt_nr(y2);
        c = 0.0;
        sn = mk(y.re * iy, -y.im * iy);
    } else {
        const double ix = rsqrt_nr(x2), ir = rsqrt_nr(x2 + y2);
        c = x2 * ix * ir;
        sn = (ix * ir) * (x * cconj(y));
    }
}

template <typename Mat>
__device__ __forceinline__ zd ld_shift(const Mat &a, int i, int j, zd sigma) {   // element of A - sigma
    const zd v = a.get(i, j);
    return i == j ? v - sigma : v;
}

template <int MAXC>
__device__ __forceinline__ zd pick(const zd (&v)[MAXC], int q) {
    zd r = mk(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < MAXC; ++i)
        if (i == q) r = v[i];
    return r;
}

// Eigenvalues of the upper Hessenberg matrix held by `a` (destroyed): shifted
// QR with Givens rotations, Wilkinson shifts, exceptional shifts every 11
// iterations without deflation, deflation from the bottom.  Must be called by
// exactly one wavefront of 64 lanes (n <= 64 * MAXC); returns 0, or -1 on
// non-convergence or NaN.
//
// One QR step A - sigma = QR, A' = RQ + sigma on the active window [l, hi] is
// a single sweep over k = l .. hi-1 without barriers:
//  * rows: lane t owns columns j = t + 64 q.  Row k (already rotated by
//    G_{k-1}) is carried in registers and row k+1 prefetched, so the only
//    cross-lane step is the broadcast (readlane) of the pivot pair
//    (a(k,k), a(k+1,k)) from the lane owning column k; R's row k is stored;
//  * columns, one step behind: lane t owns rows i = l + t + 64 r and applies
//    G_{k-1}^H to columns k-1, k (rows <= k).  Column k is carried in
//    registers; the R entries it needs were stored at least two steps earlier
//    or are broadcast from the lanes that produced them in this step or the
//    last, so no lane reads an element another lane writes in the same step.
// The shift is subtracted when diagonal entries are loaded and added back when
// final diagonal entries are stored.  `cs` is unused (kept for the callers'
// workspace layout).
template <int MAXC, typename Mat>
__device__ int hess_eigvals(Mat a, int n, double2 *ev, double2 *cs) {
    (void)cs;
    const int lane = threadIdx.x;
    int hi = n - 1, iter = 0, total = 0;
    const int max_total = 60 * n + 100;
    int status = 0;
    while (hi >= 0) {
        __syncthreads();
        if (hi == 0) {
            if (lane == 0) st(ev, 0, a.get(0, 0));
            break;
        }
        // l: the largest index in [1, hi] with a negligible subdiagonal a(l, l-1), else 0;
        // 64 subdiagonals are tested at once, from the bottom up
        int l = 0;
        for (int top = hi; top >= 1; top -= 64) {
            const int i = top - lane;
            bool small = false, bad = false;
            if (i >= 1) {
                const zd sv = a.get(i, i - 1), d0 = a.get(i - 1, i - 1), d1 = a.get(i, i);
                const double sub = fabs(sv.re) + fabs(sv.im);
                const double dia = fabs(d0.re) + fabs(d0.im) + fabs(d1.re) + fabs(d1.im);
                bad = !(sub == sub);
                small = sub <= 0.5 * DBL_EPSILON * dia || sub < 1e-300;
            }
            if (__ballot(bad)) {
                status = -1;
                break;
            }
            const unsigned long long m = __ballot(small);
            if (m) {
                l = top - __builtin_ctzll(m);
                break;
            }
        }
        if (status) break;
        if (l == hi) {
            if (lane == 0) st(ev, hi, a.get(hi, hi));
            --hi;
            iter = 0;
            continue;
        }
        if (l == hi - 1) {
            const zd p = a.get(hi - 1, hi - 1), q = a.get(hi - 1, hi), r = a.get(hi, hi - 1),
                     s = a.get(hi, hi);
            const zd half_tr = 0.5 * (p + s);
            const zd det = p * s - q * r;
            const zd disc = zsqrt(half_tr * half_tr - det);
            if (lane == 0) {
                st(ev, hi - 1, half_tr + disc);
                st(ev, hi, half_tr - disc);
            }
            hi -= 2;
            iter = 0;
            continue;
        }
        if (++total > max_total) {
            status = -1;
            break;
        }
        ++iter;
        const zd p = a.get(hi - 1, hi - 1), q = a.get(hi - 1, hi), r = a.get(hi, hi - 1),
                 s = a.get(hi, hi);
        const zd half_tr = 0.5 * (p + s), det = p * s - q * r;
        const zd disc = zsqrt(half_tr * half_tr - det);
        zd e1 = half_tr + disc, e2 = half_tr - disc;
        zd sigma = zabs(e1 - s) <= zabs(e2 - s) ? e1 : e2;
        if (iter % 11 == 10) {
            const double m = zabs(r) + zabs(a.get(hi - 1, hi - 2 >= l ? hi - 2 : hi - 1));
            sigma = s + mk(0.75 * m, 0.4375 * m);
        }
        __syncthreads();   // every lane has read the window before it changes

        zd cur[MAXC], nxt[MAXC];    // rows k and k+1 at the lane's columns
        zd col[MAXC], vk[MAXC];     // a(i, k-1) (rotated) and R(i, k) at the lane's rows
#pragma unroll
        for (int q2 = 0; q2 < MAXC; ++q2) {
            const int j = lane + 64 * q2;
            cur[q2] = nxt[q2] = col[q2] = vk[q2] = mk(0.0, 0.0);
            if (j >= l && j <= hi) {
                cur[q2] = ld_shift(a, l, j, sigma);
                nxt[q2] = ld_shift(a, l + 1, j, sigma);
            }
        }
        double cp = 1.0;            // G_{k-1}
        zd sp = mk(0.0, 0.0);
        for (int k = l; k < hi; ++k) {
            const int qk = k >> 6, lk = k & 63;
            const zd x = rdlane(pick(cur, qk), lk), y = rdlane(pick(nxt, qk), lk);
            double c;
            zd sn;
            givens(x, y, c, sn);
            // row pass: R(k, j) for j >= k; rows k+1 carried
            zd rkk = mk(0.0, 0.0), rkk1 = mk(0.0, 0.0);
#pragma unroll
            for (int q2 = 0; q2 < MAXC; ++q2) {
                const int j = lane + 64 * q2;
                if (j >= k && j <= hi) {
                    const zd u = cur[q2], v = nxt[q2];
                    const zd nr = c * u + sn * v;
                    a.set(k, j, nr);
                    if (j == k) rkk = nr;
                    if (j == k + 1) rkk1 = nr;
                    cur[q2] = j == k ? mk(0.0, 0.0) : c * v - cconj(sn) * u;
                    if (j > k && k + 2 <= hi) nxt[q2] = ld_shift(a, k + 2, j, sigma);
                }
            }
            const zd Rkk = rdlane(rkk, lk);
            const zd Rkk1 = rdlane(rkk1, (k + 1) & 63);
            // column pass, one step behind: G_{k-1}^H on columns k-1, k, rows l..k
#pragma unroll
            for (int r2 = 0; r2 < MAXC; ++r2) {
                const int i = l + lane + 64 * r2;
                if (k > l && i <= k) {
                    const zd u = i == k ? mk(0.0, 0.0) : col[r2];   // a(k, k-1) = 0 in R
                    const zd v = i == k ? Rkk : vk[r2];
                    zd o = cp * u + cconj(sp) * v;
                    if (i == k - 1) o = o + sigma;
                    a.set(i, k - 1, o);
                    col[r2] = cp * v - sp * u;
                } else if (k == l && i == l) {
                    col[r2] = Rkk;
                }
                // R(i, k+1) for the next step: stored by an earlier step, or broadcast
                if (i < k && k + 1 <= hi) vk[r2] = a.get(i, k + 1);
                if (i == k) vk[r2] = Rkk1;
            }
            cp = c;
            sp = sn;
        }
        // last row of R, then G_{hi-1}^H on columns hi-1, hi
        zd rhh = mk(0.0, 0.0);
#pragma unroll
        for (int q2 = 0; q2 < MAXC; ++q2)
            if (lane + 64 * q2 == hi) rhh = cur[q2];
        const zd Rhh = rdlane(rhh, hi & 63);
#pragma unroll
        for (int r2 = 0; r2 < MAXC; ++r2) {
            const int i = l + lane + 64 * r2;
            if (i <= hi) {
                const zd u = i == hi ? mk(0.0, 0.0) : col[r2];
                const zd v = i == hi ? Rhh : vk[r2];
                zd o1 = cp * u + cconj(sp) * v, o2 = cp * v - sp * u;
                if (i == hi - 1) o1 = o1 + sigma;
                if (i == hi) o2 = o2 + sigma;
                a.set(i, hi - 1, o1);
                a.set(i, hi, o2);
            }
        }
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
// H: (d+1) x d column-major (leading dimension ldh), the Arnoldi matrix of a
// GMRES(d) cycle; beta = ||b||.
// Lane 0 runs the Givens QR of Hbar column by column: the first d-1 rotations
// are also the QR of H_d, so r = R_d(d-1, d-1) and f = H_d^-H e_d = Q e_d / conj(r)
// (R_d^H is lower triangular, so R_d^H g = e_d has g = e_d / conj(r)); the last
// rotation gives the least-squares residual |g_d|.  The eigenvalues of
// H_d + |h_{d+1,d}|^2 f e_d^T are found in LDS (packed) when it fits.
// work (global): >= 2*d*d + 8*d + 16 complex doubles.
template <int use_lds>
__global__ __launch_bounds__(64) void k_harmonic_leja(const double2 *H, int ldh, int d, double beta,
                                                      double2 *work, double2 *roots, double *info) {
    extern __shared__ double2 lds_mat[];
    const int tid = threadIdx.x, nt = blockDim.x;
    double2 *A = work;                 // d x d (global path)
    double2 *f = work + (long)d * d;   // d
    double2 *rot = f + d;              // d rotations: (c, 0) then s
    double2 *rs = rot + d;             // d
    double2 *tmp = rs + d;             // d
    double *S = (double *)(tmp + d);   // d doubles
    int *taken = (int *)(S + d);       // d ints
    __shared__ int s_status;
    __shared__ double s_res;
    if (tid == 0) {
        s_status = 0;
        zd gk = mk(beta, 0.0);
        zd rdd = mk(0.0, 0.0);
        for (int j = 0; j < d; ++j) {
            zd x = ld(H, (long)j * ldh);
            for (int i = 0; i < j; ++i) {
                const double c = rot[i].x;
                const zd sn = ld(rs, i);
                const zd y = ld(H, (i + 1) + (long)j * ldh);
                x = c * y - cconj(sn) * x;
            }
            if (j == d - 1) rdd = x;
            const zd y = ld(H, (j + 1) + (long)j * ldh);
            const double ax = zabs(x), ay = zabs(y), rr = hypot(ax, ay);
            double c;
            zd sn;
            if (rr == 0.0) { c = 1.0; sn = mk(0.0, 0.0); }
            else if (ax == 0.0) { c = 0.0; sn = mk(y.re / ay, -y.im / ay); }
            else { c = ax / rr; sn = (1.0 / rr) * (mk(x.re / ax, x.im / ax) * cconj(y)); }
            rot[j] = make_double2(c, 0.0);
            st(rs, j, sn);
            gk = mk(0.0, 0.0) - cconj(sn) * gk;
        }
        s_res = beta > 0 ? zabs(gk) / beta : 0.0;
        // f = Q e_{d-1} / conj(rdd), Q = G_0^H ... G_{d-2}^H
        for (int i = 0; i < d; ++i) f[i] = make_double2(0.0, 0.0);
        f[d - 1] = make_double2(1.0, 0.0);
        for (int k = d - 2; k >= 0; --k) {
            const double c = rot[k].x;
            const zd sn = ld(rs, k);
            const zd u = ld(f, k), v = ld(f, k + 1);
            st(f, k, c * u - sn * v);
            st(f, k + 1, cconj(sn) * u + c * v);
        }
        if (zabs(rdd) == 0.0) s_status = -2;
        const zd inv = zdiv(mk(1.0, 0.0), cconj(rdd));
        for (int i = 0; i < d; ++i) st(f, i, ld(f, i) * inv);
    }
    __syncthreads();
    const zd h = ld(H, d + (long)(d - 1) * ldh);
    const double h2 = h.re * h.re + h.im * h.im;
    const bool corr = h2 > 0.0 && s_status == 0;
    int rc;
    if constexpr (use_lds != 0) {
        PackedMat M{lds_mat};
        for (int j = 0; j < d; ++j)
            for (int i = tid; i <= (j + 1 < d ? j + 1 : d - 1); i += nt) {
                zd v = ld(H, i + (long)j * ldh);
                if (corr && j == d - 1) v = v + h2 * ld(f, i);
                st(&M(i, j), 0, v);
            }
        __syncthreads();
        rc = d <= 128 ? hess_eigvals<2>(M, d, roots, lds_mat + packed_hess_size(d))
                      : hess_eigvals<3>(M, d, roots, lds_mat + packed_hess_size(d));
    } else {
        GlobalMat M{A, d};
        for (long e = tid; e < (long)d * d; e += nt) {
            const int i = (int)(e % d), j = (int)(e / d);
            zd v = (i <= j + 1) ? ld(H, i + (long)j * ldh) : mk(0.0, 0.0);
            if (corr && j == d - 1) v = v + h2 * ld(f, i);
            st(A, e, v);
        }
        __syncthreads();
        rc = hess_eigvals<8>(M, d, roots, rot);   // rot/rs (2d entries) are free again
    }
    if (rc && tid == 0) s_status = -1;
    __syncthreads();
    leja_order(roots, d, tmp, S, taken);
    if (tid == 0) {
        for (int i = 0; i < d; ++i)
            if (!(roots[i].x == roots[i].x) || !(roots[i].y == roots[i].y) || (roots[i].x == 0 && roots[i].y == 0))
                s_status = -1;
        info[0] = s_res;
        info[1] = (double)s_status;
    }
}

// ----------------------------------------------------- added roots --
// Stabilisation of a high-degree polynomial (the added-roots rule for
// polynomial preconditioners): root k with log10 pof(k) > thr, pof(k) =
// prod_{i != k} |1 - theta_k / theta_i|, gets ceil((log10 pof(k) - thr) /
// digits) extra copies; the extended list is Leja ordered.  One wavefront.
// out, tmp: max_out entries; S, taken: max_out entries; count[0] = new size
// (or -1 when it would exceed max_out).
__global__ __launch_bounds__(64) void k_add_roots(const double2 *in, int d, double thr, double digits, int max_out,
                                                  double2 *out, double2 *tmp, double *S, int *taken, int *count) {
    const int tid = threadIdx.x, nt = blockDim.x;
    __shared__ int s_total;
    for (int k = tid; k < d; k += nt) {
        const zd tk = ld(in, k);
        double lp = 0.0;
        for (int i = 0; i < d; ++i) {
            if (i == k) continue;
            const zd q = mk(1.0, 0.0) - zdiv(tk, ld(in, i));
            lp += log10(zabs(q));
        }
        taken[k] = lp > thr ? (int)ceil((lp - thr) / digits) : 0;   // copies of root k
    }
    __syncthreads();
    if (tid == 0) {
        int total = d;
        for (int k = 0; k < d; ++k) total += taken[k];
        s_total = total <= max_out ? total : -1;
        if (s_total > 0) {
            for (int k = 0; k < d; ++k) out[k] = in[k];
            int pos = d;
            for (int k = 0; k < d; ++k)
                for (int c = 0; c < taken[k]; ++c) out[pos++] = in[k];
        }
        count[0] = s_total;
    }
    __syncthreads();
    if (s_total > 0) leja_order(out, s_total, tmp, S, taken);
}

int dense_add_roots(mpmc_ctx *ctx, const double *roots_dev, int d, double thr, double digits, int max_out,
                    double *out_dev, int *count_dev) {
    double2 *work = (double2 *)ws_get(ctx, WS_DENSE, (size_t)max_out * (sizeof(double2) + sizeof(double) + sizeof(int)) + 256);
    if (!work) return MPMC_ENOMEM;
    double *S = (double *)(work + max_out);
    int *taken = (int *)(S + max_out);
    k_add_roots<<<1, 64, 0, ctx->stream>>>((const double2 *)roots_dev, d, thr, digits, max_out, (double2 *)out_dev,
                                           work, S, taken, count_dev);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

static size_t lds_limit(mpmc_ctx *ctx) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) != hipSuccess) v = 65536;
    return (size_t)v;
}

template <typename K>
static bool want_lds(mpmc_ctx *ctx, K kernel, size_t bytes) {
    if (bytes + 4096 > lds_limit(ctx)) return false;   // keep room for the small static LDS arrays
    if (bytes > 65536 && hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)bytes) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return true;
}

int dense_harmonic_leja(mpmc_ctx *ctx, const double *H_dev, int ldh, int d, double beta, double *roots_dev,
                        double *info_dev) {
    if (d < 1 || d > 500) return set_err(ctx, MPMC_EINVAL, "harmonic Ritz: d=%d out of range [1, 500]", d);
    double2 *work = (double2 *)ws_get(ctx, WS_DENSE, ((size_t)d * d + 8 * d + 16) * sizeof(double2));
    if (!work) return MPMC_ENOMEM;
    const size_t lb = (size_t)(packed_hess_size(d) + 2 * d) * sizeof(double2);
    const bool lds = d <= 192 && want_lds(ctx, k_harmonic_leja<1>, lb);   // LDS path: <= 3 columns per lane
    if (lds)
        k_harmonic_leja<1><<<1, 64, lb, ctx->stream>>>((const double2 *)H_dev, ldh, d, beta, work,
                                                       (double2 *)roots_dev, info_dev);
    else
        k_harmonic_leja<0><<<1, 64, 0, ctx->stream>>>((const double2 *)H_dev, ldh, d, beta, work,
                                                      (double2 *)roots_dev, info_dev);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// ------------------------------------------------- eigenvalues of H_m --
template <int use_lds>
__global__ __launch_bounds__(64) void k_hess_eigs(const double2 *H, int ldh, int m, double2 *work, double2 *ev,
                                                  double *info) {
    extern __shared__ double2 lds_mat[];
    int rc;
    if constexpr (use_lds != 0) {
        PackedMat M{lds_mat};
        for (int j = 0; j < m; ++j)
            for (int i = threadIdx.x; i <= (j + 1 < m ? j + 1 : m - 1); i += blockDim.x) M(i, j) = H[i + (long)j * ldh];
        __syncthreads();
        rc = m <= 128 ? hess_eigvals<2>(M, m, ev, lds_mat + packed_hess_size(m))
                      : hess_eigvals<3>(M, m, ev, lds_mat + packed_hess_size(m));
    } else {
        for (long e = threadIdx.x; e < (long)m * m; e += blockDim.x) {
            const int i = (int)(e % m), j = (int)(e / m);
            work[e] = (i <= j + 1) ? H[i + (long)j * ldh] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        rc = hess_eigvals<8>(GlobalMat{work, m}, m, ev, work + (size_t)m * m);
    }
    if (threadIdx.x == 0) info[0] = rc;
}

int dense_hess_eigs(mpmc_ctx *ctx, const double *H_dev, int ldh, int m, double *ev_dev, double *info_dev) {
    if (m < 1 || m > 500) return set_err(ctx, MPMC_EINVAL, "Hessenberg eigenproblem: m=%d out of range", m);
    double2 *work = (double2 *)ws_get(ctx, WS_DENSE, ((size_t)m * m + 2 * m) * sizeof(double2));
    if (!work) return MPMC_ENOMEM;
    const size_t lb = (size_t)(packed_hess_size(m) + 2 * m) * sizeof(double2);
    const bool lds = m <= 192 && want_lds(ctx, k_hess_eigs<1>, lb);   // LDS path: <= 3 columns per lane
    if (lds)
        k_hess_eigs<1><<<1, 64, lb, ctx->stream>>>((const double2 *)H_dev, ldh, m, work, (double2 *)ev_dev, info_dev);
    else
        k_hess_eigs<0><<<1, 64, 0, ctx->stream>>>((const double2 *)H_dev, ldh, m, work, (double2 *)ev_dev, info_dev);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// ------------------------------------------- inverse iteration vectors --
// One workgroup (one wavefront) per eigenvalue mu_q: three solves of
// (H_m - mu I) y = y_prev by Hessenberg LU with adjacent-row pivoting, the row
// operations spread over the lanes; y normalised after each solve.
// Y: m x k column-major.  The factor lives in LDS (packed) when it fits.
template <typename Mat>
__device__ void inverse_iteration(Mat A, const double2 *H, int ldh, int m, zd mq, double hn, double2 *y) {
    const int tid = threadIdx.x, nt = blockDim.x;
    __shared__ int s_swap;
    __shared__ double2 s_red[64];
    for (int i = tid; i < m; i += nt) y[i] = make_double2(1.0, 0.0);
    for (int it = 0; it < 3; ++it) {
        __syncthreads();
        for (int j = 0; j < m; ++j)
            for (int i = tid; i <= (j + 1 < m ? j + 1 : m - 1); i += nt) {
                zd v = ld(H, i + (long)j * ldh);
                if (i == j) v = v - mq;
                st(&A(i, j), 0, v);
            }
        __syncthreads();
        for (int k = 0; k < m; ++k) {
            if (tid == 0) {
                s_swap = (k + 1 < m && zabs(ld(&A(k + 1, k), 0)) > zabs(ld(&A(k, k), 0))) ? 1 : 0;
            }
            __syncthreads();
            if (s_swap) {
                for (int j = k + tid; j < m; j += nt) {
                    const double2 t = A(k, j);
                    A(k, j) = A(k + 1, j);
                    A(k + 1, j) = t;
                }
                if (tid == 0) {
                    const double2 t = y[k];
                    y[k] = y[k + 1];
                    y[k + 1] = t;
                }
            }
            __syncthreads();
            if (tid == 0 && zabs(ld(&A(k, k), 0)) < DBL_EPSILON * hn) A(k, k) = make_double2(DBL_EPSILON * hn, 0.0);
            __syncthreads();
            if (k + 1 < m) {
                const zd l = zdiv(ld(&A(k + 1, k), 0), ld(&A(k, k), 0));
                for (int j = k + 1 + tid; j < m; j += nt)
                    st(&A(k + 1, j), 0, ld(&A(k + 1, j), 0) - l * ld(&A(k, j), 0));
                if (tid == 0) st(y, k + 1, ld(y, k + 1) - l * ld(y, k));
            }
            __syncthreads();
        }
        // back substitution, one row at a time with a lane reduction
        for (int i = m - 1; i >= 0; --i) {
            zd part = mk(0.0, 0.0);
            for (int j = i + 1 + tid; j < m; j += nt) part = part + ld(&A(i, j), 0) * ld(y, j);
            s_red[tid] = make_double2(part.re, part.im);
            __syncthreads();
            if (tid == 0) {
                zd acc = ld(y, i);
                for (int q = 0; q < nt; ++q) acc = acc - ld(s_red, q);
                st(y, i, zdiv(acc, ld(&A(i, i), 0)));
            }
            __syncthreads();
        }
        zd part = mk(0.0, 0.0);
        for (int i = tid; i < m; i += nt) part.re += y[i].x * y[i].x + y[i].y * y[i].y;
        s_red[tid] = make_double2(part.re, 0.0);
        __syncthreads();
        double nr = 0;
        for (int q = 0; q < nt; ++q) nr += s_red[q].x;
        nr = sqrt(nr);
        const double inv = nr > 0 ? 1.0 / nr : 0.0;
        __syncthreads();
        for (int i = tid; i < m; i += nt) y[i] = make_double2(y[i].x * inv, y[i].y * inv);
    }
    __syncthreads();
}

__global__ __launch_bounds__(64) void k_inverse_iteration(const double2 *H, int ldh, int m, const double2 *mu,
                                                          double2 *work, double2 *Y, int use_lds) {
    extern __shared__ double2 lds_mat[];
    const int q = blockIdx.x;
    __shared__ double s_hn;
    if (threadIdx.x == 0) {
        double mx = 0;
        for (int j = 0; j < m; ++j)
            for (int i = 0; i <= (j + 1 < m ? j + 1 : m - 1); ++i) {
                const double2 v = H[i + (long)j * ldh];
                mx = fmax(mx, hypot(v.x, v.y));
            }
        s_hn = mx;
    }
    __syncthreads();
    double2 *y = Y + (long)q * m;
    if (use_lds) {
        inverse_iteration(PackedMat{lds_mat}, H, ldh, m, ld(mu, q), s_hn, y);
    } else {
        inverse_iteration(GlobalMat{work + (size_t)q * m * m, m}, H, ldh, m, ld(mu, q), s_hn, y);
    }
}

int dense_inverse_iteration(mpmc_ctx *ctx, const double *H_dev, int ldh, int m, const double *mu_dev, int k,
                            double *Y_dev) {
    if (k < 1) return MPMC_OK;
    const size_t lb = (size_t)packed_hess_size(m) * sizeof(double2);
    const bool lds = want_lds(ctx, k_inverse_iteration, lb);
    double2 *work = nullptr;
    if (!lds) {
        work = (double2 *)ws_get(ctx, WS_DENSE, (size_t)k * m * m * sizeof(double2));
        if (!work) return MPMC_ENOMEM;
    }
    k_inverse_iteration<<<k, 64, lds ? lb : 0, ctx->stream>>>((const double2 *)H_dev, ldh, m, (const double2 *)mu_dev,
                                                              work, (double2 *)Y_dev, lds ? 1 : 0);
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
