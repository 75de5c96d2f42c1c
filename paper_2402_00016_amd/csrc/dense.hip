// Small dense FP64 problems of the method, solved on the device:
//  * harmonic Ritz values of a GMRES(d) cycle, eig(H_d + |h|^2 H_d^-H e_d e_d^T)
//    (Sec. 3), with the GMRES least-squares residual,
//  * eigenvalues of an upper Hessenberg matrix by the Aberth-Ehrlich
//    simultaneous iteration (one 16-lane group per eigenvalue, spread over
//    the GPU, one launch per sweep) and, when that has not converged, by
//    shifted QR with Givens rotations (Wilkinson shift, exceptional shifts,
//    bottom deflation) in one workgroup,
//  * Leja ordering of the roots (Sec. 3),
//  * Ritz vectors by inverse iteration on H - mu I (deflation, Sec. 7),
//  * per-rhs Givens updates and back substitution of restarted GMRES solves.
// The matrices are at most a few hundred rows; the QR's matrix lives in LDS
// (packed Hessenberg) up to 192 rows and in global memory (L2 resident)
// beyond.  Every loop has a fixed iteration bound.
#include <cfloat>
#include <climits>

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

// A value every lane holds identically, moved to scalar registers (so that
// branches on it are uniform).
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)b), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ zd uniform(zd v) { return mk(uniform(v.re), uniform(v.im)); }

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
// every thread of a workgroup of QR_THREADS threads (n <= QR_THREADS * MAXC);
// returns 0, or -1 on non-convergence or NaN.
//
// Control (deflation test, 1x1 / 2x2 blocks, shift) runs on the first
// wavefront and reaches the others through `sh`.  One QR step A - sigma = QR,
// A' = RQ + sigma on the active window [l, hi] is a sweep over k = l .. hi + 1
// with one barrier per k:
//  * rows: thread t owns columns j = t + QR_THREADS q and carries rows k and
//    k+1 of those columns in registers.  Every thread forms G_k from the pivot
//    pair (a(k,k), a(k+1,k)), which the owner of column k published in the
//    previous step (double-buffered by k & 1), rotates its columns, stores
//    row k of R and loads row k+2;
//  * columns, two steps behind: thread t owns rows i = l + t + QR_THREADS r
//    and applies G_{k-2}^H to columns k-2, k-1 (rows <= k-1).  Column k-2 is
//    carried in registers; column k-1 of R was stored at least one barrier
//    earlier.  The sets of entries the two passes touch in one step are
//    disjoint.
// The shift is subtracted when diagonal entries are loaded and added back when
// final diagonal entries are stored.
constexpr int QR_THREADS = 256;
struct QrShared {
    double2 xy[2][2];   // pivot pair of step k in xy[k & 1]
    double2 sigma;
    int l, hi, go, status;
};

template <int MAXC, typename Mat>
__device__ int hess_eigvals(Mat a, int n, double2 *ev, QrShared &sh) {
    const int tid = threadIdx.x;
    int hi_w = n - 1, iter = 0, total = 0;   // kept by the first wavefront
    const int max_total = 60 * n + 100;
    while (true) {
        __syncthreads();   // the matrix is final for this round; sh may be rewritten
        if (tid < 64) {
            const int lane = tid;
            int go = 1, l = 0, status = 0;
            zd sigma = mk(0.0, 0.0);
            if (hi_w < 0) {
                go = 0;
            } else if (hi_w == 0) {
                if (lane == 0) st(ev, 0, a.get(0, 0));
                go = 0;
            } else {
                // l: the largest index in [1, hi] with a negligible subdiagonal
                // a(l, l-1), else 0; 64 subdiagonals tested at once from the bottom
                for (int top = hi_w; top >= 1; top -= 64) {
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
                if (status) {
                    go = 0;
                } else if (l == hi_w) {
                    if (lane == 0) st(ev, hi_w, a.get(hi_w, hi_w));
                    --hi_w;
                    iter = 0;
                    go = 2;
                } else if (l == hi_w - 1) {
                    const zd p = a.get(hi_w - 1, hi_w - 1), q = a.get(hi_w - 1, hi_w), r = a.get(hi_w, hi_w - 1),
                             s = a.get(hi_w, hi_w);
                    const zd half_tr = 0.5 * (p + s);
                    const zd det = p * s - q * r;
                    const zd disc = zsqrt(half_tr * half_tr - det);
                    if (lane == 0) {
                        st(ev, hi_w - 1, half_tr + disc);
                        st(ev, hi_w, half_tr - disc);
                    }
                    hi_w -= 2;
                    iter = 0;
                    go = 2;
                } else if (++total > max_total) {
                    status = -1;
                    go = 0;
                } else {
                    ++iter;
                    const zd p = a.get(hi_w - 1, hi_w - 1), q = a.get(hi_w - 1, hi_w), r = a.get(hi_w, hi_w - 1),
                             s = a.get(hi_w, hi_w);
                    const zd half_tr = 0.5 * (p + s), det = p * s - q * r;
                    const zd disc = zsqrt(half_tr * half_tr - det);
                    const zd e1 = half_tr + disc, e2 = half_tr - disc;
                    sigma = zabs(e1 - s) <= zabs(e2 - s) ? e1 : e2;
                    if (iter % 11 == 10) {
                        const double m = zabs(r) + zabs(a.get(hi_w - 1, hi_w - 2 >= l ? hi_w - 2 : hi_w - 1));
                        sigma = s + mk(0.75 * m, 0.4375 * m);
                    }
                }
            }
            if (lane == 0) {
                sh.go = go;
                sh.l = l;
                sh.hi = hi_w;
                sh.status = status;
                sh.sigma = make_double2(sigma.re, sigma.im);
            }
        }
        __syncthreads();
        // the control values are the same in every lane: readfirstlane keeps
        // them (and the sweep's loop) scalar
        const int go = __builtin_amdgcn_readfirstlane(sh.go), l = __builtin_amdgcn_readfirstlane(sh.l),
                  hi = __builtin_amdgcn_readfirstlane(sh.hi);
        const zd sigma = mk(sh.sigma.x, sh.sigma.y);
        if (go == 0) break;
        if (go == 2) continue;

        // ---- one QR sweep on [l, hi]
        zd cur[MAXC], nxt[MAXC], col[MAXC];
#pragma unroll
        for (int q = 0; q < MAXC; ++q) {
            const int j = tid + QR_THREADS * q;
            cur[q] = nxt[q] = col[q] = mk(0.0, 0.0);
            if (j >= l && j <= hi) {
                cur[q] = ld_shift(a, l, j, sigma);
                nxt[q] = ld_shift(a, l + 1, j, sigma);
            }
        }
        zd x = a.get(l, l) - sigma, y = a.get(l + 1, l);
        double c1 = 1.0, c2 = 1.0;          // G_{k-1}, G_{k-2}
        zd s1 = mk(0.0, 0.0), s2 = mk(0.0, 0.0);
        __syncthreads();   // every thread has read the window before row l is overwritten
        for (int k = l; k <= hi + 1; ++k) {
            double c = 1.0;
            zd sn = mk(0.0, 0.0);
            if (k < hi) {
                if (k > l) {
                    x = mk(sh.xy[k & 1][0].x, sh.xy[k & 1][0].y);
                    y = mk(sh.xy[k & 1][1].x, sh.xy[k & 1][1].y);
                }
                givens(uniform(x), uniform(y), c, sn);
#pragma unroll
                for (int q = 0; q < MAXC; ++q) {
                    const int j = tid + QR_THREADS * q;
                    if (j >= k && j <= hi) {
                        const zd u = cur[q], v = nxt[q];
                        a.set(k, j, c * u + sn * v);                        // row k of R
                        const zd nc = j == k ? mk(0.0, 0.0) : c * v - cconj(sn) * u;
                        const zd nn = (j > k && k + 2 <= hi) ? ld_shift(a, k + 2, j, sigma) : mk(0.0, 0.0);
                        cur[q] = nc;
                        nxt[q] = nn;
                        if (j == k + 1 && k + 1 < hi) {                    // pivot pair of step k+1
                            sh.xy[(k + 1) & 1][0] = make_double2(nc.re, nc.im);
                            sh.xy[(k + 1) & 1][1] = make_double2(nn.re, nn.im);
                        }
                        if (j == hi && k == hi - 1) a.set(hi, hi, nc);     // last row of R
                    }
                }
            }
            if (k - 2 >= l) {   // column pass G_{k-2}^H on columns kk, kk+1, rows l .. kk+1
                const int kk = k - 2;
                const bool last = kk == hi - 1;
#pragma unroll
                for (int r = 0; r < MAXC; ++r) {
                    const int i = l + tid + QR_THREADS * r;
                    if (i <= kk + 1) {
                        const zd u = i == kk + 1 ? mk(0.0, 0.0) : (kk == l ? a.get(l, l) : col[r]);
                        const zd v = a.get(i, kk + 1);
                        zd o = c2 * u + cconj(s2) * v;
                        zd w = c2 * v - s2 * u;
                        if (i == kk) o = o + sigma;
                        a.set(i, kk, o);
                        if (last) {
                            if (i == hi) w = w + sigma;
                            a.set(i, hi, w);
                        } else {
                            col[r] = w;
                        }
                    }
                }
            }
            c2 = c1;
            s2 = s1;
            c1 = c;
            s1 = sn;
            __syncthreads();
        }
    }
    return sh.status;
}

// --------------------------------------------------------------- Leja --
// Orders ev[0..n) in place: candidates sorted by (Re, Im) (stable), first the
// largest modulus, then the maximiser of sum log|theta - chosen| (lowest index
// on ties; an exact duplicate, log = -inf, comes last).  Called by every
// thread of a workgroup of nt = blockDim.x threads (a multiple of 64,
// n <= SLOTS nt).  The sort is by rank (each candidate counts those that
// precede it); thread t keeps candidates j = t + nt q and their log sums in
// registers; each step is a workgroup argmax: a wavefront butterfly, then the
// per-wavefront winners through LDS (double-buffered by step parity, one
// barrier per step).  Returns false, leaving ev as it was, when a value is not
// finite.
__device__ __forceinline__ bool leja_better(double v1, int i1, double v2, int i2) {
    if (i1 == INT_MAX) return false;
    if (i2 == INT_MAX) return true;
    return v1 > v2 || (v1 == v2 && i1 < i2);
}
__device__ __forceinline__ bool key_before(double2 a, int ia, double2 b, int ib) {   // (Re, Im), then index
    return a.x < b.x || (a.x == b.x && (a.y < b.y || (a.y == b.y && ia < ib)));
}
template <int SLOTS>
__device__ bool leja_order(double2 *ev, int n) {
    constexpr int MAXN = SLOTS * QR_THREADS;
    __shared__ double2 lin[MAXN], lso[MAXN];
    __shared__ double wv[2][QR_THREADS / 64];
    __shared__ int wi[2][QR_THREADS / 64];
    const int tid = threadIdx.x, nt = blockDim.x, nw = nt / 64;
    int bad = 0;
    for (int j = tid; j < n; j += nt) {
        const double2 v = ev[j];
        lin[j] = v;
        bad |= !isfinite(v.x) || !isfinite(v.y);
    }
    if (__syncthreads_or(bad)) return false;
    for (int j = tid; j < n; j += nt) {
        const double2 v = lin[j];
        int rank = 0;
        for (int i = 0; i < n; ++i) rank += key_before(lin[i], i, v, j) ? 1 : 0;
        lso[rank] = v;
    }
    __syncthreads();
    zd c[SLOTS];
    double S[SLOTS];
    bool taken[SLOTS];
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
        const int j = tid + nt * q;
        c[q] = j < n ? mk(lso[j].x, lso[j].y) : mk(0.0, 0.0);
        S[q] = 0.0;
        taken[q] = j >= n;
    }
    int last = -1;
    for (int step = 0; step < n; ++step) {
        double bv = -INFINITY;
        int bi = INT_MAX;
        const double2 tl = last >= 0 ? lso[last] : make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) {
            if (taken[q]) continue;
            double v;
            if (step == 0) {
                v = hypot(c[q].re, c[q].im);
            } else {
                S[q] += log(hypot(c[q].re - tl.x, c[q].im - tl.y));
                v = S[q];
            }
            if (leja_better(v, tid + nt * q, bv, bi)) {
                bv = v;
                bi = tid + nt * q;
            }
        }
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) {
            const double ov = __shfl_xor(bv, m, 64);
            const int oi = __shfl_xor(bi, m, 64);
            if (leja_better(ov, oi, bv, bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if ((tid & 63) == 0) {
            wv[step & 1][tid >> 6] = bv;
            wi[step & 1][tid >> 6] = bi;
        }
        __syncthreads();
        bv = wv[step & 1][0];
        bi = wi[step & 1][0];
        for (int w = 1; w < nw; ++w)
            if (leja_better(wv[step & 1][w], wi[step & 1][w], bv, bi)) {
                bv = wv[step & 1][w];
                bi = wi[step & 1][w];
            }
        last = bi;
#pragma unroll
        for (int q = 0; q < SLOTS; ++q)
            if (tid + nt * q == last) taken[q] = true;
        if (tid == 0) lin[step] = lso[last];
    }
    __syncthreads();
    for (int j = tid; j < n; j += nt) ev[j] = lin[j];
    __syncthreads();
    return true;
}

// ------------------------------------------- Aberth-Ehrlich eigenvalues --
// All eigenvalues of an unreduced upper Hessenberg A (n x n) at once by the
// Aberth-Ehrlich simultaneous iteration (O. Aberth, Math. Comp. 27 (1973);
// L. W. Ehrlich, Comm. ACM 10 (1967)):
//   z_k <- z_k - N_k / (1 - N_k sum_{j != k} 1 / (z_k - z_j)),
// N_k = det(A - z_k) / det'(A - z_k).  The Newton ratio comes from Hyman's
// method: for B = A - z, x_{n-1} = 1 and B(i, i-1) x_{i-1} = -sum_{j >= i}
// B(i, j) x_j for i = n-1 .. 1; then det B is f = sum_j B(0, j) x_j times a
// product of subdiagonal entries that does not depend on z, so N = f / f'
// with x' from the derivative of the same recurrence.  Each root takes one
// 16-lane DPP row of a wavefront, the lanes splitting the columns
// j = lane + 16 q (x_j, x'_j in registers), so the roots of a sweep run on many
// compute units; one launch is one Jacobi sweep.  A root whose correction has
// fallen below tol |z| (or stopped shrinking below 1e-11 |z|) is frozen.
// Launches after the last root froze return at once; if roots are still
// moving after AB_SWEEPS sweeps, the QR kernels take over.
constexpr int AB_MAXN = 256;     // larger matrices go to the QR kernels directly
constexpr int AB_SWEEPS = 40;    // sweeps before the QR kernels take over
constexpr double AB_TOL = 1e-15;

struct AberthWs {
    double2 *arow;   // n x n row-major copy of A (zero below the subdiagonal)
    double2 *rsub;   // rsub[i] = -1 / A(i, i-1), i >= 1
    double2 *z;      // 2 n estimates: sweep t reads half t & 1, writes the other
    double *wprev;   // n: modulus of each root's last correction
    int *conv;       // n: frozen roots
    int *left;       // AB_SWEEPS + 1: left[t + 1] = roots still moving after sweep t
};
static size_t aberth_bytes(int n) {
    return sizeof(double2) * ((size_t)n * n + 3 * (size_t)n) + sizeof(double) * n + sizeof(int) * ((size_t)n + AB_SWEEPS + 1);
}
static AberthWs aberth_carve(void *base, int n) {
    AberthWs w;
    double2 *p = (double2 *)base;
    w.arow = p;
    p += (size_t)n * n;
    w.rsub = p;
    p += n;
    w.z = p;
    p += 2 * (size_t)n;
    w.wprev = (double *)p;
    w.conv = (int *)(w.wprev + n);
    w.left = w.conv + n;
    return w;
}
__host__ __device__ inline const double2 *aberth_result(const AberthWs &w, int n) {
    return w.z + (size_t)(AB_SWEEPS & 1) * n;
}

// Sum over the 16 lanes of a DPP row with the same bits in every lane: an
// inclusive scan with row_shr 1, 2, 4, 8 (zero fill), then lane 15 broadcast
// with row_newbcast.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double row_sum16(double v) {
    v += dpp_d<0x111>(v);
    v += dpp_d<0x112>(v);
    v += dpp_d<0x114>(v);
    v += dpp_d<0x118>(v);
    return dpp_d<0x15F>(v);
}
__device__ __forceinline__ zd row_sum16(zd v) { return mk(row_sum16(v.re), row_sum16(v.im)); }
// Sum over a group of G = 16 or 32 lanes (two DPP rows joined by a lane-16
// exchange; the same bits in every lane: a + b == b + a).
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    v = row_sum16(v);
    if constexpr (G == 32) v += __shfl_xor(v, 16, 64);
    return v;
}
template <int G>
__device__ __forceinline__ zd group_sum(zd v) { return mk(group_sum<G>(v.re), group_sum<G>(v.im)); }

// Centre = trace / n, radius = ||A - centre||_F / sqrt(n); initial estimates
// on that circle, rotated off the real axis.
__global__ __launch_bounds__(256) void k_aberth_init(const double2 *A, int lda, int n, AberthWs w) {
    __shared__ double red[3][256];
    const int tid = threadIdx.x;
    for (long e = tid; e < (long)n * n; e += 256) {
        const int i = (int)(e / n), j = (int)(e - (long)i * n);
        w.arow[e] = i <= j + 1 ? A[i + (long)j * lda] : make_double2(0.0, 0.0);
    }
    double tr = 0.0, ti = 0.0;
    int reducible = 0;
    for (int i = tid; i < n; i += 256) {
        const zd a = ld(A, i + (long)i * lda);
        tr += a.re;
        ti += a.im;
        const zd sub = i > 0 ? ld(A, i + (long)(i - 1) * lda) : mk(1.0, 0.0);
        reducible |= sub.re == 0.0 && sub.im == 0.0;
        st(w.rsub, i, i > 0 ? zdiv(mk(-1.0, 0.0), sub) : mk(0.0, 0.0));
        w.conv[i] = 0;
        w.wprev[i] = INFINITY;
    }
    for (int t = tid; t <= AB_SWEEPS; t += 256) w.left[t] = t == 0 ? n : 0;
    // A zero subdiagonal entry splits the determinant, which Hyman's
    // recurrence does not see: no sweep runs and the QR takes the matrix.
    if (__syncthreads_or(reducible) && tid == 0) {
        w.left[0] = 0;
        w.left[AB_SWEEPS] = 1;
    }
    red[0][tid] = tr;
    red[1][tid] = ti;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) {
            red[0][tid] += red[0][tid + h];
            red[1][tid] += red[1][tid + h];
        }
        __syncthreads();
    }
    const zd c = mk(red[0][0] / n, red[1][0] / n);
    double f2 = 0.0;
    for (long e = tid; e < (long)n * n; e += 256) {
        const int i = (int)(e / n), j = (int)(e - (long)i * n);
        if (i > j + 1) continue;
        zd a = ld(A, i + (long)j * lda);
        if (i == j) a = a - c;
        f2 += a.re * a.re + a.im * a.im;
    }
    red[2][tid] = f2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) red[2][tid] += red[2][tid + h];
        __syncthreads();
    }
    double R = sqrt(red[2][0] / n);
    if (!(R > 0.0) || !isfinite(R)) R = 1.0;
    for (int k = tid; k < n; k += 256) {
        const double th = 6.283185307179586 * k / n + 0.4;
        w.z[k] = make_double2(c.re + R * cos(th), c.im + R * sin(th));
    }
}

// Row sums of Hyman's recurrence for row i of A (in a[], this lane's
// columns): s = sum_j A(i, j) x_j - z x_i and s' = sum_j A(i, j) x'_j - z x'_i
// - x_i, over the slots p0 .. Q-1.  Columns below i hold x_j = 0 (not computed
// yet), so the sums need no mask.
template <int G, int Q>
__device__ __forceinline__ void hyman_row(const zd (&a)[Q], const zd (&x)[Q], const zd (&xp)[Q], int p0, int n, zd z,
                                          zd xi, zd xpi, zd &s, zd &sp) {
    s = mk(0.0, 0.0);
    sp = mk(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (q < p0) continue;    // a constant once the caller's slot loop is unrolled
        if (G * q >= n) break;   // uniform
        s = s + a[q] * x[q];
        sp = sp + a[q] * xp[q];
    }
    s = group_sum<G>(s) - z * xi;
    sp = group_sum<G>(sp) - z * xpi - xi;
}

template <int G, int Q>
__global__ __launch_bounds__(256) void k_aberth_sweep(AberthWs w, int n, int t, double tol) {
    const double2 *zin = w.z + (size_t)(t & 1) * n;
    double2 *zout = w.z + (size_t)((t + 1) & 1) * n;
    const int g = threadIdx.x & (G - 1);
    const int k = (int)((blockIdx.x * blockDim.x + threadIdx.x) / G);   // the same in all G lanes of the group
    if (k >= n) return;
    const zd zk = ld(zin, k);
    if (w.left[t] == 0 || w.conv[k]) {
        if (g == 0) st(zout, k, zk);
        return;
    }
    zd x[Q], xp[Q], a[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = g + G * q;
        x[q] = mk(j == n - 1 ? 1.0 : 0.0, 0.0);
        xp[q] = mk(0.0, 0.0);
        a[q] = j < n ? ld(w.arow, (long)(n - 1) * n + j) : mk(0.0, 0.0);
    }
    zd xi = mk(1.0, 0.0), xpi = mk(0.0, 0.0);   // x_i, x'_i of the current row (uniform)
    zd rs = ld(w.rsub, n - 1);
    int i = n - 1;
    // Rows in descending order, grouped by the slot QS of their new column
    // i - 1 (unrolled: every register index is a constant); slots below QS
    // hold no computed column yet and are neither summed nor loaded.
#pragma unroll
    for (int QS = Q - 1; QS >= 0; --QS) {
        for (; i >= 1 && i - 1 >= G * QS; --i) {
            zd an[Q];   // row i - 1, in flight while row i is summed
#pragma unroll
            for (int q = QS; q < Q; ++q) {
                const int j = g + G * q;
                an[q] = (G * q < n && j < n) ? ld(w.arow, (long)(i - 1) * n + j) : mk(0.0, 0.0);
            }
            const zd rsn = ld(w.rsub, i - 1);
            zd s, sp;
            hyman_row<G, Q>(a, x, xp, QS, n, zk, xi, xpi, s, sp);
            xi = rs * s;    // x_{i-1}, x'_{i-1}: the same bits in every lane
            xpi = rs * sp;
            const bool own = g == i - 1 - G * QS;
            x[QS].re = own ? xi.re : x[QS].re;
            x[QS].im = own ? xi.im : x[QS].im;
            xp[QS].re = own ? xpi.re : xp[QS].re;
            xp[QS].im = own ? xpi.im : xp[QS].im;
            const double mx = fmax(fmax(fabs(xi.re), fabs(xi.im)), fmax(fabs(xpi.re), fabs(xpi.im)));
            if (mx > 0x1p400) {   // a common power-of-two scale leaves f / f' unchanged
#pragma unroll
                for (int q = QS; q < Q; ++q) {
                    x[q] = 0x1p-400 * x[q];
                    xp[q] = 0x1p-400 * xp[q];
                }
                xi = 0x1p-400 * xi;
                xpi = 0x1p-400 * xpi;
            }
#pragma unroll
            for (int q = QS; q < Q; ++q) a[q] = an[q];
            rs = rsn;
        }
    }
    zd f, fp;
    hyman_row<G, Q>(a, x, xp, 0, n, zk, xi, xpi, f, fp);
    const bool flat = fp.re == 0.0 && fp.im == 0.0;
    const zd N = flat ? mk((double)NAN, (double)NAN) : zdiv(f, fp);   // NaN: no Newton step; the QR takes over
    zd S = mk(0.0, 0.0);
    for (int j = g; j < n; j += G)
        if (j != k) S = S + zdiv(mk(1.0, 0.0), zk - ld(zin, j));
    S = group_sum<G>(S);
    const zd den = mk(1.0, 0.0) - N * S;
    const zd wk = (den.re == 0.0 && den.im == 0.0) ? N : zdiv(N, den);
    if (g == 0) {
        const double aw = hypot(wk.re, wk.im), az = hypot(zk.re, zk.im);
        const bool done = aw <= tol * az || (aw <= 1e-11 * az && aw >= w.wprev[k]);
        st(zout, k, zk - wk);
        w.wprev[k] = aw;
        if (done) w.conv[k] = 1;
        else atomicAdd(&w.left[t + 1], 1);
    }
}

// Runs the iteration on A (n x n, column-major, leading dimension lda) on the
// context stream.  Afterwards w.left[AB_SWEEPS] == 0 means every root froze,
// with the eigenvalues at aberth_result(w, n).
static int aberth_run(mpmc_ctx *ctx, const double2 *A, int lda, int n, const AberthWs &w) {
    k_aberth_init<<<1, 256, 0, ctx->stream>>>(A, lda, n, w);
    // 16 lanes per root up to 128 rows, 32 beyond; at most 8 columns per lane
    const unsigned b16 = (unsigned)((n + 15) / 16), b32 = (unsigned)((n + 7) / 8);
    for (int t = 0; t < AB_SWEEPS; ++t) {
        if (n <= 32) k_aberth_sweep<16, 2><<<b16, 256, 0, ctx->stream>>>(w, n, t, AB_TOL);
        else if (n <= 64) k_aberth_sweep<16, 4><<<b16, 256, 0, ctx->stream>>>(w, n, t, AB_TOL);
        else if (n <= 128) k_aberth_sweep<16, 8><<<b16, 256, 0, ctx->stream>>>(w, n, t, AB_TOL);
        else if (n <= 160) k_aberth_sweep<32, 5><<<b32, 256, 0, ctx->stream>>>(w, n, t, AB_TOL);
        else k_aberth_sweep<32, 8><<<b32, 256, 0, ctx->stream>>>(w, n, t, AB_TOL);
    }
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// The QR kernels' hand-over: when the iteration converged, its eigenvalues
// are copied to ev and the QR is skipped (uniform: every thread reads the same
// flag).
__device__ __forceinline__ bool take_aberth(const int *left, const double2 *zab, int n, double2 *ev) {
    if (!left) return false;
    if (__builtin_amdgcn_readfirstlane(left[AB_SWEEPS]) != 0) return false;
    for (int k = threadIdx.x; k < n; k += blockDim.x) ev[k] = zab[k];
    return true;
}

// ------------------------------------------------ harmonic Ritz + Leja --
// H: (d+1) x d column-major (leading dimension ldh), the Arnoldi matrix of a
// GMRES(d) cycle; beta = ||b||.
// Lane 0 runs the Givens QR of Hbar column by column: the first d-1 rotations
// are also the QR of H_d, so r = R_d(d-1, d-1) and f = H_d^-H e_d = Q e_d / conj(r)
// (R_d^H is lower triangular, so R_d^H g = e_d has g = e_d / conj(r)); the last
// rotation gives the least-squares residual |g_d|.  Then the workgroup writes
// A = H_d + |h_{d+1,d}|^2 f e_d^T (d x d, column-major) for the eigensolvers.
// info[0] = residual / beta, info[1] = 0 or -2 (H_d singular: A = H_d).
struct HarmWs {
    double2 *A;     // d x d
    double2 *f;     // d
    double2 *rot;   // d rotations: (c, 0)
    double2 *rs;    // d: s
    void *ab;       // Aberth workspace (d <= AB_MAXN)
};
__global__ __launch_bounds__(256) void k_harmonic_build(const double2 *H, int ldh, int d, double beta, HarmWs w,
                                                        double *info) {
    const int tid = threadIdx.x, nt = blockDim.x;
    double2 *f = w.f, *rot = w.rot, *rs = w.rs;
    __shared__ int s_status;
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
        info[0] = beta > 0 ? zabs(gk) / beta : 0.0;
        info[1] = (double)s_status;
    }
    __syncthreads();
    const zd h = ld(H, d + (long)(d - 1) * ldh);
    const double h2 = h.re * h.re + h.im * h.im;
    const bool corr = h2 > 0.0 && s_status == 0;
    for (long e = tid; e < (long)d * d; e += nt) {
        const int i = (int)(e % d), j = (int)(e / d);
        zd v = (i <= j + 1) ? ld(H, i + (long)j * ldh) : mk(0.0, 0.0);
        if (corr && j == d - 1) v = v + h2 * ld(f, i);
        st(w.A, e, v);
    }
}

// Eigenvalues of A when the Aberth iteration did not converge (or was not
// run): shifted QR in LDS (packed) when it fits, else in place in global
// memory.  info[1] = -1 on QR failure.
template <int use_lds>
__global__ __launch_bounds__(QR_THREADS) void k_harmonic_qr(HarmWs w, int d, const int *ab_left,
                                                            const double2 *ab_z, double2 *roots, double *info) {
    extern __shared__ double2 lds_mat[];
    __shared__ QrShared qsh;
    if (take_aberth(ab_left, ab_z, d, roots)) return;
    int rc;
    if constexpr (use_lds != 0) {
        PackedMat M{lds_mat};
        for (int j = 0; j < d; ++j)
            for (int i = threadIdx.x; i <= (j + 1 < d ? j + 1 : d - 1); i += blockDim.x) M(i, j) = w.A[i + (long)j * d];
        __syncthreads();
        rc = hess_eigvals<1>(M, d, roots, qsh);
    } else {
        rc = hess_eigvals<2>(GlobalMat{w.A, d}, d, roots, qsh);
    }
    if (rc && threadIdx.x == 0) info[1] = -1.0;
}

// Leja order of the roots, then the checks: info[1] = -1 if a root is not
// finite or zero.
template <int SLOTS>
__global__ __launch_bounds__(QR_THREADS) void k_leja(double2 *roots, int d, double *info) {
    const bool ok = leja_order<SLOTS>(roots, d);
    if (threadIdx.x == 0) {
        bool bad = !ok;
        for (int i = 0; i < d; ++i)
            if (roots[i].x == 0 && roots[i].y == 0) bad = true;
        if (bad) info[1] = -1.0;
    }
}

// ----------------------------------------------------- added roots --
// Stabilisation of a high-degree polynomial (the added-roots rule for
// polynomial preconditioners): root k with log10 pof(k) > thr, pof(k) =
// prod_{i != k} |1 - theta_k / theta_i|, gets ceil((log10 pof(k) - thr) /
// digits) extra copies; the extended list is Leja ordered.  One workgroup.
// out: max_out entries (<= ADD_ROOTS_MAX); taken: d ints; count[0] = new size
// (or -1 when it would exceed max_out).
constexpr int ADD_ROOTS_SLOTS = 5;
constexpr int ADD_ROOTS_MAX = ADD_ROOTS_SLOTS * QR_THREADS;
__global__ __launch_bounds__(QR_THREADS) void k_add_roots(const double2 *in, int d, double thr, double digits,
                                                          int max_out, double2 *out, int *taken, int *count) {
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
    if (s_total > 0) leja_order<ADD_ROOTS_SLOTS>(out, s_total);
}

int dense_add_roots(mpmc_ctx *ctx, const double *roots_dev, int d, double thr, double digits, int max_out,
                    double *out_dev, int *count_dev) {
    if (max_out > ADD_ROOTS_MAX) return set_err(ctx, MPMC_EINVAL, "added roots: at most %d roots", ADD_ROOTS_MAX);
    int *taken = (int *)ws_get(ctx, WS_DENSE, (size_t)d * sizeof(int) + 256);
    if (!taken) return MPMC_ENOMEM;
    k_add_roots<<<1, QR_THREADS, 0, ctx->stream>>>((const double2 *)roots_dev, d, thr, digits, max_out,
                                                   (double2 *)out_dev, taken, count_dev);
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

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int dense_harmonic_leja(mpmc_ctx *ctx, const double *H_dev, int ldh, int d, double beta, double *roots_dev,
                        double *info_dev) {
    if (d < 1 || d > 500) return set_err(ctx, MPMC_EINVAL, "harmonic Ritz: d=%d out of range [1, 500]", d);
    const bool aberth = d <= AB_MAXN && !ctx->dense_qr_only;
    const size_t ba = align256(sizeof(double2) * (size_t)d * d), bv = align256(sizeof(double2) * (size_t)d);
    char *work = (char *)ws_get(ctx, WS_DENSE, ba + 3 * bv + (aberth ? aberth_bytes(d) : 0) + 256);
    if (!work) return MPMC_ENOMEM;
    HarmWs w;
    w.A = (double2 *)work;
    w.f = (double2 *)(work + ba);
    w.rot = (double2 *)(work + ba + bv);
    w.rs = (double2 *)(work + ba + 2 * bv);
    w.ab = work + ba + 3 * bv;
    k_harmonic_build<<<1, 256, 0, ctx->stream>>>((const double2 *)H_dev, ldh, d, beta, w, info_dev);
    const int *ab_left = nullptr;
    const double2 *ab_z = nullptr;
    if (aberth) {
        const AberthWs aw = aberth_carve(w.ab, d);
        RET_IF(aberth_run(ctx, w.A, d, d, aw));
        ab_left = aw.left;
        ab_z = aberth_result(aw, d);
    }
    const size_t lb = (size_t)packed_hess_size(d) * sizeof(double2);
    const bool lds = d <= 192 && want_lds(ctx, k_harmonic_qr<1>, lb);   // LDS path: one column per thread
    if (lds)
        k_harmonic_qr<1><<<1, QR_THREADS, lb, ctx->stream>>>(w, d, ab_left, ab_z, (double2 *)roots_dev, info_dev);
    else
        k_harmonic_qr<0><<<1, QR_THREADS, 0, ctx->stream>>>(w, d, ab_left, ab_z, (double2 *)roots_dev, info_dev);
    k_leja<2><<<1, QR_THREADS, 0, ctx->stream>>>((double2 *)roots_dev, d, info_dev);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// ------------------------------------------------- eigenvalues of H_m --
template <int use_lds>
__global__ __launch_bounds__(QR_THREADS) void k_hess_eigs(const double2 *H, int ldh, int m, double2 *work,
                                                          const int *ab_left, const double2 *ab_z, double2 *ev,
                                                          double *info) {
    extern __shared__ double2 lds_mat[];
    __shared__ QrShared qsh;
    if (take_aberth(ab_left, ab_z, m, ev)) {
        if (threadIdx.x == 0) info[0] = 0.0;
        return;
    }
    int rc;
    if constexpr (use_lds != 0) {
        PackedMat M{lds_mat};
        for (int j = 0; j < m; ++j)
            for (int i = threadIdx.x; i <= (j + 1 < m ? j + 1 : m - 1); i += blockDim.x) M(i, j) = H[i + (long)j * ldh];
        __syncthreads();
        rc = hess_eigvals<1>(M, m, ev, qsh);
    } else {
        for (long e = threadIdx.x; e < (long)m * m; e += blockDim.x) {
            const int i = (int)(e % m), j = (int)(e / m);
            work[e] = (i <= j + 1) ? H[i + (long)j * ldh] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        rc = hess_eigvals<2>(GlobalMat{work, m}, m, ev, qsh);
    }
    if (threadIdx.x == 0) info[0] = rc;
}

int dense_hess_eigs(mpmc_ctx *ctx, const double *H_dev, int ldh, int m, double *ev_dev, double *info_dev) {
    if (m < 1 || m > 500) return set_err(ctx, MPMC_EINVAL, "Hessenberg eigenproblem: m=%d out of range", m);
    const bool aberth = m <= AB_MAXN && !ctx->dense_qr_only;
    const size_t bq = align256(((size_t)m * m + 2 * m) * sizeof(double2));
    char *work = (char *)ws_get(ctx, WS_DENSE, bq + (aberth ? aberth_bytes(m) : 0) + 256);
    if (!work) return MPMC_ENOMEM;
    const int *ab_left = nullptr;
    const double2 *ab_z = nullptr;
    if (aberth) {
        const AberthWs aw = aberth_carve(work + bq, m);
        RET_IF(aberth_run(ctx, (const double2 *)H_dev, ldh, m, aw));
        ab_left = aw.left;
        ab_z = aberth_result(aw, m);
    }
    const size_t lb = (size_t)(packed_hess_size(m) + 2 * m) * sizeof(double2);
    const bool lds = m <= 192 && want_lds(ctx, k_hess_eigs<1>, lb);   // LDS path: one column per thread
    if (lds)
        k_hess_eigs<1><<<1, QR_THREADS, lb, ctx->stream>>>((const double2 *)H_dev, ldh, m, (double2 *)work, ab_left,
                                                           ab_z, (double2 *)ev_dev, info_dev);
    else
        k_hess_eigs<0><<<1, QR_THREADS, 0, ctx->stream>>>((const double2 *)H_dev, ldh, m, (double2 *)work, ab_left,
                                                          ab_z, (double2 *)ev_dev, info_dev);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// ------------------------------------------- inverse iteration vectors --
// One wavefront per eigenvalue mu_q: three solves of (H_m - mu I) y = y_prev by
// Hessenberg LU with adjacent-row pivoting, y normalised after each solve.
// The factor lives in LDS (packed) when it fits, else in global memory; y
// stays in registers, y_j in lane j % 64 of slot j / 64.  Every lane takes the
// same pivot decision from the factor, row operations run over the lanes, and
// the back substitution's row sums are wavefront butterflies (the same bits
// in every lane).  Y: m x k column-major.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
template <int YS>
__device__ __forceinline__ zd y_get(const zd (&y)[YS], int j) {   // j uniform
    zd v = mk(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < YS; ++q)
        if (q == (j >> 6)) v = y[q];
    return rdlane(v, j & 63);
}
template <int YS>
__device__ __forceinline__ void y_set(zd (&y)[YS], int j, zd v) {   // j uniform, v the same in every lane
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < YS; ++q)
        if (q == (j >> 6) && lane == (j & 63)) y[q] = v;
}

template <int YS, typename Mat>
__device__ void inverse_iteration(Mat A, const double2 *H, int ldh, int m, zd mq, double hn, double2 *yout) {
    const int lane = threadIdx.x & 63;
    zd y[YS];
#pragma unroll
    for (int q = 0; q < YS; ++q) y[q] = mk(lane + 64 * q < m ? 1.0 : 0.0, 0.0);
    for (int it = 0; it < 3; ++it) {
        __syncthreads();
        for (int j = 0; j < m; ++j)
            for (int i = lane; i <= (j + 1 < m ? j + 1 : m - 1); i += 64) {
                zd v = ld(H, i + (long)j * ldh);
                if (i == j) v = v - mq;
                st(&A(i, j), 0, v);
            }
        __syncthreads();
        for (int k = 0; k < m; ++k) {
            const zd akk = ld(&A(k, k), 0);
            const zd ak1 = k + 1 < m ? ld(&A(k + 1, k), 0) : mk(0.0, 0.0);
            if (k + 1 < m && zabs(ak1) > zabs(akk)) {   // uniform: every lane reads the same entries
                __syncthreads();
                for (int j = k + lane; j < m; j += 64) {
                    const double2 t = A(k, j);
                    A(k, j) = A(k + 1, j);
                    A(k + 1, j) = t;
                }
                const zd yk = y_get(y, k), yk1 = y_get(y, k + 1);
                y_set(y, k, yk1);
                y_set(y, k + 1, yk);
            }
            __syncthreads();
            zd piv = ld(&A(k, k), 0);
            if (zabs(piv) < DBL_EPSILON * hn) piv = mk(DBL_EPSILON * hn, 0.0);
            __syncthreads();
            if (lane == 0) st(&A(k, k), 0, piv);
            if (k + 1 < m) {
                const zd l = zdiv(ld(&A(k + 1, k), 0), piv);
                for (int j = k + 1 + lane; j < m; j += 64)
                    st(&A(k + 1, j), 0, ld(&A(k + 1, j), 0) - l * ld(&A(k, j), 0));
                y_set(y, k + 1, y_get(y, k + 1) - l * y_get(y, k));
            }
            __syncthreads();
        }
        for (int i = m - 1; i >= 0; --i) {
            zd part = mk(0.0, 0.0);
#pragma unroll
            for (int q = 0; q < YS; ++q) {
                const int j = lane + 64 * q;
                if (j > i && j < m) part = part + ld(&A(i, j), 0) * y[q];
            }
            const zd sum = mk(wave_sum(part.re), wave_sum(part.im));
            y_set(y, i, zdiv(y_get(y, i) - sum, ld(&A(i, i), 0)));
        }
        double nr = 0.0;
#pragma unroll
        for (int q = 0; q < YS; ++q) nr += y[q].re * y[q].re + y[q].im * y[q].im;
        nr = sqrt(wave_sum(nr));
        const double inv = nr > 0 ? 1.0 / nr : 0.0;
#pragma unroll
        for (int q = 0; q < YS; ++q) y[q] = inv * y[q];
    }
#pragma unroll
    for (int q = 0; q < YS; ++q)
        if (lane + 64 * q < m) st(yout, lane + 64 * q, y[q]);
}

template <int YS>
__global__ __launch_bounds__(64) void k_inverse_iteration(const double2 *H, int ldh, int m, const double2 *mu,
                                                          double2 *work, double2 *Y, int use_lds) {
    extern __shared__ double2 lds_mat[];
    const int q = blockIdx.x;
    double mx = 0.0;
    for (int j = 0; j < m; ++j)
        for (int i = threadIdx.x; i <= (j + 1 < m ? j + 1 : m - 1); i += 64) {
            const double2 v = H[i + (long)j * ldh];
            mx = fmax(mx, hypot(v.x, v.y));
        }
    const double hn = wave_max(mx);
    double2 *y = Y + (long)q * m;
    if (use_lds) {
        inverse_iteration<YS>(PackedMat{lds_mat}, H, ldh, m, ld(mu, q), hn, y);
    } else {
        inverse_iteration<YS>(GlobalMat{work + (size_t)q * m * m, m}, H, ldh, m, ld(mu, q), hn, y);
    }
}

int dense_inverse_iteration(mpmc_ctx *ctx, const double *H_dev, int ldh, int m, const double *mu_dev, int k,
                            double *Y_dev) {
    if (k < 1) return MPMC_OK;
    if (m > 512) return set_err(ctx, MPMC_EINVAL, "inverse iteration: m=%d above 512", m);
    const size_t lb = (size_t)packed_hess_size(m) * sizeof(double2);
    const int ys = m <= 128 ? 2 : (m <= 256 ? 4 : 8);
    const bool lds = ys == 2 ? want_lds(ctx, k_inverse_iteration<2>, lb)
                             : (ys == 4 ? want_lds(ctx, k_inverse_iteration<4>, lb) : want_lds(ctx, k_inverse_iteration<8>, lb));
    double2 *work = nullptr;
    if (!lds) {
        work = (double2 *)ws_get(ctx, WS_DENSE, (size_t)k * m * m * sizeof(double2));
        if (!work) return MPMC_ENOMEM;
    }
    const double2 *Hd = (const double2 *)H_dev, *mud = (const double2 *)mu_dev;
    double2 *Yd = (double2 *)Y_dev;
    const size_t sh = lds ? lb : 0;
    if (ys == 2) k_inverse_iteration<2><<<k, 64, sh, ctx->stream>>>(Hd, ldh, m, mud, work, Yd, lds ? 1 : 0);
    else if (ys == 4) k_inverse_iteration<4><<<k, 64, sh, ctx->stream>>>(Hd, ldh, m, mud, work, Yd, lds ? 1 : 0);
    else k_inverse_iteration<8><<<k, 64, sh, ctx->stream>>>(Hd, ldh, m, mud, work, Yd, lds ? 1 : 0);
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

MPMC_API int mpmc_set_dense_method(mpmc_ctx *ctx, int method) {
    if (!ctx) return MPMC_EINVAL;
    if (method != 0 && method != 1) return set_err(ctx, MPMC_EINVAL, "mpmc_set_dense_method: method %d", method);
    ctx->dense_qr_only = method;
    return MPMC_OK;
}
