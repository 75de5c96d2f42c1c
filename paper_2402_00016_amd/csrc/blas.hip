// Batched vector kernels on internal-layout vectors: the Gram-Schmidt dot
// products and updates of the GMRES/Arnoldi cycles, norms, quadratic forms
// eta^H Theta y of the trace estimators, precision conversions.
//
// Reductions are per right-hand side and always accumulate in FP64.  A
// workgroup is a 2-D tile: x = RT consecutive right-hand sides (the innermost
// index of the layout, so a wavefront reads one contiguous run), y = CT site
// lanes.  Each workgroup reduces its sites in LDS and writes one partial per
// (vector, workgroup, rhs); a second kernel adds the partials in a fixed order,
// so results are bitwise reproducible (no atomics).
#include <type_traits>

#include "common.h"

namespace {

constexpr int JB = 4;   // basis vectors per thread in the multi-dot

struct Tiling {
    int RT, CT;         // block = RT x CT threads
    int ntile;          // rhs tiles
    int NB;             // site blocks
};

Tiling tiling(const mpmc_ctx *ctx, int N, int groups) {
    Tiling t;
    t.RT = N >= 64 ? 64 : (N >= 32 ? 32 : (N >= 16 ? 16 : (N >= 8 ? 8 : (N >= 4 ? 4 : (N >= 2 ? 2 : 1)))));
    t.CT = 256 / t.RT;
    t.ntile = (N + t.RT - 1) / t.RT;
    const long target = (long)ctx->num_cu * 2048;   // threads in flight
    long nb = target / (256L * t.ntile * (groups > 0 ? groups : 1));
    const long maxnb = (ctx->V + t.CT - 1) / t.CT;
    if (nb < 1) nb = 1;
    if (nb > maxnb) nb = maxnb;
    if (nb > 2048) nb = 2048;
    t.NB = (int)nb;
    return t;
}

template <int P>
__device__ __forceinline__ cpx<double> ldd(const VecRef &v, long e, long si) {
    auto x = Store<P>::ld(v.d, v.sc, e, si);
    return mk((double)x.re, (double)x.im);
}

// partial[j][blk][r] = sum over this block's sites of conj(V_j) Theta w.
// Basis vector j starts vstride_b bytes after vector j-1 and is stored in
// precision PB (FP16S: its scales vscale_off bytes after its data); w in PW.
template <int PB, int PW>
__global__ __launch_bounds__(256) void k_multidot(VecRef Vb, size_t vstride_b, size_t vscale_off, int vN, int nv,
                                                  VecRef w, int N, long V, int theta, double2 *__restrict__ partial,
                                                  int NB) {
    __shared__ double2 red[JB][256];
    const int RT = blockDim.x, CT = blockDim.y;
    const int r = blockIdx.y * RT + threadIdx.x;
    const int j0 = blockIdx.z * JB;
    cpx<double> acc[JB];
#pragma unroll
    for (int q = 0; q < JB; ++q) acc[q] = mk(0.0, 0.0);
    if (r < N) {
        for (long s = (long)blockIdx.x * CT + threadIdx.y; s < V; s += (long)NB * CT) {
            cpx<double> wv[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                wv[k] = ldd<PW>(w, (s * 12 + k) * N + r, s * N + r);
                if (theta && k >= 6) wv[k] = mk(-wv[k].re, -wv[k].im);
            }
#pragma unroll
            for (int q = 0; q < JB; ++q) {
                const int j = j0 + q;
                if (j < nv) {
                    VecRef vj;
                    vj.d = (char *)Vb.d + (size_t)j * vstride_b;
                    vj.sc = PB == MPMC_FP16S ? (float *)((char *)vj.d + vscale_off) : nullptr;
                    const int vr = vN == 1 ? 0 : r;
#pragma unroll
                    for (int k = 0; k < 12; ++k)
                        acc[q] = acc[q] + conjmul(ldd<PB>(vj, (s * 12 + k) * vN + vr, s * vN + vr), wv[k]);
                }
            }
        }
    }
    const int tid = threadIdx.y * RT + threadIdx.x;
#pragma unroll
    for (int q = 0; q < JB; ++q) red[q][tid] = make_double2(acc[q].re, acc[q].im);
    __syncthreads();
    for (int h = CT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.y < h) {
#pragma unroll
            for (int q = 0; q < JB; ++q) {
                double2 a = red[q][tid], b = red[q][tid + h * RT];
                red[q][tid] = make_double2(a.x + b.x, a.y + b.y);
            }
        }
        __syncthreads();
    }
    if (threadIdx.y == 0 && r < N) {
#pragma unroll
        for (int q = 0; q < JB; ++q) {
            const int j = j0 + q;
            if (j < nv) partial[((long)j * NB + blockIdx.x) * N + r] = red[q][threadIdx.x];
        }
    }
}

// sum_b partial[j][b][r] by a 256-thread workgroup in a fixed order (thread t
// adds b = t, t + 256, ..., then a halving tree); the result is in red[0]
// for every thread after the return.
__device__ __forceinline__ void block_sum_partials(const double2 *__restrict__ partial, int NB, int N, int j, int r,
                                                   double2 *red) {
    double2 a = make_double2(0, 0);
    for (int b = threadIdx.x; b < NB; b += 256) {
        double2 v = partial[((long)j * NB + b) * N + r];
        a.x += v.x;
        a.y += v.y;
    }
    red[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[threadIdx.x].x += red[threadIdx.x + h].x;
            red[threadIdx.x].y += red[threadIdx.x + h].y;
        }
        __syncthreads();
    }
}

// out[j*N + r] (+)= sum_b partial[j][b][r]; one workgroup per (j, r).
__global__ __launch_bounds__(256) void k_reduce(const double2 *__restrict__ partial, int NB, int N,
                                                double2 *__restrict__ out, int accumulate, int only_real) {
    __shared__ double2 red[256];
    const int jr = blockIdx.x;
    const int j = jr / N, r = jr % N;
    block_sum_partials(partial, NB, N, j, r, red);
    if (threadIdx.x == 0) {
        double2 v = red[0];
        if (only_real) v.y = 0;
        if (accumulate) {
            out[jr].x += v.x;
            out[jr].y += v.y;
        } else {
            out[jr] = v;
        }
    }
}

// w += sign * sum_j h[j*N + r] V_j ; optional partial[blk][r] = sum |w|^2
// OUTH (FP16S basis, FP32 w): the result is not written back to w but to the
// FP16S vector hout (half values and per-(site, rhs) scales), for a caller
// that needs it only in that form; partial still receives the norms of the
// FP32 result.
template <int PB, int PW, bool OUTH = false>
__global__ __launch_bounds__(256) void k_multiaxpy(VecRef Vb, size_t vstride_b, size_t vscale_off, int vN, int nv,
                                                   VecRef w, int N, long V, const double2 *__restrict__ h, double sign,
                                                   double2 *__restrict__ partial, int NB, int ldh,
                                                   VecRef hout = VecRef{nullptr, nullptr}) {
    using T = typename Store<PW>::real;
    __shared__ double red[256];
    const int RT = blockDim.x, CT = blockDim.y;
    const int r = blockIdx.y * RT + threadIdx.x;
    double nrm = 0;
    if (r < N) {
        for (long s = (long)blockIdx.x * CT + threadIdx.y; s < V; s += (long)NB * CT) {
            cpx<T> acc[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                auto v = Store<PW>::ld(w.d, w.sc, (s * 12 + k) * N + r, 0);
                acc[k] = mk((T)v.re, (T)v.im);
            }
            for (int j = 0; j < nv; ++j) {
                const double2 hj = h[(long)j * ldh + r];
                const cpx<T> c = mk((T)(sign * hj.x), (T)(sign * hj.y));
                const void *vj = (const char *)Vb.d + (size_t)j * vstride_b;
                const float *vsc = PB == MPMC_FP16S ? (const float *)((const char *)vj + vscale_off) : nullptr;
                const int vr = vN == 1 ? 0 : r;
                // all twelve loads first: interleaved with the FMAs the
                // scheduler reuses one register pair and waits for each load
                cpx<T> vv[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    auto v = Store<PB>::ld(vj, vsc, (s * 12 + k) * vN + vr, s * vN + vr);
                    vv[k] = mk((T)v.re, (T)v.im);
                }
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[k] = acc[k] + c * vv[k];
            }
            if constexpr (OUTH) {
                float mx = 0.f;
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    mx = fmaxf(mx, fmaxf(fabsf(acc[k].re), fabsf(acc[k].im)));
                    nrm += (double)acc[k].re * acc[k].re + (double)acc[k].im * acc[k].im;
                }
                const float inv = mx > 0.f ? 1.0f / mx : 0.f;
                __half2 *d = reinterpret_cast<__half2 *>(hout.d);
#pragma unroll
                for (int k = 0; k < 12; ++k)
                    d[(s * 12 + k) * N + r] = __floats2half2_rn(acc[k].re * inv, acc[k].im * inv);
                hout.sc[s * N + r] = mx;
            } else {
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    Store<PW>::st(w.d, (s * 12 + k) * N + r, acc[k]);
                    nrm += (double)acc[k].re * acc[k].re + (double)acc[k].im * acc[k].im;
                }
            }
        }
    }
    if (!partial) return;
    const int tid = threadIdx.y * RT + threadIdx.x;
    red[tid] = nrm;
    __syncthreads();
    for (int hh = CT / 2; hh > 0; hh >>= 1) {
        if ((int)threadIdx.y < hh) red[tid] += red[tid + hh * RT];
        __syncthreads();
    }
    if (threadIdx.y == 0 && r < N) partial[(long)blockIdx.x * N + r] = make_double2(red[threadIdx.x], 0.0);
}

// The middle of a CGS2 step in one pass over the basis: w += sign * sum_j
// h[j*ldh + r] V_j, then partial[j][blk][r] = sum over the block's sites of
// conj(V_j) w (the second pass's dot products, summed by k_reduce).  Component
// by component, the nv <= NVMAX basis values stay in registers between the
// update and the dot, so the basis is read once instead of twice.
template <int P, int NVMAX>
__global__ __launch_bounds__(256) void k_multiaxpy_dot(VecRef Vb, size_t vstride_b, int nv, VecRef w, int N, long V,
                                                       const double2 *__restrict__ h, double sign, int ldh,
                                                       double2 *__restrict__ partial, int NB) {
    using T = typename Store<P>::real;
    __shared__ double2 red[NVMAX][256];
    const int RT = blockDim.x, CT = blockDim.y;
    const int r = blockIdx.y * RT + threadIdx.x;
    cpx<double> d[NVMAX];
#pragma unroll
    for (int j = 0; j < NVMAX; ++j) d[j] = mk(0.0, 0.0);
    if (r < N) {
        cpx<T> c[NVMAX];
#pragma unroll
        for (int j = 0; j < NVMAX; ++j) {
            const double2 hj = j < nv ? h[(long)j * ldh + r] : make_double2(0.0, 0.0);
            c[j] = mk((T)(sign * hj.x), (T)(sign * hj.y));
        }
        for (long s = (long)blockIdx.x * CT + threadIdx.y; s < V; s += (long)NB * CT) {
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const long e = (s * 12 + k) * N + r;
                const auto wv = Store<P>::ld(w.d, nullptr, e, 0);
                cpx<T> acc = mk((T)wv.re, (T)wv.im);
                cpx<T> vv[NVMAX];
#pragma unroll
                for (int j = 0; j < NVMAX; ++j) {
                    if (j < nv) {
                        const auto v = Store<P>::ld((const char *)Vb.d + (size_t)j * vstride_b, nullptr, e, 0);
                        vv[j] = mk((T)v.re, (T)v.im);
                    } else {
                        vv[j] = mk(T(0), T(0));
                    }
                }
#pragma unroll
                for (int j = 0; j < NVMAX; ++j)
                    if (j < nv) acc = acc + c[j] * vv[j];
                Store<P>::st(w.d, e, acc);
                const cpx<double> wd = mk((double)acc.re, (double)acc.im);
#pragma unroll
                for (int j = 0; j < NVMAX; ++j)
                    if (j < nv) d[j] = d[j] + conjmul(mk((double)vv[j].re, (double)vv[j].im), wd);
            }
        }
    }
    // the block's sums over its site rows (threadIdx.y), in a fixed order;
    // thread row y writes the partials of vectors j = y, y + CT, ...
    const int tid = threadIdx.y * RT + threadIdx.x;
#pragma unroll
    for (int j = 0; j < NVMAX; ++j) red[j][tid] = make_double2(d[j].re, d[j].im);
    __syncthreads();
    if (r < N) {
        for (int j = threadIdx.y; j < nv; j += CT) {
            double2 a = red[j][threadIdx.x];
            for (int y = 1; y < CT; ++y) {
                a.x += red[j][y * RT + threadIdx.x].x;
                a.y += red[j][y * RT + threadIdx.x].y;
            }
            partial[((long)j * NB + blockIdx.x) * N + r] = a;
        }
    }
}

// y = a * x + b * y   (uniform complex coefficients)
template <int P>
__global__ void k_axpby(VecRef x, VecRef y, long total, double2 a, double2 b) {
    using T = typename Store<P>::real;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    auto xv = Store<P>::ld(x.d, nullptr, e, 0);
    cpx<T> r = mk((T)a.x, (T)a.y) * mk((T)xv.re, (T)xv.im);
    if (b.x != 0.0 || b.y != 0.0) {   // y is not read when b == 0 (it may be uninitialised)
        auto yv = Store<P>::ld(y.d, nullptr, e, 0);
        r = r + mk((T)b.x, (T)b.y) * mk((T)yv.re, (T)yv.im);
    }
    Store<P>::st(y.d, e, r);
}

// y[e] = coef[r] * x[e] (coef per rhs, FP64) ; invert_sqrt: coef = 1/sqrt(re(c)) (0 if c == 0)
template <int P>
__global__ void k_scale_rhs(VecRef x, VecRef y, long total, int N, const double2 *__restrict__ coef, int mode) {
    using T = typename Store<P>::real;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int r = (int)(e % N);
    double2 c = coef[r];
    if (mode == 1) {
        const double q = c.x;
        c = make_double2(q > 0 ? 1.0 / sqrt(q) : 0.0, 0.0);
    } else if (mode == 2) {   // divide by c
        const double d = c.x * c.x + c.y * c.y;
        c = d > 0 ? make_double2(c.x / d, -c.y / d) : make_double2(0.0, 0.0);
    }
    auto xv = Store<P>::ld(x.d, nullptr, e, 0);
    Store<P>::st(y.d, e, mk((T)c.x, (T)c.y) * mk((T)xv.re, (T)xv.im));
}

// precision conversion between two non-FP16S layouts, or from FP16S
template <int PX, int PY>
__global__ void k_convert(VecRef x, VecRef y, long V, int N) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= V * N) return;
    const long s = t / N;
    const int r = (int)(t - s * N);
    using TY = typename Store<PY>::real;
    if constexpr (PY == MPMC_FP16S) {
        cpx<float> v[12];
        float mx = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            auto a = Store<PX>::ld(x.d, x.sc, (s * 12 + k) * N + r, s * N + r);
            v[k] = mk((float)a.re, (float)a.im);
            mx = fmaxf(mx, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
        }
        const float inv = mx > 0.f ? 1.0f / mx : 0.f;
        __half2 *d = reinterpret_cast<__half2 *>(y.d);
#pragma unroll
        for (int k = 0; k < 12; ++k) d[(s * 12 + k) * N + r] = __floats2half2_rn(v[k].re * inv, v[k].im * inv);
        y.sc[s * N + r] = mx;
    } else {
        cpx<TY> v[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            auto a = Store<PX>::ld(x.d, x.sc, (s * 12 + k) * N + r, s * N + r);
            v[k] = mk((TY)a.re, (TY)a.im);
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) Store<PY>::st(y.d, (s * 12 + k) * N + r, v[k]);
    }
}

// y (FP16S) = coef[r] * x (FP32): k_scale_rhs followed by k_convert in one
// pass, with the same arithmetic (the product in FP32, then the per-(site,
// rhs) scale and the half-precision values).
__global__ void k_convert_scaled_h(VecRef x, VecRef y, long V, int N, const double2 *__restrict__ coef) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= V * N) return;
    const long s = t / N;
    const int r = (int)(t - s * N);
    const double2 c = coef[r];
    cpx<float> v[12];
    float mx = 0.f;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const auto a = Store<MPMC_FP32>::ld(x.d, nullptr, (s * 12 + k) * N + r, 0);
        v[k] = mk((float)c.x, (float)c.y) * mk(a.re, a.im);
        mx = fmaxf(mx, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
    }
    const float inv = mx > 0.f ? 1.0f / mx : 0.f;
    __half2 *d = reinterpret_cast<__half2 *>(y.d);
#pragma unroll
    for (int k = 0; k < 12; ++k) d[(s * 12 + k) * N + r] = __floats2half2_rn(v[k].re * inv, v[k].im * inv);
    y.sc[s * N + r] = mx;
}

template <typename F>
int dispatch_prec(mpmc_ctx *ctx, int prec, F &&f) {
    switch (prec) {
        case MPMC_FP64: f(std::integral_constant<int, MPMC_FP64>()); break;
        case MPMC_FP32: f(std::integral_constant<int, MPMC_FP32>()); break;
        default: return set_err(ctx, MPMC_EINVAL, "precision %d not supported by this kernel", prec);
    }
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// acc[r] += sign * c * t[r]
__global__ void k_scale_acc(const double2 *t, int N, double2 c, double sign, double2 *acc) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    const double2 v = t[r];
    acc[r].x += sign * (c.x * v.x - c.y * v.y);
    acc[r].y += sign * (c.x * v.y + c.y * v.x);
}

// ---- single vectors (nrhs == 1): one thread per complex element ----
// partial[j][blk] = sum over this block's elements of conj(V_j) Theta w
template <int P>
__global__ __launch_bounds__(256) void k_multidot1(VecRef Vb, long vstride, int nv, VecRef w, long n, int theta,
                                                   double2 *__restrict__ partial, int NB) {
    using T = typename Store<P>::real;
    __shared__ double2 red[JB][256];
    const int j0 = blockIdx.y * JB;
    cpx<double> acc[JB];
#pragma unroll
    for (int q = 0; q < JB; ++q) acc[q] = mk(0.0, 0.0);
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)NB * 256) {
        cpx<double> wv = ldd<P>(w, e, 0);
        if (theta && (e % 12) >= 6) wv = mk(-wv.re, -wv.im);
        // loads of the JB vectors issued together (index clamped to the last
        // vector, its contribution masked) instead of one guarded load each
        cpx<double> vq[JB];
#pragma unroll
        for (int q = 0; q < JB; ++q) {
            const int j = j0 + q < nv ? j0 + q : nv - 1;
            VecRef vj;
            vj.d = (char *)Vb.d + (size_t)j * vstride * sizeof(T) * 2;
            vj.sc = nullptr;
            vq[q] = ldd<P>(vj, e, 0);
        }
#pragma unroll
        for (int q = 0; q < JB; ++q)
            if (j0 + q < nv) acc[q] = acc[q] + conjmul(vq[q], wv);
    }
#pragma unroll
    for (int q = 0; q < JB; ++q) red[q][threadIdx.x] = make_double2(acc[q].re, acc[q].im);
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
#pragma unroll
            for (int q = 0; q < JB; ++q) {
                red[q][threadIdx.x].x += red[q][threadIdx.x + h].x;
                red[q][threadIdx.x].y += red[q][threadIdx.x + h].y;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < JB; ++q)
            if (j0 + q < nv) partial[(long)(j0 + q) * NB + blockIdx.x] = red[q][0];
    }
}

// w += sign * sum_j h[j*ldh] V_j ; optional partial[blk] = sum |w|^2
template <int P>
__global__ __launch_bounds__(256) void k_multiaxpy1(VecRef Vb, long vstride, int nv, VecRef w, long n,
                                                    const double2 *__restrict__ h, int ldh, double sign,
                                                    double2 *__restrict__ partial, int NB) {
    using T = typename Store<P>::real;
    __shared__ double red[256];
    double nrm = 0;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)NB * 256) {
        auto v0 = Store<P>::ld(w.d, nullptr, e, 0);
        cpx<T> acc = mk((T)v0.re, (T)v0.im);
        // four basis vectors per iteration, their loads issued together
        int j = 0;
        for (; j + 4 <= nv; j += 4) {
            cpx<T> vq[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const void *vj = (const char *)Vb.d + (size_t)(j + q) * vstride * sizeof(T) * 2;
                auto v = Store<P>::ld(vj, nullptr, e, 0);
                vq[q] = mk((T)v.re, (T)v.im);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double2 hj = h[(long)(j + q) * ldh];
                acc = acc + mk((T)(sign * hj.x), (T)(sign * hj.y)) * vq[q];
            }
        }
        for (; j < nv; ++j) {
            const double2 hj = h[(long)j * ldh];
            const void *vj = (const char *)Vb.d + (size_t)j * vstride * sizeof(T) * 2;
            auto v = Store<P>::ld(vj, nullptr, e, 0);
            acc = acc + mk((T)(sign * hj.x), (T)(sign * hj.y)) * mk((T)v.re, (T)v.im);
        }
        Store<P>::st(w.d, e, acc);
        nrm += (double)acc.re * acc.re + (double)acc.im * acc.im;
    }
    if (!partial) return;
    red[threadIdx.x] = nrm;
    __syncthreads();
    for (int hh = 128; hh > 0; hh >>= 1) {
        if ((int)threadIdx.x < hh) red[threadIdx.x] += red[threadIdx.x + hh];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = make_double2(red[0], 0.0);
}

// End of one single-vector FP64 Arnoldi step, one workgroup: ||w||^2 from the
// partials of the second update (the same sum as k_reduce), then on the first
// wavefront H(:, j) += h2, h_{j+1,j} = ||w||, the breakdown test against the
// running Frobenius norm and the coefficient 1/h of the new basis vector (0
// after a breakdown, which keeps later vectors zero).
__global__ __launch_bounds__(256) void k_arnoldi_finish(const double2 *__restrict__ partial, int NB, double2 *Hcol,
                                                        const double2 *h2, int j, double *state, double2 *scale) {
    // state[0] = running ||H||_F^2, state[1] = d_eff (or -1 while none)
    __shared__ double2 red[256];
    block_sum_partials(partial, NB, 1, 0, 0, red);
    const double wn2 = red[0].x;
    if (threadIdx.x >= 64) return;
    double f = 0.0;
    for (int i = threadIdx.x; i <= j; i += 64) {
        double2 v = Hcol[i];
        v.x += h2[i].x;
        v.y += h2[i].y;
        Hcol[i] = v;
        f += v.x * v.x + v.y * v.y;
    }
    for (int o = 32; o > 0; o >>= 1) f += __shfl_xor(f, o);
    if (threadIdx.x != 0) return;
    double fro = state[0] + f;
    const double hn = sqrt(fmax(wn2, 0.0));
    fro += hn * hn;
    state[0] = fro;
    const bool broken = state[1] >= 0;
    if (broken || hn <= 1e-14 * sqrt(fro) || !(hn == hn)) {
        Hcol[j + 1] = make_double2(0.0, 0.0);
        if (!broken) state[1] = j + 1;
        scale[0] = make_double2(0.0, 0.0);
    } else {
        Hcol[j + 1] = make_double2(hn, 0.0);
        scale[0] = make_double2(1.0 / hn, 0.0);
    }
}

int nb_single(const mpmc_ctx *ctx, long n, int groups) {
    long nb = (long)ctx->num_cu * 8 / (groups > 0 ? groups : 1);
    const long maxnb = (n + 255) / 256;
    if (nb < 8) nb = 8;
    if (nb > maxnb) nb = maxnb;
    if (nb > 2048) nb = 2048;
    return (int)nb;
}

}  // namespace

int blas_scale_acc(mpmc_ctx *ctx, const double *t, int N, double2 c, double sign, double *acc) {
    k_scale_acc<<<grid_for(N, 64), 64, 0, ctx->stream>>>((const double2 *)t, N, c, sign, (double2 *)acc);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// h[j*N + r] (+)= V_j^H Theta w for j < nv.  Vb: nv vectors spaced vstride
// elements (complex) apart.
int blas_multi_dot(mpmc_ctx *ctx, const void *Vb, long vstride, int vN, int nv, const void *w, int nrhs, int prec,
                   double *h_dev, int accumulate, int theta) {
    if (nv <= 0) return MPMC_OK;
    const int groups = (nv + JB - 1) / JB;
    if (nrhs == 1 && vN == 1) {
        const int NB = nb_single(ctx, ctx->n, groups);
        double2 *part = (double2 *)ws_get(ctx, WS_PARTIAL, (size_t)nv * NB * sizeof(double2));
        if (!part) return MPMC_ENOMEM;
        int rc = dispatch_prec(ctx, prec, [&](auto P) {
            k_multidot1<decltype(P)::value><<<dim3(NB, groups), 256, 0, ctx->stream>>>(
                vref(ctx, Vb, 1, prec), vstride, nv, vref(ctx, w, 1, prec), ctx->n, theta, part, NB);
        });
        RET_IF(rc);
        k_reduce<<<nv, 256, 0, ctx->stream>>>(part, NB, 1, (double2 *)h_dev, accumulate, 0);
        HIP_OR_RET(ctx, hipGetLastError());
        return MPMC_OK;
    }
    Tiling t = tiling(ctx, nrhs, groups);
    double2 *part = (double2 *)ws_get(ctx, WS_PARTIAL, (size_t)nv * t.NB * nrhs * sizeof(double2));
    if (!part) return MPMC_ENOMEM;
    dim3 blk(t.RT, t.CT), grd(t.NB, t.ntile, groups);
    const size_t es = prec == MPMC_FP64 ? 16 : 8;
    int rc = dispatch_prec(ctx, prec, [&](auto P) {
        k_multidot<decltype(P)::value, decltype(P)::value><<<grd, blk, 0, ctx->stream>>>(
            vref(ctx, Vb, nrhs, prec), (size_t)vstride * es, 0, vN, nv, vref(ctx, w, nrhs, prec), nrhs, ctx->V, theta,
            part, t.NB);
    });
    RET_IF(rc);
    k_reduce<<<nv * nrhs, 256, 0, ctx->stream>>>(part, t.NB, nrhs, (double2 *)h_dev, accumulate, 0);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// FP16S basis (nrhs-wide batches vstride_b bytes apart) against an FP32 w.
int blas_multi_dot_h(mpmc_ctx *ctx, const void *Vb, size_t vstride_b, int nv, const void *w, int nrhs,
                     double *h_dev, int accumulate) {
    if (nv <= 0) return MPMC_OK;
    const int groups = (nv + JB - 1) / JB;
    Tiling t = tiling(ctx, nrhs, groups);
    double2 *part = (double2 *)ws_get(ctx, WS_PARTIAL, (size_t)nv * t.NB * nrhs * sizeof(double2));
    if (!part) return MPMC_ENOMEM;
    dim3 blk(t.RT, t.CT), grd(t.NB, t.ntile, groups);
    k_multidot<MPMC_FP16S, MPMC_FP32><<<grd, blk, 0, ctx->stream>>>(
        VecRef{const_cast<void *>(Vb), nullptr}, vstride_b, fp16s_scale_offset(ctx, nrhs), nrhs, nv,
        vref(ctx, w, nrhs, MPMC_FP32), nrhs, ctx->V, 0, part, t.NB);
    HIP_OR_RET(ctx, hipGetLastError());
    k_reduce<<<nv * nrhs, 256, 0, ctx->stream>>>(part, t.NB, nrhs, (double2 *)h_dev, accumulate, 0);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

int blas_dot(mpmc_ctx *ctx, const void *x, const void *y, int nrhs, int prec, int theta, double *out_dev) {
    return blas_multi_dot(ctx, x, 0, nrhs, 1, y, nrhs, prec, out_dev, 0, theta);
}

int blas_norm2(mpmc_ctx *ctx, const void *x, int nrhs, int prec, double *out_dev) {
    return blas_multi_dot(ctx, x, 0, nrhs, 1, x, nrhs, prec, out_dev, 0, 0);
}

int blas_arnoldi_update(mpmc_ctx *ctx, const void *V, long vstride, int nv, void *w, const double *h2, double *Hcol,
                        int j, double *state, double *scale, int prec) {
    const int NB = nb_single(ctx, ctx->n, 1);
    double2 *part = (double2 *)ws_get(ctx, WS_PARTIAL, (size_t)NB * sizeof(double2));
    if (!part) return MPMC_ENOMEM;
    if (prec == MPMC_FP64)
        k_multiaxpy1<MPMC_FP64><<<NB, 256, 0, ctx->stream>>>(vref(ctx, V, 1, prec), vstride, nv, vref(ctx, w, 1, prec),
                                                             ctx->n, (const double2 *)h2, 1, -1.0, part, NB);
    else if (prec == MPMC_FP32)
        k_multiaxpy1<MPMC_FP32><<<NB, 256, 0, ctx->stream>>>(vref(ctx, V, 1, prec), vstride, nv, vref(ctx, w, 1, prec),
                                                             ctx->n, (const double2 *)h2, 1, -1.0, part, NB);
    else
        return set_err(ctx, MPMC_EINVAL, "Arnoldi vectors are FP64 or FP32");
    HIP_OR_RET(ctx, hipGetLastError());
    k_arnoldi_finish<<<1, 256, 0, ctx->stream>>>(part, NB, (double2 *)Hcol, (const double2 *)h2, j, state,
                                                 (double2 *)scale);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// w += sign * sum_j h[j*ldh + r] V_j ; if norm2_dev: norm2_dev[r] = ||w_r||^2 (after update)
int blas_multi_axpy(mpmc_ctx *ctx, const void *Vb, long vstride, int vN, int nv, void *w, int nrhs, int prec,
                    const double *h_dev, int ldh, double sign, double *norm2_dev) {
    if (nrhs == 1 && vN == 1) {
        const int NB = nb_single(ctx, ctx->n, 1);
        double2 *part = nullptr;
        if (norm2_dev) {
            part = (double2 *)ws_get(ctx, WS_PARTIAL, (size_t)NB * sizeof(double2));
            if (!part) return MPMC_ENOMEM;
        }
        int rc = dispatch_prec(ctx, prec, [&](auto P) {
            k_multiaxpy1<decltype(P)::value><<<NB, 256, 0, ctx->stream>>>(vref(ctx, Vb, 1, prec), vstride, nv,
                                                                          vref(ctx, w, 1, prec), ctx->n,
                                                                          (const double2 *)h_dev, ldh, sign, part, NB);
        });
        RET_IF(rc);
        if (norm2_dev) {
            k_reduce<<<1, 256, 0, ctx->stream>>>(part, NB, 1, (double2 *)norm2_dev, 0, 1);
            HIP_OR_RET(ctx, hipGetLastError());
        }
        return MPMC_OK;
    }
    Tiling t = tiling(ctx, nrhs, 1);
    double2 *part = nullptr;
    if (norm2_dev) {
        part = (double2 *)ws_get(ctx, WS_PARTIAL, (size_t)t.NB * nrhs * sizeof(double2));
        if (!part) return MPMC_ENOMEM;
    }
    dim3 blk(t.RT, t.CT), grd(t.NB, t.ntile, 1);
    const size_t es = prec == MPMC_FP64 ? 16 : 8;
    int rc = dispatch_prec(ctx, prec, [&](auto P) {
        k_multiaxpy<decltype(P)::value, decltype(P)::value><<<grd, blk, 0, ctx->stream>>>(
            vref(ctx, Vb, nrhs, prec), (size_t)vstride * es, 0, vN, nv, vref(ctx, w, nrhs, prec), nrhs, ctx->V,
            (const double2 *)h_dev, sign, part, t.NB, ldh);
    });
    RET_IF(rc);
    if (norm2_dev) {
        k_reduce<<<nrhs, 256, 0, ctx->stream>>>(part, t.NB, nrhs, (double2 *)norm2_dev, 0, 1);
        HIP_OR_RET(ctx, hipGetLastError());
    }
    return MPMC_OK;
}

// w (FP32) += sign * sum_j h[j*ldh + r] V_j with an FP16S basis
int blas_multi_axpy_h(mpmc_ctx *ctx, const void *Vb, size_t vstride_b, int nv, void *w, int nrhs,
                      const double *h_dev, int ldh, double sign, double *norm2_dev, void *out_h) {
    Tiling t = tiling(ctx, nrhs, 1);
    double2 *part = nullptr;
    if (norm2_dev) {
        part = (double2 *)ws_get(ctx, WS_PARTIAL, (size_t)t.NB * nrhs * sizeof(double2));
        if (!part) return MPMC_ENOMEM;
    }
    dim3 blk(t.RT, t.CT), grd(t.NB, t.ntile, 1);
    if (out_h)
        k_multiaxpy<MPMC_FP16S, MPMC_FP32, true><<<grd, blk, 0, ctx->stream>>>(
            VecRef{const_cast<void *>(Vb), nullptr}, vstride_b, fp16s_scale_offset(ctx, nrhs), nrhs, nv,
            vref(ctx, w, nrhs, MPMC_FP32), nrhs, ctx->V, (const double2 *)h_dev, sign, part, t.NB, ldh,
            vref(ctx, out_h, nrhs, MPMC_FP16S));
    else
        k_multiaxpy<MPMC_FP16S, MPMC_FP32><<<grd, blk, 0, ctx->stream>>>(
            VecRef{const_cast<void *>(Vb), nullptr}, vstride_b, fp16s_scale_offset(ctx, nrhs), nrhs, nv,
            vref(ctx, w, nrhs, MPMC_FP32), nrhs, ctx->V, (const double2 *)h_dev, sign, part, t.NB, ldh);
    HIP_OR_RET(ctx, hipGetLastError());
    if (norm2_dev) {
        k_reduce<<<nrhs, 256, 0, ctx->stream>>>(part, t.NB, nrhs, (double2 *)norm2_dev, 0, 1);
        HIP_OR_RET(ctx, hipGetLastError());
    }
    return MPMC_OK;
}

// w += sign * sum_j h[j*ldh + r] V_j, then h2[j*nrhs + r] = V_j^H w (j < nv):
// one pass over the basis for FP32 storage and nv <= 16 (one basis vector per
// right-hand side), blas_multi_axpy + blas_multi_dot otherwise (an FP64
// version would need twice the registers and spills).
int blas_multi_axpy_dot(mpmc_ctx *ctx, const void *Vb, long vstride, int nv, void *w, int nrhs, int prec,
                        const double *h_dev, int ldh, double sign, double *h2_dev) {
    constexpr int NVMAX = 16;
    if (nv > NVMAX || nrhs < 2 || prec != MPMC_FP32) {
        RET_IF(blas_multi_axpy(ctx, Vb, vstride, nrhs, nv, w, nrhs, prec, h_dev, ldh, sign, nullptr));
        return blas_multi_dot(ctx, Vb, vstride, nrhs, nv, w, nrhs, prec, h2_dev, 0, 0);
    }
    if (nv <= 0) return MPMC_OK;
    Tiling t = tiling(ctx, nrhs, 1);
    double2 *part = (double2 *)ws_get(ctx, WS_PARTIAL, (size_t)nv * t.NB * nrhs * sizeof(double2));
    if (!part) return MPMC_ENOMEM;
    dim3 blk(t.RT, t.CT), grd(t.NB, t.ntile, 1);
    k_multiaxpy_dot<MPMC_FP32, NVMAX><<<grd, blk, 0, ctx->stream>>>(
        vref(ctx, Vb, nrhs, prec), (size_t)vstride * 8, nv, vref(ctx, w, nrhs, prec), nrhs, ctx->V,
        (const double2 *)h_dev, sign, ldh, part, t.NB);
    HIP_OR_RET(ctx, hipGetLastError());
    k_reduce<<<nv * nrhs, 256, 0, ctx->stream>>>(part, t.NB, nrhs, (double2 *)h2_dev, 0, 0);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

int blas_axpby(mpmc_ctx *ctx, const void *x, void *y, int nrhs, int prec, double2 a, double2 b) {
    const long total = ctx->V * 12 * nrhs;
    return dispatch_prec(ctx, prec, [&](auto P) {
        k_axpby<decltype(P)::value><<<grid_for(total, 256), 256, 0, ctx->stream>>>(
            vref(ctx, x, nrhs, prec), vref(ctx, y, nrhs, prec), total, a, b);
    });
}

// y = coef[r] x  (mode 0), y = x / sqrt(re coef[r]) (mode 1), y = x / coef[r] (mode 2)
int blas_scale_rhs(mpmc_ctx *ctx, const void *x, void *y, int nrhs, int prec, const double *coef_dev, int mode) {
    const long total = ctx->V * 12 * nrhs;
    return dispatch_prec(ctx, prec, [&](auto P) {
        k_scale_rhs<decltype(P)::value><<<grid_for(total, 256), 256, 0, ctx->stream>>>(
            vref(ctx, x, nrhs, prec), vref(ctx, y, nrhs, prec), total, nrhs, (const double2 *)coef_dev, mode);
    });
}

// y's per-(site, rhs) scales *= Re coef[r] (FP16S y; its half values stay)
__global__ void k_scale_h(float *__restrict__ sc, long total, int N, const double2 *__restrict__ coef) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    sc[t] = sc[t] * (float)coef[t % N].x;
}

int blas_scale_h(mpmc_ctx *ctx, void *y, int nrhs, const double *coef_dev) {
    const long total = ctx->V * nrhs;
    k_scale_h<<<grid_for(total, 256), 256, 0, ctx->stream>>>(vref(ctx, y, nrhs, MPMC_FP16S).sc, total, nrhs,
                                                            (const double2 *)coef_dev);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

int blas_convert_scaled_h(mpmc_ctx *ctx, const void *x, void *y, int nrhs, const double *coef_dev) {
    k_convert_scaled_h<<<grid_for(ctx->V * nrhs, 256), 256, 0, ctx->stream>>>(
        vref(ctx, x, nrhs, MPMC_FP32), vref(ctx, y, nrhs, MPMC_FP16S), ctx->V, nrhs, (const double2 *)coef_dev);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

int blas_convert(mpmc_ctx *ctx, const void *x, int px, void *y, int py, int nrhs) {
    const long work = ctx->V * nrhs;
    VecRef xr = vref(ctx, x, nrhs, px), yr = vref(ctx, y, nrhs, py);
    const unsigned g = grid_for(work, 256);
    hipStream_t st = ctx->stream;
#define CONV(A, B) \
    if (px == A && py == B) k_convert<A, B><<<g, 256, 0, st>>>(xr, yr, ctx->V, nrhs); else
    CONV(MPMC_FP64, MPMC_FP32)
    CONV(MPMC_FP32, MPMC_FP64)
    CONV(MPMC_FP64, MPMC_FP16S)
    CONV(MPMC_FP16S, MPMC_FP64)
    CONV(MPMC_FP32, MPMC_FP16S)
    CONV(MPMC_FP16S, MPMC_FP32)
    CONV(MPMC_FP64, MPMC_FP64)
    CONV(MPMC_FP32, MPMC_FP32)
    return set_err(ctx, MPMC_EINVAL, "blas_convert: %d -> %d unsupported", px, py);
#undef CONV
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

int blas_zero(mpmc_ctx *ctx, void *y, int nrhs, int prec) {
    HIP_OR_RET(ctx, hipMemsetAsync(y, 0, vec_bytes(ctx, nrhs, prec), ctx->stream));
    return MPMC_OK;
}
