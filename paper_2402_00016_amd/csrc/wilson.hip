// Multi-right-hand-side Wilson-Dirac operator for gfx950.
//
//   (M psi)(x) = psi(x) - kappa sum_mu [ (1 - g gamma_mu) U_mu(x) psi(x+mu)
//                                      + (1 + g gamma_mu) U_mu(x-mu)^H psi(x-mu) ]
// g = +1 for M, -1 for M^H (the operator the paper calls the Wilson-Dirac
// matrix, Sec. 1-2; written out in include/mpmc.h).
//
// Design: one thread per (site, rhs) of the internal layout
// [site][spin*3+colour][rhs], so the lanes of a wavefront read consecutive
// right-hand sides of the same site: every spinor load is a contiguous
// 64-lane access and the site's links and neighbour indices are the same
// address for all lanes (one cache line serves the whole wavefront).  Each
// hop is done on half spinors: (1 +- gamma_mu) has rank 2, so the neighbour
// spinor is projected to two colour vectors, rotated by the SU(3) link and
// expanded back, halving the link multiplications.  Workgroups are numbered
// so each XCD sweeps one contiguous block of sites (stencil neighbours stay in
// that XCD's L2).
#include "common.h"

// Phase codes: 0 -> +1, 1 -> +i, 2 -> -1, 3 -> -i.
template <int CODE, typename T>
__device__ __forceinline__ cpx<T> mulc(cpx<T> z) {
    if constexpr (CODE == 0) return z;
    if constexpr (CODE == 1) return times_i(z);
    if constexpr (CODE == 2) return mk(-z.re, -z.im);
    return times_mi(z);
}

// Projector (1 - gamma_mu) in the DeGrand-Rossi basis, as half spinor
//   h0 = psi0 + c0 psi_{j0},  h1 = psi1 + c1 psi_{j1}
// and its expansion back to four spin components
//   out = (h0, h1, d2 h_{k2}, d3 h_{k3}).
// (1 + gamma_mu) has every c and d negated.
template <int MU>
struct Proj;
template <>
struct Proj<0> {  // gamma_x
    static constexpr int j0 = 3, c0 = 3, j1 = 2, c1 = 3, k2 = 1, d2 = 1, k3 = 0, d3 = 1;
};
template <>
struct Proj<1> {  // gamma_y
    static constexpr int j0 = 3, c0 = 0, j1 = 2, c1 = 2, k2 = 1, d2 = 2, k3 = 0, d3 = 0;
};
template <>
struct Proj<2> {  // gamma_z
    static constexpr int j0 = 2, c0 = 3, j1 = 3, c1 = 1, k2 = 0, d2 = 1, k3 = 1, d3 = 3;
};
template <>
struct Proj<3> {  // gamma_t
    static constexpr int j0 = 2, c0 = 2, j1 = 3, c1 = 2, k2 = 0, d2 = 2, k3 = 1, d3 = 2;
};

struct WParams {
    VecRef b;          // operand of M
    VecRef a;          // additive term (d == nullptr: none)
    VecRef out;
    VecRef y;          // accumulator y += gamma * out (d == nullptr: none)
    const int *nbr;
    const void *links;
    long V;
    int N;
    double kappa;
    double2 alpha, beta, gamma;
    float g;           // +1: M, -1: M^H
    int theta;         // 1: multiply M b by gamma5 before combining
};

template <typename T>
__device__ __forceinline__ cpx<T> ldlink(const void *links, long idx) {
    if constexpr (sizeof(T) == 8) {
        double2 v = reinterpret_cast<const double2 *>(links)[idx];
        return mk(v.x, v.y);
    } else {
        float2 v = reinterpret_cast<const float2 *>(links)[idx];
        return mk(v.x, v.y);
    }
}

template <int P, int MU, bool FWD>
__device__ __forceinline__ void hop(const WParams &p, long s, int r, cpx<typename Store<P>::real> acc[4][3]) {
    using T = typename Store<P>::real;
    using Pr = Proj<MU>;
    const int raw = p.nbr[s * 8 + (FWD ? 0 : 4) + MU];
    const long sn = (long)(raw & 0x7fffffff);
    const T bsign = raw < 0 ? T(-1) : T(1);
    // (1 - g gamma) forward, (1 + g gamma) backward
    const T sg = FWD ? T(p.g) : T(-p.g);
    cpx<T> psi[4][3];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            auto v = Store<P>::ld(p.b.d, p.b.sc, (sn * 12 + sp * 3 + c) * p.N + r, sn * p.N + r);
            psi[sp][c] = mk((T)v.re, (T)v.im);
        }
    cpx<T> h[2][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        h[0][c] = psi[0][c] + sg * mulc<Pr::c0>(psi[Pr::j0][c]);
        h[1][c] = psi[1][c] + sg * mulc<Pr::c1>(psi[Pr::j1][c]);
    }
    // link of this hop: U_mu(x) forward, U_mu(x-mu)^H backward
    const long lb = ((FWD ? s : sn) * 4 + MU) * 9;
    cpx<T> u[3][3];
#pragma unroll
    for (int i = 0; i < 9; ++i) u[i / 3][i % 3] = ldlink<T>(p.links, lb + i);
    cpx<T> uh[2][3];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cpx<T> t = mk(T(0), T(0));
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                if constexpr (FWD) t = t + u[a][bb] * h[q][bb];
                else t = t + conjmul(u[bb][a], h[q][bb]);
            }
            uh[q][a] = bsign * t;
        }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[0][a] = acc[0][a] + uh[0][a];
        acc[1][a] = acc[1][a] + uh[1][a];
        acc[2][a] = acc[2][a] + sg * mulc<Pr::d2>(uh[Pr::k2][a]);
        acc[3][a] = acc[3][a] + sg * mulc<Pr::d3>(uh[Pr::k3][a]);
    }
}

template <int P>
__global__ __launch_bounds__(256) void k_wilson(WParams p) {
    using T = typename Store<P>::real;
    const unsigned tile = xcd_tile(blockIdx.x, gridDim.x);
    const long t = (long)tile * blockDim.x + threadIdx.x;
    if (t >= p.V * p.N) return;
    const long s = t / p.N;
    const int r = (int)(t - s * p.N);

    cpx<T> acc[4][3];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[sp][c] = mk(T(0), T(0));
    hop<P, 0, true>(p, s, r, acc);
    hop<P, 0, false>(p, s, r, acc);
    hop<P, 1, true>(p, s, r, acc);
    hop<P, 1, false>(p, s, r, acc);
    hop<P, 2, true>(p, s, r, acc);
    hop<P, 2, false>(p, s, r, acc);
    hop<P, 3, true>(p, s, r, acc);
    hop<P, 3, false>(p, s, r, acc);

    const T kap = (T)p.kappa;
    const cpx<T> al = mk((T)p.alpha.x, (T)p.alpha.y);
    const cpx<T> be = mk((T)p.beta.x, (T)p.beta.y);
    const cpx<T> ga = mk((T)p.gamma.x, (T)p.gamma.y);
    cpx<T> o[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const long e = (s * 12 + k) * p.N + r;
        auto bv = Store<P>::ld(p.b.d, p.b.sc, e, s * p.N + r);
        cpx<T> mb = mk((T)bv.re - kap * acc[k / 3][k % 3].re, (T)bv.im - kap * acc[k / 3][k % 3].im);
        if (p.theta && k >= 6) mb = mk(-mb.re, -mb.im);
        cpx<T> v = be * mb;
        if (p.a.d) {
            auto av = Store<P>::ld(p.a.d, p.a.sc, e, s * p.N + r);
            v = v + al * mk((T)av.re, (T)av.im);
        }
        o[k] = v;
    }
    if constexpr (P == MPMC_FP16S) {
        float mx = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) mx = fmaxf(mx, fmaxf(fabsf(o[k].re), fabsf(o[k].im)));
        const float inv = mx > 0.f ? 1.0f / mx : 0.f;
        __half2 *d = reinterpret_cast<__half2 *>(p.out.d);
#pragma unroll
        for (int k = 0; k < 12; ++k) d[(s * 12 + k) * p.N + r] = __floats2half2_rn(o[k].re * inv, o[k].im * inv);
        p.out.sc[s * p.N + r] = mx;
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) Store<P>::st(p.out.d, (s * 12 + k) * p.N + r, o[k]);
        if (p.y.d) {
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const long e = (s * 12 + k) * p.N + r;
                auto yv = Store<P>::ld(p.y.d, nullptr, e, 0);
                Store<P>::st(p.y.d, e, mk((T)yv.re, (T)yv.im) + ga * o[k]);
            }
        }
    }
}

int wilson_launch_full(mpmc_ctx *ctx, const void *b, const void *a, void *out, void *y, int nrhs, int prec,
                       double2 alpha, double2 beta, double2 gamma, int dagger, int theta) {
    if (prec == MPMC_FP16S && y) return set_err(ctx, MPMC_EINVAL, "FP16S output cannot accumulate");
    WParams p;
    p.b = vref(ctx, b, nrhs, prec);
    p.a = a ? vref(ctx, a, nrhs, prec) : VecRef{nullptr, nullptr};
    p.out = vref(ctx, out, nrhs, prec);
    p.y = y ? vref(ctx, y, nrhs, prec) : VecRef{nullptr, nullptr};
    p.nbr = ctx->nbr;
    p.links = prec == MPMC_FP64 ? (const void *)ctx->links64 : (const void *)ctx->links32;
    p.V = ctx->V;
    p.N = nrhs;
    p.kappa = ctx->kappa;
    p.alpha = alpha;
    p.beta = beta;
    p.gamma = gamma;
    p.g = dagger ? -1.f : 1.f;
    p.theta = theta;
    const long work = ctx->V * nrhs;
    const int B = 256;
    const unsigned grid = grid_for(work, B);
    if (prec == MPMC_FP64) k_wilson<MPMC_FP64><<<grid, B, 0, ctx->stream>>>(p);
    else if (prec == MPMC_FP32) k_wilson<MPMC_FP32><<<grid, B, 0, ctx->stream>>>(p);
    else k_wilson<MPMC_FP16S><<<grid, B, 0, ctx->stream>>>(p);
    HIP_OR_RET(ctx, hipGetLastError());
    ctx->mvps += (uint64_t)nrhs;
    return MPMC_OK;
}

MPMC_API int mpmc_apply_M(mpmc_ctx *ctx, const void *x, void *y, int nrhs, int prec, int dagger, int theta) {
    if (!ctx) return MPMC_EINVAL;
    if (!x || !y || nrhs < 1 || !prec_ok(prec) || (theta != MPMC_THETA_I && theta != MPMC_THETA_G5))
        return set_err(ctx, MPMC_EINVAL, "mpmc_apply_M: bad argument");
    if (x == y) return set_err(ctx, MPMC_EINVAL, "mpmc_apply_M: x and y must not alias");
    return wilson_launch_full(ctx, x, nullptr, y, nullptr, nrhs, prec, make_double2(0, 0), make_double2(1, 0),
                              make_double2(0, 0), dagger ? 1 : 0, theta == MPMC_THETA_G5 ? 1 : 0);
}
