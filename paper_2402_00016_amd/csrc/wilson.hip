// Multi-right-hand-side Wilson-Dirac operator for gfx950.
//
//   (M psi)(x) = psi(x) - kappa sum_mu [ (1 - g gamma_mu) U_mu(x) psi(x+mu)
//                                      + (1 + g gamma_mu) U_mu(x-mu)^H psi(x-mu) ]
// g = +1 for M, -1 for M^H (the operator the paper calls the Wilson-Dirac
// matrix, Sec. 1-2; written out in include/mpmc.h).
//
// Design.  One thread per (site, rhs) of the internal layout
// [site][spin*3+colour][rhs]: the lanes of a wavefront read consecutive
// right-hand sides of the same site, so every spinor load is one contiguous
// 64-lane access.  When the batch size is a multiple of 64 every wavefront
// sits on a single site ("uniform" kernels): the neighbour indices are
// wave-uniform (scalar loads), and each SU(3) link is fetched with ONE vector
// load in which lane i holds dword i of the link, then broadcast to SGPRs
// with v_readlane at use (one VGPR per link in flight instead of 18-36).
// Each hop works on half spinors: the rank-2 projector (1 +- gamma_mu) maps
// the neighbour spinor to two colour vectors, the link multiplies those two
// (FMA chains in FP32), and the result is expanded back.  Workgroups are
// numbered so that each XCD sweeps one contiguous range of tiles.  The
// uniform kernel has six variants (occupancy target x three traversal orders,
// one of them 4D-blocked through a site table) that the autotuner chooses
// between; they compute identical bits.  FP16S operands
// can be written out as FP32 (the FP16 Krylov bases of the solves).
//
// Kernels:
//   k_wilson     out = alpha a + beta Theta op(b) [; y += gamma out]
//   k_wilson_dot one step of a polynomial recurrence on a batch of noise
//                vectors, w' = w - c M w, without forming p(M) eta: the
//                quadratic form eta^H Theta w' is accumulated on the fly
//                (eta regenerated from 2-bit Z(4) codes), so a step moves one
//                spinor read and one spinor write per (site, rhs).
#include <algorithm>

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

template <int P>
struct LinkT {
    using type = float2;
};
template <>
struct LinkT<MPMC_FP64> {
    using type = double2;
};

// Read-only inputs of a Wilson application.
template <int P>
struct WIn {
    const void *__restrict__ b;                  // operand of M
    const float *__restrict__ bsc;               // its FP16S scales
    const int *__restrict__ nbr;
    const typename LinkT<P>::type *__restrict__ links;
    __amdgpu_buffer_rsrc_t vrs;                  // narrow-chunk kernels: all of b (< 4 GiB)
};

// Element k of site sn, rhs r.  The row base (sn*12 + k)*N is formed as a
// pointer first (wave-uniform in the uniform kernels, so it lives in SGPRs) and
// the lane offset r*sizeof(element) is a 32-bit unsigned byte offset shared by
// every access of the thread: the backend can then use SGPR-base +
// VGPR-offset addressing instead of a 64-bit address per load.
template <typename E, bool UNI>
__device__ __forceinline__ E at(const void *base, long row, uint32_t voff) {
    return *reinterpret_cast<const E *>(reinterpret_cast<const char *>(reinterpret_cast<const E *>(base) + row) + voff);
}
template <typename E, bool UNI>
__device__ __forceinline__ void at_w(void *base, long row, uint32_t voff, E v) {
    *reinterpret_cast<E *>(reinterpret_cast<char *>(reinterpret_cast<E *>(base) + row) + voff) = v;
}

template <int P>
struct Elem {
    using type = float2;
};
template <>
struct Elem<MPMC_FP64> {
    using type = double2;
};
template <>
struct Elem<MPMC_FP16S> {
    using type = __half2;
};

template <int P, bool UNI>
__device__ __forceinline__ cpx<typename Store<P>::real> ldspin(const void *b, const float *bsc, long sn, int k,
                                                                int N, uint32_t r) {
    using T = typename Store<P>::real;
    const long row = (sn * 12 + k) * (long)N;
    if constexpr (P == MPMC_FP16S) {
        const float2 f = __half22float2(at<__half2, UNI>(b, row, r * 4u));
        const float sc = at<float, UNI>(bsc, sn * (long)N, r * 4u);
        return mk(f.x * sc, f.y * sc);
    } else if constexpr (P == MPMC_FP32) {
        const float2 v = at<float2, UNI>(b, row, r * 8u);
        return mk((T)v.x, (T)v.y);
    } else {
        const double2 v = at<double2, UNI>(b, row, r * 16u);
        return mk(v.x, v.y);
    }
}

template <int P, bool UNI>
__device__ __forceinline__ void stspin(void *o, long s, int k, int N, uint32_t r, cpx<typename Store<P>::real> v) {
    const long row = (s * 12 + k) * (long)N;
    if constexpr (P == MPMC_FP32) {
        at_w<float2, UNI>(o, row, r * 8u, make_float2(v.re, v.im));
    } else {
        at_w<double2, UNI>(o, row, r * 16u, make_double2(v.re, v.im));
    }
}

// Buffer-resource access for the uniform kernels: one 4-SGPR descriptor per
// site covers its 12 x N elements; component k sits at the scalar offset
// k*N*sizeof(element) and the lane's right-hand side at the shared VGPR offset
// r*sizeof(element).  Out-of-range accesses return 0 (hardware bounds check).
// Values cross the builtins as whole vectors (bit_cast of the full vector).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
constexpr int kBufWord3 = 0x00020000;   // gfx9-family raw buffer descriptor word 3

template <int P>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t site_rsrc(const void *base, long site, int N) {
    constexpr int es = P == MPMC_FP64 ? 16 : 8;
    const char *p = reinterpret_cast<const char *>(base) + site * 12L * N * es;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(p), (short)0, 12 * N * es, kBufWord3);
}

template <int P>
__device__ __forceinline__ cpx<typename Store<P>::real> ldbuf(__amdgpu_buffer_rsrc_t rs, int k, int N, uint32_t r) {
    if constexpr (P == MPMC_FP64) {
        const f64x2 v = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(r * 16u), k * N * 16, 0));
        return mk(v.x, v.y);
    } else {
        const f32x2 v = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(r * 8u), k * N * 8, 0));
        return mk(v.x, v.y);
    }
}

// A store of more than 64 bits of data has a hazard: a VALU write to its data
// registers in the next cycle can replace the data before the store reads it.
// The compiler guards global stores but not buffer stores whose scalar offset
// is a register (it assumes the hazard away), and such writes follow these
// stores in the generated code; a complex double is therefore stored as two
// 64-bit halves.
template <int P>
__device__ __forceinline__ void stbuf(__amdgpu_buffer_rsrc_t rs, int k, int N, uint32_t r,
                                      cpx<typename Store<P>::real> v) {
    if constexpr (P == MPMC_FP64) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v.re), rs, (int)(r * 16u), k * N * 16, 0);
        __builtin_amdgcn_sched_barrier(0);   // keeps the halves from being merged back into one store
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v.im), rs, (int)(r * 16u + 8u), k * N * 16, 0);
    } else {
        f32x2 d;
        d.x = v.re;
        d.y = v.im;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, d), rs, (int)(r * 8u), k * N * 8, 0);
    }
}

// Per-site accessor: buffer resource in the uniform FP32/FP64 kernels, plain
// global addressing otherwise.
template <int P, bool UNI>
struct SiteAcc {
    static constexpr bool kBuf = UNI && P != MPMC_FP16S;
    __amdgpu_buffer_rsrc_t rs;
    const void *b;
    const float *bsc;
    long site;
    int N;
    uint32_t r;
    __device__ __forceinline__ SiteAcc(const void *b_, const float *bsc_, long site_, int N_, uint32_t r_)
        : b(b_), bsc(bsc_), site(site_), N(N_), r(r_) {
        if constexpr (kBuf) rs = site_rsrc<P>(b_, site_, N_);
    }
    __device__ __forceinline__ cpx<typename Store<P>::real> ld(int k) const {
        if constexpr (kBuf) return ldbuf<P>(rs, k, N, r);
        else return ldspin<P, UNI>(b, bsc, site, k, N, r);
    }
    // FP32 store with the non-temporal policy (cache-policy bit 1): the L2
    // keeps the line first in line for eviction, leaving its capacity to lines
    // that other workgroups of the XCD are about to read
    __device__ __forceinline__ void st_stream(int k, cpx<float> v) const {
        static_assert(kBuf && P == MPMC_FP32, "FP32 buffer accessor only");
        f32x2 d;
        d.x = v.re;
        d.y = v.im;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, d), rs, (int)(r * 8u), k * N * 8, 2);
    }
    __device__ __forceinline__ void st(int k, cpx<typename Store<P>::real> v) const {
        if constexpr (kBuf) stbuf<P>(rs, k, N, r, v);
        else stspin<P, UNI>(const_cast<void *>(b), site, k, N, r, v);
    }
};

// One hop split in two so consecutive hops can be software-pipelined: fetch()
// issues the neighbour's 12 spinor loads and the link's 9 loads; apply() does
// the projection, the SU(3) multiply and the accumulation.
template <int P>
struct HopData {
    using T = typename Store<P>::real;
    cpx<T> psi[12];
    cpx<T> u[9];       // generic kernels: the link, per lane
    uint32_t lw[3];    // uniform kernels: the link spread over lanes (dword i of the link in lane i);
                       // narrow-chunk kernels: over each 16-lane row (dword 16 v + i in lane i of lw[v])
    T bsign;
};

// Uniform kernels load a link with ONE vector load in which lane i fetches
// dword i of the 18 (FP32) or 36 (FP64) dwords; the values move to SGPRs with
// v_readlane at use.  One VGPR per link in flight, and its completion is
// tracked in order with the spinor loads (scalar loads complete out of order,
// which would make each hop wait for the prefetched next link).
template <int P>
__device__ __forceinline__ void load_link_lanes(const typename LinkT<P>::type *lk, uint32_t lw[2]) {
    const uint32_t *d = reinterpret_cast<const uint32_t *>(lk);
    const unsigned lane = threadIdx.x & 63u;
    if constexpr (P == MPMC_FP64) {
        lw[0] = d[lane < 36u ? lane : 0u];
    } else {
        lw[0] = d[lane < 18u ? lane : 0u];
    }
}

template <int P>
__device__ __forceinline__ cpx<typename Store<P>::real> link_lane(const uint32_t lw[2], int i) {
    if constexpr (P == MPMC_FP64) {
        const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)lw[0], 4 * i + 0);
        const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)lw[0], 4 * i + 1);
        const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)lw[0], 4 * i + 2);
        const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)lw[0], 4 * i + 3);
        return mk(__builtin_bit_cast(double, ((uint64_t)b << 32) | a), __builtin_bit_cast(double, ((uint64_t)d << 32) | c));
    } else {
        const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)lw[0], 2 * i + 0);
        const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)lw[0], 2 * i + 1);
        return mk(__builtin_bit_cast(float, a), __builtin_bit_cast(float, b));
    }
}

// Narrow-chunk kernels (two or four sites per wavefront, one site per group
// of 16 or 32 lanes): every 16-lane row loads its site's link, lane i of the
// row dword i (and 16 + i, 32 + i), and a value is broadcast within the rows
// with DPP row_newbcast.  Spinors go through one buffer resource covering the
// whole operand: the lane's site row is a 32-bit VGPR offset, the component a
// scalar offset.
template <int P>
__device__ __forceinline__ void load_link_rows(const typename LinkT<P>::type *lk, uint32_t lw[3]) {
    const uint32_t *d = reinterpret_cast<const uint32_t *>(lk);
    const unsigned i = threadIdx.x & 15u;
    lw[0] = d[i];
    if constexpr (P == MPMC_FP64) {
        lw[1] = d[16 + i];
        lw[2] = d[32 + (i < 4u ? i : 0u)];
    } else {
        lw[1] = d[16 + (i < 2u ? i : 0u)];
    }
}
template <int D>
__device__ __forceinline__ uint32_t link_row_dword(const uint32_t lw[3]) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)lw[D / 16], 0x150 + (D % 16), 0xf, 0xf, true);
}
template <int P, int I>
__device__ __forceinline__ cpx<typename Store<P>::real> link_row_t(const uint32_t lw[3]) {
    if constexpr (P == MPMC_FP64) {
        const uint32_t a = link_row_dword<4 * I>(lw), b = link_row_dword<4 * I + 1>(lw);
        const uint32_t c = link_row_dword<4 * I + 2>(lw), d = link_row_dword<4 * I + 3>(lw);
        return mk(__builtin_bit_cast(double, ((uint64_t)b << 32) | a), __builtin_bit_cast(double, ((uint64_t)d << 32) | c));
    } else {
        return mk(__builtin_bit_cast(float, link_row_dword<2 * I>(lw)), __builtin_bit_cast(float, link_row_dword<2 * I + 1>(lw)));
    }
}
template <int P>
__device__ __forceinline__ cpx<typename Store<P>::real> link_row(const uint32_t lw[3], int i) {
    switch (i) {   // i is a constant after unrolling; the DPP control must be one
    case 0: return link_row_t<P, 0>(lw);
    case 1: return link_row_t<P, 1>(lw);
    case 2: return link_row_t<P, 2>(lw);
    case 3: return link_row_t<P, 3>(lw);
    case 4: return link_row_t<P, 4>(lw);
    case 5: return link_row_t<P, 5>(lw);
    case 6: return link_row_t<P, 6>(lw);
    case 7: return link_row_t<P, 7>(lw);
    default: return link_row_t<P, 8>(lw);
    }
}

// One operand through a single buffer resource: per-lane site row offset,
// per-component scalar offset (FP64 / FP32 storage, operand < 4 GiB).
template <int P>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t vec_rsrc(const void *base, long V, int N) {
    constexpr long es = P == MPMC_FP64 ? 16 : 8;
    const unsigned long bytes = (unsigned long)V * 12 * N * es;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0,
                                             (int)(uint32_t)(bytes < 0xffffffffUL ? bytes : 0xffffffffUL), kBufWord3);
}
template <int P>
struct VecAcc {
    __amdgpu_buffer_rsrc_t rs;
    uint32_t vo;
    int N;
    __device__ __forceinline__ VecAcc(__amdgpu_buffer_rsrc_t rs_, long site, int N_, uint32_t r) : rs(rs_), N(N_) {
        constexpr long es = P == MPMC_FP64 ? 16 : 8;
        vo = (uint32_t)((site * 12 * N_ + r) * es);
    }
    __device__ __forceinline__ cpx<typename Store<P>::real> ld(int k) const {
        if constexpr (P == MPMC_FP64) {
            const f64x2 v = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)vo, k * N * 16, 0));
            return mk(v.x, v.y);
        } else {
            const f32x2 v = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)vo, k * N * 8, 0));
            return mk(v.x, v.y);
        }
    }
    __device__ __forceinline__ void st(int k, cpx<typename Store<P>::real> v) const {
        if constexpr (P == MPMC_FP64) {   // two 64-bit halves: see stbuf
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v.re), rs, (int)vo, k * N * 16, 0);
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v.im), rs, (int)(vo + 8u), k * N * 16, 0);
        } else {
            f32x2 d;
            d.x = v.re;
            d.y = v.im;
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, d), rs, (int)vo, k * N * 8, 0);
        }
    }
};

template <int P, bool UNI, int MU, bool FWD, bool NR = false>
__device__ __forceinline__ void fetch(const WIn<P> &in, long s, int r, int N, HopData<P> &H) {
    using T = typename Store<P>::real;
    const int raw = in.nbr[s * 8 + (FWD ? 0 : 4) + MU];
    const long sn = (long)(raw & 0x7fffffff);
    H.bsign = raw < 0 ? T(-1) : T(1);
    if constexpr (NR && P != MPMC_FP16S) {
        const VecAcc<P> A(in.vrs, sn, N, (uint32_t)r);
#pragma unroll
        for (int k = 0; k < 12; ++k) H.psi[k] = A.ld(k);
    } else {
        const SiteAcc<P, UNI> A(in.b, in.bsc, sn, N, (uint32_t)r);
#pragma unroll
        for (int k = 0; k < 12; ++k) H.psi[k] = A.ld(k);
    }
    const auto *lk = in.links + ((FWD ? s : sn) * 4 + MU) * 9;
    if constexpr (UNI) {
        load_link_lanes<P>(lk, H.lw);
    } else if constexpr (NR) {
        load_link_rows<P>(lk, H.lw);
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const auto lv = lk[i];
            H.u[i] = mk((T)lv.x, (T)lv.y);
        }
    }
}

template <int P, bool UNI, int MU, bool FWD, bool NR = false>
__device__ __forceinline__ void apply(const HopData<P> &H, float g, cpx<typename Store<P>::real> acc[4][3]) {
    using T = typename Store<P>::real;
    using Pr = Proj<MU>;
    const T sg = FWD ? T(g) : T(-g);   // (1 - g gamma) forward, (1 + g gamma) backward
    cpx<T> h[2][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        h[0][c] = H.psi[0 * 3 + c] + sg * mulc<Pr::c0>(H.psi[Pr::j0 * 3 + c]);
        h[1][c] = H.psi[1 * 3 + c] + sg * mulc<Pr::c1>(H.psi[Pr::j1 * 3 + c]);
    }
    // uh = U h (forward) or U^H h (backward); FP32/FP16S as explicit FMA
    // chains (four per complex multiply-add)
    cpx<T> uh[2][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cpx<T> t0, t1;
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
            // forward: U[a][bb]; backward: conj(U[bb][a])
            const int li = FWD ? a * 3 + bb : bb * 3 + a;
            cpx<T> lv;
            if constexpr (UNI) lv = link_lane<P>(H.lw, li);
            else if constexpr (NR) lv = link_row<P>(H.lw, li);
            else lv = H.u[li];
            const T ur = lv.re, ui = FWD ? lv.im : -lv.im;
            if constexpr (P == MPMC_FP64) {   // FP64 keeps fewer live registers this way
                const cpx<T> u = mk(ur, ui);
                t0 = bb == 0 ? u * h[0][0] : t0 + u * h[0][bb];
                t1 = bb == 0 ? u * h[1][0] : t1 + u * h[1][bb];
                continue;
            }
            if (bb == 0) {
                t0 = mk(ur * h[0][0].re, ur * h[0][0].im);
                t1 = mk(ur * h[1][0].re, ur * h[1][0].im);
            } else {
                t0 = mk(fma(ur, h[0][bb].re, t0.re), fma(ur, h[0][bb].im, t0.im));
                t1 = mk(fma(ur, h[1][bb].re, t1.re), fma(ur, h[1][bb].im, t1.im));
            }
            t0 = mk(fma(-ui, h[0][bb].im, t0.re), fma(ui, h[0][bb].re, t0.im));
            t1 = mk(fma(-ui, h[1][bb].im, t1.re), fma(ui, h[1][bb].re, t1.im));
        }
        uh[0][a] = t0;
        uh[1][a] = t1;
    }
    // the boundary sign folds into the accumulation coefficients (FMA operands)
    const T c01 = H.bsign, c23 = H.bsign * sg;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[0][a] = acc[0][a] + c01 * uh[0][a];
        acc[1][a] = acc[1][a] + c01 * uh[1][a];
        acc[2][a] = acc[2][a] + c23 * mulc<Pr::d2>(uh[Pr::k2][a]);
        acc[3][a] = acc[3][a] + c23 * mulc<Pr::d3>(uh[Pr::k3][a]);
    }
}

// acc = sum over the 8 hops (the hopping term H b at (s, r)), hop i being
// direction i/2, forward for even i.  D HopData buffers rotate: the loads of
// hops i+1 .. i+D-1 are in flight while hop i computes.
#define MPMC_FENCE __builtin_amdgcn_sched_barrier(0)
template <int P, bool UNI, bool NR, int I>
__device__ __forceinline__ void fetch_hop(const WIn<P> &in, long s, int r, int N, HopData<P> &H) {
    fetch<P, UNI, I / 2, (I % 2) == 0, NR>(in, s, r, N, H);
}
template <int P, bool UNI, bool NR, int D, int I>
__device__ __forceinline__ void hop_step(const WIn<P> &in, long s, int r, int N, float g, HopData<P> (&H)[D],
                                         cpx<typename Store<P>::real> acc[4][3]) {
    if constexpr (I < 8) {
        apply<P, UNI, I / 2, (I % 2) == 0, NR>(H[I % D], g, acc);
        MPMC_FENCE;
        if constexpr (I + D < 8) {
            fetch_hop<P, UNI, NR, I + D>(in, s, r, N, H[I % D]);
            MPMC_FENCE;
        }
        hop_step<P, UNI, NR, D, I + 1>(in, s, r, N, g, H, acc);
    }
}
template <int P, bool UNI, bool NR, int D, int I>
__device__ __forceinline__ void hop_prologue(const WIn<P> &in, long s, int r, int N, HopData<P> (&H)[D]) {
    if constexpr (I < D) {
        fetch_hop<P, UNI, NR, I>(in, s, r, N, H[I]);
        MPMC_FENCE;
        hop_prologue<P, UNI, NR, D, I + 1>(in, s, r, N, H);
    }
}
template <int P, bool UNI, bool NR = false, int D = 2>
__device__ __forceinline__ void hopping(const WIn<P> &in, long s, int r, int N, float g,
                                        cpx<typename Store<P>::real> acc[4][3]) {
    using T = typename Store<P>::real;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[sp][c] = mk(T(0), T(0));
    HopData<P> H[D];
    hop_prologue<P, UNI, NR, D, 0>(in, s, r, N, H);
    hop_step<P, UNI, NR, D, 0>(in, s, r, N, g, H, acc);
}
#undef MPMC_FENCE

// Materialises the hopping term before any control flow of the epilogue.
// Without it the IR passes sink the hop arithmetic (and the loads feeding it)
// into the epilogue's per-component blocks, where each component then waits
// for its loads alone and the link values stay live in spilled SGPRs.
template <typename T>
__device__ __forceinline__ void pin_acc(cpx<T> acc[4][3]) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) asm volatile("" : "+v"(acc[sp][c].re), "+v"(acc[sp][c].im));
}

// (site, rhs) of this thread.  UNI (N % 64 == 0): each wavefront covers 64
// consecutive right-hand sides of one site, so the site follows from the
// wavefront's first thread with scalar arithmetic.
template <bool UNI, int ORDER = 0>
__device__ __forceinline__ bool locate_at(unsigned tile, long V, int N, long &s, int &r,
                                          const int *__restrict__ order) {
    const unsigned total = (unsigned)(V * N);
    if constexpr (UNI) {
        const unsigned w0 = tile * 256u + ((unsigned)__builtin_amdgcn_readfirstlane(threadIdx.x) & ~63u);
        if (w0 >= total) return false;
        if constexpr (ORDER == 0) {
            // site-major: a block holds 256/N sites x N right-hand sides
            const unsigned ss = w0 / (unsigned)N;
            s = (long)ss;
            r = (int)(w0 - ss * (unsigned)N + (threadIdx.x & 63u));
        } else {
            // chunk-major: all sites for right-hand sides [64c, 64c + 64) before
            // chunk c + 1; a block holds 4 sites x 64 right-hand sides, so the
            // working set of a sweep is 64 right-hand sides wide.  ORDER 2 takes
            // the sites of a chunk in the blocked order of the site table.
            const unsigned wv = w0 >> 6, Vu = (unsigned)V;
            const unsigned ch = wv / Vu, ss = wv - ch * Vu;
            if constexpr (ORDER == 2) s = (long)__builtin_amdgcn_readfirstlane(order[ss]);
            else s = (long)ss;
            r = (int)(ch * 64u + (threadIdx.x & 63u));
        }
    } else if constexpr (ORDER >= 3) {
        // narrow chunks: a wavefront covers S = 64 / W sites x W right-hand
        // sides of one W-wide chunk (ORDER 3: W = 16, ORDER 4: W = 32), sites
        // in the blocked order of the site table, all sites of a chunk before
        // the next chunk (needs N % 64 == 0 and V % S == 0)
        constexpr unsigned W = ORDER == 3 ? 16u : 32u, S = 64u / W;
        const unsigned w0 = tile * 256u + ((unsigned)__builtin_amdgcn_readfirstlane(threadIdx.x) & ~63u);
        if (w0 >= total) return false;
        const unsigned lane = threadIdx.x & 63u;
        const unsigned wv = w0 >> 6, wpc = (unsigned)V / S;
        const unsigned ch = wv / wpc, q = (wv - ch * wpc) * S + lane / W;
        s = (long)order[q];
        r = (int)(ch * W + lane % W);
    } else {
        const unsigned t = tile * 256u + threadIdx.x;
        if (t >= total) return false;
        const unsigned ss = t / (unsigned)N;
        s = (long)ss;
        r = (int)(t - ss * (unsigned)N);
    }
    return true;
}
template <bool UNI, int ORDER = 0>
__device__ __forceinline__ bool locate(long V, int N, long &s, int &r, const int *__restrict__ order = nullptr) {
    return locate_at<UNI, ORDER>(xcd_tile(blockIdx.x, gridDim.x), V, N, s, r, order);
}

struct WOut {
    void *out;
    float *osc;
    const void *a;          // additive term (nullptr: none; == b: reuse the operand)
    const float *asc;
    void *y;                // y += gamma * out (nullptr: none)
    double kappa;
    double2 alpha, beta, gamma;
    float g;
    int theta;
    int a_is_b;
    int out_fp32;           // FP16S kernels only: write out as FP32 (plain out = M b)
};

// Occupancy targets (minimum wavefronts per SIMD the register allocation must
// allow).  The uniform kernels come in two targets chosen by the autotuner:
// HI = 1 asks for more wavefronts (FP32/FP16S: 3, <= 168 VGPRs; FP64: 2),
// HI = 0 for more registers (FP32/FP16S: 2; FP64: no target).
template <int P, bool UNI, int HI = 1, int ORDER = 0>
struct Occ {
    static constexpr int wpe = (!UNI && ORDER < 3) ? 1 : (P == MPMC_FP64 ? (HI ? 2 : 1) : (HI ? 3 : 2));
};

// Kernel variants of the autotuner: bit 0 selects the occupancy target
// (Occ::HI), bits 1-3 the traversal order of locate() (0 site-major, 1
// chunk-major, 2 chunk-major over the blocked site order, 3 and 4 the same with
// 16- and 32-wide chunks, four and two sites per wavefront and per-lane
// links).  Orders 3 and 4 need V % 16 == 0; elsewhere they fall back to 2.
constexpr int WILSON_VARIANTS = 13;
constexpr int WILSON_COLUMN = 10;    // FP32 column-streaming kernel (k_wilson_col), 2x2x2 tiles
constexpr int WILSON_COLUMN1 = 11;   // the same with 2x2x1 tiles (two workgroups per compute unit)
constexpr int WILSON_COLUMNP = 12;   // 2x2x4 tiles, 32-wide chunks, two sites per wavefront (k_wilson_colp)

// Everything one thread does for (site s, rhs r) once located.
template <int P, bool UNI, int ORDER>
__device__ __forceinline__ void wilson_site(const WIn<P> in, const WOut o, long s, int r, int N) {
    using T = typename Store<P>::real;
    constexpr bool NR = ORDER >= 3;   // narrow chunks: row-distributed links, whole-operand buffer
    cpx<T> acc[4][3];
    hopping<P, UNI, NR>(in, s, r, N, o.g, acc);
    pin_acc(acc);
    // Epilogue without per-component control flow: all operand loads are
    // issued together, the optional terms enter through coefficients.
    const T kap = (T)o.kappa;
    const bool has_a = o.a_is_b || o.a;
    const cpx<T> al = has_a ? mk((T)o.alpha.x, (T)o.alpha.y) : mk(T(0), T(0));
    const cpx<T> be = mk((T)o.beta.x, (T)o.beta.y);
    const cpx<T> beg5 = o.theta ? mk(-be.re, -be.im) : be;   // Theta = gamma5 flips spins 2, 3
    const SiteAcc<P, UNI> B(in.b, in.bsc, s, N, (uint32_t)r);
    cpx<T> res[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) res[k] = B.ld(k);
    if (o.a && !o.a_is_b) {
        const SiteAcc<P, UNI> A(o.a, o.asc, s, N, (uint32_t)r);
        cpx<T> av[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) av[k] = A.ld(k);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const cpx<T> mb = res[k] - kap * acc[k / 3][k % 3];
            res[k] = (k >= 6 ? beg5 : be) * mb + al * av[k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const cpx<T> mb = res[k] - kap * acc[k / 3][k % 3];
            res[k] = (k >= 6 ? beg5 : be) * mb + al * res[k];
        }
    }
    if constexpr (P == MPMC_FP16S) {
        if (o.out_fp32) {
            const SiteAcc<MPMC_FP32, UNI> O(o.out, nullptr, s, N, (uint32_t)r);
#pragma unroll
            for (int k = 0; k < 12; ++k) O.st(k, res[k]);
            return;
        }
        float mx = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) mx = fmaxf(mx, fmaxf(fabsf(res[k].re), fabsf(res[k].im)));
        const float inv = mx > 0.f ? 1.0f / mx : 0.f;
        __half2 *d = reinterpret_cast<__half2 *>(o.out);
#pragma unroll
        for (int k = 0; k < 12; ++k) d[(s * 12 + k) * N + r] = __floats2half2_rn(res[k].re * inv, res[k].im * inv);
        o.osc[s * N + r] = mx;
    } else {
        const SiteAcc<P, UNI> O(o.out, nullptr, s, N, (uint32_t)r);
#pragma unroll
        for (int k = 0; k < 12; ++k) O.st(k, res[k]);
        if (o.y) {
            const cpx<T> ga = mk((T)o.gamma.x, (T)o.gamma.y);
            const SiteAcc<P, UNI> Y(o.y, nullptr, s, N, (uint32_t)r);
            cpx<T> yv[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) yv[k] = Y.ld(k);
#pragma unroll
            for (int k = 0; k < 12; ++k) Y.st(k, yv[k] + ga * res[k]);
        }
    }
}

template <int P, bool UNI, int HI = 1, int ORDER = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Occ<P, UNI, HI, ORDER>::wpe))) void k_wilson(const void *__restrict__ b, const float *__restrict__ bsc,
                                                const int *__restrict__ nbr,
                                                const typename LinkT<P>::type *__restrict__ links, WOut o, long V,
                                                int N, const int *__restrict__ order) {
    WIn<P> in{b, bsc, nbr, links};
    if constexpr (ORDER >= 3 && P != MPMC_FP16S) in.vrs = vec_rsrc<P>(b, V, N);
    long s;
    int r;
    if (!locate<UNI, ORDER>(V, N, s, r, order)) return;
    wilson_site<P, UNI, ORDER>(in, o, s, r, N);
}

// ------------------------------------------------ batched lattices --
// Several lattices (contexts) in one launch: the tile range of the grid is the
// concatenation of the lattices' tile ranges (blocked 64-wide traversal, the
// same per-element arithmetic as k_wilson<P, true, HI, 2>); a workgroup finds
// its lattice by a scalar scan of the first-tile offsets.
constexpr int WILSON_BATCH_MAX = 8;
template <int P>
struct LatticeArgs {
    const void *b;
    void *out;
    const int *nbr;
    const typename LinkT<P>::type *links;
    const int *order;
    long V;
    double kappa;
    unsigned tile0;   // first tile of this lattice in the grid
};
template <int P>
struct BatchArgs {
    LatticeArgs<P> l[WILSON_BATCH_MAX];
    int count;
};

template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Occ<P, true, 1, 2>::wpe))) void k_wilson_batch(
    BatchArgs<P> a, int N, float g, int theta) {
    const unsigned tile = xcd_tile(blockIdx.x, gridDim.x);
    int q = 0;
    for (int i = 1; i < a.count; ++i)
        if (tile >= a.l[i].tile0) q = i;
    const LatticeArgs<P> &L = a.l[q];
    WIn<P> in{L.b, nullptr, L.nbr, L.links};
    WOut o{};
    o.out = L.out;
    o.kappa = L.kappa;
    o.alpha = make_double2(0, 0);
    o.beta = make_double2(1, 0);
    o.gamma = make_double2(0, 0);
    o.g = g;
    o.theta = theta;
    long s;
    int r;
    if (!locate_at<true, 2>(tile - L.tile0, L.V, N, s, r, L.order)) return;
    wilson_site<P, true, 2>(in, o, s, r, N);
}

// ---------------------------------------------------- single vectors --
// nrhs == 1 (GMRES-polynomial and deflation Arnoldi cycles): eight lanes per
// site, one hop each, so a single-vector matvec occupies 8x more wavefronts;
// the eight 12-component contributions are summed with DPP (quad xor 1 and 2,
// then row_shr 4, which leaves the site's total in lane 4 of its group), and
// lane 4 loads the epilogue operands before the hop, so they arrive while
// the hop computes.  Workgroups are one wavefront: an 8^4 vector is 32,768
// threads, which 256-thread workgroups would put on half the compute units.
template <typename T>
__device__ __forceinline__ cpx<T> mulc_rt(cpx<T> z, int code) {
    T a = z.re, b = z.im;
    if (code & 1) {
        const T t = a;
        a = -b;
        b = t;
    }
    if (code & 2) {
        a = -a;
        b = -b;
    }
    return mk(a, b);
}

template <int CTRL>
__device__ __forceinline__ float dpp_t(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_t(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
// Sum over the 8-lane group: quad_perm [1,0,3,2] and [2,3,0,1] (every lane of
// a quad holds the quad's sum), then row_shr 4: lanes 4..7 of the group (and
// 12..15 of the next, within the same 16-lane row) add the first quad.
template <typename T>
__device__ __forceinline__ T group8_sum1(T v) {
    v += dpp_t<0xB1>(v);
    v += dpp_t<0x4E>(v);
    return v + dpp_t<0x114>(v);
}
template <typename T>
__device__ __forceinline__ cpx<T> group8_sum(cpx<T> v) { return mk(group8_sum1(v.re), group8_sum1(v.im)); }

// yinit_on: y = yinit * b + gamma * out instead of y += gamma * out (the
// first step of a polynomial, whose accumulator starts at b / theta_1; needs
// a == b), y is then not read.
template <int P>
__global__ __launch_bounds__(256) void k_wilson1(const void *__restrict__ b, const int *__restrict__ nbr,
                                                 const typename LinkT<P>::type *__restrict__ links, WOut o, long V,
                                                 double2 yinit, int yinit_on) {
    using T = typename Store<P>::real;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long s = t >> 3;
    const int h = (int)(t & 7);
    const bool live = s < V;
    const bool epi = live && h == 4;   // the lane that finishes the site
    const typename Elem<P>::type *sp = reinterpret_cast<const typename Elem<P>::type *>(b) + s * 12;
    const typename Elem<P>::type *ap = reinterpret_cast<const typename Elem<P>::type *>(o.a_is_b ? b : o.a) + s * 12;
    typename Elem<P>::type *yp = reinterpret_cast<typename Elem<P>::type *>(o.y) + s * 12;
    typename Elem<P>::type *op = reinterpret_cast<typename Elem<P>::type *>(o.out) + s * 12;
    const bool has_a = o.a_is_b || o.a;
    cpx<T> bt[12], av[12], yv[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        bt[k] = epi ? mk((T)sp[k].x, (T)sp[k].y) : mk(T(0), T(0));
        av[k] = epi && has_a ? mk((T)ap[k].x, (T)ap[k].y) : mk(T(0), T(0));
        yv[k] = epi && o.y && !yinit_on ? mk((T)yp[k].x, (T)yp[k].y) : mk(T(0), T(0));
    }
    cpx<T> c[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) c[k] = mk(T(0), T(0));
    if (live) {
        const int mu = h & 3;
        const bool fwd = h < 4;
        // (1 - gamma_mu) codes: j0, c0, j1, c1, k2, d2, k3, d3 (see Proj)
        const int j0 = mu < 2 ? 3 : 2, c0 = mu == 0 ? 3 : (mu == 1 ? 0 : (mu == 2 ? 3 : 2));
        const int j1 = mu < 2 ? 2 : 3, c1 = mu == 0 ? 3 : (mu == 1 ? 2 : (mu == 2 ? 1 : 2));
        const int k2 = mu < 2 ? 1 : 0, d2 = mu == 0 ? 1 : (mu == 1 ? 2 : (mu == 2 ? 1 : 2));
        const int k3 = mu < 2 ? 0 : 1, d3 = mu == 0 ? 1 : (mu == 1 ? 0 : (mu == 2 ? 3 : 2));
        const T sg = fwd ? T(o.g) : T(-o.g);
        const int raw = nbr[s * 8 + h];
        const long sn = (long)(raw & 0x7fffffff);
        const T bsign = raw < 0 ? T(-1) : T(1);
        const typename Elem<P>::type *bp = reinterpret_cast<const typename Elem<P>::type *>(b) + sn * 12;
        cpx<T> psi[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) psi[k] = mk((T)bp[k].x, (T)bp[k].y);
        cpx<T> hh[2][3];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            const cpx<T> pj0 = j0 == 3 ? psi[9 + cc] : psi[6 + cc];
            const cpx<T> pj1 = j1 == 3 ? psi[9 + cc] : psi[6 + cc];
            hh[0][cc] = psi[cc] + sg * mulc_rt(pj0, c0);
            hh[1][cc] = psi[3 + cc] + sg * mulc_rt(pj1, c1);
        }
        const auto *lk = links + ((fwd ? s : sn) * 4 + mu) * 9;
        cpx<T> uh[2][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cpx<T> t0 = mk(T(0), T(0)), t1 = mk(T(0), T(0));
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                const auto lv = fwd ? lk[a * 3 + bb] : lk[bb * 3 + a];
                const cpx<T> u = mk((T)lv.x, fwd ? (T)lv.y : (T)-lv.y);
                t0 = t0 + u * hh[0][bb];
                t1 = t1 + u * hh[1][bb];
            }
            uh[0][a] = bsign * t0;
            uh[1][a] = bsign * t1;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            c[a] = uh[0][a];
            c[3 + a] = uh[1][a];
            c[6 + a] = sg * mulc_rt(k2 ? uh[1][a] : uh[0][a], d2);
            c[9 + a] = sg * mulc_rt(k3 ? uh[1][a] : uh[0][a], d3);
        }
    }
    // sum the eight hops of a site (lanes 8q .. 8q+7) into lane 8q + 4
#pragma unroll
    for (int k = 0; k < 12; ++k) c[k] = group8_sum(c[k]);
    if (!epi) return;
    const T kap = (T)o.kappa;
    const cpx<T> al = mk((T)o.alpha.x, (T)o.alpha.y);
    const cpx<T> be = mk((T)o.beta.x, (T)o.beta.y);
    const cpx<T> ga = mk((T)o.gamma.x, (T)o.gamma.y);
    const cpx<T> yi = mk((T)yinit.x, (T)yinit.y);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        cpx<T> mb = bt[k] - kap * c[k];
        if (o.theta && k >= 6) mb = mk(-mb.re, -mb.im);
        cpx<T> v = be * mb;
        if (has_a) v = v + al * av[k];
        op[k].x = v.re;
        op[k].y = v.im;
        if (o.y) {
            const cpx<T> yn = (yinit_on ? yi * av[k] : yv[k]) + ga * v;
            yp[k].x = yn.re;
            yp[k].y = yn.im;
        }
    }
}

// ---------------------------------------- single vectors, large lattices --
// One site per lane, lexicographic sites (consecutive lanes, consecutive x).
// Against the generic kernel at one right-hand side: the neighbour index and
// the antiperiodic sign follow from the site's coordinates (no table load in
// each hop's dependency chain), the neighbour's 12 components arrive as
// 16-byte loads, and an FP32 link as four 16-byte loads and one 8-byte load
// (link mu of a site starts 72 mu bytes into the site's 288, so its 16-byte
// alignment is known from mu at compile time).  The hop arithmetic is the
// generic kernel's (apply), so M b is the same bit for bit; the accumulator
// start y = yinit b of a polynomial's first step is fused into the epilogue.
// Site indices are 32-bit here (the library keeps V below 2^31): the
// neighbour offset is a select between two constants, so no branch splits the
// hops (a branch would let the compiler sink each hop's arithmetic below the
// next hops' loads and hold all eight neighbours in registers at once).
struct SvGeom {
    int L[4];
    int st[4];     // site strides 1, Lx, Lx Ly, Lx Ly Lz
    int wrap[4];   // (L_mu - 1) st_mu
    int anti;      // antiperiodic in t
};

template <int P, int MU, bool FWD>
__device__ __forceinline__ void fetch_sv(const void *__restrict__ b, const typename LinkT<P>::type *__restrict__ links,
                                         const SvGeom &G, int s, const int c[4], HopData<P> &H) {
    using T = typename Store<P>::real;
    const bool edge = FWD ? c[MU] == G.L[MU] - 1 : c[MU] == 0;
    const int off = FWD ? (edge ? -G.wrap[MU] : G.st[MU]) : (edge ? G.wrap[MU] : -G.st[MU]);
    const int sn = s + off;
    H.bsign = (MU == 3 && G.anti && edge) ? T(-1) : T(1);
    if constexpr (P == MPMC_FP32) {
        const float4 *p4 = reinterpret_cast<const float4 *>(b) + (long)sn * 6;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const float4 v = p4[i];
            H.psi[2 * i] = mk(v.x, v.y);
            H.psi[2 * i + 1] = mk(v.z, v.w);
        }
        const float2 *lk = links + ((long)(FWD ? s : sn) * 4 + MU) * 9;
        if constexpr ((MU & 1) == 0) {   // 16-byte aligned: elements 0-7 as pairs, then 8
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float4 v = reinterpret_cast<const float4 *>(lk)[i];
                H.u[2 * i] = mk(v.x, v.y);
                H.u[2 * i + 1] = mk(v.z, v.w);
            }
            const float2 v8 = lk[8];
            H.u[8] = mk(v8.x, v8.y);
        } else {                          // 8 bytes past alignment: element 0, then 1-8 as pairs
            const float2 v0 = lk[0];
            H.u[0] = mk(v0.x, v0.y);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float4 v = reinterpret_cast<const float4 *>(lk + 1)[i];
                H.u[2 * i + 1] = mk(v.x, v.y);
                H.u[2 * i + 2] = mk(v.z, v.w);
            }
        }
    } else {
        const double2 *p = reinterpret_cast<const double2 *>(b) + (long)sn * 12;
#pragma unroll
        for (int k = 0; k < 12; ++k) H.psi[k] = mk(p[k].x, p[k].y);
        const double2 *lk = links + ((long)(FWD ? s : sn) * 4 + MU) * 9;
#pragma unroll
        for (int i = 0; i < 9; ++i) H.u[i] = mk(lk[i].x, lk[i].y);
    }
}

#define MPMC_FENCE __builtin_amdgcn_sched_barrier(0)
template <int P, int D, int I>
__device__ __forceinline__ void sv_step(const void *__restrict__ b, const typename LinkT<P>::type *__restrict__ links,
                                        const SvGeom &G, int s, const int c[4], float g, HopData<P> (&H)[D],
                                        cpx<typename Store<P>::real> acc[4][3]) {
    if constexpr (I < 8) {
        apply<P, false, I / 2, (I % 2) == 0, false>(H[I % D], g, acc);
        MPMC_FENCE;
        if constexpr (I + D < 8) {
            fetch_sv<P, (I + D) / 2, ((I + D) % 2) == 0>(b, links, G, s, c, H[I % D]);
            MPMC_FENCE;
        }
        sv_step<P, D, I + 1>(b, links, G, s, c, g, H, acc);
    }
}
template <int P, int D, int I>
__device__ __forceinline__ void sv_prologue(const void *__restrict__ b,
                                            const typename LinkT<P>::type *__restrict__ links, const SvGeom &G,
                                            int s, const int c[4], HopData<P> (&H)[D]) {
    if constexpr (I < D) {
        fetch_sv<P, I / 2, (I % 2) == 0>(b, links, G, s, c, H[I]);
        MPMC_FENCE;
        sv_prologue<P, D, I + 1>(b, links, G, s, c, H);
    }
}
#undef MPMC_FENCE

template <int P>
__device__ __forceinline__ void sv_load12(const void *p, int s, cpx<typename Store<P>::real> v[12]) {
    if constexpr (P == MPMC_FP32) {
        const float4 *p4 = reinterpret_cast<const float4 *>(p) + (long)s * 6;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const float4 w = p4[i];
            v[2 * i] = mk(w.x, w.y);
            v[2 * i + 1] = mk(w.z, w.w);
        }
    } else {
        const double2 *p2 = reinterpret_cast<const double2 *>(p) + (long)s * 12;
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = mk(p2[k].x, p2[k].y);
    }
}
template <int P>
__device__ __forceinline__ void sv_store12(void *p, int s, const cpx<typename Store<P>::real> v[12]) {
    if constexpr (P == MPMC_FP32) {
        float4 *p4 = reinterpret_cast<float4 *>(p) + (long)s * 6;
#pragma unroll
        for (int i = 0; i < 6; ++i) p4[i] = make_float4(v[2 * i].re, v[2 * i].im, v[2 * i + 1].re, v[2 * i + 1].im);
    } else {
        double2 *p2 = reinterpret_cast<double2 *>(p) + (long)s * 12;
#pragma unroll
        for (int k = 0; k < 12; ++k) p2[k] = make_double2(v[k].re, v[k].im);
    }
}

template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == MPMC_FP64 ? 2 : 3))) void k_wilson_sv(const void *__restrict__ b,
                                                   const typename LinkT<P>::type *__restrict__ links, WOut o,
                                                   SvGeom G, long V, double2 yinit, int yinit_on) {
    using T = typename Store<P>::real;
    const unsigned su = xcd_tile(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
    if (su >= (unsigned)V) return;
    const int s = (int)su;
    int c[4];
    {
        unsigned q = su;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const unsigned qn = q / (unsigned)G.L[mu];
            c[mu] = (int)(q - qn * (unsigned)G.L[mu]);
            q = qn;
        }
    }
    cpx<T> acc[4][3];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) acc[sp][cc] = mk(T(0), T(0));
    {
        HopData<P> H[2];
        sv_prologue<P, 2, 0>(b, links, G, s, c, H);
        sv_step<P, 2, 0>(b, links, G, s, c, o.g, H, acc);
    }
    pin_acc(acc);
    // epilogue: the generic kernel's arithmetic (wilson_site)
    const T kap = (T)o.kappa;
    const bool has_a = o.a_is_b || o.a;
    const cpx<T> al = has_a ? mk((T)o.alpha.x, (T)o.alpha.y) : mk(T(0), T(0));
    const cpx<T> be = mk((T)o.beta.x, (T)o.beta.y);
    const cpx<T> beg5 = o.theta ? mk(-be.re, -be.im) : be;
    cpx<T> bv[12], res[12];
    sv_load12<P>(b, s, bv);
    if (o.a && !o.a_is_b) {
        cpx<T> av[12];
        sv_load12<P>(o.a, s, av);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const cpx<T> mb = bv[k] - kap * acc[k / 3][k % 3];
            res[k] = (k >= 6 ? beg5 : be) * mb + al * av[k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const cpx<T> mb = bv[k] - kap * acc[k / 3][k % 3];
            res[k] = (k >= 6 ? beg5 : be) * mb + al * bv[k];
        }
    }
    sv_store12<P>(o.out, s, res);
    if (o.y) {
        const cpx<T> ga = mk((T)o.gamma.x, (T)o.gamma.y);
        cpx<T> yv[12];
        if (yinit_on) {   // y = yinit b + gamma out (b is also the additive operand here)
            const cpx<T> yi = mk((T)yinit.x, (T)yinit.y);
#pragma unroll
            for (int k = 0; k < 12; ++k) yv[k] = yi * bv[k] + ga * res[k];
        } else {
            sv_load12<P>(o.y, s, yv);
#pragma unroll
            for (int k = 0; k < 12; ++k) yv[k] = yv[k] + ga * res[k];
        }
        sv_store12<P>(o.y, s, yv);
    }
}

// ------------------------------------------------- fused level step --
// w' = w - c M w for a batch whose rhs r is noise vector eta_r (2-bit codes in
// codes[s*N + r]); partial[blk][rl] += cnext * sum_k conj(eta_k) (Theta w')_k
// summed over the block's sites.  Requires N % 64 == 0 (uniform wavefronts).
// A block of 256 threads covers spb = max(1, 256/N) sites and rpb = min(N, 256)
// right-hand sides starting at rhs (blk*256) % N.
//
// MULTI (blocked 64-wide chunks only): several recurrences side by side, each
// a run of 64-wide chunks of the right-hand-side axis (stride N); the launch
// covers the first nact right-hand sides, and chunk q takes its (c, cnext)
// from coef[2q], coef[2q + 1].
//
// CMB: the step ends a double polynomial's inner product form and combines,
// w' = alpha a + beta (w - c M w) with a second operand a (the outer
// recurrence's current vector); the quadratic form then accumulates on w'.
template <int P, int ORDER, bool MULTI = false, bool CMB = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == MPMC_FP64 ? 1 : 2))) void k_wilson_dot(const void *__restrict__ b, const int *__restrict__ nbr,
                                                    const typename LinkT<P>::type *__restrict__ links,
                                                    void *__restrict__ out, const uint32_t *__restrict__ codes,
                                                    double2 c, double2 cnext, double kappa, int theta,
                                                    double2 *__restrict__ partial, long V, int N, int first_step,
                                                    const int *__restrict__ order, int nact = 0,
                                                    const double2 *__restrict__ coef = nullptr,
                                                    const void *__restrict__ a = nullptr,
                                                    double2 alpha = double2{0, 0}, double2 beta = double2{1, 0}) {
    static_assert(!MULTI || ORDER == 2, "several recurrences need the blocked 64-wide traversal");
    static_assert(!(MULTI && CMB), "the combining step runs one recurrence");
    using T = typename Store<P>::real;
    constexpr bool U = ORDER <= 2;   // one site per wavefront (else 2 or 4, row-distributed links)
    WIn<P> in{b, nullptr, nbr, links};
    if constexpr (!U) in.vrs = vec_rsrc<P>(b, V, N);
    __shared__ double2 red[256];
    long s;
    int r;
    const bool live = locate<U, ORDER>(V, MULTI ? nact : N, s, r, order);
    if constexpr (MULTI) {
        const unsigned q = live ? (unsigned)r >> 6 : 0u;   // the wavefront's chunk
        c = coef[2 * q];
        cnext = coef[2 * q + 1];
    }
    cpx<double> dot = mk(0.0, 0.0);
    if (live) {
        cpx<T> acc[4][3];
        hopping<P, U, !U>(in, s, r, N, 1.0f, acc);
        pin_acc(acc);
        const uint32_t code = codes[s * N + r];
        const T kap = (T)kappa;
        const cpx<T> cc = mk((T)c.x, (T)c.y);
        const SiteAcc<P, U> W(in.b, nullptr, s, N, (uint32_t)r), O(out, nullptr, s, N, (uint32_t)r);
        cpx<T> wv[12], av[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) wv[k] = W.ld(k);
        if constexpr (CMB) {
            const SiteAcc<P, U> A(a, nullptr, s, N, (uint32_t)r);
#pragma unroll
            for (int k = 0; k < 12; ++k) av[k] = A.ld(k);
        }
        const cpx<T> al = mk((T)alpha.x, (T)alpha.y), be = mk((T)beta.x, (T)beta.y);
        // conj(eta_k) wn with eta_k = i^sym, by selects (no per-lane branches):
        // odd sym swaps (re, im) -> (im, -re), sym >= 2 negates; Theta = gamma5
        // negates spins 2 and 3.
        // The site's 12 terms are summed in the storage precision (exact
        // signs, 12 additions: the rounding of the stored w' is of the same
        // size), every sum over sites, steps and blocks in FP64.
        const T tsg = theta ? T(-1) : T(1);
        T sr = T(0), si = T(0);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const cpx<T> mw = wv[k] - kap * acc[k / 3][k % 3];
            cpx<T> wn = wv[k] - cc * mw;
            if constexpr (CMB) wn = al * av[k] + be * wn;
            O.st(k, wn);
            const uint32_t sym = (code >> (2 * k)) & 3u;
            const T sg = (sym & 2u) ? T(-1) : T(1);
            const T g = k >= 6 ? sg * tsg : sg;
            sr += g * ((sym & 1u) ? wn.im : wn.re);
            si += g * ((sym & 1u) ? -wn.re : wn.im);
        }
        dot = mk((double)sr, (double)si);
    }
    red[threadIdx.x] = make_double2(dot.re, dot.im);
    __syncthreads();
    if constexpr (ORDER >= 3) {
        // narrow chunks: a tile holds 256 / W sites x the W right-hand sides
        // [W c, W c + W) of chunk c (V % 16 == 0); one partial per (tile, rhs),
        // the sites summed in a fixed order
        constexpr int W = ORDER == 3 ? 16 : 32;
        if ((int)threadIdx.x < W) {
            cpx<double> sum = mk(0.0, 0.0);
#pragma unroll
            for (int g = 0; g < 256 / W; ++g) {
                const double2 v = red[threadIdx.x + g * W];
                sum = mk(sum.re + v.x, sum.im + v.y);
            }
            const unsigned tile = xcd_tile(blockIdx.x, gridDim.x);
            const cpx<double> term = mk(cnext.x, cnext.y) * sum;
            double2 *pp = partial + (long)tile * W + threadIdx.x;
            if (first_step) {
                *pp = make_double2(term.re, term.im);
            } else {
                double2 old = *pp;
                *pp = make_double2(old.x + term.re, old.y + term.im);
            }
        }
        return;
    }
    if constexpr (ORDER != 0) {
        // chunk-major tiles: the four wavefronts share the right-hand sides
        // [64c, 64c + 64) of chunk c = 4 tile / V (V % 4 == 0); one partial per
        // (tile, lane), the four sites summed in a fixed order
        if (threadIdx.x < 64) {
            const double2 a = red[threadIdx.x], b2 = red[threadIdx.x + 64], c2 = red[threadIdx.x + 128],
                          d2 = red[threadIdx.x + 192];
            const cpx<double> sum = mk(((a.x + b2.x) + c2.x) + d2.x, ((a.y + b2.y) + c2.y) + d2.y);
            const unsigned tile = xcd_tile(blockIdx.x, gridDim.x);
            const cpx<double> term = mk(cnext.x, cnext.y) * sum;
            double2 *pp = partial + (long)tile * 64 + threadIdx.x;
            if (first_step) {
                *pp = make_double2(term.re, term.im);
            } else {
                double2 old = *pp;
                *pp = make_double2(old.x + term.re, old.y + term.im);
            }
        }
        return;
    }
    const int rpb = N < 256 ? N : 256;
    const int spb = 256 / rpb;
    if ((int)threadIdx.x < rpb) {
        double2 sum = red[threadIdx.x];
        for (int q = 1; q < spb; ++q) {
            sum.x += red[threadIdx.x + q * rpb].x;
            sum.y += red[threadIdx.x + q * rpb].y;
        }
        const unsigned tile = xcd_tile(blockIdx.x, gridDim.x);
        const cpx<double> term = mk(cnext.x, cnext.y) * mk(sum.x, sum.y);
        double2 *pp = partial + (long)tile * rpb + threadIdx.x;
        if (first_step) {
            *pp = make_double2(term.re, term.im);
        } else {
            double2 old = *pp;
            *pp = make_double2(old.x + term.re, old.y + term.im);
        }
    }
}

// out[r] = sum over blocks covering rhs r of partial (fixed order)
__global__ void k_dot_finish(const double2 *__restrict__ partial, int nblocks, int N, double2 *__restrict__ out,
                             int accumulate, double sign) {
    __shared__ double2 red[256];
    const int r = blockIdx.x;
    const int rpb = N < 256 ? N : 256;
    const int per = N / rpb;              // blocks cycle through N/rpb rhs ranges
    const int rr = r % rpb, range = r / rpb;
    double2 a = make_double2(0, 0);
    for (int b = range + per * threadIdx.x; b < nblocks; b += per * blockDim.x) {
        const double2 v = partial[(long)b * rpb + rr];
        a.x += v.x;
        a.y += v.y;
    }
    red[threadIdx.x] = a;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[threadIdx.x].x += red[threadIdx.x + h].x;
            red[threadIdx.x].y += red[threadIdx.x + h].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (accumulate) {
            out[r].x += sign * red[0].x;
            out[r].y += sign * red[0].y;
        } else {
            out[r] = make_double2(sign * red[0].x, sign * red[0].y);
        }
    }
}

// out[r] = sum of partial[t*width + r%width] over the tiles t of chunk
// r/width (chunk-major fused steps), in a fixed order
__global__ void k_dot_finish_chunk(const double2 *__restrict__ partial, long tiles_per_chunk, int width,
                                   double2 *__restrict__ out, int accumulate, double sign) {
    __shared__ double2 red[256];
    const int r = blockIdx.x;
    const long t0 = (long)(r / width) * tiles_per_chunk;
    const int lane = r % width;
    double2 a = make_double2(0, 0);
    for (long t = threadIdx.x; t < tiles_per_chunk; t += blockDim.x) {
        const double2 v = partial[(t0 + t) * width + lane];
        a.x += v.x;
        a.y += v.y;
    }
    red[threadIdx.x] = a;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[threadIdx.x].x += red[threadIdx.x + h].x;
            red[threadIdx.x].y += red[threadIdx.x + h].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (accumulate) {
            out[r].x += sign * red[0].x;
            out[r].y += sign * red[0].y;
        } else {
            out[r] = make_double2(sign * red[0].x, sign * red[0].y);
        }
    }
}

// codes[s*N + r] = Z(4) symbols of noise vector first + r at site s
// (noise vectors first .. first+N-1 in columns off .. off+N-1 of rows of ld)
__global__ void k_noise_codes(uint64_t seed, uint32_t stream, uint64_t first, uint32_t *__restrict__ codes, long V,
                              int N, int ld, int off) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= V * N) return;
    const long s = t / N;
    const int r = (int)(t - s * N);
    codes[s * ld + off + r] = z4_site_symbols(seed, stream, (uint32_t)(first + r), s);
}

// -------------------------------------------------- column streaming --
// FP32 kernels in which a workgroup owns a 2 x 2 x 2 tile of (x, y, z)
// columns and 64 right-hand sides (one wavefront per column) and walks the
// columns along t.  Every wavefront keeps its own site and the next one in
// registers (the t+1 neighbour of step t is the own site of step t+1, loaded
// one step ahead) and publishes its site in LDS each step; the t-1 neighbour
// (the own column's previous site) and the three in-tile x, y, z neighbours
// come from LDS, only the three out-of-tile neighbours from global memory.
// A site's spinor is thus fetched by 4 wavefronts instead of 9 -- the Wilson
// kernels are bound by L1-miss requests to the L2 (each site-wavefront's
// loads miss the 32 KB L1), so this cuts the bound itself.  LDS holds three
// slices (t-1, t, and the one being written next) so that one barrier per
// step orders all writes and reads.  Requires even Lx, Ly, Lz, Lt >= 4 and
// nrhs % 64 == 0.
template <int TZ>
constexpr int col_waves() { return 4 * TZ; }

struct ColArgs {
    int L[4];
    int ntx, nty, ntz;   // tiles per direction
    int bx, by, bz;      // tiles per block of the traversal (each divides its extent)
    long ntiles;         // tiles per 64-wide chunk
    long nblk;           // blocks over all chunks of the launch (col_grid)
    int tap;             // antiperiodic time direction
    int rev;             // blocks in reverse order (see k_wilson_col)
};

template <int TZ>
struct ColLds {
    float2 v[3][col_waves<TZ>()][12][64];
};

// hop MU (forward or backward) from a spinor held by the lane
template <int P, int MU, bool FWD>
__device__ __forceinline__ void col_hop(const cpx<float> (&psi)[12], uint32_t lw, float bsign, float g,
                                        cpx<float> acc[4][3]) {
    HopData<P> H;
#pragma unroll
    for (int k = 0; k < 12; ++k) H.psi[k] = psi[k];
    H.lw[0] = lw;
    H.bsign = bsign;
    apply<P, true, MU, FWD>(H, g, acc);
    __builtin_amdgcn_sched_barrier(0);   // hops one after another: short live ranges
}

template <int TZ>
__device__ __forceinline__ void col_lds_read(const ColLds<TZ> &L, int buf, int w, unsigned lane,
                                             cpx<float> (&psi)[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const float2 v = L.v[buf][w][k][lane];
        psi[k] = mk(v.x, v.y);
    }
}

__device__ __forceinline__ void col_load(const void *b, long site, int N, uint32_t r, cpx<float> (&psi)[12]) {
    const SiteAcc<MPMC_FP32, true> A(b, nullptr, site, N, r);
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k] = A.ld(k);
}

__device__ __forceinline__ long col_site(const ColArgs &c, int x, int y, int z, int t) {
    return x + (long)c.L[0] * (y + (long)c.L[1] * (z + (long)c.L[2] * t));
}

// The x, y or z hops of one site: the in-tile neighbour (the wavefront's
// partner across the tile, from LDS) and the out-of-tile one (og, global
// memory; forward if the column sits at the tile's upper edge, else
// backward).  lf: U_mu(s), lb: U_mu(s - mu), both lane-distributed.
template <int MU, int TZ>
__device__ __forceinline__ void col_dir(const ColLds<TZ> &L, int curb, int w, unsigned lane, int upper,
                                        const cpx<float> (&og)[12], uint32_t lf, uint32_t lb, float g,
                                        cpx<float> acc[4][3]) {
    cpx<float> nb[12];
    col_lds_read(L, curb, w ^ (1 << MU), lane, nb);
    // forward before backward, as in every Wilson kernel (same rounding)
    if (!upper) {
        col_hop<MPMC_FP32, MU, true>(nb, lf, 1.f, g, acc);
        col_hop<MPMC_FP32, MU, false>(og, lb, 1.f, g, acc);
    } else {
        col_hop<MPMC_FP32, MU, true>(og, lf, 1.f, g, acc);
        col_hop<MPMC_FP32, MU, false>(nb, lb, 1.f, g, acc);
    }
}

// MODE 0: plain apply with the WOut epilogue (FP32 out, no FP16S);
// MODE 1: fused level step (w' = w - c M w [combined with a], eta^H Theta w').
// Per step t of a column: the loads of the t+1 site, the out-of-tile
// neighbours and the links are issued first; after the barrier the LDS hops
// run while they arrive; the t+1 site is then published for step t+1.
// TZ = 2: 2x2x2 tiles, eight wavefronts, 144 KB of LDS (one workgroup per
// compute unit; every step of a compute unit waits on one barrier).  TZ = 1:
// 2x2x1 tiles, four wavefronts, 72 KB, both z neighbours from global memory
// (five reads per site instead of four) but two independent workgroups per
// compute unit, so one's loads overlap the other's arithmetic.
template <int MODE, bool CMB, int TZ>
__global__ __launch_bounds__(256 * TZ) __attribute__((amdgpu_waves_per_eu(2))) void k_wilson_col(
    const void *__restrict__ b, const float2 *__restrict__ links, ColArgs ca, int N, WOut o,
    const uint32_t *__restrict__ codes, double2 c, double2 cnext, int theta, double2 *__restrict__ partial,
    int first_step, const void *__restrict__ a2, double2 alpha, double2 beta) {
    using T = float;
    __shared__ ColLds<TZ> L;
    // the wavefront index as a scalar: every site index below is then uniform,
    // and the buffer descriptors built from it stay in SGPRs (a per-lane
    // descriptor would make the compiler loop over lanes for each load)
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const unsigned lane = threadIdx.x & 63u;
    const int wx = w & 1, wy = (w >> 1) & 1, wz = TZ == 2 ? w >> 2 : 0;
    // Whole blocks of bx x by x bz tiles go to the XCDs (workgroup b runs on
    // XCD b % 8, in the order b / 8): a round of the workgroups an XCD runs at
    // once is one compact 3D block whose columns advance along t together, so
    // most out-of-tile neighbours were just fetched into the XCD's L2 by the
    // workgroup that owns them.  At each round the eight XCDs take eight
    // consecutive blocks of a snake that runs along z first (then x, then y),
    // so blocks that run at the same time share faces: the second read of a
    // face, from the neighbouring XCD at the same t, finds it in the
    // memory-side cache instead of HBM.  The grid is padded to a multiple of 8
    // blocks; padding workgroups return at once.
    const int bsz = ca.bx * ca.by * ca.bz, nbx = ca.ntx / ca.bx, nbz = ca.ntz / ca.bz;
    const long xcd = blockIdx.x % 8u, slot = blockIdx.x / 8u;
    const long lb = slot / bsz;
    const long gb0 = lb * 8 + xcd;
    if (gb0 >= ca.nblk) return;
    // consecutive launches of a recurrence alternate the direction of the
    // block sequence, so the first blocks of a launch read what the last
    // blocks of the previous one wrote, while it is still in the memory-side
    // cache (same arithmetic per tile: the results do not change)
    const long gb = ca.rev ? ca.nblk - 1 - gb0 : gb0;          // block over all chunks
    const long nbc = ca.ntiles / bsz;                          // blocks per 64-wide chunk
    const long chunk = gb / nbc, blk = gb - chunk * nbc;
    const int in = (int)(slot - lb * bsz);
    const unsigned tile = (unsigned)(chunk * ca.ntiles + blk * bsz + in);
    const long zrow = blk / nbz;                               // (x, y) block column of the snake
    const int bzi = (int)(zrow & 1 ? nbz - 1 - (blk - zrow * nbz) : blk - zrow * nbz);
    const int xrow = (int)(zrow / nbx);
    const int bxi = (int)(xrow & 1 ? nbx - 1 - (zrow - (long)xrow * nbx) : zrow - (long)xrow * nbx);
    const int tx = bxi * ca.bx + in % ca.bx;
    const int ty = xrow * ca.by + (in / ca.bx) % ca.by;
    const int tz = bzi * ca.bz + in / (ca.bx * ca.by);
    const int x = 2 * tx + wx, y = 2 * ty + wy, z = TZ * tz + wz, Lt = ca.L[3];
    const uint32_t r = (uint32_t)(chunk * 64 + lane);
    // out-of-tile neighbour coordinates (forward at the tile's upper edge, else
    // backward; TZ = 1: zo is the forward z neighbour, zb the backward one)
    const int xo = wx ? (x + 1 == ca.L[0] ? 0 : x + 1) : (x == 0 ? ca.L[0] - 1 : x - 1);
    const int yo = wy ? (y + 1 == ca.L[1] ? 0 : y + 1) : (y == 0 ? ca.L[1] - 1 : y - 1);
    const int zo = (TZ == 1 || wz) ? (z + 1 == ca.L[2] ? 0 : z + 1) : (z == 0 ? ca.L[2] - 1 : z - 1);
    // backward-neighbour coordinates (their forward links are this site's backward links)
    const int xb = x == 0 ? ca.L[0] - 1 : x - 1, yb = y == 0 ? ca.L[1] - 1 : y - 1, zb = z == 0 ? ca.L[2] - 1 : z - 1;
    const float g = o.g;
    const T kap = (T)o.kappa;

    {   // slices Lt-1 (read as t-1 at t = 0) and 0 of the own column
        cpx<float> v[12];
        col_load(b, col_site(ca, x, y, z, Lt - 1), N, r, v);
#pragma unroll
        for (int k = 0; k < 12; ++k) L.v[2][w][k][lane] = make_float2(v[k].re, v[k].im);
        col_load(b, col_site(ca, x, y, z, 0), N, r, v);
#pragma unroll
        for (int k = 0; k < 12; ++k) L.v[0][w][k][lane] = make_float2(v[k].re, v[k].im);
    }
    uint32_t ltprev[1];   // U_t(s - t): the forward t link of the previous site
    load_link_lanes<MPMC_FP32>(links + (col_site(ca, x, y, z, Lt - 1) * 4 + 3) * 9, ltprev);
    cpx<double> dot = mk(0.0, 0.0);

    // The out-of-tile neighbours of step t+1 are fetched during step t, each
    // into the registers its step-t value has just left (loop-carried): they
    // then travel to the L2 together with the neighbouring tiles' own loads
    // of slice t+1 (which those tiles issue during step t as well), so most of
    // them are served by the XCD's L2 instead of memory.
    cpx<float> ogx[12], ogy[12], ogz[12];
    col_load(b, col_site(ca, xo, y, z, 0), N, r, ogx);
    col_load(b, col_site(ca, x, yo, z, 0), N, r, ogy);
    col_load(b, col_site(ca, x, y, zo, 0), N, r, ogz);

    for (int t = 0; t < Lt; ++t) {
        const int curb = t % 3, prevb = (t + 2) % 3, nextb = (t + 1) % 3;
        const long s = col_site(ca, x, y, z, t);
        const bool more = t + 1 < Lt;
        // global traffic of the step: the t+1 site, the links and the noise code
        cpx<float> nx[12];
        col_load(b, col_site(ca, x, y, z, more ? t + 1 : 0), N, r, nx);
        uint32_t lf[4][1], lb[3][1];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) load_link_lanes<MPMC_FP32>(links + (s * 4 + mu) * 9, lf[mu]);
        load_link_lanes<MPMC_FP32>(links + (col_site(ca, xb, y, z, t) * 4 + 0) * 9, lb[0]);
        load_link_lanes<MPMC_FP32>(links + (col_site(ca, x, yb, z, t) * 4 + 1) * 9, lb[1]);
        load_link_lanes<MPMC_FP32>(links + (col_site(ca, x, y, zb, t) * 4 + 2) * 9, lb[2]);
        // the noise code and the step's output are touched once per launch:
        // non-temporal, so the L2 keeps the slices that neighbouring tiles read
        // (fused step 1,373 -> 1,352 us at 24^4 x 64)
        const uint32_t code = MODE == 1 ? __builtin_nontemporal_load(codes + s * N + r) : 0u;
        // slice t of every column of the tile (published one step ahead) is now
        // visible, and every read of step t-1 is done (three buffers rotate)
        __syncthreads();

        cpx<float> acc[4][3];
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) acc[sp][cc] = mk(0.f, 0.f);
        // hops in the order of every Wilson kernel: x, y, z, t, forward first
        col_dir<0>(L, curb, w, lane, wx, ogx, lf[0][0], lb[0][0], g, acc);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (TZ == 2) {
            if (more) col_load(b, col_site(ca, xo, y, z, t + 1), N, r, ogx);
        } else {
            // the backward z neighbour (both z neighbours are outside a 2x2x1 tile)
            col_load(b, col_site(ca, x, y, zb, t), N, r, ogx);
        }
        __builtin_amdgcn_sched_barrier(0);
        col_dir<1>(L, curb, w, lane, wy, ogy, lf[1][0], lb[1][0], g, acc);
        __builtin_amdgcn_sched_barrier(0);
        if (more) col_load(b, col_site(ca, x, yo, z, t + 1), N, r, ogy);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (TZ == 2) {
            col_dir<2>(L, curb, w, lane, wz, ogz, lf[2][0], lb[2][0], g, acc);
            __builtin_amdgcn_sched_barrier(0);
            if (more) col_load(b, col_site(ca, x, y, zo, t + 1), N, r, ogz);
            __builtin_amdgcn_sched_barrier(0);
        } else {
            col_hop<MPMC_FP32, 2, true>(ogz, lf[2][0], 1.f, g, acc);
            col_hop<MPMC_FP32, 2, false>(ogx, lb[2][0], 1.f, g, acc);
            __builtin_amdgcn_sched_barrier(0);
            if (more) {
                col_load(b, col_site(ca, x, y, zo, t + 1), N, r, ogz);
                col_load(b, col_site(ca, xo, y, z, t + 1), N, r, ogx);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        col_hop<MPMC_FP32, 3, true>(nx, lf[3][0], (ca.tap && t == Lt - 1) ? -1.f : 1.f, g, acc);
        {   // t backward: the own column's previous slice
            cpx<float> pv[12];
            col_lds_read(L, prevb, w, lane, pv);
            col_hop<MPMC_FP32, 3, false>(pv, ltprev[0], (ca.tap && t == 0) ? -1.f : 1.f, g, acc);
        }
        pin_acc(acc);
        // publish the t+1 site for step t+1 (that buffer was last read at step t-1)
#pragma unroll
        for (int k = 0; k < 12; ++k) L.v[nextb][w][k][lane] = make_float2(nx[k].re, nx[k].im);

        cpx<float> cur[12];
        col_lds_read(L, curb, w, lane, cur);
        const SiteAcc<MPMC_FP32, true> O(o.out, nullptr, s, N, r);
        if constexpr (MODE == 0) {
            const bool has_a = o.a_is_b || o.a;
            const cpx<T> al = has_a ? mk((T)o.alpha.x, (T)o.alpha.y) : mk(T(0), T(0));
            const cpx<T> be = mk((T)o.beta.x, (T)o.beta.y);
            const cpx<T> beg5 = o.theta ? mk(-be.re, -be.im) : be;
            cpx<T> av[12];
            if (o.a && !o.a_is_b) {
                const SiteAcc<MPMC_FP32, true> A(o.a, nullptr, s, N, r);
#pragma unroll
                for (int k = 0; k < 12; ++k) av[k] = A.ld(k);
            } else {
#pragma unroll
                for (int k = 0; k < 12; ++k) av[k] = cur[k];
            }
            cpx<T> res[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const cpx<T> mb = cur[k] - kap * acc[k / 3][k % 3];
                res[k] = (k >= 6 ? beg5 : be) * mb + al * av[k];
                O.st_stream(k, res[k]);
            }
            if (o.y) {
                const cpx<T> ga = mk((T)o.gamma.x, (T)o.gamma.y);
                const SiteAcc<MPMC_FP32, true> Y(o.y, nullptr, s, N, r);
                cpx<T> yv[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) yv[k] = Y.ld(k);
#pragma unroll
                for (int k = 0; k < 12; ++k) Y.st(k, yv[k] + ga * res[k]);
            }
        } else {
            const cpx<T> ccf = mk((T)c.x, (T)c.y);
            cpx<T> av[12];
            if constexpr (CMB) {
                const SiteAcc<MPMC_FP32, true> A(a2, nullptr, s, N, r);
#pragma unroll
                for (int k = 0; k < 12; ++k) av[k] = A.ld(k);
            }
            const cpx<T> al = mk((T)alpha.x, (T)alpha.y), be = mk((T)beta.x, (T)beta.y);
            // the site's terms in FP32, the running sum in FP64 (as k_wilson_dot)
            const T tsg = theta ? T(-1) : T(1);
            T sr = T(0), si = T(0);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const cpx<T> mw = cur[k] - kap * acc[k / 3][k % 3];
                cpx<T> wn = cur[k] - ccf * mw;
                if constexpr (CMB) wn = al * av[k] + be * wn;
                O.st_stream(k, wn);
                const uint32_t sym = (code >> (2 * k)) & 3u;
                const T sg = (sym & 2u) ? T(-1) : T(1);
                const T gg = k >= 6 ? sg * tsg : sg;
                sr += gg * ((sym & 1u) ? wn.im : wn.re);
                si += gg * ((sym & 1u) ? -wn.re : wn.im);
            }
            dot.re += (double)sr;
            dot.im += (double)si;
        }
        ltprev[0] = lf[3][0];
    }
    if constexpr (MODE == 1) {
        // per-tile partial of every right-hand side: the 8 columns summed in a fixed order
        __syncthreads();   // every wavefront is done with the slices
        double2 *red = reinterpret_cast<double2 *>(&L.v[0][0][0][0]);
        red[threadIdx.x] = make_double2(dot.re, dot.im);
        __syncthreads();
        if (threadIdx.x < 64) {
            double sx = 0, sy = 0;
#pragma unroll
            for (int q = 0; q < col_waves<TZ>(); ++q) {
                sx += red[q * 64 + threadIdx.x].x;
                sy += red[q * 64 + threadIdx.x].y;
            }
            const cpx<double> term = mk(cnext.x, cnext.y) * mk(sx, sy);
            double2 *pp = partial + (long)tile * 64 + threadIdx.x;
            if (first_step) {
                *pp = make_double2(term.re, term.im);
            } else {
                const double2 old = *pp;
                *pp = make_double2(old.x + term.re, old.y + term.im);
            }
        }
    }
}

// ------------------------------------ column streaming, 32-wide chunks --
// The same walk along t with twice the sites per workgroup: 2x2x4 tiles of
// (x, y, z) columns and 32-wide right-hand-side chunks, wavefront w holding
// the sites (w & 1, w >> 1 & 1, 2 (w >> 2) + h) of the tile in its lanes
// 32 h .. 32 h + 31 (h = 0, 1).  LDS per slice is the same 48 KB, but an
// XCD's round of 32 workgroups now covers an 8x8x8 block of sites instead of
// 8x8x4, so fewer out-of-tile neighbours fall outside the block the XCD's L2
// holds (0.75 instead of 1.0 per site) and the in-tile z neighbours cut the
// out-of-tile reads per site from three to two and a half; the links are read
// once per 32 right-hand sides instead of 64.  The two sites of a wavefront
// have different links: each 16-lane row loads its site's link and the
// values are broadcast within rows (DPP), as in the narrow-chunk traversals.

// Spinor access to the wavefront's two sites (z and z + 1): one buffer
// resource based at the lower site, the upper half's offset in the VGPR.
struct PairAcc {
    __amdgpu_buffer_rsrc_t rs;
    uint32_t vo;
    int N;
    __device__ __forceinline__ PairAcc(const void *base, long site0, uint32_t vo_, uint32_t range, int N_)
        : vo(vo_), N(N_) {
        const char *p = reinterpret_cast<const char *>(base) + site0 * 12L * N_ * 8;
        rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(p), (short)0, (int)range, kBufWord3);
    }
    __device__ __forceinline__ cpx<float> ld(int k) const {
        const f32x2 v = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)vo, k * N * 8, 0));
        return mk(v.x, v.y);
    }
    __device__ __forceinline__ void st_stream(int k, cpx<float> v) const {   // non-temporal, as in k_wilson_col
        f32x2 d;
        d.x = v.re;
        d.y = v.im;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, d), rs, (int)vo, k * N * 8, 2);
    }
    __device__ __forceinline__ void st(int k, cpx<float> v) const {
        f32x2 d;
        d.x = v.re;
        d.y = v.im;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, d), rs, (int)vo, k * N * 8, 0);
    }
};

// A link spread over 16-lane rows (as load_link_rows) at a uniform base
// (the pair's lower site) plus the lane's constant byte offset (its own site's
// link, dword i of the row): the address arithmetic stays scalar.
__device__ __forceinline__ void colp_link(const float2 *base, uint32_t off0, uint32_t off1, uint32_t (&lw)[2]) {
    const char *p = reinterpret_cast<const char *>(base);
    lw[0] = *reinterpret_cast<const uint32_t *>(p + off0);
    lw[1] = *reinterpret_cast<const uint32_t *>(p + off1);
}

__device__ __forceinline__ void colp_load(const void *b, long site0, uint32_t vo, uint32_t range, int N,
                                          cpx<float> (&psi)[12]) {
    const PairAcc A(b, site0, vo, range, N);
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k] = A.ld(k);
}

// hop MU from a spinor held by the lane, link spread over the lane's row
template <int MU, bool FWD>
__device__ __forceinline__ void colp_hop(const cpx<float> (&psi)[12], const uint32_t (&lw)[2], float bsign, float g,
                                         cpx<float> acc[4][3]) {
    HopData<MPMC_FP32> H;
#pragma unroll
    for (int k = 0; k < 12; ++k) H.psi[k] = psi[k];
    H.lw[0] = lw[0];
    H.lw[1] = lw[1];
    H.bsign = bsign;
    apply<MPMC_FP32, false, MU, FWD, true>(H, g, acc);
    __builtin_amdgcn_sched_barrier(0);
}

// the partner's spinor from LDS: wavefront wv, lane ln (both per lane)
__device__ __forceinline__ void colp_lds_read(const ColLds<2> &L, int buf, int wv, unsigned ln, cpx<float> (&psi)[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const float2 v = L.v[buf][wv][k][ln];
        psi[k] = mk(v.x, v.y);
    }
}

// x or y hops (the in-tile neighbour is the partner wavefront's same lane)
template <int MU>
__device__ __forceinline__ void colp_dir(const ColLds<2> &L, int curb, int w, unsigned lane, int upper,
                                         const cpx<float> (&og)[12], const uint32_t (&lf)[2], const uint32_t (&lb)[2],
                                         float g, cpx<float> acc[4][3]) {
    cpx<float> nb[12];
    colp_lds_read(L, curb, w ^ (1 << MU), lane, nb);
    if (!upper) {
        colp_hop<MU, true>(nb, lf, 1.f, g, acc);
        colp_hop<MU, false>(og, lb, 1.f, g, acc);
    } else {
        colp_hop<MU, true>(og, lf, 1.f, g, acc);
        colp_hop<MU, false>(nb, lb, 1.f, g, acc);
    }
}

template <int MODE, bool CMB>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void k_wilson_colp(
    const void *__restrict__ b, const float2 *__restrict__ links, ColArgs ca, int N, WOut o,
    const uint32_t *__restrict__ codes, double2 c, double2 cnext, int theta, double2 *__restrict__ partial,
    int first_step, const void *__restrict__ a2, double2 alpha, double2 beta) {
    using T = float;
    __shared__ ColLds<2> L;
    // the lane's running quadratic form in LDS (live registers are the limit here)
    __shared__ double2 dotl[MODE == 1 ? 512 : 1];
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const unsigned lane = threadIdx.x & 63u;
    const unsigned h = lane >> 5;                  // the wavefront's lower (0) or upper (1) site
    const int wx = w & 1, wy = (w >> 1) & 1, wzp = w >> 2;
    // XCD rounds and the z-first snake of blocks exactly as in k_wilson_col
    const int bsz = ca.bx * ca.by * ca.bz, nbx = ca.ntx / ca.bx, nbz = ca.ntz / ca.bz;
    const long xcd = blockIdx.x % 8u, slot = blockIdx.x / 8u;
    const long lb = slot / bsz;
    const long gb0 = lb * 8 + xcd;
    if (gb0 >= ca.nblk) return;
    const long gb = ca.rev ? ca.nblk - 1 - gb0 : gb0;
    const long nbc = ca.ntiles / bsz;
    const long chunk = gb / nbc, blk = gb - chunk * nbc;
    const int in = (int)(slot - lb * bsz);
    const unsigned tile = (unsigned)(chunk * ca.ntiles + blk * bsz + in);
    const long zrow = blk / nbz;
    const int bzi = (int)(zrow & 1 ? nbz - 1 - (blk - zrow * nbz) : blk - zrow * nbz);
    const int xrow = (int)(zrow / nbx);
    const int bxi = (int)(xrow & 1 ? nbx - 1 - (zrow - (long)xrow * nbx) : zrow - (long)xrow * nbx);
    const int tx = bxi * ca.bx + in % ca.bx;
    const int ty = xrow * ca.by + (in / ca.bx) % ca.by;
    const int tz = bzi * ca.bz + in / (ca.bx * ca.by);
    const int x = 2 * tx + wx, y = 2 * ty + wy, z0 = 4 * tz + 2 * wzp, Lt = ca.L[3];
    const uint32_t r = (uint32_t)(chunk * 32 + (lane & 31u));
    const long plane = (long)ca.L[0] * ca.L[1];   // sites between z and z + 1
    // pair accessors: lower site's resource, upper half offset plane sites
    const uint32_t pbytes = (uint32_t)(plane * 12 * N * 8);
    const uint32_t range = pbytes + (uint32_t)(12 * N * 8);
    const uint32_t vo = h * pbytes + r * 8u;
    const long lsite_off = h ? plane : 0;          // the lane's own site = pair site + lsite_off
    const int xo = wx ? (x + 1 == ca.L[0] ? 0 : x + 1) : (x == 0 ? ca.L[0] - 1 : x - 1);
    const int yo = wy ? (y + 1 == ca.L[1] ? 0 : y + 1) : (y == 0 ? ca.L[1] - 1 : y - 1);
    // the one out-of-tile z neighbour of the wavefront: below the lower site
    // (wzp = 0, needed by the lower half) or above the upper one (wzp = 1,
    // upper half); the other half finds its z neighbours in LDS
    const int zq = wzp ? (z0 + 2 == ca.L[2] ? 0 : z0 + 2) : (z0 == 0 ? ca.L[2] - 1 : z0 - 1);
    const bool zglob = (int)h == wzp;
    const int xb = x == 0 ? ca.L[0] - 1 : x - 1, yb = y == 0 ? ca.L[1] - 1 : y - 1;
    // per-lane byte offsets of the links from the pair's lower site's: a
    // row's lanes take dwords i and 16 + (i < 2 ? i : 0) of their site's link
    const unsigned li = lane & 15u;
    const uint32_t lrow0 = li * 4u, lrow1 = (16u + (li < 2u ? li : 0u)) * 4u;
    const uint32_t lh = (uint32_t)(lsite_off * 4 * 9 * 8);
    // backward z links: based at the lower of the two halves' backward sites
    // (z0 - 1 and z0, or z0 and Lz - 1 when z0 = 0), so both offsets are >= 0
    const long zbase = z0 == 0 ? 0 : -plane;
    const uint32_t lhz = (uint32_t)((z0 == 0 ? (h ? 0 : (long)(ca.L[2] - 1) * plane) : (h ? plane : 0)) * 4 * 9 * 8);
    const uint32_t cofs = (uint32_t)((lsite_off * N + r) * 4);          // noise code offset
    const float g = o.g;
    const T kap = (T)o.kappa;
    // LDS partners across z (lane ^ 32 of the own or the other z-pair wavefront)
    const unsigned lz = lane ^ 32u;
    const int wzf = h ? (w ^ 4) : w;               // forward z partner's wavefront
    const int wzb = h ? w : (w ^ 4);               // backward z partner's wavefront

    {
        cpx<float> v[12];
        colp_load(b, col_site(ca, x, y, z0, Lt - 1), vo, range, N, v);
#pragma unroll
        for (int k = 0; k < 12; ++k) L.v[2][w][k][lane] = make_float2(v[k].re, v[k].im);
        colp_load(b, col_site(ca, x, y, z0, 0), vo, range, N, v);
#pragma unroll
        for (int k = 0; k < 12; ++k) L.v[0][w][k][lane] = make_float2(v[k].re, v[k].im);
    }
    uint32_t ltprev[2];
    colp_link(links + (col_site(ca, x, y, z0, Lt - 1) * 4 + 3) * 9, lh + lrow0, lh + lrow1, ltprev);
    if constexpr (MODE == 1) dotl[threadIdx.x] = make_double2(0.0, 0.0);

    cpx<float> ogx[12], ogy[12], ogz[12];
    colp_load(b, col_site(ca, xo, y, z0, 0), vo, range, N, ogx);
    colp_load(b, col_site(ca, x, yo, z0, 0), vo, range, N, ogy);
    if (zglob) col_load(b, col_site(ca, x, y, zq, 0), N, r, ogz);

    for (int t = 0; t < Lt; ++t) {
        const int curb = t % 3, prevb = (t + 2) % 3, nextb = (t + 1) % 3;
        const long sp = col_site(ca, x, y, z0, t);   // the pair's lower site
        const bool more = t + 1 < Lt;
        cpx<float> nx[12];
        colp_load(b, col_site(ca, x, y, z0, more ? t + 1 : 0), vo, range, N, nx);
        uint32_t lf[4][2], lbk[3][2];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) colp_link(links + (sp * 4 + mu) * 9, lh + lrow0, lh + lrow1, lf[mu]);
        colp_link(links + (col_site(ca, xb, y, z0, t) * 4 + 0) * 9, lh + lrow0, lh + lrow1, lbk[0]);
        colp_link(links + (col_site(ca, x, yb, z0, t) * 4 + 1) * 9, lh + lrow0, lh + lrow1, lbk[1]);
        colp_link(links + ((sp + zbase) * 4 + 2) * 9, lhz + lrow0, lhz + lrow1, lbk[2]);
        const uint32_t code =
            MODE == 1 ? __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(
                            reinterpret_cast<const char *>(codes + sp * N) + cofs))
                      : 0u;
        __syncthreads();

        cpx<float> acc[4][3];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) acc[q][cc] = mk(0.f, 0.f);
        colp_dir<0>(L, curb, w, lane, wx, ogx, lf[0], lbk[0], g, acc);
        __builtin_amdgcn_sched_barrier(0);
        if (more) colp_load(b, col_site(ca, xo, y, z0, t + 1), vo, range, N, ogx);
        __builtin_amdgcn_sched_barrier(0);
        colp_dir<1>(L, curb, w, lane, wy, ogy, lf[1], lbk[1], g, acc);
        __builtin_amdgcn_sched_barrier(0);
        if (more) colp_load(b, col_site(ca, x, yo, z0, t + 1), vo, range, N, ogy);
        __builtin_amdgcn_sched_barrier(0);
        // z: forward, then backward; the half without an out-of-tile
        // neighbour takes the partner's spinor from LDS into ogz's registers
        {
            cpx<float> nb[12];
            if (wzp == 0) {
                colp_lds_read(L, curb, wzf, lz, nb);
                colp_hop<2, true>(nb, lf[2], 1.f, g, acc);
                if (!zglob) colp_lds_read(L, curb, wzb, lz, ogz);
                colp_hop<2, false>(ogz, lbk[2], 1.f, g, acc);
            } else {
                if (!zglob) colp_lds_read(L, curb, wzf, lz, ogz);
                colp_hop<2, true>(ogz, lf[2], 1.f, g, acc);
                colp_lds_read(L, curb, wzb, lz, nb);
                colp_hop<2, false>(nb, lbk[2], 1.f, g, acc);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        if (more && zglob) col_load(b, col_site(ca, x, y, zq, t + 1), N, r, ogz);
        __builtin_amdgcn_sched_barrier(0);
        colp_hop<3, true>(nx, lf[3], (ca.tap && t == Lt - 1) ? -1.f : 1.f, g, acc);
        {
            cpx<float> pv[12];
            colp_lds_read(L, prevb, w, lane, pv);
            colp_hop<3, false>(pv, ltprev, (ca.tap && t == 0) ? -1.f : 1.f, g, acc);
        }
        pin_acc(acc);
#pragma unroll
        for (int k = 0; k < 12; ++k) L.v[nextb][w][k][lane] = make_float2(nx[k].re, nx[k].im);

        cpx<float> cur[12];
        colp_lds_read(L, curb, w, lane, cur);
        const PairAcc O(o.out, sp, vo, range, N);
        if constexpr (MODE == 0) {
            const bool has_a = o.a_is_b || o.a;
            const cpx<T> al = has_a ? mk((T)o.alpha.x, (T)o.alpha.y) : mk(T(0), T(0));
            const cpx<T> be = mk((T)o.beta.x, (T)o.beta.y);
            const cpx<T> beg5 = o.theta ? mk(-be.re, -be.im) : be;
            cpx<T> av[12];
            if (o.a && !o.a_is_b) {
                const PairAcc A(o.a, sp, vo, range, N);
#pragma unroll
                for (int k = 0; k < 12; ++k) av[k] = A.ld(k);
            } else {
#pragma unroll
                for (int k = 0; k < 12; ++k) av[k] = cur[k];
            }
            cpx<T> res[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const cpx<T> mb = cur[k] - kap * acc[k / 3][k % 3];
                res[k] = (k >= 6 ? beg5 : be) * mb + al * av[k];
                O.st_stream(k, res[k]);
            }
            if (o.y) {
                const cpx<T> ga = mk((T)o.gamma.x, (T)o.gamma.y);
                const PairAcc Y(o.y, sp, vo, range, N);
                cpx<T> yv[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) yv[k] = Y.ld(k);
#pragma unroll
                for (int k = 0; k < 12; ++k) Y.st(k, yv[k] + ga * res[k]);
            }
        } else {
            const cpx<T> ccf = mk((T)c.x, (T)c.y);
            cpx<T> av[12];
            if constexpr (CMB) {
                const PairAcc A(a2, sp, vo, range, N);
#pragma unroll
                for (int k = 0; k < 12; ++k) av[k] = A.ld(k);
            }
            const cpx<T> al = mk((T)alpha.x, (T)alpha.y), be = mk((T)beta.x, (T)beta.y);
            const T tsg = theta ? T(-1) : T(1);
            T sr = T(0), si = T(0);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const cpx<T> mw = cur[k] - kap * acc[k / 3][k % 3];
                cpx<T> wn = cur[k] - ccf * mw;
                if constexpr (CMB) wn = al * av[k] + be * wn;
                O.st_stream(k, wn);
                const uint32_t sym = (code >> (2 * k)) & 3u;
                const T sg = (sym & 2u) ? T(-1) : T(1);
                const T gg = k >= 6 ? sg * tsg : sg;
                sr += gg * ((sym & 1u) ? wn.im : wn.re);
                si += gg * ((sym & 1u) ? -wn.re : wn.im);
            }
            const double2 d0 = dotl[threadIdx.x];
            dotl[threadIdx.x] = make_double2(d0.x + (double)sr, d0.y + (double)si);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) ltprev[q] = lf[3][q];
    }
    if constexpr (MODE == 1) {
        // per-tile partial of each of the 32 right-hand sides: the 16 columns
        // summed in a fixed order (wavefront, then lower before upper site)
        __syncthreads();
        const double2 *red = dotl;
        if (threadIdx.x < 32) {
            double sx = 0, sy = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q)
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    sx += red[q * 64 + hh * 32 + threadIdx.x].x;
                    sy += red[q * 64 + hh * 32 + threadIdx.x].y;
                }
            const cpx<double> term = mk(cnext.x, cnext.y) * mk(sx, sy);
            double2 *pp = partial + (long)tile * 32 + threadIdx.x;
            if (first_step) {
                *pp = make_double2(term.re, term.im);
            } else {
                const double2 old = *pp;
                *pp = make_double2(old.x + term.re, old.y + term.im);
            }
        }
    }
}

// ------------------------------------------------------------- launch --

static double spinor_bytes(int prec) { return prec == MPMC_FP64 ? 192.0 : (prec == MPMC_FP32 ? 96.0 : 52.0); }

// The column-streaming kernel needs even Lx, Ly (and Lz for 2x2x2 tiles),
// Lt >= 4, FP32 and 64-wide chunks.
static bool col_ok(const mpmc_ctx *ctx, int nrhs, int prec, int tz = 2) {
    const bool ok = prec == MPMC_FP32 && nrhs % 64 == 0 && ctx->dims[0] % 2 == 0 && ctx->dims[1] % 2 == 0 &&
                    ctx->dims[2] % tz == 0 && ctx->dims[3] >= 4;
    if (!ok || tz != 4) return ok;
    // 2x2x4 tiles: a wavefront's two sites (one z-plane apart) share one
    // buffer resource, whose range must stay below 2 GiB
    // (and per-lane link offsets below 2 GiB as well)
    const double range = ((double)ctx->dims[0] * ctx->dims[1] + 1) * 12.0 * nrhs * 8.0;
    return range < 2147483648.0 && (double)ctx->V * 288.0 < 2147483648.0;
}
static ColArgs col_args(const mpmc_ctx *ctx, int tz = 2) {
    ColArgs a;
    for (int mu = 0; mu < 4; ++mu) a.L[mu] = ctx->dims[mu];
    a.ntx = ctx->dims[0] / 2;
    a.nty = ctx->dims[1] / 2;
    a.ntz = ctx->dims[2] / tz;
    // blocks of 8 x 8 x 4 sites where the extents allow (32 tiles of 2x2x2,
    // 64 of 2x2x1: one round of workgroups of an XCD; 8 x 8 x 8 sites of
    // 2x2x4 tiles)
    auto ext = [](int n, int want) {
        while (want > 1 && n % want != 0) want /= 2;
        return want;
    };
    a.bx = ext(a.ntx, 4);
    a.by = ext(a.nty, 4);
    a.bz = ext(a.ntz, tz == 1 ? 4 : 2);   // 2x2x4 tiles: 4x4x2 of them, 8x8x8 sites
    a.ntiles = (long)a.ntx * a.nty * a.ntz;
    a.nblk = 0;
    a.tap = ctx->t_antiperiodic;
    a.rev = 0;
    return a;
}
// Grid of a column launch over nrhs / width chunks (sets ca.nblk).
static unsigned col_grid(ColArgs &ca, int nrhs, int width = 64) {
    const long bsz = (long)ca.bx * ca.by * ca.bz;
    ca.nblk = ca.ntiles / bsz * (nrhs / width);
    return (unsigned)(8 * ((ca.nblk + 7) / 8) * bsz);
}
static int default_variant(const mpmc_ctx *ctx, int nrhs, int prec) {
    if (col_ok(ctx, nrhs, prec)) return WILSON_COLUMN;
    return prec == MPMC_FP64 ? 4 : 5;
}
static double link_bytes(int prec) { return prec == MPMC_FP64 ? 576.0 : 288.0; }

template <int P>
static WIn<P> make_in(const mpmc_ctx *ctx, const void *b, int nrhs) {
    WIn<P> in;
    VecRef vb = vref(ctx, b, nrhs, P);
    in.b = vb.d;
    in.bsc = vb.sc;
    in.nbr = ctx->nbr;
    in.links = reinterpret_cast<const typename LinkT<P>::type *>(P == MPMC_FP64 ? (const void *)ctx->links64
                                                                                 : (const void *)ctx->links32);
    return in;
}

// Kernel variant for (nrhs, prec): pinned or tuned by the autotuner, else the default.
static int wilson_variant(const mpmc_ctx *ctx, int nrhs, int prec) {
    const auto it = ctx->tune.find(std::make_pair(nrhs, prec));
    const int v = it == ctx->tune.end() ? default_variant(ctx, nrhs, prec) : it->second;
    if (v == WILSON_COLUMN) return col_ok(ctx, nrhs, prec) ? v : (prec == MPMC_FP64 ? 4 : 5);
    if (v == WILSON_COLUMN1) return col_ok(ctx, nrhs, prec, 1) ? v : (prec == MPMC_FP64 ? 4 : 5);
    if (v == WILSON_COLUMNP) return col_ok(ctx, nrhs, prec, 4) ? v : (prec == MPMC_FP64 ? 4 : 5);
    return (v >> 1) >= 3 && ctx->V % 16 != 0 ? (v & 1) | 4 : v;
}

// The fused level step (FP32) takes the column kernel with 2x2x2 tiles where
// the lattice allows it; otherwise (FP64 and other shapes) the 64-wide
// blocked order whenever its chunk tiles hold one chunk each (V % 4 == 0),
// and the site-major order otherwise;
// a variant set explicitly for (nrhs, prec) with mpmc_tune_set selects its
// traversal (orders 0 and 1: site-major; 3 and 4 need V % 16 == 0), and
// otherwise mpmc_autotune_level's choice, once made, replaces the default.
constexpr int kDotDefaultOrder = 2;   // 64-wide blocked chunks (FP64; FP32 takes the column kernel)
constexpr int kDotColumn = 5;         // order code of the column-streaming fused step (2x2x2 tiles)
constexpr int kDotColumn1 = 6;        // the same with 2x2x1 tiles
constexpr int kDotColumnP = 7;        // 2x2x4 tiles, 32-wide chunks (k_wilson_colp)
constexpr int kDotOrders = 8;
static bool is_col_order(int o) { return o == kDotColumn || o == kDotColumn1 || o == kDotColumnP; }
static int col_order_tz(int o) { return o == kDotColumn1 ? 1 : (o == kDotColumnP ? 4 : 2); }
static int dot_order(const mpmc_ctx *ctx, int nrhs, int prec) {
    const auto td = ctx->tune_dot.find(std::make_pair(nrhs, prec));
    if (td != ctx->tune_dot.end() && ctx->tune_explicit.find(std::make_pair(nrhs, prec)) == ctx->tune_explicit.end()) {
        const int o = td->second;   // the autotuner's choice (valid for this shape by construction)
        return o;
    }
    const auto it = ctx->tune_explicit.find(std::make_pair(nrhs, prec));
    if (it != ctx->tune_explicit.end() && it->second == WILSON_COLUMN1 && col_ok(ctx, nrhs, prec, 1) && nrhs <= 256)
        return kDotColumn1;
    if (it != ctx->tune_explicit.end() && it->second == WILSON_COLUMNP && col_ok(ctx, nrhs, prec, 4) && nrhs <= 256)
        return kDotColumnP;
    if (it == ctx->tune_explicit.end() || it->second >= WILSON_COLUMN)
        if (col_ok(ctx, nrhs, prec) && nrhs <= 256) return kDotColumn;
    if (ctx->V % 4 != 0) return 0;
    const int o = (it == ctx->tune_explicit.end() || it->second >= WILSON_COLUMN) ? kDotDefaultOrder : it->second >> 1;
    if (o >= 3) return ctx->V % 16 == 0 ? o : 2;
    return o == 2 ? 2 : 0;
}
int wilson_dot_order(const mpmc_ctx *ctx, int nrhs, int prec) { return dot_order(ctx, nrhs, prec); }

static int dot_width(int order, int nrhs) {
    return order == 3 ? 16 : (order == 4 || order == kDotColumnP) ? 32
                             : (order == 2 || is_col_order(order)) ? 64 : (nrhs < 256 ? nrhs : 256);
}
static long dot_tiles_per_chunk(const mpmc_ctx *ctx, int order, int width) {
    if (is_col_order(order)) return col_args(ctx, col_order_tz(order)).ntiles;
    return ctx->V * width / 256;
}

template <int P, int V_>
static void launch_uniform(mpmc_ctx *ctx, const WIn<P> &in, const WOut &o, int nrhs, unsigned grid) {
    constexpr int ORDER = V_ >> 1;
    k_wilson<P, (ORDER <= 2), V_ & 1, ORDER><<<grid, 256, 0, ctx->stream>>>(in.b, in.bsc, in.nbr, in.links, o, ctx->V,
                                                                          nrhs, ctx->site_order);
}

// Single vectors: k_wilson1 (eight lanes per site, one hop each, one
// wavefront per workgroup) keeps a small lattice's dependent chain of
// launches short; on large lattices its scattered per-lane loads dominate and
// one site per lane (all eight hops in the lane) is faster: k_wilson_sv, or
// the generic kernel at one right-hand side.  mpmc_tune_set(ctx, 1, prec, v)
// pins one: v = 0 k_wilson1, 1 the generic kernel, 2 k_wilson_sv.
constexpr long kWilson1MaxV = 20736;   // 12^4 sites
static int single_vector_kernel(const mpmc_ctx *ctx, int prec) {
    const auto it = ctx->tune.find(std::make_pair(1, prec));
    if (it != ctx->tune.end() && it->second <= 2) return it->second;
    return ctx->V > kWilson1MaxV ? 2 : 0;
}
static SvGeom sv_geom(const mpmc_ctx *ctx) {
    SvGeom G;
    int st = 1;
    for (int mu = 0; mu < 4; ++mu) {
        G.L[mu] = ctx->dims[mu];
        G.st[mu] = st;
        G.wrap[mu] = (ctx->dims[mu] - 1) * st;
        st *= ctx->dims[mu];
    }
    G.anti = ctx->t_antiperiodic;
    return G;
}

template <int P>
static void launch_w(mpmc_ctx *ctx, const void *b, WOut &o, int nrhs, double2 yinit, int yinit_on) {
    const long work = ctx->V * nrhs;
    const unsigned grid = grid_for(work, 256);
    WIn<P> in = make_in<P>(ctx, b, nrhs);
    if constexpr (P != MPMC_FP16S) {
        if (nrhs == 1) {
            const int sv = single_vector_kernel(ctx, P);
            if (sv == 0) {
                k_wilson1<P><<<grid_for(ctx->V * 8, 64), 64, 0, ctx->stream>>>(in.b, in.nbr, in.links, o, ctx->V,
                                                                                yinit, yinit_on);
                return;
            }
            if (sv == 2) {
                k_wilson_sv<P><<<grid_for(ctx->V, 256), 256, 0, ctx->stream>>>(in.b, in.links, o, sv_geom(ctx),
                                                                               ctx->V, yinit, yinit_on);
                return;
            }
            // site per lane (the generic kernel below); the accumulator start
            // y = yinit b is its own pass
            if (yinit_on) blas_axpby(ctx, b, o.y, 1, P, yinit, make_double2(0, 0));
        }
    }
    if constexpr (P == MPMC_FP32) {
        const int cv = nrhs % 64 == 0 && !o.osc ? wilson_variant(ctx, nrhs, P) : -1;
        if (cv == WILSON_COLUMN) {
            ColArgs ca = col_args(ctx, 2);
            k_wilson_col<0, false, 2><<<col_grid(ca, nrhs), 512, 0, ctx->stream>>>(
                in.b, in.links, ca, nrhs, o, nullptr, make_double2(0, 0), make_double2(0, 0), 0, nullptr, 0, nullptr,
                make_double2(0, 0), make_double2(1, 0));
            return;
        }
        if (cv == WILSON_COLUMNP) {
            ColArgs ca = col_args(ctx, 4);
            k_wilson_colp<0, false><<<col_grid(ca, nrhs, 32), 512, 0, ctx->stream>>>(
                in.b, in.links, ca, nrhs, o, nullptr, make_double2(0, 0), make_double2(0, 0), 0, nullptr, 0, nullptr,
                make_double2(0, 0), make_double2(1, 0));
            return;
        }
        if (cv == WILSON_COLUMN1) {
            ColArgs ca = col_args(ctx, 1);
            k_wilson_col<0, false, 1><<<col_grid(ca, nrhs), 256, 0, ctx->stream>>>(
                in.b, in.links, ca, nrhs, o, nullptr, make_double2(0, 0), make_double2(0, 0), 0, nullptr, 0, nullptr,
                make_double2(0, 0), make_double2(1, 0));
            return;
        }
    }
    if (nrhs % 64 == 0) {
        const int v = wilson_variant(ctx, nrhs, P);
        switch (v >= WILSON_COLUMN ? 5 : v) {
        case 0: launch_uniform<P, 0>(ctx, in, o, nrhs, grid); break;
        case 1: launch_uniform<P, 1>(ctx, in, o, nrhs, grid); break;
        case 2: launch_uniform<P, 2>(ctx, in, o, nrhs, grid); break;
        case 3: launch_uniform<P, 3>(ctx, in, o, nrhs, grid); break;
        case 4: launch_uniform<P, 4>(ctx, in, o, nrhs, grid); break;
        case 5: launch_uniform<P, 5>(ctx, in, o, nrhs, grid); break;
        case 6: launch_uniform<P, 6>(ctx, in, o, nrhs, grid); break;
        case 7: launch_uniform<P, 7>(ctx, in, o, nrhs, grid); break;
        case 8: launch_uniform<P, 8>(ctx, in, o, nrhs, grid); break;
        default: launch_uniform<P, 9>(ctx, in, o, nrhs, grid); break;
        }
    } else {
        k_wilson<P, false><<<grid, 256, 0, ctx->stream>>>(in.b, in.bsc, in.nbr, in.links, o, ctx->V, nrhs, nullptr);
    }
}

int wilson_launch_full(mpmc_ctx *ctx, const void *b, const void *a, void *out, void *y, int nrhs, int prec,
                       double2 alpha, double2 beta, double2 gamma, int dagger, int theta, double2 yinit,
                       int yinit_on) {
    if (prec == MPMC_FP16S && y) return set_err(ctx, MPMC_EINVAL, "FP16S output cannot accumulate");
    if (yinit_on && (nrhs != 1 || !y || a != b))
        return set_err(ctx, MPMC_EINVAL, "accumulator start from the operand: single vectors with a == b only");
    WOut o;
    VecRef vo = vref(ctx, out, nrhs, prec);
    o.out = vo.d;
    o.osc = vo.sc;
    VecRef va = a ? vref(ctx, a, nrhs, prec) : VecRef{nullptr, nullptr};
    o.a = va.d;
    o.asc = va.sc;
    o.a_is_b = (a != nullptr && a == b) ? 1 : 0;
    o.y = y;
    o.kappa = ctx->kappa;
    o.alpha = alpha;
    o.beta = beta;
    o.gamma = gamma;
    o.g = dagger ? -1.f : 1.f;
    o.theta = theta;
    o.out_fp32 = 0;
    const int ev = nrhs > 1 ? timing_begin(ctx) : -1;   // single vectors: counted, no events
    if (prec == MPMC_FP64) launch_w<MPMC_FP64>(ctx, b, o, nrhs, yinit, yinit_on);
    else if (prec == MPMC_FP32) launch_w<MPMC_FP32>(ctx, b, o, nrhs, yinit, yinit_on);
    else launch_w<MPMC_FP16S>(ctx, b, o, nrhs, yinit, yinit_on);
    HIP_OR_RET(ctx, hipGetLastError());
    if (ctx->timing) {
        // algorithmic bytes: operand read once, a read once if distinct,
        // out written once, y read (unless it starts from b) and written,
        // links once per site
        const double sb = spinor_bytes(prec);
        double per = 2 * sb;
        if (a && a != b) per += sb;
        if (y) per += yinit_on ? sb : 2 * sb;
        const double bytes = (double)ctx->V * ((double)nrhs * per + link_bytes(prec));
        if (ev >= 0) timing_end(ctx, ev, prec | MPMC_TIMING_PLAIN, bytes);
        else timing_count(ctx, prec | MPMC_TIMING_SINGLE, bytes);
    }
    ctx->mvps += (uint64_t)nrhs;
    return MPMC_OK;
}

int wilson_apply_h2f(mpmc_ctx *ctx, const void *b, void *out, int nrhs) {
    WOut o;
    o.out = out;
    o.osc = nullptr;
    o.a = nullptr;
    o.asc = nullptr;
    o.a_is_b = 0;
    o.y = nullptr;
    o.kappa = ctx->kappa;
    o.alpha = make_double2(0, 0);
    o.beta = make_double2(1, 0);
    o.gamma = make_double2(0, 0);
    o.g = 1.f;
    o.theta = 0;
    o.out_fp32 = 1;
    const int ev = timing_begin(ctx);
    launch_w<MPMC_FP16S>(ctx, b, o, nrhs, make_double2(0, 0), 0);
    HIP_OR_RET(ctx, hipGetLastError());
    if (ev >= 0)
        timing_end(ctx, ev, MPMC_FP16S | MPMC_TIMING_PLAIN,
                   (double)ctx->V * ((double)nrhs * (spinor_bytes(MPMC_FP16S) + spinor_bytes(MPMC_FP32)) +
                                     link_bytes(MPMC_FP16S)));
    ctx->mvps += (uint64_t)nrhs;
    return MPMC_OK;
}

size_t wilson_dot_partial_count(const mpmc_ctx *ctx, int nrhs) {
    const long blocks = (ctx->V * nrhs + 255) / 256;
    return (size_t)blocks * (nrhs < 256 ? nrhs : 256);
}

int wilson_noise_codes(mpmc_ctx *ctx, uint64_t seed, uint32_t stream, uint64_t first, int nrhs, uint32_t *codes,
                       int ld, int off) {
    const long work = ctx->V * nrhs;
    k_noise_codes<<<grid_for(work, 256), 256, 0, ctx->stream>>>(seed, stream, first, codes, ctx->V, nrhs,
                                                                ld > 0 ? ld : nrhs, off);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

template <int P, bool CMB>
static void launch_dot(mpmc_ctx *ctx, int dord, unsigned grid, const WIn<P> &in, void *wout, const uint32_t *codes,
                       double2 c, double2 cnext, int theta, double2 *partial, int nrhs, int first_step,
                       const void *a, double2 alpha, double2 beta) {
    const int *ord = dord ? ctx->site_order : nullptr;
    if constexpr (P == MPMC_FP32) {
        if (is_col_order(dord)) {
            const int tz = col_order_tz(dord);
            ColArgs ca = col_args(ctx, tz);
            ca.rev = (int)(ctx->col_flip++ & 1u);
            const unsigned grid_c = col_grid(ca, nrhs, tz == 4 ? 32 : 64);
            WOut o{};
            o.out = wout;   // the step's output w'
            o.kappa = ctx->kappa;
            o.g = 1.f;
            if (tz == 4)
                k_wilson_colp<1, CMB><<<grid_c, 512, 0, ctx->stream>>>(
                    in.b, in.links, ca, nrhs, o, codes, c, cnext, theta, partial, first_step, a, alpha, beta);
            else if (tz == 2)
                k_wilson_col<1, CMB, 2><<<grid_c, 512, 0, ctx->stream>>>(
                    in.b, in.links, ca, nrhs, o, codes, c, cnext, theta, partial, first_step, a, alpha, beta);
            else
                k_wilson_col<1, CMB, 1><<<grid_c, 256, 0, ctx->stream>>>(
                    in.b, in.links, ca, nrhs, o, codes, c, cnext, theta, partial, first_step, a, alpha, beta);
            return;
        }
    }
    switch (dord) {
    case 2:
        k_wilson_dot<P, 2, false, CMB><<<grid, 256, 0, ctx->stream>>>(in.b, in.nbr, in.links, wout, codes, c, cnext,
                                                                      ctx->kappa, theta, partial, ctx->V, nrhs,
                                                                      first_step, ord, 0, nullptr, a, alpha, beta);
        break;
    case 3:
        k_wilson_dot<P, 3, false, CMB><<<grid, 256, 0, ctx->stream>>>(in.b, in.nbr, in.links, wout, codes, c, cnext,
                                                                      ctx->kappa, theta, partial, ctx->V, nrhs,
                                                                      first_step, ord, 0, nullptr, a, alpha, beta);
        break;
    case 4:
        k_wilson_dot<P, 4, false, CMB><<<grid, 256, 0, ctx->stream>>>(in.b, in.nbr, in.links, wout, codes, c, cnext,
                                                                      ctx->kappa, theta, partial, ctx->V, nrhs,
                                                                      first_step, ord, 0, nullptr, a, alpha, beta);
        break;
    default:
        k_wilson_dot<P, 0, false, CMB><<<grid, 256, 0, ctx->stream>>>(in.b, in.nbr, in.links, wout, codes, c, cnext,
                                                                      ctx->kappa, theta, partial, ctx->V, nrhs,
                                                                      first_step, nullptr, 0, nullptr, a, alpha, beta);
    }
}

// One fused step; with a != nullptr the combining form
// wout = alpha a + beta (w - c M w) (a may be w, must not be wout).
int wilson_dot_step(mpmc_ctx *ctx, const void *w, void *wout, const uint32_t *codes, int nrhs, int prec, double2 c,
                    double2 cnext, int theta, double *partial, int first_step, const void *a, double2 alpha,
                    double2 beta) {
    if (nrhs % 64 != 0 || (nrhs > 256 && nrhs % 256 != 0))
        return set_err(ctx, MPMC_EINVAL, "fused level step needs nrhs %% 64 == 0 (and %% 256 above 256)");
    if (a && a == wout) return set_err(ctx, MPMC_EINVAL, "fused level step: a aliases the output");
    if (!w || !wout || !codes || !partial || w == wout)
        return set_err(ctx, MPMC_EINVAL, "fused level step: null or aliased operand");
    const long work = ctx->V * nrhs;
    const unsigned grid = grid_for(work, 256);
    const int dord = dot_order(ctx, nrhs, prec);
    const int ev = timing_begin(ctx);
    if (prec == MPMC_FP64) {
        const WIn<MPMC_FP64> in = make_in<MPMC_FP64>(ctx, w, nrhs);
        if (a)
            launch_dot<MPMC_FP64, true>(ctx, dord, grid, in, wout, codes, c, cnext, theta, (double2 *)partial, nrhs,
                                        first_step, a, alpha, beta);
        else
            launch_dot<MPMC_FP64, false>(ctx, dord, grid, in, wout, codes, c, cnext, theta, (double2 *)partial, nrhs,
                                         first_step, nullptr, alpha, beta);
    } else if (prec == MPMC_FP32) {
        const WIn<MPMC_FP32> in = make_in<MPMC_FP32>(ctx, w, nrhs);
        if (a)
            launch_dot<MPMC_FP32, true>(ctx, dord, grid, in, wout, codes, c, cnext, theta, (double2 *)partial, nrhs,
                                        first_step, a, alpha, beta);
        else
            launch_dot<MPMC_FP32, false>(ctx, dord, grid, in, wout, codes, c, cnext, theta, (double2 *)partial, nrhs,
                                         first_step, nullptr, alpha, beta);
    }
    else
        return set_err(ctx, MPMC_EINVAL, "fused level step supports FP64 and FP32");
    HIP_OR_RET(ctx, hipGetLastError());
    if (ev >= 0) {
        // spinor read + write (+ the read of a), 4-byte noise code, links once
        // per site (the partial sums add 16 B per 256 threads and are not counted)
        const double per = (a ? 3 : 2) * spinor_bytes(prec) + 4.0;
        timing_end(ctx, ev, prec | MPMC_TIMING_FUSED, (double)ctx->V * ((double)nrhs * per + link_bytes(prec)));
    }
    ctx->mvps += (uint64_t)nrhs;
    return MPMC_OK;
}

// Fused step over several recurrences side by side (the blocked 64-wide
// traversal): right-hand sides [0, nact) of operands with stride nrhs, chunk
// q's coefficients at coef_dev[2q], coef_dev[2q + 1]; partial as for
// wilson_dot_step with nrhs (chunks at or beyond nact keep their sums).
int wilson_dot_step_multi(mpmc_ctx *ctx, const void *w, void *wout, const uint32_t *codes, int nrhs, int nact,
                          int prec, const double *coef_dev, int theta, double *partial, int first_step) {
    if (ctx->V % 4 != 0 || nrhs % 64 != 0 || nact % 64 != 0 || nact < 64 || nact > nrhs)
        return set_err(ctx, MPMC_EINVAL, "several recurrences need V %% 4 == 0 and 64-wide chunks");
    const unsigned grid = (unsigned)(ctx->V * nact / 256);
    const double2 *cf = (const double2 *)coef_dev;
    const int ev = timing_begin(ctx);
    if (prec == MPMC_FP64) {
        const WIn<MPMC_FP64> in = make_in<MPMC_FP64>(ctx, w, nrhs);
        k_wilson_dot<MPMC_FP64, 2, true><<<grid, 256, 0, ctx->stream>>>(
            in.b, in.nbr, in.links, wout, codes, make_double2(0, 0), make_double2(0, 0), ctx->kappa, theta,
            (double2 *)partial, ctx->V, nrhs, first_step, ctx->site_order, nact, cf);
    } else if (prec == MPMC_FP32) {
        const WIn<MPMC_FP32> in = make_in<MPMC_FP32>(ctx, w, nrhs);
        k_wilson_dot<MPMC_FP32, 2, true><<<grid, 256, 0, ctx->stream>>>(
            in.b, in.nbr, in.links, wout, codes, make_double2(0, 0), make_double2(0, 0), ctx->kappa, theta,
            (double2 *)partial, ctx->V, nrhs, first_step, ctx->site_order, nact, cf);
    } else {
        return set_err(ctx, MPMC_EINVAL, "fused level step supports FP64 and FP32");
    }
    HIP_OR_RET(ctx, hipGetLastError());
    if (ev >= 0) {
        const double per = 2 * spinor_bytes(prec) + 4.0;
        timing_end(ctx, ev, prec | MPMC_TIMING_FUSED, (double)ctx->V * ((double)nact * per + link_bytes(prec)));
    }
    ctx->mvps += (uint64_t)nact;
    return MPMC_OK;
}

// Sums of the blocked 64-wide partials for right-hand sides [0, nrhs) (the
// several-recurrence step's layout).
int wilson_dot_finish_chunks(mpmc_ctx *ctx, const double *partial, int nrhs, double *out) {
    k_dot_finish_chunk<<<nrhs, 256, 0, ctx->stream>>>((const double2 *)partial, ctx->V * 64 / 256, 64, (double2 *)out,
                                                      0, 1.0);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

int wilson_dot_finish(mpmc_ctx *ctx, const double *partial, int nrhs, int prec, double *out, int accumulate,
                      double sign) {
    const long blocks = (ctx->V * nrhs + 255) / 256;
    const int dord = dot_order(ctx, nrhs, prec);
    if (dord) {
        const int wd = dot_width(dord, nrhs);
        k_dot_finish_chunk<<<nrhs, 256, 0, ctx->stream>>>((const double2 *)partial,
                                                          dot_tiles_per_chunk(ctx, dord, wd), wd, (double2 *)out,
                                                          accumulate, sign);
    } else
        k_dot_finish<<<nrhs, 256, 0, ctx->stream>>>((const double2 *)partial, (int)blocks, nrhs, (double2 *)out,
                                                    accumulate, sign);
    HIP_OR_RET(ctx, hipGetLastError());
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

// ------------------------------------------------------ batched apply --

template <int P>
static int launch_batch(mpmc_ctx *const *ctxs, const void *const *x, void *const *y, int count, int nrhs,
                        int dagger, int theta) {
    mpmc_ctx *c0 = ctxs[0];
    BatchArgs<P> a{};
    a.count = count;
    unsigned tiles = 0;
    double bytes = 0;
    for (int i = 0; i < count; ++i) {
        const mpmc_ctx *c = ctxs[i];
        LatticeArgs<P> &L = a.l[i];
        L.b = vref(c, x[i], nrhs, P).d;
        L.out = y[i];
        L.nbr = c->nbr;
        L.links = reinterpret_cast<const typename LinkT<P>::type *>(P == MPMC_FP64 ? (const void *)c->links64
                                                                                   : (const void *)c->links32);
        L.order = c->site_order;
        L.V = c->V;
        L.kappa = c->kappa;
        L.tile0 = tiles;
        tiles += (unsigned)(c->V * nrhs / 256);
        bytes += (double)c->V * ((double)nrhs * 2 * spinor_bytes(P) + link_bytes(P));
    }
    const int ev = timing_begin(c0);
    k_wilson_batch<P><<<tiles, 256, 0, c0->stream>>>(a, nrhs, dagger ? -1.f : 1.f, theta);
    HIP_OR_RET(c0, hipGetLastError());
    if (ev >= 0) timing_end(c0, ev, P | MPMC_TIMING_PLAIN, bytes);
    for (int i = 0; i < count; ++i) ctxs[i]->mvps += (uint64_t)nrhs;
    return MPMC_OK;
}

MPMC_API int mpmc_apply_M_batch(mpmc_ctx *const *ctxs, const void *const *x, void *const *y, int count, int nrhs,
                                int prec, int dagger, int theta) {
    if (!ctxs || !ctxs[0]) return MPMC_EINVAL;
    mpmc_ctx *c0 = ctxs[0];
    if (!x || !y || count < 1 || count > WILSON_BATCH_MAX)
        return set_err(c0, MPMC_EINVAL, "mpmc_apply_M_batch: 1..%d lattices", WILSON_BATCH_MAX);
    if (nrhs < 64 || nrhs % 64 != 0 || (prec != MPMC_FP64 && prec != MPMC_FP32) ||
        (theta != MPMC_THETA_I && theta != MPMC_THETA_G5))
        return set_err(c0, MPMC_EINVAL, "mpmc_apply_M_batch: nrhs must be a multiple of 64, prec FP64 or FP32");
    long total = 0;
    for (int i = 0; i < count; ++i) {
        const mpmc_ctx *c = ctxs[i];
        if (!c || !x[i] || !y[i] || x[i] == y[i] || c->device != c0->device || c->V % 4 != 0)
            return set_err(c0, MPMC_EINVAL, "mpmc_apply_M_batch: lattice %d: null, aliasing, other device or V %% 4 != 0", i);
        total += c->V * nrhs;
    }
    if (total / 256 > 0x7fffffffL) return set_err(c0, MPMC_EINVAL, "mpmc_apply_M_batch: batch too large");
    return prec == MPMC_FP64 ? launch_batch<MPMC_FP64>(ctxs, x, y, count, nrhs, dagger, theta)
                             : launch_batch<MPMC_FP32>(ctxs, x, y, count, nrhs, dagger, theta);
}

// ------------------------------------------------------------ autotuner --

MPMC_API int mpmc_wilson_variant_count(void) { return WILSON_VARIANTS; }

MPMC_API int mpmc_tune_set(mpmc_ctx *ctx, int nrhs, int prec, int variant) {
    if (!ctx) return MPMC_EINVAL;
    if (nrhs < 1 || !prec_ok(prec) || variant < -1 || variant >= WILSON_VARIANTS)
        return set_err(ctx, MPMC_EINVAL, "mpmc_tune_set: bad argument");
    const auto key = std::make_pair(nrhs, prec);
    if (variant < 0) {
        ctx->tune.erase(key);
        ctx->tune_explicit.erase(key);
    } else {
        ctx->tune[key] = variant;
        ctx->tune_explicit[key] = variant;
    }
    return MPMC_OK;
}

MPMC_API int mpmc_autotune(mpmc_ctx *ctx, int nrhs, int prec, int *variant_host, double *us_host) {
    if (!ctx) return MPMC_EINVAL;
    if (nrhs < 1 || !prec_ok(prec)) return set_err(ctx, MPMC_EINVAL, "mpmc_autotune: bad argument");
    if (us_host)
        for (int v = 0; v < WILSON_VARIANTS; ++v) us_host[v] = 0.0;
    if (nrhs % 64 != 0 || ctx->V * (long)nrhs > 0x7fffff00L) {   // one kernel shape only
        if (variant_host) *variant_host = -1;
        return MPMC_OK;
    }
    Scratch S(ctx);
    const size_t vb = vec_bytes(ctx, nrhs, prec);
    void *x = S.get(vb), *y = S.get(vb);
    if (!x || !y) return MPMC_ENOMEM;
    RET_IF(launch_noise(ctx, 1, 0, 0, nrhs, prec, x));
    hipEvent_t e0, e1;
    HIP_OR_RET(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_err(ctx, MPMC_EHIP, "mpmc_autotune: event creation failed");
    }
    const int timing = ctx->timing;
    const uint64_t mvps = ctx->mvps;
    ctx->timing = 0;
    const auto key = std::make_pair(nrhs, prec);
    int best = default_variant(ctx, nrhs, prec), rc = MPMC_OK;
    double best_us = 1e300;
    constexpr int warm = 2, reps = 5;
    for (int v = 0; v < WILSON_VARIANTS && rc == MPMC_OK; ++v) {
        ctx->tune[key] = v;
        if (wilson_variant(ctx, nrhs, prec) != v) continue;   // falls back to another variant on this shape
        for (int i = 0; i < warm + reps && rc == MPMC_OK; ++i) {
            if (i == warm && hipEventRecord(e0, ctx->stream) != hipSuccess) rc = MPMC_EHIP;
            if (rc == MPMC_OK)
                rc = wilson_launch_full(ctx, x, nullptr, y, nullptr, nrhs, prec, make_double2(0, 0), make_double2(1, 0),
                                        make_double2(0, 0), 0, 0);
        }
        float ms = 0.f;
        if (rc == MPMC_OK && (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = set_err(ctx, MPMC_EHIP, "mpmc_autotune: timing failed");
        const double us = 1e3 * ms / reps;
        if (us_host) us_host[v] = us;
        if (rc == MPMC_OK && us < best_us) {
            best_us = us;
            best = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->timing = timing;
    ctx->mvps = mvps;
    ctx->tune[key] = best;
    if (rc != MPMC_OK) return rc;
    if (variant_host) *variant_host = best;
    return MPMC_OK;
}

// Fused level step traversal (orders 0 site-major, 2 blocked 64-wide chunks,
// 3 / 4 blocked 16- / 32-wide chunks, 5 / 6 / 7 column streaming with 2x2x2 /
// 2x2x1 / 2x2x4 tiles): each valid one is timed (2 warm-up + 5 timed steps,
// best of three rounds) and the fastest kept for (nrhs, prec).
MPMC_API int mpmc_autotune_level(mpmc_ctx *ctx, int nrhs, int prec, int *order_host, double *us_host) {
    if (!ctx) return MPMC_EINVAL;
    if ((prec != MPMC_FP64 && prec != MPMC_FP32) || nrhs < 64 || nrhs % 64 != 0 || (nrhs > 256 && nrhs % 256 != 0))
        return set_err(ctx, MPMC_EINVAL, "mpmc_autotune_level: FP64/FP32 and nrhs %% 64 == 0 (%% 256 above 256)");
    if (us_host)
        for (int o = 0; o < kDotOrders; ++o) us_host[o] = 0.0;
    Scratch S(ctx);
    const size_t vb = vec_bytes(ctx, nrhs, prec);
    void *x = S.get(vb), *y = S.get(vb);
    uint32_t *codes = (uint32_t *)S.get(sizeof(uint32_t) * (size_t)ctx->V * nrhs);
    double *part = (double *)S.get(sizeof(double2) * wilson_dot_partial_count(ctx, nrhs));
    if (!x || !y || !codes || !part) return MPMC_ENOMEM;
    RET_IF(launch_noise(ctx, 1, 0, 0, nrhs, prec, x));
    RET_IF(wilson_noise_codes(ctx, 1, 0, 0, nrhs, codes));
    hipEvent_t e0, e1;
    HIP_OR_RET(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_err(ctx, MPMC_EHIP, "mpmc_autotune_level: event creation failed");
    }
    const int timing = ctx->timing;
    const uint64_t mvps = ctx->mvps;
    ctx->timing = 0;
    const auto key = std::make_pair(nrhs, prec);
    const auto ex = ctx->tune_explicit.find(key);
    const bool had_ex = ex != ctx->tune_explicit.end();
    const int ex_v = had_ex ? ex->second : 0;
    ctx->tune_explicit.erase(key);
    std::vector<int> cand = {0};
    if (ctx->V % 4 == 0) cand.push_back(2);
    if (ctx->V % 16 == 0) {
        cand.push_back(3);
        cand.push_back(4);
    }
    if (col_ok(ctx, nrhs, prec) && nrhs <= 256) cand.push_back(kDotColumn);
    if (col_ok(ctx, nrhs, prec, 1) && nrhs <= 256) cand.push_back(kDotColumn1);
    if (col_ok(ctx, nrhs, prec, 4) && nrhs <= 256) cand.push_back(kDotColumnP);
    int best = cand.back(), rc = MPMC_OK;
    double best_us = 1e300;
    // candidates timed in three interleaved rounds, each keeping its best
    // round: traversals a percent apart are then told apart reliably
    constexpr int warm = 2, reps = 5, rounds = 3;
    std::vector<double> us_min(cand.size(), 1e300);
    for (int round = 0; round < rounds && rc == MPMC_OK; ++round)
        for (size_t q = 0; q < cand.size() && rc == MPMC_OK; ++q) {
            ctx->tune_dot[key] = cand[q];
            for (int i = 0; i < warm + reps && rc == MPMC_OK; ++i) {
                if (i == warm && hipEventRecord(e0, ctx->stream) != hipSuccess) rc = MPMC_EHIP;
                if (rc == MPMC_OK)
                    rc = wilson_dot_step(ctx, (i & 1) ? y : x, (i & 1) ? x : y, codes, nrhs, prec,
                                         make_double2(0.1, 0), make_double2(0.1, 0), 0, part, i == 0);
            }
            float ms = 0.f;
            if (rc == MPMC_OK &&
                (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = set_err(ctx, MPMC_EHIP, "mpmc_autotune_level: timing failed");
            us_min[q] = std::min(us_min[q], 1e3 * ms / reps);
        }
    for (size_t q = 0; q < cand.size() && rc == MPMC_OK; ++q) {
        if (us_host) us_host[cand[q]] = us_min[q];
        if (us_min[q] < best_us) {
            best_us = us_min[q];
            best = cand[q];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->timing = timing;
    ctx->mvps = mvps;
    ctx->tune_dot[key] = best;
    if (had_ex) ctx->tune_explicit[key] = ex_v;
    if (rc != MPMC_OK) return rc;
    if (order_host) *order_host = best;
    return MPMC_OK;
}
