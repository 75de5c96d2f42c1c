// GMRES polynomials (Sec. 3) and double polynomials (Sec. 5).
//
// mpmc_gmres_poly runs one GMRES(d) cycle on the device: d Arnoldi steps with
// classical Gram-Schmidt applied twice (two fused dot/update passes per step,
// FP64 sums), breakdown detection on the device (no host round trip per
// step), then the harmonic Ritz values and their Leja order in one FP64
// one-workgroup kernel.  mpmc_apply_poly evaluates
//     p(M) x = sum_k w_k / theta_k,  w_1 = x,  w_{k+1} = w_k - M w_k / theta_k
// with one fused Wilson kernel per step (w update and y accumulation in the
// same pass), and the double polynomial as p_in(M) [p_out(phi_in(M)) x].
#include <cmath>
#include <complex>

#include <algorithm>
#include <string>

#include "common.h"

// ------------------------------------------------------------ Arnoldi --

__global__ void k_arnoldi_init(double *state, double2 *scale, const double2 *nrm2) {
    state[0] = 0.0;
    state[1] = -1.0;
    const double b = sqrt(fmax(nrm2[0].x, 0.0));
    scale[0] = make_double2(b > 0 ? 1.0 / b : 0.0, 0.0);
    state[2] = b;
}

struct OpDesc {
    const mpmc_poly *inner;   // nullptr: M; else phi_in(M) = M p_in(M)
    const mpmc_defl *defl;    // project each new vector with Q = I - Z U^H
    int prec;                 // storage of the Arnoldi vectors (FP64 or FP32; scalars are FP64)
};

static int apply_op(mpmc_ctx *ctx, const OpDesc &op, const void *x, void *y) {
    Scratch S(ctx);
    if (!op.inner) {
        RET_IF(wilson_launch_full(ctx, x, nullptr, y, nullptr, 1, op.prec, make_double2(0, 0),
                                  make_double2(1, 0), make_double2(0, 0), 0, 0));
    } else {
        void *t = S.get(vec_bytes(ctx, 1, op.prec));
        if (!t) return MPMC_ENOMEM;
        RET_IF(poly_apply_internal(ctx, op.inner, x, t, 1, op.prec));
        RET_IF(wilson_launch_full(ctx, t, nullptr, y, nullptr, 1, op.prec, make_double2(0, 0),
                                  make_double2(1, 0), make_double2(0, 0), 0, 0));
    }
    if (op.defl) RET_IF(project_any(ctx, op.defl, y, op.prec));
    return MPMC_OK;
}

// ------------------------------------ delayed reorthogonalisation --
// Classical Gram-Schmidt applied twice, with the second projection of each
// Arnoldi vector delayed by one step (the low-synchronisation "DCGS2" form of
// Swirydowicz, Langou, Ananthan, Yang and Thomas, and of Bielich et al.): at
// step j the operator is applied to the not yet reorthogonalised candidate u
// (z = A u), one pass over the basis V_j gives every inner product of the
// step (s = V_j^H u, t = V_j^H z, u^H u, u^H z), a one-workgroup kernel turns
// them into the final column j-1 of H, the single-projection column j and the
// coefficients of
//     v_j    = (u - V_j s) / nu,                nu = sqrt(u^H u - |s|^2),
//     u_next = (z - V_j (t - s c / nu) - u c / nu) / nu,   c = (u^H z - s^H t) / nu,
// and one more pass over V_j writes both vectors.  In exact arithmetic this is
// the CGS2 Arnoldi process (A V_j = V_{j+1} H_j gives A v_j from z without a
// second operator application); each step reads the basis twice instead of
// four times and issues four launches besides the operator instead of eight.

constexpr int kDcgsJB = 8;   // basis vectors per workgroup row of the dot pass

__device__ __forceinline__ double2 wave_sum2(double2 v) {
    for (int o = 32; o > 0; o >>= 1) {
        v.x += __shfl_xor(v.x, o);
        v.y += __shfl_xor(v.y, o);
    }
    return v;
}

// partial[q * NB + blk]: q < nv: V_q^H u; nv <= q < 2 nv: V_{q-nv}^H z (z may be
// null: zero); q = 2 nv: u^H u; q = 2 nv + 1: u^H z.  Row g = blockIdx.y of the
// grid takes basis vectors [g JB, g JB + JB); row 0 also the two u products.
// Used above kDcgsRunMaxV basis vectors; the run form below otherwise.
template <int P>
__global__ __launch_bounds__(256) void k_dcgs_dots(const void *__restrict__ V, size_t vstep, int nv,
                                                   const void *__restrict__ u, const void *__restrict__ z, long n,
                                                   double2 *__restrict__ partial, int NB) {
    __shared__ double2 red[2 * kDcgsJB + 2][4];
    const int j0 = blockIdx.y * kDcgsJB;
    cpx<double> sa[kDcgsJB], ta[kDcgsJB], aa = mk(0.0, 0.0), ba = mk(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < kDcgsJB; ++q) sa[q] = ta[q] = mk(0.0, 0.0);
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)NB * 256) {
        const auto u0 = Store<P>::ld(u, nullptr, e, 0);
        const cpx<double> uv = mk((double)u0.re, (double)u0.im);
        cpx<double> zv = mk(0.0, 0.0);
        if (z) {
            const auto z0 = Store<P>::ld(z, nullptr, e, 0);
            zv = mk((double)z0.re, (double)z0.im);
        }
        if (blockIdx.y == 0) {
            aa = aa + conjmul(uv, uv);
            ba = ba + conjmul(uv, zv);
        }
        cpx<double> vq[kDcgsJB];
#pragma unroll
        for (int q = 0; q < kDcgsJB; ++q) {   // loads issued together, index clamped, masked below
            const int i = j0 + q < nv ? j0 + q : (nv > 0 ? nv - 1 : 0);
            const auto v = nv > 0 ? Store<P>::ld((const char *)V + (size_t)i * vstep, nullptr, e, 0)
                                  : Store<P>::ld(u, nullptr, e, 0);
            vq[q] = mk((double)v.re, (double)v.im);
        }
#pragma unroll
        for (int q = 0; q < kDcgsJB; ++q)
            if (j0 + q < nv) {
                sa[q] = sa[q] + conjmul(vq[q], uv);
                ta[q] = ta[q] + conjmul(vq[q], zv);
            }
    }
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < kDcgsJB; ++q) {
        const double2 a = wave_sum2(make_double2(sa[q].re, sa[q].im));
        const double2 b = wave_sum2(make_double2(ta[q].re, ta[q].im));
        if (ln == 0) {
            red[q][wv] = a;
            red[kDcgsJB + q][wv] = b;
        }
    }
    const double2 a2 = wave_sum2(make_double2(aa.re, aa.im)), b2 = wave_sum2(make_double2(ba.re, ba.im));
    if (ln == 0) {
        red[2 * kDcgsJB][wv] = a2;
        red[2 * kDcgsJB + 1][wv] = b2;
    }
    __syncthreads();
    if (threadIdx.x < 2 * kDcgsJB + 2) {
        const int q = threadIdx.x;
        double2 acc = red[q][0];
        for (int w = 1; w < 4; ++w) {
            acc.x += red[q][w].x;
            acc.y += red[q][w].y;
        }
        long out = -1;
        if (q < kDcgsJB) {
            if (j0 + q < nv) out = j0 + q;
        } else if (q < 2 * kDcgsJB) {
            if (j0 + q - kDcgsJB < nv) out = nv + j0 + q - kDcgsJB;
        } else if (blockIdx.y == 0) {
            out = 2L * nv + (q - 2 * kDcgsJB);
        }
        if (out >= 0) partial[out * NB + blockIdx.x] = acc;
    }
}

// The same products with the element range split instead of the basis: a
// workgroup owns S 16-byte slots per thread (slot k of thread i at k*256 + i
// of the workgroup's run, so every load instruction is contiguous over the
// wavefront), holds its run of u and z in registers, and streams all nv basis
// vectors over it.  u and z are read once per step (the row form above reads
// them once per group of kDcgsJB vectors); per-wavefront sums wait in LDS
// until one barrier at the end.  A 16-byte slot holds two FP32 or one FP64
// complex element.
constexpr int kDcgsRunMaxV = 256;   // basis vectors the LDS of the run form holds

template <int P>
struct Slot;
template <>
struct Slot<MPMC_FP32> {   // two complex elements, kept as stored, widened at use
    using raw = float4;
    static constexpr int per = 2;
    __device__ static cpx<double> el(const float4 &w, int e) {
        return e == 0 ? mk((double)w.x, (double)w.y) : mk((double)w.z, (double)w.w);
    }
};
template <>
struct Slot<MPMC_FP64> {
    using raw = double2;
    static constexpr int per = 1;
    __device__ static cpx<double> el(const double2 &w, int) { return mk(w.x, w.y); }
};

template <int P, int S>
__global__ __launch_bounds__(256) void k_dcgs_dots_run(const void *__restrict__ V, size_t vstep, int nv,
                                                       const void *__restrict__ u, const void *__restrict__ z,
                                                       long nslots, double2 *__restrict__ partial, int NB) {
    using R = typename Slot<P>::raw;
    constexpr int E = Slot<P>::per;
    __shared__ double2 red[2 * kDcgsRunMaxV + 2][4];
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const long base = (long)blockIdx.x * 256 * S + threadIdx.x;
    R ur[S], zr[S];
    cpx<double> aa = mk(0.0, 0.0), ba = mk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const long sl = base + (long)k * 256;
        const bool in = sl < nslots;
        ur[k] = in ? reinterpret_cast<const R *>(u)[sl] : R{};
        zr[k] = in && z ? reinterpret_cast<const R *>(z)[sl] : R{};
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const cpx<double> ue = Slot<P>::el(ur[k], e), ze = Slot<P>::el(zr[k], e);
            aa = aa + conjmul(ue, ue);
            ba = ba + conjmul(ue, ze);
        }
    }
    for (int q = 0; q < nv; ++q) {
        const R *vq = reinterpret_cast<const R *>((const char *)V + (size_t)q * vstep);
        R vr[S];
#pragma unroll
        for (int k = 0; k < S; ++k) {   // loads issued together
            const long sl = base + (long)k * 256;
            vr[k] = sl < nslots ? vq[sl] : R{};
        }
        cpx<double> sa = mk(0.0, 0.0), ta = mk(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < S; ++k)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const cpx<double> ve = Slot<P>::el(vr[k], e);
                sa = sa + conjmul(ve, Slot<P>::el(ur[k], e));
                ta = ta + conjmul(ve, Slot<P>::el(zr[k], e));
            }
        const double2 a = wave_sum2(make_double2(sa.re, sa.im));
        const double2 b = wave_sum2(make_double2(ta.re, ta.im));
        if (ln == 0) {
            red[q][wv] = a;
            red[nv + q][wv] = b;
        }
    }
    const double2 a2 = wave_sum2(make_double2(aa.re, aa.im)), b2 = wave_sum2(make_double2(ba.re, ba.im));
    if (ln == 0) {
        red[2 * nv][wv] = a2;
        red[2 * nv + 1][wv] = b2;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * nv + 2; q += 256) {
        double2 acc = red[q][0];
        for (int w = 1; w < 4; ++w) {
            acc.x += red[q][w].x;
            acc.y += red[q][w].y;
        }
        partial[(long)q * NB + blockIdx.x] = acc;
    }
}

// D[q] = sum_b partial[q * NB + b] (fixed order), one workgroup per q.
__global__ __launch_bounds__(256) void k_dcgs_reduce(const double2 *__restrict__ partial, int NB,
                                                     double2 *__restrict__ D) {
    __shared__ double2 red[4];
    const int q = blockIdx.x;
    double2 a = make_double2(0.0, 0.0);
    for (int b = threadIdx.x; b < NB; b += 256) {
        const double2 v = partial[(long)q * NB + b];
        a.x += v.x;
        a.y += v.y;
    }
    a = wave_sum2(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double2 t = red[0];
        for (int w = 1; w < 4; ++w) {
            t.x += red[w].x;
            t.y += red[w].y;
        }
        D[q] = t;
    }
}

__device__ __forceinline__ double block_sum1(double v, double *red4) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = v;
    __syncthreads();
    return red4[0] + red4[1] + red4[2] + red4[3];
}

// Coefficients of step j from D (k_dcgs_reduce; nv = j basis vectors): the
// final column j-1 of H (H(0:j-1, j-1) += s, H(j, j-1) = nu, breakdown test as
// in CGS2: nu <= 1e-14 ||H||_F), then (unless last) the single-projection
// column j and C = [1/nu, -c/nu^2, 1/nu, -s_i/nu (i < j), -(t_i - s_i c/nu)/nu
// (i < j)].  After a breakdown every coefficient is 0 (later vectors stay 0).
// j = 0 also records ||b|| = nu in state[2].  ldh = d + 1; j <= d <= 500.
__global__ __launch_bounds__(256) void k_dcgs_coef(const double2 *__restrict__ D, int j, int ldh,
                                                   double2 *__restrict__ H, double *__restrict__ state,
                                                   double2 *__restrict__ C, int last) {
    __shared__ double2 sv[512], tv[512];
    __shared__ double red4[4];
    __shared__ double sh_nu;
    __shared__ int sh_bad;
    const int tid = threadIdx.x;
    for (int i = tid; i < j; i += 256) {
        sv[i] = D[i];
        tv[i] = D[j + i];
    }
    __syncthreads();
    const double2 a = D[2 * j], b = D[2 * j + 1];
    double ss = 0.0, stre = 0.0, stim = 0.0;
    for (int i = tid; i < j; i += 256) {
        ss += sv[i].x * sv[i].x + sv[i].y * sv[i].y;
        stre += sv[i].x * tv[i].x + sv[i].y * tv[i].y;   // s^H t
        stim += sv[i].x * tv[i].y - sv[i].y * tv[i].x;
    }
    ss = block_sum1(ss, red4);
    stre = block_sum1(stre, red4);
    stim = block_sum1(stim, red4);
    const double nu = sqrt(fmax(a.x - ss, 0.0));
    // the final column j-1 and its share of the running Frobenius norm
    double col = 0.0;
    if (j > 0) {
        double2 *Hc = H + (size_t)(j - 1) * ldh;
        for (int i = tid; i < j; i += 256) {
            double2 h = Hc[i];
            h.x += sv[i].x;
            h.y += sv[i].y;
            Hc[i] = h;
            col += h.x * h.x + h.y * h.y;
        }
    }
    col = block_sum1(col, red4);
    if (tid == 0) {
        bool bad = state[1] >= 0 || !(nu == nu);
        if (j == 0) {
            state[2] = nu;
            if (!(nu > 0)) bad = true;
        } else {
            const double fro = state[0] + col + nu * nu;
            state[0] = fro;
            if (!bad && nu <= 1e-14 * sqrt(fro)) bad = true;
            if (bad && state[1] < 0) state[1] = j;
            H[(size_t)(j - 1) * ldh + j] = make_double2(bad ? 0.0 : nu, 0.0);
        }
        if (bad && j == 0 && state[1] < 0) state[1] = 0;
        sh_nu = nu;
        sh_bad = bad ? 1 : 0;
    }
    __syncthreads();
    const bool bad = sh_bad != 0;
    const double inu = bad ? 0.0 : 1.0 / sh_nu;
    // c = v_j^H z = (u^H z - s^H t) / nu
    const cpx<double> c = mk((b.x - stre) * inu, (b.y - stim) * inu);
    if (tid == 0) {
        C[0] = make_double2(inu, 0.0);
        C[1] = make_double2(-c.re * inu * inu, -c.im * inu * inu);
        C[2] = make_double2(last ? 0.0 : inu, 0.0);
    }
    for (int i = tid; i < j; i += 256) {
        C[3 + i] = make_double2(-sv[i].x * inu, -sv[i].y * inu);
        // t_i - s_i c / nu
        const double r = tv[i].x - (sv[i].x * c.re - sv[i].y * c.im) * inu;
        const double m = tv[i].y - (sv[i].x * c.im + sv[i].y * c.re) * inu;
        C[3 + j + i] = make_double2(last ? 0.0 : -r * inu, last ? 0.0 : -m * inu);
    }
    if (last) return;
    // single-projection column j: h_i = (t_i - g_i) / nu (i < j), h_j = (c - g_j) / nu,
    // g = H(0:j, 0:j-1) s.  Row i per thread, all k: the entries below the
    // subdiagonal are zero (H starts zeroed), so the loop bound is uniform and
    // the loads of one k are one coalesced column segment.
    double2 *Hj = H + (size_t)j * ldh;
    for (int i = tid; i <= j; i += 256) {
        double gr = 0.0, gi = 0.0;
#pragma unroll 8
        for (int k = 0; k < j; ++k) {
            const double2 h = H[(size_t)k * ldh + i];
            gr += h.x * sv[k].x - h.y * sv[k].y;
            gi += h.x * sv[k].y + h.y * sv[k].x;
        }
        const double2 tt = i < j ? tv[i] : make_double2(c.re, c.im);
        Hj[i] = make_double2((tt.x - gr) * inu, (tt.y - gi) * inu);
    }
}

// vout = C0 u + sum_i C[3+i] V_i ; un = C1 u + C2 z + sum_i C[3+nv+i] V_i (un may
// alias u, vout may alias u; z and un may be null), over 16-byte slots (two
// FP32 or one FP64 complex element per load), eight basis vectors' loads in
// flight per iteration.
template <int P>
__device__ __forceinline__ void slot_cpx(const typename Slot<P>::raw &w, cpx<typename Store<P>::real> x[Slot<P>::per]) {
    if constexpr (P == MPMC_FP32) {
        x[0] = mk(w.x, w.y);
        x[1] = mk(w.z, w.w);
    } else {
        x[0] = mk(w.x, w.y);
    }
}
template <int P>
__device__ __forceinline__ typename Slot<P>::raw cpx_slot(const cpx<typename Store<P>::real> x[Slot<P>::per]) {
    if constexpr (P == MPMC_FP32) return make_float4(x[0].re, x[0].im, x[1].re, x[1].im);
    else return make_double2(x[0].re, x[0].im);
}

template <int P>
__global__ __launch_bounds__(256) void k_dcgs_update_run(const void *__restrict__ V, size_t vstep, int nv,
                                                         const void *u, const void *__restrict__ z, void *un,
                                                         void *vout, const double2 *__restrict__ C, long nslots) {
    using T = typename Store<P>::real;
    using R = typename Slot<P>::raw;
    constexpr int E = Slot<P>::per;
    constexpr int G = 8;
    const cpx<T> cu = mk((T)C[0].x, (T)C[0].y), bu = mk((T)C[1].x, (T)C[1].y), bz = mk((T)C[2].x, (T)C[2].y);
    for (long sl = (long)blockIdx.x * 256 + threadIdx.x; sl < nslots; sl += (long)gridDim.x * 256) {
        cpx<T> uv[E], v[E], w[E];
        slot_cpx<P>(reinterpret_cast<const R *>(u)[sl], uv);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            v[e] = cu * uv[e];
            w[e] = bu * uv[e];
        }
        if (z) {
            cpx<T> zv[E];
            slot_cpx<P>(reinterpret_cast<const R *>(z)[sl], zv);
#pragma unroll
            for (int e = 0; e < E; ++e) w[e] = w[e] + bz * zv[e];
        }
        int i = 0;
        for (; i + G <= nv; i += G) {
            R vr[G];
#pragma unroll
            for (int q = 0; q < G; ++q) vr[q] = reinterpret_cast<const R *>((const char *)V + (size_t)(i + q) * vstep)[sl];
#pragma unroll
            for (int q = 0; q < G; ++q) {
                cpx<T> x[E];
                slot_cpx<P>(vr[q], x);
                const double2 a = C[3 + i + q], bb = C[3 + nv + i + q];
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    v[e] = v[e] + mk((T)a.x, (T)a.y) * x[e];
                    w[e] = w[e] + mk((T)bb.x, (T)bb.y) * x[e];
                }
            }
        }
        for (; i < nv; ++i) {
            cpx<T> x[E];
            slot_cpx<P>(reinterpret_cast<const R *>((const char *)V + (size_t)i * vstep)[sl], x);
            const double2 a = C[3 + i], bb = C[3 + nv + i];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                v[e] = v[e] + mk((T)a.x, (T)a.y) * x[e];
                w[e] = w[e] + mk((T)bb.x, (T)bb.y) * x[e];
            }
        }
        if (un) reinterpret_cast<R *>(un)[sl] = cpx_slot<P>(w);
        reinterpret_cast<R *>(vout)[sl] = cpx_slot<P>(v);
    }
}

static int dcgs_launch_dots(mpmc_ctx *ctx, int prec, const void *V, size_t vstep, int nv, const void *u,
                            const void *z, double2 *D) {
    const long n = ctx->n;
    if (nv <= kDcgsRunMaxV) {
        // run form: 8 (FP64) or 4 (FP32) slots per thread where that still gives
        // two workgroups per compute unit (126 and 112 VGPRs), else 2
        const long nslots = prec == MPMC_FP64 ? n : n / 2;   // n = 12 V is even
        const int Sbig = prec == MPMC_FP64 ? 8 : 4;
        const int S = (nslots + 256L * Sbig - 1) / (256L * Sbig) >= 2L * ctx->num_cu ? Sbig : 2;
        const int NB = (int)((nslots + 256L * S - 1) / (256L * S));
        double2 *part = (double2 *)ws_get(ctx, WS_PARTIAL, (size_t)(2 * nv + 2) * NB * sizeof(double2));
        if (!part) return MPMC_ENOMEM;
        if (prec == MPMC_FP64) {
            if (S == 8) k_dcgs_dots_run<MPMC_FP64, 8><<<NB, 256, 0, ctx->stream>>>(V, vstep, nv, u, z, nslots, part, NB);
            else k_dcgs_dots_run<MPMC_FP64, 2><<<NB, 256, 0, ctx->stream>>>(V, vstep, nv, u, z, nslots, part, NB);
        } else {
            if (S == 4) k_dcgs_dots_run<MPMC_FP32, 4><<<NB, 256, 0, ctx->stream>>>(V, vstep, nv, u, z, nslots, part, NB);
            else k_dcgs_dots_run<MPMC_FP32, 2><<<NB, 256, 0, ctx->stream>>>(V, vstep, nv, u, z, nslots, part, NB);
        }
        HIP_OR_RET(ctx, hipGetLastError());
        k_dcgs_reduce<<<2 * nv + 2, 256, 0, ctx->stream>>>(part, NB, D);
        HIP_OR_RET(ctx, hipGetLastError());
        return MPMC_OK;
    }
    const int groups = nv > 0 ? (nv + kDcgsJB - 1) / kDcgsJB : 1;
    long nb = (long)ctx->num_cu * 8 / groups;
    const long maxnb = (n + 255) / 256;
    if (nb < 8) nb = 8;
    if (nb > maxnb) nb = maxnb;
    if (nb > 2048) nb = 2048;
    const int NB = (int)nb;
    double2 *part = (double2 *)ws_get(ctx, WS_PARTIAL, (size_t)(2 * nv + 2) * NB * sizeof(double2));
    if (!part) return MPMC_ENOMEM;
    if (prec == MPMC_FP64)
        k_dcgs_dots<MPMC_FP64><<<dim3(NB, groups), 256, 0, ctx->stream>>>(V, vstep, nv, u, z, n, part, NB);
    else
        k_dcgs_dots<MPMC_FP32><<<dim3(NB, groups), 256, 0, ctx->stream>>>(V, vstep, nv, u, z, n, part, NB);
    HIP_OR_RET(ctx, hipGetLastError());
    k_dcgs_reduce<<<2 * nv + 2, 256, 0, ctx->stream>>>(part, NB, D);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

static int dcgs_launch_update(mpmc_ctx *ctx, int prec, const void *V, size_t vstep, int nv, const void *u,
                              const void *z, void *un, void *vout, const double2 *C) {
    const long n = ctx->n;
    const long nslots = prec == MPMC_FP64 ? n : n / 2;   // 16-byte slots; n = 12 V is even
    long nb = (nslots + 255) / 256;
    if (nb > (long)ctx->num_cu * 8) nb = (long)ctx->num_cu * 8;
    if (prec == MPMC_FP64)
        k_dcgs_update_run<MPMC_FP64><<<(unsigned)nb, 256, 0, ctx->stream>>>(V, vstep, nv, u, z, un, vout, C, nslots);
    else
        k_dcgs_update_run<MPMC_FP32><<<(unsigned)nb, 256, 0, ctx->stream>>>(V, vstep, nv, u, z, un, vout, C, nslots);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// d Arnoldi steps (one rhs) from b (overwritten by v_0), vectors stored in
// op.prec.  V: (d+1) vectors of n complex elements, H: column-major (d+1) x d
// FP64, ld = d+1.  state (device): [0] ||H||_F^2, [1] d_eff or -1, [2] ||b||.
static int arnoldi_run_cgs2(mpmc_ctx *ctx, const OpDesc &op, void *V, double *H, int d, double *state,
                            Scratch &S) {
    const long n = ctx->n;
    const size_t vstep = vec_bytes(ctx, 1, op.prec);
    double2 *sc = (double2 *)S.get(sizeof(double2) * (d + 8));
    double2 *h2 = (double2 *)S.get(sizeof(double2) * (d + 8));
    void *w = S.get(vstep);
    if (!sc || !h2 || !w) return MPMC_ENOMEM;
    HIP_OR_RET(ctx, hipMemsetAsync(H, 0, sizeof(double2) * (size_t)(d + 1) * d, ctx->stream));
    if (op.defl) RET_IF(project_any(ctx, op.defl, V, op.prec));
    RET_IF(blas_norm2(ctx, V, 1, op.prec, (double *)sc));
    k_arnoldi_init<<<1, 1, 0, ctx->stream>>>(state, sc + 1, sc);
    HIP_OR_RET(ctx, hipGetLastError());
    RET_IF(blas_scale_rhs(ctx, V, V, 1, op.prec, (double *)(sc + 1), 0));
    for (int j = 0; j < d; ++j) {
        void *vj = (char *)V + (size_t)j * vstep;
        void *vj1 = (char *)V + (size_t)(j + 1) * vstep;
        double *Hcol = H + 2 * (size_t)j * (d + 1);
        RET_IF(apply_op(ctx, op, vj, w));
        // CGS pass 1: H(:, j) = V^H w ; w -= V H(:, j)
        RET_IF(blas_multi_dot(ctx, V, n, 1, j + 1, w, 1, op.prec, Hcol, 0, 0));
        RET_IF(blas_multi_axpy(ctx, V, n, 1, j + 1, w, 1, op.prec, Hcol, 1, -1.0, nullptr));
        // CGS pass 2; the norm's reduction also finishes the column (breakdown test, 1/h)
        RET_IF(blas_multi_dot(ctx, V, n, 1, j + 1, w, 1, op.prec, (double *)h2, 0, 0));
        RET_IF(blas_arnoldi_update(ctx, V, n, j + 1, w, (double *)h2, Hcol, j, state, (double *)(sc + 1), op.prec));
        RET_IF(blas_scale_rhs(ctx, w, vj1, 1, op.prec, (double *)(sc + 1), 0));
    }
    return MPMC_OK;
}

__global__ void k_dcgs_init(double *state) {
    state[0] = 0.0;
    state[1] = -1.0;
    state[2] = 0.0;
}

// The same process with the delayed second projection (see k_dcgs_dots): per
// step the operator on the candidate u, one dot pass, the coefficient kernel,
// one update pass; after the last step the candidate's delayed projection
// completes column d-1 and v_d.
static int arnoldi_run_dcgs2(mpmc_ctx *ctx, const OpDesc &op, void *V, double *H, int d, double *state,
                             Scratch &S) {
    const size_t vstep = vec_bytes(ctx, 1, op.prec);
    void *u = S.get(vstep), *z = S.get(vstep);
    double2 *D = (double2 *)S.get(sizeof(double2) * (size_t)(2 * d + 4));
    double2 *C = (double2 *)S.get(sizeof(double2) * (size_t)(2 * d + 4));
    if (!u || !z || !D || !C) return MPMC_ENOMEM;
    if (d > 500) return set_err(ctx, MPMC_EINVAL, "Arnoldi: at most 500 steps");
    HIP_OR_RET(ctx, hipMemsetAsync(H, 0, sizeof(double2) * (size_t)(d + 1) * d, ctx->stream));
    k_dcgs_init<<<1, 1, 0, ctx->stream>>>(state);
    HIP_OR_RET(ctx, hipGetLastError());
    if (op.defl) RET_IF(project_any(ctx, op.defl, V, op.prec));
    for (int j = 0; j < d; ++j) {
        const void *cur = j == 0 ? V : u;   // the candidate for v_j (the start vector at j = 0)
        RET_IF(apply_op(ctx, op, cur, z));
        RET_IF(dcgs_launch_dots(ctx, op.prec, V, vstep, j, cur, z, D));
        k_dcgs_coef<<<1, 256, 0, ctx->stream>>>(D, j, d + 1, (double2 *)H, state, C, 0);
        HIP_OR_RET(ctx, hipGetLastError());
        RET_IF(dcgs_launch_update(ctx, op.prec, V, vstep, j, cur, z, u, (char *)V + (size_t)j * vstep, C));
    }
    RET_IF(dcgs_launch_dots(ctx, op.prec, V, vstep, d, u, nullptr, D));
    k_dcgs_coef<<<1, 256, 0, ctx->stream>>>(D, d, d + 1, (double2 *)H, state, C, 1);
    HIP_OR_RET(ctx, hipGetLastError());
    return dcgs_launch_update(ctx, op.prec, V, vstep, d, u, nullptr, nullptr, (char *)V + (size_t)d * vstep, C);
}

// Automatic choice: on small lattices the step is launch-bound and the
// shorter kernels of plain CGS2 win (8^4: GMRES(129) 9.3 against 11.7 ms);
// from 16^4 sites on the step is bound by the basis passes and the delayed
// form wins (24^4 FP32: 217 against 160 ms).
constexpr long kDelayedGsMinV = 65536;

int arnoldi_run(mpmc_ctx *ctx, const OpDesc &op, void *V, double *H, int d, double *state, Scratch &S) {
    const bool plain = ctx->gs_cgs2 == 1 || (ctx->gs_cgs2 < 0 && ctx->V < kDelayedGsMinV);
    return plain ? arnoldi_run_cgs2(ctx, op, V, H, d, state, S) : arnoldi_run_dcgs2(ctx, op, V, H, d, state, S);
}

MPMC_API int mpmc_set_arnoldi_cgs2(mpmc_ctx *ctx, int on) {
    if (!ctx) return MPMC_EINVAL;
    if (on < -1 || on > 1) return set_err(ctx, MPMC_EINVAL, "mpmc_set_arnoldi_cgs2: -1, 0 or 1");
    ctx->gs_cgs2 = on;
    return MPMC_OK;
}

// ---------------------------------------------------------- handles --

static int validate_poly(const mpmc_ctx *ctx, const mpmc_poly *p) {
    if (!p) return set_err(ctx, MPMC_EINVAL, "null polynomial");
    if (p->ctx != ctx) return set_err(ctx, MPMC_ESTATE, "polynomial belongs to another context");
    if (p->inner && p->inner->inner) return set_err(ctx, MPMC_EINVAL, "only double (not triple) polynomials");
    return MPMC_OK;
}

int poly_validate(const mpmc_ctx *ctx, const mpmc_poly *p) { return validate_poly(ctx, p); }

int poly_matvecs(const mpmc_poly *p) {
    if (!p->inner) return p->d - 1;
    return (p->d - 1) * p->inner->d + (p->inner->d - 1);
}

static std::complex<double> eval_single(const std::vector<double> &roots, int d, std::complex<double> lam) {
    std::complex<double> w(1.0, 0.0);
    std::complex<double> th0(roots[0], roots[1]);
    std::complex<double> y = w / th0;
    for (int k = 0; k + 1 < d; ++k) {
        std::complex<double> th(roots[2 * k], roots[2 * k + 1]);
        std::complex<double> thn(roots[2 * k + 2], roots[2 * k + 3]);
        w = w * (1.0 - lam / th);
        y += w / thn;
    }
    return y;
}

void poly_eval_host(const mpmc_poly *p, const double *lam, double *out, int k) {
    for (int i = 0; i < k; ++i) {
        std::complex<double> l(lam[2 * i], lam[2 * i + 1]), v;
        if (!p->inner) {
            v = eval_single(p->roots, p->d, l);
        } else {
            std::complex<double> pin = eval_single(p->inner->roots, p->inner->d, l);
            v = pin * eval_single(p->roots, p->d, l * pin);
        }
        out[2 * i] = v.real();
        out[2 * i + 1] = v.imag();
    }
}

MPMC_API int mpmc_poly_create(mpmc_ctx *ctx, const double *roots_host, int d, const mpmc_poly *inner,
                              mpmc_poly **out) {
    if (!ctx) return MPMC_EINVAL;
    if (!roots_host || d < 1 || !out) return set_err(ctx, MPMC_EINVAL, "mpmc_poly_create: bad argument");
    if (inner) RET_IF(validate_poly(ctx, inner));
    if (inner && inner->inner) return set_err(ctx, MPMC_EINVAL, "mpmc_poly_create: inner must be single");
    for (int i = 0; i < d; ++i)
        if (!(std::isfinite(roots_host[2 * i]) && std::isfinite(roots_host[2 * i + 1])) ||
            (roots_host[2 * i] == 0 && roots_host[2 * i + 1] == 0))
            return set_err(ctx, MPMC_EINVAL, "mpmc_poly_create: root %d is zero or not finite", i);
    mpmc_poly *p = new mpmc_poly();
    p->ctx = ctx;
    p->d = d;
    p->roots.assign(roots_host, roots_host + 2 * d);
    p->inner = inner;
    *out = p;
    return MPMC_OK;
}

MPMC_API int mpmc_poly_add_roots(mpmc_poly *p, double log10_threshold, double digits, int *added_host) {
    if (!p || !p->ctx) return MPMC_EINVAL;
    mpmc_ctx *ctx = const_cast<mpmc_ctx *>(p->ctx);
    if (!(digits > 0) || !std::isfinite(log10_threshold))
        return set_err(ctx, MPMC_EINVAL, "mpmc_poly_add_roots: bad argument");
    const int d = p->d, max_out = std::min(2 * d + 16, 1200);
    Scratch S(ctx);
    double *in = (double *)S.get(sizeof(double) * 2 * d);
    double *out = (double *)S.get(sizeof(double) * 2 * max_out);
    int *cnt = (int *)S.get(sizeof(int) * 4);
    if (!in || !out || !cnt) return MPMC_ENOMEM;
    HIP_OR_RET(ctx, hipMemcpyAsync(in, p->roots.data(), sizeof(double) * 2 * d, hipMemcpyHostToDevice, ctx->stream));
    RET_IF(dense_add_roots(ctx, in, d, log10_threshold, digits, max_out, out, cnt));
    int total = 0;
    HIP_OR_RET(ctx, hipMemcpyAsync(&total, cnt, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    if (total < 0) return set_err(ctx, MPMC_EINVAL, "mpmc_poly_add_roots: more than %d roots", max_out);
    std::vector<double> r(2 * (size_t)total);
    HIP_OR_RET(ctx, hipMemcpyAsync(r.data(), out, sizeof(double) * 2 * total, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    if (added_host) *added_host = total - d;
    p->roots = r;
    p->d = total;
    return MPMC_OK;
}

MPMC_API int mpmc_poly_roots(const mpmc_poly *p, double *roots_host, int *d) {
    if (!p || !d) return MPMC_EINVAL;
    if (roots_host) {
        if (*d < p->d) return set_err(p->ctx, MPMC_EINVAL, "mpmc_poly_roots: capacity %d < %d", *d, p->d);
        for (int i = 0; i < 2 * p->d; ++i) roots_host[i] = p->roots[i];
    }
    *d = p->d;
    return MPMC_OK;
}

MPMC_API int mpmc_poly_info(const mpmc_poly *p, int *d, int *d_inner, int *degree, int *matvecs) {
    if (!p) return MPMC_EINVAL;
    if (d) *d = p->d;
    if (d_inner) *d_inner = p->inner ? p->inner->d : 0;
    if (degree) *degree = p->inner ? p->inner->d * p->d - 1 : p->d - 1;
    if (matvecs) *matvecs = poly_matvecs(p);
    return MPMC_OK;
}

MPMC_API int mpmc_poly_eval(const mpmc_poly *p, const double *lam_host, double *out_host, int k) {
    if (!p || (k > 0 && (!lam_host || !out_host)) || k < 0) return MPMC_EINVAL;
    poly_eval_host(p, lam_host, out_host, k);
    return MPMC_OK;
}

MPMC_API void mpmc_poly_destroy(mpmc_poly *p) { delete p; }

// ------------------------------------------------------ gmres_poly --

MPMC_API int mpmc_gmres_poly(mpmc_ctx *ctx, const mpmc_poly *inner, const mpmc_defl *defl, uint64_t seed,
                             uint32_t stream, int d, mpmc_poly **out, int *d_eff, double *relres) {
    if (!ctx) return MPMC_EINVAL;
    if (!out || d < 1 || d > 500) return set_err(ctx, MPMC_EINVAL, "mpmc_gmres_poly: bad argument (d=%d)", d);
    if (inner) RET_IF(validate_poly(ctx, inner));
    if (inner && inner->inner) return set_err(ctx, MPMC_EINVAL, "mpmc_gmres_poly: inner must be a single polynomial");
    if (defl && defl->ctx != ctx) return set_err(ctx, MPMC_ESTATE, "deflation set belongs to another context");
    *out = nullptr;
    Scratch S(ctx);
    const long n = ctx->n;
    const int prec = ctx->setup_prec;
    void *V = S.get(vec_bytes(ctx, 1, prec) * (size_t)(d + 1));
    double *H = (double *)S.get(sizeof(double2) * (size_t)(d + 1) * d);
    double *state = (double *)S.get(sizeof(double) * 8);
    double *roots = (double *)S.get(sizeof(double2) * (d + 2));
    double *info = (double *)S.get(sizeof(double) * 4);
    if (!V || !H || !state || !roots || !info) return MPMC_ENOMEM;
    (void)n;
    RET_IF(launch_noise(ctx, seed, stream, 0, 1, prec, V));
    OpDesc op{inner, (defl && defl->k > 0) ? defl : nullptr, prec};
    RET_IF(arnoldi_run(ctx, op, V, H, d, state, S));
    double hs[3];
    HIP_OR_RET(ctx, hipMemcpyAsync(hs, state, sizeof hs, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    const int de = hs[1] >= 0 ? (int)hs[1] : d;
    const double beta = hs[2];
    if (!(beta > 0)) return set_err(ctx, MPMC_ENUMERIC, "mpmc_gmres_poly: zero start vector");
    RET_IF(dense_harmonic_leja(ctx, H, d + 1, de, beta, roots, info));
    std::vector<double> r(2 * de);
    double inf[2];
    HIP_OR_RET(ctx, hipMemcpyAsync(r.data(), roots, sizeof(double) * 2 * de, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_RET(ctx, hipMemcpyAsync(inf, info, sizeof inf, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    if (inf[1] != 0) return set_err(ctx, MPMC_ENUMERIC, "mpmc_gmres_poly: small eigenproblem failed (%g)", inf[1]);
    mpmc_poly *p = new mpmc_poly();
    p->ctx = ctx;
    p->d = de;
    p->roots = r;
    p->inner = inner;
    *out = p;
    if (d_eff) *d_eff = de;
    if (relres) *relres = de < d ? 0.0 : inf[0];
    return MPMC_OK;
}

// ------------------------------------------------------ apply_poly --

// y = p(M) x for a single polynomial with caller-provided work vectors wa, wb
// (each vec_bytes(ctx, nrhs, prec), distinct from x and y).
static int apply_single_buf(mpmc_ctx *ctx, const std::vector<double> &roots, int d, const void *x, void *y,
                            int nrhs, int prec, void *wa, void *wb) {
    auto th = [&](int k) { return std::complex<double>(roots[2 * k], roots[2 * k + 1]); };
    auto inv = [&](int k) {
        std::complex<double> v = 1.0 / th(k);
        return make_double2(v.real(), v.imag());
    };
    // y = x / theta_1 (single vectors: inside the first step's launch)
    const bool fold = nrhs == 1 && d > 1;
    if (!fold) RET_IF(blas_axpby(ctx, x, y, nrhs, prec, inv(0), make_double2(0, 0)));
    if (d == 1) return MPMC_OK;
    const void *cur = x;
    for (int k = 0; k + 1 < d; ++k) {
        void *nxt = (cur == wa) ? wb : wa;
        double2 c = inv(k);
        RET_IF(wilson_launch_full(ctx, cur, cur, nxt, y, nrhs, prec, make_double2(1, 0), make_double2(-c.x, -c.y),
                                  inv(k + 1), 0, 0, inv(0), fold && k == 0));
        cur = nxt;
    }
    return MPMC_OK;
}

static int apply_single(mpmc_ctx *ctx, const std::vector<double> &roots, int d, const void *x, void *y, int nrhs,
                        int prec) {
    Scratch S(ctx);
    void *wa = S.get(vec_bytes(ctx, nrhs, prec));
    void *wb = S.get(vec_bytes(ctx, nrhs, prec));
    if (!wa || !wb) return MPMC_ENOMEM;
    return apply_single_buf(ctx, roots, d, x, y, nrhs, prec, wa, wb);
}

int poly_work_vectors(const mpmc_poly *p) { return p->inner ? 6 : 2; }

// y = p(M) x with the poly_work_vectors(p) work vectors buf[i] supplied by the caller.
int poly_apply_buf(mpmc_ctx *ctx, const mpmc_poly *p, const void *x, void *y, int nrhs, int prec, void *const *buf) {
    if (prec != MPMC_FP64 && prec != MPMC_FP32)
        return set_err(ctx, MPMC_EINVAL, "polynomial application supports FP64 and FP32 storage");
    if (!p->inner) return apply_single_buf(ctx, p->roots, p->d, x, y, nrhs, prec, buf[0], buf[1]);
    // u = p_out(phi_in) x : u = x/v_1, w_{k+1} = w_k - phi(w_k)/v_k, phi(w) = M p_in(M) w
    void *u = buf[0], *t = buf[1], *wa = buf[2], *wb = buf[3];
    auto inv = [&](int k) {
        std::complex<double> v = 1.0 / std::complex<double>(p->roots[2 * k], p->roots[2 * k + 1]);
        return make_double2(v.real(), v.imag());
    };
    RET_IF(blas_axpby(ctx, x, u, nrhs, prec, inv(0), make_double2(0, 0)));
    const void *cur = x;
    for (int k = 0; k + 1 < p->d; ++k) {
        void *nxt = (cur == wa) ? wb : wa;
        RET_IF(apply_single_buf(ctx, p->inner->roots, p->inner->d, cur, t, nrhs, prec, buf[4], buf[5]));
        double2 c = inv(k);
        RET_IF(wilson_launch_full(ctx, t, cur, nxt, u, nrhs, prec, make_double2(1, 0), make_double2(-c.x, -c.y),
                                  inv(k + 1), 0, 0));
        cur = nxt;
    }
    return apply_single_buf(ctx, p->inner->roots, p->inner->d, u, y, nrhs, prec, buf[4], buf[5]);
}

int poly_apply_internal(mpmc_ctx *ctx, const mpmc_poly *p, const void *x, void *y, int nrhs, int prec) {
    if (prec != MPMC_FP64 && prec != MPMC_FP32)
        return set_err(ctx, MPMC_EINVAL, "polynomial application supports FP64 and FP32 storage");
    Scratch S(ctx);
    const size_t vb = vec_bytes(ctx, nrhs, prec);
    void *buf[6];
    for (int i = 0; i < poly_work_vectors(p); ++i)
        if (!(buf[i] = S.get(vb))) return MPMC_ENOMEM;
    return poly_apply_buf(ctx, p, x, y, nrhs, prec, buf);
}

MPMC_API int mpmc_apply_poly(mpmc_ctx *ctx, const mpmc_poly *p, const void *x, void *y, int nrhs, int prec) {
    if (!ctx) return MPMC_EINVAL;
    RET_IF(validate_poly(ctx, p));
    if (!x || !y || nrhs < 1) return set_err(ctx, MPMC_EINVAL, "mpmc_apply_poly: bad argument");
    if (x == y) return set_err(ctx, MPMC_EINVAL, "mpmc_apply_poly: x and y must not alias");
    return poly_apply_internal(ctx, p, x, y, nrhs, prec);
}

// Arnoldi on M (inner == nullptr) or on phi_in(M) = M p_in(M), for the deflation build.
int arnoldi_run_ext(mpmc_ctx *ctx, const mpmc_poly *inner, void *V, double *H, int d, double *state, Scratch &S,
                    int prec) {
    OpDesc op{inner, nullptr, prec};
    return arnoldi_run(ctx, op, V, H, d, state, S);
}

MPMC_API int mpmc_set_setup_precision(mpmc_ctx *ctx, int prec) {
    if (!ctx) return MPMC_EINVAL;
    if (prec != MPMC_FP64 && prec != MPMC_FP32)
        return set_err(ctx, MPMC_EINVAL, "mpmc_set_setup_precision: FP64 or FP32");
    ctx->setup_prec = prec;
    return MPMC_OK;
}

// ------------------------------------------------- fused quadratic form --
// acc[r] += sign * eta_r^H Theta p(M) eta_r.  For p = p_in(M) p_out(phi_in) the
// outer factor u = p_out(phi_in) eta is formed explicitly and the inner single
// polynomial is fused: sum_k eta^H Theta w_k / theta_k with w_1 = u.

bool poly_quad_fusable(int nrhs) { return nrhs % 64 == 0 && (nrhs <= 256 || nrhs % 256 == 0); }

// ------------------------------------------------ captured recurrences --
// With mpmc_set_graph_recurrences the launch sequence of a fused recurrence is
// captured once into a hipGraph on the context's capture stream and replayed
// afterwards.  The key holds everything the launches depend on: operand,
// work-vector, code and partial-sum addresses, shape, precision, Theta, the
// traversal and the coefficients (roots), so a replay issues exactly the
// launches an eager run would.  Only kernel launches are captured.

void graphs_clear(mpmc_ctx *ctx) {
    for (auto &g : ctx->graphs) hipGraphExecDestroy(g.second);
    ctx->graphs.clear();
}

template <typename T>
static void key_put(std::string &k, const T &v) {
    k.append(reinterpret_cast<const char *>(&v), sizeof(T));
}

template <typename F>
static int run_recurrence(mpmc_ctx *ctx, const std::string &key, uint64_t mvps, F &&steps) {
    if (!ctx->use_graphs || ctx->timing || !ctx->gstream) return steps();
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        hipStream_t s0 = ctx->stream;
        ctx->stream = ctx->gstream;
        if (hipStreamBeginCapture(ctx->gstream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            ctx->stream = s0;
            return steps();
        }
        const uint64_t mv0 = ctx->mvps;
        const int rc = steps();
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(ctx->gstream, &g);
        ctx->stream = s0;
        ctx->mvps = mv0;
        if (rc != MPMC_OK || e != hipSuccess || !g) {
            if (g) hipGraphDestroy(g);
            if (rc != MPMC_OK) return rc;
            return set_err(ctx, MPMC_EHIP, "recurrence capture failed: %s", hipGetErrorString(e));
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (ei != hipSuccess) return set_err(ctx, MPMC_EHIP, "graph instantiation: %s", hipGetErrorString(ei));
        it = ctx->graphs.emplace(key, ex).first;
    }
    // replay on the capture stream, after the context stream's earlier work and before its later work
    HIP_OR_RET(ctx, hipEventRecord(ctx->gev[0], ctx->stream));
    HIP_OR_RET(ctx, hipStreamWaitEvent(ctx->gstream, ctx->gev[0], 0));
    HIP_OR_RET(ctx, hipGraphLaunch(it->second, ctx->gstream));
    HIP_OR_RET(ctx, hipEventRecord(ctx->gev[1], ctx->gstream));
    HIP_OR_RET(ctx, hipStreamWaitEvent(ctx->stream, ctx->gev[1], 0));
    ctx->mvps += mvps;
    ctx->graph_replays++;
    return MPMC_OK;
}

MPMC_API int mpmc_set_graph_recurrences(mpmc_ctx *ctx, int on) {
    if (!ctx) return MPMC_EINVAL;
    if (on != 0 && on != 1) return set_err(ctx, MPMC_EINVAL, "mpmc_set_graph_recurrences: on must be 0 or 1");
    if (on && !ctx->gstream) {
        HIP_OR_RET(ctx, hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking));
        HIP_OR_RET(ctx, hipEventCreateWithFlags(&ctx->gev[0], hipEventDisableTiming));
        HIP_OR_RET(ctx, hipEventCreateWithFlags(&ctx->gev[1], hipEventDisableTiming));
    }
    ctx->use_graphs = on;
    return MPMC_OK;
}

MPMC_API int mpmc_graph_replays(const mpmc_ctx *ctx, uint64_t *replays_host, int *graphs_host) {
    if (!ctx) return MPMC_EINVAL;
    if (replays_host) *replays_host = ctx->graph_replays;
    if (graphs_host) *graphs_host = (int)ctx->graphs.size();
    return MPMC_OK;
}

static int quad_single_fused(mpmc_ctx *ctx, const std::vector<double> &roots, int d, const void *eta, const void *x,
                             const uint32_t *codes, int nrhs, int prec, int theta, double *acc, double sign) {
    Scratch S(ctx);
    auto inv = [&](int k) {
        std::complex<double> v = 1.0 / std::complex<double>(roots[2 * k], roots[2 * k + 1]);
        return make_double2(v.real(), v.imag());
    };
    // first term (1/theta_1) eta^H Theta x
    double2 *t = (double2 *)S.get(sizeof(double2) * nrhs * 2);
    if (!t) return MPMC_ENOMEM;
    RET_IF(blas_dot(ctx, eta, x, nrhs, prec, theta, (double *)t));
    RET_IF(blas_scale_acc(ctx, (double *)t, nrhs, inv(0), sign, acc));
    if (d == 1) return MPMC_OK;
    void *wa = S.get(vec_bytes(ctx, nrhs, prec));
    void *wb = S.get(vec_bytes(ctx, nrhs, prec));
    double *part = (double *)S.get(sizeof(double2) * wilson_dot_partial_count(ctx, nrhs));
    if (!wa || !wb || !part) return MPMC_ENOMEM;
    std::string key("s");
    for (const void *q : {(const void *)x, (const void *)wa, (const void *)wb, (const void *)codes, (const void *)part})
        key_put(key, q);
    for (int v : {d, nrhs, prec, theta, wilson_dot_order(ctx, nrhs, prec)}) key_put(key, v);
    key.append(reinterpret_cast<const char *>(roots.data()), sizeof(double) * 2 * d);
    RET_IF(run_recurrence(ctx, key, (uint64_t)(d - 1) * nrhs, [&]() -> int {
        const void *cur = x;
        for (int k = 0; k + 1 < d; ++k) {
            void *nxt = (cur == wa) ? wb : wa;
            RET_IF(wilson_dot_step(ctx, cur, nxt, codes, nrhs, prec, inv(k), inv(k + 1), theta, part, k == 0));
            cur = nxt;
        }
        return MPMC_OK;
    }));
    return wilson_dot_finish(ctx, part, nrhs, prec, acc, 1, sign);
}

int poly_quad_fused(mpmc_ctx *ctx, const mpmc_poly *p, const void *eta, const uint32_t *codes, int nrhs, int prec,
                    int theta, double *acc, double sign) {
    if (!poly_quad_fusable(nrhs)) return set_err(ctx, MPMC_EINVAL, "fused quadratic form needs nrhs %% 64 == 0");
    if (!p->inner) return quad_single_fused(ctx, p->roots, p->d, eta, eta, codes, nrhs, prec, theta, acc, sign);
    // Double polynomial (Sec. 5): p(M) = p_in(M) p_out(phi(M)), phi = M p_in(M) = 1 - pi_in(M).
    // With the outer recurrence w_0 = eta, w_{k+1} = w_k - phi(w_k) / th_k^out and the
    // inner one v_0 = w_k, v_{j+1} = v_j - M v_j / th_j^in:
    //   eta^H Theta p(M) eta = sum_k (1/th_k^out) sum_{j < d_in} (1/th_j^in) eta^H Theta v_{k,j},
    //   phi(w_k) = w_k - v_{k,d_in},  so  w_{k+1} = (1 - 1/th_k^out) w_k + (1/th_k^out) v_{k,d_in}.
    // Every step is one fused launch (one spinor read and write; the step that
    // yields v_{k,d_in} also reads w_k and writes w_{k+1} directly), and every
    // term of the quadratic form is accumulated inside those launches.
    Scratch S(ctx);
    const size_t vb = vec_bytes(ctx, nrhs, prec);
    void *buf[3] = {S.get(vb), S.get(vb), S.get(vb)};
    double2 *t = (double2 *)S.get(sizeof(double2) * nrhs * 2);
    double *part = (double *)S.get(sizeof(double2) * wilson_dot_partial_count(ctx, nrhs));
    if (!buf[0] || !buf[1] || !buf[2] || !t || !part) return MPMC_ENOMEM;
    const mpmc_poly *pin = p->inner;
    const int din = pin->d, dout = p->d;
    auto cx = [](const std::vector<double> &r, int k) { return std::complex<double>(r[2 * k], r[2 * k + 1]); };
    auto d2 = [](std::complex<double> v) { return make_double2(v.real(), v.imag()); };
    auto io = [&](int k) { return 1.0 / cx(p->roots, k); };
    auto ii = [&](int j) { return 1.0 / cx(pin->roots, j); };
    // first term (k = 0, j = 0): eta^H Theta eta / (th_0^out th_0^in)
    RET_IF(blas_dot(ctx, eta, eta, nrhs, prec, theta, (double *)t));
    RET_IF(blas_scale_acc(ctx, (double *)t, nrhs, d2(io(0) * ii(0)), sign, acc));
    const int nsteps_total = (dout - 1) * din + (din - 1);
    if (nsteps_total == 0) return MPMC_OK;
    std::string key("d");
    for (const void *q : {(const void *)eta, (const void *)buf[0], (const void *)buf[1], (const void *)buf[2],
                          (const void *)codes, (const void *)part})
        key_put(key, q);
    for (int v : {din, dout, nrhs, prec, theta, wilson_dot_order(ctx, nrhs, prec)}) key_put(key, v);
    key.append(reinterpret_cast<const char *>(pin->roots.data()), sizeof(double) * 2 * din);
    key.append(reinterpret_cast<const char *>(p->roots.data()), sizeof(double) * 2 * dout);
    RET_IF(run_recurrence(ctx, key, (uint64_t)nsteps_total * nrhs, [&]() -> int {
        const void *w = eta;   // w_k
        bool first = true;
        for (int k = 0; k < dout; ++k) {
            const bool last_outer = k == dout - 1;
            const int nsteps = last_outer ? din - 1 : din;
            const void *v = w;
            for (int j = 0; j < nsteps; ++j) {
                void *dst = nullptr;
                for (void *c : buf)
                    if (c != w && c != v) {
                        dst = c;
                        break;
                    }
                const double2 c = d2(ii(j));
                if (!last_outer && j == din - 1) {
                    // v_{k,d_in} combined into w_{k+1}; accumulates the first term of step k + 1
                    RET_IF(wilson_dot_step(ctx, v, dst, codes, nrhs, prec, c, d2(io(k + 1) * ii(0)), theta, part,
                                           first, w, d2(1.0 - io(k)), d2(io(k))));
                    w = dst;
                } else {
                    RET_IF(wilson_dot_step(ctx, v, dst, codes, nrhs, prec, c, d2(io(k) * ii(j + 1)), theta, part,
                                           first));
                    v = dst;
                }
                first = false;
            }
        }
        return MPMC_OK;
    }));
    return wilson_dot_finish(ctx, part, nrhs, prec, acc, 1, sign);
}
