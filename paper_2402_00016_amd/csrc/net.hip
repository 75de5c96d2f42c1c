// Learned right preconditioner of the main solves (not part of the paper):
// a gauge-covariant linear network of three parallel-transport layers with
// 1 -> 2 -> 2 -> 1 spinor fields,
//
//     out(x)[f', s', c] = sum_p sum_{f, s} W_p[(f', s'), (f, s)] (T_p in)(x)[f, s, c],
//
// over the 9 paths p = 0 (identity), 1..4 = +mu (U_mu(x) in(x+mu)) and
// 5..8 = -mu (U_mu(x-mu)^H in(x-mu)), with the time-boundary sign of the
// Wilson operator on hops that cross it.  W_p acts on (field, spin) and as the
// identity on colour, so the network commutes with gauge transformations and
// is a fixed linear operator: inside flexible GMRES it can change the cost of
// a solve, never its converged solution.
//
// Kernels (gfx950):
//   k_net_layer  -- one layer.  A wavefront owns one site and 16 right-hand
//                   sides; per path its lanes transport the neighbour's
//                   spinors (VALU, FP32, links from the scalar cache) and the
//                   (field, spin) contraction runs on MFMA
//                   (v_mfma_f32_16x16x16_bf16: BF16 weights and transported
//                   inputs, FP32 accumulation), one MFMA per colour and path.
//                   The same kernel computes the data gradient of a layer:
//                   since T_{+mu}^H = T_{-mu} and W_p commutes with T_p, the
//                   adjoint layer is a forward layer with weights
//                   W'_q = (W_{q~})^H, q~ swapping +mu and -mu.
//   k_net_wgrad  -- weight gradient dL/dW_p^* = sum_{x, rhs, c} g(x) conj(T_p a(x))
//                   as MFMAs with the right-hand sides as the contraction
//                   index; per-wavefront partials, summed in a fixed order.
//   k_net_loss, k_net_adam, k_net_pack -- loss and output gradient, Adam,
//                   and the BF16 operand tables built from the FP32 master
//                   weights.
// Activations are FP32 internal-layout batches [site][field*12 + spin*3 + c][rhs].
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int NPATH = 9;
constexpr int NPARAM = 2304;
constexpr int FIELDS[4] = {1, 2, 2, 1};
constexpr int LAYER_OFF[4] = {0, 576, 1728, 2304};   // real parameters before layer l
constexpr int TABLE_ELEMS = NPATH * 64 * 4;          // bf16 A-operand table of one layer op
constexpr int WGRAD_BLOCKS = 1024;                   // blocks (4 wavefronts each) of the weight-gradient grid

__device__ __forceinline__ short to_bf16(float f) {
    return __builtin_bit_cast(short, (__bf16)f);
}

typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float f32x2v __attribute__((ext_vector_type(2)));

// two packed conversions (round to nearest even, as to_bf16), no permutes
__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
    const bf16x2v lo = __builtin_convertvector((f32x2v){a, b}, bf16x2v);
    const bf16x2v hi = __builtin_convertvector((f32x2v){c, d}, bf16x2v);
    const uint64_t u = (uint64_t)__builtin_bit_cast(uint32_t, lo) | ((uint64_t)__builtin_bit_cast(uint32_t, hi) << 32);
    return __builtin_bit_cast(bf16x4, u);
}

// A-operand tables.  Op 2l is the forward map of layer l, op 2l+1 its adjoint.
// For the MFMA D[i][n] = sum_k A[i][k] B[k][n] of one path, row i = 2o + ro is
// output complex channel o = field*4 + spin (ro: real/imag part) and
// k = 2 ci + ri the input channel ci = field*4 + spin of that path; lane l
// holds A[l % 16][4 (l / 16) + j], j < 4.  The complex product in real form:
//   [Re o]   [ Re w  -Im w ] [Re t]
//   [Im o] = [ Im w   Re w ] [Im t]
__global__ void k_net_pack(const float *__restrict__ theta, short *__restrict__ tables) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * TABLE_ELEMS) return;
    const int op = t / TABLE_ELEMS;
    const int rem = t - op * TABLE_ELEMS;
    const int p = rem / 256, lane = (rem / 4) % 64, j = rem % 4;
    const int layer = op >> 1, adj = op & 1;
    const int fin = FIELDS[layer], fout = FIELDS[layer + 1];
    const int i = lane % 16, k = 4 * (lane / 16) + j;
    const int o = i >> 1, ro = i & 1, ci = k >> 1, ri = k & 1;
    // op output / input channel counts
    const int nout = 4 * (adj ? fin : fout), nin = 4 * (adj ? fout : fin);
    float v = 0.f;
    if (o < nout && ci < nin) {
        // weight W_q[o][ci] of the op; the adjoint uses conj(W_{q~}[ci][o])
        int q = p, row = o, col = ci;
        float sg = 1.f;
        if (adj) {
            q = p == 0 ? 0 : (p <= 4 ? p + 4 : p - 4);
            row = ci;
            col = o;
            sg = -1.f;
        }
        const int base = LAYER_OFF[layer] + 2 * ((q * 4 * fout + row) * 4 * fin + col);
        const float wr = theta[base], wi = sg * theta[base + 1];
        v = (ro == ri) ? wr : (ro == 0 ? -wi : wi);
    }
    tables[t] = to_bf16(v);
}

template <typename T>
__device__ __forceinline__ T uni(T v) {
    return __builtin_amdgcn_readfirstlane(v);
}

// Transport of two spins (s0, s0+1) x 3 colours of field f from the path's
// source site into t[2][3] (lanes with !act produce zeros).
struct PathSrc {
    long src;
    float sgn;
    const float2 *U;   // null for the identity path
    bool dag;
};

// nbw: the site's eight neighbour words, lane i holding entry i & 7 (one load
// per wavefront instead of one dependent load per path).
__device__ __forceinline__ PathSrc path_src(int nbw, const float2 *__restrict__ links, long site, int p) {
    PathSrc ps;
    ps.src = site;
    ps.sgn = 1.f;
    ps.U = nullptr;
    ps.dag = false;
    if (p > 0) {
        const int mu = (p - 1) & 3;
        const int v = __builtin_amdgcn_readlane(nbw, p - 1);   // forward entries 0..3, backward 4..7
        ps.src = v & 0x7fffffff;
        ps.sgn = v < 0 ? -1.f : 1.f;
        ps.dag = p > 4;
        ps.U = links + ((ps.dag ? ps.src : site) * 4 + mu) * 9;
    }
    return ps;
}

__device__ __forceinline__ void transport(const PathSrc &ps, const float2 (&a)[2][3], float2 (&t)[2][3]) {
    if (!ps.U) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) t[s][c] = a[s][c];
        return;
    }
    // w[c][d] = sgn U[c][d], or sgn conj(U[d][c]) for the backward path: the
    // signs are flipped as bits of wave-uniform values (scalar instructions),
    // so the lanes run only the 72 FMAs of the two 3x3 complex products
    const uint32_t sm = ps.sgn < 0.f ? 0x80000000u : 0u;
    const uint32_t cm = ps.dag ? 0x80000000u : 0u;
    float wr[9], wi[9], nwi[9];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const float2 x = ps.U[ps.dag ? d * 3 + c : c * 3 + d];
            wr[c * 3 + d] = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, x.x) ^ sm);
            wi[c * 3 + d] = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, x.y) ^ sm ^ cm);
            nwi[c * 3 + d] = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, x.y) ^ sm ^ cm ^ 0x80000000u);
        }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float re = wr[c * 3] * a[s][0].x, im = wr[c * 3] * a[s][0].y;
            re = fmaf(nwi[c * 3], a[s][0].y, re);
            im = fmaf(wi[c * 3], a[s][0].x, im);
#pragma unroll
            for (int d = 1; d < 3; ++d) {
                re = fmaf(wr[c * 3 + d], a[s][d].x, re);
                re = fmaf(nwi[c * 3 + d], a[s][d].y, re);
                im = fmaf(wr[c * 3 + d], a[s][d].y, im);
                im = fmaf(wi[c * 3 + d], a[s][d].x, im);
            }
            t[s][c] = make_float2(re, im);
        }
}

// One layer (or its adjoint): out = sum_p W_p T_p in.  Wave = (site, 16 rhs).
// Sites are taken in the blocked order of the site table (4^4 blocks where the
// extents allow): the neighbours of a block's sites are mostly in the block,
// whose inputs stay in the L2 of the XCD that runs it, where the lexicographic
// order put the z and t neighbours (576 and 13824 sites away at 24^4) out of
// any L2's reach.  Each wave writes only its own site, so the order does not
// change the result.
// Workgroups (4 units each) are dealt to the XCDs by whole site blocks: at
// each round XCD k works on block 8 i + k, so every XCD's L2 sees one compact
// block at a time while the eight XCDs work on consecutive, mostly adjacent
// blocks (face reads that cross to a neighbouring XCD's block at the same time
// are served by the memory-side cache).  wpb = workgroups per site block; the
// grid is padded to whole rounds and padding workgroups return.
template <int FIN, int FOUT>
__global__ __launch_bounds__(256) void k_net_layer(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                   const float2 *__restrict__ links, const int *__restrict__ nbr,
                                                   const bf16x4 *__restrict__ table, int N, int nrb,
                                                   unsigned nunits, const int *__restrict__ order, unsigned wpb) {
    const int lane = threadIdx.x & 63;
    const unsigned xcd = blockIdx.x % 8u, slot = blockIdx.x / 8u;
    const unsigned round = slot / wpb;
    const unsigned wg = (round * 8u + xcd) * wpb + (slot - round * wpb);
    const unsigned unit = uni(wg * 4u + (threadIdx.x >> 6));
    if (unit >= nunits) return;
    const unsigned q = unit / (unsigned)nrb;
    const long site = uni(order[q]);
    const int rb = (int)(unit - q * (unsigned)nrb);
    const int n = lane & 15, g = lane >> 4;
    const int rhs = rb * 16 + n;
    const int f = g >> 1, s0 = 2 * (g & 1);
    const bool act = rhs < N && f < FIN;
    constexpr int CIN = 12 * FIN, COUT = 12 * FOUT;

    f32x4 acc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nbw = nbr[site * 8 + (lane & 7)];

#pragma unroll 3
    for (int p = 0; p < NPATH; ++p) {
        const bf16x4 A = table[p * 64 + lane];
        const PathSrc ps = path_src(nbw, links, site, p);
        float2 a[2][3];
        const float2 *src = in + (ps.src * CIN + f * 12 + s0 * 3) * (long)N + rhs;
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) a[s][c] = act ? src[(s * 3 + c) * (long)N] : make_float2(0.f, 0.f);
        float2 t[2][3];
        transport(ps, a, t);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const bf16x4 B = pack4(t[0][c].x, t[0][c].y, t[1][c].x, t[1][c].y);
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc[c], 0, 0, 0);
        }
    }
    // lane holds rows 4g..4g+3 = complex outputs o = 2g, 2g+1 (o = field*4 + spin)
    if (rhs < N && 2 * g < 4 * FOUT) {
#pragma unroll
        for (int oo = 0; oo < 2; ++oo) {
            const int o = 2 * g + oo;
            const int fo = o >> 2, so = o & 3;
            float2 *dst = out + (site * COUT + fo * 12 + so * 3) * (long)N + rhs;
#pragma unroll
            for (int c = 0; c < 3; ++c) dst[c * (long)N] = make_float2(acc[c][2 * oo], acc[c][2 * oo + 1]);
        }
    }
}

// Weight gradient of one layer: P_p[i][b] = sum_{x, rhs, c} g_i(x, rhs, c) t_{p,b}(x, rhs, c)
// with i = 2o + ro over the output channels (g = dL/d out^*) and b = 2 ci + ri
// over the path's transported input channels.  Each wavefront sums its units
// (site, 16 rhs) in registers; the four wavefronts of a block are added in LDS
// and the block writes partial[block][p][lane*4 + r] = P_p[4 (lane/16) + r][lane % 16].
template <int FIN, int FOUT>
__global__ __launch_bounds__(256) void k_net_wgrad(const float2 *__restrict__ a_in, const float2 *__restrict__ gout,
                                                   const float2 *__restrict__ links, const int *__restrict__ nbr,
                                                   float *__restrict__ partial, int N, int nrb, unsigned nunits,
                                                   const int *__restrict__ order) {
    // transposition buffer [wave][colour][b][rhs] (bf16), reused for the block sum
    __shared__ float red[4][NPATH * 256];
    short(*lds)[3][16][16] = reinterpret_cast<short(*)[3][16][16]>(&red[0][0]);
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const unsigned wave = blockIdx.x * 4u + wv;
    const unsigned nwaves = gridDim.x * 4u;
    const int n = lane & 15, g = lane >> 4;
    const int f = g >> 1, s0 = 2 * (g & 1);
    constexpr int CIN = 12 * FIN, COUT = 12 * FOUT;
    // output-gradient operand: row i = lane % 16 -> channel o = i/2, part i&1
    const int oi = (lane & 15) >> 1, opart = lane & 1;

    f32x4 acc[NPATH];
#pragma unroll
    for (int p = 0; p < NPATH; ++p) acc[p] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (unsigned unit = wave; unit < nunits; unit += nwaves) {
        const unsigned u = uni(unit);
        const unsigned q = u / (unsigned)nrb;
        const long site = uni(order[q]);   // blocked site order, as in k_net_layer
        const int rb = (int)(u - q * (unsigned)nrb);
        // A operands: g_i at rhs rb*16 + 4g + j, one per colour
        bf16x4 Ag[3];
        {
            const bool ok = oi < 4 * FOUT;
            const int fo = oi >> 2, so = oi & 3;
            const float2 *gp = gout + (site * COUT + fo * 12 + so * 3) * (long)N;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r = rb * 16 + 4 * g + j;
                    float2 w = (ok && r < N) ? gp[c * (long)N + r] : make_float2(0.f, 0.f);
                    v[j] = opart ? w.y : w.x;
                }
                Ag[c] = pack4(v[0], v[1], v[2], v[3]);
            }
        }
        const int rhs = rb * 16 + n;
        const bool act = rhs < N && f < FIN;
        const int nbw = nbr[site * 8 + (lane & 7)];
#pragma unroll 1
        for (int p = 0; p < NPATH; ++p) {
            const PathSrc ps = path_src(nbw, links, site, p);
            float2 a[2][3];
            const float2 *src = a_in + (ps.src * CIN + f * 12 + s0 * 3) * (long)N + rhs;
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int c = 0; c < 3; ++c) a[s][c] = act ? src[(s * 3 + c) * (long)N] : make_float2(0.f, 0.f);
            float2 t[2][3];
            transport(ps, a, t);
            // lane (rhs n, group g) owns b = 4g + j: write, then read back transposed
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                lds[wv][c][4 * g + 0][n] = to_bf16(t[0][c].x);
                lds[wv][c][4 * g + 1][n] = to_bf16(t[0][c].y);
                lds[wv][c][4 * g + 2][n] = to_bf16(t[1][c].x);
                lds[wv][c][4 * g + 3][n] = to_bf16(t[1][c].y);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                // B[k = rhs 4g + j][n = b = lane % 16]
                const bf16x4 Bt = *reinterpret_cast<const bf16x4 *>(&lds[wv][c][lane & 15][4 * g]);
                acc[p] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Ag[c], Bt, acc[p], 0, 0, 0);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    __syncthreads();   // all transpositions done before the buffer is reused
#pragma unroll
    for (int p = 0; p < NPATH; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wv][p * 256 + lane * 4 + r] = acc[p][r];
    __syncthreads();
    float *dst = partial + (size_t)blockIdx.x * NPATH * 256;
    for (int e = threadIdx.x; e < NPATH * 256; e += 256) dst[e] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
}

// Sum the per-block partials in a fixed order: block (p, chunk) of 256
// threads owns 64 entries of P_p; thread slice q < 4 adds parts w = q mod 4,
// then the four slices are combined in order.  psum[p*256 + e] (FP64).
__global__ __launch_bounds__(256) void k_net_wgrad_sum(const float *__restrict__ partial, int nwaves,
                                                       double *__restrict__ psum) {
    __shared__ double red[4][64];
    const int p = blockIdx.x >> 2, chunk = blockIdx.x & 3;
    const int e = chunk * 64 + (threadIdx.x & 63), q = threadIdx.x >> 6;
    double s = 0.0;
    for (int w = q; w < nwaves; w += 4) s += (double)partial[((size_t)w * NPATH + p) * 256 + e];
    red[q][threadIdx.x & 63] = s;
    __syncthreads();
    if (q == 0) psum[p * 256 + e] = ((red[0][e & 63] + red[1][e & 63]) + red[2][e & 63]) + red[3][e & 63];
}

// Map P (psum, entry lane*4 + r = P[4 (lane/16) + r][lane % 16]) to the real
// gradient of the parameters of one layer:
//   dL/dW^* = Re: P[2o][2ci] + P[2o+1][2ci+1],  Im: P[2o+1][2ci] - P[2o][2ci+1];
//   d loss/d Re w = 2 Re(dL/dW^*), d loss/d Im w = 2 Im(dL/dW^*).
__global__ void k_net_wgrad_map(const double *__restrict__ psum, int layer, double *__restrict__ grad) {
    const int fin = FIELDS[layer], fout = FIELDS[layer + 1];
    const int npar = LAYER_OFF[layer + 1] - LAYER_OFF[layer];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npar) return;
    const int part = t & 1, idx = t >> 1;
    const int ci = idx % (4 * fin), o = (idx / (4 * fin)) % (4 * fout), p = idx / (16 * fin * fout);
    auto at = [&](int i, int b) { return psum[p * 256 + ((i >> 2) * 16 + b) * 4 + (i & 3)]; };
    const double v = part == 0 ? at(2 * o, 2 * ci) + at(2 * o + 1, 2 * ci + 1)
                               : at(2 * o + 1, 2 * ci) - at(2 * o, 2 * ci + 1);
    grad[LAYER_OFF[layer] + t] = 2.0 * v;
}

// g = (out - e) / (||e_r||^2 P) and per-block partial sums of |out - e|^2 / (||e_r||^2 P)
__global__ __launch_bounds__(256) void k_net_loss(const float2 *__restrict__ out, const float2 *__restrict__ e,
                                                  const double2 *__restrict__ en2, long total, int N, double invP,
                                                  float2 *__restrict__ gdst, double *__restrict__ lpart) {
    __shared__ double red[256];
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (i < total) {
        const int r = (int)(i % N);
        const double en = en2[r].x;
        const double w = en > 0 ? invP / en : 0.0;
        const float2 a = out[i], b = e[i];
        const float dx = a.x - b.x, dy = a.y - b.y;
        gdst[i] = make_float2((float)(w * dx), (float)(w * dy));
        l = w * ((double)dx * dx + (double)dy * dy);
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

// Deterministic sum of n partials: 256 threads add strided subsets in a fixed
// order, then a fixed tree.
__global__ __launch_bounds__(256) void k_sum_fixed(const double *__restrict__ part, int n, double *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Adam (Kingma & Ba, 2015) on the FP32 master weights.
__global__ void k_net_adam(float *__restrict__ theta, const double *__restrict__ grad, float *__restrict__ m,
                           float *__restrict__ v, double lr, double b1, double b2, double eps, double c1,
                           double c2) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NPARAM) return;
    const double gr = grad[t];
    const double mm = b1 * m[t] + (1.0 - b1) * gr;
    const double vv = b2 * v[t] + (1.0 - b2) * gr * gr;
    m[t] = (float)mm;
    v[t] = (float)vv;
    theta[t] = (float)(theta[t] - lr * (mm / c1) / (sqrt(vv / c2) + eps));
}

}  // namespace

struct mpmc_net {
    mpmc_ctx *ctx;
    float *theta;    // FP32 master weights [NPARAM]
    float *adam_m;
    float *adam_v;
    double *grad;    // [NPARAM]
    short *tables;   // 6 layer ops x TABLE_ELEMS bf16
    double *loss;    // [1]
    long adam_t;
};

namespace {

int net_pack(mpmc_net *net) {
    mpmc_ctx *ctx = net->ctx;
    k_net_pack<<<grid_for(6 * TABLE_ELEMS, 256), 256, 0, ctx->stream>>>(net->theta, net->tables);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// op: 2*layer (+1 for the adjoint); fin/fout are the op's own field counts
int launch_layer(mpmc_ctx *ctx, const mpmc_net *net, int op, const void *in, void *out, int N) {
    const int layer = op >> 1, adj = op & 1;
    const int fin = adj ? FIELDS[layer + 1] : FIELDS[layer];
    const int fout = adj ? FIELDS[layer] : FIELDS[layer + 1];
    const int nrb = (N + 15) / 16;
    const long units = ctx->V * nrb;
    if (units > 0xFFFFFFFFL - 4) return set_err(ctx, MPMC_EINVAL, "network: batch too large");
    // sites per block of the default site order (extent 4, 2 or 1 per direction)
    long bsites = 1;
    for (int mu = 0; mu < 4; ++mu) bsites *= ctx->dims[mu] % 4 == 0 ? 4 : (ctx->dims[mu] % 2 == 0 ? 2 : 1);
    const long wpb = std::max<long>(1, bsites * nrb / 4);          // workgroups per site block
    const long nwg = (units + 3) / 4;
    const long rounds = (nwg + 8 * wpb - 1) / (8 * wpb);
    if (rounds * 8 * wpb > 0x7FFFFFFFL) return set_err(ctx, MPMC_EINVAL, "network: batch too large");
    const unsigned blocks = (unsigned)(rounds * 8 * wpb);
    const bf16x4 *tab = reinterpret_cast<const bf16x4 *>(net->tables + (size_t)op * TABLE_ELEMS);
    const float2 *L = reinterpret_cast<const float2 *>(ctx->links32);
    const float2 *x = (const float2 *)in;
    float2 *y = (float2 *)out;
#define LAYER(A, B)                                                                                       \
    if (fin == A && fout == B)                                                                            \
        k_net_layer<A, B><<<blocks, 256, 0, ctx->stream>>>(x, y, L, ctx->nbr, tab, N, nrb, (unsigned)units, \
                                                           ctx->site_order, (unsigned)wpb);                  \
    else
    LAYER(1, 2)
    LAYER(2, 2)
    LAYER(2, 1)
    return set_err(ctx, MPMC_EINVAL, "network: bad layer shape");
#undef LAYER
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

int launch_wgrad(mpmc_ctx *ctx, mpmc_net *net, int layer, const void *a_in, const void *gout, int N,
                 float *partial, double *psum) {
    const int fin = FIELDS[layer], fout = FIELDS[layer + 1];
    const int nrb = (N + 15) / 16;
    const long units = ctx->V * nrb;
    const unsigned blocks = (unsigned)std::min<long>(WGRAD_BLOCKS, (units + 3) / 4);
    const float2 *L = reinterpret_cast<const float2 *>(ctx->links32);
    const float2 *a = (const float2 *)a_in;
    const float2 *gg = (const float2 *)gout;
#define WG(A, B)                                                                                              \
    if (fin == A && fout == B)                                                                                \
        k_net_wgrad<A, B><<<blocks, 256, 0, ctx->stream>>>(a, gg, L, ctx->nbr, partial, N, nrb, (unsigned)units, \
                                                           ctx->site_order);                                      \
    else
    WG(1, 2)
    WG(2, 2)
    WG(2, 1)
    return set_err(ctx, MPMC_EINVAL, "network: bad layer shape");
#undef WG
    HIP_OR_RET(ctx, hipGetLastError());
    k_net_wgrad_sum<<<NPATH * 4, 256, 0, ctx->stream>>>(partial, (int)blocks, psum);
    HIP_OR_RET(ctx, hipGetLastError());
    const int npar = LAYER_OFF[layer + 1] - LAYER_OFF[layer];
    k_net_wgrad_map<<<grid_for(npar, 64), 64, 0, ctx->stream>>>(psum, layer, net->grad);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

int check_net(const mpmc_net *net) {
    if (!net || !net->ctx) return MPMC_EINVAL;
    return MPMC_OK;
}

// Loss and gradient for P pairs (R, E); leaves the gradient in net->grad and
// the loss in net->loss (device).
int net_loss_grad(mpmc_net *net, const void *R, const void *E, int P) {
    mpmc_ctx *ctx = net->ctx;
    Scratch S(ctx);
    const size_t v1 = vec_bytes(ctx, P, MPMC_FP32), v2 = 2 * v1;
    void *a1 = S.get(v2), *a2 = S.get(v2), *a3 = S.get(v1), *g3 = S.get(v1), *g2 = S.get(v2), *g1 = S.get(v2);
    const long total = ctx->V * 12 * P;
    const unsigned lblocks = grid_for(total, 256);
    double *en2 = (double *)S.get(sizeof(double2) * P);
    double *lpart = (double *)S.get(sizeof(double) * lblocks);
    float *partial = (float *)S.get(sizeof(float) * (size_t)WGRAD_BLOCKS * NPATH * 256);
    double *psum = (double *)S.get(sizeof(double) * NPATH * 256);
    if (!a1 || !a2 || !a3 || !g3 || !g2 || !g1 || !en2 || !lpart || !partial || !psum) return MPMC_ENOMEM;
    RET_IF(launch_layer(ctx, net, 0, R, a1, P));
    RET_IF(launch_layer(ctx, net, 2, a1, a2, P));
    RET_IF(launch_layer(ctx, net, 4, a2, a3, P));
    RET_IF(blas_norm2(ctx, E, P, MPMC_FP32, en2));
    k_net_loss<<<lblocks, 256, 0, ctx->stream>>>((const float2 *)a3, (const float2 *)E, (const double2 *)en2, total,
                                                 P, 1.0 / P, (float2 *)g3, lpart);
    HIP_OR_RET(ctx, hipGetLastError());
    k_sum_fixed<<<1, 256, 0, ctx->stream>>>(lpart, (int)lblocks, net->loss);
    HIP_OR_RET(ctx, hipGetLastError());
    RET_IF(launch_wgrad(ctx, net, 2, a2, g3, P, partial, psum));
    RET_IF(launch_layer(ctx, net, 5, g3, g2, P));
    RET_IF(launch_wgrad(ctx, net, 1, a1, g2, P, partial, psum));
    RET_IF(launch_layer(ctx, net, 3, g2, g1, P));
    RET_IF(launch_wgrad(ctx, net, 0, R, g1, P, partial, psum));
    return MPMC_OK;
}

}  // namespace

// y = N(x) for FP32 internal-layout batches (used by the solves)
int net_apply_internal(mpmc_ctx *ctx, const mpmc_net *net, const void *x, void *y, int N) {
    Scratch S(ctx);
    const size_t v2 = 2 * vec_bytes(ctx, N, MPMC_FP32);
    void *a1 = S.get(v2), *a2 = S.get(v2);
    if (!a1 || !a2) return MPMC_ENOMEM;
    RET_IF(launch_layer(ctx, net, 0, x, a1, N));
    RET_IF(launch_layer(ctx, net, 2, a1, a2, N));
    return launch_layer(ctx, net, 4, a2, y, N);
}

const mpmc_ctx *net_context(const mpmc_net *net) { return net ? net->ctx : nullptr; }

MPMC_API int mpmc_net_n_params(void) { return NPARAM; }

MPMC_API void mpmc_net_destroy(mpmc_net *net) {
    if (!net) return;
    (void)hipFree(net->theta);
    (void)hipFree(net->adam_m);
    (void)hipFree(net->adam_v);
    (void)hipFree(net->grad);
    (void)hipFree(net->tables);
    (void)hipFree(net->loss);
    delete net;
}

MPMC_API int mpmc_net_set_weights(mpmc_net *net, const double *theta_host) {
    RET_IF(check_net(net));
    mpmc_ctx *ctx = net->ctx;
    if (!theta_host) return set_err(ctx, MPMC_EINVAL, "mpmc_net_set_weights: null weights");
    std::vector<float> f(NPARAM);
    for (int i = 0; i < NPARAM; ++i) {
        if (!std::isfinite(theta_host[i])) return set_err(ctx, MPMC_EINVAL, "mpmc_net_set_weights: weight %d not finite", i);
        f[i] = (float)theta_host[i];
    }
    HIP_OR_RET(ctx, hipMemcpyAsync(net->theta, f.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice, ctx->stream));
    HIP_OR_RET(ctx, hipMemsetAsync(net->adam_m, 0, sizeof(float) * NPARAM, ctx->stream));
    HIP_OR_RET(ctx, hipMemsetAsync(net->adam_v, 0, sizeof(float) * NPARAM, ctx->stream));
    net->adam_t = 0;
    RET_IF(net_pack(net));
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    return MPMC_OK;
}

MPMC_API int mpmc_net_get_weights(const mpmc_net *net, double *theta_host) {
    RET_IF(check_net(net));
    mpmc_ctx *ctx = net->ctx;
    if (!theta_host) return set_err(ctx, MPMC_EINVAL, "mpmc_net_get_weights: null output");
    std::vector<float> f(NPARAM);
    HIP_OR_RET(ctx, hipMemcpyAsync(f.data(), net->theta, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < NPARAM; ++i) theta_host[i] = f[i];
    return MPMC_OK;
}

MPMC_API int mpmc_net_create(mpmc_ctx *ctx, const double *theta_host, mpmc_net **out) {
    if (!ctx) return MPMC_EINVAL;
    if (!out || !theta_host) return set_err(ctx, MPMC_EINVAL, "mpmc_net_create: null argument");
    *out = nullptr;
    mpmc_net *net = new mpmc_net();
    net->ctx = ctx;
    hipError_t e = hipMalloc(&net->theta, sizeof(float) * NPARAM);
    if (e == hipSuccess) e = hipMalloc(&net->adam_m, sizeof(float) * NPARAM);
    if (e == hipSuccess) e = hipMalloc(&net->adam_v, sizeof(float) * NPARAM);
    if (e == hipSuccess) e = hipMalloc(&net->grad, sizeof(double) * NPARAM);
    if (e == hipSuccess) e = hipMalloc(&net->tables, sizeof(short) * 6 * TABLE_ELEMS);
    if (e == hipSuccess) e = hipMalloc(&net->loss, sizeof(double));
    if (e != hipSuccess) {
        mpmc_net_destroy(net);
        return set_err(ctx, MPMC_ENOMEM, "mpmc_net_create: %s", hipGetErrorString(e));
    }
    int rc = mpmc_net_set_weights(net, theta_host);
    if (rc != MPMC_OK) {
        mpmc_net_destroy(net);
        return rc;
    }
    *out = net;
    return MPMC_OK;
}

MPMC_API int mpmc_net_apply(mpmc_net *net, const void *x, void *y, int nrhs) {
    RET_IF(check_net(net));
    mpmc_ctx *ctx = net->ctx;
    if (!x || !y || nrhs < 1) return set_err(ctx, MPMC_EINVAL, "mpmc_net_apply: bad argument");
    if (x == y) return set_err(ctx, MPMC_EINVAL, "mpmc_net_apply: x and y must not alias");
    return net_apply_internal(ctx, net, x, y, nrhs);
}

MPMC_API int mpmc_net_loss_grad(mpmc_net *net, const void *R, const void *E, int npairs, double *loss_host,
                                double *grad_host) {
    RET_IF(check_net(net));
    mpmc_ctx *ctx = net->ctx;
    if (!R || !E || npairs < 1) return set_err(ctx, MPMC_EINVAL, "mpmc_net_loss_grad: bad argument");
    RET_IF(net_loss_grad(net, R, E, npairs));
    if (loss_host)
        HIP_OR_RET(ctx, hipMemcpyAsync(loss_host, net->loss, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    if (grad_host)
        HIP_OR_RET(ctx, hipMemcpyAsync(grad_host, net->grad, sizeof(double) * NPARAM, hipMemcpyDeviceToHost,
                                       ctx->stream));
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    return MPMC_OK;
}

MPMC_API int mpmc_net_train(mpmc_net *net, const void *R, const void *E, int npairs, int steps, double lr,
                            double *loss_host) {
    RET_IF(check_net(net));
    mpmc_ctx *ctx = net->ctx;
    if (!R || !E || npairs < 1 || steps < 1 || !(lr > 0))
        return set_err(ctx, MPMC_EINVAL, "mpmc_net_train: bad argument");
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    Scratch S(ctx);
    double *lossv = (double *)S.get(sizeof(double) * steps);
    if (!lossv) return MPMC_ENOMEM;
    for (int s = 0; s < steps; ++s) {
        RET_IF(net_loss_grad(net, R, E, npairs));
        HIP_OR_RET(ctx, hipMemcpyAsync(lossv + s, net->loss, sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
        ++net->adam_t;
        const double c1 = 1.0 - std::pow(b1, (double)net->adam_t), c2 = 1.0 - std::pow(b2, (double)net->adam_t);
        k_net_adam<<<grid_for(NPARAM, 256), 256, 0, ctx->stream>>>(net->theta, net->grad, net->adam_m, net->adam_v,
                                                                  lr, b1, b2, eps, c1, c2);
        HIP_OR_RET(ctx, hipGetLastError());
        RET_IF(net_pack(net));
    }
    if (loss_host)
        HIP_OR_RET(ctx, hipMemcpyAsync(loss_host, lossv, sizeof(double) * steps, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    return MPMC_OK;
}
