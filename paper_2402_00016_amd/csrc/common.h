// Internal declarations shared by the HIP sources of libmpmc.so (gfx950).
// Nothing here is part of the C ABI; the ABI is include/mpmc.h.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mpmc.h"

#define MPMC_API extern "C" __attribute__((visibility("default")))

// ---------------------------------------------------------------- context --

struct WsBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct mpmc_ctx {
    int dims[4];
    long V;            // sites
    long n;            // 12 V complex unknowns
    double kappa;
    int t_antiperiodic;
    hipStream_t stream;
    int device;
    // device data
    double *links64;   // canonical [V][4][3][3] complex double
    float *links32;    // same, complex float
    int *nbr;          // [V][8]: forward mu=0..3 then backward mu=0..3; bit 31 = time-boundary sign
    int *site_order;   // [V]: blocked traversal order of the sites (4D blocks of 4 where the extent allows)
    uint64_t mvps;     // right-hand-side operator applications issued
    std::string err;
    std::vector<WsBuf> ws;      // fixed workspace slots (reduction partials, dense scratch)
    std::vector<WsBuf> stack;   // scoped scratch buffers (see Scratch)
    int top;
    int num_cu;
    // optional launch timing of the Wilson kernels (mpmc_timing_*)
    int timing;
    std::vector<hipEvent_t> ev_pool;
    struct TimedLaunch {
        int ev0, ev1, prec;
        double bytes;
    };
    std::vector<TimedLaunch> timed;   // ev0 < 0: counted without events
    int timed_events = 0;             // events of ev_pool in use since the last enable
    // Wilson kernel variant per (nrhs, prec), set by mpmc_autotune / mpmc_tune_set
    std::map<std::pair<int, int>, int> tune;
    std::map<std::pair<int, int>, int> tune_explicit;   // variants set by mpmc_tune_set (not by the autotuner)
    std::map<std::pair<int, int>, int> tune_dot;        // fused level step traversal chosen by mpmc_autotune
    // polynomial right preconditioner of the solves inside mpmc_level_estimate
    const struct mpmc_poly *level_pp = nullptr;
    // small eigenproblems: 0 = Aberth-Ehrlich with the QR as fallback, 1 = QR only
    int dense_qr_only = 0;
    // deflate the solve level M^-1 - p_1 of mpmc_level_estimate (mpmc_set_solve_level_deflation)
    int solve_level_defl = 0;
    // storage precision of the single-vector Arnoldi cycles (mpmc_gmres_poly, mpmc_deflate)
    int setup_prec = MPMC_FP64;
    // their Gram-Schmidt: 0 = CGS2 with the second projection delayed one step, 1 = plain CGS2,
    // -1 = by lattice size (plain below 16^4 sites)
    int gs_cgs2 = -1;
    // projections per inner GMRES step of mpmc_solve / mpmc_solve_batch: 1, 2, or 0 = one for
    // FP32 and FP16S inner cycles, two for FP64 ones
    int solve_gs_passes = 0;
    unsigned col_flip = 0;   // column-kernel launches alternate their block order (bit 0)
    // fused polynomial recurrences replayed from captured hipGraphs (mpmc_set_graph_recurrences)
    int use_graphs = 0;
    hipStream_t gstream = nullptr;          // capture / replay stream (default priority)
    hipEvent_t gev[2] = {nullptr, nullptr}; // ordering between the context stream and gstream
    std::map<std::string, hipGraphExec_t> graphs;   // key: operands, shape and coefficients of a recurrence
    uint64_t graph_replays = 0;
    // distance colourings of mpmc_poly_trace_probe by polynomial degree: k, m[4], W[4][4]
    std::map<int, std::vector<int>> colourings;
};

struct mpmc_poly {
    const mpmc_ctx *ctx;
    std::vector<double> roots;  // 2*d doubles (complex), Leja ordered
    int d;
    const mpmc_poly *inner;     // not owned; the caller keeps p_in alive
};

struct mpmc_defl {
    const mpmc_ctx *ctx;
    int k;
    std::vector<double> lam;    // 2*k doubles (complex)
    double *Z;                  // device FP64 internal layout, k single-rhs vectors [k][n]
    double *U;                  // same
    double *lam_dev;            // device copy of lam
};

// Fixed workspace slots, used only inside one kernel launch sequence.
enum WsSlot {
    WS_PARTIAL = 0,   // reduction partials
    WS_DENSE,         // small dense FP64 matrices
    WS_NSLOTS
};

void *ws_get(mpmc_ctx *ctx, int slot, size_t bytes);   // nullptr on failure (ctx->err set)

// Scoped scratch: buffers taken from the context's stack are released when
// the Scratch object is destroyed.  Buffers are kept between calls, so a
// repeated call sequence allocates only the first time.
void *stack_get(mpmc_ctx *ctx, size_t bytes);
struct Scratch {
    mpmc_ctx *ctx;
    int base;
    explicit Scratch(mpmc_ctx *c) : ctx(c), base(c->top) {}
    ~Scratch() { ctx->top = base; }
    void *get(size_t bytes) { return stack_get(ctx, bytes); }
    Scratch(const Scratch &) = delete;
    Scratch &operator=(const Scratch &) = delete;
};

int set_err(const mpmc_ctx *ctx, int code, const char *fmt, ...);

#define HIP_OR_RET(ctx, call)                                                              \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return set_err((ctx), MPMC_EHIP, "%s: %s (%s:%d)", #call, hipGetErrorString(e_), \
                           __FILE__, __LINE__);                                            \
    } while (0)

#define RET_IF(x)            \
    do {                     \
        int rc_ = (x);       \
        if (rc_ != MPMC_OK)  \
            return rc_;      \
    } while (0)

static inline int prec_ok(int prec) { return prec == MPMC_FP64 || prec == MPMC_FP32 || prec == MPMC_FP16S; }

size_t vec_bytes(const mpmc_ctx *ctx, int nrhs, int prec);
size_t fp16s_scale_offset(const mpmc_ctx *ctx, int nrhs);

// ------------------------------------------------------- complex helpers --

template <typename T>
struct cpx {
    T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cpx<T> mk(T r, T i) {
    cpx<T> c;
    c.re = r;
    c.im = i;
    return c;
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
    return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return mk(s * a.re, s * a.im); }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> conjmul(cpx<T> a, cpx<T> b) {  // conj(a) * b
    return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return mk(a.re, -a.im); }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> times_i(cpx<T> a) { return mk(-a.im, a.re); }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> times_mi(cpx<T> a) { return mk(a.im, -a.re); }

// ------------------------------------------------- storage of one element --
// Element (s, k, r) of an internal-layout batch lives at e = (s*12 + k)*N + r;
// FP16S vectors keep one FP32 scale per (s, r) at sc = s*N + r.

template <int P>
struct Store;

template <>
struct Store<MPMC_FP64> {
    using real = double;
    __device__ static cpx<double> ld(const void *d, const float *, long e, long) {
        double2 v = reinterpret_cast<const double2 *>(d)[e];
        return mk(v.x, v.y);
    }
    __device__ static void st(void *d, long e, cpx<double> v) {
        reinterpret_cast<double2 *>(d)[e] = make_double2(v.re, v.im);
    }
};

template <>
struct Store<MPMC_FP32> {
    using real = float;
    __device__ static cpx<float> ld(const void *d, const float *, long e, long) {
        float2 v = reinterpret_cast<const float2 *>(d)[e];
        return mk(v.x, v.y);
    }
    __device__ static void st(void *d, long e, cpx<float> v) {
        reinterpret_cast<float2 *>(d)[e] = make_float2(v.re, v.im);
    }
};

template <>
struct Store<MPMC_FP16S> {
    using real = float;
    __device__ static cpx<float> ld(const void *d, const float *sc, long e, long si) {
        __half2 h = reinterpret_cast<const __half2 *>(d)[e];
        float s = sc[si];
        float2 f = __half22float2(h);
        return mk(f.x * s, f.y * s);
    }
};

// Host-side view of a vector batch: data pointer plus the FP16S scale array.
struct VecRef {
    void *d;
    float *sc;
};

VecRef vref(const mpmc_ctx *ctx, const void *p, int nrhs, int prec);

// ------------------------------------------------------------- Philox --
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from the
// published round function: two 32x32->64 multiplies per round, key bumped
// by the Weyl constants between rounds.

struct u32x4 {
    uint32_t v[4];
};

__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t lo0 = 0xD2511F53u * c0;
        uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2;
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    u32x4 o;
    o.v[0] = c0;
    o.v[1] = c1;
    o.v[2] = c2;
    o.v[3] = c3;
    return o;
}

// Z(4) symbols of the 12 components of site s for noise index idx: bits 2k..2k+1
// of the returned word hold the symbol of component s*12 + k.
__device__ __forceinline__ uint32_t z4_site_symbols(uint64_t seed, uint32_t stream, uint32_t idx, long s) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const long c0 = s * 12;
    const uint32_t b0 = (uint32_t)(c0 >> 6);
    const uint32_t b1 = (uint32_t)((c0 + 11) >> 6);
    u32x4 w0 = philox10(b0, idx, stream, 0u, k0, k1);
    u32x4 w1 = w0;
    if (b1 != b0) w1 = philox10(b1, idx, stream, 0u, k0, k1);
    uint32_t out = 0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const long c = c0 + k;
        const u32x4 &w = ((uint32_t)(c >> 6) == b0) ? w0 : w1;
        const int j = (int)(c & 63);
        const uint32_t sym = (w.v[j >> 4] >> (2 * (j & 15))) & 3u;
        out |= sym << (2 * k);
    }
    return out;
}

template <typename T>
__device__ __forceinline__ cpx<T> z4_value(uint32_t sym) {
    // i^sym
    return mk<T>(sym == 0 ? T(1) : (sym == 2 ? T(-1) : T(0)), sym == 1 ? T(1) : (sym == 3 ? T(-1) : T(0)));
}

// ------------------------------------------------------------ launches --

static inline unsigned grid_for(long work, int block) {
    return (unsigned)((work + block - 1) / block);
}

// Map the hardware workgroup id to a logical tile id so that each of the 8
// XCDs (which receive workgroups round-robin) processes one contiguous range
// of tiles, keeping stencil neighbours in the same XCD's L2.
__device__ __forceinline__ unsigned xcd_tile(unsigned bid, unsigned nblocks) {
    const unsigned nx = 8;
    const unsigned per = nblocks / nx, rem = nblocks % nx;
    const unsigned xcd = bid % nx, slot = bid / nx;
    // XCD x receives per (+1 if x < rem) workgroups and owns the tile range
    // starting at x*per + min(x, rem).
    return xcd * per + (xcd < rem ? xcd : rem) + slot;
}

// ---------------------------------------------------- cross-file host API --
// context.hip
int launch_noise(mpmc_ctx *ctx, uint64_t seed, uint32_t stream, uint64_t first, int nrhs, int prec, void *internal,
                 int ld = 0, int off = 0);   // columns off .. off+nrhs-1 of an operand of ld right-hand sides

// blas.hip.  Basis vectors Vb[j] are spaced vstride complex elements apart and
// hold vN right-hand sides (vN == nrhs, or vN == 1 for single vectors that are
// shared by all right-hand sides, e.g. deflation vectors).
int blas_multi_dot(mpmc_ctx *ctx, const void *Vb, long vstride, int vN, int nv, const void *w, int nrhs,
                   int prec, double *h_dev, int accumulate, int theta);
int blas_dot(mpmc_ctx *ctx, const void *x, const void *y, int nrhs, int prec, int theta, double *out_dev);
int blas_norm2(mpmc_ctx *ctx, const void *x, int nrhs, int prec, double *out_dev);
int blas_multi_axpy(mpmc_ctx *ctx, const void *Vb, long vstride, int vN, int nv, void *w, int nrhs, int prec,
                    const double *h_dev, int ldh, double sign, double *norm2_dev);
int blas_multi_axpy_dot(mpmc_ctx *ctx, const void *Vb, long vstride, int nv, void *w, int nrhs, int prec,
                        const double *h_dev, int ldh, double sign, double *h2_dev);
// Second Gram-Schmidt pass of one single-vector FP64 Arnoldi step: w -= V h2,
// then H(:, j) += h2, h_{j+1,j} = ||w|| with the breakdown test against the
// running Frobenius norm in state[0] (state[1] = d_eff or -1), and scale[0] =
// 1 / h_{j+1,j} (0 after a breakdown).  Two launches.
int blas_arnoldi_update(mpmc_ctx *ctx, const void *V, long vstride, int nv, void *w, const double *h2, double *Hcol,
                        int j, double *state, double *scale, int prec);
// FP16S Krylov bases (nrhs-wide FP16S batches spaced vstride_b bytes apart)
// against FP32 working vectors
int blas_multi_dot_h(mpmc_ctx *ctx, const void *Vb, size_t vstride_b, int nv, const void *w, int nrhs,
                     double *h_dev, int accumulate);
// out_h (FP16S, may be null): write the result there instead of back to w
int blas_multi_axpy_h(mpmc_ctx *ctx, const void *Vb, size_t vstride_b, int nv, void *w, int nrhs,
                      const double *h_dev, int ldh, double sign, double *norm2_dev, void *out_h = nullptr);
// the per-(site, rhs) scales of FP16S y *= Re coef[r] (coef per rhs, complex FP64, device)
int blas_scale_h(mpmc_ctx *ctx, void *y, int nrhs, const double *coef_dev);
int blas_axpby(mpmc_ctx *ctx, const void *x, void *y, int nrhs, int prec, double2 a, double2 b);
int blas_scale_rhs(mpmc_ctx *ctx, const void *x, void *y, int nrhs, int prec, const double *coef_dev, int mode);
int blas_convert(mpmc_ctx *ctx, const void *x, int px, void *y, int py, int nrhs);
// y (FP16S) = coef[r] x (FP32), coef per rhs (complex FP64, device)
int blas_convert_scaled_h(mpmc_ctx *ctx, const void *x, void *y, int nrhs, const double *coef_dev);
int blas_zero(mpmc_ctx *ctx, void *y, int nrhs, int prec);
int blas_scale_acc(mpmc_ctx *ctx, const double *t, int N, double2 c, double sign, double *acc);

// wilson.hip: out (FP32) = M b for an FP16S operand b
int wilson_apply_h2f(mpmc_ctx *ctx, const void *b, void *out, int nrhs);
// wilson.hip: out = alpha a + beta Theta op(b); y += gamma out (y may be null);
// yinit_on (single vectors, a == b): y = yinit b + gamma out, y not read
int wilson_launch_full(mpmc_ctx *ctx, const void *b, const void *a, void *out, void *y, int nrhs, int prec,
                       double2 alpha, double2 beta, double2 gamma, int dagger, int theta,
                       double2 yinit = double2{0.0, 0.0}, int yinit_on = 0);
// fused level step (see wilson.hip): w' = w - c M w; partial += cnext eta^H Theta w'
size_t wilson_dot_partial_count(const mpmc_ctx *ctx, int nrhs);
// codes of noise vectors first .. first+nrhs-1 into columns off .. of rows of
// ld entries (ld = 0: ld = nrhs)
int wilson_noise_codes(mpmc_ctx *ctx, uint64_t seed, uint32_t stream, uint64_t first, int nrhs, uint32_t *codes,
                       int ld = 0, int off = 0);
int wilson_dot_step_multi(mpmc_ctx *ctx, const void *w, void *wout, const uint32_t *codes, int nrhs, int nact,
                          int prec, const double *coef_dev, int theta, double *partial, int first_step);
int wilson_dot_finish_chunks(mpmc_ctx *ctx, const double *partial, int nrhs, double *out);
int wilson_dot_step(mpmc_ctx *ctx, const void *w, void *wout, const uint32_t *codes, int nrhs, int prec, double2 c,
                    double2 cnext, int theta, double *partial, int first_step, const void *a = nullptr,
                    double2 alpha = double2{0, 0}, double2 beta = double2{1, 0});
int wilson_dot_finish(mpmc_ctx *ctx, const double *partial, int nrhs, int prec, double *out, int accumulate,
                      double sign);
// timing hooks around one launch (no-ops unless timing is enabled)
int timing_begin(mpmc_ctx *ctx);
void timing_end(mpmc_ctx *ctx, int ev0, int prec, double bytes);
void timing_count(mpmc_ctx *ctx, int prec, double bytes);   // a launch without events

// dense.hip
int dense_harmonic_leja(mpmc_ctx *ctx, const double *H_dev, int ldh, int d, double beta, double *roots_dev,
                        double *info_dev);
int dense_hess_eigs(mpmc_ctx *ctx, const double *H_dev, int ldh, int m, double *ev_dev, double *info_dev);
int dense_inverse_iteration(mpmc_ctx *ctx, const double *H_dev, int ldh, int m, const double *mu_dev, int k,
                            double *Y_dev);
int dense_add_roots(mpmc_ctx *ctx, const double *roots_dev, int d, double thr, double digits, int max_out,
                    double *out_dev, int *count_dev);
int dense_givens_step(mpmc_ctx *ctx, double *H, int ldc, int j, int N, double *cs, double *g, double *res);
int dense_backsolve(mpmc_ctx *ctx, const double *H, int ldc, int k, int N, const double *g, double *y);

// krylov.hip
int poly_apply_internal(mpmc_ctx *ctx, const mpmc_poly *p, const void *x, void *y, int nrhs, int prec);
int poly_work_vectors(const mpmc_poly *p);
int poly_apply_buf(mpmc_ctx *ctx, const mpmc_poly *p, const void *x, void *y, int nrhs, int prec, void *const *buf);
int poly_validate(const mpmc_ctx *ctx, const mpmc_poly *p);
// Device address of `device`'s copy of the fixed scratch array of
// mpmc_apply_poly_noalloc (looked up once per device); nullptr on failure.
void *noalloc_scratch(int device);
// acc[r] += sign * eta_r^H Theta p(M) eta_r without forming p(M) eta (fused steps)
int poly_quad_fused(mpmc_ctx *ctx, const mpmc_poly *p, const void *eta, const uint32_t *codes, int nrhs, int prec,
                    int theta, double *acc, double sign);
bool poly_quad_fusable(int nrhs);
void graphs_clear(mpmc_ctx *ctx);
int wilson_dot_order(const mpmc_ctx *ctx, int nrhs, int prec);   // traversal of the fused step
int poly_matvecs(const mpmc_poly *p);
void poly_eval_host(const mpmc_poly *p, const double *lam, double *out, int k);

// deflate.hip (FP64, nrhs internal-layout vectors x)
//   c[i*nrhs + r] = u_i^H x_r (divided by lambda_i if divide_by_lambda)
int defl_coeffs(mpmc_ctx *ctx, const mpmc_defl *d, const void *x, int nrhs, double *c_dev, int divide_by_lambda);
//   x_r += sign * sum_i c[i*nrhs + r] z_i
int defl_add(mpmc_ctx *ctx, const mpmc_defl *d, const double *c_dev, void *x, int nrhs, double sign);
//   x <- (I - Z U^H) x
int defl_project(mpmc_ctx *ctx, const mpmc_defl *d, void *x, int nrhs);
int project_any(mpmc_ctx *ctx, const mpmc_defl *d, void *x, int prec);   // one vector in FP64 or FP32

// net.hip: y = N(x) for FP32 internal-layout batches (learned preconditioner)
int net_apply_internal(mpmc_ctx *ctx, const mpmc_net *net, const void *x, void *y, int nrhs);
const mpmc_ctx *net_context(const mpmc_net *net);

// solve.hip
// Optional record of (residual, error) pairs at the start of each outer cycle
// (network training data): batches of nrhs FP32 vectors.
struct SolveSnap {
    void *R, *E;   // max batches each, spaced vec_bytes(ctx, nrhs, FP32) apart
    int max;
    int count;     // out
};
int solve_internal(mpmc_ctx *ctx, const void *b, void *x, int nrhs, const mpmc_defl *defl, const mpmc_net *net,
                   int restart, double tol, int inner_prec, int max_outer, int *iters, double *relres_host,
                   SolveSnap *snap = nullptr, const mpmc_poly *pp = nullptr);
