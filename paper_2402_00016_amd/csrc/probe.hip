// Exact trace of a polynomial by probing (Sec. 6: the last term Tr(p_K(M)) is
// computed exactly with probing; the paper cites the probing literature).
//
// Sites are coloured by c(x) = sum_mu (x_mu mod a_mu) * prod_{nu<mu} a_nu with
// a_mu dividing L_mu.  For colour c and spin-colour index alpha the probe vector
// v_{c,alpha} has a 1 at component alpha of every site of colour c and 0
// elsewhere, so v^H Theta p(M) v adds the diagonal entries (s, alpha) of
// Theta p(M) over that colour plus the entries between distinct same-colour
// sites.  p(M) of degree D only couples sites at taxicab distance <= D; distinct
// sites of one colour differ by a nonzero multiple of a_mu along some axis with
// a_mu < L_mu, so the sum is the exact trace when every such a_mu satisfies
// D < a_mu <= L_mu / 2 (a_mu = L_mu gives every site its own colour).
#include <algorithm>
#include <cmath>
#include <complex>
#include <new>
#include <vector>

#include "common.h"

namespace {

struct Colouring {
    int L[4], a[4];
};

// probe r of the batch is (colour c0 + r / 12, alpha = r % 12)
template <int P>
__global__ void k_probe(Colouring cl, long V, int N, long c0, VecRef out) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= V * N) return;
    const long s = t / N;
    const int r = (int)(t - s * N);
    long q = s, col = 0, mul = 1;
    for (int mu = 0; mu < 4; ++mu) {
        const long x = q % cl.L[mu];
        q /= cl.L[mu];
        col += (x % cl.a[mu]) * mul;
        mul *= cl.a[mu];
    }
    const long c = c0 + r / 12;
    const int alpha = r % 12;
    using R = typename Store<P>::real;
#pragma unroll
    for (int k = 0; k < 12; ++k)
        Store<P>::st(out.d, (s * 12 + k) * N + r, mk((R)((col == c && k == alpha) ? 1 : 0), (R)0));
}

}  // namespace

// ------------------------------------------------ distance colouring --
// Exact probing needs colours such that two distinct sites of one colour are
// further apart (taxicab distance on the periodic lattice) than the degree D
// of the polynomial: (p(M))_{xy} vanishes for dist(x, y) > D because M only
// couples nearest neighbours.  The colourings here are lattice codes: k <= 3
// linear forms c_i(x) = (sum_mu W[i][mu] x_mu) mod m_i with every m_i
// dividing every extent L_mu (so each form is well defined on the torus), and
// colour(x) = sum_i c_i(x) prod_{l<i} m_l.  Such a colouring is translation
// invariant, so it is valid exactly when W delta != 0 (mod m) for every
// displacement delta with 0 < |delta|_1 <= D that is not a period of the
// lattice.  Candidates are tried by increasing colour count prod m_i, each
// with a fixed pseudo-random sequence of W; if none passes, every site gets
// its own colour (forms x_mu mod L_mu), which is always valid.

namespace {

struct LinCol {
    int k;
    int m[4];
    int W[4][4];
};

// Displacements 0 < |d|_1 <= D that are not periods of the lattice.  A colour
// W x mod m with m dividing every L_mu depends on d only modulo L, so when the
// ball is larger than the lattice the residues r with torus distance
// sum_mu min(r_mu, L_mu - r_mu) <= D stand for it (the same conditions, at
// most V - 1 of them; the ball of radius 256 alone would hold ~10^9).
static void ball_displacements(const int L[4], int D, std::vector<int> &out) {
    out.clear();
    const double ball = std::pow(2.0 * D + 1.0, 4.0);
    const long V = (long)L[0] * L[1] * L[2] * L[3];
    if (ball > 4.0 * (double)V) {
        for (long q = 0; q < V; ++q) {
            int r[4];
            long t = q;
            int dist = 0;
            for (int mu = 0; mu < 4; ++mu) {
                r[mu] = (int)(t % L[mu]);
                t /= L[mu];
                dist += std::min(r[mu], L[mu] - r[mu]);
            }
            if (q != 0 && dist <= D) out.insert(out.end(), r, r + 4);
        }
        return;
    }
    for (int a = -D; a <= D; ++a)
        for (int b = -(D - std::abs(a)); b <= D - std::abs(a); ++b)
            for (int c = -(D - std::abs(a) - std::abs(b)); c <= D - std::abs(a) - std::abs(b); ++c) {
                const int r = D - std::abs(a) - std::abs(b) - std::abs(c);
                for (int e = -r; e <= r; ++e) {
                    const int d[4] = {a, b, c, e};
                    bool period = true;
                    for (int mu = 0; mu < 4; ++mu)
                        if (((d[mu] % L[mu]) + L[mu]) % L[mu] != 0) period = false;
                    if (period) continue;   // includes d = 0
                    out.insert(out.end(), d, d + 4);
                }
            }
}

static bool colouring_valid(const LinCol &c, const std::vector<int> &disp) {
    const size_t nd = disp.size() / 4;
    for (size_t q = 0; q < nd; ++q) {
        const int *d = &disp[4 * q];
        bool same = true;
        for (int i = 0; i < c.k && same; ++i) {
            long v = 0;
            for (int mu = 0; mu < 4; ++mu) v += (long)c.W[i][mu] * d[mu];
            if (((v % c.m[i]) + c.m[i]) % c.m[i] != 0) same = false;
        }
        if (same) return false;
    }
    return true;
}

static LinCol identity_colouring(const int L[4]) {
    LinCol c{};
    c.k = 4;
    for (int mu = 0; mu < 4; ++mu) {
        c.m[mu] = L[mu];
        for (int nu = 0; nu < 4; ++nu) c.W[mu][nu] = mu == nu ? 1 : 0;
    }
    return c;
}

// Largest residue set the search enumerates (16 bytes each); beyond it, and
// whenever D reaches across the whole torus, every site is its own colour.
constexpr long kColourSearchMaxV = 1L << 24;

static LinCol find_colouring(const int L[4], int D) {
    const long V = (long)L[0] * L[1] * L[2] * L[3];
    int diameter = 0;
    for (int mu = 0; mu < 4; ++mu) diameter += L[mu] / 2;
    if (D >= diameter && V > 1) return identity_colouring(L);   // every pair of sites conflicts
    if (std::pow(2.0 * D + 1.0, 4.0) > 4.0 * (double)V && V > kColourSearchMaxV) return identity_colouring(L);
    std::vector<int> disp;
    ball_displacements(L, D, disp);
    if (disp.empty()) {   // D = 0: one colour
        LinCol c{};
        c.k = 1;
        c.m[0] = 1;
        return c;
    }
    int g = L[0];
    for (int mu = 1; mu < 4; ++mu) {
        int a = g, b = L[mu];
        while (b) {
            const int t = a % b;
            a = b;
            b = t;
        }
        g = a;
    }
    std::vector<int> divs;
    for (int d = 2; d <= g; ++d)
        if (g % d == 0) divs.push_back(d);
    struct Cand {
        long prod;
        std::vector<int> ms;
    };
    std::vector<Cand> cands;
    const int nd = (int)divs.size();
    for (int a = 0; a < nd; ++a) {
        cands.push_back({divs[a], {divs[a]}});
        for (int b = a; b < nd; ++b) {
            cands.push_back({(long)divs[a] * divs[b], {divs[a], divs[b]}});
            for (int c = b; c < nd; ++c) cands.push_back({(long)divs[a] * divs[b] * divs[c], {divs[a], divs[b], divs[c]}});
        }
    }
    std::stable_sort(cands.begin(), cands.end(), [](const Cand &x, const Cand &y) { return x.prod < y.prod; });
    uint64_t st = 0x9E3779B97F4A7C15ull;   // fixed seed: the colouring depends on (L, D) only
    auto next = [&st]() {
        st ^= st << 13;
        st ^= st >> 7;
        st ^= st << 17;
        return st;
    };
    constexpr int kTries = 2000;
    for (const Cand &cd : cands) {
        if (cd.prod >= V) break;
        LinCol c{};
        c.k = (int)cd.ms.size();
        for (int i = 0; i < c.k; ++i) c.m[i] = cd.ms[i];
        for (int t = 0; t < kTries; ++t) {
            for (int i = 0; i < c.k; ++i)
                for (int mu = 0; mu < 4; ++mu) c.W[i][mu] = (int)(next() % (uint64_t)c.m[i]);
            if (colouring_valid(c, disp)) return c;
        }
    }
    return identity_colouring(L);
}

struct ProbeCol {
    int k, L[4], m[4], W[4][4];
    long c0;   // colour of probe 0 of the batch; probe r is (colour c0 + r / 12, alpha = r % 12)
};

__device__ __forceinline__ long site_colour(const ProbeCol &pc, long s) {
    int x[4];
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (int)(s % pc.L[mu]);
        s /= pc.L[mu];
    }
    long col = 0, mul = 1;
    for (int i = 0; i < pc.k; ++i) {
        long v = 0;
        for (int mu = 0; mu < 4; ++mu) v += (long)pc.W[i][mu] * x[mu];
        col += (v % pc.m[i]) * mul;
        mul *= pc.m[i];
    }
    return col;
}

template <int P>
__global__ void k_probe_lin(ProbeCol pc, long V, int N, VecRef out) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= V * N) return;
    const long s = t / N;
    const int r = (int)(t - s * N);
    const bool on = site_colour(pc, s) == pc.c0 + r / 12;
    const int alpha = r % 12;
    using R = typename Store<P>::real;
#pragma unroll
    for (int k = 0; k < 12; ++k) Store<P>::st(out.d, (s * 12 + k) * N + r, mk((R)((on && k == alpha) ? 1 : 0), (R)0));
}

}  // namespace

MPMC_API int mpmc_probe_colouring(const int dims[4], int distance, int *k_host, int *moduli_host, int *W_host,
                                  long *ncolours_host) {
    if (!dims || distance < 0 || !k_host || !moduli_host || !W_host || !ncolours_host) return MPMC_EINVAL;
    for (int mu = 0; mu < 4; ++mu)
        if (dims[mu] < 1 || dims[mu] > 1024) return MPMC_EINVAL;
    LinCol c;
    try {
        c = find_colouring(dims, distance);
    } catch (const std::bad_alloc &) {
        return MPMC_ENOMEM;
    }
    *k_host = c.k;
    long nc = 1;
    for (int i = 0; i < 4; ++i) {
        moduli_host[i] = i < c.k ? c.m[i] : 1;
        if (i < c.k) nc *= c.m[i];
        for (int mu = 0; mu < 4; ++mu) W_host[4 * i + mu] = i < c.k ? c.W[i][mu] : 0;
    }
    *ncolours_host = nc;
    return MPMC_OK;
}

MPMC_API int mpmc_poly_trace_probe(mpmc_ctx *ctx, const mpmc_poly *p, int theta, int prec, int max_batch,
                                   double *trace_host, long *nprobe_host, uint64_t *mvps_host) {
    if (!ctx) return MPMC_EINVAL;
    if (!p || !trace_host || (prec != MPMC_FP64 && prec != MPMC_FP32) ||
        (theta != MPMC_THETA_I && theta != MPMC_THETA_G5) || max_batch < 0)
        return set_err(ctx, MPMC_EINVAL, "mpmc_poly_trace_probe: bad argument");
    if (p->ctx != ctx) return set_err(ctx, MPMC_ESTATE, "mpmc_poly_trace_probe: polynomial from another context");
    int degree = 0;
    mpmc_poly_info(p, nullptr, nullptr, &degree, nullptr);
    auto it = ctx->colourings.find(degree);
    if (it == ctx->colourings.end()) {
        LinCol c;
        try {
            c = find_colouring(ctx->dims, degree);
        } catch (const std::bad_alloc &) {
            return set_err(ctx, MPMC_ENOMEM, "mpmc_poly_trace_probe: colouring search out of host memory");
        }
        std::vector<int> enc(1 + 4 + 16, 0);
        enc[0] = c.k;
        for (int i = 0; i < c.k; ++i) {
            enc[1 + i] = c.m[i];
            for (int mu = 0; mu < 4; ++mu) enc[5 + 4 * i + mu] = c.W[i][mu];
        }
        it = ctx->colourings.emplace(degree, enc).first;
    }
    ProbeCol pc{};
    pc.k = it->second[0];
    long ncol = 1;
    for (int i = 0; i < pc.k; ++i) {
        pc.m[i] = it->second[1 + i];
        ncol *= pc.m[i];
        for (int mu = 0; mu < 4; ++mu) pc.W[i][mu] = it->second[5 + 4 * i + mu];
    }
    for (int mu = 0; mu < 4; ++mu) pc.L[mu] = ctx->dims[mu];
    const uint64_t mvp0 = ctx->mvps;
    const long nprobe = ncol * 12;
    // batches of whole colours (a multiple of 12 probes), 192 by default
    long B = max_batch > 0 ? max_batch : 192;
    B = std::max<long>(12, (B / 12) * 12);
    B = std::min(B, nprobe);
    Scratch S(ctx);
    void *v = S.get(vec_bytes(ctx, (int)B, prec));
    void *y = S.get(vec_bytes(ctx, (int)B, prec));
    double2 *acc = (double2 *)S.get(sizeof(double2) * B);
    if (!v || !y || !acc) return MPMC_ENOMEM;
    std::vector<double> qh(2 * B);
    std::complex<double> tr(0, 0);
    for (long p0 = 0; p0 < nprobe; p0 += B) {
        const int nb = (int)std::min(B, nprobe - p0);
        pc.c0 = p0 / 12;
        const long work = ctx->V * nb;
        VecRef vo = vref(ctx, v, nb, prec);
        if (prec == MPMC_FP64) k_probe_lin<MPMC_FP64><<<grid_for(work, 256), 256, 0, ctx->stream>>>(pc, ctx->V, nb, vo);
        else k_probe_lin<MPMC_FP32><<<grid_for(work, 256), 256, 0, ctx->stream>>>(pc, ctx->V, nb, vo);
        HIP_OR_RET(ctx, hipGetLastError());
        RET_IF(poly_apply_internal(ctx, p, v, y, nb, prec));
        RET_IF(blas_dot(ctx, v, y, nb, prec, theta == MPMC_THETA_G5 ? 1 : 0, (double *)acc));
        HIP_OR_RET(ctx, hipMemcpyAsync(qh.data(), acc, sizeof(double2) * nb, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
        for (int r = 0; r < nb; ++r) tr += std::complex<double>(qh[2 * r], qh[2 * r + 1]);
    }
    trace_host[0] = tr.real();
    trace_host[1] = tr.imag();
    if (nprobe_host) *nprobe_host = nprobe;
    if (mvps_host) *mvps_host = ctx->mvps - mvp0;
    return MPMC_OK;
}

MPMC_API int mpmc_poly_trace(mpmc_ctx *ctx, const mpmc_poly *p, int theta, const int period[4], int prec,
                             int max_batch, double *trace_host, int *exact_host, uint64_t *mvps_host) {
    if (!ctx) return MPMC_EINVAL;
    if (!p || !period || !trace_host || (prec != MPMC_FP64 && prec != MPMC_FP32) ||
        (theta != MPMC_THETA_I && theta != MPMC_THETA_G5))
        return set_err(ctx, MPMC_EINVAL, "mpmc_poly_trace: bad argument");
    if (p->ctx != ctx) return set_err(ctx, MPMC_ESTATE, "mpmc_poly_trace: polynomial from another context");
    Colouring cl;
    long ncol = 1;
    int degree = 0;
    mpmc_poly_info(p, nullptr, nullptr, &degree, nullptr);
    int exact = 1;
    for (int mu = 0; mu < 4; ++mu) {
        cl.L[mu] = ctx->dims[mu];
        cl.a[mu] = period[mu];
        if (period[mu] < 1 || ctx->dims[mu] % period[mu] != 0)
            return set_err(ctx, MPMC_EINVAL, "mpmc_poly_trace: period[%d]=%d must divide L=%d", mu, period[mu],
                           ctx->dims[mu]);
        ncol *= period[mu];
        if (period[mu] < ctx->dims[mu] && !(period[mu] > degree && 2 * period[mu] <= ctx->dims[mu])) exact = 0;
    }
    const uint64_t mvp0 = ctx->mvps;
    const long nprobe = ncol * 12;
    // batches are whole multiples of 12 (all alpha of a colour) and of 64 when possible
    long B = max_batch > 0 ? max_batch : 192;
    B = std::max<long>(12, (B / 12) * 12);
    B = std::min(B, nprobe);
    Scratch S(ctx);
    void *v = S.get(vec_bytes(ctx, (int)B, prec));
    void *y = S.get(vec_bytes(ctx, (int)B, prec));
    double2 *q = (double2 *)S.get(sizeof(double2) * B);
    if (!v || !y || !q) return MPMC_ENOMEM;
    std::vector<double> qh(2 * B);
    std::complex<double> tr(0, 0);
    for (long p0 = 0; p0 < nprobe; p0 += B) {
        const int nb = (int)std::min(B, nprobe - p0);
        VecRef o = vref(ctx, v, nb, prec);
        const long work = ctx->V * nb;
        if (prec == MPMC_FP64) k_probe<MPMC_FP64><<<grid_for(work, 256), 256, 0, ctx->stream>>>(cl, ctx->V, nb, p0 / 12, o);
        else k_probe<MPMC_FP32><<<grid_for(work, 256), 256, 0, ctx->stream>>>(cl, ctx->V, nb, p0 / 12, o);
        HIP_OR_RET(ctx, hipGetLastError());
        RET_IF(poly_apply_internal(ctx, p, v, y, nb, prec));
        RET_IF(blas_dot(ctx, v, y, nb, prec, theta == MPMC_THETA_G5 ? 1 : 0, (double *)q));
        HIP_OR_RET(ctx, hipMemcpyAsync(qh.data(), q, sizeof(double2) * nb, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
        for (int r = 0; r < nb; ++r) tr += std::complex<double>(qh[2 * r], qh[2 * r + 1]);
    }
    trace_host[0] = tr.real();
    trace_host[1] = tr.imag();
    if (exact_host) *exact_host = exact;
    if (mvps_host) *mvps_host = ctx->mvps - mvp0;
    return MPMC_OK;
}
