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
#include <complex>
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
