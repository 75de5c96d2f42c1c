// Main solves M x = b for a batch of right-hand sides (Sec. 1: the main
// expense of the method; Sec. 8: deflated GMRES).
//
// Mixed-precision defect correction: the outer loop keeps x and r = b - M x in
// FP64 and tests the TRUE residual; each inner restarted GMRES(m) cycle runs in
// the inner precision (FP64 or FP32 storage, FP64 dot products) on r and
// returns a correction e, x += e.  All right-hand sides advance together: one
// Wilson launch, one Gram-Schmidt dot launch and one update launch per inner
// iteration serve the whole batch, and the per-rhs Hessenberg/Givens state
// lives on the device.  With a learned preconditioner N the inner cycle is
// flexible GMRES (z_j = N v_j, Arnoldi on M z_j, correction sum_j y_j z_j).
// With a polynomial preconditioner p (the paper's PP-GMRES, Sec. 8) the inner
// cycle is right-preconditioned GMRES on M p(M) and the correction is p(M) V y.
// With a deflation set, x starts at Z Lambda^-1 U^H b and
// each restart adds Z Lambda^-1 U^H r (projection of the small eigen-components).
#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "common.h"

namespace {

constexpr int kSolveBatchMax = 8;   // lattices per batched solve (the batched Wilson launch's limit)

// H column j (rows 0..j) += h2; h_{j+1,j} = sqrt(nrm2); scale = 1/h_{j+1,j}
__global__ void k_finalize_batch(double2 *Hcol, const double2 *h2, int j, int N, const double2 *nrm2,
                                 double2 *scale) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    if (h2)
        for (int i = 0; i <= j; ++i) {
            Hcol[(long)i * N + r].x += h2[(long)i * N + r].x;
            Hcol[(long)i * N + r].y += h2[(long)i * N + r].y;
        }
    const double hn = sqrt(fmax(nrm2[r].x, 0.0));
    Hcol[(long)(j + 1) * N + r] = make_double2(hn, 0.0);
    scale[r] = make_double2(hn > 1e-290 ? 1.0 / hn : 0.0, 0.0);
}

__global__ void k_init_g(double2 *g, int m, int N, const double2 *rn2) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)(m + 1) * N) return;
    const int r = (int)(t % N);
    g[t] = t < N ? make_double2(sqrt(fmax(rn2[r].x, 0.0)), 0.0) : make_double2(0.0, 0.0);
}

// One context's solve: the outer defect-correction loop and the current
// inner GMRES(m) cycle as a state object.  solve_internal drives one;
// mpmc_solve_batch drives several contexts in lockstep, with the Wilson
// operator of all of them in one batched launch per inner iteration.  The
// sequence of library calls per context is the same either way.
class Gmres {
  public:
    Gmres(mpmc_ctx *ctx, const void *b, void *x, int N, const mpmc_defl *defl, const mpmc_net *net, int m,
          double tol, int inner_prec, int max_outer, SolveSnap *snap, const mpmc_poly *pp)
        : ctx_(ctx), S_(ctx), b_(b), x_(x), N_(N), defl_(defl), net_(net), m_(m), tol_(tol), inner_prec_(inner_prec),
          max_outer_(max_outer), snap_(snap), pp_(pp) {}
    int init();
    // Starts the next outer cycle; *go = false once converged or out of cycles.
    int begin_cycle(bool *go);
    // The vector the operator acts on at inner step j: v_j, or z_j = N v_j.
    int operand(int j, const void **opin);
    // Where the operator's output goes (inner precision, nrhs vectors).
    void *wvec() const { return w_; }
    // w = M op(v_j) on this context alone (polynomial, FP16 basis or plain).
    int matvec(int j, const void *opin);
    // Gram-Schmidt, Hessenberg column and Givens step of inner step j;
    // *more = false when the cycle ends (restart length or targets reached).
    int orthogonalize(int j, bool *more);
    // Correction e = V y (Z y, p(M) V y) and x += e.
    int end_cycle();
    int finish(int *iters_out, double *relres_host);
    // The plain FP64/FP32 form, whose operator a batched launch can apply.
    bool batchable() const { return !pp_ && !half_; }

  private:
    int true_residual();
    void *basis(int j) const {
        return half_ ? (void *)((char *)V_ + (size_t)j * vbb_) : (void *)((char *)V_ + (size_t)j * vstride_ * es_);
    }

    mpmc_ctx *ctx_;
    Scratch S_;
    const void *b_;
    void *x_;
    int N_;
    const mpmc_defl *defl_;
    const mpmc_net *net_;
    int m_;
    double tol_;
    int inner_prec_, max_outer_;
    SolveSnap *snap_;
    const mpmc_poly *pp_;
    // storage
    int pb_ = 0, pw_ = 0;
    bool half_ = false;
    size_t vb64_ = 0, vbi_ = 0, vbb_ = 0, es_ = 0;
    long vstride_ = 0;
    double *r_ = nullptr, *H_ = nullptr, *h2_ = nullptr, *cs_ = nullptr, *g_ = nullptr, *y_ = nullptr;
    double *res_ = nullptr, *sc_ = nullptr, *dc_ = nullptr, *nrm_ = nullptr, *scale_ = nullptr;
    void *V_ = nullptr, *Zb_ = nullptr, *w_ = nullptr, *corr_ = nullptr, *tp_ = nullptr, *tq_ = nullptr;
    void *xsnap_ = nullptr;
    // state
    std::vector<double> bn2_, rn2_, resh_, rel_, rel_start_, target_;
    bool use_net_ = false, converged_ = false;
    const mpmc_net *cnet_ = nullptr;
    int outer_ = 0, total_ = 0, jdone_ = 0;
    int check_every_ = 10;   // inner steps between convergence checks
};

int Gmres::init() {
    mpmc_ctx *ctx = ctx_;
    const int N = N_, m = m_;
    if (pp_ && net_) return set_err(ctx, MPMC_EINVAL, "mpmc_solve: polynomial and learned preconditioner are exclusive");
    if (pp_ && pp_->ctx != ctx) return set_err(ctx, MPMC_ESTATE, "mpmc_solve: polynomial belongs to another context");
    if (net_ && net_context(net_) != ctx)
        return set_err(ctx, MPMC_ESTATE, "mpmc_solve: network belongs to another context");
    if (net_ && inner_prec_ != MPMC_FP32 && inner_prec_ != MPMC_FP16S)
        return set_err(ctx, MPMC_EINVAL, "mpmc_solve: the learned preconditioner runs with FP32 arithmetic "
                                         "(FP32 or FP16S inner cycles) only");
    if (inner_prec_ != MPMC_FP64 && inner_prec_ != MPMC_FP32 && inner_prec_ != MPMC_FP16S)
        return set_err(ctx, MPMC_EINVAL, "mpmc_solve: inner precision must be FP64, FP32 or FP16S");
    // basis vectors in pb (FP16S: half + per-(site, rhs) scale, storage only);
    // working vectors (w, e) and arithmetic in pw
    pb_ = inner_prec_;
    pw_ = inner_prec_ == MPMC_FP64 ? MPMC_FP64 : MPMC_FP32;
    half_ = pb_ == MPMC_FP16S;
    vb64_ = vec_bytes(ctx, N, MPMC_FP64);
    vbi_ = vec_bytes(ctx, N, pw_);
    vbb_ = vec_bytes(ctx, N, pb_);
    vstride_ = ctx->n * N;   // complex elements between basis vectors (FP64/FP32 bases)
    es_ = inner_prec_ == MPMC_FP64 ? 16 : 8;
    r_ = (double *)S_.get(vb64_);
    V_ = S_.get(vbb_ * (m + 1));
    Zb_ = net_ ? S_.get(vbi_ * m) : nullptr;   // flexible GMRES: preconditioned basis z_j = N v_j
    w_ = S_.get(vbi_);
    corr_ = S_.get(vbi_);
    tp_ = pp_ ? S_.get(vbi_) : nullptr;          // p(M) v_j (polynomial right preconditioning)
    tq_ = (pp_ || net_) && half_ ? S_.get(vbi_) : nullptr;  // FP32 copy of an FP16S basis vector
    H_ = (double *)S_.get(sizeof(double2) * (size_t)(m + 1) * (m + 1) * N);
    h2_ = (double *)S_.get(sizeof(double2) * (size_t)(m + 1) * N);
    cs_ = (double *)S_.get(sizeof(double2) * (size_t)2 * m * N);
    g_ = (double *)S_.get(sizeof(double2) * (size_t)(m + 1) * N);
    y_ = (double *)S_.get(sizeof(double2) * (size_t)m * N);
    res_ = (double *)S_.get(sizeof(double) * N);
    sc_ = (double *)S_.get(sizeof(double2) * 4 * N);   // [0..N) norms, [N..2N) scales
    dc_ = defl_ && defl_->k ? (double *)S_.get(sizeof(double2) * (size_t)defl_->k * N) : nullptr;
    xsnap_ = snap_ ? S_.get(vb64_ * (size_t)snap_->max) : nullptr;   // FP64 iterates x_k of the record
    if (snap_ && !xsnap_) return MPMC_ENOMEM;
    if (!r_ || !V_ || (net_ && !Zb_) || (pp_ && !tp_) || ((pp_ || net_) && half_ && !tq_) || !w_ || !corr_ || !H_ || !h2_ ||
        !cs_ || !g_ || !y_ || !res_ || !sc_ || (defl_ && defl_->k && !dc_))
        return MPMC_ENOMEM;
    nrm_ = sc_;
    scale_ = sc_ + 2 * N;
    // A convergence check copies the residual estimates to the host and waits
    // for the stream: ~50 us of idle GPU, nothing against a step on 2^22 or
    // more (site, rhs) pairs (24^4 x 64: ~7 ms), so large batches check after
    // every step (24^4 x 64 FP16S: 50 -> 33 inner steps, 0.43 -> 0.27 s);
    // small ones every 10 (8^4 x 128: 30 steps either way, and every 8 took 40).
    check_every_ = ctx->V * (long)N >= (1L << 22) ? 1 : 10;

    bn2_.assign(2 * N, 0.0);
    rn2_.assign(2 * N, 0.0);
    resh_.assign(N, 0.0);
    rel_.assign(N, 1.0);
    target_.assign(N, 0.0);
    RET_IF(blas_norm2(ctx, b_, N, MPMC_FP64, nrm_));
    HIP_OR_RET(ctx, hipMemcpyAsync(bn2_.data(), nrm_, sizeof(double2) * N, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_RET(ctx, hipMemsetAsync(x_, 0, vb64_, ctx->stream));
    if (dc_) {
        RET_IF(defl_coeffs(ctx, defl_, b_, N, dc_, 1));
        RET_IF(defl_add(ctx, defl_, dc_, x_, N, 1.0));
    }
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < N; ++i)
        if (!std::isfinite(bn2_[2 * i])) return set_err(ctx, MPMC_ENUMERIC, "mpmc_solve: rhs %d is not finite", i);
    // The network is only a preconditioner: a cycle run with it that does not
    // cut some unconverged residual by 10% switches it off for the rest of the
    // solve, which then continues as plain (deflated) GMRES.
    use_net_ = net_ != nullptr;
    return MPMC_OK;
}

int Gmres::true_residual() {
    mpmc_ctx *ctx = ctx_;
    const int N = N_;
    RET_IF(wilson_launch_full(ctx, x_, b_, r_, nullptr, N, MPMC_FP64, make_double2(1, 0), make_double2(-1, 0),
                              make_double2(0, 0), 0, 0));
    RET_IF(blas_norm2(ctx, r_, N, MPMC_FP64, nrm_));
    HIP_OR_RET(ctx, hipMemcpyAsync(rn2_.data(), nrm_, sizeof(double2) * N, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    bool all = true;
    for (int i = 0; i < N; ++i) {
        if (!std::isfinite(rn2_[2 * i])) return set_err(ctx, MPMC_ENUMERIC, "mpmc_solve: residual %d is not finite", i);
        rel_[i] = bn2_[2 * i] > 0 ? std::sqrt(std::max(rn2_[2 * i], 0.0) / bn2_[2 * i]) : 0.0;
        if (rel_[i] > tol_) all = false;
    }
    converged_ = all;
    return MPMC_OK;
}

int Gmres::begin_cycle(bool *go) {
    mpmc_ctx *ctx = ctx_;
    const int N = N_, m = m_;
    *go = false;
    if (outer_ >= max_outer_) return MPMC_OK;
    ++outer_;
    RET_IF(true_residual());
    if (converged_) return MPMC_OK;
    if (use_net_ && !rel_start_.empty())
        for (int i = 0; i < N; ++i)
            if (rel_[i] > tol_ && rel_[i] > 0.9 * rel_start_[i]) use_net_ = false;
    if (dc_) {
        RET_IF(defl_coeffs(ctx, defl_, r_, N, dc_, 1));
        RET_IF(defl_add(ctx, defl_, dc_, x_, N, 1.0));
        RET_IF(true_residual());
        if (converged_) return MPMC_OK;
    }
    rel_start_ = rel_;
    cnet_ = use_net_ ? net_ : nullptr;
    if (snap_ && snap_->count < snap_->max) {   // r_k now; e_k = x* - x_k (FP64) at the end
        const size_t vb32 = vec_bytes(ctx, N, MPMC_FP32);
        RET_IF(blas_convert(ctx, r_, MPMC_FP64, (char *)snap_->R + (size_t)snap_->count * vb32, MPMC_FP32, N));
        HIP_OR_RET(ctx, hipMemcpyAsync((char *)xsnap_ + (size_t)snap_->count * vb64_, x_, vb64_,
                                       hipMemcpyDeviceToDevice, ctx->stream));
        ++snap_->count;
    }
    // inner targets: the final tolerance for an FP64 cycle; FP32 cycles
    // stop near single precision and the outer loop corrects the rest
    for (int i = 0; i < N; ++i) {
        const double rn = std::sqrt(std::max(rn2_[2 * i], 0.0)), bn = std::sqrt(std::max(bn2_[2 * i], 0.0));
        double t = 0.5 * tol_ * bn;
        if (inner_prec_ == MPMC_FP32) t = std::max(t, 2e-6 * rn);
        if (half_) t = std::max(t, 1e-3 * rn);   // FP16 basis: the Arnoldi relation holds to ~2^-11
        target_[i] = t;
    }
    if (half_) {
        RET_IF(blas_convert(ctx, r_, MPMC_FP64, w_, MPMC_FP32, N));
        RET_IF(blas_scale_rhs(ctx, w_, w_, N, MPMC_FP32, nrm_, 1));
        RET_IF(blas_convert(ctx, w_, MPMC_FP32, V_, MPMC_FP16S, N));
    } else {
        RET_IF(blas_convert(ctx, r_, MPMC_FP64, V_, inner_prec_, N));
        RET_IF(blas_scale_rhs(ctx, V_, V_, N, inner_prec_, nrm_, 1));
    }
    HIP_OR_RET(ctx, hipMemsetAsync(H_, 0, sizeof(double2) * (size_t)(m + 1) * (m + 1) * N, ctx->stream));
    k_init_g<<<grid_for((long)(m + 1) * N, 256), 256, 0, ctx->stream>>>((double2 *)g_, m, N, (const double2 *)nrm_);
    HIP_OR_RET(ctx, hipGetLastError());
    jdone_ = 0;
    *go = true;
    return MPMC_OK;
}

int Gmres::operand(int j, const void **opin) {
    *opin = basis(j);
    if (cnet_) {   // z_j = N v_j (FP32; an FP16S basis vector is widened first)
        const void *vj = basis(j);
        if (half_) {
            RET_IF(blas_convert(ctx_, vj, MPMC_FP16S, tq_, MPMC_FP32, N_));
            vj = tq_;
        }
        void *zj = (char *)Zb_ + (size_t)j * vbi_;
        RET_IF(net_apply_internal(ctx_, cnet_, vj, zj, N_));
        *opin = zj;
    }
    return MPMC_OK;
}

int Gmres::matvec(int j, const void *opin) {
    mpmc_ctx *ctx = ctx_;
    const int N = N_;
    if (pp_) {   // w = M p(M) v_j
        const void *src = basis(j);
        if (half_) {
            RET_IF(blas_convert(ctx, basis(j), MPMC_FP16S, tq_, MPMC_FP32, N));
            src = tq_;
        }
        RET_IF(poly_apply_internal(ctx, pp_, src, tp_, N, pw_));
        return wilson_launch_full(ctx, tp_, nullptr, w_, nullptr, N, pw_, make_double2(0, 0), make_double2(1, 0),
                                  make_double2(0, 0), 0, 0);
    }
    if (half_ && !cnet_) return wilson_apply_h2f(ctx, basis(j), w_, N);
    return wilson_launch_full(ctx, opin, nullptr, w_, nullptr, N, pw_, make_double2(0, 0), make_double2(1, 0),
                              make_double2(0, 0), 0, 0);
}

int Gmres::orthogonalize(int j, bool *more) {
    mpmc_ctx *ctx = ctx_;
    const int N = N_, m = m_;
    double *Hcol = H_ + 2 * (size_t)j * (m + 1) * N;
    // FP32 and FP16S cycles stop at 2e-6 and 1e-3 of their start, far above
    // the loss of orthogonality of one classical projection in FP32
    // arithmetic; FP64 cycles run to the final tolerance and project twice
    const bool once = ctx->solve_gs_passes == 1 || (ctx->solve_gs_passes == 0 && inner_prec_ != MPMC_FP64);
    if (once && half_) {   // w - V h goes straight into the FP16S basis slot j+1 (unnormalised)
        RET_IF(blas_multi_dot_h(ctx, V_, vbb_, j + 1, w_, N, Hcol, 0));
        RET_IF(blas_multi_axpy_h(ctx, V_, vbb_, j + 1, w_, N, Hcol, N, -1.0, nrm_, basis(j + 1)));
    } else if (once) {
        RET_IF(blas_multi_dot(ctx, V_, vstride_, N, j + 1, w_, N, pw_, Hcol, 0, 0));
        RET_IF(blas_multi_axpy(ctx, V_, vstride_, N, j + 1, w_, N, pw_, Hcol, N, -1.0, nrm_));
    } else if (half_) {
        RET_IF(blas_multi_dot_h(ctx, V_, vbb_, j + 1, w_, N, Hcol, 0));
        RET_IF(blas_multi_axpy_h(ctx, V_, vbb_, j + 1, w_, N, Hcol, N, -1.0, nullptr));
        RET_IF(blas_multi_dot_h(ctx, V_, vbb_, j + 1, w_, N, h2_, 0));
        RET_IF(blas_multi_axpy_h(ctx, V_, vbb_, j + 1, w_, N, h2_, N, -1.0, nrm_));
    } else {
        RET_IF(blas_multi_dot(ctx, V_, vstride_, N, j + 1, w_, N, pw_, Hcol, 0, 0));
        RET_IF(blas_multi_axpy_dot(ctx, V_, vstride_, j + 1, w_, N, pw_, Hcol, N, -1.0, h2_));
        RET_IF(blas_multi_axpy(ctx, V_, vstride_, N, j + 1, w_, N, pw_, h2_, N, -1.0, nrm_));
    }
    k_finalize_batch<<<grid_for(N, 64), 64, 0, ctx->stream>>>((double2 *)Hcol, once ? nullptr : (const double2 *)h2_,
                                                              j, N, (const double2 *)nrm_, (double2 *)scale_);
    HIP_OR_RET(ctx, hipGetLastError());
    if (once && half_) {   // v_{j+1} = (w - V h) / h_{j+1,j}: only the per-(site, rhs) scales change
        RET_IF(blas_scale_h(ctx, basis(j + 1), N, scale_));
    } else if (half_) {    // v_{j+1} = w / h_{j+1,j} straight into the FP16S basis (w is not needed after)
        RET_IF(blas_convert_scaled_h(ctx, w_, basis(j + 1), N, scale_));
    } else {
        RET_IF(blas_scale_rhs(ctx, w_, basis(j + 1), N, inner_prec_, scale_, 0));
    }
    RET_IF(dense_givens_step(ctx, H_, m + 1, j, N, cs_, g_, res_));
    jdone_ = j + 1;
    *more = j + 1 < m;
    if ((j + 1) % check_every_ == 0 && j + 1 < m) {
        HIP_OR_RET(ctx, hipMemcpyAsync(resh_.data(), res_, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
        bool all = true;
        for (int i = 0; i < N; ++i) all = all && resh_[i] <= target_[i];
        if (all) *more = false;
    }
    return MPMC_OK;
}

int Gmres::end_cycle() {
    mpmc_ctx *ctx = ctx_;
    const int N = N_, m = m_;
    RET_IF(dense_backsolve(ctx, H_, m + 1, jdone_, N, g_, y_));
    HIP_OR_RET(ctx, hipMemsetAsync(corr_, 0, vbi_, ctx->stream));
    if (cnet_)   // flexible GMRES: e = Z y (FP32)
        RET_IF(blas_multi_axpy(ctx, Zb_, vstride_, N, jdone_, corr_, N, pw_, y_, N, 1.0, nullptr));
    else if (half_)
        RET_IF(blas_multi_axpy_h(ctx, V_, vbb_, jdone_, corr_, N, y_, N, 1.0, nullptr));
    else
        RET_IF(blas_multi_axpy(ctx, V_, vstride_, N, jdone_, corr_, N, inner_prec_, y_, N, 1.0, nullptr));
    if (pp_) {   // correction p(M) V y
        RET_IF(poly_apply_internal(ctx, pp_, corr_, tp_, N, pw_));
        HIP_OR_RET(ctx, hipMemcpyAsync(corr_, tp_, vbi_, hipMemcpyDeviceToDevice, ctx->stream));
    }
    // x += e (in FP64)
    RET_IF(blas_convert(ctx, corr_, pw_, r_, MPMC_FP64, N));
    RET_IF(blas_axpby(ctx, r_, x_, N, MPMC_FP64, make_double2(1, 0), make_double2(1, 0)));
    total_ += jdone_;
    return MPMC_OK;
}

int Gmres::finish(int *iters_out, double *relres_host) {
    mpmc_ctx *ctx = ctx_;
    const int N = N_;
    if (!converged_) RET_IF(true_residual());
    if (snap_ && snap_->count > 0) {
        const size_t vb32 = vec_bytes(ctx, N, MPMC_FP32);
        for (int k = 0; k < snap_->count; ++k) {
            void *xk = (char *)xsnap_ + (size_t)k * vb64_;
            RET_IF(blas_axpby(ctx, x_, xk, N, MPMC_FP64, make_double2(1, 0), make_double2(-1, 0)));
            RET_IF(blas_convert(ctx, xk, MPMC_FP64, (char *)snap_->E + (size_t)k * vb32, MPMC_FP32, N));
        }
    }
    if (iters_out) *iters_out = total_;
    if (relres_host)
        for (int i = 0; i < N; ++i) relres_host[i] = rel_[i];
    if (!converged_)
        return set_err(ctx, MPMC_ENOCONV, "mpmc_solve: not converged after %d outer cycles", max_outer_);
    return MPMC_OK;
}

}  // namespace

int solve_internal(mpmc_ctx *ctx, const void *b, void *x, int N, const mpmc_defl *defl, const mpmc_net *net,
                   int m, double tol, int inner_prec, int max_outer, int *iters_out, double *relres_host,
                   SolveSnap *snap, const mpmc_poly *pp) {
    Gmres G(ctx, b, x, N, defl, net, m, tol, inner_prec, max_outer, snap, pp);
    RET_IF(G.init());
    for (;;) {
        bool go = false;
        RET_IF(G.begin_cycle(&go));
        if (!go) break;
        for (int j = 0; j < m; ++j) {
            const void *opin = nullptr;
            RET_IF(G.operand(j, &opin));
            RET_IF(G.matvec(j, opin));
            bool more = false;
            RET_IF(G.orthogonalize(j, &more));
            if (!more) break;
        }
        RET_IF(G.end_cycle());
    }
    return G.finish(iters_out, relres_host);
}

MPMC_API int mpmc_solve_batch(mpmc_ctx *const *ctxs, int count, const void *const *b, void *const *x, int nrhs,
                              const mpmc_defl *const *defl, const mpmc_net *const *net, int restart, double tol,
                              int inner_prec, int max_outer, int *iters_host, double *relres_host) {
    if (!ctxs || !ctxs[0]) return MPMC_EINVAL;
    mpmc_ctx *c0 = ctxs[0];
    if (count < 1 || count > kSolveBatchMax || !b || !x || nrhs < 64 || nrhs % 64 != 0 || restart < 1 ||
        restart > 400 || !(tol > 0) || max_outer < 1 || (inner_prec != MPMC_FP64 && inner_prec != MPMC_FP32))
        return set_err(c0, MPMC_EINVAL, "mpmc_solve_batch: bad argument");
    for (int i = 0; i < count; ++i) {
        const mpmc_ctx *c = ctxs[i];
        if (!c || !b[i] || !x[i] || b[i] == x[i] || c->device != c0->device || c->stream != c0->stream ||
            c->V % 4 != 0)
            return set_err(c0, MPMC_EINVAL, "mpmc_solve_batch: lattice %d: null, aliasing, other device or stream, "
                                            "or V %% 4 != 0", i);
        for (int k = 0; k < i; ++k)
            if (ctxs[k] == c) return set_err(c0, MPMC_EINVAL, "mpmc_solve_batch: context %d appears twice", i);
        if (defl && defl[i] && defl[i]->ctx != c)
            return set_err(c0, MPMC_ESTATE, "mpmc_solve_batch: deflation set %d belongs to another context", i);
    }
    std::vector<std::unique_ptr<Gmres>> G;
    for (int i = 0; i < count; ++i) {
        G.emplace_back(new Gmres(ctxs[i], b[i], x[i], nrhs, defl ? defl[i] : nullptr, net ? net[i] : nullptr, restart,
                                 tol, inner_prec, max_outer, nullptr, nullptr));
        RET_IF(G.back()->init());
    }
    std::vector<char> live(count, 1);
    for (;;) {
        std::vector<int> act;
        for (int i = 0; i < count; ++i) {
            if (!live[i]) continue;
            bool go = false;
            RET_IF(G[i]->begin_cycle(&go));
            if (go) act.push_back(i);
            else live[i] = 0;
        }
        if (act.empty()) break;
        std::vector<int> run = act;
        for (int j = 0; j < restart && !run.empty(); ++j) {
            mpmc_ctx *cs[kSolveBatchMax];
            const void *xs[kSolveBatchMax];
            void *ys[kSolveBatchMax];
            for (size_t k = 0; k < run.size(); ++k) {
                RET_IF(G[run[k]]->operand(j, &xs[k]));
                ys[k] = G[run[k]]->wvec();
                cs[k] = ctxs[run[k]];
            }
            // one launch applies M on every lattice still iterating
            RET_IF(mpmc_apply_M_batch(cs, xs, ys, (int)run.size(), nrhs, inner_prec, 0, MPMC_THETA_I));
            std::vector<int> next;
            for (int i : run) {
                bool more = false;
                RET_IF(G[i]->orthogonalize(j, &more));
                if (more) next.push_back(i);
            }
            run = next;
        }
        for (int i : act) RET_IF(G[i]->end_cycle());
    }
    int rc = MPMC_OK;
    for (int i = 0; i < count; ++i) {
        const int ri = G[i]->finish(iters_host ? iters_host + i : nullptr, relres_host ? relres_host + (size_t)i * nrhs
                                                                                     : nullptr);
        if (rc == MPMC_OK && ri != MPMC_OK) {
            rc = ri;
            if (i > 0) set_err(c0, ri, "mpmc_solve_batch: lattice %d: %s", i, mpmc_last_error(ctxs[i]));
        }
    }
    return rc;
}

MPMC_API int mpmc_solve_pairs(mpmc_ctx *ctx, const void *b, void *x, int nrhs, const mpmc_defl *defl, int restart,
                              double tol, int inner_prec, int max_outer, void *R_snap, void *E_snap, int max_snap,
                              int *nsnap_host, int *iters_host, double *relres_host) {
    if (!ctx) return MPMC_EINVAL;
    if (!b || !x || nrhs < 1 || restart < 1 || restart > 400 || !(tol > 0) || max_outer < 1 || !R_snap || !E_snap ||
        max_snap < 1 || !nsnap_host)
        return set_err(ctx, MPMC_EINVAL, "mpmc_solve_pairs: bad argument");
    if (b == x) return set_err(ctx, MPMC_EINVAL, "mpmc_solve_pairs: b and x must not alias");
    if (defl && defl->ctx != ctx) return set_err(ctx, MPMC_ESTATE, "deflation set belongs to another context");
    SolveSnap sn{R_snap, E_snap, max_snap, 0};
    const int rc = solve_internal(ctx, b, x, nrhs, defl, nullptr, restart, tol, inner_prec, max_outer, iters_host,
                                  relres_host, &sn, nullptr);
    *nsnap_host = sn.count;
    return rc;
}

MPMC_API int mpmc_set_solve_gs_passes(mpmc_ctx *ctx, int passes) {
    if (!ctx) return MPMC_EINVAL;
    if (passes < 0 || passes > 2) return set_err(ctx, MPMC_EINVAL, "mpmc_set_solve_gs_passes: 0, 1 or 2");
    ctx->solve_gs_passes = passes;
    return MPMC_OK;
}

MPMC_API int mpmc_solve(mpmc_ctx *ctx, const void *b, void *x, int nrhs, const mpmc_defl *defl, const mpmc_net *net,
                        int restart, double tol, int inner_prec, int max_outer, int *iters_host, double *relres_host) {
    if (!ctx) return MPMC_EINVAL;
    if (!b || !x || nrhs < 1 || restart < 1 || restart > 400 || !(tol > 0) || max_outer < 1)
        return set_err(ctx, MPMC_EINVAL, "mpmc_solve: bad argument");
    if (b == x) return set_err(ctx, MPMC_EINVAL, "mpmc_solve: b and x must not alias");
    if (defl && defl->ctx != ctx) return set_err(ctx, MPMC_ESTATE, "deflation set belongs to another context");
    return solve_internal(ctx, b, x, nrhs, defl, net, restart, tol, inner_prec, max_outer, iters_host, relres_host,
                          nullptr, nullptr);
}

MPMC_API int mpmc_solve_pp(mpmc_ctx *ctx, const void *b, void *x, int nrhs, const mpmc_defl *defl, const mpmc_poly *pp,
                           int restart, double tol, int inner_prec, int max_outer, int *iters_host,
                           double *relres_host) {
    if (!ctx) return MPMC_EINVAL;
    if (!b || !x || !pp || nrhs < 1 || restart < 1 || restart > 400 || !(tol > 0) || max_outer < 1)
        return set_err(ctx, MPMC_EINVAL, "mpmc_solve_pp: bad argument");
    if (b == x) return set_err(ctx, MPMC_EINVAL, "mpmc_solve_pp: b and x must not alias");
    if (defl && defl->ctx != ctx) return set_err(ctx, MPMC_ESTATE, "deflation set belongs to another context");
    return solve_internal(ctx, b, x, nrhs, defl, nullptr, restart, tol, inner_prec, max_outer, iters_host, relres_host,
                          nullptr, pp);
}

MPMC_API int mpmc_set_level_solve_poly(mpmc_ctx *ctx, const mpmc_poly *pp) {
    if (!ctx) return MPMC_EINVAL;
    if (pp && pp->ctx != ctx) return set_err(ctx, MPMC_ESTATE, "polynomial belongs to another context");
    ctx->level_pp = pp;
    return MPMC_OK;
}
