// Context management, layout conversion and Z(4) noise generation.
#include <cstdarg>
#include <cstring>

#include "common.h"

static thread_local std::string g_create_err;

int set_err(const mpmc_ctx *ctx, int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        const_cast<mpmc_ctx *>(ctx)->err = buf;
    else
        g_create_err = buf;
    return code;
}

void *ws_get(mpmc_ctx *ctx, int slot, size_t bytes) {
    if (slot < 0 || slot >= WS_NSLOTS) return nullptr;
    WsBuf &b = ctx->ws[slot];
    if (bytes == 0) bytes = 256;
    if (b.bytes < bytes) {
        if (b.ptr) {
            // the stream may still use the old buffer
            hipStreamSynchronize(ctx->stream);
            hipFree(b.ptr);
            b.ptr = nullptr;
            b.bytes = 0;
        }
        size_t want = (bytes + 4095) & ~size_t(4095);
        if (hipMalloc(&b.ptr, want) != hipSuccess) {
            b.ptr = nullptr;
            set_err(ctx, MPMC_ENOMEM, "workspace slot %d: hipMalloc(%zu) failed", slot, want);
            return nullptr;
        }
        b.bytes = want;
    }
    return b.ptr;
}

// Frees the cached scratch buffers of stack levels >= from (none of them is
// in use: live Scratch objects only hold levels below ctx->top).
static void release_stack_from(mpmc_ctx *ctx, int from) {
    bool synced = false;
    for (int i = from; i < (int)ctx->stack.size(); ++i) {
        WsBuf &b = ctx->stack[i];
        if (!b.ptr) continue;
        if (!synced) {
            hipStreamSynchronize(ctx->stream);
            synced = true;
        }
        hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
}

void *stack_get(mpmc_ctx *ctx, size_t bytes) {
    if ((int)ctx->stack.size() <= ctx->top) ctx->stack.resize(ctx->top + 1);
    WsBuf &b = ctx->stack[ctx->top];
    if (bytes == 0) bytes = 256;
    if (b.bytes < bytes) {
        if (b.ptr) {
            hipStreamSynchronize(ctx->stream);
            if (ctx->gstream) hipStreamSynchronize(ctx->gstream);
            graphs_clear(ctx);   // captured recurrences may refer to this buffer
            hipFree(b.ptr);
            b.ptr = nullptr;
            b.bytes = 0;
        }
        size_t want = (bytes + 4095) & ~size_t(4095);
        if (hipMalloc(&b.ptr, want) != hipSuccess) {
            // retry once after dropping the cached buffers of deeper levels
            (void)hipGetLastError();
            release_stack_from(ctx, ctx->top + 1);
            if (hipMalloc(&b.ptr, want) != hipSuccess) {
                (void)hipGetLastError();
                b.ptr = nullptr;
                set_err(ctx, MPMC_ENOMEM, "scratch: hipMalloc(%zu) failed", want);
                return nullptr;
            }
        }
        b.bytes = want;
    }
    ctx->top++;
    return b.ptr;
}

MPMC_API int mpmc_release_workspace(mpmc_ctx *ctx) {
    if (!ctx) return MPMC_EINVAL;
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->gstream) HIP_OR_RET(ctx, hipStreamSynchronize(ctx->gstream));
    graphs_clear(ctx);   // captured recurrences refer to the buffers released here
    release_stack_from(ctx, ctx->top);
    for (auto &b : ctx->ws) {
        if (b.ptr) hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    return MPMC_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t fp16s_scale_offset(const mpmc_ctx *ctx, int nrhs) { return align256((size_t)ctx->V * 12 * nrhs * 4); }

size_t vec_bytes(const mpmc_ctx *ctx, int nrhs, int prec) {
    const size_t elems = (size_t)ctx->V * 12 * nrhs;
    switch (prec) {
        case MPMC_FP64: return elems * 16;
        case MPMC_FP32: return elems * 8;
        case MPMC_FP16S: return fp16s_scale_offset(ctx, nrhs) + (size_t)ctx->V * nrhs * 4;
    }
    return 0;
}

VecRef vref(const mpmc_ctx *ctx, const void *p, int nrhs, int prec) {
    VecRef r;
    r.d = const_cast<void *>(p);
    r.sc = prec == MPMC_FP16S ? (float *)((char *)p + fp16s_scale_offset(ctx, nrhs)) : nullptr;
    return r;
}

// ------------------------------------------------------------ create --

static void build_neighbours(const int L[4], int t_anti, std::vector<int> &nbr) {
    const long V = (long)L[0] * L[1] * L[2] * L[3];
    nbr.resize(V * 8);
    for (long s = 0; s < V; ++s) {
        int c[4];
        long q = s;
        for (int mu = 0; mu < 4; ++mu) {
            c[mu] = (int)(q % L[mu]);
            q /= L[mu];
        }
        for (int dir = 0; dir < 2; ++dir)
            for (int mu = 0; mu < 4; ++mu) {
                int cc[4] = {c[0], c[1], c[2], c[3]};
                bool crossed;
                if (dir == 0) {
                    cc[mu] = (c[mu] + 1) % L[mu];
                    crossed = (c[mu] == L[mu] - 1);
                } else {
                    cc[mu] = (c[mu] + L[mu] - 1) % L[mu];
                    crossed = (c[mu] == 0);
                }
                long t = cc[0] + (long)L[0] * (cc[1] + (long)L[1] * (cc[2] + (long)L[2] * cc[3]));
                unsigned v = (unsigned)t;
                if (t_anti && mu == 3 && crossed) v |= 0x80000000u;
                nbr[s * 8 + dir * 4 + mu] = (int)v;
            }
    }
}

// Traversal order of the blocked Wilson kernels: the lattice is cut into 4D
// blocks (extent 4 along each direction whose length is a multiple of 4,
// else 2, else 1), blocks in lexicographic order, sites lexicographic inside a
// block.  Consecutive workgroups then work on compact 4D regions, so the
// neighbours a wavefront reads were mostly fetched by nearby wavefronts of
// the same XCD shortly before.
static void build_site_order(const int L[4], std::vector<int> &order) {
    int b[4], nb[4];
    for (int mu = 0; mu < 4; ++mu) {
        b[mu] = L[mu] % 4 == 0 ? 4 : (L[mu] % 2 == 0 ? 2 : 1);
        nb[mu] = L[mu] / b[mu];
    }
    const long V = (long)L[0] * L[1] * L[2] * L[3];
    order.resize(V);
    long q = 0;
    for (int k3 = 0; k3 < nb[3]; ++k3)
        for (int k2 = 0; k2 < nb[2]; ++k2)
            for (int k1 = 0; k1 < nb[1]; ++k1)
                for (int k0 = 0; k0 < nb[0]; ++k0)
                    for (int i3 = 0; i3 < b[3]; ++i3)
                        for (int i2 = 0; i2 < b[2]; ++i2)
                            for (int i1 = 0; i1 < b[1]; ++i1)
                                for (int i0 = 0; i0 < b[0]; ++i0) {
                                    const long x = k0 * b[0] + i0, y = k1 * b[1] + i1, z = k2 * b[2] + i2,
                                               t = k3 * b[3] + i3;
                                    order[q++] = (int)(x + L[0] * (y + (long)L[1] * (z + (long)L[2] * t)));
                                }
}

// Replace the traversal order of the blocked kernels (NULL: the default
// blocked order).  The order must be a permutation of the sites.
MPMC_API int mpmc_set_site_order(mpmc_ctx *ctx, const int *order_host) {
    if (!ctx) return MPMC_EINVAL;
    std::vector<int> order;
    if (order_host) {
        order.assign(order_host, order_host + ctx->V);
        std::vector<char> seen(ctx->V, 0);
        for (long i = 0; i < ctx->V; ++i) {
            const int s = order[i];
            if (s < 0 || s >= ctx->V || seen[s])
                return set_err(ctx, MPMC_EINVAL, "mpmc_set_site_order: entry %ld (%d) is not a permutation", i, s);
            seen[s] = 1;
        }
    } else {
        build_site_order(ctx->dims, order);
    }
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    HIP_OR_RET(ctx, hipMemcpy(ctx->site_order, order.data(), (size_t)ctx->V * sizeof(int), hipMemcpyHostToDevice));
    return MPMC_OK;
}

MPMC_API int mpmc_create(const int dims[4], double kappa, int t_antiperiodic, const double *links_host,
                         void *stream, mpmc_ctx **out) {
    if (!dims || !links_host || !out) return set_err(nullptr, MPMC_EINVAL, "mpmc_create: null argument");
    *out = nullptr;
    long V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (dims[mu] < 1 || dims[mu] > 1024) return set_err(nullptr, MPMC_EINVAL, "mpmc_create: bad dims[%d]=%d", mu, dims[mu]);
        V *= dims[mu];
    }
    if (V > (1L << 30)) return set_err(nullptr, MPMC_EINVAL, "mpmc_create: lattice too large");
    if (!(kappa == kappa)) return set_err(nullptr, MPMC_EINVAL, "mpmc_create: kappa is NaN");
    mpmc_ctx *c = new mpmc_ctx();
    memcpy(c->dims, dims, sizeof c->dims);
    c->V = V;
    c->n = 12 * V;
    c->kappa = kappa;
    c->t_antiperiodic = t_antiperiodic ? 1 : 0;
    c->stream = (hipStream_t)stream;
    c->links64 = nullptr;
    c->links32 = nullptr;
    c->nbr = nullptr;
    c->site_order = nullptr;
    c->mvps = 0;
    c->ws.resize(WS_NSLOTS);
    c->top = 0;
    c->timing = 0;
    hipGetDevice(&c->device);
    hipDeviceProp_t prop;
    c->num_cu = (hipGetDeviceProperties(&prop, c->device) == hipSuccess) ? prop.multiProcessorCount : 256;

    const size_t nl = (size_t)V * 4 * 9;
    std::vector<float> l32(nl * 2);
    for (size_t i = 0; i < nl * 2; ++i) l32[i] = (float)links_host[i];
    std::vector<int> nbr;
    build_neighbours(dims, c->t_antiperiodic, nbr);
    std::vector<int> order;
    build_site_order(dims, order);
    hipError_t e = hipMalloc(&c->links64, nl * 16);
    if (e == hipSuccess) e = hipMalloc(&c->links32, nl * 8);
    if (e == hipSuccess) e = hipMalloc(&c->nbr, (size_t)V * 8 * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&c->site_order, (size_t)V * sizeof(int));
    if (e == hipSuccess) e = hipMemcpy(c->links64, links_host, nl * 16, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->links32, l32.data(), nl * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->nbr, nbr.data(), (size_t)V * 8 * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->site_order, order.data(), (size_t)V * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        set_err(nullptr, MPMC_ENOMEM, "mpmc_create: %s", hipGetErrorString(e));
        mpmc_destroy(c);
        return MPMC_ENOMEM;
    }
    // the device address of this device's copy of the fixed no-allocation
    // scratch array, taken once with the device current
    if (!noalloc_scratch(c->device)) {
        set_err(nullptr, MPMC_EHIP, "mpmc_create: no device address for the scratch array of mpmc_apply_poly_noalloc");
        mpmc_destroy(c);
        return MPMC_EHIP;
    }
    *out = c;
    return MPMC_OK;
}

MPMC_API void mpmc_destroy(mpmc_ctx *ctx) {
    if (!ctx) return;
    hipStreamSynchronize(ctx->stream);
    if (ctx->gstream) {
        hipStreamSynchronize(ctx->gstream);
        graphs_clear(ctx);
        hipStreamDestroy(ctx->gstream);
        for (auto e : ctx->gev)
            if (e) hipEventDestroy(e);
    }
    if (ctx->links64) hipFree(ctx->links64);
    if (ctx->links32) hipFree(ctx->links32);
    if (ctx->nbr) hipFree(ctx->nbr);
    if (ctx->site_order) hipFree(ctx->site_order);
    for (auto &b : ctx->ws)
        if (b.ptr) hipFree(b.ptr);
    for (auto &b : ctx->stack)
        if (b.ptr) hipFree(b.ptr);
    for (auto e : ctx->ev_pool) hipEventDestroy(e);
    delete ctx;
}

MPMC_API const char *mpmc_last_error(const mpmc_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

MPMC_API int mpmc_set_stream(mpmc_ctx *ctx, void *stream) {
    if (!ctx) return MPMC_EINVAL;
    hipStreamSynchronize(ctx->stream);
    ctx->stream = (hipStream_t)stream;
    return MPMC_OK;
}

MPMC_API int mpmc_vector_bytes(const mpmc_ctx *ctx, int nrhs, int prec, size_t *bytes) {
    if (!ctx || !bytes || nrhs < 1 || !prec_ok(prec)) return ctx ? set_err(ctx, MPMC_EINVAL, "mpmc_vector_bytes: bad argument") : MPMC_EINVAL;
    *bytes = vec_bytes(ctx, nrhs, prec);
    return MPMC_OK;
}

MPMC_API int mpmc_mvp_count(const mpmc_ctx *ctx, uint64_t *mvps) {
    if (!ctx || !mvps) return MPMC_EINVAL;
    *mvps = ctx->mvps;
    return MPMC_OK;
}

MPMC_API int mpmc_mvp_reset(mpmc_ctx *ctx) {
    if (!ctx) return MPMC_EINVAL;
    ctx->mvps = 0;
    return MPMC_OK;
}

// ------------------------------------------------------ pack / unpack --
// One thread per (site, rhs): 12 canonical components <-> 12 internal ones.

template <int P>
__global__ void k_pack(const double2 *__restrict__ canon, VecRef out, long V, int N) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= V * N) return;
    const long s = t / N;
    const int r = (int)(t - s * N);
    using R = typename Store<P>::real;
    cpx<double> v[12];
    double mx = 0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        double2 c = canon[((long)r * V + s) * 12 + k];
        v[k] = mk(c.x, c.y);
        mx = fmax(mx, fmax(fabs(c.x), fabs(c.y)));
    }
    if constexpr (P == MPMC_FP16S) {
        const float sc = (float)mx;
        const float inv = sc > 0 ? 1.0f / sc : 0.0f;
        __half2 *d = reinterpret_cast<__half2 *>(out.d);
#pragma unroll
        for (int k = 0; k < 12; ++k)
            d[(s * 12 + k) * N + r] = __floats2half2_rn((float)v[k].re * inv, (float)v[k].im * inv);
        out.sc[s * N + r] = sc;
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) Store<P>::st(out.d, (s * 12 + k) * N + r, mk((R)v[k].re, (R)v[k].im));
    }
}

template <int P>
__global__ void k_unpack(VecRef in, double2 *__restrict__ canon, long V, int N) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= V * N) return;
    const long s = t / N;
    const int r = (int)(t - s * N);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        auto v = Store<P>::ld(in.d, in.sc, (s * 12 + k) * N + r, s * N + r);
        canon[((long)r * V + s) * 12 + k] = make_double2((double)v.re, (double)v.im);
    }
}

MPMC_API int mpmc_pack(mpmc_ctx *ctx, const void *canon, void *internal, int nrhs, int prec) {
    if (!ctx) return MPMC_EINVAL;
    if (!canon || !internal || nrhs < 1 || !prec_ok(prec)) return set_err(ctx, MPMC_EINVAL, "mpmc_pack: bad argument");
    const long work = ctx->V * nrhs;
    VecRef o = vref(ctx, internal, nrhs, prec);
    const int B = 256;
    if (prec == MPMC_FP64) k_pack<MPMC_FP64><<<grid_for(work, B), B, 0, ctx->stream>>>((const double2 *)canon, o, ctx->V, nrhs);
    else if (prec == MPMC_FP32) k_pack<MPMC_FP32><<<grid_for(work, B), B, 0, ctx->stream>>>((const double2 *)canon, o, ctx->V, nrhs);
    else k_pack<MPMC_FP16S><<<grid_for(work, B), B, 0, ctx->stream>>>((const double2 *)canon, o, ctx->V, nrhs);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

MPMC_API int mpmc_unpack(mpmc_ctx *ctx, const void *internal, void *canon, int nrhs, int prec) {
    if (!ctx) return MPMC_EINVAL;
    if (!canon || !internal || nrhs < 1 || !prec_ok(prec)) return set_err(ctx, MPMC_EINVAL, "mpmc_unpack: bad argument");
    const long work = ctx->V * nrhs;
    VecRef i = vref(ctx, internal, nrhs, prec);
    const int B = 256;
    if (prec == MPMC_FP64) k_unpack<MPMC_FP64><<<grid_for(work, B), B, 0, ctx->stream>>>(i, (double2 *)canon, ctx->V, nrhs);
    else if (prec == MPMC_FP32) k_unpack<MPMC_FP32><<<grid_for(work, B), B, 0, ctx->stream>>>(i, (double2 *)canon, ctx->V, nrhs);
    else k_unpack<MPMC_FP16S><<<grid_for(work, B), B, 0, ctx->stream>>>(i, (double2 *)canon, ctx->V, nrhs);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

// -------------------------------------------------------------- noise --

template <int P>
// N noise vectors into columns off .. off+N-1 of an operand of ld right-hand sides
__global__ void k_noise(uint64_t seed, uint32_t stream, uint64_t first, VecRef out, long V, int N, int ld, int off) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= V * N) return;
    const long s = t / N;
    const int r = (int)(t - s * N);
    const uint32_t sym = z4_site_symbols(seed, stream, (uint32_t)(first + r), s);
    using R = typename Store<P>::real;
    if constexpr (P == MPMC_FP16S) {
        __half2 *d = reinterpret_cast<__half2 *>(out.d);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            cpx<float> v = z4_value<float>((sym >> (2 * k)) & 3u);
            d[(s * 12 + k) * ld + off + r] = __floats2half2_rn(v.re, v.im);
        }
        out.sc[s * ld + off + r] = 1.0f;
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k)
            Store<P>::st(out.d, (s * 12 + k) * ld + off + r, z4_value<R>((sym >> (2 * k)) & 3u));
    }
}

int launch_noise(mpmc_ctx *ctx, uint64_t seed, uint32_t stream, uint64_t first, int nrhs, int prec, void *internal,
                 int ld, int off) {
    if (ld <= 0) ld = nrhs;
    const long work = ctx->V * nrhs;
    VecRef o = vref(ctx, internal, ld, prec);
    const int B = 256;
    if (prec == MPMC_FP64)
        k_noise<MPMC_FP64><<<grid_for(work, B), B, 0, ctx->stream>>>(seed, stream, first, o, ctx->V, nrhs, ld, off);
    else if (prec == MPMC_FP32)
        k_noise<MPMC_FP32><<<grid_for(work, B), B, 0, ctx->stream>>>(seed, stream, first, o, ctx->V, nrhs, ld, off);
    else
        k_noise<MPMC_FP16S><<<grid_for(work, B), B, 0, ctx->stream>>>(seed, stream, first, o, ctx->V, nrhs, ld, off);
    HIP_OR_RET(ctx, hipGetLastError());
    return MPMC_OK;
}

MPMC_API int mpmc_noise(mpmc_ctx *ctx, uint64_t seed, uint32_t stream, uint64_t first, int nrhs, int prec,
                        void *internal) {
    if (!ctx) return MPMC_EINVAL;
    if (!internal || nrhs < 1 || !prec_ok(prec) || first + (uint64_t)nrhs > 0x100000000ull)
        return set_err(ctx, MPMC_EINVAL, "mpmc_noise: bad argument");
    return launch_noise(ctx, seed, stream, first, nrhs, prec, internal);
}

// ------------------------------------------------------------- timing --

int timing_begin(mpmc_ctx *ctx) {
    if (!ctx->timing) return -1;
    const int i = ctx->timed_events;
    ctx->timed_events += 2;
    while ((int)ctx->ev_pool.size() < i + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        ctx->ev_pool.push_back(e);
    }
    if (hipEventRecord(ctx->ev_pool[i], ctx->stream) != hipSuccess) return -1;
    return i;
}

void timing_end(mpmc_ctx *ctx, int ev0, int prec, double bytes) {
    if (ev0 < 0) return;
    if (hipEventRecord(ctx->ev_pool[ev0 + 1], ctx->stream) != hipSuccess) return;
    ctx->timed.push_back({ev0, ev0 + 1, prec, bytes});
}

void timing_count(mpmc_ctx *ctx, int prec, double bytes) {
    if (ctx->timing) ctx->timed.push_back({-1, -1, prec, bytes});
}

MPMC_API int mpmc_timing_enable(mpmc_ctx *ctx, int on) {
    if (!ctx) return MPMC_EINVAL;
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    ctx->timing = on ? 1 : 0;
    ctx->timed.clear();
    ctx->timed_events = 0;
    return MPMC_OK;
}

MPMC_API int mpmc_timing_read(mpmc_ctx *ctx, int prec, uint64_t *launches, double *ms, double *bytes) {
    if (!ctx || !launches || !ms || !bytes) return MPMC_EINVAL;
    HIP_OR_RET(ctx, hipStreamSynchronize(ctx->stream));
    uint64_t cnt = 0;
    double t = 0, b = 0;
    for (const auto &L : ctx->timed) {
        // L.prec = precision | kind; prec selects a precision, optionally one kind
        if ((L.prec & 15) != (prec & 15)) continue;
        if ((prec & ~15) && !(L.prec & prec & ~15)) continue;
        float e = 0;
        if (L.ev0 >= 0) HIP_OR_RET(ctx, hipEventElapsedTime(&e, ctx->ev_pool[L.ev0], ctx->ev_pool[L.ev1]));
        ++cnt;
        t += e;
        b += L.bytes;
    }
    *launches = cnt;
    *ms = t;
    *bytes = b;
    return MPMC_OK;
}
