/*
 * mpmc.h -- C ABI of libmpmc.so: Multipolynomial Monte Carlo trace estimation
 * of Tr(Theta M^-1) for the Wilson-Dirac matrix M on one AMD Instinct MI355X
 * (gfx950).  Every vector operation and every small dense eigenproblem behind
 * these calls is a HIP kernel of this library; there is no CPU fallback.  The
 * host code does only O(k d) scalar work: the scalar polynomial values
 * p(lambda_i) of the deflation coefficients (mpmc_poly_eval, the level
 * estimators), the sums of k exact-correction terms and of the per-probe
 * values of mpmc_poly_trace*, and the selection of Ritz pairs; it also builds
 * index tables (neighbours, traversal orders, probing colourings).
 *
 * Paper: P. Lashomb, R. B. Morgan, T. Whyte, W. Wilcox, "Multipolynomial Monte
 * Carlo Trace Estimation", Lattice 2023 (arXiv:2402.00016).  Citations below
 * name its sections and equations.
 *
 * ---------------------------------------------------------------------------
 * Conventions shared by all calls
 * ---------------------------------------------------------------------------
 * Lattice:   dims = {Lx, Ly, Lz, Lt}; site s = x + Lx*(y + Ly*(z + Lz*t));
 *            V = Lx*Ly*Lz*Lt sites, n = 12 V complex unknowns.
 * Operator:  (M psi)(x) = psi(x) - kappa sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                              + (1 + gamma_mu) U_mu(x-mu)^H psi(x-mu) ]
 *            DeGrand-Rossi gammas, periodic space, a factor -1 on hops across
 *            the time boundary when t_antiperiodic != 0.  M^H = g5 M g5.
 * Theta:     MPMC_THETA_I (identity) or MPMC_THETA_G5 (gamma5 = diag(1,1,-1,-1)
 *            in spin), the inserted operator of Tr(Theta M^-1) (Sec. 1 eq. 1).
 * Canonical vectors: complex double, [rhs][site][spin 4][colour 3]; component
 *            c = (s*4 + spin)*3 + colour.
 * Internal vectors ("internal layout", what the kernels read and write):
 *            element (s, k = spin*3 + colour, r) of a batch of nrhs vectors at
 *            index (s*12 + k)*nrhs + r, i.e. site-major with the right-hand
 *            sides innermost, so neighbouring lanes of a wavefront read
 *            neighbouring right-hand sides of the same site.
 *              MPMC_FP64  -- complex double (16 B per element)
 *              MPMC_FP32  -- complex float  (8 B per element)
 *              MPMC_FP16S -- complex half (4 B per element) followed, at byte
 *                            offset align256(V*12*nrhs*4), by one float scale
 *                            per (site, rhs) at index s*nrhs + r; the value is
 *                            half * scale (storage format; arithmetic is FP32).
 *            mpmc_vector_bytes() returns the buffer size.
 * Noise:     Z(4) entries i^k, k from Philox4x32-10 (Salmon et al., SC'11):
 *            key = (seed mod 2^32, seed >> 32), counter = (c / 64, noise index,
 *            stream, 0), k = (word[(c % 64) / 16] >> 2 (c % 16)) & 3.
 *            Noise vectors are regenerated from (seed, stream, index), never
 *            stored by the caller (Z(4) noise vectors, Sec. 1).
 *
 * Memory and ownership: every pointer named x, y, b, Z, U, canon or internal
 * is a DEVICE pointer owned by the caller (e.g. a torch tensor's data_ptr()),
 * unless its name ends in _host.  Handles (mpmc_ctx, mpmc_poly, mpmc_defl,
 * mpmc_net) are owned by the library and released only by their _destroy
 * call.  The library allocates its own device workspace inside the context;
 * mpmc_apply_poly_noalloc instead carves its work vectors from a fixed
 * 64 MiB device array per GPU and allocates nothing.
 *
 * Ordering: work is enqueued on the context's HIP stream.  Calls that return
 * values through _host pointers or through d_eff/relres/iters outputs
 * synchronise that stream before returning; the others do not.
 *
 * Errors: every int-returning call returns MPMC_OK (0) or a negative status;
 * mpmc_last_error(ctx) returns a message for the last failure on ctx
 * (mpmc_last_error(NULL) for failures of mpmc_create).  No exceptions cross
 * the ABI.  A context is not thread-safe; calls on one context must not
 * overlap.
 */
#ifndef MPMC_H
#define MPMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpmc_ctx mpmc_ctx;
typedef struct mpmc_poly mpmc_poly;
typedef struct mpmc_defl mpmc_defl;
typedef struct mpmc_net mpmc_net;

enum {
    MPMC_OK = 0,
    MPMC_EINVAL = -1,   /* bad argument (null pointer, size, enum value)        */
    MPMC_ENOMEM = -2,   /* device allocation failed                             */
    MPMC_EHIP = -3,     /* HIP runtime error                                    */
    MPMC_ENOCONV = -4,  /* iteration limit reached; outputs hold the last iterate */
    MPMC_ENUMERIC = -5, /* NaN/Inf detected in a residual or a small eigenproblem */
    MPMC_ESTATE = -6    /* handle belongs to another context / wrong kind       */
};

enum { MPMC_FP64 = 0, MPMC_FP32 = 1, MPMC_FP16S = 2 };
enum { MPMC_THETA_I = 0, MPMC_THETA_G5 = 1 };

/* ------------------------------------------------------------------ context */

/* Create a context for one lattice.  links_host: canonical gauge field,
 * complex double [V][4][3][3] (U[s][mu][a][b] = row a, column b of U_mu(s)),
 * host memory, copied to the device.  stream: hipStream_t or NULL (null
 * stream).  The Wilson-Dirac matrix itself is defined only implicitly by the
 * paper (Sec. 1-2); its form is the one stated at the top of this header. */
int mpmc_create(const int dims[4], double kappa, int t_antiperiodic,
                const double *links_host, void *stream, mpmc_ctx **out);
void mpmc_destroy(mpmc_ctx *ctx);
const char *mpmc_last_error(const mpmc_ctx *ctx);
int mpmc_set_stream(mpmc_ctx *ctx, void *stream);

/* Bytes of an internal-layout buffer holding nrhs vectors in precision prec. */
int mpmc_vector_bytes(const mpmc_ctx *ctx, int nrhs, int prec, size_t *bytes);

/* Number of right-hand-side operator applications (Table 1's "MVP") issued on
 * this context since creation or the last reset. */
int mpmc_mvp_count(const mpmc_ctx *ctx, uint64_t *mvps_host);
int mpmc_mvp_reset(mpmc_ctx *ctx);

/* Free the device workspace the context keeps between calls (Krylov bases,
 * reduction partials, ...); later calls allocate again as needed.  Useful
 * between workloads of very different sizes on a full GPU.  Synchronises. */
int mpmc_release_workspace(mpmc_ctx *ctx);

/* Launch timing of the Wilson-Dirac kernels (the multi-RHS "Dslash", alone or
 * fused into a polynomial step).  While enabled, HIP events are recorded on the
 * context stream around every multi-RHS launch together with the launch's
 * algorithmic HBM bytes: spinor bytes per (site, rhs) for each operand read
 * once and each output written once, plus the links once per site.
 * Single-vector launches (nrhs = 1, the Arnoldi cycles) are counted with their
 * bytes but get no events (two event records would cost about as much as the
 * launch).  mpmc_timing_read synchronises and returns, for launches of
 * precision prec since the last enable, the count, the summed kernel time (ms,
 * multi-RHS launches only) and the summed algorithmic bytes; it leaves timing
 * enabled.  prec may be or-ed with MPMC_TIMING_FUSED (only the fused level
 * steps, k_wilson_dot), MPMC_TIMING_PLAIN (only the other multi-RHS Wilson
 * launches) or MPMC_TIMING_SINGLE (only single-vector launches: time 0);
 * without a flag every kind is summed. */
enum { MPMC_TIMING_PLAIN = 16, MPMC_TIMING_FUSED = 32, MPMC_TIMING_SINGLE = 64 };
int mpmc_timing_enable(mpmc_ctx *ctx, int on);
int mpmc_timing_read(mpmc_ctx *ctx, int prec, uint64_t *launches_host, double *ms_host, double *bytes_host);

/* Canonical complex double <-> internal layout of precision prec (device to
 * device; FP16S packing picks the per-(site, rhs) scale max|component|). */
int mpmc_pack(mpmc_ctx *ctx, const void *canon, void *internal, int nrhs, int prec);
int mpmc_unpack(mpmc_ctx *ctx, const void *internal, void *canon, int nrhs, int prec);

/* Z(4) noise vectors with indices first .. first+nrhs-1 of (seed, stream),
 * written in internal layout of precision prec (values are exact in every
 * precision).  Sec. 1: the Hutchinson noise. */
int mpmc_noise(mpmc_ctx *ctx, uint64_t seed, uint32_t stream, uint64_t first,
               int nrhs, int prec, void *internal);

/* ------------------------------------------------------------------ operator */

/* y = Theta * op(x), op = M (dagger = 0) or M^H (dagger = 1), for nrhs
 * internal-layout vectors of precision prec; x and y must not overlap.  The
 * matrix-vector product ("MVP") of Table 1. */
int mpmc_apply_M(mpmc_ctx *ctx, const void *x, void *y, int nrhs, int prec,
                 int dagger, int theta);

/* -------------------------------------------------------------- polynomials */

/* One GMRES(d) cycle (Sec. 3): Arnoldi with CGS2 for d steps from the
 * normalised Z(4) vector (seed, stream, index 0), then the harmonic Ritz values
 * eig(H_d + |h_{d+1,d}|^2 H_d^-H e_d e_d^T) in Leja order (largest modulus
 * first, then maximal sum of log distances), all in FP64 on the device (the
 * eigenvalues by mpmc_set_dense_method's solver).
 * The polynomial p has degree d-1 and satisfies pi(M) = 1 - M p(M) with
 * pi(M) = prod_i (1 - M/theta_i).
 * inner == NULL: the cycle runs on M.  inner != NULL: it runs on
 *   phi_in(M) = M p_in(M) and the result is the double polynomial
 *   p_in(M) p_out(phi_in(M)) of degree d_in*d - 1 (Sec. 5).
 * defl != NULL: the start vector and every Arnoldi vector are projected with
 *   Q = I - Z U^H, so the polynomial fits the undeflated spectrum (Sec. 7).
 * Outputs: *out (new handle), *d_eff (< d after a happy breakdown, which is not
 * an error), *relres = ||pi(op) b|| / ||b|| from the GMRES least squares.
 * Synchronises. */
int mpmc_gmres_poly(mpmc_ctx *ctx, const mpmc_poly *inner, const mpmc_defl *defl,
                    uint64_t seed, uint32_t stream, int d, mpmc_poly **out,
                    int *d_eff, double *relres);

/* Build a polynomial from given Leja-ordered roots (complex double, host),
 * optionally as the outer factor of a double polynomial with inner. */
int mpmc_poly_create(mpmc_ctx *ctx, const double *roots_host, int d,
                     const mpmc_poly *inner, mpmc_poly **out);
/* Roots (complex double, host, capacity *d on entry) and sizes.  degree is
 * the degree of p; matvecs the MVPs per vector of mpmc_apply_poly. */
int mpmc_poly_roots(const mpmc_poly *p, double *roots_host, int *d);
int mpmc_poly_info(const mpmc_poly *p, int *d, int *d_inner, int *degree, int *matvecs);
/* Scalar p(lambda) for k complex values (host in, host out): used for the
 * deflation coefficients p_l(lambda_i) - p_{l+1}(lambda_i) (Sec. 7). */
int mpmc_poly_eval(const mpmc_poly *p, const double *lam_host, double *out_host, int k);
void mpmc_poly_destroy(mpmc_poly *p);
/* Stabilise a high-degree polynomial by added roots (for p of degree ~200 and
 * beyond, where the product form loses accuracy): every root theta_k whose
 * product of other factors pof(k) = prod_{i != k} |1 - theta_k/theta_i| has
 * log10 pof(k) > log10_threshold (4 is the usual choice) gets
 * ceil((log10 pof(k) - log10_threshold) / digits) extra copies (digits: 14);
 * the extended list is Leja ordered (copies last) and replaces p's roots, so
 * p's degree grows by *added_host.  The residual polynomial becomes
 * pi(z) prod_k (1 - z/theta_k)^{copies_k} and 1 - z p(z) = pi(z) still holds
 * for the new roots.  Computed on the device.  Synchronises. */
int mpmc_poly_add_roots(mpmc_poly *p, double log10_threshold, double digits, int *added_host);

/* y = p(M) x for nrhs internal-layout vectors of precision prec (FP64 or FP32):
 * y = sum_k w_k / theta_k, w_1 = x, w_{k+1} = w_k - M w_k / theta_k (Sec. 3,
 * with the expansion read so that pi = 1 - M p holds), and for a double
 * polynomial p_in(M) [p_out(phi_in(M)) x] (Sec. 5).  x and y must not overlap. */
int mpmc_apply_poly(mpmc_ctx *ctx, const mpmc_poly *p, const void *x, void *y,
                    int nrhs, int prec);

/* mpmc_apply_poly for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result bit for bit, with its work vectors (2 for a
 * single polynomial, 6 for a double one, each mpmc_vector_bytes(nrhs, prec)
 * rounded up to 256 bytes) in one fixed 64 MiB device array of the library
 * that every GPU it runs on holds until the process ends (its address is
 * taken in mpmc_create).  No hipMalloc, hipFree or event creation happens in
 * the call.  Every call on one GPU shares that GPU's array, from every context
 * and thread: calls that overlap on one GPU (two streams, two threads, a
 * second call before the first has finished on the device) race and give
 * undefined results; calls ordered on one stream are safe.  The array keeps
 * the last call's contents; no part of it needs to start at zero.  Errors:
 * MPMC_EINVAL for bad arguments, aliasing x and y, precisions other than FP64
 * and FP32, and work vectors beyond 64 MiB (message names the limit);
 * MPMC_ESTATE while launch timing is on (it creates events). */
int mpmc_apply_poly_noalloc(mpmc_ctx *ctx, const mpmc_poly *p, const void *x, void *y,
                            int nrhs, int prec);

/* Exact Tr(Theta p(M)) by probing (Sec. 6: the last term of the
 * multipolynomial formula is computed exactly with probing).  Sites are
 * coloured by c(x) = sum_mu (x_mu mod period[mu]) prod_{nu<mu} period[nu]
 * (period[mu] must divide L_mu); probe vector (c, alpha) is 1 on spin-colour
 * component alpha of every site of colour c.  The sum of v^H Theta p(M) v over
 * the 12 * prod(period) probes is the exact trace when, for every mu with
 * period[mu] < L_mu, deg(p) < period[mu] <= L_mu / 2; *exact_host reports
 * whether that holds (period[mu] = L_mu for all mu is always exact).
 * prec: FP64 or FP32; probes are processed max_batch (rounded to a multiple
 * of 12, 0 = 192) at a time.  trace_host: complex double; mvps_host may be NULL.
 * Synchronises. */
int mpmc_poly_trace(mpmc_ctx *ctx, const mpmc_poly *p, int theta, const int period[4], int prec,
                    int max_batch, double *trace_host, int *exact_host, uint64_t *mvps_host);

/* Distance colouring for exact probing (host only, no device work).  Sites x
 * of the periodic lattice dims get colours from k <= 4 linear forms
 *   c_i(x) = (sum_mu W[4 i + mu] x_mu) mod moduli[i],
 *   colour(x) = sum_i c_i(x) prod_{l < i} moduli[l],
 * such that two distinct sites at taxicab distance <= distance on the torus
 * never share a colour (every modulus divides every extent, so each form is
 * defined on the torus; the colouring is translation invariant).  The forms
 * are searched by increasing colour count with a fixed pseudo-random sequence
 * (the result depends on dims and distance only); without a valid candidate
 * every site gets its own colour (forms x_mu mod L_mu), and so without a
 * search when distance reaches the torus diameter (sum of L_mu / 2) or when
 * the distance ball exceeds 4 V displacements on a lattice of more than 2^24
 * sites.  Outputs (host):
 * *k_host, moduli_host[4] (unused entries 1), W_host[16] (row-major k x 4,
 * unused rows 0), *ncolours_host = prod moduli.  EINVAL for a null pointer,
 * distance < 0 or an extent outside 1 .. 1024; ENOMEM if the host search
 * cannot allocate. */
int mpmc_probe_colouring(const int dims[4], int distance, int *k_host, int *moduli_host, int *W_host,
                         long *ncolours_host);

/* Exact Tr(Theta p(M)) by probing with the distance colouring (Sec. 6: the
 * last term of the multipolynomial formula is computed exactly by probing).
 * p(M) of degree D couples only sites at taxicab distance <= D, so with the
 * colouring of mpmc_probe_colouring(dims, D) the probe vectors v_{c,alpha}
 * (1 on spin-colour component alpha of every site of colour c) satisfy
 * sum_{c,alpha} v^H Theta p(M) v = Tr(Theta p(M)) exactly.  12 * ncolours
 * probes, processed max_batch (rounded down to a multiple of 12; 0 = 192) at
 * a time; each costs the MVPs of one mpmc_apply_poly.  prec: FP64 or FP32
 * (quadratic forms accumulated in FP64).  Outputs (host): trace_host (complex
 * double), *nprobe_host (may be NULL), *mvps_host (may be NULL).  The
 * colouring is cached in the context per degree.  Synchronises. */
int mpmc_poly_trace_probe(mpmc_ctx *ctx, const mpmc_poly *p, int theta, int prec, int max_batch,
                          double *trace_host, long *nprobe_host, uint64_t *mvps_host);

/* ---------------------------------------------------------------- deflation */

/* Eigenpairs for deflation (Sec. 7, acceptance rule of Sec. 8): m steps of
 * polynomial-preconditioned Arnoldi on phi_in(M) = M p_in(M) (on M itself if
 * p_in == NULL) from the Z(4) vector (seed, stream, 0); Ritz values of H_m by
 * mpmc_set_dense_method's FP64 solver on the device, Ritz vectors by inverse
 * iteration; the nev Ritz values
 * of smallest modulus give z = V_m s (unit norm) and lambda = z^H M z; left
 * vectors u_i = g5 z_j with lambda_j the conjugate partner of lambda_i (j = i
 * when |Im lambda_i| < real_tol), scaled to u_i^H z_i = 1; a pair is accepted
 * when ||M z - lambda z|| and ||M^H u - conj(lambda) u||/||u|| are both below
 * accept_tol.  *k_out = accepted count (may be 0).  Synchronises. */
int mpmc_deflate(mpmc_ctx *ctx, const mpmc_poly *p_in, uint64_t seed, uint32_t stream,
                 int m, int nev, double accept_tol, double real_tol,
                 mpmc_defl **out, int *k_out);
/* Import k eigentriples: lam_host complex double [k]; Z, U canonical complex
 * double [k][n] device arrays (copied). */
int mpmc_defl_create(mpmc_ctx *ctx, const double *lam_host, const void *Z, const void *U,
                     int k, mpmc_defl **out);
/* Export: lam_host [k] and, if non-NULL, Z/U canonical [k][n] device buffers. */
int mpmc_defl_export(const mpmc_defl *d, double *lam_host, void *Z, void *U, int *k);
void mpmc_defl_destroy(mpmc_defl *d);
/* Keep only the first k eigentriples (they are stored by increasing |lambda|),
 * e.g. the k lowest of a larger accepted set.  k larger than the set is a no-op. */
int mpmc_defl_keep(mpmc_defl *d, int k);

/* -------------------------------------------------------------------- solve */

/* x = M^-1 b for nrhs FP64 internal-layout vectors (Sec. 1: the main expense;
 * Sec. 8: deflated GMRES).  Restarted GMRES(restart) with FP64 defect
 * correction: the outer loop forms r = b - M x in FP64, the inner cycle runs
 * in inner_prec (MPMC_FP64; MPMC_FP32; or MPMC_FP16S = Krylov basis stored
 * as FP16 with one FP32 scale per (site, rhs), arithmetic in FP32, each inner
 * cycle stopped at 1e-3 of its starting residual), and x += e in FP64, until every
 * right-hand side has ||b - M x|| / ||b|| <= tol (true FP64 residual).  With
 * defl, x starts from Z Lambda^-1 U^H b and each restart adds Z Lambda^-1 U^H r.
 * net (may be NULL) is a right preconditioner inside the inner cycle
 * (flexible GMRES with the preconditioned vectors z_j = N v_j kept in FP32;
 * requires inner_prec = MPMC_FP32 or MPMC_FP16S, whose FP16 basis vectors are
 * widened to FP32 before N); it changes cost, never
 * the converged x.  An inner cycle ends when every right-hand side's
 * residual estimate meets its target, tested after every inner step when
 * V * nrhs >= 2^22 and every 10 steps otherwise (a test waits for the
 * stream).  Gram-Schmidt: see mpmc_set_solve_gs_passes.  Outputs (host):
 * iters_host = total inner iterations, relres_host[nrhs] = final true
 * relative residuals.  Returns MPMC_ENOCONV after max_outer cycles.
 * Synchronises. */
int mpmc_solve(mpmc_ctx *ctx, const void *b, void *x, int nrhs, const mpmc_defl *defl,
               const mpmc_net *net, int restart, double tol, int inner_prec,
               int max_outer, int *iters_host, double *relres_host);

/* Several lattices in ONE launch (not in the paper: batching of independent
 * problems): y[i] = M_i x[i] for the contexts ctxs[0..count), 1 <= count <= 8,
 * all on the device of ctxs[0] and run on ctxs[0]'s stream.  Every context
 * keeps its own lattice, kappa and links; nrhs (a multiple of 64) right-hand
 * sides per lattice, prec FP64 or FP32, internal layout, V % 4 == 0 for every
 * lattice.  The grid concatenates the lattices' tile ranges (4D-blocked,
 * 64-wide chunks), so each lattice's result is bit-identical to mpmc_apply_M
 * with Wilson variant 4 or 5.  x[i] and y[i] must not alias.  Counts nrhs MVPs
 * on every context; the launch's algorithmic bytes enter ctxs[0]'s timing.
 * Asynchronous. */
int mpmc_apply_M_batch(mpmc_ctx *const *ctxs, const void *const *x, void *const *y, int count, int nrhs,
                       int prec, int dagger, int theta);

/* mpmc_solve for several lattices at once (not in the paper: batching of
 * independent problems, e.g. uneven lattices that share one network): the
 * contexts ctxs[0..count), 1 <= count <= 8, distinct, on one device and one
 * stream, each with its own b[i], x[i] (nrhs FP64 internal-layout vectors,
 * nrhs a multiple of 64, the same for all), deflation set defl[i] and network
 * net[i] (defl, net or their entries may be NULL).  The solves advance in
 * lockstep: every inner iteration applies M on all lattices still iterating
 * with ONE mpmc_apply_M_batch launch; Gram-Schmidt, Givens steps and the
 * outer loop stay per lattice.  inner_prec FP64 or FP32.  Each lattice's
 * iterates equal those of its own mpmc_solve with Wilson variant 4/5 (the
 * batched launch's traversal; every variant gives the same bits).  Outputs
 * (host, may be NULL): iters_host[count], relres_host[count * nrhs].
 * Returns the first failing lattice's code (MPMC_ENOCONV when one did not
 * converge; every lattice still runs to its end).  Synchronises. */
int mpmc_solve_batch(mpmc_ctx *const *ctxs, int count, const void *const *b, void *const *x, int nrhs,
                     const mpmc_defl *const *defl, const mpmc_net *const *net, int restart, double tol,
                     int inner_prec, int max_outer, int *iters_host, double *relres_host);

/* ---------------------------------------------------------------- autotuner */
/* The multi-RHS Wilson kernel (nrhs a multiple of 64) has variants
 * 0 .. mpmc_wilson_variant_count() - 1 (currently 13) that differ only in how
 * the work is laid out on the GPU, never in the arithmetic (results are
 * bit-identical):
 *   0-9, bit 0 -- occupancy target: 1 = more wavefronts per SIMD (FP32/FP16S:
 *               3, FP64: 2), 0 = more registers per wavefront (FP32/FP16S: 2,
 *               FP64: 1);
 *   0-9, bits 1-3 -- traversal: 0 = site-major (a workgroup covers 256/nrhs
 *               sites x nrhs right-hand sides), 1 = 64-wide right-hand-side
 *               chunks (a workgroup covers 4 sites x 64 right-hand sides; all
 *               sites of a chunk before the next chunk), 2 = chunks as in 1 with
 *               the sites of a chunk in the order of the site table
 *               (mpmc_set_site_order; default 4D blocks of extent 4), 3 and 4 =
 *               as in 2 with 16- and 32-wide chunks (a wavefront covers 4 or 2
 *               sites, links loaded per lane; need V % 16 == 0, else 2);
 *   10       -- column streaming (FP32, even Lx, Ly, Lz, Lt >= 4; else 5): a
 *               workgroup of 8 wavefronts owns a 2 x 2 x 2 tile of (x, y, z)
 *               columns and 64 right-hand sides and walks the columns along
 *               t; the t-1 and the in-tile x, y, z neighbours come from LDS,
 *               the t+1 site from registers, so each site's spinor is read
 *               from memory 4 times instead of 9;
 *   11       -- column streaming with 2 x 2 x 1 tiles (FP32, even Lx, Ly,
 *               Lt >= 4; else 5): 4 wavefronts per workgroup and half the
 *               LDS, so two workgroups share a compute unit; both z
 *               neighbours come from memory (5 reads per site);
 *   12       -- column streaming with 2 x 2 x 4 tiles and 32-wide
 *               right-hand-side chunks (FP32, even Lx, Ly, Lz % 4 == 0,
 *               Lt >= 4, buffer ranges below 2 GiB; else 5): a wavefront holds
 *               two sites of a column pair (32 lanes each), so an XCD's
 *               concurrent workgroups cover twice the sites and fewer
 *               neighbours fall outside them (3.5 reads per site).
 * Defaults: variant 10 where it applies (FP32), else 5 for FP32/FP16S and 4
 * for FP64.
 * mpmc_autotune times every variant on (nrhs, prec) with scratch vectors of
 * the context (2 warm-up + 5 timed launches each, HIP events) and keeps the
 * fastest for all later Wilson launches on ctx with that (nrhs, prec),
 * including those inside polynomials and solves.
 * variant_host (may be NULL) receives the choice (-1 when nrhs is not a
 * multiple of 64: nothing to tune); us_host (may be NULL) receives
 * double[mpmc_wilson_variant_count()] microseconds per launch per variant
 * (0 for a variant that does not apply to the shape and is not timed).  Does not count MVPs and
 * does not enter mpmc_timing_read.  Synchronises. */
int mpmc_autotune(mpmc_ctx *ctx, int nrhs, int prec, int *variant_host, double *us_host);
/* Number of Wilson kernel variants (the length of mpmc_autotune's us_host). */
int mpmc_wilson_variant_count(void);
/* Pin a variant for (nrhs, prec); -1 restores the default.  A pinned variant
 * also fixes the traversal of the fused polynomial step of the level
 * estimators (variants 0-3: site-major, 4-9: blocked chunks, 10, 11 and 12:
 * column streaming with 2x2x2, 2x2x1 and 2x2x4 tiles), overriding
 * mpmc_autotune_level.  For nrhs = 1 (single vectors) variant 0 selects
 * eight lanes per site (one hop each), 1 the generic kernel with one site per
 * lane, 2 the single-vector kernel with one site per lane (coordinate-derived
 * neighbours; the same results as 1 bit for bit); the default is 0 up to 12^4
 * sites and 2 above. */
int mpmc_tune_set(mpmc_ctx *ctx, int nrhs, int prec, int variant);
/* Autotune the fused polynomial step of mpmc_level_estimate (the dominant
 * kernel of the polynomial levels, Sec. 6): every traversal valid for the
 * shape -- order 0 site-major, 2 blocked 64-wide chunks, 3 / 4 blocked 16- /
 * 32-wide chunks (V % 16 == 0), 5 / 6 / 7 column streaming (FP32, as
 * variants 10 / 11 / 12) --
 * is timed on (nrhs, prec) (2 warm-up + 5 timed steps, HIP events, best of
 * three interleaved rounds) and the fastest is kept for later level
 * estimates on ctx.  Without this call the step takes the column streaming
 * kernel with 2x2x2 tiles where it applies, else blocked 64-wide chunks
 * (V % 4 == 0), else site-major.  prec FP64 or FP32, nrhs a multiple of 64
 * (and of 256 above 256).  order_host (may be NULL): the choice; us_host
 * (may be NULL): double[8] microseconds per step by order (0
 * for orders not tried).  Samples are the same up to the grouping of the FP64
 * partial sums.  Does not count MVPs.  Synchronises. */
int mpmc_autotune_level(mpmc_ctx *ctx, int nrhs, int prec, int *order_host, double *us_host);

/* Captured polynomial recurrences.  on = 1: the launch sequence of each
 * fused polynomial recurrence of the level estimators (every step of
 * eta^H Theta p(M) eta, single and double polynomials, Sec. 3 and 5) is
 * captured once into a hipGraph on a stream the context creates (default
 * priority) and replayed from then on; the replay is ordered after the
 * earlier and before the later work of the context stream.  The key of a
 * captured graph is every input of its launches (operand and work-buffer
 * addresses, shape, precision, Theta, traversal, roots), so results are
 * bit-identical to the launches run one by one.  Launch timing
 * (mpmc_timing_enable) switches replay off while it is on.  Graphs are
 * dropped by mpmc_release_workspace, when a work buffer grows and by
 * mpmc_destroy.  on = 0 (default): launches one by one.  EINVAL unless on is
 * 0 or 1; EHIP if the stream or events cannot be created. */
int mpmc_set_graph_recurrences(mpmc_ctx *ctx, int on);
/* Replays of captured recurrences since creation and graphs held (host, may be NULL). */
int mpmc_graph_replays(const mpmc_ctx *ctx, uint64_t *replays_host, int *graphs_host);

/* Traversal order of the blocked multi-RHS Wilson kernels (variants 4-9 and
 * the fused level step): order_host[i] is the i-th site visited (int[V], a
 * permutation of 0 .. V-1, host memory, copied); workgroups take consecutive
 * entries and each XCD one contiguous eighth of them.  NULL restores the
 * default (4D blocks of extent 4, lexicographic).  Operator results do not
 * depend on the order; the fused level step sums its per-workgroup partials
 * in a different grouping (FP64 rounding only).  EINVAL if not a
 * permutation.  Synchronises. */
int mpmc_set_site_order(mpmc_ctx *ctx, const int *order_host);

/* ------------------------------------------------- learned preconditioner */
/* Not part of the paper: a small learned right preconditioner N for the main
 * solves (used by mpmc_solve / mpmc_level_estimate through their net
 * argument, inside flexible GMRES with FP32 inner cycles).  N is a
 * gauge-covariant LINEAR network of three parallel-transport layers with
 * 1 -> 2 -> 2 -> 1 spinor fields:
 *   out(x)[f', s', c] = sum_p sum_{f,s} W_p[(f',s'),(f,s)] (T_p in)(x)[f, s, c],
 * p = 0: identity; p = 1..4: +mu, U_mu(x) in(x+mu); p = 5..8: -mu,
 * U_mu(x-mu)^H in(x-mu), with the operator's time-boundary sign.  W_p acts on
 * (field, spin), not on colour, so N commutes with gauge transformations.
 * Arithmetic: BF16 weights and transported inputs on MFMA with FP32
 * accumulation; activations stored in FP32.
 * Weights (host, double[mpmc_net_n_params()] = 2304): for layer 0, 1, 2; for
 * p < 9; for o < 4*f_out; for i < 4*f_in (o, i = field*4 + spin): Re then Im
 * of W_p[o][i].  The device keeps FP32 master weights.
 * Training loss over P pairs (r_j, e_j):
 *   L = (1/P) sum_j ||N r_j - e_j||^2 / ||e_j||^2. */
int mpmc_net_n_params(void);
/* New network with the given weights (copied).  Owned by the caller; it
 * references ctx, which must outlive it. */
int mpmc_net_create(mpmc_ctx *ctx, const double *theta_host, mpmc_net **out);
void mpmc_net_destroy(mpmc_net *net);
/* Replace the weights (and reset the optimiser state).  Synchronises. */
int mpmc_net_set_weights(mpmc_net *net, const double *theta_host);
/* Current weights (FP32 master values widened to double).  Synchronises. */
int mpmc_net_get_weights(const mpmc_net *net, double *theta_host);
/* y = N x for nrhs FP32 internal-layout vectors (x and y must not alias). */
int mpmc_net_apply(mpmc_net *net, const void *x, void *y, int nrhs);
/* Loss L and its gradient dL/dtheta (host double[2304], same order as the
 * weights; NULL skips) for npairs pairs given as FP32 internal-layout
 * batches R (inputs r_j) and E (targets e_j).  Synchronises. */
int mpmc_net_loss_grad(mpmc_net *net, const void *R, const void *E, int npairs,
                       double *loss_host, double *grad_host);
/* steps Adam updates (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) of
 * the weights on the pairs (R, E); loss_host (may be NULL) receives the loss
 * before each update, double[steps].  The optimiser state persists across
 * calls on the same net.  Synchronises. */
int mpmc_net_train(mpmc_net *net, const void *R, const void *E, int npairs, int steps,
                   double lr, double *loss_host);

/* Polynomial-preconditioned deflated solve (Sec. 8, the paper's solver):
 * as mpmc_solve, with each inner cycle right-preconditioned GMRES on M p(M)
 * and the correction p(M) V y, for a single or double polynomial pp of this
 * context (typically a low-degree GMRES polynomial).  The outer loop still
 * tests the true FP64 residual.  Synchronises. */
int mpmc_solve_pp(mpmc_ctx *ctx, const void *b, void *x, int nrhs, const mpmc_defl *defl,
                  const mpmc_poly *pp, int restart, double tol, int inner_prec, int max_outer,
                  int *iters_host, double *relres_host);
/* Eigenvalue solver of the small dense FP64 problems (the harmonic Ritz
 * values of mpmc_gmres_poly, Sec. 3, and the Ritz values of mpmc_deflate,
 * Sec. 7).  method 0 (default): Aberth-Ehrlich simultaneous iteration on the
 * Hessenberg matrix (Newton ratios by Hyman's determinant recurrence), one
 * 16-lane group per eigenvalue across the GPU, for matrices up to 256 rows;
 * if it has not converged after 40 sweeps (or for larger matrices) the
 * shifted Hessenberg QR runs instead.  method 1: the shifted QR only.  The
 * eigenvalues agree to rounding; they come out in a different order before
 * the Leja ordering.  Returns MPMC_EINVAL for another method. */
int mpmc_set_dense_method(mpmc_ctx *ctx, int method);

/* Storage precision of the single-vector Arnoldi cycles behind
 * mpmc_gmres_poly (Sec. 3, Sec. 5) and mpmc_deflate (Sec. 7): MPMC_FP64 (the
 * default) or MPMC_FP32 (vectors and operator applications in FP32, every
 * inner product, the Hessenberg matrix, the harmonic Ritz / Ritz values, Leja
 * ordering, the Ritz vectors, Rayleigh quotients and acceptance residuals in
 * FP64).  FP32 halves the traffic of the setup; the polynomials then differ
 * from the FP64 ones at the level of FP32 rounding, which leaves the
 * multipolynomial estimate unbiased (any polynomials telescope).  EINVAL for
 * another precision. */
int mpmc_set_setup_precision(mpmc_ctx *ctx, int prec);
/* Gram-Schmidt of those Arnoldi cycles.  Both are classical Gram-Schmidt
 * applied twice (the Hessenberg matrices agree to rounding).  on = 0: the
 * second projection of each vector is delayed to the next step (the operator
 * is applied to the once-projected candidate u, one pass over the basis gives
 * V^H u, V^H (A u), u^H u and u^H A u, one more pass writes the finished
 * vector and the next candidate): two basis passes and four launches per step
 * besides the operator.  on = 1: the two projections in sequence (four basis
 * passes, eight shorter launches).  on = -1 (the default): 1 below 16^4
 * sites, where the steps are launch-bound, else 0.  EINVAL otherwise. */
int mpmc_set_arnoldi_cgs2(mpmc_ctx *ctx, int on);
/* Gram-Schmidt of the inner GMRES cycles of mpmc_solve, mpmc_solve_pp,
 * mpmc_solve_batch and the solves inside mpmc_level_estimate (Sec. 3's GMRES
 * used as the solver of the M^-1 level): passes = 2 projects each new Krylov
 * vector twice (classical Gram-Schmidt twice, orthogonal to working
 * precision); passes = 1 projects it once, which halves the basis traffic of
 * a step; passes = 0 (the default) takes 1 for FP32 and FP16S inner cycles,
 * whose targets (2e-6 and 1e-3 of the cycle's start) lie far above the loss
 * of orthogonality of one projection, and 2 for FP64 inner cycles, which run
 * to the final tolerance.  The outer FP64 defect correction checks the true
 * residual either way, so the choice changes iteration counts and time, never
 * the tolerance met.  EINVAL otherwise. */
int mpmc_set_solve_gs_passes(mpmc_ctx *ctx, int passes);

/* Polynomial preconditioner used by the main solves inside mpmc_level_estimate
 * when no network is given (NULL: none, the default).  The context keeps the
 * pointer: the caller keeps pp alive while it is set. */
int mpmc_set_level_solve_poly(mpmc_ctx *ctx, const mpmc_poly *pp);

/* mpmc_solve (no network) that also records training pairs for the learned
 * preconditioner from the solve itself: at the start of each outer cycle k <
 * max_snap, batch k of R_snap receives r_k = b - M x_k and batch k of E_snap
 * the error e_k = x - x_k of that iterate against the converged x (FP32
 * internal layout, nrhs vectors per batch, batches spaced
 * mpmc_vector_bytes(ctx, nrhs, MPMC_FP32) apart; caller-owned device
 * buffers of max_snap batches).  *nsnap_host = batches written.  Synchronises. */
int mpmc_solve_pairs(mpmc_ctx *ctx, const void *b, void *x, int nrhs, const mpmc_defl *defl,
                     int restart, double tol, int inner_prec, int max_outer, void *R_snap,
                     void *E_snap, int max_snap, int *nsnap_host, int *iters_host,
                     double *relres_host);

/* ---------------------------------------------------------------- estimators */

/* Samples of one Monte Carlo level (Sec. 2 eq. 2, Sec. 6, Sec. 7), for noise
 * vectors eta_j = Z(4)(seed, stream, first + j), j < nnoise:
 *   X_j = eta_j^H Theta A eta_j - [deflation term],
 *   A = upper - lower, upper = M^-1 when the upper handle is NULL (solved with
 *   mpmc_solve to solve_tol with GMRES(solve_restart), solve_inner_prec, defl
 *   and net), lower = 0 when the lower handle is NULL.
 * When both are polynomials and defl is given, the deflation term is
 *   sum_i c_i (eta^H Theta z_i)(u_i^H eta), c_i = upper(lambda_i) - lower(lambda_i),
 * and *corr_host = sum_i c_i u_i^H Theta z_i (the exact trace of the removed
 * part).  The solve level (upper NULL, lower a polynomial) with defl uses the
 * set inside its solves and, when mpmc_set_solve_level_deflation(ctx, 1) is
 * in effect, is deflated the same way with c_i = 1/lambda_i - lower(lambda_i).
 * Otherwise *corr_host = 0.
 * prec: precision of the polynomial applications (MPMC_FP64 or MPMC_FP32);
 * dot products and samples are accumulated in FP64 (in the fused steps the
 * twelve terms of one site in prec first).  Noise vectors are
 * processed in batches of at most max_batch right-hand sides (0 = all).
 * samples_host: complex double [nnoise]; mvps_host (may be NULL): MVPs used.
 * Synchronises. */
int mpmc_level_estimate(mpmc_ctx *ctx, const mpmc_poly *upper, const mpmc_poly *lower,
                        const mpmc_defl *defl, int theta, uint64_t seed, uint32_t stream,
                        uint64_t first, int nnoise, int prec, int max_batch,
                        double solve_tol, int solve_restart, int solve_inner_prec,
                        const mpmc_net *net, double *samples_host, double *corr_host,
                        uint64_t *mvps_host);

/* Deflation of the solve level M^-1 - p_1 in mpmc_level_estimate (Sec. 7's
 * level deflation with M^-1 as the upper operator): on = 1 subtracts
 * sum_i (1/lambda_i - p_1(lambda_i)) (eta^H Theta z_i)(u_i^H eta) from every
 * sample and returns the exact trace of the removed part as the correction;
 * needed when p_1 is the deflated double polynomial (mpmc_gmres_poly with a
 * deflation set), which does not approximate 1/lambda on the deflated
 * eigenvalues.  on = 0 (the default): no subtraction.  The estimate is
 * unbiased either way; only its variance changes.  EINVAL unless on is 0 or 1. */
int mpmc_set_solve_level_deflation(mpmc_ctx *ctx, int on);

/* The polynomial levels of the multipolynomial formula (Sec. 6) together:
 * term t has the samples, correction and precision semantics of
 * mpmc_level_estimate(ctx, upper[t], lower[t], defl, theta, seed, streams[t],
 * first, nnoise, prec, 0, ...) -- bit for bit when that call's fused step
 * takes the blocked 64-wide traversal (variants 4/5 pinned with
 * mpmc_tune_set), else up to the grouping of the FP64 partial sums -- with
 * upper[t] != NULL (the solve term stays with mpmc_level_estimate) and
 * lower[t] possibly NULL.
 * Every single-polynomial recurrence of the batch (the upper and the lower
 * polynomial of each term, on that term's noise) occupies its own run of
 * nnoise right-hand sides of one operand, runs ordered by decreasing degree,
 * and step s of all recurrences still running is ONE fused launch; the
 * per-chunk coefficients come from a table uploaded once.  Terms with a
 * double polynomial, and all terms when nnoise % 64 != 0 or V % 4 != 0, run
 * one by one through mpmc_level_estimate.  nterms <= 64.
 * samples_host: complex double [nterms][nnoise]; corr_host (may be NULL):
 * complex double [nterms]; mvps_host (may be NULL): MVPs used.  Device
 * memory: 3 operands of nterms*2*nnoise right-hand sides in precision prec
 * plus 4 bytes per (site, rhs) of noise codes.  Synchronises. */
int mpmc_level_estimate_multi(mpmc_ctx *ctx, int nterms, const mpmc_poly *const *upper,
                              const mpmc_poly *const *lower, const mpmc_defl *defl, int theta,
                              uint64_t seed, const uint32_t *streams, uint64_t first, int nnoise,
                              int prec, double *samples_host, double *corr_host,
                              uint64_t *mvps_host);

#ifdef __cplusplus
}
#endif
#endif /* MPMC_H */
