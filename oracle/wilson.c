/*
 * Oracle (test infrastructure only; never linked into the product path):
 * plain FP64 matrix-free Wilson-Dirac operator on the CPU.
 *
 * The paper (Sec. 1-2) names the Wilson-Dirac matrix M and the hopping
 * parameter kappa (Sec. 4) without writing M out; this file follows the
 * reading recorded in the design notes:
 *
 *   (M psi)(x) = psi(x) - kappa * sum_mu [ (1 - g*gamma_mu) U_mu(x)       psi(x+mu)
 *                                        + (1 + g*gamma_mu) U_mu(x-mu)^H psi(x-mu) ]
 *
 * with g = +1 for M and g = -1 for M^dagger, gamma_mu in the DeGrand-Rossi
 * basis, periodic boundaries in space and a factor -1 on every hop that
 * crosses the time boundary when t_antiperiodic is set.
 *
 * Nothing here is blocked or fused: the spin projector is applied as a full
 * 4x4 matrix to the colour-rotated neighbour spinor, exactly as the formula
 * reads.
 *
 * Layouts (canonical, shared with the inputs only):
 *   site  s = x + Lx*(y + Ly*(z + Lz*t))
 *   links U[s][mu][a][b] complex double (row a, column b), mu = 0..3 = x,y,z,t
 *   spinor psi[r][s][spin][colour] complex double, r = right-hand side
 */
#include <complex.h>
#include <omp.h>
#include <stddef.h>

/* OpenMP team size of the operator (the baseline timing reports it). */
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int oracle_max_threads(void) { return omp_get_max_threads(); }

typedef double complex cplx;

/* DeGrand-Rossi gamma matrices, gamma[mu][row][col], mu = 0..3 = x,y,z,t. */
static const cplx GAMMA[4][4][4] = {
    {{0, 0, 0, I}, {0, 0, I, 0}, {0, -I, 0, 0}, {-I, 0, 0, 0}},
    {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}},
    {{0, 0, I, 0}, {0, 0, 0, -I}, {-I, 0, 0, 0}, {0, I, 0, 0}},
    {{0, 0, 1, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}},
};

static void coords_of(long s, const int L[4], int c[4]) {
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int)(s % L[mu]);
        s /= L[mu];
    }
}

static long site_of(const int c[4], const int L[4]) {
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

/* y = M x (dagger = 0) or y = M^H x (dagger = 1) for nrhs vectors. */
void oracle_wilson_apply(const int *dims, double kappa, int t_antiperiodic,
                         const double *links, const double *xin, double *yout,
                         long nrhs, int dagger) {
    const int L[4] = {dims[0], dims[1], dims[2], dims[3]};
    const long V = (long)L[0] * L[1] * L[2] * L[3];
    const cplx *U = (const cplx *)links;
    const cplx *X = (const cplx *)xin;
    cplx *Y = (cplx *)yout;
    const double g = dagger ? -1.0 : 1.0;

    /* small problems run serially: an idle OpenMP team spinning between calls
       would otherwise compete with the BLAS threads of the Python driver */
#pragma omp parallel for collapse(2) schedule(static) if (nrhs * V >= 8192)
    for (long r = 0; r < nrhs; ++r) {
        for (long s = 0; s < V; ++s) {
            const cplx *x = X + r * V * 12;
            cplx *y = Y + r * V * 12;
            int c[4];
            coords_of(s, L, c);
            cplx acc[4][3];
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 3; ++b) acc[a][b] = 0;

            for (int mu = 0; mu < 4; ++mu) {
                /* forward hop: (1 - g gamma_mu) U_mu(x) psi(x+mu) */
                int cf[4] = {c[0], c[1], c[2], c[3]};
                cf[mu] = (c[mu] + 1) % L[mu];
                double sgn_f = (t_antiperiodic && mu == 3 && c[3] == L[3] - 1) ? -1.0 : 1.0;
                long sf = site_of(cf, L);
                const cplx *Uf = U + (s * 4 + mu) * 9;
                cplx tmp[4][3];
                for (int sp = 0; sp < 4; ++sp)
                    for (int a = 0; a < 3; ++a) {
                        cplx t = 0;
                        for (int b = 0; b < 3; ++b) t += Uf[a * 3 + b] * x[(sf * 4 + sp) * 3 + b];
                        tmp[sp][a] = t;
                    }
                for (int al = 0; al < 4; ++al)
                    for (int be = 0; be < 4; ++be) {
                        cplx P = (al == be ? 1.0 : 0.0) - g * GAMMA[mu][al][be];
                        if (P == 0) continue;
                        for (int a = 0; a < 3; ++a) acc[al][a] += sgn_f * P * tmp[be][a];
                    }

                /* backward hop: (1 + g gamma_mu) U_mu(x-mu)^H psi(x-mu) */
                int cb[4] = {c[0], c[1], c[2], c[3]};
                cb[mu] = (c[mu] + L[mu] - 1) % L[mu];
                double sgn_b = (t_antiperiodic && mu == 3 && c[3] == 0) ? -1.0 : 1.0;
                long sb = site_of(cb, L);
                const cplx *Ub = U + (sb * 4 + mu) * 9;
                for (int sp = 0; sp < 4; ++sp)
                    for (int a = 0; a < 3; ++a) {
                        cplx t = 0;
                        for (int b = 0; b < 3; ++b) t += conj(Ub[b * 3 + a]) * x[(sb * 4 + sp) * 3 + b];
                        tmp[sp][a] = t;
                    }
                for (int al = 0; al < 4; ++al)
                    for (int be = 0; be < 4; ++be) {
                        cplx P = (al == be ? 1.0 : 0.0) + g * GAMMA[mu][al][be];
                        if (P == 0) continue;
                        for (int a = 0; a < 3; ++a) acc[al][a] += sgn_b * P * tmp[be][a];
                    }
            }
            for (int al = 0; al < 4; ++al)
                for (int a = 0; a < 3; ++a)
                    y[(s * 4 + al) * 3 + a] = x[(s * 4 + al) * 3 + a] - kappa * acc[al][a];
        }
    }
}
