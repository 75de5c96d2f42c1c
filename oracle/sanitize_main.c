/*
 * Test infrastructure only: a stand-alone driver that runs the oracle's C
 * Wilson operator under AddressSanitizer and UndefinedBehaviorSanitizer (host
 * build with gcc).  It applies M and M^H to a few vectors on lattices of
 * several shapes (extents 1 and 2 included, where hops wrap onto the same
 * site) and checks gamma5-hermiticity, <y, M x> = <M^H y, x>, on the result,
 * so that the sanitizers see every access of both code paths.  Exit status 0
 * when the identity holds; the sanitizers abort on any invalid access.
 */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_wilson_apply(const int *dims, double kappa, int t_antiperiodic, const double *links, const double *xin,
                         double *yout, long nrhs, int dagger);

static double rnd(unsigned long *s) {
    *s = *s * 6364136223846793005UL + 1442695040888963407UL;
    return (double)(*s >> 11) / 9007199254740992.0 - 0.5;
}

static int run(const int L[4], long nrhs) {
    const long V = (long)L[0] * L[1] * L[2] * L[3], n = 12 * V;
    double complex *U = malloc(sizeof(double complex) * V * 36);
    double complex *x = malloc(sizeof(double complex) * n * nrhs), *y = malloc(sizeof(double complex) * n * nrhs);
    double complex *Mx = malloc(sizeof(double complex) * n * nrhs), *Mhy = malloc(sizeof(double complex) * n * nrhs);
    if (!U || !x || !y || !Mx || !Mhy) return 2;
    unsigned long s = 12345;
    for (long i = 0; i < V * 36; ++i) U[i] = rnd(&s) + I * rnd(&s);   /* any matrices: the identity holds */
    for (long i = 0; i < n * nrhs; ++i) {
        x[i] = rnd(&s) + I * rnd(&s);
        y[i] = rnd(&s) + I * rnd(&s);
    }
    oracle_wilson_apply(L, 0.13, 1, (const double *)U, (const double *)x, (double *)Mx, nrhs, 0);
    oracle_wilson_apply(L, 0.13, 1, (const double *)U, (const double *)y, (double *)Mhy, nrhs, 1);
    int bad = 0;
    for (long r = 0; r < nrhs; ++r) {
        double complex a = 0, b = 0;
        double na = 0;
        for (long i = 0; i < n; ++i) {
            a += conj(y[r * n + i]) * Mx[r * n + i];
            b += conj(Mhy[r * n + i]) * x[r * n + i];
            na += cabs(y[r * n + i]) * cabs(Mx[r * n + i]);
        }
        if (cabs(a - b) > 1e-12 * na) bad = 1;
    }
    free(U); free(x); free(y); free(Mx); free(Mhy);
    return bad;
}

int main(void) {
    const int shapes[][4] = {{1, 1, 1, 1}, {2, 2, 2, 2}, {3, 1, 2, 4}, {4, 4, 2, 2}, {2, 3, 4, 5}};
    for (int q = 0; q < 5; ++q) {
        const int rc = run(shapes[q], q % 2 ? 3 : 1);
        if (rc) {
            printf("adjoint identity failed on shape %d\n", q);
            return rc;
        }
    }
    printf("sanitized oracle operator ok\n");
    return 0;
}
