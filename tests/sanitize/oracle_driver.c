/*
 * Sanitizer driver of the oracle's C hop (test infrastructure): runs the hop
 * over small lattices, flavour counts, rhs counts, daggers and output
 * parities under AddressSanitizer / UndefinedBehaviorSanitizer, and checks
 * that it is linear (D(a + 2b) = D a + 2 D b) and that a parity-restricted
 * output is the full output masked to that parity.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_hop(double *out, const double *in, const double *U, const int *dims, int nf, int nrhs, int dagger,
            double tsign, int out_parity);

static double frand(unsigned *s)
{
    *s = *s * 1103515245u + 12345u;
    return ((*s >> 8) & 0xffff) / 32768.0 - 1.0;
}

int main(void)
{
    static const int lattices[][4] = {{2, 2, 2, 2}, {4, 2, 2, 4}, {2, 4, 2, 4}, {4, 4, 4, 4}, {6, 4, 2, 2}};
    unsigned seed = 7;
    int failures = 0;
    for (size_t li = 0; li < sizeof(lattices) / sizeof(lattices[0]); li++) {
        const int *d = lattices[li];
        const long V = (long)d[0] * d[1] * d[2] * d[3];
        for (int nf = 1; nf <= 2; nf++)
            for (int nrhs = 1; nrhs <= 2; nrhs++) {
                const long ns = 2 * (long)nrhs * V * nf * 12;   /* doubles of a spinor field */
                const long nu = 2 * 4 * V * 9;                   /* doubles of the links */
                double *U = malloc(nu * sizeof(double)), *a = malloc(ns * sizeof(double));
                double *b = malloc(ns * sizeof(double)), *c = malloc(ns * sizeof(double));
                double *ya = malloc(ns * sizeof(double)), *yb = malloc(ns * sizeof(double));
                double *yc = malloc(ns * sizeof(double)), *yp = malloc(ns * sizeof(double));
                for (long i = 0; i < nu; i++) U[i] = frand(&seed);
                for (long i = 0; i < ns; i++) {
                    a[i] = frand(&seed);
                    b[i] = frand(&seed);
                    c[i] = a[i] + 2.0 * b[i];
                }
                for (int dag = 0; dag <= 1; dag++) {
                    if (orc_hop(ya, a, U, d, nf, nrhs, dag, -1.0, -1) || orc_hop(yb, b, U, d, nf, nrhs, dag, -1.0, -1) ||
                        orc_hop(yc, c, U, d, nf, nrhs, dag, -1.0, -1)) {
                        printf("orc_hop failed\n");
                        return 2;
                    }
                    double err = 0.0, nrm = 0.0;
                    for (long i = 0; i < ns; i++) {
                        err = fmax(err, fabs(yc[i] - ya[i] - 2.0 * yb[i]));
                        nrm = fmax(nrm, fabs(yc[i]));
                    }
                    if (err > 1e-12 * (nrm + 1.0)) {
                        printf("linearity %d %d %d %d: %g\n", (int)li, nf, nrhs, dag, err);
                        failures++;
                    }
                    for (int par = 0; par <= 1; par++) {
                        orc_hop(yp, a, U, d, nf, nrhs, dag, -1.0, par);
                        for (long s = 0; s < nrhs * V; s++) {
                            const long lex = s % V;
                            const int x = lex % d[0], y = (lex / d[0]) % d[1], z = (lex / d[0] / d[1]) % d[2],
                                      t = lex / d[0] / d[1] / d[2];
                            const int p = (x + y + z + t) & 1;
                            for (long k = 0; k < 2 * nf * 12; k++) {
                                const double want = (p == par) ? ya[s * 2 * nf * 12 + k] : 0.0;
                                if (yp[s * 2 * nf * 12 + k] != want) {
                                    failures++;
                                    break;
                                }
                            }
                        }
                    }
                }
                free(U); free(a); free(b); free(c); free(ya); free(yb); free(yc); free(yp);
            }
    }
    printf("oracle driver: %d failures\n", failures);
    return failures ? 1 : 0;
}
