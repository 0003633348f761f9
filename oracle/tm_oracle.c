/*
 * FP64 CPU oracle for the Wilson twisted-mass Dirac operator.
 *
 * TEST INFRASTRUCTURE ONLY: this file is compiled into liboracle.so, which is
 * loaded by the tests, by the smoke check and by the CPU-baseline leg of the
 * benchmark, never by the library's product path.  It shares no code, header,
 * table or constant with the HIP implementation.
 *
 * What is defined here is the Wilson hopping term that Eq. (2.1) calls D_W,
 * written out directly from its textbook definition (Wilson parameter r = 1):
 *
 *   (D psi)(x)  = sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *   (D^+ psi)(x)= sum_mu [ (1 + g_mu) U_mu(x) psi(x+mu) + (1 - g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *
 * with the gamma matrices of the non-relativistic basis of Sec. 2 (in 2x2
 * blocks g_k = [[0, i s_k], [-i s_k, 0]], g_4 = diag(1, 1, -1, -1)), periodic
 * boundaries in x, y, z and a factor `tsign` on every hop that crosses the
 * t = Lt-1 <-> 0 boundary (tsign = -1: antiperiodic).  The dagger is
 * implemented directly, not as g5 D g5, so that g5-hermiticity is a
 * non-trivial check.  The projectors act as full 4x4 matrices; no
 * spin-projection shortcut is used.  Flavour is a spectator of D.
 *
 * Canonical layouts (complex128 stored as interleaved re, im):
 *   site index  lex = x + Lx*(y + Ly*(z + Lz*t)),  parity (x+y+z+t) & 1
 *   spinor      [nrhs][lex][nf][4 spin][3 colour]
 *   links       [mu][lex][3][3]  (row-major; U_mu(x) carries colour from x+mu to x)
 */
#include <complex.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* gamma_mu for mu = 0..3 (x, y, z, t), [mu][row][col] */
static void build_gammas(cplx g[4][4][4])
{
    const cplx iu = _Complex_I;
    cplx sigma[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -iu}, {iu, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(g, 0, sizeof(cplx) * 64);
    for (int k = 0; k < 3; k++)
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                g[k][a][2 + b] = iu * sigma[k][a][b];      /* upper-right  i s_k */
                g[k][2 + a][b] = -iu * sigma[k][a][b];     /* lower-left  -i s_k */
            }
    g[3][0][0] = g[3][1][1] = 1;
    g[3][2][2] = g[3][3][3] = -1;
}

/* Export the four gamma matrices as 4*4*4 complex (tests check the Clifford algebra). */
void orc_gammas(double *out)
{
    cplx g[4][4][4];
    build_gammas(g);
    memcpy(out, g, sizeof(g));
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the later parallel loops (timing on one core or on all). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * out = D psi (dagger = 0) or D^+ psi (dagger = 1).  When out_parity is 0 or 1
 * only output sites of that parity are computed and all other output sites are
 * set to zero (this gives the even-odd blocks D_eo, D_oe); out_parity = -1
 * computes every site.
 */
int orc_hop(double *out_, const double *in_, const double *U_, const int *dims,
            int nf, int nrhs, int dagger, double tsign, int out_parity)
{
    cplx g[4][4][4];
    build_gammas(g);
    /* projectors for the forward (x+mu) and backward (x-mu) hops */
    cplx pf[4][4][4], pb[4][4][4];
    const double sf = dagger ? +1.0 : -1.0;   /* forward: 1 - g (D) or 1 + g (D^+) */
    for (int mu = 0; mu < 4; mu++)
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) {
                cplx one = (a == b) ? 1.0 : 0.0;
                pf[mu][a][b] = one + sf * g[mu][a][b];
                pb[mu][a][b] = one - sf * g[mu][a][b];
            }

    const int L[4] = {dims[0], dims[1], dims[2], dims[3]};
    const long V = (long)L[0] * L[1] * L[2] * L[3];
    const long ss = (long)nf * 12;             /* complex numbers per site */
    cplx *out = (cplx *)out_;
    const cplx *in = (const cplx *)in_;
    const cplx *U = (const cplx *)U_;

#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        int c[4];
        long r = s;
        for (int d = 0; d < 4; d++) { c[d] = (int)(r % L[d]); r /= L[d]; }
        const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
        for (int rhs = 0; rhs < nrhs; rhs++) {
            cplx *o = out + ((long)rhs * V + s) * ss;
            if (out_parity >= 0 && par != out_parity) {
                for (long k = 0; k < ss; k++) o[k] = 0;
                continue;
            }
            for (int f = 0; f < nf; f++) {
                cplx acc[4][3] = {{0}};
                for (int mu = 0; mu < 4; mu++) {
                    for (int dir = 0; dir < 2; dir++) {     /* 0: forward, 1: backward */
                        int n[4] = {c[0], c[1], c[2], c[3]};
                        double sign = 1.0;
                        if (dir == 0) {
                            n[mu] = (c[mu] + 1) % L[mu];
                            if (mu == 3 && c[3] == L[3] - 1) sign = tsign;
                        } else {
                            n[mu] = (c[mu] - 1 + L[mu]) % L[mu];
                            if (mu == 3 && c[3] == 0) sign = tsign;
                        }
                        const long sn = n[0] + (long)L[0] * (n[1] + (long)L[1] * (n[2] + (long)L[2] * n[3]));
                        const cplx *psi = in + ((long)rhs * V + sn) * ss + (long)f * 12;
                        /* link: forward U_mu(x); backward U_mu(x-mu)^+ */
                        const cplx *u = U + ((long)mu * V + (dir == 0 ? s : sn)) * 9;
                        cplx chi[4][3];
                        for (int sp = 0; sp < 4; sp++)
                            for (int a = 0; a < 3; a++) {
                                cplx t = 0;
                                for (int b = 0; b < 3; b++) {
                                    cplx m = (dir == 0) ? u[a * 3 + b] : conj(u[b * 3 + a]);
                                    t += m * psi[sp * 3 + b];
                                }
                                chi[sp][a] = t;
                            }
                        cplx (*P)[4] = (dir == 0) ? pf[mu] : pb[mu];
                        for (int sp = 0; sp < 4; sp++)
                            for (int a = 0; a < 3; a++) {
                                cplx t = 0;
                                for (int sq = 0; sq < 4; sq++) t += P[sp][sq] * chi[sq][a];
                                acc[sp][a] += sign * t;
                            }
                    }
                }
                for (int sp = 0; sp < 4; sp++)
                    for (int a = 0; a < 3; a++) o[f * 12 + sp * 3 + a] = acc[sp][a];
            }
        }
    }
    return 0;
}
