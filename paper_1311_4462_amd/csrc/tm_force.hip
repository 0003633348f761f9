// Gauge force of S = phi^+ (M^+ M)^-1 phi (M: the preconditioned operator of
// Eq. 2.2 or 2.3) from colour outer products of four spinor fields.
//
// With X = (M^+ M)^-1 phi, Y = M X, A = Y (asym) or R_ee^-+ Y (sym) on even
// sites and R_oo^-+ (D^+)_oe A on odd sites, B = X on even and R_oo^-1 D_oe X
// on odd sites, a link variation changes S by dS = 2 kappa^2 Re <A, dD B>.
// For the link U_mu(x) (boundary factor s):
//   G = 2 kappa^2 s sum_{flavour, spin} [ (1 - g_mu) A(x) B(x+mu)^+ + B(x) ((1 + g_mu) A(x+mu))^+ ]
// is the unconstrained gradient (dS = Re tr(G^+ dU)) and F = -1/2 T_A(U G^+)
// the traceless anti-Hermitian force (dS/dw^a = -2 tr(F T^a) for
// U -> exp(w^a T^a) U).  Because (1 -+ g_mu)/2 is a projector of rank two,
// sum_spin ((1 - g) A)_s B_s^+ = sum_j hA_j hB_j^+ with hA, hB the two-spin
// projections of A and B: each term is two 3x3 outer products.
#include "tm_fields.h"

namespace twm {

// two-spin projection of a full site vector v under (1 - SIG g_mu) (time: the
// kept spin pair, without the factor 2)
template <int MU, int SIG, typename T>
__device__ __forceinline__ void half_proj(const cx<T> *v, cx<T> (&h)[2][3])
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if constexpr (MU == 0) {
            if constexpr (SIG > 0) {
                h[0][c] = v[c] + times_mi(v[9 + c]);
                h[1][c] = v[3 + c] + times_mi(v[6 + c]);
            } else {
                h[0][c] = v[c] + times_i(v[9 + c]);
                h[1][c] = v[3 + c] + times_i(v[6 + c]);
            }
        } else if constexpr (MU == 1) {
            if constexpr (SIG > 0) {
                h[0][c] = v[c] - v[9 + c];
                h[1][c] = v[3 + c] + v[6 + c];
            } else {
                h[0][c] = v[c] + v[9 + c];
                h[1][c] = v[3 + c] - v[6 + c];
            }
        } else if constexpr (MU == 2) {
            if constexpr (SIG > 0) {
                h[0][c] = v[c] + times_mi(v[6 + c]);
                h[1][c] = v[3 + c] + times_i(v[9 + c]);
            } else {
                h[0][c] = v[c] + times_i(v[6 + c]);
                h[1][c] = v[3 + c] + times_mi(v[9 + c]);
            }
        } else {
            const int o = (SIG > 0) ? 6 : 0;
            h[0][c] = v[o + c];
            h[1][c] = v[o + 3 + c];
        }
    }
}

// G += sum_j p_j q_j^+   (3x3 outer products)
template <typename T>
__device__ __forceinline__ void add_outer(cx<T> (&G)[3][3], const cx<T> (&p)[2][3], const cx<T> (&q)[2][3])
{
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) G[a][b] = G[a][b] + cmul(p[j][a], conjg(q[j][b]));
}

struct ForceArgs {
    int X[4];
    uint32_t vh;
    int nf;
    double tsign;
    double k2x2;        // 2 kappa^2
    double coeff;
    int accumulate;
    const void *gauge[2];
    SpinorPtr Ae, Wo, Xe, Zo;   // A and B on even / odd sites
    void *F;
    void *G;            // nullable
};

template <int P, int NF, int MU>
__device__ __forceinline__ void force_terms(cx<typename Prec<P>::real> (&G)[3][3], const ForceArgs &a,
                                            int par, uint32_t cb, uint32_t nb)
{
    using real = typename Prec<P>::real;
    const SpinorPtr &A_x = par == 0 ? a.Ae : a.Wo;
    const SpinorPtr &B_x = par == 0 ? a.Xe : a.Zo;
    const SpinorPtr &A_n = par == 0 ? a.Wo : a.Ae;
    const SpinorPtr &B_n = par == 0 ? a.Zo : a.Xe;
#pragma unroll
    for (int f = 0; f < NF; f++) {
        cx<real> v[12], w[12];
        cx<real> hA[2][3], hB[2][3];
        // (1 - g) A(x) B(x+mu)^+
        SpinorIO<P>::template load<0, 12>(v, A_x, a.vh, f, cb);
        SpinorIO<P>::template load<0, 12>(w, B_n, a.vh, f, nb);
        half_proj<MU, 1>(v, hA);
        half_proj<MU, 1>(w, hB);
        add_outer(G, hA, hB);
        // B(x) ((1 + g) A(x+mu))^+
        SpinorIO<P>::template load<0, 12>(v, A_n, a.vh, f, nb);
        SpinorIO<P>::template load<0, 12>(w, B_x, a.vh, f, cb);
        half_proj<MU, -1>(v, hA);
        half_proj<MU, -1>(w, hB);
        add_outer(G, hB, hA);
    }
}

template <int P, int NF, int RECON, typename FT>
__global__ void __launch_bounds__(256) force_kernel(const ForceArgs a)
{
    using real = typename Prec<P>::real;
    const uint32_t cb = blockIdx.x * 256 + threadIdx.x;
    const int par = blockIdx.y;
    const int mu = blockIdx.z;
    if (cb >= a.vh) return;
    const int Lx = a.X[0], Ly = a.X[1], Lz = a.X[2], Lt = a.X[3];
    const int xh_n = Lx >> 1;
    const int xh = cb % xh_n;
    int rest = cb / xh_n;
    const int y = rest % Ly;
    rest /= Ly;
    const int z = rest % Lz;
    const int t = rest / Lz;
    const int x = 2 * xh + ((y + z + t + par) & 1);
    const uint32_t base = cb - xh;
    const uint32_t sy = xh_n, sz = (uint32_t)xh_n * Ly, st = (uint32_t)xh_n * Ly * Lz;

    cx<real> G[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) G[i][j] = mk((real)0, (real)0);
    real s = (real)a.k2x2;
    if (mu == 0) {
        const int xp = (x + 1 == Lx) ? 0 : x + 1;
        force_terms<P, NF, 0>(G, a, par, cb, base + (xp >> 1));
    } else if (mu == 1) {
        force_terms<P, NF, 1>(G, a, par, cb, (y == Ly - 1) ? cb - (uint32_t)(Ly - 1) * sy : cb + sy);
    } else if (mu == 2) {
        force_terms<P, NF, 2>(G, a, par, cb, (z == Lz - 1) ? cb - (uint32_t)(Lz - 1) * sz : cb + sz);
    } else {
        force_terms<P, NF, 3>(G, a, par, cb, (t == Lt - 1) ? cb - (uint32_t)(Lt - 1) * st : cb + st);
        s *= (real)2;                                   // the time projector keeps 2 psi
        if (t == Lt - 1) s *= (real)a.tsign;
    }
    const real c = (real)a.coeff;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) G[i][j] = (s * c) * G[i][j];

    // F = -1/2 T_A(U G^+), T_A(M) = (M - M^+)/2 - tr(M - M^+)/6
    cx<real> u[3][3];
    LinkIO<P, RECON>::load(u, a.gauge[par], a.vh, mu, cb);
    cx<real> M[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<real> acc = cmul(u[i][0], conjg(G[j][0]));
            acc = acc + cmul(u[i][1], conjg(G[j][1]));
            acc = acc + cmul(u[i][2], conjg(G[j][2]));
            M[i][j] = acc;
        }
    const real trim = (M[0][0].im + M[1][1].im + M[2][2].im) / (real)3;   // Im tr M / 3
    const long lex = 2L * base + x;
    const long V = 2L * a.vh;
    FT *F = (FT *)a.F + ((long)mu * V + lex) * 9;
    FT *Gout = a.G ? (FT *)a.G + ((long)mu * V + lex) * 9 : nullptr;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            // (M - M^+)/2 at (i, j) = (M_ij - conj(M_ji)) / 2
            real re = (real)0.5 * (M[i][j].re - M[j][i].re);
            real im = (real)0.5 * (M[i][j].im + M[j][i].im);
            if (i == j) im -= trim;
            re *= (real)-0.5;
            im *= (real)-0.5;
            FT f;
            f.x = re;
            f.y = im;
            if (a.accumulate) {
                const FT o = F[i * 3 + j];
                f.x += o.x;
                f.y += o.y;
            }
            F[i * 3 + j] = f;
            if (Gout) {
                FT gv;
                gv.x = G[i][j].re;
                gv.y = G[i][j].im;
                if (a.accumulate) {
                    const FT o = Gout[i * 3 + j];
                    gv.x += o.x;
                    gv.y += o.y;
                }
                Gout[i * 3 + j] = gv;
            }
        }
}

hipError_t force_launch(int prec, int nf, int force_prec, void *F, void *G, const void *gauge0,
                        const void *gauge1, int recon, SpinorPtr A[2], SpinorPtr Bv[2],
                        const int *X, uint32_t vh, double tsign, double coeff, int accumulate,
                        double kappa, hipStream_t st)
{
    ForceArgs a;
    for (int d = 0; d < 4; d++) a.X[d] = X[d];
    a.vh = vh;
    a.nf = nf;
    a.tsign = tsign;
    a.k2x2 = 2.0 * kappa * kappa;
    a.coeff = coeff;
    a.accumulate = accumulate;
    a.gauge[0] = gauge0;
    a.gauge[1] = gauge1;
    a.Ae = A[0];
    a.Wo = A[1];
    a.Xe = Bv[0];
    a.Zo = Bv[1];
    a.F = F;
    a.G = G;
    dim3 grid((vh + 255) / 256, 2, 4);
#define TM_FK(P, NF, R, FT)                                                                     \
    if (prec == P && nf == NF && recon == R && force_prec == (sizeof(FT) == 16 ? TM_FP64 : TM_FP32)) { \
        hipLaunchKernelGGL((force_kernel<P, NF, R, FT>), grid, dim3(256), 0, st, a);            \
        return hipGetLastError();                                                               \
    }
    TM_FK(TM_FP64, 1, 12, double2) TM_FK(TM_FP64, 2, 12, double2)
    TM_FK(TM_FP64, 1, 18, double2) TM_FK(TM_FP64, 2, 18, double2)
    TM_FK(TM_FP32, 1, 12, float2) TM_FK(TM_FP32, 2, 12, float2)
    TM_FK(TM_FP32, 1, 18, float2) TM_FK(TM_FP32, 2, 18, float2)
    TM_FK(TM_FP64, 1, 12, float2) TM_FK(TM_FP64, 2, 12, float2)
    TM_FK(TM_FP32, 1, 12, double2) TM_FK(TM_FP32, 2, 12, double2)
#undef TM_FK
    return hipErrorInvalidConfiguration;
}

}  // namespace twm
