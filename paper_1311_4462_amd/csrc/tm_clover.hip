// Twisted-clover term (the future work of Sec. 4): per site, from the links,
// the four-leaf clover field strength F_munu = (Q_munu - Q_munu^+)/8 and the
// chiral blocks of A = 1 + i kappa c_sw sum_{mu<nu} sigma_munu F_munu and of
// B = (A^2 + a^2 - b^2)^-1 (layout and use: CloverIO / apply_clover).
//
// In the chiral basis sigma_jk = -eps_jkl diag(s_l, s_l) and
// sigma_j4 = diag(s_j, -s_j) (s_l the Pauli matrices), so on the block of
// chirality chi
//     A_chi = 1 + i kappa c_sw sum_l s_l (x) G_l,
//     G_1 = -F_yz + chi F_xt,  G_2 = F_xz + chi F_yt,  G_3 = -F_xy + chi F_zt,
// i.e. the 6x6 matrix [[G_3, G_1 - i G_2], [G_1 + i G_2, -G_3]] on
// (spin pair, colour).  Everything is computed in FP64, once per gauge field.
#include "tm_fields.h"

namespace twm {

namespace {

struct M3 {
    cx<double> e[3][3];
};

__device__ M3 mmul(const M3 &a, const M3 &b)
{
    M3 c;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cx<double> s = mk(0.0, 0.0);
            for (int k = 0; k < 3; k++) s = s + cmul(a.e[i][k], b.e[k][j]);
            c.e[i][j] = s;
        }
    return c;
}

__device__ M3 hc(const M3 &a)
{
    M3 c;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) c.e[i][j] = conjg(a.e[j][i]);
    return c;
}

struct Geo {
    int X[4];
    long V;
};

// link U_mu at coordinates c (periodic), from canonical [mu][lex][3][3]
__device__ M3 link_at(const double2 *U, const Geo &g, int mu, int x, int y, int z, int t)
{
    x = (x + g.X[0]) % g.X[0];
    y = (y + g.X[1]) % g.X[1];
    z = (z + g.X[2]) % g.X[2];
    t = (t + g.X[3]) % g.X[3];
    const long lex = x + (long)g.X[0] * (y + (long)g.X[1] * (z + (long)g.X[2] * t));
    const double2 *p = U + ((long)mu * g.V + lex) * 9;
    M3 m;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) m.e[i][j] = mk(p[3 * i + j].x, p[3 * i + j].y);
    return m;
}

// F_munu(x) = (Q - Q^+)/8 with Q the four counter-clockwise leaves at x
__device__ M3 field_strength(const double2 *U, const Geo &g, const int (&c)[4], int mu, int nu)
{
    auto L = [&](int m, int dm, int dn) {
        int q[4] = {c[0], c[1], c[2], c[3]};
        q[mu] += dm;
        q[nu] += dn;
        return link_at(U, g, m, q[0], q[1], q[2], q[3]);
    };
    const M3 l1 = mmul(mmul(L(mu, 0, 0), L(nu, 1, 0)), mmul(hc(L(mu, 0, 1)), hc(L(nu, 0, 0))));
    const M3 l2 = mmul(mmul(L(nu, 0, 0), hc(L(mu, -1, 1))), mmul(hc(L(nu, -1, 0)), L(mu, -1, 0)));
    const M3 l3 = mmul(mmul(hc(L(mu, -1, 0)), hc(L(nu, -1, -1))), mmul(L(mu, -1, -1), L(nu, 0, -1)));
    const M3 l4 = mmul(mmul(hc(L(nu, 0, -1)), L(mu, 0, -1)), mmul(L(nu, 1, -1), hc(L(mu, 0, 0))));
    M3 f;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            const cx<double> q = l1.e[i][j] + l2.e[i][j] + l3.e[i][j] + l4.e[i][j];
            const cx<double> qt = conjg(l1.e[j][i] + l2.e[j][i] + l3.e[j][i] + l4.e[j][i]);
            f.e[i][j] = 0.125 * (q - qt);
        }
    return f;
}

// 6x6 complex inverse by Gauss-Jordan with partial pivoting; false if singular
__device__ bool inv6(cx<double> (&a)[6][6], cx<double> (&r)[6][6])
{
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 6; j++) r[i][j] = mk(i == j ? 1.0 : 0.0, 0.0);
    for (int col = 0; col < 6; col++) {
        int piv = col;
        double best = 0.0;
        for (int i = col; i < 6; i++) {
            const double m = a[i][col].re * a[i][col].re + a[i][col].im * a[i][col].im;
            if (m > best) {
                best = m;
                piv = i;
            }
        }
        if (!(best > 1e-200)) return false;
        if (piv != col)
            for (int j = 0; j < 6; j++) {
                const cx<double> t = a[col][j];
                a[col][j] = a[piv][j];
                a[piv][j] = t;
                const cx<double> u = r[col][j];
                r[col][j] = r[piv][j];
                r[piv][j] = u;
            }
        const cx<double> p = a[col][col];
        const double pn = p.re * p.re + p.im * p.im;
        const cx<double> ip = mk(p.re / pn, -p.im / pn);
        for (int j = 0; j < 6; j++) {
            a[col][j] = cmul(a[col][j], ip);
            r[col][j] = cmul(r[col][j], ip);
        }
        for (int i = 0; i < 6; i++) {
            if (i == col) continue;
            const cx<double> f = a[i][col];
            for (int j = 0; j < 6; j++) {
                a[i][j] = a[i][j] - cmul(f, a[col][j]);
                r[i][j] = r[i][j] - cmul(f, r[col][j]);
            }
        }
    }
    return true;
}

// Hermitian 6x6 -> 36 reals (diagonal re, then upper entries re, im)
__device__ void pack_herm(double (&d)[36], const cx<double> (&m)[6][6])
{
    for (int i = 0; i < 6; i++) d[i] = m[i][i].re;
    int o = 6;
    for (int i = 0; i < 6; i++)
        for (int j = i + 1; j < 6; j++) {
            d[o++] = m[i][j].re;
            d[o++] = m[i][j].im;
        }
}

__global__ void __launch_bounds__(64) clover_build_kernel(void *d64_0, void *d64_1, void *d32_0, void *d32_1,
                                                          const double2 *U, Geo g, uint32_t vh, double kc,
                                                          double shift, int *bad)
{
    const uint32_t cb = blockIdx.x * blockDim.x + threadIdx.x;
    const int par = blockIdx.y;
    if (cb >= vh) return;
    const int xh_n = g.X[0] >> 1;
    const int xh = (int)(cb % xh_n);
    int rest = (int)(cb / xh_n);
    const int y = rest % g.X[1];
    rest /= g.X[1];
    const int z = rest % g.X[2];
    const int t = rest / g.X[2];
    const int x = 2 * xh + ((y + z + t + par) & 1);
    const int c[4] = {x, y, z, t};

    for (int chi = 0; chi < 2; chi++) {
        const double sc = chi == 0 ? 1.0 : -1.0;
        // G_l = base_l + chi t_l (recomputed per block to keep the live state small)
        M3 G[3];
        {
            const M3 fyz = field_strength(U, g, c, 1, 2), fxt = field_strength(U, g, c, 0, 3);
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) G[0].e[i][j] = sc * fxt.e[i][j] - fyz.e[i][j];
        }
        {
            const M3 fxz = field_strength(U, g, c, 0, 2), fyt = field_strength(U, g, c, 1, 3);
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) G[1].e[i][j] = fxz.e[i][j] + sc * fyt.e[i][j];
        }
        {
            const M3 fxy = field_strength(U, g, c, 0, 1), fzt = field_strength(U, g, c, 2, 3);
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) G[2].e[i][j] = sc * fzt.e[i][j] - fxy.e[i][j];
        }
        // A = 1 + i kc [[G3, G1 - i G2], [G1 + i G2, -G3]]
        cx<double> A[6][6];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                const cx<double> g1 = G[0].e[i][j], g2 = G[1].e[i][j], g3 = G[2].e[i][j];
                const cx<double> e00 = g3, e01 = g1 - times_i(g2), e10 = g1 + times_i(g2), e11 = (-1.0) * g3;
                A[i][j] = kc * times_i(e00);
                A[i][j + 3] = kc * times_i(e01);
                A[i + 3][j] = kc * times_i(e10);
                A[i + 3][j + 3] = kc * times_i(e11);
            }
        for (int i = 0; i < 6; i++) A[i][i] = A[i][i] + mk(1.0, 0.0);
        double d[36];
        pack_herm(d, A);
        if (d64_0) CloverIO<TM_FP64>::store(par ? d64_1 : d64_0, vh, chi, cb, d);
        if (d32_0) CloverIO<TM_FP32>::store(par ? d32_1 : d32_0, vh, chi, cb, d);
        // B = (A^2 + a^2 - b^2)^-1
        cx<double> S[6][6], Bi[6][6];
        for (int i = 0; i < 6; i++)
            for (int j = 0; j < 6; j++) {
                cx<double> s = mk(i == j ? shift : 0.0, 0.0);
                for (int k = 0; k < 6; k++) s = s + cmul(A[i][k], A[k][j]);
                S[i][j] = s;
            }
        if (!inv6(S, Bi)) {
            *bad = 1;
            return;
        }
        // symmetrise against rounding before packing the upper triangle
        for (int i = 0; i < 6; i++)
            for (int j = i; j < 6; j++) {
                const cx<double> m = 0.5 * (Bi[i][j] + conjg(Bi[j][i]));
                Bi[i][j] = m;
                Bi[j][i] = conjg(m);
            }
        pack_herm(d, Bi);
        for (int k = 0; k < 36; k++)
            if (!isfinite(d[k])) *bad = 1;
        if (d64_0) CloverIO<TM_FP64>::store(par ? d64_1 : d64_0, vh, 2 + chi, cb, d);
        if (d32_0) CloverIO<TM_FP32>::store(par ? d32_1 : d32_0, vh, 2 + chi, cb, d);
    }
}

}  // namespace

hipError_t clover_build(void *const *d64, void *const *d32, const void *links, const int *X, uint32_t vh,
                        double kc, double shift, int *bad, hipStream_t st)
{
    Geo g{{X[0], X[1], X[2], X[3]}, 2L * vh};
    dim3 grid((vh + 63) / 64, 2);
    hipLaunchKernelGGL(clover_build_kernel, grid, dim3(64), 0, st, d64 ? d64[0] : nullptr,
                       d64 ? d64[1] : nullptr, d32 ? d32[0] : nullptr, d32 ? d32[1] : nullptr,
                       (const double2 *)links, g, vh, kc, shift, bad);
    return hipGetLastError();
}

}  // namespace twm
