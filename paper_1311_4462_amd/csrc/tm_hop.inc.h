// Fused Wilson twisted-mass hop kernel (Sec. 2.1: the hop fused with the local
// twist R^-1 and with the kappa^2 xpay of Eqs. 2.2 / 2.3, for one flavour or
// for the non-degenerate doublet with each link loaded once for both flavours).
//
// One thread computes one output site for NR right-hand sides and NF
// flavours.  For every direction it loads the link (rebuilding row 2 from
// rows 0, 1 when 12 reals are stored), loads the neighbour (only the spin
// pair the time projector keeps, in the basis of Sec. 2), spin-projects to a
// half spinor, multiplies by U or U^+, and rebuilds the lower spin pair.
// The epilogue applies the twist / xpay of tm_epilogue and optionally adds
// the squared norm of the output to a deterministic two-stage reduction.
#pragma once

#include "tm_fields.h"

namespace twm {

// acc += k f g with k = +1 (K = 0), -1 (K = 1), +i (K = 2) or -i (K = 3):
// two FMAs.
template <int K, typename T>
__device__ __forceinline__ void acc_k(cx<T> &acc, T f, cx<T> g)
{
    if constexpr (K == 0) {
        acc.re = fma(f, g.re, acc.re);
        acc.im = fma(f, g.im, acc.im);
    } else if constexpr (K == 1) {
        acc.re = fma(-f, g.re, acc.re);
        acc.im = fma(-f, g.im, acc.im);
    } else if constexpr (K == 2) {
        acc.re = fma(-f, g.im, acc.re);
        acc.im = fma(f, g.re, acc.im);
    } else {
        acc.re = fma(f, g.im, acc.re);
        acc.im = fma(-f, g.re, acc.im);
    }
}

// Row a of U h (BWD: of U^+ h) as two FMA chains of six terms.
template <bool BWD, typename T>
__device__ __forceinline__ cx<T> link_row(const cx<T> (&u)[3][3], const cx<T> (&h)[3], int a)
{
    T re, im;
    if constexpr (!BWD) {
        re = u[a][0].re * h[0].re;
        re = fma(-u[a][0].im, h[0].im, re);
        im = u[a][0].re * h[0].im;
        im = fma(u[a][0].im, h[0].re, im);
#pragma unroll
        for (int b = 1; b < 3; b++) {
            re = fma(u[a][b].re, h[b].re, re);
            re = fma(-u[a][b].im, h[b].im, re);
            im = fma(u[a][b].re, h[b].im, im);
            im = fma(u[a][b].im, h[b].re, im);
        }
    } else {
        re = u[0][a].re * h[0].re;
        re = fma(u[0][a].im, h[0].im, re);
        im = u[0][a].re * h[0].im;
        im = fma(-u[0][a].im, h[0].re, im);
#pragma unroll
        for (int b = 1; b < 3; b++) {
            re = fma(u[b][a].re, h[b].re, re);
            re = fma(u[b][a].im, h[b].im, re);
            im = fma(u[b][a].re, h[b].im, im);
            im = fma(-u[b][a].im, h[b].re, im);
        }
    }
    return mk(re, im);
}

// Spin projection of the neighbour v to the half spinor h:
//   SIG = +1: projector (1 - g_mu);  SIG = -1: projector (1 + g_mu).
// v holds the 12 elements of the neighbour (or, for MU == 3, only the 6
// elements of the spin pair the projector keeps, at v[0..5]).
template <int MU, int SIG, typename T>
__device__ __forceinline__ void project(cx<T> (&h)[2][3], const cx<T> *v)
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if constexpr (MU == 0) {          // i s_1 psiL = (i psi3, i psi2)
            if constexpr (SIG > 0) {
                h[0][c] = v[c] + times_mi(v[9 + c]);
                h[1][c] = v[3 + c] + times_mi(v[6 + c]);
            } else {
                h[0][c] = v[c] + times_i(v[9 + c]);
                h[1][c] = v[3 + c] + times_i(v[6 + c]);
            }
        } else if constexpr (MU == 1) {   // i s_2 psiL = (psi3, -psi2)
            if constexpr (SIG > 0) {
                h[0][c] = v[c] - v[9 + c];
                h[1][c] = v[3 + c] + v[6 + c];
            } else {
                h[0][c] = v[c] + v[9 + c];
                h[1][c] = v[3 + c] - v[6 + c];
            }
        } else if constexpr (MU == 2) {   // i s_3 psiL = (i psi2, -i psi3)
            if constexpr (SIG > 0) {
                h[0][c] = v[c] + times_mi(v[6 + c]);
                h[1][c] = v[3 + c] + times_i(v[9 + c]);
            } else {
                h[0][c] = v[c] + times_i(v[6 + c]);
                h[1][c] = v[3 + c] + times_mi(v[9 + c]);
            }
        } else {                          // time: 2 psiL (SIG > 0) or 2 psiU
            h[0][c] = v[c];
            h[1][c] = v[3 + c];
        }
    }
}

// Rebuild the lower spin pair from the six link products g[s][c] (s: row of
// the half spinor, c: colour) and accumulate with the factor sgn (boundary
// sign, and 2 for the time projector) through the accumulating FMAs.
template <int MU, int SIG, typename T>
__device__ __forceinline__ void accumulate_hop(cx<T> (&acc)[12], const cx<T> (&g)[2][3], T sgn)
{
    const T f = (MU == 3) ? (T)2 * sgn : sgn;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const cx<T> g0 = g[0][c], g1 = g[1][c];
        if constexpr (MU == 3) {
            if constexpr (SIG > 0) {
                acc_k<0>(acc[6 + c], f, g0);
                acc_k<0>(acc[9 + c], f, g1);
            } else {
                acc_k<0>(acc[c], f, g0);
                acc_k<0>(acc[3 + c], f, g1);
            }
        } else {
            acc_k<0>(acc[c], f, g0);
            acc_k<0>(acc[3 + c], f, g1);
            // lower pair: SIG * i s_k g
            if constexpr (MU == 0) {          // (i g1, i g0)
                acc_k<(SIG > 0 ? 2 : 3)>(acc[6 + c], f, g1);
                acc_k<(SIG > 0 ? 2 : 3)>(acc[9 + c], f, g0);
            } else if constexpr (MU == 1) {   // (g1, -g0)
                acc_k<(SIG > 0 ? 0 : 1)>(acc[6 + c], f, g1);
                acc_k<(SIG > 0 ? 1 : 0)>(acc[9 + c], f, g0);
            } else {                          // (i g0, -i g1)
                acc_k<(SIG > 0 ? 2 : 3)>(acc[6 + c], f, g0);
                acc_k<(SIG > 0 ? 3 : 2)>(acc[9 + c], f, g1);
            }
        }
    }
}

// Multiply the half spinor by the link (BWD: by U^+) as FMA chains and
// accumulate.
template <int MU, int SIG, bool BWD, typename T>
__device__ __forceinline__ void mul_accumulate(cx<T> (&acc)[12], const cx<T> (&u)[3][3],
                                               const cx<T> (&h)[2][3], T sgn)
{
    cx<T> g[2][3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        g[0][c] = link_row<BWD>(u, h[0], c);
        g[1][c] = link_row<BWD>(u, h[1], c);
    }
    accumulate_hop<MU, SIG>(acc, g, sgn);
}

// ---- binary16: projection and link products on packed pairs
//
// The projected half spinor h is rounded once to binary16 (the precision the
// neighbour is stored in) and each real part of a link product becomes three
// two-term dot products with FP32 accumulation (binary16 products are exact
// in FP32):
//   U h:   re = sum_b u_ab . (h.re, -h.im),  im = sum_b u_ab . (h.im,  h.re)
//   U^+ h: re = sum_b u_ba . (h.re,  h.im),  im = sum_b u_ba . (h.im, -h.re)
// The two pairs each product needs, p = (h.re, +-h.im) and s = (h.im, +-h.re),
// come straight from the stored words, one packed addition each.
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
// h = a + k b of two stored words (k = +1, -1, +i, -i for K = 0..3):
//   p = (h.re, -h.im) if BWD is false, else (h.re, h.im);
//   s = (h.im, h.re) if BWD is false, else (h.im, -h.re).
// Each is one packed addition with per-lane operand halves (op_sel: low
// lane, op_sel_hi: high lane) and per-lane signs of the operands.
template <int K, bool BWD>
__device__ __forceinline__ void pair_cadd(f16x2 &p, f16x2 &s, uint32_t a, uint32_t b)
{
    uint32_t x, y;
#define TM_PK(D, MODS) __asm__("v_pk_add_f16 %0, %1, %2 " MODS : "=v"(D) : "v"(a), "v"(b))
    if constexpr (K == 0) {          // h = (a.re + b.re, a.im + b.im)
        if constexpr (!BWD) {
            TM_PK(x, "neg_hi:[1,1]");
            TM_PK(y, "op_sel:[1,1] op_sel_hi:[0,0]");
        } else {
            TM_PK(x, "");
            TM_PK(y, "op_sel:[1,1] op_sel_hi:[0,0] neg_hi:[1,1]");
        }
    } else if constexpr (K == 1) {   // h = (a.re - b.re, a.im - b.im)
        if constexpr (!BWD) {
            TM_PK(x, "neg_lo:[0,1] neg_hi:[1,0]");
            TM_PK(y, "op_sel:[1,1] op_sel_hi:[0,0] neg_lo:[0,1] neg_hi:[0,1]");
        } else {
            TM_PK(x, "neg_lo:[0,1] neg_hi:[0,1]");
            TM_PK(y, "op_sel:[1,1] op_sel_hi:[0,0] neg_lo:[0,1] neg_hi:[1,0]");
        }
    } else if constexpr (K == 2) {   // h = (a.re - b.im, a.im + b.re)
        if constexpr (!BWD) {
            TM_PK(x, "op_sel:[0,1] op_sel_hi:[1,0] neg_lo:[0,1] neg_hi:[1,1]");
            TM_PK(y, "op_sel:[1,0] op_sel_hi:[0,1] neg_hi:[0,1]");
        } else {
            TM_PK(x, "op_sel:[0,1] op_sel_hi:[1,0] neg_lo:[0,1]");
            TM_PK(y, "op_sel:[1,0] op_sel_hi:[0,1] neg_hi:[1,0]");
        }
    } else {                         // h = (a.re + b.im, a.im - b.re)
        if constexpr (!BWD) {
            TM_PK(x, "op_sel:[0,1] op_sel_hi:[1,0] neg_hi:[1,0]");
            TM_PK(y, "op_sel:[1,0] op_sel_hi:[0,1] neg_lo:[0,1]");
        } else {
            TM_PK(x, "op_sel:[0,1] op_sel_hi:[1,0] neg_hi:[0,1]");
            TM_PK(y, "op_sel:[1,0] op_sel_hi:[0,1] neg_lo:[0,1] neg_hi:[1,1]");
        }
    }
#undef TM_PK
    p = __builtin_bit_cast(f16x2, x);
    s = __builtin_bit_cast(f16x2, y);
}

template <int MU, int SIG, bool BWD>
__device__ __forceinline__ void project_pairs(f16x2 (&hp)[2][3], f16x2 (&hs)[2][3], const uint32_t *w)
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if constexpr (MU == 0) {
            pair_cadd<(SIG > 0 ? 3 : 2), BWD>(hp[0][c], hs[0][c], w[c], w[9 + c]);
            pair_cadd<(SIG > 0 ? 3 : 2), BWD>(hp[1][c], hs[1][c], w[3 + c], w[6 + c]);
        } else if constexpr (MU == 1) {
            pair_cadd<(SIG > 0 ? 1 : 0), BWD>(hp[0][c], hs[0][c], w[c], w[9 + c]);
            pair_cadd<(SIG > 0 ? 0 : 1), BWD>(hp[1][c], hs[1][c], w[3 + c], w[6 + c]);
        } else if constexpr (MU == 2) {
            pair_cadd<(SIG > 0 ? 3 : 2), BWD>(hp[0][c], hs[0][c], w[c], w[6 + c]);
            pair_cadd<(SIG > 0 ? 2 : 3), BWD>(hp[1][c], hs[1][c], w[3 + c], w[9 + c]);
        } else {
            // time: h is the stored spin pair; sign flips and the swap are
            // bit operations on the word
#pragma unroll
            for (int r = 0; r < 2; r++) {
                const uint32_t v = w[3 * r + c];
                const uint32_t sw = (v >> 16) | (v << 16);
                hp[r][c] = __builtin_bit_cast(f16x2, BWD ? v : v ^ 0x80000000u);
                hs[r][c] = __builtin_bit_cast(f16x2, BWD ? sw ^ 0x80000000u : sw);
            }
        }
    }
}

// d = u . v + c with FP32 accumulation.  Written with the compiler's builtin
// so that the wait states a dot product's result needs before another VALU
// instruction reads it are inserted.
__device__ __forceinline__ float dot2_acc(f16x2 u, f16x2 v, float c)
{
    return __builtin_amdgcn_fdot2(u, v, c, false);
}

// Row a of U h (BWD: of U^+ h) from the pairs of pair_cadd.
template <bool BWD>
__device__ __forceinline__ cx<float> link_row_pairs(const f16x2 (&u)[3][3], const f16x2 (&hp)[3],
                                                    const f16x2 (&hs)[3], int a)
{
    float re = dot2_acc(BWD ? u[0][a] : u[a][0], hp[0], 0.f);
    float im = dot2_acc(BWD ? u[0][a] : u[a][0], hs[0], 0.f);
#pragma unroll
    for (int b = 1; b < 3; b++) {
        re = dot2_acc(BWD ? u[b][a] : u[a][b], hp[b], re);
        im = dot2_acc(BWD ? u[b][a] : u[a][b], hs[b], im);
    }
    return mk(re, im);
}

// Project, multiply by the link and accumulate one hop (BWD: U^+).
template <int MU, int SIG, bool BWD, typename T>
__device__ __forceinline__ void hop_accumulate(cx<T> (&acc)[12], const cx<T> (&u)[3][3],
                                               const cx<T> *v, T sgn)
{
    cx<T> h[2][3];
    project<MU, SIG>(h, v);
    mul_accumulate<MU, SIG, BWD>(acc, u, h, sgn);
}

// binary16 neighbour vec at site nb, hop in direction MU with a link already
// in packed pairs (u2[a][b] = (re, im) of U_ab): projection, the three
// two-term dot products per real part, accumulation with the site scale.
template <int MU, int SIG, bool BWD>
__device__ __forceinline__ void load_hop_pairs(cx<float> (&acc)[12], const f16x2 (&u2)[3][3], const SpinorPtr &in,
                                               uint32_t vh, uint32_t vec, uint32_t nb, float sgn, bool tnt)
{
    constexpr int P = TM_FP16;
    float sc;
    uint32_t w[12];
    if constexpr (MU == 3) {
        constexpr int K0 = SIG > 0 ? 6 : 0;
        if (tnt)
            SpinorIO<P>::template load_words<K0, 6, true>(w, in, vh, vec, nb, sc);
        else
            SpinorIO<P>::template load_words<K0, 6, false>(w, in, vh, vec, nb, sc);
    } else {
        SpinorIO<P>::template load_words<0, 12>(w, in, vh, vec, nb, sc);
    }
    f16x2 hp[2][3], hs[2][3];
    project_pairs<MU, SIG, BWD>(hp, hs, w);
    cx<float> g[2][3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        g[0][c] = link_row_pairs<BWD>(u2, hp[0], hs[0], c);
        g[1][c] = link_row_pairs<BWD>(u2, hp[1], hs[1], c);
    }
    accumulate_hop<MU, SIG>(acc, g, sgn * sc);
}

// A link as packed binary16 pairs.
__device__ __forceinline__ void link_pairs(f16x2 (&u2)[3][3], const cx<float> (&u)[3][3])
{
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) u2[a][b] = (f16x2){(_Float16)u[a][b].re, (_Float16)u[a][b].im};
}

// Load the neighbour vector vec at site nb for a hop in direction MU and
// accumulate it.  The half-precision site scale enters with the hop's factor;
// binary16 neighbours go through the packed pairs above, the other formats
// through project() and the FMA chains.
template <int P, int MU, int SIG, bool BWD>
__device__ __forceinline__ void load_hop(cx<typename Prec<P>::real> (&acc)[12],
                                         const cx<typename Prec<P>::real> (&u)[3][3], const SpinorPtr &in,
                                         uint32_t vh, uint32_t vec, uint32_t nb, typename Prec<P>::real sgn,
                                         bool tnt = false)
{
    using real = typename Prec<P>::real;
    real sc;
    if constexpr (P == TM_FP16) {
        f16x2 u2[3][3];
        link_pairs(u2, u);
        load_hop_pairs<MU, SIG, BWD>(acc, u2, in, vh, vec, nb, sgn, tnt);
        (void)sc;
    } else {
        cx<real> v[12], h[2][3];
        if constexpr (MU == 3) {
            constexpr int K0 = SIG > 0 ? 6 : 0;
            if (tnt)
                SpinorIO<P>::template load_unscaled<K0, 6, true>(v, in, vh, vec, nb, sc);
            else
                SpinorIO<P>::template load_unscaled<K0, 6, false>(v, in, vh, vec, nb, sc);
        } else {
            SpinorIO<P>::template load_unscaled<0, 12>(v, in, vh, vec, nb, sc);
        }
        project<MU, SIG>(h, v);
        mul_accumulate<MU, SIG, BWD>(acc, u, h, sgn * sc);
    }
}

// Doublet sites are split over lane pairs: lane 2k holds flavour 0 and lane
// 2k+1 flavour 1 of the same site (both load the same link, which the memory
// pipeline coalesces into one request); the flavour-mixing twist exchanges
// the partner's values with a lane-xor-1 shuffle.  This keeps the per-thread
// state of the doublet kernel at that of the one-flavour kernel.
template <int NF>
constexpr bool nd_split()
{
    return NF == 2 && kNdSplit;
}
template <int NF>
constexpr int flavours_per_thread()
{
    return nd_split<NF>() ? 1 : NF;
}

template <typename T>
__device__ __forceinline__ cx<T> partner(cx<T> a)
{
    return mk(__shfl_xor(a.re, 1, 64), __shfl_xor(a.im, 1, 64));
}

// This lane's flavour of R v or R^-1 v for a split doublet (the other
// flavour's v comes from the partner lane):
//   (R v)_f = v_f + i ta t3_f g5 v_f + b v_(1-f),
//   (R^-1 v)_f = c (v_f - i ta t3_f g5 v_f - b v_(1-f)).
template <typename T>
__device__ __forceinline__ void twist_split(cx<T> (&o)[12], const cx<T> (&v)[12], const Twist &tw,
                                            bool inverse, int fl)
{
    const T s = inverse ? (T)-1 : (T)1;
    const T c = inverse ? (T)tw.c : (T)1;
    const T t3 = fl ? (T)-tw.ta : (T)tw.ta;
    const T b = (T)tw.b;
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const int kk = (k < 6) ? k + 6 : k - 6;
        const cx<T> r = v[k] + (s * t3) * times_i(v[kk]) + (s * b) * partner(v[k]);
        o[k] = c * r;
    }
}

// One direction, forward (FWD) or backward, for all rhs and flavours.
template <int P, int NF, int NR, bool DAG, bool TWL, int RECON, bool LNT, int MU, bool FWD,
          bool LDSS = false>
__device__ __forceinline__ void hop_direction(
    cx<typename Prec<P>::real> (&acc)[NR][flavours_per_thread<NF>()][12], const HopProblem &pb,
    uint32_t nb, uint32_t link_cb, int link_par, int r0, typename Prec<P>::real sgn, int fl,
    const float4 *lds = nullptr, uint32_t lo = 0, uint32_t span = 0, int nts = 0)
{
    using real = typename Prec<P>::real;
    constexpr int SIG = (FWD != DAG) ? 1 : -1;   // D: 1 - g forward; D^+ swaps
    const uint32_t vh = pb.vh;
    cx<real> u[3][3];
    LinkIO<P, RECON, LNT>::load(u, pb.gauge[link_par], vh, MU, link_cb);
    if constexpr (nd_split<NF>()) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<real> v[12];
            const uint32_t vec = (uint32_t)((r0 + r) * NF + fl);
            if constexpr (TWL) {
                cx<real> w[12];
                SpinorIO<P>::template load<0, 12>(w, pb.in, vh, vec, nb);
                twist_split(v, w, pb.tw, true, fl);
                if constexpr (MU == 3)
                    hop_accumulate<MU, SIG, !FWD>(acc[r][0], u, v + (SIG > 0 ? 6 : 0), sgn);
                else
                    hop_accumulate<MU, SIG, !FWD>(acc[r][0], u, v, sgn);
            } else {
                load_hop<P, MU, SIG, !FWD>(acc[r][0], u, pb.in, vh, vec, nb, sgn, (nts & kNtTime) != 0);
            }
        }
    } else if constexpr (TWL) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<real> v[NF][12];
#pragma unroll
            for (int f = 0; f < NF; f++)
                SpinorIO<P>::template load<0, 12>(v[f], pb.in, vh, (uint32_t)((r0 + r) * NF + f), nb);
            apply_twist<real, NF>(v, pb.tw, true);
#pragma unroll
            for (int f = 0; f < NF; f++) {
                if constexpr (MU == 3)
                    hop_accumulate<MU, SIG, !FWD>(acc[r][f], u, v[f] + (SIG > 0 ? 6 : 0), sgn);
                else
                    hop_accumulate<MU, SIG, !FWD>(acc[r][f], u, v[f], sgn);
            }
        }
    } else {
        if constexpr (LDSS && MU < 2) {
            // x and y neighbours of the block's sites come from the staged copy
            static_assert(P == TM_FP32 && NF == 1 && NR == 1, "LDS staging: FP32, one flavour, one rhs");
            const uint32_t o = nb - lo;
            if (o < span) {
                cx<real> v[12];
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    const float4 c = lds[k * span + o];
                    v[2 * k] = mk(c.x, c.y);
                    v[2 * k + 1] = mk(c.z, c.w);
                }
                hop_accumulate<MU, SIG, !FWD>(acc[0][0], u, v, sgn);
                return;
            }
        }
#pragma unroll
        for (int r = 0; r < NR; r++)
#pragma unroll
            for (int f = 0; f < NF; f++) {
                load_hop<P, MU, SIG, !FWD>(acc[r][f], u, pb.in, vh, (uint32_t)((r0 + r) * NF + f), nb, sgn,
                                           (nts & kNtTime) != 0);
            }
    }
}

// Waves per SIMD the register allocation is held to (a 64-lane wave has 512
// VGPRs per SIMD lane budget / waves).  Light variants get 4 (<= 128 VGPRs),
// heavy ones (FP64, two flavours, several rhs) 2 (<= 256 VGPRs).  The
// half-precision doublet without twist-on-load is held to 4: left at 2 it
// takes 129 VGPRs (three waves); at 4 it spills one or two and runs 3-4%
// faster (32^3 x 64 M: FP16 229 -> 222 us, BF16 237 -> 227 us).
#ifndef TM_HOP_WAVES_LIGHT
#define TM_HOP_WAVES_LIGHT 4
#endif
#ifndef TM_HOP_WAVES_ND
#define TM_HOP_WAVES_ND 2
#endif
#ifndef TM_HOP_WAVES_ND_HALF
#define TM_HOP_WAVES_ND_HALF 4
#endif
template <int P, int NF, int NR, bool CLV = false, bool TWL = false>
constexpr int hop_waves()
{
    constexpr int NFT = flavours_per_thread<NF>();
    // FP64 clover epilogues (two 6x6 blocks per chirality) get a wave less
    if constexpr (CLV && P == TM_FP64) return NFT == 2 ? 1 : 2;
    if constexpr ((P == TM_FP16 || P == TM_BF16) && NFT == 2 && NR == 1 && !TWL) return TM_HOP_WAVES_ND_HALF;
    return (P == TM_FP64 && NFT * NR == 1) ? 3
           : (P != TM_FP64 && NFT == 2 && NR == 1) ? TM_HOP_WAVES_ND
           : (P == TM_FP64 || NFT * NR > 1) ? 2 : TM_HOP_WAVES_LIGHT;
}

// Keeps the compiler from hoisting the loads of all eight hops ahead of the
// arithmetic, which needs far more registers than the occupancy target
// allows: the accumulators are pinned to registers at this point and no
// memory access moves across it.
template <typename T, int NR, int NFT>
__device__ __forceinline__ void dir_fence(cx<T> (&acc)[NR][NFT][12])
{
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int f = 0; f < NFT; f++)
#pragma unroll
            for (int k = 0; k < 12; k++)
                __asm__ volatile("" : "+v"(acc[r][f][k].re), "+v"(acc[r][f][k].im)::"memory");
}
// Fence granularity: 1 after each direction pair (forward + backward hop),
// 2 after every hop (register-heavy variants: FP64, two flavours, several
// rhs), 0 none.  TM_FENCE_MODE overrides it at build time.
template <int P, int NF, int NR>
constexpr int fence_mode()
{
#ifdef TM_FENCE_MODE
    return TM_FENCE_MODE;
#else
    return (P == TM_FP64 || flavours_per_thread<NF>() * NR > 1) ? 2 : 1;
#endif
}
#define TM_DIR_FENCE()                                   \
    do {                                                 \
        if (fence_mode<P, NF, NR>() != 0) dir_fence(acc); \
    } while (0)
#define TM_HOP_FENCE()                                   \
    do {                                                 \
        if (fence_mode<P, NF, NR>() == 2) dir_fence(acc); \
    } while (0)

// Epilogue of one output site for the thread's rhs: the twist / xpay of
// tm_epilogue, the store, and the squared norm of the result for the
// reduction (added to nrm).
template <int P, int NF, int NR, bool CLV>
__device__ __forceinline__ void hop_epilogue(cx<typename Prec<P>::real> (&acc)[NR][flavours_per_thread<NF>()][12],
                                             const HopProblem &pb, int epi, uint32_t cb, int r0, int fl,
                                             double (&nrm)[NR], int nts)
{
    using real = typename Prec<P>::real;
    // the xpay operand and the output, non-temporally where nts asks
    auto load_x = [&](cx<real> *X, uint32_t vec) {
        if (nts & kNtX)
            SpinorIO<P>::template load<0, 12, true>(X, pb.x, pb.vh, vec, cb);
        else
            SpinorIO<P>::template load<0, 12, false>(X, pb.x, pb.vh, vec, cb);
    };
    auto store_out = [&](const cx<real> *A, uint32_t vec) {
        if (nts & kNtOut)
            SpinorIO<P>::template store<true>(pb.out, pb.vh, vec, cb, A);
        else
            SpinorIO<P>::template store<false>(pb.out, pb.vh, vec, cb, A);
    };
    // CG residual update (the solver's last hop of A p): the output holds r
    // and becomes r - alpha A, so A p itself is never stored
    auto update_out = [&](cx<real> *A, uint32_t vec, int rhs) {
        const real al = (real)pb.upd[rhs].alpha;
        cx<real> Rv[12];
        if (nts & kNtOut)
            SpinorIO<P>::template load<0, 12, true>(Rv, pb.out, pb.vh, vec, cb);
        else
            SpinorIO<P>::template load<0, 12, false>(Rv, pb.out, pb.vh, vec, cb);
#pragma unroll
        for (int k = 0; k < 12; k++) A[k] = Rv[k] - al * A[k];
    };
    const real kk = (real)pb.k;
    const uint32_t vh = pb.vh;
    constexpr bool SPLIT = nd_split<NF>();
    constexpr int NFT = flavours_per_thread<NF>();
    if constexpr (SPLIT) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<real> (&A)[12] = acc[r][0];
            cx<real> T[12];
            if (epi == TM_EPI_TWINV || epi == TM_EPI_X_PLUS_K_TWINV_D) {
                twist_split(T, A, pb.tw, true, fl);
#pragma unroll
                for (int k = 0; k < 12; k++) A[k] = T[k];
            }
            if (epi >= TM_EPI_RX_PLUS_KD) {
                cx<real> X[12];
                load_x(X, (uint32_t)((r0 + r) * NF + fl));
                if (epi == TM_EPI_RX_PLUS_KD) {
                    twist_split(T, X, pb.tw, false, fl);
#pragma unroll
                    for (int k = 0; k < 12; k++) X[k] = T[k];
                }
#pragma unroll
                for (int k = 0; k < 12; k++) A[k] = X[k] + kk * A[k];
                if (epi == TM_EPI_TWINV_X_PLUS_KD) {
                    twist_split(T, A, pb.tw, true, fl);
#pragma unroll
                    for (int k = 0; k < 12; k++) A[k] = T[k];
                }
            }
            if (pb.upd) update_out(A, (uint32_t)((r0 + r) * NF + fl), r0 + r);
            store_out(A, (uint32_t)((r0 + r) * NF + fl));
            if (pb.red.op != FIN_NONE) {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < 12; k++)
                    s += (double)A[k].re * A[k].re + (double)A[k].im * A[k].im;
                nrm[r] += s;
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<real> (&A)[NFT][12] = acc[r];
            auto twist = [&](cx<real> (&v)[NF][12], bool inverse) {
                if constexpr (CLV) {
                    if constexpr (P == TM_FP64 || P == TM_FP32)
                        apply_clover<P, NF>(v, pb.clov, vh, cb, pb.tw, inverse);
                } else {
                    apply_twist<real, NF>(v, pb.tw, inverse);
                }
            };
            if (epi == TM_EPI_TWINV || epi == TM_EPI_X_PLUS_K_TWINV_D) twist(A, true);
            if (epi >= TM_EPI_RX_PLUS_KD) {
                cx<real> X[NF][12];
#pragma unroll
                for (int f = 0; f < NF; f++)
                    load_x(X[f], (uint32_t)((r0 + r) * NF + f));
                if (epi == TM_EPI_RX_PLUS_KD) twist(X, false);
#pragma unroll
                for (int f = 0; f < NF; f++)
#pragma unroll
                    for (int k = 0; k < 12; k++) A[f][k] = X[f][k] + kk * A[f][k];
                if (epi == TM_EPI_TWINV_X_PLUS_KD) twist(A, true);
            }
#pragma unroll
            for (int f = 0; f < NF; f++) {
                if (pb.upd) update_out(A[f], (uint32_t)((r0 + r) * NF + f), r0 + r);
                store_out(A[f], (uint32_t)((r0 + r) * NF + f));
                if (pb.red.op != FIN_NONE) {
                    double s = 0.0;
#pragma unroll
                    for (int k = 0; k < 12; k++)
                        s += (double)A[f][k].re * A[f][k].re + (double)A[f][k].im * A[f][k].im;
                    nrm[r] += s;
                }
            }
        }
    }
}

// Site (checkerboard index) of position j of the processing order: j itself
// (lexicographic), or with z-chunking (pb.zc > 0) the lattice cut into slabs
// of ts time slices (one XCD's share of the blocks), inside a slab bricks of
// zc consecutive z-planes of one time slice, all ts slices of a brick column
// before the next column, so the two time neighbours of a site are read a
// few planes apart (while they can still be in L2).
__device__ __forceinline__ uint32_t site_of(const HopProblem &pb, uint32_t j)
{
    if (pb.zc <= 0) return j;
    const uint32_t pl = (uint32_t)(pb.X[0] >> 1) * (uint32_t)pb.X[1];   // sites of an (x, y) plane
    const uint32_t brick = (uint32_t)pb.zc * pl;
    const uint32_t column = (uint32_t)pb.ts * brick;                   // ts bricks, one per slice
    const uint32_t slab = column * (uint32_t)(pb.X[2] / pb.zc);
    const uint32_t so = j / slab, r1 = j - so * slab;
    const uint32_t ch = r1 / column, r2 = r1 - ch * column;
    const uint32_t ti = r2 / brick, r = r2 - ti * brick;
    return ((so * (uint32_t)pb.ts + ti) * (uint32_t)pb.X[2] + ch * (uint32_t)pb.zc) * pl + r;
}

// CLV: twisted clover, the epilogue's twist is the per-site R(x) (clover
// blocks of the output parity); twist-on-load is not combined with it.
// LDSS: the input spinors of the block's sites and of one y-row either side
// are staged in LDS (FP32, one flavour, one rhs, lexicographic site order);
// x and y neighbours are then read from there.
template <int P, int NF, int NR, bool DAG, bool TWL, int RECON, bool LNT, int BS, bool CLV = false,
          bool LDSS = false>
__global__ void __launch_bounds__(BS, (hop_waves<P, NF, NR, CLV, TWL>())) hop_kernel(const HopBatch B)
{
    using real = typename Prec<P>::real;
    static_assert(!CLV || (!TWL && NR == 1 && !nd_split<NF>() && (P == TM_FP64 || P == TM_FP32)),
                  "clover epilogues: FP64 / FP32, one rhs per thread, no twist-on-load");
    __shared__ double red_sh[BS / 64];
    if (B.gate && *B.gate == 0) return;   // gated launch not needed this iteration

    const int lb = B.xcd_remap ? xcd_logical_block(blockIdx.x, B.total_blocks) : (int)blockIdx.x;
    int pi = 0;
    for (int i = 1; i < B.nprob; i++)
        if (lb >= B.p[i].blk_start) pi = i;
    const HopProblem &pb = B.p[pi];

    constexpr bool SPLIT = nd_split<NF>();
    constexpr int NFT = flavours_per_thread<NF>();
    constexpr int SPB = SPLIT ? BS / 2 : BS;          // sites per block
    const int lbl = lb - pb.blk_start;
    const int sb = lbl / pb.ngrp;
    const int grp = lbl - sb * pb.ngrp;
    const int r0 = grp * NR;
    const int fl = SPLIT ? (int)(threadIdx.x & 1) : 0;  // this lane's flavour (split doublet)
    // j: the site in processing order (site_of)
    const uint32_t j = (uint32_t)sb * SPB + (SPLIT ? threadIdx.x >> 1 : threadIdx.x);
    const uint32_t vh = pb.vh;
    const bool valid = j < vh;
    uint32_t cb = j;
    [[maybe_unused]] uint32_t st_lo = 0, st_span = 0;
    [[maybe_unused]] extern __shared__ float4 st_lds[];
    if constexpr (LDSS) {
        // every thread takes part in staging (lexicographic order: the block's
        // sites are the contiguous range [sb * BS, sb * BS + BS)) of the
        // block's rhs (one rhs per thread and one flavour: vector r0)
        const uint32_t row = (uint32_t)(pb.X[0] >> 1);
        const uint32_t b0 = (uint32_t)sb * BS;
        st_lo = b0 > row ? b0 - row : 0;
        const uint32_t hi = min(vh, b0 + BS + row);
        st_span = hi > st_lo ? hi - st_lo : 0;
        const uint32_t span_max = BS + 2 * row;
        for (uint32_t k = 0; k < 6; k++) {
            const float4 *src = (const float4 *)((const char *)pb.in.data + ((size_t)r0 * 6 + k) * vh * 16);
            for (uint32_t o = threadIdx.x; o < span_max; o += BS)
                if (o < st_span) st_lds[k * st_span + o] = src[st_lo + o];
        }
        __syncthreads();
    }
    if (valid) cb = site_of(pb, j);

    double nrm[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) nrm[r] = 0.0;

    if (valid) {
        const int Lx = pb.X[0], Ly = pb.X[1], Lz = pb.X[2], Lt = pb.X[3];
        const int xh_n = Lx >> 1;
        const int xh = (int)(cb % xh_n);
        int rest = (int)(cb / xh_n);
        const int y = rest % Ly;
        rest /= Ly;
        const int z = rest % Lz;
        const int t = rest / Lz;
        const int par = pb.out_parity;
        const int x = 2 * xh + ((y + z + t + par) & 1);
        const uint32_t base = cb - xh;
        const uint32_t sy = xh_n, sz = (uint32_t)xh_n * Ly, st = (uint32_t)xh_n * Ly * Lz;
        const int npar = 1 - par;

        cx<real> acc[NR][NFT][12];
#pragma unroll
        for (int r = 0; r < NR; r++)
#pragma unroll
            for (int f = 0; f < NFT; f++)
#pragma unroll
                for (int k = 0; k < 12; k++) acc[r][f][k] = mk((real)0, (real)0);

        const real one = (real)1;
        // x direction
        {
            const int xp = (x + 1 == Lx) ? 0 : x + 1;
            const int xm = (x == 0) ? Lx - 1 : x - 1;
            const uint32_t nf_ = base + (xp >> 1), nb_ = base + (xm >> 1);
            hop_direction<P, NF, NR, DAG, TWL, RECON, LNT, 0, true, LDSS>(acc, pb, nf_, cb, par, r0, one, fl, st_lds, st_lo, st_span);
            TM_HOP_FENCE();
            hop_direction<P, NF, NR, DAG, TWL, RECON, LNT, 0, false, LDSS>(acc, pb, nb_, nb_, npar, r0, one, fl, st_lds, st_lo, st_span);
            TM_DIR_FENCE();
        }
        // y direction
        {
            const uint32_t nf_ = (y == Ly - 1) ? cb - (uint32_t)(Ly - 1) * sy : cb + sy;
            const uint32_t nb_ = (y == 0) ? cb + (uint32_t)(Ly - 1) * sy : cb - sy;
            hop_direction<P, NF, NR, DAG, TWL, RECON, LNT, 1, true, LDSS>(acc, pb, nf_, cb, par, r0, one, fl, st_lds, st_lo, st_span);
            TM_HOP_FENCE();
            hop_direction<P, NF, NR, DAG, TWL, RECON, LNT, 1, false, LDSS>(acc, pb, nb_, nb_, npar, r0, one, fl, st_lds, st_lo, st_span);
            TM_DIR_FENCE();
        }
        // z direction
        {
            const uint32_t nf_ = (z == Lz - 1) ? cb - (uint32_t)(Lz - 1) * sz : cb + sz;
            const uint32_t nb_ = (z == 0) ? cb + (uint32_t)(Lz - 1) * sz : cb - sz;
            hop_direction<P, NF, NR, DAG, TWL, RECON, LNT, 2, true, LDSS>(acc, pb, nf_, cb, par, r0, one, fl, st_lds, st_lo, st_span);
            TM_HOP_FENCE();
            hop_direction<P, NF, NR, DAG, TWL, RECON, LNT, 2, false, LDSS>(acc, pb, nb_, nb_, npar, r0, one, fl, st_lds, st_lo, st_span);
            TM_DIR_FENCE();
        }
        // t direction (boundary factor on hops across t = Lt-1 <-> 0)
        {
            const uint32_t nf_ = (t == Lt - 1) ? cb - (uint32_t)(Lt - 1) * st : cb + st;
            const uint32_t nb_ = (t == 0) ? cb + (uint32_t)(Lt - 1) * st : cb - st;
            const real sf = (t == Lt - 1) ? (real)pb.tsign : one;
            const real sbk = (t == 0) ? (real)pb.tsign : one;
            hop_direction<P, NF, NR, DAG, TWL, RECON, LNT, 3, true, LDSS>(acc, pb, nf_, cb, par, r0, sf, fl, st_lds, st_lo, st_span, B.nt_streams);
            TM_HOP_FENCE();
            hop_direction<P, NF, NR, DAG, TWL, RECON, LNT, 3, false, LDSS>(acc, pb, nb_, nb_, npar, r0, sbk, fl, st_lds, st_lo, st_span, B.nt_streams);
            TM_DIR_FENCE();
        }

        hop_epilogue<P, NF, NR, CLV>(acc, pb, B.epi, cb, r0, fl, nrm, B.nt_streams);
    }

    if (pb.red.op != FIN_NONE) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const double s = block_sum<BS>(nrm[r], red_sh);
            if (threadIdx.x == 0) pb.red.partials[(long)(r0 + r) * pb.nsb + sb] = s;
        }
    }
}

// Host-side dispatch over the compile-time variants built for precision P.

// attr != null: report the variant's attributes instead of launching it
#define TM_HOP_RUN(KERNEL)                                                                        \
    do {                                                                                          \
        if (attr) return hipFuncGetAttributes(attr, reinterpret_cast<const void *>(&KERNEL));     \
        hipLaunchKernelGGL((KERNEL), dim3(B.total_blocks), dim3(bs), lds, st, B);                  \
        return hipGetLastError();                                                                 \
    } while (0)

#define TM_HOP_CASE(P, NF, NR, DAG, TWL, RECON, LNT, BS)                                          \
    if (!clv && !ldss && nf == NF && nr == NR && dagger == DAG && twl == TWL && recon == RECON &&  \
        lnt == LNT && bs == BS) {                                                                   \
        TM_HOP_RUN((hop_kernel<P, NF, NR, DAG, TWL, RECON, LNT, BS>));                             \
    }

// twisted-clover epilogues (FP64 / FP32, one rhs per thread, no twist-on-load)
#define TM_HOP_CASE_CLV(P, NF, DAG, RECON, LNT, BS)                                                 \
    if (clv && nf == NF && nr == 1 && dagger == DAG && twl == 0 && recon == RECON && lnt == LNT &&  \
        bs == BS) {                                                                                 \
        TM_HOP_RUN((hop_kernel<P, NF, 1, DAG, false, RECON, LNT, BS, true>));                       \
    }
// LDS-staged x / y neighbours (FP32, one flavour, one rhs, 12-real links)
#define TM_HOP_CASE_LDSS(P, DAG, LNT, BS)                                                          \
    if (ldss && !clv && nf == 1 && nr == 1 && dagger == DAG && twl == 0 && recon == 12 &&          \
        lnt == LNT && bs == BS) {                                                                   \
        TM_HOP_RUN((hop_kernel<P, 1, 1, DAG, false, 12, LNT, BS, false, true>));                    \
    }
#define TM_HOP_CASES_LDSS(P, BS)                                               \
    TM_HOP_CASE_LDSS(P, 0, true, BS) TM_HOP_CASE_LDSS(P, 1, true, BS)          \
    TM_HOP_CASE_LDSS(P, 0, false, BS) TM_HOP_CASE_LDSS(P, 1, false, BS)

#define TM_HOP_CASES_CLV(P, NF, RECON, BS)               \
    TM_HOP_CASE_CLV(P, NF, 0, RECON, true, BS)           \
    TM_HOP_CASE_CLV(P, NF, 1, RECON, true, BS)           \
    TM_HOP_CASE_CLV(P, NF, 0, RECON, false, BS)          \
    TM_HOP_CASE_CLV(P, NF, 1, RECON, false, BS)

// both daggers, both link-load policies
#define TM_HOP_CASES(P, NF, NR, RECON, BS)          \
    TM_HOP_CASE(P, NF, NR, 0, 0, RECON, true, BS)  \
    TM_HOP_CASE(P, NF, NR, 1, 0, RECON, true, BS)  \
    TM_HOP_CASE(P, NF, NR, 0, 0, RECON, false, BS) \
    TM_HOP_CASE(P, NF, NR, 1, 0, RECON, false, BS)

// twist-on-load variants: non-temporal links, 256 threads
#define TM_HOP_CASES_TWL(P, NF, NR, RECON)          \
    TM_HOP_CASE(P, NF, NR, 0, 1, RECON, true, 256) \
    TM_HOP_CASE(P, NF, NR, 1, 1, RECON, true, 256)

#define TM_HOP_DEFINE(P)                                                                       \
    template <>                                                                                \
    hipError_t launch_hop_prec<P>(const HopBatch &B, int nf, int nr, int dagger, int twl,      \
                                  int recon, int bs, bool lnt, unsigned lds, bool clv,         \
                                  bool ldss, hipStream_t st, hipFuncAttributes *attr)          \
    {                                                                                          \
        if constexpr (P == TM_FP32) {                                                          \
            TM_HOP_CASES_LDSS(P, 256)                                                          \
            TM_HOP_CASES_LDSS(P, 64)                                                           \
        }                                                                                      \
        if constexpr (P == TM_FP64 || P == TM_FP32) {                                          \
            TM_HOP_CASES_CLV(P, 1, 12, 256)                                                    \
            TM_HOP_CASES_CLV(P, 1, 12, 64)                                                     \
            TM_HOP_CASES_CLV(P, 1, 18, 256)                                                    \
            if constexpr (!kNdSplit) {                                                         \
                TM_HOP_CASES_CLV(P, 2, 12, 256)                                                \
                TM_HOP_CASES_CLV(P, 2, 12, 64)                                                 \
                TM_HOP_CASES_CLV(P, 2, 18, 256)                                                \
            }                                                                                  \
        }                                                                                      \
        TM_HOP_CASES(P, 1, 1, 12, 256)                                                         \
        TM_HOP_CASES(P, 1, 1, 12, 128)                                                         \
        TM_HOP_CASES(P, 1, 1, 12, 64)                                                          \
        TM_HOP_CASES(P, 1, 1, 18, 256)                                                         \
        TM_HOP_CASES(P, 2, 1, 12, 256)                                                         \
        TM_HOP_CASES(P, 2, 1, 12, 128)                                                         \
        TM_HOP_CASES(P, 2, 1, 12, 64)                                                          \
        TM_HOP_CASES(P, 2, 1, 18, 256)                                                         \
        TM_HOP_CASES(P, 1, 1, 8, 256)                                                          \
        TM_HOP_CASES(P, 1, 1, 8, 128)                                                          \
        TM_HOP_CASES(P, 1, 1, 8, 64)                                                           \
        TM_HOP_CASES(P, 2, 1, 8, 256)                                                          \
        TM_HOP_CASES(P, 2, 1, 8, 128)                                                          \
        TM_HOP_CASES(P, 2, 1, 8, 64)                                                           \
        if constexpr (P != TM_FP64) {                                                          \
            TM_HOP_CASES(P, 1, 4, 12, 256)                                                     \
            TM_HOP_CASES(P, 1, 4, 12, 128)                                                     \
            TM_HOP_CASES_TWL(P, 1, 4, 12)                                                      \
        }                                                                                      \
        TM_HOP_CASES(P, 1, 2, 12, 256)                                                         \
        TM_HOP_CASES(P, 1, 2, 12, 128)                                                         \
        TM_HOP_CASES_TWL(P, 1, 2, 12)                                                          \
        TM_HOP_CASES_TWL(P, 1, 1, 12)                                                          \
        TM_HOP_CASES_TWL(P, 1, 1, 18)                                                          \
        TM_HOP_CASES_TWL(P, 2, 1, 12)                                                          \
        TM_HOP_CASES_TWL(P, 2, 1, 18)                                                          \
        TM_HOP_CASES_TWL(P, 1, 1, 8)                                                           \
        TM_HOP_CASES_TWL(P, 2, 1, 8)                                                           \
        return hipErrorInvalidConfiguration;                                                   \
    }

}  // namespace twm
