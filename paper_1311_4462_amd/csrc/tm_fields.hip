// Field conversion kernels: canonical complex128 full-lattice arrays <->
// native parity-split, chunked, per-precision layouts; the standalone twist.
#include "tm_fields.h"

namespace twm {

// cb (checkerboard index of a site of parity par) -> lexicographic index
__device__ __forceinline__ long lex_of(uint32_t cb, int par, const int *X)
{
    const int xh_n = X[0] >> 1;
    const int xh = cb % xh_n;
    int rest = cb / xh_n;
    const int y = rest % X[1];
    rest /= X[1];
    const int z = rest % X[2];
    const int t = rest / X[2];
    const int x = 2 * xh + ((y + z + t + par) & 1);
    return 2L * (cb - xh) + x;
}

struct Dims {
    int X[4];
};

// ---------------------------------------------------------------- gauge

// 8-real links need |a2|^2 + |a3|^2 > 0 (row 0 not of the form (a1, 0, 0));
// links below this bound are flagged and the upload is refused.
constexpr double kRecon8MinN = 1e-10;

template <int P, int RECON>
__global__ void gauge_pack_kernel(void *dst0, void *dst1, const double2 *src, Dims d, uint32_t vh,
                                  int *bad)
{
    const uint32_t cb = blockIdx.x * blockDim.x + threadIdx.x;
    const int mu = blockIdx.y;
    const int par = blockIdx.z;
    if (cb >= vh) return;
    const long V = 2L * vh;
    const long s = lex_of(cb, par, d.X);
    const double2 *u = src + ((long)mu * V + s) * 9;
    double2 e[9];
    for (int k = 0; k < 9; k++) e[k] = u[k];
    if constexpr (RECON == 8) {
        const double n = e[1].x * e[1].x + e[1].y * e[1].y + e[2].x * e[2].x + e[2].y * e[2].y;
        if (!(n >= kRecon8MinN)) *bad = 1;
    }
    LinkIO<P, RECON>::store(par ? dst1 : dst0, vh, mu, cb, e);
}

hipError_t gauge_pack(int prec, int recon, void *dst0, void *dst1, const void *src, const int *X,
                      uint32_t vh, int *bad, hipStream_t st)
{
    Dims d{{X[0], X[1], X[2], X[3]}};
    dim3 grid((vh + 255) / 256, 4, 2);
    const double2 *s = (const double2 *)src;
#define TM_GP(P, R)                                                                           \
    if (prec == P && recon == R) {                                                            \
        hipLaunchKernelGGL((gauge_pack_kernel<P, R>), grid, dim3(256), 0, st, dst0, dst1, s, d, vh, bad); \
        return hipGetLastError();                                                             \
    }
    TM_GP(TM_FP64, 12) TM_GP(TM_FP64, 18) TM_GP(TM_FP64, 8) TM_GP(TM_FP32, 12) TM_GP(TM_FP32, 18)
    TM_GP(TM_FP32, 8) TM_GP(TM_FP16, 12) TM_GP(TM_FP16, 18) TM_GP(TM_FP16, 8) TM_GP(TM_BF16, 12)
    TM_GP(TM_BF16, 18) TM_GP(TM_BF16, 8)
#undef TM_GP
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- spinor

// Chiral <-> internal spin basis: the map S = H (x) 1_2, H = [[1, 1], [1, -1]]
// / sqrt 2 on the (upper, lower) spin pairs, is real, orthogonal and its own
// inverse, so one routine serves both directions (components k = 3 spin + c).
__device__ inline void swap_basis(double2 (&w)[12])
{
    const double r = 0.70710678118654752440;
#pragma unroll
    for (int k = 0; k < 6; k++) {
        const double2 a = w[k], b = w[k + 6];
        w[k] = make_double2(r * (a.x + b.x), r * (a.y + b.y));
        w[k + 6] = make_double2(r * (a.x - b.x), r * (a.y - b.y));
    }
}

template <int P>
__global__ void spinor_pack_kernel(SpinorPtr dst, const double2 *src, Dims d, uint32_t vh,
                                   int par, int nf, int basis)
{
    using real = typename Prec<P>::real;
    const uint32_t cb = blockIdx.x * blockDim.x + threadIdx.x;
    const int vec = blockIdx.y;          // rhs * nf + f
    if (cb >= vh) return;
    const int rhs = vec / nf, f = vec % nf;
    const long V = 2L * vh;
    const long s = lex_of(cb, par, d.X);
    const double2 *p = src + (((long)rhs * V + s) * nf + f) * 12;
    double2 w[12];
    for (int k = 0; k < 12; k++) w[k] = p[k];
    if (basis == TM_BASIS_CHIRAL) swap_basis(w);
    cx<real> v[12];
    for (int k = 0; k < 12; k++) v[k] = mk((real)w[k].x, (real)w[k].y);
    SpinorIO<P>::store(dst, vh, vec, cb, v);
}

template <int P>
__global__ void spinor_unpack_kernel(double2 *dst, SpinorPtr src, Dims d, uint32_t vh, int par,
                                     int nf, int basis)
{
    using real = typename Prec<P>::real;
    const uint32_t cb = blockIdx.x * blockDim.x + threadIdx.x;
    const int vec = blockIdx.y;
    if (cb >= vh) return;
    const int rhs = vec / nf, f = vec % nf;
    const long V = 2L * vh;
    const long s = lex_of(cb, par, d.X);
    cx<real> v[12];
    SpinorIO<P>::template load<0, 12>(v, src, vh, vec, cb);
    double2 w[12];
    for (int k = 0; k < 12; k++) w[k] = make_double2((double)v[k].re, (double)v[k].im);
    if (basis == TM_BASIS_CHIRAL) swap_basis(w);
    double2 *p = dst + (((long)rhs * V + s) * nf + f) * 12;
    for (int k = 0; k < 12; k++) p[k] = w[k];
}

hipError_t spinor_pack(int prec, SpinorPtr dst, const void *src, const int *X, uint32_t vh, int par,
                       int nf, int nrhs, int basis, hipStream_t st)
{
    Dims d{{X[0], X[1], X[2], X[3]}};
    dim3 grid((vh + 255) / 256, nf * nrhs);
    const double2 *s = (const double2 *)src;
    switch (prec) {
    case TM_FP64: hipLaunchKernelGGL(spinor_pack_kernel<TM_FP64>, grid, dim3(256), 0, st, dst, s, d, vh, par, nf, basis); break;
    case TM_FP32: hipLaunchKernelGGL(spinor_pack_kernel<TM_FP32>, grid, dim3(256), 0, st, dst, s, d, vh, par, nf, basis); break;
    case TM_FP16: hipLaunchKernelGGL(spinor_pack_kernel<TM_FP16>, grid, dim3(256), 0, st, dst, s, d, vh, par, nf, basis); break;
    case TM_BF16: hipLaunchKernelGGL(spinor_pack_kernel<TM_BF16>, grid, dim3(256), 0, st, dst, s, d, vh, par, nf, basis); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t spinor_unpack(int prec, void *dst, SpinorPtr src, const int *X, uint32_t vh, int par,
                         int nf, int nrhs, int basis, hipStream_t st)
{
    Dims d{{X[0], X[1], X[2], X[3]}};
    dim3 grid((vh + 255) / 256, nf * nrhs);
    double2 *o = (double2 *)dst;
    switch (prec) {
    case TM_FP64: hipLaunchKernelGGL(spinor_unpack_kernel<TM_FP64>, grid, dim3(256), 0, st, o, src, d, vh, par, nf, basis); break;
    case TM_FP32: hipLaunchKernelGGL(spinor_unpack_kernel<TM_FP32>, grid, dim3(256), 0, st, o, src, d, vh, par, nf, basis); break;
    case TM_FP16: hipLaunchKernelGGL(spinor_unpack_kernel<TM_FP16>, grid, dim3(256), 0, st, o, src, d, vh, par, nf, basis); break;
    case TM_BF16: hipLaunchKernelGGL(spinor_unpack_kernel<TM_BF16>, grid, dim3(256), 0, st, o, src, d, vh, par, nf, basis); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- twist

template <int P, int NF>
__global__ void twist_kernel(SpinorPtr out, SpinorPtr in, uint32_t vh, Twist tw, int inverse,
                             const void *clov, const int *gate)
{
    using real = typename Prec<P>::real;
    if (gate && *gate == 0) return;   // gated launch not needed this iteration
    const uint32_t cb = blockIdx.x * blockDim.x + threadIdx.x;
    const int rhs = blockIdx.y;
    if (cb >= vh) return;
    cx<real> v[NF][12];
    for (int f = 0; f < NF; f++) SpinorIO<P>::template load<0, 12>(v[f], in, vh, rhs * NF + f, cb);
    if constexpr (P == TM_FP64 || P == TM_FP32) {
        if (clov)
            apply_clover<P, NF>(v, clov, vh, cb, tw, inverse != 0);
        else
            apply_twist<real, NF>(v, tw, inverse != 0);
    } else {
        apply_twist<real, NF>(v, tw, inverse != 0);
    }
    for (int f = 0; f < NF; f++) SpinorIO<P>::store(out, vh, rhs * NF + f, cb, v[f]);
}

hipError_t twist_apply(int prec, int nf, SpinorPtr out, SpinorPtr in, uint32_t vh, int nrhs,
                       Twist tw, int inverse, hipStream_t st, const void *clov, const int *gate)
{
    dim3 grid((vh + 255) / 256, nrhs);
#define TM_TW(P, NF)                                                                            \
    if (prec == P && nf == NF) {                                                                \
        hipLaunchKernelGGL((twist_kernel<P, NF>), grid, dim3(256), 0, st, out, in, vh, tw, inverse, \
                           clov, gate);                                                         \
        return hipGetLastError();                                                               \
    }
    TM_TW(TM_FP64, 1) TM_TW(TM_FP64, 2) TM_TW(TM_FP32, 1) TM_TW(TM_FP32, 2)
    TM_TW(TM_FP16, 1) TM_TW(TM_FP16, 2) TM_TW(TM_BF16, 1) TM_TW(TM_BF16, 2)
#undef TM_TW
    return hipErrorInvalidValue;
}

}  // namespace twm
