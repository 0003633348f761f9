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

template <int P, int RECON>
__global__ void gauge_pack_kernel(void *dst0, void *dst1, const double2 *src, Dims d, uint32_t vh)
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
    LinkIO<P, RECON>::store(par ? dst1 : dst0, vh, mu, cb, e);
}

hipError_t gauge_pack(int prec, int recon, void *dst0, void *dst1, const void *src, const int *X,
                      uint32_t vh, hipStream_t st)
{
    Dims d{{X[0], X[1], X[2], X[3]}};
    dim3 grid((vh + 255) / 256, 4, 2);
    const double2 *s = (const double2 *)src;
#define TM_GP(P, R)                                                                           \
    if (prec == P && recon == R) {                                                            \
        hipLaunchKernelGGL((gauge_pack_kernel<P, R>), grid, dim3(256), 0, st, dst0, dst1, s, d, vh); \
        return hipGetLastError();                                                             \
    }
    TM_GP(TM_FP64, 12) TM_GP(TM_FP64, 18) TM_GP(TM_FP32, 12) TM_GP(TM_FP32, 18)
    TM_GP(TM_FP16, 12) TM_GP(TM_FP16, 18) TM_GP(TM_BF16, 12) TM_GP(TM_BF16, 18)
#undef TM_GP
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- spinor

template <int P>
__global__ void spinor_pack_kernel(SpinorPtr dst, const double2 *src, Dims d, uint32_t vh,
                                   int par, int nf)
{
    using real = typename Prec<P>::real;
    const uint32_t cb = blockIdx.x * blockDim.x + threadIdx.x;
    const int vec = blockIdx.y;          // rhs * nf + f
    if (cb >= vh) return;
    const int rhs = vec / nf, f = vec % nf;
    const long V = 2L * vh;
    const long s = lex_of(cb, par, d.X);
    const double2 *p = src + (((long)rhs * V + s) * nf + f) * 12;
    cx<real> v[12];
    for (int k = 0; k < 12; k++) v[k] = mk((real)p[k].x, (real)p[k].y);
    SpinorIO<P>::store(dst, vh, vec, cb, v);
}

template <int P>
__global__ void spinor_unpack_kernel(double2 *dst, SpinorPtr src, Dims d, uint32_t vh, int par,
                                     int nf)
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
    double2 *p = dst + (((long)rhs * V + s) * nf + f) * 12;
    for (int k = 0; k < 12; k++) p[k] = make_double2((double)v[k].re, (double)v[k].im);
}

hipError_t spinor_pack(int prec, SpinorPtr dst, const void *src, const int *X, uint32_t vh, int par,
                       int nf, int nrhs, hipStream_t st)
{
    Dims d{{X[0], X[1], X[2], X[3]}};
    dim3 grid((vh + 255) / 256, nf * nrhs);
    const double2 *s = (const double2 *)src;
    switch (prec) {
    case TM_FP64: hipLaunchKernelGGL(spinor_pack_kernel<TM_FP64>, grid, dim3(256), 0, st, dst, s, d, vh, par, nf); break;
    case TM_FP32: hipLaunchKernelGGL(spinor_pack_kernel<TM_FP32>, grid, dim3(256), 0, st, dst, s, d, vh, par, nf); break;
    case TM_FP16: hipLaunchKernelGGL(spinor_pack_kernel<TM_FP16>, grid, dim3(256), 0, st, dst, s, d, vh, par, nf); break;
    case TM_BF16: hipLaunchKernelGGL(spinor_pack_kernel<TM_BF16>, grid, dim3(256), 0, st, dst, s, d, vh, par, nf); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t spinor_unpack(int prec, void *dst, SpinorPtr src, const int *X, uint32_t vh, int par,
                         int nf, int nrhs, hipStream_t st)
{
    Dims d{{X[0], X[1], X[2], X[3]}};
    dim3 grid((vh + 255) / 256, nf * nrhs);
    double2 *o = (double2 *)dst;
    switch (prec) {
    case TM_FP64: hipLaunchKernelGGL(spinor_unpack_kernel<TM_FP64>, grid, dim3(256), 0, st, o, src, d, vh, par, nf); break;
    case TM_FP32: hipLaunchKernelGGL(spinor_unpack_kernel<TM_FP32>, grid, dim3(256), 0, st, o, src, d, vh, par, nf); break;
    case TM_FP16: hipLaunchKernelGGL(spinor_unpack_kernel<TM_FP16>, grid, dim3(256), 0, st, o, src, d, vh, par, nf); break;
    case TM_BF16: hipLaunchKernelGGL(spinor_unpack_kernel<TM_BF16>, grid, dim3(256), 0, st, o, src, d, vh, par, nf); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- twist

template <int P, int NF>
__global__ void twist_kernel(SpinorPtr out, SpinorPtr in, uint32_t vh, Twist tw, int inverse)
{
    using real = typename Prec<P>::real;
    const uint32_t cb = blockIdx.x * blockDim.x + threadIdx.x;
    const int rhs = blockIdx.y;
    if (cb >= vh) return;
    cx<real> v[NF][12];
    for (int f = 0; f < NF; f++) SpinorIO<P>::template load<0, 12>(v[f], in, vh, rhs * NF + f, cb);
    apply_twist<real, NF>(v, tw, inverse != 0);
    for (int f = 0; f < NF; f++) SpinorIO<P>::store(out, vh, rhs * NF + f, cb, v[f]);
}

hipError_t twist_apply(int prec, int nf, SpinorPtr out, SpinorPtr in, uint32_t vh, int nrhs,
                       Twist tw, int inverse, hipStream_t st)
{
    dim3 grid((vh + 255) / 256, nrhs);
#define TM_TW(P, NF)                                                                            \
    if (prec == P && nf == NF) {                                                                \
        hipLaunchKernelGGL((twist_kernel<P, NF>), grid, dim3(256), 0, st, out, in, vh, tw, inverse); \
        return hipGetLastError();                                                               \
    }
    TM_TW(TM_FP64, 1) TM_TW(TM_FP64, 2) TM_TW(TM_FP32, 1) TM_TW(TM_FP32, 2)
    TM_TW(TM_FP16, 1) TM_TW(TM_FP16, 2) TM_TW(TM_BF16, 1) TM_TW(TM_BF16, 2)
#undef TM_TW
    return hipErrorInvalidValue;
}

}  // namespace twm
