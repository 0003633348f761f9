// Solver BLAS on native fields: fused CG updates, conversions and FP64
// reductions (wave shuffles, then LDS, then a deterministic last-block sum).
// One launch covers up to kMaxProblems problems and all their rhs; block b of
// a problem handles rhs b / nblk and grid-strides over the sites.
#include "tm_fields.h"

namespace twm {

template <int P>
__device__ __forceinline__ void load_d(cx<double> (&v)[12], const SpinorPtr &s, uint32_t vh,
                                       uint32_t vec, uint32_t cb)
{
    using real = typename Prec<P>::real;
    cx<real> t[12];
    SpinorIO<P>::template load<0, 12>(t, s, vh, vec, cb);
#pragma unroll
    for (int k = 0; k < 12; k++) v[k] = mk((double)t[k].re, (double)t[k].im);
}

template <int P>
__device__ __forceinline__ void store_d(const SpinorPtr &s, uint32_t vh, uint32_t vec, uint32_t cb,
                                        const cx<double> (&v)[12])
{
    using real = typename Prec<P>::real;
    cx<real> t[12];
#pragma unroll
    for (int k = 0; k < 12; k++) t[k] = mk((real)v[k].re, (real)v[k].im);
    SpinorIO<P>::store(s, vh, vec, cb, t);
}

__device__ __forceinline__ double nrm2_12(const cx<double> (&v)[12])
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 12; k++) s += v[k].re * v[k].re + v[k].im * v[k].im;
    return s;
}

template <int OP, int PA, int PB, int BS>
__global__ void __launch_bounds__(BS) blas_kernel(const BlasBatch B)
{
    __shared__ double red_sh[BS / 64];
    if (B.gate && *B.gate == 0) return;   // gated launch not needed this iteration

    const int lb = blockIdx.x;
    int pi = 0;
    for (int i = 1; i < B.nprob; i++)
        if (lb >= B.p[i].blk_start) pi = i;
    const BlasProblem &pb = B.p[pi];
    const int local = lb - pb.blk_start;
    const int rhs = local / pb.nblk;
    const int blk = local - rhs * pb.nblk;
    const uint32_t vh = pb.vh;
    const int nf = B.nf;

    double acc0 = 0.0, acc1 = 0.0;
    double alpha = 0.0, beta = 0.0;
    if constexpr (OP == OP_CG_UPDATE) alpha = pb.red.cg[rhs].alpha;
    if constexpr (OP == OP_XPAY) beta = pb.red.cg[rhs].beta;

    for (uint32_t cb = blk * BS + threadIdx.x; cb < vh; cb += pb.nblk * BS) {
        for (int f = 0; f < nf; f++) {
            const uint32_t vec = rhs * nf + f;
            if constexpr (OP == OP_CG_UPDATE) {
                cx<double> x[12], p[12], r[12], ap[12];
                load_d<PA>(x, pb.v[0], vh, vec, cb);
                load_d<PB>(p, pb.v[1], vh, vec, cb);
                load_d<PB>(r, pb.v[2], vh, vec, cb);
                load_d<PB>(ap, pb.v[3], vh, vec, cb);
#pragma unroll
                for (int k = 0; k < 12; k++) {
                    x[k] = x[k] + alpha * p[k];
                    r[k] = r[k] - alpha * ap[k];
                }
                store_d<PA>(pb.v[0], vh, vec, cb, x);
                store_d<PB>(pb.v[2], vh, vec, cb, r);
                acc0 += nrm2_12(r);
            } else if constexpr (OP == OP_XPAY) {
                cx<double> r[12], p[12];
                load_d<PB>(r, pb.v[0], vh, vec, cb);
                load_d<PB>(p, pb.v[1], vh, vec, cb);
#pragma unroll
                for (int k = 0; k < 12; k++) p[k] = r[k] + beta * p[k];
                store_d<PB>(pb.v[1], vh, vec, cb, p);
            } else if constexpr (OP == OP_RESIDUAL) {
                cx<double> c[12], y[12];
                load_d<PA>(c, pb.v[0], vh, vec, cb);
                if (pb.v[1].data) {          // y absent: r = c (zero initial guess)
                    load_d<PA>(y, pb.v[1], vh, vec, cb);
#pragma unroll
                    for (int k = 0; k < 12; k++) c[k] = c[k] - y[k];
                }
                // the norm is that of the FP64 residual, before any rounding
                acc0 += nrm2_12(c);
                store_d<PB>(pb.v[2], vh, vec, cb, c);
                if (pb.v[3].data) store_d<PB>(pb.v[3], vh, vec, cb, c);
            } else if constexpr (OP == OP_CONVERT) {
                cx<double> a[12];
                load_d<PA>(a, pb.v[0], vh, vec, cb);
                store_d<PB>(pb.v[1], vh, vec, cb, a);
            } else if constexpr (OP == OP_ACCUM_ZERO) {
                cx<double> y[12], x[12];
                load_d<PA>(y, pb.v[0], vh, vec, cb);
                load_d<PB>(x, pb.v[1], vh, vec, cb);
#pragma unroll
                for (int k = 0; k < 12; k++) {
                    y[k] = y[k] + x[k];
                    x[k] = mk(0.0, 0.0);
                }
                store_d<PA>(pb.v[0], vh, vec, cb, y);
                store_d<PB>(pb.v[1], vh, vec, cb, x);
            } else if constexpr (OP == OP_NORM2) {
                cx<double> a[12];
                load_d<PA>(a, pb.v[0], vh, vec, cb);
                acc0 += nrm2_12(a);
            } else if constexpr (OP == OP_DOT) {
                cx<double> a[12], b[12];
                load_d<PA>(a, pb.v[0], vh, vec, cb);
                load_d<PA>(b, pb.v[1], vh, vec, cb);
#pragma unroll
                for (int k = 0; k < 12; k++) {
                    const cx<double> t = cjmul(a[k], b[k]);
                    acc0 += t.re;
                    acc1 += t.im;
                }
            }
        }
    }

    if constexpr (OP == OP_CG_UPDATE || OP == OP_RESIDUAL || OP == OP_NORM2 || OP == OP_DOT) {
        if (pb.red.op != FIN_NONE) {
            if constexpr (OP == OP_DOT) {
                const double s0 = block_sum<BS>(acc0, red_sh);
                const double s1 = block_sum<BS>(acc1, red_sh);
                if (threadIdx.x == 0) {
                    pb.red.partials[(long)(2 * rhs) * pb.nblk + blk] = s0;
                    pb.red.partials[(long)(2 * rhs + 1) * pb.nblk + blk] = s1;
                }
            } else {
                const double s0 = block_sum<BS>(acc0, red_sh);
                if (threadIdx.x == 0) pb.red.partials[(long)rhs * pb.nblk + blk] = s0;
            }
        }
    }
}

// One block per problem: add the partials in a fixed order, then finish.
__global__ void __launch_bounds__(256) finish_kernel(const FinishBatch F)
{
    __shared__ double sh[4];
    if (F.gate && *F.gate == 0) return;
    const Reduce &rd = F.r[blockIdx.x];
    finish_reduce<256>(rd, rd.nvec, rd.nblk, sh);
}

__global__ void decide_kernel(const DecideArgs D)
{
    if (threadIdx.x != 0) return;
    int need = 0;
    for (int i = 0; i < D.nprob; i++)
        for (int r = 0; r < D.nrhs[i]; r++) {
            const CGScalars &c = D.cg[i][r];
            if (c.pending || (c.active && c.rr < D.delta2 * c.maxrr)) need = 1;
        }
    *D.gate = need;
    if (need) *D.count += 1;
}

hipError_t launch_decide(const DecideArgs &D, hipStream_t st)
{
    hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(64), 0, st, D);
    return hipGetLastError();
}

hipError_t launch_finish(const FinishBatch &F, hipStream_t st)
{
    hipLaunchKernelGGL(finish_kernel, dim3(F.nprob), dim3(256), 0, st, F);
    return hipGetLastError();
}

#define TM_BL(OP, PA, PB)                                                                   \
    if (op == OP && pa == PA && pb == PB) {                                                 \
        hipLaunchKernelGGL((blas_kernel<OP, PA, PB, 256>), dim3(B.total_blocks), dim3(256), \
                           0, st, B);                                                       \
        return hipGetLastError();                                                           \
    }
#define TM_BL_ALL_B(OP, PA) TM_BL(OP, PA, TM_FP64) TM_BL(OP, PA, TM_FP32) TM_BL(OP, PA, TM_FP16) TM_BL(OP, PA, TM_BF16)
#define TM_BL_SAME(OP) TM_BL(OP, TM_FP64, TM_FP64) TM_BL(OP, TM_FP32, TM_FP32) TM_BL(OP, TM_FP16, TM_FP16) TM_BL(OP, TM_BF16, TM_BF16)

hipError_t launch_blas(int op, int pa, int pb, const BlasBatch &B, hipStream_t st)
{
    // CG update: FP64 solution with FP64 vectors (plain CG); FP32 partial
    // solution with low-precision vectors (mixed CG).
    TM_BL(OP_CG_UPDATE, TM_FP64, TM_FP64)
    TM_BL(OP_CG_UPDATE, TM_FP32, TM_FP32)
    TM_BL(OP_CG_UPDATE, TM_FP32, TM_FP16)
    TM_BL(OP_CG_UPDATE, TM_FP32, TM_BF16)
    TM_BL_SAME(OP_XPAY)
    TM_BL_ALL_B(OP_RESIDUAL, TM_FP64)
    TM_BL_ALL_B(OP_CONVERT, TM_FP64)
    TM_BL_ALL_B(OP_CONVERT, TM_FP32)
    TM_BL_ALL_B(OP_CONVERT, TM_FP16)
    TM_BL_ALL_B(OP_CONVERT, TM_BF16)
    TM_BL(OP_ACCUM_ZERO, TM_FP64, TM_FP32)
    TM_BL(OP_ACCUM_ZERO, TM_FP64, TM_FP64)
    TM_BL_SAME(OP_NORM2)
    TM_BL_SAME(OP_DOT)
    return hipErrorInvalidConfiguration;
}

}  // namespace twm
