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

// FP64 / FP32 fields are flat arrays of 16-byte chunks, [rhs][flavour][row][cb]
// with rows of vh chunks, so element-wise operations stream them chunk by
// chunk: a unit is U complex numbers (U = 1 when every operand is FP64, else
// 2 = one FP32 chunk = two FP64 chunks of rows 2j, 2j+1), u counts the units
// of one rhs and cb = u mod vh.
template <int P, int U>
__device__ __forceinline__ void unit_load(cx<double> (&v)[U], const SpinorPtr &s, size_t rbase, size_t u,
                                          uint32_t cb, uint32_t vh)
{
    if constexpr (P == TM_FP64) {
        const double2 *d = (const double2 *)s.data + rbase;
        if constexpr (U == 1) {
            const double2 a = d[u];
            v[0] = mk(a.x, a.y);
        } else {
            const size_t i0 = 2 * u - cb;
            const double2 a = d[i0], b = d[i0 + vh];
            v[0] = mk(a.x, a.y);
            v[1] = mk(b.x, b.y);
        }
    } else {
        const float4 a = ((const float4 *)s.data)[rbase + u];
        v[0] = mk((double)a.x, (double)a.y);
        v[1] = mk((double)a.z, (double)a.w);
    }
}

template <int P, int U>
__device__ __forceinline__ void unit_store(const SpinorPtr &s, size_t rbase, size_t u, uint32_t cb,
                                           uint32_t vh, const cx<double> (&v)[U])
{
    if constexpr (P == TM_FP64) {
        double2 *d = (double2 *)s.data + rbase;
        if constexpr (U == 1) {
            d[u] = make_double2(v[0].re, v[0].im);
        } else {
            const size_t i0 = 2 * u - cb;
            d[i0] = make_double2(v[0].re, v[0].im);
            d[i0 + vh] = make_double2(v[1].re, v[1].im);
        }
    } else {
        ((float4 *)s.data)[rbase + u] =
            make_float4((float)v[0].re, (float)v[0].im, (float)v[1].re, (float)v[1].im);
    }
}

template <int U>
__device__ __forceinline__ double unit_nrm2(const cx<double> (&v)[U])
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < U; k++) s += v[k].re * v[k].re + v[k].im * v[k].im;
    return s;
}

#ifndef TM_BLAS_UNROLL
#define TM_BLAS_UNROLL 4
#endif

// the chunk-streaming path serves operations whose operands are all FP64 / FP32
template <int PA, int PB>
constexpr bool blas_flat()
{
    return (PA == TM_FP64 || PA == TM_FP32) && (PB == TM_FP64 || PB == TM_FP32);
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
    if constexpr (OP == OP_CG_UPDATE || OP == OP_XPAY_X || OP == OP_ACCUM_STEP)
        alpha = pb.red.cg[rhs].alpha;
    if constexpr (OP == OP_XPAY || OP == OP_XPAY_X) beta = pb.red.cg[rhs].beta;

    if constexpr (blas_flat<PA, PB>()) {
        constexpr int U = (PA == TM_FP64 && PB == TM_FP64) ? 1 : 2;
        const size_t units = (size_t)nf * (12 / U) * vh;
        // chunk offsets of this rhs in each operand (FP64: 12 rows, FP32: 6)
        const size_t ra = (size_t)rhs * nf * (PA == TM_FP64 ? 12 : 6) * vh;
        const size_t rb = (size_t)rhs * nf * (PB == TM_FP64 ? 12 : 6) * vh;
        // TM_BLAS_UNROLL units per thread and pass, their loads issued together
        constexpr int UN = TM_BLAS_UNROLL;
        const size_t stride = (size_t)pb.nblk * BS * UN;
        for (size_t u0 = (size_t)blk * BS * UN + threadIdx.x; u0 < units; u0 += stride) {
            cx<double> a0[UN][U], a1[UN][U], a2[UN][U], a3[UN][U];
            uint32_t cbs[UN];
            bool ok[UN];
#pragma unroll
            for (int q = 0; q < UN; q++) {
                const size_t u = u0 + (size_t)q * BS;
                ok[q] = u < units;
                cbs[q] = (uint32_t)(u % vh);
                if (!ok[q]) continue;
                if constexpr (OP == OP_CG_UPDATE) {
                    unit_load<PA, U>(a0[q], pb.v[0], ra, u, cbs[q], vh);
                    unit_load<PB, U>(a1[q], pb.v[1], rb, u, cbs[q], vh);
                    unit_load<PB, U>(a2[q], pb.v[2], rb, u, cbs[q], vh);
                    unit_load<PB, U>(a3[q], pb.v[3], rb, u, cbs[q], vh);
                } else if constexpr (OP == OP_XPAY_X) {
                    unit_load<PA, U>(a0[q], pb.v[0], ra, u, cbs[q], vh);
                    unit_load<PB, U>(a1[q], pb.v[1], rb, u, cbs[q], vh);
                    unit_load<PB, U>(a2[q], pb.v[2], rb, u, cbs[q], vh);
                } else if constexpr (OP == OP_XPAY) {
                    unit_load<PB, U>(a0[q], pb.v[0], rb, u, cbs[q], vh);
                    unit_load<PB, U>(a1[q], pb.v[1], rb, u, cbs[q], vh);
                } else if constexpr (OP == OP_RESIDUAL) {
                    unit_load<PA, U>(a0[q], pb.v[0], ra, u, cbs[q], vh);
                    if (pb.v[1].data) unit_load<PA, U>(a1[q], pb.v[1], ra, u, cbs[q], vh);
                } else if constexpr (OP == OP_CONVERT || OP == OP_NORM2) {
                    unit_load<PA, U>(a0[q], pb.v[0], ra, u, cbs[q], vh);
                } else if constexpr (OP == OP_ACCUM_ZERO) {
                    unit_load<PA, U>(a0[q], pb.v[0], ra, u, cbs[q], vh);
                    unit_load<PB, U>(a1[q], pb.v[1], rb, u, cbs[q], vh);
                } else if constexpr (OP == OP_ACCUM_STEP) {  // PB = FP32 here: x_lo and p alike
                    unit_load<PA, U>(a0[q], pb.v[0], ra, u, cbs[q], vh);
                    unit_load<PB, U>(a1[q], pb.v[1], rb, u, cbs[q], vh);
                    unit_load<PB, U>(a2[q], pb.v[2], rb, u, cbs[q], vh);
                } else if constexpr (OP == OP_DOT) {
                    unit_load<PA, U>(a0[q], pb.v[0], ra, u, cbs[q], vh);
                    unit_load<PA, U>(a1[q], pb.v[1], ra, u, cbs[q], vh);
                }
            }
#pragma unroll
            for (int q = 0; q < UN; q++) {
                if (!ok[q]) continue;
                const size_t u = u0 + (size_t)q * BS;
                const uint32_t cb = cbs[q];
                if constexpr (OP == OP_CG_UPDATE) {          // x += alpha p, r -= alpha Ap, |r|^2
#pragma unroll
                    for (int k = 0; k < U; k++) {
                        a0[q][k] = a0[q][k] + alpha * a1[q][k];
                        a2[q][k] = a2[q][k] - alpha * a3[q][k];
                    }
                    unit_store<PA, U>(pb.v[0], ra, u, cb, vh, a0[q]);
                    unit_store<PB, U>(pb.v[2], rb, u, cb, vh, a2[q]);
                    acc0 += unit_nrm2<U>(a2[q]);
                } else if constexpr (OP == OP_XPAY_X) {      // x += alpha p, then p = r + beta p
#pragma unroll
                    for (int k = 0; k < U; k++) {
                        a0[q][k] = a0[q][k] + alpha * a1[q][k];
                        a1[q][k] = a2[q][k] + beta * a1[q][k];
                    }
                    unit_store<PA, U>(pb.v[0], ra, u, cb, vh, a0[q]);
                    unit_store<PB, U>(pb.v[1], rb, u, cb, vh, a1[q]);
                } else if constexpr (OP == OP_XPAY) {        // p = r + beta p
#pragma unroll
                    for (int k = 0; k < U; k++) a1[q][k] = a0[q][k] + beta * a1[q][k];
                    unit_store<PB, U>(pb.v[1], rb, u, cb, vh, a1[q]);
                } else if constexpr (OP == OP_RESIDUAL) {    // r = c - y, |r|^2
                    if (pb.v[1].data) {
#pragma unroll
                        for (int k = 0; k < U; k++) a0[q][k] = a0[q][k] - a1[q][k];
                    }
                    acc0 += unit_nrm2<U>(a0[q]);
                    unit_store<PB, U>(pb.v[2], rb, u, cb, vh, a0[q]);
                    if (pb.v[3].data) unit_store<PB, U>(pb.v[3], rb, u, cb, vh, a0[q]);
                } else if constexpr (OP == OP_CONVERT) {
#pragma unroll
                    for (int k = 0; k < U; k++) a0[q][k] = B.scale * a0[q][k];
                    unit_store<PB, U>(pb.v[1], rb, u, cb, vh, a0[q]);
                } else if constexpr (OP == OP_ACCUM_ZERO) {  // y += x, x = 0
#pragma unroll
                    for (int k = 0; k < U; k++) {
                        a0[q][k] = a0[q][k] + a1[q][k];
                        a1[q][k] = mk(0.0, 0.0);
                    }
                    unit_store<PA, U>(pb.v[0], ra, u, cb, vh, a0[q]);
                    unit_store<PB, U>(pb.v[1], rb, u, cb, vh, a1[q]);
                } else if constexpr (OP == OP_ACCUM_STEP) {  // y += x + alpha p, x = 0
#pragma unroll
                    for (int k = 0; k < U; k++) {
                        a0[q][k] = a0[q][k] + (a1[q][k] + alpha * a2[q][k]);
                        a1[q][k] = mk(0.0, 0.0);
                    }
                    unit_store<PA, U>(pb.v[0], ra, u, cb, vh, a0[q]);
                    unit_store<PB, U>(pb.v[1], rb, u, cb, vh, a1[q]);
                } else if constexpr (OP == OP_NORM2) {
                    acc0 += unit_nrm2<U>(a0[q]);
                } else if constexpr (OP == OP_DOT) {
#pragma unroll
                    for (int k = 0; k < U; k++) {
                        const cx<double> t = cjmul(a0[q][k], a1[q][k]);
                        acc0 += t.re;
                        acc1 += t.im;
                    }
                }
            }
        }
    } else
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
            } else if constexpr (OP == OP_XPAY_X) {
                cx<double> x[12], p[12], r[12];
                load_d<PA>(x, pb.v[0], vh, vec, cb);
                load_d<PB>(p, pb.v[1], vh, vec, cb);
                load_d<PB>(r, pb.v[2], vh, vec, cb);
#pragma unroll
                for (int k = 0; k < 12; k++) {
                    x[k] = x[k] + alpha * p[k];
                    p[k] = r[k] + beta * p[k];
                }
                store_d<PA>(pb.v[0], vh, vec, cb, x);
                store_d<PB>(pb.v[1], vh, vec, cb, p);
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
#pragma unroll
                for (int k = 0; k < 12; k++) a[k] = B.scale * a[k];
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
            } else if constexpr (OP == OP_ACCUM_STEP) {
                // x_lo is FP32 whatever the direction's format PB
                cx<double> y[12], x[12], p[12];
                load_d<PA>(y, pb.v[0], vh, vec, cb);
                load_d<TM_FP32>(x, pb.v[1], vh, vec, cb);
                load_d<PB>(p, pb.v[2], vh, vec, cb);
#pragma unroll
                for (int k = 0; k < 12; k++) {
                    y[k] = y[k] + (x[k] + alpha * p[k]);
                    x[k] = mk(0.0, 0.0);
                }
                store_d<PA>(pb.v[0], vh, vec, cb, y);
                store_d<TM_FP32>(pb.v[1], vh, vec, cb, x);
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

// Final reduction of partials[v][0..nblk) for v in [v0, v1) by one block,
// then the finishing operation.  Fixed summation order: each thread keeps
// four running sums over strides of 4 BS (its loads independent, so they are
// in flight together), then the block sum.
template <int BS>
__device__ void finish_reduce(const Reduce &rd, int v0, int v1, int nblk, double *sh)
{
    for (int v = v0; v < v1; v++) {
        const double *part = rd.partials + (long)v * nblk;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int i = threadIdx.x;
        for (; i + 3 * BS < nblk; i += 4 * BS) {
            s0 += part[i];
            s1 += part[i + BS];
            s2 += part[i + 2 * BS];
            s3 += part[i + 3 * BS];
        }
        for (; i < nblk; i += BS) s0 += part[i];
        double s = block_sum<BS>((s0 + s1) + (s2 + s3), sh);
        if (threadIdx.x == 0) {
            if (rd.op == FIN_STORE) {
                rd.out[v] = s;
            } else if (rd.op == FIN_ALPHA) {
                CGScalars &c = rd.cg[v];
                c.pap = s;
                c.alpha = (c.active && s > 0.0) ? c.rr / s : 0.0;
            } else if (rd.op == FIN_BETA) {
                CGScalars &c = rd.cg[v];
                if (c.active) {
                    c.beta = (c.rr > 0.0) ? s / c.rr : 0.0;
                    c.rr_old = c.rr;
                    c.rr = s;
                    c.maxrr = fmax(c.maxrr, s);
                    c.hist[c.niter % kHistory] = s;
                    c.niter++;
                    if (s <= c.stop2) {
                        c.active = 0;
                        c.pending = 1;
                    }
                } else {
                    c.beta = 0.0;
                }
            } else if (rd.op == FIN_RELIABLE) {
                // the residual was replaced by the true one (reliable update):
                // continue the recurrence with beta = |r_true|^2 / |r_prev|^2
                CGScalars &c = rd.cg[v];
                // progress of the true residual from one replacement to the
                // next, for rhs that were iterating (a converged rhs shares
                // the replacements of the others without moving)
                if (c.active || c.pending) {
                    if (c.rr_upd > 0.0 && s >= c.stall_f2 * c.rr_upd)
                        c.stall++;
                    else
                        c.stall = 0;
                    c.rr_upd = s;
                }
                c.beta = (c.rr_old > 0.0) ? s / c.rr_old : 0.0;
                // the step alpha p of this iteration is in x already (taken
                // before the replacement); a later pass of it adds nothing
                c.alpha = 0.0;
                c.rr = s;
                c.maxrr = s;
                c.active = (s > c.stop2) ? 1 : 0;
                c.pending = 0;
            } else if (rd.op == FIN_STORE_RR) {
                // a fresh residual: restart the recurrence for this rhs
                CGScalars &c = rd.cg[v];
                c.rr = s;
                c.rr_old = s;
                c.maxrr = s;
                c.beta = 0.0;
                c.active = (s > c.stop2) ? 1 : 0;
                c.pending = 0;
                c.rr_upd = s;
                c.stall = 0;
            }
        }
    }
}

// One block per (problem, vector): add the vector's partials in a fixed
// order, then finish.  A hop launch leaves one partial per site block (16384
// for 2^20 sites in blocks of 64), so the block is wide.
constexpr int kFinishThreads = 1024;
__global__ void __launch_bounds__(kFinishThreads) finish_kernel(const FinishBatch F)
{
    __shared__ double sh[kFinishThreads / 64];
    if (F.gate && *F.gate == 0) return;
    const Reduce &rd = F.r[blockIdx.x];
    const int v = (int)blockIdx.y;
    if (v >= rd.nvec) return;
    finish_reduce<kFinishThreads>(rd, v, v + 1, rd.nblk, sh);
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

__global__ void run_kernel(const RunArgs R)
{
    if (threadIdx.x != 0) return;
    int run = 0;
    for (int i = 0; i < R.nprob; i++)
        for (int r = 0; r < R.nrhs[i]; r++) {
            const CGScalars &c = R.cg[i][r];
            if (c.active || (R.with_pending && c.pending)) run = 1;
        }
    if (*R.iters >= R.maxiter) run = 0;
    *R.run = run;
    if (run) *R.iters += 1;
}

hipError_t launch_run(const RunArgs &R, hipStream_t st)
{
    hipLaunchKernelGGL(run_kernel, dim3(1), dim3(64), 0, st, R);
    return hipGetLastError();
}

hipError_t launch_decide(const DecideArgs &D, hipStream_t st)
{
    hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(64), 0, st, D);
    return hipGetLastError();
}

hipError_t launch_finish(const FinishBatch &F, hipStream_t st)
{
    int nv = 1;
    for (int i = 0; i < F.nprob; i++) nv = std::max(nv, F.r[i].nvec);
    hipLaunchKernelGGL(finish_kernel, dim3(F.nprob, nv), dim3(kFinishThreads), 0, st, F);
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
    // with the residual updated by the hop: the step fused with the new direction
    TM_BL(OP_XPAY_X, TM_FP64, TM_FP64)
    TM_BL(OP_XPAY_X, TM_FP32, TM_FP32)
    TM_BL(OP_XPAY_X, TM_FP32, TM_FP16)
    TM_BL(OP_XPAY_X, TM_FP32, TM_BF16)
    TM_BL_SAME(OP_XPAY)
    TM_BL_ALL_B(OP_RESIDUAL, TM_FP64)
    TM_BL_ALL_B(OP_CONVERT, TM_FP64)
    TM_BL_ALL_B(OP_CONVERT, TM_FP32)
    TM_BL_ALL_B(OP_CONVERT, TM_FP16)
    TM_BL_ALL_B(OP_CONVERT, TM_BF16)
    TM_BL(OP_ACCUM_ZERO, TM_FP64, TM_FP32)
    TM_BL(OP_ACCUM_ZERO, TM_FP64, TM_FP64)
    TM_BL(OP_ACCUM_STEP, TM_FP64, TM_FP32)
    TM_BL(OP_ACCUM_STEP, TM_FP64, TM_FP16)
    TM_BL(OP_ACCUM_STEP, TM_FP64, TM_BF16)
    TM_BL_SAME(OP_NORM2)
    TM_BL_SAME(OP_DOT)
    return hipErrorInvalidConfiguration;
}

}  // namespace twm
