// Host-callable launchers of the HIP kernels (internal to the library).
#pragma once

#include "tm_impl.h"

namespace twm {

hipError_t gauge_pack(int prec, int recon, void *dst0, void *dst1, const void *src, const int *X,
                      uint32_t vh, int *bad, hipStream_t st);
hipError_t spinor_pack(int prec, SpinorPtr dst, const void *src, const int *X, uint32_t vh, int par,
                       int nf, int nrhs, int basis, hipStream_t st);
hipError_t spinor_unpack(int prec, void *dst, SpinorPtr src, const int *X, uint32_t vh, int par,
                         int nf, int nrhs, int basis, hipStream_t st);
// gate (nullable): the launch does nothing when *gate == 0
hipError_t twist_apply(int prec, int nf, SpinorPtr out, SpinorPtr in, uint32_t vh, int nrhs,
                       Twist tw, int inverse, hipStream_t st, const void *clov = nullptr,
                       const int *gate = nullptr);

// Device address of the allocation-free call's scratch array on `device`
// (the current device), resolved once per device and kept.
hipError_t noalloc_scratch(int device, void **ptr);

// Launch the hop variant selected by the arguments, or, when attr is not
// null, only fill attr with its function attributes (static LDS, registers).
template <int P>
hipError_t launch_hop_prec(const HopBatch &B, int nf, int nr, int dagger, int twl, int recon,
                           int bs, bool lnt, unsigned lds, bool clv, bool ldss, hipStream_t st,
                           hipFuncAttributes *attr = nullptr);
// clover blocks of both parities (FP64 and / or FP32 destinations, nullable)
hipError_t clover_build(void *const *d64, void *const *d32, const void *links, const int *X, uint32_t vh,
                        double kc, double shift, int *bad, hipStream_t st);

// ---------------------------------------------------------------- BLAS

enum BlasOp {
    OP_CG_UPDATE = 0,   // v0 (PA) += alpha v1; v2 -= alpha v3; |v2|^2        (v1..v3: PB)
    OP_XPAY = 1,        // v1 = v0 + beta v1                                  (PB)
    OP_RESIDUAL = 2,    // v2 (PB) = v0 - v1 (PA; v1 null: 0); v3 (PB, optional) = v2; |v2|^2
    OP_CONVERT = 3,     // v1 (PB) = scale v0 (PA)
    OP_ACCUM_ZERO = 4,  // v0 (PA) += v1 (PB); v1 = 0
    OP_NORM2 = 5,       // |v0|^2 (PA)
    OP_DOT = 6,         // <v0, v1> (PA), re / im
    OP_XPAY_X = 8,      // v0 (PA) += alpha v1; v1 = v2 + beta v1  (v1, v2: PB): step and new direction
    OP_ACCUM_STEP = 9   // v0 (PA) += v1 (FP32) + alpha v2 (PB); v1 = 0: a reliable update's solution
};

struct BlasProblem {
    uint32_t vh;
    int nrhs;
    int blk_start;      // first block of this problem
    int nblk;           // blocks per rhs
    SpinorPtr v[4];
    Reduce red;
};

struct BlasBatch {
    int nprob;
    int total_blocks;
    int nf;
    double scale;        // OP_CONVERT's factor (1: a plain conversion)
    const int *gate;     // nullable: skip the launch when *gate == 0
    BlasProblem p[kMaxProblems];
};

hipError_t launch_blas(int op, int pa, int pb, const BlasBatch &B, hipStream_t st);
hipError_t launch_finish(const FinishBatch &F, hipStream_t st);
hipError_t launch_decide(const DecideArgs &D, hipStream_t st);
hipError_t launch_run(const RunArgs &R, hipStream_t st);

// force
hipError_t force_launch(int prec, int nf, int force_prec, void *F, void *G, const void *gauge0,
                        const void *gauge1, int recon, SpinorPtr A[2], SpinorPtr Bv[2],
                        const int *X, uint32_t vh, double tsign, double coeff, int accumulate,
                        double kappa, hipStream_t st);

}  // namespace twm
