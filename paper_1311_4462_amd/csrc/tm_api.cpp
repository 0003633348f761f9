// Host runtime behind include/tm.h: contexts, packed gauge fields, argument
// validation, operator composition (Eqs. 2.2 - 2.4) and the CG drivers.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "tm_fields.h"

using namespace twm;

namespace {
// Named ranges of host-side work for profilers (roctx; next to no cost
// without a profiler attached): the solver stages, one open at a time.
struct Phase {
    bool open = false;
    void enter(const char *name)
    {
        if (open) roctxRangePop();
        roctxRangePushA(name);
        open = true;
    }
    ~Phase()
    {
        if (open) roctxRangePop();
    }
};
}  // namespace

// ------------------------------------------------------------------ objects

struct Buf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct tm_ctx {
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;   // used for graph capture when stream is the null stream
    int device = 0;
    std::string last_error;
    std::map<std::string, Buf> ws;
    double *host_scratch = nullptr;   // pinned, for reduction results
    size_t host_scratch_bytes = 0;
    int tuning = 0;
    std::map<std::string, int> tuned;  // kernel key -> block size
    int force_bs = 0;                  // TM_HOP_BS: fixed block size (0: tuned / default)
    int force_lnt = -1;                // TM_LINK_NT: 1 / 0 fixes the link load policy
    int force_zc = -1;                 // TM_HOP_ZC: fixed brick depth of the site order (0: lexicographic)
    int force_wcap = -1;               // TM_HOP_WCAP: fixed cap of resident waves per SIMD (0: none)
    int force_ldss = -1;               // TM_HOP_LDS: 1 / 0 forces the LDS-staged variant where it exists
    int force_nr = 0;                  // TM_HOP_NR: 1, 2 or 4 rhs per thread where instantiated (0: default)
    int force_nt = -1;                 // TM_HOP_NT: non-temporal stream mask of the hop launches (see HopCfg)
    int cg_fuse = 1;                   // TM_CG_FUSE=0: CG residual update as a separate BLAS pass
    int verbose = 0;                   // TM_VERBOSE=1: solver progress on stderr
    const int *gate = nullptr;         // set while enqueuing gated (device-decided) launches
    int xcd_remap = 1;
    unsigned lds_per_cu = 0;           // from the runtime at context creation
    unsigned lds_per_block = 0;
    std::map<std::string, unsigned> static_lds;   // hop variant -> static LDS bytes
    // allocation-free calls (tm_mat_pc_noalloc): this device's scratch array
    // (address resolved at creation), and while such a call runs, the
    // temporaries it takes from there; no workspace may grow then and the
    // tuner (which times launches into extra buffers) does not run
    void *scratch = nullptr;
    hipError_t scratch_err = hipSuccess;
    bool no_alloc = false;
    void *tmp_override[2] = {nullptr, nullptr};   // odd temporary, twist-on-load temporary
};

struct tm_gauge {
    tm_params p{};
    int recon = 12;
    int nf = 1;
    uint32_t vh = 0;
    void *links[4][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
    // twisted clover (csw != 0): A and B blocks per site, FP64 / FP32, per parity
    void *clov[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    bool clover() const { return p.csw != 0.0; }
    const void *clov_of(int prec, int par) const { return prec <= TM_FP32 ? clov[prec][par] : nullptr; }
};

namespace {

int fail(tm_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->last_error = buf;
    }
    return code;
}

#define TM_HIP(ctx, call)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(ctx, TM_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                  \
    } while (0)

#define TM_TRY(expr)          \
    do {                      \
        int rc_ = (expr);     \
        if (rc_ < 0) return rc_; \
    } while (0)

bool valid_prec(int p) { return p >= TM_FP64 && p <= TM_BF16; }

int check_params(tm_ctx *ctx, const tm_params *p)
{
    if (!p) return fail(ctx, TM_ERR_ARG, "null params");
    for (int d = 0; d < 4; d++)
        if (p->dims[d] < 2 || (p->dims[d] & 1))
            return fail(ctx, TM_ERR_DIMS, "extent %d of dimension %d is not even and >= 2",
                        p->dims[d], d);
    const double V = (double)p->dims[0] * p->dims[1] * p->dims[2] * p->dims[3];
    if (V / 2 > 2.0e8) return fail(ctx, TM_ERR_LIMIT, "lattice too large for one device");
    if (p->flavor != TM_TWIST_PLUS && p->flavor != TM_TWIST_MINUS && p->flavor != TM_TWIST_NDEG)
        return fail(ctx, TM_ERR_ARG, "bad twist flavor %d", p->flavor);
    if (!std::isfinite(p->kappa) || !std::isfinite(p->mu) || !std::isfinite(p->epsilon) ||
        !std::isfinite(p->csw))
        return fail(ctx, TM_ERR_ARG, "non-finite operator parameter");
    const double a = 2 * p->kappa * p->mu;
    const double b = p->flavor == TM_TWIST_NDEG ? 2 * p->kappa * p->epsilon : 0.0;
    if (std::fabs(1 + a * a - b * b) < 1e-12)
        return fail(ctx, TM_ERR_SINGULAR, "twist R is singular: 1 + a^2 - b^2 = %g", 1 + a * a - b * b);
    return TM_OK;
}

int nflav(const tm_params &p) { return p.flavor == TM_TWIST_NDEG ? 2 : 1; }
uint32_t half_volume(const tm_params &p)
{
    return (uint32_t)((long)p.dims[0] * p.dims[1] * p.dims[2] * p.dims[3] / 2);
}

Twist make_twist(const tm_params &p, int dagger)
{
    const double a = 2 * p.kappa * p.mu;
    Twist t;
    if (p.flavor == TM_TWIST_NDEG) {
        t.ta = dagger ? -a : a;
        t.b = 2 * p.kappa * p.epsilon;
    } else {
        const double s = (p.flavor == TM_TWIST_PLUS) ? 1.0 : -1.0;
        t.ta = dagger ? -s * a : s * a;
        t.b = 0.0;
    }
    t.c = 1.0 / (1.0 + t.ta * t.ta - t.b * t.b);
    return t;
}

SpinorPtr sptr(const void *p, int prec, uint32_t vh, int nf, int nrhs)
{
    SpinorPtr s;
    s.data = const_cast<void *>(p);
    s.scale = (prec == TM_FP16 || prec == TM_BF16)
                  ? (float *)((char *)const_cast<void *>(p) + chunk_bytes(prec, vh, nf, nrhs))
                  : nullptr;
    return s;
}

void *workspace(tm_ctx *ctx, const std::string &name, size_t bytes, int *rc)
{
    if (ctx->no_alloc) {
        // an allocation-free call may only use a buffer that is already there
        auto it = ctx->ws.find(name);
        if (it != ctx->ws.end() && it->second.ptr && it->second.bytes >= bytes) return it->second.ptr;
        *rc = fail(ctx, TM_ERR_LIMIT, "allocation-free call: workspace %s of %zu bytes not available",
                   name.c_str(), bytes);
        return nullptr;
    }
    Buf &b = ctx->ws[name];
    if (b.bytes >= bytes && b.ptr) return b.ptr;
    if (b.ptr) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    if (hipMalloc(&b.ptr, bytes) != hipSuccess) {
        b.ptr = nullptr;
        *rc = fail(ctx, TM_ERR_NOMEM, "workspace %s: cannot allocate %zu bytes", name.c_str(), bytes);
        return nullptr;
    }
    // counters must start at zero; everything else is written before use
    (void)hipMemsetAsync(b.ptr, 0, bytes, ctx->stream);
    b.bytes = bytes;
    return b.ptr;
}

double *host_scratch(tm_ctx *ctx, size_t n, int *rc)
{
    const size_t bytes = n * sizeof(double);
    if (ctx->host_scratch_bytes >= bytes) return ctx->host_scratch;
    if (ctx->host_scratch) (void)hipHostFree(ctx->host_scratch);
    ctx->host_scratch = nullptr;
    ctx->host_scratch_bytes = 0;
    if (hipHostMalloc((void **)&ctx->host_scratch, bytes, hipHostMallocDefault) != hipSuccess) {
        *rc = fail(ctx, TM_ERR_NOMEM, "pinned host buffer of %zu bytes", bytes);
        return nullptr;
    }
    ctx->host_scratch_bytes = bytes;
    return ctx->host_scratch;
}

// Input-parity temporary of a twist-on-load pass (twisted clover), one per
// problem slot and precision.
void *twl_tmp(tm_ctx *ctx, int slot, const tm_gauge *g, int prec, int nrhs, int *rc)
{
    if (ctx->no_alloc && slot == 0 && ctx->tmp_override[1]) return ctx->tmp_override[1];
    char name[64];
    snprintf(name, sizeof(name), "twl_tmp_%d_%d", slot, prec);
    return workspace(ctx, name, spinor_field_bytes(prec, g->vh, g->nf, nrhs), rc);
}

// Reduction slot i: a partial-sum buffer (stream ordered, so consecutive
// launches can share one slot; a batched launch uses one per problem).
struct RedSlot {
    double *partials;
};

int red_slot(tm_ctx *ctx, int i, size_t npartials, RedSlot *out)
{
    int rc = TM_OK;
    char name[64];
    snprintf(name, sizeof(name), "red_partials_%d", i);
    out->partials = (double *)workspace(ctx, name, std::max<size_t>(npartials, 64) * sizeof(double), &rc);
    if (!out->partials) return rc;
    return TM_OK;
}

// ------------------------------------------------------------------ hop launch

struct HopCall {
    const tm_gauge *g;
    int prec;
    int out_parity;
    int dagger;
    int twl;
    int epi;
    const void *in;
    void *out;
    const void *x;
    double k;
    int nrhs;
    int fin;                 // FinOp for |out|^2 (FIN_NONE: no reduction)
    CGScalars *cg;
    double *red_out;
    int upd = 0;             // CG residual update: out -= alpha (epilogue result), alpha from cg
};

#ifndef TM_FP64_NR
#define TM_FP64_NR 2
#endif
constexpr int kFp64Nr = TM_FP64_NR;

// rhs per thread (one flavour, 12-real links): 4 for the reduced precisions,
// 2 for FP64 (an FP64 site vector for 4 rhs alone needs 192 VGPRs); force
// (1, 2 or 4) overrides where that variant exists.
int choose_nr(int prec, int nf, int nrhs, int recon, int force)
{
    if (nf != 1 || recon != 12) return 1;
    if (force == 1 || force == 2 || (force == 4 && prec != TM_FP64)) return nrhs % force ? 1 : force;
    const int want = (prec == TM_FP64) ? kFp64Nr : 4;
    return nrhs % want ? 1 : want;
}

// Launch configurations instantiated for a hop variant (see TM_HOP_DEFINE):
// block size, and whether links are loaded non-temporally (bypassing the
// caches: best when the working set exceeds the 256 MB last-level cache) or
// ordinarily (they can then stay cache resident across launches).
// wcap > 0 caps the resident waves per SIMD at about wcap by giving each
// block an otherwise unused share of the 160 KiB of LDS of a compute unit:
// fewer waves in flight keep more of the neighbour spinors they share in L2.
struct HopCfg {
    int bs;
    bool lnt;
    int wcap;
    int zc = 0;     // z-planes per brick of the site order (0: lexicographic)
    bool ldss = false;   // x / y neighbours staged in LDS (FP32, one flavour, one rhs)
    int nr = 1;     // right-hand sides per thread
    // streams accessed non-temporally (HopBatch::nt_streams): 1 output
    // stores, 2 xpay operand loads, 4 time-neighbour loads.  Streaming the
    // single-use fields past L2 leaves it to the neighbour spinors that are
    // re-read; where a launch's output is read back soon from the last-level
    // cache (working sets within it) ordinary stores do better.
    int nt = 0;
};
// cache code of a tuned configuration: block size in bits 0-9, the
// non-temporal stream mask in bits 10-12
int cfg_code(const HopCfg &c)
{
    const int l2nr = c.nr == 4 ? 2 : c.nr == 2 ? 1 : 0;
    return c.bs | ((c.nt & 7) << 10) | (c.lnt ? 1 << 16 : 0) | (c.ldss ? 1 << 17 : 0) | (l2nr << 18) |
           (c.wcap << 20) | (c.zc << 24);
}
HopCfg cfg_decode(int code)
{
    HopCfg c{code & 0x3ff, ((code >> 16) & 1) != 0, (code >> 20) & 0xf, (code >> 24) & 0x7f,
             ((code >> 17) & 1) != 0};
    c.nr = 1 << ((code >> 18) & 3);
    c.nt = (code >> 10) & 7;
    return c;
}
// bricks of at most `target` z-planes: the largest divisor of Lz below Lz
int zc_for(int target, int Lz)
{
    for (int d = std::min(target, Lz - 1); d >= 2; d--)
        if (Lz % d == 0) return d;
    return 0;
}
// Resident-block arithmetic of the wave cap assumes LDS footprints that are
// multiples of 2560 bytes: a multiple of every LDS allocation unit of CDNA
// parts (512 and 1280 bytes), so the dispatcher rounds nothing up.
constexpr unsigned kLdsUnit = 2560;
constexpr unsigned kLdsPerCUDefault = 160u << 10;   // gfx950, when the runtime cannot be asked
}  // namespace

// Dynamic LDS of one hop block (see tm_plan_hop_lds in tm.h).
int tm_plan_hop_lds(int block_size, int wave_cap, unsigned staging_bytes, unsigned lds_per_cu,
                    unsigned lds_per_block, unsigned static_lds, unsigned *dyn_bytes)
{
    if (!dyn_bytes || block_size <= 0 || block_size % 64 || wave_cap < 0 || wave_cap > 8 || lds_per_cu == 0 ||
        lds_per_block == 0)
        return TM_ERR_ARG;
    const unsigned long cap = std::min(lds_per_cu, lds_per_block);
    unsigned long want = staging_bytes;
    if (wave_cap > 0) {
        // a compute unit has 4 SIMDs: `blocks` resident blocks of block_size
        // threads give wave_cap waves per SIMD
        const unsigned long blocks = std::max(1, 4 * wave_cap * 64 / block_size);
        const unsigned long f = std::min<unsigned long>(lds_per_cu / blocks, cap) / kLdsUnit * kLdsUnit;
        // the footprint must admit `blocks` blocks and not one more
        if (f <= static_lds || (blocks + 1) * f <= lds_per_cu) return TM_ERR_LIMIT;
        want = std::max(want, f - static_lds);
    }
    if (want + static_lds > cap) return TM_ERR_LIMIT;
    *dyn_bytes = (unsigned)want;
    return TM_OK;
}

namespace {
// LDS of the staged x / y neighbours: six FP32 chunk rows of the block's
// sites and one y-row either side
unsigned hop_staging_bytes(int bs, int row)
{
    return (unsigned)(6 * (bs + 2 * row) * 16);
}
std::vector<HopCfg> cfg_candidates(int prec, int nf, int nr, int twl, int recon, bool clv)
{
    if (twl) return {{256, true, 0}};
    std::vector<int> bss = (recon == 18) ? std::vector<int>{256}
                           : clv ? std::vector<int>{64, 256}
                           : (nr == 1) ? std::vector<int>{64, 128, 256} : std::vector<int>{128, 256};
    std::vector<HopCfg> out;
    for (int b : bss)
        for (int w : {0, 4, 3, 2}) {
            out.push_back({b, true, w});
            out.push_back({b, false, w});
        }
    // LDS-staged x / y neighbours: FP32, one flavour, one rhs, 12-real links
    if (prec == TM_FP32 && nf == 1 && nr == 1 && recon == 12 && !clv)
        for (int b : {64, 256})
            for (int w : {0, 3, 2}) {
                out.push_back({b, true, w, 0, true});
                out.push_back({b, false, w, 0, true});
            }
    return out;
}

// Default when not tuned: 256 threads; ordinary link loads when the launch's
// links and three spinor fields fit well inside the last-level cache.
HopCfg default_cfg(int twl, size_t working_set)
{
    if (twl) return {256, true, 0};
    return {256, working_set > (size_t)200 << 20, 0};
}

std::string tune_key(int prec, int nf, int nr, int dagger, int twl, int epi, int recon, long vh_total,
                     bool clv)
{
    char key[128];
    snprintf(key, sizeof(key), "hop_p%d_f%d_r%d_d%d_t%d_e%d_c%d%s_v%ld", prec, nf, nr, dagger, twl, epi, recon,
             clv ? "w" : "",
             vh_total);
    return key;
}

void save_tune(tm_ctx *ctx, const std::string &key, int bs)
{
    const char *path = getenv("TM_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d\n", key.c_str(), bs);
    fclose(f);
    (void)ctx;
}

void load_tune(tm_ctx *ctx)
{
    const char *path = getenv("TM_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char key[160];
    int bs;
    while (fscanf(f, "%159s %d", key, &bs) == 2) ctx->tuned[key] = bs;
    fclose(f);
}

hipError_t dispatch_hop(const HopBatch &B, int prec, int nf, int nr, int dagger, int twl, int recon,
                        const HopCfg &c, bool clv, unsigned lds, hipStream_t st, hipFuncAttributes *attr = nullptr)
{
    switch (prec) {
    case TM_FP64: return launch_hop_prec<TM_FP64>(B, nf, nr, dagger, twl, recon, c.bs, c.lnt, lds, clv, c.ldss, st, attr);
    case TM_FP32: return launch_hop_prec<TM_FP32>(B, nf, nr, dagger, twl, recon, c.bs, c.lnt, lds, clv, c.ldss, st, attr);
    case TM_FP16: return launch_hop_prec<TM_FP16>(B, nf, nr, dagger, twl, recon, c.bs, c.lnt, lds, clv, c.ldss, st, attr);
    case TM_BF16: return launch_hop_prec<TM_BF16>(B, nf, nr, dagger, twl, recon, c.bs, c.lnt, lds, clv, c.ldss, st, attr);
    }
    return hipErrorInvalidValue;
}

// Dynamic LDS of a hop launch: the staged rows (LDS-staged variant) and the
// wave-cap reservation, planned against the compute unit's LDS (from the
// runtime) and the variant's own static LDS (from its function attributes).
// A request that cannot be met is refused (TM_ERR_LIMIT; quiet: without
// recording an error, for the tuner's candidate filter), never dispatched.
int hop_lds_plan(tm_ctx *ctx, const HopBatch &B, int prec, int nf, int nr, int dagger, int twl, int recon,
                 const HopCfg &c, bool clv, unsigned *lds, bool quiet = false)
{
    unsigned staging = 0;
    if (c.ldss) {
        int row = 0;
        for (int i = 0; i < B.nprob; i++) row = std::max(row, B.p[i].X[0] / 2);
        staging = hop_staging_bytes(c.bs, row);
    }
    *lds = 0;
    if (c.wcap <= 0 && staging == 0) return TM_OK;
    char key[96];
    snprintf(key, sizeof(key), "%d_%d_%d_%d_%d_%d_%d_%d_%d_%d", prec, nf, nr, dagger, twl, recon, c.bs, (int)c.lnt,
             (int)clv, (int)c.ldss);
    unsigned static_lds;
    auto it = ctx->static_lds.find(key);
    if (it != ctx->static_lds.end()) {
        static_lds = it->second;
    } else {
        hipFuncAttributes attr;
        memset(&attr, 0, sizeof(attr));
        const hipError_t e = dispatch_hop(B, prec, nf, nr, dagger, twl, recon, c, clv, 0, nullptr, &attr);
        if (e != hipSuccess)
            return quiet ? TM_ERR_HIP : fail(ctx, TM_ERR_HIP, "hop attributes: %s", hipGetErrorString(e));
        static_lds = (unsigned)attr.sharedSizeBytes;
        ctx->static_lds[key] = static_lds;
    }
    const unsigned cu = ctx->lds_per_cu ? ctx->lds_per_cu : kLdsPerCUDefault;
    const unsigned blk = ctx->lds_per_block ? ctx->lds_per_block : cu;
    const int rc = tm_plan_hop_lds(c.bs, c.wcap, staging, cu, blk, static_lds, lds);
    if (rc != TM_OK && !quiet)
        return fail(ctx, TM_ERR_LIMIT,
                    "hop launch: LDS request beyond the compute unit (block %d, wave cap %d, staging %u B, "
                    "static %u B, %u B per CU, %u B per block)",
                    c.bs, c.wcap, staging, static_lds, cu, blk);
    return rc;
}

// One launch of the fused hop over up to kMaxProblems problems (same
// precision, flavour count, recon, dagger, epilogue and rhs grouping).
int build_hop_batch(tm_ctx *ctx, const HopCall *calls, int n, int nr, int bs, HopBatch *B, int zc = 0,
                    int nt = 0)
{
    const int prec = calls[0].prec, nf = calls[0].g->nf;
    memset(B, 0, sizeof(*B));
    B->nprob = n;
    B->gate = ctx->gate;
    B->epi = calls[0].epi;
    B->xcd_remap = ctx->xcd_remap;
    B->nt_streams = nt;
    int blocks = 0;
    for (int i = 0; i < n; i++) {
        const HopCall &c = calls[i];
        const tm_gauge *g = c.g;
        if (!g->links[prec][0]) return fail(ctx, TM_ERR_PREC, "gauge not built in precision %d", prec);
        HopProblem &hp = B->p[i];
        for (int d = 0; d < 4; d++) hp.X[d] = g->p.dims[d];
        hp.vh = (int)g->vh;
        hp.nrhs = c.nrhs;
        hp.blk_start = blocks;
        const int spb = (nf == 2 && kNdSplit) ? bs / 2 : bs;      // sites per block
        hp.nsb = (int)((g->vh + spb - 1) / spb);
        hp.ngrp = c.nrhs / nr;
        hp.out_parity = c.out_parity;
        hp.zc = zc ? zc_for(zc, g->p.dims[2]) : 0;
        // slabs of about an eighth of the time extent (one XCD's share)
        hp.ts = 1;
        for (int d = (g->p.dims[3] + 7) / 8; d >= 1; d--)
            if (g->p.dims[3] % d == 0) {
                hp.ts = d;
                break;
            }
        hp.tsign = g->p.t_antiperiodic ? -1.0 : 1.0;
        hp.tw = make_twist(g->p, c.dagger);
        hp.k = c.k;
        hp.gauge[0] = g->links[prec][0];
        hp.gauge[1] = g->links[prec][1];
        hp.clov = g->clov_of(prec, c.out_parity);
        if (g->clover() && !hp.clov) return fail(ctx, TM_ERR_PREC, "clover term not built in precision %d", prec);
        hp.in = sptr(c.in, prec, g->vh, nf, c.nrhs);
        hp.out = sptr(c.out, prec, g->vh, nf, c.nrhs);
        hp.x = c.x ? sptr(c.x, prec, g->vh, nf, c.nrhs) : SpinorPtr{nullptr, nullptr};
        if (c.upd && !c.cg) return fail(ctx, TM_ERR_ARG, "internal: residual update needs CG scalars");
        hp.upd = c.upd ? c.cg : nullptr;
        hp.red.op = c.fin;
        if ((c.fin == FIN_ALPHA || c.fin == FIN_BETA || c.fin == FIN_STORE_RR || c.fin == FIN_RELIABLE) && !c.cg)
            return fail(ctx, TM_ERR_ARG, "internal: hop reduction needs CG scalars");
        if (c.fin == FIN_STORE && !c.red_out) return fail(ctx, TM_ERR_ARG, "internal: no reduction output");
        if (c.fin != FIN_NONE) {
            RedSlot rs;
            TM_TRY(red_slot(ctx, i, (size_t)hp.nsb * c.nrhs, &rs));
            hp.red.partials = rs.partials;
            hp.red.cg = c.cg;
            hp.red.out = c.red_out;
            hp.red.nvec = c.nrhs;
            hp.red.nblk = hp.nsb;
        }
        blocks += hp.nsb * hp.ngrp;
    }
    B->total_blocks = blocks;
    return TM_OK;
}

// The second stage of the reductions of a launch (one block per problem).
template <typename Prob>
int finish_reductions(tm_ctx *ctx, const Prob *p, int n)
{
    FinishBatch F;
    memset(&F, 0, sizeof(F));
    bool any = false;
    for (int i = 0; i < n; i++) {
        F.r[i] = p[i].red;
        if (p[i].red.op != FIN_NONE) any = true;
        else F.r[i].nvec = 0;
    }
    if (!any) return TM_OK;
    F.nprob = n;
    F.gate = ctx->gate;
    TM_HIP(ctx, launch_finish(F, ctx->stream));
    return TM_OK;
}

int launch_hops(tm_ctx *ctx, const HopCall *calls, int n)
{
    if (n < 1 || n > kMaxProblems) return fail(ctx, TM_ERR_LIMIT, "too many problems in a batch");
    const tm_gauge *g0 = calls[0].g;
    const int prec = calls[0].prec, nf = g0->nf, recon = g0->recon;
    const int dagger = calls[0].dagger, twl = calls[0].twl;
    const bool clv = g0->clover();
    if (clv && twl) {
        // twisted clover: the neighbours' R^-1 (R^-+) is a separate pass over
        // the input into a temporary of the input parity, then a plain hop
        HopCall pre[kMaxProblems];
        for (int i = 0; i < n; i++) {
            const HopCall &c = calls[i];
            int rc = TM_OK;
            void *tmp = twl_tmp(ctx, i, c.g, prec, c.nrhs, &rc);
            if (!tmp) return rc;
            const void *cl = c.g->clov_of(prec, 1 - c.out_parity);
            if (!cl) return fail(ctx, TM_ERR_PREC, "clover term not built in precision %d", prec);
            TM_HIP(ctx, twist_apply(prec, nf, sptr(tmp, prec, c.g->vh, nf, c.nrhs),
                                    sptr(c.in, prec, c.g->vh, nf, c.nrhs), c.g->vh, c.nrhs,
                                    make_twist(c.g->p, c.dagger), 1, ctx->stream, cl, ctx->gate));
            pre[i] = c;
            pre[i].in = tmp;
            pre[i].twl = 0;
        }
        return launch_hops(ctx, pre, n);
    }
    // rhs per thread: the instantiated groupings that divide every problem's
    // rhs count are tuning candidates; the heuristic choice is the default
    std::vector<int> nrs;
    for (int q : {1, 2, 4}) {
        bool ok = q == 1 || (nf == 1 && recon == 12 && !clv && !(q == 4 && prec == TM_FP64));
        for (int i = 0; i < n && ok; i++) ok = calls[i].nrhs % q == 0;
        if (ok) nrs.push_back(q);
    }
    if (ctx->force_nr && std::find(nrs.begin(), nrs.end(), ctx->force_nr) != nrs.end()) nrs = {ctx->force_nr};
    int nr_def = 1 << 30;
    for (int i = 0; i < n; i++) nr_def = std::min(nr_def, choose_nr(prec, nf, calls[i].nrhs, recon, ctx->force_nr));
    if (clv || std::find(nrs.begin(), nrs.end(), nr_def) == nrs.end()) nr_def = 1;
    // LDS staging only where the block's rows fit in half a compute unit's LDS
    int xrow = 0;
    for (int i = 0; i < n; i++) xrow = std::max(xrow, calls[i].g->p.dims[0] / 2);
    const unsigned lds_cu = ctx->lds_per_cu ? ctx->lds_per_cu : kLdsPerCUDefault;
    auto staging_fits = [&](int bs) { return hop_staging_bytes(bs, xrow) <= lds_cu / 2; };
    std::vector<HopCfg> cand;
    for (int q : nrs)
        for (HopCfg c : cfg_candidates(prec, nf, q, twl, recon, clv)) {
            c.nr = q;
            if (c.ldss && !staging_fits(c.bs)) continue;
            cand.push_back(c);
        }
    long vh_total = 0;
    size_t wset = 0;
    for (int i = 0; i < n; i++) {
        const tm_gauge *g = calls[i].g;
        vh_total += (long)g->vh * calls[i].nrhs;
        wset += 2 * gauge_parity_bytes(prec, recon, g->vh) + 3 * spinor_field_bytes(prec, g->vh, nf, calls[i].nrhs);
    }
    HopCfg cfg = default_cfg(twl, wset);
    cfg.nr = nr_def;
    const std::string key = tune_key(prec, nf, nrs.back(), dagger, twl, calls[0].epi, recon, vh_total, clv);
    auto it = ctx->tuned.find(key);
    if (ctx->force_bs || ctx->force_lnt >= 0) {
        HopCfg want{ctx->force_bs ? ctx->force_bs : cfg.bs, ctx->force_lnt >= 0 ? ctx->force_lnt != 0 : cfg.lnt,
                    0};
        want.nr = nr_def;
        for (const HopCfg &c : cand)
            if (c.bs == want.bs && c.lnt == want.lnt && c.wcap == 0 && c.nr == want.nr) cfg = want;
    } else if (it != ctx->tuned.end()) {
        cfg = cfg_decode(it->second);
    } else if (ctx->tuning && cand.size() > 1 && !ctx->gate && !ctx->no_alloc) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        (void)hipStreamIsCapturing(ctx->stream, &cs);
        if (cs == hipStreamCaptureStatusNone) {
            // time the instantiated configurations on the real launch: rhs per
            // thread x block size x link-load policy x wave cap in
            // lexicographic site order, then the four best of those with each
            // brick depth of the site order.  Trials write a scratch output
            // wherever a call's output is also one of its inputs (an in-place
            // xpay or a residual update would otherwise accumulate over the
            // repeated launches).
            HopCall tc[kMaxProblems];
            for (int i = 0; i < n; i++) {
                tc[i] = calls[i];
                if (tc[i].out == tc[i].x || tc[i].out == tc[i].in || tc[i].upd) {
                    char name[48];
                    snprintf(name, sizeof(name), "tune_out_%d", i);
                    int rc = TM_OK;
                    tc[i].out = workspace(ctx, name, spinor_field_bytes(prec, tc[i].g->vh, nf, tc[i].nrhs), &rc);
                    if (!tc[i].out) return rc;
                }
            }
            hipEvent_t e0, e1;
            TM_HIP(ctx, hipEventCreate(&e0));
            TM_HIP(ctx, hipEventCreate(&e1));
            // each trial: one untimed launch, then `reps` timed back to back
            auto trial = [&](const HopCfg &c, int reps, float *ms_per) -> int {
                HopBatch B;
                unsigned lds = 0;
                TM_TRY(build_hop_batch(ctx, tc, n, c.nr, c.bs, &B, c.zc, c.nt));
                TM_TRY(hop_lds_plan(ctx, B, prec, nf, c.nr, dagger, twl, recon, c, clv, &lds));
                TM_HIP(ctx, dispatch_hop(B, prec, nf, c.nr, dagger, twl, recon, c, clv, lds, ctx->stream));
                TM_HIP(ctx, hipEventRecord(e0, ctx->stream));
                for (int r = 0; r < reps; r++)
                    TM_HIP(ctx, dispatch_hop(B, prec, nf, c.nr, dagger, twl, recon, c, clv, lds, ctx->stream));
                TM_HIP(ctx, hipEventRecord(e1, ctx->stream));
                TM_HIP(ctx, hipEventSynchronize(e1));
                float ms = 0.f;
                TM_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
                *ms_per = ms / reps;
                return TM_OK;
            };
            // stage 1: every candidate briefly, lexicographic site order
            // (candidates whose LDS request the compute unit cannot hold are
            // skipped)
            std::vector<std::pair<float, HopCfg>> t1;
            for (const HopCfg &c : cand) {
                HopBatch B;
                unsigned lds = 0;
                TM_TRY(build_hop_batch(ctx, tc, n, c.nr, c.bs, &B, c.zc, c.nt));
                if (hop_lds_plan(ctx, B, prec, nf, c.nr, dagger, twl, recon, c, clv, &lds, true) != TM_OK) continue;
                float ms;
                TM_TRY(trial(c, 4, &ms));
                t1.push_back({ms, c});
            }
            std::sort(t1.begin(), t1.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
            // stage 2: the four fastest, each in lexicographic order and in
            // bricks of 8, 4 and 2 z-planes (the LDS-staged variant needs the
            // lexicographic order), timed longer: the best of three batches
            // of eight launches, which is less sensitive to clock changes
            float best = 1e30f;
            auto timed = [&](const HopCfg &c, float *ms) -> int {
                *ms = 1e30f;
                for (int rep = 0; rep < 3; rep++) {
                    float m;
                    TM_TRY(trial(c, 8, &m));
                    *ms = std::min(*ms, m);
                }
                return TM_OK;
            };
            std::vector<std::pair<float, HopCfg>> t2;
            for (size_t i = 0; i < std::min<size_t>(4, t1.size()); i++)
                for (int z : {0, 8, 4, 2}) {
                    HopCfg c = t1[i].second;
                    if (z && c.ldss) break;
                    c.zc = z;
                    float ms;
                    TM_TRY(timed(c, &ms));
                    t2.push_back({ms, c});
                    if (ms < best) {
                        best = ms;
                        cfg = c;
                    }
                }
            // stage 3: the three best of stage 2 with the single-use streams
            // non-temporal (output; with the xpay operand and / or the time
            // neighbours): which helps depends on the site order and on the
            // block shape, so they are tried together
            std::sort(t2.begin(), t2.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
            for (size_t i = 0; i < std::min<size_t>(3, t2.size()); i++)
                for (int nt : {1, 3, 5, 7}) {
                    HopCfg c = t2[i].second;
                    c.nt = nt;
                    float ms;
                    TM_TRY(timed(c, &ms));
                    if (ms < best) {
                        best = ms;
                        cfg = c;
                    }
                }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            const int code = cfg_code(cfg);
            ctx->tuned[key] = code;
            save_tune(ctx, key, code);
        }
    }
    if (ctx->force_zc >= 0) cfg.zc = ctx->force_zc;
    if (ctx->force_ldss >= 0 && (ctx->force_ldss == 0 || (prec == TM_FP32 && nf == 1 && cfg.nr == 1 &&
                                                            recon == 12 && !clv && !twl &&
                                                            staging_fits(cfg.bs))))
        cfg.ldss = ctx->force_ldss != 0;
    if (cfg.ldss) cfg.zc = 0;
    if (ctx->force_wcap >= 0) cfg.wcap = ctx->force_wcap;
    if (ctx->force_nt >= 0) cfg.nt = ctx->force_nt;
    HopBatch B;
    unsigned lds = 0;
    TM_TRY(build_hop_batch(ctx, calls, n, cfg.nr, cfg.bs, &B, cfg.zc, cfg.nt));
    TM_TRY(hop_lds_plan(ctx, B, prec, nf, cfg.nr, dagger, twl, recon, cfg, clv, &lds));
    TM_HIP(ctx, dispatch_hop(B, prec, nf, cfg.nr, dagger, twl, recon, cfg, clv, lds, ctx->stream));
    TM_TRY(finish_reductions(ctx, B.p, n));
    return TM_OK;
}

int hop1(tm_ctx *ctx, const HopCall &c) { return launch_hops(ctx, &c, 1); }

// ------------------------------------------------------------------ BLAS launch

constexpr size_t kBlasMaxBlocks = 4096;   // blocks per rhs of a BLAS launch
#ifndef TM_BLAS_UNROLL
#define TM_BLAS_UNROLL 4
#endif
constexpr size_t kBlasUnroll = TM_BLAS_UNROLL;   // units per thread and pass (streaming path)

struct BlasCall {
    uint32_t vh;
    int nrhs;
    const void *v[4];
    int fin;
    CGScalars *cg;
    double *red_out;
};

int launch_blas_batch(tm_ctx *ctx, int op, int pa, int pb, int nf, const BlasCall *calls, int n,
                      double scale = 1.0)
{
    if (n < 1 || n > kMaxProblems) return fail(ctx, TM_ERR_LIMIT, "too many problems in a batch");
    BlasBatch B;
    memset(&B, 0, sizeof(B));
    B.nprob = n;
    B.nf = nf;
    B.scale = scale;
    B.gate = ctx->gate;
    int blocks = 0;
    for (int i = 0; i < n; i++) {
        const BlasCall &c = calls[i];
        BlasProblem &bp = B.p[i];
        bp.vh = c.vh;
        bp.nrhs = c.nrhs;
        bp.blk_start = blocks;
        // units one rhs streams: chunks when every operand is FP64 / FP32
        // (one complex when both are FP64, else two), sites otherwise
        const bool flat = pa <= TM_FP32 && pb <= TM_FP32;
        const size_t units = flat ? (size_t)nf * ((pa == TM_FP64 && pb == TM_FP64) ? 12 : 6) * c.vh : c.vh;
        const size_t per_block = flat ? 256 * kBlasUnroll : 256;
        bp.nblk = (int)std::min<size_t>((units + per_block - 1) / per_block, kBlasMaxBlocks);
        // vector precisions per operation (see BlasOp)
        int vp[4] = {pa, pa, pa, pa};
        switch (op) {
        case OP_CG_UPDATE: vp[1] = vp[2] = vp[3] = pb; break;
        case OP_XPAY_X: vp[1] = vp[2] = pb; break;
        case OP_XPAY: vp[0] = vp[1] = pb; break;
        case OP_RESIDUAL: vp[2] = vp[3] = pb; break;
        case OP_CONVERT: vp[1] = pb; break;
        case OP_ACCUM_ZERO: vp[1] = pb; break;
        case OP_ACCUM_STEP: vp[1] = TM_FP32; vp[2] = pb; break;
        default: break;
        }
        for (int j = 0; j < 4; j++)
            bp.v[j] = c.v[j] ? sptr(c.v[j], vp[j], c.vh, nf, c.nrhs) : SpinorPtr{nullptr, nullptr};
        bp.red.op = c.fin;
        bp.red.cg = c.cg;
        // the CG updates read alpha and the xpays beta from the scalars
        const bool scalar_op = op == OP_CG_UPDATE || op == OP_XPAY_X || op == OP_XPAY || op == OP_ACCUM_STEP;
        if ((scalar_op || c.fin == FIN_ALPHA || c.fin == FIN_BETA || c.fin == FIN_STORE_RR ||
             c.fin == FIN_RELIABLE) && !c.cg)
            return fail(ctx, TM_ERR_ARG, "internal: BLAS op %d needs CG scalars", op);
        if (c.fin == FIN_STORE && !c.red_out) return fail(ctx, TM_ERR_ARG, "internal: no reduction output");
        if (c.fin != FIN_NONE) {
            RedSlot rs;
            TM_TRY(red_slot(ctx, i, (size_t)bp.nblk * c.nrhs * 2, &rs));
            bp.red.partials = rs.partials;
            bp.red.cg = c.cg;
            bp.red.out = c.red_out;
            bp.red.nvec = (op == OP_DOT) ? 2 * c.nrhs : c.nrhs;
            bp.red.nblk = bp.nblk;
        }
        blocks += bp.nblk * c.nrhs;
    }
    B.total_blocks = blocks;
    TM_HIP(ctx, launch_blas(op, pa, pb, B, ctx->stream));
    TM_TRY(finish_reductions(ctx, B.p, n));
    return TM_OK;
}

int blas1(tm_ctx *ctx, int op, int pa, int pb, int nf, const BlasCall &c, double scale = 1.0)
{
    return launch_blas_batch(ctx, op, pa, pb, nf, &c, 1, scale);
}

// ------------------------------------------------------------------ operators

// Odd temporary of the preconditioned operator, one per problem slot and precision.
void *odd_tmp(tm_ctx *ctx, int slot, const tm_gauge *g, int prec, int nrhs, int *rc)
{
    if (ctx->no_alloc && slot == 0 && ctx->tmp_override[0]) return ctx->tmp_override[0];
    char name[64];
    snprintf(name, sizeof(name), "odd_tmp_%d_%d", slot, prec);
    return workspace(ctx, name, spinor_field_bytes(prec, g->vh, g->nf, nrhs), rc);
}

// The two fused kernels of the preconditioned operator (Sec. 2.1):
//   asym:  t = R_oo^-1 D_oe x;   out = R_ee x - kappa^2 D_eo t
//   sym:   t = R_oo^-1 D_oe x;   out = x - kappa^2 R_ee^-1 D_eo t
//   asym^+: the same with D^+ and R^+ (twist of -mu)
//   sym^+:  t = R_oo^-+ D^+_oe R_ee^-+ x (twist on load); out = x - kappa^2 D^+_eo t
// Over n problems at once; `fin` reduces |out|^2 per rhs.
int mat_pc_batch(tm_ctx *ctx, const tm_gauge *const *g, void *const *out, const void *const *in,
                 const int *nrhs, int n, int prec, int pc, int dagger, int fin, CGScalars *const *cg,
                 bool upd = false)
{
    HopCall k1[kMaxProblems], k2[kMaxProblems];
    for (int i = 0; i < n; i++) {
        int rc = TM_OK;
        void *tmp = odd_tmp(ctx, i, g[i], prec, nrhs[i], &rc);
        if (!tmp) return rc;
        const double k2c = -g[i]->p.kappa * g[i]->p.kappa;
        k1[i] = HopCall{g[i], prec, 1, dagger, 0, TM_EPI_TWINV, in[i], tmp, nullptr, 0.0, nrhs[i],
                        FIN_NONE, nullptr, nullptr};
        k2[i] = HopCall{g[i], prec, 0, dagger, 0, TM_EPI_RX_PLUS_KD, tmp, out[i], in[i], k2c, nrhs[i],
                        fin, cg ? cg[i] : nullptr, nullptr, upd ? 1 : 0};
        if (pc == TM_PC_SYM) {
            if (!dagger) {
                k2[i].epi = TM_EPI_X_PLUS_K_TWINV_D;
            } else {
                k1[i].twl = 1;
                k2[i].epi = TM_EPI_X_PLUS_KD;
            }
        }
    }
    TM_TRY(launch_hops(ctx, k1, n));
    TM_TRY(launch_hops(ctx, k2, n));
    return TM_OK;
}

int check_gauge_prec(tm_ctx *ctx, const tm_gauge *g, int prec)
{
    if (!g) return fail(ctx, TM_ERR_ARG, "null gauge");
    if (!valid_prec(prec)) return fail(ctx, TM_ERR_PREC, "bad precision %d", prec);
    if (!g->links[prec][0]) return fail(ctx, TM_ERR_PREC, "gauge not built in precision %d", prec);
    if (g->clover() && prec > TM_FP32)
        return fail(ctx, TM_ERR_PREC, "the twisted-clover operator runs in FP64 and FP32");
    return TM_OK;
}

}  // namespace

// ================================================================== C ABI

extern "C" {

const char *tm_error_string(int code)
{
    switch (code) {
    case TM_OK: return "ok";
    case TM_NOT_CONVERGED: return "solver did not converge within maxiter";
    case TM_ERR_ARG: return "invalid argument";
    case TM_ERR_DIMS: return "lattice extents must be even and >= 2";
    case TM_ERR_PARITY: return "parity must be 0 (even) or 1 (odd)";
    case TM_ERR_PREC: return "precision not available";
    case TM_ERR_SINGULAR: return "twist R is singular (1 + a^2 - b^2 = 0)";
    case TM_ERR_NAN: return "non-finite value";
    case TM_ERR_HIP: return "HIP runtime error";
    case TM_ERR_NOMEM: return "out of device memory";
    case TM_ERR_LIMIT: return "size beyond a library limit";
    }
    return "unknown error";
}

const char *tm_last_error(tm_ctx *ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

int tm_ctx_create(tm_ctx **ctx, void *hip_stream)
{
    if (!ctx) return TM_ERR_ARG;
    tm_ctx *c = new tm_ctx();
    c->stream = (hipStream_t)hip_stream;
    // Without a device the context still validates arguments (every check
    // runs before the first HIP call); device work then fails with TM_ERR_HIP.
    if (hipGetDevice(&c->device) != hipSuccess) c->device = -1;
    if (c->device >= 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, c->device) ==
                hipSuccess && v > 0)
            c->lds_per_cu = (unsigned)v;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, c->device) == hipSuccess && v > 0)
            c->lds_per_block = (unsigned)v;
        else if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) == hipSuccess &&
                 v > 0)
            c->lds_per_block = (unsigned)v;
        (void)hipGetLastError();
        // the allocation-free call's scratch on this (the current) device
        c->scratch_err = noalloc_scratch(c->device, &c->scratch);
        if (c->scratch_err != hipSuccess) c->scratch = nullptr;
        (void)hipGetLastError();
    }
    const char *e = getenv("TM_XCD_REMAP");
    if (e) c->xcd_remap = atoi(e);
    e = getenv("TM_HOP_BS");
    if (e) c->force_bs = atoi(e);
    e = getenv("TM_LINK_NT");
    if (e) c->force_lnt = atoi(e) ? 1 : 0;
    e = getenv("TM_HOP_ZC");
    if (e) c->force_zc = std::max(0, atoi(e));
    e = getenv("TM_HOP_LDS");
    if (e) c->force_ldss = atoi(e) ? 1 : 0;
    e = getenv("TM_HOP_NR");
    if (e) c->force_nr = atoi(e);
    e = getenv("TM_HOP_NT");
    if (e) c->force_nt = atoi(e) & 7;
    e = getenv("TM_CG_FUSE");
    if (e) c->cg_fuse = atoi(e) ? 1 : 0;
    e = getenv("TM_VERBOSE");
    if (e) c->verbose = atoi(e);
    e = getenv("TM_HOP_WCAP");
    if (e) c->force_wcap = std::min(8, std::max(0, atoi(e)));
    e = getenv("TM_TUNE");
    if (e) c->tuning = atoi(e) ? 1 : 0;
    load_tune(c);
    *ctx = c;
    return TM_OK;
}

int tm_ctx_set_stream(tm_ctx *ctx, void *hip_stream)
{
    if (!ctx) return TM_ERR_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return TM_OK;
}

int tm_ctx_destroy(tm_ctx *ctx)
{
    if (!ctx) return TM_ERR_ARG;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &kv : ctx->ws)
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    if (ctx->host_scratch) (void)hipHostFree(ctx->host_scratch);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
    delete ctx;
    return TM_OK;
}

int tm_set_tuning(tm_ctx *ctx, int enable)
{
    if (!ctx) return TM_ERR_ARG;
    ctx->tuning = enable ? 1 : 0;
    return TM_OK;
}

int tm_gauge_create(tm_ctx *ctx, tm_gauge **gout, const void *links_dev, const tm_params *p,
                    int recon, unsigned prec_mask)
{
    if (!ctx) return TM_ERR_ARG;
    if (!gout || !links_dev) return fail(ctx, TM_ERR_ARG, "null gauge output or links");
    TM_TRY(check_params(ctx, p));
    if (p->t_antiperiodic != 0 && p->t_antiperiodic != 1)
        return fail(ctx, TM_ERR_ARG, "t_antiperiodic must be 0 or 1");
    if (recon != 12 && recon != 18 && recon != 8) return fail(ctx, TM_ERR_ARG, "recon must be 8, 12 or 18");
    if (prec_mask == 0 || (prec_mask & ~0xFu)) return fail(ctx, TM_ERR_PREC, "bad precision mask");
    if (p->csw != 0.0) {
        if (prec_mask & ~((1u << TM_FP64) | (1u << TM_FP32)))
            return fail(ctx, TM_ERR_PREC, "the twisted-clover operator runs in FP64 and FP32");
        if (recon == 8) return fail(ctx, TM_ERR_ARG, "twisted clover with 12- or 18-real links");
    }
    int rc = TM_OK;
    int *bad = (int *)workspace(ctx, "gauge_bad", sizeof(int), &rc);
    if (!bad) return rc;
    TM_HIP(ctx, hipMemsetAsync(bad, 0, sizeof(int), ctx->stream));
    tm_gauge *g = new tm_gauge();
    g->p = *p;
    g->recon = recon;
    g->nf = nflav(*p);
    g->vh = half_volume(*p);
    for (int prec = 0; prec < 4; prec++) {
        if (!(prec_mask & (1u << prec))) continue;
        for (int par = 0; par < 2; par++) {
            if (hipMalloc(&g->links[prec][par], gauge_parity_bytes(prec, recon, g->vh)) != hipSuccess) {
                g->links[prec][par] = nullptr;
                tm_gauge_destroy(g);
                return fail(ctx, TM_ERR_NOMEM, "cannot allocate packed links");
            }
        }
        hipError_t e = gauge_pack(prec, recon, g->links[prec][0], g->links[prec][1], links_dev,
                                  p->dims, g->vh, bad, ctx->stream);
        if (e != hipSuccess) {
            tm_gauge_destroy(g);
            return fail(ctx, TM_ERR_HIP, "gauge pack: %s", hipGetErrorString(e));
        }
    }
    if (g->clover()) {
        void *d[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
        for (int prec = 0; prec < 2; prec++) {
            if (!(prec_mask & (1u << prec))) continue;
            for (int par = 0; par < 2; par++) {
                if (hipMalloc(&g->clov[prec][par], clover_parity_bytes(prec, g->vh)) != hipSuccess) {
                    g->clov[prec][par] = nullptr;
                    tm_gauge_destroy(g);
                    return fail(ctx, TM_ERR_NOMEM, "cannot allocate the clover term");
                }
                d[prec][par] = g->clov[prec][par];
            }
        }
        const double a = 2 * p->kappa * p->mu;
        const double b = p->flavor == TM_TWIST_NDEG ? 2 * p->kappa * p->epsilon : 0.0;
        hipError_t ce = clover_build(d[0][0] ? d[0] : nullptr, d[1][0] ? d[1] : nullptr, links_dev, p->dims,
                                     g->vh, p->kappa * p->csw, a * a - b * b, bad, ctx->stream);
        if (ce != hipSuccess) {
            tm_gauge_destroy(g);
            return fail(ctx, TM_ERR_HIP, "clover build: %s", hipGetErrorString(ce));
        }
    }
    int hbad = 0;
    hipError_t e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        tm_gauge_destroy(g);
        return fail(ctx, TM_ERR_HIP, "gauge pack: %s", hipGetErrorString(e));
    }
    if (hbad) {
        tm_gauge_destroy(g);
        if (p->csw != 0.0)
            return fail(ctx, TM_ERR_SINGULAR, "twisted clover: A^2 + a^2 - b^2 is singular at some site");
        return fail(ctx, TM_ERR_ARG, "8-real links: a link has |U01|^2 + |U02|^2 < 1e-10 "
                                     "(not representable; use 12 or 18)");
    }
    *gout = g;
    return TM_OK;
}

int tm_gauge_destroy(tm_gauge *g)
{
    if (!g) return TM_ERR_ARG;
    // hipFree waits for outstanding device work; the gauge holds no reference
    // to the context that built it, so either may be destroyed first.
    for (int prec = 0; prec < 4; prec++)
        for (int par = 0; par < 2; par++)
            if (g->links[prec][par]) (void)hipFree(g->links[prec][par]);
    for (int prec = 0; prec < 2; prec++)
        for (int par = 0; par < 2; par++)
            if (g->clov[prec][par]) (void)hipFree(g->clov[prec][par]);
    delete g;
    return TM_OK;
}

size_t tm_gauge_bytes(const tm_gauge *g, int prec)
{
    if (!g || !valid_prec(prec) || !g->links[prec][0]) return 0;
    return 2 * gauge_parity_bytes(prec, g->recon, g->vh);
}

size_t tm_spinor_bytes(const tm_params *p, int prec, int nrhs)
{
    if (!p || !valid_prec(prec) || nrhs < 1) return 0;
    if (check_params(nullptr, p) != TM_OK) return 0;
    return spinor_field_bytes(prec, half_volume(*p), nflav(*p), nrhs);
}

int tm_spinor_pack(tm_ctx *ctx, void *dst, const void *src, const tm_params *p, int prec,
                   int parity, int nrhs, int basis)
{
    if (!ctx) return TM_ERR_ARG;
    TM_TRY(check_params(ctx, p));
    if (!dst || !src) return fail(ctx, TM_ERR_ARG, "null field");
    if (!valid_prec(prec)) return fail(ctx, TM_ERR_PREC, "bad precision");
    if (parity != 0 && parity != 1) return fail(ctx, TM_ERR_PARITY, "bad parity %d", parity);
    if (nrhs < 1) return fail(ctx, TM_ERR_ARG, "nrhs must be >= 1");
    if (basis != TM_BASIS_INTERNAL && basis != TM_BASIS_CHIRAL) return fail(ctx, TM_ERR_ARG, "bad basis %d", basis);
    const uint32_t vh = half_volume(*p);
    const int nf = nflav(*p);
    TM_HIP(ctx, spinor_pack(prec, sptr(dst, prec, vh, nf, nrhs), src, p->dims, vh, parity, nf, nrhs,
                            basis, ctx->stream));
    return TM_OK;
}

int tm_spinor_unpack(tm_ctx *ctx, void *dst, const void *src, const tm_params *p, int prec,
                     int parity, int nrhs, int basis)
{
    if (!ctx) return TM_ERR_ARG;
    TM_TRY(check_params(ctx, p));
    if (!dst || !src) return fail(ctx, TM_ERR_ARG, "null field");
    if (!valid_prec(prec)) return fail(ctx, TM_ERR_PREC, "bad precision");
    if (parity != 0 && parity != 1) return fail(ctx, TM_ERR_PARITY, "bad parity %d", parity);
    if (nrhs < 1) return fail(ctx, TM_ERR_ARG, "nrhs must be >= 1");
    if (basis != TM_BASIS_INTERNAL && basis != TM_BASIS_CHIRAL) return fail(ctx, TM_ERR_ARG, "bad basis %d", basis);
    const uint32_t vh = half_volume(*p);
    const int nf = nflav(*p);
    TM_HIP(ctx, spinor_unpack(prec, dst, sptr(src, prec, vh, nf, nrhs), p->dims, vh, parity, nf,
                              nrhs, basis, ctx->stream));
    return TM_OK;
}

int tm_dslash(tm_ctx *ctx, void *out, const void *in, const tm_gauge *g, int prec,
              int out_parity, int dagger, int twist_on_load, int epi, const void *x,
              double k, int nrhs)
{
    if (!ctx) return TM_ERR_ARG;
    TM_TRY(check_gauge_prec(ctx, g, prec));
    if (!out || !in) return fail(ctx, TM_ERR_ARG, "null field");
    if (out == in) return fail(ctx, TM_ERR_ARG, "out and in must not alias");
    if (out_parity != 0 && out_parity != 1) return fail(ctx, TM_ERR_PARITY, "bad parity");
    if ((int)epi < TM_EPI_NONE || (int)epi > TM_EPI_X_PLUS_KD) return fail(ctx, TM_ERR_ARG, "bad epilogue");
    if ((int)epi >= TM_EPI_RX_PLUS_KD && !x) return fail(ctx, TM_ERR_ARG, "epilogue needs x");
    if (nrhs < 1) return fail(ctx, TM_ERR_ARG, "nrhs must be >= 1");
    if (!std::isfinite(k)) return fail(ctx, TM_ERR_ARG, "non-finite k");
    HopCall c{g, prec, out_parity, dagger ? 1 : 0, twist_on_load ? 1 : 0, (int)epi, in, out, x, k,
              nrhs, FIN_NONE, nullptr, nullptr};
    return hop1(ctx, c);
}

int tm_mat_pc(tm_ctx *ctx, void *out_e, const void *in_e, const tm_gauge *g, int prec,
              int pc, int dagger, int nrhs)
{
    if (!ctx) return TM_ERR_ARG;
    TM_TRY(check_gauge_prec(ctx, g, prec));
    if (!out_e || !in_e) return fail(ctx, TM_ERR_ARG, "null field");
    if (out_e == in_e) return fail(ctx, TM_ERR_ARG, "out and in must not alias");
    if (pc != TM_PC_ASYM && pc != TM_PC_SYM) return fail(ctx, TM_ERR_ARG, "bad pc type");
    if (nrhs < 1) return fail(ctx, TM_ERR_ARG, "nrhs must be >= 1");
    return mat_pc_batch(ctx, &g, &out_e, &in_e, &nrhs, 1, prec, pc, dagger ? 1 : 0, FIN_NONE, nullptr);
}

int tm_mat_pc_noalloc(tm_ctx *ctx, void *out_e, const void *in_e, const tm_gauge *g, int prec, int pc,
                      int dagger, int nrhs)
{
    if (!ctx) return TM_ERR_ARG;
    TM_TRY(check_gauge_prec(ctx, g, prec));
    if (!out_e || !in_e) return fail(ctx, TM_ERR_ARG, "null field");
    if (out_e == in_e) return fail(ctx, TM_ERR_ARG, "out and in must not alias");
    if (pc != TM_PC_ASYM && pc != TM_PC_SYM) return fail(ctx, TM_ERR_ARG, "bad pc type");
    if (nrhs < 1) return fail(ctx, TM_ERR_ARG, "nrhs must be >= 1");
    // the odd temporary, and for the twisted-clover sym^+ form the
    // twist-on-load temporary, both from the device scratch
    const size_t field = (spinor_field_bytes(prec, g->vh, g->nf, nrhs) + 255) & ~(size_t)255;
    const bool twl = g->clover() && pc == TM_PC_SYM && dagger;
    const size_t need = twl ? 2 * field : field;
    if (need > kNoAllocScratchBytes)
        return fail(ctx, TM_ERR_LIMIT,
                    "tm_mat_pc_noalloc: temporaries of %zu bytes exceed the %zu-byte device scratch", need,
                    kNoAllocScratchBytes);
    if (!ctx->scratch)
        return fail(ctx, TM_ERR_HIP, "tm_mat_pc_noalloc: device scratch unavailable (%s)",
                    hipGetErrorString(ctx->scratch_err));
    ctx->tmp_override[0] = ctx->scratch;
    ctx->tmp_override[1] = twl ? (char *)ctx->scratch + field : nullptr;
    ctx->no_alloc = true;
    const int rc = mat_pc_batch(ctx, &g, &out_e, &in_e, &nrhs, 1, prec, pc, dagger ? 1 : 0, FIN_NONE, nullptr);
    ctx->no_alloc = false;
    ctx->tmp_override[0] = ctx->tmp_override[1] = nullptr;
    return rc;
}

int tm_twist(tm_ctx *ctx, void *out, const void *in, const tm_gauge *g, int prec, int parity,
             int dagger, int inverse, int nrhs)
{
    if (!ctx) return TM_ERR_ARG;
    TM_TRY(check_gauge_prec(ctx, g, prec));
    if (!out || !in) return fail(ctx, TM_ERR_ARG, "null field");
    if (parity != 0 && parity != 1) return fail(ctx, TM_ERR_PARITY, "bad parity");
    if (nrhs < 1) return fail(ctx, TM_ERR_ARG, "nrhs must be >= 1");
    TM_HIP(ctx, twist_apply(prec, g->nf, sptr(out, prec, g->vh, g->nf, nrhs),
                            sptr(in, prec, g->vh, g->nf, nrhs), g->vh, nrhs,
                            make_twist(g->p, dagger ? 1 : 0), inverse ? 1 : 0, ctx->stream,
                            g->clov_of(prec, parity)));
    return TM_OK;
}

int tm_twist_inv(tm_ctx *ctx, void *out, const void *in, const tm_gauge *g, int prec, int parity,
                 int dagger, int nrhs)
{
    return tm_twist(ctx, out, in, g, prec, parity, dagger, 1, nrhs);
}

int tm_prepare(tm_ctx *ctx, void *bhat_e, const void *b_e, const void *b_o, const tm_gauge *g,
               int prec, int pc, int nrhs)
{
    if (!ctx) return TM_ERR_ARG;
    TM_TRY(check_gauge_prec(ctx, g, prec));
    if (!bhat_e || !b_e || !b_o) return fail(ctx, TM_ERR_ARG, "null field");
    if (bhat_e == b_o) return fail(ctx, TM_ERR_ARG, "bhat_e and b_o must not alias");
    if (pc != TM_PC_ASYM && pc != TM_PC_SYM) return fail(ctx, TM_ERR_ARG, "bad pc type");
    if (nrhs < 1) return fail(ctx, TM_ERR_ARG, "nrhs must be >= 1");
    HopCall c{g, prec, 0, 0, 1, pc == TM_PC_SYM ? TM_EPI_TWINV_X_PLUS_KD : TM_EPI_X_PLUS_KD, b_o,
              bhat_e, b_e, g->p.kappa, nrhs, FIN_NONE, nullptr, nullptr};
    return hop1(ctx, c);
}

int tm_reconstruct_odd(tm_ctx *ctx, void *x_o, const void *x_e, const void *b_o, const tm_gauge *g,
                       int prec, int nrhs)
{
    if (!ctx) return TM_ERR_ARG;
    TM_TRY(check_gauge_prec(ctx, g, prec));
    if (!x_o || !x_e || !b_o) return fail(ctx, TM_ERR_ARG, "null field");
    if (x_o == x_e) return fail(ctx, TM_ERR_ARG, "x_o and x_e must not alias");
    if (nrhs < 1) return fail(ctx, TM_ERR_ARG, "nrhs must be >= 1");
    HopCall c{g, prec, 1, 0, 0, TM_EPI_TWINV_X_PLUS_KD, x_e, x_o, b_o, g->p.kappa, nrhs, FIN_NONE,
              nullptr, nullptr};
    return hop1(ctx, c);
}

static int reduce_to_host(tm_ctx *ctx, int op, int prec, const tm_params *p, const void *x,
                          const void *y, int nrhs, double *out_host, int nout)
{
    int rc = TM_OK;
    double *dres = (double *)workspace(ctx, "red_result", (size_t)nout * sizeof(double), &rc);
    if (!dres) return rc;
    double *h = host_scratch(ctx, nout, &rc);
    if (!h) return rc;
    BlasCall c{half_volume(*p), nrhs, {x, y, nullptr, nullptr}, FIN_STORE, nullptr, dres};
    TM_TRY(blas1(ctx, op, prec, prec, nflav(*p), c));
    TM_HIP(ctx, hipMemcpyAsync(h, dres, nout * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    TM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    memcpy(out_host, h, nout * sizeof(double));
    return TM_OK;
}

int tm_norm2(tm_ctx *ctx, double *out_host, const void *x, const tm_params *p, int prec, int nrhs)
{
    if (!ctx) return TM_ERR_ARG;
    TM_TRY(check_params(ctx, p));
    if (!out_host || !x) return fail(ctx, TM_ERR_ARG, "null pointer");
    if (!valid_prec(prec)) return fail(ctx, TM_ERR_PREC, "bad precision");
    if (nrhs < 1) return fail(ctx, TM_ERR_ARG, "nrhs must be >= 1");
    return reduce_to_host(ctx, OP_NORM2, prec, p, x, nullptr, nrhs, out_host, nrhs);
}

int tm_dot(tm_ctx *ctx, double *out_host, const void *x, const void *y, const tm_params *p,
           int prec, int nrhs)
{
    if (!ctx) return TM_ERR_ARG;
    TM_TRY(check_params(ctx, p));
    if (!out_host || !x || !y) return fail(ctx, TM_ERR_ARG, "null pointer");
    if (!valid_prec(prec)) return fail(ctx, TM_ERR_PREC, "bad precision");
    if (nrhs < 1) return fail(ctx, TM_ERR_ARG, "nrhs must be >= 1");
    return reduce_to_host(ctx, OP_DOT, prec, p, x, y, nrhs, out_host, 2 * nrhs);
}

int tm_convert(tm_ctx *ctx, void *dst, int dst_prec, const void *src, int src_prec,
               const tm_params *p, int nrhs)
{
    if (!ctx) return TM_ERR_ARG;
    TM_TRY(check_params(ctx, p));
    if (!dst || !src) return fail(ctx, TM_ERR_ARG, "null field");
    if (!valid_prec(dst_prec) || !valid_prec(src_prec)) return fail(ctx, TM_ERR_PREC, "bad precision");
    if (nrhs < 1) return fail(ctx, TM_ERR_ARG, "nrhs must be >= 1");
    BlasCall c{half_volume(*p), nrhs, {src, dst, nullptr, nullptr}, FIN_NONE, nullptr, nullptr};
    return blas1(ctx, OP_CONVERT, src_prec, dst_prec, nflav(*p), c);
}

int tm_scale(tm_ctx *ctx, void *dst, int dst_prec, const void *src, int src_prec, double a, const tm_params *p,
             int nrhs)
{
    if (!ctx) return TM_ERR_ARG;
    TM_TRY(check_params(ctx, p));
    if (!dst || !src) return fail(ctx, TM_ERR_ARG, "null field");
    if (!valid_prec(dst_prec) || !valid_prec(src_prec)) return fail(ctx, TM_ERR_PREC, "bad precision");
    if (nrhs < 1) return fail(ctx, TM_ERR_ARG, "nrhs must be >= 1");
    if (!std::isfinite(a)) return fail(ctx, TM_ERR_ARG, "non-finite factor");
    BlasCall c{half_volume(*p), nrhs, {src, dst, nullptr, nullptr}, FIN_NONE, nullptr, nullptr};
    return blas1(ctx, OP_CONVERT, src_prec, dst_prec, nflav(*p), c, a);
}

// ------------------------------------------------------------------ CG

namespace {

struct CGProblem {
    const tm_gauge *g;
    int nrhs;
    void *x;            // FP64 solution (user)
    const void *b;      // FP64 rhs (user)
    // FP64 work vectors
    void *c, *y, *mid, *r64, *p64, *mp64, *ap64;
    // low-precision work vectors (mixed)
    void *rlo, *plo, *mplo, *aplo, *xlo;
    CGScalars *cg;      // device [nrhs]
    double *dres;       // device [2*nrhs] norms
    double cc[64];      // |c|^2 per rhs (host)
};

int cg_setup_vectors(tm_ctx *ctx, CGProblem &pr, int slot, int inner)
{
    int rc = TM_OK;
    const tm_gauge *g = pr.g;
    const size_t b64 = spinor_field_bytes(TM_FP64, g->vh, g->nf, pr.nrhs);
    char name[64];
    auto vec = [&](const char *tag, size_t bytes) -> void * {
        snprintf(name, sizeof(name), "cg_%s_%d", tag, slot);
        return workspace(ctx, name, bytes, &rc);
    };
    pr.c = vec("c", b64);
    pr.y = vec("y", b64);
    pr.mid = vec("mid", b64);
    if (!pr.c || !pr.y || !pr.mid) return rc;
    if (inner == TM_FP64) {
        pr.r64 = vec("r", b64);
        pr.p64 = vec("p", b64);
        pr.mp64 = vec("mp", b64);
        pr.ap64 = vec("ap", b64);
        if (!pr.r64 || !pr.p64 || !pr.mp64 || !pr.ap64) return rc;
    } else {
        const size_t bl = spinor_field_bytes(inner, g->vh, g->nf, pr.nrhs);
        pr.rlo = vec("rlo", bl);
        pr.plo = vec("plo", bl);
        pr.mplo = vec("mplo", bl);
        pr.aplo = vec("aplo", bl);
        pr.xlo = vec("xlo", spinor_field_bytes(TM_FP32, g->vh, g->nf, pr.nrhs));
        if (!pr.rlo || !pr.plo || !pr.mplo || !pr.aplo || !pr.xlo) return rc;
    }
    pr.cg = (CGScalars *)vec("scalars", sizeof(CGScalars) * pr.nrhs);
    pr.dres = (double *)vec("dres", sizeof(double) * 2 * pr.nrhs);
    if (!pr.cg || !pr.dres) return rc;
    return TM_OK;
}

// norms of n problems' vectors (FP64 fields) into host array out[prob][rhs]
int norms_fp64(tm_ctx *ctx, std::vector<CGProblem> &pr, void *const *v, std::vector<std::vector<double>> &out)
{
    const int n = (int)pr.size();
    BlasCall calls[kMaxProblems];
    for (int i = 0; i < n; i++)
        calls[i] = BlasCall{pr[i].g->vh, pr[i].nrhs, {v[i], nullptr, nullptr, nullptr}, FIN_STORE,
                            nullptr, pr[i].dres};
    TM_TRY(launch_blas_batch(ctx, OP_NORM2, TM_FP64, TM_FP64, pr[0].g->nf, calls, n));
    int total = 0;
    for (auto &p : pr) total += p.nrhs;
    int rc = TM_OK;
    double *h = host_scratch(ctx, total, &rc);
    if (!h) return rc;
    int off = 0;
    for (int i = 0; i < n; i++) {
        TM_HIP(ctx, hipMemcpyAsync(h + off, pr[i].dres, pr[i].nrhs * sizeof(double),
                                   hipMemcpyDeviceToHost, ctx->stream));
        off += pr[i].nrhs;
    }
    TM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    out.assign(n, {});
    off = 0;
    for (int i = 0; i < n; i++) {
        out[i].assign(h + off, h + off + pr[i].nrhs);
        off += pr[i].nrhs;
    }
    return TM_OK;
}

int read_scalars(tm_ctx *ctx, std::vector<CGProblem> &pr, std::vector<std::vector<CGScalars>> &out)
{
    const int n = (int)pr.size();
    int total = 0;
    for (auto &p : pr) total += p.nrhs;
    int rc = TM_OK;
    double *h = host_scratch(ctx, total * sizeof(CGScalars) / sizeof(double), &rc);
    if (!h) return rc;
    CGScalars *hs = (CGScalars *)h;
    int off = 0;
    for (int i = 0; i < n; i++) {
        TM_HIP(ctx, hipMemcpyAsync(hs + off, pr[i].cg, pr[i].nrhs * sizeof(CGScalars),
                                   hipMemcpyDeviceToHost, ctx->stream));
        off += pr[i].nrhs;
    }
    TM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    out.assign(n, {});
    off = 0;
    for (int i = 0; i < n; i++) {
        out[i].assign(hs + off, hs + off + pr[i].nrhs);
        off += pr[i].nrhs;
    }
    return TM_OK;
}

// Normal operator in FP64 on all problems: out = M^+ M in (mid: M in)
int normal_op64(tm_ctx *ctx, std::vector<CGProblem> &pr, int pc, void *const *out, void *const *mid,
                const void *const *in)
{
    const int n = (int)pr.size();
    const tm_gauge *gs[kMaxProblems];
    int nr[kMaxProblems];
    for (int i = 0; i < n; i++) {
        gs[i] = pr[i].g;
        nr[i] = pr[i].nrhs;
    }
    TM_TRY(mat_pc_batch(ctx, gs, mid, in, nr, n, TM_FP64, pc, 0, FIN_NONE, nullptr));
    TM_TRY(mat_pc_batch(ctx, gs, out, (const void *const *)mid, nr, n, TM_FP64, pc, 1, FIN_NONE, nullptr));
    return TM_OK;
}

// r = c - A x (FP64) written to r (precision rp) and, if p given, to p; the
// norm finishes with `fin` into the CG scalars (or dres when fin == FIN_STORE).
int true_residual(tm_ctx *ctx, std::vector<CGProblem> &pr, int pc, int rp, void *const *r,
                  void *const *p, int fin)
{
    const int n = (int)pr.size();
    void *ys[kMaxProblems], *mids[kMaxProblems];
    const void *xs[kMaxProblems];
    for (int i = 0; i < n; i++) {
        ys[i] = pr[i].y;
        xs[i] = pr[i].x;
        mids[i] = pr[i].mid;
    }
    TM_TRY(normal_op64(ctx, pr, pc, ys, mids, xs));
    BlasCall calls[kMaxProblems];
    for (int i = 0; i < n; i++)
        calls[i] = BlasCall{pr[i].g->vh, pr[i].nrhs, {pr[i].c, pr[i].y, r[i], p ? p[i] : nullptr},
                            fin, pr[i].cg, pr[i].dres};
    return launch_blas_batch(ctx, OP_RESIDUAL, TM_FP64, rp, pr[0].g->nf, calls, n);
}

// cg_run's internal status: a mixed solve stopped on stalled reliable updates
// (x holds the accumulated solution; the caller continues in a wider format)
constexpr int kStalled = 100;

struct GraphCache {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    ~GraphCache()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// The CG driver over n problems (plain FP64 or mixed with reliable updates).
int cg_run(tm_ctx *ctx, std::vector<CGProblem> &pr, const tm_cg_params *par, tm_cg_result *res)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int n = (int)pr.size();
    const int pc = par->pc;
    const int inner = par->inner;
    const bool mixed = inner != TM_FP64;
    // reliable-update threshold: by default 0.01 for FP16 inner iterations,
    // 0.02 for BF16 (its 8-bit mantissa lets the iterated residual drift from
    // the true one sooner: on the 32^3 x 64 doublet 50 iterations and 6
    // updates at 0.02 against 61 and 5 at 0.01) and 0.001 for FP32 (the
    // residual is replaced once it has dropped by 1/delta since the last
    // replacement)
    // Below a floor set by the inner format's precision the iterated residual
    // stagnates before it has dropped by delta and no update would come
    // (measured: BF16 at 0.002 never converges), so delta is raised to it.
    const double delta_floor = inner == TM_FP32 ? 1e-5 : (inner == TM_FP16 ? 2e-3 : 1e-2);
    const double delta_default = inner == TM_FP32 ? 1e-3 : (inner == TM_FP16 ? 1e-2 : 2e-2);
    const double delta = std::max(par->delta > 0 ? par->delta : delta_default, delta_floor);
    const int check_every = par->check_every > 0 ? par->check_every : 8;
    const int nf = pr[0].g->nf;

    Phase phase;
    phase.enter("tm_cg: setup");
    for (int i = 0; i < n; i++) TM_TRY(cg_setup_vectors(ctx, pr[i], i, inner));
    // Every buffer an iteration touches exists before any graph capture: the
    // reduction slots at their largest size and the odd temporaries.
    for (int i = 0; i < n; i++) {
        RedSlot rs;
        // hop partials (one per 64-site block at most) and BLAS partials
        // (up to kBlasMaxBlocks per rhs, two per block for a dot product)
        const size_t need = std::max<size_t>(((pr[i].g->vh + 63) / 64) * pr[i].nrhs,
                                             (size_t)2 * kBlasMaxBlocks * pr[i].nrhs);
        TM_TRY(red_slot(ctx, i, need, &rs));
        int rc = TM_OK;
        if (!odd_tmp(ctx, i, pr[i].g, TM_FP64, pr[i].nrhs, &rc)) return rc;
        if (!odd_tmp(ctx, i, pr[i].g, inner, pr[i].nrhs, &rc)) return rc;
        if (pr[i].g->clover()) {
            if (!twl_tmp(ctx, i, pr[i].g, TM_FP64, pr[i].nrhs, &rc)) return rc;
            if (!twl_tmp(ctx, i, pr[i].g, inner, pr[i].nrhs, &rc)) return rc;
        }
    }

    const tm_gauge *gs[kMaxProblems];
    int nr[kMaxProblems];
    for (int i = 0; i < n; i++) {
        gs[i] = pr[i].g;
        nr[i] = pr[i].nrhs;
    }
    // c = M^+ b (solution MAT) or c = b (MATDAG_MAT)
    {
        void *cs[kMaxProblems];
        const void *bs[kMaxProblems];
        for (int i = 0; i < n; i++) {
            cs[i] = pr[i].c;
            bs[i] = pr[i].b;
        }
        if (par->solution == TM_SOLUTION_MATDAG_MAT) {
            BlasCall cp[kMaxProblems];
            for (int i = 0; i < n; i++)
                cp[i] = BlasCall{pr[i].g->vh, pr[i].nrhs, {pr[i].b, pr[i].c, nullptr, nullptr}, FIN_NONE,
                                 nullptr, nullptr};
            TM_TRY(launch_blas_batch(ctx, OP_CONVERT, TM_FP64, TM_FP64, nf, cp, n));
        } else {
            TM_TRY(mat_pc_batch(ctx, gs, cs, bs, nr, n, TM_FP64, pc, 1, FIN_NONE, nullptr));
        }
        std::vector<std::vector<double>> cc;
        TM_TRY(norms_fp64(ctx, pr, cs, cc));
        for (int i = 0; i < n; i++)
            for (int r = 0; r < pr[i].nrhs; r++) {
                pr[i].cc[r] = cc[i][r];
                if (!std::isfinite(cc[i][r])) return fail(ctx, TM_ERR_NAN, "non-finite source norm");
            }
    }
    // scalars
    {
        int rc = TM_OK;
        int total = 0;
        for (auto &p : pr) total += p.nrhs;
        double *h = host_scratch(ctx, total * sizeof(CGScalars) / sizeof(double) + 1, &rc);
        if (!h) return rc;
        CGScalars *hs = (CGScalars *)h;
        int off = 0;
        for (int i = 0; i < n; i++) {
            for (int r = 0; r < pr[i].nrhs; r++) {
                CGScalars s{};
                s.stop2 = par->tol * par->tol * pr[i].cc[r];
                s.active = pr[i].cc[r] > 0 ? 1 : 0;
                const double sf = par->stall_factor > 0 ? par->stall_factor : 1.0;
                s.stall_f2 = sf * sf;
                hs[off + r] = s;
            }
            TM_HIP(ctx, hipMemcpyAsync(pr[i].cg, hs + off, pr[i].nrhs * sizeof(CGScalars),
                                       hipMemcpyHostToDevice, ctx->stream));
            off += pr[i].nrhs;
        }
        TM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    if (!par->use_x0)
        for (int i = 0; i < n; i++)
            TM_HIP(ctx, hipMemsetAsync(pr[i].x, 0, spinor_field_bytes(TM_FP64, pr[i].g->vh, nf, pr[i].nrhs),
                                       ctx->stream));
    if (mixed)
        for (int i = 0; i < n; i++)
            TM_HIP(ctx, hipMemsetAsync(pr[i].xlo, 0, spinor_field_bytes(TM_FP32, pr[i].g->vh, nf, pr[i].nrhs),
                                       ctx->stream));

    // initial residual r = c - A x (x = 0 or the guess), p = r
    void *rv[kMaxProblems], *pv[kMaxProblems], *mpv[kMaxProblems], *apv[kMaxProblems], *xv[kMaxProblems];
    for (int i = 0; i < n; i++) {
        rv[i] = mixed ? pr[i].rlo : pr[i].r64;
        pv[i] = mixed ? pr[i].plo : pr[i].p64;
        mpv[i] = mixed ? pr[i].mplo : pr[i].mp64;
        apv[i] = mixed ? pr[i].aplo : pr[i].ap64;
        xv[i] = mixed ? pr[i].xlo : pr[i].x;
    }
    const int lp = mixed ? inner : TM_FP64;
    const int xp = mixed ? TM_FP32 : TM_FP64;
    if (par->use_x0) {
        TM_TRY(true_residual(ctx, pr, pc, lp, rv, pv, FIN_STORE_RR));
    } else {
        // x = 0: r = p = c, no operator application needed
        BlasCall calls[kMaxProblems];
        for (int i = 0; i < n; i++)
            calls[i] = BlasCall{pr[i].g->vh, pr[i].nrhs, {pr[i].c, nullptr, rv[i], pv[i]}, FIN_STORE_RR,
                                pr[i].cg, pr[i].dres};
        TM_TRY(launch_blas_batch(ctx, OP_RESIDUAL, TM_FP64, lp, nf, calls, n));
    }

    // One CG iteration over all problems, every stage one batched launch:
    // M p (|M p|^2 -> alpha), then r -= alpha M^+ M p inside the last hop of
    // M^+ (|r|^2 -> beta; A p is never stored); the step x += alpha p is
    // taken by the pass that forms the next direction (xpay below).  With
    // TM_CG_FUSE=0: A p stored, then one BLAS pass x += alpha p, r -= alpha A p,
    // and the direction update alone.
    auto iteration_core = [&]() -> int {
        CGScalars *cgs[kMaxProblems];
        for (int i = 0; i < n; i++) cgs[i] = pr[i].cg;
        TM_TRY(mat_pc_batch(ctx, gs, mpv, (const void *const *)pv, nr, n, lp, pc, 0, FIN_ALPHA, cgs));
        if (ctx->cg_fuse)
            return mat_pc_batch(ctx, gs, rv, (const void *const *)mpv, nr, n, lp, pc, 1, FIN_BETA, cgs, true);
        TM_TRY(mat_pc_batch(ctx, gs, apv, (const void *const *)mpv, nr, n, lp, pc, 1, FIN_NONE, nullptr));
        BlasCall up[kMaxProblems];
        for (int i = 0; i < n; i++)
            up[i] = BlasCall{pr[i].g->vh, pr[i].nrhs, {xv[i], pv[i], rv[i], apv[i]}, FIN_BETA, pr[i].cg, nullptr};
        return launch_blas_batch(ctx, OP_CG_UPDATE, xp, lp, nf, up, n);
    };
    // p = r + beta p (beta of the CG recurrence, or of a residual replacement),
    // fused: x += alpha p first, from the same read of p (alpha is zero once
    // a reliable update has taken the step)
    auto xpay = [&]() -> int {
        BlasCall xp_[kMaxProblems];
        if (ctx->cg_fuse) {
            for (int i = 0; i < n; i++)
                xp_[i] = BlasCall{pr[i].g->vh, pr[i].nrhs, {xv[i], pv[i], rv[i], nullptr}, FIN_NONE, pr[i].cg,
                                  nullptr};
            return launch_blas_batch(ctx, OP_XPAY_X, xp, lp, nf, xp_, n);
        }
        for (int i = 0; i < n; i++)
            xp_[i] = BlasCall{pr[i].g->vh, pr[i].nrhs, {rv[i], pv[i], nullptr, nullptr}, FIN_NONE, pr[i].cg, nullptr};
        return launch_blas_batch(ctx, OP_XPAY, lp, lp, nf, xp_, n);
    };
    // reliable update: x += x_lo; r = c - A x in FP64 rounded into r_lo; beta = |r|^2 / |r_prev|^2
    // (fused iterations: the step of this iteration goes into x here as well,
    // x += x_lo + alpha p, and the residual replacement then sets alpha to
    // zero for the xpay)
    auto reliable_update = [&]() -> int {
        if (ctx->cg_fuse) {
            BlasCall up[kMaxProblems];
            for (int i = 0; i < n; i++)
                up[i] = BlasCall{pr[i].g->vh, pr[i].nrhs, {pr[i].x, pr[i].xlo, pv[i], nullptr}, FIN_NONE,
                                 pr[i].cg, nullptr};
            TM_TRY(launch_blas_batch(ctx, OP_ACCUM_STEP, TM_FP64, lp, nf, up, n));
            return true_residual(ctx, pr, pc, lp, rv, nullptr, FIN_RELIABLE);
        }
        BlasCall acc[kMaxProblems];
        for (int i = 0; i < n; i++)
            acc[i] = BlasCall{pr[i].g->vh, pr[i].nrhs, {pr[i].x, pr[i].xlo, nullptr, nullptr}, FIN_NONE,
                              nullptr, nullptr};
        TM_TRY(launch_blas_batch(ctx, OP_ACCUM_ZERO, TM_FP64, TM_FP32, nf, acc, n));
        return true_residual(ctx, pr, pc, lp, rv, nullptr, FIN_RELIABLE);
    };

    // Device-side control of every iteration (eager or captured):
    //   flags[0]  reliable-update gate (mixed: decided on the device each
    //             iteration, its launches gated by it)
    //   flags[1]  number of reliable updates taken
    //   flags[2]  run flag: some rhs still iterates; every launch of an
    //             iteration is gated by it, so iterations enqueued after
    //             convergence do nothing
    //   flags[3]  iterations that ran
    int *flags = nullptr;
    {
        int rc = TM_OK;
        flags = (int *)workspace(ctx, "cg_flags", 256, &rc);
        if (!flags) return rc;
        TM_HIP(ctx, hipMemsetAsync(flags, 0, 256, ctx->stream));
    }
    int *const upd_gate = flags, *const upd_count = flags + 1, *const run_flag = flags + 2,
              *const iter_count = flags + 3;
    RunArgs RA;
    memset(&RA, 0, sizeof(RA));
    DecideArgs D;
    memset(&D, 0, sizeof(D));
    RA.nprob = D.nprob = n;
    for (int i = 0; i < n; i++) {
        RA.nrhs[i] = D.nrhs[i] = pr[i].nrhs;
        RA.cg[i] = D.cg[i] = pr[i].cg;
    }
    RA.with_pending = mixed ? 1 : 0;
    RA.maxiter = par->maxiter;
    RA.run = run_flag;
    RA.iters = iter_count;
    D.delta2 = delta * delta;
    D.gate = upd_gate;
    D.count = upd_count;

    // Tune every hop the iterations launch before any launch is gated or
    // captured (the tuner times real launches and is skipped in both cases):
    // the inner operator and its dagger from p, and for reliable updates the
    // FP64 normal operator; the scratch vectors written are overwritten by
    // the first iteration.
    if (ctx->tuning) {
        TM_TRY(mat_pc_batch(ctx, gs, mpv, (const void *const *)pv, nr, n, lp, pc, 0, FIN_NONE, nullptr));
        TM_TRY(mat_pc_batch(ctx, gs, apv, (const void *const *)mpv, nr, n, lp, pc, 1, FIN_NONE, nullptr));
        if (mixed) {
            void *ys[kMaxProblems], *mids[kMaxProblems];
            const void *xs[kMaxProblems];
            for (int i = 0; i < n; i++) {
                ys[i] = pr[i].y;
                mids[i] = pr[i].mid;
                xs[i] = pr[i].c;
            }
            TM_TRY(normal_op64(ctx, pr, pc, ys, mids, xs));
        }
    }

    auto iteration = [&]() -> int {
        TM_HIP(ctx, launch_run(RA, ctx->stream));
        ctx->gate = run_flag;
        int rc = iteration_core();
        if (rc == TM_OK && mixed) {
            rc = (launch_decide(D, ctx->stream) == hipSuccess) ? TM_OK
                                                                : fail(ctx, TM_ERR_HIP, "decide launch");
            if (rc == TM_OK) {
                ctx->gate = upd_gate;
                rc = reliable_update();
                ctx->gate = run_flag;
            }
        }
        if (rc == TM_OK) rc = xpay();
        ctx->gate = nullptr;
        return rc;
    };

    GraphCache gc;
    const int gk = par->graph_iters;
    if (gk > 0) {
        TM_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
        int rc = TM_OK;
        for (int k = 0; k < gk && rc == TM_OK; k++) rc = iteration();
        ctx->gate = nullptr;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->stream, &graph);
        if (rc != TM_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(ctx, TM_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
        gc.graph = graph;
        TM_HIP(ctx, hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0));
    }

    // Host side: chunks of iterations (one graph, or check_every eager
    // iterations) are enqueued one ahead of the check of the previous chunk,
    // whose scalars and flags come back with one small asynchronous copy into
    // pinned memory; the chunk enqueued speculatively after convergence runs
    // gated and does nothing.
    int total_rhs = 0;
    for (auto &p : pr) total_rhs += p.nrhs;
    const size_t snap_bytes = (size_t)total_rhs * sizeof(CGScalars) + 4 * sizeof(int);
    char *snap[2];
    hipEvent_t snap_ev[2] = {nullptr, nullptr};
    {
        int rc = TM_OK;
        double *h = host_scratch(ctx, 2 * ((snap_bytes + 255) / 256) * 256 / sizeof(double), &rc);
        if (!h) return rc;
        snap[0] = (char *)h;
        snap[1] = snap[0] + (snap_bytes + 255) / 256 * 256;
        for (int k = 0; k < 2; k++) TM_HIP(ctx, hipEventCreateWithFlags(&snap_ev[k], hipEventDisableTiming));
    }
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard()
        {
            for (int k = 0; k < 2; k++)
                if (e[k]) (void)hipEventDestroy(e[k]);
        }
    } ev_guard{snap_ev};
    const int chunk = gk > 0 ? gk : check_every;
    auto enqueue_chunk = [&](int slot) -> int {
        if (gk > 0) {
            TM_HIP(ctx, hipGraphLaunch(gc.exec, ctx->stream));
        } else {
            for (int k = 0; k < chunk; k++) TM_TRY(iteration());
        }
        size_t off = 0;
        for (int i = 0; i < n; i++) {
            TM_HIP(ctx, hipMemcpyAsync(snap[slot] + off, pr[i].cg, pr[i].nrhs * sizeof(CGScalars),
                                       hipMemcpyDeviceToHost, ctx->stream));
            off += pr[i].nrhs * sizeof(CGScalars);
        }
        TM_HIP(ctx, hipMemcpyAsync(snap[slot] + off, flags, 4 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        TM_HIP(ctx, hipEventRecord(snap_ev[slot], ctx->stream));
        return TM_OK;
    };
    // copy a snapshot into sc / the flag counters
    int hflags[4] = {0, 0, 0, 0};
    std::vector<std::vector<CGScalars>> sc;
    auto unpack = [&](int slot) {
        sc.assign(n, {});
        size_t off = 0;
        for (int i = 0; i < n; i++) {
            const CGScalars *c = (const CGScalars *)(snap[slot] + off);
            sc[i].assign(c, c + pr[i].nrhs);
            off += pr[i].nrhs * sizeof(CGScalars);
        }
        memcpy(hflags, snap[slot] + off, sizeof(hflags));
    };
    auto all_inactive = [&]() {
        for (int i = 0; i < n; i++)
            for (int r = 0; r < pr[i].nrhs; r++)
                if (sc[i][r].active || (mixed && sc[i][r].pending)) return false;
        return true;
    };
    const int max_stalls = par->max_stalls == 0 ? 3 : par->max_stalls;
    phase.enter("tm_cg: iterations");
    int status = TM_OK;
    bool stalled = false;
    long enqueued = 0;            // iterations enqueued (an upper bound of those run)
    int slot = 0;
    bool in_flight = false;       // a chunk whose snapshot is not yet read
    for (;;) {
        bool launched = false;
        if (enqueued < par->maxiter) {
            TM_TRY(enqueue_chunk(slot));
            enqueued += chunk;
            launched = true;
        }
        if (!in_flight) {
            // the first chunk: nothing to check yet
            in_flight = launched;
            slot ^= 1;
            if (!launched) break;
            continue;
        }
        // check the previous chunk while this one runs
        const int prev = slot ^ 1;
        TM_HIP(ctx, hipEventSynchronize(snap_ev[prev]));
        unpack(prev);
        if (ctx->verbose) {
            // the largest iterated residual over the rhs still iterating
            double worst = 0.0;
            int live = 0;
            for (int i = 0; i < n; i++)
                for (int r = 0; r < pr[i].nrhs; r++) {
                    const CGScalars &s = sc[i][r];
                    if (!(s.active || (mixed && s.pending))) continue;
                    live++;
                    if (pr[i].cc[r] > 0) worst = std::max(worst, std::sqrt(s.rr / pr[i].cc[r]));
                }
            fprintf(stderr, "tm_cg: %d iterations, %d reliable updates, %d rhs iterating, max |r|/|c| %.3e\n",
                    hflags[3], mixed ? hflags[1] : 0, live, worst);
        }
        bool bad = false, stall = false;
        for (int i = 0; i < n; i++)
            for (int r = 0; r < pr[i].nrhs; r++) {
                const CGScalars &s = sc[i][r];
                if (!std::isfinite(s.rr) || !std::isfinite(s.alpha)) bad = true;
                if (mixed && max_stalls > 0 && s.stall >= max_stalls) stall = true;
            }
        if (bad) {
            (void)hipStreamSynchronize(ctx->stream);
            return fail(ctx, TM_ERR_NAN, "non-finite residual after %d iterations", hflags[3]);
        }
        bool done = false;
        if (stall) {
            stalled = true;
            done = true;
        } else if (all_inactive()) {
            if (mixed) {
                done = true;    // the verifying reliable update ran on the device
            } else {
                // plain CG: verify with the true residual (after the chunk in
                // flight, which runs gated), restart from it if it is not small enough
                TM_TRY(true_residual(ctx, pr, pc, TM_FP64, rv, pv, FIN_STORE_RR));
                TM_TRY(read_scalars(ctx, pr, sc));
                done = all_inactive();
                if (!done) {
                    // the chunk enqueued above was a no-op: iterate afresh
                    launched = false;
                    in_flight = false;
                }
            }
        }
        if (done) break;
        if (!launched && in_flight && enqueued >= par->maxiter) {
            status = TM_NOT_CONVERGED;
            break;
        }
        slot ^= 1;
    }
    // the last snapshot of the device state (all work enqueued so far done)
    phase.enter("tm_cg: final residuals");
    TM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    TM_TRY(read_scalars(ctx, pr, sc));
    {
        TM_HIP(ctx, hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, ctx->stream));
        TM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    if (status == TM_OK && !stalled && !all_inactive()) status = TM_NOT_CONVERGED;
    const int iters = hflags[3];
    const int updates = mixed ? hflags[1] : 0;
    // mixed: the verifying update left x and rr consistent; plain: the
    // verification above did
    bool true_valid = (status == TM_OK && !stalled);
    if (mixed && (status == TM_NOT_CONVERGED || stalled)) {
        BlasCall acc[kMaxProblems];
        for (int i = 0; i < n; i++)
            acc[i] = BlasCall{pr[i].g->vh, pr[i].nrhs, {pr[i].x, pr[i].xlo, nullptr, nullptr}, FIN_NONE,
                              nullptr, nullptr};
        TM_TRY(launch_blas_batch(ctx, OP_ACCUM_ZERO, TM_FP64, TM_FP32, nf, acc, n));
        true_valid = false;
    }
    if (stalled) {
        TM_HIP(ctx, hipStreamSynchronize(ctx->stream));
        int off = 0;
        for (int i = 0; i < n; i++)
            for (int r = 0; r < pr[i].nrhs; r++, off++) {
                res[off].iters = iters;
                res[off].reliable_updates = updates;
            }
        return kStalled;
    }
    TM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();

    // reported residuals, recomputed in FP64 from x
    std::vector<std::vector<double>> rn, rp, bb;
    {
        void *r64[kMaxProblems];
        for (int i = 0; i < n; i++) {
            int rc = TM_OK;
            char name[64];
            snprintf(name, sizeof(name), "cg_rtrue_%d", i);
            r64[i] = workspace(ctx, name, spinor_field_bytes(TM_FP64, pr[i].g->vh, nf, pr[i].nrhs), &rc);
            if (!r64[i]) return rc;
        }
        if (true_valid) {
            // the last step computed the FP64 residual of this x (in the scalars)
            rn.assign(n, {});
            for (int i = 0; i < n; i++)
                for (int r = 0; r < pr[i].nrhs; r++) rn[i].push_back(sc[i][r].rr);
        } else {
            TM_TRY(true_residual(ctx, pr, pc, TM_FP64, r64, nullptr, FIN_NONE));
            TM_TRY(norms_fp64(ctx, pr, r64, rn));
        }
        // |b - M x|: y = M x, r = b - y  (MATDAG_MAT: y = M^+ M x, left in y by the
        // residual above)
        void *ys[kMaxProblems];
        const void *xs[kMaxProblems];
        for (int i = 0; i < n; i++) {
            ys[i] = pr[i].y;
            xs[i] = pr[i].x;
        }
        if (par->solution != TM_SOLUTION_MATDAG_MAT || true_valid)
            TM_TRY(par->solution != TM_SOLUTION_MATDAG_MAT
                       ? mat_pc_batch(ctx, gs, ys, xs, nr, n, TM_FP64, pc, 0, FIN_NONE, nullptr)
                       : normal_op64(ctx, pr, pc, ys, r64, xs));
        BlasCall calls[kMaxProblems];
        for (int i = 0; i < n; i++)
            calls[i] = BlasCall{pr[i].g->vh, pr[i].nrhs, {pr[i].b, pr[i].y, r64[i], nullptr}, FIN_NONE,
                                nullptr, nullptr};
        TM_TRY(launch_blas_batch(ctx, OP_RESIDUAL, TM_FP64, TM_FP64, nf, calls, n));
        TM_TRY(norms_fp64(ctx, pr, r64, rp));
        void *bv[kMaxProblems];
        for (int i = 0; i < n; i++) bv[i] = const_cast<void *>(pr[i].b);
        TM_TRY(norms_fp64(ctx, pr, bv, bb));
    }
    int off = 0;
    for (int i = 0; i < n; i++)
        for (int r = 0; r < pr[i].nrhs; r++, off++) {
            tm_cg_result &o = res[off];
            o.iters = iters;
            o.reliable_updates = updates;
            o.true_rel_res_normal = pr[i].cc[r] > 0 ? std::sqrt(rn[i][r] / pr[i].cc[r]) : 0.0;
            o.true_rel_res_pc = bb[i][r] > 0 ? std::sqrt(rp[i][r] / bb[i][r]) : 0.0;
            o.seconds = secs;
            o.true_rel_res_full = -1.0;
            o.precision_fallbacks = 0;
            // the last iterated residuals of this rhs, oldest first
            const CGScalars &s = sc[i][r];
            const int len = std::min(s.niter, kHistory);
            o.history_len = len;
            for (int j = 0; j < len; j++) {
                const double h = s.hist[(s.niter - len + j) % kHistory];
                o.res_history[j] = pr[i].cc[r] > 0 ? std::sqrt(h / pr[i].cc[r]) : 0.0;
            }
            if (!std::isfinite(o.true_rel_res_normal)) status = fail(ctx, TM_ERR_NAN, "non-finite residual");
            if (status == TM_OK && o.true_rel_res_normal > par->tol * 1.0000001) status = TM_NOT_CONVERGED;
            if (ctx->verbose)
                fprintf(stderr, "tm_cg: problem %d rhs %d: %d iterations, %d reliable updates, true |r|/|c| "
                        "%.3e (preconditioned system %.3e), %.4f s\n",
                        i, r, o.iters, o.reliable_updates, o.true_rel_res_normal, o.true_rel_res_pc, o.seconds);
        }
    return status;
}

// cg_run with the precision fallback: a mixed solve whose reliable updates
// stopped making progress continues from its x with the next wider inner
// format (FP16 / BF16 -> FP32 -> FP64); iterations, updates and time add up.
int cg_solve(tm_ctx *ctx, std::vector<CGProblem> &pr, const tm_cg_params *par, tm_cg_result *res)
{
    const auto t0 = std::chrono::steady_clock::now();
    tm_cg_params p = *par;
    int total = 0;
    for (auto &q : pr) total += q.nrhs;
    int iters = 0, updates = 0, fallbacks = 0;
    for (;;) {
        const int rc = cg_run(ctx, pr, &p, res);
        if (rc < 0) return rc;
        iters += res[0].iters;
        updates += res[0].reliable_updates;
        if (rc != kStalled) {
            const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            for (int k = 0; k < total; k++) {
                res[k].iters = iters;
                res[k].reliable_updates = updates;
                res[k].precision_fallbacks = fallbacks;
                res[k].seconds = secs;
            }
            return rc;
        }
        fallbacks++;
        int next = (p.inner == TM_FP16 || p.inner == TM_BF16) ? TM_FP32 : TM_FP64;
        for (auto &q : pr)
            if (!q.g->links[next][0]) next = TM_FP64;   // the wider format is not built
        p.inner = next;
        p.use_x0 = 1;
        p.maxiter = std::max(1, p.maxiter - res[0].iters);
    }
}

int check_cg(tm_ctx *ctx, const tm_gauge *g, const tm_cg_params *par)
{
    if (!par) return fail(ctx, TM_ERR_ARG, "null cg params");
    if (!(par->tol > 0) || par->maxiter < 1) return fail(ctx, TM_ERR_ARG, "tol must be > 0, maxiter >= 1");
    if (par->pc != TM_PC_ASYM && par->pc != TM_PC_SYM) return fail(ctx, TM_ERR_ARG, "bad pc type");
    if (par->outer != TM_FP64) return fail(ctx, TM_ERR_PREC, "outer precision must be FP64");
    if (!valid_prec(par->inner)) return fail(ctx, TM_ERR_PREC, "bad inner precision");
    if (par->nrhs < 1 || par->nrhs > 64) return fail(ctx, TM_ERR_LIMIT, "nrhs must be in 1..64");
    if (par->graph_iters < 0 || par->graph_iters > 256) return fail(ctx, TM_ERR_ARG, "graph_iters in 0..256");
    if (par->solution != TM_SOLUTION_MAT && par->solution != TM_SOLUTION_MATDAG_MAT)
        return fail(ctx, TM_ERR_ARG, "bad solution type");
    Phase phase;
    phase.enter("tm_solve");
    TM_TRY(check_gauge_prec(ctx, g, TM_FP64));
    TM_TRY(check_gauge_prec(ctx, g, par->inner));
    return TM_OK;
}

}  // namespace

namespace {
// Graph capture needs a stream other than the null stream: for the duration of
// a solve with graph_iters > 0 the context's work moves to a private stream
// (ordered after the caller's stream, and the caller's stream after it).
struct StreamSwap {
    tm_ctx *ctx;
    hipStream_t saved;
    bool active = false;
    StreamSwap(tm_ctx *c, bool want) : ctx(c), saved(c->stream)
    {
        if (!want || c->stream != nullptr) return;
        if (!c->own_stream && hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess)
            return;
        (void)hipStreamSynchronize(saved);
        c->stream = c->own_stream;
        active = true;
    }
    ~StreamSwap()
    {
        if (!active) return;
        (void)hipStreamSynchronize(ctx->stream);
        ctx->stream = saved;
    }
};
}  // namespace

int tm_cg(tm_ctx *ctx, void *x_e, const void *b_e, const tm_gauge *g, const tm_cg_params *par,
          tm_cg_result *res)
{
    if (!ctx) return TM_ERR_ARG;
    TM_TRY(check_cg(ctx, g, par));
    if (!x_e || !b_e || !res) return fail(ctx, TM_ERR_ARG, "null pointer");
    if (x_e == b_e) return fail(ctx, TM_ERR_ARG, "x and b must not alias");
    std::vector<CGProblem> pr(1);
    pr[0] = CGProblem{};
    pr[0].g = g;
    pr[0].nrhs = par->nrhs;
    pr[0].x = x_e;
    pr[0].b = b_e;
    StreamSwap sw(ctx, par->graph_iters > 0);
    return cg_solve(ctx, pr, par, res);
}

int tm_cg_batched(tm_ctx *ctx, int nproblems, const tm_gauge *const *g, void *const *x_e,
                  const void *const *b_e, const int *nrhs, const tm_cg_params *par, tm_cg_result *res)
{
    if (!ctx) return TM_ERR_ARG;
    if (nproblems < 1 || nproblems > kMaxProblems)
        return fail(ctx, TM_ERR_LIMIT, "nproblems must be in 1..%d", kMaxProblems);
    if (!g || !x_e || !b_e || !nrhs || !res) return fail(ctx, TM_ERR_ARG, "null pointer");
    std::vector<CGProblem> pr(nproblems);
    for (int i = 0; i < nproblems; i++) {
        tm_cg_params pi = *par;
        pi.nrhs = nrhs[i];
        TM_TRY(check_cg(ctx, g[i], &pi));
        if (!x_e[i] || !b_e[i]) return fail(ctx, TM_ERR_ARG, "null field");
        if (g[i]->nf != g[0]->nf || g[i]->recon != g[0]->recon)
            return fail(ctx, TM_ERR_ARG, "batched problems must share flavour count and recon");
        pr[i] = CGProblem{};
        pr[i].g = g[i];
        pr[i].nrhs = nrhs[i];
        pr[i].x = x_e[i];
        pr[i].b = b_e[i];
    }
    StreamSwap sw(ctx, par->graph_iters > 0);
    return cg_solve(ctx, pr, par, res);
}

namespace {

// FP64 field of one parity from the solver's own workspace
void *solve_field(tm_ctx *ctx, const char *tag, const tm_gauge *g, int nrhs, int *rc)
{
    char name[64];
    snprintf(name, sizeof(name), "solve_%s", tag);
    return workspace(ctx, name, spinor_field_bytes(TM_FP64, g->vh, g->nf, nrhs), rc);
}

// |a - b|^2 per rhs (b may be null: |a|^2) of FP64 fields into host h[nrhs];
// d receives a - b.
int diff_norm2(tm_ctx *ctx, const tm_gauge *g, const void *a, const void *b, void *d, int nrhs,
               std::vector<double> &h)
{
    int rc = TM_OK;
    double *dres = (double *)workspace(ctx, "solve_norms", (size_t)nrhs * sizeof(double), &rc);
    if (!dres) return rc;
    double *hs = host_scratch(ctx, nrhs, &rc);
    if (!hs) return rc;
    BlasCall c{g->vh, nrhs, {a, b, d, nullptr}, FIN_STORE, nullptr, dres};
    TM_TRY(blas1(ctx, OP_RESIDUAL, TM_FP64, TM_FP64, g->nf, c));
    TM_HIP(ctx, hipMemcpyAsync(hs, dres, nrhs * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    TM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    h.assign(hs, hs + nrhs);
    return TM_OK;
}

// out = M in (dagger: M^+ in) on both parities, FP64:
//   out_e = R in_e - kappa D_eo in_o,  out_o = R in_o - kappa D_oe in_e
int full_op64(tm_ctx *ctx, const tm_gauge *g, void *oe, void *oo, const void *ie, const void *io,
              int dagger, int nrhs)
{
    const double k = -g->p.kappa;
    TM_TRY(hop1(ctx, HopCall{g, TM_FP64, 0, dagger, 0, TM_EPI_RX_PLUS_KD, io, oe, ie, k, nrhs,
                             FIN_NONE, nullptr, nullptr}));
    return hop1(ctx, HopCall{g, TM_FP64, 1, dagger, 0, TM_EPI_RX_PLUS_KD, ie, oo, io, k, nrhs,
                             FIN_NONE, nullptr, nullptr});
}

// Accumulates one CG run's report into the solve's report.
void add_report(tm_cg_result *acc, const tm_cg_result *r, int nrhs)
{
    for (int i = 0; i < nrhs; i++) {
        acc[i].iters += r[i].iters;
        acc[i].reliable_updates += r[i].reliable_updates;
        acc[i].precision_fallbacks += r[i].precision_fallbacks;
        acc[i].true_rel_res_normal = r[i].true_rel_res_normal;
        acc[i].true_rel_res_pc = r[i].true_rel_res_pc;
        acc[i].history_len = r[i].history_len;
        for (int j = 0; j < r[i].history_len; j++) acc[i].res_history[j] = r[i].res_history[j];
    }
}

// CG on one preconditioned system: x solves A x = b (solution MAT) or
// A^+ A x = b (MATDAG_MAT).  With the direct solve type a MAT solve is
// restarted from its x, with the normal tolerance scaled down, until
// |b - A x| <= tol |b| for every rhs (at most six runs, normal tolerance
// >= 1e-15).
int solve_pc(tm_ctx *ctx, const tm_gauge *g, void *x, const void *b, const tm_solve_params *par,
             int solution, tm_cg_result *acc, int *status)
{
    const int nrhs = par->cg.nrhs;
    tm_cg_params q = par->cg;
    q.solution = solution;
    q.use_x0 = 0;
    std::vector<tm_cg_result> r(nrhs);
    std::vector<CGProblem> pr(1);
    for (int run = 0;; run++) {
        pr[0] = CGProblem{};
        pr[0].g = g;
        pr[0].nrhs = nrhs;
        pr[0].x = x;
        pr[0].b = b;
        const int rc = cg_solve(ctx, pr, &q, r.data());
        if (rc < 0) return rc;
        add_report(acc, r.data(), nrhs);
        if (rc == TM_NOT_CONVERGED) {
            *status = TM_NOT_CONVERGED;
            return TM_OK;
        }
        if (par->solve_type != TM_SOLVE_DIRECT_PC || solution != TM_SOLUTION_MAT) return TM_OK;
        double worst = 0.0;
        for (int i = 0; i < nrhs; i++) worst = std::max(worst, r[i].true_rel_res_pc / par->cg.tol);
        if (worst <= 1.0) return TM_OK;
        int used = 0;
        for (int i = 0; i < nrhs; i++) used = std::max(used, acc[i].iters);
        if (run == 5 || q.tol <= 1e-15 || used >= par->cg.maxiter) {
            *status = TM_NOT_CONVERGED;
            return TM_OK;
        }
        q.tol = std::max(1e-15, q.tol / worst * 0.5);
        q.use_x0 = 1;
        q.maxiter = par->cg.maxiter - used;
    }
}

}  // namespace

int tm_solve(tm_ctx *ctx, void *x_e, void *x_o, const void *b_e, const void *b_o, const tm_gauge *g,
             const tm_solve_params *par, tm_cg_result *res)
{
    if (!ctx) return TM_ERR_ARG;
    if (!par) return fail(ctx, TM_ERR_ARG, "null solve params");
    TM_TRY(check_cg(ctx, g, &par->cg));
    if (!x_e || !x_o || !b_e || !b_o || !res) return fail(ctx, TM_ERR_ARG, "null pointer");
    if (x_e == x_o || x_e == b_e || x_e == b_o || x_o == b_e || x_o == b_o || b_e == b_o)
        return fail(ctx, TM_ERR_ARG, "solution and source halves must be distinct buffers");
    if (par->solve_type != TM_SOLVE_NORMOP_PC && par->solve_type != TM_SOLVE_DIRECT_PC)
        return fail(ctx, TM_ERR_ARG, "bad solve type");
    if (par->solution != TM_SOLUTION_MAT && par->solution != TM_SOLUTION_MATDAG_MAT)
        return fail(ctx, TM_ERR_ARG, "bad solution type");
    Phase phase;
    phase.enter("tm_solve");
    const auto t0 = std::chrono::steady_clock::now();
    const int nrhs = par->cg.nrhs;
    const int pc = par->cg.pc;
    const double kappa = g->p.kappa;
    StreamSwap sw(ctx, par->cg.graph_iters > 0);
    for (int i = 0; i < nrhs; i++) res[i] = tm_cg_result{};
    int status = TM_OK;
    int rc = TM_OK;
    void *e0 = solve_field(ctx, "e0", g, nrhs, &rc);
    void *e1 = solve_field(ctx, "e1", g, nrhs, &rc);
    void *o0 = solve_field(ctx, "o0", g, nrhs, &rc);
    if (!e0 || !e1 || !o0) return rc;
    // source of the M x = y stage: b itself, or y from the M^+ y = b stage
    const void *src_e = b_e, *src_o = b_o;
    void *y_e = nullptr, *y_o = nullptr;
    if (par->solution == TM_SOLUTION_MATDAG_MAT) {
        y_e = solve_field(ctx, "ye", g, nrhs, &rc);
        y_o = solve_field(ctx, "yo", g, nrhs, &rc);
        if (!y_e || !y_o) return rc;
        // c = b_e + kappa D^+_eo R_oo^-+ b_o   (e0)
        TM_TRY(hop1(ctx, HopCall{g, TM_FP64, 0, 1, 1, TM_EPI_X_PLUS_KD, b_o, e0, b_e, kappa, nrhs,
                                 FIN_NONE, nullptr, nullptr}));
        // z: A^+ A z = c   (x_e serves as z)
        TM_TRY(solve_pc(ctx, g, x_e, e0, par, TM_SOLUTION_MATDAG_MAT, res, &status));
        // y_e = A z, sym: R_ee^-+ A z
        if (pc == TM_PC_ASYM) {
            TM_TRY(mat_pc_batch(ctx, &g, &y_e, (const void *const *)&x_e, &nrhs, 1, TM_FP64, pc, 0,
                                FIN_NONE, nullptr));
        } else {
            TM_TRY(mat_pc_batch(ctx, &g, &e1, (const void *const *)&x_e, &nrhs, 1, TM_FP64, pc, 0,
                                FIN_NONE, nullptr));
            TM_HIP(ctx, twist_apply(TM_FP64, g->nf, sptr(y_e, TM_FP64, g->vh, g->nf, nrhs),
                                    sptr(e1, TM_FP64, g->vh, g->nf, nrhs), g->vh, nrhs,
                                    make_twist(g->p, 1), 1, ctx->stream, g->clov_of(TM_FP64, 0)));
        }
        // y_o = R_oo^-+ (b_o + kappa D^+_oe y_e)
        TM_TRY(hop1(ctx, HopCall{g, TM_FP64, 1, 1, 0, TM_EPI_TWINV_X_PLUS_KD, y_e, y_o, b_o, kappa,
                                 nrhs, FIN_NONE, nullptr, nullptr}));
        src_e = y_e;
        src_o = y_o;
    }
    // M x = src: b^ = src_e + kappa D_eo R_oo^-1 src_o (sym: R_ee^-1 of it)   (e0)
    TM_TRY(hop1(ctx, HopCall{g, TM_FP64, 0, 0, 1,
                             pc == TM_PC_SYM ? TM_EPI_TWINV_X_PLUS_KD : TM_EPI_X_PLUS_KD, src_o, e0,
                             src_e, kappa, nrhs, FIN_NONE, nullptr, nullptr}));
    TM_TRY(solve_pc(ctx, g, x_e, e0, par, TM_SOLUTION_MAT, res, &status));
    // x_o = R_oo^-1 (src_o + kappa D_oe x_e)
    TM_TRY(hop1(ctx, HopCall{g, TM_FP64, 1, 0, 0, TM_EPI_TWINV_X_PLUS_KD, x_e, x_o, src_o, kappa, nrhs,
                             FIN_NONE, nullptr, nullptr}));
    // residual of the full system: v = M x (e1, o0); MATDAG_MAT: v = M^+ M x (e0, o1)
    const void *ve = e1, *vo = o0;
    TM_TRY(full_op64(ctx, g, e1, o0, x_e, x_o, 0, nrhs));
    if (par->solution == TM_SOLUTION_MATDAG_MAT) {
        void *o1 = solve_field(ctx, "o1", g, nrhs, &rc);
        if (!o1) return rc;
        TM_TRY(full_op64(ctx, g, e0, o1, e1, o0, 1, nrhs));
        ve = e0;
        vo = o1;
    }
    void *d = y_e ? y_e : solve_field(ctx, "d", g, nrhs, &rc);
    if (!d) return rc;
    std::vector<double> re, ro, be, bo;
    TM_TRY(diff_norm2(ctx, g, b_e, ve, d, nrhs, re));
    TM_TRY(diff_norm2(ctx, g, b_o, vo, d, nrhs, ro));
    TM_TRY(diff_norm2(ctx, g, b_e, nullptr, d, nrhs, be));
    TM_TRY(diff_norm2(ctx, g, b_o, nullptr, d, nrhs, bo));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < nrhs; i++) {
        const double bb = be[i] + bo[i];
        res[i].true_rel_res_full = bb > 0 ? std::sqrt((re[i] + ro[i]) / bb) : 0.0;
        res[i].seconds = secs;
        if (!std::isfinite(res[i].true_rel_res_full)) return fail(ctx, TM_ERR_NAN, "non-finite residual");
    }
    return status;
}

int tm_force(tm_ctx *ctx, void *F_dev, int force_prec, const void *X_e, const tm_gauge *g,
             int prec, int pc, double coeff, int accumulate, void *G_dev)
{
    if (!ctx) return TM_ERR_ARG;
    TM_TRY(check_gauge_prec(ctx, g, prec));
    if (prec != TM_FP64 && prec != TM_FP32)
        return fail(ctx, TM_ERR_PREC, "force fields must be FP64 or FP32");
    if (force_prec != TM_FP64 && force_prec != TM_FP32)
        return fail(ctx, TM_ERR_PREC, "force output must be FP64 or FP32");
    if (!F_dev || !X_e) return fail(ctx, TM_ERR_ARG, "null pointer");
    if (pc != TM_PC_ASYM && pc != TM_PC_SYM) return fail(ctx, TM_ERR_ARG, "bad pc type");
    if (!std::isfinite(coeff)) return fail(ctx, TM_ERR_ARG, "non-finite coeff");
    if (g->recon != 12 && g->recon != 18)
        return fail(ctx, TM_ERR_ARG, "the force kernel reads 12- or 18-real links");
    if (g->clover()) return fail(ctx, TM_ERR_ARG, "no force for the twisted-clover operator");
    int rc = TM_OK;
    const size_t fb = spinor_field_bytes(prec, g->vh, g->nf, 1);
    void *Y = workspace(ctx, "force_y", fb, &rc);
    void *Ae = pc == TM_PC_SYM ? workspace(ctx, "force_ae", fb, &rc) : Y;
    void *Zo = workspace(ctx, "force_z", fb, &rc);
    void *Wo = workspace(ctx, "force_w", fb, &rc);
    if (!Y || !Ae || !Zo || !Wo) return rc;
    // Y = M X
    const int one = 1;
    TM_TRY(mat_pc_batch(ctx, &g, &Y, &X_e, &one, 1, prec, pc, 0, FIN_NONE, nullptr));
    // A_e = Y (asym) or R_ee^-+ Y (sym)
    if (pc == TM_PC_SYM)
        TM_HIP(ctx, twist_apply(prec, g->nf, sptr(Ae, prec, g->vh, g->nf, 1), sptr(Y, prec, g->vh, g->nf, 1),
                                g->vh, 1, make_twist(g->p, 1), 1, ctx->stream));
    // Z_o = R_oo^-1 D_oe X;   W_o = R_oo^-+ (D^+)_oe A_e
    TM_TRY(hop1(ctx, HopCall{g, prec, 1, 0, 0, TM_EPI_TWINV, X_e, Zo, nullptr, 0.0, 1, FIN_NONE,
                             nullptr, nullptr}));
    TM_TRY(hop1(ctx, HopCall{g, prec, 1, 1, 0, TM_EPI_TWINV, Ae, Wo, nullptr, 0.0, 1, FIN_NONE,
                             nullptr, nullptr}));
    SpinorPtr A[2] = {sptr(Ae, prec, g->vh, g->nf, 1), sptr(Wo, prec, g->vh, g->nf, 1)};
    SpinorPtr B[2] = {sptr(X_e, prec, g->vh, g->nf, 1), sptr(Zo, prec, g->vh, g->nf, 1)};
    TM_HIP(ctx, force_launch(prec, g->nf, force_prec, F_dev, G_dev, g->links[prec][0], g->links[prec][1],
                             g->recon, A, B, g->p.dims, g->vh, g->p.t_antiperiodic ? -1.0 : 1.0, coeff,
                             accumulate ? 1 : 0, g->p.kappa, ctx->stream));
    return TM_OK;
}

}  // extern "C"
