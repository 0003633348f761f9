// Sanitizer driver of the library's host layer (test infrastructure): with no
// device present it drives the argument validation of every entry point that
// validates before device work, the launch planner and the error strings,
// under AddressSanitizer / UndefinedBehaviorSanitizer.
#include <cstdio>
#include <cstring>

#include "tm.h"

static int failures = 0;
#define EXPECT(cond)                                                  \
    do {                                                              \
        if (!(cond)) {                                                \
            std::printf("failed at line %d: %s\n", __LINE__, #cond);  \
            failures++;                                               \
        }                                                             \
    } while (0)

int main()
{
    for (int code = -12; code <= 3; code++) EXPECT(tm_error_string(code) != nullptr);
    tm_ctx *ctx = nullptr;
    EXPECT(tm_ctx_create(&ctx, nullptr) == TM_OK && ctx);
    EXPECT(tm_ctx_create(nullptr, nullptr) == TM_ERR_ARG);
    EXPECT(tm_set_tuning(ctx, 1) == TM_OK);

    tm_params p;
    std::memset(&p, 0, sizeof(p));
    const int dims[4] = {4, 4, 4, 8};
    std::memcpy(p.dims, dims, sizeof(dims));
    p.kappa = 0.16;
    p.mu = 0.1;
    p.flavor = TM_TWIST_NDEG;
    p.epsilon = 0.2;
    p.t_antiperiodic = 1;
    for (int prec = 0; prec < 4; prec++)
        for (int nrhs = 1; nrhs <= 3; nrhs++) EXPECT(tm_spinor_bytes(&p, (tm_prec)prec, nrhs) > 0);
    EXPECT(tm_spinor_bytes(&p, (tm_prec)7, 1) == 0);
    EXPECT(tm_spinor_bytes(nullptr, TM_FP32, 1) == 0);

    // gauge creation: bad extents, bad recon, singular twist, null pointers
    tm_gauge *g = nullptr;
    const void *dummy = reinterpret_cast<const void *>(0x1000);
    p.dims[1] = 5;
    EXPECT(tm_gauge_create(ctx, &g, dummy, &p, 12, 3) == TM_ERR_DIMS);
    EXPECT(std::strlen(tm_last_error(ctx)) > 0);
    p.dims[1] = 4;
    EXPECT(tm_gauge_create(ctx, &g, dummy, &p, 11, 3) == TM_ERR_ARG);
    EXPECT(tm_gauge_create(ctx, &g, nullptr, &p, 12, 3) == TM_ERR_ARG);
    EXPECT(tm_gauge_create(ctx, nullptr, dummy, &p, 12, 3) == TM_ERR_ARG);
    tm_params q = p;
    q.mu = 0.0;
    q.epsilon = 1.0 / (2 * q.kappa);    // b = 1: 1 + a^2 - b^2 = 0
    EXPECT(tm_gauge_create(ctx, &g, dummy, &q, 12, 3) == TM_ERR_SINGULAR);

    // operator calls with a null gauge / null fields
    void *f = reinterpret_cast<void *>(0x2000);
    EXPECT(tm_mat_pc(ctx, f, dummy, nullptr, TM_FP32, TM_PC_ASYM, 0, 1) < 0);
    EXPECT(tm_dslash(ctx, f, dummy, nullptr, TM_FP32, 0, 0, 0, TM_EPI_NONE, nullptr, 0.0, 1) < 0);
    tm_cg_params cp;
    std::memset(&cp, 0, sizeof(cp));
    tm_cg_result res[2];
    EXPECT(tm_cg(ctx, f, dummy, nullptr, &cp, res) < 0);
    EXPECT(tm_cg(ctx, f, dummy, nullptr, nullptr, res) < 0);

    // launch planner
    unsigned dyn = 0;
    for (int bs = 64; bs <= 256; bs *= 2)
        for (int w = 0; w <= 4; w++) {
            const int rc = tm_plan_hop_lds(bs, w, 0, 160u << 10, 160u << 10, 64, &dyn);
            EXPECT(rc == TM_OK);
            EXPECT(dyn + 64 <= (160u << 10));
        }
    EXPECT(tm_plan_hop_lds(256, 1, 0, 160u << 10, 64u << 10, 0, &dyn) == TM_ERR_LIMIT);
    EXPECT(tm_plan_hop_lds(96, 1, 0, 160u << 10, 160u << 10, 0, &dyn) == TM_ERR_ARG);
    EXPECT(tm_plan_hop_lds(256, 1, 0, 160u << 10, 160u << 10, 0, nullptr) == TM_ERR_ARG);

    EXPECT(tm_ctx_destroy(ctx) == TM_OK);
    EXPECT(tm_ctx_destroy(nullptr) == TM_ERR_ARG);
    std::printf("abi driver: %d failures\n", failures);
    return failures ? 1 : 0;
}
