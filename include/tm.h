/*
 * tm.h - C ABI of an MI355X-native library for the even-odd preconditioned
 * Wilson twisted-mass Dirac operator (Strelchenko, Alexandrou, Koutsou,
 * Vaquero, "Implementation of the twisted mass fermion operator in the QUDA
 * library", LATTICE 2013, arXiv:1311.4462).
 *
 * Operator conventions (the paper leaves these open; every entry point follows
 * them):
 *   - Lattice extents dims = {Lx, Ly, Lz, Lt}, all even and >= 2.  Site
 *     lex = x + Lx*(y + Ly*(z + Lz*t)); parity (x+y+z+t) & 1, even = 0;
 *     checkerboard index cb = lex >> 1.
 *   - Gamma matrices of the non-relativistic basis of Sec. 2, in 2x2 blocks
 *     g_k = [[0, i s_k], [-i s_k, 0]], g_4 = diag(1, 1, -1, -1),
 *     g5 = g1 g2 g3 g4 = [[0, 1], [1, 0]].
 *   - Hop (Wilson term of Eq. 2.1, r = 1):
 *       (D psi)(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu),
 *     periodic in x, y, z; if t_antiperiodic, hops across t = Lt-1 <-> 0 get -1.
 *     D^+ swaps the two projectors.
 *   - M = R - kappa D (Eq. 2.1 times 2 kappa), R = 1 + i a g5 t3 + b t1 with
 *     a = 2 kappa mu, b = 2 kappa epsilon; one flavour: R = 1 +- i a g5
 *     (TM_TWIST_PLUS / TM_TWIST_MINUS, Sec. 2.2).  Flavour 0 has t3 = +1.
 *     R^-1 = (1 - i a g5 t3 - b t1) / (1 + a^2 - b^2); R^+ = R(-mu, eps).
 *   - Preconditioned even-even operators: asym = R_ee - kappa^2 D_eo R_oo^-1 D_oe
 *     (Eq. 2.2), sym = 1 - kappa^2 R_ee^-1 D_eo R_oo^-1 D_oe (Eq. 2.3).
 *
 * Native field layouts (device memory, owned by the caller):
 *   spinor, one parity, nrhs right-hand sides, nf flavours (1, or 2 for the
 *   doublet): chunks [rhs][flavour][chunk][cb], each chunk holding
 *   consecutive (spin, colour) complex numbers k = 3*spin + colour:
 *       TM_FP64: 16-byte chunks of 1 complex  (12 chunks per site)
 *       TM_FP32: 16-byte chunks of 2 complex  (6 chunks)
 *       TM_FP16 / TM_BF16: 16-byte chunks of 4 complex (3 chunks), followed
 *       (at a 256-byte aligned offset) by a float scale per [rhs][flavour][cb];
 *       stored value = true value / scale, scale = max |real component| of
 *       the site's 24 reals for that flavour.
 *   Spin components 0, 1 (the "upper" pair, elements 0-5) occupy the first
 *   half of the site's bytes, so a time hop reads only half of a neighbour.
 *   Packed links (library owned): per parity [mu][cb] rows of 16 bytes, then
 *   narrower rows for what does not fill 16 bytes; 12-real storage keeps rows
 *   0 and 1 of each link, 8-real storage four complex slots (FP32: two rows,
 *   FP16/BF16: one row).
 *   Canonical (host-side exchange) layout, complex128, full lattice:
 *       spinor [nrhs][lex][nf][4][3], links [mu][lex][3][3] (row-major).
 *
 * Enumerated arguments are passed as int holding a value of the named enum
 * (prec: tm_prec, pc: tm_pc, epi: tm_epilogue); other values are rejected.
 *
 * Errors: every call returns TM_OK (0), an error (< 0) or the warning
 * TM_NOT_CONVERGED (> 0).  Nothing aborts and no exception crosses the ABI.
 * Arguments are validated before any device work; tm_last_error() returns a
 * message for the last failing call on a context.  All device work is
 * enqueued on the context's stream and is asynchronous unless stated.
 */
#ifndef TM_H
#define TM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TM_OK = 0,
    TM_NOT_CONVERGED = 1,
    TM_ERR_ARG = -1,       /* null pointer, bad enum, size mismatch           */
    TM_ERR_DIMS = -2,      /* an extent is odd or < 2                         */
    TM_ERR_PARITY = -3,    /* parity not 0 / 1                                */
    TM_ERR_PREC = -4,      /* precision not built for this gauge / operation  */
    TM_ERR_SINGULAR = -5,  /* |1 + a^2 - b^2| < 1e-12: R has no inverse       */
    TM_ERR_NAN = -6,       /* non-finite residual or norm                      */
    TM_ERR_HIP = -7,       /* HIP runtime error (text in tm_last_error)       */
    TM_ERR_NOMEM = -8,     /* device allocation failed                        */
    TM_ERR_LIMIT = -9      /* size beyond a documented limit                  */
};

typedef enum { TM_FP64 = 0, TM_FP32 = 1, TM_FP16 = 2, TM_BF16 = 3 } tm_prec;
typedef enum { TM_TWIST_PLUS = 1, TM_TWIST_MINUS = -1, TM_TWIST_NDEG = 2 } tm_flavor;
typedef enum { TM_PC_ASYM = 0, TM_PC_SYM = 1 } tm_pc;
/* Solution type of the normal-equation solve (Sec. 2.2, solution_type):
 * TM_SOLUTION_MAT: x solves M x = b (CG on M^+ M x = M^+ b);
 * TM_SOLUTION_MATDAG_MAT: x solves M^+ M x = b.                              */
typedef enum { TM_SOLUTION_MAT = 0, TM_SOLUTION_MATDAG_MAT = 1 } tm_solution;
/* Solve type of tm_solve (Sec. 2.2, solver_type): which residual of the
 * preconditioned system the tolerance bounds.
 * TM_SOLVE_NORMOP_PC: the normal residual |M^+b - M^+M x| / |M^+b| (as tm_cg);
 * TM_SOLVE_DIRECT_PC: the system's own residual |b - M x| / |b| (CG restarted
 * from its current x with a tighter normal tolerance until this holds).      */
typedef enum { TM_SOLVE_NORMOP_PC = 0, TM_SOLVE_DIRECT_PC = 1 } tm_solve_type;
/* Spin basis of canonical spinors (Sec. 2: the library computes in the
 * non-relativistic basis and converts from a chiral one on the way in/out).
 * TM_BASIS_CHIRAL: g_k = [[0, -i s_k], [i s_k, 0]], g_4 = [[0, 1], [1, 0]],
 * g5 = diag(1, 1, -1, -1); psi_chiral = S psi_internal with the real
 * orthogonal, self-inverse S = H (x) 1_2, H = [[1, 1], [1, -1]] / sqrt 2 on
 * the (upper, lower) spin pairs: components 0 and 2, 1 and 3 mix.          */
typedef enum { TM_BASIS_INTERNAL = 0, TM_BASIS_CHIRAL = 1 } tm_basis;

/* Epilogue of tm_dslash, with A = D in (or D^+ in), x the optional field of the
 * output parity and R, R^-1 daggered when dagger = 1:                          */
typedef enum {
    TM_EPI_NONE = 0,              /* out = A                    */
    TM_EPI_TWINV = 1,             /* out = R^-1 A               */
    TM_EPI_RX_PLUS_KD = 2,        /* out = R x + k A            */
    TM_EPI_X_PLUS_K_TWINV_D = 3,  /* out = x + k R^-1 A         */
    TM_EPI_TWINV_X_PLUS_KD = 4,   /* out = R^-1 (x + k A)       */
    TM_EPI_X_PLUS_KD = 5          /* out = x + k A              */
} tm_epilogue;

typedef struct {
    int dims[4];          /* Lx, Ly, Lz, Lt: even, >= 2; at most 2e8 sites per
                             parity (TM_ERR_LIMIT beyond: 32-bit site indices) */
    double kappa;         /* hopping parameter                                  */
    double mu;            /* bare twisted mass of Eq. (2.1) (lattice units)      */
    double epsilon;       /* bare flavour splitting of Eq. (2.1); doublet only   */
    int flavor;           /* tm_flavor                                          */
    int t_antiperiodic;   /* 1: antiperiodic in t, 0: periodic                  */
    double csw;           /* twisted clover (Sec. 4, future work): c_sw of
                             R(x) = A(x) + i a g5 t3 + b t1,
                             A = 1 + i kappa c_sw sum_{mu<nu} sigma_munu F_munu,
                             sigma_munu = (i/2)[g_mu, g_nu], F_munu = (Q - Q^+)/8
                             with Q the four plaquette leaves at x; 0: none.
                             FP64 / FP32 only; not with 8-real links or tm_force. */
} tm_params;

typedef struct {
    int pc;               /* tm_pc                                              */
    double tol;           /* stop when |M^+b - M^+M x| <= tol |M^+b| (FP64)     */
    int maxiter;          /* iteration cap (inner iterations for mixed)         */
    int outer;            /* precision of x and b: TM_FP64                      */
    int inner;            /* TM_FP64 (plain CG) or TM_FP32 / FP16 / BF16 (mixed) */
    double delta;         /* reliable-update threshold (mixed); 0: 0.01 (FP16), 0.02 (BF16), 0.001 (FP32);
                             raised to 2e-3 (FP16), 1e-2 (BF16), 1e-5 (FP32) at least */
    int use_x0;           /* 1: x holds the initial guess                       */
    int nrhs;             /* right-hand sides solved together (>= 1)            */
    int graph_iters;      /* > 0: capture this many iterations in a hipGraph    */
    int check_every;      /* iterations between host convergence checks (eager
                             solves; 0 -> 8).  Every iteration is gated on the
                             device by the convergence state, so iterations
                             enqueued after convergence do nothing and the
                             iteration count is exact for any period.        */
    int solution;         /* tm_solution                                        */
    double stall_factor;  /* mixed: a reliable update whose true |r| is not
                             below stall_factor times the |r| of the previous
                             update made no progress (0 -> 1)                 */
    int max_stalls;       /* mixed: after this many consecutive updates without
                             progress the solve continues from its x with the
                             next wider inner precision (FP16/BF16 -> FP32 ->
                             FP64); 0 -> 3, < 0: never                        */
} tm_cg_params;

typedef struct {
    int iters;                    /* CG iterations performed                     */
    int reliable_updates;         /* FP64 residual replacements (mixed)          */
    double true_rel_res_normal;   /* |M^+b - M^+M x| / |M^+b|, FP64, recomputed  */
    double true_rel_res_pc;       /* |b - M x| / |b| (MATDAG_MAT: |b - M^+M x|/|b|) */
    double seconds;               /* wall time of the solve (host clock)         */
    double true_rel_res_full;     /* tm_solve: |b - M x| / |b| (MATDAG_MAT:
                                     |b - M^+M x| / |b|) over both parities;
                                     tm_cg: -1                                    */
    int precision_fallbacks;      /* inner-precision promotions after stalls     */
    int history_len;              /* entries of res_history (<= 16)              */
    double res_history[16];       /* iterated |r| / |M^+b| of this rhs's last
                                     history_len iterations, oldest first (the
                                     precision of the inner iterations)          */
} tm_cg_result;

typedef struct {
    tm_cg_params cg;      /* pc, tol, maxiter, inner, delta, nrhs, graph_iters,
                             check_every of every CG run (its use_x0 and
                             solution are set by tm_solve)                    */
    int solve_type;       /* tm_solve_type                                      */
    int solution;         /* tm_solution of the full system                     */
} tm_solve_params;

typedef struct tm_ctx tm_ctx;
typedef struct tm_gauge tm_gauge;

/* Context: binds a HIP stream (NULL = the null stream) and owns workspace.
 * Create/destroy synchronise the stream.                                      */
int tm_ctx_create(tm_ctx **ctx, void *hip_stream);
int tm_ctx_destroy(tm_ctx *ctx);
int tm_ctx_set_stream(tm_ctx *ctx, void *hip_stream);
const char *tm_error_string(int code);
const char *tm_last_error(tm_ctx *ctx);

/* Gauge field + operator parameters (the Dirac operator object, Sec. 2.1).
 * links_dev: complex128 canonical links [4][V][3][3] on the device (read only
 * during the call).  recon (Sec. 3, link reconstruction): 18 (full links),
 * 12 (rows 0 and 1 stored, row 2 rebuilt as conj(row0 x row1)) or 8 (U01,
 * U02, U10 and the phases of U00 and U20 stored; the other entries rebuilt
 * from unit rows/columns, row orthogonality and det U = 1; the phases are
 * 16-bit fixed point in FP16/BF16).  8 needs |U01|^2 + |U02|^2 >= 1e-10 on
 * every link (else TM_ERR_ARG: e.g. the unit gauge field) and is not read by
 * tm_force.  prec_mask: bit (1 << tm_prec) for every precision to build.
 * Validates dims (TM_ERR_DIMS) and the twist (TM_ERR_SINGULAR).  Synchronises
 * the stream.                                                                 */
int tm_gauge_create(tm_ctx *ctx, tm_gauge **g, const void *links_dev, const tm_params *p,
                    int recon, unsigned prec_mask);
int tm_gauge_destroy(tm_gauge *g);
/* Device bytes held by the packed links of one precision (0 if not built).    */
size_t tm_gauge_bytes(const tm_gauge *g, int prec);

/* Bytes of one parity of a native spinor field (all rhs, flavours, scales).   */
size_t tm_spinor_bytes(const tm_params *p, int prec, int nrhs);

/* Canonical complex128 full-lattice field [nrhs][V][nf][4][3] (device) <->
 * native field of one parity.  Unpack writes only the sites of that parity.
 * basis (tm_basis) is the spin basis of the canonical field; the conversion
 * is applied in FP64 on the way (Sec. 2, converting routines).               */
int tm_spinor_pack(tm_ctx *ctx, void *dst_native, const void *src_canonical,
                   const tm_params *p, int prec, int parity, int nrhs, int basis);
int tm_spinor_unpack(tm_ctx *ctx, void *dst_canonical, const void *src_native,
                     const tm_params *p, int prec, int parity, int nrhs, int basis);

/* Fused hop (Sec. 2.1: the hop fused with its local epilogue): out (parity out_parity) = epilogue of
 * D in or D^+ in (in has the other parity).  twist_on_load = 1 applies R^-1
 * (R^-+ if dagger) to every neighbour before the hop, i.e. A = D R^-1 in.
 * x may be NULL for TM_EPI_NONE / TM_EPI_TWINV.  All fields share prec.       */
int tm_dslash(tm_ctx *ctx, void *out, const void *in, const tm_gauge *g, int prec,
              int out_parity, int dagger, int twist_on_load, int epi,
              const void *x, double k, int nrhs);

/* Preconditioned operator of Eq. (2.2) (TM_PC_ASYM) or Eq. (2.3) (TM_PC_SYM),
 * or its dagger, on even fields: two fused hop kernels with an odd temporary
 * held by the context.  out_e and in_e must not alias.                        */
int tm_mat_pc(tm_ctx *ctx, void *out_e, const void *in_e, const tm_gauge *g, int prec,
              int pc, int dagger, int nrhs);

/* tm_mat_pc for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and launch shapes as tm_mat_pc, with the odd temporary (and,
 * for the twisted-clover sym^+ form, the twist-on-load temporary) taken from
 * a 256 MiB device scratch array that every GPU the library runs on holds
 * from context creation until the process ends.  It allocates nothing and
 * runs no autotuning (launch shapes already tuned in this context are used,
 * else the defaults).  Sizes: the temporaries (one odd spinor field of
 * tm_spinor_bytes(p, prec, nrhs), rounded up to 256 bytes; two for clover
 * sym^+) must fit in the 256 MiB, else TM_ERR_LIMIT before any launch (the
 * 32^3 x 64 FP32 doublet needs 192 MiB).  Nothing in the scratch needs to
 * start at zero: the first kernel writes the whole temporary before the
 * second reads it.  The scratch is shared by every call on one GPU, from any
 * context, and keeps the last call's contents: calls that overlap on one GPU
 * (other streams, other host threads) race.  Errors as tm_mat_pc, plus
 * TM_ERR_HIP if the scratch's device address could not be resolved.          */
int tm_mat_pc_noalloc(tm_ctx *ctx, void *out_e, const void *in_e, const tm_gauge *g, int prec,
                      int pc, int dagger, int nrhs);

/* out = R^-1 in (R^-+ in if dagger) on one parity; inverse = 0 gives R, R^+.
 * The twist is site-local: uniform for twisted mass, the site's clover blocks
 * of that parity for twisted clover.                                          */
int tm_twist(tm_ctx *ctx, void *out, const void *in, const tm_gauge *g, int prec,
             int parity, int dagger, int inverse, int nrhs);
int tm_twist_inv(tm_ctx *ctx, void *out, const void *in, const tm_gauge *g, int prec,
                 int parity, int dagger, int nrhs);

/* Right-hand side of Eq. (2.2) / (2.3): bhat_e = b_e + kappa D_eo R_oo^-1 b_o
 * (asym), R_ee^-1 times that (sym).  (The printed equations omit the kappa
 * that the kappa^2 of their left-hand side requires.)                         */
int tm_prepare(tm_ctx *ctx, void *bhat_e, const void *b_e, const void *b_o, const tm_gauge *g,
               int prec, int pc, int nrhs);

/* Odd half of the solution (Eq. 2.4 read for the unpreconditioned even
 * solution): x_o = R_oo^-1 (b_o + kappa D_oe x_e).                            */
int tm_reconstruct_odd(tm_ctx *ctx, void *x_o, const void *x_e, const void *b_o,
                       const tm_gauge *g, int prec, int nrhs);

/* CG on the normal equations of the preconditioned operator (NORMOP_PC solve,
 * Sec. 2.2): M^+ M x = M^+ b (solution TM_SOLUTION_MAT) or M^+ M x = b
 * (TM_SOLUTION_MATDAG_MAT); tol applies to the residual of that system.  x_e, b_e: native even fields in precision
 * par->outer (TM_FP64), par->nrhs right-hand sides.  inner = TM_FP64: plain
 * FP64 CG; inner = FP32 / FP16 / BF16: mixed precision with reliable updates
 * (low-precision iterations; FP64 true residual, reductions and solution
 * accumulation).  An iteration updates the residual inside the last hop of
 * M^+ M p (M^+ M p is not stored) and takes the step x += alpha p in the pass
 * that forms the next direction; TM_CG_FUSE=0 in the environment at context
 * creation selects separate passes instead (same arithmetic, more traffic).
 * TM_VERBOSE=1 (read at context creation) prints the progress at every host
 * check and each rhs's final residuals to stderr.
 * res: array of par->nrhs results.  Synchronous.  Returns TM_NOT_CONVERGED if
 * some rhs missed tol within maxiter (x, res filled).                        */
int tm_cg(tm_ctx *ctx, void *x_e, const void *b_e, const tm_gauge *g, const tm_cg_params *par,
          tm_cg_result *res);

/* One CG over several independent problems of uneven lattice size (each its
 * own gauge / operator, nrhs[i] sources), every stage of an iteration being
 * one kernel launch over all problems.  At most 8 problems.                   */
int tm_cg_batched(tm_ctx *ctx, int nproblems, const tm_gauge *const *g, void *const *x_e,
                  const void *const *b_e, const int *nrhs, const tm_cg_params *par,
                  tm_cg_result *res);

/* Full-system solve (Sec. 2.2, solution_type x solver_type; Eqs. 2.2-2.4).
 * b_e, b_o: FP64 native source halves; x_e, x_o: FP64 native solution halves
 * (written; must not alias the sources).  nrhs = par->cg.nrhs.
 *   TM_SOLUTION_MAT: M x = b.  b^ = b_e + kappa D_eo R_oo^-1 b_o (sym: R_ee^-1
 *     times that), CG on the preconditioned system, then
 *     x_o = R_oo^-1 (b_o + kappa D_oe x_e).
 *   TM_SOLUTION_MATDAG_MAT: M^+ M x = b, as two solves M^+ y = b, M x = y.  The
 *     first takes the Schur route of M^+ (R^+, D^+ in place of R, D): with A
 *     the preconditioned operator, z solves A^+ A z = c for
 *     c = b_e + kappa D^+_eo R_oo^-+ b_o, y_e = A z (sym: R_ee^-+ A z) and
 *     y_o = R_oo^-+ (b_o + kappa D^+_oe y_e).
 * res[nrhs]: iterations and reliable updates summed over every CG run,
 * residuals of the last one, and true_rel_res_full.  Returns TM_NOT_CONVERGED
 * if a CG run missed its tolerance (x still written).  Workspace: up to five
 * FP64 fields of one parity besides tm_cg's.                                  */
int tm_solve(tm_ctx *ctx, void *x_e, void *x_o, const void *b_e, const void *b_o,
             const tm_gauge *g, const tm_solve_params *par, tm_cg_result *res);

/* Native-field BLAS used by the solvers, exposed for tests and clients.
 * Results are written to host memory (synchronous).                           */
int tm_norm2(tm_ctx *ctx, double *out_host, const void *x, const tm_params *p, int prec,
             int nrhs);
int tm_dot(tm_ctx *ctx, double *out_host /* 2*nrhs: re, im */, const void *x, const void *y,
           const tm_params *p, int prec, int nrhs);
/* dst = src converted between precisions (same parity, nrhs).                 */
int tm_convert(tm_ctx *ctx, void *dst, int dst_prec, const void *src, int src_prec,
               const tm_params *p, int nrhs);
/* dst = a src, converted between precisions as tm_convert (dst may be src
 * when the precisions agree); a must be finite.  Used for the chain rule of
 * the action's gradient with respect to the source (2 dS/dS_out X).          */
int tm_scale(tm_ctx *ctx, void *dst, int dst_prec, const void *src, int src_prec, double a,
             const tm_params *p, int nrhs);

/* Gauge force for S = phi^+ (M^+ M)^-1 phi with M the asymmetric (or
 * symmetric) preconditioned operator and X = (M^+ M)^-1 phi given (even,
 * native, precision prec).  F_dev: complex [4][V][3][3] canonical, FP32
 * (force_prec = TM_FP32) or FP64, the traceless anti-Hermitian dS/dU in the
 * convention dS/dw^a = -2 tr(F T^a) for U -> exp(w^a T^a) U, T^a = i lambda_a/2;
 * scaled by coeff and added to F_dev if accumulate.  G_dev (nullable, same
 * type and shape): the unconstrained complex gradient with dS = Re tr(G^+ dU). */
int tm_force(tm_ctx *ctx, void *F_dev, int force_prec, const void *X_e, const tm_gauge *g,
             int prec, int pc, double coeff, int accumulate, void *G_dev);

/* Autotuner: 1 enables the timing-based choice of the hop launch per kernel
 * variant and shape -- right-hand sides per thread (1, 2 or 4 where they
 * divide every problem's count; one flavour, 12-real links), block size,
 * link-load policy, cap of resident waves per SIMD, LDS staging (FP32 one
 * flavour), then the four fastest of those in each depth of the brick site
 * order, then the three best of those with their single-use streams (output
 * stores; with the xpay operand and / or the time-neighbour loads) accessed
 * non-temporally -- cached per
 * context and persisted to $TM_TUNE_CACHE if set; 0 disables (defaults are
 * then used).
 * Read at context creation, for experiments: TM_HOP_NR, TM_HOP_BS,
 * TM_LINK_NT, TM_HOP_WCAP, TM_HOP_ZC, TM_HOP_LDS, TM_HOP_NT (mask: 1 output,
 * 2 xpay operand, 4 time neighbours) fix one of those choices,
 * TM_XCD_REMAP=0 turns off the XCD-aware block order.                         */
int tm_set_tuning(tm_ctx *ctx, int enable);

/* Launch planner of the hop kernel (host arithmetic only: no device work,
 * callable without a GPU).  dyn_bytes receives the dynamic LDS one workgroup
 * of block_size threads requests so that a compute unit holds at most
 * wave_cap waves per SIMD (0: no cap; a cap keeps the neighbour spinors the
 * resident waves share in L2) and at least staging_bytes for staged
 * neighbours, given the compute unit's LDS (lds_per_cu), the most one
 * workgroup may use (lds_per_block) and the kernel's static LDS (its function
 * attributes).  Footprints are planned in multiples of 2560 bytes, so the
 * dispatcher rounds none of them up.  Returns TM_ERR_LIMIT when no request
 * meets both limits (the library never dispatches such a launch shape: the
 * tuner skips it, a forced one fails with TM_ERR_LIMIT) and TM_ERR_ARG on bad
 * arguments (block_size not a positive multiple of 64, wave_cap outside
 * 0..8, zero limits, null dyn_bytes).                                        */
int tm_plan_hop_lds(int block_size, int wave_cap, unsigned staging_bytes, unsigned lds_per_cu,
                    unsigned lds_per_block, unsigned static_lds, unsigned *dyn_bytes);

#ifdef __cplusplus
}
#endif
#endif /* TM_H */
