/*
 * deinsum.h -- C ABI of the MI355X (gfx950) MTTKRP / TTMc library.
 *
 * The library computes the two local multilinear kernels that dominate
 * Deinsum's run time (Ziogas et al., "Deinsum: Practically I/O Optimal
 * Multilinear Algebra", arXiv 2206.08301):
 *   - mode-n MTTKRP (Sec. III-B; benchmark forms MTTKRP-O3-M{0,1,2} and
 *     MTTKRP-O5-M{0,2,4} of Tab. IV), computed without ever forming the
 *     Khatri-Rao product in memory (the fused schedule of Sec. IV-E);
 *   - the mode-n TTM chain, TTMc (Sec. III-B; TTMc-O5-M0 of Tab. IV).
 * Problems are stated in Einstein notation (Sec. III-A), as the paper's
 * front end takes them; the parser accepts exactly these two families.
 *
 * Conventions for every entry point
 *   - All functions are extern "C" and return a deinsum_status (0 = OK,
 *     negative = error).  On error a message is available from
 *     deinsum_last_error() (thread-local, valid until the next call on the
 *     same thread).
 *   - Tensors are dense and row-major (last index contiguous), as NumPy
 *     C order.  X is I_0 x .. x I_{N-1}.  A factor operand "<m><r>" is an
 *     I_m x R matrix, R contiguous.  The MTTKRP output is I_n x R; the TTMc
 *     output has the dims of X with every contracted I_m replaced by R_m,
 *     in place (the output string of the spec).
 *   - Arrays named X, U, M, Y, workspace are DEVICE pointers owned by the
 *     caller; the library never frees or retains them.  dims / ranks are
 *     host arrays read during the call only.  Device pointers must be
 *     aligned to their element size; 16-byte alignment (torch's default)
 *     lets the kernels use vector loads.
 *   - The output is overwritten (the paper zero-initialises, then
 *     accumulates); it must not overlap X or any factor.
 *   - Argument errors are reported synchronously and nothing is enqueued.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *     and the call returns without synchronising.  A device fault surfaces
 *     as DEINSUM_ERR_DEVICE from a later call or from the caller's sync.
 *   - Workspace: with opts->workspace NULL a call takes the library pool's
 *     buffer for its device and stream (grow-only; growing it synchronises
 *     that stream).  Calls on one stream reuse it in stream order; calls on
 *     different streams use different buffers, so they may run concurrently.
 *     Up to 16 streams per device hold a buffer at once; a 17th stream takes
 *     the least recently used one after a device synchronise.  A caller
 *     buffer in opts->workspace is the caller's to order across streams.
 *   - Results are deterministic: for a given problem, plan and device the
 *     output is bitwise identical run to run (fixed reduction order, no
 *     floating-point atomics).
 */
#ifndef DEINSUM_H
#define DEINSUM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DEINSUM_MAX_ORDER 8
#define DEINSUM_MAX_RANK 256

typedef enum deinsum_status {
    DEINSUM_OK = 0,
    DEINSUM_ERR_INVALID_ARG = -1, /* null pointer, overlap, bad enum      */
    DEINSUM_ERR_PARSE = -2,       /* malformed einsum string              */
    DEINSUM_ERR_UNSUPPORTED = -3, /* well-formed but not MTTKRP / TTMc    */
    DEINSUM_ERR_SHAPE = -4,       /* dims or ranks < 1 or too large       */
    DEINSUM_ERR_NO_MEMORY = -5,   /* workspace too small / alloc failed   */
    DEINSUM_ERR_DEVICE = -6,      /* HIP runtime error                    */
    DEINSUM_ERR_BUSY = -7         /* resource temporarily unavailable     */
} deinsum_status;

typedef enum deinsum_kind { DEINSUM_MTTKRP = 1, DEINSUM_TTMC = 2, DEINSUM_MTTKRP_MM = 3 } deinsum_kind;

/* Element types.  DEINSUM_FX20 names X held in the FX20 storage below
 * (deinsum_fx20_encode); it is only a storage code of X (opts.x_dtype). */
typedef enum deinsum_dtype { DEINSUM_F64 = 0, DEINSUM_F32 = 1, DEINSUM_BF16 = 2, DEINSUM_FX20 = 3 } deinsum_dtype;

/*
 * Arithmetic form.  The paper fixes no precision (Sec. VI-A); FP64 is the
 * plain form, the others trade accuracy for HBM bytes.
 *   FP64   : X, factors, output FP64; FP64 matrix-core products.
 *   FP32   : X and factors FP32; FP32 matrix-core products over one slice
 *            of the contiguous mode, FP64 accumulation and reduction
 *            beyond it; output FP32 or FP64.
 *   BF16   : X BF16, factors FP32 (rounded to BF16 on the device); BF16
 *            matrix-core products with FP32 accumulation, FP64 beyond one
 *            slice; output FP32 or FP64.
 *   BF16X3 : X and factors FP32, each split on the device into hi + lo
 *            BF16 parts; products hi*hi + hi*lo + lo*hi on the matrix cores
 *            with FP32 accumulation, FP64 beyond one slice.
 *   FX20   : X in the 3-byte FX20 storage below (deinsum_fx20_encode),
 *            factors FP32.  Last-mode-contiguous free modes: each factor
 *            slice is scaled per column by a power of two and split into
 *            FP16 hi + lo parts; X's FP16 part h and int8 part l feed FP16
 *            matrix-core products h*hi + h*lo + l*hi with FP32 accumulation,
 *            FP64 beyond one slice.  Free mode = last mode: X decoded to FP32,
 *            FP32 matrix-core products.  Output FP32 or FP64.  Reads 3 bytes
 *            per element of X instead of 8.
 *   AUTO   : the library picks the form from opts.tol and the storage of the
 *            operands (opts.x_dtype, opts.u_dtype): among the compiled forms
 *            that read that storage, the cheapest whose estimated error
 *            (deinsum_estimate_error) is at most tol.  Forms by X storage:
 *            F64 -> FP64; F32 -> BF16X3, FP32 (BF16X3 first: the same bytes
 *            and the faster of the two); BF16 -> BF16; FX20 -> FX20.  When no
 *            form reading that storage meets tol the call fails with
 *            DEINSUM_ERR_UNSUPPORTED before anything is enqueued (pick the
 *            storage with deinsum_choose_storage).  The report names the form
 *            that ran and its estimate.  MTTKRP, MTTKRP-GEMM chain and TTMc
 *            (TTMc forms: FP64, FP32, BF16, FX20).
 */
typedef enum deinsum_precision {
    DEINSUM_PREC_FP64 = 0,
    DEINSUM_PREC_FP32 = 1,
    DEINSUM_PREC_BF16 = 2,
    DEINSUM_PREC_BF16X3 = 3,
    DEINSUM_PREC_FX20 = 4,
    DEINSUM_PREC_AUTO = 5
} deinsum_precision;

/* Parsed einsum (deinsum_parse).  Letters are ASCII a-z / A-Z. */
typedef struct deinsum_spec {
    int32_t kind;                           /* deinsum_kind                           */
    int32_t order;                          /* N, 2 <= N <= 8                         */
    int32_t free_mode;                      /* n                                      */
    int32_t n_factors;                      /* N - 1                                  */
    int32_t factor_mode[DEINSUM_MAX_ORDER]; /* operand k contracts mode factor_mode[k] */
    int32_t operand_of_mode[DEINSUM_MAX_ORDER]; /* inverse map; -1 for the free mode  */
    char tensor_idx[DEINSUM_MAX_ORDER + 1]; /* letters of X                           */
    char rank_idx[DEINSUM_MAX_ORDER + 1];   /* rank letter per MODE ('-' at n)        */
    char out_idx[DEINSUM_MAX_ORDER + 2];    /* output letters                         */
} deinsum_spec;

/* Optional per-call report (filled when deinsum_opts.report != NULL). */
typedef struct deinsum_report {
    int32_t plan_id;            /* kernel family chosen (see plan_name)         */
    int32_t tile_m, tile_k;     /* output rows per wave, contraction slice      */
    int32_t waves_per_group;    /* waves per workgroup                          */
    int64_t groups;             /* workgroups launched by the main kernel       */
    int64_t partials;           /* partial outputs reduced in the fixed-order pass */
    size_t workspace_bytes;     /* workspace used                                */
    double alg_bytes;           /* X once + factors once + output once           */
    double alg_flops;           /* flops of the two-stage method                 */
    char plan_name[48];
    double tuned_us;            /* deinsum_tune_*: median time of the chosen plan */
    int32_t precision;          /* the form that ran (resolves DEINSUM_PREC_AUTO) */
    double est_err;             /* deinsum_estimate_error of that form for this call */
} deinsum_report;

typedef struct deinsum_opts {
    int32_t precision;        /* deinsum_precision (default FP64)                    */
    int32_t out_dtype;        /* DEINSUM_F64 or DEINSUM_F32 (F64 required for FP64)  */
    void *workspace;          /* optional caller device buffer; NULL = the library
                                 pool's buffer for this device and stream           */
    size_t workspace_bytes;   /* its size                                            */
    int32_t plan_hint;        /* MTTKRP: 0 = autotuned plan if cached, else the
                                 heuristic; 1 / 2 = heuristic, and the free mode
                                 must be < N-1 / = N-1 (tests); 3 = free mode 0
                                 of an order-3 tensor, reduced forms: mode-1
                                 tiles walked per output row (tests).
                                 TTMc: 0 = autotuned fused-kernel variant if cached,
                                 else the default; k >= 1 = compiled variant k-1
                                 for the ranks (tests, tuning)                        */
    int32_t split_hint;       /* 0 = planner choice; else outer-chunk count          */
    deinsum_report *report;   /* optional host out-parameter                         */
    double tol;               /* DEINSUM_PREC_AUTO: largest acceptable estimated
                                 normwise relative error (> 0)                        */
    int32_t x_dtype;          /* DEINSUM_PREC_AUTO: storage of X (deinsum_dtype)     */
    int32_t u_dtype;          /* DEINSUM_PREC_AUTO: factor dtype, DEINSUM_F64 or
                                 DEINSUM_F32 (the FP64 form takes F64 factors, every
                                 other form F32)                                      */
    int32_t deterministic;    /* 1 (default): bitwise reproducible results.  Every
                                 compiled path reduces in a fixed order, so 0 is
                                 accepted and gives the same results               */
} deinsum_opts;

/* Fill *opts with defaults: FP64, F64 output, library workspace, planner choice,
 * tol 1e-12, x_dtype = u_dtype = F64, deterministic 1. */
void deinsum_opts_init(deinsum_opts *opts);

/*
 * Parse an einsum string of the MTTKRP or TTMc family (host only, no GPU).
 *   MTTKRP: "<X>,<f_1>,...,<f_{N-1}>-><n><r>", X has N distinct letters,
 *           each factor is "<mode letter><r>" with one shared rank letter r
 *           not in X, each mode but the free mode n appears in exactly one
 *           factor (any order), e.g. "ijk,ja,ka->ia" (Tab. IV).
 *   TTMc  : same operands with a distinct rank letter per factor; the output
 *           is X's letters with each contracted letter replaced by its rank
 *           letter in place, e.g. "ijklm,jb,kc,ld,me->ibcde" (Tab. IV).
 * Whitespace is ignored.  Rejected with DEINSUM_ERR_PARSE: missing "->",
 * ellipsis, non-letters, a letter repeated inside an operand, empty
 * operands.  Rejected with DEINSUM_ERR_UNSUPPORTED: anything else outside
 * the two families (a factor with its letters swapped, a factor on the free
 * mode, a mode contracted twice or not at all, other output orders,
 * N > 8).  N = 2 specs whose output is "<n><r>" parse as MTTKRP.
 */
deinsum_status deinsum_parse(const char *spec, deinsum_spec *out);

/*
 * Workspace (device bytes) a call with these arguments needs.  ranks: for
 * MTTKRP ranks[0] = R; for TTMc one rank per factor operand (operand order);
 * for the MTTKRP-GEMM chain ranks[0] = R, ranks[1] = L.
 */
deinsum_status deinsum_workspace_size(const deinsum_spec *spec, const int64_t *dims,
                                      const int64_t *ranks, const deinsum_opts *opts,
                                      size_t *bytes);

/*
 * Mode-n MTTKRP (Sec. III-B, Tab. IV):
 *   M[i_n, r] = sum_{i_m, m != n} X[i_0..i_{N-1}] * prod_{m != n} U^{m}[i_m, r]
 * spec  : parsed MTTKRP spec; dims: N host sizes of X in its letter order.
 * R     : rank, 1 <= R <= 256.
 * X     : device tensor, dtype by precision (FP64: f64; FP32, BF16X3: f32; BF16: bf16;
 *         FX20: the buffer written by deinsum_fx20_encode, 256-byte aligned).
 * U     : host array of N-1 device pointers in OPERAND order (operand k is
 *         I_{factor_mode[k]} x R; f64 for FP64, f32 otherwise).
 * M     : device I_n x R output, dtype opts->out_dtype.
 * opts  : NULL for defaults.
 */
deinsum_status deinsum_mttkrp(const deinsum_spec *spec, const int64_t *dims, int64_t R,
                              const void *X, const void *const *U, void *M,
                              const deinsum_opts *opts, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): deinsum_mttkrp with its
 * workspace (partial output tiles, outer-weight table, merged factor) taken from
 * a fixed library-owned device array of DEINSUM_NOALLOC_SCRATCH_BYTES per device
 * instead of the library pool or a caller buffer.  The call allocates nothing:
 * no hipMalloc / hipFree, no allocating library routine.  The array is set aside
 * when the library's code object is loaded on a device and held until the
 * process ends; its device address is looked up on the first call on each device.
 * Arguments, results and plans are those of deinsum_mttkrp (bitwise the same
 * output), except:
 *   - opts->workspace must be NULL (DEINSUM_ERR_INVALID_ARG otherwise);
 *   - a problem whose plan needs more than DEINSUM_NOALLOC_SCRATCH_BYTES of
 *     workspace (deinsum_workspace_size) is rejected with DEINSUM_ERR_NO_MEMORY
 *     before anything is enqueued (e.g. 80^5 FP64, R = 24, needs 133 MiB).
 * Every call on one device shares that device's array and leaves its contents
 * behind (nothing in it needs to start at zero: each call writes every workspace
 * byte it reads).  Calls that overlap on one device -- on different streams,
 * or from different threads without ordering -- race on the array and give
 * wrong results; order them on one stream or with events.
 */
#define DEINSUM_NOALLOC_SCRATCH_BYTES (64u << 20)
deinsum_status deinsum_mttkrp_noalloc(const deinsum_spec *spec, const int64_t *dims, int64_t R,
                                      const void *X, const void *const *U, void *M,
                                      const deinsum_opts *opts, void *stream);

/*
 * The MTTKRP-GEMM chain of the paper's running example (Sec. II-A), e.g.
 * "ijk,ja,ka,al->il": the MTTKRP operands followed by one more operand
 * "<rank letter><l>", output "<free letter><l>":
 *   Y[i_n, l] = sum_r M[i_n, r] * C[r, l],  M the mode-n MTTKRP above.
 * spec : parsed DEINSUM_MTTKRP_MM spec (factor_mode, free_mode as for MTTKRP).
 * R, L : rank (1..256) and the chain's output width (1..4096).
 * X, U : as for deinsum_mttkrp (U: the N-1 factor operands in operand order).
 * C    : device R x L matrix, row-major, f64 for FP64 and f32 otherwise.
 * Y    : device I_n x L output, dtype opts->out_dtype; must not overlap the inputs.
 * M is formed in FP64 in the workspace (deinsum_workspace_size with ranks
 * {R, L}) and the product is summed in FP64 in increasing r.  Errors as for
 * deinsum_mttkrp; asynchronous on `stream`.
 */
deinsum_status deinsum_mttkrp_mm(const deinsum_spec *spec, const int64_t *dims, int64_t R, int64_t L,
                                 const void *X, const void *const *U, const void *C, void *Y,
                                 const deinsum_opts *opts, void *stream);

/*
 * Mode-n TTMc (Sec. III-B, Tab. IV): the chain X x_m U^{m} over every m != n,
 * each product contracting the factor's first index (I_m x R_m):
 *   Y[r_0..i_n..r_{N-1}] = sum_{i_m, m != n} X[i] * prod_{m != n} U^{m}[i_m, r_m]
 * ranks : host array of N-1 ranks in operand order, each 1..64.
 * Forms: FP64 (X, U f64), FP32 (X, U f32), BF16 (X bf16, U f32; BF16 matrix
 * cores for the first contraction, FP32 for the second, FP64 sums beyond) and
 * FX20 (X the FX20 buffer, U f32: the first contraction on the FP16 matrix cores
 * as h*uh + h*ul + l*uh with the factor scaled per column by a power of two and
 * split into FP16 hi + lo, FP32 sums over the whole contracted extent, then
 * scaled back; the rest as FP32).
 * Other arguments as for deinsum_mttkrp.
 */
deinsum_status deinsum_ttmc(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks,
                            const void *X, const void *const *U, void *Y,
                            const deinsum_opts *opts, void *stream);

/* Message of the last error on this thread ("" if none). */
const char *deinsum_last_error(void);

/*
 * Synthetic input (setup, not part of the method): fill `count` elements of
 * the device array X (dtype f64 / f32 / bf16) with the counter-based
 * SplitMix64 stream (Steele, Lea & Flood, OOPSLA 2014).  Element e gets
 * z = mix64(seed + (offset + e + 1) * 0x9E3779B97F4A7C15) mapped by `dist`:
 *   0 uniform: 2 * ((z >> 11) * 2^-53) - 1 (exact in f64, rounded to
 *              nearest even for f32 / bf16);
 *   1 int5   : ((z >> 32) mod 5) - 2;   2 int3: ((z >> 32) mod 3) - 1.
 * Asynchronous on `stream`.
 */
deinsum_status deinsum_synth_fill(void *X, int32_t dtype, int64_t count, uint64_t seed,
                                  int64_t offset, int32_t dist, void *stream);

/*
 * FX20 storage of a tensor X of `count` elements: 20-bit fixed point with one
 * power-of-two scale, X[i] ~ m[i] * 2^e, e = (exponent of max|X|) - 19 (so
 * max|X| < 2^(e+19)), m[i] = X[i] * 2^-e rounded to nearest even, |m[i]| <= 2^19.
 * m is kept as m = 256 h + l with h = floor((m + 128) / 256) in [-2048, 2048]
 * and l = m - 256 h in [-128, 127].  The absolute error of every element is at
 * most 2^(e-1) <= 2^-20 max|X|; the normwise relative error of X is at most
 * 2^-19 * max|X| / rms(X) (3.3e-6 for uniform data, about 1e-6 in practice).
 * Layout of the buffer (256-byte aligned, deinsum_fx20_size bytes):
 *   bytes [0, 256)                 header: uint32 magic 0x30325846 ("FX20"),
 *                                  int32 e, int64 count, double max|X|,
 *                                  uint64 S = sum of (x 2^-(e+19))^2 in units
 *                                  of 2^-24, uint64 E = sum of the squared
 *                                  rounding errors (x - m 2^e)^2 2^-2e in units
 *                                  of 2^-28 (both from per-wave FP64 sums,
 *                                  rounded, added as integers: deterministic),
 *                                  so ||X - X_fx20|| / ||X|| = 2^-21 sqrt(E/S);
 *                                  zeros;
 *   bytes [256, 256 + A(2 count))  FP16 plane: h[i] as IEEE binary16 (exact);
 *   then A(count) bytes            int8 plane: l[i] (two's complement),
 * with A(b) = b rounded up to a multiple of 256.  X keeps its row-major index
 * order in both planes.  MTTKRP with DEINSUM_PREC_FX20 takes the buffer's
 * base address as X; a buffer whose header does not match the call's element
 * count yields NaN outputs.
 */
deinsum_status deinsum_fx20_size(int64_t count, size_t *bytes);

/* Encode `count` elements of src (DEINSUM_F64 or DEINSUM_F32, device) into the
 * FX20 buffer dst of dst_bytes >= deinsum_fx20_size(count) bytes (device,
 * 256-byte aligned).  Asynchronous on `stream`; deterministic. */
deinsum_status deinsum_fx20_encode(const void *src, int32_t src_dtype, int64_t count, void *dst, size_t dst_bytes,
                                   void *stream);

/*
 * Error estimate of an arithmetic form: the rule behind DEINSUM_PREC_AUTO and
 * deinsum_report.est_err.  *est_err estimates the normwise relative error
 * ||M - M*||_F / ||M*||_F against the exact result for the FP64 operands the
 * caller's storage was rounded from.  It is a root-sum-square model of
 * independent rounding errors, for data whose sums do not cancel much more than
 * sums of random-sign terms (it is not a bound for adversarial data), doubled
 * as a margin:
 *   est = 2 sqrt(dx^2 + d_op^2 + (N-2) d_st^2 + d_drop^2 + d_acc^2)
 * with u = 2^-53 (FP64), 2^-24 (FP32), 2^-8 (BF16), 2^-11 (FP16) and a value
 * rounded to nearest carrying a relative error of rms u/sqrt(3), a hi + lo
 * split of one format u^2/3:
 *   dx     : X as the form reads it -- 0 (F64), 2^-24/sqrt3 (F32),
 *            2^-8/sqrt3 (BF16), sqrt((2^-24/sqrt3)^2 + (2^-16/3)^2) (BF16X3),
 *            and for FX20 the exact value recorded in the buffer's header;
 *   d_op   : the factor operand of the matrix-core product, likewise (FP32
 *            factors; BF16-rounded, BF16-split or FP16-split on the device);
 *   d_st   : each of the other N-2 factors, applied in FP64 from FP32 storage
 *            (2^-24/sqrt3; 0 in the FP64 form);
 *   d_drop : product terms left out -- BF16X3 lo*lo (2^-16/3), FX20 l*u_lo
 *            (2^-22/3);
 *   d_acc  : 2^-53 sqrt(L/3) for FP64 sums over the L = prod_{m != n} I_m
 *            terms, plus 2^-24 sqrt(k/3) for the k terms summed in FP32 before
 *            each fold into FP64 (MTTKRP: the plan's slice of the matrix-core
 *            mode; fused TTMc pass: I_a + I_c), doubled for FX20 (its FP32 tile
 *            holds an offset removed after the fold).
 * opts->precision names the form, or DEINSUM_PREC_AUTO with tol / x_dtype /
 * u_dtype to ask which form AUTO picks (*precision receives it).  X is read
 * only for FX20: its header is copied to the host on `stream`, which this
 * synchronises; X may be NULL otherwise.  Host only otherwise.
 */
deinsum_status deinsum_estimate_error(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks,
                                      const void *X, const deinsum_opts *opts, int32_t *precision,
                                      double *est_err, void *stream);

/*
 * Storage of X for a tolerance (host only): the cheapest storage of X -- bytes
 * per element BF16 2, FX20 3, F32 4, F64 8 -- for which a form reading it has
 * deinsum_estimate_error <= tol for this problem (factors F32, or F64 for the
 * F64 storage).  FX20 is considered only when max_abs > 0 and rms > 0 (max |x|
 * and the root-mean-square of X, e.g. from deinsum_tensor_stats); its storage
 * error is then modelled as 2^(e-1) / (sqrt(3) rms), e the FX20 exponent of
 * max_abs.  *x_dtype receives the storage, *precision the form AUTO then runs,
 * *est_err its estimate.  No storage meets tol: DEINSUM_ERR_UNSUPPORTED.
 */
deinsum_status deinsum_choose_storage(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks,
                                      double tol, double max_abs, double rms, int32_t *x_dtype,
                                      int32_t *precision, double *est_err);

/* max |x| and sqrt(mean x^2) over `count` elements of the device array X (F64,
 * F32 or BF16).  Synchronises `stream` and returns the values on the host.
 * Deterministic (integer-exact max; squares summed per wave in a fixed order and
 * added in fixed point).  Uses the library's workspace pool (16 bytes). */
deinsum_status deinsum_tensor_stats(const void *X, int32_t dtype, int64_t count, double *max_abs, double *rms,
                                    void *stream);

/* Elementwise conversion f64 -> f32 / bf16 or f32 -> bf16, round to nearest even. */
deinsum_status deinsum_convert(const void *src, int32_t src_dtype, void *dst, int32_t dst_dtype,
                               int64_t count, void *stream);

/*
 * Batched launch (many MTTKRP jobs of uneven shape and rank, e.g. the
 * per-mode products of CP-ALS sweeps over many tensors).  Jobs added to a
 * batch run in ONE persistent kernel inside a hipGraph that is captured once
 * and replayed at every launch, after an asynchronous upload of the launched
 * jobs' descriptors: outer-weight tables -> persistent kernel (workgroups pull
 * units of all jobs from one device work queue) -> fixed-order reduction of
 * every job.  A job's result depends only
 * on its own shape and plan, so it is bitwise identical whether it runs alone
 * or with other jobs.  FP64 and FP32 forms, ranks 1..64.
 *
 * Ownership and threading: the batch object is owned by the caller and used
 * from one thread.  Device buffers of added jobs (X, U, M) must stay valid
 * until the launch that uses them has completed on its stream.  The library
 * owns the batch's descriptors, work queue and workspace arena.
 */
typedef struct deinsum_batch deinsum_batch;

/* Create a batch with room for max_jobs column blocks (grows on demand). */
deinsum_status deinsum_batch_create(int32_t max_jobs, deinsum_batch **out);

/* Add one MTTKRP job (arguments as deinsum_mttkrp; opts->precision FP64 or
 * FP32, opts->split_hint honoured, opts->workspace ignored).  *job_id (optional)
 * receives the job's index in this batch.  Host only; nothing is enqueued. */
deinsum_status deinsum_batch_add_mttkrp(deinsum_batch *b, const deinsum_spec *spec, const int64_t *dims, int64_t R,
                                        const void *X, const void *const *U, void *M, const deinsum_opts *opts,
                                        int32_t *job_id);

/* Enqueue every added job on `stream` as one graph replay.  Returns without
 * synchronising; a later launch first waits for this one's descriptor upload. */
deinsum_status deinsum_batch_launch(deinsum_batch *b, void *stream);

/* Forget the added jobs (the next adds start a new batch). */
deinsum_status deinsum_batch_reset(deinsum_batch *b);

/* Counters: jobs added, work units, graph captures so far, launches so far (any may be NULL). */
deinsum_status deinsum_batch_info(const deinsum_batch *b, int32_t *jobs, int64_t *units, int32_t *graph_captures,
                                  int64_t *launches);

/* Wait for the batch's last launch and free its resources. */
deinsum_status deinsum_batch_destroy(deinsum_batch *b);

/*
 * Request serving for CP-ALS on resident tensors.  A request (tensor t, mode n)
 * asks for one alternating-least-squares factor update of t: M = the mode-n
 * MTTKRP of t with its current factors, then U^n <- M V^{-1} with V the
 * Hadamard product of the other factors' Gram matrices, columns normalised.
 * Requests of one tensor are served in arrival order (each sees the factors
 * the previous one wrote); requests of different tensors are independent.
 *
 * With batched=1 a native scheduler thread runs continuous batching: whenever
 * one of `epochs_in_flight` (1 or 2) epoch slots is free it admits every ready
 * request (head of its tensor's queue, tensor idle) in arrival order while the
 * epoch has slots and the sum of the admitted requests' MTTKRP workspaces stays
 * within hbm_budget_bytes, and runs the epoch as one batch launch
 * (deinsum_batch_*) plus one batched update kernel on the slot's stream (an
 * small epoch: see direct_max_jobs).  With
 * batched=0 every request is launched on arrival (deinsum_mttkrp + one update
 * kernel) on a single stream: the per-request baseline.
 *
 * Latency of a request = host clock when its completion is observed minus its
 * arrival time; both are seconds since deinsum_server_start.
 *
 * Ownership and threading: the caller owns X and the factors (device memory,
 * FP64 or FP32 by `precision`, factors row-major dims[m] x R) and keeps them
 * valid until deinsum_server_destroy; the server overwrites the factors.
 * add_tensor before start; submit may be called from any thread after start;
 * results after drain.  The server uses the device current at create.
 */
typedef struct deinsum_server deinsum_server;

typedef struct deinsum_server_config {
    int32_t batched;            /* 1: continuous batching; 0: one launch per request */
    int32_t max_jobs_per_epoch; /* requests admitted into one epoch, 1..65536         */
    int32_t epochs_in_flight;   /* 1 or 2 epochs on the device at once                */
    int32_t als_update;         /* 1: run the factor update after each MTTKRP         */
    int64_t max_requests;       /* capacity of the request table                     */
    size_t hbm_budget_bytes;    /* admission limit on summed MTTKRP workspace         */
    int32_t direct_max_jobs;    /* batched: an epoch of at most this many requests
                                   runs them with the per-request launches, one after
                                   the other on the slot's stream (no descriptor
                                   upload or batch graph); their results then match
                                   the batched ones within the form's tolerance, not
                                   bitwise.  0 = every epoch is a batch launch: each
                                   result is bitwise the same alone and in any mix.
                                   0..max_jobs_per_epoch                            */
} deinsum_server_config;

/* Defaults: batched, 256 jobs per epoch, 2 in flight, update on, 1<<20 requests, 4 GiB,
 * direct_max_jobs 4. */
void deinsum_server_config_init(deinsum_server_config *cfg);

deinsum_status deinsum_server_create(const deinsum_server_config *cfg, deinsum_server **out);

/* Register a tensor (order 2..8, rank 1..64, precision DEINSUM_PREC_FP64 or
 * DEINSUM_PREC_FP32).  U holds `order` factor pointers, by mode. */
deinsum_status deinsum_server_add_tensor(deinsum_server *s, int32_t order, const int64_t *dims, int64_t R,
                                         int32_t precision, const void *X, void *const *U, int32_t *tensor_id);

/* Start the clock and the scheduler thread. */
deinsum_status deinsum_server_start(deinsum_server *s);

/* Submit one request; arrival_s < 0 means "now".  Thread-safe.  Returns
 * DEINSUM_ERR_BUSY when the request table is full. */
deinsum_status deinsum_server_submit(deinsum_server *s, int32_t tensor_id, int32_t mode, double arrival_s,
                                     int64_t *request_id);

/* Submit n requests, each at its scheduled arrival time (seconds since start,
 * non-decreasing), sleeping in between: an open-loop load generator. */
deinsum_status deinsum_server_replay(deinsum_server *s, int64_t n, const double *arrival_s, const int32_t *tensor_id,
                                     const int32_t *mode);

/* Block until every submitted request has finished, successfully or not.
 * Returns DEINSUM_OK when all succeeded, else the status of the first failed
 * request (deinsum_last_error names it and counts the failures). */
deinsum_status deinsum_server_drain(deinsum_server *s);

/* State of one request (deinsum_server_poll).  A failed request holds the
 * negative deinsum_status it failed with: DEINSUM_ERR_NO_MEMORY when its MTTKRP
 * workspace alone exceeds hbm_budget_bytes (it is never admitted), the status of
 * the library call that could not be enqueued, or DEINSUM_ERR_DEVICE when the
 * device reported an error for the launch that carried it.  A failure ends that
 * request only: other requests, and later requests of the same tensor (which
 * then see the factors as they were), are served as usual. */
typedef enum deinsum_request_status {
    DEINSUM_REQ_DONE = 0,     /* served; result written                         */
    DEINSUM_REQ_PENDING = 1,  /* submitted, not yet launched                    */
    DEINSUM_REQ_RUNNING = 2   /* launched on the device                         */
} deinsum_request_status;
/* Flag of a served request: the factor update's V had a pivot below
 * 1e-14 * max diag(V) (rank deficiency) and was regularised by that floor, so
 * the update is not the exact least-squares solution. */
#define DEINSUM_REQ_REGULARISED 1

/* Non-blocking query of request `request_id`: *status (deinsum_request_status or
 * a negative deinsum_status), *flags (DEINSUM_REQ_* bits, valid when DONE) and
 * *done_s (seconds since start when it finished, -1 before).  Thread-safe; any
 * output may be NULL. */
deinsum_status deinsum_server_poll(const deinsum_server *s, int64_t request_id, int32_t *status, int32_t *flags,
                                   double *done_s);

/* Per request i < n: arrival, completion (seconds since start, -1 if not done)
 * and the epoch (batched) or launch index that served it.  Arrays may be NULL. */
deinsum_status deinsum_server_results(const deinsum_server *s, int64_t n, double *arrival_s, double *done_s,
                                      int64_t *epoch);

/* Requests served successfully, epochs (or launches) issued, largest epoch. */
deinsum_status deinsum_server_stats(const deinsum_server *s, int64_t *completed, int64_t *epochs, int64_t *max_batch);

/* Stop the scheduler after the submitted requests finish, free everything. */
deinsum_status deinsum_server_destroy(deinsum_server *s);

/*
 * Decompositions built on the two kernels: the paper motivates MTTKRP and TTMc
 * by the CP and Tucker decompositions that spend their time in them (Sec. I).
 * Both run on the device around deinsum_mttkrp / deinsum_ttmc on `stream` and
 * return when done (they read one convergence scalar per sweep, HOOI also one
 * per subspace iteration, so they synchronise `stream`).  Deterministic.
 *
 * deinsum_cp_als: CP-ALS (Kolda & Bader, SIAM Review 2009, Sec. 3.4).  A sweep
 *   updates the modes in increasing order: M = the mode-n MTTKRP, then
 *   U^n = M V^{-1}, V the Hadamard product of the Grams U^m^T U^m (m != n),
 *   columns scaled to unit norm, the norms kept in lambda (the update of the
 *   request server; a pivot below 1e-14 max diag V is floored and flagged).
 *   After each sweep, fit = 1 - ||X - [[lambda; U]]||_F / ||X||_F from
 *   ||X||^2 - 2 <X, [[lambda; U]]> + ||[[lambda; U]]||^2 (the inner product
 *   from the last mode's MTTKRP and factor, the model norm from lambda and the
 *   Grams), so fits within ~1e-8 of 1 are not resolved.  Stops after
 *   max_sweeps or when the fit changes by less than tol.
 *   order 2..8, R 1..64.  X, U: device, F64 (precision FP64) or F32 (FP32,
 *   BF16X3: the MTTKRP form); U holds `order` factors by mode (dims[m] x R),
 *   read as the starting point and overwritten with the result; lambda: device,
 *   R doubles, out.
 * deinsum_tucker_hooi: higher-order orthogonal iteration (Kolda & Bader, Sec.
 *   4.2).  A sweep updates the modes in increasing order: Y = the TTMc of mode
 *   n (every other mode contracted with its factor), then U^n = the ranks[n]
 *   leading left singular vectors of the mode-n unfolding of Y: subspace
 *   iteration Q <- orth(Y_(n) orth(Y_(n)^T Q)) from the current U^n, CholeskyQR
 *   twice for each orth, until ||Q_new - Q Q^T Q_new||_F < iter_tol or
 *   max_iters; then Rayleigh-Ritz (cyclic Jacobi on the ranks[n]^2 matrix
 *   (Y^T Q)^T (Y^T Q)), columns by decreasing singular value, each signed so
 *   that its entry of largest magnitude is positive.  After each sweep the core
 *   G = Y x_{N-1} U^{N-1}^T (row-major ranks[0] x .. x ranks[N-1], FP64) and
 *   fit = 1 - sqrt(||X||^2 - ||G||^2) / ||X||.  Stops as CP-ALS.  ranks[m] in
 *   1..min(64, dims[m]) and at most the product of the other ranks.  X, U:
 *   device, F64 (FP64) or F32 (FP32); U: `order` factors dims[m] x ranks[m]
 *   with orthonormal columns, read as the start and overwritten; core: device,
 *   prod(ranks) doubles, out.
 * Errors as for deinsum_mttkrp / deinsum_ttmc; the drivers allocate their small
 * state (FP64 intermediates) with hipMalloc and free it before returning.
 */
typedef struct deinsum_decomp_opts {
    int32_t precision;    /* MTTKRP / TTMc form (see above)                          */
    int32_t max_sweeps;   /* >= 1 (default 25)                                       */
    double tol;           /* stop when |fit - previous fit| < tol (default 1e-10)     */
    int32_t max_iters;    /* HOOI: subspace iterations per mode update (default 200) */
    double iter_tol;      /* HOOI: subspace change to stop at (default 1e-11)        */
    double *fit_trace;    /* optional host array of max_sweeps doubles: fit per sweep */
} deinsum_decomp_opts;

#define DEINSUM_DECOMP_REGULARISED 1    /* a CP update floored a pivot of V          */
#define DEINSUM_DECOMP_MAX_ITERS 2      /* a HOOI subspace iteration hit max_iters   */
#define DEINSUM_DECOMP_RANK_DEFICIENT 4 /* a HOOI orthonormalisation met rank loss   */

typedef struct deinsum_decomp_result {
    int32_t sweeps;       /* sweeps run                                             */
    int32_t flags;        /* DEINSUM_DECOMP_* bits                                  */
    double fit;           /* fit after the last sweep                               */
    int64_t iters;        /* HOOI: subspace iterations, all modes and sweeps        */
} deinsum_decomp_result;

void deinsum_decomp_opts_init(deinsum_decomp_opts *opts);
deinsum_status deinsum_cp_als(int32_t order, const int64_t *dims, int64_t R, const void *X, void *const *U,
                              double *lambda, const deinsum_decomp_opts *opts, deinsum_decomp_result *result,
                              void *stream);
deinsum_status deinsum_tucker_hooi(int32_t order, const int64_t *dims, const int64_t *ranks, const void *X,
                                   void *const *U, double *core, const deinsum_decomp_opts *opts,
                                   deinsum_decomp_result *result, void *stream);

/*
 * Autotuner.  deinsum_tune_mttkrp runs the MTTKRP on the caller's buffers
 * (M is overwritten) once with every compiled tile shape for the problem's
 * precision and free mode (column width 16*nt, rows per wave, slice of the
 * contiguous mode) and a few outer-chunk counts around the heuristic's, times
 * `reps` runs of each on `stream` with HIP events, and stores the fastest in a
 * process-wide plan cache.  deinsum_mttkrp and deinsum_workspace_size consult
 * that cache first when plan_hint = split_hint = 0, so a tuned problem keeps
 * its plan.  deinsum_tune_batch_mttkrp does the same for a job of the batched
 * launch (its column width and split), which deinsum_batch_add_mttkrp then
 * uses.  For mode 0 of an order-3 FP64 problem (R <= 64) the candidates also
 * include running it through the fused TTMc pass (every compiled variant) and
 * taking the diagonal of the R x R result; that plan is also the default, untuned,
 * for tensors of at least 2^26 elements whose last mode has at least 256 entries.
 * *best (optional) describes the winner, tuned_us its median time.
 * The cache is keyed by path, order, free mode, precision, rank and dims; when
 * the environment variable DEINSUM_TUNE_CACHE names a file it is read on first
 * use and rewritten after every tuning call.  Host-synchronous.
 */
deinsum_status deinsum_tune_mttkrp(const deinsum_spec *spec, const int64_t *dims, int64_t R, const void *X,
                                   const void *const *U, void *M, const deinsum_opts *opts, int32_t reps,
                                   deinsum_report *best, void *stream);
deinsum_status deinsum_tune_batch_mttkrp(const deinsum_spec *spec, const int64_t *dims, int64_t R, const void *X,
                                         const void *const *U, void *M, const deinsum_opts *opts, int32_t reps,
                                         deinsum_report *best, void *stream);
/* The same for a TTMc problem: times every compiled fused-kernel variant for its
 * ranks on the caller's buffers (Y is overwritten) and caches the fastest, which
 * deinsum_ttmc uses when plan_hint = 0. */
deinsum_status deinsum_tune_ttmc(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks, const void *X,
                                 const void *const *U, void *Y, const deinsum_opts *opts, int32_t reps,
                                 deinsum_report *best, void *stream);
/* Read entries from / write the whole cache to a text file, one entry per line:
 * key nt ni mt xnt split order xcd us.  For TTMc keys the split column holds the
 * variant; an MTTKRP entry with order 2 runs through the fused TTMc pass with
 * variant `split`. */
deinsum_status deinsum_tune_load(const char *path);
deinsum_status deinsum_tune_save(const char *path);
/* Forget every cached plan. */
deinsum_status deinsum_tune_clear(void);
/* Number of cached plans. */
deinsum_status deinsum_tune_entries(int64_t *entries);

/*
 * Kernel timing, for measurement.  With enable = 1 (capacity 1..2^20 launches) the
 * main kernel of every later MTTKRP / TTMc call -- the streaming MTTKRP kernel
 * (kind 1) or the fused TTMc pass (kind 2), whichever the plan launches -- is
 * bracketed by two HIP events on the call's stream, so its own duration is known
 * apart from the call's small set-up and reduction kernels; launches past the
 * capacity are not recorded.  enable = 0 stops recording.  deinsum_kernel_times
 * waits for the recorded events, copies up to max_n (kind, milliseconds) pairs in
 * launch order into the host arrays, sets *n and forgets the records.
 */
deinsum_status deinsum_kernel_timing(int32_t enable, int64_t capacity);
deinsum_status deinsum_kernel_times(int64_t max_n, int32_t *kind, double *ms, int64_t *n);

/* Release the library's device workspace pools and plan caches. */
deinsum_status deinsum_shutdown(void);

/* Library version string. */
const char *deinsum_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DEINSUM_H */
