// abi.cpp -- the extern "C" entry points: argument validation, planning,
// workspace management and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "accuracy.h"
#include "internal.h"
#include "kernels.h"
#include "krp.h"
#include "mttkrp.h"
#include "plan.h"
#include "ttmc.h"
#include "tune.h"

namespace deinsum {

deinsum_status check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(DEINSUM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return DEINSUM_OK;
}

// ------------------------------------------------------------------ workspace pool
// Grow-only device buffers, one per (device, stream): calls with no workspace of
// their own on one stream reuse that stream's buffer in stream order, and calls on
// different streams never share one.  Up to kPoolStreams streams per device keep a
// buffer; a further stream takes the least recently used one after a device
// synchronise (nothing may still be using it).
struct Pool {
    void *stream = nullptr;
    void *ptr = nullptr;
    size_t bytes = 0;
    uint64_t last_use = 0;
};
constexpr int kPoolStreams = 16;
std::mutex g_pool_mu;
Pool g_pool[64][kPoolStreams];
uint64_t g_pool_clock = 0;

deinsum_status pool_get(size_t bytes, void *stream, void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return fail(DEINSUM_ERR_DEVICE, "workspace: no current HIP device");
    std::lock_guard<std::mutex> lk(g_pool_mu);
    Pool *p = nullptr, *lru = nullptr;
    for (Pool &q : g_pool[dev]) {
        if (q.ptr && q.stream == stream) {
            p = &q;
            break;
        }
        if (!lru || (!q.ptr && lru->ptr) || (q.ptr && lru->ptr && q.last_use < lru->last_use)) lru = &q;
    }
    if (!p) {
        p = lru;
        if (p->ptr) {  // evict: its stream's work may still be running
            if (hipDeviceSynchronize() != hipSuccess)
                return fail(DEINSUM_ERR_DEVICE, "workspace: device synchronise failed");
            (void)hipFree(p->ptr);
            *p = Pool{};
        }
        p->stream = stream;
    }
    p->last_use = ++g_pool_clock;
    if (p->bytes < bytes) {
        if (p->ptr) {
            // Earlier work on this stream may still use the old buffer.
            if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess)
                return fail(DEINSUM_ERR_DEVICE, "workspace: stream synchronise failed");
            (void)hipFree(p->ptr);
            p->ptr = nullptr;
            p->bytes = 0;
        }
        size_t want = std::max<size_t>(bytes, size_t(1) << 20);
        if (hipMalloc(&p->ptr, want) != hipSuccess) {
            (void)hipGetLastError();
            *p = Pool{};
            return fail(DEINSUM_ERR_NO_MEMORY, "workspace: hipMalloc of " + std::to_string(want) + " bytes failed");
        }
        p->bytes = want;
    }
    *out = p->ptr;
    return DEINSUM_OK;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return na && nb && pa < pb + nb && pb < pa + na;
}

deinsum_status check_dims(const deinsum_spec *spec, const int64_t *dims)
{
    if (!spec || !dims) return fail(DEINSUM_ERR_INVALID_ARG, "null spec or dims");
    if (spec->order < 2 || spec->order > DEINSUM_MAX_ORDER || spec->free_mode < 0 ||
        spec->free_mode >= spec->order || spec->n_factors != spec->order - 1)
        return fail(DEINSUM_ERR_INVALID_ARG, "spec is not a parsed deinsum_spec");
    // Every mode but the free one is contracted with exactly one factor operand.
    unsigned seen = 0;
    for (int k = 0; k < spec->n_factors; ++k) {
        const int m = spec->factor_mode[k];
        if (m < 0 || m >= spec->order || m == spec->free_mode || (seen >> m & 1u) || spec->operand_of_mode[m] != k)
            return fail(DEINSUM_ERR_INVALID_ARG, "spec is not a parsed deinsum_spec (factor modes)");
        seen |= 1u << m;
    }
    for (int m = 0; m < spec->order; ++m)
        if (dims[m] < 0) return fail(DEINSUM_ERR_SHAPE, "dims must be >= 0");
    // Element count must fit comfortably in 62 bits.
    long double total = 1;
    for (int m = 0; m < spec->order; ++m) total *= static_cast<long double>(dims[m]);
    if (total > 4.0e18L) return fail(DEINSUM_ERR_SHAPE, "tensor too large");
    return DEINSUM_OK;
}

namespace {

// ------------------------------------------------------------------ no-alloc scratch
// Workspace of deinsum_mttkrp_noalloc: a fixed device array that every device holding
// the library keeps until the process ends.  Host code never passes `scratch` itself
// (on the host it names a stand-in, not device memory): the device address is looked
// up once per device with hipGetSymbolAddress and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[DEINSUM_NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void *g_scratch_ptr[64];

deinsum_status scratch_get(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return fail(DEINSUM_ERR_DEVICE, "mttkrp_noalloc: no current HIP device");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(DEINSUM_ERR_DEVICE, std::string("mttkrp_noalloc: hipGetSymbolAddress(scratch) failed: ") +
                                                hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return DEINSUM_OK;
}

size_t x_elem_bytes(int prec)
{
    switch (prec) {
    case DEINSUM_PREC_FP64: return 8;
    case DEINSUM_PREC_BF16: return 2;
    case DEINSUM_PREC_FX20: return 3;  // algorithmic bytes; the buffer adds a header and plane padding
    default: return 4;
    }
}
size_t u_elem_bytes(int prec) { return prec == DEINSUM_PREC_FP64 ? 8 : 4; }
size_t dtype_bytes(int dt) { return dt == DEINSUM_F64 ? 8 : (dt == DEINSUM_F32 ? 4 : 2); }

deinsum_status resolve_opts(const deinsum_opts *in, deinsum_opts *o)
{
    deinsum_opts_init(o);
    if (in) *o = *in;
    if (o->precision < DEINSUM_PREC_FP64 || o->precision > DEINSUM_PREC_AUTO)
        return fail(DEINSUM_ERR_INVALID_ARG, "opts.precision is not a deinsum_precision");
    if (o->out_dtype != DEINSUM_F64 && o->out_dtype != DEINSUM_F32)
        return fail(DEINSUM_ERR_INVALID_ARG, "opts.out_dtype must be DEINSUM_F64 or DEINSUM_F32");
    if (o->precision == DEINSUM_PREC_FP64 && o->out_dtype != DEINSUM_F64)
        return fail(DEINSUM_ERR_INVALID_ARG, "the FP64 form writes an F64 output");
    if (o->workspace == nullptr && o->workspace_bytes != 0)
        return fail(DEINSUM_ERR_INVALID_ARG, "opts.workspace_bytes set without a workspace");
    if (o->deterministic != 0 && o->deterministic != 1)
        return fail(DEINSUM_ERR_INVALID_ARG, "opts.deterministic must be 0 or 1");
    if (o->precision == DEINSUM_PREC_AUTO) {
        if (!(o->tol > 0)) return fail(DEINSUM_ERR_INVALID_ARG, "DEINSUM_PREC_AUTO needs opts.tol > 0");
        if (o->x_dtype < DEINSUM_F64 || o->x_dtype > DEINSUM_FX20)
            return fail(DEINSUM_ERR_INVALID_ARG, "opts.x_dtype is not a deinsum_dtype");
        if (o->u_dtype != DEINSUM_F64 && o->u_dtype != DEINSUM_F32)
            return fail(DEINSUM_ERR_INVALID_ARG, "opts.u_dtype must be DEINSUM_F64 or DEINSUM_F32");
    }
    return DEINSUM_OK;
}

// ------------------------------------------------------------------ form choice (AUTO)
// Forms reading X stored as x_dtype with factors of u_dtype, cheapest first.
int form_candidates(int kind, int x_dtype, int u_dtype, int out[2])
{
    if (u_dtype == DEINSUM_F64) {
        if (x_dtype != DEINSUM_F64) return 0;
        out[0] = P_FP64;
        return 1;
    }
    switch (x_dtype) {
    case DEINSUM_F32:
        if (kind == DEINSUM_TTMC) {
            out[0] = P_FP32;
            return 1;
        }
        out[0] = P_BF16X3;
        out[1] = P_FP32;
        return 2;
    case DEINSUM_BF16: out[0] = P_BF16; return 1;
    case DEINSUM_FX20:
        out[0] = P_FX20;
        return 1;
    default: return 0;
    }
}

const char *form_name(int p)
{
    static const char *names[] = {"FP64", "FP32", "BF16", "BF16X3", "FX20", "AUTO"};
    return (p >= 0 && p <= 5) ? names[p] : "?";
}


__global__ void zero_fill_kernel(unsigned char *p, int64_t n)
{
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = 0;
}

deinsum_status zero_bytes(void *p, int64_t n, hipStream_t s)
{
    if (n <= 0) return DEINSUM_OK;
    const unsigned g = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 4096));
    zero_fill_kernel<<<g, 256, 0, s>>>(static_cast<unsigned char *>(p), n);
    return check_launch("zero_fill");
}

// ------------------------------------------------------------------ MTTKRP
struct MttkrpCall {
    MttkrpProblem pb;                  // as planned (last two modes merged if `merged`)
    MttkrpProblem orig;                // as called
    MttkrpPlan plan;
    const void *X;
    const void *U[DEINSUM_MAX_ORDER];  // by mode of the problem as called
    void *M;
    int out_dtype;
    bool merged = false;
    size_t krp_bytes = 0;              // merged factor at the start of the workspace (256-aligned)
    bool via_ttmc = false;             // order-3 mode 0 through the fused TTMc pass
    int ttmc_variant = 0;              // its TTMc plan_hint
    size_t ttmc_bytes = 0;
};

size_t call_workspace(const MttkrpCall &c) { return c.via_ttmc ? c.ttmc_bytes : c.krp_bytes + c.plan.workspace; }

// Mode 0 of an order-3 FP64 tensor can run through the fused TTMc pass: there a wave
// streams contiguous runs of one X row per K step, where the K-contiguous kernel
// reads 16 rows I_1 I_2 elements apart; the extra stage-2 work (the full R x R
// product whose diagonal is M) is small.  Taken when the tuner measured it faster,
// else for long rows of a tensor of at least 2^26 elements.
bool via_ttmc_eligible(const MttkrpProblem &pb, const deinsum_opts &o)
{
    return o.plan_hint == 0 && o.split_hint == 0 && pb.N == 3 && pb.n == 0 && pb.prec == P_FP64 && pb.R <= 64;
}

// The FX20, BF16 and BF16x3 matrix-core K step takes 32 contiguous elements of the
// contiguous mode (8 per lane), so a short or ragged last mode leaves lanes idle.
// When the free mode is n <= N-3, the last two modes are both contracted and X's
// memory is also an order N-1 tensor with them merged; its factor is their
// Khatri-Rao product (I_{N-2} I_{N-1} x R), built per call into the workspace.
// Only for N >= 4: at N = 3 the two merged modes are all the contracted modes, so
// their product would be the whole Khatri-Rao product, which is never stored.
bool merge_last_two(const MttkrpProblem &pb, int plan_hint)
{
    if (plan_hint != 0 || pb.N < 4 || pb.n > pb.N - 3) return false;
    if (pb.prec != P_FX20 && pb.prec != P_BF16 && pb.prec != P_BF16X3) return false;
    const int64_t ia = pb.dims[pb.N - 2], ib = pb.dims[pb.N - 1];
    if (ib % 32 == 0 && ib >= 256) return false;
    return ia * ib * pb.R * static_cast<int64_t>(u_elem_bytes(pb.prec)) <= (int64_t(64) << 20);
}

deinsum_status prepare_mttkrp(const deinsum_spec *spec, const int64_t *dims, int64_t R,
                              const deinsum_opts &o, MttkrpCall *call)
{
    if (deinsum_status st = check_dims(spec, dims)) return st;
    if (spec->kind != DEINSUM_MTTKRP) return fail(DEINSUM_ERR_INVALID_ARG, "spec is not an MTTKRP");
    if (R < 1 || R > DEINSUM_MAX_RANK)
        return fail(DEINSUM_ERR_SHAPE, "rank must be 1.." + std::to_string(DEINSUM_MAX_RANK));
    MttkrpProblem &pb = call->pb;
    pb.N = spec->order;
    pb.n = spec->free_mode;
    for (int m = 0; m < pb.N; ++m) pb.dims[m] = dims[m];
    pb.R = R;
    pb.prec = o.precision;
    call->out_dtype = o.out_dtype;
    call->orig = pb;
    call->merged = merge_last_two(pb, o.plan_hint);
    call->krp_bytes = 0;
    if (call->merged) {
        const int64_t ia = pb.dims[pb.N - 2], ib = pb.dims[pb.N - 1];
        call->krp_bytes = (static_cast<size_t>(ia * ib * R) * u_elem_bytes(pb.prec) + 255) / 256 * 256;
        pb.dims[pb.N - 2] = ia * ib;
        pb.dims[pb.N - 1] = 0;
        pb.N -= 1;
    }
    call->via_ttmc = false;
    if (!call->merged && via_ttmc_eligible(pb, o)) {
        TuneChoice tc;
        bool cached = tune_lookup(tune_key(TUNE_STREAM, pb), &tc);
        if (cached && tc.order != kTuneViaTtmc) {  // a stream-kernel entry counts only if that kernel exists
            int count = 0;
            const StreamKernelInfo *table = stream_kernels(&count);
            bool found = false;
            for (int i = 0; i < count; ++i) {
                const StreamKernelInfo &k = table[i];
                found |= k.prec == pb.prec && k.layout == L_KCONTIG && k.nt == tc.nt && k.ni == tc.ni &&
                         k.mt == tc.mt && k.xnt == tc.xnt;
            }
            cached = found;
        }
        if (cached) {
            call->via_ttmc = tc.order == kTuneViaTtmc;
            call->ttmc_variant = tc.split + 1;
        } else {
            call->via_ttmc = pb.dims[2] >= 256 && pb.dims[0] * pb.dims[1] * pb.dims[2] >= (int64_t(1) << 26);
            call->ttmc_variant = 0;
        }
        if (call->via_ttmc &&
            mttkrp_via_ttmc_workspace(pb.dims, R, pb.prec, call->ttmc_variant, &call->ttmc_bytes) != DEINSUM_OK) {
            call->ttmc_variant = 0;  // a cached variant that is no longer compiled: the default one
            if (deinsum_status st = mttkrp_via_ttmc_workspace(pb.dims, R, pb.prec, 0, &call->ttmc_bytes)) return st;
        }
    }
    return plan_mttkrp(pb, o.plan_hint, o.split_hint, &call->plan);
}

// Estimated error (accuracy.cpp) of the MTTKRP of this problem in form `prec`: the FP32
// chain length is the plan's slice of the matrix-core mode.  X is read only for FX20
// (its header, synchronising `s`); NULL there means the storage error is not known.
deinsum_status mttkrp_estimate(const deinsum_spec *spec, const int64_t *dims, int64_t R, int prec, const void *X,
                               hipStream_t s, double *est)
{
    deinsum_spec ms = *spec;
    ms.kind = DEINSUM_MTTKRP;
    deinsum_opts o;
    deinsum_opts_init(&o);
    o.precision = prec;
    o.out_dtype = prec == P_FP64 ? DEINSUM_F64 : DEINSUM_F32;
    ErrInputs in;
    in.prec = prec;
    in.order = spec->order;
    double nx = 1;
    bool empty = false;
    for (int m = 0; m < spec->order; ++m) {
        nx *= static_cast<double>(dims[m]);
        empty |= dims[m] == 0;
    }
    if (empty) {  // an empty sum (M = 0) or an empty output: exact
        *est = 0;
        return DEINSUM_OK;
    }
    in.L = nx / static_cast<double>(dims[spec->free_mode]);
    if (prec != P_FP64) {
        MttkrpCall c{};
        if (deinsum_status st = prepare_mttkrp(&ms, dims, R, o, &c)) return st;
        in.k32 = c.plan.slice;
    }
    if (prec == P_FX20 && X) {
        double e = 0;
        if (deinsum_status st = fx20_storage_error(X, static_cast<int64_t>(nx), s, &e)) return st;
        in.x_storage = e;
    }
    *est = estimate_error(in);
    return DEINSUM_OK;
}

// The same for TTMc: the fused pass sums over modes a and c in FP32 in the reduced forms.
// x_storage: FX20's storage error from the header (< 0: not known).
double ttmc_estimate(const deinsum_spec *spec, const int64_t *dims, int prec, double x_storage = -1)
{
    const int N = spec->order, n = spec->free_mode;
    ErrInputs in;
    in.prec = prec;
    in.order = N;
    double nx = 1;
    for (int m = 0; m < N; ++m) nx *= static_cast<double>(dims[m]);
    if (nx == 0) return 0;
    in.L = nx / static_cast<double>(dims[n]);
    if (N == 2) {
        in.k32 = static_cast<double>(dims[1 - n]);
    } else {
        const int c = N - 1, a = (n == N - 1 || N - 2 != n) ? N - 2 : N - 3;
        in.k32 = static_cast<double>(dims[a]) + (n == N - 1 ? 0.0 : static_cast<double>(dims[c]));
    }
    in.x_storage = x_storage;
    return estimate_error(in);
}

// Resolves opts->precision when it is DEINSUM_PREC_AUTO: the cheapest form reading
// opts->x_dtype / u_dtype storage whose estimate is at most opts->tol.  Without X
// (workspace queries) the FX20 form is taken unchecked: it is the only form reading
// that storage.  *est receives the chosen form's estimate (for an explicit form too
// when want_est; NaN when it was not computed).
deinsum_status resolve_form(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks, const void *X,
                            deinsum_opts *o, bool want_est, hipStream_t s, double *est)
{
    *est = NAN;
    if (deinsum_status st = check_dims(spec, dims)) return st;
    if (!ranks) return fail(DEINSUM_ERR_INVALID_ARG, "null ranks");
    const bool ttmc = spec->kind == DEINSUM_TTMC;
    auto estimate = [&](int prec, const void *x, double *e) -> deinsum_status {
        if (ttmc) {
            double xs = -1;
            if (prec == P_FX20 && x) {
                double nx = 1;
                for (int m = 0; m < spec->order; ++m) nx *= static_cast<double>(dims[m]);
                if (deinsum_status st = fx20_storage_error(x, static_cast<int64_t>(nx), s, &xs)) return st;
            }
            *e = ttmc_estimate(spec, dims, prec, xs);
            return DEINSUM_OK;
        }
        return mttkrp_estimate(spec, dims, ranks[0], prec, x, s, e);
    };
    if (o->precision != DEINSUM_PREC_AUTO) {
        if (want_est) return estimate(o->precision, X, est);
        return DEINSUM_OK;
    }
    int cand[2];
    const int nc = form_candidates(spec->kind, o->x_dtype, o->u_dtype, cand);
    if (nc == 0)
        return fail(DEINSUM_ERR_UNSUPPORTED, std::string("DEINSUM_PREC_AUTO: no compiled ") +
                                                 (ttmc ? "TTMc" : "MTTKRP") + " form reads this X / factor storage");
    double best = INFINITY;
    for (int i = 0; i < nc; ++i) {
        double e = 0;
        if (cand[i] == P_FX20 && !X) {
            o->precision = P_FX20;
            return DEINSUM_OK;
        }
        if (deinsum_status st = estimate(cand[i], X, &e)) return st;
        if (e <= o->tol) {
            o->precision = cand[i];
            *est = e;
            return DEINSUM_OK;
        }
        best = std::min(best, e);
    }
    char msg[192];
    std::snprintf(msg, sizeof(msg),
                  "DEINSUM_PREC_AUTO: no form reading this storage meets tol %.3g (best estimate %.3g); "
                  "store X for the tolerance (deinsum_choose_storage)",
                  o->tol, best);
    return fail(DEINSUM_ERR_UNSUPPORTED, msg);
}

deinsum_status run_mttkrp(const MttkrpCall &c, void *ws_all, hipStream_t s)
{
    const MttkrpProblem &pb = c.pb;
    const MttkrpPlan &p = c.plan;
    if (c.via_ttmc)
        return run_mttkrp_via_ttmc(pb.dims, pb.R, c.X, c.U[1], c.U[2], c.M, pb.prec, c.out_dtype, c.ttmc_variant,
                                   ws_all, c.ttmc_bytes, s);
    const void *Uf[DEINSUM_MAX_ORDER];  // factors by mode of the planned problem
    for (int m = 0; m < c.orig.N; ++m) Uf[m] = c.U[m];
    void *ws = ws_all;
    if (c.merged) {
        const int a = c.orig.N - 2;
        if (deinsum_status st = launch_krp2(c.U[a], c.U[a + 1], c.orig.dims[a], c.orig.dims[a + 1], pb.R,
                                            static_cast<int>(u_elem_bytes(pb.prec)), ws_all, s))
            return st;
        Uf[a] = ws_all;
        ws = static_cast<char *>(ws_all) + c.krp_bytes;
    }
    const int N = pb.N, n = pb.n;
    const bool kout = p.family == PLAN_MTTKRP_KOUT;
    const bool kcontig = p.family == PLAN_MTTKRP_KCONTIG || kout;
    const int gmode = kcontig ? N - 1 : N - 2;
    const size_t ub = u_elem_bytes(pb.prec), xb = x_elem_bytes(pb.prec);
    int64_t stride[DEINSUM_MAX_ORDER];
    {
        int64_t st = 1;
        for (int m = N - 1; m >= 0; --m) {
            stride[m] = st;
            st *= pb.dims[m];
        }
    }
    const int cols_pad = 16 * p.nt;
    const bool fx20 = pb.prec == P_FX20;
    int64_t nx = 1;
    for (int m = 0; m < N; ++m) nx *= pb.dims[m];
    const Fx20Header *hx = fx20 ? static_cast<const Fx20Header *>(c.X) : nullptr;
    for (int64_t cb = 0; cb < p.col_blocks; ++cb) {
        const int64_t col0 = cb * cols_pad;
        const int ncols = static_cast<int>(std::min<int64_t>(cols_pad, pb.R - col0));
        auto ucol = [&](int m) {
            return static_cast<const void *>(static_cast<const char *>(Uf[m]) + col0 * ub);
        };
        StreamArgs a{};
        a.X = fx20 ? static_cast<const void *>(static_cast<const char *>(c.X) + kFx20Header) : c.X;
        a.X2 = fx20 ? static_cast<const void *>(static_cast<const char *>(c.X) + fx20_lo_offset(nx)) : nullptr;
        a.Ug = ucol(gmode);
        a.ldu = pb.R;
        int k = 0;
        for (int m = 0; m < N; ++m) {
            if (m == n || m == gmode) continue;
            a.od.dim[k] = pb.dims[m];
            a.od.xstride[k] = stride[m];
            a.od.U[k] = ucol(m);
            ++k;
        }
        a.od.n_outer = k;
        a.In = pb.dims[n];
        a.Ig = pb.dims[gmode];
        a.stride_n = stride[n];
        a.stride_g = stride[gmode];
        a.ncols = ncols;
        a.n_tiles = static_cast<int>(p.n_tiles);
        a.n_kgroups = static_cast<int>(p.n_kgroups);
        a.wk = p.wk;
        a.O = 1;
        for (int i = 0; i < k; ++i) a.O *= a.od.dim[i];
        const int64_t w_rows = a.O;  // rows of the outer-weight table
        if (kout) {
            a.O = pb.dims[0];  // the walk's outer range: output rows (od holds mode 1)
            a.n_tiles = static_cast<int>(p.n_tiles);
        }
        a.o_per_chunk = p.o_per_chunk;
        a.order = p.order;
        a.xcd_remap = p.xcd;
        a.n_chunks = p.n_chunks;
        a.n_groups = p.groups;
        const int64_t contig = kcontig ? a.Ig : a.In;  // extent of the contiguous mode
        if (fx20)  // planes are 256-byte aligned; runs of 16 (K-contiguous) or MT (M-contiguous) elements
            a.vec_ok = kcontig ? (contig % 16 == 0) : (contig % p.mt == 0);
        else
            a.vec_ok = ((contig * xb) % 16 == 0) && (reinterpret_cast<uintptr_t>(c.X) % 16 == 0);
        a.P = static_cast<double *>(ws);
        double *W = reinterpret_cast<double *>(static_cast<char *>(ws) + p.w_offset);
        a.W = W;
        a.ldw = cols_pad;
        if (kout) {
            if (deinsum_status st = launch_kout_weights(a.od.U[0], pb.dims[1], pb.R, ncols, p.nt, pb.prec,
                                                        reinterpret_cast<float *>(W), s))
                return st;
        } else if (deinsum_status st = launch_outer_weights(a.od, w_rows, pb.R, ncols, cols_pad, pb.prec, W, s)) {
            return st;
        }
        const int kt = ktimer_begin(s, KK_MTTKRP_STREAM);
        const deinsum_status lst = launch_mttkrp_stream(*p.kernel, a, p.groups, p.waves, s);
        ktimer_end(kt, s);
        if (lst) return lst;
        // L_KOUT partials are [slice][row][col]: one tile of all I_0 rows per partial.
        if (deinsum_status st = launch_reduce_partials(a.P, p.parts, kout ? 1 : p.n_tiles,
                                                       kout ? static_cast<int>(pb.dims[0]) : p.tile_rows,
                                                       cols_pad, pb.dims[n], ncols,
                                                       static_cast<char *>(c.M) + col0 * dtype_bytes(c.out_dtype),
                                                       c.out_dtype, pb.R, hx, nx, s))
            return st;
    }
    return DEINSUM_OK;
}

// pb: the problem as called (algorithmic bytes and flops); p: the plan that ran;
// merged: the last two modes ran as one (" m2" ends the plan name); ttmc_variant >= 0:
// the call ran through the fused TTMc pass with that plan_hint (geometry fields zero).
void fill_report(deinsum_report *r, const MttkrpProblem &pb, const MttkrpPlan &p, size_t ws_bytes,
                 bool merged = false, int ttmc_variant = -1, double est = NAN)
{
    if (!r) return;
    std::memset(r, 0, sizeof(*r));
    r->precision = pb.prec;
    r->est_err = est;
    r->plan_id = p.family;
    r->tile_m = p.tile_rows;
    r->tile_k = p.slice;
    r->waves_per_group = p.waves;
    r->groups = p.groups * p.col_blocks;
    r->partials = p.parts;
    r->workspace_bytes = ws_bytes;
    double nx = 1, fsum = 0;
    for (int m = 0; m < pb.N; ++m) nx *= static_cast<double>(pb.dims[m]);
    for (int m = 0; m < pb.N; ++m)
        if (m != pb.n) fsum += static_cast<double>(pb.dims[m]) * static_cast<double>(pb.R);
    r->alg_bytes = nx * x_elem_bytes(pb.prec) + fsum * u_elem_bytes(pb.prec) +
                   static_cast<double>(pb.dims[pb.n]) * pb.R * 8.0;
    // Two-stage flops: GEMM over one mode (2 nX R) + Hadamard of each stage-1 row.
    const int g = (pb.n == pb.N - 1) ? pb.N - 2 : pb.N - 1;
    r->alg_flops = 2.0 * nx * pb.R + 2.0 * (nx / static_cast<double>(pb.dims[g])) * pb.R * std::max(1, pb.N - 2);
    std::snprintf(r->plan_name, sizeof(r->plan_name), "%s c%lld o%d x%d%s", p.name.c_str(),
                  static_cast<long long>(p.n_chunks), p.order, p.xcd, merged ? " m2" : "");
    if (ttmc_variant >= 0) {
        r->plan_id = 0;
        r->tile_m = r->tile_k = r->waves_per_group = 0;
        r->groups = r->partials = 0;
        std::snprintf(r->plan_name, sizeof(r->plan_name), "mttkrp_via_ttmc hint%d", ttmc_variant);
    }
}

// Median of the event-timed durations of `reps` back-to-back runs (one warm-up first).
template <class F>
deinsum_status time_median(F &&run, int reps, hipStream_t s, double *us)
{
    hipEvent_t ev[2];
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
        return fail(DEINSUM_ERR_DEVICE, "tune: event creation failed");
    std::vector<float> t;
    deinsum_status st = run();
    for (int r = 0; r < reps && st == DEINSUM_OK; ++r) {
        (void)hipEventRecord(ev[0], s);
        st = run();
        (void)hipEventRecord(ev[1], s);
        if (hipEventSynchronize(ev[1]) != hipSuccess) st = fail(DEINSUM_ERR_DEVICE, "tune: event sync failed");
        float ms = 0;
        (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
        t.push_back(ms);
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (st) return st;
    std::sort(t.begin(), t.end());
    *us = 1e3 * t[t.size() / 2];
    return DEINSUM_OK;
}

}  // namespace
}  // namespace deinsum

using namespace deinsum;

extern "C" {

void deinsum_opts_init(deinsum_opts *opts)
{
    if (!opts) return;
    std::memset(opts, 0, sizeof(*opts));
    opts->precision = DEINSUM_PREC_FP64;
    opts->out_dtype = DEINSUM_F64;
    opts->tol = 1e-12;
    opts->x_dtype = DEINSUM_F64;
    opts->u_dtype = DEINSUM_F64;
    opts->deterministic = 1;
}

const char *deinsum_version(void) { return "deinsum-mi355x 0.1 (gfx950)"; }

deinsum_status deinsum_parse(const char *spec, deinsum_spec *out) { return parse_spec(spec, out); }

deinsum_status deinsum_workspace_size(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks,
                                      const deinsum_opts *opts, size_t *bytes)
{
    if (!bytes || !ranks) return fail(DEINSUM_ERR_INVALID_ARG, "null ranks or bytes");
    deinsum_opts o;
    if (deinsum_status st = resolve_opts(opts, &o)) return st;
    if (o.precision == DEINSUM_PREC_AUTO) {
        double est = 0;
        if (deinsum_status st = resolve_form(spec, dims, ranks, nullptr, &o, false, nullptr, &est)) return st;
    }
    if (spec && spec->kind == DEINSUM_TTMC) return ttmc_workspace_size(spec, dims, ranks, o, bytes);
    if (spec && spec->kind == DEINSUM_MTTKRP_MM) {  // the MTTKRP's, then M in FP64
        deinsum_spec ms = *spec;
        ms.kind = DEINSUM_MTTKRP;
        MttkrpCall c{};
        if (deinsum_status st = prepare_mttkrp(&ms, dims, ranks[0], o, &c)) return st;
        *bytes = (call_workspace(c) + 255) / 256 * 256 + static_cast<size_t>(dims[spec->free_mode] * ranks[0]) * 8;
        clear_error();
        return DEINSUM_OK;
    }
    MttkrpCall c{};
    if (deinsum_status st = prepare_mttkrp(spec, dims, ranks[0], o, &c)) return st;
    *bytes = call_workspace(c);
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_mttkrp(const deinsum_spec *spec, const int64_t *dims, int64_t R, const void *X,
                              const void *const *U, void *M, const deinsum_opts *opts, void *stream)
{
    deinsum_opts o;
    if (deinsum_status st = resolve_opts(opts, &o)) return st;
    MttkrpCall c{};
    if (deinsum_status st = check_dims(spec, dims)) return st;
    if (spec->kind != DEINSUM_MTTKRP) return fail(DEINSUM_ERR_INVALID_ARG, "spec is not an MTTKRP");
    if (R < 1 || R > DEINSUM_MAX_RANK)
        return fail(DEINSUM_ERR_SHAPE, "rank must be 1.." + std::to_string(DEINSUM_MAX_RANK));
    if (!U || !M) return fail(DEINSUM_ERR_INVALID_ARG, "null factor table or output");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double est = NAN;
    if (o.precision == DEINSUM_PREC_AUTO || o.report) {
        const int64_t r1[1] = {R};
        if (deinsum_status st = resolve_form(spec, dims, r1, X, &o, o.report != nullptr, s, &est)) return st;
        if (o.precision == DEINSUM_PREC_FP64 && o.out_dtype != DEINSUM_F64)
            return fail(DEINSUM_ERR_INVALID_ARG, "the FP64 form writes an F64 output");
    }
    const int N = spec->order, n = spec->free_mode;
    int64_t nx = 1;
    bool empty = false;
    for (int m = 0; m < N; ++m) {
        nx *= dims[m];
        if (dims[m] == 0) empty = true;
    }
    const size_t xb = x_elem_bytes(o.precision), ub = u_elem_bytes(o.precision);
    const size_t mbytes = static_cast<size_t>(dims[n]) * R * dtype_bytes(o.out_dtype);
    if (!X && nx) return fail(DEINSUM_ERR_INVALID_ARG, "null X");
    for (int k = 0; k < N - 1; ++k) {
        const int m = spec->factor_mode[k];
        if (!U[k] && dims[m]) return fail(DEINSUM_ERR_INVALID_ARG, "null factor operand " + std::to_string(k));
        if (overlaps(M, mbytes, U[k], static_cast<size_t>(dims[m]) * R * ub))
            return fail(DEINSUM_ERR_INVALID_ARG, "output overlaps factor operand " + std::to_string(k));
        c.U[m] = U[k];
    }
    const bool fx20 = o.precision == DEINSUM_PREC_FX20;
    const size_t xbytes = fx20 ? static_cast<size_t>(fx20_bytes(nx)) : static_cast<size_t>(nx) * xb;
    if (overlaps(M, mbytes, X, xbytes)) return fail(DEINSUM_ERR_INVALID_ARG, "output overlaps X");
    if (reinterpret_cast<uintptr_t>(M) % dtype_bytes(o.out_dtype) != 0 ||
        reinterpret_cast<uintptr_t>(X) % (fx20 ? 256 : xb) != 0)
        return fail(DEINSUM_ERR_INVALID_ARG, fx20 ? "an FX20 X buffer must be 256-byte aligned"
                                                  : "X and M must be aligned to their element size");
    if (dims[n] == 0) { clear_error(); return DEINSUM_OK; }
    if (empty) {  // an empty sum: M = 0
        if (deinsum_status st = zero_bytes(M, static_cast<int64_t>(mbytes), s)) return st;
        clear_error();
        return DEINSUM_OK;
    }
    if (deinsum_status st = prepare_mttkrp(spec, dims, R, o, &c)) return st;
    c.X = X;
    c.M = M;
    void *ws = o.workspace;
    if (ws) {
        if (o.workspace_bytes < call_workspace(c))
            return fail(DEINSUM_ERR_NO_MEMORY, "workspace too small: need " + std::to_string(call_workspace(c)) + " bytes");
    } else if (deinsum_status st = pool_get(call_workspace(c), stream, &ws)) {
        return st;
    }
    fill_report(o.report, c.orig, c.plan, call_workspace(c), c.merged, c.via_ttmc ? c.ttmc_variant : -1, est);
    if (deinsum_status st = run_mttkrp(c, ws, s)) return st;
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_mttkrp_noalloc(const deinsum_spec *spec, const int64_t *dims, int64_t R, const void *X,
                                      const void *const *U, void *M, const deinsum_opts *opts, void *stream)
{
    deinsum_opts o;
    if (deinsum_status st = resolve_opts(opts, &o)) return st;
    if (o.workspace) return fail(DEINSUM_ERR_INVALID_ARG, "mttkrp_noalloc: opts.workspace must be NULL");
    // The plan's workspace must fit the fixed array; checked before anything is enqueued.
    if (deinsum_status st = check_dims(spec, dims)) return st;
    if (spec->kind != DEINSUM_MTTKRP) return fail(DEINSUM_ERR_INVALID_ARG, "spec is not an MTTKRP");
    const int64_t r[1] = {R};
    size_t need = 0;
    if (deinsum_status st = deinsum_workspace_size(spec, dims, r, &o, &need)) return st;
    if (need > DEINSUM_NOALLOC_SCRATCH_BYTES)
        return fail(DEINSUM_ERR_NO_MEMORY, "mttkrp_noalloc: the plan needs " + std::to_string(need) +
                                               " bytes of workspace, more than the fixed " +
                                               std::to_string(static_cast<size_t>(DEINSUM_NOALLOC_SCRATCH_BYTES)) +
                                               "-byte scratch array; call deinsum_mttkrp");
    void *ptr = nullptr;
    if (deinsum_status st = scratch_get(&ptr)) return st;
    o.workspace = ptr;
    o.workspace_bytes = DEINSUM_NOALLOC_SCRATCH_BYTES;
    return deinsum_mttkrp(spec, dims, R, X, U, M, &o, stream);
}

deinsum_status deinsum_mttkrp_mm(const deinsum_spec *spec, const int64_t *dims, int64_t R, int64_t L,
                                 const void *X, const void *const *U, const void *C, void *Y,
                                 const deinsum_opts *opts, void *stream)
{
    deinsum_opts o;
    if (deinsum_status st = resolve_opts(opts, &o)) return st;
    if (deinsum_status st = check_dims(spec, dims)) return st;
    if (spec->kind != DEINSUM_MTTKRP_MM) return fail(DEINSUM_ERR_INVALID_ARG, "spec is not an MTTKRP-GEMM chain");
    if (R < 1 || R > DEINSUM_MAX_RANK)
        return fail(DEINSUM_ERR_SHAPE, "rank must be 1.." + std::to_string(DEINSUM_MAX_RANK));
    if (L < 1 || L > 4096) return fail(DEINSUM_ERR_SHAPE, "chain width L must be 1..4096");
    if (!C || !Y) return fail(DEINSUM_ERR_INVALID_ARG, "null C or Y");
    if (o.precision == DEINSUM_PREC_AUTO) {  // the MTTKRP's form; the product is summed in FP64
        const int64_t r1[1] = {R};
        double est = 0;
        if (deinsum_status st = resolve_form(spec, dims, r1, X, &o, false, static_cast<hipStream_t>(stream), &est))
            return st;
        if (o.precision == DEINSUM_PREC_FP64 && o.out_dtype != DEINSUM_F64)
            return fail(DEINSUM_ERR_INVALID_ARG, "the FP64 form writes an F64 output");
    }
    const int n = spec->free_mode;
    const size_t cb = u_elem_bytes(o.precision), yb = dtype_bytes(o.out_dtype);
    const size_t ybytes = static_cast<size_t>(dims[n] * L) * yb;
    if (overlaps(Y, ybytes, C, static_cast<size_t>(R * L) * cb)) return fail(DEINSUM_ERR_INVALID_ARG, "Y overlaps C");
    {
        int64_t nx = 1;
        for (int m = 0; m < spec->order; ++m) nx *= dims[m];
        const size_t xbytes = o.precision == DEINSUM_PREC_FX20 ? static_cast<size_t>(fx20_bytes(nx))
                                                                : static_cast<size_t>(nx) * x_elem_bytes(o.precision);
        if (overlaps(Y, ybytes, X, xbytes)) return fail(DEINSUM_ERR_INVALID_ARG, "Y overlaps X");
        if (U)
            for (int k = 0; k < spec->order - 1; ++k)
                if (overlaps(Y, ybytes, U[k], static_cast<size_t>(dims[spec->factor_mode[k]] * R) * cb))
                    return fail(DEINSUM_ERR_INVALID_ARG, "Y overlaps factor operand " + std::to_string(k));
    }
    deinsum_spec ms = *spec;
    ms.kind = DEINSUM_MTTKRP;
    const int64_t ranks[2] = {R, L};
    size_t total = 0;
    if (deinsum_status st = deinsum_workspace_size(spec, dims, ranks, &o, &total)) return st;
    const size_t mbytes = static_cast<size_t>(dims[n] * R) * 8;
    const size_t mws = total - mbytes;  // the MTTKRP's workspace, 256-aligned
    void *ws = o.workspace;
    if (ws) {
        if (o.workspace_bytes < total)
            return fail(DEINSUM_ERR_NO_MEMORY, "workspace too small: need " + std::to_string(total) + " bytes");
    } else if (deinsum_status st = pool_get(total, stream, &ws)) {
        return st;
    }
    double *M = reinterpret_cast<double *>(static_cast<char *>(ws) + mws);
    if (overlaps(Y, ybytes, M, mbytes)) return fail(DEINSUM_ERR_INVALID_ARG, "Y overlaps the workspace");
    deinsum_opts o2 = o;
    o2.out_dtype = DEINSUM_F64;
    o2.workspace = ws;
    o2.workspace_bytes = mws;
    o2.report = o.report;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (deinsum_status st = deinsum_mttkrp(&ms, dims, R, X, U, M, &o2, stream)) return st;
    if (dims[n] == 0) return DEINSUM_OK;
    if (deinsum_status st = launch_chain_mm(M, C, static_cast<int>(cb), dims[n], R, L, Y, o.out_dtype, s)) return st;
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_tune_mttkrp(const deinsum_spec *spec, const int64_t *dims, int64_t R, const void *X,
                                   const void *const *U, void *M, const deinsum_opts *opts, int32_t reps,
                                   deinsum_report *best, void *stream)
{
    if (reps < 1 || reps > 1000) return fail(DEINSUM_ERR_INVALID_ARG, "tune: reps must be 1..1000");
    deinsum_opts o;
    if (deinsum_status st = resolve_opts(opts, &o)) return st;
    if (o.precision == DEINSUM_PREC_AUTO) {
        const int64_t r1[1] = {R};
        double est = 0;
        if (!spec) return fail(DEINSUM_ERR_INVALID_ARG, "null spec");
        if (deinsum_status st = resolve_form(spec, dims, r1, X, &o, false, static_cast<hipStream_t>(stream), &est))
            return st;
    }
    o.plan_hint = 0;
    o.split_hint = 0;
    o.workspace = nullptr;
    o.workspace_bytes = 0;
    o.report = nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // Validates every argument exactly as a plain call does.
    if (deinsum_status st = deinsum_mttkrp(spec, dims, R, X, U, M, &o, stream)) return st;
    MttkrpCall c{};
    for (int m = 0; m < spec->order; ++m)
        if (dims[m] == 0) return DEINSUM_OK;  // nothing to tune
    if (deinsum_status st = prepare_mttkrp(spec, dims, R, o, &c)) return st;
    for (int k = 0; k < spec->order - 1; ++k) c.U[spec->factor_mode[k]] = U[k];
    c.X = X;
    c.M = M;
    const int layout = c.pb.n == c.pb.N - 1 ? L_MCONTIG : L_KCONTIG;
    const bool try_kout = c.pb.N == 3 && c.pb.n == 0 && c.pb.prec != P_FP64 && c.pb.dims[0] < (int64_t(1) << 31);
    const char *vb = std::getenv("DEINSUM_TUNE_VERBOSE");
    const bool verbose = vb && vb[0] && vb[0] != '0';
    int count = 0;
    const StreamKernelInfo *table = stream_kernels(&count);
    double best_us = -1;
    MttkrpPlan best_plan;
    TuneChoice choice;
    for (int i = 0; i < count; ++i) {
        const StreamKernelInfo &k = table[i];
        const bool kout = k.layout == L_KOUT;
        if (k.prec != c.pb.prec || (k.layout != layout && !(kout && try_kout))) continue;
        MttkrpPlan p0;
        if (plan_geometry(c.pb, &k, 0, &p0) != DEINSUM_OK) continue;
        int splits[8];
        const int ns = tune_splits(p0.n_chunks, p0.O, splits);
        for (int si = 0; si < ns; ++si)
            for (int variant = 0; variant < (kout ? 1 : 4); ++variant) {
                MttkrpCall cc = c;
                cc.via_ttmc = false;
                if (deinsum_status st = plan_geometry(c.pb, &k, splits[si], &cc.plan)) return st;
                cc.plan.order = variant & 1;
                cc.plan.xcd = variant >> 1;
                void *ws = nullptr;
                if (deinsum_status st = pool_get(call_workspace(cc), stream, &ws)) return st;
                double us = 0;
                if (deinsum_status st = time_median([&] { return run_mttkrp(cc, ws, s); }, reps, s, &us)) return st;
                if (verbose)
                    std::fprintf(stderr, "[deinsum tune] %s split %d order %d xcd %d: %.1f us\n", cc.plan.name.c_str(),
                                 splits[si], cc.plan.order, cc.plan.xcd, us);
                if (best_us < 0 || us < best_us) {
                    best_us = us;
                    best_plan = cc.plan;
                    choice.nt = k.nt;
                    choice.ni = k.ni;
                    choice.mt = k.mt;
                    choice.xnt = k.xnt;
                    choice.split = splits[si];
                    choice.order = kout ? kTuneKout : cc.plan.order;
                    choice.xcd = cc.plan.xcd;
                    choice.us = us;
                }
            }
    }
    int best_ttmc = -1;  // plan_hint of the fused TTMc pass when it wins
    if (!c.merged && via_ttmc_eligible(c.pb, o)) {
        for (int v = 1; v <= 64; ++v) {
            MttkrpCall cc = c;
            cc.via_ttmc = true;
            cc.ttmc_variant = v;
            if (mttkrp_via_ttmc_workspace(c.pb.dims, c.pb.R, c.pb.prec, v, &cc.ttmc_bytes) != DEINSUM_OK) break;
            void *ws = nullptr;
            if (deinsum_status st = pool_get(cc.ttmc_bytes, stream, &ws)) return st;
            double us = 0;
            if (deinsum_status st = time_median([&] { return run_mttkrp(cc, ws, s); }, reps, s, &us)) return st;
            if (verbose) std::fprintf(stderr, "[deinsum tune] mttkrp_via_ttmc hint %d: %.1f us\n", v, us);
            if (best_us < 0 || us < best_us) {
                best_us = us;
                best_ttmc = v;
                choice = TuneChoice{};
                choice.nt = choice.ni = choice.mt = 1;
                choice.order = kTuneViaTtmc;
                choice.split = v - 1;
                choice.us = us;
            }
        }
    }
    if (best_us < 0) return fail(DEINSUM_ERR_UNSUPPORTED, "tune: no candidate plan");
    tune_store(tune_key(TUNE_STREAM, c.pb), choice);
    if (best) {
        MttkrpCall cb = c;
        cb.plan = best_plan;
        cb.via_ttmc = best_ttmc >= 0;
        if (cb.via_ttmc)
            (void)mttkrp_via_ttmc_workspace(c.pb.dims, c.pb.R, c.pb.prec, best_ttmc, &cb.ttmc_bytes);
        fill_report(best, c.orig, best_plan, call_workspace(cb), c.merged, best_ttmc);
        best->tuned_us = best_us;
    }
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_tune_ttmc(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks, const void *X,
                                 const void *const *U, void *Y, const deinsum_opts *opts, int32_t reps,
                                 deinsum_report *best, void *stream)
{
    if (reps < 1 || reps > 1000) return fail(DEINSUM_ERR_INVALID_ARG, "tune_ttmc: reps must be 1..1000");
    deinsum_opts o;
    if (deinsum_status st = resolve_opts(opts, &o)) return st;
    if (o.precision == DEINSUM_PREC_AUTO) {
        double est = 0;
        if (!spec) return fail(DEINSUM_ERR_INVALID_ARG, "null spec");
        if (deinsum_status st = resolve_form(spec, dims, ranks, X, &o, false, static_cast<hipStream_t>(stream), &est))
            return st;
    }
    o.workspace = nullptr;
    o.workspace_bytes = 0;
    o.report = nullptr;
    o.plan_hint = 1;  // validates every argument as a plain call does (variant 0)
    if (deinsum_status st = deinsum_ttmc(spec, dims, ranks, X, U, Y, &o, stream)) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double best_us = -1;
    int best_v = 0;
    const int nvar = (spec->order == 2 && spec->free_mode == 0) ? 1 : 64;  // that case runs the MTTKRP kernel
    int count = 0;
    for (int v = 0; v < nvar; ++v) {
        o.plan_hint = v + 1;
        size_t need = 0;
        if (deinsum_workspace_size(spec, dims, ranks, &o, &need) != DEINSUM_OK) break;  // no variant v
        count = v + 1;
    }
    // Two interleaved passes over the variants, each variant keeping its faster median,
    // so that clock or thermal drift during the sweep does not favour one position.
    std::vector<double> us_of(static_cast<size_t>(count), -1.0);
    for (int pass = 0; pass < 2; ++pass)
        for (int v = 0; v < count; ++v) {
            o.plan_hint = v + 1;
            double us = 0;
            if (deinsum_status st = time_median([&] { return deinsum_ttmc(spec, dims, ranks, X, U, Y, &o, stream); },
                                                reps, s, &us))
                return st;
            if (us_of[v] < 0 || us < us_of[v]) us_of[v] = us;
        }
    for (int v = 0; v < count; ++v)
        if (best_us < 0 || us_of[v] < best_us) {
            best_us = us_of[v];
            best_v = v;
        }
    TuneChoice c;
    c.nt = c.ni = c.mt = 1;
    c.split = best_v;  // TTMc entries: the fused-kernel variant
    c.us = best_us;
    tune_store(ttmc_tune_key(spec, dims, ranks, o.precision), c);
    if (best) {
        std::memset(best, 0, sizeof(*best));
        std::snprintf(best->plan_name, sizeof(best->plan_name), "ttmc fused variant %d", best_v);
        best->tuned_us = best_us;
    }
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_ttmc(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks, const void *X,
                            const void *const *U, void *Y, const deinsum_opts *opts, void *stream)
{
    deinsum_opts o;
    if (deinsum_status st = resolve_opts(opts, &o)) return st;
    if (deinsum_status st = check_dims(spec, dims)) return st;
    if (spec->kind != DEINSUM_TTMC) return fail(DEINSUM_ERR_INVALID_ARG, "spec is not a TTMc");
    if (!ranks) return fail(DEINSUM_ERR_INVALID_ARG, "null ranks");
    double est = NAN;
    if (o.precision == DEINSUM_PREC_AUTO || o.report) {
        if (deinsum_status st = resolve_form(spec, dims, ranks, X, &o, o.report != nullptr,
                                             static_cast<hipStream_t>(stream), &est))
            return st;
        if (o.precision == DEINSUM_PREC_FP64 && o.out_dtype != DEINSUM_F64)
            return fail(DEINSUM_ERR_INVALID_ARG, "the FP64 form writes an F64 output");
    }
    void *ws = o.workspace;
    size_t need = 0;
    if (deinsum_status st = ttmc_workspace_size(spec, dims, ranks, o, &need)) return st;
    if (ws) {
        if (o.workspace_bytes < need)
            return fail(DEINSUM_ERR_NO_MEMORY, "workspace too small: need " + std::to_string(need) + " bytes");
    } else if (need) {
        if (deinsum_status st = pool_get(need, stream, &ws)) return st;
    }
    if (deinsum_status st = run_ttmc(spec, dims, ranks, X, U, Y, o, ws, need, static_cast<hipStream_t>(stream)))
        return st;
    if (o.report) {
        deinsum_report *r = o.report;
        std::memset(r, 0, sizeof(*r));
        r->precision = o.precision;
        r->est_err = est;
        r->workspace_bytes = need;
        double nx = 1, ny = 1, fac = 0;
        for (int m = 0; m < spec->order; ++m) {
            nx *= static_cast<double>(dims[m]);
            if (m == spec->free_mode) {
                ny *= static_cast<double>(dims[m]);
            } else {
                const double rm = static_cast<double>(ranks[spec->operand_of_mode[m]]);
                ny *= rm;
                fac += static_cast<double>(dims[m]) * rm;
            }
        }
        r->alg_bytes = nx * static_cast<double>(x_elem_bytes(o.precision)) +
                       fac * static_cast<double>(u_elem_bytes(o.precision)) + ny * dtype_bytes(o.out_dtype);
        std::snprintf(r->plan_name, sizeof(r->plan_name), "ttmc %s", form_name(o.precision));
    }
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_estimate_error(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks,
                                      const void *X, const deinsum_opts *opts, int32_t *precision, double *est_err,
                                      void *stream)
{
    if (!precision || !est_err) return fail(DEINSUM_ERR_INVALID_ARG, "estimate_error: null output");
    deinsum_opts o;
    if (deinsum_status st = resolve_opts(opts, &o)) return st;
    if (!spec) return fail(DEINSUM_ERR_INVALID_ARG, "null spec");
    if (o.precision == DEINSUM_PREC_FX20 && !X)
        return fail(DEINSUM_ERR_INVALID_ARG, "estimate_error: the FX20 estimate reads X's header");
    if (o.precision == DEINSUM_PREC_AUTO && o.x_dtype == DEINSUM_FX20 && !X)
        return fail(DEINSUM_ERR_INVALID_ARG, "estimate_error: the FX20 estimate reads X's header");
    if (spec->kind == DEINSUM_TTMC && o.precision == DEINSUM_PREC_BF16X3)
        return fail(DEINSUM_ERR_UNSUPPORTED, "TTMc supports the FP64, FP32, BF16 and FX20 forms");
    double est = NAN;
    if (deinsum_status st = resolve_form(spec, dims, ranks, X, &o, true, static_cast<hipStream_t>(stream), &est))
        return st;
    *precision = o.precision;
    *est_err = est;
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_choose_storage(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks, double tol,
                                      double max_abs, double rms, int32_t *x_dtype, int32_t *precision,
                                      double *est_err)
{
    if (!spec || !dims || !ranks || !x_dtype || !precision || !est_err)
        return fail(DEINSUM_ERR_INVALID_ARG, "choose_storage: null argument");
    if (!(tol > 0)) return fail(DEINSUM_ERR_INVALID_ARG, "choose_storage: tol must be > 0");
    if (deinsum_status st = check_dims(spec, dims)) return st;
    const bool ttmc = spec->kind == DEINSUM_TTMC;
    // (storage, form), cheapest storage first; within F32 the faster form first.
    const int order_x[] = {DEINSUM_BF16, DEINSUM_FX20, DEINSUM_F32, DEINSUM_F32, DEINSUM_F64};
    const int order_p[] = {P_BF16, P_FX20, P_BF16X3, P_FP32, P_FP64};
    double best = INFINITY;
    for (int i = 0; i < 5; ++i) {
        const int p = order_p[i];
        if (ttmc && p == P_BF16X3) continue;
        double e = 0;
        if (p == P_FX20) {
            const double dx = fx20_storage_model(max_abs, rms);
            if (!(dx >= 0)) continue;  // no statistics of X: FX20 not considered
            if (ttmc) {
                e = ttmc_estimate(spec, dims, P_FX20, dx);
                if (e <= tol) {
                    *x_dtype = order_x[i];
                    *precision = p;
                    *est_err = e;
                    clear_error();
                    return DEINSUM_OK;
                }
                best = std::min(best, e);
                continue;
            }
            ErrInputs in;
            in.prec = P_FX20;
            in.order = spec->order;
            double nx = 1;
            for (int m = 0; m < spec->order; ++m) nx *= static_cast<double>(dims[m]);
            in.L = nx > 0 ? nx / static_cast<double>(dims[spec->free_mode]) : 1;
            deinsum_spec ms = *spec;
            ms.kind = DEINSUM_MTTKRP;
            deinsum_opts o;
            deinsum_opts_init(&o);
            o.precision = P_FX20;
            o.out_dtype = DEINSUM_F32;
            MttkrpCall c{};
            if (nx > 0) {
                if (deinsum_status st = prepare_mttkrp(&ms, dims, ranks[0], o, &c)) return st;
                in.k32 = c.plan.slice;
            }
            in.x_storage = dx;
            e = nx > 0 ? estimate_error(in) : 0.0;
        } else if (ttmc) {
            e = ttmc_estimate(spec, dims, p);
        } else if (deinsum_status st = mttkrp_estimate(spec, dims, ranks[0], p, nullptr, nullptr, &e)) {
            return st;
        }
        if (e <= tol) {
            *x_dtype = order_x[i];
            *precision = p;
            *est_err = e;
            clear_error();
            return DEINSUM_OK;
        }
        best = std::min(best, e);
    }
    char msg[160];
    std::snprintf(msg, sizeof(msg), "choose_storage: no storage meets tol %.3g (best estimate %.3g)", tol, best);
    return fail(DEINSUM_ERR_UNSUPPORTED, msg);
}

deinsum_status deinsum_synth_fill(void *X, int32_t dtype, int64_t count, uint64_t seed, int64_t offset, int32_t dist,
                                  void *stream)
{
    if (count < 0 || offset < 0) return fail(DEINSUM_ERR_INVALID_ARG, "negative count or offset");
    if (count == 0) return DEINSUM_OK;
    if (!X) return fail(DEINSUM_ERR_INVALID_ARG, "null X");
    if (dist < 0 || dist > 2) return fail(DEINSUM_ERR_INVALID_ARG, "dist must be 0 (uniform), 1 (int5) or 2 (int3)");
    return launch_synth_fill(X, dtype, count, seed, offset, dist, static_cast<hipStream_t>(stream));
}

deinsum_status deinsum_convert(const void *src, int32_t src_dtype, void *dst, int32_t dst_dtype, int64_t count,
                               void *stream)
{
    if (count < 0) return fail(DEINSUM_ERR_INVALID_ARG, "negative count");
    if (count == 0) return DEINSUM_OK;
    if (!src || !dst) return fail(DEINSUM_ERR_INVALID_ARG, "null pointer");
    if (overlaps(src, count * dtype_bytes(src_dtype), dst, count * dtype_bytes(dst_dtype)))
        return fail(DEINSUM_ERR_INVALID_ARG, "convert: buffers overlap");
    return launch_convert(src, src_dtype, dst, dst_dtype, count, static_cast<hipStream_t>(stream));
}

deinsum_status deinsum_shutdown(void)
{
    std::lock_guard<std::mutex> lk(g_pool_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (int d = 0; d < 64; ++d) {
        bool synced = false;
        for (Pool &q : g_pool[d]) {
            if (!q.ptr) continue;
            if (!synced) {
                (void)hipSetDevice(d);
                (void)hipDeviceSynchronize();
                synced = true;
            }
            (void)hipFree(q.ptr);
            q = Pool{};
        }
    }
    (void)hipSetDevice(cur);
    clear_error();
    return DEINSUM_OK;
}

}  // extern "C"
