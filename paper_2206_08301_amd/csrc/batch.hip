// batch.hip -- many MTTKRP jobs of uneven shape and rank in one persistent launch.
//
// An epoch is an asynchronous copy of the jobs' descriptors (pinned host ->
// device, only the jobs of this launch) followed by one replay of a captured
// hipGraph:
//   queue reset (a kernel; no memset node)
//   -> batched outer-weight table of every job
//   -> ONE persistent kernel: each workgroup takes the next unit of the global
//      work queue (a vector atomic counter), finds its job by binary search over
//      the jobs' unit ranges and runs the job's streaming unit (the same device
//      code as the per-call kernels, dispatched on the job's variant)
//   -> batched fixed-order reduction of every job's partial tiles.
// Every size is read from the device descriptor, so one captured graph serves
// every epoch; a job's result depends only on its own plan, never on the other
// jobs in the batch (bitwise identical alone or in a mix).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "batch.h"
#include "internal.h"
#include "kernels.h"
#include "mttkrp.h"
#include "plan.h"
#include "stream.h"
#include "tune.h"

namespace deinsum {

namespace {

using namespace dev;

// Variant list of the persistent kernel (index = BatchJob::variant).
#define BATCH_VARIANTS(X)                                  \
    X(0, P_FP64, L_KCONTIG, 1, 8, 1)                       \
    X(1, P_FP64, L_KCONTIG, 2, 4, 1)                       \
    X(2, P_FP64, L_KCONTIG, 4, 4, 1)                       \
    X(3, P_FP64, L_MCONTIG, 1, 8, 2)                       \
    X(4, P_FP64, L_MCONTIG, 2, 4, 2)                       \
    X(5, P_FP64, L_MCONTIG, 4, 4, 1)                       \
    X(6, P_FP32, L_KCONTIG, 1, 8, 1)                       \
    X(7, P_FP32, L_KCONTIG, 2, 8, 1)                       \
    X(8, P_FP32, L_KCONTIG, 4, 4, 1)                       \
    X(9, P_FP32, L_MCONTIG, 1, 8, 2)                       \
    X(10, P_FP32, L_MCONTIG, 2, 8, 2)                      \
    X(11, P_FP32, L_MCONTIG, 4, 4, 1)

constexpr int kBatchNBUF = 2;

#define LDS_OF(i, P, L, NT, NI, MT) unit_lds_elems<L, NT, MT>(),
constexpr int kLdsSizes[] = {BATCH_VARIANTS(LDS_OF)};
#undef LDS_OF
constexpr int max_lds()
{
    int m = 0;
    for (int v : kLdsSizes) m = v > m ? v : m;
    return m;
}

__device__ __forceinline__ int find_job(const BatchJob *jobs, int njobs, int64_t key, int which)
{
    // last job whose range begins at or before key
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t b = which == 0 ? jobs[mid].unit_begin : (which == 1 ? jobs[mid].w_begin : jobs[mid].out_begin);
        if (b <= key) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void batch_reset_kernel(int *queue) { *queue = 0; }

__global__ void __launch_bounds__(256) batch_weights_kernel(const BatchHeader *h, const BatchJob *jobs)
{
    const int64_t total = h->total_w;
    const int njobs = h->njobs;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const BatchJob &j = jobs[find_job(jobs, njobs, e, 1)];
        const int64_t le = e - j.w_begin;
        int64_t o = le / j.a.ldw;
        const int col = static_cast<int>(le % j.a.ldw);
        double w = 0.0;
        if (col < j.a.ncols) {
            w = 1.0;
            for (int m = j.a.od.n_outer - 1; m >= 0; --m) {
                const int64_t i = o % j.a.od.dim[m];
                o /= j.a.od.dim[m];
                w *= ld_u(j.a.od.U[m], i * j.ldu + col, j.prec);
            }
        }
        const_cast<double *>(j.a.W)[le] = w;
    }
}

__global__ void __launch_bounds__(256, 2) batch_main_kernel(const BatchHeader *h, const BatchJob *jobs, int *queue)
{
    __shared__ double lds[max_lds()];
    __shared__ int s_unit;
    const int64_t total = h->total_units;
    const int njobs = h->njobs;
    for (;;) {
        __syncthreads();  // LDS of the previous unit fully consumed
        if (threadIdx.x == 0) s_unit = atomicAdd(queue, 1);
        __syncthreads();
        const int64_t unit = __builtin_amdgcn_readfirstlane(s_unit);
        if (unit >= total) break;
        const int ji = __builtin_amdgcn_readfirstlane(find_job(jobs, njobs, unit, 0));
        const BatchJob &j = jobs[ji];
        const int64_t b = unit - j.unit_begin;
        switch (j.variant) {
#define CASE(i, P, L, NT, NI, MT) \
    case i: stream_unit<P, L, NT, NI, MT, kBatchNBUF>(j.a, b, lds); break;
            BATCH_VARIANTS(CASE)
#undef CASE
        default: break;
        }
    }
}

__global__ void __launch_bounds__(256) batch_reduce_kernel(const BatchHeader *h, const BatchJob *jobs)
{
    const int64_t total = h->total_out;
    const int njobs = h->njobs;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const BatchJob &j = jobs[find_job(jobs, njobs, e, 2)];
        const int64_t le = e - j.out_begin;
        const int64_t i = le / j.a.ncols;
        const int col = static_cast<int>(le % j.a.ncols);
        const int64_t t = i / j.tile_rows, ir = i % j.tile_rows;
        const int64_t tile_elems = static_cast<int64_t>(j.tile_rows) * j.cols_pad;
        const double *p = j.a.P + t * tile_elems + ir * j.cols_pad + col;
        const int64_t part_stride = j.n_tiles * tile_elems;
        double s = 0.0;
        int64_t q = 0;
        for (; q + 8 <= j.parts; q += 8) {  // index order, eight loads in flight
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = p[(q + u) * part_stride];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; q < j.parts; ++q) s += p[q * part_stride];
        if (j.out_dtype == DEINSUM_F64) static_cast<double *>(j.out)[i * j.ldo + col] = s;
        else static_cast<float *>(j.out)[i * j.ldo + col] = static_cast<float>(s);
    }
}

#define VINFO(i, P, L, NT, NI, MT) {P, L, NT, NI, MT},
const BatchVariant kVariants[] = {BATCH_VARIANTS(VINFO)};
#undef VINFO

constexpr unsigned kAuxGrid = 1024;  // grid of the grid-stride weight and reduce kernels

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

const BatchVariant *batch_variants(int *count)
{
    *count = static_cast<int>(sizeof(kVariants) / sizeof(kVariants[0]));
    return kVariants;
}

}  // namespace deinsum

using namespace deinsum;

// ------------------------------------------------------------------------------------
// Host object.
struct deinsum_batch {
    int device = 0;
    int capacity = 0;               // jobs (column blocks) the descriptor area holds
    int persistent_groups = 0;      // workgroups of the persistent kernel
    std::vector<BatchJob> jobs;     // host staging, arena offsets in a.P / a.W
    std::vector<int32_t> job_first; // first BatchJob of each user job
    BatchHeader header{};
    size_t arena_used = 0;
    // device / pinned resources
    char *pinned = nullptr;         // header + capacity jobs
    char *d_desc = nullptr;
    int *d_queue = nullptr;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    bool inflight = false;
    int captures = 0;
    int64_t launches = 0;
};

namespace {

size_t desc_bytes(int capacity) { return sizeof(BatchHeader) + sizeof(BatchJob) * static_cast<size_t>(capacity); }

void release_graph(deinsum_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

deinsum_status ensure_capacity(deinsum_batch *b, int jobs_needed)
{
    if (jobs_needed <= b->capacity) return DEINSUM_OK;
    int cap = std::max(64, b->capacity);
    while (cap < jobs_needed) cap *= 2;
    if (b->inflight) {
        if (hipEventSynchronize(b->done) != hipSuccess) return fail(DEINSUM_ERR_DEVICE, "batch: event sync failed");
        b->inflight = false;
    }
    release_graph(b);
    if (b->pinned) (void)hipHostFree(b->pinned);
    if (b->d_desc) (void)hipFree(b->d_desc);
    b->pinned = nullptr;
    b->d_desc = nullptr;
    if (hipHostMalloc(reinterpret_cast<void **>(&b->pinned), desc_bytes(cap), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&b->d_desc), desc_bytes(cap)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DEINSUM_ERR_NO_MEMORY, "batch: descriptor allocation failed");
    }
    std::memset(b->pinned, 0, desc_bytes(cap));
    b->capacity = cap;
    return DEINSUM_OK;
}

deinsum_status capture_graph(deinsum_batch *b)
{
    release_graph(b);
    const BatchHeader *h = reinterpret_cast<const BatchHeader *>(b->d_desc);
    const BatchJob *jobs = reinterpret_cast<const BatchJob *>(b->d_desc + sizeof(BatchHeader));
    if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(DEINSUM_ERR_DEVICE, "batch: stream capture failed to begin");
    batch_reset_kernel<<<1, 1, 0, b->cap_stream>>>(b->d_queue);
    batch_weights_kernel<<<kAuxGrid, 256, 0, b->cap_stream>>>(h, jobs);
    batch_main_kernel<<<b->persistent_groups, 256, 0, b->cap_stream>>>(h, jobs, b->d_queue);
    batch_reduce_kernel<<<kAuxGrid, 256, 0, b->cap_stream>>>(h, jobs);
    hipError_t e = hipStreamEndCapture(b->cap_stream, &b->graph);
    if (e != hipSuccess || !b->graph) {
        (void)hipGetLastError();
        return fail(DEINSUM_ERR_DEVICE, std::string("batch: capture failed: ") + hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(DEINSUM_ERR_DEVICE, std::string("batch: graph instantiation failed: ") + hipGetErrorString(e));
    }
    ++b->captures;
    return DEINSUM_OK;
}

}  // namespace

extern "C" {

deinsum_status deinsum_batch_create(int32_t max_jobs, deinsum_batch **out)
{
    if (!out) return fail(DEINSUM_ERR_INVALID_ARG, "batch_create: null out");
    *out = nullptr;
    auto *b = new deinsum_batch();
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return fail(DEINSUM_ERR_DEVICE, "batch_create: no HIP device");
    }
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    b->persistent_groups = std::max(1, cus) * 2;  // two 4-wave workgroups per CU (2 waves per SIMD)
    if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&b->d_queue), 256) != hipSuccess) {
        (void)hipGetLastError();
        deinsum_batch_destroy(b);
        return fail(DEINSUM_ERR_DEVICE, "batch_create: resource creation failed");
    }
    if (deinsum_status st = ensure_capacity(b, std::max(1, max_jobs))) {
        deinsum_batch_destroy(b);
        return st;
    }
    *out = b;
    clear_error();
    return DEINSUM_OK;
}

}  // extern "C"

namespace deinsum {
namespace {

// forced_nt > 0 (tuning) fixes the column width; otherwise the tuned cache entry
// for the job, else the narrowest width that holds R.
deinsum_status batch_add(deinsum_batch *b, const deinsum_spec *spec, const int64_t *dims, int64_t R, const void *X,
                         const void *const *U, void *M, const deinsum_opts *opts, int32_t *job_id, int forced_nt)
{
    if (!b || !spec || !dims || !X || !U || !M) return fail(DEINSUM_ERR_INVALID_ARG, "batch_add: null argument");
    deinsum_opts o;
    deinsum_opts_init(&o);
    if (opts) o = *opts;
    if (spec->kind != DEINSUM_MTTKRP) return fail(DEINSUM_ERR_INVALID_ARG, "batch_add: spec is not an MTTKRP");
    if (o.precision != DEINSUM_PREC_FP64 && o.precision != DEINSUM_PREC_FP32)
        return fail(DEINSUM_ERR_UNSUPPORTED, "batch_add: the batched launch runs the FP64 and FP32 forms");
    if (o.out_dtype != DEINSUM_F64 && o.out_dtype != DEINSUM_F32)
        return fail(DEINSUM_ERR_INVALID_ARG, "batch_add: out_dtype must be F64 or F32");
    if (o.precision == DEINSUM_PREC_FP64 && o.out_dtype != DEINSUM_F64)
        return fail(DEINSUM_ERR_INVALID_ARG, "batch_add: the FP64 form writes an F64 output");
    if (R < 1 || R > 64) return fail(DEINSUM_ERR_SHAPE, "batch_add: rank must be 1..64");
    if (deinsum_status st = check_dims(spec, dims)) return st;
    const int N = spec->order, n = spec->free_mode;
    MttkrpProblem pb;
    pb.N = N;
    pb.n = n;
    int64_t nx = 1;
    for (int m = 0; m < N; ++m) {
        if (dims[m] < 1) return fail(DEINSUM_ERR_SHAPE, "batch_add: dims must be >= 1");
        pb.dims[m] = dims[m];
        nx *= dims[m];
    }
    {
        // Same argument checks as deinsum_mttkrp: element alignment, and an output
        // that overlaps neither X nor a factor.
        const size_t eb = o.precision == DEINSUM_PREC_FP64 ? 8 : 4, obytes = o.out_dtype == DEINSUM_F64 ? 8 : 4;
        const size_t mbytes = static_cast<size_t>(dims[n] * R) * obytes;
        if (reinterpret_cast<uintptr_t>(X) % eb != 0 || reinterpret_cast<uintptr_t>(M) % obytes != 0)
            return fail(DEINSUM_ERR_INVALID_ARG, "batch_add: X, M and the factors must be aligned to their element size");
        if (overlaps(M, mbytes, X, static_cast<size_t>(nx) * eb))
            return fail(DEINSUM_ERR_INVALID_ARG, "batch_add: output overlaps X");
        for (int k = 0; k < N - 1; ++k) {
            if (!U[k]) return fail(DEINSUM_ERR_INVALID_ARG, "batch_add: null factor");
            if (reinterpret_cast<uintptr_t>(U[k]) % eb != 0)
                return fail(DEINSUM_ERR_INVALID_ARG, "batch_add: X, M and the factors must be aligned to their element size");
            if (overlaps(M, mbytes, U[k], static_cast<size_t>(dims[spec->factor_mode[k]] * R) * eb))
                return fail(DEINSUM_ERR_INVALID_ARG, "batch_add: output overlaps factor operand " + std::to_string(k));
        }
    }
    pb.R = R;
    pb.prec = o.precision;
    int nt = R <= 16 ? 1 : (R <= 32 ? 2 : 4);
    int split = o.split_hint;
    TuneChoice tc;
    if (forced_nt > 0) nt = forced_nt;
    else if (split == 0 && tune_lookup(tune_key(TUNE_BATCH, pb), &tc)) {
        nt = tc.nt;
        split = tc.split;
    }
    const int layout = (n == N - 1) ? L_MCONTIG : L_KCONTIG;
    int vcount = 0;
    const BatchVariant *vars = batch_variants(&vcount);
    int vi = -1;
    for (int i = 0; i < vcount; ++i)
        if (vars[i].prec == pb.prec && vars[i].layout == layout && vars[i].nt == nt) vi = i;
    if (vi < 0) return fail(DEINSUM_ERR_UNSUPPORTED, "batch_add: no batched variant");
    StreamKernelInfo k{vars[vi].prec, vars[vi].layout, vars[vi].nt, vars[vi].ni, vars[vi].mt, kBatchNBUF, 0, nullptr};
    MttkrpPlan p;
    if (deinsum_status st = plan_geometry(pb, &k, split, &p)) return st;
    p.kernel = nullptr;  // points at the local k; not used past this call

    const void *Um[DEINSUM_MAX_ORDER] = {nullptr};
    for (int q = 0; q < N - 1; ++q) {
        if (!U[q]) return fail(DEINSUM_ERR_INVALID_ARG, "batch_add: null factor");
        Um[spec->factor_mode[q]] = U[q];
    }
    if (deinsum_status st = ensure_capacity(b, static_cast<int>(b->jobs.size() + p.col_blocks))) return st;

    const bool kcontig = layout == L_KCONTIG;
    const int gmode = kcontig ? N - 1 : N - 2;
    const size_t ub = pb.prec == P_FP64 ? 8 : 4;
    const size_t xb = pb.prec == P_FP64 ? 8 : 4;
    const size_t ob = o.out_dtype == DEINSUM_F64 ? 8 : 4;
    int64_t stride[DEINSUM_MAX_ORDER];
    {
        int64_t st = 1;
        for (int m = N - 1; m >= 0; --m) {
            stride[m] = st;
            st *= pb.dims[m];
        }
    }
    if (job_id) *job_id = static_cast<int32_t>(b->job_first.size());
    b->job_first.push_back(static_cast<int32_t>(b->jobs.size()));
    const int cols_pad = 16 * p.nt;
    const size_t part_bytes = p.w_offset;
    const size_t w_bytes = static_cast<size_t>(p.O) * cols_pad * sizeof(double);
    for (int64_t cb = 0; cb < p.col_blocks; ++cb) {
        const int64_t col0 = cb * cols_pad;
        const int ncols = static_cast<int>(std::min<int64_t>(cols_pad, R - col0));
        auto ucol = [&](int m) { return static_cast<const void *>(static_cast<const char *>(Um[m]) + col0 * ub); };
        BatchJob j;
        std::memset(&j, 0, sizeof(j));
        StreamArgs &a = j.a;
        a.X = X;
        a.Ug = ucol(gmode);
        a.ldu = R;
        int kk = 0;
        for (int m = 0; m < N; ++m) {
            if (m == n || m == gmode) continue;
            a.od.dim[kk] = pb.dims[m];
            a.od.xstride[kk] = stride[m];
            a.od.U[kk] = ucol(m);
            ++kk;
        }
        a.od.n_outer = kk;
        a.In = pb.dims[n];
        a.Ig = pb.dims[gmode];
        a.stride_n = stride[n];
        a.stride_g = stride[gmode];
        a.ncols = ncols;
        a.n_tiles = static_cast<int>(p.n_tiles);
        a.n_kgroups = static_cast<int>(p.n_kgroups);
        a.wk = p.wk;
        a.O = p.O;
        a.o_per_chunk = p.o_per_chunk;
        a.order = 0;  // units come from the work queue in index order
        a.xcd_remap = 0;
        a.n_chunks = p.n_chunks;
        a.n_groups = p.groups;
        const int64_t contig = kcontig ? a.Ig : a.In;
        a.vec_ok = ((contig * xb) % 16 == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0);
        a.ldw = cols_pad;
        // arena offsets (resolved to pointers at launch)
        a.P = reinterpret_cast<double *>(b->arena_used);
        b->arena_used += align256(part_bytes);
        a.W = reinterpret_cast<const double *>(b->arena_used);
        b->arena_used += align256(w_bytes);
        j.variant = vi;
        j.prec = pb.prec;
        j.unit_begin = b->header.total_units;
        j.n_units = p.groups;
        j.w_begin = b->header.total_w;
        j.ldu = R;
        j.out_begin = b->header.total_out;
        j.rows = pb.dims[n];
        j.parts = p.parts;
        j.n_tiles = p.n_tiles;
        j.tile_rows = p.tile_rows;
        j.cols_pad = cols_pad;
        j.out = static_cast<char *>(M) + col0 * ob;
        j.ldo = R;
        j.out_dtype = o.out_dtype;
        b->header.total_units += p.groups;
        b->header.total_w += p.O * cols_pad;
        b->header.total_out += pb.dims[n] * ncols;
        b->jobs.push_back(j);
    }
    (void)xb;
    clear_error();
    return DEINSUM_OK;
}

}  // namespace
}  // namespace deinsum

extern "C" {

deinsum_status deinsum_batch_add_mttkrp(deinsum_batch *b, const deinsum_spec *spec, const int64_t *dims, int64_t R,
                                        const void *X, const void *const *U, void *M, const deinsum_opts *opts,
                                        int32_t *job_id)
{
    return batch_add(b, spec, dims, R, X, U, M, opts, job_id, 0);
}

deinsum_status deinsum_tune_batch_mttkrp(const deinsum_spec *spec, const int64_t *dims, int64_t R, const void *X,
                                         const void *const *U, void *M, const deinsum_opts *opts, int32_t reps,
                                         deinsum_report *best, void *stream)
{
    if (reps < 1 || reps > 1000) return fail(DEINSUM_ERR_INVALID_ARG, "tune_batch: reps must be 1..1000");
    if (!spec || !dims) return fail(DEINSUM_ERR_INVALID_ARG, "tune_batch: null argument");
    deinsum_opts o;
    deinsum_opts_init(&o);
    if (opts) o = *opts;
    o.split_hint = 0;
    o.report = nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    MttkrpProblem pb;
    pb.N = spec->order;
    pb.n = spec->free_mode;
    pb.R = R;
    pb.prec = o.precision;
    if (pb.N < 2 || pb.N > DEINSUM_MAX_ORDER) return fail(DEINSUM_ERR_INVALID_ARG, "tune_batch: bad spec");
    for (int m = 0; m < pb.N; ++m) pb.dims[m] = dims[m];
    const int layout = (pb.n == pb.N - 1) ? L_MCONTIG : L_KCONTIG;
    int vcount = 0;
    const BatchVariant *vars = batch_variants(&vcount);
    hipEvent_t ev[2];
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
        return fail(DEINSUM_ERR_DEVICE, "tune_batch: event creation failed");
    double best_us = -1;
    TuneChoice choice;
    MttkrpPlan best_plan;
    deinsum_status st = DEINSUM_OK;
    for (int vi = 0; vi < vcount && st == DEINSUM_OK; ++vi) {
        const BatchVariant &v = vars[vi];
        if (v.prec != pb.prec || v.layout != layout) continue;
        StreamKernelInfo k{v.prec, v.layout, v.nt, v.ni, v.mt, kBatchNBUF, 0, nullptr};
        MttkrpPlan p0;
        if (plan_geometry(pb, &k, 0, &p0) != DEINSUM_OK) continue;
        int splits[8];
        const int ns = tune_splits(p0.n_chunks, p0.O, splits);
        for (int si = 0; si < ns && st == DEINSUM_OK; ++si) {
            deinsum_batch *b = nullptr;
            if ((st = deinsum_batch_create(1, &b)) != DEINSUM_OK) break;
            o.split_hint = splits[si];
            st = batch_add(b, spec, dims, R, X, U, M, &o, nullptr, v.nt);
            std::vector<float> t;
            for (int r = 0; r <= reps && st == DEINSUM_OK; ++r) {  // r = 0 captures the graph (warm-up)
                (void)hipEventRecord(ev[0], s);
                st = deinsum_batch_launch(b, s);
                (void)hipEventRecord(ev[1], s);
                if (hipEventSynchronize(ev[1]) != hipSuccess) st = fail(DEINSUM_ERR_DEVICE, "tune_batch: sync failed");
                float ms = 0;
                (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
                if (r > 0) t.push_back(ms);
            }
            deinsum_batch_destroy(b);
            if (st != DEINSUM_OK) break;
            std::sort(t.begin(), t.end());
            const double us = 1e3 * t[t.size() / 2];
            if (best_us < 0 || us < best_us) {
                best_us = us;
                choice.nt = v.nt;
                choice.ni = v.ni;
                choice.mt = v.mt;
                choice.split = splits[si];
                choice.us = us;
                (void)plan_geometry(pb, &k, splits[si], &best_plan);
            }
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (st != DEINSUM_OK) return st;
    if (best_us < 0) return fail(DEINSUM_ERR_UNSUPPORTED, "tune_batch: no batched variant for this job");
    tune_store(tune_key(TUNE_BATCH, pb), choice);
    if (best) {
        std::memset(best, 0, sizeof(*best));
        best->plan_id = best_plan.family;
        best->tile_m = best_plan.tile_rows;
        best->tile_k = best_plan.slice;
        best->waves_per_group = best_plan.waves;
        best->groups = best_plan.groups * best_plan.col_blocks;
        best->partials = best_plan.parts;
        best->workspace_bytes = best_plan.workspace;
        std::snprintf(best->plan_name, sizeof(best->plan_name), "batch %s", best_plan.name.c_str());
        best->tuned_us = best_us;
    }
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_batch_launch(deinsum_batch *b, void *stream)
{
    if (!b) return fail(DEINSUM_ERR_INVALID_ARG, "batch_launch: null batch");
    if (b->jobs.empty()) return DEINSUM_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // The pinned descriptors of the previous epoch must have been copied out.
    if (b->inflight) {
        if (hipEventSynchronize(b->done) != hipSuccess) return fail(DEINSUM_ERR_DEVICE, "batch_launch: event sync failed");
        b->inflight = false;
    }
    if (b->arena_bytes < b->arena_used) {
        if (b->arena) {
            if (hipDeviceSynchronize() != hipSuccess) return fail(DEINSUM_ERR_DEVICE, "batch_launch: sync failed");
            (void)hipFree(b->arena);
            b->arena = nullptr;
            b->arena_bytes = 0;
        }
        const size_t want = std::max(b->arena_used + b->arena_used / 4, size_t(1) << 20);
        if (hipMalloc(reinterpret_cast<void **>(&b->arena), want) != hipSuccess) {
            (void)hipGetLastError();
            return fail(DEINSUM_ERR_NO_MEMORY, "batch_launch: arena allocation failed");
        }
        b->arena_bytes = want;
    }
    BatchHeader *h = reinterpret_cast<BatchHeader *>(b->pinned);
    BatchJob *pj = reinterpret_cast<BatchJob *>(b->pinned + sizeof(BatchHeader));
    *h = b->header;
    h->njobs = static_cast<int32_t>(b->jobs.size());
    for (size_t i = 0; i < b->jobs.size(); ++i) {
        pj[i] = b->jobs[i];
        pj[i].a.P = reinterpret_cast<double *>(b->arena + reinterpret_cast<uintptr_t>(b->jobs[i].a.P));
        pj[i].a.W = reinterpret_cast<const double *>(b->arena + reinterpret_cast<uintptr_t>(b->jobs[i].a.W));
    }
    if (!b->exec)
        if (deinsum_status st = capture_graph(b)) return st;
    // Descriptors of this launch's jobs only (the graph reads h->njobs of them).
    if (hipMemcpyAsync(b->d_desc, b->pinned, desc_bytes(static_cast<int>(b->jobs.size())), hipMemcpyHostToDevice, s) !=
        hipSuccess) {
        (void)hipGetLastError();
        return fail(DEINSUM_ERR_DEVICE, "batch_launch: descriptor upload failed");
    }
    if (hipGraphLaunch(b->exec, s) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DEINSUM_ERR_DEVICE, "batch_launch: graph launch failed");
    }
    if (hipEventRecord(b->done, s) != hipSuccess) return fail(DEINSUM_ERR_DEVICE, "batch_launch: event record failed");
    b->inflight = true;
    ++b->launches;
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_batch_reset(deinsum_batch *b)
{
    if (!b) return fail(DEINSUM_ERR_INVALID_ARG, "batch_reset: null batch");
    b->jobs.clear();
    b->job_first.clear();
    b->header = BatchHeader{};
    b->arena_used = 0;
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_batch_info(const deinsum_batch *b, int32_t *jobs, int64_t *units, int32_t *graph_captures,
                                  int64_t *launches)
{
    if (!b) return fail(DEINSUM_ERR_INVALID_ARG, "batch_info: null batch");
    if (jobs) *jobs = static_cast<int32_t>(b->job_first.size());
    if (units) *units = b->header.total_units;
    if (graph_captures) *graph_captures = b->captures;
    if (launches) *launches = b->launches;
    return DEINSUM_OK;
}

deinsum_status deinsum_batch_destroy(deinsum_batch *b)
{
    if (!b) return DEINSUM_OK;
    if (b->inflight) (void)hipEventSynchronize(b->done);
    release_graph(b);
    if (b->pinned) (void)hipHostFree(b->pinned);
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_queue) (void)hipFree(b->d_queue);
    if (b->arena) (void)hipFree(b->arena);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return DEINSUM_OK;
}

}  // extern "C"
