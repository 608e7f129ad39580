// plan.cpp -- heuristic launch plans for MTTKRP (tile shape and work split).
//
// The tile is the compiled variant whose slice of mode g pads that mode the
// least (ties: the first, largest variant of the table).  The split targets
// enough workgroups to cover the 256 compute units a few times over while
// keeping every wave's walk over the outer indices long enough to amortise
// loading its factor slice and filling its prefetch ring, and the partial
// workspace a small fraction of X.
#include <algorithm>
#include <cstdio>

#include "internal.h"
#include "kernels.h"
#include "mttkrp.h"
#include "plan.h"
#include "tune.h"

namespace deinsum {

namespace {

constexpr int64_t kTargetGroups = 2048;  // 8 per compute unit
constexpr int64_t kMinSteps = 8;         // outer steps per wave
constexpr int kWaves = 4;

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
// K values per lane per matrix-core instruction.
int ke_of(int prec, int layout)
{
    (void)layout;
    return (prec == P_BF16 || prec == P_BF16X3 || prec == P_FX20) ? 8 : 1;
}

// L_KOUT (order 3, free mode 0): a unit is (k-group, chunk of output rows); every
// wave of a k-group's workgroup walks the chunk's rows, each over all mode-1 tiles.
deinsum_status plan_geometry_kout(const MttkrpProblem &pb, const StreamKernelInfo *kernel, int split_hint,
                                  MttkrpPlan *out)
{
    if (pb.N != 3 || pb.n != 0) return fail(DEINSUM_ERR_UNSUPPORTED, "the mode-1-tiled walk is for order-3 mode 0");
    MttkrpPlan p;
    p.prec = pb.prec;
    p.kernel = kernel;
    p.family = PLAN_MTTKRP_KOUT;
    p.nt = kernel->nt;
    p.ni = kernel->ni;
    p.mt = 1;
    p.col_blocks = cdiv(pb.R, 16 * p.nt);
    p.slice = 4 * p.ni * ke_of(pb.prec, L_KCONTIG);
    p.tile_rows = 16;
    const int64_t I0 = pb.dims[0], I1 = pb.dims[1], I2 = pb.dims[2];
    const int64_t nks = cdiv(I2, p.slice);
    p.waves = kWaves;
    p.wk = (nks % 4 == 0) ? 4 : (nks % 2 == 0 ? 2 : 1);
    const int wo = p.waves / p.wk;
    p.n_kgroups = cdiv(nks, p.wk);
    p.n_tiles = cdiv(I1, 16);  // mode-1 tiles per output row
    int64_t chunks = split_hint > 0 ? split_hint : cdiv(kTargetGroups, p.n_kgroups);
    chunks = std::max<int64_t>(1, std::min<int64_t>(chunks, cdiv(I0, wo)));
    p.o_per_chunk = cdiv(I0, chunks);
    p.n_chunks = cdiv(I0, p.o_per_chunk);
    p.groups = p.n_chunks * p.n_kgroups;
    p.parts = p.n_kgroups * p.wk;
    p.O = I0;
    p.order = 0;
    p.xcd = 0;
    const size_t part_bytes = static_cast<size_t>(p.parts * I0) * 16 * p.nt * sizeof(double);
    p.w_offset = (part_bytes + 255) / 256 * 256;
    p.workspace = p.w_offset + static_cast<size_t>(p.n_tiles) * 256 * p.nt * sizeof(float);  // packed FP32 U^1
    char buf[96];
    std::snprintf(buf, sizeof(buf), "mttkrp_kout<p%d,nt%d,ni%d%s> wk%d", pb.prec, p.nt, p.ni, kernel->xnt ? ",nt" : "",
                  p.wk);
    p.name = buf;
    *out = p;
    return DEINSUM_OK;
}

}  // namespace

bool kout_default(const MttkrpProblem &pb)
{
    if (pb.N != 3 || pb.n != 0 || pb.prec == P_FP64 || pb.dims[1] < 16) return false;
    const int64_t eb = pb.prec == P_FX20 ? 2 : (pb.prec == P_BF16 ? 2 : 4);
    return pb.dims[1] * pb.dims[2] * eb >= (int64_t(1) << 20);
}

deinsum_status plan_geometry(const MttkrpProblem &pb, const StreamKernelInfo *kernel, int split_hint, MttkrpPlan *out)
{
    MttkrpPlan p;
    p.prec = pb.prec;
    const int N = pb.N, n = pb.n;
    p.kernel = kernel;
    p.nt = kernel->nt;
    p.col_blocks = cdiv(pb.R, 16 * p.nt);
    const int layout = kernel->layout;
    if (layout == L_KOUT) return plan_geometry_kout(pb, kernel, split_hint, out);
    p.family = (layout == L_KCONTIG) ? PLAN_MTTKRP_KCONTIG : PLAN_MTTKRP_MCONTIG;
    if ((layout == L_MCONTIG) != (n == N - 1))
        return fail(DEINSUM_ERR_UNSUPPORTED, "kernel layout does not match the free mode");
    const int g = (layout == L_KCONTIG) ? N - 1 : N - 2;
    const int64_t Ig = pb.dims[g], In = pb.dims[n];
    int64_t O = 1;
    for (int m = 0; m < N; ++m)
        if (m != n && m != g) O *= pb.dims[m];
    p.ni = kernel->ni;
    p.mt = kernel->mt;
    p.slice = 4 * p.ni * ke_of(pb.prec, layout);
    p.tile_rows = (layout == L_KCONTIG) ? 16 : 16 * p.mt;
    const int64_t nks = cdiv(Ig, p.slice);
    p.waves = kWaves;
    p.wk = (nks % 4 == 0) ? 4 : (nks % 2 == 0 ? 2 : 1);
    const int wo = p.waves / p.wk;
    p.n_kgroups = cdiv(nks, p.wk);
    p.n_tiles = cdiv(In, p.tile_rows);
    const int64_t per_chunk = p.n_tiles * p.n_kgroups;
    int64_t chunks;
    if (split_hint > 0) {
        chunks = std::min<int64_t>(split_hint, O);
    } else {
        chunks = cdiv(kTargetGroups, per_chunk);
        chunks = std::min<int64_t>(chunks, std::max<int64_t>(1, O / (wo * kMinSteps)));
    }
    chunks = std::max<int64_t>(1, chunks);
    p.o_per_chunk = cdiv(O, chunks);
    p.n_chunks = cdiv(O, p.o_per_chunk);
    p.groups = p.n_chunks * per_chunk;
    p.parts = p.n_chunks * p.n_kgroups;
    p.O = O;
    // Chunk-major units keep the workgroups in flight on few rows of X (fewer
    // pages per XCD); the M-contiguous walk also gains from the XCD remap.
    p.order = 1;
    p.xcd = (layout == L_MCONTIG) ? 1 : 0;
    const size_t part_bytes = static_cast<size_t>(p.parts * p.n_tiles) * p.tile_rows * 16 * p.nt * sizeof(double);
    p.w_offset = (part_bytes + 255) / 256 * 256;
    p.workspace = p.w_offset + static_cast<size_t>(O) * 16 * p.nt * sizeof(double);
    char buf[96];
    std::snprintf(buf, sizeof(buf), "mttkrp_%s<p%d,nt%d,ni%d,mt%d%s> wk%d", layout == L_KCONTIG ? "kcontig" : "mcontig",
                  pb.prec, p.nt, p.ni, p.mt, kernel->xnt ? ",nt" : "", p.wk);
    p.name = buf;
    *out = p;
    return DEINSUM_OK;
}

deinsum_status plan_mttkrp(const MttkrpProblem &pb, int plan_hint, int split_hint, MttkrpPlan *out)
{
    const int N = pb.N, n = pb.n;
    const int nt = pb.R <= 16 ? 1 : (pb.R <= 32 ? 2 : 4);
    int family = (n == N - 1) ? PLAN_MTTKRP_MCONTIG : PLAN_MTTKRP_KCONTIG;
    const bool kout_ok = N == 3 && n == 0 && pb.prec != P_FP64 && pb.dims[0] < (int64_t(1) << 31);
    if (plan_hint == PLAN_MTTKRP_KOUT && kout_ok) family = PLAN_MTTKRP_KOUT;
    if (plan_hint != 0 && plan_hint != family)
        return fail(DEINSUM_ERR_UNSUPPORTED, "plan_hint does not match the free mode");
    int count = 0;
    const StreamKernelInfo *table = stream_kernels(&count);
    TuneChoice tc;
    bool tuned = plan_hint == 0 && split_hint == 0 && tune_lookup(tune_key(TUNE_STREAM, pb), &tc);
    if (tuned && tc.order == kTuneKout) {
        for (int i = 0; i < count && kout_ok; ++i) {
            const StreamKernelInfo &k = table[i];
            if (k.prec == pb.prec && k.layout == L_KOUT && k.nt == tc.nt && k.ni == tc.ni && k.xnt == tc.xnt)
                return plan_geometry(pb, &k, tc.split, out);
        }
        tuned = false;  // a variant that is no longer compiled: the untuned choice below
    } else if (tuned && tc.order != kTuneViaTtmc) {
        const int base = (n == N - 1) ? L_MCONTIG : L_KCONTIG;
        bool found = false;
        for (int i = 0; i < count; ++i) {
            const StreamKernelInfo &k = table[i];
            found |= k.prec == pb.prec && k.layout == base && k.nt == tc.nt && k.ni == tc.ni && k.mt == tc.mt &&
                     k.xnt == tc.xnt;
        }
        tuned = found;
    }
    if (plan_hint == 0 && !tuned && kout_ok && kout_default(pb)) family = PLAN_MTTKRP_KOUT;
    const int layout = family == PLAN_MTTKRP_KOUT ? L_KOUT : (family == PLAN_MTTKRP_KCONTIG ? L_KCONTIG : L_MCONTIG);
    const int g = (layout == L_MCONTIG) ? N - 2 : N - 1;
    const int64_t Ig = pb.dims[g];
    if (tuned && tc.order != kTuneViaTtmc && tc.order != kTuneKout) {
        for (int i = 0; i < count; ++i) {
            const StreamKernelInfo &k = table[i];
            if (k.prec == pb.prec && k.layout == layout && k.nt == tc.nt && k.ni == tc.ni && k.mt == tc.mt &&
                k.xnt == tc.xnt) {
                if (deinsum_status st = plan_geometry(pb, &k, tc.split, out)) return st;
                out->order = tc.order;
                out->xcd = tc.xcd;
                return DEINSUM_OK;
            }
        }
        // An entry for a variant that is no longer compiled falls back to the heuristic.
    }
    const StreamKernelInfo *best = nullptr;
    int64_t best_padded = 0, best_split = 0;
    // Short contiguous output mode (M-contiguous, rows under 64 elements): among equal
    // K padding, fewer row tiles per X row (a row split between workgroups is read in
    // partial cache lines twice).
    auto row_tiles = [&](const StreamKernelInfo &k) -> int64_t {
        return (layout == L_MCONTIG && pb.dims[n] <= 64) ? cdiv(pb.dims[n], 16LL * k.mt) : 0;
    };
    for (int i = 0; i < count; ++i) {
        const StreamKernelInfo &k = table[i];
        if (k.prec != pb.prec || k.layout != layout || k.nt != nt) continue;
        const int64_t slice = 4LL * k.ni * ke_of(pb.prec, layout);
        const int64_t padded = cdiv(Ig, slice) * slice;
        if (!best || padded < best_padded || (padded == best_padded && row_tiles(k) < best_split)) {
            best = &k;
            best_padded = padded;
            best_split = row_tiles(k);
        }
    }
    // Forms without a kernel of this column width take narrower tiles (more column blocks).
    for (int w = nt / 2; !best && w >= 1; w /= 2)
        for (int i = 0; i < count; ++i) {
            const StreamKernelInfo &k = table[i];
            if (k.prec != pb.prec || k.layout != layout || k.nt != w) continue;
            const int64_t slice = 4LL * k.ni * ke_of(pb.prec, layout);
            const int64_t padded = cdiv(Ig, slice) * slice;
            if (!best || padded < best_padded) {
                best = &k;
                best_padded = padded;
            }
        }
    if (!best) return fail(DEINSUM_ERR_UNSUPPORTED, "no compiled MTTKRP kernel for this precision and rank");
    return plan_geometry(pb, best, split_hint, out);
}

}  // namespace deinsum
