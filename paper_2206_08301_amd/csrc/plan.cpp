// plan.cpp -- heuristic launch plans for MTTKRP (tile shapes and work split).
//
// The split targets enough workgroups to cover the 256 compute units several
// times over (so the tail of the last wave of workgroups is small) while
// keeping each wave's walk over the outer indices long enough to amortise
// its register-resident factor slice, and the partial-output workspace a
// small fraction of X's bytes.
#include <algorithm>
#include <cstdio>

#include "internal.h"
#include "kernels.h"
#include "mttkrp.h"
#include "plan.h"

namespace deinsum {

namespace {

constexpr int64_t kTargetGroups = 4096;  // 16 per compute unit
constexpr int kWaves = 4;

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

size_t elem_bytes(int prec)
{
    switch (prec) {
    case P_FP64: return 8;
    case P_BF16: return 2;
    default: return 4;
    }
}

// Preferred per-lane runs (elements) of each precision, best first: a 128-byte
// run per lane, then runs that fit short contiguous modes with little padding.
const int *kl_candidates(int prec, int nt, int *count)
{
    static const int f64[3][3] = {{16, 20, 8}, {16, 20, 8}, {8, 20, 8}};
    static const int f32[3][3] = {{32, 20, 8}, {32, 20, 8}, {16, 20, 16}};
    static const int b16[3][3] = {{64, 24, 8}, {64, 24, 8}, {32, 24, 32}};
    static const int b3[3][3] = {{32, 24, 8}, {32, 24, 8}, {16, 24, 16}};
    const int row = nt == 1 ? 0 : (nt == 2 ? 1 : 2);
    *count = 3;
    switch (prec) {
    case P_FP64: return f64[row];
    case P_FP32: return f32[row];
    case P_BF16: return b16[row];
    default: return b3[row];
    }
}

}  // namespace

deinsum_status plan_mttkrp(const MttkrpProblem &pb, int plan_hint, int split_hint, MttkrpPlan *out)
{
    MttkrpPlan p;
    p.prec = pb.prec;
    const int N = pb.N, n = pb.n;
    const int64_t R = pb.R;
    p.nt = R <= 16 ? 1 : (R <= 32 ? 2 : 4);
    p.col_blocks = cdiv(R, 16 * p.nt);
    p.family = (n == N - 1) ? PLAN_MTTKRP_MCONTIG : PLAN_MTTKRP_KCONTIG;
    if (plan_hint == PLAN_MTTKRP_KCONTIG || plan_hint == PLAN_MTTKRP_MCONTIG) {
        if ((plan_hint == PLAN_MTTKRP_MCONTIG) != (n == N - 1))
            return fail(DEINSUM_ERR_UNSUPPORTED, "plan_hint does not match the free mode");
    }
    const size_t eb = elem_bytes(pb.prec);

    if (p.family == PLAN_MTTKRP_KCONTIG) {
        const int64_t Ig = pb.dims[N - 1];
        const int64_t In = pb.dims[n];
        int64_t O = 1;
        for (int m = 0; m < N - 1; ++m)
            if (m != n) O *= pb.dims[m];
        int cnt = 0;
        const int *cands = kl_candidates(pb.prec, p.nt, &cnt);
        // Pick the run with the least padded k; ties go to the earlier (larger) run.
        int best = -1;
        int64_t best_padded = 0;
        for (int i = 0; i < cnt; ++i) {
            if (!kcontig_available(pb.prec, p.nt, cands[i])) continue;
            const int64_t ks = 4 * cands[i];
            const int64_t padded = cdiv(Ig, ks) * ks;
            if (best < 0 || padded < best_padded) {
                best = i;
                best_padded = padded;
            }
        }
        if (best < 0) return fail(DEINSUM_ERR_UNSUPPORTED, "no K-contiguous kernel for this precision and rank");
        p.kl = cands[best];
        const int64_t nks = cdiv(Ig, 4 * p.kl);
        p.wk = (nks % 4 == 0) ? 4 : (nks % 2 == 0 ? 2 : 1);
        p.wo = kWaves / p.wk;
        p.n_kgroups = cdiv(nks, p.wk);
        p.n_tiles = cdiv(In, 16);
        const int64_t per_chunk = p.n_tiles * p.n_kgroups;
        int64_t chunks = split_hint > 0 ? split_hint : cdiv(kTargetGroups, per_chunk);
        chunks = std::max<int64_t>(1, std::min<int64_t>(chunks, cdiv(O, 4 * p.wo)));  // >= 4 steps per wave
        if (split_hint > 0) chunks = std::max<int64_t>(1, std::min<int64_t>(split_hint, O));
        p.o_per_chunk = cdiv(O, chunks);
        p.n_chunks = cdiv(O, p.o_per_chunk);
        p.groups = p.n_chunks * per_chunk;
        p.parts = p.n_chunks * p.n_kgroups;
        p.workspace = static_cast<size_t>(p.parts * p.n_tiles) * 16 * 16 * p.nt * sizeof(double);
        char buf[96];
        std::snprintf(buf, sizeof(buf), "mttkrp_kcontig<p%d,nt%d,kl%d> wk%d wo%d", pb.prec, p.nt, p.kl, p.wk, p.wo);
        p.name = buf;
    } else {
        if (pb.prec != P_FP64 && pb.prec != P_FP32)
            return fail(DEINSUM_ERR_UNSUPPORTED,
                        "MTTKRP on the last (contiguous) mode supports the FP64 and FP32 forms");
        const int64_t In = pb.dims[N - 1];
        const int64_t Ig = pb.dims[N - 2];
        int64_t O = 1;
        for (int m = 0; m < N - 2; ++m) O *= pb.dims[m];
        p.mt = (pb.prec == P_FP64) ? 2 : 4;
        if (p.nt == 4) p.mt = (pb.prec == P_FP64) ? 2 : 4;
        if (!mcontig_available(pb.prec, p.nt, p.mt))
            return fail(DEINSUM_ERR_UNSUPPORTED, "no M-contiguous kernel for this precision and rank");
        p.n_tiles = cdiv(In, 16 * p.mt);
        int64_t want = split_hint > 0 ? split_hint : cdiv(kTargetGroups, p.n_tiles);
        // Split the outer indices first, then i_g (keeping >= 64 i_g rows per workgroup).
        int64_t oc = std::max<int64_t>(1, std::min<int64_t>(want, O));
        int64_t igc = 1;
        if (oc < want) igc = std::max<int64_t>(1, std::min<int64_t>(cdiv(want, oc), cdiv(Ig, 64)));
        p.o_per_chunk = cdiv(O, oc);
        p.n_chunks = cdiv(O, p.o_per_chunk);
        p.ig_per_chunk = cdiv(cdiv(Ig, igc), 16) * 16;
        p.n_igchunks = cdiv(Ig, p.ig_per_chunk);
        p.groups = p.n_tiles * p.n_chunks * p.n_igchunks;
        p.parts = p.n_chunks * p.n_igchunks;
        p.workspace = static_cast<size_t>(p.parts * p.n_tiles) * 16 * p.mt * 16 * p.nt * sizeof(double);
        char buf[96];
        std::snprintf(buf, sizeof(buf), "mttkrp_mcontig<p%d,nt%d,mt%d>", pb.prec, p.nt, p.mt);
        p.name = buf;
    }
    (void)eb;
    *out = p;
    return DEINSUM_OK;
}

}  // namespace deinsum
