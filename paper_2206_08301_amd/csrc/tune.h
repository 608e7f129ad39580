// tune.h -- process-wide cache of autotuned MTTKRP plans (host only).
#pragma once

#include <string>

#include "plan.h"

namespace deinsum {

enum TunePath { TUNE_STREAM = 0, TUNE_BATCH = 1 };
constexpr int kTuneViaTtmc = 2;
constexpr int kTuneKout = 3;  // order field: the L_KOUT kernel (nt, ni, mt, xnt) with `split` chunks

// A tuned choice: the tile shape (kernel variant) and the outer-chunk count.
struct TuneChoice {
    int nt = 0, ni = 0, mt = 0, xnt = 0;
    int split = 0;
    int order = 0, xcd = 0;  // unit order and XCD remap of the per-call kernel; order
                             // kTuneViaTtmc: mode 0 runs through the fused TTMc pass,
                             // split holding its variant
    double us = 0;           // measured median time of the winner
};

std::string tune_key(int path, const MttkrpProblem &pb);
// Looks the key up (the file named by DEINSUM_TUNE_CACHE is read on first use).
bool tune_lookup(const std::string &key, TuneChoice *out);
// Records a choice; rewrites the DEINSUM_TUNE_CACHE file when that variable is set.
void tune_store(const std::string &key, const TuneChoice &c);

// Split candidates around the heuristic chunk count c0, within [1, O].
int tune_splits(int64_t c0, int64_t O, int out[8]);

}  // namespace deinsum
