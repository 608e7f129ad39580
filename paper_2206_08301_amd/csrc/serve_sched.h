// serve_sched.h -- admission rule of the request server's continuous batching
// (host only, no device code, so it is testable on its own).
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <vector>

namespace deinsum {

// Admit requests into one epoch.  `pending` holds request ids in arrival order.
// A request is admitted when its tensor is idle, it heads its tensor's queue
// (requests of one tensor run in arrival order), the epoch has fewer than
// `max_jobs` requests, and the workspace of the admitted requests plus
// `in_use` stays within `budget` -- except that an empty epoch always admits
// its first candidate, so the server makes progress whatever the budget.
// Admitted ids are appended to `out` (arrival order), removed from `pending`,
// their tensors marked busy, and `footprint` grows by their workspace.
template <class TensorOf, class IsHead, class IsBusy, class WsOf, class SetBusy>
void admit_epoch(std::deque<int64_t> &pending, size_t max_jobs, size_t in_use, size_t budget,
                 std::vector<int64_t> &out, size_t &footprint, TensorOf tensor_of, IsHead is_head, IsBusy is_busy,
                 WsOf ws_of, SetBusy set_busy)
{
    for (auto it = pending.begin(); it != pending.end() && out.size() < max_jobs;) {
        const int64_t r = *it;
        const auto t = tensor_of(r);
        const size_t ws = ws_of(r);
        if (!is_busy(t) && is_head(r) && (in_use + footprint + ws <= budget || out.empty())) {
            set_busy(t);
            out.push_back(r);
            footprint += ws;
            it = pending.erase(it);
        } else {
            ++it;
        }
    }
}

}  // namespace deinsum
