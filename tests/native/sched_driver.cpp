// Scenarios for the request server's admission rule (serve_sched.h), with
// plain vectors standing in for the server's tensors and requests.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <vector>

#include "serve_sched.h"

using deinsum::admit_epoch;

struct World {
    std::vector<int> req_tensor;
    std::vector<size_t> req_ws;
    std::vector<std::deque<int64_t>> fifo;  // per tensor, arrival order
    std::vector<char> busy;
    int add(int t, size_t ws)
    {
        const int r = static_cast<int>(req_tensor.size());
        req_tensor.push_back(t);
        req_ws.push_back(ws);
        if (static_cast<int>(fifo.size()) <= t) fifo.resize(t + 1), busy.resize(t + 1, 0);
        fifo[t].push_back(r);
        return r;
    }
    std::vector<int64_t> admit(std::deque<int64_t> &pending, size_t cap, size_t in_use, size_t budget, size_t &fp)
    {
        std::vector<int64_t> out;
        fp = 0;
        admit_epoch(
            pending, cap, in_use, budget, out, fp, [&](int64_t r) { return req_tensor[r]; },
            [&](int64_t r) { return !fifo[req_tensor[r]].empty() && fifo[req_tensor[r]].front() == r; },
            [&](int t) { return busy[t] != 0; }, [&](int64_t r) { return req_ws[r]; }, [&](int t) { busy[t] = 1; });
        return out;
    }
    void complete(const std::vector<int64_t> &done)
    {
        for (int64_t r : done) {
            busy[req_tensor[r]] = 0;
            fifo[req_tensor[r]].pop_front();
        }
    }
};

static int failures = 0;
#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            std::printf("FAILED line %d: %s\n", __LINE__, #c);                     \
            ++failures;                                                            \
        }                                                                          \
    } while (0)

int main()
{
    {  // one request per tensor per epoch, arrival order kept
        World w;
        std::deque<int64_t> p;
        for (int q = 0; q < 9; ++q) p.push_back(w.add(q % 3, 10));
        size_t fp;
        auto e1 = w.admit(p, 100, 0, 1000, fp);
        CHECK((e1 == std::vector<int64_t>{0, 1, 2}) && fp == 30 && p.size() == 6);
        auto e2 = w.admit(p, 100, 30, 1000, fp);
        CHECK(e2.empty());  // every tensor busy: nothing admitted
        w.complete(e1);
        auto e3 = w.admit(p, 100, 0, 1000, fp);
        CHECK((e3 == std::vector<int64_t>{3, 4, 5}));
    }
    {  // slot cap
        World w;
        std::deque<int64_t> p;
        for (int q = 0; q < 5; ++q) p.push_back(w.add(q, 1));
        size_t fp;
        auto e = w.admit(p, 2, 0, 1000, fp);
        CHECK((e == std::vector<int64_t>{0, 1}) && p.size() == 3);
    }
    {  // HBM budget: skip what does not fit, keep looking for smaller requests
        World w;
        std::deque<int64_t> p;
        p.push_back(w.add(0, 60));
        p.push_back(w.add(1, 50));
        p.push_back(w.add(2, 30));
        size_t fp;
        auto e = w.admit(p, 100, 0, 100, fp);
        CHECK((e == std::vector<int64_t>{0, 2}) && fp == 90);
        // budget already used by an epoch in flight: an empty epoch still takes one request
        auto e2 = w.admit(p, 100, 500, 100, fp);
        CHECK((e2 == std::vector<int64_t>{1}) && fp == 50 && p.empty());
    }
    {  // a later request of a busy tensor never overtakes its predecessor
        World w;
        std::deque<int64_t> p;
        int a = w.add(0, 1), b = w.add(0, 1), c = w.add(1, 1);
        p = {a, b, c};
        size_t fp;
        auto e = w.admit(p, 100, 0, 1000, fp);
        CHECK((e == std::vector<int64_t>{a, c}));
        w.complete(e);
        auto e2 = w.admit(p, 100, 0, 1000, fp);
        CHECK((e2 == std::vector<int64_t>{b}));
    }
    {  // drain: every request is admitted exactly once, in per-tensor order
        World w;
        std::deque<int64_t> p;
        std::srand(7);
        for (int q = 0; q < 500; ++q) p.push_back(w.add(std::rand() % 17, 1 + std::rand() % 50));
        std::vector<int> seen(500, 0);
        std::vector<int64_t> last(17, -1);
        size_t fp;
        int epochs = 0;
        while (!p.empty() && epochs < 10000) {
            auto e = w.admit(p, 8, 0, 120, fp);
            CHECK(!e.empty());
            for (int64_t r : e) {
                ++seen[r];
                CHECK(r > last[w.req_tensor[r]]);
                last[w.req_tensor[r]] = r;
            }
            w.complete(e);
            ++epochs;
        }
        for (int r = 0; r < 500; ++r) CHECK(seen[r] == 1);
    }
    std::printf(failures ? "sched: %d failures\n" : "sched: ok\n", failures);
    return failures ? 1 : 0;
}
