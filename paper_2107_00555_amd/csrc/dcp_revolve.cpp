// dcp_revolve.cpp -- binomial checkpointing schedule for the reverse sweep
// (host code only).
//
// Reversing T steps from the state u_a of a held buffer with s free snapshot
// slots and one work buffer: advance to a split point m, store u_m in a free
// slot, reverse [m, b) with one slot fewer, then reverse [a, m) with the slot
// free again.  With no free slot, each step t of [a, b) is recomputed from
// u_a into the work buffer.  With c = s + 1 snapshots (the held state
// counts) and r repetitions at most, beta(c, r) = C(c + r, c) steps can be
// reversed (the binomial count of Griewank and Walther's checkpointing);
// the split m - a is taken in
//     [max(beta(c, r-2), l - beta(c-1, r)), min(beta(c, r-1), l - beta(c-1, r-1))]
// for l = b - a and the least r with beta(c, r) >= l.  Every split in that
// range gives the least number of forward steps, r*l - beta(c+1, r-1)
// (checked against an exhaustive dynamic program for l < 260, s < 8, and by
// the tests on the schedules this file emits).
#include <algorithm>
#include <cstdint>
#include <vector>

#include "dcp.h"
#include "dcp_internal.h"

namespace dcp {

namespace {

constexpr int64_t kSat = (int64_t)1 << 62;

// C(c + r, c), saturating at 2^62; 0 for r < 0.
int64_t beta(int64_t c, int64_t r) {
    if (r < 0 || c < 0) return 0;
    int64_t v = 1;
    const int64_t k = std::min(c, r);
    for (int64_t i = 1; i <= k; ++i) {
        // v * (c + r - k + i) / i, exact at every step
        const int64_t num = c + r - k + i;
        if (v > kSat / num) return kSat;
        v = v * num / i;
    }
    return v;
}

struct Task {
    int64_t a, b;
    int32_t src, free0, nfree;
};

}  // namespace

bool revolve_schedule(int64_t T, int32_t nslots, std::vector<RvOp> *ops, int64_t *forward_steps) {
    ops->clear();
    int64_t fwd = 0;
    if (T <= 0 || nslots < 0) {
        if (forward_steps) *forward_steps = 0;
        return T >= 0 && nslots >= 0;
    }
    const int32_t W = nslots;
    std::vector<Task> stack;
    stack.push_back(Task{0, T, kRvOrigin, 0, nslots});
    while (!stack.empty()) {
        const Task k = stack.back();
        stack.pop_back();
        const int64_t l = k.b - k.a;
        if (l == 1) {
            ops->push_back(RvOp{kRvAdjoint, k.src, -1, k.a, k.a});
            continue;
        }
        if (k.nfree == 0) {
            for (int64_t t = k.b - 1; t > k.a; --t) {
                ops->push_back(RvOp{kRvAdvance, k.src, W, k.a, t});
                fwd += t - k.a;
                ops->push_back(RvOp{kRvAdjoint, W, -1, t, t});
            }
            ops->push_back(RvOp{kRvAdjoint, k.src, -1, k.a, k.a});
            continue;
        }
        const int64_t c = (int64_t)k.nfree + 1;
        int64_t r = 0;
        while (beta(c, r) < l) ++r;
        const int64_t lo = std::max({beta(c, r - 2), l - beta(c - 1, r), (int64_t)1});
        const int64_t hi = std::min({beta(c, r - 1), l - beta(c - 1, r - 1), l - 1});
        const int64_t m = k.a + std::max(lo, std::min(hi, l - 1));
        const int32_t slot = k.free0;
        ops->push_back(RvOp{kRvAdvance, k.src, slot, k.a, m});
        fwd += m - k.a;
        // the right part first (pushed last), with one slot fewer
        stack.push_back(Task{k.a, m, k.src, k.free0, k.nfree});
        stack.push_back(Task{m, k.b, slot, k.free0 + 1, k.nfree - 1});
    }
    if (forward_steps) *forward_steps = fwd;
    return true;
}

}  // namespace dcp

extern "C" int dcp_revolve_schedule(int64_t T, int32_t nslots, int64_t *ops, int64_t cap, int64_t *nops,
                                    int64_t *forward_steps) {
    if (!nops) return DCP_E_NULL;
    if (T < 0 || nslots < 0 || cap < 0) return DCP_E_ARG;
    std::vector<dcp::RvOp> v;
    if (!dcp::revolve_schedule(T, nslots, &v, forward_steps)) return DCP_E_ARG;
    *nops = (int64_t)v.size();
    if (ops) {
        if (cap < (int64_t)v.size()) return DCP_E_WORKSPACE;
        for (size_t i = 0; i < v.size(); ++i) {
            ops[5 * i + 0] = v[i].kind;
            ops[5 * i + 1] = v[i].src;
            ops[5 * i + 2] = v[i].dst;
            ops[5 * i + 3] = v[i].t0;
            ops[5 * i + 4] = v[i].t1;
        }
    }
    return DCP_OK;
}
