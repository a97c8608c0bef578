// Checkpoint schedules of the discrete adjoint (host only); see llg_schedule.hpp.
#include "llg_schedule.hpp"

#include <algorithm>
#include <cmath>

#include "../../include/llg.h"

namespace llg {

int64_t binomial_beta(int64_t s, int64_t r) {
    // C(s + r, s) = prod_{i=1..r} (s + i) / i, exact in integers while below the cap
    const int64_t cap = (int64_t)1 << 62;
    if (s < 0 || r < 0) return 0;
    long double v = 1.0L;
    int64_t b = 1;
    for (int64_t i = 1; i <= r; ++i) {
        v = v * (long double)(s + i) / (long double)i;
        if (v >= (long double)cap) return cap;
        b = (int64_t)((__int128)b * (s + i) / i);  // exact: the running product is C(s + i, i)
    }
    return b;
}

int64_t binomial_reps(int64_t l, int64_t s) {
    int64_t r = 0;
    while (binomial_beta(s, r) < l) ++r;
    return r;
}

namespace {

// Reverse steps [a, b): m_a sits in slot ca; free holds the unused slots.
void revolve(int64_t a, int64_t b, int ca, std::vector<int>& free, std::vector<PlanAct>& out) {
    const int64_t l = b - a;
    if (l == 1) {
        out.push_back({P_LOAD, a, a, ca});
        out.push_back({P_BSTEP, a, a + 1, -1});
        return;
    }
    if (free.empty()) {
        // no slot left: every step is reached again from m_a
        for (int64_t k = b - 1; k >= a; --k) {
            out.push_back({P_LOAD, a, a, ca});
            if (k > a) out.push_back({P_ADV, a, k, -1});
            out.push_back({P_BSTEP, k, k + 1, -1});
        }
        return;
    }
    // s snapshots in use for this range: the one holding m_a and the free ones
    const int64_t s = (int64_t)free.size() + 1;
    const int64_t r = binomial_reps(l, s);
    const int64_t mid = a + std::max<int64_t>(1, l - binomial_beta(s - 1, r));
    out.push_back({P_LOAD, a, a, ca});
    out.push_back({P_ADV, a, mid, -1});
    const int c = free.back();
    free.pop_back();
    out.push_back({P_SAVE, mid, mid, c});
    revolve(mid, b, c, free, out);
    free.push_back(c);
    revolve(a, mid, ca, free, out);
}

}  // namespace

void binomial_plan(int64_t n, int slots, Plan& out) {
    out.acts.clear();
    std::vector<int> free;
    for (int c = slots - 1; c >= 1; --c) free.push_back(c);
    revolve(0, n, 0, free, out.acts);
    // the forward pass runs everything before the load that precedes the first transposed step
    size_t first_b = 0;
    while (first_b < out.acts.size() && out.acts[first_b].op != P_BSTEP) ++first_b;
    size_t split = first_b;
    while (split > 0 && out.acts[split].op != P_LOAD) --split;
    out.split = split;
}

int64_t segment_length(int64_t n, int32_t policy, int32_t param) {
    if (n <= 0) return 1;
    if (policy == LLG_CKPT_ALL) return n;
    if (policy == LLG_CKPT_BINOMIAL) return 1;
    if (param > 0) return std::min<int64_t>(param, n);
    const int64_t K = (int64_t)std::ceil(std::sqrt((double)n));
    return std::max<int64_t>(1, K);
}

int binomial_slots(int64_t n, int32_t param) {
    const int64_t s = param > 0 ? param : 32;
    return (int)std::max<int64_t>(1, std::min<int64_t>(s, n));
}

size_t store_bytes(int64_t N3, size_t tsz, int64_t n, int32_t policy, int32_t param, int state_mult) {
    if (policy == LLG_CKPT_BINOMIAL) return (size_t)(binomial_slots(n, param) * state_mult * N3 + 8 * N3) * tsz;
    const int64_t K = segment_length(n, policy, param);
    const int64_t nsnap = (n + K - 1) / K;
    const int64_t halves = nsnap > 1 ? 2 : 1;
    return (size_t)(nsnap * state_mult * N3 + 8 * K * N3 * halves) * tsz;
}

int64_t recompute_steps(int64_t n, int32_t policy, int32_t param) {
    if (policy != LLG_CKPT_BINOMIAL) return n;
    Plan p;
    binomial_plan(n, binomial_slots(n, param), p);
    int64_t steps = 0;
    for (size_t i = p.split; i < p.acts.size(); ++i) {
        const PlanAct& q = p.acts[i];
        if (q.op == P_ADV) steps += q.b - q.a;
        if (q.op == P_BSTEP) steps += 1;
    }
    return steps;
}

}  // namespace llg
