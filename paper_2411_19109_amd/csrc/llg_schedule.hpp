// Checkpoint schedules of the discrete adjoint (host only).
//
// The forward run keeps snapshots of m; the adjoint restores them and
// recomputes forward steps, storing the four RK4 stage states and fields of
// the steps it is about to transpose.  Three policies:
//   SQRT      snapshots every K steps; each K-step segment is recomputed once
//             with stage stores.  With more than one segment the stage store is
//             double-buffered so that the recomputation of the next segment can
//             run while the current one is transposed.
//   ALL       one segment covering the whole run (stage store of every step).
//   BINOMIAL  s snapshot slots and a stage store of one step; the recursive
//             schedule of Griewank's binomial checkpointing (Revolve): to reverse
//             l steps with s snapshots (one holding the range start) and at most r sweeps over any
//             step, place the next snapshot so that the right part can be
//             reversed with s-1 slots and the left part with r-1 repetitions,
//             using beta(s, r) = C(s + r, s) = beta(s - 1, r) + beta(s, r - 1).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace llg {

enum PlanOp : int { P_LOAD = 0, P_ADV = 1, P_SAVE = 2, P_BSTEP = 3 };

// LOAD: state := snapshot slot (which holds m at step a)
// ADV:  advance the state from step a to step b (plain forward steps)
// SAVE: snapshot slot := state (at step a)
// BSTEP: recompute step a with stage stores from the state m_a, then transpose it
struct PlanAct {
    int op;
    int64_t a, b;
    int slot;
};

struct Plan {
    std::vector<PlanAct> acts;
    size_t split = 0;  // actions [0, split) run inside the forward pass
};

// beta(s, r) = C(s + r, s), saturated at 2^62.
int64_t binomial_beta(int64_t s, int64_t r);

// Smallest r with beta(s, r) >= l (l >= 1, s >= 1).
int64_t binomial_reps(int64_t l, int64_t s);

// Binomial schedule for n steps with `slots` snapshot slots (slot 0 holds m_0).
void binomial_plan(int64_t n, int slots, Plan& out);

// Segment length of the SQRT / ALL policies.
int64_t segment_length(int64_t n, int32_t policy, int32_t param);

// Snapshot slots of the BINOMIAL policy (param 0 -> 32, at most n).
int binomial_slots(int64_t n, int32_t param);

// Device bytes of the checkpoint store: snapshots (state_mult arrays of N3 each:
// a float state is kept as hi + lo) and stage-state slots.
size_t store_bytes(int64_t N3, size_t tsz, int64_t n, int32_t policy, int32_t param, int state_mult);

// Forward steps the adjoint recomputes (after the forward pass) under a policy.
int64_t recompute_steps(int64_t n, int32_t policy, int32_t param);

}  // namespace llg
