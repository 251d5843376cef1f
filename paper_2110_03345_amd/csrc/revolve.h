// Binomial checkpointing schedule for reversing a chain of time steps
// (Griewank & Walther, "Algorithm 799: revolve", ACM TOMS 26(1), 2000),
// written from the published description: with s free snapshot slots, the
// minimal number of forward steps that reverses l steps is
//     C(l, 0) = l (l - 1) / 2,
//     C(l, s) = t l - beta(s + 2, t - 1),  t = min{t : beta(s + 1, t) >= l},
// where beta(c, t) = (c + t)! / (c! t!).  The schedule is produced by the
// recursion  advance to m, store x_m, reverse [m, b) with s - 1 slots, free,
// restore x_a, reverse [a, m) with s slots, choosing m to minimise
// m + C(l - m, s - 1) + C(m, s).
#pragma once

#include <cstdint>
#include <memory>
#include <vector>

namespace stride {

enum class Act : uint8_t { Advance, Store, Restore, Free, Reverse };

struct Action {
    Act type;
    int step;   // Advance: target index; Store/Restore/Free/Reverse: state index
};

// Minimal forward steps to reverse l steps from a stored x_0 with s free slots.
long long revolve_cost(long long l, long long s);

// Schedule reversing states 0..nt-1 (nt reverse operations) with at most
// `snaps` simultaneously stored states besides x_0.  The first Reverse comes
// after the working state has advanced through every index 0..nt-1 once.
std::vector<Action> revolve_schedule(int nt, int snaps);

struct ScheduleStats {
    long long forward_steps;   // total Advance steps (nt - 1 = no recompute)
    int peak_fields;           // distinct wavefields alive at once, including
                               // the working state and a step's output
    int max_snaps;             // largest number of stored states at once
};

// Replays a schedule against a reference-counted pool of wavefields: a state
// x_i is the pair (u^i, u^{i-1}); consecutive stored states share a field.
ScheduleStats schedule_stats(const std::vector<Action>& sched);

struct CachedSchedule {
    std::vector<Action> actions;
    ScheduleStats stats;
};

// revolve_schedule + schedule_stats, memoised per (nt, snaps) for the process.
std::shared_ptr<const CachedSchedule> cached_schedule(int nt, int snaps);

// Largest snapshot count whose schedule fits in `fields` wavefields
// (fields >= 3 required); returns -1 when even 0 snapshots do not fit.
int snaps_for_fields(int nt, long long fields);

}  // namespace stride
