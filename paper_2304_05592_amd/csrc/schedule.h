// Binomial checkpointing schedule (host only).
#pragma once

#include <cstdint>
#include <vector>

namespace awe {

enum ScheduleOp : int32_t { kAdvance = 0, kStore = 1, kRestore = 2, kReverse = 3 };

// Actions (op, a, b) reversing levels n..1 with nslots free restart slots; S_0 is the zero
// state.  ADVANCE a -> b; STORE slot a <- state b; RESTORE slot a (-1: zero state) = state b;
// REVERSE level a (the current state is a or a + 1: S_j holds u^j and u^{j-1}).
void build_schedule(int nsteps, int nslots, std::vector<int32_t>& actions);

// Minimal number of forward steps for l reversals with s free slots when every reversal needs
// its own state (the classic law; the schedule above pairs the reversals and needs fewer).
long long schedule_cost(long long l, int s);

}  // namespace awe
