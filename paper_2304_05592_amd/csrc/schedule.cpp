// Binomial checkpointing schedule for the reverse (adjoint) sweep.
//
// The adjoint-state gradient needs the forward states S_j = (u^j, u^{j-1}) in reverse
// order j = n, n-1, ..., 1 while the forward recursion only runs forward.  With s restart
// slots (S_0 = 0 needs none) the schedule below stores some states during a forward sweep
// and recomputes the others from the nearest stored state.  It minimises the number of
// forward steps: the l-th reversal of a segment, counted from its stored start, costs r
// steps for C(s + r, s) consecutive values of l (the binomial law of optimal
// checkpointing), so the cost T(l, s) is convex in l and the optimal place of the next
// checkpoint is found by bisection on the discrete derivative.
#include "schedule.h"

#include <algorithm>
#include <cstdint>
#include <vector>

namespace awe {

namespace {

// Number of reversals whose cost is at most r with s free slots: C(s + r + 1, s + 1) - 1,
// saturated at `cap`.
long long cum(int s, long long r, long long cap) {
  // C(s + r + 1, s + 1) computed incrementally as prod_{i=1}^{s+1} (r + i) / i
  long double v = 1.0L;
  for (int i = 1; i <= s + 1; ++i) {
    v = v * (long double)(r + i) / (long double)i;
    if (v > (long double)cap * 4) return cap;
  }
  long long c = (long long)(v + 0.5L) - 1;
  return std::min(c, cap);
}

// Steps needed by the l-th reversal (l >= 1) with s free slots.
long long inc(long long l, int s) {
  if (s == 0) return l;
  long long lo = 1, hi = 1;
  while (cum(s, hi, l + 1) < l) hi *= 2;
  while (lo < hi) {
    long long mid = (lo + hi) / 2;
    if (cum(s, mid, l + 1) >= l) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// Position c in [1, l] of the next checkpoint for a segment of l reversals.
long long best_split(long long l, int s) {
  // delta(c) = 1 - inc(l - c, s - 1) + inc(c, s) is nondecreasing; take the first c >= 1
  // with delta(c) >= 0 (c = l when none).
  long long lo = 1, hi = l;
  while (lo < hi) {
    long long mid = (lo + hi) / 2;
    long long delta = 1 - inc(l - mid, s - 1) + inc(mid, s);
    if (delta >= 0) hi = mid; else lo = mid + 1;
  }
  return lo;
}

struct Builder {
  std::vector<int32_t>* out;
  int cur = 0;                 // current forward state held in the working buffers
  std::vector<int> slots;      // stack of stored states
  int max_depth = 0;

  void emit(int op, int a, int b) {
    out->push_back(op);
    out->push_back(a);
    out->push_back(b);
  }
  int slot_of(int state) const {
    for (int i = (int)slots.size() - 1; i >= 0; --i)
      if (slots[i] == state) return i;
    return -1;
  }
  void restore(int a) {
    if (cur == a) return;
    emit(kRestore, a == 0 ? -1 : slot_of(a), a);
    cur = a;
  }
  void advance(int to) {
    if (to > cur) emit(kAdvance, cur, to);
    cur = to;
  }
  // Reversals b, b-1, ..., a+1 with S_a restorable and s free slots.
  void ops(int a, int b, int s) {
    while (b > a) {
      const long long l = b - a;
      if (s == 0) {
        for (int j = b; j > a; --j) {
          restore(a);
          advance(j);
          emit(kReverse, j, 0);
        }
        return;
      }
      const int c = (int)best_split(l, s);
      restore(a);
      advance(a + c);
      if (c == l) {
        emit(kReverse, b, 0);
        b -= 1;
        continue;
      }
      slots.push_back(a + c);
      max_depth = std::max(max_depth, (int)slots.size());
      emit(kStore, (int)slots.size() - 1, a + c);
      ops(a + c, b, s - 1);
      restore(a + c);
      emit(kReverse, a + c, 0);
      slots.pop_back();
      b = a + c - 1;
    }
  }
};

}  // namespace

void build_schedule(int nsteps, int nslots, std::vector<int32_t>& actions) {
  actions.clear();
  Builder b;
  b.out = &actions;
  b.ops(0, nsteps, nslots);
}

long long schedule_cost(long long l, int s) {
  long long t = 0;
  for (long long i = 1; i <= l; ++i) t += inc(i, s);
  return t;
}

}  // namespace awe
