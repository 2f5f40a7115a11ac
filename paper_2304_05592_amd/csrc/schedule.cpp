// Binomial checkpointing schedule for the reverse (adjoint) sweep.
//
// The adjoint-state gradient needs the forward levels u^j in reverse order j = n, n-1, ..., 1
// while the forward recursion only runs forward.  With s restart slots (S_0 = 0 needs none)
// the schedule below stores some states S_j = (u^j, u^{j-1}) during a forward sweep and
// recomputes the others from the nearest stored state.  Every state, reached or restored,
// holds two consecutive levels and an adjoint step reads only its own one, so the reversals
// run in pairs from the top of a segment, (b, b-1), (b-2, b-3), ..., each pair served by one
// state.  The binomial law of optimal checkpointing then applies to the pairs: the l-th
// reversal of a segment, counted from its stored start, costs r steps for C(s + r, s)
// consecutive values of l, so the cost T(l, s) is convex in l and the optimal place of the
// next checkpoint is found by bisection on the discrete derivative; each pair counts two
// steps.  For an even length this is the fewest forward steps of the paired problem; for an
// odd one the lowest pair is the single level a+1, which can cost one step more.
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
  // Reverse j, and j - 1 as well when it lies in the segment: the state S_j in the working
  // buffers (reached, or restored) holds both u^j and u^{j-1}, and a reversal reads only its own
  // level.  Returns the next level still to reverse.
  int reverse_pair(int j, int a) {
    emit(kReverse, j, 0);
    if (j - 1 > a) {
      emit(kReverse, j - 1, 0);
      return j - 2;
    }
    return j - 1;
  }
  // Reversals b, b-1, ..., a+1 with S_a restorable and s free slots.
  void ops(int a, int b, int s) {
    while (b > a) {
      const long long l = b - a;
      if (s == 0) {
        for (int j = b; j > a;) {
          restore(a);
          advance(j);
          j = reverse_pair(j, a);
        }
        return;
      }
      // the reversals run in pairs from the top (b, b-1), (b-2, b-3), ...: the binomial law
      // applies to the pairs, the lowest of which is the single level a+1 when l is odd, so
      // the next checkpoint goes after k pairs, at a + 2k - (l odd)
      const long long k = best_split((l + 1) / 2, s);
      const int c = (int)(2 * k - (l & 1));
      restore(a);
      advance(a + c);
      if (c == l) {
        b = reverse_pair(b, a);
        continue;
      }
      slots.push_back(a + c);
      max_depth = std::max(max_depth, (int)slots.size());
      emit(kStore, (int)slots.size() - 1, a + c);
      ops(a + c, b, s - 1);
      restore(a + c);
      slots.pop_back();
      b = reverse_pair(a + c, a);
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
