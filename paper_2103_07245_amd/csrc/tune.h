// Autotune cache: the launch plan chosen for a shape class by timing candidate
// plans on the device (pbpqlp_tune_factor, pbpqlp_tune_batch).
//
// A shape class is (storage type, precision plan, lp32 = l rounded up to 32,
// ceil(log2 m), ceil(log2 n), batched or not).  A plan is the contraction
// split of the A-streaming passes and the Gram workgroup target; every other
// tile shape is fixed per precision and exact per l, so these two are what
// changes the work decomposition from one matrix size to another.
#pragma once
#include <stdint.h>

namespace pbq {

struct TuneKey {
  int dt, sketch, power, proj, lp32, mb, nb, batched;
  bool operator<(const TuneKey& o) const;
};

struct TunePlan {
  int split_k = 0;          // 0: the built-in heuristic
  int gram_wg = 0;          // 0: the built-in default
  double ms = 0.0;          // measured time of the plan
};

TuneKey tune_key(int dt, int sketch, int power, int proj, int l, int64_t m, int64_t n, bool batched);
bool tune_lookup(const TuneKey& k, TunePlan* out);
void tune_store(const TuneKey& k, const TunePlan& p);

}  // namespace pbq
