// Autotuner of the launch plan per shape class (host code).
//
// pbpqlp_tune_factor times every candidate plan of one problem -- the
// contraction split of the streaming passes (automatic, 1, 2, 4, 8, 16) and
// the Gram workgroup target (default, 64, 256, 1024) -- with HIP events on the
// caller's stream, and keeps the fastest for the problem's shape class.
// pbpqlp_tune_batch does the same for the Gram target of a batch plan.  Later
// calls whose options leave both choices automatic (split_k = 0,
// gram_workgroups = 0) use the cached plan of their class.  The cache is
// process-wide, guarded by a reader-writer lock, and can be written to and
// read from a text file (one class per line).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <shared_mutex>
#include <vector>

#include "../../include/pbpqlp.h"
#include "tune.h"

namespace pbq {

bool TuneKey::operator<(const TuneKey& o) const {
  const int a[8] = {dt, sketch, power, proj, lp32, mb, nb, batched};
  const int b[8] = {o.dt, o.sketch, o.power, o.proj, o.lp32, o.mb, o.nb, o.batched};
  return std::lexicographical_compare(a, a + 8, b, b + 8);
}

namespace {
std::shared_mutex g_mu;
std::map<TuneKey, TunePlan>& cache() {
  static std::map<TuneKey, TunePlan> c;
  return c;
}
int ceil_log2(int64_t x) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < x) ++b;
  return b;
}
}  // namespace

TuneKey tune_key(int dt, int sketch, int power, int proj, int l, int64_t m, int64_t n, bool batched) {
  TuneKey k;
  k.dt = dt;
  k.sketch = sketch;
  k.power = power;
  k.proj = proj;
  k.lp32 = (l + 31) / 32 * 32;
  k.mb = ceil_log2(m);
  k.nb = ceil_log2(n);
  k.batched = batched ? 1 : 0;
  return k;
}

bool tune_lookup(const TuneKey& k, TunePlan* out) {
  std::shared_lock<std::shared_mutex> lk(g_mu);
  auto it = cache().find(k);
  if (it == cache().end()) return false;
  *out = it->second;
  return true;
}

void tune_store(const TuneKey& k, const TunePlan& p) {
  std::unique_lock<std::shared_mutex> lk(g_mu);
  cache()[k] = p;
}

}  // namespace pbq

using namespace pbq;

namespace {

TuneKey key_of(int64_t m, int64_t n, int k, int p, pbpqlp_dtype dt, const pbpqlp_opts* opts, bool batched) {
  pbpqlp_opts o;
  pbpqlp_default_opts(&o);
  if (opts) o = *opts;
  return tune_key((int)dt, o.sketch_prec, o.power_prec, o.proj_prec, k + p, m, n, batched);
}

// Median of `reps` timed runs of fn() on stream st (after one warm-up run).
template <class F>
pbpqlp_status time_runs(F fn, hipStream_t st, int reps, double* ms_out) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return PBPQLP_EHIP;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return PBPQLP_EHIP;
  }
  pbpqlp_status s = fn();
  std::vector<float> t;
  for (int r = 0; r < reps && s == PBPQLP_OK; ++r) {
    if (hipEventRecord(a, st) != hipSuccess) s = PBPQLP_EHIP;
    if (!s) s = fn();
    if (!s && hipEventRecord(b, st) != hipSuccess) s = PBPQLP_EHIP;
    float ms = 0.f;
    if (!s && (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess))
      s = PBPQLP_EHIP;
    t.push_back(ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (s) return s;
  std::sort(t.begin(), t.end());
  *ms_out = t[t.size() / 2];
  return PBPQLP_OK;
}

}  // namespace

extern "C" {

pbpqlp_status pbpqlp_tune_factor(const void* A, int64_t m, int64_t n, int64_t lda, pbpqlp_dtype dt,
                                 int k, int p, int q, uint64_t seed, const pbpqlp_opts* opts,
                                 pbpqlp_tune_plan* out, void* stream) {
  if (!A || k < 1 || p < 0 || m < 1 || n < 1 || k + p > (m < n ? m : n)) return PBPQLP_EINVAL;
  if (dt != PBPQLP_F64 && dt != PBPQLP_F32) return PBPQLP_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int l = k + p;
  const size_t el = dt == PBPQLP_F64 ? 8 : 4;
  // outputs and the result record of the trial runs
  char* buf = nullptr;
  const size_t bytes = ((size_t)(m + n) * l * el + 255) / 256 * 256 + (size_t)l * l * 8 + 256;
  if (hipMallocAsync((void**)&buf, bytes, st) != hipSuccess) return PBPQLP_ENOMEM;
  void* Q = buf;
  void* P = buf + (size_t)m * l * el;
  double* L = (double*)(buf + ((size_t)(m + n) * l * el + 255) / 256 * 256);
  pbpqlp_info* info = (pbpqlp_info*)((char*)L + (size_t)l * l * 8);
  pbpqlp_opts base;
  pbpqlp_default_opts(&base);
  if (opts) base = *opts;
  base.workspace = nullptr;
  base.workspace_bytes = 0;
  const int splits[] = {0, 1, 2, 4, 8, 16};
  const int grams[] = {0, 64, 512, 1024};
  TunePlan best;
  best.ms = -1.0;
  pbpqlp_status s = PBPQLP_OK;
  for (int sk : splits) {
    for (int gw : grams) {
      pbpqlp_opts o = base;
      // a trial plan is explicit: 0 would read the cache being filled; the
      // heuristic split is marked by -1 and the default Gram target is 256
      o.split_k = sk;
      o.gram_workgroups = gw == 0 ? 256 : gw;
      if (sk == 0) o.split_k = -1;
      double ms = 0.0;
      s = time_runs([&]() {
        return pbpqlp_factor(A, m, n, lda, dt, k, p, q, seed, Q, l, L, l, P, l, &o, info, stream);
      }, st, 3, &ms);
      if (s) break;
      if (best.ms < 0.0 || ms < best.ms) {
        best.ms = ms;
        best.split_k = sk == 0 ? -1 : sk;
        best.gram_wg = o.gram_workgroups;
      }
    }
    if (s) break;
  }
  (void)hipFreeAsync(buf, st);
  if (s) return s;
  tune_store(key_of(m, n, k, p, dt, opts, false), best);
  if (out) {
    out->split_k = best.split_k;
    out->gram_workgroups = best.gram_wg;
    out->ms = best.ms;
  }
  return PBPQLP_OK;
}

pbpqlp_status pbpqlp_tune_batch(int count, const pbpqlp_problem* problems, pbpqlp_dtype dt,
                                const pbpqlp_opts* opts, pbpqlp_tune_plan* out, void* stream) {
  if (count < 1 || !problems) return PBPQLP_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  pbpqlp_opts base;
  pbpqlp_default_opts(&base);
  if (opts) base = *opts;
  const int grams[] = {4, 16, 64, 256};
  TunePlan best;
  best.ms = -1.0;
  for (int gw : grams) {
    pbpqlp_opts o = base;
    o.gram_workgroups = gw;
    pbpqlp_batch* b = nullptr;
    pbpqlp_status s = pbpqlp_batch_create(count, problems, dt, &o, &b);
    if (s) return s;
    double ms = 0.0;
    s = time_runs([&]() { return pbpqlp_batch_run(b, stream); }, st, 3, &ms);
    (void)hipStreamSynchronize(st);
    pbpqlp_batch_destroy(b);
    if (s) return s;
    if (best.ms < 0.0 || ms < best.ms) {
      best.ms = ms;
      best.split_k = 1;
      best.gram_wg = gw;
    }
  }
  // one class per batch: the key of its first problem, marked batched
  const pbpqlp_problem& p0 = problems[0];
  tune_store(key_of(p0.m, p0.n, p0.k, p0.p, dt, opts, true), best);
  if (out) {
    out->split_k = best.split_k;
    out->gram_workgroups = best.gram_wg;
    out->ms = best.ms;
  }
  return PBPQLP_OK;
}

pbpqlp_status pbpqlp_tune_lookup(int64_t m, int64_t n, int k, int p, pbpqlp_dtype dt,
                                 const pbpqlp_opts* opts, int batched, pbpqlp_tune_plan* out) {
  if (!out) return PBPQLP_EINVAL;
  TunePlan t;
  if (!tune_lookup(key_of(m, n, k, p, dt, opts, batched != 0), &t)) return PBPQLP_EINVAL;
  out->split_k = t.split_k;
  out->gram_workgroups = t.gram_wg;
  out->ms = t.ms;
  return PBPQLP_OK;
}

void pbpqlp_tune_clear(void) {
  std::unique_lock<std::shared_mutex> lk(g_mu);
  cache().clear();
}

pbpqlp_status pbpqlp_tune_save(const char* path) {
  if (!path) return PBPQLP_EINVAL;
  FILE* fp = std::fopen(path, "w");
  if (!fp) return PBPQLP_EINVAL;
  std::shared_lock<std::shared_mutex> lk(g_mu);
  bool ok = std::fprintf(fp, "# pbpqlp autotune v1: dt sketch power proj lp32 log2m log2n batched split_k gram_wg ms\n") > 0;
  for (const auto& kv : cache()) {
    const TuneKey& k = kv.first;
    const TunePlan& t = kv.second;
    ok = ok && std::fprintf(fp, "%d %d %d %d %d %d %d %d %d %d %.6f\n", k.dt, k.sketch, k.power, k.proj,
                            k.lp32, k.mb, k.nb, k.batched, t.split_k, t.gram_wg, t.ms) > 0;
  }
  const bool closed = std::fclose(fp) == 0;
  return ok && closed ? PBPQLP_OK : PBPQLP_EINVAL;
}

pbpqlp_status pbpqlp_tune_load(const char* path) {
  if (!path) return PBPQLP_EINVAL;
  FILE* fp = std::fopen(path, "r");
  if (!fp) return PBPQLP_EINVAL;
  char line[512];
  std::vector<std::pair<TuneKey, TunePlan>> rows;
  bool ok = std::fgets(line, sizeof(line), fp) && std::strncmp(line, "# pbpqlp autotune v1", 20) == 0;
  while (ok && std::fgets(line, sizeof(line), fp)) {
    TuneKey k;
    TunePlan t;
    if (line[0] == '\n' || line[0] == '#') continue;
    const int got = std::sscanf(line, "%d %d %d %d %d %d %d %d %d %d %lf", &k.dt, &k.sketch, &k.power,
                                &k.proj, &k.lp32, &k.mb, &k.nb, &k.batched, &t.split_k, &t.gram_wg, &t.ms);
    ok = got == 11 && t.split_k >= -1 && t.gram_wg >= 0;
    if (ok) rows.push_back({k, t});
  }
  std::fclose(fp);
  if (!ok) return PBPQLP_EINVAL;
  std::unique_lock<std::shared_mutex> lk(g_mu);
  for (const auto& r : rows) cache()[r.first] = r.second;
  return PBPQLP_OK;
}

}  // extern "C"
