// Autotuner of the synthesis kernels: times the candidate kernel shapes of one
// problem and grid on the device and keeps the fastest.
//
// Synthesis. The stages are independent, so each is tuned alone with the
// others switched off: first the modal sum's row blocking (rows of the
// synthesis matrix per wavefront), then the transform (kind, radix of the
// factored y pass, tiling). The default configuration and the winner are then
// timed as whole calls in the same sweep; the winner is kept only if it beats
// the default there.
//
// Batched synthesis. One persistent kernel: the radix P of its factored y pass,
// the number of resident blocks per CU and the work items taken per grab of
// the queue counter are swept jointly.
//
// Every candidate is timed twice, interleaved with the others, and its
// smaller mean is used, so that a slow first pass (clocks ramping up, caches
// cold) does not decide.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <limits>
#include <vector>

#include "scw_internal.h"

namespace scw {
namespace {

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Mean milliseconds of `reps` calls of `run` after one warm-up call.
int time_calls(const std::function<int()>& run, hipStream_t st, int reps, double* ms) {
  Events ev;
  SCW_HIP(hipEventCreate(&ev.a));
  SCW_HIP(hipEventCreate(&ev.b));
  int rc = run();
  if (rc) return rc;
  SCW_HIP(hipEventRecord(ev.a, st));
  for (int i = 0; i < reps; ++i)
    if ((rc = run())) return rc;
  SCW_HIP(hipEventRecord(ev.b, st));
  SCW_HIP(hipEventSynchronize(ev.b));
  float t = 0.f;
  SCW_HIP(hipEventElapsedTime(&t, ev.a, ev.b));
  *ms = (double)t / reps;
  return SCW_OK;
}

// Sweeps candidates 0..n-1 twice; returns the index of the fastest (-1 if
// none ran). `run(i)` returns SCW_EINVAL for a candidate the shape cannot
// run, which is skipped.
int sweep(int n, const std::function<int(int)>& prepare, const std::function<int()>& run,
          hipStream_t st, int reps, std::vector<double>& best_ms, int* counted) {
  best_ms.assign(n, std::numeric_limits<double>::infinity());
  std::vector<char> ok(n, 1);
  for (int pass = 0; pass < 2; ++pass)
    for (int i = 0; i < n; ++i) {
      if (!ok[i]) continue;
      int rc = prepare(i);
      double ms = 0;
      if (rc == SCW_OK) rc = time_calls(run, st, reps, &ms);
      if (rc == SCW_EINVAL) {
        ok[i] = 0;
        continue;
      }
      if (rc) return rc;
      best_ms[i] = std::min(best_ms[i], ms);
    }
  int best = -1;
  for (int i = 0; i < n; ++i) {
    if (!ok[i]) continue;
    ++*counted;
    if (best < 0 || best_ms[i] < best_ms[best]) best = i;
  }
  return best;
}

}  // namespace

// Restores a solution's explicit configuration when the tuner returns (the
// tuner's result lives in the context, keyed by shape and precision), and
// frees the plans the candidates were built with: they were used only by the
// tuner's own launches on its stream, which it has synchronised by then.
struct ConfigGuard {
  Solution& s;
  scw_synth_config saved;
  size_t n_plans;
  explicit ConfigGuard(Solution& sol) : s(sol), saved(sol.cfg), n_plans(sol.plans.size()) {}
  void drop_candidate_plans() {
    if (s.plans.size() > n_plans) s.plans.resize(n_plans);
  }
  ~ConfigGuard() { s.cfg = saved; }
};

int tune_synthesis(Context& c, Solution& s, const scw_grid& g, int precision, void* E,
                   hipStream_t st, int reps, scw_tune_report* rep) {
  const std::string key = synth_key(s, g, precision);
  ConfigGuard guard(s);
  // candidates are timed without the context's tuned entry for this shape
  auto prior = c.tuned_synth.find(key);
  const bool had_prior = prior != c.tuned_synth.end();
  const scw_synth_config prior_cfg = had_prior ? prior->second : scw_synth_config{};
  c.tuned_synth.erase(key);
  auto use = [&](const scw_synth_config& cf) { s.cfg = cf; };
  // on an error the stream is drained, the candidate plans freed and the
  // context's earlier entry for this shape restored
  auto bail = [&](int r) {
    (void)hipStreamSynchronize(st);
    guard.drop_candidate_plans();
    if (had_prior) c.tuned_synth[key] = prior_cfg;
    return r;
  };
  Plan* last = nullptr;
  // builds the plan of the current configuration without launching kernels
  auto plan_only = [&]() {
    int r = synthesize(c, s, g, precision, E, st, 0, nullptr, false, &last);
    if (r == SCW_EINVAL) set_error(SCW_OK, "");
    return r;
  };
  auto stage = [&](int mask) {
    return [&, mask]() { return synthesize(c, s, g, precision, E, st, mask, nullptr); };
  };
  int counted = 0;
  scw_synth_config best{};
  std::vector<double> ms;
  // stage 1: modal-sum row blocking (the FP32 kernel of the single and split modes)
  if (precision != SCW_FP64) {
    const int rows[] = {2, 4, 8, 16};
    auto prep = [&](int i) {
      use(scw_synth_config{rows[i], 0, 0, 0});
      int r = plan_only();
      if (r == SCW_OK && last->modal_rw != rows[i]) r = SCW_EINVAL;  // capped: a duplicate
      return r;
    };
    const int b = sweep(4, prep, stage(kStageModal), st, reps, ms, &counted);
    if (b < -1) return bail(b);
    if (b < 0) return bail(fail(SCW_EINVAL, "no modal-sum configuration ran"));
    best.modal_rows = rows[b];
  }
  // stage 2: the transform, on the spectra of one complete call
  {
    use(scw_synth_config{best.modal_rows, 0, 0, 0});
    int rc = synthesize(c, s, g, precision, E, st, kStageAll, nullptr);
    if (rc) return bail(rc);
    const bool split = precision == SCW_BF16X3 || precision == SCW_FP16X3;
    std::vector<scw_synth_config> cands;
    if (!split)
      for (int P = 2; P <= 32; P *= 2)
        for (int cols : {64, 32}) cands.push_back({best.modal_rows, SCW_XFORM_FFT, P, cols});
    if (precision != SCW_FP64)
      for (int t : {0, 1, 2, 4, 8}) cands.push_back({best.modal_rows, SCW_XFORM_MFMA, 0, t});
    if (!split)
      for (int t : {0, 1, 2, 4}) cands.push_back({best.modal_rows, SCW_XFORM_DIRECT, 0, t});
    auto prep = [&](int i) {
      use(cands[i]);
      return plan_only();
    };
    const int b = sweep((int)cands.size(), prep, stage(kStageTransform), st, reps, ms, &counted);
    if (b < -1) return bail(b);
    if (b < 0) return bail(fail(SCW_EINVAL, "no transform configuration ran"));
    best = cands[b];
  }
  // the winner against the default as whole calls, alternately, twice each
  double best_ms = 1e300, default_ms = 1e300;
  for (int pass = 0; pass < 2; ++pass) {
    double t = 0;
    use(scw_synth_config{});
    int rc = time_calls(stage(kStageAll), st, reps, &t);
    if (rc) return bail(rc);
    default_ms = std::min(default_ms, t);
    use(best);
    if ((rc = time_calls(stage(kStageAll), st, reps, &t))) return bail(rc);
    best_ms = std::min(best_ms, t);
  }
  if (best_ms > default_ms) {  // the stage winners did not pay off as a whole
    best = scw_synth_config{};
    best_ms = default_ms;
  }
  SCW_HIP(hipStreamSynchronize(st));
  guard.drop_candidate_plans();
  c.tuned_synth[key] = best;
  // the field of the chosen configuration, as the caller's later calls
  // without an explicit configuration will compute it
  use(scw_synth_config{});
  Plan* chosen = nullptr;
  int rc = synthesize(c, s, g, precision, E, st, kStageAll, nullptr, false, &chosen);
  if (rc) return rc;
  SCW_HIP(hipStreamSynchronize(st));
  if (rep) {
    *rep = scw_tune_report{};
    rep->n_candidates = counted;
    rep->default_ms = default_ms;
    rep->best_ms = best_ms;
    const Plan& pl = *chosen;
    rep->config.modal_rows = precision == SCW_FP64 ? 0 : pl.modal_rw;
    rep->config.transform = pl.fft_p ? SCW_XFORM_FFT : (pl.mfma ? SCW_XFORM_MFMA : SCW_XFORM_DIRECT);
    rep->config.fft_radix = pl.fft_p;
    rep->config.tiles = pl.tiles;
  }
  return SCW_OK;
}

int tune_batch(scw_batch* b, void* E, hipStream_t st, int reps, scw_tune_report* rep) {
  using Shape = Context::BatchShape;
  const Shape def{b->P, std::max(1, b->grid_blocks / std::max(1, b->cus)), b->chunk};
  std::vector<Shape> cands;
  for (int P = 2; P <= 32; P *= 2)
    for (int pc : {1, 2, 4, 8})
      for (int ch : {1, 4, 16}) cands.push_back({P, pc, ch});
  auto run = [&]() -> int {
    SCW_HIP(launch_batch(batch_args(b, E), st));
    return SCW_OK;
  };
  double default_ms = 0;
  int rc = time_calls(run, st, reps, &default_ms);
  if (rc) return rc;
  auto prep = [&](int i) {
    int r = batch_set_shape(b, cands[i].P, cands[i].blocks_per_cu, cands[i].chunk);
    if (r == SCW_EINVAL) set_error(SCW_OK, "");
    return r;
  };
  std::vector<double> ms;
  int counted = 0;
  const int best = sweep((int)cands.size(), prep, run, st, reps, ms, &counted);
  Shape win = def;
  double best_ms = default_ms;
  if (best >= 0 && ms[best] < default_ms) {
    win = cands[best];
    best_ms = ms[best];
  }
  if ((rc = batch_set_shape(b, win.P, win.blocks_per_cu, win.chunk))) return rc;
  b->ctx->tuned_batch[batch_key(b->grid)] = win;
  if ((rc = run())) return rc;
  SCW_HIP(hipStreamSynchronize(st));
  if (rep) {
    *rep = scw_tune_report{};
    rep->n_candidates = counted;
    rep->default_ms = default_ms;
    rep->best_ms = best_ms;
    rep->batch_radix = win.P;
    rep->batch_blocks_per_cu = win.blocks_per_cu;
    rep->batch_chunk = win.chunk;
  }
  return SCW_OK;
}

}  // namespace scw

extern "C" {

int scw_tune_synthesis(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid, int precision,
                       void* E_dev, void* hip_stream, int reps, scw_tune_report* report) {
  if (!ctx || !sol || !grid || !E_dev) return scw::fail(SCW_EINVAL, "null argument");
  if (reps < 1 || reps > 1000) return scw::fail(SCW_EINVAL, "reps must be in [1, 1000]");
  // validate the request as scw_synthesize would
  int rc = scw_synthesize(ctx, sol, grid, precision, E_dev, hip_stream);
  if (rc) return rc;
  return scw::tune_synthesis(ctx->c, sol->s, *grid, precision, E_dev,
                             reinterpret_cast<hipStream_t>(hip_stream), reps, report);
}

int scw_batch_tune(scw_batch* batch, void* E_dev, void* hip_stream, int reps,
                   scw_tune_report* report) {
  if (!batch || !E_dev) return scw::fail(SCW_EINVAL, "null argument");
  if (reps < 1 || reps > 1000) return scw::fail(SCW_EINVAL, "reps must be in [1, 1000]");
  SCW_HIP(hipSetDevice(batch->ctx->device));
  return scw::tune_batch(batch, E_dev, reinterpret_cast<hipStream_t>(hip_stream), reps, report);
}

}  // extern "C"
