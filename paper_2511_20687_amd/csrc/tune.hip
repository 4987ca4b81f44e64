// Launch-configuration autotuner of a context.  The method (Alg. 1) fixes what
// every Schwarz sweep computes; how fast it runs depends on the FE launch shape
// (column kernel: threads per workgroup and layers per thread; layer-staged
// kernel: layers per workgroup), the OpInf evaluation path (fused or batched)
// and the launch mode (host launches, or replays of a captured graph on one or
// two streams, or fused sweeps of one launch each).  None of these changes the
// results.  The tuner times short trial runs from the context's current state
// and descends one coordinate at a time: FE shape per FOM subdomain, OpInf path
// per OpInf subdomain, launch mode, sweep fusion.
// The choice is cached per configuration (precision, batch, subdomain sizes,
// reduced sizes) for the lifetime of the process.
#include <hip/hip_runtime.h>

#include <chrono>
#include <map>
#include <mutex>
#include <string>

#include "runtime.hpp"

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(OSAM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace osam {

namespace {
std::mutex g_tune_mu;
std::map<std::string, osam_tuning> g_tune_cache;

std::string tune_key(const Ctx &c) {
  std::string k = std::to_string(c.prec) + "/" + std::to_string(c.batch);
  for (const auto &d : c.sds) {
    k += "|" + std::to_string(d->rom) + ":" + std::to_string(d->desc.nx) + "x" + std::to_string(d->desc.ny) + "x" +
         std::to_string(d->nzs);
    if (d->rom) k += ":" + std::to_string(d->r) + "," + std::to_string(d->rs) + "," + std::to_string(d->oh.quadratic);
  }
  return k;
}
}  // namespace

int32_t Ctx::apply_tuning(const osam_tuning &t) {
  for (size_t i = 0; i < sds.size(); ++i) {
    Subdomain &d = *sds[i];
    if (!d.rom) {
      d.fe_xs = t.fe_xs[i] != 0;
      if (!choose_fe_launch(d, t.fe_block[i], t.fe_kc[i])) return fail(OSAM_E_INVALID, "cached FE launch does not apply");
    } else if (d.rom_path != t.rom_path[i]) {
      d.rom_path = t.rom_path[i];
      int32_t st = setup_pre(d);
      if (st) return st;
    }
  }
  graph_rounds = t.graph_rounds;
  graph_streams = t.graph_streams;
  fuse = t.fusion_kc > 0;
  fuse_kc = fuse ? t.fusion_kc : 1;
  return OSAM_OK;
}

int32_t Ctx::autotune(int64_t n, const osam_schwarz_opts &op, osam_tuning *out) {
  if (n < 1) return fail(OSAM_E_INVALID, "trial steps must be >= 1");
  int32_t st = couple();
  if (st) return st;
  if ((st = wire())) return st;
  for (int b = 0; b < batch; ++b)
    if (!initialized[b]) return fail(OSAM_E_ORDER, "autotune needs every instance initialised");
  const bool was_timing = timing;
  timing = false;
  const std::string key = tune_key(*this);
  osam_tuning t{};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      t = it->second;
      t.from_cache = 1;
      st = apply_tuning(t);
      timing = was_timing;
      if (!st && out) *out = t;
      return st;
    }
  }
  // wall time per controller step of a trial (after a short warm-up): runs of n and
  // 2n steps, the difference per step, so that what every run pays once (graph
  // capture and instantiation, host set-up) cancels
  auto trial = [&](double *ms) -> int32_t {
    int32_t s = run(2, op, nullptr);
    if (s) return s;
    HIPCHK(hipStreamSynchronize(stream));
    double t[2];
    for (int k = 0; k < 2; ++k) {
      const auto t0 = std::chrono::steady_clock::now();
      if ((s = run(n * (k + 1), op, nullptr))) return s;
      HIPCHK(hipStreamSynchronize(stream));
      t[k] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    // noise can make the longer run look no longer: then the plain per-step time of it
    *ms = t[1] > t[0] ? (t[1] - t[0]) / (double)n : t[1] / (2.0 * (double)n);
    return OSAM_OK;
  };
  graph_rounds = 0;
  graph_streams = 1;
  fuse = false;
  double best = 0.0;
  if ((st = trial(&best))) return st;
  // 1. FE launch shape, one FOM subdomain at a time
  const int shapes[][2] = {{256, 1}, {128, 1}, {64, 1}, {64, 2}, {256, 8}, {64, 8}, {1024, 4}, {1024, 8}, {1024, 16}};
  for (size_t i = 0; i < sds.size(); ++i) {
    Subdomain &d = *sds[i];
    if (d.rom) continue;
    int bb = d.fe_block, bk = d.fe_kc;
    bool bx = d.fe_xs;
    for (const auto &sh : shapes)
      for (int xs = 0; xs < (sh[0] == 1024 ? 1 : 2); ++xs) {
        d.fe_xs = xs != 0;
        if (!choose_fe_launch(d, sh[0], sh[1])) continue;
        double ms;
        if ((st = trial(&ms))) return st;
        if (ms < best) {
          best = ms;
          bb = d.fe_block;
          bk = d.fe_kc;
          bx = d.fe_xs;
        }
      }
    d.fe_xs = bx;
    choose_fe_launch(d, bb, bk);
  }
  // 2. OpInf path (FP32 contexts: fused or batched)
  if (prec == OSAM_FP32) {
    for (size_t i = 0; i < sds.size(); ++i) {
      Subdomain &d = *sds[i];
      if (!d.rom) continue;
      int bestp = d.pre ? 2 : 1;   // the path in use at the baseline
      for (int p = 1; p <= 2; ++p) {
        d.rom_path = p;
        if ((st = setup_pre(d))) return st;
        double ms;
        if ((st = trial(&ms))) return st;
        if (ms < best) {
          best = ms;
          bestp = p;
        }
      }
      d.rom_path = bestp;
      if ((st = setup_pre(d))) return st;
    }
  }
  // 3. launch mode
  const int modes[][2] = {{32, 1}, {128, 1}, {32, 2}};
  int gr = 0, gs = 1;
  for (const auto &m : modes) {
    graph_rounds = m[0];
    graph_streams = m[1];
    double ms;
    if ((st = trial(&ms))) return st;
    if (ms < best) {
      best = ms;
      gr = m[0];
      gs = m[1];
    }
  }
  graph_rounds = gr;
  graph_streams = gs;
  // 4. fused sweeps (layers per thread of the FE part) with host launches or graphs
  int fkc = 0;
  if (fusion_unsupported().empty()) {
    const int fmodes[][2] = {{1, 0}, {1, 32}, {1, 128}, {2, 32}, {4, 32}};
    for (const auto &m : fmodes) {
      fuse = true;
      fuse_kc = m[0];
      graph_rounds = m[1];
      graph_streams = 1;
      double ms;
      if ((st = trial(&ms))) return st;
      if (ms < best) {
        best = ms;
        fkc = m[0];
        gr = m[1];
        gs = 1;
      }
    }
  }
  fuse = fkc > 0;
  fuse_kc = fuse ? fkc : 1;
  graph_rounds = gr;
  graph_streams = gs;
  for (size_t i = 0; i < sds.size() && i < 8; ++i) {
    t.fe_block[i] = sds[i]->rom ? 0 : sds[i]->fe_block;
    t.fe_kc[i] = sds[i]->rom ? 0 : sds[i]->fe_kc;
    t.fe_xs[i] = sds[i]->rom ? 0 : (sds[i]->fe_xs ? 1 : 0);
    t.rom_path[i] = sds[i]->rom ? (sds[i]->pre ? 2 : 1) : 0;
  }
  t.graph_rounds = gr;
  t.graph_streams = gs;
  t.fusion_kc = fkc;
  t.ms_per_step = best;
  t.from_cache = 0;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = t;
  }
  timing = was_timing;
  if (out) *out = t;
  return OSAM_OK;
}

}  // namespace osam

using namespace osam;

int32_t osam_autotune(osam_ctx *c, int64_t trial_steps, const osam_schwarz_opts *opts, osam_tuning *out) {
  if (!c || !opts) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  return ctx->autotune(trial_steps, *opts, out);
}
