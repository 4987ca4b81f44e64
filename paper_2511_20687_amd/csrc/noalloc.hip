// run_noalloc: the controller loop of run without any device allocation, for
// callers that cannot allocate (work under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  The per-workgroup partial sums of Eq.
// conv_criterion (FOM step kernels, and the per-subdomain sums of the window
// engine) live in a file-scope device array instead of the context's buffers;
// everything else the loop touches was allocated when the context was wired.
#include <mutex>

#include "runtime.hpp"

namespace osam {

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;   // 32 MiB per device
constexpr int kMaxDevices = 64;

// Each GPU the library runs on holds its own copy until the process ends.  In
// host code this name is only a stand-in: kernels receive the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

}  // namespace

// Device address of `scratch` on `device`, which must be the current device;
// looked up once per device (osam_ctx_create calls this with the context's device).
int32_t static_scratch_address(int device, void **out) {
  if (device < 0 || device >= kMaxDevices || !out) return OSAM_E_INVALID;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[device]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return OSAM_E_HIP;
    g_addr[device] = p;
  }
  *out = g_addr[device];
  return OSAM_OK;
}

}  // namespace osam

using namespace osam;

extern "C" int32_t run_noalloc(osam_ctx *c, int64_t n_steps, const osam_schwarz_opts *opts,
                               osam_instance_info *info) {
  if (!c || !opts || n_steps < 0) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  if (!ctx->static_scratch) return ctx->fail(OSAM_E_HIP, "no device address for the static scratch array");
  if (!ctx->coupled || !ctx->wired)
    return ctx->fail(OSAM_E_ORDER, "run_noalloc needs a wired context (set the initial conditions first)");
  for (int b = 0; b < ctx->batch; ++b)
    if (!ctx->initialized[b]) return ctx->fail(OSAM_E_ORDER, "instance without initial condition");
  const bool win = ctx->window_mode();
  if (win && !ctx->win_ready)
    return ctx->fail(OSAM_E_ORDER, "run_noalloc: the window engine allocates its buffers in a first run call");
  // slices of the scratch array, 256-byte aligned
  auto round = [](size_t n) { return (n + 255) / 256 * 256; };
  std::vector<size_t> off(ctx->sds.size(), 0);
  size_t need = 0;
  for (size_t i = 0; i < ctx->sds.size(); ++i) {
    const Subdomain &d = *ctx->sds[i];
    if (d.rom || win) continue;
    off[i] = need;
    need += round(sizeof(double) * 4 * (size_t)ctx->batch * d.max_nblocks);   // two sweep parities
  }
  const size_t win_off = need;
  if (win) need += round(sizeof(double) * 2 * (size_t)ctx->batch * ctx->sds.size());
  if (need > kScratchBytes)
    return ctx->fail(OSAM_E_INVALID, "run_noalloc needs " + std::to_string(need) +
                                         " bytes of partial sums, more than its 32 MiB maximum");
  char *base = static_cast<char *>(ctx->static_scratch);
  std::vector<double *> saved(ctx->sds.size());
  for (size_t i = 0; i < ctx->sds.size(); ++i) {
    Subdomain &d = *ctx->sds[i];
    saved[i] = d.partials;
    if (!d.rom && !win) d.partials = reinterpret_cast<double *>(base + off[i]);
  }
  double *saved_sums = ctx->win_sums;
  if (win) ctx->win_sums = reinterpret_cast<double *>(base + win_off);
  // no graph instantiation and no timing events (both allocate)
  const int saved_rounds = ctx->graph_rounds;
  const bool saved_timing = ctx->timing;
  ctx->graph_rounds = 0;
  ctx->timing = false;
  hipSetDevice(ctx->device);
  const int32_t st = ctx->run(n_steps, *opts, info);
  ctx->graph_rounds = saved_rounds;
  ctx->timing = saved_timing;
  ctx->win_sums = saved_sums;
  for (size_t i = 0; i < ctx->sds.size(); ++i) ctx->sds[i]->partials = saved[i];
  return st;
}
