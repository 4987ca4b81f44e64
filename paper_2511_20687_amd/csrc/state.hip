// Setting the accepted state of a subdomain (osam_set_state) and raw per-instance
// checkpoints (osam_checkpoint_size / osam_save_checkpoint / osam_load_checkpoint).
#include <cmath>
#include <cstring>

#include "runtime.hpp"

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) return ctx->fail(OSAM_E_HIP, hipGetErrorString(e_));         \
  } while (0)

namespace osam {

namespace {

// Every per-instance device range that carries state from one controller step to the
// next: the accepted state in all its roles, the values pushed for the next step, the
// predictor of OpInf subdomains.  (ptr, bytes) per range; the instance's offset added.
std::vector<std::pair<char *, size_t>> instance_ranges(Ctx *ctx, int inst) {
  std::vector<std::pair<char *, size_t>> out;
  const size_t es = ctx->esize();
  for (auto &sp : ctx->sds) {
    Subdomain &d = *sp;
    if (!d.rom) {
      const size_t n = (size_t)d.is * es, off = (size_t)inst * n;
      for (int k = 0; k < 3; ++k) out.push_back({(char *)d.u[k] + off, n});
      for (int k = 0; k < 2; ++k) {
        out.push_back({(char *)d.v[k] + off, n});
        out.push_back({(char *)d.a[k] + off, n});
      }
    } else {
      const size_t n = (size_t)d.r * es, off = (size_t)inst * n;
      for (int k = 0; k < 2; ++k) {
        out.push_back({(char *)d.q[k] + off, n});
        out.push_back({(char *)d.qd[k] + off, n});
        out.push_back({(char *)d.qdd[k] + off, n});
      }
      out.push_back({(char *)d.qpred + off, n});
      for (int f = 0; f < 2; ++f)
        for (int k = 0; k < 3; ++k)
          if (d.sface[f][k]) {
            const size_t m = (size_t)3 * d.npl * es;
            out.push_back({(char *)d.sface[f][k] + (size_t)inst * m, m});
          }
    }
  }
  return out;
}

int32_t ready(Ctx *ctx, int inst) {
  if (inst < 0 || inst >= ctx->batch) return ctx->fail(OSAM_E_INVALID, "bad instance");
  if (!ctx->wired || !ctx->initialized[inst])
    return ctx->fail(OSAM_E_ORDER, "the instance needs its initial condition first (osam_set_initial)");
  return OSAM_OK;
}

}  // namespace

}  // namespace osam

using namespace osam;

extern "C" int32_t osam_set_state(osam_ctx *c, int32_t sdi, int32_t inst, const double *x, const double *xd,
                                  const double *xdd) {
  if (!c || !x || !xd || !xdd) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  if (sdi < 0 || sdi >= (int)ctx->sds.size()) return ctx->fail(OSAM_E_INVALID, "bad subdomain id");
  int32_t st = ready(ctx, inst);
  if (st) return st;
  hipSetDevice(ctx->device);
  if ((st = ctx->sync_status())) return st;
  Subdomain &d = *ctx->sds[sdi];
  const long long s = ctx->h_status[inst].step;
  const bool window = ctx->window_mode();
  if (!d.rom) {
    // [3][n_nodes] fields into the roles of the current step
    const size_t off = (size_t)inst * d.is * ctx->esize();
    std::vector<double> buf((size_t)3 * d.cs, 0.0);
    const double *src[3] = {x, xd, xdd};
    void *dst[3] = {(char *)d.u[s % 3] + off, (char *)d.v[s % 2] + off, (char *)d.a[s % 2] + off};
    for (int k = 0; k < 3; ++k) {
      for (int cc = 0; cc < 3; ++cc)
        std::memcpy(buf.data() + (size_t)cc * d.cs, src[k] + (size_t)cc * d.nnodes, sizeof(double) * d.nnodes);
      if ((st = ctx->upload(dst[k], buf.data(), buf.size()))) return st;
    }
    // OpInf destinations fed by this subdomain: its accepted values on their faces (the
    // HOLD data of the next step)
    const int me = sdi;
    for (auto &sp : ctx->sds) {
      Subdomain &o = *sp;
      if (!o.rom) continue;
      for (int f = 0; f < 2; ++f) {
        if (o.face_type[f] == kFaceClamped || o.proj[f].src != me || !o.sface[f][s % 3]) continue;
        const int L = o.proj[f].src_layer;
        std::vector<double> fv((size_t)3 * o.npl);
        for (int cc = 0; cc < 3; ++cc)
          for (int nid = 0; nid < o.npl; ++nid)
            fv[(size_t)cc * o.npl + nid] = x[(size_t)cc * d.nnodes + (size_t)L * d.npl + nid];
        if ((st = ctx->upload((char *)o.sface[f][s % 3] + (size_t)inst * 3 * o.npl * ctx->esize(), fv.data(),
                              fv.size())))
          return st;
      }
    }
  } else {
    const int r = d.r, par = (int)(s % 2);
    const size_t off = (size_t)inst * r * ctx->esize();
    if ((st = ctx->upload((char *)d.q[par] + off, x, r))) return st;
    if ((st = ctx->upload((char *)d.qd[par] + off, xd, r))) return st;
    if ((st = ctx->upload((char *)d.qdd[par] + off, xdd, r))) return st;
    // the next step's q(t_k) as the step kernel forms it: fma(h, q'', fma(dt, q', q)) in the
    // context precision
    const double dt = d.desc.dt, h = 0.5 * dt * dt;
    std::vector<double> qp(r), q1(r);
    for (int k = 0; k < r; ++k) {
      if (ctx->prec == OSAM_FP64) qp[k] = std::fma(h, xdd[k], std::fma(dt, xd[k], x[k]));
      else qp[k] = (double)std::fma((float)h, (float)xdd[k], std::fma((float)dt, (float)xd[k], (float)x[k]));
      q1[k] = x[k] + dt * xd[k] + h * xdd[k];
    }
    if ((st = ctx->upload((char *)d.qpred + off, qp.data(), r))) return st;
    // FOM destinations: (Pi Phi) q(t_k+1) on their faces, in the role of the next step
    int e = 0;
    for (auto &sp : ctx->sds) {
      Subdomain &fd = *sp;
      if (fd.rom) continue;
      for (int f = 0; f < 2; ++f) {
        if (fd.face_type[f] == kFaceClamped || fd.proj[f].src != sdi) continue;
        if (e >= (int)d.piphi_h.size()) return ctx->fail(OSAM_E_ORDER, "transfer rows not wired");
        const std::vector<double> &pp = d.piphi_h[e++];
        const int n = 3 * fd.npl;
        std::vector<double> sv(n, 0.0);
        for (int k = 0; k < r; ++k)
          for (int m = 0; m < n; ++m) sv[m] += pp[(size_t)k * n + m] * q1[k];
        const size_t lay = (size_t)(f == 0 ? 0 : fd.nzs) * fd.npl;
        for (int cc = 0; cc < 3; ++cc) {
          const size_t o = ((size_t)inst * fd.is + (size_t)cc * fd.cs + lay) * ctx->esize();
          if ((st = ctx->upload((char *)fd.u[(s + 1) % 3] + o, sv.data() + (size_t)cc * fd.npl, fd.npl))) return st;
        }
      }
    }
  }
  // the single-step engine recomputes what it derives from the accepted state of FOM
  // subdomains (a = M^-1(-K u), the next predictor, the pushed faces) before the next step;
  // the window engine steps from the accepted state as given (an implicit step's
  // acceleration equals M^-1(-K u) only to the tolerance of its solve)
  if (window) ctx->h_status[inst].flags &= ~kNeedInit;
  else ctx->h_status[inst].flags |= kNeedInit;
  HIPCHK(hipMemcpyAsync(ctx->d_status + inst, ctx->h_status + inst, sizeof(Status), hipMemcpyHostToDevice,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return OSAM_OK;
}

extern "C" int32_t osam_checkpoint_size(osam_ctx *c, int64_t *bytes) {
  if (!c || !bytes) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  if (!ctx->wired) return ctx->fail(OSAM_E_ORDER, "the context is not wired yet (osam_set_initial)");
  size_t n = sizeof(Status);
  for (auto &r : instance_ranges(ctx, 0)) n += r.second;
  *bytes = (int64_t)n;
  return OSAM_OK;
}

extern "C" int32_t osam_save_checkpoint(osam_ctx *c, int32_t inst, void *host) {
  if (!c || !host) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  int32_t st = ready(ctx, inst);
  if (st) return st;
  hipSetDevice(ctx->device);
  if ((st = ctx->sync_status())) return st;
  char *p = static_cast<char *>(host);
  std::memcpy(p, ctx->h_status + inst, sizeof(Status));
  p += sizeof(Status);
  for (auto &r : instance_ranges(ctx, inst)) {
    HIPCHK(hipMemcpyAsync(p, r.first, r.second, hipMemcpyDeviceToHost, ctx->stream));
    p += r.second;
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return OSAM_OK;
}

extern "C" int32_t osam_load_checkpoint(osam_ctx *c, int32_t inst, const void *host) {
  if (!c || !host) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  int32_t st = ready(ctx, inst);
  if (st) return st;
  hipSetDevice(ctx->device);
  if ((st = ctx->sync_status())) return st;
  const char *p = static_cast<const char *>(host);
  Status s;
  std::memcpy(&s, p, sizeof(Status));
  p += sizeof(Status);
  for (auto &r : instance_ranges(ctx, inst)) {
    HIPCHK(hipMemcpyAsync(r.first, p, r.second, hipMemcpyHostToDevice, ctx->stream));
    p += r.second;
  }
  s.flags &= ~(kFinished | kNeedInit);
  ctx->h_status[inst] = s;
  HIPCHK(hipMemcpyAsync(ctx->d_status + inst, ctx->h_status + inst, sizeof(Status), hipMemcpyHostToDevice,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return OSAM_OK;
}
