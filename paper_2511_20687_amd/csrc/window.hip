// Host side of the window engine (window.hpp, window_kernels.hip): the Schwarz
// controller of Alg. 1 for subdomains that take several Newmark steps per
// controller step (Sec. 4.1: dt_i = dt / n_sub_i, Schwarz data through the
// temporal interpolant Xi) or the implicit Newmark scheme (beta > 0), and for any
// context on request (osam_set_engine).  Instances advance one controller step
// at a time: every Schwarz iteration launches each subdomain's sub-steps in the
// multiplicative (or additive) order, then the decision of Eq. conv_criterion;
// after min_iter iterations the host reads the per-instance status back to stop
// iterating once every instance has converged.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "runtime.hpp"
#include "window.hpp"

#define HIPCHK(x)                                                              \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) return fail(OSAM_E_HIP, hipGetErrorString(e_));      \
  } while (0)

namespace osam {

bool Ctx::window_mode() const {
  if (engine == 1) return true;
  for (const auto &s : sds)
    if (s->desc.beta != 0.0 || s->desc.gamma != 0.5 || s->n_sub > 1 || !s->oh.C3.empty() ||
        (!s->rom && s->desc.material != OSAM_LINEAR_ELASTIC))
      return true;
  return false;
}

// (I - c A)^-1 by Gauss-Jordan elimination with partial pivoting (A column-major,
// result row-major); false if singular.
static bool invert_shifted(const std::vector<double> &A, int r, double c, std::vector<double> &out) {
  std::vector<double> M((size_t)r * 2 * r, 0.0);
  for (int i = 0; i < r; ++i) {
    for (int j = 0; j < r; ++j) M[(size_t)i * 2 * r + j] = (i == j ? 1.0 : 0.0) - c * A[(size_t)j * r + i];
    M[(size_t)i * 2 * r + r + i] = 1.0;
  }
  for (int k = 0; k < r; ++k) {
    int p = k;
    for (int i = k + 1; i < r; ++i)
      if (std::fabs(M[(size_t)i * 2 * r + k]) > std::fabs(M[(size_t)p * 2 * r + k])) p = i;
    if (M[(size_t)p * 2 * r + k] == 0.0) return false;
    if (p != k)
      for (int j = 0; j < 2 * r; ++j) std::swap(M[(size_t)p * 2 * r + j], M[(size_t)k * 2 * r + j]);
    const double d = M[(size_t)k * 2 * r + k];
    for (int j = 0; j < 2 * r; ++j) M[(size_t)k * 2 * r + j] /= d;
    for (int i = 0; i < r; ++i) {
      if (i == k) continue;
      const double f = M[(size_t)i * 2 * r + k];
      if (f == 0.0) continue;
      for (int j = 0; j < 2 * r; ++j) M[(size_t)i * 2 * r + j] -= f * M[(size_t)k * 2 * r + j];
    }
  }
  out.assign((size_t)r * r, 0.0);
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) out[(size_t)i * r + j] = M[(size_t)i * 2 * r + r + j];
  return true;
}

int32_t Ctx::window_setup() {
  if (win_ready) return OSAM_OK;
  int32_t st = OSAM_OK;
  HIPCHK(hipStreamSynchronize(stream));
  for (void *p : win_allocs) dfree(p);
  win_allocs.clear();
  auto get = [&](size_t n, bool zero) -> void * {
    void *p = alloc_t(n, &st);
    if (!st) {
      win_allocs.push_back(p);
      if (zero) (void)hipMemsetAsync(p, 0, n * esize(), stream);
    }
    return p;
  };
  const int S = (int)sds.size();
  for (int i = 0; i < S; ++i) {
    Subdomain &d = *sds[i];
    WinBufs &w = d.win;
    w = WinBufs{};
    const size_t nb = (size_t)batch * (d.rom ? d.r : d.is);
    for (int k = 0; k < 2; ++k) {
      if (!d.rom) {
        w.wu[k] = get(nb, true);
        w.wv[k] = get(nb, true);
        w.wa[k] = get(nb, true);
        if (d.n_sub > 1) {
          w.tu[k] = get(nb, true);
          w.tv[k] = get(nb, true);
          w.ta[k] = get(nb, true);
        }
      } else {
        w.wq[k] = get(nb, true);
        w.wqd[k] = get(nb, true);
        w.wqdd[k] = get(nb, true);
        if (d.n_sub > 1) {
          w.tq[k] = get(nb, true);
          w.tqd[k] = get(nb, true);
          w.tqdd[k] = get(nb, true);
        }
      }
    }
    const bool implicit = d.desc.beta != 0.0;
    if (!d.rom && implicit) {
      // the faces of the CG vectors stay zero (the operator acts on free DOFs)
      w.cr = get(nb, true);
      w.cp = get(nb, true);
      w.cq = get(nb, true);
    }
    if (d.rom) {
      if (d.r > 4 * kWinRomThreads) return fail(OSAM_E_INVALID, "window engine: r above 1024");
      w.sbuf = get((size_t)batch * 2 * 3 * d.npl, true);
      const long long r2 = d.oh.quadratic ? (long long)d.r * (d.r + 1) / 2 : 0;
      const long long r3 = d.oh.C3.empty() ? 0 : (long long)d.r * (d.r + 1) * (d.r + 2) / 6;
      w.kbuf = get((size_t)batch * (r2 + r3 + 1), false);
      if (r3) {
        std::vector<double> Cr((size_t)d.r * r3);
        for (int a = 0; a < d.r; ++a)
          for (long long m = 0; m < r3; ++m) Cr[(size_t)a * r3 + m] = d.oh.C3[(size_t)m * d.r + a];
        w.C3 = get(Cr.size(), false);
        if (st) return fail(st, "out of device memory (window engine)");
        if ((st = upload(w.C3, Cr.data(), Cr.size()))) return st;
      }
      if (implicit) {
        const double h = d.desc.dt / d.n_sub;
        std::vector<double> Mi;
        if (!invert_shifted(d.oh.A, d.r, d.desc.beta * h * h, Mi))
          return fail(OSAM_E_SINGULAR, "I - beta dt^2 A is singular");
        w.Minv = get(Mi.size(), false);
        if (st) return fail(st, "out of device memory (window engine)");
        if ((st = upload(w.Minv, Mi.data(), Mi.size()))) return st;
      }
    }
    for (int f = 0; f < 2; ++f) {
      if (d.face_type[f] == kFaceClamped) continue;
      const Subdomain &src = *sds[d.proj[f].src];
      for (int p = 0; p < 2; ++p) w.traj[f][p] = get((size_t)src.n_sub * batch * 3 * d.npl, true);
    }
    w.iters = (int *)get((size_t)batch * (prec == OSAM_FP64 ? 1 : 2), true);
    if (st) return fail(st, "out of device memory (window engine)");
  }
  // rows of Pi Phi for every face an OpInf subdomain feeds
  for (int i = 0; i < S; ++i) {
    Subdomain &d = *sds[i];
    for (int f = 0; f < 2; ++f) {
      if (d.face_type[f] == kFaceClamped) continue;
      Subdomain &src = *sds[d.proj[f].src];
      if (!src.rom) continue;
      std::vector<double> rows;
      if ((st = phi_layer_rows(src, d.proj[f].src_layer, rows))) return st;
      void *p = get(rows.size(), false);
      if (st) return fail(st, "out of device memory (window engine)");
      if ((st = upload(p, rows.data(), rows.size()))) return st;
      src.win.exp_rows.push_back({2 * i + f, p});
    }
  }
  win_sums = (double *)get((size_t)batch * S * 2 * (prec == OSAM_FP64 ? 1 : 2), true);
  if (st) return fail(st, "out of device memory (window engine)");
  HIPCHK(hipStreamSynchronize(stream));
  win_ready = true;
  return OSAM_OK;
}

template <typename T>
static void fill_src(Ctx &c, Subdomain &d, int f, WinSrc<T> &S) {
  std::memset(&S, 0, sizeof(S));
  if (d.face_type[f] == kFaceClamped) return;
  const int j = d.proj[f].src;
  Subdomain &s = *c.sds[j];
  S.kind = s.rom ? 2 : 1;
  S.sd = j;
  S.n_sub = s.n_sub;
  S.layer = d.proj[f].src_layer;
  S.npl = d.npl;
  S.batch = c.batch;
  if (!s.rom) {
    S.cs = s.cs;
    S.is = s.is;
    for (int k = 0; k < 3; ++k) S.u[k] = (const T *)s.u[k];
    for (int k = 0; k < 2; ++k) {
      S.v[k] = (const T *)s.v[k];
      S.a[k] = (const T *)s.a[k];
    }
  } else {
    S.r = s.r;
    for (int k = 0; k < 2; ++k) {
      S.q[k] = (const T *)s.q[k];
      S.qd[k] = (const T *)s.qd[k];
      S.qdd[k] = (const T *)s.qdd[k];
    }
    for (auto &e : s.win.exp_rows) {
      const Subdomain &dd = *c.sds[e.first / 2];
      if (&dd == &d && e.first % 2 == f) S.rows = (const T *)e.second;
    }
  }
  for (int p = 0; p < 2; ++p) S.traj[p] = (const T *)d.win.traj[f][p];
}

// The faces subdomain i feeds: trajectory buffers of the destinations and the
// source-local layer (FOM) or the Pi Phi rows (OpInf) of each.
template <typename T>
static int fill_exports(Ctx &c, int i, T *(&traj)[kWinMaxExp][2], int *layer, const T **rows) {
  int n = 0;
  Subdomain &s = *c.sds[i];
  for (size_t k = 0; k < c.sds.size(); ++k) {
    Subdomain &d = *c.sds[k];
    for (int f = 0; f < 2; ++f) {
      if (d.face_type[f] == kFaceClamped || d.proj[f].src != i) continue;
      if (n >= kWinMaxExp) return -1;
      traj[n][0] = (T *)d.win.traj[f][0];
      traj[n][1] = (T *)d.win.traj[f][1];
      if (layer) layer[n] = d.proj[f].src_layer;
      if (rows) {
        rows[n] = nullptr;
        for (auto &e : s.win.exp_rows)
          if (e.first == (int)(2 * k + f)) rows[n] = (const T *)e.second;
      }
      ++n;
    }
  }
  return n;
}

template <typename T>
static int32_t launch_window_sd(Ctx &c, int i, int l, const Opts &o, bool svk_init = false) {
  Subdomain &d = *c.sds[i];
  const WinBufs &w = d.win;
  const bool implicit = d.desc.beta != 0.0;
  const T h = (T)(d.desc.dt / d.n_sub);
  hipError_t e;
  if (!d.rom) {
    WinFomArgs<T> A;
    std::memset(&A, 0, sizeof(A));
    A.material = d.desc.material;
    const osam_subdomain_desc &g = d.desc;
    A.lam = (T)(g.E * g.nu / ((1 + g.nu) * (1 - 2 * g.nu)));
    A.mu = (T)(g.E / (2 * (1 + g.nu)));
    A.hx = (T)(g.Lx / g.nx);
    A.hy = (T)(g.Ly / g.ny);
    A.hz = (T)(g.Lz / g.nz);
    A.rho = (T)g.rho;
    A.lateral_fix = g.lateral_fix;
    A.nfree_nodes = d.nfree_nodes;
    A.rec_ncols = d.rec.n_cols;
    A.rec_a0 = d.rec.every > 0 && d.rec.n_cols > 0 ? (T *)d.rec.a : nullptr;
    A.nx = d.nx;
    A.ny = d.ny;
    A.nzs = d.nzs;
    A.npl = d.npl;
    A.cs = d.cs;
    A.is = d.is;
    A.nnodes = d.nnodes;
    for (int k = 0; k < 3; ++k) A.u[k] = (T *)d.u[k];
    for (int k = 0; k < 2; ++k) {
      A.v[k] = (T *)d.v[k];
      A.a[k] = (T *)d.a[k];
      A.wu[k] = (T *)w.wu[k];
      A.wv[k] = (T *)w.wv[k];
      A.wa[k] = (T *)w.wa[k];
      A.tu[k] = (T *)w.tu[k];
      A.tv[k] = (T *)w.tv[k];
      A.ta[k] = (T *)w.ta[k];
    }
    A.cr = (T *)w.cr;
    A.cp = (T *)w.cp;
    A.cq = (T *)w.cq;
    A.coef = (const T *)d.coef;
    for (int k = 0; k < 27; ++k) A.cb[k] = (T)d.cb[k];
    A.dt = h;
    A.beta = (T)d.desc.beta;
    A.gamma = (T)d.desc.gamma;
    A.n_sub = d.n_sub;
    A.l = l;
    A.implicit = implicit;
    const double tol = c.prec == OSAM_FP64 ? 1e-14 : 1e-6;
    A.cg_tol2 = tol * tol;
    A.cg_max = 1000;
    A.additive = o.additive;
    A.guess = o.guess;
    for (int f = 0; f < 2; ++f) fill_src<T>(c, d, f, A.src[f]);
    A.nexp = fill_exports<T>(c, i, A.exp_traj, A.exp_layer, nullptr);
    if (A.nexp < 0) return c.fail(OSAM_E_INVALID, "window engine: a subdomain feeds more than 4 faces");
    A.status = c.d_status;
    A.sd = i;
    A.nsd = (int)c.sds.size();
    A.sums = c.win_sums;
    A.cg_iters = w.iters;
    e = svk_init ? launch_win_svk_init<T>(A, c.batch, c.stream) : launch_win_fom<T>(A, c.batch, c.stream);
  } else {
    WinRomArgs<T> A;
    std::memset(&A, 0, sizeof(A));
    A.r = d.r;
    A.rs = d.rs;
    A.r2 = d.oh.quadratic ? d.r * (d.r + 1) / 2 : 0;
    A.r3 = d.oh.C3.empty() ? 0 : d.r * (d.r + 1) * (d.r + 2) / 6;
    A.A = (const T *)d.d_A;
    A.H = (const T *)d.d_H;
    A.C3 = (const T *)w.C3;
    A.B = (const T *)d.d_B;
    A.c = (const T *)d.d_c;
    A.Minv = (const T *)w.Minv;
    for (int k = 0; k < 2; ++k) {
      A.q[k] = (T *)d.q[k];
      A.qd[k] = (T *)d.qd[k];
      A.qdd[k] = (T *)d.qdd[k];
      A.wq[k] = (T *)w.wq[k];
      A.wqd[k] = (T *)w.wqd[k];
      A.wqdd[k] = (T *)w.wqdd[k];
      A.tq[k] = (T *)w.tq[k];
      A.tqd[k] = (T *)w.tqd[k];
      A.tqdd[k] = (T *)w.tqdd[k];
    }
    A.sbuf = (T *)w.sbuf;
    A.kbuf = (T *)w.kbuf;
    A.npl = d.npl;
    for (int f = 0; f < 2; ++f) {
      A.phis[f] = d.face_type[f] == kFaceClamped ? nullptr : (const T *)d.face_phis[f];
      fill_src<T>(c, d, f, A.src[f]);
    }
    A.dt = h;
    A.beta = (T)d.desc.beta;
    A.gamma = (T)d.desc.gamma;
    A.n_sub = d.n_sub;
    A.l = l;
    A.implicit = implicit;
    A.newton_max = 50;
    const double tol = c.prec == OSAM_FP64 ? 1e-14 : 1e-6;
    A.newton_tol2 = tol * tol;
    A.additive = o.additive;
    A.guess = o.guess;
    A.nexp = fill_exports<T>(c, i, A.exp_traj, nullptr, A.exp_rows);
    if (A.nexp < 0) return c.fail(OSAM_E_INVALID, "window engine: a subdomain feeds more than 4 faces");
    A.status = c.d_status;
    A.sd = i;
    A.nsd = (int)c.sds.size();
    A.sums = c.win_sums;
    A.newton_iters = w.iters;
    e = launch_win_rom<T>(A, c.batch, c.stream);
  }
  if (e != hipSuccess) return c.fail(OSAM_E_HIP, hipGetErrorString(e));
  return OSAM_OK;
}

template <typename T>
static int32_t launch_window_accept(Ctx &c, int i) {
  Subdomain &d = *c.sds[i];
  WinAcceptArgs<T> A;
  std::memset(&A, 0, sizeof(A));
  A.rom = d.rom;
  A.cs = d.cs;
  A.is = d.is;
  A.nnodes = d.nnodes;
  A.npl = d.npl;
  A.nzs = d.nzs;
  A.nfree_nodes = d.nfree_nodes;
  A.nsch_nodes = d.nsch_nodes;
  A.face_off_hi = d.face_off_hi;
  for (int f = 0; f < 2; ++f) A.face_sch[f] = d.face_type[f] != kFaceClamped;
  for (int k = 0; k < 3; ++k) A.u[k] = (T *)d.u[k];
  for (int k = 0; k < 2; ++k) {
    A.v[k] = (T *)d.v[k];
    A.a[k] = (T *)d.a[k];
    A.wu[k] = (const T *)d.win.wu[k];
    A.wv[k] = (const T *)d.win.wv[k];
    A.wa[k] = (const T *)d.win.wa[k];
    A.q[k] = (T *)d.q[k];
    A.qd[k] = (T *)d.qd[k];
    A.qdd[k] = (T *)d.qdd[k];
    A.wq[k] = (const T *)d.win.wq[k];
    A.wqd[k] = (const T *)d.win.wqd[k];
    A.wqdd[k] = (const T *)d.win.wqdd[k];
  }
  A.r = d.r;
  A.rec_u = (T *)d.rec.u;
  A.rec_a = d.rom ? nullptr : (T *)d.rec.a;
  A.rec_s = d.rom ? nullptr : (T *)d.rec.s;
  A.rec_every = d.rec.every;
  A.rec_ncols = d.rec.n_cols;
  A.status = c.d_status;
  const hipError_t e = launch_win_accept<T>(A, c.batch, c.stream);
  if (e != hipSuccess) return c.fail(OSAM_E_HIP, hipGetErrorString(e));
  return OSAM_OK;
}

int32_t Ctx::run_window(int64_t n_steps, const Opts &o, osam_instance_info *info) {
  int32_t st = window_setup();
  if (st) return st;
  const bool f64 = prec == OSAM_FP64;
  // Saint Venant-Kirchhoff subdomains: the set-up's a0 used the linear stiffness
  for (size_t i = 0; i < sds.size(); ++i)
    if (!sds[i]->rom && sds[i]->desc.material == OSAM_SVK) {
      st = f64 ? launch_window_sd<double>(*this, (int)i, 1, o, true) : launch_window_sd<float>(*this, (int)i, 1, o, true);
      if (st) return st;
    }
  for (int64_t k = 0; k < n_steps; ++k) {
    bool any = false;
    for (int b = 0; b < batch; ++b) {
      Status &S = h_status[b];
      S.pad0 = 0;
      if (S.flags & kNonfinite) continue;
      S.target = S.step + 1;
      S.flags &= ~kFinished;
      S.iter = 0;
      S.pad0 = 1;   // takes part in this controller step (read by the acceptance)
      any = true;
    }
    HIPCHK(hipMemcpyAsync(d_status, h_status, sizeof(Status) * batch, hipMemcpyHostToDevice, stream));
    if (!any) break;
    for (int n = 1; n <= o.max_iter; ++n) {
      for (size_t i = 0; i < sds.size(); ++i)
        for (int l = 1; l <= sds[i]->n_sub; ++l) {
          st = f64 ? launch_window_sd<double>(*this, (int)i, l, o) : launch_window_sd<float>(*this, (int)i, l, o);
          if (st) return st;
        }
      const hipError_t e = launch_win_decide(d_status, win_sums, o, batch, stream);
      if (e != hipSuccess) return fail(OSAM_E_HIP, hipGetErrorString(e));
      // read the status back only from the iteration count the previous step needed on
      // (iterations of instances that have converged are no-ops)
      if (n >= std::max(o.min_iter, win_iters_hint) || n == o.max_iter) {
        if ((st = sync_status())) return st;
        bool done = true;
        for (int b = 0; b < batch; ++b)
          if ((h_status[b].pad0 & 1) && !(h_status[b].flags & kFinished)) done = false;
        if (done) break;
      }
    }
    win_iters_hint = 0;
    for (int b = 0; b < batch; ++b)
      if (h_status[b].pad0 & 1) win_iters_hint = std::max(win_iters_hint, h_status[b].last_iters);
    for (size_t i = 0; i < sds.size(); ++i) {
      st = f64 ? launch_window_accept<double>(*this, (int)i) : launch_window_accept<float>(*this, (int)i);
      if (st) return st;
    }
  }
  if ((st = sync_status())) return st;
  bool nonfinite = false;
  for (int b = 0; b < batch; ++b) {
    Status &S = h_status[b];
    nonfinite |= (S.flags & kNonfinite) != 0;
    if (info) {
      osam_instance_info &I = info[b];
      I.steps = S.step;
      I.last_iters = S.last_iters;
      I.last_converged = S.last_conv;
      I.abs2 = S.abs2;
      I.den2 = S.den2;
      I.total_iters = S.total_iters;
      I.max_iters = S.max_iters;
      I.unconverged = S.unconverged;
      I.status = (S.flags & kNonfinite) ? OSAM_E_NONFINITE : OSAM_OK;
    }
  }
  if (nonfinite) return fail(OSAM_E_NONFINITE, "non-finite state or norm");
  return OSAM_OK;
}

}  // namespace osam

using namespace osam;

extern "C" int32_t osam_set_engine(osam_ctx *c, int32_t engine) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  if (engine < 0 || engine > 2) return ctx->fail(OSAM_E_INVALID, "engine must be 0, 1 or 2");
  ctx->engine = engine;
  return OSAM_OK;
}

extern "C" int32_t osam_get_solver_stats(osam_ctx *c, int32_t sd, int32_t *iters) {
  if (!c || !iters) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  if (sd < 0 || sd >= (int)ctx->sds.size()) return ctx->fail(OSAM_E_INVALID, "bad subdomain id");
  const Subdomain &d = *ctx->sds[sd];
  if (!d.win.iters) {
    for (int b = 0; b < ctx->batch; ++b) iters[b] = 0;
    return OSAM_OK;
  }
  if (hipMemcpyAsync(iters, d.win.iters, sizeof(int) * ctx->batch, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess)
    return ctx->fail(OSAM_E_HIP, "reading solver statistics");
  return OSAM_OK;
}
