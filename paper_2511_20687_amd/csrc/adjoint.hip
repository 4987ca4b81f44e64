// Host driver of run_adjoint: the trajectory misfit of the coupled rollout and
// its gradient with respect to the OpInf operators and the initial state, by a
// checkpointed discrete adjoint of the converged explicit step map (see
// adjoint_kernels.hip).  Segments of K steps: a forward pass stores the state
// at every segment start; then, last segment first, the segment is recomputed
// with its displacements taped and swept backward.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "adjoint.hpp"
#include "runtime.hpp"

namespace osam {

template <typename T> hipError_t launch_stencil(const SlabGeo<T> &, const T *, T *, int, int, bool, hipStream_t);
template <typename T> hipError_t launch_fom_elem(const SlabGeo<T> &, int, T *, T *, T *, T *, T, T, hipStream_t);
template <typename T> int fom_misfit_blocks(const SlabGeo<T> &);
template <typename T>
hipError_t launch_fom_misfit(const SlabGeo<T> &, T *, const T *, const T *, double *, hipStream_t);
template <typename T>
hipError_t launch_layer_copy(T *, long long, long long, const T *, long long, long long, int, int, hipStream_t);
template <typename T>
hipError_t launch_lift_face(const T *, const T *, int, T *, long long, long long, int, hipStream_t);
template <typename T>
hipError_t launch_rows_dot(const T *, int, int, const T *, long long, long long, int, T *, hipStream_t);
template <typename T>
hipError_t launch_rows_tdot(const T *, int, int, const T *, T *, long long, long long, int, hipStream_t);
template <typename T> hipError_t launch_rom_fwd(const RomAdj<T> &, hipStream_t);
template <typename T> hipError_t launch_rom_adj(const RomAdj<T> &, hipStream_t);
template <typename T> hipError_t launch_rom_adj_pred(const RomAdj<T> &, hipStream_t);

namespace {

template <typename T>
struct AdjSd {
  bool rom = false;
  // FOM
  SlabGeo<T> G{};
  long long n3 = 0;            // 3 * cs
  T *u = nullptr;              // state displacement (points into tape or checkpoint)
  T *v = nullptr, *a = nullptr, *vn = nullptr, *an = nullptr;
  T *U = nullptr, *V = nullptr, *Aa = nullptr, *Aa2 = nullptr, *mu = nullptr, *out = nullptr;
  T *tape = nullptr;           // [K + 1][3 cs]
  T *ckpt = nullptr;           // [nseg][3][3 cs]  (u, v, a)
  double *part = nullptr;      // [K][misfit blocks]
  int nblk = 0;
  // OpInf
  int r = 0, rs = 0, r2 = 0;
  T *q = nullptr, *qd = nullptr, *qdd = nullptr;
  T *Q = nullptr, *Qd = nullptr, *Qdd = nullptr, *Qdd2 = nullptr;
  T *gh = nullptr, *gbar = nullptr, *gh0 = nullptr;
  T *tq = nullptr, *tg = nullptr;   // [K + 1][r], [K + 1][max(rs, 1)]
  T *rckpt = nullptr;               // [nseg][3][r]
  double *dA = nullptr, *dH = nullptr, *dB = nullptr, *dc = nullptr, *rpart = nullptr;
};

struct Bail {
  int32_t code = OSAM_OK;
  std::string msg;
  bool ok(hipError_t e, const char *what) {
    if (e == hipSuccess || code) return code == OSAM_OK;
    code = OSAM_E_HIP;
    msg = std::string(what) + ": " + hipGetErrorString(e);
    return false;
  }
};

}  // namespace

template <typename T>
static int32_t adjoint_impl(Ctx *ctx, int64_t n, int64_t K, const osam_misfit &M, double *J_out,
                            const osam_grads &Gr) {
  const int S = (int)ctx->sds.size();
  hipStream_t s = ctx->stream;
  const long long step0 = ctx->h_status[0].step;
  const int nseg = (int)((n + K - 1) / K);
  const long long n_obs = n / M.every;
  std::vector<AdjSd<T>> A(S);
  std::vector<void *> mine;
  int32_t st = OSAM_OK;
  auto al = [&](size_t count) -> T * {
    void *p = ctx->arena_alloc(count * sizeof(T), &st);
    if (p) {
      mine.push_back(p);
      hipMemsetAsync(p, 0, count * sizeof(T), s);
    }
    return static_cast<T *>(p);
  };
  auto ald = [&](size_t count) -> double * {
    void *p = ctx->arena_alloc(count * sizeof(double), &st);
    if (p) {
      mine.push_back(p);
      hipMemsetAsync(p, 0, count * sizeof(double), s);
    }
    return static_cast<double *>(p);
  };
  auto release = [&]() {
    hipStreamSynchronize(s);
    for (void *p : mine) ctx->dfree(p);
  };
  Bail B;
  const T dt = (T)ctx->sds[0]->desc.dt, g = (T)(0.5 * ctx->sds[0]->desc.dt),
          h = (T)(0.5 * ctx->sds[0]->desc.dt * ctx->sds[0]->desc.dt);

  // ---- set-up: geometry, buffers, start state of instance 0
  for (int i = 0; i < S; ++i) {
    Subdomain &d = *ctx->sds[i];
    AdjSd<T> &X = A[i];
    X.rom = d.rom;
    if (!d.rom) {
      const osam_subdomain_desc &D = d.desc;
      SlabGeo<T> &G = X.G;
      G.nx = D.nx;
      G.ny = D.ny;
      G.nzs = d.nzs;
      G.npl = d.npl;
      G.cs = d.cs;
      G.coef = (const T *)d.coef;
      const double me = D.rho * (D.Lx / D.nx) * (D.Ly / D.ny) * (D.Lz / D.nz) / 8.0;
      for (int cy = 0; cy < 3; ++cy)
        for (int cx = 0; cx < 3; ++cx) G.mass[cx + 3 * cy] = (T)(me * (cx == 1 ? 2 : 1) * (cy == 1 ? 2 : 1) * 2);
      G.held = D.lateral_fix;
      X.n3 = 3 * d.cs;
      X.v = al(X.n3);
      X.a = al(X.n3);
      X.vn = al(X.n3);
      X.an = al(X.n3);
      X.U = al(X.n3);
      X.V = al(X.n3);
      X.Aa = al(X.n3);
      X.Aa2 = al(X.n3);
      X.mu = al(X.n3);
      X.out = al(X.n3);
      X.tape = al((size_t)(K + 1) * X.n3);
      X.ckpt = al((size_t)nseg * 3 * X.n3);
      X.nblk = fom_misfit_blocks(G);
      X.part = ald((size_t)(K + 1) * X.nblk);
      if (st) break;
      const long long bo = 0;   // instance 0
      B.ok(hipMemcpyAsync(X.tape, (T *)d.u[step0 % 3] + bo, X.n3 * sizeof(T), hipMemcpyDeviceToDevice, s), "copy");
      B.ok(hipMemcpyAsync(X.v, (T *)d.v[step0 % 2] + bo, X.n3 * sizeof(T), hipMemcpyDeviceToDevice, s), "copy");
      B.ok(hipMemcpyAsync(X.a, (T *)d.a[step0 % 2] + bo, X.n3 * sizeof(T), hipMemcpyDeviceToDevice, s), "copy");
      X.u = X.tape;
    } else {
      X.r = d.r;
      X.rs = d.rs;
      X.r2 = d.oh.quadratic ? d.r * (d.r + 1) / 2 : 0;
      const int rsx = std::max(d.rs, 1);
      X.q = al(X.r);
      X.qd = al(X.r);
      X.qdd = al(X.r);
      X.Q = al(X.r);
      X.Qd = al(X.r);
      X.Qdd = al(X.r);
      X.Qdd2 = al(X.r);
      X.gh = al(rsx);
      X.gbar = al(rsx);
      X.gh0 = al(rsx);
      X.tq = al((size_t)(K + 1) * X.r);
      X.tg = al((size_t)(K + 1) * rsx);
      X.rckpt = al((size_t)nseg * 3 * X.r);
      X.dA = ald((size_t)X.r * X.r);
      X.dH = ald((size_t)X.r * std::max(X.r2, 1));
      X.dB = ald((size_t)X.r * rsx);
      X.dc = ald(X.r);
      X.rpart = ald((size_t)K + 1);
      if (st) break;
      B.ok(hipMemcpyAsync(X.q, (T *)d.q[step0 % 2], X.r * sizeof(T), hipMemcpyDeviceToDevice, s), "copy");
      B.ok(hipMemcpyAsync(X.qd, (T *)d.qd[step0 % 2], X.r * sizeof(T), hipMemcpyDeviceToDevice, s), "copy");
      B.ok(hipMemcpyAsync(X.qdd, (T *)d.qdd[step0 % 2], X.r * sizeof(T), hipMemcpyDeviceToDevice, s), "copy");
      if (d.rs > 0) {
        std::vector<double> g0 = d.gh0.empty() ? std::vector<double>() : d.gh0[0];
        g0.resize(d.rs, 0.0);
        if ((st = ctx->upload(X.gh0, g0.data(), d.rs))) break;
      }
    }
  }
  if (st || B.code) {
    release();
    return st ? ctx->fail(st, "out of device memory for the adjoint") : ctx->fail(B.code, B.msg);
  }

  // export rows of OpInf sources, in the order wire() stores them
  auto export_rows = [&](int src, int dst, int f) -> const T * {
    int e = 0;
    for (int i = 0; i < S; ++i) {
      const Subdomain &dd = *ctx->sds[i];
      if (dd.rom) continue;
      for (int ff = 0; ff < 2; ++ff) {
        if (dd.face_type[ff] == kFaceClamped || dd.proj[ff].src != src) continue;
        if (i == dst && ff == f) return (const T *)ctx->sds[src]->piphi_d[e];
        ++e;
      }
    }
    return nullptr;
  };
  auto face_layer = [&](const Subdomain &d, int f) -> long long { return (long long)(f == 0 ? 0 : d.nzs) * d.npl; };
  auto rom_args = [&](int i, int j) {
    Subdomain &d = *ctx->sds[i];
    AdjSd<T> &X = A[i];
    const int rsx = std::max(X.rs, 1);
    RomAdj<T> R{};
    R.r = X.r;
    R.rs = X.rs;
    R.r2 = X.r2;
    R.A = (const T *)d.d_A;
    R.H = (const T *)d.d_H;
    R.B = (const T *)d.d_B;
    R.c = (const T *)d.d_c;
    R.dt = dt;
    R.g = g;
    R.h = h;
    R.q = X.q;
    R.qd = X.qd;
    R.qdd = X.qdd;
    R.gh = X.gh;
    R.tape_q = X.tq + (size_t)j * X.r;
    R.tape_g = X.tg + (size_t)j * rsx;
    R.Q = X.Q;
    R.Qd = X.Qd;
    R.Qdd = X.Qdd;
    R.Qdd_prev = X.Qdd2;
    R.dA = X.dA;
    R.dH = X.dH;
    R.dB = X.dB;
    R.dc = d.d_c ? X.dc : nullptr;
    R.gbar = X.gbar;
    return R;
  };

  // ---- forward step k-1 -> k into tape slot j
  auto fwd_step = [&](int j) {
    for (int i = 0; i < S; ++i) {   // predictors
      AdjSd<T> &X = A[i];
      if (X.rom) continue;
      T *un = X.tape + (size_t)j * X.n3;
      B.ok(launch_fom_elem<T>(X.G, 0, un, X.u, X.v, X.a, dt, h, s), "predictor");
    }
    for (int i = 0; i < S; ++i)
      if (A[i].rom) {
        RomAdj<T> R = rom_args(i, j);
        R.mode = 2;   // predictor only (writes the tape)
        B.ok(launch_rom_fwd<T>(R, s), "rom predictor");
      }
    for (int i = 0; i < S; ++i) {   // faces / g^
      Subdomain &d = *ctx->sds[i];
      AdjSd<T> &X = A[i];
      if (X.rom && X.rs > 0) B.ok(hipMemsetAsync(X.gh, 0, X.rs * sizeof(T), s), "memset");
      for (int f = 0; f < 2; ++f) {
        if (d.face_type[f] == kFaceClamped) continue;
        const int src = d.proj[f].src;
        Subdomain &sd = *ctx->sds[src];
        AdjSd<T> &Y = A[src];
        if (!X.rom) {
          T *un = X.tape + (size_t)j * X.n3;
          if (!Y.rom)
            B.ok(launch_layer_copy<T>(un, d.cs, face_layer(d, f), Y.tape + (size_t)j * Y.n3, sd.cs,
                                      (long long)d.proj[f].src_layer * sd.npl, d.npl, 0, s), "face copy");
          else
            B.ok(launch_lift_face<T>(export_rows(src, i, f), Y.tq + (size_t)j * Y.r, Y.r, un, d.cs,
                                     face_layer(d, f), d.npl, s), "face lift");
        } else if (X.rs > 0) {
          if (!Y.rom)
            B.ok(launch_rows_dot<T>((const T *)d.face_phis[f], X.rs, 3 * d.npl, Y.tape + (size_t)j * Y.n3, sd.cs,
                                    (long long)d.proj[f].src_layer * sd.npl, d.npl, X.gh, s), "g^");
          else
            B.ok(launch_rows_dot<T>((const T *)d.face_tm[f], X.rs, Y.r, Y.tq + (size_t)j * Y.r, 0, 0, Y.r, X.gh,
                                    s), "g^");
        }
      }
    }
    for (int i = 0; i < S; ++i) {   // accelerations, velocities
      AdjSd<T> &X = A[i];
      if (X.rom) {
        RomAdj<T> R = rom_args(i, j);
        R.mode = 0;
        B.ok(launch_rom_fwd<T>(R, s), "rom step");
      } else {
        T *un = X.tape + (size_t)j * X.n3;
        B.ok(launch_stencil<T>(X.G, un, X.an, 1, X.G.nzs - 1, false, s), "stencil");
        B.ok(launch_fom_elem<T>(X.G, 1, X.vn, X.v, X.a, X.an, g, T(0), s), "velocity");
        X.u = un;
        std::swap(X.v, X.vn);
        std::swap(X.a, X.an);
      }
    }
  };
  auto save_ckpt = [&](int seg) {
    for (int i = 0; i < S; ++i) {
      AdjSd<T> &X = A[i];
      if (X.rom) {
        T *c = X.rckpt + (size_t)seg * 3 * X.r;
        B.ok(hipMemcpyAsync(c, X.q, X.r * sizeof(T), hipMemcpyDeviceToDevice, s), "ckpt");
        B.ok(hipMemcpyAsync(c + X.r, X.qd, X.r * sizeof(T), hipMemcpyDeviceToDevice, s), "ckpt");
        B.ok(hipMemcpyAsync(c + 2 * X.r, X.qdd, X.r * sizeof(T), hipMemcpyDeviceToDevice, s), "ckpt");
      } else {
        T *c = X.ckpt + (size_t)seg * 3 * X.n3;
        B.ok(hipMemcpyAsync(c, X.u, X.n3 * sizeof(T), hipMemcpyDeviceToDevice, s), "ckpt");
        B.ok(hipMemcpyAsync(c + X.n3, X.v, X.n3 * sizeof(T), hipMemcpyDeviceToDevice, s), "ckpt");
        B.ok(hipMemcpyAsync(c + 2 * X.n3, X.a, X.n3 * sizeof(T), hipMemcpyDeviceToDevice, s), "ckpt");
      }
    }
  };
  auto load_ckpt = [&](int seg) {
    for (int i = 0; i < S; ++i) {
      AdjSd<T> &X = A[i];
      if (X.rom) {
        const T *c = X.rckpt + (size_t)seg * 3 * X.r;
        B.ok(hipMemcpyAsync(X.q, c, X.r * sizeof(T), hipMemcpyDeviceToDevice, s), "ckpt");
        B.ok(hipMemcpyAsync(X.qd, c + X.r, X.r * sizeof(T), hipMemcpyDeviceToDevice, s), "ckpt");
        B.ok(hipMemcpyAsync(X.qdd, c + 2 * X.r, X.r * sizeof(T), hipMemcpyDeviceToDevice, s), "ckpt");
        B.ok(hipMemcpyAsync(X.tq, c, X.r * sizeof(T), hipMemcpyDeviceToDevice, s), "ckpt");   // slot 0 = q_k0
      } else {
        const T *c = X.ckpt + (size_t)seg * 3 * X.n3;
        B.ok(hipMemcpyAsync(X.tape, c, X.n3 * sizeof(T), hipMemcpyDeviceToDevice, s), "ckpt");
        B.ok(hipMemcpyAsync(X.v, c + X.n3, X.n3 * sizeof(T), hipMemcpyDeviceToDevice, s), "ckpt");
        B.ok(hipMemcpyAsync(X.a, c + 2 * X.n3, X.n3 * sizeof(T), hipMemcpyDeviceToDevice, s), "ckpt");
        X.u = X.tape;
      }
    }
  };

  // ---- forward pass with checkpoints
  for (int seg = 0; seg < nseg && !B.code; ++seg) {
    if (seg > 0) {   // the last state becomes slot 0 of the next segment
      for (int i = 0; i < S; ++i)
        if (!A[i].rom && A[i].u != A[i].tape)
          B.ok(hipMemcpyAsync(A[i].tape, A[i].u, A[i].n3 * sizeof(T), hipMemcpyDeviceToDevice, s), "copy");
      for (int i = 0; i < S; ++i) A[i].u = A[i].tape;
    }
    save_ckpt(seg);
    const long long k0 = (long long)seg * K, k1 = std::min<long long>(n, k0 + K);
    for (long long k = k0 + 1; k <= k1 && !B.code; ++k) fwd_step((int)(k - k0));
  }

  // ---- reverse sweep
  double J = 0.0;
  std::vector<double> hp;
  for (int seg = nseg - 1; seg >= 0 && !B.code; --seg) {
    const long long k0 = (long long)seg * K, k1 = std::min<long long>(n, k0 + K);
    load_ckpt(seg);
    for (long long k = k0 + 1; k <= k1 && !B.code; ++k) fwd_step((int)(k - k0));
    std::vector<char> observed((size_t)(k1 - k0 + 1), 0);
    for (long long k = k1; k > k0 && !B.code; --k) {
      const int j = (int)(k - k0);
      const bool obs_k = (k % M.every) == 0 && k / M.every <= n_obs;
      observed[j] = obs_k;
      const long long oi = k / M.every - 1;
      // 1. velocity transpose and misfit
      for (int i = 0; i < S; ++i) {
        AdjSd<T> &X = A[i];
        Subdomain &d = *ctx->sds[i];
        if (X.rom) {
          RomAdj<T> R = rom_args(i, j);
          R.mode = 0;
          R.obs = obs_k && M.obs[i] ? (const T *)M.obs[i] + (size_t)oi * X.r : nullptr;
          R.partial = X.rpart + j;
          B.ok(launch_rom_adj<T>(R, s), "rom adjoint");
        } else {
          B.ok(launch_fom_elem<T>(X.G, 5, X.Aa2, X.Aa, X.V, nullptr, g, T(0), s), "adjoint velocity");
          if (obs_k && M.obs[i])
            B.ok(launch_fom_misfit<T>(X.G, X.U, X.tape + (size_t)j * X.n3,
                                      (const T *)M.obs[i] + (size_t)oi * 3 * d.nfree_nodes,
                                      X.part + (size_t)j * X.nblk, s), "misfit");
        }
      }
      // 2. FOM acceleration transpose and its faces
      for (int i = 0; i < S; ++i) {
        AdjSd<T> &X = A[i];
        if (X.rom) continue;
        Subdomain &d = *ctx->sds[i];
        B.ok(launch_fom_elem<T>(X.G, 2, X.mu, X.Aa, nullptr, nullptr, T(0), T(0), s), "mu");
        B.ok(launch_stencil<T>(X.G, X.mu, X.out, 0, X.G.nzs, true, s), "adjoint stencil");
        B.ok(launch_fom_elem<T>(X.G, 3, X.U, X.out, nullptr, nullptr, T(0), T(0), s), "accumulate");
        for (int f = 0; f < 2; ++f) {
          if (d.face_type[f] == kFaceClamped) continue;
          const int src = d.proj[f].src;
          Subdomain &sd = *ctx->sds[src];
          AdjSd<T> &Y = A[src];
          if (!Y.rom)
            B.ok(launch_layer_copy<T>(Y.U, sd.cs, (long long)d.proj[f].src_layer * sd.npl, X.out, d.cs,
                                      face_layer(d, f), d.npl, 1, s), "face adjoint");
          else
            B.ok(launch_rows_dot<T>(export_rows(src, i, f), Y.r, 3 * d.npl, X.out, d.cs, face_layer(d, f), d.npl,
                                    Y.Q, s), "face adjoint");
        }
      }
      // 3. g^ transpose into the sources
      for (int i = 0; i < S; ++i) {
        AdjSd<T> &X = A[i];
        if (!X.rom || X.rs == 0) continue;
        Subdomain &d = *ctx->sds[i];
        for (int f = 0; f < 2; ++f) {
          if (d.face_type[f] == kFaceClamped) continue;
          const int src = d.proj[f].src;
          Subdomain &sd = *ctx->sds[src];
          AdjSd<T> &Y = A[src];
          if (!Y.rom)
            B.ok(launch_rows_tdot<T>((const T *)d.face_phis[f], X.rs, 3 * d.npl, X.gbar, Y.U, sd.cs,
                                     (long long)d.proj[f].src_layer * sd.npl, d.npl, s), "g^ adjoint");
          else
            B.ok(launch_rows_tdot<T>((const T *)d.face_tm[f], X.rs, Y.r, X.gbar, Y.Q, 0, 0, Y.r, s), "g^ adjoint");
        }
      }
      // 4. predictor transpose; the accumulators move to step k-1
      for (int i = 0; i < S; ++i) {
        AdjSd<T> &X = A[i];
        if (X.rom) {
          RomAdj<T> R = rom_args(i, j);
          B.ok(launch_rom_adj_pred<T>(R, s), "rom predictor adjoint");
          std::swap(X.Qdd, X.Qdd2);
        } else {
          B.ok(launch_fom_elem<T>(X.G, 4, X.U, nullptr, X.V, X.Aa2, dt, h, s), "predictor adjoint");
          std::swap(X.Aa, X.Aa2);
        }
      }
    }
    // misfit of this segment, summed in a fixed order
    for (int i = 0; i < S && !B.code; ++i) {
      AdjSd<T> &X = A[i];
      const size_t cnt = X.rom ? (size_t)K + 1 : (size_t)(K + 1) * X.nblk;
      hp.resize(cnt);
      if (!B.ok(hipMemcpyAsync(hp.data(), X.rom ? X.rpart : X.part, cnt * sizeof(double), hipMemcpyDeviceToHost, s),
                "download"))
        break;
      B.ok(hipStreamSynchronize(s), "sync");
      if (!M.obs[i]) continue;
      for (long long k = k0 + 1; k <= k1; ++k) {
        const int j = (int)(k - k0);
        if (!observed[j]) continue;
        if (X.rom) J += hp[j];
        else
          for (int bl = 0; bl < X.nblk; ++bl) J += hp[(size_t)j * X.nblk + bl];
      }
    }
  }
  // ---- initial state: a_0 = C u_0 (+ constant faces), q''_0 = f(q_0, g^_0)
  for (int i = 0; i < S && !B.code; ++i) {
    AdjSd<T> &X = A[i];
    if (X.rom) {
      B.ok(hipMemcpyAsync(X.tq, X.rckpt, X.r * sizeof(T), hipMemcpyDeviceToDevice, s), "copy");
      if (X.rs > 0) B.ok(hipMemcpyAsync(X.tg, X.gh0, X.rs * sizeof(T), hipMemcpyDeviceToDevice, s), "copy");
      RomAdj<T> R = rom_args(i, 0);
      R.mode = 1;
      R.obs = nullptr;
      R.partial = nullptr;
      B.ok(launch_rom_adj<T>(R, s), "rom adjoint (initial)");
    } else {
      B.ok(launch_fom_elem<T>(X.G, 2, X.mu, X.Aa, nullptr, nullptr, T(0), T(0), s), "mu");
      B.ok(launch_stencil<T>(X.G, X.mu, X.out, 1, X.G.nzs - 1, true, s), "adjoint stencil");
      B.ok(launch_fom_elem<T>(X.G, 3, X.U, X.out, nullptr, nullptr, T(0), T(0), s), "accumulate");
    }
  }
  // ---- outputs
  for (int i = 0; i < S && !B.code; ++i) {
    AdjSd<T> &X = A[i];
    Subdomain &d = *ctx->sds[i];
    if (!X.rom) {
      const long long nf = d.nfree_nodes;
      // held lateral components start at zero whatever u0, v0 say: no gradient there
      B.ok(launch_fom_elem<T>(X.G, 6, X.U, nullptr, nullptr, nullptr, T(0), T(0), s), "mask");
      B.ok(launch_fom_elem<T>(X.G, 6, X.V, nullptr, nullptr, nullptr, T(0), T(0), s), "mask");
      for (int c = 0; c < 3; ++c) {
        if (Gr.du0[i])
          B.ok(hipMemcpyAsync((T *)Gr.du0[i] + c * nf, X.U + c * d.cs + d.npl, nf * sizeof(T),
                              hipMemcpyDeviceToDevice, s), "du0");
        if (Gr.dv0[i])
          B.ok(hipMemcpyAsync((T *)Gr.dv0[i] + c * nf, X.V + c * d.cs + d.npl, nf * sizeof(T),
                              hipMemcpyDeviceToDevice, s), "dv0");
      }
      continue;
    }
    const int r = X.r, rs = X.rs, r2 = X.r2;
    auto down_d = [&](const double *src, size_t cnt) {
      std::vector<double> v(cnt);
      B.ok(hipMemcpyAsync(v.data(), src, cnt * sizeof(double), hipMemcpyDeviceToHost, s), "download");
      B.ok(hipStreamSynchronize(s), "sync");
      return v;
    };
    auto colmajor = [&](const std::vector<double> &rm, int rows, int cols, double *dst) {
      for (int a = 0; a < rows; ++a)
        for (int b = 0; b < cols; ++b) dst[(size_t)a + (size_t)b * rows] = rm[(size_t)a * cols + b];
    };
    if (Gr.dA[i]) colmajor(down_d(X.dA, (size_t)r * r), r, r, Gr.dA[i]);
    if (Gr.dH[i] && r2 > 0) colmajor(down_d(X.dH, (size_t)r * r2), r, r2, Gr.dH[i]);
    if (Gr.dB[i] && rs > 0) colmajor(down_d(X.dB, (size_t)r * rs), r, rs, Gr.dB[i]);
    if (Gr.dc[i] && d.d_c) {
      auto v = down_d(X.dc, r);
      std::copy(v.begin(), v.end(), Gr.dc[i]);
    }
    if (Gr.dq0[i] && ctx->download(Gr.dq0[i], X.Q, r)) B.ok(hipErrorUnknown, "dq0 download");
    if (Gr.dqd0[i] && ctx->download(Gr.dqd0[i], X.Qd, r)) B.ok(hipErrorUnknown, "dqd0 download");
  }
  if (!B.code) B.ok(hipStreamSynchronize(s), "sync");
  release();
  if (B.code) return ctx->fail(B.code, B.msg);
  if (J_out) *J_out = J;
  return OSAM_OK;
}

int32_t Ctx::run_adjoint(int64_t n, int64_t K, const osam_misfit &M, double *J, const osam_grads &G) {
  if (batch != 1) return fail(OSAM_E_INVALID, "run_adjoint needs a context with batch 1");
  if (n < 1 || K < 1 || M.every < 1) return fail(OSAM_E_INVALID, "n_steps, checkpoint_every and every must be >= 1");
  if ((int)sds.size() > 8) return fail(OSAM_E_INVALID, "too many subdomains");
  int32_t st = couple();
  if (st) return st;
  if ((st = wire())) return st;
  if (!initialized[0]) return fail(OSAM_E_ORDER, "instance 0 has no initial condition");
  if ((st = sync_status())) return st;
  if ((st = init_pending())) return st;
  if (prec == OSAM_FP64) return adjoint_impl<double>(this, n, K, M, J, G);
  return adjoint_impl<float>(this, n, K, M, J, G);
}

}  // namespace osam

extern "C" int32_t run_adjoint(osam_ctx *c, int64_t n_steps, int64_t checkpoint_every, const osam_misfit *misfit,
                               double *J, const osam_grads *grads) {
  if (!c || !misfit || !grads) return OSAM_E_INVALID;
  osam::Ctx *ctx = reinterpret_cast<osam::Ctx *>(c);
  ctx->err.clear();
  hipSetDevice(ctx->device);
  return ctx->run_adjoint(n_steps, checkpoint_every, *misfit, J, *grads);
}
