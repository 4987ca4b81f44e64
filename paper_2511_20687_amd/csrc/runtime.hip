// Host runtime of libosam: the C ABI of include/osam.h.
//
// The runtime owns device memory, builds the per-subdomain stencil
// coefficients and pointwise projections, wires the Schwarz transfers between
// FOM and OpInf subdomains, and drives the controller: it enqueues whole
// "rounds" (one Schwarz sweep = one kernel per subdomain, in index order) and
// lets every instance iterate at its own pace on the device (status words in
// device memory, Sec. 4.1 Alg. 1 executed by the kernels).  The host only
// waits between chunks of rounds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/osam.h"
#include "stencil.hpp"
#include "osam_device.hpp"
#include "runtime.hpp"

namespace osam {

// kernel launchers (fe_kernels.hip / rom_kernels.hip / learn_kernels.hip)
template <typename T> hipError_t launch_fe(const FeArgs<T> &, int, int, int, hipStream_t);
template <typename T> hipError_t launch_rom(const RomArgs<T> &, int, hipStream_t);
template <typename T> size_t rom_smem_bytes(int, int, int);
template <typename T>
hipError_t launch_project(const T *, long long, long long, const T *, long long, long long, double *, int,
                          int, hipStream_t);
template <typename T>
hipError_t launch_lift(const T *, long long, long long, int, const T *, T *, long long, long long, hipStream_t);

// ---------------------------------------------------------------------------
// Element stiffness of a box hex8 (hx, hy, hz), isotropic linear elasticity
// (App. A.1), 2x2x2 Gauss rule:
//   K_ab^pq = int lam dN_a/dx_p dN_b/dx_q + mu (dN_a/dx_q dN_b/dx_p + delta_pq grad N_a . grad N_b)
// Local corner a = cx + 2 cy + 4 cz, (cx, cy, cz) in {0,1}^3.
static void box_stiffness(double hx, double hy, double hz, double lam, double mu, double K[24][24]) {
  std::memset(K, 0, sizeof(double) * 24 * 24);
  const double g = 1.0 / std::sqrt(3.0);
  const double h[3] = {hx, hy, hz};
  const double detJ = hx * hy * hz / 8.0;
  for (int gz = 0; gz < 2; ++gz)
    for (int gy = 0; gy < 2; ++gy)
      for (int gx = 0; gx < 2; ++gx) {
        const double xi[3] = {gx ? g : -g, gy ? g : -g, gz ? g : -g};
        double dN[8][3];
        for (int a = 0; a < 8; ++a) {
          const double s[3] = {(a & 1) ? 1.0 : -1.0, (a & 2) ? 1.0 : -1.0, (a & 4) ? 1.0 : -1.0};
          const double f[3] = {1 + s[0] * xi[0], 1 + s[1] * xi[1], 1 + s[2] * xi[2]};
          dN[a][0] = 0.125 * s[0] * f[1] * f[2] * 2.0 / h[0];
          dN[a][1] = 0.125 * s[1] * f[0] * f[2] * 2.0 / h[1];
          dN[a][2] = 0.125 * s[2] * f[0] * f[1] * 2.0 / h[2];
        }
        for (int a = 0; a < 8; ++a)
          for (int b = 0; b < 8; ++b) {
            const double gg = dN[a][0] * dN[b][0] + dN[a][1] * dN[b][1] + dN[a][2] * dN[b][2];
            for (int p = 0; p < 3; ++p)
              for (int q = 0; q < 3; ++q) {
                double v = lam * dN[a][p] * dN[b][q] + mu * dN[a][q] * dN[b][p];
                if (p == q) v += mu * gg;
                K[3 * a + p][3 * b + q] += v * detJ;
              }
          }
      }
}

// Stencil blocks C_d = -K_d / m for the 9 cross-section cases (free z-layer),
// layout [case][26][3][3], case = cx + 3 cy (0: index 0, 1: interior, 2: index n).
static void stencil_coefficients(const osam_subdomain_desc &d, std::vector<double> &C) {
  const double hx = d.Lx / d.nx, hy = d.Ly / d.ny, hz = d.Lz / d.nz;
  const double lam = d.E * d.nu / ((1 + d.nu) * (1 - 2 * d.nu));
  const double mu = d.E / (2 * (1 + d.nu));
  double K[24][24];
  box_stiffness(hx, hy, hz, lam, mu, K);
  C.assign(9 * 26 * 9, 0.0);
  for (int cy = 0; cy < 3; ++cy)
    for (int cx = 0; cx < 3; ++cx) {
      const int cse = cx + 3 * cy;
      int nel = 0;
      double Kd[27][3][3] = {};
      for (int oz = 0; oz < 2; ++oz)
        for (int oy = 0; oy < 2; ++oy)
          for (int ox = 0; ox < 2; ++ox) {
            // octant element: lower corner at node + (ox-1, oy-1, oz-1)
            if ((cx == 0 && ox == 0) || (cx == 2 && ox == 1)) continue;
            if ((cy == 0 && oy == 0) || (cy == 2 && oy == 1)) continue;
            ++nel;
            const int nc[3] = {1 - ox, 1 - oy, 1 - oz};
            const int an = nc[0] + 2 * nc[1] + 4 * nc[2];
            for (int dz = -1; dz <= 1; ++dz)
              for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                  const int mc[3] = {nc[0] + dx, nc[1] + dy, nc[2] + dz};
                  if (mc[0] < 0 || mc[0] > 1 || mc[1] < 0 || mc[1] > 1 || mc[2] < 0 || mc[2] > 1) continue;
                  const int am = mc[0] + 2 * mc[1] + 4 * mc[2];
                  const int d27 = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                  for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q) Kd[d27][p][q] += K[3 * an + p][3 * am + q];
                }
          }
      const double m = d.rho * hx * hy * hz / 8.0 * nel;
      for (int d27 = 0; d27 < 27; ++d27) {
        if (d27 == 13) continue;
        const int d26 = d27 < 13 ? d27 : d27 - 1;
        for (int p = 0; p < 3; ++p)
          for (int q = 0; q < 3; ++q) C[(cse * 26 + d26) * 9 + p * 3 + q] = -Kd[d27][p][q] / m;
      }
    }
}

// The 27 distinct values of the interior block (structure: box_index, box_sign),
// checked against every entry: false if the block does not have that structure.
static bool box_coefficients(const double *Ci, double cb[27]) {
  double cmax = 0.0;
  for (int i = 0; i < 234; ++i) cmax = std::max(cmax, std::fabs(Ci[i]));
  bool have[27] = {};
  for (int d27 = 0; d27 < 27; ++d27) {
    if (d27 == 13) continue;
    const int d26 = d27 < 13 ? d27 : d27 - 1;
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) {
        const double v = Ci[d26 * 9 + p * 3 + q];
        const int bi = box_index(d27, p, q);
        if (bi < 0) {
          if (std::fabs(v) > 1e-12 * cmax) return false;
          continue;
        }
        const double x = v * box_sign(d27, p, q);
        if (!have[bi]) {
          cb[bi] = x;
          have[bi] = true;
        } else if (std::fabs(x - cb[bi]) > 1e-12 * cmax) {
          return false;
        }
      }
  }
  return true;
}

// ---------------------------------------------------------------------------
#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return ctx->fail(OSAM_E_HIP, std::string(#expr) + ": " +     \
                                                            hipGetErrorString(e_));    \
  } while (0)

int32_t Ctx::fail(int32_t code, const std::string &msg) {
  err = msg;
  return code;
}

// Device memory comes from large 2 MiB-aligned blocks carved by the context
// (first fit over freed chunks, no coalescing): the many small per-subdomain
// buffers then share large pages instead of each holding its own small-page
// allocation, which keeps the kernels' address-translation misses down.
void *Ctx::arena_alloc(size_t bytes, int32_t *st) {
  constexpr size_t kAlign = 256, kPage = size_t(2) << 20, kBlock = size_t(64) << 20;
  bytes = (std::max<size_t>(bytes, 1) + kAlign - 1) / kAlign * kAlign;
  for (auto &c : chunks)
    if (c.free && c.bytes >= bytes) {
      c.free = false;
      return c.ptr;
    }
  if (!arena_cur || arena_used + bytes > arena_cap) {
    const size_t cap = std::max(kBlock, (bytes + kPage - 1) / kPage * kPage);
    void *raw = nullptr;
    if (hipMalloc(&raw, cap + kPage) != hipSuccess) {
      *st = OSAM_E_OOM;
      return nullptr;
    }
    allocs.push_back(raw);
    const uintptr_t a = (reinterpret_cast<uintptr_t>(raw) + kPage - 1) / kPage * kPage;
    arena_cur = reinterpret_cast<char *>(a);
    arena_cap = cap;
    arena_used = 0;
  }
  char *p = arena_cur + arena_used;
  arena_used += bytes;
  chunks.push_back({p, bytes, false});
  return p;
}

template <typename T>
static T *dalloc(Ctx *ctx, size_t n, int32_t *st) {
  return static_cast<T *>(ctx->arena_alloc(n * sizeof(T), st));
}

void Ctx::dfree(void *p) {
  if (!p) return;
  for (auto &c : chunks)
    if (c.ptr == p) {
      c.free = true;
      return;
    }
}

size_t Ctx::esize() const { return prec == OSAM_FP64 ? 8 : 4; }

// upload float64 host data converted to the context precision
int32_t Ctx::upload(void *dst, const double *src, size_t n) {
  Ctx *ctx = this;
  if (prec == OSAM_FP64) {
    HIPCHK(hipMemcpyAsync(dst, src, n * 8, hipMemcpyHostToDevice, stream));
    HIPCHK(hipStreamSynchronize(stream));
  } else {
    std::vector<float> tmp(src, src + n);
    HIPCHK(hipMemcpyAsync(dst, tmp.data(), n * 4, hipMemcpyHostToDevice, stream));
    HIPCHK(hipStreamSynchronize(stream));
  }
  return OSAM_OK;
}

int32_t Ctx::download(double *dst, const void *src, size_t n) {
  Ctx *ctx = this;
  if (prec == OSAM_FP64) {
    HIPCHK(hipMemcpyAsync(dst, src, n * 8, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
  } else {
    std::vector<float> tmp(n);
    HIPCHK(hipMemcpyAsync(tmp.data(), src, n * 4, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    for (size_t i = 0; i < n; ++i) dst[i] = tmp[i];
  }
  return OSAM_OK;
}

void *Ctx::alloc_t(size_t n, int32_t *st) {
  return prec == OSAM_FP64 ? (void *)dalloc<double>(this, n, st) : (void *)dalloc<float>(this, n, st);
}

}  // namespace osam

using namespace osam;

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int32_t osam_version(void) { return 10000; }

int32_t osam_ctx_create(osam_ctx **out, int32_t device, int32_t precision, int32_t batch, void *stream) {
  if (!out) return OSAM_E_INVALID;
  *out = nullptr;
  if (precision != OSAM_FP64 && precision != OSAM_FP32 && precision != OSAM_FP32_BF16H) return OSAM_E_INVALID;
  if (batch < 1) return OSAM_E_INVALID;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return OSAM_E_HIP;
  if (hipSetDevice(device) != hipSuccess) return OSAM_E_HIP;
  auto *ctx = new (std::nothrow) Ctx();
  if (!ctx) return OSAM_E_OOM;
  ctx->device = device;
  ctx->prec = precision;
  ctx->batch = batch;
  // the static scratch array of run_noalloc, looked up once per device (null on failure:
  // run_noalloc then reports it)
  if (static_scratch_address(device, &ctx->static_scratch) != OSAM_OK) ctx->static_scratch = nullptr;
  if (stream) {
    ctx->stream = static_cast<hipStream_t>(stream);
    ctx->own_stream = false;
  } else {
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
      delete ctx;
      return OSAM_E_HIP;
    }
    ctx->own_stream = true;
  }
  int32_t st = OSAM_OK;
  ctx->d_status = dalloc<Status>(ctx, batch, &st);
  if (st == OSAM_OK) ctx->d_status_alt = dalloc<Status>(ctx, batch, &st);
  if (st == OSAM_OK) ctx->rom_sums = dalloc<double>(ctx, (size_t)2 * batch * kMaxSd * 2, &st);
  if (st != OSAM_OK) {
    osam_ctx_destroy(reinterpret_cast<osam_ctx *>(ctx));
    return st;
  }
  if (hipHostMalloc(reinterpret_cast<void **>(&ctx->h_status), sizeof(Status) * batch) != hipSuccess) {
    osam_ctx_destroy(reinterpret_cast<osam_ctx *>(ctx));
    return OSAM_E_HIP;
  }
  std::memset(ctx->h_status, 0, sizeof(Status) * batch);
  hipMemcpy(ctx->d_status, ctx->h_status, sizeof(Status) * batch, hipMemcpyHostToDevice);
  hipMemcpy(ctx->d_status_alt, ctx->h_status, sizeof(Status) * batch, hipMemcpyHostToDevice);
  ctx->initialized.assign(batch, 0);
  *out = reinterpret_cast<osam_ctx *>(ctx);
  return OSAM_OK;
}

void osam_ctx_destroy(osam_ctx *c) {
  if (!c) return;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  hipSetDevice(ctx->device);
  if (ctx->stream) hipStreamSynchronize(ctx->stream);
  for (void *p : ctx->allocs) hipFree(p);
  ctx->allocs.clear();
  if (ctx->h_status) hipHostFree(ctx->h_status);
  for (hipEvent_t e : ctx->ev_pool) hipEventDestroy(e);
  if (ctx->aux) {
    hipStreamSynchronize(ctx->aux);
    hipStreamDestroy(ctx->aux);
    hipEventDestroy(ctx->fork_ev);
    hipEventDestroy(ctx->join_ev);
  }
  if (ctx->own_stream && ctx->stream) hipStreamDestroy(ctx->stream);
  delete ctx;
}

const char *osam_last_error(const osam_ctx *c) {
  if (!c) return "null context";
  return reinterpret_cast<const Ctx *>(c)->err.c_str();
}

int32_t create_subdomain(osam_ctx *c, const osam_subdomain_desc *d, int32_t *sd_id) {
  if (!c || !d) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  if ((int)ctx->sds.size() >= kMaxSd) return ctx->fail(OSAM_E_INVALID, "too many subdomains");
  if (ctx->coupled) return ctx->fail(OSAM_E_ORDER, "create_subdomain after osam_couple");
  if (d->nx < 1 || d->ny < 1 || d->nz < 2 || d->z_lo < 0 || d->z_hi > d->nz || d->z_hi - d->z_lo < 2)
    return ctx->fail(OSAM_E_INVALID, "bad grid or layer range");
  if (!(d->Lx > 0 && d->Ly > 0 && d->Lz > 0 && d->E > 0 && d->rho > 0 && d->nu > -1 && d->nu < 0.5 &&
        d->dt > 0))
    return ctx->fail(OSAM_E_INVALID, "bad geometry, material or dt");
  if (!(d->beta >= 0.0 && d->beta <= 0.5 && d->gamma >= 0.5 && d->gamma <= 1.0))
    return ctx->fail(OSAM_E_INVALID, "Newmark parameters outside 0 <= beta <= 1/2, 1/2 <= gamma <= 1");
  if (d->n_sub < 0 || d->n_sub > 64) return ctx->fail(OSAM_E_INVALID, "n_sub must be in 0..64");
  if (d->material != OSAM_LINEAR_ELASTIC && d->material != OSAM_SVK)
    return ctx->fail(OSAM_E_INVALID, "material must be OSAM_LINEAR_ELASTIC or OSAM_SVK");
  if (d->material == OSAM_SVK && d->beta != 0.0)
    return ctx->fail(OSAM_E_INVALID, "the Saint Venant-Kirchhoff material takes the explicit scheme (beta = 0)");
  const bool ext_lo = d->z_lo == 0, ext_hi = d->z_hi == d->nz;
  if ((ext_lo || ext_hi) && !d->clamp_ends)
    return ctx->fail(OSAM_E_INVALID, "traction-free exterior z-faces are not supported (clamp_ends = 1)");
  if (d->lateral_fix < 0 || d->lateral_fix > 7) return ctx->fail(OSAM_E_INVALID, "lateral_fix must be in 0..7");
  if (!ctx->sds.empty()) {
    const auto &d0 = ctx->sds[0]->desc;
    if (d0.nx != d->nx || d0.ny != d->ny || d0.nz != d->nz || d0.Lx != d->Lx || d0.Ly != d->Ly ||
        d0.Lz != d->Lz || d0.dt != d->dt)
      return ctx->fail(OSAM_E_INVALID,
                       "all subdomains must share the global grid and time step in this version");
    if (d0.lateral_fix != d->lateral_fix)
      return ctx->fail(OSAM_E_INVALID, "all subdomains must share the lateral boundary condition");
  }
  auto sd = std::make_unique<Subdomain>();
  sd->desc = *d;
  sd->nx = d->nx;
  sd->ny = d->ny;
  sd->nzs = d->z_hi - d->z_lo;
  sd->npl = (d->nx + 1) * (d->ny + 1);
  sd->nnodes = (long long)sd->npl * (sd->nzs + 1);
  sd->cs = (sd->nnodes + 63) / 64 * 64;
  sd->is = 3 * sd->cs;
  sd->nfree_nodes = (long long)sd->npl * (sd->nzs - 1);
  sd->face_type[0] = ext_lo ? kFaceClamped : kFaceFom;
  sd->face_type[1] = ext_hi ? kFaceClamped : kFaceFom;
  sd->nsch_nodes = (long long)sd->npl * ((ext_lo ? 0 : 1) + (ext_hi ? 0 : 1));
  sd->face_off_hi = ext_lo ? 0 : sd->npl;
  sd->n_sub = d->n_sub > 1 ? d->n_sub : 1;

  // stencil coefficients
  std::vector<double> C;
  stencil_coefficients(*d, C);
  if (!box_coefficients(C.data() + 4 * 234, sd->cb))
    return ctx->fail(OSAM_E_INVALID, "interior stencil lacks the mirror symmetries of a box element");
  // lateral Dirichlet components: zero rows of every lateral case, so the
  // acceleration of a held component is exactly zero (u, v start at zero)
  for (int cse = 0; cse < 9; ++cse) {
    if (cse == 4) continue;
    for (int p = 0; p < 3; ++p) {
      if (!(d->lateral_fix & (1 << p))) continue;
      for (int d26 = 0; d26 < 26; ++d26)
        for (int q = 0; q < 3; ++q) C[(cse * 26 + d26) * 9 + p * 3 + q] = 0.0;
    }
  }
  int32_t st = OSAM_OK;
  sd->coef = ctx->alloc_t(C.size(), &st);
  if (st) return ctx->fail(st, "out of device memory");
  if ((st = ctx->upload(sd->coef, C.data(), C.size()))) return st;
  // state buffers are allocated when the coupling is wired (FOM subdomains only)
  // boundary columns grouped by stencil case (a wave never mixes groups, so all
  // its lanes share one coefficient block)
  std::vector<int> bnd;
  sd->nbg = 0;
  for (int cse = 0; cse < 9; ++cse) {
    if (cse == 4) continue;
    const size_t start = bnd.size();
    for (int iy = 0; iy <= d->ny; ++iy)
      for (int ix = 0; ix <= d->nx; ++ix) {
        const int cx = ix == 0 ? 0 : (ix == d->nx ? 2 : 1), cy = iy == 0 ? 0 : (iy == d->ny ? 2 : 1);
        if (cx + 3 * cy == cse) bnd.push_back(ix + (d->nx + 1) * iy);
      }
    if (bnd.size() > start) {
      sd->bg_start[sd->nbg] = (int)start;
      sd->bg_n[sd->nbg] = (int)(bnd.size() - start);
      ++sd->nbg;
    }
  }
  sd->n_bnd = (int)bnd.size();
  sd->n_int = (d->nx - 1) * (d->ny - 1);
  sd->bnd_cols = dalloc<int>(ctx, bnd.size(), &st);
  if (st) return ctx->fail(st, "out of device memory");
  HIPCHK(hipMemcpy(sd->bnd_cols, bnd.data(), bnd.size() * sizeof(int), hipMemcpyHostToDevice));
  ctx->choose_fe_launch(*sd, 0, 0);
  sd->partials = dalloc<double>(ctx, (size_t)ctx->batch * sd->max_nblocks * 4, &st);
  if (st) return ctx->fail(st, "out of device memory");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (sd_id) *sd_id = (int32_t)ctx->sds.size();
  ctx->sds.push_back(std::move(sd));
  return OSAM_OK;
}

int32_t osam_couple(osam_ctx *c) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  return ctx->couple();
}

int32_t osam_sizes(osam_ctx *c, int32_t sdi, int64_t *n_nodes, int64_t *n_free, int64_t *n_sch, int32_t *r,
                   int32_t *r_s) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  if (sdi < 0 || sdi >= (int)ctx->sds.size()) return ctx->fail(OSAM_E_INVALID, "bad subdomain id");
  const Subdomain &s = *ctx->sds[sdi];
  if (n_nodes) *n_nodes = s.nnodes;
  if (n_free) *n_free = 3 * s.nfree_nodes;
  if (n_sch) *n_sch = 3 * s.nsch_nodes;
  if (r) *r = s.rom ? s.r : 0;
  if (r_s) *r_s = s.rom ? s.rs : 0;
  return OSAM_OK;
}

int32_t osam_set_initial(osam_ctx *c, int32_t inst, const double *u0, const double *v0) {
  if (!c || !u0 || !v0) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  if (inst < 0 || inst >= ctx->batch) return ctx->fail(OSAM_E_INVALID, "bad instance");
  if (ctx->sds.empty()) return ctx->fail(OSAM_E_ORDER, "no subdomains");
  int32_t st = ctx->couple();
  if (st) return st;
  return ctx->set_initial(inst, u0, v0);
}

int32_t osam_set_record(osam_ctx *c, int32_t sdi, const osam_record *rec) {
  if (!c || !rec) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  if (sdi < 0 || sdi >= (int)ctx->sds.size()) return ctx->fail(OSAM_E_INVALID, "bad subdomain id");
  if (rec->every < 0 || rec->n_cols < 0) return ctx->fail(OSAM_E_INVALID, "bad record sizes");
  ctx->sds[sdi]->rec = *rec;
  return OSAM_OK;
}

int32_t osam_get_state(osam_ctx *c, int32_t sdi, int32_t inst, double *u, double *v, double *a) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  if (sdi < 0 || sdi >= (int)ctx->sds.size() || inst < 0 || inst >= ctx->batch)
    return ctx->fail(OSAM_E_INVALID, "bad subdomain or instance");
  return ctx->get_state(sdi, inst, u, v, a);
}

int32_t osam_get_reduced(osam_ctx *c, int32_t sdi, int32_t inst, double *q, double *qd, double *qdd) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  if (sdi < 0 || sdi >= (int)ctx->sds.size() || inst < 0 || inst >= ctx->batch)
    return ctx->fail(OSAM_E_INVALID, "bad subdomain or instance");
  Subdomain &s = *ctx->sds[sdi];
  if (!s.rom) return ctx->fail(OSAM_E_INVALID, "not an OpInf subdomain");
  int32_t st = ctx->sync_status();
  if (st) return st;
  const int par = (int)(ctx->h_status[inst].step % 2);
  const size_t off = (size_t)inst * s.r * ctx->esize();
  if (q && (st = ctx->download(q, (char *)s.q[par] + off, s.r))) return st;
  if (qd && (st = ctx->download(qd, (char *)s.qd[par] + off, s.r))) return st;
  if (qdd && (st = ctx->download(qdd, (char *)s.qdd[par] + off, s.r))) return st;
  return OSAM_OK;
}

int32_t osam_set_opinf(osam_ctx *c, int32_t sdi, int32_t r, int32_t r_s, const double *Phi, const double *PhiS,
                       const double *A, const double *H, const double *B, const double *cvec) {
  if (!c || !Phi || !A) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  if (sdi < 0 || sdi >= (int)ctx->sds.size()) return ctx->fail(OSAM_E_INVALID, "bad subdomain id");
  Subdomain &s = *ctx->sds[sdi];
  if (r < 1 || r > 128 || r_s < 0 || (r_s > 0 && (!PhiS || !B)))
    return ctx->fail(OSAM_E_INVALID, "bad reduced dimensions (1 <= r <= 128)");
  if (r_s > 0 && s.nsch_nodes == 0) return ctx->fail(OSAM_E_INVALID, "no Schwarz DOFs for r_s > 0");
  OpinfHost oh;
  oh.r = r;
  oh.rs = r_s;
  oh.quadratic = H != nullptr;
  const long long nf = 3 * s.nfree_nodes, ns = 3 * s.nsch_nodes;
  oh.Phi.assign(Phi, Phi + (size_t)nf * r);
  // rows of lateral components held at zero carry no displacement
  if (s.desc.lateral_fix) {
    const int nxp = s.desc.nx + 1;
    for (long long fn = 0; fn < s.nfree_nodes; ++fn) {
      const int nid = (int)(fn % s.npl), ix = nid % nxp, iy = nid / nxp;
      if (!(ix == 0 || ix == s.desc.nx || iy == 0 || iy == s.desc.ny)) continue;
      for (int cc = 0; cc < 3; ++cc)
        if (s.desc.lateral_fix & (1 << cc))
          for (int k = 0; k < r; ++k) oh.Phi[(size_t)(cc * s.nfree_nodes + fn) + (size_t)k * nf] = 0.0;
    }
  }
  if (r_s > 0) oh.PhiS.assign(PhiS, PhiS + (size_t)ns * r_s);
  // column-major [r x r] -> keep column-major on host; kernels take row-major
  oh.A.assign(A, A + (size_t)r * r);
  if (H) oh.H.assign(H, H + (size_t)r * (r * (r + 1) / 2));
  if (B && r_s > 0) oh.B.assign(B, B + (size_t)r * r_s);
  if (cvec) oh.c.assign(cvec, cvec + r);
  return ctx->install_opinf(sdi, oh);
}

int32_t osam_get_opinf(osam_ctx *c, int32_t sdi, double *Phi, double *PhiS, double *A, double *H, double *B,
                       double *cvec) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  if (sdi < 0 || sdi >= (int)ctx->sds.size()) return ctx->fail(OSAM_E_INVALID, "bad subdomain id");
  Subdomain &s = *ctx->sds[sdi];
  if (!s.rom) return ctx->fail(OSAM_E_INVALID, "not an OpInf subdomain");
  const OpinfHost &o = s.oh;
  if (Phi) {
    if (!o.Phi.empty()) {
      std::copy(o.Phi.begin(), o.Phi.end(), Phi);
    } else {
      int32_t st = ctx->download(Phi, s.d_Phi, (size_t)3 * s.nfree_nodes * s.r);
      if (st) return st;
    }
  }
  if (PhiS) std::copy(o.PhiS.begin(), o.PhiS.end(), PhiS);
  if (A) std::copy(o.A.begin(), o.A.end(), A);
  if (H && o.quadratic) std::copy(o.H.begin(), o.H.end(), H);
  if (B) std::copy(o.B.begin(), o.B.end(), B);
  if (cvec && !o.c.empty()) std::copy(o.c.begin(), o.c.end(), cvec);
  return OSAM_OK;
}

int32_t osam_set_opinf_cubic(osam_ctx *c, int32_t sdi, const double *C3) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  if (sdi < 0 || sdi >= (int)ctx->sds.size()) return ctx->fail(OSAM_E_INVALID, "bad subdomain id");
  Subdomain &s = *ctx->sds[sdi];
  if (!s.rom) return ctx->fail(OSAM_E_ORDER, "osam_set_opinf_cubic follows osam_set_opinf or learn_opinf");
  const long long r = s.r, r3 = r * (r + 1) * (r + 2) / 6;
  if (C3) s.oh.C3.assign(C3, C3 + (size_t)r * r3);
  else s.oh.C3.clear();
  // the initial states (q''0) and the window engine's buffers depend on it
  ctx->win_ready = false;
  std::fill(ctx->initialized.begin(), ctx->initialized.end(), 0);
  return OSAM_OK;
}

int32_t osam_get_opinf_cubic(osam_ctx *c, int32_t sdi, double *C3) {
  if (!c || !C3) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  if (sdi < 0 || sdi >= (int)ctx->sds.size()) return ctx->fail(OSAM_E_INVALID, "bad subdomain id");
  const Subdomain &s = *ctx->sds[sdi];
  if (!s.rom) return ctx->fail(OSAM_E_INVALID, "not an OpInf subdomain");
  const long long r = s.r, r3 = r * (r + 1) * (r + 2) / 6;
  if (s.oh.C3.empty()) std::fill(C3, C3 + (size_t)r * r3, 0.0);
  else std::copy(s.oh.C3.begin(), s.oh.C3.end(), C3);
  return OSAM_OK;
}

int32_t schwarz_step(osam_ctx *c, const osam_schwarz_opts *opts, osam_instance_info *info) {
  if (!c || !opts) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  return ctx->run(1, *opts, info, /*host_sweeps=*/true);
}

int32_t run(osam_ctx *c, int64_t n_steps, const osam_schwarz_opts *opts, osam_instance_info *info) {
  if (!c || !opts || n_steps < 0) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  return ctx->run(n_steps, *opts, info);
}

int32_t osam_set_timing(osam_ctx *c, int32_t enable) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->timing = enable != 0;
  ctx->ev_used.clear();
  ctx->ev_next = 0;
  return OSAM_OK;
}

int32_t osam_get_timing(osam_ctx *c, int32_t sd, double *ms, int64_t *launches) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  if (sd < 0 || sd >= (int)ctx->sds.size()) return ctx->fail(OSAM_E_INVALID, "bad subdomain id");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  double tot = 0.0;
  int64_t n = 0;
  for (auto &u : ctx->ev_used) {
    if (u.first != sd) continue;
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, ctx->ev_pool[u.second.first], ctx->ev_pool[u.second.second]));
    tot += t;
    ++n;
  }
  if (ms) *ms = tot;
  if (launches) *launches = n;
  return OSAM_OK;
}

int32_t osam_set_reduced(osam_ctx *c, int32_t sdi, int32_t inst, const double *q0, const double *qd0) {
  if (!c || !q0 || !qd0) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  if (sdi < 0 || sdi >= (int)ctx->sds.size()) return ctx->fail(OSAM_E_INVALID, "bad subdomain id");
  if (inst < 0 || inst >= ctx->batch) return ctx->fail(OSAM_E_INVALID, "bad instance");
  Subdomain &d = *ctx->sds[sdi];
  if (!d.rom) return ctx->fail(OSAM_E_INVALID, "not an OpInf subdomain");
  if (!ctx->initialized[inst] || !(ctx->h_status[inst].flags & kNeedInit) || (int)d.gh0.size() <= inst)
    return ctx->fail(OSAM_E_ORDER, "osam_set_reduced must follow osam_set_initial before any step");
  std::vector<double> q(q0, q0 + d.r), qd(qd0, qd0 + d.r);
  hipSetDevice(ctx->device);
  return ctx->rom_start(sdi, inst, q, qd);
}

int32_t osam_set_fe_launch(osam_ctx *c, int32_t sd, int32_t block, int32_t kc) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  if (sd < 0 || sd >= (int)ctx->sds.size()) return ctx->fail(OSAM_E_INVALID, "bad subdomain id");
  Subdomain &s = *ctx->sds[sd];
  if (s.rom) return ctx->fail(OSAM_E_INVALID, "not a FOM subdomain");
  if (!(block == 0 || block == 64 || block == 128 || block == 256 || block == 1024) || kc < 0)
    return ctx->fail(OSAM_E_INVALID, "block must be 0, 64, 128, 256 or 1024 and kc >= 0");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (!ctx->choose_fe_launch(s, block, kc))
    return ctx->fail(OSAM_E_INVALID, "the layer-staged variant needs FP32 and a cross-section that fits the LDS");
  return OSAM_OK;
}

int32_t osam_set_fe_xshare(osam_ctx *c, int32_t sd, int32_t enable) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  if (sd < 0 || sd >= (int)ctx->sds.size()) return ctx->fail(OSAM_E_INVALID, "bad subdomain id");
  Subdomain &s = *ctx->sds[sd];
  if (s.rom) return ctx->fail(OSAM_E_INVALID, "not a FOM subdomain");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  s.fe_xs = enable != 0;
  if (!ctx->choose_fe_launch(s, s.fe_block, s.fe_kc)) return ctx->fail(OSAM_E_INVALID, "FE launch shape");
  return OSAM_OK;
}

int32_t osam_get_fe_launch(osam_ctx *c, int32_t sd, int32_t *block, int32_t *kc) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  if (sd < 0 || sd >= (int)ctx->sds.size()) return ctx->fail(OSAM_E_INVALID, "bad subdomain id");
  const Subdomain &s = *ctx->sds[sd];
  if (block) *block = s.fe_block;
  if (kc) *kc = s.fe_kc;
  return OSAM_OK;
}

int32_t osam_set_graph(osam_ctx *c, int32_t rounds, int32_t streams) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  if (rounds < 0 || rounds > 4096 || (rounds % 2) != 0 || streams < 1 || streams > 2)
    return ctx->fail(OSAM_E_INVALID, "graph rounds must be 0 or an even number up to 4096, streams 1 or 2");
  ctx->graph_rounds = rounds;
  ctx->graph_streams = streams;
  return OSAM_OK;
}

int32_t osam_set_fusion(osam_ctx *c, int32_t enable, int32_t kc) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  ctx->err.clear();
  if (kc < 0 || kc > 4096) return ctx->fail(OSAM_E_INVALID, "kc must be in 0 .. 4096");
  if (enable) {
    int nfe = 0, nrom = 0;
    for (const auto &d : ctx->sds) (d->rom ? nrom : nfe)++;
    if ((int)ctx->sds.size() > kSweepMax || nfe > kSweepFe || nrom > kSweepRom)
      return ctx->fail(OSAM_E_INVALID, "a fused sweep takes at most 4 subdomains, 3 of them FOM and 2 OpInf");
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->fuse = enable != 0;
  ctx->fuse_kc = kc > 0 ? kc : 1;
  return OSAM_OK;
}

int32_t osam_set_rom_path(osam_ctx *c, int32_t sd, int32_t path) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  if (sd < 0 || sd >= (int)ctx->sds.size() || path < 0 || path > 2)
    return ctx->fail(OSAM_E_INVALID, "bad subdomain id or path");
  Subdomain &s = *ctx->sds[sd];
  s.rom_path = path;
  if (ctx->wired && s.rom) return ctx->setup_pre(s);
  return OSAM_OK;
}

int32_t osam_get_rom_path(osam_ctx *c, int32_t sd, int32_t *path) {
  if (!c || !path) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  if (sd < 0 || sd >= (int)ctx->sds.size()) return ctx->fail(OSAM_E_INVALID, "bad subdomain id");
  int32_t st = ctx->wire();
  if (st) return st;
  const Subdomain &s = *ctx->sds[sd];
  *path = !s.rom ? 0 : (s.pre ? 2 : 1);
  return OSAM_OK;
}

int32_t osam_sync(osam_ctx *c) {
  if (!c) return OSAM_E_INVALID;
  Ctx *ctx = reinterpret_cast<Ctx *>(c);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return OSAM_OK;
}

}  // extern "C"
