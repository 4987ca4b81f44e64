// Host-side controller of libosam: coupling set-up (pointwise projections,
// Sec. 4.1), wiring of FOM/OpInf transfers (Sec. 4.2), initial states, and the
// device-paced Schwarz time loop (Alg. 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "persist.hpp"
#include "runtime.hpp"

namespace osam {

template <typename T>
hipError_t launch_fe(const FeArgs<T> &, int, int, int, hipStream_t, hipEvent_t = nullptr, hipEvent_t = nullptr);
template <typename T>
hipError_t launch_rom(const RomArgs<T> &, int, hipStream_t, hipEvent_t = nullptr, hipEvent_t = nullptr);
hipError_t launch_finish(const Status *, Status *, const FinishArgs &, const Opts &, int, hipStream_t);
template <typename T>
size_t rom_smem_bytes(int, int, int);
template <typename T>
hipError_t launch_sweep(const SweepArgs<T> &, int, bool, size_t, hipStream_t, hipEvent_t, hipEvent_t);
template <typename T>
hipError_t launch_project(const T *, long long, long long, const T *, long long, long long, double *, int,
                          int, hipStream_t);
template <typename T>
hipError_t launch_lift(const T *, long long, long long, int, const T *, T *, long long, long long, hipStream_t);

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(OSAM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

double *Ctx::scratch(size_t n, int32_t *st) {
  if (n > scratch_n) {
    dfree(d_scratch);
    d_scratch = static_cast<double *>(arena_alloc(n * sizeof(double), st));
    scratch_n = d_scratch ? n : 0;
    if (!d_scratch) return nullptr;
  }
  return d_scratch;
}

// Launch shape of the FE kernel: waves x instances.  block/kc = 0 selects the
// default (256 threads, one layer per thread).  The column kernel packs waves
// in super-chunks of bl chunks of kc layers: per chunk ceil(n_int / 64)
// interior waves, and per boundary case group of n columns either ceil(n / 64)
// waves per chunk (n >= 64) or one wave per min(64 / n, bl) chunks.  FE launches
// use bl = 1; fused sweeps bl = 2 (fewer workgroups, so that they fit in one
// round next to the OpInf workgroups).
constexpr int kFusedBndChunks = 2;
static int fe_bnd_waves(const Subdomain &s, int chunks, int bl) {
  int w = 0;
  for (int g = 0; g < s.nbg; ++g) {
    const int n = s.bg_n[g], L = std::min(64 / std::max(n, 1), bl);
    w += n >= 64 ? (n + 63) / 64 * chunks : (chunks + L - 1) / L;
  }
  return w;
}
static int fe_waves_in(const Subdomain &s, int chunks, int wi, int bl) {
  const int nsc = (chunks + bl - 1) / bl, last = chunks - (nsc - 1) * bl;
  return (nsc - 1) * (wi * bl + fe_bnd_waves(s, bl, bl)) + wi * last + fe_bnd_waves(s, last, bl);
}
static int fe_interior_waves(const Subdomain &s, bool xs) {   // per chunk
  return xs ? ((s.ny - 1) * (s.nx + 1) + 61) / 62 : (s.n_int + 63) / 64;
}
static int fe_waves(const Subdomain &s, int kc, int bl = 1) {
  return fe_waves_in(s, (s.nzs - 1 + kc - 1) / kc, fe_interior_waves(s, s.fe_xs), bl);
}

bool Ctx::choose_fe_launch(Subdomain &s, int block, int kc) {
  const int nl = s.nzs - 1;
  // bound on the workgroups of any shape, with either interior layout
  s.max_nblocks = std::max(s.max_nblocks, fe_waves_in(s, nl, std::max(fe_interior_waves(s, false),
                                                                      fe_interior_waves(s, true)), 1) + nl);
  if (block == 1024) {
    // layer-staged interior + column kernel for the boundary (FP32, cross-section fits the LDS)
    if (prec == OSAM_FP64 || s.npl > kFeLdsMaxNodes) return false;
    if (kc <= 0) kc = 8;
    kc = std::max(1, std::min(kc, nl));
    s.fe_block = 1024;
    s.fe_kc = kc;
    s.fe_chunks = (nl + kc - 1) / kc;
    s.fe_nblocks = s.fe_chunks + fe_waves_in(s, nl, 0, 1);   // + the boundary launch
    return true;
  }
  int bs = block > 0 ? block : 256;
  if (kc <= 0) kc = 1;   // one node layer per thread: a single memory round trip
  kc = std::max(1, std::min(kc, nl));
  s.fe_block = bs;
  s.fe_kc = kc;
  s.fe_chunks = (nl + kc - 1) / kc;
  s.fe_nblocks = (fe_waves(s, kc) + bs / 64 - 1) / (bs / 64);
  return true;
}

// ---------------------------------------------------------------------------
// Pointwise projection Pi (Sec. 4.1): trilinear interpolation of the source's
// FE field at every node of a Schwarz face.  Reference coordinates on a box
// grid follow from the cell index; values within 1e-9 of a grid line snap to it
// so that conforming faces become exact injections.
static void locate(double f, int n, int &i, double &t) {
  i = (int)std::floor(f);
  i = std::max(0, std::min(n - 1, i));
  t = f - i;
  if (std::fabs(t) < 1e-9) t = 0.0;
  if (std::fabs(t - 1.0) < 1e-9) t = 1.0;
}

int32_t Ctx::couple() {
  if (coupled) return OSAM_OK;
  const int S = (int)sds.size();
  for (int i = 0; i < S; ++i) {
    Subdomain &d = *sds[i];
    for (int f = 0; f < 2; ++f) {
      if (d.face_type[f] == kFaceClamped) continue;
      const int layer = f == 0 ? d.desc.z_lo : d.desc.z_hi;
      int src = -1;
      for (int j = 0; j < S && src < 0; ++j)
        if (j != i && sds[j]->desc.z_lo < layer && layer < sds[j]->desc.z_hi) src = j;
      if (src < 0) return fail(OSAM_E_OUTSIDE, "Schwarz face of subdomain " + std::to_string(i) +
                                                   " lies in no other subdomain");
      const Subdomain &sj = *sds[src];
      const osam_subdomain_desc &g = sj.desc;
      const double hx = g.Lx / g.nx, hy = g.Ly / g.ny, hz = g.Lz / g.nz;
      const double z = layer * (d.desc.Lz / d.desc.nz);
      FaceProj &P = d.proj[f];
      P.src = src;
      std::vector<std::vector<std::pair<int, double>>> rows(d.npl);
      int width = 1;
      for (int iy = 0; iy <= d.ny; ++iy)
        for (int ix = 0; ix <= d.nx; ++ix) {
          const double x = ix * (d.desc.Lx / d.nx), y = iy * (d.desc.Ly / d.ny);
          int ci, cj, ck;
          double tx, ty, tz;
          locate(x / hx, g.nx, ci, tx);
          locate(y / hy, g.ny, cj, ty);
          locate(z / hz - g.z_lo, sj.nzs, ck, tz);
          auto &row = rows[ix + (d.nx + 1) * iy];
          for (int c = 0; c < 8; ++c) {
            const int ox = c & 1, oy = (c >> 1) & 1, oz = (c >> 2) & 1;
            const double w = (ox ? tx : 1 - tx) * (oy ? ty : 1 - ty) * (oz ? tz : 1 - tz);
            if (w == 0.0) continue;
            const int kk = ck + oz;
            if (kk < 1 || kk > sj.nzs - 1)
              return fail(OSAM_E_OUTSIDE, "projection touches a constrained node of the source");
            row.push_back({(ci + ox) + (g.nx + 1) * ((cj + oy) + (g.ny + 1) * kk), w});
          }
          width = std::max(width, (int)row.size());
        }
      P.width = width;
      P.idx.assign((size_t)d.npl * width, 0);
      P.wt.assign((size_t)d.npl * width, 0.0);
      for (int n = 0; n < d.npl; ++n)
        for (size_t w = 0; w < rows[n].size(); ++w) {
          P.idx[(size_t)n * width + w] = rows[n][w].first;
          P.wt[(size_t)n * width + w] = rows[n][w].second;
        }
      // conforming slabs: the projection must be the injection node -> node
      P.src_layer = layer - g.z_lo;
      for (int n = 0; n < d.npl; ++n)
        if (width != 1 || P.wt[n] != 1.0 || P.idx[n] != n + P.src_layer * sj.npl)
          return fail(OSAM_E_INVALID, "non-conforming Schwarz faces are not supported");
    }
  }
  HIPCHK(hipStreamSynchronize(stream));
  coupled = true;
  wired = false;
  return OSAM_OK;
}

// ---------------------------------------------------------------------------
// Wiring: face-value buffers of OpInf subdomains fed by a FOM, Phi_S face
// blocks and ROM-to-ROM transfer matrices, Pi Phi export rows.
// Batched OpInf path (FP32 contexts, rom_pre_kernels.hip), chosen per subdomain:
// always in the BF16-H precision, on request, or automatically for batches of
// 8 and more or a compressed quadratic width of 1024 and more.  Builds A (FP32)
// and H (FP32, or BF16 in the BF16-H precision) in MFMA fragment order, the
// quadratic pair table and the partial-sum buffers.
static uint16_t bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

int32_t Ctx::setup_pre(Subdomain &d) {
  HIPCHK(hipStreamSynchronize(stream));
  void *old[] = {d.pre_fa, d.pre_fh, d.pre_blocks, d.pre_f0, d.pre_g};
  for (void *p : old) dfree(p);
  d.pre_fa = nullptr;
  d.pre_fh = nullptr;
  d.pre_blocks = nullptr;
  d.pre_f0 = nullptr;
  d.pre_g = nullptr;
  d.pre = false;
  if (!d.rom) return OSAM_OK;
  const int r = d.r, rs = d.rs, r2 = d.oh.quadratic ? r * (r + 1) / 2 : 0;
  const bool bf16 = prec == OSAM_FP32_BF16H;
  const bool want = prec != OSAM_FP64 && r <= 256 && rs <= 512 &&
                    (bf16 || d.rom_path == 2 || (d.rom_path == 0 && (batch >= 8 || r2 >= 1024)));
  if (!want) return OSAM_OK;
  d.pre_prec = bf16 ? 1 : 0;
  d.pre_nrt = (r + 15) / 16;
  d.pre_nkba = (r + 3) / 4;
  // H's K blocks: row i of the compressed triangle (columns j = i .. r-1) cut
  // into blocks of kw columns, the last one zero-padded
  const int kw = bf16 ? 16 : 4;
  std::vector<int> blk;
  for (int i = 0; i < r && r2 > 0; ++i)
    for (int j0 = i; j0 < r; j0 += kw) blk.push_back(i | (j0 << 16));
  d.pre_nkbh = (int)blk.size();
  const int nit = (batch + 15) / 16, nkb = d.pre_nkba + d.pre_nkbh;
  d.pre_ni = nit >= 4 ? 4 : (nit >= 2 ? 2 : 1);
  const int ngrp = (nit + d.pre_ni - 1) / d.pre_ni;
  // K splits: about 512 workgroups, at most 16 partial sums for the step kernel to add
  d.pre_ks = std::max(1, std::min({16, (512 + d.pre_nrt * ngrp - 1) / (d.pre_nrt * ngrp), std::max(1, nkb / 16)}));
  auto Aij = [&](int i, int k) -> double { return i < r && k < r ? d.oh.A[(size_t)k * r + i] : 0.0; };
  // H[i][m(a, b)], m(a, b) = a r - a (a - 1) / 2 + (b - a): compressed index of q_a q_b (a <= b)
  auto Hab = [&](int i, int a, int b) -> double {
    if (i >= r || b >= r) return 0.0;
    const size_t m = (size_t)a * r - (size_t)a * (a - 1) / 2 + (b - a);
    return d.oh.H[m * r + i];
  };
  int32_t st = OSAM_OK;
  // lane l of the 16x16x4 block (rt, kb) holds M[16 rt + l % 16][4 kb + l / 16]
  {
    std::vector<float> fa((size_t)d.pre_nrt * d.pre_nkba * 64);
    for (int rt = 0; rt < d.pre_nrt; ++rt)
      for (int kb = 0; kb < d.pre_nkba; ++kb)
        for (int l = 0; l < 64; ++l)
          fa[((size_t)rt * d.pre_nkba + kb) * 64 + l] = (float)Aij(rt * 16 + l % 16, kb * 4 + l / 16);
    d.pre_fa = static_cast<float *>(arena_alloc(fa.size() * 4, &st));
    if (st) return fail(st, "out of device memory");
    HIPCHK(hipMemcpy(d.pre_fa, fa.data(), fa.size() * 4, hipMemcpyHostToDevice));
  }
  if (r2 > 0 && !bf16) {
    // lane l of H block (rt, kb) = (i, j0): H[16 rt + l % 16][m(i, j0 + l / 16)]
    std::vector<float> fh((size_t)d.pre_nrt * d.pre_nkbh * 64);
    for (int rt = 0; rt < d.pre_nrt; ++rt)
      for (int kb = 0; kb < d.pre_nkbh; ++kb) {
        const int i = blk[kb] & 0xffff, j0 = blk[kb] >> 16;
        for (int l = 0; l < 64; ++l)
          fh[((size_t)rt * d.pre_nkbh + kb) * 64 + l] = (float)Hab(rt * 16 + l % 16, i, j0 + l / 16);
      }
    d.pre_fh = arena_alloc(fh.size() * 4, &st);
    if (st) return fail(st, "out of device memory");
    HIPCHK(hipMemcpy(d.pre_fh, fh.data(), fh.size() * 4, hipMemcpyHostToDevice));
  } else if (r2 > 0) {
    // lane l of the 16x16x16 block (rt, kb) = (i, j0): H[16 rt + l % 16][m(i, j0 + 4 (l / 16) + j)], j < 4
    std::vector<uint16_t> fh((size_t)d.pre_nrt * d.pre_nkbh * 64 * 4);
    for (int rt = 0; rt < d.pre_nrt; ++rt)
      for (int kb = 0; kb < d.pre_nkbh; ++kb) {
        const int i = blk[kb] & 0xffff, j0 = blk[kb] >> 16;
        for (int l = 0; l < 64; ++l)
          for (int j = 0; j < 4; ++j)
            fh[(((size_t)rt * d.pre_nkbh + kb) * 64 + l) * 4 + j] =
                bf16_rne((float)Hab(rt * 16 + l % 16, i, j0 + 4 * (l / 16) + j));
      }
    d.pre_fh = arena_alloc(fh.size() * 2, &st);
    if (st) return fail(st, "out of device memory");
    HIPCHK(hipMemcpy(d.pre_fh, fh.data(), fh.size() * 2, hipMemcpyHostToDevice));
  }
  if (blk.empty()) blk.push_back(0);
  d.pre_blocks = static_cast<int *>(arena_alloc(blk.size() * sizeof(int), &st));
  d.pre_f0 = static_cast<float *>(arena_alloc((size_t)d.pre_ks * batch * r * sizeof(float), &st));
  long long nfd = 0;
  for (int f = 0; f < 2; ++f)
    if (d.face_type[f] != kFaceClamped && !sds[d.proj[f].src]->rom) nfd += 3LL * d.npl;
  d.pre_gs = nfd > 0 && rs > 0 ? (int)std::max(1LL, std::min(64LL, (nfd + 2047) / 2048)) : 0;
  if (d.pre_gs > 0) d.pre_g = static_cast<double *>(arena_alloc((size_t)d.pre_gs * batch * rs * sizeof(double), &st));
  if (st) return fail(st, "out of device memory");
  HIPCHK(hipMemcpy(d.pre_blocks, blk.data(), blk.size() * sizeof(int), hipMemcpyHostToDevice));
  d.pre = true;
  return OSAM_OK;
}

int32_t Ctx::wire() {
  if (wired) return OSAM_OK;
  int32_t st = OSAM_OK;
  const int S = (int)sds.size();
  for (int i = 0; i < S; ++i) {
    Subdomain &d = *sds[i];
    for (int f = 0; f < 2; ++f) {
      if (d.face_type[f] == kFaceClamped) continue;
      const Subdomain &src = *sds[d.proj[f].src];
      const int n = 3 * d.npl;
      if (d.rom && !src.rom && !d.sface[f][0]) {
        for (int k = 0; k < 3; ++k) {
          d.sface[f][k] = alloc_t((size_t)batch * n, &st);
          if (st) return fail(st, "oom");
          HIPCHK(hipMemsetAsync(d.sface[f][k], 0, (size_t)batch * n * esize(), stream));
        }
      }
      if (d.rom) {
        const long long off = f == 0 ? 0 : d.face_off_hi;
        const long long ns = 3 * d.nsch_nodes;
        // Phi_S block of this face: [rs][3 npl]
        std::vector<double> blk((size_t)d.rs * n);
        for (int k = 0; k < d.rs; ++k)
          for (int c = 0; c < 3; ++c)
            for (int nid = 0; nid < d.npl; ++nid)
              blk[(size_t)k * n + c * d.npl + nid] = d.oh.PhiS[(size_t)k * ns + c * d.nsch_nodes + off + nid];
        if (!d.face_phis[f]) {
          d.face_phis[f] = alloc_t(blk.size(), &st);
          if (st) return fail(st, "oom");
        }
        if ((st = upload(d.face_phis[f], blk.data(), blk.size()))) return st;
        if (src.rom) {
          // T = Phi_S,face^T (Pi Phi_src), [rs][r_src] row-major; Pi is the injection
          std::vector<double> rows;
          if ((st = phi_layer_rows(const_cast<Subdomain &>(src), d.proj[f].src_layer, rows))) return st;
          std::vector<double> tm((size_t)d.rs * src.r, 0.0);
          for (int j = 0; j < src.r; ++j)
            for (int m = 0; m < n; ++m) {
              const double pv = rows[(size_t)j * n + m];
              for (int k = 0; k < d.rs; ++k) tm[(size_t)k * src.r + j] += blk[(size_t)k * n + m] * pv;
            }
          if (!d.face_tm[f]) {
            d.face_tm[f] = alloc_t(tm.size(), &st);
            if (st) return fail(st, "oom");
          }
          if ((st = upload(d.face_tm[f], tm.data(), tm.size()))) return st;
        }
      }
    }
  }
  // exports: every FOM face fed by a ROM gets Pi Phi rows, stored at the source
  for (int j = 0; j < S; ++j) {
    Subdomain &s = *sds[j];
    if (!s.rom) continue;
    s.piphi_h.clear();
  }
  for (int i = 0; i < S; ++i) {
    Subdomain &d = *sds[i];
    if (d.rom) continue;
    for (int f = 0; f < 2; ++f) {
      if (d.face_type[f] == kFaceClamped) continue;
      Subdomain &src = *sds[d.proj[f].src];
      if (!src.rom) continue;
      std::vector<double> pp;
      if ((st = phi_layer_rows(src, d.proj[f].src_layer, pp))) return st;
      src.piphi_h.push_back(pp);
    }
  }
  // device copies of the export rows (order: FOM subdomains ascending, low face first)
  for (int j = 0; j < S; ++j) {
    Subdomain &s = *sds[j];
    if (!s.rom) continue;
    s.piphi_d.clear();
    s.piphi_rm.clear();
    const int r4 = (s.r + 3) / 4 * 4;
    for (auto &pp : s.piphi_h) {
      void *p = alloc_t(pp.size(), &st);
      if (st) return fail(st, "oom");
      if ((st = upload(p, pp.data(), pp.size()))) return st;
      s.piphi_d.push_back(p);
      // row-major copy [n][r4] (zero-padded): one thread's row in 16-byte loads
      const size_t n = pp.size() / (size_t)s.r;
      std::vector<double> rm(n * r4, 0.0);
      for (size_t m = 0; m < n; ++m)
        for (int k = 0; k < s.r; ++k) rm[m * r4 + k] = pp[(size_t)k * n + m];
      void *q = alloc_t(rm.size(), &st);
      if (st) return fail(st, "oom");
      if ((st = upload(q, rm.data(), rm.size()))) return st;
      s.piphi_rm.push_back(q);
    }
  }
  // FOM state buffers only for FOM subdomains
  for (int i = 0; i < S; ++i) {
    Subdomain &d = *sds[i];
    const size_t nb = (size_t)batch * d.is;
    if (!d.rom && !d.u[0]) {
      for (int k = 0; k < 3; ++k) {
        d.u[k] = alloc_t(nb, &st);
        if (st) return fail(st, "out of device memory for FOM state");
        HIPCHK(hipMemsetAsync(d.u[k], 0, nb * esize(), stream));
      }
      for (int k = 0; k < 2; ++k) {
        d.v[k] = alloc_t(nb, &st);
        d.a[k] = alloc_t(nb, &st);
        if (st) return fail(st, "out of device memory for FOM state");
        HIPCHK(hipMemsetAsync(d.v[k], 0, nb * esize(), stream));
        HIPCHK(hipMemsetAsync(d.a[k], 0, nb * esize(), stream));
      }
    }
  }
  HIPCHK(hipStreamSynchronize(stream));
  for (int i = 0; i < S; ++i)
    if (sds[i]->rom && (st = setup_pre(*sds[i]))) return st;
  wired = true;
  return OSAM_OK;
}

// ---------------------------------------------------------------------------
int32_t Ctx::sync_status() {
  HIPCHK(hipMemcpyAsync(h_status, d_status, sizeof(Status) * batch, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  return OSAM_OK;
}

static void kron2_host(const std::vector<double> &q, std::vector<double> &k) {
  const int r = (int)q.size();
  k.clear();
  for (int i = 0; i < r; ++i)
    for (int j = i; j < r; ++j) k.push_back(q[i] * q[j]);
}

// Reduced initial state of OpInf subdomain i, instance inst: q0, q'0 given,
// q''0 = f(q0, g^0) with the stored g^0, the first recorded column, and the
// FOM neighbours' faces at t_1 = (Pi Phi) of the reduced predictor.
int32_t Ctx::rom_start(int i, int inst, const std::vector<double> &q, const std::vector<double> &qd) {
  Subdomain &d = *sds[i];
  int32_t st = OSAM_OK;
  const std::vector<double> &gh = d.gh0[inst];
  std::vector<double> qdd(d.r, 0.0), k2;
  kron2_host(q, k2);
  const int r2 = d.r * (d.r + 1) / 2;
  for (int i2 = 0; i2 < d.r; ++i2) {
    double s = d.oh.c.empty() ? 0.0 : d.oh.c[i2];
    for (int j = 0; j < d.r; ++j) s += d.oh.A[(size_t)j * d.r + i2] * q[j];
    if (d.oh.quadratic)
      for (int m = 0; m < r2; ++m) s += d.oh.H[(size_t)m * d.r + i2] * k2[m];
    if (!d.oh.C3.empty()) {
      // cubic term: q_a q_b q_c, a <= b <= c, lexicographic
      size_t m = 0;
      for (int a = 0; a < d.r; ++a)
        for (int b = a; b < d.r; ++b)
          for (int cc = b; cc < d.r; ++cc, ++m) s += d.oh.C3[m * d.r + i2] * q[a] * q[b] * q[cc];
    }
    for (int l = 0; l < d.rs; ++l) s += d.oh.B[(size_t)l * d.r + i2] * gh[l];
    qdd[i2] = s;
  }
  const size_t off = (size_t)inst * d.r * esize();
  if ((st = upload((char *)d.q[0] + off, q.data(), d.r))) return st;
  if ((st = upload((char *)d.qd[0] + off, qd.data(), d.r))) return st;
  if ((st = upload((char *)d.qdd[0] + off, qdd.data(), d.r))) return st;
  if (d.rec.every > 0 && d.rec.u && d.rec.n_cols > 0) {
    if ((st = upload((char *)d.rec.u + (size_t)inst * d.rec.n_cols * d.r * esize(), q.data(), d.r))) return st;
  }
  std::vector<double> q1(d.r);
  for (int k = 0; k < d.r; ++k) q1[k] = q[k] + d.desc.dt * qd[k] + 0.5 * d.desc.dt * d.desc.dt * qdd[k];
  // the predictor as the step kernel forms it: in the context precision, fma(h, q'', fma(dt, q', q))
  {
    std::vector<double> qp(d.r);
    for (int k = 0; k < d.r; ++k) {
      if (prec == OSAM_FP64) {
        qp[k] = std::fma(0.5 * d.desc.dt * d.desc.dt, qdd[k], std::fma(d.desc.dt, qd[k], q[k]));
      } else {
        const float h = (float)(0.5 * d.desc.dt * d.desc.dt), dt = (float)d.desc.dt;
        qp[k] = (double)std::fma(h, (float)qdd[k], std::fma(dt, (float)qd[k], (float)q[k]));
      }
    }
    if ((st = upload((char *)d.qpred + off, qp.data(), d.r))) return st;
  }
  int e = 0;
  for (size_t i2 = 0; i2 < sds.size(); ++i2) {
    Subdomain &fd = *sds[i2];
    if (fd.rom) continue;
    for (int f = 0; f < 2; ++f) {
      if (fd.face_type[f] == kFaceClamped || fd.proj[f].src != i) continue;
      const std::vector<double> &pp = d.piphi_h[e++];
      const int n = 3 * fd.npl;
      std::vector<double> sv(n, 0.0);
      for (int k = 0; k < d.r; ++k)
        for (int m = 0; m < n; ++m) sv[m] += pp[(size_t)k * n + m] * q1[k];
      const size_t lay = (size_t)(f == 0 ? 0 : fd.nzs) * fd.npl;
      for (int c = 0; c < 3; ++c) {
        const size_t o = ((size_t)inst * fd.is + (size_t)c * fd.cs + lay) * esize();
        if ((st = upload((char *)fd.u[1] + o, sv.data() + (size_t)c * fd.npl, fd.npl))) return st;
      }
    }
  }
  return OSAM_OK;
}

int32_t Ctx::set_initial(int inst, const double *u0g, const double *v0g) {
  int32_t st = wire();
  if (st) return st;
  st = sync_status();
  if (st) return st;
  const osam_subdomain_desc &g0 = sds[0]->desc;
  const long long nxp = g0.nx + 1, nyp = g0.ny + 1;
  const long long ng = nxp * nyp * (g0.nz + 1);
  for (size_t i = 0; i < sds.size(); ++i) {
    Subdomain &d = *sds[i];
    std::vector<double> u((size_t)3 * d.cs, 0.0), v((size_t)3 * d.cs, 0.0);
    for (int kl = 0; kl <= d.nzs; ++kl) {
      const bool clamped = (kl == 0 && d.face_type[0] == kFaceClamped) ||
                           (kl == d.nzs && d.face_type[1] == kFaceClamped);
      const bool face = kl == 0 || kl == d.nzs;
      for (int nid = 0; nid < d.npl; ++nid) {
        const long long gid = nid + nxp * nyp * (kl + d.desc.z_lo);
        const int ix = nid % (int)nxp, iy = nid / (int)nxp;
        const bool lateral = ix == 0 || ix == g0.nx || iy == 0 || iy == g0.ny;
        for (int c = 0; c < 3; ++c) {
          const size_t li = (size_t)c * d.cs + (size_t)kl * d.npl + nid;
          // held lateral components are zero on free layers; Schwarz faces keep the IC
          const bool held = !face && lateral && (d.desc.lateral_fix & (1 << c));
          u[li] = clamped || held ? 0.0 : u0g[c * ng + gid];
          v[li] = face || held ? 0.0 : v0g[c * ng + gid];
        }
      }
    }
    if (!d.rom) {
      const size_t off = (size_t)inst * d.is * esize();
      if ((st = upload((char *)d.u[0] + off, u.data(), u.size()))) return st;
      if ((st = upload((char *)d.v[0] + off, v.data(), v.size()))) return st;
    } else {
      // q0 = Phi^T u0, q'0 = Phi^T v0 on free DOFs (device projection, FP64 sums)
      const int nchunks = 64;
      double *part = scratch((size_t)2 * d.r * nchunks + (size_t)3 * d.cs * 2, &st);
      if (st) return fail(st, "oom");
      void *fld = (char *)part + sizeof(double) * 2 * d.r * nchunks;
      std::vector<double> q(d.r), qd(d.r);
      for (int which = 0; which < 2; ++which) {
        if ((st = upload(fld, which == 0 ? u.data() : v.data(), u.size()))) return st;
        hipError_t e;
        if (prec == OSAM_FP64)
          e = launch_project<double>((const double *)d.d_Phi, 3 * d.nfree_nodes, d.nfree_nodes,
                                     (const double *)fld, d.cs, d.npl, part, nchunks, d.r, stream);
        else
          e = launch_project<float>((const float *)d.d_Phi, 3 * d.nfree_nodes, d.nfree_nodes,
                                    (const float *)fld, d.cs, d.npl, part, nchunks, d.r, stream);
        if (e != hipSuccess) return fail(OSAM_E_HIP, hipGetErrorString(e));
        std::vector<double> hp((size_t)d.r * nchunks);
        HIPCHK(hipMemcpyAsync(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        for (int k = 0; k < d.r; ++k) {
          double s = 0.0;
          for (int cch = 0; cch < nchunks; ++cch) s += hp[(size_t)k * nchunks + cch];
          (which == 0 ? q : qd)[k] = s;
        }
      }
      // g^0 = Phi_S^T s0 with s0 = IC on the Schwarz DOFs; q''0 = f(q0, g^0)
      const long long ns = 3 * d.nsch_nodes;
      std::vector<double> s0(ns, 0.0), gh(d.rs, 0.0);
      for (int c = 0; c < 3; ++c)
        for (int f = 0; f < 2; ++f) {
          if (d.face_type[f] == kFaceClamped) continue;
          const int kl = f == 0 ? 0 : d.nzs;
          const long long off = f == 0 ? 0 : d.face_off_hi;
          for (int nid = 0; nid < d.npl; ++nid)
            s0[c * d.nsch_nodes + off + nid] = u[(size_t)c * d.cs + (size_t)kl * d.npl + nid];
        }
      for (int k = 0; k < d.rs; ++k) {
        double s = 0.0;
        for (long long m = 0; m < ns; ++m) s += d.oh.PhiS[(size_t)k * ns + m] * s0[m];
        gh[k] = s;
      }
      if ((int)d.gh0.size() < batch) d.gh0.resize(batch);
      d.gh0[inst] = gh;
      if ((st = rom_start((int)i, inst, q, qd))) return st;
      // own faces fed by a FOM: role U0 (t_0) holds the IC
      for (int f = 0; f < 2; ++f) {
        if (!d.sface[f][0]) continue;
        const int kl = f == 0 ? 0 : d.nzs;
        std::vector<double> fv((size_t)3 * d.npl);
        for (int c = 0; c < 3; ++c)
          for (int nid = 0; nid < d.npl; ++nid)
            fv[(size_t)c * d.npl + nid] = u[(size_t)c * d.cs + (size_t)kl * d.npl + nid];
        if ((st = upload((char *)d.sface[f][0] + (size_t)inst * 3 * d.npl * esize(), fv.data(), fv.size())))
          return st;
      }
    }
  }
  Status &S = h_status[inst];
  std::memset(&S, 0, sizeof(Status));
  S.flags = kNeedInit;
  HIPCHK(hipMemcpyAsync(d_status + inst, &S, sizeof(Status), hipMemcpyHostToDevice, stream));
  HIPCHK(hipStreamSynchronize(stream));
  initialized[inst] = 1;
  return OSAM_OK;
}

// a0 = M^-1(-K u0) and the first predictor for instances flagged kNeedInit.
int32_t Ctx::init_pending() {
  bool any = false;
  for (int b = 0; b < batch; ++b) any |= (h_status[b].flags & kNeedInit) != 0;
  if (!any) return OSAM_OK;
  Opts o{};
  o.nsd = (int)sds.size();
  for (size_t i = 0; i < sds.size(); ++i)
    if (!sds[i]->rom) {
      int32_t st = launch_fe_sd((int)i, o, 1);
      if (st) return st;
    }
  int32_t st = sync_status();
  if (st) return st;
  for (int b = 0; b < batch; ++b) h_status[b].flags &= ~kNeedInit;
  HIPCHK(hipMemcpyAsync(d_status, h_status, sizeof(Status) * batch, hipMemcpyHostToDevice, stream));
  return OSAM_OK;
}

// ---------------------------------------------------------------------------
// What the decider of a sweep gathers: the FOM subdomains' partial sums and
// the OpInf subdomains (other than the last) whose sums are in the output status.
// defer: every OpInf kernel leaves its sums in the output status (graph mode)
// fused: the FOM partials come from the FE part of a fused sweep
static FinishArgs finish_args(Ctx &c, bool defer = false, bool fused = false) {
  FinishArgs F;
  std::memset(&F, 0, sizeof(F));
  const int last = (int)c.sds.size() - 1;
  for (int i = 0; i <= last; ++i) {
    const Subdomain &d = *c.sds[i];
    if (d.rom) {
      if (i != last || defer) F.rom_sd[F.nrom++] = i;
      continue;
    }
    F.sd[F.nfom] = i;
    F.nblocks[F.nfom] = fused ? d.fz_nblocks : d.fe_nblocks;
    F.part[F.nfom] = d.partials;
    ++F.nfom;
  }
  return F;
}

template <typename T>
static void fill_fe_args(Ctx &c, Subdomain &s, int sdi, const Opts &o, FeArgs<T> &A) {
  std::memset(&A, 0, sizeof(A));
  A.nx = s.nx;
  A.ny = s.ny;
  A.nzs = s.nzs;
  A.npl = s.npl;
  A.cs = s.cs;
  A.is = s.is;
  for (int k = 0; k < 3; ++k) A.u[k] = (T *)s.u[k];
  for (int k = 0; k < 2; ++k) {
    A.v[k] = (T *)s.v[k];
    A.a[k] = (T *)s.a[k];
  }
  A.coef = (const T *)s.coef;
  for (int i = 0; i < 27; ++i) A.cb[i] = (T)s.cb[i];
  A.dt = (T)s.desc.dt;
  A.half_dt = (T)(0.5 * s.desc.dt);
  A.half_dt2 = (T)(0.5 * s.desc.dt * s.desc.dt);
  for (int f = 0; f < 2; ++f) A.face_src[f] = s.face_type[f] == kFaceClamped ? -1 : s.proj[f].src;
  // pushes: every face of another subdomain whose source is this one
  A.npush = 0;
  for (size_t i = 0; i < c.sds.size(); ++i) {
    Subdomain &d = *c.sds[i];
    for (int f = 0; f < 2; ++f) {
      if (d.face_type[f] == kFaceClamped || d.proj[f].src != sdi) continue;
      PushDev<T> &Pd = A.push[A.npush++];
      Pd.layer = d.proj[f].src_layer;
      if (d.rom) {
        for (int k = 0; k < 3; ++k) Pd.role[k] = (T *)d.sface[f][k];
        Pd.cs = d.npl;
        Pd.is = 3LL * d.npl;
      } else {
        const long long lay = (long long)(f == 0 ? 0 : d.nzs) * d.npl;
        for (int k = 0; k < 3; ++k) Pd.role[k] = (T *)d.u[k] + lay;
        Pd.cs = d.cs;
        Pd.is = d.is;
      }
    }
  }
  A.status = c.d_status;
  A.sd = sdi;
  A.opts = o;
  A.skip_rows = s.desc.lateral_fix & 7;
  A.partials = s.partials;
  A.kc = s.fe_kc;
  A.n_chunks = s.fe_chunks;
  A.n_int = s.n_int;
  A.n_bnd = s.n_bnd;
  A.nblocks = s.fe_nblocks;
  A.part_stride = s.fe_nblocks;
  A.part_off = 0;
  A.bnd_cols = s.bnd_cols;
  A.nbg = s.nbg;
  A.xs = s.fe_xs ? 1 : 0;
  A.bnd_l = 1;
  for (int g = 0; g < 8; ++g) {
    A.bg_start[g] = s.bg_start[g];
    A.bg_n[g] = s.bg_n[g];
  }
  A.rec_u = (T *)s.rec.u;
  A.rec_a = (T *)s.rec.a;
  A.rec_s = (T *)s.rec.s;
  A.rec_every = s.rec.every;
  A.rec_ncols = s.rec.n_cols;
  A.nfree_nodes = s.nfree_nodes;
  A.nsch_nodes = s.nsch_nodes;
  A.face_off_hi = s.face_off_hi;
}

int32_t Ctx::launch_fe_sd(int sdi, const Opts &o, int mode, hipEvent_t ev0, hipEvent_t ev1, hipStream_t st) {
  Subdomain &s = *sds[sdi];
  hipError_t e;
  hipStream_t stream = st ? st : this->stream;
  if (prec == OSAM_FP64) {
    FeArgs<double> A;
    fill_fe_args<double>(*this, s, sdi, o, A);
    e = launch_fe<double>(A, batch, s.fe_block, mode, stream, ev0, ev1);
  } else {
    FeArgs<float> A;
    fill_fe_args<float>(*this, s, sdi, o, A);
    if (s.fe_block == 1024) {
      // interior: layer-staged workgroups (partials 0 .. fe_chunks-1); boundary: the
      // column kernel over the boundary blocks only (partials after those)
      FeArgs<float> Ab = A;
      A.nblocks = s.fe_chunks;
      e = launch_fe<float>(A, batch, 1024, mode, stream, ev0, nullptr);
      if (e == hipSuccess) {
        const int nl = s.nzs - 1;
        Ab.kc = 1;
        Ab.n_chunks = nl;
        Ab.n_int = 0;   // boundary groups only
        Ab.xs = 0;
        Ab.nblocks = fe_waves_in(s, nl, 0, 1);
        Ab.part_off = s.fe_chunks;
        e = launch_fe<float>(Ab, batch, 64, mode, stream, nullptr, ev1);
      }
    } else {
      e = launch_fe<float>(A, batch, s.fe_block, mode, stream, ev0, ev1);
    }
  }
  if (e != hipSuccess) return fail(OSAM_E_HIP, std::string("fe kernel: ") + hipGetErrorString(e));
  return OSAM_OK;
}

template <typename T>
static void fill_rom_args(Ctx &c, Subdomain &s, int sdi, const Opts &o, RomArgs<T> &A) {
  std::memset(&A, 0, sizeof(A));
  A.r = s.r;
  A.rs = s.rs;
  A.r2 = s.oh.quadratic ? s.r * (s.r + 1) / 2 : 0;
  A.A = (const T *)s.d_A;
  A.H = (const T *)s.d_H;
  A.B = s.rs > 0 ? (const T *)s.d_B : nullptr;
  A.c = (const T *)s.d_c;
  if (s.pre) {   // f0 (and the FOM-fed g^) arrive as partial sums
    A.A = nullptr;
    A.H = nullptr;
    A.c = nullptr;
    A.r2 = 0;
    A.f0part = (const T *)s.pre_f0;
    A.f0_ks = s.pre_ks;
    A.f0_stride = (long long)c.batch * s.r;
    A.gpart = s.pre_g;
    A.g_gs = s.pre_gs;
    A.g_stride = (long long)c.batch * s.rs;
  }
  A.qpred = (T *)s.qpred;
  for (int k = 0; k < 2; ++k) {
    A.q[k] = (T *)s.q[k];
    A.qd[k] = (T *)s.qd[k];
    A.qdd[k] = (T *)s.qdd[k];
  }
  A.dt = (T)s.desc.dt;
  A.half_dt = (T)(0.5 * s.desc.dt);
  A.half_dt2 = (T)(0.5 * s.desc.dt * s.desc.dt);
  int nf = 0;
  for (int f = 0; f < 2; ++f) {
    if (s.face_type[f] == kFaceClamped || s.rs == 0) continue;
    const FaceProj &P = s.proj[f];
    const Subdomain &src = *c.sds[P.src];
    if (s.pre_g && !src.rom) continue;   // summed by rom_ghat_kernel
    RomFaceIn<T> &F = A.fin[nf++];
    F.src_sd = P.src;
    F.n = 3 * s.npl;
    F.phis = (const T *)s.face_phis[f];
    if (src.rom) {
      F.type = 3;
      F.src_r = src.r;
      F.tm = (const T *)s.face_tm[f];
      for (int k = 0; k < 2; ++k) {
        F.src_q[k] = (T *)src.q[k];
        F.src_qd[k] = (const T *)src.qd[k];
        F.src_qdd[k] = (const T *)src.qdd[k];
      }
      F.src_dt = (T)src.desc.dt;
      F.src_half_dt2 = (T)(0.5 * src.desc.dt * src.desc.dt);
    } else {
      F.type = kFaceFom;
      for (int k = 0; k < 3; ++k) F.sface[k] = (const T *)s.sface[f][k];
    }
  }
  A.nfaces = nf;
  int ne = 0;
  for (size_t i = 0; i < c.sds.size(); ++i) {
    Subdomain &fd = *c.sds[i];
    if (fd.rom) continue;
    for (int f = 0; f < 2; ++f) {
      if (fd.face_type[f] == kFaceClamped || fd.proj[f].src != sdi) continue;
      RomExport<T> &E = A.ex[ne];
      const long long lay = (long long)(f == 0 ? 0 : fd.nzs) * fd.npl;
      for (int k = 0; k < 3; ++k) E.role[k] = (T *)fd.u[k] + lay;
      E.cs = fd.cs;
      E.is = fd.is;
      E.npl = fd.npl;
      E.prow = (const T *)s.piphi_rm[ne];
      E.r4 = (s.r + 3) / 4 * 4;
      ++ne;
    }
  }
  A.nexp = ne;
  A.status = c.d_status;
  A.status_out = c.d_status_alt;
  A.sd = sdi;
  A.opts = o;
  A.finish = finish_args(c);
  A.rec_q = (T *)s.rec.u;
  A.rec_every = s.rec.every;
  A.rec_ncols = s.rec.n_cols;
}

static void fill_pre_args(Ctx &c, Subdomain &s, int sdi, const Opts &o, RomPreArgs &P) {
  std::memset(&P, 0, sizeof(P));
  P.r = s.r;
  P.rs = s.rs;
  P.r2 = s.oh.quadratic ? s.r * (s.r + 1) / 2 : 0;
  P.batch = c.batch;
  P.prec = s.pre_prec;
  P.nkba = s.pre_nkba;
  P.nkbh = s.pre_nkbh;
  P.nrt = s.pre_nrt;
  P.ks = s.pre_ks;
  P.nit = (c.batch + 15) / 16;
  P.ni = s.pre_ni;
  P.frag_a = s.pre_fa;
  P.frag_h = s.pre_fh;
  P.blocks = s.pre_blocks;
  P.c = (const float *)s.d_c;
  P.qpred = (const float *)s.qpred;
  P.f0part = s.pre_f0;
  int nf = 0;
  for (int f = 0; f < 2 && s.pre_g; ++f) {
    if (s.face_type[f] == kFaceClamped || c.sds[s.proj[f].src]->rom) continue;
    P.fn[nf] = 3LL * s.npl;
    P.fsrc[nf] = s.proj[f].src;
    P.phis[nf] = (const float *)s.face_phis[f];
    for (int k = 0; k < 3; ++k) P.sface[nf][k] = (const float *)s.sface[f][k];
    ++nf;
  }
  P.nface = nf;
  P.gs = s.pre_gs;
  P.gpart = s.pre_g;
  P.status = c.d_status;
  P.sd = sdi;
  P.opts = o;
}

int32_t Ctx::launch_rom_sd(int sdi, const Opts &o, hipEvent_t ev0, hipEvent_t ev1, hipStream_t st, bool defer) {
  Subdomain &s = *sds[sdi];
  hipError_t e;
  hipStream_t stream = st ? st : this->stream;
  if (s.pre) {
    RomPreArgs P;
    fill_pre_args(*this, s, sdi, o, P);
    e = launch_rom_pre(P, stream);
    if (e != hipSuccess) return fail(OSAM_E_HIP, std::string("batched OpInf kernels: ") + hipGetErrorString(e));
  }
  if (prec == OSAM_FP64) {
    RomArgs<double> A;
    fill_rom_args<double>(*this, s, sdi, o, A);
    A.defer = defer;
    e = launch_rom<double>(A, batch, stream, ev0, ev1);
  } else {
    RomArgs<float> A;
    fill_rom_args<float>(*this, s, sdi, o, A);
    A.defer = defer;
    e = launch_rom<float>(A, batch, stream, ev0, ev1);
  }
  if (e != hipSuccess) return fail(OSAM_E_HIP, std::string("rom kernel: ") + hipGetErrorString(e));
  return OSAM_OK;
}

hipEvent_t Ctx::next_event() {
  if (ev_next == ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ev_pool.push_back(e);
  }
  return ev_pool[ev_next++];
}

int32_t Ctx::launch_round(const Opts &o) {
  for (size_t i = 0; i < sds.size(); ++i) {
    // timing: the events are stamped with the kernel's own start and end
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timing) {
      const int a = (int)ev_next;
      e0 = next_event();
      const int b = (int)ev_next;
      e1 = next_event();
      if (!e0 || !e1) return fail(OSAM_E_HIP, "event create");
      ev_used.push_back({(int)i, {a, b}});
    }
    int32_t st = sds[i]->rom ? launch_rom_sd((int)i, o, e0, e1) : launch_fe_sd((int)i, o, 0, e0, e1);
    if (st) return st;
  }
  // a ROM kernel that ends the sweep takes the decision itself
  if (!sds.back()->rom) {
    const hipError_t e = launch_finish(d_status, d_status_alt, finish_args(*this), o, batch, stream);
    if (e != hipSuccess) return fail(OSAM_E_HIP, std::string("finish kernel: ") + hipGetErrorString(e));
  }
  // the decider wrote the other buffer: it is the input of the next round
  std::swap(d_status, d_status_alt);
  return OSAM_OK;
}

// One Schwarz sweep with the FOM kernels on the context stream and the OpInf
// kernels on the auxiliary stream.  Within a sweep no kernel reads what another
// writes: every source pushes its next-step displacement into the role of the
// next step, which no kernel of the sweep reads, so the two streams only meet
// at the finisher, which takes the decision of Eq. conv_criterion.
int32_t Ctx::launch_round_concurrent(const Opts &o) {
  bool any_rom = false;
  for (auto &d : sds) any_rom |= d->rom;
  if (any_rom) {
    HIPCHK(hipEventRecord(fork_ev, stream));
    HIPCHK(hipStreamWaitEvent(aux, fork_ev, 0));
  }
  int32_t st;
  for (size_t i = 0; i < sds.size(); ++i)
    if (!sds[i]->rom && (st = launch_fe_sd((int)i, o, 0))) return st;
  for (size_t i = 0; i < sds.size(); ++i)
    if (sds[i]->rom && (st = launch_rom_sd((int)i, o, nullptr, nullptr, aux, true))) return st;
  if (any_rom) {
    HIPCHK(hipEventRecord(join_ev, aux));
    HIPCHK(hipStreamWaitEvent(stream, join_ev, 0));
  }
  const hipError_t e = launch_finish(d_status, d_status_alt, finish_args(*this, true), o, batch, stream);
  if (e != hipSuccess) return fail(OSAM_E_HIP, std::string("finish kernel: ") + hipGetErrorString(e));
  std::swap(d_status, d_status_alt);
  return OSAM_OK;
}

// ---------------------------------------------------------------------------
// Fused sweeps.  Every FOM step runs as the column kernel with 512-thread
// workgroups (the OpInf step's workgroup size), fuse_kc layers per thread.
void Ctx::fuse_layout(Subdomain &s) {
  const int nl = s.nzs - 1;
  s.fz_kc = std::max(1, std::min(fuse_kc, nl));
  s.fz_chunks = (nl + s.fz_kc - 1) / s.fz_kc;
  // (x-shared interior rows with one layer per thread, else the plain layout); 8 waves per
  // workgroup; <= max_nblocks
  s.fz_nblocks = (fe_waves_in(s, s.fz_chunks, fe_interior_waves(s, s.fz_kc == 1 && s.fe_xs), kFusedBndChunks) + 7) / 8;
}

std::string Ctx::fusion_unsupported() const {
  int nfe = 0, nrom = 0;
  for (const auto &d : sds) {
    if (d->rom) {
      ++nrom;
      const size_t smem = prec == OSAM_FP64
                              ? rom_smem_bytes<double>(d->r, d->rs, d->oh.quadratic ? d->r * (d->r + 1) / 2 : 0)
                              : rom_smem_bytes<float>(d->r, d->rs,
                                                      d->oh.quadratic && !d->pre ? d->r * (d->r + 1) / 2 : 0);
      if (smem > 65536) return "an OpInf subdomain's step needs more than 64 KB of LDS";
    } else {
      ++nfe;
    }
  }
  if ((int)sds.size() > kSweepMax || nfe > kSweepFe || nrom > kSweepRom)
    return "a fused sweep takes at most 4 subdomains, 3 of them FOM and 2 OpInf";
  return "";
}

// fold: take the previous sweep's decision in this sweep's workgroups (its partials and
// OpInf sums in parity 1 - par); par: the parity of the buffers this sweep writes them to.
// sums: the OpInf steps leave their sums in rom_sums (parity par) rather than in the output
// status (the sweeps of a graph with folded decisions).
template <typename T>
static int32_t fused_sweep(Ctx &c, const Opts &o, hipEvent_t ev0, hipEvent_t ev1, bool fold, int par, bool sums) {
  SweepArgs<T> S;
  std::memset(&S, 0, sizeof(S));
  S.n = (int)c.sds.size();
  S.opts = o;
  if (fold) {
    S.fold = 1;
    S.prev = c.fused_finish_args(1 - par);
    S.st_prev = c.d_status;
    S.st_cur = c.d_status_alt;
  }
  int nfe = 0, nrom = 0;
  bool one = true;
  size_t smem = 0;
  // grid order: the OpInf steps (few workgroups, the longest chain of dependent
  // steps) first, so they are dispatched before the FE workgroups fill the chip
  std::vector<int> order;
  for (int pass = 0; pass < 2; ++pass)
    for (int i = 0; i < S.n; ++i)
      if (c.sds[i]->rom == (pass == 0)) order.push_back(i);
  for (int slot = 0; slot < S.n; ++slot) {
    const int i = order[slot];
    Subdomain &d = *c.sds[i];
    if (!d.rom) {
      FeArgs<T> &A = S.fe[nfe];
      fill_fe_args<T>(c, d, i, o, A);
      A.kc = d.fz_kc;
      A.n_chunks = d.fz_chunks;
      A.bnd_l = kFusedBndChunks;
      A.xs = d.fz_kc == 1 && d.fe_xs ? 1 : 0;   // the layout fuse_layout counted
      A.nblocks = d.fz_nblocks;
      A.part_stride = d.fz_nblocks;
      A.part_off = 0;
      A.partials = d.partials_of(par, c.batch);
      one = one && d.fz_kc == 1;
      S.nblk[slot] = d.fz_nblocks;
      S.fe_idx[slot] = nfe++;
      S.rom_idx[slot] = -1;
    } else {
      RomArgs<T> &A = S.rom[nrom];
      fill_rom_args<T>(c, d, i, o, A);
      A.defer = 1;
      if (sums) A.sums_out = c.rom_sums + (size_t)par * c.batch * kMaxSd * 2;
      // an OpInf source runs side by side with this step: take its predictor
      // from its accepted state (the value it writes in this sweep)
      for (int f = 0; f < A.nfaces; ++f)
        if (A.fin[f].type == 3) A.fin[f].pred = 1;
      int rows = 0;
      for (int e = 0; e < A.nexp; ++e) rows = std::max(rows, 3 * A.ex[e].npl);
      S.nblk[slot] = rows > 0 ? (rows + 511) / 512 : 1;
      S.fe_idx[slot] = -1;
      S.rom_idx[slot] = nrom++;
      smem = std::max(smem, rom_smem_bytes<T>(A.r, A.rs, A.r2));
    }
  }
  const hipError_t e = launch_sweep<T>(S, c.batch, one, smem, c.stream, ev0, ev1);
  if (e != hipSuccess) return c.fail(OSAM_E_HIP, std::string("sweep kernel: ") + hipGetErrorString(e));
  return OSAM_OK;
}

// One Schwarz sweep as one launch (after the batched OpInf parts), then the
// finisher.  Sources push into the next step's roles and write their sums to
// their own slots, so the subdomains' steps are independent within the sweep
// (an OpInf source's displacement is formed from its accepted state).
// The finisher's arguments for the partials and OpInf sums a fused sweep wrote to the
// buffers of parity par (graph mode with folded decisions).
FinishArgs Ctx::fused_finish_args(int par) {
  FinishArgs F = finish_args(*this, true, true);
  for (int k = 0; k < F.nfom; ++k) F.part[k] = sds[F.sd[k]]->partials_of(par, batch);
  F.rom_sums = rom_sums + (size_t)par * batch * kMaxSd * 2;
  return F;
}

// r, n: the sweep's place in a sequence of n sweeps launched back to back (a captured
// graph, or a chunk of eager launches).  Without batched OpInf parts, every sweep but the
// first takes the previous sweep's decision itself (SweepArgs), the buffers alternating by
// round parity, and only the last sweep is followed by the finisher.  Otherwise (and for
// n = 0) every sweep has its finisher.
int32_t Ctx::launch_round_fused(const Opts &o, long long r, long long n) {
  const std::string why = fusion_unsupported();
  if (!why.empty()) return fail(OSAM_E_INVALID, why);
  RomPreArgs pre[kSweepRom];
  int npre = 0;
  for (size_t i = 0; i < sds.size(); ++i) {
    Subdomain &d = *sds[i];
    if (!d.rom) fuse_layout(d);
    else if (d.pre) fill_pre_args(*this, d, (int)i, o, pre[npre++]);
  }
  if (npre > 0) {   // the batched parts of every OpInf subdomain, f0 in one launch
    const hipError_t e = launch_rom_pre_multi(pre, npre, stream);
    if (e != hipSuccess) return fail(OSAM_E_HIP, std::string("batched OpInf kernels: ") + hipGetErrorString(e));
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timing) {   // every subdomain reports the fused launch
    const int a = (int)ev_next;
    e0 = next_event();
    const int b = (int)ev_next;
    e1 = next_event();
    if (!e0 || !e1) return fail(OSAM_E_HIP, "event create");
    for (size_t i = 0; i < sds.size(); ++i) ev_used.push_back({(int)i, {a, b}});
  }
  const bool folding = n > 0 && npre == 0;
  const bool fold = folding && r > 0;
  const int par = folding ? (int)(r & 1) : 0;
  int32_t st = prec == OSAM_FP64 ? fused_sweep<double>(*this, o, e0, e1, fold, par, folding)
                                 : fused_sweep<float>(*this, o, e0, e1, fold, par, folding);
  if (st) return st;
  if (fold) std::swap(d_status, d_status_alt);   // the sweep stored the status it started from
  if (folding && r < n - 1) return OSAM_OK;
  const FinishArgs F = folding ? fused_finish_args(par) : finish_args(*this, true, true);
  const hipError_t e = launch_finish(d_status, d_status_alt, F, o, batch, stream);
  if (e != hipSuccess) return fail(OSAM_E_HIP, std::string("finish kernel: ") + hipGetErrorString(e));
  std::swap(d_status, d_status_alt);
  return OSAM_OK;
}

// ---------------------------------------------------------------------------
// Persistent OpInf engine (engine 2): every step of the call in one launch of
// rom_persist_kernel, one workgroup per instance (persist_kernels.hip).
std::string Ctx::persist_unsupported(const Opts &o) const {
  if ((int)sds.size() > kPersistMax) return "at most 4 subdomains";
  for (const auto &dp : sds) {
    const Subdomain &d = *dp;
    if (!d.rom) return "every subdomain must be an OpInf model";
    if (d.desc.beta != 0.0 || d.desc.gamma != 0.5 || d.n_sub > 1 || !d.oh.C3.empty())
      return "explicit single-step OpInf subdomains only (beta = 0, gamma = 1/2, n_sub = 1, no cubic term)";
    if (d.r > 128) return "r above 128";   // the OpInf step's rows: 8 waves x 16 rows
  }
  if (o.additive) return "the multiplicative variant only";
  return "";
}

template <typename T>
static int32_t persist_launch(Ctx &c, const Opts &o) {
  PersistArgs<T> P;
  std::memset(&P, 0, sizeof(P));
  P.nsd = (int)c.sds.size();
  P.status = c.d_status;
  P.opts = o;
  for (int i = 0; i < kMaxSd; ++i) P.slot[i] = 0;
  // state blocks, then the scratch shared by the subdomains, then operators while they fit
  long long off = 0;
  int max_rs = 1, max_r2 = 1, max_r = 1;
  for (int i = 0; i < P.nsd; ++i) {
    Subdomain &d = *c.sds[i];
    RomArgs<T> &A = P.sd[i];
    fill_rom_args<T>(c, d, i, o, A);
    // the whole step here: operators, not the batched parts
    A.A = (const T *)d.d_A;
    A.H = (const T *)d.d_H;
    A.c = (const T *)d.d_c;
    A.r2 = d.oh.quadratic ? d.r * (d.r + 1) / 2 : 0;
    A.f0part = nullptr;
    A.gpart = nullptr;
    P.slot[i] = i;
    PersistLayout &Y = P.lay[i];
    for (int p = 0; p < 2; ++p) {
      Y.q[p] = (int)off;
      off += d.r;
      Y.v[p] = (int)off;
      off += d.r;
      Y.a[p] = (int)off;
      off += d.r;
    }
    Y.q1 = (int)off;
    off += d.r;
    Y.qp = (int)off;
    off += d.r;
    Y.f0 = (int)off;
    off += d.r;
    Y.am = Y.h = Y.bm = Y.c = Y.tm[0] = Y.tm[1] = -1;
    max_rs = std::max(max_rs, d.rs);
    max_r2 = std::max(max_r2, A.r2);
    max_r = std::max(max_r, d.r);
  }
  P.sh_off = (int)off;
  off += max_rs;
  P.k2_off = (int)off;
  off += max_r2;
  P.rows_off = (int)off;
  off += max_r;
  const long long cap = (long long)(kPersistLds / sizeof(T));
  if (off > cap) return c.fail(OSAM_E_INVALID, "persistent OpInf engine: the reduced states exceed the LDS");
  auto place = [&](int &slot, long long n) {
    if (n > 0 && off + n <= cap) {
      slot = (int)off;
      off += n;
    }
  };
  // what every sweep reads (B, c and the transfer blocks, small) always goes to LDS, then A
  // and H (read once per step) while they fit
  for (int i = 0; i < P.nsd; ++i) {
    PersistLayout &Y = P.lay[i];
    const RomArgs<T> &A = P.sd[i];
    for (int f = 0; f < A.nfaces; ++f) {
      Y.tm[f] = (int)off;
      off += (long long)A.rs * A.fin[f].src_r;
    }
    if (A.B) {
      Y.bm = (int)off;
      off += (long long)A.r * A.rs;
    }
    if (A.c) {
      Y.c = (int)off;
      off += A.r;
    }
  }
  if (off > cap) return c.fail(OSAM_E_INVALID, "persistent OpInf engine: the reduced states exceed the LDS");
  for (int i = 0; i < P.nsd; ++i) place(P.lay[i].am, (long long)P.sd[i].r * P.sd[i].r);
  for (int i = 0; i < P.nsd; ++i)
    if (P.sd[i].r2 > 0) place(P.lay[i].h, (long long)P.sd[i].r * P.sd[i].r2);
  const hipError_t e = launch_rom_persist<T>(P, c.batch, (size_t)off * sizeof(T), c.stream);
  if (e != hipSuccess) return c.fail(OSAM_E_HIP, std::string("persistent OpInf kernel: ") + hipGetErrorString(e));
  return OSAM_OK;
}

int32_t Ctx::run_persist(int64_t n_steps, const Opts &o, osam_instance_info *info) {
  const std::string why = persist_unsupported(o);
  if (!why.empty()) return fail(OSAM_E_INVALID, "persistent OpInf engine: " + why);
  bool any = false;
  for (int b = 0; b < batch; ++b) {
    Status &S = h_status[b];
    if (S.flags & kNonfinite) continue;
    S.target = S.step + n_steps;
    S.flags &= ~kFinished;
    if (n_steps == 0) S.flags |= kFinished;
    S.iter = 0;
    any |= n_steps > 0;
  }
  HIPCHK(hipMemcpyAsync(d_status, h_status, sizeof(Status) * batch, hipMemcpyHostToDevice, stream));
  int32_t st = OSAM_OK;
  if (any) st = prec == OSAM_FP64 ? persist_launch<double>(*this, o) : persist_launch<float>(*this, o);
  if (st) return st;
  if ((st = sync_status())) return st;
  return instance_info(info);
}

int32_t Ctx::run(int64_t n_steps, const osam_schwarz_opts &op, osam_instance_info *info, bool host_sweeps) {
  if (!(op.tol_abs >= 0) || !(op.tol_rel >= 0) || op.min_iter < 1 || op.max_iter < op.min_iter ||
      op.max_iter > 1000000 || (op.guess != OSAM_GUESS_HOLD && op.guess != OSAM_GUESS_PREDICTOR) ||
      (op.additive != 0 && op.additive != 1))
    return fail(OSAM_E_INVALID, "bad Schwarz options");
  int32_t st = couple();
  if (st) return st;
  if ((st = wire())) return st;
  for (int b = 0; b < batch; ++b)
    if (!initialized[b]) return fail(OSAM_E_ORDER, "instance without initial condition");
  if ((st = sync_status())) return st;
  if ((st = init_pending())) return st;
  Opts o{};
  o.tol_abs2 = op.tol_abs * op.tol_abs;
  o.tol_rel2 = op.tol_rel * op.tol_rel;
  o.min_iter = op.min_iter;
  o.max_iter = op.max_iter;
  o.guess = op.guess;
  o.additive = op.additive;
  o.nsd = (int)sds.size();
  if (engine == 2) return run_persist(n_steps, o, info);
  if (window_mode()) return run_window(n_steps, o, info);
  bool any = false;
  for (int b = 0; b < batch; ++b) {
    Status &S = h_status[b];
    if (S.flags & kNonfinite) continue;
    S.target = S.step + n_steps;
    S.flags &= ~kFinished;
    if (n_steps == 0) S.flags |= kFinished;
    S.iter = 0;
    any |= n_steps > 0;
  }
  HIPCHK(hipMemcpyAsync(d_status, h_status, sizeof(Status) * batch, hipMemcpyHostToDevice, stream));
  // graph mode: capture graph_rounds sweeps (an even number, so the status buffers
  // are back in their roles after each replay) and replay whole graphs; sweeps
  // of finished instances are no-ops, so a replay may run past the last step
  struct ExecGuard {
    hipGraphExec_t g = nullptr;
    ~ExecGuard() {
      if (g) (void)hipGraphExecDestroy(g);
    }
  } guard;
  hipGraphExec_t &gexec = guard.g;
  // a single controller step (schwarz_step) launches its sweeps from the host: a captured
  // graph would replay graph_rounds sweeps for it
  const bool graph = graph_rounds > 0 && !timing && any && !host_sweeps;
  if (graph) {
    if (!aux) {
      HIPCHK(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&join_ev, hipEventDisableTiming));
    }
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    for (int r = 0; r < graph_rounds && !st; ++r)
      st = fuse ? launch_round_fused(o, r, graph_rounds)
                : (graph_streams == 2 ? launch_round_concurrent(o) : launch_round(o));
    const hipError_t ec = hipStreamEndCapture(stream, &g);
    if (st) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (ec != hipSuccess) return fail(OSAM_E_HIP, std::string("graph capture: ") + hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(OSAM_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
  }
  // every step ends within max_iter sweeps: bound the total work the host enqueues
  const long long round_cap = n_steps * (long long)o.max_iter + 8 + (graph ? 2LL * graph_rounds : 0);
  long long rounds_done = 0;
  while (any) {
    // every step needs at least min_iter sweeps: never enqueue more than the
    // least any unfinished instance still needs
    long long rounds = 0;
    for (int b = 0; b < batch; ++b) {
      const Status &S = h_status[b];
      if (S.flags & kFinished) continue;
      rounds = std::max(rounds, (S.target - S.step) * o.min_iter - S.iter);
    }
    rounds = std::max<long long>(1, rounds);
    if (graph) rounds = (rounds + graph_rounds - 1) / graph_rounds * graph_rounds;
    if (rounds_done + rounds > round_cap)
      return fail(OSAM_E_HIP, "controller did not finish within n_steps * max_iter sweeps");
    for (long long k = 0; k < rounds; k += graph ? graph_rounds : 1) {
      if (graph) {
        const hipError_t e = hipGraphLaunch(gexec, stream);
        if (e != hipSuccess) return fail(OSAM_E_HIP, std::string("graph launch: ") + hipGetErrorString(e));
      } else if ((st = fuse ? launch_round_fused(o, k, rounds) : launch_round(o))) {
        return st;
      }
    }
    rounds_done += rounds;
    if ((st = sync_status())) return st;
    any = false;
    for (int b = 0; b < batch; ++b) any |= !(h_status[b].flags & kFinished);
  }
  if ((st = sync_status())) return st;
  return instance_info(info);
}

// The host copy of the statuses into info (may be null); OSAM_E_NONFINITE if any instance
// went non-finite.
int32_t Ctx::instance_info(osam_instance_info *info) {
  bool nonfinite = false;
  for (int b = 0; b < batch; ++b) {
    const Status &S = h_status[b];
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

// ---------------------------------------------------------------------------
int32_t Ctx::get_state(int sdi, int inst, double *u, double *v, double *a) {
  int32_t st = sync_status();
  if (st) return st;
  Subdomain &d = *sds[sdi];
  const long long step = h_status[inst].step;
  std::vector<double> tmp((size_t)3 * d.cs);
  auto out = [&](double *dst) {
    for (int c = 0; c < 3; ++c)
      std::memcpy(dst + (size_t)c * d.nnodes, tmp.data() + (size_t)c * d.cs, sizeof(double) * d.nnodes);
  };
  if (!d.rom) {
    if (!d.u[0]) return fail(OSAM_E_ORDER, "no state");
    const size_t off = (size_t)inst * d.is * esize();
    void *bufs[3] = {(char *)d.u[step % 3] + off, (char *)d.v[step % 2] + off, (char *)d.a[step % 2] + off};
    double *dst[3] = {u, v, a};
    for (int k = 0; k < 3; ++k) {
      if (!dst[k]) continue;
      if ((st = download(tmp.data(), bufs[k], tmp.size()))) return st;
      out(dst[k]);
    }
    return OSAM_OK;
  }
  // lifted OpInf field: Phi q on free nodes, zero elsewhere
  double *scr = scratch((size_t)3 * d.cs + 8, &st);
  if (st) return fail(st, "oom");
  void *qs[3] = {d.q[step % 2], d.qd[step % 2], d.qdd[step % 2]};
  double *dst[3] = {u, v, a};
  for (int k = 0; k < 3; ++k) {
    if (!dst[k]) continue;
    HIPCHK(hipMemsetAsync(scr, 0, (size_t)3 * d.cs * esize(), stream));
    const size_t qo = (size_t)inst * d.r * esize();
    hipError_t e;
    if (prec == OSAM_FP64)
      e = launch_lift<double>((const double *)d.d_Phi, 3 * d.nfree_nodes, d.nfree_nodes, d.r,
                              (const double *)((char *)qs[k] + qo), (double *)scr, d.cs, d.npl, stream);
    else
      e = launch_lift<float>((const float *)d.d_Phi, 3 * d.nfree_nodes, d.nfree_nodes, d.r,
                             (const float *)((char *)qs[k] + qo), (float *)scr, d.cs, d.npl, stream);
    if (e != hipSuccess) return fail(OSAM_E_HIP, hipGetErrorString(e));
    if ((st = download(tmp.data(), scr, tmp.size()))) return st;
    out(dst[k]);
  }
  return OSAM_OK;
}

// ---------------------------------------------------------------------------
// Rows of Phi on one free node layer (all 3 components): [r][3 npl], the rows
// the pointwise projection (an injection) reads when lifting to a neighbour.
int32_t Ctx::phi_layer_rows(Subdomain &s, int layer, std::vector<double> &out) {
  const int n = 3 * s.npl;
  const long long nf = 3 * s.nfree_nodes;
  if (layer < 1 || layer > s.nzs - 1) return fail(OSAM_E_OUTSIDE, "projection reads a constrained layer");
  out.assign((size_t)s.r * n, 0.0);
  if (!s.oh.Phi.empty()) {
    for (int k = 0; k < s.r; ++k)
      for (int c = 0; c < 3; ++c)
        for (int nid = 0; nid < s.npl; ++nid)
          out[(size_t)k * n + c * s.npl + nid] =
              s.oh.Phi[(size_t)k * nf + c * s.nfree_nodes + (size_t)(layer - 1) * s.npl + nid];
    return OSAM_OK;
  }
  for (int k = 0; k < s.r; ++k)
    for (int c = 0; c < 3; ++c) {
      const size_t off = ((size_t)k * nf + c * s.nfree_nodes + (size_t)(layer - 1) * s.npl) * esize();
      int32_t st = download(out.data() + (size_t)k * n + c * s.npl, (const char *)s.d_Phi + off, s.npl);
      if (st) return st;
    }
  return OSAM_OK;
}

template <typename T>
__global__ void convert_kernel(const double *in, T *out, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (T)in[i];
}

int32_t Ctx::install_opinf_device(int sdi, const OpinfHost &oh, const double *phi_dev) {
  int32_t st = install_opinf(sdi, oh);
  if (st) return st;
  Subdomain &d = *sds[sdi];
  const long long n = 3 * d.nfree_nodes * (long long)oh.r;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (prec == OSAM_FP64)
    hipLaunchKernelGGL(convert_kernel<double>, dim3(blocks), dim3(256), 0, stream, phi_dev, (double *)d.d_Phi, n);
  else
    hipLaunchKernelGGL(convert_kernel<float>, dim3(blocks), dim3(256), 0, stream, phi_dev, (float *)d.d_Phi, n);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(stream));
  return OSAM_OK;
}

int32_t Ctx::install_opinf(int sdi, const OpinfHost &oh) {
  Subdomain &d = *sds[sdi];
  int32_t st = OSAM_OK;
  const int r = oh.r, rs = oh.rs, r2 = r * (r + 1) / 2;
  const long long nf = 3 * d.nfree_nodes;
  // free any previous OpInf data and the FOM state buffers
  void *old[] = {d.d_A, d.d_H, d.d_B, d.d_c, d.d_Phi, d.q[0], d.q[1], d.qd[0], d.qd[1], d.qdd[0], d.qdd[1], d.qpred,
                 d.u[0], d.u[1], d.u[2], d.v[0], d.v[1], d.a[0], d.a[1], d.face_phis[0], d.face_phis[1],
                 d.face_tm[0], d.face_tm[1], d.pre_fa, d.pre_fh, d.pre_blocks, d.pre_f0, d.pre_g};
  HIPCHK(hipStreamSynchronize(stream));
  for (void *p : old) dfree(p);
  d.d_A = d.d_H = d.d_B = d.d_c = d.d_Phi = nullptr;
  for (int k = 0; k < 2; ++k) d.q[k] = d.qd[k] = d.qdd[k] = nullptr;
  d.qpred = nullptr;
  for (int k = 0; k < 3; ++k) d.u[k] = nullptr;
  for (int k = 0; k < 2; ++k) d.v[k] = d.a[k] = nullptr;
  for (int k = 0; k < 2; ++k) d.face_phis[k] = d.face_tm[k] = nullptr;
  d.pre_fa = nullptr;
  d.pre_fh = nullptr;
  d.pre_blocks = nullptr;
  d.pre_f0 = nullptr;
  d.pre_g = nullptr;
  d.pre = false;
  // row-major copies for the kernels
  std::vector<double> Ar((size_t)r * r), Hr, Br;
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) Ar[(size_t)i * r + j] = oh.A[(size_t)j * r + i];
  if (oh.quadratic) {
    Hr.resize((size_t)r * r2);
    for (int i = 0; i < r; ++i)
      for (int m = 0; m < r2; ++m) Hr[(size_t)i * r2 + m] = oh.H[(size_t)m * r + i];
  }
  if (rs > 0) {
    Br.resize((size_t)r * rs);
    for (int i = 0; i < r; ++i)
      for (int l = 0; l < rs; ++l) Br[(size_t)i * rs + l] = oh.B[(size_t)l * r + i];
  }
  d.d_A = alloc_t(Ar.size(), &st);
  if (oh.quadratic) d.d_H = alloc_t(Hr.size(), &st);
  if (rs > 0) d.d_B = alloc_t(Br.size(), &st);
  if (!oh.c.empty()) d.d_c = alloc_t(r, &st);
  d.d_Phi = alloc_t((size_t)nf * r, &st);
  for (int k = 0; k < 2; ++k) {
    d.q[k] = alloc_t((size_t)batch * r, &st);
    d.qd[k] = alloc_t((size_t)batch * r, &st);
    d.qdd[k] = alloc_t((size_t)batch * r, &st);
  }
  // rounded up to whole groups of 64 instances (the batched f0 kernel reads groups)
  const size_t npred = (size_t)(batch + 63) / 64 * 64 * r;
  d.qpred = alloc_t(npred, &st);
  if (st) return fail(st, "out of device memory for OpInf data");
  HIPCHK(hipMemsetAsync(d.qpred, 0, npred * esize(), stream));
  if ((st = upload(d.d_A, Ar.data(), Ar.size()))) return st;
  if (oh.quadratic && (st = upload(d.d_H, Hr.data(), Hr.size()))) return st;
  if (rs > 0 && (st = upload(d.d_B, Br.data(), Br.size()))) return st;
  if (!oh.c.empty() && (st = upload(d.d_c, oh.c.data(), r))) return st;
  if (!oh.Phi.empty() && (st = upload(d.d_Phi, oh.Phi.data(), oh.Phi.size()))) return st;
  d.oh = oh;
  d.rec = osam_record{};
  d.rom = true;
  d.r = r;
  d.rs = rs;
  wired = false;
  win_ready = false;
  std::fill(initialized.begin(), initialized.end(), 0);
  HIPCHK(hipStreamSynchronize(stream));
  return OSAM_OK;
}

}  // namespace osam
