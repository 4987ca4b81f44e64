// Device code of the OpInf step kernel (see rom_kernels.hip), shared by the step
// kernel and the fused sweep kernel.
#pragma once
#include <hip/hip_runtime.h>

#include "osam_device.hpp"
#include "stencil.hpp"

namespace osam {

__device__ __forceinline__ double wave_sum_d(double x) { return wave_total(x); }

// The value lane l (wave-uniform) holds.
__device__ __forceinline__ float lane_value(float x, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
}
__device__ __forceinline__ double lane_value(double x, int l) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

constexpr int kRomThreads = 512;
constexpr int kRomWaves = kRomThreads / 64;   // 8
constexpr int kRowsPerWave = 16;              // rows i = wave + 8 j: r <= 128
constexpr int kFaceDofs = 4;                  // face DOFs per thread on the fast g^ path
// Register widths of the two variants: modes of the push row held (the rest streams at
// the push) and reduced face modes of the first FOM face held (more take the general
// loop); narrow for models with r <= 40 and r_S <= 2.  The held entries are added in one
// order either way, so both widths give the same bits where they apply.
constexpr int kPushNarrow = 40, kPushWide = 64, kFaceNarrow = 2, kFaceWide = 8;

// 16-byte vectors (push rows are read a row per thread, 16 bytes per load)
template <typename T>
constexpr int kVec16 = 16 / (int)sizeof(T);
template <typename T>
using Vec16 = T __attribute__((ext_vector_type(16 / sizeof(T))));

// Sum of NV per-thread values over the workgroup in a fixed order; the totals
// land in out[0..NV) (LDS) for every thread after the call.
template <int NV, typename T>
__device__ __forceinline__ void block_reduce(double (&v)[NV], double (*red)[kRomWaves], T *out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum_d(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][wid] = v[k];
  }
  __syncthreads();
  if ((int)threadIdx.x < NV) {
    double t = 0.0;
    for (int w = 0; w < kRomWaves; ++w) t += red[threadIdx.x][w];
    out[threadIdx.x] = (T)t;
  }
  __syncthreads();
}

// block_reduce restricted to the entries whose bit is set in `used` (wave-uniform): the
// others are zero on every thread and give 0 without their wave reductions.
template <int NV, typename T>
__device__ __forceinline__ void block_reduce_used(double (&v)[NV], unsigned used, double (*red)[kRomWaves],
                                                  T *out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k)
    if ((used >> k) & 1u) v[k] = wave_sum_d(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][wid] = ((used >> k) & 1u) ? v[k] : 0.0;
  }
  __syncthreads();
  if ((int)threadIdx.x < NV) {
    double t = 0.0;
    for (int w = 0; w < kRomWaves; ++w) t += red[threadIdx.x][w];
    out[threadIdx.x] = (T)t;
  }
  __syncthreads();
}

// Grid (G, batch): the G workgroups of an instance each take one slice of the
// push rows and recompute the (small) reduced step redundantly, so the push
// streams through G CUs instead of one; workgroup 0 alone stores the state and
// the sums and, when this subdomain ends the sweep, decides.  Every load that
// does not depend on this step's results is issued first, in one straight-line
// batch (indices clamped into range, values zeroed afterwards), speculatively
// for both state parities and all three face roles.
// Variants (register budget): kRomPre = f0 and the FOM-fed g^ arrive as
// partial sums (no A rows, no quadratic term, no FOM face here);
// kRomNoPushRegs = no push row held in registers (no FOM neighbour);
// kRomWide = the wide register widths (r > kPushNarrow or r_S > kFaceNarrow), else narrow.
// Registers held for modes a model does not have are spent for nothing: with the wide
// widths at r = 40, r_S = 1 the fused sweep kernel spilled 40 VGPRs (132 bytes of scratch
// per lane); with the narrow ones it needs 247 VGPRs and spills none, and a Schwarz sweep
// of the 24x24x240 FOM-OpInf bar takes 14.5 instead of 15.5 us.
constexpr int kRomPre = 1, kRomNoPushRegs = 2, kRomWide = 4;

template <typename T>
__host__ __device__ inline int rom_variant(const RomArgs<T> &A) {
  return (A.f0part ? kRomPre : 0) |
         (A.nexp == 0 ? kRomNoPushRegs : (A.r > kPushNarrow || A.rs > kFaceNarrow ? kRomWide : 0));
}
// The variant of a kernel holding several OpInf subdomains: the batched parts and no push
// registers only if every subdomain has them, the wide push row if any needs it.
__host__ __device__ inline int rom_variant_join(int a, int b) {
  const int v = (a & b & (kRomPre | kRomNoPushRegs)) | ((a | b) & kRomWide);
  return (v & kRomNoPushRegs) ? (v & ~kRomWide) : v;
}

// The status a step starts from, read from A.status[b] (flags, step, iteration).
template <typename T>
struct StatusOf {
  const RomArgs<T> &A;
  __device__ __forceinline__ StepState operator()() const {
    const Status *p = A.status + blockIdx.y;
    StepState s;
    s.step = p->step;
    s.iter = p->iter;
    s.flags = p->flags;
    return s;
  }
};

// state(): the status this step starts from (StatusOf, or the folded decision of a fused
// sweep); every thread of the workgroup calls it once, after the loads of phase 1 are
// issued, so that those loads (which do not depend on it) go out first.
template <typename T, int V, typename State>
__device__ __forceinline__ void rom_body(const RomArgs<T> &A, int g, State state) {
  constexpr bool PRE = (V & kRomPre) != 0, PUSHREG = (V & kRomNoPushRegs) == 0;
  constexpr int kPushK = (V & kRomWide) ? kPushWide : kPushNarrow;
  constexpr int FR = (V & kRomWide) ? kFaceWide : kFaceNarrow;   // face modes held
  const int b = blockIdx.y;
  const int r = A.r, rs = A.rs, r2 = A.r2;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const long long qo = (long long)b * r;
  const bool last = !A.defer && A.sd == A.opts.nsd - 1;
  const FinishArgs &F = A.finish;

  extern __shared__ unsigned char smem_raw[];
  T *q1s = reinterpret_cast<T *>(smem_raw);   // q(t_k): Newmark predictor of the accepted state
  T *qps = q1s + r;                            // q(t_k+1) predictor, input of the pushes
  T *qdd1s = qps + r;                          // row sums of q''(t_k)
  T *sh = qdd1s + r;                           // g^ (max(rs, 1))
  T *k2 = sh + (rs > 0 ? rs : 1);              // q (x) q, compressed (r2)
  __shared__ double red[12][kRomWaves];
  __shared__ double tot[12];
  __shared__ double nsum[2];

  // ---- 1. loads independent of this step's results (and of its status)
  const int tq = min(tid, r - 1);
  T xq[2], xqd[2], xqdd[2], x_c = T(0);
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    xq[p] = A.q[p][qo + tq];
    xqd[p] = A.qd[p][qo + tq];
    xqdd[p] = A.qdd[p][qo + tq];
  }
  if (A.c) x_c = A.c[tq];
  // batched path: this row's f0 and this thread's mode of g^ (partial sums, fixed order)
  T x_f0 = T(0);
  double x_g = 0.0;
  // (buffer loads: one per-lane offset, the split in the uniform offset)
  if (A.f0part) {
    const Field<T> F0(A.f0part);
    const unsigned vo = (unsigned)((qo + tq) * (long long)sizeof(T));
    for (int k = 0; k < A.f0_ks; ++k) x_f0 += F0.ld(vo, (unsigned)(k * A.f0_stride * (long long)sizeof(T)));
  }
  if (A.gpart && rs > 0) {
    const Field<double> G(A.gpart);
    const unsigned vo = (unsigned)(((long long)b * rs + min(tid, rs - 1)) * 8);
    for (int k = 0; k < A.g_gs; ++k) x_g += G.ld(vo, (unsigned)(k * A.g_stride * 8));
  }
  T arow[kRowsPerWave][2], brow[kRowsPerWave];
  const int l0 = min(lane, r - 1), l1 = min(lane + 64, r - 1), lb = min(lane, rs > 0 ? rs - 1 : 0);
#pragma unroll
  for (int j = 0; j < kRowsPerWave; ++j) {
    const int i = wid + kRomWaves * j;
    arow[j][0] = arow[j][1] = brow[j] = T(0);
    if (i < r) {   // wave-uniform
      if (!PRE && A.A) {
        arow[j][0] = A.A[(long long)i * r + l0];
        if (r > 64) arow[j][1] = A.A[(long long)i * r + l1];
      }
      if (A.B) brow[j] = A.B[(long long)i * rs + lb];
    }
  }
  // first face when fed by a FOM: values of all three roles and up to 8 modes
  const bool small_face = !PRE && A.nfaces > 0 && A.fin[0].type == kFaceFom &&
                          A.fin[0].n <= kFaceDofs * kRomThreads && rs <= FR;
  T fv[3][kFaceDofs], fph[kFaceDofs][FR];
  if (small_face) {
    const RomFaceIn<T> &f = A.fin[0];
#pragma unroll
    for (int d = 0; d < kFaceDofs; ++d) {
      const long long m = min(tid + kRomThreads * d, f.n - 1);
#pragma unroll
      for (int ro = 0; ro < 3; ++ro) fv[ro][d] = f.sface[ro][(long long)b * f.n + m];
#pragma unroll
      for (int kk = 0; kk < FR; ++kk) fph[d][kk] = kk < rs ? f.phis[(long long)kk * f.n + m] : T(0);
    }
  }
  // this thread's push row (export 0): (Pi Phi)[m, 0..r)
  const bool reg_push = PUSHREG && A.nexp > 0;
  T pv[kPushK];
  if (reg_push) {
    const RomExport<T> &ex = A.ex[0];
    const int n = 3 * ex.npl;
    const long long m = min(g * kRomThreads + tid, n - 1);
    const Vec16<T> *row = reinterpret_cast<const Vec16<T> *>(ex.prow + m * ex.r4);
#pragma unroll
    for (int j = 0; j < kPushK / kVec16<T>; ++j) {
      const Vec16<T> v = j * kVec16<T> < r ? row[j] : Vec16<T>(T(0));
#pragma unroll
      for (int e = 0; e < kVec16<T>; ++e) pv[j * kVec16<T> + e] = v[e];
    }
  }
  // the FOM workgroups' partial sums, when this workgroup decides
  bool small_part = !PRE && last && g == 0 && F.nfom <= 2;
  for (int k = 0; k < F.nfom; ++k) small_part = small_part && F.nblocks[k] <= kFaceDofs * kRomThreads;
  double2 pa[2][kFaceDofs];
  if (small_part && F.nfom > 0) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int kk = min(k, F.nfom - 1);
      const double2 *pp = reinterpret_cast<const double2 *>(F.part[kk]) + (long long)b * F.nblocks[kk];
#pragma unroll
      for (int d = 0; d < kFaceDofs; ++d) pa[k][d] = pp[min(tid + kRomThreads * d, F.nblocks[kk] - 1)];
    }
  }
  const StepState ss = state();
  const int flags = ss.flags;
  const long long step = ss.step;
  const int iter = ss.iter;
  if (flags & kFinished) {
    if (last && g == 0 && wid == 0) finish_sweep<4>(A.status, A.status_out, F, A.opts, b);   // carries the status over
    return;
  }
  const int n_iter = iter + 1;
  const int s2 = (int)(step % 2);
  const T x_q0 = xq[s2], x_qd0 = xqd[s2], x_qdd0 = xqdd[s2];
  const T x_old_q = n_iter >= 2 ? xq[1 - s2] : x_q0;
  const T x_old_v = n_iter >= 2 ? xqd[1 - s2] : x_qd0;
#pragma unroll
  for (int j = 0; j < kRowsPerWave; ++j) {
    if (lane >= r) arow[j][0] = T(0);
    if (lane + 64 >= r) arow[j][1] = T(0);
    if (lane >= rs) brow[j] = T(0);
  }

  // ---- 2. predictor q(t_k) = q + dt q' + dt^2/2 q''
  if (tid < r) {
    q1s[tid] = newmark_pred<T>(x_q0, x_qd0, x_qdd0, A.dt, A.half_dt2);
    qdd1s[tid] = x_f0;   // rows add A q + H (q (x) q) + B g^ below
  }
  for (int k = tid; k < rs; k += kRomThreads) sh[k] = k == tid ? (T)x_g : T(0);

  // ---- 3. reduced boundary input g^ (and the FOM partial sums, same reduction)
  if (PRE) {
    __syncthreads();   // sh is complete
  } else {
    double part[FR + 4];   // face modes, then the FOM partial sums
#pragma unroll
    for (int kk = 0; kk < FR + 4; ++kk) part[kk] = 0.0;
    if (small_face) {
      const RomFaceIn<T> &f = A.fin[0];
      const bool hold = n_iter == 1 && (f.src_sd > A.sd || A.opts.additive) && A.opts.guess == 0;
      const int ro = hold ? (int)(step % 3) : (int)((step + 1) % 3);
#pragma unroll
      for (int d = 0; d < kFaceDofs; ++d) {
        const bool ok = tid + kRomThreads * d < f.n;
        const T sv = ok ? (ro == 0 ? fv[0][d] : (ro == 1 ? fv[1][d] : fv[2][d])) : T(0);
#pragma unroll
        for (int kk = 0; kk < FR; ++kk)
          if (kk < rs) part[kk] += (double)(fph[d][kk] * sv);
      }
    }
    if (small_part) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int d = 0; d < kFaceDofs; ++d)
          if (k < F.nfom && tid + kRomThreads * d < F.nblocks[k]) {
            part[FR + 2 * k] += pa[k][d].x;
            part[FR + 1 + 2 * k] += pa[k][d].y;
          }
    }
    const unsigned used = (small_face ? (1u << rs) - 1u : 0u) |
                          (small_part ? ((1u << (2 * min(F.nfom, 2))) - 1u) << FR : 0u);
    block_reduce_used<FR + 4>(part, used, red, tot);
    if (small_face && tid < rs) sh[tid] = (T)tot[tid];
  }
  for (int fi = small_face ? 1 : 0; fi < A.nfaces; ++fi) {
    const RomFaceIn<T> &f = A.fin[fi];
    const bool hold = n_iter == 1 && (f.src_sd > A.sd || A.opts.additive) && A.opts.guess == 0;
    if (f.type == kFaceFom) {
      // g^_k += sum_m Phi_S[m, k] s_m : threads over the face DOFs, 8 modes per pass
      const T *src = f.sface[hold ? (int)(step % 3) : (int)((step + 1) % 3)] + (long long)b * f.n;
      for (int k0 = 0; k0 < rs; k0 += 8) {
        double part[8];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) part[kk] = 0.0;
        for (int m0 = 0; m0 < f.n; m0 += 2 * kRomThreads) {
          T sv[2], ph[2][8];
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            const long long m = min(m0 + tid + kRomThreads * d, f.n - 1);
            sv[d] = m0 + tid + kRomThreads * d < f.n ? src[m] : T(0);
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) ph[d][kk] = f.phis[(long long)min(k0 + kk, rs - 1) * f.n + m];
          }
#pragma unroll
          for (int d = 0; d < 2; ++d)
#pragma unroll
            for (int kk = 0; kk < 8; ++kk)
              if (k0 + kk < rs) part[kk] += (double)(ph[d][kk] * sv[d]);
        }
        block_reduce<8>(part, red, tot + 0);
        if (tid < 8 && k0 + tid < rs) sh[k0 + tid] += (T)tot[tid];
        __syncthreads();
      }
    } else {
      // ROM source: g^ += (Phi_S,face^T Pi Phi_src) q_src, one wave per mode
      const long long so = (long long)b * f.src_r;
      // the source's predictor at t_k when it is not read back from this sweep:
      // fused sweeps, and the first sweep of a step before the source has run
      // (PREDICTOR guess with the source later in the sweep)
      const bool pred = !hold && (f.pred || (n_iter == 1 && (f.src_sd > A.sd || A.opts.additive)));
      const T *qs = f.src_q[hold || pred ? s2 : 1 - s2] + so;
      for (int k = wid; k < rs; k += kRomWaves) {
        double v = 0.0;
        for (int j = lane; j < f.src_r; j += 64) {
          const T x = pred ? newmark_pred<T>(qs[j], f.src_qd[s2][so + j], f.src_qdd[s2][so + j], f.src_dt,
                                             f.src_half_dt2)
                           : qs[j];
          v += (double)(f.tm[(long long)k * f.src_r + j] * x);
        }
        v = wave_sum_d(v);
        if (lane == 0) sh[k] += (T)v;
      }
      __syncthreads();
    }
  }
  __syncthreads();

  // ---- 4. compressed quadratic vector q_i q_j (i <= j), row by row
  if (!PRE && r2 > 0) {
    for (int idx = tid; idx < r * r; idx += kRomThreads) {
      const int i = idx / r, j = idx - i * r;
      if (j >= i) k2[i * r - (i * (i - 1)) / 2 + (j - i)] = q1s[i] * q1s[j];
    }
    __syncthreads();
  }

  // ---- 5. q''(t_k) rows: (A q + H k2) + B g^ (+ c below), one wave per row: the first
  // term by the wave's reduction, the second serially over the modes of g^
#pragma unroll
  for (int j = 0; j < kRowsPerWave; ++j) {
    const int i = wid + kRomWaves * j;
    if (i >= r) break;
    T s = PRE ? T(0) : arow[j][0] * (lane < r ? q1s[lane] : T(0)) + arow[j][1] * (lane + 64 < r ? q1s[lane + 64] : T(0));
    if (!PRE && r2 > 0) {
      const T *Hr = A.H + (long long)i * r2;
#pragma unroll 4
      for (int m = lane; m < r2; m += 64) s += Hr[m] * k2[m];
    }
    if (!PRE) s = wave_total(s);   // the row of A q + H (q (x) q): fixed over a step's sweeps
    // B g^, serial over the modes of g^ (every lane the same value; lane l holds B[i, l])
    T bs = T(0);
    for (int l = 0; l < rs && l < 64; ++l) bs += lane_value(brow[j], l) * sh[l];
    for (int l = 64; l < rs; ++l) bs += A.B[(long long)i * rs + l] * sh[l];
    if (lane == 0) qdd1s[i] += s + bs;
  }
  __syncthreads();

  // ---- 6. velocity, convergence sums, next predictor (workgroup 0 stores the state after the
  // push: stores and loads share one completion counter, so stores issued here would hold the
  // push's first use of its preloaded row until they complete)
  double nrm[2] = {0.0, 0.0};
  T qn = T(0), vn = T(0), an = T(0);
  if (tid < r) {
    qn = q1s[tid];
    an = qdd1s[tid] + x_c;
    vn = x_qd0 + A.half_dt * (x_qdd0 + an);
    qps[tid] = newmark_pred<T>(qn, vn, an, A.dt, A.half_dt2);
    if (g == 0) {
      const double d = ((double)qn - (double)x_old_q) + (double)A.dt * ((double)vn - (double)x_old_v);
      nrm[0] = d * d;
      const double e = (double)qn + (double)A.dt * (double)vn;
      nrm[1] = e * e;
    }
  }
  block_reduce<2>(nrm, red, nsum);   // also publishes qps to every thread

  // ---- 7. push (Pi Phi) q(t_k+1) into the FOM neighbours' faces (role of step k+1)
  const int role = (int)((step + 2) % 3);
  for (int e = 0; e < A.nexp; ++e) {
    const RomExport<T> &ex = A.ex[e];
    const int n = 3 * ex.npl;
    const int m = g * kRomThreads + tid;
    T acc0 = T(0), acc1 = T(0);
    if (PUSHREG && e == 0) {
      // branch-free: every LDS read in range (index clamped), modes >= r add a zero product,
      // so the reads go out together instead of one round trip per mode
#pragma unroll
      for (int k = 0; k < kPushK; k += 2) {
        acc0 += (k < r ? pv[k] : T(0)) * qps[min(k, r - 1)];
        acc1 += (k + 1 < r ? pv[k + 1] : T(0)) * qps[min(k + 1, r - 1)];
      }
    }
    const Vec16<T> *row = reinterpret_cast<const Vec16<T> *>(ex.prow + (long long)min(m, n - 1) * ex.r4);
    for (int k0 = PUSHREG && e == 0 ? kPushK : 0; k0 < r; k0 += 16) {
      T pw[16];
#pragma unroll
      for (int j = 0; j < 16 / kVec16<T>; ++j) {
        const int k = k0 + j * kVec16<T>;
        const Vec16<T> v = k < ex.r4 ? row[k / kVec16<T>] : Vec16<T>(T(0));
#pragma unroll
        for (int q = 0; q < kVec16<T>; ++q) pw[j * kVec16<T> + q] = v[q];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (k0 + u < r) acc0 += pw[u] * qps[k0 + u];
    }
    if (m < n) {
      const int c = m / ex.npl, nid = m - c * ex.npl;
      ex.role[role][(long long)b * ex.is + c * ex.cs + nid] = acc0 + acc1;
    }
  }

  if (g == 0 && tid < r) {   // the state of this iterate
    A.q[1 - s2][qo + tid] = qn;
    A.qd[1 - s2][qo + tid] = vn;
    A.qdd[1 - s2][qo + tid] = an;
    A.qpred[qo + tid] = qps[tid];   // the next step's q(t_k) if this iterate is accepted
    if (A.rec_q && A.rec_every > 0 && ((step + 1) % A.rec_every) == 0) {
      const long long col = (step + 1) / A.rec_every;
      if (col < A.rec_ncols) A.rec_q[((long long)b * A.rec_ncols + col) * r + tid] = qn;
    }
  }

  // ---- 8. sums of this subdomain; the last subdomain of the sweep decides
  if (g != 0) return;
  if (last) {
    if (wid == 0)
      finish_sweep<4>(A.status, A.status_out, F, A.opts, b, A.sd, nsum[0], nsum[1], small_part ? tot + FR : nullptr);
  } else if (tid == 0) {
    if (A.sums_out) {
      A.sums_out[((long long)b * kMaxSd + A.sd) * 2] = nsum[0];
      A.sums_out[((long long)b * kMaxSd + A.sd) * 2 + 1] = nsum[1];
    } else {
      A.status_out[b].sd_abs2[A.sd] = nsum[0];
      A.status_out[b].sd_den2[A.sd] = nsum[1];
    }
  }
}

}  // namespace osam
