// Persistent OpInf engine (osam_set_engine(ctx, 2)): a context whose subdomains are
// all OpInf models runs every controller step of a run call in one launch, one
// workgroup per instance holding every subdomain's reduced state in LDS (and the
// operators, where they fit).  Per controller step, Alg. 1: sweeps in the
// multiplicative order until Eq. conv_criterion holds or max_iter sweeps are done.
// Each subdomain's iterate is the explicit central-difference step of
// Eq. opinf_model_schwarz, its boundary input g^ taken from the ROM neighbours through
// Phi_S,face^T Pi Phi_src (Sec. 4.2.3).  No workgroup waits for another: instances are
// independent, and a workgroup leaves when its instance reaches its target step.
//
// The arithmetic of a subdomain step is the OpInf step kernel's (rom_body without the
// batched parts) in its order: rows i = wave + 8 j with the lanes over the columns and
// one wave reduction per row, g^ one wave per mode, the FP64 sums of Eq.
// conv_criterion by the same workgroup reduction, the decision by decide().  So the
// iterates, sums, iteration counts and records are those of the single-step path.
#include <hip/hip_runtime.h>

#include "persist.hpp"
#include "rom_body.hpp"

namespace osam {

namespace {

// An operator in LDS when the host placed it there (offset >= 0), else in global memory.
template <typename T>
__device__ __forceinline__ const T *op(const T *lds, int off, const T *glob) {
  return off >= 0 ? lds + off : glob;
}

}  // namespace

template <typename T>
__global__ void __launch_bounds__(kRomThreads) rom_persist_kernel(PersistArgs<T> P) {
  extern __shared__ unsigned char persist_raw[];
  T *L = reinterpret_cast<T *>(persist_raw);
  __shared__ Status st;
  __shared__ double red[12][kRomWaves];
  __shared__ double nsum[2];
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  constexpr int kWords = sizeof(Status) / 4;
  if (tid < kWords) reinterpret_cast<unsigned *>(&st)[tid] = reinterpret_cast<const unsigned *>(P.status + b)[tid];
  __syncthreads();

  // the state (both parities) and the operators into LDS
  for (int s = 0; s < P.nsd; ++s) {
    const RomArgs<T> &A = P.sd[s];
    const PersistLayout &Y = P.lay[s];
    const long long qo = (long long)b * A.r;
    for (int i = tid; i < A.r; i += kRomThreads) {
      for (int p = 0; p < 2; ++p) {
        L[Y.q[p] + i] = A.q[p][qo + i];
        L[Y.v[p] + i] = A.qd[p][qo + i];
        L[Y.a[p] + i] = A.qdd[p][qo + i];
      }
      L[Y.qp + i] = A.qpred[qo + i];
    }
    if (Y.am >= 0)
      for (int i = tid; i < A.r * A.r; i += kRomThreads) L[Y.am + i] = A.A[i];
    if (Y.h >= 0)
      for (int i = tid; i < A.r * A.r2; i += kRomThreads) L[Y.h + i] = A.H[i];
    if (Y.bm >= 0)
      for (int i = tid; i < A.r * A.rs; i += kRomThreads) L[Y.bm + i] = A.B[i];
    if (Y.c >= 0)
      for (int i = tid; i < A.r; i += kRomThreads) L[Y.c + i] = A.c[i];
    for (int f = 0; f < A.nfaces; ++f)
      if (Y.tm[f] >= 0)
        for (int i = tid; i < A.rs * A.fin[f].src_r; i += kRomThreads) L[Y.tm[f] + i] = A.fin[f].tm[i];
  }
  __syncthreads();

  // the state by step parity as in global memory: the accepted state in parity step % 2,
  // the step's iterates in the other
  T *sh = L + P.sh_off;     // g^ (max rs)
  T *k2 = L + P.k2_off;     // q (x) q, compressed (max r2)
  T *rows = L + P.rows_off; // q''(t_k) before c
  while (!(st.flags & kFinished)) {
    const long long step = st.step;
    const int n_iter = st.iter + 1;
    const int s2 = (int)(step % 2);
    // a new step: every subdomain's predictor q(t_k) = q + dt q' + dt^2/2 q''
    if (n_iter == 1) {
      for (int s = 0; s < P.nsd; ++s) {
        const RomArgs<T> &A = P.sd[s];
        const PersistLayout &Y = P.lay[s];
        if (tid < A.r)
          L[Y.q1 + tid] = newmark_pred<T>(L[Y.q[s2] + tid], L[Y.v[s2] + tid], L[Y.a[s2] + tid], A.dt, A.half_dt2);
      }
      __syncthreads();
    }
    for (int s = 0; s < P.nsd; ++s) {
      const RomArgs<T> &A = P.sd[s];
      const PersistLayout &Y = P.lay[s];
      const int r = A.r, rs = A.rs, r2 = A.r2;
      const T *Am = op<T>(L, Y.am, A.A), *Hm = op<T>(L, Y.h, A.H), *Bm = op<T>(L, Y.bm, A.B);
      // ---- g^: ROM sources, one wave per mode (sources later in the sweep give their
      // accepted state (HOLD) or their predictor (PREDICTOR) in the step's first sweep)
      for (int k = tid; k < rs; k += kRomThreads) sh[k] = T(0);
      if (tid < r) rows[tid] = T(0);
      __syncthreads();
      for (int fi = 0; fi < A.nfaces; ++fi) {
        const RomFaceIn<T> &f = A.fin[fi];
        const PersistLayout &Ys = P.lay[P.slot[f.src_sd]];
        const bool hold = n_iter == 1 && f.src_sd > A.sd && P.opts.guess == 0;
        const bool pred = !hold && n_iter == 1 && f.src_sd > A.sd;
        const T *qs = L + (hold ? Ys.q[s2] : (pred ? Ys.q1 : Ys.q[1 - s2]));
        const T *tm = op<T>(L, Y.tm[fi], f.tm);
        for (int k = wid; k < rs; k += kRomWaves) {
          double v = 0.0;
          for (int j = lane; j < f.src_r; j += 64) v += (double)(tm[(long long)k * f.src_r + j] * qs[j]);
          v = wave_sum_d(v);
          if (lane == 0) sh[k] += (T)v;
        }
        __syncthreads();
      }
      // ---- compressed quadratic vector q_i q_j (i <= j)
      const T *q1 = L + Y.q1;
      if (r2 > 0 && (Y.pre < 0 || n_iter == 1)) {
        for (int idx = tid; idx < r * r; idx += kRomThreads) {
          const int i = idx / r, j = idx - i * r;
          if (j >= i) k2[i * r - (i * (i - 1)) / 2 + (j - i)] = q1[i] * q1[j];
        }
        __syncthreads();
      }
      // ---- rows of q''(t_k): A q + H k2 + B g^, one wave per row
      const int l0 = min(lane, r - 1), l1 = min(lane + 64, r - 1), lb = min(lane, rs > 0 ? rs - 1 : 0);
#pragma unroll 1
      for (int j = 0; j < kRowsPerWave; ++j) {
        const int i = wid + kRomWaves * j;
        if (i >= r) break;
        T bb = Bm ? Bm[(long long)i * rs + lb] : T(0);
        if (lane >= rs) bb = T(0);
        T sacc;
        if (Y.pre >= 0 && n_iter > 1) {
          // the lane's A and H terms of the row depend on q(t_k) only: the step's first
          // sweep left them here
          sacc = L[Y.pre + i * 64 + lane];
        } else {
          T a0 = Am[(long long)i * r + l0], a1 = r > 64 ? Am[(long long)i * r + l1] : T(0);
          if (lane >= r) a0 = T(0);
          if (lane + 64 >= r) a1 = T(0);
          sacc = a0 * (lane < r ? q1[lane] : T(0)) + a1 * (lane + 64 < r ? q1[lane + 64] : T(0));
          if (r2 > 0) {
            const T *Hr = Hm + (long long)i * r2;
#pragma unroll 4
            for (int m = lane; m < r2; m += 64) sacc += Hr[m] * k2[m];
          }
          if (Y.pre >= 0) L[Y.pre + i * 64 + lane] = sacc;
        }
        if (lane < rs) sacc += bb * sh[lane];
        for (int l = 64 + lane; l < rs; l += 64) sacc += Bm[(long long)i * rs + l] * sh[l];
        sacc = wave_total(sacc);
        if (lane == 0) rows[i] += sacc;
      }
      __syncthreads();
      // ---- velocity, sums of Eq. conv_criterion, next predictor
      double nrm[2] = {0.0, 0.0};
      if (tid < r) {
        const T cc = Y.c >= 0 ? L[Y.c + tid] : (A.c ? A.c[tid] : T(0));
        const T qn = q1[tid], an = rows[tid] + cc;
        const T qd0 = L[Y.v[s2] + tid], qdd0 = L[Y.a[s2] + tid];
        const T vn = qd0 + A.half_dt * (qdd0 + an);
        const T old_q = n_iter >= 2 ? L[Y.q[1 - s2] + tid] : L[Y.q[s2] + tid];
        const T old_v = n_iter >= 2 ? L[Y.v[1 - s2] + tid] : qd0;
        const double d = ((double)qn - (double)old_q) + (double)A.dt * ((double)vn - (double)old_v);
        nrm[0] = d * d;
        const double e = (double)qn + (double)A.dt * (double)vn;
        nrm[1] = e * e;
        L[Y.q[1 - s2] + tid] = qn;
        L[Y.v[1 - s2] + tid] = vn;
        L[Y.a[1 - s2] + tid] = an;
        L[Y.qp + tid] = newmark_pred<T>(qn, vn, an, A.dt, A.half_dt2);
      }
      block_reduce<2>(nrm, red, nsum);
      if (tid == 0) {
        st.sd_abs2[A.sd] = nsum[0];
        st.sd_den2[A.sd] = nsum[1];
      }
    }
    // ---- the decision after the sweep (the finisher's), and the accepted step
    if (tid == 0) decide(st, P.opts.nsd - 1, P.opts);
    __syncthreads();
    if (st.step != step) {   // accepted: the iterate (parity 1 - s2) is the new state; records
      for (int s = 0; s < P.nsd; ++s) {
        const RomArgs<T> &A = P.sd[s];
        const PersistLayout &Y = P.lay[s];
        if (tid < A.r && A.rec_q && A.rec_every > 0 && ((step + 1) % A.rec_every) == 0) {
          const long long col = (step + 1) / A.rec_every;
          if (col < A.rec_ncols) A.rec_q[((long long)b * A.rec_ncols + col) * A.r + tid] = L[Y.q[1 - s2] + tid];
        }
      }
    }
    __syncthreads();
  }

  // ---- back to global memory: both parities, the predictor, the status
  for (int s = 0; s < P.nsd; ++s) {
    const RomArgs<T> &A = P.sd[s];
    const PersistLayout &Y = P.lay[s];
    const long long qo = (long long)b * A.r;
    for (int i = tid; i < A.r; i += kRomThreads) {
      for (int p = 0; p < 2; ++p) {
        A.q[p][qo + i] = L[Y.q[p] + i];
        A.qd[p][qo + i] = L[Y.v[p] + i];
        A.qdd[p][qo + i] = L[Y.a[p] + i];
      }
      A.qpred[qo + i] = L[Y.qp + i];
    }
  }
  if (tid < kWords) reinterpret_cast<unsigned *>(P.status + b)[tid] = reinterpret_cast<const unsigned *>(&st)[tid];
}

template <typename T>
hipError_t launch_rom_persist(const PersistArgs<T> &P, int batch, size_t lds, hipStream_t s) {
  if (lds > kPersistLds) return hipErrorInvalidValue;
  if (lds > 65536) {
    static bool attr = false;
    if (!attr) {
      const hipError_t e = hipFuncSetAttribute((const void *)rom_persist_kernel<T>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPersistLds);
      if (e != hipSuccess) return e;
      attr = true;
    }
  }
  hipLaunchKernelGGL(rom_persist_kernel<T>, dim3(batch), dim3(kRomThreads), lds, s, P);
  return hipGetLastError();
}

template hipError_t launch_rom_persist<float>(const PersistArgs<float> &, int, size_t, hipStream_t);
template hipError_t launch_rom_persist<double>(const PersistArgs<double> &, int, size_t, hipStream_t);

}  // namespace osam
