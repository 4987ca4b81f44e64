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
// batched parts) in its order: the (A q + H (q (x) q)) row i by wave i mod 8 with the
// lanes over the columns and one wave reduction (once per step here: q(t_k) is fixed over
// the step's sweeps), B g^ added serially over the modes of g^, g^ one wave per mode, the
// FP64 sums of Eq. conv_criterion by the same workgroup reduction, the decision by
// decide().  So the iterates, sums, iteration counts and records are those of the
// single-step path.
#include <hip/hip_runtime.h>

#include "persist.hpp"
#include "rom_body.hpp"

namespace osam {

// NSD: the number of subdomains (every loop over them unrolled: the per-subdomain
// arguments are read with constant offsets).
template <typename T, int NSD>
__global__ void __launch_bounds__(kRomThreads) rom_persist_kernel(PersistArgs<T> P) {
  extern __shared__ unsigned char persist_raw[];
  T *L = reinterpret_cast<T *>(persist_raw);
  __shared__ Status st;
  __shared__ double red[2][kRomWaves];
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  constexpr int kWords = sizeof(Status) / 4;
  if (tid < kWords) reinterpret_cast<unsigned *>(&st)[tid] = reinterpret_cast<const unsigned *>(P.status + b)[tid];

  // the state (both parities) and the operators into LDS
#pragma unroll
  for (int s = 0; s < NSD; ++s) {
    const RomArgs<T> &A = P.sd[s];
    const PersistLayout &Y = P.lay[s];
    const long long qo = (long long)b * A.r;
    for (int i = tid; i < A.r; i += kRomThreads) {
#pragma unroll
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
#pragma unroll
    for (int f = 0; f < 2; ++f)
      if (f < A.nfaces && Y.tm[f] >= 0)
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
#pragma unroll
      for (int s = 0; s < NSD; ++s) {
        const RomArgs<T> &A = P.sd[s];
        const PersistLayout &Y = P.lay[s];
        if (tid < A.r)
          L[Y.q1 + tid] = newmark_pred<T>(L[Y.q[s2] + tid], L[Y.v[s2] + tid], L[Y.a[s2] + tid], A.dt, A.half_dt2);
      }
      __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < NSD; ++s) {
      const RomArgs<T> &A = P.sd[s];
      const PersistLayout &Y = P.lay[s];
      const int r = A.r, rs = A.rs, r2 = A.r2;
      // B, c and the transfer blocks are always in LDS; A and H where the host placed them
      // (separate loads for the two places: no generic-address loads)
      const T *q1 = L + Y.q1;
      // ---- g^ from the ROM sources, one wave per mode over the faces in order (sources
      // later in the sweep give their accepted state (HOLD) or their predictor
      // (PREDICTOR) in the step's first sweep); the compressed q (x) q alongside
      for (int k = wid; k < rs; k += kRomWaves) {
        T g = T(0);
#pragma unroll
        for (int fi = 0; fi < 2; ++fi) {
          if (fi >= A.nfaces) break;
          const RomFaceIn<T> &f = A.fin[fi];
          const PersistLayout &Ys = P.lay[P.slot[f.src_sd]];
          const bool hold = n_iter == 1 && f.src_sd > A.sd && P.opts.guess == 0;
          const bool pred = !hold && n_iter == 1 && f.src_sd > A.sd;
          const T *qs = L + (hold ? Ys.q[s2] : (pred ? Ys.q1 : Ys.q[1 - s2]));
          const T *tm = L + Y.tm[fi];
          double v = 0.0;
          for (int j = lane; j < f.src_r; j += 64) v += (double)(tm[k * f.src_r + j] * qs[j]);
          v = wave_sum_d(v);
          g += (T)v;
        }
        if (lane == 0) sh[k] = g;
      }
      if (r2 > 0 && n_iter == 1) {
        for (int idx = tid; idx < r * r; idx += kRomThreads) {
          const int i = idx / r, j = idx - i * r;
          if (j >= i) k2[i * r - (i * (i - 1)) / 2 + (j - i)] = q1[i] * q1[j];
        }
      }
      __syncthreads();
      // ---- the (A q + H k2) row of each mode, one wave per row: at the step's first sweep
      // (q(t_k) is fixed over the step's sweeps)
      T *f0 = L + Y.f0;
      if (n_iter == 1) {
        const int l0 = min(lane, r - 1), l1 = min(lane + 64, r - 1);
#pragma unroll 4
        for (int j = 0; j < kRowsPerWave; ++j) {
          const int i = wid + kRomWaves * j;
          if (i >= r) break;
          T a0, a1 = T(0);
          if (Y.am >= 0) {
            a0 = L[Y.am + i * r + l0];
            if (r > 64) a1 = L[Y.am + i * r + l1];
          } else {
            a0 = A.A[(long long)i * r + l0];
            if (r > 64) a1 = A.A[(long long)i * r + l1];
          }
          if (lane >= r) a0 = T(0);
          if (lane + 64 >= r) a1 = T(0);
          T sacc = a0 * (lane < r ? q1[lane] : T(0)) + a1 * (lane + 64 < r ? q1[lane + 64] : T(0));
          if (r2 > 0) {
            if (Y.h >= 0) {
              const T *Hr = L + Y.h + i * r2;
#pragma unroll 4
              for (int m = lane; m < r2; m += 64) sacc += Hr[m] * k2[m];
            } else {
              const T *Hr = A.H + (long long)i * r2;
#pragma unroll 4
              for (int m = lane; m < r2; m += 64) sacc += Hr[m] * k2[m];
            }
          }
          sacc = wave_total(sacc);
          if (lane == 0) f0[i] = sacc;
        }
        __syncthreads();
      }
      // ---- q''(t_k) = (A q + H k2) + B g^ (serial over the modes of g^) + c, velocity,
      // sums of Eq. conv_criterion, next predictor: one thread per mode
      double nrm0 = 0.0, nrm1 = 0.0;
      if (tid < r) {
        T bs = T(0);
        for (int l = 0; l < rs; ++l) bs += L[Y.bm + tid * rs + l] * sh[l];
        const T row = T(0) + (f0[tid] + bs);
        const T cc = Y.c >= 0 ? L[Y.c + tid] : T(0);
        const T qn = q1[tid], an = row + cc;
        const T qd0 = L[Y.v[s2] + tid], qdd0 = L[Y.a[s2] + tid];
        const T vn = qd0 + A.half_dt * (qdd0 + an);
        const T old_q = n_iter >= 2 ? L[Y.q[1 - s2] + tid] : L[Y.q[s2] + tid];
        const T old_v = n_iter >= 2 ? L[Y.v[1 - s2] + tid] : qd0;
        const double d = ((double)qn - (double)old_q) + (double)A.dt * ((double)vn - (double)old_v);
        nrm0 = d * d;
        const double e = (double)qn + (double)A.dt * (double)vn;
        nrm1 = e * e;
        L[Y.q[1 - s2] + tid] = qn;
        L[Y.v[1 - s2] + tid] = vn;
        L[Y.a[1 - s2] + tid] = an;
        L[Y.qp + tid] = newmark_pred<T>(qn, vn, an, A.dt, A.half_dt2);
      }
      // the workgroup sums in the step kernel's order (wave sums, then the waves in order);
      // thread 0 alone needs them
      if (wid * 64 < r) {   // waves holding modes; the others contribute zeros
        nrm0 = wave_sum_d(nrm0);
        nrm1 = wave_sum_d(nrm1);
      }
      if (lane == 0) {
        red[0][wid] = wid * 64 < r ? nrm0 : 0.0;
        red[1][wid] = wid * 64 < r ? nrm1 : 0.0;
      }
      __syncthreads();
      if (tid == 0) {
        double t0 = 0.0, t1 = 0.0;
        for (int w = 0; w < kRomWaves; ++w) t0 += red[0][w];
        for (int w = 0; w < kRomWaves; ++w) t1 += red[1][w];
        st.sd_abs2[A.sd] = t0;
        st.sd_den2[A.sd] = t1;
      }
    }
    // ---- the decision after the sweep (the finisher's), and the accepted step
    if (tid == 0) decide(st, P.opts.nsd - 1, P.opts);
    __syncthreads();
    if (st.step != step) {   // accepted: the iterate (parity 1 - s2) is the new state; records
#pragma unroll
      for (int s = 0; s < NSD; ++s) {
        const RomArgs<T> &A = P.sd[s];
        const PersistLayout &Y = P.lay[s];
        if (tid < A.r && A.rec_q && A.rec_every > 0 && ((step + 1) % A.rec_every) == 0) {
          const long long col = (step + 1) / A.rec_every;
          if (col < A.rec_ncols) A.rec_q[((long long)b * A.rec_ncols + col) * A.r + tid] = L[Y.q[1 - s2] + tid];
        }
      }
    }
  }

  // ---- back to global memory: both parities, the predictor, the status
#pragma unroll
  for (int s = 0; s < NSD; ++s) {
    const RomArgs<T> &A = P.sd[s];
    const PersistLayout &Y = P.lay[s];
    const long long qo = (long long)b * A.r;
    for (int i = tid; i < A.r; i += kRomThreads) {
#pragma unroll
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

template <typename T, int NSD>
static hipError_t launch_nsd(const PersistArgs<T> &P, int batch, size_t lds, hipStream_t s) {
  if (lds > 65536) {
    static bool attr = false;
    if (!attr) {
      const hipError_t e = hipFuncSetAttribute((const void *)rom_persist_kernel<T, NSD>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPersistLds);
      if (e != hipSuccess) return e;
      attr = true;
    }
  }
  hipLaunchKernelGGL((rom_persist_kernel<T, NSD>), dim3(batch), dim3(kRomThreads), lds, s, P);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rom_persist(const PersistArgs<T> &P, int batch, size_t lds, hipStream_t s) {
  if (lds > kPersistLds) return hipErrorInvalidValue;
  switch (P.nsd) {
    case 1: return launch_nsd<T, 1>(P, batch, lds, s);
    case 2: return launch_nsd<T, 2>(P, batch, lds, s);
    case 3: return launch_nsd<T, 3>(P, batch, lds, s);
    case 4: return launch_nsd<T, 4>(P, batch, lds, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_rom_persist<float>(const PersistArgs<float> &, int, size_t, hipStream_t);
template hipError_t launch_rom_persist<double>(const PersistArgs<double> &, int, size_t, hipStream_t);

}  // namespace osam
