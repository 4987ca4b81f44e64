// Batched parts of the OpInf step for large batches and large reduced models
// (Sec. 4.2, Eq. opinf_model_schwarz: q'' = A q + H (q (x) q) + B g^ + c).
//
//  * rom_f0_kernel: f0 = A q + H (q (x) q) + c at the step's Newmark predictor
//    q(t_k).  With the explicit scheme that predictor depends only on the
//    accepted state, so f0 is fixed for all Schwarz iterations of a step and is
//    evaluated once, at the step's first iteration.  It is one contraction
//    M z with M = [A | H] (r x K, K = r + r(r+1)/2) and z = [q; q (x) q] per
//    instance, run on the matrix cores over tiles of 16 rows x 16 instances.
//    The linear part always takes FP32 operands (v_mfma_f32_16x16x4_f32); the
//    quadratic part FP32 operands too, or BF16 operands with FP32 accumulation
//    (v_mfma_f32_16x16x16_bf16) in the BF16-H precision.  M is stored in MFMA
//    fragment order, so every wave reads one contiguous block per instruction;
//    z is formed on the fly
//    from the predictor staged in LDS and a table of the (i, j) pairs of the
//    compressed quadratic vector.  K is split over workgroups; each split
//    writes its own partial tile (no atomics), reduced in a fixed order by the
//    step kernel.
//  * rom_ghat_kernel: g^ = Phi_S^T s over the faces fed by FOM neighbours, split
//    over the face DOFs, FP64 partial sums per split.
#include <hip/hip_ext.h>

#include "osam_device.hpp"

namespace osam {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ short to_bf16(float x) {
  unsigned u = __builtin_bit_cast(unsigned, x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

constexpr int kPreThreads = 256;

template <int PREC>
__global__ void __launch_bounds__(kPreThreads) rom_f0_kernel(RomPreArgs P) {
  const int it = blockIdx.y;
  const int rt = blockIdx.x % P.nrt, ksi = blockIdx.x / P.nrt;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  extern __shared__ float q1s[];   // [16][r]: the predictor of the tile's instances
  __shared__ f4_t red[4][64];

  // only when some instance of the tile starts a step
  bool need = false;
  if (tid < 16) {
    const int b = it * 16 + tid;
    if (b < P.batch) {
      const Status &S = P.status[b];
      need = !(S.flags & kFinished) && S.iter == 0;
    }
  }
  if (!__syncthreads_or(need)) return;

  const int r = P.r;
  for (int e = tid; e < 16 * r; e += kPreThreads) {
    const int bl = e / r, k = e - bl * r;
    const int b = min(it * 16 + bl, P.batch - 1);
    const int s2 = (int)(P.status[b].step % 2);
    const long long o = (long long)b * r + k;
    q1s[e] = newmark_pred<float>(P.q[s2][o], P.qd[s2][o], P.qdd[s2][o], P.dt, P.half_dt2);
  }
  __syncthreads();

  // this split's K blocks (A blocks first, then H blocks), round robin over the waves
  const int nkb = P.nkba + P.nkbh;
  const int per = (nkb + P.ks - 1) / P.ks;
  const int kb0 = ksi * per, kb1 = min(nkb, kb0 + per);
  const int col = lane & 15, grp = lane >> 4;
  const float *qc = q1s + col * r;
  f4_t acc = {0.f, 0.f, 0.f, 0.f};
  auto quad = [&](int m) -> float {   // (q (x) q)[m] of instance col
    if (m >= P.r2) return 0.f;
    const int pr = P.pairs[m];
    return qc[pr & 0xffff] * qc[pr >> 16];
  };
  for (int kb = kb0 + wid; kb < kb1; kb += 4) {
    if (kb < P.nkba) {   // linear part, FP32 operands
      const float a = P.frag_a[((long long)rt * P.nkba + kb) * 64 + lane];
      const int k = kb * 4 + grp;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, k < r ? qc[k] : 0.f, acc, 0, 0, 0);
    } else if (PREC == 0) {
      const int kh = kb - P.nkba;
      const float a = reinterpret_cast<const float *>(P.frag_h)[((long long)rt * P.nkbh + kh) * 64 + lane];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, quad(kh * 4 + grp), acc, 0, 0, 0);
    } else {
      const int kh = kb - P.nkba;
      const s4_t a = reinterpret_cast<const s4_t *>(P.frag_h)[((long long)rt * P.nkbh + kh) * 64 + lane];
      s4_t z;
#pragma unroll
      for (int j = 0; j < 4; ++j) z[j] = to_bf16(quad(kh * 16 + 4 * grp + j));
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, z, acc, 0, 0, 0);
    }
  }
  red[wid][lane] = acc;
  __syncthreads();
  if (wid == 0) {
    f4_t t = red[0][lane];
#pragma unroll
    for (int w = 1; w < 4; ++w) t += red[w][lane];
    // result register i of lane l: row 4 (l / 16) + i, column (instance) l % 16
    const int b = it * 16 + col;
    if (b < P.batch) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rt * 16 + 4 * grp + i;
        if (row < r) {
          float v = t[i];
          if (ksi == 0 && P.c) v += P.c[row];
          P.f0part[((long long)ksi * P.batch + b) * r + row] = v;
        }
      }
    }
  }
}

// grid (gs, batch): workgroup (split, instance) sums its slice of the FOM-fed
// face DOFs for every mode; gpart[split][b][k] in FP64.
__global__ void __launch_bounds__(kPreThreads) rom_ghat_kernel(RomPreArgs P) {
  const int gsi = blockIdx.x, b = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const Status &S = P.status[b];
  if (S.flags & kFinished) return;
  const int n_iter = S.iter + 1;
  const long long step = S.step;
  __shared__ double red[4][8];
  for (int k0 = 0; k0 < P.rs; k0 += 8) {
    double part[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) part[kk] = 0.0;
    for (int f = 0; f < P.nface; ++f) {
      const long long n = P.fn[f];
      const long long per = (n + P.gs - 1) / P.gs;
      const long long m0 = gsi * per, m1 = min(n, m0 + per);
      const bool hold = n_iter == 1 && P.fsrc[f] > P.sd && P.opts.guess == 0;
      const float *src = P.sface[f][hold ? (int)(step % 3) : (int)((step + 1) % 3)] + (long long)b * n;
      for (long long m = m0 + tid; m < m1; m += kPreThreads) {
        const float sv = src[m];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
          if (k0 + kk < P.rs) part[kk] += (double)(P.phis[f][(long long)(k0 + kk) * n + m] * sv);
      }
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) part[kk] += __shfl_xor(part[kk], o, 64);
    if (lane == 0)
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) red[wid][kk] = part[kk];
    __syncthreads();
    if (tid < 8 && k0 + tid < P.rs)
      P.gpart[((long long)gsi * P.batch + b) * P.rs + k0 + tid] =
          ((red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]));
    __syncthreads();
  }
}

hipError_t launch_rom_pre(const RomPreArgs &P, hipStream_t s) {
  if (P.nkba + P.nkbh > 0) {
    const dim3 grid(P.nrt * P.ks, P.nit);
    const size_t smem = sizeof(float) * 16 * (size_t)P.r;
    if (P.prec == 0) hipLaunchKernelGGL(rom_f0_kernel<0>, grid, dim3(kPreThreads), smem, s, P);
    else hipLaunchKernelGGL(rom_f0_kernel<1>, grid, dim3(kPreThreads), smem, s, P);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (P.nface > 0 && P.rs > 0) {
    hipLaunchKernelGGL(rom_ghat_kernel, dim3(P.gs, P.batch), dim3(kPreThreads), 0, s, P);
    return hipGetLastError();
  }
  return hipSuccess;
}

}  // namespace osam
