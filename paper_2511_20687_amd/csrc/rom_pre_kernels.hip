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
//    fragment order, so every wave reads one contiguous block per instruction
//    and applies it to up to 4 tiles of 16 instances; H's K blocks are padded
//    per row i of the compressed triangle, so z = q_i q_j is formed on the fly
//    from the predictor staged in LDS with a wave-uniform (i, j0) per block.
//    K is split over workgroups; each split writes its own partial tile (no
//    atomics), reduced in a fixed order by the step kernel.
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
// K blocks per wave and round (FP32 blocks are 4 wide, BF16 16 wide); the next
// round's fragments are in flight while a round computes
template <int PREC>
constexpr int kPreUnroll = PREC == 0 ? 16 : 8;

// Fragments of the K blocks kb = base, base + 4, ... (wave-strided) of one
// round, A blocks (HP = false) or H blocks (HP = true); indices past the range
// are clamped into it (their products are never accumulated), so every load is
// issued without a branch and stays in flight while the previous round computes.
template <int PREC, bool HP>
struct Frags {
  float a[kPreUnroll<PREC>];    // FP32 operand (A blocks; H blocks when PREC == 0)
  s4_t h[kPreUnroll<PREC>];     // BF16 operand (H blocks when PREC == 1)
  int ij[kPreUnroll<PREC>];     // H block: row i of the triangle | first column j0 << 16
};

template <int PREC, bool HP>
__device__ __forceinline__ void load_frags(const RomPreArgs &P, int rt, int base, int hi, int lane,
                                           Frags<PREC, HP> &F) {
#pragma unroll
  for (int u = 0; u < kPreUnroll<PREC>; ++u) {
    const int kb = min(base + 4 * u, hi - 1);   // wave-uniform
    if (!HP) {
      F.a[u] = P.frag_a[((long long)rt * P.nkba + kb) * 64 + lane];
    } else {
      const int kh = kb - P.nkba;
      F.ij[u] = P.blocks[kh];
      if (PREC == 0) F.a[u] = reinterpret_cast<const float *>(P.frag_h)[((long long)rt * P.nkbh + kh) * 64 + lane];
      else F.h[u] = reinterpret_cast<const s4_t *>(P.frag_h)[((long long)rt * P.nkbh + kh) * 64 + lane];
    }
  }
}

// acc[n] += M[rows of tile rt][K blocks lo .. hi-1 of this wave] z[.., tile n]
template <int PREC, int NI, bool HP>
__device__ __forceinline__ void mfma_range(const RomPreArgs &P, const float *q1s, int rt, int lo, int hi, int wid,
                                           int lane, f4_t (&acc)[NI]) {
  const int r = P.r, col = lane & 15, g4 = lane >> 4;
  if (lo + wid >= hi) return;
  Frags<PREC, HP> cur, nxt;
  load_frags<PREC, HP>(P, rt, lo + wid, hi, lane, nxt);
  for (int base = lo + wid; base < hi; base += 4 * kPreUnroll<PREC>) {
    cur = nxt;
    if (base + 4 * kPreUnroll<PREC> < hi) load_frags<PREC, HP>(P, rt, base + 4 * kPreUnroll<PREC>, hi, lane, nxt);
#pragma unroll
    for (int u = 0; u < kPreUnroll<PREC>; ++u) {
      const int kb = base + 4 * u;
      if (kb >= hi) break;
      if (!HP) {   // linear part, FP32 operands
        const int k = kb * 4 + g4;
#pragma unroll
        for (int n = 0; n < NI; ++n) {
          const float z = k < r ? q1s[(n * 16 + col) * r + min(k, r - 1)] : 0.f;
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur.a[u], z, acc[n], 0, 0, 0);
        }
      } else {
        const int i = cur.ij[u] & 0xffff, j0 = cur.ij[u] >> 16;
#pragma unroll
        for (int n = 0; n < NI; ++n) {
          const float *qc = q1s + (n * 16 + col) * r;
          const float qi = qc[i];
          if (PREC == 0) {
            const int j = j0 + g4;
            const float z = j < r ? qi * qc[min(j, r - 1)] : 0.f;
            acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur.a[u], z, acc[n], 0, 0, 0);
          } else {
            s4_t z;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              const int j = j0 + 4 * g4 + jj;
              z[jj] = to_bf16(j < r ? qi * qc[min(j, r - 1)] : 0.f);
            }
            acc[n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(cur.h[u], z, acc[n], 0, 0, 0);
          }
        }
      }
    }
  }
}

// Grid (row tiles x K splits, instance groups of NI tiles of 16).  Every wave
// takes every fourth K block of its split and applies each fragment of M to
// the NI instance tiles; K block kb of H covers columns j0 .. j0 + 3 (FP32) or
// j0 .. j0 + 15 (BF16) of row i of the triangle (rows padded to whole blocks),
// so z = q_i q_j needs no per-lane index table.
template <int PREC, int NI>
__device__ __forceinline__ void f0_body(const RomPreArgs &P, int bxl) {
  const int b0 = blockIdx.y * NI * 16;
  const int rt = bxl % P.nrt, ksi = bxl / P.nrt;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  extern __shared__ float q1s[];   // [NI * 16][r]: the predictor of the group's instances
  __shared__ int start[NI * 16];   // instance starts a step: its f0 partials are written

  // this group's status (loads in flight during the staging below)
  int flags = kFinished, iter = 1;
  if (tid < NI * 16 && b0 + tid < P.batch) {
    const Status &S = P.status[b0 + tid];
    flags = S.flags;
    iter = S.iter;
  }
  // the group's predictors are contiguous ([batch rounded up to 64][r], 16-byte aligned)
  const int r = P.r, n4 = NI * 4 * r;
  const float4 *qp = reinterpret_cast<const float4 *>(P.qpred + (long long)b0 * r);
#pragma unroll 8
  for (int i4 = tid; i4 < n4; i4 += kPreThreads) reinterpret_cast<float4 *>(q1s)[i4] = qp[i4];
  // only when some instance of the group starts a step
  const bool need = tid < NI * 16 && !(flags & kFinished) && iter == 0;
  if (tid < NI * 16) start[tid] = need;
  if (!__syncthreads_or(need)) return;

  const int nkb = P.nkba + P.nkbh;
  const int per = (nkb + P.ks - 1) / P.ks;
  const int kb0 = ksi * per, kb1 = min(nkb, kb0 + per);
  const int col = lane & 15, g4 = lane >> 4;
  f4_t acc[NI];
#pragma unroll
  for (int n = 0; n < NI; ++n) acc[n] = f4_t{0.f, 0.f, 0.f, 0.f};
  mfma_range<PREC, NI, false>(P, q1s, rt, kb0, min(kb1, P.nkba), wid, lane, acc);   // A blocks
  mfma_range<PREC, NI, true>(P, q1s, rt, max(kb0, P.nkba), kb1, wid, lane, acc);    // H blocks
  __syncthreads();   // the predictor is no longer read: its LDS takes the wave sums
  f4_t *red = reinterpret_cast<f4_t *>(q1s);   // [4 waves][NI][64]
#pragma unroll
  for (int n = 0; n < NI; ++n) red[(wid * NI + n) * 64 + lane] = acc[n];
  __syncthreads();
  if (wid < NI) {
    const int n = wid;
    f4_t t = red[n * 64 + lane];
#pragma unroll
    for (int w = 1; w < 4; ++w) t += red[(w * NI + n) * 64 + lane];
    // result register i of lane l: row 4 (l / 16) + i, column (instance) l % 16
    const int b = b0 + n * 16 + col;
    if (b < P.batch && start[n * 16 + col]) {   // instances within a step keep their f0
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rt * 16 + 4 * g4 + i;
        if (row < r) {
          float v = t[i];
          if (ksi == 0 && P.c) v += P.c[row];
          P.f0part[((long long)ksi * P.batch + b) * r + row] = v;
        }
      }
    }
  }
}

template <int PREC, int NI>
__global__ void __launch_bounds__(kPreThreads) rom_f0_kernel(RomPreArgs P) {
  f0_body<PREC, NI>(P, blockIdx.x);
}

// f0 of several OpInf subdomains in one launch: subdomain i owns the next
// nrt * ks workgroups of the grid (x)
struct RomPreMulti {
  int n;
  RomPreArgs p[2];
};

template <int PREC, int NI>
__global__ void __launch_bounds__(kPreThreads) rom_f0_multi_kernel(RomPreMulti M) {
  const int n0 = M.p[0].nrt * M.p[0].ks;
  if ((int)blockIdx.x < n0) f0_body<PREC, NI>(M.p[0], blockIdx.x);
  else f0_body<PREC, NI>(M.p[1], blockIdx.x - n0);
}

size_t rom_f0_smem_bytes(int r, int ni) {
  const size_t q = sizeof(float) * 16 * (size_t)ni * r, red = sizeof(f4_t) * 4 * (size_t)ni * 64;
  return q > red ? q : red;
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
      const bool hold = n_iter == 1 && (P.fsrc[f] > P.sd || P.opts.additive) && P.opts.guess == 0;
      const float *src = P.sface[f][hold ? (int)(step % 3) : (int)((step + 1) % 3)] + (long long)b * n;
      for (long long m = m0 + tid; m < m1; m += kPreThreads) {
        const float sv = src[m];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
          if (k0 + kk < P.rs) part[kk] += (double)(P.phis[f][(long long)(k0 + kk) * n + m] * sv);
      }
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) part[kk] = wave_total(part[kk]);
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

template <int PREC>
static void launch_f0(const RomPreArgs &P, dim3 grid, size_t smem, hipStream_t s) {
  if (P.ni == 4) hipLaunchKernelGGL((rom_f0_kernel<PREC, 4>), grid, dim3(kPreThreads), smem, s, P);
  else if (P.ni == 2) hipLaunchKernelGGL((rom_f0_kernel<PREC, 2>), grid, dim3(kPreThreads), smem, s, P);
  else hipLaunchKernelGGL((rom_f0_kernel<PREC, 1>), grid, dim3(kPreThreads), smem, s, P);
}

template <int PREC>
static void launch_f0_multi(const RomPreMulti &M, dim3 grid, size_t smem, hipStream_t s) {
  const int ni = M.p[0].ni;
  if (ni == 4) hipLaunchKernelGGL((rom_f0_multi_kernel<PREC, 4>), grid, dim3(kPreThreads), smem, s, M);
  else if (ni == 2) hipLaunchKernelGGL((rom_f0_multi_kernel<PREC, 2>), grid, dim3(kPreThreads), smem, s, M);
  else hipLaunchKernelGGL((rom_f0_multi_kernel<PREC, 1>), grid, dim3(kPreThreads), smem, s, M);
}

// The batched parts of n (1 or 2) OpInf subdomains of one context: the f0
// contractions in one launch when both have one (same precision and instance
// grouping), then the g^ splits of each.
hipError_t launch_rom_pre_multi(const RomPreArgs *P, int n, hipStream_t s) {
  if (n == 2 && P[0].nkba + P[0].nkbh > 0 && P[1].nkba + P[1].nkbh > 0 && P[0].prec == P[1].prec &&
      P[0].ni == P[1].ni && P[0].nit == P[1].nit) {
    RomPreMulti M;
    M.n = 2;
    size_t smem = 0;
    for (int i = 0; i < 2; ++i) {
      if (!(P[i].ni == 1 || P[i].ni == 2 || P[i].ni == 4) || P[i].ni * 4 * P[i].r > 16 * kPreThreads)
        return hipErrorInvalidValue;
      M.p[i] = P[i];
      smem = std::max(smem, rom_f0_smem_bytes(P[i].r, P[i].ni));
    }
    if (smem > 65536) return hipErrorInvalidValue;
    const dim3 grid(P[0].nrt * P[0].ks + P[1].nrt * P[1].ks, (P[0].nit + P[0].ni - 1) / P[0].ni);
    if (P[0].prec == 0) launch_f0_multi<0>(M, grid, smem, s);
    else launch_f0_multi<1>(M, grid, smem, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int i = 0; i < 2; ++i)
      if (P[i].nface > 0 && P[i].rs > 0) {
        hipLaunchKernelGGL(rom_ghat_kernel, dim3(P[i].gs, P[i].batch), dim3(kPreThreads), 0, s, P[i]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
    return hipSuccess;
  }
  for (int i = 0; i < n; ++i) {
    const hipError_t e = launch_rom_pre(P[i], s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_rom_pre(const RomPreArgs &P, hipStream_t s) {
  if (P.nkba + P.nkbh > 0) {
    if (!(P.ni == 1 || P.ni == 2 || P.ni == 4) || P.ni * 4 * P.r > 16 * kPreThreads) return hipErrorInvalidValue;
    const size_t smem = rom_f0_smem_bytes(P.r, P.ni);
    if (smem > 65536) return hipErrorInvalidValue;
    const dim3 grid(P.nrt * P.ks, (P.nit + P.ni - 1) / P.ni);
    if (P.prec == 0) launch_f0<0>(P, grid, smem, s);
    else launch_f0<1>(P, grid, smem, s);
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
