// One Schwarz sweep (Alg. 1 inner loop) of every subdomain in a single launch.
//
// Within a sweep no step kernel reads what another writes: every source pushes
// its next-step displacement into the buffer role of the next step, which no
// kernel of the sweep reads, and the convergence sums go to separate partial
// buffers.  So the FOM step (fe_body) and the OpInf step (rom_body) of all
// subdomains can run side by side: subdomain i owns the workgroups
// [off_i, off_i + nblk_i) of one grid (OpInf steps first), and a finisher reduces
// the sums and takes the decision of Eq. conv_criterion (in graph mode the next
// sweep's workgroups take it themselves, see SweepArgs).  Results equal those of
// separate launches; the sweep costs one dispatch and the longest subdomain
// instead of the sum of them.
#include <hip/hip_ext.h>

#include "fe_body.hpp"
#include "rom_body.hpp"

namespace osam {

// FE: 0 no FOM subdomain in the sweep, 1 one node layer per thread, 2 several.
// V: the OpInf body's variant, what every OpInf subdomain of the sweep allows.
// The previous sweep's decision, taken by every workgroup (folded decisions, see SweepArgs)
// on an LDS copy of the status, which keeps the registers of the step bodies free: the
// sums go into the copy one by one and decide() updates it in place (the finisher's
// arithmetic in the finisher's order).  Every thread of the workgroup calls it.
__device__ inline void fold_decision(const Status *prev, Status *next, const FinishArgs &F, const Opts &o,
                                     Status &cur) {
  constexpr int kWords = sizeof(Status) / 4;
  static_assert(sizeof(Status) % 4 == 0, "status is copied by 32-bit words");
  const int b = blockIdx.y, tid = threadIdx.x, lane = tid & 63;
  if (tid < kWords) reinterpret_cast<unsigned *>(&cur)[tid] = reinterpret_cast<const unsigned *>(prev + b)[tid];
  __syncthreads();
  if (tid < 64 && !(cur.flags & kFinished)) {
    for (int k = 0; k < F.nfom; ++k) {
      const double2 t = fom_sums<4>(F, k, b, lane);
      if (lane == 0) {
        cur.sd_abs2[F.sd[k]] = t.x;
        cur.sd_den2[F.sd[k]] = t.y;
      }
    }
    if (lane == 0) {
      for (int k = 0; k < F.nrom; ++k) {
        const int j = F.rom_sd[k];
        const double2 v = reinterpret_cast<const double2 *>(F.rom_sums)[(long long)b * kMaxSd + j];
        cur.sd_abs2[j] = v.x;
        cur.sd_den2[j] = v.y;
      }
      decide(cur, o.nsd - 1, o);
    }
  }
  __syncthreads();
  if (blockIdx.x == 0 && tid < kWords)
    reinterpret_cast<unsigned *>(next + b)[tid] = reinterpret_cast<const unsigned *>(&cur)[tid];
}

// FOLD: the variant with folded decisions (S.fold set), a kernel of its own because the
// decision code in front of the step bodies changes their register allocation.
template <typename T, int FE, int V, bool FOLD>
__global__ void __launch_bounds__(kRomThreads) sweep_kernel(SweepArgs<T> S) {
  __shared__ Status cur;
  int x = blockIdx.x, i = 0;
  while (i + 1 < S.n && x >= S.nblk[i]) x -= S.nblk[i++];
  // the folded decision's result in scalar registers (workgroup-uniform values)
  auto folded = [&]() {
    fold_decision(S.st_prev, S.st_cur, S.prev, S.opts, cur);
    StepState ss;
    const unsigned long long su = (unsigned long long)cur.step;
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)su);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(su >> 32));
    ss.step = (long long)(((unsigned long long)hi << 32) | lo);
    ss.iter = __builtin_amdgcn_readfirstlane(cur.iter);
    ss.flags = __builtin_amdgcn_readfirstlane(cur.flags);
    return ss;
  };
  if (FE == 0 || S.rom_idx[i] >= 0) {
    // an OpInf step issues its operand loads before it takes the decision
    const RomArgs<T> &A = S.rom[S.rom_idx[i]];
    if (FOLD) rom_body<T, V>(A, x, folded);
    else rom_body<T, V>(A, x, StatusOf<T>{A});
  } else {
    StepState ss;
    const StepState *st = nullptr;
    if (FOLD) {
      ss = folded();
      st = &ss;
    }
    fe_body<T, kModeStep, FE == 1, true, FE == 1>(S.fe[S.fe_idx[i]], x, st);   // x-shared rows with one layer
  }
}

template <typename T, int V, bool FOLD>
static bool launch_sweep_f(const SweepArgs<T> &S, dim3 grid, int fe, size_t smem, hipStream_t s, hipEvent_t ev0,
                           hipEvent_t ev1) {
  const dim3 block(kRomThreads);
  if (fe == 0) hipExtLaunchKernelGGL((sweep_kernel<T, 0, V, FOLD>), grid, block, (uint32_t)smem, s, ev0, ev1, 0, S);
  else if (fe == 1) hipExtLaunchKernelGGL((sweep_kernel<T, 1, V, FOLD>), grid, block, (uint32_t)smem, s, ev0, ev1, 0, S);
  else hipExtLaunchKernelGGL((sweep_kernel<T, 2, V, FOLD>), grid, block, (uint32_t)smem, s, ev0, ev1, 0, S);
  return true;
}
template <typename T, int V>
static bool launch_sweep_v(const SweepArgs<T> &S, dim3 grid, int fe, size_t smem, hipStream_t s, hipEvent_t ev0,
                           hipEvent_t ev1) {
  return S.fold ? launch_sweep_f<T, V, true>(S, grid, fe, smem, s, ev0, ev1)
                : launch_sweep_f<T, V, false>(S, grid, fe, smem, s, ev0, ev1);
}

template <typename T>
hipError_t launch_sweep(const SweepArgs<T> &S, int batch, bool one, size_t smem, hipStream_t s, hipEvent_t ev0,
                        hipEvent_t ev1) {
  int total = 0, v = kRomPre | kRomNoPushRegs, nfe = 0;
  for (int i = 0; i < S.n; ++i) {
    total += S.nblk[i];
    if (S.rom_idx[i] >= 0) v = rom_variant_join(v, rom_variant(S.rom[S.rom_idx[i]]));
    else ++nfe;
  }
  const int fe = nfe == 0 ? 0 : (one ? 1 : 2);
  if (total <= 0 || smem > 65536) return hipErrorInvalidValue;
  const dim3 grid(total, batch);
  bool ok;
  if constexpr (sizeof(T) == 8) {   // the batched parts are FP32 only
    if (v & kRomNoPushRegs) ok = launch_sweep_v<T, kRomNoPushRegs>(S, grid, fe, smem, s, ev0, ev1);
    else if (v & kRomWide) ok = launch_sweep_v<T, kRomWide>(S, grid, fe, smem, s, ev0, ev1);
    else ok = launch_sweep_v<T, 0>(S, grid, fe, smem, s, ev0, ev1);
  } else {
    if (v == 5) ok = launch_sweep_v<T, 5>(S, grid, fe, smem, s, ev0, ev1);
    else if (v == 4) ok = launch_sweep_v<T, 4>(S, grid, fe, smem, s, ev0, ev1);
    else if (v == 3) ok = launch_sweep_v<T, 3>(S, grid, fe, smem, s, ev0, ev1);
    else if (v == 2) ok = launch_sweep_v<T, 2>(S, grid, fe, smem, s, ev0, ev1);
    else if (v == 1) ok = launch_sweep_v<T, 1>(S, grid, fe, smem, s, ev0, ev1);
    else ok = launch_sweep_v<T, 0>(S, grid, fe, smem, s, ev0, ev1);
  }
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

template hipError_t launch_sweep<float>(const SweepArgs<float> &, int, bool, size_t, hipStream_t, hipEvent_t,
                                        hipEvent_t);
template hipError_t launch_sweep<double>(const SweepArgs<double> &, int, bool, size_t, hipStream_t, hipEvent_t,
                                         hipEvent_t);

}  // namespace osam
