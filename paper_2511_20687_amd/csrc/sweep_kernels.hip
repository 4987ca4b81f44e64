// One Schwarz sweep (Alg. 1 inner loop) of every subdomain in a single launch.
//
// Within a sweep no step kernel reads what another writes: every source pushes
// its next-step displacement into the buffer role of the next step, which no
// kernel of the sweep reads, and the convergence sums go to separate partial
// buffers.  So the FOM step (fe_body) and the OpInf step (rom_body) of all
// subdomains can run side by side: subdomain i owns the workgroups
// [off_i, off_i + nblk_i) of one grid (OpInf steps first), and a finisher reduces
// the sums and takes the decision of Eq. conv_criterion.  Results equal those of
// separate launches; the sweep costs one dispatch and the longest subdomain
// instead of the sum of them.
#include <hip/hip_ext.h>

#include "fe_body.hpp"
#include "rom_body.hpp"

namespace osam {

// FE: 0 no FOM subdomain in the sweep, 1 one node layer per thread, 2 several.
// V: the OpInf body's variant, what every OpInf subdomain of the sweep allows.
template <typename T, int FE, int V>
__global__ void __launch_bounds__(kRomThreads) sweep_kernel(SweepArgs<T> S) {
  int x = blockIdx.x, i = 0;
  while (i + 1 < S.n && x >= S.nblk[i]) x -= S.nblk[i++];
  if (FE == 0 || S.rom_idx[i] >= 0) rom_body<T, V>(S.rom[S.rom_idx[i]], x);
  else fe_body<T, kModeStep, FE == 1, true, false>(S.fe[S.fe_idx[i]], x);
}

// FP64: one FE layer per thread only (fe != 2).
template <typename T, int V>
static bool launch_sweep_v(const SweepArgs<T> &S, dim3 grid, int fe, size_t smem, hipStream_t s, hipEvent_t ev0,
                           hipEvent_t ev1) {
  const dim3 block(kRomThreads);
  if (fe == 0) hipExtLaunchKernelGGL((sweep_kernel<T, 0, V>), grid, block, (uint32_t)smem, s, ev0, ev1, 0, S);
  else if (fe == 1) hipExtLaunchKernelGGL((sweep_kernel<T, 1, V>), grid, block, (uint32_t)smem, s, ev0, ev1, 0, S);
  else if constexpr (sizeof(T) == 4)
    hipExtLaunchKernelGGL((sweep_kernel<T, 2, V>), grid, block, (uint32_t)smem, s, ev0, ev1, 0, S);
  else return false;
  return true;
}

template <typename T>
hipError_t launch_sweep(const SweepArgs<T> &S, int batch, bool one, size_t smem, hipStream_t s, hipEvent_t ev0,
                        hipEvent_t ev1) {
  int total = 0, v = kRomPre | kRomNoPushRegs, nfe = 0;
  for (int i = 0; i < S.n; ++i) {
    total += S.nblk[i];
    if (S.rom_idx[i] >= 0) v &= rom_variant(S.rom[S.rom_idx[i]]);
    else ++nfe;
  }
  const int fe = nfe == 0 ? 0 : (one ? 1 : 2);
  if (total <= 0 || smem > 65536) return hipErrorInvalidValue;
  const dim3 grid(total, batch);
  bool ok;
  if constexpr (sizeof(T) == 8) {   // the batched parts are FP32 only
    if (v & kRomNoPushRegs) ok = launch_sweep_v<T, kRomNoPushRegs>(S, grid, fe, smem, s, ev0, ev1);
    else ok = launch_sweep_v<T, 0>(S, grid, fe, smem, s, ev0, ev1);
  } else {
    if (v == 3) ok = launch_sweep_v<T, 3>(S, grid, fe, smem, s, ev0, ev1);
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
