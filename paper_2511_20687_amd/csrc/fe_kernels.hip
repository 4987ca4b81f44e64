// Matrix-free hex8 explicit Newmark step of one FOM subdomain (all instances),
// with the FP64 convergence sums of Eq. conv_criterion and the push of the
// next-step displacement to the neighbours' faces.
//
// Method: Sec. 2 (lumped-mass Galerkin hex8, Eq. matrix_vector_form_with_dbcs)
// and Sec. 4.1 (explicit Newmark-beta, beta = 0, gamma = 1/2; Schwarz data on
// d_S Omega_i by pointwise projection, an injection on the conforming slabs).
// One controller step = one Newmark step.
//
// Design (gfx950):
//  * On a uniform box grid the assembled stiffness row of a node is a 27-point
//    stencil of 3x3 blocks K_d that depends only on which of the 8 surrounding
//    elements exist (9 cases in the x-y cross-section: interior, 4 faces,
//    4 edges; z-layers 1..nzs-1 always have elements above and below).  The
//    host folds -1/m (lumped mass) into the blocks: a = sum_d C_d (u_{i+d} - u_i).
//    Relative displacements keep FP32 accurate (the rows of K sum to zero).
//  * The interior coefficient block travels in the kernel arguments, so it is
//    read with scalar loads and never occupies vector registers (150 of its 234
//    entries are used: the isotropic stencil's structural zeros are skipped at
//    compile time); the 8 boundary cases (edge columns only) read theirs from
//    memory.  Interior and boundary columns (grouped by case, padded to whole
//    waves) run in separate workgroups.
//  * Launch shape: a thread owns one node column and kc consecutive z-layers.
//    kc = 1 issues every load of the node (three 3x3 neighbourhoods, the state)
//    at once, one memory round trip per node; kc > 1 marches a rolling
//    two-layer window up the column (fewer loads per node, one round trip per
//    layer).  Workgroups are renumbered so each XCD gets a contiguous range of
//    z-chunks and neighbouring layers meet in the same L2.
//  * The displacement at t_k on free nodes is the Newmark predictor, which the
//    previous step already produced (buffer P); an iteration reads P, V0, A0
//    and the previous iterate's V1, and writes V1, A1 and the next predictor
//    P2 = P + dt V1 + dt^2/2 A1.  Face layers of P / U0 hold the neighbour's
//    pushed values.  No atomics or fences: every workgroup stores one pair of
//    FP64 partial sums, reduced in a fixed order after the sweep.
//  * Buffer roles rotate with the instance's accepted-step count, so each
//    instance advances at its own pace and the host never waits per step.
#include <hip/hip_ext.h>

#include "fe_body.hpp"

namespace osam {

template <typename T, int MODE, bool ONE>
__global__ void __launch_bounds__(256) fe_kernel(FeArgs<T> A) {
  fe_body<T, MODE, ONE>(A, blockIdx.x);
}

// Layer-staged variant for the interior columns (FP32, cross-sections up to
// kLdsMaxNodes nodes; the boundary columns go to the column kernel in a
// launch of their own): one workgroup of kLdsThreads threads owns kc
// consecutive free layers of one instance and the whole x-y cross-section.
// Every displacement layer is read from memory once, with coalesced loads,
// into one of three LDS slots (layers k-1, k, k+1), and the 27-point
// neighbourhoods come from LDS, so the texture units see one request per value
// instead of one per neighbour.  Layer k+2 is in flight while layer k is
// computed, and each node's state loads are issued one node ahead.
constexpr int kLdsThreads = 1024;
constexpr int kLdsPer = 5;                                     // nodes of a layer per thread
constexpr int kLdsMaxNodes = kFeLdsMaxNodes;                   // 4535: 3 slots x 3 components in 160 KB
static_assert(kLdsMaxNodes <= kLdsPer * kLdsThreads, "layer share");

template <int MODE>
__global__ void __launch_bounds__(kLdsThreads) fe_lds_kernel(FeArgs<float> A) {
  const int total = A.nblocks * (int)gridDim.y;
  const int logical = xcd_block(blockIdx.x + (int)gridDim.x * blockIdx.y, total);
  const int b = logical / A.nblocks, chunk = logical - b * A.nblocks;
  const Status *stp = A.status + b;
  const int flags = stp->flags;
  if (MODE == kModeStep && (flags & kFinished)) return;
  if (MODE == kModeInit && !(flags & kNeedInit)) return;
  const long long step = stp->step;
  const int n_iter = stp->iter + 1;
  const Roles<float> R = roles<float, MODE>(A, b, step, n_iter);
  const int nx = A.nx, nxp = nx + 1, npl = A.npl, nzs = A.nzs;
  const int k0 = 1 + chunk * A.kc, k1 = min(k0 + A.kc, nzs);
  const int tid = threadIdx.x;
  const int nval = 3 * npl;
  extern __shared__ float lds[];   // [3 slots][3 components][npl]
  const Strides B = strides(A);

  // layer L through registers into its LDS slot (faces 0 and nzs come from the face roles)
  float pre[3][kLdsPer];
  auto issue = [&](int L) {
    const Field<float> F(L == 0 ? R.Flo : (L == nzs ? R.Fhi : R.Pin));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const unsigned so = (unsigned)L * B.npl + c * B.cs;
#pragma unroll
      for (int j = 0; j < kLdsPer; ++j) pre[c][j] = F.ld((unsigned)min(tid + j * kLdsThreads, npl - 1) * 4u, so);
    }
  };
  auto store = [&](int L) {
    float *S = lds + (L % 3) * nval;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int j = 0; j < kLdsPer; ++j) {
        const int e = tid + j * kLdsThreads;
        if (e < npl) S[c * npl + e] = pre[c][j];
      }
  };
  // interior column w = ix - 1 + (nx - 1)(iy - 1): division by a float reciprocal, corrected
  const float inv = 1.0f / (float)(nx - 1);
  auto column = [&](int w) {
    int q = (int)((float)w * inv), r = w - q * (nx - 1);
    if (r < 0) {
      --q;
      r += nx - 1;
    } else if (r >= nx - 1) {
      ++q;
      r -= nx - 1;
    }
    return (r + 1) + nxp * (q + 1);
  };

  long long rcol = 0, rbase = 0;
  bool rec = false;
  if (A.rec_every > 0) {
    rcol = (MODE == kModeInit ? step : step + 1) / A.rec_every;   // the state this launch completes
    rec = rcol < A.rec_ncols && ((MODE == kModeInit ? step : step + 1) % A.rec_every) == 0;
    rbase = ((long long)b * A.rec_ncols + rcol) * 3 * A.nfree_nodes;
  }

  // pipeline: LDS <- layers k0-1, k0, k0+1; registers <- layer k0+2
  issue(k0 - 1);
  store(k0 - 1);
  issue(k0);
  store(k0);
  issue(k0 + 1);
  store(k0 + 1);
  if (k0 + 1 < k1) issue(k0 + 2);
  __syncthreads();

  double acc_abs = 0.0, acc_den = 0.0;
  for (int k = k0; k < k1; ++k) {
    const float *Sl = lds + ((k - 1) % 3) * nval, *Sc = lds + (k % 3) * nval, *Sh = lds + ((k + 1) % 3) * nval;
    // one column at a time; the next column's state loads are issued before this one is computed
    int nnid = column(tid);
    float nv0[3], na0[3], nold[3];
    if (tid < A.n_int) state_loads<float, MODE, true>(R, B, k, nnid, n_iter, nv0, na0, nold);
#pragma unroll 1
    for (int w = tid; w < A.n_int; w += kLdsThreads) {
      const int nid0 = nnid;
      float v0[3], a0[3], old[3], ctr[3], acc[3], wc[9][3];
      float sm[3] = {0.f, 0.f, 0.f}, s0[3] = {0.f, 0.f, 0.f}, sp[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        v0[c] = nv0[c];
        a0[c] = na0[c];
        old[c] = nold[c];
      }
      if (w + kLdsThreads < A.n_int) {
        nnid = column(w + kLdsThreads);
        state_loads<float, MODE, true>(R, B, k, nnid, n_iter, nv0, na0, nold);
      }
      // the centre row of layer k (columns x-1, x, x+1), then the x-resolved sums slab by slab
#pragma unroll
      for (int rx = 0; rx < 3; ++rx)
#pragma unroll
        for (int c = 0; c < 3; ++c) wc[3 + rx][c] = Sc[c * npl + nid0 + rx - 1];
#pragma unroll
      for (int c = 0; c < 3; ++c) ctr[c] = wc[4][c];
#pragma unroll
      for (int dz = -1; dz <= 1; ++dz) {
        const float *S = (dz < 0 ? Sl : (dz == 0 ? Sc : Sh)) + nid0;
        float wv[9][3];
#pragma unroll
        for (int n = 0; n < 9; ++n)
#pragma unroll
          for (int c = 0; c < 3; ++c) wv[n][c] = S[c * npl + (n / 3 - 1) * nxp + (n % 3 - 1)];
        xslab<float>(A.cb, dz + 1, wv, wc, sm, s0, sp);
        __builtin_amdgcn_sched_barrier(0);   // one slab of neighbours live at a time
      }
#pragma unroll
      for (int p = 0; p < 3; ++p) acc[p] = x_combine(s0[p], sm[p], sp[p], kx_diag(A.cb, p), wc[3][p], ctr[p], wc[5][p]);
      if (rec && A.rec_s && ((k == 1 && A.face_src[0] >= 0) || (k == nzs - 1 && A.face_src[1] >= 0))) {
        float wf[9][3];
        const float *S = k == 1 ? Sl : Sh;
#pragma unroll
        for (int c = 0; c < 3; ++c) wf[4][c] = S[c * npl + nid0];
        record_face<float>(A, b, k == 1 ? 0 : 1, nid0, wf, rcol);
      }
      update_node<float, MODE, true>(A, R, b, k, nid0, ctr, acc, v0, a0, old, n_iter, rec, rbase, acc_abs, acc_den);
    }
    if (k + 1 < k1) {
      __syncthreads();              // every column of layer k is done with slot (k-1) % 3
      store(k + 2);                 // layer k+2 (already in registers) takes that slot
      if (k + 2 < k1) issue(k + 3);
      __syncthreads();
    }
  }
  if (MODE == kModeInit) return;

  __shared__ double red[2][kLdsThreads / 64];
  acc_abs = wave_sum(acc_abs);
  acc_den = wave_sum(acc_den);
  const int lane = tid & 63, wid = tid >> 6;
  if (lane == 0) {
    red[0][wid] = acc_abs;
    red[1][wid] = acc_den;
  }
  __syncthreads();
  if (tid == 0) {
    double sa = 0.0, sd = 0.0;
    for (int i = 0; i < kLdsThreads / 64; ++i) {
      sa += red[0][i];
      sd += red[1][i];
    }
    double *pp = A.partials + ((long long)b * A.part_stride + A.part_off + chunk) * 2;
    pp[0] = sa;
    pp[1] = sd;
  }
}

__global__ void __launch_bounds__(64) finish_kernel(const Status *in, Status *out, FinishArgs F, Opts o) {
  finish_sweep(in, out, F, o, blockIdx.x);
}

hipError_t launch_finish(const Status *in, Status *out, const FinishArgs &F, const Opts &o, int batch,
                         hipStream_t s) {
  hipLaunchKernelGGL(finish_kernel, dim3(batch), dim3(64), 0, s, in, out, F, o);
  return hipGetLastError();
}

// Host-side launcher -------------------------------------------------------
// ev0/ev1 (optional): events stamped with the kernel's own start and end.
template <typename T>
hipError_t launch_fe(const FeArgs<T> &A, int batch, int block, int mode, hipStream_t s, hipEvent_t ev0,
                     hipEvent_t ev1) {
  if (block == kLdsThreads) {
    if constexpr (sizeof(T) != 4) {
      return hipErrorInvalidValue;
    } else {
      const size_t smem = sizeof(float) * 9 * (size_t)A.npl;
      if (A.npl > kLdsMaxNodes) return hipErrorInvalidValue;
      if (smem > 64 * 1024) {   // dynamic LDS beyond the default limit must be requested
        const void *f = mode == kModeInit ? (const void *)fe_lds_kernel<kModeInit> : (const void *)fe_lds_kernel<kModeStep>;
        const hipError_t ea = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (ea != hipSuccess) return ea;
      }
      const dim3 grid(A.nblocks, batch);
      if (mode == kModeInit)
        hipExtLaunchKernelGGL(fe_lds_kernel<kModeInit>, grid, dim3(kLdsThreads), smem, s, ev0, ev1, 0, A);
      else
        hipExtLaunchKernelGGL(fe_lds_kernel<kModeStep>, grid, dim3(kLdsThreads), smem, s, ev0, ev1, 0, A);
      return hipGetLastError();
    }
  }
  dim3 grid(A.nblocks, batch);
  const bool one = A.kc == 1;
  if (mode == kModeInit) {
    if (one) hipExtLaunchKernelGGL((fe_kernel<T, kModeInit, true>), grid, dim3(block), 0, s, ev0, ev1, 0, A);
    else hipExtLaunchKernelGGL((fe_kernel<T, kModeInit, false>), grid, dim3(block), 0, s, ev0, ev1, 0, A);
  } else {
    if (one) hipExtLaunchKernelGGL((fe_kernel<T, kModeStep, true>), grid, dim3(block), 0, s, ev0, ev1, 0, A);
    else hipExtLaunchKernelGGL((fe_kernel<T, kModeStep, false>), grid, dim3(block), 0, s, ev0, ev1, 0, A);
  }
  return hipGetLastError();
}

template hipError_t launch_fe<float>(const FeArgs<float> &, int, int, int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_fe<double>(const FeArgs<double> &, int, int, int, hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace osam
