// Matrix-free hex8 explicit Newmark step of one FOM subdomain (all instances),
// with the FP64 convergence sums of Eq. conv_criterion, the on-device controller
// decision, and the push of the next-step displacement to the neighbours' faces.
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
//  * One thread owns a node column (ix, iy) and marches up a chunk of z-layers
//    with a rolling two-layer window: 27 loads per node, 150 non-zero FMAs per
//    interior node (structural zeros of the isotropic stencil are skipped at
//    compile time).  Interior columns and the boundary columns (grouped by
//    stencil case, padded to whole waves) run in separate workgroups, so every
//    wave reads one coefficient block through scalar loads.
//  * The displacement at t_k on free nodes is the Newmark predictor, which the
//    previous step already produced (buffer P); an iteration reads P, V0, A0
//    and the previous iterate's V1, and writes V1, A1 and the next predictor
//    P2 = P + dt V1 + dt^2/2 A1.  Face layers of P / U0 hold the neighbour's
//    pushed values.  No atomics on data; FP64 norm partials are summed in a
//    fixed order by the last workgroup (deterministic).
//  * Buffer roles rotate with the instance's accepted-step count, so each
//    instance advances at its own pace and the host never waits per step.
#include "osam_device.hpp"

namespace osam {

constexpr int kModeStep = 0;
constexpr int kModeInit = 1;

// Isotropic stencil on a box grid, interior node: the (p, q) block entry of
// offset d vanishes when p != q and d_p == 0 or d_q == 0 (mirror symmetry).
__host__ __device__ constexpr int d27_axis(int d27, int p) {
  return p == 0 ? d27 % 3 - 1 : (p == 1 ? (d27 % 9) / 3 - 1 : d27 / 9 - 1);
}
__host__ __device__ constexpr bool interior_zero(int d27, int p, int q) {
  return p != q && (d27_axis(d27, p) == 0 || d27_axis(d27, q) == 0);
}

// 3x3 neighbourhood of node layer L (SoA buffer P, component stride cs).
template <typename T, bool INTERIOR>
__device__ __forceinline__ void load_layer(T (&w)[9][3], const T *P, long long cs, int L, int npl,
                                           int nxp, int ix, int iy, int nx, int ny) {
#pragma unroll
  for (int n = 0; n < 9; ++n) {
    int jx = ix + n % 3 - 1, jy = iy + n / 3 - 1;
    if (!INTERIOR) {
      jx = jx < 0 ? 0 : (jx > nx ? nx : jx);
      jy = jy < 0 ? 0 : (jy > ny ? ny : jy);
    }
    const T *p = P + (long long)L * npl + (jx + nxp * jy);
#pragma unroll
    for (int c = 0; c < 3; ++c) w[n][c] = p[c * cs];
  }
}

// Contribution of one z-slab (dz = DZ) of the 27-point stencil to the node
// whose own value is ctr: acc += sum_n C_(dx,dy,DZ) (w[n] - ctr).
template <typename T, bool INTERIOR, int DZ>
__device__ __forceinline__ void slab(const T (&w)[9][3], const T (&ctr)[3], const T *C, T (&acc)[3]) {
#pragma unroll
  for (int n = 0; n < 9; ++n) {
    const int d27 = (DZ + 1) * 9 + n;
    if (d27 == 13) continue;
    const int d26 = d27 < 13 ? d27 : d27 - 1;
    const T du[3] = {w[n][0] - ctr[0], w[n][1] - ctr[1], w[n][2] - ctr[2]};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (INTERIOR && interior_zero(d27, p, q)) continue;
        acc[p] += C[d26 * 9 + p * 3 + q] * du[q];
      }
    }
  }
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

template <typename T, int MODE, bool INTERIOR>
__device__ __forceinline__ void fe_columns(const FeArgs<T> &A, int b, int t, int chunk, long long step,
                                           int iter, double &acc_abs, double &acc_den) {
  const int nx = A.nx, ny = A.ny, nxp = nx + 1, npl = A.npl, nzs = A.nzs;
  const long long cs = A.cs;
  const long long boff = (long long)b * A.is;
  const int s3 = (int)(step % 3), s2 = (int)(step % 2);
  // roles: U0 = u[s%3], P = u[(s+1)%3], P2 = u[(s+2)%3]; V0 = v[s%2], V1 = v[(s+1)%2]
  const int rP = (s3 + 1) % 3, rP2 = (s3 + 2) % 3;
  T *U0 = A.u[s3] + boff;
  T *P = A.u[rP] + boff;
  T *P2 = A.u[rP2] + boff;
  T *V0 = A.v[s2] + boff, *V1 = A.v[1 - s2] + boff;
  T *A0 = A.a[s2] + boff, *A1 = A.a[1 - s2] + boff;
  const int n_iter = iter + 1;

  int ix, iy, cse;
  if (INTERIOR) {
    if (t >= A.n_int) return;
    ix = 1 + t % (nx - 1);
    iy = 1 + t / (nx - 1);
    cse = 4;
  } else {
    if (t >= A.n_bnd) return;
    const int col = A.bnd_cols[t];
    if (col < 0) return;   // padding of a case group
    ix = col % nxp;
    iy = col / nxp;
    // every wave holds one case group: make the case (and the coefficient block) wave-uniform
    cse = __builtin_amdgcn_readfirstlane((ix == 0 ? 0 : (ix == nx ? 2 : 1)) + 3 * (iy == 0 ? 0 : (iy == ny ? 2 : 1)));
  }
  const T *C = A.coef + cse * 234;

  // Face layers: HOLD at iteration 1 when the source comes later in the sweep
  // reads the neighbour's value at t_{k-1} (role U0), otherwise at t_k (role P).
  const T *Pin = (MODE == kModeInit) ? U0 : P;
  const T *Flo = Pin, *Fhi = Pin;
  if (MODE == kModeStep && n_iter == 1 && A.opts.guess == 0) {
    if (A.face_src[0] > A.sd) Flo = U0;
    if (A.face_src[1] > A.sd) Fhi = U0;
  }
  const int k0 = 1 + chunk * A.kc;
  const int k1 = min(k0 + A.kc, nzs);
  const int nid0 = ix + nxp * iy;

  // rolling window: cur = layer k, nxt = layer k+1; acc holds the partial force
  // of layer k from layers k-1 and k until layer k+1 arrives.
  T cur[9][3], nxt[9][3], acc[3], ctr[3];
  load_layer<T, INTERIOR>(nxt, k0 == 1 ? Flo : Pin, cs, k0 - 1, npl, nxp, ix, iy, nx, ny);
  load_layer<T, INTERIOR>(cur, Pin, cs, k0, npl, nxp, ix, iy, nx, ny);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    ctr[c] = cur[4][c];
    acc[c] = T(0);
  }
  slab<T, INTERIOR, -1>(nxt, ctr, C, acc);
  slab<T, INTERIOR, 0>(cur, ctr, C, acc);

  const long long rcol = (MODE == kModeInit) ? 0 : (step + 1) / (A.rec_every > 0 ? A.rec_every : 1);
  const bool rec = A.rec_every > 0 && rcol < A.rec_ncols &&
                   (MODE == kModeInit || ((step + 1) % A.rec_every) == 0);
  const long long rbase = ((long long)b * A.rec_ncols + rcol) * 3 * A.nfree_nodes;
  if (rec && A.rec_s && k0 == 1 && A.face_src[0] >= 0) {
    const long long so = ((long long)b * A.rec_ncols + rcol) * 3 * A.nsch_nodes;
#pragma unroll
    for (int c = 0; c < 3; ++c) A.rec_s[so + (long long)c * A.nsch_nodes + nid0] = nxt[4][c];
  }

  for (int k = k0; k < k1; ++k) {
    // keep the stencil coefficients out of registers: re-read every layer
    __asm__ volatile("" ::: "memory");
    load_layer<T, INTERIOR>(nxt, k + 1 == nzs ? Fhi : Pin, cs, k + 1, npl, nxp, ix, iy, nx, ny);
    slab<T, INTERIOR, 1>(nxt, ctr, C, acc);
    const long long id = (long long)k * npl + nid0;
    T out[3];   // value pushed to neighbours: the displacement at the next step
    if (MODE == kModeInit) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T a1 = acc[c];
        const T u0 = ctr[c];
        const T v0 = V0[c * cs + id];
        A0[c * cs + id] = a1;
        out[c] = u0 + A.dt * v0 + A.half_dt2 * a1;
        P[c * cs + id] = out[c];
        if (rec) {
          const long long ro = rbase + (long long)c * A.nfree_nodes + (long long)(k - 1) * npl + nid0;
          if (A.rec_u) A.rec_u[ro] = u0;
          if (A.rec_a) A.rec_a[ro] = a1;
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T a1 = acc[c];
        const T p = ctr[c];
        const T v0 = V0[c * cs + id];
        const T a0 = A0[c * cs + id];
        const T v1 = v0 + A.half_dt * (a0 + a1);
        double dlt;
        if (n_iter >= 2) {
          const T v1old = V1[c * cs + id];
          dlt = (double)A.dt * ((double)v1 - (double)v1old);
        } else {
          // iterate 0 = state at t_{k-1} (only tested when min_iter = 1)
          const T u0 = U0[c * cs + id];
          dlt = ((double)p - (double)u0) + (double)A.dt * ((double)v1 - (double)v0);
        }
        acc_abs += dlt * dlt;
        const double den = (double)p + (double)A.dt * (double)v1;
        acc_den += den * den;
        V1[c * cs + id] = v1;
        A1[c * cs + id] = a1;
        out[c] = p + A.dt * v1 + A.half_dt2 * a1;
        P2[c * cs + id] = out[c];
        if (rec) {
          const long long ro = rbase + (long long)c * A.nfree_nodes + (long long)(k - 1) * npl + nid0;
          if (A.rec_u) A.rec_u[ro] = p;
          if (A.rec_a) A.rec_a[ro] = a1;
        }
      }
    }
    // push to the faces fed by this layer (next-step role: P2, or P when initialising)
    for (int e = 0; e < A.npush; ++e) {
      const PushDev<T> &Pd = A.push[e];
      if (Pd.layer != k) continue;
      T *dst = Pd.role[MODE == kModeInit ? rP : rP2] + (long long)b * Pd.is + nid0;
#pragma unroll
      for (int c = 0; c < 3; ++c) dst[c * Pd.cs] = out[c];
    }
    if (k + 1 < k1) {
      // start layer k+1: contributions of layers k (dz = -1) and k+1 (dz = 0)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        ctr[c] = nxt[4][c];
        acc[c] = T(0);
      }
      slab<T, INTERIOR, -1>(cur, ctr, C, acc);
      slab<T, INTERIOR, 0>(nxt, ctr, C, acc);
#pragma unroll
      for (int n = 0; n < 9; ++n)
#pragma unroll
        for (int c = 0; c < 3; ++c) cur[n][c] = nxt[n][c];
    }
  }
  if (rec && A.rec_s && k1 == nzs && A.face_src[1] >= 0) {
    const long long so = ((long long)b * A.rec_ncols + rcol) * 3 * A.nsch_nodes;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      A.rec_s[so + (long long)c * A.nsch_nodes + A.face_off_hi + nid0] = nxt[4][c];
  }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(256) fe_kernel(FeArgs<T> A) {
  const int b = blockIdx.y;
  Status *stp = A.status + b;
  const int flags = stp->flags;
  if (MODE == kModeStep && (flags & kFinished)) return;
  if (MODE == kModeInit && !(flags & kNeedInit)) return;
  const long long step = stp->step;
  const int iter = stp->iter;

  double acc_abs = 0.0, acc_den = 0.0;
  const int bx = blockIdx.x;
  if (bx < A.int_blocks * A.n_chunks) {
    const int t = (bx % A.int_blocks) * blockDim.x + threadIdx.x;
    fe_columns<T, MODE, true>(A, b, t, bx / A.int_blocks, step, iter, acc_abs, acc_den);
  } else {
    const int bb = bx - A.int_blocks * A.n_chunks;
    const int nbb = A.nblocks / A.n_chunks - A.int_blocks;
    const int t = (bb % nbb) * blockDim.x + threadIdx.x;
    fe_columns<T, MODE, false>(A, b, t, bb / nbb, step, iter, acc_abs, acc_den);
  }
  if (MODE == kModeInit) return;

  // deterministic block reduction of the two FP64 sums
  __shared__ double red[2][16];
  __shared__ int is_last;
  acc_abs = wave_sum(acc_abs);
  acc_den = wave_sum(acc_den);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) {
    red[0][wid] = acc_abs;
    red[1][wid] = acc_den;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sd = 0.0;
    for (int i = 0; i < nw; ++i) {
      sa += red[0][i];
      sd += red[1][i];
    }
    double *pp = A.partials + ((long long)b * A.nblocks + bx) * 2;
    pp[0] = sa;
    pp[1] = sd;
    __threadfence();
    const unsigned prev = __hip_atomic_fetch_add(A.counters + b, 1u, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    is_last = (prev == (unsigned)(A.nblocks - 1));
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  // last workgroup of this instance: sum the partials in a fixed order
  double sa = 0.0, sd = 0.0;
  const double *pp = A.partials + (long long)b * A.nblocks * 2;
  for (int i = threadIdx.x; i < A.nblocks; i += blockDim.x) {
    sa += __builtin_nontemporal_load(pp + 2 * i);
    sd += __builtin_nontemporal_load(pp + 2 * i + 1);
  }
  sa = wave_sum(sa);
  sd = wave_sum(sd);
  __syncthreads();
  if (lane == 0) {
    red[0][wid] = sa;
    red[1][wid] = sd;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, td = 0.0;
    for (int i = 0; i < nw; ++i) {
      ta += red[0][i];
      td += red[1][i];
    }
    Status &S = *stp;
    S.sd_abs2[A.sd] = ta;
    S.sd_den2[A.sd] = td;
    A.counters[b] = 0u;
    decide(S, A.sd, A.opts);
    __threadfence();
  }
}

// Host-side launcher -------------------------------------------------------
template <typename T>
hipError_t launch_fe(const FeArgs<T> &A, int batch, int block, int mode, hipStream_t s) {
  dim3 grid(A.nblocks, batch);
  if (mode == kModeInit)
    hipLaunchKernelGGL((fe_kernel<T, kModeInit>), grid, dim3(block), 0, s, A);
  else
    hipLaunchKernelGGL((fe_kernel<T, kModeStep>), grid, dim3(block), 0, s, A);
  return hipGetLastError();
}

template hipError_t launch_fe<float>(const FeArgs<float> &, int, int, int, hipStream_t);
template hipError_t launch_fe<double>(const FeArgs<double> &, int, int, int, hipStream_t);

}  // namespace osam
