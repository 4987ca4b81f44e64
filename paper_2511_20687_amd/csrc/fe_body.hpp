// Device code of the FE explicit-step kernel (see fe_kernels.hip): per-node
// update, column marching and the workgroup body, shared by the step kernel
// and the fused sweep kernel.
#pragma once
#include <hip/hip_runtime.h>

#include "osam_device.hpp"
#include "stencil.hpp"

namespace osam {

constexpr int kModeStep = 0;
constexpr int kModeInit = 1;

__device__ __forceinline__ double wave_sum(double x) { return wave_total(x); }

// Per-thread view of one instance's buffers in the roles of its current step.
template <typename T>
struct Roles {
  T *U0, *P, *P2, *V0, *V1, *A0, *A1;
  const T *Pin, *Flo, *Fhi;
  int rP, rP2;
};

template <typename T, int MODE>
__device__ __forceinline__ Roles<T> roles(const FeArgs<T> &A, int b, long long step, int n_iter) {
  Roles<T> R;
  const long long boff = (long long)b * A.is;
  const int s3 = (int)(step % 3), s2 = (int)(step % 2);
  // U0 = u[s%3], P = u[(s+1)%3], P2 = u[(s+2)%3]; V0 = v[s%2], V1 = v[(s+1)%2]
  R.rP = (s3 + 1) % 3;
  R.rP2 = (s3 + 2) % 3;
  R.U0 = A.u[s3] + boff;
  R.P = A.u[R.rP] + boff;
  R.P2 = A.u[R.rP2] + boff;
  R.V0 = A.v[s2] + boff;
  R.V1 = A.v[1 - s2] + boff;
  R.A0 = A.a[s2] + boff;
  R.A1 = A.a[1 - s2] + boff;
  // Face layers: HOLD at iteration 1 when the source has not advanced in this
  // iteration (it comes later in the sweep, or every source in the additive
  // variant) reads the neighbour's value at t_{k-1} (role U0), otherwise at t_k
  // (role P; with the explicit step a source's t_k displacement is fixed by its
  // state at t_{k-1}, so later iterations read the same data in either variant).
  R.Pin = (MODE == kModeInit) ? R.U0 : R.P;
  R.Flo = R.Pin;
  R.Fhi = R.Pin;
  if (MODE == kModeStep && n_iter == 1 && A.opts.guess == 0) {
    if (A.face_src[0] > A.sd || A.opts.additive) R.Flo = R.U0;
    if (A.face_src[1] > A.sd || A.opts.additive) R.Fhi = R.U0;
  }
  return R;
}

template <typename T>
__device__ __forceinline__ Strides strides(const FeArgs<T> &A) {
  return Strides{(unsigned)(A.cs * (long long)sizeof(T)), (unsigned)A.npl * (unsigned)sizeof(T),
                 (unsigned)(A.nx + 1) * (unsigned)sizeof(T)};
}

// Newmark update of node (layer k, column nid0) from its acceleration, with
// the convergence sums, records and pushes.
// UK: the layer k is wave-uniform (its offset goes into the scalar offset of the
// buffer accesses); otherwise every lane has its own layer (boundary waves that
// hold several layers) and the layer offset goes into the per-lane offset.
template <typename T, int MODE, bool UK>
__device__ __forceinline__ void update_node(const FeArgs<T> &A, const Roles<T> &R, int b, int k, int nid0,
                                            const T (&ctr)[3], const T (&acc)[3], const T (&v0)[3],
                                            const T (&a0)[3], const T (&old)[3], int n_iter, bool rec,
                                            long long rbase, double &acc_abs, double &acc_den) {
  const Strides B = strides(A);
  const unsigned vo = (unsigned)nid0 * (unsigned)sizeof(T) + (UK ? 0u : (unsigned)k * B.npl);
  T out[3];   // value pushed to neighbours: the displacement at the next step
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T a1 = acc[c];
    const unsigned so = (UK ? (unsigned)k * B.npl : 0u) + c * B.cs;   // wave-uniform part of the offset
    if (MODE == kModeInit) {
      Field<T>(R.A0).st(a1, vo, so);
      out[c] = ctr[c] + A.dt * v0[c] + A.half_dt2 * a1;
      Field<T>(R.P).st(out[c], vo, so);
    } else {
      const T p = ctr[c];
      const T v1 = v0[c] + A.half_dt * (a0[c] + a1);
      double dlt;
      if (n_iter >= 2)
        dlt = (double)A.dt * ((double)v1 - (double)old[c]);   // old = previous iterate's V1
      else   // iterate 0 = state at t_{k-1} (only tested when min_iter = 1); old = U0
        dlt = ((double)p - (double)old[c]) + (double)A.dt * ((double)v1 - (double)v0[c]);
      acc_abs += dlt * dlt;
      const double den = (double)p + (double)A.dt * (double)v1;
      acc_den += den * den;
      Field<T>(R.V1).st(v1, vo, so);
      Field<T>(R.A1).st(a1, vo, so);
      out[c] = p + A.dt * v1 + A.half_dt2 * a1;
      Field<T>(R.P2).st(out[c], vo, so);
    }
    if (rec) {
      const long long ro = rbase + (long long)c * A.nfree_nodes + (long long)(k - 1) * A.npl + nid0;
      if (A.rec_u) A.rec_u[ro] = ctr[c];
      if (A.rec_a) A.rec_a[ro] = a1;
    }
  }
  // push to the faces fed by this layer (next-step role: P2, or P when initialising)
  for (int e = 0; e < A.npush; ++e) {
    const PushDev<T> &Pd = A.push[e];
    if (Pd.layer != k) continue;
    T *dst = Pd.role[MODE == kModeInit ? R.rP : R.rP2] + (long long)b * Pd.is + nid0;
#pragma unroll
    for (int c = 0; c < 3; ++c) dst[c * Pd.cs] = out[c];
  }
}

template <typename T>
__device__ __forceinline__ void record_face(const FeArgs<T> &A, int b, int f, int nid0, const T (&w)[9][3],
                                            long long rcol) {
  const long long so = ((long long)b * A.rec_ncols + rcol) * 3 * A.nsch_nodes + (f ? A.face_off_hi : 0);
#pragma unroll
  for (int c = 0; c < 3; ++c) A.rec_s[so + (long long)c * A.nsch_nodes + nid0] = w[4][c];
}

template <typename T>
__device__ __forceinline__ void record_face_value(const FeArgs<T> &A, int b, int f, int nid0, const T (&u)[3],
                                                  long long rcol) {
  const long long so = ((long long)b * A.rec_ncols + rcol) * 3 * A.nsch_nodes + (f ? A.face_off_hi : 0);
#pragma unroll
  for (int c = 0; c < 3; ++c) A.rec_s[so + (long long)c * A.nsch_nodes + nid0] = u[c];
}

// v0, a0 and the previous iterate (V1, or U0 at the first iteration) of one node.
template <typename T, int MODE, bool UK>
__device__ __forceinline__ void state_loads(const Roles<T> &R, const Strides &B, int k, int nid0, int n_iter,
                                            T (&v0)[3], T (&a0)[3], T (&old)[3]) {
  const unsigned vo = (unsigned)nid0 * (unsigned)sizeof(T) + (UK ? 0u : (unsigned)k * B.npl);
  const Field<T> FV(R.V0), FA(R.A0), FO(n_iter >= 2 ? R.V1 : R.U0);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const unsigned so = (UK ? (unsigned)k * B.npl : 0u) + c * B.cs;
    v0[c] = FV.ld(vo, so);
    a0[c] = MODE == kModeInit ? T(0) : FA.ld(vo, so);
    old[c] = MODE == kModeInit ? T(0) : FO.ld(vo, so);
  }
}

// One layer's 3x3 neighbourhood: interior columns through wave-uniform row bases,
// boundary columns (clamped indices) through per-lane addresses.
// XS: interior rows shared across lanes (load_layer_xshare).
// xf (boundary, wave-uniform): the columns are on an x-face (load_layer_xface, FP32), else on
// a y-face (load_layer_yface, FP32).
template <typename T, bool INTERIOR, bool XS = false>
__device__ __forceinline__ void layer(T (&w)[9][3], const T *P, const Strides &B, long long cs, int L, int npl,
                                      int nxp, int ix, int iy, int nx, int ny, int nid0, bool xf = false) {
  if (INTERIOR && XS) load_layer_xshare<T>(w, P, B, L, (unsigned)(nid0 - nxp) * (unsigned)sizeof(T));
  else if (INTERIOR) load_layer_uniform<T>(w, P, B, L, (unsigned)(nid0 - nxp - 1) * (unsigned)sizeof(T));
  else if constexpr (sizeof(T) == 4) {
    if (xf) load_layer_xface(w, P, cs, L, npl, nxp, ix, iy, nx, ny);
    else load_layer_yface(w, P, cs, L, npl, nxp, ix, iy, ny);
  } else load_layer<T, false>(w, P, cs, L, npl, nxp, ix, iy, nx, ny);
}

// One layer k of the x-shared interior layout in x-resolved form (xrow): lane j
// forms S_dx(j) from its own x-centred values and node i takes S_-1 and S_+1
// from lanes i-1 and i+1 (DPP wave shifts), so only 3-vectors cross lanes and no
// 3x3 neighbourhood is held in registers.  Every lane of the wave takes part
// (t: see fe_columns, XS).
template <typename T, int MODE>
__device__ __forceinline__ void fe_xs_one(const FeArgs<T> &A, int b, int t, int k, long long step, int iter,
                                          double &acc_abs, double &acc_den) {
  const int nx = A.nx, ny = A.ny, nxp = nx + 1, nzs = A.nzs;
  const int n_iter = iter + 1;
  const int nf = (ny - 1) * nxp, f = min(max(t, 0), nf - 1), lane = threadIdx.x & 63;
  const int ix = f % nxp;
  const bool act = t == f && lane >= 1 && lane <= 62 && ix >= 1 && ix < nx;
  const Roles<T> R = roles<T, MODE>(A, b, step, n_iter);
  const int nid0 = f + nxp;   // ix + nxp * iy with iy = 1 + f / nxp
  const Strides B = strides(A);
  long long rcol = 0, rbase = 0;
  bool rec = false;
  if (A.rec_every > 0) {
    rcol = (MODE == kModeInit ? step : step + 1) / A.rec_every;   // the state this launch completes
    rec = rcol < A.rec_ncols && ((MODE == kModeInit ? step : step + 1) % A.rec_every) == 0;
    rbase = ((long long)b * A.rec_ncols + rcol) * 3 * A.nfree_nodes;
  }
  const unsigned voff = (unsigned)f * (unsigned)sizeof(T);   // (nid0 - nxp) bytes
  T x[3][3][3], v0[3], a0[3], old[3];   // x[dz][dy][c] at this lane's x
  load_rows<T>(x[0], k == 1 ? R.Flo : R.Pin, B, k - 1, voff);
  load_rows<T>(x[1], R.Pin, B, k, voff);
  load_rows<T>(x[2], k + 1 == nzs ? R.Fhi : R.Pin, B, k + 1, voff);
  state_loads<T, MODE, true>(R, B, k, nid0, n_iter, v0, a0, old);
  if (act && rec && A.rec_s) {
    if (k == 1 && A.face_src[0] >= 0) record_face_value<T>(A, b, 0, nid0, x[0][1], rcol);
    if (k == nzs - 1 && A.face_src[1] >= 0) record_face_value<T>(A, b, 1, nid0, x[2][1], rcol);
  }
  T ctr[3], sm[3], s0[3], sp[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    ctr[c] = x[1][1][c];
    sm[c] = s0[c] = sp[c] = T(0);
  }
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      if (dz == 1 && dy == 1) continue;   // the node's own row: u_row(j) - u(j) = 0
      const T du[3] = {x[dz][dy][0] - ctr[0], x[dz][dy][1] - ctr[1], x[dz][dy][2] - ctr[2]};
      xrow<T>(A.cb, dz * 9 + dy * 3, du, sm);
      xrow<T>(A.cb, dz * 9 + dy * 3 + 1, du, s0);
      xrow<T>(A.cb, dz * 9 + dy * 3 + 2, du, sp);
    }
  T acc[3];
#pragma unroll
  for (int p = 0; p < 3; ++p)
    acc[p] = x_combine(s0[p], lane_prev(sm[p]), lane_next(sp[p]), kx_diag(A.cb, p), lane_prev(ctr[p]), ctr[p],
                       lane_next(ctr[p]));
  if (!act) return;
  update_node<T, MODE, true>(A, R, b, k, nid0, ctr, acc, v0, a0, old, n_iter, rec, rbase, acc_abs, acc_den);
}

// Column t (interior index, or entry of the boundary list), layers k0 .. k1-1
// (ONE: the single layer k0, every load issued at once).  Interior waves have
// one k0; a boundary wave may give each lane its own k0.
// XS (interior only): t indexes the nodes of rows 1 .. ny-1 including their
// boundary columns, 62 per wave from lane 1 (lanes 0 and 63 and the boundary
// columns only supply x-neighbours); every lane runs through, and only lanes
// of interior nodes store.
template <typename T, int MODE, bool INTERIOR, bool ONE, bool UK = INTERIOR, bool XS = false>
__device__ __forceinline__ void fe_columns(const FeArgs<T> &A, int b, int t, int k0, long long step,
                                           int iter, double &acc_abs, double &acc_den) {
  if constexpr (INTERIOR && XS && ONE) {
    fe_xs_one<T, MODE>(A, b, t, k0, step, iter, acc_abs, acc_den);
    return;
  }
  const int nx = A.nx, ny = A.ny, nxp = nx + 1, npl = A.npl, nzs = A.nzs;
  const long long cs = A.cs;
  const int n_iter = iter + 1;
  int ix, iy, cse;
  bool act = true;   // this lane's node is updated
  if (INTERIOR && XS) {
    const int nf = (ny - 1) * nxp, f = min(max(t, 0), nf - 1), lane = threadIdx.x & 63;
    ix = f % nxp;
    iy = 1 + f / nxp;
    cse = 4;
    act = t == f && lane >= 1 && lane <= 62 && ix >= 1 && ix < nx;
  } else if (INTERIOR) {
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
  const bool xf = !INTERIOR && cse % 3 != 1;   // x-face columns (wave-uniform)
  const Roles<T> R = roles<T, MODE>(A, b, step, n_iter);
  const int k1 = ONE ? k0 + 1 : min(k0 + A.kc, nzs);
  const int nid0 = ix + nxp * iy;
  const Strides B = strides(A);

  // records (the division only when recording is on)
  long long rcol = 0, rbase = 0;
  bool rec = false;
  if (A.rec_every > 0) {
    rcol = (MODE == kModeInit ? step : step + 1) / A.rec_every;   // the state this launch completes
    rec = rcol < A.rec_ncols && ((MODE == kModeInit ? step : step + 1) % A.rec_every) == 0;
    rbase = ((long long)b * A.rec_ncols + rcol) * 3 * A.nfree_nodes;
  }

  if (ONE) {
    const int k = k0;
    T w0[9][3], w1[9][3], w2[9][3], v0[3], a0[3], old[3], acc[3], ctr[3];
    layer<T, INTERIOR, XS>(w0, k == 1 ? R.Flo : R.Pin, B, cs, k - 1, npl, nxp, ix, iy, nx, ny, nid0, xf);
    layer<T, INTERIOR, XS>(w1, R.Pin, B, cs, k, npl, nxp, ix, iy, nx, ny, nid0, xf);
    layer<T, INTERIOR, XS>(w2, k + 1 == nzs ? R.Fhi : R.Pin, B, cs, k + 1, npl, nxp, ix, iy, nx, ny, nid0, xf);
    state_loads<T, MODE, UK>(R, B, k, nid0, n_iter, v0, a0, old);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ctr[c] = w1[4][c];
      acc[c] = T(0);
    }
    if (INTERIOR) {
      T sm[3] = {T(0), T(0), T(0)}, s0[3] = {T(0), T(0), T(0)}, sp[3] = {T(0), T(0), T(0)};
      xslab<T>(A.cb, 0, w0, w1, sm, s0, sp);
      xslab<T>(A.cb, 1, w1, w1, sm, s0, sp);
      xslab<T>(A.cb, 2, w2, w1, sm, s0, sp);
#pragma unroll
      for (int p = 0; p < 3; ++p) acc[p] = x_combine(s0[p], sm[p], sp[p], kx_diag(A.cb, p), w1[3][p], ctr[p], w1[5][p]);
    } else {
      slab<T, -1>(C, w0, ctr, acc, A.skip_rows);
      slab<T, 0>(C, w1, ctr, acc, A.skip_rows);
      slab<T, 1>(C, w2, ctr, acc, A.skip_rows);
    }
    if (!act) return;
    update_node<T, MODE, UK>(A, R, b, k, nid0, ctr, acc, v0, a0, old, n_iter, rec, rbase, acc_abs, acc_den);
    if (rec && A.rec_s) {
      if (k == 1 && A.face_src[0] >= 0) record_face<T>(A, b, 0, nid0, w0, rcol);
      if (k == nzs - 1 && A.face_src[1] >= 0) record_face<T>(A, b, 1, nid0, w2, rcol);
    }
    return;
  }

  // rolling window: cur = layer k, nxt = layer k+1; acc holds the partial force
  // of layer k from layers k-1 and k until layer k+1 arrives.
  // (interior: the x-resolved sums sm, s0, sp instead of acc until layer k+1 arrives)
  T cur[9][3], nxt[9][3], acc[3], ctr[3], sm[3], s0[3], sp[3];
  layer<T, INTERIOR, XS>(nxt, k0 == 1 ? R.Flo : R.Pin, B, cs, k0 - 1, npl, nxp, ix, iy, nx, ny, nid0, xf);
  layer<T, INTERIOR, XS>(cur, R.Pin, B, cs, k0, npl, nxp, ix, iy, nx, ny, nid0, xf);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    ctr[c] = cur[4][c];
    acc[c] = sm[c] = s0[c] = sp[c] = T(0);
  }
  if (INTERIOR) {
    xslab<T>(A.cb, 0, nxt, cur, sm, s0, sp);
    xslab<T>(A.cb, 1, cur, cur, sm, s0, sp);
  } else {
    slab<T, -1>(C, nxt, ctr, acc, A.skip_rows);
    slab<T, 0>(C, cur, ctr, acc, A.skip_rows);
  }
  if (act && rec && A.rec_s && k0 == 1 && A.face_src[0] >= 0) record_face<T>(A, b, 0, nid0, nxt, rcol);

  for (int k = k0; k < k1; ++k) {
    T v0[3], a0[3], old[3];
    state_loads<T, MODE, UK>(R, B, k, nid0, n_iter, v0, a0, old);
    layer<T, INTERIOR, XS>(nxt, k + 1 == nzs ? R.Fhi : R.Pin, B, cs, k + 1, npl, nxp, ix, iy, nx, ny, nid0, xf);
    if (INTERIOR) {
      xslab<T>(A.cb, 2, nxt, cur, sm, s0, sp);
#pragma unroll
      for (int p = 0; p < 3; ++p) acc[p] = x_combine(s0[p], sm[p], sp[p], kx_diag(A.cb, p), cur[3][p], ctr[p], cur[5][p]);
    } else {
      slab<T, 1>(C, nxt, ctr, acc, A.skip_rows);
    }
    if (act)
      update_node<T, MODE, UK>(A, R, b, k, nid0, ctr, acc, v0, a0, old, n_iter, rec, rbase, acc_abs, acc_den);
    if (k + 1 < k1) {
      // start layer k+1: contributions of layers k (dz = -1) and k+1 (dz = 0)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        ctr[c] = nxt[4][c];
        acc[c] = sm[c] = s0[c] = sp[c] = T(0);
      }
      if (INTERIOR) {
        xslab<T>(A.cb, 0, cur, nxt, sm, s0, sp);
        xslab<T>(A.cb, 1, nxt, nxt, sm, s0, sp);
      } else {
        slab<T, -1>(C, cur, ctr, acc, A.skip_rows);
        slab<T, 0>(C, nxt, ctr, acc, A.skip_rows);
      }
#pragma unroll
      for (int n = 0; n < 9; ++n)
#pragma unroll
        for (int c = 0; c < 3; ++c) cur[n][c] = nxt[n][c];
    }
  }
  if (act && rec && A.rec_s && k1 == nzs && A.face_src[1] >= 0) record_face<T>(A, b, 1, nid0, nxt, rcol);
}

// Fixed-order workgroup reduction of the two FP64 sums into the workgroup's
// partial slot; the sweep's finisher adds the partials (no fences or atomics).
template <typename T>
__device__ __forceinline__ void store_partials(const FeArgs<T> &A, int b, int bx, double acc_abs, double acc_den) {
  __shared__ double red[2][16];
  acc_abs = wave_sum(acc_abs);
  acc_den = wave_sum(acc_den);
  const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
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
    double *pp = A.partials + ((long long)b * A.part_stride + A.part_off + bx) * 2;
    pp[0] = sa;
    pp[1] = sd;
  }
}

// PACKB: boundary waves may hold several layer chunks (A.bnd_l > 1, fused
// sweeps); otherwise every wave has one layer chunk and one wave-uniform layer.
// XSOK: the x-shared interior layout (A.xs) is compiled in (fused sweeps: with one layer
// per thread only).
// st (optional): flags, step and iteration of the status this step starts from, when the
// caller holds them (folded decisions of fused sweeps); else read from A.status[b].
template <typename T, int MODE, bool ONE, bool PACKB = false, bool XSOK = true>
__device__ __forceinline__ void fe_body(const FeArgs<T> &A, int xblk, const StepState *st = nullptr) {
  const int b = blockIdx.y;
  const Status *stp = A.status + b;
  const int flags = st ? st->flags : stp->flags;
  if (MODE == kModeStep && (flags & kFinished)) return;
  if (MODE == kModeInit && !(flags & kNeedInit)) return;
  const long long step = st ? st->step : stp->step;
  const int iter = st ? st->iter : stp->iter;

  double acc_abs = 0.0, acc_den = 0.0;
  const int bx = xcd_block(xblk, A.nblocks);
  // work by wave, in super-chunks of A.bnd_l layer chunks (the grid order is
  // layer order, so every XCD gets its share of both kinds): per super-chunk of
  // cs chunks, wi groups of 64 interior columns per chunk, then the boundary:
  // case group g of n columns takes, per wave, L = min(64 / n, A.bnd_l) chunks
  // of its columns when n < 64 (one lane range per chunk, each lane its own
  // layers; fewer waves, but every load touches up to L times more lines),
  // else 64 of its columns in one chunk
  // interior waves per chunk: 64 interior columns each, or (A.xs) 62 nodes of
  // the rows 1 .. ny-1 counted with their boundary columns
  const bool xs = XSOK && A.xs;
  const int wi = xs ? ((A.ny - 1) * (A.nx + 1) + 61) / 62 : (A.n_int + 63) >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(bx * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int bl = PACKB ? A.bnd_l : 1;
  auto bnd_waves = [&](int cs) {   // boundary waves of a super-chunk of cs chunks
    int w = 0;
    for (int g = 0; g < A.nbg; ++g) {
      const int ng = A.bg_n[g], L = min(64 / ng, bl);
      w += ng >= 64 ? ((ng + 63) >> 6) * cs : (cs + L - 1) / L;
    }
    return w;
  };
  const int nsc = (A.n_chunks + bl - 1) / bl;
  const int wfull = wi * bl + bnd_waves(bl);
  const int sc = min(wave / wfull, nsc - 1);
  const int c0 = sc * bl, cs = min(bl, A.n_chunks - c0);
  int v = wave - sc * wfull;
  if (v < wi * cs) {
    const int chunk = c0 + v / wi, wc = v - (v / wi) * wi;
    if (XSOK && xs)
      fe_columns<T, MODE, true, ONE, true, XSOK>(A, b, wc * 62 + lane - 1, 1 + chunk * A.kc, step, iter, acc_abs,
                                                 acc_den);
    else
      fe_columns<T, MODE, true, ONE>(A, b, wc * 64 + lane, 1 + chunk * A.kc, step, iter, acc_abs, acc_den);
  } else {
    v -= wi * cs;
    int t = -1, k0 = 0;
    for (int g = 0; g < A.nbg; ++g) {
      const int ng = A.bg_n[g];
      if (ng >= 64) {
        const int per = (ng + 63) >> 6, nw = per * cs;
        if (v < nw) {
          const int chunk = v / per, col = (v - chunk * per) * 64 + lane;
          if (col < ng) {
            t = A.bg_start[g] + col;
            k0 = 1 + (c0 + chunk) * A.kc;
          }
          break;
        }
        v -= nw;
      } else {
        const int L = min(64 / ng, bl), nw = (cs + L - 1) / L;
        if (v < nw) {
          const int lb = lane / ng, chunk = v * L + lb;
          if (lb < L && chunk < cs) {
            t = A.bg_start[g] + lane - lb * ng;
            k0 = 1 + (c0 + chunk) * A.kc;
          }
          break;
        }
        v -= nw;
      }
    }
    if (t >= 0) {
      if (PACKB) fe_columns<T, MODE, false, ONE, false>(A, b, t, k0, step, iter, acc_abs, acc_den);
      else fe_columns<T, MODE, false, ONE, true>(A, b, t, __builtin_amdgcn_readfirstlane(k0), step, iter, acc_abs, acc_den);
    }
  }
  if (MODE == kModeInit) return;
  store_partials(A, b, bx, acc_abs, acc_den);
}

}  // namespace osam
