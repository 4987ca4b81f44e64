// Kernels of the window engine (window.hpp): one Newmark sub-step of a FOM or an
// OpInf subdomain inside a Schwarz iteration, with its Schwarz data taken from the
// neighbours' trajectories through the temporal interpolant Xi (Sec. 4.1), the
// convergence decision of Eq. conv_criterion and the acceptance of a step.
//
// One workgroup holds one instance of one subdomain for the whole sub-step, so
// the phases of the step (predictor and Schwarz data, force, the implicit solve,
// trajectory capture, norms) are separated by workgroup barriers and every
// reduction is a fixed-order workgroup sum.
#include <hip/hip_runtime.h>

#include "stencil.hpp"
#include "window.hpp"

namespace osam {

namespace {

// Sum over the workgroup, returned to every thread (fixed order: waves, then the
// per-wave totals in wave order).  Every thread must call it.
template <int NT>
__device__ __forceinline__ double block_sum(double x, double *red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  x = wave_total(x);
  if (lane == 0) red[w] = x;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

// Value of source S's accepted state (t_{k-1}) at face DOF m = c npl + nid; with
// pred, its Newmark displacement predictor tau later (u + tau v + tau^2/2 a).
template <typename T>
__device__ T src_accepted(const WinSrc<T> &S, int b, long long step, int m, T tau, bool pred) {
  if (S.kind == 1) {
    const int c = m / S.npl, nid = m - c * S.npl;
    const long long o = (long long)b * S.is + (long long)c * S.cs + (long long)S.layer * S.npl + nid;
    const T u = S.u[step % 3][o];
    if (!pred) return u;
    return u + tau * S.v[step & 1][o] + T(0.5) * tau * tau * S.a[step & 1][o];
  }
  const int n = 3 * S.npl;
  const T *q = S.q[step & 1] + (long long)b * S.r;
  const T *qd = S.qd[step & 1] + (long long)b * S.r;
  const T *qdd = S.qdd[step & 1] + (long long)b * S.r;
  T s = T(0);
  for (int k = 0; k < S.r; ++k) {
    const T x = pred ? q[k] + tau * qd[k] + T(0.5) * tau * tau * qdd[k] : q[k];
    s += S.rows[(long long)k * n + m] * x;
  }
  return s;
}

// Schwarz datum at face DOF m for the destination's sub-step l of n_dst (time
// t_{k-1} + l dt_dst).  n: Schwarz iteration (1-based); ready: the source has a
// trajectory to read (Alg. 1: it has run in this iteration, or in the previous
// one), from the buffer of iteration parity par.  Xi: linear interpolation in
// time between the source's trajectory points around the destination time (its
// own point when the times coincide, point 0 being the accepted state).  Before
// the source has run in a step, the initial guess: HOLD its accepted value,
// PREDICTOR its Newmark predictor at the destination time.
template <typename T>
__device__ T face_value(const WinSrc<T> &S, int b, long long step, int m, int l, int n_dst, T dt_dst, bool ready,
                        int par, int guess) {
  if (!ready) return src_accepted(S, b, step, m, T(l) * dt_dst, guess == 1);   // 1: PREDICTOR
  const int num = l * S.n_sub, m0 = num / n_dst, rem = num - m0 * n_dst;
  const long long slab = (long long)S.batch * 3 * S.npl, off = (long long)b * 3 * S.npl + m;
  auto pt = [&](int j) -> T {
    return j == 0 ? src_accepted(S, b, step, m, T(0), false) : S.traj[par][(long long)(j - 1) * slab + off];
  };
  if (rem == 0) return pt(m0);
  const T w = T(rem) / T(n_dst);
  return (T(1) - w) * pt(m0) + w * pt(m0 + 1);
}

// Iteration-parity buffer to read source j's trajectory from, for subdomain sd
// in iteration n (1-based); false when the source has not run yet in this step.
__device__ __forceinline__ bool src_ready(int j, int sd, int n, int additive, int &par) {
  const bool now = !additive && j < sd;   // multiplicative: already run in this iteration
  if (now) {
    par = n & 1;
    return true;
  }
  par = (n - 1) & 1;
  return n >= 2;
}

// -M^-1 K u at free node (k, ix, iy) of one instance (field U, component stride
// cs): the 27-point stencil sum_d C_d (u_{i+d} - u_i); interior nodes use the
// interior block's 27 distinct values, boundary columns their case block.
template <typename T>
__device__ __forceinline__ void node_force(const WinFomArgs<T> &A, const T *coef, const T *U, int k, int ix, int iy,
                                           T (&acc)[3]) {
  const int nx = A.nx, ny = A.ny, nxp = nx + 1, npl = A.npl;
  const long long cs = A.cs;
  T ctr[3];
  {
    const long long o = (long long)k * npl + ix + nxp * iy;
#pragma unroll
    for (int c = 0; c < 3; ++c) ctr[c] = U[c * cs + o];
  }
  acc[0] = acc[1] = acc[2] = T(0);
  const int cx = ix == 0 ? 0 : (ix == nx ? 2 : 1), cy = iy == 0 ? 0 : (iy == ny ? 2 : 1);
  const bool interior = cx == 1 && cy == 1;
  const T *C = coef + (cx + 3 * cy) * 234;
  // one z-slab (9 neighbours) at a time keeps the live values to a slab
#pragma unroll
  for (int dz = 0; dz < 3; ++dz) {
    T w[9][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int jx = min(max(ix + dx - 1, 0), nx), jy = min(max(iy + dy - 1, 0), ny);
        const long long o = (long long)(k + dz - 1) * npl + jx + nxp * jy;
#pragma unroll
        for (int c = 0; c < 3; ++c) w[dy * 3 + dx][c] = U[c * cs + o];
      }
#pragma unroll
    for (int n9 = 0; n9 < 9; ++n9) {
      const int d27 = dz * 9 + n9;
      if (d27 == 13) continue;
      const T d[3] = {w[n9][0] - ctr[0], w[n9][1] - ctr[1], w[n9][2] - ctr[2]};
      if (interior) {
        xrow<T>(A.cb, d27, d, acc);
      } else {
        const int d26 = d27 < 13 ? d27 : d27 - 1;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
          for (int q = 0; q < 3; ++q) acc[p] += C[d26 * 9 + p * 3 + q] * d[q];
      }
    }
  }
}

// -M^-1 f(u) at free node (k, ix, iy) for the Saint Venant-Kirchhoff material
// (App. A.2): f_a = sum over the node's elements and their 2x2x2 Gauss points of
// w det(J) P grad N_a, with F = I + grad u, E = (F^T F - I)/2, S = lam tr(E) I +
// 2 mu E, P = F S (total Lagrangian).  Box elements: dN_b/dX are products of
// the 1D factors (1 +- xi)/2 and +-1/h; det(J) = hx hy hz / 8, unit weights.
template <typename T>
__device__ __forceinline__ void node_force_svk(const WinFomArgs<T> &A, const T *U, int k, int ix, int iy,
                                               T (&acc)[3]) {
  const int nx = A.nx, ny = A.ny, nxp = nx + 1, npl = A.npl;
  const long long cs = A.cs;
  const T g = T(0.57735026918962576451);   // 1/sqrt(3)
  const T ih[3] = {T(1) / A.hx, T(1) / A.hy, T(1) / A.hz};
  const T wdet = A.hx * A.hy * A.hz / T(8);
  T f[3] = {T(0), T(0), T(0)};
  int nel = 0;
  for (int oz = 0; oz < 2; ++oz)
    for (int oy = 0; oy < 2; ++oy)
      for (int ox = 0; ox < 2; ++ox) {
        // element with lower corner (ix - 1 + ox, iy - 1 + oy, k - 1 + oz); this node is its corner (1-ox, 1-oy, 1-oz)
        const int ex = ix - 1 + ox, ey = iy - 1 + oy, ez = k - 1 + oz;
        if (ex < 0 || ex >= nx || ey < 0 || ey >= ny) continue;
        ++nel;
        const int ca[3] = {1 - ox, 1 - oy, 1 - oz};
        T ue[8][3];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const long long o = (long long)(ez + (b >> 2)) * npl + (ex + (b & 1)) + nxp * (ey + ((b >> 1) & 1));
#pragma unroll
          for (int c = 0; c < 3; ++c) ue[b][c] = U[c * cs + o];
        }
#pragma unroll
        for (int gp = 0; gp < 8; ++gp) {
          const T xi[3] = {(gp & 1) ? g : -g, ((gp >> 1) & 1) ? g : -g, (gp >> 2) ? g : -g};
          // 1D factors (1 + s xi)/2 per axis and corner coordinate d (s = 2d - 1)
          T h1[3][2], dh[2] = {T(-0.5), T(0.5)};
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) {
            h1[ax][0] = T(0.5) * (T(1) - xi[ax]);
            h1[ax][1] = T(0.5) * (T(1) + xi[ax]);
          }
          T Gu[3][3] = {};
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            const int d0 = b & 1, d1 = (b >> 1) & 1, d2 = b >> 2;
            const T dN[3] = {T(2) * dh[d0] * h1[1][d1] * h1[2][d2] * ih[0], T(2) * dh[d1] * h1[0][d0] * h1[2][d2] * ih[1],
                             T(2) * dh[d2] * h1[0][d0] * h1[1][d1] * ih[2]};
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int j = 0; j < 3; ++j) Gu[i][j] += ue[b][i] * dN[j];
          }
          T F[3][3], E[3][3];
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) F[i][j] = Gu[i][j] + (i == j ? T(1) : T(0));
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              T s = T(0);
#pragma unroll
              for (int m = 0; m < 3; ++m) s += F[m][i] * F[m][j];
              E[i][j] = T(0.5) * (s - (i == j ? T(1) : T(0)));
            }
          const T tr = E[0][0] + E[1][1] + E[2][2];
          const T dNa[3] = {T(2) * dh[ca[0]] * h1[1][ca[1]] * h1[2][ca[2]] * ih[0],
                            T(2) * dh[ca[1]] * h1[0][ca[0]] * h1[2][ca[2]] * ih[1],
                            T(2) * dh[ca[2]] * h1[0][ca[0]] * h1[1][ca[1]] * ih[2]};
          // S dN_a, then f += w det(J) F (S dN_a)
          T sd[3];
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            T s = T(0);
#pragma unroll
            for (int j = 0; j < 3; ++j) s += (T(2) * A.mu * E[i][j] + (i == j ? A.lam * tr : T(0))) * dNa[j];
            sd[i] = s;
          }
#pragma unroll
          for (int i = 0; i < 3; ++i) f[i] += wdet * (F[i][0] * sd[0] + F[i][1] * sd[1] + F[i][2] * sd[2]);
        }
      }
  const T m = A.rho * wdet * T(nel);
  const bool lateral = ix == 0 || ix == nx || iy == 0 || iy == ny;
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[c] = (lateral && (A.lateral_fix & (1 << c))) ? T(0) : -f[c] / m;
}

// Weight of a free node in the lumped-mass inner product (proportional to its
// mass: the number of adjacent elements).
__device__ __forceinline__ double mass_weight(int ix, int iy, int nx, int ny) {
  return (ix == 0 || ix == nx ? 1.0 : 2.0) * (iy == 0 || iy == ny ? 1.0 : 2.0);
}

}  // namespace

// One Newmark sub-step of a FOM subdomain for every unfinished instance
// (Sec. 4.1 textbook Newmark-beta with row-sum lumped mass):
//   u~ = u + dt v + (1/2 - beta) dt^2 a on free DOFs, Schwarz data on the faces;
//   beta = 0: u+ = u~, a+ = M^-1(-K u+);
//   beta > 0: (M + beta dt^2 K_ff) a+ = -K [u~; u_c]  by conjugate gradients in the
//             M inner product (M^-1 K is self-adjoint there), u+ = u~ + beta dt^2 a+;
//   v+ = v + dt ((1 - gamma) a + gamma a+).
// LDS: the displacement being formed and the CG vectors live in the workgroup's LDS
// (subdomains small enough: the latency-bound sizes), the results are copied out once.
template <typename T, bool LDS, bool SVK>
__global__ __launch_bounds__(kWinFomThreads) void win_fom_kernel(WinFomArgs<T> A) {
  constexpr int NT = kWinFomThreads;
  __shared__ double red[NT / 64];
  extern __shared__ unsigned char win_lds[];
  const int b = blockIdx.y, tid = threadIdx.x;
  const Status st = A.status[b];
  if (st.flags & kFinished) return;
  const int n = st.iter + 1, l = A.l;
  const long long step = st.step, ib = (long long)b * A.is;
  const long long cs = A.cs;
  const int npl = A.npl, nzs = A.nzs, nx = A.nx, ny = A.ny, nxp = nx + 1;
  const T *ui, *vi, *ai;
  if (l == 1) {
    ui = A.u[step % 3] + ib;
    vi = A.v[step & 1] + ib;
    ai = A.a[step & 1] + ib;
  } else {
    ui = A.tu[(l - 1) & 1] + ib;
    vi = A.tv[(l - 1) & 1] + ib;
    ai = A.ta[(l - 1) & 1] + ib;
  }
  T *uo, *vo, *ao;
  if (l == A.n_sub) {
    uo = A.wu[n & 1] + ib;
    vo = A.wv[n & 1] + ib;
    ao = A.wa[n & 1] + ib;
  } else {
    uo = A.tu[l & 1] + ib;
    vo = A.tv[l & 1] + ib;
    ao = A.ta[l & 1] + ib;
  }
  const T dt = A.dt, pc = (T(0.5) - A.beta) * dt * dt;
  const bool implicit = !SVK && A.implicit;   // the SVK material takes the explicit scheme
  int par[2] = {0, 0};
  bool ready[2] = {false, false};
  for (int f = 0; f < 2; ++f)
    if (A.src[f].kind) ready[f] = src_ready(A.src[f].sd, A.sd, n, A.additive, par[f]);
  // working vectors: the displacement U and the acceleration / CG iterate X, and the CG
  // residual R, direction P and product Q ([3][cs] each)
  const long long v3 = 3 * cs;
  T *const ls = reinterpret_cast<T *>(win_lds);
  T *const uo_g = uo, *const ao_g = ao;
  if (LDS) {
    uo = ls;
    if (implicit) ao = ls + v3;
  }
  T *const Rw = LDS ? ls + 2 * v3 : A.cr + ib, *const Pw = LDS ? ls + 3 * v3 : A.cp + ib;
  T *const Qw = LDS ? ls + 4 * v3 : A.cq + ib;
  // the case blocks of the boundary columns (LDS: after the working vectors)
  const T *coef = A.coef;
  if (LDS) {
    T *lc = ls + (implicit ? 5 : 1) * v3;
    for (int i = tid; i < 9 * 234; i += NT) lc[i] = A.coef[i];
    coef = lc;   // read after the barrier that ends the predictor phase
  }

  // predictor on free layers, Schwarz data (or zero) on the two faces
  const long long nn = A.nnodes;
  if (LDS && implicit)   // the faces of the CG direction stay zero
    for (long long g = tid; g < 2 * npl; g += NT) {
      const long long gg = g < npl ? g : g - npl + (long long)nzs * npl;
#pragma unroll
      for (int c = 0; c < 3; ++c) Pw[c * cs + gg] = T(0);
    }
  for (long long g = tid; g < nn; g += NT) {
    const int k = (int)(g / npl), nid = (int)(g - (long long)k * npl);
    if (k == 0 || k == nzs) {
      const int f = k == 0 ? 0 : 1;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long o = c * cs + g;
        uo[o] = A.src[f].kind ? face_value<T>(A.src[f], b, step, c * npl + nid, l, A.n_sub, dt, ready[f], par[f],
                                              A.guess)
                              : T(0);
        vo[o] = T(0);
        ao[o] = T(0);
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long o = c * cs + g;
        uo[o] = ui[o] + dt * vi[o] + pc * ai[o];
      }
    }
  }
  __syncthreads();

  // force at the predicted displacement
  const long long nfn = (long long)npl * (nzs - 1);
  double bb = 0.0;
  for (long long h = tid; h < nfn; h += NT) {
    const long long g = h + npl;
    const int k = (int)(g / npl), nid = (int)(g - (long long)k * npl);
    const int ix = nid % nxp, iy = nid / nxp;
    T acc[3];
    if constexpr (SVK) node_force_svk<T>(A, uo, k, ix, iy, acc);
    else node_force<T>(A, coef, uo, k, ix, iy, acc);
    if (!implicit) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long o = c * cs + g;
        vo[o] = vi[o] + dt * ((T(1) - A.gamma) * ai[o] + A.gamma * acc[c]);
        ao[o] = acc[c];
      }
    } else {
      const double wgt = mass_weight(ix, iy, nx, ny);
      T *R = Rw;
      // first iterate: the previous Schwarz iterate's acceleration at the same time (one
      // sub-step per controller step), else the acceleration of the state stepped from
      const T *x0 = (n >= 2 && A.n_sub == 1) ? A.wa[(n - 1) & 1] + ib : ai;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long o = c * cs + g;
        R[o] = acc[c];   // right-hand side b
        ao[o] = x0[o];
        bb += wgt * (double)acc[c] * (double)acc[c];
      }
    }
  }
  if (implicit) {
    // conjugate gradients on (I + c L) x = b, L = M^-1 K_ff (c = beta dt^2), in the
    // inner product weighted by the lumped mass; x lives in ao, r in cr, p in cp, q in cq
    T *R = Rw, *P = Pw, *Q = Qw;
    const T cc = A.beta * dt * dt;
    bb = block_sum<NT>(bb, red);   // also orders the writes of x0 before the stencil reads
    // r0 = b - (I + c L) x0, p0 = r0
    double rho = 0.0;
    for (long long h = tid; h < nfn; h += NT) {
      const long long g = h + npl;
      const int k = (int)(g / npl), nid = (int)(g - (long long)k * npl);
      const int ix = nid % nxp, iy = nid / nxp;
      T acc[3];
      node_force<T>(A, coef, ao, k, ix, iy, acc);
      const double wgt = mass_weight(ix, iy, nx, ny);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long o = c * cs + g;
        const T ax = ao[o] - cc * acc[c];
        const T rr = R[o] - ax;
        R[o] = rr;
        P[o] = rr;
        rho += wgt * (double)rr * (double)rr;
      }
    }
    rho = block_sum<NT>(rho, red);
    int it = 0;
    const double stop = A.cg_tol2 * bb;
    while (rho > stop && it < A.cg_max) {
      ++it;
      // q = (I + c L) p and <p, q>
      double pq = 0.0;
      for (long long h = tid; h < nfn; h += NT) {
        const long long g = h + npl;
        const int k = (int)(g / npl), nid = (int)(g - (long long)k * npl);
        const int ix = nid % nxp, iy = nid / nxp;
        T acc[3];
        node_force<T>(A, coef, P, k, ix, iy, acc);
        const double wgt = mass_weight(ix, iy, nx, ny);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const long long o = c * cs + g;
          const T qq = P[o] - cc * acc[c];
          Q[o] = qq;
          pq += wgt * (double)P[o] * (double)qq;
        }
      }
      pq = block_sum<NT>(pq, red);
      const double alpha = rho / pq;
      double rho1 = 0.0;
      for (long long h = tid; h < nfn; h += NT) {
        const long long g = h + npl;
        const int nid = (int)(g % npl);
        const double wgt = mass_weight(nid % nxp, nid / nxp, nx, ny);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const long long o = c * cs + g;
          ao[o] = (T)((double)ao[o] + alpha * (double)P[o]);
          const T rr = (T)((double)R[o] - alpha * (double)Q[o]);
          R[o] = rr;
          rho1 += wgt * (double)rr * (double)rr;
        }
      }
      rho1 = block_sum<NT>(rho1, red);
      const double bet = rho1 / rho;
      rho = rho1;
      for (long long h = tid; h < nfn; h += NT) {
        const long long g = h + npl;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const long long o = c * cs + g;
          P[o] = (T)((double)R[o] + bet * (double)P[o]);
        }
      }
      __syncthreads();
    }
    if (tid == 0 && A.cg_iters && it > A.cg_iters[b]) A.cg_iters[b] = it;
    for (long long h = tid; h < nfn; h += NT) {
      const long long g = h + npl;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long o = c * cs + g;
        const T x = ao[o];
        uo[o] = uo[o] + cc * x;
        vo[o] = vi[o] + dt * ((T(1) - A.gamma) * ai[o] + A.gamma * x);
      }
    }
  }
  if (LDS) {
    __syncthreads();
    for (long long g = tid; g < nn; g += NT)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        uo_g[c * cs + g] = uo[c * cs + g];
        if (implicit) ao_g[c * cs + g] = ao[c * cs + g];
      }
  }
  __syncthreads();

  // trajectory of the faces this subdomain feeds
  const int nf3 = 3 * npl;
  for (int e = 0; e < A.nexp; ++e) {
    T *dst = A.exp_traj[e][n & 1] + ((long long)(l - 1) * gridDim.y + b) * nf3;
    const long long lay = (long long)A.exp_layer[e] * npl;
    for (int m = tid; m < nf3; m += NT) {
      const int c = m / npl, nid = m - c * npl;
      dst[m] = uo[c * cs + lay + nid];
    }
  }

  // Eq. conv_criterion sums at the end of the window: ||du + dt dv||^2 against the
  // previous iterate (the accepted state at the first), ||u + dt v||^2
  if (l == A.n_sub) {
    const T *up = n == 1 ? A.u[step % 3] + ib : A.wu[(n - 1) & 1] + ib;
    const T *vp = n == 1 ? A.v[step & 1] + ib : A.wv[(n - 1) & 1] + ib;
    double sa = 0.0, sd = 0.0;
    for (long long h = tid; h < nfn; h += NT) {
      const long long g = h + npl;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long o = c * cs + g;
        const double d = ((double)uo[o] - (double)up[o]) + (double)dt * ((double)vo[o] - (double)vp[o]);
        const double e = (double)uo[o] + (double)dt * (double)vo[o];
        sa += d * d;
        sd += e * e;
      }
    }
    sa = block_sum<NT>(sa, red);
    sd = block_sum<NT>(sd, red);
    if (tid == 0) {
      A.sums[((long long)b * A.nsd + A.sd) * 2] = sa;
      A.sums[((long long)b * A.nsd + A.sd) * 2 + 1] = sd;
    }
  }
}

// One Newmark sub-step of an OpInf subdomain (Eq. opinf_model_schwarz):
// q'' = f(q, g^) = A q + H (q (x) q) + C (q (x) q (x) q) + B g^ + c with g^ = Phi_S^T s.
//   beta = 0: q+ = q~, q''+ = f(q+, g^);
//   beta > 0: q+ solves q+ - beta dt^2 f(q+, g^) = q~ by Newton's method with the
//             Jacobian of the linear part, I - beta dt^2 A (its inverse precomputed),
//             q''+ = (q+ - q~) / (beta dt^2);
//   q'+ = q' + dt ((1 - gamma) q'' + gamma q''+).
template <typename T>
__global__ __launch_bounds__(kWinRomThreads) void win_rom_kernel(WinRomArgs<T> A) {
  constexpr int NT = kWinRomThreads;
  __shared__ double red[NT / 64];
  extern __shared__ unsigned char smem_raw[];
  T *qs = reinterpret_cast<T *>(smem_raw);   // [r] current q
  T *qt = qs + A.r;                          // [r] predictor q~
  T *gh = qt + A.r;                          // [rs] g^
  T *fr = gh + A.rs;                         // [r] f or the Newton residual
  const int b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const Status st = A.status[b];
  if (st.flags & kFinished) return;
  const int n = st.iter + 1, l = A.l, r = A.r, rs = A.rs;
  const long long step = st.step, ib = (long long)b * r;
  const T *qi, *qdi, *qddi;
  if (l == 1) {
    qi = A.q[step & 1] + ib;
    qdi = A.qd[step & 1] + ib;
    qddi = A.qdd[step & 1] + ib;
  } else {
    qi = A.tq[(l - 1) & 1] + ib;
    qdi = A.tqd[(l - 1) & 1] + ib;
    qddi = A.tqdd[(l - 1) & 1] + ib;
  }
  T *qo, *qdo, *qddo;
  if (l == A.n_sub) {
    qo = A.wq[n & 1] + ib;
    qdo = A.wqd[n & 1] + ib;
    qddo = A.wqdd[n & 1] + ib;
  } else {
    qo = A.tq[l & 1] + ib;
    qdo = A.tqd[l & 1] + ib;
    qddo = A.tqdd[l & 1] + ib;
  }
  const T dt = A.dt;
  const int nf3 = 3 * A.npl;
  const int guess = A.guess;
  // Schwarz values on the faces, then g^ = Phi_S^T s
  T *sb = A.sbuf + (long long)b * 2 * nf3;
  for (int f = 0; f < 2; ++f) {
    if (!A.src[f].kind) continue;
    int par = 0;
    const bool ready = src_ready(A.src[f].sd, A.sd, n, A.additive, par);
    for (int m = tid; m < nf3; m += NT)
      sb[f * nf3 + m] = face_value<T>(A.src[f], b, step, m, l, A.n_sub, dt, ready, par, guess);
  }
  __syncthreads();
  for (int k = wv; k < rs; k += NT / 64) {
    T s = T(0);
    for (int f = 0; f < 2; ++f) {
      if (!A.phis[f]) continue;
      const T *ph = A.phis[f] + (long long)k * nf3;
      for (int m = lane; m < nf3; m += 64) s += ph[m] * sb[f * nf3 + m];
    }
    s = wave_total(s);
    if (lane == 0) gh[k] = s;
  }
  const T pc = (T(0.5) - A.beta) * dt * dt;
  for (int i = tid; i < r; i += NT) {
    const T x = qi[i] + dt * qdi[i] + pc * qddi[i];
    qt[i] = x;
    qs[i] = x;
  }
  __syncthreads();

  // f(qs, g^) into fr: compressed powers into kbuf, then one wave per row
  T *kb = A.kbuf + (long long)b * (A.r2 + A.r3);
  auto rhs = [&]() {
    if (A.r2) {
      int off = 0;
      for (int i = 0; i < r; ++i) {
        for (int j = i + tid; j < r; j += NT) kb[off + j - i] = qs[i] * qs[j];
        off += r - i;
      }
    }
    if (A.r3) {
      int off = A.r2;
      for (int i = 0; i < r; ++i)
        for (int j = i; j < r; ++j) {
          const T qij = qs[i] * qs[j];
          for (int k = j + tid; k < r; k += NT) kb[off + k - j] = qij * qs[k];
          off += r - j;
        }
    }
    __syncthreads();
    for (int i = wv; i < r; i += NT / 64) {
      T s = T(0);
      for (int j = lane; j < r; j += 64) s += A.A[(long long)i * r + j] * qs[j];
      if (A.H)
        for (int j = lane; j < A.r2; j += 64) s += A.H[(long long)i * A.r2 + j] * kb[j];
      if (A.C3)
        for (int j = lane; j < A.r3; j += 64) s += A.C3[(long long)i * A.r3 + j] * kb[A.r2 + j];
      if (A.B)
        for (int j = lane; j < rs; j += 64) s += A.B[(long long)i * rs + j] * gh[j];
      s = wave_total(s);
      if (lane == 0) fr[i] = s + (A.c ? A.c[i] : T(0));
    }
    __syncthreads();
  };

  rhs();
  if (!A.implicit) {
    for (int i = tid; i < r; i += NT) qddo[i] = fr[i];
  } else {
    const T cc = A.beta * dt * dt;
    int it = 0;
    for (;;) {
      // residual R = q - c f(q) - q~ (in fr), correction dq = Minv R
      for (int i = tid; i < r; i += NT) fr[i] = qs[i] - cc * fr[i] - qt[i];
      __syncthreads();
      double dn = 0.0, qn = 0.0;
      T dq[4];   // r <= 4 NT (checked by the host)
      int cnt = 0;
      for (int i = tid; i < r; i += NT, ++cnt) {
        T s = T(0);
        for (int j = 0; j < r; ++j) s += A.Minv[(long long)i * r + j] * fr[j];
        dq[cnt] = s;
      }
      __syncthreads();
      cnt = 0;
      for (int i = tid; i < r; i += NT, ++cnt) {
        const T x = qs[i] - dq[cnt];
        qs[i] = x;
        dn += (double)dq[cnt] * (double)dq[cnt];
        qn += (double)x * (double)x;
      }
      dn = block_sum<NT>(dn, red);
      qn = block_sum<NT>(qn, red);
      ++it;
      if (!(dn > A.newton_tol2 * qn) || it >= A.newton_max) break;
      rhs();
    }
    if (tid == 0 && A.newton_iters && it > A.newton_iters[b]) A.newton_iters[b] = it;
    for (int i = tid; i < r; i += NT) qddo[i] = (qs[i] - qt[i]) / cc;
  }
  for (int i = tid; i < r; i += NT) {
    qo[i] = qs[i];
    qdo[i] = qdi[i] + dt * ((T(1) - A.gamma) * qddi[i] + A.gamma * qddo[i]);
  }
  __syncthreads();

  // lifted values on the faces this subdomain feeds: Pi Phi q
  for (int e = 0; e < A.nexp; ++e) {
    T *dst = A.exp_traj[e][n & 1] + ((long long)(l - 1) * gridDim.y + b) * nf3;
    const T *rows = A.exp_rows[e];
    for (int m = tid; m < nf3; m += NT) {
      T s = T(0);
      for (int k = 0; k < r; ++k) s += rows[(long long)k * nf3 + m] * qs[k];
      dst[m] = s;
    }
  }

  // Eq. conv_criterion in reduced coordinates (Phi orthonormal)
  if (l == A.n_sub) {
    const T *qp = n == 1 ? A.q[step & 1] + ib : A.wq[(n - 1) & 1] + ib;
    const T *qdp = n == 1 ? A.qd[step & 1] + ib : A.wqd[(n - 1) & 1] + ib;
    double sa = 0.0, sd = 0.0;
    for (int i = tid; i < r; i += NT) {
      const double d = ((double)qs[i] - (double)qp[i]) + (double)dt * ((double)qdo[i] - (double)qdp[i]);
      const double e = (double)qs[i] + (double)dt * (double)qdo[i];
      sa += d * d;
      sd += e * e;
    }
    sa = block_sum<NT>(sa, red);
    sd = block_sum<NT>(sd, red);
    if (tid == 0) {
      A.sums[((long long)b * A.nsd + A.sd) * 2] = sa;
      A.sums[((long long)b * A.nsd + A.sd) * 2 + 1] = sd;
    }
  }
}

// Initial acceleration a0 = -M^-1 f(u0) of a Saint Venant-Kirchhoff subdomain for the
// instances that have not advanced yet (step 0), and column 0 of its acceleration record
// (the set-up computed them with the linear stiffness).
template <typename T>
__global__ __launch_bounds__(kWinFomThreads) void win_svk_init_kernel(WinFomArgs<T> A) {
  const int b = blockIdx.y;
  const Status st = A.status[b];
  if (st.step != 0 || (st.flags & kNonfinite)) return;
  const long long ib = (long long)b * A.is;
  const T *u = A.u[0] + ib;
  T *a = A.a[0] + ib;
  const int npl = A.npl, nxp = A.nx + 1;
  const long long nfn = (long long)npl * (A.nzs - 1);
  for (long long h = threadIdx.x; h < nfn; h += kWinFomThreads) {
    const long long g = h + npl;
    const int k = (int)(g / npl), nid = (int)(g - (long long)k * npl);
    T acc[3];
    node_force_svk<T>(A, u, k, nid % nxp, nid / nxp, acc);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a[c * A.cs + g] = acc[c];
      if (A.rec_a0) A.rec_a0[(long long)b * A.rec_ncols * 3 * A.nfree_nodes + c * A.nfree_nodes + h] = acc[c];
    }
  }
}

// Eq. conv_criterion after the last subdomain of an iteration (one thread per instance).
__global__ void win_decide_kernel(Status *status, const double *sums, Opts o, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  Status s = status[b];
  if (s.flags & kFinished) return;
  for (int i = 0; i < kMaxSd; ++i)
    if (i < o.nsd) {
      s.sd_abs2[i] = sums[((long long)b * o.nsd + i) * 2];
      s.sd_den2[i] = sums[((long long)b * o.nsd + i) * 2 + 1];
    }
  decide(s, o.nsd - 1, o);
  status[b] = s;
}

// Acceptance: instances that took part in this controller step (pad0 & 1) and
// converged (or hit the cap) copy their last iterate into the roles of the new
// step and record it when the step is a recorded one.
template <typename T>
__global__ void win_accept_kernel(WinAcceptArgs<T> A) {
  const int b = blockIdx.y;
  const Status st = A.status[b];
  if (!(st.pad0 & 1) || !(st.flags & kFinished) || (st.flags & kNonfinite)) return;
  const long long step = st.step;   // the new step
  const int par = st.last_iters & 1;
  long long col = -1;
  if (A.rec_every > 0 && step % A.rec_every == 0 && step / A.rec_every < A.rec_ncols) col = step / A.rec_every;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (A.rom) {
    if (t >= A.r) return;
    const long long o = (long long)b * A.r + t;
    A.q[step & 1][o] = A.wq[par][o];
    A.qd[step & 1][o] = A.wqd[par][o];
    A.qdd[step & 1][o] = A.wqdd[par][o];
    if (col >= 0 && A.rec_u) A.rec_u[((long long)b * A.rec_ncols + col) * A.r + t] = A.wq[par][o];
    return;
  }
  if (t >= A.nnodes) return;
  const long long ib = (long long)b * A.is;
  const int k = (int)(t / A.npl), nid = (int)(t - (long long)k * A.npl);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const long long o = ib + (long long)c * A.cs + t;
    const T u = A.wu[par][o], v = A.wv[par][o], a = A.wa[par][o];
    A.u[step % 3][o] = u;
    A.v[step & 1][o] = v;
    A.a[step & 1][o] = a;
    if (col < 0) continue;
    if (k >= 1 && k < A.nzs) {
      const long long ro = ((long long)b * A.rec_ncols + col) * 3 * A.nfree_nodes + (long long)c * A.nfree_nodes +
                           (long long)(k - 1) * A.npl + nid;
      if (A.rec_u) A.rec_u[ro] = u;
      if (A.rec_a) A.rec_a[ro] = a;
    } else if (A.rec_s && A.face_sch[k == 0 ? 0 : 1]) {
      const long long so = ((long long)b * A.rec_ncols + col) * 3 * A.nsch_nodes + (long long)c * A.nsch_nodes +
                           (k == 0 ? 0 : A.face_off_hi) + nid;
      A.rec_s[so] = u;
    }
  }
}

template <typename T>
hipError_t launch_win_fom(const WinFomArgs<T> &A, int batch, hipStream_t s) {
  // small subdomains keep their working vectors in LDS (one vector explicit, five implicit)
  const size_t lds = sizeof(T) * (3 * (size_t)A.cs * (A.implicit ? 5 : 1) + 9 * 234);
  const bool svk = A.material != 0;
  if (lds <= kWinLdsBytes) {
    const void *f = svk ? (const void *)win_fom_kernel<T, true, true> : (const void *)win_fom_kernel<T, true, false>;
    if (lds > 64 * 1024) {   // dynamic LDS beyond the default limit must be requested
      const hipError_t ea = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (ea != hipSuccess) return ea;
    }
    if (svk) hipLaunchKernelGGL((win_fom_kernel<T, true, true>), dim3(1, batch), dim3(kWinFomThreads), lds, s, A);
    else hipLaunchKernelGGL((win_fom_kernel<T, true, false>), dim3(1, batch), dim3(kWinFomThreads), lds, s, A);
  } else if (svk) {
    hipLaunchKernelGGL((win_fom_kernel<T, false, true>), dim3(1, batch), dim3(kWinFomThreads), 0, s, A);
  } else {
    hipLaunchKernelGGL((win_fom_kernel<T, false, false>), dim3(1, batch), dim3(kWinFomThreads), 0, s, A);
  }
  return hipGetLastError();
}
template <typename T>
hipError_t launch_win_svk_init(const WinFomArgs<T> &A, int batch, hipStream_t s) {
  hipLaunchKernelGGL(win_svk_init_kernel<T>, dim3(1, batch), dim3(kWinFomThreads), 0, s, A);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_win_rom(const WinRomArgs<T> &A, int batch, hipStream_t s) {
  const size_t smem = sizeof(T) * (3 * (size_t)A.r + A.rs);
  hipLaunchKernelGGL(win_rom_kernel<T>, dim3(1, batch), dim3(kWinRomThreads), smem, s, A);
  return hipGetLastError();
}
hipError_t launch_win_decide(Status *st, const double *sums, const Opts &o, int batch, hipStream_t s) {
  hipLaunchKernelGGL(win_decide_kernel, dim3((batch + 63) / 64), dim3(64), 0, s, st, sums, o, batch);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_win_accept(const WinAcceptArgs<T> &A, int batch, hipStream_t s) {
  const long long n = A.rom ? A.r : A.nnodes;
  hipLaunchKernelGGL(win_accept_kernel<T>, dim3((unsigned)((n + 255) / 256), batch), dim3(256), 0, s, A);
  return hipGetLastError();
}

template hipError_t launch_win_fom<double>(const WinFomArgs<double> &, int, hipStream_t);
template hipError_t launch_win_fom<float>(const WinFomArgs<float> &, int, hipStream_t);
template hipError_t launch_win_svk_init<double>(const WinFomArgs<double> &, int, hipStream_t);
template hipError_t launch_win_svk_init<float>(const WinFomArgs<float> &, int, hipStream_t);
template hipError_t launch_win_rom<double>(const WinRomArgs<double> &, int, hipStream_t);
template hipError_t launch_win_rom<float>(const WinRomArgs<float> &, int, hipStream_t);
template hipError_t launch_win_accept<double>(const WinAcceptArgs<double> &, int, hipStream_t);
template hipError_t launch_win_accept<float>(const WinAcceptArgs<float> &, int, hipStream_t);

}  // namespace osam
