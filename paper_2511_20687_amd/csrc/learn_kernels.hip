// Dense FP64 kernels of the OpInf learning stage (Sec. 3.1, 3.2, 4.2.1, Alg. 3).
//
//  * gemm64: C = alpha op(A) op(B) + beta C, column-major, FP64 accumulation on
//    the FP64 matrix cores (v_mfma_f64_16x16x4); A/B may be FP32 (snapshots are
//    stored in the run precision and widened on load).  64x64 tile per
//    workgroup, 4 waves of 32x32, optional split-K with a fixed-order reduction.
//  * symmetric eigensolvers for the snapshot Gram (a one-workgroup cyclic Jacobi
//    for the Rayleigh-Ritz blocks of the subspace iteration, a cyclic Jacobi with
//    one launch per round for whole Grams), small (LDS) and blocked Cholesky,
//    triangular solves and inverses: the pieces of the POD and of the regularised
//    normal equations.
//  * data matrix D = [Q^T | (Q (x) Q)^T | S^^T | 1] and the batched FP64
//    frozen-boundary rollouts of Alg. 3 (one workgroup per lambda x trajectory).
#include <hip/hip_runtime.h>

namespace osam {

typedef double d4_t __attribute__((ext_vector_type(4)));

// dynamic LDS of one workgroup: gfx950's 160 KB less room for a kernel's static LDS
constexpr size_t kLdsDyn = 159 * 1024;
constexpr int kCholLdsMaxN = 200;        // n (n + 1) / 2 doubles <= kLdsDyn

__device__ __forceinline__ double wsum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Block-wide sum (blockDim.x multiple of 64, <= 1024), result broadcast.
__device__ double block_sum(double x, double *sh) {
  x = wsum(x);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = x;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += sh[i];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------------------
template <typename TA, typename TB, bool TRA, bool TRB>
__global__ void __launch_bounds__(256) gemm64_kernel(int M, int N, long long K, double alpha, const TA *A,
                                                     long long lda, const TB *B, long long ldb, double beta,
                                                     double *C, long long ldc, long long kchunk, double *work) {
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const long long kbeg = (long long)blockIdx.z * kchunk;
  const long long kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid & 1, wn = wid >> 1;
  d4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

  for (long long k0 = kbeg; k0 < kend; k0 += 16) {
#pragma unroll
    for (int e = tid; e < 1024; e += 256) {
      int mm, kk;
      if (!TRA) { mm = e & 63; kk = e >> 6; } else { kk = e & 15; mm = e >> 4; }
      const long long gm = m0 + mm, gk = k0 + kk;
      double v = 0.0;
      if (gm < M && gk < kend) v = TRA ? (double)A[gk + gm * lda] : (double)A[gm + gk * lda];
      As[kk][mm] = v;
    }
#pragma unroll
    for (int e = tid; e < 1024; e += 256) {
      int nn, kk;
      if (!TRB) { kk = e & 15; nn = e >> 4; } else { nn = e & 63; kk = e >> 6; }
      const long long gn = n0 + nn, gk = k0 + kk;
      double v = 0.0;
      if (gn < N && gk < kend) v = TRB ? (double)B[gn + gk * ldb] : (double)B[gk + gn * ldb];
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int kr = kk + (lane >> 4), cc = lane & 15;
      const double a0 = As[kr][wm * 32 + cc], a1 = As[kr][wm * 32 + 16 + cc];
      const double b0 = Bs[kr][wn * 32 + cc], b1 = Bs[kr][wn * 32 + 16 + cc];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // v_mfma_f64_16x16x4: result register i of lane l is row l/16 + 4i, column l%16
        const long long row = m0 + wm * 32 + bm * 16 + (lane >> 4) + 4 * i;
        const long long col = n0 + wn * 32 + bn * 16 + (lane & 15);
        if (row < M && col < N) {
          const double v = acc[bm][bn][i];
          if (work) {
            work[(long long)blockIdx.z * M * N + row + col * M] = v;
          } else {
            const double old = (beta != 0.0) ? C[row + col * ldc] : 0.0;
            C[row + col * ldc] = alpha * v + beta * old;
          }
        }
      }
}

__global__ void splitk_reduce_kernel(int M, int N, int ks, double alpha, const double *work, double beta,
                                     double *C, long long ldc) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)M * N) return;
  const long long row = idx % M, col = idx / M;
  double s = 0.0;
  for (int z = 0; z < ks; ++z) s += work[(long long)z * M * N + idx];
  const double old = (beta != 0.0) ? C[row + col * ldc] : 0.0;
  C[row + col * ldc] = alpha * s + beta * old;
}

template <typename TA, typename TB>
hipError_t gemm64(bool tra, bool trb, int M, int N, long long K, double alpha, const TA *A, long long lda,
                  const TB *B, long long ldb, double beta, double *C, long long ldc, double *work,
                  long long work_n, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int tm = (M + 63) / 64, tn = (N + 63) / 64;
  int ks = 1;
  const int tiles = tm * tn;
  if (work && K > 4096 && tiles < 512) {
    ks = (int)std::min<long long>((1024 + tiles - 1) / tiles, (K + 2047) / 2048);
    while (ks > 1 && (long long)ks * M * N > work_n) --ks;
  }
  long long kchunk = (K + ks - 1) / ks;
  kchunk = (kchunk + 15) / 16 * 16;
  if (kchunk <= 0) kchunk = 16;
  ks = (int)((K + kchunk - 1) / kchunk);
  if (ks < 1) ks = 1;
  dim3 grid(tm, tn, ks);
  double *wk = ks > 1 ? work : nullptr;
#define GEMM_CASE(a, b)                                                                                 \
  hipLaunchKernelGGL((gemm64_kernel<TA, TB, a, b>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, \
                     beta, C, ldc, kchunk, wk)
  if (!tra && !trb) GEMM_CASE(false, false);
  else if (tra && !trb) GEMM_CASE(true, false);
  else if (!tra && trb) GEMM_CASE(false, true);
  else GEMM_CASE(true, true);
#undef GEMM_CASE
  if (ks > 1) {
    const long long n = (long long)M * N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, M, N, ks,
                       alpha, work, beta, C, ldc);
  }
  return hipGetLastError();
}
template hipError_t gemm64<double, double>(bool, bool, int, int, long long, double, const double *, long long,
                                           const double *, long long, double, double *, long long, double *,
                                           long long, hipStream_t);
template hipError_t gemm64<float, float>(bool, bool, int, int, long long, double, const float *, long long,
                                         const float *, long long, double, double *, long long, double *,
                                         long long, hipStream_t);
template hipError_t gemm64<double, float>(bool, bool, int, int, long long, double, const double *, long long,
                                          const float *, long long, double, double *, long long, double *,
                                          long long, hipStream_t);
template hipError_t gemm64<float, double>(bool, bool, int, int, long long, double, const float *, long long,
                                          const double *, long long, double, double *, long long, double *,
                                          long long, hipStream_t);

// ---------------------------------------------------------------------------
// Cyclic Jacobi for a small symmetric matrix A (k x k, column-major, destroyed),
// one workgroup.  Round-robin ordering: k/2 disjoint rotations per round.
// Eigenvalues (descending) in w, eigenvectors in the columns of V.  LDS: A and V
// are worked on in LDS (2 k^2 doubles of dynamic LDS) and V is written back at the end.
template <bool LDS>
__global__ void __launch_bounds__(1024) jacobi_eig_kernel(double *Ag, double *Vg, double *w, int k, int max_sweeps,
                                                         int *pairs_ws, double *cs_ws) {
  extern __shared__ double jlds[];
  __shared__ double sh[16];
  __shared__ int done;
  double *A = LDS ? jlds : Ag;
  double *V = LDS ? jlds + (size_t)k * k : Vg;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int kk = k + (k & 1);          // even number of players (a dummy when k is odd)
  const int np = kk / 2;
  for (long long i = tid; i < (long long)k * k; i += bs) {
    V[i] = ((i % k) == (i / k)) ? 1.0 : 0.0;
    if (LDS) A[i] = Ag[i];
  }
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence test: off-diagonal vs total Frobenius norm
    double off = 0.0, tot = 0.0;
    for (long long i = tid; i < (long long)k * k; i += bs) {
      const double a = A[i];
      tot += a * a;
      if ((i % k) != (i / k)) off += a * a;
    }
    off = block_sum(off, sh);
    tot = block_sum(tot, sh);
    if (tid == 0) done = (off <= 1e-30 * tot) || tot == 0.0;
    __syncthreads();
    if (done) break;
    for (int rnd = 0; rnd < kk - 1; ++rnd) {
      // pairs of this round
      for (int t = tid; t < np; t += bs) {
        int p, q;
        if (t == 0) {
          p = kk - 1;
          q = rnd;
        } else {
          p = (rnd + t) % (kk - 1);
          q = (rnd - t + (kk - 1)) % (kk - 1);
        }
        if (p > q) { const int x = p; p = q; q = x; }
        double c = 1.0, s = 0.0;
        if (q < k) {
          const double apq = A[p + (long long)q * k];
          if (apq != 0.0) {
            const double app = A[p + (long long)p * k], aqq = A[q + (long long)q * k];
            const double theta = (aqq - app) / (2.0 * apq);
            const double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            s = tt * c;
          }
        }
        pairs_ws[2 * t] = p;
        pairs_ws[2 * t + 1] = q;
        cs_ws[2 * t] = c;
        cs_ws[2 * t + 1] = s;
      }
      __syncthreads();
      // rows p, q: A <- J^T A
      for (long long e = tid; e < (long long)np * k; e += bs) {
        const int t = (int)(e / k), j = (int)(e % k);
        const int p = pairs_ws[2 * t], q = pairs_ws[2 * t + 1];
        if (q >= k) continue;
        const double c = cs_ws[2 * t], s = cs_ws[2 * t + 1];
        if (s == 0.0) continue;
        const double ap = A[p + (long long)j * k], aq = A[q + (long long)j * k];
        A[p + (long long)j * k] = c * ap - s * aq;
        A[q + (long long)j * k] = s * ap + c * aq;
      }
      __syncthreads();
      // columns p, q: A <- A J ; V <- V J
      for (long long e = tid; e < (long long)np * k; e += bs) {
        const int t = (int)(e / k), i = (int)(e % k);
        const int p = pairs_ws[2 * t], q = pairs_ws[2 * t + 1];
        if (q >= k) continue;
        const double c = cs_ws[2 * t], s = cs_ws[2 * t + 1];
        if (s == 0.0) continue;
        const double ap = A[i + (long long)p * k], aq = A[i + (long long)q * k];
        A[i + (long long)p * k] = c * ap - s * aq;
        A[i + (long long)q * k] = s * ap + c * aq;
        const double vp = V[i + (long long)p * k], vq = V[i + (long long)q * k];
        V[i + (long long)p * k] = c * vp - s * vq;
        V[i + (long long)q * k] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  // sort descending (selection by one thread on indices, then permute columns)
  if (tid == 0) {
    for (int i = 0; i < k; ++i) pairs_ws[i] = i;
    for (int i = 0; i < k; ++i) {
      int best = i;
      for (int j = i + 1; j < k; ++j)
        if (A[pairs_ws[j] + (long long)pairs_ws[j] * k] > A[pairs_ws[best] + (long long)pairs_ws[best] * k]) best = j;
      const int x = pairs_ws[i]; pairs_ws[i] = pairs_ws[best]; pairs_ws[best] = x;
    }
    for (int i = 0; i < k; ++i) w[i] = A[pairs_ws[i] + (long long)pairs_ws[i] * k];
  }
  __syncthreads();
  // permuted copy of V into A (A is scratch now), then into the output
  for (long long e = tid; e < (long long)k * k; e += bs) {
    const int i = (int)(e % k), j = (int)(e / k);
    A[e] = V[i + (long long)pairs_ws[j] * k];
  }
  __syncthreads();
  for (long long e = tid; e < (long long)k * k; e += bs) Vg[e] = A[e];
}

hipError_t launch_jacobi(double *A, double *V, double *w, int k, int *pairs_ws, double *cs_ws, hipStream_t s) {
  const size_t lds = (size_t)2 * k * k * sizeof(double);
  if (lds <= kLdsDyn) {
    static bool attr = false;
    if (!attr && lds > 65536) {
      const hipError_t e = hipFuncSetAttribute((const void *)jacobi_eig_kernel<true>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsDyn);
      if (e != hipSuccess) return e;
      attr = true;
    }
    hipLaunchKernelGGL(jacobi_eig_kernel<true>, dim3(1), dim3(1024), lds, s, A, V, w, k, 60, pairs_ws, cs_ws);
  } else {
    hipLaunchKernelGGL(jacobi_eig_kernel<false>, dim3(1), dim3(1024), 0, s, A, V, w, k, 60, pairs_ws, cs_ws);
  }
  return hipGetLastError();
}

// out[j] = || Z[:, j] - theta[j] Y[:, j] ||^2 for the k leading columns of the n-row blocks
// Z and Y (ld n): the residuals of Ritz pairs.  One workgroup per column.
__global__ void __launch_bounds__(256) ritz_resid_kernel(const double *Z, const double *Y, const double *theta,
                                                        long long n, double *out) {
  __shared__ double sh[16];
  const int j = blockIdx.x;
  const double th = theta[j];
  const double *z = Z + (size_t)j * n, *y = Y + (size_t)j * n;
  double acc = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = z[i] - th * y[i];
    acc += d * d;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) out[j] = acc;
}

hipError_t launch_ritz_resid(const double *Z, const double *Y, const double *theta, long long n, int k, double *out,
                             hipStream_t s) {
  hipLaunchKernelGGL(ritz_resid_kernel, dim3(k), dim3(256), 0, s, Z, Y, theta, n, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi for the full snapshot Gram (n up to a few thousand), one launch
// per round of the round-robin ordering: n/2 disjoint rotations.  Every thread
// owns one 2x2 block A[{p1,q1},{p2,q2}] of the pair (t1, t2), recomputes both
// rotations from the unmodified input (ping-pong buffers, so all threads see
// the same values) and writes J1^T B J2; the same thread rotates rows 2 t2,
// 2 t2 + 1 of the eigenvector columns p1, q1.  Index n (odd n) is a dummy.
__device__ __forceinline__ void rr_pair(int t, int rnd, int nn, int &p, int &q) {
  if (t == 0) {
    p = nn - 1;
    q = rnd;
  } else {
    p = (rnd + t) % (nn - 1);
    q = (rnd - t + (nn - 1)) % (nn - 1);
  }
  if (p > q) {
    const int x = p;
    p = q;
    q = x;
  }
}

__device__ __forceinline__ void rot_params(const double *A, long long n, int p, int q, double &c, double &s) {
  c = 1.0;
  s = 0.0;
  if (q >= n) return;
  const double apq = A[p + q * n];
  if (apq == 0.0) return;
  const double app = A[p + p * n], aqq = A[q + q * n];
  const double theta = (aqq - app) / (2.0 * apq);
  const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
  c = 1.0 / sqrt(t * t + 1.0);
  s = t * c;
}

__global__ void jacobi_round_kernel(const double *A, double *Ao, const double *V, double *Vo, int n, int nn, int rnd) {
  const int half = nn / 2;
  const int t1 = blockIdx.x * blockDim.x + threadIdx.x, t2 = blockIdx.y;
  if (t1 >= half) return;
  int p1, q1, p2, q2;
  rr_pair(t1, rnd, nn, p1, q1);
  rr_pair(t2, rnd, nn, p2, q2);
  double c1, s1, c2, s2;
  rot_params(A, n, p1, q1, c1, s1);
  rot_params(A, n, p2, q2, c2, s2);
  const long long N = n;
  const bool q1v = q1 < n, q2v = q2 < n;
  const double b00 = A[p1 + p2 * N];
  const double b01 = q2v ? A[p1 + q2 * N] : 0.0;
  const double b10 = q1v ? A[q1 + p2 * N] : 0.0;
  const double b11 = (q1v && q2v) ? A[q1 + q2 * N] : 0.0;
  // rows (J1^T B)
  const double r00 = c1 * b00 - s1 * b10, r01 = c1 * b01 - s1 * b11;
  const double r10 = s1 * b00 + c1 * b10, r11 = s1 * b01 + c1 * b11;
  // columns ((J1^T B) J2)
  double o00 = c2 * r00 - s2 * r01, o01 = s2 * r00 + c2 * r01;
  double o10 = c2 * r10 - s2 * r11, o11 = s2 * r10 + c2 * r11;
  if (t1 == t2) {
    o01 = 0.0;   // the annihilated pair
    o10 = 0.0;
  }
  Ao[p1 + p2 * N] = o00;
  if (q2v) Ao[p1 + q2 * N] = o01;
  if (q1v) Ao[q1 + p2 * N] = o10;
  if (q1v && q2v) Ao[q1 + q2 * N] = o11;
  // eigenvectors: V <- V J1 on rows 2 t2, 2 t2 + 1
  for (int rr = 0; rr < 2; ++rr) {
    const long long i = 2LL * t2 + rr;
    if (i >= n) continue;
    const double vp = V[i + p1 * N];
    const double vq = q1v ? V[i + q1 * N] : 0.0;
    Vo[i + p1 * N] = c1 * vp - s1 * vq;
    if (q1v) Vo[i + q1 * N] = s1 * vp + c1 * vq;
  }
}

// per-block partial sums of the off-diagonal and total squared entries
__global__ void offnorm_kernel(const double *A, long long n, double *part) {
  __shared__ double sh[16];
  double off = 0.0, tot = 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += (long long)gridDim.x * blockDim.x) {
    const double a = A[e];
    tot += a * a;
    if ((e % n) != (e / n)) off += a * a;
  }
  off = block_sum(off, sh);
  tot = block_sum(tot, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = off;
    part[2 * blockIdx.x + 1] = tot;
  }
}

__global__ void identity_kernel(double *V, long long n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n * n) V[e] = ((e % n) == (e / n)) ? 1.0 : 0.0;
}

__global__ void gather_cols_kernel(const double *V, long long n, const int *order, int k, double *out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const long long i = e % n, j = e / n;
  out[e] = V[i + (long long)order[j] * n];
}

hipError_t launch_jacobi_round(const double *A, double *Ao, const double *V, double *Vo, int n, int rnd, hipStream_t s) {
  const int nn = n + (n & 1), half = nn / 2;
  dim3 grid((half + 255) / 256, half);
  hipLaunchKernelGGL(jacobi_round_kernel, grid, dim3(256), 0, s, A, Ao, V, Vo, n, nn, rnd);
  return hipGetLastError();
}
hipError_t launch_offnorm(const double *A, long long n, double *part, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(offnorm_kernel, dim3(nblocks), dim3(256), 0, s, A, n, part);
  return hipGetLastError();
}
hipError_t launch_identity(double *V, long long n, hipStream_t s) {
  hipLaunchKernelGGL(identity_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, V, n);
  return hipGetLastError();
}

// d[i] = A[i, i] for the n x n matrix A (ld n).
__global__ void diag_kernel(const double *A, long long n, double *d) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = A[i + i * n];
}

hipError_t launch_diag(const double *A, long long n, double *d, hipStream_t s) {
  hipLaunchKernelGGL(diag_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, n, d);
  return hipGetLastError();
}
hipError_t launch_gather_cols(const double *V, long long n, const int *order, int k, double *out, hipStream_t s) {
  hipLaunchKernelGGL(gather_cols_kernel, dim3((unsigned)((n * k + 255) / 256)), dim3(256), 0, s, V, n, order, k, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Unblocked Cholesky of a small SPD matrix (n <= ~512), one workgroup, in place
// (lower triangle, column-major, leading dimension lda).  shift is added to the
// diagonal first.  info = 0 on success, j+1 if pivot j is not positive.
__global__ void __launch_bounds__(1024) chol_small_kernel(double *A, int n, long long lda, double shift, int *info) {
  __shared__ double piv;
  const int tid = threadIdx.x, bs = blockDim.x;
  if (tid == 0) *info = 0;
  for (int i = tid; i < n; i += bs) A[i + i * lda] += shift;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      const double d = A[j + j * lda];
      if (!(d > 0.0)) {
        *info = j + 1;
        piv = 0.0;
      } else {
        piv = sqrt(d);
        A[j + j * lda] = piv;
      }
    }
    __syncthreads();
    if (!(piv > 0.0)) return;
    for (int i = j + 1 + tid; i < n; i += bs) A[i + j * lda] /= piv;
    __syncthreads();
    const int m = n - j - 1;
    for (long long e = tid; e < (long long)m * m; e += bs) {
      const int i = j + 1 + (int)(e % m), l = j + 1 + (int)(e / m);
      if (i >= l) A[i + l * lda] -= A[i + j * lda] * A[l + j * lda];
    }
    __syncthreads();
  }
  for (long long e = tid; e < (long long)n * n; e += bs) {
    const int i = (int)(e % n), l = (int)(e / n);
    if (i < l) A[i + l * lda] = 0.0;
  }
}

hipError_t launch_chol_small(double *A, int n, long long lda, double shift, int *info, hipStream_t s) {
  hipLaunchKernelGGL(chol_small_kernel, dim3(1), dim3(1024), 0, s, A, n, lda, shift, info);
  return hipGetLastError();
}

// The same factorisation with the lower triangle packed in LDS (column-major packed
// storage, n (n + 1) / 2 doubles): for the Gram blocks of Cholesky-QR, n <= kCholLdsMaxN.
__global__ void __launch_bounds__(1024) chol_lds_kernel(double *A, int n, long long lda, double shift, int *info) {
  extern __shared__ double P[];
  __shared__ double piv;
  const int tid = threadIdx.x, bs = blockDim.x;
  // packed offset of (i, l), i >= l: the columns before l hold n + (n - 1) + ... entries
  auto at = [&](int i, int l) -> double & { return P[(long long)l * n - (long long)l * (l - 1) / 2 + (i - l)]; };
  if (tid == 0) *info = 0;
  for (long long e = tid; e < (long long)n * n; e += bs) {
    const int i = (int)(e % n), l = (int)(e / n);
    if (i >= l) at(i, l) = A[i + l * lda] + (i == l ? shift : 0.0);
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      const double d = at(j, j);
      if (!(d > 0.0)) {
        *info = j + 1;
        piv = 0.0;
      } else {
        piv = sqrt(d);
        at(j, j) = piv;
      }
    }
    __syncthreads();
    if (!(piv > 0.0)) return;
    for (int i = j + 1 + tid; i < n; i += bs) at(i, j) /= piv;
    __syncthreads();
    const int m = n - j - 1;
    for (int e = tid; e < m * m; e += bs) {
      const int i = j + 1 + e % m, l = j + 1 + e / m;
      if (i >= l) at(i, l) -= at(i, j) * at(l, j);
    }
    __syncthreads();
  }
  for (long long e = tid; e < (long long)n * n; e += bs) {
    const int i = (int)(e % n), l = (int)(e / n);
    A[i + l * lda] = i >= l ? at(i, l) : 0.0;
  }
}

hipError_t launch_chol_lds(double *A, int n, long long lda, double shift, int *info, hipStream_t s) {
  if (n > kCholLdsMaxN) return launch_chol_small(A, n, lda, shift, info, s);
  const size_t lds = (size_t)n * (n + 1) / 2 * sizeof(double);
  static bool attr = false;
  if (!attr && lds > 65536) {
    const hipError_t e =
        hipFuncSetAttribute((const void *)chol_lds_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsDyn);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(chol_lds_kernel, dim3(1), dim3(1024), lds, s, A, n, lda, shift, info);
  return hipGetLastError();
}

// Li <- L^-1 for a lower-triangular L (k x k, ld k, k <= 192).  One wavefront per column j
// of the inverse: forward substitution L x = e_j, each lane holding the entries x_l with
// l = lane (mod 64) and the dot products reduced across the wave.
__global__ void __launch_bounds__(256) trtri_lower_kernel(const double *L, int k, double *Li) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= k) return;
  double x0 = 0.0, x1 = 0.0, x2 = 0.0;   // x_lane, x_{lane+64}, x_{lane+128}
  const double xj = 1.0 / L[j + (long long)j * k];
  if (lane == (j & 63)) {
    if ((j >> 6) == 0) x0 = xj;
    else if ((j >> 6) == 1) x1 = xj;
    else x2 = xj;
  }
  double *col = Li + (long long)j * k;
  for (int i = lane; i < j; i += 64) col[i] = 0.0;
  if (lane == 0) col[j] = xj;
  for (int i = j + 1; i < k; ++i) {
    const double *row = L + i;
    double acc = 0.0;
    int l = lane;
    if (l >= j && l < i) acc += row[(long long)l * k] * x0;
    l += 64;
    if (l >= j && l < i) acc += row[(long long)l * k] * x1;
    l += 64;
    if (l >= j && l < i) acc += row[(long long)l * k] * x2;
    acc = wsum(acc);
    const double xi = -acc / L[i + (long long)i * k];
    if (lane == (i & 63)) {
      if ((i >> 6) == 0) x0 = xi;
      else if ((i >> 6) == 1) x1 = xi;
      else x2 = xi;
    }
    if (lane == 0) col[i] = xi;
  }
}

hipError_t launch_trtri_lower(const double *L, int k, double *Li, hipStream_t s) {
  if (k > 192) return hipErrorInvalidValue;
  hipLaunchKernelGGL(trtri_lower_kernel, dim3((unsigned)((k + 3) / 4)), dim3(256), 0, s, L, k, Li);
  return hipGetLastError();
}

// W[:, j] *= f[j]  (or /= f[j] when inv), skipping zero columns.
__global__ void colscale_kernel(double *W, long long m, int k, const double *f, int inv) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * k) return;
  const int j = (int)(idx / m);
  const double s = f[j];
  if (inv) {
    if (s > 0.0) W[idx] /= s;
  } else {
    W[idx] *= s;
  }
}

hipError_t launch_colscale(double *W, long long m, int k, const double *f, int inv, hipStream_t s) {
  const long long n = m * k;
  hipLaunchKernelGGL(colscale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, m, k, f, inv);
  return hipGetLastError();
}

// Sign convention for singular vectors: flip column j so that its entry of
// largest magnitude is positive (one block per column; ties -> smallest index).
__global__ void sign_fix_kernel(double *W, long long m) {
  __shared__ double bv[1024];
  __shared__ long long bi[1024];
  const int j = blockIdx.x;
  double best = -1.0;
  long long bidx = 0;
  for (long long i = threadIdx.x; i < m; i += blockDim.x) {
    const double a = fabs(W[i + j * m]);
    if (a > best) { best = a; bidx = i; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double o = bv[threadIdx.x + s];
      const long long oi = bi[threadIdx.x + s];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const double sg = W[bi[0] + j * m] < 0.0 ? -1.0 : 1.0;
  for (long long i = threadIdx.x; i < m; i += blockDim.x) W[i + j * m] *= sg;
}
hipError_t launch_sign_fix(double *W, long long m, int k, hipStream_t s) {
  hipLaunchKernelGGL(sign_fix_kernel, dim3(k), dim3(1024), 0, s, W, m);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Blocked Cholesky pieces for the least-squares matrices (n up to a few 1000).
// Diagonal block factor: one workgroup, nb <= 64, in LDS.
__global__ void __launch_bounds__(256) potrf_diag_kernel(double *A, long long lda, int j0, int nb, int *info) {
  __shared__ double T[64][65];
  __shared__ double piv;
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += blockDim.x) T[e % nb][e / nb] = A[(j0 + e % nb) + (long long)(j0 + e / nb) * lda];
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (tid == 0) {
      const double d = T[j][j];
      if (!(d > 0.0)) {
        if (*info == 0) *info = j0 + j + 1;
        piv = 0.0;
      } else {
        piv = sqrt(d);
      }
      T[j][j] = piv;
    }
    __syncthreads();
    if (!(piv > 0.0)) return;
    for (int i = j + 1 + tid; i < nb; i += blockDim.x) T[i][j] /= piv;
    __syncthreads();
    const int m = nb - j - 1;
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int i = j + 1 + e % m, l = j + 1 + e / m;
      if (i >= l) T[i][l] -= T[i][j] * T[l][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += blockDim.x) {
    const int i = e % nb, l = e / nb;
    A[(j0 + i) + (long long)(j0 + l) * lda] = (i >= l) ? T[i][l] : 0.0;
  }
}

// Panel below the diagonal block: L21 = A21 L11^-T (one thread per row).
__global__ void trsm_panel_kernel(double *A, long long lda, int n, int j0, int nb, const int *info) {
  if (*info) return;
  const int i = j0 + nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int j = 0; j < nb; ++j) {
    double s = A[i + (long long)(j0 + j) * lda];
    for (int l = 0; l < j; ++l) s -= A[i + (long long)(j0 + l) * lda] * A[(j0 + j) + (long long)(j0 + l) * lda];
    A[i + (long long)(j0 + j) * lda] = s / A[(j0 + j) + (long long)(j0 + j) * lda];
  }
}

hipError_t launch_potrf_diag(double *A, long long lda, int j0, int nb, int *info, hipStream_t s) {
  hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, s, A, lda, j0, nb, info);
  return hipGetLastError();
}
hipError_t launch_trsm_panel(double *A, long long lda, int n, int j0, int nb, const int *info, hipStream_t s) {
  const int rows = n - j0 - nb;
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(trsm_panel_kernel, dim3((rows + 255) / 256), dim3(256), 0, s, A, lda, n, j0, nb, info);
  return hipGetLastError();
}

// Triangular solve of one diagonal block for many right-hand sides:
// lower: Y_j <- L_jj^-1 Y_j ; upper (transposed lower): Y_j <- L_jj^-T Y_j.
__global__ void trsv_block_kernel(const double *L, long long lda, int j0, int nb, double *Y, long long ldy, int nrhs,
                                  int transpose) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  double *y = Y + (long long)c * ldy + j0;
  if (!transpose) {
    for (int j = 0; j < nb; ++j) {
      double s = y[j];
      for (int l = 0; l < j; ++l) s -= L[(j0 + j) + (long long)(j0 + l) * lda] * y[l];
      y[j] = s / L[(j0 + j) + (long long)(j0 + j) * lda];
    }
  } else {
    for (int j = nb - 1; j >= 0; --j) {
      double s = y[j];
      for (int l = j + 1; l < nb; ++l) s -= L[(j0 + l) + (long long)(j0 + j) * lda] * y[l];
      y[j] = s / L[(j0 + j) + (long long)(j0 + j) * lda];
    }
  }
}
hipError_t launch_trsv_block(const double *L, long long lda, int j0, int nb, double *Y, long long ldy, int nrhs,
                             int transpose, hipStream_t s) {
  hipLaunchKernelGGL(trsv_block_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, s, L, lda, j0, nb, Y, ldy, nrhs,
                     transpose);
  return hipGetLastError();
}

__global__ void add_diag_kernel(double *A, long long lda, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) A[i + (long long)i * lda] += v;
}
hipError_t launch_add_diag(double *A, long long lda, int n, double v, hipStream_t s) {
  hipLaunchKernelGGL(add_diag_kernel, dim3((n + 255) / 256), dim3(256), 0, s, A, lda, n, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Normalisation of the least-squares data: alpha = max_t ||Q[:, t]||_2 (one
// workgroup, columns strided over its threads), then x <- (mul * x) / div.
__global__ void __launch_bounds__(1024) colnorm_max_kernel(const double *Q, int r, long long T, double *out) {
  __shared__ double red[1024];
  double m = 0.0;
  for (long long t = threadIdx.x; t < T; t += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < r; ++i) {
      const double q = Q[i + t * r];
      s += q * q;
    }
    m = fmax(m, s);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(red[0]);
}
hipError_t launch_colnorm_max(const double *Q, int r, long long T, double *out, hipStream_t s) {
  hipLaunchKernelGGL(colnorm_max_kernel, dim3(1), dim3(1024), 0, s, Q, r, T, out);
  return hipGetLastError();
}

__global__ void scale_kernel(double *x, long long n, double mul, double div) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = (mul * x[i]) / div;
}
hipError_t launch_scale(double *x, long long n, double mul, double div, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, mul, div);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Data matrix of Eq. opinf_schwarz_inference, D (T x p, column-major):
// columns [q_i | q_i q_j (i<=j, row by row) | q_i q_j q_k (i<=j<=k, lexicographic;
// the cubic ansatz of COpInf) | s^_l | 1].
__global__ void data_matrix_kernel(const double *Q, int r, const double *Sh, int rs, long long T, int quad,
                                   int cubic, int with_c, double *D) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  int col = 0;
  for (int i = 0; i < r; ++i) D[t + (long long)(col++) * T] = Q[i + t * r];
  if (quad)
    for (int i = 0; i < r; ++i) {
      const double qi = Q[i + t * r];
      for (int j = i; j < r; ++j) D[t + (long long)(col++) * T] = qi * Q[j + t * r];
    }
  if (cubic)
    for (int i = 0; i < r; ++i)
      for (int j = i; j < r; ++j) {
        const double qij = Q[i + t * r] * Q[j + t * r];
        for (int k = j; k < r; ++k) D[t + (long long)(col++) * T] = qij * Q[k + t * r];
      }
  for (int l = 0; l < rs; ++l) D[t + (long long)(col++) * T] = Sh[l + t * rs];
  if (with_c) D[t + (long long)col * T] = 1.0;
}
hipError_t launch_data_matrix(const double *Q, int r, const double *Sh, int rs, long long T, int quad, int cubic,
                              int with_c, double *D, hipStream_t s) {
  hipLaunchKernelGGL(data_matrix_kernel, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, Q, r, Sh, rs, T, quad,
                     cubic, with_c, D);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Alg. 3 rollouts.  Instance = (lambda, trajectory).  Operators of lambda l:
// X_l (p x r, column-major, the ridge solution O^T), so q'' = X^T [q; q(x)q; s^; 1].
// Each workgroup runs the T-step explicit Newmark recursion with the Schwarz
// input frozen to the training data, and accumulates ||q - q_train||^2,
// ||q_train||^2, max ||q||, max ||q_train|| and a non-finite flag.
__global__ void __launch_bounds__(256) rollout_kernel(const double *X, int p, int r, int r2, int r3, int rs, int with_c,
                                                      const double *Q, const double *Qd0, const double *Qdd,
                                                      const double *Sh, long long T, int ntraj, double dt,
                                                      int stride, double *out) {
  extern __shared__ double sm[];
  double *z = sm;               // [p] regressor vector
  double *q = z + p;            // [r]
  double *qd = q + r;
  double *qdd = qd + r;
  __shared__ double red[16];
  const int inst = blockIdx.x;
  const int l = inst / ntraj, tr = inst % ntraj;
  const double *Xl = X + (long long)l * p * r;
  const double *Qt = Q + (long long)tr * T * r;
  const double *Qddt = Qdd + (long long)tr * T * r;
  const double *Sht = Sh + (long long)tr * T * rs;
  const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63, wid = tid >> 6, nw = bs >> 6;
  for (int i = tid; i < r; i += bs) {
    q[i] = Qt[i];
    qd[i] = Qd0[(long long)tr * r + i];
    qdd[i] = Qddt[i];
  }
  __syncthreads();
  double err2 = 0.0, ref2 = 0.0, qmax = 0.0, rmax = 0.0;
  int bad = 0;
  {
    double n0 = 0.0;
    for (int i = tid; i < r; i += bs) n0 += q[i] * q[i];
    n0 = block_sum(n0, red);
    ref2 += n0;
    qmax = rmax = sqrt(n0);
  }
  for (long long j = 0; j + 1 < T && !bad; ++j) {
    // `stride` steps from snapshot j to j+1; the boundary input in between is
    // interpolated linearly between the two snapshots (the last step takes S^_{j+1})
    for (int m = 1; m <= stride; ++m) {
      // predictor and regressors at the next step
      for (int i = tid; i < r; i += bs) {
        const double qn = q[i] + dt * qd[i] + 0.5 * dt * dt * qdd[i];
        z[i] = qn;
      }
      __syncthreads();
      if (r2 > 0)
        for (int e = tid; e < r * r; e += bs) {
          const int i = e / r, jj = e - i * r;
          if (jj >= i) z[r + i * r - (i * (i - 1)) / 2 + (jj - i)] = z[i] * z[jj];
        }
      if (r3 > 0)
        for (int e = tid; e < r * r; e += bs) {
          // pair (i, jj), i <= jj: the run of columns q_i q_jj q_k, k = jj .. r-1
          const int i = e / r, jj = e - i * r;
          if (jj < i) continue;
          int base = 0;
          for (int a = 0; a < i; ++a) base += (r - a) * (r - a + 1) / 2;
          for (int b = i; b < jj; ++b) base += r - b;
          const double qij = z[i] * z[jj];
          for (int k = jj; k < r; ++k) z[r + r2 + base + (k - jj)] = qij * z[k];
        }
      const double w1 = (double)m / (double)stride;
      for (int e = tid; e < rs; e += bs)
        z[r + r2 + r3 + e] = Sht[j * rs + e] + w1 * (Sht[(j + 1) * rs + e] - Sht[j * rs + e]);
      if (with_c && tid == 0) z[p - 1] = 1.0;
      __syncthreads();
      // q'' = X^T z : one wave per output
      for (int i = wid; i < r; i += nw) {
        double s = 0.0;
        const double *xc = Xl + (long long)i * p;
        for (int mm = lane; mm < p; mm += 64) s += xc[mm] * z[mm];
        s = wsum(s);
        if (lane == 0) {
          const double an = s;
          qd[i] = qd[i] + 0.5 * dt * (qdd[i] + an);
          qdd[i] = an;
        }
      }
      __syncthreads();
      for (int i = tid; i < r; i += bs) q[i] = z[i];
      __syncthreads();
    }
    double e2 = 0.0, rr = 0.0, nn = 0.0;
    for (int i = tid; i < r; i += bs) {
      const double d = q[i] - Qt[(j + 1) * r + i];
      e2 += d * d;
      rr += Qt[(j + 1) * r + i] * Qt[(j + 1) * r + i];
      nn += q[i] * q[i];
    }
    e2 = block_sum(e2, red);
    rr = block_sum(rr, red);
    nn = block_sum(nn, red);
    err2 += e2;
    ref2 += rr;
    qmax = fmax(qmax, sqrt(nn));
    rmax = fmax(rmax, sqrt(rr));
    if (!isfinite(nn) || !isfinite(e2)) bad = 1;
  }
  if (tid == 0) {
    double *o = out + (long long)inst * 5;
    o[0] = err2;
    o[1] = ref2;
    o[2] = qmax;
    o[3] = rmax;
    o[4] = bad ? 1.0 : 0.0;
  }
}
hipError_t launch_rollout(const double *X, int p, int r, int r2, int r3, int rs, int with_c, const double *Q,
                          const double *Qd0, const double *Qdd, const double *Sh, long long T, int ntraj, int nlam,
                          double dt, int stride, double *out, hipStream_t s) {
  const size_t smem = sizeof(double) * (size_t)(p + 3 * r);
  if (smem > 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rollout_kernel, dim3(nlam * ntraj), dim3(256), smem, s, X, p, r, r2, r3, rs, with_c, Q, Qd0,
                     Qdd, Sh, T, ntraj, dt, stride, out);
  return hipGetLastError();
}

}  // namespace osam
