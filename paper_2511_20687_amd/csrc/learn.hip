// OpInf learning on the GPU (Sec. 3.1 POD, Sec. 3.2 / Eq. opinf_schwarz_inference
// regularised least squares, Alg. 3 lambda selection), all in FP64 on device.
//
// POD by the method of snapshots: C = X^T X (FP64 MFMA Gram of the FP32/FP64
// snapshot matrix X, n x T), all its eigenpairs by cyclic Jacobi (one launch per
// round of n/2 disjoint rotations), then Phi = X V Lambda^-1/2 re-orthonormalised
// by Cholesky-QR and sign-normalised (largest-magnitude entry positive).  When
// n < T the n x n matrix X X^T is decomposed instead and Phi = V.
// Least squares: D = [Q^T | (Q (x) Q)^T | S^^T | 1]; primal normal equations
// (D^T D + lambda I) X = D^T R when p <= T, dual form X = D^T (D D^T + lambda I)^-1 R
// otherwise; blocked Cholesky.  Alg. 3: every lambda's operators are rolled
// out over the training time grid (Schwarz input frozen to the training data)
// in one batched kernel; lambda* = first minimiser of the relative trajectory
// error, non-finite or blow-up (||q|| > 1e6 max ||q_train||) = +inf.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <random>
#include <vector>

#include "runtime.hpp"

namespace osam {

template <typename TA, typename TB>
hipError_t gemm64(bool, bool, int, int, long long, double, const TA *, long long, const TB *, long long, double,
                  double *, long long, double *, long long, hipStream_t);
hipError_t launch_chol_lds(double *, int, long long, double, int *, hipStream_t);
hipError_t launch_trtri_lower(const double *, int, double *, hipStream_t);
hipError_t launch_ritz_resid(const double *, const double *, const double *, long long, int, double *, hipStream_t);
hipError_t launch_colscale(double *, long long, int, const double *, int, hipStream_t);
hipError_t launch_sign_fix(double *, long long, int, hipStream_t);
hipError_t launch_potrf_diag(double *, long long, int, int, int *, hipStream_t);
hipError_t launch_trsm_panel(double *, long long, int, int, int, const int *, hipStream_t);
hipError_t launch_trsv_block(const double *, long long, int, int, double *, long long, int, int, hipStream_t);
hipError_t launch_add_diag(double *, long long, int, double, hipStream_t);
hipError_t launch_colnorm_max(const double *, int, long long, double *, hipStream_t);
hipError_t launch_scale(double *, long long, double, double, hipStream_t);
hipError_t launch_data_matrix(const double *, int, const double *, int, long long, int, int, int, double *,
                              hipStream_t);
hipError_t launch_jacobi_round(const double *, double *, const double *, double *, int, int, hipStream_t);
hipError_t launch_offnorm(const double *, long long, double *, int, hipStream_t);
hipError_t launch_identity(double *, long long, hipStream_t);
hipError_t launch_diag(const double *, long long, double *, hipStream_t);
hipError_t launch_gather_cols(const double *, long long, const int *, int, double *, hipStream_t);
hipError_t launch_jacobi(double *, double *, double *, int, int *, double *, hipStream_t);
hipError_t launch_rollout(const double *, int, int, int, int, int, int, const double *, const double *,
                          const double *, const double *, long long, int, int, double, int, double *, hipStream_t);

namespace {

// Device allocations of one learning call, released together.
struct Arena {
  std::vector<void *> ptrs;
  ~Arena() {
    for (void *p : ptrs) hipFree(p);
  }
  double *d(size_t n) {
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(double)) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return static_cast<double *>(p);
  }
  int *i(size_t n) {
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(int)) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return static_cast<int *>(p);
  }
};

struct Learner {
  Ctx *ctx;
  hipStream_t s;
  Arena ar;
  double *work = nullptr;     // split-K workspace
  long long work_n = 0;
  std::string err;
  int code = OSAM_OK;

  bool ok(hipError_t e, const char *what) {
    if (e != hipSuccess && code == OSAM_OK) {
      code = OSAM_E_HIP;
      err = std::string(what) + ": " + hipGetErrorString(e);
    }
    return code == OSAM_OK;
  }
  bool fail(int c, const std::string &m) {
    if (code == OSAM_OK) {
      code = c;
      err = m;
    }
    return false;
  }
  double *alloc(size_t n) {
    double *p = ar.d(n);
    if (!p) fail(OSAM_E_OOM, "out of device memory in learning");
    return p;
  }
  template <typename TA, typename TB>
  bool gemm(bool ta, bool tb, int M, int N, long long K, double alpha, const TA *A, long long lda, const TB *B,
            long long ldb, double beta, double *C, long long ldc) {
    return ok(gemm64<TA, TB>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, work, work_n, s), "gemm");
  }
  bool sync() { return ok(hipStreamSynchronize(s), "sync"); }
  std::vector<double> down(const double *p, size_t n) {
    std::vector<double> h(n);
    ok(hipMemcpyAsync(h.data(), p, n * 8, hipMemcpyDeviceToHost, s), "copy");
    sync();
    return h;
  }
  // the diagonal of the n x n device matrix A (ld n), on the host
  std::vector<double> diagonal(const double *A, int n) {
    double *d = alloc(n);
    if (!d) return std::vector<double>(n, 0.0);
    ok(launch_diag(A, n, d, s), "diagonal");
    return down(d, (size_t)n);
  }
  void up(double *p, const std::vector<double> &h) {
    ok(hipMemcpyAsync(p, h.data(), h.size() * 8, hipMemcpyHostToDevice, s), "copy");
    sync();
  }

  // Workspace of Cholesky-QR on m x k blocks: the Gram / its factor (k x k), the inverse
  // factor (k x k), the second block the products go to (m x k), the factorisation flag.
  struct QrWork {
    double *G = nullptr, *Li = nullptr, *Wt = nullptr;
    int *info = nullptr;
  };
  bool qr_work(QrWork &w, long long m, int k) {
    w.G = alloc((size_t)k * k);
    w.Li = alloc((size_t)k * k);
    w.Wt = alloc((size_t)m * k);
    w.info = ar.i(1);
    if (!w.info) return fail(OSAM_E_OOM, "out of device memory in learning");
    return code == OSAM_OK;
  }

  // One Cholesky-QR pass: G = W^T W + shift I = L L^T, W <- W L^-T (the product with the
  // explicit inverse factor, a GEMM; W and w.Wt swap).  Returns false (without recording an
  // error) when the factorisation breaks down.
  bool cholqr_pass(double *&W, long long m, int k, double shift, QrWork &w) {
    if (!gemm<double, double>(true, false, k, k, m, 1.0, W, m, W, m, 0.0, w.G, k)) return false;
    if (!ok(launch_chol_lds(w.G, k, k, shift, w.info, s), "chol")) return false;
    int hinfo = 0;
    ok(hipMemcpyAsync(&hinfo, w.info, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    sync();
    if (code || hinfo != 0) return false;
    if (!ok(launch_trtri_lower(w.G, k, w.Li, s), "trtri")) return false;
    if (!gemm<double, double>(false, true, (int)m, k, k, 1.0, W, m, w.Li, k, 0.0, w.Wt, m)) return false;
    std::swap(W, w.Wt);
    return code == OSAM_OK;
  }

  // Cholesky-QR2: W (m x k) <- W R^-1 with orthonormal columns.  Returns false
  // (without recording an error) when the block is numerically rank deficient.
  bool cholqr(double *&W, long long m, int k, QrWork &w) {
    return cholqr_pass(W, m, k, 0.0, w) && cholqr_pass(W, m, k, 0.0, w);
  }

  // All eigenpairs of the symmetric matrix C (n x n, destroyed) by cyclic
  // Jacobi sweeps until off(A)^2 <= 1e-30 ||A||^2.  theta: descending (host);
  // V: device n x k, the eigenvectors of the k largest.
  bool eig_all(double *C, int n, int k, std::vector<double> &theta, double *&V) {
    double *A1 = alloc((size_t)n * n), *V0 = alloc((size_t)n * n), *V1 = alloc((size_t)n * n);
    const int nb = 256;
    double *part = alloc(2 * nb);
    int *ord = ar.i(n);
    if (code) return false;
    ok(launch_identity(V0, n, s), "identity");
    double *Ain = C, *Aout = A1, *Vin = V0, *Vout = V1;
    const int nn = n + (n & 1);
    for (int sweep = 0; sweep < 40; ++sweep) {
      ok(launch_offnorm(Ain, n, part, nb, s), "offnorm");
      std::vector<double> h = down(part, 2 * nb);
      double off = 0.0, tot = 0.0;
      for (int i = 0; i < nb; ++i) {
        off += h[2 * i];
        tot += h[2 * i + 1];
      }
      if (code) return false;
      if (off <= 1e-30 * tot || tot == 0.0) break;
      for (int rnd = 0; rnd < nn - 1; ++rnd) {
        if (!ok(launch_jacobi_round(Ain, Aout, Vin, Vout, n, rnd, s), "jacobi round")) return false;
        std::swap(Ain, Aout);
        std::swap(Vin, Vout);
      }
    }
    // eigenvalues = diagonal, sorted descending (stable on ties)
    const std::vector<double> diag = diagonal(Ain, n);
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return diag[a] > diag[b]; });
    theta.resize(n);
    for (int i = 0; i < n; ++i) theta[i] = diag[order[i]];
    ok(hipMemcpyAsync(ord, order.data(), sizeof(int) * n, hipMemcpyHostToDevice, s), "copy");
    V = alloc((size_t)n * k);
    if (code) return false;
    ok(launch_gather_cols(Vin, n, ord, k, V, s), "gather");
    sync();
    return code == OSAM_OK;
  }

  // Orthonormal basis of the column space of W (m x k) by shifted Cholesky-QR (Fukaya,
  // Kannan, Nakatsukasa, Yamamoto, Yanagisawa 2020): Cholesky-QR passes on W^T W + s I with
  // s = 11 (m k + k (k + 1)) u ||W||_F^2 of the current block until its Gram is within 0.1 of
  // the identity entrywise, then one unshifted pass.  Blocks with kappa(W) up to 1/u take
  // two shifted passes (the shifted Cholesky-QR3 of the paper cited).  Directions of W below
  // that (columns that are numerically dependent: the part of the subspace iteration's
  // block beyond the numerical rank of the Gram) grow by about 1/sqrt(s) per further
  // shifted pass until the block is well conditioned, and come out as orthonormal directions
  // of no significance.  Returns false (code OK) when 12 shifted passes do not get there.
  bool orth(double *&W, long long m, int k, QrWork &w) {
    std::vector<double> g((size_t)k * k);
    for (int pass = 0; pass < 12; ++pass) {
      if (!gemm<double, double>(true, false, k, k, m, 1.0, W, m, W, m, 0.0, w.G, k)) return false;
      ok(hipMemcpyAsync(g.data(), w.G, g.size() * sizeof(double), hipMemcpyDeviceToHost, s), "copy");
      sync();
      if (code) return false;
      double fro2 = 0.0, dev = 0.0;
      for (int j = 0; j < k; ++j) {
        fro2 += g[(size_t)j * (k + 1)];
        for (int i = 0; i < k; ++i) dev = std::max(dev, std::fabs(g[i + (size_t)j * k] - (i == j ? 1.0 : 0.0)));
      }
      if (!(fro2 > 0.0) || !std::isfinite(fro2)) return false;
      if (dev <= 0.1) return cholqr_pass(W, m, k, 0.0, w);
      const double shift = 11.0 * ((double)m * k + (double)k * (k + 1)) * std::numeric_limits<double>::epsilon() * fro2;
      if (!ok(launch_chol_lds(w.G, k, k, shift, w.info, s), "chol")) return false;
      int hinfo = 0;
      ok(hipMemcpyAsync(&hinfo, w.info, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
      sync();
      if (code || hinfo != 0) return false;
      if (!ok(launch_trtri_lower(w.G, k, w.Li, s), "trtri")) return false;
      if (!gemm<double, double>(false, true, (int)m, k, k, 1.0, W, m, w.Li, k, 0.0, w.Wt, m)) return false;
      std::swap(W, w.Wt);
    }
    return false;
  }

  // Rayleigh-Ritz on the n x b orthonormal block Y: H = Y^T (C Y), its eigenpairs by one
  // workgroup's cyclic Jacobi, Y <- Y W (Ritz vectors), Z <- Z W (= C Y); w: the Ritz values
  // (device, descending).
  bool rayleigh_ritz(const double *C, int n, int b, double *&Y, double *&Z, double *&Y2, double *H, double *Wm,
                     double *w, int *pws, double *cws) {
    if (!gemm<double, double>(false, false, n, b, n, 1.0, C, n, Y, n, 0.0, Z, n)) return false;
    if (!gemm<double, double>(true, false, b, b, n, 1.0, Y, n, Z, n, 0.0, H, b)) return false;
    if (!ok(launch_jacobi(H, Wm, w, b, pws, cws, s), "jacobi")) return false;
    if (!gemm<double, double>(false, false, n, b, b, 1.0, Y, n, Wm, b, 0.0, Y2, n)) return false;
    std::swap(Y, Y2);
    if (!gemm<double, double>(false, false, n, b, b, 1.0, Z, n, Wm, b, 0.0, Y2, n)) return false;
    std::swap(Z, Y2);
    return code == OSAM_OK;
  }

  // The k largest eigenpairs of the symmetric positive semidefinite C (n x n, kept):
  // block subspace iteration Y <- orth(C Y) (shifted Cholesky-QR) with a Rayleigh-Ritz
  // step every 4 iterations, block b = min(n, k + 32), from a seeded Gaussian start; for
  // b == n the Rayleigh-Ritz step is the whole eigen-decomposition.  Converged when each of
  // the k leading Ritz pairs has ||C y - theta y|| <= 1e-13 theta_1.  theta: the k leading
  // Ritz values (host, descending); V: device n x k.  Returns false with code OK when it
  // did not converge within 400 iterations or the block lost rank (the caller falls back
  // to eig_all).
  bool eig_top(const double *C, int n, int k, std::vector<double> &theta, double *&V) {
    const int b = std::min(n, k + 32);
    double *Y = alloc((size_t)n * b), *Z = alloc((size_t)n * b), *Y2 = alloc((size_t)n * b);
    double *H = alloc((size_t)b * b), *Wm = alloc((size_t)b * b), *w = alloc(b), *res = alloc(k);
    double *cws = alloc((size_t)b + 2);
    int *pws = ar.i((size_t)b + 2);
    QrWork qw;
    if (!qr_work(qw, n, b) || code || !pws) return fail(OSAM_E_OOM, "out of device memory in learning");
    if (b == n) {
      ok(launch_identity(Y, n, s), "identity");
    } else {
      std::vector<double> y((size_t)n * b);
      std::mt19937_64 gen(0x5eed0f00dULL);
      std::normal_distribution<double> nd(0.0, 1.0);
      for (double &v : y) v = nd(gen);
      up(Y, y);
      if (!orth(Y, n, b, qw)) return false;
    }
    std::vector<double> th;
    for (int it = 0; it < 400; ++it) {
      if (b < n) {   // Y <- orth(C Y)
        if (!gemm<double, double>(false, false, n, b, n, 1.0, C, n, Y, n, 0.0, Z, n)) return false;
        std::swap(Y, Z);
        if (!orth(Y, n, b, qw)) return false;
      }
      if (b < n && it % 4 != 3) continue;
      if (!rayleigh_ritz(C, n, b, Y, Z, Y2, H, Wm, w, pws, cws)) return false;
      th = down(w, (size_t)k);
      if (b == n) break;
      // residuals of the k leading Ritz pairs: Z - Y diag(theta) (Z = C Y after the rotation)
      if (!ok(launch_ritz_resid(Z, Y, w, n, k, res, s), "residual")) return false;
      const std::vector<double> r2 = down(res, (size_t)k);
      if (code) return false;
      double worst = 0.0;
      for (double v : r2) worst = std::max(worst, std::sqrt(v));
      if (!(worst > 1e-13 * std::max(th[0], 0.0))) break;
      if (it == 399) return false;
    }
    theta = th;
    V = Y;
    return code == OSAM_OK;
  }

  // POD basis of X (nr x nc, column-major, ld nr, type T): Phi (device nr x r, FP64); sigma:
  // the leading singular values computed (at least min_k of them when r is fixed).
  template <typename T>
  bool pod(const T *X, long long nr, long long nc, int r_fixed, double energy, int min_k, double *&Phi, int &r,
           std::vector<double> &sigma) {
    const bool snap = nr >= nc;
    const int n = (int)(snap ? nc : nr);
    double *C = alloc((size_t)n * n);
    if (code) return false;
    if (snap) {
      if (!gemm<T, T>(true, false, n, n, nr, 1.0, X, nr, X, nr, 0.0, C, n)) return false;
    } else {
      if (!gemm<T, T>(false, true, n, n, nc, 1.0, X, nr, X, nr, 0.0, C, n)) return false;
    }
    std::vector<double> theta;
    double *V = nullptr;
    const int kmax = std::min(n, 128);   // POD bases hold at most 128 modes
    if (r_fixed > 128) return fail(OSAM_E_INVALID, "POD basis larger than 128 modes");
    // the total energy is the trace of the Gram (the sum of all its eigenvalues)
    const std::vector<double> dg = diagonal(C, n);
    double trace = 0.0;
    for (double v : dg) trace += v;
    if (code) return false;
    // energy criterion (Eq. pod_energy): smallest r with E_r >= energy, over the leading
    // eigenvalues at hand (0 when they do not reach it)
    const double tot = std::max(trace, 0.0);
    auto energy_r = [&](const std::vector<double> &th) {
      double cum = 0.0;
      for (size_t i = 0; i < th.size(); ++i) {
        cum += std::max(th[i], 0.0);
        if (tot > 0.0 && cum >= energy * tot) return (int)i + 1;
      }
      return 0;
    };
    // the leading eigenpairs only: the r asked for (at least min_k, the singular values
    // reported), or for the energy criterion 16, 64, then 128 of them until the criterion is
    // met; the full cyclic Jacobi when the subspace iteration does not converge
    bool top = false;
    if (r_fixed > 0) {
      top = eig_top(C, n, std::min(n, std::max(r_fixed, min_k)), theta, V);
    } else {
      for (int kk : {16, 64, 128}) {
        kk = std::min(kk, kmax);
        top = eig_top(C, n, kk, theta, V);
        if (!top || energy_r(theta) > 0 || kk == kmax) break;
      }
    }
    if (!top) {
      if (code) return false;
      if (!eig_all(C, n, kmax, theta, V)) return false;
    }
    if (r_fixed > 0) {
      r = std::min(r_fixed, n);
    } else {
      r = energy_r(theta);
      if (r == 0) r = (int)theta.size() < n ? kmax + 1 : n;   // not met within the leading kmax
    }
    if (r < 1) return fail(OSAM_E_INVALID, "empty POD basis");
    if (r > 128) return fail(OSAM_E_INVALID, "POD basis larger than 128 modes");
    sigma.assign(theta.begin(), theta.end());
    for (double &v : sigma) v = std::sqrt(std::max(v, 0.0));
    Phi = alloc((size_t)nr * r);
    if (code) return false;
    if (snap) {
      for (int j = 0; j < r; ++j)
        if (!(theta[j] > 0.0)) return fail(OSAM_E_SINGULAR, "zero singular value inside the POD basis");
      if (!gemm<T, double>(false, false, (int)nr, r, nc, 1.0, X, nr, V, nc, 0.0, Phi, nr)) return false;
      std::vector<double> sv(r);
      for (int j = 0; j < r; ++j) sv[j] = 1.0 / std::sqrt(theta[j]);
      double *f = alloc(r);
      up(f, sv);
      ok(launch_colscale(Phi, nr, r, f, 0, s), "colscale");
      QrWork qw;
      if (!qr_work(qw, nr, r)) return false;
      if (!cholqr(Phi, nr, r, qw)) {
        if (code) return false;
        return fail(OSAM_E_SINGULAR, "POD basis is not of full rank");
      }
    } else {
      ok(hipMemcpyAsync(Phi, V, (size_t)nr * r * 8, hipMemcpyDeviceToDevice, s), "copy");
    }
    ok(launch_sign_fix(Phi, nr, r, s), "signfix");
    return code == OSAM_OK;
  }

  // Blocked Cholesky of A (n x n, ld n) in place; returns false when not SPD.
  bool potrf(double *A, int n, int *info, bool &spd) {
    ok(hipMemsetAsync(info, 0, sizeof(int), s), "memset");
    for (int j0 = 0; j0 < n; j0 += 64) {
      const int nb = std::min(64, n - j0);
      ok(launch_potrf_diag(A, n, j0, nb, info, s), "potrf");
      ok(launch_trsm_panel(A, n, n, j0, nb, info, s), "trsm");
      const int m = n - j0 - nb;
      if (m > 0) {
        double *L21 = A + (j0 + nb) + (long long)j0 * n;
        double *A22 = A + (j0 + nb) + (long long)(j0 + nb) * n;
        if (!gemm<double, double>(false, true, m, m, nb, -1.0, L21, n, L21, n, 1.0, A22, n)) return false;
      }
    }
    int h = 0;
    ok(hipMemcpyAsync(&h, info, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    sync();
    spd = (h == 0);
    return code == OSAM_OK;
  }

  // Y (n x m, ld n) <- (L L^T)^-1 Y
  bool potrs(const double *L, int n, double *Y, int m) {
    for (int j0 = 0; j0 < n; j0 += 64) {
      const int nb = std::min(64, n - j0);
      ok(launch_trsv_block(L, n, j0, nb, Y, n, m, 0, s), "trsv");
      const int rest = n - j0 - nb;
      if (rest > 0 &&
          !gemm<double, double>(false, false, rest, m, nb, -1.0, L + (j0 + nb) + (long long)j0 * n, n, Y + j0, n, 1.0,
                                Y + j0 + nb, n))
        return false;
    }
    for (int j0 = ((n - 1) / 64) * 64; j0 >= 0; j0 -= 64) {
      const int nb = std::min(64, n - j0);
      ok(launch_trsv_block(L, n, j0, nb, Y, n, m, 1, s), "trsv");
      if (j0 > 0 &&
          !gemm<double, double>(true, false, j0, m, nb, -1.0, L + j0, n, Y + j0, n, 1.0, Y, n))
        return false;
    }
    return code == OSAM_OK;
  }
};

}  // namespace

template <typename T>
static int32_t learn_impl(Ctx *ctx, int sdi, const osam_opinf_desc &d) {
  Subdomain &sd = *ctx->sds[sdi];
  Learner L;
  L.ctx = ctx;
  L.s = ctx->stream;
  const long long N = 3 * sd.nfree_nodes, NS = 3 * sd.nsch_nodes;
  const int ntraj = d.n_traj;
  const long long Tn = d.T, Tt = (long long)ntraj * Tn;
  const T *U = static_cast<const T *>(d.U);
  const T *Udd = static_cast<const T *>(d.Udd);
  const T *S = static_cast<const T *>(d.S);
  const T *V0 = static_cast<const T *>(d.V0);
  L.work_n = 1 << 26;   // 512 MB split-K workspace upper bound
  L.work = L.alloc((size_t)L.work_n);
  if (L.code) return ctx->fail(L.code, L.err);

  // 1. POD bases (interior and Schwarz boundary)
  double *Phi = nullptr, *PhiS = nullptr;
  int r = 0, rs = 0;
  std::vector<double> sig, sigS;
  if (!L.pod<T>(U, N, Tt, d.r, d.energy, 16, Phi, r, sig)) return ctx->fail(L.code, L.err);
  if (NS > 0) {
    if (!L.pod<T>(S, NS, Tt, d.r_s, d.energy_bnd, 1, PhiS, rs, sigS)) return ctx->fail(L.code, L.err);
  }
  const int quad = d.form == OSAM_QUADRATIC || d.form == OSAM_CUBIC;
  const int cubic = d.form == OSAM_CUBIC;
  const int r2 = quad ? r * (r + 1) / 2 : 0;
  const int r3 = cubic ? r * (r + 1) * (r + 2) / 6 : 0;
  const int with_c = d.with_c ? 1 : 0;
  const int p = r + r2 + r3 + rs + with_c;

  // 2. reduced data Q = Phi^T U, Qdd = Phi^T U'', S^ = Phi_S^T S, q'0 = Phi^T v0
  double *Q = L.alloc((size_t)r * Tt), *Qdd = L.alloc((size_t)r * Tt), *Qd0 = L.alloc((size_t)r * ntraj);
  double *Sh = L.alloc((size_t)std::max(rs, 1) * Tt);
  if (L.code) return ctx->fail(L.code, L.err);
  L.gemm<double, T>(true, false, r, (int)Tt, N, 1.0, Phi, N, U, N, 0.0, Q, r);
  L.gemm<double, T>(true, false, r, (int)Tt, N, 1.0, Phi, N, Udd, N, 0.0, Qdd, r);
  L.gemm<double, T>(true, false, r, ntraj, N, 1.0, Phi, N, V0, N, 0.0, Qd0, r);
  if (rs > 0) L.gemm<double, T>(true, false, rs, (int)Tt, NS, 1.0, PhiS, NS, S, NS, 0.0, Sh, rs);
  // normalised variables of the fit: tau = t/dt, q/alpha, s^/alpha (Sec. 4.2.1 leaves
  // the units open; the regularisation grid of Sec. 5 presumes operators of order one)
  const double dt = sd.desc.dt, dt2 = dt * dt;
  double *amax = L.alloc(1);
  if (L.code) return ctx->fail(L.code, L.err);
  L.ok(launch_colnorm_max(Q, r, Tt, amax, L.s), "alpha");
  double alpha = L.down(amax, 1)[0];
  if (L.code) return ctx->fail(L.code, L.err);
  if (!(alpha > 0.0) || !std::isfinite(alpha)) {
    if (!std::isfinite(alpha)) return ctx->fail(OSAM_E_NONFINITE, "non-finite training snapshots");
    alpha = 1.0;
  }
  L.ok(launch_scale(Q, (long long)r * Tt, 1.0, alpha, L.s), "scale");
  L.ok(launch_scale(Qdd, (long long)r * Tt, dt2, alpha, L.s), "scale");
  L.ok(launch_scale(Qd0, (long long)r * ntraj, dt, alpha, L.s), "scale");
  if (rs > 0) L.ok(launch_scale(Sh, (long long)rs * Tt, 1.0, alpha, L.s), "scale");
  double *D = L.alloc((size_t)Tt * p);
  if (L.code) return ctx->fail(L.code, L.err);
  L.ok(launch_data_matrix(Q, r, Sh, rs, Tt, quad, cubic, with_c, D, L.s), "data matrix");

  // 3. normal equations (primal when p <= T, dual otherwise)
  const bool primal = p <= Tt;
  const int n = primal ? p : (int)Tt;
  double *G = L.alloc((size_t)n * n), *Gl = L.alloc((size_t)n * n);
  double *F = L.alloc((size_t)n * r);              // primal: D^T R ; dual: R
  const int nlam = std::max(1, d.n_lambda);
  double *Xall = L.alloc((size_t)nlam * p * r);
  int *info = L.ar.i(1);
  if (L.code) return ctx->fail(L.code, L.err);
  if (primal) {
    L.gemm<double, double>(true, false, p, p, Tt, 1.0, D, Tt, D, Tt, 0.0, G, p);
    L.gemm<double, double>(true, true, p, r, Tt, 1.0, D, Tt, Qdd, r, 0.0, F, p);
  } else {
    L.gemm<double, double>(false, true, (int)Tt, (int)Tt, p, 1.0, D, Tt, D, Tt, 0.0, G, Tt);
    // R = Qdd^T (Tt x r)
    std::vector<double> qh = L.down(Qdd, (size_t)r * Tt), rh((size_t)Tt * r);
    for (long long t = 0; t < Tt; ++t)
      for (int i = 0; i < r; ++i) rh[(size_t)t + (size_t)i * Tt] = qh[(size_t)i + (size_t)t * r];
    L.up(F, rh);
  }
  std::vector<double> lam(d.lambdas ? std::vector<double>(d.lambdas, d.lambdas + nlam) : std::vector<double>{0.0});
  std::vector<char> spd_ok(nlam, 0);
  double *Ysol = L.alloc((size_t)n * r);
  if (L.code) return ctx->fail(L.code, L.err);
  for (int l = 0; l < nlam; ++l) {
    L.ok(hipMemcpyAsync(Gl, G, (size_t)n * n * 8, hipMemcpyDeviceToDevice, L.s), "copy");
    L.ok(launch_add_diag(Gl, n, n, lam[l], L.s), "diag");
    bool spd = false;
    if (!L.potrf(Gl, n, info, spd)) return ctx->fail(L.code, L.err);
    double *X = Xall + (size_t)l * p * r;
    if (!spd) {
      L.ok(hipMemsetAsync(X, 0, (size_t)p * r * 8, L.s), "memset");
      continue;
    }
    spd_ok[l] = 1;
    L.ok(hipMemcpyAsync(Ysol, F, (size_t)n * r * 8, hipMemcpyDeviceToDevice, L.s), "copy");
    if (!L.potrs(Gl, n, Ysol, r)) return ctx->fail(L.code, L.err);
    if (primal) {
      L.ok(hipMemcpyAsync(X, Ysol, (size_t)p * r * 8, hipMemcpyDeviceToDevice, L.s), "copy");
    } else {
      L.gemm<double, double>(true, false, p, r, Tt, 1.0, D, Tt, Ysol, Tt, 0.0, X, p);
    }
  }

  // 4. Alg. 3: frozen-boundary rollouts of every lambda on every trajectory
  std::vector<double> E(nlam, std::numeric_limits<double>::infinity());
  int best = 0;
  if (nlam > 1) {
    double *ro = L.alloc((size_t)nlam * ntraj * 5);
    if (L.code) return ctx->fail(L.code, L.err);
    L.ok(launch_rollout(Xall, p, r, r2, r3, rs, with_c, Q, Qd0, Qdd, Sh, Tn, ntraj, nlam, 1.0, std::max(1, d.stride), ro,
                        L.s),
         "rollout");
    std::vector<double> h = L.down(ro, (size_t)nlam * ntraj * 5);
    if (L.code) return ctx->fail(L.code, L.err);
    for (int l = 0; l < nlam; ++l) {
      if (!spd_ok[l]) continue;
      double acc = 0.0;
      bool bad = false;
      for (int t = 0; t < ntraj; ++t) {
        const double *o = &h[((size_t)l * ntraj + t) * 5];
        if (o[4] != 0.0 || !(o[2] <= 1e6 * o[3]) || !(o[1] > 0.0)) bad = true;
        acc += std::sqrt(o[0] / o[1]);
      }
      E[l] = bad ? std::numeric_limits<double>::infinity() : acc / ntraj;
    }
    for (int l = 1; l < nlam; ++l)
      if (E[l] < E[best]) best = l;
  } else {
    E[0] = 0.0;
  }
  if (!spd_ok[best]) return ctx->fail(OSAM_E_SINGULAR, "no regularisation parameter gives an SPD system");

  // 5. operators of lambda* (the fit at lambda* is the refit of Alg. 3), in physical units
  std::vector<double> X = L.down(Xall + (size_t)best * p * r, (size_t)p * r);
  OpinfHost oh;
  oh.r = r;
  oh.rs = rs;
  oh.quadratic = quad != 0;
  oh.A.assign((size_t)r * r, 0.0);
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) oh.A[(size_t)i + (size_t)j * r] = X[(size_t)j + (size_t)i * p] / dt2;
  if (quad) {
    oh.H.assign((size_t)r * r2, 0.0);
    for (int i = 0; i < r; ++i)
      for (int m = 0; m < r2; ++m) oh.H[(size_t)i + (size_t)m * r] = X[(size_t)(r + m) + (size_t)i * p] / (dt2 * alpha);
  }
  if (cubic) {
    oh.C3.assign((size_t)r * r3, 0.0);
    for (int i = 0; i < r; ++i)
      for (int m = 0; m < r3; ++m)
        oh.C3[(size_t)i + (size_t)m * r] = X[(size_t)(r + r2 + m) + (size_t)i * p] / (dt2 * alpha * alpha);
  }
  if (rs > 0) {
    oh.B.assign((size_t)r * rs, 0.0);
    for (int i = 0; i < r; ++i)
      for (int l2 = 0; l2 < rs; ++l2)
        oh.B[(size_t)i + (size_t)l2 * r] = X[(size_t)(r + r2 + r3 + l2) + (size_t)i * p] / dt2;
    oh.PhiS = L.down(PhiS, (size_t)NS * rs);
  }
  if (with_c) {
    oh.c.assign(r, 0.0);
    for (int i = 0; i < r; ++i) oh.c[i] = X[(size_t)(p - 1) + (size_t)i * p] * alpha / dt2;
  }
  if (L.code) return ctx->fail(L.code, L.err);
  int32_t st = ctx->install_opinf_device(sdi, oh, Phi);
  if (st) return st;
  if (d.sigma_out) {
    const long long nsig = std::min<long long>(N, Tt);
    for (long long i = 0; i < nsig; ++i) d.sigma_out[i] = i < (long long)sig.size() ? sig[i] : 0.0;
  }
  if (d.E_lambda_out)
    for (int l = 0; l < nlam; ++l) d.E_lambda_out[l] = E[l];
  if (d.lambda_star_out) *d.lambda_star_out = lam[best];
  if (d.r_out) *d.r_out = r;
  if (d.rs_out) *d.rs_out = rs;
  return OSAM_OK;
}

int32_t Ctx::learn(int sdi, const osam_opinf_desc &d) {
  Subdomain &sd = *sds[sdi];
  if (sd.rom) return fail(OSAM_E_INVALID, "subdomain is already an OpInf model");
  if (d.n_traj < 1 || d.T < 2 || !d.U || !d.Udd || !d.V0 || (sd.nsch_nodes > 0 && !d.S))
    return fail(OSAM_E_INVALID, "bad snapshot description");
  if (d.form != OSAM_LINEAR && d.form != OSAM_QUADRATIC && d.form != OSAM_CUBIC) return fail(OSAM_E_INVALID, "bad form");
  if (d.r <= 0 && !(d.energy > 0.0 && d.energy <= 1.0)) return fail(OSAM_E_INVALID, "bad energy threshold");
  if (d.n_lambda < 0 || (d.n_lambda > 0 && !d.lambdas)) return fail(OSAM_E_INVALID, "bad lambda grid");
  for (int l = 0; l < d.n_lambda; ++l)
    if (!(d.lambdas[l] >= 0.0)) return fail(OSAM_E_INVALID, "lambda must be >= 0");
  if (prec == OSAM_FP64) return learn_impl<double>(this, sdi, d);
  return learn_impl<float>(this, sdi, d);
}

}  // namespace osam

extern "C" int32_t learn_opinf(osam_ctx *c, int32_t sd, const osam_opinf_desc *desc) {
  if (!c || !desc) return OSAM_E_INVALID;
  osam::Ctx *ctx = reinterpret_cast<osam::Ctx *>(c);
  ctx->err.clear();
  if (sd < 0 || sd >= (int)ctx->sds.size()) return ctx->fail(OSAM_E_INVALID, "bad subdomain id");
  hipSetDevice(ctx->device);
  return ctx->learn(sd, *desc);
}
