// Device structures of the window engine: the Schwarz controller for subdomains
// that advance a controller step in several Newmark steps (Sec. 4.1, mixed time
// steps with the temporal interpolant Xi) or with the implicit Newmark scheme
// (Sec. 4.1, beta > 0).  Unlike the explicit single-step path, a subdomain's
// free DOFs then depend on the Schwarz data of every iteration, so each Schwarz
// iteration restarts the window from the accepted state at t_{k-1} and marches
// its sub-steps, reading the neighbours' trajectories over the window.
#pragma once
#include "osam_device.hpp"

namespace osam {

constexpr int kWinMaxExp = 4;   // faces of other subdomains one subdomain feeds
constexpr int kWinFomThreads = 512;
constexpr int kWinRomThreads = 256;
constexpr size_t kWinLdsBytes = 144 * 1024;   // dynamic LDS of the FOM kernel's LDS-resident variant

// The source of one Schwarz face.
template <typename T>
struct WinSrc {
  int kind;             // 0: clamped face (no source), 1: FOM source, 2: OpInf source
  int sd;               // the source's index in the Schwarz order
  int n_sub;            // the source's Newmark steps per controller step
  int layer;            // source-local node layer that coincides with the face
  int npl;              // nodes per layer (the grid is shared)
  int r;                // OpInf source: reduced dimension
  long long cs, is;     // FOM source: component and instance strides
  const T *u[3], *v[2], *a[2];      // FOM source: accepted state by role (step % 3, step % 2)
  const T *q[2], *qd[2], *qdd[2];   // OpInf source: accepted state by step parity, [batch][r]
  const T *rows;        // OpInf source: rows of Pi Phi on the face, [r][3 npl]
  const T *traj[2];     // the source's face values after its sub-steps 1 .. n_sub, by the
                        // parity of the Schwarz iteration that wrote them: [n_sub][batch][3 npl]
  int batch;
};

template <typename T>
struct WinFomArgs {
  int nx, ny, nzs, npl;
  long long cs, is, nnodes;
  T *u[3], *v[2], *a[2];          // accepted state by role
  T *wu[2], *wv[2], *wa[2];       // state at the end of the window, by iteration parity
  T *tu[2], *tv[2], *ta[2];       // states after the inner sub-steps of the window
  T *cr, *cp, *cq;                // conjugate-gradient vectors [batch][3][cs] (implicit)
  const T *coef;                  // [9 cases][26 offsets][3][3]: -K_d / m
  T cb[27];                       // the interior block's 27 distinct values
  T dt, beta, gamma;              // sub-step and Newmark parameters
  int n_sub, l;                   // sub-steps per controller step, this sub-step (1 .. n_sub)
  int implicit;
  double cg_tol2;                 // relative residual (M-norm) at which CG stops, squared
  int cg_max;
  int additive, guess;
  WinSrc<T> src[2];               // low and high z-face
  int nexp;
  T *exp_traj[kWinMaxExp][2];     // faces fed by this subdomain: [n_sub][batch][3 npl] by parity
  int exp_layer[kWinMaxExp];
  const Status *status;
  int sd, nsd;
  double *sums;                   // [batch][nsd][2]: Eq. conv_criterion sums of this iteration
  int *cg_iters;                  // [batch]: most CG iterations of any solve (statistics)
  // Saint Venant-Kirchhoff material (App. A.2): the internal force of the box
  // elements evaluated at the 2x2x2 Gauss points instead of the linear stencil
  int material;                   // 0 linear elastic, 1 Saint Venant-Kirchhoff
  T lam, mu, hx, hy, hz, rho;
  int lateral_fix;                // components held at zero on the lateral faces
  T *rec_a0;                      // SVK initial state: column 0 of the acceleration record, or null
  long long rec_ncols, nfree_nodes;
};

template <typename T>
struct WinRomArgs {
  int r, rs, r2, r3;              // r2 = r(r+1)/2 (quadratic), r3 = r(r+1)(r+2)/6 (cubic), else 0
  const T *A, *H, *C3, *B, *c;    // row-major [r][...]; null when absent
  const T *Minv;                  // [r][r] row-major (I - beta dt^2 A)^-1 (implicit)
  T *q[2], *qd[2], *qdd[2];       // accepted state by step parity, [batch][r]
  T *wq[2], *wqd[2], *wqdd[2];    // end of the window by iteration parity
  T *tq[2], *tqd[2], *tqdd[2];    // inner sub-steps
  T *sbuf;                        // [batch][2][3 npl]: Schwarz values of the current sub-step
  T *kbuf;                        // [batch][r2 + r3]: compressed powers of the current q
  int npl;
  const T *phis[2];               // [rs][3 npl] block of Phi_S per face (null: clamped)
  WinSrc<T> src[2];
  T dt, beta, gamma;
  int n_sub, l, implicit, newton_max;
  double newton_tol2;             // relative size of the last correction at which Newton stops, squared
  int additive, guess;
  int nexp;
  T *exp_traj[kWinMaxExp][2];
  const T *exp_rows[kWinMaxExp];  // [r][3 npl] rows of Pi Phi on each fed face
  const Status *status;
  int sd, nsd;
  double *sums;
  int *newton_iters;              // [batch]
};

// Acceptance of a converged window: the end state becomes the accepted state of
// the new step (roles of step + 1), records are written.
template <typename T>
struct WinAcceptArgs {
  int rom;
  long long cs, is, nnodes;       // FOM
  int npl, nzs;
  long long nfree_nodes, nsch_nodes, face_off_hi;
  int face_sch[2];                // 1: the face is a Schwarz face (recorded in s)
  T *u[3], *v[2], *a[2];
  const T *wu[2], *wv[2], *wa[2];
  int r;                          // OpInf
  T *q[2], *qd[2], *qdd[2];
  const T *wq[2], *wqd[2], *wqdd[2];
  T *rec_u, *rec_a, *rec_s;
  long long rec_every, rec_ncols;
  const Status *status;
};

template <typename T>
hipError_t launch_win_fom(const WinFomArgs<T> &A, int batch, hipStream_t s);
template <typename T>
hipError_t launch_win_svk_init(const WinFomArgs<T> &A, int batch, hipStream_t s);
template <typename T>
hipError_t launch_win_rom(const WinRomArgs<T> &A, int batch, hipStream_t s);
hipError_t launch_win_decide(Status *st, const double *sums, const Opts &o, int batch, hipStream_t s);
template <typename T>
hipError_t launch_win_accept(const WinAcceptArgs<T> &A, int batch, hipStream_t s);

}  // namespace osam
