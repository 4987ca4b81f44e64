// Argument structures shared by the adjoint kernels and their host driver.
#pragma once
#include <hip/hip_runtime.h>

namespace osam {

template <typename T>
struct SlabGeo {
  int nx, ny, nzs, npl;
  long long cs;            // component stride of a [3][cs] field
  const T *coef;           // [9 cases][234]
  T mass[9];               // lumped mass of a node of each case on a full layer
  int held;                // lateral components held at zero (bit mask)
};

// Arguments of the OpInf forward / adjoint kernels (one workgroup, one subdomain).
template <typename T>
struct RomAdj {
  int r, rs, r2;
  const T *A, *H, *B, *c;   // row-major operators (c may be null)
  T dt, g, h;               // dt, dt/2, dt^2/2
  // state (forward)
  T *q, *qd, *qdd;          // state at t_{k-1}, overwritten with t_k
  const T *gh;              // g^_k (forward: computed by rows_dot before the kernel)
  T *tape_q, *tape_g;       // [r], [rs] at this step (forward writes, adjoint reads)
  // adjoint
  T *Q, *Qd, *Qdd, *Qdd_prev;   // adjoints of q, q', q'' at t_k and the accumulator of q''_{k-1}
  const T *obs;             // observed q at this step or null
  double *dA, *dH, *dB, *dc;    // FP64 gradient accumulators, row-major
  T *gbar;                  // out: B^T Qdd (rs)
  double *partial;          // misfit partial (1 value)
  int mode;                 // adjoint: 0 = full step, 1 = initial state (no velocity / predictor / g^ outputs)
};

}  // namespace osam
