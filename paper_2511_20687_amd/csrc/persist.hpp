// Arguments of the persistent OpInf engine (persist_kernels.hip): every subdomain's
// OpInf step arguments and where its state and operators live in the workgroup's LDS.
#pragma once
#include "osam_device.hpp"

namespace osam {

constexpr int kPersistMax = 4;                  // OpInf subdomains of one context
constexpr size_t kPersistLds = 159 * 1024;      // dynamic LDS of the workgroup

// Offsets (elements of the context precision) into the dynamic LDS; -1: the operator
// stays in global memory.
struct PersistLayout {
  int q[2], v[2], a[2];   // state by step parity (accepted: step % 2; iterates: the other)
  int q1, qp;             // predictor q(t_k) of the step; predictor of the latest iterate
  int f0;                 // the (A q + H (q (x) q)) rows of the step
  int am, h, bm, c;       // A [r][r], H [r][r2] (or -1: global), B [r][rs], c [r] (row-major)
  int tm[2];              // Phi_S,face^T Pi Phi_src [rs][r_src] per face (B, c, tm: always in LDS)
};

template <typename T>
struct PersistArgs {
  int nsd;
  int slot[kMaxSd];       // context subdomain id -> slot in sd[] / lay[]
  int sh_off, k2_off, rows_off;   // scratch shared by the subdomains: g^, q (x) q, rows
  Status *status;
  Opts opts;
  PersistLayout lay[kPersistMax];
  RomArgs<T> sd[kPersistMax];
};
static_assert(sizeof(PersistArgs<double>) <= 4096, "persistent kernel arguments exceed 4 KB");

template <typename T>
hipError_t launch_rom_persist(const PersistArgs<T> &P, int batch, size_t lds, hipStream_t s);

}  // namespace osam
