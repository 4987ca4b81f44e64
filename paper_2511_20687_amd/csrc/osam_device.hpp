// Device-side data structures shared by the libosam kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osam {

constexpr int kMaxSd = 8;
// largest cross-section (nodes per layer) of the layer-staged FE variant: three
// layers of three FP32 components in 160 KB of LDS
constexpr int kFeLdsMaxNodes = 160 * 1024 / (9 * 4) - 16;

// Per-instance controller state, in device memory.  Only the kernels modify it
// while a run is in flight; the host reads it back between chunks of work.
struct Status {
  long long step;          // accepted controller steps
  long long target;        // the instance stops when step == target
  int iter;                // Schwarz iterations done in the current step
  int flags;               // kFinished | kNonfinite
  int last_iters, last_conv;
  long long total_iters, unconverged;
  int max_iters, pad0;
  double abs2, den2;       // last evaluated criterion
  double sd_abs2[kMaxSd];  // this iteration's per-subdomain sums
  double sd_den2[kMaxSd];
};
// What a step body needs of the status it starts from.
struct StepState {
  long long step;
  int iter, flags;
};
constexpr int kFinished = 1;
constexpr int kNonfinite = 2;
constexpr int kNeedInit = 4;

struct Opts {
  double tol_abs2, tol_rel2;
  int min_iter, max_iter, guess, nsd;
  int additive;   // 1: every face reads the previous iteration (the first: `guess`)
};

// Convergence decision of Eq. conv_criterion after the last subdomain of a
// Schwarz sweep (executed by a single thread).
__device__ inline void decide(Status &st, int sd, const Opts &o) {
  if (sd != o.nsd - 1) return;
  const int n = st.iter + 1;
  double a = 0.0, d = 0.0;
#pragma unroll
  for (int i = 0; i < kMaxSd; ++i)
    if (i < o.nsd) {
      a += st.sd_abs2[i];
      d += st.sd_den2[i];
    }
  const bool tested = n >= o.min_iter;
  if (!isfinite(d) || (tested && !isfinite(a))) {
    st.abs2 = a;
    st.den2 = d;
    st.flags |= kFinished | kNonfinite;
    return;
  }
  bool conv = false;
  if (tested) {
    conv = (a < o.tol_abs2) || (a < o.tol_rel2 * d);
    st.abs2 = a;
    st.den2 = d;
  }
  if (conv || n >= o.max_iter) {
    st.step += 1;
    st.last_iters = n;
    st.last_conv = conv ? 1 : 0;
    st.total_iters += n;
    if (n > st.max_iters) st.max_iters = n;
    if (!conv) st.unconverged += 1;
    st.iter = 0;
    if (st.step >= st.target) st.flags |= kFinished;
  } else {
    st.iter = n;
  }
}

// End of a Schwarz sweep.  Every FOM step kernel leaves one pair of FP64
// partial sums per workgroup, every OpInf kernel that does not end the sweep
// leaves its two sums in the output status; the decider (one wave) reduces the
// FOM partials in a fixed order and takes the decision.  Running it after the
// sweep, instead of in a "last workgroup" of each FOM kernel, avoids
// device-scope fences and atomics, which serialise across the XCDs' separate L2
// caches.  The status is double-buffered per round: every kernel of a round
// reads `in`, the decider writes the whole of `out` (also for finished
// instances), so a kernel with several workgroups can decide without racing
// the status reads of its other workgroups.
struct FinishArgs {
  int nfom, nrom;
  int sd[kMaxSd];
  int nblocks[kMaxSd];
  const double *part[kMaxSd];   // [batch][nblocks][2]
  int rom_sd[kMaxSd];           // OpInf subdomains whose sums are in `out` already
  const double *rom_sums;       // or, when not null, in this [batch][kMaxSd][2] array
};

// Sum over the 64 lanes of a wave (every lane active), returned to every lane.
// An inclusive scan with DPP row shifts (1, 2, 4, 8 within rows of 16) and the
// row broadcasts of lanes 15 and 31 leaves the total in lane 63; the additions
// stay in the vector ALU (no LDS permutes), six dependent steps in all.
template <int CTRL, int ROW, int BANK>
__device__ __forceinline__ float dpp_src(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROW, BANK, true));
}
template <int CTRL, int ROW, int BANK>
__device__ __forceinline__ double dpp_src(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, ROW, BANK, true);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROW, BANK, true);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ float lane63(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 63));
}
__device__ __forceinline__ double lane63(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), 63);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T wave_total(T x) {
  x += dpp_src<0x111, 0xf, 0xf>(x);   // row_shr:1
  x += dpp_src<0x112, 0xf, 0xf>(x);   // row_shr:2
  x += dpp_src<0x114, 0xf, 0xe>(x);   // row_shr:4, lanes 4..15 of each row
  x += dpp_src<0x118, 0xf, 0xc>(x);   // row_shr:8, lanes 8..15 of each row
  x += dpp_src<0x142, 0xa, 0xf>(x);   // row_bcast:15 into rows 1 and 3
  x += dpp_src<0x143, 0xc, 0xf>(x);   // row_bcast:31 into rows 2 and 3
  return lane63(x);
}

__device__ __forceinline__ double wave_sum64(double x) { return wave_total(x); }

// The value held by lane l - 1 (wave_shr:1) or lane l + 1 (wave_shl:1), moved by
// the vector ALU rather than an LDS permute.  Lane 0 (lane_prev) and lane 63
// (lane_next) have no source and receive 0.  Every lane must be active.
template <typename T>
__device__ __forceinline__ T lane_prev(T x) { return dpp_src<0x138, 0xf, 0xf>(x); }
template <typename T>
__device__ __forceinline__ T lane_next(T x) { return dpp_src<0x130, 0xf, 0xf>(x); }

// Sums of FOM subdomain k's partials, computed by one wave (lane 0 holds them).
// Loads are issued in batches of U per lane before any is consumed.
template <int U>
__device__ inline double2 fom_sums(const FinishArgs &F, int k, int b, int lane) {
  const int nb = F.nblocks[k];
  const double2 *pp = reinterpret_cast<const double2 *>(F.part[k]) + (long long)b * nb;
  double sa = 0.0, sd = 0.0;
  for (int base = 0; base < nb; base += 64 * U) {
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = pp[min(base + u * 64 + lane, nb - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (base + u * 64 + lane < nb) {
        sa += v[u].x;
        sd += v[u].y;
      }
  }
  return make_double2(wave_sum64(sa), wave_sum64(sd));
}

// The sums of a sweep gathered into the status s it started from, and the decision of
// Eq. conv_criterion taken: by one whole wave, every lane ends with the same s.
// rom_src: the status holding the OpInf subdomains' sums (when F.rom_sums is null).
// own_sd >= 0 with own_abs2/own_den2: the calling OpInf kernel's own sums.
// pre (optional): the FOM sums already reduced by the caller, [abs2, den2] per FOM subdomain.
// U: partial-sum loads in flight per lane (registers: 4 U).
template <int U>
__device__ inline void gather_decide(Status &s, const Status *rom_src, const FinishArgs &F, const Opts &o, int b,
                                     int own_sd, double own_abs2, double own_den2, const double *pre) {
  const int lane = threadIdx.x & 63;
  if (s.flags & kFinished) return;
  // per-subdomain sums, written with compile-time indices only (no private-memory indexing)
  for (int k = 0; k < F.nfom; ++k) {
    const double2 t = pre ? make_double2(pre[2 * k], pre[2 * k + 1]) : fom_sums<U>(F, k, b, lane);
    const int j = F.sd[k];
#pragma unroll
    for (int i = 0; i < kMaxSd; ++i)
      if (i == j) {
        s.sd_abs2[i] = t.x;
        s.sd_den2[i] = t.y;
      }
  }
  for (int k = 0; k < F.nrom; ++k) {
    const int j = F.rom_sd[k];
    double ta, td;
    if (F.rom_sums) {
      const double2 v = reinterpret_cast<const double2 *>(F.rom_sums)[(long long)b * kMaxSd + j];
      ta = v.x;
      td = v.y;
    } else {
      ta = rom_src[b].sd_abs2[j];
      td = rom_src[b].sd_den2[j];
    }
#pragma unroll
    for (int i = 0; i < kMaxSd; ++i)
      if (i == j) {
        s.sd_abs2[i] = ta;
        s.sd_den2[i] = td;
      }
  }
#pragma unroll
  for (int i = 0; i < kMaxSd; ++i)
    if (i == own_sd) {
      s.sd_abs2[i] = own_abs2;
      s.sd_den2[i] = own_den2;
    }
  decide(s, o.nsd - 1, o);
}

// The decider: called by one whole wave (lane 0 writes `out`).  Arguments as gather_decide.
template <int U = 16>
__device__ inline void finish_sweep(const Status *in, Status *out, const FinishArgs &F, const Opts &o, int b,
                                    int own_sd = -1, double own_abs2 = 0.0, double own_den2 = 0.0,
                                    const double *pre = nullptr) {
  Status s = in[b];
  gather_decide<U>(s, out, F, o, b, own_sd, own_abs2, own_den2, pre);
  if ((threadIdx.x & 63) == 0) out[b] = s;
}

// Faces and pushes.  All subdomains share one global grid, so a Schwarz face of
// subdomain i coincides with a node layer of its source j (the pointwise
// projection is an injection).  Every source writes the displacement it will
// have at the next controller step (its Newmark predictor) straight into the
// face values of its destinations, into the buffer role of the next step;
// buffer roles rotate with the instance's step count (U0 = role s%3, P =
// (s+1)%3, P2 = (s+2)%3).  A destination then finds on its face:
//   role U0 : the source at t_{k-1}  (HOLD guess, Sec. 4.1)
//   role P  : the source at t_k      (newest iterate; equal across iterations
//                                     for the explicit scheme)
enum FaceType : int { kFaceClamped = 0, kFaceFom = 1, kFaceStage = 2 };

template <typename T>
struct PushDev {
  int layer;               // source-local node layer that feeds the face
  int pad;
  T *role[3];              // destination face-value buffers by role, at the face start
  long long cs, is;        // destination component / instance strides
};

// Arguments of the FE explicit-step kernel (one subdomain, all instances).
template <typename T>
struct FeArgs {
  int nx, ny, nzs, npl;
  long long cs, is;        // component stride, instance stride (elements)
  T *u[3];                 // rotating displacement buffers (U0, P, P2 by step parity)
  T *v[2];
  T *a[2];
  const T *coef;           // [9 cases][26 offsets][3][3]: -K_d / m
  int skip_rows;           // components held on the lateral faces (zero rows of the boundary cases)
  T cb[27];                // the interior block's 27 distinct values (box_index)
  T dt, half_dt, half_dt2;
  int face_src[2];         // source subdomain of the low / high face, -1 if clamped
  int npush;
  PushDev<T> push[2];
  Status *status;
  int sd;
  Opts opts;
  double *partials;        // [batch][part_stride][2], this launch's workgroups from part_off
  int part_stride, part_off;
  int kc, n_chunks, n_int, n_bnd, nblocks;   // nblocks: workgroups of the launch (waves packed, see fe_body)
  const int *bnd_cols;     // boundary columns (ids in the layer), grouped by cross-section case
  int nbg;                 // case groups of the boundary list (at most 8)
  int xs;                  // 1: interior waves share x-neighbours across lanes (62 nodes per wave)
  int bnd_l;               // layer chunks per boundary wave (1..4): a wave of a group of
                           // n < 64 columns holds min(64 / n, bnd_l) chunks
  int bg_start[8], bg_n[8];   // first entry and number of columns of each group
  // records: [batch][ncols][len]
  T *rec_u, *rec_a, *rec_s;
  long long rec_every, rec_ncols;
  long long nfree_nodes, nsch_nodes, face_off_hi;  // Schwarz nodes of low face come first
};

template <typename T>
struct RomFaceIn {
  int type;                // kFaceFom: pushed values in sface; 3: ROM source (tm q_src)
  int src_sd;
  int n;                   // Schwarz DOFs of this face (3*npl)
  int src_r;
  const T *sface[3];       // [batch][n] face values by role (kFaceFom)
  const T *phis;           // [rs][n] column-major block of Phi_S for this face
  const T *tm;             // [rs][src_r] row-major: Phi_S,face^T Pi Phi_src (ROM source)
  T *src_q[2];             // source reduced displacement buffers [batch][src_r]
  // ROM source: its displacement at t_k is its explicit predictor, formed from
  // its accepted state at t_{k-1} (src_qd, src_qdd) where it is not read back
  // from what the source wrote in this sweep; pred = 1 always (fused sweeps)
  int pred;
  T src_dt, src_half_dt2;
  const T *src_qd[2], *src_qdd[2];
};

// Explicit Newmark predictor q + dt q' + dt^2/2 q'' in one fixed rounding order,
// shared by an OpInf step and the faces that read its displacement.
template <typename T>
__device__ __forceinline__ T newmark_pred(T q, T qd, T qdd, T dt, T half_dt2) {
  return fma(half_dt2, qdd, fma(dt, qd, q));
}

template <typename T>
struct RomExport {
  T *role[3];              // destination face values by role, at the face start
  long long cs, is;        // destination component / instance strides
  int npl;
  const T *prow;           // [3 npl][r4] row-major rows of Pi Phi for the face, zero-padded
  int r4;                  // row stride: r rounded up to a multiple of 4 (16-byte rows)
};

template <typename T>
struct RomArgs {
  int r, rs, r2;           // r2 = r(r+1)/2 when quadratic else 0
  const T *A;              // [r][r] row-major
  const T *H;              // [r][r2] row-major or null
  const T *B;              // [r][rs] row-major or null
  const T *c;              // [r] or null
  T *q[2], *qd[2], *qdd[2];  // [batch][r] by step parity
  T *qpred;                // [batch][r]: Newmark predictor of the latest state
  T dt, half_dt, half_dt2;
  int nfaces, nexp;
  RomFaceIn<T> fin[2];
  RomExport<T> ex[2];
  Status *status;          // this round's input status
  Status *status_out;      // written by the decider of the round
  int sd;
  Opts opts;
  FinishArgs finish;       // used when this is the last subdomain of the sweep
  T *rec_q;
  long long rec_every, rec_ncols;
  // batched path: f0 = A q + H (q (x) q) + c and g^ of the FOM-fed faces come
  // precomputed as partial sums (A, H, c and FOM faces are then absent above)
  int defer;               // 1: never decide, leave the sums for the finisher kernel
  double *sums_out;        // deferred sums: [batch][kMaxSd][2] when not null, else status_out
  const T *f0part;         // [f0_ks][batch][r] or null
  int f0_ks;
  const double *gpart;     // [g_gs][batch][rs] or null
  int g_gs;
  long long f0_stride, g_stride;   // batch * r, batch * rs
};

// Batched OpInf parts (FP32 contexts): f0 on the matrix cores, g^ of FOM faces.
struct RomPreArgs {
  int r, rs, r2, batch;
  int prec;                // 0: FP32 operands, 1: BF16 operands (FP32 accumulation)
  int nkba, nkbh;          // K blocks of A (FP32, 4 wide) and of H (4 wide FP32 / 16 wide BF16)
  int nrt, ks, nit, ni;    // row tiles of 16, K splits, instance tiles of 16, tiles per workgroup
  const float *frag_a;     // A in MFMA fragment order (FP32)
  const void *frag_h;      // H in MFMA fragment order (FP32 or BF16), null when linear
  const int *blocks;       // H K block -> row i of the triangle | first column j0 << 16
  const float *c;
  const float *qpred;      // [batch][r]: the predictor q(t_k) of each instance starting a step
  float *f0part;           // [ks][batch][r]
  int nface, gs;           // FOM-fed faces, DOF splits
  long long fn[2];
  int fsrc[2];
  const float *phis[2];
  const float *sface[2][3];
  double *gpart;           // [gs][batch][rs]
  const Status *status;
  int sd;
  Opts opts;
};

hipError_t launch_rom_pre(const RomPreArgs &P, hipStream_t s);
hipError_t launch_rom_pre_multi(const RomPreArgs *P, int n, hipStream_t s);

// One Schwarz sweep in a single launch: the subdomain in slot i owns the next
// nblk[i] workgroups of the grid (x), instances along y; fe_idx / rom_idx pick
// its arguments (rom_idx < 0: a FOM step).  Kernel arguments stay below 4 KB.
constexpr int kSweepMax = 4, kSweepFe = 3, kSweepRom = 2;
//
// Folded decisions (graph mode): with fold = 1 the previous sweep had no finisher.  Wave 0
// of every workgroup then reduces that sweep's partial sums (`prev`, double-buffered by
// sweep parity) in the finisher's fixed order and takes the same decision on st_prev, so
// every workgroup starts from the same status, the one the finisher would have written;
// workgroup 0 of each instance stores it in st_cur for the sweep after.  The bodies read
// the status from the workgroup's copy and ignore their own status pointers.
template <typename T>
struct SweepArgs {
  int n;
  int nblk[kSweepMax], fe_idx[kSweepMax], rom_idx[kSweepMax];
  int fold;
  FinishArgs prev;
  const Status *st_prev;
  Status *st_cur;
  Opts opts;
  FeArgs<T> fe[kSweepFe];
  RomArgs<T> rom[kSweepRom];
};
static_assert(sizeof(SweepArgs<double>) <= 4096, "sweep kernel arguments exceed 4 KB");

}  // namespace osam
