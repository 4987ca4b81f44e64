// Host-side objects of libosam (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/osam.h"
#include "osam_device.hpp"

namespace osam {

// OpInf data in float64 on the host (column-major as installed), kept for
// read-back, initial states and re-wiring.
struct OpinfHost {
  int r = 0, rs = 0;
  bool quadratic = false;
  std::vector<double> Phi, PhiS, A, H, B, c;   // Phi [nfree x r], PhiS [nsch x rs], A [r x r], ...
  std::vector<double> C3;                      // cubic operator [r x r(r+1)(r+2)/6] (COpInf) or empty
};

// Buffers of the window engine (window.hip), per subdomain.
struct WinBufs {
  void *wu[2] = {}, *wv[2] = {}, *wa[2] = {};   // FOM: end of the window by iteration parity
  void *tu[2] = {}, *tv[2] = {}, *ta[2] = {};   // FOM: inner sub-steps
  void *cr = nullptr, *cp = nullptr, *cq = nullptr;   // FOM: CG vectors
  void *wq[2] = {}, *wqd[2] = {}, *wqdd[2] = {}, *tq[2] = {}, *tqd[2] = {}, *tqdd[2] = {};   // OpInf
  void *sbuf = nullptr, *kbuf = nullptr, *Minv = nullptr, *C3 = nullptr;
  void *traj[2][2] = {};           // per own Schwarz face: the source's trajectory by iteration parity
  std::vector<std::pair<int, void *>> exp_rows;   // OpInf source: (2 dst + face, [r][3 npl] rows)
  int *iters = nullptr;            // [batch] CG / Newton iteration statistics
};

// Pointwise projection of one z-face: ELL rows over the face's npl nodes.
struct FaceProj {
  int src = -1;          // source subdomain
  int width = 0;
  std::vector<int> idx;  // [npl][width] source node ids
  std::vector<double> wt;
  int src_layer = 0;     // source-local node layer that coincides with the face
};

struct Subdomain {
  osam_subdomain_desc desc{};
  int nx = 0, ny = 0, nzs = 0, npl = 0;
  long long nnodes = 0, cs = 0, is = 0, nfree_nodes = 0, nsch_nodes = 0, face_off_hi = 0;
  int face_type[2] = {0, 0};    // geometry: clamped or Schwarz
  FaceProj proj[2];
  // FOM buffers
  void *u[3] = {}, *v[2] = {}, *a[2] = {};
  void *coef = nullptr;
  double cb[27];               // the interior block's distinct values (kernel arguments)
  std::vector<std::vector<double>> gh0;   // OpInf: g^ at t_0 per instance (from the initial condition)
  int *bnd_cols = nullptr;          // boundary columns grouped by cross-section case
  int n_int = 0, n_bnd = 0;
  int nbg = 0, bg_start[8] = {}, bg_n[8] = {};   // the case groups of bnd_cols
  bool fe_xs = true;               // interior waves share x-neighbours across lanes
  double *partials = nullptr;        // two halves of [batch][max_nblocks][2], by sweep parity
  double *partials_of(int par, int batch) const {
    return partials + (size_t)par * batch * max_nblocks * 2;
  }
  // FE launch shape: fe_block 64/128/256 = column kernel; 1024 = layer-staged kernel for the
  // interior (fe_chunks workgroups of fe_kc layers) plus the column kernel (64 threads, one
  // layer per thread) for the boundary columns; fe_nblocks = workgroup partials per instance
  int fe_block = 256, fe_kc = 8, fe_chunks = 1, fe_nblocks = 0, max_nblocks = 0;
  // FE part of a fused sweep: 512-thread workgroups of the column kernel, fz_kc layers per thread
  int fz_kc = 1, fz_chunks = 1, fz_nblocks = 0;
  // OpInf
  bool rom = false;
  int r = 0, rs = 0;
  OpinfHost oh;
  void *d_A = nullptr, *d_H = nullptr, *d_B = nullptr, *d_c = nullptr;   // row-major
  // batched OpInf path: f0 = A q + H (q (x) q) + c once per step on the matrix
  // cores, g^ of FOM-fed faces split over the face DOFs (FP32 contexts)
  int rom_path = 0;                // 0 automatic, 1 fused, 2 batched
  bool pre = false;                // batched path wired
  float *pre_fa = nullptr;         // A in MFMA fragment order (FP32)
  void *pre_fh = nullptr;          // H in MFMA fragment order (FP32 or BF16)
  int *pre_blocks = nullptr;       // H K block -> row i of the triangle | first column j0 << 16
  float *pre_f0 = nullptr;         // [ks][batch][r]
  double *pre_g = nullptr;         // [gs][batch][rs]
  int pre_prec = 0, pre_nkba = 0, pre_nkbh = 0, pre_nrt = 0, pre_ks = 1, pre_gs = 1, pre_ni = 1;
  void *d_Phi = nullptr;           // [r][nfree] column-major
  void *q[2] = {}, *qd[2] = {}, *qdd[2] = {};
  void *qpred = nullptr;           // [batch][r]: Newmark predictor of the latest state (next step's q(t_k))
  void *face_phis[2] = {};         // [rs][3 npl] Phi_S block per Schwarz face
  void *face_tm[2] = {};           // [rs][r_src] for ROM sources
  void *sface[2][3] = {};          // OpInf: pushed face values by role, [batch][3 npl] (FOM source)
  std::vector<std::vector<double>> piphi_h;  // host copy per export
  std::vector<void *> piphi_d;               // device copy per export ([r][3 npl], column-major)
  std::vector<void *> piphi_rm;              // row-major device copy per export ([3 npl][r rounded up to 4])
  // records
  osam_record rec{};
  // window engine
  int n_sub = 1;
  WinBufs win;
};

struct Ctx {
  int device = 0;
  int prec = OSAM_FP64;
  int batch = 1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<std::unique_ptr<Subdomain>> sds;
  Status *d_status = nullptr;       // status every kernel of the next round reads
  Status *d_status_alt = nullptr;   // written by that round's decider; swapped after each round
  double *rom_sums = nullptr;       // [2][batch][kMaxSd][2]: OpInf sums of fused sweeps by parity
  Status *h_status = nullptr;   // pinned mirror
  std::vector<void *> allocs;   // hipMalloc'ed arena blocks (freed at destroy)
  struct Chunk {
    char *ptr;
    size_t bytes;
    bool free;
  };
  std::vector<Chunk> chunks;    // carved pieces of the blocks
  char *arena_cur = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  void *arena_alloc(size_t bytes, int32_t *st);
  std::vector<char> initialized;
  bool coupled = false;
  bool wired = false;
  std::string err;
  double avg_iters = 3.0;
  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<int, int>>> ev_used;   // (sd, (start idx, stop idx))
  size_t ev_next = 0;
  // scratch
  double *d_scratch = nullptr;
  size_t scratch_n = 0;

  int32_t fail(int32_t code, const std::string &msg);
  void dfree(void *p);
  size_t esize() const;
  void *alloc_t(size_t n, int32_t *st);
  int32_t upload(void *dst, const double *src, size_t n);
  int32_t download(double *dst, const void *src, size_t n);
  double *scratch(size_t n, int32_t *st);

  bool choose_fe_launch(Subdomain &s, int block, int kc);
  int32_t couple();
  int32_t wire();
  int32_t setup_pre(Subdomain &d);
  int32_t set_initial(int inst, const double *u0, const double *v0);
  int32_t init_pending();
  int32_t get_state(int sd, int inst, double *u, double *v, double *a);
  int32_t install_opinf(int sd, const OpinfHost &oh);
  int32_t install_opinf_device(int sd, const OpinfHost &oh, const double *phi_dev);
  int32_t phi_layer_rows(Subdomain &s, int layer, std::vector<double> &out);
  int32_t sync_status();
  int32_t run(int64_t n_steps, const osam_schwarz_opts &o, osam_instance_info *info, bool host_sweeps = false);
  int32_t launch_round(const Opts &o);
  // graph mode: rounds replayed from a captured HIP graph, the FOM and OpInf
  // kernels of a round on two streams, the decision in the finisher kernel
  int graph_rounds = 0, graph_streams = 1;
  hipStream_t aux = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  int32_t launch_round_concurrent(const Opts &o);
  // fused sweeps: every subdomain's step in one launch (sweep_kernels.hip)
  bool fuse = false;
  int fuse_kc = 1;
  std::string fusion_unsupported() const;
  void fuse_layout(Subdomain &s);
  int32_t launch_round_fused(const Opts &o, long long r = 0, long long n = 0);
  FinishArgs fused_finish_args(int par);
  int32_t autotune(int64_t n, const osam_schwarz_opts &op, osam_tuning *out);
  int32_t apply_tuning(const osam_tuning &t);
  hipEvent_t next_event();
  int32_t rom_start(int i, int inst, const std::vector<double> &q, const std::vector<double> &qd);
  int32_t run_adjoint(int64_t n, int64_t K, const osam_misfit &m, double *J, const osam_grads &g);
  int32_t launch_fe_sd(int sdi, const Opts &o, int mode, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                       hipStream_t st = nullptr);
  int32_t launch_rom_sd(int sdi, const Opts &o, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                        hipStream_t st = nullptr, bool defer = false);
  int32_t learn(int sd, const osam_opinf_desc &d);
  // window engine (window.hip): sub-stepped or implicit subdomains, or on request
  int engine = 0;                  // 0 automatic, 1 window engine for every run, 2 persistent OpInf
  bool win_ready = false;
  std::vector<void *> win_allocs;
  double *win_sums = nullptr;      // [batch][nsd][2]
  int win_iters_hint = 0;          // iterations the last controller step took (read-backs start there)
  bool window_mode() const;
  int32_t window_setup();
  int32_t run_window(int64_t n_steps, const Opts &o, osam_instance_info *info);
  int32_t run_persist(int64_t n_steps, const Opts &o, osam_instance_info *info);
  std::string persist_unsupported(const Opts &o) const;
  int32_t instance_info(osam_instance_info *info);
  // device address of the static scratch array on this context's device (noalloc.hip)
  void *static_scratch = nullptr;
};

int32_t static_scratch_address(int device, void **out);

}  // namespace osam
