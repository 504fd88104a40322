// Internal declarations of the fcw library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "cube.h"
#include "fcw.h"

namespace fcw {

constexpr int kMaxP = 8;
constexpr int kMaxNl = 256;  // largest n_loc built (3-D elasticity p=3: 192)

// Cell classes as exported (FCW_ARR_CELL_CLASS).
constexpr int8_t kClsOut = 0, kClsUncut = 1, kClsCut = 2;
// Per-cell step info: >= 0 is the cut-cell index; negative codes below.
constexpr int32_t kInfoOut = -1, kInfoUncut = -2;

// 1-D tables of the reference element, FP64, device resident.
struct RefTables {
  double gll_x[kMaxP + 1], gll_w[kMaxP + 1];  // GLL nodes / weights (p+1 points)
  double gl_x[kMaxP + 1], gl_w[kMaxP + 1];    // GL nodes / weights (p+1 points)
};

// Point-source data prepared on the device for one step call.
struct SourceDev {
  int32_t cell[3];  // cell coordinates containing the source
  int32_t pad;
  double f0;
  double b[kMaxNl];  // rho * amp * dir_c * N_a(x_s), local (comp-major) order
};

// An observer point prepared on the device: the cell holding it and the values N_a(x_r)
// of that cell's shape functions (local node order, x fastest).
struct RecDev {
  int32_t cell[3];
  int32_t pad;
  double w[kMaxNl];
};

struct Ctx {
  // problem
  int dim = 2, ncomp = 1, p = 1, depth = 0, precision = FCW_FP64;
  int ncells[3] = {1, 1, 1};
  int npts[3] = {1, 1, 1};  // nodes per direction
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, h = 1;
  double alpha = 1e-12, rho = 1, c = 1, E = 1, nu = 0.3;
  int64_t ncell_total = 0, nnodes = 0, ndof = 0;
  int n_s = 0, n_loc = 0;
  hipStream_t stream = nullptr;
  int state = 0;  // 1 assembled, 2 stabilised
  int tile_choice = 0;             // step tile configuration (autotuned)
  std::vector<double> tune_us;     // us per step of each configuration, last autotune
  bool poisoned = false;
  std::vector<double> void_c, void_r;  // host copies
  int nvoids = 0;
  CubeGeo cube{};  // rotated-cube domain (cube.on = 0: none)

  // counts
  int64_t n_cut_cand = 0;  // cut cells before reclassification
  int64_t n_cut = 0, n_uncut = 0, n_out = 0;
  double dt_crit = 0.0, min_margin = 0.0;

  // device buffers (FP64 setup data)
  double* d_void_c = nullptr;
  double* d_void_r = nullptr;
  int8_t* d_cls = nullptr;        // [ncells]
  int32_t* d_info = nullptr;      // [ncells]
  int32_t* d_cut_cells = nullptr; // [n_cut_cand] cell index per cut candidate
  int32_t* d_cut_vptr = nullptr;  // [n_cut_cand+1] offsets into d_cut_vidx
  int32_t* d_cut_vidx = nullptr;  // void indices meeting each cut candidate
  int32_t* d_all_void = nullptr;  // [n_cut_cand] tree found only void boxes
  RefTables* d_tab = nullptr;
  double* d_kref = nullptr;       // [n_loc^2]
  double* d_mfull = nullptr;      // [n_s^2]
  double* d_lref = nullptr;       // [n_s]
  double* d_kcut = nullptr;       // [n_cut_cand * n_loc^2]
  double* d_mcut = nullptr;       // [n_cut_cand * n_s^2]
  double* d_lumped = nullptr;     // [n_cut_cand * n_s]
  double* d_margin = nullptr;     // [n_cut_cand]
  int32_t* d_evs_fail = nullptr;  // [1]
  double* d_mass = nullptr;       // [nnodes]

  // per-step operands in the step precision
  void* d_invm = nullptr;     // [nnodes]
  void* d_kref_s = nullptr;   // [n_loc^2]
  void* d_kref_bf = nullptr;  // BF16 form: K_ref split into bf16 hi + lo, MFMA fragment order
  void* d_kcut_s = nullptr;   // [n_cut_cand * n_loc(n_loc+1)/2], packed upper, column-major
  double* d_invm64 = nullptr; // [nnodes] FP64 copy for the Lanczos iteration
  // analytic inverse mass of nodes whose cells are all uncut: invm = cm * invw_x * invw_y
  // (* invw_z), with the 1-D inverse assembled GLL weights invw; mflag has one bit per
  // node (rows of np[0] nodes, mflag_wpr words each) set where invm must be read instead
  double* d_invw = nullptr;       // [np0 + np1 + np2]
  uint32_t* d_mflag = nullptr;    // [np1 * np2][mflag_wpr]
  int mflag_wpr = 0;
  double cm = 0.0;

  // scratch
  void* d_ubuf = nullptr;
  size_t ubuf_bytes = 0;
  void* d_ycut = nullptr;     // [nrhs][n_cut_cand][n_loc] cut-cell products of a step
  size_t ycut_bytes = 0;
  SourceDev* d_src = nullptr;
  bool d_src_active = false;  // the sources of the current batched call are set
  int src_cap = 0;
  std::vector<fcw_source> src_staged;  // host copy of the sources d_src was computed from
  // volumetric (Gaussian) sources of the staged set: load entries (DOF, value) of
  // right-hand side r in [g_off[r], g_off[r+1]) (host and device copies)
  bool g_active = false;
  std::vector<int32_t> g_off;
  int32_t* d_goff = nullptr;
  int64_t* d_gdof = nullptr;
  double* d_gval = nullptr;
  size_t g_cap = 0;
  std::vector<int8_t> h_cls;  // host copy of the cell classes (volumetric sources)
  // receivers of the current run (FCW_MAX_RECEIVERS) and reduction buffers of the
  // growth checks and energies: [64 rhs][3][kRedBlocks] partial sums and [64][3] totals
  RecDev* d_rec = nullptr;
  double* d_red = nullptr;
  double* h_red = nullptr;  // pinned copy of the totals
  // work list of the persistent step kernel (device + pinned staging)
  void* d_wl = nullptr;
  void* h_wl = nullptr;
  size_t wl_bytes = 0;
  hipEvent_t wl_event = nullptr;
  // cached graph of a batched run: valid for the same launch sequence
  hipGraphExec_t graph_exec = nullptr;
  const void* graph_fn = nullptr;
  int graph_nitems = 0, graph_nsteps = 0, graph_nprob = 0, graph_ncutprob = 0;
  int64_t graph_ncut = 0;
  void* graph_wl = nullptr;
  int64_t footprint = 0;
  bool skip_cut = false;  // step calls launch the main kernel only (kernel timing)
  // IMEX (implicit DOFs = nodes of cut cells): Cholesky factors of S = M^cc + beta dt^2
  // K^cc and of M^cc, each with its transpose, for the step size imex_dt
  int64_t imex_nc = -1;            // implicit DOFs (-1: not prepared)
  int64_t imex_ncn = 0;            // implicit nodes
  double imex_dt = 0.0;
  int64_t* d_imex_dofs = nullptr;  // [imex_nc] global DOF of each implicit DOF
  double* d_imex_s = nullptr;      // set-up only: [3][n_b^2] L of S (row-major, lower), L^T, S^{-1}
  double* d_imex_m = nullptr;      // set-up only: the same for M^cc
  double* d_imex_sp = nullptr;     // S^{-1} as its upper 32 x 32 tiles, block by block
  double* d_imex_mp = nullptr;     // (M^cc)^{-1}, the same
  int32_t* d_imex_kptr = nullptr;  // [imex_nc+1] the implicit rows of K, compressed: offsets,
  int32_t* d_imex_kcol = nullptr;  // columns (-(implicit index + 1) for implicit DOFs)
  double* d_imex_kval = nullptr;   // and values
  // the implicit set splits into blocks (connected through shared cells) that S and M^cc
  // never couple; b and x of the tiled products run in block order
  int32_t imex_nblk = 0;           // blocks
  int64_t imex_largest = 0;        // DOFs of the largest block
  int64_t imex_ntiles = 0;         // packed tiles over all blocks
  int64_t imex_part = 0;           // tile-product partials per right-hand side
  int32_t* d_imex_cpos = nullptr;     // [imex_nc] block-order position of each implicit DOF
  int32_t* d_imex_members = nullptr;  // [imex_nc] implicit DOF at each block-order position
  int32_t* d_imex_pblk = nullptr;     // [imex_nc] block of each block-order position
  void* d_imex_blocks = nullptr;      // [imex_nblk] block descriptors
  void* d_imex_tiles = nullptr;       // [imex_ntiles] descriptor of each packed tile
  double* d_imex_work = nullptr;   // per-call work vectors
  size_t imex_work_bytes = 0;
  int32_t* d_imex_flag = nullptr;  // [1] non-positive pivot seen

  size_t state_bytes() const { return precision == FCW_FP64 ? 8 : 4; }
};

// The analytic inverse mass of a node all of whose cells are uncut (the assembled GLL
// diagonal factorises over the directions); setup and step kernels use this one
// expression so the stored and the computed values agree bit for bit.
template <typename T>
__host__ __device__ inline T analytic_invm(double cm, double iwx, double iwy, double iwz) {
  return (T)(((cm * iwx) * iwy) * iwz);
}

// error reporting (thread-local message)
void set_error(const char* fmt, ...);
void clear_error();
fcw_status hip_fail(hipError_t e, const char* what);

#define FCW_HIP(call)                                      \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return ::fcw::hip_fail(e_, #call); \
  } while (0)

// ---- launchers implemented in the .hip sources ----
// setup.hip
fcw_status setup_reference(Ctx& c);
fcw_status setup_classify(Ctx& c);
fcw_status setup_integrate(Ctx& c);
fcw_status setup_reclassify(Ctx& c);
fcw_status setup_stabilize(Ctx& c, double eps, double f_lambda);
fcw_status setup_mass_and_pack(Ctx& c);
// Load vectors of nrhs point sources into c.d_src (allocated on first use when null).
// remember: skip the work when the sources equal the last staged ones, and record them.
constexpr int kMaxSrc = 64;
fcw_status prepare_sources(Ctx& c, int nrhs, const fcw_source* src, bool remember = true);
// exclusive scan of n int32 on the context's stream; the total goes to *total_host (syncs)
fcw_status exclusive_scan(Ctx& c, const int32_t* in, int32_t* out, int64_t n,
                          int32_t* total_host);
// imex.hip: semi-explicit scheme (implicit DOFs = nodes of cut cells)
void imex_free(Ctx& c);
fcw_status imex_prepare(Ctx& c, double dt);
// consistent: central differences with the consistent cut-DOF mass instead (v_c, a_c unused)
fcw_status imex_run(Ctx& c, int nrhs, double* u, double* d, double* v_c, double* a_c, double t0,
                    double dt, int nsteps, int start, bool consistent);
// api.hip: argument checks of a step call (no allocation, nothing enqueued)
fcw_status check_step_call(const fcw_ctx* c, int32_t nrhs, const void* u, const void* d,
                           const fcw_source* src, double dt, int32_t nsteps);
// cutcell.hip: cut-cell products y = K_e u_e, once per cut cell and step
fcw_status ensure_ycut(Ctx& c, int nrhs);
size_t cutprob_size(int fp64);
int64_t cutprob_fill(const Ctx& c, void* out, const void* ua, const void* ub, int nrhs,
                     int nsteps, int64_t blk0);
fcw_status launch_cut(const Ctx& kind, hipStream_t s, const void* probs, int nprob,
                      const void* one, int64_t nblk, int j);
fcw_status launch_cut_products(Ctx& c, int nrhs, const void* u);
// step.hip
bool step_supported(const Ctx& c);
fcw_status launch_apply(Ctx& c, int nrhs, const void* u, void* r);
int tile_candidates(const Ctx& c, int i, int tile[3], std::string* name = nullptr);
// Work queued after each step of a call (observer traces): fn(arg, stream, j) after step j
// of the call has been queued, and once with j = -1 before the first step.
struct StepHook {
  fcw_status (*fn)(void* arg, hipStream_t s, int j);
  void* arg;
};
fcw_status run_steps(Ctx& c, int choice, int nrhs, void* u, void* d, void* scratch, double t0,
                     double dt, int nsteps, int start, const StepHook* hook = nullptr);
// one batched group of 2-D problems (see fcw_run)
struct GroupMember {
  Ctx* ctx;
  int nrhs;
  void *u, *d, *scratch;
  double t0, dt;
  int nsteps, start;
};
fcw_status run_group(Ctx& owner, const std::vector<GroupMember>& m, bool graph,
                     const StepHook* hook = nullptr);
// observe.hip: receivers, traces, growth checks and energies of fcw_run
fcw_status prepare_receivers(Ctx& c, int nrec, const double* x);  // setup.hip; into c.d_rec
struct TraceTarget {
  Ctx* ctx;
  const void* u;     // caller state of the call (the final state lands here)
  const void* ub;    // its ping-pong partner
  int nrhs, nsteps;  // of this call (fixes which buffer holds the state after step j)
  int nrec;
  double* traces;    // [nrhs][tlen][nrec][ncomp]
  int64_t tlen, k0;  // rows per right-hand side; row of the call's initial state
};
fcw_status launch_traces(hipStream_t s, const TraceTarget* t, int n, int j);
// volumetric loads: before step k of a call (hook call j = k - 1) the increment d of each
// target takes dt^2 M^{-1} f_t(t_k) b (dt^2 / 2 on a start call's first step)
struct LoadTarget {
  Ctx* ctx;
  void* d;
  int nrhs, nsteps, start;
  double t0, dt;
};
fcw_status launch_gauss_loads(hipStream_t s, const LoadTarget* t, int n, int j);
// per right-hand side sums over the DOFs into c.h_red[rhs * 3 + q] (synchronises):
// energy = false: q = 0 sum d_i^2;  energy = true: q = 0 sum m_i d_i^2, q = 1 u.Ku,
// q = 2 d.Ku, with Ku in `r` (m_i the lumped mass)
fcw_status state_sums(Ctx& c, hipStream_t s, int nrhs, const void* u, const void* d,
                      const void* r, bool energy);
bool groupable_2d(const Ctx& a, const Ctx& b);
// one batched group of 3-D problems of one kind (dim 3, same p, ncomp and precision)
fcw_status run_group3d(Ctx& owner, const std::vector<GroupMember>& m, bool graph,
                       const StepHook* hook = nullptr);
bool groupable_3d(const Ctx& a, const Ctx& b);
fcw_status launch_apply_scaled64(Ctx& c, const double* v, double* w);
// lanczos.hip
fcw_status lanczos_lambda_max(Ctx& c, int max_iter, double rtol, double* lmax);
// the iteration on any FP64 operator w = apply(arg, v) of length n (already scaled by
// M^{-1/2} on both sides); the start vector is nonzero where mask[i % nmask] > 0, n =
// nmask * ncomp
struct LanczosOp {
  hipStream_t stream;
  int64_t n;
  const double* mask;
  int64_t nmask;
  int ncomp;
  fcw_status (*apply)(void* arg, const double* v, double* w);
  void* arg;
};
fcw_status lanczos_run(const LanczosOp& op, int max_iter, double rtol, double* lmax);

// small helpers usable on host and device
__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

}  // namespace fcw

struct fcw_ctx : public fcw::Ctx {};
