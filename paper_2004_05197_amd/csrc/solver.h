// Solver instance shared by the single-cell and the batch C ABI.
//
// An instance owns one grid shape and ncell cells of that shape; every cell
// has lpc load slots, so the kernels see nslot = ncell * lpc independent
// "loads" (slot l = cell l / lpc, macro strain l % lpc).  A single-cell handle
// is an instance with ncell = 1.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/cellfft.h"
#include "kernels.h"

namespace cellfft {

template <typename T> struct Fields {
  T* x = nullptr;  // [nslot][d n] each
  T* r = nullptr;
  T* p = nullptr;
  T* q = nullptr;
  cpx<T>* S = nullptr;
  cpx<T>* R = nullptr;  // residual transformed along x, [nslot][d n / 2]
  cpx<T>* tw[3] = {nullptr, nullptr, nullptr};
  T* trig[3] = {nullptr, nullptr, nullptr};
  T* symtab = nullptr;   // 3D: [ncell][ny][nz][nx/2][6]
  T* symtabB = nullptr;  // 3D: [ncell][2][nz][6]
  float* edge = nullptr; // FP32 row-wave operator: edge rows [nslot][rw_edge_floats]
  T* med = nullptr;      // 2D: per-cell (lambda0, mu0) [ncell][2]
  std::vector<T> med_h;  // host copy of med (source of its upload)
  std::vector<double> sym_lam0, sym_mu0;  // reference medium of each cell's table
  bool ready = false;
};

}  // namespace cellfft

struct cell_s {
  int dev = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  cellfft::Geom g{};
  int d = 3, nv = 6;
  long long n = 0, lstride = 0;
  long long s_zs = 0, s_ls = 0;  // spectrum S: complex values per (component, z) plane, per slot
  int precision = CELL_FP64;
  double tol = 1e-10;
  int max_iter = 10000;
  int lpc = 6;    // load slots per cell
  int ncell = 1;  // cells of this grid
  int nslot = 6;  // ncell * lpc
  bool use_graphs = true;
  int dbg_negate_q = 0;     // CELLFFT_DEBUG_NEGATE_Q=1: the linear K-apply writes -K p
  int stag_window = 256;    // CELLFFT_STAG_WINDOW: CG iterations without progress that count as
                            // stagnation (0: never)
  cellfft::Sched sched{};  // kernel variants (autotuner)
  bool tuned = false;
  // material, per cell
  double* mat64 = nullptr;  // [ncell][n][2] (lambda, mu)
  float* mat32 = nullptr;
  double* E64 = nullptr;    // [ncell][n]
  std::vector<char> have_mat;
  std::vector<double> lam0, mu0, maxmod;
  cellfft::Fields<float> f32;
  cellfft::Fields<double> f64;
  double* x64 = nullptr;  // mixed precision FP64 solution [nslot][d n]
  double* x0 = nullptr;   // initial guesses of the linear solve [lpc][d n] (single cell; on first use)
  std::vector<char> x0_set;  // per load slot: a guess is set
  // scalars, reductions
  cellfft::LoadState* st = nullptr;
  cellfft::LoadState* st_h = nullptr;
  double* parts = nullptr;
  int maxblk = 0;
  double* res2 = nullptr;
  double* res2_h = nullptr;
  double* sparts = nullptr;
  double* sbar = nullptr;  // [nslot][6]
  int* mask = nullptr;     // [nslot] slots of a masked residual / merge launch
  int* mask_h = nullptr;
  double* hparts = nullptr;
  double* hres = nullptr;
  double* grad = nullptr;
  // residual history of the last linear solve: ||r_k||^2 per slot (the
  // iterated residual, k = 0 the initial one), hist_n[l] entries of
  // hist_cap kept, relative to hist_fn2[l] = ||f||^2
  double* hist = nullptr;
  int hist_cap = 0;
  std::vector<int> hist_n;
  std::vector<double> hist_fn2;
  double* scratch = nullptr;
  int hblk = 0;
  // neo-Hookean Newton path
  int op = 0;                   // PCG operator: 0 linear elasticity, 1 neo-Hookean tangent,
                                // 2 surrogate stencil (while one is set)
  double* hy_u = nullptr;       // Newton state [nslot][d n]
  float* hy_u32 = nullptr;      // its FP32 rounding (mixed-precision tangent)
  double* hy_ut = nullptr;      // line-search trial state
  double* hy_rhs = nullptr;     // f(u) = -grad Pi [nslot][d n]
  double* hy_F = nullptr;       // [nslot][9] macroscopic deformation gradients
  float* hy_F32 = nullptr;      // the same rounded to FP32
  // surrogate stencil operator (op 2): sampling step, spline degree, the
  // interpolated stencil blocks [63][n] (FP64, FP32), exact load vectors
  // [slot][3][n], per-block component sums and component means [slot][3]
  int sr_M = 0, sr_q = 0;
  double* sr64 = nullptr;
  float* sr32 = nullptr;
  double* sr_rhs = nullptr;
  double* sr_parts = nullptr;
  double* sr_mean = nullptr;
  double sr_setup_s = 0.0;
  double* hy_t = nullptr;       // [nslot] line-search steps
  double* hy_vparts = nullptr;  // [nslot][10][maxblk] energy / stress partials
  double* hy_vals = nullptr;    // [nslot][10]
  double* hy_vals_h = nullptr;  // pinned host copy
  bool linear_results = false;  // homog / residual hold the last linear solve
  std::vector<int> negcurv;     // per slot: iterations at a negative-curvature stop (0: none)
  // last solve
  int nload_solved = 0;
  double eps_v[6][6] = {};
  bool solved = false;
  bool solved_unit = false;
  int solved_op = 0;          // operator of the last solve (op values above)
  std::vector<double> homog;  // [ncell][nval] from the last solve
  // per-kernel event timing
  bool prof = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_kind;
  int ev_used = 0;
  double prof_ms[CELL_NKERNEL] = {};
  long long prof_cnt[CELL_NKERNEL] = {};
};

struct cell_batch_s {
  std::vector<cell_s*> cls;           // one instance per distinct grid configuration
  std::vector<int> cls_of, idx_of;    // cell i -> (instance, index within it)
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int dev = 0;
  int nv = 6;
};

namespace cellfft {

cell_status fail(cell_status s, const std::string& m);
const char* last_error_message();

// instance lifecycle (ncell cells of one grid, all on one stream)
cell_status instance_create(const cell_config* cfg, int ncell, hipStream_t shared_stream, cell_s** out);
void instance_destroy(cell_s* c);
cell_status instance_set_material(cell_s* c, int cell, const double* E, const double* nu, int on_device);
// solves nload macro strains (host [nload][nv]) for every cell; infos: ncell entries or nullptr;
// afterwards c->homog holds [ncell][nload*nload + nload*nv]
cell_status instance_solve(cell_s* c, int nload, const double* eps, cell_info* infos);
// single steps on slot 0 of cell 0 (host vectors [d][n]); invalidate the last solve
cell_status instance_apply_operator(cell_s* c, int precision, const double* u, double* q);
cell_status instance_apply_precond(cell_s* c, int precision, const double* r, double* z);
// neo-Hookean single steps on slot 0: p != nullptr: out = K_T(u) p (precision);
// p == nullptr: out = f(u) = -grad Pi in FP64, vals[10] = sum |s| W, sum |s| P
cell_status instance_hyper_step(cell_s* c, int precision, const double* Fbar, const double* u, const double* p,
                                double* out, double* vals);
// surrogate stencil operator: M = 0 switches it off; else sample every M-th
// node, B-spline degree q; later solves use it (op 2)
cell_status instance_set_surrogate(cell_s* c, int M, int q);
// the interpolated stencil blocks [7][3][3][n] (host, FP64)
cell_status instance_get_surrogate(cell_s* c, double* out);
cell_status instance_profile(cell_s* c, int enable);
cell_status instance_profile_read(cell_s* c, double* ms_out, long long* launches_out);
// autotuner: schedule from the cache (unless force) or by timing the variants
cell_status instance_autotune(cell_s* c, int force);
// neo-Hookean cell problem for nload macroscopic deformation gradients
// (host [nload][d][d]); results per cell: P_out [ncell][nload][d][d] (mean
// first Piola stress), infos [ncell] (may be nullptr)
cell_status instance_hyper_solve(cell_s* c, int nload, const double* Fbar, double tol, int max_newton,
                                 double* P_out, cell_hyper_info* infos);
void instance_get_schedule(cell_s* c, int* out);            // SCHED_NFIELD ints
cell_status instance_set_schedule(cell_s* c, const int* in);
// FFT preconditioner on device vectors of slot 0 (FP64): prepare once, then
// z = K_ref^{-1} r ([d][n], device, the handle's stream)
cell_status instance_precond_prepare(cell_s* c);
cell_status instance_precond_device(cell_s* c, const double* r, double* z);
// strain-based projection CG (3D, FP64) for nload macro strains (host
// [nload][6]); mean stresses [nload][6] (host); iterations in info
cell_status instance_solve_projection(cell_s* c, int nload, const double* eps, double* stress_out, cell_info* info);
// initial guess of load slot `load` for later linear solves with the exact
// operator (u0 [d][n], host or device; nullptr clears it)
cell_status instance_set_guess(cell_s* c, int load, const double* u0, int on_device);

// An in-flight solve of one instance.  Phases: solve_begin, then
// { solve_launch; synchronise the instance's stream; solve_poll } until
// done, then solve_end (statuses, homogenisation).  Several instances on one
// stream can interleave their launches and share one synchronisation.
struct SolveRun {
  cell_s* c = nullptr;
  int nload = 0;
  cell_info* infos = nullptr;  // ncell entries or nullptr
  std::vector<double> fn2, rr_ru;
  std::vector<int> fin, nref, active;
  // stagnation: smallest ||r||^2 seen at the polls and the iteration that
  // last halved it; restarts taken; slots marked for the stagnation refresh;
  // slots that ended on stagnation
  std::vector<double> best;
  std::vector<int> best_it, restarts, stag_pending, stagnated;
  hipGraphExec_t gexec = nullptr;  // CHUNK iterations, captured at the first launch
  cell_status result = CELL_OK;
  bool done = false;
  SolveRun() = default;
  SolveRun(const SolveRun&) = delete;
  SolveRun& operator=(const SolveRun&) = delete;
  ~SolveRun() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
  }
};
cell_status solve_begin(SolveRun& R, cell_s* c, int nload, const double* eps, cell_info* infos);
cell_status solve_launch(SolveRun& R);
// the pieces of solve_launch, for callers that capture several instances'
// chunks into one graph: whether the instance launches from graphs (not
// while profiling), its CHUNK iterations (eager, or into an open capture on
// its stream), the copy of its slot states to the host
bool solve_graphs(const SolveRun& R);
cell_status solve_enqueue_chunk(SolveRun& R);
cell_status solve_copy_states(SolveRun& R);
cell_status solve_poll(SolveRun& R);
cell_status solve_end(SolveRun& R);

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DevGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

double now_s();

}  // namespace cellfft
