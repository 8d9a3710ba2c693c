// Host driver and C ABI of the cell-problem solver (see include/cellfft.h).
//
// One PCG iteration is the kernel sequence
//   K-apply (q = K p, alpha = rz / pq)
//   -> x forward pass (r -= alpha q, ||r||^2, FFT_x)
//   -> y pass (FFT_y)            [3D]
//   -> last pass (FFT, z_hat = K_ref^{-1} r_hat, r.z, beta, inverse FFT)
//   -> y pass (inverse FFT_y)    [3D]
//   -> x inverse pass (inverse FFT_x, x += alpha p, p = z + beta p)
// with every scalar kept on the device; the host reads the per-load states
// once per chunk of iterations.  Mixed precision: the bulk runs in FP32 and
// the FP32 iterate is a correction to an FP64 solution; whenever the
// iterated residual has dropped by a factor DELTA since the last FP64
// residual (or the iterated test passes), the correction is merged into the
// FP64 solution and the residual is recomputed in FP64 (reliable update).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cellfft.h"
#include "kernels.h"

using namespace cellfft;

namespace {

thread_local std::string g_err;

cell_status fail(cell_status s, const std::string& m) {
  g_err = m;
  return s;
}

#define HIPCHK(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail(CELL_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define STCHK(call)                    \
  do {                                 \
    cell_status s_ = (call);           \
    if (s_ < 0) return s_;             \
  } while (0)

constexpr int CHUNK = 8;          // iterations between host polls
constexpr double DELTA = 0.05;    // reliable-update trigger (residual reduction)

template <typename T> struct Fields {
  T* x = nullptr;
  T* r = nullptr;
  T* p = nullptr;
  T* q = nullptr;
  cpx<T>* S = nullptr;
  cpx<T>* tw[3] = {nullptr, nullptr, nullptr};
  T* trig[3] = {nullptr, nullptr, nullptr};
  T* symtab = nullptr;   // 3D: tabulated K_ref^{-1}/n (see k_symtab)
  T* symtabB = nullptr;
  double sym_lam0 = -1.0, sym_mu0 = -1.0;  // reference medium of the table
  bool ready = false;
};

__global__ void k_merge(double* x64, float* x32, long long count) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    x64[i] += (double)x32[i];
    x32[i] = 0.0f;
  }
}

__global__ void k_colsum(const double* u, long long n, int ncomp, double* parts, int nblk) {
  __shared__ double sh[NT / WAVE];
  for (int c = 0; c < ncomp; ++c) {
    double v = 0.0;
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT)
      v += u[c * n + i];
    const double s = block_sum<NT>(v, sh);
    if (threadIdx.x == 0) parts[(long long)c * nblk + blockIdx.x] = s;
  }
}

__global__ void k_sum_rows2(const double* parts, int nblk, double scale, double* out) {
  __shared__ double sh[NT / WAVE];
  const double* row = parts + (long long)blockIdx.x * nblk;
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += NT) v += row[i];
  const double s = block_sum<NT>(v, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s * scale;
}

__global__ void k_sub_mean(const double* u, const double* mean, long long n, int ncomp, double* out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n * ncomp;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = u[i] - mean[i / n];
}

}  // namespace

struct cell_s {
  int dev = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Geom g{};
  int d = 3, nv = 6;
  long long n = 0, lstride = 0;
  int precision = CELL_FP64;
  double tol = 1e-10;
  int max_iter = 10000;
  int max_loads = 6;
  double* mat64 = nullptr;
  float* mat32 = nullptr;
  double* E64 = nullptr;
  bool have_mat = false;
  double lam0 = 0, mu0 = 0, maxmod = 0;
  Fields<float> f32;
  Fields<double> f64;
  double* x64 = nullptr;  // mixed-precision FP64 solution
  LoadState* st = nullptr;
  LoadState* st_h = nullptr;
  double* parts = nullptr;
  unsigned* cnt = nullptr;
  int maxblk = 0;
  double* res2 = nullptr;
  double* res2_h = nullptr;
  double* sparts = nullptr;  // per-block stress sums of the residual launch
  double* sbar = nullptr;    // [max_loads][6] stress sums of the last residual per load
  double* hparts = nullptr;
  double* hres = nullptr;
  double* grad = nullptr;
  double* scratch = nullptr;  // small device scratch (means)
  int hblk = 0;
  int nload_solved = 0;
  double energy[36] = {};  // energy-form C among the loads of the last solve
  double eps_v[6][6] = {};
  bool solved = false;
  bool solved_unit = false;
  // per-kernel HIP-event timing (cell_profile)
  bool prof = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_kind;
  int ev_used = 0;
  double prof_ms[CELL_NKERNEL] = {};
  long long prof_cnt[CELL_NKERNEL] = {};
};

namespace {

RedBuf red_of(cell_s* c) { return RedBuf{c->parts, c->cnt, c->maxblk, c->max_loads}; }

constexpr int PROF_PAIRS = 256;

// Sum the elapsed times of the recorded event pairs (all complete: called
// after a stream synchronisation) and recycle the pool.
cell_status prof_collect(cell_s* c) {
  for (int i = 0; i < c->ev_used; ++i) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
    c->prof_ms[c->ev_kind[i]] += ms;
    c->prof_cnt[c->ev_kind[i]] += 1;
  }
  c->ev_used = 0;
  return CELL_OK;
}

// Brackets one kernel launch with an event pair on the handle's stream.
struct ProfScope {
  cell_s* c;
  int slot = -1;
  ProfScope(cell_s* c_, int kind) : c(c_) {
    if (!c->prof) return;
    if (c->ev_used == PROF_PAIRS) {
      (void)hipStreamSynchronize(c->stream);
      (void)prof_collect(c);
    }
    slot = c->ev_used++;
    c->ev_kind[slot] = kind;
    (void)hipEventRecord(c->ev[2 * slot], c->stream);
  }
  ~ProfScope() {
    if (slot >= 0) (void)hipEventRecord(c->ev[2 * slot + 1], c->stream);
  }
};

template <typename T> Fields<T>& fields(cell_s* c);
template <> Fields<float>& fields<float>(cell_s* c) { return c->f32; }
template <> Fields<double>& fields<double>(cell_s* c) { return c->f64; }

template <typename T> const T* mat_of(cell_s* c);
template <> const float* mat_of<float>(cell_s* c) { return c->mat32; }
template <> const double* mat_of<double>(cell_s* c) { return c->mat64; }

const double* solution64(cell_s* c) { return c->precision == CELL_MIXED ? c->x64 : c->f64.x; }

template <typename T>
cell_status ensure_fields(cell_s* c) {
  Fields<T>& F = fields<T>(c);
  if (F.ready) return CELL_OK;
  const size_t bytes = sizeof(T) * (size_t)c->lstride * c->max_loads;
  T** bufs[4] = {&F.x, &F.r, &F.p, &F.q};
  for (T** b : bufs) {
    if (hipMalloc((void**)b, bytes) != hipSuccess) return fail(CELL_E_NOMEM, "device allocation of a field failed");
    HIPCHK(hipMemset(*b, 0, bytes));
  }
  if (hipMalloc((void**)&F.S, bytes) != hipSuccess) return fail(CELL_E_NOMEM, "device allocation of the spectrum failed");
  const int N[3] = {c->g.nx, c->g.ny, c->g.nz};
  for (int a = 0; a < c->d; ++a) {
    std::vector<cpx<T>> tw(N[a]);
    std::vector<T> tr(2 * N[a]);
    for (int m = 0; m < N[a]; ++m) {
      const double ang = -2.0 * M_PI * (double)m / N[a];
      tw[m] = cpx<T>{(T)std::cos(ang), (T)std::sin(ang)};
    }
    // (sin, cos) of theta = pi k / N, exactly mirrored: k -> N - k keeps the
    // sine and flips the cosine, so the symbol is bitwise symmetric under
    // wavevector negation.
    for (int k = 0; k <= N[a] / 2; ++k) {
      double s = std::sin(M_PI * k / N[a]), co = std::cos(M_PI * k / N[a]);
      if (2 * k == N[a]) { s = 1.0; co = 0.0; }
      tr[2 * k] = (T)s;
      tr[2 * k + 1] = (T)co;
      if (k > 0 && k < N[a] - k) {
        tr[2 * (N[a] - k)] = (T)s;
        tr[2 * (N[a] - k) + 1] = (T)(-co);
      }
    }
    HIPCHK(hipMalloc((void**)&F.tw[a], sizeof(cpx<T>) * N[a]));
    HIPCHK(hipMalloc((void**)&F.trig[a], sizeof(T) * 2 * N[a]));
    HIPCHK(hipMemcpy(F.tw[a], tw.data(), sizeof(cpx<T>) * N[a], hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(F.trig[a], tr.data(), sizeof(T) * 2 * N[a], hipMemcpyHostToDevice));
  }
  if (c->d == 2) {  // unused third axis: a 1-entry table keeps kernel args valid
    HIPCHK(hipMalloc((void**)&F.trig[2], sizeof(T) * 2));
    T z2[2] = {T(0), T(1)};
    HIPCHK(hipMemcpy(F.trig[2], z2, sizeof(T) * 2, hipMemcpyHostToDevice));
  }
  F.ready = true;
  return CELL_OK;
}

void voigt_to_tensor(int d, const double* v, double* t) {
  for (int i = 0; i < 6; ++i) t[i] = 0.0;
  if (d == 3) {
    t[0] = v[0];
    t[1] = v[1];
    t[2] = v[2];
    t[3] = 0.5 * v[3];
    t[4] = 0.5 * v[4];
    t[5] = 0.5 * v[5];
  } else {
    t[0] = v[0];
    t[1] = v[1];
    t[5] = 0.5 * v[2];
  }
}

template <typename T>
KArgs<T> kargs(cell_s* c, int mode, const T* u, void* out, const T* mat, int nload) {
  KArgs<T> a{};
  a.u = u;
  a.out = out;
  a.mat = mat;
  a.lstride = c->lstride;
  a.g = c->g;
  for (int l = 0; l < 6; ++l) voigt_to_tensor(c->d, c->eps_v[l], a.eps[l]);
  a.nload = nload;
  a.mode = mode;
  a.st = c->st;
  a.only_load = -1;
  a.res2 = c->res2;
  a.red = red_of(c);
  return a;
}

template <typename T>
PArgs<T> make_pargs(cell_s* c, int nload) {
  Fields<T>& F = fields<T>(c);
  PArgs<T> pa{};
  pa.S = F.S;
  pa.lstrideC = c->lstride / 2;
  pa.nx = c->g.nx;
  pa.ny = c->g.ny;
  pa.nz = c->g.nz;
  pa.tw = F.tw[c->d - 1];
  for (int a = 0; a < 3; ++a) pa.trig[a] = F.trig[a];
  pa.lam0 = (T)c->lam0;
  pa.mu0 = (T)c->mu0;
  pa.w = (T)(c->d == 3 ? c->g.h[0] * c->g.h[1] * c->g.h[2] / 6.0 : c->g.h[0] * c->g.h[1] / 2.0);
  for (int a = 0; a < 3; ++a) pa.ih[a] = (T)(1.0 / c->g.h[a]);
  pa.inv_n = (T)(1.0 / (double)c->n);
  pa.nload = nload;
  pa.tab = nullptr;
  pa.tabB = nullptr;
  pa.st = c->st;
  pa.red = red_of(c);
  return pa;
}

// 3D: (re)builds the tabulated inverse symbol when the reference medium
// changed, and points pa at it
template <typename T>
cell_status ensure_symtab(cell_s* c, PArgs<T>& pa) {
  if (c->d != 3) return CELL_OK;
  Fields<T>& F = fields<T>(c);
  if (!F.symtab) {
    const size_t entries = (size_t)c->g.ny * c->g.nz * (c->g.nx / 2);
    if (hipMalloc((void**)&F.symtab, sizeof(T) * 6 * entries) != hipSuccess ||
        hipMalloc((void**)&F.symtabB, sizeof(T) * 6 * 2 * c->g.nz) != hipSuccess)
      return fail(CELL_E_NOMEM, "device allocation of the symbol table failed");
  }
  if (F.sym_lam0 != c->lam0 || F.sym_mu0 != c->mu0) {
    HIPCHK(launch_symtab<T>(pa, F.symtab, F.symtabB, c->stream));
    F.sym_lam0 = c->lam0;
    F.sym_mu0 = c->mu0;
  }
  pa.tab = F.symtab;
  pa.tabB = F.symtabB;
  return CELL_OK;
}

// one PCG iteration (or the initial preconditioning if !kapply)
template <typename T>
cell_status iteration(cell_s* c, int nload, bool kapply) {
  Fields<T>& F = fields<T>(c);
  hipStream_t s = c->stream;
  if (kapply) {
    KArgs<T> ka = kargs<T>(c, 0, F.p, F.q, mat_of<T>(c), nload);
    ProfScope ps(c, CELL_K_APPLY);
    HIPCHK(launch_stencil<T>(ka, s));
  }
  XArgs<T> xa{};
  xa.r = F.r;
  xa.q = F.q;
  xa.S = F.S;
  xa.x = F.x;
  xa.p = F.p;
  xa.lstride = c->lstride;
  xa.nrows = (int)(c->lstride / c->g.nx);
  xa.tw = F.tw[0];
  xa.st = c->st;
  xa.red = red_of(c);
  {
    ProfScope ps(c, CELL_K_XFWD);
    HIPCHK(launch_xfwd<T>(xa, c->g.nx, nload, s));
  }
  HIPCHK(launch_finalize(xa.red, c->st, c->res2, RED_RR, xpass_blocks(c->g.nx, xa.nrows, sizeof(T) == 8), nload,
                         -1, s));
  YArgs<T> ya{};
  ya.S = F.S;
  ya.lstrideC = c->lstride / 2;
  ya.nx = c->g.nx;
  ya.ny = c->g.ny;
  ya.nz = c->g.nz;
  ya.ncomp = c->d;
  ya.tw = F.tw[1];
  ya.st = c->st;
  PArgs<T> pa = make_pargs<T>(c, nload);
  STCHK(ensure_symtab<T>(c, pa));
  if (c->d == 3) {
    ProfScope ps(c, CELL_K_YFWD);
    HIPCHK(launch_ypass<T>(ya, false, nload, s));
  }
  {
    ProfScope ps(c, CELL_K_LAST);
    HIPCHK(launch_last<T>(pa, c->d, nload, s));
  }
  HIPCHK(launch_finalize(pa.red, c->st, c->res2, RED_RZ, last_pass_blocks(c->d, c->g.nx, c->g.ny, sizeof(T) == 8),
                         nload, -1, s));
  if (c->d == 3) {
    ProfScope ps(c, CELL_K_YINV);
    HIPCHK(launch_ypass<T>(ya, true, nload, s));
  }
  {
    ProfScope ps(c, CELL_K_XINV);
    HIPCHK(launch_xinv<T>(xa, c->g.nx, nload, s));
  }
  return CELL_OK;
}

// r = f - K u in FP64 for one load (or all: load < 0); ||r||^2 -> res2_h
template <typename T>
cell_status residual(cell_s* c, int nload, int load, const double* u) {
  Fields<T>& F = fields<T>(c);
  KArgs<double> ka = kargs<double>(c, 1, u, nullptr, c->mat64, nload);
  ka.only_load = load;
  ka.sparts = c->sparts;
  ka.sbar = c->sbar;
  {
    ProfScope ps(c, CELL_K_RESIDUAL);
    if (sizeof(T) == 4) {
      HIPCHK(launch_residual_mixed(ka, reinterpret_cast<float*>(F.r), c->stream));
    } else {
      ka.out = F.r;
      HIPCHK(launch_stencil<double>(ka, c->stream));
    }
  }
  HIPCHK(hipMemcpyAsync(c->res2_h, c->res2, sizeof(double) * c->max_loads, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CELL_OK;
}

template <typename T>
cell_status run_solve(cell_s* c, int nload, cell_info* info) {
  STCHK(ensure_fields<T>(c));
  Fields<T>& F = fields<T>(c);
  const bool mixed = sizeof(T) == 4;
  hipStream_t s = c->stream;
  const size_t fb = sizeof(T) * (size_t)c->lstride * nload;
  HIPCHK(hipMemsetAsync(F.x, 0, fb, s));
  HIPCHK(hipMemsetAsync(F.p, 0, fb, s));
  HIPCHK(hipMemsetAsync(F.q, 0, fb, s));
  if (mixed) HIPCHK(hipMemsetAsync(c->x64, 0, sizeof(double) * (size_t)c->lstride * nload, s));
  // load vectors f = -B^T D eps_bar, ||f||^2
  STCHK(residual<T>(c, nload, -1, nullptr));
  std::vector<double> fn2(nload), rr_ru(nload);
  std::vector<int> fin(nload, 0), nref(nload, 0);
  // scale of the load vector without cancellation, for the homogeneous test
  double emax = 0.0;
  for (int l = 0; l < nload; ++l)
    for (int i = 0; i < c->nv; ++i) emax = std::max(emax, std::fabs(c->eps_v[l][i]));
  const double hmin = std::min(c->g.h[0], std::min(c->g.h[1], c->d == 3 ? c->g.h[2] : c->g.h[1]));
  const double wvol = c->d == 3 ? c->g.h[0] * c->g.h[1] * c->g.h[2] : c->g.h[0] * c->g.h[1];
  const double fscale = std::sqrt((double)c->n) * wvol * c->maxmod * emax / hmin;
  for (int l = 0; l < c->max_loads; ++l) {
    LoadState& S = c->st_h[l];
    std::memset(&S, 0, sizeof(S));
    S.state = ST_IDLE;
    S.maxit = c->max_iter;
    S.first = 1;
    if (l >= nload) continue;
    fn2[l] = c->res2_h[l];
    rr_ru[l] = fn2[l];
    S.rr = fn2[l];
    S.thr = c->tol * c->tol * fn2[l];
    if (std::sqrt(fn2[l]) <= 1e-13 * fscale) {  // homogeneous: f = 0 up to round-off, u = 0
      S.state = ST_DONE;
      fin[l] = 1;
    } else {
      S.state = ST_ACTIVE;
    }
  }
  HIPCHK(hipMemcpyAsync(c->st, c->st_h, sizeof(LoadState) * c->max_loads, hipMemcpyHostToDevice, s));
  STCHK(iteration<T>(c, nload, false));
  cell_status result = CELL_OK;
  bool done = false;
  while (!done) {
    for (int i = 0; i < CHUNK; ++i) STCHK(iteration<T>(c, nload, true));
    HIPCHK(hipMemcpyAsync(c->st_h, c->st, sizeof(LoadState) * c->max_loads, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (c->prof) STCHK(prof_collect(c));
    done = true;
    for (int l = 0; l < nload; ++l) {
      if (fin[l]) continue;
      LoadState& S = c->st_h[l];
      if (S.state == ST_BREAKDOWN) {
        fin[l] = 1;
        result = fail(CELL_E_BREAKDOWN, "CG breakdown in load " + std::to_string(l));
        continue;
      }
      // CONVERGED: the converging iteration has completed (its operator
      // finalisation, which marks DONE, has not run yet)
      const bool finished = S.state == ST_DONE || S.state == ST_CONVERGED;
      const bool ru = finished || (mixed && S.state == ST_ACTIVE && S.rr < DELTA * DELTA * rr_ru[l]);
      if (ru) {
        const double* u64;
        if (mixed) {
          const long long off = (long long)l * c->lstride;
          {
            ProfScope ps(c, CELL_K_MERGE);
            hipLaunchKernelGGL(k_merge, dim3(1024), dim3(256), 0, s, c->x64 + off,
                               reinterpret_cast<float*>(F.x) + off, c->lstride);
          }
          HIPCHK(hipGetLastError());
          u64 = c->x64;
        } else {
          u64 = reinterpret_cast<const double*>(F.x);
        }
        STCHK(residual<T>(c, nload, l, u64));
        const double rt = c->res2_h[l];
        rr_ru[l] = rt;
        nref[l] += 1;
        if (!(rt == rt)) {
          fin[l] = 1;
          result = fail(CELL_E_BREAKDOWN, "non-finite residual in load " + std::to_string(l));
          continue;
        }
        if (rt <= S.thr || (finished && S.maxit_hit) || S.iters >= c->max_iter) {
          fin[l] = 1;
          S.rr = rt;
          S.state = ST_DONE;
        } else {
          S.state = ST_ACTIVE;
          S.rr = rt;
        }
        HIPCHK(hipMemcpyAsync(c->st + l, &S, sizeof(LoadState), hipMemcpyHostToDevice, s));
      }
      if (!fin[l]) done = false;
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  bool all_conv = true;
  for (int l = 0; l < nload; ++l) {
    const LoadState& S = c->st_h[l];
    const double rel = fn2[l] > 0 ? std::sqrt(rr_ru[l] / fn2[l]) : 0.0;
    if (info) {
      info->iters[l] = S.iters;
      info->refinements[l] = nref[l];
      info->relres[l] = fin[l] && S.state == ST_DONE && nref[l] == 0 ? 0.0 : rel;
    }
    if (rel > c->tol && fn2[l] > 0 && nref[l] > 0) all_conv = false;
  }
  if (info) info->nload = nload;
  if (result < 0) return result;
  return all_conv ? CELL_OK : CELL_NOT_CONVERGED;
}

cell_status solve_loads(cell_s* c, int nload, const double* eps, cell_info* info) {
  for (int l = 0; l < 6; ++l)
    for (int i = 0; i < 6; ++i) c->eps_v[l][i] = (l < nload && i < c->nv) ? eps[l * c->nv + i] : 0.0;
  c->solved = false;
  c->solved_unit = false;
  cell_status st;
  if (c->precision == CELL_MIXED) st = run_solve<float>(c, nload, info);
  else st = run_solve<double>(c, nload, info);
  if (st >= 0) {
    c->solved = true;
    c->nload_solved = nload;
  }
  return st;
}

// C* (energy form) and mean stresses of the solved loads; uses the final
// residuals and stress sums left by the last FP64 residual of every load
cell_status homogenize(cell_s* c, int nload, std::vector<double>& out) {
  HArgs h{};
  h.u = solution64(c);
  h.mat = c->mat64;
  h.E = c->E64;
  h.lstride = c->lstride;
  h.g = c->g;
  for (int l = 0; l < 6; ++l) voigt_to_tensor(c->d, c->eps_v[l], h.eps[l]);
  h.nload = nload;
  if (c->precision == CELL_MIXED) {
    h.r = c->f32.r;
    h.r_fp64 = 0;
  } else {
    h.r = c->f64.r;
    h.r_fp64 = 1;
  }
  h.sbar = c->sbar;
  h.parts = c->hparts;
  h.result = c->hres;
  h.nblk = c->hblk;
  {
    ProfScope ps(c, CELL_K_HOMOG);
    HIPCHK(launch_homog(h, c->stream));
  }
  const int nval = nload * nload + nload * c->nv;
  out.resize(nval);
  HIPCHK(hipMemcpyAsync(out.data(), c->hres, sizeof(double) * nval, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->prof) STCHK(prof_collect(c));
  return CELL_OK;
}

bool size_ok(int n) { return fft_size_ok(n); }

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

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

}  // namespace

// ======================================================================= ABI
extern "C" {

const char* cell_last_error(void) { return g_err.c_str(); }

void cell_destroy(cell_t c) {
  if (!c) return;
  DevGuard dg(c->dev);
  (void)hipDeviceSynchronize();
  auto fr = [](void* p) {
    if (p) (void)hipFree(p);
  };
  fr(c->mat64);
  fr(c->mat32);
  fr(c->E64);
  for (void* p : {(void*)c->f32.x, (void*)c->f32.r, (void*)c->f32.p, (void*)c->f32.q, (void*)c->f32.S,
                  (void*)c->f32.symtab, (void*)c->f32.symtabB, (void*)c->f64.x, (void*)c->f64.r,
                  (void*)c->f64.p, (void*)c->f64.q, (void*)c->f64.S, (void*)c->f64.symtab,
                  (void*)c->f64.symtabB})
    fr(p);
  for (int a = 0; a < 3; ++a) {
    fr(c->f32.tw[a]);
    fr(c->f32.trig[a]);
    fr(c->f64.tw[a]);
    fr(c->f64.trig[a]);
  }
  fr(c->x64);
  fr(c->st);
  fr(c->parts);
  fr(c->cnt);
  fr(c->res2);
  fr(c->sparts);
  fr(c->sbar);
  fr(c->hparts);
  fr(c->hres);
  fr(c->grad);
  fr(c->scratch);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->st_h) (void)hipHostFree(c->st_h);
  if (c->res2_h) (void)hipHostFree(c->res2_h);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

cell_status cell_create(const cell_config* cfg, cell_t* out) {
  if (!cfg || !out) return fail(CELL_E_ARG, "null argument");
  *out = nullptr;
  if (cfg->dim != 2 && cfg->dim != 3) return fail(CELL_E_ARG, "dim must be 2 or 3");
  for (int a = 0; a < cfg->dim; ++a) {
    if (cfg->n[a] < 1) return fail(CELL_E_ARG, "grid sizes must be positive");
    if (!size_ok(cfg->n[a]))
      return fail(CELL_E_UNSUPPORTED, "grid size " + std::to_string(cfg->n[a]) +
                                          " has no FFT plan (supported: 4,6,8,12,16,24,32,48,64,96,128,192,256)");
    if (!(cfg->len[a] >= 0.0) || !std::isfinite(cfg->len[a])) return fail(CELL_E_ARG, "invalid cell length");
  }
  if (cfg->precision != CELL_FP64 && cfg->precision != CELL_MIXED) return fail(CELL_E_ARG, "invalid precision");
  if (cfg->tol < 0.0 || !std::isfinite(cfg->tol)) return fail(CELL_E_ARG, "invalid tolerance");
  if (cfg->max_iter < 0) return fail(CELL_E_ARG, "invalid max_iter");
  const int nv = cfg->dim == 3 ? 6 : 3;
  if (cfg->max_loads < 0 || cfg->max_loads > nv) return fail(CELL_E_ARG, "max_loads must be in [0, nv]");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(CELL_E_DEVICE, "no HIP device");
  int dev = cfg->device;
  if (dev < 0) HIPCHK(hipGetDevice(&dev));
  if (dev >= ndev) return fail(CELL_E_ARG, "device ordinal out of range");
  DevGuard dg(dev);
  cell_s* c = new cell_s();
  c->dev = dev;
  c->d = cfg->dim;
  c->nv = nv;
  c->g.dim = cfg->dim;
  c->g.nx = cfg->n[0];
  c->g.ny = cfg->n[1];
  c->g.nz = cfg->dim == 3 ? cfg->n[2] : 1;
  c->n = (long long)c->g.nx * c->g.ny * c->g.nz;
  c->g.n = c->n;
  for (int a = 0; a < 3; ++a) {
    const double L = (a < cfg->dim && cfg->len[a] > 0.0) ? cfg->len[a] : 1.0;
    const int N = a == 0 ? c->g.nx : a == 1 ? c->g.ny : c->g.nz;
    c->g.h[a] = L / N;
  }
  c->lstride = (long long)c->d * c->n;
  c->precision = cfg->precision;
  c->tol = cfg->tol > 0.0 ? cfg->tol : (cfg->precision == CELL_MIXED ? 1e-6 : 1e-10);
  c->max_iter = cfg->max_iter > 0 ? cfg->max_iter : 10000;
  c->max_loads = cfg->max_loads > 0 ? cfg->max_loads : nv;
  cell_status st = CELL_OK;
  auto bail = [&](cell_status s) {
    cell_destroy(c);
    return s;
  };
  if (cfg->stream) {
    c->stream = (hipStream_t)cfg->stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) return bail(fail(CELL_E_DEVICE, "hipStreamCreate failed"));
    c->own_stream = true;
  }
  // reduction buffers sized for the largest grid of any reducing kernel
  const int nrows = (int)(c->lstride / c->g.nx);
  int mb = std::max(xpass_blocks(c->g.nx, nrows, true), xpass_blocks(c->g.nx, nrows, false));
  mb = std::max(mb, stencil_blocks(c->g));
  mb = std::max(mb, (c->g.nx / 2 + 3) / 4 * c->g.ny * c->g.nz + 8);
  mb = std::max(mb, (c->g.nx / 2 + 7) / 8 * c->g.ny * c->g.nz + 8);
  c->maxblk = mb;
  auto dmalloc = [&](void** p, size_t bytes) -> bool { return hipMalloc(p, bytes) == hipSuccess; };
  if (!dmalloc((void**)&c->parts, sizeof(double) * (size_t)RED_NSLOT * c->max_loads * mb) ||
      !dmalloc((void**)&c->cnt, sizeof(unsigned) * RED_NSLOT * c->max_loads) ||
      !dmalloc((void**)&c->st, sizeof(LoadState) * c->max_loads) ||
      !dmalloc((void**)&c->res2, sizeof(double) * c->max_loads) ||
      !dmalloc((void**)&c->sparts, sizeof(double) * 6 * (size_t)c->max_loads * mb) ||
      !dmalloc((void**)&c->sbar, sizeof(double) * 6 * c->max_loads) ||
      !dmalloc((void**)&c->mat64, sizeof(double) * 2 * c->n) ||
      !dmalloc((void**)&c->mat32, sizeof(float) * 2 * c->n) ||
      !dmalloc((void**)&c->E64, sizeof(double) * c->n) ||
      !dmalloc((void**)&c->grad, sizeof(double) * c->n) ||
      !dmalloc((void**)&c->scratch, sizeof(double) * 64 * 1024))
    return bail(fail(CELL_E_NOMEM, "device allocation failed"));
  c->hblk = homog_blocks(c->g);
  const int nvalmax = c->max_loads * c->max_loads + c->max_loads * nv;
  if (!dmalloc((void**)&c->hparts, sizeof(double) * (size_t)nvalmax * c->hblk) ||
      !dmalloc((void**)&c->hres, sizeof(double) * nvalmax))
    return bail(fail(CELL_E_NOMEM, "device allocation failed"));
  if (c->precision == CELL_MIXED &&
      !dmalloc((void**)&c->x64, sizeof(double) * (size_t)c->lstride * c->max_loads))
    return bail(fail(CELL_E_NOMEM, "device allocation failed"));
  if (hipHostMalloc((void**)&c->st_h, sizeof(LoadState) * c->max_loads) != hipSuccess ||
      hipHostMalloc((void**)&c->res2_h, sizeof(double) * c->max_loads) != hipSuccess)
    return bail(fail(CELL_E_NOMEM, "pinned host allocation failed"));
  if (hipMemset(c->cnt, 0, sizeof(unsigned) * RED_NSLOT * c->max_loads) != hipSuccess ||
      hipMemset(c->st, 0, sizeof(LoadState) * c->max_loads) != hipSuccess)
    return bail(fail(CELL_E_DEVICE, "hipMemset failed"));
  if (c->precision == CELL_MIXED) st = ensure_fields<float>(c);
  else st = ensure_fields<double>(c);
  if (st < 0) return bail(st);
  *out = c;
  return CELL_OK;
}

cell_status cell_set_material(cell_t c, const double* E, const double* nu, int on_device) {
  if (!c || !E || !nu) return fail(CELL_E_ARG, "null argument");
  DevGuard dg(c->dev);
  const long long n = c->n;
  std::vector<double> Eh(n), nh(n);
  if (on_device) {
    HIPCHK(hipMemcpyAsync(Eh.data(), E, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(nh.data(), nu, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  } else {
    std::memcpy(Eh.data(), E, sizeof(double) * n);
    std::memcpy(nh.data(), nu, sizeof(double) * n);
  }
  std::vector<double> m64(2 * n);
  std::vector<float> m32(2 * n);
  double kmin = INFINITY, kmax = 0, mmin = INFINITY, mmax = 0, modmax = 0;
  for (long long v = 0; v < n; ++v) {
    const double e = Eh[v], p = nh[v];
    if (!std::isfinite(e) || !(e > 0.0))
      return fail(CELL_E_NONFINITE, "Young's modulus must be finite and positive (voxel " + std::to_string(v) + ")");
    if (!std::isfinite(p) || !(p > -1.0) || !(p < 0.5))
      return fail(CELL_E_ARG, "Poisson ratio must lie in (-1, 0.5) (voxel " + std::to_string(v) + ")");
    const double lam = p * e / ((1.0 + p) * (1.0 - 2.0 * p));
    const double mu = e / (2.0 * (1.0 + p));
    m64[2 * v] = lam;
    m64[2 * v + 1] = mu;
    m32[2 * v] = (float)lam;
    m32[2 * v + 1] = (float)mu;
    const double bulk = lam + (c->d == 3 ? 2.0 * mu / 3.0 : mu);
    kmin = std::min(kmin, bulk);
    kmax = std::max(kmax, bulk);
    mmin = std::min(mmin, mu);
    mmax = std::max(mmax, mu);
    modmax = std::max(modmax, std::fabs(lam) + 2.0 * mu);
  }
  HIPCHK(hipMemcpyAsync(c->mat64, m64.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->mat32, m32.data(), sizeof(float) * 2 * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->E64, Eh.data(), sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const double K0 = std::sqrt(kmin * kmax), mu0 = std::sqrt(mmin * mmax);
  c->mu0 = mu0;
  c->lam0 = K0 - (c->d == 3 ? 2.0 * mu0 / 3.0 : mu0);
  c->maxmod = modmax;
  c->have_mat = true;
  c->solved = false;
  c->solved_unit = false;
  return CELL_OK;
}

cell_status cell_solve(cell_t c, int nload, const double* macro_strain, double* mean_stress_out,
                       cell_info* info) {
  const double t0 = now_s();
  if (!c || !macro_strain) return fail(CELL_E_ARG, "null argument");
  if (nload < 1 || nload > c->max_loads) return fail(CELL_E_ARG, "nload must be in [1, max_loads]");
  if (!c->have_mat) return fail(CELL_E_STATE, "cell_set_material has not been called");
  for (int i = 0; i < nload * c->nv; ++i)
    if (!std::isfinite(macro_strain[i])) return fail(CELL_E_ARG, "non-finite macro strain");
  DevGuard dg(c->dev);
  if (info) std::memset(info, 0, sizeof(*info));
  cell_status st = solve_loads(c, nload, macro_strain, info);
  if (st < 0) return st;
  std::vector<double> h;
  STCHK(homogenize(c, nload, h));
  for (int i = 0; i < nload * nload; ++i) c->energy[i] = h[i];
  if (mean_stress_out)
    for (int J = 0; J < nload; ++J)
      for (int q = 0; q < c->nv; ++q) mean_stress_out[J * c->nv + q] = h[nload * nload + J * c->nv + q];
  if (info) {
    double cmax = 0.0, gap = 0.0;
    for (int i = 0; i < nload * nload; ++i) cmax = std::max(cmax, std::fabs(h[i]));
    for (int J = 0; J < nload; ++J) {
      double se = 0.0;
      for (int q = 0; q < c->nv; ++q) se += h[nload * nload + J * c->nv + q] * c->eps_v[J][q];
      gap = std::max(gap, std::fabs(h[J * nload + J] - se));
    }
    info->hill_mandel_gap = cmax > 0 ? gap / cmax : 0.0;
    info->seconds = now_s() - t0;
  }
  return st;
}

cell_status cell_effective_stiffness(cell_t c, double* C_out, cell_info* info) {
  const double t0 = now_s();
  if (!c || !C_out) return fail(CELL_E_ARG, "null argument");
  if (!c->have_mat) return fail(CELL_E_STATE, "cell_set_material has not been called");
  if (c->max_loads < c->nv) return fail(CELL_E_ARG, "max_loads must be nv for the effective stiffness");
  DevGuard dg(c->dev);
  if (info) std::memset(info, 0, sizeof(*info));
  const int nv = c->nv;
  std::vector<double> eye(nv * nv, 0.0);
  for (int i = 0; i < nv; ++i) eye[i * nv + i] = 1.0;
  cell_status st = solve_loads(c, nv, eye.data(), info);
  if (st < 0) return st;
  std::vector<double> h;
  STCHK(homogenize(c, nv, h));
  for (int i = 0; i < nv * nv; ++i) c->energy[i] = h[i];
  double cmax = 0.0, smax = 0.0, sgap = 0.0, hgap = 0.0;
  for (int I = 0; I < nv; ++I)
    for (int J = 0; J < nv; ++J) {
      C_out[I * nv + J] = h[I * nv + J];
      cmax = std::max(cmax, std::fabs(h[I * nv + J]));
      const double sIJ = h[nv * nv + J * nv + I];  // mean stress of load J, component I
      const double sJI = h[nv * nv + I * nv + J];
      smax = std::max(smax, std::fabs(sIJ));
      sgap = std::max(sgap, std::fabs(sIJ - sJI));
    }
  for (int J = 0; J < nv; ++J) hgap = std::max(hgap, std::fabs(h[J * nv + J] - h[nv * nv + J * nv + J]));
  c->solved_unit = true;
  if (info) {
    info->sym_gap = smax > 0 ? sgap / smax : 0.0;
    info->hill_mandel_gap = cmax > 0 ? hgap / cmax : 0.0;
    info->seconds = now_s() - t0;
  }
  return st;
}

cell_status cell_adjoint(cell_t c, const double* dJ_dC, double* dJ_dE_out, int on_device) {
  if (!c || !dJ_dC || !dJ_dE_out) return fail(CELL_E_ARG, "null argument");
  if (!c->solved_unit) return fail(CELL_E_STATE, "cell_adjoint needs a preceding cell_effective_stiffness");
  DevGuard dg(c->dev);
  const int nv = c->nv;
  HArgs h{};
  h.u = solution64(c);
  h.mat = c->mat64;
  h.E = c->E64;
  h.lstride = c->lstride;
  h.g = c->g;
  for (int l = 0; l < 6; ++l) voigt_to_tensor(c->d, c->eps_v[l], h.eps[l]);
  h.nload = nv;
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J) {
      const double v = (I < nv && J < nv) ? dJ_dC[I * nv + J] : 0.0;
      if (!std::isfinite(v)) return fail(CELL_E_ARG, "non-finite dJ/dC");
      h.a[I][J] = v;
    }
  h.grad = on_device ? dJ_dE_out : c->grad;
  h.nblk = c->hblk;
  HIPCHK(launch_grad(h, c->stream));
  if (!on_device)
    HIPCHK(hipMemcpyAsync(dJ_dE_out, c->grad, sizeof(double) * c->n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CELL_OK;
}

cell_status cell_get_displacement(cell_t c, int load, double* u_out, int on_device) {
  if (!c || !u_out) return fail(CELL_E_ARG, "null argument");
  if (!c->solved) return fail(CELL_E_STATE, "no solution available");
  if (load < 0 || load >= c->nload_solved) return fail(CELL_E_ARG, "load index out of range");
  DevGuard dg(c->dev);
  const double* u = solution64(c) + (long long)load * c->lstride;
  const int nblk = 256;
  double* parts = c->scratch;
  double* mean = c->scratch + 8 * nblk;
  hipLaunchKernelGGL(k_colsum, dim3(nblk), dim3(NT), 0, c->stream, u, c->n, c->d, parts, nblk);
  hipLaunchKernelGGL(k_sum_rows2, dim3(c->d), dim3(NT), 0, c->stream, (const double*)parts, nblk,
                     1.0 / (double)c->n, mean);
  double* dst = on_device ? u_out : c->scratch + 16 * nblk;
  if (on_device) {
    hipLaunchKernelGGL(k_sub_mean, dim3(1024), dim3(256), 0, c->stream, u, (const double*)mean, c->n, c->d, dst);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return CELL_OK;
  }
  // host output: subtract on the device into the spectrum-sized scratch of the
  // FP64 residual field is not available in mixed mode, so stage through a
  // temporary device buffer
  double* tmp = nullptr;
  if (hipMalloc((void**)&tmp, sizeof(double) * c->lstride) != hipSuccess)
    return fail(CELL_E_NOMEM, "device allocation failed");
  hipLaunchKernelGGL(k_sub_mean, dim3(1024), dim3(256), 0, c->stream, u, (const double*)mean, c->n, c->d, tmp);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(u_out, tmp, sizeof(double) * c->lstride, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) return fail(CELL_E_DEVICE, hipGetErrorString(e));
  return CELL_OK;
}

cell_status cell_profile(cell_t c, int enable) {
  if (!c) return fail(CELL_E_ARG, "null argument");
  DevGuard dg(c->dev);
  HIPCHK(hipStreamSynchronize(c->stream));
  if (enable && c->ev.empty()) {
    c->ev.resize(2 * PROF_PAIRS);
    c->ev_kind.resize(PROF_PAIRS);
    for (auto& e : c->ev) HIPCHK(hipEventCreate(&e));
  }
  if (c->prof) STCHK(prof_collect(c));
  c->prof = enable != 0;
  for (int k = 0; k < CELL_NKERNEL; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_cnt[k] = 0;
  }
  return CELL_OK;
}

cell_status cell_profile_read(cell_t c, double* ms_out, long long* launches_out) {
  if (!c || !ms_out || !launches_out) return fail(CELL_E_ARG, "null argument");
  DevGuard dg(c->dev);
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->prof) STCHK(prof_collect(c));
  for (int k = 0; k < CELL_NKERNEL; ++k) {
    ms_out[k] = c->prof_ms[k];
    launches_out[k] = c->prof_cnt[k];
  }
  return CELL_OK;
}

cell_status cell_energy_matrix(cell_t c, double* C_out) {
  if (!c || !C_out) return fail(CELL_E_ARG, "null argument");
  if (!c->solved) return fail(CELL_E_STATE, "no solution available");
  for (int i = 0; i < c->nload_solved * c->nload_solved; ++i) C_out[i] = c->energy[i];
  return CELL_OK;
}

cell_status cell_get_residual(cell_t c, int load, double* r_out, int on_device) {
  if (!c || !r_out) return fail(CELL_E_ARG, "null argument");
  if (!c->solved) return fail(CELL_E_STATE, "no solution available");
  if (load < 0 || load >= c->nload_solved) return fail(CELL_E_ARG, "load index out of range");
  DevGuard dg(c->dev);
  const long long off = (long long)load * c->lstride;
  if (c->precision == CELL_MIXED) {
    std::vector<float> h(c->lstride);
    HIPCHK(hipMemcpyAsync(h.data(), c->f32.r + off, sizeof(float) * c->lstride, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (on_device) {
      std::vector<double> d(h.begin(), h.end());
      HIPCHK(hipMemcpy(r_out, d.data(), sizeof(double) * c->lstride, hipMemcpyHostToDevice));
    } else {
      for (long long i = 0; i < c->lstride; ++i) r_out[i] = (double)h[i];
    }
  } else {
    HIPCHK(hipMemcpyAsync(r_out, c->f64.r + off, sizeof(double) * c->lstride,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  return CELL_OK;
}

cell_status cell_reference_medium(cell_t c, double* lam0, double* mu0) {
  if (!c || !lam0 || !mu0) return fail(CELL_E_ARG, "null argument");
  if (!c->have_mat) return fail(CELL_E_STATE, "cell_set_material has not been called");
  *lam0 = c->lam0;
  *mu0 = c->mu0;
  return CELL_OK;
}

}  // extern "C"

namespace {

template <typename T>
cell_status upload_field(cell_s* c, T* dst, const double* src) {
  std::vector<T> h(c->lstride);
  for (long long i = 0; i < c->lstride; ++i) h[i] = (T)src[i];
  HIPCHK(hipMemcpyAsync(dst, h.data(), sizeof(T) * c->lstride, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CELL_OK;
}

template <typename T>
cell_status download_field(cell_s* c, double* dst, const T* src) {
  std::vector<T> h(c->lstride);
  HIPCHK(hipMemcpyAsync(h.data(), src, sizeof(T) * c->lstride, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (long long i = 0; i < c->lstride; ++i) dst[i] = (double)h[i];
  return CELL_OK;
}

void diag_state(cell_s* c) {
  for (int l = 0; l < c->max_loads; ++l) {
    LoadState& S = c->st_h[l];
    std::memset(&S, 0, sizeof(S));
    S.state = l == 0 ? ST_ACTIVE : ST_IDLE;
    S.thr = -1.0;
    S.maxit = 1 << 30;
    S.first = 1;
  }
}

template <typename T>
cell_status apply_operator(cell_s* c, const double* u, double* q) {
  STCHK(ensure_fields<T>(c));
  Fields<T>& F = fields<T>(c);
  c->solved = c->solved_unit = false;
  STCHK(upload_field<T>(c, F.p, u));
  diag_state(c);
  HIPCHK(hipMemcpyAsync(c->st, c->st_h, sizeof(LoadState) * c->max_loads, hipMemcpyHostToDevice, c->stream));
  for (int l = 0; l < 6; ++l)
    for (int i = 0; i < 6; ++i) c->eps_v[l][i] = 0.0;
  KArgs<T> ka = kargs<T>(c, 0, F.p, F.q, mat_of<T>(c), 1);
  HIPCHK(launch_stencil<T>(ka, c->stream));
  return download_field<T>(c, q, F.q);
}

template <typename T>
cell_status apply_precond(cell_s* c, const double* r, double* z) {
  STCHK(ensure_fields<T>(c));
  Fields<T>& F = fields<T>(c);
  c->solved = c->solved_unit = false;
  STCHK(upload_field<T>(c, F.r, r));
  HIPCHK(hipMemsetAsync(F.p, 0, sizeof(T) * c->lstride, c->stream));
  HIPCHK(hipMemsetAsync(F.q, 0, sizeof(T) * c->lstride, c->stream));
  diag_state(c);
  HIPCHK(hipMemcpyAsync(c->st, c->st_h, sizeof(LoadState) * c->max_loads, hipMemcpyHostToDevice, c->stream));
  STCHK(iteration<T>(c, 1, false));
  return download_field<T>(c, z, F.p);
}

}  // namespace

extern "C" {

cell_status cell_apply_operator(cell_t c, int precision, const double* u, double* q_out) {
  if (!c || !u || !q_out) return fail(CELL_E_ARG, "null argument");
  if (!c->have_mat) return fail(CELL_E_STATE, "cell_set_material has not been called");
  DevGuard dg(c->dev);
  if (precision == CELL_FP64) return apply_operator<double>(c, u, q_out);
  if (precision == CELL_MIXED) return apply_operator<float>(c, u, q_out);
  return fail(CELL_E_ARG, "invalid precision");
}

cell_status cell_apply_preconditioner(cell_t c, int precision, const double* r, double* z_out) {
  if (!c || !r || !z_out) return fail(CELL_E_ARG, "null argument");
  if (!c->have_mat) return fail(CELL_E_STATE, "cell_set_material has not been called");
  DevGuard dg(c->dev);
  if (precision == CELL_FP64) return apply_precond<double>(c, r, z_out);
  if (precision == CELL_MIXED) return apply_precond<float>(c, r, z_out);
  return fail(CELL_E_ARG, "invalid precision");
}

}  // extern "C"
