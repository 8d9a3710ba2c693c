// Solver instance: device state, the PCG loop, reliable updates and the
// homogenisation, for ncell cells of one grid (see solver.h).
//
// One PCG iteration is the kernel sequence
//   K-apply (q = K p)                 -> finalize (alpha = rz / pq)
//   -> x forward pass (r -= alpha q, ||r||^2, FFT_x)       -> finalize (rr)
//   -> y pass (FFT_y)                                       [3D]
//   -> last pass (FFT, z_hat = K_ref^{-1} r_hat, r.z, inverse FFT) -> finalize (beta)
//   -> y pass (inverse FFT_y)                               [3D]
//   -> x inverse pass (inverse FFT_x, x += alpha p, p = z + beta p)
// over all slots at once, with every scalar on the device.  The host reads
// the per-slot states once per chunk of iterations; the chunk is captured
// once per solve as a HIP graph and replayed.  Mixed precision: the bulk
// runs in FP32 and the FP32 iterate is a correction to an FP64 solution;
// whenever a slot's iterated residual has dropped by DELTA since its last
// FP64 residual (or the iterated test passes), the correction is merged and
// the residual recomputed in FP64 (reliable update), batched over slots.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>

#include "solver.h"

namespace cellfft {

namespace {

thread_local std::string g_err;

#define HIPCHK(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail(CELL_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define STCHK(call)          \
  do {                       \
    cell_status s_ = (call); \
    if (s_ < 0) return s_;   \
  } while (0)

constexpr int CHUNK = 8;         // iterations between host polls
constexpr double DELTA = 0.05;   // reliable-update trigger (residual reduction)
constexpr int PROF_PAIRS = 256;  // event pairs before a forced collection

// first entry of every slot's residual history: the initial ||r||^2
__global__ void k_hist_init(double* hist, int cap, const LoadState* st, int ns) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < ns) hist[(long long)l * cap] = st[l].rr;
}

// x64[slot] += x32[slot], x32[slot] = 0 for the masked slots
__global__ void k_merge(double* x64, float* x32, long long len, const int* mask) {
  const int l = blockIdx.y;
  if (!mask[l]) return;
  double* a = x64 + (long long)l * len;
  float* b = x32 + (long long)l * len;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (long long)gridDim.x * blockDim.x) {
    a[i] += (double)b[i];
    b[i] = 0.0f;
  }
}

}  // namespace

cell_status fail(cell_status s, const std::string& m) {
  g_err = m;
  return s;
}

const char* last_error_message() { return g_err.c_str(); }

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

namespace {

RedBuf red_of(cell_s* c) { return RedBuf{c->parts, c->maxblk, c->nslot, c->hist, c->hist_cap}; }

template <typename T> Fields<T>& fields(cell_s* c);
template <> Fields<float>& fields<float>(cell_s* c) { return c->f32; }
template <> Fields<double>& fields<double>(cell_s* c) { return c->f64; }

template <typename T> const T* mat_of(cell_s* c);
template <> const float* mat_of<float>(cell_s* c) { return c->mat32; }
template <> const double* mat_of<double>(cell_s* c) { return c->mat64; }

// ------------------------------------------------------------- profiling
// Adds the elapsed times of the recorded event pairs (all complete: called
// after a stream synchronisation) and recycles the pool.
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

// brackets one kernel launch with an event pair on the instance's stream
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

// ------------------------------------------------------------- buffers
template <typename T>
cell_status ensure_fields(cell_s* c) {
  Fields<T>& F = fields<T>(c);
  if (F.ready) return CELL_OK;
  const size_t bytes = sizeof(T) * (size_t)c->lstride * c->nslot;
  T** bufs[4] = {&F.x, &F.r, &F.p, &F.q};
  for (T** b : bufs) {
    if (hipMalloc((void**)b, bytes) != hipSuccess) return fail(CELL_E_NOMEM, "device allocation of a field failed");
    HIPCHK(hipMemset(*b, 0, bytes));
  }
  const size_t sbytes = sizeof(cpx<T>) * (size_t)c->s_ls * c->nslot;
  if (hipMalloc((void**)&F.S, sbytes) != hipSuccess || hipMalloc((void**)&F.R, bytes) != hipSuccess)
    return fail(CELL_E_NOMEM, "device allocation of the spectrum failed");
  HIPCHK(hipMemset(F.S, 0, sbytes));
  if (sizeof(T) == 4 && rw_fits(c->g)) {
    const size_t eb = sizeof(float) * (size_t)rw_edge_floats(c->g) * c->nslot;
    if (hipMalloc((void**)&F.edge, eb) != hipSuccess) return fail(CELL_E_NOMEM, "device allocation of the edge rows failed");
    HIPCHK(hipMemset(F.edge, 0, eb));
  }
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
    // wavevector negation
    for (int k = 0; k <= N[a] / 2; ++k) {
      double s = std::sin(M_PI * k / N[a]), co = std::cos(M_PI * k / N[a]);
      if (2 * k == N[a]) {
        s = 1.0;
        co = 0.0;
      }
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
  if (c->d == 2) {  // unused third axis: a one-entry table keeps kernel args valid
    HIPCHK(hipMalloc((void**)&F.trig[2], sizeof(T) * 2));
    T z2[2] = {T(0), T(1)};
    HIPCHK(hipMemcpy(F.trig[2], z2, sizeof(T) * 2, hipMemcpyHostToDevice));
  }
  F.sym_lam0.assign(c->ncell, -1.0);
  F.sym_mu0.assign(c->ncell, -1.0);
  F.ready = true;
  return CELL_OK;
}

template <typename T> void free_fields(Fields<T>& F) {
  auto fr = [](void* p) {
    if (p) (void)hipFree(p);
  };
  fr(F.x);
  fr(F.r);
  fr(F.p);
  fr(F.q);
  fr(F.S);
  fr(F.R);
  fr(F.edge);
  fr(F.symtab);
  fr(F.symtabB);
  fr(F.med);
  for (int a = 0; a < 3; ++a) {
    fr(F.tw[a]);
    fr(F.trig[a]);
  }
  F = Fields<T>();
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
KArgs<T> kargs(cell_s* c, int mode, const T* u, void* out, const T* mat) {
  KArgs<T> a{};
  a.u = u;
  a.out = out;
  a.mat = mat;
  a.lstride = c->lstride;
  a.g = c->g;
  for (int l = 0; l < 6; ++l) voigt_to_tensor(c->d, c->eps_v[l], a.eps[l]);
  a.nload = c->nslot;
  a.lpc = c->lpc;
  a.mat_stride = 2 * c->n;
  a.mode = mode;
  a.st = c->st;
  a.only_load = -1;
  a.mask = nullptr;
  a.res2 = c->res2;
  a.sparts = nullptr;
  a.sbar = nullptr;
  a.negate = c->dbg_negate_q;
  if constexpr (sizeof(T) == 4) {
    // the FP32 row-wave operator (when the schedule selects it) fixes up its
    // edge rows itself unless the caller's x forward pass adds them
    a.edge = c->f32.edge;
    a.edge_stride = rw_edge_floats(c->g);
    a.edge_fused = 0;
  }
  a.red = red_of(c);
  return a;
}

// last-pass arguments for the reference medium of cell 0 (the symbol
// table carries the per-cell media)
template <typename T>
PArgs<T> make_pargs(cell_s* c, int cell) {
  Fields<T>& F = fields<T>(c);
  PArgs<T> pa{};
  pa.S = F.S;
  pa.lstrideC = c->s_ls;
  pa.zsS = c->s_zs;
  pa.nx = c->g.nx;
  pa.ny = c->g.ny;
  pa.nz = c->g.nz;
  pa.tw = F.tw[c->d - 1];
  for (int a = 0; a < 3; ++a) pa.trig[a] = F.trig[a];
  pa.lam0 = (T)c->lam0[cell];
  pa.mu0 = (T)c->mu0[cell];
  pa.w = (T)(c->d == 3 ? c->g.h[0] * c->g.h[1] * c->g.h[2] / 6.0 : c->g.h[0] * c->g.h[1] / 2.0);
  for (int a = 0; a < 3; ++a) pa.ih[a] = (T)(1.0 / c->g.h[a]);
  pa.inv_n = (T)(1.0 / (double)c->n);
  pa.nload = c->nslot;
  pa.lpc = c->lpc;
  pa.tab = nullptr;
  pa.tabB = nullptr;
  pa.tab_stride = 0;
  pa.tabB_stride = 0;
  pa.med = nullptr;
  pa.Sin = nullptr;
  pa.st = c->st;
  pa.red = red_of(c);
  return pa;
}

// 3D: (re)builds each cell's tabulated inverse symbol when its reference
// medium changed; 2D: uploads the per-cell media.  Points pa at the tables.
template <typename T>
cell_status ensure_symtab(cell_s* c, PArgs<T>& pa) {
  Fields<T>& F = fields<T>(c);
  if (c->d == 2) {
    bool changed = !F.med;
    if (!F.med) {
      if (hipMalloc((void**)&F.med, sizeof(T) * 2 * c->ncell) != hipSuccess)
        return fail(CELL_E_NOMEM, "device allocation of the reference media failed");
      F.med_h.assign(2 * c->ncell, T(0));
    }
    for (int cell = 0; cell < c->ncell; ++cell)
      if (F.sym_lam0[cell] != c->lam0[cell] || F.sym_mu0[cell] != c->mu0[cell]) {
        F.med_h[2 * cell] = (T)c->lam0[cell];
        F.med_h[2 * cell + 1] = (T)c->mu0[cell];
        F.sym_lam0[cell] = c->lam0[cell];
        F.sym_mu0[cell] = c->mu0[cell];
        changed = true;
      }
    if (changed)
      HIPCHK(hipMemcpyAsync(F.med, F.med_h.data(), sizeof(T) * 2 * c->ncell, hipMemcpyHostToDevice, c->stream));
    pa.med = F.med;
    return CELL_OK;
  }
  const long long entries = (long long)c->g.ny * c->g.nz * (c->g.nx / 2);
  const long long stride = 6 * entries, strideB = 6 * 2 * (long long)c->g.nz;
  if (!F.symtab) {
    if (hipMalloc((void**)&F.symtab, sizeof(T) * stride * c->ncell) != hipSuccess ||
        hipMalloc((void**)&F.symtabB, sizeof(T) * strideB * c->ncell) != hipSuccess)
      return fail(CELL_E_NOMEM, "device allocation of the symbol table failed");
  }
  for (int cell = 0; cell < c->ncell; ++cell) {
    if (!c->have_mat[cell]) continue;
    if (F.sym_lam0[cell] != c->lam0[cell] || F.sym_mu0[cell] != c->mu0[cell]) {
      PArgs<T> pc = make_pargs<T>(c, cell);
      HIPCHK(launch_symtab<T>(pc, F.symtab + cell * stride, F.symtabB + cell * strideB, c->stream));
      F.sym_lam0[cell] = c->lam0[cell];
      F.sym_mu0[cell] = c->mu0[cell];
    }
  }
  pa.tab = F.symtab;
  pa.tabB = F.symtabB;
  pa.tab_stride = stride;
  pa.tabB_stride = strideB;
  return CELL_OK;
}

template <typename T>
XArgs<T> xargs(cell_s* c) {
  Fields<T>& F = fields<T>(c);
  XArgs<T> xa{};
  xa.r = F.r;
  xa.q = F.q;
  xa.R = F.R;
  xa.S = F.S;
  xa.x = F.x;
  xa.p = F.p;
  xa.lstride = c->lstride;
  xa.nrows = (int)(c->lstride / c->g.nx);
  xa.ny = c->g.ny;
  xa.zsS = c->s_zs;
  xa.lsS = c->s_ls;
  xa.tw = F.tw[0];
  xa.mode = 0;
  xa.mask = nullptr;
  xa.st = c->st;
  xa.red = red_of(c);
  xa.qmean = c->op == 2 ? c->sr_mean : nullptr;
  xa.comp_rows = c->g.ny * (c->d == 3 ? c->g.nz : 1);
  if constexpr (sizeof(T) == 4) {
    if (c->f32.edge && c->op == 0 && stencil_effective_tile(c->g, false, c->sched.st_tile) == ST_RW) {
      xa.edge = c->f32.edge;
      xa.edge_stride = rw_edge_floats(c->g);
      xa.edge_rows = rw_rows(c->g.nx);
    }
  }
  return xa;
}

// neo-Hookean operator arguments (state u in the arithmetic type)
template <typename T> const T* hy_state(cell_s* c);
template <> const float* hy_state<float>(cell_s* c) { return c->hy_u32; }
template <> const double* hy_state<double>(cell_s* c) { return c->hy_u; }

template <typename T> const T* fbar_of(cell_s* c);
template <> const float* fbar_of<float>(cell_s* c) { return c->hy_F32; }
template <> const double* fbar_of<double>(cell_s* c) { return c->hy_F; }

template <typename T>
HyArgs<T> hyargs(cell_s* c) {
  HyArgs<T> h{};
  h.u = hy_state<T>(c);
  h.mat = mat_of<T>(c);
  h.mat_stride = 2 * c->n;
  h.lstride = c->lstride;
  h.g = c->g;
  h.Fbar = c->hy_F;
  h.FbarT = fbar_of<T>(c);
  h.nload = c->nslot;
  h.lpc = c->lpc;
  h.st = c->st;
  h.mask = nullptr;
  h.res2 = c->res2;
  h.vparts = c->hy_vparts;
  h.vals = c->hy_vals;
  h.red = red_of(c);
  return h;
}

// surrogate stencil operator arguments (stencil copy in the arithmetic type)
template <typename T> const T* sr_stencil(cell_s* c);
template <> const float* sr_stencil<float>(cell_s* c) { return c->sr32; }
template <> const double* sr_stencil<double>(cell_s* c) { return c->sr64; }

template <typename T>
SArgs<T> sargs(cell_s* c) {
  SArgs<T> a{};
  a.s = sr_stencil<T>(c);
  a.lstride = c->lstride;
  a.g = c->g;
  a.nslot = c->nslot;
  a.st = c->st;
  a.cparts = c->sr_parts;
  a.mean = c->sr_mean;
  a.red = red_of(c);
  return a;
}

// one PCG iteration over all slots (or the initial preconditioning if !kapply)
template <typename T>
cell_status iteration(cell_s* c, bool kapply) {
  Fields<T>& F = fields<T>(c);
  hipStream_t s = c->stream;
  const int ns = c->nslot;
  if (kapply) {
    ProfScope ps(c, CELL_K_APPLY);
    if (c->op == 1) {
      HyArgs<T> ha = hyargs<T>(c);
      ha.p = F.p;
      ha.out = F.q;
      HIPCHK(launch_hyper_tangent<T>(ha, s));
    } else if (c->op == 2) {
      SArgs<T> sa = sargs<T>(c);
      sa.p = F.p;
      sa.out = F.q;
      HIPCHK(launch_sr_apply<T>(sa, s));
    } else {
      KArgs<T> ka = kargs<T>(c, 0, F.p, F.q, mat_of<T>(c));
      ka.edge_fused = 1;  // the x forward pass below adds the edge rows
      HIPCHK(launch_stencil<T>(ka, c->sched, s));
    }
  }
  XArgs<T> xa = xargs<T>(c);
  if (kapply) {
    // R -= alpha FFT_x(q), ||r||^2
    {
      ProfScope ps(c, CELL_K_XFWD);
      HIPCHK(launch_xfwd<T>(xa, c->g.nx, ns, c->sched, s));
    }
    HIPCHK(launch_finalize(xa.red, c->st, c->res2, RED_RR,
                           xpass_blocks(c->g.nx, xa.nrows, sizeof(T) == 8, c->sched), ns, -1, nullptr, s));
  } else {
    // first preconditioning: R = FFT_x(r) of the active slots
    xa.mode = 1;
    ProfScope ps(c, CELL_K_XFWD);
    HIPCHK(launch_xfwd<T>(xa, c->g.nx, ns, c->sched, s));
  }
  YArgs<T> ya{};
  ya.S = F.S;
  ya.Sin = F.R;
  ya.lstrideC = c->lstride / 2;
  ya.zsS = c->s_zs;
  ya.lsS = c->s_ls;
  ya.nx = c->g.nx;
  ya.ny = c->g.ny;
  ya.nz = c->g.nz;
  ya.ncomp = c->d;
  ya.tw = F.tw[1];
  ya.st = c->st;
  PArgs<T> pa = make_pargs<T>(c, 0);
  STCHK(ensure_symtab<T>(c, pa));
  if (c->d == 2) pa.Sin = F.R;  // 2D: the last pass follows the x pass
  if (c->d == 3) {
    ProfScope ps(c, CELL_K_YFWD);
    HIPCHK(launch_ypass<T>(ya, false, ns, c->sched, s));
  }
  {
    ProfScope ps(c, CELL_K_LAST);
    HIPCHK(launch_last<T>(pa, c->d, ns, c->sched, s));
  }
  HIPCHK(launch_finalize(pa.red, c->st, c->res2, RED_RZ,
                         last_pass_blocks(c->d, c->g.nx, c->g.ny, sizeof(T) == 8, c->sched), ns, -1, nullptr, s));
  if (c->d == 3) {
    ProfScope ps(c, CELL_K_YINV);
    HIPCHK(launch_ypass<T>(ya, true, ns, c->sched, s));
  }
  {
    xa.mode = 0;
    ProfScope ps(c, CELL_K_XINV);
    HIPCHK(launch_xinv<T>(xa, c->g.nx, ns, c->sched, s));
  }
  return CELL_OK;
}

// r = f - K u in FP64 for the masked slots (mask == nullptr: all); the
// launch also sums |s| sigma per slot (mean stresses); ||r||^2 -> res2_h
template <typename T>
cell_status residual(cell_s* c, const double* u, const int* mask) {
  Fields<T>& F = fields<T>(c);
  if (c->op == 1) {
    // Newton step: r = f(u) - K_T(u) du
    HyArgs<double> ha = hyargs<double>(c);
    ha.p = u;
    ha.rhs = c->hy_rhs;
    ha.out = F.r;
    ha.mask = mask;
    {
      ProfScope ps(c, CELL_K_RESIDUAL);
      if (u)
        HIPCHK(launch_hyper_tangent_residual(ha, sizeof(T) == 4, c->stream));
      else  // du = 0: r = f
        HIPCHK(launch_rhs_residual(c->hy_rhs, F.r, sizeof(T) == 4, c->lstride, (long long)c->d * c->n, c->nslot, mask,
                                   red_of(c), c->st, c->res2, c->stream));
    }
    HIPCHK(hipMemcpyAsync(c->res2_h, c->res2, sizeof(double) * c->nslot, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return CELL_OK;
  }
  if (c->op == 2) {
    // surrogate: r = P (f - Kt u) (f exact, computed at the start of the solve)
    {
      ProfScope ps(c, CELL_K_RESIDUAL);
      if (u) {
        SArgs<double> sa = sargs<double>(c);
        sa.p = u;
        sa.out = F.r;
        sa.rhs = c->sr_rhs;
        sa.mask = mask;
        HIPCHK(launch_sr_residual(sa, sizeof(T) == 4, c->res2, c->stream));
      } else {
        HIPCHK(launch_rhs_residual(c->sr_rhs, F.r, sizeof(T) == 4, c->lstride, (long long)c->d * c->n, c->nslot,
                                   mask, red_of(c), c->st, c->res2, c->stream));
      }
    }
    HIPCHK(hipMemcpyAsync(c->res2_h, c->res2, sizeof(double) * c->nslot, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return CELL_OK;
  }
  KArgs<double> ka = kargs<double>(c, 1, u, nullptr, c->mat64);
  ka.mask = mask;
  ka.sparts = c->sparts;
  ka.sbar = c->sbar;
  {
    ProfScope ps(c, CELL_K_RESIDUAL);
    if (sizeof(T) == 4) {
      HIPCHK(launch_residual_mixed(ka, reinterpret_cast<float*>(F.r), c->sched, c->stream));
    } else {
      ka.out = F.r;
      HIPCHK(launch_stencil<double>(ka, c->sched, c->stream));
    }
  }
  HIPCHK(hipMemcpyAsync(c->res2_h, c->res2, sizeof(double) * c->nslot, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CELL_OK;
}

template <typename T>
cell_status begin_t(SolveRun& R) {
  cell_s* c = R.c;
  STCHK(ensure_fields<T>(c));
  Fields<T>& F = fields<T>(c);
  hipStream_t s = c->stream;
  const int ns = c->nslot;
  const size_t fb = sizeof(T) * (size_t)c->lstride * ns;
  HIPCHK(hipMemsetAsync(F.x, 0, fb, s));
  HIPCHK(hipMemsetAsync(F.p, 0, fb, s));
  HIPCHK(hipMemsetAsync(F.q, 0, fb, s));
  if (c->precision == CELL_MIXED) HIPCHK(hipMemsetAsync(c->x64, 0, sizeof(double) * (size_t)c->lstride * ns, s));
  if (c->op == 2) {
    // the exact load vectors f = -B^T D eps_bar (FP64) for the surrogate path
    KArgs<double> ka = kargs<double>(c, 1, nullptr, nullptr, c->mat64);
    ka.out = c->sr_rhs;
    ProfScope ps(c, CELL_K_RESIDUAL);
    HIPCHK(launch_stencil<double>(ka, c->sched, s));
  }
  // load vectors f = -B^T D eps_bar and ||f||^2 for every slot
  STCHK(residual<T>(c, nullptr, nullptr));
  R.fn2.assign(ns, 0.0);
  R.rr_ru.assign(ns, 0.0);
  R.fin.assign(ns, 1);
  R.nref.assign(ns, 0);
  R.active.assign(ns, 0);
  double emax = 0.0;
  for (int l = 0; l < R.nload; ++l)
    for (int i = 0; i < c->nv; ++i) emax = std::max(emax, std::fabs(c->eps_v[l][i]));
  const double hmin = std::min(c->g.h[0], std::min(c->g.h[1], c->d == 3 ? c->g.h[2] : c->g.h[1]));
  const double wvol = c->d == 3 ? c->g.h[0] * c->g.h[1] * c->g.h[2] : c->g.h[0] * c->g.h[1];
  R.done = true;
  for (int l = 0; l < ns; ++l) {
    LoadState& S = c->st_h[l];
    std::memset(&S, 0, sizeof(S));
    S.state = ST_IDLE;
    S.maxit = c->max_iter;
    S.first = 1;
    S.negok = c->op == 1;
    c->negcurv[l] = 0;
    const int cell = l / c->lpc, j = l % c->lpc;
    if (j >= R.nload) continue;
    R.active[l] = 1;
    R.fn2[l] = c->res2_h[l];
    R.rr_ru[l] = R.fn2[l];
    S.rr = R.fn2[l];
    S.thr = c->tol * c->tol * R.fn2[l];
    // scale of the load vector without cancellation (homogeneous-cell test)
    const double fscale = std::sqrt((double)c->n) * wvol * c->maxmod[cell] * emax / hmin;
    if (std::sqrt(R.fn2[l]) <= 1e-13 * fscale) {  // homogeneous: f = 0 up to round-off, u = 0
      S.state = ST_DONE;
    } else {
      S.state = ST_ACTIVE;
      R.fin[l] = 0;
      R.done = false;
    }
  }
  // initial guesses (linear solves with the exact operator): x = x0 and
  // r = f - K x0 in FP64 for the active slots that have one; a slot whose
  // guess already passes the test is final with 0 iterations
  if (c->op == 0 && c->x0 && !R.done) {
    bool any = false;
    for (int l = 0; l < ns; ++l) {
      c->mask_h[l] = 0;
      const int j = l % c->lpc;
      if (R.fin[l] || !c->x0_set[j]) continue;
      double* dst = (sizeof(T) == 4 ? c->x64 : reinterpret_cast<double*>(F.x)) + (long long)l * c->lstride;
      HIPCHK(hipMemcpyAsync(dst, c->x0 + (long long)j * c->lstride, sizeof(double) * c->lstride,
                            hipMemcpyDeviceToDevice, s));
      c->mask_h[l] = 1;
      any = true;
    }
    if (any) {
      HIPCHK(hipMemcpyAsync(c->mask, c->mask_h, sizeof(int) * ns, hipMemcpyHostToDevice, s));
      const double* u64 = sizeof(T) == 4 ? c->x64 : reinterpret_cast<const double*>(F.x);
      STCHK(residual<T>(c, u64, c->mask));
      R.done = true;
      for (int l = 0; l < ns; ++l) {
        LoadState& S = c->st_h[l];
        if (c->mask_h[l]) {
          const double rt = c->res2_h[l];
          if (!(rt == rt) || rt > 1e300) return fail(CELL_E_ARG, "non-finite residual of the initial guess of load " +
                                                                     std::to_string(l % c->lpc));
          S.rr = rt;
          R.rr_ru[l] = rt;
          R.nref[l] = 1;
          if (rt <= S.thr) {
            S.state = ST_DONE;
            R.fin[l] = 1;
          }
        }
        if (!R.fin[l]) R.done = false;
      }
    }
  }
  R.best.assign(ns, 0.0);
  R.best_it.assign(ns, 0);
  R.restarts.assign(ns, 0);
  R.stag_pending.assign(ns, 0);
  R.stagnated.assign(ns, 0);
  for (int l = 0; l < ns; ++l) R.best[l] = c->st_h[l].rr;
  HIPCHK(hipMemcpyAsync(c->st, c->st_h, sizeof(LoadState) * ns, hipMemcpyHostToDevice, s));
  // residual history: entry 0 is the initial ||r||^2 of every slot
  hipLaunchKernelGGL(k_hist_init, dim3((ns + NT - 1) / NT), dim3(NT), 0, s, c->hist, c->hist_cap,
                     (const LoadState*)c->st, ns);
  HIPCHK(hipGetLastError());
  for (int l = 0; l < ns; ++l) {
    c->hist_n[l] = 0;
    c->hist_fn2[l] = R.fn2[l];
  }
  STCHK(iteration<T>(c, false));
  return CELL_OK;
}

// the CHUNK iterations of one launch on the instance's stream (eager, or
// into a capture the caller has opened on that stream)
template <typename T>
cell_status chunk_t(SolveRun& R) {
  for (int i = 0; i < CHUNK; ++i) STCHK(iteration<T>(R.c, true));
  return CELL_OK;
}

// queues CHUNK iterations and the copy of the slot states to the host
template <typename T>
cell_status launch_t(SolveRun& R) {
  cell_s* c = R.c;
  hipStream_t s = c->stream;
  // per-launch event timing needs eager launches (events recorded inside a
  // captured graph carry no timestamps)
  if (!solve_graphs(R)) {
    STCHK(chunk_t<T>(R));
  } else {
    if (!R.gexec) {  // capture once per solve: the launch arguments are fixed for its duration
      hipGraph_t graph = nullptr;
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      cell_status st = chunk_t<T>(R);
      hipError_t e = hipStreamEndCapture(s, &graph);
      if (st < 0) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
      }
      if (e != hipSuccess) return fail(CELL_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&R.gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) {
        R.gexec = nullptr;
        return fail(CELL_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      }
    }
    HIPCHK(hipGraphLaunch(R.gexec, s));
  }
  return solve_copy_states(R);
}

// after the stream has drained: reliable updates (FP64 residual, plus the
// merge of the FP32 correction in mixed precision) of the slots that need
// one, batched in one masked launch; sets R.done when every slot is final
template <typename T>
cell_status poll_t(SolveRun& R) {
  cell_s* c = R.c;
  Fields<T>& F = fields<T>(c);
  const bool mixed = sizeof(T) == 4;
  hipStream_t s = c->stream;
  const int ns = c->nslot;
  if (c->prof) STCHK(prof_collect(c));
  bool any = false;
  for (int l = 0; l < ns; ++l) {
    c->mask_h[l] = 0;
    if (R.fin[l]) continue;
    LoadState& S = c->st_h[l];
    if (S.state == ST_BREAKDOWN) {
      R.fin[l] = 1;
      R.result = fail(CELL_E_BREAKDOWN, "CG breakdown in slot " + std::to_string(l));
      continue;
    }
    // CONVERGED: the converging iteration has completed (its operator
    // finalisation, which marks DONE, has not run yet); NEGCURV: stopped on
    // p.Kp <= 0 with the previous iterate
    const bool finished = S.state == ST_DONE || S.state == ST_CONVERGED || S.state == ST_NEGCURV;
    // stagnation: stag_window iterations without halving the smallest
    // ||r||^2 seen so far; the slot gets an FP64 residual refresh, then a
    // restart (the first time) or the end of its iteration (the second)
    if (!finished && S.state == ST_ACTIVE && c->stag_window > 0) {
      if (S.rr < 0.5 * R.best[l]) {
        R.best[l] = S.rr;
        R.best_it[l] = S.iters;
      } else if (S.iters - R.best_it[l] >= c->stag_window) {
        R.stag_pending[l] = 1;
      }
    }
    if (finished || R.stag_pending[l] || (mixed && S.state == ST_ACTIVE && S.rr < DELTA * DELTA * R.rr_ru[l])) {
      c->mask_h[l] = 1;
      any = true;
    }
  }
  if (any) {
    HIPCHK(hipMemcpyAsync(c->mask, c->mask_h, sizeof(int) * ns, hipMemcpyHostToDevice, s));
    const double* u64 = reinterpret_cast<const double*>(F.x);
    if (mixed) {
      ProfScope ps(c, CELL_K_MERGE);
      hipLaunchKernelGGL(k_merge, dim3(256, ns), dim3(256), 0, s, c->x64, reinterpret_cast<float*>(F.x), c->lstride,
                         (const int*)c->mask);
      HIPCHK(hipGetLastError());
      u64 = c->x64;
    }
    STCHK(residual<T>(c, u64, c->mask));
    {
      // the iteration keeps r transformed along x: refresh it
      XArgs<T> xa = xargs<T>(c);
      xa.mode = 1;
      xa.mask = c->mask;
      ProfScope ps(c, CELL_K_XFWD);
      HIPCHK(launch_xfwd<T>(xa, c->g.nx, ns, c->sched, s));
    }
    for (int l = 0; l < ns; ++l) {
      if (!c->mask_h[l]) continue;
      LoadState& S = c->st_h[l];
      const bool finished = S.state == ST_DONE || S.state == ST_CONVERGED;
      if (S.state == ST_NEGCURV) {
        c->negcurv[l] = S.iters;  // operator applications, the last one with p.Kp <= 0
        R.fin[l] = 1;
        S.state = ST_DONE;
        S.rr = c->res2_h[l];
        R.rr_ru[l] = S.rr;
        continue;
      }
      const double rt = c->res2_h[l];
      R.rr_ru[l] = rt;
      R.nref[l] += 1;
      if (!(rt == rt)) {
        R.fin[l] = 1;
        S.state = ST_DONE;
        R.result = fail(CELL_E_BREAKDOWN, "non-finite residual in slot " + std::to_string(l));
        continue;
      }
      const bool stag = R.stag_pending[l] != 0;
      R.stag_pending[l] = 0;
      if (rt <= S.thr || (finished && S.maxit_hit) || S.iters >= c->max_iter) {
        R.fin[l] = 1;
        S.state = ST_DONE;
      } else if (stag && R.restarts[l] > 0) {
        // stagnated again after a restart: the iterate stays as it is
        R.fin[l] = 1;
        S.state = ST_DONE;
        R.stagnated[l] = 1;
      } else {
        S.state = ST_ACTIVE;
        if (stag) {
          // restart: the next direction update takes beta = 0 (p = z of
          // the refreshed residual); progress is measured from here
          R.restarts[l] += 1;
          S.first = 1;
          R.best[l] = rt;
          R.best_it[l] = S.iters;
        }
      }
      S.rr = rt;
    }
    HIPCHK(hipMemcpyAsync(c->st, c->st_h, sizeof(LoadState) * ns, hipMemcpyHostToDevice, s));
  }
  R.done = true;
  for (int l = 0; l < ns; ++l)
    if (!R.fin[l]) R.done = false;
  return CELL_OK;
}

cell_status end_t(SolveRun& R) {
  cell_s* c = R.c;
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->prof) STCHK(prof_collect(c));
  if (R.gexec) {
    (void)hipGraphExecDestroy(R.gexec);
    R.gexec = nullptr;
  }
  bool all_conv = true;
  for (int l = 0; l < c->nslot; ++l) {
    c->hist_n[l] = R.active[l] ? std::min(c->st_h[l].iters + 1, c->hist_cap) : 0;
    if (!R.active[l]) continue;
    const double rel = (R.fn2[l] > 0 && R.nref[l] > 0) ? std::sqrt(R.rr_ru[l] / R.fn2[l]) : 0.0;
    if (R.infos) {
      cell_info& I = R.infos[l / c->lpc];
      const int j = l % c->lpc;
      I.iters[j] = c->st_h[l].iters;
      I.refinements[j] = R.nref[l];
      I.relres[j] = rel;
      I.nload = R.nload;
    }
    if (rel > c->tol) all_conv = false;
  }
  if (R.result < 0) return R.result;
  if (all_conv) return CELL_OK;
  std::string msg;
  for (int l = 0; l < c->nslot; ++l)
    if (R.active[l] && R.stagnated[l])
      msg += (msg.empty() ? "CG stagnated (no halving of ||r||^2 in " + std::to_string(c->stag_window) +
                                " iterations, also after a restart) in slot "
                          : ", ") +
             std::to_string(l);
  if (!msg.empty()) return fail(CELL_NOT_CONVERGED, msg);
  return CELL_NOT_CONVERGED;
}

// C* (energy form) and mean stresses of every cell from the final
// residuals and stress sums left by the last FP64 residual of every slot
cell_status homogenize(cell_s* c, int nload) {
  HArgs h{};
  h.u = c->precision == CELL_MIXED ? c->x64 : c->f64.x;
  h.mat = c->mat64;
  h.E = c->E64;
  h.lstride = c->lstride;
  h.g = c->g;
  for (int l = 0; l < 6; ++l) voigt_to_tensor(c->d, c->eps_v[l], h.eps[l]);
  h.nload = nload;
  h.lpc = c->lpc;
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
    HIPCHK(launch_homog(h, c->ncell, c->stream));
  }
  const int nval = nload * nload + nload * c->nv;
  c->homog.assign((size_t)nval * c->ncell, 0.0);
  HIPCHK(hipMemcpyAsync(c->homog.data(), c->hres, sizeof(double) * nval * c->ncell, hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->prof) STCHK(prof_collect(c));
  return CELL_OK;
}

}  // namespace

void apply_cached_schedule(cell_s* c);

// =================================================================== instance
void instance_destroy(cell_s* c) {
  if (!c) return;
  DevGuard dg(c->dev);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  auto fr = [](void* p) {
    if (p) (void)hipFree(p);
  };
  fr(c->mat64);
  fr(c->mat32);
  fr(c->E64);
  free_fields(c->f32);
  free_fields(c->f64);
  fr(c->x64);
  fr(c->x0);
  fr(c->st);
  fr(c->parts);
  fr(c->res2);
  fr(c->sparts);
  fr(c->sbar);
  fr(c->mask);
  fr(c->hparts);
  fr(c->hres);
  fr(c->grad);
  fr(c->hist);
  fr(c->scratch);
  fr(c->hy_u);
  fr(c->hy_u32);
  fr(c->hy_ut);
  fr(c->hy_rhs);
  fr(c->hy_F);
  fr(c->hy_F32);
  fr(c->sr64);
  fr(c->sr32);
  fr(c->sr_rhs);
  fr(c->sr_parts);
  fr(c->sr_mean);
  fr(c->hy_t);
  fr(c->hy_vparts);
  fr(c->hy_vals);
  if (c->hy_vals_h) (void)hipHostFree(c->hy_vals_h);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->st_h) (void)hipHostFree(c->st_h);
  if (c->res2_h) (void)hipHostFree(c->res2_h);
  if (c->mask_h) (void)hipHostFree(c->mask_h);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

cell_status instance_create(const cell_config* cfg, int ncell, hipStream_t shared_stream, cell_s** out) {
  if (!cfg || !out) return fail(CELL_E_ARG, "null argument");
  *out = nullptr;
  if (ncell < 1) return fail(CELL_E_ARG, "ncell must be positive");
  if (cfg->dim != 2 && cfg->dim != 3) return fail(CELL_E_ARG, "dim must be 2 or 3");
  for (int a = 0; a < cfg->dim; ++a) {
    if (cfg->n[a] < 1) return fail(CELL_E_ARG, "grid sizes must be positive");
    if (!fft_size_ok(cfg->n[a]))
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
  const char* zp = std::getenv("CELLFFT_ZPAD");
  const long long zpad = zp ? std::atoll(zp) : 32;  // complex values
  if (zpad < 0 || zpad > (1 << 20)) return fail(CELL_E_ARG, "CELLFFT_ZPAD out of range");
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
  if (c->d == 3) {
    // pad each (component, z) plane of the spectrum: the z pass reads one
    // row segment per plane, and unpadded planes of a power-of-two size
    // would put all of them on the same memory channels
    c->s_zs = (long long)c->g.ny * (c->g.nx / 2) + zpad;
    c->s_ls = 3LL * c->g.nz * c->s_zs;
  } else {
    c->s_zs = (long long)c->g.ny * (c->g.nx / 2);
    c->s_ls = c->lstride / 2;
  }
  c->precision = cfg->precision;
  c->tol = cfg->tol > 0.0 ? cfg->tol : (cfg->precision == CELL_MIXED ? 1e-6 : 1e-10);
  c->max_iter = cfg->max_iter > 0 ? cfg->max_iter : 10000;
  c->lpc = cfg->max_loads > 0 ? cfg->max_loads : nv;
  c->ncell = ncell;
  c->nslot = ncell * c->lpc;
  const char* ge = std::getenv("CELLFFT_GRAPHS");
  c->use_graphs = !(ge && ge[0] == '0');
  // debugging aid for the failure path: the linear K-apply returns -K p, so
  // the first p.Kp is negative and every solve ends in CELL_E_BREAKDOWN
  const char* nq = std::getenv("CELLFFT_DEBUG_NEGATE_Q");
  c->dbg_negate_q = (nq && nq[0] == '1') ? 1 : 0;
  const char* sw = std::getenv("CELLFFT_STAG_WINDOW");
  if (sw && sw[0]) c->stag_window = std::max(0, std::atoi(sw));
  c->have_mat.assign(ncell, 0);
  c->x0_set.assign(c->lpc, 0);
  c->lam0.assign(ncell, 0.0);
  c->mu0.assign(ncell, 0.0);
  c->maxmod.assign(ncell, 0.0);
  auto bail = [&](cell_status s) {
    instance_destroy(c);
    return s;
  };
  if (shared_stream) {
    c->stream = shared_stream;
  } else if (cfg->stream) {
    c->stream = (hipStream_t)cfg->stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) return bail(fail(CELL_E_DEVICE, "hipStreamCreate failed"));
    c->own_stream = true;
  }
  // reduction buffers sized for the largest grid of any reducing kernel
  // under any schedule
  const int mb = max_reduction_blocks(c->g);
  c->maxblk = mb;
  const int ns = c->nslot;
  auto dmalloc = [&](void** p, size_t bytes) -> bool { return hipMalloc(p, bytes) == hipSuccess; };
  if (!dmalloc((void**)&c->parts, sizeof(double) * (size_t)RED_NSLOT * ns * mb) ||
      !dmalloc((void**)&c->st, sizeof(LoadState) * ns) || !dmalloc((void**)&c->res2, sizeof(double) * ns) ||
      !dmalloc((void**)&c->sparts, sizeof(double) * 6 * (size_t)ns * mb) ||
      !dmalloc((void**)&c->sbar, sizeof(double) * 6 * ns) || !dmalloc((void**)&c->mask, sizeof(int) * ns) ||
      !dmalloc((void**)&c->mat64, sizeof(double) * 2 * c->n * ncell) ||
      !dmalloc((void**)&c->mat32, sizeof(float) * 2 * c->n * ncell) ||
      !dmalloc((void**)&c->E64, sizeof(double) * c->n * ncell) || !dmalloc((void**)&c->grad, sizeof(double) * c->n) ||
      !dmalloc((void**)&c->scratch, sizeof(double) * 64 * 1024))
    return bail(fail(CELL_E_NOMEM, "device allocation failed"));
  c->hist_cap = std::min(c->max_iter + 1, 4096);
  if (!dmalloc((void**)&c->hist, sizeof(double) * (size_t)c->hist_cap * ns))
    return bail(fail(CELL_E_NOMEM, "device allocation failed"));
  c->hist_n.assign(ns, 0);
  c->hist_fn2.assign(ns, 0.0);
  c->hblk = homog_blocks(c->g);
  const int nvalmax = c->lpc * c->lpc + c->lpc * nv;
  if (!dmalloc((void**)&c->hparts, sizeof(double) * (size_t)c->lpc * c->lpc * c->hblk * ncell) ||
      !dmalloc((void**)&c->hres, sizeof(double) * (size_t)nvalmax * ncell))
    return bail(fail(CELL_E_NOMEM, "device allocation failed"));
  if (c->precision == CELL_MIXED && !dmalloc((void**)&c->x64, sizeof(double) * (size_t)c->lstride * ns))
    return bail(fail(CELL_E_NOMEM, "device allocation failed"));
  if (hipHostMalloc((void**)&c->st_h, sizeof(LoadState) * ns) != hipSuccess ||
      hipHostMalloc((void**)&c->res2_h, sizeof(double) * ns) != hipSuccess ||
      hipHostMalloc((void**)&c->mask_h, sizeof(int) * ns) != hipSuccess)
    return bail(fail(CELL_E_NOMEM, "pinned host allocation failed"));
  c->negcurv.assign(ns, 0);
  if (hipMemset(c->st, 0, sizeof(LoadState) * ns) != hipSuccess ||
      hipMemset(c->mask, 0, sizeof(int) * ns) != hipSuccess)
    return bail(fail(CELL_E_DEVICE, "hipMemset failed"));
  cell_status st = c->precision == CELL_MIXED ? ensure_fields<float>(c) : ensure_fields<double>(c);
  if (st < 0) return bail(st);
  apply_cached_schedule(c);
  *out = c;
  return CELL_OK;
}

namespace {

// Material setup on the device (Lame parameters of Sec. 6.3 from (E, nu)).
// k_mat_check: validity and the reference-medium extremes, one partial row
// per block (MAT_NP values: min/max bulk modulus, min/max shear modulus,
// max |lambda| + 2 mu, first voxel with an invalid E, first with an invalid
// nu), reduced over the blocks on the host; k_mat_convert: (lambda, mu) in
// FP64 and FP32 and the copy of E, written only once the check has passed,
// so a rejected material leaves the previous one in place.
constexpr int MAT_NP = 7;
constexpr int MAT_BLOCKS = 1024;

__device__ __forceinline__ void lame_of(double e, double p, double& lam, double& mu) {
  lam = p * e / ((1.0 + p) * (1.0 - 2.0 * p));
  mu = e / (2.0 * (1.0 + p));
}

__global__ __launch_bounds__(NT) void k_mat_check(const double* E, const double* nu, long long n, int d,
                                                  double* parts) {
  double v[MAT_NP] = {INFINITY, 0.0, INFINITY, 0.0, 0.0, (double)n, (double)n};
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const double e = E[i], p = nu[i];
    const bool okE = isfinite(e) && e > 0.0, okN = isfinite(p) && p > -1.0 && p < 0.5;
    if (!okE) v[5] = fmin(v[5], (double)i);
    if (!okN) v[6] = fmin(v[6], (double)i);
    if (okE && okN) {
      double lam, mu;
      lame_of(e, p, lam, mu);
      const double bulk = lam + (d == 3 ? 2.0 * mu / 3.0 : mu);
      v[0] = fmin(v[0], bulk);
      v[1] = fmax(v[1], bulk);
      v[2] = fmin(v[2], mu);
      v[3] = fmax(v[3], mu);
      v[4] = fmax(v[4], fabs(lam) + 2.0 * mu);
    }
  }
  __shared__ double sh[NT / WAVE][MAT_NP];
#pragma unroll
  for (int k = 0; k < MAT_NP; ++k) {
    const bool mx = k == 1 || k == 3 || k == 4;
    double x = v[k];
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
      const double y = __shfl_xor(x, o, WAVE);
      x = mx ? fmax(x, y) : fmin(x, y);
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE][k] = x;
  }
  __syncthreads();
  if (threadIdx.x < MAT_NP) {
    const int k = threadIdx.x;
    const bool mx = k == 1 || k == 3 || k == 4;
    double x = sh[0][k];
    for (int w = 1; w < NT / WAVE; ++w) x = mx ? fmax(x, sh[w][k]) : fmin(x, sh[w][k]);
    parts[(long long)blockIdx.x * MAT_NP + k] = x;
  }
}

__global__ __launch_bounds__(NT) void k_mat_convert(const double* E, const double* nu, long long n, double* mat64,
                                                    float* mat32, double* E64) {
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const double e = E[i], p = nu[i];
    double lam, mu;
    lame_of(e, p, lam, mu);
    mat64[2 * i] = lam;
    mat64[2 * i + 1] = mu;
    mat32[2 * i] = (float)lam;
    mat32[2 * i + 1] = (float)mu;
    E64[i] = e;
  }
}

}  // namespace

cell_status instance_set_material(cell_s* c, int cell, const double* E, const double* nu, int on_device) {
  if (!c || !E || !nu) return fail(CELL_E_ARG, "null argument");
  if (cell < 0 || cell >= c->ncell) return fail(CELL_E_ARG, "cell index out of range");
  DevGuard dg(c->dev);
  // a surrogate built from the previous material no longer applies
  c->sr_M = 0;
  if (c->op == 2) c->op = 0;
  const long long n = c->n;
  hipStream_t s = c->stream;
  // host inputs are staged in a temporary device buffer
  double* stage = nullptr;
  const double *Ed = E, *nd = nu;
  if (!on_device) {
    if (hipMalloc((void**)&stage, sizeof(double) * 2 * n) != hipSuccess)
      return fail(CELL_E_NOMEM, "device allocation failed (material staging)");
    const hipError_t e1 = hipMemcpyAsync(stage, E, sizeof(double) * n, hipMemcpyHostToDevice, s);
    const hipError_t e2 = hipMemcpyAsync(stage + n, nu, sizeof(double) * n, hipMemcpyHostToDevice, s);
    if (e1 != hipSuccess || e2 != hipSuccess) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(stage);
      return fail(CELL_E_DEVICE, std::string("material upload: ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    }
    Ed = stage;
    nd = stage + n;
  }
  auto done = [&](cell_status st) {
    if (stage) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(stage);
    }
    return st;
  };
  const int nb = (int)std::min<long long>(MAT_BLOCKS, (n + NT - 1) / NT);
  std::vector<double> parts((size_t)nb * MAT_NP);
  hipLaunchKernelGGL(k_mat_check, dim3(nb), dim3(NT), 0, s, Ed, nd, n, c->d, c->scratch);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(parts.data(), c->scratch, sizeof(double) * parts.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return done(fail(CELL_E_DEVICE, std::string("material check: ") + hipGetErrorString(e)));
  double kmin = INFINITY, kmax = 0, mmin = INFINITY, mmax = 0, modmax = 0, badE = (double)n, badN = (double)n;
  for (int b = 0; b < nb; ++b) {
    const double* q = parts.data() + (size_t)b * MAT_NP;
    kmin = std::min(kmin, q[0]);
    kmax = std::max(kmax, q[1]);
    mmin = std::min(mmin, q[2]);
    mmax = std::max(mmax, q[3]);
    modmax = std::max(modmax, q[4]);
    badE = std::min(badE, q[5]);
    badN = std::min(badN, q[6]);
  }
  // the first invalid voxel decides; at one voxel an invalid E is reported first
  if (badE < (double)n && badE <= badN)
    return done(fail(CELL_E_NONFINITE, "Young's modulus must be finite and positive (voxel " +
                                           std::to_string((long long)badE) + ")"));
  if (badN < (double)n)
    return done(fail(CELL_E_ARG, "Poisson ratio must lie in (-1, 0.5) (voxel " + std::to_string((long long)badN) + ")"));
  const long long off = (long long)cell * n;
  hipLaunchKernelGGL(k_mat_convert, dim3(nb), dim3(NT), 0, s, Ed, nd, n, c->mat64 + 2 * off, c->mat32 + 2 * off,
                     c->E64 + off);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return done(fail(CELL_E_DEVICE, std::string("material conversion: ") + hipGetErrorString(e)));
  done(CELL_OK);
  const double K0 = std::sqrt(kmin * kmax), mu0 = std::sqrt(mmin * mmax);
  c->mu0[cell] = mu0;
  c->lam0[cell] = K0 - (c->d == 3 ? 2.0 * mu0 / 3.0 : mu0);
  c->maxmod[cell] = modmax;
  c->have_mat[cell] = 1;
  c->solved = false;
  c->solved_unit = false;
  return CELL_OK;
}

cell_status solve_begin(SolveRun& R, cell_s* c, int nload, const double* eps, cell_info* infos) {
  for (int cell = 0; cell < c->ncell; ++cell)
    if (!c->have_mat[cell]) return fail(CELL_E_STATE, "material not set for cell " + std::to_string(cell));
  for (int l = 0; l < 6; ++l)
    for (int i = 0; i < 6; ++i) c->eps_v[l][i] = (l < nload && i < c->nv) ? eps[l * c->nv + i] : 0.0;
  c->solved = false;
  c->solved_unit = false;
  if (infos) std::memset(infos, 0, sizeof(cell_info) * c->ncell);
  R.c = c;
  R.nload = nload;
  R.infos = infos;
  R.result = CELL_OK;
  return c->precision == CELL_MIXED ? begin_t<float>(R) : begin_t<double>(R);
}

cell_status solve_launch(SolveRun& R) {
  return R.c->precision == CELL_MIXED ? launch_t<float>(R) : launch_t<double>(R);
}

bool solve_graphs(const SolveRun& R) { return R.c->use_graphs && !R.c->prof; }

cell_status solve_enqueue_chunk(SolveRun& R) {
  return R.c->precision == CELL_MIXED ? chunk_t<float>(R) : chunk_t<double>(R);
}

cell_status solve_copy_states(SolveRun& R) {
  cell_s* c = R.c;
  HIPCHK(hipMemcpyAsync(c->st_h, c->st, sizeof(LoadState) * c->nslot, hipMemcpyDeviceToHost, c->stream));
  return CELL_OK;
}

cell_status solve_poll(SolveRun& R) {
  return R.c->precision == CELL_MIXED ? poll_t<float>(R) : poll_t<double>(R);
}

cell_status solve_end(SolveRun& R) {
  cell_s* c = R.c;
  const cell_status st = end_t(R);
  if (st < 0) return st;
  if (c->op == 2) {
    // surrogate solutions: the exact residual and stress sums at u~ for the
    // energy-form C* of their strain fields
    const double* u = c->precision == CELL_MIXED ? c->x64 : c->f64.x;
    c->op = 0;
    const cell_status sr = c->precision == CELL_MIXED ? residual<float>(c, u, nullptr) : residual<double>(c, u, nullptr);
    c->op = 2;
    STCHK(sr);
  }
  if (c->op == 0 || c->op == 2) {
    STCHK(homogenize(c, R.nload));
    c->linear_results = true;
  }
  c->solved = true;
  c->solved_op = c->op;
  c->nload_solved = R.nload;
  return st;
}

cell_status instance_solve(cell_s* c, int nload, const double* eps, cell_info* infos) {
  SolveRun R;
  STCHK(solve_begin(R, c, nload, eps, infos));
  while (!R.done) {
    STCHK(solve_launch(R));
    HIPCHK(hipStreamSynchronize(c->stream));
    STCHK(solve_poll(R));
  }
  return solve_end(R);
}

// =================================================== neo-Hookean (Newton)
namespace {

cell_status ensure_hyper(cell_s* c) {
  if (c->hy_u) return CELL_OK;
  const size_t fb = sizeof(double) * (size_t)c->lstride * c->nslot;
  auto dm = [&](void** p, size_t b) { return hipMalloc(p, b) == hipSuccess; };
  if (!dm((void**)&c->hy_u, fb) || !dm((void**)&c->hy_ut, fb) || !dm((void**)&c->hy_rhs, fb) ||
      !dm((void**)&c->hy_F, sizeof(double) * 9 * c->nslot) || !dm((void**)&c->hy_F32, sizeof(float) * 9 * c->nslot) ||
      !dm((void**)&c->hy_t, sizeof(double) * c->nslot) ||
      !dm((void**)&c->hy_vparts, sizeof(double) * 10 * (size_t)c->nslot * c->maxblk) ||
      !dm((void**)&c->hy_vals, sizeof(double) * 10 * c->nslot) ||
      (c->precision == CELL_MIXED && !dm((void**)&c->hy_u32, sizeof(float) * (size_t)c->lstride * c->nslot)))
    return fail(CELL_E_NOMEM, "device allocation of the Newton state failed");
  if (hipHostMalloc((void**)&c->hy_vals_h, sizeof(double) * 10 * c->nslot) != hipSuccess)
    return fail(CELL_E_NOMEM, "pinned host allocation failed");
  return CELL_OK;
}

// f(u), ||f||^2, sum |s| W and sum |s| P of the masked slots at state u
// (FP64); results in res2_h and hy_vals_h
cell_status hyper_eval(cell_s* c, const double* u, const int* mask) {
  HyArgs<double> ha = hyargs<double>(c);
  ha.u = u;
  ha.out = c->hy_rhs;
  ha.mask = mask;
  {
    ProfScope ps(c, CELL_K_RESIDUAL);
    HIPCHK(launch_hyper_residual(ha, c->stream));
  }
  HIPCHK(hipMemcpyAsync(c->res2_h, c->res2, sizeof(double) * c->nslot, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(c->hy_vals_h, c->hy_vals, sizeof(double) * 10 * c->nslot, hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CELL_OK;
}

// per-slot macroscopic gradients in FP64 and FP32 (synchronous)
cell_status upload_fbar(cell_s* c, const std::vector<double>& Fh) {
  std::vector<float> f32(Fh.begin(), Fh.end());
  HIPCHK(hipMemcpyAsync(c->hy_F, Fh.data(), sizeof(double) * Fh.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->hy_F32, f32.data(), sizeof(float) * f32.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CELL_OK;
}

// per-slot max |x| from the partials of launch_amax_slots (synchronous)
cell_status read_amax(cell_s* c, std::vector<double>& amax) {
  const int nb = c->maxblk < AMAX_BLOCKS ? c->maxblk : AMAX_BLOCKS;
  std::vector<double> h((size_t)nb * c->nslot);
  HIPCHK(hipMemcpyAsync(h.data(), c->hy_vparts, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  amax.assign(c->nslot, 0.0);
  for (int l = 0; l < c->nslot; ++l)
    for (int b = 0; b < nb; ++b) amax[l] = std::max(amax[l], h[(size_t)l * nb + b]);
  return CELL_OK;
}

// the pinned mask is read by the copy when the stream reaches it: drain the
// stream before rewriting it (an earlier queued copy would see the new mask)
cell_status upload_mask(cell_s* c, const std::vector<int>& m) {
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int l = 0; l < c->nslot; ++l) c->mask_h[l] = m[l];
  HIPCHK(hipMemcpyAsync(c->mask, c->mask_h, sizeof(int) * c->nslot, hipMemcpyHostToDevice, c->stream));
  return CELL_OK;
}

cell_status hyper_run(cell_s* c, int nload, const double* Fb, double tol, int max_newton, double* P_out,
                      cell_hyper_info* infos) {
  const int ns = c->nslot, d = c->d, lpc = c->lpc;
  const long long len = c->lstride;
  hipStream_t s = c->stream;
  STCHK(c->precision == CELL_MIXED ? ensure_fields<float>(c) : ensure_fields<double>(c));
  STCHK(ensure_hyper(c));
  c->solved = false;
  c->solved_unit = false;
  c->linear_results = false;
  std::vector<double> Fh(9 * (size_t)ns, 0.0);
  std::vector<int> act(ns, 0), done(ns, 1), searching(ns, 0);
  std::vector<double> scale(ns, 0.0), E(ns, 0.0), fn(ns, 0.0), slope(ns, 0.0), t(ns, 1.0), dE(ns, 0.0),
      lastE(ns, 0.0);
  const double vol = d == 3 ? c->g.h[0] * c->g.h[1] * c->g.h[2] * c->n : c->g.h[0] * c->g.h[1] * c->n;
  const double hmin = std::min(c->g.h[0], std::min(c->g.h[1], d == 3 ? c->g.h[2] : c->g.h[1]));
  for (int l = 0; l < ns; ++l) {
    const int j = l % lpc;
    for (int a = 0; a < 3; ++a) Fh[9 * l + 4 * a] = 1.0;
    if (j >= nload) continue;
    act[l] = 1;
    done[l] = 0;
    double fmax = 1.0;
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        Fh[9 * l + 3 * a + b] = Fb[(j * d + a) * d + b];
        fmax = std::max(fmax, std::fabs(Fb[(j * d + a) * d + b]));
      }
    scale[l] = vol * c->maxmod[l / lpc] * fmax;
    // rounding level of the energy sum (terms of size modulus (|F|^2 + d))
    dE[l] = 1e-13 * vol * c->maxmod[l / lpc] * d * (1.0 + fmax * fmax);
  }
  STCHK(upload_fbar(c, Fh));
  HIPCHK(launch_zero_slots(c->hy_u, len, ns, nullptr, s));
  STCHK(upload_mask(c, act));
  STCHK(hyper_eval(c, c->hy_u, c->mask));
  std::vector<double> ref(ns, 0.0);
  for (int l = 0; l < ns; ++l) {
    if (!act[l]) continue;
    fn[l] = std::sqrt(c->res2_h[l]);
    E[l] = c->hy_vals_h[10 * l];
    if (!std::isfinite(E[l])) return fail(CELL_E_ARG, "the macroscopic gradient has det <= 0 in slot " + std::to_string(l));
    ref[l] = std::max(fn[l], scale[l]);
  }
  std::vector<int> nit(ns, 0), ncg(ns, 0), nneg(ns, 0);
  std::vector<double> zeros(36, 0.0);
  std::vector<cell_info> cgi(c->ncell);
  double* du = c->precision == CELL_MIXED ? c->x64 : c->f64.x;
  for (int it = 0;; ++it) {
    bool all = true;
    for (int l = 0; l < ns; ++l) {
      if (!act[l]) continue;
      done[l] = fn[l] <= tol * ref[l];
      if (!done[l]) all = false;
    }
    if (all || it >= max_newton) break;
    // tangent state; the converged slots get a zero right-hand side (their
    // PCG stops at once)
    if (c->precision == CELL_MIXED) HIPCHK(launch_round_slots(c->hy_u, c->hy_u32, len, ns, s));
    STCHK(upload_mask(c, done));
    HIPCHK(launch_zero_slots(c->hy_rhs, len, ns, c->mask, s));
    // f has zero nodal mean per component exactly; its rounding part lies in
    // the operator's null space, which the PCG cannot reduce (it would set a
    // floor ~1e-16 |P| / ||f|| under the relative tolerance near the solution)
    {
      std::vector<int> live(ns, 0);
      for (int l = 0; l < ns; ++l) live[l] = act[l] && !done[l];
      STCHK(upload_mask(c, live));
      HIPCHK(launch_remove_mean(c->hy_rhs, len, c->n, d, ns, c->mask, c->hy_vparts, 10 * c->maxblk / 3, s));
    }
    // inner PCG on K_T du = f (maxit > 0: at most that many iterations)
    auto inner_solve = [&](int maxit) -> cell_status {
      const int keep = c->max_iter;
      if (maxit > 0) c->max_iter = maxit;
      c->op = 1;
      SolveRun R;
      cell_status st = solve_begin(R, c, nload, zeros.data(), cgi.data());
      while (st >= 0 && !R.done) {
        st = solve_launch(R);
        if (st >= 0) {
          const hipError_t e = hipStreamSynchronize(s);
          if (e != hipSuccess) st = fail(CELL_E_DEVICE, hipGetErrorString(e));
        }
        if (st >= 0) st = solve_poll(R);
      }
      if (st >= 0) st = solve_end(R);
      c->op = c->sr_M > 0 ? 2 : 0;
      c->max_iter = keep;
      if (st < 0) return st;
      // negative curvature in the first iteration leaves du = 0: take the
      // first direction, the preconditioned residual (a descent direction)
      std::vector<int> first_dir(ns, 0);
      bool any_first = false;
      for (int l = 0; l < ns; ++l)
        if (act[l] && !done[l] && c->negcurv[l] == 1) first_dir[l] = any_first = true;
      if (any_first) {
        STCHK(upload_mask(c, first_dir));
        if (c->precision == CELL_MIXED)
          HIPCHK(launch_widen_slots(reinterpret_cast<const float*>(c->f32.p), c->x64, len, ns, c->mask, s));
        else
          HIPCHK(launch_copy_slots(c->f64.p, c->f64.x, len, ns, c->mask, s));
      }
      return CELL_OK;
    };
    auto slopes = [&](const std::vector<int>& m) -> cell_status {
      STCHK(upload_mask(c, m));
      HIPCHK(launch_dot_slots(c->hy_rhs, du, len, ns, c->mask, red_of(c), c->st, c->res2, s));
      HIPCHK(hipMemcpyAsync(c->res2_h, c->res2, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int l = 0; l < ns; ++l)
        if (m[l]) slope[l] = c->res2_h[l];
      return CELL_OK;
    };
    STCHK(inner_solve(0));
    for (int l = 0; l < ns; ++l) {
      searching[l] = act[l] && !done[l];
      t[l] = 1.0;
      if (searching[l]) {
        ncg[l] += cgi[l / lpc].iters[l % lpc];
        if (c->negcurv[l] > 0) nneg[l] += 1;
      }
    }
    STCHK(slopes(searching));
    // one PCG iteration for the masked slots (alpha_0 z_0 with z_0 = M^-1 f,
    // or z_0 on negative curvature), keeping the du of the other searching
    // slots; a descent direction by construction
    auto one_step = [&](const std::vector<int>& m) -> cell_status {
      std::vector<int> keep_du(ns, 0);
      for (int l = 0; l < ns; ++l) keep_du[l] = searching[l] && !m[l];
      STCHK(upload_mask(c, keep_du));
      HIPCHK(launch_copy_slots(du, c->hy_ut, len, ns, c->mask, s));
      STCHK(inner_solve(1));
      STCHK(upload_mask(c, keep_du));
      HIPCHK(launch_copy_slots(c->hy_ut, du, len, ns, c->mask, s));
      for (int l = 0; l < ns; ++l)
        if (m[l]) {
          ncg[l] += cgi[l / lpc].iters[l % lpc];
          nneg[l] += 1;
        }
      STCHK(slopes(m));
      for (int l = 0; l < ns; ++l)
        if (m[l] && !(slope[l] > 0.0))
          return fail(CELL_E_BREAKDOWN, "no descent direction in slot " + std::to_string(l));
      return CELL_OK;
    };
    // first trial step: t = 1, or the step that moves no node by more than
    // one voxel edge (guards against the huge steps of a nearly singular K_T)
    auto first_trial = [&](const std::vector<int>& m) -> cell_status {
      std::vector<double> amax;
      STCHK(upload_mask(c, m));
      HIPCHK(launch_amax_slots(du, len, ns, c->mask, c->hy_vparts, c->maxblk, s));
      STCHK(read_amax(c, amax));
      for (int l = 0; l < ns; ++l)
        if (m[l]) t[l] = amax[l] * 1.0 > hmin ? hmin / amax[l] : 1.0;
      return CELL_OK;
    };
    // an indefinite K_T can also give a converged du that is no descent
    // direction (f.du <= 0, negative curvature never met): those slots take
    // one PCG iteration instead
    {
      std::vector<int> redo(ns, 0);
      bool any_redo = false;
      for (int l = 0; l < ns; ++l) {
        redo[l] = searching[l] && !(slope[l] > 0.0);
        any_redo = any_redo || redo[l];
      }
      if (any_redo) STCHK(one_step(redo));
    }
    STCHK(first_trial(searching));
    // backtracking line search on the energy; a slot whose search fails
    // retries once from the one-iteration step
    std::vector<int> retried(ns, 0);
    for (int ls = 0;; ++ls) {
      bool any = false;
      for (int l = 0; l < ns; ++l) any = any || searching[l];
      if (!any) break;
      if (ls >= 40) {
        std::vector<int> fail_m(ns, 0);
        bool again = true;
        int lf = -1;
        for (int l = 0; l < ns; ++l)
          if (searching[l]) {
            fail_m[l] = 1;
            if (retried[l]) again = false, lf = l;
          }
        if (!again) {
          char msg[256];
          std::snprintf(msg, sizeof msg,
                        "Newton line search found no admissible step (slot %d, Newton step %d: f.du %.3e, "
                        "||f|| %.3e, energy %.9e, last trial energy %.9e)",
                        lf, it, slope[lf], fn[lf], E[lf], lastE[lf]);
          return fail(CELL_E_BREAKDOWN, msg);
        }
        // f(u) again for these slots (the trials overwrote it), zero mean
        STCHK(upload_mask(c, fail_m));
        STCHK(hyper_eval(c, c->hy_u, c->mask));
        HIPCHK(launch_remove_mean(c->hy_rhs, len, c->n, d, ns, c->mask, c->hy_vparts, 10 * c->maxblk / 3, s));
        STCHK(one_step(fail_m));
        STCHK(first_trial(fail_m));
        for (int l = 0; l < ns; ++l)
          if (fail_m[l]) retried[l] = 1;
        ls = 0;
      }
      STCHK(upload_mask(c, searching));
      HIPCHK(hipMemcpyAsync(c->hy_t, t.data(), sizeof(double) * ns, hipMemcpyHostToDevice, s));
      HIPCHK(launch_axpy_slots(c->hy_u, c->hy_t, du, c->hy_ut, len, ns, c->mask, s));
      STCHK(hyper_eval(c, c->hy_ut, c->mask));
      std::vector<int> acc(ns, 0);
      for (int l = 0; l < ns; ++l) {
        if (!searching[l]) continue;
        const double Et = c->hy_vals_h[10 * l], fnt = std::sqrt(c->res2_h[l]);
        lastE[l] = Et;
        // Armijo on the energy; where the change is below the energy's
        // rounding level, a decrease of the residual norm instead
        const bool armijo = Et <= E[l] - 1e-4 * t[l] * slope[l];
        const bool flat = Et - E[l] <= dE[l] && fnt <= (1.0 - 1e-4 * t[l]) * fn[l];
        if (std::isfinite(Et) && (armijo || flat)) {
          acc[l] = 1;
          searching[l] = 0;
          E[l] = Et;
          fn[l] = fnt;
          nit[l] += 1;
        } else {
          t[l] *= 0.5;
        }
      }
      STCHK(upload_mask(c, acc));
      HIPCHK(launch_copy_slots(c->hy_ut, c->hy_u, len, ns, c->mask, s));
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  // results of the last accepted evaluation of every slot
  if (P_out)
    for (int l = 0; l < ns; ++l) {
      if (!act[l]) continue;
      const int cell = l / lpc, j = l % lpc;
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b)
          P_out[(((size_t)cell * nload + j) * d + a) * d + b] = c->hy_vals_h[10 * l + 1 + 3 * a + b] / vol;
    }
  if (infos)
    for (int l = 0; l < ns; ++l) {
      if (!act[l]) continue;
      cell_hyper_info& I = infos[l / lpc];
      const int j = l % lpc;
      I.nload = nload;
      I.newton_iters[j] = nit[l];
      I.cg_iters[j] = ncg[l];
      I.indefinite_steps[j] = nneg[l];
      I.resnorm[j] = ref[l] > 0 ? fn[l] / ref[l] : 0.0;
      I.energy[j] = E[l] / vol;
    }
  // the fluctuations are the displacement results (mean removed on output)
  double* sol = c->precision == CELL_MIXED ? c->x64 : c->f64.x;
  HIPCHK(launch_copy_slots(c->hy_u, sol, len, ns, nullptr, s));
  HIPCHK(hipStreamSynchronize(s));
  c->solved = true;
  c->solved_op = 1;
  c->nload_solved = nload;
  bool conv = true;
  for (int l = 0; l < ns; ++l)
    if (act[l] && !(fn[l] <= tol * ref[l])) conv = false;
  return conv ? CELL_OK : CELL_NOT_CONVERGED;
}

}  // namespace

cell_status instance_hyper_solve(cell_s* c, int nload, const double* Fbar, double tol, int max_newton,
                                 double* P_out, cell_hyper_info* infos) {
  for (int cell = 0; cell < c->ncell; ++cell)
    if (!c->have_mat[cell]) return fail(CELL_E_STATE, "material not set for cell " + std::to_string(cell));
  if (infos) std::memset(infos, 0, sizeof(cell_hyper_info) * c->ncell);
  const double t0 = now_s();
  const cell_status st = hyper_run(c, nload, Fbar, tol, max_newton, P_out, infos);
  c->op = c->sr_M > 0 ? 2 : 0;
  if (infos && st >= 0)
    for (int cell = 0; cell < c->ncell; ++cell) infos[cell].seconds = now_s() - t0;
  return st;
}

// ============================================ surrogate stencil operator
namespace {

// periodic system a x_{i-1} + b x_i + a x_{i+1} = d_i with a = 1/6, b = 2/3:
// the cubic B-spline interpolation conditions along one lattice axis.
// Sherman-Morrison on the Thomas algorithm: A = T + u w^T with the corners
// of A moved into u w^T, u = (g, 0, .., 0, a), w = (1, 0, .., 0, a / g),
// g = -b, and T's first and last diagonal entries b - g and b - a^2 / g.
// The data-independent parts (the Thomas pivots den_i, the superdiagonal
// ratios cp_i and z = T^{-1} u) are the same for every line of a length;
// cubic_consts computes them once per axis, k_sr_cubic solves every line.
constexpr double SR_A = 1.0 / 6.0, SR_B = 2.0 / 3.0, SR_G = -2.0 / 3.0;

void cubic_consts(int n, double* den, double* cp, double* z) {
  auto diag = [&](int i) { return i == 0 ? SR_B - SR_G : (i == n - 1 ? SR_B - SR_A * SR_A / SR_G : SR_B); };
  den[0] = diag(0);
  cp[0] = SR_A / den[0];
  for (int i = 1; i < n; ++i) {
    den[i] = diag(i) - SR_A * cp[i - 1];
    cp[i] = SR_A / den[i];
  }
  for (int i = 0; i < n; ++i) z[i] = i == 0 ? SR_G : (i == n - 1 ? SR_A : 0.0);
  z[0] /= den[0];
  for (int i = 1; i < n; ++i) z[i] = (z[i] - SR_A * z[i - 1]) / den[i];
  for (int i = n - 2; i >= 0; --i) z[i] -= cp[i] * z[i + 1];
}

// every line along `axis` of every stencil value, in place in S[value][ci]
__global__ __launch_bounds__(NT) void k_sr_cubic(double* S, long long nc, int ncx, int ncy, int ncz, int axis,
                                                 const double* den, const double* cp, const double* z) {
  const int n = axis == 0 ? ncx : (axis == 1 ? ncy : ncz);
  const long long lines = nc / n;
  const long long stride = axis == 0 ? 1 : (axis == 1 ? ncx : (long long)ncx * ncy);
  for (long long w = blockIdx.x * (long long)NT + threadIdx.x; w < lines * SR_NVAL; w += (long long)gridDim.x * NT) {
    const long long v = w / lines, li = w - v * lines;
    long long base;
    if (axis == 0) base = li * ncx;                                    // li = cy + ncy cz
    else if (axis == 1) base = (li / ncx) * ncx * ncy + li % ncx;      // li = cx + ncx cz
    else base = li;                                                    // li = cx + ncx cy
    double* f = S + v * nc + base;
    if (n == 1) continue;  // the periodic sum of the spline over all shifts is 1
    if (n == 2) {
      const double d0 = f[0], d1 = f[stride], det = SR_B * SR_B - 4.0 * SR_A * SR_A;
      f[0] = (SR_B * d0 - 2.0 * SR_A * d1) / det;
      f[stride] = (SR_B * d1 - 2.0 * SR_A * d0) / det;
      continue;
    }
    double prev = f[0] / den[0];
    f[0] = prev;
    for (int i = 1; i < n; ++i) {
      prev = (f[i * stride] - SR_A * prev) / den[i];
      f[i * stride] = prev;
    }
    for (int i = n - 2; i >= 0; --i) {
      prev = f[i * stride] - cp[i] * prev;
      f[i * stride] = prev;
    }
    const double fact = (f[0] + SR_A / SR_G * f[(n - 1) * stride]) / (1.0 + z[0] + SR_A / SR_G * z[n - 1]);
    for (int i = 0; i < n; ++i) f[i * stride] -= fact * z[i];
  }
}

// stencil functions of the exact operator at the lattice nodes (every M-th
// node): K[X, X + delta] = sum over the simplices holding both nodes of
// |s| (lam g1 g2^T + mu g2 g1^T + mu g1.g2 I), g the barycentric gradients
__constant__ int kSrPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
__constant__ int kSrOff[SR_NOFF] = {1, 2, 4, 3, 6, 5, 7};  // offsets as corner bit masks (x | y << 1 | z << 2)

__global__ __launch_bounds__(NT) void k_sr_sample(const double* mat, Geom g, int M, int ncx, int ncy, int ncz,
                                                  double* S) {
  const long long nc = (long long)ncx * ncy * ncz;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const double ih[3] = {1.0 / g.h[0], 1.0 / g.h[1], 1.0 / g.h[2]};
  const double vol = g.h[0] * g.h[1] * g.h[2] / 6.0;
  for (long long w = blockIdx.x * (long long)NT + threadIdx.x; w < nc * SR_NOFF; w += (long long)gridDim.x * NT) {
    const int k = (int)(w / nc);
    const long long ci = w - (long long)k * nc;
    const int cx = (int)(ci % ncx), cy = (int)((ci / ncx) % ncy), cz = (int)(ci / ((long long)ncx * ncy));
    const int X[3] = {cx * M, cy * M, cz * M};
    const int off = kSrOff[k];
    double blk[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int c1 = 0; c1 < 8; ++c1) {
      if (c1 & off) continue;
      const int c2 = c1 | off;
      const int vx = (X[0] - (c1 & 1) + nx) % nx, vy = (X[1] - ((c1 >> 1) & 1) + ny) % ny;
      const int vz = (X[2] - ((c1 >> 2) & 1) + nz) % nz;
      const long long vid = ((long long)vz * ny + vy) * nx + vx;
      const double lam = mat[2 * vid], mu = mat[2 * vid + 1];
      for (int t = 0; t < 6; ++t) {
        int path[4] = {0, 0, 0, 0}, m1 = -1, m2 = -1;
        for (int m = 0; m < 3; ++m) path[m + 1] = path[m] | (1 << kSrPerm[t][m]);
        for (int m = 0; m < 4; ++m) {
          if (path[m] == c1) m1 = m;
          if (path[m] == c2) m2 = m;
        }
        if (m1 < 0 || m2 < 0) continue;
        double g1[3] = {0.0, 0.0, 0.0}, g2[3] = {0.0, 0.0, 0.0};
        if (m1 > 0) g1[kSrPerm[t][m1 - 1]] += ih[kSrPerm[t][m1 - 1]];
        if (m1 < 3) g1[kSrPerm[t][m1]] -= ih[kSrPerm[t][m1]];
        if (m2 > 0) g2[kSrPerm[t][m2 - 1]] += ih[kSrPerm[t][m2 - 1]];
        if (m2 < 3) g2[kSrPerm[t][m2]] -= ih[kSrPerm[t][m2]];
        const double dg = g1[0] * g2[0] + g1[1] * g2[1] + g1[2] * g2[2];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b)
            blk[3 * a + b] += vol * (lam * g1[a] * g2[b] + mu * g1[b] * g2[a] + (a == b ? mu * dg : 0.0));
      }
    }
    for (int e = 0; e < 9; ++e) S[(long long)(9 * k + e) * nc + ci] = blk[e];
  }
}

}  // namespace

cell_status instance_set_surrogate(cell_s* c, int M, int q) {
  if (M == 0) {
    // results of a surrogate solve are not those of the exact operator:
    // drop them so that no getter or the adjoint reports them as exact
    if (c->sr_M > 0) c->solved = c->solved_unit = c->linear_results = false;
    c->sr_M = 0;
    if (c->op == 2) c->op = 0;
    return CELL_OK;
  }
  if (c->d != 3) return fail(CELL_E_UNSUPPORTED, "the surrogate stencil operator is implemented in 3D");
  if (c->ncell != 1 || c->nslot > 6) return fail(CELL_E_UNSUPPORTED, "the surrogate stencil operator needs a single-cell handle");
  if (!c->have_mat[0]) return fail(CELL_E_STATE, "cell_set_material has not been called");
  if (M < 0 || (q != 1 && q != 3)) return fail(CELL_E_ARG, "M must be >= 0 and q 1 or 3");
  const int nx = c->g.nx, ny = c->g.ny, nz = c->g.nz;
  if (nx % M || ny % M || nz % M) return fail(CELL_E_ARG, "M must divide every grid size");
  DevGuard dg(c->dev);
  const double t0 = now_s();
  const long long n = c->n;
  const int ncx = nx / M, ncy = ny / M, ncz = nz / M;
  const long long nc = (long long)ncx * ncy * ncz;
  auto dm = [&](void** p, size_t bytes) { return *p != nullptr || hipMalloc(p, bytes) == hipSuccess; };
  if (!dm((void**)&c->sr64, sizeof(double) * sr_len(n)) || !dm((void**)&c->sr32, sizeof(float) * sr_len(n)) ||
      !dm((void**)&c->sr_rhs, sizeof(double) * (size_t)c->lstride * c->nslot) ||
      !dm((void**)&c->sr_parts, sizeof(double) * 3 * (size_t)c->nslot * c->maxblk) ||
      !dm((void**)&c->sr_mean, sizeof(double) * 3 * c->nslot))
    return fail(CELL_E_NOMEM, "device allocation of the surrogate stencil failed");
  // the sampled stencil functions, then (cubic) their interpolation
  // coefficients along x, y and z, in one device buffer [value][lattice node]
  const int nmax = std::max(ncx, std::max(ncy, ncz));
  double* coef = nullptr;
  if (hipMalloc((void**)&coef, sizeof(double) * ((size_t)SR_NVAL * nc + 9 * (size_t)nmax)) != hipSuccess)
    return fail(CELL_E_NOMEM, "device allocation of the spline coefficients failed");
  double* consts = coef + (size_t)SR_NVAL * nc;  // per axis: den, cp, z
  std::vector<double> ch(9 * (size_t)nmax, 0.0);
  const int nax[3] = {ncx, ncy, ncz};
  for (int ax = 0; ax < 3; ++ax)
    if (nax[ax] > 2) cubic_consts(nax[ax], &ch[(3 * ax) * nmax], &ch[(3 * ax + 1) * nmax], &ch[(3 * ax + 2) * nmax]);
  const int sblocks = (int)std::min<long long>(4096, (nc * SR_NOFF + NT - 1) / NT);
  hipLaunchKernelGGL(k_sr_sample, dim3(sblocks), dim3(NT), 0, c->stream, (const double*)c->mat64, c->g, M, ncx, ncy,
                     ncz, coef);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && q == 3) {
    e = hipMemcpyAsync(consts, ch.data(), sizeof(double) * ch.size(), hipMemcpyHostToDevice, c->stream);
    for (int ax = 0; ax < 3 && e == hipSuccess; ++ax) {
      const long long work = nc / nax[ax] * SR_NVAL;
      hipLaunchKernelGGL(k_sr_cubic, dim3((unsigned)std::min<long long>(4096, (work + NT - 1) / NT)), dim3(NT), 0,
                         c->stream, coef, nc, ncx, ncy, ncz, ax, (const double*)consts + (3 * ax) * nmax,
                         (const double*)consts + (3 * ax + 1) * nmax, (const double*)consts + (3 * ax + 2) * nmax);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = launch_sr_expand(coef, ncx, ncy, ncz, M, q, c->g, c->sr64, c->sr32, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->sr_mean, 0, sizeof(double) * 3 * c->nslot, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(coef);
  if (e != hipSuccess) return fail(CELL_E_DEVICE, hipGetErrorString(e));
  c->sr_M = M;
  c->sr_q = q;
  c->op = 2;
  c->solved = c->solved_unit = c->linear_results = false;
  c->sr_setup_s = now_s() - t0;
  return CELL_OK;
}

cell_status instance_get_surrogate(cell_s* c, double* out) {
  if (c->sr_M == 0) return fail(CELL_E_STATE, "no surrogate stencil operator is set");
  DevGuard dg(c->dev);
  const long long n = c->n;
  std::vector<double> buf(sr_len(n));
  HIPCHK(hipMemcpyAsync(buf.data(), c->sr64, sizeof(double) * buf.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  // chunked device layout -> [value][node]: each chunk holds a run of up to
  // SR_CHUNK consecutive nodes per value
  for (long long i0 = 0; i0 < n; i0 += SR_CHUNK) {
    const long long len = std::min<long long>(SR_CHUNK, n - i0);
    const double* src = buf.data() + sr_chunk(i0);
    for (int v = 0; v < SR_NVAL; ++v)
      std::copy(src + (long long)v * SR_CHUNK, src + (long long)v * SR_CHUNK + len, out + (long long)v * n + i0);
  }
  return CELL_OK;
}

// ============================================ single-step entry points (tests)
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

// slot 0 active, the others idle
void diag_state(cell_s* c) {
  for (int l = 0; l < c->nslot; ++l) {
    LoadState& S = c->st_h[l];
    std::memset(&S, 0, sizeof(S));
    S.state = l == 0 ? ST_ACTIVE : ST_IDLE;
    S.thr = -1.0;
    S.maxit = 1 << 30;
    S.first = 1;
  }
}

template <typename T>
cell_status apply_operator_t(cell_s* c, const double* u, double* q) {
  STCHK(ensure_fields<T>(c));
  Fields<T>& F = fields<T>(c);
  c->solved = c->solved_unit = false;
  STCHK(upload_field<T>(c, F.p, u));
  diag_state(c);
  HIPCHK(hipMemcpyAsync(c->st, c->st_h, sizeof(LoadState) * c->nslot, hipMemcpyHostToDevice, c->stream));
  for (int l = 0; l < 6; ++l)
    for (int i = 0; i < 6; ++i) c->eps_v[l][i] = 0.0;
  if (c->op == 2) {  // the surrogate operator while one is set (output before projection)
    SArgs<T> sa = sargs<T>(c);
    sa.p = F.p;
    sa.out = F.q;
    HIPCHK(launch_sr_apply<T>(sa, c->stream));
    return download_field<T>(c, q, F.q);
  }
  KArgs<T> ka = kargs<T>(c, 0, F.p, F.q, mat_of<T>(c));
  HIPCHK(launch_stencil<T>(ka, c->sched, c->stream));
  return download_field<T>(c, q, F.q);
}

template <typename T>
cell_status apply_precond_t(cell_s* c, const double* r, double* z) {
  STCHK(ensure_fields<T>(c));
  Fields<T>& F = fields<T>(c);
  c->solved = c->solved_unit = false;
  STCHK(upload_field<T>(c, F.r, r));
  HIPCHK(hipMemsetAsync(F.p, 0, sizeof(T) * c->lstride, c->stream));
  HIPCHK(hipMemsetAsync(F.q, 0, sizeof(T) * c->lstride, c->stream));
  diag_state(c);
  HIPCHK(hipMemcpyAsync(c->st, c->st_h, sizeof(LoadState) * c->nslot, hipMemcpyHostToDevice, c->stream));
  STCHK(iteration<T>(c, false));
  return download_field<T>(c, z, F.p);
}

}  // namespace

cell_status instance_precond_prepare(cell_s* c) { return ensure_fields<double>(c); }

cell_status instance_precond_device(cell_s* c, const double* r, double* z) {
  Fields<double>& F = c->f64;
  hipStream_t s = c->stream;
  const size_t bytes = sizeof(double) * c->lstride;
  HIPCHK(hipMemcpyAsync(F.r, r, bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemsetAsync(F.p, 0, bytes, s));
  HIPCHK(hipMemsetAsync(F.q, 0, bytes, s));
  // the slot states are the same on every call (slot 0 active, alpha = beta = 0)
  diag_state(c);
  HIPCHK(hipMemcpyAsync(c->st, c->st_h, sizeof(LoadState) * c->nslot, hipMemcpyHostToDevice, s));
  STCHK(iteration<double>(c, false));
  HIPCHK(hipMemcpyAsync(z, F.p, bytes, hipMemcpyDeviceToDevice, s));
  return CELL_OK;
}

// neo-Hookean single steps on slot 0: q = K_T(u) p in the given precision,
// or (p == nullptr) f = -grad Pi(u) in FP64 with the 10 sums |s| W, |s| P
template <typename T>
cell_status hyper_step_t(cell_s* c, const double* Fbar, const double* u, const double* p, double* out,
                         double* vals) {
  STCHK(ensure_fields<T>(c));
  STCHK(ensure_hyper(c));
  Fields<T>& F = fields<T>(c);
  HIPCHK(hipStreamSynchronize(c->stream));  // the pinned states are rewritten below
  c->solved = c->solved_unit = c->linear_results = false;
  std::vector<double> Fh(9 * (size_t)c->nslot, 0.0);
  for (int l = 0; l < c->nslot; ++l)
    for (int a = 0; a < 3; ++a) Fh[9 * l + 4 * a] = 1.0;
  for (int a = 0; a < c->d; ++a)
    for (int b = 0; b < c->d; ++b) Fh[3 * a + b] = Fbar[a * c->d + b];
  STCHK(upload_fbar(c, Fh));
  HIPCHK(hipMemcpyAsync(c->hy_u, u, sizeof(double) * c->lstride, hipMemcpyHostToDevice, c->stream));
  if (c->hy_u32) HIPCHK(launch_round_slots(c->hy_u, c->hy_u32, c->lstride, 1, c->stream));
  diag_state(c);
  HIPCHK(hipMemcpyAsync(c->st, c->st_h, sizeof(LoadState) * c->nslot, hipMemcpyHostToDevice, c->stream));
  std::vector<int> m(c->nslot, 0);
  m[0] = 1;
  STCHK(upload_mask(c, m));
  if (p) {
    STCHK(upload_field<T>(c, F.p, p));
    HyArgs<T> ha = hyargs<T>(c);
    if (sizeof(T) == 4 && !c->hy_u32) return fail(CELL_E_ARG, "FP32 tangent needs a mixed-precision handle");
    ha.p = F.p;
    ha.out = F.q;
    HIPCHK(launch_hyper_tangent<T>(ha, c->stream));
    return download_field<T>(c, out, F.q);
  }
  STCHK(hyper_eval(c, c->hy_u, c->mask));
  std::vector<double> h(c->lstride);
  HIPCHK(hipMemcpyAsync(out, c->hy_rhs, sizeof(double) * c->lstride, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (vals)
    for (int v = 0; v < 10; ++v) vals[v] = c->hy_vals_h[v];
  return CELL_OK;
}

cell_status instance_hyper_step(cell_s* c, int precision, const double* Fbar, const double* u, const double* p,
                                double* out, double* vals) {
  if (precision == CELL_FP64 || !p) return hyper_step_t<double>(c, Fbar, u, p, out, vals);
  if (precision == CELL_MIXED) return hyper_step_t<float>(c, Fbar, u, p, out, vals);
  return fail(CELL_E_ARG, "invalid precision");
}

cell_status instance_apply_operator(cell_s* c, int precision, const double* u, double* q) {
  if (precision == CELL_FP64) return apply_operator_t<double>(c, u, q);
  if (precision == CELL_MIXED) return apply_operator_t<float>(c, u, q);
  return fail(CELL_E_ARG, "invalid precision");
}

cell_status instance_apply_precond(cell_s* c, int precision, const double* r, double* z) {
  if (precision == CELL_FP64) return apply_precond_t<double>(c, r, z);
  if (precision == CELL_MIXED) return apply_precond_t<float>(c, r, z);
  return fail(CELL_E_ARG, "invalid precision");
}

cell_status instance_profile(cell_s* c, int enable) {
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

cell_status instance_profile_read(cell_s* c, double* ms_out, long long* launches_out) {
  DevGuard dg(c->dev);
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->prof) STCHK(prof_collect(c));
  for (int k = 0; k < CELL_NKERNEL; ++k) {
    ms_out[k] = c->prof_ms[k];
    launches_out[k] = c->prof_cnt[k];
  }
  return CELL_OK;
}

// ================================================================= autotuner
// Times the compiled variants of each iteration kernel on the instance's own
// buffers (every slot active, scalars harmless) and keeps the fastest:
// stencil tile and z extent, rows per block of the x passes, columns per
// block of the y pass, columns per block and radix order of the last pass.
// Results are cached per (device architecture, grid, precision, slot count)
// in the JSON file named by CELLFFT_TUNE_CACHE (none: no cache).  The
// fields touched are the ones every solve reinitialises.
namespace {

constexpr int TUNE_REPS = 5;

std::string tune_key(cell_s* c) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, c->dev) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
  }
  return arch + "|" + std::to_string(c->d) + "d|" + std::to_string(c->g.nx) + "x" + std::to_string(c->g.ny) + "x" +
         std::to_string(c->g.nz) + "|" + (c->precision == CELL_MIXED ? "f32" : "f64") + "|" +
         std::to_string(c->nslot);
}

void sched_to_ints(const Sched& sc, int* v) {
  v[0] = sc.st_tile;
  v[1] = sc.st_tz;
  v[2] = sc.x_var;
  v[3] = sc.y_var;
  v[4] = sc.z_var;
  v[5] = sc.z_radix;
}

bool sched_from_ints(const int* v, Sched* sc) {
  const bool ok = v[0] >= 0 && v[0] < ST_NTILE && (v[1] == 8 || v[1] == 16 || v[1] == 32 || v[1] == 64) &&
                  (v[2] >= 0 && v[2] <= 3) && (v[3] >= 0 && v[3] <= 3) && (v[4] >= 0 && v[4] <= 3) &&
                  (v[5] == 0 || v[5] == 1);
  if (!ok) return false;
  sc->st_tile = v[0];
  sc->st_tz = v[1];
  sc->x_var = v[2];
  sc->y_var = v[3];
  sc->z_var = v[4];
  sc->z_radix = v[5];
  return true;
}

// cache file: {"<key>": [tile, tz, x, y, z, radix], ...}, one entry per line
std::map<std::string, std::vector<int>> cache_read(const char* path) {
  std::map<std::string, std::vector<int>> out;
  FILE* f = std::fopen(path, "r");
  if (!f) return out;
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    const char* q0 = std::strchr(line, '"');
    if (!q0) continue;
    const char* q1 = std::strchr(q0 + 1, '"');
    if (!q1) continue;
    const char* br = std::strchr(q1, '[');
    if (!br) continue;
    std::vector<int> v(SCHED_NFIELD);
    if (std::sscanf(br, "[%d , %d , %d , %d , %d , %d]", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) == SCHED_NFIELD)
      out[std::string(q0 + 1, q1)] = v;
  }
  std::fclose(f);
  return out;
}

bool cache_write(const char* path, const std::map<std::string, std::vector<int>>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : m) {
    std::fprintf(f, "  \"%s\": [%d, %d, %d, %d, %d, %d]%s\n", kv.first.c_str(), kv.second[0], kv.second[1],
                 kv.second[2], kv.second[3], kv.second[4], kv.second[5], ++i < m.size() ? "," : "");
  }
  std::fprintf(f, "}\n");
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

struct TuneTimer {
  cell_s* c;
  hipEvent_t ev[2 * TUNE_REPS] = {};
  explicit TuneTimer(cell_s* c_) : c(c_) {}
  ~TuneTimer() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  cell_status init() {
    for (hipEvent_t& e : ev) HIPCHK(hipEventCreate(&e));
    return CELL_OK;
  }
  // mean milliseconds of one launch sequence; the slot states are reset
  // before every repetition (outside the timed pair)
  template <typename F>
  cell_status time(F&& launch, double* ms_out) {
    hipStream_t s = c->stream;
    HIPCHK(hipMemcpyAsync(c->st, c->st_h, sizeof(LoadState) * c->nslot, hipMemcpyHostToDevice, s));
    STCHK(launch());  // warm-up
    for (int r = 0; r < TUNE_REPS; ++r) {
      HIPCHK(hipMemcpyAsync(c->st, c->st_h, sizeof(LoadState) * c->nslot, hipMemcpyHostToDevice, s));
      HIPCHK(hipEventRecord(ev[2 * r], s));
      STCHK(launch());
      HIPCHK(hipEventRecord(ev[2 * r + 1], s));
    }
    HIPCHK(hipStreamSynchronize(s));
    double tot = 0.0;
    for (int r = 0; r < TUNE_REPS; ++r) {
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]));
      tot += ms;
    }
    *ms_out = tot / TUNE_REPS;
    return CELL_OK;
  }
};

template <typename T>
cell_status tune_t(cell_s* c) {
  STCHK(ensure_fields<T>(c));
  Fields<T>& F = fields<T>(c);
  hipStream_t s = c->stream;
  const int ns = c->nslot;
  c->solved = c->solved_unit = false;
  for (int l = 0; l < ns; ++l) {
    LoadState& S = c->st_h[l];
    std::memset(&S, 0, sizeof(S));
    S.state = ST_ACTIVE;
    S.rz = 1.0;
    S.thr = -1.0;
    S.maxit = 1 << 30;
  }
  // benign data: the fields start from zero
  const size_t fb = sizeof(T) * (size_t)c->lstride * ns;
  HIPCHK(hipMemsetAsync(F.x, 0, fb, s));
  HIPCHK(hipMemsetAsync(F.r, 0, fb, s));
  HIPCHK(hipMemsetAsync(F.p, 0, fb, s));
  HIPCHK(hipMemsetAsync(F.q, 0, fb, s));
  HIPCHK(hipMemsetAsync(F.S, 0, sizeof(cpx<T>) * (size_t)c->s_ls * ns, s));
  HIPCHK(hipMemsetAsync(F.R, 0, fb, s));
  PArgs<T> pa = make_pargs<T>(c, 0);
  if (c->d == 2) pa.Sin = F.R;
  STCHK(ensure_symtab<T>(c, pa));
  XArgs<T> xa = xargs<T>(c);
  YArgs<T> ya{};
  ya.S = F.S;
  ya.Sin = F.R;
  ya.lstrideC = c->lstride / 2;
  ya.zsS = c->s_zs;
  ya.lsS = c->s_ls;
  ya.nx = c->g.nx;
  ya.ny = c->g.ny;
  ya.nz = c->g.nz;
  ya.ncomp = c->d;
  ya.tw = F.tw[1];
  ya.st = c->st;
  KArgs<T> ka = kargs<T>(c, 0, F.p, F.q, mat_of<T>(c));
  TuneTimer tm(c);
  STCHK(tm.init());
  Sched best = c->sched;
  const bool fp64 = sizeof(T) == 8;
  double ms, bms;
  // stencil: tiles that fit the grid (or the runtime tile) x z extents
  bms = 1e300;
  bool any_tile = false;
  for (int t = 0; t < ST_NTILE; ++t) {
    if (!stencil_tile_fits(c->g, fp64, t)) continue;
    any_tile = true;
    for (int tz = ST_TZ_MIN; tz <= 64; tz *= 2) {
      if (tz > c->g.nz && tz > ST_TZ_MIN) continue;  // clamps to nz: already timed
      Sched sc = best;
      sc.st_tile = t;
      sc.st_tz = tz;
      STCHK(tm.time([&]() -> cell_status {
        HIPCHK(launch_stencil<T>(ka, sc, s));
        return CELL_OK;
      }, &ms));
      if (ms < bms) {
        bms = ms;
        best.st_tile = t;
        best.st_tz = tz;
      }
    }
  }
  if (!any_tile && c->d == 3) {
    for (int tz = ST_TZ_MIN; tz <= 64; tz *= 2) {
      if (tz > c->g.nz && tz > ST_TZ_MIN) continue;  // clamps to nz: already timed
      Sched sc = best;
      sc.st_tz = tz;
      STCHK(tm.time([&]() -> cell_status {
        HIPCHK(launch_stencil<T>(ka, sc, s));
        return CELL_OK;
      }, &ms));
      if (ms < bms) {
        bms = ms;
        best.st_tz = tz;
      }
    }
  }
  // x passes (forward and inverse together)
  bms = 1e300;
  for (int v = 0; v < 4; ++v) {
    Sched sc = best;
    sc.x_var = v;
    STCHK(tm.time([&]() -> cell_status {
      HIPCHK(launch_xfwd<T>(xa, c->g.nx, ns, sc, s));
      HIPCHK(launch_xinv<T>(xa, c->g.nx, ns, sc, s));
      return CELL_OK;
    }, &ms));
    if (ms < bms) {
      bms = ms;
      best.x_var = v;
    }
  }
  // y pass (3D; forward and inverse)
  if (c->d == 3) {
    bms = 1e300;
    for (int v = 0; v < 4; ++v) {
      Sched sc = best;
      sc.y_var = v;
      STCHK(tm.time([&]() -> cell_status {
        HIPCHK(launch_ypass<T>(ya, false, ns, sc, s));
        HIPCHK(launch_ypass<T>(ya, true, ns, sc, s));
        return CELL_OK;
      }, &ms));
      if (ms < bms) {
        bms = ms;
        best.y_var = v;
      }
    }
  }
  // last pass: columns and threads per block x radix order
  bms = 1e300;
  for (int v = 0; v < (c->d == 3 ? 4 : 2); ++v)
    for (int rp = 0; rp < (c->d == 3 ? 2 : 1); ++rp) {
      Sched sc = best;
      sc.z_var = v;
      sc.z_radix = rp;
      STCHK(tm.time([&]() -> cell_status {
        HIPCHK(launch_last<T>(pa, c->d, ns, sc, s));
        return CELL_OK;
      }, &ms));
      if (ms < bms) {
        bms = ms;
        best.z_var = v;
        best.z_radix = rp;
      }
    }
  c->sched = best;
  return CELL_OK;
}

}  // namespace

cell_status instance_autotune(cell_s* c, int force) {
  for (int cell = 0; cell < c->ncell; ++cell)
    if (!c->have_mat[cell]) return fail(CELL_E_STATE, "material not set for cell " + std::to_string(cell));
  DevGuard dg(c->dev);
  const char* path = std::getenv("CELLFFT_TUNE_CACHE");
  const std::string key = tune_key(c);
  std::map<std::string, std::vector<int>> cache;
  if (path && *path) cache = cache_read(path);
  if (!force) {
    auto it = cache.find(key);
    Sched sc;
    if (it != cache.end() && sched_from_ints(it->second.data(), &sc)) {
      c->sched = sc;
      c->tuned = true;
      return CELL_OK;
    }
  }
  const bool prof = c->prof;
  c->prof = false;
  cell_status st = c->precision == CELL_MIXED ? tune_t<float>(c) : tune_t<double>(c);
  c->prof = prof;
  if (st < 0) return st;
  c->tuned = true;
  if (path && *path) {
    std::vector<int> v(SCHED_NFIELD);
    sched_to_ints(c->sched, v.data());
    cache = cache_read(path);  // merge with entries written meanwhile
    cache[key] = v;
    if (!cache_write(path, cache)) return fail(CELL_E_ARG, std::string("cannot write the tuning cache ") + path);
  }
  return CELL_OK;
}

// the cached schedule of the instance's key, if CELLFFT_TUNE_CACHE names a
// cache that has one
void apply_cached_schedule(cell_s* c) {
  const char* path = std::getenv("CELLFFT_TUNE_CACHE");
  if (!path || !*path) return;
  const auto cache = cache_read(path);
  auto it = cache.find(tune_key(c));
  Sched sc;
  if (it != cache.end() && sched_from_ints(it->second.data(), &sc)) {
    c->sched = sc;
    c->tuned = true;
  }
}

void instance_get_schedule(cell_s* c, int* out) { sched_to_ints(c->sched, out); }

cell_status instance_set_schedule(cell_s* c, const int* in) {
  Sched sc;
  if (!sched_from_ints(in, &sc)) return fail(CELL_E_ARG, "invalid schedule");
  c->sched = sc;
  return CELL_OK;
}

cell_status instance_set_guess(cell_s* c, int load, const double* u0, int on_device) {
  if (load < 0 || load >= c->lpc) return fail(CELL_E_ARG, "load index out of range");
  if (!u0) {
    c->x0_set[load] = 0;
    return CELL_OK;
  }
  const long long m = c->lstride;
  if (!on_device)
    for (long long i = 0; i < m; ++i)
      if (!std::isfinite(u0[i])) return fail(CELL_E_ARG, "non-finite initial guess");
  if (!c->x0 && hipMalloc((void**)&c->x0, sizeof(double) * m * c->lpc) != hipSuccess) {
    c->x0 = nullptr;
    return fail(CELL_E_NOMEM, "device allocation of the initial guesses failed");
  }
  HIPCHK(hipMemcpyAsync(c->x0 + (long long)load * m, u0, sizeof(double) * m,
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->x0_set[load] = 1;
  return CELL_OK;
}

}  // namespace cellfft
