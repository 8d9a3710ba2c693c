// C ABI of the cell-problem solver (include/cellfft.h): argument checks,
// the single-cell handle (an instance with one cell) and the batch handle
// (one instance per distinct grid, all on one stream, solved in lockstep).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>

#include "solver.h"

using namespace cellfft;

namespace {

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

__global__ void k_widen(const float* in, long long n, double* out) {
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT)
    out[i] = (double)in[i];
}

const double* solution64(cell_s* c) { return c->precision == CELL_MIXED ? c->x64 : c->f64.x; }

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

// homogenised values of one cell of the last solve: C (energy form)
// [nload][nload] then mean stresses [nload][nv]
const double* homog_of(cell_s* c, int cell) {
  const int nl = c->nload_solved;
  return c->homog.data() + (size_t)cell * (nl * nl + nl * c->nv);
}

// Hill-Mandel gap of one cell: energy form against mean stress . macro strain
double hill_mandel(cell_s* c, int cell) {
  const int nl = c->nload_solved, nv = c->nv;
  const double* h = homog_of(c, cell);
  double cmax = 0.0, gap = 0.0;
  for (int i = 0; i < nl * nl; ++i) cmax = std::max(cmax, std::fabs(h[i]));
  for (int J = 0; J < nl; ++J) {
    double se = 0.0;
    for (int q = 0; q < nv; ++q) se += h[nl * nl + J * nv + q] * c->eps_v[J][q];
    gap = std::max(gap, std::fabs(h[J * nl + J] - se));
  }
  return cmax > 0 ? gap / cmax : 0.0;
}

// unit loads: C* of one cell and the asymmetry of its mean-stress form
void unit_results(cell_s* c, int cell, double* C_out, double* sym_gap) {
  const int nv = c->nv;
  const double* h = homog_of(c, cell);
  double smax = 0.0, sgap = 0.0;
  for (int I = 0; I < nv; ++I)
    for (int J = 0; J < nv; ++J) {
      C_out[I * nv + J] = h[I * nv + J];
      const double sIJ = h[nv * nv + J * nv + I];  // mean stress of load J, component I
      const double sJI = h[nv * nv + I * nv + J];
      smax = std::max(smax, std::fabs(sIJ));
      sgap = std::max(sgap, std::fabs(sIJ - sJI));
    }
  *sym_gap = smax > 0 ? sgap / smax : 0.0;
}

cell_status check_strains(int nload, int nv, const double* eps) {
  for (int i = 0; i < nload * nv; ++i)
    if (!std::isfinite(eps[i])) return fail(CELL_E_ARG, "non-finite macro strain");
  return CELL_OK;
}

// mean-zero displacement of load `load` of cell `cell` of the last solve
cell_status slot_displacement(cell_s* c, int cell, int load, double* u_out, int on_device) {
  if (!c->solved) return fail(CELL_E_STATE, "no solution available");
  if (load < 0 || load >= c->nload_solved) return fail(CELL_E_ARG, "load index out of range");
  DevGuard dg(c->dev);
  const double* u = solution64(c) + ((long long)cell * c->lpc + load) * c->lstride;
  const int nblk = 256;
  double* parts = c->scratch;
  double* mean = c->scratch + 8 * nblk;
  hipLaunchKernelGGL(k_colsum, dim3(nblk), dim3(NT), 0, c->stream, u, c->n, c->d, parts, nblk);
  hipLaunchKernelGGL(k_sum_rows2, dim3(c->d), dim3(NT), 0, c->stream, (const double*)parts, nblk,
                     1.0 / (double)c->n, mean);
  if (on_device) {
    hipLaunchKernelGGL(k_sub_mean, dim3(1024), dim3(256), 0, c->stream, u, (const double*)mean, c->n, c->d, u_out);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return CELL_OK;
  }
  // host output: subtract the means on the device into a temporary buffer
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

// final residual of load `load` of cell `cell` (FP32 rounding in mixed mode)
cell_status slot_residual(cell_s* c, int cell, int load, double* r_out, int on_device) {
  if (!c->solved || !c->linear_results) return fail(CELL_E_STATE, "no linear solution available");
  if (load < 0 || load >= c->nload_solved) return fail(CELL_E_ARG, "load index out of range");
  DevGuard dg(c->dev);
  const long long off = ((long long)cell * c->lpc + load) * c->lstride;
  if (c->precision == CELL_MIXED && on_device) {
    // widened on the device, in order on the handle's stream
    const int nb = (int)std::min<long long>(1024, (c->lstride + NT - 1) / NT);
    hipLaunchKernelGGL(k_widen, dim3(nb), dim3(NT), 0, c->stream, (const float*)(c->f32.r + off), c->lstride, r_out);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
  } else if (c->precision == CELL_MIXED) {
    std::vector<float> h(c->lstride);
    HIPCHK(hipMemcpyAsync(h.data(), c->f32.r + off, sizeof(float) * c->lstride, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (long long i = 0; i < c->lstride; ++i) r_out[i] = (double)h[i];
  } else {
    HIPCHK(hipMemcpyAsync(r_out, c->f64.r + off, sizeof(double) * c->lstride,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  return CELL_OK;
}

}  // namespace

// ======================================================================= ABI
extern "C" {

const char* cell_last_error(void) { return last_error_message(); }

int cell_debug_bounds_violations(void) {
#ifdef CELLFFT_BOUNDS_CHECK
  if (hipDeviceSynchronize() != hipSuccess) return -2;
  unsigned long long sum = 0;
  for (unsigned int v : {oob_take_fft(), oob_take_stencil(), oob_take_hyper(), oob_take_surrogate()}) {
    if (v == 0xffffffffu) return -2;
    sum += v;
  }
  return sum > 0x7fffffffull ? 0x7fffffff : (int)sum;
#else
  return -1;
#endif
}

cell_status cell_create(const cell_config* cfg, cell_t* out) { return instance_create(cfg, 1, nullptr, out); }

void cell_destroy(cell_t c) { instance_destroy(c); }

cell_status cell_set_material(cell_t c, const double* E, const double* nu, int on_device) {
  if (!c) return fail(CELL_E_ARG, "null argument");
  return instance_set_material(c, 0, E, nu, on_device);
}

cell_status cell_solve(cell_t c, int nload, const double* macro_strain, double* mean_stress_out,
                       cell_info* info) {
  const double t0 = now_s();
  if (!c || !macro_strain) return fail(CELL_E_ARG, "null argument");
  if (nload < 1 || nload > c->lpc) return fail(CELL_E_ARG, "nload must be in [1, max_loads]");
  if (!c->have_mat[0]) return fail(CELL_E_STATE, "cell_set_material has not been called");
  STCHK(check_strains(nload, c->nv, macro_strain));
  DevGuard dg(c->dev);
  const cell_status st = instance_solve(c, nload, macro_strain, info);
  if (st < 0) return st;
  const double* h = homog_of(c, 0);
  if (mean_stress_out)
    for (int J = 0; J < nload; ++J)
      for (int q = 0; q < c->nv; ++q) mean_stress_out[J * c->nv + q] = h[nload * nload + J * c->nv + q];
  if (info) {
    info->hill_mandel_gap = hill_mandel(c, 0);
    info->seconds = now_s() - t0;
  }
  return st;
}

cell_status cell_effective_stiffness(cell_t c, double* C_out, cell_info* info) {
  const double t0 = now_s();
  if (!c || !C_out) return fail(CELL_E_ARG, "null argument");
  if (!c->have_mat[0]) return fail(CELL_E_STATE, "cell_set_material has not been called");
  if (c->lpc < c->nv) return fail(CELL_E_ARG, "max_loads must be nv for the effective stiffness");
  DevGuard dg(c->dev);
  const int nv = c->nv;
  std::vector<double> eye(nv * nv, 0.0);
  for (int i = 0; i < nv; ++i) eye[i * nv + i] = 1.0;
  const cell_status st = instance_solve(c, nv, eye.data(), info);
  if (st < 0) return st;
  double sgap = 0.0;
  unit_results(c, 0, C_out, &sgap);
  c->solved_unit = true;
  if (info) {
    info->sym_gap = sgap;
    info->hill_mandel_gap = hill_mandel(c, 0);
    info->seconds = now_s() - t0;
  }
  return st;
}

cell_status cell_adjoint(cell_t c, const double* dJ_dC, double* dJ_dE_out, int on_device) {
  if (!c || !dJ_dC || !dJ_dE_out) return fail(CELL_E_ARG, "null argument");
  if (c->sr_M > 0) return fail(CELL_E_STATE, "the adjoint needs the exact operator (a surrogate stencil operator is set)");
  if (!c->solved_unit) return fail(CELL_E_STATE, "cell_adjoint needs a preceding cell_effective_stiffness");
  if (c->solved_op != 0) return fail(CELL_E_STATE, "the last solve did not use the exact operator");
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
  h.lpc = c->lpc;
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

cell_status cell_solve_projection(cell_t c, int nload, const double* macro_strain, double* mean_stress_out,
                                  cell_info* info) {
  const double t0 = now_s();
  if (!c || !macro_strain) return fail(CELL_E_ARG, "null argument");
  if (nload < 1 || nload > 6) return fail(CELL_E_ARG, "nload must be in [1, 6]");
  STCHK(check_strains(nload, c->nv, macro_strain));
  DevGuard dg(c->dev);
  const cell_status st = instance_solve_projection(c, nload, macro_strain, mean_stress_out, info);
  if (info && st >= 0) info->seconds = now_s() - t0;
  return st;
}

cell_status cell_set_initial_guess(cell_t c, int load, const double* u0, int on_device) {
  if (!c) return fail(CELL_E_ARG, "null argument");
  DevGuard dg(c->dev);
  return instance_set_guess(c, load, u0, on_device);
}

cell_status cell_get_displacement(cell_t c, int load, double* u_out, int on_device) {
  if (!c || !u_out) return fail(CELL_E_ARG, "null argument");
  return slot_displacement(c, 0, load, u_out, on_device);
}

cell_status cell_energy_matrix(cell_t c, double* C_out) {
  if (!c || !C_out) return fail(CELL_E_ARG, "null argument");
  if (!c->solved || !c->linear_results) return fail(CELL_E_STATE, "no linear solution available");
  const double* h = homog_of(c, 0);
  for (int i = 0; i < c->nload_solved * c->nload_solved; ++i) C_out[i] = h[i];
  return CELL_OK;
}

cell_status cell_get_residual(cell_t c, int load, double* r_out, int on_device) {
  if (!c || !r_out) return fail(CELL_E_ARG, "null argument");
  return slot_residual(c, 0, load, r_out, on_device);
}

cell_status cell_get_residual_history(cell_t c, int load, double* hist_out, int capacity, int* count_out) {
  if (!c || !count_out || (!hist_out && capacity > 0)) return fail(CELL_E_ARG, "null argument");
  if (capacity < 0) return fail(CELL_E_ARG, "negative capacity");
  if (load < 0 || load >= c->lpc) return fail(CELL_E_ARG, "load index out of range");
  const int n = c->hist_n.empty() ? 0 : c->hist_n[load];
  if (n == 0) return fail(CELL_E_STATE, "no solve of this load yet");
  *count_out = n;
  const int m = std::min(n, capacity);
  if (m == 0) return CELL_OK;
  DevGuard dg(c->dev);
  std::vector<double> h(m);
  HIPCHK(hipMemcpyAsync(h.data(), c->hist + (long long)load * c->hist_cap, sizeof(double) * m,
                        hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const double fn2 = c->hist_fn2[load];
  for (int k = 0; k < m; ++k) hist_out[k] = fn2 > 0.0 ? std::sqrt(h[k] / fn2) : 0.0;
  return CELL_OK;
}

cell_status cell_reference_medium(cell_t c, double* lam0, double* mu0) {
  if (!c || !lam0 || !mu0) return fail(CELL_E_ARG, "null argument");
  if (!c->have_mat[0]) return fail(CELL_E_STATE, "cell_set_material has not been called");
  *lam0 = c->lam0[0];
  *mu0 = c->mu0[0];
  return CELL_OK;
}

cell_status cell_apply_operator(cell_t c, int precision, const double* u, double* q_out) {
  if (!c || !u || !q_out) return fail(CELL_E_ARG, "null argument");
  if (!c->have_mat[0]) return fail(CELL_E_STATE, "cell_set_material has not been called");
  DevGuard dg(c->dev);
  return instance_apply_operator(c, precision, u, q_out);
}

cell_status cell_apply_preconditioner(cell_t c, int precision, const double* r, double* z_out) {
  if (!c || !r || !z_out) return fail(CELL_E_ARG, "null argument");
  if (!c->have_mat[0]) return fail(CELL_E_STATE, "cell_set_material has not been called");
  DevGuard dg(c->dev);
  return instance_apply_precond(c, precision, r, z_out);
}

cell_status cell_profile(cell_t c, int enable) {
  if (!c) return fail(CELL_E_ARG, "null argument");
  return instance_profile(c, enable);
}

cell_status cell_profile_read(cell_t c, double* ms_out, long long* launches_out) {
  if (!c || !ms_out || !launches_out) return fail(CELL_E_ARG, "null argument");
  return instance_profile_read(c, ms_out, launches_out);
}

cell_status cell_solve_hyper(cell_t c, int nload, const double* F_bar, double tol, int max_newton, double* P_out,
                             cell_hyper_info* info) {
  const double t0 = now_s();
  if (!c || !F_bar) return fail(CELL_E_ARG, "null argument");
  if (nload < 1 || nload > c->lpc) return fail(CELL_E_ARG, "nload must be in [1, max_loads]");
  if (!c->have_mat[0]) return fail(CELL_E_STATE, "cell_set_material has not been called");
  if (tol < 0.0 || !std::isfinite(tol) || max_newton < 0) return fail(CELL_E_ARG, "invalid tol or max_newton");
  const int d = c->d;
  for (int j = 0; j < nload; ++j) {
    const double* F = F_bar + j * d * d;
    for (int i = 0; i < d * d; ++i)
      if (!std::isfinite(F[i])) return fail(CELL_E_ARG, "non-finite F_bar");
    const double det = d == 3 ? F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
                                    F[2] * (F[3] * F[7] - F[4] * F[6])
                              : F[0] * F[3] - F[1] * F[2];
    if (!(det > 0.0)) return fail(CELL_E_ARG, "F_bar must have a positive determinant");
  }
  DevGuard dg(c->dev);
  const cell_status st =
      instance_hyper_solve(c, nload, F_bar, tol > 0.0 ? tol : 1e-10, max_newton > 0 ? max_newton : 50, P_out, info);
  if (info) info->seconds = now_s() - t0;
  return st;
}

cell_status cell_apply_hyper_tangent(cell_t c, int precision, const double* F_bar, const double* u, const double* p,
                                     double* q_out) {
  if (!c || !F_bar || !u || !p || !q_out) return fail(CELL_E_ARG, "null argument");
  if (!c->have_mat[0]) return fail(CELL_E_STATE, "cell_set_material has not been called");
  DevGuard dg(c->dev);
  return instance_hyper_step(c, precision, F_bar, u, p, q_out, nullptr);
}

cell_status cell_hyper_residual(cell_t c, const double* F_bar, const double* u, double* f_out, double* sums_out) {
  if (!c || !F_bar || !u || !f_out) return fail(CELL_E_ARG, "null argument");
  if (!c->have_mat[0]) return fail(CELL_E_STATE, "cell_set_material has not been called");
  DevGuard dg(c->dev);
  return instance_hyper_step(c, CELL_FP64, F_bar, u, nullptr, f_out, sums_out);
}

cell_status cell_set_surrogate(cell_t c, int M, int q, double* setup_seconds) {
  if (!c) return fail(CELL_E_ARG, "null argument");
  DevGuard dg(c->dev);
  const cell_status st = instance_set_surrogate(c, M, q);
  if (st >= 0 && setup_seconds) *setup_seconds = c->sr_setup_s;
  return st;
}

cell_status cell_get_surrogate_stencil(cell_t c, double* blocks_out) {
  if (!c || !blocks_out) return fail(CELL_E_ARG, "null argument");
  return instance_get_surrogate(c, blocks_out);
}

cell_status cell_autotune(cell_t c, int force) {
  if (!c) return fail(CELL_E_ARG, "null argument");
  return instance_autotune(c, force);
}

cell_status cell_get_schedule(cell_t c, int* sched_out) {
  if (!c || !sched_out) return fail(CELL_E_ARG, "null argument");
  instance_get_schedule(c, sched_out);
  return CELL_OK;
}

cell_status cell_set_schedule(cell_t c, const int* sched) {
  if (!c || !sched) return fail(CELL_E_ARG, "null argument");
  return instance_set_schedule(c, sched);
}

// ================================================================== batches
void cell_batch_destroy(cell_batch_t b) {
  if (!b) return;
  {
    DevGuard dg(b->dev);
    for (cell_s* c : b->cls) instance_destroy(c);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  }
  delete b;
}

cell_status cell_batch_create(const cell_config* cfgs, int ncell, cell_batch_t* out) {
  if (!cfgs || !out) return fail(CELL_E_ARG, "null argument");
  *out = nullptr;
  if (ncell < 1) return fail(CELL_E_ARG, "ncell must be positive");
  const cell_config& c0 = cfgs[0];
  for (int i = 1; i < ncell; ++i) {
    const cell_config& ci = cfgs[i];
    if (ci.dim != c0.dim || ci.precision != c0.precision || ci.tol != c0.tol || ci.max_iter != c0.max_iter ||
        ci.max_loads != c0.max_loads || ci.stream != c0.stream || ci.device != c0.device)
      return fail(CELL_E_ARG, "batched cells must share dim, precision, tol, max_iter, max_loads, stream and device");
  }
  int dev = c0.device;
  if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return fail(CELL_E_DEVICE, "no HIP device");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(CELL_E_DEVICE, "no HIP device");
  if (dev >= ndev) return fail(CELL_E_ARG, "device ordinal out of range");
  DevGuard dg(dev);
  cell_batch_s* b = new cell_batch_s();
  b->dev = dev;
  auto bail = [&](cell_status s) {
    cell_batch_destroy(b);
    return s;
  };
  if (c0.stream) {
    b->stream = (hipStream_t)c0.stream;
  } else {
    if (hipStreamCreate(&b->stream) != hipSuccess) return bail(fail(CELL_E_DEVICE, "hipStreamCreate failed"));
    b->own_stream = true;
  }
  // group the cells by grid (sizes and edge lengths); one instance per group
  using Key = std::tuple<int, int, int, double, double, double>;
  std::map<Key, std::vector<int>> groups;
  for (int i = 0; i < ncell; ++i) {
    const cell_config& ci = cfgs[i];
    const int nz = ci.dim == 3 ? ci.n[2] : 1;
    const double lz = ci.dim == 3 ? ci.len[2] : 0.0;
    groups[Key(ci.n[0], ci.n[1], nz, ci.len[0], ci.len[1], lz)].push_back(i);
  }
  b->cls_of.assign(ncell, -1);
  b->idx_of.assign(ncell, -1);
  for (auto& kv : groups) {
    cell_config cfg = cfgs[kv.second[0]];
    cfg.device = dev;
    cell_s* c = nullptr;
    const cell_status st = instance_create(&cfg, (int)kv.second.size(), b->stream, &c);
    if (st < 0) return bail(st);
    for (size_t j = 0; j < kv.second.size(); ++j) {
      b->cls_of[kv.second[j]] = (int)b->cls.size();
      b->idx_of[kv.second[j]] = (int)j;
    }
    b->cls.push_back(c);
  }
  b->nv = b->cls[0]->nv;
  *out = b;
  return CELL_OK;
}

cell_status cell_batch_set_material(cell_batch_t b, int cell, const double* E, const double* nu, int on_device) {
  if (!b) return fail(CELL_E_ARG, "null argument");
  if (cell < 0 || cell >= (int)b->cls_of.size()) return fail(CELL_E_ARG, "cell index out of range");
  return instance_set_material(b->cls[b->cls_of[cell]], b->idx_of[cell], E, nu, on_device);
}

namespace {
struct GraphExec {
  hipGraphExec_t g = nullptr;
  void reset() {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  ~GraphExec() { reset(); }
};
}  // namespace

// every instance's PCG advances in lockstep: one chunk of iterations per
// unfinished instance, one stream synchronisation, then the polls.  With
// graphs the chunks of all unfinished instances are one captured graph (in
// instance order, as the eager launches would queue them), captured again
// when an instance finishes
static cell_status batch_run(cell_batch_t b, int nload, const double* eps, std::vector<std::vector<cell_info>>& inf) {
  const int ng = (int)b->cls.size();
  std::vector<SolveRun> runs(ng);
  inf.assign(ng, {});
  for (int k = 0; k < ng; ++k) {
    inf[k].assign(b->cls[k]->ncell, cell_info{});
    STCHK(solve_begin(runs[k], b->cls[k], nload, eps, inf[k].data()));
  }
  GraphExec ge;
  std::vector<int> in_graph;  // the instances the current graph launches
  for (;;) {
    std::vector<int> act;
    bool graphs = true;
    for (int k = 0; k < ng; ++k)
      if (!runs[k].done) {
        act.push_back(k);
        graphs = graphs && solve_graphs(runs[k]);
      }
    if (act.empty()) break;
    if (!graphs) {
      ge.reset();
      for (int k : act) STCHK(solve_launch(runs[k]));
    } else {
      if (!ge.g || act != in_graph) {
        ge.reset();
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        cell_status st = CELL_OK;
        for (size_t i = 0; i < act.size() && st >= 0; ++i) st = solve_enqueue_chunk(runs[act[i]]);
        hipError_t e = hipStreamEndCapture(b->stream, &graph);
        if (st < 0) {
          if (graph) (void)hipGraphDestroy(graph);
          return st;
        }
        if (e != hipSuccess) return fail(CELL_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&ge.g, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
          ge.g = nullptr;
          return fail(CELL_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        in_graph = act;
      }
      HIPCHK(hipGraphLaunch(ge.g, b->stream));
      for (int k : act) STCHK(solve_copy_states(runs[k]));
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    for (int k : act) STCHK(solve_poll(runs[k]));
  }
  cell_status worst = CELL_OK;
  for (int k = 0; k < ng; ++k) {
    const cell_status st = solve_end(runs[k]);
    if (st < 0) return st;
    if (st == CELL_NOT_CONVERGED) worst = st;
  }
  return worst;
}

cell_status cell_batch_solve(cell_batch_t b, int nload, const double* macro_strain, double* mean_stress_out,
                             cell_info* infos) {
  const double t0 = now_s();
  if (!b || !macro_strain) return fail(CELL_E_ARG, "null argument");
  if (nload < 1 || nload > b->cls[0]->lpc) return fail(CELL_E_ARG, "nload must be in [1, max_loads]");
  STCHK(check_strains(nload, b->nv, macro_strain));
  DevGuard dg(b->dev);
  std::vector<std::vector<cell_info>> inf;
  const cell_status st = batch_run(b, nload, macro_strain, inf);
  if (st < 0) return st;
  const int ncell = (int)b->cls_of.size(), nv = b->nv;
  const double dt = now_s() - t0;
  for (int i = 0; i < ncell; ++i) {
    cell_s* c = b->cls[b->cls_of[i]];
    const int j = b->idx_of[i];
    const double* h = homog_of(c, j);
    if (mean_stress_out)
      for (int J = 0; J < nload; ++J)
        for (int q = 0; q < nv; ++q) mean_stress_out[((size_t)i * nload + J) * nv + q] = h[nload * nload + J * nv + q];
    if (infos) {
      infos[i] = inf[b->cls_of[i]][j];
      infos[i].hill_mandel_gap = hill_mandel(c, j);
      infos[i].seconds = dt;
    }
  }
  return st;
}

cell_status cell_batch_effective_stiffness(cell_batch_t b, double* C_out, cell_info* infos) {
  const double t0 = now_s();
  if (!b || !C_out) return fail(CELL_E_ARG, "null argument");
  const int nv = b->nv;
  if (b->cls[0]->lpc < nv) return fail(CELL_E_ARG, "max_loads must be nv for the effective stiffness");
  DevGuard dg(b->dev);
  std::vector<double> eye(nv * nv, 0.0);
  for (int i = 0; i < nv; ++i) eye[i * nv + i] = 1.0;
  std::vector<std::vector<cell_info>> inf;
  const cell_status st = batch_run(b, nv, eye.data(), inf);
  if (st < 0) return st;
  const int ncell = (int)b->cls_of.size();
  const double dt = now_s() - t0;
  for (int i = 0; i < ncell; ++i) {
    cell_s* c = b->cls[b->cls_of[i]];
    const int j = b->idx_of[i];
    double sgap = 0.0;
    unit_results(c, j, C_out + (size_t)i * nv * nv, &sgap);
    if (infos) {
      infos[i] = inf[b->cls_of[i]][j];
      infos[i].sym_gap = sgap;
      infos[i].hill_mandel_gap = hill_mandel(c, j);
      infos[i].seconds = dt;
    }
  }
  return st;
}

cell_status cell_batch_get_displacement(cell_batch_t b, int cell, int load, double* u_out, int on_device) {
  if (!b || !u_out) return fail(CELL_E_ARG, "null argument");
  if (cell < 0 || cell >= (int)b->cls_of.size()) return fail(CELL_E_ARG, "cell index out of range");
  return slot_displacement(b->cls[b->cls_of[cell]], b->idx_of[cell], load, u_out, on_device);
}

cell_status cell_batch_get_residual(cell_batch_t b, int cell, int load, double* r_out, int on_device) {
  if (!b || !r_out) return fail(CELL_E_ARG, "null argument");
  if (cell < 0 || cell >= (int)b->cls_of.size()) return fail(CELL_E_ARG, "cell index out of range");
  return slot_residual(b->cls[b->cls_of[cell]], b->idx_of[cell], load, r_out, on_device);
}

cell_status cell_batch_profile(cell_batch_t b, int enable) {
  if (!b) return fail(CELL_E_ARG, "null argument");
  for (cell_s* c : b->cls) STCHK(instance_profile(c, enable));
  return CELL_OK;
}

cell_status cell_batch_profile_read(cell_batch_t b, double* ms_out, long long* launches_out) {
  if (!b || !ms_out || !launches_out) return fail(CELL_E_ARG, "null argument");
  for (int k = 0; k < CELL_NKERNEL; ++k) {
    ms_out[k] = 0.0;
    launches_out[k] = 0;
  }
  for (cell_s* c : b->cls) {
    double ms[CELL_NKERNEL];
    long long cnt[CELL_NKERNEL];
    STCHK(instance_profile_read(c, ms, cnt));
    for (int k = 0; k < CELL_NKERNEL; ++k) {
      ms_out[k] += ms[k];
      launches_out[k] += cnt[k];
    }
  }
  return CELL_OK;
}

int cell_batch_groups(cell_batch_t b) { return b ? (int)b->cls.size() : 0; }

cell_status cell_batch_autotune(cell_batch_t b, int force) {
  if (!b) return fail(CELL_E_ARG, "null argument");
  for (cell_s* c : b->cls) STCHK(instance_autotune(c, force));
  return CELL_OK;
}

}  // extern "C"
