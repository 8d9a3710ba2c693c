// Strain-based Fourier projection variant of the cell solve (3D, FP64).
//
// Conjugate gradients on compatible strain fields e = B u, one Voigt strain
// per Kuhn simplex (six per voxel), instead of nodal displacements:
//   A e = B M^-1 B^T D e,   M = B^T D0 B (the Fourier reference operator),
//   <a, b>_0 = sum_s |s| a_s . D0 b_s  (D0: the reference medium).
// On compatible fields A is self-adjoint and positive for <., .>_0, and
// <B z, B z>_0 = z.M z, <A B p, B p>_0 = p.K p, so the iterates are B u_k of
// the displacement PCG with the same preconditioner: same alpha, beta and
// iteration count when stopped on the same residual ||f - K u_k||.  It moves
// 36 strain values per voxel and array (about twelve times the bytes of a
// displacement-PCG iteration): a cross-check of the iteration, run by the
// host one step at a time, not a production path.
//
// Kernels: strains of a nodal field (B z), nodal divergence of the stresses
// of a strain field (B^T D p, voxel corner forces then a fixed-order
// eight-voxel gather), the <., .>_0 and ||.||^2 partial sums, vector
// updates.  The preconditioner is the instance's FFT passes on slot 0.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "solver.h"

namespace cellfft {

namespace {

#define STCHK(call)          \
  do {                       \
    cell_status s_ = (call); \
    if (s_ < 0) return s_;   \
  } while (0)

constexpr int SP_NV = 36;  // 6 simplices x 6 Voigt components per voxel

__constant__ int kSpPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

__device__ __forceinline__ int spwrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ long long sp_node(const Geom& g, int i, int j, int k) {
  return ((long long)spwrap(k, g.nz) * g.ny + spwrap(j, g.ny)) * g.nx + spwrap(i, g.nx);
}

// e[v][t][6] = B_t z on voxel v (engineering shear); adds e_bar if given
__global__ __launch_bounds__(NT) void k_sp_strain(Geom g, const double* z, const double* ebar, double* e) {
  const long long n = g.n;
  for (long long v = (long long)blockIdx.x * NT + threadIdx.x; v < n; v += (long long)gridDim.x * NT) {
    const int i = (int)(v % g.nx), j = (int)((v / g.nx) % g.ny), k = (int)(v / ((long long)g.nx * g.ny));
    double u[8][3];
    for (int c = 0; c < 8; ++c) {
      const long long nd = sp_node(g, i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1));
      for (int q = 0; q < 3; ++q) u[c][q] = z[q * n + nd];
    }
    for (int t = 0; t < 6; ++t) {
      double G[3][3];
      int cn = 0;
      for (int s = 0; s < 3; ++s) {
        const int ax = kSpPerm[t][s];
        const int nx = cn | (1 << ax);
        for (int q = 0; q < 3; ++q) G[q][ax] = (u[nx][q] - u[cn][q]) / g.h[ax];
        cn = nx;
      }
      double* out = e + (v * 6 + t) * 6;
      out[0] = G[0][0];
      out[1] = G[1][1];
      out[2] = G[2][2];
      out[3] = G[1][2] + G[2][1];
      out[4] = G[0][2] + G[2][0];
      out[5] = G[0][1] + G[1][0];
      if (ebar)
        for (int c = 0; c < 6; ++c) out[c] += ebar[c];
    }
  }
}

// corner forces of voxel v: cf[v][corner][3] = sum_t |s| B_t^T D_v e_t
// (e_t + ebar if ebar is given)
__global__ __launch_bounds__(NT) void k_sp_corner(Geom g, const double* mat, const double* e, const double* ebar,
                                                  double* cf) {
  const long long n = g.n;
  const double vol = g.h[0] * g.h[1] * g.h[2] / 6.0;
  for (long long v = (long long)blockIdx.x * NT + threadIdx.x; v < n; v += (long long)gridDim.x * NT) {
    const double lam = mat[2 * v], mu = mat[2 * v + 1];
    double f[8][3] = {};
    for (int t = 0; t < 6; ++t) {
      const double* et = e + (v * 6 + t) * 6;
      double s[6];
      for (int c = 0; c < 6; ++c) s[c] = et[c] + (ebar ? ebar[c] : 0.0);
      const double tr = s[0] + s[1] + s[2];
      // stress tensor from the Voigt strain (engineering shear)
      double S[3][3];
      S[0][0] = lam * tr + 2.0 * mu * s[0];
      S[1][1] = lam * tr + 2.0 * mu * s[1];
      S[2][2] = lam * tr + 2.0 * mu * s[2];
      S[1][2] = S[2][1] = mu * s[3];
      S[0][2] = S[2][0] = mu * s[4];
      S[0][1] = S[1][0] = mu * s[5];
      // the gradient column along the path's step j is the difference of
      // its end and start corners over h: its flux goes from start to end
      int cn = 0;
      for (int st = 0; st < 3; ++st) {
        const int ax = kSpPerm[t][st];
        const int nx = cn | (1 << ax);
        const double w = vol / g.h[ax];
        for (int q = 0; q < 3; ++q) {
          f[nx][q] += w * S[q][ax];
          f[cn][q] -= w * S[q][ax];
        }
        cn = nx;
      }
    }
    for (int c = 0; c < 8; ++c)
      for (int q = 0; q < 3; ++q) cf[(v * 8 + c) * 3 + q] = f[c][q];
  }
}

// out[q][i] = sign * sum over the eight voxels holding node i of their
// corner forces at i (fixed order)
__global__ __launch_bounds__(NT) void k_sp_gather(Geom g, const double* cf, double sign, double* out) {
  const long long n = g.n;
  for (long long nd = (long long)blockIdx.x * NT + threadIdx.x; nd < n; nd += (long long)gridDim.x * NT) {
    const int i = (int)(nd % g.nx), j = (int)((nd / g.nx) % g.ny), k = (int)(nd / ((long long)g.nx * g.ny));
    double acc[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < 8; ++c) {
      const long long v = sp_node(g, i - (c & 1), j - ((c >> 1) & 1), k - ((c >> 2) & 1));
      for (int q = 0; q < 3; ++q) acc[q] += cf[(v * 8 + c) * 3 + q];
    }
    for (int q = 0; q < 3; ++q) out[q * n + nd] = sign * acc[q];
  }
}

// per-block partials of <a, b>_0 (mode 0, strain fields, reference medium
// lam0, mu0), ||a||^2 over m values (mode 1), or the stress sums
// sum |s| D_v (ebar + a_t) per Voigt component (mode 2, six partial rows)
__global__ __launch_bounds__(NT) void k_sp_reduce(int mode, Geom g, const double* a, const double* b, long long m,
                                                  double lam0, double mu0, const double* mat, const double* ebar,
                                                  double* parts) {
  __shared__ double sh[NT / WAVE];
  const double vol = g.h[0] * g.h[1] * g.h[2] / 6.0;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (long long x = (long long)blockIdx.x * NT + threadIdx.x; x < m; x += (long long)gridDim.x * NT) {
    if (mode == 1) {
      acc[0] += a[x] * a[x];
    } else {
      // x indexes a (voxel, simplex) strain
      const double* p = a + x * 6;
      double s[6];
      for (int c = 0; c < 6; ++c) s[c] = p[c] + (mode == 2 ? ebar[c] : 0.0);
      const double la = mode == 2 ? mat[2 * (x / 6)] : lam0, mu = mode == 2 ? mat[2 * (x / 6) + 1] : mu0;
      const double tr = s[0] + s[1] + s[2];
      double S[6];
      for (int c = 0; c < 3; ++c) S[c] = la * tr + 2.0 * mu * s[c];
      for (int c = 3; c < 6; ++c) S[c] = mu * s[c];
      if (mode == 0) {
        const double* q = b + x * 6;
        acc[0] += vol * (q[0] * S[0] + q[1] * S[1] + q[2] * S[2] + q[3] * S[3] + q[4] * S[4] + q[5] * S[5]);
      } else {
        for (int c = 0; c < 6; ++c) acc[c] += vol * S[c];
      }
    }
  }
  const int rows = mode == 2 ? 6 : 1;
  for (int r = 0; r < rows; ++r) {
    const double s = block_sum<NT>(acc[r], sh);
    if (threadIdx.x == 0) parts[r * gridDim.x + blockIdx.x] = s;
  }
}

// y = a x + b y over m values
__global__ __launch_bounds__(NT) void k_sp_axpby(long long m, double a, const double* x, double b, double* y) {
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < m; i += (long long)gridDim.x * NT)
    y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];  // b = 0: y need not hold numbers
}

constexpr int SP_BLOCKS = 1024;

}  // namespace

// strain-projection CG for nload macro strains (host [nload][6]); mean
// stresses out [nload][6]; infos: iterations and final relative residuals
cell_status instance_solve_projection(cell_s* c, int nload, const double* eps, double* stress_out, cell_info* info) {
  if (c->d != 3) return fail(CELL_E_UNSUPPORTED, "the strain-based projection variant is implemented in 3D");
  if (c->ncell != 1) return fail(CELL_E_UNSUPPORTED, "the strain-based projection variant needs a single-cell handle");
  if (!c->have_mat[0]) return fail(CELL_E_STATE, "cell_set_material has not been called");
  if (c->op != 0) return fail(CELL_E_STATE, "the strain-based projection variant needs the exact operator");
  const Geom g = c->g;
  const long long n = g.n;
  const long long ms = n * SP_NV;
  hipStream_t s = c->stream;
  c->solved = c->solved_unit = c->linear_results = false;
  // scratch: strains e, p, rho, Ap; nodal r, w, z; corner forces; partials
  std::vector<void*> bufs;
  auto dalloc = [&](size_t bytes) -> double* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    bufs.push_back(p);
    return static_cast<double*>(p);
  };
  struct Free {
    std::vector<void*>& b;
    hipStream_t s;
    ~Free() {
      (void)hipStreamSynchronize(s);  // no launch may still use the buffers
      for (void* p : b) (void)hipFree(p);
    }
  } freer{bufs, s};
  double* e = dalloc(sizeof(double) * ms);
  double* p = dalloc(sizeof(double) * ms);
  double* rho = dalloc(sizeof(double) * ms);
  double* Ap = dalloc(sizeof(double) * ms);
  double* r = dalloc(sizeof(double) * 3 * n);
  double* w = dalloc(sizeof(double) * 3 * n);
  double* zb = dalloc(sizeof(double) * 3 * n);
  double* cf = dalloc(sizeof(double) * 24 * n);
  double* parts = dalloc(sizeof(double) * 6 * SP_BLOCKS);
  double* ebar_d = dalloc(sizeof(double) * 6);
  if (!e || !p || !rho || !Ap || !r || !w || !zb || !cf || !parts || !ebar_d)
    return fail(CELL_E_NOMEM, "device allocation for the strain-based projection variant failed");
  {
    const cell_status st = instance_precond_prepare(c);
    if (st < 0) return st;
  }
  const double lam0 = c->lam0[0], mu0 = c->mu0[0];
  const dim3 grid(SP_BLOCKS), blk(NT);
  std::vector<double> ph(6 * SP_BLOCKS);
  auto reduce = [&](int mode, const double* a, const double* b, long long m, const double* eb, double* res) -> cell_status {
    hipLaunchKernelGGL(k_sp_reduce, grid, blk, 0, s, mode, g, a, b, m, lam0, mu0, (const double*)c->mat64, eb, parts);
    if (hipGetLastError() != hipSuccess) return fail(CELL_E_DEVICE, "strain projection reduction launch failed");
    const int rows = mode == 2 ? 6 : 1;
    if (hipMemcpyAsync(ph.data(), parts, sizeof(double) * rows * SP_BLOCKS, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(CELL_E_DEVICE, "strain projection reduction failed");
    for (int rr = 0; rr < rows; ++rr) {
      double acc = 0.0;
      for (int b2 = 0; b2 < SP_BLOCKS; ++b2) acc += ph[rr * SP_BLOCKS + b2];
      res[rr] = acc;
    }
    return CELL_OK;
  };
  // nodal divergence of the stresses of a strain field: out = sign B^T D (e + ebar)
  auto divergence = [&](const double* ef, const double* eb, double sign, double* out) -> cell_status {
    hipLaunchKernelGGL(k_sp_corner, grid, blk, 0, s, g, (const double*)c->mat64, ef, eb, cf);
    hipLaunchKernelGGL(k_sp_gather, grid, blk, 0, s, g, (const double*)cf, sign, out);
    return hipGetLastError() == hipSuccess ? CELL_OK : fail(CELL_E_DEVICE, "strain projection divergence failed");
  };
  auto strain_of = [&](const double* z, double* out) -> cell_status {
    hipLaunchKernelGGL(k_sp_strain, grid, blk, 0, s, g, z, (const double*)nullptr, out);
    return hipGetLastError() == hipSuccess ? CELL_OK : fail(CELL_E_DEVICE, "strain projection gradient failed");
  };
  auto axpby = [&](long long m, double a, const double* x, double b, double* y) -> cell_status {
    hipLaunchKernelGGL(k_sp_axpby, grid, blk, 0, s, m, a, x, b, y);
    return hipGetLastError() == hipSuccess ? CELL_OK : fail(CELL_E_DEVICE, "strain projection update failed");
  };
  cell_status result = CELL_OK;
  if (info) std::memset(info, 0, sizeof(cell_info));
  for (int J = 0; J < nload; ++J) {
    double eb[6];
    for (int q = 0; q < 6; ++q) eb[q] = eps[J * 6 + q];
    // eb stays alive until the copy has run: the reductions below synchronise
    // the stream before the next load overwrites it
    if (hipMemcpyAsync(ebar_d, eb, sizeof(eb), hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(CELL_E_DEVICE, "strain projection upload failed");
    // f = -B^T D ebar, e = 0
    if (hipMemsetAsync(e, 0, sizeof(double) * ms, s) != hipSuccess)
      return fail(CELL_E_DEVICE, "strain projection memset failed");
    STCHK(divergence(e, ebar_d, -1.0, r));
    double fn2 = 0.0;
    STCHK(reduce(1, r, nullptr, 3 * n, nullptr, &fn2));
    int it = 0;
    double rel = 0.0;
    // the homogeneous-cell test of the displacement path (f = 0 up to round-off)
    double emax = 0.0;
    for (int q = 0; q < 6; ++q) emax = std::max(emax, std::fabs(eb[q]));
    const double hmin = std::min(g.h[0], std::min(g.h[1], g.h[2]));
    const double fscale = std::sqrt((double)n) * g.h[0] * g.h[1] * g.h[2] * c->maxmod[0] * emax / hmin;
    if (std::sqrt(fn2) > 1e-13 * fscale) {
      // rho = B M^-1 r, p = rho, gamma = <rho, rho>_0
      STCHK(instance_precond_device(c, r, zb));
      STCHK(strain_of(zb, rho));
      STCHK(axpby(ms, 1.0, rho, 0.0, p));
      double gam = 0.0;
      STCHK(reduce(0, rho, rho, 6 * n, nullptr, &gam));
      double rr = fn2;
      while (it < c->max_iter) {
        STCHK(divergence(p, nullptr, 1.0, w));  // w = B^T D p
        STCHK(instance_precond_device(c, w, zb));
        STCHK(strain_of(zb, Ap));               // Ap = B M^-1 B^T D p
        double pAp = 0.0;
        STCHK(reduce(0, Ap, p, 6 * n, nullptr, &pAp));
        if (!(pAp > 0.0) || !std::isfinite(pAp)) {
          result = fail(CELL_E_BREAKDOWN, "strain projection CG breakdown");
          break;
        }
        const double alpha = gam / pAp;
        STCHK(axpby(ms, alpha, p, 1.0, e));
        STCHK(axpby(ms, -alpha, Ap, 1.0, rho));
        STCHK(axpby(3 * n, -alpha, w, 1.0, r));  // r = f - K u_k
        ++it;
        STCHK(reduce(1, r, nullptr, 3 * n, nullptr, &rr));
        if (rr <= c->tol * c->tol * fn2) break;
        double gnew = 0.0;
        STCHK(reduce(0, rho, rho, 6 * n, nullptr, &gnew));
        const double beta = gnew / gam;
        gam = gnew;
        STCHK(axpby(ms, 1.0, rho, beta, p));
      }
      rel = std::sqrt(rr / fn2);
    }
    if (result < 0) return result;
    if (rel > c->tol) result = CELL_NOT_CONVERGED;
    // mean stress (1/|Y|) sum |s| D (ebar + e)
    double sb[6];
    STCHK(reduce(2, e, nullptr, 6 * n, ebar_d, sb));
    const double Y = g.h[0] * g.h[1] * g.h[2] * (double)n;
    if (stress_out)
      for (int q = 0; q < 6; ++q) stress_out[J * 6 + q] = sb[q] / Y;
    if (info && J < 6) {
      info->iters[J] = it;
      info->relres[J] = rel;
      info->nload = nload;
    }
  }
  return result;
}

}  // namespace cellfft
