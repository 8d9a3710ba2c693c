// Surrogate stencil operator (gfx950): the 3D periodic P1 elasticity
// operator with its stencil functions replaced by B-spline interpolants of
// their values at every M-th node (Sec. 3.3, eq. SurrogateRoughDefinition)
// and the symmetric kernel-preserving diagonal of Sec. 3.4 (eq.
// DefinitionOfSurrogateMatrixSymmetricKernel).
//
// With A_d(i) the stencil block coupling node i with node i + d (d one of
// the seven nonzero 0/1 offsets), the surrogate applies
//   q_i = sum_d [ A_d(i) (p_{i+d} - p_i) + A_d(i-d)^T (p_{i-d} - p_i) ]
//         + skew(R_i) p_i,   R_i = sum_d A_d(i) + A_d(i-d)^T,
// skew(X) = (X - X^T) / 2: the off-diagonal blocks, their transposes, and
// minus the symmetric part of the block row sum R_i on the diagonal.  Where
// the interpolated blocks' row sums are not symmetric the translations leave
// the kernel by that small skew part, so the PCG iterates the projected operator P Kt P (P:
// zero nodal mean per component): every launch also returns the component
// means of its output, which the x pass removes from the transform.
#include "kernels.h"

namespace cellfft {

namespace {

__device__ __forceinline__ int swrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// offsets in the stencil order (x, y, z, xy, yz, xz, xyz)
__device__ constexpr int SOFF[SR_NOFF][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0},
                                             {0, 1, 1}, {1, 0, 1}, {1, 1, 1}};

// centred cardinal B-spline of degree 1 or 3
__device__ __forceinline__ double bspl(int q, double x) {
  const double a = fabs(x);
  if (q == 1) return a < 1.0 ? 1.0 - a : 0.0;
  if (a < 1.0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
  if (a < 2.0) {
    const double t = 2.0 - a;
    return t * t * t / 6.0;
  }
  return 0.0;
}

}  // namespace

// value of every stencil function at every node: sum over the lattice
// points j within the spline support of c_j prod_a B_q(i_a / M - j_a)
__global__ __launch_bounds__(NT) void k_sr_expand(const double* coef, int ncx, int ncy, int ncz, int M, int q, Geom g,
                                                  double* s64, float* s32) {
  const long long n = g.n;
  const long long nc = (long long)ncx * ncy * ncz;
  const int np = q + 1;  // lattice points per axis in the support
  for (long long node = (long long)blockIdx.x * NT + threadIdx.x; node < n; node += (long long)gridDim.x * NT) {
    const int i = (int)(node % g.nx), j = (int)((node / g.nx) % g.ny), k = (int)(node / ((long long)g.nx * g.ny));
    const int ix = i / M, iy = j / M, iz = k / M;
    const double tx = (double)(i - ix * M) / M, ty = (double)(j - iy * M) / M, tz = (double)(k - iz * M) / M;
    const int b0 = q == 1 ? 0 : -1;  // first lattice offset in the support
    double wx[4], wy[4], wz[4];
    int jx[4], jy[4], jz[4];
    for (int m = 0; m < np; ++m) {
      wx[m] = bspl(q, tx - (b0 + m));
      wy[m] = bspl(q, ty - (b0 + m));
      wz[m] = bspl(q, tz - (b0 + m));
      jx[m] = ((ix + b0 + m) % ncx + ncx) % ncx;
      jy[m] = ((iy + b0 + m) % ncy + ncy) % ncy;
      jz[m] = ((iz + b0 + m) % ncz + ncz) % ncz;
    }
    for (int v = 0; v < SR_NVAL; ++v) {
      const double* cv = coef + (long long)v * nc;
      double s = 0.0;
      for (int mz = 0; mz < np; ++mz)
        for (int my = 0; my < np; ++my) {
          const double* row = cv + ((long long)jz[mz] * ncy + jy[my]) * ncx;
          const double wzy = wz[mz] * wy[my];
          for (int mx = 0; mx < np; ++mx) s += wzy * wx[mx] * row[jx[mx]];
        }
      s64[(long long)v * n + node] = s;
      s32[(long long)v * n + node] = (float)s;
    }
  }
}

// MODE 0: q = Kt p (T) for the active slots, p.q partials.
// MODE 1: r = f - Kt u (FP64, written as TO) for the masked slots.
// Both: per-block component sums of the output (for its mean).
template <typename T, typename TO, int MODE>
__global__ __launch_bounds__(NT) void k_sr_apply(SArgs<T> a) {
  __shared__ double sh[NT / WAVE];
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const long long n = a.g.n;
  bool live[6];
#pragma unroll
  for (int l = 0; l < 6; ++l)
    live[l] = l < a.nslot && (MODE == 0 ? a.st[l].state == ST_ACTIVE : (a.mask ? a.mask[l] != 0 : true));
  double dot[6] = {0, 0, 0, 0, 0, 0};
  double csum[6][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (long long node = (long long)blockIdx.x * NT + threadIdx.x; node < n; node += (long long)gridDim.x * NT) {
    const int i = (int)(node % nx), j = (int)((node / nx) % ny), k = (int)(node / ((long long)nx * ny));
    T acc[6][3];
#pragma unroll
    for (int l = 0; l < 6; ++l)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[l][c] = T(0);
    // skew part of the block row sum (its diagonal correction)
    T rs[3][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
#pragma unroll
    for (int d = 0; d < SR_NOFF; ++d) {
      const long long jp =
          ((long long)swrap(k + SOFF[d][2], nz) * ny + swrap(j + SOFF[d][1], ny)) * nx + swrap(i + SOFF[d][0], nx);
      const long long jm =
          ((long long)swrap(k - SOFF[d][2], nz) * ny + swrap(j - SOFF[d][1], ny)) * nx + swrap(i - SOFF[d][0], nx);
      T A[3][3], B[3][3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          A[r][c] = a.s[(long long)(9 * d + 3 * r + c) * n + node];  // A_d(i)
          B[r][c] = a.s[(long long)(9 * d + 3 * r + c) * n + jm];    // A_d(i - d)
        }
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) rs[r][c] += A[r][c] + B[c][r];
#pragma unroll
      for (int l = 0; l < 6; ++l) {
        if (!live[l]) continue;
        const T* p = a.p + l * a.lstride;
        T pi[3], dp[3], dm[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          pi[c] = p[c * n + node];
          dp[c] = p[c * n + jp] - pi[c];
          dm[c] = p[c * n + jm] - pi[c];
        }
#pragma unroll
        for (int r = 0; r < 3; ++r)
          acc[l][r] += A[r][0] * dp[0] + A[r][1] * dp[1] + A[r][2] * dp[2] + B[0][r] * dm[0] + B[1][r] * dm[1] +
                       B[2][r] * dm[2];
      }
    }
    // the edge form above applies -R_i to p_i; the diagonal is -sym(R_i):
    // add skew(R_i) p_i
#pragma unroll
    for (int l = 0; l < 6; ++l) {
      if (!live[l]) continue;
      const T* p = a.p + l * a.lstride;
      T pi[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) pi[c] = p[c * n + node];
#pragma unroll
      for (int r = 0; r < 3; ++r)
        acc[l][r] += T(0.5) * ((rs[r][0] - rs[0][r]) * pi[0] + (rs[r][1] - rs[1][r]) * pi[1] +
                               (rs[r][2] - rs[2][r]) * pi[2]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long o = l * a.lstride + c * n + node;
        if (MODE == 0) {
          reinterpret_cast<T*>(a.out)[o] = acc[l][c];
          dot[l] += (double)pi[c] * (double)acc[l][c];
          csum[l][c] += (double)acc[l][c];
        } else {
          const double r = a.rhs[o] - (double)acc[l][c];
          reinterpret_cast<TO*>(a.out)[o] = (TO)r;
          csum[l][c] += r;
        }
      }
    }
  }
  const int nb = gridDim.x;
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    if (!live[l]) continue;  // uniform across the block
    if (MODE == 0) {
      const double s = block_sum<NT>(dot[l], sh);
      if (threadIdx.x == 0) a.red.slot_parts(RED_PQ, l)[blockIdx.x] = s;
    }
    for (int c = 0; c < 3; ++c) {
      const double s = block_sum<NT>(csum[l][c], sh);
      if (threadIdx.x == 0) a.cparts[((long long)l * 3 + c) * nb + blockIdx.x] = s;
    }
  }
}

// component means of the output from the partial sums (fixed order); the
// same liveness as the launch that wrote them
template <int MODE>
__global__ __launch_bounds__(NT) void k_sr_mean(const double* cparts, int nb, long long n, const LoadState* st,
                                                 const int* mask, double* mean) {
  __shared__ double sh[NT / WAVE];
  const int c = blockIdx.x, l = blockIdx.y;
  const bool live = MODE == 0 ? st[l].state == ST_ACTIVE : (mask ? mask[l] != 0 : true);
  if (!live) return;
  const double* row = cparts + ((long long)l * 3 + c) * nb;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += NT) s += row[b];
  s = block_sum<NT>(s, sh);
  if (threadIdx.x == 0) mean[l * 3 + c] = s / (double)n;
}

// r -= mean (per slot and component), ||r||^2 partials
template <typename TO>
__global__ __launch_bounds__(NT) void k_sr_fix(TO* r, long long lstride, long long n, const double* mean,
                                               const int* mask, RedBuf red) {
  __shared__ double sh[NT / WAVE];
  const int l = blockIdx.y;
  if (mask && mask[l] == 0) return;
  TO* v = r + (long long)l * lstride;
  double s = 0.0;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < 3 * n; e += (long long)gridDim.x * NT) {
    const double x = (double)v[e] - mean[l * 3 + (int)(e / n)];
    v[e] = (TO)x;
    s += x * x;
  }
  s = block_sum<NT>(s, sh);
  if (threadIdx.x == 0) red.slot_parts(RED_RES, l)[blockIdx.x] = s;
}

hipError_t launch_sr_expand(const double* coef, int ncx, int ncy, int ncz, int M, int q, const Geom& g, double* s64,
                            float* s32, hipStream_t s) {
  const long long nb = (g.n + NT - 1) / NT;
  hipLaunchKernelGGL(k_sr_expand, dim3((unsigned)(nb < 65535 ? nb : 65535)), dim3(NT), 0, s, coef, ncx, ncy, ncz, M, q,
                     g, s64, s32);
  return hipGetLastError();
}

static int sr_blocks(const Geom& g, int maxblk) {
  long long nb = (g.n + NT - 1) / NT;
  if (nb > 4096) nb = 4096;
  if (nb > maxblk) nb = maxblk;
  return (int)nb;
}

template <typename T>
hipError_t launch_sr_apply(const SArgs<T>& a, hipStream_t s) {
  if (a.nslot > 6) return hipErrorInvalidValue;
  const int nb = sr_blocks(a.g, a.red.maxblk);
  hipLaunchKernelGGL((k_sr_apply<T, T, 0>), dim3(nb), dim3(NT), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sr_mean<0>, dim3(3, a.nslot), dim3(NT), 0, s, (const double*)a.cparts, nb,
                     a.g.n, (const LoadState*)a.st, (const int*)nullptr, a.mean);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(a.red, a.st, nullptr, RED_PQ, nb, a.nslot, -1, nullptr, s);
}

hipError_t launch_sr_residual(const SArgs<double>& a, bool out32, double* res2, hipStream_t s) {
  if (a.nslot > 6) return hipErrorInvalidValue;
  const int nb = sr_blocks(a.g, a.red.maxblk);
  if (out32) hipLaunchKernelGGL((k_sr_apply<double, float, 1>), dim3(nb), dim3(NT), 0, s, a);
  else hipLaunchKernelGGL((k_sr_apply<double, double, 1>), dim3(nb), dim3(NT), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sr_mean<1>, dim3(3, a.nslot), dim3(NT), 0, s, (const double*)a.cparts, nb,
                     a.g.n, (const LoadState*)a.st, a.mask, a.mean);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nf = a.red.maxblk < 1024 ? a.red.maxblk : 1024;
  if (out32)
    hipLaunchKernelGGL(k_sr_fix<float>, dim3(nf, a.nslot), dim3(NT), 0, s, static_cast<float*>(a.out), a.lstride,
                       a.g.n, (const double*)a.mean, a.mask, a.red);
  else
    hipLaunchKernelGGL(k_sr_fix<double>, dim3(nf, a.nslot), dim3(NT), 0, s, static_cast<double*>(a.out), a.lstride,
                       a.g.n, (const double*)a.mean, a.mask, a.red);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(a.red, a.st, res2, RED_RES, nf, a.nslot, -1, a.mask, s);
}

template hipError_t launch_sr_apply<float>(const SArgs<float>&, hipStream_t);
template hipError_t launch_sr_apply<double>(const SArgs<double>&, hipStream_t);

}  // namespace cellfft
