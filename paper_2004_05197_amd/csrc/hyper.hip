// Compressible neo-Hookean cell problem (gfx950): the nonlinear residual,
// the tangent operator and the small vector kernels of Newton's method.
//
// Energy density (Sec. 2.2, eq. NeoHookeanEnergy), J = det F:
//   W(F) = lambda/2 (ln J)^2 - mu ln J + mu/2 (|F|^2 - d),
//   P(F) = mu (F - F^-T) + lambda ln J F^-T,
//   dP   = mu dF + (mu - lambda ln J) F^-T dF^T F^-T + lambda tr(F^-1 dF) F^-T,
// with F = F_bar + grad u on every simplex of the Kuhn subdivision (2D: the
// in-plane block, plane strain).  On simplex s with axis order
// (p_0, .., p_{d-1}) and path vertices v_0 = 0, v_{k+1} = v_k + e_{p_k},
// grad u has the columns (u(v_{k+1}) - u(v_k)) / h_{p_k} and the
// barycentric gradient of v_k is e_{p_{k-1}}/h_{p_{k-1}} - e_{p_k}/h_{p_k}.
//
// The kernels are node-centric gathers: every thread owns one node and sums
// the contributions of the simplices of its 2^d voxels that contain it, so
// each output is written once, without atomics (deterministic).
//   MODE 0: q = K_T(u) p, p.q partials                     (T = float/double)
//   MODE 1: r = rhs - K_T(u) du, ||r||^2 partials          (FP64, r as TO)
//   MODE 2: f = -sum |s| B^T P(F), ||f||^2 partials, and per own voxel the
//           sums of |s| W and |s| P (energy, mean stress)  (FP64)
#include "kernels.h"

namespace cellfft {

namespace {

__device__ __forceinline__ int hwrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <int D> struct KuhnPerm;
template <> struct KuhnPerm<3> {
  static constexpr int n = 6;
  static constexpr int p[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
};
template <> struct KuhnPerm<2> {
  static constexpr int n = 2;
  static constexpr int p[2][2] = {{0, 1}, {1, 0}};
};

// inverse (cofactor / det), det
template <typename T>
__device__ __forceinline__ T inv3(const T (&F)[3][3], T (&Fi)[3][3]) {
  const T c00 = F[1][1] * F[2][2] - F[1][2] * F[2][1];
  const T c01 = F[1][2] * F[2][0] - F[1][0] * F[2][2];
  const T c02 = F[1][0] * F[2][1] - F[1][1] * F[2][0];
  const T det = F[0][0] * c00 + F[0][1] * c01 + F[0][2] * c02;
  const T id = T(1) / det;
  Fi[0][0] = c00 * id;
  Fi[1][0] = c01 * id;
  Fi[2][0] = c02 * id;
  Fi[0][1] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) * id;
  Fi[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) * id;
  Fi[2][1] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) * id;
  Fi[0][2] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) * id;
  Fi[1][2] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) * id;
  Fi[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) * id;
  return det;
}

// Tangent arithmetic.  FP32: the hardware reciprocal and logarithm (about
// 1 ulp).  FP64 with FASTLN (the FP64 residual refreshes of mixed-precision
// solves, whose iterated operator is the FP32 tangent anyway): a reciprocal
// refined by one Newton step (FP64-accurate) and ln J to FP32 accuracy, which
// only perturbs the coefficient mu - lambda ln J, by ~1e-7 relative, the
// size of the FP32 tangent's own rounding.  FP64 otherwise: the correctly
// rounded division and log (the FP64 solve iterates this same operator).
template <bool FASTLN> __device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
template <bool FASTLN> __device__ __forceinline__ double rcp_t(double x) {
  if constexpr (FASTLN) {
    const double r = (double)__builtin_amdgcn_rcpf((float)x);
    return r * (2.0 - x * r);
  } else {
    return 1.0 / x;
  }
}
template <bool FASTLN> __device__ __forceinline__ float log_t(float x) { return __logf(x); }
template <bool FASTLN> __device__ __forceinline__ double log_t(double x) {
  if constexpr (FASTLN) return (double)__logf((float)x);
  else return log(x);
}

// inverse via cofactors and rcp_t(det); returns det
template <bool FASTLN, typename T>
__device__ __forceinline__ T inv3r(const T (&F)[3][3], T (&Fi)[3][3]) {
  const T c00 = F[1][1] * F[2][2] - F[1][2] * F[2][1];
  const T c01 = F[1][2] * F[2][0] - F[1][0] * F[2][2];
  const T c02 = F[1][0] * F[2][1] - F[1][1] * F[2][0];
  const T det = F[0][0] * c00 + F[0][1] * c01 + F[0][2] * c02;
  const T id = rcp_t<FASTLN>(det);
  Fi[0][0] = c00 * id;
  Fi[1][0] = c01 * id;
  Fi[2][0] = c02 * id;
  Fi[0][1] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) * id;
  Fi[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) * id;
  Fi[2][1] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) * id;
  Fi[0][2] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) * id;
  Fi[1][2] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) * id;
  Fi[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) * id;
  return det;
}

template <typename T>
__device__ __forceinline__ T inv2(const T (&F)[2][2], T (&Fi)[2][2]) {
  const T det = F[0][0] * F[1][1] - F[0][1] * F[1][0];
  const T id = T(1) / det;
  Fi[0][0] = F[1][1] * id;
  Fi[1][1] = F[0][0] * id;
  Fi[0][1] = -F[0][1] * id;
  Fi[1][0] = -F[1][0] * id;
  return det;
}

template <typename T, int D>
__device__ __forceinline__ T invD(const T (&F)[D][D], T (&Fi)[D][D]) {
  if constexpr (D == 3) return inv3(F, Fi);
  else return inv2(F, Fi);
}

}  // namespace

template <typename T, typename TO, int MODE, int D>
__global__ __launch_bounds__(NT) void k_hyper(HyArgs<T> a) {
  __shared__ double sh[NT / WAVE];
  constexpr int NCORN = 1 << D;
  const int l = blockIdx.y;
  bool live;
  if (MODE == 0) live = a.st[l].state == ST_ACTIVE;
  else live = a.mask ? a.mask[l] != 0 : true;
  if (!live) return;
  const Geom& g = a.g;
  const int nx = g.nx, ny = g.ny, nz = D == 3 ? g.nz : 1;
  const long long n = g.n;
  T ih[3] = {T(1.0 / g.h[0]), T(1.0 / g.h[1]), T(1.0 / g.h[2])};
  const T vol = T(D == 3 ? g.h[0] * g.h[1] * g.h[2] / 6.0 : g.h[0] * g.h[1] / 2.0);
  const T* u = a.u + l * a.lstride;
  const T* p = a.p ? a.p + l * a.lstride : nullptr;
  const T* matl = a.mat + (long long)(l / a.lpc) * a.mat_stride;
  T Fb[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) Fb[i][j] = (T)a.Fbar[l * 9 + i * 3 + j];
  double acc = 0.0;
  double own[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};  // MODE 2: |s| W, |s| P (row-major 3 x 3)
  for (long long node = (long long)blockIdx.x * NT + threadIdx.x; node < n; node += (long long)gridDim.x * NT) {
    const int i = (int)(node % nx);
    const int j = (int)((node / nx) % ny);
    const int k = D == 3 ? (int)(node / ((long long)nx * ny)) : 0;
    T force[D];
#pragma unroll
    for (int c = 0; c < D; ++c) force[c] = T(0);
    // the node is corner `cn` of the voxel at node - offset(cn) (cn is
    // uniform across the block; the simplex loop is unrolled, the corner
    // loop is not, to keep the register footprint of one voxel)
#pragma unroll 1
    for (int cn = 0; cn < NCORN; ++cn) {
      const int vi = hwrap(i - (cn & 1), nx), vj = hwrap(j - ((cn >> 1) & 1), ny);
      const int vk = D == 3 ? hwrap(k - ((cn >> 2) & 1), nz) : 0;
      const long long vid = ((long long)vk * ny + vj) * nx + vi;
      const T lam = matl[2 * vid], mu = matl[2 * vid + 1];
      T uu[NCORN][D], pp[NCORN][D];
#pragma unroll
      for (int q = 0; q < NCORN; ++q) {
        const long long nd = ((long long)(D == 3 ? hwrap(vk + ((q >> 2) & 1), nz) : 0) * ny +
                              hwrap(vj + ((q >> 1) & 1), ny)) * nx + hwrap(vi + (q & 1), nx);
#pragma unroll
        for (int c = 0; c < D; ++c) {
          uu[q][c] = u[c * n + nd];
          pp[q][c] = (MODE != 2 && p) ? p[c * n + nd] : T(0);
        }
      }
#pragma unroll
      for (int t = 0; t < KuhnPerm<D>::n; ++t) {
        int path[D + 1];
        path[0] = 0;
#pragma unroll
        for (int m = 0; m < D; ++m) path[m + 1] = path[m] | (1 << KuhnPerm<D>::p[t][m]);
        bool on_path = false;
#pragma unroll
        for (int m = 0; m <= D; ++m) on_path = on_path || path[m] == cn;
        const bool own_voxel = MODE == 2 && cn == 0;
        if (!on_path && !own_voxel) continue;
        // F = F_bar + grad u, dG = grad p
        T F[D][D], dG[D][D];
#pragma unroll
        for (int m = 0; m < D; ++m) {
          const int ax = KuhnPerm<D>::p[t][m];
#pragma unroll
          for (int c = 0; c < D; ++c) {
            F[c][ax] = Fb[c][ax] + (uu[path[m + 1]][c] - uu[path[m]][c]) * ih[ax];
            dG[c][ax] = (pp[path[m + 1]][c] - pp[path[m]][c]) * ih[ax];
          }
        }
        T Fi[D][D];
        const T J = invD<T, D>(F, Fi);
        const T lnJ = J > T(0) ? log(J) : T(NAN);
        T P[D][D];
        if (MODE == 2) {
          T ff = T(0);
#pragma unroll
          for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) {
              P[r][c] = mu * (F[r][c] - Fi[c][r]) + lam * lnJ * Fi[c][r];
              ff += F[r][c] * F[r][c];
            }
          if (own_voxel) {
            own[0] += (double)(vol * (T(0.5) * lam * lnJ * lnJ - mu * lnJ + T(0.5) * mu * (ff - T(D))));
#pragma unroll
            for (int r = 0; r < D; ++r)
#pragma unroll
              for (int c = 0; c < D; ++c) own[1 + r * 3 + c] += (double)(vol * P[r][c]);
          }
        } else {
          // dP = mu dG + (mu - lam lnJ) (Fi dG Fi)^T + lam tr(Fi dG) Fi^T
          T M[D][D], tr = T(0);
#pragma unroll
          for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) {
              T s1 = T(0);
#pragma unroll
              for (int x = 0; x < D; ++x) s1 += Fi[r][x] * dG[x][c];
              M[r][c] = s1;  // (Fi dG)_rc
            }
#pragma unroll
          for (int r = 0; r < D; ++r) tr += M[r][r];
          T N[D][D];
#pragma unroll
          for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) {
              T s1 = T(0);
#pragma unroll
              for (int x = 0; x < D; ++x) s1 += M[r][x] * Fi[x][c];
              N[r][c] = s1;  // (Fi dG Fi)_rc
            }
          const T cm = mu - lam * lnJ, cl = lam * tr;
#pragma unroll
          for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) P[r][c] = mu * dG[r][c] + cm * N[c][r] + cl * Fi[c][r];
        }
        // node force: |s| P g_m for the path vertex v_m = this corner,
        // g_m = e_{p_{m-1}}/h_{p_{m-1}} - e_{p_m}/h_{p_m}
#pragma unroll
        for (int m = 0; m <= D; ++m) {
          if (path[m] != cn) continue;
#pragma unroll
          for (int c = 0; c < D; ++c) {
            T v = T(0);
            if (m > 0) v += P[c][KuhnPerm<D>::p[t][m > 0 ? m - 1 : 0]] * ih[KuhnPerm<D>::p[t][m > 0 ? m - 1 : 0]];
            if (m < D) v -= P[c][KuhnPerm<D>::p[t][m < D ? m : 0]] * ih[KuhnPerm<D>::p[t][m < D ? m : 0]];
            force[c] += vol * v;
          }
        }
      }
    }
    // outputs
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const long long o = l * a.lstride + c * n + node;
      if (MODE == 0) {
        reinterpret_cast<TO*>(a.out)[o] = (TO)force[c];
        acc += (double)(p ? p[c * n + node] : T(0)) * (double)force[c];
      } else if (MODE == 1) {
        const double rv = a.rhs[o] - (double)force[c];
        reinterpret_cast<TO*>(a.out)[o] = (TO)rv;
        acc += rv * rv;
      } else {
        const double fv = -(double)force[c];
        reinterpret_cast<double*>(a.out)[o] = fv;
        acc += fv * fv;
      }
    }
  }
  const double bs = block_sum<NT>(acc, sh);
  if (threadIdx.x == 0) a.red.put(MODE == 0 ? RED_PQ : RED_RES, l, blockIdx.x, bs);
  if (MODE == 2) {
    for (int v = 0; v < 10; ++v) {
      const double s = block_sum<NT>(own[v], sh);
      if (threadIdx.x == 0) a.vparts[((long long)l * 10 + v) * a.red.maxblk + blockIdx.x] = s;
    }
  }
}

// =========================================== tiled tangent product (3D)
// Voxel-centric form of K_T(u) p: every simplex is evaluated once per tile
// (plus the one-voxel halo on the low x and y sides) instead of once per
// vertex.  Block: BX x BY node tile marching tz node planes along z; the u
// and p values of node planes k and k+1 sit in LDS.  Per voxel layer k every
// thread evaluates voxel (tx-1, ty-1) (whose corner (1,1,*) is its own node)
// and keeps the (1,1,*) corner forces; the BX+BY+1 halo voxels go to the
// first threads.  Corner forces (0,0,*), (1,0,*), (0,1,*) are exchanged
// through LDS; the (.,.,1) corners are carried to the next plane.

// nodal forces of one voxel: f[corner][c] += K_T-product contributions of
// the six Kuhn simplices (corners as bit masks x | y << 1 | z << 2); u and p
// of corner (ox, oy, oz) at lds[oz][field * 3 + c][base + oy * PW + ox].
// lam, mu arrive multiplied by w: |s| h^-2 on uniform grids (UNI: all
// 1/h factors of grad p, dP and the nodal gradient folded into w), |s| else.
template <typename T, int PW, int PP, bool UNI, bool FASTLN>
__device__ __forceinline__ void hyper_voxel3(const T* pl0, const T* pl1, int base, const T (&Fb)[3][3], T lamw,
                                             T muw, const T (&ih)[3], T (&f)[8][3]) {
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) f[q][c] = T(0);
  auto ld = [&](int q, int fld, int c) -> T {
    const T* pl = (q & 4) ? pl1 : pl0;
    return pl[(fld * 3 + c) * PP + base + ((q >> 1) & 1) * PW + (q & 1)];
  };
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    constexpr int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int path[4];
    path[0] = 0;
#pragma unroll
    for (int m = 0; m < 3; ++m) path[m + 1] = path[m] | (1 << perm[t][m]);
    // F = F_bar + grad u; dG = grad p (UNI: h dG, the edge differences)
    T F[3][3], dG[3][3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int ax = perm[t][m];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        F[c][ax] = Fb[c][ax] + (ld(path[m + 1], 0, c) - ld(path[m], 0, c)) * ih[ax];
        const T dp = ld(path[m + 1], 1, c) - ld(path[m], 1, c);
        dG[c][ax] = UNI ? dp : dp * ih[ax];
      }
    }
    T Fi[3][3];
    const T J = inv3r<FASTLN>(F, Fi);
    const T lnJ = J > T(0) ? log_t<FASTLN>(J) : T(NAN);
    T M[3][3], tr = T(0);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) M[r][c] = Fi[r][0] * dG[0][c] + Fi[r][1] * dG[1][c] + Fi[r][2] * dG[2][c];
    tr = M[0][0] + M[1][1] + M[2][2];
    const T cm = muw - lamw * lnJ, cl = lamw * tr;
    // Q[c][m] = |s| dP[c][p_m] / h_{p_m}; dP[r][c] = mu dG + cm (M Fi)^T + cl Fi^T
    T Q[3][3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int ax = perm[t][m];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T N = M[ax][0] * Fi[0][c] + M[ax][1] * Fi[1][c] + M[ax][2] * Fi[2][c];  // (M Fi)[ax][c]
        const T v = muw * dG[c][ax] + cm * N + cl * Fi[ax][c];
        Q[c][m] = UNI ? v : v * ih[ax];
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      f[path[0]][c] -= Q[c][0];
      f[path[1]][c] += Q[c][0] - Q[c][1];
      f[path[2]][c] += Q[c][1] - Q[c][2];
      f[path[3]][c] += Q[c][2];
    }
    // keep the next simplex's LDS reads below this point (register pressure)
    __builtin_amdgcn_sched_barrier(0);
  }
}

// nodal forces of one voxel in residual form, f[corner][c] += |s| P(F) g,
// F = F_bar + grad u (u of corner (ox, oy, oz) at lds[oz][c][base + oy PW +
// ox]); with count, the voxel's sums of |s| W and |s| P go to own10
template <typename T, int PW, int PP>
__device__ __forceinline__ void hyper_voxel3_res(const T* pl0, const T* pl1, int base, const T (&Fb)[3][3], T lam,
                                                 T mu, const T (&ih)[3], T vol, T (&f)[8][3], bool count,
                                                 double (&own10)[10]) {
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) f[q][c] = T(0);
  auto ld = [&](int q, int c) -> T {
    const T* pl = (q & 4) ? pl1 : pl0;
    return pl[c * PP + base + ((q >> 1) & 1) * PW + (q & 1)];
  };
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    constexpr int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int path[4];
    path[0] = 0;
#pragma unroll
    for (int m = 0; m < 3; ++m) path[m + 1] = path[m] | (1 << perm[t][m]);
    T F[3][3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int ax = perm[t][m];
#pragma unroll
      for (int c = 0; c < 3; ++c) F[c][ax] = Fb[c][ax] + (ld(path[m + 1], c) - ld(path[m], c)) * ih[ax];
    }
    T Fi[3][3];
    const T J = inv3(F, Fi);
    const T lnJ = J > T(0) ? log(J) : T(NAN);
    T P[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) P[r][c] = mu * (F[r][c] - Fi[c][r]) + lam * lnJ * Fi[c][r];
    if (count) {
      T ff = T(0);
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          ff += F[r][c] * F[r][c];
          own10[1 + 3 * r + c] += (double)(vol * P[r][c]);
        }
      own10[0] += (double)(vol * (T(0.5) * lam * lnJ * lnJ - mu * lnJ + T(0.5) * mu * (ff - T(3))));
    }
    T Q[3][3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int ax = perm[t][m];
#pragma unroll
      for (int c = 0; c < 3; ++c) Q[c][m] = P[c][ax] * (vol * ih[ax]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      f[path[0]][c] -= Q[c][0];
      f[path[1]][c] += Q[c][0] - Q[c][1];
      f[path[2]][c] += Q[c][1] - Q[c][2];
      f[path[3]][c] += Q[c][2];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// MODE 0: q = K_T(u) p (T), p.q partials.  MODE 1: r = rhs - K_T(u) du
// (FP64 arithmetic, written as TO; du == nullptr: zero), ||r||^2.  MODE 2:
// f = -sum |s| B^T P(F) (FP64), ||f||^2 and the |s| W, |s| P sums of the
// voxels owned by the tile (voxel below-left-behind each of its nodes).
template <typename T, typename TO, int MODE, bool UNI, int BX, int BY>
__global__ __launch_bounds__(BX* BY) void k_hyper3t(HyArgs<T> a, int tz, int nxt, int nyt, int nzt) {
  constexpr int NTH = BX * BY;
  constexpr int PW = BX + 2, PP = PW * (BY + 2);
  constexpr int VW = BX + 1, VV = VW * (BY + 1);
  constexpr int NPL = (MODE == 2 ? 3 : 6) * PP;  // u (and p), three components each, per node plane
  constexpr int PF = (NPL + NTH - 1) / NTH;
  constexpr int NEXTRA = BX + BY + 1;
  __shared__ T pl[2 * NPL];
  __shared__ T cb[18 * VV];
  __shared__ double sh[NTH / WAVE];
  const int tid = threadIdx.x;
  const int tx = tid % BX, ty = tid / BX;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int n = (int)a.g.n;
  const int nxy = nx * ny;
  const int ntiles = nxt * nyt * nzt;
  const int item = xcd_order(blockIdx.x, ntiles * a.nload);
  if (item < 0) return;
  const int l = item % a.nload;
  const int blk = item / a.nload;
  if (MODE == 0 ? a.st[l].state != ST_ACTIVE : (a.mask && a.mask[l] == 0)) return;
  const int bxi = blk % nxt, byi = (blk / nxt) % nyt, bzi = blk / (nxt * nyt);
  const int x0 = bxi * BX, y0 = byi * BY, z0 = bzi * tz;
  const T ih[3] = {T(1.0 / a.g.h[0]), T(1.0 / a.g.h[1]), T(1.0 / a.g.h[2])};
  const T vol = T(a.g.h[0] * a.g.h[1] * a.g.h[2] / 6.0);
  // material weight of the tangent: |s| (UNI: |s| / h^2)
  const T wt = UNI ? T(a.g.h[0] * a.g.h[1] * a.g.h[2] / (6.0 * a.g.h[0] * a.g.h[0])) : vol;
  // F_bar in the arithmetic type (uniform loads: scalar registers)
  T Fb[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Fb[i][j] = a.FbarT[l * 9 + i * 3 + j];
  const bool has_extra = tid < NEXTRA;
  const int ex = tid < BY ? BX - 1 : tid - BY - 1;
  const int ey = tid < BY ? tid - 1 : BY - 1;
  // in-plane offset of prefetch element e (field e / (3 PP), component,
  // wrapped x and y); recomputed per plane to keep registers free
  auto poff = [&](int e) {
    const int fc = e / PP, rem = e - fc * PP;
    const int py = rem / PW, px = rem - py * PW;
    return (fc % 3) * n + hwrap(y0 - 1 + py, ny) * nx + hwrap(x0 - 1 + px, nx);
  };
  const int vown = hwrap(y0 + ty - 1, ny) * nx + hwrap(x0 + tx - 1, nx);
  const int vext = hwrap(y0 + ey, ny) * nx + hwrap(x0 + ex, nx);
  const int bown = ty * PW + tx;
  const int bext = (ey + 1) * PW + (ex + 1);
  const int cown = ty * VW + tx;
  const int cext = (ey + 1) * VW + (ex + 1);
  const T* u = a.u + l * a.lstride;
  const T* p = (MODE != 2 && a.p) ? a.p + l * a.lstride : nullptr;
  TO* out = reinterpret_cast<TO*>(a.out) + l * a.lstride;
  const double* rhs = MODE == 1 ? a.rhs + l * a.lstride : nullptr;
  const T* matl = a.mat + (long long)(l / a.lpc) * a.mat_stride;
  T pf[PF];
  auto fetch_plane = [&](int zp) {
    const int zoff = hwrap(zp, nz) * nxy;
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = tid + q * NTH;
      if (e < NPL) pf[q] = e < 3 * PP ? u[poff(e) + zoff] : (p ? p[poff(e) + zoff] : T(0));
    }
  };
  auto store_plane = [&](int slot) {
#pragma unroll
    for (int q = 0; q < PF; ++q)
      if (tid + q * NTH < NPL) pl[slot * NPL + tid + q * NTH] = pf[q];
  };
  double acc = 0.0;
  double own10[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  T carry[3] = {T(0), T(0), T(0)};
  fetch_plane(z0 - 1);
  store_plane(0);
  fetch_plane(z0);
  store_plane(1);
  int zm = hwrap(z0 - 1, nz) * nxy;
  T lam0 = matl[2 * (zm + vown)], mu0 = matl[2 * (zm + vown) + 1];
  T lame = T(0), mue = T(0);
  if (has_extra) {
    lame = matl[2 * (zm + vext)];
    mue = matl[2 * (zm + vext) + 1];
  }
  __syncthreads();
  for (int L = 0; L <= tz; ++L) {
    const int k = z0 - 1 + L;
    const int s0 = L & 1, s1 = (L + 1) & 1;
    if (L < tz) fetch_plane(k + 2);
    T lam1 = T(0), mu1 = T(0), lame1 = T(0), mue1 = T(0);
    if (L < tz) {
      const int zn = hwrap(k + 1, nz) * nxy;
      lam1 = matl[2 * (zn + vown)];
      mu1 = matl[2 * (zn + vown) + 1];
      if (has_extra) {
        lame1 = matl[2 * (zn + vext)];
        mue1 = matl[2 * (zn + vext) + 1];
      }
    }
    // pass 0: the thread's own voxel, whose (1,1,*) corners stay in
    // registers; pass 1: the halo voxel (if any); one code body
    T own[2][3];
#pragma nounroll
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 1 && !has_extra) break;
      T f[8][3];
      if constexpr (MODE == 2) {
        // the voxel of layer k belongs to the node above it (plane k + 1)
        const bool count = pass == 0 && L < tz && z0 + L < nz;
        hyper_voxel3_res<T, PW, PP>(pl + s0 * NPL, pl + s1 * NPL, pass == 0 ? bown : bext, Fb,
                                    pass == 0 ? lam0 : lame, pass == 0 ? mu0 : mue, ih, vol, f, count, own10);
      } else {
        constexpr bool FASTLN = sizeof(T) == 4 || sizeof(TO) == 4;
        hyper_voxel3<T, PW, PP, UNI, FASTLN>(pl + s0 * NPL, pl + s1 * NPL, pass == 0 ? bown : bext, Fb,
                                     (pass == 0 ? lam0 : lame) * wt, (pass == 0 ? mu0 : mue) * wt, ih, f);
      }
      const int ci = pass == 0 ? cown : cext;
#pragma unroll
      for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          cb[((0 * 2 + oz) * 3 + c) * VV + ci] = f[0 + 4 * oz][c];
          cb[((1 * 2 + oz) * 3 + c) * VV + ci] = f[1 + 4 * oz][c];
          cb[((2 * 2 + oz) * 3 + c) * VV + ci] = f[2 + 4 * oz][c];
          if (pass == 0) own[oz][c] = f[3 + 4 * oz][c];
        }
    }
    __syncthreads();
    T pk[3] = {T(0), T(0), T(0)};
    if constexpr (MODE == 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) pk[c] = pl[s0 * NPL + (3 + c) * PP + (ty + 1) * PW + (tx + 1)];
    }
    {
      const int i00 = (ty + 1) * VW + (tx + 1);
      const int i10 = (ty + 1) * VW + tx;
      const int i01 = ty * VW + (tx + 1);
      T val[3], nc[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        val[c] = carry[c] + own[0][c] + cb[(0 * 3 + c) * VV + i00] + cb[(6 + c) * VV + i10] + cb[(12 + c) * VV + i01];
        nc[c] = own[1][c] + cb[(3 + c) * VV + i00] + cb[(9 + c) * VV + i10] + cb[(15 + c) * VV + i01];
      }
      if (L >= 1 && k < nz) {
        const int node = k * nxy + (y0 + ty) * nx + (x0 + tx);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if constexpr (MODE == 0) {
            out[c * n + node] = (TO)val[c];
            acc += (double)pk[c] * (double)val[c];
          } else if constexpr (MODE == 1) {
            const double r = rhs[c * n + node] - (double)val[c];
            out[c * n + node] = (TO)r;
            acc += r * r;
          } else {
            const double fv = -(double)val[c];
            out[c * n + node] = (TO)fv;
            acc += fv * fv;
          }
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) carry[c] = nc[c];
    }
    if (L < tz) store_plane(s0);
    lam0 = lam1;
    mu0 = mu1;
    lame = lame1;
    mue = mue1;
    __syncthreads();
  }
  const double bs = block_sum<NTH>(acc, sh);
  if (tid == 0) a.red.put(MODE == 0 ? RED_PQ : RED_RES, l, blk, bs);
  if constexpr (MODE == 2) {
    for (int v = 0; v < 10; ++v) {
      const double sv = block_sum<NTH>(own10[v], sh);
      if (tid == 0) a.vparts[((long long)l * 10 + v) * a.red.maxblk + blk] = sv;
    }
  }
}

// per slot: fixed-order sums of nval partial rows -> vals[slot][nval]
__global__ __launch_bounds__(NT) void k_sum_vals(const double* parts, int maxblk, int nparts, int nval,
                                                 const int* mask, double* vals) {
  __shared__ double sh[NT / WAVE];
  const int v = blockIdx.x, l = blockIdx.y;
  if (mask && mask[l] == 0) return;
  const double* row = parts + ((long long)l * nval + v) * maxblk;
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += NT) s += row[i];
  s = block_sum<NT>(s, sh);
  if (threadIdx.x == 0) vals[(long long)l * nval + v] = s;
}

// y[slot] = x[slot] + t[slot] * d[slot] for the masked slots
__global__ void k_axpy_slots(const double* x, const double* t, const double* d, double* y, long long len,
                             const int* mask) {
  const int l = blockIdx.y;
  if (mask && mask[l] == 0) return;
  const double tl = t[l];
  const long long o = (long long)l * len;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (long long)gridDim.x * blockDim.x)
    y[o + i] = x[o + i] + tl * d[o + i];
}

// y[slot] = (TO) x[slot] for the masked slots (mask == nullptr: all)
template <typename TI, typename TO>
__global__ void k_copy_slots(const TI* x, TO* y, long long len, const int* mask) {
  const int l = blockIdx.y;
  if (mask && mask[l] == 0) return;
  const long long o = (long long)l * len;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (long long)gridDim.x * blockDim.x)
    y[o + i] = (TO)x[o + i];
}

// x[slot] = 0 for the masked slots
__global__ void k_zero_slots(double* x, long long len, const int* mask) {
  const int l = blockIdx.y;
  if (mask && mask[l] == 0) return;
  const long long o = (long long)l * len;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (long long)gridDim.x * blockDim.x)
    x[o + i] = 0.0;
}

// partials of a[slot] . b[slot] (FP64) into the RES slot of the reduction buffer
__global__ __launch_bounds__(NT) void k_dot_slots(const double* x, const double* y, long long len, const int* mask,
                                                  RedBuf red) {
  __shared__ double sh[NT / WAVE];
  const int l = blockIdx.y;
  if (mask && mask[l] == 0) return;
  const long long o = (long long)l * len;
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < len; i += (long long)gridDim.x * NT)
    s += x[o + i] * y[o + i];
  s = block_sum<NT>(s, sh);
  if (threadIdx.x == 0) red.put(RED_RES, l, blockIdx.x, s);
}

// per (slot, component): partial sums of the n nodal values
__global__ __launch_bounds__(NT) void k_comp_parts(const double* x, long long lstride, long long n, int nb,
                                                   const int* mask, double* parts) {
  __shared__ double sh[NT / WAVE];
  const int c = blockIdx.y, l = blockIdx.z;
  if (mask && mask[l] == 0) return;
  const double* v = x + (long long)l * lstride + (long long)c * n;
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)nb * NT) s += v[i];
  s = block_sum<NT>(s, sh);
  if (threadIdx.x == 0) parts[((long long)l * 3 + c) * nb + blockIdx.x] = s;
}

// x -= mean over the nodes, per (slot, component); every block adds the
// partials in the same order, so all blocks subtract the same mean
__global__ __launch_bounds__(NT) void k_sub_mean(double* x, long long lstride, long long n, int nb,
                                                 const int* mask, const double* parts) {
  __shared__ double sh[NT / WAVE];
  const int c = blockIdx.y, l = blockIdx.z;
  if (mask && mask[l] == 0) return;
  const double* row = parts + ((long long)l * 3 + c) * nb;
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += NT) s += row[i];
  const double mean = block_sum<NT>(s, sh) / (double)n;
  double* v = x + (long long)l * lstride + (long long)c * n;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) v[i] -= mean;
}

hipError_t launch_remove_mean(double* x, long long lstride, long long n, int d, int nslot, const int* mask,
                              double* parts, int maxparts, hipStream_t s) {
  long long nb = (n + 4LL * NT - 1) / (4LL * NT);
  if (nb > 1024) nb = 1024;
  if (nb > maxparts) nb = maxparts;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_comp_parts, dim3((unsigned)nb, d, nslot), dim3(NT), 0, s, (const double*)x, lstride, n, (int)nb,
                     mask, parts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sub_mean, dim3(256, d, nslot), dim3(NT), 0, s, x, lstride, n, (int)nb, mask,
                     (const double*)parts);
  return hipGetLastError();
}

// r = rhs (the residual at du = 0) as TO for the masked slots, ||r||^2 partials
template <typename TO>
__global__ __launch_bounds__(NT) void k_rhs_residual(const double* rhs, TO* r, long long lstride, long long m,
                                                     const int* mask, RedBuf red) {
  __shared__ double sh[NT / WAVE];
  const int l = blockIdx.y;
  if (mask && mask[l] == 0) return;
  const long long o = (long long)l * lstride;
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < m; i += (long long)gridDim.x * NT) {
    const double v = rhs[o + i];
    r[o + i] = (TO)v;
    s += v * v;
  }
  s = block_sum<NT>(s, sh);
  if (threadIdx.x == 0) red.put(RED_RES, l, blockIdx.x, s);
}

hipError_t launch_rhs_residual(const double* rhs, void* r, bool out32, long long lstride, long long m, int nslot,
                               const int* mask, const RedBuf& red, LoadState* st, double* res2, hipStream_t s) {
  const int nb = red.maxblk < 1024 ? red.maxblk : 1024;
  if (out32)
    hipLaunchKernelGGL(k_rhs_residual<float>, dim3(nb, nslot), dim3(NT), 0, s, rhs, static_cast<float*>(r), lstride, m,
                       mask, red);
  else
    hipLaunchKernelGGL(k_rhs_residual<double>, dim3(nb, nslot), dim3(NT), 0, s, rhs, static_cast<double*>(r), lstride,
                       m, mask, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(red, st, res2, RED_RES, nb, nslot, -1, mask, s);
}

// per-block maxima of |x[slot]| -> parts[slot][AMAX_BLOCKS]
__global__ __launch_bounds__(NT) void k_amax_slots(const double* x, long long len, const int* mask, double* parts) {
  __shared__ double sh[NT];
  const int l = blockIdx.y;
  if (mask && mask[l] == 0) return;
  const long long o = (long long)l * len;
  double m = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < len; i += (long long)gridDim.x * NT)
    m = fmax(m, fabs(x[o + i]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) parts[(long long)l * gridDim.x + blockIdx.x] = sh[0];
}

hipError_t launch_amax_slots(const double* x, long long len, int nslot, const int* mask, double* parts, int maxparts,
                             hipStream_t s) {
  const int nb = maxparts < AMAX_BLOCKS ? maxparts : AMAX_BLOCKS;
  hipLaunchKernelGGL(k_amax_slots, dim3(nb, nslot), dim3(NT), 0, s, x, len, mask, parts);
  return hipGetLastError();
}

int hyper_blocks(const Geom& g, int maxblk) {
  const long long nb = (g.n + NT - 1) / NT;
  return (int)(nb < maxblk ? nb : maxblk);
}

template <typename T, typename TO, int MODE>
static hipError_t launch_hyper_impl(const HyArgs<T>& a, hipStream_t s) {
  const int nb = hyper_blocks(a.g, a.red.maxblk);
  dim3 grid(nb, a.nload);
  if (a.g.dim == 3) hipLaunchKernelGGL((k_hyper<T, TO, MODE, 3>), grid, dim3(NT), 0, s, a);
  else hipLaunchKernelGGL((k_hyper<T, TO, MODE, 2>), grid, dim3(NT), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_finalize(a.red, a.st, a.res2, MODE == 0 ? RED_PQ : RED_RES, nb, a.nload, -1, MODE == 0 ? nullptr : a.mask, s);
  if (e != hipSuccess || MODE != 2) return e;
  hipLaunchKernelGGL(k_sum_vals, dim3(10, a.nload), dim3(NT), 0, s, (const double*)a.vparts, a.red.maxblk, nb, 10,
                     a.mask, a.vals);
  return hipGetLastError();
}

// tile of the voxel-centric tangent kernel: BX x BY nodes
template <typename T> struct HyTile;
template <> struct HyTile<float> {
  static constexpr int BX = 16, BY = 16;
};
template <> struct HyTile<double> {
  static constexpr int BX = 16, BY = 8;
};

// tiles along z for the voxel-centric kernel: the smallest tz >= 8 whose
// partial count fits the reduction rows; 0 if the grid does not tile
template <typename T>
static int hyper_tile_tz(const Geom& g, int maxblk) {
  constexpr int BX = HyTile<T>::BX, BY = HyTile<T>::BY;
  if (g.dim != 3 || g.nx % BX || g.ny % BY || g.nz < 2) return 0;
  for (int tz = 8; tz <= 256; tz *= 2) {
    const long long parts = (long long)(g.nx / BX) * (g.ny / BY) * ((g.nz + tz - 1) / tz);
    if (parts <= maxblk) return tz;
  }
  return 0;
}

// tiled kernel where the grid tiles (3D), else the node-centric one
template <typename T, typename TO, int MODE>
static hipError_t launch_hyper_any(const HyArgs<T>& a, hipStream_t s) {
  constexpr int BX = HyTile<T>::BX, BY = HyTile<T>::BY;
  const int tz = hyper_tile_tz<T>(a.g, a.red.maxblk);
  if (tz == 0) return launch_hyper_impl<T, TO, MODE>(a, s);
  const int nxt = a.g.nx / BX, nyt = a.g.ny / BY, nzt = (a.g.nz + tz - 1) / tz;
  const int nparts = nxt * nyt * nzt;
  const bool uni = a.g.h[0] == a.g.h[1] && a.g.h[1] == a.g.h[2];
  if (uni)
    hipLaunchKernelGGL((k_hyper3t<T, TO, MODE, true, BX, BY>), dim3(xcd_grid(nparts * a.nload)), dim3(BX * BY), 0, s,
                       a, tz, nxt, nyt, nzt);
  else
    hipLaunchKernelGGL((k_hyper3t<T, TO, MODE, false, BX, BY>), dim3(xcd_grid(nparts * a.nload)), dim3(BX * BY), 0, s,
                       a, tz, nxt, nyt, nzt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_finalize(a.red, a.st, a.res2, MODE == 0 ? RED_PQ : RED_RES, nparts, a.nload, -1,
                      MODE == 0 ? nullptr : a.mask, s);
  if (e != hipSuccess || MODE != 2) return e;
  hipLaunchKernelGGL(k_sum_vals, dim3(10, a.nload), dim3(NT), 0, s, (const double*)a.vparts, a.red.maxblk, nparts, 10,
                     a.mask, a.vals);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_hyper_tangent(const HyArgs<T>& a, hipStream_t s) {
  return launch_hyper_any<T, T, 0>(a, s);
}

hipError_t launch_hyper_tangent_residual(const HyArgs<double>& a, bool out32, hipStream_t s) {
  return out32 ? launch_hyper_any<double, float, 1>(a, s) : launch_hyper_any<double, double, 1>(a, s);
}

hipError_t launch_hyper_residual(const HyArgs<double>& a, hipStream_t s) {
  return launch_hyper_any<double, double, 2>(a, s);
}

hipError_t launch_axpy_slots(const double* x, const double* t, const double* d, double* y, long long len, int nslot,
                             const int* mask, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_slots, dim3(512, nslot), dim3(256), 0, s, x, t, d, y, len, mask);
  return hipGetLastError();
}

hipError_t launch_copy_slots(const double* x, double* y, long long len, int nslot, const int* mask, hipStream_t s) {
  hipLaunchKernelGGL((k_copy_slots<double, double>), dim3(512, nslot), dim3(256), 0, s, x, y, len, mask);
  return hipGetLastError();
}

hipError_t launch_round_slots(const double* x, float* y, long long len, int nslot, hipStream_t s) {
  hipLaunchKernelGGL((k_copy_slots<double, float>), dim3(512, nslot), dim3(256), 0, s, x, y, len,
                     (const int*)nullptr);
  return hipGetLastError();
}

hipError_t launch_widen_slots(const float* x, double* y, long long len, int nslot, const int* mask, hipStream_t s) {
  hipLaunchKernelGGL((k_copy_slots<float, double>), dim3(512, nslot), dim3(256), 0, s, x, y, len, mask);
  return hipGetLastError();
}

hipError_t launch_zero_slots(double* x, long long len, int nslot, const int* mask, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_slots, dim3(512, nslot), dim3(256), 0, s, x, len, mask);
  return hipGetLastError();
}

hipError_t launch_dot_slots(const double* x, const double* y, long long len, int nslot, const int* mask,
                            const RedBuf& red, LoadState* st, double* res2, hipStream_t s) {
  const int nb = red.maxblk < 1024 ? red.maxblk : 1024;
  hipLaunchKernelGGL(k_dot_slots, dim3(nb, nslot), dim3(NT), 0, s, x, y, len, mask, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(red, st, res2, RED_RES, nb, nslot, -1, mask, s);
}

template hipError_t launch_hyper_tangent<float>(const HyArgs<float>&, hipStream_t);
template hipError_t launch_hyper_tangent<double>(const HyArgs<double>&, hipStream_t);

#ifdef CELLFFT_BOUNDS_CHECK
unsigned int oob_take_hyper() { return oob_take(); }
#endif

}  // namespace cellfft
