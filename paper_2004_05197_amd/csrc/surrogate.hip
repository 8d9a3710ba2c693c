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
#include <type_traits>

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
      const long long o = sr_chunk(node) + (long long)v * SR_CHUNK;
      s64[o] = s;
      s32[o] = (float)s;
    }
  }
}

// MODE 0: q = Kt p (T) for the active slots, p.q partials.
// MODE 1: r = f - Kt u (FP64, written as TO) for the masked slots.
// Both: per-block component sums of the output (for its mean).
//
// A block owns a BX x BY tile of nodes in tz planes and applies all six
// slots, so every stencil value is read from HBM once per launch.  Its
// neighbours' blocks A_d(i - d) and the direction vectors around the tile
// are read by the blocks running beside it on the same XCD (tiles are dealt
// to XCDs in contiguous runs, ordered so that those blocks form a short
// stack of planes) and mostly come from L2.  The stencil is laid out in
// 64-node chunks (sr_chunk), so one wavefront's 63 stencil loads read one
// contiguous 16 KB region.
template <typename T, typename TO, int MODE, int BX, int BY>
__global__ __launch_bounds__(BX* BY) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1))) void k_sr_apply3t(SArgs<T> a, int tz, int nxt, int nyt, int nzt, int gy) {
  static_assert(BX * BY == NT, "one tile row per thread");
  constexpr int NSUM = 24;  // per slot: p.q and the three component sums
  __shared__ double sh[(NT / WAVE) * NSUM];
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const long long n = a.g.n;
  const int blk = xcd_order(blockIdx.x, nxt * nyt * nzt);
  if (blk < 0) return;  // whole block
  // tile order: x tiles fastest, then gy tiles in y, then z, then the
  // groups of gy tile rows, so that the blocks running together on one XCD
  // cover a short stack of planes and reuse each other's planes from L2
  int r = blk;
  const int xi = r % nxt;
  r /= nxt;
  const int yl = r % gy;
  r /= gy;
  const int zi = r % nzt, yi = (r / nzt) * gy + yl;
  const int tx = threadIdx.x % BX, ty = threadIdx.x / BX;
  const int x = xi * BX + tx, y = yi * BY + ty;
  const int z0 = zi * tz, z1 = min(z0 + tz, nz);
  bool live[6];
#pragma unroll
  for (int l = 0; l < 6; ++l)
    live[l] = l < a.nslot && (MODE == 0 ? a.st[l].state == ST_ACTIVE : (a.mask ? a.mask[l] != 0 : true));
  // per-thread sums over the column's tz nodes in T, across the block in
  // FP64
  T dot[6], csum[6][3];
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    dot[l] = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) csum[l][c] = T(0);
  }
  // every slot is computed (a slot beyond nslot reads slot 0): no branch
  // on liveness splits the loads of one offset into dependent groups;
  // only live slots are stored and summed
  const T* pv[6];
#pragma unroll
  for (int l = 0; l < 6; ++l) pv[l] = a.p + (l < a.nslot ? l : 0) * a.lstride;
  if (x < nx && y < ny) {
    const int xs[3] = {swrap(x - 1, nx), x, swrap(x + 1, nx)};
    const int ys[3] = {swrap(y - 1, ny), y, swrap(y + 1, ny)};
    for (int z = z0; z < z1; ++z) {
      const int zs[3] = {swrap(z - 1, nz), z, swrap(z + 1, nz)};
      const long long node = ((long long)z * ny + y) * nx + x;
      const T* so = a.s + sr_chunk(node);
      T acc[6][3], pi[6][3];
#pragma unroll
      for (int l = 0; l < 6; ++l)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          acc[l][c] = T(0);
          pi[l][c] = pv[l][c * n + node];
        }
      // the edge form below applies -R_i to p_i; the diagonal is -sym(R_i):
      // the skew part of the block row sum R_i is added at the end
      T rs[3][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
      // one offset at a time keeps the live registers to one pair of blocks;
      // BELOW: an offset with a z component, whose A_d(i - d) lies in the
      // plane below
      auto offset = [&](const int d, auto below) {
        constexpr bool BELOW = decltype(below)::value;
        const int m = (0x7563421 >> (4 * d)) & 7;  // offset d as bits x | y << 1 | z << 2
        const int ox = m & 1, oy = (m >> 1) & 1, oz = m >> 2;
        const long long jp = ((long long)zs[1 + oz] * ny + ys[1 + oy]) * nx + xs[1 + ox];
        const long long jm = ((long long)zs[1 - oz] * ny + ys[1 - oy]) * nx + xs[1 - ox];
        const T* sm = a.s + sr_chunk(jm);
        // all 54 loads of the offset first, then the arithmetic: the
        // scheduler would otherwise interleave them one load per wait.
        // A_d(i) is read once per launch, and the blocks of the plane below
        // were last touched a whole plane of the XCD's tiles ago: both
        // stream past L2 (non-temporal), which keeps L2 for the direction
        // vectors and the in-plane neighbour blocks
        T A[3][3], B[3][3], pp[6][3], pm[6][3];
#pragma unroll
        for (int e = 0; e < 9; ++e) {
          A[e / 3][e % 3] = __builtin_nontemporal_load(so + (9 * d + e) * SR_CHUNK);  // A_d(i)
          if constexpr (BELOW) B[e / 3][e % 3] = __builtin_nontemporal_load(sm + (9 * d + e) * SR_CHUNK);
          else B[e / 3][e % 3] = sm[(9 * d + e) * SR_CHUNK];  // A_d(i - d)
        }
#pragma unroll
        for (int l = 0; l < 6; ++l)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            pp[l][c] = pv[l][c * n + jp];
            pm[l][c] = pv[l][c * n + jm];
          }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) rs[r][c] += A[r][c] + B[c][r];
#pragma unroll
        for (int l = 0; l < 6; ++l) {
          T dp[3], dm[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            dp[c] = pp[l][c] - pi[l][c];
            dm[c] = pm[l][c] - pi[l][c];
          }
#pragma unroll
          for (int r = 0; r < 3; ++r)
            acc[l][r] += A[r][0] * dp[0] + A[r][1] * dp[1] + A[r][2] * dp[2] + B[0][r] * dm[0] + B[1][r] * dm[1] +
                         B[2][r] * dm[2];
        }
      };
      // the in-plane offsets x, y, xy, then z, yz, xz, xyz
#pragma unroll 1
      for (int k = 0; k < 3; ++k) offset((0x310 >> (4 * k)) & 15, std::false_type());
#pragma unroll 1
      for (int k = 0; k < 4; ++k) offset((0x6542 >> (4 * k)) & 15, std::true_type());
#pragma unroll
      for (int l = 0; l < 6; ++l) {
        if (!live[l]) continue;
#pragma unroll
        for (int r = 0; r < 3; ++r)
          acc[l][r] += T(0.5) * ((rs[r][0] - rs[0][r]) * pi[l][0] + (rs[r][1] - rs[1][r]) * pi[l][1] +
                                 (rs[r][2] - rs[2][r]) * pi[l][2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const long long o = l * a.lstride + c * n + node;
          if (MODE == 0) {
            reinterpret_cast<T*>(a.out)[o] = acc[l][c];
            dot[l] += pi[l][c] * acc[l][c];
            csum[l][c] += acc[l][c];
          } else {
            const double r = a.rhs[o] - (double)acc[l][c];
            reinterpret_cast<TO*>(a.out)[o] = (TO)r;
            csum[l][c] += r;
          }
        }
      }
    }
  }
  // the 24 block sums in one pass: wave sums, one barrier, one thread each
  const int nb = nxt * nyt * nzt;
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    const double dw = wave_sum((double)dot[l]);
    if (lane == 0) sh[wv * NSUM + l] = dw;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double cw = wave_sum((double)csum[l][c]);
      if (lane == 0) sh[wv * NSUM + 6 + 3 * l + c] = cw;
    }
  }
  __syncthreads();
  const int k = threadIdx.x;
  if (k < NSUM) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / WAVE; ++w) s += sh[w * NSUM + k];
    if (k < 6) {
      if (MODE == 0 && live[k]) a.red.put(RED_PQ, k, blk, s);
    } else {
      const int l = (k - 6) / 3, c = (k - 6) % 3;
      if (live[l]) a.cparts[((long long)l * 3 + c) * nb + blk] = s;
    }
  }
}

// FP32 operator for grids with nx a multiple of 64: one wavefront per tile
// row of 64 nodes, so the x neighbours of a direction-vector row are the
// next and previous lanes.  Each (load, component) row the stencil needs is
// read once per node (own row, y +- 1, z +- 1, (y+1, z+1), (y-1, z-1): 7
// instead of 15 gathered positions), the +-x shifted copies come from DPP
// wave rotations, and the 8 values beyond the row ends (lane 63's right and
// lane 0's left neighbour of the shifted rows) are gathered by lanes 0-7 in
// one load and put in place with readlane before the rotation.
namespace {
// lane i <- lane i + 1 (LEFT) or i - 1, and the lane at the far end
// receives edge (a wave-uniform value): the value rotated out of lane 0
// (LEFT) or 63 is replaced by edge first, then the row is rotated by one
template <bool LEFT>
__device__ __forceinline__ float wshift(float v, int lane, float edge) {
  const float t = lane == (LEFT ? 0 : WAVE - 1) ? edge : v;
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(t), LEFT ? 0x134 : 0x13C, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_value(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
}  // namespace

template <int BY>
__global__ __launch_bounds__(WAVE* BY) __attribute__((amdgpu_waves_per_eu(3))) void k_sr_apply3w(SArgs<float> a, int nxt,
                                                                                                 int nyt, int nzt,
                                                                                                 int gy) {
  static_assert(WAVE * BY == NT, "one tile row per wavefront");
  constexpr int NSUM = 24;
  __shared__ double sh[(NT / WAVE) * NSUM];
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const long long n = a.g.n;
  const int blk = xcd_order(blockIdx.x, nxt * nyt * nzt);
  if (blk < 0) return;  // whole block
  int r = blk;
  const int xi = r % nxt;
  r /= nxt;
  const int yl = r % gy;
  r /= gy;
  const int z = r % nzt, yi = (r / nzt) * gy + yl;
  const int lane = threadIdx.x % WAVE;
  const int ty = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int x0 = xi * WAVE, x = x0 + lane, y = yi * BY + ty;
  bool live[6];
#pragma unroll
  for (int l = 0; l < 6; ++l) live[l] = l < a.nslot && a.st[l].state == ST_ACTIVE;
  float dot[6], csum[6][3];
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    dot[l] = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) csum[l][c] = 0.f;
  }
  const float* pv[6];
#pragma unroll
  for (int l = 0; l < 6; ++l) pv[l] = a.p + (l < a.nslot ? l : 0) * a.lstride;
  if (y < ny) {  // whole wavefront
    const int ym = swrap(y - 1, ny), yp = swrap(y + 1, ny);
    const int zm = swrap(z - 1, nz), zp = swrap(z + 1, nz);
    // row starts (flat index of x = 0) of the seven rows
    const long long r00 = ((long long)z * ny + y) * nx, rp0 = ((long long)z * ny + yp) * nx;
    const long long rm0 = ((long long)z * ny + ym) * nx, r0p = ((long long)zp * ny + y) * nx;
    const long long r0m = ((long long)zm * ny + y) * nx, rpp = ((long long)zp * ny + yp) * nx;
    const long long rmm = ((long long)zm * ny + ym) * nx;
    const long long node = r00 + x;
    const int xr = swrap(x0 + WAVE, nx), xl = swrap(x0 - 1, nx);
    // lanes 0-7 gather the row-end values: +x / -x of the own row, then the
    // shifted rows of xy, xz, xyz (right end of the + row, left end of the - row)
    long long eidx = node;
    switch (lane) {
      case 0: eidx = r00 + xr; break;
      case 1: eidx = r00 + xl; break;
      case 2: eidx = rp0 + xr; break;
      case 3: eidx = rm0 + xl; break;
      case 4: eidx = r0p + xr; break;
      case 5: eidx = r0m + xl; break;
      case 6: eidx = rpp + xr; break;
      case 7: eidx = rmm + xl; break;
      default: break;
    }
    const float* so = a.s + sr_chunk(node);
    float acc[6][3], pi[6][3], E[6][3];
#pragma unroll
    for (int l = 0; l < 6; ++l)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[l][c] = 0.f;
        pi[l][c] = pv[l][c * n + node];
        E[l][c] = pv[l][c * n + eidx];
      }
    float rs[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    // offset d: A_d(i) from the own chunk, A_d(i - d) from the chunk of
    // jm, then the update with p_{i+d} = pp, p_{i-d} = pm
    auto stencil = [&](int d, long long jm, float (&A)[3][3], float (&B)[3][3], bool below) {
      const float* sm = a.s + sr_chunk(jm);
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        A[e / 3][e % 3] = __builtin_nontemporal_load(so + (9 * d + e) * SR_CHUNK);
        if (below) B[e / 3][e % 3] = __builtin_nontemporal_load(sm + (9 * d + e) * SR_CHUNK);
        else B[e / 3][e % 3] = sm[(9 * d + e) * SR_CHUNK];
      }
    };
    // pp(l, c), pm(l, c): p_{i+d} and p_{i-d} of load l, component c
    auto update = [&](const float (&A)[3][3], const float (&B)[3][3], auto pp, auto pm) {
#pragma unroll
      for (int rr = 0; rr < 3; ++rr)
#pragma unroll
        for (int c = 0; c < 3; ++c) rs[rr][c] += A[rr][c] + B[c][rr];
#pragma unroll
      for (int l = 0; l < 6; ++l) {
        float dp[3], dm[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          dp[c] = pp(l, c) - pi[l][c];
          dm[c] = pm(l, c) - pi[l][c];
        }
#pragma unroll
        for (int rr = 0; rr < 3; ++rr)
          acc[l][rr] += A[rr][0] * dp[0] + A[rr][1] * dp[1] + A[rr][2] * dp[2] + B[0][rr] * dm[0] +
                        B[1][rr] * dm[1] + B[2][rr] * dm[2];
      }
    };
    // a pair of rows (+, -): the aligned offset d0 and the x-shifted offset
    // d1 (edges ke, ke + 1 of the gather); the own row pairs with itself
    auto pair = [&](long long rplus, long long rminus, int d0, int d1, int ke, auto below) {
      constexpr bool BELOW = decltype(below)::value;
      __builtin_amdgcn_sched_barrier(0);
      float rp[6][3], rm[6][3];
      float A[3][3], B[3][3];
      if (d0 >= 0) {
#pragma unroll
        for (int l = 0; l < 6; ++l)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            rp[l][c] = pv[l][c * n + rplus + x];
            rm[l][c] = pv[l][c * n + rminus + x];
          }
        stencil(d0, rminus + x, A, B, BELOW);
        __builtin_amdgcn_sched_barrier(0);
        update(A, B, [&](int l, int c) { return rp[l][c]; }, [&](int l, int c) { return rm[l][c]; });
      } else {
#pragma unroll
        for (int l = 0; l < 6; ++l)
#pragma unroll
          for (int c = 0; c < 3; ++c) rp[l][c] = rm[l][c] = pi[l][c];
      }
      stencil(d1, rminus + (lane ? x - 1 : xl), A, B, BELOW);
      __builtin_amdgcn_sched_barrier(0);
      update(
          A, B, [&](int l, int c) { return wshift<true>(rp[l][c], lane, lane_value(E[l][c], ke)); },
          [&](int l, int c) { return wshift<false>(rm[l][c], lane, lane_value(E[l][c], ke + 1)); });
    };
    // offsets in the stencil order x 0, y 1, z 2, xy 3, yz 4, xz 5, xyz 6
    pair(r00, r00, -1, 0, 0, std::false_type());
    pair(rp0, rm0, 1, 3, 2, std::false_type());
    pair(r0p, r0m, 2, 5, 4, std::true_type());
    pair(rpp, rmm, 4, 6, 6, std::true_type());
    // every slot is finished and stored without a branch (a per-slot
    // branch here let the compiler sink work into six blocks and spill): a
    // converged slot's q is not read again, and a slot beyond nslot, which
    // computed slot 0's q from slot 0's p, stores it over slot 0's q
#pragma unroll
    for (int l = 0; l < 6; ++l) {
#pragma unroll
      for (int rr = 0; rr < 3; ++rr)
        acc[l][rr] += 0.5f * ((rs[rr][0] - rs[0][rr]) * pi[l][0] + (rs[rr][1] - rs[1][rr]) * pi[l][1] +
                              (rs[rr][2] - rs[2][rr]) * pi[l][2]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        dot[l] += pi[l][c] * acc[l][c];
        csum[l][c] += acc[l][c];
      }
    }
#pragma unroll
    for (int l = 0; l < 6; ++l)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        reinterpret_cast<float*>(a.out)[(l < a.nslot ? l : 0) * a.lstride + c * n + node] = acc[l][c];
  }
  const int nb = nxt * nyt * nzt;
  const int wv = threadIdx.x / WAVE;
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    const double dw = wave_sum((double)dot[l]);
    if (lane == 0) sh[wv * NSUM + l] = dw;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double cw = wave_sum((double)csum[l][c]);
      if (lane == 0) sh[wv * NSUM + 6 + 3 * l + c] = cw;
    }
  }
  __syncthreads();
  const int k = threadIdx.x;
  if (k < NSUM) {
    double s2 = 0.0;
#pragma unroll
    for (int w = 0; w < NT / WAVE; ++w) s2 += sh[w * NSUM + k];
    if (k < 6) {
      if (live[k]) a.red.put(RED_PQ, k, blk, s2);
    } else {
      const int l = (k - 6) / 3, c = (k - 6) % 3;
      if (live[l]) a.cparts[((long long)l * 3 + c) * nb + blk] = s2;
    }
  }
}

// component means of the output from the partial sums (fixed order); the
// same liveness as the launch that wrote them
// (one partial per tile: tens of thousands per slot and component, so each
// thread keeps 8 independent sums and issues 8 loads per round trip)
constexpr int NTM = 1024;
template <int MODE>
__global__ __launch_bounds__(NTM) void k_sr_mean(const double* cparts, int nb, long long n, const LoadState* st,
                                                  const int* mask, double* mean) {
  __shared__ double sh[NTM / WAVE];
  const int c = blockIdx.x, l = blockIdx.y;
  const bool live = MODE == 0 ? st[l].state == ST_ACTIVE : (mask ? mask[l] != 0 : true);
  if (!live) return;
  const double* row = cparts + ((long long)l * 3 + c) * nb;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int b = threadIdx.x;
  for (; b + 7 * NTM < nb; b += 8 * NTM)
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] += row[b + k * NTM];
  for (; b < nb; b += NTM) acc[0] += row[b];
  double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  s = block_sum<NTM>(s, sh);
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
  if (threadIdx.x == 0) red.put(RED_RES, l, blockIdx.x, s);
}

hipError_t launch_sr_expand(const double* coef, int ncx, int ncy, int ncz, int M, int q, const Geom& g, double* s64,
                            float* s32, hipStream_t s) {
  const long long nb = (g.n + NT - 1) / NT;
  hipLaunchKernelGGL(k_sr_expand, dim3((unsigned)(nb < 65535 ? nb : 65535)), dim3(NT), 0, s, coef, ncx, ncy, ncz, M, q,
                     g, s64, s32);
  return hipGetLastError();
}

namespace {
constexpr int SR_BX = 64, SR_BY = 4;

struct SrGrid {
  int tz, nxt, nyt, nzt, gy, nb;
};

SrGrid sr_grid(const Geom& g) {
  SrGrid t;
  t.nxt = (g.nx + SR_BX - 1) / SR_BX;
  t.nyt = (g.ny + SR_BY - 1) / SR_BY;
  // one plane per block, groups of up to 4 tile rows (4 x 4 = 16 rows): the
  // order that measured fastest at 256^3 (planes per block 1 to 16, groups
  // of 1 to 64 tile rows); gy divides nyt so the order covers every tile once
  t.tz = 1;
  t.gy = t.nyt % 4 == 0 ? 4 : (t.nyt % 2 == 0 ? 2 : 1);
  t.nzt = g.nz;
  t.nb = t.nxt * t.nyt * t.nzt;
  return t;
}
}  // namespace

template <typename T>
hipError_t launch_sr_apply(const SArgs<T>& a, hipStream_t s) {
  if (a.nslot > 6 || a.g.dim != 3) return hipErrorInvalidValue;
  const SrGrid t = sr_grid(a.g);
  if (t.nb > a.red.maxblk) return hipErrorInvalidValue;
  if constexpr (std::is_same<T, float>::value) {
    if (a.g.nx % WAVE == 0 && t.tz == 1)
      hipLaunchKernelGGL(k_sr_apply3w<SR_BY>, dim3(xcd_grid(t.nb)), dim3(NT), 0, s, a, t.nxt, t.nyt, t.nzt, t.gy);
    else
      hipLaunchKernelGGL((k_sr_apply3t<T, T, 0, SR_BX, SR_BY>), dim3(xcd_grid(t.nb)), dim3(NT), 0, s, a, t.tz,
                         t.nxt, t.nyt, t.nzt, t.gy);
  } else {
    hipLaunchKernelGGL((k_sr_apply3t<T, T, 0, SR_BX, SR_BY>), dim3(xcd_grid(t.nb)), dim3(NT), 0, s, a, t.tz, t.nxt,
                       t.nyt, t.nzt, t.gy);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sr_mean<0>, dim3(3, a.nslot), dim3(NTM), 0, s, (const double*)a.cparts, t.nb,
                     a.g.n, (const LoadState*)a.st, (const int*)nullptr, a.mean);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(a.red, a.st, nullptr, RED_PQ, t.nb, a.nslot, -1, nullptr, s);
}

hipError_t launch_sr_residual(const SArgs<double>& a, bool out32, double* res2, hipStream_t s) {
  if (a.nslot > 6 || a.g.dim != 3) return hipErrorInvalidValue;
  const SrGrid t = sr_grid(a.g);
  if (t.nb > a.red.maxblk) return hipErrorInvalidValue;
  const dim3 grid(xcd_grid(t.nb));
  if (out32)
    hipLaunchKernelGGL((k_sr_apply3t<double, float, 1, SR_BX, SR_BY>), grid, dim3(NT), 0, s, a, t.tz, t.nxt, t.nyt,
                       t.nzt, t.gy);
  else
    hipLaunchKernelGGL((k_sr_apply3t<double, double, 1, SR_BX, SR_BY>), grid, dim3(NT), 0, s, a, t.tz, t.nxt, t.nyt,
                       t.nzt, t.gy);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sr_mean<1>, dim3(3, a.nslot), dim3(NTM), 0, s, (const double*)a.cparts, t.nb,
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

int sr_max_blocks(const Geom& g) { return g.dim == 3 ? sr_grid(g).nb : 0; }

template hipError_t launch_sr_apply<float>(const SArgs<float>&, hipStream_t);
template hipError_t launch_sr_apply<double>(const SArgs<double>&, hipStream_t);

#ifdef CELLFFT_BOUNDS_CHECK
unsigned int oob_take_surrogate() { return oob_take(); }
#endif

}  // namespace cellfft
