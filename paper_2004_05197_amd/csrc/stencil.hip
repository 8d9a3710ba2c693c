// Fused P1 finite-element operator on the Kuhn subdivision (gfx950).
//
// Per voxel and per simplex s (3D: the 6 axis permutations p, vertices
// v0 = 0, v_j = v_{j-1} + e_{p_j}; 2D: the 2 triangles), the displacement
// gradient is exact from successive differences along the monotone vertex
// path, G[:, p_j] = (u(v_j) - u(v_{j-1})) / h_{p_j}; the stress is the linear
// isotropic law sigma = lambda tr(eps) I + 2 mu eps (eps = sym G); the
// divergence scatter B^T sigma sends |s| sigma[:, p_j] / h_{p_j} with
// opposite signs to the two ends of path step j.  2D is plane strain.
//
// k_stencil3   3D, z-marching tiles of bx x by nodes: each layer of voxels
//              is computed once per tile (plus a one-voxel halo), corner
//              contributions are exchanged through LDS, the +z contributions
//              are carried in registers to the next node plane.
//              mode 0: q = K p with p.q partials, alpha = rz / pq finalised
//              mode 1: r = -B^T D (eps_bar + B u) with ||r||^2 (FP64)
// k_stencil2   2D analogue (node-centric gather; the 2D grids are small)
// k_udotr      u^I . r^J products; with the residual launch's mean stresses
//              they give the energy-form effective stiffness (k_homog_combine)
// k_grad       per-voxel derivative of sum_IJ a_IJ C*_IJ w.r.t. E
#include <algorithm>
#include <type_traits>

#include "kernels.h"

namespace cellfft {

__constant__ int kPerm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

template <int I, int J> struct SymIdx;  // tensor (I, J) -> storage (00,11,22,12,02,01)
template <> struct SymIdx<0, 0> { static constexpr int v = 0; };
template <> struct SymIdx<1, 1> { static constexpr int v = 1; };
template <> struct SymIdx<2, 2> { static constexpr int v = 2; };
template <> struct SymIdx<1, 2> { static constexpr int v = 3; };
template <> struct SymIdx<2, 1> { static constexpr int v = 3; };
template <> struct SymIdx<0, 2> { static constexpr int v = 4; };
template <> struct SymIdx<2, 0> { static constexpr int v = 4; };
template <> struct SymIdx<0, 1> { static constexpr int v = 5; };
template <> struct SymIdx<1, 0> { static constexpr int v = 5; };

__host__ __device__ constexpr int sym_idx(int i, int j) {
  return i == j ? i : (i + j == 3 ? 3 : (i + j == 2 ? 4 : 5));
}

// Edge formulation of one voxel.  The 12 edges of the six monotone paths
// are: first edges along a from corner 0 (e0[a]), middle edges along b from
// corner 1<<a (em[a][b], a != b), last edges along a into corner 7 (el[a]).
// The first and last edges are shared by two simplices, the middle ones
// belong to one.  Simplex s with axis order (p0, p1, p2) has the gradient
// columns G[:, p0] = e0[p0], G[:, p1] = em[p0][p1], G[:, p2] = el[p2]
// (differences, scaled by 1/h_a unless UNI) and sends the flux column
// sigma_s[:, p_j] from the start to the end of its step j; the fluxes of a
// shared edge are summed first, then each corner gets the signed sum of the
// fluxes of its edges (12 edges instead of 18 simplex steps).
// UNI (equal edge lengths h): differences unscaled, lw = lambda |s| / h^2,
//   mw = mu |s| / h^2, sb = |s| D eps_bar / h: corner forces need no scaling.
// !UNI: differences and fluxes times 1/h_a, lw = lambda |s|, sb = |s| D eps_bar.
// One Kuhn simplex (compile-time axis order A0, A1, A2) given the edge
// differences of its path: first edge along A0 from corner 0 (e0[A0]),
// middle edge along A1 from corner 1<<A0 (em[A0][A1]), last edge along A2
// into corner 7 (el[A2]).  Computes the stress and adds its three flux
// columns to the edge fluxes (F0 / FL: first use assigns).
template <typename T, int A0, int A1, int A2, bool F0, bool FL, bool MACRO>
__device__ __forceinline__ void tet3(const T (&e0)[3][3], const T (&em)[3][3][3], const T (&el)[3][3], T lw,
                                     T mw2, T mw, const T* sb, T (&p0)[3][3], T (&pm)[3][3][3], T (&pl)[3][3],
                                     T* sacc) {
  T G[3][3];  // G[k][a]: component k of the gradient along axis a
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    G[k][A0] = e0[A0][k];
    G[k][A1] = em[A0][A1][k];
    G[k][A2] = el[A2][k];
  }
  const T lt = lw * (G[0][0] + G[1][1] + G[2][2]);
  T s[6];
  s[0] = lt + mw2 * G[0][0];
  s[1] = lt + mw2 * G[1][1];
  s[2] = lt + mw2 * G[2][2];
  s[3] = mw * (G[1][2] + G[2][1]);
  s[4] = mw * (G[0][2] + G[2][0]);
  s[5] = mw * (G[0][1] + G[1][0]);
  if (MACRO) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      s[i] += sb[i];
      sacc[i] += s[i];
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T t0 = s[sym_idx(k, A0)], t1 = s[sym_idx(k, A1)], t2 = s[sym_idx(k, A2)];
    p0[A0][k] = F0 ? t0 : p0[A0][k] + t0;
    pm[A0][A1][k] = t1;
    pl[A2][k] = FL ? t2 : pl[A2][k] + t2;
  }
}

// MACRO: sb added to every simplex stress and the 6 stresses (in the
// caller's scaling) summed into sacc[6] (which the caller zeroes).
template <typename T, bool MACRO, bool UNI>
__device__ __forceinline__ void voxel3(const T (&u)[8][3], T lw, T mw, const T* ih, const T* sb,
                                       T (&f)[8][3], T* sacc) {
  const T mw2 = mw + mw;
  T e0[3][3], em[3][3][3], el[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      e0[a][k] = u[1 << a][k] - u[0][k];
      el[a][k] = u[7][k] - u[7 ^ (1 << a)][k];
      if (!UNI) {
        e0[a][k] *= ih[a];
        el[a][k] *= ih[a];
      }
#pragma unroll
      for (int b = 0; b < 3; ++b)
        if (b != a) {
          em[a][b][k] = u[(1 << a) | (1 << b)][k] - u[1 << a][k];
          if (!UNI) em[a][b][k] *= ih[b];
        }
    }
  T p0[3][3], pm[3][3][3], pl[3][3];
  tet3<T, 0, 1, 2, true, true, MACRO>(e0, em, el, lw, mw2, mw, sb, p0, pm, pl, sacc);
  tet3<T, 0, 2, 1, false, true, MACRO>(e0, em, el, lw, mw2, mw, sb, p0, pm, pl, sacc);
  tet3<T, 1, 0, 2, true, false, MACRO>(e0, em, el, lw, mw2, mw, sb, p0, pm, pl, sacc);
  tet3<T, 1, 2, 0, false, true, MACRO>(e0, em, el, lw, mw2, mw, sb, p0, pm, pl, sacc);
  tet3<T, 2, 0, 1, true, false, MACRO>(e0, em, el, lw, mw2, mw, sb, p0, pm, pl, sacc);
  tet3<T, 2, 1, 0, false, false, MACRO>(e0, em, el, lw, mw2, mw, sb, p0, pm, pl, sacc);
  if (!UNI) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        p0[a][k] *= ih[a];
        pl[a][k] *= ih[a];
#pragma unroll
        for (int b = 0; b < 3; ++b)
          if (b != a) pm[a][b][k] *= ih[b];
      }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    f[0][k] = -(p0[0][k] + p0[1][k] + p0[2][k]);
    f[7][k] = pl[0][k] + pl[1][k] + pl[2][k];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int b = (a + 1) % 3, c = (a + 2) % 3;
      f[1 << a][k] = p0[a][k] - pm[a][b][k] - pm[a][c][k];            // first-edge end, middle-edge starts
      f[7 ^ (1 << a)][k] = pm[b][c][k] + pm[c][b][k] - pl[a][k];      // middle-edge ends, last-edge start
    }
  }
}

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// element at a 32-bit byte offset from a block-uniform base pointer: the
// access takes the scalar-base + 32-bit vector-offset form (one add per
// access instead of a 64-bit address computation); offsets stay below 4 GiB
// for every supported grid (3 x 256^3 FP64 values per load: 402 MB).
template <typename T>
__device__ __forceinline__ T ld_off(const T* base, unsigned boff) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff);
}
template <typename T>
__device__ __forceinline__ void st_off(T* base, unsigned boff, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + boff) = v;
}
// the same with the extent [lo, hi) of the buffer the access may touch: the
// bounds-checked build compares the address with it (the normal build
// expands to the plain access, lo and hi unevaluated)
#ifdef CELLFFT_BOUNDS_CHECK
template <typename T>
__device__ __forceinline__ T ld_off_ck(const T* base, unsigned boff, const void* lo, const void* hi) {
  return ck_ld(reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff), 0, lo, hi);
}
template <typename T>
__device__ __forceinline__ void st_off_ck(T* base, unsigned boff, T v, const void* lo, const void* hi) {
  ck_st(reinterpret_cast<T*>(reinterpret_cast<char*>(base) + boff), 0, lo, hi, v);
}
#define LD_OFF(base, boff, lo, hi) ld_off_ck(base, boff, lo, hi)
#define ST_OFF(base, boff, v, lo, hi) st_off_ck(base, boff, v, lo, hi)
#else
#define LD_OFF(base, boff, lo, hi) ld_off(base, boff)
#define ST_OFF(base, boff, v, lo, hi) st_off(base, boff, v)
#endif

// macro stress D eps_bar (tensor storage) scaled by sc, with lw/mw already
// holding the |s| (and 1/h^2) factors of the caller
template <typename T>
__device__ __forceinline__ void macro_stress(const double* e, T lw, T mw, T sc, T* sb) {
  const T tr = (T)(e[0] + e[1] + e[2]);
  sb[0] = sc * (lw * tr + T(2) * mw * (T)e[0]);
  sb[1] = sc * (lw * tr + T(2) * mw * (T)e[1]);
  sb[2] = sc * (lw * tr + T(2) * mw * (T)e[2]);
  sb[3] = sc * (T(2) * mw * (T)e[3]);
  sb[4] = sc * (T(2) * mw * (T)e[4]);
  sb[5] = sc * (T(2) * mw * (T)e[5]);
}

// =========================================================== 3D stencil
// Block: bx x by node tile, marching tz node planes along z.  Per layer k
// (voxels between node planes k and k+1) every thread computes voxel
// (tx-1, ty-1) of the tile (the node's lower-left-back voxel) and keeps its
// (1,1,*) corners; the (bx+by+1) halo voxels are spread over the first
// threads.  The (0,0,*), (1,0,*), (0,1,*) corners go to LDS for the three
// neighbouring nodes; the (.,.,1) corners are carried to the next plane.
// Node plane k+2 and the material of layer k+1 are prefetched into
// registers while layer k is computed.
constexpr int PF_MAX = 8;  // ceil(3 (bx+2)(by+2) / 256) for every tile used

template <typename T, typename TO, int MODE, bool UNI>
__global__ __launch_bounds__(NT) void k_stencil3(KArgs<T> a, int bx, int by, int tz) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* pl = reinterpret_cast<T*>(smem_raw);
  const int PW = bx + 2, PH = by + 2, PP = PW * PH;
  T* cb = pl + 6 * PP;
  const int VW = bx + 1, VV = VW * (by + 1);
  __shared__ double sh[NT / WAVE];
  const int tid = threadIdx.x;
  const int tx = tid % bx, ty = tid / bx;
  const bool worker = ty < by;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const long long n = a.g.n;
  const int x0 = blockIdx.x * bx, y0 = blockIdx.y * by, z0 = blockIdx.z * tz;
  const T ih[3] = {(T)(1.0 / a.g.h[0]), (T)(1.0 / a.g.h[1]), (T)(1.0 / a.g.h[2])};
  const double wd = a.g.h[0] * a.g.h[1] * a.g.h[2] / 6.0;
  const T w = (T)((UNI ? wd / (a.g.h[0] * a.g.h[0]) : wd) * (MODE == 0 && a.negate ? -1.0 : 1.0));
  const T msc = (T)(UNI ? a.g.h[0] : 1.0);  // macro stress scale relative to lw, mw
  const int nextra = bx + by + 1;
  const bool has_extra = tid < nextra;
  // voxel handled as the extra of this thread (relative to the tile)
  const int ex = tid < by ? bx - 1 : tid - by - 1;
  const int ey = tid < by ? tid - 1 : by - 1;
  const int blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  // per prefetch slot: offset of this thread's plane element within a
  // z-plane of the field (component c, wrapped x and y), -1 if unused
  int poff[PF_MAX];
#pragma unroll
  for (int q = 0; q < PF_MAX; ++q) {
    const int e = tid + q * NT;
    poff[q] = -1;
    if (e < 3 * PP) {
      const int c = e / PP, rem = e - c * PP;
      const int py = rem / PW, px = rem - py * PW;
      poff[q] = c * (int)n + wrapi(y0 - 1 + py, ny) * nx + wrapi(x0 - 1 + px, nx);
    }
  }
  for (int l = 0; l < a.nload; ++l) {
    bool live;
    if (MODE == 0) live = a.st[l].state == ST_ACTIVE;
    else live = a.mask ? a.mask[l] != 0 : (a.only_load < 0 || a.only_load == l);
    if (!live) continue;
    const T* u = a.u ? a.u + l * a.lstride : nullptr;
    TO* out = reinterpret_cast<TO*>(a.out) + l * a.lstride;
    const double* eb = a.eps[l % a.lpc];
    const T* matl = a.mat + (long long)(l / a.lpc) * a.mat_stride;
    T pf[PF_MAX];
    auto fetch_plane = [&](int zp) {
      const int zoff = wrapi(zp, nz) * (ny * nx);
#pragma unroll
      for (int q = 0; q < PF_MAX; ++q)
        if (poff[q] >= 0) pf[q] = u ? u[poff[q] + zoff] : T(0);
    };
    auto store_plane = [&](int slot) {
      T* dst = pl + slot * 3 * PP;
#pragma unroll
      for (int q = 0; q < PF_MAX; ++q)
        if (poff[q] >= 0) dst[tid + q * NT] = pf[q];
    };
    auto mat_of = [&](int vx, int vy, int k, T& lw, T& mw) {
      const long long vid = ((long long)wrapi(k, nz) * ny + wrapi(y0 + vy, ny)) * nx + wrapi(x0 + vx, nx);
      lw = matl[2 * vid];  // raw: scaled by w where used (no wait at the load)
      mw = matl[2 * vid + 1];
    };
    // computes voxel (vx, vy) of layer k from planes in slots s0 (k), s1 (k+1)
    auto voxel = [&](int vx, int vy, int s0, int s1, T lw, T mw, T (&own)[2][3], T* sv) {
      const T* p0 = pl + s0 * 3 * PP;
      const T* p1 = pl + s1 * 3 * PP;
      T uu[8][3];
#pragma unroll
      for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int oy = 0; oy < 2; ++oy)
#pragma unroll
          for (int ox = 0; ox < 2; ++ox)
#pragma unroll
            for (int c = 0; c < 3; ++c)
              uu[ox + 2 * oy + 4 * oz][c] = (oz ? p1 : p0)[c * PP + (vy + 1 + oy) * PW + (vx + 1 + ox)];
      T f[8][3];
      T sb[6];
      if (MODE == 1) {
        macro_stress(eb, lw, mw, msc, sb);
        voxel3<T, true, UNI>(uu, lw, mw, ih, sb, f, sv);
      } else {
        voxel3<T, false, UNI>(uu, lw, mw, ih, sb, f, sv);
      }
      const int vi = (vy + 1) * VW + (vx + 1);
#pragma unroll
      for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          cb[((0 * 2 + oz) * 3 + c) * VV + vi] = f[0 + 4 * oz][c];  // corner (0,0)
          cb[((1 * 2 + oz) * 3 + c) * VV + vi] = f[1 + 4 * oz][c];  // corner (1,0)
          cb[((2 * 2 + oz) * 3 + c) * VV + vi] = f[2 + 4 * oz][c];  // corner (0,1)
          own[oz][c] = f[3 + 4 * oz][c];                            // corner (1,1)
        }
    };
    double acc = 0.0;
    double sacc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    T carry[3] = {T(0), T(0), T(0)};
    fetch_plane(z0 - 1);
    store_plane(0);
    fetch_plane(z0);
    store_plane(1);
    T lw0 = T(0), mw0 = T(0), lwe = T(0), mwe = T(0);
    if (worker) mat_of(tx - 1, ty - 1, z0 - 1, lw0, mw0);
    if (has_extra) mat_of(ex, ey, z0 - 1, lwe, mwe);
    __syncthreads();
    for (int L = 0; L <= tz; ++L) {
      const int k = z0 - 1 + L;
      const int s0 = L & 1, s1 = (L + 1) & 1;
      if (L < tz) fetch_plane(k + 2);
      T lw1 = T(0), mw1 = T(0), lwe1 = T(0), mwe1 = T(0);
      if (L < tz) {
        if (worker) mat_of(tx - 1, ty - 1, k + 1, lw1, mw1);
        if (has_extra) mat_of(ex, ey, k + 1, lwe1, mwe1);
      }
      T own[2][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
      T pk[3] = {T(0), T(0), T(0)};  // p at this thread's node of plane k
      if (worker && MODE == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) pk[c] = pl[s0 * 3 * PP + c * PP + (ty + 1) * PW + (tx + 1)];
      }
      // pass 0: the thread's own voxel, pass 1: its halo voxel (if any);
      // one code body so the two are not interleaved (register pressure)
#pragma nounroll
      for (int pass = 0; pass < 2; ++pass) {
        const bool doit = pass == 0 ? worker : has_extra;
        if (!doit) continue;
        T o[2][3];
        T sv[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
        voxel(pass == 0 ? tx - 1 : ex, pass == 0 ? ty - 1 : ey, s0, s1, (pass == 0 ? lw0 : lwe) * w,
              (pass == 0 ? mw0 : mwe) * w, o, sv);
        if (pass == 0) {
#pragma unroll
          for (int z = 0; z < 2; ++z)
#pragma unroll
            for (int c = 0; c < 3; ++c) own[z][c] = o[z][c];
          // the voxel below-left-behind a valid node is owned exactly once
          if (MODE == 1 && L < tz && z0 + L < nz && x0 + tx < nx && y0 + ty < ny) {
#pragma unroll
            for (int i = 0; i < 6; ++i) sacc[i] += (double)sv[i];
          }
        }
      }
      __syncthreads();
      if (worker) {
        const int i00 = (ty + 1) * VW + (tx + 1);  // voxel (tx, ty)
        const int i10 = (ty + 1) * VW + tx;        // voxel (tx-1, ty)
        const int i01 = ty * VW + (tx + 1);        // voxel (tx, ty-1)
        T val[3], nc[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          val[c] = carry[c] + own[0][c] + cb[((0 * 2 + 0) * 3 + c) * VV + i00] +
                   cb[((1 * 2 + 0) * 3 + c) * VV + i10] + cb[((2 * 2 + 0) * 3 + c) * VV + i01];
          nc[c] = own[1][c] + cb[((0 * 2 + 1) * 3 + c) * VV + i00] +
                  cb[((1 * 2 + 1) * 3 + c) * VV + i10] + cb[((2 * 2 + 1) * 3 + c) * VV + i01];
        }
        const int gx = x0 + tx, gy = y0 + ty;
        if (L >= 1 && k < nz && gx < nx && gy < ny) {
          const long long node = ((long long)k * ny + gy) * nx + gx;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            if (MODE == 0) {
              out[c * n + node] = (TO)val[c];
              acc += (double)pk[c] * (double)val[c];
            } else {
              out[c * n + node] = (TO)(-val[c]);
              acc += (double)val[c] * (double)val[c];
            }
          }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) carry[c] = nc[c];
      }
      if (L < tz) store_plane(s0);
      lw0 = lw1;
      mw0 = mw1;
      lwe = lwe1;
      mwe = mwe1;
      __syncthreads();
    }
    const double bs = block_sum<NT>(acc, sh);
    if (tid == 0) a.red.put(MODE == 0 ? RED_PQ : RED_RES, l, blk, bs);
    if (MODE == 1 && a.sparts) {
      for (int i = 0; i < 6; ++i) {
        const double v = block_sum<NT>(sacc[i], sh);
        if (tid == 0) a.sparts[((long long)l * 6 + i) * a.red.maxblk + blk] = v * (double)msc;
      }
    }
  }
}

// Same scheme with compile-time tile shape (BX x BY nodes, NTH = BX * BY
// threads): all LDS offsets are constants and every per-voxel global index is
// a precomputed in-plane offset plus the plane base, so the loop body is the
// simplex arithmetic, LDS traffic and a handful of adds.
template <typename T, typename TO, int MODE, bool UNI, int BX, int BY>
__global__ __launch_bounds__(BX* BY) void k_stencil3t(KArgs<T> a, int tz, int nxt, int nyt, int nzt) {
  constexpr int NTH = BX * BY;
  constexpr int PW = BX + 2, PP = PW * (BY + 2);
  constexpr int VW = BX + 1, VV = VW * (BY + 1);
  constexpr int PF = (3 * PP + NTH - 1) / NTH;
  constexpr int NEXTRA = BX + BY + 1;
  __shared__ T pl[2 * 3 * PP];
  __shared__ T cb[18 * VV];
  __shared__ T mt[2 * VV];  // (lambda, mu) of the layer's voxels, by their cb index
  __shared__ double sh[NTH / WAVE];
  const int tid = threadIdx.x;
  const int tx = tid % BX, ty = tid / BX;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int n = (int)a.g.n;
  const int nxy = nx * ny;
  // logical work item = (tile, load), load fastest, tiles x-then-y-then-z
  const int ntiles = nxt * nyt * nzt;
  const int item = xcd_order(blockIdx.x, ntiles * a.nload);
  if (item < 0) return;
  const int l = item % a.nload;
  const int blk = item / a.nload;
  {
    bool live;
    if (MODE == 0) live = a.st[l].state == ST_ACTIVE;
    else live = a.mask ? a.mask[l] != 0 : (a.only_load < 0 || a.only_load == l);
    if (!live) return;
  }
  const int bxi = blk % nxt, byi = (blk / nxt) % nyt, bzi = blk / (nxt * nyt);
  const int x0 = bxi * BX, y0 = byi * BY, z0 = bzi * tz;
  const T ih[3] = {(T)(1.0 / a.g.h[0]), (T)(1.0 / a.g.h[1]), (T)(1.0 / a.g.h[2])};
  const double wd = a.g.h[0] * a.g.h[1] * a.g.h[2] / 6.0;
  const T w = (T)((UNI ? wd / (a.g.h[0] * a.g.h[0]) : wd) * (MODE == 0 && a.negate ? -1.0 : 1.0));
  const T msc = (T)(UNI ? a.g.h[0] : 1.0);
  const bool has_extra = tid < NEXTRA;
  const int ex = tid < BY ? BX - 1 : tid - BY - 1;
  const int ey = tid < BY ? tid - 1 : BY - 1;
  // byte offsets (in-plane part) of the node values this thread stages
  unsigned poff[PF];
  bool pon[PF];
#pragma unroll
  for (int q = 0; q < PF; ++q) {
    const int e = tid + q * NTH;
    pon[q] = e < 3 * PP;
    poff[q] = 0;
    if (pon[q]) {
      const int c = e / PP, rem = e - c * PP;
      const int py = rem / PW, px = rem - py * PW;
      poff[q] = (unsigned)(c * n + wrapi(y0 - 1 + py, ny) * nx + wrapi(x0 - 1 + px, nx)) * (unsigned)sizeof(T);
    }
  }
  // in-plane voxel offsets (material) and LDS corner bases of the two voxels
  const int vown = wrapi(y0 + ty - 1, ny) * nx + wrapi(x0 + tx - 1, nx);
  const int vext = wrapi(y0 + ey, ny) * nx + wrapi(x0 + ex, nx);
  const int bown = ty * PW + tx;              // voxel (tx-1, ty-1): corner (0,0) at (tx, ty)
  const int bext = (ey + 1) * PW + (ex + 1);
  const int cown = ty * VW + tx;              // cb index of voxel (tx-1, ty-1)
  const int cext = (ey + 1) * VW + (ex + 1);
  const bool out_ok = (x0 + tx < nx) && (y0 + ty < ny);
  {
    const T* u = a.u ? a.u + l * a.lstride : nullptr;
    TO* out = reinterpret_cast<TO*>(a.out) + l * a.lstride;
    const T* matl = a.mat + (long long)(l / a.lpc) * a.mat_stride;
#ifdef CELLFFT_BOUNDS_CHECK
    // extents of the slot's fields and the cell's material
    const T* u_hi = u ? u + a.lstride : nullptr;
    const TO* out_hi = out + a.lstride;
    const T* mat_hi = matl + 2 * a.g.n;
#endif
    T sbd[6];
    if (MODE == 1) {
      const double* e = a.eps[l % a.lpc];
#pragma unroll
      for (int i = 0; i < 6; ++i) sbd[i] = (T)e[i];
    }
    T pf[PF];
    auto fetch_plane = [&](int zp) {
      const unsigned zb = (unsigned)(wrapi(zp, nz) * nxy) * (unsigned)sizeof(T);
#pragma unroll
      for (int q = 0; q < PF; ++q)
        if (pon[q]) pf[q] = u ? LD_OFF(u, poff[q] + zb, u, u_hi) : T(0);
    };
    // the material goes through LDS like the node planes: loaded one layer
    // ahead, stored after the layer's last use, so no wait for a load falls
    // inside the voxel computations
    using T2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
    T2 mo, me;
    const T2* mat2 = reinterpret_cast<const T2*>(matl);
    auto fetch_mat = [&](int zl) {
      const int zo = wrapi(zl, nz) * nxy;
      mo = LD_OFF(mat2, (unsigned)(zo + vown) * (unsigned)sizeof(T2), matl, mat_hi);
      if (has_extra) me = LD_OFF(mat2, (unsigned)(zo + vext) * (unsigned)sizeof(T2), matl, mat_hi);
    };
    auto store_mat = [&]() {
      mt[2 * cown] = mo.x;
      mt[2 * cown + 1] = mo.y;
      if (has_extra) {
        mt[2 * cext] = me.x;
        mt[2 * cext + 1] = me.y;
      }
    };
    auto store_plane = [&](int slot) {
#pragma unroll
      for (int q = 0; q < PF; ++q)
        if (pon[q]) pl[slot * 3 * PP + tid + q * NTH] = pf[q];
    };
    auto voxel = [&](int base, int ci, int s0, int s1, T lw, T mw, T (&own)[2][3], T* sv) {
      T uu[8][3];
#pragma unroll
      for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int oy = 0; oy < 2; ++oy)
#pragma unroll
          for (int ox = 0; ox < 2; ++ox)
#pragma unroll
            for (int c = 0; c < 3; ++c)
              uu[ox + 2 * oy + 4 * oz][c] = pl[(oz ? s1 : s0) * 3 * PP + c * PP + base + oy * PW + ox];
      T f[8][3];
      if (MODE == 1) {
        T sb[6];
        const T tr = sbd[0] + sbd[1] + sbd[2];
        sb[0] = msc * (lw * tr + T(2) * mw * sbd[0]);
        sb[1] = msc * (lw * tr + T(2) * mw * sbd[1]);
        sb[2] = msc * (lw * tr + T(2) * mw * sbd[2]);
        sb[3] = msc * (T(2) * mw * sbd[3]);
        sb[4] = msc * (T(2) * mw * sbd[4]);
        sb[5] = msc * (T(2) * mw * sbd[5]);
        voxel3<T, true, UNI>(uu, lw, mw, ih, sb, f, sv);
      } else {
        voxel3<T, false, UNI>(uu, lw, mw, ih, nullptr, f, sv);
      }
#pragma unroll
      for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          cb[((0 * 2 + oz) * 3 + c) * VV + ci] = f[0 + 4 * oz][c];
          cb[((1 * 2 + oz) * 3 + c) * VV + ci] = f[1 + 4 * oz][c];
          cb[((2 * 2 + oz) * 3 + c) * VV + ci] = f[2 + 4 * oz][c];
          own[oz][c] = f[3 + 4 * oz][c];
        }
    };
    double acc = 0.0;
    double sacc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    T carry[3] = {T(0), T(0), T(0)};
    fetch_plane(z0 - 1);
    store_plane(0);
    fetch_plane(z0);
    store_plane(1);
    fetch_mat(z0 - 1);
    store_mat();
    __syncthreads();
    for (int L = 0; L <= tz; ++L) {
      const int k = z0 - 1 + L;
      const int s0 = L & 1, s1 = (L + 1) & 1;
      if (L < tz) {
        fetch_plane(k + 2);
        fetch_mat(k + 1);
      }
      T pk[3] = {T(0), T(0), T(0)};
      if (MODE == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) pk[c] = pl[s0 * 3 * PP + c * PP + (ty + 1) * PW + (tx + 1)];
      }
      T own[2][3];
#pragma nounroll
      for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1 && !has_extra) break;
        T o[2][3];
        T sv[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
        const int ci = pass == 0 ? cown : cext;
        voxel(pass == 0 ? bown : bext, ci, s0, s1, mt[2 * ci] * w, mt[2 * ci + 1] * w, o, sv);
        if (pass == 0) {
#pragma unroll
          for (int z = 0; z < 2; ++z)
#pragma unroll
            for (int c = 0; c < 3; ++c) own[z][c] = o[z][c];
          if (MODE == 1 && L < tz && z0 + L < nz) {
#pragma unroll
            for (int i = 0; i < 6; ++i) sacc[i] += (double)sv[i];
          }
        }
      }
      __syncthreads();
      {
        const int i00 = (ty + 1) * VW + (tx + 1);
        const int i10 = (ty + 1) * VW + tx;
        const int i01 = ty * VW + (tx + 1);
        T val[3], nc[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          val[c] = carry[c] + own[0][c] + cb[(0 * 3 + c) * VV + i00] + cb[(6 + c) * VV + i10] +
                   cb[(12 + c) * VV + i01];
          nc[c] = own[1][c] + cb[(3 + c) * VV + i00] + cb[(9 + c) * VV + i10] + cb[(15 + c) * VV + i01];
        }
        if (L >= 1 && k < nz && out_ok) {
          const unsigned nb = (unsigned)(k * nxy + (y0 + ty) * nx + (x0 + tx)) * (unsigned)sizeof(TO);
          const unsigned cs = (unsigned)n * (unsigned)sizeof(TO);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            if (MODE == 0) {
              ST_OFF(out, nb + c * cs, (TO)val[c], out, out_hi);
              acc += (double)pk[c] * (double)val[c];
            } else {
              ST_OFF(out, nb + c * cs, (TO)(-val[c]), out, out_hi);
              acc += (double)val[c] * (double)val[c];
            }
          }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) carry[c] = nc[c];
      }
      if (L < tz) {
        store_plane(s0);
        store_mat();
      }
      __syncthreads();
    }
    const double bs = block_sum<NTH>(acc, sh);
    if (tid == 0) a.red.put(MODE == 0 ? RED_PQ : RED_RES, l, blk, bs);
    if (MODE == 1 && a.sparts) {
      for (int i = 0; i < 6; ++i) {
        const double v = block_sum<NTH>(sacc[i], sh);
        if (tid == 0) a.sparts[((long long)l * 6 + i) * a.red.maxblk + blk] = v * (double)msc;
      }
    }
  }
}

// =========================================================== 2D stencil
// plane strain, 2 triangles per pixel: (0,0)->(1,0)->(1,1), (0,0)->(0,1)->(1,1)
template <typename T, int A0, int A1, bool MACRO>
__device__ __forceinline__ void simplex2(const T (&u)[4][2], T lw, T mw, const T* ih, const T* sb,
                                         T (&f)[4][2], T* sacc) {
  constexpr int c0 = 0, c1 = 1 << A0, c2 = 3;
  T G[2][2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    G[k][A0] = (u[c1][k] - u[c0][k]) * ih[A0];
    G[k][A1] = (u[c2][k] - u[c1][k]) * ih[A1];
  }
  const T lt = lw * (G[0][0] + G[1][1]);
  T s[3];  // 00, 11, 01
  s[0] = lt + T(2) * mw * G[0][0];
  s[1] = lt + T(2) * mw * G[1][1];
  s[2] = mw * (G[0][1] + G[1][0]);
  if (MACRO) {
    s[0] += sb[0];
    s[1] += sb[1];
    s[2] += sb[2];
    sacc[0] += s[0];
    sacc[1] += s[1];
    sacc[2] += s[2];
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const T t1 = s[k == A0 ? k : 2] * ih[A0];
    const T t2 = s[k == A1 ? k : 2] * ih[A1];
    f[c0][k] -= t1;
    f[c1][k] += t1 - t2;
    f[c2][k] += t2;
  }
}

template <typename T, typename TO, int MODE>
__global__ __launch_bounds__(NT) void k_stencil2(KArgs<T> a) {
  __shared__ double sh[NT / WAVE];
  const int l = blockIdx.y;
  bool live;
  if (MODE == 0) live = a.st[l].state == ST_ACTIVE;
  else live = a.mask ? a.mask[l] != 0 : (a.only_load < 0 || a.only_load == l);
  if (!live) return;
  const int nx = a.g.nx, ny = a.g.ny;
  const long long n = a.g.n;
  const T ih[2] = {(T)(1.0 / a.g.h[0]), (T)(1.0 / a.g.h[1])};
  const T w = (T)(a.g.h[0] * a.g.h[1] / 2.0 * (MODE == 0 && a.negate ? -1.0 : 1.0));
  const T* u = a.u ? a.u + l * a.lstride : nullptr;
  TO* out = reinterpret_cast<TO*>(a.out) + l * a.lstride;
  const double* eb = a.eps[l % a.lpc];
  const T* matl = a.mat + (long long)(l / a.lpc) * a.mat_stride;
  double acc = 0.0;
  double sacc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const long long node = (long long)blockIdx.x * NT + threadIdx.x;
  if (node < n) {
    const int i = (int)(node % nx), j = (int)(node / nx);
    T val[2] = {T(0), T(0)};
    // the node is corner (ox, oy) of pixel (i - ox, j - oy)
#pragma unroll
    for (int oy = 0; oy < 2; ++oy)
#pragma unroll
      for (int ox = 0; ox < 2; ++ox) {
        const int pi = wrapi(i - ox, nx), pj = wrapi(j - oy, ny);
        T uu[4][2];
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
          for (int cx = 0; cx < 2; ++cx) {
            const long long nd = (long long)wrapi(pj + cy, ny) * nx + wrapi(pi + cx, nx);
#pragma unroll
            for (int c = 0; c < 2; ++c) uu[cx + 2 * cy][c] = u ? u[c * n + nd] : T(0);
          }
        const long long vid = (long long)pj * nx + pi;
        const T lw = matl[2 * vid] * w, mw = matl[2 * vid + 1] * w;
        T sb[3];
        if (MODE == 1) {
          const T tr = (T)(eb[0] + eb[1]);
          sb[0] = lw * tr + T(2) * mw * (T)eb[0];
          sb[1] = lw * tr + T(2) * mw * (T)eb[1];
          sb[2] = T(2) * mw * (T)eb[5];
        }
        T f[4][2] = {};
        T sv[3] = {T(0), T(0), T(0)};
        simplex2<T, 0, 1, MODE == 1>(uu, lw, mw, ih, sb, f, sv);
        simplex2<T, 1, 0, MODE == 1>(uu, lw, mw, ih, sb, f, sv);
        val[0] += f[ox + 2 * oy][0];
        val[1] += f[ox + 2 * oy][1];
        if (MODE == 1 && ox == 0 && oy == 0) {  // pixel (i, j) is owned by node (i, j)
          sacc[0] += (double)sv[0];
          sacc[1] += (double)sv[1];
          sacc[5] += (double)sv[2];
        }
      }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (MODE == 0) {
        out[c * n + node] = (TO)val[c];
        acc += (double)(u ? u[c * n + node] : T(0)) * (double)val[c];
      } else {
        out[c * n + node] = (TO)(-val[c]);
        acc += (double)val[c] * (double)val[c];
      }
    }
  }
  const int cslot = MODE == 0 ? RED_PQ : RED_RES;
  const double bs = block_sum<NT>(acc, sh);
  if (threadIdx.x == 0) a.red.put(cslot, l, blockIdx.x, bs);
  if (MODE == 1 && a.sparts) {
    for (int i = 0; i < 6; ++i) {
      const double v = block_sum<NT>(sacc[i], sh);
      if (threadIdx.x == 0) a.sparts[((long long)l * 6 + i) * a.red.maxblk + blockIdx.x] = v;
    }
  }
}

// =============================================== 3D row-wave stencil (FP32)
// q = K p for grids with nx = 64 V (V = 1, 2, 4), one wavefront per periodic
// x row: lane i holds nodes and voxels x = V i .. V i + V - 1 of its row, so
// the x neighbours are the next and previous lanes and the wave rotation
// that reaches them wraps exactly like the periodic grid (no x halo).  A
// block has NW waves for the voxel rows y0 .. y0 + NW - 1 and marches
// tz node planes along z (one halo layer below, as the tiled kernel).  Wave
// w owns node row y0 + w: it adds its voxel row's lower-side corner forces,
// the upper-side forces of wave w - 1 (through LDS, double buffered by step
// parity) and the upper-z forces of the previous layer (carried in a
// per-lane LDS area, which keeps the registers of two waves per SIMD, or
// of one at four voxels per lane).  The upper-side forces of the last wave belong to node row
// y0 + NW of the next tile: they go to the edge rows, which the x
// forward pass (or the fix-up launch) adds to q.  p.q is summed from every
// contribution with the p of its node, so it needs no fix-up.
template <int V> __device__ __forceinline__ void rw_load(const float* p, float* o) {
  if constexpr (V == 4) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    o[0] = t.x;
    o[1] = t.y;
    o[2] = t.z;
    o[3] = t.w;
  } else if constexpr (V == 2) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    o[0] = t.x;
    o[1] = t.y;
  } else {
    o[0] = *p;
  }
}
template <int V> __device__ __forceinline__ void rw_store(float* p, const float* o) {
  if constexpr (V == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(o[0], o[1], o[2], o[3]);
  } else if constexpr (V == 2) {
    *reinterpret_cast<float2*>(p) = make_float2(o[0], o[1]);
  } else {
    *p = o[0];
  }
}
// lane i <- lane i + 1 (ROL) or lane i - 1 (ROR), wrapping around the wave
__device__ __forceinline__ float rw_rol(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x134, 0xF, 0xF, false));
}
__device__ __forceinline__ float rw_ror(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x13C, 0xF, 0xF, false));
}

template <int V, int NW, bool UNI>
__global__ __launch_bounds__(NW* WAVE) __attribute__((amdgpu_waves_per_eu(V == 4 ? 1 : 2))) void k_stencil_rw(
    KArgs<float> a, int tz, int nyt, int nzt) {
  constexpr int NTH = NW * WAVE;
  // xch: upper-row forces to the next wave, [parity][wave][comp][lane][V];
  // car: this lane's plane-(k+1) parts carried to the next layer,
  // [wave][own / upper row][comp][x node][lane] (lane fastest: no bank
  // conflicts for the one-value accesses)
  __shared__ float xch[2 * NW * 3 * WAVE * V];
  __shared__ float car[NW * 2 * 3 * V * WAVE];
  __shared__ double sh[NTH / WAVE];
  const int tid = threadIdx.x;
  const int lane = tid & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(tid / WAVE);
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int n = (int)a.g.n;
  const int nxy = nx * ny;
  const int ntiles = nyt * nzt;
  const int item = xcd_order(blockIdx.x, ntiles * a.nload);
  if (item < 0) return;
  const int l = item % a.nload;
  const int blk = item / a.nload;
  if (a.st[l].state != ST_ACTIVE) return;
  const int byi = blk % nyt, bzi = blk / nyt;
  const int y0 = byi * NW, z0 = bzi * tz;
  const int yv = y0 + w;                       // voxel row, between node rows yv and yv1
  const int yv1 = yv + 1 == ny ? 0 : yv + 1;
  const int xb = lane * V;
  const float ih[3] = {(float)(1.0 / a.g.h[0]), (float)(1.0 / a.g.h[1]), (float)(1.0 / a.g.h[2])};
  const double wd = a.g.h[0] * a.g.h[1] * a.g.h[2] / 6.0;
  const float wgt = (float)((UNI ? wd / (a.g.h[0] * a.g.h[0]) : wd) * (a.negate ? -1.0 : 1.0));
  const float* u = a.u + l * a.lstride;
  float* out = reinterpret_cast<float*>(a.out) + l * a.lstride;
  const float* matl = a.mat + (long long)(l / a.lpc) * a.mat_stride;
  float* edge = a.edge + l * a.edge_stride;
  const int ety = byi + 1 == nyt ? 0 : byi + 1;  // tile of node row y0 + NW
  const int roff[2] = {yv * nx + xb, yv1 * nx + xb};
  float* carw = car + w * (2 * 3 * V * WAVE) + lane;
  auto cidx = [](int r, int c, int j) { return ((r * 3 + c) * V + j) * WAVE; };
  // node planes in registers: u at node rows yv / yv1, x nodes xb .. xb + V
  // (the last one from the next lane); three plane sets and three material
  // sets rotate (bottom, top, prefetch) so that no step copies registers
  using Plane = float[2][3][V + 1];
  using Mat = float[2 * V];
  Plane P0, P1, P2;
  Mat M0, M1, M2;
  auto load_plane = [&](int zp, Plane& dst) {
    const int zoff = (zp < 0 ? zp + nz : (zp >= nz ? zp - nz : zp)) * nxy;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) rw_load<V>(u + c * n + zoff + roff[r], dst[r][c]);
  };
  auto load_mat = [&](int zl, Mat& dst) {
    const int zoff = (zl < 0 ? zl + nz : (zl >= nz ? zl - nz : zl)) * nxy;
    const float* m = matl + 2 * (zoff + roff[0]);
#pragma unroll
    for (int i = 0; i < 2 * V; i += (V == 1 ? 2 : 4)) {
      if constexpr (V == 1) {
        const float2 t = *reinterpret_cast<const float2*>(m);
        dst[0] = t.x;
        dst[1] = t.y;
      } else {
        const float4 t = *reinterpret_cast<const float4*>(m + i);
        dst[i] = t.x;
        dst[i + 1] = t.y;
        dst[i + 2] = t.z;
        dst[i + 3] = t.w;
      }
    }
  };
  auto complete = [&](Plane& pl) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) pl[r][c][V] = rw_rol(pl[r][c][0]);
  };
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int j = 0; j < V; ++j) carw[cidx(r, c, j)] = 0.0f;
  double acc = 0.0;
  // one layer: k between node planes k and k + 1, bottom plane ub, top
  // plane ut (loaded one step earlier, completed here), material mc;
  // prefetches plane k + 2 into un and the material of layer k + 1 into mn
  auto step = [&](int L, Plane& ub, Plane& ut, Plane& un, Mat& mc, Mat& mn) {
    const int k = z0 - 1 + L;
    complete(ut);
    if (L < tz) {
      load_plane(k + 2, un);
      load_mat(k + 1, mn);
    }
    const bool store = L >= 1 && k < nz;
    const int slot = L & 1;
    // node x column j of this lane gets corners (0, ., .) of voxel j and
    // (1, ., .) of voxel j - 1 (for j = 0: the previous lane's last voxel);
    // per column: own row plane k (P), upper row plane k (U, to the next
    // wave), and the plane-(k+1) parts (to the carries)
    float P[3][V], U[3][V];
    float h00[3], h10[3], h01[3], h11[3];  // corners (1, ., .) of the last voxel
#pragma unroll
    for (int i = 0; i < V; ++i) {
      float uu[8][3], f[8][3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        uu[0][c] = ub[0][c][i];
        uu[1][c] = ub[0][c][i + 1];
        uu[2][c] = ub[1][c][i];
        uu[3][c] = ub[1][c][i + 1];
        uu[4][c] = ut[0][c][i];
        uu[5][c] = ut[0][c][i + 1];
        uu[6][c] = ut[1][c][i];
        uu[7][c] = ut[1][c][i + 1];
      }
      voxel3<float, false, UNI>(uu, mc[2 * i] * wgt, mc[2 * i + 1] * wgt, ih, nullptr, f, nullptr);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float c0 = carw[cidx(0, c, i)], c1 = carw[cidx(1, c, i)];
        if (i > 0) {  // column i is complete
          P[c][i] = f[0][c] + h00[c] + c0;
          U[c][i] = f[2][c] + h10[c] + c1;
          carw[cidx(0, c, i)] = f[4][c] + h01[c];
          carw[cidx(1, c, i)] = f[6][c] + h11[c];
        } else {  // column 0 still lacks the previous lane's last voxel
          P[c][0] = f[0][c] + c0;
          U[c][0] = f[2][c] + c1;
          carw[cidx(0, c, 0)] = f[4][c];
          carw[cidx(1, c, 0)] = f[6][c];
        }
        // corners (1, ., .) of voxel i: column i + 1, or the next lane
        h00[c] = f[1][c];
        h10[c] = f[3][c];
        h01[c] = f[5][c];
        h11[c] = f[7][c];
      }
    }
    // column 0 of this lane: corners (1, ., .) of the previous lane's last voxel
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      P[c][0] += rw_ror(h00[c]);
      U[c][0] += rw_ror(h10[c]);
      carw[cidx(0, c, 0)] += rw_ror(h01[c]);
      carw[cidx(1, c, 0)] += rw_ror(h11[c]);
    }
    // p.q of every contribution made here, each with the p of its node
    // (own row: ub[0]; upper row: ub[1]); FP32 within the step
    float pq = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i = 0; i < V; ++i) pq += ub[0][c][i] * P[c][i] + ub[1][c][i] * U[c][i];
    if (store) acc += (double)pq;
    // upper node row, plane k: to the next wave, or (last wave) to the edge rows
    if (w < NW - 1) {
#pragma unroll
      for (int c = 0; c < 3; ++c) rw_store<V>(xch + (((slot * NW + w) * 3 + c) * WAVE + lane) * V, U[c]);
    } else if (store) {
#pragma unroll
      for (int c = 0; c < 3; ++c) rw_store<V>(edge + ((long long)(c * nz + k) * nyt + ety) * nx + xb, U[c]);
    }
    __syncthreads();
    if (store) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float lo[V];
        if (w > 0) {
          rw_load<V>(xch + (((slot * NW + w - 1) * 3 + c) * WAVE + lane) * V, lo);
        } else {
#pragma unroll
          for (int i = 0; i < V; ++i) lo[i] = 0.0f;
        }
#pragma unroll
        for (int i = 0; i < V; ++i) lo[i] += P[c][i];
        rw_store<V>(out + c * n + k * nxy + roff[0], lo);
      }
    }
  };
  load_plane(z0 - 1, P0);
  load_plane(z0, P1);
  load_mat(z0 - 1, M0);
  complete(P0);
  for (int L = 0; L <= tz; L += 3) {
    step(L, P0, P1, P2, M0, M1);
    if (L + 1 <= tz) step(L + 1, P1, P2, P0, M1, M2);
    if (L + 2 <= tz) step(L + 2, P2, P0, P1, M2, M0);
  }
  const double bs = block_sum<NTH>(acc, sh);
  if (tid == 0) a.red.put(RED_PQ, l, blk, bs);
}

// q[rows y = 0 mod rows] += edge rows, for the active slots (the row-wave
// operator's fix-up when no x forward pass follows)
__global__ __launch_bounds__(NT) void k_rw_edge_fix(float* q, const float* edge, long long lstride,
                                                    long long estride, int nx, int ny, int nz, int nyt, int rows,
                                                    const LoadState* st) {
  const int l = blockIdx.y;
  if (st[l].state != ST_ACTIVE) return;
  const long long total = 3LL * nz * nyt * nx;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < total; e += (long long)gridDim.x * NT) {
    const int x = (int)(e % nx);
    const long long r = e / nx;  // (c nz + z) nyt + t
    const int t = (int)(r % nyt);
    const long long cz = r / nyt;
    q[l * lstride + (cz * ny + (long long)t * rows) * nx + x] += edge[l * estride + e];
  }
}

// fixed-order sums of the per-block stress partials: sbar[l][i]
__global__ __launch_bounds__(NT) void k_stress_finalize(const double* sparts, int maxblk, int nparts,
                                                        int only_load, const int* mask, double* sbar) {
  __shared__ double sh[NT / WAVE];
  const int i = blockIdx.x, l = blockIdx.y;
  if (mask ? mask[l] == 0 : (only_load >= 0 && l != only_load)) return;
  const double* row = sparts + ((long long)l * 6 + i) * maxblk;
  double v = 0.0;
  for (int b = threadIdx.x; b < nparts; b += NT) v += row[b];
  const double s = block_sum<NT>(v, sh);
  if (threadIdx.x == 0) sbar[l * 6 + i] = s;
}

// ============================================== homogenisation (FP64, once)
// Total strain of every simplex: eps = eps_bar + sym(G).  Accumulates per
// block  C_IJ += |s| eps^I : sigma^J  and  sbar_J += |s| sigma^J.
template <int D>
__device__ __forceinline__ void simplex_strain(const double* ucorner /*[nc][D]*/, const int* path,
                                               const double* ih, const double* eb, double* e) {
  // path: D axes; corners along the monotone path
  double G[3][3] = {};
  int c = 0;
  for (int j = 0; j < D; ++j) {
    const int a = path[j];
    const int cn = c | (1 << a);
    for (int k = 0; k < D; ++k) G[k][a] = (ucorner[cn * D + k] - ucorner[c * D + k]) * ih[a];
    c = cn;
  }
  if (D == 3) {
    e[0] = eb[0] + G[0][0];
    e[1] = eb[1] + G[1][1];
    e[2] = eb[2] + G[2][2];
    e[3] = eb[3] + 0.5 * (G[1][2] + G[2][1]);
    e[4] = eb[4] + 0.5 * (G[0][2] + G[2][0]);
    e[5] = eb[5] + 0.5 * (G[0][1] + G[1][0]);
  } else {
    e[0] = eb[0] + G[0][0];
    e[1] = eb[1] + G[1][1];
    e[2] = 0.0;
    e[3] = 0.0;
    e[4] = 0.0;
    e[5] = eb[5] + 0.5 * (G[0][1] + G[1][0]);
  }
}

__device__ __forceinline__ void stress_from_strain(const double* e, double lam, double mu, double* s) {
  const double tr = e[0] + e[1] + e[2];
  s[0] = lam * tr + 2.0 * mu * e[0];
  s[1] = lam * tr + 2.0 * mu * e[1];
  s[2] = lam * tr + 2.0 * mu * e[2];
  s[3] = 2.0 * mu * e[3];
  s[4] = 2.0 * mu * e[4];
  s[5] = 2.0 * mu * e[5];
}

__device__ __forceinline__ double contract(const double* e, const double* s) {
  return e[0] * s[0] + e[1] * s[1] + e[2] * s[2] + 2.0 * (e[3] * s[3] + e[4] * s[4] + e[5] * s[5]);
}

__device__ __forceinline__ void gather_corners(const HArgs& a, int l, int i, int j, int k, double* uc) {
  const int D = a.g.dim;
  const int nc = D == 3 ? 8 : 4;
  const double* u = a.u + l * a.lstride;
  for (int c = 0; c < nc; ++c) {
    const int ox = c & 1, oy = (c >> 1) & 1, oz = (c >> 2) & 1;
    const long long nd = ((long long)wrapi(k + oz, a.g.nz) * a.g.ny + wrapi(j + oy, a.g.ny)) * a.g.nx +
                         wrapi(i + ox, a.g.nx);
    for (int q = 0; q < D; ++q) uc[c * D + q] = u[q * a.g.n + nd];
  }
}

// Effective stiffness without a second pass over the strains: for any
// fluctuation u^I and residual r^J = f^J - K u^J,
//   (1/|Y|) sum |s| eps^I : D eps^J = eps_bar^I . sigma_bar^J - (u^I . r^J) / |Y|,
// because sum |s| (B u^I)^T D (eps_bar^J + B u^J) = -(u^I)^T r^J.  The
// mean stresses sigma_bar come from the residual launch; this kernel forms
// the nload x nload dot products u^I . r^J (FP64 accumulation).
template <typename TR>
__global__ __launch_bounds__(NT) void k_udotr(HArgs a) {
  __shared__ double sh[NT / WAVE];
  const int nl = a.nload;
  const long long len = a.lstride;
  const int cell = blockIdx.y;
  const TR* r = reinterpret_cast<const TR*>(a.r) + (long long)cell * a.lpc * len;
  const double* u = a.u + (long long)cell * a.lpc * len;
  double* parts = a.parts + (long long)cell * nl * nl * a.nblk;
  double acc[6][6] = {};
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < len; i += (long long)gridDim.x * NT) {
    double uu[6], rr[6];
#pragma unroll
    for (int I = 0; I < 6; ++I) {
      uu[I] = I < nl ? u[I * len + i] : 0.0;
      rr[I] = I < nl ? (double)r[I * len + i] : 0.0;
    }
#pragma unroll
    for (int I = 0; I < 6; ++I)
#pragma unroll
      for (int J = 0; J < 6; ++J) acc[I][J] += uu[I] * rr[J];
  }
  for (int t = 0; t < nl * nl; ++t) {
    double v = 0.0;
#pragma unroll
    for (int I = 0; I < 6; ++I)
#pragma unroll
      for (int J = 0; J < 6; ++J)
        if (I * nl + J == t) v = acc[I][J];
    const double bs = block_sum<NT>(v, sh);
    if (threadIdx.x == 0) parts[(long long)t * a.nblk + blockIdx.x] = bs;
  }
}

// one block: C_IJ and the Voigt mean stresses from the dot products and
// the stress sums (result layout [nl*nl] C then [nl][nv] mean stress)
__global__ __launch_bounds__(NT) void k_homog_combine(HArgs a, double inv_vol) {
  __shared__ double sh[NT / WAVE];
  __shared__ double dots[36];
  const int nl = a.nload;
  const int cell = blockIdx.x;
  const double* parts = a.parts + (long long)cell * nl * nl * a.nblk;
  const double* sbar = a.sbar + (long long)cell * a.lpc * 6;
  double* result = a.result + (long long)cell * (nl * nl + nl * (a.g.dim == 3 ? 6 : 3));
  for (int t = 0; t < nl * nl; ++t) {
    double v = 0.0;
    for (int b = threadIdx.x; b < a.nblk; b += NT) v += parts[(long long)t * a.nblk + b];
    const double s = block_sum<NT>(v, sh);
    if (threadIdx.x == 0) dots[t] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int D = a.g.dim;
    const int nv = D == 3 ? 6 : 3;
    for (int I = 0; I < nl; ++I)
      for (int J = 0; J < nl; ++J) {
        const double* e = a.eps[I];
        const double* sg = sbar + 6 * J;
        const double es = e[0] * sg[0] + e[1] * sg[1] + e[2] * sg[2] + 2.0 * (e[3] * sg[3] + e[4] * sg[4] + e[5] * sg[5]);
        result[I * nl + J] = (es - dots[I * nl + J]) * inv_vol;
      }
    for (int J = 0; J < nl; ++J)
      for (int q = 0; q < nv; ++q) {
        const int src = D == 3 ? q : (q == 2 ? 5 : q);
        result[nl * nl + J * nv + q] = sbar[6 * J + src] * inv_vol;
      }
  }
}

// one block per value: fixed-order sum of the block partials
__global__ __launch_bounds__(NT) void k_sum_rows(const double* parts, int nblk, double scale, double* out) {
  __shared__ double sh[NT / WAVE];
  const double* row = parts + (long long)blockIdx.x * nblk;
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += NT) v += row[i];
  const double s = block_sum<NT>(v, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s * scale;
}

__global__ __launch_bounds__(NT) void k_grad(HArgs a) {
  const int D = a.g.dim;
  const int nl = a.nload;
  const double ih[3] = {1.0 / a.g.h[0], 1.0 / a.g.h[1], 1.0 / a.g.h[2]};
  const double w = D == 3 ? a.g.h[0] * a.g.h[1] * a.g.h[2] / 6.0 : a.g.h[0] * a.g.h[1] / 2.0;
  const double vol = a.g.h[0] * a.g.h[1] * (D == 3 ? a.g.h[2] : 1.0) * a.g.n;
  const int nsimp = D == 3 ? 6 : 2;
  const int perm2[2][2] = {{0, 1}, {1, 0}};
  for (long long v = (long long)blockIdx.x * NT + threadIdx.x; v < a.g.n; v += (long long)gridDim.x * NT) {
    const int i = (int)(v % a.g.nx);
    const int j = (int)((v / a.g.nx) % a.g.ny);
    const int k = (int)(v / ((long long)a.g.nx * a.g.ny));
    const double E = a.E[v];
    const double lam = a.mat[2 * v] / E, mu = a.mat[2 * v + 1] / E;
    double uc[6][24];
    for (int l = 0; l < nl; ++l) gather_corners(a, l, i, j, k, uc[l]);
    double g = 0.0;
    for (int p = 0; p < nsimp; ++p) {
      int path[3];
      for (int q = 0; q < D; ++q) path[q] = D == 3 ? kPerm3[p][q] : perm2[p][q];
      double e[6][6], s[6][6];
      for (int l = 0; l < nl; ++l) {
        if (D == 3) simplex_strain<3>(uc[l], path, ih, a.eps[l], e[l]);
        else simplex_strain<2>(uc[l], path, ih, a.eps[l], e[l]);
        stress_from_strain(e[l], lam, mu, s[l]);
      }
      for (int I = 0; I < nl; ++I)
        for (int J = 0; J < nl; ++J)
          if (a.a[I][J] != 0.0) g += a.a[I][J] * w * contract(e[I], s[J]);
    }
    a.grad[v] = g / vol;
  }
}

// ================================================================ launchers
struct Tile3 {
  int bx, by, tz;
};

// runtime tile (any grid): x extent the largest divisor of nx up to 64
// (fp32) / 32 (fp64, LDS budget), z extent from the schedule
static Tile3 pick_tile3(const Geom& g, bool fp64, int tz) {
  Tile3 t;
  t.bx = 1;
  for (int d = fp64 ? 32 : 64; d >= 1; --d)
    if (g.nx % d == 0) { t.bx = d; break; }
  t.by = NT / t.bx;
  if (t.by > g.ny) t.by = g.ny;
  t.tz = g.nz >= tz ? tz : g.nz;
  return t;
}

// compile-time tiles (BX x BY threads), in schedule order
// (BX + BY + 1 halo voxels are computed twice, once here and once by the
// neighbouring tile: the 512-thread tiles halve that share)
void stencil_tile_dims(bool fp64, int t, int* bx, int* by) {
  static const int f32[ST_NTILE][2] = {{64, 4}, {32, 8}, {16, 16}, {64, 8}, {32, 16}, {64, 8}};
  static const int f64[ST_NTILE][2] = {{32, 8}, {16, 16}, {64, 4}, {32, 16}, {16, 32}, {32, 8}};
  if (t < 0 || t >= ST_NTILE) t = 0;
  *bx = (fp64 ? f64 : f32)[t][0];
  *by = (fp64 ? f64 : f32)[t][1];
}

int rw_rows(int nx) { return nx == 256 ? 4 : 8; }

bool rw_fits(const Geom& g) {
  return g.dim == 3 && (g.nx == 64 || g.nx == 128 || g.nx == 256) && g.ny % rw_rows(g.nx) == 0 &&
         g.n < (1LL << 29);
}

long long rw_edge_floats(const Geom& g) { return 3LL * g.nz * (g.ny / rw_rows(g.nx)) * g.nx; }

bool stencil_tile_fits(const Geom& g, bool fp64, int t) {
  if (t == ST_RW) return !fp64 && rw_fits(g);
  int bx, by;
  stencil_tile_dims(fp64, t, &bx, &by);
  return g.dim == 3 && g.nx % bx == 0 && g.ny % by == 0 && g.n < (1LL << 29);
}

// the tile a schedule runs: its own if it fits the grid, else the first one
// that fits, else -1 (runtime tile)
static int effective_tile(const Geom& g, bool fp64, int t) {
  if (stencil_tile_fits(g, fp64, t)) return t;
  for (int u = 0; u < ST_NTILE; ++u)
    if (stencil_tile_fits(g, fp64, u)) return u;
  return -1;
}

int stencil_effective_tile(const Geom& g, bool fp64, int t) { return effective_tile(g, fp64, t); }

static int sched_tz(const Geom& g, const Sched& sc) {
  const int tz = sc.st_tz < ST_TZ_MIN ? ST_TZ_MIN : sc.st_tz;
  return g.nz >= tz ? tz : g.nz;
}

template <typename T>
static size_t stencil3_lds(const Tile3& t) {
  return sizeof(T) * (6 * (t.bx + 2) * (t.by + 2) + 18 * (t.bx + 1) * (t.by + 1));
}

int stencil_blocks(const Geom& g, const Sched& sc, bool fp64) {
  if (g.dim == 2) return (int)((g.n + NT - 1) / NT);
  const int tz = sched_tz(g, sc);
  const int nzt = (g.nz + tz - 1) / tz;
  const int t = effective_tile(g, fp64, sc.st_tile);
  if (t == ST_RW) return (g.ny / rw_rows(g.nx)) * nzt;
  if (t >= 0) {
    int bx, by;
    stencil_tile_dims(fp64, t, &bx, &by);
    return (g.nx / bx) * (g.ny / by) * nzt;
  }
  const Tile3 rt = pick_tile3(g, fp64, tz);
  return (g.nx / rt.bx) * ((g.ny + rt.by - 1) / rt.by) * nzt;
}

int max_reduction_blocks(const Geom& g) {
  int mb = 0;
  const int nrows = g.dim * g.ny * g.nz;
  for (int fp64 = 0; fp64 < 2; ++fp64) {
    for (int v = 0; v < 4; ++v) {
      Sched sc;
      sc.x_var = v & 1;
      sc.z_var = v;
      mb = std::max(mb, xpass_blocks(g.nx, nrows, fp64, sc));
      mb = std::max(mb, last_pass_blocks(g.dim, g.nx, g.ny, fp64, sc));
    }
    for (int t = 0; t < ST_NTILE; ++t)
      for (int tz = ST_TZ_MIN; tz <= 64; tz *= 2) {
        Sched sc;
        sc.st_tile = t;
        sc.st_tz = tz;
        mb = std::max(mb, stencil_blocks(g, sc, fp64));
      }
  }
  return std::max(mb, sr_max_blocks(g));
}

template <typename T, typename TO, int MODE, int BX, int BY>
static void launch_tile3(const KArgs<T>& a, int tz, int& nparts, hipStream_t s) {
  const Geom& g = a.g;
  const int nxt = g.nx / BX, nyt = g.ny / BY, nzt = (g.nz + tz - 1) / tz;
  nparts = nxt * nyt * nzt;
  dim3 grid(xcd_grid(nparts * a.nload));
  const bool uni = g.h[0] == g.h[1] && g.h[1] == g.h[2];
  if (uni)
    hipLaunchKernelGGL((k_stencil3t<T, TO, MODE, true, BX, BY>), grid, dim3(BX * BY), 0, s, a, tz, nxt, nyt, nzt);
  else
    hipLaunchKernelGGL((k_stencil3t<T, TO, MODE, false, BX, BY>), grid, dim3(BX * BY), 0, s, a, tz, nxt, nyt, nzt);
}

template <int V>
static void launch_rw_v(const KArgs<float>& a, int tz, int& nparts, hipStream_t s) {
  constexpr int NW = V == 4 ? 4 : 8;  // rw_rows(64 V)
  const Geom& g = a.g;
  const int nyt = g.ny / NW, nzt = (g.nz + tz - 1) / tz;
  nparts = nyt * nzt;
  dim3 grid(xcd_grid(nparts * a.nload));
  const bool uni = g.h[0] == g.h[1] && g.h[1] == g.h[2];
  if (uni) hipLaunchKernelGGL((k_stencil_rw<V, NW, true>), grid, dim3(NW * WAVE), 0, s, a, tz, nyt, nzt);
  else hipLaunchKernelGGL((k_stencil_rw<V, NW, false>), grid, dim3(NW * WAVE), 0, s, a, tz, nyt, nzt);
}

template <typename T, typename TO, int MODE>
static hipError_t launch_stencil_impl(const KArgs<T>& a, const Sched& sc, hipStream_t s) {
  const Geom& g = a.g;
  constexpr bool fp64 = sizeof(T) == 8;
  int nparts = 0;
  int tile = g.dim == 3 ? effective_tile(g, fp64, sc.st_tile) : -1;
  if (tile == ST_RW) {
    if constexpr (!fp64 && sizeof(TO) == 4 && MODE == 0) {
      if (a.edge) {
        const int tz = sched_tz(g, sc);
        if (g.nx == 256) launch_rw_v<4>(a, tz, nparts, s);
        else if (g.nx == 128) launch_rw_v<2>(a, tz, nparts, s);
        else launch_rw_v<1>(a, tz, nparts, s);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (nparts > a.red.maxblk) return hipErrorInvalidValue;
        if (!a.edge_fused) {
          hipLaunchKernelGGL(k_rw_edge_fix, dim3(256, a.nload), dim3(NT), 0, s, reinterpret_cast<float*>(a.out),
                             (const float*)a.edge, a.lstride, a.edge_stride, g.nx, g.ny, g.nz, g.ny / rw_rows(g.nx),
                             rw_rows(g.nx), (const LoadState*)a.st);
          e = hipGetLastError();
          if (e != hipSuccess) return e;
        }
        return launch_finalize(a.red, a.st, a.res2, RED_PQ, nparts, a.nload, a.only_load, nullptr, s);
      }
    }
    // the row-wave kernel needs FP32, mode 0 and the edge rows: a compiled tile instead
    tile = -1;
    for (int u = 0; u < ST_RW; ++u)
      if (stencil_tile_fits(g, fp64, u)) {
        tile = u;
        break;
      }
  }
  if (tile >= 0) {
    const int tz = sched_tz(g, sc);
    // tile order as in stencil_tile_dims
    if constexpr (fp64) {
      switch (tile) {
        case 0: launch_tile3<T, TO, MODE, 32, 8>(a, tz, nparts, s); break;
        case 1: launch_tile3<T, TO, MODE, 16, 16>(a, tz, nparts, s); break;
        case 2: launch_tile3<T, TO, MODE, 64, 4>(a, tz, nparts, s); break;
        case 3: launch_tile3<T, TO, MODE, 32, 16>(a, tz, nparts, s); break;
        default: launch_tile3<T, TO, MODE, 16, 32>(a, tz, nparts, s); break;
      }
    } else {
      switch (tile) {
        case 0: launch_tile3<T, TO, MODE, 64, 4>(a, tz, nparts, s); break;
        case 1: launch_tile3<T, TO, MODE, 32, 8>(a, tz, nparts, s); break;
        case 2: launch_tile3<T, TO, MODE, 16, 16>(a, tz, nparts, s); break;
        case 3: launch_tile3<T, TO, MODE, 64, 8>(a, tz, nparts, s); break;
        default: launch_tile3<T, TO, MODE, 32, 16>(a, tz, nparts, s); break;
      }
    }
  } else if (g.dim == 3) {
    const Tile3 t = pick_tile3(g, fp64, sched_tz(g, sc));
    dim3 grid(g.nx / t.bx, (g.ny + t.by - 1) / t.by, (g.nz + t.tz - 1) / t.tz);
    nparts = grid.x * grid.y * grid.z;
    const size_t lds = stencil3_lds<T>(t);
    if (3 * (t.bx + 2) * (t.by + 2) > PF_MAX * NT) return hipErrorInvalidValue;
    const bool uni = g.h[0] == g.h[1] && g.h[1] == g.h[2];
    if (uni) hipLaunchKernelGGL((k_stencil3<T, TO, MODE, true>), grid, dim3(NT), lds, s, a, t.bx, t.by, t.tz);
    else hipLaunchKernelGGL((k_stencil3<T, TO, MODE, false>), grid, dim3(NT), lds, s, a, t.bx, t.by, t.tz);
  } else {
    dim3 grid((unsigned)((g.n + NT - 1) / NT), a.nload);
    nparts = grid.x;
    hipLaunchKernelGGL((k_stencil2<T, TO, MODE>), grid, dim3(NT), 0, s, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nparts > a.red.maxblk) return hipErrorInvalidValue;
  e = launch_finalize(a.red, a.st, a.res2, MODE == 0 ? RED_PQ : RED_RES, nparts, a.nload, a.only_load,
                      MODE == 1 ? a.mask : nullptr, s);
  if (e != hipSuccess || MODE != 1 || !a.sparts) return e;
  hipLaunchKernelGGL(k_stress_finalize, dim3(6, a.nload), dim3(NT), 0, s, (const double*)a.sparts, a.red.maxblk,
                     nparts, a.only_load, a.mask, a.sbar);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stencil(const KArgs<T>& a, const Sched& sc, hipStream_t s) {
  if (a.mode == 0) return launch_stencil_impl<T, T, 0>(a, sc, s);
  return launch_stencil_impl<T, T, 1>(a, sc, s);
}

hipError_t launch_residual_mixed(const KArgs<double>& a, float* out32, const Sched& sc, hipStream_t s) {
  KArgs<double> b = a;
  b.out = out32;
  return launch_stencil_impl<double, float, 1>(b, sc, s);
}

int homog_blocks(const Geom& g) {
  long long nb = (g.n + NT - 1) / NT;
  return (int)(nb < 1024 ? nb : 1024);
}

hipError_t launch_homog(const HArgs& a, int ncell, hipStream_t s) {
  if (a.r_fp64) hipLaunchKernelGGL(k_udotr<double>, dim3(a.nblk, ncell), dim3(NT), 0, s, a);
  else hipLaunchKernelGGL(k_udotr<float>, dim3(a.nblk, ncell), dim3(NT), 0, s, a);
  const double vol = a.g.h[0] * a.g.h[1] * (a.g.dim == 3 ? a.g.h[2] : 1.0) * a.g.n;
  hipLaunchKernelGGL(k_homog_combine, dim3(ncell), dim3(NT), 0, s, a, 1.0 / vol);
  return hipGetLastError();
}

hipError_t launch_grad(const HArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_grad, dim3(a.nblk), dim3(NT), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_stencil<float>(const KArgs<float>&, const Sched&, hipStream_t);
template hipError_t launch_stencil<double>(const KArgs<double>&, const Sched&, hipStream_t);

#ifdef CELLFFT_BOUNDS_CHECK
unsigned int oob_take_stencil() { return oob_take(); }
#endif

}  // namespace cellfft
