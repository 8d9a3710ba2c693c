// Device-side building blocks shared by the cell-problem kernels (gfx950).
//
//  * cpx<T>            minimal complex type (T = float | double)
//  * block reductions  wave64 shuffle trees + fixed-order cross-wave sum, so
//                      every FP64 reduction is deterministic (no float atomics)
//  * XCD order         mapping of block ids so that the blocks of one XCD
//                      take a contiguous range of the logical work list
//  * LDS FFT engine    in-place Stockham autosort FFT over a tile of columns
//                      held in LDS, compile-time length N = 2^a 3^b, radix
//                      16/8/4/3/2 codelets in registers, twiddles from a table.
//  * checked accesses  ck_ld / ck_st: plain global loads and stores, which the
//                      bounds-checked debug build (-DCELLFFT_BOUNDS_CHECK)
//                      compares with the extent of the buffer they address
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cellfft {

// ---------------------------------------------------------------- checked accesses
// p + i must lie in [lo, hi), the part of the buffer that the access may
// touch (usually the slot's field).  In the bounds-checked build an access
// outside is not performed (a load yields zero) and is counted in this
// module's device counter (read by oob_count); in the normal build lo and hi
// are unused and the helpers are the plain accesses.
#ifdef CELLFFT_BOUNDS_CHECK
static __device__ unsigned int g_oob_count;
__device__ __forceinline__ bool ck_in(const void* a, const void* lo, const void* hi) {
  if (a >= lo && a < hi) return true;
  atomicAdd(&g_oob_count, 1u);
  return false;
}
// host: read and clear this module's counter (current device)
static inline unsigned int oob_take() {
  unsigned int v = 0, z = 0;
  if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_oob_count), sizeof(v)) != hipSuccess) return 0xffffffffu;
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_oob_count), &z, sizeof(z)) != hipSuccess) return 0xffffffffu;
  return v;
}
#endif
template <typename T>
__device__ __forceinline__ T ck_ld(const T* p, long long i, const void* lo, const void* hi) {
#ifdef CELLFFT_BOUNDS_CHECK
  if (!ck_in(p + i, lo, hi)) return T{};
#endif
  return p[i];
}
template <typename T>
__device__ __forceinline__ void ck_st(T* p, long long i, const void* lo, const void* hi, const T& v) {
#ifdef CELLFFT_BOUNDS_CHECK
  if (!ck_in(p + i, lo, hi)) return;
#endif
  p[i] = v;
}
// the kernels' form: in the normal build the plain expression, lo and hi
// unevaluated (the extents are computed only in the checked build)
#ifdef CELLFFT_BOUNDS_CHECK
#define CK_LD(p, i, lo, hi) ck_ld(p, i, lo, hi)
#define CK_ST(p, i, lo, hi, v) ck_st(p, i, lo, hi, v)
#else
#define CK_LD(p, i, lo, hi) ((p)[i])
#define CK_ST(p, i, lo, hi, v) ((p)[i] = (v))
#endif

// ---------------------------------------------------------------- complex
template <typename T> struct cpx { T re, im; };

template <typename T> __device__ __forceinline__ cpx<T> mk(T a, T b) { return cpx<T>{a, b}; }
template <typename T> __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cpx<T> operator*(cpx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T> __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cpx<T> conj(cpx<T> a) { return {a.re, -a.im}; }
// multiply by -i (forward sign) or +i (inverse sign)
template <typename T, bool INV> __device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) {
  if (INV) return {-a.im, a.re};   // +i * a
  return {a.im, -a.re};            // -i * a
}

// ---------------------------------------------------------------- reductions
constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Sum over the block; the result is valid in thread 0.  sh must hold NT/64
// doubles.  Order is fixed by the lane/wave structure (deterministic).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  v = wave_sum(v);
  if ((tid & (WAVE - 1)) == 0) sh[tid / WAVE] = v;
  __syncthreads();
  double s = 0.0;
  if (tid == 0) {
#pragma unroll
    for (int w = 0; w < NT / WAVE; ++w) s += sh[w];
  }
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------- XCD order
// Workgroups of a launch are dealt round-robin to the 8 XCDs (each with its
// own L2).  xcd_order maps the hardware block id so that every XCD receives
// a contiguous range of the logical work list: consecutive logical items
// (tiles that share cache lines, or the load cases of one tile that share
// the material) then run back to back on the same L2.  Launch 8 * chunk
// blocks, chunk = ceil(total / 8); returns -1 for padding blocks.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_order(int b, int total) {
  const int chunk = (total + NXCD - 1) / NXCD;
  const int logical = (b % NXCD) * chunk + b / NXCD;
  return logical < total ? logical : -1;
}
inline int xcd_grid(int total) { return NXCD * ((total + NXCD - 1) / NXCD); }

// ---------------------------------------------------------------- FFT codelets
template <typename T, int R, bool INV> struct Dft;

template <typename T, bool INV> struct Dft<T, 2, INV> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    cpx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <typename T, bool INV> struct Dft<T, 3, INV> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    const T h = T(0.86602540378443864676);  // sqrt(3)/2
    cpx<T> t = v[1] + v[2];
    cpx<T> m = v[0] - t * T(0.5);
    cpx<T> d = (v[1] - v[2]) * h;
    v[0] = v[0] + t;
    cpx<T> id = mul_mi<T, INV>(d);  // -i d (fwd) / +i d (inv)
    v[1] = m + id;
    v[2] = m - id;
  }
};

template <typename T, bool INV> struct Dft<T, 4, INV> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    cpx<T> t0 = v[0] + v[2], t1 = v[0] - v[2];
    cpx<T> t2 = v[1] + v[3], t3 = mul_mi<T, INV>(v[1] - v[3]);
    v[0] = t0 + t2;
    v[2] = t0 - t2;
    v[1] = t1 + t3;
    v[3] = t1 - t3;
  }
};

template <typename T, bool INV> struct Dft<T, 8, INV> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    const T r = T(0.70710678118654752440);
    cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<T, 4, INV>::run(e);
    Dft<T, 4, INV>::run(o);
    // o[k] *= W8^k, W8 = exp(-+ 2 pi i / 8)
    cpx<T> o1 = o[1], o3 = o[3];
    if (!INV) {
      o[1] = mk<T>((o1.re + o1.im) * r, (o1.im - o1.re) * r);
      o[3] = mk<T>((o3.im - o3.re) * r, -(o3.re + o3.im) * r);
    } else {
      o[1] = mk<T>((o1.re - o1.im) * r, (o1.im + o1.re) * r);
      o[3] = mk<T>(-(o3.re + o3.im) * r, (o3.re - o3.im) * r);
    }
    o[2] = mul_mi<T, INV>(o[2]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = e[k] + o[k];
      v[k + 4] = e[k] - o[k];
    }
  }
};

// 16-point DFT as 4 x 4: four 4-point DFTs over n1 (n = 4 n1 + n2), the
// twiddles W16^(n2 k1), four 4-point DFTs over n2; output k = k1 + 4 k2.
// W16^m = exp(-+ 2 pi i m / 16) with the sign of the transform.
template <typename T, bool INV> struct Dft<T, 16, INV> {
  static __device__ __forceinline__ cpx<T> tw(cpx<T> a, T c, T s) {
    // a * (c - i s) forward, a * (c + i s) inverse
    return INV ? mk<T>(a.re * c - a.im * s, a.im * c + a.re * s) : mk<T>(a.re * c + a.im * s, a.im * c - a.re * s);
  }
  static __device__ __forceinline__ void run(cpx<T>* v) {
    const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);  // cos, sin of pi/8
    const T r = T(0.70710678118654752440);
    cpx<T> a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      cpx<T> t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
      Dft<T, 4, INV>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) a[n2][k1] = t[k1];
    }
    a[1][1] = tw(a[1][1], c1, s1);   // W^1
    a[1][2] = tw(a[1][2], r, r);     // W^2
    a[1][3] = tw(a[1][3], s1, c1);   // W^3
    a[2][1] = tw(a[2][1], r, r);     // W^2
    a[2][2] = mul_mi<T, INV>(a[2][2]);  // W^4
    a[2][3] = tw(a[2][3], -r, r);    // W^6
    a[3][1] = tw(a[3][1], s1, c1);   // W^3
    a[3][2] = tw(a[3][2], -r, r);    // W^6
    a[3][3] = tw(a[3][3], -c1, -s1);  // W^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cpx<T> t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      Dft<T, 4, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
  }
};

// radix schedules: RP = 0: 8 first (except 16 = 4*4), then 4, 2, 3;
// RP = 1: 16 first, then as RP = 0 (fewer, larger stages)
__host__ __device__ constexpr int pick_radix(int n, int rp = 0) {
  return (rp == 1 && n % 16 == 0) ? 16
                                  : ((n % 8 == 0 && n != 16) ? 8 : (n % 4 == 0) ? 4 : (n % 2 == 0) ? 2 : (n % 3 == 0) ? 3 : n);
}

// Tile layouts.  ColMajorTile: element (n, c) at n*CS + c (columns fastest,
// used for pencils gathered from strided global memory).  RowTile: element
// (n, c) at c*RS + n (rows of contiguous data, used by the x passes).
template <int CS> struct ColTile {
  static __device__ __forceinline__ int at(int n, int c) { return n * CS + c; }
  static constexpr bool col_fast = true;
};
template <int RS> struct RowTile {
  static __device__ __forceinline__ int at(int n, int c) { return c * RS + n; }
  static constexpr bool col_fast = false;
};
// RowTile with one padding element after every 8: the radix-8 Stockham
// writes (stride 8 complex values) then fall on distinct LDS banks.
// Rows need RS >= N + N/8.
__host__ __device__ constexpr int pad8(int n) { return n + (n >> 3); }
template <int RS> struct RowTileP {
  static __device__ __forceinline__ int at(int n, int c) { return c * RS + pad8(n); }
  static constexpr bool col_fast = false;
};

// One Stockham stage (radix R, span NS) over NCOL columns of length N.
// tw[m * TWS] = exp(-2 pi i m / N) for m in [0, N).
template <typename T, int N, int R, int NS, bool INV, int NCOL, int NT, int TWS, class L>
__device__ __forceinline__ void fft_stage(cpx<T>* buf, const cpx<T>* __restrict__ tw) {
  constexpr int NB = N / R;
  constexpr int TOT = NB * NCOL;
  constexpr int PER = (TOT + NT - 1) / NT;
  const int tid = threadIdx.x;
  cpx<T> v[PER][R];
  int dst[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * NT;
    if ((TOT % NT == 0) || b < TOT) {
      int j, col;
      if (L::col_fast) { col = b % NCOL; j = b / NCOL; }
      else { j = b % NB; col = b / NB; }
      const int k = j % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[L::at(j + r * NB, col)];
      if (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> w = tw[(r * k * (N / (NS * R))) * TWS];
          if (INV) w.im = -w.im;
          v[q][r] = cmul(v[q][r], w);
        }
      }
      Dft<T, R, INV>::run(v[q]);
      dst[q] = ((j / NS) * NS * R + k) | (col << 20);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * NT;
    if ((TOT % NT == 0) || b < TOT) {
      const int idx = dst[q] & 0xFFFFF, col = dst[q] >> 20;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[L::at(idx + r * NS, col)] = v[q][r];
    }
  }
  __syncthreads();
}

template <typename T, int N, int REM, int NS, bool INV, int NCOL, int NT, int TWS, class L, int RP>
__device__ __forceinline__ void fft_stages(cpx<T>* buf, const cpx<T>* __restrict__ tw) {
  if constexpr (REM > 1) {
    constexpr int R = pick_radix(REM, RP);
    static_assert(REM % R == 0, "length must be 2^a 3^b");
    fft_stage<T, N, R, NS, INV, NCOL, NT, TWS, L>(buf, tw);
    fft_stages<T, N, REM / R, NS * R, INV, NCOL, NT, TWS, L, RP>(buf, tw);
  }
}

// In-place FFT (unnormalised; INV uses the +i sign) of NCOL columns of length
// N held in LDS, radix schedule RP.  Must be called by all NT threads; ends
// with a barrier.
template <typename T, int N, bool INV, int NCOL, int NT, int TWS, class L, int RP = 0>
__device__ __forceinline__ void fft_lds(cpx<T>* buf, const cpx<T>* __restrict__ tw) {
  fft_stages<T, N, N, 1, INV, NCOL, NT, TWS, L, RP>(buf, tw);
}

}  // namespace cellfft
