// FFT passes of the preconditioned CG iteration (gfx950).
//
// Spectrum layout ("packed half spectrum"): every x-row of nx reals becomes
// nx/2 complex slots; slot 0 holds X[0] + i X[nx/2] (both real), slots
// 1..nx/2-1 hold X[k].  After the y pass, column slot 0 is unmixed per
// z-plane: rows 1..ny/2-1 hold the spectrum of the X[0] field (wavevector
// (0, ky)), rows ny/2+1..ny-1 the spectrum of the X[nx/2] field
// (wavevector (nx/2, ky)), row 0 holds the two real ky = 0, ny/2 values of
// the X[0] field and row ny/2 those of the X[nx/2] field ("real pairs").
// The last pass (z in 3D, y in 2D) separates each real pair with the
// mirrored frequency of the same pencil.  The spectrum therefore has
// exactly the size of a real field and every pencil is self-contained.
//
// Kernels (all unnormalised DFTs; 1/n is folded into the preconditioner):
//   k_xfwd   r -= alpha q, ||r||^2 partials, real-to-complex FFT along x
//   k_ypass  complex FFT along y (+ slot-0 unmix / remix)
//   k_zpass  FFT along z, z_hat = K_ref^{-1} r_hat / n, r.z partials
//            (Parseval), inverse FFT along z          [3D]
//   k_ylast  same with y as the last axis               [2D]
//   k_xinv   complex-to-real FFT along x, x += alpha p, p = z + beta p
#include "kernels.h"

namespace cellfft {

// ------------------------------------------------------------------ helpers
template <typename T> struct V2;
template <> struct V2<float> { using type = float2; };
template <> struct V2<double> { using type = double2; };

template <typename T> __device__ __forceinline__ bool finite_pos(T v) { return v > T(0) && v < T(1e300); }

__device__ __forceinline__ bool load_live(const LoadState* st, bool allow_converged) {
  const int s = st->state;
  return s == ST_ACTIVE || (allow_converged && s == ST_CONVERGED);
}

// rows per block of the x passes: about 2048 (fp32) / 1024 (fp64) complex
// values, halved by schedule variant V = 1
template <typename T, int M, int V> constexpr int x_rpb() {
  constexpr int tgt = (sizeof(T) == 4 ? 2048 : 1024) >> V;
  return (tgt / M) < 1 ? 1 : (tgt / M);
}
// columns per block of the y pass and of the last pass (variant V halves them)
template <typename T, int V> constexpr int y_tx() { return (sizeof(T) == 4 ? 16 : 8) >> V; }
template <typename T, int V> constexpr int z_tx() { return (sizeof(T) == 4 ? 8 : 4) >> V; }
// threads per block of the y and last passes (more waves per CU to hide
// the load -> FFT -> store latency of each tile)
constexpr int NTY = 512;
constexpr int NTZ = 512;

// ================================================================= x forward
// MODE 0 (iteration): R -= alpha FFT_x(q) with the ||r||^2 partials from R
// by Parseval along x (packed slot 0 holds the two real values X[0] and
// X[nx/2], weight 1; slots k >= 1 stand for k and nx - k, weight 2).
// MODE 1 (after a residual recomputation): R = FFT_x(r).
template <typename T, int M, int V, int RP, int MODE>
__global__ __launch_bounds__(NT) void k_xfwd(XArgs<T> a) {
  constexpr int RPB = x_rpb<T, M, V>();
  constexpr int RS = pad8(M) + 1;  // padded rows (RowTileP)
  constexpr int QX = (RPB * M + NT - 1) / NT;
  using T2 = typename V2<T>::type;
  __shared__ cpx<T> buf[RPB * RS];
  __shared__ cpx<T> tws[2 * M];
  __shared__ double sh[NT / WAVE];
  const int l = blockIdx.y;
  LoadState* st = a.st + l;
  if (MODE == 0) {
    if (!load_live(st, false)) return;
  } else {
    if (a.mask ? a.mask[l] == 0 : !load_live(st, true)) return;
  }
  const T alpha = MODE == 0 ? (T)st->alpha : T(0);
  const int tid = threadIdx.x;
  for (int i = tid; i < 2 * M; i += NT) tws[i] = a.tw[i];
  // XCD order: consecutive row groups (contiguous memory) on one XCD
  const int rb = xcd_order(blockIdx.x, (a.nrows + RPB - 1) / RPB);
  if (rb < 0) return;
  const int row0 = rb * RPB;
  const T2* in2 = reinterpret_cast<const T2*>((MODE == 0 ? a.q : a.r) + l * a.lstride);
  cpx<T>* R = a.R + l * (a.lstride / 2);
#ifdef CELLFFT_BOUNDS_CHECK
  // extents of the slot's fields
  const T2* in2_hi = in2 + a.lstride / 2;
  const cpx<T>* R_hi = R + a.lstride / 2;
#endif
  // row-wave operator: q's rows y = 0 mod edge_rows still lack the edge rows
  const T2* edge2 = (MODE == 0 && a.edge) ? reinterpret_cast<const T2*>(a.edge + l * a.edge_stride) : nullptr;
#ifdef CELLFFT_BOUNDS_CHECK
  const T2* edge2_hi = edge2 ? edge2 + a.edge_stride / 2 : nullptr;
#endif
  const int erows = a.edge_rows > 0 ? a.edge_rows : 1;  // a power of two
  const int eshift = __builtin_ctz(erows);
  const int nyt = a.ny >> eshift;
  // blocks inside one (component, z) plane (the usual case): y and the plane
  // index without a division per element
  const bool inplane = (a.ny % RPB) == 0;
  const int yb = row0 % a.ny, pb = row0 / a.ny;
  cpx<T> rv[QX];  // mode 0: this thread's R values, loaded with q
  {
    // every load first, then the LDS stores (a loop that stores each value
    // as it arrives waits out one memory latency per element)
    cpx<T> v[QX];
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int e = tid + q * NT;
      const int rr = e / M, m = e - rr * M;
      const int row = row0 + rr;
      v[q] = {T(0), T(0)};
      if (e < RPB * M && row < a.nrows) {
        const long long off = (long long)row * M + m;
        const T2 w = CK_LD(in2, off, in2, in2_hi);
        v[q] = {w.x, w.y};
        if (MODE == 0) rv[q] = CK_LD(R, off, R, R_hi);
        if (MODE == 0 && edge2) {
          // row = (c nz + z) ny + y
          const int y = inplane ? yb + rr : row % a.ny;
          if ((y & (erows - 1)) == 0) {
            const int pl = inplane ? pb : row / a.ny;
            const T2 ed = CK_LD(edge2, ((long long)pl * nyt + (y >> eshift)) * M + m, edge2, edge2_hi);
            v[q].re += ed.x;
            v[q].im += ed.y;
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int e = tid + q * NT;
      const int rr = e / M, m = e - rr * M;
      if (e < RPB * M) buf[rr * RS + pad8(m)] = v[q];
    }
  }
  __syncthreads();
  fft_lds<T, M, false, RPB, NT, 2, RowTileP<RS>, RP>(buf, tws);
  // split the half-length transform into the packed real spectrum
  constexpr int KH = M / 2 + 1;
  for (int e = tid; e < RPB * KH; e += NT) {
    const int rr = e / KH, k = e - rr * KH;
    cpx<T>* Z = buf + rr * RS;
    if (k == 0) {
      const cpx<T> z0 = Z[0];
      T dc = z0.re + z0.im;
      if (MODE == 0 && a.qmean) {
        // projected operator: q's per-component mean leaves the DC term only
        const int row = row0 + rr;
        if (row < a.nrows) dc -= (T)(2.0 * M * a.qmean[l * 3 + row / a.comp_rows]);
      }
      Z[0] = {dc, z0.re - z0.im};
    } else {
      const cpx<T> zk = Z[pad8(k)], zm = Z[pad8(M - k)];
      const cpx<T> E = (zk + conj(zm)) * T(0.5);
      const cpx<T> D = (zk - conj(zm)) * T(0.5);
      const cpx<T> O = {D.im, -D.re};  // D / i
      const cpx<T> WO = cmul(tws[k], O);
      Z[pad8(k)] = E + WO;
      if (M - k != k) Z[pad8(M - k)] = conj(E - WO);
    }
  }
  __syncthreads();
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < QX; ++q) {
    const int e = tid + q * NT;
    if (e >= RPB * M) break;
    const int rr = e / M, m = e - rr * M;
    const int row = row0 + rr;
    if (row < a.nrows) {
      const long long off = (long long)row * M + m;
      const cpx<T> h = buf[rr * RS + pad8(m)];
      if (MODE == 0) {
        cpx<T> v = rv[q];
        v.re -= alpha * h.re;
        v.im -= alpha * h.im;
        CK_ST(R, off, R, R_hi, v);
        acc += (m == 0 ? 1.0 : 2.0) * ((double)v.re * v.re + (double)v.im * v.im);
      } else {
        CK_ST(R, off, R, R_hi, h);
      }
    }
  }
  if (MODE == 0) {
    // ||r||^2 partial of this block (finalised by k_finalize)
    const double bs = block_sum<NT>(acc * (1.0 / (2.0 * M)), sh);
    if (tid == 0) a.red.put(RED_RR, l, rb, bs);
  }
}

// ================================================================= x inverse
template <typename T, int M, int V, int RP>
__global__ __launch_bounds__(NT) void k_xinv(XArgs<T> a) {
  constexpr int RPB = x_rpb<T, M, V>();
  constexpr int RS = pad8(M) + 1;  // padded rows (RowTileP)
  using T2 = typename V2<T>::type;
  __shared__ cpx<T> buf[RPB * RS];
  __shared__ cpx<T> tws[2 * M];
  const int l = blockIdx.y;
  LoadState* st = a.st + l;
  if (!load_live(st, true)) return;
  const T alpha = (T)st->alpha;
  const T beta = (T)st->beta;
  const int tid = threadIdx.x;
  for (int i = tid; i < 2 * M; i += NT) tws[i] = a.tw[i];
  // XCD order: consecutive row groups (contiguous memory) on one XCD
  const int rb = xcd_order(blockIdx.x, (a.nrows + RPB - 1) / RPB);
  if (rb < 0) return;
  const int row0 = rb * RPB;
  const cpx<T>* S = a.S + l * a.lsS;
#ifdef CELLFFT_BOUNDS_CHECK
  const cpx<T>* S_hi = S + a.lsS;  // the slot's spectrum
#endif
  // S rows live in padded (component, z) planes of zsS complex values
  const int zr0 = row0 / a.ny, yb = row0 - zr0 * a.ny;
  {
    // every load first, then the LDS stores (see the forward pass)
    constexpr int QX = (RPB * M + NT - 1) / NT;
    cpx<T> v[QX];
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int e = tid + q * NT;
      const int rr = e / M, m = e - rr * M;
      const int row = row0 + rr;
      int y = yb + rr, zr = zr0;
      if (RPB <= a.ny) {
        if (y >= a.ny) {
          y -= a.ny;
          ++zr;
        }
      } else {
        zr += y / a.ny;
        y -= (y / a.ny) * a.ny;
      }
      v[q] = (e < RPB * M && row < a.nrows) ? CK_LD(S, (long long)zr * a.zsS + (long long)y * M + m, S, S_hi)
                                            : cpx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int e = tid + q * NT;
      const int rr = e / M, m = e - rr * M;
      if (e < RPB * M) buf[rr * RS + pad8(m)] = v[q];
    }
  }
  __syncthreads();
  constexpr int KH = M / 2 + 1;
  for (int e = tid; e < RPB * KH; e += NT) {
    const int rr = e / KH, k = e - rr * KH;
    cpx<T>* X = buf + rr * RS;
    if (k == 0) {
      const cpx<T> x0 = X[0];
      X[0] = {x0.re + x0.im, x0.re - x0.im};
    } else {
      const cpx<T> xk = X[pad8(k)], xm = X[pad8(M - k)];
      const cpx<T> E = xk + conj(xm);
      const cpx<T> O = cmul(xk - conj(xm), conj(tws[k]));
      X[pad8(k)] = {E.re - O.im, E.im + O.re};  // E + i O
      if (M - k != k) X[pad8(M - k)] = {E.re + O.im, -E.im + O.re};  // conj(E) + i conj(O)
    }
  }
  __syncthreads();
  fft_lds<T, M, true, RPB, NT, 2, RowTileP<RS>, RP>(buf, tws);
  T2* x2 = reinterpret_cast<T2*>(a.x + l * a.lstride);
  T2* p2 = reinterpret_cast<T2*>(a.p + l * a.lstride);
#ifdef CELLFFT_BOUNDS_CHECK
  const T2* x2_hi = x2 + a.lstride / 2;
  const T2* p2_hi = p2 + a.lstride / 2;
#endif
  // x += alpha p, p = z + beta p: all of a thread's p and x loads first
  constexpr int QO = (RPB * M + NT - 1) / NT;
  T2 po[QO], xv[QO];
#pragma unroll
  for (int q = 0; q < QO; ++q) {
    const int e = tid + q * NT;
    const int rr = e / M, m = e - rr * M;
    const int row = row0 + rr;
    if (e < RPB * M && row < a.nrows) {
      const long long off = (long long)row * M + m;
      po[q] = CK_LD(p2, off, p2, p2_hi);
      xv[q] = CK_LD(x2, off, x2, x2_hi);
    }
  }
#pragma unroll
  for (int q = 0; q < QO; ++q) {
    const int e = tid + q * NT;
    const int rr = e / M, m = e - rr * M;
    const int row = row0 + rr;
    if (e < RPB * M && row < a.nrows) {
      const long long off = (long long)row * M + m;
      const cpx<T> z = buf[rr * RS + pad8(m)];
      T2 xn = xv[q];
      xn.x += alpha * po[q].x;
      xn.y += alpha * po[q].y;
      CK_ST(x2, off, x2, x2_hi, xn);
      T2 pn;
      pn.x = z.re + beta * po[q].x;
      pn.y = z.im + beta * po[q].y;
      CK_ST(p2, off, p2, p2_hi, pn);
    }
  }
}

// ================================================================= y pass 3D
template <typename T, int N, bool INV, int V, int RP>
__global__ __launch_bounds__(NTY) void k_ypass(YArgs<T> a) {
  constexpr int TX = y_tx<T, V>();
  __shared__ cpx<T> buf[N * TX];
  __shared__ cpx<T> tws[N];
  const int l = blockIdx.y;
  if (!load_live(a.st + l, true)) return;
  const int M = a.nx / 2;
  const int ntile = (M + TX - 1) / TX;
  // XCD order: the slot tiles of one (component, z) plane, which share
  // DRAM pages, run back to back on one XCD
  int b = xcd_order(blockIdx.x, ntile * a.nz * a.ncomp);
  if (b < 0) return;
  const int tile = b % ntile;
  b /= ntile;
  const int z = b % a.nz;
  const int c = b / a.nz;
  const int s0 = tile * TX;
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NTY) tws[i] = a.tw[i];
  cpx<T>* base = a.S + l * a.lsS + (long long)(c * a.nz + z) * a.zsS + s0;
  const cpx<T>* src = (!INV && a.Sin) ? a.Sin + l * a.lstrideC + ((long long)(c * a.nz + z) * a.ny) * M + s0 : base;
#ifdef CELLFFT_BOUNDS_CHECK
  // the slot's spectrum and input
  const cpx<T>* S_lo = a.S + l * a.lsS;
  const cpx<T>* S_hi = S_lo + a.lsS;
  const cpx<T>* src_lo = (!INV && a.Sin) ? a.Sin + l * a.lstrideC : S_lo;
  const cpx<T>* src_hi = (!INV && a.Sin) ? src_lo + a.lstrideC : S_hi;
#endif
  // all of a thread's loads before the first LDS store (see the z pass)
  {
    constexpr int PER = (N * TX + NTY - 1) / NTY;
    cpx<T> v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + q * NTY;
      const int y = e / TX, s = e - y * TX;
      v[q] = (e < N * TX && s0 + s < M) ? CK_LD(src, (long long)y * M + s, src_lo, src_hi) : cpx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + q * NTY;
      if (e < N * TX) buf[e] = v[q];
    }
  }
  __syncthreads();
  if (INV && s0 == 0) {
    // remix column 0: c(k) = A(k) + i B(k)
    cpx<T> v[(N + NTY - 1) / NTY];
#pragma unroll
    for (int q = 0; q < (N + NTY - 1) / NTY; ++q) {
      const int k = tid + q * NTY;
      if (k < N) {
        const cpx<T> rk = buf[k * TX], rm = buf[((N - k) % N) * TX];
        if (k == 0) v[q] = {rk.re, buf[(N / 2) * TX].re};
        else if (k == N / 2) v[q] = {buf[0].im, rk.im};
        else if (k < N / 2) v[q] = {rk.re + rm.im, rk.im + rm.re};       // r_k + i conj(r_{N-k})
        else v[q] = {rm.re - rk.im, -rm.im + rk.re};                     // conj(r_{N-k}) + i r_k
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (N + NTY - 1) / NTY; ++q) {
      const int k = tid + q * NTY;
      if (k < N) buf[k * TX] = v[q];
    }
    __syncthreads();
  }
  fft_lds<T, N, INV, TX, NTY, 1, ColTile<TX>, RP>(buf, tws);
  if (!INV && s0 == 0) {
    // unmix column 0 into the X[0] field (rows < N/2) and X[nx/2] field
    cpx<T> v[(N + NTY - 1) / NTY];
#pragma unroll
    for (int q = 0; q < (N + NTY - 1) / NTY; ++q) {
      const int k = tid + q * NTY;
      if (k < N) {
        const cpx<T> ck = buf[k * TX], cm = buf[((N - k) % N) * TX];
        if (k == 0) v[q] = {ck.re, buf[(N / 2) * TX].re};
        else if (k == N / 2) v[q] = {buf[0].im, ck.im};
        else if (k < N / 2) v[q] = {(ck.re + cm.re) * T(0.5), (ck.im - cm.im) * T(0.5)};  // (c_k + conj c_-k)/2
        else v[q] = {(ck.im + cm.im) * T(0.5), (cm.re - ck.re) * T(0.5)};              // (c_k - conj c_-k)/(2i)
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (N + NTY - 1) / NTY; ++q) {
      const int k = tid + q * NTY;
      if (k < N) buf[k * TX] = v[q];
    }
    __syncthreads();
  }
  for (int e = tid; e < N * TX; e += NTY) {
    const int y = e / TX, s = e - y * TX;
    if (s0 + s < M) CK_ST(base, (long long)y * M + s, S_lo, S_hi, buf[e]);
  }
}

// ===================================================== reference symbol
// Fourier symbol of the homogeneous reference operator on the Kuhn mesh
// (real symmetric), theta_a = pi k_a / N_a, sigma_a = 2 sin(theta_a) / h_a:
//   K_cc = d! w [lam sigma_c^2 + mu (|sigma|^2 + sigma_c^2)]
//   K_cd = 2 w (lam + mu) sigma_c sigma_d [2 cos(th_c + th_d) + cos(th_c + th_d + 2 th_e)]  (3D)
//   K_01 = 2 w (lam + mu) sigma_0 sigma_1 cos(th_0 + th_1)                                   (2D)
// Applies z = K^{-1} r * inv_n to a complex 3-vector (2-vector).
// Inverse of the symbol times inv_n, as (00, 11, 22, 01, 02, 12).
template <typename T>
__device__ __forceinline__ void sym_inv3(const PArgs<T>& P, int kx, int ky, int kz, T* m) {
  const T sx = P.trig[0][2 * kx], cx = P.trig[0][2 * kx + 1];
  const T sy = P.trig[1][2 * ky], cy = P.trig[1][2 * ky + 1];
  const T sz = P.trig[2][2 * kz], cz = P.trig[2][2 * kz + 1];
  const T gx = T(2) * sx * P.ih[0], gy = T(2) * sy * P.ih[1], gz = T(2) * sz * P.ih[2];
  const T gx2 = gx * gx, gy2 = gy * gy, gz2 = gz * gz;
  const T ss = gx2 + gy2 + gz2;
  const T c6 = T(6) * P.w;
  const T lam = P.lam0, mu = P.mu0;
  const T a00 = c6 * (lam * gx2 + mu * (ss + gx2));
  const T a11 = c6 * (lam * gy2 + mu * (ss + gy2));
  const T a22 = c6 * (lam * gz2 + mu * (ss + gz2));
  const T co = T(2) * P.w * (lam + mu);
  // pair (c, d) with third axis e: cos(tc + td) and cos(tc + td + 2 te)
  auto off = [&](T sc, T cc, T sd, T cd, T se, T ce, T gc, T gd) {
    const T c2 = cc * cd - sc * sd;
    const T s2 = sc * cd + cc * sd;
    const T c2e = T(1) - T(2) * se * se;
    const T s2e = T(2) * se * ce;
    return co * gc * gd * (T(2) * c2 + (c2 * c2e - s2 * s2e));
  };
  const T a01 = off(sx, cx, sy, cy, sz, cz, gx, gy);
  const T a02 = off(sx, cx, sz, cz, sy, cy, gx, gz);
  const T a12 = off(sy, cy, sz, cz, sx, cx, gy, gz);
  const T b00 = a11 * a22 - a12 * a12;
  const T b11 = a00 * a22 - a02 * a02;
  const T b22 = a00 * a11 - a01 * a01;
  const T b01 = a02 * a12 - a01 * a22;
  const T b02 = a01 * a12 - a11 * a02;
  const T b12 = a01 * a02 - a00 * a12;
  const T det = a00 * b00 + a01 * b01 + a02 * b02;
  const T s = P.inv_n / det;
  m[0] = b00 * s;
  m[1] = b11 * s;
  m[2] = b22 * s;
  m[3] = b01 * s;
  m[4] = b02 * s;
  m[5] = b12 * s;
}

template <typename T>
__device__ __forceinline__ void sym_apply3(const T* m, const cpx<T>* r, cpx<T>* z) {
  z[0] = r[0] * m[0] + r[1] * m[3] + r[2] * m[4];
  z[1] = r[0] * m[3] + r[1] * m[1] + r[2] * m[5];
  z[2] = r[0] * m[4] + r[1] * m[5] + r[2] * m[2];
}

template <typename T>
__device__ __forceinline__ void sym_solve3(const PArgs<T>& P, int kx, int ky, int kz,
                                           const cpx<T>* r, cpx<T>* z) {
  T m[6];
  sym_inv3(P, kx, ky, kz, m);
  sym_apply3(m, r, z);
}

// tabulated inverse (6 consecutive values)
template <typename T, typename I>
__device__ __forceinline__ void sym_load(const T* tab, I idx, T* m) {
  using T2 = typename V2<T>::type;
  const T2* t2 = reinterpret_cast<const T2*>(tab + 6 * idx);
  const T2 a = t2[0], b = t2[1], c = t2[2];
  m[0] = a.x;
  m[1] = a.y;
  m[2] = b.x;
  m[3] = b.y;
  m[4] = c.x;
  m[5] = c.y;
}

// Table of K_ref^{-1}/n in the stored spectrum order: entry (y, kz, slot)
// holds the wavevector the z pass meets there (slot 0: the X[0] family for
// y < ny/2, the X[nx/2] family for y > ny/2 and the first family of the two
// real-pair rows); tabB holds the second family of the real-pair rows.
// The zero frequency entry is 0.
template <typename T>
__global__ __launch_bounds__(NT) void k_symtab(PArgs<T> a, T* tab, T* tabB) {
  const int M = a.nx / 2;
  const long long total = (long long)a.ny * a.nz * M;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < total + 2LL * a.nz;
       i += (long long)gridDim.x * NT) {
    T m[6];
    if (i < total) {
      const int slot = (int)(i % M);
      const int kz = (int)((i / M) % a.nz);
      const int y = (int)(i / ((long long)M * a.nz));
      int kx = slot, ky = y;
      if (slot == 0) kx = (y <= a.ny / 2) ? (y == a.ny / 2 ? M : 0) : M;
      if (slot == 0 && (y == 0 || y == a.ny / 2)) ky = 0;
      if (slot == 0 && y == 0 && kz == 0) {
        for (int q = 0; q < 6; ++q) m[q] = T(0);
      } else {
        sym_inv3(a, kx, ky, kz, m);
      }
      for (int q = 0; q < 6; ++q) tab[6 * i + q] = m[q];
    } else {
      const long long j = i - total;
      const int r = (int)(j / a.nz), kz = (int)(j % a.nz);
      sym_inv3(a, r == 0 ? 0 : M, a.ny / 2, kz, m);
      for (int q = 0; q < 6; ++q) tabB[6 * j + q] = m[q];
    }
  }
}

template <typename T>
__device__ __forceinline__ void sym_solve2(const PArgs<T>& P, T lam0, T mu0, int kx, int ky,
                                           const cpx<T>* r, cpx<T>* z) {
  const T sx = P.trig[0][2 * kx], cx = P.trig[0][2 * kx + 1];
  const T sy = P.trig[1][2 * ky], cy = P.trig[1][2 * ky + 1];
  const T gx = T(2) * sx * P.ih[0], gy = T(2) * sy * P.ih[1];
  const T gx2 = gx * gx, gy2 = gy * gy, ss = gx2 + gy2;
  const T c2w = T(2) * P.w;
  const T a00 = c2w * (lam0 * gx2 + mu0 * (ss + gx2));
  const T a11 = c2w * (lam0 * gy2 + mu0 * (ss + gy2));
  const T a01 = c2w * (lam0 + mu0) * gx * gy * (cx * cy - sx * sy);
  const T det = a00 * a11 - a01 * a01;
  const T s = P.inv_n / det;
  z[0] = (r[0] * a11 - r[1] * a01) * s;
  z[1] = (r[1] * a00 - r[0] * a01) * s;
}

template <typename T, int NC>
__device__ __forceinline__ T redot(const cpx<T>* r, const cpx<T>* z) {
  T s = T(0);
#pragma unroll
  for (int c = 0; c < NC; ++c) s += r[c].re * z[c].re + r[c].im * z[c].im;
  return s;
}

// ===================================================== z pass (3D, last)
// One tile (slot columns s0..s0+TX-1 of row y, 3 components, all kz) held in
// LDS: forward FFT along z, z_hat = K_ref^{-1} r_hat / n (table or closed
// form), r.z partial (Parseval weights) into acc, inverse FFT.  Called by
// every thread of the block; ends with a barrier.
template <typename T, int N, int TX, int RP, int NTH>
__device__ __forceinline__ void zpass_tile(const PArgs<T>& a, int l, int y, int s0, cpx<T>* buf,
                                           const cpx<T>* tws, double& acc) {
  constexpr int NC = 3 * TX;
  const int M = a.nx / 2;
  const int tid = threadIdx.x;
  fft_lds<T, N, false, NC, NTH, 1, ColTile<NC>, RP>(buf, tws);
  const bool pair_row = (s0 == 0) && (y == 0 || y == a.ny / 2);
  // ordinary wavevectors (weight 2: each stands for itself and its conjugate)
  constexpr int QS = (N * TX + NTH - 1) / NTH;
  if (a.tab) {
    // all of a thread's table entries are loaded before the first use
    // this row's entries: the row base once, 32-bit offsets per element
    const T* tab = a.tab + (long long)(l / a.lpc) * a.tab_stride + (long long)y * a.nz * M * 6;
    T m[QS][6];
#pragma unroll
    for (int q = 0; q < QS; ++q) {
      const int e = tid + q * NTH;
      const int kz = e / TX, s = e - kz * TX;
      const int slot = s0 + s;
      if (e < N * TX && slot < M) sym_load(tab, (unsigned)kz * (unsigned)M + (unsigned)slot, m[q]);
    }
#pragma unroll
    for (int q = 0; q < QS; ++q) {
      const int e = tid + q * NTH;
      const int kz = e / TX, s = e - kz * TX;
      const int slot = s0 + s;
      if (e >= N * TX || slot >= M || (slot == 0 && pair_row)) continue;
      cpx<T> r[3], z[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) r[c] = buf[kz * NC + c * TX + s];
      sym_apply3(m[q], r, z);
      acc += 2.0 * (double)redot<T, 3>(r, z);
#pragma unroll
      for (int c = 0; c < 3; ++c) buf[kz * NC + c * TX + s] = z[c];
    }
  }
  for (int e = tid; e < N * TX && !a.tab; e += NTH) {
    const int kz = e / TX, s = e - kz * TX;
    const int slot = s0 + s;
    if (slot >= M || (slot == 0 && pair_row)) continue;
    cpx<T> r[3], z[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = buf[kz * NC + c * TX + s];
    {
      const int kx = slot == 0 ? (y < a.ny / 2 ? 0 : M) : slot;
      sym_solve3(a, kx, y, kz, r, z);
    }
    acc += 2.0 * (double)redot<T, 3>(r, z);
#pragma unroll
    for (int c = 0; c < 3; ++c) buf[kz * NC + c * TX + s] = z[c];
  }
  if (pair_row) {
    // column slot 0 of rows ky = 0, ny/2: w = A_hat + i B_hat with A, B real
    // along z; A: (kx, ky) = (0 | M, 0), B: (0 | M, ny/2).
    const int kxf = (y == 0) ? 0 : M;
    constexpr int Q = (N + NTH - 1) / NTH;
    cpx<T> out[Q][3];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int kz = tid + q * NTH;
      if (kz < N) {
        const int km = (N - kz) % N;
        cpx<T> A[3], B[3], zA[3], zB[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const cpx<T> wk = buf[kz * NC + c * TX], wm = buf[km * NC + c * TX];
          A[c] = {(wk.re + wm.re) * T(0.5), (wk.im - wm.im) * T(0.5)};
          B[c] = {(wk.im + wm.im) * T(0.5), (wm.re - wk.re) * T(0.5)};
        }
        if (a.tab) {
          T mA[6], mB[6];
          sym_load(a.tab + (long long)(l / a.lpc) * a.tab_stride, ((long long)y * a.nz + kz) * M, mA);
          sym_load(a.tabB + (long long)(l / a.lpc) * a.tabB_stride, (long long)(y == 0 ? 0 : 1) * a.nz + kz, mB);
          sym_apply3(mA, A, zA);
          sym_apply3(mB, B, zB);
        } else {
          if (y == 0 && kz == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) zA[c] = {T(0), T(0)};
          } else {
            sym_solve3(a, kxf, 0, kz, A, zA);
          }
          sym_solve3(a, kxf, a.ny / 2, kz, B, zB);
        }
        acc += (double)redot<T, 3>(A, zA) + (double)redot<T, 3>(B, zB);
#pragma unroll
        for (int c = 0; c < 3; ++c) out[q][c] = {zA[c].re - zB[c].im, zA[c].im + zB[c].re};
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int kz = tid + q * NTH;
      if (kz < N) {
#pragma unroll
        for (int c = 0; c < 3; ++c) buf[kz * NC + c * TX] = out[q][c];
      }
    }
  }
  __syncthreads();
  fft_lds<T, N, true, NC, NTH, 1, ColTile<NC>, RP>(buf, tws);
}

// logical item = (y, slot tile, load), load fastest: the load cases of a
// tile share its symbol-table lines and neighbouring tiles (which share
// 128-byte spectrum lines) stay close, all on one XCD
template <typename T, int N, int TX, int RP, int NTH>
__global__ __launch_bounds__(NTH) void k_zpass(PArgs<T> a) {
  constexpr int NC = 3 * TX;  // columns: component-major, then slot
  __shared__ cpx<T> buf[N * NC];
  __shared__ cpx<T> tws[N];
  __shared__ double sh[NTH / WAVE];
  const int M = a.nx / 2;
  const int ntile = (M + TX - 1) / TX;
  const int per_load = ntile * a.ny;
  const int item = xcd_order(blockIdx.x, per_load * a.nload);
  if (item < 0) return;
  const int l = item % a.nload;
  const int pb = item / a.nload;  // partial index within the load
  if (!load_live(a.st + l, true)) return;
  const int tile = pb % ntile;
  const int y = pb / ntile;
  const int s0 = tile * TX;
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NTH) tws[i] = a.tw[i];
  cpx<T>* base = a.S + l * a.lstrideC + (long long)y * M + s0;
#ifdef CELLFFT_BOUNDS_CHECK
  const cpx<T>* S_lo = a.S + l * a.lstrideC;  // the slot's spectrum
  const cpx<T>* S_hi = S_lo + a.lstrideC;
#endif
  // global <-> LDS copies: thread t keeps one column (t mod NC: component
  // and slot) and walks z in steps of ZS = NTH / NC, so each element costs
  // one address add (32-bit offsets from the block's base: a load's
  // spectrum holds fewer than 2^31 complex values) and its LDS index is a
  // constant offset; the NTH mod NC threads left over idle
  constexpr int ZS = NTH / NC;
  constexpr int QZ = (N + ZS - 1) / ZS;
  const int col = tid % NC, zi = tid / NC;
  const bool act = zi < ZS && s0 + col % TX < M;
  const unsigned zstride = (unsigned)a.zsS;                  // z plane (padded)
  const unsigned off0 = (unsigned)(col / TX) * ((unsigned)a.nz * zstride) + (unsigned)zi * zstride + (unsigned)(col % TX);
  const unsigned ostep = (unsigned)ZS * zstride;
  // all of a thread's loads are issued before the first LDS store (a
  // strided loop that stores each value as it arrives waits out one memory
  // latency per element)
  {
    cpx<T> v[QZ];
#pragma unroll
    for (int q = 0; q < QZ; ++q) {
      const int z = zi + q * ZS;
      v[q] = (act && (N % ZS == 0 || z < N)) ? CK_LD(base, off0 + (unsigned)q * ostep, S_lo, S_hi) : cpx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int q = 0; q < QZ; ++q) {
      const int z = zi + q * ZS;
      if (zi < ZS && (N % ZS == 0 || z < N)) buf[(zi + q * ZS) * NC + col] = v[q];
    }
  }
  __syncthreads();
  double acc = 0.0;
  zpass_tile<T, N, TX, RP, NTH>(a, l, y, s0, buf, tws, acc);
  if (act) {
    // (a plain loop: unrolled, its addresses would stay live through the FFT)
    unsigned off = off0;
    for (int z = zi; z < N; z += ZS, off += ostep) CK_ST(base, off, S_lo, S_hi, buf[z * NC + col]);
  }
  const double bs = block_sum<NTH>(acc, sh);
  if (tid == 0) a.red.put(RED_RZ, l, pb, bs);
}

// ===================================================== y pass (2D, last)
template <typename T, int N, int V>
__global__ __launch_bounds__(NTZ) void k_ylast(PArgs<T> a) {
  constexpr int TX = z_tx<T, V>();
  constexpr int NC = 2 * TX;
  __shared__ cpx<T> buf[N * NC];
  __shared__ cpx<T> tws[N];
  __shared__ double sh[NTZ / WAVE];
  const int l = blockIdx.y;
  if (!load_live(a.st + l, true)) return;
  const int M = a.nx / 2;
  const int s0 = blockIdx.x * TX;
  // reference medium of the slot's cell
  const T* md = a.med ? a.med + 2 * (l / a.lpc) : nullptr;
  const T lam0 = md ? md[0] : a.lam0, mu0 = md ? md[1] : a.mu0;
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NTZ) tws[i] = a.tw[i];
  cpx<T>* base = a.S + l * a.lstrideC + s0;
  const cpx<T>* src = (a.Sin ? a.Sin : a.S) + l * a.lstrideC + s0;
  const long long cstride = (long long)a.ny * M;
  for (int e = tid; e < N * NC; e += NTZ) {
    const int y = e / NC, rem = e - y * NC;
    const int c = rem / TX, s = rem - c * TX;
    buf[e] = (s0 + s < M) ? src[c * cstride + (long long)y * M + s] : cpx<T>{T(0), T(0)};
  }
  __syncthreads();
  fft_lds<T, N, false, NC, NTZ, 1, ColTile<NC>>(buf, tws);
  double acc = 0.0;
  for (int e = tid; e < N * TX; e += NTZ) {
    const int ky = e / TX, s = e - ky * TX;
    const int slot = s0 + s;
    if (slot >= M || slot == 0) continue;
    cpx<T> r[2], z[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) r[c] = buf[ky * NC + c * TX + s];
    sym_solve2(a, lam0, mu0, slot, ky, r, z);
    acc += 2.0 * (double)redot<T, 2>(r, z);
#pragma unroll
    for (int c = 0; c < 2; ++c) buf[ky * NC + c * TX + s] = z[c];
  }
  if (s0 == 0) {
    constexpr int Q = (N + NTZ - 1) / NTZ;
    cpx<T> out[Q][2];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int ky = tid + q * NTZ;
      if (ky < N) {
        const int km = (N - ky) % N;
        cpx<T> A[2], B[2], zA[2], zB[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const cpx<T> wk = buf[ky * NC + c * TX], wm = buf[km * NC + c * TX];
          A[c] = {(wk.re + wm.re) * T(0.5), (wk.im - wm.im) * T(0.5)};
          B[c] = {(wk.im + wm.im) * T(0.5), (wm.re - wk.re) * T(0.5)};
        }
        if (ky == 0) {
          zA[0] = zA[1] = {T(0), T(0)};
        } else {
          sym_solve2(a, lam0, mu0, 0, ky, A, zA);
        }
        sym_solve2(a, lam0, mu0, M, ky, B, zB);
        acc += (double)redot<T, 2>(A, zA) + (double)redot<T, 2>(B, zB);
#pragma unroll
        for (int c = 0; c < 2; ++c) out[q][c] = {zA[c].re - zB[c].im, zA[c].im + zB[c].re};
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int ky = tid + q * NTZ;
      if (ky < N) {
#pragma unroll
        for (int c = 0; c < 2; ++c) buf[ky * NC + c * TX] = out[q][c];
      }
    }
  }
  __syncthreads();
  fft_lds<T, N, true, NC, NTZ, 1, ColTile<NC>>(buf, tws);
  for (int e = tid; e < N * NC; e += NTZ) {
    const int y = e / NC, rem = e - y * NC;
    const int c = rem / TX, s = rem - c * TX;
    if (s0 + s < M) base[c * cstride + (long long)y * M + s] = buf[e];
  }
  const double bs = block_sum<NTZ>(acc, sh);
  if (tid == 0) a.red.put(RED_RZ, l, blockIdx.x, bs);
}

// ================================================================ finalize
// One block per load: fixed-order sum of the per-block partials written by
// the producing kernel, then the scalar update of that reduction.
template <int NTF>
__global__ __launch_bounds__(NTF) void k_finalize(RedBuf red, LoadState* st, double* res2, int slot,
                                                 int nparts, int only_load, const int* mask) {
  __shared__ double sh[NTF / WAVE];
  const int l = blockIdx.x;
  LoadState* S = st + l;
  bool live;
  switch (slot) {
    case RED_PQ: live = S->state == ST_ACTIVE || S->state == ST_CONVERGED; break;
    case RED_RR: live = S->state == ST_ACTIVE; break;
    case RED_RZ: live = S->state == ST_ACTIVE || S->state == ST_CONVERGED; break;
    default: live = mask ? mask[l] != 0 : (only_load < 0 || only_load == l); break;
  }
  if (!live) return;
  if (slot == RED_PQ && S->state == ST_CONVERGED) {
    // the iteration that converged has completed (preconditioning and
    // updates ran); no operator was applied to this load in this one
    if (threadIdx.x == 0) S->state = ST_DONE;
    return;
  }
  const double* parts = red.slot_parts(slot, l);
  double v = 0.0;
  for (int i = threadIdx.x; i < nparts; i += NTF) v += CK_LD(parts, i, parts, parts + red.maxblk);
  const double s = block_sum<NTF>(v, sh);
  if (threadIdx.x != 0) return;
  switch (slot) {
    case RED_PQ:
      S->pq = s;
      S->iters += 1;
      if (!(s == s) || !(s < 1e300)) S->state = ST_BREAKDOWN;
      else if (!(s > 0.0)) S->state = S->negok ? ST_NEGCURV : ST_BREAKDOWN;
      else S->alpha = S->rz / s;
      break;
    case RED_RR:
      S->rr = s;
      if (red.hist) red.hist[(long long)l * red.hist_cap + min(S->iters, red.hist_cap - 1)] = s;
      if (!(s == s) || s > 1e300) S->state = ST_BREAKDOWN;
      else if (s <= S->thr) S->state = ST_CONVERGED;
      else if (S->iters >= S->maxit) {
        S->state = ST_CONVERGED;
        S->maxit_hit = 1;
      }
      break;
    case RED_RZ: {
      const bool conv = S->state == ST_CONVERGED;
      if (!(s == s) || (!(s > 0.0) && !conv)) {
        S->state = ST_BREAKDOWN;
        break;
      }
      S->beta = (S->first || !(S->rz > 0.0)) ? 0.0 : s / S->rz;
      S->rz = s;
      S->first = 0;
      break;
    }
    default:
      res2[l] = s;
      break;
  }
}

hipError_t launch_finalize(const RedBuf& red, LoadState* st, double* res2, int slot, int nparts, int nload,
                           int only_load, const int* mask, hipStream_t s) {
  // one block per load: 1024 threads for the long partial lists (x passes),
  // 256 for short ones
  if (nparts > 4096)
    hipLaunchKernelGGL(k_finalize<1024>, dim3(nload), dim3(1024), 0, s, red, st, res2, slot, nparts, only_load, mask);
  else
    hipLaunchKernelGGL(k_finalize<NT>, dim3(nload), dim3(NT), 0, s, red, st, res2, slot, nparts, only_load, mask);
  return hipGetLastError();
}

int last_pass_blocks(int dim, int nx, int ny, bool fp64, const Sched& sc) {
  const int B = fp64 ? 4 : 8;
  const int TX = dim == 2 ? B >> (sc.z_var & 1) : (sc.z_var == 1 ? B / 2 : sc.z_var == 3 ? 2 * B : B);
  const int ntile = (nx / 2 + TX - 1) / TX;
  return dim == 3 ? ntile * ny : ntile;
}

// ================================================================ dispatch
#define CELLFFT_NSIZES(X) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256)
#define CELLFFT_MSIZES(X) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128)

bool fft_size_ok(int n) {
  switch (n) {
#define C_(v) case v:
    CELLFFT_NSIZES(C_)
#undef C_
    return true;
    default:
      return false;
  }
}

int xpass_blocks(int nx, int nrows, bool fp64, const Sched& sc) {
  const int M = nx / 2;
  const int tgt = (fp64 ? 1024 : 2048) >> (sc.x_var & 1);
  const int rpb = (tgt / M) < 1 ? 1 : tgt / M;
  return (nrows + rpb - 1) / rpb;
}

template <typename T, int V, int RP>
static hipError_t launch_xfwd_v(const XArgs<T>& a, int nx, dim3 grid, hipStream_t s) {
  switch (nx / 2) {
#define C_(m)                                                                               \
  case m:                                                                                   \
    if (a.mode == 0) hipLaunchKernelGGL((k_xfwd<T, m, V, RP, 0>), grid, dim3(NT), 0, s, a); \
    else hipLaunchKernelGGL((k_xfwd<T, m, V, RP, 1>), grid, dim3(NT), 0, s, a);             \
    break;
    CELLFFT_MSIZES(C_)
#undef C_
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int V, int RP>
static hipError_t launch_xinv_v(const XArgs<T>& a, int nx, dim3 grid, hipStream_t s) {
  switch (nx / 2) {
#define C_(m) case m: hipLaunchKernelGGL((k_xinv<T, m, V, RP>), grid, dim3(NT), 0, s, a); break;
    CELLFFT_MSIZES(C_)
#undef C_
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xfwd(const XArgs<T>& a, int nx, int nload, const Sched& sc, hipStream_t s) {
  const dim3 grid(xcd_grid(xpass_blocks(nx, a.nrows, sizeof(T) == 8, sc)), nload);
  switch (sc.x_var) {
    case 0: return launch_xfwd_v<T, 0, 0>(a, nx, grid, s);
    case 1: return launch_xfwd_v<T, 1, 0>(a, nx, grid, s);
    case 2: return launch_xfwd_v<T, 0, 1>(a, nx, grid, s);
    default: return launch_xfwd_v<T, 1, 1>(a, nx, grid, s);
  }
}

template <typename T>
hipError_t launch_xinv(const XArgs<T>& a, int nx, int nload, const Sched& sc, hipStream_t s) {
  const dim3 grid(xcd_grid(xpass_blocks(nx, a.nrows, sizeof(T) == 8, sc)), nload);
  switch (sc.x_var) {
    case 0: return launch_xinv_v<T, 0, 0>(a, nx, grid, s);
    case 1: return launch_xinv_v<T, 1, 0>(a, nx, grid, s);
    case 2: return launch_xinv_v<T, 0, 1>(a, nx, grid, s);
    default: return launch_xinv_v<T, 1, 1>(a, nx, grid, s);
  }
}

template <typename T, int V, int RP>
static hipError_t launch_ypass_v(const YArgs<T>& a, bool inverse, int nload, hipStream_t s) {
  constexpr int TX = y_tx<T, V>();
  const int M = a.nx / 2;
  const int ntile = (M + TX - 1) / TX;
  dim3 grid(xcd_grid(ntile * a.nz * a.ncomp), nload);
  switch (a.ny) {
#define C_(n)                                                                     \
  case n:                                                                         \
    if (inverse) hipLaunchKernelGGL((k_ypass<T, n, true, V, RP>), grid, dim3(NTY), 0, s, a); \
    else hipLaunchKernelGGL((k_ypass<T, n, false, V, RP>), grid, dim3(NTY), 0, s, a);       \
    break;
    CELLFFT_NSIZES(C_)
#undef C_
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ypass(const YArgs<T>& a, bool inverse, int nload, const Sched& sc, hipStream_t s) {
  switch (sc.y_var) {
    case 0: return launch_ypass_v<T, 0, 0>(a, inverse, nload, s);
    case 1: return launch_ypass_v<T, 1, 0>(a, inverse, nload, s);
    case 2: return launch_ypass_v<T, 0, 1>(a, inverse, nload, s);
    default: return launch_ypass_v<T, 1, 1>(a, inverse, nload, s);
  }
}

template <typename T, int TX, int RP, int NTH>
static hipError_t launch_zpass_v(const PArgs<T>& a, int nload, hipStream_t s) {
  const int ntile = (a.nx / 2 + TX - 1) / TX;
  dim3 grid(xcd_grid(ntile * a.ny * nload));
  switch (a.nz) {
#define C_(n) case n: hipLaunchKernelGGL((k_zpass<T, n, TX, RP, NTH>), grid, dim3(NTH), 0, s, a); break;
    CELLFFT_NSIZES(C_)
#undef C_
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int V>
static hipError_t launch_ylast_v(const PArgs<T>& a, int nload, hipStream_t s) {
  constexpr int TX = z_tx<T, V>();
  const int ntile = (a.nx / 2 + TX - 1) / TX;
  dim3 grid(ntile, nload);
  switch (a.ny) {
#define C_(n) case n: hipLaunchKernelGGL((k_ylast<T, n, V>), grid, dim3(NTZ), 0, s, a); break;
    CELLFFT_NSIZES(C_)
#undef C_
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_last(const PArgs<T>& a, int dim, int nload, const Sched& sc, hipStream_t s) {
  // z_var (3D): columns x threads per block = B x 512, B/2 x 512, B x 768,
  // 2B x 1024 with B = 8 (fp32) / 4 (fp64); wider column tiles read longer
  // row segments of each z plane, more threads hide more latency
  if (dim == 3) {
    constexpr int B = sizeof(T) == 4 ? 8 : 4;
    switch (sc.z_var * 2 + sc.z_radix) {
      case 0: return launch_zpass_v<T, B, 0, NTZ>(a, nload, s);
      case 1: return launch_zpass_v<T, B, 1, NTZ>(a, nload, s);
      case 2: return launch_zpass_v<T, B / 2, 0, NTZ>(a, nload, s);
      case 3: return launch_zpass_v<T, B / 2, 1, NTZ>(a, nload, s);
      case 4: return launch_zpass_v<T, B, 0, 768>(a, nload, s);
      case 5: return launch_zpass_v<T, B, 1, 768>(a, nload, s);
      case 6: return launch_zpass_v<T, 2 * B, 0, 1024>(a, nload, s);
      default: return launch_zpass_v<T, 2 * B, 1, 1024>(a, nload, s);
    }
  }
  return (sc.z_var & 1) ? launch_ylast_v<T, 1>(a, nload, s) : launch_ylast_v<T, 0>(a, nload, s);
}

template <typename T>
hipError_t launch_symtab(const PArgs<T>& a, T* tab, T* tabB, hipStream_t s) {
  hipLaunchKernelGGL(k_symtab<T>, dim3(2048), dim3(NT), 0, s, a, tab, tabB);
  return hipGetLastError();
}

template hipError_t launch_symtab<float>(const PArgs<float>&, float*, float*, hipStream_t);
template hipError_t launch_symtab<double>(const PArgs<double>&, double*, double*, hipStream_t);
template hipError_t launch_xfwd<float>(const XArgs<float>&, int, int, const Sched&, hipStream_t);
template hipError_t launch_xfwd<double>(const XArgs<double>&, int, int, const Sched&, hipStream_t);
template hipError_t launch_xinv<float>(const XArgs<float>&, int, int, const Sched&, hipStream_t);
template hipError_t launch_xinv<double>(const XArgs<double>&, int, int, const Sched&, hipStream_t);
template hipError_t launch_ypass<float>(const YArgs<float>&, bool, int, const Sched&, hipStream_t);
template hipError_t launch_ypass<double>(const YArgs<double>&, bool, int, const Sched&, hipStream_t);
template hipError_t launch_last<float>(const PArgs<float>&, int, int, const Sched&, hipStream_t);
template hipError_t launch_last<double>(const PArgs<double>&, int, int, const Sched&, hipStream_t);

#ifdef CELLFFT_BOUNDS_CHECK
unsigned int oob_take_fft() { return oob_take(); }
#endif

}  // namespace cellfft
