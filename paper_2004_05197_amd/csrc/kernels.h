// Launch-parameter blocks and host launch wrappers of the cell-problem
// kernels.  Every wrapper checks that the requested size has a compiled
// instantiation and returns a hipError_t (hipErrorInvalidValue otherwise).
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"
#include "state.h"

namespace cellfft {

constexpr int NT = 256;  // threads per block of every kernel

// Reduction plumbing: per-block partials[slot][load][blk], summed in fixed
// order by a finalize kernel
struct RedBuf {
  double* parts;
  int maxblk;
  int maxload;
  double* hist = nullptr;  // per load: ||r_k||^2 after k iterations, hist_cap entries
  int hist_cap = 0;
  __host__ __device__ double* slot_parts(int slot, int load) const {
    return parts + ((long long)slot * maxload + load) * maxblk;
  }
  // partial blk of (slot, load); checked against its row in the debug build
  __device__ void put(int slot, int load, int blk, double v) const {
#ifdef CELLFFT_BOUNDS_CHECK
    if (slot < 0 || slot >= RED_NSLOT || load < 0 || load >= maxload) {
      atomicAdd(&g_oob_count, 1u);
      return;
    }
#endif
    double* row = slot_parts(slot, load);
    CK_ST(row, blk, row, row + maxblk, v);
  }
};

// Launch schedule of an instance: which compiled variant of each kernel
// runs.  Chosen by the autotuner (or left at the defaults); every variant
// computes the same result up to the order of floating-point sums inside a
// block, and the tests check each against the oracle.
struct Sched {
  int st_tile = 0;  // 3D stencil tile (BX x BY threads): fp32 {64x4, 32x8, 16x16,
                    // 64x8, 32x16, row-wave}, fp64 {32x8, 16x16, 64x4, 32x16, 16x32};
                    // a tile that does not fit the grid falls back to the first that
                    // does, else to the runtime-tile kernel
  int st_tz = 32;   // z extent of a stencil tile (8, 16, 32 or 64)
  int x_var = 0;    // x passes: rows per block = 2048 / (nx/2) (0, 2) or 1024 / (nx/2)
                    // (1, 3) complex values (fp64: 1024, 512); radix 8 first (0, 1)
                    // or radix 16 first (2, 3)
  int y_var = 0;    // y pass columns per block: 16 (0, 2) or 8 (1, 3) (fp64: 8, 4);
                    // radix 8 first (0, 1) or radix 16 first (2, 3)
  int z_var = 0;    // last pass columns x threads per block: 8 x 512 (0), 4 x 512 (1),
                    // 3D also 8 x 768 (2), 16 x 1024 (3)
                    // (fp64 half the columns); 2D: 2, 3 as 0, 1
  int z_radix = 0;  // last pass radix order: radix 8 first (0) or radix 16 first (1)
};
constexpr int SCHED_NFIELD = 6;
constexpr int ST_NTILE = 6;   // tile 5: the FP32 row-wave operator (falls back in FP64)
constexpr int ST_RW = 5;
constexpr int ST_TZ_MIN = 8;

struct Geom {
  int dim;
  int nx, ny, nz;      // nz = 1 in 2D
  long long n;         // voxels = nodes
  double h[3];         // voxel edge lengths
};

// ---------------------------------------------------------------- x passes
template <typename T> struct XArgs {
  const T* r;      // residual in real space (xfwd mode 1)
  const T* q;      // K p (xfwd mode 0)
  cpx<T>* R;       // residual transformed along x (packed half spectrum of every
                   // x row), the form in which the iteration keeps r
  cpx<T>* S;       // packed half spectrum, same element count as a real field
  T* x;            // iterate (xinv: x += alpha p_old)
  T* p;            // direction (xinv: p = z + beta p_old)
  long long lstride;  // reals per load in r/q/x/p (= d n); R stride = lstride/2
  int nrows;       // rows of length nx per load = d * ny * nz
  int ny;          // rows per (component, z) plane
  long long zsS;   // S: complex values per (component, z) plane (ny nx/2 + padding)
  long long lsS;   // S: complex values per load
  const cpx<T>* tw;   // nx twiddles exp(-2 pi i m / nx)
  int mode;        // xfwd: 0: R -= alpha FFT_x(q), ||r||^2 partials (Parseval);
                   //       1: R = FFT_x(r) for the slots in mask (or the active ones)
  const int* mask;
  LoadState* st;
  RedBuf red;
  const double* qmean;  // xfwd mode 0, nullptr or [slot][3]: per-component mean of q,
                        // removed from its transform (the projected operator P K P)
  int comp_rows;        // rows per component (ny nz) for qmean
  const T* edge;        // xfwd mode 0, nullptr or the row-wave operator's edge rows
                        // (added to q's rows y = 0 mod edge_rows), [load][3][nz][ny / edge_rows][nx]
  long long edge_stride;
  int edge_rows;
};

// ---------------------------------------------------------------- y pass (3D)
template <typename T> struct YArgs {
  cpx<T>* S;
  const cpx<T>* Sin;    // forward pass: read from here (the x-transformed residual,
                        // unpadded planes), write S; nullptr: in place
  long long lstrideC;   // complex elements per load of Sin (unpadded)
  long long zsS, lsS;   // S: complex values per (component, z) plane and per load
  int nx, ny, nz, ncomp;
  const cpx<T>* tw;     // ny twiddles
  LoadState* st;
};

// --------------------------------------------- last pass with preconditioner
template <typename T> struct PArgs {
  cpx<T>* S;
  const cpx<T>* Sin;    // 2D: read from here, write S (nullptr: in place)
  long long lstrideC;   // S: complex values per load (3D: 3 nz zsS)
  long long zsS;        // S: complex values per (component, z) plane (3D; padded so
                        // that the z pass's plane-strided reads spread over channels)
  int nx, ny, nz;
  const cpx<T>* tw;     // twiddles of the last axis (nz in 3D, ny in 2D)
  const T* trig[3];     // per axis: (sin(pi k / N_a), cos(pi k / N_a)), k < N_a
  T lam0, mu0;          // reference medium
  T w;                  // simplex weight |s| = h_x h_y (h_z) / d!
  T ih[3];              // 1 / h_a
  T inv_n;              // 1 / (nx ny nz): folds the unnormalised inverse DFT
  int nload;            // slots in the launch (cells x loads per cell)
  int lpc;              // load slots per cell
  long long tab_stride;  // symbol-table values per cell (tab, tabB)
  long long tabB_stride;
  const T* tab;         // 3D: tabulated K_ref^{-1} / n per stored wavevector
                        // ([ny][nz][nx/2][6]: 00,11,22,01,02,12), or nullptr
  const T* tabB;        // 3D: second family of the two real-pair rows [2][nz][6]
  const T* med;         // 2D: per-cell (lambda0, mu0) pairs [ncell][2]; nullptr =
                        // every slot uses (lam0, mu0)
  LoadState* st;
  RedBuf red;
};

// ---------------------------------------------------------------- stencils
template <typename T> struct KArgs {
  const T* u;           // input displacement (nullptr = zero field)
  void* out;            // output field (T, or float for the mixed residual)
  const T* mat;         // per voxel (lambda, mu) pairs
  long long lstride;    // reals per load
  Geom g;
  double eps[6][6];     // macro strains per load, tensor order (00,11,22,12,02,01)
  int nload;            // slots in the launch (cells x loads per cell)
  int lpc;              // load slots per cell: slot l belongs to cell l / lpc and
                        // uses macro strain eps[l % lpc]
  long long mat_stride; // material values (2 per voxel) per cell
  int mode;             // 0: out = K u, partial u.out ; 1: out = -B^T D (eps + B u), partial out.out
  LoadState* st;        // mode 0: per-load scalars (alpha = rz / pq)
  int only_load;        // mode 1: >= 0 restricts to one slot
  const int* mask;      // mode 1: if set, the slots with mask[l] != 0 (overrides only_load)
  double* res2;         // mode 1: per-load ||out||^2 (FP64)
  double* sparts;       // mode 1 (optional): per-block sums of |s| sigma over the
                        // block's own voxels, [load][6][maxblk] (tensor storage
                        // 00,11,22,12,02,01); nullptr = not accumulated
  double* sbar;         // mode 1 (optional): [load][6] finalised stress sums
  int negate;           // mode 0, debugging only: 1 writes -K u (forces a CG breakdown)
  // row-wave FP32 operator (mode 0): contributions of each tile's last voxel
  // row to the first node row of the next tile, [load][3][nz][ny / rows][nx]
  // with rows = rw_rows(nx)
  // floats; edge_fused = 1: the x forward pass adds them to q (else the
  // launch adds them itself); nullptr: the row-wave kernel is not used
  float* edge;
  long long edge_stride;  // floats per load
  int edge_fused;
  RedBuf red;
};

// ------------------------------------------------- neo-Hookean (Newton) path
template <typename T> struct HyArgs {
  const T* u;           // Newton state: F = F_bar + grad u, [slot][d][n]
  const T* p;           // mode 0: direction; mode 1: correction du (nullptr = 0)
  void* out;            // mode 0: q (T); mode 1: r (float or double); mode 2: f (double)
  const double* rhs;    // mode 1: Newton right-hand side [slot][d][n]
  const T* mat;         // (lambda, mu) per voxel, [cell][n][2]
  long long mat_stride;
  long long lstride;    // reals per slot
  Geom g;
  const double* Fbar;   // [slot][3][3] macroscopic deformation gradients (row-major)
  const T* FbarT;       // the same in the arithmetic type
  int nload;            // slots in the launch
  int lpc;              // slots per cell
  LoadState* st;        // mode 0: per-slot state (active slots only)
  const int* mask;      // modes 1, 2: slots to compute (nullptr = all)
  double* res2;         // per-slot ||out||^2 (modes 1, 2)
  double* vparts;       // mode 2: per-block sums [slot][10][maxblk]: |s| W, |s| P (3 x 3)
  double* vals;         // mode 2: [slot][10] finalised sums
  RedBuf red;
};

// q = K_T(u) p (T arithmetic) with the PCG scalar update of the p.q partials
template <typename T> hipError_t launch_hyper_tangent(const HyArgs<T>& a, hipStream_t s);
// r = rhs - K_T(u) du in FP64 (written as float if out32), ||r||^2
hipError_t launch_hyper_tangent_residual(const HyArgs<double>& a, bool out32, hipStream_t s);
// f = -sum |s| B^T P(F) in FP64, ||f||^2, energy and mean-stress sums
hipError_t launch_hyper_residual(const HyArgs<double>& a, hipStream_t s);
int hyper_blocks(const Geom& g, int maxblk);
hipError_t launch_axpy_slots(const double* x, const double* t, const double* d, double* y, long long len, int nslot,
                             const int* mask, hipStream_t s);
hipError_t launch_copy_slots(const double* x, double* y, long long len, int nslot, const int* mask, hipStream_t s);
hipError_t launch_round_slots(const double* x, float* y, long long len, int nslot, hipStream_t s);
// x[slot][c] -= its mean over the n nodes, per component, for the masked
// slots; parts: scratch of at least 3 * nslot * maxparts doubles
hipError_t launch_remove_mean(double* x, long long lstride, long long n, int d, int nslot, const int* mask,
                              double* parts, int maxparts, hipStream_t s);
// ------------------------------------------------- surrogate stencil operator
// Stencil functions of the 3D operator: the 3 x 3 block coupling node i with
// node i + delta for the seven offsets delta in {x, y, z, xy, yz, xz, xyz}
// (0/1 vectors), value k = 9 delta + 3 a + b (row a, column b).
constexpr int SR_NOFF = 7;
constexpr int SR_NVAL = 63;
// Stencil layout: runs of SR_CHUNK consecutive nodes store their 63 values
// value-major (value v of node i at sr_chunk(i) + v * SR_CHUNK), so one
// wavefront's stencil reads cover one contiguous 16 KB (FP32) region
constexpr int SR_CHUNK = 64;
__host__ __device__ inline long long sr_chunk(long long node) {
  return (node / SR_CHUNK) * (SR_NVAL * SR_CHUNK) + node % SR_CHUNK;
}
inline long long sr_len(long long n) { return (n + SR_CHUNK - 1) / SR_CHUNK * SR_CHUNK * SR_NVAL; }
template <typename T> struct SArgs {
  const T* s;           // surrogate stencil blocks, chunked layout (sr_chunk)
  const T* p;           // mode 0: direction; mode 1: iterate u [slot][3][n]
  void* out;            // mode 0: q (T); mode 1: r (TO)
  const double* rhs;    // mode 1: load vectors f [slot][3][n]
  long long lstride;
  Geom g;
  int nslot;            // <= 6
  LoadState* st;        // mode 0 liveness
  const int* mask;      // mode 1 slots
  double* cparts;       // per-block component sums [slot][3][nb]
  double* mean;         // [slot][3] component means of the output
  RedBuf red;
};
// B-spline expansion of the stencil coefficients on the lattice of every
// M-th node (degree q in {1, 3}) to every node, FP64 and FP32 copies
hipError_t launch_sr_expand(const double* coef, int ncx, int ncy, int ncz, int M, int q, const Geom& g, double* s64,
                            float* s32, hipStream_t s);
// partial sums written by the surrogate operator's launches (for the
// reduction buffers)
int sr_max_blocks(const Geom& g);
// q = Kt p for the active slots, p.q partials, per-component means of q
template <typename T> hipError_t launch_sr_apply(const SArgs<T>& a, hipStream_t s);
// r = P (f - Kt u) in FP64 (written as float if out32) for the masked
// slots, ||r||^2 -> res2
hipError_t launch_sr_residual(const SArgs<double>& a, bool out32, double* res2, hipStream_t s);

// r = rhs over the first m reals of every masked slot (float if out32),
// ||r||^2 -> res2 (the Newton residual at du = 0)
hipError_t launch_rhs_residual(const double* rhs, void* r, bool out32, long long lstride, long long m, int nslot,
                               const int* mask, const RedBuf& red, LoadState* st, double* res2, hipStream_t s);
// max |x[slot]| partials: parts[slot][nb], nb = min(maxparts, AMAX_BLOCKS)
constexpr int AMAX_BLOCKS = 256;
hipError_t launch_amax_slots(const double* x, long long len, int nslot, const int* mask, double* parts, int maxparts,
                             hipStream_t s);
hipError_t launch_widen_slots(const float* x, double* y, long long len, int nslot, const int* mask, hipStream_t s);
hipError_t launch_zero_slots(double* x, long long len, int nslot, const int* mask, hipStream_t s);
// per-slot x . y (FP64) into res2 for the masked slots
hipError_t launch_dot_slots(const double* x, const double* y, long long len, int nslot, const int* mask,
                            const RedBuf& red, LoadState* st, double* res2, hipStream_t s);

// effective stiffness / adjoint
struct HArgs {
  const double* u;      // solved fluctuations [nload][d][n]
  const double* mat;    // (lambda, mu) pairs (FP64)
  const double* E;      // Young's modulus per voxel (gradient only)
  long long lstride;
  Geom g;
  double eps[6][6];
  int nload;            // solved loads per cell
  int lpc;              // load slots per cell (slot of load j of cell c: c lpc + j)
  double a[6][6];       // gradient weights dJ/dC_IJ
  double* grad;         // per-voxel gradient output
  const void* r;        // residual fields f - K u [nload][d][n] (float or double)
  int r_fp64;           // 1: r is double
  const double* sbar;   // [nload][6]: sum over simplices of |s| sigma (tensor storage)
  double* parts;        // per-block partials [nval][nblk]
  double* result;       // [nload*nload + nload*nv]: C (energy form), mean stress
  int nblk;
};

template <typename T> hipError_t launch_xfwd(const XArgs<T>& a, int nx, int nload, const Sched& sc, hipStream_t s);
template <typename T> hipError_t launch_xinv(const XArgs<T>& a, int nx, int nload, const Sched& sc, hipStream_t s);
template <typename T>
hipError_t launch_ypass(const YArgs<T>& a, bool inverse, int nload, const Sched& sc, hipStream_t s);
template <typename T> hipError_t launch_last(const PArgs<T>& a, int dim, int nload, const Sched& sc, hipStream_t s);
// fills a.tab / a.tabB (3D) from the closed-form symbol of the reference medium
template <typename T> hipError_t launch_symtab(const PArgs<T>& a, T* tab, T* tabB, hipStream_t s);
template <typename T> hipError_t launch_stencil(const KArgs<T>& a, const Sched& sc, hipStream_t s);
hipError_t launch_residual_mixed(const KArgs<double>& a, float* out32, const Sched& sc, hipStream_t s);
hipError_t launch_homog(const HArgs& a, int ncell, hipStream_t s);
hipError_t launch_grad(const HArgs& a, hipStream_t s);

// fixed-order sum of per-block partials and the scalar update of `slot`
// (one block per load)
hipError_t launch_finalize(const RedBuf& red, LoadState* st, double* res2, int slot, int nparts, int nload,
                           int only_load, const int* mask, hipStream_t s);
int last_pass_blocks(int dim, int nx, int ny, bool fp64, const Sched& sc);

// blocks used by each kernel under a schedule (reduction parts), and the
// most over every schedule (for sizing the partials buffers)
int xpass_blocks(int nx, int nrows, bool fp64, const Sched& sc);
int stencil_blocks(const Geom& g, const Sched& sc, bool fp64);
int max_reduction_blocks(const Geom& g);
// stencil tile variant t of a precision: (BX, BY), and whether it fits the grid
void stencil_tile_dims(bool fp64, int t, int* bx, int* by);
bool stencil_tile_fits(const Geom& g, bool fp64, int t);
// the row-wave operator: voxel rows (waves) per block for a row length
// (4 at nx = 256, else 8), its grid condition (3D, nx in {64, 128, 256},
// ny a multiple of the rows per block) and its edge-row floats per load
int rw_rows(int nx);
bool rw_fits(const Geom& g);
// the tile a schedule's stencil launches run (-1: runtime tile)
int stencil_effective_tile(const Geom& g, bool fp64, int t);
long long rw_edge_floats(const Geom& g);
int homog_blocks(const Geom& g);
bool fft_size_ok(int n);      // y/z length (and x length)

#ifdef CELLFFT_BOUNDS_CHECK
// read and clear each module's out-of-range access counter (current device)
unsigned int oob_take_fft();
unsigned int oob_take_stencil();
unsigned int oob_take_hyper();
unsigned int oob_take_surrogate();
#endif

}  // namespace cellfft
