// Launch-parameter blocks and host launch wrappers of the cell-problem
// kernels.  Every wrapper checks that the requested size has a compiled
// instantiation and returns a hipError_t (hipErrorInvalidValue otherwise).
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"
#include "state.h"

namespace cellfft {

constexpr int NT = 256;  // threads per block of every kernel

// Reduction plumbing: partials[slot][load][blk], counters[slot][load]
struct RedBuf {
  double* parts;
  unsigned* cnt;
  int maxblk;
  int maxload;
  __host__ __device__ double* slot_parts(int slot, int load) const {
    return parts + ((long long)slot * maxload + load) * maxblk;
  }
  __host__ __device__ unsigned* slot_cnt(int slot, int load) const {
    return cnt + slot * maxload + load;
  }
};

struct Geom {
  int dim;
  int nx, ny, nz;      // nz = 1 in 2D
  long long n;         // voxels = nodes
  double h[3];         // voxel edge lengths
};

// ---------------------------------------------------------------- x passes
template <typename T> struct XArgs {
  T* r;            // residual (xfwd: updated in place)
  const T* q;      // K p (xfwd)
  cpx<T>* S;       // packed half spectrum, same element count as a real field
  T* x;            // iterate (xinv: x += alpha p_old)
  T* p;            // direction (xinv: p = z + beta p_old)
  long long lstride;  // reals per load in r/q/x/p (= d n); S stride = lstride/2
  int nrows;       // rows of length nx per load = d * ny * nz
  const cpx<T>* tw;   // nx twiddles exp(-2 pi i m / nx)
  LoadState* st;
  RedBuf red;
};

// ---------------------------------------------------------------- y pass (3D)
template <typename T> struct YArgs {
  cpx<T>* S;
  long long lstrideC;   // complex elements per load
  int nx, ny, nz, ncomp;
  const cpx<T>* tw;     // ny twiddles
  LoadState* st;
};

// --------------------------------------------- last pass with preconditioner
template <typename T> struct PArgs {
  cpx<T>* S;
  long long lstrideC;
  int nx, ny, nz;
  const cpx<T>* tw;     // twiddles of the last axis (nz in 3D, ny in 2D)
  const T* trig[3];     // per axis: (sin(pi k / N_a), cos(pi k / N_a)), k < N_a
  T lam0, mu0;          // reference medium
  T w;                  // simplex weight |s| = h_x h_y (h_z) / d!
  T ih[3];              // 1 / h_a
  T inv_n;              // 1 / (nx ny nz): folds the unnormalised inverse DFT
  int nload;            // load cases in the launch
  const T* tab;         // 3D: tabulated K_ref^{-1} / n per stored wavevector
                        // ([ny][nz][nx/2][6]: 00,11,22,01,02,12), or nullptr
  const T* tabB;        // 3D: second family of the two real-pair rows [2][nz][6]
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
  int nload;
  int mode;             // 0: out = K u, partial u.out ; 1: out = -B^T D (eps + B u), partial out.out
  LoadState* st;        // mode 0: per-load scalars (alpha = rz / pq)
  int only_load;        // mode 1: >= 0 restricts to one load
  double* res2;         // mode 1: per-load ||out||^2 (FP64)
  double* sparts;       // mode 1 (optional): per-block sums of |s| sigma over the
                        // block's own voxels, [load][6][maxblk] (tensor storage
                        // 00,11,22,12,02,01); nullptr = not accumulated
  double* sbar;         // mode 1 (optional): [load][6] finalised stress sums
  RedBuf red;
};

// effective stiffness / adjoint
struct HArgs {
  const double* u;      // solved fluctuations [nload][d][n]
  const double* mat;    // (lambda, mu) pairs (FP64)
  const double* E;      // Young's modulus per voxel (gradient only)
  long long lstride;
  Geom g;
  double eps[6][6];
  int nload;
  double a[6][6];       // gradient weights dJ/dC_IJ
  double* grad;         // per-voxel gradient output
  const void* r;        // residual fields f - K u [nload][d][n] (float or double)
  int r_fp64;           // 1: r is double
  const double* sbar;   // [nload][6]: sum over simplices of |s| sigma (tensor storage)
  double* parts;        // per-block partials [nval][nblk]
  double* result;       // [nload*nload + nload*nv]: C (energy form), mean stress
  int nblk;
};

template <typename T> hipError_t launch_xfwd(const XArgs<T>& a, int nx, int nload, hipStream_t s);
template <typename T> hipError_t launch_xinv(const XArgs<T>& a, int nx, int nload, hipStream_t s);
template <typename T> hipError_t launch_ypass(const YArgs<T>& a, bool inverse, int nload, hipStream_t s);
template <typename T> hipError_t launch_last(const PArgs<T>& a, int dim, int nload, hipStream_t s);
// fills a.tab / a.tabB (3D) from the closed-form symbol of the reference medium
template <typename T> hipError_t launch_symtab(const PArgs<T>& a, T* tab, T* tabB, hipStream_t s);
template <typename T> hipError_t launch_stencil(const KArgs<T>& a, hipStream_t s);
hipError_t launch_residual_mixed(const KArgs<double>& a, float* out32, hipStream_t s);
hipError_t launch_homog(const HArgs& a, hipStream_t s);
hipError_t launch_grad(const HArgs& a, hipStream_t s);

// fixed-order sum of per-block partials and the scalar update of `slot`
// (one block per load)
hipError_t launch_finalize(const RedBuf& red, LoadState* st, double* res2, int slot, int nparts, int nload,
                           int only_load, hipStream_t s);
int last_pass_blocks(int dim, int nx, int ny, bool fp64);

// blocks used by each kernel (for sizing the partials buffer)
int xpass_blocks(int nx, int nrows, bool fp64);
int stencil_blocks(const Geom& g);
int homog_blocks(const Geom& g);
bool fft_size_ok(int n);      // y/z length (and x length)

}  // namespace cellfft
