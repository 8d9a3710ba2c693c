// Per-load solver scalars and launch parameter blocks shared by the kernels
// and the host driver.
#pragma once
#include <stdint.h>

namespace cellfft {

// CG load states
enum : int {
  ST_IDLE = 0,       // not part of the current solve
  ST_ACTIVE = 1,     // iterating
  ST_CONVERGED = 2,  // residual test passed in this iteration; the iteration
                     // still completes (preconditioning + direction update)
  ST_DONE = 3,       // iteration finished after convergence / max_iter
  ST_BREAKDOWN = -1,  // p.Kp <= 0 or r.z <= 0 or non-finite scalar
  ST_NEGCURV = -2     // p.Kp <= 0 in a solve that allows it (Newton steps):
                      // the iterate of the previous iteration is kept
};

// Device-resident per-load scalars.  All reductions are FP64.
struct LoadState {
  double rz;      // r^T z of the current direction
  double alpha;   // step length of the current iteration
  double beta;    // direction update coefficient
  double rr;      // ||r||^2 of the iterated residual
  double pq;      // p^T K p
  double thr;     // convergence threshold on rr: tol^2 ||f||^2
  int state;
  int iters;      // completed operator applications (CG iterations)
  int maxit;
  int first;      // 1 until the first preconditioning has set rz
  int maxit_hit;  // 1 if the iteration stopped on max_iter
  int negok;      // 1: p.Kp <= 0 ends the iteration (ST_NEGCURV), else breakdown
};

// Reduction slots (one counter and one partials row per slot and load)
enum : int { RED_PQ = 0, RED_RR = 1, RED_RZ = 2, RED_XINV = 3, RED_RES = 4, RED_NSLOT = 5 };

}  // namespace cellfft
