// Operator product q = K u for callers that cannot allocate device memory
// (work recorded under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc).  Same stencil kernel and schedule as
// cell_apply_operator in FP64, on the caller's device arrays; the per-block
// partials of u.Ku and the one-slot scalar block of the reduction live in a
// fixed-size array of this file instead of the handle's buffers, and no
// lazily allocated field buffer is touched.
#include <map>
#include <mutex>

#include "solver.h"

using namespace cellfft;

namespace {

// Scratch of the allocation-free entry point, one copy per device (held by
// every device the library runs on until the process ends):
//   [0, 256)          LoadState of the single slot (state, p.Kp)
//   [256, BYTES)      per-block partials of u.Ku, RED_PQ row of a one-slot RedBuf
constexpr size_t NOALLOC_BYTES = size_t(1) << 20;
constexpr size_t NOALLOC_STATE_BYTES = 256;
constexpr int NOALLOC_MAXBLK = (int)((NOALLOC_BYTES - NOALLOC_STATE_BYTES) / sizeof(double));
static_assert(sizeof(LoadState) <= NOALLOC_STATE_BYTES, "scalar block does not fit");

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// Device address of `scratch` per device.  The host-side name is only a
// stand-in for the symbol; the address comes from hipGetSymbolAddress with
// the device current, once per device.
std::mutex g_mu;
std::map<int, unsigned char*> g_addr;

cell_status scratch_address(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_addr.find(dev);
  if (it != g_addr.end()) {
    *out = it->second;
    return CELL_OK;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(CELL_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_addr[dev] = static_cast<unsigned char*>(p);
  *out = static_cast<unsigned char*>(p);
  return CELL_OK;
}

// the slot's scalars: active, so the stencil kernel and the finalize run
// (a kernel, not a memset, so that the sequence can be captured)
__global__ void k_noalloc_init(LoadState* st) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  LoadState s{};
  s.state = ST_ACTIVE;
  s.maxit = 1 << 30;
  s.first = 1;
  s.negok = 1;  // p.Kp <= 0 is reported, not a breakdown
  *st = s;
}

__global__ void k_noalloc_out(const LoadState* st, double* uKu) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *uKu = st->pq;
}

}  // namespace

extern "C" cell_status cell_apply_operator_noalloc(cell_t c, const double* u, double* q_out, double* uKu_out) {
  if (!c || !u || !q_out) return fail(CELL_E_ARG, "null argument");
  if (!c->have_mat[0]) return fail(CELL_E_STATE, "cell_set_material has not been called");
  if (c->sr_M > 0) return fail(CELL_E_UNSUPPORTED, "the allocation-free product applies the exact operator only");
  if (c->ncell != 1) return fail(CELL_E_ARG, "a single-cell handle is required");
  const int nparts = stencil_blocks(c->g, c->sched, true);
  if (nparts > NOALLOC_MAXBLK)
    return fail(CELL_E_ARG, "grid too large for the allocation-free scratch (" + std::to_string(nparts) +
                                " stencil blocks, at most " + std::to_string(NOALLOC_MAXBLK) + ")");
  DevGuard dg(c->dev);
  unsigned char* base = nullptr;
  const cell_status st = scratch_address(c->dev, &base);
  if (st < 0) return st;
  LoadState* ls = reinterpret_cast<LoadState*>(base);
  KArgs<double> a{};
  a.u = u;
  a.out = q_out;
  a.mat = c->mat64;
  a.lstride = c->lstride;
  a.g = c->g;
  a.nload = 1;
  a.lpc = c->lpc;
  a.mat_stride = 2 * c->n;
  a.mode = 0;
  a.st = ls;
  a.only_load = -1;
  a.negate = c->dbg_negate_q;
  a.red = RedBuf{reinterpret_cast<double*>(base + NOALLOC_STATE_BYTES), NOALLOC_MAXBLK, 1};
  hipLaunchKernelGGL(k_noalloc_init, dim3(1), dim3(64), 0, c->stream, ls);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_stencil<double>(a, c->sched, c->stream);
  if (e == hipSuccess && uKu_out) {
    hipLaunchKernelGGL(k_noalloc_out, dim3(1), dim3(64), 0, c->stream, (const LoadState*)ls, uKu_out);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return fail(CELL_E_DEVICE, std::string("cell_apply_operator_noalloc: ") + hipGetErrorString(e));
  return CELL_OK;
}
