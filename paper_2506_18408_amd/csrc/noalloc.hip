// Allocation-free variant of the fused SpMV+sketch export, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// Its workspace (control block, tile bounds, per-workgroup sketch and scalar
// partial rows, reduced sketch row, packed sketch columns) lives in one
// static device array of kNoAllocScratchBytes per GPU, which every GPU the
// library runs on holds until the process ends.  In host code the array's
// name is only a host-side stand-in: its device address is taken once per
// device, with that device current, by hipGetSymbolAddress, and only that
// address is ever passed to kernels.  Every call on a GPU shares that GPU's
// array, so calls that overlap on one GPU (other streams or threads) race;
// each call fully writes every region it reads, so nothing needs clearing
// between calls.
#include <mutex>

#include "kernels.hpp"

struct sfgmres_ctx;

namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kNoAllocScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on the current device (taken on the
// first call there), or nullptr with *err set.
void* scratch_of_current_device(hipError_t* err) {
  int dev = -1;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

}  // namespace

extern "C" {

int sfgmres_noalloc_scratch_bytes(size_t* bytes) {
  if (!bytes) return SFGMRES_ERR_INVALID;
  *bytes = kNoAllocScratchBytes;
  return SFGMRES_OK;
}

int sfgmres_spmv_sketch_noalloc(sfgmres_handle h, const sfgmres_csr* A, const double* u,
                                double scale, double* w, int32_t s, int32_t zeta, uint64_t seed,
                                const double* U, int64_t ldu, int32_t nwin, double* c,
                                double* dots, double* norm2, void* stream) {
  if (!h) return SFGMRES_ERR_INVALID;
  if (!A || A->n < 1 || A->nnz < 0 || A->n >= ((int64_t)1 << 31) ||
      A->nnz >= ((int64_t)1 << 31) || s < 1 || s > SFGMRES_MAX_S || zeta < 1 || zeta > s ||
      zeta > SFGMRES_MAX_ZETA)
    return sfg::spmv_sketch_impl(h, A, u, scale, w, s, zeta, seed, U, ldu, nwin, c, dots, norm2,
                                 nullptr, 0, stream);  // (reports the invalid argument)
  if (sfg::spmv_sketch_workspace(A->n, A->nnz, s, zeta) > kNoAllocScratchBytes)
    return sfg::report_error(h, SFGMRES_ERR_WORKSPACE,
                             "problem too large for the 64 MiB static scratch of the "
                             "allocation-free entry point");
  hipError_t e = hipSuccess;
  void* ws = scratch_of_current_device(&e);
  if (!ws)
    return sfg::report_error(h, SFGMRES_ERR_HIP,
                             std::string("hipGetSymbolAddress(scratch) failed: ") +
                                 hipGetErrorString(e));
  return sfg::spmv_sketch_impl(h, A, u, scale, w, s, zeta, seed, U, ldu, nwin, c, dots, norm2, ws,
                               kNoAllocScratchBytes, stream);
}

}  // extern "C"
