// Launcher interface between the host driver (solver.hip) and the kernel
// translation units (spmv.hip, qr.hip, vec.hip).  Every launcher enqueues on
// `st` and returns the hipError_t of the launch.
#pragma once

#include "common.hpp"

namespace sfg {

enum SpmvMode : int {
  kModeInner = 0,    // w = scale * A u ; S w ; <w, U_l> ; ||w||^2            (predicated)
  kModeOuter = 1,    // w = A z ; <w, v_1> ; ||v_j - w||^2 ; last block stores h_{1,j}
  kModeResid = 2,    // w = b - A x ; ||w||^2 ; ||b||^2 ; last block stores beta, ||b||
  kModeTrueRes = 3,  // ||b - A x||^2 ; last block stores it
  kModePlain = 4,    // as kModeInner without predication (test export)
};

struct SpmvArgs {
  int64_t n;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const void* val;          // double* (FP64) or float* (mixed inner)
  const int32_t* tiles;     // ntiles+1 row boundaries
  int32_t ntiles;
  int32_t has_x;            // kModeResid: 0 means x = 0
  const void* x;            // input vector, same type as val
  const double* scale_ptr;  // kModeInner: device scalar multiplying A u (NULL: scale_val)
  double scale_val;
  void* w;                  // output vector, same type as val (NULL = not written)
  const double* b;          // kModeResid / kModeTrueRes
  const double* vj;         // kModeOuter: v_j
  const double* v0;         // kModeOuter: v_1
  int32_t s, zeta;          // sketch (s = 0: none)
  uint32_t k0, k1;          // Philox key
  const void* U;            // window base (same type as val), column-major
  int64_t ldu;
  int32_t l0, nwin;         // window columns [l0, l0 + nwin)
  double* part;             // gridDim.x rows of E doubles
  int32_t E;
  DevCtl* ctl;
  double* out0;             // ticket outputs (see modes)
  HostStatus* hs;           // device pointer of the host status block
};

// Number of Philox blocks needed for zeta nonzeros per column.
inline int zeta_blocks(int zeta) { return (zeta + 3) / 4; }

hipError_t launch_tiles(const int32_t* row_ptr, int64_t n, int64_t nnz, int32_t wt,
                        int32_t* tiles, int32_t ntiles, hipStream_t st);
hipError_t launch_spmv(int mode, bool fp32, int grid, const SpmvArgs& a, hipStream_t st);

// Reduce-then-decide kernel (sketched QR step and its variants).
enum RqMode : int {
  kRqStep = 0,    // reduce c_i, window dots, ||w||^2; Householder update; ICE; C1-C3
  kRqInit = 1,    // reduce d0 = S v_j; reset the inner-cycle state
  kRqReduce = 2,  // reduce into out_c / out_dots / out_norm2 only (test export)
};

struct RqArgs {
  const double* part;
  int32_t G, E;             // partial rows and stride
  int32_t s, m, t, nwin, l0;
  int32_t step;             // kRqStep: 0-based inner step i
  int32_t forced_k;         // kRqInit: replay dimension for the coming cycle (0 = off)
  double inv_sqrt_zeta;
  DevCtl* ctl;
  HostStatus* hs;
  double* red;              // reduced entries (E)
  double* V;                // s x m Householder vectors (column-major)
  double* T;                // m x m compact-WY factor (row-major)
  double* R;                // m x m triangular factor (column-major)
  double* d;                // s: Q^T S v_j
  double* tau;
  double* ice_x;
  double* ice_z;
  double* sigma;            // basis scales
  double* coef;             // kMaxT: window coefficients for the Arnoldi update
  double* out_c;            // kRqReduce
  double* out_dots;
  double* out_norm2;
};

hipError_t launch_rq(int mode, const RqArgs& a, hipStream_t st);

// Vector kernels (vec.hip).
hipError_t launch_init_ctl(DevCtl* ctl, int32_t m, int32_t t, int32_t s, double cond_threshold,
                           double tol, hipStream_t st);
hipError_t launch_arnoldi_update(bool fp32, int grid, int64_t n, const void* W, void* B,
                                 int64_t ldb, int32_t l0, int32_t nwin, int32_t inext,
                                 const double* coef, double* sigma, double* part, DevCtl* ctl,
                                 HostStatus* hs, int32_t step, hipStream_t st);
hipError_t launch_mgs(int grid, int64_t n, double* W, const double* Vcur, const double* Vnext,
                      const double* hcur, double* hout, double* part, DevCtl* ctl, int last,
                      double* H, double* HR, double* cs, double* sn, double* g, int32_t j,
                      int32_t ldh, HostStatus* hs, hipStream_t st);
hipError_t launch_normalize_sketch(bool fp32, int grid, int64_t n, const double* W,
                                   const double* hptr, double* Vout, void* Bout, int32_t s,
                                   int32_t zeta, uint32_t k0, uint32_t k1, double* part,
                                   int32_t E, hipStream_t st);
hipError_t launch_finalize(const DevCtl* ctl, const double* R, const double* d,
                           const double* sigma, int32_t m, double* y, hipStream_t st);
hipError_t launch_combine(bool fp32, int64_t n, const void* B, int64_t ldb, const double* y,
                          const int32_t* kdev, int32_t khost, const double* add,
                          double* out, hipStream_t st);
hipError_t launch_backsolve(const double* HR, const double* g, int32_t J, int32_t ldh,
                            double* y, hipStream_t st);
hipError_t launch_cast_f32(const double* src, float* dst, int64_t count, hipStream_t st);
hipError_t launch_copy_or_zero(const double* src, double* dst, int64_t n, hipStream_t st);
hipError_t launch_gradient(const int32_t* row_ptr, const int32_t* col_idx, int64_t n,
                           const double* lam, const double* x, double* grad, hipStream_t st);
hipError_t launch_transpose(const int32_t* row_ptr, const int32_t* col_idx, const double* val,
                            int64_t n, int64_t nnz, int32_t* rp_t, int32_t* col_t,
                            double* val_t, int32_t* perm, int32_t* cursor, int32_t* scan_tmp,
                            hipStream_t st);
hipError_t launch_sketch_materialize(int64_t n, int32_t s, int32_t zeta, uint32_t k0,
                                     uint32_t k1, int32_t* rows, int8_t* signs,
                                     hipStream_t st);

size_t transpose_scan_tmp_ints(int64_t n);

}  // namespace sfg
