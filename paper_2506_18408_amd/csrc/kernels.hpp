// Launcher interface between the host driver (solver.hip) and the kernel
// translation units (spmv.hip, qr.hip, vec.hip).  Every launcher enqueues on
// `st` and returns the hipError_t of the launch.
#pragma once

#include <string>

#include "common.hpp"

namespace sfg {

enum SpmvMode : int {
  kModeInner = 0,    // y = sigma A u ; S y ; <y, U_l> ; ||y||^2  (predicated on the stop flag)
  kModeOuter = 1,    // w = A z ; <w, v_1> ; ||v_j - w||^2
  kModeResid = 2,    // w = b - A x ; ||w||^2 ; ||b||^2
  kModeTrueRes = 3,  // ||b - A x||^2
  kModePlain = 4,    // as kModeInner with a scale, without predication (test export)
  kModeRestart = 5,  // finisher only: beta = ||b - A x|| of a restart (kModeResid SpMV)
  kModePowers = 6,   // matrix powers: y_l = A y_{l-1} on one slab of rows per task group
};

// Matrix powers (kModePowers): the grid is split into ptasks groups of
// workgroups; group l computes the rows of one slab of y_{l+1} = A y_l (its
// tiles [tile0, tile0 + ntiles)), when active, and adds its sketch and
// squared-norm partials to the rows of its level (overwriting them when
// `first`, the level's first slab).
constexpr int kMaxPowTasks = 8;
struct PowTask {
  int32_t tile0, ntiles;
  int32_t active, first;
  const void* x;
  void* w;
  double* part;    // the level's sketch partial rows (one per workgroup of the group)
  double* dpart;   // the level's scalar partial rows
};

// Diagonals of a matrix the inner SpMV reads by diagonal (diagonal storage
// for stencil-like patterns: at most kDiaMax distinct offsets j - i, rows of
// at most kShortRow nonzeros).
constexpr int kDiaMax = 8;
struct DiaOffsets {
  int32_t off[kDiaMax];
};
hipError_t launch_dia_detect(const int32_t* row_ptr, const int32_t* col_idx, int64_t n,
                             int32_t maxlen, int32_t* work, hipStream_t st);
hipError_t launch_dia_fill(const int32_t* row_ptr, const int32_t* col_idx, const double* val,
                           int64_t n, int64_t ld, int32_t nd, const DiaOffsets& offs,
                           double* dia64, float* dia32, hipStream_t st);

struct SpmvArgs {
  int64_t n;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const void* val;          // double* (FP64) or float* (mixed inner)
  const int32_t* tiles;     // ntiles+1 row boundaries
  const int32_t* tp;        // ntiles+1 first nonzero of each tile
  int32_t ntiles;
  int32_t short_tiles;      // 1: tiles of kRowTile rows, every row at most kShortRow nonzeros
  int32_t has_x;            // kModeResid: 0 means x = 0
  int32_t stream_matrix;    // kModeInner, FP64 values: read the matrix with streaming loads
  const void* x;            // input vector, same type as val
  const double* scale_ptr;  // kModeInner: device scalar sigma (NULL: 1)
  double scale_val;         // kModePlain: w = scale * A u
  void* w;                  // output vector, same type as val (NULL = not written)
  const double* b;          // kModeResid / kModeTrueRes
  const double* vj;         // kModeOuter: v_j
  const double* v0;         // kModeOuter: v_1
  int32_t s;                // sketch rows (0: no sketch)
  int32_t zeta;             // nonzeros per sketch column
  const SkGroup* skp;       // packed sketch
  int32_t sketch_gen;       // kModeInner, FP64, zeta <= 8: generate the sketch columns
  // kModeInner: the matrix by diagonal (ndiag > 0): value d of row r at
  // dia_val[d * dia_ld + r] (same type as val; 0 off the matrix), column
  // r + dia_off[d]; offsets increasing
  const void* dia_val;
  int64_t dia_ld;
  int32_t ndiag;
  int32_t dia_off[kDiaMax];
  uint32_t sk_k0, sk_k1;    // the sketch's Philox key (sketch_gen)
  const void* U;            // window base (same type as val), column-major
  int64_t ldu;
  int32_t l0, nwin;         // window columns [l0, l0 + nwin)
  double* part;             // sketch rows: gridDim.x rows of s doubles
  double* dpart;            // scalar rows: gridDim.x rows of kDP doubles
  DevCtl* ctl;
  // kModeInner, t = 0 after a cycle's first step (sig_part non-NULL): the
  // scale sigma_i = 1/||u_i|| is formed from the previous step's scalar rows
  // (sig_G <= kWave * kSigLoads of them) instead of read from scale_ptr;
  // workgroup 0 stores it to sig_out and flags u_i = 0 as a breakdown at
  // sig_step.
  const double* sig_part;
  int32_t sig_G, sig_step;
  double* sig_out;
  // kModePowers
  int32_t ptasks;
  PowTask ptask[kMaxPowTasks];
};
constexpr int kSigLoads = 4;
static_assert(kSpmvGrid <= kWave * kSigLoads, "sig_part rows per lane");

// Number of Philox4x32 blocks (four entries each) that generate one sketch
// column.
__host__ __device__ inline int zeta_blocks(int zeta) { return (zeta + 3) / 4; }

// Row tiles of the SpMV kernels (rows_per_tile > 0: fixed row count, else
// about wt nonzeros each) and the longest row (written to *out).
hipError_t launch_tiles(const int32_t* row_ptr, int64_t n, int32_t wt, int32_t rows_per_tile,
                        int32_t* tiles, int32_t* tp, int32_t ntiles, hipStream_t st);
hipError_t launch_max_rowlen(const int32_t* row_ptr, int64_t n, int32_t* part, int32_t* out,
                             hipStream_t st);
hipError_t launch_max_bandwidth(const int32_t* row_ptr, const int32_t* col_idx, int64_t n,
                                int32_t* part, int32_t* out, hipStream_t st);
// Waves per SpMV workgroup for an s-row sketch (0: none), bounded by LDS.
int spmv_waves(int s, bool short_tiles, bool dia = false);
// zb = sk_groups(zeta) with a sketch, else 0.  ev0/ev1 non-null: the launch
// records them at the kernel's own start and end (timing of the kernel alone).
hipError_t launch_spmv(int mode, bool fp32, int grid, const SpmvArgs& a, int zb, hipStream_t st,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// One-workgroup finisher of the scalar SpMV variants: sums the scalar rows
// (entries kMaxT, kMaxT+1) in slot order and records the mode's scalars.
hipError_t launch_spmv_finish(int mode, const double* dpart, int32_t G, DevCtl* ctl,
                              double* out0, HostStatus* hs, hipStream_t st);

// Sketch generation (Philox4x32-10 + Floyd) into the packed format, and its
// export as (row, sign) arrays for tests.
hipError_t launch_sketch_pack(int64_t n, int32_t s, int32_t zeta, uint32_t k0, uint32_t k1,
                              SkGroup* skp, hipStream_t st);
// The identity as a packed sketch (zeta = 1, column r -> row r, sign +1);
// a test option that needs s == n.
hipError_t launch_sketch_identity(int64_t n, SkGroup* skp, hipStream_t st);
hipError_t launch_sketch_unpack(int64_t n, int32_t zeta, const SkGroup* skp, int32_t* rows,
                                int8_t* signs, hipStream_t st);

// Multi-workgroup reduction of sketch rows: for the ring slots
// (first + y) mod nring, y < nslots, red[slot][e] = sum over the G rows
// (stride `stride`) of part[slot][row][e], e < count, in slot order.
// Predicated on the stop flag when `predicated`.
hipError_t launch_reduce_slots(const double* part, int32_t G, int32_t stride, int32_t count,
                               int32_t first, int32_t nslots, int32_t nring, int64_t slot_part,
                               int64_t slot_red, double* red, const DevCtl* ctl, bool predicated,
                               hipStream_t st);

// Truncated-Arnoldi coefficients of inner step `step` (one workgroup): for
// t > 0 sigma_step = 1/||u_step|| (from the Arnoldi norm partials) and
// coef[l] = sigma_step sigma_l^2 <y, u_l>, coef[kMaxT] = sigma_step; for
// t = 0 sigma_{step+1} = 1/||y||.  A zero vector records its step in
// ctl->brk_step (first one only) and zero coefficients.
struct CoefArgs {
  const double* dpart;      // scalar rows of the fused SpMV (G rows of kDP)
  int32_t G;
  const double* vpart;      // t > 0, step > 0: norm partials of u_step
  int32_t Gv;
  int32_t t, nwin, l0, step;
  DevCtl* ctl;
  double* sigma;
  double* coef;             // kMaxT + 1: window coefficients, then the scale of y
};
hipError_t launch_coef(const CoefArgs& a, hipStream_t st);

// Decision kernel (one workgroup): appends columns k0 .. k0+ncols-1 to the
// sketched QR and decides after each of them.
struct QrBlockArgs {
  const double* red;        // reduced sketch rows, ring of nring slots (slot = column mod nring)
  int64_t slot_red;
  int32_t nring;
  int32_t s, m, t;
  int32_t k0, ncols;        // first column, columns in this launch (1..kPanel)
  int32_t pprev;            // columns of the previous panel whose T columns are still to form
  double inv_sqrt_zeta;
  DevCtl* ctl;
  HostStatus* hs;
  double* V;                // s x m Householder vectors (column-major, zeros above the unit)
  double* T;                // m x m compact-WY factor (column-major, upper triangle)
  double* R;                // m x m triangular factor (column-major)
  double* d;                // s: Q^T S v_j
  double* tau;
  double* ice_x;
  double* ice_z;
  const double* sigma;      // basis scales sigma_l = 1 / ||u_l||
};
size_t qr_block_lds_bytes(int32_t s, int32_t m);
hipError_t launch_qr_block(const QrBlockArgs& a, hipStream_t st);

// d = red[0:s] / sqrt(zeta) (= S v_j) and a reset of the inner-cycle state.
hipError_t launch_rq_init(const double* red, int32_t s, double inv_sqrt_zeta, int32_t forced_k,
                          DevCtl* ctl, double* d, double* sigma, hipStream_t st);

// Test export of one fused SpMV: out_c = red / sqrt(zeta), the window dots
// and the squared norm summed from the scalar rows (dpart may be NULL).
hipError_t launch_sketch_out(const double* red, int32_t s, double inv_sqrt_zeta,
                             const double* dpart, int32_t G, int32_t nwin, double* out_c,
                             double* out_dots, double* out_norm2, hipStream_t st);

// Vector kernels (vec.hip).
hipError_t launch_init_ctl(DevCtl* ctl, int32_t m, int32_t t, int32_t s, double cond_threshold,
                           double tol, hipStream_t st);
// Truncated-Arnoldi update of inner step `step` (t > 0) with its own
// coefficients (vec.hip).
struct ArnoldiArgs {
  int64_t n;
  const void* W;            // y = A u_step (same type as the basis)
  void* B;                  // basis, column-major, leading dimension ldb
  int64_t ldb;
  int32_t l0, nwin, inext, step;
  const double* dpart;      // scalar rows of the fused SpMV (Gd rows of kDP)
  int32_t Gd;
  const double* vprev;      // norm partials of u_step (Gv entries; unused at step 0)
  int32_t Gv;
  double* vnext;            // norm partials of u_{step+1} (one per workgroup)
  double* sigma;
  DevCtl* ctl;
};
hipError_t launch_arnoldi_update(bool fp32, int grid, const ArnoldiArgs& a, hipStream_t st);
hipError_t launch_mgs_pass(int grid, int64_t n, double* W, const double* Vcur,
                           const double* Vnext, const double* hcur, double* vpart, int last,
                           hipStream_t st);
hipError_t launch_mgs_finish(const double* vpart, int32_t G, double* hout, DevCtl* ctl, int last,
                             double* H, double* HR, double* cs, double* sn, double* g, int32_t j,
                             int32_t ldh, HostStatus* hs, hipStream_t st);
hipError_t launch_normalize_sketch(bool fp32, int grid, int64_t n, const double* W,
                                   const double* hptr, double* Vout, void* Bout, int32_t s,
                                   const SkGroup* skp, int32_t zeta, double* part,
                                   hipStream_t st);
hipError_t launch_finalize(const DevCtl* ctl, const double* R, const double* d,
                           const double* sigma, int32_t m, double* y, hipStream_t st);
// out = add + sum_l y_l B_l (l < k); with `scale` (device scalar) the sum is
// formed first and out = add + scale * sum.
hipError_t launch_combine(bool fp32, int64_t n, const void* B, int64_t ldb, const double* y,
                          const int32_t* kdev, int32_t khost, const double* add,
                          double* out, hipStream_t st, const double* scale = nullptr);
// (ffom_ctl non-null: the FFOM coefficients H_J^{-1} beta e1 instead)
hipError_t launch_backsolve(const double* HR, const double* g, int32_t J, int32_t ldh,
                            double* y, hipStream_t st, const DevCtl* ffom_ctl = nullptr);
hipError_t launch_cast_f32(const double* src, float* dst, int64_t count, hipStream_t st);
hipError_t launch_copy_or_zero(const double* src, double* dst, int64_t n, hipStream_t st);
hipError_t launch_gradient(const int32_t* row_ptr, const int32_t* col_idx, int64_t n,
                           const double* lam, const double* x, double* grad, hipStream_t st);
hipError_t launch_transpose(const int32_t* row_ptr, const int32_t* col_idx, const double* val,
                            int64_t n, int64_t nnz, int32_t* rp_t, int32_t* col_t,
                            double* val_t, int32_t* perm, int32_t* cursor, int32_t* scan_tmp,
                            hipStream_t st);

size_t transpose_scan_tmp_ints(int64_t n);

// Zero-fill ILU right preconditioner in a multicolour order (ilu.hip).
constexpr int kIluMaxColors = 4095;  // (12-bit colour field of the colouring state)
constexpr int kIluChunk = 8192;      // rows per wave when the rows are grouped by colour
constexpr int kIluLongRow = 32;      // longest row factored one thread per row
inline int64_t ilu_chunks(int64_t n) { return (n + kIluChunk - 1) / kIluChunk; }
// Factors for the triangular solves, by position p in the colour order
// (row order[p]): the off-diagonal entries of L in oci/oval[orp[p] ..
// omid[p]), those of U in [omid[p] .. orp[p+1]), each in the row's column
// order; U's diagonal in udiag[p].  The column of an entry is given by its
// position in the colour order too (the solves run on a work vector in that
// order).
struct IluFactors {
  const int32_t* order;      // rows by colour, increasing within a colour
  const int32_t* orp;        // n+1
  const int32_t* omid;       // n
  const int32_t* oci;
  const void* oval;          // FP32 when fp32, else FP64
  const void* udiag;
  const int32_t* level;      // host: order[level[c] .. level[c+1]) has colour c
  const int8_t* group;       // host: lanes per row in colour c, [2c] for L and [2c+1] for U
  int32_t ncolors;
  bool fp32;                 // FP32 copies of the values (mixed precision)
};
hipError_t launch_ilu_init(int64_t n, const int32_t* rp, const int32_t* ci, const double* val,
                           double* lu, int32_t* diag, int32_t* state, int32_t* err,
                           int32_t* maxrow, hipStream_t st);
hipError_t launch_ilu_jp_round(int64_t n, const int32_t* rp, const int32_t* ci,
                               const int32_t* rpt, const int32_t* cit, int32_t* state,
                               int32_t round, int32_t* colored, int32_t* err, hipStream_t st);
hipError_t launch_ilu_count(int64_t n, const int32_t* state, int32_t* cnt, hipStream_t st);
hipError_t launch_ilu_colors(int64_t n, const int32_t* state, int32_t* color, hipStream_t st);
// order: the rows grouped by colour (start[c] = first position of colour c),
// increasing within a colour; kind: per nonzero -1 (L), 0 (diagonal), +1 (U).
// hist holds nc * ilu_chunks(n) ints.
hipError_t launch_ilu_order(int64_t n, const int32_t* rp, const int32_t* ci,
                            const int32_t* state, int32_t nc, const int32_t* start,
                            int32_t* hist, int32_t* order, int8_t* kind, hipStream_t st);
hipError_t launch_ilu_factor(const int32_t* order, int32_t begin, int32_t end, const int32_t* rp,
                             const int32_t* ci, const int8_t* kind, const int32_t* diag,
                             const int32_t* state, double* lu, int32_t* err, bool wave_per_row,
                             hipStream_t st);
// The solve copies (orp, omid, oci, oval, udiag) from the factors on A's
// pattern (every row with its diagonal: nnz - n off-diagonal entries);
// lsum[c] = L entries of colour c (lsum zero on entry), usum[c] = U entries
// (nc each); pos (n ints) receives each row's position in the colour order.
hipError_t launch_ilu_split(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci,
                            const int8_t* kind, const int32_t* diag, const double* lu,
                            const int32_t* order, int32_t nc, const int32_t* start, int32_t* orp,
                            int32_t* omid, int32_t* oci, void* oval, void* udiag,
                            bool fp32_factors, int32_t* lsum, int32_t* usum, int32_t* pos,
                            int32_t* scan_tmp, hipStream_t st);
// Lanes per row for a colour whose rows hold `entries` off-diagonal entries
// of the solved factor in all.
int ilu_group(int64_t rows, int64_t entries);
// out = M^{-1} in (VT = float when fp32), through the work vector t (room
// for n doubles, used as n values of VT, in the colour order); FP32 vectors
// need the FP32 factors;
// with ctl, every launch does nothing once the inner cycle has stopped.
hipError_t launch_ilu_apply(bool fp32, const IluFactors& f, const void* in, double* t, void* out,
                            hipStream_t st, const DevCtl* ctl = nullptr);
// In-place exclusive scan of cnt[0 .. n) with the total stored to cnt[n]
// (vec.hip; scan_tmp holds transpose_scan_tmp_ints(n) ints).
hipError_t launch_exclusive_scan(int32_t* cnt, int64_t n, int32_t* scan_tmp, hipStream_t st);

// The fused SpMV export (sfgmres_spmv_sketch) on a workspace of ws_bytes
// bytes, and the bytes it needs (solver.hip).
int spmv_sketch_impl(sfgmres_ctx* h, const sfgmres_csr* A, const double* u, double scale,
                     double* w, int32_t s, int32_t zeta, uint64_t seed, const double* U,
                     int64_t ldu, int32_t nwin, double* c, double* dots, double* norm2, void* ws,
                     size_t ws_bytes, void* stream);
size_t spmv_sketch_workspace(int64_t n, int64_t nnz, int32_t s, int32_t zeta);
// Records msg as the handle's last error and returns code (solver.hip).
int report_error(sfgmres_ctx* h, int code, const std::string& msg);
int vec_grid(int64_t n);
int arnoldi_grid(int64_t n);

}  // namespace sfg
