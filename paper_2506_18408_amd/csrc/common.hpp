// Internal definitions shared by the sketched-FGMRES HIP kernels and the host
// driver: device control block, host-visible status block, workspace layout,
// the Philox4x32-10 generator, the sketch column definition, the packed
// sketch format and block reductions.  gfx950 only (64-lane wavefronts).
//
// Cross-workgroup reductions never use a "last workgroup finishes" ticket:
// on a multi-XCD part every agent-scope fence writes back and invalidates
// the workgroup's L2, which costs more than the reduction.  Every multi-
// workgroup kernel writes one row of partial results per workgroup, and a
// later kernel (a one-workgroup finisher, or the consumer itself) sums the
// rows in slot order, so results are also reproducible bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sfgmres.h"

namespace sfg {

constexpr int kWave = 64;
constexpr int kMaxT = SFGMRES_MAX_T;
constexpr int kMaxZeta = SFGMRES_MAX_ZETA;
constexpr int kMaxS = SFGMRES_MAX_S;
constexpr int kMaxM = SFGMRES_MAX_M;

// Fused SpMV: a persistent grid of at most kSpmvGrid workgroups (one per
// CU) of up to kSpmvMaxWaves waves; every wave walks its own range of tiles
// with no workgroup barrier.  A tile holds at most kWStage nonzeros: kRowTile
// rows (one per lane) when every row has at most kShortRow nonzeros, else
// about kTileNnz nonzeros, which with rows of at most kWStage - kTileNnz + 1
// nonzeros always fit the stage (longer rows take a slower per-row path).
constexpr int kSpmvMaxWaves = 16;
constexpr int kSpmvMaxThreads = kSpmvMaxWaves * 64;
constexpr int kSpmvGrid = 248;  // one CU per XCD left for the decision kernel
constexpr int kWStage = 512;
constexpr int kShortRow = 8;
constexpr int kRowTile = kWStage / kShortRow;
constexpr int kTileNnz = kWStage / 2;
// A matrix of more bytes than this per SpMV (well beyond the chip's 256 MB
// last-level cache) whose rows are too long for short-row tiles is read by
// the FP64 inner SpMV with streaming loads, so that it does not evict the x
// entries its gathers reuse.
constexpr size_t kStreamMatrixBytes = (size_t)300 << 20;
// An FP64 matrix of more bytes than this per SpMV (twice the last-level
// cache) with short rows has its inner SpMV generate the sketch columns
// (Philox + Floyd, zeta <= 8) instead of reading the packed table: the
// FP64 stream leaves the vector units idle long enough to hide the
// generator, and the 12 bytes per row of the table are saved.  (The FP32
// stream and cache-resident matrices are faster with the table.)
constexpr size_t kGenSketchBytes = (size_t)512 << 20;
// Dynamic LDS of one SpMV workgroup (bytes): with the kernel's static LDS
// (the per-wave scalar sums, at most 16 x 9 doubles) within the CU's 160 KB.
// 15 waves of s = 800 fit instead of 14 (-1.5% per 256^3 FP64 launch).
constexpr int kSpmvLdsMax = 158 * 1024;
// Bound on the number of partial rows any multi-workgroup kernel writes.
constexpr int kMaxGrid = 1024;
// Vector kernels: threads per workgroup and grid cap (one partial per
// workgroup in the vector partial buffer).
constexpr int kVecThreads = 256;
constexpr int kVecGrid = 1024;
constexpr int kArnoldiGrid = 512;  // (<= kVecGrid)
// Partial sums written by every multi-workgroup kernel, one row per
// workgroup (slot = blockIdx.x):
//   sketch rows: s accumulators (sum of +-w_r, unscaled), row stride s;
//   scalar rows: kDP doubles, row stride kDP:
//     [0, kMaxT)   dot products
//     kMaxT        squared norm
//     kMaxT + 1    second squared norm / extra scalar
constexpr int kDP = kMaxT + 2;
// Columns appended to the sketched QR by one decision launch (at most).
constexpr int kPanel = 8;

// Packed sketch: the zeta entries (row in [0, s), s <= 1024, and sign) of
// column r of S in ceil(zeta/8) groups of eight 12-bit fields, three 32-bit
// words per group (12 bytes for zeta <= 8).  Field e of a group: row bits
// 0..7 in byte e%4 of word e/4; row bits 8..10 and the sign (bit 3 set:
// negative) in the 4-bit nibble e of word 2.  Fields past zeta are zero and
// are skipped by every reader (zeta is uniform over a launch).
constexpr int kSkGroup = 8;
struct SkGroup {
  uint32_t w[3];
};
__host__ __device__ inline int sk_groups(int zeta) { return (zeta + kSkGroup - 1) / kSkGroup; }
__host__ __device__ inline int sk_row(const SkGroup& g, int e) {
  return (int)(((g.w[e >> 2] >> ((e & 3) * 8)) & 0xFFu) | (((g.w[2] >> (e * 4)) & 7u) << 8));
}
__host__ __device__ inline bool sk_neg(const SkGroup& g, int e) {
  return ((g.w[2] >> (e * 4)) & 8u) != 0;
}

// Device control block (lives in the workspace).  Scalars are written by
// one-workgroup kernels only.
struct DevCtl {
  // inner cycle
  int32_t stop_k;        // 0 while the cycle runs, else the chosen dimension k_j
  int32_t stop_step;     // inner step at which the stop was decided
  int32_t stop_reason;   // SFGMRES_STOP_*
  int32_t qr_k;          // columns in the sketched QR
  int32_t forced_k;      // >0: replay this dimension
  int32_t m, t, s;
  int32_t error;         // 0, or a negative SFGMRES_ERR_* raised on the device
  int32_t brk_step;      // inner step whose Arnoldi vector is zero (-1: none)
  double tol_abs;        // tol * ||b||
  double cond_threshold;
  double factor;         // C3 factor: FFOM residual of the previous outer step (beta at j = 1)
  double ice_smax;       // incremental condition estimate state
  double ice_znorm;
  double cond_cur, cond_prev;
  double rho_cur, rho_prev;   // sketched inner residuals at steps i and i-1
  double d0norm;
  // outer
  double beta, nb;
  double rhat2;          // ||v_j - A z_j||^2
  double rho;            // |g_{j+1}|
  double ffom;
  double hnext;          // h_{j+1,j}
  double cs_last;
  double bound;          // eq. (2.2) at the last outer step: ||r~_{j-1}|| ||v_j - A z_j||
  double delta;          // eq. (2.3): delta_j (0 before the first outer step)
  double ffom_g;         // last outer step: g_j before its own rotation (FFOM right side)
  double ffom_piv;       // ... and the pivot of column j before that rotation (H_j's R)
};

// Host-visible status block (pinned, device-mapped).
struct HostStatus {
  int32_t inner_step_done;   // last inner step whose decision kernel finished
  int32_t stop_k;            // mirror of DevCtl::stop_k
  int32_t stop_step;
  int32_t stop_reason;
  int32_t outer_j;           // outer step recorded below (1-based)
  int32_t k;
  int32_t error;
  int32_t steps_run;         // inner steps fully executed by the cycle that stopped
  double rho, ffom, hnext, cond, rho_hat, rhat_true, beta, nb, bound, delta;
};

// Offsets (bytes) of every workspace region.
struct Layout {
  size_t ctl, tiles, tp, ipart, part, dpart, vpart, red, skp, qr_V, qr_T, qr_R, qr_d, qr_c, qr_tau, ice_x, ice_z,
      sigma, hwin, yin, H, HR, cs, sn, g, yout, V, Z, B, W32, W64, X, val32, dia, dia_work, ilu,
      ilu_t64, ilu_tmp,
      mid, mid_bytes, at_rowptr, at_col, at_val, at_perm, at_cursor, scan_tmp, total;
  int64_t ld;        // leading dimension (elements) of the n-vectors
  int64_t ntiles_max;
  int32_t grid;      // persistent grid size used for the partial buffer
};


// Bytes of the packed sketch of an n-column S with zeta nonzeros per column.
inline size_t packed_sketch_bytes(int64_t n, int32_t zeta) {
  return (size_t)n * (size_t)sk_groups(zeta) * sizeof(SkGroup);
}

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon et al., SC'11): four 32-bit counter words, two key
// words, ten rounds of two 32x32->64 multiplies, Weyl key bumps.
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c0;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

// Column `col` of the sparse sign sketch: rows[d] (distinct, in [0, s)) and
// negative-sign flags for d < zeta.  ZB = number of Philox blocks generated
// (zeta <= 4 ZB).  Random word d comes from block d/4, output d%4, counter
// (col, block, 0, 0); Floyd's sampling: i = s - zeta + d,
// t = ((w >> 1) * (i + 1)) >> 31, take i if t is already chosen; the sign
// is negative when w is odd.
template <int ZB>
__device__ __forceinline__ void sketch_column(uint32_t col, int s, int zeta, uint32_t k0,
                                              uint32_t k1, int (&rows)[4 * ZB],
                                              uint32_t& negmask) {
  uint32_t w[4 * ZB];
#pragma unroll
  for (int b = 0; b < ZB; ++b) {
    uint32_t c0 = col, c1 = (uint32_t)b, c2 = 0u, c3 = 0u;
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    w[4 * b + 0] = c0;
    w[4 * b + 1] = c1;
    w[4 * b + 2] = c2;
    w[4 * b + 3] = c3;
  }
  negmask = 0u;
#pragma unroll
  for (int d = 0; d < 4 * ZB; ++d) {
    if (d < zeta) {
      const uint32_t i = (uint32_t)(s - zeta + d);
      const uint64_t u = (uint64_t)(w[d] >> 1);
      int t = (int)((u * (uint64_t)(i + 1u)) >> 31);
      bool taken = false;
#pragma unroll
      for (int e = 0; e < d; ++e) taken |= (rows[e] == t);
      rows[d] = taken ? (int)i : t;
      negmask |= (w[d] & 1u) << d;
    } else {
      rows[d] = -1;
    }
  }
}

// Packed group b of a column from its rows and sign flags (the fields of
// SkGroup: row bits 0-7 in bytes of w[0..1], row bits 8-10 and the sign in
// the nibbles of w[2]).
template <int NR>
__device__ __forceinline__ SkGroup sk_pack(const int (&rows)[NR], uint32_t neg, int zeta, int b) {
  SkGroup q{{0u, 0u, 0u}};
#pragma unroll
  for (int e = 0; e < kSkGroup; ++e) {
    const int d = kSkGroup * b + e;
    if (d < zeta && d < NR) {
      const uint32_t row = (uint32_t)rows[d];
      q.w[e >> 2] |= (row & 0xFFu) << ((e & 3) * 8);
      q.w[2] |= (((row >> 8) & 7u) | (((neg >> d) & 1u) << 3)) << (e * 4);
    }
  }
  return q;
}

// The single packed group of column `col` for zeta <= 8 (two Philox
// blocks), generated where it is used: equal to what the packing kernel
// stores for that column.
__device__ __forceinline__ SkGroup sketch_group8(uint32_t col, int s, int zeta, uint32_t k0,
                                                 uint32_t k1) {
  int rows[8];
  uint32_t neg;
  sketch_column<2>(col, s, zeta, k0, k1, rows, neg);
  return sk_pack(rows, neg, zeta, 0);
}

// Scatter of v (the value of entry `col` of a vector) into the s LDS
// accumulators through column col of the packed sketch (ZB groups).  Every
// wave owns a private copy of the s accumulators (a workgroup sums its
// copies in wave order at the end), so the order of the additions into one
// accumulator depends only on the static row-to-lane assignment and the
// sketch of a vector is reproducible bit for bit from run to run.
template <int ZB>
__device__ __forceinline__ void sketch_scatter_packed(double* lds_sk, const SkGroup* __restrict__ skp,
                                                      int zeta, int64_t col, double v) {
#pragma unroll
  for (int b = 0; b < ZB; ++b) {
    const SkGroup q = skp[col * ZB + b];
#pragma unroll
    for (int e = 0; e < kSkGroup; ++e) {
      if (b * kSkGroup + e < zeta) {
        const double a = sk_neg(q, e) ? -v : v;
        __hip_atomic_fetch_add(&lds_sk[sk_row(q, e)], a, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
}

// ------------------------------------------------------------- reductions
// A lane-to-lane move of a double with a DPP pattern (the two 32-bit halves
// moved separately).
template <int kCtrl>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xFFFFFFFFll), kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 64 lanes of a wave; every lane gets the same value.  Within
// each row of 16 lanes: exchange with lane^1 and lane^2 (quad permutes), then
// add the values 4 and 8 lanes along (row rotations), which leaves the row
// sum in lane 0 of the row; the four row sums are then read as scalars and
// added in row order.  No LDS traffic; the order is fixed, so the result is
// reproducible bit for bit.  Must be called with all 64 lanes active.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x124>(v);  // row_ror:4
  v += dpp_move<0x128>(v);  // row_ror:8
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Sum of v over the workgroup (fixed order: waves combined in wave order).
// `scratch` holds blockDim.x/64 doubles.  Every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < nw; ++i) r += scratch[i];
  __syncthreads();
  return r;
}

// Sums of NV values over the workgroup at once (fixed order, as block_sum);
// every thread gets the NV sums.  `buf` holds (blockDim.x/64) * NV doubles.
template <int NV>
__device__ __forceinline__ void block_sum_vec(double (&v)[NV], double* buf) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) buf[wid * NV + i] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double r = 0.0;
    for (int w = 0; w < nw; ++w) r += buf[w * NV + i];
    v[i] = r;
  }
  __syncthreads();
}

// Sum of src[0], src[stride], ..., src[(count-1) stride] by one workgroup
// in a fixed order (thread-strided partial sums, then block_sum).
__device__ __forceinline__ double block_sum_strided(const double* src, int count, int64_t stride,
                                                    double* scratch) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) acc += src[(int64_t)i * stride];
  return block_sum(acc, scratch);
}

// Persistent-grid logical block id: consecutive hardware workgroup ids are
// dealt round-robin to the 8 XCDs, so give each XCD a contiguous range of
// logical ids (and hence of rows / tiles) to keep gathers inside one L2.
__device__ __forceinline__ int xcd_logical_block(int b, int nb) {
  constexpr int kXcd = 8;
  if (nb % kXcd != 0) return b;
  return (b % kXcd) * (nb / kXcd) + b / kXcd;
}

// Stores into the pinned host status block (system scope).
__device__ __forceinline__ void host_store_i32(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void host_store_f64(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                     (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_SYSTEM);
}

}  // namespace sfg
