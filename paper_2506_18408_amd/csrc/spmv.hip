// Fused SpMV kernels: y = A u with the sketch S y, the truncated-Arnoldi
// dot products and the squared norm computed in the same pass (the inner
// step of sketched GMRES, Section 3 with the sketch and truncated Arnoldi of
// Section 4.1), plus the outer-loop variants of Algorithm 1 (A z_j with the
// first Gram-Schmidt dot; the initial residual b - A x0; a true residual),
// the generation of the packed sketch, and the detection and copy of a
// matrix whose nonzeros lie on a few diagonals.
//
// Design (gfx950): a persistent grid of at most one workgroup per CU (248:
// one CU per XCD stays free for the decision kernel on its own stream), of
// as many waves as the LDS holds (16; fewer for large sketches and wide
// windows); every wave walks its own sequence of tiles (every nw-th tile of
// its workgroup's contiguous, XCD-grouped range) without any workgroup
// barrier.  A tile is 64 rows (one per lane) when every row has at most 8
// nonzeros, else about 256 nonzeros.  Per wave the tiles form a software
// pipeline: while tile i is reduced, the column indices of tile i+2 and the
// values, x gathers and epilogue inputs of tile i+1 are in flight, and the
// wave waits once per tile.  General tiles stage their products in the
// wave's own LDS region and reduce each row with a group of 1..64 lanes;
// short-row tiles with FP32 values stage indices and values instead and
// let every lane gather x for its own row; a matrix copied by diagonal is
// read without indices, one row per lane, every diagonal's values and x
// entries as coalesced runs.  The row's lane then runs the
// epilogue: store, scatter +-y_r into the wave's own LDS sketch
// accumulators (the zeta rows and signs of column r of S come from the
// packed sketch, or are generated) and accumulate the dot products in
// registers.  At the end
// the workgroup adds its wave copies in wave order and writes one row of
// sketch partials and one row of scalar partials; later kernels combine the
// rows in a fixed order, so results do not depend on timing.  Waves lower
// their issue priority as they progress, so that the oldest wave of a SIMD
// does not finish far ahead of the youngest while the final barrier waits.
// At t = 0 the kernel forms its own scale sigma_i = 1/||u_i|| from the
// previous step's norm partials; an FP64 matrix far beyond the last-level
// cache is read through a streaming-load instance (irregular rows) or has
// its sketch columns generated in the kernel (short rows).
#include <hip/hip_ext.h>

#include <algorithm>

#include "kernels.hpp"

namespace sfg {

// Tile boundaries: tiles[b] = first row of tile b, tp[b] = row_ptr[tiles[b]].
// rows_per_tile > 0: fixed row count; else the first row whose first nonzero
// index is >= b * wt.
__global__ void k_tiles(const int32_t* __restrict__ row_ptr, int64_t n, int32_t wt,
                        int32_t rows_per_tile, int32_t* __restrict__ tiles,
                        int32_t* __restrict__ tp, int32_t ntiles) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > ntiles) return;
  int64_t row;
  if (b == 0) {
    row = 0;
  } else if (b == ntiles) {
    row = n;
  } else if (rows_per_tile > 0) {
    row = b * rows_per_tile < n ? b * rows_per_tile : n;
  } else {
    const int64_t target = b * (int64_t)wt;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)row_ptr[mid] < target)
        lo = mid + 1;
      else
        hi = mid;
    }
    row = lo;
  }
  tiles[b] = (int32_t)row;
  tp[b] = row_ptr[row];
}

hipError_t launch_tiles(const int32_t* row_ptr, int64_t n, int32_t wt, int32_t rows_per_tile,
                        int32_t* tiles, int32_t* tp, int32_t ntiles, hipStream_t st) {
  const int threads = 256;
  const int blocks = (int)((ntiles + 1 + threads - 1) / threads);
  hipLaunchKernelGGL(k_tiles, dim3(blocks), dim3(threads), 0, st, row_ptr, n, wt, rows_per_tile,
                     tiles, tp, ntiles);
  return hipGetLastError();
}

// Longest row: per-workgroup maxima, then one workgroup takes the maximum.
__global__ __launch_bounds__(256) void k_rowlen_part(const int32_t* __restrict__ row_ptr,
                                                     int64_t n, int32_t* __restrict__ part) {
  __shared__ int32_t sm[256];
  int32_t mx = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const int32_t len = row_ptr[r + 1] - row_ptr[r];
    mx = len > mx ? len : mx;
  }
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o && sm[threadIdx.x + o] > sm[threadIdx.x]) sm[threadIdx.x] = sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(256) void k_rowlen_final(const int32_t* __restrict__ part, int32_t G,
                                                      int32_t* __restrict__ out) {
  __shared__ int32_t sm[256];
  int32_t mx = 0;
  for (int i = threadIdx.x; i < G; i += blockDim.x) mx = part[i] > mx ? part[i] : mx;
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o && sm[threadIdx.x + o] > sm[threadIdx.x]) sm[threadIdx.x] = sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

// Bandwidth max |i - j| over the nonzeros (per-workgroup maxima, then one
// workgroup; the final kernel of the row lengths takes the maximum).
__global__ __launch_bounds__(256) void k_band_part(const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col_idx, int64_t n,
                                                   int32_t* __restrict__ part) {
  __shared__ int32_t sm[256];
  int32_t mx = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    for (int q = row_ptr[r]; q < row_ptr[r + 1]; ++q) {
      const int64_t d = (int64_t)col_idx[q] - r;
      const int32_t ad = (int32_t)(d < 0 ? -d : d);
      mx = ad > mx ? ad : mx;
    }
  }
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o && sm[threadIdx.x + o] > sm[threadIdx.x]) sm[threadIdx.x] = sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

hipError_t launch_max_bandwidth(const int32_t* row_ptr, const int32_t* col_idx, int64_t n,
                                int32_t* part, int32_t* out, hipStream_t st) {
  const int g = vec_grid(n);
  hipLaunchKernelGGL(k_band_part, dim3(g), dim3(256), 0, st, row_ptr, col_idx, n, part);
  hipLaunchKernelGGL(k_rowlen_final, dim3(1), dim3(256), 0, st, part, g, out);
  return hipGetLastError();
}

hipError_t launch_max_rowlen(const int32_t* row_ptr, int64_t n, int32_t* part, int32_t* out,
                             hipStream_t st) {
  const int g = vec_grid(n);
  hipLaunchKernelGGL(k_rowlen_part, dim3(g), dim3(256), 0, st, row_ptr, n, part);
  hipLaunchKernelGGL(k_rowlen_final, dim3(1), dim3(256), 0, st, part, g, out);
  return hipGetLastError();
}

// ------------------------------------------------------- diagonal storage
// Detection: the offsets j - i of the first row of the longest length are
// the candidates; every nonzero is checked against them.  work[0] = that
// row, work[1] = 1 if some nonzero lies off the candidates, work[2] = the
// number of candidates, work[3 ..] = the candidates (increasing: the row's
// columns are sorted).
__global__ void k_dia_init(int32_t* work) {
  work[0] = 0x7FFFFFFF;
  work[1] = 0;
  work[2] = 0;
}

__global__ void k_dia_pick(const int32_t* __restrict__ row_ptr, int64_t n, int32_t len,
                           int32_t* work) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride)
    if (row_ptr[r + 1] - row_ptr[r] == len) {
      atomicMin(&work[0], (int32_t)r);
      return;  // (a later row of this thread cannot be smaller)
    }
}

__global__ void k_dia_cand(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                           int32_t* work) {
  const int r = work[0];
  const int q0 = row_ptr[r], q1 = row_ptr[r + 1];
  const int cnt = q1 - q0 < kDiaMax ? q1 - q0 : kDiaMax;
  work[2] = cnt;
  for (int k = 0; k < cnt; ++k) work[3 + k] = col_idx[q0 + k] - r;
}

__global__ void k_dia_check(const int32_t* __restrict__ row_ptr,
                            const int32_t* __restrict__ col_idx, int64_t n, int32_t* work) {
  const int cnt = work[2];
  int32_t off[kDiaMax];
#pragma unroll
  for (int k = 0; k < kDiaMax; ++k) off[k] = k < cnt ? work[3 + k] : 0x7FFFFFFF;
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n && !bad; r += stride)
    for (int q = row_ptr[r]; q < row_ptr[r + 1]; ++q) {
      const int64_t d = (int64_t)col_idx[q] - r;
      bool hit = false;
#pragma unroll
      for (int k = 0; k < kDiaMax; ++k) hit |= k < cnt && d == off[k];
      if (!hit) bad = true;
    }
  if (bad) atomicOr(&work[1], 1);
}

hipError_t launch_dia_detect(const int32_t* row_ptr, const int32_t* col_idx, int64_t n,
                             int32_t maxlen, int32_t* work, hipStream_t st) {
  const int g = vec_grid(n);
  hipLaunchKernelGGL(k_dia_init, dim3(1), dim3(1), 0, st, work);
  hipLaunchKernelGGL(k_dia_pick, dim3(g), dim3(256), 0, st, row_ptr, n, maxlen, work);
  hipLaunchKernelGGL(k_dia_cand, dim3(1), dim3(1), 0, st, row_ptr, col_idx, work);
  hipLaunchKernelGGL(k_dia_check, dim3(g), dim3(256), 0, st, row_ptr, col_idx, n, work);
  return hipGetLastError();
}

// Values by diagonal: thread per row, each diagonal's entry found among the
// row's (at most kShortRow) nonzeros, 0 where the row has none.
__global__ void k_dia_fill(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                           const double* __restrict__ val, int64_t n, int64_t ld, int32_t nd,
                           DiaOffsets offs, double* __restrict__ dia64,
                           float* __restrict__ dia32) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const int q0 = row_ptr[r], q1 = row_ptr[r + 1];
    for (int d = 0; d < nd; ++d) {
      const int64_t c = r + offs.off[d];
      double v = 0.0;
      for (int q = q0; q < q1; ++q)
        if (col_idx[q] == c) v = val[q];
      if (dia64) dia64[(int64_t)d * ld + r] = v;
      if (dia32) dia32[(int64_t)d * ld + r] = static_cast<float>(v);
    }
  }
}

hipError_t launch_dia_fill(const int32_t* row_ptr, const int32_t* col_idx, const double* val,
                           int64_t n, int64_t ld, int32_t nd, const DiaOffsets& offs,
                           double* dia64, float* dia32, hipStream_t st) {
  hipLaunchKernelGGL(k_dia_fill, dim3(vec_grid(n)), dim3(256), 0, st, row_ptr, col_idx, val, n, ld,
                     nd, offs, dia64, dia32);
  return hipGetLastError();
}

// LDS stage of one wave, in doubles.  General tiles: the staged products
// (padded so that a row's first kShortRow products can be read without a
// bound).  Short-row tiles (FP32 values): the column indices, then the
// values, each padded the same way.  Diagonal storage: none.
constexpr int kGenStage = kWStage + kShortRow;
constexpr int kShortStage = (kGenStage * 4 + kGenStage * 4) / 8;
__host__ __device__ constexpr int stage_doubles(bool short_tiles, bool dia = false) {
  if (dia) return 0;
  return short_tiles ? kShortStage : kGenStage;
}
// Doubles of LDS per wave: the stage, then, when sketching, the s sketch
// accumulators.
__host__ __device__ constexpr int wave_lds_doubles(int s, bool short_tiles, bool dia = false) {
  return stage_doubles(short_tiles, dia) + (s > 0 ? s : 0);
}

// s_waitcnt operand that waits for every outstanding vector memory access
// only (gfx9 encoding: vmcnt 0, expcnt 7, lgkmcnt 15).
constexpr int kWaitVmem0 = 0x0F70;

// Ordering of a wave's own LDS accesses across lanes (the hardware runs a
// wave's LDS instructions in order; this keeps the compiler from moving
// accesses across the point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Wide windows (NW > 4) hold twice the window registers: 12 waves at most,
// so the compiler has 168 registers per lane instead of 128 (no spills).
template <int NW>
constexpr int spmv_max_threads() { return NW > 4 ? 12 * kWave : kSpmvMaxThreads; }

// How the inner SpMV reads its operands (an instance parameter): cached
// matrix loads and the packed sketch; streaming matrix loads (a matrix that
// cannot stay in the last-level cache); cached loads with the sketch
// columns generated in the epilogue's prefetch; or the matrix by diagonal
// (no column indices) with the packed or the generated sketch.
constexpr int kLdCached = 0;
constexpr int kLdStream = 1;
constexpr int kLdGen = 2;
constexpr int kLdDia = 3;
constexpr int kLdDiaGen = 4;

// A matrix load: cached, or streaming (NT) for a matrix that cannot stay in
// the last-level cache.
template <bool NT, typename T>
__device__ __forceinline__ T mat_load(const T* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

template <typename VT, int ZB, int MODE, int NW, int LD>
__global__ __launch_bounds__(spmv_max_threads<NW>()) void k_spmv(SpmvArgs a) {
  constexpr bool NT = LD == kLdStream;
  constexpr bool kGen = LD == kLdGen || LD == kLdDiaGen;
  constexpr bool kDia = LD == kLdDia || LD == kLdDiaGen;
  static_assert(!kGen || (ZB == 1 && MODE == kModeInner), "generated sketch: zeta <= 8");
  static_assert(!kDia || (ZB > 0 && MODE == kModeInner), "diagonal storage: inner SpMV");
  constexpr bool kSketch = ZB > 0;
  constexpr bool kInnerLike = (MODE == kModeInner || MODE == kModePlain || MODE == kModePowers);
  constexpr bool kPowers = MODE == kModePowers;
  constexpr int kU = kWStage / kWave;
  // per wave: the products of its tile, then (sketching) its s accumulators
  extern __shared__ double lds[];

  // (a launch past the cycle's stop does nothing; the flag is tested once
  // this wave's first tile bounds are in flight)
  const int stop_k = MODE == kModeInner ? a.ctl->stop_k : 0;

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);  // (uniform: scalar loop control)
  const int nw = blockDim.x / kWave;
  const int S = kSketch ? a.s : 0;
  const int zeta = a.zeta;
  // (the short-row path pays for itself with FP32 values only: staging FP64
  // values doubles its LDS traffic, and their row-wise reads conflict)
  const bool short_tiles = sizeof(VT) == 4 && a.short_tiles != 0;
  const int stage = stage_doubles(short_tiles, kDia);
  const int wstride = wave_lds_doubles(S, short_tiles, kDia);
  double* const prod = lds + (size_t)wv * wstride;
  double* const wave_sk = prod + stage;
  // this wave's tiles: workgroups take contiguous ranges (XCD-grouped);
  // inside a range the waves take every nw-th tile, so the waves of a CU
  // work on neighbouring tiles at the same time (shared DRAM pages and
  // cached x entries)
  int G = gridDim.x;
  int g = xcd_logical_block(blockIdx.x, G);
  int tile0 = 0, ntiles = a.ntiles;
  const void* xin = a.x;
  void* wout = a.w;
  double* part_row = a.part + (int64_t)blockIdx.x * (kSketch ? a.s : 0);
  double* dpart_row = a.dpart + (int64_t)blockIdx.x * kDP;
  bool accumulate = false;
  if constexpr (kPowers) {
    // (XCD-grouped logical ids: each task group spans whole XCDs when the
    // grid is a multiple of 8 ptasks)
    const int gp = G / a.ptasks;
    const int task = g / gp;
    const PowTask& T = a.ptask[task < a.ptasks ? task : a.ptasks - 1];
    if (task >= a.ptasks || !T.active) return;
    const int gi = g - task * gp;
    tile0 = T.tile0;
    ntiles = T.ntiles;
    xin = T.x;
    wout = T.w;
    part_row = T.part + (int64_t)gi * a.s;
    dpart_row = T.dpart + (int64_t)gi * kDP;
    accumulate = !T.first;
    G = gp;
    g = gi;
  }
  const int t0 = tile0 + (int)(((int64_t)ntiles * g) / G) + wv;
  const int t1 = tile0 + (int)(((int64_t)ntiles * (g + 1)) / G);

  const int32_t* __restrict__ row_ptr = a.row_ptr;
  const int32_t* __restrict__ col_idx = a.col_idx;
  const VT* __restrict__ val = static_cast<const VT*>(a.val);
  const VT* __restrict__ x = static_cast<const VT*>(xin);
  VT* __restrict__ w = static_cast<VT*>(wout);
  const VT* __restrict__ U = static_cast<const VT*>(a.U);
  const bool has_x = (MODE != kModeResid) || a.has_x;
  // (t = 0 has no window: only the NW = 0 instances carry the sigma path)
  const bool sig_here = MODE == kModeInner && NW == 0 && a.sig_part != nullptr;
  double scale = (MODE == kModePlain)                 ? a.scale_val
                 : (MODE == kModeInner && !sig_here) ? (a.scale_ptr ? *a.scale_ptr : 1.0)
                                                     : 1.0;
  const int nwin = NW < a.nwin ? NW : a.nwin;

  if (kSketch)
    for (int q = lane; q < S; q += kWave) wave_sk[q] = 0.0;

  double dacc[NW > 0 ? NW : 1];
#pragma unroll
  for (int l = 0; l < (NW > 0 ? NW : 1); ++l) dacc[l] = 0.0;
  double n2 = 0.0, ex = 0.0;

  // inputs of the epilogue of row r, independent of the row sum
  struct Pre {
    VT u[NW > 0 ? NW : 1];  // (converted at use, so the loads stay in flight)
    SkGroup sk[ZB > 0 ? ZB : 1];
    double b0, b1;
  };
  auto load_pre = [&](int r, Pre& p) {
    if constexpr (kInnerLike) {
#pragma unroll
      for (int l = 0; l < NW; ++l)
        p.u[l] = l < nwin ? U[(int64_t)(a.l0 + l) * a.ldu + r] : VT(0);
      if constexpr (kGen) {
        p.sk[0] = sketch_group8((uint32_t)r, a.s, a.zeta, a.sk_k0, a.sk_k1);
      } else {
#pragma unroll
        for (int b = 0; b < ZB; ++b) p.sk[b] = a.skp[(int64_t)r * ZB + b];
      }
    } else if constexpr (MODE == kModeOuter) {
      p.b0 = a.v0[r];
      p.b1 = a.vj[r];
    } else {
      p.b0 = a.b[r];
    }
  };
  auto epilogue = [&](int r, double y, const Pre& p) {
    if constexpr (kInnerLike) {
      const VT wvv = static_cast<VT>(scale * y);
      if (w) w[r] = wvv;
      const double wd = static_cast<double>(wvv);
      if constexpr (kSketch) {
#pragma unroll
        for (int b = 0; b < ZB; ++b) {
#pragma unroll
          for (int e = 0; e < kSkGroup; ++e) {
            if (b * kSkGroup + e < zeta) {  // (uniform)
              const double av = sk_neg(p.sk[b], e) ? -wd : wd;
              __hip_atomic_fetch_add(&wave_sk[sk_row(p.sk[b], e)], av, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
            }
          }
        }
      }
#pragma unroll
      for (int l = 0; l < NW; ++l) dacc[l] += wd * static_cast<double>(p.u[l]);
      n2 += wd * wd;
    } else if constexpr (MODE == kModeOuter) {
      w[r] = static_cast<VT>(y);
      dacc[0] += y * p.b0;
      const double dl = p.b1 - y;
      ex += dl * dl;
    } else if constexpr (MODE == kModeResid) {
      const double br = p.b0;
      const double wr = br - y;
      w[r] = static_cast<VT>(wr);
      n2 += wr * wr;
      ex += br * br;
    } else {  // kModeTrueRes
      const double wr = p.b0 - y;
      n2 += wr * wr;
    }
  };

  // Software pipeline over this wave's tiles; iteration i reduces tile i
  // while the column indices of tile i+2, the values and x entries of tile
  // i+1 and the epilogue inputs of tile i+1 are in flight.  Every request is made a whole iteration before its first use,
  // so a wave waits once per tile.  All lanes load (indices clamped into the
  // tile), so no load sits behind a lane-divergent branch.
  struct TileB {
    int r0, r1, p0, L;
  };
  // the bounds of this wave's tiles, 64 at a time: lane j holds those of its
  // tile 64 c + j; taken with readlane.  A chunk is loaded where nothing else
  // is outstanding and waited for at once, so the common path never waits.
  int ch_r0 = 0, ch_r1 = 0, ch_p0 = 0, ch_p1 = 0;
  const int nt = t0 < t1 ? (t1 - t0 + nw - 1) / nw : 0;
  auto request_chunk = [&](int c) {
    int tj = t0 + (c * kWave + lane) * nw;
    tj = tj < t1 ? tj : t1 - 1;
    ch_r0 = a.tiles[tj];
    ch_r1 = a.tiles[tj + 1];
    ch_p0 = a.tp[tj];
    ch_p1 = a.tp[tj + 1];
  };
  auto load_chunk = [&](int c) {
    request_chunk(c);
    __builtin_amdgcn_s_waitcnt(kWaitVmem0);
  };
  auto tile_bounds = [&](int j) {
    TileB bt;
    bt.r0 = __builtin_amdgcn_readlane(ch_r0, j & 63);
    bt.r1 = __builtin_amdgcn_readlane(ch_r1, j & 63);
    bt.p0 = __builtin_amdgcn_readlane(ch_p0, j & 63);
    bt.L = __builtin_amdgcn_readlane(ch_p1, j & 63) - bt.p0;
    return bt;
  };
  auto staged = [&](const TileB& bt) { return has_x && bt.L > 0 && bt.L <= kWStage; };
  int ci[kU];
  VT vg[kU], xg[kU];
  // (full blocks of 64 entries at fixed offsets from one address; the last,
  // partial block with its index clamped into the tile).  Ordinary loads: the
  // matrix is read again by every inner step, and the chip's last-level
  // cache keeps much of it between steps; streaming (non-temporal) loads
  // made each FP64 step ~10% slower.  A matrix far larger than that cache
  // with irregular rows (NT, chosen by the host) takes streaming loads: it
  // cannot stay resident, and cached loads of it would evict the x entries
  // its random gathers reuse (1M power-law rows, FP64: -5% per solve).
  auto fetch = [&](const TileB& bt) {  // column indices
    if (!staged(bt)) return;
    const int32_t* cb = col_idx + bt.p0 + lane;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if ((u + 1) * kWave <= bt.L) {
        ci[u] = mat_load<NT>(cb + u * kWave);
      } else if (u * kWave < bt.L) {
        const int q = u * kWave + lane;
        ci[u] = mat_load<NT>(&col_idx[bt.p0 + (q < bt.L ? q : bt.L - 1)]);
      }
    }
  };
  auto gather = [&](const TileB& bt) {  // values and x entries
    if (!staged(bt)) return;
    const VT* vb = val + bt.p0 + lane;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if ((u + 1) * kWave <= bt.L) {
        vg[u] = mat_load<NT>(vb + u * kWave);
        xg[u] = x[ci[u]];
      } else if (u * kWave < bt.L) {
        const int q = u * kWave + lane;
        vg[u] = mat_load<NT>(&val[bt.p0 + (q < bt.L ? q : bt.L - 1)]);
        xg[u] = x[ci[u]];
      }
    }
  };
  // rows of a tile: groups of gsz lanes, one row per group at a time
  auto group_size = [&](int nrows) {
    int gsz = 1;
    while (gsz < kWave && nrows * gsz * 2 <= kWave) gsz <<= 1;
    return gsz;
  };
  // epilogue inputs of the first row of this lane's group
  struct Epi {
    Pre pre;
    int q0, q1;
  };
  Epi ecur{};
  auto epi_load = [&](const TileB& bt) {
    const int nrows = bt.r1 - bt.r0;
    if (nrows <= 0 || bt.L > kWStage) return;
    const int grp = lane / group_size(nrows);
    const int r = bt.r0 + (grp < nrows ? grp : nrows - 1);
    ecur.q0 = row_ptr[r];
    ecur.q1 = row_ptr[r + 1];
    load_pre(r, ecur.pre);
  };
  auto reduce = [&](const TileB& bt) {
    const int r0 = bt.r0, r1 = bt.r1, p0 = bt.p0, L = bt.L;
    if (r0 >= r1) return;
    if (L <= kWStage) {
      const int nrows = r1 - r0;
      const int gsz = group_size(nrows);
      const int ngroups = kWave / gsz;
      const int grp = lane / gsz;
      const int gl = lane & (gsz - 1);
      auto row_sum = [&](int qa, int qe) {
        double acc = 0.0;
        if (!has_x) return acc;
        if (gsz == 1) {
          // the first kShortRow products requested together (the stage is
          // padded by kShortRow), added in order
          double v[kShortRow];
#pragma unroll
          for (int k = 0; k < kShortRow; ++k) v[k] = prod[qa + k];
#pragma unroll
          for (int k = 0; k < kShortRow; ++k)
            if (qa + k < qe) acc += v[k];
          for (int q = qa + kShortRow; q < qe; ++q) acc += prod[q];
          return acc;
        }
        for (int q = qa + gl; q < qe; q += gsz) acc += prod[q];
        for (int off = gsz >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        return acc;
      };
      if (grp < nrows) {
        const double acc = row_sum(ecur.q0 - p0, ecur.q1 - p0);
        if (gl == 0) epilogue(r0 + grp, acc, ecur.pre);
      }
      for (int rr = grp + ngroups; rr < nrows; rr += ngroups) {  // (only with > 64 rows)
        const int r = r0 + rr;
        Pre pre;
        if (gl == 0) load_pre(r, pre);
        const double acc = row_sum(row_ptr[r] - p0, row_ptr[r + 1] - p0);
        if (gl == 0) epilogue(r, acc, pre);
      }
    } else {
      // a tile whose rows exceed the stage: the whole wave per row
      for (int r = r0; r < r1; ++r) {
        double acc = 0.0;
        if (has_x) {
          const int qa = row_ptr[r];
          const int qe = row_ptr[r + 1];
          for (int q = qa + lane; q < qe; q += kWave)
            acc += static_cast<double>(val[q]) * static_cast<double>(x[col_idx[q]]);
        }
        acc = wave_sum(acc);
        if (lane == 0) {
          Pre pre;
          load_pre(r, pre);
          epilogue(r, acc, pre);
        }
      }
    }
  };

  // t = 0 after a cycle's first step: sigma_i = 1/||u_i|| from the previous
  // step's norm partials, requested before this wave's first tile bounds and
  // summed by every wave in one fixed order (lane, then the wave's DPP
  // tree), so that all waves hold the same value.  It replaces a
  // one-workgroup kernel between the two SpMVs.
  double sgp[kSigLoads];
  if (sig_here) {
#pragma unroll
    for (int u = 0; u < kSigLoads; ++u) {
      const int g = lane + u * kWave;
      sgp[u] = a.sig_part[(int64_t)(g < a.sig_G ? g : a.sig_G - 1) * kDP + kMaxT];
    }
  }
  if (nt > 0) request_chunk(0);
  if (stop_k != 0) {
    __builtin_amdgcn_s_waitcnt(kWaitVmem0);  // (no load left in flight at exit)
    return;
  }
  if (sig_here) {
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < kSigLoads; ++u) v += lane + u * kWave < a.sig_G ? sgp[u] : 0.0;
    const double n2 = wave_sum(v);
    scale = n2 == 0.0 ? 0.0 : 1.0 / sqrt(n2);
    if (blockIdx.x == 0 && tid == 0) {
      *a.sig_out = scale;
      if (n2 == 0.0 && a.ctl->brk_step < 0) a.ctl->brk_step = a.sig_step;  // u_step = 0
    }
  }
  // Wave pacing.  At equal priority a SIMD issues for its oldest wave
  // first, so the waves of a workgroup finish in order of age (for the
  // 128^3 stencil the last group of four 12 us after the first, while the
  // barrier below waits for all of them).  A wave starts at priority 3 and
  // steps down after 1/4, 1/2 and 3/4 of its tiles, so waves that are
  // ahead yield to those behind.  The tile assignment is unchanged.
  __builtin_amdgcn_s_setprio(3);
  int pstage = 0;
  auto pace = [&](int i) {
    const int st = (4 * i >= nt) + (2 * i >= nt) + (4 * i >= 3 * nt);
    if (st != pstage) {
      pstage = st;
      if (st == 1)
        __builtin_amdgcn_s_setprio(2);
      else if (st == 2)
        __builtin_amdgcn_s_setprio(1);
      else
        __builtin_amdgcn_s_setprio(0);
    }
  };
  if constexpr (kDia) {
    // Diagonal storage, tiles of kRowTile rows (one row per lane): the
    // values and x entries of every diagonal arrive as coalesced runs, and
    // there are no column indices to read.  The row sum is formed in the
    // row's column order (offsets increasing) from the same products as the
    // CSR paths form (FP64: each product rounded before it is added, as the
    // staged products; FP32: as the short-row path), so y, and with the same
    // tiles and lanes everything after it, equals the CSR path's bit for
    // bit.  Entries off the matrix hold 0 and add nothing.  Pipeline: the
    // loads of tile i+1 are in flight while tile i is summed and its
    // epilogue runs.
    const VT* __restrict__ dv = static_cast<const VT*>(a.dia_val);
    const int64_t dld = a.dia_ld;
    const int nd = a.ndiag;
    const int64_t nlast = a.n - 1;
    VT fv[kDiaMax], fx[kDiaMax];
    Pre fpre{};
    int fr0 = 0, frows = 0;
    auto dia_fetch = [&](const TileB& bt) {
      fr0 = bt.r0;
      frows = bt.r1 - bt.r0;
      const int r = bt.r0 + (lane < frows ? lane : frows - 1);
#pragma unroll
      for (int d = 0; d < kDiaMax; ++d)
        if (d < nd) {
          fv[d] = dv[(int64_t)d * dld + r];
          int64_t c = (int64_t)r + a.dia_off[d];
          c = c < 0 ? 0 : (c > nlast ? nlast : c);
          fx[d] = x[c];
        }
      load_pre(r, fpre);
    };
    if (nt > 0) {
      __builtin_amdgcn_s_waitcnt(kWaitVmem0);  // (the first chunk, requested above)
      dia_fetch(tile_bounds(0));
    }
    for (int i = 0; i < nt; ++i) {
      pace(i);
      __builtin_amdgcn_s_waitcnt(kWaitVmem0);
      if (i + 1 < nt && ((i + 1) & 63) == 0) load_chunk((i + 1) >> 6);
      VT cv[kDiaMax], cx[kDiaMax];
#pragma unroll
      for (int d = 0; d < kDiaMax; ++d) {
        cv[d] = fv[d];
        cx[d] = fx[d];
      }
      const Pre pre = fpre;
      const int r0 = fr0, nrows = frows;
      if (i + 1 < nt) dia_fetch(tile_bounds(i + 1));
      double acc = 0.0;
      if constexpr (sizeof(VT) == 8) {
        // (the CSR path rounds each product into its LDS stage before the
        // row sum: no fused multiply-add here either)
#pragma clang fp contract(off)
#pragma unroll
        for (int d = 0; d < kDiaMax; ++d)
          if (d < nd) {
            const double pr = static_cast<double>(cv[d]) * static_cast<double>(cx[d]);
            acc += pr;
          }
      } else {
        // (as the short-row path: the product and the add in one statement)
#pragma unroll
        for (int d = 0; d < kDiaMax; ++d)
          if (d < nd) acc += static_cast<double>(cv[d]) * static_cast<double>(cx[d]);
      }
      if (lane < nrows) epilogue(r0 + lane, acc, pre);
    }
  } else if (short_tiles && has_x) {
    // Short-row tiles (at most kRowTile rows of at most kShortRow nonzeros):
    // the column indices and values arrive coalesced, in nonzero order, and
    // are staged in LDS; every lane then reads its own row back and gathers
    // x for it, so gather k of the wave fetches entry k of 64 consecutive
    // rows (for a stencil, one contiguous run of x per offset).  The row sum
    // is formed in registers in nonzero order.  Pipeline as in the general
    // case: the indices, values and row bounds of tile i+2, the x entries
    // and epilogue inputs of tile i+1 are in flight while tile i finishes.
    int* const cis = reinterpret_cast<int*>(prod);
    VT* const vls = reinterpret_cast<VT*>(cis + kGenStage);
    int fq0 = 0, fq1 = 0;       // row bounds of this lane's row, fetched tile
    int q0c = 0, q1c = 0;       // ... of the tile being gathered / reduced
    int lmax = 0;               // longest row of the gathered tile (uniform)
    Pre epre{};                 // epilogue inputs of this lane's row
    auto pre_load = [&](const TileB& bt) {
      const int nrows = bt.r1 - bt.r0;
      load_pre(bt.r0 + (lane < nrows ? lane : nrows - 1), epre);
    };
    auto fetch_s = [&](const TileB& bt) {
      const int32_t* cb = col_idx + bt.p0 + lane;
      const VT* vb = val + bt.p0 + lane;
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if ((u + 1) * kWave <= bt.L) {
          ci[u] = *(cb + u * kWave);
          vg[u] = *(vb + u * kWave);
        } else if (u * kWave < bt.L) {
          const int q = u * kWave + lane;
          const int e = bt.p0 + (q < bt.L ? q : bt.L - 1);
          ci[u] = col_idx[e];
          vg[u] = val[e];
        }
      }
      const int nrows = bt.r1 - bt.r0;
      const int r = bt.r0 + (lane < nrows ? lane : nrows - 1);
      fq0 = row_ptr[r];
      fq1 = row_ptr[r + 1];
    };
    // fetched registers -> LDS (nonzero order), then this lane's row back
    // and its x gathers; the row bounds move along with the tile
    auto stage_gather = [&](const TileB& bt) {
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (u * kWave < bt.L) {
          cis[u * kWave + lane] = ci[u];
          vls[u * kWave + lane] = vg[u];
        }
      }
      q0c = fq0 - bt.p0;
      q1c = fq1 - bt.p0;
      int len = q1c - q0c;
      // (the longest row of the tile bounds the gathers every lane makes)
      int m = len;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(m, off, kWave);
        m = o > m ? o : m;
      }
      lmax = __builtin_amdgcn_readfirstlane(m);
      wave_sync();
      const int c0 = cis[q0c];
#pragma unroll
      for (int k = 0; k < kShortRow; ++k) {
        if (k < lmax) {
          const int ck = cis[q0c + k];
          xg[k] = x[k < len ? ck : c0];  // (past the row's end: its first entry again)
        }
      }
    };
    TileB bc{}, bg{}, bf{};
    if (nt > 0) {
      __builtin_amdgcn_s_waitcnt(kWaitVmem0);  // (the first chunk, requested above)
      bg = tile_bounds(0);
      fetch_s(bg);
      __builtin_amdgcn_s_waitcnt(kWaitVmem0);
      stage_gather(bg);
      pre_load(bg);
    }
    if (nt > 1) {
      bf = tile_bounds(1);
      fetch_s(bf);
    }
    for (int i = 0; i < nt; ++i) {
      pace(i);
      __builtin_amdgcn_s_waitcnt(kWaitVmem0);
      if (i + 2 < nt && ((i + 2) & 63) == 0) load_chunk((i + 2) >> 6);
      bc = bg;
      const int nrows = bc.r1 - bc.r0;
      // the row sum of this lane's row, entries in order
      double v[kShortRow];
#pragma unroll
      for (int k = 0; k < kShortRow; ++k) v[k] = static_cast<double>(vls[q0c + k]);
      double acc = 0.0;
      const int len = q1c - q0c;
#pragma unroll
      for (int k = 0; k < kShortRow; ++k)
        if (k < lmax && k < len) acc += v[k] * static_cast<double>(xg[k]);
      const Pre pre = epre;
      wave_sync();  // the stage is read: the next tile may overwrite it
      if (i + 1 < nt) {
        bg = bf;
        stage_gather(bg);
        pre_load(bg);
      }
      if (lane < nrows) epilogue(bc.r0 + lane, acc, pre);
      if (i + 2 < nt) {
        bf = tile_bounds(i + 2);
        fetch_s(bf);
      }
      wave_sync();
    }
  } else {
    TileB bc{}, bg{}, bf{};
    if (nt > 0) {
      __builtin_amdgcn_s_waitcnt(kWaitVmem0);  // (the first chunk, requested above)
      bg = tile_bounds(0);
      fetch(bg);
      gather(bg);
      epi_load(bg);
    }
    if (nt > 1) {
      bf = tile_bounds(1);
      fetch(bf);
    }
    for (int i = 0; i < nt; ++i) {
      pace(i);
      // the one wait of the iteration: every request of the previous one
      // (vector memory count 0; export and LDS/scalar counts left alone)
      __builtin_amdgcn_s_waitcnt(kWaitVmem0);
      if (i + 2 < nt && ((i + 2) & 63) == 0) load_chunk((i + 2) >> 6);
      bc = bg;
      if (staged(bc)) {
  #pragma unroll
        for (int u = 0; u < kU; ++u)
          if (u * kWave < bc.L)
            prod[u * kWave + lane] = static_cast<double>(vg[u]) * static_cast<double>(xg[u]);
      }
      if (i + 1 < nt) {
        bg = bf;
        gather(bg);
      }
      if (i + 2 < nt) {
        bf = tile_bounds(i + 2);
        fetch(bf);
      }
      wave_sync();
      reduce(bc);
      if (i + 1 < nt) epi_load(bg);
      wave_sync();
    }

  }

  // One sketch row and one scalar row of partial sums per workgroup (fixed
  // slot = blockIdx.x).  Each wave reduces its scalar partials as soon as
  // its own tiles are done (the waves of a workgroup finish at different
  // times), so a single barrier remains; after it the wave sums, and the
  // wave copies of the sketch, are added in wave order: the order of a
  // block-wide sum.
  constexpr int kNS = kInnerLike ? NW + 1 : 2;  // scalar sums per wave
  static_assert(kSpmvLdsMax + kSpmvMaxWaves * kNS * 8 <= 160 * 1024, "LDS of one CU");
  __shared__ double wsums[kSpmvMaxWaves * kNS];
  {
    double sv[kNS];
    if constexpr (kInnerLike) {
#pragma unroll
      for (int l = 0; l < NW; ++l) sv[l] = l < nwin ? wave_sum(dacc[l]) : 0.0;
      sv[kNS - 1] = wave_sum(n2);
    } else {
      sv[0] = wave_sum(MODE == kModeOuter ? dacc[0] : n2);
      sv[1] = wave_sum(ex);
    }
    if (lane == 0)
#pragma unroll
      for (int i = 0; i < kNS; ++i) wsums[wv * kNS + i] = sv[i];
  }
  __syncthreads();
  if constexpr (kSketch) {
    double* prow = part_row;
    for (int q = tid; q < S; q += blockDim.x) {
      const double* sk0 = lds + stage + q;  // wave 0's copy
      double v = sk0[0];
      for (int k = 1; k < nw; ++k) v += sk0[(size_t)k * wstride];
      prow[q] = accumulate ? prow[q] + v : v;
    }
  }
  if (tid < kNS) {
    double r = 0.0;
    for (int k = 0; k < nw; ++k) r += wsums[k * kNS + tid];
    if (accumulate && tid == kNS - 1) r += dpart_row[kMaxT];
    double* drow = dpart_row;
    if (!kInnerLike)
      drow[kMaxT + tid] = r;  // (reference or outer dot, then the second sum)
    else if (tid == kNS - 1)
      drow[kMaxT] = r;        // ||w||^2
    else if (tid < nwin)
      drow[tid] = r;          // window dots
  }
}

struct LaunchCfg {
  int grid;
  int waves;
  size_t lds;
  hipStream_t st;
  hipEvent_t ev0, ev1;
};

template <typename VT, int ZB, int MODE, int NW, int LD>
static hipError_t launch_ld(const LaunchCfg& c, const SpmvArgs& a) {
  static bool attr_set = false;  // dynamic LDS above the default limit
  if (!attr_set) {
    const hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spmv<VT, ZB, MODE, NW, LD>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kSpmvLdsMax);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const dim3 block(c.waves * kWave);
  if (c.ev0)
    hipExtLaunchKernelGGL((k_spmv<VT, ZB, MODE, NW, LD>), dim3(c.grid), block, c.lds, c.st,
                          c.ev0, c.ev1, 0, a);
  else
    hipLaunchKernelGGL((k_spmv<VT, ZB, MODE, NW, LD>), dim3(c.grid), block, c.lds, c.st, a);
  return hipGetLastError();
}

// (only the FP64 inner SpMV has streaming-load and generated-sketch
// instances)
template <typename VT, int ZB, int MODE, int NW>
static hipError_t launch_one(const LaunchCfg& c, const SpmvArgs& a) {
  if constexpr (MODE == kModeInner && ZB > 0) {
    if (a.ndiag > 0) {
      if constexpr (sizeof(VT) == 8 && ZB == 1)
        if (a.sketch_gen) return launch_ld<VT, ZB, MODE, NW, kLdDiaGen>(c, a);
      return launch_ld<VT, ZB, MODE, NW, kLdDia>(c, a);
    }
  }
  if constexpr (sizeof(VT) == 8 && MODE == kModeInner) {
    if (a.stream_matrix) return launch_ld<VT, ZB, MODE, NW, kLdStream>(c, a);
    if constexpr (ZB == 1)
      if (a.sketch_gen) return launch_ld<VT, ZB, MODE, NW, kLdGen>(c, a);
  }
  return launch_ld<VT, ZB, MODE, NW, kLdCached>(c, a);
}

template <typename VT, int MODE, int NW>
static hipError_t launch_spmv_zb(int zb, LaunchCfg c, const SpmvArgs& a) {
  const bool short_tiles = sizeof(VT) == 4 && a.short_tiles != 0;
  const bool dia = MODE == kModeInner && zb > 0 && a.ndiag > 0;
  const size_t per_wave =
      (size_t)wave_lds_doubles(zb > 0 ? a.s : 0, short_tiles, dia) * sizeof(double);
  c.waves = std::min(spmv_waves(zb > 0 ? a.s : 0, short_tiles, dia), spmv_max_threads<NW>() / kWave);
  c.lds = per_wave * c.waves;
  switch (zb) {
    case 0:
      return launch_one<VT, 0, MODE, NW>(c, a);
    case 1:
      return launch_one<VT, 1, MODE, NW>(c, a);
    default:
      return launch_one<VT, 2, MODE, NW>(c, a);
  }
}

template <typename VT, int MODE>
static hipError_t launch_spmv_nw(int zb, const LaunchCfg& c, const SpmvArgs& a) {
  if (a.nwin <= 0) return launch_spmv_zb<VT, MODE, 0>(zb, c, a);
  if (a.nwin <= 2) return launch_spmv_zb<VT, MODE, 2>(zb, c, a);
  if (a.nwin <= 4) return launch_spmv_zb<VT, MODE, 4>(zb, c, a);
  return launch_spmv_zb<VT, MODE, kMaxT>(zb, c, a);
}

// (the largest count that fits: 14 waves rather than 8 for s = 800)
int spmv_waves(int s, bool short_tiles, bool dia) {
  const size_t per_wave = (size_t)wave_lds_doubles(s, short_tiles, dia) * sizeof(double);
  const size_t fit = (size_t)kSpmvLdsMax / per_wave;
  return (int)std::max<size_t>(1, std::min<size_t>(kSpmvMaxWaves, fit));
}

hipError_t launch_spmv(int mode, bool fp32, int grid, const SpmvArgs& a, int zb, hipStream_t st,
                       hipEvent_t ev0, hipEvent_t ev1) {
  const LaunchCfg c{grid, 0, 0, st, ev0, ev1};
  switch (mode) {
    case kModeInner:
      return fp32 ? launch_spmv_nw<float, kModeInner>(zb, c, a)
                  : launch_spmv_nw<double, kModeInner>(zb, c, a);
    case kModePlain:
      return launch_spmv_nw<double, kModePlain>(zb, c, a);
    case kModePowers:
      return launch_spmv_zb<double, kModePowers, 0>(zb, c, a);
    case kModeOuter:
      return launch_spmv_zb<double, kModeOuter, 1>(0, c, a);
    case kModeResid:
      return launch_spmv_zb<double, kModeResid, 0>(0, c, a);
    default:
      return launch_spmv_zb<double, kModeTrueRes, 0>(0, c, a);
  }
}

// ---------------------------------------------------------------- finisher
constexpr int kFinishThreads = 256;

__global__ __launch_bounds__(kFinishThreads) void k_spmv_finish(int mode, const double* dpart,
                                                              int32_t G, DevCtl* c,
                                                              double* out0, HostStatus* hs) {
  __shared__ double scratch[kFinishThreads / kWave];
  const double t0s = block_sum_strided(dpart + kMaxT, G, kDP, scratch);
  const double t1s = block_sum_strided(dpart + kMaxT + 1, G, kDP, scratch);
  if (threadIdx.x != 0) return;
  if (mode == kModeOuter) {
    out0[0] = t0s;  // h_{1,j}
    c->rhat2 = t1s;
  } else if (mode == kModeResid) {
    const double beta = sqrt(t0s);
    const double nb = sqrt(t1s);
    c->beta = beta;
    c->nb = nb;
    c->factor = beta;
    c->tol_abs = c->tol_abs * nb;  // tol_abs held the relative tol until here
    out0[0] = beta;                // g_1 = beta
    if (!isfinite(beta) || !isfinite(nb)) c->error = SFGMRES_ERR_NONFINITE;
    host_store_f64(&hs->beta, beta);
    host_store_f64(&hs->nb, nb);
    host_store_i32(&hs->error, c->error);
  } else if (mode == kModeRestart) {
    // a restart of restarted sGMRES: the new residual norm, which is also
    // the next cycle's C3 factor (||b|| and the tolerance are set already)
    const double beta = sqrt(t0s);
    c->beta = beta;
    c->factor = beta;
    out0[0] = beta;
    if (!isfinite(beta) && c->error == 0) c->error = SFGMRES_ERR_NONFINITE;
    host_store_f64(&hs->beta, beta);
    host_store_i32(&hs->error, c->error);
    // the finished cycle's summary (the FGMRES path publishes it with its
    // last Gram-Schmidt pass)
    const bool c2 = c->stop_reason == SFGMRES_STOP_C2;
    host_store_i32(&hs->k, c->stop_k);
    host_store_i32(&hs->stop_reason, c->stop_reason);
    host_store_f64(&hs->cond, c2 ? c->cond_prev : c->cond_cur);
    host_store_f64(&hs->rho_hat, c2 ? c->rho_prev : c->rho_cur);
  } else {
    out0[0] = t0s;
  }
}

hipError_t launch_spmv_finish(int mode, const double* dpart, int32_t G, DevCtl* ctl,
                              double* out0, HostStatus* hs, hipStream_t st) {
  hipLaunchKernelGGL(k_spmv_finish, dim3(1), dim3(kFinishThreads), 0, st, mode, dpart, G, ctl,
                     out0, hs);
  return hipGetLastError();
}

// ------------------------------------------------------------ packed sketch
// (ZB Philox blocks of four entries generate a column; it is stored as
// sk_groups(zeta) packed groups)
template <int ZB>
__global__ void k_sketch_pack(int64_t n, int32_t s, int32_t zeta, uint32_t k0, uint32_t k1,
                              SkGroup* __restrict__ skp) {
  constexpr int kG = (4 * ZB + kSkGroup - 1) / kSkGroup;
  const int ng = sk_groups(zeta);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    int rows[4 * ZB];
    uint32_t neg;
    sketch_column<ZB>((uint32_t)r, s, zeta, k0, k1, rows, neg);
#pragma unroll
    for (int b = 0; b < kG; ++b) {
      if (b >= ng) break;
      skp[r * ng + b] = sk_pack(rows, neg, zeta, b);
    }
  }
}

hipError_t launch_sketch_pack(int64_t n, int32_t s, int32_t zeta, uint32_t k0, uint32_t k1,
                              SkGroup* skp, hipStream_t st) {
  const int grid = vec_grid(n);
  switch (zeta_blocks(zeta)) {
    case 1:
      hipLaunchKernelGGL(k_sketch_pack<1>, dim3(grid), dim3(256), 0, st, n, s, zeta, k0, k1, skp);
      break;
    case 2:
      hipLaunchKernelGGL(k_sketch_pack<2>, dim3(grid), dim3(256), 0, st, n, s, zeta, k0, k1, skp);
      break;
    case 3:
      hipLaunchKernelGGL(k_sketch_pack<3>, dim3(grid), dim3(256), 0, st, n, s, zeta, k0, k1, skp);
      break;
    default:
      hipLaunchKernelGGL(k_sketch_pack<4>, dim3(grid), dim3(256), 0, st, n, s, zeta, k0, k1, skp);
      break;
  }
  return hipGetLastError();
}

__global__ void k_sketch_identity(int64_t n, SkGroup* __restrict__ skp) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const uint32_t row = (uint32_t)r;  // (n <= SFGMRES_MAX_S: 11 bits)
    SkGroup q{{row & 0xFFu, 0u, (row >> 8) & 7u}};
    skp[r] = q;
  }
}

hipError_t launch_sketch_identity(int64_t n, SkGroup* skp, hipStream_t st) {
  hipLaunchKernelGGL(k_sketch_identity, dim3(vec_grid(n)), dim3(256), 0, st, n, skp);
  return hipGetLastError();
}

__global__ void k_sketch_unpack(int64_t n, int32_t zeta, const SkGroup* __restrict__ skp,
                                int32_t* __restrict__ rows, int8_t* __restrict__ signs) {
  const int ng = sk_groups(zeta);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    for (int d = 0; d < zeta; ++d) {
      const SkGroup q = skp[r * ng + d / kSkGroup];
      rows[r * zeta + d] = (int32_t)sk_row(q, d % kSkGroup);
      signs[r * zeta + d] = sk_neg(q, d % kSkGroup) ? (int8_t)-1 : (int8_t)1;
    }
  }
}

hipError_t launch_sketch_unpack(int64_t n, int32_t zeta, const SkGroup* skp, int32_t* rows,
                                int8_t* signs, hipStream_t st) {
  hipLaunchKernelGGL(k_sketch_unpack, dim3(vec_grid(n)), dim3(256), 0, st, n, zeta, skp, rows,
                     signs);
  return hipGetLastError();
}

}  // namespace sfg
