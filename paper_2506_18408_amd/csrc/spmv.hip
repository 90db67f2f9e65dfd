// Fused CSR SpMV kernels: w = A u with the sketch S w, the truncated-Arnoldi
// dot products and squared norms computed in the same pass (the inner step of
// sketched GMRES, Section 3 with the sketch and truncated Arnoldi of
// Section 4.1), plus the outer-loop variants of Algorithm 1 (A z_j with the
// first Gram-Schmidt dot; the initial residual b - A x0; a true residual).
//
// Design (gfx950): a persistent grid of 256-thread workgroups walks
// nnz-balanced row tiles.  A tile's nonzeros are streamed with coalesced
// loads into LDS as products val*x[col] (phase A), then groups of 1..64 lanes
// reduce one row each from LDS (phase B, group width chosen per tile from its
// row count), and the row leader runs the epilogue: scale, store, scatter
// +-w_r into the workgroup's LDS sketch accumulators (zeta Floyd-sampled rows
// generated from Philox4x32-10 in registers, no sketch stored in HBM) and
// accumulate the dot products in registers.  Each workgroup finally writes one
// row of partial sums; a separate reduction (or the last workgroup, for the
// scalar-only variants) combines the rows in a fixed order.
#include "kernels.hpp"

namespace sfg {

__global__ void k_tiles(const int32_t* __restrict__ row_ptr, int64_t n, int64_t nnz, int32_t wt,
                        int32_t* __restrict__ tiles, int32_t ntiles) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > ntiles) return;
  if (b == 0) {
    tiles[0] = 0;
    return;
  }
  if (b == ntiles) {
    tiles[ntiles] = (int32_t)n;
    return;
  }
  // first row whose first nonzero index is >= b * wt
  const int64_t target = b * (int64_t)wt;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)row_ptr[mid] < target)
      lo = mid + 1;
    else
      hi = mid;
  }
  tiles[b] = (int32_t)lo;
}

hipError_t launch_tiles(const int32_t* row_ptr, int64_t n, int64_t nnz, int32_t wt,
                        int32_t* tiles, int32_t ntiles, hipStream_t st) {
  const int threads = 256;
  const int blocks = (int)((ntiles + 1 + threads - 1) / threads);
  hipLaunchKernelGGL(k_tiles, dim3(blocks), dim3(threads), 0, st, row_ptr, n, nnz, wt, tiles,
                     ntiles);
  return hipGetLastError();
}

template <typename VT, int ZB, int MODE>
__global__ __launch_bounds__(kSpmvThreads) void k_spmv(SpmvArgs a) {
  constexpr bool kSketch = ZB > 0;
  constexpr bool kInnerLike = (MODE == kModeInner || MODE == kModePlain);
  __shared__ double prod[kTileCap];
  extern __shared__ double lds_sk[];  // s doubles when sketching
  __shared__ double scratch[kSpmvThreads / kWave];
  __shared__ int lds_flag;

  if (MODE == kModeInner && a.ctl->stop_k != 0) return;

  const int tid = threadIdx.x;
  const int G = gridDim.x;
  const int g = xcd_logical_block(blockIdx.x, G);
  const int t0 = (int)(((int64_t)a.ntiles * g) / G);
  const int t1 = (int)(((int64_t)a.ntiles * (g + 1)) / G);

  const int32_t* __restrict__ row_ptr = a.row_ptr;
  const int32_t* __restrict__ col_idx = a.col_idx;
  const VT* __restrict__ val = static_cast<const VT*>(a.val);
  const VT* __restrict__ x = static_cast<const VT*>(a.x);
  VT* __restrict__ w = static_cast<VT*>(a.w);
  const VT* __restrict__ U = static_cast<const VT*>(a.U);
  const bool has_x = (MODE != kModeResid) || a.has_x;
  const double scale = kInnerLike ? (a.scale_ptr ? *a.scale_ptr : a.scale_val) : 1.0;

  if (kSketch)
    for (int q = tid; q < a.s; q += kSpmvThreads) lds_sk[q] = 0.0;

  double dacc[kMaxT];
#pragma unroll
  for (int l = 0; l < kMaxT; ++l) dacc[l] = 0.0;
  double n2 = 0.0, ex = 0.0;

  auto epilogue = [&](int r, double y) {
    if constexpr (kInnerLike) {
      const VT wv = static_cast<VT>(scale * y);
      if (w) w[r] = wv;
      const double wd = static_cast<double>(wv);
      if constexpr (kSketch) sketch_scatter<ZB>(lds_sk, (uint32_t)r, wd, a.s, a.zeta, a.k0, a.k1);
#pragma unroll
      for (int l = 0; l < kMaxT; ++l)
        if (l < a.nwin) dacc[l] += wd * static_cast<double>(U[(int64_t)(a.l0 + l) * a.ldu + r]);
      n2 += wd * wd;
    } else if constexpr (MODE == kModeOuter) {
      w[r] = static_cast<VT>(y);
      dacc[0] += y * a.v0[r];
      const double dl = a.vj[r] - y;
      ex += dl * dl;
    } else if constexpr (MODE == kModeResid) {
      const double br = a.b[r];
      const double wr = br - y;
      w[r] = static_cast<VT>(wr);
      n2 += wr * wr;
      ex += br * br;
    } else {  // kModeTrueRes
      const double wr = a.b[r] - y;
      n2 += wr * wr;
    }
  };

  __syncthreads();
  for (int tl = t0; tl < t1; ++tl) {
    const int r0 = a.tiles[tl];
    const int r1 = a.tiles[tl + 1];
    if (r0 >= r1) continue;
    const int p0 = row_ptr[r0];
    const int L = row_ptr[r1] - p0;
    if (L <= kTileCap) {
      // phase A: coalesced stream of the tile's nonzeros into LDS products
      if (has_x) {
        constexpr int kU = 8;
        for (int base = 0; base < L; base += kU * kSpmvThreads) {
          int cidx[kU];
          double vv[kU];
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int q = base + u * kSpmvThreads + tid;
            if (q < L) {
              cidx[u] = __builtin_nontemporal_load(&col_idx[p0 + q]);
              vv[u] = static_cast<double>(__builtin_nontemporal_load(&val[p0 + q]));
            }
          }
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int q = base + u * kSpmvThreads + tid;
            if (q < L) prod[q] = vv[u] * static_cast<double>(x[cidx[u]]);
          }
        }
      }
      __syncthreads();
      // phase B: groups of gsz lanes reduce one row each
      const int nrows = r1 - r0;
      int gsz = 1;
      while (gsz < kWave && nrows * gsz * 2 <= kSpmvThreads) gsz <<= 1;
      const int ngroups = kSpmvThreads / gsz;
      const int grp = tid / gsz;
      const int gl = tid & (gsz - 1);
      for (int rr = grp; rr < nrows; rr += ngroups) {
        const int r = r0 + rr;
        double acc = 0.0;
        if (has_x) {
          const int qa = row_ptr[r] - p0;
          const int qe = row_ptr[r + 1] - p0;
          for (int q = qa + gl; q < qe; q += gsz) acc += prod[q];
        }
        for (int off = gsz >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        if (gl == 0) epilogue(r, acc);
      }
      __syncthreads();
    } else {
      // tile holding a row longer than the LDS capacity: whole workgroup per row
      for (int r = r0; r < r1; ++r) {
        double acc = 0.0;
        if (has_x) {
          const int qa = row_ptr[r];
          const int qe = row_ptr[r + 1];
          for (int q = qa + tid; q < qe; q += kSpmvThreads)
            acc += static_cast<double>(val[q]) * static_cast<double>(x[col_idx[q]]);
        }
        acc = block_sum(acc, scratch);
        if (tid == 0) epilogue(r, acc);
      }
    }
  }

  // one row of partial sums per workgroup (fixed slot = blockIdx.x)
  double* prow = a.part + (int64_t)blockIdx.x * a.E;
  const int sb = kSketch ? a.s : 0;
  if constexpr (kSketch) {
    __syncthreads();
    for (int q = tid; q < a.s; q += kSpmvThreads) prow[q] = lds_sk[q];
  }
  if constexpr (kInnerLike) {
#pragma unroll
    for (int l = 0; l < kMaxT; ++l) {
      if (l < a.nwin) {
        const double v = block_sum(dacc[l], scratch);
        if (tid == 0) prow[sb + l] = v;
      }
    }
    const double v = block_sum(n2, scratch);
    if (tid == 0) prow[sb + kMaxT] = v;
    return;
  } else {
    const double s0 = block_sum(MODE == kModeOuter ? dacc[0] : n2, scratch);
    const double s1 = block_sum(ex, scratch);
    if (tid == 0) {
      prow[kMaxT] = s0;
      prow[kMaxT + 1] = s1;
    }
    if (!last_block_arrival(&a.ctl->ticket[0], G, &lds_flag)) return;
    // the last workgroup combines the scalar partials in slot order
    double t0s = 0.0, t1s = 0.0;
    for (int i = tid; i < G; i += kSpmvThreads) {
      t0s += a.part[(int64_t)i * a.E + kMaxT];
      t1s += a.part[(int64_t)i * a.E + kMaxT + 1];
    }
    t0s = block_sum(t0s, scratch);
    t1s = block_sum(t1s, scratch);
    if (tid == 0) {
      DevCtl* c = a.ctl;
      if (MODE == kModeOuter) {
        a.out0[0] = t0s;   // h_{1,j}
        c->rhat2 = t1s;
      } else if (MODE == kModeResid) {
        const double beta = sqrt(t0s);
        const double nb = sqrt(t1s);
        c->beta = beta;
        c->nb = nb;
        c->factor = beta;
        c->tol_abs = c->tol_abs * nb;  // tol_abs held the relative tol until here
        a.out0[0] = beta;              // g_1 = beta
        if (!isfinite(beta) || !isfinite(nb)) c->error = SFGMRES_ERR_NONFINITE;
        host_store_f64(&a.hs->beta, beta);
        host_store_f64(&a.hs->nb, nb);
        host_store_i32(&a.hs->error, c->error);
        __threadfence_system();
      } else {
        a.out0[0] = t0s;
      }
    }
  }
}

template <typename VT, int MODE>
static hipError_t launch_spmv_t(int zb, int grid, const SpmvArgs& a, hipStream_t st) {
  const size_t lds = zb > 0 ? (size_t)a.s * sizeof(double) : 0;
  switch (zb) {
    case 0:
      hipLaunchKernelGGL((k_spmv<VT, 0, MODE>), dim3(grid), dim3(kSpmvThreads), lds, st, a);
      break;
    case 1:
      hipLaunchKernelGGL((k_spmv<VT, 1, MODE>), dim3(grid), dim3(kSpmvThreads), lds, st, a);
      break;
    case 2:
      hipLaunchKernelGGL((k_spmv<VT, 2, MODE>), dim3(grid), dim3(kSpmvThreads), lds, st, a);
      break;
    case 3:
      hipLaunchKernelGGL((k_spmv<VT, 3, MODE>), dim3(grid), dim3(kSpmvThreads), lds, st, a);
      break;
    default:
      hipLaunchKernelGGL((k_spmv<VT, 4, MODE>), dim3(grid), dim3(kSpmvThreads), lds, st, a);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_spmv(int mode, bool fp32, int grid, const SpmvArgs& a, hipStream_t st) {
  const int zb = a.s > 0 ? zeta_blocks(a.zeta) : 0;
  switch (mode) {
    case kModeInner:
      return fp32 ? launch_spmv_t<float, kModeInner>(zb, grid, a, st)
                  : launch_spmv_t<double, kModeInner>(zb, grid, a, st);
    case kModePlain:
      return launch_spmv_t<double, kModePlain>(zb, grid, a, st);
    case kModeOuter:
      hipLaunchKernelGGL((k_spmv<double, 0, kModeOuter>), dim3(grid), dim3(kSpmvThreads), 0, st,
                         a);
      return hipGetLastError();
    case kModeResid:
      hipLaunchKernelGGL((k_spmv<double, 0, kModeResid>), dim3(grid), dim3(kSpmvThreads), 0, st,
                         a);
      return hipGetLastError();
    default:
      hipLaunchKernelGGL((k_spmv<double, 0, kModeTrueRes>), dim3(grid), dim3(kSpmvThreads), 0,
                         st, a);
      return hipGetLastError();
  }
}

}  // namespace sfg
