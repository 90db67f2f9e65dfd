// Vector kernels of the sketched-FGMRES path: the truncated-Arnoldi update
// (Section 4.1), the outer modified Gram-Schmidt passes and the Givens update
// of the Hessenberg least-squares problem (Algorithm 1), the normalisation of
// v_{j+1} fused with its sketch, the small triangular solves, the tall-skinny
// combinations z_j = B_k y and x = x0 + Z y, the float32 value cast, and the
// adjoint's CSR transpose and value gradient.
//
// Streaming loops load every input of kUnroll elements per thread before
// they compute and store, so each thread keeps several loads in flight.
#include "kernels.hpp"

namespace sfg {

constexpr int kUnroll = 4;

int vec_grid(int64_t n) {
  int64_t g = (n + kVecThreads * kUnroll - 1) / (kVecThreads * kUnroll);
  if (g > kVecGrid) g = kVecGrid;
  if (g < 1) g = 1;
  return (int)g;
}

// The Arnoldi update's grid: every workgroup sums the fused SpMV's scalar
// rows and the previous update's norm partials itself, so it runs on at most
// kArnoldiGrid workgroups of longer stretches (13.6 -> 13.0 us for the 128^3
// FP64 update against 1024 workgroups).
int arnoldi_grid(int64_t n) {
  const int g = vec_grid(n);
  return g < kArnoldiGrid ? g : kArnoldiGrid;
}

// ---------------------------------------------------------------- control
__global__ void k_init_ctl(DevCtl* c, int32_t m, int32_t t, int32_t s, double cond_threshold,
                           double tol) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  DevCtl z = {};
  z.m = m;
  z.t = t;
  z.s = s;
  z.cond_threshold = cond_threshold;
  z.tol_abs = tol;  // relative until the residual finisher multiplies by ||b||
  z.factor = INFINITY;
  *c = z;
}

hipError_t launch_init_ctl(DevCtl* ctl, int32_t m, int32_t t, int32_t s, double cond_threshold,
                           double tol, hipStream_t st) {
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(64), 0, st, ctl, m, t, s, cond_threshold, tol);
  return hipGetLastError();
}

// ------------------------------------------------ truncated Arnoldi update
// u_{i+1} = sigma_i y - sum_l sigma_i sigma_l^2 <y, u_l> u_l over the window,
// with y = A u_i and sigma_i = 1/||u_i|| (Section 4.1 with an unnormalised
// basis).  Every workgroup first forms the coefficients itself: the window
// dots from the fused SpMV's scalar rows and ||u_i||^2 from the previous
// update's norm partials, summed in the same fixed order, so all workgroups
// use bit-identical values; workgroup 0 records sigma_i, and a zero u_i as a
// truncated-Arnoldi breakdown (first one only, zero coefficients).  The
// first stretch of the vectors is requested before that reduction.  Each
// workgroup writes its partial ||u_{i+1}||^2 to vnext[blockIdx.x].
template <typename VT, int NW>
__global__ __launch_bounds__(kVecThreads) void k_arnoldi(ArnoldiArgs a) {
  constexpr int kNV = kMaxT + 1;  // window dots, then ||u_i||^2
  __shared__ double buf[(kVecThreads / kWave) * kNV];
  __shared__ double scratch[kVecThreads / kWave];
  __shared__ double cf[kMaxT + 1];
  DevCtl* ctl = a.ctl;
  const int tid = threadIdx.x;
  const int step = a.step;
  const int nwin = a.nwin < NW ? a.nwin : NW;
  const int64_t n = a.n;
  const VT* __restrict__ W = static_cast<const VT*>(a.W);
  VT* B = static_cast<VT*>(a.B);
  VT* out = B + (int64_t)a.inext * a.ldb;
  const VT* win = B + (int64_t)a.l0 * a.ldb;
  // Workgroup stretches of kS elements: the full ones at wg0 + k gstride,
  // k < nfull, then at most one partial stretch.  Over the full stretches
  // the next stretch is requested before the current one is written, with
  // no lane-dependent branch, so a stretch waits only for its own loads.
  constexpr int kS = kVecThreads * kUnroll;
  const int64_t wg0 = (int64_t)blockIdx.x * kS;
  const int64_t gstride = (int64_t)gridDim.x * kS;
  const int64_t nfull = n >= wg0 + kS ? (n - wg0 - kS) / gstride + 1 : 0;
  // window columns past nwin read column l0 again (their coefficient is 0)
  int64_t woff[NW];
#pragma unroll
  for (int l = 0; l < NW; ++l) woff[l] = (int64_t)(l < nwin ? l : 0) * a.ldb;
  // y and the oldest window column are read for the last time in the inner
  // step: streaming loads, so they do not displace the matrix from the
  // last-level cache
  auto load_full = [&](int64_t k, VT (&yv)[kUnroll], VT (&bv)[NW][kUnroll]) {
    const int64_t r0 = wg0 + k * gstride + tid;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t r = r0 + u * kVecThreads;
      yv[u] = __builtin_nontemporal_load(&W[r]);
#pragma unroll
      for (int l = 0; l < NW; ++l)
        bv[l][u] = l == 0 ? __builtin_nontemporal_load(&win[r]) : win[woff[l] + r];
    }
  };

  // The coefficients' inputs are requested first, all at once and without
  // lane-dependent branches (addresses clamped into range, the values past
  // the counts selected away when summed), then the first stretch: loads
  // return in order, so the reduction costs one memory round trip, which
  // overlaps the stretch's transfer, instead of one per block of partials.
  // The sums keep the fixed order: block u, then thread, then wave.
  const int stopped = ctl->stop_k;
  const int Gd = a.Gd, Gv = a.Gv;  // (both >= 1)
  constexpr int kUV = kVecGrid / kVecThreads;
  double dv[NW], pv[kUV], sgw[NW];
  {
    const double* row = a.dpart + (int64_t)(tid < Gd ? tid : Gd - 1) * kDP;
#pragma unroll
    for (int l = 0; l < NW; ++l) dv[l] = row[l < nwin ? l : 0];
  }
#pragma unroll
  for (int u = 0; u < kUV; ++u) {
    const int g = tid + u * kVecThreads;
    pv[u] = a.vprev[g < Gv ? g : Gv - 1];
  }
#pragma unroll
  for (int l = 0; l < NW; ++l) {
    const int li = a.l0 + l;
    sgw[l] = a.sigma[li < step ? li : 0];
  }
  // first full stretch (independent of the coefficients)
  VT yA[kUnroll], bA[NW][kUnroll], yB[kUnroll], bB[NW][kUnroll];
  if (nfull > 0) load_full(0, yA, bA);
  // v[l] = <y, u_{l0+l}> (l < nwin), v[NW] = ||u_i||^2
  double v[NW + 1];
#pragma unroll
  for (int l = 0; l <= NW; ++l) v[l] = 0.0;
#pragma unroll
  for (int l = 0; l < NW; ++l)
    if (l < nwin) v[l] += tid < Gd ? dv[l] : 0.0;
#pragma unroll
  for (int u = 1; u < kMaxGrid / kVecThreads; ++u) {
    if (u * kVecThreads < Gd) {  // (uniform; the inner-step grid stays below kVecThreads)
      const int g = tid + u * kVecThreads;
      const double* row = a.dpart + (int64_t)(g < Gd ? g : Gd - 1) * kDP;
#pragma unroll
      for (int l = 0; l < NW; ++l)
        if (l < nwin) v[l] += g < Gd ? row[l] : 0.0;
    }
  }
#pragma unroll
  for (int u = 0; u < kUV; ++u)
    v[NW] += (step > 0 && tid + u * kVecThreads < Gv) ? pv[u] : 0.0;
  block_sum_vec<NW + 1>(v, buf);
  if (stopped != 0) return;
  if (tid == 0) {
    bool brk = false;
    double sig = 1.0;
    if (step > 0) {
      brk = v[NW] == 0.0;
      sig = brk ? 0.0 : 1.0 / sqrt(v[NW]);
    }
    for (int l = 0; l < NW; ++l) {
      const int li = a.l0 + l;
      const double sg = li == step ? sig : (li < step ? sgw[l] : 0.0);
      cf[l] = l < nwin ? sig * sg * sg * v[l] : 0.0;
    }
    cf[kMaxT] = sig;
    if (blockIdx.x == 0) {
      a.sigma[step] = sig;
      if (brk && ctl->brk_step < 0) ctl->brk_step = step;  // u_step = 0
    }
  }
  __syncthreads();
  const double ys = cf[kMaxT];
  double n2 = 0.0;
  auto update = [&](int64_t r0, const VT (&yv)[kUnroll], const VT (&bv)[NW][kUnroll],
                    bool full) {
    double acc[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc[u] = ys * static_cast<double>(yv[u]);
#pragma unroll
    for (int l = 0; l < NW; ++l)
      if (sizeof(VT) == 4 || l < nwin)  // (FP32: branch-free, the extra terms are 0)
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc[u] -= cf[l] * static_cast<double>(bv[l][u]);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t r = r0 + u * kVecThreads;
      if (full || r < n) {
        const VT o = static_cast<VT>(acc[u]);
        out[r] = o;
        const double od = static_cast<double>(o);
        n2 += od * od;
      }
    }
  };
  // full stretches.  FP32: two register sets in turn (the next stretch in
  // flight while one is written; 15.9 -> 11.3 us for the 128^3 update).
  // FP64 is bandwidth bound here and keeps the plain order and its exact
  // rounding (the window terms past nwin are skipped, not multiplied by 0,
  // which would let the compiler pair its fused multiply-adds differently).
  if constexpr (sizeof(VT) == 8) {
    // (the partial stretch below covers whatever the loop leaves)
    for (int64_t k = 0; k < nfull; ++k) {
      if (k > 0) {
        const int64_t r0 = wg0 + k * gstride + tid;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int64_t r = r0 + u * kVecThreads;
          yA[u] = r < n ? __builtin_nontemporal_load(&W[r]) : VT(0);
#pragma unroll
          for (int l = 0; l < NW; ++l)
            bA[l][u] = (l < nwin && r < n)
                           ? (l == 0 ? __builtin_nontemporal_load(&win[r]) : win[woff[l] + r])
                           : VT(0);
        }
      }
      update(wg0 + k * gstride + tid, yA, bA, false);
    }
  } else
  for (int64_t k = 0; k < nfull; k += 2) {
    const int64_t ra = wg0 + k * gstride + tid;
    if (k + 1 >= nfull) {
      update(ra, yA, bA, true);
      break;
    }
    load_full(k + 1, yB, bB);
    update(ra, yA, bA, true);
    if (k + 2 >= nfull) {
      update(ra + gstride, yB, bB, true);
      break;
    }
    load_full(k + 2, yA, bA);
    update(ra + gstride, yB, bB, true);
  }
  // the partial stretch
  {
    const int64_t r0 = wg0 + nfull * gstride + tid;
    if (wg0 + nfull * gstride < n) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t r = r0 + u * kVecThreads;
        yA[u] = r < n ? W[r] : VT(0);
#pragma unroll
        for (int l = 0; l < NW; ++l) bA[l][u] = r < n ? win[woff[l] + r] : VT(0);
      }
      update(r0, yA, bA, false);
    }
  }
  n2 = block_sum(n2, scratch);
  if (tid == 0) a.vnext[blockIdx.x] = n2;
}

template <typename VT>
static void launch_arnoldi_t(int grid, const ArnoldiArgs& a, hipStream_t st) {
  if (a.nwin <= 2)
    hipLaunchKernelGGL((k_arnoldi<VT, 2>), dim3(grid), dim3(kVecThreads), 0, st, a);
  else if (a.nwin <= 4)
    hipLaunchKernelGGL((k_arnoldi<VT, 4>), dim3(grid), dim3(kVecThreads), 0, st, a);
  else
    hipLaunchKernelGGL((k_arnoldi<VT, kMaxT>), dim3(grid), dim3(kVecThreads), 0, st, a);
}

hipError_t launch_arnoldi_update(bool fp32, int grid, const ArnoldiArgs& a, hipStream_t st) {
  if (fp32)
    launch_arnoldi_t<float>(grid, a, st);
  else
    launch_arnoldi_t<double>(grid, a, st);
  return hipGetLastError();
}

// ------------------------------------------- outer Gram-Schmidt + Givens
// Pass l of modified Gram-Schmidt at outer step j: w <- w - h_{l,j} v_l and
// the partial sums of the next coefficient <w, v_{l+1}>, or for the last
// pass of ||w||^2.
__global__ __launch_bounds__(kVecThreads) void k_mgs_pass(int64_t n, double* __restrict__ W,
                                                          const double* __restrict__ Vcur,
                                                          const double* __restrict__ Vnext,
                                                          const double* hcur,
                                                          double* __restrict__ vpart,
                                                          int last) {
  __shared__ double scratch[kVecThreads / kWave];
  const int tid = threadIdx.x;
  const double h = *hcur;
  double acc = 0.0;
  const int64_t step = (int64_t)gridDim.x * kVecThreads * kUnroll;
  for (int64_t base = (int64_t)blockIdx.x * kVecThreads * kUnroll + tid; base < n; base += step) {
    double wv[kUnroll], vc[kUnroll], vn[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t r = base + u * kVecThreads;
      const bool ok = r < n;
      wv[u] = ok ? W[r] : 0.0;
      vc[u] = ok ? Vcur[r] : 0.0;
      vn[u] = (ok && !last) ? Vnext[r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t r = base + u * kVecThreads;
      const double x = wv[u] - h * vc[u];
      if (r < n) W[r] = x;
      acc += x * (last ? x : vn[u]);
    }
  }
  acc = block_sum(acc, scratch);
  if (tid == 0) vpart[blockIdx.x] = acc;
}

hipError_t launch_mgs_pass(int grid, int64_t n, double* W, const double* Vcur,
                           const double* Vnext, const double* hcur, double* vpart, int last,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_mgs_pass, dim3(grid), dim3(kVecThreads), 0, st, n, W, Vcur, Vnext, hcur,
                     vpart, last);
  return hipGetLastError();
}

// Sums the pass partials in slot order: the next coefficient h_{l+1,j}, or,
// after the last pass, h_{j+1,j} = ||w||; then rotates column j of the
// Hessenberg matrix with the previous Givens rotations, forms rotation j,
// updates g and publishes |g_{j+1}| (the minimised residual) and the FFOM
// residual |g_{j+1}| / |c_j| (eq. (2.1) via the standard FOM/GMRES relation).
__global__ __launch_bounds__(kVecThreads) void k_mgs_finish(const double* vpart, int32_t G,
                                                            double* hout, DevCtl* ctl, int last,
                                                            double* H, double* HR, double* cs,
                                                            double* sn, double* g, int32_t j,
                                                            int32_t ldh, HostStatus* hs) {
  __shared__ double scratch[kVecThreads / kWave];
  const double tsum = block_sum_strided(vpart, G, 1, scratch);
  if (threadIdx.x != 0) return;
  if (!last) {
    *hout = tsum;
    return;
  }
  const double hn = sqrt(tsum);
  *hout = hn;
  ctl->hnext = hn;
  double* col = H + (int64_t)j * ldh;
  double* rc = HR + (int64_t)j * ldh;
  for (int i = 0; i <= j + 1; ++i) rc[i] = col[i];
  for (int i = 0; i < j; ++i) {
    const double t1 = cs[i] * rc[i] + sn[i] * rc[i + 1];
    const double t2 = -sn[i] * rc[i] + cs[i] * rc[i + 1];
    rc[i] = t1;
    rc[i + 1] = t2;
  }
  const double av = rc[j], bvv = rc[j + 1];
  const double rr = hypot(av, bvv);
  double c = 1.0, s = 0.0;
  if (rr != 0.0) {
    c = av / rr;
    s = bvv / rr;
  }
  rc[j] = rr;
  rc[j + 1] = 0.0;
  cs[j] = c;
  sn[j] = s;
  const double gj = g[j];
  g[j + 1] = -s * gj;
  g[j] = c * gj;
  // (the first j rotations triangularise H_j, the square part, up to its
  // last pivot av: FFOM's H_j^{-1} beta e1 is that triangle with pivot av
  // and right side gj)
  ctl->ffom_g = gj;
  ctl->ffom_piv = av;
  const double rho = fabs(g[j + 1]);
  const double ffom = (c != 0.0) ? rho / fabs(c) : INFINITY;
  // eq. (2.2) with the previous FFOM residual (beta at j = 1) and the
  // recursion eq. (2.3), both on the inner residual ||v_j - A z_j||
  const double rhat = sqrt(ctl->rhat2);
  const double bound = ctl->factor * rhat;
  const double q = 1.0 - ctl->delta * ctl->delta;
  const double delta = q > 0.0 ? rhat / sqrt(q) : NAN;
  ctl->bound = bound;
  ctl->delta = delta;
  ctl->rho = rho;
  ctl->ffom = ffom;
  ctl->factor = ffom;
  if ((!isfinite(rho) || !isfinite(hn)) && ctl->error == 0) ctl->error = SFGMRES_ERR_NONFINITE;
  // h_{j+1,j} = 0 with a zero pivot: H_j is singular (z_j = 0), and the
  // minimiser is not defined by the triangle
  if (hn == 0.0 && rr == 0.0 && ctl->error == 0) ctl->error = SFGMRES_ERR_BREAKDOWN;
  const bool c2 = ctl->stop_reason == SFGMRES_STOP_C2;
  host_store_i32(&hs->outer_j, j + 1);
  host_store_i32(&hs->k, ctl->stop_k);
  host_store_i32(&hs->stop_reason, ctl->stop_reason);
  host_store_i32(&hs->error, ctl->error);
  host_store_f64(&hs->rho, rho);
  host_store_f64(&hs->ffom, ffom);
  host_store_f64(&hs->hnext, hn);
  host_store_f64(&hs->cond, c2 ? ctl->cond_prev : ctl->cond_cur);
  host_store_f64(&hs->rho_hat, c2 ? ctl->rho_prev : ctl->rho_cur);
  host_store_f64(&hs->rhat_true, rhat);
  host_store_f64(&hs->bound, bound);
  host_store_f64(&hs->delta, delta);
}

hipError_t launch_mgs_finish(const double* vpart, int32_t G, double* hout, DevCtl* ctl, int last,
                             double* H, double* HR, double* cs, double* sn, double* g, int32_t j,
                             int32_t ldh, HostStatus* hs, hipStream_t st) {
  hipLaunchKernelGGL(k_mgs_finish, dim3(1), dim3(kVecThreads), 0, st, vpart, G, hout, ctl, last,
                     H, HR, cs, sn, g, j, ldh, hs);
  return hipGetLastError();
}

// ------------------------------------------ v_{j+1} = w / h fused with S v
// hptr == NULL: plain sketch of W (no normalisation, no copies).
template <typename VT, int ZB>
__global__ __launch_bounds__(kVecThreads) void k_normsk(int64_t n, const double* __restrict__ W,
                                                        const double* hptr,
                                                        double* __restrict__ Vout,
                                                        VT* __restrict__ Bout,
                                                        const SkGroup* __restrict__ skp,
                                                        int32_t zeta, int32_t s,
                                                        double* __restrict__ part) {
  extern __shared__ double lds_sk[];  // per-wave copies of the s accumulators
  constexpr int kWaves = kVecThreads / kWave;
  const int tid = threadIdx.x;
  double* const wave_sk = lds_sk + (tid / kWave) * s;
  for (int q = tid; q < kWaves * s; q += kVecThreads) lds_sk[q] = 0.0;
  __syncthreads();
  const double h = hptr ? *hptr : 1.0;
  const int G = gridDim.x;
  const int gi = xcd_logical_block(blockIdx.x, G);
  const int64_t r0 = n * gi / G;
  const int64_t r1 = n * (gi + 1) / G;
  for (int64_t r = r0 + tid; r < r1; r += kVecThreads) {
    double v;
    if (hptr)
      v = h != 0.0 ? W[r] / h : 0.0;
    else
      v = W[r];
    if (Vout) Vout[r] = v;
    if (Bout) Bout[r] = static_cast<VT>(v);
    sketch_scatter_packed<ZB>(wave_sk, skp, zeta, r, v);
  }
  __syncthreads();
  double* prow = part + (int64_t)blockIdx.x * s;
  for (int q = tid; q < s; q += kVecThreads) {
    double acc = lds_sk[q];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) acc += lds_sk[w * s + q];
    prow[q] = acc;
  }
}

template <typename VT>
static void launch_normsk_t(int zb, int grid, size_t lds, hipStream_t st, int64_t n,
                            const double* W, const double* hptr, double* Vout, VT* Bout,
                            const SkGroup* skp, int32_t zeta, int32_t s, double* part) {
  if (zb == 1)
    hipLaunchKernelGGL((k_normsk<VT, 1>), dim3(grid), dim3(kVecThreads), lds, st, n, W, hptr,
                       Vout, Bout, skp, zeta, s, part);
  else
    hipLaunchKernelGGL((k_normsk<VT, 2>), dim3(grid), dim3(kVecThreads), lds, st, n, W, hptr,
                       Vout, Bout, skp, zeta, s, part);
}

hipError_t launch_normalize_sketch(bool fp32, int grid, int64_t n, const double* W,
                                   const double* hptr, double* Vout, void* Bout, int32_t s,
                                   const SkGroup* skp, int32_t zeta, double* part,
                                   hipStream_t st) {
  const size_t lds = (size_t)(kVecThreads / kWave) * s * sizeof(double);
  const int zb = sk_groups(zeta);
  if (fp32)
    launch_normsk_t<float>(zb, grid, lds, st, n, W, hptr, Vout, static_cast<float*>(Bout), skp,
                           zeta, s, part);
  else
    launch_normsk_t<double>(zb, grid, lds, st, n, W, hptr, Vout, static_cast<double*>(Bout), skp,
                            zeta, s, part);
  return hipGetLastError();
}

// ----------------------------------------------- small triangular solves
// y = R^{-1} d[0:k] for the inner dimension k chosen on the device, then
// y_l * sigma_l so that z_j = sum_l y_l u_l over the unnormalised vectors.
// When the upper triangle of R_k fits in LDS it is loaded there at once by
// the whole workgroup and wave 0 substitutes alone (lane p owning rows p,
// p + 64, ...; the right-hand side stays in registers, no barrier per
// column); otherwise columns are staged kFinChunk at a time with one
// barrier per column.
constexpr int kFinThreads = 256;
constexpr int kFinChunk = 8;
constexpr int kFinRows = kMaxM / kWave;
constexpr int kFinLds = 12288;  // doubles of R held in LDS (k x k block: k <= 110)

__global__ __launch_bounds__(kFinThreads) void k_finalize(const DevCtl* ctl, const double* R,
                                                          const double* d, const double* sigma,
                                                          int32_t m, double* y) {
  __shared__ double rhs[kMaxM];
  __shared__ double ys[kMaxM];
  __shared__ double col[kFinChunk][kMaxM];
  __shared__ double tri[kFinLds];  // R[0:k, 0:k], column l at l * k
  const int k = ctl->stop_k;
  if (k <= 0 || k > m) return;
  const int tid = threadIdx.x;
  if (k * k <= kFinLds) {
    // the k x k block at once (entries below the diagonal are read, unused)
    constexpr int kB = 8;
    for (int i0 = 0; i0 < k * k; i0 += kFinThreads * kB) {
      double v[kB];
#pragma unroll
      for (int b = 0; b < kB; ++b) {
        const int i = i0 + b * kFinThreads + tid;
        v[b] = i < k * k ? R[(int64_t)(i / k) * m + i % k] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < kB; ++b) {
        const int i = i0 + b * kFinThreads + tid;
        if (i < k * k) tri[i] = v[b];
      }
    }
    __syncthreads();
    if (tid >= kWave) return;
    const int lane = tid;
    double r[kFinRows], yv[kFinRows];
#pragma unroll
    for (int u = 0; u < kFinRows; ++u) {
      const int p = lane + u * kWave;
      r[u] = p < k ? d[p] : 0.0;
      yv[u] = 0.0;
    }
    for (int l = k - 1; l >= 0; --l) {
      const double* cl = tri + l * k;
      const int ul = l / kWave;
      double dl = 0.0, rl = 0.0;
#pragma unroll
      for (int u = 0; u < kFinRows; ++u)
        if (u == ul) rl = r[u];
      dl = cl[l];  // (same address in every lane)
      const double yl = read_lane(rl, l % kWave) / dl;
#pragma unroll
      for (int u = 0; u < kFinRows; ++u) {
        if (u > ul) break;  // (uniform: the rows of blocks past ul are done)
        const int p = lane + u * kWave;
        if (p == l) yv[u] = yl;
        if (p < l) r[u] -= cl[p] * yl;
      }
    }
#pragma unroll
    for (int u = 0; u < kFinRows; ++u) {
      const int p = lane + u * kWave;
      if (p < k) y[p] = yv[u] * sigma[p];
    }
    return;
  }
  for (int p = tid; p < k; p += kFinThreads) rhs[p] = d[p];
  for (int hi = k - 1; hi >= 0; hi -= kFinChunk) {
    const int lo = hi - kFinChunk + 1 > 0 ? hi - kFinChunk + 1 : 0;
    __syncthreads();
    for (int c = lo; c <= hi; ++c)
      for (int p = tid; p <= hi; p += kFinThreads) col[c - lo][p] = R[(int64_t)c * m + p];
    __syncthreads();
    for (int l = hi; l >= lo; --l) {
      const double yl = rhs[l] / col[l - lo][l];
      if (tid == 0) ys[l] = yl;
      for (int p = tid; p < l; p += kFinThreads) rhs[p] -= col[l - lo][p] * yl;
      __syncthreads();
    }
  }
  for (int p = tid; p < k; p += kFinThreads) y[p] = ys[p] * sigma[p];
}

hipError_t launch_finalize(const DevCtl* ctl, const double* R, const double* d,
                           const double* sigma, int32_t m, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, st, ctl, R, d, sigma, m, y);
  return hipGetLastError();
}

// Back substitution with the Givens-rotated Hessenberg factor (column-major,
// leading dimension ldh): y = HR[0:J,0:J]^{-1} g[0:J] (FGMRES).  With `ctl`
// the last row takes the FFOM pivot and right side recorded by the last
// Givens update instead, which gives y = H_J^{-1} beta e1 (FFOM, Algorithm
// 1); a zero pivot (H_J singular) gives NaN.
__global__ __launch_bounds__(kWave) void k_backsolve(const double* HR, const double* g,
                                                     int32_t J, int32_t ldh, double* y,
                                                     const DevCtl* ctl) {
  extern __shared__ double sh[];
  double* rhs = sh;
  double* ys = sh + J;
  const int tid = threadIdx.x;
  for (int p = tid; p < J; p += kWave) rhs[p] = g[p];
  __syncthreads();
  const bool ffom = ctl != nullptr;
  if (ffom && tid == 0) rhs[J - 1] = ctl->ffom_g;
  __syncthreads();
  const double piv_last = ffom ? ctl->ffom_piv : HR[(int64_t)(J - 1) * ldh + J - 1];
  if (ffom && piv_last == 0.0) {
    for (int p = tid; p < J; p += kWave) y[p] = NAN;
    return;
  }
  for (int l = J - 1; l >= 0; --l) {
    const double yl = rhs[l] / (l == J - 1 ? piv_last : HR[(int64_t)l * ldh + l]);
    if (tid == 0) ys[l] = yl;
    for (int p = tid; p < l; p += kWave) rhs[p] -= HR[(int64_t)l * ldh + p] * yl;
    __syncthreads();
  }
  for (int p = tid; p < J; p += kWave) y[p] = ys[p];
}

hipError_t launch_backsolve(const double* HR, const double* g, int32_t J, int32_t ldh,
                            double* y, hipStream_t st, const DevCtl* ffom_ctl) {
  hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(kWave), (size_t)2 * J * sizeof(double), st, HR,
                     g, J, ldh, y, ffom_ctl);
  return hipGetLastError();
}

// ------------------------------------------------- tall-skinny combination
// out = add + sum_{l<k} y_l B[:, l], k read from the device (kdev) or given.
// Each thread owns one 16-byte group of rows (four FP32 or two FP64 rows,
// one load per column; the columns are 256-byte aligned with a leading
// dimension that is a multiple of 64 elements) and sums every row over the
// columns in order; rows past the last full group are done one by one.
template <typename VT>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};

template <typename VT>
__global__ __launch_bounds__(kVecThreads) void k_combine(int64_t n, const VT* __restrict__ B,
                                                         int64_t ldb,
                                                         const double* __restrict__ y,
                                                         const int32_t* kdev, int32_t khost,
                                                         const double* add, double* out,
                                                         const double* scale) {
  using V = typename Vec16<VT>::type;
  constexpr int kG = 16 / (int)sizeof(VT);
  extern __shared__ double ys[];
  const int k = kdev ? *kdev : khost;
  for (int l = threadIdx.x; l < k; l += kVecThreads) ys[l] = y[l];
  __syncthreads();
  const double sc = scale ? *scale : 1.0;
  const int64_t stride = (int64_t)gridDim.x * kVecThreads;
  const int64_t ng = n / kG;
  // (with a scale the sum is formed first, then out = add + scale * sum;
  // add and out may be the same vector)
  for (int64_t gi = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; gi < ng; gi += stride) {
    const int64_t r0 = gi * kG;
    double acc[kG];
#pragma unroll
    for (int c = 0; c < kG; ++c) acc[c] = scale ? 0.0 : (add ? add[r0 + c] : 0.0);
    for (int l = 0; l < k; ++l) {
      const V b = *reinterpret_cast<const V*>(B + (int64_t)l * ldb + r0);
#pragma unroll
      for (int c = 0; c < kG; ++c) acc[c] += ys[l] * static_cast<double>(b[c]);
    }
#pragma unroll
    for (int c = 0; c < kG; ++c)
      out[r0 + c] = scale ? (add ? add[r0 + c] : 0.0) + sc * acc[c] : acc[c];
  }
  for (int64_t r = ng * kG + (int64_t)blockIdx.x * kVecThreads + threadIdx.x; r < n; r += stride) {
    double acc = scale ? 0.0 : (add ? add[r] : 0.0);
    for (int l = 0; l < k; ++l) acc += ys[l] * static_cast<double>(B[(int64_t)l * ldb + r]);
    out[r] = scale ? (add ? add[r] : 0.0) + sc * acc : acc;
  }
}

hipError_t launch_combine(bool fp32, int64_t n, const void* B, int64_t ldb, const double* y,
                          const int32_t* kdev, int32_t khost, const double* add, double* out,
                          hipStream_t st, const double* scale) {
  const int kmax = kdev ? kMaxM : khost;
  const size_t lds = (size_t)(kmax > 0 ? kmax : 1) * sizeof(double);
  const int grid = vec_grid(n * kUnroll / (fp32 ? 4 : 2));
  if (fp32)
    hipLaunchKernelGGL(k_combine<float>, dim3(grid), dim3(kVecThreads), lds, st, n,
                       static_cast<const float*>(B), ldb, y, kdev, khost, add, out, scale);
  else
    hipLaunchKernelGGL(k_combine<double>, dim3(grid), dim3(kVecThreads), lds, st, n,
                       static_cast<const double*>(B), ldb, y, kdev, khost, add, out, scale);
  return hipGetLastError();
}

// ------------------------------------------------------------ elementwise
__global__ void k_cast_f32(const double* __restrict__ src, float* __restrict__ dst,
                           int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    dst[i] = static_cast<float>(src[i]);
}

hipError_t launch_cast_f32(const double* src, float* dst, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast_f32, dim3(vec_grid(count)), dim3(kVecThreads), 0, st, src, dst,
                     count);
  return hipGetLastError();
}

__global__ void k_copy_or_zero(const double* __restrict__ src, double* __restrict__ dst,
                               int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src ? src[i] : 0.0;
}

hipError_t launch_copy_or_zero(const double* src, double* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_or_zero, dim3(vec_grid(n)), dim3(kVecThreads), 0, st, src, dst, n);
  return hipGetLastError();
}

// grad[p] = -lam[row(p)] * x[col(p)].  A workgroup takes kVecThreads rows
// at a time: their bounds in LDS, then the rows' nonzeros (one contiguous
// range) one per thread, each thread finding its row by binary search over
// the bounds, so that the column indices are read and the gradient written
// in whole runs.
__global__ __launch_bounds__(kVecThreads) void k_gradient(const int32_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col_idx,
                                                          int64_t n, const double* __restrict__ lam,
                                                          const double* __restrict__ x,
                                                          double* __restrict__ grad) {
  __shared__ int32_t rb[kVecThreads + 1];
  for (int64_t r0 = (int64_t)blockIdx.x * kVecThreads; r0 < n;
       r0 += (int64_t)gridDim.x * kVecThreads) {
    const int nr = (int)(n - r0 < kVecThreads ? n - r0 : kVecThreads);
    const int64_t rr = r0 + threadIdx.x;
    rb[threadIdx.x] = row_ptr[rr < n ? rr : n];
    if (threadIdx.x == 0) rb[kVecThreads] = row_ptr[r0 + kVecThreads < n ? r0 + kVecThreads : n];
    __syncthreads();
    const int p0 = rb[0], p1 = rb[nr];
    for (int p = p0 + threadIdx.x; p < p1; p += kVecThreads) {
      int lo = 0, hi = nr;  // the row: the last k with rb[k] <= p
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rb[mid] <= p)
          lo = mid;
        else
          hi = mid;
      }
      grad[p] = -lam[r0 + lo] * x[col_idx[p]];
    }
    __syncthreads();
  }
}

hipError_t launch_gradient(const int32_t* row_ptr, const int32_t* col_idx, int64_t n,
                           const double* lam, const double* x, double* grad, hipStream_t st) {
  hipLaunchKernelGGL(k_gradient, dim3(vec_grid(n)), dim3(kVecThreads), 0, st, row_ptr, col_idx,
                     n, lam, x, grad);
  return hipGetLastError();
}

// ------------------------------------------------------------ transpose
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;
constexpr int kScanChunk = kScanThreads * kScanPer;

size_t transpose_scan_tmp_ints(int64_t n) { return (size_t)((n + kScanChunk - 1) / kScanChunk) + 2; }

__global__ void k_zero_i32(int32_t* p, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    p[i] = 0;
}

__global__ void k_count_cols(const int32_t* __restrict__ col_idx, int64_t nnz, int32_t* cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += stride)
    atomicAdd(&cnt[col_idx[p]], 1);
}

// exclusive scan helpers: per-thread sums of kScanPer items, then a
// workgroup scan of the thread sums (waves via shuffles, wave totals in LDS)
__device__ static int block_exclusive_scan(int v, int* wtot, int& total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  int incl = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int o = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += o;
  }
  if (lane == kWave - 1) wtot[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < kScanThreads / kWave; ++i) {
      const int t = wtot[i];
      wtot[i] = run;
      run += t;
    }
    wtot[kScanThreads / kWave] = run;
  }
  __syncthreads();
  total = wtot[kScanThreads / kWave];
  const int excl = incl - v + wtot[wid];
  __syncthreads();
  return excl;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(const int32_t* cnt, int64_t n,
                                                            int32_t* bsum) {
  __shared__ int wtot[kScanThreads / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
  int v = 0;
  for (int u = 0; u < kScanPer; ++u)
    if (base + u < n) v += cnt[base + u];
  int total;
  block_exclusive_scan(v, wtot, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(int32_t* bsum, int64_t nb) {
  __shared__ int wtot[kScanThreads / kWave + 1];
  int carry = 0;
  for (int64_t base = 0; base < nb; base += kScanThreads) {
    const int64_t i = base + threadIdx.x;
    const int v = i < nb ? bsum[i] : 0;
    int total;
    const int ex = block_exclusive_scan(v, wtot, total);
    if (i < nb) bsum[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t* cnt, int64_t n,
                                                             const int32_t* bsum,
                                                             int32_t* out) {
  __shared__ int wtot[kScanThreads / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
  int loc[kScanPer];
  int v = 0;
  for (int u = 0; u < kScanPer; ++u) {
    loc[u] = (base + u < n) ? cnt[base + u] : 0;
    v += loc[u];
  }
  int total;
  int ex = block_exclusive_scan(v, wtot, total) + bsum[blockIdx.x];
  for (int u = 0; u < kScanPer; ++u) {
    if (base + u < n) out[base + u] = ex;
    ex += loc[u];
  }
}

__global__ void k_fill_transpose(const int32_t* __restrict__ row_ptr,
                                 const int32_t* __restrict__ col_idx, int64_t n,
                                 const int32_t* __restrict__ rp_t, int32_t* cursor,
                                 int32_t* __restrict__ col_t, int32_t* __restrict__ perm) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      const int c = col_idx[p];
      const int pos = rp_t[c] + atomicAdd(&cursor[c], 1);
      col_t[pos] = (int32_t)i;
      perm[pos] = p;
    }
  }
}

// Sort each row of A^T by (column, source position) with an in-place
// heapsort, then gather the values.
__device__ static bool pair_less(int a0, int a1, int b0, int b1) {
  return a0 < b0 || (a0 == b0 && a1 < b1);
}

__device__ static void sift_down(int32_t* k0, int32_t* k1, int start, int end) {
  int root = start;
  while (2 * root + 1 <= end) {
    int child = 2 * root + 1;
    int sw = root;
    if (pair_less(k0[sw], k1[sw], k0[child], k1[child])) sw = child;
    if (child + 1 <= end && pair_less(k0[sw], k1[sw], k0[child + 1], k1[child + 1]))
      sw = child + 1;
    if (sw == root) return;
    const int t0 = k0[root], t1 = k1[root];
    k0[root] = k0[sw];
    k1[root] = k1[sw];
    k0[sw] = t0;
    k1[sw] = t1;
    root = sw;
  }
}

__global__ void k_sort_rows(const int32_t* __restrict__ rp_t, int64_t n, int32_t* col_t,
                            int32_t* perm, const double* __restrict__ val,
                            double* __restrict__ val_t) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const int a = rp_t[r];
    const int len = rp_t[r + 1] - a;
    int32_t* k0 = col_t + a;
    int32_t* k1 = perm + a;
    if (len > 1) {
      for (int st = (len - 2) / 2; st >= 0; --st) sift_down(k0, k1, st, len - 1);
      for (int end = len - 1; end > 0; --end) {
        const int t0 = k0[0], t1 = k1[0];
        k0[0] = k0[end];
        k1[0] = k1[end];
        k0[end] = t0;
        k1[end] = t1;
        sift_down(k0, k1, 0, end - 1);
      }
    }
    if (val_t)
      for (int q = 0; q < len; ++q) val_t[a + q] = val[k1[q]];
  }
}

__global__ void k_copy_i32_last(const int32_t* src, int32_t* dst) { *dst = *src; }

hipError_t launch_exclusive_scan(int32_t* cnt, int64_t n, int32_t* scan_tmp, hipStream_t st) {
  const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
  if (nb > 0) {
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(kScanThreads), 0, st, cnt, n,
                       scan_tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, scan_tmp, nb);
    // (each thread reads its own items before it writes them)
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, st, cnt, n,
                       scan_tmp, cnt);
  } else {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(kVecThreads), 0, st, scan_tmp, (int64_t)1);
  }
  hipLaunchKernelGGL(k_copy_i32_last, dim3(1), dim3(1), 0, st, scan_tmp + nb, cnt + n);
  return hipGetLastError();
}

// A pattern equal to its transpose (every stencil): row c of A^T has the
// columns of row c of A, so the transpose needs no counting or sorting;
// entry q = (c, r) of A^T takes the value of entry (r, c) of A, found in row
// r (a linear scan of a short row, else a binary search; perm[q] = its
// position).  *bad is set when a mirror entry is missing or a row's columns
// are not increasing; the caller then builds the transpose the general way,
// which overwrites everything.
__global__ __launch_bounds__(kVecThreads) void k_transpose_sym(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const double* __restrict__ val, int64_t n, int32_t* __restrict__ rp_t,
    int32_t* __restrict__ col_t, double* __restrict__ val_t, int32_t* __restrict__ perm,
    int32_t* bad) {
  // (a workgroup takes kVecThreads rows at a time, their bounds in LDS, and
  // their nonzeros one per thread, so that every array is read and written
  // in whole runs)
  __shared__ int32_t rb[kVecThreads + 1];
  bool ok = true;
  for (int64_t r0 = (int64_t)blockIdx.x * kVecThreads; r0 < n;
       r0 += (int64_t)gridDim.x * kVecThreads) {
    const int nr = (int)(n - r0 < kVecThreads ? n - r0 : kVecThreads);
    const int64_t rr = r0 + threadIdx.x;
    const int32_t b = row_ptr[rr < n ? rr : n];
    rb[threadIdx.x] = b;
    if (rr < n) rp_t[rr] = b;
    if (threadIdx.x == 0 && r0 + nr == n) rp_t[n] = row_ptr[n];
    if (threadIdx.x == 0) rb[kVecThreads] = row_ptr[r0 + kVecThreads < n ? r0 + kVecThreads : n];
    __syncthreads();
    const int q0 = rb[0], q1 = rb[nr];
    for (int q = q0 + threadIdx.x; q < q1; q += kVecThreads) {
      int lo = 0, hi = nr;  // the row: the last k with rb[k] <= q
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rb[mid] <= q)
          lo = mid;
        else
          hi = mid;
      }
      const int c = (int)(r0 + lo);
      const int r = col_idx[q];
      ok &= q == rb[lo] || col_idx[q - 1] < r;
      col_t[q] = r;
      const int a0 = row_ptr[r], a1 = row_ptr[r + 1];
      int p = -1;
      if (a1 - a0 <= kShortRow) {
        // (a short row: its columns requested together)
#pragma unroll
        for (int k = 0; k < kShortRow; ++k)
          if (a0 + k < a1 && col_idx[a0 + k] == c) p = a0 + k;
      } else {
        int l = a0, h = a1;
        while (l < h) {
          const int mid = (l + h) >> 1;
          if (col_idx[mid] < c)
            l = mid + 1;
          else
            h = mid;
        }
        if (l < a1 && col_idx[l] == c) p = l;
      }
      ok &= p >= 0;
      p = p >= 0 ? p : q;
      perm[q] = p;
      if (val_t) val_t[q] = val[p];
    }
    __syncthreads();
  }
  if (!ok) atomicOr(bad, 1);
}

hipError_t launch_transpose(const int32_t* row_ptr, const int32_t* col_idx, const double* val,
                            int64_t n, int64_t nnz, int32_t* rp_t, int32_t* col_t,
                            double* val_t, int32_t* perm, int32_t* cursor, int32_t* scan_tmp,
                            hipStream_t st) {
  // (cursor[0] holds the flag of the symmetric-pattern attempt)
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(kVecThreads), 0, st, cursor, (int64_t)1);
  hipLaunchKernelGGL(k_transpose_sym, dim3(vec_grid(n)), dim3(kVecThreads), 0, st, row_ptr,
                     col_idx, val, n, rp_t, col_t, val_t, perm, cursor);
  int32_t bad = 1;
  hipError_t e = hipMemcpyAsync(&bad, cursor, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  if (!bad) return hipGetLastError();
  const int g = vec_grid(n + 1);
  hipLaunchKernelGGL(k_zero_i32, dim3(g), dim3(kVecThreads), 0, st, cursor, n + 1);
  hipLaunchKernelGGL(k_count_cols, dim3(vec_grid(nnz > 0 ? nnz : 1)), dim3(kVecThreads), 0, st,
                     col_idx, nnz, cursor);
  const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(kScanThreads), 0, st, cursor, n,
                     scan_tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, scan_tmp, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, st, cursor, n,
                     scan_tmp, rp_t);
  // rp_t[n] = nnz
  hipLaunchKernelGGL(k_copy_i32_last, dim3(1), dim3(1), 0, st, scan_tmp + nb, rp_t + n);
  hipLaunchKernelGGL(k_zero_i32, dim3(g), dim3(kVecThreads), 0, st, cursor, n + 1);
  hipLaunchKernelGGL(k_fill_transpose, dim3(vec_grid(n)), dim3(kVecThreads), 0, st, row_ptr,
                     col_idx, n, rp_t, cursor, col_t, perm);
  hipLaunchKernelGGL(k_sort_rows, dim3(vec_grid(n)), dim3(kVecThreads), 0, st, rp_t, n, col_t,
                     perm, val, val_t);
  return hipGetLastError();
}

}  // namespace sfg
