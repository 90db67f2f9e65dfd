// Coefficients, reductions and decisions of the inner sGMRES cycle
// (Section 3, with the truncated Arnoldi basis of Section 4.1).
//
// k_coef (one workgroup; t = 0, and the last step of a cycle: otherwise the
// truncated-Arnoldi update forms these coefficients itself) sums the
// window dots and ||y||^2 of the fused SpMV's scalar rows, forms
// sigma_i = 1/||u_i|| of the current (unnormalised) Arnoldi vector from the
// norm partials of the previous Arnoldi update, and stores the coefficients
// of the next vector: u_{i+1} = sigma_i y - sum_l sigma_i sigma_l^2 <y, u_l> u_l,
// i.e. A b_i minus its projections h_l b_l on the window b_l = sigma_l u_l
// with h_l = sigma_i sigma_l <y, u_l>; for t = 0 it stores
// sigma_{i+1} = 1/||y|| of the next power-basis vector y = A b_i.
//
// The sketched least-squares problem only decides when the cycle stops and
// gives the final coefficients y_k: the Krylov basis never waits for it.  So
// p consecutive inner steps run first, each leaving the raw sketch S y_i as
// per-workgroup partial rows in its ring slot, and then
//
// k_reduce_slots (many workgroups) sums the partial rows of the p slots in
// slot order, and
//
// k_qr_block (one workgroup, 1024 threads; both run on a stream of their
// own, concurrently with the next inner steps) appends the p columns
// c_i = S A b_i / sqrt(zeta) (b_i = sigma_i u_i; for t = 0 the SpMV already
// returned A b_i) to the Householder QR of S A B, in float64:
//   * blocked update with the existing reflectors in compact-WY form
//     (Q = I - V T V^T, T upper triangular): A = V^T C, B = T^T A,
//     C <- C - V B, one pass over V (twice) and T for all p columns;
//   * the p new reflectors column by column (right-looking inside the
//     panel, four waves; the other twelve exit after the blocked update),
//     with d = Q^T S v_j carried along, the sketched least-squares
//     residual ||d[i+1:]|| (the estimate C3 uses) and Bischof's incremental
//     condition estimate of R (the estimate C2 uses) after every column;
//   * the decision after every column, in this order: a zero Arnoldi vector
//     (truncated-Arnoldi breakdown), a forced replay dimension, C2 (estimate
//     above threshold: drop the column), C3 (bound of eq. (2.2) below tol),
//     C1 (i = m).  Column i's decision uses the quantities a one-column
//     update gives (R_i is the leading block of R_k), so the blocking
//     changes rounding only; steps run past the stop are discarded;
//   * T extended by the previous panel's reflectors at the start of the
//     next launch, where all waves are present (a cycle's last panel never
//     pays for it).
// It is the only writer of the stop flag.  k_rq_init takes d0 = S v_j and
// resets the cycle state; k_sketch_out is the test export of one fused SpMV.
#include "kernels.hpp"

namespace sfg {

// ------------------------------------------------------------ coefficients
constexpr int kCoefThreads = 256;

__global__ __launch_bounds__(kCoefThreads) void k_coef(CoefArgs a) {
  constexpr int kNV = kMaxT + 2;  // window dots, ||y||^2, ||u_step||^2
  __shared__ double buf[(kCoefThreads / kWave) * kNV];
  DevCtl* ctl = a.ctl;
  const int tid = threadIdx.x;
  const int step = a.step;
  // every load first (one round trip): the scalar rows of the SpMV, the
  // norm partials of the Arnoldi update, the window's sigmas, the stop flag
  double v[kNV];
#pragma unroll
  for (int l = 0; l < kNV; ++l) v[l] = 0.0;
#pragma unroll
  for (int u = 0; u < kMaxGrid / kCoefThreads; ++u) {
    const int g = tid + u * kCoefThreads;
    if (g < a.G) {
      const double* row = a.dpart + (int64_t)g * kDP;
#pragma unroll
      for (int l = 0; l < kMaxT; ++l)
        if (l < a.nwin) v[l] += row[l];
      v[kMaxT] += row[kMaxT];
    }
  }
  const bool use_u = a.t > 0 && step > 0;
#pragma unroll
  for (int u = 0; u < kVecGrid / kCoefThreads; ++u) {
    const int g = tid + u * kCoefThreads;
    if (use_u && g < a.Gv) v[kMaxT + 1] += a.vpart[g];
  }
  double sgw[kMaxT];
#pragma unroll
  for (int l = 0; l < kMaxT; ++l)
    sgw[l] = (tid == 0 && l < a.nwin && a.l0 + l < step) ? a.sigma[a.l0 + l] : 0.0;
  const int stopped = ctl->stop_k;
  block_sum_vec<kNV>(v, buf);
  if (stopped != 0 || tid != 0) return;
  if (a.t > 0) {
    double sig = 1.0;
    bool brk = false;
    if (step > 0) {
      brk = v[kMaxT + 1] == 0.0;
      sig = brk ? 0.0 : 1.0 / sqrt(v[kMaxT + 1]);
    }
    a.sigma[step] = sig;
    if (brk && ctl->brk_step < 0) ctl->brk_step = step;  // u_step = 0
    for (int l = 0; l < a.nwin; ++l) {
      const double sg = (a.l0 + l == step) ? sig : sgw[l];
      a.coef[l] = sig * sg * sg * v[l];
    }
    a.coef[kMaxT] = sig;
  } else {
    const double n2 = v[kMaxT];
    if (n2 == 0.0) {
      if (ctl->brk_step < 0) ctl->brk_step = step + 1;  // the next power-basis vector is zero
      a.sigma[step + 1] = 0.0;
    } else {
      a.sigma[step + 1] = 1.0 / sqrt(n2);
    }
  }
}

hipError_t launch_coef(const CoefArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_coef, dim3(1), dim3(kCoefThreads), 0, st, a);
  return hipGetLastError();
}

// ------------------------------------------------------------ reductions
constexpr int kRedThreads = 256;
constexpr int kRedSlice = 8;  // entries per reduction workgroup

__global__ __launch_bounds__(kRedThreads) void k_reduce_slots(
    const double* __restrict__ part, int32_t G, int32_t stride, int32_t count, int32_t first,
    int32_t nring, int64_t slot_part, int64_t slot_red, double* __restrict__ red,
    const DevCtl* ctl, int predicated) {
  __shared__ double sl[kRedThreads];
  if (predicated && ctl->stop_k != 0) return;
  const int slot = (first + (int)blockIdx.y) % nring;
  const double* p = part + slot * slot_part;
  const int tid = threadIdx.x;
  const int e = blockIdx.x * kRedSlice + (tid % kRedSlice);
  const int rg = tid / kRedSlice;
  constexpr int nrg = kRedThreads / kRedSlice;
  constexpr int kRU = 8;  // rows in flight per thread
  double acc = 0.0;
  if (e < count) {
    int r = rg;
    for (; r + (kRU - 1) * nrg < G; r += kRU * nrg) {
      double v[kRU];
#pragma unroll
      for (int u = 0; u < kRU; ++u) v[u] = p[(int64_t)(r + u * nrg) * stride + e];
#pragma unroll
      for (int u = 0; u < kRU; ++u) acc += v[u];
    }
    for (; r < G; r += nrg) acc += p[(int64_t)r * stride + e];
  }
  sl[tid] = acc;
  __syncthreads();
  if (tid < kRedSlice) {
    double t = 0.0;
    for (int r = 0; r < nrg; ++r) t += sl[r * kRedSlice + tid];
    if (e < count) red[slot * slot_red + e] = t;
  }
}

hipError_t launch_reduce_slots(const double* part, int32_t G, int32_t stride, int32_t count,
                               int32_t first, int32_t nslots, int32_t nring, int64_t slot_part,
                               int64_t slot_red, double* red, const DevCtl* ctl, bool predicated,
                               hipStream_t st) {
  const int nb = (count + kRedSlice - 1) / kRedSlice;
  hipLaunchKernelGGL(k_reduce_slots, dim3(nb, nslots), dim3(kRedThreads), 0, st, part, G, stride,
                     count, first, nring, slot_part, slot_red, red, ctl, predicated ? 1 : 0);
  return hipGetLastError();
}

// ------------------------------------------------------------- decisions
// Top eigenvalue / unit eigenvector of [[a, b], [b, d]] via the symmetric
// Schur rotation (Golub & Van Loan, Sec. 8.5.2).
__device__ static void top_eig2(double a, double b, double d, double& lam, double& vs,
                                double& vc) {
  if (b == 0.0) {
    if (a > d) {
      lam = a;
      vs = 1.0;
      vc = 0.0;
    } else {
      lam = d;
      vs = 0.0;
      vc = 1.0;
    }
    return;
  }
  const double zeta = (d - a) / (2.0 * b);
  const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + tt * tt);
  const double s = tt * c;
  const double l1 = a - tt * b;  // eigenvector (c, -s)
  const double l2 = d + tt * b;  // eigenvector (s, c)
  if (l1 >= l2) {
    lam = l1;
    vs = c;
    vc = -s;
  } else {
    lam = l2;
    vs = s;
    vc = c;
  }
}

// The host status block needs no fence: the device flag is the authority,
// and a host that reads a stale value only enqueues steps that exit at once.
// One sketch row per thread: every row-wise quantity of the panel (its
// kPanel columns, d, the condition-estimate vectors) lives in registers.
constexpr int kQrThreads = 1024;
static_assert(kQrThreads >= kMaxS && kQrThreads >= kMaxM, "one row per thread");
constexpr int kQrWaves = kQrThreads / kWave;
constexpr int kRB = 32;  // reduction entries per wave (>= kPanel (kPanel - 1) / 2)

size_t qr_block_lds_bytes(int32_t s, int32_t m) {
  return sizeof(double) * ((size_t)kPanel * s + s + 2 * (size_t)m + 2 * (size_t)m * kPanel +
                           (size_t)kQrWaves * kRB);
}

// Householder reflector for a column whose entry at the pivot row is alpha
// and whose squared norm below it is x2: H = I - tau v v^T with v = 1 at the
// pivot and (entry / den) below, H c = beta e_pivot.
__device__ __forceinline__ void reflector(double alpha, double x2, double& beta, double& tau,
                                          double& den) {
  if (x2 == 0.0) {
    beta = alpha;
    tau = 0.0;
    den = 0.0;
  } else {
    beta = -copysign(sqrt(alpha * alpha + x2), alpha);
    tau = (beta - alpha) / beta;
    den = alpha - beta;
  }
}

// Sum over the 16 lanes of a row of the wave (quad exchanges, then the
// values 4 and 8 lanes along); lane 0 of the row holds the sum.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x124>(v);  // row_ror:4
  v += dpp_move<0x128>(v);  // row_ror:8
  return v;
}

// y = V^T X over rows >= q0 for the k0 reflectors V (global, column-major,
// s rows) and the kPanel columns X (LDS, column-major), masked to rows
// >= q0 + j in column j when `masked` (columns j >= ncol read as zero).  X
// may be in LDS or in global memory.  A wave takes four reflectors at
// once, 16 lanes along the rows of each (coalesced 128-byte segments), so
// each output needs only a 16-lane reduction.  Output y[j * ldy + l] (LDS).
__device__ __forceinline__ void vt_panel(const double* __restrict__ V, int s, int k0, int q0,
                                         const double* X, int ncol, bool masked, double* y,
                                         int ldy) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int c = lane >> 4;
  const int ql = lane & 15;
  for (int lb = wid * 4; lb < k0; lb += kQrWaves * 4) {
    const int l = lb + c;
    const bool has = l < k0;
    const double* Vl = V + (int64_t)(has ? l : 0) * s;
    double acc[kPanel];
#pragma unroll
    for (int j = 0; j < kPanel; ++j) acc[j] = 0.0;
#pragma unroll 4
    for (int q = q0 + ql; q < s; q += 16) {
      const double v = has ? Vl[q] : 0.0;
#pragma unroll
      for (int j = 0; j < kPanel; ++j) {
        const double xq = (j < ncol && (!masked || q >= q0 + j)) ? X[j * s + q] : 0.0;
        acc[j] += v * xq;
      }
    }
#pragma unroll
    for (int j = 0; j < kPanel; ++j) {
      const double r = row16_sum(acc[j]);
      if (ql == 0 && has) y[j * ldy + l] = r;
    }
  }
}

// Shared scalars of the decision kernel.
struct QrShared {
  double tau[kPanel];
  double beta[kPanel];
  double wm[kPanel][kPanel];  // wm[x][y] = v_{kb+x}^T v_{kb+y}, x < y
  int stopped, done;
};

constexpr int kPanelWaves = 4;  // waves that factorise the panel (one per SIMD)
constexpr int kPanelThreads = kPanelWaves * kWave;
constexpr int kRowsPT = (kMaxS + kPanelThreads - 1) / kPanelThreads;  // rows per panel thread

// Sums of NV values over the kPanelWaves panel waves; every one of their
// threads gets the NV sums (wave sums, one barrier, the wave partials added
// in wave order).  Only the panel waves are alive when it is called.
// Callers alternate two buffers: a thread writes buffer b only after the
// barrier of the call that used the other one, which every thread reaches
// only after reading buffer b the time before.
template <int NV>
__device__ __forceinline__ void panel_sum(double (&v)[NV], double* rbuf, int& par) {
  double* buf = rbuf + par * (kPanelWaves * 16);
  par ^= 1;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) buf[wid * 16 + i] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < kPanelWaves; ++w) r += buf[w * 16 + i];
    v[i] = r;
  }
}

__global__ __launch_bounds__(kQrThreads) void k_qr_block(QrBlockArgs a) {
  extern __shared__ double lds[];
  __shared__ QrShared sh;
  const int s = a.s;
  const int m = a.m;
  // LDS: panel (kPanel columns of s, column-major), d (s), the condition
  // estimate vectors x and z (m each), AU and BX (m x kPanel, column-major),
  // reduction buffer
  double* Cp = lds;
  double* dv = Cp + (size_t)kPanel * s;
  double* xv = dv + s;
  double* zv = xv + m;
  double* AU = zv + m;
  double* BX = AU + (size_t)m * kPanel;
  double* rbuf = BX + (size_t)m * kPanel;

  DevCtl* ctl = a.ctl;
  const int q = threadIdx.x;
  const int lane = q & (kWave - 1);
  const int wid = q / kWave;
  const int k0 = a.k0;
  const int p = a.ncols;
  const double* __restrict__ V = a.V;
  const bool row = q < s;

  // ---- every input at once: panel rows, d, estimate vectors --------------
#pragma unroll
  for (int j = 0; j < kPanel; ++j) {
    const int col = k0 + j;
    double v = 0.0;
    if (j < p && row) {
      const double sc = (a.t > 0 ? a.sigma[col] : 1.0) * a.inv_sqrt_zeta;
      v = a.red[(int64_t)(col % a.nring) * a.slot_red + q] * sc;
    }
    if (row) Cp[j * s + q] = v;
  }
  if (row) dv[q] = a.d[q];
  if (q < k0) {
    xv[q] = a.ice_x[q];
    zv[q] = a.ice_z[q];
  }
  if (ctl->stop_k != 0) return;
  __syncthreads();

  // ---- T extended by the previous panel's reflectors kb .. k0-1 ----------
  // (deferred to this launch, where all waves are present; a cycle's last
  // panel never needs it)
  const int pp = a.pprev;
  if (pp > 0) {
    const int kb = k0 - pp;
    const double* Vn = V + (int64_t)kb * s;  // the new reflectors, zero above their units
    // U = V_old^T V_new over rows >= kb
    vt_panel(V, s, kb, kb, Vn, pp, true, AU, m);
    // wm[x][y] = v_{kb+x}^T v_{kb+y} (x < y): wave sums, column y at a time,
    // into the reduction buffer (entry y (y - 1) / 2 + x), then one thread
    // per entry adds the waves in wave order
    {
      double cr[kPanel];
#pragma unroll
      for (int x = 0; x < kPanel; ++x) cr[x] = (row && x < pp && q >= kb + x) ? Vn[(int64_t)x * s + q] : 0.0;
#pragma unroll
      for (int y = 1; y < kPanel; ++y)
#pragma unroll
        for (int x = 0; x < y; ++x) {
          const double w = wave_sum(cr[x] * cr[y]);
          if (lane == 0) rbuf[wid * kRB + y * (y - 1) / 2 + x] = w;
        }
      __syncthreads();  // also publishes AU
      if (q < kPanel * (kPanel - 1) / 2) {
        int y = 1;
        while (y * (y + 1) / 2 <= q) ++y;
        const int x = q - y * (y - 1) / 2;
        double r = 0.0;
        for (int w = 0; w < kQrWaves; ++w) r += rbuf[w * kRB + q];
        sh.wm[x][y] = r;
      }
      if (q < kPanel) sh.tau[q] = q < pp ? a.tau[kb + q] : 0.0;
      __syncthreads();
    }
    // row r = q of X = T_old U, then of the new columns:
    // T(0:kk, kk) = -tau_kk T(0:kk, 0:kk) [U(:, j); wm(0:j, j)], T(kk, kk) = tau_kk
    if (q < k0) {
      double xr[kPanel], tn[kPanel];
#pragma unroll
      for (int j = 0; j < kPanel; ++j) xr[j] = 0.0;
      if (q < kb) {
        int l = q;
        for (; l + 8 <= kb; l += 8) {
          double tv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) tv[u] = a.T[(int64_t)(l + u) * m + q];
#pragma unroll
          for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int j = 0; j < kPanel; ++j) xr[j] += tv[u] * AU[j * m + l + u];
        }
        for (; l < kb; ++l) {
          const double tv = a.T[(int64_t)l * m + q];
#pragma unroll
          for (int j = 0; j < kPanel; ++j) xr[j] += tv * AU[j * m + l];
        }
      }
#pragma unroll
      for (int j = 0; j < kPanel; ++j) {
        const int kk = kb + j;
        tn[j] = 0.0;
        if (q < kk) {
          double acc = xr[j];
#pragma unroll
          for (int jj = 0; jj < j; ++jj)
            if (q <= kb + jj) acc += tn[jj] * sh.wm[jj][j];
          tn[j] = -sh.tau[j] * acc;
        } else if (q == kk) {
          tn[j] = sh.tau[j];
        }
        if (j < pp && q <= kk) a.T[(int64_t)kk * m + q] = tn[j];
      }
    }
    __syncthreads();  // T complete for B = T^T A below
  }
  const double* __restrict__ T = a.T;

  if (k0 > 0) {
    // A = V^T C, then B = T^T A (four columns of T per wave, 16 lanes over
    // its rows), then C <- C - V B (a thread per row)
    vt_panel(V, s, k0, 0, Cp, kPanel, false, AU, m);
    __syncthreads();
    {
      const int c = lane >> 4;
      const int rl = lane & 15;
      for (int lb = wid * 4; lb < k0; lb += kQrWaves * 4) {
        const int l = lb + c;
        const bool has = l < k0;
        double acc[kPanel];
#pragma unroll
        for (int j = 0; j < kPanel; ++j) acc[j] = 0.0;
        const int rmax = lb + 3 < k0 ? lb + 3 : k0 - 1;  // rows of the wave's last column
        for (int r = rl; r <= rmax; r += 16) {
          const double tv = (has && r <= l) ? T[(int64_t)l * m + r] : 0.0;
#pragma unroll
          for (int j = 0; j < kPanel; ++j) acc[j] += tv * AU[j * m + r];
        }
#pragma unroll
        for (int j = 0; j < kPanel; ++j) {
          const double rr = row16_sum(acc[j]);
          if (rl == 0 && has) BX[j * m + l] = rr;
        }
      }
    }
    __syncthreads();
    if (row) {
      double acc[kPanel];
#pragma unroll
      for (int j = 0; j < kPanel; ++j) acc[j] = 0.0;
      int l = 0;
      for (; l + 8 <= k0; l += 8) {
        double vl[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) vl[u] = V[(int64_t)(l + u) * s + q];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int j = 0; j < kPanel; ++j) acc[j] += vl[u] * BX[j * m + l + u];
      }
      for (; l < k0; ++l) {
        const double vl = V[(int64_t)l * s + q];
#pragma unroll
        for (int j = 0; j < kPanel; ++j) acc[j] += vl * BX[j * m + l];
      }
#pragma unroll
      for (int j = 0; j < kPanel; ++j) Cp[j * s + q] -= acc[j];
    }
    __syncthreads();
  }

  // ---- the panel, column by column, in the first kPanelWaves waves --------
  // Column kk = k0 + j: reflector on rows >= kk; d and the later panel
  // columns updated; ||d[kk+1:]|| (C3); Bischof's incremental estimate with
  // the new column [R(0:kk, kk); beta] (C2); the decision.  Thread t owns
  // rows t, t + 256, ... (of the panel, d, x and z); the scalars are computed
  // identically by every panel thread from the reduced sums.  The other
  // waves are done.
  if (wid >= kPanelWaves) return;
  const int t = q;
  const int forced_k = ctl->forced_k;
  const int brk_step = ctl->brk_step;
  const double cond_thr = ctl->cond_threshold;
  const double factor = ctl->factor;
  const double tol_abs = ctl->tol_abs;
  double smax = ctl->ice_smax, znorm = ctl->ice_znorm;
  double cond_cur = ctl->cond_cur, cond_prev = ctl->cond_prev;
  double rho_cur = ctl->rho_cur, rho_prev = ctl->rho_prev;
  int err = ctl->error;
  int par = 0;
  double beta, tau, den;
  {
    double r2[2] = {0.0, 0.0};
#pragma unroll
    for (int u = 0; u < kRowsPT; ++u) {
      const int r = t + u * kPanelThreads;
      if (r < s) {
        const double c0 = Cp[r];
        if (r > k0) r2[0] += c0 * c0;
        if (r == k0) r2[1] = c0;
      }
    }
    panel_sum<2>(r2, rbuf, par);
    reflector(r2[1], r2[0], beta, tau, den);
  }
  int stop_k = 0, stop_step = 0, stop_reason = 0, qr_k = k0;
  int stopped = 0;
  int done = k0;
  for (int j = 0; j < p; ++j) {
    const int kk = k0 + j;
    if (brk_step == kk) {
      // this column's Arnoldi vector is zero: keep the kk columns before it
      stop_k = kk;
      stop_step = kk;
      stop_reason = SFGMRES_STOP_BREAKDOWN;
      stopped = 1;
      break;
    }
    if (t == 0) {
      sh.tau[j] = tau;
      sh.beta[j] = beta;
    }
    double* cj = Cp + j * s;
    const double inv = den != 0.0 ? 1.0 / den : 0.0;
    // v^T d, v^T C[:, j'] (j' > j; the others masked below) and the
    // estimate's x^T r, z^T r with r = R's new column (rows < kk of column j)
    double red[kPanel + 3];
#pragma unroll
    for (int i = 0; i < kPanel + 3; ++i) red[i] = 0.0;
#pragma unroll
    for (int u = 0; u < kRowsPT; ++u) {
      const int r = t + u * kPanelThreads;
      if (r < s) {
        const double c = cj[r];
        const double dr = dv[r];
        const int ri = r < kk ? r : 0;  // (x and z hold m entries)
        const double xr = r < kk ? xv[ri] : 0.0;
        const double zr = r < kk ? zv[ri] : 0.0;
        double cc[kPanel];
#pragma unroll
        for (int jj = 0; jj < kPanel; ++jj) cc[jj] = Cp[jj * s + r];
        const double v = r < kk ? 0.0 : (r == kk ? 1.0 : c * inv);
        const double rc = r < kk ? c : 0.0;
        red[0] += v * dr;
#pragma unroll
        for (int jj = 0; jj < kPanel; ++jj) red[1 + jj] += v * cc[jj];
        red[kPanel + 1] += xr * rc;
        red[kPanel + 2] += zr * rc;
      }
    }
    panel_sum<kPanel + 3>(red, rbuf, par);
    // the reflector replaces rows >= kk of column j (rows < kk hold R's new
    // column); d <- H d, C[:, j'] <- H C[:, j'] for j' > j; ||d[kk+1:]||^2
    // and the next column's squared tail and pivot (branch-free: columns
    // jj < j keep their values, every column of the row is stored)
    double rm[kPanel];
#pragma unroll
    for (int jj = 0; jj < kPanel; ++jj) rm[jj] = jj > j ? red[1 + jj] : 0.0;
    double r3[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < kRowsPT; ++u) {
      const int r = t + u * kPanelThreads;
      if (r < s && r >= kk) {
        double x[kPanel];
#pragma unroll
        for (int jj = 0; jj < kPanel; ++jj) x[jj] = Cp[jj * s + r];
        const double dr = dv[r];
        double v = 0.0;
#pragma unroll
        for (int jj = 0; jj < kPanel; ++jj)
          if (jj == j) v = r == kk ? 1.0 : x[jj] * inv;
        const double tv = tau * v;
        const double dn = dr - tv * red[0];
        double nn = 0.0;
#pragma unroll
        for (int jj = 0; jj < kPanel; ++jj) {
          x[jj] = jj == j ? v : x[jj] - tv * rm[jj];
          if (jj == j + 1) nn = x[jj];
        }
        dv[r] = dn;
#pragma unroll
        for (int jj = 0; jj < kPanel; ++jj) Cp[jj * s + r] = x[jj];
        if (r > kk) r3[0] += dn * dn;
        if (r > kk + 1) r3[1] += nn * nn;
        if (r == kk + 1) r3[2] = nn;
      }
    }
    panel_sum<3>(r3, rbuf, par);
    const double rho_hat = sqrt(r3[0]);
    const double ax = red[kPanel + 1], bz = red[kPanel + 2];
    const double gam = beta;
    double kappa;
    if (gam == 0.0 || smax < 0.0) {
      smax = -1.0;  // singular from here on
      kappa = INFINITY;
    } else if (kk == 0) {
      smax = fabs(gam);
      znorm = 1.0 / fabs(gam);
      kappa = smax * znorm;
      if (t == 0) {
        xv[0] = 1.0;
        zv[0] = 1.0 / gam;
      }
    } else {
      double lam, s1, c1, s2, c2;
      top_eig2(smax * smax + ax * ax, ax * gam, gam * gam, lam, s1, c1);
      smax = sqrt(lam);
      const double g2 = gam * gam;
      top_eig2(znorm * znorm + bz * bz / g2, -bz / g2, 1.0 / g2, lam, s2, c2);
      znorm = sqrt(lam);
      kappa = smax * znorm;
#pragma unroll
      for (int u = 0; u < kRowsPT; ++u) {
        const int r = t + u * kPanelThreads;
        if (r < kk) {
          xv[r] *= s1;
          zv[r] *= s2;
        } else if (r == kk) {
          xv[kk] = c1;
          zv[kk] = (c2 - s2 * bz) / gam;
        }
      }
    }
    const int ncols = kk + 1;
    qr_k = ncols;
    cond_prev = cond_cur;
    rho_prev = rho_cur;
    cond_cur = kappa;
    rho_cur = rho_hat;
    int stop = 0, reason = 0;
    if (ncols == 1 && beta == 0.0) {
      err = SFGMRES_ERR_BREAKDOWN;
      stop = 1;
      reason = SFGMRES_STOP_BREAKDOWN;
    } else if (forced_k > 0) {
      if (ncols >= forced_k) {
        stop = forced_k;
        reason = SFGMRES_STOP_FORCED;
      }
    } else if (ncols > 1 && kappa > cond_thr) {
      stop = ncols - 1;
      reason = SFGMRES_STOP_C2;
    } else if (factor * rho_hat <= tol_abs) {
      stop = ncols;
      reason = SFGMRES_STOP_C3;
    } else if (ncols >= m) {
      stop = m;
      reason = SFGMRES_STOP_C1;
    }
    if (!isfinite(rho_hat) && err == 0) err = SFGMRES_ERR_NONFINITE;
    done = ncols;
    if (stop) {
      stop_k = stop;
      stop_step = ncols;
      stop_reason = reason;
      stopped = 1;
      break;
    }
    reflector(r3[2], r3[1], beta, tau, den);
  }
  const int ndone = done - k0;  // columns whose reflector was formed
  if (t == 0) {
    ctl->stop_k = stop_k;
    ctl->stop_step = stop_step;
    ctl->stop_reason = stop_reason;
    ctl->qr_k = qr_k;
    ctl->error = err;
    ctl->ice_smax = smax;
    ctl->ice_znorm = znorm;
    ctl->cond_cur = cond_cur;
    ctl->cond_prev = cond_prev;
    ctl->rho_cur = rho_cur;
    ctl->rho_prev = rho_prev;
  }
  __syncthreads();  // sh.tau, sh.beta and the panel rows for the write-back

  // ---- write back (V, R and tau of the formed columns; d; x and z) --------
  for (int j = 0; j < ndone; ++j) {
    const int kk = k0 + j;
#pragma unroll
    for (int u = 0; u < kRowsPT; ++u) {
      const int r = t + u * kPanelThreads;
      if (r < s) {
        const double cjr = Cp[j * s + r];
        a.V[(int64_t)kk * s + r] = r < kk ? 0.0 : cjr;
        if (r < kk) a.R[(int64_t)kk * m + r] = cjr;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kRowsPT; ++u) {
    const int r = t + u * kPanelThreads;
    if (r < s) a.d[r] = dv[r];
    if (r >= k0 && r < done) {
      a.R[(int64_t)r * m + r] = sh.beta[r - k0];
      a.tau[r] = sh.tau[r - k0];
    }
    if (r < done) {
      a.ice_x[r] = xv[r];
      a.ice_z[r] = zv[r];
    }
  }
  if (t == 0) {
    (void)stopped;
    host_store_i32(&a.hs->stop_k, stop_k);
    host_store_i32(&a.hs->stop_step, stop_step);
    host_store_i32(&a.hs->stop_reason, stop_reason);
    host_store_i32(&a.hs->error, err);
    host_store_i32(&a.hs->steps_run, k0 + p);
    host_store_i32(&a.hs->inner_step_done, done);
  }
}

hipError_t launch_qr_block(const QrBlockArgs& a, hipStream_t st) {
  const size_t lds = qr_block_lds_bytes(a.s, a.m);
  static bool attr_set = false;
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_qr_block),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)qr_block_lds_bytes(kMaxS, kMaxM));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_qr_block, dim3(1), dim3(kQrThreads), lds, st, a);
  return hipGetLastError();
}

// d0 = S v_j (reduced, times 1/sqrt(zeta)); reset the inner-cycle state.
__global__ __launch_bounds__(256) void k_rq_init(const double* red, int32_t s, double inv_sqrt_zeta,
                                                 int32_t forced_k, DevCtl* ctl, double* d,
                                                 double* sigma) {
  __shared__ double scratch[256 / kWave];
  double nrm = 0.0;
  for (int q = threadIdx.x; q < s; q += blockDim.x) {
    const double v = red[q] * inv_sqrt_zeta;
    d[q] = v;
    nrm += v * v;
  }
  nrm = block_sum(nrm, scratch);
  if (threadIdx.x == 0) {
    ctl->d0norm = sqrt(nrm);
    ctl->stop_k = 0;
    ctl->stop_step = 0;
    ctl->stop_reason = 0;
    ctl->qr_k = 0;
    ctl->forced_k = forced_k;
    ctl->ice_smax = 0.0;
    ctl->ice_znorm = 0.0;
    ctl->cond_cur = ctl->cond_prev = 0.0;
    ctl->rho_cur = ctl->rho_prev = 0.0;
    ctl->brk_step = -1;
    sigma[0] = 1.0;
  }
}

hipError_t launch_rq_init(const double* red, int32_t s, double inv_sqrt_zeta, int32_t forced_k,
                          DevCtl* ctl, double* d, double* sigma, hipStream_t st) {
  hipLaunchKernelGGL(k_rq_init, dim3(1), dim3(256), 0, st, red, s, inv_sqrt_zeta, forced_k, ctl,
                     d, sigma);
  return hipGetLastError();
}

// Test export of one fused SpMV: the reduced sketch times 1/sqrt(zeta), the
// window dots and ||w||^2 summed from the scalar rows in slot order.
__global__ __launch_bounds__(256) void k_sketch_out(const double* red, int32_t s,
                                                    double inv_sqrt_zeta, const double* dpart,
                                                    int32_t G, int32_t nwin, double* out_c,
                                                    double* out_dots, double* out_norm2) {
  __shared__ double scratch[256 / kWave];
  for (int q = threadIdx.x; q < s; q += blockDim.x) out_c[q] = red[q] * inv_sqrt_zeta;
  if (!dpart) return;
  for (int l = 0; l < nwin; ++l) {
    const double v = block_sum_strided(dpart + l, G, kDP, scratch);
    if (threadIdx.x == 0 && out_dots) out_dots[l] = v;
  }
  const double v = block_sum_strided(dpart + kMaxT, G, kDP, scratch);
  if (threadIdx.x == 0 && out_norm2) out_norm2[0] = v;
}

hipError_t launch_sketch_out(const double* red, int32_t s, double inv_sqrt_zeta,
                             const double* dpart, int32_t G, int32_t nwin, double* out_c,
                             double* out_dots, double* out_norm2, hipStream_t st) {
  hipLaunchKernelGGL(k_sketch_out, dim3(1), dim3(256), 0, st, red, s, inv_sqrt_zeta, dpart, G,
                     nwin, out_c, out_dots, out_norm2);
  return hipGetLastError();
}

}  // namespace sfg
