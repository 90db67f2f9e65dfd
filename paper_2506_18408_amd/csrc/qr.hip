// Reduce and decide: the sketched least-squares step of one inner sGMRES
// step (Section 3).
//
// k_reduce_rows (many workgroups) combines the per-workgroup partial rows of
// the fused SpMV (raw sketch S y, truncated-Arnoldi dots, ||y||^2), each
// workgroup summing a 16-entry slice over all rows in slot order.
//
// k_rq (one workgroup) then, in float64:
//   * forms sigma_i = 1/||u_i|| of the current (unnormalised) Arnoldi vector
//     from the norm partials of the previous Arnoldi update, and the new
//     column c_i = S A b_i / sqrt(zeta) of S A B_i (b_i = sigma_i u_i; for
//     t > 0 the SpMV returned y = A u_i, for t = 0 already y = A b_i);
//   * appends c_i to the Householder QR of S A B_i (compact-WY form
//     Q = I - V T V^T: c <- c - V T^T V^T c, a new reflector for c[i:],
//     T extended by -tau T V^T v), carries d = Q^T S v_j along, and reads the
//     sketched least-squares residual ||d[i+1:]|| (the estimate used by C3);
//   * extends the incremental condition estimate of R (Bischof's ICE: top
//     eigenpairs of two 2x2 matrices);
//   * applies C2 (estimate above threshold: drop column i), C3 (bound of
//     eq. (2.2) below tol), C1 (i = m), or a forced replay dimension;
//   * stores the truncated-Arnoldi coefficients sigma_i sigma_l^2 <y, u_l>
//     and the scale sigma_i of y for the vector update, or, for t = 0, the
//     scale of the next power-basis vector.
// The mode kRqInit instead takes d0 = S v_j and resets the cycle state.
#include "kernels.hpp"

namespace sfg {

constexpr int kRqThreads = 1024;
constexpr int kRedThreads = 1024;
constexpr int kRedSlice = 16;  // entries per reduction workgroup

__global__ __launch_bounds__(kRedThreads) void k_reduce_rows(const double* __restrict__ part,
                                                             int32_t G, int32_t E,
                                                             double* __restrict__ red,
                                                             const DevCtl* ctl, int predicated) {
  __shared__ double sl[kRedThreads];
  if (predicated && ctl->stop_k != 0) return;
  const int tid = threadIdx.x;
  const int e = blockIdx.x * kRedSlice + (tid % kRedSlice);
  const int rg = tid / kRedSlice;
  constexpr int nrg = kRedThreads / kRedSlice;
  double acc = 0.0;
  if (e < E)
    for (int r = rg; r < G; r += nrg) acc += part[(int64_t)r * E + e];
  sl[tid] = acc;
  __syncthreads();
  if (tid < kRedSlice) {
    double t = 0.0;
    for (int r = 0; r < nrg; ++r) t += sl[r * kRedSlice + tid];
    if (e < E) red[e] = t;
  }
}

hipError_t launch_reduce_rows(const double* part, int32_t G, int32_t E, double* red,
                              const DevCtl* ctl, bool predicated, hipStream_t st) {
  const int nb = (E + kRedSlice - 1) / kRedSlice;
  hipLaunchKernelGGL(k_reduce_rows, dim3(nb), dim3(kRedThreads), 0, st, part, G, E, red, ctl,
                     predicated ? 1 : 0);
  return hipGetLastError();
}

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

__device__ static void publish_inner(HostStatus* hs, const DevCtl* c, int done) {
  host_store_i32(&hs->stop_k, c->stop_k);
  host_store_i32(&hs->stop_step, c->stop_step);
  host_store_i32(&hs->stop_reason, c->stop_reason);
  host_store_i32(&hs->error, c->error);
  __threadfence_system();
  host_store_i32(&hs->inner_step_done, done);
  __threadfence_system();
}

__global__ __launch_bounds__(kRqThreads) void k_rq(RqArgs a, int mode) {
  __shared__ double scratch[kRqThreads / kWave];
  __shared__ double cv[kMaxS];
  __shared__ double av[kMaxM];
  __shared__ double bv[kMaxM];
  __shared__ double bc[8];

  DevCtl* ctl = a.ctl;
  if (mode == kRqStep && ctl->stop_k != 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wid = tid / kWave;
  constexpr int nw = kRqThreads / kWave;

  const int s = a.s;
  const int m = a.m;
  const double* red = a.red;

  if (mode == kRqReduce) {
    for (int q = tid; q < s; q += kRqThreads) a.out_c[q] = red[q] * a.inv_sqrt_zeta;
    if (a.out_dots && tid < a.nwin) a.out_dots[tid] = red[s + tid];
    if (a.out_norm2 && tid == 0) a.out_norm2[0] = red[s + kMaxT];
    return;
  }

  if (mode == kRqInit) {
    double nrm = 0.0;
    for (int q = tid; q < s; q += kRqThreads) {
      const double v = red[q] * a.inv_sqrt_zeta;
      a.d[q] = v;
      nrm += v * v;
    }
    nrm = block_sum(nrm, scratch);
    if (tid == 0) {
      ctl->d0norm = sqrt(nrm);
      ctl->stop_k = 0;
      ctl->stop_step = 0;
      ctl->stop_reason = 0;
      ctl->qr_k = 0;
      ctl->forced_k = a.forced_k;
      ctl->ice_smax = 0.0;
      ctl->ice_znorm = 0.0;
      ctl->cond_cur = ctl->cond_prev = 0.0;
      ctl->rho_cur = ctl->rho_prev = 0.0;
      a.sigma[0] = 1.0;
    }
    return;
  }

  // ---- kRqStep: one column appended to the sketched QR -------------------
  const int k = ctl->qr_k;  // existing columns; the new one has index k
  const int step = a.step;  // == k
  // sigma_i of the current Arnoldi vector u_i
  if (a.t > 0 && step > 0) {
    const double n2u = block_sum_strided(a.vpart, a.Gv, 1, scratch);
    if (n2u == 0.0) {
      // u_i = 0: truncated Arnoldi broke down; keep the i columns built so far
      if (tid == 0) {
        ctl->stop_k = step;
        ctl->stop_step = step;
        ctl->stop_reason = SFGMRES_STOP_BREAKDOWN;
        publish_inner(a.hs, ctl, step);
      }
      return;
    }
    if (tid == 0) bc[0] = 1.0 / sqrt(n2u);
  } else if (tid == 0) {
    bc[0] = a.sigma[step];
  }
  __syncthreads();
  const double sig = bc[0];
  if (tid == 0) a.sigma[step] = sig;
  const double cscale = (a.t > 0 ? sig : 1.0) * a.inv_sqrt_zeta;
  for (int q = tid; q < s; q += kRqThreads) cv[q] = red[q] * cscale;
  __syncthreads();

  // a = V^T c  (column l of V is zero above row l, one at row l)
  for (int l = wid; l < k; l += nw) {
    double acc = 0.0;
    for (int q = l + lane; q < s; q += kWave) acc += a.V[(int64_t)l * s + q] * cv[q];
    acc = wave_sum(acc);
    if (lane == 0) av[l] = acc;
  }
  __syncthreads();
  // b = T^T a  (T upper triangular, row-major)
  for (int l = tid; l < k; l += kRqThreads) {
    double acc = 0.0;
    for (int p = 0; p <= l; ++p) acc += a.T[(int64_t)p * m + l] * av[p];
    bv[l] = acc;
  }
  __syncthreads();
  // c <- c - V b
  for (int q = tid; q < s; q += kRqThreads) {
    double acc = 0.0;
    const int lmax = q < k - 1 ? q : k - 1;
    for (int l = 0; l <= lmax; ++l) acc += a.V[(int64_t)l * s + q] * bv[l];
    cv[q] -= acc;
  }
  __syncthreads();
  // new reflector for c[k:]
  double x2 = 0.0;
  for (int q = k + 1 + tid; q < s; q += kRqThreads) x2 += cv[q] * cv[q];
  x2 = block_sum(x2, scratch);
  if (tid == 0) {
    const double alpha = cv[k];
    double beta, tau, den;
    if (x2 == 0.0) {
      beta = alpha;
      tau = 0.0;
      den = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + x2), alpha);
      tau = (beta - alpha) / beta;
      den = alpha - beta;
    }
    bc[0] = beta;
    bc[1] = tau;
    bc[2] = den;
    a.tau[k] = tau;
    a.R[(int64_t)k * m + k] = beta;
  }
  __syncthreads();
  const double beta = bc[0];
  const double tau = bc[1];
  const double den = bc[2];
  // store the reflector (unit at row k) in V and the new column of R
  for (int q = tid; q < s; q += kRqThreads) {
    double v;
    if (q < k)
      v = 0.0;
    else if (q == k)
      v = 1.0;
    else
      v = den != 0.0 ? cv[q] / den : 0.0;
    a.V[(int64_t)k * s + q] = v;
    if (q < k) a.R[(int64_t)k * m + q] = cv[q];
    if (q > k) cv[q] = v;
  }
  if (tid == 0) cv[k] = 1.0;
  __syncthreads();
  // keep R's new column (rows < k; cv[0:k] is untouched above) for the estimate
  for (int p = tid; p < k; p += kRqThreads) bv[p] = cv[p];
  __syncthreads();
  // u = V_old^T v_k (over rows >= k) -> av
  for (int l = wid; l < k; l += nw) {
    double acc = 0.0;
    for (int q = k + lane; q < s; q += kWave) acc += a.V[(int64_t)l * s + q] * cv[q];
    acc = wave_sum(acc);
    if (lane == 0) av[l] = acc;
  }
  __syncthreads();
  // T[:k, k] = -tau T[:k, :k] u ; T[k, k] = tau
  for (int p = wid; p < k; p += nw) {
    double acc = 0.0;
    for (int l = p + lane; l < k; l += kWave) acc += a.T[(int64_t)p * m + l] * av[l];
    acc = wave_sum(acc);
    if (lane == 0) a.T[(int64_t)p * m + k] = -tau * acc;
  }
  if (tid == 0) a.T[(int64_t)k * m + k] = tau;
  // d <- H_k d
  double dl = 0.0;
  for (int q = k + tid; q < s; q += kRqThreads) dl += cv[q] * a.d[q];
  dl = block_sum(dl, scratch);
  for (int q = k + tid; q < s; q += kRqThreads) a.d[q] -= tau * cv[q] * dl;
  __syncthreads();
  double rr = 0.0;
  for (int q = k + 1 + tid; q < s; q += kRqThreads) rr += a.d[q] * a.d[q];
  rr = block_sum(rr, scratch);
  const double rho_hat = sqrt(rr);

  // incremental condition estimate with the new column [bv[0:k]; beta]
  double ax = 0.0, bz = 0.0;
  for (int p = tid; p < k; p += kRqThreads) {
    ax += a.ice_x[p] * bv[p];
    bz += a.ice_z[p] * bv[p];
  }
  ax = block_sum(ax, scratch);
  bz = block_sum(bz, scratch);
  if (tid == 0) {
    const double gam = beta;
    double kappa;
    if (gam == 0.0 || ctl->ice_smax < 0.0) {
      ctl->ice_smax = -1.0;  // singular from here on
      kappa = INFINITY;
      bc[3] = 0.0;
      bc[4] = 0.0;
      bc[5] = 0.0;
      bc[6] = 0.0;
    } else if (k == 0) {
      ctl->ice_smax = fabs(gam);
      ctl->ice_znorm = 1.0 / fabs(gam);
      a.ice_x[0] = 1.0;
      a.ice_z[0] = 1.0 / gam;
      kappa = ctl->ice_smax * ctl->ice_znorm;
      bc[3] = 0.0;
    } else {
      double lam, vs, vc;
      const double sm = ctl->ice_smax;
      top_eig2(sm * sm + ax * ax, ax * gam, gam * gam, lam, vs, vc);
      bc[3] = vs;
      bc[4] = vc;
      ctl->ice_smax = sqrt(lam);
      const double zn = ctl->ice_znorm;
      const double g2 = gam * gam;
      top_eig2(zn * zn + bz * bz / g2, -bz / g2, 1.0 / g2, lam, vs, vc);
      bc[5] = vs;
      bc[6] = vc;
      ctl->ice_znorm = sqrt(lam);
      kappa = ctl->ice_smax * ctl->ice_znorm;
    }
    bc[7] = kappa;
  }
  __syncthreads();
  if (k > 0 && bc[7] < INFINITY) {
    const double s1 = bc[3], c1 = bc[4], s2 = bc[5], c2 = bc[6];
    for (int p = tid; p < k; p += kRqThreads) {
      a.ice_x[p] *= s1;
      a.ice_z[p] *= s2;
    }
    if (tid == 0) {
      a.ice_x[k] = c1;
      a.ice_z[k] = (c2 - s2 * bz) / beta;
    }
  }

  if (tid == 0) {
    const double kappa = bc[7];
    const int ncols = k + 1;
    ctl->qr_k = ncols;
    ctl->cond_prev = ctl->cond_cur;
    ctl->rho_prev = ctl->rho_cur;
    ctl->cond_cur = kappa;
    ctl->rho_cur = rho_hat;
    int stop = 0, reason = 0;
    if (ncols == 1 && beta == 0.0) {
      ctl->error = SFGMRES_ERR_BREAKDOWN;
      stop = 1;
      reason = SFGMRES_STOP_BREAKDOWN;
    } else if (ctl->forced_k > 0) {
      if (ncols >= ctl->forced_k) {
        stop = ctl->forced_k;
        reason = SFGMRES_STOP_FORCED;
      }
    } else if (ncols > 1 && kappa > ctl->cond_threshold) {
      stop = ncols - 1;
      reason = SFGMRES_STOP_C2;
    } else if (ctl->factor * rho_hat <= ctl->tol_abs) {
      stop = ncols;
      reason = SFGMRES_STOP_C3;
    } else if (ncols >= m) {
      stop = m;
      reason = SFGMRES_STOP_C1;
    }
    if (!stop) {
      if (a.t == 0) {
        // power basis: the next vector is y = A b_i itself; sigma_{i+1} = 1/||y||
        const double n2 = red[s + kMaxT];
        if (n2 == 0.0) {
          stop = ncols;
          reason = SFGMRES_STOP_BREAKDOWN;
        } else {
          a.sigma[step + 1] = 1.0 / sqrt(n2);
        }
      } else {
        // u_{i+1} = sigma_i y - sum_l sigma_i sigma_l^2 <y, u_l> u_l: A b_i
        // minus its projections h_l b_l on the window b_l = sigma_l u_l,
        // h_l = sigma_i sigma_l <y, u_l>; ||u_{i+1}|| = h_{i+1,i}
        for (int l = 0; l < a.nwin; ++l) {
          const double sg = (a.l0 + l == step) ? sig : a.sigma[a.l0 + l];
          a.coef[l] = sig * sg * sg * red[s + l];
        }
        a.coef[kMaxT] = sig;
      }
    }
    if (!isfinite(rho_hat) && ctl->error == 0) ctl->error = SFGMRES_ERR_NONFINITE;
    if (stop) {
      ctl->stop_k = stop;
      ctl->stop_step = step + 1;
      ctl->stop_reason = reason;
    }
    publish_inner(a.hs, ctl, step + 1);
  }
}

hipError_t launch_rq(int mode, const RqArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_rq, dim3(1), dim3(kRqThreads), 0, st, a, mode);
  return hipGetLastError();
}

}  // namespace sfg
