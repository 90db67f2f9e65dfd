// Zero-fill ILU right preconditioning (the "-p" runs of the paper's Section
// 4.4 and Table 1): M = L U on A's pattern, applied to every inner basis
// vector (the inner operator is A M^{-1}) and to the inner solution
// (z_j = M^{-1} B_k y_k).
//
// Elimination order: by colour of a proper colouring of the symmetrised
// graph of A, then by index.  Unknowns of one colour are never coupled, so
// each colour is one level of the factorisation and of each triangular
// solve, run as one launch over the rows of that colour (one thread per
// row).  The colouring is Jones & Plassmann's: in rounds, every uncoloured
// vertex whose priority p(i) = (2654435761 i) mod 2^32 beats every
// neighbour that was uncoloured when the round began takes the smallest
// colour that none of its coloured neighbours has.  Two such vertices are
// never adjacent, so the vertices of a round colour themselves independently;
// each vertex's state is one 32-bit word (round << 12 | colour, or -1), so a
// reader sees either the state before the round or the final one.
//
// Factorisation: the IKJ form of Gaussian elimination restricted to the
// pattern (Saad, Section 10.3.2): row i takes its entries of lower colour in
// (colour, index) order, divides each by the pivot of its row k and
// subtracts l_ik u_kj from every entry a_ij of its own pattern with colour(j)
// > colour(k).  Rows of earlier colours are final (earlier launches); every
// thread writes only its own row.
#include "kernels.hpp"

namespace sfg {

constexpr int kIluThreads = 256;

__device__ __forceinline__ uint32_t ilu_priority(int64_t i) {
  return (uint32_t)((uint64_t)i * 2654435761ull);
}

// Factor values start as A's; diagonal positions; every row must list its
// columns in increasing order with the diagonal present (err bits 1, 2).
__global__ void k_ilu_init(int64_t n, const int32_t* __restrict__ rp,
                           const int32_t* __restrict__ ci, const double* __restrict__ val,
                           double* __restrict__ lu, int32_t* __restrict__ diag,
                           int32_t* __restrict__ state, int32_t* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int q0 = rp[i], q1 = rp[i + 1];
    int d = -1;
    int prev = -1;
    bool sorted = true;
    for (int q = q0; q < q1; ++q) {
      const int c = ci[q];
      lu[q] = val[q];
      if (c <= prev) sorted = false;
      prev = c;
      if (c == (int)i) d = q;
    }
    diag[i] = d;
    state[i] = -1;
    if (!sorted) atomicOr(err, 1);
    if (d < 0) atomicOr(err, 2);
  }
}

// One Jones-Plassmann round r: neighbours are the columns of row i of A and
// of A^T (CSR of the transpose), the diagonal excluded.
__global__ void k_ilu_jp_round(int64_t n, const int32_t* __restrict__ rp,
                               const int32_t* __restrict__ ci, const int32_t* __restrict__ rpt,
                               const int32_t* __restrict__ cit, int32_t* state, int32_t r,
                               int32_t* colored, int32_t* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (state[i] != -1) continue;
    const uint32_t pi = ilu_priority(i);
    // a neighbour uncoloured when the round began: state -1, or coloured in
    // this very round
    auto open_at_start = [&](int32_t st) { return st == -1 || (st >> 12) == r; };
    bool is_max = true;
    for (int pass = 0; pass < 2 && is_max; ++pass) {
      const int32_t* P = pass ? rpt : rp;
      const int32_t* C = pass ? cit : ci;
      for (int q = P[i]; q < P[i + 1]; ++q) {
        const int j = C[q];
        if (j == (int)i) continue;
        if (open_at_start(state[j]) && ilu_priority(j) > pi) {
          is_max = false;
          break;
        }
      }
    }
    if (!is_max) continue;
    // smallest colour not held by a neighbour coloured in an earlier round:
    // colours below 64 through a bit mask, then a scan per candidate
    uint64_t low = 0;
    int cmax = -1;
    for (int pass = 0; pass < 2; ++pass) {
      const int32_t* P = pass ? rpt : rp;
      const int32_t* C = pass ? cit : ci;
      for (int q = P[i]; q < P[i + 1]; ++q) {
        const int j = C[q];
        if (j == (int)i) continue;
        const int32_t st = state[j];
        if (open_at_start(st)) continue;
        const int c = st & 0xFFF;
        if (c < 64) low |= 1ull << c;
        cmax = c > cmax ? c : cmax;
      }
    }
    int c = 0;
    if (~low != 0ull) {
      c = __builtin_ctzll(~low);
    } else {
      c = 64;
      for (;; ++c) {
        bool used = false;
        for (int pass = 0; pass < 2 && !used; ++pass) {
          const int32_t* P = pass ? rpt : rp;
          const int32_t* C = pass ? cit : ci;
          for (int q = P[i]; q < P[i + 1]; ++q) {
            const int j = C[q];
            const int32_t st = state[j];
            if (j != (int)i && !open_at_start(st) && (st & 0xFFF) == c) {
              used = true;
              break;
            }
          }
        }
        if (!used) break;
      }
    }
    if (c >= kIluMaxColors) {
      atomicOr(err, 4);
      c = kIluMaxColors - 1;
    }
    state[i] = (r << 12) | c;
    atomicAdd(colored, 1);
  }
}

// Rows per colour (and the number of colours).
__global__ void k_ilu_count(int64_t n, const int32_t* __restrict__ state, int32_t* cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    atomicAdd(&cnt[state[i] & 0xFFF], 1);
}

// Level lists: the rows of colour c in order[start[c] .. start[c+1]) (in
// any order inside a colour: their computations are independent); the
// entry kinds (-1: colour below the row's, i.e. L; 0: diagonal; +1: U).
__global__ void k_ilu_scatter(int64_t n, const int32_t* __restrict__ rp,
                              const int32_t* __restrict__ ci, const int32_t* __restrict__ state,
                              const int32_t* __restrict__ start, int32_t* cursor,
                              int32_t* __restrict__ order, int8_t* __restrict__ kind) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int c = state[i] & 0xFFF;
    order[start[c] + atomicAdd(&cursor[c], 1)] = (int32_t)i;
    for (int q = rp[i]; q < rp[i + 1]; ++q) {
      const int j = ci[q];
      const int cj = state[j] & 0xFFF;
      kind[q] = j == (int)i ? 0 : (cj < c ? -1 : 1);
    }
  }
}

// Position of column j in row i (sorted columns), or -1.
__device__ __forceinline__ int find_col(const int32_t* __restrict__ ci, int q0, int q1, int j) {
  int lo = q0, hi = q1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (ci[mid] < j)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < q1 && ci[lo] == j) ? lo : -1;
}

// One colour of the factorisation.
__global__ __launch_bounds__(kIluThreads) void k_ilu_factor(
    const int32_t* __restrict__ order, int32_t begin, int32_t end, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ ci, const int8_t* __restrict__ kind,
    const int32_t* __restrict__ diag, const int32_t* __restrict__ state, double* lu,
    int32_t* err) {
  const int idx = begin + blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= end) return;
  const int i = order[idx];
  const int q0 = rp[i], q1 = rp[i + 1];
  const int ci_col = state[i] & 0xFFF;
  // lower entries in (colour, index) order: colours ascending, then the
  // row's own (index) order
  for (int cc = 0; cc < ci_col; ++cc) {
    for (int q = q0; q < q1; ++q) {
      if (kind[q] != -1) continue;
      const int k = ci[q];
      if ((state[k] & 0xFFF) != cc) continue;
      const double piv = lu[diag[k]];
      if (piv == 0.0) {
        atomicOr(err, 8);
        return;
      }
      const double l = lu[q] / piv;
      lu[q] = l;
      const int ck = cc;
      for (int r = rp[k]; r < rp[k + 1]; ++r) {
        const int j = ci[r];
        if (j == k || (state[j] & 0xFFF) <= ck) continue;  // (colour(j) > colour(k) only)
        const int p = find_col(ci, q0, q1, j);
        if (p >= 0) lu[p] -= l * lu[r];
      }
    }
  }
  if (lu[diag[i]] == 0.0) atomicOr(err, 8);
}

// One colour of the forward solve L t = in (t in FP64), or of the backward
// solve U t = t with the result also written to out (the vector type of
// the caller).  In place: t_k of earlier colours are final.
template <typename VT, bool kForward>
__global__ __launch_bounds__(kIluThreads) void k_ilu_solve(
    const int32_t* __restrict__ order, int32_t begin, int32_t end, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ ci, const int8_t* __restrict__ kind,
    const int32_t* __restrict__ diag, const double* __restrict__ lu, const VT* __restrict__ in,
    double* t, VT* __restrict__ out, const DevCtl* ctl) {
  const int idx = begin + blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= end) return;
  if (ctl && ctl->stop_k != 0) return;
  const int i = order[idx];
  double acc = kForward ? static_cast<double>(in[i]) : t[i];
  const int8_t want = kForward ? -1 : 1;
  for (int q = rp[i]; q < rp[i + 1]; ++q)
    if (kind[q] == want) acc -= lu[q] * t[ci[q]];
  if (kForward) {
    t[i] = acc;
  } else {
    const double z = acc / lu[diag[i]];
    t[i] = z;
    out[i] = static_cast<VT>(z);
  }
}

__global__ void k_ilu_colors(int64_t n, const int32_t* __restrict__ state,
                             int32_t* __restrict__ color) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    color[i] = state[i] & 0xFFF;
}

static int ilu_grid(int64_t n) {
  const int64_t g = (n + kIluThreads - 1) / kIluThreads;
  return (int)(g < 2048 ? (g > 0 ? g : 1) : 2048);
}

hipError_t launch_ilu_init(int64_t n, const int32_t* rp, const int32_t* ci, const double* val,
                           double* lu, int32_t* diag, int32_t* state, int32_t* err,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_ilu_init, dim3(ilu_grid(n)), dim3(kIluThreads), 0, st, n, rp, ci, val,
                     lu, diag, state, err);
  return hipGetLastError();
}

hipError_t launch_ilu_jp_round(int64_t n, const int32_t* rp, const int32_t* ci,
                               const int32_t* rpt, const int32_t* cit, int32_t* state,
                               int32_t round, int32_t* colored, int32_t* err, hipStream_t st) {
  hipLaunchKernelGGL(k_ilu_jp_round, dim3(ilu_grid(n)), dim3(kIluThreads), 0, st, n, rp, ci, rpt,
                     cit, state, round, colored, err);
  return hipGetLastError();
}

hipError_t launch_ilu_colors(int64_t n, const int32_t* state, int32_t* color, hipStream_t st) {
  hipLaunchKernelGGL(k_ilu_colors, dim3(ilu_grid(n)), dim3(kIluThreads), 0, st, n, state, color);
  return hipGetLastError();
}

hipError_t launch_ilu_count(int64_t n, const int32_t* state, int32_t* cnt, hipStream_t st) {
  hipLaunchKernelGGL(k_ilu_count, dim3(ilu_grid(n)), dim3(kIluThreads), 0, st, n, state, cnt);
  return hipGetLastError();
}

hipError_t launch_ilu_scatter(int64_t n, const int32_t* rp, const int32_t* ci,
                              const int32_t* state, const int32_t* start, int32_t* cursor,
                              int32_t* order, int8_t* kind, hipStream_t st) {
  hipLaunchKernelGGL(k_ilu_scatter, dim3(ilu_grid(n)), dim3(kIluThreads), 0, st, n, rp, ci,
                     state, start, cursor, order, kind);
  return hipGetLastError();
}

hipError_t launch_ilu_factor(const int32_t* order, int32_t begin, int32_t end, const int32_t* rp,
                             const int32_t* ci, const int8_t* kind, const int32_t* diag,
                             const int32_t* state, double* lu, int32_t* err, hipStream_t st) {
  if (end <= begin) return hipSuccess;
  const int grid = (end - begin + kIluThreads - 1) / kIluThreads;
  hipLaunchKernelGGL(k_ilu_factor, dim3(grid), dim3(kIluThreads), 0, st, order, begin, end, rp,
                     ci, kind, diag, state, lu, err);
  return hipGetLastError();
}

hipError_t launch_ilu_apply(bool fp32, const IluFactors& f, const void* in, double* t, void* out,
                            hipStream_t st, const DevCtl* ctl) {
  for (int c = 0; c < f.ncolors; ++c) {
    const int b = f.level[c], e = f.level[c + 1];
    if (e <= b) continue;
    const int grid = (e - b + kIluThreads - 1) / kIluThreads;
    if (fp32)
      hipLaunchKernelGGL((k_ilu_solve<float, true>), dim3(grid), dim3(kIluThreads), 0, st,
                         f.order, b, e, f.rp, f.ci, f.kind, f.diag, f.lu,
                         static_cast<const float*>(in), t, static_cast<float*>(out), ctl);
    else
      hipLaunchKernelGGL((k_ilu_solve<double, true>), dim3(grid), dim3(kIluThreads), 0, st,
                         f.order, b, e, f.rp, f.ci, f.kind, f.diag, f.lu,
                         static_cast<const double*>(in), t, static_cast<double*>(out), ctl);
  }
  for (int c = f.ncolors - 1; c >= 0; --c) {
    const int b = f.level[c], e = f.level[c + 1];
    if (e <= b) continue;
    const int grid = (e - b + kIluThreads - 1) / kIluThreads;
    if (fp32)
      hipLaunchKernelGGL((k_ilu_solve<float, false>), dim3(grid), dim3(kIluThreads), 0, st,
                         f.order, b, e, f.rp, f.ci, f.kind, f.diag, f.lu,
                         static_cast<const float*>(in), t, static_cast<float*>(out), ctl);
    else
      hipLaunchKernelGGL((k_ilu_solve<double, false>), dim3(grid), dim3(kIluThreads), 0, st,
                         f.order, b, e, f.rp, f.ci, f.kind, f.diag, f.lu,
                         static_cast<const double*>(in), t, static_cast<double*>(out), ctl);
  }
  return hipGetLastError();
}

}  // namespace sfg
