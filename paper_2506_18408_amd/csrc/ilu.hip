// Zero-fill ILU right preconditioning (the "-p" runs of the paper's Section
// 4.4 and Table 1): M = L U on A's pattern, applied to every inner basis
// vector (the inner operator is A M^{-1}) and to the inner solution
// (z_j = M^{-1} B_k y_k).
//
// Elimination order: by colour of a proper colouring of the symmetrised
// graph of A, then by index.  Unknowns of one colour are never coupled, so
// each colour is one level of the factorisation and of each triangular
// solve, run as one launch over the rows of that colour.  The colouring is
// Jones & Plassmann's: in rounds, every uncoloured vertex whose priority
// p(i) = (2654435761 i) mod 2^32 beats every neighbour that was uncoloured
// when the round began takes the smallest colour that none of its coloured
// neighbours has.  Two such vertices are never adjacent, so the vertices of
// a round colour themselves independently; each vertex's state is one
// 32-bit word (round << 12 | colour, or -1), so a reader sees either the
// state before the round or the final one.
//
// The rows are then listed by colour, in increasing index within a colour
// (per-chunk colour counts, a scan per colour, and one wave per chunk that
// places its rows with ballots), so the rows a launch works on are in
// memory order.
//
// Factorisation: the IKJ form of Gaussian elimination restricted to the
// pattern (Saad, Section 10.3.2): row i takes its entries of lower colour in
// (colour, index) order, divides each by the pivot of its row k and
// subtracts l_ik u_kj from every entry a_ij of its own pattern with colour(j)
// > colour(k).  Rows of earlier colours are final (earlier launches); every
// row is written only by the thread (short rows) or the wave (long rows,
// the updates from one row k spread over the lanes) that owns it.
//
// Triangular solves: a copy of the factors in the colour order, with the L
// and U entries of each row contiguous and their columns given as positions
// in that order, so the rows of a colour are read as one stream; a group of
// 1..64 lanes per row, by the colour's mean row length.  They run on a work
// vector in the colour order, of the caller's vector type (the rows of a
// colour are one contiguous run of it); the caller's vectors stay in A's
// numbering, read by the forward solve and written by the backward one
// through the row order.
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
                           int32_t* __restrict__ state, int32_t* err, int32_t* maxrow) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int longest = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int q0 = rp[i], q1 = rp[i + 1];
    longest = q1 - q0 > longest ? q1 - q0 : longest;
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
  // (one atomic per wave)
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const int o = __shfl_xor(longest, off, kWave);
    longest = o > longest ? o : longest;
  }
  if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(maxrow, longest);
}

// One Jones-Plassmann round r: neighbours are the columns of row i of A and
// of A^T (CSR of the transpose), the diagonal excluded.  A row's neighbour
// states are read eight at a time (independent loads in flight together):
// a thread per row otherwise waits one memory round trip per neighbour, and
// the longest rows set the time of the round.
__global__ __launch_bounds__(kIluThreads) void k_ilu_jp_round(
    int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
    const int32_t* __restrict__ rpt, const int32_t* __restrict__ cit, int32_t* state, int32_t r,
    int32_t* colored, int32_t* err) {
  constexpr int kB = 8;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int mine = 0;  // rows this thread coloured
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
      const int q1 = P[i + 1];
      for (int q = P[i]; q < q1 && is_max; q += kB) {
        int j[kB];
        int32_t sj[kB];
#pragma unroll
        for (int k = 0; k < kB; ++k) j[k] = q + k < q1 ? C[q + k] : (int)i;
#pragma unroll
        for (int k = 0; k < kB; ++k) sj[k] = state[j[k]];
#pragma unroll
        for (int k = 0; k < kB; ++k)
          if (j[k] != (int)i && open_at_start(sj[k]) && ilu_priority(j[k]) > pi) is_max = false;
      }
    }
    if (!is_max) continue;
    // smallest colour not held by a neighbour coloured in an earlier round:
    // colours below 64 through a bit mask, then a scan per candidate
    uint64_t low = 0;
    for (int pass = 0; pass < 2; ++pass) {
      const int32_t* P = pass ? rpt : rp;
      const int32_t* C = pass ? cit : ci;
      const int q1 = P[i + 1];
      for (int q = P[i]; q < q1; q += kB) {
        int j[kB];
        int32_t sj[kB];
#pragma unroll
        for (int k = 0; k < kB; ++k) j[k] = q + k < q1 ? C[q + k] : (int)i;
#pragma unroll
        for (int k = 0; k < kB; ++k) sj[k] = state[j[k]];
#pragma unroll
        for (int k = 0; k < kB; ++k) {
          if (j[k] == (int)i || open_at_start(sj[k])) continue;
          const int c = sj[k] & 0xFFF;
          if (c < 64) low |= 1ull << c;
        }
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
    ++mine;
  }
  // (one atomic per wave)
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) mine += __shfl_xor(mine, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0 && mine > 0) atomicAdd(colored, mine);
}

// Rows per colour: a histogram per workgroup in LDS, added to cnt once.
__global__ __launch_bounds__(kIluThreads) void k_ilu_count(int64_t n,
                                                           const int32_t* __restrict__ state,
                                                           int32_t* cnt) {
  __shared__ int32_t h[kIluMaxColors];
  for (int c = threadIdx.x; c < kIluMaxColors; c += blockDim.x) h[c] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    atomicAdd(&h[state[i] & 0xFFF], 1);
  __syncthreads();
  for (int c = threadIdx.x; c < kIluMaxColors; c += blockDim.x)
    if (h[c]) atomicAdd(&cnt[c], h[c]);
}

// Rows of each colour in chunk b (kIluChunk rows): hist[c * nchunk + b].
__global__ __launch_bounds__(kIluThreads) void k_ilu_hist(int64_t n,
                                                          const int32_t* __restrict__ state,
                                                          int32_t nc, int64_t nchunk,
                                                          int32_t* __restrict__ hist) {
  __shared__ int32_t h[kIluMaxColors];
  for (int c = threadIdx.x; c < nc; c += blockDim.x) h[c] = 0;
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * kIluChunk;
  const int64_t r1 = r0 + kIluChunk < n ? r0 + kIluChunk : n;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) atomicAdd(&h[state[i] & 0xFFF], 1);
  __syncthreads();
  for (int c = threadIdx.x; c < nc; c += blockDim.x) hist[(int64_t)c * nchunk + blockIdx.x] = h[c];
}

// Workgroup c: hist[c * nchunk + b] <- start[c] + rows of colour c in the
// chunks before b (the first position of chunk b's rows of colour c).
constexpr int kIluScanThreads = 1024;
__global__ __launch_bounds__(kIluScanThreads) void k_ilu_hist_scan(int64_t nchunk,
                                                                   const int32_t* __restrict__ start,
                                                                   int32_t* hist) {
  __shared__ int32_t wsum[kIluScanThreads / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int32_t* hc = hist + (int64_t)blockIdx.x * nchunk;
  int carry = start[blockIdx.x];
  for (int64_t base = 0; base < nchunk; base += kIluScanThreads) {
    const int64_t b = base + threadIdx.x;
    const int v = b < nchunk ? hc[b] : 0;
    int incl = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int o = __shfl_up(incl, off, kWave);
      if (lane >= off) incl += o;
    }
    if (lane == kWave - 1) wsum[wid] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < kIluScanThreads / kWave; ++w) {
      before += w < wid ? wsum[w] : 0;
      total += wsum[w];
    }
    if (b < nchunk) hc[b] = carry + before + incl - v;
    carry += total;
    __syncthreads();
  }
}

// The kind of every entry: -1 (column of lower colour: L), 0 (diagonal),
// +1 (U).
__global__ void k_ilu_kind(int64_t n, const int32_t* __restrict__ rp,
                           const int32_t* __restrict__ ci, const int32_t* __restrict__ state,
                           int8_t* __restrict__ kind) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int c = state[i] & 0xFFF;
    for (int q = rp[i]; q < rp[i + 1]; ++q) {
      const int j = ci[q];
      const int cj = state[j] & 0xFFF;
      kind[q] = j == (int)i ? 0 : (cj < c ? -1 : 1);
    }
  }
}

// One wave per chunk places the chunk's rows, 64 at a time in index order:
// a lane's rank among the lanes of its colour comes from 12 ballots (one
// per colour bit), and the wave's running count per colour sits in LDS.
__global__ __launch_bounds__(kWave) void k_ilu_place(int64_t n, const int32_t* __restrict__ state,
                                                     int32_t nc, int64_t nchunk,
                                                     const int32_t* __restrict__ off,
                                                     int32_t* __restrict__ order) {
  __shared__ int32_t run[kIluMaxColors];
  const int lane = threadIdx.x;
  for (int c = lane; c < nc; c += kWave) run[c] = 0;
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * kIluChunk;
  const int64_t r1 = r0 + kIluChunk < n ? r0 + kIluChunk : n;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int64_t base = r0; base < r1; base += kWave) {  // (uniform)
    const int64_t i = base + lane;
    const bool valid = i < r1;
    const int c = valid ? (state[i] & 0xFFF) : 0xFFF;  // (colours are < 0xFFF)
    uint64_t same = ~0ull;
#pragma unroll
    for (int bit = 0; bit < 12; ++bit) {
      const bool on = (c >> bit) & 1;
      const uint64_t bal = __ballot(on);
      same &= on ? bal : ~bal;
    }
    const int rank = __popcll(same & below);
    const int size = __popcll(same);
    if (valid) order[off[(int64_t)c * nchunk + blockIdx.x] + run[c] + rank] = (int32_t)i;
    // (every lane has read run[c] above; the group's last lane advances it)
    if (valid && rank == size - 1) run[c] += size;
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

// One colour of the factorisation with one wave per row (long rows): the
// row's lower entries are visited in (colour, index) order, 64 at a time
// per colour with a ballot; the updates from row k are spread over the
// lanes (each lane a different column j, so a different entry of row i).
__global__ __launch_bounds__(kIluThreads) void k_ilu_factor_wave(
    const int32_t* __restrict__ order, int32_t begin, int32_t end, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ ci, const int8_t* __restrict__ kind,
    const int32_t* __restrict__ diag, const int32_t* __restrict__ state, double* lu,
    int32_t* err) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t pos = begin + ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (pos >= end) return;  // (whole waves)
  const int i = order[pos];
  const int q0 = rp[i], q1 = rp[i + 1];
  const int ci_col = state[i] & 0xFFF;
  for (int cc = 0; cc < ci_col; ++cc) {
    for (int base = q0; base < q1; base += kWave) {
      const int q = base + lane;
      int k = -1;
      if (q < q1 && kind[q] == -1) {
        const int kk = ci[q];
        if ((state[kk] & 0xFFF) == cc) k = kk;
      }
      uint64_t m = __ballot(k >= 0);
      while (m) {
        const int l0 = __builtin_ctzll(m);
        m &= m - 1;
        const int kq = __builtin_amdgcn_readlane(k, l0);
        const int qq = base + l0;
        const double piv = lu[diag[kq]];
        if (piv == 0.0) {
          if (lane == 0) atomicOr(err, 8);
          return;
        }
        // (every lane reads l_ik before lane 0 stores it: the store needs
        // the loaded value)
        const double l = lu[qq] / piv;
        if (lane == 0) lu[qq] = l;
        const int k0 = rp[kq], k1 = rp[kq + 1];
        for (int r = k0 + lane; r < k1; r += kWave) {
          const int j = ci[r];
          if (j == kq || (state[j] & 0xFFF) <= cc) continue;
          const int p = find_col(ci, q0, q1, j);
          if (p >= 0) lu[p] -= l * lu[r];
        }
      }
    }
  }
  if (lane == 0 && lu[diag[i]] == 0.0) atomicOr(err, 8);
}

// The solve copies: entry counts per position (L and U together), scanned
// into orp by the caller's scan.
__global__ void k_ilu_split_count(int64_t n, const int32_t* __restrict__ rp,
                                  const int32_t* __restrict__ order, int32_t* __restrict__ orp) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const int i = order[p];
    orp[p] = rp[i + 1] - rp[i] - 1;  // (every row holds its diagonal)
  }
}

template <typename FT>
__global__ void k_ilu_split_fill(int64_t n, const int32_t* __restrict__ rp,
                                 const int32_t* __restrict__ ci, const int8_t* __restrict__ kind,
                                 const int32_t* __restrict__ diag, const double* __restrict__ lu,
                                 const int32_t* __restrict__ order,
                                 const int32_t* __restrict__ orp, int32_t* __restrict__ omid,
                                 int32_t* __restrict__ oci, FT* __restrict__ oval,
                                 FT* __restrict__ udiag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const int i = order[p];
    const int q0 = rp[i], q1 = rp[i + 1];
    int o = orp[p];
    for (int q = q0; q < q1; ++q)
      if (kind[q] == -1) {
        oci[o] = ci[q];
        oval[o] = static_cast<FT>(lu[q]);
        ++o;
      }
    omid[p] = o;
    for (int q = q0; q < q1; ++q)
      if (kind[q] == 1) {
        oci[o] = ci[q];
        oval[o] = static_cast<FT>(lu[q]);
        ++o;
      }
    udiag[p] = static_cast<FT>(lu[diag[i]]);
  }
}

// L entries of each colour: workgroups (x, c) sum a strided part of colour
// c's positions and add it to lsum[c] (zeroed by the caller); usum[c] =
// all of the colour's entries minus lsum[c], by k_ilu_level_usum.
constexpr int kIluSumSplit = 64;
__global__ __launch_bounds__(kIluThreads) void k_ilu_level_sums(const int32_t* __restrict__ start,
                                                                const int32_t* __restrict__ orp,
                                                                const int32_t* __restrict__ omid,
                                                                int32_t* lsum) {
  __shared__ int32_t part[kIluThreads / kWave];
  const int c = blockIdx.y;
  const int b = start[c], e = start[c + 1];
  int v = 0;
  for (int p = b + blockIdx.x * blockDim.x + threadIdx.x; p < e; p += gridDim.x * blockDim.x)
    v += omid[p] - orp[p];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int l = 0;
    for (int w = 0; w < kIluThreads / kWave; ++w) l += part[w];
    if (l) atomicAdd(&lsum[c], l);
  }
}

__global__ void k_ilu_level_usum(int32_t nc, const int32_t* __restrict__ start,
                                 const int32_t* __restrict__ orp, const int32_t* __restrict__ lsum,
                                 int32_t* usum) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x)
    usum[c] = (orp[start[c + 1]] - orp[start[c]]) - lsum[c];
}

// One colour of the forward solve L t = in or of the backward solve U t = t
// (result also to out), on a work vector of the caller's vector type VT in
// the colour order: t[p] belongs to row order[p], and the entries of position p
// are oval/pci[s0[p] .. s1[p]) with pci the positions of their columns.  The
// rows of a colour are then one contiguous run of t, and the entries of a
// row point into the other colours' runs near the row's own relative place,
// so the t accesses stream; only in and out are reached through order.  G
// lanes per row; one lane per row subtracts the products in the row's
// column order.  In place: t entries of earlier colours (forward) or later
// ones (backward) are final.  Factor values of type FT (FP32 copies in mixed
// precision), every product and sum in FP64; each row's result is stored
// rounded to VT, as the inner SpMV stores its output.
template <typename VT, typename FT, bool kForward, int G>
__global__ __launch_bounds__(kIluThreads) void k_ilu_solve(
    const int32_t* __restrict__ order, const VT* __restrict__ in, VT* __restrict__ out,
    int32_t begin, int32_t end, const int32_t* __restrict__ s0, const int32_t* __restrict__ s1,
    const int32_t* __restrict__ pci, const FT* __restrict__ oval,
    const FT* __restrict__ udiag, VT* t, const DevCtl* ctl) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t pos = begin + gid / G;
  const int sub = (int)(gid % G);
  if (pos >= end) return;  // (whole groups: G divides the wave)
  if (ctl && ctl->stop_k != 0) return;
  const int qa = s0[pos], qb = s1[pos];
  double acc;
  if constexpr (G == 1) {
    acc = kForward ? static_cast<double>(in[order[pos]]) : static_cast<double>(t[pos]);
    // (four entries' loads in flight at once, subtracted in order)
    for (int q = qa; q < qb; q += 4) {
      const int m = qb - q;
      int c[4];
      FT v[4];
      double tv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < m) {
          c[k] = pci[q + k];
          v[k] = oval[q + k];
        }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < m) tv[k] = static_cast<double>(t[c[k]]);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < m) acc -= static_cast<double>(v[k]) * tv[k];
    }
  } else {
    double part = 0.0;
    for (int q = qa + sub; q < qb; q += G) part += static_cast<double>(oval[q]) * static_cast<double>(t[pci[q]]);
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) part += __shfl_xor(part, off, G);
    acc = (kForward ? static_cast<double>(in[order[pos]]) : static_cast<double>(t[pos])) - part;
  }
  if (sub != 0) return;
  if (kForward) {
    t[pos] = static_cast<VT>(acc);
  } else {
    const double z = acc / static_cast<double>(udiag[pos]);
    t[pos] = static_cast<VT>(z);
    out[order[pos]] = static_cast<VT>(z);
  }
}

// pos[order[p]] = p, then the solve copies' column indices (entries [0,
// count)) turned into positions in place.
__global__ void k_ilu_pos(int64_t n, const int32_t* __restrict__ order, int32_t* __restrict__ pos) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
    pos[order[p]] = (int32_t)p;
}

__global__ void k_ilu_pci(int64_t count, const int32_t* __restrict__ pos, int32_t* oci) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += stride)
    oci[q] = pos[oci[q]];
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
                           int32_t* maxrow, hipStream_t st) {
  hipLaunchKernelGGL(k_ilu_init, dim3(ilu_grid(n)), dim3(kIluThreads), 0, st, n, rp, ci, val,
                     lu, diag, state, err, maxrow);
  return hipGetLastError();
}

hipError_t launch_ilu_jp_round(int64_t n, const int32_t* rp, const int32_t* ci,
                               const int32_t* rpt, const int32_t* cit, int32_t* state,
                               int32_t round, int32_t* colored, int32_t* err, hipStream_t st) {
  // (a thread per row: the rows of a round wait on memory, not on issue)
  const int64_t g = (n + kIluThreads - 1) / kIluThreads;
  hipLaunchKernelGGL(k_ilu_jp_round, dim3((int)(g < 65535 ? (g > 0 ? g : 1) : 65535)),
                     dim3(kIluThreads), 0, st, n, rp, ci, rpt, cit, state, round, colored, err);
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

hipError_t launch_ilu_order(int64_t n, const int32_t* rp, const int32_t* ci,
                            const int32_t* state, int32_t nc, const int32_t* start,
                            int32_t* hist, int32_t* order, int8_t* kind, hipStream_t st) {
  const int64_t nchunk = ilu_chunks(n);
  if (nc <= 0 || nchunk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ilu_hist, dim3((unsigned)nchunk), dim3(kIluThreads), 0, st, n, state, nc,
                     nchunk, hist);
  hipLaunchKernelGGL(k_ilu_hist_scan, dim3((unsigned)nc), dim3(kIluScanThreads), 0, st, nchunk,
                     start, hist);
  hipLaunchKernelGGL(k_ilu_place, dim3((unsigned)nchunk), dim3(kWave), 0, st, n, state, nc, nchunk,
                     hist, order);
  hipLaunchKernelGGL(k_ilu_kind, dim3(ilu_grid(n)), dim3(kIluThreads), 0, st, n, rp, ci, state,
                     kind);
  return hipGetLastError();
}

hipError_t launch_ilu_factor(const int32_t* order, int32_t begin, int32_t end, const int32_t* rp,
                             const int32_t* ci, const int8_t* kind, const int32_t* diag,
                             const int32_t* state, double* lu, int32_t* err, bool wave_per_row,
                             hipStream_t st) {
  if (end <= begin) return hipSuccess;
  if (wave_per_row) {
    const int64_t threads = (int64_t)(end - begin) * kWave;
    const int grid = (int)((threads + kIluThreads - 1) / kIluThreads);
    hipLaunchKernelGGL(k_ilu_factor_wave, dim3(grid), dim3(kIluThreads), 0, st, order, begin, end,
                       rp, ci, kind, diag, state, lu, err);
  } else {
    const int grid = (end - begin + kIluThreads - 1) / kIluThreads;
    hipLaunchKernelGGL(k_ilu_factor, dim3(grid), dim3(kIluThreads), 0, st, order, begin, end, rp,
                       ci, kind, diag, state, lu, err);
  }
  return hipGetLastError();
}

hipError_t launch_ilu_split(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci,
                            const int8_t* kind, const int32_t* diag, const double* lu,
                            const int32_t* order, int32_t nc, const int32_t* start, int32_t* orp,
                            int32_t* omid, int32_t* oci, void* oval, void* udiag,
                            bool fp32_factors, int32_t* lsum, int32_t* usum, int32_t* pos,
                            int32_t* scan_tmp, hipStream_t st) {
  hipLaunchKernelGGL(k_ilu_split_count, dim3(ilu_grid(n)), dim3(kIluThreads), 0, st, n, rp, order,
                     orp);
  const hipError_t e = launch_exclusive_scan(orp, n, scan_tmp, st);
  if (e != hipSuccess) return e;
  if (fp32_factors)
    hipLaunchKernelGGL(k_ilu_split_fill<float>, dim3(ilu_grid(n)), dim3(kIluThreads), 0, st, n,
                       rp, ci, kind, diag, lu, order, orp, omid, oci, static_cast<float*>(oval),
                       static_cast<float*>(udiag));
  else
    hipLaunchKernelGGL(k_ilu_split_fill<double>, dim3(ilu_grid(n)), dim3(kIluThreads), 0, st, n,
                       rp, ci, kind, diag, lu, order, orp, omid, oci, static_cast<double*>(oval),
                       static_cast<double*>(udiag));
  // (every row holds its diagonal: nnz - n off-diagonal entries)
  hipLaunchKernelGGL(k_ilu_pos, dim3(ilu_grid(n)), dim3(kIluThreads), 0, st, n, order, pos);
  hipLaunchKernelGGL(k_ilu_pci, dim3(ilu_grid(nnz - n)), dim3(kIluThreads), 0, st, nnz - n, pos,
                     oci);
  if (nc > 0) {
    // (lsum is zero: the caller clears the counter block at set-up)
    hipLaunchKernelGGL(k_ilu_level_sums, dim3(kIluSumSplit, (unsigned)nc), dim3(kIluThreads), 0, st,
                       start, orp, omid, lsum);
    hipLaunchKernelGGL(k_ilu_level_usum, dim3((unsigned)((nc + kIluThreads - 1) / kIluThreads)),
                       dim3(kIluThreads), 0, st, nc, start, orp, lsum, usum);
  }
  return hipGetLastError();
}

int ilu_group(int64_t rows, int64_t entries) {
  if (rows <= 0) return 1;
  const double mean = (double)entries / (double)rows;
  int g = 1;
  while (g < kWave && mean >= 3.0 * g) g <<= 1;
  return g == 2 ? 1 : g;
}

template <typename VT, typename FT, bool kForward, int G>
static void ilu_solve_launch(const IluFactors& f, int b, int e, const int32_t* s0,
                             const int32_t* s1, const VT* in, double* t, VT* out, hipStream_t st,
                             const DevCtl* ctl) {
  const int64_t threads = (int64_t)(e - b) * G;
  const int grid = (int)((threads + kIluThreads - 1) / kIluThreads);
  hipLaunchKernelGGL((k_ilu_solve<VT, FT, kForward, G>), dim3(grid), dim3(kIluThreads), 0, st,
                     f.order, in, out, b, e, s0, s1, f.oci, static_cast<const FT*>(f.oval),
                     static_cast<const FT*>(f.udiag), reinterpret_cast<VT*>(t), ctl);
}

template <typename VT, typename FT, bool kForward>
static void ilu_solve_colour(const IluFactors& f, int c, const VT* in, double* t, VT* out,
                             hipStream_t st, const DevCtl* ctl) {
  const int b = f.level[c], e = f.level[c + 1];
  if (e <= b) return;
  const int32_t* s0 = kForward ? f.orp : f.omid;
  const int32_t* s1 = kForward ? f.omid : f.orp + 1;
  switch (f.group[2 * c + (kForward ? 0 : 1)]) {
    case 1:
      return ilu_solve_launch<VT, FT, kForward, 1>(f, b, e, s0, s1, in, t, out, st, ctl);
    case 4:
      return ilu_solve_launch<VT, FT, kForward, 4>(f, b, e, s0, s1, in, t, out, st, ctl);
    case 8:
      return ilu_solve_launch<VT, FT, kForward, 8>(f, b, e, s0, s1, in, t, out, st, ctl);
    case 16:
      return ilu_solve_launch<VT, FT, kForward, 16>(f, b, e, s0, s1, in, t, out, st, ctl);
    case 32:
      return ilu_solve_launch<VT, FT, kForward, 32>(f, b, e, s0, s1, in, t, out, st, ctl);
    default:
      return ilu_solve_launch<VT, FT, kForward, 64>(f, b, e, s0, s1, in, t, out, st, ctl);
  }
}

template <typename VT, typename FT>
static hipError_t ilu_apply_vt(const IluFactors& f, const VT* in, double* t, VT* out,
                               hipStream_t st, const DevCtl* ctl) {
  for (int c = 0; c < f.ncolors; ++c) ilu_solve_colour<VT, FT, true>(f, c, in, t, out, st, ctl);
  for (int c = f.ncolors - 1; c >= 0; --c)
    ilu_solve_colour<VT, FT, false>(f, c, in, t, out, st, ctl);
  return hipGetLastError();
}

hipError_t launch_ilu_apply(bool fp32, const IluFactors& f, const void* in, double* t, void* out,
                            hipStream_t st, const DevCtl* ctl) {
  const float* fi = static_cast<const float*>(in);
  const double* di = static_cast<const double*>(in);
  float* fo = static_cast<float*>(out);
  double* dout = static_cast<double*>(out);
  if (f.fp32)
    return fp32 ? ilu_apply_vt<float, float>(f, fi, t, fo, st, ctl)
                : ilu_apply_vt<double, float>(f, di, t, dout, st, ctl);
  // (FP64 factors serve FP64 vectors only)
  if (fp32) return hipErrorInvalidValue;
  return ilu_apply_vt<double, double>(f, di, t, dout, st, ctl);
}

}  // namespace sfg
