// Host driver and C ABI of the sketched-FGMRES solver (include/sfgmres.h).
//
// One call runs Algorithm 1 of Guettel & Pearson (arXiv 2506.18408) on the
// caller's stream: the sketch S is generated once (packed), then the initial
// residual, then per outer step one sGMRES cycle (Section 3), then z_j =
// B_k y, the outer SpMV, modified Gram-Schmidt, the Givens update and the
// normalised v_{j+1} with its sketch.
//
// The inner steps run on the caller's stream.  Step i is the fused SpMV
// y = A u_i (+ S y as per-workgroup partial rows in ring slot i mod 2p, the
// window dots and ||y||^2 as scalar rows) and, for t > 0, the
// truncated-Arnoldi update u_{i+1} with its own coefficients (else a
// one-workgroup coefficient kernel).  After every p steps (a panel), a
// second stream reduces the panel's sketch rows and runs one decision
// kernel that appends its p columns to the sketched QR and decides after
// each column (C1-C3), while the caller's stream goes on with the next
// steps; the SpMV grid leaves a CU per XCD free for it.  Only the decision
// ends the cycle, so the steps between the stop and the moment the flag is
// seen (up to p - 1 inside the panel, and about one past it) are computed
// and discarded.  The inner basis is kept unnormalised (u_i = the
// orthogonalised A b_{i-1}, of norm h_{i,i-1}, with sigma_i = 1/||u_i|| held
// on the device), so no kernel waits for a scalar its predecessor has just
// reduced.
// The host stays up to `lookahead` inner steps ahead of the last decided
// column: every inner kernel is predicated on the device's stop flag, and
// the host polls a pinned status block (written by the decision kernel) to
// stop enqueuing once the cycle has ended.  The host synchronises once per
// outer step to read the minimised residual.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <thread>
#include <vector>

#include "kernels.hpp"

struct sfgmres_ctx {
  int device = 0;
  sfg::HostStatus* hs_host = nullptr;
  sfg::HostStatus* hs_dev = nullptr;
  std::string err;
  std::vector<hipEvent_t> ev;  // timing events (profile option)
  hipStream_t dec = nullptr;    // the decision stream (slot reductions, sketched QR)
  std::vector<hipEvent_t> sync; // panel hand-over events (no timing)
  std::vector<hipEvent_t> pev;  // phase marks (phase_timers option)
};

namespace sfg {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// C2 threshold.  The paper's 1e15 is a double-precision choice (a column
// is dropped once the sketched basis is within a few digits of singular in
// FP64); with an FP32 basis the same margin is reached at 1e15 u64/u32 =
// 1e15 2^-29.  Measured on the 128^3 system in mixed precision: t = 0,
// 162 -> 53 ms; the paper's t = 0, zeta = 1, s = 1000, k_max = 500:
// 1312 -> 68 ms; t = 2 unchanged; 256^3, t = 2: 1.53 -> 1.33 s.
double cond_threshold_of(const sfgmres_options& o) {
  if (o.cond_threshold > 0.0) return o.cond_threshold;
  return o.precision == SFGMRES_MIXED ? 1e15 * 0x1p-29 : 1e15;
}

// Columns per decision launch and the host's lookahead (in inner steps).
int panel_cols(const sfgmres_options& o) { return o.panel > 0 ? o.panel : kPanel; }
int lookahead_steps(const sfgmres_options& o) {
  const int p = panel_cols(o);
  return o.lookahead > 0 ? std::max(o.lookahead, p) : 2 * p;
}

struct IluWs {
  size_t lu, kind, diag, state, order, cnt, t_rp, t_ci, t_perm, t_cursor, t_scan, hist, orp, omid,
      oci, oval, udiag, total;
};
// Ints of the ILU counter block: counts, level starts, L and U entries per
// colour, then the error flags, coloured rows and the longest row.
constexpr size_t kIluCntInts = 4 * (kIluMaxColors + 1) + 8;

// The ILU regions of a workspace (appended to `off`).
IluWs ilu_regions(int64_t n, int64_t nnz, size_t off) {
  IluWs W{};
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  W.lu = take((size_t)nnz * 8);
  W.kind = take((size_t)nnz);
  W.diag = take((size_t)n * 4);
  W.state = take((size_t)n * 4);
  W.order = take((size_t)n * 4);
  W.cnt = take(kIluCntInts * 4);
  W.t_rp = take((size_t)(n + 1) * 4);
  W.t_ci = take((size_t)nnz * 4);
  W.t_perm = take((size_t)nnz * 4);
  W.t_cursor = take((size_t)(n + 1) * 4);
  W.t_scan = take(transpose_scan_tmp_ints(n) * 4);
  W.hist = take((size_t)kIluMaxColors * (size_t)ilu_chunks(n) * 4);
  W.orp = take((size_t)(n + 1) * 4);
  W.omid = take((size_t)n * 4);
  W.oci = take((size_t)nnz * 4);
  W.oval = take((size_t)nnz * 8);
  W.udiag = take((size_t)n * 8);
  W.total = off;
  return W;
}

Layout make_layout(int64_t n, int64_t nnz, int32_t m, int32_t t, int32_t s, int32_t zeta,
                   int32_t J, int32_t precision, int32_t adjoint, int32_t panel, int32_t precond,
                   int32_t mid_outer, int32_t matrix_format) {
  (void)t;
  Layout L{};
  const bool f32 = precision == SFGMRES_MIXED;
  L.ld = (n + 63) / 64 * 64;
  L.ntiles_max = n / kRowTile + nnz / kTileNnz + 3;
  L.grid = kMaxGrid;
  const size_t vt = f32 ? 4 : 8;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.ctl = take(sizeof(DevCtl));
  L.tiles = take((size_t)(L.ntiles_max + 1) * 4);
  L.tp = take((size_t)(L.ntiles_max + 1) * 4);
  L.ipart = take((size_t)(kVecGrid + 1) * 4);
  L.part = take((size_t)2 * panel * kMaxGrid * s * 8);  // two panels of sketch rows
  L.dpart = take((size_t)2 * kMaxGrid * kDP * 8);  // two: inner steps alternate
  L.vpart = take((size_t)2 * kVecGrid * 8);  // two: read by one Arnoldi update, written by it
  L.red = take((size_t)2 * panel * s * 8);
  L.skp = take(packed_sketch_bytes(n, zeta));
  L.qr_V = take((size_t)s * m * 8);
  L.qr_T = take((size_t)m * m * 8);
  L.qr_R = take((size_t)m * m * 8);
  L.qr_d = take((size_t)s * 8);
  L.qr_c = take(64 * 8);  // small device scalars
  L.qr_tau = take((size_t)m * 8);
  L.ice_x = take((size_t)(m + 1) * 8);
  L.ice_z = take((size_t)(m + 1) * 8);
  L.sigma = take((size_t)(m + 2) * 8);
  L.hwin = take((size_t)(kMaxT + 1) * 8);
  L.yin = take((size_t)(m + 1) * 8);
  L.H = take((size_t)(J + 1) * J * 8);
  L.HR = take((size_t)(J + 1) * J * 8);
  L.cs = take((size_t)J * 8);
  L.sn = take((size_t)J * 8);
  L.g = take((size_t)(J + 1) * 8);
  L.yout = take((size_t)(J + 1) * 8);
  L.V = take((size_t)(J + 1) * L.ld * 8);
  L.Z = take((size_t)J * L.ld * 8);
  L.B = take((size_t)(m + 1) * L.ld * vt);
  L.W32 = take(f32 ? (size_t)L.ld * 4 : 0);
  L.W64 = take((size_t)L.ld * 8);
  L.X = take((size_t)L.ld * 8);
  L.val32 = take(f32 ? (size_t)nnz * 4 : 0);
  // the matrix by diagonal for the inner SpMV (matrix_format AUTO): up to
  // kDiaMax diagonals of ld values in the inner SpMV's precision, and the
  // detection's work words
  const bool dia_ok = matrix_format == SFGMRES_MATRIX_AUTO;
  L.dia = take(dia_ok ? (size_t)kDiaMax * (size_t)L.ld * vt : 0);
  L.dia_work = take(dia_ok ? (size_t)(4 + kDiaMax) * 4 : 0);
  // ILU(0): factor values, entry kinds, diagonal positions, colouring state,
  // rows by colour, counters (per-colour counts, cursors and starts, then
  // the error and coloured-count words), the transposed pattern for the
  // colouring, the FP64 work vector and the preconditioned inner vector
  // (placed before the adjoint's regions: the adjoint solve runs on this
  // layout without them)
  const bool ilu = precond == SFGMRES_PRECOND_ILU0;
  L.ilu = off;
  if (ilu) off = ilu_regions(n, nnz, off).total;
  L.ilu_t64 = take(ilu ? (size_t)L.ld * 8 : 0);
  L.ilu_tmp = take(ilu ? (size_t)L.ld * vt : 0);
  // two-level FGMRES: the lower level's whole solve workspace
  L.mid_bytes = mid_outer > 0
                    ? make_layout(n, nnz, m, t, s, zeta, mid_outer, precision, 0, panel, precond, 0,
                                  matrix_format)
                          .total
                    : 0;
  L.mid = take(L.mid_bytes);
  if (adjoint) {
    L.at_rowptr = take((size_t)(n + 1) * 4);
    L.at_col = take((size_t)nnz * 4);
    L.at_val = take((size_t)nnz * 8);
    L.at_perm = take((size_t)nnz * 4);
    L.at_cursor = take((size_t)(n + 1) * 4);
    L.scan_tmp = take(transpose_scan_tmp_ints(n) * 4);
  }
  L.total = off;
  return L;
}

}  // namespace sfg

using namespace sfg;

namespace {

#define SFG_HIP(call)                                                           \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      h->err = std::string(#call) + " failed: " + hipGetErrorString(e_);       \
      return SFGMRES_ERR_HIP;                                                   \
    }                                                                           \
  } while (0)

int fail(sfgmres_handle h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

sfgmres_options defaults() {
  sfgmres_options o;
  memset(&o, 0, sizeof(o));
  o.precision = SFGMRES_FP64;
  o.max_outer = 100;
  o.cond_threshold = 0.0;  // the precision's default
  o.record_true_residual = 0;
  o.profile = 0;
  o.lookahead = 0;
  o.panel = 0;
  o.outer = SFGMRES_OUTER_FGMRES;
  o.precond = SFGMRES_PRECOND_NONE;
  o.mid_outer = 0;
  o.sketch_source = SFGMRES_SKETCH_AUTO;
  o.matrix_format = SFGMRES_MATRIX_AUTO;
  return o;
}

bool sketch_args_ok(int64_t n, int32_t s, int32_t zeta) {
  return n >= 1 && n < ((int64_t)1 << 31) && s >= 1 && s <= SFGMRES_MAX_S && zeta >= 1 &&
         zeta <= s && zeta <= SFGMRES_MAX_ZETA;
}

int check_params(sfgmres_handle h, int64_t n, int64_t nnz, int32_t m, int32_t t, int32_t s,
                 int32_t zeta, double tol, const sfgmres_options& o) {
  if (n < 1) return fail(h, SFGMRES_ERR_INVALID, "n must be >= 1");
  if (nnz < 0 || nnz >= (int64_t)1 << 31) return fail(h, SFGMRES_ERR_INVALID, "nnz out of range");
  if (n >= (int64_t)1 << 31) return fail(h, SFGMRES_ERR_INVALID, "n must be < 2^31");
  if (m < 1 || m > SFGMRES_MAX_M) return fail(h, SFGMRES_ERR_INVALID, "need 1 <= m <= 512");
  if (s <= m || s > SFGMRES_MAX_S) return fail(h, SFGMRES_ERR_INVALID, "need m < s <= 1024");
  if (t < 0 || t > m || t > SFGMRES_MAX_T)
    return fail(h, SFGMRES_ERR_INVALID, "need 0 <= t <= min(m, 8)");
  if (zeta < 1 || zeta > s || zeta > SFGMRES_MAX_ZETA)
    return fail(h, SFGMRES_ERR_INVALID, "need 1 <= zeta <= min(s, 16)");
  if (!(tol > 0.0) || !isfinite(tol)) return fail(h, SFGMRES_ERR_INVALID, "tol must be > 0");
  if (o.precision != SFGMRES_FP64 && o.precision != SFGMRES_MIXED)
    return fail(h, SFGMRES_ERR_INVALID, "unknown precision");
  if (o.profile < 0) return fail(h, SFGMRES_ERR_INVALID, "need profile >= 0");
  if (o.max_outer < 1 || o.max_outer > SFGMRES_MAX_OUTER)
    return fail(h, SFGMRES_ERR_INVALID, "need 1 <= max_outer <= 2000");
  if (!(o.cond_threshold >= 0.0) || std::isinf(o.cond_threshold))
    return fail(h, SFGMRES_ERR_INVALID, "cond_threshold must be finite and >= 0 (0: default)");
  if (o.lookahead < 0 || o.lookahead > 64)
    return fail(h, SFGMRES_ERR_INVALID, "need 0 <= lookahead <= 64");
  if (o.panel < 0 || o.panel > kPanel) return fail(h, SFGMRES_ERR_INVALID, "need 0 <= panel <= 8");
  if (o.outer != SFGMRES_OUTER_FGMRES && o.outer != SFGMRES_OUTER_RESTARTED)
    return fail(h, SFGMRES_ERR_INVALID, "outer must be SFGMRES_OUTER_FGMRES or _RESTARTED");
  if (o.identity_sketch != 0 && o.identity_sketch != 1)
    return fail(h, SFGMRES_ERR_INVALID, "identity_sketch must be 0 or 1");
  if (o.identity_sketch && (s != n || zeta != 1))
    return fail(h, SFGMRES_ERR_INVALID, "identity_sketch needs s == n and zeta == 1");
  if (o.phase_timers != 0 && o.phase_timers != 1)
    return fail(h, SFGMRES_ERR_INVALID, "phase_timers must be 0 or 1");
  if (o.precond != SFGMRES_PRECOND_NONE && o.precond != SFGMRES_PRECOND_ILU0)
    return fail(h, SFGMRES_ERR_INVALID, "precond must be SFGMRES_PRECOND_NONE or _ILU0");
  if (o.precond != SFGMRES_PRECOND_NONE && o.outer != SFGMRES_OUTER_FGMRES)
    return fail(h, SFGMRES_ERR_INVALID, "precond needs the FGMRES outer iteration");
  if (o.mid_outer < 0 || o.mid_outer > SFGMRES_MAX_OUTER)
    return fail(h, SFGMRES_ERR_INVALID, "need 0 <= mid_outer <= 2000");
  if (o.mid_outer > 0 && o.outer != SFGMRES_OUTER_FGMRES)
    return fail(h, SFGMRES_ERR_INVALID, "mid_outer needs the FGMRES outer iteration");
  if (o.matrix_format != SFGMRES_MATRIX_AUTO && o.matrix_format != SFGMRES_MATRIX_CSR)
    return fail(h, SFGMRES_ERR_INVALID, "matrix_format must be AUTO or CSR");
  if (o.sketch_source < SFGMRES_SKETCH_AUTO || o.sketch_source > SFGMRES_SKETCH_GEN)
    return fail(h, SFGMRES_ERR_INVALID, "sketch_source must be AUTO, TABLE or GEN");
  if (o.sketch_source == SFGMRES_SKETCH_GEN &&
      (o.precision != SFGMRES_FP64 || zeta > kSkGroup || o.identity_sketch))
    return fail(h, SFGMRES_ERR_INVALID,
                "sketch_source GEN needs FP64, zeta <= 8 and the random sketch");
  return SFGMRES_OK;
}

// Persistent grid of the SpMV kernels: one workgroup per CU at most, at
// least one tile per wave, a multiple of the 8 XCDs.  (Small systems are
// latency bound: spreading them over every CU beats deeper per-wave
// pipelines, 57.7 -> 42.4 ms for the 512^2 solve with 4096 tiles.)
int spmv_grid(int64_t ntiles) {
  int64_t g = std::min<int64_t>((ntiles + kSpmvMaxWaves - 1) / kSpmvMaxWaves, kSpmvGrid);
  if (g >= 8) g -= g % 8;
  return (int)std::max<int64_t>(g, 1);
}

// Grid of the row-range sketch kernel (one partial row each, <= kMaxGrid).
int rows_grid(int64_t n) {
  int64_t g = std::min<int64_t>((n + 1023) / 1024, kMaxGrid);
  if (g >= 8) g -= g % 8;
  return (int)std::max<int64_t>(g, 1);
}

// Tiling of the SpMV kernels for A: 256-row tiles (one row per lane) when
// every row has at most kShortRow nonzeros, else tiles of about kTileNnz
// nonzeros.  Reads the longest row back to the host (one synchronisation).
struct Tiling {
  int32_t ntiles;
  int32_t grid;
  int32_t max_row;
};

int plan_tiling(sfgmres_handle h, const sfgmres_csr* A, int32_t* tiles, int32_t* tp,
                int32_t* ipart, hipStream_t st, Tiling* T) {
  int32_t* out = ipart + kVecGrid;
  SFG_HIP(launch_max_rowlen(A->row_ptr, A->n, ipart, out, st));
  int32_t maxlen = 0;
  SFG_HIP(hipMemcpyAsync(&maxlen, out, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SFG_HIP(hipStreamSynchronize(st));
  int32_t rpt = 0;
  int64_t ntiles;
  if (maxlen <= kShortRow) {
    rpt = kRowTile;
    ntiles = (A->n + rpt - 1) / rpt;
  } else {
    ntiles = A->nnz / kTileNnz + 1;
  }
  SFG_HIP(launch_tiles(A->row_ptr, A->n, kTileNnz, rpt, tiles, tp, (int32_t)ntiles, st));
  T->ntiles = (int32_t)ntiles;
  T->grid = spmv_grid(ntiles);
  T->max_row = maxlen;
  return SFGMRES_OK;
}

struct Ptrs {
  DevCtl* ctl;
  int32_t *tiles, *tp, *ipart;
  double *part, *dpart, *vpart, *red, *V, *T, *R, *d, *scal, *tau, *ice_x, *ice_z, *sigma, *coef, *yin,
      *H, *HR, *cs, *sn, *g, *yout, *Vb, *Zb, *W64, *X;
  SkGroup* skp;
  void* Bb;
  float *W32, *val32;
};

Ptrs make_ptrs(char* base, const Layout& L) {
  Ptrs p;
  p.ctl = reinterpret_cast<DevCtl*>(base + L.ctl);
  p.tiles = reinterpret_cast<int32_t*>(base + L.tiles);
  p.tp = reinterpret_cast<int32_t*>(base + L.tp);
  p.ipart = reinterpret_cast<int32_t*>(base + L.ipart);
  p.part = reinterpret_cast<double*>(base + L.part);
  p.dpart = reinterpret_cast<double*>(base + L.dpart);
  p.vpart = reinterpret_cast<double*>(base + L.vpart);
  p.red = reinterpret_cast<double*>(base + L.red);
  p.skp = reinterpret_cast<SkGroup*>(base + L.skp);
  p.V = reinterpret_cast<double*>(base + L.qr_V);
  p.T = reinterpret_cast<double*>(base + L.qr_T);
  p.R = reinterpret_cast<double*>(base + L.qr_R);
  p.d = reinterpret_cast<double*>(base + L.qr_d);
  p.scal = reinterpret_cast<double*>(base + L.qr_c);
  p.tau = reinterpret_cast<double*>(base + L.qr_tau);
  p.ice_x = reinterpret_cast<double*>(base + L.ice_x);
  p.ice_z = reinterpret_cast<double*>(base + L.ice_z);
  p.sigma = reinterpret_cast<double*>(base + L.sigma);
  p.coef = reinterpret_cast<double*>(base + L.hwin);
  p.yin = reinterpret_cast<double*>(base + L.yin);
  p.H = reinterpret_cast<double*>(base + L.H);
  p.HR = reinterpret_cast<double*>(base + L.HR);
  p.cs = reinterpret_cast<double*>(base + L.cs);
  p.sn = reinterpret_cast<double*>(base + L.sn);
  p.g = reinterpret_cast<double*>(base + L.g);
  p.yout = reinterpret_cast<double*>(base + L.yout);
  p.Vb = reinterpret_cast<double*>(base + L.V);
  p.Zb = reinterpret_cast<double*>(base + L.Z);
  p.Bb = base + L.B;
  p.W32 = reinterpret_cast<float*>(base + L.W32);
  p.W64 = reinterpret_cast<double*>(base + L.W64);
  p.X = reinterpret_cast<double*>(base + L.X);
  p.val32 = reinterpret_cast<float*>(base + L.val32);
  return p;
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Host spin on the pinned status block until `pred` holds; fails after 60 s
// without the device making progress.
template <typename Pred>
bool spin_until(sfgmres_ctx* h, Pred pred) {
  volatile HostStatus* hs = h->hs_host;
  int last = hs->inner_step_done;
  double t0 = now_ms();
  int spins = 0;
  while (!pred()) {
    const int cur = hs->inner_step_done;
    if (cur != last) {
      last = cur;
      t0 = now_ms();
    }
    if (++spins > 64) {
      std::this_thread::yield();
      if (now_ms() - t0 > 60000.0) return false;
    }
  }
  return true;
}

// Host side of the ILU factors: level starts and lanes per row per colour.
struct IluHost {
  std::vector<int32_t> level;
  std::vector<int8_t> group;
};

// ILU(0) set-up on the device: diagonal positions and the check of the
// pattern, the transposed pattern, Jones-Plassmann rounds until every row
// is coloured, rows grouped by colour (level starts read back to the
// host), the factorisation one colour at a time, and the copies of the
// factors in the colour order for the triangular solves (their values in
// FP32 when fp32: the mixed-precision solves read those).
int ilu_setup(sfgmres_handle h, const sfgmres_csr* A, char* base, const IluWs& L,
              hipStream_t st, IluFactors* F, IluHost* host, bool fp32) {
  const int64_t n = A->n, nnz = A->nnz;
  double* lu = reinterpret_cast<double*>(base + L.lu);
  int8_t* kind = reinterpret_cast<int8_t*>(base + L.kind);
  int32_t* diag = reinterpret_cast<int32_t*>(base + L.diag);
  int32_t* state = reinterpret_cast<int32_t*>(base + L.state);
  int32_t* order = reinterpret_cast<int32_t*>(base + L.order);
  int32_t* cnt = reinterpret_cast<int32_t*>(base + L.cnt);
  int32_t* start = cnt + (kIluMaxColors + 1);
  int32_t* lsum = start + (kIluMaxColors + 1);
  int32_t* usum = lsum + (kIluMaxColors + 1);
  int32_t* err = usum + (kIluMaxColors + 1);
  int32_t* colored = err + 1;
  int32_t* maxrow = err + 2;
  int32_t* trp = reinterpret_cast<int32_t*>(base + L.t_rp);
  int32_t* tci = reinterpret_cast<int32_t*>(base + L.t_ci);
  int32_t* scan_tmp = reinterpret_cast<int32_t*>(base + L.t_scan);
  SFG_HIP(hipMemsetAsync(cnt, 0, kIluCntInts * 4, st));
  SFG_HIP(launch_ilu_init(n, A->row_ptr, A->col_idx, A->val, lu, diag, state, err, maxrow, st));
  SFG_HIP(launch_transpose(A->row_ptr, A->col_idx, nullptr, n, nnz, trp, tci, nullptr,
                           reinterpret_cast<int32_t*>(base + L.t_perm),
                           reinterpret_cast<int32_t*>(base + L.t_cursor), scan_tmp, st));
  int32_t hv[3] = {0, 0, 0};
  SFG_HIP(hipMemcpyAsync(hv, err, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SFG_HIP(hipStreamSynchronize(st));
  if (hv[0] & 3)
    return fail(h, SFGMRES_ERR_INVALID,
                "ILU(0) needs strictly increasing columns in every row and every diagonal entry");
  const bool long_rows = hv[2] > kIluLongRow;
  // (the globally highest-priority uncoloured vertex colours itself in every
  // round, so at most n rounds; the round number sits above the 12 colour bits)
  const int64_t max_rounds = std::min<int64_t>(n + 1, (int64_t)1 << 19);
  // (four rounds per look at the counters: a round after the last one
  // changes nothing)
  int64_t r = 0;
  for (;;) {
    if (r >= max_rounds) return fail(h, SFGMRES_ERR_INVALID, "ILU colouring did not finish");
    const int64_t burst = std::min<int64_t>(4, max_rounds - r);
    for (int64_t k = 0; k < burst; ++k, ++r)
      SFG_HIP(launch_ilu_jp_round(n, A->row_ptr, A->col_idx, trp, tci, state, (int32_t)r,
                                  colored, err, st));
    SFG_HIP(hipMemcpyAsync(hv, err, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SFG_HIP(hipStreamSynchronize(st));
    if (hv[1] >= n || hv[0]) break;
  }
  if (hv[0] & 4) return fail(h, SFGMRES_ERR_INVALID, "ILU colouring needs more than 4095 colours");
  SFG_HIP(launch_ilu_count(n, state, cnt, st));
  std::vector<int32_t> hc(kIluMaxColors + 1, 0);
  SFG_HIP(hipMemcpyAsync(hc.data(), cnt, hc.size() * 4, hipMemcpyDeviceToHost, st));
  SFG_HIP(hipStreamSynchronize(st));
  int nc = 0;
  for (int c = 0; c < kIluMaxColors; ++c)
    if (hc[c]) nc = c + 1;
  std::vector<int32_t>& lev = host->level;
  lev.assign(nc + 1, 0);
  for (int c = 0; c < nc; ++c) lev[c + 1] = lev[c] + hc[c];
  SFG_HIP(hipMemcpyAsync(start, lev.data(), (size_t)(nc + 1) * 4, hipMemcpyHostToDevice, st));
  SFG_HIP(launch_ilu_order(n, A->row_ptr, A->col_idx, state, nc, start,
                           reinterpret_cast<int32_t*>(base + L.hist), order, kind, st));
  for (int c = 0; c < nc; ++c)
    SFG_HIP(launch_ilu_factor(order, lev[c], lev[c + 1], A->row_ptr, A->col_idx, kind, diag, state,
                              lu, err, long_rows, st));
  int32_t* orp = reinterpret_cast<int32_t*>(base + L.orp);
  int32_t* omid = reinterpret_cast<int32_t*>(base + L.omid);
  int32_t* oci = reinterpret_cast<int32_t*>(base + L.oci);
  void* oval = base + L.oval;
  void* udiag = base + L.udiag;
  // (the transpose's cursor array is free again and holds the positions)
  SFG_HIP(launch_ilu_split(n, nnz, A->row_ptr, A->col_idx, kind, diag, lu, order, nc, start, orp,
                           omid, oci, oval, udiag, fp32, lsum, usum,
                           reinterpret_cast<int32_t*>(base + L.t_cursor), scan_tmp, st));
  std::vector<int32_t> sums(2 * (size_t)(kIluMaxColors + 1));
  SFG_HIP(hipMemcpyAsync(hv, err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SFG_HIP(hipMemcpyAsync(sums.data(), lsum, sums.size() * 4, hipMemcpyDeviceToHost, st));
  SFG_HIP(hipStreamSynchronize(st));
  if (hv[0] & 8) return fail(h, SFGMRES_ERR_BREAKDOWN, "zero pivot in the ILU(0) factorisation");
  host->group.assign(2 * (size_t)nc, 1);
  for (int c = 0; c < nc; ++c) {
    const int64_t rows = lev[c + 1] - lev[c];
    host->group[2 * c] = (int8_t)ilu_group(rows, sums[c]);
    host->group[2 * c + 1] = (int8_t)ilu_group(rows, sums[(kIluMaxColors + 1) + c]);
  }
  F->order = order;
  F->orp = orp;
  F->omid = omid;
  F->oci = oci;
  F->oval = oval;
  F->udiag = udiag;
  F->level = lev.data();
  F->group = host->group.data();
  F->ncolors = nc;
  F->fp32 = fp32;
  return SFGMRES_OK;
}

// Timing events of the phase_timers option (created once per handle).
constexpr int kPhaseMarks = 8;
int ensure_marks(sfgmres_handle h) {
  while ((int)h->pev.size() < kPhaseMarks) {
    hipEvent_t e;
    SFG_HIP(hipEventCreate(&e));
    h->pev.push_back(e);
  }
  return SFGMRES_OK;
}

int solve_impl(sfgmres_handle h, const sfgmres_csr* A, const double* b, const double* x0,
               double* x, int32_t m, int32_t t, int32_t s, int32_t zeta, double tol,
               uint64_t seed, const sfgmres_options& o, sfgmres_info* info, void* ws,
               size_t ws_bytes, hipStream_t st, const IluFactors* shared_ilu = nullptr) {
  const double t_start = now_ms();
  const int64_t n = A->n, nnz = A->nnz;
  int rc = check_params(h, n, nnz, m, t, s, zeta, tol, o);
  if (rc) return rc;
  if (!A->row_ptr || (nnz > 0 && (!A->col_idx || !A->val)) || !b || !x)
    return fail(h, SFGMRES_ERR_INVALID, "null array argument");
  const int pc = panel_cols(o);
  const Layout L = make_layout(n, nnz, m, t, s, zeta, o.max_outer, o.precision, 0, pc, o.precond,
                               o.mid_outer, o.matrix_format);
  if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(h, SFGMRES_ERR_WORKSPACE, "workspace missing, too small or not 256-byte aligned");
  char* base = static_cast<char*>(ws);
  const Ptrs P = make_ptrs(base, L);
  const bool f32 = o.precision == SFGMRES_MIXED;
  const int J = o.max_outer;
  const int ldh = J + 1;
  const int64_t ld = L.ld;
  const size_t vt = f32 ? 4 : 8;
  const int zb = sk_groups(zeta);
  const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu);
  const uint32_t k1 = (uint32_t)(seed >> 32);
  const double inv_sqrt_zeta = 1.0 / sqrt((double)zeta);
  const int lookahead = lookahead_steps(o);
  const int nring = 2 * pc;                         // ring of two panels
  const int64_t slot_part = (int64_t)kMaxGrid * s;  // ring slot of sketch rows
  const int64_t slot_red = s;                       // ring slot of reduced rows
  HostStatus* hsd = h->hs_dev;
  volatile HostStatus* hsh = h->hs_host;
  auto Bcol = [&](int64_t l) -> void* { return static_cast<char*>(P.Bb) + l * ld * vt; };
  auto Vcol = [&](int64_t l) { return P.Vb + l * ld; };
  auto Zcol = [&](int64_t l) { return P.Zb + l * ld; };
  const int32_t* forced = info ? info->forced_k : nullptr;
  if (forced)
    for (int j = 0; j < o.max_outer; ++j)
      if (forced[j] < 0 || forced[j] > m)
        return fail(h, SFGMRES_ERR_INVALID, "forced_k entries must lie in [0, m]");

  if (info) {
    info->outer_iters = 0;
    info->converged = 0;
    info->total_inner = 0;
    info->rel_residual = NAN;
    info->true_rel_residual = NAN;
    info->spmv_ms = 0.0;
    info->spmv_launches = 0;
    for (double& v : info->phase_ms) v = 0.0;
  }
  // Phase timers: marks recorded on the caller's stream at phase
  // boundaries; after each synchronisation the elapsed time between two
  // marks is added to the phase that lies between them.
  const bool timers = o.phase_timers != 0;
  enum { kMarkStart, kMarkSetup, kMarkCycle, kMarkDecided, kMarkZ, kMarkOuter, kMarkA, kMarkB };
  if (timers) {
    rc = ensure_marks(h);
    if (rc) return rc;
  }
  double phase[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  auto mark = [&](int slot) -> hipError_t {
    return timers ? hipEventRecord(h->pev[slot], st) : hipSuccess;
  };
  auto add_phase = [&](int ph, int a, int b) -> hipError_t {
    if (!timers) return hipSuccess;
    float ms = 0.f;
    const hipError_t e = hipEventElapsedTime(&ms, h->pev[a], h->pev[b]);
    phase[ph] += ms;
    return e;
  };
  // hand-over events: per panel, "its steps are enqueued" and "its rows are
  // reduced", then one for the last decision
  const int npanels = (m + pc - 1) / pc;
  while ((int)h->sync.size() < 2 * npanels + 1) {
    hipEvent_t e;
    SFG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h->sync.push_back(e);
  }
  hipEvent_t* ev_steps = h->sync.data();
  hipEvent_t* ev_red = h->sync.data() + npanels;
  hipEvent_t ev_dec = h->sync[2 * npanels];
  if (o.profile && (int)h->ev.size() < 2 * m) {
    for (int i = (int)h->ev.size(); i < 2 * m; ++i) {
      hipEvent_t e;
      SFG_HIP(hipEventCreate(&e));
      h->ev.push_back(e);
    }
  }

  // ---- setup: control block, nnz-balanced tiles, float32 values, sketch --
  SFG_HIP(mark(kMarkStart));
  Tiling tiling{};
  rc = plan_tiling(h, A, P.tiles, P.tp, P.ipart, st, &tiling);
  if (rc) return rc;
  const int32_t ntiles = tiling.ntiles;
  const int Gp = tiling.grid;
  const int Gn = rows_grid(n);
  // (with a lower level, the preconditioner belongs to its sGMRES cycles;
  // the top level factors A once and hands the factors down)
  const bool mid = o.mid_outer > 0;
  const bool ilu = o.precond == SFGMRES_PRECOND_ILU0 && !mid;
  IluFactors F{};
  IluHost ilu_host;
  double* ilu_t64 = reinterpret_cast<double*>(base + L.ilu_t64);
  void* ilu_tmp = base + L.ilu_tmp;
  if (o.precond == SFGMRES_PRECOND_ILU0) {
    if (shared_ilu) {
      F = *shared_ilu;
    } else {
      rc = ilu_setup(h, A, base, ilu_regions(n, nnz, L.ilu), st, &F, &ilu_host, f32);
      if (rc) return rc;
    }
  }
  const int G2 = vec_grid(n);
  const int Ga = arnoldi_grid(n);  // the Arnoldi update (and its norm partials)
  memset((void*)hsh, 0, sizeof(HostStatus));
  SFG_HIP(launch_init_ctl(P.ctl, m, t, s, cond_threshold_of(o), tol, st));
  if (f32) SFG_HIP(launch_cast_f32(A->val, P.val32, nnz, st));
  if (o.identity_sketch)
    SFG_HIP(launch_sketch_identity(n, P.skp, st));
  else
    SFG_HIP(launch_sketch_pack(n, s, zeta, k0, k1, P.skp, st));

  SpmvArgs base_args{};
  base_args.n = n;
  base_args.row_ptr = A->row_ptr;
  base_args.col_idx = A->col_idx;
  base_args.val = A->val;
  base_args.tiles = P.tiles;
  base_args.tp = P.tp;
  base_args.ntiles = ntiles;
  base_args.short_tiles = tiling.max_row <= kShortRow;
  base_args.stream_matrix =
      !f32 && tiling.max_row > kShortRow && (size_t)nnz * 12 > kStreamMatrixBytes;
  base_args.part = P.part;
  base_args.dpart = P.dpart;
  base_args.ctl = P.ctl;
  base_args.scale_val = 1.0;
  base_args.skp = P.skp;
  base_args.zeta = zeta;
  base_args.sketch_gen =
      o.sketch_source == SFGMRES_SKETCH_GEN ||
      (o.sketch_source == SFGMRES_SKETCH_AUTO && !f32 && zb == 1 && !o.identity_sketch &&
       tiling.max_row <= kShortRow && (size_t)nnz * 12 > kGenSketchBytes);
  if (base_args.sketch_gen) base_args.stream_matrix = 0;
  if (info) info->sketch_generated = base_args.sketch_gen;
  // the matrix by diagonal, when every nonzero lies on the diagonals of the
  // first longest row (at most kDiaMax of them, rows of at most kShortRow
  // nonzeros: 64-row tiles) and the padding stays below half of nnz
  if (o.matrix_format == SFGMRES_MATRIX_AUTO && tiling.max_row > 0 &&
      tiling.max_row <= kShortRow) {
    int32_t* dw = reinterpret_cast<int32_t*>(base + L.dia_work);
    SFG_HIP(launch_dia_detect(A->row_ptr, A->col_idx, n, tiling.max_row, dw, st));
    int32_t hw[3 + kDiaMax] = {};
    SFG_HIP(hipMemcpyAsync(hw, dw, sizeof(hw), hipMemcpyDeviceToHost, st));
    SFG_HIP(hipStreamSynchronize(st));
    if (hw[1] == 0 && hw[2] > 0 && hw[2] <= kDiaMax && (int64_t)hw[2] * n <= nnz + nnz / 2) {
      DiaOffsets offs{};
      for (int k = 0; k < hw[2]; ++k) offs.off[k] = hw[3 + k];
      void* dv = base + L.dia;
      SFG_HIP(launch_dia_fill(A->row_ptr, A->col_idx, A->val, n, L.ld, hw[2], offs,
                              f32 ? nullptr : static_cast<double*>(dv),
                              f32 ? static_cast<float*>(dv) : nullptr, st));
      base_args.dia_val = dv;
      base_args.dia_ld = L.ld;
      base_args.ndiag = hw[2];
      for (int k = 0; k < kDiaMax; ++k) base_args.dia_off[k] = offs.off[k];
    }
  }
  if (base_args.ndiag > 0) base_args.stream_matrix = 0;
  if (info) {
    info->dia_diagonals = base_args.ndiag;
    info->matrix_streamed = base_args.stream_matrix;
  }
  base_args.sk_k0 = k0;
  base_args.sk_k1 = k1;

  QrBlockArgs qa{};
  qa.red = P.red;
  qa.slot_red = slot_red;
  qa.nring = nring;
  qa.s = s;
  qa.m = m;
  qa.t = t;
  qa.inv_sqrt_zeta = inv_sqrt_zeta;
  qa.ctl = P.ctl;
  qa.hs = hsd;
  qa.V = P.V;
  qa.T = P.T;
  qa.R = P.R;
  qa.d = P.d;
  qa.tau = P.tau;
  qa.ice_x = P.ice_x;
  qa.ice_z = P.ice_z;
  qa.sigma = P.sigma;

  // S v for the normalised vector just written: sketch rows into ring slot
  // 0, reduced, then d0 and the cycle reset
  auto sketch_v_and_init = [&](const double* W, const double* hptr, double* vout,
                               int32_t forced_k) -> int {
    SFG_HIP(launch_normalize_sketch(f32, Gn, n, W, hptr, vout, Bcol(0), s, P.skp, zeta, P.part,
                                    st));
    SFG_HIP(launch_reduce_slots(P.part, Gn, s, s, 0, 1, nring, slot_part, slot_red, P.red, P.ctl,
                                false, st));
    SFG_HIP(launch_rq_init(P.red, s, inv_sqrt_zeta, forced_k, P.ctl, P.d, P.sigma, st));
    return SFGMRES_OK;
  };

  // ---- r0 = b - A x0, beta, ||b||, v_1, S v_1 -----------------------------
  {
    SpmvArgs a = base_args;
    a.has_x = x0 != nullptr;
    a.x = x0;
    a.w = P.W64;
    a.b = b;
    SFG_HIP(launch_spmv(kModeResid, false, Gp, a, 0, st));
    SFG_HIP(launch_spmv_finish(kModeResid, P.dpart, Gp, P.ctl, P.g, hsd, st));
  }
  rc = sketch_v_and_init(P.W64, &P.ctl->beta, Vcol(0), forced ? forced[0] : 0);
  if (rc) return rc;
  SFG_HIP(mark(kMarkSetup));
  SFG_HIP(hipStreamSynchronize(st));
  SFG_HIP(add_phase(0, kMarkStart, kMarkSetup));
  if (hsh->error) return fail(h, hsh->error, "non-finite initial residual or right-hand side");
  const double beta = hsh->beta;
  const double nb = hsh->nb;
  if (!isfinite(beta) || !isfinite(nb))
    return fail(h, SFGMRES_ERR_NONFINITE, "non-finite initial residual or right-hand side");

  auto finish_info = [&](int status, int J_done, bool conv, double rel, double trel) {
    if (info) {
      info->outer_iters = J_done;
      info->converged = conv ? 1 : 0;
      info->rel_residual = rel;
      info->true_rel_residual = trel;
      info->status = status;
      info->solve_ms = now_ms() - t_start;
      for (int q = 0; q < 8; ++q) info->phase_ms[q] = phase[q];
    }
    return status;
  };

  if (nb == 0.0) {
    SFG_HIP(launch_copy_or_zero(nullptr, x, n, st));
    SFG_HIP(hipStreamSynchronize(st));
    return finish_info(SFGMRES_OK, 0, true, 0.0, 0.0);
  }
  if (info && info->residual_history) info->residual_history[0] = beta / nb;
  if (beta <= tol * nb) {
    SFG_HIP(launch_copy_or_zero(x0, x, n, st));
    SFG_HIP(hipStreamSynchronize(st));
    return finish_info(SFGMRES_OK, 0, true, beta / nb, beta / nb);
  }

  auto true_residual = [&](double* xv, double* r2) -> int {
    SpmvArgs a = base_args;
    a.x = xv;
    a.b = b;
    SFG_HIP(launch_spmv(kModeTrueRes, false, Gp, a, 0, st));
    SFG_HIP(launch_spmv_finish(kModeTrueRes, P.dpart, Gp, P.ctl, P.scal, hsd, st));
    SFG_HIP(mark(kMarkB));
    SFG_HIP(hipMemcpyAsync(r2, P.scal, sizeof(double), hipMemcpyDeviceToHost, st));
    SFG_HIP(hipStreamSynchronize(st));
    return SFGMRES_OK;
  };

  // ---- outer loop: FGMRES (Algorithm 1), or restarted sGMRES --------------
  const bool restarted = o.outer == SFGMRES_OUTER_RESTARTED;
  double beta_cur = beta;  // restarted: ||b - A x|| of the current iterate, held in x
  if (restarted) SFG_HIP(launch_copy_or_zero(x0, x, n, st));
  int J_done = 0;
  bool conv = false;
  double rho_last = beta;
  int total_inner = 0;
  double factor_host = beta;  // ||r~_{j-1}|| of eq. (2.2) (beta for j = 1)
  for (int j = 0; j < J; ++j) {
    int mid_k = 0, mid_inner = 0;
    if (mid) {
      // two-level FGMRES (Section 5): z_j from a lower-level FGMRES solve of
      // A z = v_j, at most mid_outer steps, stopped once eq. (2.2) predicts
      // the top-level tolerance (its residual times ||r~_{j-1}|| below
      // tol ||b||)
      SFG_HIP(mark(kMarkCycle));
      sfgmres_options om = o;
      om.max_outer = o.mid_outer;
      om.mid_outer = 0;
      om.record_true_residual = 0;
      om.profile = 0;
      om.phase_timers = 0;
      sfgmres_info mi;
      memset(&mi, 0, sizeof(mi));
      const double tol_mid = isfinite(factor_host) ? tol * nb / factor_host : tol * nb;
      const int mrc = solve_impl(h, A, Vcol(j), nullptr, Zcol(j), m, t, s, zeta, tol_mid, seed,
                                 om, &mi, base + L.mid, L.mid_bytes, st,
                                 o.precond == SFGMRES_PRECOND_ILU0 ? &F : nullptr);
      if (mrc < 0) return mrc;
      mid_k = mi.outer_iters;
      mid_inner = mi.total_inner;
      SFG_HIP(mark(kMarkDecided));
    } else {
      // inner sGMRES cycle: predicated steps, a decision launch per panel, a
      // bounded lookahead
      hsh->stop_k = 0;
      hsh->inner_step_done = 0;
      hsh->stop_step = 0;
      hsh->steps_run = 0;
      SFG_HIP(mark(kMarkCycle));
      int panel0 = 0;  // first column of the open panel
      for (int i = 0; i < m; ++i) {
        if (i >= lookahead) {
          const int need = i - lookahead + 1;
          if (!spin_until(h, [&] { return hsh->stop_k != 0 || hsh->inner_step_done >= need ||
                                          hsh->error != 0; })) {
            return fail(h, SFGMRES_ERR_TIMEOUT, "device made no progress for 60 s");
          }
        }
        if (hsh->stop_k != 0 || hsh->error != 0) break;
        const int nwin = std::min(t, i + 1);
        const int l0 = i + 1 - nwin;
        // this step's ring slot was read by the reduction of the panel two
        // panels back
        if (i % pc == 0 && i >= nring) SFG_HIP(hipStreamWaitEvent(st, ev_red[i / pc - 2], 0));
        SpmvArgs a = base_args;
        a.val = f32 ? static_cast<const void*>(P.val32) : static_cast<const void*>(A->val);
        a.x = Bcol(i);
        if (ilu) {
          // the inner operator A M^{-1}: the SpMV reads M^{-1} u_i (the solves
          // are predicated on the stop flag as the SpMV is)
          SFG_HIP(launch_ilu_apply(f32, F, Bcol(i), ilu_t64, ilu_tmp, st, P.ctl));
          a.x = ilu_tmp;
        }
        // t = 0: y = sigma_i A u_i = A b_i is the next (unnormalised) power-basis
        // vector, sigma_i formed by the SpMV itself from the previous step's
        // norm partials (sigma_0 is set with the cycle); t > 0: y = A u_i,
        // scaled inside the Arnoldi update.  Scalar rows alternate between two
        // buffers, so a step reads its predecessor's while writing its own.
        double* const dcur = P.dpart + (int64_t)(i & 1) * kMaxGrid * kDP;
        a.dpart = dcur;
        a.scale_ptr = (t == 0 && i == 0) ? P.sigma : nullptr;
        if (t == 0 && i > 0) {
          a.sig_part = P.dpart + (int64_t)((i - 1) & 1) * kMaxGrid * kDP;
          a.sig_G = Gp;
          a.sig_step = i;
          a.sig_out = P.sigma + i;
        }
        a.w = (t == 0) ? Bcol(i + 1) : (f32 ? static_cast<void*>(P.W32) : static_cast<void*>(P.W64));
        a.s = s;
        a.U = P.Bb;
        a.ldu = ld;
        a.l0 = l0;
        a.nwin = nwin;
        a.part = P.part + (int64_t)(i % nring) * slot_part;
        const bool timed = o.profile > 0 && i % o.profile == o.profile - 1;
        SFG_HIP(launch_spmv(kModeInner, f32, Gp, a, zb, st, timed ? h->ev[2 * i] : nullptr,
                            timed ? h->ev[2 * i + 1] : nullptr));
        // t > 0: sigma and the window coefficients inside the Arnoldi update
        // (norm partials alternate between two buffers), or a one-workgroup
        // kernel at the cycle's last step; t = 0: nothing (the next SpMV
        // forms sigma)
        double* vprev = P.vpart + (int64_t)(i & 1) * kVecGrid;
        double* vnext = P.vpart + (int64_t)((i + 1) & 1) * kVecGrid;
        if (t > 0 && i + 1 < m) {
          ArnoldiArgs aa{};
          aa.n = n;
          aa.W = f32 ? static_cast<const void*>(P.W32) : static_cast<const void*>(P.W64);
          aa.B = P.Bb;
          aa.ldb = ld;
          aa.l0 = l0;
          aa.nwin = nwin;
          aa.inext = i + 1;
          aa.step = i;
          aa.dpart = dcur;
          aa.Gd = Gp;
          aa.vprev = vprev;
          aa.Gv = Ga;
          aa.vnext = vnext;
          aa.sigma = P.sigma;
          aa.ctl = P.ctl;
          SFG_HIP(launch_arnoldi_update(f32, Ga, aa, st));
        } else if (t > 0) {
          CoefArgs ca{};
          ca.dpart = dcur;
          ca.G = Gp;
          ca.vpart = vprev;
          ca.Gv = Ga;
          ca.t = t;
          ca.nwin = nwin;
          ca.l0 = l0;
          ca.step = i;
          ca.ctl = P.ctl;
          ca.sigma = P.sigma;
          ca.coef = P.coef;
          SFG_HIP(launch_coef(ca, st));
        }
        if (i + 1 - panel0 == pc || i + 1 == m) {
          // the panel's reduction and decision on the decision stream, after
          // its steps; the inner steps go on meanwhile (they read the stop
          // flag at their start, so a decision seen late costs a discarded
          // step, never a wrong result)
          const int ncols = i + 1 - panel0;
          const int pidx = panel0 / pc;
          SFG_HIP(hipEventRecord(ev_steps[pidx], st));
          SFG_HIP(hipStreamWaitEvent(h->dec, ev_steps[pidx], 0));
          SFG_HIP(launch_reduce_slots(P.part, Gp, s, s, panel0 % nring, ncols, nring, slot_part,
                                      slot_red, P.red, P.ctl, true, h->dec));
          SFG_HIP(hipEventRecord(ev_red[pidx], h->dec));
          QrBlockArgs q = qa;
          q.k0 = panel0;
          q.ncols = ncols;
          q.pprev = panel0 > 0 ? pc : 0;  // every panel before the last is full
          SFG_HIP(launch_qr_block(q, h->dec));
          SFG_HIP(hipEventRecord(ev_dec, h->dec));
          panel0 = i + 1;
        }
      }
      // the cycle's last decision (and every earlier one) before its results
      SFG_HIP(hipStreamWaitEvent(st, ev_dec, 0));
      SFG_HIP(mark(kMarkDecided));
      // z_j = B_k y_k
      SFG_HIP(launch_finalize(P.ctl, P.R, P.d, P.sigma, m, P.yin, st));
      if (restarted) {
        // the cycle solved A z = r_j / beta_j: x <- x + beta_j z, then the new
        // residual r_{j+1} = b - A x and beta_{j+1} (also the next C3 factor)
        SFG_HIP(launch_combine(f32, n, P.Bb, ld, P.yin, &P.ctl->stop_k, 0, x, x, st,
                               &P.ctl->beta));
        SpmvArgs a = base_args;
        a.has_x = 1;
        a.x = x;
        a.w = P.W64;
        a.b = b;
        SFG_HIP(launch_spmv(kModeResid, false, Gp, a, 0, st));
        SFG_HIP(launch_spmv_finish(kModeRestart, P.dpart, Gp, P.ctl, P.scal, hsd, st));
        SFG_HIP(mark(kMarkZ));
        SFG_HIP(hipStreamSynchronize(st));
        SFG_HIP(add_phase(1, kMarkCycle, kMarkDecided));
        SFG_HIP(add_phase(2, kMarkDecided, kMarkZ));
        const int err = hsh->error;
        const int kj = hsh->k;
        beta_cur = hsh->beta;
        J_done = j + 1;
        total_inner += kj;
        if (info) {
          info->total_inner = total_inner;
          if (info->residual_history) info->residual_history[j + 1] = beta_cur / nb;
          if (info->inner_k) info->inner_k[j] = kj;
          if (info->stop_reason) info->stop_reason[j] = hsh->stop_reason;
          if (info->cond_at_stop) info->cond_at_stop[j] = hsh->cond;
          if (info->inner_sketched_residual) info->inner_sketched_residual[j] = hsh->rho_hat;
          if (info->inner_true_residual) info->inner_true_residual[j] = NAN;
          if (info->ffom_residual) info->ffom_residual[j] = NAN;
          if (info->true_residual_history) info->true_residual_history[j] = beta_cur / nb;
        }
        if (o.profile > 0) {
          const int worked = std::min((int)hsh->steps_run, m);
          for (int i = o.profile - 1; i < worked; i += o.profile) {
            float ms = 0.f;
            SFG_HIP(hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]));
            if (info) {
              info->spmv_ms += ms;
              info->spmv_launches += 1;
            }
          }
        }
        if (err) {
          finish_info(err, J_done, false, beta_cur / nb, beta_cur / nb);
          return fail(h, err,
                      err == SFGMRES_ERR_BREAKDOWN ? "sketch of A v_j is zero (singular inner problem)"
                                                   : "non-finite residual of a restart");
        }
        if (beta_cur <= tol * nb) {
          conv = true;
          break;
        }
        // v_{j+1} = r_{j+1} / beta_{j+1}, its copy as the next cycle's b_1, S v
        rc = sketch_v_and_init(P.W64, &P.ctl->beta, Vcol(0),
                               (forced && j + 1 < J) ? forced[j + 1] : 0);
        if (rc) return rc;
        continue;
      }
      if (ilu) {
        // z_j = M^{-1} B_k y_k
        SFG_HIP(launch_combine(f32, n, P.Bb, ld, P.yin, &P.ctl->stop_k, 0, nullptr, P.W64, st));
        SFG_HIP(launch_ilu_apply(false, F, P.W64, ilu_t64, Zcol(j), st));
      } else {
        SFG_HIP(launch_combine(f32, n, P.Bb, ld, P.yin, &P.ctl->stop_k, 0, nullptr, Zcol(j), st));
      }
    }
    SFG_HIP(mark(kMarkZ));
    // w = A z_j with h_{1,j}; modified Gram-Schmidt; Givens
    {
      SpmvArgs a = base_args;
      a.x = Zcol(j);
      a.w = P.W64;
      a.v0 = Vcol(0);
      a.vj = Vcol(j);
      SFG_HIP(launch_spmv(kModeOuter, false, Gp, a, 0, st));
      SFG_HIP(launch_spmv_finish(kModeOuter, P.dpart, Gp, P.ctl, P.H + (int64_t)j * ldh, hsd,
                                 st));
    }
    for (int l = 0; l <= j; ++l) {
      const bool last = l == j;
      double* hcol = P.H + (int64_t)j * ldh;
      SFG_HIP(launch_mgs_pass(G2, n, P.W64, Vcol(l), last ? Vcol(l) : Vcol(l + 1), hcol + l,
                              P.vpart, last ? 1 : 0, st));
      SFG_HIP(launch_mgs_finish(P.vpart, G2, hcol + l + 1, P.ctl, last ? 1 : 0, P.H, P.HR, P.cs,
                                P.sn, P.g, j, ldh, hsd, st));
    }
    // v_{j+1}, its copy as the next cycle's b_1, and S v_{j+1}
    rc = sketch_v_and_init(P.W64, P.H + (int64_t)j * ldh + j + 1, Vcol(j + 1),
                           (forced && j + 1 < J) ? forced[j + 1] : 0);
    if (rc) return rc;
    SFG_HIP(mark(kMarkOuter));
    SFG_HIP(hipStreamSynchronize(st));
    SFG_HIP(add_phase(1, kMarkCycle, kMarkDecided));
    SFG_HIP(add_phase(2, kMarkDecided, kMarkZ));
    SFG_HIP(add_phase(3, kMarkZ, kMarkOuter));
    const int err = hsh->error;
    const int kj = mid ? mid_k : hsh->k;
    const double rho = hsh->rho;
    factor_host = hsh->ffom;
    J_done = j + 1;
    total_inner += mid ? mid_inner : kj;
    if (o.profile > 0 && !mid) {
      const int worked = std::min((int)hsh->steps_run, m);
      for (int i = o.profile - 1; i < worked; i += o.profile) {
        float ms = 0.f;
        SFG_HIP(hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]));
        if (info) {
          info->spmv_ms += ms;
          info->spmv_launches += 1;
        }
      }
    }
    if (info) {
      info->total_inner = total_inner;
      if (info->residual_history) info->residual_history[j + 1] = rho / nb;
      if (info->inner_k) info->inner_k[j] = kj;
      if (info->stop_reason) info->stop_reason[j] = mid ? SFGMRES_STOP_MID : hsh->stop_reason;
      if (info->cond_at_stop) info->cond_at_stop[j] = mid ? NAN : hsh->cond;
      if (info->inner_sketched_residual)
        info->inner_sketched_residual[j] = mid ? NAN : hsh->rho_hat;
      if (info->inner_true_residual) info->inner_true_residual[j] = hsh->rhat_true;
      if (info->ffom_residual) info->ffom_residual[j] = hsh->ffom;
      if (info->bound) info->bound[j] = hsh->bound;
      if (info->delta_bound) info->delta_bound[j] = hsh->delta;
    }
    if (err) {
      finish_info(err, J_done, false, rho / nb, NAN);
      return fail(h, err,
                  err == SFGMRES_ERR_BREAKDOWN
                      ? "singular inner problem (S A v_j = 0) or singular H_j with h_{j+1,j} = 0"
                      : "non-finite value in the outer recurrence");
    }
    rho_last = rho;
    if (o.record_true_residual) {
      SFG_HIP(mark(kMarkA));
      SFG_HIP(launch_backsolve(P.HR, P.g, J_done, ldh, P.yout, st));
      SFG_HIP(launch_combine(false, n, P.Zb, ld, P.yout, nullptr, J_done, x0, P.X, st));
      double r2 = 0.0;
      rc = true_residual(P.X, &r2);
      if (rc) return rc;
      SFG_HIP(add_phase(4, kMarkA, kMarkB));
      if (info && info->true_residual_history) info->true_residual_history[j] = sqrt(r2) / nb;
    }
    if (hsh->hnext == 0.0 || rho <= tol * nb) {
      conv = true;
      break;
    }
  }

  if (restarted) {  // x holds the iterate and beta_cur its true residual
    SFG_HIP(hipStreamSynchronize(st));
    const int status = conv ? SFGMRES_OK : SFGMRES_NOT_CONVERGED;
    return finish_info(status, J_done, conv, beta_cur / nb, beta_cur / nb);
  }

  // ---- x = x0 + Z y, true residual, FFOM iterate ---------------------------
  SFG_HIP(mark(kMarkA));
  SFG_HIP(launch_backsolve(P.HR, P.g, J_done, ldh, P.yout, st));
  SFG_HIP(launch_combine(false, n, P.Zb, ld, P.yout, nullptr, J_done, x0, x, st));
  if (info && info->ffom_x) {
    // x~_J = x0 + Z_J H_J^{-1} beta e1 (Algorithm 1, FFOM)
    SFG_HIP(launch_backsolve(P.HR, P.g, J_done, ldh, P.yout, st, P.ctl));
    SFG_HIP(launch_combine(false, n, P.Zb, ld, P.yout, nullptr, J_done, x0, info->ffom_x, st));
  }
  double r2 = 0.0;
  rc = true_residual(x, &r2);
  if (rc) return rc;
  SFG_HIP(add_phase(5, kMarkA, kMarkB));
  const int status = conv ? SFGMRES_OK : SFGMRES_NOT_CONVERGED;
  return finish_info(status, J_done, conv, rho_last / nb, sqrt(r2) / nb);
}

// Workspace of the stand-alone sketch and SpMV entry points.
struct SmallLayout {
  size_t ctl, tiles, tp, ipart, part, dpart, red, skp, total;
};

SmallLayout small_layout(int64_t n, int64_t nnz, int32_t s, int32_t zeta) {
  SmallLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.ctl = take(sizeof(DevCtl));
  const size_t ntiles_max = (size_t)(n / kRowTile + nnz / kTileNnz + 3);
  L.tiles = take((ntiles_max + 1) * 4);
  L.tp = take((ntiles_max + 1) * 4);
  L.ipart = take((size_t)(kVecGrid + 1) * 4);
  L.part = take((size_t)kMaxGrid * s * 8);
  L.dpart = take((size_t)kMaxGrid * kDP * 8);
  L.red = take((size_t)s * 8);
  L.skp = take(packed_sketch_bytes(n, zeta));
  L.total = off;
  return L;
}

// Workspace of the matrix-powers export: as the fused-SpMV export, with a
// group of partial rows per level.
struct PowersLayout {
  size_t ctl, tiles, tp, ipart, part, dpart, red, skp, total;
};

PowersLayout powers_layout(int64_t n, int64_t nnz, int32_t p, int32_t s, int32_t zeta) {
  PowersLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.ctl = take(sizeof(DevCtl));
  const size_t ntiles_max = (size_t)(n / kRowTile + nnz / kTileNnz + 3);
  L.tiles = take((ntiles_max + 1) * 4);
  L.tp = take((ntiles_max + 1) * 4);
  L.ipart = take((size_t)(kVecGrid + 1) * 4);
  L.part = take((size_t)kSpmvGrid * s * 8);  // p groups of kSpmvGrid / p rows
  L.dpart = take((size_t)kSpmvGrid * kDP * 8);
  L.red = take((size_t)p * s * 8);
  L.skp = take(packed_sketch_bytes(n, zeta));
  L.total = off;
  return L;
}

}  // namespace

namespace sfg {

int report_error(sfgmres_ctx* h, int code, const std::string& msg) { return fail(h, code, msg); }

size_t spmv_sketch_workspace(int64_t n, int64_t nnz, int32_t s, int32_t zeta) {
  return small_layout(n, nnz, s, zeta).total;
}

// The fused SpMV export on a given workspace (the entry points with and
// without a workspace argument share it).
int spmv_sketch_impl(sfgmres_handle h, const sfgmres_csr* A, const double* u, double scale,
                     double* w, int32_t s, int32_t zeta, uint64_t seed, const double* U,
                     int64_t ldu, int32_t nwin, double* c, double* dots, double* norm2, void* ws,
                     size_t ws_bytes, void* stream) {
  if (!h) return SFGMRES_ERR_INVALID;
  if (!A || !A->row_ptr || !u || !c || !norm2 || (A->nnz > 0 && (!A->col_idx || !A->val)))
    return fail(h, SFGMRES_ERR_INVALID, "null array argument");
  if (A->nnz < 0 || A->nnz >= ((int64_t)1 << 31) || !sketch_args_ok(A->n, s, zeta) || nwin < 0 ||
      nwin > SFGMRES_MAX_T || (nwin > 0 && (!U || !dots || ldu < A->n)))
    return fail(h, SFGMRES_ERR_INVALID, "invalid sizes");
  const SmallLayout L = small_layout(A->n, A->nnz, s, zeta);
  if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(h, SFGMRES_ERR_WORKSPACE, "workspace missing, too small or not 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  DevCtl* ctl = reinterpret_cast<DevCtl*>(base + L.ctl);
  int32_t* tiles = reinterpret_cast<int32_t*>(base + L.tiles);
  int32_t* tp = reinterpret_cast<int32_t*>(base + L.tp);
  int32_t* ipart = reinterpret_cast<int32_t*>(base + L.ipart);
  double* part = reinterpret_cast<double*>(base + L.part);
  double* dpart = reinterpret_cast<double*>(base + L.dpart);
  double* red = reinterpret_cast<double*>(base + L.red);
  SkGroup* skp = reinterpret_cast<SkGroup*>(base + L.skp);
  Tiling tiling{};
  const int prc = plan_tiling(h, A, tiles, tp, ipart, st, &tiling);
  if (prc) return prc;
  const int32_t ntiles = tiling.ntiles;
  const int Gp = tiling.grid;
  SFG_HIP(launch_init_ctl(ctl, 1, 0, s, 1e15, 1.0, st));
  SFG_HIP(launch_sketch_pack(A->n, s, zeta, (uint32_t)(seed & 0xFFFFFFFFu),
                             (uint32_t)(seed >> 32), skp, st));
  SpmvArgs a{};
  a.n = A->n;
  a.row_ptr = A->row_ptr;
  a.col_idx = A->col_idx;
  a.val = A->val;
  a.tiles = tiles;
  a.tp = tp;
  a.ntiles = ntiles;
  a.short_tiles = tiling.max_row <= kShortRow;
  a.x = u;
  a.scale_val = scale;
  a.w = w;
  a.s = s;
  a.skp = skp;
  a.zeta = zeta;
  a.U = U;
  a.ldu = ldu;
  a.l0 = 0;
  a.nwin = nwin;
  a.part = part;
  a.dpart = dpart;
  a.ctl = ctl;
  SFG_HIP(launch_spmv(kModePlain, false, Gp, a, sk_groups(zeta), st));
  SFG_HIP(launch_reduce_slots(part, Gp, s, s, 0, 1, 1, 0, 0, red, ctl, false, st));
  SFG_HIP(launch_sketch_out(red, s, 1.0 / sqrt((double)zeta), dpart, Gp, nwin, c, dots, norm2,
                            st));
  SFG_HIP(hipStreamSynchronize(st));
  return SFGMRES_OK;
}

}  // namespace sfg

extern "C" {

int sfgmres_default_options(sfgmres_options* opt) {
  if (!opt) return SFGMRES_ERR_INVALID;
  *opt = defaults();
  return SFGMRES_OK;
}

int sfgmres_workspace_bytes(int64_t n, int64_t nnz, int32_t m, int32_t t, int32_t s, int32_t zeta,
                            const sfgmres_options* opt, int32_t adjoint, size_t* bytes) {
  if (!bytes) return SFGMRES_ERR_INVALID;
  const sfgmres_options o = opt ? *opt : defaults();
  if (n < 1 || nnz < 0 || m < 1 || s <= m || s > SFGMRES_MAX_S || m > SFGMRES_MAX_M || t < 0 ||
      zeta < 1 || zeta > SFGMRES_MAX_ZETA || o.max_outer < 1 || o.max_outer > SFGMRES_MAX_OUTER ||
      o.lookahead < 0 || o.lookahead > 64 || o.panel < 0 || o.panel > kPanel)
    return SFGMRES_ERR_INVALID;
  *bytes = make_layout(n, nnz, m, t, s, zeta, o.max_outer, o.precision, adjoint ? 1 : 0,
                       panel_cols(o), o.precond, o.mid_outer, o.matrix_format)
               .total;
  return SFGMRES_OK;
}

int sfgmres_create(sfgmres_handle* out) {
  if (!out) return SFGMRES_ERR_INVALID;
  *out = nullptr;
  sfgmres_ctx* c = new (std::nothrow) sfgmres_ctx();
  if (!c) return SFGMRES_ERR_INVALID;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return SFGMRES_ERR_HIP;
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, sizeof(HostStatus), hipHostMallocMapped | hipHostMallocCoherent) !=
      hipSuccess) {
    delete c;
    return SFGMRES_ERR_HIP;
  }
  memset(p, 0, sizeof(HostStatus));
  c->hs_host = static_cast<HostStatus*>(p);
  void* dp = nullptr;
  if (hipHostGetDevicePointer(&dp, p, 0) != hipSuccess) {
    (void)hipHostFree(p);
    delete c;
    return SFGMRES_ERR_HIP;
  }
  c->hs_dev = static_cast<HostStatus*>(dp);
  // the decision stream: default priority, no implicit ordering with the
  // null stream
  if (hipStreamCreateWithFlags(&c->dec, hipStreamNonBlocking) != hipSuccess) {
    (void)hipHostFree(p);
    delete c;
    return SFGMRES_ERR_HIP;
  }
  *out = c;
  return SFGMRES_OK;
}

void sfgmres_destroy(sfgmres_handle h) {
  if (!h) return;
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->pev) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->sync) (void)hipEventDestroy(e);
  if (h->dec) (void)hipStreamDestroy(h->dec);
  if (h->hs_host) (void)hipHostFree(h->hs_host);
  delete h;
}

const char* sfgmres_last_error(sfgmres_handle h) { return h ? h->err.c_str() : "null handle"; }

int sfgmres_solve(sfgmres_handle h, const sfgmres_csr* A, const double* b, const double* x0,
                  double* x, int32_t m, int32_t t, int32_t s, int32_t zeta, double tol,
                  uint64_t seed, const sfgmres_options* opt, sfgmres_info* info, void* ws,
                  size_t ws_bytes, void* stream) {
  if (!h) return SFGMRES_ERR_INVALID;
  if (!A) return fail(h, SFGMRES_ERR_INVALID, "null matrix");
  h->err.clear();
  const sfgmres_options o = opt ? *opt : defaults();
  try {
    return solve_impl(h, A, b, x0, x, m, t, s, zeta, tol, seed, o, info, ws, ws_bytes,
                      static_cast<hipStream_t>(stream));
  } catch (...) {
    return fail(h, SFGMRES_ERR_INVALID, "internal exception");
  }
}

int sfgmres_solve_adjoint(sfgmres_handle h, const sfgmres_csr* A, const double* g,
                          double* lambda, const double* x, double* grad_val, int32_t m,
                          int32_t t, int32_t s, int32_t zeta, double tol, uint64_t seed,
                          const sfgmres_options* opt, sfgmres_info* info, void* ws,
                          size_t ws_bytes, void* stream) {
  if (!h) return SFGMRES_ERR_INVALID;
  if (!A || !A->row_ptr) return fail(h, SFGMRES_ERR_INVALID, "null matrix");
  h->err.clear();
  const sfgmres_options o = opt ? *opt : defaults();
  int rc = check_params(h, A->n, A->nnz, m, t, s, zeta, tol, o);
  if (rc) return rc;
  if ((A->nnz > 0 && (!A->col_idx || !A->val)) || !g || !lambda)
    return fail(h, SFGMRES_ERR_INVALID, "null array argument");
  const Layout L = make_layout(A->n, A->nnz, m, t, s, zeta, o.max_outer, o.precision, 1,
                               panel_cols(o), o.precond, o.mid_outer, o.matrix_format);
  if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(h, SFGMRES_ERR_WORKSPACE, "workspace missing, too small or not 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  int32_t* rp_t = reinterpret_cast<int32_t*>(base + L.at_rowptr);
  int32_t* col_t = reinterpret_cast<int32_t*>(base + L.at_col);
  double* val_t = reinterpret_cast<double*>(base + L.at_val);
  int32_t* perm = reinterpret_cast<int32_t*>(base + L.at_perm);
  int32_t* cursor = reinterpret_cast<int32_t*>(base + L.at_cursor);
  int32_t* scan_tmp = reinterpret_cast<int32_t*>(base + L.scan_tmp);
  // (phase_timers: the transpose and the gradient are timed with the last
  // two phase marks, each read before the solve reuses them)
  const bool timers = o.phase_timers != 0;
  if (timers) {
    rc = ensure_marks(h);
    if (rc) return rc;
    SFG_HIP(hipEventRecord(h->pev[kPhaseMarks - 2], st));
  }
  SFG_HIP(launch_transpose(A->row_ptr, A->col_idx, A->val, A->n, A->nnz, rp_t, col_t, val_t, perm,
                           cursor, scan_tmp, st));
  float t_transpose = 0.f;
  if (timers) {
    SFG_HIP(hipEventRecord(h->pev[kPhaseMarks - 1], st));
    SFG_HIP(hipEventSynchronize(h->pev[kPhaseMarks - 1]));
    SFG_HIP(hipEventElapsedTime(&t_transpose, h->pev[kPhaseMarks - 2], h->pev[kPhaseMarks - 1]));
  }
  sfgmres_csr AT{A->n, A->nnz, rp_t, col_t, val_t};
  try {
    rc = solve_impl(h, &AT, g, nullptr, lambda, m, t, s, zeta, tol, seed, o, info, ws, L.at_rowptr,
                    st);
  } catch (...) {
    return fail(h, SFGMRES_ERR_INVALID, "internal exception");
  }
  if (info && timers) info->phase_ms[6] = t_transpose;
  if (rc < 0) return rc;
  if (x && grad_val) {
    if (timers) SFG_HIP(hipEventRecord(h->pev[kPhaseMarks - 2], st));
    SFG_HIP(launch_gradient(A->row_ptr, A->col_idx, A->n, lambda, x, grad_val, st));
    if (timers) SFG_HIP(hipEventRecord(h->pev[kPhaseMarks - 1], st));
    SFG_HIP(hipStreamSynchronize(st));
    if (info && timers) {
      float ms = 0.f;
      SFG_HIP(hipEventElapsedTime(&ms, h->pev[kPhaseMarks - 2], h->pev[kPhaseMarks - 1]));
      info->phase_ms[7] = ms;
    }
  }
  return rc;
}

int sfgmres_transpose_workspace_bytes(int64_t n, int64_t nnz, size_t* bytes) {
  if (!bytes || n < 1 || nnz < 0) return SFGMRES_ERR_INVALID;
  *bytes = align256((size_t)(n + 1) * 4) + align256(transpose_scan_tmp_ints(n) * 4);
  return SFGMRES_OK;
}

int sfgmres_transpose(sfgmres_handle h, const sfgmres_csr* A, int32_t* row_ptr_t,
                      int32_t* col_idx_t, double* val_t, int32_t* perm, void* ws,
                      size_t ws_bytes, void* stream) {
  if (!h) return SFGMRES_ERR_INVALID;
  if (!A || !A->row_ptr || !row_ptr_t || !perm || (A->nnz > 0 && (!A->col_idx || !col_idx_t)))
    return fail(h, SFGMRES_ERR_INVALID, "null array argument");
  if (val_t && !A->val) return fail(h, SFGMRES_ERR_INVALID, "val_t needs A->val");
  size_t need = 0;
  if (sfgmres_transpose_workspace_bytes(A->n, A->nnz, &need) != SFGMRES_OK)
    return fail(h, SFGMRES_ERR_INVALID, "invalid sizes");
  if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(h, SFGMRES_ERR_WORKSPACE, "workspace missing, too small or not 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  int32_t* cursor = reinterpret_cast<int32_t*>(base);
  int32_t* scan_tmp = reinterpret_cast<int32_t*>(base + align256((size_t)(A->n + 1) * 4));
  SFG_HIP(launch_transpose(A->row_ptr, A->col_idx, A->val, A->n, A->nnz, row_ptr_t, col_idx_t,
                           val_t, perm, cursor, scan_tmp, st));
  SFG_HIP(hipStreamSynchronize(st));
  return SFGMRES_OK;
}

int sfgmres_powers_workspace_bytes(int64_t n, int64_t nnz, int32_t p, int32_t s, int32_t zeta,
                                   size_t* bytes) {
  if (!bytes || nnz < 0 || nnz >= ((int64_t)1 << 31) || p < 1 || p > kMaxPowTasks ||
      !sketch_args_ok(n, s, zeta))
    return SFGMRES_ERR_INVALID;
  *bytes = powers_layout(n, nnz, p, s, zeta).total;
  return SFGMRES_OK;
}

int sfgmres_matrix_powers(sfgmres_handle h, const sfgmres_csr* A, const double* u, int32_t p,
                          int32_t s, int32_t zeta, uint64_t seed, int64_t slab_rows, double* Y,
                          int64_t ldy, double* C, double* norm2, void* ws, size_t ws_bytes,
                          void* stream) {
  if (!h) return SFGMRES_ERR_INVALID;
  h->err.clear();
  if (!A || !A->row_ptr || !u || !Y || !C || !norm2 || (A->nnz > 0 && (!A->col_idx || !A->val)))
    return fail(h, SFGMRES_ERR_INVALID, "null array argument");
  size_t need = 0;
  if (sfgmres_powers_workspace_bytes(A->n, A->nnz, p, s, zeta, &need) != SFGMRES_OK ||
      ldy < A->n || slab_rows < 0)
    return fail(h, SFGMRES_ERR_INVALID, "invalid sizes (need 1 <= p <= 8, ldy >= n)");
  if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(h, SFGMRES_ERR_WORKSPACE, "workspace missing, too small or not 256-byte aligned");
  const int64_t n = A->n;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  const PowersLayout L = powers_layout(n, A->nnz, p, s, zeta);
  DevCtl* ctl = reinterpret_cast<DevCtl*>(base + L.ctl);
  int32_t* tiles = reinterpret_cast<int32_t*>(base + L.tiles);
  int32_t* tp = reinterpret_cast<int32_t*>(base + L.tp);
  int32_t* ipart = reinterpret_cast<int32_t*>(base + L.ipart);
  double* part = reinterpret_cast<double*>(base + L.part);
  double* dpart = reinterpret_cast<double*>(base + L.dpart);
  double* red = reinterpret_cast<double*>(base + L.red);
  SkGroup* skp = reinterpret_cast<SkGroup*>(base + L.skp);
  Tiling tiling{};
  int rc = plan_tiling(h, A, tiles, tp, ipart, st, &tiling);
  if (rc) return rc;
  // bandwidth: level l+1 of a slab reads level l within that many rows
  int32_t bw = 0;
  SFG_HIP(launch_max_bandwidth(A->row_ptr, A->col_idx, n, ipart, ipart + kVecGrid, st));
  SFG_HIP(hipMemcpyAsync(&bw, ipart + kVecGrid, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  std::vector<int32_t> trow(tiling.ntiles + 1);
  SFG_HIP(hipMemcpyAsync(trow.data(), tiles, trow.size() * 4, hipMemcpyDeviceToHost, st));
  SFG_HIP(hipStreamSynchronize(st));
  // slabs: consecutive tiles with at least max(bw, slab_rows) rows each
  // (default: about 160 MB of matrix and vectors in flight between a
  // slab's first and last level, so its rows stay in the last-level cache)
  const double row_bytes = 12.0 * (double)A->nnz / (double)n + 16.0;
  int64_t want = slab_rows;
  if (want == 0)
    want = p > 1 ? (int64_t)(160e6 / (2.0 * p * (p - 1)) / row_bytes) : n;
  want = std::max<int64_t>({want, (int64_t)bw, 1});
  std::vector<int32_t> slab{0};  // first tile of each slab
  for (int t = 1; t < tiling.ntiles; ++t)
    if (trow[t] - trow[slab.back()] >= want) slab.push_back(t);
  slab.push_back(tiling.ntiles);
  if (slab.size() > 2 && trow[tiling.ntiles] - trow[slab[slab.size() - 2]] < bw)
    slab.erase(slab.end() - 2);  // (a short last slab joins its neighbour)
  const int K = (int)slab.size() - 1;
  SFG_HIP(launch_sketch_pack(n, s, zeta, (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32),
                             skp, st));
  // launch tau computes slab tau - 2 l of level l+1: its inputs (level l on
  // the slab and its two neighbours) were finished by earlier launches
  const int gp = std::max(1, tiling.grid / p);
  SpmvArgs a{};
  a.n = n;
  a.row_ptr = A->row_ptr;
  a.col_idx = A->col_idx;
  a.val = A->val;
  a.tiles = tiles;
  a.tp = tp;
  a.ntiles = tiling.ntiles;
  a.short_tiles = tiling.max_row <= kShortRow;
  a.s = s;
  a.skp = skp;
  a.zeta = zeta;
  a.ctl = ctl;
  a.ptasks = p;
  for (int tau = 0; tau < K + 2 * (p - 1); ++tau) {
    for (int l = 0; l < p; ++l) {
      const int k = tau - 2 * l;
      PowTask& T = a.ptask[l];
      T.active = (k >= 0 && k < K) ? 1 : 0;
      T.first = k == 0 ? 1 : 0;
      T.tile0 = T.active ? slab[k] : 0;
      T.ntiles = T.active ? slab[k + 1] - slab[k] : 0;
      T.x = l == 0 ? static_cast<const void*>(u) : static_cast<const void*>(Y + (l - 1) * ldy);
      T.w = Y + l * ldy;
      T.part = part + (int64_t)l * gp * s;
      T.dpart = dpart + (int64_t)l * gp * kDP;
    }
    SFG_HIP(launch_spmv(kModePowers, false, gp * p, a, sk_groups(zeta), st));
  }
  SFG_HIP(launch_reduce_slots(part, gp, s, s, 0, p, p, (int64_t)gp * s, s, red, ctl, false, st));
  for (int l = 0; l < p; ++l)
    SFG_HIP(launch_sketch_out(red + (int64_t)l * s, s, 1.0 / sqrt((double)zeta),
                              dpart + (int64_t)l * gp * kDP, gp, 0, C + (int64_t)l * s, nullptr,
                              norm2 + l, st));
  SFG_HIP(hipStreamSynchronize(st));
  return SFGMRES_OK;
}

int sfgmres_ilu_workspace_bytes(int64_t n, int64_t nnz, size_t* bytes) {
  if (!bytes || n < 1 || n >= ((int64_t)1 << 31) || nnz < 0 || nnz >= ((int64_t)1 << 31))
    return SFGMRES_ERR_INVALID;
  *bytes = ilu_regions(n, nnz, 0).total;
  return SFGMRES_OK;
}

int sfgmres_ilu0(sfgmres_handle h, const sfgmres_csr* A, double* lu, int32_t* color, void* ws,
                 size_t ws_bytes, void* stream) {
  if (!h) return SFGMRES_ERR_INVALID;
  if (!A || !A->row_ptr || !A->col_idx || !A->val || !lu || !color)
    return fail(h, SFGMRES_ERR_INVALID, "null array argument");
  size_t need = 0;
  if (sfgmres_ilu_workspace_bytes(A->n, A->nnz, &need) != SFGMRES_OK)
    return fail(h, SFGMRES_ERR_INVALID, "invalid sizes");
  if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(h, SFGMRES_ERR_WORKSPACE, "workspace missing, too small or not 256-byte aligned");
  h->err.clear();
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  const IluWs W = ilu_regions(A->n, A->nnz, 0);
  IluFactors F{};
  IluHost host;
  const int rc = ilu_setup(h, A, base, W, st, &F, &host, false);
  if (rc) return rc;
  SFG_HIP(hipMemcpyAsync(lu, base + W.lu, (size_t)A->nnz * 8, hipMemcpyDeviceToDevice, st));
  SFG_HIP(launch_ilu_colors(A->n, reinterpret_cast<const int32_t*>(base + W.state), color, st));
  SFG_HIP(hipStreamSynchronize(st));
  return SFGMRES_OK;
}

int sfgmres_sketch_workspace_bytes(int64_t n, int32_t s, int32_t zeta, size_t* bytes) {
  if (!bytes || !sketch_args_ok(n, s, zeta)) return SFGMRES_ERR_INVALID;
  *bytes = small_layout(n, 0, s, zeta).total;
  return SFGMRES_OK;
}

int sfgmres_sketch_materialize(sfgmres_handle h, int64_t n, int32_t s, int32_t zeta,
                               uint64_t seed, int32_t* rows, int8_t* signs, void* ws,
                               size_t ws_bytes, void* stream) {
  if (!h) return SFGMRES_ERR_INVALID;
  if (!sketch_args_ok(n, s, zeta)) return fail(h, SFGMRES_ERR_INVALID, "invalid (n, s, zeta)");
  if (!rows || !signs) return fail(h, SFGMRES_ERR_INVALID, "null array argument");
  const SmallLayout L = small_layout(n, 0, s, zeta);
  if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(h, SFGMRES_ERR_WORKSPACE, "workspace missing, too small or not 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  SkGroup* skp = reinterpret_cast<SkGroup*>(static_cast<char*>(ws) + L.skp);
  SFG_HIP(launch_sketch_pack(n, s, zeta, (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32),
                             skp, st));
  SFG_HIP(launch_sketch_unpack(n, zeta, skp, rows, signs, st));
  SFG_HIP(hipStreamSynchronize(st));
  return SFGMRES_OK;
}

int sfgmres_sketch_apply(sfgmres_handle h, int64_t n, int32_t s, int32_t zeta, uint64_t seed,
                         const double* w, double* out, void* ws, size_t ws_bytes,
                         void* stream) {
  if (!h) return SFGMRES_ERR_INVALID;
  if (!sketch_args_ok(n, s, zeta)) return fail(h, SFGMRES_ERR_INVALID, "invalid (n, s, zeta)");
  if (!w || !out) return fail(h, SFGMRES_ERR_INVALID, "null array argument");
  const SmallLayout L = small_layout(n, 0, s, zeta);
  if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(h, SFGMRES_ERR_WORKSPACE, "workspace missing, too small or not 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  DevCtl* ctl = reinterpret_cast<DevCtl*>(base + L.ctl);
  double* part = reinterpret_cast<double*>(base + L.part);
  double* red = reinterpret_cast<double*>(base + L.red);
  SkGroup* skp = reinterpret_cast<SkGroup*>(base + L.skp);
  const int G = rows_grid(n);
  SFG_HIP(launch_init_ctl(ctl, 1, 0, s, 1e15, 1.0, st));
  SFG_HIP(launch_sketch_pack(n, s, zeta, (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32),
                             skp, st));
  SFG_HIP(launch_normalize_sketch(false, G, n, w, nullptr, nullptr, nullptr, s, skp, zeta, part,
                                  st));
  SFG_HIP(launch_reduce_slots(part, G, s, s, 0, 1, 1, 0, 0, red, ctl, false, st));
  SFG_HIP(launch_sketch_out(red, s, 1.0 / sqrt((double)zeta), nullptr, 0, 0, out, nullptr,
                            nullptr, st));
  SFG_HIP(hipStreamSynchronize(st));
  return SFGMRES_OK;
}

int sfgmres_spmv_workspace_bytes(int64_t n, int64_t nnz, int32_t s, int32_t zeta, size_t* bytes) {
  if (!bytes || nnz < 0 || !sketch_args_ok(n, s, zeta)) return SFGMRES_ERR_INVALID;
  *bytes = small_layout(n, nnz, s, zeta).total;
  return SFGMRES_OK;
}

int sfgmres_spmv_sketch(sfgmres_handle h, const sfgmres_csr* A, const double* u, double scale,
                        double* w, int32_t s, int32_t zeta, uint64_t seed, const double* U,
                        int64_t ldu, int32_t nwin, double* c, double* dots, double* norm2,
                        void* ws, size_t ws_bytes, void* stream) {
  return sfg::spmv_sketch_impl(h, A, u, scale, w, s, zeta, seed, U, ldu, nwin, c, dots, norm2, ws,
                               ws_bytes, stream);
}

}  // extern "C"
