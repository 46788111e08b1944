// Host side of the MI355X Biot LBM library: validation, conversion to lattice
// units, per-problem workspace layout, boundary-link terms, the batched engine
// (device descriptors, tile lists, the multigrid schedule of Algorithm 4 inside
// the coupled step of Algorithm 5, HIP-graph capture) and the C ABI of
// biotlbm.h.  A single solver is an engine of one problem.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/biotlbm.h"
#include "lbm_engine.h"

using namespace biot;

namespace {

thread_local std::string g_err;

bp_status fail(bp_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(call)                                                                                      \
  do {                                                                                                    \
    hipError_t e_ = (call);                                                                               \
    if (e_ != hipSuccess) return fail(BP_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define BPCHK(call)               \
  do {                            \
    bp_status st_ = (call);       \
    if (st_ != BP_OK) return st_; \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// D2Q8 / D2Q9 velocity sets (Table 1, Fig. 1)
const int CX8[8] = {1, 0, -1, 0, 1, -1, -1, 1};
const int CY8[8] = {0, 1, 0, -1, 1, 1, -1, -1};
const double W8[8] = {1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
const int CX9[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int CY9[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const double W9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

int side_len(int side, int nx, int ny) { return (side == kLeft || side == kRight) ? ny : nx; }

bool enters_through(int side, int cx, int cy) {
  switch (side) {
    case kLeft: return cx > 0;
    case kRight: return cx < 0;
    case kBottom: return cy > 0;
    default: return cy < 0;
  }
}

int default_levels(int nx, int ny) {
  int L = 1;
  while (nx % 2 == 0 && ny % 2 == 0 && nx / 2 >= 2 && ny / 2 >= 2) {
    nx /= 2;
    ny /= 2;
    ++L;
  }
  return L;
}

int pitch_for(int nx) { return (nx + 31) / 32 * 32; }

bp_status validate(const bp_problem* p) {
  if (!p) return fail(BP_ERR_ARG, "null problem");
  if (p->nx < 1 || p->ny < 1) return fail(BP_ERR_ARG, "nx, ny must be >= 1");
  if (!(p->dx > 0) || !(p->dt > 0)) return fail(BP_ERR_ARG, "dx and dt must be > 0");
  if (!(p->c0 > 0)) return fail(BP_ERR_ARG, "c0 must be > 0");
  if (!(p->mu > 0) || !(p->lambda + p->mu > 0)) return fail(BP_ERR_ARG, "need mu > 0 and lambda + mu > 0");
  if (!(p->alpha >= 0 && p->alpha <= 1)) return fail(BP_ERR_ARG, "alpha must lie in [0, 1]");
  if (!(p->r >= 0 && p->r <= 1)) return fail(BP_ERR_ARG, "r must lie in [0, 1]");
  if (!(p->gamma > 0 && p->gamma <= 1)) return fail(BP_ERR_ARG, "gamma must lie in (0, 1]");
  if (p->K < 1) return fail(BP_ERR_ARG, "K must be >= 1");
  if (p->pressure_gradient != 0 && p->pressure_gradient != 1)
    return fail(BP_ERR_ARG, "pressure_gradient must be 0 (first moments) or 1 (central difference)");
  if (p->cycle < BP_CYCLE_V || p->cycle > BP_CYCLE_FMG)
    return fail(BP_ERR_ARG, "cycle must be V (0), W (1), F (2) or full multigrid (3)");
  if (p->fstar_literal != 0 && p->fstar_literal != 1) return fail(BP_ERR_ARG, "fstar_literal must be 0 or 1");
  if (p->coarse_sweeps < 0 || p->coarse_sweeps % 2 != 0)
    return fail(BP_ERR_ARG, "coarse_sweeps must be 0 or an even number >= 2");
  if (p->lag != 0 && p->lag != 1) return fail(BP_ERR_ARG, "lag must be 0 or 1");
  if (p->ne_fixed < 0) return fail(BP_ERR_ARG, "ne_fixed must be >= 0");
  if (p->ne_fixed == 0 && (!(p->ne_tol > 0) || p->ne_max < 1))
    return fail(BP_ERR_ARG, "adaptive mode needs ne_tol > 0 and ne_max >= 1");
  if (p->prec < BP_FP64 || p->prec > BP_FP64_SHIFTED) return fail(BP_ERR_ARG, "unknown precision");
  if (!p->kappa && !(p->kappa_uniform > 0)) return fail(BP_ERR_ARG, "kappa must be > 0");
  for (int s = 0; s < 4; ++s) {
    if (p->side[s].el < 0 || p->side[s].el > 3) return fail(BP_ERR_ARG, "bad elastic side type");
    const int n = side_len(s, p->nx, p->ny);
    const bool per = p->side[s].el == BP_EL_PERIODIC;
    for (int i = 0; i < n; ++i) {
      const int ft = p->side[s].flow_type ? p->side[s].flow_type[i] : p->side[s].flow_uniform;
      if (ft < 0 || ft > 3) return fail(BP_ERR_ARG, "bad flow side type");
      if ((ft == BP_FLOW_PERIODIC) != per) return fail(BP_ERR_ARG, "periodic must be set for both fields of a side");
    }
  }
  if ((p->side[kLeft].el == BP_EL_PERIODIC) != (p->side[kRight].el == BP_EL_PERIODIC) ||
      (p->side[kBottom].el == BP_EL_PERIODIC) != (p->side[kTop].el == BP_EL_PERIODIC))
    return fail(BP_ERR_ARG, "periodic sides must come in opposite pairs");
  const int L = p->levels > 0 ? p->levels : default_levels(p->nx, p->ny);
  if (L > kMaxLevels || p->nx % (1 << (L - 1)) || p->ny % (1 << (L - 1)))
    return fail(BP_ERR_SHAPE, "nx and ny must be divisible by 2^(levels-1) (at most 16 levels)");
  if (p->lag && (L != 1 || p->ne_fixed < 1))
    return fail(BP_ERR_ARG, "the lagged self-force is Algorithm 1: one level and a fixed N_E");
  const int cx = p->nx >> (L - 1), cy = p->ny >> (L - 1);
  const bool perx = p->side[kLeft].el == BP_EL_PERIODIC, pery = p->side[kBottom].el == BP_EL_PERIODIC;
  if ((!perx && cx < 2) || (!pery && cy < 2))
    return fail(BP_ERR_SHAPE, "a non-periodic direction needs >= 2 cells on the coarsest level");
  return BP_OK;
}

// ---------------------------------------------------------------- layout
// shifted storage keeps its references in FP64 above this many finest cells
// (BIOT_REF64_CELLS sets another bound, BIOT_REF64 = 0 / 1 overrides either
// for FP32 populations)
constexpr int64_t kRef64Cells = 4096 * 4096;
struct LevelLay {
  int nx = 0, ny = 0, pitch = 0;
  int64_t plane = 0;
  bool dbl = false;
  size_t oA = 0, oB = 0, oR = 0;  // oR == SIZE_MAX: none
};

// offsets of all device buffers of one problem, relative to its base
struct Layout {
  int L = 1, nx = 0, ny = 0, pitch = 0;
  int64_t plane = 0;
  bool fdbl = true, shift = false, ref64 = true;
  int cycle = BP_CYCLE_V;
  bool full_tail = false;    // the whole problem fits one workgroup (adaptive cycles)
  std::vector<LevelLay> lv;  // 1..L
  size_t off_f[2], off_D[3], off_pout, off_fbody, off_src, off_omf, off_Ft, off_eref, off_eref2, off_pref[2];
  size_t off_eta, off_sig, off_part, off_part2, off_scal, off_ttab, off_addt, off_elbc[4], off_ftype[4], off_flbc[4];
  size_t off_dlag[2] = {SIZE_MAX, SIZE_MAX};
  bool lag = false;
  int ntiles_fine = 0, ntiles_fine2 = 0;
  int tail_depth = 0;  // depth of the coarse tail's top level (0: no tail)
  size_t total = 0;
};

// the coarse tail covers every level from the largest coarse level whose
// populations and collision results fit the tail kernel's LDS down to level 1
int tail_depth_of(const Layout& lo) {
  if (const char* e = std::getenv("BIOT_NO_TAIL"))
    if (std::atoi(e) != 0) return 0;
  for (int l = lo.L - 1; l >= 1; --l) {
    const LevelLay& v = lo.lv[l];
    const int cap = v.dbl ? kTailCellsF64 : kTailCellsF32;
    if (v.nx * v.ny <= cap) return lo.L - l;
  }
  return 0;
}

void make_layout(const bp_problem* p, Layout& lo) {
  lo.L = p->levels > 0 ? p->levels : default_levels(p->nx, p->ny);
  lo.nx = p->nx;
  lo.ny = p->ny;
  lo.pitch = pitch_for(p->nx);
  lo.plane = (int64_t)lo.pitch * p->ny;
  lo.fdbl = (p->prec == BP_FP64 || p->prec == BP_FP64_SHIFTED);
  lo.shift = (p->prec == BP_FP32_SHIFTED || p->prec == BP_FP64_SHIFTED);
  lo.cycle = p->cycle;
  lo.lag = p->lag != 0;
  const size_t fs = lo.fdbl ? 8 : 4;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  lo.lv.assign(lo.L + 1, LevelLay());
  for (int l = lo.L; l >= 1; --l) {
    LevelLay& v = lo.lv[l];
    v.nx = p->nx >> (lo.L - l);
    v.ny = p->ny >> (lo.L - l);
    v.pitch = pitch_for(v.nx);
    v.plane = (int64_t)v.pitch * v.ny;
    // the coarsest level is kept in FP64 in every precision mode
    v.dbl = (l == 1 && lo.L > 1) ? true : lo.fdbl;
    const size_t es = v.dbl ? 8 : 4;
    v.oA = take(8 * v.plane * es);
    v.oB = take(8 * v.plane * es);
    v.oR = (l < lo.L) ? take(8 * v.plane * es) : SIZE_MAX;
  }
  lo.off_f[0] = take(9 * lo.plane * fs);
  lo.off_f[1] = take(9 * lo.plane * fs);
  for (int k = 0; k < 3; ++k) lo.off_D[k] = take(lo.plane * 8);
  lo.off_pout = take(lo.plane * 8);
  lo.off_fbody = take(2 * lo.plane * 8);
  lo.off_src = take(lo.plane * 8);
  lo.off_omf = take(lo.plane * 8);
  lo.off_Ft = take(2 * lo.plane * fs);
  // references of shifted storage: FP64 with FP64 populations and on grids
  // above kRef64Cells cells (an FP32 reference's neighbour differences keep
  // about eps_32 * N relative accuracy), else FP32
  int64_t ref64_cells = kRef64Cells;
  if (const char* e = std::getenv("BIOT_REF64_CELLS")) ref64_cells = std::atoll(e);
  lo.ref64 = lo.fdbl || (int64_t)p->nx * p->ny > ref64_cells;
  if (const char* e = std::getenv("BIOT_REF64")) lo.ref64 = lo.fdbl || std::atoi(e) != 0;
  const size_t rs = lo.ref64 ? 8 : 4;
  lo.off_eref = lo.shift ? take(2 * lo.plane * rs) : SIZE_MAX;
  lo.off_eref2 = lo.shift ? take(2 * lo.plane * rs) : SIZE_MAX;
  for (int k = 0; k < 2; ++k) lo.off_pref[k] = lo.shift ? take(lo.plane * rs) : SIZE_MAX;
  const size_t N = (size_t)p->nx * p->ny;
  lo.off_eta = take(2 * N * 8);
  lo.off_sig = take(3 * N * 8);
  lo.ntiles_fine = sweep_tiles(p->nx, p->ny);
  lo.tail_depth = tail_depth_of(lo);
  lo.off_part = take((size_t)lo.ntiles_fine * 2 * 8);
  // partials of the multi-application sweeps: as many tiles as the largest
  // of the geometries a finest-level launch may take (two or four
  // applications, with or without the restriction, either region)
  lo.ntiles_fine2 = 0;
  for (int A = 2; A <= 5; ++A)
    for (int alt = 0; alt < 2; ++alt)
      lo.ntiles_fine2 = std::max(lo.ntiles_fine2, sweepn_tiles(p->nx, p->ny, lo.fdbl, A, lo.shift, alt && A != 4));
  lo.off_part2 = take((size_t)lo.ntiles_fine2 * 2 * 8);
  lo.off_scal = take(128);
  if (lo.lag)
    for (int k = 0; k < 2; ++k) lo.off_dlag[k] = take(lo.plane * fs);
  // a problem whose finest level fits the tail kernel, with the coarse tail
  // right below it, runs each adaptive cycle after the stopping test in one
  // workgroup (unshifted storage; BIOT_NO_FULL_TAIL=1 switches it off)
  lo.full_tail = !lo.shift && lo.L >= 2 && lo.tail_depth == 1 && lo.L - 1 <= kTailMaxLevel &&
                 (int64_t)p->nx * p->ny <= (lo.fdbl ? kTailCellsF64 : kTailCellsF32) && lo.cycle != BP_CYCLE_FMG;
  if (const char* e = std::getenv("BIOT_NO_FULL_TAIL"))
    if (std::atoi(e) != 0) lo.full_tail = false;
  // gather tables of the coarse tail's levels (8 words per cell, level 1
  // first), and of the finest level for the whole-problem tail
  size_t tcells = 0;
  if (lo.tail_depth > 0)
    for (int l = 1; l <= (lo.full_tail ? lo.L : lo.L - lo.tail_depth); ++l) tcells += (size_t)lo.lv[l].nx * lo.lv[l].ny;
  lo.off_ttab = take(tcells * 8 * sizeof(uint32_t));
  lo.off_addt = lo.full_tail ? take(8 * lo.plane * fs) : SIZE_MAX;
  for (int s = 0; s < 4; ++s) {
    const int n = side_len(s, p->nx, p->ny);
    lo.off_elbc[s] = take((size_t)n * 8 * 8);
    lo.off_ftype[s] = take((size_t)n);
    lo.off_flbc[s] = take((size_t)n * 9 * 8);
  }
  lo.total = off;
}

// bytes of the engine's own area (descriptors and work lists) for a set of
// problems
// entries this problem adds to the engine's tile lists (see engine_upload):
// schedule lists (full and restriction sets), inspection lists and
// two-application lists for every level, its tail entry, the finest level again for the flow step, and the
// finest level's cell blocks (twice: per-cell kernels and initialisation)
size_t tile_entries_for(const Layout& lo) {
  size_t t = 2;  // the tail entry, at its depth and in the list of every problem's tail
  for (int l = 1; l <= lo.L; ++l)
  {
    t += (size_t)sweep_tiles(lo.lv[l].nx, lo.lv[l].ny) * 4;
    const bool sh = lo.shift && l == lo.L;
    for (int A = 2; A <= 5; ++A)  // either region
      t += (size_t)std::max(sweepn_tiles(lo.lv[l].nx, lo.lv[l].ny, lo.lv[l].dbl, A, sh, false),
                            sweepn_tiles(lo.lv[l].nx, lo.lv[l].ny, lo.lv[l].dbl, A, sh, A != 4));
  }
  t += (size_t)sweep_tiles(lo.nx, lo.ny);
  t += (size_t)cell_blocks(lo.nx, lo.ny) * 2;
  return t;
}

size_t engine_bytes(size_t nprobs, size_t tile_entries) {
  return align_up(nprobs * sizeof(ProbD)) + align_up(tile_entries * sizeof(int2)) + 2 * align_up(nprobs * sizeof(int));
}

// ------------------------------------------------------- boundary terms
// value of side data at the midpoint of the link leaving boundary cell i of
// `side` in direction (ox, oy).  Data are given at face centres; a diagonal
// link ends at a corner point of the face, whose value is the mean of the two
// face values beside it; at the end of a side the second value comes from the
// perpendicular side: periodic wrap, the mirror image for a symmetry wall (the
// component normal to the mirror changes sign), otherwise linear extrapolation.
void link_value(const bp_problem* p, int side, int i, int ox, int oy, const double* vals, int ncomp,
                double out[2]) {
  const int n = side_len(side, p->nx, p->ny);
  const bool xwall = (side == kLeft || side == kRight);
  for (int k = 0; k < ncomp; ++k) out[k] = vals ? vals[ncomp * i + k] : 0.0;
  if (ox == 0 || oy == 0) return;
  const int t = i + (xwall ? oy : ox);
  double other[2] = {0.0, 0.0};
  if (t >= 0 && t < n) {
    for (int k = 0; k < ncomp; ++k) other[k] = vals ? vals[ncomp * t + k] : 0.0;
  } else {
    const int perp = xwall ? (t < 0 ? kBottom : kTop) : (t < 0 ? kLeft : kRight);
    int kind;  // 0 periodic, 1 mirror, 2 extrapolate
    if (ncomp == 2) {
      const int e = p->side[perp].el;
      kind = e == BP_EL_PERIODIC ? 0 : (e == BP_EL_SYMMETRY ? 1 : 2);
    } else {
      // flow type of the perpendicular side at the corner cell (that side's
      // arrays are indexed by this cell's coordinate along it)
      const int ci = xwall ? (side == kLeft ? 0 : p->nx - 1) : (side == kBottom ? 0 : p->ny - 1);
      const int ft = p->side[perp].flow_type ? p->side[perp].flow_type[ci] : p->side[perp].flow_uniform;
      kind = ft == BP_FLOW_PERIODIC ? 0 : (ft == BP_FLOW_SYMMETRY ? 1 : 2);
    }
    if (kind == 0) {
      const int tw = ((t % n) + n) % n;
      for (int k = 0; k < ncomp; ++k) other[k] = vals ? vals[ncomp * tw + k] : 0.0;
    } else if (kind == 1) {
      const int mc = xwall ? 1 : 0;
      for (int k = 0; k < ncomp; ++k) other[k] = (ncomp == 2 && k == mc) ? -out[k] : out[k];
    } else {
      const int in = 2 * i - t;
      if (in < 0 || in >= n) return;
      for (int k = 0; k < ncomp; ++k) other[k] = 2.0 * out[k] - (vals ? vals[ncomp * in + k] : 0.0);
    }
  }
  for (int k = 0; k < ncomp; ++k) out[k] = 0.5 * (out[k] + other[k]);
}

void elastic_terms(const bp_problem* p, int side, double h, std::vector<double>& out) {
  const int n = side_len(side, p->nx, p->ny);
  out.assign((size_t)n * 8, 0.0);
  const int type = p->side[side].el;
  if (type != BP_EL_DIRICHLET && type != BP_EL_TRACTION) return;
  const int nxn = side == kLeft ? -1 : (side == kRight ? 1 : 0);
  const int nyn = side == kBottom ? -1 : (side == kTop ? 1 : 0);
  for (int i = 0; i < n; ++i)
    for (int q = 0; q < 8; ++q) {
      if (!enters_through(side, CX8[q], CY8[q])) continue;
      double d[2];
      link_value(p, side, i, -CX8[q], -CY8[q], p->side[side].el_value, 2, d);
      double term;
      if (type == BP_EL_DIRICHLET) {
        // fullway bounce-back data term of eq. BC:elasticity
        term = 6.0 * W8[q] * (CX8[q] * d[0] + CY8[q] * d[1]);
      } else {
        // traction correction of eq. BC:traction, scaled by h (c0-scaled traction)
        const double tx = p->c0 * d[0], ty = p->c0 * d[1];
        const double snn = nxn * tx + nyn * ty;
        const double s12 = nxn != 0 ? nxn * ty : nyn * tx;
        const double vs = (CX8[q] != 0 && CY8[q] != 0) ? -0.5 * CX8[q] * CY8[q] * s12 : -snn;
        term = h * vs;
      }
      out[(size_t)8 * i + q] = term;
    }
}

void flow_terms(const bp_problem* p, int side, std::vector<double>& out, std::vector<int8_t>& types) {
  const int n = side_len(side, p->nx, p->ny);
  out.assign((size_t)n * 9, 0.0);
  types.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    types[i] = (int8_t)(p->side[side].flow_type ? p->side[side].flow_type[i] : p->side[side].flow_uniform);
    if (types[i] != BP_FLOW_DIRICHLET) continue;
    for (int k = 1; k < 9; ++k) {
      if (!enters_through(side, CX9[k], CY9[k])) continue;
      double d[2];
      link_value(p, side, i, -CX9[k], -CY9[k], p->side[side].p_value, 1, d);
      out[(size_t)9 * i + k] = 2.0 * W9[k] * p->c0 * d[0];  // eq. BC:pressure
    }
  }
}

double geq_host(int q, double ex, double ey) { return 3.0 * W8[q] * (CX8[q] * ex + CY8[q] * ey); }

// ------------------------------------------------------------- problems
struct Prob {
  Layout lo;
  char* base = nullptr;
  ProbD d{};  // host copy of the device descriptor
  int nx = 0, ny = 0, L = 1, K = 4;
  double h = 0, dt = 0, c0 = 1;
  int ne_fixed = 3, ne_max = 50;
  double ne_tol = 0;
  bool has_body = false, has_src = false;
  int step = 0;
  int64_t total_cycles = 0;
  int last_ne = 0;
  int prev_ne = 0;  // the count of the step before the last (adaptive prediction)
  double last_ratio = -1.0;
  // adaptive statistics: steps, steps stopped at ne_max above the tolerance,
  // largest and summed end-of-step ratios
  int ad_steps = 0, ad_at_cap = 0;
  double ad_max_ratio = 0.0, ad_sum_ratio = 0.0;
  bp_status status = BP_OK;
  int64_t user_id = -1;
  bool fresh = true;     // initial conditions not yet written
  bool evicted = false;  // diverged: no longer stepped (batch)
};

template <typename T>
bp_status upload_planes(hipStream_t st, void* dst, int nx, int ny, int pitch, int64_t plane, const double* src,
                        int m) {
  std::vector<T> tmp((size_t)m * plane, T(0));
  for (int c = 0; c < m; ++c)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        tmp[(size_t)c * plane + (size_t)y * pitch + x] = src ? T(src[((size_t)c * ny + y) * nx + x]) : T(0);
  HIPCHK(hipMemcpyAsync(dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return BP_OK;
}

template <typename T>
bp_status download_planes(hipStream_t st, const void* srcd, int nx, int ny, int pitch, int64_t plane, double* dst,
                          int m) {
  std::vector<T> tmp((size_t)m * plane);
  HIPCHK(hipMemcpyAsync(tmp.data(), srcd, tmp.size() * sizeof(T), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int c = 0; c < m; ++c)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        dst[((size_t)c * ny + y) * nx + x] = double(tmp[(size_t)c * plane + (size_t)y * pitch + x]);
  return BP_OK;
}

bp_status up(hipStream_t st, bool dbl, void* dst, int nx, int ny, int pitch, int64_t plane, const double* src, int m) {
  return dbl ? upload_planes<double>(st, dst, nx, ny, pitch, plane, src, m)
             : upload_planes<float>(st, dst, nx, ny, pitch, plane, src, m);
}
bp_status down(hipStream_t st, bool dbl, const void* srcd, int nx, int ny, int pitch, int64_t plane, double* dst,
               int m) {
  return dbl ? download_planes<double>(st, srcd, nx, ny, pitch, plane, dst, m)
             : download_planes<float>(st, srcd, nx, ny, pitch, plane, dst, m);
}

bp_status upload_loads(hipStream_t st, Prob& P, const double* body_f, const double* source_s) {
  const int nx = P.nx, ny = P.ny;
  const size_t N = (size_t)nx * ny;
  P.has_body = body_f != nullptr;
  P.has_src = source_s != nullptr;
  std::vector<double> b(2 * N), sv(N);
  if (body_f)
    for (size_t k = 0; k < 2 * N; ++k) b[k] = P.h * P.h * P.c0 * body_f[k];
  if (source_s)
    for (size_t k = 0; k < N; ++k) sv[k] = P.dt * source_s[k];
  BPCHK(upload_planes<double>(st, P.base + P.lo.off_fbody, nx, ny, P.lo.pitch, P.lo.plane, body_f ? b.data() : nullptr, 2));
  BPCHK(upload_planes<double>(st, P.base + P.lo.off_src, nx, ny, P.lo.pitch, P.lo.plane, source_s ? sv.data() : nullptr, 1));
  P.d.fbody = P.has_body ? (const double*)(P.base + P.lo.off_fbody) : nullptr;
  P.d.src = P.has_src ? (const double*)(P.base + P.lo.off_src) : nullptr;
  return BP_OK;
}

// set up one problem inside device memory at `base` (layout lo already made)
bp_status setup_problem(const bp_problem* p, const Layout& lo, char* base, hipStream_t st, Prob& P) {
  P.lo = lo;
  P.base = base;
  P.nx = p->nx;
  P.ny = p->ny;
  P.L = lo.L;
  P.K = p->K;
  P.h = p->dx;
  P.dt = p->dt;
  P.c0 = p->c0;
  P.ne_fixed = p->ne_fixed;
  P.ne_tol = p->ne_tol;
  P.ne_max = p->ne_max;
  ProbD& d = P.d;
  std::memset(&d, 0, sizeof(d));
  d.L = lo.L;
  for (int l = 1; l <= lo.L; ++l) {
    const LevelLay& v = lo.lv[l];
    d.lv[l].gA = base + v.oA;
    d.lv[l].gB = base + v.oB;
    d.lv[l].r = v.oR == SIZE_MAX ? nullptr : (void*)(base + v.oR);
    d.lv[l].nx = v.nx;
    d.lv[l].ny = v.ny;
    d.lv[l].pitch = v.pitch;
    d.lv[l].tiles_x = sweep_tiles_x(v.nx);
    for (int A = 2; A <= 5; ++A) d.lv[l].tiles_xn[A] = sweepn_tiles_x(v.nx, A, false);  // A = 5: set per depth
    d.lv[l].dbl = v.dbl ? 1 : 0;
    d.lv[l].plane = v.plane;
  }
  const double lam = p->c0 * p->lambda, mu = p->c0 * p->mu, lm = lam + mu;
  d.om_s = 2.0 / (3.0 * lm + 1.0);            // Table 2
  d.om_d = 2.0 / (6.0 * mu + 1.0);
  d.b_s = 3.0 * lm / (3.0 * lm + 1.0);        // eq. moments:bared
  d.b_d = 6.0 * mu / (6.0 * mu + 1.0);
  d.beta22 = 1.0 / (12.0 * lm + 4.0);         // eq. moments:collision:22
  d.kD = -d.b_s / (2.0 * lm);                 // eq. LBM:divergence
  // self-dependence constant of eq. MG:selfdependence: the implicit share r of
  // the centred source (eq. source:implicit), or the printed value for every r
  d.cstar = (p->fstar_literal ? 1.0 : p->r) * p->alpha * p->alpha / 2.0;
  d.csweeps = p->coarse_sweeps > 0 ? p->coarse_sweeps : 2 * p->K;
  d.gamma = p->gamma;
  d.alpha = p->alpha;
  d.alpha_h = p->alpha / p->dx;
  d.h = p->dx;
  d.r = p->r;
  d.inv_c0h = 1.0 / (p->c0 * p->dx);
  d.grad_central = p->pressure_gradient;
  for (int k = 0; k < 4; ++k) d.el[k] = p->side[k].el;
  d.f[0] = base + lo.off_f[0];
  d.f[1] = base + lo.off_f[1];
  for (int k = 0; k < 3; ++k) d.D[k] = (double*)(base + lo.off_D[k]);
  d.pout = (double*)(base + lo.off_pout);
  d.Ft = base + lo.off_Ft;
  d.eref = lo.shift ? (void*)(base + lo.off_eref) : nullptr;
  d.eref2 = lo.shift ? (void*)(base + lo.off_eref2) : nullptr;
  d.ref64 = lo.ref64 ? 1 : 0;
  for (int k = 0; k < 2; ++k) d.pref[k] = lo.shift ? (void*)(base + lo.off_pref[k]) : nullptr;
  d.eta = (double*)(base + lo.off_eta);
  d.sig = (double*)(base + lo.off_sig);
  d.partials = (double*)(base + lo.off_part);
  d.partials2 = (double*)(base + lo.off_part2);
  d.ntiles_fine2 = lo.ntiles_fine2;
  d.norm2 = (double*)(base + lo.off_scal);
  d.phase = (int*)(base + lo.off_scal + 32);
  d.flags = (int*)(base + lo.off_scal + 40);
  d.ad = (int*)(base + lo.off_scal + 48);
  d.ad_ratio = (double*)(base + lo.off_scal + 56);  // right after ad: one read for both
  d.gref = (double*)(base + lo.off_scal + 64);
  for (int k = 0; k < 2; ++k) d.dlag[k] = lo.lag ? (void*)(base + lo.off_dlag[k]) : nullptr;
  d.ntiles_fine = lo.ntiles_fine;
  d.ttab = (uint32_t*)(base + lo.off_ttab);
  HIPCHK(launch_fill_zero(base, lo.total, st));
  if (lo.tail_depth > 0) {
    size_t o = 0;
    for (int l = 1; l <= (lo.full_tail ? lo.L : lo.L - lo.tail_depth); ++l) {
      HIPCHK(launch_tail_tables(d.el, lo.lv[l].nx, lo.lv[l].ny, d.ttab + o, st));
      o += (size_t)8 * lo.lv[l].nx * lo.lv[l].ny;
    }
  }

  // permeability -> lattice relaxation rate of the flow LBM (eq. pressure:rate)
  const size_t N = (size_t)p->nx * p->ny;
  auto omega_of = [&](double kap) { return 1.0 / (3.0 * (kap / p->c0) * p->dt / (p->dx * p->dx) + 0.5); };
  if (p->kappa) {
    std::vector<double> om(N);
    for (size_t k = 0; k < N; ++k) {
      if (!(p->kappa[k] > 0)) return fail(BP_ERR_ARG, "kappa must be > 0 everywhere");
      om[k] = omega_of(p->kappa[k]);
    }
    BPCHK(upload_planes<double>(st, base + lo.off_omf, p->nx, p->ny, lo.pitch, lo.plane, om.data(), 1));
    d.omf = (const double*)(base + lo.off_omf);
    d.omf_u = om[0];
  } else {
    d.omf = nullptr;
    d.omf_u = omega_of(p->kappa_uniform);
  }
  std::vector<double> ets[4];
  for (int k = 0; k < 4; ++k) {
    std::vector<double>& et = ets[k];
    std::vector<double> ft;
    std::vector<int8_t> ty;
    elastic_terms(p, k, p->dx, et);
    flow_terms(p, k, ft, ty);
    double* elbc = (double*)(base + lo.off_elbc[k]);
    int8_t* ftype = (int8_t*)(base + lo.off_ftype[k]);
    double* flbc = (double*)(base + lo.off_flbc[k]);
    HIPCHK(hipMemcpyAsync(elbc, et.data(), et.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(flbc, ft.data(), ft.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ftype, ty.data(), ty.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    const bool used = (p->side[k].el == BP_EL_DIRICHLET || p->side[k].el == BP_EL_TRACTION);
    d.elbc[k] = used ? elbc : nullptr;
    d.ftype[k] = ftype;
    d.flbc[k] = flbc;
  }
  d.addt = nullptr;
  if (lo.full_tail) {
    // the finest level's wall terms per cell and population, added to the
    // pulled value by the whole-problem tail: the data of the halfway rule
    // (Dirichlet or traction) that the pull takes, chosen as the sweeps
    // choose it (at a corner the y-wall's rule unless that wall is a
    // symmetry wall; two symmetry walls reflect diagonally, with no data)
    const int nx = p->nx, ny = p->ny;
    const bool perx = p->side[BP_LEFT].el == BP_EL_PERIODIC, pery = p->side[BP_BOTTOM].el == BP_EL_PERIODIC;
    auto data = [&](int side) -> const double* {
      const int el = p->side[side].el;
      return (el == BP_EL_DIRICHLET || el == BP_EL_TRACTION) ? ets[side].data() : nullptr;
    };
    std::vector<double> add((size_t)8 * N, 0.0);
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const bool wl = !perx && x == 0, wr = !perx && x == nx - 1;
        const bool wb = !pery && y == 0, wt = !pery && y == ny - 1;
        for (int q = 0; q < 8; ++q) {
          const int cx = CX8[q], cy = CY8[q];
          const bool ox = (cx > 0 && wl) || (cx < 0 && wr);
          const bool oy = (cy > 0 && wb) || (cy < 0 && wt);
          if (!(ox || oy)) continue;
          const int elx = p->side[cx > 0 ? BP_LEFT : BP_RIGHT].el;
          const int ely = p->side[cy > 0 ? BP_BOTTOM : BP_TOP].el;
          bool usex;
          if (ox && oy) {
            if (elx == BP_EL_SYMMETRY && ely == BP_EL_SYMMETRY) continue;
            usex = ely == BP_EL_SYMMETRY;
          } else if (ox) {
            if (elx == BP_EL_SYMMETRY) continue;
            usex = true;
          } else {
            if (ely == BP_EL_SYMMETRY) continue;
            usex = false;
          }
          const double* bc = data(usex ? (cx > 0 ? BP_LEFT : BP_RIGHT) : (cy > 0 ? BP_BOTTOM : BP_TOP));
          if (bc) add[(size_t)q * N + (size_t)y * nx + x] = bc[8 * (usex ? y : x) + q];
        }
      }
    BPCHK(up(st, lo.fdbl, base + lo.off_addt, nx, ny, lo.pitch, lo.plane, add.data(), 8));
    d.addt = base + lo.off_addt;
  }
  BPCHK(upload_loads(st, P, p->body_f, p->source_s));
  return BP_OK;
}

// ---------------------------------------------------------------- engine
enum OpKind { OP_SWEEP, OP_TAIL, OP_FORCE, OP_REBASE_EL, OP_REBASE_FORCE, OP_AD_RESET, OP_FLOW, OP_FINALIZE, OP_ADVANCE, OP_INIT, OP_EXTRACT };

struct Op {
  OpKind kind;
  int mode = 0;           // sweep mode
  int apps = 1;           // smoothing applications per launch
  int tdbl = 0, cdbl = 0; // sweep storage types (level, coarser level)
  bool shift = false;
  bool ref64 = false;     // shifted storage: a problem of the launch keeps FP64 references
  SweepL sw{};
  CellL cl{};
  ProbL pl{};
  TailL tl{};
  int count = 0;          // tiles / problems
  bool alt = false;       // multi-application launch: the alternative region
  int set = 0;            // sweeps: the tile-list set (engine_upload)
  int group = 0;          // sweeps: the storage group of the tile list
};

// tile-list key of a depth: full set or restriction set, one of three
// storage groups (level FP32 / coarser FP32, FP32 / FP64, FP64 / FP64)
// set 0: full set of the time-step schedule (problems not inside their coarse
// tail at this depth), set 1: its restriction set (problems with a coarser
// level), sets 2 and 3: the same without the tail (inspection operations),
// sets 4..7: set 0 in the tiles of the multi-application sweeps with 2, 4, 3
// and 5 applications (the last two end with the residual and restriction)
constexpr int kSetFused = 4, kSetQuad = 5, kSetFusedR = 6, kSetQuadR = 7;
int set_apps(int set) {
  switch (set) {
    case kSetFused: return 2;
    case kSetQuad: return 4;
    case kSetFusedR: return 3;
    case kSetQuadR: return 5;
    default: return 1;
  }
}
// the restriction joins the last pre-smoothing launch on depths of at most
// this many cells in all: by default on every depth.  Small depths are
// latency-bound, and on large ones the fused launch still saves the separate
// restriction sweep's pass over the populations (the 256-problem batch and
// the 2048^2 strip step about 4% faster than with a separate sweep there)
constexpr int64_t kFuseResCells = int64_t(1) << 40;
// a depth whose launches cover at most this many cells in all takes four
// applications per launch: the launch is bound by the dependent work of one
// block, and its 32 x 32 regions (16 x 16 outputs) put 256 blocks on the 256
// CUs at 256^2 cells; the redundant halo work costs little there
// (BIOT_QUAD_MAX_CELLS overrides the bound)
constexpr int64_t kQuadMaxCells = 256 * 256;
// above this many cells in all, a depth's launch of four applications with
// the restriction takes the 64-column regions: 12 x 12 outputs of the narrow
// region would need about two blocks per CU there
constexpr int64_t kQuadNarrowResCells = 128 * 128;
// a depth of at most this many cells in all takes pairs on tall regions (one
// block per CU); larger ones keep two 8-wave blocks per CU, which hide each
// other's barrier waits (BIOT_TALL_MAX_CELLS overrides the bound)
constexpr int64_t kTallMaxCells = 512 * 512;
struct DepthLists {
  int off[8][3] = {};
  int cnt[8][3] = {};
  bool quad = false;  // four applications per launch
  bool fres = false;  // restriction fused into the last pre-smoothing launch
  bool qwide = false; // its four-application form on 64-column regions
  bool tall = false;  // pairs on tall regions
  int tail_off = 0, tail_cnt = 0;  // problems whose coarse tail starts here
};

struct Engine {
  hipStream_t stream = nullptr;
  bool fdbl = true, shift = false;
  bool ref64 = false;  // shifted storage: some problem keeps FP64 references
  int K = 4, ne = 3, maxL = 1;
  int cycle = BP_CYCLE_V;  // cycle shape of every problem (V for full multigrid's later cycles)
  bool fmg = false;        // the first cycle of a step is a full-multigrid cycle
  bool lag = false;        // Algorithm 1 with the lagged self-force (one problem, one level)
  int csweeps = 0;         // coarsest-level sweeps of every problem on the tile path (0: 2K)
  std::vector<Prob*> probs;
  // engine area (device): descriptors, tile lists, problem ids
  char* area = nullptr;
  size_t area_bytes = 0;
  ProbD* d_probs = nullptr;
  int2* d_tiles = nullptr;
  int* d_pids = nullptr;
  int* d_div = nullptr;   // divergence flags by problem index (k_finalize)
  size_t tiles_cap = 0, probs_cap = 0;
  std::vector<DepthLists> depth;  // per depth
  int fine_off = 0, fine_cnt = 0; // depth-0 full-set tiles of every problem (flow)
  int cell_off = 0, cell_cnt = 0; // finest-level cell blocks
  int init_off = 0, init_cnt = 0; // cell blocks of the problems still to initialise
  std::vector<Op> step_ops;
  std::vector<ProbD> pd_host;  // the descriptors last uploaded (tile counts are patched per schedule)
  hipGraphExec_t graph = nullptr;
  hipGraphExec_t graph4 = nullptr;  // four steps in one graph (one graph boundary instead of four)
  bool graph_valid = false, use_graph = true;
  // adaptive schedule (single-problem engines): its fixed pieces, each an op
  // list and, with a stream, a captured graph (enum AdPiece below)
  std::vector<Op> ad_ops[17];
  bool ad_loop = false;  // AD_HEAD runs every cycle of a step (whole-problem tail)
  hipGraphExec_t ad_graph[17] = {};
  hipEvent_t ad_event = nullptr;  // after the copy of the stop flag (engines that may allocate)
  bool ad_valid = false;
  bool xcd_order = true;
  // V-cycles run the coarse tails of every problem in one launch at the
  // deepest point of the cycle when the tails start at several depths
  bool merge_tails = true;
  int tail_all_off = 0, tail_all_cnt = 0, tail_depths = 0;
  bool fuse = true;  // two-application sweeps in the fixed-cycle schedule
  bool quad = true;  // four-application sweeps on small coarse levels
  // launch-shape bounds (cells a depth covers in all); bp_tuning
  int64_t quad_max_cells = kQuadMaxCells;
  int64_t tall_max_cells = kTallMaxCells;
  int64_t fres_max_cells = kFuseResCells;
  int64_t qnarrow_max_cells = kQuadNarrowResCells;
  bool fuse_res = true;  // restriction fused into pre-smoothing on latency-bound depths
  double* host_pin = nullptr;
  bool own_pin = false;        // host_pin from hipHostMalloc (else host_buf)
  double host_buf[4] = {};     // staging of engines that allocate nothing
};

int tgroup(const Engine& E, const Prob& P, int depth) {
  if (E.fdbl) return 2;
  const int l = P.L - depth;
  if (l == 1 && P.L > 1) return 2;      // FP64 coarsest level
  if (l == 2) return 1;                 // FP32 level with an FP64 coarser level
  return 0;
}

// Workgroups of a launch are dealt to the 8 XCDs round-robin (block i runs on
// XCD i mod 8) and each XCD has its own L2.  Reordering a list segment so that
// XCD k receives a contiguous run of its row-major tiles keeps neighbouring
// tiles, which share halo rows and columns, on one L2.
constexpr int kXcds = 8;
void xcd_order(std::vector<int2>& tiles, size_t off) {
  const size_t n = tiles.size() - off;
  if (n <= (size_t)kXcds) return;
  std::vector<int2> seg(tiles.begin() + off, tiles.end());
  size_t start = 0;
  for (int x = 0; x < kXcds; ++x) {
    const size_t cnt = n / kXcds + ((size_t)x < n % kXcds ? 1 : 0);
    for (size_t k = 0; k < cnt; ++k) tiles[off + k * kXcds + x] = seg[start + k];
    start += cnt;
  }
}

// four applications per launch at depth d (FP64 shifted storage has no LDS
// room for them on the finest level)
bool quad_at(const Engine& E, int d) { return E.depth[d].quad && !(d == 0 && E.fdbl && E.shift); }
// the alternative region for A applications per launch at depth d
bool alt_at(const Engine& E, int d, int A) {
  return (A == 2 || A == 3) ? E.depth[d].tall : (A == 5 && E.depth[d].qwide);
}

// write descriptors and tile lists for the current problem set
bp_status engine_upload(Engine& E) {
  const size_t np = E.probs.size();
  if (np > E.probs_cap) return fail(BP_ERR_WORKSPACE, "too many problems for the engine area");
  std::vector<ProbD> pd(np);
  for (size_t i = 0; i < np; ++i) pd[i] = E.probs[i]->d;
  E.maxL = 1;
  E.ref64 = false;
  for (auto* P : E.probs) {
    E.maxL = std::max(E.maxL, P->L);
    E.ref64 = E.ref64 || (P->lo.shift && P->lo.ref64);
  }
  std::vector<int2> tiles;
  E.depth.assign(E.maxL, DepthLists());
  for (int d = 0; d < E.maxL; ++d) {
    int64_t depth_cells = 0;
    for (size_t i = 0; i < np; ++i) {
      const Prob& P = *E.probs[i];
      const int l = P.L - d, td = P.lo.tail_depth;
      if (l >= 1 && !(td > 0 && d >= td)) depth_cells += (int64_t)P.lo.lv[l].nx * P.lo.lv[l].ny;
    }
    E.depth[d].quad = E.quad && depth_cells <= E.quad_max_cells;
    E.depth[d].fres = E.fuse_res && depth_cells <= E.fres_max_cells;
    E.depth[d].qwide = depth_cells > E.qnarrow_max_cells;
    E.depth[d].tall = depth_cells <= E.tall_max_cells;
    for (size_t i = 0; i < np; ++i) {  // tiles along x of the level at this depth, by its A = 5 width
      const int l = E.probs[i]->L - d;
      if (l >= 1) pd[i].lv[l].tiles_xn[5] = sweepn_tiles_x(E.probs[i]->lo.lv[l].nx, 5, alt_at(E, d, 5));
    }
    for (int set = 0; set < 8; ++set)
      for (int g = 0; g < 3; ++g) {
        E.depth[d].off[set][g] = (int)tiles.size();
        for (size_t i = 0; i < np; ++i) {
          const Prob& P = *E.probs[i];
          const int l = P.L - d;
          const int td = P.lo.tail_depth;
          if (l < 1 || (set < 4 && (set & 1) && l < 2) || tgroup(E, P, d) != g) continue;
          if ((set < 2 || set >= kSetFused) && td > 0 && d >= td) continue;  // inside the problem's coarse tail
          const LevelLay& v = P.lo.lv[l];
          const int A = set_apps(set);
          const int nt = set >= kSetFused ? sweepn_tiles(v.nx, v.ny, v.dbl, A, E.shift && d == 0, alt_at(E, d, A))
                                          : sweep_tiles(v.nx, v.ny);
          for (int t = 0; t < nt; ++t) tiles.push_back(make_int2((int)i, t));
        }
        if (E.xcd_order) xcd_order(tiles, E.depth[d].off[set][g]);
        E.depth[d].cnt[set][g] = (int)tiles.size() - E.depth[d].off[set][g];
      }
    E.depth[d].tail_off = (int)tiles.size();
    for (size_t i = 0; i < np; ++i)
      if (E.probs[i]->lo.tail_depth == d && d > 0) tiles.push_back(make_int2((int)i, 0));
    E.depth[d].tail_cnt = (int)tiles.size() - E.depth[d].tail_off;
  }
  // every problem's tail, with the depth of its top level
  E.tail_all_off = (int)tiles.size();
  for (size_t i = 0; i < np; ++i)
    if (E.probs[i]->lo.tail_depth > 0) tiles.push_back(make_int2((int)i, E.probs[i]->lo.tail_depth));
  E.tail_all_cnt = (int)tiles.size() - E.tail_all_off;
  E.tail_depths = 0;
  for (int d = 1; d < E.maxL; ++d) E.tail_depths += E.depth[d].tail_cnt > 0 ? 1 : 0;
  E.fine_off = (int)tiles.size();
  for (size_t i = 0; i < np; ++i) {
    const Prob& P = *E.probs[i];
    const int nt = sweep_tiles(P.nx, P.ny);
    for (int t = 0; t < nt; ++t) tiles.push_back(make_int2((int)i, t));
  }
  if (E.xcd_order) xcd_order(tiles, E.fine_off);
  E.fine_cnt = (int)tiles.size() - E.fine_off;
  E.cell_off = (int)tiles.size();
  for (size_t i = 0; i < np; ++i) {
    const Prob& P = *E.probs[i];
    const int nb = cell_blocks(P.nx, P.ny);
    for (int b = 0; b < nb; ++b) tiles.push_back(make_int2((int)i, b));
  }
  E.cell_cnt = (int)tiles.size() - E.cell_off;
  E.init_off = (int)tiles.size();
  for (size_t i = 0; i < np; ++i) {
    const Prob& P = *E.probs[i];
    if (!P.fresh) continue;
    const int nb = cell_blocks(P.nx, P.ny);
    for (int b = 0; b < nb; ++b) tiles.push_back(make_int2((int)i, b));
  }
  E.init_cnt = (int)tiles.size() - E.init_off;
  if (tiles.size() > E.tiles_cap) return fail(BP_ERR_WORKSPACE, "tile lists exceed the engine area");
  // norm partials of the finest level come from the launch geometry the
  // schedule uses there
  for (size_t i = 0; i < np; ++i) {
    const Prob& P = *E.probs[i];
    const int A0 = quad_at(E, 0) ? 4 : 2;
    pd[i].ntiles_fine2 = sweepn_tiles(P.nx, P.ny, P.lo.fdbl, A0, E.shift, alt_at(E, 0, A0));
    pd[i].ntiles_test = pd[i].ntiles_fine2;  // both set again by the schedules that use them
  }
  E.pd_host = pd;
  std::vector<int> pids(np);
  for (size_t i = 0; i < np; ++i) pids[i] = (int)i;
  if (np) {
    HIPCHK(hipMemcpyAsync(E.d_probs, pd.data(), np * sizeof(ProbD), hipMemcpyHostToDevice, E.stream));
    HIPCHK(hipMemcpyAsync(E.d_pids, pids.data(), np * sizeof(int), hipMemcpyHostToDevice, E.stream));
  }
  if (!tiles.empty())
    HIPCHK(hipMemcpyAsync(E.d_tiles, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice, E.stream));
  if (E.probs_cap) HIPCHK(launch_fill_zero(E.d_div, align_up(E.probs_cap * sizeof(int)), E.stream));
  HIPCHK(hipStreamSynchronize(E.stream));
  E.graph_valid = false;
  E.ad_valid = false;
  return BP_OK;
}

void add_sweeps(Engine& E, std::vector<Op>& ops, int d, int set, int mode, int in_sel, int out_sel, int prolong,
                int partials) {
  for (int g = 0; g < 3; ++g) {
    const int cnt = E.depth[d].cnt[set][g];
    if (cnt == 0) continue;
    Op o;
    o.kind = OP_SWEEP;
    o.apps = set_apps(set);
    o.alt = alt_at(E, d, o.apps);
    o.mode = mode;
    o.tdbl = g == 2;
    o.cdbl = g >= 1;
    o.shift = E.shift && d == 0;
    o.ref64 = o.shift && E.ref64;
    o.sw.probs = E.d_probs;
    o.sw.tiles = E.d_tiles + E.depth[d].off[set][g];
    o.sw.depth = d;
    o.sw.in_sel = in_sel;
    o.sw.out_sel = out_sel;
    o.sw.prolong = prolong;
    o.sw.partials = partials;
    o.count = cnt;
    o.set = set;
    o.group = g;
    ops.push_back(o);
  }
}

// `count` smoothing applications at depth d, ping-ponging from buffer `sel`:
// with fusion, four (small coarse levels) or two applications run in one
// launch, a single launch takes an odd remainder first.  Only the first launch
// may read a zero input or add the coarse correction, only the last writes the
// norm partials.  restrict_last: the last launch, if it is a multi-application
// one, also restricts the residual of its result (*restricted tells).
// Returns the buffer holding the result.
int add_smoothing(Engine& E, std::vector<Op>& ops, int d, int set, int count, int sel, bool zero_in, bool prolong,
                  bool partials, bool fuse, bool restrict_last = false, bool* restricted = nullptr) {
  bool first = true;
  const bool quad = fuse && quad_at(E, d);
  if (restricted) *restricted = false;
  while (count > 0) {
    const int apps = (quad && count % 4 == 0) ? 4 : ((fuse && count % 2 == 0) ? 2 : 1);
    const int in = (first && zero_in) ? 2 : sel;
    const int pro = (first && prolong) ? 1 : 0;
    count -= apps;
    const int part = (partials && count == 0) ? 1 : 0;
    const bool res = restrict_last && count == 0 && apps > 1;
    const int s = apps == 4 ? (res ? kSetQuadR : kSetQuad) : (apps == 2 ? (res ? kSetFusedR : kSetFused) : set);
    add_sweeps(E, ops, d, s, kSmooth, in, 1 - sel, pro, part);
    if (res && restricted) *restricted = true;
    sel = 1 - sel;
    first = false;
  }
  return sel;
}

// Algorithm 4 at depth d for every problem that has a level there.  The
// iterate of a level starts in buffer A (zero at coarse depths) and ends in A
// after its 2K smoothing applications (the pre- and post-smoothing runs take
// the same number of launches).  tail: problems whose coarse tail starts at
// this depth run it in one launch (time-step schedule); without it every level
// is swept by the tile kernels (inspection operations).  fuse: several
// smoothing applications per launch.
// prolong_first: the first pre-smoothing application adds the coarser
// depth's buffer A (the prolongated correction of full multigrid) to its
// input.  A depth where every problem sits on its coarsest level takes the
// problems' own number of coarsest sweeps (csweeps) in place of 2K, half as
// pre- and half as post-smoothing so that the result ends in A.
void add_fmg_solve(Engine& E, std::vector<Op>& ops, int d1);

// fmg: the coarse-grid correction is computed by full multigrid from zero
// (add_fmg_solve) in place of the V-, W- or F-visit.
void add_vcycle(Engine& E, std::vector<Op>& ops, int d, bool partials_last, bool tail = true, bool fuse = false,
                int cyc = -1, bool from_zero = true, bool prolong_first = false, bool fmg = false) {
  if (d >= E.maxL) return;
  if (cyc < 0) cyc = E.cycle;
  const int full = tail ? 0 : 2, restr = full + 1;
  // the tails of a V-cycle from zero in one launch where the cycle turns
  // (problems are independent, and a problem's levels between its last
  // pre-smoothing and first post-smoothing launch are its tail's alone)
  const bool merged = tail && from_zero && cyc == BP_CYCLE_V && E.merge_tails && E.tail_depths >= 2;
  auto merged_tail = [&]() {
    Op o;
    o.kind = OP_TAIL;
    o.tl.probs = E.d_probs;
    o.tl.pids = (const int*)(E.d_tiles + E.tail_all_off);
    o.tl.depth = -1;  // each entry's own
    o.tl.K = E.K;
    o.tl.shape = BP_CYCLE_V;
    o.tl.from_zero = 1;
    o.count = E.tail_all_cnt;
    ops.push_back(o);
  };
  if (tail && !merged && E.depth[d].tail_cnt > 0) {
    Op o;
    o.kind = OP_TAIL;
    o.tl.probs = E.d_probs;
    o.tl.pids = (const int*)(E.d_tiles + E.depth[d].tail_off);
    o.tl.depth = d;
    o.tl.K = E.K;
    o.tl.shape = cyc;
    o.tl.from_zero = from_zero ? 1 : 0;
    o.count = E.depth[d].tail_cnt;
    ops.push_back(o);
  }
  bool here = false;
  for (int g = 0; g < 3; ++g) here = here || E.depth[d].cnt[full][g] > 0;
  if (!here) {
    if (merged) merged_tail();  // the deepest depth reached holds tails only
    return;
  }
  fuse = fuse && tail;
  bool deeper = false;
  for (int g = 0; g < 3; ++g) deeper = deeper || E.depth[d].cnt[restr][g] > 0;
  const int nsm = (!deeper && d > 0 && E.csweeps > 0) ? E.csweeps / 2 : E.K;  // pre- and post-smoothing steps
  bool restricted = false;
  int sel = add_smoothing(E, ops, d, full, nsm, 0, d > 0 && from_zero, prolong_first, false, fuse,
                          deeper && E.depth[d].fres, &restricted);
  if (deeper) {
    if (!restricted) add_sweeps(E, ops, d, restr, kRestrict, sel, 0, 0, 0);
    // the coarse correction: one V-visit; W: two W-visits, F: an F-visit then
    // a V-visit, the second continuing from the first's iterate (buffer A)
    // with the same restricted right-hand side; or full multigrid
    if (fmg) {
      add_fmg_solve(E, ops, d + 1);
    } else {
      add_vcycle(E, ops, d + 1, false, tail, fuse, cyc, true);
      if (cyc == BP_CYCLE_W) add_vcycle(E, ops, d + 1, false, tail, fuse, BP_CYCLE_W, false);
      if (cyc == BP_CYCLE_F) add_vcycle(E, ops, d + 1, false, tail, fuse, BP_CYCLE_V, false);
    }
  } else if (merged) {
    merged_tail();  // the cycle turns at this depth
  }
  add_smoothing(E, ops, d, full, nsm, sel, false, true, partials_last && d == 0, fuse);
}

// Full multigrid (named as future work in the conclusion) for the coarse
// correction of depths d1 and deeper, from zero, by nested iteration:
// descending, the residual of a zero iterate with the depth's right-hand side
// is restricted to the next depth; ascending from the deepest depth, each
// depth runs one V-cycle from the prolongated correction of the depth below
// (zero input plus prolongation; a problem's coarsest level takes its
// sweeps from zero).  The result ends in buffer A of depth d1, where the
// V-visit would leave it.  Every level runs on the tile kernels.
void add_fmg_solve(Engine& E, std::vector<Op>& ops, int d1) {
  for (int d = d1; d + 1 < E.maxL; ++d) add_sweeps(E, ops, d, 3, kRestrict, 2, 0, 0, 0);
  for (int d = E.maxL - 1; d >= d1; --d) add_vcycle(E, ops, d, false, false, false, BP_CYCLE_V, true, true);
}

// Algorithm 1 with the lag of eq. source:implicit (one problem of one level,
// fixed N_E): the step's 2K N_E applications as single launches, the first
// taking its own divergence, every later one that of its predecessor's input
void add_lagged_cycles(Engine& E, std::vector<Op>& ops) {
  const int napps = 2 * E.K * E.ne;
  int sel = 0;
  for (int a = 0; a < napps; ++a) {
    const size_t first = ops.size();
    add_sweeps(E, ops, 0, 0, kSmooth, sel, 1 - sel, 0, a == napps - 1 ? 1 : 0);
    for (size_t i = first; i < ops.size(); ++i) {
      ops[i].sw.lag = a == 0 ? 1 : 2;
      ops[i].sw.lag_rd = a == 0 ? 0 : (a - 1) % 2;
    }
    sel = 1 - sel;
  }
}

Op cell_op(Engine& E, OpKind k) {
  Op o;
  o.kind = k;
  o.cl.probs = E.d_probs;
  o.cl.tiles = E.d_tiles + E.cell_off;
  o.count = E.cell_cnt;
  return o;
}
Op prob_op(Engine& E, OpKind k) {
  Op o;
  o.kind = k;
  o.pl.probs = E.d_probs;
  o.pl.pids = E.d_pids;
  o.pl.div = E.d_div;
  o.count = (int)E.probs.size();
  return o;
}
Op flow_op(Engine& E) {
  Op o;
  o.kind = OP_FLOW;
  o.cl.probs = E.d_probs;
  o.cl.tiles = E.d_tiles + E.fine_off;
  o.count = E.fine_cnt;
  return o;
}

// one time step.  Shifted storage re-bases at the start of the step and the
// displacement again between V-cycles: the offsets then carry only what one
// cycle changes.  Offsets that carry a whole step's change (early steps move
// the solution by tens of per cent) lose in FP32 the stress moments,
// differences of neighbouring offsets, in proportion to the grid size.
// Between cycles the re-base rides on the cycle's last finest-level launch
// when that is a multi-application smoothing launch: it writes its output
// re-based and the new reference to the other reference buffer, which the next
// cycle reads.  Only an even number of boundaries is taken that way, so the
// step ends on buffer eref; a remaining boundary takes the re-basing kernel.
void build_step_ops(Engine& E, std::vector<Op>& ops) {
  ops.clear();
  // the step-start displacement re-base and the explicit force share a pass
  // over the cells (the previous flow step re-based the pressure)
  ops.push_back(cell_op(E, E.shift ? OP_REBASE_FORCE : OP_FORCE));
  const int fusable = (E.shift && E.fuse && E.K >= 2 && !E.lag) ? 2 * ((E.ne - 1) / 2) : 0;
  int cur = 0;  // reference buffer of the cycle
  if (E.lag) {
    // Algorithm 1 with the lagged self-force: the displacement re-base of
    // shifted storage leaves the divergence unchanged (it has no share in
    // the stress moments), so the step's applications run back to back
    add_lagged_cycles(E, ops);
  }
  for (int j = 0; j < E.ne && !E.lag; ++j) {
    if (E.shift && j > 0 && j > fusable) ops.push_back(cell_op(E, OP_REBASE_EL));
    const size_t first = ops.size();
    add_vcycle(E, ops, 0, j == E.ne - 1, true, E.fuse, -1, true, false, j == 0 && E.fmg);
    for (size_t i = first; i < ops.size(); ++i)
      if (ops[i].kind == OP_SWEEP && ops[i].sw.depth == 0) ops[i].sw.eref_in = cur;
    if (j + 1 <= fusable) {
      // the trailing launches at depth 0 (one per storage group) are the last
      // post-smoothing launch
      size_t i = ops.size();
      while (i > first && ops[i - 1].kind == OP_SWEEP && ops[i - 1].sw.depth == 0 &&
             ops[i - 1].sw.in_sel == ops.back().sw.in_sel && ops[i - 1].apps == ops.back().apps)
        --i;
      // with fusion and K >= 2 the last launch of a smoothing run holds two or
      // four applications (an odd remainder goes first)
      for (size_t k = i; k < ops.size(); ++k) ops[k].sw.rebase_out = 1;
      cur ^= 1;
    }
  }
  ops.push_back(flow_op(E));
  if (E.ne > 0) {
    // the norms of the last post-smoothing launch (the flow step leaves them
    // alone), then the step counter, in one launch
    Op f = prob_op(E, OP_FINALIZE);
    f.pl.fused = (E.fuse && E.K >= 2 && !E.lag) ? 1 : 0;  // the last post-smoothing launch was multi-application
    f.pl.advance = 1;
    ops.push_back(f);
  } else {
    ops.push_back(prob_op(E, OP_ADVANCE));
  }
}

// the multi-application launch of an op: applications per launch, then the
// level (finest or coarse), shifted storage and the region (default or ALT)
template <typename T, typename Tc, int APPS, bool RES, bool ALT>
hipError_t sweepn_launch(const Op& o, hipStream_t s) {
  if (o.sw.depth != 0) return launch_tsweep2<T, Tc, false, false, APPS, RES, ALT>(o.sw, o.count, s);
  return o.shift ? launch_tsweep2<T, Tc, true, true, APPS, RES, ALT>(o.sw, o.count, o.ref64, s)
                 : launch_tsweep2<T, Tc, true, false, APPS, RES, ALT>(o.sw, o.count, s);
}

template <typename T, typename Tc>
hipError_t sweep_launch(const Op& o, hipStream_t s) {
  switch (o.apps) {
    case 5: return o.alt ? sweepn_launch<T, Tc, 4, true, true>(o, s) : sweepn_launch<T, Tc, 4, true, false>(o, s);
    case 4: return sweepn_launch<T, Tc, 4, false, false>(o, s);
    case 3: return o.alt ? sweepn_launch<T, Tc, 2, true, true>(o, s) : sweepn_launch<T, Tc, 2, true, false>(o, s);
    case 2: return o.alt ? sweepn_launch<T, Tc, 2, false, true>(o, s) : sweepn_launch<T, Tc, 2, false, false>(o, s);
    default: break;
  }
  if (o.shift) {
    switch (o.mode) {
      case kSmooth: return launch_tsweep<T, Tc, kSmooth, true>(o.sw, o.count, s);
      case kRestrict: return launch_tsweep<T, Tc, kRestrict, true>(o.sw, o.count, s);
      default: return launch_tsweep<T, Tc, kApply, true>(o.sw, o.count, s);
    }
  }
  switch (o.mode) {
    case kSmooth: return launch_tsweep<T, Tc, kSmooth, false>(o.sw, o.count, s);
    case kRestrict: return launch_tsweep<T, Tc, kRestrict, false>(o.sw, o.count, s);
    default: return launch_tsweep<T, Tc, kApply, false>(o.sw, o.count, s);
  }
}

hipError_t run_op(const Engine& E, const Op& o) {
  hipStream_t s = E.stream;
  switch (o.kind) {
    case OP_SWEEP:
      if (o.tdbl) return sweep_launch<double, double>(o, s);
      if (o.cdbl) return sweep_launch<float, double>(o, s);
      return sweep_launch<float, float>(o, s);
    case OP_FORCE: return E.fdbl ? launch_force<double>(o.cl, o.count, s) : launch_force<float>(o.cl, o.count, s);
    case OP_REBASE_FORCE:
      return E.fdbl ? launch_rebase_force<double>(o.cl, o.count, s) : launch_rebase_force<float>(o.cl, o.count, s);
    case OP_REBASE_EL:
      return E.fdbl ? launch_rebase<double>(o.cl, o.count, s) : launch_rebase<float>(o.cl, o.count, s);
    case OP_INIT: return E.fdbl ? launch_init<double>(o.cl, o.count, s) : launch_init<float>(o.cl, o.count, s);
    case OP_FLOW:
      if (E.fdbl) return E.shift ? launch_tflow<double, true>(o.cl, o.count, s) : launch_tflow<double, false>(o.cl, o.count, s);
      return E.shift ? launch_tflow<float, true>(o.cl, o.count, s) : launch_tflow<float, false>(o.cl, o.count, s);
    case OP_EXTRACT:
      if (E.fdbl) return E.shift ? launch_extract<double, true>(o.cl, o.count, s) : launch_extract<double, false>(o.cl, o.count, s);
      return E.shift ? launch_extract<float, true>(o.cl, o.count, s) : launch_extract<float, false>(o.cl, o.count, s);
    case OP_TAIL: return launch_tail(o.tl, o.count, E.fdbl, s);
    case OP_FINALIZE: return launch_finalize(o.pl, o.count, s);
    case OP_AD_RESET: return launch_ad_reset(o.pl, s);
    case OP_ADVANCE: return launch_advance(o.pl, o.count, s);
  }
  return hipSuccess;
}

// host-side trace ranges (roctx; rocprofv3 --marker-trace records them, and
// without a tool attached they cost a call each)
struct TraceRange {
  explicit TraceRange(const char* m) { roctxRangePushA(m); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

std::string op_name(const Op& o);

// a launch's trace name: the kernel family and the multigrid depth it sweeps
std::string op_trace_name(const Op& o) {
  const int d = o.kind == OP_SWEEP ? o.sw.depth : (o.kind == OP_TAIL ? o.tl.depth : -1);
  return d >= 0 ? op_name(o) + " depth " + std::to_string(d) : op_name(o);
}

bp_status run_ops(const Engine& E, const std::vector<Op>& ops) {
  for (const Op& o : ops) {
    TraceRange r(op_trace_name(o).c_str());
    hipError_t e = run_op(E, o);
    if (e != hipSuccess) return fail(BP_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  }
  return BP_OK;
}

// capture an op list on the engine's stream into an executable graph
bp_status capture_ops(Engine& E, const std::vector<Op>& ops, hipGraphExec_t* out) {
  *out = nullptr;
  HIPCHK(hipStreamBeginCapture(E.stream, hipStreamCaptureModeThreadLocal));
  bp_status st = run_ops(E, ops);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(E.stream, &g);
  if (st != BP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(BP_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(BP_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  return BP_OK;
}

// set one per-problem tile count of the device descriptors (field at byte
// offset `field`) to the tiles of a finest-level launch of `apps`
// applications in the region `alt`, and upload the descriptors
bp_status upload_tile_counts(Engine& E, size_t field, int apps, bool alt) {
  if (E.pd_host.size() != E.probs.size()) return fail(BP_ERR_STATE, "descriptors not uploaded");
  for (size_t i = 0; i < E.probs.size(); ++i) {
    const Prob& P = *E.probs[i];
    const int n = sweepn_tiles(P.nx, P.ny, P.lo.fdbl, apps, E.shift, alt);
    std::memcpy((char*)&E.pd_host[i] + field, &n, sizeof(int));
  }
  if (!E.pd_host.empty()) {
    HIPCHK(hipMemcpyAsync(E.d_probs, E.pd_host.data(), E.pd_host.size() * sizeof(ProbD), hipMemcpyHostToDevice,
                          E.stream));
    HIPCHK(hipStreamSynchronize(E.stream));
  }
  return BP_OK;
}

bp_status build_graph(Engine& E) {
  if (E.graph) {
    (void)hipGraphExecDestroy(E.graph);
    E.graph = nullptr;
  }
  if (E.graph4) {
    (void)hipGraphExecDestroy(E.graph4);
    E.graph4 = nullptr;
  }
  E.graph_valid = false;
  build_step_ops(E, E.step_ops);
  // the step's norms are the partials of the multi-application launch that
  // carries them (the last post-smoothing launch at depth 0): its tiles
  for (const Op& o : E.step_ops)
    if (o.kind == OP_SWEEP && o.sw.depth == 0 && o.sw.partials == 1 && o.apps > 1)
      BPCHK(upload_tile_counts(E, offsetof(ProbD, ntiles_fine2), o.apps, o.alt));
  if (E.use_graph && E.stream) {
    BPCHK(capture_ops(E, E.step_ops, &E.graph));
    std::vector<Op> four;
    for (int k = 0; k < 4; ++k) four.insert(four.end(), E.step_ops.begin(), E.step_ops.end());
    BPCHK(capture_ops(E, four, &E.graph4));
  }
  E.graph_valid = true;
  return BP_OK;
}

// no_alloc: the engine allocates nothing (no pinned staging buffer, no
// captured graphs: kernels are launched directly)
bp_status engine_init(Engine& E, char* area, size_t area_bytes, size_t probs_cap, size_t tiles_cap, hipStream_t st,
                      bool fdbl, bool shift, int K, int ne, int cycle = BP_CYCLE_V, bool no_alloc = false) {
  E.stream = st;
  E.area = area;
  E.area_bytes = area_bytes;
  E.probs_cap = probs_cap;
  E.tiles_cap = tiles_cap;
  E.d_probs = (ProbD*)area;
  E.d_tiles = (int2*)(area + align_up(probs_cap * sizeof(ProbD)));
  E.d_pids = (int*)((char*)E.d_tiles + align_up(tiles_cap * sizeof(int2)));
  E.d_div = (int*)((char*)E.d_pids + align_up(probs_cap * sizeof(int)));
  E.fdbl = fdbl;
  E.shift = shift;
  E.K = K;
  E.ne = ne;
  E.fmg = cycle == BP_CYCLE_FMG;
  E.cycle = E.fmg ? BP_CYCLE_V : cycle;
  if (const char* e = std::getenv("BIOT_NO_GRAPH")) E.use_graph = (std::atoi(e) == 0);
  if (const char* e = std::getenv("BIOT_NO_XCD_ORDER")) E.xcd_order = (std::atoi(e) == 0);
  if (const char* e = std::getenv("BIOT_NO_MERGE_TAIL")) E.merge_tails = (std::atoi(e) == 0);
  if (const char* e = std::getenv("BIOT_NO_FUSE")) E.fuse = (std::atoi(e) == 0);
  if (const char* e = std::getenv("BIOT_NO_QUAD")) E.quad = (std::atoi(e) == 0);
  if (const char* e = std::getenv("BIOT_QUAD_MAX_CELLS")) E.quad_max_cells = std::atoll(e);
  if (const char* e = std::getenv("BIOT_TALL_MAX_CELLS")) E.tall_max_cells = std::atoll(e);
  if (const char* e = std::getenv("BIOT_NO_FUSE_RES")) E.fuse_res = (std::atoi(e) == 0);
  if (no_alloc) {
    E.use_graph = false;
    E.host_pin = E.host_buf;
    return BP_OK;
  }
  if (hipHostMalloc((void**)&E.host_pin, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return fail(BP_ERR_DEVICE, "hipHostMalloc failed");
  E.own_pin = true;
  if (hipEventCreateWithFlags(&E.ad_event, hipEventDisableTiming) != hipSuccess) {
    E.ad_event = nullptr;
    return fail(BP_ERR_DEVICE, "hipEventCreate failed");
  }
  return BP_OK;
}

void engine_release(Engine& E) {
  (void)hipStreamSynchronize(E.stream);  // queued work may still read the pinned staging buffer
  if (E.graph) (void)hipGraphExecDestroy(E.graph);
  E.graph = nullptr;
  if (E.graph4) (void)hipGraphExecDestroy(E.graph4);
  E.graph4 = nullptr;
  for (auto& g : E.ad_graph) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  if (E.host_pin && E.own_pin) (void)hipHostFree(E.host_pin);
  E.host_pin = nullptr;
  E.own_pin = false;
  if (E.ad_event) (void)hipEventDestroy(E.ad_event);
  E.ad_event = nullptr;
}

// time steps of every problem of the engine with a fixed number of V-cycles:
// one step, or four in one graph when `left` (the steps still to take, counted
// down by those enqueued) allows; captured HIP graphs when a stream is given,
// else direct launches
bp_status fixed_step(Engine& E, int* left = nullptr) {
  TraceRange r("coupled step");
  if (!E.graph_valid) BPCHK(build_graph(E));
  int n = 1;
  if (left && *left >= 4 && E.graph4) {
    HIPCHK(hipGraphLaunch(E.graph4, E.stream));
    n = 4;
  } else if (E.graph) {
    HIPCHK(hipGraphLaunch(E.graph, E.stream));
  } else {
    BPCHK(run_ops(E, E.step_ops));
  }
  if (left) *left -= n;
  for (auto* P : E.probs) {
    P->step += n;
    P->last_ne = E.ne;
    P->total_cycles += (int64_t)n * E.ne;
  }
  return BP_OK;
}

// adaptive number of V-cycles (single-problem engines): cycle j+1 (j >= 1)
// starts with the fixed schedule's first finest-level launch, whose first
// application also measures ||g_j - S(g_j)|| and ||g_j||; the stopping test
// follows it, and the cycle is abandoned (that launch's output discarded)
// once the ratio reaches the tolerance or j reaches N_E,max.  The test runs on
// the device (in k_finalize) and sets a stop flag that every later launch of
// the step's cycles checks.  A unit is one test and the rest of its cycle.
// The host predicts the tests a step needs (the fewer of the last two steps'
// counts: a count that alternates between two values near the tolerance is
// then predicted right every other step instead of never).  It enqueues the
// units before the last one whole, then only the last one's test, a copy of
// the flag, and, gated on a normal stop, the step's flow step and the next
// step's start and first cycle (one graph); then it reads the flag.  On the
// predicted stop no launch of an abandoned cycle is enqueued and the device
// runs on while the host reads; a stop earlier than predicted leaves launches
// that return at once; a later one takes the rest of the unit and more units
// (the gated launches returned at once).
enum AdPiece {
  AD_HEAD,    // re-base and force, the first cycle, then the stop flag's reset
  AD_HEAD_G,  // the same, run only after a normal stop of the step before
  AD_TEST,    // re-base, the first finest-level launch (norms) and the test
  AD_REST,    // the rest of the cycle that a test let through
  AD_END,     // flow step and step counter
  AD_END_G,   // the same, run only after a normal stop
  AD_FULL8,   // eight units
  AD_B1,      // AD_B1 + n - 1: n - 1 units and a test (n = 1 .. kAdUnits)
};
constexpr int kAdUnits = 8;  // graph boundaries cost ~8 us each
constexpr int AD_END_HEAD_G = AD_B1 + kAdUnits;  // AD_END_G then AD_HEAD_G in one graph
static_assert(AD_END_HEAD_G + 1 <= 17, "adaptive pieces");

void set_skip(std::vector<Op>& ops, size_t from, const int* flag) {
  for (size_t k = from; k < ops.size(); ++k) {
    Op& o = ops[k];
    o.sw.skip = flag;
    o.cl.skip = flag;
    o.pl.skip = flag;
    o.tl.skip = flag;
  }
}

void set_need(std::vector<Op>& ops, const int* flag) {
  for (Op& o : ops) {
    o.sw.need = flag;
    o.cl.need = flag;
    o.pl.need = flag;
    o.tl.need = flag;
  }
}

bp_status build_adaptive(Engine& E) {
  Prob& P = *E.probs[0];
  for (auto& g : E.ad_graph) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  E.ad_valid = false;
  for (auto& o : E.ad_ops) o.clear();
  std::vector<Op>& head = E.ad_ops[AD_HEAD];
  head.push_back(cell_op(E, E.shift ? OP_REBASE_FORCE : OP_FORCE));  // as in the fixed-cycle step
  // a problem whose finest level fits one workgroup runs each cycle (after
  // the stopping test) as one whole-problem tail launch; the cycle's result
  // ends in buffer A as the tile schedule's does
  const bool full = E.probs.size() == 1 && P.lo.full_tail && E.maxL >= 2 && E.depth[1].tail_cnt == 1;
  auto full_tail = [&](int fine_in, int fine_pre) {
    Op o;
    o.kind = OP_TAIL;
    o.tl.probs = E.d_probs;
    o.tl.pids = (const int*)(E.d_tiles + E.depth[1].tail_off);
    o.tl.depth = 0;
    o.tl.K = E.K;
    o.tl.shape = E.cycle;
    o.tl.from_zero = 0;
    o.tl.full = 1;
    o.tl.fine_in = fine_in;
    o.tl.fine_pre = fine_pre;
    o.count = 1;
    return o;
  };
  E.ad_loop = full;
  if (full) {
    // every cycle of the step, with its stopping test, in one launch
    head.push_back(prob_op(E, OP_AD_RESET));
    Op o = full_tail(0, E.K);
    o.tl.loop = 1;
    o.tl.ne_max = P.ne_max;
    o.tl.tol = P.ne_tol;
    head.push_back(o);
  } else {
    if (E.fmg)
      add_vcycle(E, head, 0, false, true, E.fuse, -1, true, false, true);
    else
      add_vcycle(E, head, 0, false, true, E.fuse);
    head.push_back(prob_op(E, OP_AD_RESET));  // last: a gated head reads the flag it resets
    E.ad_ops[AD_HEAD_G] = head;
    set_need(E.ad_ops[AD_HEAD_G], P.d.ad);
    // a later cycle with the fixed schedule's launches; its first finest-level
    // launch measures ||g - S(g)|| and ||g|| on its first application (the
    // cycle's starting iterate), and the stopping test follows it.  On a stop
    // the rest is skipped and that launch's output buffer (B) is dropped: the
    // accepted iterate is still in A.
    std::vector<Op> u;
    if (E.shift) u.push_back(cell_op(E, OP_REBASE_EL));  // as in the fixed-cycle step
    const size_t c0 = u.size();
    add_vcycle(E, u, 0, false, true, E.fuse);
    size_t i = c0;
    while (i < u.size() && u[i].kind == OP_SWEEP && u[i].sw.depth == 0 && u[i].sw.in_sel == u[c0].sw.in_sel &&
           u[i].sw.out_sel == u[c0].sw.out_sel && u[i].apps == u[c0].apps)
      u[i++].sw.partials = u[c0].apps > 1 ? 2 : 1;  // one launch per storage group
    Op fin = prob_op(E, OP_FINALIZE);  // the norms, then the stopping test
    fin.pl.decide = 1;
    fin.pl.tol = P.ne_tol;
    fin.pl.ne_max = P.ne_max;
    fin.pl.fused = u[c0].apps > 1 ? 2 : 0;
    u.insert(u.begin() + (std::ptrdiff_t)i, fin);
    // the tiles whose partials the test sums: those of that launch
    if (u[c0].apps > 1) BPCHK(upload_tile_counts(E, offsetof(ProbD, ntiles_test), u[c0].apps, u[c0].alt));
    set_skip(u, 0, P.d.ad);
    E.ad_ops[AD_TEST].assign(u.begin(), u.begin() + (std::ptrdiff_t)i + 1);
    E.ad_ops[AD_REST].assign(u.begin() + (std::ptrdiff_t)i + 1, u.end());
    for (int k = 0; k < kAdUnits; ++k) E.ad_ops[AD_FULL8].insert(E.ad_ops[AD_FULL8].end(), u.begin(), u.end());
    for (int n = 1; n <= kAdUnits; ++n) {
      std::vector<Op>& b = E.ad_ops[AD_B1 + n - 1];
      for (int k = 0; k + 1 < n; ++k) b.insert(b.end(), u.begin(), u.end());
      b.insert(b.end(), E.ad_ops[AD_TEST].begin(), E.ad_ops[AD_TEST].end());
    }
  }
  E.ad_ops[AD_END].push_back(flow_op(E));
  E.ad_ops[AD_END].push_back(prob_op(E, OP_ADVANCE));
  if (!full) {
    E.ad_ops[AD_END_G] = E.ad_ops[AD_END];
    set_need(E.ad_ops[AD_END_G], P.d.ad);
    E.ad_ops[AD_END_HEAD_G] = E.ad_ops[AD_END_G];
    E.ad_ops[AD_END_HEAD_G].insert(E.ad_ops[AD_END_HEAD_G].end(), E.ad_ops[AD_HEAD_G].begin(),
                                   E.ad_ops[AD_HEAD_G].end());
  }
  if (E.use_graph && E.stream)
    for (int k = 0; k <= AD_END_HEAD_G; ++k)
      if (!E.ad_ops[k].empty()) BPCHK(capture_ops(E, E.ad_ops[k], &E.ad_graph[k]));
  E.ad_valid = true;
  return BP_OK;
}

bp_status run_adaptive(Engine& E, int k) {
  if (E.ad_graph[k]) {
    HIPCHK(hipGraphLaunch(E.ad_graph[k], E.stream));
    return BP_OK;
  }
  return run_ops(E, E.ad_ops[k]);
}

// copy the stop flag, the cycle count and the last ratio (adjacent on the
// device) to the host
bp_status copy_stop(Engine& E, const Prob& P) {
  HIPCHK(hipMemcpyAsync(E.host_pin, P.d.ad, 2 * sizeof(int) + sizeof(double), hipMemcpyDeviceToHost, E.stream));
  if (E.ad_event) HIPCHK(hipEventRecord(E.ad_event, E.stream));
  return BP_OK;
}

// wait for that copy only (work enqueued after it keeps the device busy)
bp_status wait_stop(Engine& E) {
  if (E.ad_event)
    HIPCHK(hipEventSynchronize(E.ad_event));
  else
    HIPCHK(hipStreamSynchronize(E.stream));
  return BP_OK;
}

// one adaptive step.  head_queued: the step's start and first cycle are
// already enqueued (gated on the step before); next: enqueue the next step's
// the same way (another step of the same bp_step call follows)
bp_status adaptive_step(Engine& E, bool& head_queued, bool next) {
  TraceRange r("coupled step, adaptive cycles");
  Prob& P = *E.probs[0];
  if (!E.ad_valid) {
    BPCHK(build_adaptive(E));
    head_queued = false;
  }
  if (!head_queued) BPCHK(run_adaptive(E, AD_HEAD));
  head_queued = false;
  int* st = (int*)E.host_pin;
  if (E.ad_loop) {  // the whole-problem tail ran every cycle and test
    BPCHK(copy_stop(E, P));
    BPCHK(wait_stop(E));
    if (st[0] == 0) return fail(BP_ERR_STATE, "adaptive cycles did not stop");
    if (st[0] == 2) return fail(BP_ERR_DIVERGED, "non-finite residual norm");
    BPCHK(run_adaptive(E, AD_END));
  } else {
    // a step takes at most N_E,max tests (the last one stops)
    const int cap = std::max(1, P.ne_max);
    int want = P.last_ne > 0 ? P.last_ne : 8;
    if (P.prev_ne > 0) want = std::min(want, P.prev_ne);
    want = std::min(cap, want);
    int issued = 0;
    for (;;) {
      for (; want > kAdUnits; want -= kAdUnits, issued += kAdUnits) BPCHK(run_adaptive(E, AD_FULL8));
      BPCHK(run_adaptive(E, AD_B1 + want - 1));
      issued += want;
      BPCHK(copy_stop(E, P));
      BPCHK(run_adaptive(E, next ? AD_END_HEAD_G : AD_END_G));
      BPCHK(wait_stop(E));
      if (st[0] != 0) break;
      if (issued >= cap) return fail(BP_ERR_STATE, "adaptive cycles did not stop");
      BPCHK(run_adaptive(E, AD_REST));  // the cycle that the last test let through
      want = std::min(4, cap - issued);
    }
    if (st[0] == 2) return fail(BP_ERR_DIVERGED, "non-finite residual norm");
    head_queued = next;
  }
  const int j = st[1];
  P.prev_ne = P.last_ne;
  P.last_ne = j;
  P.last_ratio = E.host_pin[1];
  P.total_cycles += j;
  P.ad_steps += 1;
  if (!(P.last_ratio <= P.ne_tol)) P.ad_at_cap += 1;  // stopped by ne_max
  P.ad_max_ratio = std::max(P.ad_max_ratio, P.last_ratio);
  P.ad_sum_ratio += P.last_ratio;
  P.step += 1;
  return BP_OK;
}

// initial conditions of every problem of the engine
bp_status init_states(Engine& E) {
  std::vector<Op> ops{cell_op(E, OP_INIT)};
  BPCHK(run_ops(E, ops));
  HIPCHK(hipStreamSynchronize(E.stream));
  for (auto* P : E.probs) {
    P->step = 0;
    P->status = BP_OK;
    P->fresh = false;
  }
  return BP_OK;
}

// initial conditions of the problems added since the last upload only (the
// others keep their state)
bp_status init_fresh(Engine& E) {
  if (E.init_cnt == 0) return BP_OK;
  Op o = cell_op(E, OP_INIT);
  o.cl.tiles = E.d_tiles + E.init_off;
  o.count = E.init_cnt;
  std::vector<Op> ops{o};
  BPCHK(run_ops(E, ops));
  for (auto* P : E.probs)
    if (P->fresh) {
      P->step = 0;
      P->status = BP_OK;
      P->fresh = false;
    }
  return BP_OK;
}

// ---------------------------------------------------------------- tuning
void tuning_of(const Engine& E, bp_tuning* t) {
  t->quad_max_cells = E.quad_max_cells;
  t->tall_max_cells = E.tall_max_cells;
  t->fuse_res_max_cells = E.fres_max_cells;
  t->quad_res_narrow_max_cells = E.qnarrow_max_cells;
  t->ms_per_step = 0.0;
}

bp_status apply_tuning(Engine& E, const bp_tuning* t) {
  if (!t) return fail(BP_ERR_ARG, "null tuning");
  if (t->quad_max_cells < 0 || t->tall_max_cells < 0 || t->fuse_res_max_cells < 0 ||
      t->quad_res_narrow_max_cells < 0)
    return fail(BP_ERR_ARG, "tuning bounds must be >= 0");
  HIPCHK(hipStreamSynchronize(E.stream));
  E.quad_max_cells = t->quad_max_cells;
  E.tall_max_cells = t->tall_max_cells;
  E.fres_max_cells = t->fuse_res_max_cells;
  E.qnarrow_max_cells = t->quad_res_narrow_max_cells;
  return engine_upload(E);  // new depth flags and tile lists; the step graph is rebuilt
}

// mean device time of n fixed-cycle steps after one warm-up step (which also
// captures the step graph), by HIP events on the engine's stream
bp_status time_steps(Engine& E, int n, double* ms) {
  BPCHK(fixed_step(E));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(BP_ERR_DEVICE, "hipEventCreate failed");
  }
  bp_status rc = BP_OK;
  if (hipEventRecord(e0, E.stream) != hipSuccess) rc = fail(BP_ERR_DEVICE, "hipEventRecord failed");
  for (int k = 0; k < n && rc == BP_OK; ++k) rc = fixed_step(E);
  float t = 0.f;
  if (rc == BP_OK && (hipEventRecord(e1, E.stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                      hipEventElapsedTime(&t, e0, e1) != hipSuccess))
    rc = fail(BP_ERR_DEVICE, "timing events failed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = double(t) / n;
  return rc;
}

// the median of three timings of n steps (a single timing of a few steps
// varies by about the 2% a candidate must win by)
bp_status time_steps_median(Engine& E, int n, double* ms) {
  double t[3];
  for (double& v : t) BPCHK(time_steps(E, n, &v));
  std::sort(t, t + 3);
  *ms = t[1];
  return BP_OK;
}

// Coordinate descent over the four launch-shape bounds: each bound in turn
// takes the candidate whose steps run fastest (by more than 2% over the best
// so far, medians of three timings), the others held.  Timing advances the problems, so the engine is
// re-initialised at the end: only engines that have not stepped are tuned.
bp_status autotune(Engine& E, int steps, bp_tuning* out) {
  if (E.ne <= 0) return fail(BP_ERR_ARG, "autotuning needs a fixed number of V-cycles");
  for (auto* P : E.probs)
    if (P->step != 0) return fail(BP_ERR_STATE, "autotune runs before the first step");
  if (steps < 1) steps = 1;
  int64_t* knob[4] = {&E.quad_max_cells, &E.tall_max_cells, &E.fres_max_cells, &E.qnarrow_max_cells};
  static const int64_t cand[4][5] = {{0, 64 * 64, 128 * 128, 256 * 256, 512 * 512},
                                     {0, 256 * 256, 512 * 512, 1024 * 1024, 2048 * 2048},
                                     {0, 256 * 256, 512 * 512, 2048 * 2048, int64_t(1) << 40},
                                     {0, 64 * 64, 128 * 128, 256 * 256, 512 * 512}};
  BPCHK(engine_upload(E));
  double best = 0.0;
  BPCHK(time_steps_median(E, steps, &best));
  for (int k = 0; k < 4; ++k) {
    const int64_t keep = *knob[k];
    int64_t bestv = keep;
    for (int c = 0; c < 5; ++c) {
      if (cand[k][c] == keep) continue;
      *knob[k] = cand[k][c];
      BPCHK(engine_upload(E));
      double ms = 0.0;
      BPCHK(time_steps_median(E, steps, &ms));
      if (ms < 0.98 * best) {
        best = ms;
        bestv = cand[k][c];
      }
    }
    *knob[k] = bestv;
  }
  BPCHK(engine_upload(E));
  BPCHK(init_states(E));
  for (auto* P : E.probs) {
    P->total_cycles = 0;
    P->last_ne = 0;
    P->prev_ne = 0;
  }
  if (out) {
    tuning_of(E, out);
    out->ms_per_step = best;
  }
  return BP_OK;
}

bp_status extract_fields(Engine& E) {
  std::vector<Op> ops{cell_op(E, OP_EXTRACT)};
  return run_ops(E, ops);
}

bp_status fields_of(Engine& E, Prob& P, double* eta, double* p, double* sigma, int32_t* step) {
  const size_t N = (size_t)P.nx * P.ny;
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, P.d.flags, sizeof(int), hipMemcpyDeviceToHost, E.stream));
  if (eta) HIPCHK(hipMemcpyAsync(eta, P.d.eta, 2 * N * 8, hipMemcpyDeviceToHost, E.stream));
  if (sigma) HIPCHK(hipMemcpyAsync(sigma, P.d.sig, 3 * N * 8, hipMemcpyDeviceToHost, E.stream));
  HIPCHK(hipStreamSynchronize(E.stream));
  if (p) {
    BPCHK(download_planes<double>(E.stream, P.d.pout, P.nx, P.ny, P.lo.pitch, P.lo.plane, p, 1));
    for (size_t k = 0; k < N; ++k) p[k] /= P.c0;
  }
  if (step) *step = P.step;
  bool finite = true;
  if (eta)
    for (size_t k = 0; k < 2 * N && finite; ++k) finite = std::isfinite(eta[k]);
  if (flag || !finite) {
    P.status = BP_ERR_DIVERGED;
    return fail(BP_ERR_DIVERGED, "the solution is not finite");
  }
  return BP_OK;
}

// Problems whose finalize step flagged divergence since the last upload (one
// small copy and a synchronisation).  Returns them in `out`.
bp_status diverged_probs(Engine& E, std::vector<Prob*>& out) {
  out.clear();
  const size_t np = E.probs.size();
  if (np == 0 || E.ne <= 0) return BP_OK;
  std::vector<int> div(np, 0);
  HIPCHK(hipMemcpyAsync(div.data(), E.d_div, np * sizeof(int), hipMemcpyDeviceToHost, E.stream));
  HIPCHK(hipStreamSynchronize(E.stream));
  for (size_t i = 0; i < np; ++i)
    if (div[i]) out.push_back(E.probs[i]);
  return BP_OK;
}

// steps between divergence checks of batches and servers
constexpr int kDivCheckSteps = 8;

// ---- per-launch profile of a time step (bp_profile_step)
// cells an op covers: the level at its depth of every problem in its tile list
double op_cells(const Engine& E, const Op& o, int depth) {
  double cells = 0.0;
  for (const Prob* P : E.probs) {
    const int l = P->L - depth;
    if (l < 1) continue;
    const int td = P->lo.tail_depth;
    if (o.kind == OP_SWEEP) {
      const int set = o.set;
      if ((set < 4 && (set & 1) && l < 2) || tgroup(E, *P, depth) != o.group) continue;
      if ((set < 2 || set >= kSetFused) && td > 0 && depth >= td) continue;
    }
    cells += (double)P->lo.lv[l].nx * P->lo.lv[l].ny;
  }
  return cells;
}

// algorithmic bytes of one launch: every value an application must read or
// write, once per application (SoA planes; s bytes per population value)
double op_bytes(const Engine& E, const Op& o) {
  const double s = E.fdbl ? 8.0 : 4.0;
  const bool sh = E.shift;
  switch (o.kind) {
    case OP_SWEEP: {
      const int d = o.sw.depth;
      const double cells = op_cells(E, o, d);
      const double ts = o.tdbl ? 8.0 : 4.0, cs = o.cdbl ? 8.0 : 4.0;
      // per application: populations in and out, and the finest level's
      // explicit force and displacement reference, or a coarse level's rhs
      const double extra = d == 0 ? (2.0 + (sh ? 2.0 : 0.0)) * s : 8.0 * ts;
      const double app = 16.0 * ts + extra;
      const bool res = o.apps == 3 || o.apps == 5 || o.mode == kRestrict;
      const int napps = o.mode == kRestrict ? 0 : (o.apps == 3 ? 2 : (o.apps == 5 ? 4 : o.apps));
      double b = cells * napps * app;
      if (res) b += cells * (8.0 * ts + extra + 2.0 * cs);  // the residual's sweep, restricted 4:1
      if (o.sw.prolong && d + 1 < E.maxL) b += cells * 2.0 * cs;
      if (o.sw.rebase_out) b += cells * 2.0 * 2.0 * s;
      return b;
    }
    case OP_TAIL: {
      // the levels of the tail, each application's populations and rhs once
      double b = 0.0;
      for (const Prob* P : E.probs) {
        const int td = o.tl.depth < 0 ? P->lo.tail_depth : o.tl.depth;
        if (td <= 0 || P->lo.tail_depth != td) continue;
        for (int l = 1; l <= P->L - td; ++l) {
          const double n = (double)P->lo.lv[l].nx * P->lo.lv[l].ny, ls = P->lo.lv[l].dbl ? 8.0 : 4.0;
          const int apps = l == 1 ? P->d.csweeps : 2 * E.K + 1;
          b += n * apps * 24.0 * ls;
        }
      }
      return b;
    }
    case OP_FLOW: {
      double b = 0.0;
      for (const Prob* P : E.probs)
        b += (double)P->nx * P->ny * ((18.0 + 8.0 + (sh ? 2.0 : 0.0)) * s + 8.0 * 4.0 + (P->has_src ? 8.0 : 0.0) +
                                      (P->d.omf ? 8.0 : 0.0));
      return b;
    }
    case OP_FORCE:
    case OP_REBASE_EL:
    case OP_REBASE_FORCE: {
      double b = 0.0;
      for (const Prob* P : E.probs) {
        const double n = (double)P->nx * P->ny;
        const double force = (9.0 + 2.0) * s + 16.0 + (P->has_body ? 16.0 : 0.0) + (P->has_src ? 8.0 : 0.0) +
                             (P->d.omf ? 8.0 : 0.0);
        if (o.kind == OP_FORCE) b += n * force;
        if (o.kind == OP_REBASE_EL) b += n * (8.0 + 2.0) * 2.0 * s;
        if (o.kind == OP_REBASE_FORCE) b += n * ((8.0 + 2.0) * 2.0 * s + force);
      }
      return b;
    }
    default: return 0.0;
  }
}

std::string op_name(const Op& o) {
  switch (o.kind) {
    case OP_SWEEP: {
      std::string n;
      switch (o.apps) {
        case 2: n = "pair"; break;
        case 3: n = "pair+restrict"; break;
        case 4: n = "quad"; break;
        case 5: n = "quad+restrict"; break;
        default: n = o.mode == kRestrict ? "restrict" : "sweep"; break;
      }
      if (o.alt) n += " alt";
      if (o.shift) n += " shift";
      n += o.tdbl ? " f64" : " f32";
      return n;
    }
    case OP_TAIL: return o.tl.full ? "tail whole" : (o.tl.shape ? "tail shaped" : "tail");
    case OP_FLOW: return "flow";
    case OP_FORCE: return "force";
    case OP_REBASE_EL: return "rebase displacement";
    case OP_REBASE_FORCE: return "rebase+force";
    case OP_FINALIZE: return "finalize";
    case OP_ADVANCE: return "advance";
    case OP_AD_RESET: return "adaptive reset";
    case OP_INIT: return "initial conditions";
    case OP_EXTRACT: return "extract";
  }
  return "other";
}

// ---- the static workspace of bp_create_static: one array per device, held
// by the process until it ends.  In host code `scratch` names a host-side
// stand-in, never a device address: the device address comes from
// hipGetSymbolAddress, once per device with that device current.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_busy[kMaxDevices] = {};

// the current device's static workspace, reserved for one solver (released
// by bp_destroy); its contents are whatever the last solver left
bp_status scratch_acquire(int* dev_out, void** ptr_out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(BP_ERR_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(BP_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  if (g_scratch_busy[dev]) return fail(BP_ERR_STATE, "the device's static workspace is held by another solver");
  g_scratch_busy[dev] = true;
  *dev_out = dev;
  *ptr_out = g_scratch_ptr[dev];
  return BP_OK;
}

void scratch_release(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  g_scratch_busy[dev] = false;
}

// the time-step ops of an engine, launched one by one with an event before
// each (bp_profile_step, bp_batch_profile_step)
bp_status profile_engine(Engine& E, int32_t steps, bp_kernel_stat* out, int32_t cap, int32_t* n_out) {
  if (steps < 1 || !n_out || (cap > 0 && !out)) return fail(BP_ERR_ARG, "bad arguments");
  if (E.ne < 1) return fail(BP_ERR_ARG, "the profile runs fixed-cycle steps");
  for (const Prob* P : E.probs)
    if (P->status != BP_OK) return fail(BP_ERR_STATE, "a problem is in an error state");
  std::vector<Op> ops;
  build_step_ops(E, ops);
  // one entry per (name, depth), in the order of first appearance
  std::vector<std::string> names;
  std::vector<int> depth_of, slot(ops.size());
  for (size_t i = 0; i < ops.size(); ++i) {
    const std::string nm = op_name(ops[i]);
    const int d = ops[i].kind == OP_SWEEP ? ops[i].sw.depth : (ops[i].kind == OP_TAIL ? ops[i].tl.depth : -1);
    int k = 0;
    while (k < (int)names.size() && !(names[k] == nm && depth_of[k] == d)) ++k;
    if (k == (int)names.size()) {
      names.push_back(nm);
      depth_of.push_back(d);
    }
    slot[i] = k;
  }
  std::vector<double> us(names.size(), 0.0), bytes(names.size(), 0.0);
  std::vector<int> launches(names.size(), 0);
  for (size_t i = 0; i < ops.size(); ++i) {
    bytes[slot[i]] += op_bytes(E, ops[i]);
    launches[slot[i]] += 1;
  }
  std::vector<hipEvent_t> ev(ops.size() + 1, nullptr);
  bp_status rc = BP_OK;
  for (auto& e : ev)
    if (rc == BP_OK && hipEventCreate(&e) != hipSuccess) rc = fail(BP_ERR_DEVICE, "hipEventCreate failed");
  for (int k = 0; k < steps && rc == BP_OK; ++k) {
    for (size_t i = 0; i < ops.size() && rc == BP_OK; ++i) {
      if (hipEventRecord(ev[i], E.stream) != hipSuccess) rc = fail(BP_ERR_DEVICE, "hipEventRecord failed");
      TraceRange tr(op_trace_name(ops[i]).c_str());
      const hipError_t le = run_op(E, ops[i]);
      if (le != hipSuccess) rc = fail(BP_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(le));
    }
    if (rc == BP_OK && (hipEventRecord(ev[ops.size()], E.stream) != hipSuccess ||
                        hipEventSynchronize(ev[ops.size()]) != hipSuccess))
      rc = fail(BP_ERR_DEVICE, "timing events failed");
    for (size_t i = 0; i < ops.size() && rc == BP_OK; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) != hipSuccess) rc = fail(BP_ERR_DEVICE, "event time failed");
      us[slot[i]] += 1000.0 * ms;
    }
    if (rc == BP_OK)
      for (Prob* P : E.probs) {
        P->step += 1;
        P->last_ne = E.ne;
        P->total_cycles += E.ne;
      }
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (rc != BP_OK) return rc;
  *n_out = (int32_t)names.size();
  for (int k = 0; k < (int)names.size() && k < cap; ++k) {
    bp_kernel_stat& o = out[k];
    std::memset(&o, 0, sizeof(o));
    std::strncpy(o.name, names[k].c_str(), sizeof(o.name) - 1);
    o.depth = depth_of[k];
    o.launches = launches[k];
    o.us_per_step = us[k] / steps;
    o.bytes_per_step = bytes[k];
  }
  return BP_OK;
}

}  // namespace

// ===================================================================== solver
struct bp_solver {
  Engine E;
  Prob P;
  char* ws = nullptr;
  int static_dev = -1;  // device whose static workspace the solver holds (bp_create_static)
};

struct bp_batch {
  Engine E;
  std::vector<Prob> P;
};

namespace {

// a request's problem, deep-copied so that the caller's arrays may go away
// after bp_server_submit
struct HostProblem {
  bp_problem p{};
  std::vector<double> kappa, body, src;
  std::vector<int8_t> ftype[4];
  std::vector<double> elv[4], pv[4];

  explicit HostProblem(const bp_problem* q) : p(*q) {
    const size_t N = (size_t)q->nx * q->ny;
    if (q->kappa) {
      kappa.assign(q->kappa, q->kappa + N);
      p.kappa = kappa.data();
    }
    if (q->body_f) {
      body.assign(q->body_f, q->body_f + 2 * N);
      p.body_f = body.data();
    }
    if (q->source_s) {
      src.assign(q->source_s, q->source_s + N);
      p.source_s = src.data();
    }
    for (int k = 0; k < 4; ++k) {
      const size_t n = (size_t)side_len(k, q->nx, q->ny);
      const bp_side& sd = q->side[k];
      if (sd.flow_type) {
        ftype[k].assign(sd.flow_type, sd.flow_type + n);
        p.side[k].flow_type = ftype[k].data();
      }
      if (sd.el_value) {
        elv[k].assign(sd.el_value, sd.el_value + 2 * n);
        p.side[k].el_value = elv[k].data();
      }
      if (sd.p_value) {
        pv[k].assign(sd.p_value, sd.p_value + n);
        p.side[k].p_value = pv[k].data();
      }
    }
  }
  HostProblem(const HostProblem&) = delete;
  HostProblem& operator=(const HostProblem&) = delete;
};

// first-fit allocator over byte offsets of the server's pool; adjacent free
// blocks are merged on release
class Pool {
 public:
  void init(size_t off, size_t size) {
    free_.clear();
    if (size) free_[off] = size;
    total_ = size;
  }
  bool alloc(size_t bytes, size_t& off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      off = it->first;
      const size_t rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t total() const { return total_; }
  size_t free_bytes() const {
    size_t t = 0;
    for (const auto& kv : free_) t += kv.second;
    return t;
  }

 private:
  std::map<size_t, size_t> free_;
  size_t total_ = 0;
};

enum { kReqQueued = 0, kReqRunning = 1, kReqDone = 2, kReqFailed = 3 };

struct SrvReq {
  int64_t ticket = 0;
  std::unique_ptr<HostProblem> hp;
  int nsteps = 0;
  int state = kReqQueued;
  Layout lo;
  size_t tiles = 0;
  Prob P;
  size_t off = 0;
  std::vector<double> eta, p, sigma;
  bp_status status = BP_OK;
  std::string error;
};

}  // namespace

struct bp_server {
  Engine E;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Pool pool;
  int prec = 0, K = 4, ne = 3, max_slots = 0;
  size_t tiles_cap = 0, tiles_used = 0;
  int64_t next_ticket = 1;
  std::deque<SrvReq*> queue;
  std::vector<SrvReq*> active;
  std::map<int64_t, std::unique_ptr<SrvReq>> reqs;
  bool dirty = false;
  int steps_since_check = 0;
};

namespace {

// one application on one level of a single-problem engine: buffer A -> B
bp_status single_apply(bp_solver* s, int level) {
  std::vector<Op> ops;
  add_sweeps(s->E, ops, s->P.L - level, 2, kApply, 0, 1, 0, 0);
  return run_ops(s->E, ops);
}

}  // namespace

extern "C" {

const char* bp_last_error(void) { return g_err.c_str(); }

bp_status bp_workspace_bytes(const bp_problem* p, size_t* device_bytes) {
  BPCHK(validate(p));
  if (!device_bytes) return fail(BP_ERR_ARG, "null output");
  Layout lo;
  make_layout(p, lo);
  *device_bytes = lo.total + engine_bytes(1, tile_entries_for(lo));
  return BP_OK;
}

}  // extern "C"

namespace {
// bp_create on a given workspace; no_alloc: the engine allocates nothing
bp_status create_solver(const bp_problem* p, const Layout& lo, char* w, void* hip_stream, bool no_alloc,
                        bp_solver** out) {
  const size_t te = tile_entries_for(lo);
  const size_t need = lo.total + engine_bytes(1, te);
  bp_solver* s = new bp_solver();
  hipStream_t st = (hipStream_t)hip_stream;
  s->ws = w;
  bp_status rc = engine_init(s->E, w + lo.total, need - lo.total, 1, te, st, lo.fdbl, lo.shift, p->K, p->ne_fixed,
                             p->cycle, no_alloc);
  s->E.csweeps = p->coarse_sweeps;
  s->E.lag = p->lag != 0;
  if (s->E.lag) s->E.fuse = false;  // the lag runs single applications
  if (rc == BP_OK) rc = setup_problem(p, lo, w, st, s->P);
  if (rc == BP_OK) {
    s->E.probs = {&s->P};
    rc = engine_upload(s->E);
  }
  if (rc == BP_OK) rc = init_states(s->E);
  if (rc != BP_OK) {
    engine_release(s->E);
    delete s;
    return rc;
  }
  *out = s;
  return BP_OK;
}
}  // namespace

extern "C" {

bp_status bp_create(const bp_problem* p, void* device_ws, size_t ws_bytes, void* hip_stream, bp_solver** out) {
  if (!out) return fail(BP_ERR_ARG, "null output handle");
  *out = nullptr;
  BPCHK(validate(p));
  Layout lo;
  make_layout(p, lo);
  const size_t need = lo.total + engine_bytes(1, tile_entries_for(lo));
  if (!device_ws || ((uintptr_t)device_ws % kAlign) != 0 || ws_bytes < need)
    return fail(BP_ERR_WORKSPACE, "workspace missing, not 256-byte aligned or smaller than bp_workspace_bytes");
  return create_solver(p, lo, (char*)device_ws, hip_stream, false, out);
}

bp_status bp_create_static(const bp_problem* p, void* hip_stream, bp_solver** out) {
  if (!out) return fail(BP_ERR_ARG, "null output handle");
  *out = nullptr;
  BPCHK(validate(p));
  Layout lo;
  make_layout(p, lo);
  const size_t need = lo.total + engine_bytes(1, tile_entries_for(lo));
  if (need > kScratchBytes)
    return fail(BP_ERR_WORKSPACE, "the problem needs " + std::to_string(need) + " bytes; the static workspace holds " +
                                      std::to_string(kScratchBytes));
  int dev = -1;
  void* ptr = nullptr;
  BPCHK(scratch_acquire(&dev, &ptr));
  const bp_status rc = create_solver(p, lo, (char*)ptr, hip_stream, true, out);
  if (rc != BP_OK) {
    scratch_release(dev);
    return rc;
  }
  (*out)->static_dev = dev;
  return BP_OK;
}

bp_status bp_destroy(bp_solver* s) {
  if (!s) return BP_OK;
  engine_release(s->E);
  if (s->static_dev >= 0) scratch_release(s->static_dev);
  delete s;
  return BP_OK;
}

bp_status bp_step(bp_solver* s, int32_t nsteps) {
  TraceRange trace_range("bp_step");
  if (!s) return fail(BP_ERR_ARG, "null solver");
  if (s->P.status != BP_OK) return fail(BP_ERR_STATE, "solver is in an error state");
  if (nsteps < 0) return fail(BP_ERR_ARG, "nsteps < 0");
  bool head_queued = false;  // adaptive: the next step's start already enqueued
  if (s->P.ne_fixed > 0) {
    int left = nsteps;
    while (left > 0) {
      bp_status st = fixed_step(s->E, &left);
      if (st != BP_OK) {
        s->P.status = st;
        return st;
      }
    }
    return BP_OK;
  }
  for (int k = 0; k < nsteps; ++k) {
    bp_status st = adaptive_step(s->E, head_queued, k + 1 < nsteps);
    if (st != BP_OK) {
      s->P.status = st;
      return st;
    }
  }
  return BP_OK;
}

bp_status bp_set_loads(bp_solver* s, const double* body_f, const double* source_s, int32_t reinit) {
  if (!s) return fail(BP_ERR_ARG, "null solver");
  HIPCHK(hipStreamSynchronize(s->E.stream));
  const bool hb = s->P.has_body, hs = s->P.has_src;
  BPCHK(upload_loads(s->E.stream, s->P, body_f, source_s));
  if (hb != s->P.has_body || hs != s->P.has_src) BPCHK(engine_upload(s->E));
  if (reinit) BPCHK(init_states(s->E));
  return BP_OK;
}

bp_status bp_get_fields(bp_solver* s, double* eta, double* p, double* sigma, int32_t* step) {
  if (!s) return fail(BP_ERR_ARG, "null solver");
  BPCHK(extract_fields(s->E));
  return fields_of(s->E, s->P, eta, p, sigma, step);
}

bp_status bp_get_state(bp_solver* s, double* f, double* g, double* D1, double* D2, int32_t* step) {
  if (!s) return fail(BP_ERR_ARG, "null solver");
  Prob& P = s->P;
  hipStream_t st = s->E.stream;
  const int n = P.step;
  const int nx = P.nx, ny = P.ny;
  const size_t N = (size_t)nx * ny;
  const LevelLay& v = P.lo.lv[P.L];
  HIPCHK(hipStreamSynchronize(st));
  std::vector<double> pr, er;
  if (P.lo.shift) {
    pr.resize(N);
    er.resize(2 * N);
    BPCHK(down(st, P.lo.ref64, P.d.pref[n & 1], nx, ny, P.lo.pitch, P.lo.plane, pr.data(), 1));
    BPCHK(down(st, P.lo.ref64, P.d.eref, nx, ny, P.lo.pitch, P.lo.plane, er.data(), 2));
  }
  if (f) {
    BPCHK(down(st, P.lo.fdbl, P.d.f[n & 1], nx, ny, P.lo.pitch, P.lo.plane, f, 9));
    if (P.lo.shift)
      for (int i = 0; i < 9; ++i)
        for (size_t k = 0; k < N; ++k) f[i * N + k] += W9[i] * pr[k];
  }
  if (g) {
    BPCHK(down(st, v.dbl, P.d.lv[P.L].gA, nx, ny, v.pitch, v.plane, g, 8));
    if (P.lo.shift)
      for (int q = 0; q < 8; ++q)
        for (size_t k = 0; k < N; ++k) g[q * N + k] += geq_host(q, er[k], er[N + k]);
  }
  if (D1) BPCHK(download_planes<double>(st, P.d.D[(n + 2) % 3], nx, ny, P.lo.pitch, P.lo.plane, D1, 1));
  if (D2) BPCHK(download_planes<double>(st, P.d.D[(n + 1) % 3], nx, ny, P.lo.pitch, P.lo.plane, D2, 1));
  if (step) *step = P.step;
  return BP_OK;
}

bp_status bp_set_state(bp_solver* s, const double* f, const double* g, const double* D1, const double* D2,
                       int32_t step) {
  if (!s) return fail(BP_ERR_ARG, "null solver");
  if (step < 0) return fail(BP_ERR_ARG, "step < 0");
  Prob& P = s->P;
  hipStream_t st = s->E.stream;
  const int nx = P.nx, ny = P.ny;
  const LevelLay& v = P.lo.lv[P.L];
  HIPCHK(hipStreamSynchronize(st));
  P.step = step;
  const int n = step;
  int ph[2] = {n, 0};  // phase, flags
  HIPCHK(hipMemcpyAsync(P.d.phase, ph, 2 * sizeof(int), hipMemcpyHostToDevice, st));
  if (P.lo.shift) {
    // shifted storage: split the given populations as the step-start re-base
    // does, in FP64 on the host: the references are the displacement moments
    // of g and the zeroth moment of f (rounded to their storage precision),
    // the stored offsets what remains.  The offsets are small, so storing
    // them in the population precision keeps what FP32 full populations
    // would round away.  A part not given keeps its offsets and reference.
    const size_t N = (size_t)nx * ny;
    auto to_ref = [&](double x) { return P.lo.ref64 ? x : double(float(x)); };
    if (g) {
      std::vector<double> er(2 * N), dg(8 * N);
      for (size_t k = 0; k < N; ++k) {
        const double* u = g + k;
        const double m10 = (u[0] - u[2 * N]) + (u[4 * N] - u[5 * N]) + (u[7 * N] - u[6 * N]);
        const double m01 = (u[N] - u[3 * N]) + (u[4 * N] + u[5 * N]) - (u[6 * N] + u[7 * N]);
        er[k] = to_ref(m10);
        er[N + k] = to_ref(m01);
        for (int q = 0; q < 8; ++q) dg[q * N + k] = g[q * N + k] - geq_host(q, er[k], er[N + k]);
      }
      BPCHK(up(st, P.lo.ref64, P.d.eref, nx, ny, P.lo.pitch, P.lo.plane, er.data(), 2));
      BPCHK(up(st, v.dbl, P.d.lv[P.L].gA, nx, ny, v.pitch, v.plane, dg.data(), 8));
    }
    if (f) {
      std::vector<double> pr(N), df(9 * N);
      for (size_t k = 0; k < N; ++k) {
        double sum = 0.0;
        for (int i = 0; i < 9; ++i) sum += f[i * N + k];
        pr[k] = to_ref(sum);
        for (int i = 0; i < 9; ++i) df[i * N + k] = f[i * N + k] - W9[i] * pr[k];
      }
      BPCHK(up(st, P.lo.ref64, P.d.pref[n & 1], nx, ny, P.lo.pitch, P.lo.plane, pr.data(), 1));
      BPCHK(up(st, P.lo.fdbl, P.d.f[n & 1], nx, ny, P.lo.pitch, P.lo.plane, df.data(), 9));
    }
  } else {
    if (f) BPCHK(up(st, P.lo.fdbl, P.d.f[n & 1], nx, ny, P.lo.pitch, P.lo.plane, f, 9));
    if (g) BPCHK(up(st, v.dbl, P.d.lv[P.L].gA, nx, ny, v.pitch, v.plane, g, 8));
  }
  if (D1) BPCHK(upload_planes<double>(st, P.d.D[(n + 2) % 3], nx, ny, P.lo.pitch, P.lo.plane, D1, 1));
  if (D2) BPCHK(upload_planes<double>(st, P.d.D[(n + 1) % 3], nx, ny, P.lo.pitch, P.lo.plane, D2, 1));
  // the growth test takes its reference from the restored state's steps
  const double zero2[2] = {0.0, 0.0};
  HIPCHK(hipMemcpyAsync(P.d.gref, zero2, sizeof(zero2), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  P.status = BP_OK;
  return BP_OK;
}

bp_status bp_level_shape(const bp_solver* s, int32_t level, int32_t* nx, int32_t* ny) {
  if (!s || level < 1 || level > s->P.L) return fail(BP_ERR_ARG, "bad level");
  *nx = s->P.lo.lv[level].nx;
  *ny = s->P.lo.lv[level].ny;
  return BP_OK;
}

bp_status bp_apply_elastic(bp_solver* s, int32_t level, const double* g, const double* r, const double* Ft,
                           double* out) {
  if (!s || level < 1 || level > s->P.L || !g || !out) return fail(BP_ERR_ARG, "bad arguments");
  Prob& P = s->P;
  hipStream_t st = s->E.stream;
  const bool fine = level == P.L;
  if ((fine && r) || (!fine && Ft)) return fail(BP_ERR_ARG, "r applies to coarse levels, Ft to the finest");
  const LevelLay& v = P.lo.lv[level];
  LevelD& D = P.d.lv[level];
  if (fine && P.lo.shift) HIPCHK(launch_fill_zero(P.d.eref, align_up(2 * P.lo.plane * (P.lo.ref64 ? 8 : 4)), st));
  BPCHK(up(st, v.dbl, D.gA, v.nx, v.ny, v.pitch, v.plane, g, 8));
  if (!fine) BPCHK(up(st, v.dbl, D.r, v.nx, v.ny, v.pitch, v.plane, r, 8));
  if (fine) BPCHK(up(st, P.lo.fdbl, P.d.Ft, v.nx, v.ny, v.pitch, v.plane, Ft, 2));
  BPCHK(single_apply(s, level));
  BPCHK(down(st, v.dbl, D.gB, v.nx, v.ny, v.pitch, v.plane, out, 8));
  return BP_OK;
}

bp_status bp_mg_cycle(bp_solver* s, int32_t level, double* g, const double* r, const double* Ft) {
  if (!s || level < 1 || level > s->P.L || !g) return fail(BP_ERR_ARG, "bad arguments");
  Prob& P = s->P;
  Engine& E = s->E;
  hipStream_t st = E.stream;
  const bool fine = level == P.L;
  if ((fine && r) || (!fine && Ft)) return fail(BP_ERR_ARG, "r applies to coarse levels, Ft to the finest");
  const LevelLay& v = P.lo.lv[level];
  LevelD& D = P.d.lv[level];
  if (fine && P.lo.shift) HIPCHK(launch_fill_zero(P.d.eref, align_up(2 * P.lo.plane * (P.lo.ref64 ? 8 : 4)), st));
  BPCHK(up(st, v.dbl, D.gA, v.nx, v.ny, v.pitch, v.plane, g, 8));
  if (!fine) BPCHK(up(st, v.dbl, D.r, v.nx, v.ny, v.pitch, v.plane, r, 8));
  if (fine) BPCHK(up(st, P.lo.fdbl, P.d.Ft, v.nx, v.ny, v.pitch, v.plane, Ft, 2));
  // a cycle that starts on level `level` from the given iterate
  std::vector<Op> ops;
  const int d = P.L - level;
  // a zero iterate on the coarse tail's top level is what the time-step
  // schedule hands to the tail kernel: run that; any other cycle runs on the
  // tile kernels
  bool zero = !fine;
  for (size_t k = 0; k < (size_t)8 * v.nx * v.ny && zero; ++k) zero = g[k] == 0.0;
  if (E.fmg) {
    add_vcycle(E, ops, d, false, false, false, BP_CYCLE_V, false, false, true);
  } else if (E.lag) {
    // one cycle of Algorithm 1 (2K applications) as a time step starts it
    const int ne = E.ne;
    E.ne = 1;
    add_lagged_cycles(E, ops);
    E.ne = ne;
    for (auto& o : ops) o.sw.partials = 0;
  } else if (zero && d == P.lo.tail_depth) {
    add_vcycle(E, ops, d, false, true);
  } else {
    int sel = 0;
    for (int k = 0; k < E.K; ++k) {
      add_sweeps(E, ops, d, 2, kSmooth, sel, 1 - sel, 0, 0);
      sel = 1 - sel;
    }
    if (level > 1) {
      add_sweeps(E, ops, d, 3, kRestrict, sel, 0, 0, 0);
      add_vcycle(E, ops, d + 1, false, false, false, E.cycle, true);
      if (E.cycle == BP_CYCLE_W) add_vcycle(E, ops, d + 1, false, false, false, BP_CYCLE_W, false);
      if (E.cycle == BP_CYCLE_F) add_vcycle(E, ops, d + 1, false, false, false, BP_CYCLE_V, false);
    }
    for (int k = 0; k < E.K; ++k) {
      add_sweeps(E, ops, d, 2, kSmooth, sel, 1 - sel, k == 0 ? 1 : 0, 0);
      sel = 1 - sel;
    }
    if (level == 1 && P.L > 1 && E.csweeps > 0) {
      // the coarsest level of the hierarchy: its own number of sweeps
      ops.clear();
      sel = 0;
      for (int k = 0; k < E.csweeps; ++k) {
        add_sweeps(E, ops, d, 2, kSmooth, sel, 1 - sel, 0, 0);
        sel = 1 - sel;
      }
    }
  }
  BPCHK(run_ops(E, ops));
  BPCHK(down(st, v.dbl, D.gA, v.nx, v.ny, v.pitch, v.plane, g, 8));
  return BP_OK;
}

bp_status bp_explicit_force(bp_solver* s, double* Ft) {
  if (!s || !Ft) return fail(BP_ERR_ARG, "bad arguments");
  Prob& P = s->P;
  int ph = P.step;
  HIPCHK(hipMemcpyAsync(P.d.phase, &ph, sizeof(int), hipMemcpyHostToDevice, s->E.stream));
  std::vector<Op> ops{cell_op(s->E, OP_FORCE)};
  BPCHK(run_ops(s->E, ops));
  BPCHK(down(s->E.stream, P.lo.fdbl, P.d.Ft, P.nx, P.ny, P.lo.pitch, P.lo.plane, Ft, 2));
  return BP_OK;
}

bp_status bp_stats(const bp_solver* s, bp_run_stats* st) {
  if (!s || !st) return fail(BP_ERR_ARG, "bad arguments");
  st->step = s->P.step;
  st->last_ne = s->P.last_ne;
  st->total_cycles = s->P.total_cycles;
  st->last_ratio = s->P.last_ratio;
  st->levels = s->P.L;
  st->adaptive_steps = s->P.ad_steps;
  st->steps_at_cap = s->P.ad_at_cap;
  st->max_ratio = s->P.ad_steps ? s->P.ad_max_ratio : -1.0;
  st->mean_ratio = s->P.ad_steps ? s->P.ad_sum_ratio / s->P.ad_steps : -1.0;
  int flag = 0;
  if (hipMemcpy(&flag, s->P.d.flags, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(BP_ERR_DEVICE, "stats copy failed");
  st->diverged = flag;
  return BP_OK;
}

bp_status bp_get_tuning(bp_solver* s, bp_tuning* out) {
  if (!s || !out) return fail(BP_ERR_ARG, "null argument");
  tuning_of(s->E, out);
  return BP_OK;
}

bp_status bp_set_tuning(bp_solver* s, const bp_tuning* t) {
  if (!s) return fail(BP_ERR_ARG, "null solver");
  return apply_tuning(s->E, t);
}

bp_status bp_autotune(bp_solver* s, int32_t steps, bp_tuning* out) {
  TraceRange trace_range("autotune");
  if (!s) return fail(BP_ERR_ARG, "null solver");
  if (s->P.status != BP_OK) return fail(BP_ERR_STATE, "solver is in an error state");
  if (s->E.ne <= 0) return fail(BP_ERR_ARG, "autotuning needs a fixed number of V-cycles");
  if (s->P.step != 0) return fail(BP_ERR_STATE, "autotune runs before the first step");
  bp_status rc = autotune(s->E, steps, out);
  if (rc != BP_OK) s->P.status = rc;  // a failure while stepping
  return rc;
}

bp_status bp_time_kernel(bp_solver* s, int32_t which, int32_t iters, double* avg_us, double* bytes) {
  if (!s || iters < 1 || !avg_us) return fail(BP_ERR_ARG, "bad arguments");
  Engine& E = s->E;
  Prob& P = s->P;
  const double es = P.lo.fdbl ? 8.0 : 4.0;
  const double N = (double)P.nx * P.ny;
  const double shift = P.lo.shift ? 1.0 : 0.0;
  std::vector<Op> ops;
  switch (which) {
    case 0: add_sweeps(E, ops, 0, 0, kSmooth, 0, 1, 0, 0); break;
    case 4: add_sweeps(E, ops, 0, quad_at(E, 0) ? kSetQuad : kSetFused, kSmooth, 0, 1, 0, 0); break;
    case 1:
      if (P.L < 2) return fail(BP_ERR_ARG, "no coarser level");
      add_sweeps(E, ops, 0, 1, kRestrict, 0, 0, 0, 0);
      break;
    case 2: ops.push_back(flow_op(E)); break;
    default: ops.push_back(cell_op(E, OP_FORCE)); break;
  }
  std::vector<double> psave;
  if (which == 2) {  // the timed flow launches overwrite the pressure output
    psave.resize((size_t)P.lo.plane);
    HIPCHK(hipMemcpyAsync(psave.data(), P.d.pout, P.lo.plane * 8, hipMemcpyDeviceToHost, E.stream));
    HIPCHK(hipStreamSynchronize(E.stream));
  }
  // the launches are captured into one graph so that the events see device
  // time, not the host's launch rate
  BPCHK(run_ops(E, ops));  // warm-up
  HIPCHK(hipStreamSynchronize(E.stream));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  HIPCHK(hipStreamBeginCapture(E.stream, hipStreamCaptureModeThreadLocal));
  bp_status cap = BP_OK;
  for (int k = 0; k < iters && cap == BP_OK; ++k) cap = run_ops(E, ops);
  hipError_t ce = hipStreamEndCapture(E.stream, &graph);
  if (cap != BP_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return cap;
  }
  HIPCHK(ce);
  hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPCHK(ie);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipGraphLaunch(exec, E.stream));  // warm-up of the graph
  HIPCHK(hipEventRecord(e0, E.stream));
  HIPCHK(hipGraphLaunch(exec, E.stream));
  HIPCHK(hipEventRecord(e1, E.stream));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGraphExecDestroy(exec);
  if (which == 2) {
    HIPCHK(hipMemcpyAsync(P.d.pout, psave.data(), P.lo.plane * 8, hipMemcpyHostToDevice, E.stream));
    HIPCHK(hipStreamSynchronize(E.stream));
  }
  *avg_us = 1000.0 * ms / iters;
  double b;
  switch (which) {
    case 0: b = N * (16.0 + 2.0 + 2.0 * shift) * es; break;
    case 4: b = (quad_at(E, 0) ? 4.0 : 2.0) * N * (16.0 + 2.0 + 2.0 * shift) * es; break;
    case 1: {
      const double ce = P.lo.lv[P.L - 1].dbl ? 8.0 : 4.0;
      b = N * (8.0 + 2.0 + 2.0 * shift) * es + (N / 4.0) * 8.0 * ce;
      break;
    }
    case 2:
      b = N * (18.0 + 8.0 + shift) * es + N * 8.0 * (2.0 + 1.0 + 1.0) + (P.has_src ? N * 8.0 : 0.0) +
          (P.d.omf ? N * 8.0 : 0.0);
      break;
    default:
      b = N * (9.0 + 2.0) * es + N * 8.0 * 2.0 + (P.has_body ? N * 16.0 : 0.0) + (P.has_src ? N * 8.0 : 0.0) +
          (P.d.omf ? N * 8.0 : 0.0);
      break;
  }
  if (bytes) *bytes = b;
  return BP_OK;
}

bp_status bp_profile_step(bp_solver* s, int32_t steps, bp_kernel_stat* out, int32_t cap, int32_t* n_out) {
  if (!s) return fail(BP_ERR_ARG, "null solver");
  return profile_engine(s->E, steps, out, cap, n_out);
}

bp_status bp_batch_profile_step(bp_batch* b, int32_t steps, bp_kernel_stat* out, int32_t cap, int32_t* n_out) {
  if (!b) return fail(BP_ERR_ARG, "null batch");
  return profile_engine(b->E, steps, out, cap, n_out);
}

bp_status bp_device_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (!dst || !src || bytes % 16) return fail(BP_ERR_ARG, "bad copy arguments");
  HIPCHK(launch_copy(dst, src, bytes, (hipStream_t)hip_stream));
  return BP_OK;
}

// ------------------------------------------------------------------ batch
bp_status bp_batch_workspace_bytes(const bp_problem* probs, int32_t n, size_t* device_bytes) {
  if (!probs || n < 1 || !device_bytes) return fail(BP_ERR_ARG, "bad batch arguments");
  size_t total = 0, te = 0;
  for (int i = 0; i < n; ++i) {
    BPCHK(validate(&probs[i]));
    if (probs[i].prec != probs[0].prec || probs[i].K != probs[0].K || probs[i].ne_fixed != probs[0].ne_fixed ||
        probs[i].cycle != probs[0].cycle)
      return fail(BP_ERR_ARG, "a batch needs one precision, one K, one cycle shape and one fixed cycle count");
    if (probs[i].ne_fixed < 1) return fail(BP_ERR_ARG, "batched problems need a fixed V-cycle count");
    if (probs[i].lag) return fail(BP_ERR_ARG, "the lagged self-force runs on single solvers");
    if (probs[i].coarse_sweeps != probs[0].coarse_sweeps)
      return fail(BP_ERR_ARG, "a batch needs one number of coarsest-level sweeps");
    if (probs[i].coarse_sweeps > 0) {
      Layout a, b;
      make_layout(&probs[i], a);
      make_layout(&probs[0], b);
      if (a.L != b.L) return fail(BP_ERR_ARG, "coarsest-level sweeps in a batch need one hierarchy depth");
    }
    Layout lo;
    make_layout(&probs[i], lo);
    total += lo.total;
    te += tile_entries_for(lo);
  }
  *device_bytes = total + engine_bytes((size_t)n, te);
  return BP_OK;
}

bp_status bp_batch_create(const bp_problem* probs, int32_t n, void* device_ws, size_t ws_bytes, void* hip_stream,
                          bp_batch** out) {
  if (!out) return fail(BP_ERR_ARG, "null output handle");
  *out = nullptr;
  size_t need = 0;
  BPCHK(bp_batch_workspace_bytes(probs, n, &need));
  if (!device_ws || ((uintptr_t)device_ws % kAlign) != 0 || ws_bytes < need)
    return fail(BP_ERR_WORKSPACE, "workspace missing, not 256-byte aligned or too small");
  bp_batch* b = new bp_batch();
  hipStream_t st = (hipStream_t)hip_stream;
  char* w = (char*)device_ws;
  b->P.resize(n);
  size_t off = 0, te = 0;
  std::vector<Layout> los(n);
  for (int i = 0; i < n; ++i) {
    make_layout(&probs[i], los[i]);
    te += tile_entries_for(los[i]);
  }
  for (int i = 0; i < n; ++i) off += los[i].total;
  bp_status rc = engine_init(b->E, w + off, need - off, (size_t)n, te, st, los[0].fdbl, los[0].shift, probs[0].K,
                             probs[0].ne_fixed, probs[0].cycle);
  b->E.csweeps = probs[0].coarse_sweeps;
  off = 0;
  for (int i = 0; i < n && rc == BP_OK; ++i) {
    rc = setup_problem(&probs[i], los[i], w + off, st, b->P[i]);
    off += los[i].total;
  }
  if (rc == BP_OK) {
    for (auto& P : b->P) b->E.probs.push_back(&P);
    rc = engine_upload(b->E);
  }
  if (rc == BP_OK) rc = init_states(b->E);
  if (rc != BP_OK) {
    engine_release(b->E);
    delete b;
    return rc;
  }
  *out = b;
  return BP_OK;
}

// Steps every member that has not diverged; every kDivCheckSteps steps and at
// the end a member that diverged leaves the engine's launches (its state and
// fields stay as they are, its fields report BP_ERR_DIVERGED)
bp_status bp_batch_step(bp_batch* b, int32_t nsteps) {
  TraceRange trace_range("batch steps");
  if (!b) return fail(BP_ERR_ARG, "null batch");
  if (nsteps < 0) return fail(BP_ERR_ARG, "nsteps < 0");
  for (int k = 0; k < nsteps; ++k) {
    if (!b->E.probs.empty()) BPCHK(fixed_step(b->E));
    if ((k + 1) % kDivCheckSteps == 0 || k + 1 == nsteps) {
      std::vector<Prob*> bad;
      BPCHK(diverged_probs(b->E, bad));
      if (bad.empty()) continue;
      for (Prob* P : bad) {
        P->status = BP_ERR_DIVERGED;
        P->evicted = true;
      }
      b->E.probs.clear();
      for (auto& P : b->P)
        if (!P.evicted) b->E.probs.push_back(&P);
      BPCHK(engine_upload(b->E));
    }
  }
  return BP_OK;
}

bp_status bp_batch_get_fields(bp_batch* b, int32_t i, double* eta, double* p, double* sigma, int32_t* step) {
  if (!b || i < 0 || i >= (int)b->P.size()) return fail(BP_ERR_ARG, "bad batch index");
  if (b->P[i].evicted) {
    if (step) *step = b->P[i].step;
    return fail(BP_ERR_DIVERGED, "the problem diverged and left the batch");
  }
  if (!b->E.probs.empty()) BPCHK(extract_fields(b->E));
  return fields_of(b->E, b->P[i], eta, p, sigma, step);
}

bp_status bp_batch_get_tuning(bp_batch* b, bp_tuning* out) {
  if (!b || !out) return fail(BP_ERR_ARG, "null argument");
  tuning_of(b->E, out);
  return BP_OK;
}

bp_status bp_batch_set_tuning(bp_batch* b, const bp_tuning* t) {
  if (!b) return fail(BP_ERR_ARG, "null batch");
  return apply_tuning(b->E, t);
}

bp_status bp_batch_autotune(bp_batch* b, int32_t steps, bp_tuning* out) {
  if (!b) return fail(BP_ERR_ARG, "null batch");
  return autotune(b->E, steps, out);
}

bp_status bp_batch_destroy(bp_batch* b) {
  if (!b) return BP_OK;
  engine_release(b->E);
  delete b;
  return BP_OK;
}

// ------------------------------------------------------------------ server
bp_status bp_server_request_bytes(const bp_problem* p, size_t* device_bytes) {
  BPCHK(validate(p));
  if (!device_bytes) return fail(BP_ERR_ARG, "null output");
  Layout lo;
  make_layout(p, lo);
  *device_bytes = lo.total;
  return BP_OK;
}

bp_status bp_server_create(void* device_ws, size_t ws_bytes, void* hip_stream, int32_t prec, int32_t K,
                           int32_t ne_fixed, int32_t max_slots, bp_server** out) {
  if (!out) return fail(BP_ERR_ARG, "null output handle");
  *out = nullptr;
  if (prec < BP_FP64 || prec > BP_FP64_SHIFTED || K < 1 || ne_fixed < 1 || max_slots < 1)
    return fail(BP_ERR_ARG, "bad server parameters");
  if (!device_ws || ((uintptr_t)device_ws % kAlign) != 0) return fail(BP_ERR_WORKSPACE, "workspace missing or misaligned");
  const size_t tiles_cap = std::max<size_t>(65536, ws_bytes / 2048);
  const size_t area = engine_bytes((size_t)max_slots, tiles_cap);
  if (ws_bytes <= area) return fail(BP_ERR_WORKSPACE, "workspace smaller than the server's own area");
  bp_server* s = new bp_server();
  s->ws = (char*)device_ws;
  s->ws_bytes = ws_bytes;
  s->prec = prec;
  s->K = K;
  s->ne = ne_fixed;
  s->max_slots = max_slots;
  s->tiles_cap = tiles_cap;
  const bool fdbl = prec == BP_FP64 || prec == BP_FP64_SHIFTED;
  const bool shift = prec == BP_FP32_SHIFTED || prec == BP_FP64_SHIFTED;
  bp_status rc = engine_init(s->E, s->ws, area, (size_t)max_slots, tiles_cap, (hipStream_t)hip_stream, fdbl, shift,
                             K, ne_fixed);
  if (rc != BP_OK) {
    engine_release(s->E);
    delete s;
    return rc;
  }
  s->pool.init(area, ws_bytes - area);
  *out = s;
  return BP_OK;
}

bp_status bp_server_submit(bp_server* s, const bp_problem* p, int32_t nsteps, int64_t* ticket) {
  if (!s || !p || !ticket || nsteps < 1) return fail(BP_ERR_ARG, "bad request arguments");
  BPCHK(validate(p));
  if (p->prec != s->prec || p->K != s->K || p->ne_fixed != s->ne)
    return fail(BP_ERR_ARG, "a request must use the server's precision, K and fixed V-cycle count");
  if (p->cycle != BP_CYCLE_V) return fail(BP_ERR_ARG, "the server runs V-cycles");
  if (p->coarse_sweeps != 0 || p->lag != 0)
    return fail(BP_ERR_ARG, "the server runs the coarsest level's 2K sweeps and no lag");
  auto r = std::make_unique<SrvReq>();
  make_layout(p, r->lo);
  r->tiles = tile_entries_for(r->lo);
  if (r->lo.total > s->pool.total() || r->tiles > s->tiles_cap)
    return fail(BP_ERR_WORKSPACE, "the request can never fit the server's workspace");
  r->hp = std::make_unique<HostProblem>(p);
  r->nsteps = nsteps;
  r->ticket = s->next_ticket++;
  *ticket = r->ticket;
  s->queue.push_back(r.get());
  s->reqs[r->ticket] = std::move(r);
  return BP_OK;
}

namespace {

void server_retire(bp_server* s, SrvReq* r) {
  s->pool.release(r->off, r->lo.total);
  s->tiles_used -= r->tiles;
  s->active.erase(std::find(s->active.begin(), s->active.end(), r));
  s->dirty = true;
}

// admit queued requests in arrival order while slots, pool memory and tile
// list capacity allow
bp_status server_admit(bp_server* s) {
  while (!s->queue.empty() && (int)s->active.size() < s->max_slots) {
    SrvReq* r = s->queue.front();
    if (s->tiles_used + r->tiles > s->tiles_cap) break;
    size_t off = 0;
    if (!s->pool.alloc(r->lo.total, off)) break;
    s->queue.pop_front();
    r->off = off;
    bp_status rc = setup_problem(&r->hp->p, r->lo, s->ws + off, s->E.stream, r->P);
    if (rc != BP_OK) {
      s->pool.release(off, r->lo.total);
      r->state = kReqFailed;
      r->status = rc;
      r->error = bp_last_error();
      continue;
    }
    r->P.fresh = true;
    r->state = kReqRunning;
    s->tiles_used += r->tiles;
    s->active.push_back(r);
    s->dirty = true;
  }
  return BP_OK;
}

bp_status server_sync_members(bp_server* s) {
  if (!s->dirty) return BP_OK;
  s->E.probs.clear();
  for (SrvReq* r : s->active) s->E.probs.push_back(&r->P);
  BPCHK(engine_upload(s->E));
  BPCHK(init_fresh(s->E));
  s->dirty = false;
  return BP_OK;
}

}  // namespace

bp_status bp_server_advance(bp_server* s, int32_t nsteps, int32_t* n_active, int32_t* n_queued) {
  TraceRange trace_range("server steps");
  if (!s || nsteps < 0) return fail(BP_ERR_ARG, "bad server arguments");
  for (int k = 0; k < nsteps; ++k) {
    BPCHK(server_admit(s));
    BPCHK(server_sync_members(s));
    if (s->active.empty()) break;
    BPCHK(fixed_step(s->E));
    // a request that diverged fails at the next check instead of running on
    if (++s->steps_since_check >= kDivCheckSteps) {
      s->steps_since_check = 0;
      std::vector<Prob*> bad;
      BPCHK(diverged_probs(s->E, bad));
      for (Prob* P : bad)
        for (SrvReq* r : std::vector<SrvReq*>(s->active))
          if (&r->P == P) {
            r->state = kReqFailed;
            r->status = BP_ERR_DIVERGED;
            r->error = "the request's state diverged";
            server_retire(s, r);
          }
    }
    std::vector<SrvReq*> done;
    for (SrvReq* r : s->active)
      if (r->P.step >= r->nsteps) done.push_back(r);
    if (done.empty()) continue;
    BPCHK(extract_fields(s->E));
    for (SrvReq* r : done) {
      const size_t N = (size_t)r->P.nx * r->P.ny;
      r->eta.resize(2 * N);
      r->p.resize(N);
      r->sigma.resize(3 * N);
      bp_status rc = fields_of(s->E, r->P, r->eta.data(), r->p.data(), r->sigma.data(), nullptr);
      r->state = rc == BP_OK ? kReqDone : kReqFailed;
      r->status = rc;
      if (rc != BP_OK) r->error = bp_last_error();
      server_retire(s, r);
    }
  }
  if (n_active) *n_active = (int32_t)s->active.size();
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  return BP_OK;
}

bp_status bp_server_poll(const bp_server* s, int64_t ticket, int32_t* state, int32_t* steps_done) {
  if (!s) return fail(BP_ERR_ARG, "null server");
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(BP_ERR_ARG, "unknown ticket");
  const SrvReq& r = *it->second;
  if (state) *state = r.state;
  if (steps_done) *steps_done = r.state == kReqQueued ? 0 : (r.state == kReqDone ? r.nsteps : r.P.step);
  return BP_OK;
}

bp_status bp_server_result(bp_server* s, int64_t ticket, double* eta, double* p, double* sigma) {
  if (!s) return fail(BP_ERR_ARG, "null server");
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(BP_ERR_ARG, "unknown ticket");
  SrvReq& r = *it->second;
  if (r.state == kReqQueued || r.state == kReqRunning) return fail(BP_ERR_STATE, "the request has not finished");
  if (r.state == kReqFailed) {
    const bp_status st = r.status == BP_OK ? BP_ERR_STATE : r.status;
    const std::string msg = "request failed: " + r.error;
    s->reqs.erase(it);
    return fail(st, msg);
  }
  if (eta) std::memcpy(eta, r.eta.data(), r.eta.size() * sizeof(double));
  if (p) std::memcpy(p, r.p.data(), r.p.size() * sizeof(double));
  if (sigma) std::memcpy(sigma, r.sigma.data(), r.sigma.size() * sizeof(double));
  s->reqs.erase(it);
  return BP_OK;
}

bp_status bp_server_stats(const bp_server* s, size_t* pool_bytes, size_t* free_bytes, int32_t* n_active,
                          int32_t* n_queued) {
  if (!s) return fail(BP_ERR_ARG, "null server");
  if (pool_bytes) *pool_bytes = s->pool.total();
  if (free_bytes) *free_bytes = s->pool.free_bytes();
  if (n_active) *n_active = (int32_t)s->active.size();
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  return BP_OK;
}

bp_status bp_server_destroy(bp_server* s) {
  if (!s) return BP_OK;
  engine_release(s->E);
  delete s;
  return BP_OK;
}

}  // extern "C"
