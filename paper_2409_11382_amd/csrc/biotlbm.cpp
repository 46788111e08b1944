// Host side of the MI355X Biot LBM library: validation, conversion to lattice
// units, workspace layout, boundary terms, the multigrid schedule (Algorithm 4),
// the coupled step (Algorithm 5), HIP-graph capture and the C ABI of biotlbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/biotlbm.h"
#include "lbm_kernels.h"

using namespace biot;

namespace {

thread_local std::string g_err;

bp_status fail(bp_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return fail(BP_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define BPCHK(call)                    \
  do {                                 \
    bp_status st_ = (call);            \
    if (st_ != BP_OK) return st_;      \
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

// does population (cx, cy) enter the domain through `side`?
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

struct LevelBuf {
  int nx = 0, ny = 0, pitch = 0;
  int64_t plane = 0;
  bool dbl = false;     // FP64 storage
  size_t oA = 0, oB = 0, oR = 0;  // offsets (oR = 0 -> none)
  void* gA = nullptr;
  void* gB = nullptr;
  void* r = nullptr;
  int H = 16;
};

// Layout of all device buffers carved out of the caller's workspace.
struct Layout {
  int L = 1, nx = 0, ny = 0, pitch = 0;
  int64_t plane = 0;
  bool fdbl = true, shift = false;
  std::vector<LevelBuf> lv;  // 1..L
  size_t off_f[2], off_D[3], off_pout, off_fbody, off_src, off_omf, off_Ft, off_eref, off_pref;
  size_t off_eta, off_sig, off_part, off_scal, off_elbc[4], off_ftype[4], off_flbc[4];
  int max_waves = 0;
  size_t total = 0;
};

int pitch_for(int nx) { return (nx + 31) / 32 * 32; }

int choose_H(int nx, int ny) {
  if (const char* e = std::getenv("BIOT_SWEEP_H")) {
    int h = std::atoi(e);
    if (h >= 2 && h % 2 == 0) return h;
  }
  const int hs[] = {32, 16, 8, 4};
  for (int h : hs)
    if (sweep_waves(nx, ny, h) >= 2048) return h;
  return 4;
}

bp_status validate(const bp_problem* p) {
  if (!p) return fail(BP_ERR_ARG, "null problem");
  if (p->nx < 1 || p->ny < 1) return fail(BP_ERR_ARG, "nx, ny must be >= 1");
  if (!(p->dx > 0) || !(p->dt > 0)) return fail(BP_ERR_ARG, "dx and dt must be > 0");
  if (!(p->c0 > 0)) return fail(BP_ERR_ARG, "c0 must be > 0");
  if (!(p->mu > 0) || !(p->lambda + p->mu > 0)) return fail(BP_ERR_ARG, "need mu > 0 and lambda + mu > 0");
  if (!(p->alpha >= 0 && p->alpha <= 1)) return fail(BP_ERR_ARG, "alpha must lie in [0, 1]");
  if (!(p->r >= 0 && p->r <= 1)) return fail(BP_ERR_ARG, "r must lie in [0, 1]");
  if (!(p->gamma > 0 && p->gamma < 1)) return fail(BP_ERR_ARG, "gamma must lie in (0, 1)");
  if (p->K < 1) return fail(BP_ERR_ARG, "K must be >= 1");
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
  if (L > 30 || p->nx % (1 << (L - 1)) || p->ny % (1 << (L - 1)))
    return fail(BP_ERR_SHAPE, "nx and ny must be divisible by 2^(levels-1)");
  const int cx = p->nx >> (L - 1), cy = p->ny >> (L - 1);
  const bool perx = p->side[kLeft].el == BP_EL_PERIODIC, pery = p->side[kBottom].el == BP_EL_PERIODIC;
  if ((!perx && cx < 2) || (!pery && cy < 2))
    return fail(BP_ERR_SHAPE, "a non-periodic direction needs >= 2 cells on the coarsest level");
  return BP_OK;
}

void make_layout(const bp_problem* p, Layout& lo) {
  lo.L = p->levels > 0 ? p->levels : default_levels(p->nx, p->ny);
  lo.nx = p->nx;
  lo.ny = p->ny;
  lo.pitch = pitch_for(p->nx);
  lo.plane = (int64_t)lo.pitch * p->ny;
  lo.fdbl = (p->prec == BP_FP64 || p->prec == BP_FP64_SHIFTED);
  lo.shift = (p->prec == BP_FP32_SHIFTED || p->prec == BP_FP64_SHIFTED);
  const size_t fs = lo.fdbl ? 8 : 4;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  lo.lv.assign(lo.L + 1, LevelBuf());
  lo.max_waves = 1;
  for (int l = lo.L; l >= 1; --l) {
    LevelBuf& v = lo.lv[l];
    v.nx = p->nx >> (lo.L - l);
    v.ny = p->ny >> (lo.L - l);
    v.pitch = pitch_for(v.nx);
    v.plane = (int64_t)v.pitch * v.ny;
    // the coarsest level is kept in FP64 in every precision mode
    v.dbl = (l == 1 && lo.L > 1) ? true : lo.fdbl;
    const size_t es = v.dbl ? 8 : 4;
    v.oA = take(8 * v.plane * es);
    v.oB = take(8 * v.plane * es);
    v.oR = (l < lo.L) ? take(8 * v.plane * es) : 0;
    v.H = choose_H(v.nx, v.ny);
    lo.max_waves = std::max(lo.max_waves, sweep_waves(v.nx, v.ny, v.H));
  }
  lo.off_f[0] = take(9 * lo.plane * fs);
  lo.off_f[1] = take(9 * lo.plane * fs);
  for (int k = 0; k < 3; ++k) lo.off_D[k] = take(lo.plane * 8);
  lo.off_pout = take(lo.plane * 8);
  lo.off_fbody = take(2 * lo.plane * 8);
  lo.off_src = take(lo.plane * 8);
  lo.off_omf = take(lo.plane * 8);
  lo.off_Ft = take(2 * lo.plane * fs);
  lo.off_eref = lo.shift ? take(2 * lo.plane * fs) : 0;
  lo.off_pref = lo.shift ? take(lo.plane * fs) : 0;
  const size_t N = (size_t)p->nx * p->ny;
  lo.off_eta = take(2 * N * 8);
  lo.off_sig = take(3 * N * 8);
  lo.off_part = take((size_t)lo.max_waves * 2 * 8);
  lo.off_scal = take(64);
  for (int s = 0; s < 4; ++s) {
    const int n = side_len(s, p->nx, p->ny);
    lo.off_elbc[s] = take((size_t)n * 8 * 8);
    lo.off_ftype[s] = take((size_t)n);
    lo.off_flbc[s] = take((size_t)n * 9 * 8);
  }
  lo.total = off;
}

}  // namespace

// ===================================================================== solver
struct bp_solver {
  Layout lo;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  // problem scalars
  int nx = 0, ny = 0, L = 1, K = 4;
  double h = 0, dt = 0, c0 = 1, alpha = 0, r = 0.5, gamma = 0.75;
  double lam = 0, mu = 0;  // c0-scaled
  double om_s = 0, om_d = 0, b_s = 0, b_d = 0, beta22 = 0, kD = 0, cstar = 0;
  double omf_u = 1.0;
  bool het = false, has_body = false, has_src = false;
  int el[4] = {0, 0, 0, 0};
  int ne_fixed = 3, ne_max = 50;
  double ne_tol = 0;
  // device pointers
  void* f[2] = {nullptr, nullptr};
  double* D[3] = {nullptr, nullptr, nullptr};
  double *pout = nullptr, *fbody = nullptr, *src = nullptr, *omf = nullptr;
  void *Ft = nullptr, *eref = nullptr, *pref = nullptr;
  double *eta = nullptr, *sig = nullptr, *part = nullptr, *scal = nullptr;
  int *phase = nullptr, *flags = nullptr;
  double* elbc[4] = {nullptr, nullptr, nullptr, nullptr};
  bool elbc_used[4] = {false, false, false, false};
  int8_t* ftype[4] = {nullptr, nullptr, nullptr, nullptr};
  double* flbc[4] = {nullptr, nullptr, nullptr, nullptr};
  // host state
  int step = 0;
  int64_t total_cycles = 0;
  int last_ne = 0;
  double last_ratio = -1.0;
  bp_status status = BP_OK;
  hipGraphExec_t graph = nullptr;
  bool graph_valid = false;
  double* host_pin = nullptr;  // pinned 4 doubles
  bool use_graph = true;
};

namespace {

template <typename T> ElConst<T> el_const(const bp_solver* s) {
  ElConst<T> k;
  k.om_s = T(s->om_s);
  k.om_d = T(s->om_d);
  k.beta22 = T(s->beta22);
  k.kD = T(s->kD);
  k.cstar = T(s->cstar);
  k.gamma = T(s->gamma);
  return k;
}

// one sweep on level l; the instantiation follows the level's storage and its
// coarser neighbour's storage
struct SweepReq {
  int l;
  int mode;
  const void* in;
  void* out;
  const void* r;
  const void* Ft;
  const void* e;   // coarse correction (level l-1 storage)
  void* rc;        // coarse rhs (level l-1 storage)
  bool zero_g;
  double* partials;
};

template <typename T, typename Tc, bool SHIFT>
bp_status sweep_t(bp_solver* s, const SweepReq& q) {
  const LevelBuf& v = s->lo.lv[q.l];
  SweepArgs<T, Tc> a{};
  a.g = (const T*)q.in;
  a.out = (T*)q.out;
  a.r = (const T*)q.r;
  a.Ft = (const T*)q.Ft;
  a.e = (const Tc*)q.e;
  a.rc = (Tc*)q.rc;
  a.eref = SHIFT ? (const T*)s->eref : nullptr;
  a.partials = q.partials;
  a.nx = v.nx;
  a.ny = v.ny;
  a.pitch = v.pitch;
  a.plane = v.plane;
  if (q.l > 1) {
    a.cpitch = s->lo.lv[q.l - 1].pitch;
    a.cplane = s->lo.lv[q.l - 1].plane;
  }
  for (int k = 0; k < 4; ++k) {
    a.el[k] = s->el[k];
    a.bc[k] = (q.l == s->L && s->elbc_used[k]) ? s->elbc[k] : nullptr;
  }
  a.k = el_const<T>(s);
  a.H = v.H;
  a.zero_g = q.zero_g ? 1 : 0;
  hipError_t e;
  switch (q.mode) {
    case kSmooth: e = launch_sweep<T, Tc, kSmooth, SHIFT>(a, s->stream); break;
    case kRestrict: e = launch_sweep<T, Tc, kRestrict, SHIFT>(a, s->stream); break;
    default: e = launch_sweep<T, Tc, kApply, SHIFT>(a, s->stream); break;
  }
  if (e != hipSuccess) return fail(BP_ERR_DEVICE, std::string("sweep launch: ") + hipGetErrorString(e));
  return BP_OK;
}

bp_status sweep(bp_solver* s, const SweepReq& q) {
  const LevelBuf& v = s->lo.lv[q.l];
  const bool cdbl = q.l > 1 ? s->lo.lv[q.l - 1].dbl : v.dbl;
  const bool shift = s->lo.shift && q.l == s->L;
  if (v.dbl) {
    return shift ? sweep_t<double, double, true>(s, q) : sweep_t<double, double, false>(s, q);
  }
  if (cdbl) return shift ? sweep_t<float, double, true>(s, q) : sweep_t<float, double, false>(s, q);
  return shift ? sweep_t<float, float, true>(s, q) : sweep_t<float, float, false>(s, q);
}

// ELASTIC_MULTIGRID (Algorithm 4) on level l.  The level's iterate starts in gA
// (or is zero when zero_start) and ends in gA: 2K smoothing writes alternate
// between gA and gB.  When first_done, the first pre-smoothing sweep has
// already been run (its result is in gB).
bp_status vcycle(bp_solver* s, int l, bool zero_start, bool first_done, double* last_partials) {
  LevelBuf& v = s->lo.lv[l];
  const bool fine = (l == s->L);
  const void* Ft = fine ? s->Ft : nullptr;
  const void* r = fine ? nullptr : v.r;
  void* cur = v.gA;
  void* alt = v.gB;
  for (int k = 0; k < s->K; ++k) {
    if (!(k == 0 && first_done)) {
      BPCHK(sweep(s, SweepReq{l, kSmooth, cur, alt, r, Ft, nullptr, nullptr, zero_start && k == 0, nullptr}));
    }
    std::swap(cur, alt);
  }
  const void* e = nullptr;
  if (l > 1) {
    LevelBuf& c = s->lo.lv[l - 1];
    BPCHK(sweep(s, SweepReq{l, kRestrict, cur, nullptr, r, Ft, nullptr, c.r, false, fine ? last_partials : nullptr}));
    BPCHK(vcycle(s, l - 1, true, false, nullptr));
    e = c.gA;
  }
  for (int k = 0; k < s->K; ++k) {
    double* part = (fine && l == 1 && k == s->K - 1) ? last_partials : nullptr;
    BPCHK(sweep(s, SweepReq{l, kSmooth, cur, alt, r, Ft, k == 0 ? e : nullptr, nullptr, false, part}));
    std::swap(cur, alt);
  }
  return BP_OK;
}

template <typename T> bp_status launch_force_t(bp_solver* s) {
  ForceArgs<T> a{};
  a.fbuf[0] = (T*)s->f[0];
  a.fbuf[1] = (T*)s->f[1];
  for (int k = 0; k < 3; ++k) a.Dbuf[k] = s->D[k];
  a.phase = s->phase;
  a.fbody = s->has_body ? s->fbody : nullptr;
  a.src = s->has_src ? s->src : nullptr;
  a.omf = s->het ? s->omf : nullptr;
  a.omf_u = s->omf_u;
  a.alpha = s->alpha;
  a.alpha_h = s->alpha / s->h;
  a.h = s->h;
  a.r = s->r;
  a.Ft = (T*)s->Ft;
  a.nx = s->nx;
  a.ny = s->ny;
  a.pitch = s->lo.pitch;
  a.plane = s->lo.plane;
  a.perx = s->el[kLeft] == kElPeriodic;
  a.pery = s->el[kBottom] == kElPeriodic;
  HIPCHK(launch_force<T>(a, s->stream));
  return BP_OK;
}

bp_status run_force(bp_solver* s) { return s->lo.fdbl ? launch_force_t<double>(s) : launch_force_t<float>(s); }

template <typename T, bool SHIFT> bp_status launch_flow_t(bp_solver* s) {
  FlowArgs<T> a{};
  a.fbuf[0] = (T*)s->f[0];
  a.fbuf[1] = (T*)s->f[1];
  a.g = (const T*)s->lo.lv[s->L].gA;
  for (int k = 0; k < 3; ++k) a.Dbuf[k] = s->D[k];
  a.phase = s->phase;
  a.p_out = s->pout;
  a.src = s->has_src ? s->src : nullptr;
  a.omf = s->het ? s->omf : nullptr;
  a.omf_u = s->omf_u;
  a.alpha_h = s->alpha / s->h;
  a.r = s->r;
  a.kD = s->kD;
  a.pref = SHIFT ? (T*)s->pref : nullptr;
  a.nx = s->nx;
  a.ny = s->ny;
  a.pitch = s->lo.pitch;
  a.plane = s->lo.plane;
  for (int k = 0; k < 4; ++k) {
    a.ftype[k] = s->ftype[k];
    a.bc[k] = s->flbc[k];
  }
  a.H = s->lo.lv[s->L].H;
  HIPCHK((launch_flow<T, SHIFT>(a, s->stream)));
  return BP_OK;
}

bp_status run_flow(bp_solver* s) {
  if (s->lo.fdbl) return s->lo.shift ? launch_flow_t<double, true>(s) : launch_flow_t<double, false>(s);
  return s->lo.shift ? launch_flow_t<float, true>(s) : launch_flow_t<float, false>(s);
}

template <typename T> bp_status launch_rebase_t(bp_solver* s) {
  RebaseArgs<T> a{};
  a.fbuf[0] = (T*)s->f[0];
  a.fbuf[1] = (T*)s->f[1];
  a.phase = s->phase;
  a.g = (T*)s->lo.lv[s->L].gA;
  a.eref = (T*)s->eref;
  a.pref = (T*)s->pref;
  a.nx = s->nx;
  a.ny = s->ny;
  a.pitch = s->lo.pitch;
  a.plane = s->lo.plane;
  HIPCHK(launch_rebase<T>(a, s->stream));
  return BP_OK;
}

bp_status run_rebase(bp_solver* s) { return s->lo.fdbl ? launch_rebase_t<double>(s) : launch_rebase_t<float>(s); }

template <typename T> bp_status launch_init_t(bp_solver* s) {
  InitArgs<T> a{};
  a.fbuf[0] = (T*)s->f[0];
  a.fbuf[1] = (T*)s->f[1];
  a.g = (T*)s->lo.lv[s->L].gA;
  for (int k = 0; k < 3; ++k) a.Dbuf[k] = s->D[k];
  a.phase = s->phase;
  a.fbody = s->has_body ? s->fbody : nullptr;
  a.src = s->has_src ? s->src : nullptr;
  a.eref = (T*)s->eref;
  a.pref = (T*)s->pref;
  a.p_out = s->pout;
  a.nx = s->nx;
  a.ny = s->ny;
  a.pitch = s->lo.pitch;
  a.plane = s->lo.plane;
  HIPCHK(launch_init<T>(a, s->stream));
  return BP_OK;
}

bp_status run_init(bp_solver* s) { return s->lo.fdbl ? launch_init_t<double>(s) : launch_init_t<float>(s); }

template <typename T, bool SHIFT> bp_status launch_extract_t(bp_solver* s) {
  ExtractArgs<T> a{};
  a.g = (const T*)s->lo.lv[s->L].gA;
  a.Ft = (const T*)s->Ft;
  a.eref = SHIFT ? (const T*)s->eref : nullptr;
  a.kD = s->kD;
  a.cstar = s->cstar;
  a.b_s = s->b_s;
  a.b_d = s->b_d;
  a.inv_c0h = 1.0 / (s->c0 * s->h);
  a.eta = s->eta;
  a.sigma = s->sig;
  a.nx = s->nx;
  a.ny = s->ny;
  a.pitch = s->lo.pitch;
  a.plane = s->lo.plane;
  a.perx = s->el[kLeft] == kElPeriodic;
  a.pery = s->el[kBottom] == kElPeriodic;
  HIPCHK((launch_extract<T, SHIFT>(a, s->stream)));
  return BP_OK;
}

bp_status run_extract(bp_solver* s) {
  if (s->lo.fdbl) return s->lo.shift ? launch_extract_t<double, true>(s) : launch_extract_t<double, false>(s);
  return s->lo.shift ? launch_extract_t<float, true>(s) : launch_extract_t<float, false>(s);
}

int fine_waves(const bp_solver* s) {
  const LevelBuf& v = s->lo.lv[s->L];
  return sweep_waves(v.nx, v.ny, v.H);
}

// the device work of one time step with a fixed number of V-cycles
bp_status enqueue_fixed_step(bp_solver* s) {
  if (s->lo.shift) BPCHK(run_rebase(s));
  BPCHK(run_force(s));
  for (int j = 0; j < s->ne_fixed; ++j) {
    const bool last = (j == s->ne_fixed - 1);
    BPCHK(vcycle(s, s->L, false, false, last ? s->part : nullptr));
  }
  if (s->ne_fixed > 0) HIPCHK(launch_finalize(s->part, fine_waves(s), s->scal, s->flags, s->stream));
  BPCHK(run_flow(s));
  HIPCHK(launch_advance(s->phase, s->stream));
  return BP_OK;
}

bp_status build_graph(bp_solver* s) {
  if (s->graph) {
    (void)hipGraphExecDestroy(s->graph);
    s->graph = nullptr;
  }
  s->graph_valid = false;
  if (!s->use_graph || !s->stream) return BP_OK;
  HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
  bp_status st = enqueue_fixed_step(s);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s->stream, &g);
  if (st != BP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(BP_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&s->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(BP_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  s->graph_valid = true;
  return BP_OK;
}

// adaptive number of V-cycles: before V-cycle j+1 (j >= 1) the first smoothing
// sweep also measures ||g - S(g)|| and ||g||; the cycle is abandoned (the
// sweep's output discarded) once the ratio reaches the tolerance
bp_status adaptive_step(bp_solver* s) {
  if (s->lo.shift) BPCHK(run_rebase(s));
  BPCHK(run_force(s));
  LevelBuf& v = s->lo.lv[s->L];
  int j = 0;
  double ratio = -1.0;
  for (;;) {
    if (j >= 1) {
      BPCHK(sweep(s, SweepReq{s->L, kSmooth, v.gA, v.gB, nullptr, s->Ft, nullptr, nullptr, false, s->part}));
      HIPCHK(launch_finalize(s->part, fine_waves(s), s->scal, s->flags, s->stream));
      HIPCHK(hipMemcpyAsync(s->host_pin, s->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
      HIPCHK(hipStreamSynchronize(s->stream));
      const double nr = std::sqrt(s->host_pin[0]), ng = std::sqrt(s->host_pin[1]);
      ratio = ng > 0 ? nr / ng : 0.0;
      if (!std::isfinite(nr) || !std::isfinite(ng)) {
        s->status = BP_ERR_DIVERGED;
        return fail(BP_ERR_DIVERGED, "non-finite residual norm");
      }
      if (nr <= s->ne_tol * ng || j >= s->ne_max) break;
      BPCHK(vcycle(s, s->L, false, true, nullptr));
    } else {
      BPCHK(vcycle(s, s->L, false, false, nullptr));
    }
    ++j;
  }
  s->last_ne = j;
  s->last_ratio = ratio;
  s->total_cycles += j;
  BPCHK(run_flow(s));
  HIPCHK(launch_advance(s->phase, s->stream));
  return BP_OK;
}

// ------------------------------------------------------- boundary terms
// value of side data at the midpoint of the link leaving boundary cell i of
// `side` in direction (ox, oy); see the corner rules in the header comment of
// bp_create
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
      // mirror image across the perpendicular wall: the component normal to
      // that wall changes sign (tangential index of this side's data)
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

// ------------------------------------------------------------ state I/O
template <typename T>
bp_status upload_planes(bp_solver* s, void* dst, int nx, int ny, int pitch, int64_t plane, const double* src,
                        int m) {
  std::vector<T> tmp((size_t)m * plane, T(0));
  for (int c = 0; c < m; ++c)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        tmp[(size_t)c * plane + (size_t)y * pitch + x] = src ? T(src[((size_t)c * ny + y) * nx + x]) : T(0);
  HIPCHK(hipMemcpyAsync(dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  return BP_OK;
}

template <typename T>
bp_status download_planes(bp_solver* s, const void* srcd, int nx, int ny, int pitch, int64_t plane, double* dst,
                          int m) {
  std::vector<T> tmp((size_t)m * plane);
  HIPCHK(hipMemcpyAsync(tmp.data(), srcd, tmp.size() * sizeof(T), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  for (int c = 0; c < m; ++c)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        dst[((size_t)c * ny + y) * nx + x] = double(tmp[(size_t)c * plane + (size_t)y * pitch + x]);
  return BP_OK;
}

bp_status up(bp_solver* s, bool dbl, void* dst, int nx, int ny, int pitch, int64_t plane, const double* src, int m) {
  return dbl ? upload_planes<double>(s, dst, nx, ny, pitch, plane, src, m)
             : upload_planes<float>(s, dst, nx, ny, pitch, plane, src, m);
}
bp_status down(bp_solver* s, bool dbl, const void* srcd, int nx, int ny, int pitch, int64_t plane, double* dst,
               int m) {
  return dbl ? download_planes<double>(s, srcd, nx, ny, pitch, plane, dst, m)
             : download_planes<float>(s, srcd, nx, ny, pitch, plane, dst, m);
}

bp_status upload_loads(bp_solver* s, const double* body_f, const double* source_s) {
  const int nx = s->nx, ny = s->ny;
  const size_t N = (size_t)nx * ny;
  s->has_body = body_f != nullptr;
  s->has_src = source_s != nullptr;
  std::vector<double> b(2 * N), sv(N);
  if (body_f)
    for (size_t k = 0; k < 2 * N; ++k) b[k] = s->h * s->h * s->c0 * body_f[k];
  if (source_s)
    for (size_t k = 0; k < N; ++k) sv[k] = s->dt * source_s[k];
  BPCHK(upload_planes<double>(s, s->fbody, nx, ny, s->lo.pitch, s->lo.plane, body_f ? b.data() : nullptr, 2));
  BPCHK(upload_planes<double>(s, s->src, nx, ny, s->lo.pitch, s->lo.plane, source_s ? sv.data() : nullptr, 1));
  return BP_OK;
}

double geq_host(int q, double ex, double ey) { return 3.0 * W8[q] * (CX8[q] * ex + CY8[q] * ey); }

}  // namespace

// ===================================================================== C ABI
extern "C" {

const char* bp_last_error(void) { return g_err.c_str(); }

bp_status bp_workspace_bytes(const bp_problem* p, size_t* device_bytes) {
  BPCHK(validate(p));
  if (!device_bytes) return fail(BP_ERR_ARG, "null output");
  Layout lo;
  make_layout(p, lo);
  *device_bytes = lo.total;
  return BP_OK;
}

bp_status bp_create(const bp_problem* p, void* device_ws, size_t ws_bytes, void* hip_stream, bp_solver** out) {
  if (!out) return fail(BP_ERR_ARG, "null output handle");
  *out = nullptr;
  BPCHK(validate(p));
  Layout lo;
  make_layout(p, lo);
  if (!device_ws || ((uintptr_t)device_ws % kAlign) != 0 || ws_bytes < lo.total)
    return fail(BP_ERR_WORKSPACE, "workspace missing, not 256-byte aligned or smaller than bp_workspace_bytes");
  bp_solver* s = new bp_solver();
  s->lo = lo;
  s->stream = (hipStream_t)hip_stream;
  s->ws = (char*)device_ws;
  s->nx = p->nx;
  s->ny = p->ny;
  s->L = lo.L;
  s->K = p->K;
  s->h = p->dx;
  s->dt = p->dt;
  s->c0 = p->c0;
  s->alpha = p->alpha;
  s->r = p->r;
  s->gamma = p->gamma;
  s->lam = p->c0 * p->lambda;
  s->mu = p->c0 * p->mu;
  const double lm = s->lam + s->mu;
  s->om_s = 2.0 / (3.0 * lm + 1.0);            // Table 2
  s->om_d = 2.0 / (6.0 * s->mu + 1.0);
  s->b_s = 3.0 * lm / (3.0 * lm + 1.0);        // eq. moments:bared
  s->b_d = 6.0 * s->mu / (6.0 * s->mu + 1.0);
  s->beta22 = 1.0 / (12.0 * lm + 4.0);         // eq. moments:collision:22
  s->kD = -s->b_s / (2.0 * lm);                // eq. LBM:divergence
  s->cstar = s->r * s->alpha * s->alpha / 2.0; // implicit part of the centred source
  s->ne_fixed = p->ne_fixed;
  s->ne_tol = p->ne_tol;
  s->ne_max = p->ne_max;
  for (int k = 0; k < 4; ++k) s->el[k] = p->side[k].el;
  char* w = s->ws;
  for (int l = 1; l <= lo.L; ++l) {
    LevelBuf& v = s->lo.lv[l];
    v.gA = w + v.oA;
    v.gB = w + v.oB;
    v.r = v.oR ? (void*)(w + v.oR) : nullptr;
  }
  s->f[0] = w + lo.off_f[0];
  s->f[1] = w + lo.off_f[1];
  for (int k = 0; k < 3; ++k) s->D[k] = (double*)(w + lo.off_D[k]);
  s->pout = (double*)(w + lo.off_pout);
  s->fbody = (double*)(w + lo.off_fbody);
  s->src = (double*)(w + lo.off_src);
  s->omf = (double*)(w + lo.off_omf);
  s->Ft = w + lo.off_Ft;
  s->eref = lo.shift ? (void*)(w + lo.off_eref) : nullptr;
  s->pref = lo.shift ? (void*)(w + lo.off_pref) : nullptr;
  s->eta = (double*)(w + lo.off_eta);
  s->sig = (double*)(w + lo.off_sig);
  s->part = (double*)(w + lo.off_part);
  s->scal = (double*)(w + lo.off_scal);
  s->phase = (int*)(w + lo.off_scal + 32);
  s->flags = (int*)(w + lo.off_scal + 40);

  auto bail = [&](bp_status st) {
    delete s;
    return st;
  };
  if (hipHostMalloc((void**)&s->host_pin, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return bail(fail(BP_ERR_DEVICE, "hipHostMalloc failed"));
  if (launch_fill_zero(w, lo.total, s->stream) != hipSuccess) return bail(fail(BP_ERR_DEVICE, "clear failed"));

  // permeability -> lattice relaxation rate of the flow LBM (eq. pressure:rate)
  const size_t N = (size_t)p->nx * p->ny;
  auto omega_of = [&](double kap) { return 1.0 / (3.0 * (kap / p->c0) * p->dt / (p->dx * p->dx) + 0.5); };
  if (p->kappa) {
    std::vector<double> om(N);
    for (size_t k = 0; k < N; ++k) {
      if (!(p->kappa[k] > 0)) return bail(fail(BP_ERR_ARG, "kappa must be > 0 everywhere"));
      om[k] = omega_of(p->kappa[k]);
    }
    s->het = true;
    s->omf_u = om[0];
    if (upload_planes<double>(s, s->omf, p->nx, p->ny, lo.pitch, lo.plane, om.data(), 1) != BP_OK)
      return bail(BP_ERR_DEVICE);
  } else {
    s->het = false;
    s->omf_u = omega_of(p->kappa_uniform);
  }
  // boundary terms (finest level; coarse levels use homogeneous data)
  for (int k = 0; k < 4; ++k) {
    std::vector<double> et, ft;
    std::vector<int8_t> ty;
    elastic_terms(p, k, s->h, et);
    flow_terms(p, k, ft, ty);
    s->elbc[k] = (double*)(w + lo.off_elbc[k]);
    s->ftype[k] = (int8_t*)(w + lo.off_ftype[k]);
    s->flbc[k] = (double*)(w + lo.off_flbc[k]);
    s->elbc_used[k] = (p->side[k].el == BP_EL_DIRICHLET || p->side[k].el == BP_EL_TRACTION);
    if (hipMemcpyAsync(s->elbc[k], et.data(), et.size() * 8, hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->flbc[k], ft.data(), ft.size() * 8, hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->ftype[k], ty.data(), ty.size(), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
      return bail(fail(BP_ERR_DEVICE, "boundary upload failed"));
  }
  if (upload_loads(s, p->body_f, p->source_s) != BP_OK) return bail(BP_ERR_DEVICE);
  if (run_init(s) != BP_OK) return bail(BP_ERR_DEVICE);
  if (const char* e = std::getenv("BIOT_NO_GRAPH")) s->use_graph = (std::atoi(e) == 0);
  if (hipStreamSynchronize(s->stream) != hipSuccess) return bail(fail(BP_ERR_DEVICE, "init failed"));
  *out = s;
  return BP_OK;
}

bp_status bp_destroy(bp_solver* s) {
  if (!s) return BP_OK;
  if (s->graph) (void)hipGraphExecDestroy(s->graph);
  if (s->host_pin) (void)hipHostFree(s->host_pin);
  delete s;
  return BP_OK;
}

bp_status bp_step(bp_solver* s, int32_t nsteps) {
  if (!s) return fail(BP_ERR_ARG, "null solver");
  if (s->status != BP_OK) return fail(BP_ERR_STATE, "solver is in an error state");
  if (nsteps < 0) return fail(BP_ERR_ARG, "nsteps < 0");
  for (int k = 0; k < nsteps; ++k) {
    if (s->ne_fixed > 0) {
      if (s->use_graph && s->stream) {
        if (!s->graph_valid) BPCHK(build_graph(s));
        HIPCHK(hipGraphLaunch(s->graph, s->stream));
      } else {
        BPCHK(enqueue_fixed_step(s));
      }
      s->last_ne = s->ne_fixed;
      s->total_cycles += s->ne_fixed;
    } else {
      bp_status st = adaptive_step(s);
      if (st != BP_OK) {
        s->status = st;
        return st;
      }
    }
    s->step += 1;
  }
  return BP_OK;
}

bp_status bp_set_loads(bp_solver* s, const double* body_f, const double* source_s, int32_t reinit) {
  if (!s) return fail(BP_ERR_ARG, "null solver");
  HIPCHK(hipStreamSynchronize(s->stream));
  const bool had_body = s->has_body, had_src = s->has_src;
  BPCHK(upload_loads(s, body_f, source_s));
  if (had_body != s->has_body || had_src != s->has_src) s->graph_valid = false;
  if (reinit) {
    BPCHK(run_init(s));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->step = 0;
    s->status = BP_OK;
  }
  return BP_OK;
}

bp_status bp_get_fields(bp_solver* s, double* eta, double* p, double* sigma, int32_t* step) {
  if (!s) return fail(BP_ERR_ARG, "null solver");
  BPCHK(run_extract(s));
  const size_t N = (size_t)s->nx * s->ny;
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, s->flags, sizeof(int), hipMemcpyDeviceToHost, s->stream));
  if (eta) HIPCHK(hipMemcpyAsync(eta, s->eta, 2 * N * 8, hipMemcpyDeviceToHost, s->stream));
  if (sigma) HIPCHK(hipMemcpyAsync(sigma, s->sig, 3 * N * 8, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  if (p) {
    BPCHK(download_planes<double>(s, s->pout, s->nx, s->ny, s->lo.pitch, s->lo.plane, p, 1));
    for (size_t k = 0; k < N; ++k) p[k] /= s->c0;
  }
  if (step) *step = s->step;
  bool finite = true;
  if (eta)
    for (size_t k = 0; k < 2 * N && finite; ++k) finite = std::isfinite(eta[k]);
  if (flag || !finite) {
    s->status = BP_ERR_DIVERGED;
    return fail(BP_ERR_DIVERGED, "the solution is not finite");
  }
  return BP_OK;
}

bp_status bp_get_state(bp_solver* s, double* f, double* g, double* D1, double* D2, int32_t* step) {
  if (!s) return fail(BP_ERR_ARG, "null solver");
  const int n = s->step;
  const int nx = s->nx, ny = s->ny;
  const size_t N = (size_t)nx * ny;
  const LevelBuf& v = s->lo.lv[s->L];
  HIPCHK(hipStreamSynchronize(s->stream));
  std::vector<double> pr, er;
  if (s->lo.shift) {
    pr.resize(N);
    er.resize(2 * N);
    BPCHK(down(s, s->lo.fdbl, s->pref, nx, ny, s->lo.pitch, s->lo.plane, pr.data(), 1));
    BPCHK(down(s, s->lo.fdbl, s->eref, nx, ny, s->lo.pitch, s->lo.plane, er.data(), 2));
  }
  if (f) {
    BPCHK(down(s, s->lo.fdbl, s->f[n & 1], nx, ny, s->lo.pitch, s->lo.plane, f, 9));
    if (s->lo.shift)
      for (int i = 0; i < 9; ++i)
        for (size_t k = 0; k < N; ++k) f[i * N + k] += W9[i] * pr[k];
  }
  if (g) {
    BPCHK(down(s, v.dbl, v.gA, nx, ny, v.pitch, v.plane, g, 8));
    if (s->lo.shift)
      for (int q = 0; q < 8; ++q)
        for (size_t k = 0; k < N; ++k) g[q * N + k] += geq_host(q, er[k], er[N + k]);
  }
  if (D1) BPCHK(download_planes<double>(s, s->D[(n + 2) % 3], nx, ny, s->lo.pitch, s->lo.plane, D1, 1));
  if (D2) BPCHK(download_planes<double>(s, s->D[(n + 1) % 3], nx, ny, s->lo.pitch, s->lo.plane, D2, 1));
  if (step) *step = s->step;
  return BP_OK;
}

bp_status bp_set_state(bp_solver* s, const double* f, const double* g, const double* D1, const double* D2,
                       int32_t step) {
  if (!s) return fail(BP_ERR_ARG, "null solver");
  if (step < 0) return fail(BP_ERR_ARG, "step < 0");
  const int nx = s->nx, ny = s->ny;
  const LevelBuf& v = s->lo.lv[s->L];
  HIPCHK(hipStreamSynchronize(s->stream));
  s->step = step;
  const int n = step;
  // the device phase counter follows the host step count
  int ph = n;
  HIPCHK(hipMemcpyAsync(s->phase, &ph, sizeof(int), hipMemcpyHostToDevice, s->stream));
  if (s->lo.shift) {  // references to zero: stored offsets are the full populations
    HIPCHK(launch_fill_zero(s->eref, align_up(2 * s->lo.plane * (s->lo.fdbl ? 8 : 4)), s->stream));
    HIPCHK(launch_fill_zero(s->pref, align_up(s->lo.plane * (s->lo.fdbl ? 8 : 4)), s->stream));
  }
  if (f) BPCHK(up(s, s->lo.fdbl, s->f[n & 1], nx, ny, s->lo.pitch, s->lo.plane, f, 9));
  if (g) BPCHK(up(s, v.dbl, v.gA, nx, ny, v.pitch, v.plane, g, 8));
  if (D1) BPCHK(upload_planes<double>(s, s->D[(n + 2) % 3], nx, ny, s->lo.pitch, s->lo.plane, D1, 1));
  if (D2) BPCHK(upload_planes<double>(s, s->D[(n + 1) % 3], nx, ny, s->lo.pitch, s->lo.plane, D2, 1));
  int zero = 0;
  HIPCHK(hipMemcpyAsync(s->flags, &zero, sizeof(int), hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  s->status = BP_OK;
  return BP_OK;
}

bp_status bp_level_shape(const bp_solver* s, int32_t level, int32_t* nx, int32_t* ny) {
  if (!s || level < 1 || level > s->L) return fail(BP_ERR_ARG, "bad level");
  *nx = s->lo.lv[level].nx;
  *ny = s->lo.lv[level].ny;
  return BP_OK;
}

bp_status bp_apply_elastic(bp_solver* s, int32_t level, const double* g, const double* r, const double* Ft,
                           double* out) {
  if (!s || level < 1 || level > s->L || !g || !out) return fail(BP_ERR_ARG, "bad arguments");
  const bool fine = level == s->L;
  if ((fine && r) || (!fine && Ft)) return fail(BP_ERR_ARG, "r applies to coarse levels, Ft to the finest");
  LevelBuf& v = s->lo.lv[level];
  if (fine && s->lo.shift)
    HIPCHK(launch_fill_zero(s->eref, align_up(2 * s->lo.plane * (s->lo.fdbl ? 8 : 4)), s->stream));
  BPCHK(up(s, v.dbl, v.gA, v.nx, v.ny, v.pitch, v.plane, g, 8));
  if (!fine) BPCHK(up(s, v.dbl, v.r, v.nx, v.ny, v.pitch, v.plane, r, 8));
  if (fine) BPCHK(up(s, s->lo.fdbl, s->Ft, v.nx, v.ny, v.pitch, v.plane, Ft, 2));
  BPCHK(sweep(s, SweepReq{level, kApply, v.gA, v.gB, fine ? nullptr : v.r, fine ? s->Ft : nullptr, nullptr,
                          nullptr, false, nullptr}));
  BPCHK(down(s, v.dbl, v.gB, v.nx, v.ny, v.pitch, v.plane, out, 8));
  return BP_OK;
}

bp_status bp_mg_cycle(bp_solver* s, int32_t level, double* g, const double* r, const double* Ft) {
  if (!s || level < 1 || level > s->L || !g) return fail(BP_ERR_ARG, "bad arguments");
  const bool fine = level == s->L;
  if ((fine && r) || (!fine && Ft)) return fail(BP_ERR_ARG, "r applies to coarse levels, Ft to the finest");
  LevelBuf& v = s->lo.lv[level];
  if (fine && s->lo.shift)
    HIPCHK(launch_fill_zero(s->eref, align_up(2 * s->lo.plane * (s->lo.fdbl ? 8 : 4)), s->stream));
  BPCHK(up(s, v.dbl, v.gA, v.nx, v.ny, v.pitch, v.plane, g, 8));
  if (!fine) BPCHK(up(s, v.dbl, v.r, v.nx, v.ny, v.pitch, v.plane, r, 8));
  if (fine) BPCHK(up(s, s->lo.fdbl, s->Ft, v.nx, v.ny, v.pitch, v.plane, Ft, 2));
  BPCHK(vcycle(s, level, false, false, nullptr));
  BPCHK(down(s, v.dbl, v.gA, v.nx, v.ny, v.pitch, v.plane, g, 8));
  return BP_OK;
}

bp_status bp_explicit_force(bp_solver* s, double* Ft) {
  if (!s || !Ft) return fail(BP_ERR_ARG, "bad arguments");
  int ph = s->step;
  HIPCHK(hipMemcpyAsync(s->phase, &ph, sizeof(int), hipMemcpyHostToDevice, s->stream));
  BPCHK(run_force(s));
  BPCHK(down(s, s->lo.fdbl, s->Ft, s->nx, s->ny, s->lo.pitch, s->lo.plane, Ft, 2));
  return BP_OK;
}

bp_status bp_stats(const bp_solver* s, bp_run_stats* st) {
  if (!s || !st) return fail(BP_ERR_ARG, "bad arguments");
  st->step = s->step;
  st->last_ne = s->last_ne;
  st->total_cycles = s->total_cycles;
  st->last_ratio = s->last_ratio;
  st->levels = s->L;
  int flag = 0;
  if (hipMemcpy(&flag, s->flags, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(BP_ERR_DEVICE, "stats copy failed");
  st->diverged = flag;
  return BP_OK;
}

bp_status bp_time_kernel(bp_solver* s, int32_t which, int32_t iters, double* avg_us, double* bytes) {
  if (!s || iters < 1 || !avg_us) return fail(BP_ERR_ARG, "bad arguments");
  LevelBuf& v = s->lo.lv[s->L];
  const double es = s->lo.fdbl ? 8.0 : 4.0;
  const double N = (double)s->nx * s->ny;
  const double shift = s->lo.shift ? 1.0 : 0.0;
  double b = 0.0;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // keep p_out: the timed flow launches overwrite it
  std::vector<double> psave;
  if (which == 2) {
    psave.resize((size_t)s->lo.plane);
    HIPCHK(hipMemcpyAsync(psave.data(), s->pout, s->lo.plane * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
  }
  auto one = [&]() -> bp_status {
    switch (which) {
      case 0:
        return sweep(s, SweepReq{s->L, kSmooth, v.gA, v.gB, nullptr, s->Ft, nullptr, nullptr, false, nullptr});
      case 1: {
        if (s->L < 2) return fail(BP_ERR_ARG, "no coarser level");
        LevelBuf& c = s->lo.lv[s->L - 1];
        return sweep(s, SweepReq{s->L, kRestrict, v.gA, nullptr, nullptr, s->Ft, nullptr, c.r, false, nullptr});
      }
      case 2: return run_flow(s);
      default: return run_force(s);
    }
  };
  BPCHK(one());  // warm-up
  HIPCHK(hipEventRecord(e0, s->stream));
  for (int k = 0; k < iters; ++k) BPCHK(one());
  HIPCHK(hipEventRecord(e1, s->stream));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (which == 2) {
    HIPCHK(hipMemcpyAsync(s->pout, psave.data(), s->lo.plane * 8, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
  }
  *avg_us = 1000.0 * ms / iters;
  switch (which) {
    case 0: b = N * (16.0 + 2.0 + 2.0 * shift) * es; break;
    case 1: {
      const double ce = s->lo.lv[s->L - 1].dbl ? 8.0 : 4.0;
      b = N * (8.0 + 2.0 + 2.0 * shift) * es + (N / 4.0) * 8.0 * ce;
      break;
    }
    case 2:
      b = N * (18.0 + 8.0 + 2.0 * shift) * es + N * 8.0 * (2.0 + 1.0 + 1.0) + (s->has_src ? N * 8.0 : 0.0) +
          (s->het ? N * 8.0 : 0.0);
      break;
    default:
      b = N * (9.0 + 2.0) * es + N * 8.0 * 2.0 + (s->has_body ? N * 16.0 : 0.0) + (s->has_src ? N * 8.0 : 0.0) +
          (s->het ? N * 8.0 : 0.0);
      break;
  }
  if (bytes) *bytes = b;
  return BP_OK;
}

bp_status bp_device_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (!dst || !src || bytes % 16) return fail(BP_ERR_ARG, "bad copy arguments");
  HIPCHK(launch_copy(dst, src, bytes, (hipStream_t)hip_stream));
  return BP_OK;
}

}  // extern "C"
