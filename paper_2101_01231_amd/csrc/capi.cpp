// C ABI of libridg (declared in include/ridg.h): argument checking, workspace carving,
// host precompute, and the step sequence (prediction, then correction) on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <array>
#include <mutex>
#include <cstdlib>
#include <map>

#include "k_stencil3d.hpp"
#include "k_tblock.hpp"
#include "ridg_internal.hpp"

using namespace ridg;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
}  // namespace

int ridg::set_last_error(int code, const std::string& msg) { return fail(code, msg); }

namespace {

int hip_fail(int err, const char* what) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString((hipError_t)err));
  return fail(RIDG_E_DEVICE, buf);
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr int64_t kDenseScratchBytes = (int64_t)256 << 20;

struct Layout {
  size_t q0, q1, w, stage, tens, g, dc, kc, fg, fd, fk, fgs, taps, plans, items[kLayouts], item_plan[kLayouts], dense, scratch, flag, ptab, tplans, telems,
      btab, bint, nstats, total;
  size_t btab_doubles = 0, bint_ints = 0;
  int64_t n_tear = 0;
  size_t ptab_doubles = 0;
  int64_t n_items[kLayouts] = {}, n_dense = 0, scratch_elems = 0;
  size_t tens_doubles = 0;
};

size_t tensor_doubles(const RefTensors& T) {
  return T.Tt.size() + T.Cc.size() + T.Bv.size() + T.Fo.size() + T.Fn.size() + T.Cv.size() + T.CFo.size() +
         T.CFn.size() + T.Cown.size();
}

// Element work lists of the REGION solver, grouped by plan and padded so that a wavefront never
// mixes plans (padding repeats the group's last element with a "do not store" mark).
void build_items(const RegionPlans& R, int ipw, std::vector<int32_t>* items, std::vector<int32_t>* item_plan) {
  const int np = (int)R.plans.size();
  std::vector<std::vector<int32_t>> groups(np);
  for (size_t e = 0; e < R.elem_plan.size(); ++e)
    if (R.elem_plan[e] >= 0) groups[R.elem_plan[e]].push_back((int32_t)e);
  items->clear();
  item_plan->clear();
  for (int p = 0; p < np; ++p) {
    auto& gr = groups[p];
    if (gr.empty()) continue;
    for (int32_t e : gr) {
      items->push_back(e);
      item_plan->push_back(p);
    }
    int32_t last = gr.back();
    while (items->size() % ipw) {
      items->push_back(-last - 1);
      item_plan->push_back(p);
    }
  }
}

Layout make_layout(const Problem& P, const RefTensors& T, const RegionPlans* R, const int64_t n_items[kLayouts]) {
  Layout L;
  const size_t nel = (size_t)P.nel, ns = T.ns, nt = T.nt;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align_up(bytes);
    return at;
  };
  L.q0 = take(nel * ns * 8);
  L.q1 = take(nel * ns * 8);
  L.w = take(nel * nt * 8);
  L.stage = take(nel * std::max(ns, nt) * 8);
  L.tens_doubles = tensor_doubles(T);
  L.tens = take(L.tens_doubles * 8);
  L.g = take((size_t)kMaxBlocks * nt * ns * 8);
  L.dc = take((size_t)7 * ns * nt * 8);
  L.kc = take((size_t)kMaxTapUpdate * ns * ns * 8);
  {  // MFMA fragments of the constant-velocity operators (G, D, K)
    const bool pref = P.solver == RIDG_SOLVER_PREFACTORED;
    L.fg = take(pref ? mfma_fragment_doubles(kMaxBlocks, (int)nt, (int)ns) * 8 : 8);
    L.fd = take(pref ? mfma_fragment_doubles(7, (int)ns, (int)nt) * 8 : 8);
    L.fk = take(pref ? mfma_fragment_doubles(kMaxTapUpdate, (int)ns, (int)ns) * 8 : 8);
    L.fgs = take(pref ? mfma_fragment_doubles(kMaxBlocks, (int)nt, (int)ns) * 4 : 8);  // G fragments as FP32
  }
  L.taps = take((size_t)kMaxBlocks * 3 * 4);
  int64_t n_dense = 0;
  size_t nplans = 0;
  if (P.solver == RIDG_SOLVER_REGION && R) {
    nplans = R->plans.size();
    n_dense = (int64_t)R->dense_elems.size();
  } else if (P.solver == RIDG_SOLVER_DENSE) {
    n_dense = P.nel;
  }
  L.plans = take(std::max<size_t>(nplans, 1) * sizeof(PlanRec));
  for (int l = 0; l < kLayouts; ++l) {
    L.n_items[l] = n_items[l];
    L.items[l] = take(std::max<int64_t>(n_items[l], 1) * 4);
    L.item_plan[l] = take(std::max<int64_t>(n_items[l], 1) * 4);
  }
  L.n_dense = n_dense;
  L.dense = take(std::max<int64_t>(n_dense, 1) * 4);
  const int64_t N = (int64_t)std::pow(3, P.d) * nt;
  const int64_t per = N * (N + 1) * 8;
  const bool newton = P.solver == RIDG_SOLVER_NEWTON;
  L.scratch_elems = n_dense > 0 ? std::max<int64_t>(1, std::min<int64_t>(n_dense, kDenseScratchBytes / per)) : 0;
  L.scratch = take(std::max<int64_t>(L.scratch_elems, 1) * per);
  L.flag = take(256);
  if (newton) {  // Burgers tables: doubles, then the int32 index tables
    BurgersHost H;
    std::string m;
    if (build_burgers_tables(P, make_basis(P.d, P.M, P.basis), &H, &m) == RIDG_OK) {
      L.btab_doubles = H.psiv.size() + H.dpsivw.size() + H.projw.size() + H.dphivw.size() + H.psif.size() +
                       H.psifw.size() + H.phifw.size() + H.bval.size();
      L.bint_ints = H.bptr.size() + H.bp.size() + H.lift.size();
    }
  }
  L.btab = take(std::max<size_t>(L.btab_doubles, 1) * 8);
  L.bint = take(std::max<size_t>(L.bint_ints, 1) * 4);
  L.nstats = take(64);
  if (P.solver == RIDG_SOLVER_REGION) {
    const size_t nn = nt * nt;
    L.ptab_doubles = ((size_t)1 << (2 * P.d)) * nn + (size_t)P.d * 4 * nn + 2 * (size_t)P.d * 2 * nn + 2 * nt;
  }
  L.ptab = take(std::max<size_t>(L.ptab_doubles, 1) * 8);
  L.n_tear = (P.solver == RIDG_SOLVER_REGION && R) ? (int64_t)R->tear_elems.size() : 0;
  L.tplans = take(std::max<int64_t>(L.n_tear, 1) * sizeof(PlanRec));
  L.telems = take(std::max<int64_t>(L.n_tear, 1) * 4);
  L.total = off;
  return L;
}

}  // namespace

struct ridg_handle {
  Problem P;
  Basis B;
  RefTensors T;
  Layout L;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  double* Q[2] = {nullptr, nullptr};
  int cur = 0;
  double* W = nullptr;
  double* stage = nullptr;
  DevTensors dt{};
  double* G = nullptr;
  int32_t* taps = nullptr;
  int ntaps = 0;
  double g_dt = -1.0;
  std::vector<int32_t> host_taps;
  double* Dc = nullptr;  // constant-velocity correction taps
  double* Kc = nullptr;  // composite prediction+correction taps
  double* Fg = nullptr;  // MFMA fragments of G, Dc and Kc
  double* Fd = nullptr;
  double* Fk = nullptr;
  float* Fgs = nullptr;  // G fragments in FP32 (reduced-precision brick kernel)
  BrickTaps brick{};
  bool brick_ok = false;  // the brick kernel applies to this problem (3D, order 2-3, brick-divisible mesh)
  int opt_brick = 0;
  int opt_mfma = 0;
  std::vector<int32_t> host_dtaps, host_ktaps;
  int opt_composite = 0;
  int n_dtaps = 0;
  PlanRec* plans = nullptr;
  int32_t* items[kLayouts] = {};  // region work lists, one per segment layout
  int32_t* item_plan[kLayouts] = {};
  // options (ridg_set_option)
  int opt_graph = 0, opt_layout = 0, opt_fused = 0;
  hipGraphExec_t graph[2] = {nullptr, nullptr};  // two captured steps, per state-buffer parity
  hipStream_t cap = nullptr;                      // internal stream used only for capturing
  double graph_dt = -1.0;
  int32_t* dense = nullptr;
  PlanRec* tplans = nullptr;
  int32_t* telems = nullptr;
  double* scratch = nullptr;
  int32_t* flag = nullptr;
  BurgersDev bd{};            // RIDG_SOLVER_NEWTON: device view of the Burgers tables
  int32_t* nstats = nullptr;  // Newton counters: max iterations, failures, total iterations, solves
  DevGeom geom{};
  ridg_info info{};
  PlanTables pt{};
  double pt_dt = -1.0;
  // static-pivot layout: measured growth of elimination in natural order at pt_dt
  double sp_growth = 0.0;
  bool sp_ok = false;
  // constant velocity: von Neumann amplification of the step at vn_dt
  double vn_dt = -1.0;
  double vn_radius = 0.0;
  // dt of the operators that ridg_step_batch launches have read (-1: none yet)
  double batch_dt = -1.0;
  // stage timing
  bool timing = false;
  std::vector<hipEvent_t> events;  // 3 per timed step
  size_t ev_used = 0;
  // REGION solver: the dense regions run on a second stream, forked from and joined back to
  // the caller's stream around the upwind-plan kernel
  hipStream_t aux = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  ~ridg_handle() {
    for (int p = 0; p < 2; ++p)
      if (graph[p]) (void)hipGraphExecDestroy(graph[p]);
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (join_ev) (void)hipEventDestroy(join_ev);
    if (aux) (void)hipStreamDestroy(aux);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace {

int check_hip(int err, const char* what) { return err ? hip_fail(err, what) : RIDG_OK; }

DevGeom make_geom(const Problem& P) {
  DevGeom g{};
  g.d = P.d;
  g.n0 = P.n[0];
  g.n1 = P.n[1];
  g.n2 = P.n[2];
  g.h0 = P.h[0];
  g.h1 = P.h[1];
  g.h2 = P.h[2];
  for (int i = 0; i < 3; ++i) {
    g.a[i] = P.vel.a[i];
    for (int j = 0; j < 3; ++j) g.g[i][j] = P.vel.g[i][j];
  }
  return g;
}

double cfl_number(const Problem& P, double dt) {
  // affine velocity: extremes over the box are at its corners
  double best = 0.0;
  for (int c = 0; c < (1 << P.d); ++c) {
    for (int i = 0; i < P.d; ++i) {
      double v = P.vel.a[i];
      for (int j = 0; j < P.d; ++j) v += P.vel.g[i][j] * (((c >> j) & 1) ? P.L[j] : 0.0);
      best = std::max(best, std::fabs(v) * dt / P.h[i]);
    }
  }
  return best;
}

// flops of the algorithm as run (FMA = 2), per step: {prediction, correction}
std::pair<double, double> flops_model(const ridg_handle* h, double plan_flops) {
  const Problem& P = h->P;
  const double nel = (double)P.nel, nt = h->T.nt, ns = h->T.ns, d = P.d;
  const double np_active = (P.flux == RIDG_FLUX_CONST) ? 1.0 : (double)P.d;  // p-modes used per direction
  double correct = nel * 2.0 * ns * nt * np_active * 3.0 * d;  // volume + 2 faces per direction
  double predict = 0.0;
  if (P.solver == RIDG_SOLVER_PREFACTORED) {
    predict = nel * 2.0 * h->ntaps * nt * ns;
    correct = nel * 2.0 * h->n_dtaps * ns * nt;
  } else {
    double nbn = std::pow(3.0, d) * nt;
    double dense_elem = 2.0 / 3.0 * nbn * nbn * nbn + 2.0 * nbn * nbn;
    if (P.solver == RIDG_SOLVER_DENSE) {
      predict = nel * dense_elem;
    } else {
      predict = (double)h->info.n_dense_elements * dense_elem + plan_flops;
    }
  }
  return {predict, correct};
}

}  // namespace

// ---------------------------------------------------------------- autotuner
namespace {
std::mutex g_tune_mu;
std::map<std::string, std::array<int, 6>> g_tune_cache;  // problem key -> {graph, layout, fused, composite, mfma, brick}
bool g_tune_file_loaded = false;

std::string tune_key(const ridg_handle* h, int32_t steps) {
  char buf[256];
  const Problem& P = h->P;
  std::snprintf(buf, sizeof(buf), "d%d_n%dx%dx%d_M%d_f%d_s%d_p%d_r%d_k%d", P.d, P.n[0], P.n[1], P.n[2], P.M, P.flux,
                P.solver, P.precision, P.refine, steps);
  return buf;
}

void tune_file_load() {
  if (g_tune_file_loaded) return;
  g_tune_file_loaded = true;
  const char* path = std::getenv("RIDG_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {  // "<key> graph layout fused composite mfma brick"
    char key[256];
    int o[6], extra;
    if (std::sscanf(line, "%255s %d %d %d %d %d %d %d", key, &o[0], &o[1], &o[2], &o[3], &o[4], &o[5], &extra) == 7)
      g_tune_cache[key] = {o[0], o[1], o[2], o[3], o[4], o[5]};
  }
  std::fclose(f);
}

void tune_file_append(const std::string& key, const std::array<int, 6>& o) {
  const char* path = std::getenv("RIDG_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d %d %d\n", key.c_str(), o[0], o[1], o[2], o[3], o[4], o[5]);
  std::fclose(f);
}
}  // namespace

extern "C" {

const char* ridg_error_string(int code) {
  switch (code) {
    case RIDG_OK: return "ok";
    case RIDG_E_INVAL: return "invalid argument";
    case RIDG_E_NOMEM: return "workspace too small";
    case RIDG_E_DEVICE: return "device error";
    case RIDG_E_SINGULAR: return "singular region matrix";
    case RIDG_E_NONFINITE: return "non-finite value";
    case RIDG_E_UNSUPPORTED: return "unsupported problem";
    case RIDG_W_UNSTABLE: return "step may be unstable (von Neumann amplification or CFL number above 1)";
    default: return "unknown code";
  }
}

const char* ridg_last_error(void) { return g_last_error.c_str(); }

int ridg_workspace_bytes(const ridg_problem* problem, size_t* bytes) {
  if (!bytes) return fail(RIDG_E_INVAL, "bytes is NULL");
  Problem P;
  std::string msg;
  int rc = resolve_problem(problem, &P, &msg);
  if (rc) return fail(rc, msg);
  Basis B = make_basis(P.d, P.M, P.basis);
  RefTensors T = make_tensors(B);
  int64_t n_items[kLayouts] = {};
  RegionPlans R;
  if (P.solver == RIDG_SOLVER_REGION) {
    R = build_plans(P);
    for (int l = 0; l < kLayouts; ++l) {
      std::vector<int32_t> it, ip;
      build_items(R, items_per_wave(P.d, P.M, l), &it, &ip);
      n_items[l] = (int64_t)it.size();
    }
  }
  *bytes = make_layout(P, T, &R, n_items).total;
  return RIDG_OK;
}

int ridg_create(const ridg_problem* problem, void* d_workspace, size_t ws_bytes, void* hip_stream, ridg_t** out) {
  if (!out) return fail(RIDG_E_INVAL, "out is NULL");
  if (!d_workspace) return fail(RIDG_E_INVAL, "workspace is NULL");
  if ((uintptr_t)d_workspace % kAlign) return fail(RIDG_E_INVAL, "workspace must be 256-byte aligned");
  Problem P;
  std::string msg;
  int rc = resolve_problem(problem, &P, &msg);
  if (rc) return fail(rc, msg);
  ridg_handle* h = new (std::nothrow) ridg_handle();
  if (!h) return fail(RIDG_E_NOMEM, "host allocation failed");
  h->P = P;
  h->B = make_basis(P.d, P.M, P.basis);
  h->T = make_tensors(h->B);
  RegionPlans R;
  std::vector<int32_t> items[kLayouts], item_plan[kLayouts];
  double plan_flops = 0.0;
  if (P.solver == RIDG_SOLVER_REGION) {
    R = build_plans(P);
    for (int l = 0; l < kLayouts; ++l) build_items(R, items_per_wave(P.d, P.M, l), &items[l], &item_plan[l]);
    // flop tally of the plan work actually run (per element, padding excluded)
    const double nt = h->T.nt, ns = h->T.ns;
    const double np_active = (P.flux == RIDG_FLUX_CONST) ? 1.0 : (double)P.d;
    std::vector<double> per_plan(R.plans.size(), 0.0);
    for (size_t p = 0; p < R.plans.size(); ++p) {
      const PlanRec& pr = R.plans[p];
      for (int b = 0; b < pr.nb; ++b) {
        int own = 0, in = 0;
        for (int f = 0; f < 2 * P.d; ++f) (pr.blk[b].src[f] == kOwn ? own : in)++;
        per_plan[p] += 2.0 * nt * nt * np_active * (P.d + own) + 2.0 * nt * ns + in * 2.0 * nt * nt * np_active +
                       2.0 / 3.0 * nt * nt * nt + 2.0 * nt * nt;
        if (P.precision == RIDG_FP32_REFINE)  // per sweep: FP64 residual (2 nt^2) + replayed elimination (2 nt^2)
          per_plan[p] += P.refine * 4.0 * nt * nt;
      }
    }
    for (int32_t pid : R.elem_plan)
      if (pid >= 0) plan_flops += per_plan[pid];
    // tear regions: eliminated blocks carry 1 + theta_T right-hand sides
    for (const PlanRec& pr : R.tear_plans) {
      for (int b = 0; b < pr.nb; ++b) {
        int own = 0, in = 0;
        for (int f = 0; f < 2 * P.d; ++f) (pr.blk[b].src[f] == kOwn ? own : in)++;
        const double rr = (b == 0) ? nt : 1.0 + nt;  // tear equation: coupling products build its matrix
        plan_flops += 2.0 * nt * nt * np_active * (P.d + own) + 2.0 * nt + in * (2.0 * nt * nt * np_active + 2.0 * nt * rr) +
                      2.0 / 3.0 * nt * nt * nt + 2.0 * nt * nt * (b == 0 ? 1.0 : 1.0 + nt);
      }
      plan_flops += 2.0 * nt * nt;  // W_centre = alpha + B x
    }
  }
  int64_t n_items[kLayouts];
  for (int l = 0; l < kLayouts; ++l) n_items[l] = (int64_t)items[l].size();
  h->L = make_layout(P, h->T, &R, n_items);
  if (ws_bytes < h->L.total) {
    delete h;
    return fail(RIDG_E_NOMEM, "workspace smaller than ridg_workspace_bytes()");
  }
  h->stream = (hipStream_t)hip_stream;
  h->ws = (char*)d_workspace;
  h->Q[0] = (double*)(h->ws + h->L.q0);
  h->Q[1] = (double*)(h->ws + h->L.q1);
  h->W = (double*)(h->ws + h->L.w);
  h->stage = (double*)(h->ws + h->L.stage);
  h->G = (double*)(h->ws + h->L.g);
  h->Dc = (double*)(h->ws + h->L.dc);
  h->Kc = (double*)(h->ws + h->L.kc);
  h->Fg = (double*)(h->ws + h->L.fg);
  h->Fd = (double*)(h->ws + h->L.fd);
  h->Fk = (double*)(h->ws + h->L.fk);
  h->Fgs = (float*)(h->ws + h->L.fgs);
  h->brick_ok = P.solver == RIDG_SOLVER_PREFACTORED && brick_supported(P.d, P.M, P.n, P.precision == RIDG_FP32_REFINE);
  h->taps = (int32_t*)(h->ws + h->L.taps);
  h->plans = (PlanRec*)(h->ws + h->L.plans);
  for (int l = 0; l < kLayouts; ++l) {
    h->items[l] = (int32_t*)(h->ws + h->L.items[l]);
    h->item_plan[l] = (int32_t*)(h->ws + h->L.item_plan[l]);
  }
  h->dense = (int32_t*)(h->ws + h->L.dense);
  h->tplans = (PlanRec*)(h->ws + h->L.tplans);
  h->telems = (int32_t*)(h->ws + h->L.telems);
  h->scratch = (double*)(h->ws + h->L.scratch);
  h->flag = (int32_t*)(h->ws + h->L.flag);
  h->nstats = (int32_t*)(h->ws + h->L.nstats);
  // upload tensors
  const RefTensors& T = h->T;
  std::vector<double> tens;
  tens.reserve(h->L.tens_doubles);
  double* base = (double*)(h->ws + h->L.tens);
  auto push = [&](const std::vector<double>& v) {
    const double* at = base + tens.size();
    tens.insert(tens.end(), v.begin(), v.end());
    return at;
  };
  h->dt.Tt = push(T.Tt);
  h->dt.Cc = push(T.Cc);
  h->dt.Bv = push(T.Bv);
  h->dt.Fo = push(T.Fo);
  h->dt.Fn = push(T.Fn);
  h->dt.Cv = push(T.Cv);
  h->dt.CFo = push(T.CFo);
  h->dt.CFn = push(T.CFn);
  h->dt.Cown = push(T.Cown);
  h->geom = make_geom(P);
  int err = hipMemcpyAsync(base, tens.data(), tens.size() * 8, hipMemcpyHostToDevice, h->stream);
  if (!err && P.solver == RIDG_SOLVER_REGION) {
    if (!R.plans.empty())
      err = hipMemcpyAsync(h->plans, R.plans.data(), R.plans.size() * sizeof(PlanRec), hipMemcpyHostToDevice, h->stream);
    for (int l = 0; l < kLayouts && !err; ++l) {
      if (!items[l].empty())
        err = hipMemcpyAsync(h->items[l], items[l].data(), items[l].size() * 4, hipMemcpyHostToDevice, h->stream);
      if (!err && !item_plan[l].empty())
        err = hipMemcpyAsync(h->item_plan[l], item_plan[l].data(), item_plan[l].size() * 4, hipMemcpyHostToDevice,
                             h->stream);
    }
    if (!err && !R.dense_elems.empty())
      err = hipMemcpyAsync(h->dense, R.dense_elems.data(), R.dense_elems.size() * 4, hipMemcpyHostToDevice, h->stream);
    if (!err && !R.tear_elems.empty())
      err = hipMemcpyAsync(h->tplans, R.tear_plans.data(), R.tear_plans.size() * sizeof(PlanRec), hipMemcpyHostToDevice,
                           h->stream);
    if (!err && !R.tear_elems.empty())
      err = hipMemcpyAsync(h->telems, R.tear_elems.data(), R.tear_elems.size() * 4, hipMemcpyHostToDevice, h->stream);
  } else if (!err && P.solver == RIDG_SOLVER_DENSE) {
    std::vector<int32_t> all((size_t)P.nel);
    for (int64_t e = 0; e < P.nel; ++e) all[(size_t)e] = (int32_t)e;
    err = hipMemcpyAsync(h->dense, all.data(), all.size() * 4, hipMemcpyHostToDevice, h->stream);
    if (!err) err = hipStreamSynchronize(h->stream);
  }
  BurgersHost BH;  // kept alive until the uploads below have completed
  if (!err && P.solver == RIDG_SOLVER_NEWTON) {
    std::string m;
    int brc = build_burgers_tables(P, h->B, &BH, &m);
    if (brc) {
      delete h;
      return fail(brc, m);
    }
    std::vector<double> bt;
    bt.reserve(h->L.btab_doubles);
    double* bbase = (double*)(h->ws + h->L.btab);
    auto pushd = [&](const std::vector<double>& v) {
      const double* at = bbase + bt.size();
      bt.insert(bt.end(), v.begin(), v.end());
      return at;
    };
    std::vector<int32_t> bi;
    bi.reserve(h->L.bint_ints);
    int32_t* ibase = (int32_t*)(h->ws + h->L.bint);
    auto pushi = [&](const std::vector<int32_t>& v) {
      const int32_t* at = ibase + bi.size();
      bi.insert(bi.end(), v.begin(), v.end());
      return at;
    };
    BurgersDev& bd = h->bd;
    bd.Tt = h->dt.Tt;
    bd.Cc = h->dt.Cc;
    bd.psiv = pushd(BH.psiv);
    bd.dpsivw = pushd(BH.dpsivw);
    bd.projw = pushd(BH.projw);
    bd.dphivw = pushd(BH.dphivw);
    bd.psif = pushd(BH.psif);
    bd.psifw = pushd(BH.psifw);
    bd.phifw = pushd(BH.phifw);
    bd.bval = pushd(BH.bval);
    bd.bptr = pushi(BH.bptr);
    bd.bp = pushi(BH.bp);
    bd.lift = pushi(BH.lift);
    if (bt.size() != h->L.btab_doubles || bi.size() != h->L.bint_ints) {
      delete h;
      return fail(RIDG_E_NOMEM, "Burgers table layout");
    }
    err = hipMemcpyAsync(bbase, bt.data(), bt.size() * 8, hipMemcpyHostToDevice, h->stream);
    if (!err) err = hipMemcpyAsync(ibase, bi.data(), bi.size() * 4, hipMemcpyHostToDevice, h->stream);
    if (!err) err = hipStreamSynchronize(h->stream);
  }
  if (!err) err = hipMemsetAsync(h->nstats, 0, 64, h->stream);
  if (!err && P.solver == RIDG_SOLVER_REGION && (h->L.n_dense || h->L.n_tear) && h->L.n_items[0]) {
    err = hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking);
    if (!err) err = hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming);
    if (!err) err = hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming);
  }
  if (!err) err = hipMemsetAsync(h->Q[0], 0, (size_t)P.nel * T.ns * 8, h->stream);
  if (!err) err = hipStreamSynchronize(h->stream);  // host staging vectors go out of scope
  if (err) {
    delete h;
    return hip_fail(err, "ridg_create upload");
  }
  h->cur = 0;
  ridg_info& I = h->info;
  I.abi_version = RIDG_ABI_VERSION;
  I.basis = P.basis;
  if (P.basis == RIDG_BASIS_Q) h->opt_composite = 1;  // the tensor basis runs the composite stencil only
  I.theta = T.ns;
  I.theta_t = T.nt;
  I.solver = P.solver;
  I.n_elements = P.nel;
  I.n_plans = (int64_t)R.plans.size();
  I.n_dense_elements = h->L.n_dense;
  I.n_tear_elements = h->L.n_tear;
  I.n_taps = 0;
  if (P.solver == RIDG_SOLVER_PREFACTORED) {
    PlanRec rec;
    element_plan(P, 0, &rec);
    I.n_taps = rec.nb;
    h->ntaps = rec.nb;
    // tap counts do not depend on dt (face sides do not): size them once
    Prefactored pf;
    std::string m;
    if (build_prefactored(P, h->T, 1.0, &pf, &m) == RIDG_OK) {
      TapOperator dc, kc;
      build_correction_taps(P, h->T, 1.0, &dc);
      build_composite(P, pf, dc, &kc);
      h->n_dtaps = (int)dc.offs.size();
      I.flops_composite = (double)P.nel * 2.0 * kc.offs.size() * T.ns * T.ns;
    }
  }
  auto fl = flops_model(h, plan_flops);
  I.flops_predict = fl.first;
  I.flops_correct = fl.second;
  if (P.solver == RIDG_SOLVER_NEWTON) {  // per Newton iteration of every region, and per correction
    const double nt = T.nt, ns = T.ns, nb = std::pow(3.0, P.d), N = nb * nt, nf = 2.0 * P.d;
    const double q = burgers_q(P.M), nq = std::pow(q, P.d + 1), nqf = std::pow(q, P.d);
    double nnz = 0.0;
    {
      BurgersHost H2;
      std::string m2;
      if (build_burgers_tables(P, h->B, &H2, &m2) == RIDG_OK) nnz = (double)H2.bp.size();
    }
    const double fma_points = nb * nt * (nq + nf * nqf) + nb * nt * nq;              // point values, projection
    const double fma_rows = N * (nt + ns + P.d * nq + nf * nqf * (2.0 * nt + 1.0)) + nb * nnz;  // assembly
    const double fma_solve = N * N * N / 3.0 + N * N;                                      // elimination, back-solve
    I.flops_predict = (double)P.nel * 2.0 * (fma_points + fma_rows + fma_solve);
    I.flops_correct = (double)P.nel * 2.0 * (nq * (nt + P.d * ns) + nf * nqf * (2.0 * nt + ns));
  }
  I.bytes_predict = (double)P.nel * 8.0 * (T.ns + T.nt);
  I.bytes_correct = (double)P.nel * 8.0 * (2.0 * T.ns + T.nt);
  I.bytes_composite = (double)P.nel * 8.0 * 2.0 * T.ns;
  *out = h;
  return RIDG_OK;
}

int ridg_destroy(ridg_t* h) {
  delete h;
  return RIDG_OK;
}

int ridg_get_info(ridg_t* h, ridg_info* info) {
  if (!h || !info) return fail(RIDG_E_INVAL, "NULL argument");
  *info = h->info;
  return RIDG_OK;
}

int ridg_enable_timing(ridg_t* h, int32_t on) {
  if (!h) return fail(RIDG_E_INVAL, "handle is NULL");
  int err = hipStreamSynchronize(h->stream);
  if (err) return hip_fail(err, "hipStreamSynchronize");
  h->timing = on != 0;
  h->ev_used = 0;
  return RIDG_OK;
}

int ridg_get_timing(ridg_t* h, ridg_timing* out) {
  if (!h || !out) return fail(RIDG_E_INVAL, "NULL argument");
  int err = hipStreamSynchronize(h->stream);
  if (err) return hip_fail(err, "hipStreamSynchronize");
  ridg_timing t{};
  for (size_t s = 0; s + 2 < h->ev_used; s += 3) {
    float a = 0.f, b = 0.f;
    err = hipEventElapsedTime(&a, h->events[s], h->events[s + 1]);
    if (!err) err = hipEventElapsedTime(&b, h->events[s + 1], h->events[s + 2]);
    if (err) return hip_fail(err, "hipEventElapsedTime");
    t.steps += 1;
    t.predict_ms += a;
    t.correct_ms += b;
    t.max_step_ms = std::max(t.max_step_ms, (double)a + b);
  }
  h->ev_used = 0;
  *out = t;
  return RIDG_OK;
}

int ridg_newton_stats(ridg_t* h, int32_t* max_iters, int64_t* total_iters, int64_t* solves, int64_t* failures,
                      int32_t reset) {
  if (!h) return fail(RIDG_E_INVAL, "handle is NULL");
  if (h->P.solver != RIDG_SOLVER_NEWTON) return fail(RIDG_E_INVAL, "Newton statistics need RIDG_FLUX_BURGERS");
  int32_t buf[6] = {0, 0, 0, 0, 0, 0};
  int err = hipMemcpyAsync(buf, h->nstats, sizeof(buf), hipMemcpyDeviceToHost, h->stream);
  if (!err) err = hipStreamSynchronize(h->stream);
  if (!err && reset) err = hipMemsetAsync(h->nstats, 0, 64, h->stream);
  if (err) return hip_fail(err, "ridg_newton_stats");
  int64_t tot, nsol;
  std::memcpy(&tot, buf + 2, 8);
  std::memcpy(&nsol, buf + 4, 8);
  if (max_iters) *max_iters = buf[0];
  if (failures) *failures = buf[1];
  if (total_iters) *total_iters = tot;
  if (solves) *solves = nsol;
  return RIDG_OK;
}

int ridg_synchronize(ridg_t* h) {
  if (!h) return fail(RIDG_E_INVAL, "handle is NULL");
  return check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
}

int ridg_set_state(ridg_t* h, const double* q, size_t count, int32_t where) {
  if (!h || !q) return fail(RIDG_E_INVAL, "NULL argument");
  const size_t want = (size_t)h->P.nel * h->T.ns;
  if (count != want) return fail(RIDG_E_INVAL, "count must equal n_elements * theta");
  if (where == RIDG_HOST) {
    for (size_t i = 0; i < count; ++i)
      if (!std::isfinite(q[i])) return fail(RIDG_E_NONFINITE, "state contains NaN or Inf");
    int err = hipMemcpyAsync(h->stage, q, count * 8, hipMemcpyHostToDevice, h->stream);
    if (!err) err = launch_aos_to_soa(h->stage, h->Q[h->cur], h->P.nel, h->T.ns, h->stream);
    if (!err) err = hipStreamSynchronize(h->stream);
    return check_hip(err, "ridg_set_state");
  }
  if (where == RIDG_DEVICE) {
    int err = hipMemsetAsync(h->flag, 0, 4, h->stream);
    if (!err) err = launch_check_finite(q, (int64_t)count, h->flag, h->stream);
    int32_t flag = 0;
    if (!err) err = hipMemcpyAsync(&flag, h->flag, 4, hipMemcpyDeviceToHost, h->stream);
    if (!err) err = hipStreamSynchronize(h->stream);
    if (err) return hip_fail(err, "ridg_set_state");
    if (flag) return fail(RIDG_E_NONFINITE, "state contains NaN or Inf");
    return check_hip(launch_aos_to_soa(q, h->Q[h->cur], h->P.nel, h->T.ns, h->stream), "ridg_set_state");
  }
  return fail(RIDG_E_INVAL, "where must be RIDG_HOST or RIDG_DEVICE");
}

int ridg_get_state(ridg_t* h, double* q, size_t count, int32_t where) {
  if (!h || !q) return fail(RIDG_E_INVAL, "NULL argument");
  const size_t want = (size_t)h->P.nel * h->T.ns;
  if (count != want) return fail(RIDG_E_INVAL, "count must equal n_elements * theta");
  if (where == RIDG_HOST) {
    int err = launch_soa_to_aos(h->Q[h->cur], h->stage, h->P.nel, h->T.ns, h->stream);
    if (!err) err = hipMemcpyAsync(q, h->stage, count * 8, hipMemcpyDeviceToHost, h->stream);
    int32_t nfail = 0;
    if (!err && h->P.solver == RIDG_SOLVER_NEWTON)
      err = hipMemcpyAsync(&nfail, h->nstats + 1, 4, hipMemcpyDeviceToHost, h->stream);
    if (!err) err = hipStreamSynchronize(h->stream);
    if (err) return check_hip(err, "ridg_get_state");
    return nfail ? RIDG_W_NOT_CONVERGED : RIDG_OK;
  }
  if (where == RIDG_DEVICE)
    return check_hip(launch_soa_to_aos(h->Q[h->cur], q, h->P.nel, h->T.ns, h->stream), "ridg_get_state");
  return fail(RIDG_E_INVAL, "where must be RIDG_HOST or RIDG_DEVICE");
}

static int ensure_plan_tables(ridg_t* h, double dt) {
  if (h->P.solver != RIDG_SOLVER_REGION || dt == h->pt_dt) return RIDG_OK;
  HostPlanTables H = build_plan_tables(h->P, h->T, dt);
  std::vector<double> buf;
  buf.reserve(h->L.ptab_doubles);
  double* base = (double*)(h->ws + h->L.ptab);
  auto push = [&](const std::vector<double>& v) {
    const double* at = base + buf.size();
    buf.insert(buf.end(), v.begin(), v.end());
    return at;
  };
  h->pt.A0 = push(H.A0);
  h->pt.K = push(H.K);
  h->pt.Fn0 = push(H.Fn0);
  h->pt.FnC = push(H.FnC);
  h->pt.cc_val = push(H.cc_val);
  std::vector<double> idx(H.cc_idx.size(), 0.0);
  std::memcpy(idx.data(), H.cc_idx.data(), H.cc_idx.size() * 4);  // int32 payload in the last slot
  h->pt.cc_idx = (const int32_t*)push(idx);
  if (buf.size() > h->L.ptab_doubles) return fail(RIDG_E_NOMEM, "plan table layout");
  h->sp_growth = static_pivot_growth(h->P, H, h->T.nt, dt);
  h->sp_ok = h->sp_growth <= kStaticPivotMaxGrowth;
  h->info.static_pivot_growth = h->sp_growth;
  int err = hipMemcpyAsync(base, buf.data(), buf.size() * 8, hipMemcpyHostToDevice, h->stream);
  if (!err) err = hipStreamSynchronize(h->stream);
  if (err) return hip_fail(err, "upload of plan tables");
  h->pt_dt = dt;
  return RIDG_OK;
}

// Warning state of a step of size dt: the von Neumann amplification of the composed step
// (constant velocity, any solver; analysed once per dt), else the CFL number.
static int stability_warning(ridg_t* h, double dt) {
  if (h->P.flux == RIDG_FLUX_BURGERS) return RIDG_OK;  // reported through the Newton counters
  if (h->P.flux != RIDG_FLUX_CONST) return cfl_number(h->P, dt) > 1.0 ? RIDG_W_UNSTABLE : RIDG_OK;
  if (dt != h->vn_dt) {
    std::string msg;
    double rho = 0.0;
    int rc = von_neumann_radius(h->P, h->T, dt, &rho, &msg);
    if (rc) return fail(rc, msg);
    h->vn_dt = dt;
    h->vn_radius = rho;
    h->info.spectral_radius = rho;
  }
  return h->vn_radius > kUnstableRadius ? RIDG_W_UNSTABLE : RIDG_OK;
}

static int ensure_dt_tables(ridg_t* h, double dt) {
  if (h->P.solver == RIDG_SOLVER_REGION) return ensure_plan_tables(h, dt);
  if (h->P.solver != RIDG_SOLVER_PREFACTORED || dt == h->g_dt) return RIDG_OK;
  Prefactored pf;
  std::string msg;
  int rc = build_prefactored(h->P, h->T, dt, &pf, &msg);
  if (rc) return fail(rc, msg);
  h->host_taps.assign(pf.offs.size() * 3, 0);
  for (size_t t = 0; t < pf.offs.size(); ++t)
    for (int i = 0; i < 3; ++i) h->host_taps[3 * t + i] = pf.offs[t][i];
  h->ntaps = (int)pf.offs.size();
  TapOperator dc, kc;
  build_correction_taps(h->P, h->T, dt, &dc);
  build_composite(h->P, pf, dc, &kc);
  if (dc.offs.size() > 7 || kc.offs.size() > (size_t)kMaxTapUpdate) return fail(RIDG_E_UNSUPPORTED, "tap count");
  auto flat = [](const TapOperator& op, std::vector<int32_t>* v) {
    v->assign(op.offs.size() * 3, 0);
    for (size_t t = 0; t < op.offs.size(); ++t)
      for (int i = 0; i < 3; ++i) (*v)[3 * t + i] = op.offs[t][i];
  };
  flat(dc, &h->host_dtaps);
  flat(kc, &h->host_ktaps);
  const int nt = h->T.nt, ns = h->T.ns;
  const std::vector<double> fg = mfma_fragments(pf.G.data(), (int)pf.offs.size(), nt, ns);
  const std::vector<double> fd = mfma_fragments(dc.A.data(), (int)dc.offs.size(), ns, nt);
  const std::vector<double> fk = mfma_fragments(kc.A.data(), (int)kc.offs.size(), ns, ns);
  std::vector<float> fgs(fg.begin(), fg.end());
  if (h->brick_ok) {  // taps and halos of the brick kernel
    BrickTaps& b = h->brick;
    b = BrickTaps{};
    b.ng = (int)pf.offs.size();
    b.nd = (int)dc.offs.size();
    if (b.ng > 8 || b.nd > 4) return fail(RIDG_E_UNSUPPORTED, "brick kernel tap count");
    for (int i = 0; i < 3; ++i) {
      int glo = 0, ghi = 0, dlo = 0, dhi = 0;
      for (int t = 0; t < b.ng; ++t) {
        b.g[t][i] = (int8_t)pf.offs[t][i];
        glo = std::min(glo, pf.offs[t][i]);
        ghi = std::max(ghi, pf.offs[t][i]);
      }
      for (int t = 0; t < b.nd; ++t) {
        b.d[t][i] = (int8_t)dc.offs[t][i];
        dlo = std::min(dlo, dc.offs[t][i]);
        dhi = std::max(dhi, dc.offs[t][i]);
      }
      b.wlo[i] = (int8_t)dlo;
      b.whi[i] = (int8_t)dhi;
      b.qlo[i] = (int8_t)(dlo + glo);
      b.qhi[i] = (int8_t)(dhi + ghi);
    }
  }
  int err = hipMemcpyAsync(h->G, pf.G.data(), pf.G.size() * 8, hipMemcpyHostToDevice, h->stream);
  if (!err) err = hipMemcpyAsync(h->Dc, dc.A.data(), dc.A.size() * 8, hipMemcpyHostToDevice, h->stream);
  if (!err) err = hipMemcpyAsync(h->Kc, kc.A.data(), kc.A.size() * 8, hipMemcpyHostToDevice, h->stream);
  if (!err) err = hipMemcpyAsync(h->Fg, fg.data(), fg.size() * 8, hipMemcpyHostToDevice, h->stream);
  if (!err) err = hipMemcpyAsync(h->Fd, fd.data(), fd.size() * 8, hipMemcpyHostToDevice, h->stream);
  if (!err) err = hipMemcpyAsync(h->Fk, fk.data(), fk.size() * 8, hipMemcpyHostToDevice, h->stream);
  if (!err) err = hipMemcpyAsync(h->Fgs, fgs.data(), fgs.size() * 4, hipMemcpyHostToDevice, h->stream);
  if (!err) err = hipStreamSynchronize(h->stream);
  if (err) return hip_fail(err, "upload of the prefactored operators");
  h->g_dt = dt;
  return RIDG_OK;
}

static int record_event(ridg_t* h) {
  if (h->ev_used == h->events.size()) {
    hipEvent_t e;
    int err = hipEventCreate(&e);
    if (err) return err;
    h->events.push_back(e);
  }
  return hipEventRecord(h->events[h->ev_used++], h->stream);
}

static int run_predict(ridg_t* h, const double* Q, double dt) {
  const Problem& P = h->P;
  int err = 0;
  if (P.solver == RIDG_SOLVER_NEWTON) {
    err = launch_burgers_predict(P.d, P.M, h->geom, dt, Q, h->W, h->bd, P.nel, P.newton_max, h->nstats, h->stream);
  } else if (P.solver == RIDG_SOLVER_PREFACTORED) {
    err = launch_predict_prefactored(P.d, P.M, h->geom, Q, h->W, h->G, h->host_taps.data(), h->ntaps, h->stream);
  } else if (P.solver == RIDG_SOLVER_REGION) {
    // cyclic regions (tear and dense kernels) run beside the plan kernel on a forked stream
    const bool side = h->L.n_dense || h->L.n_tear;
    // the static-pivot layout runs where elimination in natural order was measured stable for this
    // dt, else the partial-pivoting layout of the same geometry (FP64) or the packed one (FP32)
    int lay = h->opt_layout;
    if (lay == kStaticPivotLayout && !h->sp_ok) lay = P.precision == RIDG_FP64 ? 4 : 1;
    const bool fork = side && h->L.n_items[lay] && h->aux;
    hipStream_t ss = fork ? h->aux : h->stream;
    if (fork) {
      err = hipEventRecord(h->fork_ev, h->stream);
      if (!err) err = hipStreamWaitEvent(h->aux, h->fork_ev, 0);
    }
    // the few cyclic regions are queued first, so their workgroups are dispatched before the
    // plan kernel's fill the chip (each is a long dependency chain on a handful of CUs)
    if (!err && h->L.n_tear)
      err = launch_predict_tear(P.d, P.M, h->geom, dt, Q, h->W, h->pt, h->tplans, h->telems, h->L.n_tear, ss);
    if (!err && h->L.n_dense)
      err = launch_predict_dense(P.d, P.M, h->geom, dt, Q, h->W, h->dt, h->dense, h->L.n_dense, h->scratch,
                                 h->L.scratch_elems, ss);
    if (!err && h->L.n_items[lay])
      err = launch_predict_plans(P.d, P.M, lay, P.precision, P.refine, h->geom, dt, Q, h->W, h->pt, h->plans,
                                 h->items[lay], h->item_plan[lay], h->L.n_items[lay], h->stream);
    if (!err && fork) err = hipEventRecord(h->join_ev, h->aux);
    if (!err && fork) err = hipStreamWaitEvent(h->stream, h->join_ev, 0);
  } else {
    err = launch_predict_dense(P.d, P.M, h->geom, dt, Q, h->W, h->dt, h->dense, h->L.n_dense, h->scratch,
                               h->L.scratch_elems, h->stream);
  }
  return err ? hip_fail(err, "prediction launch") : RIDG_OK;
}

static int direct_step(ridg_t* h, double dt) {
  const Problem& P = h->P;
  const bool pref = P.solver == RIDG_SOLVER_PREFACTORED;
  if (h->timing) {
    int err = record_event(h);
    if (err) return hip_fail(err, "timing event");
  }
  const int nk = (int)h->host_ktaps.size() / 3, nd = (int)h->host_dtaps.size() / 3;
  const bool mfma = h->opt_mfma != 0;
  const bool f32 = P.precision == RIDG_FP32_REFINE;
  if (pref && (h->opt_brick || f32)) {  // fused brick step: matrix-core predictions, FP64 correction
    int err = launch_brick_step(P.M, f32, h->geom, h->Q[h->cur], h->Q[1 - h->cur],
                                f32 ? (const void*)h->Fgs : (const void*)h->Fg, h->Dc, h->brick, h->stream);
    if (err) return hip_fail(err, "brick step launch");
    if (h->timing) {  // one fused launch: the correction stage is empty
      err = record_event(h);
      if (!err) err = record_event(h);
      if (err) return hip_fail(err, "timing event");
    }
    h->cur ^= 1;
    return RIDG_OK;
  }
  if (pref && h->opt_composite && P.basis == RIDG_BASIS_Q) {
    int err = launch_tap_composite_ns(P.d, h->T.ns, h->geom, h->Q[h->cur], h->Q[1 - h->cur], h->Kc,
                                      h->host_ktaps.data(), nk, h->stream);
    if (err) return hip_fail(err, "composite launch");
  } else if (pref && h->opt_composite == 2) {  // the same stencil marched along z through LDS
    int err = launch_tap_zmarch(h->T.ns, h->geom, h->Q[h->cur], h->Q[1 - h->cur], h->Kc, h->host_ktaps.data(), nk,
                                h->stream);
    if (err) return hip_fail(err, "z-marched composite launch");
  } else if (pref && h->opt_composite) {  // prediction and correction composed into one stencil
    const bool z2 = !mfma && z2_supported(P.d, h->T.ns, P.n[2]);  // 3D: two z-neighbours per thread
    int err = mfma ? launch_tap_mfma(P.d, P.M, kMfmaComposite, h->geom, h->Q[h->cur], h->Q[h->cur],
                                            h->Q[1 - h->cur], h->Fk, h->host_ktaps.data(), nk, h->stream)
              : z2 ? launch_tap_z2(h->T.ns, h->geom, h->Q[h->cur], h->Q[1 - h->cur], h->Kc, h->host_ktaps.data(), nk,
                                   h->stream)
                          : launch_tap_update(P.d, P.M, 1, h->geom, h->Q[h->cur], h->Q[h->cur], h->Q[1 - h->cur],
                                              h->Kc, h->host_ktaps.data(), nk, h->stream);
    if (err) return hip_fail(err, "composite launch");
  } else if (pref && mfma) {
    int err = launch_tap_mfma(P.d, P.M, kMfmaPredict, h->geom, h->Q[h->cur], nullptr, h->W, h->Fg,
                              h->host_taps.data(), h->ntaps, h->stream);
    if (err) return hip_fail(err, "prediction launch");
  } else {
    int rc = run_predict(h, h->Q[h->cur], dt);
    if (rc) return rc;
  }
  if (h->timing) {
    int err = record_event(h);
    if (err) return hip_fail(err, "timing event");
  }
  int err = 0;
  if (pref && !h->opt_composite && mfma)
    err = launch_tap_mfma(P.d, P.M, kMfmaCorrect, h->geom, h->W, h->Q[h->cur], h->Q[1 - h->cur], h->Fd,
                          h->host_dtaps.data(), nd, h->stream);
  else if (pref && !h->opt_composite)
    err = launch_tap_update(P.d, P.M, 0, h->geom, h->W, h->Q[h->cur], h->Q[1 - h->cur], h->Dc, h->host_dtaps.data(),
                            nd, h->stream);
  else if (P.solver == RIDG_SOLVER_NEWTON)
    err = launch_burgers_correct(P.d, P.M, h->geom, dt, h->Q[h->cur], h->W, h->Q[1 - h->cur], h->bd, h->stream);
  else if (!pref)
    err = launch_correct(P.d, P.M, P.flux, h->geom, dt, h->Q[h->cur], h->W, h->Q[1 - h->cur], h->dt, h->stream);
  if (err) return hip_fail(err, "correction launch");
  if (h->timing) {
    err = record_event(h);
    if (err) return hip_fail(err, "timing event");
  }
  h->cur ^= 1;
  return RIDG_OK;
}

static void drop_graphs(ridg_t* h) {
  for (int p = 0; p < 2; ++p)
    if (h->graph[p]) {
      (void)hipGraphExecDestroy(h->graph[p]);
      h->graph[p] = nullptr;
    }
  h->graph_dt = -1.0;
}

// Capture two consecutive steps starting from state buffer `parity` into an executable graph.
// The captured work contains kernels and event record/wait nodes only (no memset nodes).
static int capture_graph(ridg_t* h, double dt, int parity) {
  // capture on an internal stream (the caller's stream may be the legacy default stream, which
  // cannot be captured); the graph is then launched on the caller's stream
  if (!h->cap) {
    int e = hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking);
    if (e) return hip_fail(e, "capture stream");
  }
  const int saved = h->cur;
  const bool saved_timing = h->timing;
  hipStream_t user = h->stream;
  h->timing = false;
  h->cur = parity;
  h->stream = h->cap;
  int err = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
  int rc = RIDG_OK;
  if (!err) {
    rc = direct_step(h, dt);
    if (!rc) rc = direct_step(h, dt);
    hipGraph_t g = nullptr;
    err = hipStreamEndCapture(h->cap, &g);
    if (!err && !rc) err = hipGraphInstantiate(&h->graph[parity], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
  }
  h->stream = user;
  h->cur = saved;
  h->timing = saved_timing;
  if (rc) return rc;
  return err ? hip_fail(err, "graph capture") : RIDG_OK;
}

int ridg_step(ridg_t* h, int32_t n_steps, double dt) {
  if (!h) return fail(RIDG_E_INVAL, "handle is NULL");
  if (n_steps < 0) return fail(RIDG_E_INVAL, "n_steps must be >= 0");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RIDG_E_INVAL, "dt must be positive and finite");
  if (n_steps == 0) return RIDG_OK;
  if (h->P.solver == RIDG_SOLVER_REGION && h->P.d == 3 && h->T.nt > 64)
    return fail(RIDG_E_UNSUPPORTED, "REGION solver supports theta_T <= 64");
  int rc = ensure_dt_tables(h, dt);
  if (rc) return rc;
  const int warn = stability_warning(h, dt);
  if (warn < 0) return warn;
  if (h->opt_fused && !h->timing && h->P.solver == RIDG_SOLVER_PREFACTORED && h->P.precision == RIDG_FP64 &&
      fused_fits(h->P.d, h->P.M, h->P.nel)) {
    int err = launch_fused_prefactored(h->P.d, h->P.M, h->geom, dt, h->Q[h->cur], h->Q[1 - h->cur], h->G,
                                       h->host_taps.data(), h->ntaps, h->dt, n_steps, h->stream);
    if (err) return hip_fail(err, "fused launch");
    h->cur ^= 1;
    return warn;
  }
  if (h->opt_composite == 3 && !h->timing && n_steps >= kTBlockSteps) {  // kTBlockSteps steps per launch
    const int nk = (int)h->host_ktaps.size() / 3;
    if (!tblock_taps_supported(h->host_ktaps.data(), nk))
      return fail(RIDG_E_UNSUPPORTED, "the composite taps reach beyond the temporally blocked kernel's window");
    while (n_steps >= kTBlockSteps) {
      int err = launch_tap_tblock(h->T.ns, h->geom, h->Q[h->cur], h->Q[1 - h->cur], h->Kc, h->host_ktaps.data(), nk,
                                  h->stream);
      if (err) return hip_fail(err, "temporally blocked composite launch");
      h->cur ^= 1;
      n_steps -= kTBlockSteps;
    }
  }
  if (h->opt_graph && !h->timing && n_steps >= 2) {
    if (h->graph_dt != dt) drop_graphs(h);
    h->graph_dt = dt;
    while (n_steps >= 2) {
      if (!h->graph[h->cur]) {
        rc = capture_graph(h, dt, h->cur);
        if (rc) return rc;
      }
      int err = hipGraphLaunch(h->graph[h->cur], h->stream);
      if (err) return hip_fail(err, "graph launch");
      n_steps -= 2;  // two steps: the state returns to the same buffer
    }
  }
  for (int s = 0; s < n_steps; ++s) {
    rc = direct_step(h, dt);
    if (rc) return rc;
  }
  return warn;
}

int ridg_step_batch(ridg_t* const* handles, int32_t count, const double* dts, int32_t n_steps, void* hip_stream) {
  if (count < 0 || n_steps < 0) return fail(RIDG_E_INVAL, "count and n_steps must be >= 0");
  if (count == 0 || n_steps == 0) return RIDG_OK;
  if (!handles || !dts) return fail(RIDG_E_INVAL, "NULL argument");
  for (int i = 0; i < count; ++i) {
    ridg_t* h = handles[i];
    if (!h) return fail(RIDG_E_INVAL, "NULL handle in the batch");
    if (h->P.solver != RIDG_SOLVER_PREFACTORED || h->P.precision != RIDG_FP64 || h->P.basis != RIDG_BASIS_P)
      return fail(RIDG_E_UNSUPPORTED, "batched steps need FP64 PREFACTORED handles");
    if (!(dts[i] > 0.0) || !std::isfinite(dts[i])) return fail(RIDG_E_INVAL, "dt must be positive and finite");
    for (int j = 0; j < i; ++j)
      if (handles[j] == h) return fail(RIDG_E_INVAL, "a handle appears twice in the batch");
  }
  // a handle whose dt changed gets new operators; earlier batched launches on hip_stream may still
  // read the old ones, so the upload waits for them (not needed for operators no batch has read)
  bool rebuild = false;
  for (int i = 0; i < count; ++i) rebuild = rebuild || (handles[i]->g_dt != dts[i] && handles[i]->batch_dt >= 0.0);
  if (rebuild) {
    int err = hipStreamSynchronize((hipStream_t)hip_stream);
    if (err) return hip_fail(err, "hipStreamSynchronize before the operator upload");
  }
  for (int i = 0; i < count; ++i) {
    int rc = ensure_dt_tables(handles[i], dts[i]);
    if (rc) return rc;
    if (handles[i]->ntaps > kBatchTaps) return fail(RIDG_E_UNSUPPORTED, "more than 8 taps");
  }
  // families: same (dim, order, matrix-core option); a handle steps with the kernels it would use alone
  std::vector<std::vector<int>> fam;
  for (int i = 0; i < count; ++i) {
    bool placed = false;
    for (auto& f : fam)
      if (handles[f[0]]->P.d == handles[i]->P.d && handles[f[0]]->P.M == handles[i]->P.M &&
          (handles[f[0]]->opt_mfma != 0) == (handles[i]->opt_mfma != 0)) {
        f.push_back(i);
        placed = true;
        break;
      }
    if (!placed) fam.push_back({i});
  }
  for (int s = 0; s < n_steps; ++s) {
    for (auto& f : fam) {
      const ridg_t* h0 = handles[f[0]];
      if (h0->opt_mfma) {  // prediction, then correction, each one launch per chunk of problems
        for (size_t c0 = 0; c0 < f.size(); c0 += kBatchMax) {
          for (int kind : {kMfmaPredict, kMfmaCorrect}) {
            BatchMfmaArgs args{};
            int64_t groups = 0;
            for (size_t c = c0; c < f.size() && c < c0 + kBatchMax; ++c) {
              ridg_t* h = handles[f[c]];
              BatchMfmaDesc& d = args.d[args.count++];
              const bool pred = kind == kMfmaPredict;
              d.in = pred ? h->Q[h->cur] : h->W;
              d.base = pred ? nullptr : h->Q[h->cur];
              d.out = pred ? h->W : h->Q[1 - h->cur];
              d.frag = pred ? h->Fg : h->Fd;
              const std::vector<int32_t>& tl = pred ? h->host_taps : h->host_dtaps;
              d.ntaps = (int32_t)tl.size() / 3;
              for (int t = 0; t < d.ntaps && t < kBatchTaps; ++t)
                for (int i = 0; i < 3; ++i) d.taps[t][i] = (int8_t)tl[3 * t + i];
              for (int i = 0; i < 3; ++i) d.n[i] = h->P.n[i];
              d.tiles_per_group = mfma_tiles_per_group(h->P.nel, 0);
              d.group_begin = groups;
              groups += ((h->P.nel + 15) / 16 + d.tiles_per_group - 1) / d.tiles_per_group;
            }
            int err = launch_batch_mfma(h0->P.d, h0->P.M, kind, args, groups, hip_stream);
            if (err) return hip_fail(err, "batched MFMA launch");
          }
        }
        continue;
      }
      for (size_t c0 = 0; c0 < f.size(); c0 += kBatchMax) {
        BatchArgs args{};
        int64_t blk = 0;
        for (size_t c = c0; c < f.size() && c < c0 + kBatchMax; ++c) {
          ridg_t* h = handles[f[c]];
          BatchDesc& d = args.d[args.count++];
          d.Qin = h->Q[h->cur];
          d.Qout = h->Q[1 - h->cur];
          d.W = h->W;
          d.G = h->G;
          d.Dc = h->Dc;
          d.ndtaps = (int32_t)h->host_dtaps.size() / 3;
          for (int t = 0; t < d.ndtaps && t < 7; ++t)
            for (int i = 0; i < 3; ++i) d.dtaps[t][i] = (int8_t)h->host_dtaps[3 * t + i];
          d.block_begin = blk;
          d.nel = h->P.nel;
          for (int i = 0; i < 3; ++i) {
            d.h[i] = h->P.h[i];
            d.v[i] = h->P.vel.a[i];
            d.n[i] = h->P.n[i];
          }
          d.dt = dts[f[c]];
          d.ntaps = h->ntaps;
          for (int t = 0; t < h->ntaps; ++t)
            for (int i = 0; i < 3; ++i) d.taps[t][i] = (int8_t)h->host_taps[3 * t + i];
          blk += (h->P.nel + 255) / 256;
        }
        int err = launch_batch_step(h0->P.d, h0->P.M, args, h0->dt, hip_stream);
        if (err) return hip_fail(err, "batched step launch");
      }
    }
    for (int i = 0; i < count; ++i) handles[i]->cur ^= 1;
  }
  for (int i = 0; i < count; ++i) handles[i]->batch_dt = dts[i];
  return RIDG_OK;
}

int ridg_set_option(ridg_t* h, int32_t option, int64_t value) {
  if (!h) return fail(RIDG_E_INVAL, "handle is NULL");
  const int64_t vmax = option == RIDG_OPT_PLAN_LAYOUT ? kLayouts - 1 : (option == RIDG_OPT_COMPOSITE ? 3 : 1);
  if (value < 0 || value > vmax) return fail(RIDG_E_INVAL, "option value out of range");
  if (h->P.solver == RIDG_SOLVER_NEWTON && value)
    return fail(RIDG_E_UNSUPPORTED, "RIDG_SOLVER_NEWTON has no execution options");
  if (h->P.basis == RIDG_BASIS_Q && option != RIDG_OPT_GRAPH && value != (option == RIDG_OPT_COMPOSITE ? 1 : 0))
    return fail(RIDG_E_UNSUPPORTED, "the tensor basis runs the composite stencil (RIDG_OPT_COMPOSITE = 1) only");
  int err = hipStreamSynchronize(h->stream);
  if (err) return hip_fail(err, "hipStreamSynchronize");
  switch (option) {
    case RIDG_OPT_GRAPH:
      h->opt_graph = (int)value;
      break;
    case RIDG_OPT_PLAN_LAYOUT:
      if (h->P.solver != RIDG_SOLVER_REGION && value) return fail(RIDG_E_UNSUPPORTED, "plan layout applies to REGION");
      if (value >= 2 && value != kStaticPivotLayout && h->P.precision != RIDG_FP64)
        return fail(RIDG_E_UNSUPPORTED, "plan layouts 2 to 4 are FP64 only");
      h->opt_layout = (int)value;
      break;
    case RIDG_OPT_FUSED:
      if (value && (h->P.solver != RIDG_SOLVER_PREFACTORED || !fused_fits(h->P.d, h->P.M, h->P.nel)))
        return fail(RIDG_E_UNSUPPORTED, "fused steps need the PREFACTORED solver and a mesh that fits in LDS");
      h->opt_fused = (int)value;
      break;
    case RIDG_OPT_COMPOSITE:
      if (value && h->P.solver != RIDG_SOLVER_PREFACTORED)
        return fail(RIDG_E_UNSUPPORTED, "the composite stencil needs the PREFACTORED solver");
      if (value == 2 && !zmarch_supported(h->P.d, h->T.ns, h->P.n[0], h->P.n[1], h->P.n[2]))
        return fail(RIDG_E_UNSUPPORTED, "the z-marched composite stencil needs 3D, order 2-3, n[0] and n[1] multiples "
                                        "of 16 and n[2] a multiple of 8 (or at most 64)");
      if (value == 3 && (h->P.precision != RIDG_FP64 || !tblock_shape_supported(h->P.d, h->T.ns, h->P.n[0], h->P.n[1])))
        return fail(RIDG_E_UNSUPPORTED, "the temporally blocked composite stencil needs 2D, FP64 and n[0], n[1] "
                                        "multiples of 16");
      h->opt_composite = (int)value;
      break;
    case RIDG_OPT_MFMA:
      if (value && h->P.solver != RIDG_SOLVER_PREFACTORED)
        return fail(RIDG_E_UNSUPPORTED, "the MFMA tap kernels need the PREFACTORED solver");
      h->opt_mfma = (int)value;
      break;
    case RIDG_OPT_BRICK:
      if (value && !h->brick_ok)
        return fail(RIDG_E_UNSUPPORTED,
                    "the brick kernel needs the PREFACTORED solver, 3D, order 2-3 and a brick-divisible mesh");
      h->opt_brick = (int)value;
      break;
    default:
      return fail(RIDG_E_INVAL, "unknown option");
  }
  drop_graphs(h);
  return RIDG_OK;
}

int ridg_get_option(ridg_t* h, int32_t option, int64_t* value) {
  if (!h || !value) return fail(RIDG_E_INVAL, "NULL argument");
  switch (option) {
    case RIDG_OPT_GRAPH: *value = h->opt_graph; return RIDG_OK;
    case RIDG_OPT_PLAN_LAYOUT: *value = h->opt_layout; return RIDG_OK;
    case RIDG_OPT_FUSED: *value = h->opt_fused; return RIDG_OK;
    case RIDG_OPT_COMPOSITE: *value = h->opt_composite; return RIDG_OK;
    case RIDG_OPT_MFMA: *value = h->opt_mfma; return RIDG_OK;
    case RIDG_OPT_BRICK: *value = h->opt_brick; return RIDG_OK;
    default: return fail(RIDG_E_INVAL, "unknown option");
  }
}


int ridg_autotune(ridg_t* h, double dt, int32_t steps, double* best_ms_per_step) {
  if (!h) return fail(RIDG_E_INVAL, "handle is NULL");
  if (steps < 2 || steps > 100000) return fail(RIDG_E_INVAL, "steps must be in 2..100000");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RIDG_E_INVAL, "dt must be positive and finite");
  if (h->timing) return fail(RIDG_E_INVAL, "switch stage timing off before autotuning");
  if (h->P.solver == RIDG_SOLVER_NEWTON) return fail(RIDG_E_UNSUPPORTED, "RIDG_SOLVER_NEWTON has no options to tune");
  if (h->P.basis == RIDG_BASIS_Q) return fail(RIDG_E_UNSUPPORTED, "the tensor basis has no options to tune");
  const std::string key = tune_key(h, steps);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_file_load();
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      h->opt_graph = it->second[0];
      h->opt_layout = it->second[1];
      h->opt_fused = it->second[2];
      h->opt_composite = it->second[3];
      h->opt_mfma = it->second[4];
      h->opt_brick = it->second[5];
      drop_graphs(h);
      if (best_ms_per_step) *best_ms_per_step = -1.0;  // from the cache, not re-measured
      return RIDG_OK;
    }
  }
  std::vector<std::array<int, 6>> cands;
  const bool region = h->P.solver == RIDG_SOLVER_REGION;
  const bool pref = h->P.solver == RIDG_SOLVER_PREFACTORED;
  const bool fusable = pref && fused_fits(h->P.d, h->P.M, h->P.nel);
  {
    int rc0 = ensure_dt_tables(h, dt);  // the static-pivot check needs this dt's tables
    if (rc0) return rc0;
  }
  std::vector<int> layouts = {0};
  if (region) {
    layouts = h->P.precision == RIDG_FP64 ? std::vector<int>{0, 1, 2, 3, 4} : std::vector<int>{0, 1};
    if (h->sp_ok) layouts.push_back(kStaticPivotLayout);
  }
  const bool f32_brick = pref && h->P.precision == RIDG_FP32_REFINE;  // the brick kernel is this path
  for (int g = 0; g < 2; ++g) {
    if (f32_brick) {
      cands.push_back({g, 0, 0, 0, 0, 1});
      continue;
    }
    for (int l : layouts)
      for (int c = 0; c < (pref ? 2 : 1); ++c)
        for (int m = 0; m < (pref ? 2 : 1); ++m) cands.push_back({g, l, 0, c, m, 0});
    if (pref && zmarch_supported(h->P.d, h->T.ns, h->P.n[0], h->P.n[1], h->P.n[2])) cands.push_back({g, 0, 0, 2, 0, 0});
    if (pref && h->P.precision == RIDG_FP64 && tblock_shape_supported(h->P.d, h->T.ns, h->P.n[0], h->P.n[1]) &&
        tblock_taps_supported(h->host_ktaps.data(), (int)h->host_ktaps.size() / 3))
      cands.push_back({g, 0, 0, 3, 0, 0});
    if (h->brick_ok) cands.push_back({g, 0, 0, 0, 0, 1});
  }
  if (fusable && !f32_brick) cands.push_back({0, 0, 1, 0, 0, 0});
  // keep the state: tuning steps run on a copy that is restored afterwards
  const size_t bytes = (size_t)h->P.nel * h->T.ns * 8;
  const int cur0 = h->cur;
  int err = hipMemcpyAsync(h->stage, h->Q[cur0], bytes, hipMemcpyDeviceToDevice, h->stream);
  std::array<int, 6> pick = {h->opt_graph, h->opt_layout, h->opt_fused, h->opt_composite, h->opt_mfma, h->opt_brick};
  int rc = RIDG_OK;
  // two sweeps over the candidates, each keeping its faster time: the first candidates of a single
  // sweep would run while the clocks still ramp up
  std::vector<double> cand_ms(cands.size(), 1e300);
  for (size_t it = 0; it < 2 * cands.size() && !err && !rc; ++it) {
    const size_t c = it % cands.size();
    h->opt_graph = cands[c][0];
    h->opt_layout = cands[c][1];
    h->opt_fused = cands[c][2];
    h->opt_composite = cands[c][3];
    h->opt_mfma = cands[c][4];
    h->opt_brick = cands[c][5];
    drop_graphs(h);
    rc = ridg_step(h, 2, dt);  // warm-up (and graph capture)
    if (rc < 0) break;
    rc = RIDG_OK;
    // host clock around a synchronised run: what a caller waits for, launch and graph overheads
    // included (events on the stream have ranked graph replays ahead of slower wall times)
    // Steps of a few microseconds: the run is lengthened (4x at a time, up to 64x) until it lasts
    // 2 ms, so that the synchronisation's own cost does not decide the ranking.
    for (int n = steps; !err && !rc;) {
      err = hipStreamSynchronize(h->stream);
      const auto t0 = std::chrono::steady_clock::now();
      if (!err) rc = ridg_step(h, n, dt);
      if (rc < 0) break;
      rc = RIDG_OK;
      if (!err) err = hipStreamSynchronize(h->stream);
      const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      if (err || ms >= 2.0 || n >= 64 * steps) {
        if (!err) cand_ms[c] = std::min(cand_ms[c], ms / n);
        break;
      }
      n *= 4;
    }
    if (rc < 0) break;
    if (!err) err = hipMemcpyAsync(h->Q[cur0], h->stage, bytes, hipMemcpyDeviceToDevice, h->stream);
    h->cur = cur0;
  }
  double best = 1e300;
  for (size_t c = 0; c < cands.size(); ++c)
    if (cand_ms[c] < best) {
      best = cand_ms[c];
      pick = cands[c];
    }
  h->opt_graph = pick[0];
  h->opt_layout = pick[1];
  h->opt_fused = pick[2];
  h->opt_composite = pick[3];
  h->opt_mfma = pick[4];
  h->opt_brick = pick[5];
  drop_graphs(h);
  if (rc < 0) return rc;
  if (err) return hip_fail(err, "autotune");
  err = hipStreamSynchronize(h->stream);
  if (err) return hip_fail(err, "autotune");
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = pick;
    tune_file_append(key, pick);
  }
  if (best_ms_per_step) *best_ms_per_step = best;
  return RIDG_OK;
}

int ridg_get_prediction(ridg_t* h, double dt, double* w, size_t count, int32_t where) {
  if (!h || !w) return fail(RIDG_E_INVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RIDG_E_INVAL, "dt must be positive and finite");
  const size_t want = (size_t)h->P.nel * h->T.nt;
  if (count != want) return fail(RIDG_E_INVAL, "count must equal n_elements * theta_T");
  if (where != RIDG_HOST && where != RIDG_DEVICE) return fail(RIDG_E_INVAL, "where must be RIDG_HOST or RIDG_DEVICE");
  if (h->P.solver == RIDG_SOLVER_REGION && h->P.d == 3 && h->T.nt > 64)
    return fail(RIDG_E_UNSUPPORTED, "REGION solver supports theta_T <= 64");
  if (h->P.basis == RIDG_BASIS_Q)
    return fail(RIDG_E_UNSUPPORTED, "the tensor basis runs the composite stencil, which stores no predictions");
  int rc = ensure_dt_tables(h, dt);
  if (rc) return rc;
  rc = run_predict(h, h->Q[h->cur], dt);
  if (rc) return rc;
  if (where == RIDG_DEVICE)
    return check_hip(launch_soa_to_aos(h->W, w, h->P.nel, h->T.nt, h->stream), "ridg_get_prediction");
  int err = launch_soa_to_aos(h->W, h->stage, h->P.nel, h->T.nt, h->stream);
  if (!err) err = hipMemcpyAsync(w, h->stage, count * 8, hipMemcpyDeviceToHost, h->stream);
  if (!err) err = hipStreamSynchronize(h->stream);
  return check_hip(err, "ridg_get_prediction");
}

int ridg_host_region_matrix(const ridg_problem* problem, int64_t element, double dt, double* a, size_t count) {
  Problem P;
  std::string msg;
  int rc = resolve_problem(problem, &P, &msg);
  if (rc) return fail(rc, msg);
  if (P.flux == RIDG_FLUX_BURGERS) return fail(RIDG_E_INVAL, "the Burgers region system depends on the state");
  if (!a) return fail(RIDG_E_INVAL, "a is NULL");
  if (element < 0 || element >= P.nel) return fail(RIDG_E_INVAL, "element out of range");
  if (!std::isfinite(dt)) return fail(RIDG_E_INVAL, "dt not finite");
  Basis B = make_basis(P.d, P.M, P.basis);
  RefTensors T = make_tensors(B);
  auto offs = region_offsets(P.d);
  const size_t n = offs.size() * T.nt;
  if (count != n * n) return fail(RIDG_E_INVAL, "count must equal (3^d theta_T)^2");
  std::vector<double> A;
  assemble_region(P, T, element, dt, offs, &A);
  std::memcpy(a, A.data(), n * n * 8);
  return RIDG_OK;
}

int ridg_host_spectral_radius(const ridg_problem* problem, double dt, int32_t nk, double* radius) {
  Problem P;
  std::string msg;
  int rc = resolve_problem(problem, &P, &msg);
  if (rc) return fail(rc, msg);
  if (!radius) return fail(RIDG_E_INVAL, "radius is NULL");
  if (P.flux != RIDG_FLUX_CONST) return fail(RIDG_E_INVAL, "the von Neumann analysis needs a constant velocity");
  if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(RIDG_E_INVAL, "dt must be finite and >= 0");
  if (nk < 2 || nk > 4096 || std::pow((double)nk, P.d) > (double)(1 << 22))
    return fail(RIDG_E_INVAL, "nk must be in 2..4096 with at most 2^22 grid points");
  Basis B = make_basis(P.d, P.M, P.basis);
  RefTensors T = make_tensors(B);
  Prefactored pf;
  rc = build_prefactored(P, T, dt, &pf, &msg);
  if (rc) return fail(rc, msg);
  TapOperator dc, kc;
  build_correction_taps(P, T, dt, &dc);
  build_composite(P, pf, dc, &kc);
  *radius = spectral_radius(kc, P.d, nk);
  return RIDG_OK;
}

int ridg_host_prediction_operator(const ridg_problem* problem, double dt, double* g, size_t count) {
  Problem P;
  std::string msg;
  int rc = resolve_problem(problem, &P, &msg);
  if (rc) return fail(rc, msg);
  if (P.flux != RIDG_FLUX_CONST) return fail(RIDG_E_INVAL, "prediction operator needs a constant velocity");
  if (!g) return fail(RIDG_E_INVAL, "g is NULL");
  if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(RIDG_E_INVAL, "dt must be finite and >= 0");
  Basis B = make_basis(P.d, P.M, P.basis);
  RefTensors T = make_tensors(B);
  auto offs = region_offsets(P.d);
  const size_t nb = offs.size(), cols = nb * T.ns;
  if (count != (size_t)T.nt * cols) return fail(RIDG_E_INVAL, "count must equal theta_T * 3^d * theta");
  Prefactored pf;
  rc = build_prefactored(P, T, dt, &pf, &msg);
  if (rc) return fail(rc, msg);
  std::memset(g, 0, count * 8);
  for (size_t t = 0; t < pf.offs.size(); ++t) {
    int code = 0;
    for (int i = 0; i < P.d; ++i) code = code * 3 + (pf.offs[t][i] + 1);
    for (int k = 0; k < T.nt; ++k)
      for (int l = 0; l < T.ns; ++l)
        g[(size_t)k * cols + (size_t)code * T.ns + l] = pf.G[((size_t)t * T.nt + k) * T.ns + l];
  }
  return RIDG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- Jacobian assembly comparison (Sec. 3)
namespace {
struct AsmEntry {
  int dev, d, M;
  void* mem;  // one device block: doubles (psiv, projw, dsum, bval) then int32 (rptr, bp)
  AsmDev view;
};
std::mutex g_asm_mu;
std::vector<AsmEntry> g_asm;  // device tables per (device, dim, order), kept until the process ends

int asm_tables(int d, int M, AsmDev* out) {
  int dev = 0;
  int err = hipGetDevice(&dev);
  if (err) return hip_fail(err, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_asm_mu);
  for (const AsmEntry& a : g_asm)
    if (a.dev == dev && a.d == d && a.M == M) {
      *out = a.view;
      return RIDG_OK;
    }
  AsmHost H;
  std::string msg;
  int rc = build_assembly_tables(d, M, &H, &msg);
  if (rc) return fail(rc, msg);
  const size_t nd = H.psiv.size() + H.projw.size() + H.dsum.size() + H.bval.size();
  const size_t ni = H.rptr.size() + H.bp.size();
  void* mem = nullptr;
  err = hipMalloc(&mem, nd * 8 + ni * 4);
  if (err) return hip_fail(err, "hipMalloc of the assembly tables");
  std::vector<char> buf(nd * 8 + ni * 4);
  AsmDev v{};
  v.nt = H.nt;
  v.nq = H.nq;
  size_t off = 0;
  auto putd = [&](const std::vector<double>& x) {
    std::memcpy(buf.data() + off, x.data(), x.size() * 8);
    const double* at = (const double*)((char*)mem + off);
    off += x.size() * 8;
    return at;
  };
  auto puti = [&](const std::vector<int32_t>& x) {
    std::memcpy(buf.data() + off, x.data(), x.size() * 4);
    const int32_t* at = (const int32_t*)((char*)mem + off);
    off += x.size() * 4;
    return at;
  };
  v.psiv = putd(H.psiv);
  v.projw = putd(H.projw);
  v.dsum = putd(H.dsum);
  v.bval = putd(H.bval);
  v.rptr = puti(H.rptr);
  v.bp = puti(H.bp);
  err = hipMemcpy(mem, buf.data(), buf.size(), hipMemcpyHostToDevice);
  if (err) {
    (void)hipFree(mem);
    return hip_fail(err, "upload of the assembly tables");
  }
  g_asm.push_back({dev, d, M, mem, v});
  *out = v;
  return RIDG_OK;
}
}  // namespace

extern "C" int ridg_assemble_jacobian(int32_t method, int32_t dim, int32_t order, const double* w, int64_t n_elements,
                                      double dt_over_h, double* jac, void* hip_stream) {
  if (method < RIDG_ASM_QUADRATURE || method > RIDG_ASM_PERTURBATION) return fail(RIDG_E_INVAL, "unknown method");
  if (dim < 1 || dim > 3 || order < 1 || order > 6) return fail(RIDG_E_INVAL, "dim must be 1..3 and order 1..6");
  if (n_elements < 0 || n_elements > ((int64_t)1 << 31)) return fail(RIDG_E_INVAL, "n_elements out of range");
  if (n_elements > 0 && (!w || !jac)) return fail(RIDG_E_INVAL, "NULL array");
  if (!std::isfinite(dt_over_h)) return fail(RIDG_E_INVAL, "dt_over_h not finite");
  AsmDev t{};
  int rc = asm_tables(dim, order, &t);
  if (rc) return rc;
  int err = launch_assembly(method, t, n_elements, w, dt_over_h, jac, hip_stream);
  return err ? hip_fail(err, "assembly launch") : RIDG_OK;
}
