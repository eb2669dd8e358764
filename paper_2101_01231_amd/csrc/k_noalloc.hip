// Allocation-free whole-step entry point (ridg_advance_static): constant-velocity RIDG steps
// (prediction with the prefactored operator, Sec. 2.2; correction, Sec. 2.3) whose intermediates
// live in one file-scope device array instead of a caller-provided workspace. For callers that
// cannot allocate device memory (code under stream capture, serving loops with a fixed memory plan).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "kernels_common.hpp"

namespace ridg {
namespace {

constexpr size_t kStaticScratchBytes = (size_t)64 << 20;  // per device, held until the process ends
constexpr int kMaxDevices = 64;

// The array's name is a host-side stand-in: host code uses only the device address obtained from
// hipGetSymbolAddress below (one per device).
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

int scratch_address(void** out, std::string* msg) {
  int dev = 0;
  int err = (int)hipGetDevice(&dev);
  if (err) {
    *msg = std::string("hipGetDevice: ") + hipGetErrorString((hipError_t)err);
    return RIDG_E_DEVICE;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    *msg = "device index out of range";
    return RIDG_E_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    err = (int)hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err || !p) {
      *msg = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString((hipError_t)err);
      return RIDG_E_DEVICE;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return RIDG_OK;
}

// Host FP64 operators of one (problem, dt), kept so that repeated calls do not refactorise.
struct StaticOps {
  std::string key;
  std::vector<double> G, Dc;
  std::vector<int32_t> taps, dtaps;
};
std::deque<std::shared_ptr<const StaticOps>> g_ops;  // most recent first, at most kOpsCache entries
constexpr size_t kOpsCache = 32;

std::string ops_key(const Problem& P, double dt) {
  std::string k;
  auto add = [&](const void* p, size_t n) { k.append((const char*)p, n); };
  add(&P.d, sizeof(P.d));
  add(P.n, sizeof(P.n));
  add(&P.M, sizeof(P.M));
  add(P.vel.a, sizeof(P.vel.a));
  add(P.h, sizeof(P.h));
  add(&dt, sizeof(dt));
  return k;
}

int static_ops(const Problem& P, double dt, std::shared_ptr<const StaticOps>* out, std::string* msg) {
  const std::string key = ops_key(P, dt);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& o : g_ops)
      if (o->key == key) {
        *out = o;
        return RIDG_OK;
      }
  }
  Basis B = make_basis(P.d, P.M);
  RefTensors T = make_tensors(B);
  Prefactored pf;
  int rc = build_prefactored(P, T, dt, &pf, msg);
  if (rc) return rc;
  TapOperator dc;
  build_correction_taps(P, T, dt, &dc);
  auto o = std::make_shared<StaticOps>();
  o->key = key;
  o->G = pf.G;
  o->Dc = dc.A;
  for (const auto& t : pf.offs) o->taps.insert(o->taps.end(), {t[0], t[1], t[2]});
  for (const auto& t : dc.offs) o->dtaps.insert(o->dtaps.end(), {t[0], t[1], t[2]});
  std::lock_guard<std::mutex> lk(g_mu);
  g_ops.push_front(o);
  if (g_ops.size() > kOpsCache) g_ops.pop_back();
  *out = o;
  return RIDG_OK;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int static_fail(int code, const std::string& msg) { return set_last_error(code, msg); }

}  // namespace

// Scratch bytes ridg_advance_static needs: two coefficient-major states, the predictions, the
// prediction operator G (taps x theta_T x theta) and the correction taps (<= 7 x theta x theta_T).
size_t static_scratch_bytes(const Problem& P, int ns, int nt, int ntaps, int ndtaps) {
  return align256((size_t)P.nel * ns * 8) * 2 + align256((size_t)P.nel * nt * 8) +
         align256((size_t)ntaps * nt * ns * 8) + align256((size_t)ndtaps * ns * nt * 8);
}

}  // namespace ridg

using namespace ridg;

extern "C" int ridg_advance_static(const ridg_problem* problem, const double* q_in, double* q_out, size_t count,
                                   int32_t n_steps, double dt, void* hip_stream) {
  Problem P;
  std::string msg;
  int rc = resolve_problem(problem, &P, &msg);
  if (rc) return static_fail(rc, msg);
  if (P.flux != RIDG_FLUX_CONST || P.solver != RIDG_SOLVER_PREFACTORED || P.precision != RIDG_FP64 ||
      P.basis != RIDG_BASIS_P)
    return static_fail(RIDG_E_UNSUPPORTED, "ridg_advance_static runs constant-velocity FP64 problems (PREFACTORED, total-degree basis)");
  if (!q_in || !q_out) return static_fail(RIDG_E_INVAL, "NULL state pointer");
  const int ns = n_space(P.d, P.M), nt = n_spacetime(P.d, P.M);
  if (count != (size_t)P.nel * ns) return static_fail(RIDG_E_INVAL, "count must equal n_elements * theta");
  if (n_steps < 0) return static_fail(RIDG_E_INVAL, "n_steps must be >= 0");
  if (!(dt > 0.0) || !std::isfinite(dt)) return static_fail(RIDG_E_INVAL, "dt must be positive and finite");
  const int max_taps = P.d == 1 ? 2 : (P.d == 2 ? 4 : 8);  // upwind cone: at most 2^d taps, 1 + d correction taps
  const size_t need = static_scratch_bytes(P, ns, nt, max_taps, 1 + P.d);
  if (need > kStaticScratchBytes) {
    char buf[192];
    std::snprintf(buf, sizeof(buf), "the problem needs %zu bytes of scratch; the static scratch holds %zu",
                  need, kStaticScratchBytes);
    return static_fail(RIDG_E_NOMEM, buf);
  }
  hipStream_t stream = (hipStream_t)hip_stream;
  if (n_steps == 0) {
    if (q_out == q_in) return RIDG_OK;
    int err = (int)hipMemcpyAsync(q_out, q_in, count * 8, hipMemcpyDeviceToDevice, stream);
    return err ? static_fail(RIDG_E_DEVICE, hipGetErrorString((hipError_t)err)) : RIDG_OK;
  }
  std::shared_ptr<const StaticOps> ops;
  rc = static_ops(P, dt, &ops, &msg);
  if (rc) return static_fail(rc, msg);
  void* base = nullptr;
  rc = scratch_address(&base, &msg);
  if (rc) return static_fail(rc, msg);
  // carve the scratch: operators first, then the states and the predictions
  char* p = (char*)base;
  double* G = (double*)p;
  p += align256(ops->G.size() * 8);
  double* Dc = (double*)p;
  p += align256(ops->Dc.size() * 8);
  double* Q[2];
  Q[0] = (double*)p;
  p += align256((size_t)P.nel * ns * 8);
  Q[1] = (double*)p;
  p += align256((size_t)P.nel * ns * 8);
  double* W = (double*)p;
  const DevGeom g = [&] {
    DevGeom x{};
    x.d = P.d;
    x.n0 = P.n[0];
    x.n1 = P.n[1];
    x.n2 = P.n[2];
    x.h0 = P.h[0];
    x.h1 = P.h[1];
    x.h2 = P.h[2];
    for (int i = 0; i < 3; ++i) x.a[i] = P.vel.a[i];
    return x;
  }();
  const int ntaps = (int)ops->taps.size() / 3, ndtaps = (int)ops->dtaps.size() / 3;
  int err = (int)hipMemcpyAsync(G, ops->G.data(), ops->G.size() * 8, hipMemcpyHostToDevice, stream);
  if (!err) err = (int)hipMemcpyAsync(Dc, ops->Dc.data(), ops->Dc.size() * 8, hipMemcpyHostToDevice, stream);
  if (!err) err = launch_aos_to_soa(q_in, Q[0], P.nel, ns, stream);
  int cur = 0;
  for (int s = 0; s < n_steps && !err; ++s) {
    err = launch_predict_prefactored(P.d, P.M, g, Q[cur], W, G, ops->taps.data(), ntaps, stream);
    if (!err) err = launch_tap_update(P.d, P.M, 0, g, W, Q[cur], Q[1 - cur], Dc, ops->dtaps.data(), ndtaps, stream);
    cur ^= 1;
  }
  if (!err) err = launch_soa_to_aos(Q[cur], q_out, P.nel, ns, stream);
  return err ? static_fail(RIDG_E_DEVICE, hipGetErrorString((hipError_t)err)) : RIDG_OK;
}
