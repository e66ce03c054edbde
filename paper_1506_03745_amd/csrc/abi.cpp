// C entry points of the pbt library (declared in include/pbt.h).
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pbt.h"
#include "parallel.h"
#include "quadrature.h"
#include "system.h"

using namespace pbt;

// Scratch of pbt_matvec_dev_static, the product that allocates nothing: the
// unknowns in the internal order, the product before it is permuted back,
// and the P2P / M2P partial sums live in this array instead of buffers of
// the context.  Each device the library runs on holds its own copy until the
// process ends; every call on a device shares that copy, so calls that
// overlap on one device race.  Host code never uses the array's name as an
// address: pbt_create stores each device's address (hipGetSymbolAddress).
constexpr size_t kStaticScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {nullptr};

// Address of `device`'s copy of the scratch array, looked up once per device
// with that device current.
hipError_t scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[device] = p;
  return hipSuccess;
}

void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[device];
}

// Winding number of a closed triangle mesh (outward orientation) about point
// p: the solid angles of its triangles summed over 4 pi, each from the
// formula of Van Oosterom and Strackee, tan(Omega / 2) = a . (b x c) /
// (|a||b||c| + (a . b)|c| + (a . c)|b| + (b . c)|a|) with a, b, c the
// corners relative to p.  1 inside, 0 outside.
double winding_number(const SurfIn& S, const double* p) {
  double w = 0.0;
  for (int64_t t = 0; t < S.nt; ++t) {
    double v[3][3];
    for (int k = 0; k < 3; ++k)
      for (int d = 0; d < 3; ++d) v[k][d] = S.xyz[3 * S.tri[3 * t + k] + d] - p[d];
    const double* a = v[0];
    const double* b = v[1];
    const double* c = v[2];
    const double la = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    const double lb = std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    const double lc = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    const double num = a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2]) +
                       a[2] * (b[0] * c[1] - b[1] * c[0]);
    const double ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    const double ac = a[0] * c[0] + a[1] * c[1] + a[2] * c[2];
    const double bc = b[0] * c[0] + b[1] * c[1] + b[2] * c[2];
    w += 2.0 * std::atan2(num, la * lb * lc + ab * lc + ac * lb + bc * la);
  }
  return w / (4.0 * M_PI);
}

// Index of the first of nq points whose winding number about S is on the
// wrong side (inside = true: must be > 1/2), or -1.
int64_t first_misplaced(const SurfIn& S, const double* xyz, int64_t nq, bool inside) {
  std::vector<char> bad(nq, 0);
  parallel_for(nq, [&](int64_t k) {
    const double w = winding_number(S, xyz + 3 * k);
    bad[k] = inside ? !(w > 0.5) : !(w < 0.5);
  }, 4);
  for (int64_t k = 0; k < nq; ++k)
    if (bad[k]) return k;
  return -1;
}

}  // namespace

struct pbt_ctx {
  int device = 0;
  pbt_params prm{};
  double eps_out = 80.0, kappa = 0.125;
  std::vector<std::unique_ptr<SurfIn>> surfs;
  std::map<std::vector<bool>, std::unique_ptr<System>> systems;
  hipStream_t stream = nullptr;
  std::string err;
  bool frozen = false;
  int gs_passes = 0;   // Gram-Schmidt passes per Arnoldi step (0 = automatic), every system
  // work of the last solve / interaction_energy / gradient / solve_batch call
  struct CallStats {
    double t0 = 0, t_setup = 0;
    int64_t apps = 0, pairs = 0;
    int32_t iters = 0;
    std::map<const System*, int64_t> start, start_pairs;
  } cs;
  bool profile = false;   // per-kernel event timing of every product (pbt_profile)
  double prof_batch[16] = {0};   // totals of the batched systems (built and released per call)
  pbt_result last_stats{};
  // last solution
  std::vector<bool> sol_mask;
  std::vector<double> sol_x;   // host copy of dsol, made when first asked for
  bool sol_on_host = false;
  DBuf<double> dx, dy, db, dsol, dt;   // dt: a vector in the boundary's layout
};

namespace {

double wall_now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Adds the operator applications system S made since it stood at apps0
// (and the dense-equivalent pairs since pairs0).
void stats_account(pbt_ctx* c, const System& S, int64_t apps0, int64_t pairs0) {
  c->cs.apps += S.applications() - apps0;
  c->cs.pairs += S.pairs_done() - pairs0;
}

pbt_status fail(pbt_ctx* c, int st, const std::string& m) {
  if (c) c->err = m;
  return (pbt_status)st;
}

template <typename F>
pbt_status guarded(pbt_ctx* c, F&& f) {
  if (!c) return PBT_E_INVALID;
  try {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != c->device) {
      if (hipSetDevice(c->device) != hipSuccess) return fail(c, PBT_E_DEVICE, "hipSetDevice failed");
    }
    return f();
  } catch (const Error& e) {
    return fail(c, e.status, e.what());
  } catch (const std::bad_alloc&) {
    return fail(c, PBT_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(c, PBT_E_DEVICE, e.what());
  }
}

// guarded() plus the work counters read by pbt_last_stats.
template <typename F>
pbt_status tracked(pbt_ctx* c, F&& f) {
  if (!c) return PBT_E_INVALID;
  c->cs = pbt_ctx::CallStats{};
  c->cs.t0 = wall_now();
  for (auto& kv : c->systems) {
    c->cs.start[kv.second.get()] = kv.second->applications();
    c->cs.start_pairs[kv.second.get()] = kv.second->pairs_done();
  }
  const pbt_status st = guarded(c, f);
  for (auto& kv : c->systems) {
    auto it = c->cs.start.find(kv.second.get());
    const bool had = it != c->cs.start.end();
    stats_account(c, *kv.second, had ? it->second : 0, had ? c->cs.start_pairs[kv.second.get()] : 0);
  }
  pbt_result r{};
  r.iters = c->cs.iters;
  r.matvecs = (int32_t)std::min<int64_t>(c->cs.apps, INT32_MAX);
  r.dense_pairs = c->cs.pairs;
  r.t_setup_s = c->cs.t_setup;
  r.t_solve_s = wall_now() - c->cs.t0;
  c->last_stats = r;
  return st;
}

std::string check_params(const pbt_params& p) {
  if (!(p.k_far == 1 || p.k_far == 3 || p.k_far == 4 || p.k_far == 7)) return "k_far must be 1, 3, 4 or 7";
  if (!(p.k_near == 1 || p.k_near == 3 || p.k_near == 4 || p.k_near == 7 || p.k_near == 19))
    return "k_near must be 1, 3, 4, 7 or 19";
  if (p.k_self_edge < 1 || p.k_self_edge > 64) return "k_self_edge must be 1..64";
  if (p.ncrit < 1) return "ncrit must be >= 1";
  if (p.taylor_p < 0 || p.taylor_p > kMaxP) return "taylor_p must be 0..8";
  if (!(p.theta > 0.0 && p.theta < 1.0)) return "theta must be in (0, 1)";
  if (!(p.tol > 0.0)) return "tol must be > 0";
  if (p.restart < 1 || p.restart > 1024) return "restart must be 1..1024";
  if (p.max_iter < 1) return "max_iter must be >= 1";
  if (p.prec != PBT_FP64 && p.prec != PBT_MIXED) return "prec must be PBT_FP64 or PBT_MIXED";
  if (!(p.near_factor > 0.0) || !std::isfinite(p.near_factor) || p.near_factor > 1e3)
    return "near_factor must be in (0, 1000]";
  if (p.precond != 0 && p.precond != 1) return "precond must be 0 or 1";
  return "";
}

std::vector<bool> mask_of(const pbt_ctx* c) {
  std::vector<bool> m;
  for (auto& s : c->surfs) m.push_back(s->enabled);
  return m;
}

System& system_for(pbt_ctx* c) {
  std::vector<bool> m = mask_of(c);
  auto it = c->systems.find(m);
  if (it != c->systems.end()) {
    it->second->set_gs_passes(c->gs_passes);
    return *it->second;
  }

  std::vector<const SurfIn*> on;
  for (auto& s : c->surfs)
    if (s->enabled) on.push_back(s.get());
  if (on.empty()) throw Error(PBT_E_STATE, "no enabled surface");
  for (const SurfIn* s : on)
    if (s->kind == PBT_MOLECULE && !(s->eps_in > 0)) throw Error(PBT_E_STATE, "molecule without eps_in");
  for (const SurfIn* s : on)
    if ((s->kind == PBT_STERN || s->kind == PBT_CAVITY) && !s->parent)
      throw Error(PBT_E_STATE, "Stern surface or cavity without its molecule");
  c->frozen = true;
  const double t0 = wall_now();
  auto sys = std::make_unique<System>(on, c->prm, c->eps_out, c->kappa, c->stream);
  c->cs.t_setup += wall_now() - t0;
  System& r = *sys;
  r.set_gs_passes(c->gs_passes);
  if (c->profile) r.set_profile(true);
  c->systems[m] = std::move(sys);
  return r;
}

// Device buffers of the _dev entry points: `ptr` must be device (or
// managed) memory of this context's device; `n` doubles are copied to the
// host in the order of `stream` (the call waits for them).
void check_dev_ptr(const pbt_ctx* c, const void* ptr) {
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, ptr) != hipSuccess) {
    (void)hipGetLastError();
    throw Error(PBT_E_INVALID, "not a device pointer");
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
    throw Error(PBT_E_INVALID, "not a device pointer");
  if (at.device != c->device) throw Error(PBT_E_INVALID, "device pointer of another device");
}

std::vector<double> from_dev(const pbt_ctx* c, const double* ptr, int64_t n, hipStream_t st) {
  std::vector<double> h((size_t)std::max<int64_t>(n, 0));
  if (n <= 0) return h;
  check_dev_ptr(c, ptr);
  PBT_HIP(hipMemcpyAsync(h.data(), ptr, n * sizeof(double), hipMemcpyDeviceToHost, st));
  PBT_HIP(hipStreamSynchronize(st));
  return h;
}

void to_dev(const pbt_ctx* c, double* ptr, const std::vector<double>& h, hipStream_t st) {
  if (h.empty()) return;
  check_dev_ptr(c, ptr);
  PBT_HIP(hipMemcpyAsync(ptr, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, st));
  PBT_HIP(hipStreamSynchronize(st));
}

int local_of(const pbt_ctx* c, int id) {
  int k = 0;
  for (int i = 0; i < id; ++i) k += c->surfs[i]->enabled ? 1 : 0;
  return k;
}

pbt_status solve_impl(pbt_ctx* c, const double* x0, pbt_result* res) {
  System& S = system_for(c);
  const int64_t n = S.n();
  pbt_result r{};
  const double t0 = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
  const int64_t apply0 = S.applications();
  c->db.alloc(n);
  c->dx.alloc(n);
  S.rhs(c->db.p, c->stream);
  if (x0) {
    for (int64_t i = 0; i < n; ++i)
      if (!std::isfinite(x0[i])) return fail(c, PBT_E_INVALID, "non-finite initial guess");
    c->dt.alloc(n);
    PBT_HIP(hipMemcpyAsync(c->dt.p, x0, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    S.to_internal(c->dt.p, c->dx.p, c->stream);
  }
  PBT_HIP(hipStreamSynchronize(c->stream));
  const double t1 = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
  const bool ok = S.solve(c->db.p, c->dx.p, x0 != nullptr, &r, c->stream);
  S.energies(c->dx.p, &r, c->stream);
  PBT_HIP(hipStreamSynchronize(c->stream));
  const double t2 = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
  r.t_setup_s = t1 - t0;
  r.t_solve_s = t2 - t1;
  r.p2p_pairs = S.plan().p2p_pairs;
  r.m2p_pairs = S.plan().m2p_pairs;
  r.dense_pairs = S.dense_pairs();
  r.p2p_fused_pairs = S.plan().p2p_fused_pairs;
  r.m2p_fused_pairs = S.plan().m2p_fused_pairs;
  r.matvecs = (int32_t)(S.applications() - apply0);
  c->cs.iters = std::max(c->cs.iters, r.iters);
  if (!std::isfinite(r.F_total) || !std::isfinite(r.rel_resid)) {
    // outputs untouched; no solution to read back
    c->sol_mask.clear();
    return fail(c, PBT_E_NUMERIC, "non-finite energy or residual");
  }
  // the solution stays on the device until pbt_get_solution asks for it
  c->dsol.alloc(n);
  PBT_HIP(hipMemcpyAsync(c->dsol.p, c->dx.p, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  c->sol_on_host = false;
  c->sol_mask = mask_of(c);
  if (res) *res = r;
  if (!ok) return fail(c, PBT_E_NOCONVERGE, "GMRES did not reach the tolerance within max_iter");
  return PBT_OK;
}

}  // namespace

extern "C" {

void pbt_default_params(pbt_params* p) {
  if (!p) return;
  p->k_far = 3;
  p->k_near = 19;
  p->k_self_edge = 9;
  p->ncrit = 300;
  p->taylor_p = 6;
  p->theta = 0.5;
  p->tol = 1e-6;
  p->restart = 100;
  p->max_iter = 1000;
  p->prec = PBT_FP64;
  p->treecode = 1;
  p->near_factor = 2.0;
  p->precond = 1;
}

pbt_status pbt_create(pbt_ctx** out, int32_t hip_device, const pbt_params* params) {
  if (!out) return PBT_E_INVALID;
  *out = nullptr;
  pbt_params p;
  pbt_default_params(&p);
  if (params) p = *params;
  if (!check_params(p).empty()) return PBT_E_INVALID;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return PBT_E_DEVICE;
  if (hipSetDevice(hip_device) != hipSuccess) return PBT_E_DEVICE;
  if (scratch_init(hip_device) != hipSuccess) return PBT_E_DEVICE;
  auto c = new (std::nothrow) pbt_ctx();
  if (!c) return PBT_E_NOMEM;
  c->device = hip_device;
  c->prm = p;
  if (hipStreamCreate(&c->stream) != hipSuccess) {
    delete c;
    return PBT_E_DEVICE;
  }
  *out = c;
  return PBT_OK;
}

void pbt_destroy(pbt_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  c->systems.clear();
  c->dx.release();
  c->dy.release();
  c->db.release();
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* pbt_last_error(const pbt_ctx* c) { return c ? c->err.c_str() : "null context"; }

pbt_status pbt_set_params(pbt_ctx* c, const pbt_params* p) {
  if (!c || !p) return fail(c, PBT_E_INVALID, "null argument");
  const std::string m = check_params(*p);
  if (!m.empty()) return fail(c, PBT_E_INVALID, m);
  return guarded(c, [&] {
    c->prm = *p;
    c->systems.clear();
    return PBT_OK;
  });
}

pbt_status pbt_set_solvent(pbt_ctx* c, double eps_out, double kappa) {
  if (!c) return PBT_E_INVALID;
  if (!(eps_out > 0) || !std::isfinite(eps_out) || !(kappa >= 0) || !std::isfinite(kappa))
    return fail(c, PBT_E_INVALID, "eps_out must be > 0 and kappa >= 0");
  if (c->frozen && (eps_out != c->eps_out || kappa != c->kappa)) c->systems.clear();
  c->eps_out = eps_out;
  c->kappa = kappa;
  return PBT_OK;
}

pbt_status pbt_add_surface(pbt_ctx* c, pbt_kind kind, const double* xyz, int64_t nv,
                           const int32_t* tri, int64_t nt, const double* bc, int32_t* id) {
  if (!c) return PBT_E_INVALID;
  if (c->frozen) return fail(c, PBT_E_STATE, "geometry is frozen after the first solve");
  if (kind != PBT_MOLECULE && kind != PBT_CHARGED && kind != PBT_POTENTIAL && kind != PBT_STERN &&
      kind != PBT_CAVITY)
    return fail(c, PBT_E_INVALID, "unknown surface kind");
  if (!xyz || !tri || nv < 3 || nt < 1 || nt > (int64_t)1 << 28)
    return fail(c, PBT_E_INVALID, "empty or oversized mesh");
  const bool imposed = kind == PBT_CHARGED || kind == PBT_POTENTIAL;
  if (imposed && !bc) return fail(c, PBT_E_INVALID, "boundary values required");
  for (int64_t i = 0; i < 3 * nv; ++i)
    if (!std::isfinite(xyz[i])) return fail(c, PBT_E_INVALID, "non-finite vertex coordinate");
  for (int64_t i = 0; i < 3 * nt; ++i)
    if (tri[i] < 0 || tri[i] >= nv) return fail(c, PBT_E_INVALID, "vertex index out of range");
  for (int64_t t = 0; t < nt; ++t) {
    const double* a = xyz + 3 * tri[3 * t];
    const double* b = xyz + 3 * tri[3 * t + 1];
    const double* d = xyz + 3 * tri[3 * t + 2];
    const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double e2[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
    const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                 cz = e1[0] * e2[1] - e1[1] * e2[0];
    if (!(0.5 * std::sqrt(cx * cx + cy * cy + cz * cz) >= 1e-12))
      return fail(c, PBT_E_INVALID, "degenerate panel (area < 1e-12 A^2)");
  }
  if (imposed)
    for (int64_t t = 0; t < nt; ++t)
      if (!std::isfinite(bc[t])) return fail(c, PBT_E_INVALID, "non-finite boundary value");
  auto s = std::make_unique<SurfIn>();
  s->kind = kind;
  s->nv = nv;
  s->nt = nt;
  s->xyz.assign(xyz, xyz + 3 * nv);
  s->tri.assign(tri, tri + 3 * nt);
  if (imposed) s->bc.assign(bc, bc + nt);
  c->surfs.push_back(std::move(s));
  if (id) *id = (int32_t)c->surfs.size() - 1;
  return PBT_OK;
}

pbt_status pbt_set_bc(pbt_ctx* c, int32_t id, const double* bc) {
  if (!c) return PBT_E_INVALID;
  if (id < 0 || id >= (int)c->surfs.size() || !bc) return fail(c, PBT_E_INVALID, "bad surface id");
  SurfIn& s = *c->surfs[id];
  if (s.kind != PBT_CHARGED && s.kind != PBT_POTENTIAL)
    return fail(c, PBT_E_INVALID, "only charged and potential surfaces have imposed boundary values");
  for (int64_t t = 0; t < s.nt; ++t)
    if (!std::isfinite(bc[t])) return fail(c, PBT_E_INVALID, "non-finite boundary value");
  s.bc.assign(bc, bc + s.nt);
  ++s.version;
  return PBT_OK;
}

pbt_status pbt_set_charges(pbt_ctx* c, int32_t mol_id, double eps_in, const double* xyz,
                           const double* q, int64_t nq) {
  if (!c) return PBT_E_INVALID;
  if (mol_id < 0 || mol_id >= (int)c->surfs.size() || c->surfs[mol_id]->kind != PBT_MOLECULE)
    return fail(c, PBT_E_INVALID, "not a molecule id");
  if (!(eps_in > 0) || !std::isfinite(eps_in)) return fail(c, PBT_E_INVALID, "eps_in must be > 0");
  if (nq < 0 || (nq > 0 && (!xyz || !q))) return fail(c, PBT_E_INVALID, "bad charge arrays");
  for (int64_t i = 0; i < 3 * nq; ++i)
    if (!std::isfinite(xyz[i])) return fail(c, PBT_E_INVALID, "non-finite charge position");
  for (int64_t i = 0; i < nq; ++i)
    if (!std::isfinite(q[i])) return fail(c, PBT_E_INVALID, "non-finite charge");
  SurfIn& s = *c->surfs[mol_id];
  // charges lie in the molecule's interior region: inside its surface and
  // outside its cavities (checked when their positions change)
  if (nq > 0 && !(s.qxyz.size() == (size_t)(3 * nq) && std::equal(xyz, xyz + 3 * nq, s.qxyz.begin()))) {
    const int64_t k = first_misplaced(s, xyz, nq, true);
    if (k >= 0) return fail(c, PBT_E_INVALID, "charge " + std::to_string(k) + " lies outside its molecule");
    for (const auto& cv : c->surfs)
      if (cv->kind == PBT_CAVITY && cv->parent == &s) {
        const int64_t kc = first_misplaced(*cv, xyz, nq, false);
        if (kc >= 0) return fail(c, PBT_E_INVALID, "charge " + std::to_string(kc) + " lies inside a cavity");
      }
  }
  if (c->frozen && s.eps_in != eps_in) {
    // eps_in enters the operator: drop prepared systems that contain it
    c->systems.clear();
  }
  s.eps_in = eps_in;
  s.qxyz.assign(xyz, xyz + 3 * nq);
  s.q.assign(q, q + nq);
  ++s.version;
  return PBT_OK;
}

pbt_status pbt_set_bc_dev(pbt_ctx* c, int32_t id, const double* bc_dev, void* stream) {
  if (!c) return PBT_E_INVALID;
  if (id < 0 || id >= (int)c->surfs.size() || !bc_dev) return fail(c, PBT_E_INVALID, "bad surface id");
  std::vector<double> bc;
  const pbt_status st = guarded(c, [&] {
    bc = from_dev(c, bc_dev, c->surfs[id]->nt, stream ? (hipStream_t)stream : c->stream);
    return PBT_OK;
  });
  if (st != PBT_OK) return st;
  return pbt_set_bc(c, id, bc.data());
}

pbt_status pbt_set_charges_dev(pbt_ctx* c, int32_t mol_id, double eps_in, const double* xyz_dev,
                               const double* q_dev, int64_t nq, void* stream) {
  if (!c) return PBT_E_INVALID;
  if (mol_id < 0 || mol_id >= (int)c->surfs.size() || c->surfs[mol_id]->kind != PBT_MOLECULE)
    return fail(c, PBT_E_INVALID, "not a molecule id");
  if (nq < 0 || (nq > 0 && !q_dev)) return fail(c, PBT_E_INVALID, "bad charge arrays");
  if (!xyz_dev && (int64_t)c->surfs[mol_id]->q.size() != nq)
    return fail(c, PBT_E_INVALID, "xyz_dev is NULL but the number of charges changes");
  std::vector<double> xyz, q;
  const pbt_status st = guarded(c, [&] {
    const hipStream_t s = stream ? (hipStream_t)stream : c->stream;
    q = from_dev(c, q_dev, nq, s);
    if (xyz_dev) xyz = from_dev(c, xyz_dev, 3 * nq, s);
    return PBT_OK;
  });
  if (st != PBT_OK) return st;
  if (!xyz_dev) xyz = c->surfs[mol_id]->qxyz;
  return pbt_set_charges(c, mol_id, eps_in, xyz.data(), q.data(), nq);
}

pbt_status pbt_set_stern(pbt_ctx* c, int32_t stern_id, int32_t mol_id, double eps_layer) {
  if (!c) return PBT_E_INVALID;
  const int ns = (int)c->surfs.size();
  if (stern_id < 0 || stern_id >= ns || c->surfs[stern_id]->kind != PBT_STERN)
    return fail(c, PBT_E_INVALID, "not a Stern surface id");
  if (mol_id < 0 || mol_id >= ns || c->surfs[mol_id]->kind != PBT_MOLECULE)
    return fail(c, PBT_E_INVALID, "not a molecule id");
  if (!(eps_layer > 0) || !std::isfinite(eps_layer)) return fail(c, PBT_E_INVALID, "eps_layer must be > 0");
  if (c->frozen) return fail(c, PBT_E_STATE, "geometry is frozen after the first solve");
  for (int k = 0; k < ns; ++k)
    if (k != stern_id && c->surfs[k]->kind == PBT_STERN && c->surfs[k]->parent == c->surfs[mol_id].get())
      return fail(c, PBT_E_INVALID, "the molecule already has a Stern surface");
  c->surfs[stern_id]->parent = c->surfs[mol_id].get();
  c->surfs[stern_id]->eps_in = eps_layer;
  return PBT_OK;
}

pbt_status pbt_set_cavity(pbt_ctx* c, int32_t cav_id, int32_t mol_id, double eps_cavity) {
  if (!c) return PBT_E_INVALID;
  const int ns = (int)c->surfs.size();
  if (cav_id < 0 || cav_id >= ns || c->surfs[cav_id]->kind != PBT_CAVITY)
    return fail(c, PBT_E_INVALID, "not a cavity id");
  if (mol_id < 0 || mol_id >= ns || c->surfs[mol_id]->kind != PBT_MOLECULE)
    return fail(c, PBT_E_INVALID, "not a molecule id");
  if (!(eps_cavity > 0) || !std::isfinite(eps_cavity)) return fail(c, PBT_E_INVALID, "eps_cavity must be > 0");
  if (c->frozen) return fail(c, PBT_E_STATE, "geometry is frozen after the first solve");
  const SurfIn& M = *c->surfs[mol_id];
  const int64_t k = first_misplaced(*c->surfs[cav_id], M.qxyz.data(), (int64_t)M.q.size(), false);
  if (k >= 0) return fail(c, PBT_E_INVALID, "charge " + std::to_string(k) + " lies inside the cavity");
  c->surfs[cav_id]->parent = c->surfs[mol_id].get();
  c->surfs[cav_id]->eps_in = eps_cavity;
  return PBT_OK;
}

pbt_status pbt_enable(pbt_ctx* c, int32_t id, int32_t on) {
  if (!c) return PBT_E_INVALID;
  if (id < 0 || id >= (int)c->surfs.size()) return fail(c, PBT_E_INVALID, "bad surface id");
  c->surfs[id]->enabled = on != 0;
  return PBT_OK;
}

pbt_status pbt_prepare(pbt_ctx* c) {
  return guarded(c, [&] {
    system_for(c);
    return PBT_OK;
  });
}

pbt_status pbt_num_unknowns(pbt_ctx* c, int64_t* n) {
  if (!c || !n) return fail(c, PBT_E_INVALID, "null argument");
  int64_t k = 0;
  for (auto& s : c->surfs)
    if (s->enabled) k += (s->kind == PBT_CHARGED || s->kind == PBT_POTENTIAL) ? s->nt : 2 * s->nt;
  *n = k;
  return PBT_OK;
}

pbt_status pbt_solve(pbt_ctx* c, const double* x0, pbt_result* res) {
  return tracked(c, [&] { return solve_impl(c, x0, res); });
}

pbt_status pbt_get_solution(pbt_ctx* c, int32_t id, double* phi, double* dphidn) {
  return guarded(c, [&] {
    if (id < 0 || id >= (int)c->surfs.size()) return fail(c, PBT_E_INVALID, "bad surface id");
    if (c->sol_mask.empty() || c->sol_mask.size() != c->surfs.size() || !c->sol_mask[id])
      return fail(c, PBT_E_STATE, "no solution for this surface");
    if (!c->sol_on_host) {
      c->sol_x = c->dsol.download(c->stream);
      c->sol_on_host = true;
    }
    std::vector<bool> cur = mask_of(c);
    auto it = c->systems.find(c->sol_mask);
    if (it == c->systems.end()) return fail(c, PBT_E_STATE, "solution's system was released");
    int k = 0;
    for (int i = 0; i < id; ++i) k += c->sol_mask[i] ? 1 : 0;
    it->second->unpack(c->sol_x, k, phi, dphidn);
    return PBT_OK;
  });
}

pbt_status pbt_get_solution_dev(pbt_ctx* c, int32_t id, double* phi_dev, double* dphidn_dev, void* stream) {
  if (!c) return PBT_E_INVALID;
  if (id < 0 || id >= (int)c->surfs.size()) return fail(c, PBT_E_INVALID, "bad surface id");
  const int64_t nt = c->surfs[id]->nt;
  std::vector<double> phi(nt), d(nt);
  const pbt_status st = pbt_get_solution(c, id, phi.data(), d.data());
  if (st != PBT_OK) return st;
  return guarded(c, [&] {
    const hipStream_t s = stream ? (hipStream_t)stream : c->stream;
    if (phi_dev) to_dev(c, phi_dev, phi, s);
    if (dphidn_dev) to_dev(c, dphidn_dev, d, s);
    return PBT_OK;
  });
}

pbt_status pbt_interaction_energy(pbt_ctx* c, double* F_int, pbt_result* parts) {
  return tracked(c, [&] {
    const int ns = (int)c->surfs.size();
    std::vector<bool> saved = mask_of(c);
    pbt_status worst = PBT_OK;
    auto restore = [&] { for (int i = 0; i < ns; ++i) c->surfs[i]->enabled = saved[i]; };
    std::vector<pbt_result> r(ns + 1);
    for (int i = 0; i < ns; ++i) c->surfs[i]->enabled = true;
    pbt_status st;
    try {
      st = solve_impl(c, nullptr, &r[0]);
      if (st != PBT_OK && st != PBT_E_NOCONVERGE) { restore(); return st; }
      if (st != PBT_OK) worst = st;
      for (int k = 0; k < ns; ++k) {
        // a molecule is isolated together with its Stern surface and
        // cavities, which are no components of their own (entries stay zero)
        if (c->surfs[k]->kind == PBT_STERN || c->surfs[k]->kind == PBT_CAVITY) continue;
        for (int i = 0; i < ns; ++i)
          c->surfs[i]->enabled = i == k || c->surfs[i]->parent == c->surfs[k].get();
        st = solve_impl(c, nullptr, &r[k + 1]);
        if (st != PBT_OK && st != PBT_E_NOCONVERGE) { restore(); return st; }
        if (st != PBT_OK) worst = st;
      }
    } catch (...) {
      restore();
      throw;
    }
    restore();
    double f = r[0].F_total;
    for (int k = 0; k < ns; ++k) f -= r[k + 1].F_total;
    if (F_int) *F_int = f;
    if (parts) for (int k = 0; k <= ns; ++k) parts[k] = r[k];
    return worst;
  });
}

pbt_status pbt_matvec_dev(pbt_ctx* c, const double* x_dev, double* y_dev, int32_t transpose,
                          pbt_precision prec, void* stream) {
  return guarded(c, [&] {
    if (!x_dev || !y_dev) return fail(c, PBT_E_INVALID, "null buffer");
    System& S = system_for(c);
    hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    const int64_t n = S.n();
    c->dx.alloc(n);
    c->dy.alloc(n);
    S.to_internal(x_dev, c->dx.p, st);
    if (transpose) S.matvec_t(c->dx.p, c->dy.p, prec == PBT_MIXED, nullptr, st);
    else S.matvec(c->dx.p, c->dy.p, prec == PBT_MIXED, st, true);
    S.to_boundary(c->dy.p, y_dev, st);
    return PBT_OK;
  });
}

pbt_status pbt_matvec_dev_static(pbt_ctx* c, const double* x_dev, double* y_dev, pbt_precision prec,
                                 void* stream) {
  return guarded(c, [&] {
    if (!x_dev || !y_dev) return fail(c, PBT_E_INVALID, "null buffer");
    if (prec != PBT_FP64 && prec != PBT_MIXED) return fail(c, PBT_E_INVALID, "prec must be PBT_FP64 or PBT_MIXED");
    // the prepared system of the enabled surfaces (found without building a key)
    System* S = nullptr;
    for (auto& kv : c->systems) {
      bool same = kv.first.size() == c->surfs.size();
      for (size_t i = 0; same && i < kv.first.size(); ++i) same = kv.first[i] == c->surfs[i]->enabled;
      if (same) {
        S = kv.second.get();
        break;
      }
    }
    if (!S) return fail(c, PBT_E_STATE, "no prepared system for the enabled surfaces (pbt_prepare allocates; call it first)");
    unsigned char* base = static_cast<unsigned char*>(scratch_of(c->device));
    if (!base) return fail(c, PBT_E_DEVICE, "no scratch address for this device");
    const bool fp32 = prec == PBT_MIXED;
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t nb = up((size_t)S->n() * sizeof(double));
    const size_t pb = up(S->part_need(fp32)), ppb = up(S->ppart_need(fp32));
    if (2 * nb + pb + ppb > kStaticScratchBytes)
      return fail(c, PBT_E_INVALID, "the system needs " + std::to_string(2 * nb + pb + ppb) +
                                        " bytes of scratch; the static array holds " +
                                        std::to_string(kStaticScratchBytes));
    double* xi = reinterpret_cast<double*>(base);
    double* yi = reinterpret_cast<double*>(base + nb);
    const System::ExtParts ext{base + 2 * nb, base + 2 * nb + pb};
    const hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    S->to_internal(x_dev, xi, st);
    S->matvec(xi, yi, fp32, st, false, false, nullptr, &ext);
    S->to_boundary(yi, y_dev, st);
    return PBT_OK;
  });
}

pbt_status pbt_matvec(pbt_ctx* c, const double* x, double* y, int32_t transpose, pbt_precision prec) {
  return guarded(c, [&] {
    if (!x || !y) return fail(c, PBT_E_INVALID, "null buffer");
    System& S = system_for(c);
    const int64_t n = S.n();
    c->dx.alloc(n);
    c->dy.alloc(n);
    c->dt.alloc(n);
    PBT_HIP(hipMemcpyAsync(c->dt.p, x, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    S.to_internal(c->dt.p, c->dx.p, c->stream);
    if (transpose) S.matvec_t(c->dx.p, c->dy.p, prec == PBT_MIXED, nullptr, c->stream);
    else S.matvec(c->dx.p, c->dy.p, prec == PBT_MIXED, c->stream, true);
    S.to_boundary(c->dy.p, c->dt.p, c->stream);
    PBT_HIP(hipMemcpyAsync(y, c->dt.p, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    PBT_HIP(hipStreamSynchronize(c->stream));
    return PBT_OK;
  });
}

pbt_status pbt_rhs(pbt_ctx* c, double* b) {
  return guarded(c, [&] {
    if (!b) return fail(c, PBT_E_INVALID, "null buffer");
    System& S = system_for(c);
    c->db.alloc(S.n());
    c->dt.alloc(S.n());
    S.rhs(c->db.p, c->stream);
    S.to_boundary(c->db.p, c->dt.p, c->stream);
    PBT_HIP(hipMemcpyAsync(b, c->dt.p, S.n() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    PBT_HIP(hipStreamSynchronize(c->stream));
    return PBT_OK;
  });
}

// One system's contribution: forward solve, adjoint solve, gradient terms.
// Returns dF_total/dq of molecule `mol` and dF_total/dsigma of surface `sig`
// (reduced units), looked up by surface identity.
static pbt_status system_gradient(pbt_ctx* c, int mol, int sig, std::vector<double>* dq,
                                  std::vector<double>* dsig) {
  System& S = system_for(c);
  const int64_t n = S.n();
  pbt_result r{};
  DBuf<double> b, x, g, lam;
  b.alloc(n);
  x.alloc(n);
  g.alloc(n);
  lam.alloc(n);
  S.rhs(b.p, c->stream);
  const bool ok1 = S.solve(b.p, x.p, false, &r, c->stream);
  S.adjoint_rhs(x.p, g.p, c->stream);
  pbt_result ra{};
  const bool ok2 = S.solve_t(g.p, lam.p, &ra, c->stream);
  std::vector<std::vector<double>> gq, gs;
  S.gradient_terms(x.p, lam.p, gq, gs, c->stream);
  for (int e = 0; e < S.n_surfaces(); ++e) {
    if (mol >= 0 && S.surface(e) == c->surfs[mol].get() && dq) *dq = gq[e];
    if (sig >= 0 && S.surface(e) == c->surfs[sig].get() && dsig) *dsig = gs[e];
  }
  if (!ok1 || !ok2) return fail(c, PBT_E_NOCONVERGE, "forward or adjoint GMRES did not converge");
  return PBT_OK;
}

pbt_status pbt_gradient(pbt_ctx* c, int32_t sigma_id, double* dF_dsigma, int32_t mol_id, double* dF_dq) {
  return tracked(c, [&] {
    const int ns = (int)c->surfs.size();
    if (sigma_id >= ns || mol_id >= ns || (sigma_id < 0 && mol_id < 0))
      return fail(c, PBT_E_INVALID, "bad surface ids");
    if (sigma_id >= 0 && (c->surfs[sigma_id]->kind != PBT_CHARGED || !dF_dsigma))
      return fail(c, PBT_E_INVALID, "sigma_id must name a charged surface (and dF_dsigma be given)");
    if (mol_id >= 0 && (c->surfs[mol_id]->kind != PBT_MOLECULE || !dF_dq))
      return fail(c, PBT_E_INVALID, "mol_id must name a molecule (and dF_dq be given)");
    std::vector<bool> saved = mask_of(c);
    // a component: the surface alone, or a molecule with its Stern surface
    // and cavities
    auto set_mask = [&](int only) {
      for (int i = 0; i < ns; ++i)
        c->surfs[i]->enabled = only < 0 || i == only || (only >= 0 && c->surfs[i]->parent == c->surfs[only].get());
    };
    pbt_status worst = PBT_OK;
    std::vector<double> dq_a, ds_a, dq_i, ds_i;
    try {
      set_mask(-1);
      pbt_status st = system_gradient(c, mol_id, sigma_id, &dq_a, &ds_a);
      if (st != PBT_OK && st != PBT_E_NOCONVERGE) throw Error(st, c->err);
      if (st != PBT_OK) worst = st;
      if (sigma_id >= 0) {
        set_mask(sigma_id);
        st = system_gradient(c, -1, sigma_id, nullptr, &ds_i);
        if (st != PBT_OK && st != PBT_E_NOCONVERGE) throw Error(st, c->err);
        if (st != PBT_OK) worst = st;
      }
      if (mol_id >= 0) {
        set_mask(mol_id);
        st = system_gradient(c, mol_id, -1, &dq_i, nullptr);
        if (st != PBT_OK && st != PBT_E_NOCONVERGE) throw Error(st, c->err);
        if (st != PBT_OK) worst = st;
      }
    } catch (...) {
      for (int i = 0; i < ns; ++i) c->surfs[i]->enabled = saved[i];
      throw;
    }
    for (int i = 0; i < ns; ++i) c->surfs[i]->enabled = saved[i];
    if (sigma_id >= 0)
      for (size_t k = 0; k < ds_a.size(); ++k) dF_dsigma[k] = (ds_a[k] - ds_i[k]) * kKcalPerUnit * kSigmaSI;
    if (mol_id >= 0)
      for (size_t k = 0; k < dq_a.size(); ++k) dF_dq[k] = (dq_a[k] - dq_i[k]) * kKcalPerUnit;
    return worst;
  });
}

pbt_status pbt_gradient_dev(pbt_ctx* c, int32_t sigma_id, double* dF_dsigma_dev, int32_t mol_id, double* dF_dq_dev,
                            void* stream) {
  if (!c) return PBT_E_INVALID;
  const int ns = (int)c->surfs.size();
  if (sigma_id >= ns || mol_id >= ns || (sigma_id < 0 && mol_id < 0)) return fail(c, PBT_E_INVALID, "bad surface ids");
  if ((sigma_id >= 0 && !dF_dsigma_dev) || (mol_id >= 0 && !dF_dq_dev))
    return fail(c, PBT_E_INVALID, "null gradient buffer");
  std::vector<double> ds(sigma_id >= 0 ? c->surfs[sigma_id]->nt : 0);
  std::vector<double> dq(mol_id >= 0 ? c->surfs[mol_id]->q.size() : 0);
  // both buffers checked before any work, so a bad pointer leaves nothing done
  pbt_status st = guarded(c, [&] {
    if (sigma_id >= 0 && !ds.empty()) check_dev_ptr(c, dF_dsigma_dev);
    if (mol_id >= 0 && !dq.empty()) check_dev_ptr(c, dF_dq_dev);
    return PBT_OK;
  });
  if (st != PBT_OK) return st;
  st = pbt_gradient(c, sigma_id, sigma_id >= 0 ? ds.data() : nullptr, mol_id, mol_id >= 0 ? dq.data() : nullptr);
  if (st != PBT_OK && st != PBT_E_NOCONVERGE) return st;
  const std::string msg = c->err;
  const pbt_status cp = guarded(c, [&] {
    const hipStream_t s = stream ? (hipStream_t)stream : c->stream;
    if (sigma_id >= 0) to_dev(c, dF_dsigma_dev, ds, s);
    if (mol_id >= 0) to_dev(c, dF_dq_dev, dq, s);
    return PBT_OK;
  });
  if (cp != PBT_OK) return cp;
  if (st != PBT_OK) c->err = msg;
  return st;
}

// Batched rigid placements (orientation sweep).  Up to kBatch assemblies are
// put into one block-diagonal system: group g holds the molecule moved by
// placement g and copies of every other enabled surface; interaction and
// near lists never cross groups, so each operator launch serves all of them
// and GMRES advances them in lock-step.  The global relative tolerance is
// tol / sqrt(G); every group's own relative residual is then checked and the
// solve continued (from its iterate) until each is below tol.  The isolated
// energies are computed once (the discrete problem of a rigidly moved body
// is the same problem up to rounding and, with the treecode, its tree).
pbt_status pbt_solve_batch(pbt_ctx* c, int32_t mol_id, const double* rot, const double* shift, int32_t nb,
                           double* F_int) {
  return tracked(c, [&] {
    const int ns = (int)c->surfs.size();
    if (mol_id < 0 || mol_id >= ns || c->surfs[mol_id]->kind != PBT_MOLECULE)
      return fail(c, PBT_E_INVALID, "mol_id must name a molecule");
    if (nb < 0 || (nb > 0 && (!rot || !shift || !F_int))) return fail(c, PBT_E_INVALID, "bad batch arrays");
    for (int64_t i = 0; i < 9LL * nb; ++i)
      if (!std::isfinite(rot[i])) return fail(c, PBT_E_INVALID, "non-finite rotation");
    for (int64_t i = 0; i < 3LL * nb; ++i)
      if (!std::isfinite(shift[i])) return fail(c, PBT_E_INVALID, "non-finite shift");
    if (nb == 0) return PBT_OK;
    std::vector<bool> saved = mask_of(c);
    auto restore = [&] { for (int i = 0; i < ns; ++i) c->surfs[i]->enabled = saved[i]; };
    // the moving component: the molecule with its Stern surface and cavities
    auto nested_in = [&](int i, int root) { return c->surfs[i]->parent == c->surfs[root].get(); };
    std::vector<char> moving(ns, 0);
    for (int i = 0; i < ns; ++i) moving[i] = i == mol_id || (saved[i] && nested_in(i, mol_id));
    std::vector<int> others;
    for (int i = 0; i < ns; ++i)
      if (saved[i] && !moving[i]) others.push_back(i);
    // isolated energies, once: one solve per component (a molecule with its
    // nested surfaces, or any other surface alone)
    double f_iso = 0.0;
    pbt_status worst = PBT_OK;
    const bool say = std::getenv("PBT_SETUP_TIMES") != nullptr;
    double tb = wall_now();
    auto phase = [&](const char* what) {
      if (!say) return;
      PBT_HIP(hipStreamSynchronize(c->stream));
      const double u = wall_now();
      std::fprintf(stderr, "[batch] %-16s %8.2f ms\n", what, 1e3 * (u - tb));
      tb = u;
    };
    try {
      std::vector<int> comps;
      for (int i = 0; i < ns; ++i)
        if ((i == mol_id || saved[i]) && c->surfs[i]->kind != PBT_STERN && c->surfs[i]->kind != PBT_CAVITY)
          comps.push_back(i);
      for (int k : comps) {
        for (int i = 0; i < ns; ++i) c->surfs[i]->enabled = i == k || (saved[i] && nested_in(i, k));
        pbt_result r{};
        pbt_status st = solve_impl(c, nullptr, &r);
        if (st != PBT_OK && st != PBT_E_NOCONVERGE) { restore(); return st; }
        if (st != PBT_OK) worst = st;
        f_iso += r.F_total;
      }
    } catch (...) {
      restore();
      throw;
    }
    restore();
    phase("isolated solves");
    const int kBatch = 64;
    std::vector<int> placed;   // the surfaces of one placement: the moving ones, then the others
    for (int i = 0; i < ns; ++i)
      if (moving[i]) placed.push_back(i);
    placed.insert(placed.end(), others.begin(), others.end());
    for (int b0 = 0; b0 < nb; b0 += kBatch) {
      const int G = std::min(kBatch, nb - b0);
      std::vector<std::unique_ptr<SurfIn>> own;
      std::vector<const SurfIn*> list;
      for (int g = 0; g < G; ++g) {
        const double* R = rot + 9 * (int64_t)(b0 + g);
        const double* t = shift + 3 * (int64_t)(b0 + g);
        auto mv = [&](const std::vector<double>& in) {
          std::vector<double> o(in.size());
          for (size_t i = 0; i + 2 < in.size(); i += 3)
            for (int d = 0; d < 3; ++d)
              o[i + d] = R[3 * d] * in[i] + R[3 * d + 1] * in[i + 1] + R[3 * d + 2] * in[i + 2] + t[d];
          return o;
        };
        std::vector<std::pair<const SurfIn*, SurfIn*>> copies;   // original -> this placement's copy
        for (int k : placed) {
          const SurfIn& S0 = *c->surfs[k];
          auto o = std::make_unique<SurfIn>(S0);
          if (moving[k]) {
            o->xyz = mv(S0.xyz);
            o->qxyz = mv(S0.qxyz);
          }
          o->group = g;
          o->shared = moving[k] ? -1 : k;
          copies.push_back({&S0, o.get()});
          list.push_back(o.get());
          own.push_back(std::move(o));
        }
        // nested surfaces point at their molecule's copy in the same placement
        for (auto& cp : copies)
          if (cp.second->parent)
            for (auto& q : copies)
              if (q.first == cp.second->parent) cp.second->parent = q.second;
      }
      phase("placements");
      const double ts = wall_now();
      System S(list, c->prm, c->eps_out, c->kappa, c->stream);
      c->cs.t_setup += wall_now() - ts;
      phase("system");
      if (c->profile) S.set_profile(true);
      const int64_t n = S.n();
      DBuf<double> b, x;
      b.alloc(n);
      x.alloc(n);
      S.rhs(b.p, c->stream);
      phase("rhs");
      // one Krylov space per placement, each to the requested tolerance
      pbt_result r{};
      if (!S.solve(b.p, x.p, false, &r, c->stream)) worst = PBT_E_NOCONVERGE;
      phase("solve");
      c->cs.iters = std::max(c->cs.iters, r.iters);
      std::vector<pbt_result> e = S.energies_by_group(x.p, G, c->stream);
      for (int g = 0; g < G; ++g) F_int[b0 + g] = e[g].F_total - f_iso;
      phase("energies");
      stats_account(c, S, 0, 0);
      if (c->profile) S.add_profile(c->prof_batch);
    }
    if (worst != PBT_OK) return fail(c, worst, "a batched solve did not reach the tolerance");
    return PBT_OK;
  });
}

// Autotuner: times the operator of the enabled system for candidate P2P and
// M2P segment sizes (coordinate search: P2P first, then M2P) and then for
// the four schedules of the far field against P2P, in the solve's
// interaction precision, keeps the fastest, and remembers it per system
// shape in memory and, if given, in a text cache file
// ("key seg_src 4*seg_box+schedule ms" per line).
constexpr int kFarModes = 7;        // far-field schedules (System::set_far_mode)
constexpr int kTunedFarModes = 4;   // the ones the autotuner tries

pbt_status pbt_autotune(pbt_ctx* c, const char* cache_path) {
  return guarded(c, [&] {
    System& S = system_for(c);
    const bool fp32 = c->prm.prec == PBT_MIXED;
    char key[256];
    std::snprintf(key, sizeof key, "np%lld_n%lld_p2p%lld_m2p%lld_P%d_%s", (long long)S.np(), (long long)S.n(),
                  (long long)S.plan().p2p_pairs, (long long)S.plan().m2p_pairs, c->prm.taylor_p,
                  fp32 ? "fp32" : "fp64");
    static std::map<std::string, std::pair<int64_t, int64_t>> memo;
    auto it = memo.find(key);
    if (it == memo.end() && cache_path) {
      if (FILE* f = std::fopen(cache_path, "r")) {
        char k[256];
        long long a, b;
        double ms;
        while (std::fscanf(f, "%255s %lld %lld %lf", k, &a, &b, &ms) == 4)
          if (std::string(k) == key) memo[key] = {a, b};
        std::fclose(f);
        it = memo.find(key);
      }
    }
    if (it != memo.end()) {
      S.set_segments(it->second.first, it->second.second / 8, c->stream);
      S.set_far_mode((int)(it->second.second % 8));
      return PBT_OK;
    }
    // each candidate: the better of two averages of `reps` products, which
    // rejects one-off slow measurements
    const int reps = 5;
    auto timed = [&] {
      const double a = S.time_products(fp32, reps, c->stream);
      return std::min(a, S.time_products(fp32, reps, c->stream));
    };
    // two sweeps of coordinate search over (P2P segment, M2P segment,
    // schedule): the schedule found in the first sweep can prefer other
    // segment lengths.  Each phase re-times the incumbent first, so a lucky
    // earlier measurement does not keep it.
    int64_t best_src = S.seg_src(), best_box = S.seg_box();
    int best_mode = S.far_mode();
    double best = 0.0;
    for (int sweep = 0; sweep < 2; ++sweep) {
      S.set_segments(best_src, best_box, c->stream);
      best = timed();
      for (int64_t cand : {64, 96, 128, 192, 256, 384, 512, 1024, 2048}) {
        if (cand == best_src) continue;
        S.set_segments(cand, best_box, c->stream);
        const double t = timed();
        if (t < best) { best = t; best_src = cand; }
      }
      S.set_segments(best_src, best_box, c->stream);
      best = timed();
      for (int64_t cand : {1, 2, 4, 8, 16, 32}) {
        if (cand == best_box) continue;
        S.set_segments(best_src, cand, c->stream);
        const double t = timed();
        if (t < best) { best = t; best_box = cand; }
      }
      S.set_segments(best_src, best_box, c->stream);
      // scheduling of the far field against P2P (serial, two streams, joint
      // launch, moments inside P2P).  The split schedules 4-6 are not
      // candidates: their joint launch runs P2P at the M2P kernel's
      // occupancy, which the FP64 products (same schedule) pay for, and they
      // were not faster in the FP32 products either.  The schedules are
      // timed round-robin, three rounds, each keeping its best time, so a
      // drift of the clocks during the search favours none of them.
      double tm[kTunedFarModes];
      for (double& v : tm) v = 1e30;
      for (int round = 0; round < 3; ++round)
        for (int mode = 0; mode < kTunedFarModes; ++mode) {
          S.set_far_mode(mode);
          tm[mode] = std::min(tm[mode], timed());
        }
      best_mode = 0;
      for (int mode = 1; mode < kTunedFarModes; ++mode)
        if (tm[mode] < tm[best_mode]) best_mode = mode;
      // a schedule less than 3 % faster than the serial one is within the
      // spread of the timings: the serial schedule, where each kernel has
      // the machine to itself, is kept
      if (tm[0] <= 1.03 * tm[best_mode]) best_mode = 0;
      best = tm[best_mode];
      S.set_far_mode(best_mode);
    }
    S.set_far_mode(best_mode);
    memo[key] = {best_src, best_box * 8 + best_mode};
    if (cache_path) {
      if (FILE* f = std::fopen(cache_path, "a")) {
        std::fprintf(f, "%s %lld %lld %.6f\n", key, (long long)best_src, (long long)(best_box * 8 + best_mode), best);
        std::fclose(f);
      }
    }
    return PBT_OK;
  });
}

pbt_status pbt_last_stats(pbt_ctx* c, pbt_result* out) {
  if (!c || !out) return PBT_E_INVALID;
  *out = c->last_stats;
  return PBT_OK;
}

pbt_status pbt_set_schedule(pbt_ctx* c, int32_t mode) {
  if (!c) return PBT_E_INVALID;
  if (mode < 0 || mode >= kFarModes) return fail(c, PBT_E_INVALID, "schedule must be 0..6");
  return guarded(c, [&] {
    system_for(c).set_far_mode(mode);
    return PBT_OK;
  });
}

pbt_status pbt_get_schedule(pbt_ctx* c, int32_t* mode) {
  if (!c || !mode) return PBT_E_INVALID;
  return guarded(c, [&] {
    *mode = system_for(c).far_mode();
    return PBT_OK;
  });
}

pbt_status pbt_get_launch_shape(pbt_ctx* c, int64_t* out) {
  if (!c || !out) return PBT_E_INVALID;
  return guarded(c, [&] {
    System& S = system_for(c);
    const int64_t npairs = (int64_t)S.plan().p2p.size() / 2, nm2p = (int64_t)S.plan().m2p.size() / 2;
    out[0] = S.seg_src();
    out[1] = S.seg_box();
    out[2] = ((npairs + 3) / 4 + 7) / 8 * 8 * 256;
    out[3] = ((nm2p + 3) / 4 + 7) / 8 * 8 * 256;
    return PBT_OK;
  });
}

pbt_status pbt_set_gram_schmidt(pbt_ctx* c, int32_t passes) {
  if (!c) return PBT_E_INVALID;
  if (passes < 0 || passes > 2) return fail(c, PBT_E_INVALID, "Gram-Schmidt passes must be 0, 1 or 2");
  c->gs_passes = passes;
  return PBT_OK;
}

pbt_status pbt_quadrature_rule(int32_t npts, double* bary, double* w) {
  if (!bary || !w) return PBT_E_INVALID;
  std::vector<double> b, ww;
  if (npts < 0) {
    if (npts < -64) return PBT_E_INVALID;
    gauss_legendre01(-npts, b, ww);
  } else if (!triangle_rule(npts, b, ww)) {
    return PBT_E_INVALID;
  }
  std::memcpy(bary, b.data(), b.size() * sizeof(double));
  std::memcpy(w, ww.data(), ww.size() * sizeof(double));
  return PBT_OK;
}

pbt_status pbt_last_matvec_timing(pbt_ctx* c, double out[5]) {
  return guarded(c, [&] {
    if (!out) return fail(c, PBT_E_INVALID, "null buffer");
    System& S = system_for(c);
    S.timing(out);
    return PBT_OK;
  });
}

pbt_status pbt_profile(pbt_ctx* c, int32_t on) {
  if (!c) return PBT_E_INVALID;
  return guarded(c, [&] {
    c->profile = on != 0;
    for (auto& kv : c->systems) kv.second->set_profile(c->profile);
    for (double& v : c->prof_batch) v = 0.0;
    return PBT_OK;
  });
}

pbt_status pbt_kernel_times(pbt_ctx* c, double* out) {
  if (!c || !out) return fail(c, PBT_E_INVALID, "null argument");
  return guarded(c, [&] {
    for (int k = 0; k < 16; ++k) out[k] = c->prof_batch[k];
    for (auto& kv : c->systems) kv.second->add_profile(out);
    return PBT_OK;
  });
}

}  // extern "C"
