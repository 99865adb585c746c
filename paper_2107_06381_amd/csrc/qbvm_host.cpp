// Host executor of the PinT quasi-boundary value solver: FFT planning, plans,
// solve orchestration, regularisation-parameter choice, batched graphs, C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/qbvm.h"
#include "qbvm_fft_plan.hpp"
#include "qbvm_internal.hpp"
#include "qbvm_schedule.hpp"

using namespace qbvm;
using qbvm::sched::Launch;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

static int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess) {                                                                \
      return set_error(_e == hipErrorOutOfMemory ? QBVM_ENOMEM : QBVM_EHIP,                \
                       std::string(#expr) + ": " + hipGetErrorString(_e));                 \
    }                                                                                      \
  } while (0)

// ------------------------------------------------------------- FFT planning
namespace {

constexpr long double kPiL = 3.141592653589793238462643383279502884L;
constexpr int kThreads = 256;

struct FftTables {
  FftPlanDev dev{};
  std::vector<void*> allocs;
};

template <class T>
hipError_t upload(const std::vector<T>& v, const T** dst, std::vector<void*>& allocs) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(1, v.size()) * sizeof(T));
  if (e != hipSuccess) return e;
  allocs.push_back(p);
  if (!v.empty()) e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  *dst = static_cast<const T*>(p);
  return e;
}

// Build the device tables of a forward DFT of logical length n.
int build_fft(int n, FftTables& t, bool sine) {
  plan::HostFft h;
  std::string err;
  if (!plan::build_tables(n, h, err, sine)) return set_error(QBVM_EUNSUPPORTED, err);
  t.dev = h.dev;
  FftPlanDev& d = t.dev;
  HIP_TRY(upload(h.tw, &d.tw, t.allocs));
  HIP_TRY(upload(h.kspec, &d.kspec, t.allocs));
  HIP_TRY(upload(h.chirp, &d.chirp, t.allocs));
  HIP_TRY(upload(h.rin, &d.rin, t.allocs));
  HIP_TRY(upload(h.rout, &d.rout, t.allocs));
  HIP_TRY(upload(h.gfwd, &d.gfwd, t.allocs));
  HIP_TRY(upload(h.ginvt, &d.ginvt, t.allocs));
  return QBVM_OK;
}

std::mutex g_mu;
std::map<std::tuple<int, int, bool>, std::unique_ptr<FftTables>> g_fft_cache;  // (device, n, sine)
// tuned variants: (device, role 0 rows / 1 cols / 2 time, N) -> variant
std::map<std::tuple<int, int, int>, int> g_tuned;
std::map<int, bool> g_roots_ready;

// sine: tables of a sine transform's length-n DFT (n = 2(m+1)); a Bluestein length gets
// the symmetric form of the compile-time Bluestein sine passes
int get_fft(int device, int n, const FftTables** out, bool sine = false) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_roots_ready[device]) {
    const std::vector<c64> roots = plan::radix_roots();
    upload_radix_roots(roots.data(), (int)roots.size());
    HIP_TRY(hipGetLastError());
    g_roots_ready[device] = true;
  }
  auto key = std::make_tuple(device, n, sine);
  auto it = g_fft_cache.find(key);
  if (it == g_fft_cache.end()) {
    auto t = std::make_unique<FftTables>();
    const int rc = build_fft(n, *t, sine);
    if (rc != QBVM_OK) {
      for (void* p : t->allocs) (void)hipFree(p);
      return rc;
    }
    it = g_fft_cache.emplace(key, std::move(t)).first;
  }
  *out = it->second.get();
  return QBVM_OK;
}



}  // namespace


// ------------------------------------------------------------- profiling
namespace {

struct ProfPending {
  int kind;
  hipEvent_t a, b;
  double bytes, flops;
};
struct ProfAgg {
  std::string name;
  long long n = 0;
  double ms = 0, bytes = 0, flops = 0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfPending> g_pending;
std::vector<ProfAgg> g_agg;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t prof_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

int prof_kind(const char* name) {
  for (size_t i = 0; i < g_agg.size(); ++i)
    if (g_agg[i].name == name) return (int)i;
  g_agg.push_back(ProfAgg{name});
  return (int)g_agg.size() - 1;
}

// Brackets one direct launch with events when profiling is on (never for graph nodes).
struct ProfScope {
  bool on = false;
  ProfPending p{};
  hipStream_t s = nullptr;
  ProfScope(const char* name, hipStream_t stream, double bytes, double flops, const NodeCtx* nc) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on || nc) return;
    on = true;
    s = stream;
    p.kind = prof_kind(name);
    p.a = prof_event();
    p.b = prof_event();
    p.bytes = bytes;
    p.flops = flops;
    (void)hipEventRecord(p.a, s);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(p.b, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_pending.push_back(p);
  }
};

double fft_flops(const FftPlanDev& f) {
  const double core = 5.0 * f.nc * std::log2((double)f.nc);
  return f.kind == kStockham ? core : 2.0 * core + 6.0 * f.nc;
}

}  // namespace

extern "C" void qbvm_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
}

extern "C" void qbvm_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& p : g_pending) {
    (void)hipEventSynchronize(p.b);
    g_event_pool.push_back(p.a);
    g_event_pool.push_back(p.b);
  }
  g_pending.clear();
  g_agg.clear();
}

extern "C" int qbvm_profile_count(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& p : g_pending) {
    (void)hipEventSynchronize(p.b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p.a, p.b);
    ProfAgg& a = g_agg[p.kind];
    a.n += 1;
    a.ms += ms;
    a.bytes += p.bytes;
    a.flops += p.flops;
    g_event_pool.push_back(p.a);
    g_event_pool.push_back(p.b);
  }
  g_pending.clear();
  return (int)g_agg.size();
}

extern "C" int qbvm_profile_get(int i, char* name_buf, int buf_len, long long* launches, double* total_ms,
                                double* bytes, double* flops) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (i < 0 || i >= (int)g_agg.size()) return set_error(QBVM_EINVAL, "profile index out of range");
  const ProfAgg& a = g_agg[i];
  if (name_buf && buf_len > 0) {
    std::strncpy(name_buf, a.name.c_str(), buf_len - 1);
    name_buf[buf_len - 1] = 0;
  }
  if (launches) *launches = a.n;
  if (total_ms) *total_ms = a.ms;
  if (bytes) *bytes = a.bytes;
  if (flops) *flops = a.flops;
  return QBVM_OK;
}

// ------------------------------------------------------------------ plans
struct qbvm_plan_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int d = 0, m = 0, n = 0, Nt = 0;
  double L = 1, T = 1, h = 0, tau = 0, hd = 0;
  long long nmodes = 0;
  const FftTables* tfft = nullptr;  // length N_t
  const FftTables* sfft = nullptr;  // length 2(m+1)
  int S_time = 1, S_dst = 1;
  int var_rows = 5, var_cols = 6, var_time = 4;  // set per transform length in create_plan
  int var_gen = 1;                                // time kernel of the general right-hand side
  bool plane = true;  // plane pass (x_2 and x_1 together) where the shape allows it
  int var_plane = 0;  // plane-pass variant
  double* mu1d = nullptr;
  double* ghat = nullptr;
  double* yrow = nullptr;
  c64* s2 = nullptr;
  double* W = nullptr;  // padded level workspace (d >= 2 power-of-two pipeline)
  c64* tabs = nullptr;  // per-solve time-transform tables, 3 N_t
  double* op = nullptr;  // 1D spatial operator: [m-1] lower, [m] diagonal, [m-1] upper (3m doubles)
  bool has_op = false;
  // 2D/3D operator -div(kappa grad u): Step (b) by batched preconditioned COCG
  bool kop = false;
  double* kx = nullptr;  // faces between x_1 neighbours, m^(d-1) (m+1)
  double* ky = nullptr;  // between x_2 neighbours
  double* kz = nullptr;  // 3D: between x_3 neighbours
  double kbar = 1.0, kry_tol = 1e-12;
  int kry_maxit = 200;
  int kry_H = 0, kry_nblk = 0;
  double* kry = nullptr;       // x, r, z, p, p', q: 6 vectors of 2 H m^2 doubles
  double* kry_part = nullptr;  // [3][H][nblk] complex partial sums
  double* kry_sys = nullptr;   // [H][8] per-system scalars
  int kry_iters = 0, kry_breakdowns = 0;
  double kry_relres = 0.0;
  bool no_sine = false;  // 1D only: the sine transform of length 2(m+1) exceeds the FFT core
  double* partial = nullptr;
  unsigned* counter = nullptr;
  double* dscal = nullptr;   // [0] delta, [1] alpha_pred, [2] log10 alpha_pred, [3] D, [4] alpha_final, ...
  double* bstate = nullptr;  // kBState doubles
  float* feats = nullptr;
  float* model = nullptr;
  bool has_model = false;
  int* bin_perm = nullptr;
  int* bin_off = nullptr;
  // result mailbox: coherent mapped host memory the final row kernel writes into
  double* mbox = nullptr;      // host view, 8 doubles
  double* mbox_dev = nullptr;  // device view
  double mbox_seq = 0.0;
  int wg_row = 1;
  // grow-only batch workspace
  double* bws = nullptr;
  size_t bws_bytes = 0;
  long long bytes = 0;
  std::vector<void*> allocs;
};

namespace {

template <class T>
hipError_t dalloc(qbvm_plan_s* p, T** out, size_t count) {
  void* q = nullptr;
  const size_t b = std::max<size_t>(1, count) * sizeof(T);
  hipError_t e = hipMalloc(&q, b);
  if (e != hipSuccess) return e;
  p->allocs.push_back(q);
  p->bytes += (long long)b;
  *out = static_cast<T*>(q);
  return hipSuccess;
}

int validate_grid(const qbvm_grid* g) {
  if (!g) return set_error(QBVM_EINVAL, "grid is NULL");
  if (g->d < 1 || g->d > 3) return set_error(QBVM_EINVAL, "d must be 1, 2 or 3");
  if (g->m < 1 || g->n < 1) return set_error(QBVM_EINVAL, "m and n must be >= 1");
  if (!(g->L > 0) || !(g->T > 0) || !std::isfinite(g->L) || !std::isfinite(g->T))
    return set_error(QBVM_EINVAL, "L and T must be positive and finite");
  const int mmax = g->d == 1 ? QBVM_MAX_M_1D : (g->d == 2 ? QBVM_MAX_M_2D : QBVM_MAX_M_3D);
  const int ntmax = g->d == 1 ? QBVM_MAX_NT : QBVM_MAX_NT_MD;
  if (g->m > mmax || g->n + 1 > ntmax) return set_error(QBVM_EUNSUPPORTED, "grid exceeds the size limits");
  return QBVM_OK;
}

// bins of the learned-alpha features (same arithmetic and order as the definition)
void feature_bins(int d, int m, std::vector<int>& perm, std::vector<int>& off) {
  long long nm = 1;
  for (int i = 0; i < d; ++i) nm *= m;
  std::vector<int> bin(nm);
  const double lo = std::sqrt((double)d), hi = (double)m * std::sqrt((double)d);
  for (long long k = 0; k < nm; ++k) {
    long long r = k, ksq = 0;
    for (int i = 0; i < d; ++i) {
      const long long q = r / m, ki = r - q * m + 1;
      ksq += ki * ki;
      r = q;
    }
    int b = 0;
    if (m > 1) {
      const double rho = std::sqrt((double)ksq);
      const double t = (rho - lo) / (hi - lo) * 32.0;
      b = (int)std::floor(t);
      b = std::min(31, std::max(0, b));
    }
    bin[k] = b;
  }
  off.assign(33, 0);
  for (long long k = 0; k < nm; ++k) off[bin[k] + 1]++;
  for (int b = 0; b < 32; ++b) off[b + 1] += off[b];
  perm.assign(nm, 0);
  std::vector<int> cur(off.begin(), off.end() - 1);
  for (long long k = 0; k < nm; ++k) perm[cur[bin[k]]++] = (int)k;
}

void destroy_plan(qbvm_plan_s* p) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  (void)hipStreamSynchronize(p->stream);
  for (void* q : p->allocs) (void)hipFree(q);
  if (p->bws) (void)hipFree(p->bws);
  if (p->mbox) (void)hipHostFree(p->mbox);
  (void)hipSetDevice(cur);
  delete p;
}

sched::Geom geom(const qbvm_plan_s* p);

int create_plan(qbvm_plan_s** out, const qbvm_grid* grid, hipStream_t stream) {
  *out = nullptr;
  int rc = validate_grid(grid);
  if (rc) return rc;
  auto* p = new (std::nothrow) qbvm_plan_s();
  if (!p) return set_error(QBVM_ENOMEM, "host allocation failed");
  std::unique_ptr<qbvm_plan_s, void (*)(qbvm_plan_s*)> guard(p, destroy_plan);
  HIP_TRY(hipGetDevice(&p->device));
  p->stream = stream;
  p->d = grid->d;
  p->m = grid->m;
  p->n = grid->n;
  p->Nt = grid->n + 1;
  p->L = grid->L;
  p->T = grid->T;
  p->h = grid->L / (grid->m + 1);
  p->tau = grid->T / grid->n;
  p->hd = std::pow(p->h, p->d);
  p->nmodes = 1;
  for (int i = 0; i < p->d; ++i) p->nmodes *= p->m;
  rc = get_fft(p->device, p->Nt, &p->tfft);
  if (rc) return rc;
  rc = get_fft(p->device, 2 * (p->m + 1), &p->sfft, true);
  if (rc == QBVM_EUNSUPPORTED && p->d == 1) {
    // the 1D solve never needs the sine transform (Step (b) is tridiagonal); only the
    // calls that work in the sine basis are refused on this plan
    static const FftTables kNoSine{};
    p->sfft = &kNoSine;
    p->no_sine = true;
    rc = QBVM_OK;
  }
  if (rc) return rc;
  p->S_time = plan::signals_for(p->tfft->dev.nc);
  p->S_dst = p->no_sine ? 1 : plan::signals_for(p->sfft->dev.nc);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto pick = [&](int role, int N, int& var) {
      auto it = g_tuned.find(std::make_tuple(p->device, role, N));
      if (it != g_tuned.end()) var = it->second;
    };
    // untuned defaults: the variants the autotuner keeps for these lengths on MI355X
    const int Ns = p->sfft->dev.p2, Nt2 = p->tfft->dev.p2;
    p->var_rows = Ns >= 512 ? 7 : 5;
    p->var_cols = Ns >= 512 ? 6 : 1;
    p->var_time = (Nt2 && Nt2 <= 256) ? 5 : 4;
    pick(0, p->sfft->dev.p2, p->var_rows);
    pick(1, p->sfft->dev.p2, p->var_cols);
    pick(2, p->tfft->dev.p2, p->var_time);
    if (p->tfft->dev.gtA) {
      p->var_time = 1;
      pick(3, p->Nt, p->var_time);
    }
    p->var_gen = 1;
    pick(4, p->tfft->dev.p2, p->var_gen);
  }
  // eigenvalues of the 1D three-point stencil: (4/h^2) sin^2(k pi/(2(m+1)))
  std::vector<double> mu(p->m);
  for (int k = 1; k <= p->m; ++k) {
    const long double s = sinl((long double)k * kPiL / (2.0L * (p->m + 1)));
    mu[k - 1] = (double)(4.0L / ((long double)p->h * p->h) * s * s);
  }
  HIP_TRY(dalloc(p, &p->mu1d, p->m));
  HIP_TRY(hipMemcpy(p->mu1d, mu.data(), sizeof(double) * p->m, hipMemcpyHostToDevice));
  HIP_TRY(dalloc(p, &p->ghat, p->nmodes));
  HIP_TRY(dalloc(p, &p->yrow, p->nmodes));
  if (p->d == 1) {
    HIP_TRY(dalloc(p, &p->s2, (size_t)p->Nt * p->m));
  }
  if (sched::use_padded(geom(p))) HIP_TRY(dalloc(p, &p->W, (size_t)sched::padded_elems(geom(p))));
  HIP_TRY(dalloc(p, &p->tabs, 3 * (size_t)p->Nt));
  // four lanes per mode in the row kernel (64 modes per 256-lane workgroup)
  p->wg_row = (int)std::max<long long>(1, std::min<long long>(4096, (p->nmodes + 63) / 64));
  HIP_TRY(dalloc(p, &p->partial, std::max<long long>(p->wg_row, 32)));  // row reduction; 32 feature bins
  HIP_TRY(dalloc(p, &p->counter, 1));
  HIP_TRY(hipMemset(p->counter, 0, sizeof(unsigned)));
  HIP_TRY(dalloc(p, &p->dscal, 16));
  HIP_TRY(dalloc(p, &p->bstate, kBState));
  HIP_TRY(dalloc(p, &p->feats, 33));
  HIP_TRY(dalloc(p, &p->model, QBVM_MODEL_FLOATS));
  std::vector<int> perm, off;
  feature_bins(p->d, p->m, perm, off);
  HIP_TRY(dalloc(p, &p->bin_perm, perm.size()));
  HIP_TRY(dalloc(p, &p->bin_off, off.size()));
  HIP_TRY(hipMemcpy(p->bin_perm, perm.data(), sizeof(int) * perm.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->bin_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipHostMalloc((void**)&p->mbox, 8 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
  for (int i = 0; i < 8; ++i) p->mbox[i] = 0.0;
  HIP_TRY(hipHostGetDevicePointer((void**)&p->mbox_dev, p->mbox, 0));
  guard.release();
  *out = p;
  return QBVM_OK;
}

sched::Geom geom(const qbvm_plan_s* p) {
  sched::Geom g{};
  g.d = p->d;
  g.m = p->m;
  g.n = p->n;
  g.Nt = p->Nt;
  g.h = p->h;
  g.tau = p->tau;
  g.nmodes = p->nmodes;
  g.S_time = p->S_time;
  g.S_dst = p->S_dst;
  g.tfft = p->tfft->dev;
  g.sfft = p->sfft->dev;
  g.mu1d = p->mu1d;
  g.var_rows = p->var_rows;
  g.var_cols = p->var_cols;
  g.var_time = p->var_time;
  return g;
}

// d passes of the orthonormal DST-I over a [batch][m]^d array
// input_transform: the data are g_delta (one or a batch of instances), else solution levels
// tab (optional): per-solve time tables computed as side work of the last pass
// (power-of-two passes only; returns QBVM_EUNSUPPORTED before enqueueing otherwise)
int run_dst(const qbvm_plan_s* p, const double* in, double* out, long long batch, bool input_transform,
            NodeCtx* nc = nullptr, hipStream_t stream = nullptr, const TabJob* tab = nullptr) {
  if (p->no_sine) return set_error(QBVM_EUNSUPPORTED, "sine transform of length 2(m+1) exceeds the FFT core");
  hipStream_t s = nc ? stream : p->stream;
  auto passes = sched::dst_passes(geom(p), in, out, batch, input_transform);
  if (tab) {
    if (!passes.back().args.fft.p2) return QBVM_EUNSUPPORTED;
    passes.back().args.tab = *tab;
  }
  for (const auto& L : passes) {
    const double elems = (double)L.args.outer * L.args.inner * L.args.len;
    const int role = input_transform ? 0 : (L.args.inner == 1 ? 1 : 2);
    static const char* names[3] = {"dst_input", "dst_rows", "dst_cols"};
    ProfScope ps(names[role], s, 16.0 * elems, 0.5 * (double)L.args.outer * L.args.inner * fft_flops(L.args.fft),
                 nc);
    HIP_TRY(launch_dst(L.args, L.nwg, L.args.threads, L.lds, s, nc, role));
  }
  return QBVM_OK;
}

int check_alpha(double alpha, int variant) {
  if (!(alpha > 0) || !std::isfinite(alpha)) return set_error(QBVM_EINVAL, "alpha must be positive and finite");
  if (variant != QBVM_PQ && variant != QBVM_PM) return set_error(QBVM_EINVAL, "variant must be QBVM_PQ or QBVM_PM");
  return QBVM_OK;
}

// Enqueue one full solve (every level).  alpha_dev (optional) overrides alpha.
// W: padded workspace for the aligned pipeline (nullptr: in-place pipeline in y).
int enqueue_full(const qbvm_plan_s* p, double alpha, const double* alpha_dev, int variant, const double* g,
                 double* y, c64* s2, NodeCtx* nc, hipStream_t stream, double* W = nullptr) {
  const sched::Geom G = geom(p);
  const SolveScalars sc = sched::host_scalars(alpha, variant, p->tau);
  if (W && p->d >= 2 && sched::use_padded(G)) {
    // the last input pass also fills the per-solve time tables (one launch fewer)
    const TabJob job{p->tabs, p->Nt, variant, p->tau, alpha, alpha_dev};
    int rc = run_dst(p, g, p->ghat, 1, true, nc, stream, &job);
    if (rc) return rc;
    auto t = sched::time_step_padded(G, sc, alpha_dev, variant, p->ghat, W);
    t.args.tabs = p->tabs;
    {
      const double nm = (double)p->nmodes;
      ProfScope ps("time_spectral", stream, 8.0 * nm * (1.0 + p->Nt),
                   0.5 * nm * (fft_flops(p->tfft->dev) + 28.0 * p->Nt), nc);
      HIP_TRY(launch_time(t.args, t.nwg, t.args.threads, t.lds, stream, nc));
    }
    if (p->plane && sched::use_plane(G)) {
      const double elems = (double)p->Nt * p->nmodes;
      for (const auto& L : sched::plane_pre_passes(G, W)) {
        ProfScope ps("dst_cols", stream, 16.0 * elems, 0.5 * elems / p->m * fft_flops(p->sfft->dev), nc);
        HIP_TRY(launch_dst(L.args, L.nwg, L.args.threads, L.lds, stream, nc, 2));
      }
      const PlaneArgs pa = sched::plane_args(G, W, y);
      ProfScope ps("dst_plane", stream, 16.0 * elems, elems / p->m * fft_flops(p->sfft->dev), nc);
      HIP_TRY(launch_plane(pa, p->var_plane, stream, nc));
      return QBVM_OK;
    }
    const auto passes = sched::padded_passes(G, W, y);
    for (size_t i = 0; i < passes.size(); ++i) {
      const bool rows = i + 1 == passes.size();
      const double elems = (double)p->Nt * p->nmodes;
      ProfScope ps(rows ? "dst_rows" : "dst_cols", stream, 16.0 * elems,
                   0.5 * (double)p->Nt * p->nmodes / p->m * fft_flops(p->sfft->dev), nc);
      HIP_TRY(launch_dst(passes[i].args, passes[i].nwg, passes[i].args.threads, passes[i].lds, stream, nc,
                         rows ? 1 : 2));
    }
    return QBVM_OK;
  }
  if (p->d == 1) {
    const double cells = (double)p->Nt * p->m;
    {
      ProfScope ps("tridiag_1d", stream, 8.0 * p->m + 16.0 * cells, 150.0 * cells, nc);
      auto ta = sched::thomas_step(G, sc, alpha_dev, variant, g, s2);
      if (p->has_op) {
        ta.args.op_lo = p->op;
        ta.args.op_di = p->op + p->m;
        ta.args.op_up = p->op + 2 * p->m;
      }
      // a single solve owns the plan's tables: the time kernel's gamma table is side work
      // here; batched instances may share a plan concurrently and keep it in LDS
      if (!nc) ta.args.tab = TabJob{p->tabs, p->Nt, variant, p->tau, alpha, alpha_dev, 1};
      HIP_TRY(launch_thomas(ta.args, ta.nwg, ta.lds, stream, nc));
    }
    auto t = sched::time1d_step(G, sc, alpha_dev, variant, s2, y);
    if (!nc) {
      t.args.gitab = p->tabs;
      t.lds = sched::lds_time1d(G, 0);
    }
    ProfScope ps("time_1d", stream, 24.0 * cells, 0.5 * p->m * (fft_flops(p->tfft->dev) + 8.0 * p->Nt), nc);
    HIP_TRY(launch_time1d(t.args, t.nwg, kThreads, t.lds, stream, nc));
    return QBVM_OK;
  }
  // g_hat = Q g_delta, kept in the level-0 slot of y (each time tile reads only its own modes)
  int rc = run_dst(p, g, y, 1, true, nc, stream);
  if (rc) return rc;
  const auto t = sched::time_step(G, sc, alpha_dev, variant, y, y, 0, p->Nt);
  {
    const double nm = (double)p->nmodes;
    ProfScope ps("time_spectral", stream, 8.0 * nm * (1.0 + p->Nt),
                 0.5 * nm * (fft_flops(p->tfft->dev) + 28.0 * p->Nt), nc);
    HIP_TRY(launch_time(t.args, t.nwg, t.args.threads, t.lds, stream, nc));
  }
  return run_dst(p, y, y, p->Nt, false, nc, stream);
}

// one level of Step (c) per mode; optional mode output and discrepancy reduction
int enqueue_row(const qbvm_plan_s* p, int count, const double* ghat, int level, double alpha,
                const double* alpha_dev, int variant, double* yrow, bool reduce, double* bstate, int mode,
                double* dout, double* partial, unsigned* counter, int wg_per_inst, double* host_out = nullptr,
                const double* report_bs = nullptr, double host_seq = 0.0) {
  RowArgs r{};
  r.Nt = p->Nt;
  r.d = p->d;
  r.m = p->m;
  r.level = level;
  r.count = count;
  r.nmodes = p->nmodes;
  r.tau = p->tau;
  r.hd = p->hd;
  r.variant = variant;
  r.mu1d = p->mu1d;
  r.ghat = ghat;
  r.yrow = yrow;
  r.partial = reduce ? partial : nullptr;
  r.counter = counter;
  r.wg_per_inst = wg_per_inst;
  r.alpha = alpha;
  r.alpha_dev = alpha_dev;
  r.bstate = bstate;
  r.mode = mode;
  r.dout = dout;
  r.host_out = host_out;
  r.report_bs = report_bs;
  r.host_seq = host_seq;
  const size_t lds = sizeof(c64) * 2 * p->Nt;
  ProfScope ps("dft_row", p->stream, 8.0 * count * p->nmodes * (yrow ? 2.0 : 1.0),
               14.0 * count * (double)p->nmodes * p->Nt, nullptr);
  HIP_TRY(launch_row(r, (long long)count * wg_per_inst, kThreads, lds, p->stream));
  return QBVM_OK;
}

// Full or single-level solve with the 2D/3D operator -div(kappa grad u): Step (a) is the
// broadcast of f0 (rank one), Step (b) the batched preconditioned COCG over the shifts
// j < H (w_{N_t-1-j} = conj w_j: A, f0 real, d_{N_t-1-j} = conj d_j), Step (c) the
// inverse time transform per pair of points.  g is f0 up to the factor f0s, which the
// per-solve gamma table carries.  Synchronous.
int kop_solve(qbvm_plan_s* p, double alpha, int variant, const double* g, double* y, int lev_first,
              int lev_count) {
  const int H = p->kry_H, Nt = p->Nt;
  const long long M = p->nmodes;
  const size_t V = 2 * (size_t)H * (size_t)M;
  std::vector<double> gh((size_t)M);
  HIP_TRY(hipMemcpyAsync(gh.data(), g, sizeof(double) * (size_t)M, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  double gn2 = 0.0;
  for (double v : gh) gn2 += v * v;
  if (!std::isfinite(gn2)) return set_error(QBVM_EINVAL, "g_delta is not finite");
  p->kry_iters = 0;
  p->kry_relres = 0.0;
  p->kry_breakdowns = 0;
  if (gn2 == 0.0) {
    HIP_TRY(hipMemsetAsync(y, 0, sizeof(double) * (size_t)lev_count * (size_t)M, p->stream));
    return QBVM_OK;
  }
  HIP_TRY(launch_tab_job(TabJob{p->tabs, Nt, variant, p->tau, alpha, nullptr, 0}, p->stream));
  KrylovArgs a{};
  a.d = p->d;
  a.m = p->m;
  a.H = H;
  a.nblk = p->kry_nblk;
  a.ppt = kKryPointsPerLane;
  a.M = M;
  a.ih2 = 1.0 / (p->h * p->h);
  a.kbar = p->kbar;
  a.tol2 = p->kry_tol * p->kry_tol * gn2;
  a.kx = p->kx;
  a.ky = p->ky;
  a.kz = p->kz;
  a.mu1d = p->mu1d;
  a.shift = p->tabs;
  a.g = g;
  a.x = p->kry;
  a.r = p->kry + V;
  a.z = p->kry + 2 * V;
  double* pbuf[2] = {p->kry + 3 * V, p->kry + 4 * V};
  a.q = p->kry + 5 * V;
  a.part = p->kry_part;
  a.sys = p->kry_sys;
  // z = P^{-1} r: sine transform, division by s_j + kbar mu_k (with the partial sums of
  // r^T z), inverse sine transform (the orthonormal transform is its own inverse)
  const double hm = (double)H * (double)M;  // complex unknowns of Step (b)
  auto step = [&](int which, const char* name, double bytes_per) -> int {
    ProfScope ps(name, p->stream, bytes_per * hm, 0.0, nullptr);
    HIP_TRY(launch_krylov(a, which, p->stream));
    return QBVM_OK;
  };
  auto precond = [&]() -> int {
    int rc = run_dst(p, a.r, a.z, 2LL * H, false);
    if (rc) return rc;
    rc = step(kKryPrecond, "kry_precond", 32.0);  // z read and written
    if (rc) return rc;
    return run_dst(p, a.z, a.z, 2LL * H, false);
  };
  a.init = 1;
  a.pin = a.z;  // first direction p = z (beta = 0)
  a.pout = pbuf[0];
  HIP_TRY(launch_krylov(a, kKryInit, p->stream));
  int rc = precond();
  if (rc) return rc;
  HIP_TRY(launch_krylov(a, kKryScalars, p->stream));
  a.init = 0;
  std::vector<double> sys((size_t)H * 8);
  int active = H;
  for (int it = 1; it <= p->kry_maxit && active > 0; ++it) {
    rc = step(kKryApply, "kry_apply", 64.0);  // z, p in; p, q out
    if (rc) return rc;
    rc = step(kKryUpdate, "kry_update", 96.0);  // x, r, p, q in; x, r out
    if (rc) return rc;
    rc = precond();
    if (rc) return rc;
    HIP_TRY(launch_krylov(a, kKryScalars, p->stream));
    HIP_TRY(hipMemcpyAsync(sys.data(), a.sys, sizeof(double) * sys.size(), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->kry_iters = it;
    active = 0;
    for (int j = 0; j < H; ++j) active += sys[(size_t)j * 8 + 7] == 1.0;
    a.pin = a.pout;
    a.pout = a.pout == pbuf[0] ? pbuf[1] : pbuf[0];
  }
  double worst = 0.0;
  int breakdowns = 0;
  for (int j = 0; j < H; ++j) {
    worst = std::max(worst, std::sqrt(sys[(size_t)j * 8 + 6] / gn2));
    breakdowns += sys[(size_t)j * 8 + 7] == -1.0;
  }
  p->kry_relres = worst;
  p->kry_breakdowns = breakdowns;
  KryTimeArgs t{};
  t.Nt = Nt;
  t.H = H;
  t.S = p->S_time;
  t.lev_first = lev_first;
  t.lev_count = lev_count;
  t.M = M;
  t.w = a.x;
  t.gi = p->tabs + Nt;
  t.y = y;
  t.fft = p->tfft->dev;
  const long long nwg = (M + 2LL * t.S - 1) / (2LL * t.S);
  const size_t lds = sizeof(c64) * ((size_t)t.S * t.fft.nc + 2 * (size_t)t.S);
  {
    ProfScope ps("kry_time", p->stream, 16.0 * hm + 8.0 * (double)lev_count * (double)M,
                 0.5 * (double)M * fft_flops(p->tfft->dev), nullptr);
    HIP_TRY(launch_kry_time(t, nwg, lds, p->stream));
  }
  if (active > 0 || worst > p->kry_tol)
    return set_error(QBVM_ENOCONV, "diffusion operator: " + std::to_string(active) + " of " + std::to_string(H) +
                                       " shifted systems above tolerance after " + std::to_string(p->kry_iters) +
                                       " iterations (" + std::to_string(breakdowns) + " breakdowns)");
  return QBVM_OK;
}

// Wait until the final row kernel has posted sequence number seq in the mailbox
// (polling coherent host memory instead of a copy and a stream synchronisation);
// after 0.2 s of polling fall back to synchronising the stream.
int wait_mailbox(qbvm_plan_s* p, double seq) {
  volatile double* box = p->mbox;
  const auto t0 = std::chrono::steady_clock::now();
  for (unsigned spin = 0;; ++spin) {
    if (box[0] == seq) break;
    if ((spin & 1023u) == 1023u && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(200)) {
      HIP_TRY(hipStreamSynchronize(p->stream));
      if (box[0] != seq) return set_error(QBVM_EHIP, "result mailbox not written");
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return QBVM_OK;
}

// kappa at the faces of a d = 2 or 3 plan: each array has m^(d-1) (m+1) entries
int set_diffusion(qbvm_plan_s* p, int d, const double* kx, const double* ky, const double* kz, double tol,
                  int max_iter) {
  if (!kx) {
    p->kop = false;
    return QBVM_OK;
  }
  if (p->d != d) return set_error(QBVM_EINVAL, "the operator's dimension differs from the plan's");
  if (!ky || (d == 3 && !kz)) return set_error(QBVM_EINVAL, "ky (and kz in 3D) must not be NULL");
  if (!(tol > 0.0 && tol < 1.0)) return set_error(QBVM_EINVAL, "tol must lie in (0, 1)");
  if (max_iter < 1) return set_error(QBVM_EINVAL, "max_iter must be >= 1");
  if (p->m > kKryMaxM) return set_error(QBVM_EUNSUPPORTED, "diffusion operator: m above the stencil kernel's LDS tile");
  const int m = p->m;
  const size_t nf = (size_t)(p->nmodes / m) * (m + 1);
  double lo = INFINITY, hi = 0.0;
  for (const double* k : {kx, ky, kz}) {
    if (!k) continue;
    for (size_t i = 0; i < nf; ++i) {
      const double v = k[i];
      if (!(v > 0.0) || !std::isfinite(v)) return set_error(QBVM_EINVAL, "kappa must be positive and finite");
      lo = std::min(lo, v);
      hi = std::max(hi, v);
    }
  }
  const int H = (p->Nt + 1) / 2;
  const long long M = p->nmodes;
  const long long TP = (long long)kKryPointsPerLane * kKryThreads;
  const int nblk = (int)((M + TP - 1) / TP);
  HIP_TRY(hipStreamSynchronize(p->stream));  // solves in flight may still read the old operator
  if (!p->kx) {
    HIP_TRY(dalloc(p, &p->kx, nf));
    HIP_TRY(dalloc(p, &p->ky, nf));
    if (d == 3) HIP_TRY(dalloc(p, &p->kz, nf));
    HIP_TRY(dalloc(p, &p->kry, 12 * (size_t)H * (size_t)M));
    HIP_TRY(dalloc(p, &p->kry_part, 3 * 2 * (size_t)H * (size_t)nblk));
    HIP_TRY(dalloc(p, &p->kry_sys, 8 * (size_t)H));
  }
  HIP_TRY(hipMemcpy(p->kx, kx, sizeof(double) * nf, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->ky, ky, sizeof(double) * nf, hipMemcpyHostToDevice));
  if (d == 3) HIP_TRY(hipMemcpy(p->kz, kz, sizeof(double) * nf, hipMemcpyHostToDevice));
  p->kbar = 0.5 * (lo + hi);
  p->kry_tol = tol;
  p->kry_maxit = max_iter;
  p->kry_H = H;
  p->kry_nblk = nblk;
  p->kop = true;
  return QBVM_OK;
}
}  // namespace

// ======================================================================= ABI
extern "C" {

int qbvm_version(void) { return 1; }

const char* qbvm_strerror(int code) {
  switch (code) {
    case QBVM_OK: return "ok";
    case QBVM_EINVAL: return "invalid argument";
    case QBVM_ENOMEM: return "out of memory";
    case QBVM_EHIP: return "HIP runtime error";
    case QBVM_ENOROOT: return "discrepancy principle has no root in the bracket";
    case QBVM_EUNSUPPORTED: return "unsupported size";
    case QBVM_ENOMODEL: return "no learned-alpha model attached to the plan";
    case QBVM_ENOCONV: return "iterative Step (b) did not reach its tolerance";
    default: return "unknown error";
  }
}

const char* qbvm_last_error(void) { return g_last_error.c_str(); }

int qbvm_plan(qbvm_plan_t* out, const qbvm_grid* grid, void* hip_stream) {
  if (!out) return set_error(QBVM_EINVAL, "out is NULL");
  *out = nullptr;
  qbvm_plan_s* p = nullptr;
  const int rc = create_plan(&p, grid, (hipStream_t)hip_stream);
  if (rc) return rc;
  *out = p;
  return QBVM_OK;
}

void qbvm_plan_destroy(qbvm_plan_t p) { destroy_plan(p); }

int qbvm_plan_set_stream(qbvm_plan_t p, void* hip_stream) {
  if (!p) return set_error(QBVM_EINVAL, "plan is NULL");
  p->stream = (hipStream_t)hip_stream;
  return QBVM_OK;
}

long long qbvm_plan_workspace_bytes(qbvm_plan_t p) { return p ? p->bytes : 0; }

int qbvm_solve(qbvm_plan_t p, double alpha, int variant, const double* g_delta, double* y, int output) {
  if (!p || !g_delta || !y) return set_error(QBVM_EINVAL, "NULL argument");
  int rc = check_alpha(alpha, variant);
  if (rc) return rc;
  if (output != QBVM_OUT_ALL && output != QBVM_OUT_Y0 && output != QBVM_OUT_YN)
    return set_error(QBVM_EINVAL, "output must be QBVM_OUT_ALL, QBVM_OUT_Y0 or QBVM_OUT_YN");
  if (p->kop)
    return kop_solve(p, alpha, variant, g_delta, y, output == QBVM_OUT_YN ? p->n : 0,
                     output == QBVM_OUT_ALL ? p->Nt : 1);
  if (output == QBVM_OUT_ALL)
    return enqueue_full(p, alpha, nullptr, variant, g_delta, y, p->s2, nullptr, p->stream, p->W);
  const int level = output == QBVM_OUT_Y0 ? 0 : p->n;
  if (p->has_op || p->no_sine) {  // no sine basis: the tridiagonal path, one level of Step (c)
    const sched::Geom G = geom(p);
    const SolveScalars sc = sched::host_scalars(alpha, variant, p->tau);
    auto ta = sched::thomas_step(G, sc, nullptr, variant, g_delta, p->s2);
    if (p->has_op) {
      ta.args.op_lo = p->op;
      ta.args.op_di = p->op + p->m;
      ta.args.op_up = p->op + 2 * p->m;
    }
    HIP_TRY(launch_thomas(ta.args, ta.nwg, ta.lds, p->stream, nullptr));
    auto t = sched::time1d_step(G, sc, nullptr, variant, p->s2, y);
    t.args.lev_first = level;
    t.args.lev_count = 1;
    t.lds = sched::lds_time1d(G, 1);
    HIP_TRY(launch_time1d(t.args, t.nwg, kThreads, t.lds, p->stream, nullptr));
    return QBVM_OK;
  }
  rc = run_dst(p, g_delta, p->ghat, 1, true);
  if (rc) return rc;
  rc = enqueue_row(p, 1, p->ghat, level, alpha, nullptr, variant, p->yrow, false, nullptr, 0, nullptr, nullptr,
                   nullptr, p->wg_row);
  if (rc) return rc;
  return run_dst(p, p->yrow, y, 1, false);
}

int qbvm_plan_set_operator_1d(qbvm_plan_t p, const double* lower, const double* diag, const double* upper) {
  if (!p) return set_error(QBVM_EINVAL, "plan is NULL");
  if (!diag) {
    p->has_op = false;
    return QBVM_OK;
  }
  if (p->d != 1) return set_error(QBVM_EINVAL, "a spatial operator can be set on 1D plans only");
  const int m = p->m;
  if (m > 1 && (!lower || !upper)) return set_error(QBVM_EINVAL, "lower and upper diagonals are required");
  std::vector<double> h(3 * (size_t)m, 0.0);
  for (int i = 0; i < m; ++i) {
    h[(size_t)m + i] = diag[i];
    if (i + 1 < m) {
      h[i] = lower[i];
      h[2 * (size_t)m + i] = upper[i];
    }
  }
  for (double v : h)
    if (!std::isfinite(v)) return set_error(QBVM_EINVAL, "operator entries must be finite");
  if (!p->op) HIP_TRY(dalloc(p, &p->op, 3 * (size_t)m));
  HIP_TRY(hipStreamSynchronize(p->stream));  // solves in flight may still read the old operator
  HIP_TRY(hipMemcpy(p->op, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice));
  p->has_op = true;
  return QBVM_OK;
}

int qbvm_plan_set_operator_2d(qbvm_plan_t p, const double* kx, const double* ky, double tol, int max_iter) {
  if (!p) return set_error(QBVM_EINVAL, "plan is NULL");
  return set_diffusion(p, 2, kx, ky, nullptr, tol, max_iter);
}

int qbvm_plan_set_operator_3d(qbvm_plan_t p, const double* kx, const double* ky, const double* kz, double tol,
                              int max_iter) {
  if (!p) return set_error(QBVM_EINVAL, "plan is NULL");
  return set_diffusion(p, 3, kx, ky, kz, tol, max_iter);
}

int qbvm_plan_operator_stats(qbvm_plan_t p, int* iterations, double* max_rel_residual, int* breakdowns) {
  if (!p) return set_error(QBVM_EINVAL, "plan is NULL");
  if (iterations) *iterations = p->kry_iters;
  if (max_rel_residual) *max_rel_residual = p->kry_relres;
  if (breakdowns) *breakdowns = p->kry_breakdowns;
  return QBVM_OK;
}

int qbvm_solve_general(qbvm_plan_t p, double alpha, int variant, const double* f, double* y) {
  if (!p || !f || !y) return set_error(QBVM_EINVAL, "NULL argument");
  if (p->has_op || p->kop) return set_error(QBVM_EUNSUPPORTED, "general right-hand side with a spatial operator set");
  if (p->no_sine) return set_error(QBVM_EUNSUPPORTED, "sine transform of length 2(m+1) exceeds the FFT core");
  int rc = check_alpha(alpha, variant);
  if (rc) return rc;
  const sched::Geom G = geom(p);
  auto gs = sched::general_schedule(G, f, y, p->W, p->tabs, p->var_gen);
  if (gs.time.lds > 160 * 1024) return set_error(QBVM_EUNSUPPORTED, "time transform too long for the general solve");
  const TabJob job{p->tabs, p->Nt, variant, p->tau, alpha, nullptr, 1};
  const bool side_job = gs.in.back().args.fft.p2 != 0;  // the tables as side work of the last input pass
  if (side_job) gs.in.back().args.tab = job;
  const double elems = (double)p->Nt * p->nmodes;
  auto passes = [&](const std::vector<sched::Launch<DstArgs>>& v) -> int {
    for (const auto& L : v) {
      const int role = L.args.inner == 1 ? 1 : 2;
      ProfScope ps(role == 1 ? "dst_rows" : "dst_cols", p->stream, 16.0 * elems,
                   0.5 * (double)L.args.outer * L.args.inner * fft_flops(L.args.fft), nullptr);
      HIP_TRY(launch_dst(L.args, L.nwg, L.args.threads, L.lds, p->stream, nullptr, role));
    }
    return QBVM_OK;
  };
  rc = passes(gs.in);
  if (rc) return rc;
  if (!side_job) HIP_TRY(launch_tab_job(job, p->stream));
  {
    ProfScope ps("time_general", p->stream, 16.0 * elems,
                 (double)p->nmodes * (fft_flops(p->tfft->dev) + 40.0 * p->Nt), nullptr);
    HIP_TRY(launch_time_general(gs.time.args, gs.time.nwg, gs.time.lds, p->stream));
  }
  return passes(gs.out);
}

int qbvm_discrepancy(qbvm_plan_t p, double alpha, int variant, const double* g_delta, double* D_out) {
  if (!p || !g_delta || !D_out) return set_error(QBVM_EINVAL, "NULL argument");
  if (p->has_op || p->kop) return set_error(QBVM_EUNSUPPORTED, "discrepancy with a spatial operator set");
  if (p->no_sine) return set_error(QBVM_EUNSUPPORTED, "sine transform of length 2(m+1) exceeds the FFT core");
  int rc = check_alpha(alpha, variant);
  if (rc) return rc;
  rc = run_dst(p, g_delta, p->ghat, 1, true);
  if (rc) return rc;
  const double seq = (p->mbox_seq += 1.0);
  rc = enqueue_row(p, 1, p->ghat, p->n, alpha, nullptr, variant, nullptr, true, nullptr, 0, p->dscal + 3,
                   p->partial, p->counter, p->wg_row, p->mbox_dev, nullptr, seq);
  if (rc) return rc;
  rc = wait_mailbox(p, seq);
  if (rc) return rc;
  *D_out = p->mbox[2];
  return QBVM_OK;
}

static int enqueue_bisection(qbvm_plan_t p, int variant, int count, const double* ghat, const double* deltas,
                             double delta_val, const qbvm_alpha_opts* o, double* bstate, double* alphas_out,
                             int* hits_out, double* partial, unsigned* counter, int wpi) {
  HIP_TRY(launch_bisect_init(bstate, count, deltas, delta_val, o->tau_dp, o->log10_lo, o->log10_hi, p->stream));
  int rc = enqueue_row(p, count, ghat, p->n, 0.0, nullptr, variant, nullptr, true, bstate, 2, nullptr, partial,
                       counter, wpi);
  if (rc) return rc;
  rc = enqueue_row(p, count, ghat, p->n, 0.0, nullptr, variant, nullptr, true, bstate, 3, nullptr, partial,
                   counter, wpi);
  if (rc) return rc;
  for (int it = 0; it < o->steps; ++it) {
    rc = enqueue_row(p, count, ghat, p->n, 0.0, nullptr, variant, nullptr, true, bstate, 1, nullptr, partial,
                     counter, wpi);
    if (rc) return rc;
  }
  HIP_TRY(launch_bisect_finish(bstate, count, alphas_out, hits_out, p->stream));
  return QBVM_OK;
}

static int check_opts(const qbvm_alpha_opts* o) {
  if (!o) return set_error(QBVM_EINVAL, "opts is NULL");
  if (!(o->tau_dp > 0) || !(o->log10_lo < o->log10_hi) || o->steps < 0 || o->steps > 200)
    return set_error(QBVM_EINVAL, "invalid bisection options");
  return QBVM_OK;
}

int qbvm_choose_alpha(qbvm_plan_t p, int variant, const double* g_delta, double delta, const qbvm_alpha_opts* o,
                      double* alpha_out, qbvm_alpha_info* info) {
  if (!p || !g_delta || !alpha_out) return set_error(QBVM_EINVAL, "NULL argument");
  if (p->has_op || p->kop) return set_error(QBVM_EUNSUPPORTED, "alpha choice with a spatial operator set");
  if (p->no_sine) return set_error(QBVM_EUNSUPPORTED, "sine transform of length 2(m+1) exceeds the FFT core");
  int rc = check_opts(o);
  if (rc) return rc;
  if (!(delta > 0) || !std::isfinite(delta)) return set_error(QBVM_EINVAL, "delta must be positive");
  if (variant != QBVM_PQ && variant != QBVM_PM) return set_error(QBVM_EINVAL, "invalid variant");
  if (o->use_learned && !p->has_model) return set_error(QBVM_ENOMODEL, "no model attached");
  qbvm_alpha_info inf{};
  rc = run_dst(p, g_delta, p->ghat, 1, true);
  if (rc) return rc;
  if (o->use_learned) {
    HIP_TRY(launch_feat_predict(p->hd, p->ghat, delta, p->bin_perm, p->bin_off, p->model, p->feats, p->dscal + 1,
                                p->partial, p->counter, p->stream));
    const double seq = (p->mbox_seq += 1.0);
    rc = enqueue_row(p, 1, p->ghat, p->n, 0.0, p->dscal + 1, variant, nullptr, true, nullptr, 0, p->dscal + 3,
                     p->partial, p->counter, p->wg_row, p->mbox_dev, nullptr, seq);
    if (rc) return rc;
    rc = wait_mailbox(p, seq);
    if (rc) return rc;
    const double a_hat = p->mbox[1], D = p->mbox[2];
    inf.alpha_learned = a_hat;
    inf.iterations = 1;
    inf.discrepancy = D;
    const double ratio = D / delta;
    if (std::isfinite(a_hat) && a_hat > 0 && ratio >= o->win_lo && ratio <= o->win_hi) {
      *alpha_out = a_hat;
      if (info) *info = inf;
      return QBVM_OK;
    }
    inf.used_fallback = 1;
  }
  rc = enqueue_bisection(p, variant, 1, p->ghat, nullptr, delta, o, p->bstate, p->dscal + 4, nullptr, p->partial,
                         p->counter, p->wg_row);
  if (rc) return rc;
  const double seq = (p->mbox_seq += 1.0);
  rc = enqueue_row(p, 1, p->ghat, p->n, 0.0, p->dscal + 4, variant, nullptr, true, nullptr, 0, p->dscal + 3,
                   p->partial, p->counter, p->wg_row, p->mbox_dev, p->bstate, seq);
  if (rc) return rc;
  rc = wait_mailbox(p, seq);
  if (rc) return rc;
  *alpha_out = p->mbox[1];
  inf.discrepancy = p->mbox[2];
  inf.iterations += (int)p->mbox[3] + 1;
  inf.bracket_hit = p->mbox[4] != 0.0 ? 1 : 0;
  if (info) *info = inf;
  return inf.bracket_hit ? set_error(QBVM_ENOROOT, "discrepancy root outside the bracket") : QBVM_OK;
}

int qbvm_choose_alpha_each(qbvm_plan_t p, int variant, int count, const double* g_deltas, const double* deltas,
                           const qbvm_alpha_opts* o, double* alphas_out, qbvm_alpha_info* infos_out,
                           double* seconds_out) {
  if (!p || !g_deltas || !deltas || !alphas_out || count < 0) return set_error(QBVM_EINVAL, "invalid argument");
  for (int i = 0; i < count; ++i) {
    qbvm_alpha_info inf{};
    const auto t0 = std::chrono::steady_clock::now();
    const int rc = qbvm_choose_alpha(p, variant, g_deltas + (size_t)i * p->nmodes, deltas[i], o, alphas_out + i,
                                     &inf);
    const auto t1 = std::chrono::steady_clock::now();
    if (rc != QBVM_OK && rc != QBVM_ENOROOT) return rc;
    if (infos_out) infos_out[i] = inf;
    if (seconds_out) seconds_out[i] = std::chrono::duration<double>(t1 - t0).count();
  }
  return QBVM_OK;
}

static int ensure_batch_ws(qbvm_plan_t p, size_t bytes) {
  if (p->bws_bytes >= bytes) return QBVM_OK;
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (p->bws) HIP_TRY(hipFree(p->bws));
  p->bws = nullptr;
  p->bws_bytes = 0;
  HIP_TRY(hipMalloc((void**)&p->bws, bytes));
  p->bws_bytes = bytes;
  return QBVM_OK;
}

int qbvm_bisect_batched(qbvm_plan_t p, int variant, int count, const double* g_deltas, const double* deltas,
                        const qbvm_alpha_opts* o, double* alphas_out, int* hits_out) {
  if (!p || !g_deltas || !deltas || !alphas_out) return set_error(QBVM_EINVAL, "NULL argument");
  if (p->has_op || p->kop) return set_error(QBVM_EUNSUPPORTED, "alpha choice with a spatial operator set");
  if (p->no_sine) return set_error(QBVM_EUNSUPPORTED, "sine transform of length 2(m+1) exceeds the FFT core");
  int rc = check_opts(o);
  if (rc) return rc;
  if (count < 1) return set_error(QBVM_EINVAL, "count must be >= 1");
  if (variant != QBVM_PQ && variant != QBVM_PM) return set_error(QBVM_EINVAL, "invalid variant");
  const int wpi = (int)std::max<long long>(1, std::min<long long>(64, (p->nmodes + 255) / 256));
  const size_t gh = (size_t)count * p->nmodes * sizeof(double);
  const size_t bs = (size_t)count * kBState * sizeof(double);
  const size_t pa = (size_t)count * wpi * sizeof(double);
  const size_t co = (size_t)count * sizeof(unsigned);
  rc = ensure_batch_ws(p, gh + bs + pa + co + 256);
  if (rc) return rc;
  char* base = reinterpret_cast<char*>(p->bws);
  double* ghat = reinterpret_cast<double*>(base);
  double* bstate = reinterpret_cast<double*>(base + gh);
  double* partial = reinterpret_cast<double*>(base + gh + bs);
  unsigned* counter = reinterpret_cast<unsigned*>(base + gh + bs + pa);
  HIP_TRY(hipMemsetAsync(counter, 0, co, p->stream));
  rc = run_dst(p, g_deltas, ghat, count, true);
  if (rc) return rc;
  return enqueue_bisection(p, variant, count, ghat, deltas, 0.0, o, bstate, alphas_out, hits_out, partial, counter,
                           wpi);
}

int qbvm_features(qbvm_plan_t p, int count, const double* g_deltas, const double* deltas, float* feats) {
  if (!p || !g_deltas || !deltas || !feats) return set_error(QBVM_EINVAL, "NULL argument");
  if (count < 1) return set_error(QBVM_EINVAL, "count must be >= 1");
  if (p->no_sine) return set_error(QBVM_EUNSUPPORTED, "sine transform of length 2(m+1) exceeds the FFT core");
  const size_t gh = (size_t)count * p->nmodes * sizeof(double);
  int rc = ensure_batch_ws(p, gh + 256);
  if (rc) return rc;
  double* ghat = p->bws;
  rc = run_dst(p, g_deltas, ghat, count, true);
  if (rc) return rc;
  HIP_TRY(launch_features(count, p->nmodes, p->hd, ghat, deltas, p->bin_perm, p->bin_off, feats, p->stream));
  return QBVM_OK;
}

int qbvm_set_alpha_model(qbvm_plan_t p, const float* model) {
  if (!p || !model) return set_error(QBVM_EINVAL, "NULL argument");
  for (int i = 0; i < QBVM_MODEL_FLOATS; ++i)
    if (!std::isfinite(model[i])) return set_error(QBVM_EINVAL, "model contains a non-finite value");
  for (int i = 0; i < 33; ++i)
    if (!(model[QBVM_MLP_PARAMS + 33 + i] > 0)) return set_error(QBVM_EINVAL, "feature std must be positive");
  HIP_TRY(hipMemcpyAsync(p->model, model, sizeof(float) * QBVM_MODEL_FLOATS, hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->has_model = true;
  return QBVM_OK;
}

// ------------------------------------------------------------- network ABI
static std::mutex g_mlp_mu;
static std::map<int, std::pair<float*, size_t>> g_mlp_scratch;

int qbvm_mlp_forward(const float* params, int B, const float* X, float* out, void* stream) {
  if (!params || !X || !out || B < 1) return set_error(QBVM_EINVAL, "invalid argument");
  HIP_TRY(launch_mlp_forward(params, B, X, out, (hipStream_t)stream));
  return QBVM_OK;
}

int qbvm_mlp_loss_grad(const float* params, int B, const float* X, const float* y, float* grad, float* loss,
                       void* stream) {
  if (!params || !X || !y || !grad || !loss || B < 1) return set_error(QBVM_EINVAL, "invalid argument");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  const size_t need = (size_t)B * (64 * 3 + 1) * sizeof(float);
  float* scratch = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mlp_mu);
    auto& e = g_mlp_scratch[dev];
    if (e.second < need) {
      HIP_TRY(hipDeviceSynchronize());
      if (e.first) HIP_TRY(hipFree(e.first));
      e.first = nullptr;
      e.second = 0;
      HIP_TRY(hipMalloc((void**)&e.first, need));
      e.second = need;
    }
    scratch = e.first;
  }
  HIP_TRY(launch_mlp_loss_grad(params, B, X, y, grad, loss, scratch, 0, (hipStream_t)stream));
  return QBVM_OK;
}

int qbvm_mlp_loss_grad_noalloc(const float* params, int B, const float* X, const float* y, float* grad,
                               float* loss, void* stream) {
  if (!params || !X || !y || !grad || !loss || B < 1) return set_error(QBVM_EINVAL, "invalid argument");
  if (B > QBVM_NOALLOC_MAX_BATCH)
    return set_error(QBVM_EINVAL, "batch exceeds QBVM_NOALLOC_MAX_BATCH (" + std::to_string(QBVM_NOALLOC_MAX_BATCH) +
                                      ") samples of the fixed scratch array");
  HIP_TRY(launch_mlp_loss_grad_static(params, B, X, y, grad, loss, (hipStream_t)stream));
  return QBVM_OK;
}

int qbvm_adam_step(float* params, const float* grad, float* m, float* v, int n, int step, float lr, float beta1,
                   float beta2, float eps, void* stream) {
  if (!params || !grad || !m || !v || n < 1 || step < 1) return set_error(QBVM_EINVAL, "invalid argument");
  HIP_TRY(launch_adam(params, grad, m, v, n, step, lr, beta1, beta2, eps, (hipStream_t)stream));
  return QBVM_OK;
}

}  // extern "C"


// ------------------------------------------------------------- autotuner
namespace {

// median-free minimum of a few timed launches of one schedule step
template <class F>
int time_min_ms(hipStream_t s, F launch, double* out_ms) {
  hipEvent_t a, b;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  double best = 1e30;
  for (int rep = 0; rep < 4; ++rep) {
    HIP_TRY(hipEventRecord(a, s));
    const int rc = launch();
    if (rc) return rc;
    HIP_TRY(hipEventRecord(b, s));
    HIP_TRY(hipEventSynchronize(b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, a, b));
    if (rep > 0) best = std::min(best, (double)ms);  // first launch is a warm-up
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *out_ms = best;
  return QBVM_OK;
}

}  // namespace

// rows variants 0, 1, 3 .. 7; columns the same; time variants 0 .. kTimeVariants2 - 1;
// general right-hand-side time variants 0 .. kTimeVariants2 - 1; separate x_2 + x_1 passes;
// plane-pass variants 0 .. kPlaneVariants - 1
constexpr int kAutotuneTimings = 14 + 2 * p2sz::kTimeVariants2 + 1 + p2sz::kPlaneVariants;
constexpr double kKeepMargin = 1.03;

extern "C" int qbvm_plan_autotune(qbvm_plan_t p, double* ms_out) {
  if (!p) return set_error(QBVM_EINVAL, "plan is NULL");
  double ms[kAutotuneTimings];
  for (double& x : ms) x = -1.0;
  const size_t ny = (size_t)p->Nt * p->nmodes;
  double* scratch = nullptr;
  HIP_TRY(hipMalloc((void**)&scratch, ny * sizeof(double)));
  std::unique_ptr<double, void (*)(double*)> guard(scratch, [](double* q) { (void)hipFree(q); });
  HIP_TRY(hipMemsetAsync(scratch, 0, ny * sizeof(double), p->stream));
  HIP_TRY(hipMemsetAsync(p->ghat, 0, p->nmodes * sizeof(double), p->stream));
  if (p->W) HIP_TRY(hipMemsetAsync(p->W, 0, sched::padded_elems(geom(p)) * sizeof(double), p->stream));
  const int Ns = p->sfft->dev.p2, Nt2 = p->tfft->dev.p2;
  if (Ns && p->d >= 2) {
    for (int role = 0; role < 2; ++role) {
      double best = 1e30;
      int bestv = -1;
      for (int V : {0, 1, 3, 4, 5, 6, 7}) {
        if (!p2sz::dst_valid(Ns, V)) continue;
        sched::Geom G = geom(p);
        G.var_rows = G.var_cols = V;
        const bool pad = p->W != nullptr;
        auto passes = pad ? sched::padded_passes(G, p->W, scratch) : sched::dst_passes(G, scratch, scratch, p->Nt, false);
        // 3D with the plane pass: the only columns pass is the x_3 pass (stride P1 m)
        if (pad && role == 1 && p->d == 3 && sched::use_plane(G)) passes = sched::plane_pre_passes(G, p->W);
        const auto& L = pad ? passes[role == 0 ? passes.size() - 1 : 0] : passes[role == 0 ? 0 : 1];
        double t = 0;
        const int rc = time_min_ms(p->stream, [&]() -> int {
          HIP_TRY(launch_dst(L.args, L.nwg, L.args.threads, L.lds, p->stream, nullptr, role + 1));
          return QBVM_OK;
        }, &t);
        if (rc) return rc;
        ms[role * 7 + (V < 2 ? V : V - 1)] = t;
        if (t < best) {
          best = t;
          bestv = V;
        }
      }
      // keep the current variant unless another is clearly faster (timings of close
      // variants jitter by a few percent from run to run)
      int& cur = role == 0 ? p->var_rows : p->var_cols;
      const double tc = p2sz::dst_valid(Ns, cur) ? ms[role * 7 + (cur < 2 ? cur : cur - 1)] : -1.0;
      if (bestv >= 0 && !(tc > 0 && tc <= kKeepMargin * best)) cur = bestv;
    }
  }
  if (p->W && sched::use_plane(geom(p))) {
    // plane-pass variants against the x_2 columns pass plus the x_1 rows pass they replace
    const sched::Geom G = geom(p);
    const auto passes = sched::padded_passes(G, p->W, scratch);
    double sep = 0.0;
    for (size_t i = passes.size() - 2; i < passes.size(); ++i) {
      const auto& L = passes[i];
      const bool rows = i + 1 == passes.size();
      double t = 0;
      const int rc = time_min_ms(p->stream, [&]() -> int {
        HIP_TRY(launch_dst(L.args, L.nwg, L.args.threads, L.lds, p->stream, nullptr, rows ? 1 : 2));
        return QBVM_OK;
      }, &t);
      if (rc) return rc;
      sep += t;
    }
    ms[kAutotuneTimings - p2sz::kPlaneVariants - 1] = sep;
    double best = 1e30;
    int bestv = -1;
    const PlaneArgs pa = sched::plane_args(G, p->W, scratch);
    for (int V = 0; V < p2sz::kPlaneVariants; ++V) {
      double t = 0;
      const int rc = time_min_ms(p->stream, [&]() -> int {
        HIP_TRY(launch_plane(pa, V, p->stream, nullptr));
        return QBVM_OK;
      }, &t);
      if (rc) return rc;
      ms[kAutotuneTimings - p2sz::kPlaneVariants + V] = t;
      if (t < best) {
        best = t;
        bestv = V;
      }
    }
    const double tcur = p->plane ? ms[kAutotuneTimings - p2sz::kPlaneVariants + p->var_plane] : sep;
    if (!(tcur <= kKeepMargin * std::min(best, sep))) {
      p->plane = best < sep;
      if (p->plane) p->var_plane = bestv;
    }
  }
  const bool gt = p->tfft->dev.gtA != 0;
  if ((Nt2 && p2sz::time_valid(Nt2, 0)) || gt) {
    double best = 1e30;
    int bestv = -1;
    for (int V = 0; V < (gt ? p2sz::kGtVariants : p2sz::kTimeVariants2); ++V) {
      if (!gt && !p2sz::time_valid(Nt2, V)) continue;
      sched::Geom G = geom(p);
      G.var_time = V;
      const SolveScalars sc = sched::host_scalars(1e-3, QBVM_PQ, p->tau);
      const auto t = p->W ? sched::time_step_padded(G, sc, nullptr, QBVM_PQ, p->ghat, p->W)
                          : sched::time_step(G, sc, nullptr, QBVM_PQ, scratch, scratch, 0, p->Nt);
      double tm = 0;
      const int rc = time_min_ms(p->stream, [&]() -> int {
        HIP_TRY(launch_time(t.args, t.nwg, t.args.threads, t.lds, p->stream, nullptr));
        return QBVM_OK;
      }, &tm);
      if (rc) return rc;
      ms[14 + V] = tm;
      if (tm < best) {
        best = tm;
        bestv = V;
      }
    }
    const double tcur = (p->var_time >= 0 && p->var_time < p2sz::kTimeVariants2) ? ms[14 + p->var_time] : -1.0;
    if (bestv >= 0 && !(tcur > 0 && tcur <= kKeepMargin * best)) p->var_time = bestv;
  }
  const sched::Geom G0 = geom(p);
  if (p->W && sched::use_padded_general(G0)) {
    // general right-hand-side time kernel in place on W, tables of one solve
    HIP_TRY(launch_tab_job(TabJob{p->tabs, p->Nt, QBVM_PQ, p->tau, 1e-3, nullptr, 1}, p->stream));
    constexpr int o = 14 + p2sz::kTimeVariants2;
    double best = 1e30;
    int bestv = -1;
    for (int V = 0; V < p2sz::kTimeVariants2; ++V) {
      if (!p2sz::time_general_valid(Nt2, V)) continue;
      const auto gs = sched::general_schedule(G0, scratch, scratch, p->W, p->tabs, V);
      double tm = 0;
      const int rc = time_min_ms(p->stream, [&]() -> int {
        HIP_TRY(launch_time_general(gs.time.args, gs.time.nwg, gs.time.lds, p->stream));
        return QBVM_OK;
      }, &tm);
      if (rc) return rc;
      ms[o + V] = tm;
      if (tm < best) {
        best = tm;
        bestv = V;
      }
    }
    const double tcur = p2sz::time_general_valid(Nt2, p->var_gen) ? ms[o + p->var_gen] : -1.0;
    if (bestv >= 0 && !(tcur > 0 && tcur <= kKeepMargin * best)) p->var_gen = bestv;
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (Ns && p->d >= 2) {
      g_tuned[std::make_tuple(p->device, 0, Ns)] = p->var_rows;
      g_tuned[std::make_tuple(p->device, 1, Ns)] = p->var_cols;
    }
    if (Nt2 && p->d >= 2) g_tuned[std::make_tuple(p->device, 2, Nt2)] = p->var_time;
    if (gt && p->d >= 2) g_tuned[std::make_tuple(p->device, 3, p->Nt)] = p->var_time;
    if (p->W && sched::use_padded_general(G0)) g_tuned[std::make_tuple(p->device, 4, Nt2)] = p->var_gen;
  }
  if (ms_out)
    for (int i = 0; i < kAutotuneTimings; ++i) ms_out[i] = ms[i];
  return QBVM_OK;
}

extern "C" int qbvm_plan_set_plane(qbvm_plan_t p, int variant) {
  if (!p) return set_error(QBVM_EINVAL, "plan is NULL");
  if (variant < 0) {
    p->plane = false;
    return QBVM_OK;
  }
  if (variant >= p2sz::kPlaneVariants) return set_error(QBVM_EINVAL, "no such plane-pass variant");
  if (!sched::use_plane(geom(p)))
    return set_error(QBVM_EUNSUPPORTED, "the plane pass needs d >= 2, m = 127 and the padded pipeline");
  p->plane = true;
  p->var_plane = variant;
  return QBVM_OK;
}

extern "C" int qbvm_plan_get_plane(qbvm_plan_t p, int* variant) {
  if (!p || !variant) return set_error(QBVM_EINVAL, "NULL argument");
  *variant = p->plane && sched::use_plane(geom(p)) ? p->var_plane : -1;
  return QBVM_OK;
}

extern "C" int qbvm_plan_get_variants(qbvm_plan_t p, int* var_rows, int* var_cols, int* var_time,
                                      int* var_general) {
  if (!p) return set_error(QBVM_EINVAL, "plan is NULL");
  if (var_rows) *var_rows = p->var_rows;
  if (var_cols) *var_cols = p->var_cols;
  if (var_time) *var_time = p->var_time;
  if (var_general) *var_general = p->var_gen;
  return QBVM_OK;
}

extern "C" int qbvm_plan_set_variants(qbvm_plan_t p, int var_rows, int var_cols, int var_time, int var_general) {
  if (!p) return set_error(QBVM_EINVAL, "plan is NULL");
  const int Ns = p->sfft->dev.p2, Nt2 = p->tfft->dev.p2;
  const bool gt = p->tfft->dev.gtA != 0;
  auto dst_ok = [&](int V) { return V == -1 || (Ns && p->d >= 2 && p2sz::dst_valid(Ns, V)); };
  const bool time_ok = var_time == -1 || (p->d >= 2 && ((Nt2 && p2sz::time_valid(Nt2, var_time)) ||
                                                        (gt && var_time >= 0 && var_time < p2sz::kGtVariants)));
  const bool gen_ok = var_general == -1 ||
                      (p->W && sched::use_padded_general(geom(p)) && p2sz::time_general_valid(Nt2, var_general));
  if (!dst_ok(var_rows) || !dst_ok(var_cols) || !time_ok || !gen_ok)
    return set_error(QBVM_EINVAL, "kernel variant not available for this plan's transform lengths");
  if (var_rows != -1) p->var_rows = var_rows;
  if (var_cols != -1) p->var_cols = var_cols;
  if (var_time != -1) p->var_time = var_time;
  if (var_general != -1) p->var_gen = var_general;
  return QBVM_OK;
}

// ================================================================ batched
namespace {

struct BatchEntry {
  int device = 0;
  std::vector<qbvm_grid> grids;
  std::vector<int> variants, outputs;
  std::vector<const double*> gs;  // buffers the graph's arguments refer to now
  std::vector<double*> ys;
  std::vector<qbvm_plan_s*> plans;  // owned by g_batch_plans
  double* alphas_dev = nullptr;
  std::vector<void*> ws;             // per-instance workspaces
  std::vector<c64*> s2;              // 1D, every level: shifted solutions [N_t][m]
  std::vector<double*> ghat, yrow;   // one level: sine coefficients and the level's modes
  // 1D instances with every level: two persistent launches over argument tables
  std::vector<int> b1d;              // their instance indices
  std::vector<ThomasArgs> targs;     // host copies of the tables (rewritten for new buffers)
  std::vector<Time1dArgs> t1args;
  ThomasArgs* targs_dev = nullptr;
  Time1dArgs* t1args_dev = nullptr;
  int* items_dev = nullptr;          // tridiagonal items, then narrow and wide time items
  int n_tri = 0, n_t1[2] = {0, 0};
  size_t lds_tri = 0, lds_t1[2] = {0, 0};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipGraphNode_t> nodes;  // kernel nodes of the per-instance chains, in launch order
  unsigned long long last_use = 0;
};

constexpr size_t kBatchCacheEntries = 8;
std::mutex g_batch_mu;
std::vector<std::unique_ptr<BatchEntry>> g_batches;
std::map<std::tuple<int, int, int, int, double, double>, qbvm_plan_s*> g_batch_plans;
unsigned long long g_batch_clock = 0;

bool same_grid(const qbvm_grid& a, const qbvm_grid& b) {
  return a.d == b.d && a.m == b.m && a.n == b.n && a.L == b.L && a.T == b.T;
}

void free_entry(BatchEntry* e) {
  if (e->exec) (void)hipGraphExecDestroy(e->exec);
  if (e->graph) (void)hipGraphDestroy(e->graph);
  for (void* w : e->ws) (void)hipFree(w);
  if (e->alphas_dev) (void)hipFree(e->alphas_dev);
  if (e->targs_dev) (void)hipFree(e->targs_dev);
  if (e->t1args_dev) (void)hipFree(e->t1args_dev);
  if (e->items_dev) (void)hipFree(e->items_dev);
}

// 1D instance with every level: it runs in the batched tridiagonal and time launches
bool in_batch_1d(const BatchEntry* e, int i) { return e->plans[i]->d == 1 && e->outputs[i] == QBVM_OUT_ALL; }

// Argument blocks of the batched 1D launches for the entry's current buffers.
void fill_batch_1d_args(BatchEntry* e) {
  for (size_t k = 0; k < e->b1d.size(); ++k) {
    const int i = e->b1d[k];
    const qbvm_plan_s* p = e->plans[i];
    const sched::Geom G = geom(p);
    const SolveScalars sc = sched::host_scalars(1.0, e->variants[i], p->tau);  // alpha from the table
    e->targs[k] = sched::thomas_step(G, sc, e->alphas_dev + i, e->variants[i], e->gs[i], e->s2[i]).args;
    e->t1args[k] = sched::time1d_step(G, sc, e->alphas_dev + i, e->variants[i], e->s2[i], e->ys[i]).args;
  }
}

// The per-instance chains in a fixed order (nc records or updates their nodes): all
// levels of a d >= 2 instance, or one level (d >= 1) by the sine transform of g, one DFT
// row per mode and the sine transform back.
int enqueue_instances(BatchEntry* e, NodeCtx& base, hipStream_t stream) {
  const int count = (int)e->grids.size();
  for (int i = 0; i < count; ++i) {
    if (in_batch_1d(e, i)) continue;
    qbvm_plan_s* p = e->plans[i];
    NodeCtx nc = base;
    nc.dep = nullptr;
    nc.has_dep = false;
    int rc;
    if (e->outputs[i] == QBVM_OUT_ALL) {
      rc = enqueue_full(p, 1.0, e->alphas_dev + i, e->variants[i], e->gs[i], e->ys[i], nullptr, &nc, stream);
    } else {
      rc = run_dst(p, e->gs[i], e->ghat[i], 1, true, &nc, stream);
      if (!rc) {
        RowArgs r{};
        r.Nt = p->Nt;
        r.d = p->d;
        r.m = p->m;
        r.level = e->outputs[i] == QBVM_OUT_Y0 ? 0 : p->n;
        r.count = 1;
        r.nmodes = p->nmodes;
        r.tau = p->tau;
        r.hd = p->hd;
        r.variant = e->variants[i];
        r.mu1d = p->mu1d;
        r.ghat = e->ghat[i];
        r.yrow = e->yrow[i];
        r.wg_per_inst = p->wg_row;
        r.alpha = 1.0;
        r.alpha_dev = e->alphas_dev + i;
        HIP_TRY(launch_row(r, p->wg_row, kThreads, sizeof(c64) * 2 * p->Nt, stream, &nc));
        rc = run_dst(p, e->yrow[i], e->ys[i], 1, false, &nc, stream);
      }
    }
    if (rc) return rc;
    base.next = nc.next;
  }
  return QBVM_OK;
}

int build_entry(BatchEntry* e, int count, hipStream_t stream) {
  e->plans.resize(count);
  for (int i = 0; i < count; ++i) {
    const qbvm_grid& g = e->grids[i];
    auto key = std::make_tuple(e->device, g.d, g.m, g.n, g.L, g.T);
    auto it = g_batch_plans.find(key);
    if (it == g_batch_plans.end()) {
      qbvm_plan_s* p = nullptr;
      const int rc = create_plan(&p, &g, stream);
      if (rc) return rc;
      it = g_batch_plans.emplace(key, p).first;
    }
    e->plans[i] = it->second;
    if (e->outputs[i] != QBVM_OUT_ALL && e->plans[i]->no_sine)
      return set_error(QBVM_EUNSUPPORTED, "single-level output of a 1D grid without its sine transform");
  }
  HIP_TRY(hipMalloc((void**)&e->alphas_dev, sizeof(double) * count));
  e->s2.assign(count, nullptr);
  e->ghat.assign(count, nullptr);
  e->yrow.assign(count, nullptr);
  for (int i = 0; i < count; ++i) {
    const qbvm_plan_s* p = e->plans[i];
    void* w = nullptr;
    if (in_batch_1d(e, i)) {
      HIP_TRY(hipMalloc(&w, sizeof(c64) * (size_t)p->Nt * p->m));
      e->ws.push_back(w);
      e->s2[i] = static_cast<c64*>(w);
      e->b1d.push_back(i);
    } else if (e->outputs[i] != QBVM_OUT_ALL) {
      HIP_TRY(hipMalloc(&w, sizeof(double) * 2 * (size_t)p->nmodes));
      e->ws.push_back(w);
      e->ghat[i] = static_cast<double*>(w);
      e->yrow[i] = e->ghat[i] + p->nmodes;
    }
  }
  HIP_TRY(hipGraphCreate(&e->graph, 0));
  NodeCtx nc{e->graph, nullptr, false};
  nc.nodes = &e->nodes;
  int rc = enqueue_instances(e, nc, stream);
  if (rc) return rc;
  if (!e->b1d.empty()) {
    const size_t nb = e->b1d.size();
    e->targs.resize(nb);
    e->t1args.resize(nb);
    fill_batch_1d_args(e);
    std::vector<int> items;  // (instance, workgroup) pairs: tridiagonal, narrow time, wide time
    for (size_t k = 0; k < nb; ++k) {
      const qbvm_plan_s* p = e->plans[e->b1d[k]];
      const auto ta = sched::thomas_step(geom(p), SolveScalars{}, nullptr, 0, nullptr, nullptr);
      for (long long w = 0; w < ta.nwg; ++w) items.insert(items.end(), {(int)k, (int)w});
      e->lds_tri = std::max(e->lds_tri, ta.lds);
    }
    e->n_tri = (int)(items.size() / 2);
    for (int wide = 0; wide < 2; ++wide) {
      const size_t before = items.size();
      for (size_t k = 0; k < nb; ++k) {
        const qbvm_plan_s* p = e->plans[e->b1d[k]];
        if ((p->tfft->dev.wide != 0) != (wide != 0)) continue;
        const auto t = sched::time1d_step(geom(p), SolveScalars{}, nullptr, 0, nullptr, nullptr);
        for (long long w = 0; w < t.nwg; ++w) items.insert(items.end(), {(int)k, (int)w});
        e->lds_t1[wide] = std::max(e->lds_t1[wide], t.lds);
      }
      e->n_t1[wide] = (int)((items.size() - before) / 2);
    }
    HIP_TRY(hipMalloc((void**)&e->targs_dev, sizeof(ThomasArgs) * nb));
    HIP_TRY(hipMalloc((void**)&e->t1args_dev, sizeof(Time1dArgs) * nb));
    HIP_TRY(hipMalloc((void**)&e->items_dev, sizeof(int) * items.size()));
    HIP_TRY(hipMemcpy(e->items_dev, items.data(), sizeof(int) * items.size(), hipMemcpyHostToDevice));
    NodeCtx n1{e->graph, nullptr, false};
    HIP_TRY(launch_tri1d_batch(Batch1dArgs{e->targs_dev, e->items_dev, e->n_tri}, e->lds_tri, stream, &n1));
    const hipGraphNode_t tri = n1.dep;
    const int* it = e->items_dev + 2 * e->n_tri;
    for (int wide = 0; wide < 2; ++wide) {
      if (e->n_t1[wide] == 0) continue;
      NodeCtx n2{e->graph, tri, true};
      HIP_TRY(launch_time1d_batch(Batch1dArgs{e->t1args_dev, it, e->n_t1[wide]}, wide != 0, e->lds_t1[wide], stream,
                                  &n2));
      it += 2 * e->n_t1[wide];
    }
  }
  HIP_TRY(hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0));
  return QBVM_OK;
}

}  // namespace

extern "C" int qbvm_solve_batched(int count, const qbvm_grid* grids, const double* alphas, const int* variants,
                                  const double* const* g_deltas, double* const* ys, const int* outputs,
                                  void* hip_stream) {
  if (count < 1 || !grids || !alphas || !variants || !g_deltas || !ys || !outputs)
    return set_error(QBVM_EINVAL, "NULL argument or count < 1");
  for (int i = 0; i < count; ++i) {
    int rc = validate_grid(&grids[i]);
    if (rc) return rc;
    rc = check_alpha(alphas[i], variants[i]);
    if (rc) return rc;
    if (!g_deltas[i] || !ys[i]) return set_error(QBVM_EINVAL, "NULL instance pointer");
    if (outputs[i] != QBVM_OUT_ALL && outputs[i] != QBVM_OUT_Y0 && outputs[i] != QBVM_OUT_YN)
      return set_error(QBVM_EINVAL, "output must be QBVM_OUT_ALL, QBVM_OUT_Y0 or QBVM_OUT_YN");
  }
  hipStream_t stream = (hipStream_t)hip_stream;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_batch_mu);
  BatchEntry* hit = nullptr;
  for (auto& e : g_batches) {
    if (e->device != dev || (int)e->grids.size() != count) continue;
    bool ok = true;
    for (int i = 0; i < count && ok; ++i)
      ok = same_grid(e->grids[i], grids[i]) && e->variants[i] == variants[i] && e->outputs[i] == outputs[i];
    if (ok) {
      hit = e.get();
      break;
    }
  }
  if (!hit) {
    if (g_batches.size() >= kBatchCacheEntries) {  // drop the least recently used entry
      auto lru = std::min_element(g_batches.begin(), g_batches.end(),
                                  [](const auto& x, const auto& y) { return x->last_use < y->last_use; });
      HIP_TRY(hipDeviceSynchronize());  // its graph may still run
      free_entry(lru->get());
      g_batches.erase(lru);
    }
    auto e = std::make_unique<BatchEntry>();
    e->device = dev;
    e->grids.assign(grids, grids + count);
    e->variants.assign(variants, variants + count);
    e->outputs.assign(outputs, outputs + count);
    e->gs.assign(g_deltas, g_deltas + count);
    e->ys.assign(ys, ys + count);
    const int rc = build_entry(e.get(), count, stream);
    if (rc) {
      free_entry(e.get());
      return rc;
    }
    g_batches.push_back(std::move(e));
    hit = g_batches.back().get();
  } else {
    bool moved = false;
    for (int i = 0; i < count && !moved; ++i) moved = hit->gs[i] != g_deltas[i] || hit->ys[i] != ys[i];
    if (moved) {  // same launch sequence on new buffers: rewrite the recorded arguments
      hit->gs.assign(g_deltas, g_deltas + count);
      hit->ys.assign(ys, ys + count);
      NodeCtx nc{hit->graph, nullptr, false};
      nc.nodes = &hit->nodes;
      nc.exec = hit->exec;
      const int rc = enqueue_instances(hit, nc, stream);
      if (rc) return rc;
      if (nc.next != hit->nodes.size()) return set_error(QBVM_EHIP, "batched graph update out of step");
      if (!hit->b1d.empty()) fill_batch_1d_args(hit);
    }
  }
  hit->last_use = ++g_batch_clock;
  // pageable sources: the runtime stages them before returning, so no host-side wait is needed
  HIP_TRY(hipMemcpyAsync(hit->alphas_dev, alphas, sizeof(double) * count, hipMemcpyHostToDevice, stream));
  if (!hit->b1d.empty()) {
    HIP_TRY(hipMemcpyAsync(hit->targs_dev, hit->targs.data(), sizeof(ThomasArgs) * hit->targs.size(),
                           hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(hit->t1args_dev, hit->t1args.data(), sizeof(Time1dArgs) * hit->t1args.size(),
                           hipMemcpyHostToDevice, stream));
  }
  HIP_TRY(hipGraphLaunch(hit->exec, stream));
  return QBVM_OK;
}

extern "C" void qbvm_batched_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  (void)hipDeviceSynchronize();
  for (auto& e : g_batches) free_entry(e.get());
  g_batches.clear();
  for (auto& kv : g_batch_plans) destroy_plan(kv.second);
  g_batch_plans.clear();
}
