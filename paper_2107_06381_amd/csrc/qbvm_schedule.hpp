// Launch schedule of one solve: argument blocks and grid sizes of every kernel,
// independent of the HIP runtime so the CPU build of the kernels can replay it.
#pragma once

#include <cmath>
#include <vector>

#include "qbvm_types.hpp"
#include "qbvm_p2_sizes.hpp"

namespace qbvm {
namespace sched {

constexpr int kThreads = 256;

// What a plan fixes about its grid and FFT tables.
struct Geom {
  int d, m, n, Nt;
  double h, tau;
  long long nmodes;
  int S_time, S_dst;
  FftPlanDev tfft;  // length N_t
  FftPlanDev sfft;  // length 2(m+1)
  const double* mu1d;
  int var_rows = 1, var_cols = 1, var_time = 1;  // power-of-two kernel variants (levels)
};

// Padded pipeline (d >= 2, power-of-two sine and time kernels): the time kernel writes
// levels into a workspace whose x_1 rows have pitch P1 (a multiple of 64 doubles, so
// every column tile is aligned), the strided sine passes run in place there, and the
// contiguous x_1 pass goes last and writes the unpadded output.
inline long long padded_pitch(int m) { return ((long long)m + 63) / 64 * 64; }
inline bool use_padded(const Geom& g) {
  return g.d >= 2 && g.sfft.p2 && ((g.tfft.p2 && p2sz::time_valid(g.tfft.p2, 0)) || g.tfft.gtA);
}
inline long long padded_elems(const Geom& g) { return (long long)g.Nt * (g.nmodes / g.m) * padded_pitch(g.m); }

template <class A>
struct Launch {
  A args;
  long long nwg;
  size_t lds;
};

inline size_t lds_dst(const Geom& g) { return sizeof(c64) * ((size_t)g.S_dst * g.sfft.nc + 2 * g.S_dst); }
// Runtime-engine kernels copy the twiddle table (nc entries) into LDS when that keeps the
// workgroup within 80 KB, i.e. two workgroups per CU.
constexpr size_t kTwLdsBudget = 80 * 1024;
inline bool tw_fits_lds(size_t lds, int nc) { return lds + sizeof(c64) * (size_t)nc <= kTwLdsBudget; }
inline size_t lds_time(const Geom& g, int lev_count) {
  const int S = g.S_time;
  return sizeof(c64) * ((size_t)S * g.tfft.nc + 2 * S + g.Nt + lev_count) + sizeof(double) * 4 * S;
}
inline size_t lds_time1d(const Geom& g, int lev_count) {
  const int S = g.S_time;
  return sizeof(c64) * ((size_t)S * g.tfft.nc + 2 * S + lev_count);
}

// d passes of the orthonormal DST-I over a [batch][m]^d array (in -> out, then in place)
// input_transform: g_delta (small batch) -> the one-signal variant; else the tuned ones
inline std::vector<Launch<DstArgs>> dst_passes(const Geom& g, const double* in, double* out, long long batch,
                                               bool input_transform = false) {
  std::vector<Launch<DstArgs>> v;
  const int m = g.m;
  long long inner = 1;
  const long long rest = g.nmodes / m;  // m^{d-1}
  const double scale = 0.5 * std::sqrt(2.0 / (m + 1));
  for (int ax = 0; ax < g.d; ++ax) {
    DstArgs a{};
    a.in = ax == 0 ? in : out;
    a.out = out;
    a.len = m;
    a.inner = inner;
    a.outer = batch * (rest / inner);
    a.S = g.S_dst;
    a.scale = scale;
    a.fft = g.sfft;
    a.threads = kThreads;
    a.in_pitch = a.out_pitch = m;
    a.kstride = inner;
    a.ostride = (long long)m * inner;
    a.colmod = 0;
    a.colvalid = 0;
    size_t lds = lds_dst(g);
    if (g.sfft.p2) {  // compile-time power-of-two kernels
      const int N = g.sfft.p2;
      int V = input_transform ? 2 : (inner > 1 ? g.var_cols : g.var_rows);
      if (!p2sz::dst_valid(N, V)) V = 0;
      a.var = V;
      a.S = p2sz::dst_S(N, V);
      a.threads = p2sz::dst_T(N, V);
      lds = p2sz::dst_lds(N, V, inner > 1);
    } else if (g.sfft.bp2) {  // Bluestein on the compile-time engine
      a.S = p2sz::blue_S(g.sfft.bp2);
      a.threads = p2sz::blue_T(g.sfft.bp2);
      lds = p2sz::blue_lds(g.sfft.bp2);
    }
    long long nwg;
    if (inner == 1) {
      nwg = (a.outer + 2 * a.S - 1) / (2 * a.S);
      a.tiles_per_outer = 1;
    } else {
      a.tiles_per_outer = (inner + 2 * a.S - 1) / (2 * a.S);
      nwg = a.outer * a.tiles_per_outer;
    }
    if (!g.sfft.p2 && !g.sfft.bp2 && tw_fits_lds(lds, g.sfft.nc)) {
      a.tw_lds = 1;
      lds += sizeof(c64) * (size_t)g.sfft.nc;
    }
    v.push_back({a, nwg, lds});
    inner *= m;
  }
  return v;
}

// geometry of one sine pass from its strides (shared by the padded passes)
inline Launch<DstArgs> dst_pass_custom(const Geom& g, const double* in, double* out, long long outer,
                                       long long inner, long long in_pitch, long long out_pitch, long long kstride,
                                       long long ostride, int colmod, int colvalid, int V) {
  DstArgs a{};
  a.in = in;
  a.out = out;
  a.len = g.m;
  a.outer = outer;
  a.inner = inner;
  a.scale = 0.5 * std::sqrt(2.0 / (g.m + 1));
  a.fft = g.sfft;
  a.in_pitch = in_pitch;
  a.out_pitch = out_pitch;
  a.kstride = kstride;
  a.ostride = ostride;
  a.colmod = colmod;
  a.colvalid = colvalid;
  const int N = g.sfft.p2;
  if (!p2sz::dst_valid(N, V)) V = 0;
  a.var = V;
  a.S = p2sz::dst_S(N, V);
  a.threads = p2sz::dst_T(N, V);
  long long nwg;
  if (inner == 1) {
    nwg = (outer + 2 * a.S - 1) / (2 * a.S);
    a.tiles_per_outer = 1;
  } else {
    a.tiles_per_outer = (inner + 2 * a.S - 1) / (2 * a.S);
    nwg = outer * a.tiles_per_outer;
  }
  return {a, nwg, p2sz::dst_lds(N, V, inner > 1)};
}

// Padded-pipeline sine passes over all levels: strided axes in place on W, then
// the x_1 pass W -> y.
inline void strided_passes(const Geom& g, double* W, std::vector<Launch<DstArgs>>& v) {
  const int m = g.m;
  const long long P1 = padded_pitch(m);
  long long kstride = P1;  // axis 1 (x_2)
  long long blocks = (long long)g.Nt * (g.nmodes / m / m);  // outer blocks for axis 1
  for (int ax = 1; ax < g.d; ++ax) {
    // columns of one block: all (x_ax-1 .. x_1) positions below this axis, padded rows
    v.push_back(dst_pass_custom(g, W, W, blocks, kstride, 0, 0, kstride, kstride * m, (int)P1, m, g.var_cols));
    kstride *= m;
    blocks /= m;
  }
}
inline std::vector<Launch<DstArgs>> padded_passes(const Geom& g, double* W, double* y) {
  std::vector<Launch<DstArgs>> v;
  strided_passes(g, W, v);
  const int m = g.m;
  v.push_back(dst_pass_custom(g, W, y, (long long)g.Nt * (g.nmodes / m), 1, padded_pitch(m), m, 0, 0, 0, 0,
                              g.var_rows));
  return v;
}

// Plane pass (d >= 2, sine length 256, i.e. m = 127): after the time kernel, the x_3
// sine pass runs in place on W (3D), then one kernel applies the x_2 and x_1 transforms
// to every [m][P1] plane of W and writes y: 16 bytes per unknown fewer than a columns
// pass and a rows pass.
inline bool use_plane(const Geom& g) {
  return use_padded(g) && g.sfft.p2 == 256 && p2sz::plane_valid(256, 0) && g.m == 127 &&
         padded_pitch(g.m) == p2sz::plane_pitch(256);
}
inline std::vector<Launch<DstArgs>> plane_pre_passes(const Geom& g, double* W) {
  std::vector<Launch<DstArgs>> v;
  if (g.d == 3) {
    const int m = g.m;
    const long long P1 = padded_pitch(m), ks = P1 * m;
    v.push_back(dst_pass_custom(g, W, W, g.Nt, ks, 0, 0, ks, ks * m, (int)P1, m, g.var_cols));
  }
  return v;
}
inline PlaneArgs plane_args(const Geom& g, const double* W, double* y) {
  PlaneArgs a{};
  a.in = W;
  a.out = y;
  a.m = g.m;
  a.in_pitch = (int)padded_pitch(g.m);
  a.planes = (long long)g.Nt * (g.nmodes / ((long long)g.m * g.m));
  a.in_plane = (long long)g.m * a.in_pitch;
  a.out_plane = (long long)g.m * g.m;
  a.scale = 0.5 * std::sqrt(2.0 / (g.m + 1));
  a.fft = g.sfft;
  return a;
}

// Spectral time kernel writing levels [lev_first, lev_first + lev_count) to y.
inline Launch<TimeArgs> time_step(const Geom& g, SolveScalars sc, const double* alpha_dev, int variant,
                                  const double* ghat, double* y, int lev_first, int lev_count) {
  TimeArgs t{};
  t.Nt = g.Nt;
  t.d = g.d;
  t.m = g.m;
  t.S = g.S_time;
  t.nmodes = g.nmodes;
  t.ystride = g.nmodes;
  t.lev_first = lev_first;
  t.lev_count = lev_count;
  t.lev_dst0 = 0;
  t.tau = g.tau;
  t.sc = sc;
  t.mu1d = g.mu1d;
  t.ghat = ghat;
  t.y = y;
  t.alpha_dev = alpha_dev;
  t.variant = variant;
  t.fft = g.tfft;
  t.threads = kThreads;
  t.pitch = 0;
  t.tiles_per_row = 0;
  size_t lds = lds_time(g, lev_count);
  if (g.tfft.gtA && lev_first == 0 && lev_count == g.Nt) {
    const int V = (g.var_time >= 0 && g.var_time < p2sz::kGtVariants) ? g.var_time : 0;
    t.var = V;
    t.S = p2sz::gt_S(V);
    t.threads = p2sz::gt_T(g.tfft.gtA, V);
    t.fft.p2 = 0;
    lds = p2sz::gt_lds(g.tfft.gtA, g.tfft.gtB, V);
  } else if (g.tfft.p2 && p2sz::time_valid(g.tfft.p2, 0) && lev_first == 0 && lev_count == g.Nt) {
    const int N = g.tfft.p2;
    const int V = p2sz::time_valid(N, g.var_time) ? g.var_time : 0;
    t.var = V;
    t.S = p2sz::time_S(N, V);
    t.threads = p2sz::time_T(V);
    lds = p2sz::time_lds(N, V, g.Nt);
  } else {
    t.fft.p2 = 0;  // generic kernel
    t.fft.gtA = t.fft.gtB = 0;
    if (tw_fits_lds(lds, g.tfft.nc)) {
      t.tw_lds = 1;
      lds += sizeof(c64) * (size_t)g.tfft.nc;
    }
  }
  const long long nwg = (g.nmodes + 2LL * t.S - 1) / (2LL * t.S);
  return {t, nwg, lds};
}

// Time kernel of the padded pipeline: every level into W with x_1 pitch P1.
inline Launch<TimeArgs> time_step_padded(const Geom& g, SolveScalars sc, const double* alpha_dev, int variant,
                                         const double* ghat, double* W) {
  Launch<TimeArgs> L = time_step(g, sc, alpha_dev, variant, ghat, W, 0, g.Nt);
  const long long P1 = padded_pitch(g.m);
  const long long rows = g.nmodes / g.m;
  L.args.pitch = P1;
  L.args.ystride = rows * P1;
  L.args.tiles_per_row = (int)((g.m + 2LL * L.args.S - 1) / (2LL * L.args.S));
  L.nwg = rows * L.args.tiles_per_row;
  return L;
}

// Time kernel of the general right-hand side: fgen (sine basis, every level) -> y, in
// place allowed; tables [d_j/tau | gamma_l^{-1}/N_t | gamma_t] in tabs.
inline Launch<TimeArgs> time_general_step(const Geom& g, const double* fgen, double* y, const c64* tabs) {
  TimeArgs t{};
  t.Nt = g.Nt;
  t.d = g.d;
  t.m = g.m;
  t.S = g.S_time;
  t.nmodes = g.nmodes;
  t.ystride = g.nmodes;
  t.lev_first = 0;
  t.lev_count = g.Nt;
  t.tau = g.tau;
  t.mu1d = g.mu1d;
  t.y = y;
  t.fgen = fgen;
  t.tabs = tabs;
  t.fft = g.tfft;
  t.fft.p2 = 0;
  t.fft.gtA = t.fft.gtB = 0;
  t.threads = 256;
  const size_t lds = sizeof(c64) * ((size_t)t.S * g.tfft.nc + (size_t)t.S * g.Nt + 2 * (size_t)t.S) +
                     sizeof(double) * 2 * (size_t)t.S;
  return {t, (g.nmodes + 2LL * t.S - 1) / (2LL * t.S), lds};
}

// General right-hand side, every level: sine transform of f, time kernel, sine
// transform back.  Padded (d >= 2, power-of-two sine and time lengths, W given): the
// x_1 pass f -> W (padded rows), the strided passes and the time kernel in W, then the
// padded output passes W -> y.  Otherwise the passes run in y and the generic time
// kernel between them.  tabs: [d_j/tau | gamma_l^{-1}/N_t | gamma_t], filled by a job
// attached to the last input pass (padded) or by a launch of its own.
inline bool use_padded_general(const Geom& g) {
  return g.d >= 2 && g.sfft.p2 && g.tfft.p2 && p2sz::time_general_valid(g.tfft.p2, 0);
}
struct GeneralSchedule {
  bool padded = false;
  std::vector<Launch<DstArgs>> in, out;
  Launch<TimeArgs> time;
};
inline GeneralSchedule general_schedule(const Geom& g, const double* f, double* y, double* W, const c64* tabs,
                                        int var_gen) {
  GeneralSchedule gs;
  if (W && use_padded_general(g)) {
    gs.padded = true;
    const int m = g.m;
    const long long P1 = padded_pitch(m);
    gs.in.push_back(dst_pass_custom(g, f, W, (long long)g.Nt * (g.nmodes / m), 1, m, P1, 0, 0, 0, 0, g.var_rows));
    strided_passes(g, W, gs.in);
    const int N = g.tfft.p2;
    const int V = p2sz::time_general_valid(N, var_gen) ? var_gen : 0;
    auto t = time_general_step(g, W, W, tabs);
    t.args.fft = g.tfft;
    t.args.var = V;
    t.args.S = p2sz::time_S(N, V);
    t.args.threads = p2sz::time_T(V);
    t.args.pitch = P1;
    const long long rows = g.nmodes / m;
    t.args.ystride = rows * P1;
    t.args.tiles_per_row = (int)((m + 2LL * t.args.S - 1) / (2LL * t.args.S));
    t.nwg = rows * t.args.tiles_per_row;
    t.lds = p2sz::time_general_lds(N, V, g.Nt);
    gs.time = t;
    gs.out = padded_passes(g, W, y);
  } else {
    gs.in = dst_passes(g, f, y, g.Nt, false);
    gs.time = time_general_step(g, y, y, tabs);
    gs.out = dst_passes(g, y, y, g.Nt, false);
  }
  return gs;
}

// 1D Step (b): partition solver with P = ceil(m/8) lanes per shift's system and
// S = 256/P systems per workgroup; LDS holds the 2P boundary equations of each system.
inline Launch<ThomasArgs> thomas_step(const Geom& g, SolveScalars sc, const double* alpha_dev, int variant,
                                      const double* gd, c64* s2) {
  ThomasArgs ta{};
  ta.Nt = g.Nt;
  ta.m = g.m;
  ta.tau = g.tau;
  ta.h = g.h;
  ta.sc = sc;
  ta.alpha_dev = alpha_dev;
  ta.variant = variant;
  ta.g = gd;
  ta.s2 = s2;
  ta.P = g.m == 1 ? 1 : (g.m + 7) / 8;
  ta.S = ta.P >= 256 ? 1 : 256 / ta.P;
  const long long nwg = (g.Nt + ta.S - 1) / ta.S;
  return {ta, nwg, sizeof(c64) * 4 * 2 * (size_t)ta.P * ta.S};
}

inline Launch<Time1dArgs> time1d_step(const Geom& g, SolveScalars sc, const double* alpha_dev, int variant,
                                      const c64* s2, double* y) {
  Time1dArgs t{};
  t.Nt = g.Nt;
  t.m = g.m;
  t.S = g.S_time;
  t.lev_first = 0;
  t.lev_count = g.Nt;
  t.ystride = g.m;
  t.sc = sc;
  t.alpha_dev = alpha_dev;
  t.variant = variant;
  t.tau = g.tau;
  t.s2 = s2;
  t.y = y;
  t.fft = g.tfft;
  const long long nwg = (g.m + 2LL * t.S - 1) / (2LL * t.S);
  return {t, nwg, lds_time1d(g, g.Nt)};
}

// omega and the f0 scale (Section 3.1: omega = -1/alpha, f0 = g/(tau alpha);
// Section 3.2: omega = -tau/alpha, f0 = g/alpha)
inline SolveScalars host_scalars(double alpha, int variant, double tau) {
  SolveScalars sc;
  sc.alpha = alpha;
  if (variant == 0) {
    sc.logabsw = -std::log(alpha);
    sc.f0s = 1.0 / (tau * alpha);
  } else {
    sc.logabsw = std::log(tau) - std::log(alpha);
    sc.f0s = 1.0 / alpha;
  }
  return sc;
}

}  // namespace sched
}  // namespace qbvm
