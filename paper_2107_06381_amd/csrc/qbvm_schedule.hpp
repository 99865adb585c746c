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

template <class A>
struct Launch {
  A args;
  long long nwg;
  size_t lds;
};

inline size_t lds_dst(const Geom& g) { return sizeof(c64) * ((size_t)g.S_dst * g.sfft.nc + 2 * g.S_dst); }
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
    size_t lds = lds_dst(g);
    if (g.sfft.p2) {  // compile-time power-of-two kernels
      const int N = g.sfft.p2;
      int V = input_transform ? 2 : (inner > 1 ? g.var_cols : g.var_rows);
      if (!p2sz::dst_valid(N, V)) V = 0;
      a.var = V;
      a.S = p2sz::dst_S(N, V);
      a.threads = p2sz::dst_T(N, V);
      lds = p2sz::dst_lds(N, V, inner > 1);
    }
    long long nwg;
    if (inner == 1) {
      nwg = (a.outer + 2 * a.S - 1) / (2 * a.S);
      a.tiles_per_outer = 1;
    } else {
      a.tiles_per_outer = (inner + 2 * a.S - 1) / (2 * a.S);
      nwg = a.outer * a.tiles_per_outer;
    }
    v.push_back({a, nwg, lds});
    inner *= m;
  }
  return v;
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
  size_t lds = lds_time(g, lev_count);
  if (g.tfft.p2 && p2sz::time_valid(g.tfft.p2, 0) && lev_first == 0 && lev_count == g.Nt) {
    const int N = g.tfft.p2;
    const int V = p2sz::time_valid(N, g.var_time) ? g.var_time : 0;
    t.var = V;
    t.S = p2sz::time_S(N, V);
    t.threads = p2sz::time_T(V);
    lds = p2sz::time_lds(N, V, g.Nt);
  } else {
    t.fft.p2 = 0;  // generic kernel
  }
  const long long nwg = (g.nmodes + 2LL * t.S - 1) / (2LL * t.S);
  return {t, nwg, lds};
}

inline ThomasArgs thomas_step(const Geom& g, SolveScalars sc, const double* alpha_dev, int variant,
                              const double* gd, c64* s2, c64* cp) {
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
  ta.cp = cp;
  return ta;
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
