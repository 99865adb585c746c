// Host-side FFT planning: Stockham factorisation, Rader and Bluestein tables,
// twiddles and radix roots, computed in long double and rounded once to double.
// Plain C++ (no HIP runtime), shared by the executor and the CPU build of the
// kernels used in the tests.
#pragma once

#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "qbvm_types.hpp"
#include "qbvm_p2_sizes.hpp"

namespace qbvm {
namespace plan {

constexpr long double kPiL = 3.141592653589793238462643383279502884L;
constexpr int kThreads = 256;
constexpr int kMaxCore = kElemsPerThread * kThreads;  // 4096

inline bool is_prime(int n) {
  if (n < 2) return false;
  for (int p = 2; (long long)p * p <= n; ++p)
    if (n % p == 0) return false;
  return true;
}

inline std::vector<int> prime_factors(int n) {
  std::vector<int> f;
  for (int p = 2; (long long)p * p <= n; ++p)
    while (n % p == 0) {
      f.push_back(p);
      n /= p;
    }
  if (n > 1) f.push_back(n);
  return f;
}

inline bool supported_odd(int p, int maxodd) {
  static const int odd[] = {3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47};
  for (int q : odd)
    if (q == p) return p <= maxodd;
  return false;
}

inline bool smooth(int n, int maxodd) {
  for (int p : prime_factors(n))
    if (p != 2 && !supported_odd(p, maxodd)) return false;
  return true;
}

// radices of a Stockham factorisation: 16s, then 8/4/2, then odd primes ascending
inline std::vector<int> radices(int n) {
  std::vector<int> r;
  int e = 0;
  while (n % 2 == 0) {
    n /= 2;
    ++e;
  }
  while (e >= 4) {
    r.push_back(16);
    e -= 4;
  }
  if (e == 3) r.push_back(8);
  if (e == 2) r.push_back(4);
  if (e == 1) r.push_back(2);
  for (int p : prime_factors(n)) r.push_back(p);
  return r;
}

inline std::complex<long double> unit_root(long long k, long long n, int sign) {
  // exp(sign * 2 pi i k / n) with k reduced mod n
  k %= n;
  if (k < 0) k += n;
  const long double a = 2.0L * kPiL * (long double)k / (long double)n;
  return {cosl(a), sign * sinl(a)};
}

inline int primitive_root(int p) {
  const std::vector<int> f = prime_factors(p - 1);
  for (int g = 2; g < p; ++g) {
    bool ok = true;
    for (int q : f) {
      long long x = 1, b = g, e = (p - 1) / q;
      while (e) {
        if (e & 1) x = x * b % p;
        b = b * b % p;
        e >>= 1;
      }
      if (x == 1) {
        ok = false;
        break;
      }
    }
    if (ok) return g;
  }
  return -1;
}

// direct DFT (forward, long double) divided by the length
inline std::vector<c64> dft_over_len(const std::vector<std::complex<long double>>& b) {
  const long long M = (long long)b.size();
  std::vector<std::complex<long double>> W(M);
  for (long long k = 0; k < M; ++k) W[k] = unit_root(k, M, -1);
  std::vector<c64> out(M);
  for (long long k = 0; k < M; ++k) {
    std::complex<long double> s = 0;
    for (long long j = 0; j < M; ++j) s += b[j] * W[(j * k) % M];
    s /= (long double)M;
    out[k] = {(double)s.real(), (double)s.imag()};
  }
  return out;
}

struct HostFft {
  FftPlanDev dev{};  // pointers left null; the caller points them at its copies
  std::vector<c64> tw, kspec, chirp;
  std::vector<int> rin, rout, gfwd, ginvt;
};

inline bool is_p2_core(int nc) { return nc >= 64 && nc <= 4096 && (nc & (nc - 1)) == 0; }

inline void fill_stages(FftPlanDev& d, int nc) {
  const std::vector<int> r = radices(nc);
  d.nc = nc;
  d.nstages = (int)r.size();
  int ns = 1;
  d.wide = 0;
  for (size_t i = 0; i < r.size(); ++i) {
    d.st[i].radix = r[i];
    d.st[i].ns = ns;
    d.st[i].twstride = nc / (ns * r[i]);
    ns *= r[i];
    if (r[i] % 2 == 1 && r[i] > kMaxOddRadixNarrow) d.wide = 1;
  }
}

// Tables of a forward DFT of logical length n; returns false (with a message) if
// the core transform would exceed what one workgroup handles.  sine: the DFT of a sine
// transform's odd extension (n = 2(m+1), input x_{n-j} = -x_j with x_0 = x_{n/2} = 0, only
// outputs 1..n/2-1 used).  A sine length without a power-of-two kernel gets the symmetric
// Bluestein form run by the compile-time sine kernel (`bp2`): with h = n/2 and w_t = exp(i pi t^2/n),
// the chirp-weighted input a_j = x_j conj(w_j) obeys a_{j+h} = -a_{h-j}, so the inputs
// j >= h are the negated mirror image of the first half and their transform is the first
// half's at -k times exp(-2 pi i k h/P).  The convolution then runs over inputs j < h and
// outputs k < h only, on a power-of-two core P >= n - 1 (64..4096), with two kernel
// spectra: kspec[k] for the first half and kspec[P + k] (the phase and the sign folded
// in) for the mirrored one.  No other kernel reads these tables.
inline bool build_tables(int n, HostFft& t, std::string& err, bool sine = false) {
  FftPlanDev& d = t.dev;
  d.n = n;
  const bool sym = sine && n % 2 == 0;
  int symP = 64;
  while (symP < n - 1) symP *= 2;
  // Prefer cores whose radices are all <= 7 (the narrow kernels keep a butterfly in
  // registers without spilling): Stockham, Rader on n - 1, else Bluestein if its core
  // fits; only lengths beyond that use the wide kernels (odd radices up to 47).
  int nc;
  int blue = 2 * n - 1;
  while (!smooth(blue, kMaxOddRadixNarrow)) ++blue;
  if (sym && !is_p2_core(n) && symP <= kMaxCore) {
    // every sine length without a power-of-two kernel, 7-smooth ones included: the
    // symmetric form on the compile-time engine measured faster than the runtime
    // Stockham engine (2D m = 159, N = 320: whole solve 182 -> 147 us)
    d.kind = kBluestein;
    nc = symP;
  } else if (smooth(n, kMaxOddRadixNarrow)) {
    d.kind = kStockham;
    nc = n;
  } else if (is_prime(n) && smooth(n - 1, kMaxOddRadixNarrow)) {
    d.kind = kRader;
    nc = n - 1;
  } else if (sym && symP <= kMaxCore) {
    d.kind = kBluestein;
    nc = symP;
  } else if (blue <= kMaxCore) {
    // Bluestein core: the 7-smooth length >= 2n - 1 with the fewest element-stages
    // (length x number of Stockham stages), since the engine's cost per stage is mostly
    // one LDS round trip per element: 640 = 16.8.5 (3 stages) beats 625 = 5^4 (4)
    d.kind = kBluestein;
    nc = blue;
    long long best = (long long)blue * (long long)radices(blue).size();
    for (int c = blue + 1; c < 2 * blue && c <= kMaxCore; ++c) {
      if (!smooth(c, kMaxOddRadixNarrow)) continue;
      const long long cost = (long long)c * (long long)radices(c).size();
      if (cost < best) {
        best = cost;
        nc = c;
      }
    }
  } else if (smooth(n, kMaxOddRadixWide)) {
    d.kind = kStockham;
    nc = n;
  } else if (is_prime(n) && smooth(n - 1, kMaxOddRadixWide)) {
    d.kind = kRader;
    nc = n - 1;
  } else {
    d.kind = kBluestein;
    nc = blue;
  }
  if (nc > kMaxCore) {
    err = "FFT length " + std::to_string(n) + " needs a core of " + std::to_string(nc) + " > 4096";
    return false;
  }
  if ((int)radices(nc).size() > kMaxStages) {
    err = "too many FFT stages";
    return false;
  }
  fill_stages(d, nc);
  t.tw.resize(nc);
  for (int k = 0; k < nc; ++k) {
    auto w = unit_root(k, nc, -1);
    t.tw[k] = {(double)w.real(), (double)w.imag()};
  }
  if (d.kind == kRader) {
    const int g = primitive_root(n);
    t.rin.assign(n, 0);
    t.rout.assign(n, 0);
    long long x = 1;
    t.gfwd.assign(n - 1, 0);
    t.ginvt.assign(n - 1, 0);
    for (int q = 0; q < n - 1; ++q) {  // g^q
      t.rin[(int)x] = q;
      t.gfwd[q] = (int)x;
      x = x * g % n;
    }
    long long ginv = 1, b = g, e = n - 2;  // g^{-1} = g^{n-2}
    while (e) {
      if (e & 1) ginv = ginv * b % n;
      b = b * b % n;
      e >>= 1;
    }
    std::vector<std::complex<long double>> bb(n - 1);
    x = 1;
    for (int p = 0; p < n - 1; ++p) {  // g^{-p}
      t.rout[(int)x] = p;
      t.ginvt[p] = (int)x;
      bb[p] = unit_root(x, n, -1);
      x = x * ginv % n;
    }
    t.kspec = dft_over_len(bb);
  } else if (d.kind == kBluestein) {
    t.chirp.resize(n);
    std::vector<std::complex<long double>> w(n);  // w_t = w_{-t}, t < n
    for (long long k = 0; k < n; ++k) {
      const long long e2 = (k * k) % (2LL * n);
      w[k] = unit_root(e2, 2LL * n, +1);  // exp(i pi k^2/n)
      t.chirp[k] = {(double)w[k].real(), (double)w[k].imag()};
    }
    auto wt = [&](long long x) { return w[x < 0 ? -x : x]; };
    if (sym && nc == symP) {
      // offsets s = k - j in [-(h-1), h-1] of outputs k < h and inputs j < h; the first
      // half's kernel is w_s, the mirrored half's w_{s-h}
      const long long h = n / 2, P = nc;
      std::vector<std::complex<long double>> blo(P, 0), bhi(P, 0);
      for (long long x = -(h - 1); x <= h - 1; ++x) {
        blo[(x + P) % P] = wt(x);
        bhi[(x + P) % P] = wt(x - h);
      }
      const std::vector<c64> Blo = dft_over_len(blo), Bhi = dft_over_len(bhi);
      t.kspec.resize(2 * P);
      for (long long k = 0; k < P; ++k) {
        t.kspec[k] = Blo[k];
        const std::complex<long double> ph = -unit_root(k * h, P, -1);
        const std::complex<long double> v = ph * std::complex<long double>(Bhi[k].re, Bhi[k].im);
        t.kspec[P + k] = {(double)v.real(), (double)v.imag()};
      }
    } else {
      // kernel b_t = w_t at offsets t in (-n, n): t >= 0 at position t, t < 0 at nc + t
      std::vector<std::complex<long double>> bb(nc, 0);
      for (long long k = 0; k < n; ++k) {
        bb[k] = w[k];
        if (k > 0) bb[nc - k] = w[k];
      }
      t.kspec = dft_over_len(bb);
    }
  }
  d.p2 = (d.kind != kBluestein && is_p2_core(nc)) ? nc : 0;
  d.bp2 = (d.kind == kBluestein && sym && nc == symP) ? nc : 0;
  d.gtA = d.gtB = 0;
  for (const auto& pr : p2sz::kGtPairs)
    if (pr[0] * pr[1] == n) {
      d.gtA = pr[0];
      d.gtB = pr[1];
    }
  return true;
}

// exp(-2 pi i k/R) for R = 1..64 at index R (R-1)/2 + k
inline std::vector<c64> radix_roots() {
  std::vector<c64> roots(2080);
  for (int R = 1; R <= 64; ++R)
    for (int k = 0; k < R; ++k) {
      auto w = unit_root(k, R, -1);
      roots[R * (R - 1) / 2 + k] = {(double)w.real(), (double)w.imag()};
    }
  return roots;
}

// signals per workgroup for a core length: S * nc <= 4096, at most 32
inline int signals_for(int nc) { return nc >= kMaxCore ? 1 : (kMaxCore / nc > 32 ? 32 : kMaxCore / nc); }

}  // namespace plan
}  // namespace qbvm
