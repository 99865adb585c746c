// Solve-path kernel bodies on the power-of-two FFT of qbvm_fft_p2.hpp: global
// memory is read and written straight from the FFT registers, coalesced, and
// LDS carries only the inter-stage exchanges and small tables.
#pragma once

#include "qbvm_bodies.hpp"
#include "qbvm_fft_p2.hpp"
#include "qbvm_p2_sizes.hpp"

namespace qbvm {


// value of the odd extension v_n = [0, x_1..x_m, 0, -x_m..-x_1] at n (0 <= n < 2(m+1)), or -1
__device__ __forceinline__ int odd_ext_index(int n, int m, double& sign) {
  const int M = m + 1;
  if (n >= 1 && n <= m) {
    sign = 1.0;
    return n - 1;
  }
  if (n > M) {
    sign = -1.0;
    return 2 * M - n - 1;
  }
  sign = 0.0;
  return -1;
}

// Twiddle accessor of the given table mode; modes 1 and 2 copy the table into LDS
// at tw_lds (the caller synchronises before the first use).
template <int N, int TWM = (p2sz::tw_in_lds(N) ? 1 : 0), int E = 8>
__device__ __forceinline__ auto p2_twiddles(const FftPlanDev& f, c64* tw_lds, int t, int T, int u = 0) {
  if constexpr (TWM == 3) {  // per-lane registers, loaded once
    (void)tw_lds;
    (void)t;
    (void)T;
    return p2_tw_regs<N, E>(f.tw, u);
  } else if constexpr (TWM == 2) {
    for (int i = t; i < 64 + N / 64; i += T) tw_lds[i] = i < 64 ? f.tw[i] : f.tw[(i - 64) * 64];
    return TwSplit{tw_lds, tw_lds + 64};
  } else if constexpr (TWM == 1) {
    for (int i = t; i < N; i += T) tw_lds[i] = f.tw[i];
    return TwFull{tw_lds};
  } else {
    return TwFull{f.tw};
  }
}

// The sine passes are persistent: a workgroup takes the tiles first, first + step,
// ... and loads the lines of its next tile into registers while the current tile
// is transformed, so global-load latency overlaps the FFT.  Lines past the end are
// read at a clamped, valid address and zeroed before the transform.

// Rows of [outer][m] (inner == 1): lanes walk along lines, two lines per signal.
template <int N, int E, int S, int TWM, int PM = 1>
__device__ __forceinline__ void dst_rows_p2_body(const DstArgs& a, long long first, long long step, c64* lds) {
  using L = P2Layout<N, E, S, false, true, PM>;
  c64* buf = lds;
  const int t = threadIdx.x, s = L::sig(t), u = L::lane(t);
  tab_job_run(a.tab, first * L::T + t, step * L::T);
  const auto tw = p2_twiddles<N, TWM, E>(a.fft, buf + L::lds_elems(), t, L::T, u);
  __syncthreads();
  const int m = a.len;
  const long long ntiles = (a.outer + 2LL * S - 1) / (2LL * S);
  const long long last = a.outer - 1;
  double ra[E], rb[E];
  auto fetch = [&](long long tile) {
    const long long la = tile * 2LL * S + 2 * s, lb = la + 1;
    const double* xa = a.in + (la < last ? la : last) * a.in_pitch;
    const double* xb = a.in + (lb < last ? lb : last) * a.in_pitch;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      double sg;
      const int i = odd_ext_index(p2_in_pos<N, E, 0>(u, e), m, sg);
      ra[e] = xa[i < 0 ? 0 : i];
      rb[e] = xb[i < 0 ? 0 : i];
    }
  };
  if (first < ntiles) fetch(first);
  for (long long tile = first; tile < ntiles; tile += step) {
    const long long la = tile * 2LL * S + 2 * s, lb = la + 1;
    const bool oka = la < a.outer, okb = lb < a.outer;
    c64 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      double sg;
      (void)odd_ext_index(p2_in_pos<N, E, 0>(u, e), m, sg);
      v[e] = {oka ? sg * ra[e] : 0.0, okb ? sg * rb[e] : 0.0};
    }
    if (tile + step < ntiles) fetch(tile + step);
    p2_fft<N, E, L>(v, s, u, buf, tw);
    double* oa = a.out + la * a.out_pitch;
    double* ob = a.out + lb * a.out_pitch;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = p2_out_pos<N, E>(u, e);
      if (i >= 1 && i <= m) {
        if (oka) oa[i - 1] = -v[e].im * a.scale;
        if (okb) ob[i - 1] = v[e].re * a.scale;
      }
    }
  }
}

// column c of a columns pass holds data (32-bit form: inner < 2^31 is checked on the host)
__device__ __forceinline__ bool dst_col_ok32(const DstArgs& a, long long c) {
  return c < a.inner && (a.colmod == 0 || ((int)c % a.colmod) < a.colvalid);
}

// Columns of [outer][m][inner] (inner > 1): lanes of a wave take consecutive columns.
// VEC2: the two columns of a signal are one aligned 16-byte pair (padded layout:
// inner, kstride and ostride even); a pair with only its first column valid is
// stored whole, its second value landing in a padding column.
template <int N, int E, int S, bool VEC2, int TWM>
__device__ __forceinline__ void dst_cols_p2_body(const DstArgs& a, long long first, long long step, c64* lds) {
  using L = P2Layout<N, E, S, true>;
  c64* buf = lds;
  const int t = threadIdx.x, s = L::sig(t), u = L::lane(t);
  tab_job_run(a.tab, first * L::T + t, step * L::T);
  const auto tw = p2_twiddles<N, TWM, E>(a.fft, buf + L::lds_elems(), t, L::T, u);
  __syncthreads();
  const int m = a.len;
  const long long tpo = a.tiles_per_outer;
  const long long ntiles = a.outer * tpo;
  const long long cmax = a.inner - (VEC2 ? 2 : 1);
  double ra[E], rb[E];
  auto fetch = [&](long long tile) {
    const long long o = tile / tpo;
    const long long ca = (tile - o * tpo) * 2LL * S + 2 * s;
    const double* base = a.in + o * a.ostride;
    const long long pa = ca < cmax ? ca : cmax;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      double sg;
      const int i = odd_ext_index(p2_in_pos<N, E, 0>(u, e), m, sg);
      const double* row = base + (long long)(i < 0 ? 0 : i) * a.kstride;
      if constexpr (VEC2) {
        const c64 w = *reinterpret_cast<const c64*>(row + pa);  // (column pa, column pa + 1)
        ra[e] = w.re;
        rb[e] = w.im;
      } else {
        ra[e] = row[pa];
        rb[e] = row[ca + 1 < cmax ? ca + 1 : cmax];
      }
    }
  };
  if (first < ntiles) fetch(first);
  for (long long tile = first; tile < ntiles; tile += step) {
    const long long o = tile / tpo;
    const long long ca = (tile - o * tpo) * 2LL * S + 2 * s, cb = ca + 1;
    const bool oka = dst_col_ok32(a, ca), okb = dst_col_ok32(a, cb);
    c64 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      double sg;
      (void)odd_ext_index(p2_in_pos<N, E, 0>(u, e), m, sg);
      v[e] = {oka ? sg * ra[e] : 0.0, okb ? sg * rb[e] : 0.0};
    }
    if (tile + step < ntiles) fetch(tile + step);
    p2_fft<N, E, L>(v, s, u, buf, tw);
    double* obase = a.out + o * a.ostride;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = p2_out_pos<N, E>(u, e);
      if (i >= 1 && i <= m) {
        double* row = obase + (long long)(i - 1) * a.kstride;
        if constexpr (VEC2) {
          if (oka) *reinterpret_cast<c64*>(row + ca) = c64{-v[e].im * a.scale, v[e].re * a.scale};
        } else {
          if (oka) row[ca] = -v[e].im * a.scale;
          if (okb) row[cb] = v[e].re * a.scale;
        }
      }
    }
  }
}

// Spectral time kernel, every level written.  RADER: N_t = N + 1 prime; else N_t = N.
template <int N, int E, int S, bool RADER, bool PAD = true>
__device__ __forceinline__ void time_p2_body(const TimeArgs& a, long long wg, c64* lds) {
  static_assert(S >= 1, "time kernel needs N <= 2048");
  using L = P2Layout<N, E, S, true, PAD>;
  const int Nt = a.Nt;
  c64* buf = lds;
  constexpr int TWM = p2sz::time_tw_mode(N, E);
  c64* twl = buf + L::lds_elems();
  c64* ks = twl + p2sz::tw_elems(N, TWM);
  c64* dt = ks + N;
  c64* gi = dt + Nt;
  int* gfw = reinterpret_cast<int*>(gi + Nt);
  int* gbw = gfw + N;
  const int t = threadIdx.x, s = L::sig(t), u = L::lane(t);

  SolveScalars sc = a.sc;
  if (a.alpha_dev) sc = scalars_from_alpha(*a.alpha_dev, a.variant, a.tau);
  const double croot = exp(sc.logabsw / (double)Nt);
  const double inv_tau = 1.0 / a.tau;
  const double gscale = sc.f0s / (double)Nt;
  if (a.tabs) {  // d_j/tau and gamma_l^{-1} f0s/N_t precomputed for this solve
    for (int j = t; j < Nt; j += L::T) {
      dt[j] = a.tabs[j];
      gi[j] = a.tabs[Nt + j];
    }
  } else {
    for (int j = t; j < Nt; j += L::T) {
      dt[j] = shift_over_tau(j, Nt, croot, inv_tau);
      gi[j] = inv_gamma(j, Nt, sc.logabsw, gscale);
    }
  }
  if constexpr (RADER) {
    for (int i = t; i < N; i += L::T) {
      ks[i] = a.fft.kspec[i];
      gfw[i] = a.fft.gfwd[i];
      gbw[i] = a.fft.ginvt[i];
    }
  }
  const auto tw = p2_twiddles<N, TWM, E>(a.fft, twl, t, L::T, u);
  __syncthreads();

  // modes of this tile: flattened (pitch 0) or 2S consecutive x_1 of one padded row
  long long ka, oa;
  bool oka, okb;
  if (a.pitch > 0) {
    const long long row = wg / a.tiles_per_row;
    const int c1 = (int)(wg - row * a.tiles_per_row) * 2 * S + 2 * s;
    ka = row * a.m + c1;
    oa = row * a.pitch + c1;
    oka = c1 < a.m;
    okb = c1 + 1 < a.m;
  } else {
    ka = wg * 2LL * S + 2 * s;
    oa = ka;
    oka = ka < a.nmodes;
    okb = ka + 1 < a.nmodes;
  }
  const long long kb = ka + 1;
  const double ga = oka ? a.ghat[ka] : 0.0, gb = okb ? a.ghat[kb] : 0.0;
  const double mua = oka ? mode_mu(ka, a.d, a.m, a.mu1d) : 0.0;
  const double mub = okb ? mode_mu(kb, a.d, a.m, a.mu1d) : 0.0;
  // Steps (a)+(b): u_j = g_a/(d_j/tau + mu_a) + i g_b/(d_j/tau + mu_b)
  auto input = [&](int j) -> c64 {
    const c64 z = dt[j];
    const double xa = z.re + mua, xb = z.re + mub;
    const double ia = ga * recip_nr(xa * xa + z.im * z.im);
    const double ib = gb * recip_nr(xb * xb + z.im * z.im);
    return {ia * xa + ib * z.im, ib * xb - ia * z.im};
  };
  c64 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int q = p2_in_pos<N, E, 0>(u, e);
    v[e] = input(RADER ? gfw[q] : q);
  }
  p2_fft<N, E, L>(v, s, u, buf, tw);
  // padded rows (pitch > 0): the pair is one aligned 16-byte store; a pair whose
  // second mode is past the row end writes that value into the row padding
  const bool pair = a.pitch > 0;
  auto store = [&](int l, c64 X) {
    const c64 yv = cmul(gi[l], X);
    double* yl = a.y + (long long)l * a.ystride;
    if (pair) {
      if (oka) *reinterpret_cast<c64*>(yl + oa) = yv;
    } else {
      if (oka) yl[oa] = yv.re;
      if (okb) yl[oa + 1] = yv.im;
    }
  };
  if constexpr (RADER) {
    const c64 x0 = input(0);
    const c64 sum = v[0];  // position 0 on lane u == 0: sum_{j>=1} x_j
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cconj(cmul(v[e], ks[p2_out_pos<N, E>(u, e)]));
    p2_out_to_in<N, E, L>(v, s, u, buf);
    p2_fft<N, E, L>(v, s, u, buf, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) store(gbw[p2_out_pos<N, E>(u, e)], cadd(x0, cconj(v[e])));
    if (u == 0) store(0, cadd(x0, sum));
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) store(p2_out_pos<N, E>(u, e), v[e]);
  }
}

}  // namespace qbvm

namespace qbvm {
// the host-side LDS sizes must cover the layouts used by the bodies
template <int N>
constexpr bool p2_first_radix_ok() {
  return p2sz::first_radix(N, 16) == P2Radices<N, 16>::R[0] && p2sz::first_radix(N, 8) == P2Radices<N, 8>::R[0];
}
static_assert(p2_first_radix_ok<64>() && p2_first_radix_ok<128>() && p2_first_radix_ok<256>() &&
                  p2_first_radix_ok<512>() && p2_first_radix_ok<1024>() && p2_first_radix_ok<2048>() &&
                  p2_first_radix_ok<4096>(),
              "first-radix table out of step with P2Radices");
}  // namespace qbvm
