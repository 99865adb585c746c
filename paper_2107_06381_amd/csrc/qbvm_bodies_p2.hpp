// Solve-path kernel bodies on the power-of-two FFT of qbvm_fft_p2.hpp: global
// memory is read and written straight from the FFT registers, coalesced, and
// LDS carries only the inter-stage exchanges and small tables.
#pragma once

#include "qbvm_bodies.hpp"
#include "qbvm_fft_p2.hpp"
#include "qbvm_p2_sizes.hpp"

// An optimisation barrier on an integer: the compiler must assume its value changed, so
// expressions of it are recomputed after this point rather than kept live from before.
#ifndef QBVM_OPAQUE
#define QBVM_OPAQUE(x) asm volatile("" : "+v"(x))
#endif

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

// Plane pass: per plane [m][in_pitch] of the level workspace (one time level, and one
// x_3 position in 3D), the x_2 sine transform of its columns and the x_1 sine transform
// of its rows, written unpadded to y.  Both are orthonormal DST-I of length m with
// N = 2(m+1): two real lines a, b packed as a + i b, odd extension, length-N DFT, line a
// from -Im and line b from Re of outputs 1..m (as in k_dst).  The transforms of
// different axes commute, and the plane is the smallest unit that both need whole.
// E values per lane (N/E lanes per signal, SR signals per round; E = 16: one LDS exchange
// per transform): the column pairs run in rounds (SigFast: lanes of a wave on consecutive
// pairs, coalesced 16-byte loads) and each lane keeps its outputs 1..m in registers, so
// the whole transformed plane is held by the workgroup; then for each round of row pairs
// the rows it needs go through LDS (transposed, [x_2][k_1] doubles), are read back along
// the rows (PosFast) and transformed, and the results are stored along the rows of y.
// One LDS region carries every exchange and these rows in turn; the twiddle table
// follows it.  Persistent: workgroup `first` takes planes first, first + step, ...
template <int N, int V>
__device__ __forceinline__ void dst_plane_p2_body(const PlaneArgs& a, long long first, long long step, c64* lds) {
  constexpr int E = p2sz::plane_E(V);
  constexpr int T = p2sz::plane_T(V);
  constexpr int SR = p2sz::plane_SR(N, V);
  constexpr int R = p2sz::plane_rounds(N, V);
  constexpr int U = N / E;  // lanes per signal
  using LC = P2Layout<N, E, SR, true>;
  using LR = P2Layout<N, E, SR, false, true, 1>;
  static_assert(LC::T == T && LR::T == T, "plane pass: lanes");
  static_assert(R * SR * 4 == N, "plane pass: whole rounds of pairs");
  static_assert(P2Radices<N, E>::R[0] == E, "input slot e of lane u holds position u + U e");
  // Output slot e of lane u holds position u + U (e/RL) + (N/RL) (e%RL) (last radix RL), so
  // the outputs below N/2 (the useful ones, 1..m; the others are mirror images) are
  // u + U h, h < E/2, in slot RL (h % D) + h / D with D = E/RL.
  constexpr int RL = P2Radices<N, E>::R[P2Radices<N, E>::K - 1];
  constexpr int D = E / RL;
  static_assert(D * RL == E && N / RL == U * D, "plane pass: output layout");
  constexpr int H = E / 2;
  // Row round j takes rows RJ j - 1 + (0 .. RJ-1), i.e. outputs [RJ j, RJ (j+1)): the HJ
  // useful slots h = HJ j + (0 .. HJ-1) of every lane.
  constexpr int HJ = H / R;
  constexpr int RJ = U * HJ;
  static_assert(HJ * R == H && RJ == 2 * SR, "plane pass: row rounds tile the useful outputs");
  auto slot = [](int h) { return RL * (h % D) + h / D; };
  c64* buf = lds;
  double* plane = reinterpret_cast<double*>(lds);
  const int t = threadIdx.x;
  const auto tw = p2_twiddles<N, 1, E>(a.fft, lds + p2sz::plane_region_elems(N, V), t, T);
  __syncthreads();
  const int m = a.m, PL = a.in_pitch;
  const double scale = a.scale;
  // odd extension of a line of m values at position pos: index (clamped) and sign
  auto ext = [m](int pos, double& sg) {
    const int i = odd_ext_index(pos, m, sg);
    return i < 0 ? 0 : i;
  };
  for (long long pl = first; pl < a.planes; pl += step) {
    const double* src = a.in + pl * a.in_plane;
    double* dst = a.out + pl * a.out_plane;
    // Lane coordinates are re-derived in every round: the empty asm keeps the compiler from
    // hoisting the exchange addresses of all rounds out of the loops, which holds them all
    // live at once and spills.
    // ---- x_2 transforms: column pairs (2c, 2c+1), c = r SR + sc; every pair read is in
    // the padded row (2c + 1 < in_pitch), a missing second column is zeroed
    c64 keep[R][H];
    if constexpr (p2sz::plane_preload(V)) {
      c64 v[R][E];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        int tt = t;
        QBVM_OPAQUE(tt);
        const int sc = LC::sig(tt), uc = LC::lane(tt);
        const int col = 2 * (r * SR + sc);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          double sg;
          const int i = ext(uc + U * e, sg);
          v[r][e] = *reinterpret_cast<const c64*>(src + (long long)i * PL + col);
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        int tt = t;
        QBVM_OPAQUE(tt);
        const int sc = LC::sig(tt), uc = LC::lane(tt);
        const double mb = 2 * (r * SR + sc) + 1 < m ? 1.0 : 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          double sg;
          (void)ext(uc + U * e, sg);
          v[r][e] = {sg * v[r][e].re, (mb * sg) * v[r][e].im};
        }
        p2_fft<N, E, LC>(v[r], sc, uc, buf, tw);
#pragma unroll
        for (int h = 0; h < H; ++h) keep[r][h] = v[r][slot(h)];
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        int tt = t;
        QBVM_OPAQUE(tt);
        const int sc = LC::sig(tt), uc = LC::lane(tt);
        const int col = 2 * (r * SR + sc);
        const double mb = col + 1 < m ? 1.0 : 0.0;
        c64 v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
          double sg;
          const int i = ext(uc + U * e, sg);
          const c64 w = *reinterpret_cast<const c64*>(src + (long long)i * PL + col);
          v[e] = {sg * w.re, (mb * sg) * w.im};
        }
        p2_fft<N, E, LC>(v, sc, uc, buf, tw);
#pragma unroll
        for (int h = 0; h < H; ++h) keep[r][h] = v[slot(h)];
      }
    }
    // ---- x_1 transforms, round j: rows RJ j - 1 + (0 .. RJ-1) through LDS as [row][k_1]
#pragma unroll
    for (int j = 0; j < R; ++j) {
      int tt = t;
      QBVM_OPAQUE(tt);
      const int sc = LC::sig(tt), uc = LC::lane(tt);
      const int sr = LR::sig(tt), ur = LR::lane(tt);
      // the previous exchange has been read by every lane: the region takes these rows
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int h = 0; h < HJ; ++h)  // output k = uc + U (HJ j + h), local row k - RJ j
          *reinterpret_cast<c64*>(plane + (size_t)(uc + U * h) * PL + 2 * (r * SR + sc)) =
              c64{-keep[r][HJ * j + h].im * scale, keep[r][HJ * j + h].re * scale};
      __syncthreads();
      const int row = RJ * j - 1 + 2 * sr;  // row pair (row, row + 1), local rows 2 sr, 2 sr + 1
      const double ma = (row >= 0 && row < m) ? 1.0 : 0.0, mb = (row + 1 < m) ? 1.0 : 0.0;
      c64 w[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        double sg;
        const int i = ext(ur + U * e, sg);
        w[e] = {(ma * sg) * plane[(size_t)(2 * sr) * PL + i], (mb * sg) * plane[(size_t)(2 * sr + 1) * PL + i]};
      }
      __syncthreads();  // the rows are read before the exchange reuses the region
      p2_fft<N, E, LR>(w, sr, ur, buf, tw);
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int k = ur + U * h;  // output k of the row pair = y[row][k - 1]
        const c64 x = w[slot(h)];
        if (k >= 1) {
          if (ma != 0.0) dst[(long long)row * m + k - 1] = -x.im * scale;
          if (mb != 0.0) dst[(long long)(row + 1) * m + k - 1] = x.re * scale;
        }
      }
    }
  }
}

// Length-N_t DFT X_l = sum_j x_j e^{-2 pi i jl/N_t} of each signal of the workgroup on the
// compile-time engine: N_t = N, or N_t = N + 1 prime (Rader: a cyclic convolution of
// length N carried out by two length-N transforms).  input(j, e) returns x_j for the
// lane's register slot e (-1: x_0 of a Rader length); emit(l, X_l, e) receives each
// output the lane holds, every l < N_t once per signal (e = -1: X_0 of a Rader length).
template <int N, int E, class L, bool RADER, class TW, class In, class Out>
__device__ __forceinline__ void p2_time_dft(In input, Out emit, int s, int u, c64* buf, const TW& tw,
                                            const c64* ks, const int* gfw, const int* gbw) {
  c64 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int q = p2_in_pos<N, E, 0>(u, e);
    v[e] = input(RADER ? gfw[q] : q, e);
  }
  p2_fft<N, E, L>(v, s, u, buf, tw);
  if constexpr (RADER) {
    const c64 x0 = input(0, -1);
    const c64 sum = v[0];  // position 0 on lane u == 0: sum_{j>=1} x_j
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cconj(cmul(v[e], ks[p2_out_pos<N, E>(u, e)]));
    p2_out_to_in<N, E, L>(v, s, u, buf);
    p2_fft<N, E, L>(v, s, u, buf, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) emit(gbw[p2_out_pos<N, E>(u, e)], cadd(x0, cconj(v[e])), e);
    if (u == 0) emit(0, cadd(x0, sum), -1);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) emit(p2_out_pos<N, E>(u, e), v[e], e);
  }
}

// LDS after the exchange buffer: twiddles, Rader kernel spectrum and index maps, tables.
template <int N, int E, class L, bool RADER>
struct TimeLds {
  static constexpr int TWM = p2sz::time_tw_mode(N, E);
  c64* buf;
  c64* twl;
  c64* ks;
  c64* dt;
  c64* gi;
  int* gfw;
  int* gbw;
  __device__ __forceinline__ explicit TimeLds(c64* lds, int Nt) {
    buf = lds;
    twl = buf + L::lds_elems();
    ks = twl + p2sz::tw_elems(N, TWM);
    dt = ks + N;
    gi = dt + Nt;
    gfw = reinterpret_cast<int*>(gi + Nt);
    gbw = gfw + N;
  }
  // past the two index maps: further per-kernel tables
  __device__ __forceinline__ c64* extra() const { return reinterpret_cast<c64*>(gbw + N); }
  __device__ __forceinline__ void load_rader(const FftPlanDev& f, int t, int T) const {
    if constexpr (RADER) {
      for (int i = t; i < N; i += T) {
        ks[i] = f.kspec[i];
        gfw[i] = f.gfwd[i];
        gbw[i] = f.ginvt[i];
      }
    }
  }
};

// Modes of a time tile: flattened (pitch 0) or 2S consecutive x_1 of one padded row.
struct TimeTile {
  long long ka, oa;
  bool oka, okb;
  __device__ __forceinline__ TimeTile(const TimeArgs& a, long long wg, int S, int s) {
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
  }
  // gamma_l^{-1} X_l to level l: real part -> first mode, imaginary part -> second.
  // Padded rows (pitch > 0): the pair is one aligned 16-byte store; a pair whose second
  // mode is past the row end writes that value into the row padding.
  __device__ __forceinline__ void store(const TimeArgs& a, int l, c64 yv) const {
    double* yl = a.y + (long long)l * a.ystride;
    if (a.pitch > 0) {
      if (oka) *reinterpret_cast<c64*>(yl + oa) = yv;
    } else {
      if (oka) yl[oa] = yv.re;
      if (okb) yl[oa + 1] = yv.im;
    }
  }
};

// Spectral time kernel, every level written.  RADER: N_t = N + 1 prime; else N_t = N.
// Persistent: workgroup `first` takes tiles first, first + step, ... < a.ntiles; the
// per-solve tables are loaded once, and the sine coefficients and eigenvalues of the
// next tile are loaded while the current one is transformed.
template <int N, int E, int S, bool RADER, bool PAD, bool PAIR>
__device__ __forceinline__ void time_p2_body(const TimeArgs& a, long long first, long long step, c64* lds) {
  static_assert(S >= 1, "time kernel needs N <= 2048");
  using L = P2Layout<N, E, S, true, PAD>;
  using M = TimeLds<N, E, L, RADER>;
  using Tile = TimeTileR<PAIR>;
  const long long ntiles = a.ntiles;
  if (first >= ntiles) return;  // whole workgroup, before any barrier
  const int Nt = a.Nt;
  const M sh(lds, Nt);
  const int t = threadIdx.x, s = L::sig(t), u = L::lane(t);

  long long wg = first;
  double ga, gb, mua, mub;
  Tile(a, wg, S, s).fetch(a, ga, gb, mua, mub);

  const SolveScalars sc = solve_scalars(a.sc, a.alpha_dev, a.variant, a.tau);
  const double croot = exp(sc.logabsw / (double)Nt);
  const double inv_tau = 1.0 / a.tau;
  const double gscale = sc.f0s / (double)Nt;
  if (a.tabs) {  // d_j/tau and gamma_l^{-1} f0s/N_t precomputed for this solve
    for (int j = t; j < Nt; j += L::T) {
      sh.dt[j] = a.tabs[j];
      sh.gi[j] = a.tabs[Nt + j];
    }
  } else {
    for (int j = t; j < Nt; j += L::T) {
      sh.dt[j] = shift_over_tau(j, Nt, croot, inv_tau);
      sh.gi[j] = inv_gamma(j, Nt, sc.logabsw, gscale);
    }
  }
  sh.load_rader(a.fft, t, L::T);
  const auto tw = p2_twiddles<N, M::TWM, E>(a.fft, sh.twl, t, L::T, u);
  __syncthreads();

  for (;;) {
    const Tile tile(a, wg, S, s);
    const long long nx = wg + step;
    double nga = 0.0, ngb = 0.0, nmua = 0.0, nmub = 0.0;
    if (nx < ntiles) Tile(a, nx, S, s).fetch(a, nga, ngb, nmua, nmub);
    // Steps (a)+(b): u_j = g_a/(d_j/tau + mu_a) + i g_b/(d_j/tau + mu_b)
    auto input = [&](int j, int) -> c64 {
      const c64 z = sh.dt[j];
      const double xa = z.re + mua, xb = z.re + mub;
      double qa, qb;
      recip2_nr(xa * xa + z.im * z.im, xb * xb + z.im * z.im, qa, qb);
      const double ia = ga * qa, ib = gb * qb;
      return {ia * xa + ib * z.im, ib * xb - ia * z.im};
    };
    auto emit = [&](int l, c64 X, int) { tile.store(a, l, cmul(sh.gi[l], X)); };
    p2_time_dft<N, E, L, RADER>(input, emit, s, u, sh.buf, tw, sh.ks, sh.gfw, sh.gbw);
    if (nx >= ntiles) break;
    wg = nx;
    ga = nga;
    gb = ngb;
    mua = nmua;
    mub = nmub;
  }
}

// Time kernel of the general right-hand side on the compile-time engine.  Per signal
// (modes a, b packed as f_a + i f_b, levels t < N_t read from fgen):
//   z_j = sum_t gamma_t f_t e^{+2 pi i jt/N_t} = conj(DFT(conj(gamma f)))_j;
//   for real f_a, f_b the two modes' transforms separate through the pair (j, N_t-1-j):
//   Z_a(N_t-1-j) = conj Z_a(j), so Z_a = (z_j + conj z_{N_t-1-j})/2 and
//   Z_b = (z_j - conj z_{N_t-1-j})/(2i);
//   w_j = Z_a/(d_j/tau + mu_a) + i Z_b/(d_j/tau + mu_b);
//   y_l = gamma_l^{-1}/N_t DFT(w)_l, real part -> mode a, imaginary part -> mode b.
// The z exchange reuses the engine buffer ([j][s], position 0 of a Rader length in
// its own slot).  fgen and y may alias: a tile reads every level before it writes.
template <int N, int E, int S, bool RADER, bool PAD = true>
__device__ __forceinline__ void time_general_p2_body(const TimeArgs& a, long long wg, c64* lds) {
  static_assert(S >= 1, "time kernel needs N <= 2048");
  using L = P2Layout<N, E, S, true, PAD>;
  using M = TimeLds<N, E, L, RADER>;
  static_assert((size_t)N * S <= L::lds_elems(), "z exchange fits the engine buffer");
  const int Nt = a.Nt;
  const M sh(lds, Nt);
  c64* gam = sh.extra();
  c64* side = gam + Nt;   // S: z_0 of a Rader length
  double* mus = reinterpret_cast<double*>(side + S);  // 2 S
  const int t = threadIdx.x, s = L::sig(t), u = L::lane(t);
  for (int j = t; j < Nt; j += L::T) {
    sh.dt[j] = a.tabs[j];
    sh.gi[j] = a.tabs[Nt + j];
    gam[j] = a.tabs[2 * Nt + j];
  }
  sh.load_rader(a.fft, t, L::T);
  const auto tw = p2_twiddles<N, M::TWM, E>(a.fft, sh.twl, t, L::T, u);
  const TimeTile tile(a, wg, S, s);
  if (u == 0) {
    mus[2 * s] = tile.oka ? mode_mu(tile.ka, a.d, a.m, a.mu1d) : 0.0;
    mus[2 * s + 1] = tile.okb ? mode_mu(tile.ka + 1, a.d, a.m, a.mu1d) : 0.0;
  }
  __syncthreads();

  const bool pair = a.pitch > 0;
  auto load = [&](int j, int) -> c64 {
    const double* fl = a.fgen + (long long)j * a.ystride;
    c64 f = {0.0, 0.0};
    if (pair) {
      if (tile.oka) f = *reinterpret_cast<const c64*>(fl + tile.oa);
      if (!tile.okb) f.im = 0.0;  // row padding
    } else {
      if (tile.oka) f.re = fl[tile.oa];
      if (tile.okb) f.im = fl[tile.oa + 1];
    }
    return cconj(cmul(gam[j], f));
  };
  auto zslot = [&](int j) -> c64& {
    if constexpr (RADER) return j == 0 ? side[s] : sh.buf[(size_t)(j - 1) * S + s];
    else return sh.buf[(size_t)j * S + s];
  };
  c64 zk[E], z0 = {0.0, 0.0};
  int jk[E];
  auto keep = [&](int j, c64 X, int e) {
    if (e < 0) z0 = X;
    else {
      zk[e] = X;
      jk[e] = j;
    }
  };
  p2_time_dft<N, E, L, RADER>(load, keep, s, u, sh.buf, tw, sh.ks, sh.gfw, sh.gbw);
  __syncthreads();  // the engine buffer is free: z = conj X, natural order
#pragma unroll
  for (int e = 0; e < E; ++e) zslot(jk[e]) = cconj(zk[e]);
  if (RADER && u == 0) zslot(0) = cconj(z0);
  __syncthreads();
  const double mua = mus[2 * s], mub = mus[2 * s + 1];
  auto wfun = [&](int j) -> c64 {
    const c64 zj = zslot(j);
    const c64 zr = cconj(zslot(Nt - 1 - j));
    const c64 za = {0.5 * (zj.re + zr.re), 0.5 * (zj.im + zr.im)};
    const c64 zb = {0.5 * (zj.im - zr.im), -0.5 * (zj.re - zr.re)};
    const c64 z = sh.dt[j];
    const double xa = z.re + mua, xb = z.re + mub;
    double qa, qb;
    recip2_nr(xa * xa + z.im * z.im, xb * xb + z.im * z.im, qa, qb);
    const c64 wa = {(za.re * xa + za.im * z.im) * qa, (za.im * xa - za.re * z.im) * qa};
    const c64 wb = {(zb.re * xb + zb.im * z.im) * qb, (zb.im * xb - zb.re * z.im) * qb};
    return {wa.re - wb.im, wa.im + wb.re};
  };
  // the second transform writes the engine buffer: gather this lane's inputs first
  c64 w[E], w0 = {0.0, 0.0};
#pragma unroll
  for (int e = 0; e < E; ++e) w[e] = wfun(RADER ? sh.gfw[p2_in_pos<N, E, 0>(u, e)] : p2_in_pos<N, E, 0>(u, e));
  if constexpr (RADER) w0 = wfun(0);
  __syncthreads();
  auto winput = [&](int, int e) -> c64 { return e < 0 ? w0 : w[e]; };
  auto emit = [&](int l, c64 X, int) { tile.store(a, l, cmul(sh.gi[l], X)); };
  p2_time_dft<N, E, L, RADER>(winput, emit, s, u, sh.buf, tw, sh.ks, sh.gfw, sh.gbw);
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
