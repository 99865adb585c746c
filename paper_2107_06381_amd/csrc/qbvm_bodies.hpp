// Kernel bodies of the solve path, written against the HIP device model
// (threadIdx, blockDim, __syncthreads, LDS pointer passed in).  Included by the
// gfx950 kernels and, with a thin shim, by the CPU build used in the tests.
#pragma once

#include <type_traits>

#include "qbvm_fft_dev.hpp"

namespace qbvm {

// ------------------------------------------------------------------ helpers
// omega and f0 scale from alpha (Sections 3.1, 3.2)
__device__ __forceinline__ SolveScalars scalars_from_alpha(double alpha, int variant, double tau) {
  SolveScalars s;
  if (variant == 0) {
    s.logabsw = -log(alpha);          // |omega| = 1/alpha
    s.f0s = 1.0 / (tau * alpha);
  } else {
    s.logabsw = log(tau) - log(alpha);  // |omega| = tau/alpha
    s.f0s = 1.0 / alpha;
  }
  return s;
}

// The solve's scalars on the device, from alpha in a device table entry or from the value
// the host passed: every path (one solve, batched, alpha choice) derives them with the
// same arithmetic, so they give bitwise the same results for the same alpha.
__device__ __forceinline__ SolveScalars solve_scalars(const SolveScalars& host, const double* alpha_dev,
                                                      int variant, double tau) {
  SolveScalars s = scalars_from_alpha(alpha_dev ? *alpha_dev : host.alpha, variant, tau);
  s.alpha = alpha_dev ? *alpha_dev : host.alpha;
  return s;
}

// d_j / tau with d_j = 1 - omega^{1/N_t} theta^j = 1 - |omega|^{1/N_t} exp(i pi (2j+1)/N_t)
__device__ __forceinline__ c64 shift_over_tau(int j, int Nt, double croot, double inv_tau) {
  double sn, cs;
  sincospi((double)(2 * j + 1) / (double)Nt, &sn, &cs);
  return {(1.0 - croot * cs) * inv_tau, -croot * sn * inv_tau};
}

// scale * gamma_l^{-1} = scale * |omega|^{-l/N_t} exp(-i pi l/N_t)
__device__ __forceinline__ c64 inv_gamma(int l, int Nt, double logabsw, double scale) {
  double sn, cs;
  sincospi((double)l / (double)Nt, &sn, &cs);
  const double g = exp(-(double)l * logabsw / (double)Nt) * scale;
  return {g * cs, -g * sn};
}

// 1/x for positive normal x: the hardware reciprocal estimate refined by two Newton
// steps (a few ulp), in place of an IEEE division
__device__ __forceinline__ double recip_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// 1/x and 1/y for positive x, y (their product within the FP64 range) from one reciprocal:
// r = 1/(x y) refined by two Newton steps, then 1/x = y r and 1/y = x r.
__device__ __forceinline__ void recip2_nr(double x, double y, double& rx, double& ry) {
  const double r = recip_nr(x * y);
  rx = y * r;
  ry = x * r;
}

// entries j = gid, gid + gstride, ... of a TabJob (Sections 3.1-3.3: omega from alpha,
// then the shifts d_j and the inverse scaling gamma_l^{-1})
__device__ __forceinline__ void tab_job_run(const TabJob& t, long long gid, long long gstride) {
  if (!t.out || gid >= t.Nt) return;
  const SolveScalars sc = scalars_from_alpha(t.alpha_dev ? *t.alpha_dev : t.alpha, t.variant, t.tau);
  const double croot = exp(sc.logabsw / (double)t.Nt);
  for (long long j = gid; j < t.Nt; j += gstride) {
    t.out[j] = shift_over_tau((int)j, t.Nt, croot, 1.0 / t.tau);
    t.out[t.Nt + j] = inv_gamma((int)j, t.Nt, sc.logabsw, (t.general ? 1.0 : sc.f0s) / (double)t.Nt);
    if (t.general) {  // gamma_t = |omega|^{t/N_t} exp(i pi t/N_t)
      double sn, cs;
      sincospi((double)j / (double)t.Nt, &sn, &cs);
      const double gm = exp((double)j * sc.logabsw / (double)t.Nt);
      t.out[2 * t.Nt + j] = {gm * cs, gm * sn};
    }
  }
}

// eigenvalue of -Lap_h for flattened mode index k (x_1 fastest)
__device__ __forceinline__ double mode_mu(long long k, int d, int m, const double* __restrict__ mu1d) {
  double mu = 0.0;
  for (int i = 0; i < d; ++i) {
    const long long q = k / m;
    mu += mu1d[k - q * m];
    k = q;
  }
  return mu;
}

// Modes of a rank-one time tile and their data.  PAIR: 2S consecutive x_1 of one padded
// row (each lane's two modes stored as one aligned 16-byte pair, a second mode past the row
// end landing in the padding); else 2S consecutive flattened modes.  The eigenvalue of a
// padded-row mode is mu(x_1) plus the eigenvalue of its row, taken with 32-bit index
// arithmetic (row < m^(d-1) < 2^31).
template <bool PAIR>
struct TimeTileR {
  long long ka, oa;
  int row, c1;  // PAIR: padded row and first x_1 of the lane's pair
  bool oka, okb;
  __device__ __forceinline__ TimeTileR(const TimeArgs& a, long long wg, int S, int s) {
    if constexpr (PAIR) {
      const int w = (int)wg;
      row = w / a.tiles_per_row;
      c1 = (w - row * a.tiles_per_row) * 2 * S + 2 * s;
      ka = (long long)row * a.m + c1;
      oa = (long long)row * a.pitch + c1;
      oka = c1 < a.m;
      okb = c1 + 1 < a.m;
    } else {
      row = c1 = 0;
      ka = wg * 2LL * S + 2 * s;
      oa = ka;
      oka = ka < a.nmodes;
      okb = ka + 1 < a.nmodes;
    }
  }
  // sine coefficients and eigenvalues of the lane's two modes (zero past the end)
  __device__ __forceinline__ void fetch(const TimeArgs& a, double& ga, double& gb, double& mua,
                                        double& mub) const {
    ga = oka ? a.ghat[ka] : 0.0;
    gb = okb ? a.ghat[ka + 1] : 0.0;
    if constexpr (PAIR) {
      double mrow = 0.0;
      int r = row;
      for (int i = 1; i < a.d; ++i) {
        const int q = r / a.m;
        mrow += a.mu1d[r - q * a.m];
        r = q;
      }
      mua = oka ? a.mu1d[c1] + mrow : 0.0;
      mub = okb ? a.mu1d[c1 + 1] + mrow : 0.0;
    } else {
      mua = oka ? mode_mu(ka, a.d, a.m, a.mu1d) : 0.0;
      mub = okb ? mode_mu(ka + 1, a.d, a.m, a.mu1d) : 0.0;
    }
  }
  // gamma_l^{-1} X_l to level l: real part -> first mode, imaginary part -> second
  __device__ __forceinline__ void store(const TimeArgs& a, int l, c64 yv) const {
    double* yl = a.y + (long long)l * a.ystride;
    if constexpr (PAIR) {
      if (oka) *reinterpret_cast<c64*>(yl + oa) = yv;
    } else {
      if (oka) yl[oa] = yv.re;
      if (okb) yl[oa + 1] = yv.im;
    }
  }
};

// column c of a columns pass holds data (see DstArgs)
__device__ __forceinline__ bool dst_col_ok(const DstArgs& a, long long c) {
  return c < a.inner && (a.colmod == 0 || (int)(c % a.colmod) < a.colvalid);
}

// ================================================================ k_dst ====
// Orthonormal DST-I along the `len` axis of [outer][len][inner]: X_i = sqrt(2/(m+1)) *
// sum_k x_k sin(pi i k/(m+1)).  Two real lines a, b are packed as a + i b into one
// length-2(m+1) DFT of their odd extensions v = [0, x, 0, -reverse(x)]:
// DFT(v_a + i v_b)_i = -2i S_a(i) + 2 S_b(i).
template <bool WIDE>
__device__ __forceinline__ void dst_body(const DstArgs& a, long long wg, c64* lds) {
  const int S = a.S, m = a.len, nc = a.fft.nc, N = a.fft.n;
  const int nl = 2 * S;
  c64* buf = lds;
  c64* side = lds + (size_t)S * nc;
  const bool contig = (a.inner == 1);
  long long o = 0, i0 = 0;
  if (contig) {
    i0 = wg * nl;  // first line (outer index)
  } else {
    o = wg / a.tiles_per_outer;
    i0 = (wg - o * a.tiles_per_outer) * nl;
  }
  for (int e = threadIdx.x; e < S * nc; e += blockDim.x) buf[e] = {0.0, 0.0};
  const c64* tw = stage_twiddles(a.fft, a.tw_lds, side + 2 * S);
  __syncthreads();
  double* bp = reinterpret_cast<double*>(buf);
  const int tot = nl * m, T = blockDim.x;
  // element e: contiguous lines (q, k) = (e / m, e mod m); columns (k, q) = (e / nl, e mod nl)
  LaneWalk w(contig ? m : nl);
  for (int e0 = threadIdx.x; e0 < tot; e0 += kBatch * T) {
    double xv[kBatch];
    int qv[kBatch], p1v[kBatch], p2v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      // indices past the data are clamped to the last valid element, so every load of
      // the batch is unconditional; the value is then replaced by 0
      const int q = contig ? w.j : w.s, k = min(contig ? w.s : w.j, m - 1);
      const bool live = e0 + u * T < tot;
      double x;
      if (contig) {
        const long long line = i0 + q;
        x = a.in[min(line, a.outer - 1) * a.in_pitch + k];
        if (!(live && line < a.outer)) x = 0.0;
      } else {
        const long long i = i0 + q;
        x = a.in[o * a.ostride + k * a.kstride + min(i, a.inner - 1)];
        if (!(live && dst_col_ok(a, i))) x = 0.0;
      }
      qv[u] = q;
      p1v[u] = fft_in_pos(a.fft, k + 1);
      p2v[u] = fft_in_pos(a.fft, N - 1 - k);
      xv[u] = x;
      w.next();
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      if (e0 + u * T < tot) {
        const int s = qv[u] >> 1, comp = qv[u] & 1;
        bp[2 * ((size_t)p1v[u] * S + s) + comp] = xv[u];
        bp[2 * ((size_t)p2v[u] * S + s) + comp] = -xv[u];
      }
    }
  }
  __syncthreads();
  if (a.fft.kind == kBluestein) fft_bluestein_prep(buf, S, a.fft);
  fft_run<WIDE>(buf, S, a.fft, side, tw);
  LaneWalk wo(contig ? m : nl);
  for (int e0 = threadIdx.x; e0 < tot; e0 += kBatch * T) {
    FftOutAt at[kBatch];
    int qv[kBatch], kv[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      qv[u] = contig ? wo.j : wo.s;
      kv[u] = contig ? wo.s : wo.j;
      at[u] = fft_out_at(a.fft, min(kv[u], m - 1) + 1);
      wo.next();
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      if (e0 + u * T >= tot) continue;
      const int q = qv[u], k = kv[u];
      long long dst;
      bool ok;
      if (contig) {
        const long long line = i0 + q;
        ok = line < a.outer;
        dst = line * a.out_pitch + k;
      } else {
        const long long i = i0 + q;
        ok = dst_col_ok(a, i);
        dst = o * a.ostride + k * a.kstride + i;
      }
      const int s = q >> 1, comp = q & 1;
      const c64 V = fft_out(buf, S, a.fft, s, at[u], side);
      const double val = comp == 0 ? -V.im : V.re;
      if (ok) a.out[dst] = val * a.scale;
    }
  }
}


// =============================================================== k_time ====
template <bool WIDE>
__device__ __forceinline__ void time_body(const TimeArgs& a, long long wg, c64* lds) {
  const int S = a.S, Nt = a.Nt, nc = a.fft.nc;
  c64* buf = lds;
  c64* side = buf + (size_t)S * nc;
  c64* dt = side + 2 * S;
  c64* gi = dt + Nt;
  double* mus = reinterpret_cast<double*>(gi + a.lev_count);
  double* gh = mus + 2 * S;

  const SolveScalars sc = solve_scalars(a.sc, a.alpha_dev, a.variant, a.tau);
  const double croot = exp(sc.logabsw / (double)Nt);
  const double inv_tau = 1.0 / a.tau;
  const double gscale = sc.f0s / (double)Nt;
  for (int j = threadIdx.x; j < Nt; j += blockDim.x) dt[j] = shift_over_tau(j, Nt, croot, inv_tau);
  for (int li = threadIdx.x; li < a.lev_count; li += blockDim.x)
    gi[li] = inv_gamma(a.lev_first + li, Nt, sc.logabsw, gscale);
  const long long k0 = wg * 2LL * S;
  for (int q = threadIdx.x; q < 2 * S; q += blockDim.x) {
    const long long k = k0 + q;
    if (k < a.nmodes) {
      mus[q] = mode_mu(k, a.d, a.m, a.mu1d);
      gh[q] = a.ghat[k];
    } else {
      mus[q] = 0.0;
      gh[q] = 0.0;
    }
  }
  const c64* tw = stage_twiddles(a.fft, a.tw_lds, reinterpret_cast<c64*>(gh + 2 * S));
  __syncthreads();
  // Steps (a)+(b): u_j = g_a/(d_j/tau + mu_a) + i g_b/(d_j/tau + mu_b); for a Bluestein
  // length the chirp weight conj(w_j) is applied here and the core beyond N_t is zeroed
  // (the engine's separate pre-processing pass is not needed)
  const int T = blockDim.x;
  LaneWalk w(S);
  auto place = [&](auto blue_tag) {
    constexpr bool BLUE = decltype(blue_tag)::value;
    for (int e0 = threadIdx.x; e0 < S * Nt; e0 += kBatch * T) {
      int pv[kBatch], jv[kBatch], sv[kBatch];
      c64 cw[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        jv[u] = w.j;
        sv[u] = w.s;
        pv[u] = fft_in_pos(a.fft, min(w.j, Nt - 1));
        if constexpr (BLUE) cw[u] = cconj(a.fft.chirp[min(w.j, Nt - 1)]);
        w.next();
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        if (e0 + u * T >= S * Nt) continue;
        const int j = jv[u], s = sv[u];
        const c64 z = dt[j];
        const double xa = z.re + mus[2 * s], xb = z.re + mus[2 * s + 1];
        const double ia = gh[2 * s] / (xa * xa + z.im * z.im);
        const double ib = gh[2 * s + 1] / (xb * xb + z.im * z.im);
        // A = ia (xa - i z.im), B = ib (xb - i z.im); u = A + i B
        c64 uu = {ia * xa + ib * z.im, ib * xb - ia * z.im};
        if constexpr (BLUE) uu = cmul(uu, cw[u]);
        if (pv[u] < 0) side[s] = uu;
        else buf[(size_t)pv[u] * S + s] = uu;
      }
    }
    if constexpr (BLUE)
      for (int e = threadIdx.x; e < S * (nc - Nt); e += T) buf[(size_t)S * Nt + e] = {0.0, 0.0};
  };
  if (a.fft.kind == kBluestein) place(std::true_type{});
  else place(std::false_type{});
  __syncthreads();
  fft_run<WIDE>(buf, S, a.fft, side, tw);
  // Step (c): gamma_l^{-1}/N_t * X_l; real part -> mode a, imaginary part -> mode b
  const int tot = S * a.lev_count;
  LaneWalk wo(S);
  for (int e0 = threadIdx.x; e0 < tot; e0 += kBatch * T) {
    FftOutAt at[kBatch];
    int lv[kBatch], sv[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      lv[u] = wo.j;
      sv[u] = wo.s;
      at[u] = fft_out_at(a.fft, a.lev_first + min(wo.j, a.lev_count - 1));
      wo.next();
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      if (e0 + u * T >= tot) continue;
      const int li = lv[u], s = sv[u];
      const c64 v = cmul(gi[li], fft_out(buf, S, a.fft, s, at[u], side));
      const long long ka = k0 + 2 * s;
      double* yl = a.y + (long long)(a.lev_dst0 + li) * a.ystride;
      if (ka < a.nmodes) yl[ka] = v.re;
      if (ka + 1 < a.nmodes) yl[ka + 1] = v.im;
    }
  }
}


// ======================================================== k_time_general ====
// Steps (a)-(c) for a general right-hand side (every level), per pair of sine modes:
//   z_j = sum_t theta^{jt} gamma_t f_t          (Step (a), the factor 1/sqrt(N_t) moved to (c))
//   w_j = z_j / (d_j/tau + mu_k)                (Step (b))
//   y_l = gamma_l^{-1}/N_t sum_j theta^{-jl} w_j  (Step (c)), real.
// Two real modes a, b share one transform.  Step (a) of a real sequence satisfies
// z(N_t-1-j) = conj z(j) (gamma_t theta^{jt} is |omega|^{t/N_t} exp(i pi t(2j+1)/N_t)),
// which separates z_a and z_b before their different shifts; the results of Step (c)
// are real, so w = w_a + i w_b packs them again.  The sums over theta^{+jt} run on the
// forward engine through conj(sum_t conj(u_t) theta^{-jt}).  Tables (global, per
// solve): d_j/tau, gamma_l^{-1}/N_t, gamma_t.  In place: fgen may equal y.
template <bool WIDE>
__device__ __forceinline__ void time_general_body(const TimeArgs& a, long long wg, c64* lds) {
  const int S = a.S, Nt = a.Nt, nc = a.fft.nc;
  c64* buf = lds;                               // S * nc, engine layout
  c64* zb = buf + (size_t)S * nc;               // S * N_t, natural order [j][s]
  c64* side = zb + (size_t)S * Nt;              // 2 S
  double* mus = reinterpret_cast<double*>(side + 2 * S);  // 2 S
  const c64* dt = a.tabs;
  const c64* gi = a.tabs + Nt;
  const c64* gam = a.tabs + 2 * Nt;
  const long long k0 = wg * 2LL * S;
  for (int q = threadIdx.x; q < 2 * S; q += blockDim.x) {
    const long long k = k0 + q;
    mus[q] = k < a.nmodes ? mode_mu(k, a.d, a.m, a.mu1d) : 0.0;
  }
  // Step (a) input: conj(gamma_t (f_a(t) + i f_b(t))), placed for the engine
  for (int e = threadIdx.x; e < S * Nt; e += blockDim.x) {
    const int t = e / S, s = e - t * S;
    const long long ka = k0 + 2 * s;
    const double* ft = a.fgen + (long long)t * a.ystride;
    const c64 f = {ka < a.nmodes ? ft[ka] : 0.0, ka + 1 < a.nmodes ? ft[ka + 1] : 0.0};
    const c64 u = cconj(cmul(gam[t], f));
    const int pos = fft_in_pos(a.fft, t);
    if (pos < 0) side[s] = u;
    else buf[(size_t)pos * S + s] = u;
  }
  __syncthreads();
  if (a.fft.kind == kBluestein) fft_bluestein_prep(buf, S, a.fft);
  fft_run<WIDE>(buf, S, a.fft, side);
  for (int e = threadIdx.x; e < S * Nt; e += blockDim.x) {
    const int j = e / S, s = e - j * S;
    zb[(size_t)j * S + s] = cconj(fft_out(buf, S, a.fft, s, j, side));
  }
  __syncthreads();
  // separate, Step (b), pack, place for the second transform
  for (int e = threadIdx.x; e < S * Nt; e += blockDim.x) {
    const int j = e / S, s = e - j * S;
    const c64 zj = zb[(size_t)j * S + s];
    const c64 zr = cconj(zb[(size_t)(Nt - 1 - j) * S + s]);
    const c64 za = {0.5 * (zj.re + zr.re), 0.5 * (zj.im + zr.im)};  // (z + conj z')/2
    const c64 zbm = {0.5 * (zj.im - zr.im), -0.5 * (zj.re - zr.re)};  // (z - conj z')/(2i)
    const c64 z = dt[j];
    const double xa = z.re + mus[2 * s], xb = z.re + mus[2 * s + 1];
    double qa, qb;
    recip2_nr(xa * xa + z.im * z.im, xb * xb + z.im * z.im, qa, qb);
    // w_a = za / (xa + i z.im), w_b = zbm / (xb + i z.im)
    const c64 wa = {(za.re * xa + za.im * z.im) * qa, (za.im * xa - za.re * z.im) * qa};
    const c64 wb = {(zbm.re * xb + zbm.im * z.im) * qb, (zbm.im * xb - zbm.re * z.im) * qb};
    const c64 w = {wa.re - wb.im, wa.im + wb.re};  // w_a + i w_b
    const int pos = fft_in_pos(a.fft, j);
    if (pos < 0) side[s] = w;
    else buf[(size_t)pos * S + s] = w;
  }
  __syncthreads();
  if (a.fft.kind == kBluestein) fft_bluestein_prep(buf, S, a.fft);
  fft_run<WIDE>(buf, S, a.fft, side);
  // Step (c): gamma_l^{-1}/N_t X_l; real part -> mode a, imaginary part -> mode b
  for (int e = threadIdx.x; e < S * Nt; e += blockDim.x) {
    const int l = e / S, s = e - l * S;
    const c64 v = cmul(gi[l], fft_out(buf, S, a.fft, s, l, side));
    const long long ka = k0 + 2 * s;
    double* yl = a.y + (long long)l * a.ystride;
    if (ka < a.nmodes) yl[ka] = v.re;
    if (ka + 1 < a.nmodes) yl[ka + 1] = v.im;
  }
}

// ============================================================= k_tri1d =====
// Step (b) in 1D for each shift j: (d_j/tau I + A) s = f0 with A = -Lap_h (the
// three-point Dirichlet stencil, 2/h^2 on the diagonal, -1/h^2 beside it) or a
// tridiagonal operator given by the caller.  Row i reads l_i s_{i-1} + (d_j/tau + b_i) s_i
// + u_i s_{i+1} = f0_i (l_0 = u_{m-1} = 0).
//
// Partition method with parallel cyclic reduction: the P lanes of a system each take
// a chunk [lo, hi) of 2..8 consecutive rows (P = ceil(m/8), rows spread evenly).
// Eliminating a chunk's interior rows, with its first and last unknowns F_p = s_lo and
// L_p = s_{hi-1} kept as parameters, gives per chunk
//   interior:  s_i + c_i s_{i+1} + a_i F_p = d_i           (downward sweep)
//   first row: l_lo L_{p-1} + (b_lo + u_lo A) F_p + u_lo C L_p = f_lo - u_lo D
//   last row:  -l_{hi-1} a' F_p + (b_{hi-1} - l_{hi-1} c') L_p + u_{hi-1} F_{p+1} = f_{hi-1} - l_{hi-1} d'
// with (c', a', d') those of the last interior row and s_{lo+1} = D + C L_p + A F_p from
// the upward recurrence.  In the order F_0, L_0, F_1, L_1, ... the 2P boundary equations
// are tridiagonal; PCR solves them in LDS in ceil(log2 2P) steps, then each lane
// recovers its interior rows.  No pivoting: the shifted operator must be diagonally
// dominant enough for elimination without it (diffusion operators are).
__device__ __forceinline__ c64 cdiv_nr(c64 a, c64 b) {
  const double q = recip_nr(b.re * b.re + b.im * b.im);
  return {(a.re * b.re + a.im * b.im) * q, (a.im * b.re - a.re * b.im) * q};
}

struct TriEq {
  c64 lo, di, up, rh;
};

__device__ __forceinline__ void tri1d_body(const ThomasArgs& a, long long wg, c64* lds) {
  const int Nt = a.Nt, m = a.m, P = a.P;
  const int t = threadIdx.x, sl = t / P, p = t - sl * P;
  tab_job_run(a.tab, wg * blockDim.x + t, (long long)gridDim.x * blockDim.x);
  const long long jl = wg * a.S + sl;
  const bool live = sl < a.S && jl < Nt;
  const int j = live ? (int)jl : 0;
  const SolveScalars sc = solve_scalars(a.sc, a.alpha_dev, a.variant, a.tau);
  const double croot = exp(sc.logabsw / (double)Nt);
  const c64 z = shift_over_tau(j, Nt, croot, 1.0 / a.tau);
  const double ih2 = 1.0 / (a.h * a.h);
  const bool op = a.op_di != nullptr;
  auto bdiag = [&](int i) -> c64 { return {z.re + (op ? a.op_di[i] : 2.0 * ih2), z.im}; };
  auto lower = [&](int i) -> double { return i > 0 ? (op ? a.op_lo[i - 1] : -ih2) : 0.0; };
  auto upper = [&](int i) -> double { return i + 1 < m ? (op ? a.op_up[i] : -ih2) : 0.0; };
  auto rhs = [&](int i) -> double { return sc.f0s * a.g[i]; };
  c64* out = a.s2 + jl * (long long)m;
  if (m == 1) {  // one row, one lane: s = f0 / (d_j/tau + b)
    if (live) out[0] = cdiv_nr({rhs(0), 0.0}, bdiag(0));
    return;
  }
  const int lo = (int)((long long)p * m / P), hi = (int)((long long)(p + 1) * m / P);
  const int ni = hi - lo - 2;  // interior rows, 0..6
  // downward sweep over the interior, from the virtual row s_lo - F_p = 0
  c64 cr[6], ar[6], dr[6];
  c64 cpv = {0.0, 0.0}, apv = {-1.0, 0.0}, dpv = {0.0, 0.0};
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    if (q < ni) {
      const int i = lo + 1 + q;
      const double l = lower(i);
      const c64 den = {bdiag(i).re - l * cpv.re, bdiag(i).im - l * cpv.im};
      const c64 inv = cdiv_nr({1.0, 0.0}, den);
      cpv = cscale(inv, upper(i));
      apv = cscale(cmul(apv, inv), -l);
      dpv = cmul({rhs(i) - l * dpv.re, -l * dpv.im}, inv);
      cr[q] = cpv;
      ar[q] = apv;
      dr[q] = dpv;
    }
  }
  TriEq e1, e2;
  {
    const int i = hi - 1;
    const double l = lower(i);
    e2.lo = cscale(apv, -l);
    e2.di = {bdiag(i).re - l * cpv.re, bdiag(i).im - l * cpv.im};
    e2.up = {upper(i), 0.0};
    e2.rh = {rhs(i) - l * dpv.re, -l * dpv.im};
  }
  {
    // upward recurrence: s_i = D + C L_p + A F_p, from the virtual row s_{hi-1} = L_p
    c64 D = {0.0, 0.0}, C = {1.0, 0.0}, A = {0.0, 0.0};
#pragma unroll
    for (int q = 5; q >= 0; --q) {
      if (q < ni) {
        D = csub(dr[q], cmul(cr[q], D));
        C = cscale(cmul(cr[q], C), -1.0);
        A = csub(cscale(ar[q], -1.0), cmul(cr[q], A));
      }
    }
    const double u = upper(lo);
    e1.lo = {lower(lo), 0.0};
    e1.di = cadd(bdiag(lo), cscale(A, u));
    e1.up = cscale(C, u);
    e1.rh = {rhs(lo) - u * D.re, -u * D.im};
  }
  // PCR over the 2P boundary equations of each system (identity outside the range).
  // LDS: four coefficient arrays per system; equation q sits in slot q/2 (q even) or
  // P + q/2 (q odd), so the lanes of a step always read consecutive 16-byte slots.
  const int n2 = 2 * P;
  c64* elo = lds + (size_t)sl * 4 * n2;
  c64* edi = elo + n2;
  c64* eup = edi + n2;
  c64* erh = eup + n2;
  auto slot = [&](int q) { return (q & 1) ? P + (q >> 1) : (q >> 1); };
  auto put = [&](int q, const TriEq& e) {
    const int k = slot(q);
    elo[k] = e.lo;
    edi[k] = e.di;
    eup[k] = e.up;
    erh[k] = e.rh;
  };
  auto get = [&](int q) -> TriEq {
    const int k = slot(q);
    return {elo[k], edi[k], eup[k], erh[k]};
  };
  const TriEq id = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
  const bool own = sl < a.S;
  if (own) {
    put(2 * p, e1);
    put(2 * p + 1, e2);
  }
  __syncthreads();
  for (int st = 1; st < n2; st *= 2) {
    TriEq nw[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = 2 * p + h;
      const TriEq c = h ? e2 : e1;
      const TriEq L = (own && q - st >= 0) ? get(q - st) : id;
      const TriEq R = (own && q + st < n2) ? get(q + st) : id;
      const c64 k1 = cdiv_nr(c.lo, L.di), k2 = cdiv_nr(c.up, R.di);
      nw[h].lo = cscale(cmul(L.lo, k1), -1.0);
      nw[h].up = cscale(cmul(R.up, k2), -1.0);
      nw[h].di = csub(csub(c.di, cmul(L.up, k1)), cmul(R.lo, k2));
      nw[h].rh = csub(csub(c.rh, cmul(L.rh, k1)), cmul(R.rh, k2));
    }
    e1 = nw[0];
    e2 = nw[1];
    __syncthreads();
    if (own) {
      put(2 * p, e1);
      put(2 * p + 1, e2);
    }
    __syncthreads();
  }
  if (!live) return;
  const c64 F = cdiv_nr(e1.rh, e1.di), L = cdiv_nr(e2.rh, e2.di);
  out[lo] = F;
  out[hi - 1] = L;
  c64 x = L;
#pragma unroll
  for (int q = 5; q >= 0; --q) {
    if (q < ni) {
      x = csub(csub(dr[q], cmul(cr[q], x)), cmul(ar[q], F));
      out[lo + 1 + q] = x;
    }
  }
}


// ============================================================= k_time1d ====
// Step (c) in 1D: per grid point, X_l = sum_j S2(x, j) exp(-2 pi i jl/N_t); y^l = Re(gamma_l^{-1} X_l)/N_t.
template <bool WIDE>
__device__ __forceinline__ void time1d_body(const Time1dArgs& a, long long wg, c64* lds) {
  const int S = a.S, Nt = a.Nt, nc = a.fft.nc, m = a.m;
  c64* buf = lds;
  c64* side = buf + (size_t)S * nc;
  // gamma_l^{-1}/N_t of the written levels: from the per-solve table, else into LDS
  const c64* gi = a.gitab ? a.gitab + Nt + a.lev_first : side + 2 * S;
  if (!a.gitab) {
    const double gscale = 1.0 / (double)Nt;
    const SolveScalars sc = solve_scalars(a.sc, a.alpha_dev, a.variant, a.tau);
    c64* gl = side + 2 * S;
    for (int li = threadIdx.x; li < a.lev_count; li += blockDim.x)
      gl[li] = inv_gamma(a.lev_first + li, Nt, sc.logabsw, gscale);
  }
  const long long x0 = wg * 2LL * S;
  for (int e = threadIdx.x; e < S * Nt; e += blockDim.x) {
    const int j = e / S, s = e - j * S;  // consecutive lanes: consecutive points of one shift
    const long long xa = x0 + 2 * s, xb = xa + 1;
    const c64* row = a.s2 + (long long)j * m;
    const c64 A = xa < m ? row[xa] : c64{0.0, 0.0};
    const c64 B = xb < m ? row[xb] : c64{0.0, 0.0};
    const c64 u = {A.re - B.im, A.im + B.re};
    const int pos = fft_in_pos(a.fft, j);
    if (pos < 0) side[s] = u;
    else buf[(size_t)pos * S + s] = u;
  }
  __syncthreads();
  if (a.fft.kind == kBluestein) fft_bluestein_prep(buf, S, a.fft);
  fft_run<WIDE>(buf, S, a.fft, side);
  const int tot = S * a.lev_count;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int li = e / S, s = e - li * S;
    const c64 X = fft_out(buf, S, a.fft, s, a.lev_first + li, side);
    const c64 v = cmul(gi[li], X);
    const long long xa = x0 + 2 * s;
    double* yl = a.y + (long long)li * a.ystride;
    if (xa < m) yl[xa] = v.re;
    if (xa + 1 < m) yl[xa + 1] = v.im;
  }
}


}  // namespace qbvm
