// Spectral time kernel for N_t = A * B with gcd(A, B) = 1, B an odd prime (Good-Thomas).
//
// With input index n = (B a + A b) mod N_t and output index
// k = (B c1 k1 + A c2 k2) mod N_t, c1 = B^{-1} mod A, c2 = A^{-1} mod B, the DFT of
// length N_t is exactly the two-dimensional DFT over (a, b) -> (k1, k2) with no
// twiddle factors.  Lane (s, a) of a workgroup computes the length-B DFT of row a
// of signal s in registers (symmetric-pair form, outputs streamed to LDS), then,
// after one exchange, lengths-A DFTs over a for its share of k2.  Signal s packs
// two sine modes as in the power-of-two kernel (real part -> first mode).
#pragma once

#include "qbvm_bodies.hpp"

namespace qbvm {

constexpr int gt_inv_mod(int x, int m) {
  for (int i = 1; i < m; ++i)
    if ((x * i) % m == 1) return i;
  return 0;
}

// Direct DFT of odd prime length B on registers v (destroyed), outputs to out[k * ostride].
template <int B>
__device__ __forceinline__ void gt_dft_odd_store(c64 (&v)[B], c64* out, int ostride) {
  constexpr int H = (B - 1) / 2;
  constexpr int base = B * (B - 1) / 2;
  const c64 x0 = v[0];
  c64 s0 = x0;
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    const c64 p = v[j], q = v[B - j];
    v[j] = cadd(p, q);      // a_j
    v[B - j] = csub(p, q);  // b_j
    s0 = cadd(s0, v[j]);
  }
  out[0] = s0;
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    c64 Ak = x0, Bk = {0.0, 0.0};
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const c64 w = c_root[base + (j * k) % B];
      Ak.re += v[j].re * w.re;
      Ak.im += v[j].im * w.re;
      Bk.re -= v[B - j].re * w.im;
      Bk.im -= v[B - j].im * w.im;
    }
    out[k * ostride] = {Ak.re + Bk.im, Ak.im - Bk.re};
    out[(B - k) * ostride] = {Ak.re - Bk.im, Ak.im + Bk.re};
  }
}

template <int A, int B, int S>
constexpr size_t gt_lds_bytes(int Nt) {
  return sizeof(c64) * ((size_t)A * B * S + 2 * (size_t)Nt);
}

template <int A, int B, int S>
__device__ __forceinline__ void time_gt_body(const TimeArgs& a, long long wg, c64* lds) {
  constexpr int N = A * B;
  constexpr int c1 = gt_inv_mod(B % A, A);
  constexpr int c2 = gt_inv_mod(A % B, B);
  static_assert(A >= 2 && c1 > 0, "A and B must be coprime");
  static_assert(c2 > 0, "A and B must be coprime");
  constexpr int T = A * S;
  c64* Y = lds;            // [k2][a][s]
  c64* dt = lds + (size_t)N * S;
  c64* gi = dt + N;
  const int t = threadIdx.x, s = t % S, ra = t / S;

  SolveScalars sc = a.sc;
  if (a.alpha_dev) sc = scalars_from_alpha(*a.alpha_dev, a.variant, a.tau);
  if (a.tabs) {
    for (int j = t; j < N; j += T) {
      dt[j] = a.tabs[j];
      gi[j] = a.tabs[N + j];
    }
  } else {
    const double croot = exp(sc.logabsw / (double)N);
    for (int j = t; j < N; j += T) {
      dt[j] = shift_over_tau(j, N, croot, 1.0 / a.tau);
      gi[j] = inv_gamma(j, N, sc.logabsw, sc.f0s / (double)N);
    }
  }
  __syncthreads();

  long long ka, oa;
  bool oka, okb;
  if (a.pitch > 0) {
    const long long row = wg / a.tiles_per_row;
    const int cc = (int)(wg - row * a.tiles_per_row) * 2 * S + 2 * s;
    ka = row * a.m + cc;
    oa = row * a.pitch + cc;
    oka = cc < a.m;
    okb = cc + 1 < a.m;
  } else {
    ka = wg * 2LL * S + 2 * s;
    oa = ka;
    oka = ka < a.nmodes;
    okb = ka + 1 < a.nmodes;
  }
  const double ga = oka ? a.ghat[ka] : 0.0, gb = okb ? a.ghat[ka + 1] : 0.0;
  const double mua = oka ? mode_mu(ka, a.d, a.m, a.mu1d) : 0.0;
  const double mub = okb ? mode_mu(ka + 1, a.d, a.m, a.mu1d) : 0.0;

  // Steps (a)+(b) on row ra: x[ra, b] = u_{(B ra + A b) mod N}
  c64 v[B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    int n = B * ra + A * b;
    n = n >= N ? n - N : n;
    n = n >= N ? n - N : n;
    const c64 z = dt[n];
    const double xa = z.re + mua, xb = z.re + mub;
    const double ia = ga * recip_nr(xa * xa + z.im * z.im);
    const double ib = gb * recip_nr(xb * xb + z.im * z.im);
    v[b] = {ia * xa + ib * z.im, ib * xb - ia * z.im};
  }
  // length-B DFT over b -> Y[k2][ra][s]
  gt_dft_odd_store<B>(v, Y + (size_t)ra * S + s, A * S);
  __syncthreads();
  // length-A DFTs over a for k2 = ra, ra + A, ...; Step (c) scaling and store
  for (int k2 = ra; k2 < B; k2 += A) {
    c64 w[A];
#pragma unroll
    for (int q = 0; q < A; ++q) w[q] = Y[((size_t)k2 * A + q) * S + s];
    Bfly<A>::run(w);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      const int l = (B * c1 * k1 + A * c2 * k2) % N;
      const c64 yv = cmul(gi[l], w[k1]);
      double* yl = a.y + (long long)l * a.ystride;
      if (a.pitch > 0) {  // aligned pair; a second mode past the row end lands in the padding
        if (oka) *reinterpret_cast<c64*>(yl + oa) = yv;
      } else {
        if (oka) yl[oa] = yv.re;
        if (okb) yl[oa + 1] = yv.im;
      }
    }
  }
}

}  // namespace qbvm
