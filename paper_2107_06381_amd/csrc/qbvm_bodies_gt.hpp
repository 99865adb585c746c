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

// cos and sin of 2 pi r / B as compile-time constants (Taylor series after reduction
// to [0, pi/2]), so the DFT below takes its roots as scalar immediates.
constexpr double gt_series(double x, bool sine) {
  double term = sine ? x : 1.0, sum = term;
  for (int n = sine ? 1 : 0; n < 40; n += 2) {
    term *= -x * x / (double)((n + 1) * (n + 2));
    sum += term;
  }
  return sum;
}

template <int B>
struct GtRoots {
  double c[B], s[B];
  constexpr GtRoots() : c(), s() {
    constexpr double pi = 3.141592653589793238462643383279502884;
    for (int r = 0; r < B; ++r) {
      const int q = r <= B / 2 ? r : B - r;  // angle 2 pi q / B in [0, pi]; sin flips for r > B/2
      double th = 2.0 * pi * (double)q / (double)B;
      double sg_c = 1.0;
      if (th > pi / 2) {
        th = pi - th;
        sg_c = -1.0;
      }
      c[r] = sg_c * gt_series(th, false);
      s[r] = (r <= B / 2 ? 1.0 : -1.0) * gt_series(th, true);
    }
  }
};

// ---- Rader's algorithm for a prime row length B with B - 1 = 42 = 6 x 7 (the 43-point
// rows of N_t = 129): X_0 = sum_n x_n and, with g a primitive root mod B,
// X_{g^-p} = x_0 + sum_q x_{g^q} w^{g^(q-p)}, w = e^{-2 pi i/B}: a cyclic convolution of
// length 42 of a_q = x_{g^q} with b_m = w^{g^-m}, carried out as
// conj(DFT42(conj(DFT42(a) . DFT42(b)/42))).  DFT42 is the prime-factor (Good-Thomas)
// algorithm over 6 x 7 (DFT6 itself over 2 x 3) with every index and root a compile-time
// constant, so the whole row transform stays in registers.
constexpr int gt_prim_root(int P) {
  for (int g = 2; g < P; ++g) {
    int x = 1, order = 0;
    do {
      x = x * g % P;
      ++order;
    } while (x != 1);
    if (order == P - 1) return g;
  }
  return 0;
}

// Odd-length DFT on registers x[0..R) in natural order (symmetric form, compile-time roots).
template <int R>
__device__ __forceinline__ void gt_odd_dft(c64* x) {
  constexpr GtRoots<R> W{};
  constexpr int H = (R - 1) / 2;
  c64 a[H], b[H];
  const c64 x0 = x[0];
  c64 s = x0;
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    a[j - 1] = cadd(x[j], x[R - j]);
    b[j - 1] = csub(x[j], x[R - j]);
    s = cadd(s, a[j - 1]);
  }
  x[0] = s;
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    c64 A = x0, Bk = {0.0, 0.0};
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const int r = (j * k) % R;
      A.re += a[j - 1].re * W.c[r];
      A.im += a[j - 1].im * W.c[r];
      Bk.re += b[j - 1].re * W.s[r];
      Bk.im += b[j - 1].im * W.s[r];
    }
    x[k] = {A.re + Bk.im, A.im - Bk.re};      // A - i B
    x[R - k] = {A.re - Bk.im, A.im + Bk.re};  // A + i B
  }
}

// DFT6 = 2 x 3 prime-factor: n = (3 n1 + 2 n2) mod 6, k = (3 k1 + 4 k2) mod 6.
__device__ __forceinline__ void gt_dft6(c64* x) {
  c64 t[2][3];
#pragma unroll
  for (int n1 = 0; n1 < 2; ++n1) {
#pragma unroll
    for (int n2 = 0; n2 < 3; ++n2) t[n1][n2] = x[(3 * n1 + 2 * n2) % 6];
    gt_odd_dft<3>(t[n1]);
  }
#pragma unroll
  for (int k2 = 0; k2 < 3; ++k2) {
    x[(4 * k2) % 6] = cadd(t[0][k2], t[1][k2]);
    x[(3 + 4 * k2) % 6] = csub(t[0][k2], t[1][k2]);
  }
}

// DFT42 = 6 x 7 prime-factor: n = (7 n1 + 6 n2) mod 42, k = (7 k1 + 36 k2) mod 42.
__device__ __forceinline__ void gt_dft42(c64* x) {
  c64 t[6][7];
#pragma unroll
  for (int n1 = 0; n1 < 6; ++n1) {
#pragma unroll
    for (int n2 = 0; n2 < 7; ++n2) t[n1][n2] = x[(7 * n1 + 6 * n2) % 42];
    gt_odd_dft<7>(t[n1]);
  }
#pragma unroll
  for (int k2 = 0; k2 < 7; ++k2) {
    c64 u[6];
#pragma unroll
    for (int n1 = 0; n1 < 6; ++n1) u[n1] = t[n1][k2];
    gt_dft6(u);
#pragma unroll
    for (int k1 = 0; k1 < 6; ++k1) x[(7 * k1 + 36 * k2) % 42] = u[k1];
  }
}

// Rader tables of a prime B (B - 1 = 42): g^q, g^-p and the kernel spectrum DFT42(b)/42.
template <int B>
struct GtRader {
  int gq[B - 1], gmp[B - 1];
  double bre[B - 1], bim[B - 1];
  constexpr GtRader() : gq(), gmp(), bre(), bim() {
    static_assert(B - 1 == 42, "Rader rows are built on the 42-point prime-factor DFT");
    constexpr int g = gt_prim_root(B);
    int ginv = 1;
    for (int i = 0; i < B - 2; ++i) ginv = ginv * g % B;  // g^(B-2) = g^-1
    int x = 1, y = 1;
    for (int q = 0; q < B - 1; ++q) {
      gq[q] = x;
      gmp[q] = y;
      x = x * g % B;
      y = y * ginv % B;
    }
    const GtRoots<B> w{};
    const GtRoots<B - 1> f{};
    for (int k = 0; k < B - 1; ++k) {
      double re = 0.0, im = 0.0;
      for (int m = 0; m < B - 1; ++m) {
        const double br = w.c[gmp[m]], bi = -w.s[gmp[m]];  // b_m = w^{g^-m}
        const int r = (m * k) % (B - 1);
        re += br * f.c[r] + bi * f.s[r];  // b_m e^{-2 pi i mk/42}
        im += bi * f.c[r] - br * f.s[r];
      }
      bre[k] = re / (double)(B - 1);
      bim[k] = im / (double)(B - 1);
    }
  }
};

// In-place DFT of a prime-length row on registers (natural order in and out).
template <int B>
__device__ __forceinline__ void gt_rader_dft(c64 (&v)[B]) {
  constexpr GtRader<B> K{};
  const c64 x0 = v[0];
  c64 a[B - 1];
#pragma unroll
  for (int q = 0; q < B - 1; ++q) a[q] = v[K.gq[q]];
  gt_dft42(a);
  const c64 X0 = cadd(x0, a[0]);
#pragma unroll
  for (int q = 0; q < B - 1; ++q) a[q] = cconj(cmul(a[q], c64{K.bre[q], K.bim[q]}));
  gt_dft42(a);
  v[0] = X0;
#pragma unroll
  for (int p = 0; p < B - 1; ++p) v[K.gmp[p]] = cadd(x0, cconj(a[p]));
}

template <int B>
constexpr int gt_pairs() { return (B - 1) / 2; }

// Output slots of chunk ch (KC symmetric pairs per chunk; chunk 0 also holds k = 0).
template <int B, int KC>
constexpr int gt_chunk_first(int ch) { return 1 + ch * KC; }
template <int B, int KC>
constexpr int gt_chunk_last(int ch) {
  return gt_chunk_first<B, KC>(ch) + KC - 1 < gt_pairs<B>() ? gt_chunk_first<B, KC>(ch) + KC - 1 : gt_pairs<B>();
}
template <int B, int KC>
constexpr int gt_chunk_slots(int ch) {
  return (ch == 0 ? 1 : 0) + 2 * (gt_chunk_last<B, KC>(ch) - gt_chunk_first<B, KC>(ch) + 1);
}

// PAIR: levels in padded rows (pitch > 0), each lane's two modes stored as one
// aligned 16-byte pair (a second mode past the row end lands in the padding).
// One tile per workgroup (the row DFT keeps a lane's registers nearly full, and a tile
// loop with the next tile's coefficients in flight spilled); the tile's coefficients are
// requested before the tables are staged, so their latency overlaps that prologue.
// RADER: the length-B row DFTs by Rader's algorithm (gt_rader_dft) instead of the direct
// symmetric form.
template <int A, int B, int S, int KC, bool PAIR, bool RADER = false>
__device__ __forceinline__ void time_gt_body(const TimeArgs& a, long long wg, c64* lds) {
  constexpr int N = A * B;
  constexpr int H = gt_pairs<B>();
  constexpr int NCH = (H + KC - 1) / KC;
  constexpr int c1 = gt_inv_mod(B % A, A);
  constexpr int c2 = gt_inv_mod(A % B, B);
  static_assert(A >= 2 && c1 > 0, "A and B must be coprime");
  static_assert(c2 > 0, "A and B must be coprime");
  constexpr int T = A * S;
  constexpr GtRoots<B> R{};
  using Tile = TimeTileR<PAIR>;
  c64* dt = lds;
  c64* gi = dt + N;
  c64* Y = gi + N;  // [slot][a][s] for one chunk of outputs
  static_assert(S % 64 == 0, "one row index per wave");
  const int t = threadIdx.x, s = t % S;
  const int ra = __builtin_amdgcn_readfirstlane(t / S);  // uniform across the wave

  const Tile tile(a, wg, S, s);
  double ga, gb, mua, mub;
  tile.fetch(a, ga, gb, mua, mub);

  const SolveScalars sc = solve_scalars(a.sc, a.alpha_dev, a.variant, a.tau);
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

  // Steps (a)+(b) on row ra: x[ra, b] = u_{(B ra + A b) mod N}
  c64 v[B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    int n = B * ra + A * b;
    n = n >= N ? n - N : n;
    n = n >= N ? n - N : n;
    const c64 z = dt[n];
    const double xa = z.re + mua, xb = z.re + mub;
    double qa, qb;
    recip2_nr(xa * xa + z.im * z.im, xb * xb + z.im * z.im, qa, qb);
    const double ia = ga * qa, ib = gb * qb;
    v[b] = {ia * xa + ib * z.im, ib * xb - ia * z.im};
  }
  // length-B DFT over b: Rader's algorithm in registers, or the symmetric form
  // (a_j = x_j + x_{B-j}, b_j = x_j - x_{B-j}) evaluated chunk by chunk below
  c64 x0 = v[0], s0 = x0;
  if constexpr (RADER) {
    gt_rader_dft<B>(v);
    s0 = v[0];
  } else {
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const c64 p = v[j], q = v[B - j];
      v[j] = cadd(p, q);
      v[B - j] = csub(p, q);
      s0 = cadd(s0, v[j]);
    }
  }
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int klo = gt_chunk_first<B, KC>(ch), khi = gt_chunk_last<B, KC>(ch);
    const int base = ch == 0 ? 1 : 0;
    if (ch == 0) Y[(size_t)ra * S + s] = s0;
#pragma unroll
    for (int k = klo; k <= khi; ++k) {
      const int sl = base + 2 * (k - klo);
      if constexpr (RADER) {
        Y[((size_t)sl * A + ra) * S + s] = v[k];
        Y[((size_t)(sl + 1) * A + ra) * S + s] = v[B - k];
      } else {
        c64 Ak = x0, Bk = {0.0, 0.0};
#pragma unroll
        for (int j = 1; j <= H; ++j) {
          const int r = (j * k) % B;
          Ak.re += v[j].re * R.c[r];
          Ak.im += v[j].im * R.c[r];
          Bk.re += v[B - j].re * R.s[r];  // X_k = A_k - i B_k, B_k = sum_j b_j sin(2 pi jk/B)
          Bk.im += v[B - j].im * R.s[r];
        }
        Y[((size_t)sl * A + ra) * S + s] = {Ak.re + Bk.im, Ak.im - Bk.re};        // X_k
        Y[((size_t)(sl + 1) * A + ra) * S + s] = {Ak.re - Bk.im, Ak.im + Bk.re};  // X_{B-k}
      }
    }
    __syncthreads();
    // length-A DFTs over a for this chunk's k2; Step (c) scaling and store
    const int nsl = gt_chunk_slots<B, KC>(ch);
#pragma unroll
    for (int q0 = 0; q0 < (2 * KC + 1 + A - 1) / A; ++q0) {
      const int sl = ra + q0 * A;
      if (sl < nsl) {
        const int k2 = (ch == 0 && sl == 0) ? 0 : (((sl - base) & 1) ? B - (klo + (sl - base) / 2) : klo + (sl - base) / 2);
        c64 w[A];
#pragma unroll
        for (int q = 0; q < A; ++q) w[q] = Y[((size_t)sl * A + q) * S + s];
        Bfly<A>::run(w);
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
          const int l = (B * c1 * k1 + A * c2 * k2) % N;
          tile.store(a, l, cmul(gi[l], w[k1]));
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace qbvm
