// Sine passes of lengths without a fast kernel of their own: the length-N DFT of the
// packed odd extensions (N = 2(m+1), as in k_dst) by Bluestein's identity
//   X_k = conj(w_k) sum_j a_j w_{k-j},   a_j = x_j conj(w_j),   w_j = exp(i pi j^2 / N),
// in a form that uses the odd symmetry.  With h = N/2 = m+1: w_{N-j} = w_j (N even) and
// x_{N-j} = -x_j give a_{j+h} = -a_{h-j}, so the inputs j >= h are the negated mirror image
// of the first half a_lo (j < h).  On a cyclic core of P >= N - 1 points the second half's
// transform is -A_lo(-k) exp(-2 pi i k h/P), and the convolution for outputs k < h is
//   conv = IDFT( A_lo(k) K_lo(k) + A_lo(-k) K_hi(k) )
// with K_lo the spectrum of w_s and K_hi that of w_{s-h} (s in [-(h-1), h-1]) times
// -exp(-2 pi i k h/P), both divided by P (host tables, kspec[0..P) and kspec[P..2P)).
// Both transforms run on the compile-time power-of-two engine; the inverse one as
// conj(FFT(conj(.))).
#pragma once

#include "qbvm_bodies_p2.hpp"

namespace qbvm {

// One tile of 2S lines per workgroup (rows of [outer][m] or 2S consecutive columns of
// [outer][m][inner], as in k_dst).  The lines are staged in LDS with coalesced loads, each
// lane gathers the E positions it holds in the engine's input order, the forward
// transform runs in registers, its output goes through LDS once so that every lane can
// read the bins k and -k of its next input positions, the inverse transform runs in
// registers, and outputs 1..m go back through LDS to coalesced stores.  The staging area
// is the exchange buffer itself.
template <int P>
__device__ __forceinline__ void dst_blue_body(const DstArgs& a, long long wg, c64* lds) {
  constexpr int E = p2sz::kBlueE, S = p2sz::blue_S(P);
  using L = P2Layout<P, E, S, false, true, 1>;
  constexpr int T = L::T;
  c64* buf = lds;
  const int t = threadIdx.x, s = L::sig(t), u = L::lane(t);
  const int m = a.len, nl = 2 * S;
  const auto tw = p2_twiddles<P, p2sz::blue_tw_mode(P), E>(a.fft, buf + L::lds_elems(), t, T);
  const bool contig = (a.inner == 1);
  long long o = 0, i0 = 0;
  if (contig) {
    i0 = wg * nl;
  } else {
    o = wg / a.tiles_per_outer;
    i0 = (wg - o * a.tiles_per_outer) * nl;
  }
  // chirps of the lane's input positions (only 1..m carry data), fetched while the lines load
  c64 cw[E];
#pragma unroll
  for (int e = 0; e < E; ++e) cw[e] = a.fft.chirp[min(p2_in_pos<P, E, 0>(u, e), m)];
  double* xs = reinterpret_cast<double*>(buf);  // staged lines: [2S][m]
  const int tot = nl * m;
  {
    // element e: rows (q, k) = (e / m, e mod m); columns (k, q) = (e / nl, e mod nl)
    LaneWalk w(contig ? m : nl);
    for (int e0 = t; e0 < tot; e0 += kBatch * T) {
      double xv[kBatch];
      int dv[kBatch];
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        // indices past the data are clamped to the last valid element, so every load of
        // the batch is unconditional; the value is then replaced by 0
        const int q = contig ? w.j : w.s, k = min(contig ? w.s : w.j, m - 1);
        const bool live = e0 + b * T < tot;
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
        xv[b] = x;
        dv[b] = q * m + k;
        w.next();
      }
#pragma unroll
      for (int b = 0; b < kBatch; ++b)
        if (e0 + b * T < tot) xs[dv[b]] = xv[b];
    }
  }
  __syncthreads();
  // a_lo(j) = (x_a(j) + i x_b(j)) conj(w_j) for j = 1..m, 0 elsewhere on the core
  c64 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int pos = p2_in_pos<P, E, 0>(u, e);
    const bool on = pos >= 1 && pos <= m;
    const int i = on ? pos - 1 : 0;
    const c64 x = {xs[(2 * s) * m + i], xs[(2 * s + 1) * m + i]};
    v[e] = on ? cmul(x, cconj(cw[e])) : c64{0.0, 0.0};
  }
  __syncthreads();  // the exchanges overwrite the staged lines
  p2_fft<P, E, L>(v, s, u, buf, tw);
  // bins k and -k of the lane's next input positions, through the exchange buffer
#pragma unroll
  for (int e = 0; e < E; ++e) buf[L::at(s, p2_out_pos<P, E>(u, e))] = v[e];
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int q = p2_in_pos<P, E, 0>(u, e);
    const c64 A = buf[L::at(s, q)], Am = buf[L::at(s, (P - q) & (P - 1))];
    v[e] = cconj(cadd(cmul(A, a.fft.kspec[q]), cmul(Am, a.fft.kspec[P + q])));
  }
  __syncthreads();
  p2_fft<P, E, L>(v, s, u, buf, tw);
#pragma unroll
  for (int e = 0; e < E; ++e) cw[e] = cconj(a.fft.chirp[min(p2_out_pos<P, E>(u, e), m)]);
  // outputs 1..m: X_k = conj(w_k) conj(v); line 2s from -Im, line 2s+1 from Re (every lane
  // has passed the last exchange's closing barrier, so the buffer is free)
  double* ys = xs;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = p2_out_pos<P, E>(u, e);
    if (k >= 1 && k <= m) {
      const c64 X = cmul(cw[e], cconj(v[e]));
      ys[(2 * s) * m + k - 1] = -X.im * a.scale;
      ys[(2 * s + 1) * m + k - 1] = X.re * a.scale;
    }
  }
  __syncthreads();
  LaneWalk w(contig ? m : nl);
  for (int e = t; e < tot; e += T) {
    const int q = contig ? w.j : w.s, k = contig ? w.s : w.j;
    w.next();
    if (contig) {
      const long long line = i0 + q;
      if (line < a.outer) a.out[line * a.out_pitch + k] = ys[q * m + k];
    } else {
      const long long i = i0 + q;
      if (dst_col_ok(a, i)) a.out[o * a.ostride + k * a.kstride + i] = ys[q * m + k];
    }
  }
}

}  // namespace qbvm
