// Workgroup-cooperative batched complex FFT in LDS for gfx950 (FP64).
//
// A workgroup transforms S signals at once.  Signal s, element k lives at
// buf[k * S + s] (signals fastest), so consecutive lanes touch consecutive
// 16-byte words.  Each Stockham stage is done in place: every lane first reads
// the inputs of its butterflies into registers, the workgroup synchronises, then
// each lane twiddles, transforms and writes its outputs to their autosorted
// positions.  A lane owns at most kElemsPerThread complex values per stage; the
// host picks S so that S * nc <= kElemsPerThread * blockDim.x.
//
// Logical lengths that are not products of the supported radices are handled
// on top of the same core: a prime n with smooth n-1 by Rader's permutation to a
// cyclic convolution of length n-1, anything else by Bluestein's chirp to a
// smooth length P >= 2n-1.  Both evaluate the convolution as
// conj(FFT(conj(FFT(a) * K))) with the kernel spectrum K precomputed on the host.
#pragma once

#include "qbvm_types.hpp"

namespace qbvm {

// exp(-2 pi i k / R) for R = 1..64, at c_root[R (R-1)/2 + k].
extern __constant__ c64 c_root[2080];

__device__ __forceinline__ c64 cadd(c64 a, c64 b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ c64 csub(c64 a, c64 b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ c64 cmul(c64 a, c64 b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ c64 cconj(c64 a) { return {a.re, -a.im}; }
__device__ __forceinline__ c64 cscale(c64 a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ c64 mul_negi(c64 a) { return {a.im, -a.re}; }  // a * (-i)

// Element loops of the workgroup (e = threadIdx.x + i * blockDim.x) run in batches of
// kBatch: a batch issues all of its global loads before it uses any of them, so it
// waits for memory once instead of once per element.
constexpr int kBatch = 8;

// (j, s) = (e / S, e mod S) for e = threadIdx.x + i * blockDim.x, i = 0, 1, ...: one
// division at the start, then an add with carry per step.
struct LaneWalk {
  int j, s, dj, ds, S;
  __device__ __forceinline__ explicit LaneWalk(int S_) : S(S_) {
    const int T = (int)blockDim.x, t = (int)threadIdx.x;
    j = t / S;
    s = t - j * S;
    dj = T / S;
    ds = T - dj * S;
  }
  __device__ __forceinline__ void next() {
    s += ds;
    j += dj;
    if (s >= S) {
      s -= S;
      ++j;
    }
  }
};

// ---------------------------------------------------------------- butterflies
__device__ __forceinline__ void bfly4(c64& x0, c64& x1, c64& x2, c64& x3) {
  const c64 t0 = cadd(x0, x2), t1 = csub(x0, x2);
  const c64 t2 = cadd(x1, x3), t3 = mul_negi(csub(x1, x3));
  x0 = cadd(t0, t2);
  x1 = cadd(t1, t3);
  x2 = csub(t0, t2);
  x3 = csub(t1, t3);
}

template <int R>
struct Bfly;

template <>
struct Bfly<2> {
  static __device__ __forceinline__ void run(c64* v) {
    const c64 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <>
struct Bfly<4> {
  static __device__ __forceinline__ void run(c64* v) { bfly4(v[0], v[1], v[2], v[3]); }
};

template <>
struct Bfly<8> {
  static __device__ __forceinline__ void run(c64* v) {
    constexpr double r = 0.70710678118654752440;
    c64 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    c64 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    bfly4(e0, e1, e2, e3);
    bfly4(o0, o1, o2, o3);
    o1 = {r * (o1.re + o1.im), r * (o1.im - o1.re)};    // * exp(-i pi/4)
    o2 = mul_negi(o2);                                  // * exp(-i pi/2)
    o3 = {r * (o3.im - o3.re), -r * (o3.re + o3.im)};   // * exp(-3 i pi/4)
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
  }
};

template <>
struct Bfly<16> {
  // 4 x 4 decomposition: n = p + 4q, k = k1 + 4 k2.
  static __device__ __forceinline__ void run(c64* v) {
    constexpr double c1 = 0.92387953251128675613;  // cos(pi/8)
    constexpr double s1 = 0.38268343236508977173;  // sin(pi/8)
    constexpr double r = 0.70710678118654752440;
#pragma unroll
    for (int p = 0; p < 4; ++p) bfly4(v[p], v[p + 4], v[p + 8], v[p + 12]);
    // Y_p[k1] sits at v[p + 4 k1]; multiply by exp(-2 pi i p k1 / 16)
    auto tw = [](c64 a, double wr, double wi) { return c64{a.re * wr - a.im * wi, a.re * wi + a.im * wr}; };
    v[5] = tw(v[5], c1, -s1);         // p=1,k1=1
    v[9] = tw(v[9], r, -r);           // p=1,k1=2
    v[13] = tw(v[13], s1, -c1);       // p=1,k1=3
    v[6] = tw(v[6], r, -r);           // p=2,k1=1
    v[10] = mul_negi(v[10]);          // p=2,k1=2
    v[14] = tw(v[14], -r, -r);        // p=2,k1=3
    v[7] = tw(v[7], s1, -c1);         // p=3,k1=1
    v[11] = tw(v[11], -r, -r);        // p=3,k1=2
    v[15] = tw(v[15], -c1, s1);       // p=3,k1=3
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) bfly4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // X_{k1 + 4 k2} = v[4 k1 + k2]: transpose the 4 x 4 register block
    c64 t[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = t[i];
  }
};

// Odd radix R: X_k = x_0 + sum_j (x_j + x_{R-j}) cos(2 pi jk/R) - i sum_j (x_j - x_{R-j}) sin(2 pi jk/R)
template <int R>
struct Bfly {
  static_assert(R % 2 == 1 && R >= 3, "odd radix");
  static __device__ __forceinline__ void run(c64* v) {
    constexpr int H = (R - 1) / 2;
    constexpr int base = R * (R - 1) / 2;
    c64 a[H], b[H];
    const c64 x0 = v[0];
    c64 s = x0;
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      a[j - 1] = cadd(v[j], v[R - j]);
      b[j - 1] = csub(v[j], v[R - j]);
      s = cadd(s, a[j - 1]);
    }
    v[0] = s;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      c64 A = x0, B = {0.0, 0.0};
#pragma unroll
      for (int j = 1; j <= H; ++j) {
        const c64 w = c_root[base + (j * k) % R];
        A.re += a[j - 1].re * w.re;
        A.im += a[j - 1].im * w.re;
        B.re -= b[j - 1].re * w.im;
        B.im -= b[j - 1].im * w.im;
      }
      v[k] = {A.re + B.im, A.im - B.re};
      v[R - k] = {A.re - B.im, A.im + B.re};
    }
  }
};

// ---------------------------------------------------------- Stockham stage
template <int R>
__device__ __forceinline__ void fft_stage(c64* __restrict__ buf, int S, int nc, int ns, int twstride,
                                          const c64* __restrict__ tw) {
  constexpr int MB = (kElemsPerThread + R - 1) / R;
  const int q = nc / R;
  // butterfly b = threadIdx.x + i T: signal s = b mod S, index j = b / S (valid for j < q),
  // k = j mod ns; all three advance without a division per butterfly
  LaneWalk w(S);
  const int dk = w.dj % ns;
  int k = w.j % ns;
  c64 v[MB][R];
  int jj[MB], ss[MB], kk[MB];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    jj[i] = w.j;
    ss[i] = w.s;
    kk[i] = k;
    if (w.j < q) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[(w.j + r * q) * S + w.s];
    }
    const int j_old = w.j;
    w.next();
    k += dk + (w.j - j_old - w.dj);  // + carry
    if (k >= ns) k -= ns;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    if (jj[i] < q) {
      const int j = jj[i], s = ss[i], kr = kk[i];
      if (kr != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], tw[kr * r * twstride]);
      }
      Bfly<R>::run(v[i]);
      const int base = (j - kr) * R + kr;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(base + r * ns) * S + s] = v[i][r];
    }
  }
  __syncthreads();
}

// tw: the plan's twiddle table, or a copy of it in LDS
template <bool WIDE>
__device__ __forceinline__ void fft_core(c64* buf, int S, const FftPlanDev& p, const c64* __restrict__ tw) {
  for (int i = 0; i < p.nstages; ++i) {
    const int R = p.st[i].radix, ns = p.st[i].ns, tws = p.st[i].twstride;
    switch (R) {
      case 2: fft_stage<2>(buf, S, p.nc, ns, tws, tw); break;
      case 3: fft_stage<3>(buf, S, p.nc, ns, tws, tw); break;
      case 4: fft_stage<4>(buf, S, p.nc, ns, tws, tw); break;
      case 5: fft_stage<5>(buf, S, p.nc, ns, tws, tw); break;
      case 7: fft_stage<7>(buf, S, p.nc, ns, tws, tw); break;
      case 8: fft_stage<8>(buf, S, p.nc, ns, tws, tw); break;
      case 16: fft_stage<16>(buf, S, p.nc, ns, tws, tw); break;
      default:
        if constexpr (WIDE) {
          switch (R) {
            case 11: fft_stage<11>(buf, S, p.nc, ns, tws, tw); break;
            case 13: fft_stage<13>(buf, S, p.nc, ns, tws, tw); break;
            case 17: fft_stage<17>(buf, S, p.nc, ns, tws, tw); break;
            case 19: fft_stage<19>(buf, S, p.nc, ns, tws, tw); break;
            case 23: fft_stage<23>(buf, S, p.nc, ns, tws, tw); break;
            case 29: fft_stage<29>(buf, S, p.nc, ns, tws, tw); break;
            case 31: fft_stage<31>(buf, S, p.nc, ns, tws, tw); break;
            case 37: fft_stage<37>(buf, S, p.nc, ns, tws, tw); break;
            case 41: fft_stage<41>(buf, S, p.nc, ns, tws, tw); break;
            case 43: fft_stage<43>(buf, S, p.nc, ns, tws, tw); break;
            case 47: fft_stage<47>(buf, S, p.nc, ns, tws, tw); break;
            default: break;
          }
        }
        break;
    }
  }
}

// Position in the core buffer of logical input element j (-1: Rader x_0, kept aside).
__device__ __forceinline__ int fft_in_pos(const FftPlanDev& p, int j) {
  if (p.kind == kRader) return j == 0 ? -1 : p.rin[j];
  return j;
}

// Bluestein pre-processing after raw placement: x_j * conj(w_j) for j < n, 0 beyond.
__device__ __forceinline__ void fft_bluestein_prep(c64* buf, int S, const FftPlanDev& p) {
  const int tot = S * p.nc, T = blockDim.x;
  LaneWalk w(S);
  for (int e0 = threadIdx.x; e0 < tot; e0 += kBatch * T) {
    c64 cw[kBatch];
    int jv[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      jv[u] = w.j;
      cw[u] = p.chirp[min(w.j, p.n - 1)];  // clamped: the loads need no branch
      w.next();
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int e = e0 + u * T;
      if (e < tot) buf[e] = jv[u] < p.n ? cmul(buf[e], cconj(cw[u])) : c64{0.0, 0.0};
    }
  }
  __syncthreads();
}

// Run the transform on placed input (Bluestein input already pre-processed).
// side[0..S) holds Rader's x_0; side[S..2S) receives sum_{j>=1} x_j.
template <bool WIDE>
__device__ __forceinline__ void fft_run(c64* buf, int S, const FftPlanDev& p, c64* side, const c64* tw) {
  fft_core<WIDE>(buf, S, p, tw);
  if (p.kind == kStockham) return;
  const int tot = S * p.nc, T = blockDim.x;
  LaneWalk w(S);
  for (int e0 = threadIdx.x; e0 < tot; e0 += kBatch * T) {
    c64 ks[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      ks[u] = p.kspec[min(w.j, p.nc - 1)];
      w.next();
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int e = e0 + u * T;
      if (e < tot) {
        const c64 x = buf[e];
        if (p.kind == kRader && e < S) side[S + e] = x;  // position 0: e == s
        buf[e] = cconj(cmul(x, ks[u]));
      }
    }
  }
  __syncthreads();
  fft_core<WIDE>(buf, S, p, tw);
}

template <bool WIDE>
__device__ __forceinline__ void fft_run(c64* buf, int S, const FftPlanDev& p, c64* side) {
  fft_run<WIDE>(buf, S, p, side, p.tw);
}

// Copy of the twiddle table into LDS at dst (nc entries) when the kernel's flag asks for it;
// returns the table the transform reads (the caller synchronises before the transform).
__device__ __forceinline__ const c64* stage_twiddles(const FftPlanDev& p, int in_lds, c64* dst) {
  if (!in_lds) return p.tw;
  const int T = blockDim.x;
  for (int i0 = threadIdx.x; i0 < p.nc; i0 += kBatch * T) {
    c64 v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) v[u] = p.tw[min(i0 + u * T, p.nc - 1)];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (i0 + u * T < p.nc) dst[i0 + u * T] = v[u];
  }
  return dst;
}

// What the read of logical output k needs from the plan's global tables (Rader's
// output position, Bluestein's chirp), fetched ahead of the LDS read by batched loops.
struct FftOutAt {
  int pos;  // core position; -1: Rader's X_0
  c64 w;    // Bluestein: conj(chirp_k)
};
__device__ __forceinline__ FftOutAt fft_out_at(const FftPlanDev& p, int k) {
  FftOutAt o{k, {1.0, 0.0}};
  if (p.kind == kRader) o.pos = k == 0 ? -1 : p.rout[k];
  else if (p.kind == kBluestein) o.w = cconj(p.chirp[k]);
  return o;
}

// Logical output of signal s at o after fft_run.
__device__ __forceinline__ c64 fft_out(const c64* buf, int S, const FftPlanDev& p, int s, const FftOutAt& o,
                                       const c64* side) {
  if (p.kind == kStockham) return buf[o.pos * S + s];
  if (p.kind == kRader) {
    const c64 x0 = side[s];
    if (o.pos < 0) return cadd(x0, side[S + s]);
    return cadd(x0, cconj(buf[o.pos * S + s]));
  }
  return cmul(o.w, cconj(buf[o.pos * S + s]));
}

// Logical output X_k of signal s after fft_run.
__device__ __forceinline__ c64 fft_out(const c64* buf, int S, const FftPlanDev& p, int s, int k,
                                       const c64* side) {
  return fft_out(buf, S, p, s, fft_out_at(p, k), side);
}

}  // namespace qbvm
