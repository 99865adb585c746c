// Compile-time FFT of a power-of-two length N (64..4096) for gfx950, FP64.
//
// Every lane owns E (8 or 16) complex values throughout: P = N/E lanes form the
// team of one signal and a workgroup of T lanes carries S = T/P signals.  A
// stage of radix R <= E gives each lane E/R butterflies; inputs and outputs of a
// stage stay in registers, and LDS is used only to exchange values between
// consecutive stages.  Two lane layouts:
//   SigFast: lanes of a wave belong to different signals (lane = s + S u); LDS
//            holds [position][signal], so every exchange access is consecutive.
//   PosFast: lanes of a wave walk along one signal (lane = u + P s); LDS holds
//            [signal][position] with one pad slot per 16 positions.
// Stockham autosort indexing: butterfly j of a stage with radix R, after the
// radices NS already applied, reads positions j + r N/R and writes
// (j - k) R + k + r NS with k = j mod NS, after twiddling input r by
// exp(-2 pi i k r / (NS R)).  After the last stage lane (u, b) holds X at
// positions u + b P + r N/R_last, r < R_last.
#pragma once

#include "qbvm_fft_dev.hpp"

namespace qbvm {

// Radix sequences per (N, E); every radix divides E.
template <int N, int E>
struct P2Radices;
#define QBVM_P2_RADICES(NN, EE, ...)                          \
  template <>                                                 \
  struct P2Radices<NN, EE> {                                  \
    static constexpr int R[] = {__VA_ARGS__};                 \
    static constexpr int K = sizeof(R) / sizeof(int);         \
  };
QBVM_P2_RADICES(64, 16, 8, 8)
QBVM_P2_RADICES(128, 16, 16, 8)
QBVM_P2_RADICES(256, 16, 16, 16)
QBVM_P2_RADICES(512, 16, 8, 8, 8)
QBVM_P2_RADICES(1024, 16, 16, 8, 8)
QBVM_P2_RADICES(2048, 16, 16, 16, 8)
QBVM_P2_RADICES(4096, 16, 16, 16, 16)
QBVM_P2_RADICES(64, 8, 8, 8)
QBVM_P2_RADICES(128, 8, 8, 8, 2)
QBVM_P2_RADICES(256, 8, 8, 8, 4)
QBVM_P2_RADICES(512, 8, 8, 8, 8)
QBVM_P2_RADICES(1024, 8, 8, 8, 8, 2)
QBVM_P2_RADICES(2048, 8, 8, 8, 8, 4)
QBVM_P2_RADICES(4096, 8, 8, 8, 8, 8)
#undef QBVM_P2_RADICES

template <int N, int E>
constexpr int p2_ns(int stage) {
  int ns = 1;
  for (int i = 0; i < stage; ++i) ns *= P2Radices<N, E>::R[i];
  return ns;
}

constexpr int p2_log2(int x) { return x <= 1 ? 0 : 1 + p2_log2(x / 2); }

// SigFast pads one slot per R0 positions (R0 = first radix): the stage-0 writes of
// consecutive lane groups are R0 apart, and the pad makes their LDS bank groups
// alternate.  PosFast pads one slot per 16 positions.
// PosFast position maps (PM): 0 = one pad slot per 16 positions; 1 = XOR of the
// low four position bits with the next four (no pad, fewer bank conflicts in the
// exchanges measured on gfx950); 2 = one pad slot per 8.
template <int N, int E, int S, bool SIGFAST, bool SPAD = true, int PM = 1>
struct P2Layout {
  static constexpr int P = N / E;
  static constexpr int T = S * P;
  static constexpr int R0 = P2Radices<N, E>::R[0];
  static constexpr int LR0 = SPAD ? p2_log2(R0) : 30;  // no pad: pos >> 30 == 0
  static constexpr int NPAD = PM == 1 ? N : (PM == 2 ? N + N / 8 : N + N / 16);
  static constexpr int NPADS = SPAD ? N + N / R0 : N;
  static constexpr size_t lds_elems() { return SIGFAST ? (size_t)NPADS * S : (size_t)NPAD * S; }
  static __device__ __forceinline__ int sig(int t) { return SIGFAST ? (t % S) : (t / P); }
  static __device__ __forceinline__ int lane(int t) { return SIGFAST ? (t / S) : (t % P); }
  static __device__ __forceinline__ int pmap(int pos) {
    if constexpr (PM == 1) return pos ^ ((pos >> 4) & 15);
    else if constexpr (PM == 2) return pos + (pos >> 3);
    else return pos + (pos >> 4);
  }
  static __device__ __forceinline__ int at(int s, int pos) {
    return SIGFAST ? (pos + (pos >> LR0)) * S + s : s * NPAD + pmap(pos);
  }
};

// Position held in register slot e (= b R + r) before stage STAGE.
template <int N, int E, int STAGE>
__device__ __forceinline__ int p2_in_pos(int u, int e) {
  constexpr int R = P2Radices<N, E>::R[STAGE];
  return u + (e / R) * (N / E) + (e % R) * (N / R);
}

// Position of register slot e after the last stage.
template <int N, int E>
__device__ __forceinline__ int p2_out_pos(int u, int e) {
  return p2_in_pos<N, E, P2Radices<N, E>::K - 1>(u, e);
}

// Twiddle sources, w(i) = exp(-2 pi i idx / N): a full table, or a two-level one
// with w(i) = hi[i / 64] * lo[i % 64] (64 + N/64 entries, one extra product).
struct TwFull {
  const c64* t;
  __device__ __forceinline__ c64 operator()(int i) const { return t[i]; }
};
struct TwSplit {
  const c64* lo;
  const c64* hi;
  __device__ __forceinline__ c64 operator()(int i) const { return cmul(hi[i >> 6], lo[i & 63]); }
};

// Per-lane twiddles kept in registers for a whole persistent kernel: every stage
// after the first multiplies input r of butterfly b by exp(-2 pi i k r/(NS R)) with
// k = (u + b N/E) mod NS, which depends on the lane only.
template <int N, int E>
constexpr int p2_tw_off(int stage) {
  int off = 0;
  for (int st = 1; st < stage; ++st) off += (E / P2Radices<N, E>::R[st]) * (P2Radices<N, E>::R[st] - 1);
  return off;
}
template <int N, int E>
constexpr int p2_tw_count() { return p2_tw_off<N, E>(P2Radices<N, E>::K); }

template <int N, int E>
struct TwReg {
  c64 w[p2_tw_count<N, E>() > 0 ? p2_tw_count<N, E>() : 1];
};

template <int N, int E, int STAGE>
__device__ __forceinline__ void p2_tw_fill_stage(TwReg<N, E>& T, const c64* __restrict__ tw, int u) {
  if constexpr (STAGE < P2Radices<N, E>::K) {
    constexpr int R = P2Radices<N, E>::R[STAGE];
    constexpr int NS = p2_ns<N, E>(STAGE);
#pragma unroll
    for (int b = 0; b < E / R; ++b) {
      const int k = (u + b * (N / E)) & (NS - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) T.w[p2_tw_off<N, E>(STAGE) + b * (R - 1) + r - 1] = tw[k * r * (N / (NS * R))];
    }
    p2_tw_fill_stage<N, E, STAGE + 1>(T, tw, u);
  }
}

// Load the lane's register twiddles from the full table (global memory).
template <int N, int E>
__device__ __forceinline__ TwReg<N, E> p2_tw_regs(const c64* __restrict__ tw, int u) {
  TwReg<N, E> T;
  p2_tw_fill_stage<N, E, 1>(T, tw, u);
  return T;
}

template <int N, int E, int STAGE>
__device__ __forceinline__ void p2_twiddle_group(c64* v, int b, int u, const TwReg<N, E>& tw) {
  constexpr int R = P2Radices<N, E>::R[STAGE];
  (void)u;
#pragma unroll
  for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw.w[p2_tw_off<N, E>(STAGE) + b * (R - 1) + r - 1]);
}

template <int N, int E, int STAGE, class TW>
__device__ __forceinline__ void p2_twiddle_group(c64* v, int b, int u, const TW& tw) {
  constexpr int R = P2Radices<N, E>::R[STAGE];
  constexpr int NS = p2_ns<N, E>(STAGE);
  const int k = (u + b * (N / E)) & (NS - 1);
  if (k != 0) {
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw(k * r * (N / (NS * R))));
  }
}

// Twiddle and butterflies of stage STAGE on the lane's E registers.
template <int N, int E, int STAGE, class TW>
__device__ __forceinline__ void p2_compute(c64 (&v)[E], int u, const TW& tw) {
  constexpr int R = P2Radices<N, E>::R[STAGE];
  constexpr int NS = p2_ns<N, E>(STAGE);
  constexpr int B = E / R;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    if constexpr (NS > 1) p2_twiddle_group<N, E, STAGE>(&v[b * R], b, u, tw);
    Bfly<R>::run(&v[b * R]);
  }
}

// Exchange after stage STAGE: write its outputs, read the inputs of STAGE+1.
template <int N, int E, int STAGE, class L>
__device__ __forceinline__ void p2_exchange(c64 (&v)[E], int s, int u, c64* __restrict__ buf) {
  constexpr int R = P2Radices<N, E>::R[STAGE];
  constexpr int NS = p2_ns<N, E>(STAGE);
  constexpr int B = E / R;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = u + b * (N / E);
    const int k = j & (NS - 1);
#pragma unroll
    for (int r = 0; r < R; ++r) buf[L::at(s, (j - k) * R + k + r * NS)] = v[b * R + r];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = buf[L::at(s, p2_in_pos<N, E, STAGE + 1>(u, e))];
  __syncthreads();
}

template <int N, int E, int STAGE, class L, class TW>
__device__ __forceinline__ void p2_stages(c64 (&v)[E], int s, int u, c64* buf, const TW& tw) {
  p2_compute<N, E, STAGE>(v, u, tw);
  if constexpr (STAGE + 1 < P2Radices<N, E>::K) {
    p2_exchange<N, E, STAGE, L>(v, s, u, buf);
    p2_stages<N, E, STAGE + 1, L>(v, s, u, buf, tw);
  }
}

// Whole forward DFT on registers loaded in stage-0 order (slot e = position p2_in_pos<N,E,0>).
template <int N, int E, class L, class TW>
__device__ __forceinline__ void p2_fft(c64 (&v)[E], int s, int u, c64* buf, const TW& tw) {
  p2_stages<N, E, 0, L>(v, s, u, buf, tw);
}

// Re-order registers from the final layout to the stage-0 layout (identity when
// the first and last radices agree, else one exchange through LDS).
template <int N, int E, class L>
__device__ __forceinline__ void p2_out_to_in(c64 (&v)[E], int s, int u, c64* buf) {
  constexpr int K = P2Radices<N, E>::K;
  if constexpr (P2Radices<N, E>::R[0] != P2Radices<N, E>::R[K - 1]) {
#pragma unroll
    for (int e = 0; e < E; ++e) buf[L::at(s, p2_out_pos<N, E>(u, e))] = v[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = buf[L::at(s, p2_in_pos<N, E, 0>(u, e))];
    __syncthreads();
  }
}

}  // namespace qbvm
