// Compile-time FFT of a power-of-two length N (64..4096) for gfx950, FP64.
//
// Every lane owns E = 16 complex values throughout: P = N/16 lanes form the team
// of one signal and a workgroup of T lanes carries S = T/P signals.  A stage of
// radix R (16 or 8) gives each lane 16/R butterflies; inputs and outputs of a
// stage stay in registers, and LDS is used only to exchange values between
// consecutive stages.  Two lane layouts:
//   SigFast: lanes of a wave belong to different signals (lane = s + S u); LDS
//            holds [position][signal], so every exchange access is consecutive.
//   PosFast: lanes of a wave walk along one signal (lane = u + P s); LDS holds
//            [signal][position] with one pad slot per 16 positions.
// Stockham autosort indexing: a butterfly j of a stage with radix R, after the
// radices NS already applied, reads positions j + r N/R and writes
// (j - k) R + k + r NS with k = j mod NS, after twiddling input r by
// exp(-2 pi i k r / (NS R)).  After the last stage lane (u, b) holds X at
// positions u + b P + r N/R_last, r < R_last.
#pragma once

#include "qbvm_fft_dev.hpp"

namespace qbvm {

template <int N>
struct P2Radices;
template <> struct P2Radices<64> { static constexpr int K = 2; static constexpr int R[2] = {8, 8}; };
template <> struct P2Radices<128> { static constexpr int K = 2; static constexpr int R[2] = {16, 8}; };
template <> struct P2Radices<256> { static constexpr int K = 2; static constexpr int R[2] = {16, 16}; };
template <> struct P2Radices<512> { static constexpr int K = 3; static constexpr int R[3] = {8, 8, 8}; };
template <> struct P2Radices<1024> { static constexpr int K = 3; static constexpr int R[3] = {16, 8, 8}; };
template <> struct P2Radices<2048> { static constexpr int K = 3; static constexpr int R[3] = {16, 16, 8}; };
template <> struct P2Radices<4096> { static constexpr int K = 3; static constexpr int R[3] = {16, 16, 16}; };

template <int N>
constexpr int p2_ns(int stage) {
  int ns = 1;
  for (int i = 0; i < stage; ++i) ns *= P2Radices<N>::R[i];
  return ns;
}

template <int N, int S, bool SIGFAST>
struct P2Layout {
  static constexpr int P = N / 16;
  static constexpr int T = S * P;
  static constexpr int NPAD = N + N / 16;
  static constexpr size_t lds_elems() { return SIGFAST ? (size_t)N * S : (size_t)NPAD * S; }
  static __device__ __forceinline__ int sig(int t) { return SIGFAST ? (t % S) : (t / P); }
  static __device__ __forceinline__ int lane(int t) { return SIGFAST ? (t / S) : (t % P); }
  static __device__ __forceinline__ int at(int s, int pos) {
    return SIGFAST ? pos * S + s : s * NPAD + pos + (pos >> 4);
  }
};

// Position held in register slot e (= b R + r) before stage `stage`.
template <int N, int STAGE>
__device__ __forceinline__ int p2_in_pos(int u, int e) {
  constexpr int R = P2Radices<N>::R[STAGE];
  return u + (e / R) * (N / 16) + (e % R) * (N / R);
}

// Position of register slot e after the last stage.
template <int N>
__device__ __forceinline__ int p2_out_pos(int u, int e) {
  return p2_in_pos<N, P2Radices<N>::K - 1>(u, e);
}

// Twiddle and butterflies of stage STAGE on the lane's 16 registers.
template <int N, int STAGE>
__device__ __forceinline__ void p2_compute(c64 (&v)[16], int u, const c64* __restrict__ tw) {
  constexpr int R = P2Radices<N>::R[STAGE];
  constexpr int NS = p2_ns<N>(STAGE);
  constexpr int B = 16 / R;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    if constexpr (NS > 1) {
      const int j = u + b * (N / 16);
      const int k = j & (NS - 1);
      if (k != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[b * R + r] = cmul(v[b * R + r], tw[k * r * (N / (NS * R))]);
      }
    }
    Bfly<R>::run(&v[b * R]);
  }
}

// Exchange after stage STAGE: write outputs, read inputs of stage STAGE+1.
template <int N, int STAGE, class L>
__device__ __forceinline__ void p2_exchange(c64 (&v)[16], int s, int u, c64* __restrict__ buf) {
  constexpr int R = P2Radices<N>::R[STAGE];
  constexpr int NS = p2_ns<N>(STAGE);
  constexpr int B = 16 / R;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = u + b * (N / 16);
    const int k = j & (NS - 1);
#pragma unroll
    for (int r = 0; r < R; ++r) buf[L::at(s, (j - k) * R + k + r * NS)] = v[b * R + r];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 16; ++e) v[e] = buf[L::at(s, p2_in_pos<N, STAGE + 1>(u, e))];
  __syncthreads();
}

// Whole forward DFT on registers loaded in stage-0 order (slot e = position p2_in_pos<N,0>).
template <int N, class L>
__device__ __forceinline__ void p2_fft(c64 (&v)[16], int s, int u, c64* buf, const c64* tw) {
  p2_compute<N, 0>(v, u, tw);
  if constexpr (P2Radices<N>::K >= 2) {
    p2_exchange<N, 0, L>(v, s, u, buf);
    p2_compute<N, 1>(v, u, tw);
  }
  if constexpr (P2Radices<N>::K >= 3) {
    p2_exchange<N, 1, L>(v, s, u, buf);
    p2_compute<N, 2>(v, u, tw);
  }
}

// Re-order registers from the final layout to the stage-0 layout (identity when
// the first and last radices agree, else one exchange through LDS).
template <int N, class L>
__device__ __forceinline__ void p2_out_to_in(c64 (&v)[16], int s, int u, c64* buf) {
  constexpr int K = P2Radices<N>::K;
  if constexpr (P2Radices<N>::R[0] != P2Radices<N>::R[K - 1]) {
#pragma unroll
    for (int e = 0; e < 16; ++e) buf[L::at(s, p2_out_pos<N>(u, e))] = v[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = buf[L::at(s, p2_in_pos<N, 0>(u, e))];
    __syncthreads();
  }
}

}  // namespace qbvm
