// Launch geometry of the power-of-two kernels (plain C++, shared by the host,
// the kernels and the CPU build).  Variants differ in the complex values per
// lane E and the signals per workgroup S:
//   sine passes: 0 = E16, 256 lanes; 1 = E8, 256 lanes; 2 = E8, one signal, register
//                twiddles (input transform); 3 = E16, 512 lanes; 4 = E8, 512 lanes; 5, 6 = as 1, 4 with
//                the lane's twiddles in registers (no LDS table, a third fewer LDS
//                accesses per tile); 7 = E8, one wave per workgroup (64/P signals;
//                one signal of N/8 lanes above N = 512) with register twiddles:
//                barriers stay inside one wave
//   time kernel: 0 = E16, 128 lanes; 1 = E8, 256 lanes; 2, 3 = as 0, 1 without the
//                bank-conflict pad (less LDS, more workgroups per CU); 4 = E8, 512
//                lanes; 5 = E16, 256 lanes (both unpadded: twice the signals per
//                workgroup, which changes how evenly the tiles fill the CUs)
#pragma once

#include <cstddef>
#include <cstdint>

#include "qbvm_types.hpp"

namespace qbvm {
namespace p2sz {

constexpr int kDstVariants = 8;
constexpr int kTimeVariants = 2;
constexpr int kTimeMaxN = 2048;

constexpr int dst_E(int V) { return (V == 0 || V == 3) ? 16 : 8; }
constexpr int dst_T(int N, int V) {
  return V == 2 ? N / 8 : (V == 7 ? (N / 8 < 64 ? 64 : N / 8) : ((V == 3 || V == 4 || V == 6) ? 512 : 256));
}
constexpr int dst_S(int N, int V) { return V == 2 ? 1 : dst_T(N, V) * dst_E(V) / N; }
constexpr size_t dst_lds(int N, int V, bool cols);
constexpr bool dst_valid(int N, int V) {
  return V >= 0 && V < kDstVariants && N >= 64 && N <= 4096 && (N & (N - 1)) == 0 && dst_S(N, V) >= 1 &&
         dst_T(N, V) <= 512 && dst_lds(N, V, false) <= 160 * 1024 && dst_lds(N, V, true) <= 160 * 1024;
}

constexpr int kTimeVariants2 = 6;
constexpr int time_E(int V) { return (V == 0 || V == 2 || V == 5) ? 16 : 8; }
constexpr int time_T(int V) { return V == 4 ? 512 : (V == 5 ? 256 : ((V % 2) == 0 ? 128 : 256)); }
constexpr bool time_pad(int V) { return V < 2; }
constexpr int time_S(int N, int V) { return time_T(V) * time_E(V) / N; }
constexpr size_t time_lds(int N, int V, int Nt);
constexpr bool time_valid(int N, int V) {
  return V >= 0 && V < kTimeVariants2 && N >= 64 && N <= kTimeMaxN && (N & (N - 1)) == 0 && time_S(N, V) >= 1 &&
         time_lds(N, V, N + 1) <= 160 * 1024;
}

constexpr bool tw_in_lds(int N) { return N <= 1024; }
// twiddles: 0 = full table, global; 1 = full table, LDS; 2 = two-level table, LDS;
// 3 = per-lane registers
// (E = 16 keeps at most 15 twiddles per lane for N <= 256, more above)
constexpr int dst_tw_mode(int N, int V) {
  return (V >= 5 || V == 2 || (dst_E(V) == 16 && N <= 256)) ? 3 : (tw_in_lds(N) ? 1 : 0);
}
constexpr int tw_elems(int N, int mode) { return mode == 1 ? N : (mode == 2 ? 64 + N / 64 : 0); }

// first radix of the (N, E) sequence (mirrors P2Radices, checked there by static_assert)
constexpr int first_radix(int N, int E) { return (E == 16 && N >= 128 && N != 512) ? 16 : 8; }

// exchange buffer ([signal][position] XOR-mapped for rows, [position][signal] padded for
// columns) + twiddles
constexpr size_t dst_lds(int N, int V, bool cols) {
  return sizeof(c64) * ((cols ? (size_t)(N + N / first_radix(N, dst_E(V))) : (size_t)N) * dst_S(N, V) +
                        tw_elems(N, dst_tw_mode(N, V)));
}

// time kernels: the lane's twiddles in registers for E = 8, and for E = 16 up to N = 256
constexpr int time_tw_mode(int N, int E) { return (E == 8 || N <= 256) ? 3 : (tw_in_lds(N) ? 1 : 0); }

// exchange buffer, twiddles, Rader kernel spectrum, d_j/tau and gamma_l^{-1}, two index maps
constexpr size_t time_lds(int N, int V, int Nt) {
  return sizeof(c64) * ((size_t)(N + (time_pad(V) ? N / first_radix(N, time_E(V)) : 0)) * time_S(N, V) +
                        tw_elems(N, time_tw_mode(N, time_E(V))) + N +
                        2 * (size_t)Nt) +
         sizeof(int) * 2 * (size_t)N;
}

// general right-hand side: the same, plus gamma_t, the z_0 slot of a Rader length and
// the two mode eigenvalues of each signal
constexpr size_t time_general_lds(int N, int V, int Nt) {
  return time_lds(N, V, Nt) + sizeof(c64) * ((size_t)Nt + (size_t)time_S(N, V)) + sizeof(double) * 2 * (size_t)time_S(N, V);
}
constexpr bool time_general_valid(int N, int V) {
  return time_valid(N, V) && time_general_lds(N, V, N + 1) <= 160 * 1024;
}

// Columns pass whose two columns per signal form aligned 16-byte pairs: padded
// rows (colmod > 0) and even strides, 16-byte aligned buffers.
inline bool dst_pairs_aligned(const DstArgs& a) {
  return a.colmod > 0 && a.colmod % 2 == 0 && a.inner % 2 == 0 && a.kstride % 2 == 0 && a.ostride % 2 == 0 &&
         (reinterpret_cast<std::uintptr_t>(a.in) % 16) == 0 && (reinterpret_cast<std::uintptr_t>(a.out) % 16) == 0;
}

// Good-Thomas time kernels (N_t = A * B, gcd 1, B an odd prime): S = 64 signals per
// workgroup (A waves); the B-point outputs are exchanged in chunks of KC symmetric
// pairs (KC = 7 for the even variants, 5 for the odd ones).
constexpr int kGtPairs[][2] = {{3, 43}};
constexpr bool gt_supported(int A, int B) {
  for (const auto& p : kGtPairs)
    if (p[0] == A && p[1] == B) return true;
  return false;
}
// Good-Thomas variants: 0, 1 direct 43-point rows (output chunks of 7 or 5 pairs); 2, 3 the
// same with Rader rows
constexpr int kGtVariants = 4;
constexpr int gt_S(int) { return 64; }
constexpr int gt_KC(int V) { return V % 2 == 0 ? 7 : 5; }
constexpr bool gt_rader(int V) { return V >= 2; }
constexpr int gt_T(int A, int V) { return A * gt_S(V); }
constexpr size_t gt_lds(int A, int B, int V) {
  return sizeof(c64) * ((size_t)(2 * gt_KC(V) + 1) * A * gt_S(V) + 2 * (size_t)A * B);
}

// Plane pass (x_2 and x_1 sine transforms of one [m][P1] plane per iteration), variants:
//   0: E = 16, 512 lanes;  1: E = 8, 1024 lanes;  2: as 0, the column loads of both rounds
//   issued before the first transform.
// With sine length N = 2(m+1), N/E lanes carry a signal and SR = T E/N signals run per
// round; the N/4 column (row) pairs of a plane take N/(4 SR) rounds.  One LDS region
// serves the exchanges of a round (columns: padded [position][signal]; rows: XOR-mapped
// [signal][position]) and, between them, the 2 SR rows of the transposed plane that the
// next round of row pairs reads; the twiddle table follows it.
constexpr int kPlaneVariants = 3;
constexpr int plane_T(int V) { return V == 1 ? 1024 : 512; }
constexpr int plane_E(int V) { return V == 1 ? 8 : 16; }
constexpr bool plane_preload(int V) { return V == 2; }
constexpr int plane_SR(int N, int V) { return plane_T(V) * plane_E(V) / N; }
constexpr int plane_rounds(int N, int V) { return (N / 4 + plane_SR(N, V) - 1) / plane_SR(N, V); }
constexpr size_t cmax(size_t x, size_t y) { return x > y ? x : y; }
constexpr int plane_pitch(int N) { return (N / 2 - 1 + 63) / 64 * 64; }  // P1 of m = N/2 - 1
constexpr size_t plane_region_elems(int N, int V) {  // in c64 units
  return cmax(cmax((size_t)(N + N / first_radix(N, plane_E(V))) * plane_SR(N, V), (size_t)N * plane_SR(N, V)),
              (size_t)2 * plane_SR(N, V) * plane_pitch(N) / 2);
}
constexpr size_t plane_lds(int N, int V) { return sizeof(c64) * (plane_region_elems(N, V) + (size_t)N); }
constexpr bool plane_valid(int N, int V) {
  return N == 256 && V >= 0 && V < kPlaneVariants && plane_lds(N, V) <= 160 * 1024;
}

// Bluestein sine pass on a power-of-two core of P points (64 .. 4096, P >= N - 1 for the
// sine length N, symmetric form): E = 8 values per lane, 256 lanes (512 from P = 1024), S = T E / P
// signals (2S lines) per workgroup.  LDS: the exchange buffer ([signal][position],
// XOR-mapped), then for P <= 1024 the twiddle table; the staged input and output lines
// (2S m doubles, m < P/2) reuse the exchange buffer.
constexpr int kBlueE = 8;
constexpr int blue_T(int P) { return P >= 1024 ? 512 : 256; }
constexpr int blue_S(int P) { return blue_T(P) * kBlueE / P; }
constexpr int blue_tw_mode(int P) { return P <= 1024 ? 1 : 0; }
constexpr size_t blue_lds(int P) {
  return sizeof(c64) * ((size_t)P * blue_S(P) + (blue_tw_mode(P) == 1 ? (size_t)P : 0));
}
constexpr bool blue_valid(int P) { return P >= 64 && P <= 4096 && (P & (P - 1)) == 0; }

}  // namespace p2sz
}  // namespace qbvm
