// Launch geometry of the power-of-two kernels (plain C++, mirrors qbvm_bodies_p2.hpp).
#pragma once

#include <cstddef>

#include "qbvm_types.hpp"

namespace qbvm {
namespace p2sz {

constexpr int kDstThreads = 256;
constexpr int kTimeThreads = 128;
constexpr int kTimeMaxN = 2048;  // S = 2048/N >= 1

inline int dst_S(int N) { return kDstThreads * 16 / N; }
inline int time_S(int N) { return kTimeThreads * 16 / N; }
inline bool tw_in_lds(int N) { return N <= 1024; }

// exchange buffer ([signal][position] padded for rows, [position][signal] for columns) + twiddles
inline size_t dst_lds(int N, bool cols) {
  const size_t S = (size_t)dst_S(N);
  const size_t buf = cols ? (size_t)N * S : (size_t)(N + N / 16) * S;
  return sizeof(c64) * (buf + (tw_in_lds(N) ? N : 0));
}

inline size_t time_lds(int N, int Nt) {
  const size_t S = (size_t)time_S(N);
  return sizeof(c64) * ((size_t)N * S + (tw_in_lds(N) ? N : 0) + N + 2 * (size_t)Nt) + sizeof(int) * 2 * (size_t)N;
}

}  // namespace p2sz
}  // namespace qbvm
