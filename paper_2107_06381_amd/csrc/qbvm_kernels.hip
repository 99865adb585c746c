// gfx950 kernels of the PinT quasi-boundary value solver (arXiv 2107.06381).
//
// Solve pipeline for one instance (Section 3.3, eq. "3step"):
//   d = 2, 3: the Dirichlet stencil is diagonalised by the orthonormal type-I sine
//     transform Q in every dimension, so Step (b)'s N_t complex-shifted solves
//     (d_j/tau - Lap_h) S2(:,j) = S1(:,j) become Q diag(1/(d_j/tau + mu_k)) Q.
//     Q commutes with the time transforms (they act on different Kronecker
//     factors), so Q is applied once to g_delta before and once per level after:
//        k_dst   : g_hat = Q g_delta                        (d passes)
//        k_time  : per mode k, Step (a) for the rank-one right-hand side
//                  (S1(k,j) = f0_hat_k/sqrt(N_t) for every j), Step (b) as a
//                  division, Step (c) as a length-N_t DFT with the inverse omega
//                  scaling, real part -> y_hat[t][k]
//        k_dst   : y[t] = Q y_hat[t]                        (d passes per level)
//   d = 1: paper order, Step (b) by a complex Thomas sweep per shift d_j
//     (k_tri1d), Step (c) as a length-N_t DFT per grid point (k_time1d).
// Two real sequences are packed into one complex transform wherever the result
// of each is real (sine transforms; time transforms after the inverse scaling).
#include "../../include/qbvm.h"
#include "qbvm_internal.hpp"
#include "qbvm_bodies.hpp"
#include "qbvm_bodies_p2.hpp"
#include "qbvm_bodies_gt.hpp"
#include "qbvm_bodies_krylov.hpp"
#include "qbvm_p2_sizes.hpp"

#include <cmath>
#include <map>
#include <mutex>
#include <set>
#include <tuple>

namespace qbvm {

__constant__ c64 c_root[2080];

void upload_radix_roots(const c64* roots, int count) {
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_root), roots, sizeof(c64) * count, 0, hipMemcpyHostToDevice);
}

// Power-of-two kernels, one symbol per (N, variant); the input transform always
// uses variant 2, the passes over the solution levels variants 0 or 1.
// Workgroups are dispatched to the 8 XCDs round-robin (block b on XCD b mod 8), each
// XCD with its own L2.  The persistent kernels renumber the blocks so that every XCD
// holds a contiguous range of logical workgroups: tiles in flight on one XCD are then
// neighbours, and a cache line shared by two tiles is fetched into one L2 only.
__device__ __forceinline__ long long xcd_contiguous(unsigned b, unsigned G) {
  constexpr unsigned X = 8;
  const unsigned per = G / X, rem = G % X, x = b % X, i = b / X;
  return x < rem ? (long long)x * (per + 1) + i : (long long)rem * (per + 1) + (long long)(x - rem) * per + i;
}

// The sine-pass kernels are persistent: the grid is sized to the resident capacity
// and every workgroup strides over the tiles.
template <int N, int V>
__global__ __launch_bounds__(p2sz::dst_T(N, V)) void k_dst_rows_p2(DstArgs a) {
  extern __shared__ c64 lds[];
  dst_rows_p2_body<N, p2sz::dst_E(V), p2sz::dst_S(N, V), p2sz::dst_tw_mode(N, V)>(
      a, xcd_contiguous(blockIdx.x, gridDim.x), gridDim.x, lds);
}

template <int N, int V, bool VEC2>
__global__ __launch_bounds__(p2sz::dst_T(N, V)) void k_dst_cols_p2(DstArgs a) {
  extern __shared__ c64 lds[];
  dst_cols_p2_body<N, p2sz::dst_E(V), p2sz::dst_S(N, V), VEC2, p2sz::dst_tw_mode(N, V)>(
      a, xcd_contiguous(blockIdx.x, gridDim.x), gridDim.x, lds);
}

// Persistent over the tiles (a.ntiles); PAIR: modes in padded rows, 16-byte pair stores.
template <int N, int V, bool RADER, bool PAIR>
__global__ __launch_bounds__(p2sz::time_T(V)) void k_time_p2(TimeArgs a) {
  extern __shared__ c64 lds[];
  time_p2_body<N, p2sz::time_E(V), p2sz::time_S(N, V), RADER, p2sz::time_pad(V), PAIR>(a, blockIdx.x, gridDim.x,
                                                                                       lds);
}

// two waves per SIMD: the lane's B-point row stays in registers
template <int A, int B, int V, bool PAIR>
__global__ __launch_bounds__(p2sz::gt_T(A, V), 2) void k_time_gt(TimeArgs a) {
  extern __shared__ c64 lds[];
  time_gt_body<A, B, p2sz::gt_S(V), p2sz::gt_KC(V), PAIR, p2sz::gt_rader(V)>(a, blockIdx.x, lds);
}

template <int V>
static const void* time_gt_fn_v(bool pair) {
  return pair ? (const void*)&k_time_gt<3, 43, V, true> : (const void*)&k_time_gt<3, 43, V, false>;
}

static const void* time_gt_fn(int A, int B, int V, bool pair) {
  if (A == 3 && B == 43) {
    switch (V) {
      case 0: return time_gt_fn_v<0>(pair);
      case 1: return time_gt_fn_v<1>(pair);
      case 2: return time_gt_fn_v<2>(pair);
      case 3: return time_gt_fn_v<3>(pair);
      default: return nullptr;
    }
  }
  return nullptr;
}

template <int N, int V>
static const void* dst_fn_nv(bool cols, bool vec2) {
  if constexpr (p2sz::dst_valid(N, V)) {
    if (!cols) return (const void*)&k_dst_rows_p2<N, V>;
    return vec2 ? (const void*)&k_dst_cols_p2<N, V, true> : (const void*)&k_dst_cols_p2<N, V, false>;
  } else {
    return nullptr;
  }
}

template <int N>
static const void* dst_fn_n(int V, bool cols, bool vec2) {
  switch (V) {
    case 0: return dst_fn_nv<N, 0>(cols, vec2);
    case 1: return dst_fn_nv<N, 1>(cols, vec2);
    case 2: return dst_fn_nv<N, 2>(cols, vec2);
    case 3: return dst_fn_nv<N, 3>(cols, vec2);
    case 4: return dst_fn_nv<N, 4>(cols, vec2);
    case 5: return dst_fn_nv<N, 5>(cols, vec2);
    case 6: return dst_fn_nv<N, 6>(cols, vec2);
    case 7: return dst_fn_nv<N, 7>(cols, vec2);
    default: return nullptr;
  }
}

// a Rader length N + 1 is prime only at N = 256 in this range
template <int N, int V>
static const void* time_fn_nv(bool rader, bool pair) {
  if constexpr (p2sz::time_valid(N, V)) {
    if constexpr (N == 256) {
      if (rader) return pair ? (const void*)&k_time_p2<N, V, true, true> : (const void*)&k_time_p2<N, V, true, false>;
    }
    if (rader) return nullptr;
    return pair ? (const void*)&k_time_p2<N, V, false, true> : (const void*)&k_time_p2<N, V, false, false>;
  } else {
    return nullptr;
  }
}

template <int N>
static const void* time_fn_n(int V, bool rader, bool pair) {
  switch (V) {
    case 0: return time_fn_nv<N, 0>(rader, pair);
    case 1: return time_fn_nv<N, 1>(rader, pair);
    case 2: return time_fn_nv<N, 2>(rader, pair);
    case 3: return time_fn_nv<N, 3>(rader, pair);
    case 4: return time_fn_nv<N, 4>(rader, pair);
    case 5: return time_fn_nv<N, 5>(rader, pair);
    default: return nullptr;
  }
}

#define QBVM_P2_SWITCH(N, F, ...)                      \
  switch (N) {                                         \
    case 64: return F<64>(__VA_ARGS__);                \
    case 128: return F<128>(__VA_ARGS__);              \
    case 256: return F<256>(__VA_ARGS__);              \
    case 512: return F<512>(__VA_ARGS__);              \
    case 1024: return F<1024>(__VA_ARGS__);            \
    case 2048: return F<2048>(__VA_ARGS__);            \
    case 4096: return F<4096>(__VA_ARGS__);            \
    default: return nullptr;                           \
  }

// general right-hand side; a Rader length N + 1 is prime only at N = 256 in this range
template <int N, int V, bool RADER>
__global__ __launch_bounds__(p2sz::time_T(V)) void k_time_general_p2(TimeArgs a) {
  extern __shared__ c64 lds[];
  time_general_p2_body<N, p2sz::time_E(V), p2sz::time_S(N, V), RADER, p2sz::time_pad(V)>(a, blockIdx.x, lds);
}

template <int N, int V>
static const void* general_fn_nv(bool rader) {
  if constexpr (p2sz::time_general_valid(N, V)) {
    if constexpr (N == 256) {
      if (rader) return (const void*)&k_time_general_p2<N, V, true>;
    }
    return rader ? nullptr : (const void*)&k_time_general_p2<N, V, false>;
  } else {
    return nullptr;
  }
}

template <int N>
static const void* general_fn_n(int V, bool rader) {
  switch (V) {
    case 0: return general_fn_nv<N, 0>(rader);
    case 1: return general_fn_nv<N, 1>(rader);
    case 2: return general_fn_nv<N, 2>(rader);
    case 3: return general_fn_nv<N, 3>(rader);
    case 4: return general_fn_nv<N, 4>(rader);
    case 5: return general_fn_nv<N, 5>(rader);
    default: return nullptr;
  }
}

static const void* dst_p2_fn(int N, int V, bool cols, bool vec2) { QBVM_P2_SWITCH(N, dst_fn_n, V, cols, vec2) }
static const void* general_p2_fn(int N, int V, bool rader) { QBVM_P2_SWITCH(N, general_fn_n, V, rader) }
static const void* time_p2_fn(int N, int V, bool rader, bool pair) { QBVM_P2_SWITCH(N, time_fn_n, V, rader, pair) }

// ROLE only separates the kernel symbols (0: transform of g_delta, 1: rows of the
// levels, 2: strided columns of the levels) so per-kernel profiles stay apart.
template <bool WIDE, int ROLE>
__global__ __launch_bounds__(256) void k_dst(DstArgs a) {
  extern __shared__ c64 lds[];
  dst_body<WIDE>(a, blockIdx.x, lds);
}

template <bool WIDE>
__global__ __launch_bounds__(256) void k_time(TimeArgs a) {
  extern __shared__ c64 lds[];
  time_body<WIDE>(a, blockIdx.x, lds);
}

__global__ __launch_bounds__(256) void k_tri1d(ThomasArgs a) {
  extern __shared__ c64 lds[];
  tri1d_body(a, blockIdx.x, lds);
}

template <bool WIDE>
__global__ __launch_bounds__(256) void k_time1d(Time1dArgs a) {
  extern __shared__ c64 lds[];
  time1d_body<WIDE>(a, blockIdx.x, lds);
}

// Batched 1D instances: persistent launches over an argument table (see Batch1dArgs).
// Every item runs the same body as the per-instance kernels; the barrier between items
// keeps an item's first LDS writes behind the previous item's last reads.  Instances
// whose own launch has fewer lanes (P S < 256 in the tridiagonal solver) leave the
// extra lanes idle, as the body's ownership tests already do within one launch.
__global__ __launch_bounds__(256) void k_tri1d_batch(Batch1dArgs b) {
  extern __shared__ c64 lds[];
  const ThomasArgs* args = static_cast<const ThomasArgs*>(b.args);
  for (int it = blockIdx.x; it < b.nitems; it += gridDim.x) {
    if (it != (int)blockIdx.x) __syncthreads();
    const ThomasArgs a = args[b.items[2 * it]];
    tri1d_body(a, b.items[2 * it + 1], lds);
  }
}

template <bool WIDE>
__global__ __launch_bounds__(256) void k_time1d_batch(Batch1dArgs b) {
  extern __shared__ c64 lds[];
  const Time1dArgs* args = static_cast<const Time1dArgs*>(b.args);
  for (int it = blockIdx.x; it < b.nitems; it += gridDim.x) {
    if (it != (int)blockIdx.x) __syncthreads();
    const Time1dArgs a = args[b.items[2 * it]];
    time1d_body<WIDE>(a, b.items[2 * it + 1], lds);
  }
}

// ================================================================ k_row ====
// One level l of Step (c) per sine mode, directly as one DFT row:
//   Y_k(l) = Re( f0s/N_t * gamma_l^{-1} * g_hat_k * sum_j exp(-2 pi i jl/N_t) / (d_j/tau + mu_k) ).
// Optionally writes Y_k(l), and reduces sum_k (Y_k(l) - g_hat_k)^2 per instance (the
// discrepancy by Parseval), finishing in the last workgroup of each instance.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Cross-workgroup hand-off of reduction partials.  Partials and counters are only
// written and read with device-scope atomic stores/loads, which are coherent across
// the XCDs' L2 caches, so publishing needs no L2 write-back or invalidation (a
// device-scope fence would issue both, once per workgroup): wait for the partial's
// store to complete, then count the workgroup in.  The last workgroup's loads
// depend on the value the count returned.
__device__ __forceinline__ unsigned publish_and_count(double* slot, double v, unsigned* counter) {
  __hip_atomic_store(slot, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_s_waitcnt(0);
  return __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kRowLanes = 4;

__global__ __launch_bounds__(256) void k_row(RowArgs a) {
  extern __shared__ c64 lds[];
  const int Nt = a.Nt;
  c64* dt = lds;          // d_j / tau
  c64* w = dt + Nt;       // exp(-2 pi i j l / N_t)
  __shared__ double red[8];
  __shared__ int s_skip;
  __shared__ double s_alpha;
  const int inst = blockIdx.x / a.wg_per_inst;
  const int wsub = blockIdx.x - inst * a.wg_per_inst;
  double* bs = a.bstate ? a.bstate + (size_t)inst * kBState : nullptr;
  if (threadIdx.x == 0) {
    double alpha = a.alpha_dev ? *a.alpha_dev : a.alpha;
    int skip = 0;
    if (bs) {
      const bool done = bs[6] != 0.0 || bs[7] != 0.0;  // hit flag or end reached
      if (a.mode == 1) { alpha = exp10(0.5 * (bs[0] + bs[1])); skip = done; }
      else if (a.mode == 2) { alpha = exp10(bs[1]); skip = done; }
      else if (a.mode == 3) { alpha = exp10(bs[0]); skip = done; }
    }
    s_alpha = alpha;
    s_skip = skip;
  }
  __syncthreads();
  if (s_skip) return;
  const SolveScalars sc = scalars_from_alpha(s_alpha, a.variant, a.tau);
  const double croot = exp(sc.logabsw / (double)Nt);
  const double inv_tau = 1.0 / a.tau;
  for (int j = threadIdx.x; j < Nt; j += blockDim.x) {
    dt[j] = shift_over_tau(j, Nt, croot, inv_tau);
    double sn, cs;
    const long long jl = ((long long)j * a.level) % Nt;
    sincospi(2.0 * (double)jl / (double)Nt, &sn, &cs);
    w[j] = {cs, -sn};
  }
  __syncthreads();
  const c64 gi = inv_gamma(a.level, Nt, sc.logabsw, sc.f0s / (double)Nt);
  const double* gh = a.ghat + (size_t)inst * a.nmodes;
  double acc = 0.0;
  // kRowLanes lanes share one mode, each summing every kRowLanes-th shift j
  const long long per = ((a.nmodes + a.wg_per_inst - 1) / a.wg_per_inst);
  const long long kb = wsub * per;
  const long long ke = kb + per < a.nmodes ? kb + per : a.nmodes;
  const int sub = threadIdx.x % kRowLanes;
  const int mpb = blockDim.x / kRowLanes;
  for (long long kbase = kb; kbase < ke; kbase += mpb) {
    const long long k = kbase + threadIdx.x / kRowLanes;
    const bool live = k < ke;
    double sr = 0.0, si = 0.0, mu = 0.0;
    if (live) {
      mu = mode_mu(k, a.d, a.m, a.mu1d);
      for (int j = sub; j < Nt; j += kRowLanes) {
        const c64 z = dt[j];
        const double x = z.re + mu;
        const double q = recip_nr(x * x + z.im * z.im);
        // w_j / (x + i z.im) = w_j (x - i z.im) q
        const c64 ww = w[j];
        sr += (ww.re * x + ww.im * z.im) * q;
        si += (ww.im * x - ww.re * z.im) * q;
      }
    }
#pragma unroll
    for (int off = kRowLanes / 2; off >= 1; off >>= 1) {
      sr += __shfl_xor(sr, off, 64);
      si += __shfl_xor(si, off, 64);
    }
    if (live && sub == 0) {
      const double g = gh[k];
      const double Y = (gi.re * sr - gi.im * si) * g;
      if (a.yrow) a.yrow[(size_t)inst * a.nmodes + k] = Y;
      const double r = Y - g;
      acc += r * r;
    }
  }
  if (!a.partial) return;
  acc = wave_sum(acc);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  __shared__ int s_last;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    const unsigned prev = publish_and_count(&a.partial[blockIdx.x], t, &a.counter[inst]);
    s_last = (prev == (unsigned)(a.wg_per_inst - 1));
  }
  __syncthreads();
  if (!s_last) return;
  // the last workgroup of the instance sums the partials (fixed order per lane, then a fixed tree)
  double t = 0.0;
  for (int i = threadIdx.x; i < a.wg_per_inst; i += blockDim.x)
    t += __hip_atomic_load(&a.partial[(size_t)inst * a.wg_per_inst + i], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  t = wave_sum(t);
  __syncthreads();
  if (lane == 0) red[wv] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) tot += red[i];
    const double D = sqrt(a.hd * tot);
    __hip_atomic_store(&a.counter[inst], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (a.dout) a.dout[inst] = D;
    if (bs) {
      const double target = bs[2];
      if (a.mode == 1) {
        const double mid = 0.5 * (bs[0] + bs[1]);
        if (D > target) bs[1] = mid;
        else bs[0] = mid;
        bs[5] += 1.0;
      } else if (a.mode == 2) {          // D(10^hi) <= target: root above the bracket
        if (D <= target) { bs[6] = 1.0; bs[7] = 2.0; }
        bs[5] += 1.0;
      } else if (a.mode == 3) {          // D(10^lo) > target: root below the bracket
        if (D > target) { bs[6] = 1.0; bs[7] = 1.0; }
        bs[5] += 1.0;
      }
      bs[3] = D;
      bs[4] = s_alpha;
    }
    if (a.host_out && inst == 0) {  // system-scope vector stores; the sequence number last
      __hip_atomic_store(&a.host_out[1], s_alpha, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(&a.host_out[2], D, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      if (a.report_bs) {
        __hip_atomic_store(&a.host_out[3], a.report_bs[5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&a.host_out[4], a.report_bs[6], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
      __builtin_amdgcn_s_waitcnt(0);
      __hip_atomic_store(&a.host_out[0], a.host_seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

__global__ void k_bisect_init(double* bs, int count, const double* deltas, double delta_val, double tau_dp,
                              double lo, double hi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double* b = bs + (size_t)i * kBState;
  b[0] = lo;
  b[1] = hi;
  b[2] = tau_dp * (deltas ? deltas[i] : delta_val);
  b[3] = 0.0;
  b[4] = 0.0;
  b[5] = 0.0;
  b[6] = 0.0;
  b[7] = 0.0;
}

__global__ void k_bisect_finish(const double* bs, int count, double* alphas, int* hits) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double* b = bs + (size_t)i * kBState;
  double u = 0.5 * (b[0] + b[1]);
  if (b[6] != 0.0) u = (b[7] == 2.0) ? b[1] : b[0];
  alphas[i] = exp10(u);
  if (hits) hits[i] = b[6] != 0.0 ? 1 : 0;
}

// ========================================================== k_features ====
// One workgroup per instance: 32 bins of rho = |k|_2 over [sqrt(d), m sqrt(d)],
// feature_b = log10(h^d sum_{k in b} g_hat_k^2 + 1e-300); feature_32 = log10(delta).
// The modes of bin b are perm[off[b] .. off[b+1]) (built on the host); each bin is
// reduced in a fixed order, so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_features(long long nm, double hd, const double* ghat,
                                                  const double* deltas, const int* perm,
                                                  const int* off, float* feats) {
  __shared__ double red[4];
  const int inst = blockIdx.x;
  const double* g = ghat + (size_t)inst * nm;
  for (int b = 0; b < 32; ++b) {
    double t = 0.0;
    for (int i = off[b] + threadIdx.x; i < off[b + 1]; i += blockDim.x) {
      const double v = g[perm[i]];
      t += v * v;
    }
    t = wave_sum(t);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
      const double e = (red[0] + red[1]) + (red[2] + red[3]);
      feats[(size_t)inst * 33 + b] = (float)log10(e * hd + 1e-300);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) feats[(size_t)inst * 33 + 32] = (float)log10(deltas[inst]);
}

// ================================================================ network ==
// 33 -> 64 -> 64 -> 1 with exact-erf GELU; FP32.
__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

constexpr int kW1 = 0, kB1 = 64 * 33, kW2 = kB1 + 64, kB2 = kW2 + 64 * 64, kW3 = kB2 + 64, kB3 = kW3 + 64,
              kNP = kB3 + 1;

// thread per sample; parameters staged in LDS
__device__ __forceinline__ float mlp_eval(const float* P, const float* x, float* h1, float* h2) {
  float a1[64];
#pragma unroll 4
  for (int o = 0; o < 64; ++o) {
    float t = P[kB1 + o];
    for (int i = 0; i < 33; ++i) t += P[kW1 + o * 33 + i] * x[i];
    if (h1) h1[o] = t;
    a1[o] = gelu_f(t);
  }
  float out = P[kB3];
  for (int o = 0; o < 64; ++o) {
    float t = P[kB2 + o];
#pragma unroll 8
    for (int i = 0; i < 64; ++i) t += P[kW2 + o * 64 + i] * a1[i];
    if (h2) h2[o] = t;
    out += P[kW3 + o] * gelu_f(t);
  }
  return out;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* params, int B, const float* X, float* out) {
  __shared__ float P[kNP];
  for (int i = threadIdx.x; i < kNP; i += blockDim.x) P[i] = params[i];
  __syncthreads();
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float x[33];
  for (int i = 0; i < 33; ++i) x[i] = X[(size_t)b * 33 + i];
  out[b] = mlp_eval(P, x, nullptr, nullptr);
}

// Per-sample forward and backward: stores a1, dH2, dH1 and the residual for the
// parameter-gradient reduction that follows.
__global__ __launch_bounds__(256) void k_mlp_sample_grad(const float* params, int B, const float* X,
                                                         const float* y, float* A1, float* DH2,
                                                         float* DH1, float* R) {
  __shared__ float P[kNP];
  for (int i = threadIdx.x; i < kNP; i += blockDim.x) P[i] = params[i];
  __syncthreads();
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float x[33], h1[64], h2[64];
  for (int i = 0; i < 33; ++i) x[i] = X[(size_t)b * 33 + i];
  const float out = mlp_eval(P, x, h1, h2);
  const float r = out - y[b];
  R[b] = r;
  const float dout = 2.0f * r / (float)B;
  float dh2[64];
  for (int o = 0; o < 64; ++o) {
    dh2[o] = dout * P[kW3 + o] * gelu_grad_f(h2[o]);
    DH2[(size_t)b * 64 + o] = dh2[o];
    A1[(size_t)b * 64 + o] = gelu_f(h1[o]);
  }
  for (int i = 0; i < 64; ++i) {
    float t = 0.0f;
    for (int o = 0; o < 64; ++o) t += dh2[o] * P[kW2 + o * 64 + i];
    DH1[(size_t)b * 64 + i] = t * gelu_grad_f(h1[i]);
  }
}

// One thread per parameter: sum over the batch in sample order (deterministic).
__global__ __launch_bounds__(256) void k_mlp_param_grad(int B, const float* X, const float* A1,
                                                        const float* DH2, const float* DH1,
                                                        const float* R, const float* params,
                                                        float* grad, float* loss) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kNP) return;
  float g = 0.0f;
  if (t < kB1) {  // W1[o][i] = sum_b DH1[b][o] X[b][i]
    const int o = t / 33, i = t - o * 33;
    for (int b = 0; b < B; ++b) g += DH1[(size_t)b * 64 + o] * X[(size_t)b * 33 + i];
  } else if (t < kW2) {
    const int o = t - kB1;
    for (int b = 0; b < B; ++b) g += DH1[(size_t)b * 64 + o];
  } else if (t < kB2) {
    const int o = (t - kW2) / 64, i = (t - kW2) - o * 64;
    for (int b = 0; b < B; ++b) g += DH2[(size_t)b * 64 + o] * A1[(size_t)b * 64 + i];
  } else if (t < kW3) {
    const int o = t - kB2;
    for (int b = 0; b < B; ++b) g += DH2[(size_t)b * 64 + o];
  } else if (t < kB3) {  // W3[o] = sum_b dout_b * gelu(h2_b[o]); gelu(h2) recovered from DH2? no: recompute
    g = 0.0f;            // filled by k_mlp_w3_grad
  } else {
    for (int b = 0; b < B; ++b) g += 2.0f * R[b] / (float)B;
  }
  grad[t] = g;
  if (t == 0) {
    float l = 0.0f;
    for (int b = 0; b < B; ++b) l += R[b] * R[b];
    *loss = l / (float)B;
  }
}

// W3 gradient needs a2 = gelu(h2): recompute h2 per sample, thread per (sample), then reduce.
__global__ __launch_bounds__(64) void k_mlp_w3_grad(const float* params, int B, const float* A1,
                                                    const float* R, float* grad) {
  // one workgroup of 64 threads: thread o accumulates sum_b dout_b gelu(h2_b[o]) in sample order
  const int o = threadIdx.x;
  float w2[64];
  for (int i = 0; i < 64; ++i) w2[i] = params[kW2 + o * 64 + i];
  const float b2 = params[kB2 + o];
  float g = 0.0f;
  for (int b = 0; b < B; ++b) {
    float t = b2;
    for (int i = 0; i < 64; ++i) t += w2[i] * A1[(size_t)b * 64 + i];
    g += (2.0f * R[b] / (float)B) * gelu_f(t);
  }
  grad[kW3 + o] = g;
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Single-instance alpha prediction: standardise features, evaluate, de-standardise.
// Thread o of one 64-lane wave owns hidden unit o of both layers.
__global__ __launch_bounds__(64) void k_predict(const float* model, const float* feats, double* alpha_out) {
  __shared__ float x[33];
  __shared__ float a1[64];
  const int o = threadIdx.x;
  if (o < 33) x[o] = (feats[o] - model[kNP + o]) / model[kNP + 33 + o];
  __syncthreads();
  float t = model[kB1 + o];
  for (int i = 0; i < 33; ++i) t += model[kW1 + o * 33 + i] * x[i];
  a1[o] = gelu_f(t);
  __syncthreads();
  float u = model[kB2 + o];
  for (int i = 0; i < 64; ++i) u += model[kW2 + o * 64 + i] * a1[i];
  float c = model[kW3 + o] * gelu_f(u);
  // sum over the wave in a fixed tree order
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
  if (o == 0) {
    const float out = c + model[kB3];
    const double l10 = (double)(out * model[kNP + 67] + model[kNP + 66]);
    alpha_out[0] = exp10(l10);
    alpha_out[1] = l10;
  }
}

// One instance on 32 workgroups, one per bin: each reduces its bin in a fixed order
// and publishes the sum; the last workgroup to finish forms the 33 features and
// runs the network.  Writes alpha_out[0] = alpha, [1] = log10 alpha.  counter[0]
// must be zero on entry and is zero again on exit.
__global__ __launch_bounds__(256) void k_feat_predict(double hd, const double* ghat, double delta, const int* perm,
                                                      const int* off, const float* model, float* feats,
                                                      double* alpha_out, double* partial, unsigned* counter) {
  __shared__ double red[4];
  __shared__ float x[33];
  __shared__ float a1[64];
  __shared__ bool s_last;
  const int b = blockIdx.x;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double t = 0.0;
  for (int i = off[b] + (int)threadIdx.x; i < off[b + 1]; i += (int)blockDim.x) {
    const double v = ghat[perm[i]];
    t += v * v;
  }
  t = wave_sum(t);
  if (lane == 0) red[wv] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) sum += red[i];
    const unsigned prev = publish_and_count(&partial[b], sum, counter);
    s_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!s_last) return;
  if (threadIdx.x < 33) {
    const int i = threadIdx.x;
    const double f = i < 32 ? log10(__hip_atomic_load(&partial[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) * hd +
                                    1e-300)
                            : log10(delta);
    feats[i] = (float)f;
    x[i] = ((float)f - model[kNP + i]) / model[kNP + 33 + i];
  }
  if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if (threadIdx.x < 64) {
    const int o = threadIdx.x;
    float u = model[kB1 + o];
    for (int i = 0; i < 33; ++i) u += model[kW1 + o * 33 + i] * x[i];
    a1[o] = gelu_f(u);
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int o = threadIdx.x;
    float u = model[kB2 + o];
    for (int i = 0; i < 64; ++i) u += model[kW2 + o * 64 + i] * a1[i];
    float c = model[kW3 + o] * gelu_f(u);
    for (int sft = 32; sft >= 1; sft >>= 1) c += __shfl_xor(c, sft, 64);
    if (o == 0) {
      const float out = c + model[kB3];
      const double l10 = (double)(out * model[kNP + 67] + model[kNP + 66]);
      alpha_out[0] = exp10(l10);
      alpha_out[1] = l10;
    }
  }
}

hipError_t launch_feat_predict(double hd, const double* ghat, double delta, const int* perm, const int* off,
                               const float* model, float* feats, double* alpha_out, double* partial,
                               unsigned* counter, hipStream_t s) {
  hipLaunchKernelGGL(k_feat_predict, dim3(32), dim3(256), 0, s, hd, ghat, delta, perm, off, model, feats,
                     alpha_out, partial, counter);
  return hipGetLastError();
}

template <bool WIDE>
__global__ __launch_bounds__(256) void k_time_general(TimeArgs a) {
  extern __shared__ c64 lds[];
  time_general_body<WIDE>(a, blockIdx.x, lds);
}

__global__ void k_tab_job(TabJob t) {
  tab_job_run(t, (long long)blockIdx.x * blockDim.x + threadIdx.x, (long long)gridDim.x * blockDim.x);
}

__global__ void k_copy_scale(const double* in, double* out, long long n, double s) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i] * s;
}

// ================================================================ launches ==
// Dynamic LDS above 64 KiB: declare the device's per-workgroup maximum once per
// kernel.  The runtime may not need (or accept) the attribute; a refusal is
// cleared here so it cannot surface later as a stale error of another call.
static void allow_big_lds(const void* f) {
  static std::mutex mu;
  static std::set<const void*> done;
  std::lock_guard<std::mutex> lk(mu);
  if (!done.insert(f).second) return;
  int dev = 0, maxlds = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, maxlds) != hipSuccess)
    (void)hipGetLastError();
}

// Workgroups of a persistent kernel over `tiles` tiles: the resident capacity of
// the device (occupancy x compute units), lowered to even out the tiles per
// workgroup.  Capacities are cached per (kernel, block, LDS, device).
static long long persistent_grid(const void* f, int threads, size_t lds, long long tiles) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, int, size_t, int>, long long> cap_of;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return tiles;
  }
  long long cap;
  {
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_tuple(f, threads, lds, dev);
    auto it = cap_of.find(key);
    if (it == cap_of.end()) {
      int cus = 0, per = 0;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, threads, lds) != hipSuccess) {
        (void)hipGetLastError();
        cus = per = 0;
      }
      it = cap_of.emplace(key, (long long)(per < 1 ? 1 : per) * (cus < 1 ? 1 : cus)).first;
    }
    cap = it->second;
  }
  if (tiles <= cap) return tiles;
  const long long rounds = (tiles + cap - 1) / cap;
  return (tiles + rounds - 1) / rounds;
}

template <class A>
static hipError_t enqueue1(const void* f, dim3 grid, dim3 block, size_t lds, hipStream_t s, const A& a,
                           NodeCtx* nc) {
  void* args[] = {const_cast<A*>(&a)};
  allow_big_lds(f);
  if (!nc) return hipLaunchKernel(f, grid, block, args, lds, s);
  hipKernelNodeParams p{};
  p.func = const_cast<void*>(f);
  p.gridDim = grid;
  p.blockDim = block;
  p.sharedMemBytes = (unsigned)lds;
  p.kernelParams = args;
  p.extra = nullptr;
  if (nc->exec) {  // same launch sequence, new arguments: update the recorded node
    if (!nc->nodes || nc->next >= nc->nodes->size()) return hipErrorInvalidValue;
    return hipGraphExecKernelNodeSetParams(nc->exec, (*nc->nodes)[nc->next++], &p);
  }
  hipGraphNode_t node;
  const hipError_t e = hipGraphAddKernelNode(&node, nc->graph, nc->has_dep ? &nc->dep : nullptr,
                                             nc->has_dep ? 1 : 0, &p);
  if (e == hipSuccess) {
    nc->dep = node;
    nc->has_dep = true;
    if (nc->nodes) nc->nodes->push_back(node);
  }
  return e;
}

hipError_t launch_dst(const DstArgs& a, long long nwg, int threads, size_t lds, hipStream_t s, NodeCtx* nc,
                      int role) {
  static const void* tab[2][3] = {
      {(const void*)&k_dst<false, 0>, (const void*)&k_dst<false, 1>, (const void*)&k_dst<false, 2>},
      {(const void*)&k_dst<true, 0>, (const void*)&k_dst<true, 1>, (const void*)&k_dst<true, 2>}};
  const void* f = tab[a.fft.wide ? 1 : 0][role < 0 ? 0 : (role > 2 ? 2 : role)];
  if (a.fft.p2) {
    f = dst_p2_fn(a.fft.p2, a.var, a.inner > 1, a.inner > 1 && p2sz::dst_pairs_aligned(a));
    if (!f) return hipErrorInvalidValue;
    allow_big_lds(f);
    nwg = persistent_grid(f, threads, lds, nwg);
  } else if (a.fft.bp2) {
    f = dst_blue_fn(a.fft.bp2);
    if (!f || threads != p2sz::blue_T(a.fft.bp2) || a.S != p2sz::blue_S(a.fft.bp2)) return hipErrorInvalidValue;
  }
  return enqueue1(f, dim3((unsigned)nwg), dim3(threads), lds, s, a, nc);
}

hipError_t launch_time(const TimeArgs& a, long long nwg, int threads, size_t lds, hipStream_t s, NodeCtx* nc) {
  const void* f = a.fft.wide ? (const void*)&k_time<true> : (const void*)&k_time<false>;
  if (a.pitch > 0 && nwg >= (1LL << 31)) return hipErrorInvalidValue;  // 32-bit tile index
  if (a.fft.p2) {  // persistent over a.ntiles tiles
    f = time_p2_fn(a.fft.p2, a.var, a.fft.kind == kRader, a.pitch > 0);
    if (!f) return hipErrorInvalidValue;
    allow_big_lds(f);
    TimeArgs b = a;
    b.ntiles = nwg;
    return enqueue1(f, dim3((unsigned)persistent_grid(f, threads, lds, nwg)), dim3(threads), lds, s, b, nc);
  } else if (a.fft.gtA) {
    f = time_gt_fn(a.fft.gtA, a.fft.gtB, a.var, a.pitch > 0);
    if (!f) return hipErrorInvalidValue;
  }
  return enqueue1(f, dim3((unsigned)nwg), dim3(threads), lds, s, a, nc);
}

hipError_t launch_time_general(const TimeArgs& a, long long nwg, size_t lds, hipStream_t s) {
  const void* f = a.fft.wide ? (const void*)&k_time_general<true> : (const void*)&k_time_general<false>;
  if (a.fft.p2) {
    f = general_p2_fn(a.fft.p2, a.var, a.fft.kind == kRader);
    if (!f) return hipErrorInvalidValue;
  }
  return enqueue1(f, dim3((unsigned)nwg), dim3(a.threads), lds, s, a, nullptr);
}

// Step (c) of the 2D variable-coefficient path (runtime engine, any N_t)
template <bool WIDE>
__global__ __launch_bounds__(256) void k_kry_time(KryTimeArgs a) {
  extern __shared__ c64 lds[];
  kry_time_body<WIDE>(a, blockIdx.x, lds);
}

hipError_t launch_kry_time(const KryTimeArgs& a, long long nwg, size_t lds, hipStream_t s) {
  if (a.S < 1 || a.lev_first < 0 || a.lev_count < 1 || a.lev_first + a.lev_count > a.Nt || nwg * 2LL * a.S < a.M)
    return hipErrorInvalidValue;
  const void* f = a.fft.wide ? (const void*)&k_kry_time<true> : (const void*)&k_kry_time<false>;
  allow_big_lds(f);
  void* args[] = {const_cast<KryTimeArgs*>(&a)};
  return hipLaunchKernel(f, dim3((unsigned)nwg), dim3(256), args, lds, s);
}

hipError_t launch_tab_job(const TabJob& t, hipStream_t s) {
  return enqueue1((const void*)&k_tab_job, dim3((unsigned)((t.Nt + 255) / 256)), dim3(256), 0, s, t, nullptr);
}

hipError_t launch_thomas(const ThomasArgs& a, long long nwg, size_t lds, hipStream_t s, NodeCtx* nc) {
  if (a.P < 1 || a.S < 1 || a.P * a.S > 256 || (a.m > 1 && (a.m + a.P - 1) / a.P > 8)) return hipErrorInvalidValue;
  return enqueue1((const void*)&k_tri1d, dim3((unsigned)nwg), dim3(a.P * a.S), lds, s, a, nc);
}

hipError_t launch_time1d(const Time1dArgs& a, long long nwg, int threads, size_t lds, hipStream_t s,
                         NodeCtx* nc) {
  const void* f = a.fft.wide ? (const void*)&k_time1d<true> : (const void*)&k_time1d<false>;
  return enqueue1(f, dim3((unsigned)nwg), dim3(threads), lds, s, a, nc);
}

hipError_t launch_row(const RowArgs& a, long long nwg, int threads, size_t lds, hipStream_t s, NodeCtx* nc) {
  return enqueue1((const void*)&k_row, dim3((unsigned)nwg), dim3(threads), lds, s, a, nc);
}

hipError_t launch_tri1d_batch(const Batch1dArgs& b, size_t lds, hipStream_t s, NodeCtx* nc) {
  const void* f = (const void*)&k_tri1d_batch;
  allow_big_lds(f);
  const long long nwg = persistent_grid(f, 256, lds, b.nitems);
  return enqueue1(f, dim3((unsigned)nwg), dim3(256), lds, s, b, nc);
}

hipError_t launch_time1d_batch(const Batch1dArgs& b, bool wide, size_t lds, hipStream_t s, NodeCtx* nc) {
  const void* f = wide ? (const void*)&k_time1d_batch<true> : (const void*)&k_time1d_batch<false>;
  allow_big_lds(f);
  const long long nwg = persistent_grid(f, 256, lds, b.nitems);
  return enqueue1(f, dim3((unsigned)nwg), dim3(256), lds, s, b, nc);
}

hipError_t launch_bisect_init(double* bstate, int count, const double* deltas, double delta_val, double tau_dp,
                              double lo, double hi, hipStream_t s) {
  hipLaunchKernelGGL(k_bisect_init, dim3((count + 255) / 256), dim3(256), 0, s, bstate, count, deltas,
                     delta_val, tau_dp, lo, hi);
  return hipGetLastError();
}

hipError_t launch_bisect_finish(const double* bstate, int count, double* alphas, int* hits, hipStream_t s) {
  hipLaunchKernelGGL(k_bisect_finish, dim3((count + 255) / 256), dim3(256), 0, s, bstate, count, alphas,
                     hits);
  return hipGetLastError();
}

hipError_t launch_features(int count, long long nm, double hd, const double* ghat, const double* deltas,
                           const int* perm, const int* off, float* feats, hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3(count), dim3(256), 0, s, nm, hd, ghat, deltas, perm, off, feats);
  return hipGetLastError();
}

hipError_t launch_predict(const float* model, const float* feats, double* alpha_out, hipStream_t s) {
  hipLaunchKernelGGL(k_predict, dim3(1), dim3(64), 0, s, model, feats, alpha_out);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* p, int B, const float* X, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_forward, dim3((B + 255) / 256), dim3(256), 0, s, p, B, X, out);
  return hipGetLastError();
}

hipError_t launch_mlp_loss_grad(const float* p, int B, const float* X, const float* y, float* grad,
                                float* loss, float* scratch, int, hipStream_t s) {
  float* A1 = scratch;
  float* DH2 = A1 + (size_t)B * 64;
  float* DH1 = DH2 + (size_t)B * 64;
  float* R = DH1 + (size_t)B * 64;
  hipLaunchKernelGGL(k_mlp_sample_grad, dim3((B + 255) / 256), dim3(256), 0, s, p, B, X, y, A1, DH2, DH1, R);
  hipLaunchKernelGGL(k_mlp_param_grad, dim3((kNP + 255) / 256), dim3(256), 0, s, B, X, A1, DH2, DH1, R, p,
                     grad, loss);
  hipLaunchKernelGGL(k_mlp_w3_grad, dim3(1), dim3(64), 0, s, p, B, A1, R, grad);
  return hipGetLastError();
}

// Allocation-free loss and gradient (for callers that cannot allocate): the per-sample
// activations a1, dH2, dH1 (64 floats each) and residuals of at most
// QBVM_NOALLOC_MAX_BATCH samples live in this file-scope array, one copy per GPU for the
// life of the process.  In host code the array's name is only a stand-in; kernels get the
// device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) float mlp_scratch[(size_t)QBVM_NOALLOC_MAX_BATCH * (64 * 3 + 1)];

static std::mutex g_mlp_scratch_mu;
static std::map<int, float*> g_mlp_scratch_addr;  // device -> address of its mlp_scratch

hipError_t mlp_scratch_address(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_mlp_scratch_mu);
  auto it = g_mlp_scratch_addr.find(dev);
  if (it == g_mlp_scratch_addr.end()) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(mlp_scratch));
    if (e != hipSuccess) return e;
    it = g_mlp_scratch_addr.emplace(dev, static_cast<float*>(ptr)).first;
  }
  *out = it->second;
  return hipSuccess;
}

hipError_t launch_mlp_loss_grad_static(const float* p, int B, const float* X, const float* y, float* grad,
                                       float* loss, hipStream_t s) {
  if (B < 1 || B > QBVM_NOALLOC_MAX_BATCH) return hipErrorInvalidValue;
  float* ptr = nullptr;
  const hipError_t e = mlp_scratch_address(&ptr);
  if (e != hipSuccess) return e;
  return launch_mlp_loss_grad(p, B, X, y, grad, loss, ptr, 0, s);
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, int step, float lr, float b1,
                       float b2, float eps, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_copy_scale(const double* in, double* out, long long n, double sc, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n, sc);
  return hipGetLastError();
}

}  // namespace qbvm
