// Minimal stand-ins for the HIP device model so the kernel bodies compile as
// plain C++: one std::thread per lane, a std::barrier for __syncthreads, and the
// LDS block as an exactly sized heap buffer (so AddressSanitizer sees overruns).
#pragma once

#include <barrier>
#include <cmath>

#define __device__
#define __global__
#define __host__
#define __forceinline__ inline
#define __constant__
#define __launch_bounds__(x)

struct EmuDim {
  unsigned x = 0, y = 0, z = 0;
};
inline thread_local EmuDim threadIdx;
inline thread_local EmuDim blockDim;
inline thread_local EmuDim blockIdx;
inline thread_local EmuDim gridDim;
inline std::barrier<>* g_emu_barrier = nullptr;

inline void __syncthreads() { g_emu_barrier->arrive_and_wait(); }

inline void sincospi(double x, double* s, double* c) {
  const long double a = 3.141592653589793238462643383279502884L * (long double)x;
  *s = (double)sinl(a);
  *c = (double)cosl(a);
}
inline double exp10(double x) { return std::pow(10.0, x); }
// HIP's integer min of device code
inline int min(int a, int b) { return b < a ? b : a; }
inline long long min(long long a, long long b) { return b < a ? b : a; }
// the hardware reciprocal estimate, exact here (the bodies refine it by Newton steps)
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
// every lane of the emulated wave holds the same value where the bodies use this
#define __builtin_amdgcn_readfirstlane(x) (x)
// the bodies' optimisation barrier, on a general-purpose register here
#define QBVM_OPAQUE(x) asm volatile("" : "+r"(x))
