// Kernels of the 2D/3D variable-coefficient Step (b): batched preconditioned conjugate
// orthogonal conjugate gradients over the shifted systems (its Step (c) kernel runs on the
// runtime FFT engine and lives with that engine's constant tables in qbvm_kernels.hip).
#include "qbvm_internal.hpp"
#include "qbvm_bodies_krylov.hpp"

namespace qbvm {

__global__ __launch_bounds__(kKryThreads) void k_kry_init(KrylovArgs a) { kry_init_body(a, blockIdx.x); }

__global__ __launch_bounds__(kKryThreads) void k_kry_apply(KrylovArgs a) {
  __shared__ c64 red[kKryThreads];
  extern __shared__ c64 pl[];
  kry_apply_body(a, blockIdx.x, red, pl);
}

__global__ __launch_bounds__(kKryThreads) void k_kry_update(KrylovArgs a) {
  __shared__ c64 red[kKryThreads];
  kry_update_body(a, blockIdx.x, red);
}

__global__ __launch_bounds__(kKryThreads) void k_kry_precond(KrylovArgs a) {
  __shared__ c64 red[kKryThreads];
  kry_precond_body(a, blockIdx.x, red);
}

__global__ __launch_bounds__(kKryThreads) void k_kry_scalars(KrylovArgs a) {
  __shared__ c64 red[kKryThreads];
  kry_scalars_body(a, blockIdx.x, red);
}

hipError_t launch_krylov(const KrylovArgs& a, int step, hipStream_t s) {
  if (a.H < 1 || a.nblk < 1 || a.ppt < 1 || (a.d != 2 && a.d != 3) || (a.d == 3 && !a.kz) ||
      a.M != (long long)a.m * a.m * (a.d == 3 ? a.m : 1) ||
      (long long)a.nblk * a.ppt * kKryThreads < a.M)
    return hipErrorInvalidValue;
  const void* f = nullptr;
  unsigned grid = (unsigned)((long long)a.H * a.nblk);
  switch (step) {
    case kKryInit: f = (const void*)&k_kry_init; break;
    case kKryApply: f = (const void*)&k_kry_apply; break;
    case kKryUpdate: f = (const void*)&k_kry_update; break;
    case kKryPrecond: f = (const void*)&k_kry_precond; break;
    case kKryScalars:
      f = (const void*)&k_kry_scalars;
      grid = (unsigned)a.H;
      break;
    default: return hipErrorInvalidValue;
  }
  size_t lds = 0;
  if (step == kKryApply) {
    lds = kry_apply_lds(a.m);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    if (lds > 64 * 1024) {
      const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
  }
  void* args[] = {const_cast<KrylovArgs*>(&a)};
  return hipLaunchKernel(f, dim3(grid), dim3(kKryThreads), args, lds, s);
}

}  // namespace qbvm
