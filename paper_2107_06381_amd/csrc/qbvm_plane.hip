// gfx950 plane pass of the solve pipeline (d >= 2, sine length 2(m+1) = 256): the x_2
// and x_1 orthonormal sine transforms of every [m][P1] plane of the level workspace in
// one kernel (see dst_plane_p2_body), in place of a columns pass and a rows pass.  Each
// plane is read once and written once: 16 bytes per unknown instead of 32.
#include "qbvm_internal.hpp"
#include "qbvm_bodies_p2.hpp"
#include "qbvm_p2_sizes.hpp"

#include <map>
#include <mutex>
#include <tuple>

namespace qbvm {

template <int N, int V>
__global__ __launch_bounds__(p2sz::plane_T(V)) void k_dst_plane_p2(PlaneArgs a) {
  extern __shared__ c64 lds[];
  dst_plane_p2_body<N, V>(a, blockIdx.x, gridDim.x, lds);
}

// Resident workgroups of the plane kernel on the current device (one per CU at its LDS
// size), cached per device; the dynamic-LDS limit is raised once per device.
static hipError_t plane_grid(const void* f, int threads, size_t lds, long long planes, long long* nwg) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, int>, long long> cap_of;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cap_of.find(std::make_tuple(f, dev));
  if (it == cap_of.end()) {
    int maxlds = 0, cus = 0, per = 0;
    e = hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    if ((size_t)maxlds < lds) return hipErrorInvalidValue;
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, maxlds);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, threads, lds);
    if (e != hipSuccess) return e;
    it = cap_of.emplace(std::make_tuple(f, dev), (long long)(per < 1 ? 1 : per) * (cus < 1 ? 1 : cus)).first;
  }
  *nwg = planes < it->second ? planes : it->second;
  return hipSuccess;
}

hipError_t launch_plane(const PlaneArgs& a, int var, hipStream_t s, NodeCtx* nc) {
  if (a.fft.p2 != 256 || !p2sz::plane_valid(256, var) || a.in_pitch != p2sz::plane_pitch(256) || a.m != 127)
    return hipErrorInvalidValue;
  static const void* fns[p2sz::kPlaneVariants] = {(const void*)&k_dst_plane_p2<256, 0>,
                                                  (const void*)&k_dst_plane_p2<256, 1>,
                                                  (const void*)&k_dst_plane_p2<256, 2>};
  const void* f = fns[var];
  const int threads = p2sz::plane_T(var);
  const size_t lds = p2sz::plane_lds(256, var);
  long long nwg = 0;
  hipError_t e = plane_grid(f, threads, lds, a.planes, &nwg);
  if (e != hipSuccess || nwg < 1) return e != hipSuccess ? e : hipErrorInvalidValue;
  void* args[] = {const_cast<PlaneArgs*>(&a)};
  if (!nc) return hipLaunchKernel(f, dim3((unsigned)nwg), dim3(threads), args, lds, s);
  hipKernelNodeParams p{};
  p.func = const_cast<void*>(f);
  p.gridDim = dim3((unsigned)nwg);
  p.blockDim = dim3(threads);
  p.sharedMemBytes = (unsigned)lds;
  p.kernelParams = args;
  p.extra = nullptr;
  if (nc->exec) {  // same launch sequence, new arguments: update the recorded node
    if (!nc->nodes || nc->next >= nc->nodes->size()) return hipErrorInvalidValue;
    return hipGraphExecKernelNodeSetParams(nc->exec, (*nc->nodes)[nc->next++], &p);
  }
  hipGraphNode_t node;
  e = hipGraphAddKernelNode(&node, nc->graph, nc->has_dep ? &nc->dep : nullptr, nc->has_dep ? 1 : 0, &p);
  if (e == hipSuccess) {
    nc->dep = node;
    nc->has_dep = true;
    if (nc->nodes) nc->nodes->push_back(node);
  }
  return e;
}

}  // namespace qbvm
