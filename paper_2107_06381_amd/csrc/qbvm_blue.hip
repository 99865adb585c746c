// Bluestein sine passes on the compile-time power-of-two engine (qbvm_bodies_blue.hpp),
// one kernel per core length P.
#include "qbvm_internal.hpp"
#include "qbvm_bodies_blue.hpp"

namespace qbvm {

template <int P>
__global__ __launch_bounds__(p2sz::blue_T(P)) void k_dst_blue(DstArgs a) {
  extern __shared__ c64 lds[];
  dst_blue_body<P>(a, blockIdx.x, lds);
}

const void* dst_blue_fn(int P) {
  switch (P) {
    case 64: return (const void*)&k_dst_blue<64>;
    case 128: return (const void*)&k_dst_blue<128>;
    case 256: return (const void*)&k_dst_blue<256>;
    case 512: return (const void*)&k_dst_blue<512>;
    case 1024: return (const void*)&k_dst_blue<1024>;
    case 2048: return (const void*)&k_dst_blue<2048>;
    case 4096: return (const void*)&k_dst_blue<4096>;
    default: return nullptr;
  }
}

}  // namespace qbvm
