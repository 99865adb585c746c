// Internal interface between the host executor and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "qbvm_types.hpp"

namespace qbvm {

// Optional graph target: when non-null the launch wrappers add a kernel node that
// depends on `dep` (if has_dep) instead of launching, and update `dep`.
struct NodeCtx {
  hipGraph_t graph;
  hipGraphNode_t dep;
  bool has_dep;
  // optional: the launches append their node handles here; with `exec` set they instead set
  // the parameters of the recorded nodes, in the same order, of that instantiated graph
  // (new buffers for an unchanged launch sequence)
  std::vector<hipGraphNode_t>* nodes = nullptr;
  hipGraphExec_t exec = nullptr;
  size_t next = 0;
};

// Batched 1D instances (every level): one launch per step over a device table of the
// instances' argument blocks; item w = (instance, workgroup of its own launch).
struct Batch1dArgs {
  const void* args;  // ThomasArgs[] or Time1dArgs[]
  const int* items;  // 2 ints per item: instance, workgroup
  int nitems;
};

// ---- 2D variable-coefficient Step (b) and its Step (c) (qbvm_krylov.hip) ----
hipError_t launch_krylov(const KrylovArgs& a, int step, hipStream_t s);
hipError_t launch_kry_time(const KryTimeArgs& a, long long nwg, size_t lds, hipStream_t s);

// ---- Bluestein sine passes on a power-of-two core (qbvm_blue.hip) ----------
const void* dst_blue_fn(int P);  // kernel of core length P (64 .. 4096), else null

// ---- launch wrappers (defined in qbvm_kernels.hip) ------------------------
void upload_radix_roots(const c64* roots, int count);  // constant-memory roots per device
hipError_t launch_dst(const DstArgs& a, long long nwg, int threads, size_t lds, hipStream_t s,
                      NodeCtx* nc = nullptr, int role = 0);
hipError_t launch_time(const TimeArgs& a, long long nwg, int threads, size_t lds, hipStream_t s,
                       NodeCtx* nc = nullptr);
// general right-hand side time kernel (256 threads) and the per-solve table kernel
hipError_t launch_time_general(const TimeArgs& a, long long nwg, size_t lds, hipStream_t s);
hipError_t launch_tab_job(const TabJob& t, hipStream_t s);
// plane pass (qbvm_plane.hip): x_2 and x_1 transforms of every plane, sine length 256
hipError_t launch_plane(const PlaneArgs& a, int var, hipStream_t s, NodeCtx* nc = nullptr);
hipError_t launch_thomas(const ThomasArgs& a, long long nwg, size_t lds, hipStream_t s, NodeCtx* nc = nullptr);
hipError_t launch_time1d(const Time1dArgs& a, long long nwg, int threads, size_t lds, hipStream_t s,
                         NodeCtx* nc = nullptr);
hipError_t launch_row(const RowArgs& a, long long nwg, int threads, size_t lds, hipStream_t s,
                      NodeCtx* nc = nullptr);
hipError_t launch_tri1d_batch(const Batch1dArgs& b, size_t lds, hipStream_t s, NodeCtx* nc);
hipError_t launch_time1d_batch(const Batch1dArgs& b, bool wide, size_t lds, hipStream_t s, NodeCtx* nc);
hipError_t launch_bisect_init(double* bstate, int count, const double* deltas, double delta_val,
                              double tau_dp, double lo, double hi, hipStream_t s);
// 32 workgroups; partial holds >= 32 doubles; counter[0] is zero on entry and exit
hipError_t launch_feat_predict(double hd, const double* ghat, double delta, const int* perm, const int* off,
                               const float* model, float* feats, double* alpha_out, double* partial,
                               unsigned* counter, hipStream_t s);
hipError_t launch_bisect_finish(const double* bstate, int count, double* alphas, int* hits,
                                hipStream_t s);
hipError_t launch_features(int count, long long nm, double hd, const double* ghat,
                           const double* deltas, const int* perm, const int* off, float* feats,
                           hipStream_t s);
hipError_t launch_predict(const float* model, const float* feats, double* alpha_out,
                          hipStream_t s);
hipError_t launch_mlp_forward(const float* p, int B, const float* X, float* out, hipStream_t s);
hipError_t launch_mlp_loss_grad(const float* p, int B, const float* X, const float* y,
                                float* grad, float* loss, float* scratch, int nscratch_wg,
                                hipStream_t s);
// same kernels on the file-scope scratch array (B <= QBVM_NOALLOC_MAX_BATCH); allocates nothing
hipError_t launch_mlp_loss_grad_static(const float* p, int B, const float* X, const float* y,
                                       float* grad, float* loss, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, int step, float lr,
                       float b1, float b2, float eps, hipStream_t s);
hipError_t launch_copy_scale(const double* in, double* out, long long n, double s, hipStream_t st);

}  // namespace qbvm
