// Plain data types shared by the host planner, the kernels and the CPU build of
// the kernel bodies (no HIP runtime dependency).
#pragma once

#include <cstdint>

namespace qbvm {

// Complex FP64 value; 16-byte aligned so LDS and global accesses are b128.
struct alignas(16) c64 {
  double re, im;
};

constexpr int kMaxStages = 16;
constexpr int kElemsPerThread = 16;   // complex values a thread holds in one FFT stage
constexpr int kMaxOddRadixWide = 47;  // largest odd prime radix of the wide kernel variant
constexpr int kMaxOddRadixNarrow = 7; // largest odd prime radix of the narrow variant

// One Stockham stage on a core transform of length nc: radix R, ns = product of the
// radices already applied, twiddle of element r of butterfly j: tw[(j % ns) * r * twstride].
struct FftStage {
  int radix;
  int ns;
  int twstride;
};

enum FftKind : int { kStockham = 0, kRader = 1, kBluestein = 2 };

// Forward DFT X_k = sum_j x_j exp(-2 pi i jk/n) of logical length n, computed on a
// core Stockham transform of length nc (= n, n-1 for Rader, P for Bluestein).
struct FftPlanDev {
  int n;
  int kind;
  int nc;
  int nstages;
  int wide;  // 1 if some stage radix exceeds the narrow variant
  FftStage st[kMaxStages];
  const c64* tw;     // nc values exp(-2 pi i k/nc)
  const c64* kspec;  // Rader: FFT_{n-1}(b)/(n-1); Bluestein: FFT_P(b)/P
  const c64* chirp;  // Bluestein: exp(i pi (k^2 mod 2n)/n), k < n
  const int* rin;    // Rader: rin[j] = q with g^q = j (mod n), j = 1..n-1
  const int* rout;   // Rader: rout[k] = p with g^{-p} = k (mod n), k = 1..n-1
  const int* gfwd;   // Rader: gfwd[q] = g^q mod n, q < n-1
  const int* ginvt;  // Rader: ginvt[p] = g^{-p} mod n, p < n-1
  int p2;            // core length if it has a compile-time power-of-two kernel (64..4096), else 0
  int gtA, gtB;      // n = gtA * gtB handled by the compile-time Good-Thomas time kernel (else 0)
  int bp2;           // sine tables in the symmetric Bluestein form of the compile-time sine
                     // kernel: its power-of-two core (kspec holds 2 bp2 values), else 0
};

// Per-solve scalars derived from (alpha, variant, tau).
struct SolveScalars {
  double logabsw;   // ln|omega|
  double f0s;       // f0 = f0s * g_delta
  double alpha;     // the regularisation parameter itself (kernels derive the two above from it)
};

// Arguments of the spectral time kernel: one tile of sine modes x all N_t levels.
struct TimeArgs {
  int Nt;
  int d;
  int m;
  int S;              // complex signals per workgroup (2 S modes)
  long long nmodes;   // m^d
  long long ystride;  // distance between levels in y
  int lev_first;      // first level written
  int lev_count;      // number of levels written
  int lev_dst0;       // level index in y of lev_first (0 when writing one level)
  double tau;
  SolveScalars sc;
  const double* mu1d;   // m eigenvalues of the 1D stencil
  const double* ghat;   // nmodes sine coefficients of g_delta
  double* y;
  const double* alpha_dev;  // if non-null, alpha is read from here (device-side choice)
  int variant;
  int threads;  // workgroup size of the launch
  int var;      // power-of-two kernel variant
  long long pitch;   // > 0: y rows of m modes padded to this pitch (tiles never straddle rows)
  int tiles_per_row;
  long long ntiles;  // tiles of the launch (set at launch; persistent kernels stride over them)
  int tw_lds;        // runtime engine: twiddles copied into LDS after the per-signal tables
  const c64* tabs;   // optional: [N_t] d_j/tau then [N_t] f0s/N_t gamma_l^{-1} for this solve
  const double* fgen; // general right-hand side in the sine basis, levels ystride apart (general solve)
  FftPlanDev fft;
};

// Per-solve time tables d_j/tau and f0s/N_t gamma_l^{-1} (j, l < N_t), computed as side
// work by the workgroups of a kernel that runs before the time transform.
struct TabJob {
  c64* out;                 // [N_t] d_j/tau then [N_t] f0s/N_t gamma_l^{-1}; nullptr: no job
  int Nt;
  int variant;
  double tau;
  double alpha;
  const double* alpha_dev;  // if non-null, alpha is read from here
  int general;              // 1: [N_t] gamma_l^{-1}/N_t (no f0s), then [N_t] gamma_t as well
};

// Sine-transform pass: data viewed as [outer][len][inner]; transform along len.
// Rows pass (inner == 1): line l is in[l*in_pitch + k], k < len, written to out[l*out_pitch + k].
// Columns pass (inner > 1): point k of column c in block o is at o*ostride + k*kstride + c
// (the same in input and output); column c is valid iff c < inner and, when colmod > 0,
// c % colmod < colvalid (padded rows).
struct DstArgs {
  const double* in;
  double* out;
  long long outer;
  long long inner;
  int len;     // m
  int S;       // complex signals per workgroup (2 S lines)
  long long tiles_per_outer;  // ceil(inner / (2S)) when inner > 1
  double scale;
  int threads;   // workgroup size of the launch
  int var;       // power-of-two kernel variant
  long long in_pitch, out_pitch;
  long long kstride, ostride;
  int colmod, colvalid;
  TabJob tab;  // optional side work (power-of-two kernels)
  int tw_lds;  // runtime engine: twiddles copied into LDS after the side slots
  FftPlanDev fft;
};

// Plane pass (d >= 2): the x_2 and x_1 sine transforms of every plane [m][in_pitch] of
// `in` (planes in_plane apart; columns m .. in_pitch-1 are padding), written unpadded
// to `out` (planes out_plane = m*m apart).
struct PlaneArgs {
  const double* in;
  double* out;
  long long planes;
  long long in_plane;
  long long out_plane;
  int m;
  int in_pitch;  // even
  double scale;  // orthonormal DST-I factor of one transform, sqrt(2/(m+1)), halved (see k_dst)
  FftPlanDev fft;  // length 2(m+1)
};

// 1D paper-order Step (b): complex Thomas per shift j.
struct ThomasArgs {
  int Nt;
  int m;
  double tau;
  double h;
  SolveScalars sc;
  const double* alpha_dev;  // if non-null, alpha is read from here
  int variant;
  const double* g;   // m
  c64* s2;           // [Nt][m] solution of (d_j/tau - Lap_h) s = f0, one row per shift
  int P;             // lanes per system (each holds a chunk of at most 8 rows)
  int S;             // systems per workgroup
  TabJob tab;        // optional side work: the per-solve tables of the time kernel
  // optional spatial operator A in place of -Lap_h (op_di == nullptr: the Dirichlet
  // stencil): A[i][i-1] = op_lo[i-1], A[i][i] = op_di[i], A[i][i+1] = op_up[i]
  const double* op_lo;
  const double* op_di;
  const double* op_up;
};

// 2D/3D Step (b) with the operator A = -div(kappa grad u) ((2d+1)-point conservative form,
// kappa at the cell faces): the shifted systems (s_j I + A) w_j = g, s_j = d_j/tau, for
// j < H = ceil(N_t/2) (the others are their conjugates), by batched conjugate orthogonal
// conjugate gradients preconditioned with the constant-coefficient solve
// (s_j I + kbar (-Lap_h))^{-1} in the sine basis.  Complex vectors are [2][H][M] doubles
// (real block, then imaginary block), M = m^d points, x_1 fastest.
constexpr int kKryThreads = 256;       // lanes per workgroup of the Krylov kernels
constexpr int kKryPointsPerLane = 4;   // points per lane (workgroup: 1024 points of one system)
// dynamic LDS of the operator kernel: the workgroup's points and one grid row either side,
// plus the static reduction buffer
constexpr size_t kry_apply_lds(int m) {
  return 16 * ((size_t)kKryPointsPerLane * kKryThreads + 2 * (size_t)m);
}
constexpr int kKryMaxM = (int)((160 * 1024 - 16 * kKryThreads) / 16 - kKryPointsPerLane * kKryThreads) / 2;
enum KryStep { kKryInit = 0, kKryApply, kKryUpdate, kKryPrecond, kKryScalars };
struct KrylovArgs {
  int d;          // 2 or 3
  int m;
  int H;
  int nblk;       // workgroups per system
  int ppt;        // points per lane
  long long M;
  double ih2;     // 1/h^2
  double kbar;    // preconditioner coefficient
  double tol2;    // converged when |r_j|^2 <= tol2
  int init;       // scalars kernel: first call (no residual partial sums yet)
  const double* kx;    // [m^(d-2)][m][m+1] faces between x_1 neighbours
  const double* ky;    // [m^(d-2)][m+1][m] faces between x_2 neighbours
  const double* kz;    // 3D: [m+1][m][m] faces between x_3 neighbours
  const double* mu1d;  // eigenvalues of the 1D Dirichlet stencil
  const c64* shift;    // [N_t] d_j/tau (per-solve table)
  const double* g;     // right-hand side, M
  double* x;
  double* r;
  double* z;
  const double* pin;   // search direction of the previous iteration
  double* pout;        // search direction of this iteration
  double* q;
  double* part;        // [3][H][nblk][2] partial sums: sigma, |r|^2, rho
  double* sys;         // [H][8] per-system scalars (see qbvm_bodies_krylov.hpp)
};

// Step (c) for the 2D/3D operator path: y_l = Re(gamma_l^{-1}/N_t sum_j theta^{-jl} w_j) per
// point, w_j for j >= H taken as conj(w_{N_t-1-j}); two points share one transform.
struct KryTimeArgs {
  int Nt;
  int H;
  int S;
  int lev_first, lev_count;
  long long M;
  const double* w;     // [2][H][M]
  const c64* gi;       // [N_t] f0s/N_t gamma_l^{-1} (per-solve table)
  double* y;           // lev_count levels of M
  FftPlanDev fft;      // length N_t (runtime engine)
};

// 1D Step (c) from the Thomas output: inverse DFT per spatial point.
struct Time1dArgs {
  int Nt;
  int m;
  int S;
  int lev_first, lev_count;
  long long ystride;
  SolveScalars sc;
  const double* alpha_dev;
  int variant;
  double tau;
  const c64* s2;
  double* y;
  const c64* gitab;  // optional per-solve table ([N_t] d_j/tau, [N_t] gamma_l^{-1}/N_t); else in LDS
  FftPlanDev fft;
};

// One level of Step (c) computed directly (one DFT row per sine mode), with
// optional output of the mode amplitudes and of the squared misfit to ghat.
struct RowArgs {
  int Nt;
  int d;
  int m;
  int level;
  int count;          // instances (batched label generation), each nmodes modes
  long long nmodes;
  double tau;
  double hd;          // h^d
  int variant;
  const double* mu1d;
  const double* ghat;     // count * nmodes
  double* yrow;           // optional output count * nmodes
  double* partial;        // per-workgroup partial sums (count * wg_per_inst)
  unsigned int* counter;  // per-instance completion counters
  int wg_per_inst;
  // alpha source: fixed value, or per-instance device-side bisection state
  double alpha;
  const double* alpha_dev;  // if non-null (mode 0), alpha is read from here
  double* bstate;         // if non-null: per instance {lo, hi, target, D, alpha, it, hit, pad}
  int mode;               // 0: fixed alpha (D to dout); 1: bisection step; 2: endpoint check
  double* dout;           // per-instance D (device)
  // optional result mailbox in mapped host memory (instance 0 only): [1] alpha, [2] D,
  // [3] iterations and [4] bracket flag of report_bs (if set), then [0] = host_seq
  double* host_out;
  const double* report_bs;
  double host_seq;
};

// Bisection state layout (doubles per instance).
constexpr int kBState = 8;  // lo, hi, target, D, alpha, iters, hit, done

}  // namespace qbvm
