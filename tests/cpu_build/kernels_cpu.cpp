// CPU build of the solve-path kernel bodies and of the launch schedule, for the
// host-side tests: indexing is checked by AddressSanitizer, results against the
// oracle.  Usage:
//   kernels_cpu fft   n S in.bin out.bin          (S signals, signal-major complex)
//   kernels_cpu solve d m n L T alpha variant in.bin out.bin [var_rows var_cols var_time [padded [plane]]]
//       (plane: 0 = separate x_2 / x_1 passes, v + 1 = plane-pass variant v)
//   kernels_cpu dst   d m batch in.bin out.bin [var_rows var_cols input]
//   kernels_cpu general d m n L T alpha variant f.bin out.bin [padded var_gen]   (general right-hand side)
//   kernels_cpu opdiff d m n L T alpha variant g.bin out.bin kx.bin ky.bin kz.bin tol max_iter stats.bin
//       (2D/3D operator -div(kappa grad u): batched preconditioned COCG and Step (c), every
//       level; kz.bin unused for d = 2; stats.bin: iterations, largest relative residual,
//       breakdowns as three doubles)
//   kernels_cpu solveop m n L T alpha variant in.bin out.bin op.bin level   (1D, tridiagonal operator;
//       op.bin: lower[m-1] diag[m] upper[m-1]; level -1: every level, else that level only)
#include "hip_cpu_shim.hpp"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "../../paper_2107_06381_amd/csrc/qbvm_bodies_p2.hpp"
#include "../../paper_2107_06381_amd/csrc/qbvm_bodies_blue.hpp"
#include "../../paper_2107_06381_amd/csrc/qbvm_bodies_gt.hpp"
#include "../../paper_2107_06381_amd/csrc/qbvm_bodies_krylov.hpp"
#include "../../paper_2107_06381_amd/csrc/qbvm_fft_plan.hpp"
#include "../../paper_2107_06381_amd/csrc/qbvm_schedule.hpp"

namespace qbvm {
c64 c_root[2080];
}
using namespace qbvm;
using sched::Launch;

template <class F>
static void run_grid(long long nwg, int T, size_t lds_bytes, F body) {
  std::barrier<> bar(T);
  g_emu_barrier = &bar;
  char* lds = new char[lds_bytes > 0 ? lds_bytes : 1];
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t)
    th.emplace_back([&, t] {
      threadIdx.x = t;
      blockDim.x = T;
      gridDim.x = (unsigned)nwg;
      for (long long wg = 0; wg < nwg; ++wg) {
        blockIdx.x = (unsigned)wg;
        body(wg, reinterpret_cast<c64*>(lds));
        bar.arrive_and_wait();
      }
    });
  for (auto& x : th) x.join();
  delete[] lds;
  g_emu_barrier = nullptr;
}

struct Tables {
  plan::HostFft h;
  FftPlanDev dev;
};

// sine: the tables of a sine transform (symmetric Bluestein form for the compile-time kernel)
static Tables make_tables(int n, bool sine = false) {
  Tables t;
  std::string err;
  if (!plan::build_tables(n, t.h, err, sine)) {
    fprintf(stderr, "plan failed: %s\n", err.c_str());
    exit(3);
  }
  t.dev = t.h.dev;
  t.dev.tw = t.h.tw.data();
  t.dev.kspec = t.h.kspec.empty() ? nullptr : t.h.kspec.data();
  t.dev.chirp = t.h.chirp.empty() ? nullptr : t.h.chirp.data();
  t.dev.rin = t.h.rin.empty() ? nullptr : t.h.rin.data();
  t.dev.rout = t.h.rout.empty() ? nullptr : t.h.rout.data();
  t.dev.gfwd = t.h.gfwd.empty() ? nullptr : t.h.gfwd.data();
  t.dev.ginvt = t.h.ginvt.empty() ? nullptr : t.h.ginvt.data();
  return t;
}

static std::vector<char> read_file(const char* path) {
  FILE* f = fopen(path, "rb");
  if (!f) exit(4);
  fseek(f, 0, SEEK_END);
  long n = ftell(f);
  fseek(f, 0, SEEK_SET);
  std::vector<char> b(n);
  if (n && fread(b.data(), 1, n, f) != (size_t)n) exit(4);
  fclose(f);
  return b;
}

static void write_file(const char* path, const void* p, size_t n) {
  FILE* f = fopen(path, "wb");
  if (!f || fwrite(p, 1, n, f) != n) exit(5);
  fclose(f);
}

template <bool W>
static void fft_signals(const Tables& t, int S, const c64* in, c64* out) {
  const FftPlanDev& p = t.dev;
  const size_t lds = sizeof(c64) * ((size_t)S * p.nc + 2 * S);
  run_grid(1, 256, lds, [&](long long, c64* L) {
    c64* buf = L;
    c64* side = L + (size_t)S * p.nc;
    for (int e = threadIdx.x; e < S * p.n; e += blockDim.x) {
      const int j = e / S, s = e - j * S;
      const int pos = fft_in_pos(p, j);
      if (pos < 0) side[s] = in[(size_t)s * p.n + j];
      else buf[(size_t)pos * S + s] = in[(size_t)s * p.n + j];
    }
    __syncthreads();
    if (p.kind == kBluestein) fft_bluestein_prep(buf, S, p);
    fft_run<W>(buf, S, p, side);
    for (int e = threadIdx.x; e < S * p.n; e += blockDim.x) {
      const int k = e / S, s = e - k * S;
      out[(size_t)s * p.n + k] = fft_out(buf, S, p, s, k, side);
    }
  });
}

static sched::Geom geom(int d, int m, int n, double L, double T, const Tables& tt, const Tables& st,
                        const std::vector<double>& mu) {
  sched::Geom g{};
  g.d = d;
  g.m = m;
  g.n = n;
  g.Nt = n + 1;
  g.h = L / (m + 1);
  g.tau = T / n;
  g.nmodes = 1;
  for (int i = 0; i < d; ++i) g.nmodes *= m;
  g.tfft = tt.dev;
  g.sfft = st.dev;
  g.S_time = plan::signals_for(tt.dev.nc);
  g.S_dst = plan::signals_for(st.dev.nc);
  g.mu1d = mu.data();
  return g;
}

#define P2_DISPATCH(N, CALL)                       \
  switch (N) {                                    \
    case 64: { constexpr int NN = 64; CALL; break; }     \
    case 128: { constexpr int NN = 128; CALL; break; }   \
    case 256: { constexpr int NN = 256; CALL; break; }   \
    case 512: { constexpr int NN = 512; CALL; break; }   \
    case 1024: { constexpr int NN = 1024; CALL; break; } \
    case 2048: { constexpr int NN = 2048; CALL; break; } \
    case 4096: { constexpr int NN = 4096; CALL; break; } \
    default: exit(9);                              \
  }

template <int N, int V>
static void dst_p2_nv(const Launch<DstArgs>& Lz) {
  if constexpr (p2sz::dst_valid(N, V)) {
    const DstArgs& A = Lz.args;
    constexpr int E = p2sz::dst_E(V), S = p2sz::dst_S(N, V);
    constexpr int TWL = p2sz::dst_tw_mode(N, V);
    // persistent bodies on a small grid, so every workgroup walks several tiles
    const long long G = Lz.nwg < 3 ? Lz.nwg : 3;
    if (A.inner > 1 && p2sz::dst_pairs_aligned(A))
      run_grid(G, A.threads, Lz.lds, [&](long long wg, c64* l) { dst_cols_p2_body<N, E, S, true, TWL>(A, wg, G, l); });
    else if (A.inner > 1)
      run_grid(G, A.threads, Lz.lds, [&](long long wg, c64* l) { dst_cols_p2_body<N, E, S, false, TWL>(A, wg, G, l); });
    else
      run_grid(G, A.threads, Lz.lds, [&](long long wg, c64* l) { dst_rows_p2_body<N, E, S, TWL>(A, wg, G, l); });
  } else {
    exit(11);
  }
}

template <int N>
static void dst_p2_n(const Launch<DstArgs>& Lz) {
  switch (Lz.args.var) {
    case 0: dst_p2_nv<N, 0>(Lz); break;
    case 1: dst_p2_nv<N, 1>(Lz); break;
    case 2: dst_p2_nv<N, 2>(Lz); break;
    case 3: dst_p2_nv<N, 3>(Lz); break;
    case 4: dst_p2_nv<N, 4>(Lz); break;
    case 5: dst_p2_nv<N, 5>(Lz); break;
    case 6: dst_p2_nv<N, 6>(Lz); break;
    case 7: dst_p2_nv<N, 7>(Lz); break;
    default: exit(12);
  }
}

template <int N, int V>
static void time_p2_nv(const Launch<TimeArgs>& t) {
  if constexpr (p2sz::time_valid(N, V)) {
    const TimeArgs& A = t.args;
    constexpr int E = p2sz::time_E(V), S = p2sz::time_S(N, V);
    constexpr bool PAD = p2sz::time_pad(V);
    // persistent body on a small grid, so every workgroup walks several tiles
    TimeArgs B = A;
    B.ntiles = t.nwg;
    const long long G = t.nwg < 3 ? t.nwg : 3;
    auto run = [&](auto rader, auto pair) {
      run_grid(G, A.threads, t.lds, [&](long long wg, c64* l) {
        time_p2_body<N, E, S, decltype(rader)::value, PAD, decltype(pair)::value>(B, wg, G, l);
      });
    };
    if (A.fft.kind == kRader) {
      if (A.pitch > 0) run(std::true_type{}, std::true_type{});
      else run(std::true_type{}, std::false_type{});
    } else {
      if (A.pitch > 0) run(std::false_type{}, std::true_type{});
      else run(std::false_type{}, std::false_type{});
    }
  } else {
    exit(13);
  }
}

template <int N>
static void time_p2_n(const Launch<TimeArgs>& t) {
  switch (t.args.var) {
    case 0: time_p2_nv<N, 0>(t); break;
    case 1: time_p2_nv<N, 1>(t); break;
    case 2: time_p2_nv<N, 2>(t); break;
    case 3: time_p2_nv<N, 3>(t); break;
    case 4: time_p2_nv<N, 4>(t); break;
    case 5: time_p2_nv<N, 5>(t); break;
    default: exit(14);
  }
}

#define P2_SWITCH(N, F, ARG)                         \
  switch (N) {                                       \
    case 64: F<64>(ARG); break;                      \
    case 128: F<128>(ARG); break;                    \
    case 256: F<256>(ARG); break;                    \
    case 512: F<512>(ARG); break;                    \
    case 1024: F<1024>(ARG); break;                  \
    case 2048: F<2048>(ARG); break;                  \
    case 4096: F<4096>(ARG); break;                  \
    default: exit(9);                                \
  }

static void run_time_fast(const Launch<TimeArgs>& t) {
  const TimeArgs& A = t.args;
  if (A.fft.gtA == 3 && A.fft.gtB == 43) {
    auto run = [&](auto v, auto pair) {
      constexpr int V = decltype(v)::value;
      run_grid(t.nwg, A.threads, t.lds, [&](long long wg, c64* l) {
        time_gt_body<3, 43, p2sz::gt_S(V), p2sz::gt_KC(V), decltype(pair)::value, p2sz::gt_rader(V)>(A, wg, l);
      });
    };
    auto runv = [&](auto v) {
      if (A.pitch > 0) run(v, std::true_type{});
      else run(v, std::false_type{});
    };
    switch (A.var) {
      case 0: runv(std::integral_constant<int, 0>{}); break;
      case 1: runv(std::integral_constant<int, 1>{}); break;
      case 2: runv(std::integral_constant<int, 2>{}); break;
      default: runv(std::integral_constant<int, 3>{}); break;
    }
    return;
  }
  if (!A.fft.p2) exit(15);
  P2_SWITCH(A.fft.p2, time_p2_n, t)
}

template <int N, int V>
static void general_p2_nv(const Launch<TimeArgs>& t) {
  if constexpr (p2sz::time_general_valid(N, V)) {
    const TimeArgs& A = t.args;
    constexpr int E = p2sz::time_E(V), S = p2sz::time_S(N, V);
    constexpr bool PAD = p2sz::time_pad(V);
    if (A.threads != p2sz::time_T(V)) exit(19);
    if constexpr (N == 256) {
      if (A.fft.kind == kRader) {
        run_grid(t.nwg, A.threads, t.lds, [&](long long wg, c64* l) { time_general_p2_body<N, E, S, true, PAD>(A, wg, l); });
        return;
      }
    }
    if (A.fft.kind == kRader) exit(13);
    run_grid(t.nwg, A.threads, t.lds, [&](long long wg, c64* l) { time_general_p2_body<N, E, S, false, PAD>(A, wg, l); });
  } else {
    exit(13);
  }
}

template <int N>
static void general_p2_n(const Launch<TimeArgs>& t) {
  switch (t.args.var) {
    case 0: general_p2_nv<N, 0>(t); break;
    case 1: general_p2_nv<N, 1>(t); break;
    case 2: general_p2_nv<N, 2>(t); break;
    case 3: general_p2_nv<N, 3>(t); break;
    case 4: general_p2_nv<N, 4>(t); break;
    case 5: general_p2_nv<N, 5>(t); break;
    default: exit(14);
  }
}

template <int P>
static void dst_blue_n(const Launch<DstArgs>& Lz) {
  const DstArgs& A = Lz.args;
  if (A.threads != p2sz::blue_T(P) || A.S != p2sz::blue_S(P) || Lz.lds != p2sz::blue_lds(P)) exit(21);
  run_grid(Lz.nwg, A.threads, Lz.lds, [&](long long wg, c64* l) { dst_blue_body<P>(A, wg, l); });
}

static void run_dst_generic(const Launch<DstArgs>& Lz) {
  const DstArgs& A = Lz.args;
  if (A.fft.bp2) {
    P2_SWITCH(A.fft.bp2, dst_blue_n, Lz)
    return;
  }
  if (A.fft.wide) run_grid(Lz.nwg, A.threads, Lz.lds, [&](long long wg, c64* l) { dst_body<true>(A, wg, l); });
  else run_grid(Lz.nwg, A.threads, Lz.lds, [&](long long wg, c64* l) { dst_body<false>(A, wg, l); });
}

static void run_dst(const sched::Geom& g, const double* in, double* out, long long batch, bool input,
                    const TabJob* tab = nullptr) {
  auto passes = sched::dst_passes(g, in, out, batch, input);
  if (tab) {
    if (!passes.back().args.fft.p2) exit(15);
    passes.back().args.tab = *tab;
  }
  for (const auto& Lz : passes) {
    const DstArgs& A = Lz.args;
    const int T = A.threads;
    if (A.fft.p2) {
      P2_SWITCH(A.fft.p2, dst_p2_n, Lz)
    } else if (A.fft.bp2) {
      P2_SWITCH(A.fft.bp2, dst_blue_n, Lz)
    } else if (A.fft.wide) {
      run_grid(Lz.nwg, T, Lz.lds, [&](long long wg, c64* l) { dst_body<true>(A, wg, l); });
    } else {
      run_grid(Lz.nwg, T, Lz.lds, [&](long long wg, c64* l) { dst_body<false>(A, wg, l); });
    }
  }
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  const std::vector<c64> roots = plan::radix_roots();
  std::memcpy(c_root, roots.data(), sizeof(c64) * roots.size());
  const std::string cmd = argv[1];
  if (cmd == "fft" && argc == 6) {
    const int n = atoi(argv[2]), S = atoi(argv[3]);
    Tables t = make_tables(n);
    if ((long long)S * t.dev.nc > 4096) return 6;
    auto raw = read_file(argv[4]);
    if (raw.size() != sizeof(c64) * (size_t)S * n) return 7;
    std::vector<c64> in(S * (size_t)n), out(S * (size_t)n);
    std::memcpy(in.data(), raw.data(), raw.size());
    if (t.dev.wide) fft_signals<true>(t, S, in.data(), out.data());
    else fft_signals<false>(t, S, in.data(), out.data());
    write_file(argv[5], out.data(), sizeof(c64) * out.size());
    printf("kind=%d nc=%d wide=%d stages=%d\n", t.dev.kind, t.dev.nc, t.dev.wide, t.dev.nstages);
    return 0;
  }
  if (cmd == "dst" && (argc == 7 || argc == 10)) {
    const int d = atoi(argv[2]), m = atoi(argv[3]);
    const long long batch = atoll(argv[4]);
    Tables tt = make_tables(2), st = make_tables(2 * (m + 1), true);
    std::vector<double> mu(m, 0.0);
    sched::Geom g = geom(d, m, 1, 1.0, 1.0, tt, st, mu);
    bool input = batch == 1;
    if (argc == 10) {
      g.var_rows = atoi(argv[7]);
      g.var_cols = atoi(argv[8]);
      input = atoi(argv[9]) != 0;
    }
    auto raw = read_file(argv[5]);
    const size_t N = (size_t)batch * g.nmodes;
    if (raw.size() != N * sizeof(double)) return 7;
    double* in = new double[N];
    double* out = new double[N];
    std::memcpy(in, raw.data(), raw.size());
    run_dst(g, in, out, batch, input);
    write_file(argv[6], out, N * sizeof(double));
    delete[] in;
    delete[] out;
    return 0;
  }
  if (cmd == "general" && (argc == 11 || argc == 13)) {
    const int d = atoi(argv[2]), m = atoi(argv[3]), n = atoi(argv[4]);
    const double L = atof(argv[5]), T = atof(argv[6]), alpha = atof(argv[7]);
    const int variant = atoi(argv[8]);
    const bool want_pad = argc == 13 && atoi(argv[11]) != 0;
    const int var_gen = argc == 13 ? atoi(argv[12]) : 0;
    Tables tt = make_tables(n + 1), st = make_tables(2 * (m + 1), true);
    const double h = L / (m + 1);
    std::vector<double> mu(m);
    for (int k = 1; k <= m; ++k) {
      const long double s = sinl((long double)k * plan::kPiL / (2.0L * (m + 1)));
      mu[k - 1] = (double)(4.0L / ((long double)h * h) * s * s);
    }
    sched::Geom g = geom(d, m, n, L, T, tt, st, mu);
    auto raw = read_file(argv[9]);
    const size_t ny = (size_t)g.Nt * g.nmodes;
    if (raw.size() != ny * sizeof(double)) return 7;
    double* y = new double[ny];
    double* f = new double[ny];
    std::memcpy(f, raw.data(), raw.size());
    double* W = nullptr;
    if (want_pad) {
      if (!sched::use_padded_general(g)) return 17;
      W = new double[sched::padded_elems(g)];
      for (long long i = 0; i < sched::padded_elems(g); ++i) W[i] = std::nan("");  // pad slots must not leak
    }
    std::vector<c64> tabs(3 * (size_t)g.Nt, c64{std::nan(""), std::nan("")});
    auto gs = sched::general_schedule(g, f, y, W, tabs.data(), var_gen);
    if (gs.padded != want_pad) return 18;
    if (gs.time.lds > 160 * 1024) return 16;
    const TabJob job{tabs.data(), g.Nt, variant, g.tau, alpha, nullptr, 1};
    // the host attaches the tables to the last input pass when it is a power-of-two kernel
    const bool side_job = gs.in.back().args.fft.p2 != 0;
    if (side_job) gs.in.back().args.tab = job;
    for (const auto& Lz : gs.in) {
      if (Lz.args.fft.p2) {
        P2_SWITCH(Lz.args.fft.p2, dst_p2_n, Lz)
      } else {
        run_dst_generic(Lz);
      }
    }
    if (!side_job) tab_job_run(job, 0, 1);
    const auto& t = gs.time;
    if (t.args.fft.p2) {
      P2_SWITCH(t.args.fft.p2, general_p2_n, t)
    } else if (t.args.fft.wide) {
      run_grid(t.nwg, 256, t.lds, [&](long long wg, c64* l) { time_general_body<true>(t.args, wg, l); });
    } else {
      run_grid(t.nwg, 256, t.lds, [&](long long wg, c64* l) { time_general_body<false>(t.args, wg, l); });
    }
    for (const auto& Lz : gs.out) {
      if (Lz.args.fft.p2) {
        P2_SWITCH(Lz.args.fft.p2, dst_p2_n, Lz)
      } else {
        run_dst_generic(Lz);
      }
    }
    write_file(argv[10], y, ny * sizeof(double));
    delete[] y;
    delete[] f;
    delete[] W;
    return 0;
  }
  if (cmd == "solveop" && argc == 12) {
    const int m = atoi(argv[2]), n = atoi(argv[3]);
    const double L = atof(argv[4]), T = atof(argv[5]), alpha = atof(argv[6]);
    const int variant = atoi(argv[7]), level = atoi(argv[11]);
    Tables tt = make_tables(n + 1), st = make_tables(2 * (m + 1), true);
    const double h = L / (m + 1);
    std::vector<double> mu(m, 0.0);
    sched::Geom g = geom(1, m, n, L, T, tt, st, mu);
    (void)h;
    auto raw = read_file(argv[8]);
    if (raw.size() != (size_t)m * sizeof(double)) return 7;
    auto rop = read_file(argv[10]);
    if (rop.size() != (size_t)(3 * m - 2) * sizeof(double)) return 8;
    std::vector<double> gd(m), opf(3 * m - 2), op(3 * (size_t)m, std::nan(""));
    std::memcpy(gd.data(), raw.data(), raw.size());
    std::memcpy(opf.data(), rop.data(), rop.size());
    for (int i = 0; i < m; ++i) {  // the library's device layout: [m] lower, [m] diag, [m] upper
      op[m + i] = opf[(m - 1) + i];
      if (i + 1 < m) {
        op[i] = opf[i];
        op[2 * (size_t)m + i] = opf[(2 * m - 1) + i];
      }
    }
    const SolveScalars sc = sched::host_scalars(alpha, variant, g.tau);
    std::vector<c64> s2((size_t)g.Nt * m, c64{std::nan(""), std::nan("")});
    auto ta = sched::thomas_step(g, sc, nullptr, variant, gd.data(), s2.data());
    ta.args.op_lo = op.data();
    ta.args.op_di = op.data() + m;
    ta.args.op_up = op.data() + 2 * m;
    // every level: the gamma table as side work of the solver kernel, as the host does
    std::vector<c64> tabs(3 * (size_t)g.Nt, c64{std::nan(""), std::nan("")});
    if (level < 0) ta.args.tab = TabJob{tabs.data(), g.Nt, variant, g.tau, alpha, nullptr, 1};
    run_grid(ta.nwg, ta.args.P * ta.args.S, ta.lds, [&](long long wg, c64* l) { tri1d_body(ta.args, wg, l); });
    const size_t ny = level < 0 ? (size_t)g.Nt * m : (size_t)m;
    std::vector<double> y(ny);
    auto t = sched::time1d_step(g, sc, nullptr, variant, s2.data(), y.data());
    if (level < 0) {
      t.args.gitab = tabs.data();
      t.lds = sched::lds_time1d(g, 0);
    }
    if (level >= 0) {
      t.args.lev_first = level;
      t.args.lev_count = 1;
      t.lds = sched::lds_time1d(g, 1);
    }
    if (t.args.fft.wide) run_grid(t.nwg, 256, t.lds, [&](long long wg, c64* l) { time1d_body<true>(t.args, wg, l); });
    else run_grid(t.nwg, 256, t.lds, [&](long long wg, c64* l) { time1d_body<false>(t.args, wg, l); });
    write_file(argv[9], y.data(), ny * sizeof(double));
    return 0;
  }
  if (cmd == "opdiff" && argc == 17) {
    // the host loop of qbvm_host.cpp::kop_solve with the emulated kernels
    const int d = atoi(argv[2]), m = atoi(argv[3]), n = atoi(argv[4]);
    const double L = atof(argv[5]), T = atof(argv[6]), alpha = atof(argv[7]);
    const int variant = atoi(argv[8]);
    const double tol = atof(argv[14]);
    const int maxit = atoi(argv[15]);
    if (d != 2 && d != 3) return 8;
    Tables tt = make_tables(n + 1), st = make_tables(2 * (m + 1), true);
    const double h = L / (m + 1);
    std::vector<double> mu(m);
    for (int k = 1; k <= m; ++k) {
      const long double sn = sinl((long double)k * plan::kPiL / (2.0L * (m + 1)));
      mu[k - 1] = (double)(4.0L / ((long double)h * h) * sn * sn);
    }
    sched::Geom g = geom(d, m, n, L, T, tt, st, mu);
    const long long M = g.nmodes;
    const size_t nf = (size_t)(M / m) * (m + 1);
    auto rg = read_file(argv[9]), rkx = read_file(argv[11]), rky = read_file(argv[12]);
    if (rg.size() != (size_t)M * 8 || rkx.size() != nf * 8 || rky.size() != nf * 8) return 7;
    std::vector<double> gv(M), kx(nf), ky(nf), kz(d == 3 ? nf : 0);
    std::memcpy(gv.data(), rg.data(), rg.size());
    std::memcpy(kx.data(), rkx.data(), rkx.size());
    std::memcpy(ky.data(), rky.data(), rky.size());
    if (d == 3) {
      auto rkz = read_file(argv[13]);
      if (rkz.size() != nf * 8) return 7;
      std::memcpy(kz.data(), rkz.data(), rkz.size());
    }
    double lo = INFINITY, hi = 0.0, gn2 = 0.0;
    for (const auto* k : {&kx, &ky, &kz})
      for (double v : *k) {
        lo = std::min(lo, v);
        hi = std::max(hi, v);
      }
    for (double v : gv) gn2 += v * v;
    const int H = (g.Nt + 1) / 2;
    const int nblk = (int)((M + (long long)kKryPointsPerLane * kKryThreads - 1) / ((long long)kKryPointsPerLane * kKryThreads));
    const size_t V = 2 * (size_t)H * (size_t)M;
    std::vector<double> work(6 * V, std::nan("")), part(3 * 2 * (size_t)H * nblk, std::nan("")),
        sys(8 * (size_t)H, std::nan(""));
    std::vector<c64> tabs(2 * (size_t)g.Nt, c64{std::nan(""), std::nan("")});
    const TabJob job{tabs.data(), g.Nt, variant, g.tau, alpha, nullptr, 0};
    tab_job_run(job, 0, 1);
    KrylovArgs a{};
    a.d = d;
    a.m = m;
    a.H = H;
    a.nblk = nblk;
    a.ppt = kKryPointsPerLane;
    a.M = M;
    a.ih2 = 1.0 / (h * h);
    a.kbar = 0.5 * (lo + hi);
    a.tol2 = tol * tol * gn2;
    a.kx = kx.data();
    a.ky = ky.data();
    a.kz = d == 3 ? kz.data() : nullptr;
    a.mu1d = mu.data();
    a.shift = tabs.data();
    a.g = gv.data();
    a.x = work.data();
    a.r = a.x + V;
    a.z = a.x + 2 * V;
    double* pbuf[2] = {a.x + 3 * V, a.x + 4 * V};
    a.q = a.x + 5 * V;
    a.part = part.data();
    a.sys = sys.data();
    const long long G = (long long)H * nblk;
    const size_t red = sizeof(c64) * kKryThreads;
    auto launch = [&](int step) {
      switch (step) {
        case kKryInit: run_grid(G, kKryThreads, 0, [&](long long wg, c64*) { kry_init_body(a, wg); }); break;
        case kKryApply:
          run_grid(G, kKryThreads, red + kry_apply_lds(m),
                   [&](long long wg, c64* l) { kry_apply_body(a, wg, l, l + kKryThreads); });
          break;
        case kKryUpdate: run_grid(G, kKryThreads, red, [&](long long wg, c64* l) { kry_update_body(a, wg, l); }); break;
        case kKryPrecond: run_grid(G, kKryThreads, red, [&](long long wg, c64* l) { kry_precond_body(a, wg, l); }); break;
        default: run_grid(H, kKryThreads, red, [&](long long wg, c64* l) { kry_scalars_body(a, wg, l); }); break;
      }
    };
    auto precond = [&]() {
      run_dst(g, a.r, a.z, 2LL * H, false);
      launch(kKryPrecond);
      run_dst(g, a.z, a.z, 2LL * H, false);
    };
    a.init = 1;
    a.pin = a.z;
    a.pout = pbuf[0];
    launch(kKryInit);
    precond();
    launch(kKryScalars);
    a.init = 0;
    int it = 0, active = H;
    while (it < maxit && active > 0) {
      ++it;
      launch(kKryApply);
      launch(kKryUpdate);
      precond();
      launch(kKryScalars);
      active = 0;
      for (int j = 0; j < H; ++j) active += sys[(size_t)j * 8 + 7] == 1.0;
      a.pin = a.pout;
      a.pout = a.pout == pbuf[0] ? pbuf[1] : pbuf[0];
    }
    double worst = 0.0, brk = 0.0;
    for (int j = 0; j < H; ++j) {
      worst = std::max(worst, std::sqrt(sys[(size_t)j * 8 + 6] / gn2));
      brk += sys[(size_t)j * 8 + 7] == -1.0;
    }
    KryTimeArgs t{};
    t.Nt = g.Nt;
    t.H = H;
    t.S = plan::signals_for(g.tfft.nc);
    t.lev_first = 0;
    t.lev_count = g.Nt;
    t.M = M;
    t.w = a.x;
    t.gi = tabs.data() + g.Nt;
    std::vector<double> y((size_t)g.Nt * M, std::nan(""));
    t.y = y.data();
    t.fft = g.tfft;
    const long long nwg = (M + 2LL * t.S - 1) / (2LL * t.S);
    const size_t lds = sizeof(c64) * ((size_t)t.S * t.fft.nc + 2 * (size_t)t.S);
    if (t.fft.wide) run_grid(nwg, 256, lds, [&](long long wg, c64* l) { kry_time_body<true>(t, wg, l); });
    else run_grid(nwg, 256, lds, [&](long long wg, c64* l) { kry_time_body<false>(t, wg, l); });
    write_file(argv[10], y.data(), y.size() * sizeof(double));
    const double stats[3] = {(double)it, worst, brk};
    write_file(argv[16], stats, sizeof(stats));
    return 0;
  }
  if (cmd == "solve" && (argc == 11 || argc == 14 || argc == 15 || argc == 16)) {
    const int d = atoi(argv[2]), m = atoi(argv[3]), n = atoi(argv[4]);
    const double L = atof(argv[5]), T = atof(argv[6]), alpha = atof(argv[7]);
    const int variant = atoi(argv[8]);
    Tables tt = make_tables(n + 1), st = make_tables(2 * (m + 1), true);
    const double h = L / (m + 1);
    std::vector<double> mu(m);
    for (int k = 1; k <= m; ++k) {
      const long double s = sinl((long double)k * plan::kPiL / (2.0L * (m + 1)));
      mu[k - 1] = (double)(4.0L / ((long double)h * h) * s * s);
    }
    sched::Geom g = geom(d, m, n, L, T, tt, st, mu);
    if (argc == 14) {
      g.var_rows = atoi(argv[11]);
      g.var_cols = atoi(argv[12]);
      g.var_time = atoi(argv[13]);
    }
    auto raw = read_file(argv[9]);
    if (raw.size() != (size_t)g.nmodes * sizeof(double)) return 7;
    double* gd = new double[g.nmodes];
    std::memcpy(gd, raw.data(), raw.size());
    const size_t ny = (size_t)g.Nt * g.nmodes;
    double* y = new double[ny];
    const SolveScalars sc = sched::host_scalars(alpha, variant, g.tau);
    const bool padded = sched::use_padded(g) && !(argc >= 15 && atoi(argv[14]) == 0);
    const bool want_plane = argc == 16 && atoi(argv[15]) != 0;
    const int pvar = want_plane ? atoi(argv[15]) - 1 : 0;  // plane argument: variant + 1
    if (want_plane && !p2sz::plane_valid(256, pvar)) return 20;
    if (want_plane && !(padded && sched::use_plane(g))) return 19;
    if (padded) {
      double* gh = new double[g.nmodes];
      double* W = new double[sched::padded_elems(g)];
      for (long long i = 0; i < sched::padded_elems(g); ++i) W[i] = std::nan("");  // pad slots must not leak
      // the last input pass fills the time tables as side work, as on the device
      std::vector<c64> tabs(2 * (size_t)g.Nt, c64{std::nan(""), std::nan("")});
      const TabJob job{tabs.data(), g.Nt, variant, g.tau, alpha, nullptr};
      run_dst(g, gd, gh, 1, true, &job);
      auto t = sched::time_step_padded(g, sc, nullptr, variant, gh, W);
      t.args.tabs = tabs.data();
      run_time_fast(t);
      if (want_plane) {
        for (const auto& Lz : sched::plane_pre_passes(g, W)) {
          P2_SWITCH(Lz.args.fft.p2, dst_p2_n, Lz)
        }
        const PlaneArgs pa = sched::plane_args(g, W, y);
        for (size_t q = 0; q < (size_t)g.Nt * g.nmodes; ++q) y[q] = std::nan("");  // every output written
        const long long G = pa.planes < 3 ? pa.planes : 3;  // a few workgroups, several planes each
        auto run_plane = [&](auto vc) {
          constexpr int PV = decltype(vc)::value;
          run_grid(G, p2sz::plane_T(PV), p2sz::plane_lds(256, PV),
                   [&](long long wg, c64* l) { dst_plane_p2_body<256, PV>(pa, wg, G, l); });
        };
        if (pvar == 0) run_plane(std::integral_constant<int, 0>{});
        else if (pvar == 1) run_plane(std::integral_constant<int, 1>{});
        else run_plane(std::integral_constant<int, 2>{});
      } else {
        for (const auto& Lz : sched::padded_passes(g, W, y)) {
          P2_SWITCH(Lz.args.fft.p2, dst_p2_n, Lz)
        }
      }
      delete[] gh;
      delete[] W;
    } else if (d == 1) {
      c64* s2 = new c64[(size_t)g.Nt * m];
      for (size_t q = 0; q < (size_t)g.Nt * m; ++q) s2[q] = c64{std::nan(""), std::nan("")};
      auto ta = sched::thomas_step(g, sc, nullptr, variant, gd, s2);
      std::vector<c64> tabs(3 * (size_t)g.Nt, c64{std::nan(""), std::nan("")});
      ta.args.tab = TabJob{tabs.data(), g.Nt, variant, g.tau, alpha, nullptr, 1};
      run_grid(ta.nwg, ta.args.P * ta.args.S, ta.lds, [&](long long wg, c64* l) { tri1d_body(ta.args, wg, l); });
      auto t = sched::time1d_step(g, sc, nullptr, variant, s2, y);
      t.args.gitab = tabs.data();
      t.lds = sched::lds_time1d(g, 0);
      if (t.args.fft.wide) run_grid(t.nwg, 256, t.lds, [&](long long wg, c64* l) { time1d_body<true>(t.args, wg, l); });
      else run_grid(t.nwg, 256, t.lds, [&](long long wg, c64* l) { time1d_body<false>(t.args, wg, l); });
      delete[] s2;
    } else {
      run_dst(g, gd, y, 1, true);
      const auto t = sched::time_step(g, sc, nullptr, variant, y, y, 0, g.Nt);
      const TimeArgs& A = t.args;
      if (A.fft.p2 || A.fft.gtA) {
        run_time_fast(t);
      } else if (A.fft.wide) {
        run_grid(t.nwg, 256, t.lds, [&](long long wg, c64* l) { time_body<true>(A, wg, l); });
      } else {
        run_grid(t.nwg, 256, t.lds, [&](long long wg, c64* l) { time_body<false>(A, wg, l); });
      }
      run_dst(g, y, y, g.Nt, false);
    }
    write_file(argv[10], y, ny * sizeof(double));
    delete[] gd;
    delete[] y;
    return 0;
  }
  return 2;
}
