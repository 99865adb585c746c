// Step (b) with a variable-coefficient 2D/3D operator (Section 3.3: the diagonalisation in
// time leaves one independent spatial system per shift, whatever the operator).  The
// systems (s_j I + A) w_j = g, A = -div(kappa grad u) in conservative (2d+1)-point form
// with kappa at the cell faces, are complex symmetric (A real symmetric, s_j complex),
// so they are solved by conjugate orthogonal conjugate gradients (CG with the bilinear
// form u^T v in place of the inner product), preconditioned by the constant-coefficient
// operator s_j I + kbar (-Lap_h), which the orthonormal sine transform diagonalises
// (eigenvalues s_j + kbar mu_k).  All H systems advance together; per system j:
//   z = P^{-1} r, rho' = r^T z, beta = rho'/rho, p = z + beta p, q = (s_j I + A) p,
//   alpha = rho'/(p^T q), x += alpha p, r -= alpha q.
// A system stops (its scalars freeze) once |r_j|^2 <= tol2.  Sums run per workgroup into
// fixed slots and are added in a fixed order: results do not depend on scheduling.
#pragma once

#include "qbvm_bodies.hpp"

namespace qbvm {

// per-system scalars, sys[j * kSysStride + ...]
constexpr int kSysRho = 0;     // complex rho = r^T z
constexpr int kSysAlpha = 2;   // complex alpha of the last update
constexpr int kSysBeta = 4;    // complex beta for the next direction
constexpr int kSysRn2 = 6;     // |r|^2
constexpr int kSysState = 7;   // 1 active, 0 converged, -1 breakdown (zero rho or p^T q)
constexpr int kSysStride = 8;

__device__ __forceinline__ c64 kry_bilinear(c64 a, c64 b) { return cmul(a, b); }

// Sum of v over the workgroup (kKryThreads lanes), fixed tree order; every lane gets it.
__device__ __forceinline__ c64 kry_wg_sum(c64 v, c64* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int w = kKryThreads / 2; w > 0; w >>= 1) {
    if (t < w) red[t] = cadd(red[t], red[t + w]);
    __syncthreads();
  }
  const c64 s = red[0];
  __syncthreads();
  return s;
}

// Sum of the nblk partial sums of system j in slot block `which` (fixed order).
__device__ __forceinline__ c64 kry_partials(const KrylovArgs& a, int which, int j, c64* red) {
  const c64* p = reinterpret_cast<const c64*>(a.part) + ((size_t)which * a.H + j) * a.nblk;
  c64 v = {0.0, 0.0};
  for (int b = threadIdx.x; b < a.nblk; b += kKryThreads) v = cadd(v, p[b]);
  return kry_wg_sum(v, red);
}

__device__ __forceinline__ void kry_store_partial(const KrylovArgs& a, int which, int j, int b, c64 v) {
  if (threadIdx.x == 0) reinterpret_cast<c64*>(a.part)[((size_t)which * a.H + j) * a.nblk + b] = v;
}

__device__ __forceinline__ c64 kry_load(const double* v, const KrylovArgs& a, int j, long long pt) {
  return {v[(size_t)j * a.M + pt], v[((size_t)a.H + j) * a.M + pt]};
}
__device__ __forceinline__ void kry_store(double* v, const KrylovArgs& a, int j, long long pt, c64 x) {
  v[(size_t)j * a.M + pt] = x.re;
  v[((size_t)a.H + j) * a.M + pt] = x.im;
}

// x = 0, r = g for every system; scalars reset.
__device__ __forceinline__ void kry_init_body(const KrylovArgs& a, long long wg) {
  const int j = (int)(wg / a.nblk), b = (int)(wg - (long long)j * a.nblk);
  const long long base = (long long)b * a.ppt * kKryThreads;
  for (int k = 0; k < a.ppt; ++k) {
    const long long pt = base + (long long)k * kKryThreads + threadIdx.x;
    if (pt < a.M) {
      kry_store(a.x, a, j, pt, {0.0, 0.0});
      kry_store(a.r, a, j, pt, {a.g[pt], 0.0});
    }
  }
  if (b == 0 && threadIdx.x < kSysStride) a.sys[(size_t)j * kSysStride + threadIdx.x] = threadIdx.x == kSysState ? 1.0 : 0.0;
}

// p = z + beta p_in at flattened point pt of system j, from global memory
__device__ __forceinline__ c64 kry_dir_at(const KrylovArgs& a, int j, long long pt, c64 beta) {
  return cadd(kry_load(a.z, a, j, pt), cmul(beta, kry_load(a.pin, a, j, pt)));
}

// New direction p = z + beta p_in (stored), q = (s_j I + A) p, partial sums of p^T q
// (slot block 0).  The workgroup's points [base, base + TP) and one grid row on either
// side are formed once into LDS (pl, TP + 2m entries), where the stencil reads its x_1
// and x_2 neighbours; in 3D the x_3 neighbours (a plane away) come from global memory.
__device__ __forceinline__ void kry_apply_body(const KrylovArgs& a, long long wg, c64* red, c64* pl) {
  const int j = (int)(wg / a.nblk), b = (int)(wg - (long long)j * a.nblk);
  const double* sy = a.sys + (size_t)j * kSysStride;
  if (sy[kSysState] != 1.0) return;  // the whole workgroup: j is uniform
  const c64 beta = {sy[kSysBeta], sy[kSysBeta + 1]};
  const c64 s = a.shift[j];
  const long long TP = (long long)a.ppt * kKryThreads;
  const long long base = (long long)b * TP;
  const long long lo = base - a.m;  // pl[e] holds point lo + e
  const long long hi = base + TP + a.m < a.M ? base + TP + a.m : a.M;
  for (long long pt = (lo > 0 ? lo : 0) + threadIdx.x; pt < hi; pt += kKryThreads) pl[pt - lo] = kry_dir_at(a, j, pt, beta);
  __syncthreads();
  const long long m2 = (long long)a.m * a.m;
  c64 acc = {0.0, 0.0};
  const c64 zero = {0.0, 0.0};
  for (int kk = 0; kk < a.ppt; ++kk) {
    const long long pt = base + (long long)kk * kKryThreads + threadIdx.x;
    if (pt < a.M) {
      const long long row = pt / a.m;  // k3 m + k2
      const int i = (int)(pt - row * a.m);
      const int k3 = (int)(row / a.m), k = (int)(row - (long long)k3 * a.m);
      const long long e = pt - lo;
      const c64 pc = pl[e];
      const c64 pw = i > 0 ? pl[e - 1] : zero, pe = i + 1 < a.m ? pl[e + 1] : zero;
      const c64 ps = k > 0 ? pl[e - a.m] : zero, pn = k + 1 < a.m ? pl[e + a.m] : zero;
      const double kw = a.kx[(size_t)row * (a.m + 1) + i], ke = a.kx[(size_t)row * (a.m + 1) + i + 1];
      const size_t yb = ((size_t)k3 * (a.m + 1) + k) * a.m + i;
      const double ks = a.ky[yb], kn = a.ky[yb + a.m];
      c64 ap = cscale(csub(pc, pw), kw);
      ap = cadd(ap, cscale(csub(pc, pe), ke));
      ap = cadd(ap, cscale(csub(pc, ps), ks));
      ap = cadd(ap, cscale(csub(pc, pn), kn));
      if (a.d == 3) {
        const c64 pd = k3 > 0 ? kry_dir_at(a, j, pt - m2, beta) : zero;
        const c64 pu = k3 + 1 < a.m ? kry_dir_at(a, j, pt + m2, beta) : zero;
        const double kd = a.kz[(size_t)pt], ku = a.kz[(size_t)pt + (size_t)m2];
        ap = cadd(ap, cscale(csub(pc, pd), kd));
        ap = cadd(ap, cscale(csub(pc, pu), ku));
      }
      const c64 qv = cadd(cmul(s, pc), cscale(ap, a.ih2));
      kry_store(a.pout, a, j, pt, pc);
      kry_store(a.q, a, j, pt, qv);
      acc = cadd(acc, kry_bilinear(pc, qv));
    }
  }
  kry_store_partial(a, 0, j, b, kry_wg_sum(acc, red));
}

// alpha = rho / (p^T q); x += alpha p, r -= alpha q; partial sums of |r|^2 (slot block 1).
__device__ __forceinline__ void kry_update_body(const KrylovArgs& a, long long wg, c64* red) {
  const int j = (int)(wg / a.nblk), b = (int)(wg - (long long)j * a.nblk);
  double* sy = a.sys + (size_t)j * kSysStride;
  if (sy[kSysState] != 1.0) return;
  const c64 sigma = kry_partials(a, 0, j, red);
  const c64 rho = {sy[kSysRho], sy[kSysRho + 1]};
  const double den = sigma.re * sigma.re + sigma.im * sigma.im;
  const c64 alpha = den > 0.0 ? c64{(rho.re * sigma.re + rho.im * sigma.im) / den,
                                    (rho.im * sigma.re - rho.re * sigma.im) / den}
                              : c64{0.0, 0.0};
  const long long base = (long long)b * a.ppt * kKryThreads;
  double rr = 0.0;
  for (int kk = 0; kk < a.ppt; ++kk) {
    const long long pt = base + (long long)kk * kKryThreads + threadIdx.x;
    if (pt < a.M) {
      const c64 xv = cadd(kry_load(a.x, a, j, pt), cmul(alpha, kry_load(a.pout, a, j, pt)));
      const c64 rv = csub(kry_load(a.r, a, j, pt), cmul(alpha, kry_load(a.q, a, j, pt)));
      kry_store(a.x, a, j, pt, xv);
      kry_store(a.r, a, j, pt, rv);
      rr += rv.re * rv.re + rv.im * rv.im;
    }
  }
  kry_store_partial(a, 1, j, b, kry_wg_sum({rr, 0.0}, red));
  if (b == 0 && threadIdx.x == 0) {
    sy[kSysAlpha] = alpha.re;
    sy[kSysAlpha + 1] = alpha.im;
    if (!(den > 0.0)) sy[kSysState] = -1.0;  // p^T q = 0: breakdown, the system stops
  }
}

// In the sine basis (after the forward transform of r into z): z_k /= s_j + kbar mu_k,
// partial sums of r^T z = sum_k rhat_k zhat_k (the transform is real orthogonal).
__device__ __forceinline__ void kry_precond_body(const KrylovArgs& a, long long wg, c64* red) {
  const int j = (int)(wg / a.nblk), b = (int)(wg - (long long)j * a.nblk);
  if (a.sys[(size_t)j * kSysStride + kSysState] != 1.0) return;
  const c64 s = a.shift[j];
  const long long base = (long long)b * a.ppt * kKryThreads;
  c64 acc = {0.0, 0.0};
  for (int kk = 0; kk < a.ppt; ++kk) {
    const long long pt = base + (long long)kk * kKryThreads + threadIdx.x;
    if (pt < a.M) {
      const long long row = pt / a.m;
      const int k1 = (int)(pt - row * a.m), k3 = (int)(row / a.m), k2 = (int)(row - (long long)k3 * a.m);
      const double mu = a.mu1d[k1] + a.mu1d[k2] + (a.d == 3 ? a.mu1d[k3] : 0.0);
      const double re = s.re + a.kbar * mu;
      const double inv = 1.0 / (re * re + s.im * s.im);
      const c64 rh = kry_load(a.z, a, j, pt);
      const c64 zh = {(rh.re * re + rh.im * s.im) * inv, (rh.im * re - rh.re * s.im) * inv};
      kry_store(a.z, a, j, pt, zh);
      acc = cadd(acc, kry_bilinear(rh, zh));
    }
  }
  kry_store_partial(a, 2, j, b, kry_wg_sum(acc, red));
}

// Per system: |r|^2 and rho' from the partial sums; beta = rho'/rho; convergence.
__device__ __forceinline__ void kry_scalars_body(const KrylovArgs& a, long long wg, c64* red) {
  const int j = (int)wg;
  double* sy = a.sys + (size_t)j * kSysStride;
  const bool active = sy[kSysState] == 1.0;
  const c64 rho_new = kry_partials(a, 2, j, red);
  const c64 rn2 = a.init ? c64{0.0, 0.0} : kry_partials(a, 1, j, red);
  if (threadIdx.x != 0 || !active) return;
  const c64 rho = {sy[kSysRho], sy[kSysRho + 1]};
  const double den = rho.re * rho.re + rho.im * rho.im;
  c64 beta = {0.0, 0.0};
  if (!a.init) {
    beta = den > 0.0 ? c64{(rho_new.re * rho.re + rho_new.im * rho.im) / den,
                           (rho_new.im * rho.re - rho_new.re * rho.im) / den}
                     : c64{0.0, 0.0};
    sy[kSysRn2] = rn2.re;
  }
  sy[kSysBeta] = beta.re;
  sy[kSysBeta + 1] = beta.im;
  sy[kSysRho] = rho_new.re;
  sy[kSysRho + 1] = rho_new.im;
  if (!a.init && rn2.re <= a.tol2) sy[kSysState] = 0.0;
  else if (!(rho_new.re != 0.0 || rho_new.im != 0.0) || (!a.init && !(den > 0.0))) sy[kSysState] = -1.0;
}

// Step (c) on the runtime engine: per pair of points (a, b), u_j = w_j(a) + i w_j(b) with
// w_j = conj(w_{N_t-1-j}) for j >= H; X = DFT(u); y_l(a) = Re(gi_l X_l), y_l(b) = Im(gi_l X_l)
// (both are real because the pair sums j, N_t-1-j are real).
template <bool WIDE>
__device__ __forceinline__ void kry_time_body(const KryTimeArgs& a, long long wg, c64* lds) {
  const int S = a.S, Nt = a.Nt, nc = a.fft.nc;
  c64* buf = lds;
  c64* side = buf + (size_t)S * nc;
  const long long p0 = wg * 2LL * S;
  for (int e = threadIdx.x; e < S * Nt; e += blockDim.x) {
    const int j = e / S, s = e - j * S;
    const bool cj = j >= a.H;
    const int jj = cj ? Nt - 1 - j : j;
    const long long pa = p0 + 2 * s;
    c64 wa = {0.0, 0.0}, wb = {0.0, 0.0};
    if (pa < a.M) wa = {a.w[(size_t)jj * a.M + pa], a.w[((size_t)a.H + jj) * a.M + pa]};
    if (pa + 1 < a.M) wb = {a.w[(size_t)jj * a.M + pa + 1], a.w[((size_t)a.H + jj) * a.M + pa + 1]};
    if (cj) {
      wa.im = -wa.im;
      wb.im = -wb.im;
    }
    const c64 u = {wa.re - wb.im, wa.im + wb.re};
    const int pos = fft_in_pos(a.fft, j);
    if (pos < 0) side[s] = u;
    else buf[(size_t)pos * S + s] = u;
  }
  __syncthreads();
  if (a.fft.kind == kBluestein) fft_bluestein_prep(buf, S, a.fft);
  fft_run<WIDE>(buf, S, a.fft, side);
  const int tot = S * a.lev_count;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int li = e / S, s = e - li * S;
    const int l = a.lev_first + li;
    const c64 v = cmul(a.gi[l], fft_out(buf, S, a.fft, s, l, side));
    const long long pa = p0 + 2 * s;
    double* yl = a.y + (long long)li * a.M;
    if (pa < a.M) yl[pa] = v.re;
    if (pa + 1 < a.M) yl[pa + 1] = v.im;
  }
}

}  // namespace qbvm
