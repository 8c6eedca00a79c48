// Transport kernels for gfx950: lead self-energies by decimation, the
// broadening factorisation, and the block forward/backward sweeps with the
// fused transmission / density reductions.
//
// One workgroup of 256 threads owns one energy at a time (energies are
// independent; the block chain of one energy is sequential).  Blocks are
// padded to a multiple of 16 (M) so that every tile is a full MFMA tile;
// the padding is decoupled from the physical basis (see qtx_api.cpp).
#include "qtx_device.h"
#include "qtx_internal.h"

namespace qtx {

// ------------------------------------------------------------ Gauss-Jordan
// The matrix is distributed over a 16 x 16 grid of lanes (thread t owns rows
// [b*(t/16), +b) and columns [b*(t%16), +b), b = M/16).  Each pivot step
// publishes the pivot column and the scaled pivot row through LDS; the pivot
// is the largest |re|+|im| among unused rows (partial pivoting without
// physical row exchanges; the permutation is undone when the result is
// written back).

template <typename R, int M> struct GJScratch {
  cpx<R> col[2][M];
  cpx<R> row[M];
  int piv[M];
  int pinv[M];
};

template <typename R, int M>
__device__ __forceinline__ int gj_pick_pivot(const cpx<R>* col, bool& used0, bool& used1) {
  const int lane = threadIdx.x & 63;
  uint64_t key = 0;
  if (lane < M && !used0) key = pivot_key(col[lane], lane, M);
  if (M > 64 && lane + 64 < M && !used1) {
    uint64_t k2 = pivot_key(col[lane + 64], lane + 64, M);
    key = k2 > key ? k2 : key;
  }
  key = wave_max_u64(key);
  const int p = M - (int)(uint32_t)key;
  if (lane == p) used0 = true;
  if (lane + 64 == p) used1 = true;
  return p;
}

// In-place inverse of the M x M matrix in LDS (row stride S).
template <typename R, int M>
__device__ void gj_inverse(cpx<R>* mat, int S, GJScratch<R, M>& sc) {
  constexpr int b = M / 16;
  const int t = threadIdx.x, gr = t >> 4, gc = t & 15;
  cpx<R> a[b][b];
#pragma unroll
  for (int rr = 0; rr < b; ++rr)
#pragma unroll
    for (int cc = 0; cc < b; ++cc) a[rr][cc] = mat[(b * gr + rr) * S + b * gc + cc];
  bool used0 = false, used1 = false;
  if (gc == 0)
#pragma unroll
    for (int rr = 0; rr < b; ++rr) sc.col[0][b * gr + rr] = a[rr][0];
  for (int j = 0; j < M; ++j) {
    const cpx<R>* col = sc.col[j & 1];
    __syncthreads();
    const int p = gj_pick_pivot<R, M>(col, used0, used1);
    const cpx<R> inv = cinv(col[p]);
    if (t == 0) sc.piv[j] = p;
    if (gr == p / b) {
      const int pr = p - b * gr;
#pragma unroll
      for (int rr = 0; rr < b; ++rr)
        if (rr == pr)
#pragma unroll
          for (int cc = 0; cc < b; ++cc) {
            const int c = b * gc + cc;
            cpx<R> v = (c == j) ? mk<R>(1, 0) : a[rr][cc];
            sc.row[c] = cmul(v, inv);
          }
    }
    __syncthreads();
    cpx<R> pv[b];
#pragma unroll
    for (int cc = 0; cc < b; ++cc) pv[cc] = sc.row[b * gc + cc];
#pragma unroll
    for (int rr = 0; rr < b; ++rr) {
      const int r = b * gr + rr;
      const cpx<R> f = col[r];
      const bool isp = (r == p);
#pragma unroll
      for (int cc = 0; cc < b; ++cc) {
        const int c = b * gc + cc;
        cpx<R> base = (c == j) ? mk<R>(0, 0) : a[rr][cc];
        a[rr][cc] = isp ? pv[cc] : cfms(base, f, pv[cc]);
      }
    }
    if (j + 1 < M && gc == (j + 1) / b) {
      const int jc = (j + 1) - b * gc;
#pragma unroll
      for (int cc = 0; cc < b; ++cc)
        if (cc == jc)
#pragma unroll
          for (int rr = 0; rr < b; ++rr) sc.col[(j + 1) & 1][b * gr + rr] = a[rr][cc];
    }
  }
  __syncthreads();
  if (t < M) sc.pinv[sc.piv[t]] = t;
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < b; ++rr)
#pragma unroll
    for (int cc = 0; cc < b; ++cc) mat[sc.pinv[b * gr + rr] * S + sc.piv[b * gc + cc]] = a[rr][cc];
  __syncthreads();
}

// Gauss-Jordan solve of eps * [ga | gb] = [alpha | beta] (M x 3M augmented,
// no explicit inverse); writes [ga | gb] row-major with leading dim 2M.
template <int M> struct GJ3Scratch {
  cpx<double> col[2][M];
  cpx<double> row[3 * M];
  int piv[M];
  int pinv[M];
};

template <int M>
__device__ void gj_solve3(const double2* eps, const double2* al, const double2* be, double2* gout,
                          GJ3Scratch<M>& sc) {
  constexpr int b = M / 16;
  const int t = threadIdx.x, gr = t >> 4, gc = t & 15;
  cpx<double> a[3][b][b];
  const double2* src[3] = {eps, al, be};
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int rr = 0; rr < b; ++rr)
#pragma unroll
      for (int cc = 0; cc < b; ++cc) a[q][rr][cc] = ldd(src[q] + (b * gr + rr) * M + b * gc + cc);
  bool used0 = false, used1 = false;
  if (gc == 0)
#pragma unroll
    for (int rr = 0; rr < b; ++rr) sc.col[0][b * gr + rr] = a[0][rr][0];
  for (int j = 0; j < M; ++j) {
    const cpx<double>* col = sc.col[j & 1];
    __syncthreads();
    const int p = gj_pick_pivot<double, M>(col, used0, used1);
    const cpx<double> inv = cinv(col[p]);
    if (t == 0) sc.piv[j] = p;
    if (gr == p / b) {
      const int pr = p - b * gr;
#pragma unroll
      for (int rr = 0; rr < b; ++rr)
        if (rr == pr)
#pragma unroll
          for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int cc = 0; cc < b; ++cc) sc.row[q * M + b * gc + cc] = cmul(a[q][rr][cc], inv);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      cpx<double> pv[b];
#pragma unroll
      for (int cc = 0; cc < b; ++cc) pv[cc] = sc.row[q * M + b * gc + cc];
#pragma unroll
      for (int rr = 0; rr < b; ++rr) {
        const int r = b * gr + rr;
        const cpx<double> f = col[r];
        const bool isp = (r == p);
#pragma unroll
        for (int cc = 0; cc < b; ++cc) a[q][rr][cc] = isp ? pv[cc] : cfms(a[q][rr][cc], f, pv[cc]);
      }
    }
    if (j + 1 < M && gc == (j + 1) / b) {
      const int jc = (j + 1) - b * gc;
#pragma unroll
      for (int cc = 0; cc < b; ++cc)
        if (cc == jc)
#pragma unroll
          for (int rr = 0; rr < b; ++rr) sc.col[(j + 1) & 1][b * gr + rr] = a[0][rr][cc];
    }
  }
  __syncthreads();
  if (t < M) sc.pinv[sc.piv[t]] = t;
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < b; ++rr) {
    const int orow = sc.pinv[b * gr + rr];
#pragma unroll
    for (int cc = 0; cc < b; ++cc) {
      const int c = b * gc + cc;
      double2 v1, v2;
      v1.x = a[1][rr][cc].re; v1.y = a[1][rr][cc].im;
      v2.x = a[2][rr][cc].re; v2.y = a[2][rr][cc].im;
      gout[orow * 2 * M + c] = v1;
      gout[orow * 2 * M + M + c] = v2;
    }
  }
  __syncthreads();
}

// ------------------------------------------------ broadening factorisation
// Gamma = i (Sigma - Sigma^H) is Hermitian but only semi-definite up to
// O(eta) (the broadening also enters the non-orthogonal couplings), so it
// is factored as Gamma = W diag(s) W^H with s = +-1 by a diagonally pivoted
// LDL^H: at each step the remaining diagonal entry of largest magnitude d
// is eliminated, column k of W is the pivot column / sqrt|d| and s_k =
// sign(d).  Exactly zero remaining diagonals (padding) end the factorisation.
template <int M> struct LDLScratch {
  cpx<double> col[M];
  double dg[M];
};

template <int M>
__device__ void gamma_ldl(const double2* sig, double2* W, double* sg, LDLScratch<M>& sc) {
  constexpr int b = M / 16;
  const int t = threadIdx.x, gr = t >> 4, gc = t & 15;
  cpx<double> a[b][b];
#pragma unroll
  for (int rr = 0; rr < b; ++rr)
#pragma unroll
    for (int cc = 0; cc < b; ++cc) {
      const int r = b * gr + rr, c = b * gc + cc;
      cpx<double> s1 = ldd(sig + r * M + c), s2 = ldd(sig + c * M + r);
      a[rr][cc] = mk<double>(-(s1.im + s2.im), s1.re - s2.re);
    }
  for (int idx = t; idx < M * M; idx += NT) W[idx] = make_double2(0.0, 0.0);
  if (t < M) sg[t] = 0.0;
  bool used0 = false, used1 = false;
  for (int k = 0; k < M; ++k) {
    if (gr == gc)
#pragma unroll
      for (int rr = 0; rr < b; ++rr) sc.dg[b * gr + rr] = a[rr][rr].re;
    __syncthreads();
    const int lane = t & 63;
    uint64_t key = 0;
    if (lane < M && !used0) key = pivot_key(mk<double>(sc.dg[lane], 0.0), lane, M);
    if (M > 64 && lane + 64 < M && !used1) {
      uint64_t k2 = pivot_key(mk<double>(sc.dg[lane + 64], 0.0), lane + 64, M);
      key = k2 > key ? k2 : key;
    }
    key = wave_max_u64(key);
    const int p = M - (int)(uint32_t)key;
    if (lane == p) used0 = true;
    if (lane + 64 == p) used1 = true;
    const double d = sc.dg[p];
    if (d == 0.0) break;                      // uniform: every thread reads the same d
    if (gc == p / b) {
      const int pc = p - b * gc;
#pragma unroll
      for (int cc = 0; cc < b; ++cc)
        if (cc == pc)
#pragma unroll
          for (int rr = 0; rr < b; ++rr) sc.col[b * gr + rr] = a[rr][cc];
    }
    __syncthreads();
    const double sq = sqrt(fabs(d));
    if (t < M) {
      cpx<double> v = sc.col[t];
      W[t * M + k] = make_double2(v.re / sq, v.im / sq);
    }
    if (t == 0) sg[k] = d > 0.0 ? 1.0 : -1.0;
    const double id = 1.0 / d;
#pragma unroll
    for (int rr = 0; rr < b; ++rr) {
      const cpx<double> fr = sc.col[b * gr + rr];
#pragma unroll
      for (int cc = 0; cc < b; ++cc) {
        const cpx<double> fc = sc.col[b * gc + cc];
        // a -= fr conj(fc) / d
        const double re = (fr.re * fc.re + fr.im * fc.im) * id;
        const double im = (fr.im * fc.re - fr.re * fc.im) * id;
        a[rr][cc].re -= re;
        a[rr][cc].im -= im;
      }
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------- decimation
// Doubling elimination of the semi-infinite lead: with on-site e and
// couplings a (slab j -> j+1) and b (j+1 -> j), eliminating every other slab
// gives e' = e - a g b - b g a, a' = -a g a, b' = -b g b with g = e^-1; the
// surface of a right lead keeps only -a g b and that of a left lead only
// -b g a.  Sigma = D0 - (converged surface block).  g [a | b] is obtained
// by a Gauss-Jordan solve, not from an explicit inverse: the explicit
// inverse loses up to two extra digits when D0 is ill-conditioned.
template <int M>
__global__ __launch_bounds__(NT) void k_decimate(Prob P, const double* E, int nE, double eta, int sides,
                                                 double tol, int maxit, double2* scratch, double2* sig,
                                                 double2* wf, double* sgn, int* iters) {
  constexpr int MT = M / 16, MM = M * M;
  __shared__ GJ3Scratch<M> sc;
  __shared__ LDLScratch<M> lsc;
  __shared__ double red[2][NWAVE];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  double2* ws = scratch + (size_t)blockIdx.x * 9 * MM;
  double2* eps = ws;
  double2* esL = ws + MM;
  double2* esR = ws + 2 * MM;
  double2* al[2] = {ws + 3 * MM, ws + 5 * MM};
  double2* be[2] = {ws + 4 * MM, ws + 6 * MM};
  double2* g = ws + 7 * MM;  // M x 2M
  const int njobs = nE * sides;
  for (int job = blockIdx.x; job < njobs; job += gridDim.x) {
    const int e = job / sides;
    const int side = (sides == 2) ? (job % 2) : -1;
    const double2* lead = (side == 1) ? P.leadR : P.leadL;
    const double V = (side == 1) ? P.VR : P.VL;
    const double2 *H00 = lead, *H01 = lead + MM, *S00 = lead + 2 * MM, *S01 = lead + 3 * MM;
    const cpx<double> zx = mk<double>(E[e] - V, eta);
    double scl = 0.0;
    for (int idx = t; idx < MM; idx += NT) {
      const int r = idx / M, c = idx - r * M;
      cpx<double> s = ldd(S00 + idx), h = ldd(H00 + idx);
      double2 d0 = make_double2(zx.re * s.re - zx.im * s.im - h.re, zx.re * s.im + zx.im * s.re - h.im);
      s = ldd(S01 + idx); h = ldd(H01 + idx);
      double2 u = make_double2(zx.re * s.re - zx.im * s.im - h.re, zx.re * s.im + zx.im * s.re - h.im);
      s = ldd(S01 + c * M + r); h = ldd(H01 + c * M + r);
      double2 l = make_double2(zx.re * s.re + zx.im * s.im - h.re, zx.im * s.re - zx.re * s.im + h.im);
      eps[idx] = d0; esL[idx] = d0; esR[idx] = d0; al[0][idx] = u; be[0][idx] = l;
      scl = fmax(scl, fabs(d0.x) + fabs(d0.y));
    }
    scl = wave_maxd(scl);
    if (lane == 0) red[0][w] = scl;
    __syncthreads();
    scl = 0.0;
    for (int q = 0; q < NWAVE; ++q) scl = fmax(scl, red[0][q]);
    int cur = 0, it = 0;
    bool conv = false;
    for (it = 1; it <= maxit; ++it) {
      gj_solve3<M>(eps, al[cur], be[cur], g, sc);
      double na = 0.0, nb = 0.0;
      for (int tj = w; tj < MT; tj += NWAVE) {
        ctile<double> a1[MT], a2[MT];
#pragma unroll
        for (int ti = 0; ti < MT; ++ti) { tzero(a1[ti]); tzero(a2[ti]); }
        cgemm_col<double, MT, MT>(a1, AGlob<double>{al[cur], M, 1.0}, BGlob<double>{g + M, 2 * M}, tj);
        cgemm_col<double, MT, MT>(a2, AGlob<double>{be[cur], M, 1.0}, BGlob<double>{g, 2 * M}, tj);
        tiles_foreach<double, MT>(a1, tj, [&](int row, int col, int ti, int r) {
          const int idx = row * M + col;
          const double r1 = a1[ti].re[r], i1 = a1[ti].im[r], r2 = a2[ti].re[r], i2 = a2[ti].im[r];
          double2 v = eps[idx];
          v.x -= r1 + r2; v.y -= i1 + i2; eps[idx] = v;
          v = esR[idx]; v.x -= r1; v.y -= i1; esR[idx] = v;
          v = esL[idx]; v.x -= r2; v.y -= i2; esL[idx] = v;
        });
#pragma unroll
        for (int ti = 0; ti < MT; ++ti) { tzero(a1[ti]); tzero(a2[ti]); }
        cgemm_col<double, MT, MT>(a1, AGlob<double>{al[cur], M, 1.0}, BGlob<double>{g, 2 * M}, tj);
        cgemm_col<double, MT, MT>(a2, AGlob<double>{be[cur], M, 1.0}, BGlob<double>{g + M, 2 * M}, tj);
        tiles_foreach<double, MT>(a1, tj, [&](int row, int col, int ti, int r) {
          const int idx = row * M + col;
          al[cur ^ 1][idx] = make_double2(-a1[ti].re[r], -a1[ti].im[r]);
          be[cur ^ 1][idx] = make_double2(-a2[ti].re[r], -a2[ti].im[r]);
          na = fmax(na, fabs(a1[ti].re[r]) + fabs(a1[ti].im[r]));
          nb = fmax(nb, fabs(a2[ti].re[r]) + fabs(a2[ti].im[r]));
        });
      }
      na = wave_maxd(na);
      nb = wave_maxd(nb);
      if (lane == 0) { red[0][w] = na; red[1][w] = nb; }
      __syncthreads();
      na = 0.0; nb = 0.0;
      for (int q = 0; q < NWAVE; ++q) { na = fmax(na, red[0][q]); nb = fmax(nb, red[1][q]); }
      cur ^= 1;
      __syncthreads();
      if (na + nb < tol * scl) { conv = true; break; }
    }
    if (!conv) it = -maxit;
    // Sigma = D0 - surface block
    for (int idx = t; idx < MM; idx += NT) {
      cpx<double> s = ldd(S00 + idx), h = ldd(H00 + idx);
      const double dr = zx.re * s.re - zx.im * s.im - h.re, di = zx.re * s.im + zx.im * s.re - h.im;
      if (side != 1) { double2 v = esL[idx]; sig[(size_t)(2 * e) * MM + idx] = make_double2(dr - v.x, di - v.y); }
      if (side != 0) { double2 v = esR[idx]; sig[(size_t)(2 * e + 1) * MM + idx] = make_double2(dr - v.x, di - v.y); }
    }
    __syncthreads();
    for (int s = 0; s < 2; ++s) {
      if ((side == 0 && s == 1) || (side == 1 && s == 0)) continue;
      gamma_ldl<M>(sig + (size_t)(2 * e + s) * MM, wf + (size_t)(2 * e + s) * MM, sgn + (size_t)(2 * e + s) * M, lsc);
      if (t == 0) iters[2 * e + s] = it;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ block sweeps
// Left-connected forward sweep for slabs i = 0..N-1:
//   Dt_i = D_i - L_i X_{i-1}      (D_0 -= Sigma_L, D_{N-1} -= Sigma_R)
//   y_i  = -L_i z_{i-1}           (y_0 = W_L: left injection, Gamma_L = W_L s W_L^H)
//   [X_i | z_i] = Dt_i^-1 [U_i | y_i],   [psiR | psiL]_{N-1} = Dt^-1 [W_R | y]
// then back substitution psi_i = [0 | z_i] - X_i psi_{i+1} for both
// injections, with the slab densities reduced on the fly and
// T = sum_{j,k} s^R_j s^L_k |(W_R^H psiL_{N-1})_{jk}|^2.
// D_i, U_i and L_i = A_{i,i-1} are generated from the stored H/S blocks and
// the potential weights while they are loaded as MFMA operands.
template <typename R, int M>
__global__ __launch_bounds__(NT) void k_sweep(Prob P, const double* E, int nE, double eta,
                                              const double2* sig, const double2* wf, const double* sgn,
                                              const int* iters, typename vec2t<R>::type* ws, size_t ws_stride,
                                              double* part, double* T, double* ldos, qtx_info* info) {
  typedef typename vec2t<R>::type V2;
  constexpr int MT = M / 16, MM = M * M, S = M + 1, LD = 2 * M;
  __shared__ cpx<R> mat[M * S];
  __shared__ GJScratch<R, M> sc;
  __shared__ double tred[NWAVE];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int N = P.N;
  V2* XZ = ws + (size_t)blockIdx.x * ws_stride;
  V2* PSI = XZ + (size_t)N * M * LD;
  double* prt = part + (size_t)blockIdx.x * NWAVE * 2 * N;
  for (int e = blockIdx.x; e < nE; e += gridDim.x) {
    const cpx<double> z = mk<double>(E[e], eta);
    const double2* sL = sig + (size_t)(2 * e) * MM;
    const double2* sR = sL + MM;
    const double2* WL = wf + (size_t)(2 * e) * MM;
    const double2* WR = WL + MM;
    const double* sgL = sgn + (size_t)(2 * e) * M;
    const double* sgR = sgL + M;
    for (int i = 0; i < N; ++i) {
      __syncthreads();
      V2* Xi = XZ + (size_t)i * M * LD;
      const double vd = P.vd(i);
      const double2* Sd = P.Sd(i);
      const double2* Hd = P.Hd(i);
      const cpx<double> zd = mk<double>(z.re - vd, z.im);
      for (int tj = w; tj < 2 * MT; tj += NWAVE) {
        ctile<R> acc[MT];
        if (tj < MT) {
          tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
            const int idx = row * M + col;
            cpx<double> s = ldd(Sd + idx), h = ldd(Hd + idx);
            double re = zd.re * s.re - zd.im * s.im - h.re;
            double im = zd.re * s.im + zd.im * s.re - h.im;
            if (i == 0) { cpx<double> q = ldd(sL + idx); re -= q.re; im -= q.im; }
            if (i == N - 1) { cpx<double> q = ldd(sR + idx); re -= q.re; im -= q.im; }
            acc[ti].re[r] = (R)re;
            acc[ti].im[r] = (R)im;
          });
        } else if (i == 0) {
          tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
            cpx<double> q = ldd(WL + row * M + col - M);
            acc[ti].re[r] = (R)q.re;
            acc[ti].im[r] = (R)q.im;
          });
        } else {
#pragma unroll
          for (int ti = 0; ti < MT; ++ti) tzero(acc[ti]);
        }
        if (i > 0) {
          const double vu = P.vu(i - 1);
          AGenCT<R> A{P.Su(i - 1), P.Hu(i - 1), mk<double>(z.re - vu, z.im), -1.0, M};
          cgemm_col<R, MT, MT>(acc, A, BGlob<R>{Xi - (size_t)M * LD, LD}, tj);
        }
        if (tj < MT) {
          tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
            mat[row * S + col] = mk<R>(acc[ti].re[r], acc[ti].im[r]);
          });
        } else {
          tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
            st2<R>(Xi + row * LD + col, mk<R>(acc[ti].re[r], acc[ti].im[r]));
          });
        }
      }
      __syncthreads();
      gj_inverse<R, M>(mat, S, sc);
      for (int tj = w; tj < 2 * MT; tj += NWAVE) {
        ctile<R> acc[MT];
#pragma unroll
        for (int ti = 0; ti < MT; ++ti) tzero(acc[ti]);
        ALds<R> A{mat, S};
        if (tj < MT) {
          if (i < N - 1) {
            const double vu = P.vu(i);
            cgemm_col<R, MT, MT>(acc, A, BGen<R>{P.Su(i), P.Hu(i), mk<double>(z.re - vu, z.im), M}, tj);
          } else {
            cgemm_col<R, MT, MT>(acc, A, BGlobD<R>{WR, M}, tj);
          }
        } else {
          cgemm_col<R, MT, MT>(acc, A, BGlob<R>{Xi, LD}, tj);
        }
        tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
          st2<R>(Xi + row * LD + col, mk<R>(acc[ti].re[r], acc[ti].im[r]));
        });
      }
    }
    __syncthreads();
    // transmission from the left-injected solution on the last slab
    {
      const V2* XN = XZ + (size_t)(N - 1) * M * LD;
      double tp = 0.0;
      for (int tj = w; tj < 2 * MT; tj += NWAVE) {
        if (tj < MT) continue;
        ctile<R> acc[MT];
#pragma unroll
        for (int ti = 0; ti < MT; ++ti) tzero(acc[ti]);
        cgemm_col<R, MT, MT>(acc, AGlobCT<R>{WR, M}, BGlob<R>{XN, LD}, tj);
        tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
          const double re = acc[ti].re[r], im = acc[ti].im[r];
          tp += sgR[row] * sgL[col - M] * (re * re + im * im);
        });
      }
      tp = wave_sum(tp);
      if (lane == 0) tred[w] = tp;
    }
    // back substitution with fused slab densities
    for (int i = N - 1; i >= 0; --i) {
      const V2* Xi = XZ + (size_t)i * M * LD;
      double pL = 0.0, pR = 0.0;
      for (int tj = w; tj < 2 * MT; tj += NWAVE) {
        ctile<R> acc[MT];
        if (i == N - 1 || tj >= MT) {
          tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
            cpx<R> v = ld2<R>(Xi + row * LD + col);
            acc[ti].re[r] = v.re;
            acc[ti].im[r] = v.im;
          });
        } else {
#pragma unroll
          for (int ti = 0; ti < MT; ++ti) tzero(acc[ti]);
        }
        if (i < N - 1) cgemm_col<R, MT, MT>(acc, AGlob<R>{Xi, LD, (R)-1}, BGlob<R>{PSI, LD}, tj);
        tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
          const double re = acc[ti].re[r], im = acc[ti].im[r];
          st2<R>(PSI + row * LD + col, mk<R>(acc[ti].re[r], acc[ti].im[r]));
          if (col < M) pR += sgR[col] * (re * re + im * im);
          else pL += sgL[col - M] * (re * re + im * im);
        });
      }
      __threadfence_block();
      pL = wave_sum(pL);
      pR = wave_sum(pR);
      if (lane == 0) {
        prt[(w * 2 + 0) * N + i] = pL;
        prt[(w * 2 + 1) * N + i] = pR;
      }
    }
    __syncthreads();
    const double ipi = 0.31830988618379067154;
    double Te = 0.0;
    for (int q = 0; q < NWAVE; ++q) Te += tred[q];
    bool bad = !isfinite(Te);
    for (int idx = t; idx < 2 * N; idx += NT) {
      const int s = idx / N, i = idx - s * N;
      double v = 0.0;
      for (int q = 0; q < NWAVE; ++q) v += prt[(q * 2 + s) * N + i];
      if (ldos) ldos[((size_t)e * 2 + s) * N + i] = v * ipi;
    }
    if (t == 0) {
      T[e] = Te;
      if (info) {
        const int i0 = iters[2 * e], i1 = iters[2 * e + 1];
        qtx_info inf;
        inf.dec_iters = (i0 < 0 || i1 < 0) ? -1 : (i0 > i1 ? i0 : i1);
        inf.refine_steps = 0;
        inf.resid = 0.0;
        inf.fell_back_fp64 = 0;
        inf.flags = ((i0 < 0 || i1 < 0) ? QTX_FLAG_DEC_NOTCONV : 0) | (bad ? QTX_FLAG_NONFINITE : 0);
        info[e] = inf;
      }
    }
  }
}

// ------------------------------------------------------------- launchers
template <int M>
hipError_t launch_decimate(const Prob& P, const double* E, int nE, double eta, int sides, double tol,
                           int maxit, double2* scratch, int grid, double2* sig, double2* wf, double* sgn,
                           int* iters, hipStream_t st) {
  hipLaunchKernelGGL((k_decimate<M>), dim3(grid), dim3(NT), 0, st, P, E, nE, eta, sides, tol, maxit,
                     scratch, sig, wf, sgn, iters);
  return hipGetLastError();
}

template <typename R, int M>
hipError_t launch_sweep(const Prob& P, const double* E, int nE, double eta, const double2* sig,
                        const double2* wf, const double* sgn, const int* iters, void* ws, size_t ws_stride,
                        double* part, int grid, double* T, double* ldos, qtx_info* info, hipStream_t st) {
  hipLaunchKernelGGL((k_sweep<R, M>), dim3(grid), dim3(NT), 0, st, P, E, nE, eta, sig, wf, sgn, iters,
                     (typename vec2t<R>::type*)ws, ws_stride, part, T, ldos, info);
  return hipGetLastError();
}

hipError_t run_decimate(int M, const Prob& P, const double* E, int nE, double eta, int sides, double tol,
                        int maxit, double2* scratch, int grid, double2* sig, double2* wf, double* sgn,
                        int* iters, hipStream_t st) {
  switch (M) {
    case 16: return launch_decimate<16>(P, E, nE, eta, sides, tol, maxit, scratch, grid, sig, wf, sgn, iters, st);
    case 32: return launch_decimate<32>(P, E, nE, eta, sides, tol, maxit, scratch, grid, sig, wf, sgn, iters, st);
    case 48: return launch_decimate<48>(P, E, nE, eta, sides, tol, maxit, scratch, grid, sig, wf, sgn, iters, st);
    case 64: return launch_decimate<64>(P, E, nE, eta, sides, tol, maxit, scratch, grid, sig, wf, sgn, iters, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t run_sweep(int M, bool fp32, const Prob& P, const double* E, int nE, double eta, const double2* sig,
                     const double2* wf, const double* sgn, const int* iters, void* ws, size_t ws_stride,
                     double* part, int grid, double* T, double* ldos, qtx_info* info, hipStream_t st) {
#define QTX_SWEEP(RR, MM) \
  return launch_sweep<RR, MM>(P, E, nE, eta, sig, wf, sgn, iters, ws, ws_stride, part, grid, T, ldos, info, st)
  if (!fp32) {
    switch (M) {
      case 16: QTX_SWEEP(double, 16);
      case 32: QTX_SWEEP(double, 32);
      case 48: QTX_SWEEP(double, 48);
      case 64: QTX_SWEEP(double, 64);
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (M) {
      case 16: QTX_SWEEP(float, 16);
      case 32: QTX_SWEEP(float, 32);
      case 48: QTX_SWEEP(float, 48);
      case 64: QTX_SWEEP(float, 64);
      default: return hipErrorInvalidValue;
    }
  }
#undef QTX_SWEEP
}

}  // namespace qtx
