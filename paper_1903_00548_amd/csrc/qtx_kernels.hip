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
// Blocked Gauss-Jordan elimination with partial pivoting (no physical row
// exchanges; the permutation is undone on the way out).  For each panel of
// 16 columns one wave eliminates the panel in registers (one matrix row per
// lane, pivot search by a DPP max reduction, no workgroup barrier), leaving
// in the panel G = E e_p, the panel transform applied to the unit vectors of
// its pivot rows.  Every other column x is then updated by
//   x' = x (pivot rows of the panel zeroed) + G y,   y_jj = x[p_jj],
// as 16x16 complex MFMA tiles shared by all waves.

template <typename R, int M> struct BGJ {
  int piv[M];        // pivot row chosen for column j
  int pinv[M];
  int ppanel[M];     // panel in which row r became a pivot, -1 before
  cpx<R> prow[16];   // pivot row of the current step (panel part)
};

// Wave-level elimination of panel k (columns 16k..16k+15) of the LDS matrix.
// The step loop is unrolled (static column index) with a scheduling barrier
// after every step so that steps do not interleave; the pivot lane
// publishes the already scaled pivot row, and the pivot row itself is
// produced by the same fused multiply-subtract as the others (base 0,
// factor -1).
template <typename R, int M>
__device__ void gj_panel(cpx<R>* mat, int S, int k, BGJ<R, M>& sc) {
  constexpr int RL = (M + 63) / 64;  // rows per lane
  const int lane = threadIdx.x & 63;
  cpx<R> pr[RL][16];
  bool used[RL];
#pragma unroll
  for (int q = 0; q < RL; ++q) {
    const int r = lane + 64 * q;
    const bool ok = r < M;
#pragma unroll
    for (int c = 0; c < 16; ++c) pr[q][c] = ok ? mat[r * S + 16 * k + c] : mk<R>(0, 0);
    used[q] = !ok || sc.ppanel[r] >= 0;
  }
#pragma unroll
  for (int jj = 0; jj < 16; ++jj) {
    uint32_t key = 0;
#pragma unroll
    for (int q = 0; q < RL; ++q)
      if (!used[q]) {
        const uint32_t kq = pivot_key32(pr[q][jj], lane + 64 * q);
        key = kq > key ? kq : key;
      }
    key = wave_max_u32(key);
    const int p = 255 - (int)(key & 0xff);
    const int pl = p & 63, pq = p >> 6;
    bool isp[RL];
    cpx<R> f[RL];
#pragma unroll
    for (int q = 0; q < RL; ++q) {
      isp[q] = (q == pq) && (lane == pl);
      f[q] = isp[q] ? mk<R>(-1, 0) : pr[q][jj];
    }
#pragma unroll
    for (int q = 0; q < RL; ++q)
      if (isp[q]) {
        const cpx<R> inv = cinv(pr[q][jj]);
#pragma unroll
        for (int c = 0; c < 16; ++c) sc.prow[c] = (c == jj) ? inv : cmul(pr[q][c], inv);
      }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const cpx<R> pvc = sc.prow[c];
#pragma unroll
      for (int q = 0; q < RL; ++q) {
        const cpx<R> base = (c == jj || isp[q]) ? mk<R>(0, 0) : pr[q][c];
        pr[q][c] = cfms(base, f[q], pvc);
      }
    }
#pragma unroll
    for (int q = 0; q < RL; ++q)
      if (isp[q]) used[q] = true;
    if (lane == 0) {
      sc.piv[16 * k + jj] = p;
      sc.ppanel[p] = k;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int q = 0; q < RL; ++q) {
    const int r = lane + 64 * q;
    if (r < M)
#pragma unroll
      for (int c = 0; c < 16; ++c) mat[r * S + 16 * k + c] = pr[q][c];
  }
}

// One 16x16 output tile of the panel update: X[ti, tc] <- masked X + G Y.
template <typename R, int M, class XLoad, class XStore>
__device__ __forceinline__ void gj_update_tile(const cpx<R>* mat, int S, int k, const cpx<R>* Y, int ldy, int ycol,
                                               int ti, const BGJ<R, M>& sc, XLoad xl, XStore xs) {
  ctile<R> acc[1];
  tiles_foreach<R, 1>(acc, 0, [&](int row, int col, int, int r) {
    const int gr = 16 * ti + row;
    cpx<R> v = sc.ppanel[gr] == k ? mk<R>(0, 0) : xl(gr, col);
    acc[0].re[r] = v.re;
    acc[0].im[r] = v.im;
  });
  cgemm_col<R, 1, 1>(acc, ALds<R>{mat + 16 * ti * S + 16 * k, S}, BLds<R>{Y + ycol, ldy}, 0);
  tiles_foreach<R, 1>(acc, 0, [&](int row, int col, int, int r) {
    xs(16 * ti + row, col, mk<R>(acc[0].re[r], acc[0].im[r]));
  });
}

// In-place inverse of the M x M LDS matrix (row stride S); Y is LDS scratch
// of 16 x M.  Ends with a barrier.
template <typename R, int M>
__device__ void gj_inverse(cpx<R>* mat, int S, cpx<R>* Y, BGJ<R, M>& sc) {
  constexpr int NP = M / 16, MT = M / 16;
  const int t = threadIdx.x, w = t >> 6;
  if (t < M) sc.ppanel[t] = -1;
  __syncthreads();
  for (int k = 0; k < NP; ++k) {
    if (w == 0) gj_panel<R, M>(mat, S, k, sc);
    __syncthreads();
    for (int idx = t; idx < 16 * M; idx += NT) {
      const int jj = idx / M, c = idx - jj * M;
      if ((c >> 4) != k) Y[idx] = mat[sc.piv[16 * k + jj] * S + c];
    }
    __syncthreads();
    for (int tile = w; tile < MT * (NP - 1); tile += NWAVE) {
      const int ti = tile % MT, tcx = tile / MT, tc = tcx + (tcx >= k ? 1 : 0);
      gj_update_tile<R, M>(
          mat, S, k, Y, M, 16 * tc, ti, sc,
          [&](int row, int col) { return mat[row * S + 16 * tc + col]; },
          [&](int row, int col, cpx<R> v) { mat[row * S + 16 * tc + col] = v; });
    }
    __syncthreads();
  }
  if (t < M) sc.pinv[sc.piv[t]] = t;
  __syncthreads();
  constexpr int b = M / 16;
  const int gr = t >> 4, gc = t & 15;
  cpx<R> a[b][b];
#pragma unroll
  for (int rr = 0; rr < b; ++rr)
#pragma unroll
    for (int cc = 0; cc < b; ++cc) a[rr][cc] = mat[(b * gr + rr) * S + b * gc + cc];
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < b; ++rr)
#pragma unroll
    for (int cc = 0; cc < b; ++cc) mat[sc.pinv[b * gr + rr] * S + sc.piv[b * gc + cc]] = a[rr][cc];
  __syncthreads();
}

// Blocked LU solve eps * X = B with partial pivoting (implicit row order).
// eps (M x M) lives in LDS (row stride S), B (M x 2M, leading dimension 2M)
// in global memory and is transformed in place; the solution rows are
// written un-permuted to out (M x 2M).  Y is LDS scratch of 16 x 3M.
// Panel factorisation on one wave (rows already chosen as pivots are
// frozen), then per panel: gather the pivot rows of the live columns,
// forward substitution with the unit lower 16x16 block, and the trailing
// update of the remaining rows as masked MFMA tiles; finally the block
// back substitution with the upper triangular factor.  Ends with a barrier.
template <int M>
__device__ void lu_panel(cpx<double>* eps, int S, int k, BGJ<double, M>& sc) {
  const int lane = threadIdx.x & 63;
  cpx<double> pr[16];
  const bool ok = lane < M;
  bool used = !ok || sc.ppanel[lane] >= 0;
#pragma unroll
  for (int c = 0; c < 16; ++c) pr[c] = ok ? eps[lane * S + 16 * k + c] : mk<double>(0, 0);
#pragma unroll 1
  for (int jj = 0; jj < 16; ++jj) {
    cpx<double> f = pr[0];
#pragma unroll
    for (int c = 1; c < 16; ++c)
      if (c == jj) f = pr[c];
    const uint32_t key = used ? 0u : pivot_key32(f, lane);
    const uint32_t kmax = wave_max_u32(key);
    const int p = 255 - (int)(kmax & 0xff);
    const cpx<double> pvt = mk<double>(readlane_d(f.re, p), readlane_d(f.im, p));
    if (lane == p)
#pragma unroll
      for (int c = 0; c < 16; ++c) sc.prow[c] = pr[c];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const bool elim = !used && lane != p;
    const cpx<double> l = cmul(f, cinv(pvt));
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      if (c > jj && elim) pr[c] = cfms(pr[c], l, sc.prow[c]);
      if (c == jj && elim) pr[c] = l;
    }
    if (lane == p) used = true;
    if (lane == 0) {
      sc.piv[16 * k + jj] = p;
      sc.ppanel[p] = k;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  if (ok)
#pragma unroll
    for (int c = 0; c < 16; ++c) eps[lane * S + 16 * k + c] = pr[c];
}

// A operand: rows of the LDS matrix restricted to columns [c0, c0+16); rows
// whose ppanel is >= 0 and <= kmax read as zero (frozen rows).
struct ALdsMask {
  const cpx<double>* p; int S; int c0; const int* ppanel; int kmax; int kmin;
  __device__ __forceinline__ cpx<double> get(int row, int k) const {
    const int pp = ppanel[row];
    const bool live = kmin < 0 ? !(pp >= 0 && pp <= kmax) : (pp >= 0 && pp < kmin);
    return live ? p[row * S + c0 + k] : mk<double>(0, 0);
  }
};

template <int M>
__device__ void lu_solve(cpx<double>* eps, int S, double2* B, double2* out, cpx<double>* Y, BGJ<double, M>& sc) {
  constexpr int NP = M / 16, MT = M / 16, W = 3 * M, LB = 2 * M;
  static_assert(3 * M - 16 <= NT, "one live column per thread");
  const int t = threadIdx.x, w = t >> 6;
  if (t < M) sc.ppanel[t] = -1;
  __syncthreads();
  // ---- forward: P A = L U, B <- L^-1 P B
  for (int k = 0; k < NP; ++k) {
    if (w == 0) lu_panel<M>(eps, S, k, sc);
    __syncthreads();
    const int c0 = 16 * (k + 1);          // first live eps column
    const int nl = M - c0 + LB;           // live columns: eps [c0, M), then B
    for (int idx = t; idx < 16 * nl; idx += NT) {
      const int jj = idx / nl, c = idx - jj * nl;
      const int p = sc.piv[16 * k + jj];
      Y[jj * W + c] = (c < M - c0) ? eps[p * S + c0 + c] : ldd(B + (size_t)p * LB + (c - (M - c0)));
    }
    __syncthreads();
    // unit lower 16x16 forward substitution, one live column per thread
    // (nl <= 3M - 16 <= NT; a loop here would let the compiler hoist all
    // 120 loads of the triangular block out of it)
    if (t < nl) {
      const int c = t;
      cpx<double> y[16];
#pragma unroll
      for (int a = 0; a < 16; ++a) y[a] = Y[a * W + c];
      // column-oriented; the scheduling barriers keep the LDS loads of one
      // column of L in flight at a time (otherwise all 120 are hoisted)
#pragma unroll
      for (int b = 0; b < 15; ++b) {
#pragma unroll
        for (int a = b + 1; a < 16; ++a) y[a] = cfms(y[a], eps[sc.piv[16 * k + a] * S + 16 * k + b], y[b]);
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int a = 0; a < 16; ++a) Y[a * W + c] = y[a];
      if (c < M - c0) {
#pragma unroll
        for (int a = 0; a < 16; ++a) eps[sc.piv[16 * k + a] * S + c0 + c] = y[a];
      } else {
#pragma unroll
        for (int a = 0; a < 16; ++a)
          B[(size_t)sc.piv[16 * k + a] * LB + (c - (M - c0))] = make_double2(y[a].re, y[a].im);
      }
    }
    __syncthreads();
    // trailing update of the rows that are not pivots yet
    const int ncol = (M - c0) / 16 + 2 * NP;
    for (int tile = w; tile < MT * ncol; tile += NWAVE) {
      const int ti = tile % MT, tcx = tile / MT;
      ctile<double> acc[1];
      const bool is_eps = tcx < (M - c0) / 16;
      const int xc = is_eps ? c0 + 16 * tcx : 16 * (tcx - (M - c0) / 16);
      tiles_foreach<double, 1>(acc, 0, [&](int row, int col, int, int r) {
        const int gr = 16 * ti + row;
        cpx<double> v = is_eps ? eps[gr * S + xc + col] : ldd(B + (size_t)gr * LB + xc + col);
        acc[0].re[r] = -v.re;
        acc[0].im[r] = -v.im;
      });
      // acc = -x + L y  (then negated on store): x - L y
      cgemm_col<double, 1, 1>(acc, ALdsMask{eps + 16 * ti * S, S, 16 * k, sc.ppanel + 16 * ti, k, -1},
                              BLds<double>{Y + 16 * tcx, W}, 0);
      tiles_foreach<double, 1>(acc, 0, [&](int row, int col, int, int r) {
        const int gr = 16 * ti + row;
        const cpx<double> v = mk<double>(-acc[0].re[r], -acc[0].im[r]);
        if (is_eps) eps[gr * S + xc + col] = v;
        else B[(size_t)gr * LB + xc + col] = make_double2(v.re, v.im);
      });
    }
    __syncthreads();
  }
  // ---- backward: U X = B, panels from the last one
  for (int k = NP - 1; k >= 0; --k) {
    if (t < LB) {
      const int c = t;
      cpx<double> y[16];
#pragma unroll
      for (int a = 0; a < 16; ++a) y[a] = ldd(B + (size_t)sc.piv[16 * k + a] * LB + c);
#pragma unroll
      for (int b = 15; b >= 0; --b) {
        y[b] = cmul(y[b], cinv(eps[sc.piv[16 * k + b] * S + 16 * k + b]));
#pragma unroll
        for (int a = 0; a < b; ++a) y[a] = cfms(y[a], eps[sc.piv[16 * k + a] * S + 16 * k + b], y[b]);
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int a = 0; a < 16; ++a) {
        Y[a * W + c] = y[a];
        B[(size_t)sc.piv[16 * k + a] * LB + c] = make_double2(y[a].re, y[a].im);
      }
    }
    __syncthreads();
    if (k > 0) {
      // rows that became pivots in earlier panels: x -= U[:, panel k] y
      for (int tile = w; tile < MT * 2 * NP; tile += NWAVE) {
        const int ti = tile % MT, tb = tile / MT;
        ctile<double> acc[1];
        tiles_foreach<double, 1>(acc, 0, [&](int row, int col, int, int r) {
          cpx<double> v = ldd(B + (size_t)(16 * ti + row) * LB + 16 * tb + col);
          acc[0].re[r] = -v.re;
          acc[0].im[r] = -v.im;
        });
        cgemm_col<double, 1, 1>(acc, ALdsMask{eps + 16 * ti * S, S, 16 * k, sc.ppanel + 16 * ti, 0, k},
                                BLds<double>{Y + 16 * tb, W}, 0);
        tiles_foreach<double, 1>(acc, 0, [&](int row, int col, int, int r) {
          B[(size_t)(16 * ti + row) * LB + 16 * tb + col] = make_double2(-acc[0].re[r], -acc[0].im[r]);
        });
      }
      __syncthreads();
    }
  }
  for (int idx = t; idx < M * LB; idx += NT) {
    const int j = idx / LB, c = idx - j * LB;
    out[idx] = B[(size_t)sc.piv[j] * LB + c];
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
// by an LU solve with partial pivoting, not from an explicit inverse (nor a
// blocked Gauss-Jordan, which inverts its 16x16 pivot blocks explicitly):
// those lose up to two extra digits when D0 is ill-conditioned.
template <int M>
__global__ __launch_bounds__(NT, 2) void k_decimate(Prob P, const double* E, int nE, double eta, int sides,
                                                 double tol, int maxit, double2* scratch, double2* sig,
                                                 double2* wf, double* sgn, int* iters) {
  constexpr int MT = M / 16, MM = M * M;
  constexpr int S = M + 1;
  __shared__ cpx<double> epsL[M * S];
  __shared__ cpx<double> Ysc[16 * 3 * M];
  __shared__ BGJ<double, M> sc;
  __shared__ LDLScratch<M> lsc;
  __shared__ double red[2][NWAVE];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  double2* ws = scratch + (size_t)blockIdx.x * 11 * MM;
  double2* eps = ws;
  double2* esL = ws + MM;
  double2* esR = ws + 2 * MM;
  double2* al[2] = {ws + 3 * MM, ws + 5 * MM};
  double2* be[2] = {ws + 4 * MM, ws + 6 * MM};
  double2* g = ws + 7 * MM;    // M x 2M: solution [g alpha | g beta]
  double2* rhs = ws + 9 * MM;  // M x 2M: right-hand side being eliminated
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
      for (int idx = t; idx < MM; idx += NT) {
        const int r = idx / M, c = idx - r * M;
        epsL[r * S + c] = ldd(eps + idx);
        rhs[r * 2 * M + c] = al[cur][idx];
        rhs[r * 2 * M + M + c] = be[cur][idx];
      }
      __syncthreads();
      lu_solve<M>(epsL, S, rhs, g, Ysc, sc);
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
__global__ __launch_bounds__(NT, 2) void k_sweep(Prob P, const double* E, int nE, double eta,
                                              const double2* sig, const double2* wf, const double* sgn,
                                              const int* iters, typename vec2t<R>::type* ws, size_t ws_stride,
                                              double* part, double* T, double* ldos, qtx_info* info) {
  typedef typename vec2t<R>::type V2;
  constexpr int MT = M / 16, MM = M * M, S = M + 1, LD = 2 * M;
  __shared__ cpx<R> mat[M * S];
  __shared__ cpx<R> Ysc[16 * M];
  __shared__ BGJ<R, M> sc;
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
      gj_inverse<R, M>(mat, S, Ysc, sc);
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
