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
// exchanges; the permutation is undone on the way out).  Each panel of 16
// columns is eliminated in registers by the four waves together (one
// matrix row per lane, four panel columns per wave), leaving in the panel
// G = E e_p, the panel transform applied to the unit vectors of its pivot
// rows.  Every other column x is then updated by
//   x' = x (pivot rows of the panel zeroed) + G y,   y_jj = x[p_jj],
// as 16x16 complex MFMA tiles shared by all waves.

template <typename R, int M> struct BGJ {
  int piv[M];        // pivot row chosen for column j
  int pinv[M];
  int ppanel[M];     // panel in which row r became a pivot, -1 before
};

// Panel width of the Gauss-Jordan elimination: 16 columns when the matrix
// is in LDS; 32 when it lives in global memory (M > 64), which halves the
// read-modify-write passes of the trailing update over the matrix and
// doubles the MFMA work per tile loaded.
template <int M> constexpr int gj_pw() { return sweep_default_pw(M); }

// LDS scratch (complex elements) that gj_inverse needs beside the matrix:
// the compacted pivot rows of the panel update, and during the panel the
// double-buffered row multipliers.
template <int M, int PW = gj_pw<M>()> constexpr int gj_scratch() {
  return PW * (M - PW) > 2 * 64 * ((M + 63) / 64) ? PW * (M - PW) : 2 * 64 * ((M + 63) / 64);
}

// Elimination of panel k (columns PW k .. PW k + PW - 1, PW = gj_pw<M>())
// of the matrix; wave w holds columns PW k + CW w .. PW k + CW w + CW - 1
// (CW = PW / 4) of every row (rows lane, lane + 64, ...).
// Step jj: the wave owning column jj finds the pivot row p (DPP max over
// the unused rows), forms the row multipliers m_r = x_rj / x_pj (the pivot
// row takes -1 / x_pj) and publishes them and p through LDS; after one
// barrier every wave reads the pivot row's entries of its own columns from
// the lane that holds row p and updates
//   x_rc <- x_rc - m_r x_pc  (c != j, with x_pc read as 0 in row p),
//   x_rj <- -m_r.
// The multipliers alternate between two LDS buffers, so that one barrier
// per step orders both the publication and the reuse.
template <typename R, int M, int PW>
__device__ __forceinline__ void gj_panel(cpx<R>* mat, int S, int k, BGJ<R, M>& sc, cpx<R>* mb) {
  constexpr int RL = (M + 63) / 64;             // rows per lane
  constexpr int CW = PW / NWAVE;
  static_assert(M <= 128, "pivot keys carry 8-bit row indices");
  const int lane = lane_id(), w = threadIdx.x >> 6;
  const int c0 = PW * k + CW * w;
  cpx<R> pr[RL][CW];
  bool used[RL];
#pragma unroll
  for (int q = 0; q < RL; ++q) {
    const int r = lane + 64 * q;
    const bool ok = r < M;
#pragma unroll
    for (int c = 0; c < CW; ++c) pr[q][c] = ok ? mat[r * S + c0 + c] : mk<R>(0, 0);
    used[q] = true;
    if (ok) used[q] = sc.ppanel[r] >= 0;
  }
#pragma unroll
  for (int jj = 0; jj < PW; ++jj) {
    const int owner = jj / CW, cj = jj % CW;
    cpx<R>* mbj = mb + (jj & 1) * 64 * RL;
    if (w == owner) {
      uint32_t key = 0;
#pragma unroll
      for (int q = 0; q < RL; ++q)
        if (!used[q]) {
          const uint32_t kq = pivot_key32(pr[q][cj], lane + 64 * q);
          key = kq > key ? kq : key;
        }
      key = wave_max_u32(key);
      const int p = 255 - (int)(key & 0xff), pl = RL == 1 ? p : p & 63, pq = RL == 1 ? 0 : p >> 6;
      cpx<R> pvt = mk<R>(0, 0);
#pragma unroll
      for (int q = 0; q < RL; ++q)
        if (q == pq) pvt = mk<R>(readlane_d(pr[q][cj].re, pl), readlane_d(pr[q][cj].im, pl));
      const cpx<R> inv = cinv(pvt);
#pragma unroll
      for (int q = 0; q < RL; ++q)
        mbj[lane + 64 * q] = (q == pq && lane == pl) ? mk<R>(-inv.re, -inv.im) : cmul(pr[q][cj], inv);
      if (lane == 0) {
        sc.piv[PW * k + jj] = p;
        sc.ppanel[p] = k;
      }
    }
    __syncthreads();
    const int p = __builtin_amdgcn_readfirstlane(sc.piv[PW * k + jj]);
    const int pl = RL == 1 ? p : p & 63, pq = RL == 1 ? 0 : p >> 6;
    cpx<R> m[RL];
#pragma unroll
    for (int q = 0; q < RL; ++q) m[q] = mbj[lane + 64 * q];
    cpx<R> prow[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      prow[c] = mk<R>(0, 0);
#pragma unroll
      for (int q = 0; q < RL; ++q)
        if (q == pq) prow[c] = mk<R>(readlane_d(pr[q][c].re, pl), readlane_d(pr[q][c].im, pl));
    }
#pragma unroll
    for (int q = 0; q < RL; ++q) {
      const bool isp = (q == pq) && (lane == pl);
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        if (c == cj && w == owner) {
          pr[q][c] = mk<R>(-m[q].re, -m[q].im);
        } else {
          const cpx<R> base = isp ? mk<R>(0, 0) : pr[q][c];
          pr[q][c] = cfms(base, m[q], prow[c]);
        }
      }
      if (isp) used[q] = true;
    }
  }
#pragma unroll
  for (int q = 0; q < RL; ++q) {
    const int r = lane + 64 * q;
    if (r < M)
#pragma unroll
      for (int c = 0; c < CW; ++c) mat[r * S + c0 + c] = pr[q][c];
  }
}

// Panel update x' = (x with the panel's pivot rows zeroed) + G y for every
// 16x16 tile outside panel k (G: the PW panel columns, y: the compacted
// pivot rows in Y, row stride M - PW).  The tiles are dealt round-robin to the
// waves; each wave runs its tiles in groups of at most four through one
// interleaved MFMA loop, so that up to eight accumulator chains are in
// flight.  A group's surplus slots recompute a valid tile and do not store.
// Above 64 (matrix in global memory) the tiles go in groups of RG along a
// tile row instead, when the rows split into whole groups and the groups
// evenly over the waves: a group then loads its panel operand once per
// step for all its tiles, where the round-robin deal has each tile of a
// tile row read it again from the caches.
template <int M, int PW> constexpr int gj_row_group() {
  constexpr int W = M / 16 - PW / 16, NG3 = (M / 16) * W / 3, NG2 = (M / 16) * W / 2;
  if (M <= 64 || W <= 0) return 0;
  if (W % 3 == 0 && NG3 % NWAVE == 0) return 3;
  if (W % 2 == 0 && NG2 % NWAVE == 0) return 2;
  return 0;
}

template <typename R, int M, int PW>
__device__ __forceinline__ void gj_update(cpx<R>* mat, int S, int k, const cpx<R>* Y, const BGJ<R, M>& sc) {
  constexpr int PT = PW / 16;
  constexpr int MT = M / 16, NTILE = MT * (MT - PT), TPW = (NTILE + NWAVE - 1) / NWAVE, WY = M - PW;
  constexpr int GRP = TPW < 4 ? TPW : 4;
  constexpr int RG = gj_row_group<M, PW>();
  if constexpr (RG > 0) {
    constexpr int WC = MT - PT, GPW = NTILE / RG / NWAVE;     // tile columns, groups per wave
    const int w = threadIdx.x >> 6, lane = lane_id(), g = lane >> 4, c = lane & 15;
#pragma unroll 1
    for (int j = 0; j < GPW; ++j) {
      const int t0 = (w + NWAVE * j) * RG;                   // first tile of the group (row-major)
      const int ti = t0 / WC, arow = 16 * ti;
      int bcol[RG], xcol[RG];
      ctile<R> acc[RG];
#pragma unroll
      for (int q = 0; q < RG; ++q) {
        const int tcx = t0 - ti * WC + q, tc = tcx + (tcx >= PT * k ? PT : 0);
        bcol[q] = 16 * tcx + c;
        xcol[q] = 16 * tc + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = arow + mf<R>::row(r, g);
          const cpx<R> v = sc.ppanel[row] == k ? mk<R>(0, 0) : mat[row * S + xcol[q]];
          acc[q].re[r] = v.re;
          acc[q].im[r] = v.im;
        }
      }
#pragma unroll
      for (int sl = 0; sl < 4 * PT; ++sl) {
        const int kk = 16 * (sl >> 2) + 4 * g + (sl & 3);
        const cpx<R> av = mat[(arow + c) * S + PW * k + kk];
        cpx<R> bv[RG];
#pragma unroll
        for (int q = 0; q < RG; ++q) bv[q] = Y[kk * WY + bcol[q]];
#pragma unroll
        for (int q = 0; q < RG; ++q) {
          acc[q].re = mf<R>::op(av.re, bv[q].re, acc[q].re);
          acc[q].im = mf<R>::op(av.re, bv[q].im, acc[q].im);
        }
#pragma unroll
        for (int q = 0; q < RG; ++q) {
          acc[q].re = mf<R>::op(-av.im, bv[q].im, acc[q].re);
          acc[q].im = mf<R>::op(av.im, bv[q].re, acc[q].im);
        }
      }
#pragma unroll
      for (int q = 0; q < RG; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          mat[(arow + mf<R>::row(r, g)) * S + xcol[q]] = mk<R>(acc[q].re[r], acc[q].im[r]);
    }
  } else if constexpr (NTILE > 0) {
    const int w = threadIdx.x >> 6, lane = lane_id(), g = lane >> 4, c = lane & 15;
#pragma unroll 1
    for (int q0 = 0; q0 < TPW; q0 += GRP) {
      int arow[GRP], bcol[GRP], xcol[GRP];
      bool keep[GRP];
      ctile<R> acc[GRP];
#pragma unroll
      for (int q = 0; q < GRP; ++q) {
        int tile = w + NWAVE * (q0 + q);
        keep[q] = (q0 + q < TPW) && tile < NTILE;
        tile = keep[q] ? tile : 0;
        const int ti = tile % MT, tcx = tile / MT, tc = tcx + (tcx >= PT * k ? PT : 0);
        arow[q] = 16 * ti;
        bcol[q] = 16 * tcx + c;
        xcol[q] = 16 * tc + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = arow[q] + mf<R>::row(r, g);
          const cpx<R> v = sc.ppanel[row] == k ? mk<R>(0, 0) : mat[row * S + xcol[q]];
          acc[q].re[r] = v.re;
          acc[q].im[r] = v.im;
        }
      }
#pragma unroll
      for (int sl = 0; sl < 4 * PT; ++sl) {
        const int kk = 16 * (sl >> 2) + 4 * g + (sl & 3);
        cpx<R> av[GRP], bv[GRP];
#pragma unroll
        for (int q = 0; q < GRP; ++q) {
          av[q] = mat[(arow[q] + c) * S + PW * k + kk];
          bv[q] = Y[kk * WY + bcol[q]];
        }
#pragma unroll
        for (int q = 0; q < GRP; ++q) {
          acc[q].re = mf<R>::op(av[q].re, bv[q].re, acc[q].re);
          acc[q].im = mf<R>::op(av[q].re, bv[q].im, acc[q].im);
        }
#pragma unroll
        for (int q = 0; q < GRP; ++q) {
          acc[q].re = mf<R>::op(-av[q].im, bv[q].im, acc[q].re);
          acc[q].im = mf<R>::op(av[q].im, bv[q].re, acc[q].im);
        }
      }
#pragma unroll
      for (int q = 0; q < GRP; ++q)
        if (keep[q])
#pragma unroll
          for (int r = 0; r < 4; ++r)
            mat[(arow[q] + mf<R>::row(r, g)) * S + xcol[q]] = mk<R>(acc[q].re[r], acc[q].im[r]);
    }
  }
}

// In-place Gauss-Jordan on the M x M matrix (row stride S; in LDS, or for
// M > 64 in the workgroup's global workspace); Y is LDS scratch of
// gj_scratch<M>() elements.  The result is the inverse up to the pivot order:
// A^-1[j][c] = mat[piv[j]][pinv[c]], so A^-1 B = P (mat (Q B)) with
// (Q B)[k] = B[piv[k]] and row r of the product landing in row pinv[r].
// Ends with a barrier.  The elimination is the latency-bound critical path
// of its workgroup, so its waves raise their issue priority over the other
// workgroup resident on the CU (which is then mostly in MFMA phases).
template <typename R, int M, int PW = gj_pw<M>()>
__device__ __forceinline__ void gj_inverse(cpx<R>* mat, int S, cpx<R>* Y, BGJ<R, M>& sc) {
  static_assert(PW == 16 || PW == 32, "panels of 16 or 32 columns");
  static_assert(M % PW == 0, "whole panels");
  constexpr int NP = M / PW;
  const int t = threadIdx.x;
  __builtin_amdgcn_s_setprio(2);
  if (t < M) sc.ppanel[t] = -1;
  __syncthreads();
  for (int k = 0; k < NP; ++k) {
    gj_panel<R, M, PW>(mat, S, k, sc, Y);
    __syncthreads();
    // pivot rows of the columns outside the panel, compacted (PW x (M-PW));
    // a single panel (M = PW) leaves nothing to update
    constexpr int WY = M - PW;
    if constexpr (WY > 0) {
      for (int idx = t; idx < PW * WY; idx += NT) {
        const int jj = idx / WY, cx = idx - jj * WY;
        const int c = cx + (cx >= PW * k ? PW : 0);
        Y[idx] = mat[sc.piv[PW * k + jj] * S + c];
      }
      __syncthreads();
      gj_update<R, M, PW>(mat, S, k, Y, sc);
      __syncthreads();
    }
  }
  if (t < M) sc.pinv[sc.piv[t]] = t;
  __syncthreads();
  __builtin_amdgcn_s_setprio(0);
}

// ------------------------------------------------ broadening factorisation
// Gamma = i (Sigma - Sigma^H) is Hermitian but only semi-definite up to
// O(eta) (the broadening also enters the non-orthogonal couplings), so it
// is factored as Gamma = W diag(s) W^H with s = +-1 by a diagonally pivoted
// LDL^H: at each step the remaining diagonal entry of largest magnitude d
// is eliminated, column k of W is the pivot column / sqrt|d| and s_k =
// sign(d).  Exactly zero remaining diagonals (padding) end the factorisation.
// The pivots come out in decreasing magnitude; *nh receives the number of
// leading columns whose pivot is at least tau times the first one (the
// columns that carry the weight of the injection).
template <int M> struct LDLScratch {
  cpx<double> col[M];
  double dg[M];
};

template <int M>
__device__ __forceinline__ void gamma_ldl(const double2* sig, double2* W, double* sg, double tau, int* nh,
                                          LDLScratch<M>& sc) {
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
  double d0 = 0.0;
  int cnt = 0;
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
    if (k == 0) d0 = fabs(d);
    if (fabs(d) >= tau * d0) cnt = k + 1;
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
  if (t == 0) *nh = cnt;
  __syncthreads();
}

// ------------------------------------------------------------ batch items
// A problem descriptor read from device memory with every field made
// wave-uniform, so that the addresses built from it stay scalar.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v) {
  const long long x = __double_as_longlong(v);
  const unsigned lo = (unsigned)uni((int)(x & 0xffffffff)), hi = (unsigned)uni((int)(x >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <class T> __device__ __forceinline__ T* uni(T* p) {
  const unsigned long long x = (unsigned long long)p;
  const unsigned lo = (unsigned)uni((int)(x & 0xffffffffull)), hi = (unsigned)uni((int)(x >> 32));
  return (T*)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ Prob load_prob(const Prob* pp) {
  Prob P;
  P.N = uni(pp->N);
  P.M = uni(pp->M);
  P.leadL = uni(pp->leadL);
  P.leadR = uni(pp->leadR);
  P.VL = uni(pp->VL);
  P.VR = uni(pp->VR);
  P.dHd = uni(pp->dHd);
  P.dHu = uni(pp->dHu);
  P.dSd = uni(pp->dSd);
  P.dSu = uni(pp->dSu);
  P.V = uni(pp->V);
  P.pot_mode = uni(pp->pot_mode);
  return P;
}

// One self-energy job of a decimation launch.  Single problem: jobs
// (energy, side), or one job per energy (side -1: both surfaces of one lead
// iteration) when both leads are the same; batch: the job list names item
// and side; self-energy cache: job j fills slot job_item[j] (both surfaces)
// for the lead job_lead[j] at the already shifted energy job_E[j].
struct DecJob {
  int e, side;
  const double2* lead;
  cpx<double> zx;          // E - V_lead + i eta
};
__device__ __forceinline__ DecJob dec_job(const Prob& P0, const BatchDesc& b, const double* E, double eta, int sides,
                                          int job) {
  DecJob J;
  if (b.job_E) {
    J.e = __builtin_amdgcn_readfirstlane(b.job_item[job]);
    J.side = -1;
    J.lead = uni(b.job_lead[job]);
    J.zx = mk<double>(b.job_E[job], eta);
    return J;
  }
  Prob P = P0;
  if (b.probs) {
    J.e = __builtin_amdgcn_readfirstlane(b.job_item[job]);
    J.side = __builtin_amdgcn_readfirstlane(b.job_side[job]);
    P = load_prob(b.probs + __builtin_amdgcn_readfirstlane(b.item_prob[J.e]));
  } else {
    J.e = job / sides;
    J.side = (sides == 2) ? (job % 2) : -1;
  }
  J.lead = (J.side == 1) ? P.leadR : P.leadL;
  J.zx = mk<double>(E[J.e] - ((J.side == 1) ? P.VR : P.VL), eta);
  return J;
}

// ------------------------------------------------ self-energy Newton step
// max(a, b), NaN if either is NaN
__device__ __forceinline__ double max_nan(double a, double b) { return (a != a) ? a : ((b != b || b > a) ? b : a); }

// Largest |re| + |im| over the workgroup with NaN propagated (a NaN
// anywhere makes the result NaN); every thread gets the same value.
// red: NWAVE doubles of LDS.  Two barriers.
__device__ __forceinline__ double block_max_nan(double v, double* red) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const double o = __shfl_xor(v, m, 64);
    v = (o != o || o > v) ? o : v;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int q = 1; q < NWAVE; ++q) r = (red[q] != red[q] || red[q] > r) ? red[q] : r;
  __syncthreads();
  return r;
}

// Each wave computes the column tiles tj = w, w + NWAVE, ... of an M x M
// product A B (FP64) into acc and hands every element to fn(idx, re, im).
template <int M, class AF, class BF, class F>
__device__ __forceinline__ void prod_cols(const AF& A, const BF& B, F fn) {
  constexpr int MT = M / 16;
  const int w = threadIdx.x >> 6;
#pragma unroll 1
  for (int tj = w; tj < MT; tj += NWAVE) {
    ctile<double> acc[MT];
#pragma unroll
    for (int ti = 0; ti < MT; ++ti) tzero(acc[ti]);
    cgemm_col<double, MT, MT>(acc, A, B, tj);
    tiles_foreach<double, MT>(acc, tj, [&](int row, int col, int ti, int r) {
      fn((unsigned)(row * M + col), acc[ti].re[r], acc[ti].im[r]);
    });
  }
}

// The doubling reaches a self-energy through a chain of eliminations whose
// rounding errors nothing corrects afterwards; within about a meV of a
// band edge of the lead the result then misses its fixed point
//   Sigma = A (D0 - Sigma)^-1 B     (right contact: A = U, B = L;
//                                     left contact:  A = L, B = U)
// by up to 1e-10 relative (Sec. "Contact self-energies": Sigma is the
// projection of the lead's outgoing Bloch modes, which this equation
// characterises), and the density of states there amplifies that error.
// The residual R = Sigma - A G B with G = (D0 - Sigma)^-1 is formed for
// every self-energy; where max|R| > tol max|Sigma| one Newton step
// Sigma += X follows, X solving the linearised fixed point
//   X - P X Q = -R,   P = A G,  Q = G B,
// a Stein equation, summed as the series X = sum_j P^j (-R) Q^j by
// doubling: X_0 = -R, X_{k+1} = X_k + P_k X_k Q_k, P_{k+1} = P_k^2,
// Q_{k+1} = Q_k^2, until a term no longer changes X (P and Q decay like
// the lead's Bloch factors, about 20 doublings at eta = 1e-6).  A
// correction that is not finite or not small against Sigma is dropped.
// ws: 7 M^2 complex doubles of free global workspace; mat, Y, sc: the
// Gauss-Jordan matrix, scratch and pivots; red: NWAVE doubles of LDS.
template <int M>
__device__ __forceinline__ void sigma_newton(double2* sig, const double2* lead, cpx<double> zx, int side, double tol,
                                             double2* ws, cpx<double>* mat, cpx<double>* Y, BGJ<double, M>& sc,
                                             double* red) {
  constexpr int MT = M / 16, MM = M * M, S = M + 1;
  const int t = threadIdx.x, w = t >> 6;
  const double2 *H00 = lead, *H01 = lead + MM, *S00 = lead + 2 * MM, *S01 = lead + 3 * MM;
  double2* Gn = ws;                 // G in natural row/column order
  double2* Q = ws + MM;
  double2* P = ws + 2 * MM;
  double2* X = ws + 3 * MM;
  double2* T1 = ws + 4 * MM;
  double2* P2 = ws + 5 * MM;
  double2* Q2 = ws + 6 * MM;
  double2* Bn = T1;                 // B in natural order until the doubling needs T1
  // D0 - Sigma into the working matrix, B (= L or U) into Bn, max|Sigma|
  double smax = 0.0;
  for (int idx = t; idx < MM; idx += NT) {
    const int r = idx / M, c = idx - r * M;
    const cpx<double> sv = ldd(S00 + idx), hv = ldd(H00 + idx), g = ldd(sig + idx);
    mat[r * S + c] = mk<double>(zx.re * sv.re - zx.im * sv.im - hv.re - g.re,
                                zx.re * sv.im + zx.im * sv.re - hv.im - g.im);
    smax = max_nan(smax, fabs(g.re) + fabs(g.im));
    if (side == 0) {                // U[r][c]
      const cpx<double> s1 = ldd(S01 + idx), h1 = ldd(H01 + idx);
      Bn[idx] = make_double2(zx.re * s1.re - zx.im * s1.im - h1.re, zx.re * s1.im + zx.im * s1.re - h1.im);
    } else {                        // L[c][r] from S01[r][c], H01[r][c] (coalesced read)
      const cpx<double> s1 = ldd(S01 + idx), h1 = ldd(H01 + idx);
      Bn[c * M + r] = make_double2(zx.re * s1.re + zx.im * s1.im - h1.re, zx.im * s1.re - zx.re * s1.im + h1.im);
    }
  }
  smax = block_max_nan(smax, red);
  gj_inverse<double, M>(mat, S, Y, sc);
  // Q = G B = P_r (mat (B rows in pivot order)), rows landing through pinv
#pragma unroll 1
  for (int tj = w; tj < MT; tj += NWAVE) {
    ctile<double> acc[MT];
#pragma unroll
    for (int ti = 0; ti < MT; ++ti) tzero(acc[ti]);
    cgemm_col<double, MT, MT>(acc, ALds<double>{mat, S}, BPerm<BGlob<double>>{BGlob<double>{Bn, M}, sc.piv}, tj);
    tiles_foreach<double, MT>(acc, tj, [&](int row, int col, int ti, int r) {
      Q[(unsigned)(sc.pinv[row] * M + col)] = make_double2(acc[ti].re[r], acc[ti].im[r]);
    });
  }
  for (int idx = t; idx < MM; idx += NT) {
    const int j = idx / M, c = idx - j * M;
    const cpx<double> v = mat[sc.piv[j] * S + sc.pinv[c]];
    Gn[idx] = make_double2(v.re, v.im);
  }
  __syncthreads();
  // A (= U or L) staged in the working matrix for the two products that use it
  for (int idx = t; idx < MM; idx += NT) {
    const int r = idx / M, c = idx - r * M;
    const cpx<double> s1 = ldd(S01 + idx), h1 = ldd(H01 + idx);
    if (side == 1)
      mat[r * S + c] = mk<double>(zx.re * s1.re - zx.im * s1.im - h1.re, zx.re * s1.im + zx.im * s1.re - h1.im);
    else
      mat[c * S + r] = mk<double>(zx.re * s1.re + zx.im * s1.im - h1.re, zx.im * s1.re - zx.re * s1.im + h1.im);
  }
  __syncthreads();
  auto store = [](double2* D) { return [D](unsigned idx, double re, double im) { D[idx] = make_double2(re, im); }; };
  const ALds<double> As{mat, S};
  // X_0 = -R = A Q - Sigma
  double cmax = 0.0;
  prod_cols<M>(As, BGlob<double>{Q, M}, [&](unsigned idx, double re, double im) {
    const double2 g = sig[idx];
    const double2 v = make_double2(re - g.x, im - g.y);
    X[idx] = v;
    cmax = max_nan(cmax, fabs(v.x) + fabs(v.y));
  });
  cmax = block_max_nan(cmax, red);
  if (!(cmax > tol * smax)) return;              // uniform; also for a non-finite residual
  prod_cols<M>(As, BGlob<double>{Gn, M}, store(P));                          // P = A G (A still staged)
  __syncthreads();
  // the A operand of every product staged in the working matrix
  auto stage = [&](const double2* src) {
    for (int idx = t; idx < MM; idx += NT) {
      const int r = idx / M, c = idx - r * M;
      const double2 v = src[idx];
      mat[r * S + c] = mk<double>(v.x, v.y);
    }
    __syncthreads();
  };
  double xmax = cmax;
#pragma unroll 1
  for (int k = 0; k < 64; ++k) {
    stage(P);
    prod_cols<M>(As, BGlob<double>{X, M}, store(T1));
    prod_cols<M>(As, BGlob<double>{P, M}, store(P2));
    __syncthreads();
    stage(T1);
    // X += T1 Q (a wave reads and writes only its own column tiles of X)
    double imax = 0.0, xm = 0.0;
    prod_cols<M>(As, BGlob<double>{Q, M}, [&](unsigned idx, double re, double im) {
      double2 v = X[idx];
      v.x += re;
      v.y += im;
      X[idx] = v;
      imax = max_nan(imax, fabs(re) + fabs(im));
      xm = max_nan(xm, fabs(v.x) + fabs(v.y));
    });
    __syncthreads();
    stage(Q);
    prod_cols<M>(As, BGlob<double>{Q, M}, store(Q2));
    imax = block_max_nan(imax, red);
    xmax = block_max_nan(xm, red);
    double2* tp = P; P = P2; P2 = tp;
    tp = Q; Q = Q2; Q2 = tp;
    if (!(imax > 1e-17 * xmax)) break;           // converged, or non-finite
  }
  if (!(xmax <= 1e-3 * smax)) return;            // not a small correction (or NaN): keep Sigma
  for (int idx = t; idx < MM; idx += NT) {
    double2 g = sig[idx];
    const double2 x = X[idx];
    g.x += x.x;
    g.y += x.y;
    sig[idx] = g;
  }
  __syncthreads();
}

// ------------------------------------------------------------- decimation
// Doubling elimination of the semi-infinite lead: with on-site e and
// couplings a (slab j -> j+1) and b (j+1 -> j), eliminating every other slab
// gives e' = e - a g b - b g a, a' = -a g a, b' = -b g b with g = e^-1; the
// surface of a right lead keeps only -a g b and that of a left lead only
// -b g a.  Sigma = D0 - (converged surface block).  Only e and the right
// surface eR are stored: the left surface is e + D0 - eR, so Sigma_L =
// eR - e and Sigma_R = D0 - eR.
// g [a | b] comes from the blocked Gauss-Jordan inverse; the product with
// the explicit inverse carries an error of order kappa(e) u, so when the
// estimate kappa_F = ||e||_F ||e^-1||_F exceeds rcond (always for rcond = 0)
// one step of iterative refinement, X <- X + e^-1 ([a | b] - e X), brings
// it back to the accuracy of an LU solve.  Well-conditioned doublings, most
// of them away from the lead's band edges, skip the step's two products.
// Two workgroups per CU at every block size: above 64 the working matrix
// lives in the global workspace, and the second workgroup on each SIMD
// hides part of its latency (at 128 the kernel spills a few registers
// and is still faster than at one workgroup per CU with no spill).  There
// the products also take their A operand through LDS in 16-column slices,
// loaded once per workgroup instead of once per wave and column tile.
template <int M>
__global__ __launch_bounds__(NT, 2) void k_decimate(Prob P0, BatchDesc b, const double* E, int nE, double eta,
                                                    int sides, DecOpts o, double2* scratch, double2* sig, double2* wf,
                                                    double* sgn, int* iters, int* nheavy) {
  const double tol = o.tol, rcond = o.rcond;
  const int maxit = o.maxit;
  constexpr int MT = M / 16, MM = M * M, S = M + 1, LB = 2 * M;
  constexpr bool BIG = M > 64;                    // working matrix in the global workspace
  // above 64 the A operand of every product comes through LDS in 16-column
  // slices (the elimination scratch, free during the products)
  constexpr bool STAGE = BIG;
  static_assert(!STAGE || gj_scratch<M>() >= M * kStageStride, "staging slice exceeds the scratch");
  static_assert(!STAGE || (2 * MT) % NWAVE == 0, "staged products need the same tile count on every wave");
  __shared__ __align__(16) cpx<double> mat_l[BIG ? 1 : M * S];
  __shared__ __align__(16) union {
    cpx<double> y[gj_scratch<M>()];
    LDLScratch<M> ldl;
  } u;
  __shared__ BGJ<double, M> sc;
  __shared__ double red[2][NWAVE];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  double2* ws = scratch + (size_t)blockIdx.x * dec_ws_elems(M);
  // C += A B over column tile tj, staged or direct
  auto prod = [&](ctile<double>(&acc)[MT], const auto& A, const auto& B, int tj) {
    if constexpr (STAGE) cgemm_col_staged<double, MT>(acc, A, B, tj, u.y);
    else cgemm_col<double, MT, MT>(acc, A, B, tj);
  };
  cpx<double>* mat;
  if constexpr (BIG) mat = (cpx<double>*)(ws + 8 * MM);
  else mat = mat_l;
  // the part touched by every doubling (e, eR, [a | b], X: 6 M^2) is kept
  // together so that the resident workgroups' share fits the last-level
  // cache; the residual is used only by the doublings that refine
  double2* eps = ws;
  double2* esR = ws + MM;
  double2* AB = ws + 2 * MM;                      // [a | b], M x 2M, updated in place
  double2* X = ws + 4 * MM;                       // [g a | g b]
  double2* Rr = ws + 6 * MM;                      // residual
  const int njobs = b.probs ? b.njobs : nE * sides;
  for (int job = blockIdx.x; job < njobs; job += gridDim.x) {
    const DecJob J = dec_job(P0, b, E, eta, sides, job);
    const int e = J.e, side = J.side;
    const double2* lead = J.lead;
    const double2 *H00 = lead, *H01 = lead + MM, *S00 = lead + 2 * MM, *S01 = lead + 3 * MM;
    const cpx<double> zx = J.zx;
    double scl = 0.0;
    for (int idx = t; idx < MM; idx += NT) {
      const int r = idx / M, c = idx - r * M;
      cpx<double> s = ldd(S00 + idx), h = ldd(H00 + idx);
      double2 d0 = make_double2(zx.re * s.re - zx.im * s.im - h.re, zx.re * s.im + zx.im * s.re - h.im);
      s = ldd(S01 + idx); h = ldd(H01 + idx);
      double2 uu = make_double2(zx.re * s.re - zx.im * s.im - h.re, zx.re * s.im + zx.im * s.re - h.im);
      s = ldd(S01 + c * M + r); h = ldd(H01 + c * M + r);
      double2 ll = make_double2(zx.re * s.re + zx.im * s.im - h.re, zx.im * s.re - zx.re * s.im + h.im);
      eps[idx] = d0; esR[idx] = d0;
      AB[r * LB + c] = uu;
      AB[r * LB + M + c] = ll;
      scl = fmax(scl, fabs(d0.x) + fabs(d0.y));
    }
    scl = wave_maxd(scl);
    if (lane == 0) red[0][w] = scl;
    __syncthreads();
    scl = 0.0;
    for (int q = 0; q < NWAVE; ++q) scl = fmax(scl, red[0][q]);
    int it = 0;
    bool conv = false;
    for (it = 1; it <= maxit; ++it) {
      double ne2 = 0.0;
      for (int idx = t; idx < MM; idx += NT) {
        const int r = idx / M, c = idx - r * M;
        const cpx<double> v = ldd(eps + idx);
        mat[r * S + c] = v;
        ne2 += v.re * v.re + v.im * v.im;
      }
      __syncthreads();
      gj_inverse<double, M>(mat, S, u.y, sc);
      // kappa_F from the two sums of squares (the inverse is stored with its
      // rows permuted, which leaves its norm unchanged); every thread sums
      // the same partials in the same order, so the decision is uniform
      bool refine_x = true;
      if (rcond > 0.0) {
        double ng2 = 0.0;
        for (int idx = t; idx < MM; idx += NT) {
          const int r = idx / M, c = idx - r * M;
          const cpx<double> v = mat[r * S + c];
          ng2 += v.re * v.re + v.im * v.im;
        }
        ne2 = wave_sum(ne2);
        ng2 = wave_sum(ng2);
        if (lane == 0) { red[0][w] = ne2; red[1][w] = ng2; }
        __syncthreads();
        ne2 = 0.0; ng2 = 0.0;
        for (int q = 0; q < NWAVE; ++q) { ne2 += red[0][q]; ng2 += red[1][q]; }
        refine_x = !(ne2 * ng2 <= rcond * rcond);      // a non-finite estimate refines
      }
      // X = e^-1 [a | b], then the refinement step if needed; each wave owns
      // whole column tiles of X, so the three products need no barrier
#pragma unroll 1
      for (int tj = w; tj < 2 * MT; tj += NWAVE) {
        ctile<double> acc[MT];
#pragma unroll
        for (int ti = 0; ti < MT; ++ti) tzero(acc[ti]);
        prod(acc, ALds<double>{mat, S}, BPerm<BGlob<double>>{BGlob<double>{AB, LB}, sc.piv}, tj);
        tiles_foreach<double, MT>(acc, tj, [&](int row, int col, int ti, int r) {
          X[(unsigned)(sc.pinv[row] * LB + col)] = make_double2(acc[ti].re[r], acc[ti].im[r]);
        });
        if (!refine_x) continue;
        __threadfence_block();
        // residual R = [a | b] - e X
        tiles_foreach<double, MT>(acc, tj, [&](int row, int col, int ti, int r) {
          const double2 v = AB[(unsigned)(row * LB + col)];
          acc[ti].re[r] = v.x;
          acc[ti].im[r] = v.y;
        });
        prod(acc, AGlob<double>{eps, M, -1.0}, BGlob<double>{X, LB}, tj);
        tiles_foreach<double, MT>(acc, tj, [&](int row, int col, int ti, int r) {
          Rr[(unsigned)(row * LB + col)] = make_double2(acc[ti].re[r], acc[ti].im[r]);
        });
        __threadfence_block();
        // X += e^-1 R (rows through the pivot order)
        tiles_foreach<double, MT>(acc, tj, [&](int row, int col, int ti, int r) {
          const double2 v = X[(unsigned)(sc.pinv[row] * LB + col)];
          acc[ti].re[r] = v.x;
          acc[ti].im[r] = v.y;
        });
        prod(acc, ALds<double>{mat, S}, BPerm<BGlob<double>>{BGlob<double>{Rr, LB}, sc.piv}, tj);
        tiles_foreach<double, MT>(acc, tj, [&](int row, int col, int ti, int r) {
          X[(unsigned)(sc.pinv[row] * LB + col)] = make_double2(acc[ti].re[r], acc[ti].im[r]);
        });
      }
      // doubling update: output column tile tj reads column tiles tj (g a)
      // and MT + tj (g b) of X, written by other waves unless M/16 == NWAVE.
      // g is dead from here on: a, then b, is copied into the working matrix
      // (LDS, or the global workspace above 64) as the shared A operand of
      // the two products that use it, so a' and b' overwrite a and b in
      // place once the copy is done.
      __syncthreads();
      double na = 0.0, nb = 0.0;
#pragma unroll 1
      for (int half = 0; half < 2; ++half) {
        const double2* Aop = AB + half * M;
        if constexpr (M == 64) {
          // a plain copy: direct global-to-LDS loads, one 64-element row
          // (1 KB) per wave instruction
          for (int r = w; r < M; r += NWAVE)
            __builtin_amdgcn_global_load_lds((const void*)(Aop + r * LB + lane),
                                             (__attribute__((address_space(3))) void*)(mat + r * S), 16, 0, 0);
          __builtin_amdgcn_s_waitcnt(0);
        } else {
          for (int idx = t; idx < MM; idx += NT) {
            const int r = idx / M, c = idx - r * M;
            mat[r * S + c] = ldd(Aop + r * LB + c);
          }
        }
        __syncthreads();
        // one accumulator column live at a time: a g b, a g a | b g a, b g b;
        // the 2 MT (product, column tile) pairs are dealt over the waves
#pragma unroll 1
        for (int pj = w; pj < 2 * MT; pj += NWAVE) {
          const int qq = pj / MT, tj = pj - qq * MT;
          const int q = half == 0 ? 2 * qq : 1 + 2 * qq;
          ctile<double> acc[MT];
#pragma unroll
          for (int ti = 0; ti < MT; ++ti) tzero(acc[ti]);
          const double2* Bop = (q == 0 || q == 3) ? X + M : X;
          prod(acc, ALds<double>{mat, S}, BGlob<double>{Bop, LB}, tj);
          tiles_foreach<double, MT>(acc, tj, [&](int row, int col, int ti, int r) {
            const unsigned idx = row * M + col;
            const double re = acc[ti].re[r], im = acc[ti].im[r];
            if (q < 2) {
              double2 v = eps[idx];
              v.x -= re; v.y -= im; eps[idx] = v;
              if (q == 0) { v = esR[idx]; v.x -= re; v.y -= im; esR[idx] = v; }
            } else {
              AB[(unsigned)(row * LB + col) + (q == 3 ? M : 0)] = make_double2(-re, -im);
              if (q == 2) na = fmax(na, fabs(re) + fabs(im));
              else nb = fmax(nb, fabs(re) + fabs(im));
            }
          });
        }
        __syncthreads();
      }
      na = wave_maxd(na);
      nb = wave_maxd(nb);
      if (lane == 0) { red[0][w] = na; red[1][w] = nb; }
      __syncthreads();
      na = 0.0; nb = 0.0;
      for (int q = 0; q < NWAVE; ++q) { na = fmax(na, red[0][q]); nb = fmax(nb, red[1][q]); }
      __syncthreads();
      if (na + nb < tol * scl) { conv = true; break; }
    }
    if (!conv) it = -maxit;
    // Sigma_L = eR - e, Sigma_R = D0 - eR
    for (int idx = t; idx < MM; idx += NT) {
      const double2 vr = esR[idx];
      if (side != 1) {
        const double2 v = eps[idx];
        sig[(size_t)(2 * e) * MM + idx] = make_double2(vr.x - v.x, vr.y - v.y);
      }
      if (side != 0) {
        cpx<double> s = ldd(S00 + idx), h = ldd(H00 + idx);
        const double dr = zx.re * s.re - zx.im * s.im - h.re, di = zx.re * s.im + zx.im * s.re - h.im;
        sig[(size_t)(2 * e + 1) * MM + idx] = make_double2(dr - vr.x, di - vr.y);
      }
    }
    for (int s = 0; s < 2; ++s) {
      if ((side == 0 && s == 1) || (side == 1 && s == 0)) continue;
      if (t == 0) iters[2 * e + s] = it;
    }
    __syncthreads();
  }
  // the job counter of the k_sigma_finish launch that follows: the first
  // element of block 7 M^2 of workgroup 0's workspace (the residual, dead
  // once that workgroup's jobs are done; the Newton step uses blocks 0-6)
  if (blockIdx.x == 0 && t == 0) *reinterpret_cast<int*>(scratch + 7 * MM) = 0;
}

// Second stage of the self-energy jobs of a decimation launch (same jobs,
// same workspace): the Newton check and step on each self-energy (option
// newton_tol >= 0), then the LDL^H factor of its broadening.  A kernel of its
// own so that the doubling loop keeps its registers.  The few self-energies
// that take a Newton step cost tens of times a check, so the jobs are dealt
// from a counter (zeroed by k_decimate) rather than by a fixed stride: a
// workgroup that draws a correction takes fewer jobs, and the launch ends
// about one correction after the last check instead of after the sum of the
// corrections that one stride happens to collect.
template <int M>
__global__ __launch_bounds__(NT, M > 64 ? 1 : 2) void k_sigma_finish(Prob P0, BatchDesc b, const double* E, int nE,
                                                                     double eta, int sides, DecOpts o,
                                                                     double2* scratch, double2* sig, double2* wf,
                                                                     double* sgn, int* nheavy) {
  constexpr int MM = M * M, S = M + 1;
  constexpr bool BIG = M > 64;
  __shared__ cpx<double> mat_l[BIG ? 1 : M * S];
  __shared__ __align__(16) union {
    cpx<double> y[gj_scratch<M>()];
    LDLScratch<M> ldl;
  } u;
  __shared__ BGJ<double, M> sc;
  __shared__ double red[NWAVE];
  __shared__ int next_job;
  const int t = threadIdx.x;
  double2* ws = scratch + (size_t)blockIdx.x * dec_ws_elems(M);
  int* counter = reinterpret_cast<int*>(scratch + 7 * MM);
  cpx<double>* mat;
  if constexpr (BIG) mat = (cpx<double>*)(ws + 8 * MM);
  else mat = mat_l;
  const int njobs = b.probs ? b.njobs : nE * sides;
  for (;;) {
    if (t == 0) next_job = atomicAdd(counter, 1);
    __syncthreads();
    const int job = __builtin_amdgcn_readfirstlane(next_job);
    __syncthreads();
    if (job >= njobs) break;
    const DecJob J = dec_job(P0, b, E, eta, sides, job);
    for (int s = 0; s < 2; ++s) {
      if ((J.side == 0 && s == 1) || (J.side == 1 && s == 0)) continue;
      const size_t k = 2 * (size_t)J.e + s;
      if (o.newton_tol >= 0.0) sigma_newton<M>(sig + k * MM, J.lead, J.zx, s, o.newton_tol, ws, mat, u.y, sc, red);
      gamma_ldl<M>(sig + k * MM, wf + k * MM, sgn + k * M, o.heavy_tol, nheavy + k, u.ldl);
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------ refinement
// -B (FP64) into the M x (M + 1) buffer stg for one block B of row i of
// A(z): which = 0: U_i = A_{i,i+1}; 1: A_ii, with the contact self-energies
// subtracted on the end slabs; 2: L_i = A_{i,i-1}.  All threads; no barrier.
template <int M>
__device__ __forceinline__ void stage_neg_block(cpx<double>* stg, const Prob& P, cpx<double> z, int i, int which,
                                                const double2* sL, const double2* sR) {
  constexpr int MM = M * M, S = M + 1;
  const int t = threadIdx.x, N = P.N;
  if (which == 0) {
    const cpx<double> zu = mk<double>(z.re - P.vu(i), z.im);
    const double2 *Su = P.Su(i), *Hu = P.Hu(i);
    for (int idx = t; idx < MM; idx += NT) {
      const int r = idx / M, k = idx - r * M;
      const cpx<double> sv = ldd(Su + idx), hv = ldd(Hu + idx);
      stg[r * S + k] = mk<double>(hv.re - (zu.re * sv.re - zu.im * sv.im), hv.im - (zu.re * sv.im + zu.im * sv.re));
    }
  } else if (which == 1) {
    const cpx<double> zd = mk<double>(z.re - P.vd(i), z.im);
    const double2 *Sd = P.Sd(i), *Hd = P.Hd(i);
    for (int idx = t; idx < MM; idx += NT) {
      const int r = idx / M, k = idx - r * M;
      const cpx<double> sv = ldd(Sd + idx), hv = ldd(Hd + idx);
      double re = zd.re * sv.re - zd.im * sv.im - hv.re, im = zd.re * sv.im + zd.im * sv.re - hv.im;
      if (i == 0) {
        const cpx<double> g = ldd(sL + idx);
        re -= g.re;
        im -= g.im;
      }
      if (i == N - 1) {
        const cpx<double> g = ldd(sR + idx);
        re -= g.re;
        im -= g.im;
      }
      stg[r * S + k] = mk<double>(-re, -im);
    }
  } else {
    const cpx<double> zu = mk<double>(z.re - P.vu(i - 1), z.im);
    const double2 *Su = P.Su(i - 1), *Hu = P.Hu(i - 1);
    for (int idx = t; idx < MM; idx += NT) {
      const int k = idx / M, r = idx - k * M;       // read S[k][r] along r
      const cpx<double> sv = ldd(Su + idx), hv = ldd(Hu + idx);
      const double re = zu.re * sv.re + zu.im * sv.im - hv.re;
      const double im = zu.im * sv.re - zu.re * sv.im + hv.im;
      stg[r * S + k] = mk<double>(-re, -im);
    }
  }
}

// Mixed-precision refinement of the heavy injected columns of one energy
// (the single-precision sweep has left its factors X_i, Dt_i^-1 and its
// solution, widened to FP64, in P64).  One step:
//   forward:  r_i = b_i - (U_i psi_{i+1} + A_ii psi_i + L_i psi_{i-1})  (FP64)
//             c_i = Dt_i^-1 (r_i - L_i c_{i-1})                          (FP32)
//   backward: d_i = c_i - X_i d_{i+1},   psi_i += d_i
// repeated until ||r||_F <= rtol ||b||_F over the refined columns, with at
// most maxstep corrections.  It stops early when a correction fails to
// halve the residual, or when the contraction observed so far could not
// reach rtol in the corrections left: the FP64 fallback then takes over.
// The refined columns are the first hR column tiles of the right injection
// and the first hL of the left one (the broadening factor orders its
// columns by decreasing weight).
// Every residual product is a full column of tiles (M rows, 16 columns) of
// an M x M block times the solution, with the block staged once per slab
// in stg (FP64, LDS for M <= 64) and read by every wave.  A wave keeps the
// same column tiles through the whole chain (up to TPP at a time), so the
// correction's dependencies (c_{i-1} -> c_i, d_{i+1} -> d_i) stay within
// the wave: the forward pass takes barriers only around the stagings, the
// backward pass none.  Returns the last relative residual; *steps receives
// the corrections applied.
template <int M, int TPP>
__device__ __forceinline__ double refine(const Prob& P, const SweepArgs& a, const double2* sL, const double2* sR,
                                         const double2* WL, const double2* WR, cpx<double> z, int hR, int hL,
                                         const float2* XZ, const float2* DI, float2* ZC, float2* YB, double2* P64,
                                         cpx<double>* stg, double* red, int* steps) {
  constexpr int MT = M / 16, MM = M * M, LD = 2 * M, S = M + 1;
  const int N = P.N, w = threadIdx.x >> 6;
  const int nc = hR + hL;
  const int npass = (nc + NWAVE * TPP - 1) / (NWAVE * TPP);
  // column tile of the q-th refined tile (right injection first); the
  // wave's u-th tile of pass p is q = (p TPP + u) NWAVE + w
  auto colt = [&](int q) { return q < hR ? q : MT + q - hR; };
  double bb = 0.0;
  for (int q = w; q < nc; q += NWAVE) {
    const int tj = colt(q);
    ctile<double> acc[MT];
    tiles_foreach<double, MT>(acc, tj, [&](int row, int col, int, int) {
      const cpx<double> v = col < M ? ldd(WR + row * M + col) : ldd(WL + row * M + col - M);
      bb += v.re * v.re + v.im * v.im;
    });
  }
  bb = block_sum(bb, red);
  double rel = 0.0, prev = 0.0;
  int s = 0;
  for (;; ++s) {
    double rr = 0.0;
    for (int i = 0; i < N; ++i) {
      const double2* Pi = P64 + (size_t)i * M * LD;
      float2* Ci = ZC + (size_t)i * M * LD;
#pragma unroll 1
      for (int pass = 0; pass < npass; ++pass) {
        int tj[TPP];
        bool act[TPP];
        ctile<double> acc[TPP][MT];
#pragma unroll
        for (int u = 0; u < TPP; ++u) {
          const int q = (pass * TPP + u) * NWAVE + w;
          act[u] = q < nc;
          tj[u] = act[u] ? colt(q) : 0;
          // b_i: W_L on the first slab (left injection), W_R on the last
          const bool bL = act[u] && i == 0 && tj[u] >= MT, bR = act[u] && i == N - 1 && tj[u] < MT;
          tiles_foreach<double, MT>(acc[u], tj[u], [&](int row, int col, int ti, int r) {
            cpx<double> v = mk<double>(0.0, 0.0);
            if (bL) v = ldd(WL + row * M + col - M);
            if (bR) v = ldd(WR + row * M + col);
            acc[u][ti].re[r] = v.re;
            acc[u][ti].im[r] = v.im;
          });
        }
#pragma unroll 1
        for (int which = 0; which < 3; ++which) {
          if ((which == 0 && i == N - 1) || (which == 2 && i == 0)) continue;
          __syncthreads();                            // the previous block's readers are done
          stage_neg_block<M>(stg, P, z, i, which, sL, sR);
          __syncthreads();
          const double2* Pb = Pi + (which == 0 ? (ptrdiff_t)M * LD : which == 2 ? -(ptrdiff_t)M * LD : 0);
#pragma unroll
          for (int u = 0; u < TPP; ++u)
            if (act[u]) cgemm_col<double, MT, MT>(acc[u], ALds<double>{stg, S}, BGlob<double>{Pb, LD}, tj[u]);
        }
#pragma unroll
        for (int u = 0; u < TPP; ++u) {
          if (!act[u]) continue;
#pragma unroll
          for (int ti = 0; ti < MT; ++ti)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              rr += acc[u][ti].re[r] * acc[u][ti].re[r] + acc[u][ti].im[r] * acc[u][ti].im[r];
          tiles_foreach<double, MT>(acc[u], tj[u], [&](int row, int col, int ti, int r) {
            YB[row * LD + col] = make_float2((float)acc[u][ti].re[r], (float)acc[u][ti].im[r]);
          });
        }
        __threadfence_block();                        // YB tiles: written and read by this wave
        // right-hand side of the correction, y_i = r_i - L_i c_{i-1}, in
        // single precision (it only feeds the single-precision solve); -L_i
        // is still staged
        if (i > 0) {
#pragma unroll
          for (int u = 0; u < TPP; ++u) {
            if (!act[u]) continue;
            ctile<float> cf[MT];
            tiles_foreach<float, MT>(cf, tj[u], [&](int row, int col, int ti, int r) {
              const float2 v = YB[row * LD + col];
              cf[ti].re[r] = v.x;
              cf[ti].im[r] = v.y;
            });
            cgemm_col<float, MT, MT>(cf, ALdsF{stg, S}, BGlob<float>{Ci - (size_t)M * LD, LD}, tj[u]);
            tiles_foreach<float, MT>(cf, tj[u], [&](int row, int col, int ti, int r) {
              YB[row * LD + col] = make_float2(cf[ti].re[r], cf[ti].im[r]);
            });
          }
          __threadfence_block();
        }
#pragma unroll
        for (int u = 0; u < TPP; ++u) {
          if (!act[u]) continue;
          ctile<float> cf[MT];
#pragma unroll
          for (int ti = 0; ti < MT; ++ti) tzero(cf[ti]);
          cgemm_col<float, MT, MT>(cf, AGlob<float>{DI + (size_t)i * MM, M, 1.0f}, BGlob<float>{YB, LD}, tj[u]);
          tiles_foreach<float, MT>(cf, tj[u], [&](int row, int col, int ti, int r) {
            Ci[row * LD + col] = make_float2(cf[ti].re[r], cf[ti].im[r]);
          });
        }
        __threadfence_block();                        // c_i tiles: read by this wave at slab i + 1
      }
    }
    rr = block_sum(rr, red);
    prev = rel;
    rel = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    // uniform exits (NaN stops too): converged, out of steps, a step that
    // did not halve the residual, or a contraction too slow to reach rtol
    // in the steps left (the single-precision factors are too inaccurate
    // for this energy: the FP64 fallback takes over)
    if (!(rel > a.rtol) || s == a.maxstep || (s > 0 && !(rel < 0.5 * prev))) break;
    if (s > 0 && s + log(rel / a.rtol) / log(prev / rel) > a.maxstep + 0.5) break;
#pragma unroll 1
    for (int i = N - 1; i >= 0; --i) {
      float2* Ci = ZC + (size_t)i * M * LD;
      double2* Pi = P64 + (size_t)i * M * LD;
#pragma unroll 1
      for (int q = w; q < nc; q += NWAVE) {
        const int tj = colt(q);
        ctile<float> acc[MT];
        tiles_foreach<float, MT>(acc, tj, [&](int row, int col, int ti, int r) {
          const float2 v = Ci[row * LD + col];
          acc[ti].re[r] = v.x;
          acc[ti].im[r] = v.y;
        });
        if (i < N - 1)
          cgemm_col<float, MT, MT>(acc, AGlob<float>{XZ + (size_t)i * M * LD, LD, -1.0f},
                                   BGlob<float>{Ci + (size_t)M * LD, LD}, tj);
        // d_i replaces c_i (read again by this wave only, at slab i - 1)
        tiles_foreach<float, MT>(acc, tj, [&](int row, int col, int ti, int r) {
          const unsigned idx = row * LD + col;
          Ci[idx] = make_float2(acc[ti].re[r], acc[ti].im[r]);
          double2 v = Pi[idx];
          v.x += (double)acc[ti].re[r];
          v.y += (double)acc[ti].im[r];
          Pi[idx] = v;
        });
      }
      __threadfence_block();
    }
  }
  *steps = s;
  return rel;
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
//
// MIX (R = float): the sweep also keeps Dt_i^-1 (in natural row/column
// order) and writes the heavy column tiles of psi, plus the whole left
// injection on the last slab, to the FP64 solution buffer; the densities of
// the light columns are reduced here, those of the heavy columns and T after
// the refinement.
//
// With a.elist (FP64 sweep only) the launch re-solves the listed energies,
// keeping the refinement diagnostics in info and marking the fallback.
//
// Two workgroups per CU at every block size.  Above 64 this caps the
// registers at 256 per lane, and the FP64 sweep spills about 70 bytes per
// lane at M = 128 (outside its MFMA loops).  A second wave per SIMD issues MFMAs while the first
// waits on its operands in L2, which more than pays for the spill.
template <typename R, int M, bool MIX, bool DM, int PW = gj_pw<M>(), int TPP = (M <= 64 ? 2 : 1)>
__global__ __launch_bounds__(NT, 2) void k_sweep(Prob P0, SweepArgs a, BatchDesc b) {
  static_assert(!DM || (!MIX && sizeof(R) == 8), "density-matrix blocks come from the FP64 sweep");
  typedef typename vec2t<R>::type V2;
  constexpr int MT = M / 16, MM = M * M, S = M + 1, LD = 2 * M;
  // M > 64: the working matrix and the staged coupling block live at the
  // end of the workgroup's global workspace (they do not fit in LDS)
  constexpr bool BIG = M > 64;
  // the working matrix; during the mixed refinement (M <= 64) the FP64
  // block staged for the residual products
  constexpr int STG = (MIX && !BIG) ? M * S : 1;
  // 16-byte alignment stated: a union of cpx arrays is only 8-byte aligned
  // by type, and without it the complex loads and stores split into pairs
  // of 8-byte LDS accesses
  __shared__ __align__(16) union {
    cpx<R> m[BIG ? 1 : M * S];
    cpx<double> stg[STG];
  } lu;
  cpx<R>* const mat_l = lu.m;
  // the elimination's scratch; above 64 (FP64) also the staged slices of
  // the A operand of the sweep's three products (-L_i, the inverse, -X_i)
  constexpr bool STAGE = BIG && !MIX && !DM;
  // FP64 at M = 64: X_i reaches the working matrix for the back
  // substitution by direct global-to-LDS loads (one 64-element row, 1 KB,
  // per wave instruction), without passing through registers; it lands
  // un-negated, so the product runs on -(initial value) and the result is
  // negated back (exact: the rounding of every step is symmetric in sign)
  constexpr bool XDMA = !BIG && !MIX && M == 64 && sizeof(cpx<R>) == 16;
  constexpr int YS = gj_scratch<M, PW>() > (STAGE ? M * kStageStride : 0) ? gj_scratch<M, PW>() : M * kStageStride;
  __shared__ __align__(16) cpx<R> Ysc[YS];
  __shared__ BGJ<R, M> sc;
  __shared__ double tred[NWAVE];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  char* wsb = a.ws + (size_t)blockIdx.x * a.ws_bytes;
  const SweepLayout L0 = sweep_layout(0, M, MIX, DM, a.ws_bytes);
  cpx<R>* mat;
  cpx<R>* Lst;                                  // -L_i, staged once per slab
  if constexpr (BIG) {
    mat = (cpx<R>*)(wsb + L0.mat);
    Lst = (cpx<R>*)(wsb + L0.lst);
  } else {
    mat = mat_l;
    Lst = mat_l;
  }
  V2* XZ = (V2*)(wsb + L0.xz);
  double* prt = a.part + (size_t)blockIdx.x * NWAVE * 2 * a.nmax * (MIX ? 2 : 1);
  double* prt2 = prt + (size_t)NWAVE * 2 * a.nmax;
  // values loaded from memory are made wave-uniform explicitly, so that
  // everything addressed through them stays in scalar registers
  const int ne = a.elist ? __builtin_amdgcn_readfirstlane(*a.ecount) : a.nE;
  for (int q = blockIdx.x; q < ne; q += gridDim.x) {
    const int e = a.elist ? __builtin_amdgcn_readfirstlane(a.elist[q]) : q;
    const Prob P = b.probs ? load_prob(b.probs + __builtin_amdgcn_readfirstlane(b.item_prob[e])) : P0;
    const int N = P.N;
    // workspace layout for this item's slab count (at most a.nmax)
    const SweepLayout Lw = sweep_layout(N, M, MIX, DM, a.ws_bytes);
    V2* PSI = (V2*)(wsb + Lw.psi);
    float2* DI = nullptr;
    float2* ZC = nullptr;
    float2* YB = nullptr;
    double2* P64 = nullptr;
    if constexpr (MIX) {
      DI = (float2*)(wsb + Lw.di);
      ZC = (float2*)(wsb + Lw.zc);
      YB = (float2*)(wsb + Lw.yb);
      P64 = (double2*)(wsb + Lw.p64);
    }
    double* ldos_e = nullptr;
    if (a.ldos) ldos_e = a.ldos + (b.probs ? b.item_ldos[e] : (size_t)e * 2 * N);
    const cpx<double> z = mk<double>(a.E[e], a.eta);
    // contact data: the left surface of slot sl and the right surface of
    // slot sr (both e, unless a self-energy cache supplies the slots)
    const int sl = a.sig_slot ? __builtin_amdgcn_readfirstlane(a.sig_slot[2 * e]) : e;
    const int sr = a.sig_slot ? __builtin_amdgcn_readfirstlane(a.sig_slot[2 * e + 1]) : e;
    const double2* sL = a.sig + (size_t)(2 * sl) * MM;
    const double2* sR = a.sig + (size_t)(2 * sr + 1) * MM;
    const double2* WL = a.wf + (size_t)(2 * sl) * MM;
    const double2* WR = a.wf + (size_t)(2 * sr + 1) * MM;
    const double* sgL = a.sgn + (size_t)(2 * sl) * M;
    const double* sgR = a.sgn + (size_t)(2 * sr + 1) * M;
    int hL = MT, hR = MT;                      // heavy column tiles (MIX)
    if constexpr (MIX) {
      hL = __builtin_amdgcn_readfirstlane(min(max((a.nheavy[2 * sl] + 15) / 16, 1), MT));
      hR = __builtin_amdgcn_readfirstlane(min(max((a.nheavy[2 * sr + 1] + 15) / 16, 1), MT));
    }
    for (int i = 0; i < N; ++i) {
      __syncthreads();
      V2* Xi = XZ + (size_t)i * M * LD;
      const double vd = P.vd(i);
      const double2* Sd = P.Sd(i);
      const double2* Hd = P.Hd(i);
      const cpx<double> zd = mk<double>(z.re - vd, z.im);
      // Stage A = -L_i = -(A_{i,i-1}) once per slab in the LDS buffer (free
      // until the new Schur complement is written): every wave reads the
      // whole of it, which from L1/L2 would exceed the cache bandwidth.
      // (M > 64 FP64: generated straight into the product's staged slices;
      // the mixed sweep above 64 stages it in a global buffer.)
      if (i > 0 && !STAGE) {
        const double vu = P.vu(i - 1);
        const cpx<double> zu = mk<double>(z.re - vu, z.im);
        const double2* Su = P.Su(i - 1);
        const double2* Hu = P.Hu(i - 1);
        for (int idx = t; idx < MM; idx += NT) {
          const int k = idx / M, r = idx - k * M;     // read S[k][r] along r
          const cpx<double> sv = ldd(Su + idx), hv = ldd(Hu + idx);
          const double re = zu.re * sv.re + zu.im * sv.im - hv.re;
          const double im = zu.im * sv.re - zu.re * sv.im + hv.im;
          Lst[r * S + k] = mk<R>((R)-re, (R)-im);
        }
        __syncthreads();
      }
      // Column tiles of [Dt | y]: the y tiles go straight to the workspace,
      // the (at most DT) Dt tile columns of this wave stay in registers until
      // every wave has finished reading L_i from the LDS buffer.  (M > 64:
      // both go straight to their buffers, in one pass, so that every wave
      // takes the same number of tiles through the staged product.)
      constexpr int DT = BIG ? 1 : (MT + NWAVE - 1) / NWAVE;
      ctile<R> dacc[DT][MT];
#pragma unroll 1
      for (int pass = 0; pass < (BIG ? 1 : 2); ++pass) {
        int nd = 0;
#pragma unroll 1
        for (int tj = w; tj < 2 * MT; tj += NWAVE) {
          const bool is_d = tj < MT;
          if (!BIG && is_d != (pass == 1)) continue;
          ctile<R> acc[MT];
          if (is_d) {
            tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
              const unsigned idx = row * M + col;
              cpx<double> sv = ldd(Sd + idx), hv = ldd(Hd + idx);
              acc[ti].re[r] = (R)(zd.re * sv.re - zd.im * sv.im - hv.re);
              acc[ti].im[r] = (R)(zd.re * sv.im + zd.im * sv.re - hv.im);
            });
            if (i == 0)
              tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
                cpx<double> v = ldd(sL + (unsigned)(row * M + col));
                acc[ti].re[r] -= (R)v.re;
                acc[ti].im[r] -= (R)v.im;
              });
            if (i == N - 1)
              tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
                cpx<double> v = ldd(sR + (unsigned)(row * M + col));
                acc[ti].re[r] -= (R)v.re;
                acc[ti].im[r] -= (R)v.im;
              });
          } else if (i == 0) {
            tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
              cpx<double> v = ldd(WL + (unsigned)(row * M + col - M));
              acc[ti].re[r] = (R)v.re;
              acc[ti].im[r] = (R)v.im;
            });
          } else {
#pragma unroll
            for (int ti = 0; ti < MT; ++ti) tzero(acc[ti]);
          }
          if (i > 0) {
            if constexpr (STAGE) {
              const cpx<double> zu = mk<double>(z.re - P.vu(i - 1), z.im);
              cgemm_col_staged<R, MT, true>(acc, AGenL<R>{P.Su(i - 1), P.Hu(i - 1), zu, M},
                                            BGlob<R>{Xi - (size_t)M * LD, LD}, tj, Ysc);
            } else {
              cgemm_col<R, MT, MT>(acc, ALds<R>{Lst, S}, BGlob<R>{Xi - (size_t)M * LD, LD}, tj);
            }
          }
          if (is_d && BIG) {
            // the Schur complement goes straight to its own buffer
            tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
              mat[row * S + col] = mk<R>(acc[ti].re[r], acc[ti].im[r]);
            });
          } else if (is_d) {
#pragma unroll
            for (int q2 = 0; q2 < DT; ++q2)
              if (q2 == nd)
#pragma unroll
                for (int ti = 0; ti < MT; ++ti) dacc[q2][ti] = acc[ti];
            ++nd;
          } else {
            tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
              st2<R>(Xi + (unsigned)(row * LD + col), mk<R>(acc[ti].re[r], acc[ti].im[r]));
            });
          }
        }
      }
      __syncthreads();
      if constexpr (!BIG) {
        int nd = 0;
#pragma unroll 1
        for (int tj = w; tj < MT; tj += NWAVE) {
#pragma unroll
          for (int q2 = 0; q2 < DT; ++q2)
            if (q2 == nd)
              tiles_foreach<R, MT>(dacc[q2], tj, [&](int row, int col, int ti, int r) {
                mat[row * S + col] = mk<R>(dacc[q2][ti].re[r], dacc[q2][ti].im[r]);
              });
          ++nd;
        }
      }
      __syncthreads();
      gj_inverse<R, M, PW>(mat, S, Ysc, sc);
      if constexpr (MIX) {
        // Dt_i^-1[j][c] = mat[piv[j]][pinv[c]]
        float2* Di = DI + (size_t)i * MM;
        for (int idx = t; idx < MM; idx += NT) {
          const int j = idx / M, c = idx - j * M;
          const cpx<R> v = mat[sc.piv[j] * S + sc.pinv[c]];
          Di[idx] = make_float2(v.re, v.im);
        }
      }
#pragma unroll 1
      for (int tj = w; tj < 2 * MT; tj += NWAVE) {
        ctile<R> acc[MT];
#pragma unroll
        for (int ti = 0; ti < MT; ++ti) tzero(acc[ti]);
        ALds<R> A{mat, S};
        // every wave takes 2 MT / NWAVE column tiles (whole: MT is 6 or 8
        // above 64), so the staged product's barriers line up
        auto prod = [&](const auto& B) {
          if constexpr (STAGE) cgemm_col_staged<R, MT>(acc, A, B, tj, Ysc);
          else cgemm_col<R, MT, MT>(acc, A, B, tj);
        };
        if (tj < MT) {
          if (i < N - 1) {
            const double vu = P.vu(i);
            prod(BPerm<BGen<R>>{BGen<R>{P.Su(i), P.Hu(i), mk<double>(z.re - vu, z.im), M}, sc.piv});
          } else {
            prod(BPerm<BGlobD<R>>{BGlobD<R>{WR, M}, sc.piv});
          }
        } else {
          prod(BPerm<BGlob<R>>{BGlob<R>{Xi, LD}, sc.piv});
        }
        // rows land through the inverse pivot order; a column tile is read
        // and written by one wave only, so the scatter needs no barrier
        tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
          st2<R>(Xi + (unsigned)(sc.pinv[row] * LD + col), mk<R>(acc[ti].re[r], acc[ti].im[r]));
        });
      }
    }
    __syncthreads();
    // transmission from the left-injected solution on the last slab
    if constexpr (!MIX) {
      const V2* XN = XZ + (size_t)(N - 1) * M * LD;
      double tp = 0.0;
#pragma unroll 1
      for (int tj = w; tj < 2 * MT; tj += NWAVE) {
        if (tj < MT) continue;
        ctile<R> acc[MT];
#pragma unroll
        for (int ti = 0; ti < MT; ++ti) tzero(acc[ti]);
        cgemm_col<R, MT, MT>(acc, AGlobCT<R>{WR, M}, BGlob<R>{XN, LD}, tj);
        const double sl = sgL[16 * tj + (lane & 15) - M];
        tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
          const double re = acc[ti].re[r], im = acc[ti].im[r];
          tp += sgR[row] * sl * (re * re + im * im);
        });
      }
      tp = wave_sum(tp);
      if (lane == 0) tred[w] = tp;
    }
    // back substitution with fused slab densities
    for (int i = N - 1; i >= 0; --i) {
      const V2* Xi = XZ + (size_t)i * M * LD;
      // psi_i overwrites psi_{i+1} column tile by column tile (one wave owns
      // a column tile); DM keeps both, in alternating buffers
      V2* PSc = PSI;
      const V2* PSn = PSI;
      if constexpr (DM) {
        PSc = PSI + (size_t)(i & 1) * M * LD;
        PSn = PSI + (size_t)((i + 1) & 1) * M * LD;
      }
      if (i < N - 1) {
        // stage -X_i in LDS once per slab (every wave reads all of it);
        // M > 64 reads X_i where it is
        if constexpr (XDMA) {
          __syncthreads();
          for (int r = w; r < M; r += NWAVE)
            __builtin_amdgcn_global_load_lds((const void*)(Xi + (unsigned)(r * LD) + lane),
                                             (__attribute__((address_space(3))) void*)(mat + r * S), 16, 0, 0);
          __builtin_amdgcn_s_waitcnt(0);
          __syncthreads();
        } else if constexpr (!BIG) {
          __syncthreads();
          for (int idx = t; idx < MM; idx += NT) {
            const int r = idx / M, c = idx - r * M;
            const cpx<R> v = ld2<R>(Xi + (unsigned)(r * LD + c));
            mat[r * S + c] = mk<R>(-v.re, -v.im);
          }
          __syncthreads();
        }
      }
      double pL = 0.0, pR = 0.0;
      // XDMA: the product accumulates -psi_i from -[0 | z_i] and +X_i
      const R sgn = (XDMA && i < N - 1) ? (R)-1 : (R)1;
#pragma unroll 1
      for (int tj = w; tj < 2 * MT; tj += NWAVE) {
        ctile<R> acc[MT];
        if (i == N - 1 || tj >= MT) {
          tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
            cpx<R> v = ld2<R>(Xi + (unsigned)(row * LD + col));
            acc[ti].re[r] = sgn * v.re;
            acc[ti].im[r] = sgn * v.im;
          });
        } else {
#pragma unroll
          for (int ti = 0; ti < MT; ++ti) tzero(acc[ti]);
        }
        if (i < N - 1) {
          if constexpr (STAGE) cgemm_col_staged<R, MT>(acc, AGlob<R>{Xi, LD, (R)-1}, BGlob<R>{PSn, LD}, tj, Ysc);
          else if constexpr (BIG) cgemm_col<R, MT, MT>(acc, AGlob<R>{Xi, LD, (R)-1}, BGlob<R>{PSn, LD}, tj);
          else cgemm_col<R, MT, MT>(acc, ALds<R>{mat, S}, BGlob<R>{PSn, LD}, tj);
        }
        const int cl = 16 * tj + (lane & 15);
        const double sg = cl < M ? sgR[cl] : sgL[cl - M];
        bool heavy = false, keep = false;
        if constexpr (MIX) {
          heavy = tj < MT ? tj < hR : tj - MT < hL;
          keep = heavy || (i == N - 1 && tj >= MT);
        }
        double pp = 0.0;
        tiles_foreach<R, MT>(acc, tj, [&](int row, int col, int ti, int r) {
          const double re = sgn * acc[ti].re[r], im = sgn * acc[ti].im[r];
          st2<R>(PSc + (unsigned)(row * LD + col), mk<R>(sgn * acc[ti].re[r], sgn * acc[ti].im[r]));
          if constexpr (MIX)
            if (keep) P64[(size_t)i * M * LD + (unsigned)(row * LD + col)] = make_double2(re, im);
          pp += re * re + im * im;
        });
        if (!heavy) {
          if (tj < MT) pR += sg * pp;
          else pL += sg * pp;
        }
      }
      __threadfence_block();
      pL = wave_sum(pL);
      pR = wave_sum(pR);
      if (lane == 0) {
        prt[(w * 2 + 0) * N + i] = pL;
        prt[(w * 2 + 1) * N + i] = pR;
      }
      if constexpr (DM) {
        // rho_ii += psi_i W psi_i^H and rho_{i,i+1} += psi_i W psi_{i+1}^H
        // into this workgroup's accumulators; W weights each injected
        // column by its sign in Gamma = V diag(s) V^H, the energy's weight
        // for its contact, and 1/pi.  A task is one column tile of one of
        // the two blocks; the products read psi where it is (L1/L2).
        __syncthreads();                        // psi_i complete
        const double ipi = 0.31830988618379067154;
        const double wl = a.dmwL[e] * ipi, wr = a.dmwR[e] * ipi;
        double2* Rb = a.rho + (size_t)blockIdx.x * a.rho_stride + (size_t)(2 * i) * MM;
        const bool fresh = a.rho_first && q == (int)blockIdx.x;
        const int ntask = (i < N - 1 ? 2 : 1) * MT;
#pragma unroll 1
        for (int task = w; task < ntask; task += NWAVE) {
          const bool off = task >= MT;
          const int tj = off ? task - MT : task;
          double2* Rt = Rb + (off ? MM : 0);
          ctile<double> acc[MT];
          if (fresh) {
#pragma unroll
            for (int ti = 0; ti < MT; ++ti) tzero(acc[ti]);
          } else {
            tiles_foreach<double, MT>(acc, tj, [&](int row, int col, int ti, int r) {
              const double2 v = Rt[(unsigned)(row * M + col)];
              acc[ti].re[r] = v.x;
              acc[ti].im[r] = v.y;
            });
          }
          cgemm_col<double, MT, 2 * MT>(acc, APsiW{PSc, LD, sgR, sgL, wr, wl, M},
                                        BPsiH{off ? PSn : PSc, LD}, tj);
          tiles_foreach<double, MT>(acc, tj, [&](int row, int col, int ti, int r) {
            Rt[(unsigned)(row * M + col)] = make_double2(acc[ti].re[r], acc[ti].im[r]);
          });
        }
        __syncthreads();                        // the next slab overwrites psi_{i+1}
      }
    }
    __syncthreads();
    int steps = 0;
    double rel = 0.0;
    if constexpr (MIX) {
      // M > 64: the staged FP64 block sits below the working matrix and
      // the coupling block at the end of the workspace
      cpx<double>* stg = lu.stg;
      if constexpr (BIG) stg = (cpx<double>*)(wsb + L0.stg);
      rel = refine<M, TPP>(P, a, sL, sR, WL, WR, z, hR, hL, (const float2*)XZ, DI, ZC, YB, P64, stg, tred, &steps);
      // transmission and the heavy columns' densities from the refined solution
      {
        const double2* PN = P64 + (size_t)(N - 1) * M * LD;
        double tp = 0.0;
#pragma unroll 1
        for (int tj = MT + w; tj < 2 * MT; tj += NWAVE) {
          ctile<double> acc[MT];
#pragma unroll
          for (int ti = 0; ti < MT; ++ti) tzero(acc[ti]);
          cgemm_col<double, MT, MT>(acc, AGlobCT<double>{WR, M}, BGlob<double>{PN, LD}, tj);
          const double sl = sgL[16 * tj + (lane & 15) - M];
          tiles_foreach<double, MT>(acc, tj, [&](int row, int col, int ti, int r) {
            const double re = acc[ti].re[r], im = acc[ti].im[r];
            tp += sgR[row] * sl * (re * re + im * im);
          });
        }
        tp = wave_sum(tp);
        if (lane == 0) tred[w] = tp;
      }
      const int npair = MT * (hR + hL);
      for (int i = 0; i < N; ++i) {
        const double2* Pi = P64 + (size_t)i * M * LD;
        double pL = 0.0, pR = 0.0;
        for (int p = w; p < npair; p += NWAVE) {
          const int ti = p % MT, qq = p / MT, tj = qq < hR ? qq : MT + qq - hR;
          const int cl = 16 * tj + (lane & 15);
          const double sg = cl < M ? sgR[cl] : sgL[cl - M];
          double pp = 0.0;
          ctile<double> acc[1];
          tiles_foreach<double, 1>(acc, tj, [&](int row, int col, int, int) {
            const double2 v = Pi[(16 * ti + row) * LD + col];
            pp += v.x * v.x + v.y * v.y;
          });
          if (tj < MT) pR += sg * pp;
          else pL += sg * pp;
        }
        pL = wave_sum(pL);
        pR = wave_sum(pR);
        if (lane == 0) {
          prt2[(w * 2 + 0) * N + i] = pL;
          prt2[(w * 2 + 1) * N + i] = pR;
        }
      }
      __threadfence_block();
      __syncthreads();
    }
    const double ipi = 0.31830988618379067154;
    double Te = 0.0;
    for (int q2 = 0; q2 < NWAVE; ++q2) Te += tred[q2];
    bool bad = !isfinite(Te);
    for (int idx = t; idx < 2 * N; idx += NT) {
      const int s = idx / N, i = idx - s * N;
      double v = 0.0;
      for (int q2 = 0; q2 < NWAVE; ++q2) v += prt[(q2 * 2 + s) * N + i];
      if constexpr (MIX)
        for (int q2 = 0; q2 < NWAVE; ++q2) v += prt2[(q2 * 2 + s) * N + i];
      if (ldos_e) ldos_e[(size_t)s * N + i] = v * ipi;
    }
    if (t == 0) {
      a.T[e] = Te;
      const int i0 = a.iters[2 * sl], i1 = a.iters[2 * sr + 1];
      const bool rbad = MIX && !(rel <= a.rtol);
      if constexpr (MIX) a.redo[e] = (rbad || bad) ? 1 : 0;
      if (a.info) {
        qtx_info inf;
        if (a.elist) {
          inf = a.info[e];             // keep the refinement record, mark the fallback
          inf.fell_back_fp64 = 1;
        } else {
          inf.refine_steps = steps;
          inf.resid = rel;
          inf.fell_back_fp64 = 0;
        }
        inf.dec_iters = (i0 < 0 || i1 < 0) ? -1 : (i0 > i1 ? i0 : i1);
        inf.flags = ((i0 < 0 || i1 < 0) ? QTX_FLAG_DEC_NOTCONV : 0) | (bad ? QTX_FLAG_NONFINITE : 0) |
                    (rbad ? QTX_FLAG_REFINE_NOTCONV : 0);
        a.info[e] = inf;
      }
    }
  }
}

// Sum of the workgroups' density-matrix accumulators, in workgroup order
// (the result does not depend on scheduling), cut from the padded M x M
// blocks to the physical m x m ones.  One thread per output element.
__global__ __launch_bounds__(NT) void k_dm_reduce(const double2* rho, int nwg, size_t stride, int N, int M, int m,
                                                  double2* out_d, double2* out_o) {
  const size_t mm = (size_t)m * m, total = (2 * (size_t)N - 1) * mm;
  for (size_t idx = (size_t)blockIdx.x * NT + threadIdx.x; idx < total; idx += (size_t)gridDim.x * NT) {
    const size_t blk = idx / mm, rem = idx - blk * mm;
    const int r = (int)(rem / m), c = (int)(rem - (size_t)r * m);
    const double2* src = rho + blk * M * M + (size_t)r * M + c;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < nwg; ++b) {
      const double2 v = src[(size_t)b * stride];
      re += v.x;
      im += v.y;
    }
    double2* dst = (blk & 1) ? out_o + (blk >> 1) * mm + rem : out_d + (blk >> 1) * mm + rem;
    *dst = make_double2(re, im);
  }
}

// Energies whose refinement failed, compacted into a list (one wave).
__global__ __launch_bounds__(64) void k_compact(const int* redo, int nE, int* elist, int* ecount) {
  const int lane = threadIdx.x;
  int base = 0;
  for (int e0 = 0; e0 < nE; e0 += 64) {
    const int e = e0 + lane;
    const bool f = e < nE && redo[e] != 0;
    const unsigned long long m = __ballot(f);
    const int pre = __popcll(m & ((1ull << lane) - 1ull));
    if (f) elist[base + pre] = e;
    base += __popcll(m);
  }
  if (lane == 0) *ecount = base;
}

// ----------------------------------------------------------- band structure
// Bands of a lead at Bloch phase k: H(k) c = E S(k) c with
// H(k) = H00 + e^{ik} H01 + e^{-ik} H01^H and S(k) likewise (Bloch's
// theorem on the slab equations; the band-structure reconstruction of the
// results section).  One workgroup per k point, on the physical m x m block:
//   1. A = H(k), B = S(k), each symmetrised (X + X^H) / 2;
//   2. B = L L^H (right-looking Cholesky, two barriers per column);
//   3. C = L^-1 A L^-H: A <- L^-1 A, A <- A^H, A <- L^-1 A (every thread
//      substitutes its own column, no barrier inside), then symmetrised;
//   4. Householder reduction of C to Hermitian tridiagonal form: step j
//      maps column j below the diagonal onto -phase |x| e_1 with
//      H = I - tau v v^H and updates the trailing block by the rank-2 form
//      C <- C - v w^H - w v^H, p = tau C v, w = p - (tau/2)(v^H p) v;
//   5. eigenvalue n by bisection on the Sturm count of the real symmetric
//      tridiagonal (d, |e|), which has the same spectrum; thread n.
// Output E[k][n] = E_n(k) + V, ascending.  Matrices in LDS for M <= 64,
// otherwise in the workgroup's slice of the global workspace.
template <int M>
__global__ __launch_bounds__(NT, 1) void k_bands(const double2* lead, int m, double V, const double* kpts, int nk,
                                               double2* work, double* E) {
  constexpr int S = M + 1;
  constexpr bool BIG = M > 64;
  __shared__ cpx<double> lds[BIG ? 1 : 2 * M * S];
  __shared__ cpx<double> vv[M], pw[M];
  __shared__ double dd[M], ee[M], red[NWAVE];
  __shared__ double scal[4];
  const int t = threadIdx.x;
  cpx<double>* A;
  if constexpr (BIG) A = (cpx<double>*)(work + (size_t)blockIdx.x * 2 * M * S);
  else A = lds;
  cpx<double>* B = A + M * S;
  const int MM = M * M;
  const double2 *H00 = lead, *H01 = lead + MM, *S00 = lead + 2 * MM, *S01 = lead + 3 * MM;
  for (int q = blockIdx.x; q < nk; q += gridDim.x) {
    const double kq = kpts[q];
    const cpx<double> ph = mk<double>(cos(kq), sin(kq));
    __syncthreads();
    // 1. Bloch matrices
    for (int idx = t; idx < m * m; idx += NT) {
      const int r = idx / m, c = idx - r * m;
      auto bloch = [&](const double2* X0, const double2* X1, int a, int b) {
        // X0[a][b] + e^{ik} X1[a][b] + e^{-ik} conj(X1[b][a])
        const cpx<double> x0 = ldd(X0 + a * M + b), x1 = ldd(X1 + a * M + b), x2 = ldd(X1 + b * M + a);
        return mk<double>(x0.re + ph.re * x1.re - ph.im * x1.im + ph.re * x2.re - ph.im * x2.im,
                          x0.im + ph.re * x1.im + ph.im * x1.re - ph.re * x2.im - ph.im * x2.re);
      };
      const cpx<double> h1 = bloch(H00, H01, r, c), h2 = bloch(H00, H01, c, r);
      const cpx<double> s1 = bloch(S00, S01, r, c), s2 = bloch(S00, S01, c, r);
      A[r * S + c] = mk<double>(0.5 * (h1.re + h2.re), 0.5 * (h1.im - h2.im));
      B[r * S + c] = mk<double>(0.5 * (s1.re + s2.re), 0.5 * (s1.im - s2.im));
    }
    __syncthreads();
    // 2. Cholesky of B (lower triangle)
    for (int j = 0; j < m; ++j) {
      const double dj = sqrt(B[j * S + j].re);
      for (int i = j + 1 + t; i < m; i += NT) {
        const cpx<double> v = B[i * S + j];
        B[i * S + j] = mk<double>(v.re / dj, v.im / dj);
      }
      __syncthreads();
      if (t == 0) B[j * S + j] = mk<double>(dj, 0.0);
      const int n = m - j - 1;
      for (int idx = t; idx < n * n; idx += NT) {
        const int i = j + 1 + idx / n, l = j + 1 + idx % n;
        if (l > i) continue;
        const cpx<double> a = B[i * S + j], b = B[l * S + j];
        cpx<double> x = B[i * S + l];
        x.re -= a.re * b.re + a.im * b.im;
        x.im -= a.im * b.re - a.re * b.im;
        B[i * S + l] = x;
      }
      __syncthreads();
    }
    // 3. C = L^-1 A L^-H
    for (int pass = 0; pass < 2; ++pass) {
      for (int c = t; c < m; c += NT) {
        for (int i = 0; i < m; ++i) {
          cpx<double> y = A[i * S + c];
          for (int k2 = 0; k2 < i; ++k2) y = cfms(y, B[i * S + k2], A[k2 * S + c]);
          const double li = B[i * S + i].re;
          A[i * S + c] = mk<double>(y.re / li, y.im / li);
        }
      }
      __syncthreads();
      // A <- (A + A^H) / 2 after the second pass, A <- A^H after the first
      for (int idx = t; idx < m * m; idx += NT) {
        const int r = idx / m, c = idx - r * m;
        if (c < r) continue;
        const cpx<double> x = A[r * S + c], y = A[c * S + r];
        if (pass == 0) {
          A[r * S + c] = cconj(y);
          A[c * S + r] = cconj(x);
        } else {
          const cpx<double> u = mk<double>(0.5 * (x.re + y.re), 0.5 * (x.im - y.im));
          A[r * S + c] = u;
          A[c * S + r] = cconj(u);
        }
      }
      __syncthreads();
    }
    // 4. Householder tridiagonalisation
    for (int j = 0; j + 2 < m; ++j) {
      const int n = m - j - 1, o = j + 1;            // trailing block rows / columns o..m-1
      double ss = 0.0;
      for (int r = t; r < n; r += NT) {
        const cpx<double> x = A[(o + r) * S + j];
        ss += x.re * x.re + x.im * x.im;
      }
      ss = block_sum(ss, red);
      const double alpha = sqrt(ss);
      const cpx<double> x0 = A[o * S + j];
      const double ax0 = sqrt(x0.re * x0.re + x0.im * x0.im);
      if (t == 0) {
        dd[j] = A[j * S + j].re;
        ee[j] = alpha;
      }
      if (alpha == 0.0) continue;                    // uniform: column already reduced
      const cpx<double> th = ax0 > 0.0 ? mk<double>(x0.re / ax0, x0.im / ax0) : mk<double>(1.0, 0.0);
      const double tau = 1.0 / (alpha * (alpha + ax0));
      for (int r = t; r < n; r += NT) {
        cpx<double> x = A[(o + r) * S + j];
        if (r == 0) x = mk<double>(x.re + th.re * alpha, x.im + th.im * alpha);
        vv[r] = x;
      }
      __syncthreads();
      // p = tau C v (rows of the trailing block), then v^H p
      double kre = 0.0, kim = 0.0;
      for (int r = t; r < n; r += NT) {
        cpx<double> acc = mk<double>(0.0, 0.0);
        for (int c = 0; c < n; ++c) {
          const cpx<double> a = A[(o + r) * S + o + c], v = vv[c];
          acc.re += a.re * v.re - a.im * v.im;
          acc.im += a.re * v.im + a.im * v.re;
        }
        acc = mk<double>(tau * acc.re, tau * acc.im);
        pw[r] = acc;
        const cpx<double> v = vv[r];
        kre += v.re * acc.re + v.im * acc.im;        // conj(v) p
        kim += v.re * acc.im - v.im * acc.re;
      }
      kre = block_sum(kre, red);
      kim = block_sum(kim, red);
      const double hre = 0.5 * tau * kre, him = 0.5 * tau * kim;
      for (int r = t; r < n; r += NT) {
        const cpx<double> v = vv[r], p = pw[r];
        pw[r] = mk<double>(p.re - (hre * v.re - him * v.im), p.im - (hre * v.im + him * v.re));
      }
      __syncthreads();
      for (int idx = t; idx < n * n; idx += NT) {
        const int r = idx / n, c = idx - r * n;
        const cpx<double> vr = vv[r], vc = vv[c], wr = pw[r], wc = pw[c];
        cpx<double> x = A[(o + r) * S + o + c];
        x.re -= vr.re * wc.re + vr.im * wc.im + wr.re * vc.re + wr.im * vc.im;
        x.im -= vr.im * wc.re - vr.re * wc.im + wr.im * vc.re - wr.re * vc.im;
        A[(o + r) * S + o + c] = x;
      }
      __syncthreads();
    }
    if (t == 0) {
      if (m >= 2) {
        const cpx<double> x = A[(m - 1) * S + m - 2];
        dd[m - 2] = A[(m - 2) * S + m - 2].re;
        ee[m - 2] = sqrt(x.re * x.re + x.im * x.im);
      }
      dd[m - 1] = A[(m - 1) * S + m - 1].re;
      ee[m - 1] = 0.0;
      double lo = dd[0], hi = dd[0];
      for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? ee[i - 1] : 0.0) + ee[i];
        lo = fmin(lo, dd[i] - r);
        hi = fmax(hi, dd[i] + r);
      }
      scal[0] = lo - 1e-12 * (fabs(lo) + 1.0);
      scal[1] = hi + 1e-12 * (fabs(hi) + 1.0);
    }
    __syncthreads();
    // 5. bisection: eigenvalue n is the smallest x with #{eigenvalues < x} > n
    for (int n = t; n < m; n += NT) {
      double lo = scal[0], hi = scal[1];
      for (int it = 0; it < 100 && hi - lo > 4e-16 * fmax(fabs(lo), fabs(hi)); ++it) {
        const double x = 0.5 * (lo + hi);
        int cnt = 0;
        double qv = dd[0] - x;
        if (qv < 0.0) ++cnt;
        for (int i = 1; i < m; ++i) {
          const double den = qv != 0.0 ? qv : 1e-300;
          qv = dd[i] - x - ee[i - 1] * ee[i - 1] / den;
          if (qv < 0.0) ++cnt;
        }
        if (cnt > n) hi = x;
        else lo = x;
      }
      E[(size_t)q * m + n] = 0.5 * (lo + hi) + V;
    }
  }
}

// ------------------------------------------------------------- launchers
template <int M>
hipError_t launch_decimate(const Prob& P, const BatchDesc& b, const double* E, int nE, double eta, int sides,
                           const DecOpts& o, double2* scratch, int grid, double2* sig, double2* wf, double* sgn,
                           int* iters, int* nheavy, hipStream_t st) {
  hipLaunchKernelGGL((k_decimate<M>), dim3(grid), dim3(NT), 0, st, P, b, E, nE, eta, sides, o, scratch, sig, wf,
                     sgn, iters, nheavy);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_sigma_finish<M>), dim3(grid), dim3(NT), 0, st, P, b, E, nE, eta, sides, o, scratch, sig, wf,
                     sgn, nheavy);
  return hipGetLastError();
}

template <typename R, int M, bool MIX, bool DM = false, int PW = gj_pw<M>(), int TPP = (M <= 64 ? 2 : 1)>
hipError_t launch_sweep(const Prob& P, const SweepArgs& a, const BatchDesc& b, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_sweep<R, M, MIX, DM, PW, TPP>), dim3(grid), dim3(NT), 0, st, P, a, b);
  return hipGetLastError();
}

hipError_t run_decimate(int M, const Prob& P, const BatchDesc& b, const double* E, int nE, double eta, int sides,
                        const DecOpts& o, double2* scratch, int grid, double2* sig, double2* wf, double* sgn,
                        int* iters, int* nheavy, hipStream_t st) {
#define QTX_DEC(MM) \
  return launch_decimate<MM>(P, b, E, nE, eta, sides, o, scratch, grid, sig, wf, sgn, iters, nheavy, st)
  switch (M) {
    case 16: QTX_DEC(16);
    case 32: QTX_DEC(32);
    case 48: QTX_DEC(48);
    case 64: QTX_DEC(64);
    case 96: QTX_DEC(96);
    case 128: QTX_DEC(128);
    default: return hipErrorInvalidValue;
  }
#undef QTX_DEC
}

// Whether (panel width, refinement tiles per wave) is a built variant for
// block size M: panels of 16 or 32 columns that divide M, and one or two
// column tiles per wave in the mixed refinement for blocks of 48 and 64
// (smaller blocks have at most one tile per wave, larger ones one).
bool sweep_variant_ok(int M, bool mixed, int pw, int tpp) {
  if (pw != 16 && pw != 32) return false;
  if (M % pw != 0) return false;
  if (!mixed) return tpp == sweep_default_tpp(M);
  if (M == 48 || M == 64) return tpp == 1 || tpp == 2;
  return tpp == sweep_default_tpp(M);
}

// Dispatch over the built variants; an invalid combination returns
// hipErrorInvalidValue.
template <int M>
hipError_t sweep_dispatch(bool mixed, int pw, int tpp, const Prob& P, const SweepArgs& a, const BatchDesc& b, int grid,
                          hipStream_t st) {
  if (!sweep_variant_ok(M, mixed, pw, tpp)) return hipErrorInvalidValue;
  constexpr int D = M <= 64 ? 2 : 1;
  if (!mixed) {
    if constexpr (M % 32 == 0)
      if (pw == 32) return launch_sweep<double, M, false, false, 32, D>(P, a, b, grid, st);
    return launch_sweep<double, M, false, false, 16, D>(P, a, b, grid, st);
  }
  if constexpr (M == 48 || M == 64) {
    if constexpr (M % 32 == 0)
      if (pw == 32) return tpp == 1 ? launch_sweep<float, M, true, false, 32, 1>(P, a, b, grid, st)
                                    : launch_sweep<float, M, true, false, 32, 2>(P, a, b, grid, st);
    return tpp == 1 ? launch_sweep<float, M, true, false, 16, 1>(P, a, b, grid, st)
                    : launch_sweep<float, M, true, false, 16, 2>(P, a, b, grid, st);
  } else {
    if constexpr (M % 32 == 0)
      if (pw == 32) return launch_sweep<float, M, true, false, 32, D>(P, a, b, grid, st);
    return launch_sweep<float, M, true, false, 16, D>(P, a, b, grid, st);
  }
}

hipError_t run_sweep(int M, bool mixed, int pw, int tpp, const Prob& P, const SweepArgs& a, const BatchDesc& b,
                     int grid, hipStream_t st) {
  switch (M) {
    case 16: return sweep_dispatch<16>(mixed, pw, tpp, P, a, b, grid, st);
    case 32: return sweep_dispatch<32>(mixed, pw, tpp, P, a, b, grid, st);
    case 48: return sweep_dispatch<48>(mixed, pw, tpp, P, a, b, grid, st);
    case 64: return sweep_dispatch<64>(mixed, pw, tpp, P, a, b, grid, st);
    case 96: return sweep_dispatch<96>(mixed, pw, tpp, P, a, b, grid, st);
    case 128: return sweep_dispatch<128>(mixed, pw, tpp, P, a, b, grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t run_sweep_dm(int M, const Prob& P, const SweepArgs& a, int grid, hipStream_t st) {
  const BatchDesc b{};
#define QTX_SWEEP_DM(MM) return launch_sweep<double, MM, false, true>(P, a, b, grid, st)
  switch (M) {
    case 16: QTX_SWEEP_DM(16);
    case 32: QTX_SWEEP_DM(32);
    case 48: QTX_SWEEP_DM(48);
    case 64: QTX_SWEEP_DM(64);
    case 96: QTX_SWEEP_DM(96);
    case 128: QTX_SWEEP_DM(128);
    default: return hipErrorInvalidValue;
  }
#undef QTX_SWEEP_DM
}

hipError_t run_dm_reduce(const double2* rho, int nwg, size_t stride, int N, int M, int m, double2* out_d,
                         double2* out_o, hipStream_t st) {
  const size_t total = (2 * (size_t)N - 1) * m * m;
  const size_t blocks = (total + NT - 1) / NT;
  const int grid = (int)(blocks < 8192 ? blocks : 8192);
  hipLaunchKernelGGL(k_dm_reduce, dim3(grid), dim3(NT), 0, st, rho, nwg, stride, N, M, m, out_d, out_o);
  return hipGetLastError();
}

hipError_t run_bands(int M, const double2* lead, int m, double V, const double* k, int nk, double2* work, int grid,
                     double* E, hipStream_t st) {
#define QTX_BANDS(MM) \
  hipLaunchKernelGGL(k_bands<MM>, dim3(grid), dim3(NT), 0, st, lead, m, V, k, nk, work, E); \
  return hipGetLastError()
  switch (M) {
    case 16: QTX_BANDS(16);
    case 32: QTX_BANDS(32);
    case 48: QTX_BANDS(48);
    case 64: QTX_BANDS(64);
    case 96: QTX_BANDS(96);
    case 128: QTX_BANDS(128);
    default: return hipErrorInvalidValue;
  }
#undef QTX_BANDS
}

template <typename R, int M, bool MIX, int PW, int TPP>
hipError_t occ_sweep(int* n) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_sweep<R, M, MIX, false, PW, TPP>, NT, 0);
}

template <int M>
hipError_t max_resident_m(bool mixed, int pw, int tpp, int* sweep_wgs, int* dec_wgs, int* dm_wgs) {
  if (!sweep_variant_ok(M, mixed, pw, tpp)) return hipErrorInvalidValue;
  constexpr int D = M <= 64 ? 2 : 1;
  hipError_t e = hipSuccess;
  if (!mixed) {
    e = occ_sweep<double, M, false, 16, D>(sweep_wgs);
    if constexpr (M % 32 == 0)
      if (pw == 32) e = occ_sweep<double, M, false, 32, D>(sweep_wgs);
  } else if constexpr (M == 48 || M == 64) {
    e = tpp == 1 ? occ_sweep<float, M, true, 16, 1>(sweep_wgs) : occ_sweep<float, M, true, 16, 2>(sweep_wgs);
    if constexpr (M % 32 == 0)
      if (pw == 32) e = tpp == 1 ? occ_sweep<float, M, true, 32, 1>(sweep_wgs) : occ_sweep<float, M, true, 32, 2>(sweep_wgs);
  } else {
    e = occ_sweep<float, M, true, 16, D>(sweep_wgs);
    if constexpr (M % 32 == 0)
      if (pw == 32) e = occ_sweep<float, M, true, 32, D>(sweep_wgs);
  }
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(dec_wgs, k_decimate<M>, NT, 0);
  if (e == hipSuccess && dm_wgs)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(dm_wgs, k_sweep<double, M, false, true>, NT, 0);
  return e;
}

hipError_t max_resident(int M, bool mixed, int pw, int tpp, int* sweep_wgs, int* dec_wgs, int* dm_wgs) {
  switch (M) {
    case 16: return max_resident_m<16>(mixed, pw, tpp, sweep_wgs, dec_wgs, dm_wgs);
    case 32: return max_resident_m<32>(mixed, pw, tpp, sweep_wgs, dec_wgs, dm_wgs);
    case 48: return max_resident_m<48>(mixed, pw, tpp, sweep_wgs, dec_wgs, dm_wgs);
    case 64: return max_resident_m<64>(mixed, pw, tpp, sweep_wgs, dec_wgs, dm_wgs);
    case 96: return max_resident_m<96>(mixed, pw, tpp, sweep_wgs, dec_wgs, dm_wgs);
    case 128: return max_resident_m<128>(mixed, pw, tpp, sweep_wgs, dec_wgs, dm_wgs);
    default: return hipErrorInvalidValue;
  }
}

hipError_t run_compact(const int* redo, int nE, int* elist, int* ecount, hipStream_t st) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(64), 0, st, redo, nE, elist, ecount);
  return hipGetLastError();
}

}  // namespace qtx
