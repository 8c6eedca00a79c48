// Device-side building blocks for the transport kernels (gfx950, wave64).
//
// Complex numbers are kept as interleaved pairs in global memory and as
// separate real/imaginary MFMA accumulators in registers.  A complex GEMM
// tile uses four real MFMAs per k-slice:
//   Cr += Ar Br - Ai Bi,   Ci += Ar Bi + Ai Br.
//
// MFMA 16x16x4 operand layouts (lane l, g = l / 16, c = l % 16):
//   A operand: A[c][g], B operand: B[g][c] (both precisions);
//   accumulator register r holds D[4r + g][c] for f64 and D[4g + r][c] for f32.
// Within a 16-wide k block we let lane group g carry k = 4g + s in the s-th
// MFMA, so each lane reads four consecutive k of one A row.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qtx {

constexpr int NT = 256;          // threads per workgroup (4 wave64)
constexpr int NWAVE = NT / 64;

template <typename R> struct cpx { R re, im; };

template <typename R> struct vec2t;
template <> struct vec2t<double> { typedef double2 type; };
template <> struct vec2t<float> { typedef float2 type; };

template <typename R>
__device__ __forceinline__ cpx<R> mk(R re, R im) { cpx<R> z; z.re = re; z.im = im; return z; }
template <typename R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return mk<R>(a.re + b.re, a.im + b.im); }
template <typename R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return mk<R>(a.re - b.re, a.im - b.im); }
template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return mk<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// a - f * p
template <typename R>
__device__ __forceinline__ cpx<R> cfms(cpx<R> a, cpx<R> f, cpx<R> p) {
  return mk<R>(a.re - f.re * p.re + f.im * p.im, a.im - f.re * p.im - f.im * p.re);
}
template <typename R>
__device__ __forceinline__ cpx<R> cconj(cpx<R> a) { return mk<R>(a.re, -a.im); }
// 1/d from the hardware reciprocal estimate refined by Newton steps
// r <- r + r (1 - d r) (each step doubles the number of correct bits).
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float recip(float d) {
  float r = __builtin_amdgcn_rcpf(d);
  float e = fmaf(-d, r, 1.0f);
  return fmaf(r, e, r);
}
template <typename R>
__device__ __forceinline__ cpx<R> cinv(cpx<R> a) {
  const R r = recip(a.re * a.re + a.im * a.im);
  return mk<R>(a.re * r, -a.im * r);
}
template <typename R>
__device__ __forceinline__ R cabs1(cpx<R> a) { return fabs(a.re) + fabs(a.im); }

template <typename R>
__device__ __forceinline__ cpx<R> ld2(const typename vec2t<R>::type* p) {
  typename vec2t<R>::type v = *p;
  return mk<R>(v.x, v.y);
}
template <typename R>
__device__ __forceinline__ void st2(typename vec2t<R>::type* p, cpx<R> a) {
  typename vec2t<R>::type v;
  v.x = a.re;
  v.y = a.im;
  *p = v;
}
__device__ __forceinline__ cpx<double> ldd(const double2* p) { double2 v = *p; return mk<double>(v.x, v.y); }

template <typename R> struct mf;
template <> struct mf<double> {
  typedef double acc __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int g) { return 4 * r + g; }
};
template <> struct mf<float> {
  typedef float acc __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int g) { return 4 * g + r; }
};

// The lane index laundered through an empty asm: per-lane offsets derived
// from it are recomputed where they are used instead of being hoisted out
// of the slab loop and kept live (in registers) across the whole sweep.
__device__ __forceinline__ int lane_id() {
  int l = threadIdx.x & 63;
  asm volatile("" : "+v"(l));
  return l;
}

template <typename R> struct ctile {
  typename mf<R>::acc re, im;
};

template <typename R>
__device__ __forceinline__ void tzero(ctile<R>& t) {
  for (int r = 0; r < 4; ++r) { t.re[r] = 0; t.im[r] = 0; }
}

// acc += a * b for one k (per lane operands)
template <typename R>
__device__ __forceinline__ void cmac(ctile<R>& t, cpx<R> a, cpx<R> b) {
  t.re = mf<R>::op(a.re, b.re, t.re);
  t.re = mf<R>::op(-a.im, b.im, t.re);
  t.im = mf<R>::op(a.re, b.im, t.im);
  t.im = mf<R>::op(a.im, b.re, t.im);
}

// ---------------------------------------------------------------- operands
// A operand loaders: frag4(row, k0, out) -> out[s] = A[row][k0 + s].
// B operand loaders: get(k, col) -> B[k][col].

template <typename R> struct ALds {            // row-major in LDS
  const cpx<R>* p; int S;
  __device__ __forceinline__ cpx<R> get(int row, int k) const { return p[row * S + k]; }
};

struct ALdsF {                                 // FP64 row-major in LDS, read as FP32
  const cpx<double>* p; int S;
  __device__ __forceinline__ cpx<float> get(int row, int k) const {
    const cpx<double> v = p[row * S + k];
    return mk<float>((float)v.re, (float)v.im);
  }
};

// A[r][k] = -L[r][k], L the coupling of a slab to the previous one, made
// from the forward coupling blocks S, H (row-major) of that previous slab:
// L[r][k] = zu S[k][r]^* - H[k][r]^* (the transposed read of A = zS - H).
template <typename R> struct AGenL {
  const double2* S; const double2* H; cpx<double> zu; int M;
  __device__ __forceinline__ cpx<R> get(int r, int k) const {
    const cpx<double> sv = ldd(S + (size_t)k * M + r), hv = ldd(H + (size_t)k * M + r);
    const double re = zu.re * sv.re + zu.im * sv.im - hv.re;
    const double im = zu.im * sv.re - zu.re * sv.im + hv.im;
    return mk<R>((R)-re, (R)-im);
  }
};

template <typename R> struct AGlob {           // row-major global, optionally negated
  const typename vec2t<R>::type* p; int ld; R sgn;
  __device__ __forceinline__ cpx<R> get(int row, int k) const {
    cpx<R> v = ld2<R>(p + (size_t)row * ld + k);
    return mk<R>(sgn * v.re, sgn * v.im);
  }
};

template <typename R> struct AGlobCT {         // A[row][k] = conj(P[k][row]) (FP64 source)
  const double2* p; int ld;
  __device__ __forceinline__ cpx<R> get(int row, int k) const {
    cpx<double> v = ldd(p + (size_t)k * ld + row);
    return mk<R>((R)v.re, (R)-v.im);
  }
};

// A[row][k] = sg * (zv * conj(S[k][row]) - conj(H[k][row])): the coupling
// block back from slab i+1 to slab i, built from the forward blocks.
template <typename R> struct AGenCT {
  const double2* S; const double2* H; cpx<double> zv; double sg; int M;
  __device__ __forceinline__ cpx<R> get(int row, int k) const {
    cpx<double> sv = ldd(S + (size_t)k * M + row);
    cpx<double> hv = ldd(H + (size_t)k * M + row);
    double re = zv.re * sv.re + zv.im * sv.im - hv.re;
    double im = zv.im * sv.re - zv.re * sv.im + hv.im;
    return mk<R>((R)(sg * re), (R)(sg * im));
  }
};

// A[row][k] = sg * (zv * S[row][k] - H[row][k]): a block of zS - H
// generated from the stored blocks (FP64 source).
template <typename R> struct AGen {
  const double2* S; const double2* H; cpx<double> zv; double sg; int M;
  __device__ __forceinline__ cpx<R> get(int row, int k) const {
    cpx<double> sv = ldd(S + (size_t)row * M + k);
    cpx<double> hv = ldd(H + (size_t)row * M + k);
    double re = zv.re * sv.re - zv.im * sv.im - hv.re;
    double im = zv.re * sv.im + zv.im * sv.re - hv.im;
    return mk<R>((R)(sg * re), (R)(sg * im));
  }
};

template <class AF> struct ARows {             // rows r0, r0 + 1, ... of another A operand
  AF a; int r0;
  __device__ __forceinline__ auto get(int row, int k) const { return a.get(row + r0, k); }
};

template <typename R> struct BLds {            // row-major in LDS
  const cpx<R>* p; int ld;
  __device__ __forceinline__ cpx<R> get(int k, int col) const { return p[k * ld + col]; }
};

template <typename R> struct BGlob {
  const typename vec2t<R>::type* p; int ld;
  __device__ __forceinline__ cpx<R> get(int k, int col) const { return ld2<R>(p + (size_t)k * ld + col); }
};

template <typename R> struct BGlobD {          // FP64 source, cast to R
  const double2* p; int ld;
  __device__ __forceinline__ cpx<R> get(int k, int col) const {
    cpx<double> v = ldd(p + (size_t)k * ld + col);
    return mk<R>((R)v.re, (R)v.im);
  }
};

template <typename R> struct BGlobF {          // FP32 source, widened to R
  const float2* p; int ld;
  __device__ __forceinline__ cpx<R> get(int k, int col) const {
    float2 v = p[(size_t)k * ld + col];
    return mk<R>((R)v.x, (R)v.y);
  }
};

template <class BF> struct BPerm {             // rows taken in the order piv[k]
  BF b; const int* piv;
  __device__ __forceinline__ auto get(int k, int col) const { return b.get(piv[k], col); }
};

// B[k][col] = zv * S[k][col] - H[k][col]
template <typename R> struct BGen {
  const double2* S; const double2* H; cpx<double> zv; int M;
  __device__ __forceinline__ cpx<R> get(int k, int col) const {
    cpx<double> sv = ldd(S + (size_t)k * M + col);
    cpx<double> hv = ldd(H + (size_t)k * M + col);
    return mk<R>((R)(zv.re * sv.re - zv.im * sv.im - hv.re), (R)(zv.re * sv.im + zv.im * sv.re - hv.im));
  }
};

// B[k][col] = zv * conj(S[col][k]) - conj(H[col][k]): the coupling block
// back from slab j+1 to slab j as a B operand.
template <typename R> struct BGenCT {
  const double2* S; const double2* H; cpx<double> zv; int M;
  __device__ __forceinline__ cpx<R> get(int k, int col) const {
    cpx<double> sv = ldd(S + (size_t)col * M + k);
    cpx<double> hv = ldd(H + (size_t)col * M + k);
    return mk<R>((R)(zv.re * sv.re + zv.im * sv.im - hv.re), (R)(zv.im * sv.re - zv.re * sv.im + hv.im));
  }
};

// A[row][k] = w_k P[row][k] with w_k = wR sR[k] for k < M and wL sL[k - M]
// above: a solution block [right-injected | left-injected] with each
// column weighted by its broadening sign and its contact's weight.
struct APsiW {
  const double2* p; int ld; const double* sR; const double* sL; double wR, wL; int M;
  __device__ __forceinline__ cpx<double> get(int row, int k) const {
    const double w = k < M ? wR * sR[k] : wL * sL[k - M];
    const cpx<double> v = ldd(p + (size_t)row * ld + k);
    return mk<double>(w * v.re, w * v.im);
  }
};

// B[k][col] = conj(P[col][k]): the conjugate transpose of a solution block.
struct BPsiH {
  const double2* p; int ld;
  __device__ __forceinline__ cpx<double> get(int k, int col) const {
    const cpx<double> v = ldd(p + (size_t)col * ld + k);
    return mk<double>(v.re, -v.im);
  }
};

// acc[ti] (ti = 0..MT-1, a full column of tiles) += A[:, 0:16*KT] * B[0:16*KT, tile tj].
// One k-slice per step (lane group g carries k = 16 kb + 4 g + s); the
// operands of the next slice are loaded while the MFMAs of the current one
// run, and the real/imaginary chains of the MT tiles are interleaved so that
// no MFMA waits on the accumulator of the one before it.
template <typename R, int MT, int KT, class AF, class BF>
__device__ __forceinline__ void cgemm_col(ctile<R> (&acc)[MT], const AF& A, const BF& B, int tj) {
  const int lane = lane_id(), g = lane >> 4, c = lane & 15;
  const int col = 16 * tj + c;
  cpx<R> bq, aq[MT];
  {
    const int k = 4 * g;
    bq = B.get(k, col);
#pragma unroll
    for (int ti = 0; ti < MT; ++ti) aq[ti] = A.get(16 * ti + c, k);
  }
#pragma unroll 2
  for (int it = 0; it < 4 * KT; ++it) {
    cpx<R> bn = bq, an[MT];
#pragma unroll
    for (int ti = 0; ti < MT; ++ti) an[ti] = aq[ti];
    if (it + 1 < 4 * KT) {
      const int k = 16 * ((it + 1) >> 2) + 4 * g + ((it + 1) & 3);
      bn = B.get(k, col);
#pragma unroll
      for (int ti = 0; ti < MT; ++ti) an[ti] = A.get(16 * ti + c, k);
    }
#pragma unroll
    for (int ti = 0; ti < MT; ++ti) {
      acc[ti].re = mf<R>::op(aq[ti].re, bq.re, acc[ti].re);
      acc[ti].im = mf<R>::op(aq[ti].re, bq.im, acc[ti].im);
    }
#pragma unroll
    for (int ti = 0; ti < MT; ++ti) {
      acc[ti].re = mf<R>::op(-aq[ti].im, bq.im, acc[ti].re);
      acc[ti].im = mf<R>::op(aq[ti].im, bq.re, acc[ti].im);
    }
    bq = bn;
#pragma unroll
    for (int ti = 0; ti < MT; ++ti) aq[ti] = an[ti];
    __builtin_amdgcn_sched_barrier(0);
  }
}

// B with its contraction index shifted by k0: B'[k][col] = B[k0 + k][col].
template <class BF> struct BOff {
  BF b; int k0;
  __device__ __forceinline__ auto get(int k, int col) const { return b.get(k0 + k, col); }
};

// Row stride (complex elements) of a staged 16-column slice of A in LDS.
constexpr int kStageStride = 17;

// cgemm_col over the whole contraction (M = 16 MT) with A staged through
// LDS in slices of 16 columns (buf: M * kStageStride elements): the
// workgroup loads each slice once, coalesced, and all its waves read it
// from LDS, where cgemm_col has every wave read all of A from the caches.
// For A in global memory that every wave needs (blocks above 64).  Takes
// two barriers per slice: every wave of the workgroup must make the same
// sequence of calls.  ACOL: the threads walk the slice down its columns
// (for an A stored transposed, so that the reads stay coalesced), else
// along its rows.
template <typename R, int MT, bool ACOL = false, class AF, class BF>
__device__ __forceinline__ void cgemm_col_staged(ctile<R> (&acc)[MT], const AF& A, const BF& B, int tj, cpx<R>* buf) {
  constexpr int M = 16 * MT;
  const int t = threadIdx.x;
#pragma unroll 1
  for (int k0 = 0; k0 < M; k0 += 16) {
    __syncthreads();                                // the previous slice is consumed
    for (int idx = t; idx < M * 16; idx += NT) {
      int r, kk;
      if constexpr (ACOL) {
        kk = idx / M;
        r = idx - kk * M;
      } else {
        r = idx >> 4;
        kk = idx & 15;
      }
      buf[r * kStageStride + kk] = A.get(r, k0 + kk);
    }
    __syncthreads();
    cgemm_col<R, MT, 1>(acc, ALds<R>{buf, kStageStride}, BOff<BF>{B, k0}, tj);
  }
}

// Visit the elements held by this lane in a column of tiles:
// fn(row, col, re, im, ti, r).
template <typename R, int MT, class F>
__device__ __forceinline__ void tiles_foreach(ctile<R> (&acc)[MT], int tj, F fn) {
  const int lane = lane_id(), g = lane >> 4, c = lane & 15;
#pragma unroll
  for (int ti = 0; ti < MT; ++ti) {
#pragma unroll
    for (int r = 0; r < 4; ++r) fn(16 * ti + mf<R>::row(r, g), 16 * tj + c, ti, r);
    // one tile's loads in flight at a time (otherwise all are hoisted)
    __builtin_amdgcn_sched_barrier(0);
  }
}

// ------------------------------------------------------------ reductions
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = __shfl_xor(lo, m, 64);
  hi = __shfl_xor(hi, m, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    uint64_t o = shfl_xor_u64(v, m);
    v = o > v ? o : v;
  }
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}
__device__ __forceinline__ double wave_maxd(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
  return v;
}

// Sum over the workgroup; every thread gets the same value (summed in the
// same order).  red: NWAVE doubles of LDS.  Contains two barriers.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < NWAVE; ++q) s += red[q];
  __syncthreads();
  return s;
}

// Max over the 64 lanes of a wave with DPP row shifts and row broadcasts;
// the result (lane 63) is returned wave-uniform.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  uint32_t o;
  o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false); v = o > v ? o : v;  // row_shr:1
  o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false); v = o > v ? o : v;  // row_shr:2
  o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false); v = o > v ? o : v;  // row_shr:4
  o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false); v = o > v ? o : v;  // row_shr:8
  o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false); v = o > v ? o : v;  // row_bcast:15
  o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false); v = o > v ? o : v;  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float readlane_d(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// 32-bit pivot key: magnitude (float, low 8 mantissa bits dropped) above
// 255 - row, so ties within 2^-15 relative go to the smaller row; used
// rows take key 0.  Rows < 128.
template <typename R>
__device__ __forceinline__ uint32_t pivot_key32(cpx<R> v, int row) {
  const float mag = (float)cabs1(v);
  return (__float_as_uint(mag) & 0xffffff00u) | (uint32_t)(255 - row);
}

// Pivot key: larger magnitude wins, ties go to the smaller row index; used
// rows get key 0 and lose to every unused row.
template <typename R>
__device__ __forceinline__ uint64_t pivot_key(cpx<R> v, int idx, int M) {
  float mag = (float)cabs1(v);
  return ((uint64_t)__float_as_uint(mag) << 32) | (uint32_t)(M - idx);
}

}  // namespace qtx
