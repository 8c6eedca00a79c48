// Contact self-energies and mode-space injection from the complex band
// structure of the leads (Sec. "Contact self-energies", the direct method):
//
//   1. the quadratic eigenvalue problem (L lambda^-1 + D0 + lambda U) c = 0
//      of a lead (A = zS - H convention: D0 = z S00 - H00, U = z S01 - H01,
//      L = z S01^H - H01^H) in the symmetric linearisation of
//      eq. linearized_eigenvalue_symmetric, [[D0, L], [U, 0]] x =
//      lambda [[-U, 0], [0, U]] x with x = [lambda c; c], brought to the
//      standard problem C x = lambda x by the block-diagonal right-hand
//      matrix: C = [[-U^-1 D0, -U^-1 L], [I, 0]].  When U is singular (a
//      coupling of lower rank than the slab) that pencil is singular too:
//      its determinant carries det U as a factor for every lambda.  The
//      quadratic is then taken in the variable nu of the disk automorphism
//      lambda = (nu + s) / (1 + conj(s) nu), |s| < 1: multiplying
//      L + lambda D0 + lambda^2 U by (1 + conj(s) nu)^2 gives
//      L' + nu D0' + nu^2 U' with U' = U + conj(s) D0 + conj(s)^2 L,
//      D0' = 2 conj(s) L + (1 + |s|^2) D0 + 2 s U, L' = L + s D0 + s^2 U,
//      whose leading coefficient is invertible unless 1/conj(s) is a Bloch
//      factor.  The mode vectors c are unchanged, |lambda| < 1, = 1, > 1
//      exactly when |nu| is, and lambda = infinity (a mode annihilated by
//      U) is the finite nu = -1/conj(s).  s = 0 (the plain form) is taken
//      when kappa_F(U) <= kModeKappa, else the first of the other shifts
//      that meets it, else the best of them;
//   2. all 2m eigenpairs of C: Householder reduction to Hessenberg form,
//      complex single-shift QR (Wilkinson shifts, Givens bulge chase) to
//      the Schur form T = Q^H C Q, eigenvectors of T by back substitution,
//      x = Q y;
//   3. the mode split of eq. hellmann-feynman: at eta = 0 a mode with
//      ||lambda| - 1| <= tol travels, in the direction of the sign of its
//      flux J = 2 Im(lambda c^H U c) (the numerator of the generalised
//      Hellmann-Feynman velocity); other modes decay to the right iff
//      |lambda| < 1; at eta > 0 the split is |lambda| < 1 alone;
//   4. Sigma_R = -U B+ Lambda+ B+^-1 and Sigma_L = -L B- Lambda-^-1 B-^-1
//      from the right- and left-going Bloch matrices;
//   5. injection of the incoming travelling modes only, eq. qtbm_system with
//      B_gamma = (-L lambda^-1 - Sigma_L) c (source) or
//      (-U lambda - Sigma_R) c (drain), each scaled by 1/sqrt|J_gamma|.
//      With modes normalised as in eq. normalization and g = 2/|v| this
//      is the same injection: sum_gamma W_gamma W_gamma^H = Gamma at eta = 0,
//      so the sweep takes W with signs +1 (and 0 on unused columns).
//
// Jobs (energy, lead) run in batches through three kernels that share one
// workspace slot per job (16 M^2 complex doubles): k_modes_hess (steps 1
// and the Hessenberg form), k_modes_qr (the Schur form; in LDS for M <= 64)
// and k_modes_post (eigenvectors and steps 3-5).  Only rows m..2m-1 of the
// Schur vectors are formed: the mode vectors c are that half of the
// eigenvectors.  The outputs have the layout of the decimation's: Sigma, W
// (padded M x M), signs (M), iteration count (the QR sweeps; -1 if the QR
// did not converge, a matrix was singular or the split did not give m modes
// each way).
#include "qtx_device.h"
#include "qtx_internal.h"

namespace qtx {
namespace {

typedef cpx<double> cd;

__device__ __forceinline__ void sto(double2* p, cd v) { *p = make_double2(v.re, v.im); }
__device__ __forceinline__ cd cdivx(cd a, cd b) {
  // a / b with IEEE division (used where accuracy matters more than speed)
  const double s = fabs(b.re) + fabs(b.im);
  const double br = b.re / s, bi = b.im / s, ar = a.re / s, ai = a.im / s;
  const double d = br * br + bi * bi;
  return mk<double>((ar * br + ai * bi) / d, (ai * br - ar * bi) / d);
}
__device__ __forceinline__ double cabsx(cd a) { return hypot(a.re, a.im); }
__device__ __forceinline__ cd csqrtx(cd z) {
  const double r = cabsx(z);
  if (r == 0.0) return mk<double>(0.0, 0.0);
  const double a = sqrt(0.5 * (r + fabs(z.re)));
  if (z.re >= 0.0) return mk<double>(a, z.im / (2.0 * a));
  return mk<double>(fabs(z.im) / (2.0 * a), z.im >= 0.0 ? a : -a);
}
__device__ __forceinline__ cd cscl(cd a, double s) { return mk<double>(a.re * s, a.im * s); }

// 1/sqrt(a), a > 0: hardware estimate and two Newton steps
// y <- y (3 - a y^2) / 2 (each roughly doubles the correct bits).
__device__ __forceinline__ double rsqrt_nr(double a) {
  double y = __builtin_amdgcn_rsq(a);
  y = y * fma(-0.5 * a, y * y, 1.5);
  return y * fma(-0.5 * a, y * y, 1.5);
}

// Givens rotation G = [[c, s], [-conj(s), c]] (c real >= 0) with
// G [x; y] = [r x / |x|; 0], r = sqrt(|x|^2 + |y|^2):
// c = |x| / r, s = (x / |x|) conj(y) / r; for x = 0, c = 0, s = conj(y) / |y|.
__device__ __forceinline__ void givens(cd x, cd y, double* c, cd* s) {
  const double ax2 = x.re * x.re + x.im * x.im, ay2 = y.re * y.re + y.im * y.im;
  const double r2 = ax2 + ay2;
  if (!(r2 > 0.0)) {
    *c = 1.0;
    *s = mk<double>(0.0, 0.0);
  } else if (ax2 == 0.0) {
    const double iy = rsqrt_nr(ay2);
    *c = 0.0;
    *s = mk<double>(y.re * iy, -y.im * iy);
  } else {
    const double ix = rsqrt_nr(ax2), ir = rsqrt_nr(r2);
    *c = ax2 * ix * ir;
    const double f = ix * ir;
    *s = cscl(cmul(x, cconj(y)), f);
  }
}

// Inverse of the n x n matrix in columns [0, n) of A (row stride ld) by
// Gauss-Jordan elimination with partial pivoting on [A | I]; the inverse is
// left in columns [n, 2n).  fcol: n complex values of LDS.  Returns false
// (uniformly) if a pivot is zero or not finite.
__device__ bool gj_invert(double2* A, int n, int ld, cd* fcol, double* sd, int* si) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int idx = t; idx < n * n; idx += NT) {
    const int r = idx / n, c = idx - r * n;
    A[(size_t)r * ld + n + c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (w == 0) {
      double best = -1.0;
      int bi = k;
      for (int i = k + lane; i < n; i += 64) {
        const double a = cabs1(ldd(A + (size_t)i * ld + k));
        if (a > best) { best = a; bi = i; }
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) { si[0] = bi; sd[0] = best; }
    }
    __syncthreads();
    const int p = si[0];
    const double pv = sd[0];
    if (!(pv > 0.0) || !isfinite(pv)) return false;
    if (p != k)
      for (int j = t; j < 2 * n; j += NT) {
        const double2 a = A[(size_t)k * ld + j];
        A[(size_t)k * ld + j] = A[(size_t)p * ld + j];
        A[(size_t)p * ld + j] = a;
      }
    __syncthreads();
    for (int i = t; i < n; i += NT) fcol[i] = ldd(A + (size_t)i * ld + k);
    __syncthreads();
    const cd pinv = cdivx(mk<double>(1.0, 0.0), fcol[k]);
    for (int j = t; j < 2 * n; j += NT) sto(A + (size_t)k * ld + j, cmul(pinv, ldd(A + (size_t)k * ld + j)));
    __syncthreads();
    for (int idx = t; idx < n * 2 * n; idx += NT) {
      const int i = idx / (2 * n), j = idx - i * 2 * n;
      if (i == k) continue;
      const cd f = fcol[i];
      sto(A + (size_t)i * ld + j, cfms(ldd(A + (size_t)i * ld + j), f, ldd(A + (size_t)k * ld + j)));
    }
    __syncthreads();
  }
  return true;
}

struct ModeShared {
  cd vec[256];          // Householder vector / Gauss-Jordan factor column
  cd lam[256];          // Bloch factors lambda
  cd lami[256];         // their inverses (0 for lambda = infinity)
  double J[256];        // fluxes
  int kind[256];        // 1 right-going, 0 left-going; +2 if travelling
  int ridx[128], lidx[128];
  double rc[256];       // rotations of one QR sweep (cosine, sine)
  cd rs[256];
  cd xy[2][2];          // the next rotation's pair, from the column update
  cd bulge;             // the entry below the subdiagonal during a sweep
  double sd[4];
  int si[8];
};

// Upper Hessenberg matrix with row stride ld in global memory.
struct HGlob {
  double2* p; int ld;
  __device__ __forceinline__ cd get(int i, int j) const { return ldd(p + (size_t)i * ld + j); }
  __device__ __forceinline__ void put(int i, int j, cd v) const { sto(p + (size_t)i * ld + j, v); }
};

// Upper Hessenberg matrix packed by rows in LDS: row i holds columns
// max(i - 1, 0) .. n - 1, n + (n - 1)(n + 2)/2 entries in all.
struct HLds {
  cd* p; int n;
  __device__ __forceinline__ int at(int i, int j) const {
    return i == 0 ? j : n + (i - 1) * (n + 1) - ((i - 1) * i) / 2 + j - (i - 1);
  }
  __device__ __forceinline__ cd get(int i, int j) const { return p[at(i, j)]; }
  __device__ __forceinline__ void put(int i, int j, cd v) const { p[at(i, j)] = v; }
};
constexpr int hpack(int n) { return n + (n - 1) * (n + 2) / 2; }

// Complex Schur form of the n x n upper Hessenberg matrix H by single-shift
// QR: deflation where a subdiagonal entry falls below eps times its
// neighbouring diagonal, Wilkinson shifts (an exceptional shift every tenth
// iteration on one eigenvalue), and an implicit sweep of Givens rotations
// G = [[c, s], [-conj(s), c]] that chases the bulge down the window.  Only
// H itself is updated inside a sweep (two barriers per rotation; the bulge
// and the next rotation's pair are passed through LDS); the sweep's
// rotations are applied to rows n/2..n-1 of the Schur vectors Q (global,
// stride ld; the only rows used later) after it, row by row without
// barriers.  Returns false if more than 30 n sweeps were needed; *total
// counts the sweeps.
template <class HA>
__device__ bool schur_qr(const HA& H, int n, double2* Qm, int ld, ModeShared& sh, int* total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const double eps = 2.220446049250313e-16;
  const int maxit = 30 * n;
  int hi = n - 1, its = 0;
  *total = 0;
  while (hi > 0) {
    if (w == 0) {
      int found = 0;
      for (int l = 1 + lane; l <= hi; l += 64) {
        const double h = cabs1(H.get(l, l - 1));
        const double tst = cabs1(H.get(l - 1, l - 1)) + cabs1(H.get(l, l));
        if (h <= eps * tst || h == 0.0) found = l > found ? l : found;
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(found, off, 64);
        found = o > found ? o : found;
      }
      if (lane == 0) {
        sh.si[1] = found;
        if (found > 0) H.put(found, found - 1, mk<double>(0.0, 0.0));
      }
    }
    __syncthreads();
    const int l = sh.si[1];
    if (l == hi) {
      --hi;
      its = 0;
      __syncthreads();          // every thread has read the deflation index
      continue;
    }
    if (++*total > maxit) return false;
    ++its;
    // shift: the eigenvalue of the trailing 2 x 2 block nearer its corner
    const cd a = H.get(hi - 1, hi - 1), b = H.get(hi - 1, hi), c = H.get(hi, hi - 1), d = H.get(hi, hi);
    cd sigma;
    if (its % 10 == 0) {
      sigma = mk<double>(d.re + 0.75 * fabs(c.re), d.im);       // exceptional shift
    } else {
      const cd hm = cscl(csub(a, d), 0.5);
      const cd r = csqrtx(cadd(cmul(hm, hm), cmul(b, c)));
      const cd mid = cscl(cadd(a, d), 0.5);
      const cd s1 = cadd(mid, r), s2 = csub(mid, r);
      sigma = cabs1(csub(s1, d)) <= cabs1(csub(s2, d)) ? s1 : s2;
    }
    const cd x0 = csub(H.get(l, l), sigma), y0 = H.get(l + 1, l);
    __syncthreads();            // every thread has read what the sweep overwrites
    for (int k = l; k < hi; ++k) {
      const cd x = k == l ? x0 : sh.xy[k & 1][0];
      const cd y = k == l ? y0 : sh.xy[k & 1][1];
      double cs;
      cd sn;
      givens(x, y, &cs, &sn);
      if (t == 0) {
        sh.rc[k - l] = cs;
        sh.rs[k - l] = sn;
      }
      // rows k, k+1 from the left by G (column k-1 of row k+1 is the bulge)
      const int j0 = k == l ? l : k - 1;
      for (int j = j0 + t; j < n; j += NT) {
        const cd p = H.get(k, j);
        const cd q = j == k - 1 ? sh.bulge : H.get(k + 1, j);
        H.put(k, j, cadd(cscl(p, cs), cmul(sn, q)));
        if (j >= k) H.put(k + 1, j, csub(cscl(q, cs), cmul(cconj(sn), p)));
      }
      __syncthreads();
      // columns k, k+1 from the right by G^H; row k+2 gets the new bulge
      const int i1 = k + 2 < hi ? k + 2 : hi;
      for (int i = t; i <= i1; i += NT) {
        const cd p = i <= k + 1 ? H.get(i, k) : mk<double>(0.0, 0.0);
        const cd q = H.get(i, k + 1);
        const cd np = cadd(cscl(p, cs), cmul(cconj(sn), q));
        H.put(i, k + 1, csub(cscl(q, cs), cmul(sn, p)));
        if (i <= k + 1) H.put(i, k, np);
        else sh.bulge = np;
        if (i == k + 1) sh.xy[(k + 1) & 1][0] = np;
        if (i == k + 2) sh.xy[(k + 1) & 1][1] = np;
      }
      __syncthreads();
    }
    // the sweep's rotations on the Schur vectors: Q <- Q G^H, row by row
    // (rows n/2.. only, the ones the mode vectors use; columns l+1..hi are
    // loaded eight at a time so that their latencies overlap)
    for (int i = n / 2 + t; i < n; i += NT) {
      double2* Qi = Qm + (size_t)i * ld;
      cd carry = ldd(Qi + l);
      for (int k0 = l; k0 < hi; k0 += 8) {
        cd v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = k0 + u < hi ? ldd(Qi + k0 + u + 1) : mk<double>(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = k0 + u;
          if (k < hi) {
            const double cs = sh.rc[k - l];
            const cd sn = sh.rs[k - l];
            sto(Qi + k, cadd(cscl(carry, cs), cmul(cconj(sn), v[u])));
            carry = csub(cscl(v[u], cs), cmul(sn, carry));
          }
        }
      }
      sto(Qi + hi, carry);
    }
  }
  return true;
}

// Cross-lane ordering of LDS accesses inside one wave (LDS executes a
// wave's accesses in order; this keeps the compiler from reordering them).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// schur_qr for n <= 128 with H in LDS: wave 0 runs the deflation tests and
// the bulge chase alone (lane-parallel rows and columns, no block barrier
// inside a sweep), writing each sweep's rotations to one of two buffers;
// meanwhile waves 1..3 apply the previous sweep's rotations to rows
// n/2..n-1 of Q.  One block barrier per sweep.
__device__ bool schur_qr_wave(const HLds& H, int n, double2* Qm, int ld, ModeShared& sh, int* total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const double eps = 2.220446049250313e-16;
  const int maxit = 30 * n;
  // wave 0 state (uniform within the wave)
  int hi = n - 1, its = 0, tot = 0, buf = 0;
  // block state: sh.si[3] = 1 while sweeps come, 0 when converged, -1 failed;
  // sh.si[4 + b], sh.si[6 + b]: window (l, hi) of the sweep in buffer b
  bool pending = false;                 // waves 1..3: a sweep waits in buffer buf ^ 1
  for (;;) {
    if (w == 0) {
      int state = 0;
      while (hi > 0) {
        int found = 0;
        for (int l = 1 + lane; l <= hi; l += 64) {
          const double h = cabs1(H.get(l, l - 1));
          const double tst = cabs1(H.get(l - 1, l - 1)) + cabs1(H.get(l, l));
          if (h <= eps * tst || h == 0.0) found = l > found ? l : found;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
          const int o = __shfl_xor(found, off, 64);
          found = o > found ? o : found;
        }
        const int l = found;
        if (l > 0 && lane == 0) H.put(l, l - 1, mk<double>(0.0, 0.0));
        wave_sync();
        if (l == hi) {
          --hi;
          its = 0;
          continue;
        }
        if (++tot > maxit) {
          state = -1;
          break;
        }
        ++its;
        const cd a = H.get(hi - 1, hi - 1), b = H.get(hi - 1, hi), c = H.get(hi, hi - 1), d = H.get(hi, hi);
        cd sigma;
        if (its % 10 == 0) {
          sigma = mk<double>(d.re + 0.75 * fabs(c.re), d.im);
        } else {
          const cd hm = cscl(csub(a, d), 0.5);
          const cd r = csqrtx(cadd(cmul(hm, hm), cmul(b, c)));
          const cd mid = cscl(cadd(a, d), 0.5);
          const cd s1 = cadd(mid, r), s2 = csub(mid, r);
          sigma = cabs1(csub(s1, d)) <= cabs1(csub(s2, d)) ? s1 : s2;
        }
        // x, y: the pair the next rotation annihilates against (y is also
        // the bulge below the subdiagonal), broadcast from the lanes that
        // produced them
        cd x = csub(H.get(l, l), sigma), y = H.get(l + 1, l);
        wave_sync();
        double* rc = sh.rc + 128 * buf;
        cd* rs = sh.rs + 128 * buf;
        for (int k = l; k < hi; ++k) {
          double cs;
          cd sn;
          givens(x, y, &cs, &sn);
          if (lane == 0) {
            rc[k - l] = cs;
            rs[k - l] = sn;
          }
          // each lane owns columns j0 + lane and j0 + lane + 64 (n <= 128):
          // both pairs are loaded before either is stored, so that the two
          // LDS round trips overlap
          const int j0 = k == l ? l : k - 1;
          {
            const int ja = j0 + lane, jb = ja + 64;
            const bool va = ja < n, vb = jb < n;
            const cd zero = mk<double>(0.0, 0.0);
            const cd pa = va ? H.get(k, ja) : zero, pb = vb ? H.get(k, jb) : zero;
            const cd qa = va ? (ja == k - 1 ? y : H.get(k + 1, ja)) : zero;
            const cd qb = vb ? H.get(k + 1, jb) : zero;
            if (va) {
              H.put(k, ja, cadd(cscl(pa, cs), cmul(sn, qa)));
              if (ja >= k) H.put(k + 1, ja, csub(cscl(qa, cs), cmul(cconj(sn), pa)));
            }
            if (vb) {
              H.put(k, jb, cadd(cscl(pb, cs), cmul(sn, qb)));
              H.put(k + 1, jb, csub(cscl(qb, cs), cmul(cconj(sn), pb)));
            }
          }
          wave_sync();
          // rows lane and lane + 64 of columns k, k+1 (row k+2 takes the bulge)
          const int i1 = k + 2 < hi ? k + 2 : hi;
          {
            const int ia = lane, ib = lane + 64;
            const bool va = ia <= i1, vb = ib <= i1;
            const cd zero = mk<double>(0.0, 0.0);
            const cd pa = va && ia <= k + 1 ? H.get(ia, k) : zero, pb = vb && ib <= k + 1 ? H.get(ib, k) : zero;
            const cd qa = va ? H.get(ia, k + 1) : zero, qb = vb ? H.get(ib, k + 1) : zero;
            const cd npa = cadd(cscl(pa, cs), cmul(cconj(sn), qa));
            const cd npb = cadd(cscl(pb, cs), cmul(cconj(sn), qb));
            if (va) {
              H.put(ia, k + 1, csub(cscl(qa, cs), cmul(sn, pa)));
              if (ia <= k + 1) H.put(ia, k, npa);
            }
            if (vb) {
              H.put(ib, k + 1, csub(cscl(qb, cs), cmul(sn, pb)));
              if (ib <= k + 1) H.put(ib, k, npb);
            }
            // next pair: new (k+1, k) and the bulge (k+2, k), from their lanes
            const cd xs = k + 1 < 64 ? npa : npb, ys = k + 2 < 64 ? npa : npb;
            x = mk<double>(readlane_d(xs.re, (k + 1) & 63), readlane_d(xs.im, (k + 1) & 63));
            y = mk<double>(readlane_d(ys.re, (k + 2) & 63), readlane_d(ys.im, (k + 2) & 63));
          }
          wave_sync();
        }
        if (lane == 0) {
          sh.si[4 + buf] = l;
          sh.si[6 + buf] = hi;
        }
        state = 1;
        break;
      }
      if (lane == 0) sh.si[3] = state;
    } else if (pending) {
      // the previous sweep's rotations on the Schur vectors: Q <- Q G^H
      const int b = buf ^ 1;
      const int l = sh.si[4 + b], h = sh.si[6 + b];
      const double* rc = sh.rc + 128 * b;
      const cd* rs = sh.rs + 128 * b;
      for (int i = n / 2 + t - 64; i < n; i += NT - 64) {   // rows the mode vectors use
        double2* Qi = Qm + (size_t)i * ld;
        cd carry = ldd(Qi + l);
        for (int k0 = l; k0 < h; k0 += 8) {
          cd v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = k0 + u < h ? ldd(Qi + k0 + u + 1) : mk<double>(0.0, 0.0);
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int k = k0 + u;
            if (k < h) {
              const double cs = rc[k - l];
              const cd sn = rs[k - l];
              sto(Qi + k, cadd(cscl(carry, cs), cmul(cconj(sn), v[u])));
              carry = csub(cscl(v[u], cs), cmul(sn, carry));
            }
          }
        }
        sto(Qi + h, carry);
      }
    }
    __syncthreads();
    const int state = sh.si[3];
    __syncthreads();                    // every thread has read the state
    if (state == 1) {                   // waves 1..3 apply this sweep in the next round
      pending = true;
      buf ^= 1;
      continue;
    }
    // converged (the last sweep was applied in this round) or failed
    *total = tot;
    return state == 0;
  }
}

}  // namespace

// Shifts s of the eigenvalue variable (step 1 of the header): 0, then three
// points of modulus about 1/2 spread around the disk.
constexpr int kModeShifts = 4;
constexpr double kModeKappa = 1e8;     // largest kappa_F of U' taken without trying the next shift
__device__ __forceinline__ cd mode_shift(int q) {
  switch (q) {
    case 1: return mk<double>(0.3108049841353322, 0.3916634548137417);      // 0.5 e^{0.9 i}
    case 2: return mk<double>(-0.42844437668447366, 0.2577506859107321);    // 0.5 e^{2.6 i}
    case 3: return mk<double>(-0.05798002243298609, -0.44624916470361087);  // 0.45 e^{-1.7 i}
    default: return mk<double>(0.0, 0.0);
  }
}

// Stage 1 (per job): C = [[-U'^-1 D0', -U'^-1 L'], [I, 0]] of the shifted
// quadratic and its Hessenberg form with the accumulated reflectors; the
// shift taken in shift[jl].  jst[jl] = 0, or -1 if no U' could be inverted.
template <int M>
__global__ __launch_bounds__(NT) void k_modes_hess(Prob P, const double* E, double eta, int sides, double tol, int m, int j0, int nb, double2* ws, int* jst, double2* shift) {
  __shared__ ModeShared sh;
  constexpr int LD = 2 * M, MM = M * M;
  constexpr size_t WS = 16 * (size_t)M * M;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  (void)lane;
  (void)w;
  const int n = 2 * m;
  const double eps = 2.220446049250313e-16;
  (void)eps;
  for (int jl = blockIdx.x; jl < nb; jl += gridDim.x) {
    const int job = j0 + jl;
    double2* Cm = ws + (size_t)jl * WS;          // C, then its Schur form T (n x n, stride LD)
    double2* Qm = Cm + 4 * (size_t)MM;           // Schur vectors
    double2* Yv = Qm + 4 * (size_t)MM;           // [D0 | L], then eigenvectors of T, then products
    double2* Ui = Yv + 4 * (size_t)MM;           // Gauss-Jordan work (m x 2m)
    double2* Cv = Ui + 2 * (size_t)MM;           // mode vectors c (m x n)
    (void)Yv;
    (void)Ui;
    (void)Cv;
    const int e = job / sides;
    const int side = sides == 2 ? job - 2 * e : -1;       // -1: both surfaces from the left lead
    const double2* lead = side == 1 ? P.leadR : P.leadL;
    const double V = side == 1 ? P.VR : P.VL;
    const cd zx = mk<double>(E[e] - V, eta);
    const double2* H00 = lead;
    const double2* H01 = lead + MM;
    const double2* S00 = lead + 2 * MM;
    const double2* S01 = lead + 3 * MM;
    auto Uel = [&](int r, int c) {             // z S01 - H01
      const cd s = ldd(S01 + r * M + c), h = ldd(H01 + r * M + c);
      return mk<double>(zx.re * s.re - zx.im * s.im - h.re, zx.re * s.im + zx.im * s.re - h.im);
    };
    auto Lel = [&](int r, int c) {             // z S01^H - H01^H
      const cd s = ldd(S01 + c * M + r), h = ldd(H01 + c * M + r);
      return mk<double>(zx.re * s.re + zx.im * s.im - h.re, zx.im * s.re - zx.re * s.im + h.im);
    };
    auto D0el = [&](int r, int c) {            // z S00 - H00
      const cd s = ldd(S00 + r * M + c), h = ldd(H00 + r * M + c);
      return mk<double>(zx.re * s.re - zx.im * s.im - h.re, zx.re * s.im + zx.im * s.re - h.im);
    };
    (void)Uel;
    (void)Lel;
    (void)D0el;
    __syncthreads();
    // sum over the workgroup, the same value in every thread
    auto bsum = [&](double v) {
      v = wave_sum(v);
      if (lane == 0) sh.rc[w] = v;
      __syncthreads();
      double r = 0.0;
      for (int q = 0; q < NWAVE; ++q) r += sh.rc[q];
      __syncthreads();
      return r;
    };
    // U' into Ui, [D0' | L'] into Yv for shift number q; ||U'||_F^2
    auto build = [&](int q) {
      const cd s = mode_shift(q), sb = cconj(s), sb2 = cmul(sb, sb), s2 = cmul(s, s);
      const double s1 = 1.0 + s.re * s.re + s.im * s.im;
      double n2 = 0.0;
      for (int idx = t; idx < m * m; idx += NT) {
        const int r = idx / m, c = idx - r * m;
        cd u = Uel(r, c), d = D0el(r, c), l = Lel(r, c);
        if (q != 0) {
          const cd u1 = cadd(u, cadd(cmul(sb, d), cmul(sb2, l)));
          const cd d1 = cadd(cscl(cmul(sb, l), 2.0), cadd(cscl(d, s1), cscl(cmul(s, u), 2.0)));
          const cd l1 = cadd(l, cadd(cmul(s, d), cmul(s2, u)));
          u = u1;
          d = d1;
          l = l1;
        }
        sto(Ui + (size_t)r * LD + c, u);
        sto(Yv + (size_t)r * LD + c, d);
        sto(Yv + (size_t)r * LD + m + c, l);
        n2 += u.re * u.re + u.im * u.im;
      }
      return bsum(n2);
    };
    // ||U'||_F^2 ||U'^-1||_F^2, or infinity if the inverse failed
    auto kappa2 = [&](double nu2, bool inv) {
      if (!inv) return (double)INFINITY;
      double n2 = 0.0;
      for (int idx = t; idx < m * m; idx += NT) {
        const int r = idx / m, c = idx - r * m;
        const cd v = ldd(Ui + (size_t)r * LD + m + c);
        n2 += v.re * v.re + v.im * v.im;
      }
      const double k2 = nu2 * bsum(n2);
      return k2 >= 0.0 ? k2 : (double)INFINITY;   // NaN counts as failed
    };
    // ---- 1. the shift, U'^-1, then C = [[-U'^-1 D0', -U'^-1 L'], [I, 0]]
    bool ok = false;
    int qs = 0, qbest = -1;
    double k2best = INFINITY;
    for (int q = 0; q < kModeShifts; ++q) {
      const double nu2 = build(q);
      const bool inv = gj_invert(Ui, m, LD, sh.vec, sh.sd, sh.si);
      const double k2 = kappa2(nu2, inv);
      if (k2 <= kModeKappa * kModeKappa) {
        ok = true;
        qs = q;
        break;
      }
      if (k2 < k2best) {
        k2best = k2;
        qbest = q;
      }
    }
    if (!ok && qbest >= 0) {
      qs = qbest;
      build(qs);
      ok = gj_invert(Ui, m, LD, sh.vec, sh.sd, sh.si);
    }
    if (t == 0) {
      const cd s = mode_shift(qs);
      shift[jl] = make_double2(s.re, s.im);
    }
    if (ok) {
      for (int idx = t; idx < m * n; idx += NT) {
        const int r = idx / n, c = idx - r * n;
        cd s = mk<double>(0.0, 0.0);
        for (int j = 0; j < m; ++j) s = cadd(s, cmul(ldd(Ui + (size_t)r * LD + m + j), ldd(Yv + (size_t)j * LD + c)));
        sto(Cm + (size_t)r * LD + c, mk<double>(-s.re, -s.im));
        sto(Cm + (size_t)(m + r) * LD + c, mk<double>(c == r ? 1.0 : 0.0, 0.0));
      }
      // only rows m..2m-1 of the Schur vectors are ever used (the c part of
      // the eigenvectors), so only they are formed
      for (int idx = t; idx < m * n; idx += NT) {
        const int r = m + idx / n, c = idx - (r - m) * n;
        sto(Qm + (size_t)r * LD + c, mk<double>(r == c ? 1.0 : 0.0, 0.0));
      }
      __syncthreads();
      // ---- 2a. Hessenberg form C <- P C P, Q <- Q P, P = I - g u u^H
      for (int k = 0; k + 2 < n; ++k) {
        if (w == 0) {
          double a2 = 0.0;
          for (int i = k + 1 + lane; i < n; i += 64) {
            const cd x = ldd(Cm + (size_t)i * LD + k);
            a2 += x.re * x.re + x.im * x.im;
            sh.vec[i] = x;
          }
          a2 = wave_sum(a2);
          if (lane == 0) {
            const double al = sqrt(a2);
            const cd x0 = ldd(Cm + (size_t)(k + 1) * LD + k);
            const double ax0 = cabsx(x0);
            const cd ph = ax0 > 0.0 ? mk<double>(x0.re / ax0, x0.im / ax0) : mk<double>(1.0, 0.0);
            sh.vec[k + 1] = cadd(x0, cscl(ph, al));
            sh.sd[0] = al > 0.0 ? 1.0 / (al * (al + ax0)) : 0.0;
            sh.sd[1] = -ph.re * al;
            sh.sd[2] = -ph.im * al;
          }
        }
        __syncthreads();
        const double g = sh.sd[0];
        if (g != 0.0) {
          // from the left, rows k+1..n-1: thread per column j >= k
          for (int j = k + t; j < n; j += NT) {
            cd s = mk<double>(0.0, 0.0);
            for (int i = k + 1; i < n; ++i) s = cadd(s, cmul(cconj(sh.vec[i]), ldd(Cm + (size_t)i * LD + j)));
            s = cscl(s, g);
            if (j == k) {
              sto(Cm + (size_t)(k + 1) * LD + k, mk<double>(sh.sd[1], sh.sd[2]));
              for (int i = k + 2; i < n; ++i) sto(Cm + (size_t)i * LD + k, mk<double>(0.0, 0.0));
            } else {
              for (int i = k + 1; i < n; ++i)
                sto(Cm + (size_t)i * LD + j, cfms(ldd(Cm + (size_t)i * LD + j), sh.vec[i], s));
            }
          }
          __syncthreads();
          // from the right, columns k+1..n-1: thread per row of C (n) and
          // of the used half of Q (m)
          for (int q0 = t; q0 < n + m; q0 += NT) {
            double2* Ri = q0 < n ? Cm + (size_t)q0 * LD : Qm + (size_t)(q0 - n + m) * LD;
            cd s = mk<double>(0.0, 0.0);
            for (int j = k + 1; j < n; ++j) s = cadd(s, cmul(ldd(Ri + j), sh.vec[j]));
            s = cscl(s, g);
            for (int j = k + 1; j < n; ++j) sto(Ri + j, cfms(ldd(Ri + j), s, cconj(sh.vec[j])));
          }
        }
        __syncthreads();
      }
    }
    if (t == 0) jst[jl] = ok ? 0 : -1;
  }
}

// Stage 2 (per job): complex Schur form T = Q^H C Q (T back in the job's C
// slot, upper triangle).  jst[jl] = QR sweeps, or -1.
template <int M>
__global__ __launch_bounds__(NT) void k_modes_qr(Prob P, const double* E, double eta, int sides, double tol, int m, int j0, int nb, double2* ws, int* jst) {
  __shared__ ModeShared sh;
  __shared__ cd Hs[M <= 64 ? hpack(2 * M) : 1];   // packed Hessenberg / Schur form (M <= 64)
  constexpr int LD = 2 * M, MM = M * M;
  constexpr size_t WS = 16 * (size_t)M * M;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  (void)lane;
  (void)w;
  const int n = 2 * m;
  const double eps = 2.220446049250313e-16;
  (void)eps;
  for (int jl = blockIdx.x; jl < nb; jl += gridDim.x) {
    const int job = j0 + jl;
    double2* Cm = ws + (size_t)jl * WS;          // C, then its Schur form T (n x n, stride LD)
    double2* Qm = Cm + 4 * (size_t)MM;           // Schur vectors
    double2* Yv = Qm + 4 * (size_t)MM;           // [D0 | L], then eigenvectors of T, then products
    double2* Ui = Yv + 4 * (size_t)MM;           // Gauss-Jordan work (m x 2m)
    double2* Cv = Ui + 2 * (size_t)MM;           // mode vectors c (m x n)
    (void)Yv;
    (void)Ui;
    (void)Cv;
    const int e = job / sides;
    const int side = sides == 2 ? job - 2 * e : -1;       // -1: both surfaces from the left lead
    const double2* lead = side == 1 ? P.leadR : P.leadL;
    const double V = side == 1 ? P.VR : P.VL;
    const cd zx = mk<double>(E[e] - V, eta);
    const double2* H00 = lead;
    const double2* H01 = lead + MM;
    const double2* S00 = lead + 2 * MM;
    const double2* S01 = lead + 3 * MM;
    auto Uel = [&](int r, int c) {             // z S01 - H01
      const cd s = ldd(S01 + r * M + c), h = ldd(H01 + r * M + c);
      return mk<double>(zx.re * s.re - zx.im * s.im - h.re, zx.re * s.im + zx.im * s.re - h.im);
    };
    auto Lel = [&](int r, int c) {             // z S01^H - H01^H
      const cd s = ldd(S01 + c * M + r), h = ldd(H01 + c * M + r);
      return mk<double>(zx.re * s.re + zx.im * s.im - h.re, zx.im * s.re - zx.re * s.im + h.im);
    };
    auto D0el = [&](int r, int c) {            // z S00 - H00
      const cd s = ldd(S00 + r * M + c), h = ldd(H00 + r * M + c);
      return mk<double>(zx.re * s.re - zx.im * s.im - h.re, zx.re * s.im + zx.im * s.re - h.im);
    };
    (void)Uel;
    (void)Lel;
    (void)D0el;
    __syncthreads();
    if (jst[jl] < 0) continue;          // uniform
    int total = 0;
    bool ok;
    if constexpr (M <= 64) {
      const HLds HL{Hs, n};
      for (int q = t; q < n * n; q += NT) {
        const int i = q / n, j = q - i * n;
        if (j >= i - 1) Hs[HL.at(i, j)] = ldd(Cm + (size_t)i * LD + j);
      }
      __syncthreads();
      ok = schur_qr_wave(HL, n, Qm, LD, sh, &total);
      __syncthreads();
      for (int q = t; q < n * n; q += NT) {
        const int i = q / n, j = q - i * n;
        if (j >= i) sto(Cm + (size_t)i * LD + j, Hs[HL.at(i, j)]);
      }
    } else {
      ok = schur_qr(HGlob{Cm, LD}, n, Qm, LD, sh, &total);
    }
    if (t == 0) jst[jl] = ok ? total : -1;
    __syncthreads();
  }
}

// Stage 3 (per job): eigenvectors, the mode split, self-energies, injection
// and the outputs of both or one surface.
template <int M>
__global__ __launch_bounds__(NT) void k_modes_post(Prob P, const double* E, double eta, int sides, double tol, int m, int j0, int nb, double2* ws, int* jst, const double2* shift,
                                                   double2* sig, double2* wf, double* sgn, int* iters, int* nheavy) {
  __shared__ ModeShared sh;
  constexpr int LD = 2 * M, MM = M * M;
  constexpr size_t WS = 16 * (size_t)M * M;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  (void)lane;
  (void)w;
  const int n = 2 * m;
  const double eps = 2.220446049250313e-16;
  (void)eps;
  for (int jl = blockIdx.x; jl < nb; jl += gridDim.x) {
    const int job = j0 + jl;
    double2* Cm = ws + (size_t)jl * WS;          // C, then its Schur form T (n x n, stride LD)
    double2* Qm = Cm + 4 * (size_t)MM;           // Schur vectors
    double2* Yv = Qm + 4 * (size_t)MM;           // [D0 | L], then eigenvectors of T, then products
    double2* Ui = Yv + 4 * (size_t)MM;           // Gauss-Jordan work (m x 2m)
    double2* Cv = Ui + 2 * (size_t)MM;           // mode vectors c (m x n)
    (void)Yv;
    (void)Ui;
    (void)Cv;
    const int e = job / sides;
    const int side = sides == 2 ? job - 2 * e : -1;       // -1: both surfaces from the left lead
    const double2* lead = side == 1 ? P.leadR : P.leadL;
    const double V = side == 1 ? P.VR : P.VL;
    const cd zx = mk<double>(E[e] - V, eta);
    const double2* H00 = lead;
    const double2* H01 = lead + MM;
    const double2* S00 = lead + 2 * MM;
    const double2* S01 = lead + 3 * MM;
    auto Uel = [&](int r, int c) {             // z S01 - H01
      const cd s = ldd(S01 + r * M + c), h = ldd(H01 + r * M + c);
      return mk<double>(zx.re * s.re - zx.im * s.im - h.re, zx.re * s.im + zx.im * s.re - h.im);
    };
    auto Lel = [&](int r, int c) {             // z S01^H - H01^H
      const cd s = ldd(S01 + c * M + r), h = ldd(H01 + c * M + r);
      return mk<double>(zx.re * s.re + zx.im * s.im - h.re, zx.im * s.re - zx.re * s.im + h.im);
    };
    auto D0el = [&](int r, int c) {            // z S00 - H00
      const cd s = ldd(S00 + r * M + c), h = ldd(H00 + r * M + c);
      return mk<double>(zx.re * s.re - zx.im * s.im - h.re, zx.re * s.im + zx.im * s.re - h.im);
    };
    (void)Uel;
    (void)Lel;
    (void)D0el;
    __syncthreads();
    // ---- 2c. eigenvectors of T (thread per eigenvalue), then c = (Q y) rows m..2m-1
    auto Tel = [&](int i, int j) -> cd { return ldd(Cm + (size_t)i * LD + j); };
    const int total = jst[jl];
    const cd sft = mk<double>(shift[jl].x, shift[jl].y);
    bool ok = total >= 0;
    if (ok) {
      for (int k = t; k < n; k += NT) {
        const cd lk = Tel(k, k);                      // nu_k
        // lambda = (nu + s) / (1 + conj(s) nu) and its inverse (s = 0: nu
        // and 1/nu exactly; lambda = infinity gives lami = 0)
        const cd num = cadd(lk, sft), den = cadd(mk<double>(1.0, 0.0), cmul(cconj(sft), lk));
        sh.lam[k] = cdivx(num, den);
        sh.lami[k] = cdivx(den, num);
        const double smin = fmax(eps * cabs1(lk), 1e-290);
        for (int i = k + 1; i < n; ++i) sto(Yv + (size_t)i * LD + k, mk<double>(0.0, 0.0));
        sto(Yv + (size_t)k * LD + k, mk<double>(1.0, 0.0));
        double big = 1.0;
        for (int i = k - 1; i >= 0; --i) {
          cd s = mk<double>(0.0, 0.0);
          for (int j = i + 1; j <= k; ++j) s = cadd(s, cmul(Tel(i, j), ldd(Yv + (size_t)j * LD + k)));
          cd dd = csub(Tel(i, i), lk);
          if (cabs1(dd) < smin) dd = mk<double>(smin, 0.0);
          const cd y = cdivx(mk<double>(-s.re, -s.im), dd);
          sto(Yv + (size_t)i * LD + k, y);
          big = fmax(big, cabs1(y));
          if (big > 1e150) {                  // rescale the partial vector
            for (int q = i; q <= k; ++q) sto(Yv + (size_t)q * LD + k, cscl(ldd(Yv + (size_t)q * LD + k), 1e-150));
            big *= 1e-150;
          }
        }
      }
      __syncthreads();
      for (int idx = t; idx < m * n; idx += NT) {
        const int r = idx / n, k = idx - r * n;
        cd s = mk<double>(0.0, 0.0);
        for (int j = 0; j <= k; ++j) s = cadd(s, cmul(ldd(Qm + (size_t)(m + r) * LD + j), ldd(Yv + (size_t)j * LD + k)));
        sto(Cv + (size_t)r * LD + k, s);
      }
      __syncthreads();
      // ---- 3. unit mode vectors, fluxes and the split
      for (int k = t; k < n; k += NT) {
        double nn = 0.0;
        for (int r = 0; r < m; ++r) {
          const cd v = ldd(Cv + (size_t)r * LD + k);
          nn += v.re * v.re + v.im * v.im;
        }
        const double sc = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        for (int r = 0; r < m; ++r) sto(Cv + (size_t)r * LD + k, cscl(ldd(Cv + (size_t)r * LD + k), sc));
        cd q = mk<double>(0.0, 0.0);                   // c^H U c
        for (int r = 0; r < m; ++r) {
          cd uc = mk<double>(0.0, 0.0);
          for (int j = 0; j < m; ++j) uc = cadd(uc, cmul(Uel(r, j), ldd(Cv + (size_t)j * LD + k)));
          q = cadd(q, cmul(cconj(ldd(Cv + (size_t)r * LD + k)), uc));
        }
        const cd lk = sh.lam[k];
        const double J = 2.0 * cmul(lk, q).im;
        const double al = cabsx(lk);
        int kind;
        if (eta > 0.0) {
          kind = al < 1.0 ? 1 : 0;
        } else {
          const bool trav = fabs(al - 1.0) <= tol;
          kind = trav ? (J > 0.0 ? 3 : 2) : (al < 1.0 ? 1 : 0);
        }
        sh.J[k] = J;
        sh.kind[k] = (nn > 0.0 && isfinite(nn)) ? kind : -1;
      }
      __syncthreads();
      if (t == 0) {
        int nr = 0, nl = 0, bad = 0;
        for (int k = 0; k < n; ++k) {
          const int kd = sh.kind[k];
          if (kd < 0) { bad = 1; continue; }
          if (kd & 1) { if (nr < m) sh.ridx[nr] = k; ++nr; }
          else { if (nl < m) sh.lidx[nl] = k; ++nl; }
        }
        sh.si[2] = (bad || nr != m || nl != m) ? 0 : 1;
      }
      __syncthreads();
      ok = sh.si[2] != 0;
    }
    // ---- 4./5. self-energies and injection of each requested surface
    for (int s = 0; s < 2; ++s) {
      if (side >= 0 && s != side) continue;
      const int slot = 2 * e + s;
      double2* So = sig + (size_t)slot * MM;
      double2* Wo = wf + (size_t)slot * MM;
      bool sok = ok;
      const int* idx = s == 0 ? sh.lidx : sh.ridx;     // Sigma_L: left-going, Sigma_R: right-going
      if (sok) {
        for (int q = t; q < m * m; q += NT) {
          const int r = q / m, c = q - r * m;
          sto(Ui + (size_t)r * LD + c, ldd(Cv + (size_t)r * LD + idx[c]));
        }
        __syncthreads();
        sok = gj_invert(Ui, m, LD, sh.vec, sh.sd, sh.si);
      }
      if (sok) {
        // F = B Lambda^(+-1) B^-1 into Yv, then Sigma = -{L, U} F
        for (int q = t; q < m * m; q += NT) {
          const int r = q / m, c = q - r * m;
          cd acc = mk<double>(0.0, 0.0);
          for (int j = 0; j < m; ++j) {
            const cd f = s == 0 ? sh.lami[idx[j]] : sh.lam[idx[j]];
            acc = cadd(acc, cmul(cmul(ldd(Cv + (size_t)r * LD + idx[j]), f), ldd(Ui + (size_t)j * LD + m + c)));
          }
          sto(Yv + (size_t)r * LD + c, acc);
        }
        __syncthreads();
        for (int q = t; q < MM; q += NT) {
          const int r = q / M, c = q - r * M;
          cd acc = mk<double>(0.0, 0.0);
          if (r < m && c < m)
            for (int j = 0; j < m; ++j)
              acc = cadd(acc, cmul(s == 0 ? Lel(r, j) : Uel(r, j), ldd(Yv + (size_t)j * LD + c)));
          sto(So + q, mk<double>(-acc.re, -acc.im));
        }
        __syncthreads();
        // column g of W: the g-th incoming travelling mode in index order
        // (right-going of the source's lead, left-going of the drain's)
        for (int q = t; q < MM; q += NT) {
          const int r = q / M, g = q - r * M;
          int k = -1, cnt = 0;
          for (int kk = 0; kk < n && k < 0; ++kk) {
            const int kd = sh.kind[kk];
            if ((s == 0 && kd == 3) || (s == 1 && kd == 2)) {
              if (cnt == g) k = kk;
              ++cnt;
            }
          }
          cd v = mk<double>(0.0, 0.0);
          if (r < m && k >= 0) {
            const cd f = s == 0 ? mk<double>(-sh.lami[k].re, -sh.lami[k].im) : mk<double>(-sh.lam[k].re, -sh.lam[k].im);
            cd acc = mk<double>(0.0, 0.0);
            for (int j = 0; j < m; ++j) {
              const cd cj = ldd(Cv + (size_t)j * LD + k);
              const cd op = cadd(cmul(f, s == 0 ? Lel(r, j) : Uel(r, j)), mk<double>(-ldd(So + r * M + j).re,
                                                                                   -ldd(So + r * M + j).im));
              acc = cadd(acc, cmul(op, cj));
            }
            v = cscl(acc, 1.0 / sqrt(fabs(sh.J[k])));
          }
          sto(Wo + q, v);
        }
        for (int c = t; c < M; c += NT) {
          int cnt = 0;
          for (int kk = 0; kk < n; ++kk) {
            const int kd = sh.kind[kk];
            cnt += (s == 0 && kd == 3) || (s == 1 && kd == 2);
          }
          sgn[(size_t)slot * M + c] = c < cnt ? 1.0 : 0.0;
          if (c == 0) nheavy[slot] = cnt;
        }
      } else {
        for (int q = t; q < MM; q += NT) {
          So[q] = make_double2(0.0, 0.0);
          Wo[q] = make_double2(0.0, 0.0);
        }
        for (int c = t; c < M; c += NT) sgn[(size_t)slot * M + c] = 0.0;
        if (t == 0) nheavy[slot] = 0;
      }
      if (t == 0) iters[slot] = sok ? (total > 0 ? total : 1) : -1;
      __syncthreads();
    }
  }
}

template <int M>
hipError_t launch_modes(const Prob& P, const double* E, int nE, double eta, int sides, double tol, int m, int num_cu,
                        double2* scratch, int* jst, double2* shift, double2* sig, double2* wf, double* sgn, int* iters,
                        int* nheavy, hipStream_t st) {
  int o1 = 0, o2 = 0, o3 = 0;
  hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&o1, k_modes_hess<M>, NT, 0);
  if (err == hipSuccess) err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&o2, k_modes_qr<M>, NT, 0);
  if (err == hipSuccess) err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&o3, k_modes_post<M>, NT, 0);
  if (err != hipSuccess) return err;
  const int njobs = nE * sides;
  const int jb = modes_batch_jobs(M, njobs);
  for (int j0 = 0; j0 < njobs; j0 += jb) {
    const int nb = njobs - j0 < jb ? njobs - j0 : jb;
    auto grid = [&](int occ) { const int g = num_cu * (occ > 0 ? occ : 1); return g < nb ? g : nb; };
    // at most two Hessenberg jobs per CU: their matrices (C and Q, 8 M^2
    // complex doubles each) then stay in the last-level cache, which the
    // reduction re-reads once per column
    hipLaunchKernelGGL(k_modes_hess<M>, dim3(grid(o1 < 2 ? o1 : 2)), dim3(NT), 0, st, P, E, eta, sides, tol, m, j0, nb, scratch,
                       jst, shift);
    hipLaunchKernelGGL(k_modes_qr<M>, dim3(grid(o2)), dim3(NT), 0, st, P, E, eta, sides, tol, m, j0, nb, scratch,
                       jst);
    hipLaunchKernelGGL(k_modes_post<M>, dim3(grid(o3)), dim3(NT), 0, st, P, E, eta, sides, tol, m, j0, nb, scratch,
                       jst, shift, sig, wf, sgn, iters, nheavy);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

hipError_t run_modes(int M, const Prob& P, const double* E, int nE, double eta, int sides, double tol, int m,
                     int num_cu, double2* scratch, int* jst, double2* shift, double2* sig, double2* wf, double* sgn,
                     int* iters, int* nheavy, hipStream_t st) {
#define QTX_MODES(MM) \
  return launch_modes<MM>(P, E, nE, eta, sides, tol, m, num_cu, scratch, jst, shift, sig, wf, sgn, iters, nheavy, st)
  switch (M) {
    case 16: QTX_MODES(16);
    case 32: QTX_MODES(32);
    case 48: QTX_MODES(48);
    case 64: QTX_MODES(64);
    case 96: QTX_MODES(96);
    case 128: QTX_MODES(128);
    default: return hipErrorInvalidValue;
  }
#undef QTX_MODES
}

}  // namespace qtx
