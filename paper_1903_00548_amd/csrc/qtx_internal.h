// Shared declarations between the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include "qtx.h"

namespace qtx {

// One transport problem as the kernels see it.  Blocks are padded to M
// (a multiple of 16) and stored row-major as interleaved complex doubles.
// Lead storage: H00, H01, S00, S01 (4 * M * M).  Device blocks: Hd (N M^2),
// Hu ((N-1) M^2), Sd (N M^2), Su ((N-1) M^2), or null when every slab copies
// the left lead.
struct Prob {
  int N, M;
  const double2* leadL;
  const double2* leadR;
  double VL, VR;
  const double2* dHd;
  const double2* dHu;
  const double2* dSd;
  const double2* dSu;
  const double* V;
  int pot_mode;

  __host__ __device__ const double2* Hd(int i) const { return dHd ? dHd + (size_t)i * M * M : leadL; }
  __host__ __device__ const double2* Hu(int i) const { return dHu ? dHu + (size_t)i * M * M : leadL + (size_t)M * M; }
  __host__ __device__ const double2* Sd(int i) const { return dSd ? dSd + (size_t)i * M * M : leadL + 2 * (size_t)M * M; }
  __host__ __device__ const double2* Su(int i) const { return dSu ? dSu + (size_t)i * M * M : leadL + 3 * (size_t)M * M; }

  // potential weight on the on-site overlap block of slab i
  __device__ double vd(int i) const {
    if (!V) return 0.0;
    if (pot_mode == QTX_POT_DIAG) return V[i];
    const double vm = i > 0 ? V[i - 1] : VL;
    const double vp = i < N - 1 ? V[i + 1] : VR;
    return 0.75 * V[i] + 0.125 * (vm + vp);
  }
  // potential weight on the coupling overlap block i -> i+1
  __device__ double vu(int i) const {
    if (!V || pot_mode == QTX_POT_DIAG) return 0.0;
    return 0.5 * (V[i] + V[i + 1]);
  }
};

hipError_t run_decimate(int M, const Prob& P, const double* E, int nE, double eta, int sides, double tol,
                        int maxit, double2* scratch, int grid, double2* sig, double2* wf, double* sgn,
                        int* iters, hipStream_t st);

hipError_t run_sweep(int M, bool fp32, const Prob& P, const double* E, int nE, double eta, const double2* sig,
                     const double2* wf, const double* sgn, const int* iters, void* ws, size_t ws_stride,
                     double* part, int grid, double* T, double* ldos, qtx_info* info, hipStream_t st);

}  // namespace qtx
