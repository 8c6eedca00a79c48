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

  __host__ __device__ __forceinline__ const double2* Hd(int i) const { return dHd ? dHd + (size_t)i * M * M : leadL; }
  __host__ __device__ __forceinline__ const double2* Hu(int i) const { return dHu ? dHu + (size_t)i * M * M : leadL + (size_t)M * M; }
  __host__ __device__ __forceinline__ const double2* Sd(int i) const { return dSd ? dSd + (size_t)i * M * M : leadL + 2 * (size_t)M * M; }
  __host__ __device__ __forceinline__ const double2* Su(int i) const { return dSu ? dSu + (size_t)i * M * M : leadL + 3 * (size_t)M * M; }

  // potential weight on the on-site overlap block of slab i
  __device__ __forceinline__ double vd(int i) const {
    if (!V) return 0.0;
    if (pot_mode == QTX_POT_DIAG) return V[i];
    const double vm = i > 0 ? V[i - 1] : VL;
    const double vp = i < N - 1 ? V[i + 1] : VR;
    return 0.75 * V[i] + 0.125 * (vm + vp);
  }
  // potential weight on the coupling overlap block i -> i+1
  __device__ __forceinline__ double vu(int i) const {
    if (!V || pot_mode == QTX_POT_DIAG) return 0.0;
    return 0.5 * (V[i] + V[i + 1]);
  }
};

// Several problems in one launch: the energies of all problems of one
// padded block size form a flat list of items (item e: problem
// item_prob[e], energy E[e]); outputs T[e], info[e], and the densities of
// item e at ldos + item_ldos[e] (2 N of its problem).  The decimation runs
// over njobs jobs (item job_item[j], contact job_side[j]: 0 left, 1 right,
// -1 both when the problem's leads are the same).  probs == nullptr: one
// problem, passed by value.
// Self-energy cache (job_E non-null): decimation job j fills slot
// job_item[j] of the cache with both surface self-energies of the lead
// job_lead[j] at the shifted energy job_E[j] (E - V already applied).
struct BatchDesc {
  const Prob* probs;
  const int* item_prob;
  const size_t* item_ldos;
  const int* job_item;
  const int* job_side;
  int njobs;
  const double* job_E;
  const double2* const* job_lead;
};

// Arguments of one sweep launch.  Energy e uses sig/wf/sgn/iters/nheavy
// at index e of the decimation outputs and writes T[e], ldos[e] and
// info[e].  Workgroup b owns bytes [b ws_bytes, (b+1) ws_bytes) of ws and
// its share of part.
struct SweepArgs {
  const double* E;
  int nE;
  double eta;
  const double2* sig;      // Sigma_L, Sigma_R per energy (2 M^2)
  const double2* wf;       // W_L, W_R per energy (2 M^2)
  const double* sgn;       // signs of the broadening factors (2 M)
  const int* iters;        // doublings per side (2), negative if capped
  const int* nheavy;       // refined columns per side (2), mixed sweep only
  const int* sig_slot;     // non-null: item e takes the left contact from slot
                           // sig_slot[2e] and the right one from sig_slot[2e+1]
                           // of sig/wf/sgn/iters/nheavy (else slot e for both)
  char* ws;
  size_t ws_bytes;
  double* part;            // per workgroup NWAVE * 2 * nmax doubles (twice that, mixed)
  int nmax;                // largest slab count of the launch
  double* T;
  double* ldos;            // may be null
  qtx_info* info;          // may be null
  const int* elist;        // non-null: solve energies elist[0 .. *ecount) only
  const int* ecount;
  int* redo;               // mixed: 1 where the refinement did not converge
  double rtol;             // mixed: stop when ||r|| <= rtol ||b||
  int maxstep;             // mixed: at most this many corrections
  // density-matrix sweep only: weights dmwL[e] (left-injected columns) and
  // dmwR[e] (right-injected) of energy e; workgroup b accumulates rho_ii
  // and rho_{i,i+1} (blocks 2i and 2i+1, M x M each) at rho + b rho_stride,
  // starting from zero at its first energy when rho_first is set
  const double* dmwL;
  const double* dmwR;
  double2* rho;
  size_t rho_stride;
  int rho_first;
};

// Per-workgroup sweep workspace.  FP64 sweep: [X_i | z_i] for N slabs plus
// the back-substitution buffer, (N + 1) M x 2M complex doubles.  Mixed
// sweep, in this order: the same in complex floats; the N inverses of the
// Schur complements (M x M floats); the correction columns (N M x 2M
// floats); one slab of right-hand sides (M x 2M floats); the refined
// solution (N M x 2M doubles).
// The density-matrix sweep (FP64) keeps a second back-substitution buffer.
// Blocks above 64 (96, 128) keep two more M x (M + 1) complex matrices of
// the sweep precision at the end: the working matrix and the staged
// coupling block, and in the mixed sweep before them one M x (M + 1) FP64
// block staged for the refinement's residual products.
inline size_t sweep_ws_bytes(int N, int M, bool mixed, bool dm = false) {
  const size_t MM = (size_t)M * M;
  const size_t big = M > 64 ? 2 * (size_t)M * (M + 1) * (mixed ? sizeof(float2) : sizeof(double2)) +
                                  (mixed ? (size_t)M * (M + 1) * sizeof(double2) : 0)
                            : 0;
  if (!mixed) return (size_t)(N + (dm ? 2 : 1)) * 2 * MM * sizeof(double2) + big;
  return ((size_t)(N + 1) * 2 * MM + (size_t)N * MM + (size_t)N * 2 * MM + 2 * MM) * sizeof(float2) +
         (size_t)N * 2 * MM * sizeof(double2) + big;
}

// Byte offsets within one workgroup's sweep workspace (ws_bytes long) of
// the regions a sweep over an item of N slabs uses, and their sizes; the
// kernels take their pointers from here, and qtx_check_layouts tests the
// layouts on the host.  FP64 sweep: [X_i | z_i] per slab, then the
// back-substitution buffer (two for the density-matrix sweep).  Mixed
// sweep: the same in complex floats, then the inverses of the Schur
// complements, the correction columns, one slab of right-hand sides and
// the refined FP64 solution.  Blocks above 64: the working matrix and the
// staged coupling block at the end, and in the mixed sweep the FP64 block
// of the refinement's residual products just below them.
struct SweepLayout {
  size_t xz, psi, di, zc, yb, p64, mat, lst, stg;
  size_t xz_n, psi_n, di_n, zc_n, yb_n, p64_n, mat_n, lst_n, stg_n;
};
__host__ __device__ inline SweepLayout sweep_layout(int N, int M, bool mixed, bool dm, size_t ws_bytes) {
  SweepLayout L{};
  const size_t MM = (size_t)M * M, LD = 2 * (size_t)M, S = (size_t)M + 1;
  const size_t el = mixed ? 8 : 16;                      // complex float / complex double
  L.xz = 0;
  L.xz_n = (size_t)N * M * LD * el;
  L.psi = L.xz + L.xz_n;
  L.psi_n = (dm ? 2 : 1) * (size_t)M * LD * el;
  if (mixed) {
    L.di = L.psi + L.psi_n;
    L.di_n = (size_t)N * MM * 8;
    L.zc = L.di + L.di_n;
    L.zc_n = (size_t)N * M * LD * 8;
    L.yb = L.zc + L.zc_n;
    L.yb_n = (size_t)M * LD * 8;
    L.p64 = L.yb + L.yb_n;
    L.p64_n = (size_t)N * M * LD * 16;
  }
  if (M > 64) {
    L.mat_n = L.lst_n = S * (size_t)M * el;
    L.mat = ws_bytes - 2 * L.mat_n;
    L.lst = L.mat + L.mat_n;
    if (mixed) {
      L.stg_n = S * (size_t)M * 16;
      L.stg = L.mat - L.stg_n;
    }
  }
  return L;
}

// Per-workgroup decimation workspace (complex doubles): e, the right surface
// block, [a | b], g [a | b], the residual, and for M > 64 the working matrix
// M x (M + 1).
__host__ __device__ constexpr size_t dec_ws_elems(int M) {
  return 8 * (size_t)M * M + (M > 64 ? (size_t)M * (M + 1) : 0);
}

// Padded block size for a physical block size m (1 <= m <= 128).
inline int padded_block(int m) { return m <= 64 ? ((m + 15) / 16) * 16 : (m <= 96 ? 96 : 128); }

// Decimation settings: stop when the couplings fall below tol |D0| (at most
// maxit doublings); refine g [a | b] when ||e||_F ||e^-1||_F > rcond (every
// doubling for rcond = 0); heavy_tol sets the count of leading broadening
// columns reported per contact; a self-energy whose fixed-point residual
// exceeds newton_tol times its largest element takes one Newton step
// (always for newton_tol = 0, never for newton_tol < 0).
struct DecOpts {
  double tol;
  double rcond;
  int maxit;
  double heavy_tol;
  double newton_tol;
};

hipError_t run_decimate(int M, const Prob& P, const BatchDesc& b, const double* E, int nE, double eta, int sides,
                        const DecOpts& o, double2* scratch, int grid, double2* sig, double2* wf, double* sgn,
                        int* iters, int* nheavy, hipStream_t st);

// Tile shapes of the sweeps (the autotuner's choices): pw, the columns of
// a Gauss-Jordan panel (16 or 32, dividing M; by default 16 up to M = 64,
// 32 above); tpp, the column tiles a wave carries at once through the mixed
// refinement (1 or 2 at M = 48 and 64, by default 2; 2 below 48 and 1 above
// 64 are the only values).
constexpr int sweep_default_pw(int M) { return M > 64 ? 32 : 16; }
constexpr int sweep_default_tpp(int M) { return M <= 64 ? 2 : 1; }
bool sweep_variant_ok(int M, bool mixed, int pw, int tpp);

// mixed = false: FP64 sweep (with a.elist: re-solve of the listed energies).
// mixed = true: FP32 sweep plus refinement of the heavy columns.  pw, tpp:
// the tile shapes above (hipErrorInvalidValue if not a built variant).
hipError_t run_sweep(int M, bool mixed, int pw, int tpp, const Prob& P, const SweepArgs& a, const BatchDesc& b,
                     int grid, hipStream_t st);

// FP64 sweep that also accumulates the density-matrix blocks (a.dmw,
// a.rho, a.rho_stride, a.rho_first; workspace sweep_ws_bytes(N, M, false,
// true)).  One problem, no energy list.
hipError_t run_sweep_dm(int M, const Prob& P, const SweepArgs& a, int grid, hipStream_t st);

// out_d[i] (m x m, i < N) and out_o[i] (i < N - 1) = the sum over the nwg
// workgroup accumulators (stride elements apart) of blocks 2i and 2i+1,
// in workgroup order.
hipError_t run_dm_reduce(const double2* rho, int nwg, size_t stride, int N, int M, int m, double2* out_d,
                         double2* out_o, hipStream_t st);

// Self-energies, injection factors and signs from the complex band
// structure of the leads (the decimation's outputs, same layout) for nE
// energies; sides = 1 when both leads are the same.  m: physical block
// size; tol: |lambda| tolerance of travelling modes at eta = 0.  The jobs
// (energy, lead) run in batches of modes_batch_jobs(M, nE * sides), each
// through three kernels (Hessenberg form, Schur form, modes and outputs);
// scratch: that many times modes_ws_elems(M) complex doubles, jst: that
// many ints, shift: that many complex doubles (the eigenvalue shift each job
// took).  iters: QR sweeps per surface, -1 on failure.
hipError_t run_modes(int M, const Prob& P, const double* E, int nE, double eta, int sides, double tol, int m,
                     int num_cu, double2* scratch, int* jst, double2* shift, double2* sig, double2* wf, double* sgn,
                     int* iters, int* nheavy, hipStream_t st);
inline size_t modes_ws_elems(int M) { return 16 * (size_t)M * M; }
inline int modes_batch_jobs(int M, int njobs) {
  const int jb = M <= 64 ? 2048 : 512;
  return njobs < jb ? njobs : jb;
}

// Fixed device scratch of the no-allocation solve: kNoAllocScratchBytes per
// GPU (a file-scope device array), its device address for `device` (which
// must be the current device) in *ptr.  The address is looked up once per
// device and kept.
constexpr size_t kNoAllocScratchBytes = (size_t)512 << 20;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(int device, char** ptr);

// Band energies of one lead (padded blocks, physical size m) at nk Bloch
// phases: E[q * m + n] = E_n(k_q) + V.  work: grid * 2 M (M + 1) complex
// doubles when M > 64 (else unused).
hipError_t run_bands(int M, const double2* lead, int m, double V, const double* k, int nk, double2* work, int grid,
                     double* E, hipStream_t st);

// Workgroups of the sweep (FP64 or mixed, tile shapes pw and tpp), of the
// decimation and (dm_wgs non-null) of the density-matrix sweep that one CU
// can hold at block size M, from the kernels' register and LDS use.
hipError_t max_resident(int M, bool mixed, int pw, int tpp, int* sweep_wgs, int* dec_wgs, int* dm_wgs = nullptr);

// elist[0 .. *ecount) = the energies e < nE with redo[e] != 0 (one wave).
hipError_t run_compact(const int* redo, int nE, int* elist, int* ecount, hipStream_t st);

}  // namespace qtx
