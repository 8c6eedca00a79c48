// Host runtime behind the C ABI declared in include/qtx.h: context state,
// validation, device copies of the leads / device blocks / potential,
// workspace management and the launch sequence of one solve:
//   decimation (lead self-energies + broadening factors, FP64)
//   -> block sweeps with fused transmission and density reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <unordered_map>
#include <string>
#include <vector>

#include "qtx.h"
#include "qtx_internal.h"

static_assert(QTX_NOALLOC_SCRATCH_BYTES == qtx::kNoAllocScratchBytes, "scratch size in qtx.h and the library agree");

namespace {

// Device buffer that grows on demand and is freed with its owner (the
// context is destroyed with its device current); not copyable.
struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  hipError_t ensure(size_t bytes) {
    if (bytes <= n) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipSuccess) n = bytes;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};


}  // namespace

struct qtx_ctx {
  int device = 0;
  int num_cu = 256;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  qtx_ctx* parent = nullptr;

  int m = 0, M = 0;
  bool lead_set[2] = {false, false};
  double Vlead[2] = {0.0, 0.0};
  std::vector<std::complex<double>> hlead[2];  // unpadded H00, H01, S00, S01
  DevBuf dlead[2];                             // padded 4 M^2

  int N = 0;
  bool dev_set = false, uniform = true;
  DevBuf ddev;                                 // padded Hd, Hu, Sd, Su
  bool pot_set = false;
  int pot_mode = QTX_POT_DIAG;
  DevBuf dV;

  // workspaces
  DevBuf wE, wT, wldos, winfo;
  DevBuf sig, wf, sgn, iters, nheavy, dscr, sws, part;
  DevBuf redo, elist, ecount;                  // mixed: energies re-solved in FP64
  DevBuf dmw, rho, dmout;                      // density-matrix blocks: weights, accumulators, sums
  double dm_bytes = 64.0 * (1ull << 30);       // cap on the per-workgroup accumulators
  double sweep_bytes = 160.0 * (1ull << 30);   // cap on the resident workgroups' sweep workspaces
  double sweep_eff = -1.0;                      // lower cap after the device ran out of memory (< 0: none)
  int se_method = 0;                           // 0 decimation, 1 complex band structure (mode space)
  double mode_tol = 1e-8;                      // |lambda| tolerance of travelling modes
  DevBuf mscr, mjst;                           // complex-band-structure workspace, per-job status

  uint64_t lead_hash[2] = {0, 0};

  // self-energy cache of batched solves, per padded block size: slot k
  // holds both surface self-energies, broadening factors, signs, doublings
  // and refined-column counts of one (lead, shifted energy)
  struct SigCache {
    int M = 0, cap = 0;
    DevBuf sig, wf, sgn, iters, nheavy;
    std::unordered_map<unsigned long long, int> index;   // key hash -> slot
    std::vector<std::pair<uint64_t, uint64_t>> key;       // per slot
    std::vector<long long> tick;                          // last call that used the slot, -1 free
    int hand = 0;                                         // next slot the replacement scan looks at
  };
  std::map<int, SigCache> sigcache;
  double sigcache_bytes = 16.0 * (1ull << 30);
  long long cache_hits = 0, cache_misses = 0, cache_calls = 0;
  std::vector<double> cache_params;                      // eta and decimation settings of the cached data
  DevBuf bslot, bjobE, bjobLead;

  // batched solves: flattened items of all problems, and the captured
  // launch sequence of the last batch shape
  DevBuf bprobs, bitem_prob, bitem_ldos, bjob_item, bjob_side, bE, bT, bldos, binfo;
  std::vector<long long> batch_sig;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool use_graph = true;

  // kernel timing: event pairs around decimation / sweep launches
  bool timing = false;
  std::vector<hipEvent_t> ev_dec, ev_sw;   // start/stop pairs
  size_t n_dec = 0, n_sw = 0;

  // tunables
  double dec_tol = 1e-14;
  double dec_rcond = 1e4;         // refine g [a | b] when ||e||_F ||e^-1||_F exceeds this
  int dec_maxit = 60;
  int chunk = 4096;
  int wg_per_cu = 2;
  int opt_pw = 0;                 // Gauss-Jordan panel width (0: default per block size)
  int opt_tpp = 0;                // mixed refinement tiles per wave (0: default per block size)
  double refine_tol = 3e-11;      // stop when ||r|| <= refine_tol ||b||
  int refine_max = 3;             // corrections per energy before the FP64 fallback
  double heavy_tol = 0.0;         // refine columns with pivot >= heavy_tol * largest (0: all)
  double newton_tol = 3e-11;      // Newton step on a self-energy whose fixed-point residual exceeds this
  std::map<int, qtx_tune> tuned[2];  // autotuned launch shape by block size (FP64, mixed)
};

namespace {

qtx_status fail(qtx_ctx* c, qtx_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

hipError_t record(qtx_ctx* c, std::vector<hipEvent_t>& v, size_t& n) {
  if (!c->timing) return hipSuccess;
  if (n >= v.size()) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    v.push_back(e);
  }
  return hipEventRecord(v[n++], c->stream);
}

qtx_status hipfail(qtx_ctx* c, hipError_t e, const char* what) {
  return fail(c, e == hipErrorOutOfMemory ? QTX_ENOMEM : QTX_EDEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

#define QTX_HIP(ctx, call)                          \
  do {                                              \
    hipError_t _e = (call);                         \
    if (_e != hipSuccess) return hipfail(ctx, _e, #call); \
  } while (0)

typedef std::complex<double> cd;

bool hermitian(const qtx_c128* A, int m, double rel) {
  double scale = 0.0;
  for (int i = 0; i < m * m; ++i) scale = std::max(scale, std::abs(cd(A[i].re, A[i].im)));
  const double tol = rel * std::max(scale, 1e-300);
  for (int r = 0; r < m; ++r)
    for (int c = 0; c <= r; ++c) {
      cd a(A[r * m + c].re, A[r * m + c].im), b(A[c * m + r].re, A[c * m + r].im);
      if (std::abs(a - std::conj(b)) > tol) return false;
    }
  return true;
}

// Pad an m x m block to M x M.  Padded basis functions get an on-site
// block with H = -1, S = 0 (so zS - H = +1 on the padding) and no coupling:
// they decouple from the physical ones, carry no broadening and add
// nothing to transmission or densities.
void pad_block(const qtx_c128* src, int m, int M, bool onsite_H, std::vector<double2>& dst, size_t off) {
  for (int r = 0; r < M; ++r)
    for (int c = 0; c < M; ++c) {
      double2 v = make_double2(0.0, 0.0);
      if (r < m && c < m) v = make_double2(src[r * m + c].re, src[r * m + c].im);
      else if (onsite_H && r == c) v = make_double2(-1.0, 0.0);
      dst[off + (size_t)r * M + c] = v;
    }
}

bool leads_identical(const qtx_ctx* c) {
  if (c->Vlead[0] != c->Vlead[1]) return false;
  return c->hlead[0] == c->hlead[1];
}

qtx_status check_ready(qtx_ctx* c) {
  if (!c->lead_set[0] || !c->lead_set[1]) return fail(c, QTX_ESTATE, "both leads must be set before solving");
  if (!c->dev_set) return fail(c, QTX_ESTATE, "device must be set before solving");
  return QTX_OK;
}

// Resident workgroups per CU for block size M: the autotuned value if there
// is one.  Otherwise blocks up to 64 take the configured count (two by
// default); larger blocks take two in FP64 and one in the mixed path, whose
// workspace (0.3-0.5 GB per workgroup at N = 400) would otherwise crowd the
// self-energy cache and the batch buffers out of device memory.
int wgs_per_cu(const qtx_ctx* c, int M, bool mixed) {
  auto it = c->tuned[mixed].find(M);
  if (it != c->tuned[mixed].end()) return it->second.workgroups_per_cu;
  if (M > 64) return mixed ? 1 : 2;
  return c->wg_per_cu;
}

// Decimation workgroups per CU: the decimation kernel is compiled for two
// per CU at every block size, so above 64 it keeps two whatever the sweep
// runs (the mixed sweeps there run one); at 64 and below it follows the
// sweep's count, which the autotuner times together with it.
int dec_wgs_per_cu(const qtx_ctx* c, int M, bool mixed) {
  return M > 64 ? 2 : wgs_per_cu(c, M, mixed);
}

// Launch shape of the sweeps at block size M: the autotuned one, else the
// default workgroups per CU with the tile shapes of the options panel_width
// and refine_tiles where the block size allows them, else the defaults.
qtx_tune tune_of(const qtx_ctx* c, int M, bool mixed) {
  auto it = c->tuned[mixed].find(M);
  if (it != c->tuned[mixed].end()) return it->second;
  qtx_tune t{wgs_per_cu(c, M, mixed), qtx::sweep_default_pw(M), qtx::sweep_default_tpp(M)};
  if (c->opt_pw && qtx::sweep_variant_ok(M, mixed, c->opt_pw, t.refine_tiles)) t.panel_width = c->opt_pw;
  if (c->opt_tpp && qtx::sweep_variant_ok(M, mixed, t.panel_width, c->opt_tpp)) t.refine_tiles = c->opt_tpp;
  return t;
}

hipError_t sweep_launch(const qtx_ctx* c, int M, bool mixed, const qtx::Prob& P, const qtx::SweepArgs& a,
                        const qtx::BatchDesc& b, int grid) {
  const qtx_tune t = tune_of(c, M, mixed);
  return qtx::run_sweep(M, mixed, t.panel_width, t.refine_tiles, P, a, b, grid, c->stream);
}

// Resident workgroups of a sweep launch over `items` energies of block size
// M: the occupancy limit, lowered until their workspaces of wsb bytes each
// fit in sweep_workspace_bytes; 0 if not even one fits.  Every energy is
// solved by one workgroup, so the grid does not change the results.
int sweep_grid(const qtx_ctx* c, int items, int M, bool mixed, size_t wsb) {
  const double budget = c->sweep_eff >= 0.0 ? std::min(c->sweep_eff, c->sweep_bytes) : c->sweep_bytes;
  const int fit = (int)std::min<double>(1 << 20, std::floor(budget / (double)wsb));
  if (fit < 1) return 0;
  return std::max(1, std::min({items, c->num_cu * wgs_per_cu(c, M, mixed), fit}));
}

// Allocates the sweep workspace (bytes).  When the device is out of memory
// (other buffers of the call, the self-energy cache or other contexts hold
// it), the context's budget drops to half of what was asked and *retry is
// set: the caller recomputes its grids, each at most half as large, and
// tries again.  The lowered budget stays until sweep_workspace_bytes is set.
hipError_t alloc_sweep_ws(qtx_ctx* c, size_t bytes, bool* retry) {
  *retry = false;
  const hipError_t e = c->sws.ensure(bytes);
  if (e != hipErrorOutOfMemory) return e;
  (void)hipGetLastError();
  c->sweep_eff = 0.5 * (double)bytes;
  *retry = true;
  return hipSuccess;
}

qtx::DecOpts dec_opts(const qtx_ctx* c) {
  return qtx::DecOpts{c->dec_tol, c->dec_rcond, c->dec_maxit, c->heavy_tol, c->newton_tol};
}

qtx::Prob make_prob(const qtx_ctx* c) {
  qtx::Prob P;
  P.N = c->N;
  P.M = c->M;
  P.leadL = c->dlead[0].as<double2>();
  P.leadR = c->dlead[1].as<double2>();
  P.VL = c->Vlead[0];
  P.VR = c->Vlead[1];
  const size_t MM = (size_t)c->M * c->M;
  if (c->uniform) {
    P.dHd = P.dHu = P.dSd = P.dSu = nullptr;
  } else {
    const double2* b = c->ddev.as<double2>();
    P.dHd = b;
    P.dHu = b + c->N * MM;
    P.dSd = b + (2 * (size_t)c->N - 1) * MM;
    P.dSu = b + (3 * (size_t)c->N - 1) * MM;
  }
  P.V = c->pot_set ? c->dV.as<double>() : nullptr;
  P.pot_mode = c->pot_mode;
  return P;
}

// The complex-band-structure self-energies are defined at eta = 0 and feed
// the FP64 sweep only.
qtx_status check_method(qtx_ctx* c, double eta, bool mixed) {
  if (c->se_method != 1) return QTX_OK;
  if (eta != 0.0) return fail(c, QTX_EINVAL, "self_energy_method 1 (complex band structure) solves at eta = 0");
  if (mixed) return fail(c, QTX_EINVAL, "self_energy_method 1 runs with QTX_FP64 only");
  return QTX_OK;
}

// Device buffers of one launch chunk of a solve: the decimation outputs per
// energy, the decimation and sweep workspaces of the resident workgroups,
// and for the mixed path the re-solve list.  Filled from the context's
// growable buffers, or carved from the fixed no-allocation scratch.
struct SolveBufs {
  double2* sig = nullptr;
  double2* wf = nullptr;
  double* sgn = nullptr;
  int* iters = nullptr;
  int* nheavy = nullptr;
  double2* dscr = nullptr;      // decimation workspace, gdec workgroups
  int gdec = 0;
  char* sws = nullptr;          // sweep workspace, grid workgroups of wsb bytes
  size_t wsb = 0;
  int grid = 0;
  double* part = nullptr;
  int* redo = nullptr;          // mixed only
  int* elist = nullptr;
  int* ecount = nullptr;
};

// Decimation workgroups for nE energies (sides lead iterations each).
int dec_grid(const qtx_ctx* c, int nE, int sides, bool mixed) {
  return std::max(1, std::min(nE * sides, c->num_cu * dec_wgs_per_cu(c, c->M, mixed)));
}

// lead self-energies, injection factors and signs for energies E_dev[0..nE)
// into b.sig / wf / sgn / iters / nheavy: by decimation, or from the
// complex band structure of the leads (option self_energy_method; its
// workspace is the context's own)
qtx_status stage_decimate(qtx_ctx* c, const double* E_dev, int nE, double eta, bool mixed, const SolveBufs& b) {
  const int M = c->M;
  const int sides = leads_identical(c) ? 1 : 2;
  if (c->se_method == 1) {
    qtx_status s = check_method(c, eta, mixed);
    if (s != QTX_OK) return s;
    const int jb = qtx::modes_batch_jobs(M, nE * sides);
    QTX_HIP(c, c->mscr.ensure((size_t)jb * qtx::modes_ws_elems(M) * sizeof(double2)));
    // per job: the status, then (16-byte aligned) the eigenvalue shift taken
    const size_t shift_off = ((size_t)jb * sizeof(int) + 15) / 16 * 16;
    QTX_HIP(c, c->mjst.ensure(shift_off + (size_t)jb * sizeof(double2)));
    QTX_HIP(c, record(c, c->ev_dec, c->n_dec));
    QTX_HIP(c, qtx::run_modes(M, make_prob(c), E_dev, nE, eta, sides, c->mode_tol, c->m, c->num_cu,
                              c->mscr.as<double2>(), c->mjst.as<int>(),
                              reinterpret_cast<double2*>(c->mjst.as<char>() + shift_off), b.sig, b.wf, b.sgn, b.iters,
                              b.nheavy, c->stream));
    QTX_HIP(c, record(c, c->ev_dec, c->n_dec));
    return QTX_OK;
  }
  qtx::Prob P = make_prob(c);
  QTX_HIP(c, record(c, c->ev_dec, c->n_dec));
  QTX_HIP(c, qtx::run_decimate(M, P, qtx::BatchDesc{}, E_dev, nE, eta, sides, dec_opts(c), b.dscr, b.gdec, b.sig,
                               b.wf, b.sgn, b.iters, b.nheavy, c->stream));
  QTX_HIP(c, record(c, c->ev_dec, c->n_dec));
  return QTX_OK;
}

// Per-energy decimation outputs of the context for nE energies.
qtx_status ensure_dec_outputs(qtx_ctx* c, int nE, SolveBufs& b) {
  const int M = c->M;
  const size_t MM = (size_t)M * M;
  QTX_HIP(c, c->sig.ensure((size_t)nE * 2 * MM * sizeof(double2)));
  QTX_HIP(c, c->wf.ensure((size_t)nE * 2 * MM * sizeof(double2)));
  QTX_HIP(c, c->sgn.ensure((size_t)nE * 2 * M * sizeof(double)));
  QTX_HIP(c, c->iters.ensure((size_t)nE * 2 * sizeof(int)));
  QTX_HIP(c, c->nheavy.ensure((size_t)nE * 2 * sizeof(int)));
  b.sig = c->sig.as<double2>();
  b.wf = c->wf.as<double2>();
  b.sgn = c->sgn.as<double>();
  b.iters = c->iters.as<int>();
  b.nheavy = c->nheavy.as<int>();
  return QTX_OK;
}

// One launch chunk of a solve on the context stream: self-energies, then
// the sweep (mixed: the single-precision sweep with refinement, the list of
// unconverged energies and their FP64 re-solve), all in the buffers b.
qtx_status enqueue_chunk(qtx_ctx* c, const double* E_dev, int ne, double eta, bool mixed, double* T_dev,
                         double* ldos_dev, qtx_info* info_dev, const SolveBufs& b) {
  qtx_status s = stage_decimate(c, E_dev, ne, eta, mixed, b);
  if (s != QTX_OK) return s;
  qtx::Prob P = make_prob(c);
  qtx::SweepArgs a{};
  a.E = E_dev;
  a.nE = ne;
  a.eta = eta;
  a.sig = b.sig;
  a.wf = b.wf;
  a.sgn = b.sgn;
  a.iters = b.iters;
  a.nheavy = b.nheavy;
  a.ws = b.sws;
  a.ws_bytes = b.wsb;
  a.part = b.part;
  a.nmax = c->N;
  a.T = T_dev;
  a.ldos = ldos_dev;
  a.info = info_dev;
  a.elist = nullptr;
  a.ecount = nullptr;
  a.redo = mixed ? b.redo : nullptr;
  a.rtol = c->refine_tol;
  a.maxstep = c->refine_max;
  QTX_HIP(c, record(c, c->ev_sw, c->n_sw));
  QTX_HIP(c, sweep_launch(c, c->M, mixed, P, a, qtx::BatchDesc{}, b.grid));
  if (mixed) {
    // energies whose refinement did not converge: FP64 sweep on the list
    QTX_HIP(c, qtx::run_compact(b.redo, ne, b.elist, b.ecount, c->stream));
    qtx::SweepArgs f = a;
    f.elist = b.elist;
    f.ecount = b.ecount;
    f.redo = nullptr;
    QTX_HIP(c, sweep_launch(c, c->M, false, P, f, qtx::BatchDesc{}, b.grid));
  }
  QTX_HIP(c, record(c, c->ev_sw, c->n_sw));
  return QTX_OK;
}

qtx_status check_solve_args(qtx_ctx* c, const double* E_dev, int nE, double eta, qtx_precision prec,
                            double* T_dev) {
  qtx_status s = check_ready(c);
  if (s != QTX_OK) return s;
  if (nE < 0 || !(eta >= 0.0)) return fail(c, QTX_EINVAL, "nE must be >= 0 and eta >= 0");
  if (nE == 0) return QTX_OK;
  if (!E_dev || !T_dev) return fail(c, QTX_EINVAL, "E and T must not be NULL");
  if (prec != QTX_FP64 && prec != QTX_MIXED) return fail(c, QTX_EINVAL, "precision must be QTX_FP64 or QTX_MIXED");
  return check_method(c, eta, prec == QTX_MIXED);
}

qtx_status solve_device_core(qtx_ctx* c, const double* E_dev, int nE, double eta, qtx_precision prec,
                             double* T_dev, double* ldos_dev, qtx_info* info_dev) {
  qtx_status s = check_solve_args(c, E_dev, nE, eta, prec, T_dev);
  if (s != QTX_OK || nE == 0) return s;
  const bool mixed = (prec == QTX_MIXED);
  const int M = c->M, N = c->N;
  const int sides = leads_identical(c) ? 1 : 2;
  for (int e0 = 0; e0 < nE; e0 += c->chunk) {
    const int ne = std::min(c->chunk, nE - e0);
    SolveBufs b;
    s = ensure_dec_outputs(c, ne, b);
    if (s != QTX_OK) return s;
    if (c->se_method != 1) {
      b.gdec = dec_grid(c, ne, sides, mixed);
      QTX_HIP(c, c->dscr.ensure((size_t)b.gdec * qtx::dec_ws_elems(M) * sizeof(double2)));
      b.dscr = c->dscr.as<double2>();
    }
    b.wsb = qtx::sweep_ws_bytes(N, M, mixed);
    for (bool retry = true; retry;) {
      b.grid = sweep_grid(c, ne, M, mixed, b.wsb);
      if (b.grid < 1)
        return fail(c, QTX_ENOMEM, "no sweep workspace of one workgroup fits (sweep_workspace_bytes or device memory)");
      QTX_HIP(c, alloc_sweep_ws(c, (size_t)b.grid * b.wsb, &retry));
    }
    b.sws = c->sws.as<char>();
    QTX_HIP(c, c->part.ensure((size_t)b.grid * 4 * 2 * N * (mixed ? 2 : 1) * sizeof(double)));
    b.part = c->part.as<double>();
    if (mixed) {
      QTX_HIP(c, c->redo.ensure((size_t)ne * sizeof(int)));
      QTX_HIP(c, c->elist.ensure((size_t)ne * sizeof(int)));
      QTX_HIP(c, c->ecount.ensure(sizeof(int)));
      b.redo = c->redo.as<int>();
      b.elist = c->elist.as<int>();
      b.ecount = c->ecount.as<int>();
    }
    s = enqueue_chunk(c, E_dev + e0, ne, eta, mixed, T_dev + e0, ldos_dev ? ldos_dev + (size_t)e0 * 2 * N : nullptr,
                      info_dev ? info_dev + e0 : nullptr, b);
    if (s != QTX_OK) return s;
  }
  return QTX_OK;
}

// Density-matrix blocks of an energy grid, enqueued on the context stream:
// decimation and the density-matrix sweep per launch chunk into one
// accumulator per workgroup, then their sum into out_d / out_o (device,
// m x m blocks).  T, ldos (or null) and info (or null) as in a solve.
qtx_status density_matrix_core(qtx_ctx* c, const double* E_dev, const double* wL_dev, const double* wR_dev, int nE,
                               double eta, double2* out_d, double2* out_o, double* T_dev, double* ldos_dev,
                               qtx_info* info_dev) {
  qtx_status s = check_ready(c);
  if (s != QTX_OK) return s;
  if (nE < 0 || !(eta >= 0.0)) return fail(c, QTX_EINVAL, "nE must be >= 0 and eta >= 0");
  const int N = c->N, m = c->m, M = c->M;
  if (!out_d || (N > 1 && !out_o)) return fail(c, QTX_EINVAL, "rho_diag (and rho_off when N > 1) must not be NULL");
  s = check_method(c, eta, false);
  if (s != QTX_OK) return s;
  const size_t mm = (size_t)m * m, nblk = 2 * (size_t)N - 1;
  if (nE == 0) {
    // the sum over no accumulators writes zeros (rho is not read); a kernel
    // rather than memsets, so that a caller may capture the call in a graph
    QTX_HIP(c, qtx::run_dm_reduce(out_d, 0, 0, N, M, m, out_d, out_o, c->stream));
    return QTX_OK;
  }
  if (!E_dev || !wL_dev || !wR_dev || !T_dev) return fail(c, QTX_EINVAL, "E, wL, wR and T must not be NULL");
  const size_t MM = (size_t)M * M, stride = nblk * MM;
  const size_t per_wg = stride * sizeof(double2);
  const int cap = (int)std::min<double>(1 << 20, std::floor(c->dm_bytes / (double)per_wg));
  if (cap < 1) return fail(c, QTX_ENOMEM, "density_matrix_bytes is below one workgroup's accumulators");
  // one accumulator per workgroup; every workgroup takes its first energy
  // in the first launch (grid <= the first launch's energies)
  const int first = std::min(c->chunk, nE);
  const size_t wsb = qtx::sweep_ws_bytes(N, M, false, true);
  int grid = 0;
  for (bool retry = true; retry;) {
    const int sgrid = sweep_grid(c, first, M, false, wsb);
    if (sgrid < 1) return fail(c, QTX_ENOMEM, "no sweep workspace of one workgroup fits (sweep_workspace_bytes or device memory)");
    grid = std::min(sgrid, cap);
    QTX_HIP(c, alloc_sweep_ws(c, (size_t)grid * wsb, &retry));
  }
  QTX_HIP(c, c->rho.ensure((size_t)grid * per_wg));
  QTX_HIP(c, c->part.ensure((size_t)grid * 4 * 2 * N * sizeof(double)));
  for (int e0 = 0; e0 < nE; e0 += c->chunk) {
    const int ne = std::min(c->chunk, nE - e0);
    SolveBufs db;
    s = ensure_dec_outputs(c, ne, db);
    if (s != QTX_OK) return s;
    if (c->se_method != 1) {
      db.gdec = dec_grid(c, ne, leads_identical(c) ? 1 : 2, false);
      QTX_HIP(c, c->dscr.ensure((size_t)db.gdec * qtx::dec_ws_elems(M) * sizeof(double2)));
      db.dscr = c->dscr.as<double2>();
    }
    s = stage_decimate(c, E_dev + e0, ne, eta, false, db);
    if (s != QTX_OK) return s;
    qtx::SweepArgs a{};
    a.E = E_dev + e0;
    a.nE = ne;
    a.eta = eta;
    a.sig = c->sig.as<double2>();
    a.wf = c->wf.as<double2>();
    a.sgn = c->sgn.as<double>();
    a.iters = c->iters.as<int>();
    a.nheavy = c->nheavy.as<int>();
    a.ws = c->sws.as<char>();
    a.ws_bytes = wsb;
    a.part = c->part.as<double>();
    a.nmax = N;
    a.T = T_dev + e0;
    a.ldos = ldos_dev ? ldos_dev + (size_t)e0 * 2 * N : nullptr;
    a.info = info_dev ? info_dev + e0 : nullptr;
    a.dmwL = wL_dev + e0;
    a.dmwR = wR_dev + e0;
    a.rho = c->rho.as<double2>();
    a.rho_stride = stride;
    a.rho_first = e0 == 0;
    QTX_HIP(c, record(c, c->ev_sw, c->n_sw));
    QTX_HIP(c, qtx::run_sweep_dm(M, make_prob(c), a, grid, c->stream));
    QTX_HIP(c, record(c, c->ev_sw, c->n_sw));
  }
  QTX_HIP(c, qtx::run_dm_reduce(c->rho.as<double2>(), grid, stride, N, M, m, out_d, out_o, c->stream));
  return QTX_OK;
}

// Layout of one solve chunk inside the fixed no-allocation scratch: every
// buffer the launch sequence uses, each at a 256-byte boundary.  Sizes
// (energies per chunk, sweep and decimation workgroups) are chosen so that
// the whole layout fits in cap bytes: the sweep workspaces take up to three
// quarters, the decimation workgroups a quarter of the rest, the per-energy
// decimation outputs what is left.  Fails when not even one energy with one
// workgroup of each kernel fits.
qtx_status plan_noalloc(qtx_ctx* c, int nE, bool mixed, char* base, size_t cap, int* chunk, SolveBufs* out) {
  const int M = c->M, N = c->N;
  const size_t MM = (size_t)M * M, AL = 256;
  const int sides = leads_identical(c) ? 1 : 2;
  auto up = [&](size_t x) { return (x + AL - 1) / AL * AL; };
  const size_t wsb = qtx::sweep_ws_bytes(N, M, mixed);
  const size_t per_wg = up(wsb) + up((size_t)4 * 2 * N * (mixed ? 2 : 1) * sizeof(double));
  const size_t dec_wg = up(qtx::dec_ws_elems(M) * sizeof(double2));
  const size_t per_e = 2 * (2 * MM * sizeof(double2)) + 2 * M * sizeof(double) + 4 * sizeof(int) +
                       (mixed ? 2 * sizeof(int) : 0);
  const size_t slack = 16 * AL;                       // alignment of the eleven regions and ecount
  if (cap <= slack || per_wg + dec_wg + per_e > cap - slack)
    return fail(c, QTX_ENOMEM,
                "problem too large for the no-allocation scratch: one energy needs " +
                    std::to_string(per_wg + dec_wg + per_e + slack) + " bytes, the scratch holds " +
                    std::to_string(cap) + " (use qtx_solve_device)");
  const size_t avail = cap - slack;
  const double budget = c->sweep_eff >= 0.0 ? std::min(c->sweep_eff, c->sweep_bytes) : c->sweep_bytes;
  long long grid = std::min<long long>({(long long)c->num_cu * wgs_per_cu(c, M, mixed), (long long)nE,
                                        (long long)(0.75 * (double)avail / (double)per_wg),
                                        (long long)std::floor(budget / (double)wsb)});
  grid = std::max<long long>(grid, 1);
  size_t rest = avail - (size_t)grid * per_wg;
  long long gdec = std::min<long long>({(long long)c->num_cu * dec_wgs_per_cu(c, M, mixed), (long long)nE * sides,
                                        (long long)(rest / 4 / dec_wg)});
  gdec = std::max<long long>(gdec, 1);
  rest -= (size_t)gdec * dec_wg;
  long long ne = std::min<long long>({(long long)nE, (long long)c->chunk, (long long)(rest / per_e)});
  if (ne < 1)
    return fail(c, QTX_ENOMEM, "problem too large for the no-allocation scratch (use qtx_solve_device)");
  grid = std::min(grid, ne);
  gdec = std::min(gdec, ne * sides);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base + off;
    off += up(bytes);
    return p;
  };
  SolveBufs b;
  b.sig = (double2*)take((size_t)ne * 2 * MM * sizeof(double2));
  b.wf = (double2*)take((size_t)ne * 2 * MM * sizeof(double2));
  b.sgn = (double*)take((size_t)ne * 2 * M * sizeof(double));
  b.iters = (int*)take((size_t)ne * 2 * sizeof(int));
  b.nheavy = (int*)take((size_t)ne * 2 * sizeof(int));
  b.gdec = (int)gdec;
  b.dscr = (double2*)take((size_t)gdec * qtx::dec_ws_elems(M) * sizeof(double2));
  b.grid = (int)grid;
  b.wsb = wsb;
  b.sws = take((size_t)grid * wsb);
  b.part = (double*)take((size_t)grid * 4 * 2 * N * (mixed ? 2 : 1) * sizeof(double));
  if (mixed) {
    b.redo = (int*)take((size_t)ne * sizeof(int));
    b.elist = (int*)take((size_t)ne * sizeof(int));
    b.ecount = (int*)take(sizeof(int));
  }
  if (off > cap) return fail(c, QTX_EDEVICE, "internal error: no-allocation layout exceeds the scratch");
  *chunk = (int)ne;
  *out = b;
  return QTX_OK;
}

}  // namespace

extern "C" {

const char* qtx_version(void) { return "qtx 0.1 (gfx950)"; }

qtx_status qtx_create(int hip_device, qtx_ctx** out) {
  if (!out) return QTX_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return QTX_EINVAL;
  if (hipSetDevice(hip_device) != hipSuccess) return QTX_EDEVICE;
  qtx_ctx* c = new qtx_ctx();
  c->device = hip_device;
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess && cu > 0)
    c->num_cu = cu;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return QTX_EDEVICE;
  }
  c->own_stream = true;
  *out = c;
  return QTX_OK;
}

void qtx_destroy(qtx_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev_dec) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ev_sw) (void)hipEventDestroy(e);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  for (auto& kv : c->sigcache) {
    DevBuf* cb[] = {&kv.second.sig, &kv.second.wf, &kv.second.sgn, &kv.second.iters, &kv.second.nheavy};
    for (DevBuf* b : cb) b->release();
  }
  c->bslot.release();
  c->bjobE.release();
  c->bjobLead.release();
  DevBuf* bufs[] = {&c->dlead[0], &c->dlead[1], &c->ddev, &c->dV, &c->wE, &c->wT, &c->wldos, &c->winfo,
                    &c->sig, &c->wf, &c->sgn, &c->iters, &c->nheavy, &c->dscr, &c->sws, &c->part,
                    &c->redo, &c->elist, &c->ecount, &c->bprobs, &c->bitem_prob, &c->bitem_ldos,
                    &c->bjob_item, &c->bjob_side, &c->bE, &c->bT, &c->bldos, &c->binfo};
  for (DevBuf* b : bufs) b->release();
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* qtx_last_error(const qtx_ctx* c) { return c ? c->err.c_str() : "null context"; }

qtx_status qtx_set_stream(qtx_ctx* c, void* st) {
  if (!c) return QTX_EINVAL;
  if (c->own_stream && c->stream) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipStreamDestroy(c->stream);
    c->stream = nullptr;
    c->own_stream = false;
  }
  if (st) {
    c->stream = (hipStream_t)st;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
      return fail(c, QTX_EDEVICE, "stream creation failed");
    c->own_stream = true;
  }
  return QTX_OK;
}

qtx_status qtx_set_lead(qtx_ctx* c, qtx_side side, int m, const qtx_c128* H00, const qtx_c128* H01,
                        const qtx_c128* S00, const qtx_c128* S01, double V_lead) {
  if (!c) return QTX_EINVAL;
  if (side != QTX_LEFT && side != QTX_RIGHT) return fail(c, QTX_EINVAL, "side must be QTX_LEFT or QTX_RIGHT");
  if (!H00 || !H01 || !S00 || !S01) return fail(c, QTX_EINVAL, "lead blocks must not be NULL");
  if (m < 1 || m > 128) return fail(c, QTX_EINVAL, "block size m must be in [1, 128]");
  if (!std::isfinite(V_lead)) return fail(c, QTX_EINVAL, "lead potential must be finite");
  const int other = 1 - side;
  if ((c->lead_set[other] || c->dev_set) && c->m != m) return fail(c, QTX_EINVAL, "m differs from the other lead / device");
  if (!hermitian(H00, m, 1e-12) || !hermitian(S00, m, 1e-12))
    return fail(c, QTX_EINVAL, "H00 and S00 must be Hermitian");
  QTX_HIP(c, hipSetDevice(c->device));
  c->m = m;
  c->M = qtx::padded_block(m);
  const int M = c->M;
  const size_t MM = (size_t)M * M;
  std::vector<double2> h(4 * MM);
  pad_block(H00, m, M, true, h, 0);
  pad_block(H01, m, M, false, h, MM);
  pad_block(S00, m, M, false, h, 2 * MM);
  pad_block(S01, m, M, false, h, 3 * MM);
  QTX_HIP(c, c->dlead[side].ensure(4 * MM * sizeof(double2)));
  QTX_HIP(c, hipMemcpy(c->dlead[side].p, h.data(), 4 * MM * sizeof(double2), hipMemcpyHostToDevice));
  auto& hl = c->hlead[side];
  hl.resize(4 * (size_t)m * m);
  const qtx_c128* srcs[4] = {H00, H01, S00, S01};
  for (int q = 0; q < 4; ++q)
    for (int i = 0; i < m * m; ++i) hl[(size_t)q * m * m + i] = cd(srcs[q][i].re, srcs[q][i].im);
  // content hash of the lead blocks (keys of the self-energy cache)
  uint64_t hh = 1469598103934665603ull ^ (uint64_t)m;
  const unsigned char* bytes = reinterpret_cast<const unsigned char*>(hl.data());
  for (size_t i = 0; i < hl.size() * sizeof(cd); ++i) hh = (hh ^ bytes[i]) * 1099511628211ull;
  c->lead_hash[side] = hh;
  c->Vlead[side] = V_lead;
  c->lead_set[side] = true;
  return QTX_OK;
}

qtx_status qtx_set_device(qtx_ctx* c, int N, int m, const qtx_c128* Hd, const qtx_c128* Hu,
                          const qtx_c128* Sd, const qtx_c128* Su) {
  if (!c) return QTX_EINVAL;
  if (N < 1) return fail(c, QTX_EINVAL, "N must be >= 1");
  if (m < 1 || m > 128) return fail(c, QTX_EINVAL, "block size m must be in [1, 128]");
  if ((c->lead_set[0] || c->lead_set[1]) && c->m != m) return fail(c, QTX_EINVAL, "m differs from the leads");
  const int given = (Hd != nullptr) + (Sd != nullptr) + ((Hu != nullptr) || N == 1) + ((Su != nullptr) || N == 1);
  const bool none = !Hd && !Hu && !Sd && !Su;
  if (!none && given != 4) return fail(c, QTX_EINVAL, "give all four device block arrays or none");
  QTX_HIP(c, hipSetDevice(c->device));
  c->m = m;
  c->M = qtx::padded_block(m);
  if (none) {
    if (!c->lead_set[0]) return fail(c, QTX_ESTATE, "a uniform device copies the left lead: set it first");
    c->uniform = true;
    c->ddev.release();
  } else {
    for (int i = 0; i < N; ++i)
      if (!hermitian(Hd + (size_t)i * m * m, m, 1e-12) || !hermitian(Sd + (size_t)i * m * m, m, 1e-12))
        return fail(c, QTX_EINVAL, "device on-site blocks must be Hermitian");
    const int M = c->M;
    const size_t MM = (size_t)M * M;
    const size_t nblk = 4 * (size_t)N - 2;
    std::vector<double2> h(nblk * MM);
    size_t off = 0;
    for (int i = 0; i < N; ++i, off += MM) pad_block(Hd + (size_t)i * m * m, m, M, true, h, off);
    for (int i = 0; i < N - 1; ++i, off += MM) pad_block(Hu + (size_t)i * m * m, m, M, false, h, off);
    for (int i = 0; i < N; ++i, off += MM) pad_block(Sd + (size_t)i * m * m, m, M, false, h, off);
    for (int i = 0; i < N - 1; ++i, off += MM) pad_block(Su + (size_t)i * m * m, m, M, false, h, off);
    QTX_HIP(c, c->ddev.ensure(nblk * MM * sizeof(double2)));
    QTX_HIP(c, hipMemcpy(c->ddev.p, h.data(), nblk * MM * sizeof(double2), hipMemcpyHostToDevice));
    c->uniform = false;
  }
  if (c->N != N) c->pot_set = false;
  c->N = N;
  c->dev_set = true;
  return QTX_OK;
}

qtx_status qtx_set_potential(qtx_ctx* c, const double* V, qtx_pot_mode mode) {
  if (!c) return QTX_EINVAL;
  if (!c->dev_set) return fail(c, QTX_ESTATE, "set the device before the potential");
  if (!V) return fail(c, QTX_EINVAL, "V must not be NULL");
  if (mode != QTX_POT_DIAG && mode != QTX_POT_LINEAR_FE) return fail(c, QTX_EINVAL, "unknown potential mode");
  for (int i = 0; i < c->N; ++i)
    if (!std::isfinite(V[i])) return fail(c, QTX_EINVAL, "potential must be finite");
  QTX_HIP(c, hipSetDevice(c->device));
  QTX_HIP(c, c->dV.ensure((size_t)c->N * sizeof(double)));
  QTX_HIP(c, hipMemcpy(c->dV.p, V, (size_t)c->N * sizeof(double), hipMemcpyHostToDevice));
  c->pot_mode = mode;
  c->pot_set = true;
  return QTX_OK;
}

qtx_status qtx_solve_device(qtx_ctx* c, const double* E_dev, int nE, double eta, qtx_precision prec,
                            double* T_dev, double* ldos_dev, qtx_info* info_dev) {
  if (!c) return QTX_EINVAL;
  if (prec != QTX_FP64 && prec != QTX_MIXED) return fail(c, QTX_EINVAL, "unknown precision");
  QTX_HIP(c, hipSetDevice(c->device));
  return solve_device_core(c, E_dev, nE, eta, prec, T_dev, ldos_dev, info_dev);
}

qtx_status qtx_solve_device_noalloc(qtx_ctx* c, const double* E_dev, int nE, double eta, qtx_precision prec,
                                    double* T_dev, double* ldos_dev, qtx_info* info_dev) {
  if (!c) return QTX_EINVAL;
  if (prec != QTX_FP64 && prec != QTX_MIXED) return fail(c, QTX_EINVAL, "unknown precision");
  QTX_HIP(c, hipSetDevice(c->device));
  qtx_status s = check_solve_args(c, E_dev, nE, eta, prec, T_dev);
  if (s != QTX_OK || nE == 0) return s;
  if (c->se_method != 0)
    return fail(c, QTX_EINVAL, "the no-allocation solve uses the decimation (self_energy_method 0)");
  char* base = nullptr;
  QTX_HIP(c, qtx::noalloc_scratch(c->device, &base));
  const bool mixed = prec == QTX_MIXED;
  int ne = 0;
  SolveBufs b;
  s = plan_noalloc(c, nE, mixed, base, qtx::kNoAllocScratchBytes, &ne, &b);
  if (s != QTX_OK) return s;
  // no kernel timing here: recording it could create events
  const bool timing = c->timing;
  c->timing = false;
  const int N = c->N;
  for (int e0 = 0; e0 < nE && s == QTX_OK; e0 += ne) {
    const int k = std::min(ne, nE - e0);
    SolveBufs bk = b;
    bk.grid = std::min(b.grid, k);
    bk.gdec = std::min(b.gdec, k * (leads_identical(c) ? 1 : 2));
    s = enqueue_chunk(c, E_dev + e0, k, eta, mixed, T_dev + e0, ldos_dev ? ldos_dev + (size_t)e0 * 2 * N : nullptr,
                      info_dev ? info_dev + e0 : nullptr, bk);
  }
  c->timing = timing;
  return s;
}

qtx_status qtx_solve(qtx_ctx* c, const double* E, int nE, double eta, qtx_precision prec, double* T,
                     double* ldos, qtx_info* info) {
  if (!c) return QTX_EINVAL;
  if (prec != QTX_FP64 && prec != QTX_MIXED) return fail(c, QTX_EINVAL, "unknown precision");
  if (nE < 0) return fail(c, QTX_EINVAL, "nE must be >= 0");
  if (nE == 0) return QTX_OK;
  if (!E || !T) return fail(c, QTX_EINVAL, "E and T must not be NULL");
  for (int e = 0; e < nE; ++e)
    if (!std::isfinite(E[e])) return fail(c, QTX_EINVAL, "energies must be finite");
  qtx_status s = check_ready(c);
  if (s != QTX_OK) return s;
  QTX_HIP(c, hipSetDevice(c->device));
  const int N = c->N;
  QTX_HIP(c, c->wE.ensure((size_t)nE * sizeof(double)));
  QTX_HIP(c, c->wT.ensure((size_t)nE * sizeof(double)));
  QTX_HIP(c, c->wldos.ensure((size_t)nE * 2 * N * sizeof(double)));
  QTX_HIP(c, c->winfo.ensure((size_t)nE * sizeof(qtx_info)));
  QTX_HIP(c, hipMemcpyAsync(c->wE.p, E, (size_t)nE * sizeof(double), hipMemcpyHostToDevice, c->stream));
  s = solve_device_core(c, c->wE.as<double>(), nE, eta, prec, c->wT.as<double>(), c->wldos.as<double>(),
                        c->winfo.as<qtx_info>());
  if (s != QTX_OK) return s;
  std::vector<qtx_info> hinfo(nE);
  QTX_HIP(c, hipMemcpyAsync(T, c->wT.p, (size_t)nE * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (ldos)
    QTX_HIP(c, hipMemcpyAsync(ldos, c->wldos.p, (size_t)nE * 2 * N * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
  QTX_HIP(c, hipMemcpyAsync(hinfo.data(), c->winfo.p, (size_t)nE * sizeof(qtx_info), hipMemcpyDeviceToHost,
                            c->stream));
  QTX_HIP(c, hipStreamSynchronize(c->stream));
  bool flagged = false;
  for (int e = 0; e < nE; ++e) flagged |= (hinfo[e].flags != 0);
  if (info) std::memcpy(info, hinfo.data(), (size_t)nE * sizeof(qtx_info));
  if (flagged) return fail(c, QTX_ENOTCONV, "some energies were flagged (see qtx_info.flags)");
  return QTX_OK;
}

qtx_status qtx_density_matrix_device(qtx_ctx* c, const double* E_dev, const double* wL_dev, const double* wR_dev,
                                     int nE, double eta, qtx_c128* rho_diag_dev, qtx_c128* rho_off_dev,
                                     double* T_dev, double* ldos_dev, qtx_info* info_dev) {
  if (!c) return QTX_EINVAL;
  QTX_HIP(c, hipSetDevice(c->device));
  return density_matrix_core(c, E_dev, wL_dev, wR_dev, nE, eta, (double2*)rho_diag_dev, (double2*)rho_off_dev,
                             T_dev, ldos_dev, info_dev);
}

qtx_status qtx_density_matrix(qtx_ctx* c, const double* E, const double* wL, const double* wR, int nE, double eta,
                              qtx_c128* rho_diag, qtx_c128* rho_off, double* T, double* ldos, qtx_info* info) {
  if (!c) return QTX_EINVAL;
  qtx_status s = check_ready(c);
  if (s != QTX_OK) return s;
  const int N = c->N, m = c->m;
  if (nE < 0 || !(eta >= 0.0)) return fail(c, QTX_EINVAL, "nE must be >= 0 and eta >= 0");
  if (!rho_diag || (N > 1 && !rho_off)) return fail(c, QTX_EINVAL, "rho_diag (and rho_off when N > 1) must not be NULL");
  const size_t mm = (size_t)m * m, nblk = 2 * (size_t)N - 1;
  if (nE == 0) {
    std::memset(rho_diag, 0, (size_t)N * mm * sizeof(qtx_c128));
    if (N > 1) std::memset(rho_off, 0, (size_t)(N - 1) * mm * sizeof(qtx_c128));
    return QTX_OK;
  }
  if (!E || !wL || !wR) return fail(c, QTX_EINVAL, "E, wL and wR must not be NULL");
  for (int e = 0; e < nE; ++e)
    if (!std::isfinite(E[e]) || !std::isfinite(wL[e]) || !std::isfinite(wR[e]))
      return fail(c, QTX_EINVAL, "energies and weights must be finite");
  QTX_HIP(c, hipSetDevice(c->device));
  QTX_HIP(c, c->wE.ensure((size_t)nE * sizeof(double)));
  QTX_HIP(c, c->wT.ensure((size_t)nE * sizeof(double)));
  QTX_HIP(c, c->wldos.ensure((size_t)nE * 2 * N * sizeof(double)));
  QTX_HIP(c, c->winfo.ensure((size_t)nE * sizeof(qtx_info)));
  QTX_HIP(c, c->dmw.ensure((size_t)2 * nE * sizeof(double)));
  QTX_HIP(c, c->dmout.ensure(nblk * mm * sizeof(double2)));
  double* wdev = c->dmw.as<double>();
  QTX_HIP(c, hipMemcpyAsync(c->wE.p, E, (size_t)nE * sizeof(double), hipMemcpyHostToDevice, c->stream));
  QTX_HIP(c, hipMemcpyAsync(wdev, wL, (size_t)nE * sizeof(double), hipMemcpyHostToDevice, c->stream));
  QTX_HIP(c, hipMemcpyAsync(wdev + nE, wR, (size_t)nE * sizeof(double), hipMemcpyHostToDevice, c->stream));
  double2* od = c->dmout.as<double2>();
  s = density_matrix_core(c, c->wE.as<double>(), wdev, wdev + nE, nE, eta, od, od + (size_t)N * mm,
                          c->wT.as<double>(), c->wldos.as<double>(), c->winfo.as<qtx_info>());
  if (s != QTX_OK) return s;
  std::vector<qtx_info> hinfo(nE);
  QTX_HIP(c, hipMemcpyAsync(rho_diag, od, (size_t)N * mm * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
  if (N > 1)
    QTX_HIP(c, hipMemcpyAsync(rho_off, od + (size_t)N * mm, (size_t)(N - 1) * mm * sizeof(double2),
                              hipMemcpyDeviceToHost, c->stream));
  if (T) QTX_HIP(c, hipMemcpyAsync(T, c->wT.p, (size_t)nE * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (ldos)
    QTX_HIP(c, hipMemcpyAsync(ldos, c->wldos.p, (size_t)nE * 2 * N * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
  QTX_HIP(c, hipMemcpyAsync(hinfo.data(), c->winfo.p, (size_t)nE * sizeof(qtx_info), hipMemcpyDeviceToHost,
                            c->stream));
  QTX_HIP(c, hipStreamSynchronize(c->stream));
  bool flagged = false;
  for (int e = 0; e < nE; ++e) flagged |= (hinfo[e].flags != 0);
  if (info) std::memcpy(info, hinfo.data(), (size_t)nE * sizeof(qtx_info));
  if (flagged) return fail(c, QTX_ENOTCONV, "some energies were flagged (see qtx_info.flags)");
  return QTX_OK;
}

qtx_status qtx_self_energy(qtx_ctx* c, const double* E, int nE, double eta, qtx_c128* sigma, qtx_c128* wfac,
                           double* sgn, int* iters) {
  if (!c) return QTX_EINVAL;
  if (nE < 0 || !(eta >= 0.0)) return fail(c, QTX_EINVAL, "nE must be >= 0 and eta >= 0");
  if (nE == 0) return QTX_OK;
  if (!E || !sigma) return fail(c, QTX_EINVAL, "E and sigma must not be NULL");
  if (!c->lead_set[0] || !c->lead_set[1]) return fail(c, QTX_ESTATE, "both leads must be set");
  if (check_method(c, eta, false) != QTX_OK) return QTX_EINVAL;
  QTX_HIP(c, hipSetDevice(c->device));
  const int m = c->m, M = c->M;
  const size_t MM = (size_t)M * M;
  QTX_HIP(c, c->wE.ensure((size_t)nE * sizeof(double)));
  QTX_HIP(c, hipMemcpyAsync(c->wE.p, E, (size_t)nE * sizeof(double), hipMemcpyHostToDevice, c->stream));
  SolveBufs db;
  qtx_status s = ensure_dec_outputs(c, nE, db);
  if (s != QTX_OK) return s;
  if (c->se_method != 1) {
    db.gdec = dec_grid(c, nE, leads_identical(c) ? 1 : 2, false);
    QTX_HIP(c, c->dscr.ensure((size_t)db.gdec * qtx::dec_ws_elems(M) * sizeof(double2)));
    db.dscr = c->dscr.as<double2>();
  }
  s = stage_decimate(c, c->wE.as<double>(), nE, eta, false, db);
  if (s != QTX_OK) return s;
  std::vector<double2> hs((size_t)nE * 2 * MM), hw;
  std::vector<double> hg;
  std::vector<int> hi((size_t)nE * 2);
  QTX_HIP(c, hipMemcpyAsync(hs.data(), c->sig.p, hs.size() * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
  if (wfac) {
    hw.resize((size_t)nE * 2 * MM);
    QTX_HIP(c, hipMemcpyAsync(hw.data(), c->wf.p, hw.size() * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
  }
  if (sgn) {
    hg.resize((size_t)nE * 2 * M);
    QTX_HIP(c, hipMemcpyAsync(hg.data(), c->sgn.p, hg.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  }
  QTX_HIP(c, hipMemcpyAsync(hi.data(), c->iters.p, hi.size() * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  QTX_HIP(c, hipStreamSynchronize(c->stream));
  bool notconv = false;
  for (int e = 0; e < nE; ++e)
    for (int sd = 0; sd < 2; ++sd) {
      const size_t b = ((size_t)e * 2 + sd);
      for (int r = 0; r < m; ++r)
        for (int q = 0; q < m; ++q) {
          const double2 v = hs[b * MM + (size_t)r * M + q];
          sigma[b * m * m + (size_t)r * m + q] = qtx_c128{v.x, v.y};
          if (wfac) {
            const double2 u = hw[b * MM + (size_t)r * M + q];
            wfac[b * m * m + (size_t)r * m + q] = qtx_c128{u.x, u.y};
          }
        }
      if (sgn)
        for (int q = 0; q < m; ++q) sgn[b * m + q] = hg[b * M + q];
      notconv |= hi[b] < 0;
    }
  if (iters)
    for (int e = 0; e < nE; ++e) iters[e] = std::max(hi[2 * e], hi[2 * e + 1]) < 0 ? -1 : std::max(hi[2 * e], hi[2 * e + 1]);
  if (notconv) return fail(c, QTX_ENOTCONV, "decimation hit its iteration cap for some energy");
  return QTX_OK;
}

qtx_status qtx_kernel_times(qtx_ctx* c, int enable, double* decimate_ms, double* sweep_ms, int* launches) {
  if (!c) return QTX_EINVAL;
  QTX_HIP(c, hipSetDevice(c->device));
  QTX_HIP(c, hipStreamSynchronize(c->stream));
  double td = 0.0, ts = 0.0;
  for (size_t k = 0; k + 1 < c->n_dec; k += 2) {
    float ms = 0.0f;
    QTX_HIP(c, hipEventElapsedTime(&ms, c->ev_dec[k], c->ev_dec[k + 1]));
    td += ms;
  }
  for (size_t k = 0; k + 1 < c->n_sw; k += 2) {
    float ms = 0.0f;
    QTX_HIP(c, hipEventElapsedTime(&ms, c->ev_sw[k], c->ev_sw[k + 1]));
    ts += ms;
  }
  if (decimate_ms) *decimate_ms = td;
  if (sweep_ms) *sweep_ms = ts;
  if (launches) *launches = (int)(c->n_sw / 2);
  c->n_dec = c->n_sw = 0;
  c->timing = enable != 0;
  return QTX_OK;
}

qtx_status qtx_set_option(qtx_ctx* c, const char* name, double value) {
  if (!c) return QTX_EINVAL;
  if (!name) return fail(c, QTX_EINVAL, "option name must not be NULL");
  const std::string n(name);
  const bool integral = std::isfinite(value) && value == std::floor(value);
  if (n == "decimation_tol") {
    if (!(value > 0.0 && value < 1.0)) return fail(c, QTX_EINVAL, "decimation_tol must be in (0, 1)");
    c->dec_tol = value;
  } else if (n == "decimation_refine_cond") {
    if (!(value >= 0.0)) return fail(c, QTX_EINVAL, "decimation_refine_cond must be >= 0");
    c->dec_rcond = value;
  } else if (n == "sigma_newton_tol") {
    if (!(value >= -1.0 && value < 1.0)) return fail(c, QTX_EINVAL, "sigma_newton_tol must be in [-1, 1)");
    c->newton_tol = value;
  } else if (n == "decimation_max_iters") {
    if (!integral || value < 1 || value > 1000) return fail(c, QTX_EINVAL, "decimation_max_iters must be in [1, 1000]");
    c->dec_maxit = (int)value;
  } else if (n == "refine_tol") {
    if (!(value > 0.0 && value < 1.0)) return fail(c, QTX_EINVAL, "refine_tol must be in (0, 1)");
    c->refine_tol = value;
  } else if (n == "refine_max_steps") {
    if (!integral || value < 0 || value > 20) return fail(c, QTX_EINVAL, "refine_max_steps must be in [0, 20]");
    c->refine_max = (int)value;
  } else if (n == "refine_weight_tol") {
    if (!(value >= 0.0 && value <= 1.0)) return fail(c, QTX_EINVAL, "refine_weight_tol must be in [0, 1]");
    c->heavy_tol = value;
  } else if (n == "workgroups_per_cu") {
    if (!integral || value < 1 || value > 4) return fail(c, QTX_EINVAL, "workgroups_per_cu must be in [1, 4]");
    c->wg_per_cu = (int)value;
    c->tuned[0].clear();
    c->tuned[1].clear();
  } else if (n == "sigma_cache_bytes") {
    if (!(value >= 0.0 && value <= 1e13)) return fail(c, QTX_EINVAL, "sigma_cache_bytes must be in [0, 1e13]");
    c->sigcache_bytes = value;
    for (auto& kv : c->sigcache) {           // shrink or drop: start over
      kv.second.index.clear();
      kv.second.key.clear();
      kv.second.tick.clear();
      kv.second.cap = 0;
    }
  } else if (n == "use_graph") {
    if (!(value == 0.0 || value == 1.0)) return fail(c, QTX_EINVAL, "use_graph must be 0 or 1");
    c->use_graph = value != 0.0;
  } else if (n == "sweep_workspace_bytes") {
    if (!(value > 0.0 && value <= 1e13)) return fail(c, QTX_EINVAL, "sweep_workspace_bytes must be in (0, 1e13]");
    c->sweep_bytes = value;
    c->sweep_eff = -1.0;
  } else if (n == "density_matrix_bytes") {
    if (!(value >= 0.0 && value <= 1e13)) return fail(c, QTX_EINVAL, "density_matrix_bytes must be in [0, 1e13]");
    c->dm_bytes = value;
  } else if (n == "self_energy_method") {
    if (!(value == 0.0 || value == 1.0)) return fail(c, QTX_EINVAL, "self_energy_method must be 0 or 1");
    c->se_method = (int)value;
  } else if (n == "mode_tol") {
    if (!(value > 0.0 && value <= 1e-2)) return fail(c, QTX_EINVAL, "mode_tol must be in (0, 1e-2]");
    c->mode_tol = value;
  } else if (n == "panel_width") {
    if (!(value == 0.0 || value == 16.0 || value == 32.0)) return fail(c, QTX_EINVAL, "panel_width must be 0, 16 or 32");
    c->opt_pw = (int)value;
    c->tuned[0].clear();
    c->tuned[1].clear();
  } else if (n == "refine_tiles") {
    if (!(value == 0.0 || value == 1.0 || value == 2.0)) return fail(c, QTX_EINVAL, "refine_tiles must be 0, 1 or 2");
    c->opt_tpp = (int)value;
    c->tuned[0].clear();
    c->tuned[1].clear();
  } else if (n == "energies_per_launch") {
    if (!integral || value < 1 || value > (1 << 20)) return fail(c, QTX_EINVAL, "energies_per_launch must be in [1, 2^20]");
    c->chunk = (int)value;
  } else {
    return fail(c, QTX_EINVAL, "unknown option: " + n);
  }
  return QTX_OK;
}

qtx_status qtx_problem_create(qtx_ctx* parent, qtx_ctx** problem) {
  if (!parent || !problem) return QTX_EINVAL;
  *problem = nullptr;
  qtx_ctx* c = new qtx_ctx();
  c->device = parent->device;
  c->num_cu = parent->num_cu;
  c->dec_tol = parent->dec_tol;
  c->dec_rcond = parent->dec_rcond;
  c->dec_maxit = parent->dec_maxit;
  c->chunk = parent->chunk;
  c->wg_per_cu = parent->wg_per_cu;
  c->opt_pw = parent->opt_pw;
  c->opt_tpp = parent->opt_tpp;
  c->tuned[0] = parent->tuned[0];
  c->tuned[1] = parent->tuned[1];
  c->refine_tol = parent->refine_tol;
  c->refine_max = parent->refine_max;
  c->heavy_tol = parent->heavy_tol;
  c->newton_tol = parent->newton_tol;
  c->use_graph = parent->use_graph;
  c->dm_bytes = parent->dm_bytes;
  c->sweep_bytes = parent->sweep_bytes;
  c->se_method = parent->se_method;
  c->mode_tol = parent->mode_tol;
  c->stream = parent->stream;
  c->own_stream = false;
  c->parent = parent;
  *problem = c;
  return QTX_OK;
}

}  // extern "C"

namespace {

// One launch group of a batch: a contiguous range of items (all of one
// padded block size) and its decimation jobs.
struct BatchChunk {
  int M, nmax, item0, nitems, job0, njobs;
};

// Decimation jobs of one block size that fill self-energy cache slots.
struct DecGroup {
  int M, job0, njobs;
};

void drop_graph(qtx_ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
  c->batch_sig.clear();
}

// The launch sequence of a batch (decimation, sweep, and for the mixed
// path the compaction and FP64 re-solve of unconverged items), chunk by
// chunk on the context stream.  Buffers must already have their sizes.
qtx_status enqueue_batch(qtx_ctx* c, const std::vector<BatchChunk>& chunks, const std::vector<DecGroup>& groups,
                         double eta, bool mixed, bool cached) {
  for (const DecGroup& g : groups) {
    if (g.njobs == 0) continue;
    qtx_ctx::SigCache& sc = c->sigcache[g.M];
    const int wg = dec_wgs_per_cu(c, g.M, mixed);
    qtx::BatchDesc b{};
    b.probs = c->bprobs.as<qtx::Prob>();
    b.job_item = c->bjob_item.as<int>() + g.job0;
    b.njobs = g.njobs;
    b.job_E = c->bjobE.as<double>() + g.job0;
    b.job_lead = c->bjobLead.as<const double2*>() + g.job0;
    qtx::Prob P0{};
    P0.M = g.M;
    const int gdec = std::max(1, std::min(g.njobs, c->num_cu * wg));
    QTX_HIP(c, qtx::run_decimate(g.M, P0, b, b.job_E, g.njobs, eta, 2, dec_opts(c), c->dscr.as<double2>(), gdec,
                                 sc.sig.as<double2>(), sc.wf.as<double2>(), sc.sgn.as<double>(), sc.iters.as<int>(),
                                 sc.nheavy.as<int>(), c->stream));
  }
  for (const BatchChunk& k : chunks) {
    const int M = k.M;
    const bool big = M > 64;
    const int wg = dec_wgs_per_cu(c, M, mixed);
    qtx::BatchDesc b{};
    b.probs = c->bprobs.as<qtx::Prob>();
    b.item_prob = c->bitem_prob.as<int>() + k.item0;
    b.item_ldos = c->bitem_ldos.as<size_t>() + k.item0;
    b.job_item = c->bjob_item.as<int>() + k.job0;
    b.job_side = c->bjob_side.as<int>() + k.job0;
    b.njobs = k.njobs;
    qtx::Prob P0{};
    P0.N = k.nmax;
    P0.M = M;
    if (!cached) {
      const int gdec = std::max(1, std::min(k.njobs, c->num_cu * wg));
      QTX_HIP(c, qtx::run_decimate(M, P0, b, c->bE.as<double>() + k.item0, k.nitems, eta, 2, dec_opts(c),
                                   c->dscr.as<double2>(), gdec, c->sig.as<double2>(), c->wf.as<double2>(),
                                   c->sgn.as<double>(), c->iters.as<int>(), c->nheavy.as<int>(), c->stream));
    }
    const int grid = sweep_grid(c, k.nitems, M, mixed, qtx::sweep_ws_bytes(k.nmax, M, mixed));
    qtx::SweepArgs a{};
    a.E = c->bE.as<double>() + k.item0;
    a.nE = k.nitems;
    a.eta = eta;
    if (cached) {
      qtx_ctx::SigCache& sc = c->sigcache[M];
      a.sig = sc.sig.as<double2>();
      a.wf = sc.wf.as<double2>();
      a.sgn = sc.sgn.as<double>();
      a.iters = sc.iters.as<int>();
      a.nheavy = sc.nheavy.as<int>();
      a.sig_slot = c->bslot.as<int>() + 2 * (size_t)k.item0;
    } else {
      a.sig = c->sig.as<double2>();
      a.wf = c->wf.as<double2>();
      a.sgn = c->sgn.as<double>();
      a.iters = c->iters.as<int>();
      a.nheavy = c->nheavy.as<int>();
      a.sig_slot = nullptr;
    }
    a.ws = c->sws.as<char>();
    a.ws_bytes = qtx::sweep_ws_bytes(k.nmax, M, mixed);
    a.part = c->part.as<double>();
    a.nmax = k.nmax;
    a.T = c->bT.as<double>() + k.item0;
    a.ldos = c->bldos.as<double>();
    a.info = c->binfo.as<qtx_info>() + k.item0;
    a.elist = nullptr;
    a.ecount = nullptr;
    a.redo = mixed ? c->redo.as<int>() : nullptr;
    a.rtol = c->refine_tol;
    a.maxstep = c->refine_max;
    QTX_HIP(c, sweep_launch(c, M, mixed, P0, a, b, grid));
    if (mixed) {
      QTX_HIP(c, qtx::run_compact(c->redo.as<int>(), k.nitems, c->elist.as<int>(), c->ecount.as<int>(), c->stream));
      qtx::SweepArgs f = a;
      f.elist = c->elist.as<int>();
      f.ecount = c->ecount.as<int>();
      f.redo = nullptr;
      QTX_HIP(c, sweep_launch(c, M, false, P0, f, b, grid));
    }
  }
  return QTX_OK;
}

}  // namespace

extern "C" {

qtx_status qtx_solve_batch(qtx_ctx* c, int nprob, qtx_ctx* const* probs, const double* const* E, const int* nE,
                           double eta, qtx_precision prec, double* const* T, double* const* ldos) {
  if (!c) return QTX_EINVAL;
  if (nprob < 0 || (nprob > 0 && (!probs || !E || !nE || !T))) return fail(c, QTX_EINVAL, "bad batch arguments");
  if (prec != QTX_FP64 && prec != QTX_MIXED) return fail(c, QTX_EINVAL, "precision must be QTX_FP64 or QTX_MIXED");
  if (!(eta >= 0.0)) return fail(c, QTX_EINVAL, "eta must be >= 0");
  for (int p = 0; p < nprob; ++p) {
    qtx_ctx* q = probs[p];
    if (!q) return fail(c, QTX_EINVAL, "NULL problem in batch");
    if (q->device != c->device) return fail(c, QTX_EINVAL, "every problem must live on the batch context's device");
    qtx_status s = check_ready(q);
    if (s != QTX_OK) return fail(c, s, std::string("problem ") + std::to_string(p) + ": " + q->err);
    if (nE[p] < 0) return fail(c, QTX_EINVAL, "nE must be >= 0");
    if (nE[p] > 0 && (!E[p] || !T[p])) return fail(c, QTX_EINVAL, "E[p] and T[p] must not be NULL");
    for (int e = 0; e < nE[p]; ++e)
      if (!std::isfinite(E[p][e])) return fail(c, QTX_EINVAL, "energies must be finite");
  }
  for (int p = 0; p < nprob; ++p)
    if (probs[p]->se_method != 0 || c->se_method != 0)
      return fail(c, QTX_EINVAL, "batched solves use the decimation (self_energy_method 0)");
  QTX_HIP(c, hipSetDevice(c->device));
  const bool mixed = (prec == QTX_MIXED);

  // problems grouped by padded block size, each group by decreasing slab
  // count, so that the grid-stride order hands out the longest items first
  std::vector<int> order(nprob);
  for (int p = 0; p < nprob; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    if (probs[x]->M != probs[y]->M) return probs[x]->M < probs[y]->M;
    return probs[x]->N > probs[y]->N;
  });
  std::vector<qtx::Prob> hprob(nprob);
  for (int p = 0; p < nprob; ++p) hprob[p] = make_prob(probs[p]);
  std::vector<int> item_prob, item_e, job_item, job_side;
  std::vector<double> hE;
  std::vector<size_t> item_ldos;
  std::vector<BatchChunk> chunks;
  size_t ldos_total = 0;
  for (size_t oi = 0; oi < order.size();) {
    const int M = probs[order[oi]]->M;
    size_t oj = oi;
    while (oj < order.size() && probs[order[oj]]->M == M) ++oj;
    BatchChunk k{M, 0, (int)item_prob.size(), 0, (int)job_item.size(), 0};
    auto close_chunk = [&]() {
      if (k.nitems > 0) chunks.push_back(k);
      k = BatchChunk{M, 0, (int)item_prob.size(), 0, (int)job_item.size(), 0};
    };
    for (size_t o = oi; o < oj; ++o) {
      const int p = order[o];
      const qtx_ctx* q = probs[p];
      const bool same = leads_identical(q);
      for (int e = 0; e < nE[p]; ++e) {
        if (k.nitems == c->chunk) close_chunk();
        item_prob.push_back(p);
        item_e.push_back(e);
        hE.push_back(E[p][e]);
        item_ldos.push_back(ldos_total);
        ldos_total += 2 * (size_t)q->N;
        const int local = k.nitems++;
        k.nmax = std::max(k.nmax, q->N);
        if (same) {
          job_item.push_back(local);
          job_side.push_back(-1);
          k.njobs += 1;
        } else {
          job_item.push_back(local);
          job_side.push_back(0);
          job_item.push_back(local);
          job_side.push_back(1);
          k.njobs += 2;
        }
      }
    }
    close_chunk();
    oi = oj;
  }
  const int nitems = (int)item_prob.size();
  if (nitems == 0) return QTX_OK;

  // self-energy cache: both contacts of every item look up (lead content,
  // shifted energy E - V); misses become decimation jobs into slots taken
  // in round-robin order (clock hand kept per cache), skipping the slots
  // this call uses
  bool cached = c->sigcache_bytes > 0;
  std::vector<int> slot2;
  std::vector<int> cjob_slot;
  std::vector<double> cjob_E;
  std::vector<const double2*> cjob_lead;
  std::vector<DecGroup> groups;
  long long hits = 0, misses = 0;
  // until this call has run its decimation jobs, the slots it assigned hold
  // no data: any early return drops the cache index
  struct CacheGuard {
    qtx_ctx* c;
    bool armed = true;
    ~CacheGuard() {
      if (!armed) return;
      for (auto& kv : c->sigcache) {
        kv.second.index.clear();
        std::fill(kv.second.tick.begin(), kv.second.tick.end(), -1);
      }
    }
  } guard{c};
  if (cached) {
    const std::vector<double> params = {eta, c->dec_tol, c->dec_rcond, (double)c->dec_maxit, c->heavy_tol,
                                        c->newton_tol};
    if (params != c->cache_params) {
      for (auto& kv : c->sigcache) {
        kv.second.index.clear();
        std::fill(kv.second.tick.begin(), kv.second.tick.end(), -1);
      }
      c->cache_params = params;
    }
    const long long now = ++c->cache_calls;
    slot2.assign(2 * (size_t)nitems, 0);
    bool overflow = false;
    for (int i = 0; i < nitems && !overflow;) {
      const int M = probs[item_prob[i]]->M;
      qtx_ctx::SigCache& sc = c->sigcache[M];
      const size_t MM = (size_t)M * M;
      const size_t entry = 2 * MM * 2 * sizeof(double2) + 2 * M * sizeof(double) + 4 * sizeof(int);
      const int cap = (int)std::min<double>(1 << 22, std::max(16.0, std::floor(c->sigcache_bytes / entry)));
      if (sc.cap != cap) {
        sc.index.clear();
        sc.key.assign(cap, {0, 0});
        sc.tick.assign(cap, -1);
        sc.cap = cap;
        sc.M = M;
        sc.hand = 0;
      }
      QTX_HIP(c, sc.sig.ensure((size_t)cap * 2 * MM * sizeof(double2)));
      QTX_HIP(c, sc.wf.ensure((size_t)cap * 2 * MM * sizeof(double2)));
      QTX_HIP(c, sc.sgn.ensure((size_t)cap * 2 * M * sizeof(double)));
      QTX_HIP(c, sc.iters.ensure((size_t)cap * 2 * sizeof(int)));
      QTX_HIP(c, sc.nheavy.ensure((size_t)cap * 2 * sizeof(int)));
      DecGroup g{M, (int)cjob_slot.size(), 0};
      int& hand = sc.hand;
      if (hand >= cap) hand = 0;
      int scanned = 0;
      for (; i < nitems && probs[item_prob[i]]->M == M; ++i) {
        const qtx_ctx* q = probs[item_prob[i]];
        for (int side = 0; side < 2 && !overflow; ++side) {
          const double Es = hE[i] - q->Vlead[side];
          uint64_t eb;
          std::memcpy(&eb, &Es, sizeof(eb));
          const std::pair<uint64_t, uint64_t> key(q->lead_hash[side], eb);
          const unsigned long long hk = key.first * 0x9E3779B97F4A7C15ull ^ key.second;
          auto it = sc.index.find(hk);
          int slot = -1;
          if (it != sc.index.end() && sc.key[it->second] == key) {
            slot = it->second;
            ++hits;
          } else {
            // clock scan for a slot not used by this call
            while (scanned < 2 * cap && sc.tick[hand] == now) {
              hand = (hand + 1) % cap;
              ++scanned;
            }
            if (sc.tick[hand] == now) {
              overflow = true;
              break;
            }
            slot = hand;
            hand = (hand + 1) % cap;
            if (sc.tick[slot] >= 0) {
              const auto& old = sc.key[slot];
              auto ot = sc.index.find(old.first * 0x9E3779B97F4A7C15ull ^ old.second);
              if (ot != sc.index.end() && ot->second == slot) sc.index.erase(ot);
            }
            if (it != sc.index.end()) sc.index.erase(it);   // hash collision: the new key takes over
            sc.key[slot] = key;
            sc.index[hk] = slot;
            cjob_slot.push_back(slot);
            cjob_E.push_back(Es);
            cjob_lead.push_back(q->dlead[side].as<double2>());
            ++misses;
          }
          sc.tick[slot] = now;
          slot2[2 * (size_t)i + side] = slot;
        }
      }
      g.njobs = (int)cjob_slot.size() - g.job0;
      groups.push_back(g);
    }
    if (overflow) {
      // this batch needs more distinct contacts than the cache holds: drop
      // what this call assigned and solve it without the cache
      for (auto& kv : c->sigcache) {
        kv.second.index.clear();
        std::fill(kv.second.tick.begin(), kv.second.tick.end(), -1);
      }
      cached = false;
      groups.clear();
      hits = misses = 0;
    }
  }

  // buffer sizes (all allocations before any capture)
  size_t sig_b = 0, dscr_b = 0, sws_b = 0, part_b = 0, per_b = 0;
  for (const DecGroup& g : groups) {
    const int wg = dec_wgs_per_cu(c, g.M, mixed);
    const size_t gdec = std::max(1, std::min(g.njobs, c->num_cu * wg));
    dscr_b = std::max(dscr_b, gdec * qtx::dec_ws_elems(g.M) * sizeof(double2));
  }
  for (const BatchChunk& k : chunks) {
    const size_t MM = (size_t)k.M * k.M;
    const int wg = dec_wgs_per_cu(c, k.M, mixed);
    const size_t gdec = std::max(1, std::min(k.njobs, c->num_cu * wg));
    sig_b = std::max(sig_b, (size_t)k.nitems * 2 * MM * sizeof(double2));
    per_b = std::max(per_b, (size_t)k.nitems);
    dscr_b = std::max(dscr_b, gdec * qtx::dec_ws_elems(k.M) * sizeof(double2));
  }
  int maxM = 16;
  for (const BatchChunk& k : chunks) maxM = std::max(maxM, k.M);
  QTX_HIP(c, c->sig.ensure(sig_b));
  QTX_HIP(c, c->wf.ensure(sig_b));
  QTX_HIP(c, c->sgn.ensure(per_b * 2 * maxM * sizeof(double)));
  QTX_HIP(c, c->iters.ensure(per_b * 2 * sizeof(int)));
  QTX_HIP(c, c->nheavy.ensure(per_b * 2 * sizeof(int)));
  QTX_HIP(c, c->dscr.ensure(dscr_b));
  for (bool retry = true; retry;) {
    sws_b = part_b = 0;
    for (const BatchChunk& k : chunks) {
      const size_t wsb = qtx::sweep_ws_bytes(k.nmax, k.M, mixed);
      const int sgrid = sweep_grid(c, k.nitems, k.M, mixed, wsb);
      if (sgrid < 1) return fail(c, QTX_ENOMEM, "no sweep workspace of one workgroup fits (sweep_workspace_bytes or device memory)");
      sws_b = std::max(sws_b, (size_t)sgrid * wsb);
      part_b = std::max(part_b, (size_t)sgrid * 4 * 2 * (size_t)k.nmax * (mixed ? 2 : 1) * sizeof(double));
    }
    QTX_HIP(c, alloc_sweep_ws(c, sws_b, &retry));
  }
  QTX_HIP(c, c->part.ensure(part_b));
  QTX_HIP(c, c->redo.ensure(per_b * sizeof(int)));
  QTX_HIP(c, c->elist.ensure(per_b * sizeof(int)));
  QTX_HIP(c, c->ecount.ensure(sizeof(int)));
  QTX_HIP(c, c->bprobs.ensure(nprob * sizeof(qtx::Prob)));
  QTX_HIP(c, c->bitem_prob.ensure(nitems * sizeof(int)));
  QTX_HIP(c, c->bitem_ldos.ensure(nitems * sizeof(size_t)));
  QTX_HIP(c, c->bjob_item.ensure(std::max(std::max(job_item.size(), cjob_slot.size()), (size_t)1) * sizeof(int)));
  QTX_HIP(c, c->bjob_side.ensure(job_side.size() * sizeof(int)));
  QTX_HIP(c, c->bE.ensure(nitems * sizeof(double)));
  QTX_HIP(c, c->bT.ensure(nitems * sizeof(double)));
  QTX_HIP(c, c->bldos.ensure(std::max<size_t>(ldos_total, 1) * sizeof(double)));
  QTX_HIP(c, c->binfo.ensure(nitems * sizeof(qtx_info)));

  QTX_HIP(c, hipMemcpyAsync(c->bprobs.p, hprob.data(), nprob * sizeof(qtx::Prob), hipMemcpyHostToDevice, c->stream));
  QTX_HIP(c, hipMemcpyAsync(c->bitem_prob.p, item_prob.data(), nitems * sizeof(int), hipMemcpyHostToDevice, c->stream));
  QTX_HIP(c, hipMemcpyAsync(c->bitem_ldos.p, item_ldos.data(), nitems * sizeof(size_t), hipMemcpyHostToDevice,
                            c->stream));
  QTX_HIP(c, hipMemcpyAsync(c->bjob_item.p, job_item.data(), job_item.size() * sizeof(int), hipMemcpyHostToDevice,
                            c->stream));
  QTX_HIP(c, hipMemcpyAsync(c->bjob_side.p, job_side.data(), job_side.size() * sizeof(int), hipMemcpyHostToDevice,
                            c->stream));
  QTX_HIP(c, hipMemcpyAsync(c->bE.p, hE.data(), nitems * sizeof(double), hipMemcpyHostToDevice, c->stream));
  if (cached) {
    QTX_HIP(c, c->bslot.ensure(slot2.size() * sizeof(int)));
    QTX_HIP(c, hipMemcpyAsync(c->bslot.p, slot2.data(), slot2.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    const size_t nj = std::max<size_t>(cjob_slot.size(), 1);
    QTX_HIP(c, c->bjob_item.ensure(std::max(nj, job_item.size()) * sizeof(int)));
    QTX_HIP(c, c->bjobE.ensure(nj * sizeof(double)));
    QTX_HIP(c, c->bjobLead.ensure(nj * sizeof(void*)));
    if (!cjob_slot.empty()) {
      QTX_HIP(c, hipMemcpyAsync(c->bjob_item.p, cjob_slot.data(), cjob_slot.size() * sizeof(int),
                                hipMemcpyHostToDevice, c->stream));
      QTX_HIP(c, hipMemcpyAsync(c->bjobE.p, cjob_E.data(), cjob_E.size() * sizeof(double), hipMemcpyHostToDevice,
                                c->stream));
      QTX_HIP(c, hipMemcpyAsync(c->bjobLead.p, cjob_lead.data(), cjob_lead.size() * sizeof(void*),
                                hipMemcpyHostToDevice, c->stream));
    }
  }
  c->cache_hits += hits;
  c->cache_misses += misses;

  // the launch sequence depends on the batch shape (and the buffers, whose
  // sizes follow from it): replay the captured graph while it is unchanged
  std::vector<long long> sig;
  sig.push_back(mixed);
  sig.push_back(c->wg_per_cu);
  for (const BatchChunk& k : chunks)
    for (bool mx : {mixed, false}) {
      const qtx_tune t = tune_of(c, k.M, mx);
      for (int v : {t.workgroups_per_cu, t.panel_width, t.refine_tiles}) sig.push_back(v);
    }
  sig.push_back(c->chunk);
  sig.push_back(c->refine_max);
  long long eb;
  std::memcpy(&eb, &eta, sizeof(eb));
  sig.push_back(eb);
  std::memcpy(&eb, &c->refine_tol, sizeof(eb));
  sig.push_back(eb);
  std::memcpy(&eb, &c->heavy_tol, sizeof(eb));
  sig.push_back(eb);
  std::memcpy(&eb, &c->dec_tol, sizeof(eb));
  sig.push_back(eb);
  std::memcpy(&eb, &c->dec_rcond, sizeof(eb));
  sig.push_back(eb);
  std::memcpy(&eb, &c->newton_tol, sizeof(eb));
  sig.push_back(eb);
  std::memcpy(&eb, &c->sweep_bytes, sizeof(eb));
  sig.push_back(eb);
  std::memcpy(&eb, &c->sweep_eff, sizeof(eb));
  sig.push_back(eb);
  sig.push_back(c->dec_maxit);
  // every buffer the captured launches read or write (a buffer that grew or
  // was released since the capture has moved, and the graph must not run)
  for (void* bp : {c->sig.p, c->wf.p, c->sgn.p, c->iters.p, c->nheavy.p, c->dscr.p, c->sws.p, c->part.p,
                   c->redo.p, c->elist.p, c->ecount.p, c->bprobs.p, c->bitem_prob.p, c->bitem_ldos.p,
                   c->bjob_item.p, c->bjob_side.p, c->bE.p, c->bT.p, c->bldos.p, c->binfo.p, c->bslot.p,
                   c->bjobE.p, c->bjobLead.p})
    sig.push_back((long long)(uintptr_t)bp);
  for (const BatchChunk& k : chunks)
    for (int v : {k.M, k.nmax, k.item0, k.nitems, k.job0, k.njobs}) sig.push_back(v);
  sig.push_back(cached);
  for (const DecGroup& g : groups)
    for (int v : {g.M, g.job0, g.njobs}) sig.push_back(v);
  for (auto& kv : c->sigcache) {
    sig.push_back(kv.first);
    for (void* bp : {kv.second.sig.p, kv.second.wf.p, kv.second.sgn.p, kv.second.iters.p, kv.second.nheavy.p})
      sig.push_back((long long)(uintptr_t)bp);
  }
  if (!c->use_graph) {
    drop_graph(c);
    qtx_status s = enqueue_batch(c, chunks, groups, eta, mixed, cached);
    if (s != QTX_OK) return s;
  } else {
    if (sig != c->batch_sig || !c->graph_exec) {
      drop_graph(c);
      QTX_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      qtx_status s = enqueue_batch(c, chunks, groups, eta, mixed, cached);
      hipGraph_t g = nullptr;
      hipError_t ce = hipStreamEndCapture(c->stream, &g);
      if (s != QTX_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
      }
      if (ce != hipSuccess) return hipfail(c, ce, "hipStreamEndCapture");
      c->graph = g;
      QTX_HIP(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
      c->batch_sig = sig;
    }
    QTX_HIP(c, hipGraphLaunch(c->graph_exec, c->stream));
  }

  std::vector<double> hT(nitems), hL(ldos ? ldos_total : 0);
  std::vector<qtx_info> hinfo(nitems);
  QTX_HIP(c, hipMemcpyAsync(hT.data(), c->bT.p, nitems * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (ldos)
    QTX_HIP(c, hipMemcpyAsync(hL.data(), c->bldos.p, ldos_total * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  QTX_HIP(c, hipMemcpyAsync(hinfo.data(), c->binfo.p, nitems * sizeof(qtx_info), hipMemcpyDeviceToHost, c->stream));
  QTX_HIP(c, hipStreamSynchronize(c->stream));
  guard.armed = false;
  bool flagged = false;
  for (int i = 0; i < nitems; ++i) {
    const int p = item_prob[i], e = item_e[i];
    T[p][e] = hT[i];
    if (ldos && ldos[p])
      std::memcpy(ldos[p] + (size_t)e * 2 * probs[p]->N, hL.data() + item_ldos[i], 2 * probs[p]->N * sizeof(double));
    flagged |= hinfo[i].flags != 0;
  }
  if (flagged) return fail(c, QTX_ENOTCONV, "some energies were flagged");
  return QTX_OK;
}

qtx_status qtx_autotune(qtx_ctx* c, const double* E, int nE, double eta, qtx_precision prec, qtx_tune* best_out,
                        qtx_tune* cand_out, double* times_ms, int* ncand_out) {
  if (!c) return QTX_EINVAL;
  if (prec != QTX_FP64 && prec != QTX_MIXED) return fail(c, QTX_EINVAL, "precision must be QTX_FP64 or QTX_MIXED");
  if (nE < 1 || !E) return fail(c, QTX_EINVAL, "need at least one sample energy");
  if (!(eta >= 0.0)) return fail(c, QTX_EINVAL, "eta must be >= 0");
  for (int e = 0; e < nE; ++e)
    if (!std::isfinite(E[e])) return fail(c, QTX_EINVAL, "energies must be finite");
  qtx_status s = check_ready(c);
  if (s != QTX_OK) return s;
  QTX_HIP(c, hipSetDevice(c->device));
  const bool mixed = prec == QTX_MIXED;
  const int M = c->M, N = c->N;
  // candidates: every built tile shape, with every workgroup count from 1 to
  // what the kernel's registers and LDS allow (at most 4; mixed sweeps above
  // 64 keep one: their workspace of 0.3-0.5 GB per workgroup at N = 400
  // bounds the count)
  std::vector<qtx_tune> cand;
  for (int pw : {16, 32})
    for (int tpp : {1, 2}) {
      if (!qtx::sweep_variant_ok(M, mixed, pw, tpp)) continue;
      int occ_sweep = 0, occ_dec = 0;
      QTX_HIP(c, qtx::max_resident(M, mixed, pw, tpp, &occ_sweep, &occ_dec));
      const int top = std::max(1, std::min(M > 64 && mixed ? 1 : 4, occ_sweep));
      for (int wg = 1; wg <= top; ++wg) cand.push_back(qtx_tune{wg, pw, tpp});
    }
  QTX_HIP(c, c->wE.ensure((size_t)nE * sizeof(double)));
  QTX_HIP(c, c->wT.ensure((size_t)nE * sizeof(double)));
  QTX_HIP(c, c->wldos.ensure((size_t)nE * 2 * N * sizeof(double)));
  QTX_HIP(c, hipMemcpyAsync(c->wE.p, E, (size_t)nE * sizeof(double), hipMemcpyHostToDevice, c->stream));
  hipEvent_t e0, e1;
  QTX_HIP(c, hipEventCreate(&e0));
  QTX_HIP(c, hipEventCreate(&e1));
  const bool timing = c->timing;
  c->timing = false;
  const bool had = c->tuned[mixed].count(M) > 0;
  const qtx_tune before = had ? c->tuned[mixed][M] : qtx_tune{};
  std::vector<double> med(cand.size(), 0.0);
  size_t best = 0;
  qtx_status st = QTX_OK;
  for (size_t k = 0; k < cand.size() && st == QTX_OK; ++k) {
    c->tuned[mixed][M] = cand[k];
    // one solve to allocate and warm up, then the median of three timed ones
    double t[3];
    for (int rep = 0; rep < 4 && st == QTX_OK; ++rep) {
      if (rep > 0 && hipEventRecord(e0, c->stream) != hipSuccess) st = fail(c, QTX_EDEVICE, "hipEventRecord");
      if (st == QTX_OK)
        st = solve_device_core(c, c->wE.as<double>(), nE, eta, prec, c->wT.as<double>(), c->wldos.as<double>(),
                               nullptr);
      if (st == QTX_OK && rep > 0) {
        float ms = 0.0f;
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
          st = fail(c, QTX_EDEVICE, "event timing failed");
        t[rep - 1] = ms;
      }
    }
    if (st != QTX_OK) break;
    std::sort(t, t + 3);
    med[k] = t[1];
    if (med[k] < med[best]) best = k;
  }
  c->timing = timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // the timed solves sized the workspaces for the largest candidate; release
  // them (a later solve on this context allocates what it needs), so that a
  // problem context tuned before a batch holds no workspace the batch needs
  (void)hipStreamSynchronize(c->stream);
  c->sws.release();
  c->dscr.release();
  if (st != QTX_OK) {
    if (had) c->tuned[mixed][M] = before;
    else c->tuned[mixed].erase(M);
    return st;
  }
  c->tuned[mixed][M] = cand[best];
  if (c->parent) c->parent->tuned[mixed][M] = cand[best];
  if (best_out) *best_out = cand[best];
  const int n = (int)std::min<size_t>(cand.size(), QTX_TUNE_MAX_CANDIDATES);
  for (int k = 0; k < n; ++k) {
    if (cand_out) cand_out[k] = cand[k];
    if (times_ms) times_ms[k] = med[k];
  }
  if (ncand_out) *ncand_out = n;
  return QTX_OK;
}

int qtx_check_layouts(char* msg, int len) {
  std::string err;
  int nsweep = 0, ndec = 0, nplan = 0;
  struct Reg {
    const char* name;
    size_t off, n, align;
  };
  auto check = [&](const std::string& what, size_t cap, const std::vector<Reg>& regs) {
    for (size_t i = 0; i < regs.size() && err.empty(); ++i) {
      const Reg& a = regs[i];
      if (a.n == 0) continue;
      if (a.off % a.align != 0) err = what + ": " + a.name + " misaligned";
      else if (a.off > cap || a.n > cap - a.off) err = what + ": " + a.name + " beyond the workspace";
      for (size_t j = 0; j < i && err.empty(); ++j) {
        const Reg& b = regs[j];
        if (b.n != 0 && a.off < b.off + b.n && b.off < a.off + a.n)
          err = what + ": " + a.name + " overlaps " + b.name;
      }
    }
  };
  const int Ms[] = {16, 32, 48, 64, 96, 128};
  // sweep workspaces: every block size and precision, items of N slabs in a
  // launch sized for nmax >= N slabs, and the FP64 re-solve that runs in the
  // mixed sweep's workspace after it
  for (int M : Ms)
    for (int N : {1, 2, 3, 7, 50, 200, 400})
      for (int extra : {0, 13})
        for (int mode = 0; mode < 3 && err.empty(); ++mode) {
          const bool mixed = mode == 1, dm = mode == 2;
          const size_t ws = qtx::sweep_ws_bytes(N + extra, M, mixed, dm);
          const std::string what = "sweep M=" + std::to_string(M) + " N=" + std::to_string(N) + "/" +
                                   std::to_string(N + extra) + (mixed ? " mixed" : dm ? " dm" : " fp64");
          for (bool fallback : {false, true}) {
            if (fallback && !mixed) continue;
            const qtx::SweepLayout L = qtx::sweep_layout(N, M, mixed && !fallback, dm, ws);
            ++nsweep;
            const size_t al = (mixed && !fallback) ? 8 : 16;
            check(what + (fallback ? " (FP64 re-solve)" : ""), ws,
                  {{"[X|z]", L.xz, L.xz_n, al}, {"psi", L.psi, L.psi_n, al}, {"Dt^-1", L.di, L.di_n, 8},
                   {"corrections", L.zc, L.zc_n, 8}, {"rhs slab", L.yb, L.yb_n, 8}, {"psi64", L.p64, L.p64_n, 16},
                   {"working matrix", L.mat, L.mat_n, al}, {"coupling block", L.lst, L.lst_n, al},
                   {"residual block", L.stg, L.stg_n, 16}});
          }
        }
  // decimation workspace: e, eR, [a | b], X, residual (8 M^2) and the
  // working matrix above 64; the Newton step reuses the first 7 M^2
  for (int M : Ms) {
    const size_t MM = (size_t)M * M, el = sizeof(double2);
    const size_t cap = qtx::dec_ws_elems(M) * el;
    ++ndec;
    check("decimation M=" + std::to_string(M), cap,
          {{"e", 0, MM * el, 16}, {"eR", MM * el, MM * el, 16}, {"[a|b]", 2 * MM * el, 2 * MM * el, 16},
           {"X", 4 * MM * el, 2 * MM * el, 16}, {"residual", 6 * MM * el, 2 * MM * el, 16},
           {"working matrix", 8 * MM * el, M > 64 ? (size_t)M * (M + 1) * el : 0, 16}});
    check("newton M=" + std::to_string(M), cap,
          {{"G, Q, P, X, T1, P2, Q2", 0, 7 * MM * el, 16}, {"job counter", 7 * MM * el, sizeof(int), 4},
           {"working matrix", 8 * MM * el, M > 64 ? (size_t)M * (M + 1) * el : 0, 16}});
  }
  // no-allocation layouts of several problems (host arithmetic only)
  for (int M : Ms)
    for (int N : {1, 16, 200, 400})
      for (int nE : {1, 64, 2048, 100000})
        for (int mode = 0; mode < 4 && err.empty(); ++mode) {
          const bool mixed = mode & 1, two = mode & 2;
          qtx_ctx c;
          c.M = M;
          c.m = M;
          c.N = N;
          c.num_cu = 256;
          if (two) c.Vlead[1] = 0.1;                  // distinct leads: two lead iterations per energy
          char* base = reinterpret_cast<char*>((uintptr_t)1 << 20);
          int ne = 0;
          SolveBufs b;
          const size_t cap = qtx::kNoAllocScratchBytes;
          if (plan_noalloc(&c, nE, mixed, base, cap, &ne, &b) != QTX_OK) continue;   // refused: nothing carved
          ++nplan;
          const size_t MM = (size_t)M * M;
          auto off = [&](const void* p) { return (size_t)(reinterpret_cast<const char*>(p) - base); };
          check("noalloc M=" + std::to_string(M) + " N=" + std::to_string(N) + " nE=" + std::to_string(nE) +
                    (mixed ? " mixed" : " fp64") + (two ? " two leads" : ""),
                cap,
                {{"sigma", off(b.sig), (size_t)ne * 2 * MM * sizeof(double2), 256},
                 {"W", off(b.wf), (size_t)ne * 2 * MM * sizeof(double2), 256},
                 {"signs", off(b.sgn), (size_t)ne * 2 * M * sizeof(double), 256},
                 {"doublings", off(b.iters), (size_t)ne * 2 * sizeof(int), 256},
                 {"heavy", off(b.nheavy), (size_t)ne * 2 * sizeof(int), 256},
                 {"decimation ws", off(b.dscr), (size_t)b.gdec * qtx::dec_ws_elems(M) * sizeof(double2), 256},
                 {"sweep ws", off(b.sws), (size_t)b.grid * b.wsb, 256},
                 {"partials", off(b.part), (size_t)b.grid * 4 * 2 * N * (mixed ? 2 : 1) * sizeof(double), 256},
                 {"redo", mixed ? off(b.redo) : 0, mixed ? (size_t)ne * sizeof(int) : 0, 256},
                 {"elist", mixed ? off(b.elist) : 0, mixed ? (size_t)ne * sizeof(int) : 0, 256},
                 {"ecount", mixed ? off(b.ecount) : 0, mixed ? sizeof(int) : 0, 256}});
          if (err.empty() && (b.grid < 1 || b.gdec < 1 || ne < 1 || b.grid > ne || b.wsb != qtx::sweep_ws_bytes(N, M, mixed)))
            err = "noalloc: inconsistent grid or chunk";
        }
  const std::string out = err.empty() ? "ok: " + std::to_string(nsweep) + " sweep, " + std::to_string(ndec) +
                                            " decimation, " + std::to_string(nplan) + " no-allocation layouts"
                                      : err;
  if (msg && len > 0) {
    std::strncpy(msg, out.c_str(), (size_t)len - 1);
    msg[len - 1] = '\0';
  }
  return err.empty() ? 0 : 1;
}

qtx_status qtx_bands(qtx_ctx* c, qtx_side side, const double* k, int nk, double* E) {
  if (!c) return QTX_EINVAL;
  if (side != QTX_LEFT && side != QTX_RIGHT) return fail(c, QTX_EINVAL, "side must be QTX_LEFT or QTX_RIGHT");
  if (nk < 0) return fail(c, QTX_EINVAL, "nk must be >= 0");
  if (!c->lead_set[side]) return fail(c, QTX_ESTATE, "the lead must be set first");
  if (nk == 0) return QTX_OK;
  if (!k || !E) return fail(c, QTX_EINVAL, "k and E must not be NULL");
  for (int q = 0; q < nk; ++q)
    if (!std::isfinite(k[q])) return fail(c, QTX_EINVAL, "k must be finite");
  QTX_HIP(c, hipSetDevice(c->device));
  const int M = c->M, m = c->m;
  const int grid = std::max(1, std::min(nk, c->num_cu));
  QTX_HIP(c, c->wE.ensure((size_t)nk * sizeof(double)));
  QTX_HIP(c, c->wT.ensure((size_t)nk * m * sizeof(double)));
  if (M > 64) QTX_HIP(c, c->dscr.ensure((size_t)grid * 2 * M * (M + 1) * sizeof(double2)));
  QTX_HIP(c, hipMemcpyAsync(c->wE.p, k, (size_t)nk * sizeof(double), hipMemcpyHostToDevice, c->stream));
  QTX_HIP(c, qtx::run_bands(M, c->dlead[side].as<double2>(), m, c->Vlead[side], c->wE.as<double>(), nk,
                            M > 64 ? c->dscr.as<double2>() : nullptr, grid, c->wT.as<double>(), c->stream));
  QTX_HIP(c, hipMemcpyAsync(E, c->wT.p, (size_t)nk * m * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  QTX_HIP(c, hipStreamSynchronize(c->stream));
  for (size_t i = 0; i < (size_t)nk * m; ++i)
    if (!std::isfinite(E[i])) return fail(c, QTX_ENOTCONV, "non-finite band energy (S(k) not positive definite?)");
  return QTX_OK;
}

qtx_status qtx_sigma_cache_stats(qtx_ctx* c, long long* hits, long long* misses, long long* slots) {
  if (!c) return QTX_EINVAL;
  long long used = 0;
  for (auto& kv : c->sigcache) used += (long long)kv.second.index.size();
  if (hits) *hits = c->cache_hits;
  if (misses) *misses = c->cache_misses;
  if (slots) *slots = used;
  return QTX_OK;
}

qtx_status qtx_charge(const double* ldos, const double* w, int nE, int N, const double* E, double muL, double muR,
                      double kT, double* charge) {
  if (!ldos || !w || !E || !charge || nE < 0 || N < 1 || !(kT > 0.0)) return QTX_EINVAL;
  for (int i = 0; i < N; ++i) charge[i] = 0.0;
  for (int k = 0; k < nE; ++k) {
    const double fL = 1.0 / (1.0 + std::exp((E[k] - muL) / kT));
    const double fR = 1.0 / (1.0 + std::exp((E[k] - muR) / kT));
    for (int i = 0; i < N; ++i)
      charge[i] += w[k] * (fL * ldos[((size_t)k * 2 + 0) * N + i] + fR * ldos[((size_t)k * 2 + 1) * N + i]);
  }
  return QTX_OK;
}

}  // extern "C"
