/*
 * qtx.h — C ABI of the open-boundary ballistic transport solver for MI355X.
 *
 * The library solves, independently for every energy E of a grid,
 *
 *     (z S - H - H_ext - Sigma_L(z) - Sigma_R(z)) psi = b,   z = E + i eta,
 *
 * for a device of N slabs whose Hamiltonian H and overlap S are block
 * tridiagonal with m x m blocks (partition-of-unity basis: linear shape
 * functions along transport times Bloch-wave enhancement functions; Sec.
 * "Matrix equations", eqs. expansion_matrix_eq and infinite_system), with
 * semi-infinite leads on both sides folded into the self-energies
 * Sigma_L, Sigma_R (Sec. "Contact self-energies"), and returns the
 * transmission T(E) (Sec. "Transmission and Ballistic Current") and the
 * slab-resolved density of states injected from each contact (the node
 * density of Sec. "Density").
 *
 * Conventions (all calls):
 *  - complex numbers are interleaved (re, im) doubles, i.e. numpy complex128;
 *  - every m x m block is row-major; the blocks of slab i are contiguous;
 *  - H01 / S01 couple slab j to slab j+1; the coupling back is their
 *    conjugate transpose; for a lead at potential energy V the shifted
 *    energy is z - V;
 *  - units: eV for energies and potentials, hbar = 1, one slab per length
 *    unit, spin degeneracy 2 included in the densities;
 *  - all host pointers are owned by the caller and only read (or written,
 *    for outputs) during the call; the library copies what it keeps;
 *  - errors are returned as status codes; qtx_last_error() gives a
 *    per-context message; no exception crosses the ABI;
 *  - a context is not thread-safe: use one context per host thread.
 */
#ifndef QTX_H
#define QTX_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qtx_ctx qtx_ctx;

typedef struct { double re, im; } qtx_c128;

typedef enum {
  QTX_OK = 0,
  QTX_EINVAL = 1,     /* bad argument: NULL pointer, size, non-Hermitian block, unset state */
  QTX_ENOMEM = 2,     /* device or host allocation failed */
  QTX_EDEVICE = 3,    /* a HIP runtime call failed */
  QTX_ENOTCONV = 4,   /* outputs written, but some energy did not converge (see qtx_info.flags) */
  QTX_ESTATE = 5      /* call out of order (e.g. solve before set_lead / set_device) */
} qtx_status;

typedef enum { QTX_LEFT = 0, QTX_RIGHT = 1 } qtx_side;

/* How the nodal potential V_i enters H_ext (Sec. "Matrix equations",
 * extrinsic-potential matrix elements):
 *  QTX_POT_DIAG:      H_ext = diag_i(V_i S_ii);
 *  QTX_POT_LINEAR_FE: V linear between nodes; blocks weighted by the hat
 *                     functions: Vd_i = 3/4 V_i + (V_{i-1} + V_{i+1}) / 8 on
 *                     S_ii and Vu_i = (V_i + V_{i+1}) / 2 on S_{i,i+1},
 *                     with V_{-1} = V_L and V_N = V_R (the lead potentials). */
typedef enum { QTX_POT_DIAG = 0, QTX_POT_LINEAR_FE = 1 } qtx_pot_mode;

/* QTX_FP64: every step in double precision.
 * QTX_MIXED: lead self-energies, residuals and refinement in double; the
 *            block sweeps in single precision with double-precision
 *            iterative refinement of the dominant injected columns. */
typedef enum { QTX_FP64 = 0, QTX_MIXED = 1 } qtx_precision;

/* Per-energy diagnostics. */
typedef struct {
  int dec_iters;        /* decimation doublings used (max over the two leads) */
  int refine_steps;     /* refinement steps (QTX_MIXED), 0 otherwise */
  double resid;         /* final relative residual of the refined columns (QTX_MIXED) */
  int fell_back_fp64;   /* 1 if the energy was re-solved in FP64 */
  int flags;            /* bit 0: decimation hit its iteration cap;
                           bit 1: non-finite output; bit 2: refinement did not converge */
} qtx_info;

#define QTX_FLAG_DEC_NOTCONV 1
#define QTX_FLAG_NONFINITE 2
#define QTX_FLAG_REFINE_NOTCONV 4

/* Create a context on HIP device `hip_device`.  *out receives the handle.
 * Returns QTX_EINVAL for a NULL out or a bad device index, QTX_EDEVICE if
 * the HIP runtime fails. */
qtx_status qtx_create(int hip_device, qtx_ctx** out);

/* Free a context and all device memory it owns.  NULL is ignored. */
void qtx_destroy(qtx_ctx* ctx);

/* Last error message of the context ("" if none); valid until the next
 * call on the same context.  A NULL context gives a static string. */
const char* qtx_last_error(const qtx_ctx* ctx);

/* Stream on which qtx_solve_device enqueues its work (a hipStream_t; a
 * torch.cuda.Stream's cuda_stream handle works).  NULL selects the
 * library's own stream.  The caller keeps ownership of the stream. */
qtx_status qtx_set_stream(qtx_ctx* ctx, void* hip_stream);

/* Lead blocks of one contact (Sec. "Contact self-energies": the blocks of
 * eq. infinite_system just outside the simulation domain).  H00, S00: m x m
 * on-site blocks, Hermitian to 1e-12 relative (else QTX_EINVAL); H01, S01:
 * coupling from lead slab j to slab j+1 along +z (the same orientation for
 * both leads).  V_lead: potential energy of the
 * lead (eV).  The blocks are deep-copied to the device.  m must agree with
 * the other lead and the device, 1 <= m <= 128. */
qtx_status qtx_set_lead(qtx_ctx* ctx, qtx_side side, int m,
                        const qtx_c128* H00, const qtx_c128* H01,
                        const qtx_c128* S00, const qtx_c128* S01, double V_lead);

/* Device blocks (eq. infinite_system restricted to N slabs).  Hd, Sd: N
 * on-site m x m blocks (N*m*m, Hermitian); Hu, Su: N-1 couplings slab i ->
 * i+1 ((N-1)*m*m).  All four NULL: every slab copies the LEFT lead's blocks
 * (set the left lead first).  Either all four or none must be given.
 * N >= 1.  Deep-copied. */
qtx_status qtx_set_device(qtx_ctx* ctx, int N, int m,
                          const qtx_c128* Hd, const qtx_c128* Hu,
                          const qtx_c128* Sd, const qtx_c128* Su);

/* Nodal potential energy V[0..N-1] (eV) and how it is projected (see
 * qtx_pot_mode).  Must follow qtx_set_device (same N).  Deep-copied. */
qtx_status qtx_set_potential(qtx_ctx* ctx, const double* V, qtx_pot_mode mode);

/* Solve an energy grid (host buffers, synchronous).
 * E[nE]: energies (eV); eta > 0: broadening added to every energy in the
 * leads and the device.  Outputs (caller-allocated host memory):
 *   T[nE]            transmission left -> right,
 *                    T = Re Tr[Gamma_R G_{N-1,0} Gamma_L G_{N-1,0}^H];
 *   ldos[nE*2*N]     or NULL; ldos[(e*2 + s)*N + i] = (1/pi) Re sum over
 *                    slab i of diag(G Gamma_s G^H), s = 0 left-, 1 right-
 *                    injected (states / eV / slab, spin 2);
 *   info[nE]         or NULL; per-energy diagnostics.
 * Returns QTX_OK, QTX_ENOTCONV (outputs written, some energy flagged), or
 * an error code (outputs undefined). */
qtx_status qtx_solve(qtx_ctx* ctx, const double* E, int nE, double eta,
                     qtx_precision prec, double* T, double* ldos, qtx_info* info);

/* Same as qtx_solve with DEVICE pointers (e.g. torch tensors' data_ptr()),
 * enqueued on the context stream without a host synchronisation.  info_dev
 * may be NULL; the other outputs as in qtx_solve.  The buffers must stay
 * alive until the stream has executed the work.  Per-energy convergence is
 * reported through info_dev only (the return value does not wait for it).
 * The call may be captured in a HIP graph on the context stream once an
 * earlier call with at least as many energies, the same precision and the
 * same method has sized the context's workspaces.  It then issues only
 * kernel launches; a replay reads the energies at E_dev and recomputes
 * everything.  A context with several captured graphs shares one workspace
 * among them, so their replays must not overlap.  A captured graph holds
 * the workspace addresses of the moment of capture: any later call on the
 * context that grows or releases a workspace (a larger energy grid or
 * slab count, another precision, qtx_autotune, qtx_density_matrix, the
 * options sweep_workspace_bytes or energies_per_launch) leaves the graph
 * pointing at freed memory, and it must be captured again before its next
 * replay. */
qtx_status qtx_solve_device(qtx_ctx* ctx, const double* E_dev, int nE, double eta,
                            qtx_precision prec, double* T_dev, double* ldos_dev,
                            qtx_info* info_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as qtx_solve_device, same arguments, same results bit for bit, but
 * it allocates nothing.  Every buffer of the solve (self-energies,
 * broadening factors, decimation and sweep workspaces, partial sums,
 * re-solve lists) is carved from a fixed device array of 512 MiB
 * (QTX_NOALLOC_SCRATCH_BYTES) that the library holds on each GPU it runs
 * on until the process ends.  The energies run in chunks with as many
 * resident workgroups as that array holds, so large problems run with
 * fewer workgroups than qtx_solve_device (slower, same results).  Returns
 * QTX_ENOMEM with a message when not even one energy of the problem fits
 * (at N = 200, m = 64 one energy needs about 27 MB in FP64).  Only the
 * decimation self-energies (self_energy_method 0); no kernel timing.
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (two streams, two contexts, two
 * threads) race and must be serialised by the caller.  Nothing in the
 * array needs to start at zero.  Asynchronous on the context stream like
 * qtx_solve_device. */
#define QTX_NOALLOC_SCRATCH_BYTES (512ull << 20)
qtx_status qtx_solve_device_noalloc(qtx_ctx* ctx, const double* E_dev, int nE, double eta,
                                    qtx_precision prec, double* T_dev, double* ldos_dev,
                                    qtx_info* info_dev);

/* Nearest-neighbour blocks of the density matrix in the slab basis (the
 * Bloch-basis density matrix of Sec. "Density", eq. density_matrices, whose
 * on-slab and neighbouring-slab blocks suffice for the density,
 * eq. density_3d_fast), accumulated over an energy grid with per-contact
 * weights:
 *   rho_ij = sum_e (1/pi) [wL[e] G_{i,0} Gamma_L G_{j,0}^H
 *                          + wR[e] G_{i,N-1} Gamma_R G_{j,N-1}^H]   at E[e],
 * i.e. the FP64 solution psi of each injecting contact weighted column by
 * column.  wL[e], wR[e] carry the quadrature weight times the occupation of
 * the contact (e.g. Simpson weight times f(E - mu)); any finite values.
 * The paper's n_{i'n'k',ink} is rho with its index pairs exchanged
 * (n[i' a][i b] = rho_{i i'}[b][a]); rho is Hermitian as a whole:
 * rho_{i+1,i} = rho_{i,i+1}^H.
 * Host buffers, row-major m x m blocks, caller-allocated:
 *   rho_diag[N*m*m]       rho_ii, i = 0..N-1;
 *   rho_off[(N-1)*m*m]    rho_{i,i+1}, i = 0..N-2 (may be NULL when N = 1);
 *   T[nE], ldos[nE*2*N], info[nE]: as in qtx_solve (each may be NULL).
 * The sum over energies is formed in a fixed order for a given grid, block
 * size and option set.  Device memory: one accumulator of (2N-1) M^2 complex
 * doubles per resident workgroup (M the padded block), at most option
 * "density_matrix_bytes" (default 64 GiB) in total; QTX_ENOMEM if not even
 * one fits.  nE = 0 zeroes the outputs.  Returns QTX_OK, QTX_ENOTCONV
 * (outputs written, some energy flagged) or an error code.  Synchronous. */
qtx_status qtx_density_matrix(qtx_ctx* ctx, const double* E, const double* wL, const double* wR,
                              int nE, double eta, qtx_c128* rho_diag, qtx_c128* rho_off,
                              double* T, double* ldos, qtx_info* info);

/* Same as qtx_density_matrix with DEVICE pointers, enqueued on the context
 * stream without a host synchronisation: E_dev, wL_dev, wR_dev [nE];
 * rho_diag_dev, rho_off_dev as rho_diag, rho_off; T_dev [nE] required,
 * ldos_dev and info_dev may be NULL.  Weights are not checked on the host
 * (a non-finite weight gives non-finite blocks).  Per-energy convergence is
 * reported through info_dev only.  The buffers must stay alive until the
 * stream has executed the work. */
qtx_status qtx_density_matrix_device(qtx_ctx* ctx, const double* E_dev, const double* wL_dev,
                                     const double* wR_dev, int nE, double eta,
                                     qtx_c128* rho_diag_dev, qtx_c128* rho_off_dev,
                                     double* T_dev, double* ldos_dev, qtx_info* info_dev);

/* Self-energies and broadening factors alone (the decimation step of the
 * solve, or the complex band structure with option self_energy_method 1;
 * exposed for verification).  Host buffers:
 *   sigma[nE*2*m*m]  Sigma_L then Sigma_R per energy (row-major, m x m);
 *   wfac[nE*2*m*m]   or NULL: W with Gamma = W diag(sgn) W^H per side
 *                    (method 1: the flux-normalised injection of the
 *                    incoming travelling modes, one per column);
 *   sgn[nE*2*m]      or NULL: the signs (+1, -1, or 0 for unused columns);
 *   iters[nE]        or NULL: doublings used (method 1: QR iterations). */
qtx_status qtx_self_energy(qtx_ctx* ctx, const double* E, int nE, double eta,
                           qtx_c128* sigma, qtx_c128* wfac, double* sgn, int* iters);

/* Tuning parameters of a context (problems created from it start with the
 * same values).  name / accepted values / default:
 *   "decimation_tol"        (0, 1)        1e-14  doubling stops when the
 *                           couplings fall below this times |D0|;
 *   "decimation_refine_cond" [0, inf]     1e4    a doubling refines its
 *                           solve with e once (X += e^-1 ([a|b] - e X))
 *                           when ||e||_F ||e^-1||_F exceeds this; 0 refines
 *                           every doubling, inf none;
 *   "decimation_max_iters"  [1, 1000]     60     doublings before
 *                           QTX_FLAG_DEC_NOTCONV;
 *   "sigma_newton_tol"      [-1, 1)       3e-11  after the doublings every
 *                           self-energy is checked against its fixed point
 *                           Sigma = A (D0 - Sigma)^-1 B (A = U, B = L for
 *                           the right contact, A = L, B = U for the left);
 *                           where the residual exceeds this times max|Sigma|
 *                           (near the lead's band edges) one Newton step
 *                           corrects it, its linear (Stein) equation summed
 *                           by doubling; 0 corrects every self-energy, a
 *                           negative value none;
 *   "refine_tol"            (0, 1)        3e-11  QTX_MIXED: refinement stops
 *                           when ||r||_F <= refine_tol ||b||_F over the
 *                           refined columns;
 *   "refine_max_steps"      [0, 20]       3      QTX_MIXED: corrections before
 *                           the energy is re-solved in FP64 (earlier when a
 *                           correction does not halve the residual, or when
 *                           the contraction seen so far cannot reach
 *                           refine_tol in the corrections left);
 *   "refine_weight_tol"     [0, 1]        0      QTX_MIXED: columns of the
 *                           broadening factor whose LDL^H pivot is at least
 *                           this times the largest are refined (whole tiles
 *                           of 16 columns, at least one tile per contact);
 *                           0 refines every column (the light columns keep
 *                           single-precision densities otherwise, which near
 *                           resonances miss 1e-8 relative);
 *   "workgroups_per_cu"     [1, 4]        2      resident energies per CU for
 *                           blocks up to 64 (blocks of 96 and 128 use two
 *                           with QTX_FP64, one with QTX_MIXED, and their lead
 *                           decimation two with either); setting it
 *                           discards autotuned values;
 *   "panel_width"           0, 16 or 32   0      columns of a Gauss-Jordan panel
 *                           in the sweeps' block inverse; 0 takes 16 up to
 *                           padded blocks of 64 and 32 above; a width that
 *                           does not divide the padded block falls back to
 *                           that default.  It changes the order of the
 *                           floating-point operations (results agree to
 *                           rounding); setting it discards autotuned values;
 *   "refine_tiles"          0, 1 or 2     0      QTX_MIXED: 16-column tiles a
 *                           wave carries at once through the refinement at
 *                           padded blocks 48 and 64 (0: 2; other blocks have
 *                           one value); results do not change; setting it
 *                           discards autotuned values;
 *   "energies_per_launch"   [1, 2^20]     4096   energies per launch chunk;
 *   "sigma_cache_bytes"     [0, 1e13]     16 GiB qtx_solve_batch keeps the lead
 *                           self-energies, broadening factors and signs of
 *                           every (lead blocks, E - V_lead) it has solved, up
 *                           to this many bytes of device memory per block
 *                           size, and reuses them (when full, entries are
 *                           replaced oldest first, never one the current
 *                           call uses); 0 disables the cache.  Changing eta
 *                           or a decimation option empties it;
 *   "self_energy_method"    0 or 1        0      how the lead self-energies
 *                           and the injection are obtained: 0 by decimation
 *                           at z = E + i eta with the full broadening
 *                           injected; 1 from the complex band structure of
 *                           each lead (the direct method of Sec. "Contact
 *                           self-energies": eq. linearized_eigenvalue_symmetric,
 *                           the Hellmann-Feynman split, Sigma = [H' - E M']
 *                           B Lambda B^-1) with only the incoming travelling
 *                           modes injected, flux-normalised (eq. qtbm_system,
 *                           the paper's mode-space QTBM).  Method 1 solves at
 *                           eta = 0 exactly (other eta: QTX_EINVAL), with
 *                           QTX_FP64 (QTX_MIXED: QTX_EINVAL), for qtx_solve,
 *                           qtx_solve_device, qtx_self_energy and
 *                           qtx_density_matrix; qtx_solve_batch rejects it.
 *                           Couplings H01 - E S01 of lower rank than the
 *                           slab (the paper's symmetric pencil is then
 *                           singular) are handled by solving the quadratic
 *                           in a shifted variable nu, lambda = (nu + s) /
 *                           (1 + conj(s) nu), |s| < 1, which keeps the mode
 *                           vectors and the unit circle; an energy whose
 *                           modes cannot be split m / m is flagged
 *                           QTX_FLAG_DEC_NOTCONV.  qtx_info.dec_iters then
 *                           counts QR iterations;
 *   "mode_tol"              (0, 1e-2]     1e-8   method 1: modes with
 *                           ||lambda| - 1| <= mode_tol travel;
 *   "sweep_workspace_bytes" (0, 1e13]     160 GiB device memory for the
 *                           sweep workspaces of the resident workgroups
 *                           ((N + 1) 2 M^2 complex per workgroup in FP64):
 *                           fewer workgroups run when they do not all fit,
 *                           with the same results.  When the device runs
 *                           out of memory for them, the context halves its
 *                           budget until they fit and keeps the lowered
 *                           value until this option is set again.  A call
 *                           whose single workgroup does not fit returns
 *                           QTX_ENOMEM;
 *   "density_matrix_bytes"  [0, 1e13]     64 GiB device memory for the
 *                           per-workgroup accumulators of qtx_density_matrix
 *                           (fewer workgroups run when they do not all fit);
 *   "use_graph"             0 or 1        1      qtx_solve_batch captures its
 *                           launch sequence in a HIP graph and replays it
 *                           while the batch shape is unchanged.
 * Integer options take an integral value.  QTX_EINVAL for an unknown name
 * or a value out of range (the setting is then unchanged). */
qtx_status qtx_set_option(qtx_ctx* ctx, const char* name, double value);

/* Band structure of one lead: the eigenvalues of the Bloch problem
 * H(k) c = E S(k) c with H(k) = H00 + e^{ik} H01 + e^{-ik} H01^H and S(k)
 * likewise (Bloch's theorem applied to the slab equations of eq.
 * infinite_system; the band-structure reconstruction of Sec. "Electronic
 * Structure").  k[nk]: Bloch phases (radians per slab).  E[nk*m] (host,
 * caller-owned): E[q*m + n] = E_n(k_q) + V_lead, ascending in n, FP64.
 * One GPU workgroup per k point.  QTX_ESTATE before qtx_set_lead(side),
 * QTX_ENOTCONV if an energy came out non-finite (S(k) not positive
 * definite).  Synchronous. */
qtx_status qtx_bands(qtx_ctx* ctx, qtx_side side, const double* k, int nk, double* E);

/* ---- batching and serving --------------------------------------------- */

/* A problem is a context that shares the parent's device and stream and
 * carries its own leads, device blocks and potential (same setters). */
qtx_status qtx_problem_create(qtx_ctx* parent, qtx_ctx** problem);

/* Solve nprob problems, each on its own energy grid E[p][0..nE[p]-1], as
 * one batch: the (problem, energy) items of all problems with the same
 * padded block size share one decimation and one sweep launch (devices of
 * different N in the same launch, longest first), and the whole launch
 * sequence is replayed from a HIP graph while the batch shape (problems,
 * their N and m, the nE[p], eta, precision, options) is unchanged.
 * T[p] (nE[p]) and ldos[p] (nE[p]*2*N_p, or NULL) are host buffers;
 * results are the same as qtx_solve on each problem alone.  Problems must
 * be fully set and live on ctx's device.  Synchronous. */
qtx_status qtx_solve_batch(qtx_ctx* ctx, int nprob, qtx_ctx* const* probs,
                           const double* const* E, const int* nE, double eta,
                           qtx_precision prec, double* const* T, double* const* ldos);

/* Launch configuration of the sweep kernels for one padded block size and
 * precision: the autotuner's choice (qtx_autotune). */
typedef struct {
  int workgroups_per_cu;  /* resident energies per CU, 1..4 */
  int panel_width;        /* columns of a Gauss-Jordan panel of the block
                             inverse, 16 or 32 (dividing the padded block) */
  int refine_tiles;       /* QTX_MIXED: 16-column tiles a wave carries at
                             once through the refinement, 1 or 2 at padded
                             blocks 48 and 64 (fixed otherwise) */
} qtx_tune;

#define QTX_TUNE_MAX_CANDIDATES 16

/* Autotuning of the sweep's launch shape and tile shapes for the context's
 * problem (the block elimination of Sec. "Extended states", eq.
 * qtbm_system, as block sweeps).  Candidates: every built combination of
 * panel width and refinement tiles at this block size, each with every
 * number of resident workgroups per CU from 1 to 4 that its register and
 * LDS use allow (mixed sweeps of blocks above 64: one).  Each candidate
 * solves the sample energies E[nE] (host, eta, prec) once to warm up and
 * three times timed with HIP events; the median decides.  The fastest is
 * stored for this block size and precision in the context (and in its
 * parent, for batched solves) and used by later solves.  The workgroup
 * count and the refinement tiles never change a result; the panel width
 * changes the rounding of the block inverses (results agree to the
 * parity tolerances).  *best (or NULL) receives it; cand[] and times_ms[] (each
 * QTX_TUNE_MAX_CANDIDATES long, or NULL) every candidate and its median
 * milliseconds, *ncand (or NULL) their count.  Takes about four times the
 * sample's solve time per candidate.  The sweep and decimation workspaces
 * the timing allocated are released on return; the next solve on the
 * context allocates what it needs. */
qtx_status qtx_autotune(qtx_ctx* ctx, const double* E, int nE, double eta, qtx_precision prec,
                        qtx_tune* best, qtx_tune* cand, double* times_ms, int* ncand);

/* Self-energy cache of qtx_solve_batch (option "sigma_cache_bytes"):
 * contact lookups that found their entry (hits) and that had to run the
 * decimation (misses) since the context was created, and the entries now
 * held.  Each may be NULL.  For callers that serve many requests on the
 * same leads and energy lattice. */
qtx_status qtx_sigma_cache_stats(qtx_ctx* ctx, long long* hits, long long* misses, long long* slots);

/* Host helper: slab charge from a solved grid with quadrature weights w:
 * charge[i] = sum_k w[k] (f((E_k - muL)/kT) ldos[k][0][i]
 *                        + f((E_k - muR)/kT) ldos[k][1][i]),
 * f the Fermi function (the energy integral of the node density, Sec.
 * "Density").  kT > 0. */
qtx_status qtx_charge(const double* ldos, const double* w, int nE, int N, const double* E,
                      double muL, double muR, double kT, double* charge);

/* Per-kernel device time of the solves since the last call (ms), from HIP
 * events recorded on the context stream around every decimation and
 * sweep launch while recording is enabled.  enable = 1 starts recording
 * (and clears the totals), 0 stops it; the outputs (each may be NULL)
 * receive the totals and the number of sweep launches accumulated before
 * this call.  Synchronises the context stream. */
qtx_status qtx_kernel_times(qtx_ctx* ctx, int enable, double* decimate_ms, double* sweep_ms, int* launches);

/* Library version string. */
const char* qtx_version(void);

/* Self-check of the library's memory layouts, host arithmetic only (no
 * device needed): every sweep workspace (block sizes 16..128, FP64, mixed,
 * density-matrix, the FP64 re-solve inside the mixed workspace, items
 * shorter than the launch's longest), the decimation and Newton
 * workspaces, and the no-allocation layouts of several problems must keep
 * their regions aligned, inside their allocation and disjoint.  Returns 0
 * with the number of layouts checked in msg[len], or 1 with a description
 * of the first violation there (msg may be NULL). */
int qtx_check_layouts(char* msg, int len);

#ifdef __cplusplus
}
#endif
#endif
