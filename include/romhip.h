/*
 * romhip.h - C interface of the MI355X (gfx950) adaptive reduced-order-model
 * hot path: full-order finite-volume residuals, backward-Euler full-order steps,
 * the Brand incremental-SVD basis update with forgetting, hyper-reduction
 * rebuilds and reduced time steps, for a batch of independent instances.
 *
 * Method: history-aware adaptive ROM via incremental SVD (Hedayat, Mohaghegh,
 * Balzano, Huang, Duraisamy): Sec. 2 (full-order model), Sec. 3 (projection and
 * hyper-reduction), Sec. 4 (correction signal, iSVD update, Alg. 1 and Alg. 2).
 *
 * Conventions shared by every call
 *   Layout.  A batch holds n_inst independent instances.  Instance b has
 *     n_cells[b] cells with n_var variables per cell (1 Burgers, 3 Euler,
 *     12 reacting model).  State vectors are concatenated instance after
 *     instance; inside an instance they are cell-major (all variables of cell 0,
 *     then cell 1, ...): element (b, cell c, var v) sits at
 *     dof_off[b] + c*n_var + v, dof_off = prefix sum of n_cells*n_var.
 *     Bases are row-major per instance: row i (a degree of freedom) of the
 *     N_b x r basis of instance b sits at (dof_off[b] + i)*r .. +r-1.
 *   Precision.  cfg.precision selects the element type of every state/basis
 *     buffer that crosses this interface: ROM_F32 -> float, ROM_F64 -> double.
 *     Singular values, reduced coordinates, core SVD, pseudo-inverses and
 *     reduced solves are always double.
 *   Memory.  Every pointer documented "device" is caller-owned device memory
 *     (e.g. a torch tensor) that the library only borrows for the enqueued
 *     work; every pointer documented "host" is read before the call returns.
 *     The handle owns all memory reachable from it; rom_destroy frees it.
 *   Streams.  Every call enqueues its work on the given hipStream_t (NULL =
 *     the default stream) and returns without synchronising, except
 *     rom_get_status and the host-side rom_get of ROM_GET_COUNTERS.
 *   Errors.  Argument and state errors are detected on the host, returned as
 *     negative rom_status values, and leave the handle unchanged.  Conditions
 *     detected on the device (Newton not converged, floors, non-finite values,
 *     degenerate residual) set per-instance flag bits read by rom_get_status.
 *     rom_last_error() returns a thread-local message for the last error.
 *   Threading.  A handle is not thread-safe; distinct handles are independent.
 */
#ifndef ROMHIP_H
#define ROMHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rom_batch* rom_handle;

typedef enum {
  ROM_OK = 0,
  ROM_E_INVAL = -1,     /* bad argument: nothing enqueued, handle unchanged */
  ROM_E_NOMEM = -2,     /* device allocation failed */
  ROM_E_DEVICE = -3,    /* a HIP runtime call failed */
  ROM_E_STATE = -6,     /* call not valid in the handle's current state */
  ROM_E_UNSUPPORTED = -7
} rom_status;

/* per-instance device flag bits (rom_get_status) */
enum {
  ROM_FLAG_NEWTON_NOCONV = 1u << 0, /* a full-order Newton solve hit its cap */
  ROM_FLAG_FLOOR = 1u << 1,         /* density/pressure/temperature floor engaged */
  ROM_FLAG_NONFINITE = 1u << 2,     /* a non-finite value was produced */
  ROM_FLAG_RHO_ZERO = 1u << 3,      /* iSVD residual below tau_rho: rho := 0 */
  ROM_FLAG_SINGULAR = 1u << 4,      /* singular reduced or sampled matrix */
  ROM_FLAG_ROM_NOCONV = 1u << 5,    /* a reduced Newton / Gauss-Newton hit its cap */
  ROM_FLAG_REORTH = 1u << 6         /* basis re-orthonormalised at least once */
};

enum { ROM_BURGERS = 0, ROM_EULER_RUSANOV = 1, ROM_EULER_HLLC = 2, ROM_REACT = 3 };
enum { ROM_F32 = 0, ROM_F64 = 1 };
enum { ROM_GALERKIN = 0, ROM_LSPG = 1 };
enum { ROM_HR_NONE = 0, ROM_HR_DEIM = 1, ROM_HR_QDEIM = 2, ROM_HR_QDEIM_FGS = 3 };
enum { ROM_UPDATE_ISVD = 0, ROM_UPDATE_WSVD = 1, ROM_UPDATE_DIRECT = 2 };
enum { ROM_SCHEME_BE = 0, ROM_SCHEME_SSPRK43 = 1 };

/*
 * Batch configuration (Alg. 1 inputs: r, n_s, w_init, z, lambda; the time step
 * and the Newton settings of Sec. 5).
 *   phys: host, n_inst * n_phys doubles, instance-major:
 *     ROM_BURGERS              n_phys = 1: viscosity nu
 *     ROM_EULER_RUSANOV/HLLC   n_phys = 1: gamma
 *     ROM_REACT                n_phys = 88: nu_u, kappa, A, k_in, x_in, T_in,
 *                              Y_in[10], then for the 12 reactions the species
 *                              indices a[12], b[12], c[12], d[12] (as doubles),
 *                              activation energies E[12], heat releases Q[12]
 *   newton_tol: sup-norm tolerance of the full-order Newton residual
 *   rom_tol:    reduced Newton stops when max|delta| <= rom_tol (1 + max|a|)
 *   reorth_every / tau_orth: every reorth_every basis updates the Gram matrix
 *               G = Phi^T Phi is formed in FP64; if max|G - I| > tau_orth the
 *               basis is replaced by Phi L^-T (G = L L^T).  0 disables.
 *   tau_rho:    iSVD residual norm below tau_rho * ||y^|| is treated as zero
 *   use_graph:  rom_step captures each adaptation window (z fine steps plus the
 *               event) into a HIP graph on first use and replays it afterwards
 *               (iSVD rule only; the windowed rules run their windows eagerly,
 *               because the window's fill level is host state)
 *   update_rule: the basis update of an adaptation event:
 *               ROM_UPDATE_ISVD   Brand's incremental SVD (Alg. 2; the method)
 *               ROM_UPDATE_WSVD   windowed SVD: the leading r left singular
 *                                 vectors of the last `window` preprocessed
 *                                 correction snapshots (App. A, Alg. A.1)
 *               ROM_UPDATE_DIRECT the Direct rule (App. A, Alg. A.2):
 *                                 Z = Phi^T Y, Phi~ = Y Z^+, Phi <- orth(Phi~)
 *               The windowed rules keep the raw snapshots of a window of
 *               `window` columns (r <= window <= 64); it starts from the last
 *               min(window, w_init) training snapshots.  The state transfer is
 *               Alg. 1's a <- Phi_new^T D (q~ - q_ref), formed in FP64.
 *   scheme:     the time discretisation of the full and reduced models:
 *               ROM_SCHEME_BE      backward Euler on the first-order finite
 *                                  volume f (implicit; Secs. 5.1-5.2)
 *               ROM_SCHEME_SSPRK43 the explicit structure of the detonation
 *                                  case (Sec. 5.3, App. D): four-stage
 *                                  third-order SSP Runge-Kutta on the
 *                                  second-order f with Barth-Jespersen limited
 *                                  face states.  fom_step is one such step
 *                                  (the coarse correction one of size z dt),
 *                                  the fine step the DEIM-Galerkin ROM of eq.
 *                                  deim_galerkin_rom advanced by the same
 *                                  scheme.  Needs ROM_GALERKIN and a sampler
 *                                  (hyper != ROM_HR_NONE); newton_* and
 *                                  rom_* settings are unused; the adjoint
 *                                  entry points return ROM_E_UNSUPPORTED.
 */
typedef struct {
  int32_t problem, precision, projection, hyper;
  int32_t n_inst;
  const int64_t* n_cells; /* host [n_inst], each >= 3 */
  const double* phys;     /* host [n_inst * n_phys] */
  int32_t n_phys;
  int32_t r, n_s, w_init, z;
  int32_t newton_max, rom_max, reorth_every;
  int32_t use_graph;
  int32_t update_rule, window;
  int32_t scheme;
  double lambda, dt, newton_tol, rom_tol, tau_orth, tau_rho;
} rom_config;

/* quantities exchanged by rom_get / rom_set (element type and size) */
enum {
  ROM_GET_BASIS = 0,   /* T[total_dof * r]       Phi                         */
  ROM_GET_SIGMA = 1,   /* double[n_inst * r]     singular values             */
  ROM_GET_A = 2,       /* double[n_inst * r]     reduced coordinates a^n     */
  ROM_GET_QTILDE = 3,  /* T[total_dof]           q_ref + D^-1 Phi a (get only) */
  ROM_GET_SAMPLES = 4, /* int32[n_inst * n_s]    DEIM rows (instance-local DOF index, pick order) */
  ROM_GET_YCORR = 5,   /* T[total_dof]           coarse correction state     */
  ROM_GET_QREF = 6,    /* T[total_dof]           reference state             */
  ROM_GET_DVAR = 7,    /* double[n_inst * n_var] diagonal of D per variable  */
  ROM_GET_PINV = 8,    /* double[n_inst * r * n_s] (P^T Phi)^+ row-major     */
  ROM_GET_COUNTERS = 9, /* int64[6] host: fine step n, updates k, events, reorths,
                          window fill level, next window slot */
  ROM_GET_UBAR = 10,   /* double[n_inst * (r+1) * (r+1)] (get only) left singular vectors
                          of the last update's core K (eq. isvd_core_matrix), row-major,
                          columns in descending order of the singular values */
  ROM_GET_WINDOW = 11  /* T[window * total_dof] raw correction snapshots of the windowed
                          rules, slot j at j * total_dof (slots in storage order; the
                          fill level and next slot are in ROM_GET_COUNTERS) */
};

/*
 * rom_create - allocate a batch handle (layout, constants, workspaces) and, if
 * q0 is not NULL, run the offline part of Alg. 1 on the device: w_init fine
 * backward-Euler steps from q0, preprocessing (q_ref = q0, D from the mean
 * square of the centred training data, Sec. 3.1 eq. variable_normalization),
 * POD to rank r, a = Phi^T D (q^{w_init} - q_ref), the first coarse step
 * y_corr (eq. coarse_fom_backward_euler), and the first sampling / rebuild.
 *   q0: device, T[total_dof] or NULL (then only fom_* calls and rom_set are
 *       valid until the reduced state is loaded).
 *   Errors: ROM_E_INVAL for inconsistent settings (r < 1, r > min N_b,
 *   n_s outside [r, 2r] with DEIM, z < 1, lambda outside [0, 1], ...).
 */
rom_status rom_create(const rom_config* cfg, const void* q0, void* stream, rom_handle* out);
rom_status rom_destroy(rom_handle h);

/*
 * fom_residual - full-order residual for every instance in one launch.
 *   q_prev == NULL: out = f(q)                       (Sec. 2 eq. fom_continuous)
 *   otherwise:      out = q - q_prev - dt f(q)       (backward-Euler residual,
 *                                                    eq. be_residual_rom_section)
 *   With ROM_SCHEME_SSPRK43, f is the limited second-order f and q_prev must
 *   be NULL (ROM_E_INVAL otherwise).
 *   q, q_prev, out: device, T[total_dof]; out must not alias q or q_prev.
 */
rom_status fom_residual(rom_handle h, const void* q, const void* q_prev, double dt, void* out,
                        void* stream);

/*
 * fom_step - one backward-Euler full-order step of size dt for every instance:
 * Newton on q - q_prev - dt f(q) = 0 from q = q_prev with the exact banded
 * Jacobian and a direct block-tridiagonal solve; stops per instance when
 * max|r| <= newton_tol, at most newton_max solves (Sec. 5.1 setup; App. B).
 * With ROM_SCHEME_SSPRK43 it is one SSPRK(4,3) step of the limited
 * second-order model (App. D): four evaluations of f, the stage combinations
 * formed in FP64.
 *   q_prev, q_out: device, T[total_dof]; may alias.
 *   iters (optional): device int32[n_inst], Newton solves used per instance
 *   (4, the stage count, on the explicit path).
 */
rom_status fom_step(rom_handle h, const void* q_prev, double dt, void* q_out, int32_t* iters,
                    void* stream);

/*
 * isvd_update - one iSVD basis update per instance (Alg. 2), with the
 * snapshot preprocessed inside: y^ = D (y - q_ref).  p and the residual by two
 * classical Gram-Schmidt passes (eq. isvd_residual), core K (eq.
 * isvd_core_matrix) decomposed in FP64, basis rotated and truncated to r
 * (eqs. isvd_updated_basis_full, isvd_truncation).  The reduced coordinates a
 * are carried to the new basis (Alg. 1 state transfer, in the exact closed
 * form a <- Ubar[:r,:r]^T a) and the re-orthonormalisation schedule runs.
 *   y: device, T[total_dof].
 */
rom_status isvd_update(rom_handle h, const void* y, void* stream);

/*
 * rom_rebuild - refresh every basis-dependent quantity (Alg. 1 sampling and
 * operator update; eq. qdeim_approximation_phi): the sample rows, the sample
 * mesh (the sampled cells and their two neighbours), the gathered basis /
 * q_ref rows and (P^T Phi)^+ in FP64.  The rows come from cfg.hyper:
 *   ROM_HR_DEIM       greedy DEIM, n_s = r .. 2r (two rounds, Sec. 3.2)
 *   ROM_HR_QDEIM      QDEIM, n_s = r: the pivots of the column-pivoted QR of
 *                     Phi^T (eq. qdeim_qr); ties go to the lowest row
 *   ROM_HR_QDEIM_FGS  QDEIM's r rows, then feature-guided sampling (eq.
 *                     fgs_selection): the n_s - r cells (r < n_s <= 2r) of
 *                     largest squared centred-difference gradient of a
 *                     feature of y_corr (Burgers u, Euler density, reacting
 *                     model temperature), each adding its feature row; cells
 *                     whose feature row is already chosen are skipped
 * All three use the hyper-reduced LSPG step.
 */
rom_status rom_rebuild(rom_handle h, void* stream);

/*
 * rom_step - advance the online loop of Alg. 1 by n_fine fine steps: each step
 * solves the reduced backward-Euler system (Galerkin: eq.
 * galerkin_continuous_rom; hyper-reduced LSPG: eq.
 * hyperreduced_lspg_stationarity) by Newton / Gauss-Newton with FP64 reduced
 * solves, and every z steps runs an adaptation event: coarse full-order step
 * of y_corr with step z dt, iSVD update, rebuild, state transfer.
 */
rom_status rom_step(rom_handle h, int32_t n_fine, void* stream);

/* copy a handle quantity to (get) or from (set) caller device memory; see ROM_GET_* */
rom_status rom_get(rom_handle h, int32_t what, void* dst, void* stream);
rom_status rom_set(rom_handle h, int32_t what, const void* src, void* stream);

/*
 * rom_save / rom_load - the whole state the online loop of Alg. 1 carries from
 * one fine step to the next, so that a run can stop and resume (or fork) with
 * the same bits: the basis Phi, sigma, the reduced coordinates a, the
 * correction state y_corr (Alg. 1 keeps it between events), q_ref, the
 * diagonal of D, the flag words, the sample rows P and (P^T Phi)^+, and the
 * host counters (fine step n, updates, events, re-orthonormalisations).
 * With a windowed update rule the snapshot window and its fill level and
 * next slot are part of the state too.
 * Format: a 256-byte header of 32 int64 words (magic "ROMHIPS1", version,
 * problem, precision, n_inst, total_dof, r, n_s, n_var, a hash of the
 * instance sizes, the four counters, total bytes, hyper, update rule, window,
 * window fill level, next window slot, then zeros), then the sections in the
 * order above and the window last, each on a 256-byte boundary, in the
 * handle's element types.
 *
 * rom_save(h, dst, &bytes, stream): dst == NULL only stores the size needed in
 *   *bytes.  Otherwise dst is caller-owned device memory of at least *bytes
 *   (8-byte aligned); the copies are enqueued on stream (kernels only, no
 *   synchronisation) and *bytes receives the size written.
 *   Errors: ROM_E_INVAL (NULL handle or bytes, dst too small or misaligned),
 *   ROM_E_STATE (no reduced state).
 * rom_load(h, src, bytes, stream): src is device memory written by rom_save
 *   for a handle of the same configuration and instance sizes.  The call
 *   synchronises the stream, reads and checks the header, then enqueues the
 *   copies and, with DEIM, a rebuild from the restored basis (the sample mesh
 *   and the column-major basis copy are derived data; the rebuild recomputes
 *   them with the same kernels, so P and (P^T Phi)^+ come back bit for bit).
 *   Window graphs captured earlier are discarded.  A handle created with
 *   q0 == NULL becomes usable for rom_step after a load.
 *   Errors: ROM_E_INVAL (NULL arguments, bytes too small, misaligned, not a
 *   saved state of this version, or a different configuration or layout):
 *   the handle is left unchanged.
 */
rom_status rom_save(rom_handle h, void* dst, size_t* bytes, void* stream);
rom_status rom_load(rom_handle h, const void* src, size_t bytes, void* stream);

/* synchronise the handle's last stream and copy the per-instance flag words to host */
rom_status rom_get_status(rom_handle h, uint32_t* host_flags);
/* zero the per-instance flag words */
rom_status rom_clear_status(rom_handle h, void* stream);

/*
 * fom_residual_vjp - vector-Jacobian product of the residual:
 *   q_prev == NULL: gq = J_f(q)^T gbar
 *   otherwise:      gq = gbar - dt J_f(q)^T gbar,  gq_prev = -gbar (if not NULL)
 *   All device, T[total_dof].
 */
rom_status fom_residual_vjp(rom_handle h, const void* q, const void* q_prev, double dt,
                            const void* gbar, void* gq, void* gq_prev, void* stream);

/*
 * fom_step_vjp - adjoint of one converged backward-Euler step q = S(q_prev):
 * given gbar = dL/dq, returns dL/dq_prev = J_r(q)^-T gbar (implicit function
 * theorem on r(q, q_prev) = q - q_prev - dt f(q) = 0).
 *   q: device, the converged step output; gbar, gq_prev: device; all T[total_dof].
 */
rom_status fom_step_vjp(rom_handle h, const void* q, double dt, const void* gbar, void* gq_prev,
                        void* stream);

/*
 * fom_rollout_vjp - gradient of a loss of the final state of a backward-Euler
 * full-order rollout with respect to its initial state (an extension beyond
 * the paper: the adjoint of eq. fom_discrete_solve iterated).  The rollout is
 * q^{k+1} = S(q^k), k = 0 .. n_steps-1, each step solved by Newton as in
 * fom_step with step dt; given gbar = dL/dq^T it returns
 *   gq0 = dL/dq^0 = J_r(q^1)^-T J_r(q^2)^-T ... J_r(q^T)^-T gbar.
 * Memory follows sqrt(T) checkpointing: the forward pass keeps one state every
 * S = ceil(n_steps / n_ckpt) steps; the backward pass recomputes one segment
 * at a time from its checkpoint and applies the step adjoints in reverse, so
 * about n_ckpt + S + 3 states are held and 2 n_steps forward steps are run.
 * The result does not depend on n_ckpt (every recomputation is bitwise
 * identical).
 *   q0, gbar, gq0: device T[total_dof] (q0 and gbar are not modified; gq0 may
 *   alias gbar).  n_ckpt = 0 chooses ceil(sqrt(n_steps)); n_ckpt > n_steps is
 *   clamped.  The checkpoint storage is allocated on the first call that needs
 *   it (hipMalloc; this call is not meant for stream capture) and kept with
 *   the handle.  Newton flags raised on the way are recorded as for fom_step.
 * Errors: ROM_E_INVAL (NULL pointers, n_steps < 1, n_ckpt < 0, dt <= 0),
 * ROM_E_NOMEM.
 */
rom_status fom_rollout_vjp(rom_handle h, const void* q0, int32_t n_steps, double dt,
                           int32_t n_ckpt, const void* gbar, void* gq0, void* stream);

/*
 * fom_rollout_vjp_noalloc - fom_rollout_vjp for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and result, bit for bit;
 * the checkpoints, segment states and the two adjoint vectors live in a
 * static device array of the library instead of handle-owned memory.
 *   Limit: (nseg + S + 3) * total_dof * sizeof(T) <= 32 MiB, where S =
 *   ceil(n_steps / C), nseg = ceil(n_steps / S), C = n_ckpt (0: ceil(sqrt(n_steps)),
 *   clamped to n_steps).  Larger requests return ROM_E_INVAL before anything
 *   is enqueued.
 *   The array is one per device, held until the process ends, and shared by
 *   every handle on that device: calls that overlap on one device (two
 *   streams, or two host threads) race on it and must be serialised by the
 *   caller.  Every byte the call reads from it was written earlier in the
 *   same call, so nothing carries over from a previous call.
 *   The call makes no allocation: no hipMalloc, hipFree or allocating library
 *   routine.  The handle must be used on the device it was created on.
 * Errors: as fom_rollout_vjp, plus ROM_E_INVAL when the plan exceeds the
 * array, ROM_E_STATE when the current device is not the handle's.
 */
rom_status fom_rollout_vjp_noalloc(rom_handle h, const void* q0, int32_t n_steps, double dt,
                                   int32_t n_ckpt, const void* gbar, void* gq0, void* stream);

/*
 * rom_offline - run Alg. 1's offline stage from q0 on an existing handle (the
 * same work as rom_create with q0: w_init training BE steps, preprocessing,
 * POD, a^{w_init}, the first coarse step, sampling and rebuild); the counters
 * restart (fine step n = w_init, no updates or events).
 *   q0: device, T[total_dof].  Errors: ROM_E_INVAL (NULL handle or q0).
 */
rom_status rom_offline(rom_handle h, const void* q0, void* stream);

/*
 * rom_rollout_vjp - gradient of <gbar, q~_end> with respect to the initial
 * state q0 through Alg. 1 as a whole: the offline stage (training BE steps,
 * preprocessing with q_ref = q0 and D, the POD, a^{w_init}, the first coarse
 * step) and n_steps fine hyper-reduced LSPG steps with their events, where
 * q~_end = q_ref + D^-1 Phi a after those steps.  The sample rows are
 * piecewise constant in q0: the forward run's rows are held fixed, and their
 * (P^T Phi)^+ is differentiated.  An HR-LSPG step is differentiated by the
 * implicit-function theorem on its vanishing weighted residual (no second
 * derivatives); events as in rom_online_vjp, plus the q_ref and D terms of
 * the preprocessing; the POD through the SVD adjoint of the training matrix
 * (distinct singular values).  The online loop keeps checkpoints at segment
 * starts (n_ckpt of them, or ceil(sqrt(n_steps)) for 0) and recomputes each
 * segment; the offline stage keeps its w_init training states.  An extension:
 * the paper differentiates nothing.
 *   q0, gbar, gq0: device, T[total_dof], caller-owned; gq0 receives dL/dq0.
 *   The handle ends at the rollout's end state (as after rom_offline and
 *   rom_step(n_steps)).  Allocates its workspace for the call.  Synchronises
 *   the stream.
 * Errors: ROM_E_INVAL (NULL pointers, n_steps < 1, n_ckpt < 0),
 * ROM_E_UNSUPPORTED (no hyper-reduction, the Galerkin projection, a windowed
 * update rule, the explicit scheme, or a re-orthonormalisation inside the
 * rollout), ROM_E_NOMEM.  A singular Gauss-Newton matrix or rho = 0 at an event
 * sets ROM_FLAG_SINGULAR for the instance.
 */
rom_status rom_rollout_vjp(rom_handle h, const void* q0, int32_t n_steps, int32_t n_ckpt,
                           const void* gbar, void* gq0, void* stream);

/*
 * rom_online_vjp - gradient through the online part of Alg. 1 (an extension
 * beyond the paper): n_fine fine Galerkin steps from the current state, with
 * the adaptation events that fall due (coarse backward-Euler step of y_corr,
 * Alg. 2's Brand update with forgetting factor lambda, the closed-form state
 * transfer a <- Ubar[:r, :r]^T a).  Given qbar = dL/dq~ for the reconstructed
 * state q~ = q_ref + D^-1 Phi a at the end, it returns the gradients of L with
 * respect to the state at the start:
 *   abar   = dL/da,      device double[n_inst * r]
 *   phibar = dL/dPhi,    device double[total_dof * r] (row-major like the basis)
 *   sigbar = dL/dsigma,  device double[n_inst * r]
 *   ycbar  = dL/dy_corr, device double[total_dof]
 * (q_ref and D are held fixed).  Each fine step is differentiated by the
 * implicit-function theorem at its converged state (a transposed r x r solve
 * with J_g = I - dt Phi^T J_f Phi); each event by the adjoints of the
 * transfer, the rotation of eq. isvd_updated_basis_full, the SVD of the core
 * matrix of eq. isvd_core_matrix (distinct singular values), the two
 * Gram-Schmidt passes, the preprocessing, and the coarse step (a transposed
 * banded solve).  The forward pass keeps n_ckpt checkpoints at segment
 * starts and records the last segment as it goes; the backward pass
 * recomputes every other segment from its checkpoint.  n_ckpt = 0 takes one
 * segment (nothing recomputed) when its records fit in half of the free
 * device memory, else ceil(sqrt(n_fine)) checkpoints.  The result does not
 * depend on n_ckpt.  The handle is left in the state that rom_step(h, n_fine)
 * would leave.
 *   qbar: device T[total_dof] (not modified).  Workspace is allocated and
 *   freed inside the call (hipMalloc; not for stream capture); the call
 *   synchronises the stream.  An event with rho = 0 (snapshot inside the
 *   basis span) is not differentiable: its instance gets ROM_FLAG_SINGULAR.
 * Errors: ROM_E_INVAL (NULL pointers, n_fine < 1, n_ckpt < 0), ROM_E_STATE
 * (no reduced state), ROM_E_UNSUPPORTED (hyper-reduction or a problem other
 * than Burgers, or a re-orthonormalisation inside the range).
 */
rom_status rom_online_vjp(rom_handle h, int32_t n_fine, int32_t n_ckpt, const void* qbar,
                          double* abar, double* phibar, double* sigbar, double* ycbar,
                          void* stream);

/*
 * Autotuning of launch shapes and solver settings, per handle.
 *   ROM_TUNE_RESIDUAL  the streaming residual of the Euler problems
 *       (fom_residual, and the residual evaluations inside the grid-wide
 *       Newton step): tiles of 1024, 512 or 256 cells (4, 2 or 1 cells per
 *       thread), a persistent grid of 1..12 resident blocks per compute unit,
 *       plain or non-temporal loads and stores of the streamed state.  Every
 *       cell is computed by the same arithmetic in every shape: outputs are
 *       bitwise identical.  Other problems have a single candidate.
 *   ROM_TUNE_DEIM_PASS the greedy DEIM pass (hyper = ROM_HR_DEIM): 4, 2 or 8
 *       candidate rows per 2048-row pass tile.  The argmax over all
 *       candidates takes the same row (lowest index on ties): P and
 *       (P^T Phi)^+ are bitwise identical.  One candidate without DEIM.
 *   ROM_TUNE_BT_PART   the part size m of the block-tridiagonal solver of
 *       the backward-Euler steps (the separator spacing of its recursive
 *       Schur complement): 16, 8 or 32 cells for 1- and 3-variable blocks (a
 *       single candidate, 8, for 12-variable blocks).  Every candidate solves
 *       the same system exactly in exact arithmetic; results differ at the
 *       level of rounding.  Changing it re-creates the solver's levels and
 *       drops captured window graphs.
 *   Candidate 0 of each target is the default.
 *
 * rom_autotune - time every candidate on the given stream and keep the
 *   fastest for the handle; *choice (optional) receives its index.
 *   RESIDUAL: 2 warm-up and 5 timed residual evaluations of q; DEIM_PASS:
 *   1 warm-up and 3 timed rebuilds (needs a reduced state; q unused, may be
 *   NULL); BT_PART: 1 warm-up and 3 timed backward-Euler steps from q with
 *   the configured dt.  q: device T[total_dof].  The handle's state is not
 *   modified.  Synchronises the stream.
 * rom_set_tuning - force candidate `choice` (choice < 0 only queries);
 *   *n_candidates (optional) receives the number of candidates.
 * Errors: ROM_E_INVAL (NULL handle, NULL q where it is used, unknown target,
 * choice out of range), ROM_E_STATE (DEIM_PASS without a reduced state).
 */
enum { ROM_TUNE_RESIDUAL = 0, ROM_TUNE_DEIM_PASS = 1, ROM_TUNE_BT_PART = 2 };
rom_status rom_autotune(rom_handle h, int32_t what, const void* q, int32_t* choice, void* stream);
rom_status rom_set_tuning(rom_handle h, int32_t what, int32_t choice, int32_t* n_candidates);

/*
 * rom_profile - time one stage of the hot path in isolation: the stage is
 * launched reps times between two HIP events recorded on the given stream and
 * the mean milliseconds per launch are written to *ms.  The handle's reduced
 * state is not modified.
 *   ROM_PROF_RESIDUAL       f(q) for the batch (one launch), q: device T[total_dof]
 *                           (the limited second-order f with ROM_SCHEME_SSPRK43)
 *   ROM_PROF_GALERKIN_PASS  one fused Galerkin pass over the basis (all instances)
 *   ROM_PROF_ISVD_PROJECT   one iSVD projection pass over the basis with snapshot q
 *   ROM_PROF_RESIDUAL_VJP   J_f(q)^T q for the batch
 *   ROM_PROF_FOM_STEP       one full backward-Euler Newton step from q (dt = cfg.dt),
 *                           or one SSPRK(4,3) step with ROM_SCHEME_SSPRK43
 * Synchronises the stream.  Errors: ROM_E_INVAL for an unknown stage or reps < 1.
 */
enum { ROM_PROF_RESIDUAL = 0, ROM_PROF_GALERKIN_PASS = 1, ROM_PROF_ISVD_PROJECT = 2,
       ROM_PROF_RESIDUAL_VJP = 3, ROM_PROF_FOM_STEP = 4 };
rom_status rom_profile(rom_handle h, int32_t stage, int32_t reps, const void* q, double* ms,
                       void* stream);

/* sizes of the handle's layout: total_dof, n_var, r, n_s (any may be NULL) */
rom_status rom_query(rom_handle h, int64_t* total_dof, int32_t* n_var, int32_t* r, int32_t* n_s);

const char* rom_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ROMHIP_H */
