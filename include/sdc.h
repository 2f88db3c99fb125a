/*
 * sdc.h -- C ABI of the MI355X (gfx950) adaptive spectral-deferred-correction
 * library for monodomain and cell-by-cell (EMI) reaction-diffusion systems.
 *
 * Problem (paper Sec. 2.2, eq. "abstract monodomain"; abstract form B z' = F(z),
 * Sec. 3):  P1 finite elements on simplices give
 *
 *     ML v' = -A v - ML * I(v, w),        w' = R(v, w),
 *
 * with ML the row-sum lumped mass, A the stiffness matrix and (I, R) the
 * Aliev-Panfilov current and gating rate (Sec. 5.1).  One step of length dt
 * is taken by SDC on M Radau-IIA nodes (Sec. 3.1) with the LU-trick
 * lower-triangular QI for the implicit diffusion and forward Euler between
 * nodes (QE) for the explicit reaction (operator splitting as basic scheme,
 * Sec. 3.2, eq. final-sdc, read as implicit-explicit).  Each node's linear
 * system (ML + dt*QI[m][m]*A) dv = b is solved by Jacobi-preconditioned CG
 * (Sec. 4.2).  Sweep k works only on the nested active index set I_k
 * (Sec. 4.2): the next set keeps the rows whose correction max_m |dv_m,i|
 * reached the drop tolerance theta (eq. "subset"); theta <= 0 gives the
 * non-adaptive method.  Every step starts with all rows active.
 *
 * Several independent instances ("batch") can share one context: they are
 * numbered consecutively (node_off), never share an element, and each runs
 * its own CG with its own scalars and stopping test.
 *
 * Conventions
 *  - All calls return int: SDC_OK (0) or a negative SDC_ERR_* code; nothing
 *    throws across the ABI.  The message of the last error of a context is
 *    returned by sdc_last_error.  After SDC_ERR_HIP the context should be
 *    destroyed.
 *  - "device" pointers are HIP device memory of the context's device, FP64
 *    unless stated, contiguous, owned by the caller; the library never frees
 *    them.  "host" arrays are read during the call and copied.
 *  - Work is enqueued on the stream given to sdc_create.  Calls that return
 *    host statistics synchronise that stream.
 *  - Node indices are int32 (0 .. N-1, N < 2^31); index lists are ascending.
 */
#ifndef SDC_H
#define SDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SDC_OK = 0,
  SDC_ERR_ARG = -1,        /* invalid argument (null pointer, size, order)   */
  SDC_ERR_HIP = -2,        /* a HIP runtime call failed                      */
  SDC_ERR_CG_MAXIT = -3,   /* a CG solve did not converge within cg_maxit    */
  SDC_ERR_STATE = -4,      /* call out of order (e.g. sweep before a step)   */
  SDC_ERR_OOM = -5,        /* device allocation failed                       */
  SDC_ERR_NONFINITE = -6   /* NaN/Inf or a non-positive CG curvature p.Hp    */
};

#define SDC_MAX_NODES 6    /* collocation nodes M supported: 1..6            */
#define SDC_MAX_SWEEPS 16  /* sweeps per step K supported: 1..16             */
#define SDC_MAX_RECORDINGS 64  /* recorded steps held for the reverse pass   */

typedef struct sdc_ctx sdc_ctx;

/* Solver settings, copied by sdc_setup_mesh. */
typedef struct {
  int32_t M;          /* Radau-IIA collocation nodes, 1..SDC_MAX_NODES         */
  int32_t K;          /* SDC sweeps per step, 1..SDC_MAX_SWEEPS                */
  double dt;          /* step length                                           */
  double theta;       /* drop tolerance TOL_drop; <= 0: all rows stay active   */
  double cg_rtol;     /* stop when ||r||_2 <= cg_rtol * ||b||_2 (active rows)  */
  int32_t cg_maxit;   /* CG iteration limit per solve (SDC_ERR_CG_MAXIT)       */
  int32_t format;     /* matrix storage: 0 = timed choice at setup, 1 = CSR,   */
                      /* 2 = diagonal (every instance's rows use <= 32        */
                      /* distinct column offsets; else SDC_ERR_ARG),          */
                      /* 3 = sliced ELL (slices of 64 rows, one wavefront,    */
                      /* entries column by column, padded to the slice's      */
                      /* longest row; not with scheme 1).  The timed choice   */
                      /* keeps the diagonal copy when it reads at most 0.6 of */
                      /* CSR's matrix bytes, else times one SpMV-shaped CG    */
                      /* start per storage built; every storage gives         */
                      /* bitwise the same results.                            */
  /* Energy-norm termination (paper Sec. 3.2), off when tol_sdc <= 0: after  */
  /* at least K_min sweeps an instance stops once                            */
  /*   sum_m dv_m^T H_m dv_m <= ((1 - rho) / rho * tol_sdc)^2                 */
  /* (its rows leave the active set); the step ends when every instance has  */
  /* stopped, or after K sweeps.  Not combined with the reverse pass.        */
  int32_t K_min;      /* 1..K (values <= 0 mean 1)                             */
  double tol_sdc;     /* TOL_SDC                                               */
  double rho;         /* assumed contraction factor, 0 < rho < 1               */
  /* Drop tolerance of the active sets.  0: theta above.  1: a-priori per     */
  /* instance and step (paper Sec. 4.1, eqs. subset and drop-tolerance):      */
  /*   TOL_drop = exp(-eta dt) (1 - rho) / (r + 1) tol_sdc,                   */
  /* from the step's first sweep: c = the instance's max_m |dv_m| (the error  */
  /* constant of Thm. 2, rho taken as known), r = the least r >= 0 with      */
  /* c rho^r <= (1 - rho) tol_sdc, eta = max(0, -min dI/dv) over its rows at  */
  /* the step's start state and the collocation values (Thm. 1, beta C_m =   */
  /* 1).  Needs tol_sdc > 0 (which also switches the energy-norm termination */
  /* on) and the monodomain model; else SDC_ERR_ARG.                          */
  int32_t drop_mode;
  /* Sweep scheme.  0: implicit diffusion, explicit reaction and gating      */
  /* (the system matrices H_m = ML + dt QI[m][m] A are fixed).  1: the       */
  /* paper's basic scheme (Sec. 3.2, eq. final-sdc): the lumped reaction     */
  /* Jacobian G_j = ML dI/dv(v_j, w_j) of the sweep's iterate joins A in the */
  /* implicit operator, H_m = ML + dt QI[m][m] (A + G_m), and the right-hand  */
  /* side carries dt sum_{j<m} QI[m][j] (A + G_j) dv_j; the gating follows    */
  /* all potentials with implicit dR/dw (Gauss-Seidel).  Monodomain only,     */
  /* not with the reverse pass; sdc_solve then uses the diagonals of the     */
  /* last sweep on its rows.                                                 */
  int32_t scheme;
  /* Rows of each step's first sweep.  0: all rows (the paper's method).     */
  /* R >= 1: a heuristic a-priori set (paper Sec. 6 names one for the first  */
  /* sweep without fixing a rule; this is the library's): each step carries  */
  /* the set its second sweep uses (its first sweep's own set when K = 1);   */
  /* a later step's first sweep takes that set and the rows a stimulus       */
  /* overwrites at its start, grown R times by their mesh neighbours         */
  /* (vertices sharing a simplex).  Rows outside keep the step's start       */
  /* values.  All rows on the first step after setup or after               */
  /* sdc_set_active(ctx, -1, ...), and on every first_full_every-th step     */
  /* counted from there (<= 0: never again).  Monodomain only, not with the */
  /* reverse pass.                                                           */
  int32_t first_rings;
  int32_t first_full_every;
  /* Solves whose instances each have at most this many active rows run as  */
  /* one launch (the whole Jacobi-PCG of an instance in one workgroup)        */
  /* instead of one launch per iteration.  0: the default and largest value  */
  /* (2048 rows; 1024 when a row of A has more than 8 stored entries);       */
  /* -1: never.  Same stopping rule, results equal to rounding.              */
  int32_t small_set_rows;
  /* CG launches over all rows with diagonal storage of 3, 7 or 19          */
  /* diagonals: 1 or 2 rows per thread, 0 = the faster of the two, timed on  */
  /* one CG iteration at setup.  Bitwise the same results either way.        */
  int32_t rows_per_thread;
  /* Optional energy-error stop of every CG solve (paper Sec. 5.1 stops at  */
  /* an estimated energy-error reduction; the estimator is the library's).  */
  /* With x0 = 0, step j lowers the squared energy error by                 */
  /* t_j = alpha_j (r_j . z_j); a solve stops after n >= cg_delay steps     */
  /* once the last cg_delay terms sum to at most cg_energy_tol^2 times all   */
  /* n terms (an estimated relative energy error of x_{n - cg_delay}), or   */
  /* at the residual test, whichever comes first.  0: off (the default);    */
  /* > 0 needs cg_delay in 1..8.  Monodomain only, not with the reverse      */
  /* pass.                                                                   */
  double cg_energy_tol;
  int32_t cg_delay;
} sdc_params;

/* Per-sweep statistics (sums over instances unless stated). */
typedef struct {
  int64_t n_active;                    /* rows of I_k                           */
  int64_t nnz_active;                  /* stored entries of A in those rows     */
  int64_t n_next;                      /* rows of I_{k+1} (selected)            */
  int32_t cg_iters_max[SDC_MAX_NODES]; /* max CG iterations over instances      */
  int64_t cg_row_iters[SDC_MAX_NODES]; /* sum_inst iters * active rows          */
  int64_t cg_nnz_iters[SDC_MAX_NODES]; /* sum_inst iters * active entries       */
  double energy;                       /* sum_inst sum_m dv_m^T H_m dv_m (only   */
                                       /* with the energy-norm termination on)   */
  int32_t n_stopped;                   /* instances stopped after this sweep     */
  double ms;                           /* stream time of the sweep, by events:   */
                                       /* from its first launch to its return    */
                                       /* (selection of the next set and the     */
                                       /* host synchronisation included)         */
} sdc_sweep_stats;

typedef struct {
  int32_t n_sweeps;
  sdc_sweep_stats sweep[SDC_MAX_SWEEPS];
} sdc_step_stats;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device`; `stream` is a hipStream_t (NULL =
 * the null stream).  *out receives the context or NULL on error. */
int sdc_create(sdc_ctx** out, int32_t device, void* stream);
void sdc_destroy(sdc_ctx* ctx);
/* Message of the last failed call (owned by ctx; valid until the next call). */
const char* sdc_last_error(const sdc_ctx* ctx);
/* Replace the stream later work is enqueued on. */
int sdc_set_stream(sdc_ctx* ctx, void* stream);

/* ---- setup (paper Sec. 2.2: P1 discretisation) ------------------------ */

/* Cell-by-cell (EMI) model (paper Sec. 2.1, eq. "cell-by-cell model", its
 * weak form, and the discrete system of eqs. "abstract reaction diffusion" /
 * "abstract gating").  The unknowns are the potentials u of every subdomain
 * (intracellular and extracellular nodes; a membrane point exists twice) and
 * the gating variables of the membrane sites:
 *
 *     M u' = -A u - b(u, w),        w_s' = R(v_s, w_s),   v_s = u_i(s) - u_e(s),
 *
 *   M = C_m sum_s l_s (e_i - e_e)(e_i - e_e)^T      (membrane mass, singular)
 *   b = sum_s l_s I(v_s, w_s) (e_i - e_e)
 *   A = elements (per-subdomain conductivity in elem_tensor)
 *       + eps * diag(robin_len)                     (Robin condition, outer boundary)
 *       + g_gap sum_g l_g (e_a - e_b)(e_a - e_b)^T  (linear gap junctions, implicit)
 *
 * In sdc_step the arrays v, w hold u [N] and the gating variable of site s
 * at its intracellular node (other entries of w are left unchanged).  The
 * drop rule measures max_m |du_m| per node; a site is updated in a sweep iff
 * its intracellular node is active.  One instance only; CSR storage; the
 * reverse pass and sdc_set_coefficients are not available for this model
 * (SDC_ERR_STATE). */
typedef struct {
  int64_t n_mem;              /* membrane sites                                 */
  const int32_t* mem_intra;   /* host int32[n_mem]: intracellular node of site s */
  const int32_t* mem_extra;   /* host int32[n_mem]: extracellular node of site s */
  const double* mem_len;      /* host double[n_mem]: lumped membrane length > 0  */
  double cm;                  /* membrane capacitance C_m > 0                   */
  int64_t n_gap;              /* gap-junction node pairs                        */
  const int32_t* gap_a;       /* host int32[n_gap]                              */
  const int32_t* gap_b;       /* host int32[n_gap]                              */
  const double* gap_len;      /* host double[n_gap]: lumped face length >= 0    */
  double g_gap;               /* gap-junction conductance per length >= 0       */
  const double* robin_len;    /* host double[N]: lumped outer-boundary length   */
  double eps;                 /* Robin coefficient >= 0                         */
} sdc_emi;

/* Assemble ML and A (or, with emi, M and A) on the host and upload
 * everything the sweeps need.
 *  dim          1, 2 or 3 (simplices with dim+1 vertices)
 *  n_inst       number of independent instances (>= 1)
 *  node_off     host int64[n_inst+1]: instance i owns nodes [node_off[i], node_off[i+1])
 *  coords       host double[N][dim]
 *  elem_off     host int64[n_inst+1]: instance i owns elements [elem_off[i], elem_off[i+1])
 *  elems        host int32[E][dim+1], global node ids inside the owning instance
 *  elem_tensor  host double[E][dim][dim]: unit conductivity tensor D_T
 *  node_sigma   host double[N]: conductivity multiplier; element value is the
 *               mean over its vertices, A = sum_T sigma_T |T| G_T D_T G_T^T
 *  ionic        host double[n_inst][6]: Aliev-Panfilov (k, a, eps0, mu1, mu2, s)
 *  emi          NULL for the monodomain model; else the cell-by-cell
 *               couplings above (n_inst must be 1; each node belongs to at
 *               most one membrane site; SDC_ERR_ARG otherwise)
 * May be called once per context. */
int sdc_setup_mesh(sdc_ctx* ctx, const sdc_params* params, int32_t dim, int32_t n_inst,
                   const int64_t* node_off, const double* coords, const int64_t* elem_off,
                   const int32_t* elems, const double* elem_tensor, const double* node_sigma,
                   const double* ionic, const sdc_emi* emi);

/* Stimulus: at the start of the step whose interval [t, t+dt) contains t_on,
 * set v = value on the listed nodes (host int32[n]) before spreading. */
int sdc_add_stimulus(sdc_ctx* ctx, double t_on, const int32_t* nodes, int64_t n, double value);

/* Sizes of the assembled system: N, nnz of A, Nw (= N for monodomain). */
int sdc_get_sizes(const sdc_ctx* ctx, int64_t* n, int64_t* nnz, int64_t* nw);

/* Copy the assembled CSR of A and the lumped mass (cell-by-cell model: the
 * diagonal of the membrane mass) to host arrays rowptr int32[N+1],
 * col int32[nnz], val double[nnz], ml double[N]. */
int sdc_get_system(sdc_ctx* ctx, int32_t* rowptr, int32_t* col, double* val, double* ml);

/* ---- time stepping (paper Sec. 3, eq. final-sdc; Sec. 4.2) ------------- */

/* One SDC step: (v, w) at time t -> (v, w) at t + dt, in place.  v, w are
 * device double[N].  stats (host, may be NULL) receives per-sweep counts.
 * The CG solves run with iteration budgets predicted from the last step's
 * counts, one host synchronisation per sweep; a budget that falls short
 * redoes the step with the synchronous loop (the same results).  A step
 * whose t does not continue the last step begun (t != t_last + dt: the
 * first step, a restart from a checkpoint, a window run again) takes the
 * synchronous loop at once. */
int sdc_step(sdc_ctx* ctx, double* v, double* w, double t, sdc_step_stats* stats);

/* The same step in parts: begin (stimulus, spread, all rows active), then
 * sdc_sweep up to K times, then end (copy the last node out). */
int sdc_begin_step(sdc_ctx* ctx, const double* v, const double* w, double t);
int sdc_sweep(sdc_ctx* ctx, sdc_sweep_stats* stats);
int sdc_end_step(sdc_ctx* ctx, double* v, double* w);

/* Copy collocation node m's current values (device double[N] each). */
int sdc_get_node(sdc_ctx* ctx, int32_t m, double* v_m, double* w_m);

/* CG step counts of the last sweep's restricted solves (Sec. 4.2), per node
 * and instance: host out int32[M][n_inst] (element m * n_inst + i), the
 * updates instance i's solve of node m performed (0 for an instance without
 * active rows).  SDC_ERR_STATE before the first sweep. */
int sdc_get_cg_iters(sdc_ctx* ctx, int32_t* out);

/* Current active set (the set the next sweep will use): idx device int32
 * with room for N entries (may be NULL to query only), *n receives its length. */
int sdc_get_active(sdc_ctx* ctx, int32_t* idx, int64_t* n);

/* Pin the active set of sweep `sweep` (1..K-1; sweep 0 uses all rows, or
 * the heuristic set of first_rings) for all following steps, replacing the
 * selection rule there: idx is a device int32[n] ascending list (copied).
 * sweep < 0 clears every pin and the set carried for the next first sweep
 * (restarting the step count of first_full_every). */
int sdc_set_active(sdc_ctx* ctx, int32_t sweep, const int32_t* idx, int64_t n);

/* Reverse-mode step (adjoint of sdc_step with every sweep's active set held
 * fixed and each restricted solve taken as exact): recomputes the step from
 * (v_n, w_n) at time t (device double[N] each, unchanged), then, given the
 * adjoints lam_v, lam_w of (v, w) at t + dt (device double[N], in), writes the
 * adjoints of (v_n, w_n) over them (out; zero on nodes a stimulus overwrote
 * at this step) and ADDS the derivatives of the same scalar with respect to
 * the nodal conductivity multipliers to g_sigma (device double[N]) and with
 * respect to each instance's Aliev-Panfilov parameter a to g_a (device
 * double[n_inst]).  The reverse solves use the forward's Jacobi-PCG on the
 * same (symmetric) restricted matrices.  Uses about (2K + 6) M N + K N extra
 * doubles of device memory, allocated on the first call. */
int sdc_adjoint_step(sdc_ctx* ctx, const double* v_n, const double* w_n, double t, double* lam_v,
                     double* lam_w, double* g_sigma, double* g_a);

/* The same reverse step in two parts, so that a checkpoint segment is
 * recomputed once: sdc_adjoint_record advances (v, w) in place by one step
 * from time t exactly like sdc_step and keeps what the reverse pass needs in
 * recording `slot` (0..SDC_MAX_RECORDINGS-1; about (2K + 2) M N doubles of
 * device memory per slot, allocated on first use); sdc_adjoint_reverse then
 * applies the reverse step of that recording (same arguments and results as
 * sdc_adjoint_step).  Slot 0 is also used by sdc_adjoint_step. */
int sdc_adjoint_record(sdc_ctx* ctx, int32_t slot, double* v, double* w, double t);
int sdc_adjoint_reverse(sdc_ctx* ctx, int32_t slot, double* lam_v, double* lam_w, double* g_sigma,
                        double* g_a);

/* The a-priori drop tolerance of the current step (drop_mode 1, after the
 * step's first sweep; zeros before any), per instance, written to host
 * out[4 * n_inst]: (TOL_drop, r, c, eta) as defined at sdc_params.drop_mode.
 * SDC_ERR_STATE when drop_mode is 0.  Synchronises the stream. */
int sdc_get_drop_tolerance(sdc_ctx* ctx, double* out);

/* Replace the nodal conductivity multipliers (host double[N], or NULL to keep)
 * and the Aliev-Panfilov parameters (host double[n_inst][6], or NULL): A is
 * reassembled on the same pattern (paper Sec. 2.2) and the node matrices,
 * Jacobi diagonals and diagonal storage are rebuilt. */
int sdc_set_coefficients(sdc_ctx* ctx, const double* node_sigma, const double* ionic);

/* ---- components (for kernel-level parity tests) ----------------------- */

/* Restricted Jacobi-PCG (paper Sec. 4.2) on H_m = ML + dt*QI[m][m]*A:
 * solve H_m[idx, idx] x = b[idx] with x = 0 off idx.  idx device int32[n]
 * ascending, each instance's rows contiguous; b, x device double[N] (x is
 * fully overwritten).  iters host int32[n_inst] (may be NULL). */
int sdc_solve(sdc_ctx* ctx, int32_t m, const int32_t* idx, int64_t n, const double* b,
              double* x, int32_t* iters);

/* Active-set compaction (paper eq. "subset", Sec. 4.2): idx_out = the
 * entries i of idx_in (device int32[n_in], ascending) with amax[i] >= theta,
 * in order; theta <= 0 keeps all.  amax device double[N]; idx_out device
 * int32[n_in]; *n_out host. */
int sdc_select(sdc_ctx* ctx, const double* amax, const int32_t* idx_in, int64_t n_in,
               double theta, int32_t* idx_out, int64_t* n_out);

/* ---- allocation-free entry point -------------------------------------- */

/* For callers that cannot allocate device memory or synchronise: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The active-set compaction of sdc_select (idx_out = the entries i of idx_in
 * with amax[i] >= theta, in their order; theta <= 0 keeps every entry; NaN
 * is dropped otherwise) with no context: it allocates nothing, does not
 * synchronise, and enqueues three kernels on `stream` (a hipStream_t; NULL =
 * the null stream) of HIP device `device`.
 *  amax     device double[n_amax]
 *  idx_in   device int32[n_in], n_in <= SDC_NOALLOC_MAX_IN
 *  idx_out  device int32[n_in] (room for all entries; only the kept ones
 *           are written)
 *  n_out    device int64[1]: the number of kept entries, or -1 when an entry
 *           of idx_in lies outside [0, n_amax) (then idx_out is not written)
 * Scratch: the per-block counts live in a library-held device array of
 * SDC_NOALLOC_MAX_IN / 256 int32 (256 KiB) per device, set up on the first
 * call on that device and kept until the process ends.  Every call on a
 * device shares it: calls that overlap on one device (different streams)
 * race and must be serialised by the caller.
 * Returns SDC_ERR_ARG for a null pointer, a negative size, n_in above
 * SDC_NOALLOC_MAX_IN or a device out of range (nothing enqueued), and
 * SDC_ERR_HIP when a launch fails. */
#define SDC_NOALLOC_MAX_IN (1 << 24)
int sdc_select_noalloc(int32_t device, void* stream, const double* amax, int64_t n_amax,
                       const int32_t* idx_in, int64_t n_in, double theta, int32_t* idx_out,
                       int64_t* n_out);

/* ---- measurement ------------------------------------------------------ */

/* Kernel timing of the CG iteration kernel (one launch per iteration: SpMV,
 * vector updates and the three dot products), taken with start/stop HIP
 * events attached to each launch on the context's stream (stamped by the
 * dispatch, so they time the kernel's execution), for every launch that
 * does work for at least one instance.  Bytes are the algorithmic minimum per launch over the instances
 * still iterating: 8 per stored matrix value in their active rows (index
 * structure is storage overhead and not counted), plus per active row
 * 4 (active-list entry; absent when every row is active) + 6*8 reads
 * (x, p, dinv and the three preconditioner-scaled CG vectors) + 5*8 writes
 * (x, p and the three vectors). */
typedef struct {
  int64_t cg_launches;
  double cg_ms;
  double cg_bytes;
  /* the same over the launches on every row of the instances (no active */
  /* list: the first sweep of each step), a subset of the above          */
  int64_t cg_all_launches;
  double cg_all_ms;
  double cg_all_bytes;
  /* sums over the timed launches of the rows and stored entries of A of the */
  /* instances still iterating (for other byte models), all launches and   */
  /* those on every row                                                     */
  double cg_rows, cg_nnz;
  double cg_all_rows, cg_all_nnz;
} sdc_profile_stats;

/* Setup outcome: storage in use (1 CSR, 2 diagonal, 3 sliced ELL), diagonals per row in the
 * diagonal storage (0 if not available), the setup timings of one SpMV-shaped
 * CG start launch over all rows in each storage (0 if not timed), the
 * number of steps redone because a predicted CG budget was too small, the
 * rows per thread of the all-rows CG launches, and the setup timings of one
 * all-rows CG iteration with one and with two rows per thread (0 if not
 * timed). */
typedef struct {
  int32_t format;
  int32_t n_diagonals;
  double t_csr_us;
  double t_dia_us;
  int64_t redone_steps;
  int32_t rows_per_thread;
  double t_rows1_us;
  double t_rows2_us;
  /* graph-captured sweeps (sdc_set_graph): steps taken that way, captures */
  /* made, and steps redone by the synchronous loop after a short budget  */
  int64_t graph_steps;
  int64_t graph_captures;
  int64_t graph_redone;
  double t_sell_us;   /* setup timing of the sliced ELL storage (0 if not timed) */
  /* order of the work maps' 256-row blocks over the 8 XCDs: each XCD takes */
  /* runs of xcd_chunk consecutive blocks in turn (about 8 stencil reaches, */
  /* the matrix bandwidth); 0 = each XCD a contiguous eighth of the map     */
  int32_t xcd_chunk;
} sdc_info;

int sdc_get_info(sdc_ctx* ctx, sdc_info* out);

/* Graph-captured sweeps for sdc_step (enable != 0; 0 returns to launches
 * from the host).  Each sweep k of a step becomes one HIP graph with a fixed
 * launch sequence: the sweep start, then per node the right-hand side, the
 * CG start, a fixed number of CG iteration launches (the last step's count
 * for that sweep and node plus one, and an eighth more, at least two;
 * launches after a solve has converged return at once) and the post-solve
 * update, then the selection of the next set.  The sets stay on the device:
 * the kernels of sweeps k >= 1 read the selected set's size there, on grids
 * of the all-rows capacity, blocks past the set returning at once.  A step
 * is K graph launches and one synchronisation, after which the CG outcomes
 * are checked; a solve that did not finish within its launches makes the
 * step be redone by the synchronous loop (the same results), and the graphs
 * are captured again when the predicted counts outgrow them.  Results equal
 * those of host-launched steps bitwise when the latter do not use the
 * one-workgroup solves (small_set_rows = -1, or sets above their size),
 * which graph steps never use.  The default options of the monodomain
 * model only (scheme 0, fixed K and theta, first sweeps on all rows,
 * residual CG stop): else SDC_ERR_ARG.  Steps with pinned sets or kernel
 * timing on run from the host.  Work memory: 2 K M n_inst int32 on the
 * device and in pinned host memory; the graphs are captured on a stream of
 * the library's own and launched on the context's stream. */
int sdc_set_graph(sdc_ctx* ctx, int32_t enable);

/* enable != 0 starts timing (and clears the totals); 0 stops it. */
int sdc_profile(sdc_ctx* ctx, int32_t enable);
int sdc_profile_read(sdc_ctx* ctx, sdc_profile_stats* out);

/* Collocation data used by the library (paper Sec. 3.1): host outputs
 * tau[M], Q[M][M] (zero-to-node integrals of the Lagrange basis),
 * QI[M][M] (U^T of Q^T = L U), QE[M][M] (forward Euler between nodes). */
int sdc_collocation(int32_t M, double* tau, double* Q, double* QI, double* QE);

#ifdef __cplusplus
}
#endif

#endif /* SDC_H */
