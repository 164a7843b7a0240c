/*
 * mb.h -- C ABI of the MI355X (gfx950) Maxwell-Bloch library, libmbhip.so.
 *
 * The library advances the one-dimensional Maxwell-Bloch equations of the
 * mbsolve paper (Sec. 2.1, eq:efield, eq:hfield, eq:master1D) on a Yee grid
 * (Sec. 2.2, eq:ediscrete, eq:hdiscrete; update form eq:eupdate,
 * eq:hupdate of Sec. 3.2) with the density matrices of an N-level quantum
 * system in every grid cell, weakly coupled in time (Fig. 1: rho lives at
 * t_{n+1/2} at the E nodes), without rotating-wave or slowly-varying
 * envelope approximations.  The density step is the exact-step/operator
 * splitting family of Sec. 2.2: a Strang splitting
 *     rho^{n+1/2} = e^{L0 dt/2} W_n e^{L0 dt/2} rho^{n-1/2},
 *     W_n(rho) = exp(+i dt E^n mu / hbar) rho exp(-i dt E^n mu / hbar),
 * where L0 = -i/hbar [H0, .] + D and D is the relaxation superoperator given
 * by scattering and pure-dephasing rates (eq:relax_pop and the dephasing
 * law of Sec. 3.1.1).  The polarization current of eq:ediscrete is
 * n3D tr{mu L0(rho^{n+1/2})} (Sec. 2; the field part drops out because
 * tr{mu [mu, rho]} = 0).  The step order is that of Alg. 1: H and rho (and p),
 * then E, then edges, sources and records.
 *
 * Conventions
 *  - SI units.  The caller passes hbar, c0, mu0, eps0 and e explicitly.
 *  - Operators are Hermitian N x N matrices given as a real diagonal plus the
 *    upper triangle packed column by column, (1,2),(1,3),(2,3),(1,4),...,
 *    each complex entry as (re, im) doubles (qm_operator, Sec. 3.1.1).
 *  - rates[i*N + j] = gamma_ij, the scattering rate from level j into
 *    level i (eq:relax_pop); the diagonal is ignored.  Pure dephasing rates
 *    use the packed pair order.
 *  - Grid: nx E nodes at x_m = m dx, dx = length/(nx-1); H nodes at
 *    x_{m+1/2}, m = 0..nx-2.  The material of a node is the first region
 *    with x_start <= x < x_end, else the first with x_start <= x <= x_end,
 *    else the right-most region if x exceeds the device by under dx/2.
 *  - Edges (Sec. 2.1): reflectivity 1 is a perfect electric conductor
 *    (E = 0), reflectivity 0 a first-order Mur absorbing boundary, and
 *    0 < R < 1 (a semi-transparent mirror) a resistive load
 *    Z_L = eta (1 - sqrt R)/(1 + sqrt R) on the edge node's half cell (eta:
 *    wave impedance of the edge material), whose amplitude reflection at
 *    normal incidence is -sqrt R.  Values outside [0, 1] are MB_ERR_ARG.
 *  - Sources act after each step at t_{n+1} = (n+1) dt at the E node nearest
 *    to their position (halves to the even node): a hard source sets E there, a
 *    soft source adds to it.  A hard source also sets E^0.
 *  - Records are sampled after step n when (n+1) is a multiple of their
 *    interval; density quantities refer to rho^{n+1/2}, E to E^{n+1}, H to
 *    H^{n+1/2}.  Every record value is delivered in double precision.
 *
 * Ownership: every host pointer passed in is read during the call only (the
 * library copies what it keeps).  Device memory belongs to the library and is
 * released by the matching destroy call.  Handles are not thread-safe; use one
 * handle per thread.  The server is internally synchronised.
 *
 * Errors: functions return MB_OK (0), a positive warning, or a negative
 * error code; mb_last_error() gives a thread-local message for the last
 * non-zero status.  No C++ exception crosses this boundary.
 */
#ifndef MB_H
#define MB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define MB_OK 0
#define MB_WARN_NOT_CP 1        /* pure dephasing admits no positive semi-definite C (Sec. 3.1.1) */
#define MB_ERR_ARG -1           /* invalid argument or inconsistent description */
#define MB_ERR_CFL -2           /* c_max * dt > dx: time step beyond the Courant limit (Sec. 3.2) */
#define MB_ERR_UNSUPPORTED -3   /* level count outside 2..8, plain variant in FP32, ... */
#define MB_ERR_OOM -4           /* device allocation failed */
#define MB_ERR_BUDGET -5        /* a request does not fit the server's device-memory budget */
#define MB_ERR_HIP -6           /* a HIP runtime call failed */
#define MB_ERR_NONFINITE -7     /* a simulation produced a non-finite field value */
#define MB_ERR_STATE -8         /* call out of order (e.g. reading a request not yet done) */
#define MB_ERR_DEVICE -9        /* a tile of a persistent launch gave up waiting (2 s) for a
                                   neighbour tile; the run's results are not valid */

/* ---- enumerations -------------------------------------------------------- */
/* Field part of the density step, W rho W^+ with A = i dt E mu / hbar:
 * MB_FIELD_EXACT takes W = exp(A) (through the eigen-decomposition of mu);
 * MB_FIELD_CAYLEY its Cayley approximant W = (I - A/2)^{-1} (I + A/2), unitary and
 * second-order accurate (the lindblad_reg_cayley class of Sec. 3.2 names the
 * form).  Both forms run on every variant; persistent Cayley launches use one
 * wave per 64 cells. */
#define MB_FIELD_EXACT 0
#define MB_FIELD_CAYLEY 1

#define MB_SRC_SECH 0   /* s(t) = amp sech(width t' - shift) sin(2 pi freq t + phase) */
#define MB_SRC_GAUSS 1  /* s(t) = amp exp(-(width t' - shift)^2) sin(2 pi freq t + phase) */
                        /* t' = t - q period, summed over q = 0..count-1 */
#define MB_SRC_TABLE 2  /* s(t_n) = table[n] for n < table_len, 0 after (sampled waveform) */

#define MB_REC_E 0       /* E at the cell                    */
#define MB_REC_H 1       /* H at x_{cell+1/2} (0 at the last cell) */
#define MB_REC_POP 2     /* rho_ii                           */
#define MB_REC_INV 3     /* rho_jj - rho_ii                  */
#define MB_REC_RHO_RE 4  /* Re rho_ij                        */
#define MB_REC_RHO_IM 5  /* Im rho_ij                        */

/* time discretisation of the density matrix (Sec. 2.2): weak coupling keeps
 * rho at t_{n+1/2} (the default), strong coupling at t_n with E; there the
 * step is driven by the midpoint field (E^n + E^{n+1})/2 and the
 * polarization current is n3D tr{mu (rho^{n+1} - rho^n)}/dt, the E update of
 * a quantum cell being an implicit equation, solved on the GPU from the cell's
 * previous polarization current by Newton steps (one in FP32, two in FP64;
 * with the Cayley field step by fixed-point iterations, two and three).
 * Strong coupling runs on the blocked variant only, with one wave per 64
 * cells. */
#define MB_COUPLING_WEAK 0
#define MB_COUPLING_STRONG 1

#define MB_VARIANT_AUTO 0     /* blocked kernel, tile shape from the tuner / defaults */
#define MB_VARIANT_PLAIN 1    /* two launches per step (Alg. 1 as written), FP64 only */
#define MB_VARIANT_BLOCKED 2  /* temporally blocked overlapped tiles, FP64 or FP32 */
#define MB_VARIANT_BLOCKED_REGS 3  /* blocked; coefficients of single-material waves held in
                                    * registers (2 and 3 levels; same results as BLOCKED) */

/* ---- description ------------------------------------------------------- */
typedef struct mb_qm {
  int32_t levels;            /* N in 2..8 */
  int32_t two_level;         /* 1: use the simplified two-level form below, 0: general form */
  double n3d;                /* density of quantum systems [1/m^3] */
  /* general form (two_level == 0) */
  const double *h0_diag;     /* N reals [J] */
  const double *h0_off;      /* N(N-1)/2 complex (re, im) [J], packed by columns */
  const double *mu_diag;     /* N reals [C m] (may be NULL: zero) */
  const double *mu_off;      /* N(N-1)/2 complex (re, im) [C m] */
  const double *rates;       /* N*N, rates[i*N+j] = gamma_ij = rate j -> i [1/s] */
  const double *pure_deph;   /* N(N-1)/2 [1/s] */
  /* explicit Lindblad operators (eq:lindbladdiss with C diagonalised):
   * D(rho) = sum_k L_k rho L_k^+ - 1/2 {L_k^+ L_k, rho}.  n_lindblad > 0
   * replaces rates and pure_deph (which may then be NULL); lindblad_ops holds
   * n_lindblad matrices of N*N complex (re, im) entries, row-major, in
   * sqrt(1/s).  At most 64 operators. */
  int32_t n_lindblad;
  const double *lindblad_ops;
  /* two-level form (Sec. 3.1.1, qm_desc_2lvl): H0 = hbar w21/2 diag(-1, 1),
   * mu = -e z21 sigma_x, gamma_12 = g1 (1-w0)/2, gamma_21 = g1 (1+w0)/2,
   * gamma_12,p = g2 - g1/2 */
  double omega21, z21, gamma1, gamma2, w0;
} mb_qm;

typedef struct mb_material {
  double eps_r, mu_r;
  double alpha0;             /* field loss [1/m]; sigma = 2 alpha0 sqrt(eps/mu) (Sec. 3.1.1) */
  double overlap;            /* Gamma of eq:efield */
  const mb_qm *qm;           /* NULL: no quantum system */
} mb_material;

typedef struct mb_region {
  double x_start, x_end;     /* [m] */
  int32_t material;          /* index into the material list */
} mb_region;

typedef struct mb_device_desc {
  double length;             /* [m] */
  double refl_left, refl_right;  /* field reflectivity of each end, in [0, 1] */
  int32_t n_materials;       /* at most 255 */
  const mb_material *materials;
  int32_t n_regions;
  const mb_region *regions;
} mb_device_desc;

typedef struct mb_source {
  int32_t kind;              /* MB_SRC_* */
  int32_t hard;              /* 1 hard, 0 soft */
  double x;                  /* position [m]; the source acts at E node round(x/dx), halves
                                to the even node (Sec. 3.2 converts positions to grid
                                indices); outside [0, nx-1] after rounding: MB_ERR_ARG */
  double amp, freq, shift, width, phase, period;
  int32_t count;             /* pulses in the train (>= 1) */
  const double *table;       /* MB_SRC_TABLE: values at t_n = n dt, n = 0..table_len-1 */
  int64_t table_len;         /* (copied at setup; ignored by the other kinds) */
} mb_source;

typedef struct mb_record {
  int32_t quantity;          /* MB_REC_* */
  int32_t i, j;              /* 0-based levels */
  int64_t cell;              /* -1: every cell (nx values per sample) */
  int64_t interval;          /* steps between samples, >= 1 */
} mb_record;

typedef struct mb_consts {
  double hbar, e, c0, mu0, eps0;
} mb_consts;

typedef struct mb_scenario_desc {
  int64_t nx;                /* 1 (single-point Lindblad solve, Sec. 3.2) or >= 3 */
  double dt;                 /* [s] */
  int64_t n_steps;
  int32_t precision;         /* 64 or 32: arithmetic of the bulk field and density updates */
  int32_t variant;           /* MB_VARIANT_* */
  int32_t block;             /* blocked variant: cells per tile, 64, 128, 192, 256 or 512
                                (0 = default; 5 and 6 levels: block * lanes <= 256;
                                7 and 8 levels: 128 or 256 with one lane, weak coupling
                                and MB_FIELD_EXACT only) */
  int32_t depth;             /* blocked variant: steps per launch = halo width (0 = default) */
  int32_t coupling;          /* MB_COUPLING_WEAK (rho half a step after E, Fig. 1) or
                                MB_COUPLING_STRONG (rho at the times of E; Sec. 2.2) */
  int32_t lanes;             /* blocked variant: waves per 64 cells that share each cell's
                                density update, 1, 2, 4 or 8 (8: 4 to 6 levels, 64-cell
                                tiles; 0 = default); results do not depend on it */
  int32_t field_step;        /* MB_FIELD_EXACT or MB_FIELD_CAYLEY: the field part of the
                                density step (see below) */
  const double *rho_diag;    /* N reals: initial density matrix (ic_density_const) */
  const double *rho_off;     /* N(N-1)/2 complex (re, im) */
  const double *e_init;      /* nx initial E values, or NULL: e_const + e_noise (2 u_m - 1) */
  int32_t n_sources;
  const mb_source *sources;
  int32_t n_records;
  const mb_record *records;
  mb_consts consts;
  /* initial field without e_init (ic_field_const / ic_field_random):
   * E_m = e_const + e_noise (2 u_m - 1), u_m = the (m+1)-th output z of
   * SplitMix64 seeded with e_seed, as (z >> 11) 2^-53 in [0, 1) (e_noise = 0:
   * no draws).  Edge and hard-source cells are then set as with e_init. */
  double e_const, e_noise;
  uint64_t e_seed;
} mb_scenario_desc;

typedef struct mb_handle mb_handle;
typedef struct mb_batch mb_batch;
typedef struct mb_server mb_server;

/* Thread-local text for the last non-zero status of this thread. */
const char *mb_last_error(void);

/* Number of HIP devices visible (0 when none). */
int mb_device_count(void);

/* ---- host-only plan queries (no GPU needed) ------------------------------ */

/* Builds the FP64 plan on the host and copies the tables of material
 * `material` in the order lam[N] (ascending eigenvalues of mu), vec[2*N*N]
 * (the eigenvectors as the columns of a row-major complex N x N matrix V,
 * (re, im) pairs), kappa[N-1] (dt (lam_q - lam_{q+1}) / hbar), p0, at[M],
 * ah[M*M], bh[M], am[M*M], bf[M], t0[K], tm[K*M], sm[M*K], as[K], bm[M*K],
 * lvl[N], block with M = N*N - 1 and K = N*(N-1).  block is 1 when the
 * kernels run the simulation's tables in the block form (every quantum
 * material has a real dipole operator, H0 diagonal and relaxation in rate
 * form: see engine.hpp; MB_BLOCK_FORM=0 in the environment turns it off), else 0.
 * The tables use the operator
 * basis with the levels reordered: the caller's level i is level lvl[i] (the
 * most populated initial level is placed last, where the trace elimination
 * drops it).  The running state sigma (populations 0..N-2 and (Re, Im) of the
 * packed pairs) advances by the Strang step of Sec. 2.2 as
 *   z = t0 + tm sigma        (Re, Im) of the coherences of V^+ rho V,
 *   d = (e^{i theta} - 1) z  pair (j,k): theta = E sum_{q=j}^{k-1} kappa_q,
 *   y = sigma + sm d         the field conjugation W rho W^+,
 *   p = at . y + p0 = at . sigma + as . d + p0,
 *   sigma' = y + am y + bf = sigma + am sigma + bm d + bf,
 * and rho^{n+1/2} = ah y + bh.
 * Returns the plan status (MB_OK, MB_WARN_NOT_CP or an error). */
int mb_plan_material(const mb_device_desc *dev, const mb_scenario_desc *scen, int32_t material,
                     double *out, int64_t capacity, int64_t *n_out);

/* Readout of record `record_id` for cells of material `material`:
 * out[0] + sum_a out[1+a] sigma_a + sum_r out[1+M+r] d_r gives the recorded
 * density quantity from the running state sigma and the field increments d
 * of the step (M+1+K doubles, names as for mb_plan_material). */
int mb_plan_readout(const mb_device_desc *dev, const mb_scenario_desc *scen, int32_t record_id,
                    int32_t material, double *out, int64_t capacity);

/* Source `source_id` as planned: its E node (round(x/dx), halves to the even
 * node) into *node and the first `capacity` values of its FP64 table s(n dt),
 * n = 0..n_steps, into values (NULL: none), their count into *n_out.  Returns
 * the plan status. */
int mb_plan_source(const mb_device_desc *dev, const mb_scenario_desc *scen, int32_t source_id, int64_t *node,
                   double *values, int64_t capacity, int64_t *n_out);

/* 1 when the blocked kernel is built for tiles of `block` cells with `lanes`
 * waves per 64 cells (1, 2, 4 or 8) at this level count (0 = no quantum
 * cells, else 2..8) and precision (64 or 32), else 0.  A run asking for more
 * lanes than are built for its tile takes the largest built count below; a
 * block that is not built even with one lane is MB_ERR_UNSUPPORTED at set-up.
 * Host-only. */
int mb_tile_supported(int32_t levels, int32_t precision, int32_t block, int32_t lanes);

/* ---- single simulation --------------------------------------------------- */

/* Device bytes the simulation occupies (state planes E, H and rho twice, the
 * initial state, material, source and record tables, record buffers): the
 * size of a caller-provided mb_setup workspace.  Host-only (no GPU call);
 * errors as mb_setup's validation. */
int mb_workspace_bytes(const mb_device_desc *dev, const mb_scenario_desc *scen, size_t *bytes);

/* Validates the description, computes every FP64 table on the host
 * (coefficients a', b', c' of Sec. 3.2, the Liouvillian and its
 * exponentials, the field eigen-basis, source values, record plan), places
 * the simulation in device memory of HIP device `hip_device` and uploads the
 * initial state.
 * workspace: NULL = the library allocates (and frees in mb_destroy); else a
 * caller-owned device pointer (hipMalloc'ed on hip_device) of ws_bytes >=
 * mb_workspace_bytes, 256-byte aligned, which must stay allocated until
 * mb_destroy (the library never frees it); too small or misaligned:
 * MB_ERR_ARG.  The engine's launch tables (a few KB) and, with automatic
 * shapes, the tuner's first timing runs are still allocated by the library.
 * Returns MB_WARN_NOT_CP (with a valid handle) when a material's dephasing
 * rates admit no completely positive dissipator. */
int mb_setup(int hip_device, const mb_device_desc *dev, const mb_scenario_desc *scen, void *workspace,
             size_t ws_bytes, mb_handle **out);

/* Enqueues n_steps time steps (-1: all remaining) on `hip_stream` (a
 * hipStream_t, NULL = the legacy default stream).  Asynchronous.  The blocked
 * variant runs its full chunks as persistent launches when every tile fits on
 * the device at once and 3 depth <= block (MB_PERSIST=0 in the environment at
 * setup switches this off); otherwise, and for the tail, one launch per chunk,
 * captured into a HIP graph.  Results are the same bits either way. */
int mb_run(mb_handle *h, int64_t n_steps, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): mb_run with the same
 * arguments, results and kernels, that allocates nothing.  The run's group
 * tables (the simulation's descriptor, its tile table and the neighbour flags
 * of persistent launches: about 16 + 4 bytes per tile plus 256 per
 * simulation) are written into the library's static device scratch of this
 * GPU (1 MiB, held until the process ends) instead of buffers the handle
 * allocates; its state, coefficient and record memory were placed by
 * mb_setup.  The launches are direct (no graph) and the call returns once they
 * are queued on `hip_stream`, after a synchronous upload of the tables; no
 * elapsed time is recorded for mb_elapsed_ms.  MB_ERR_BUDGET when the tables
 * exceed the scratch (grids of more than about 40000 tiles).  Every call on a
 * GPU rewrites that GPU's scratch: calls that overlap on one GPU (from other
 * threads, or queued on different streams) race and must be serialised by the
 * caller. */
int mb_run_static(mb_handle *h, int64_t n_steps, void *hip_stream);

/* 1 when mb_run(h, n_steps) would run its full chunks as persistent launches
 * (one launch for up to 4096 chunks; tiles wait for their neighbours' flags
 * between chunks), 2 when as work-queue persistent launches (see
 * mb_batch_run_mode), 0 when every chunk is its own launch, negative on
 * error.  Uploads pending simulation tables (synchronously). */
int mb_run_mode(mb_handle *h, int64_t n_steps);

/* Restores the initial state (from a device-resident copy made at setup),
 * clears the records and sets the step count to zero, asynchronously on
 * `hip_stream`.  A later mb_run of the same length replays the HIP graph
 * captured by the first one. */
int mb_reset(mb_handle *h, void *hip_stream);

/* Steps done so far. */
int64_t mb_steps_done(const mb_handle *h);

/* Tile shape in use: cells per tile, steps per launch (1 for the two-launch
 * variant), whether coefficients are held in registers and the waves per 64
 * cells (a level count whose kernel is not built for that many uses fewer).  With
 * MB_VARIANT_AUTO and block = depth = lanes = 0 the shape is chosen at setup by timing
 * candidate shapes on this simulation (cached per device architecture, level
 * count, precision and size class; the cache file is $MB_TUNE_CACHE or
 * ~/.cache/mbhip_tune.txt).  Any pointer may be NULL. */
int mb_shape(const mb_handle *h, int32_t *block, int32_t *depth, int32_t *regs, int32_t *lanes);

/* Samples recorded so far for record `record_id` (per-sample width 1 or nx). */
int mb_record_shape(const mb_handle *h, int record_id, int64_t *n_samples, int64_t *width);

/* Synchronises the handle's last stream and copies the samples of
 * `record_id` (n_samples * width doubles, sample-major) into `out`. */
int mb_read_records(mb_handle *h, int record_id, double *out, int64_t capacity, int64_t *n_out);

/* Copies the current state into host buffers (any may be NULL):
 * e[nx], h[nx] (h[nx-1] = 0), rho[nx*N*N*2] (complex (re, im), row-major
 * N x N per cell, zero in cells without a quantum system, rho^{n-1/2}).
 * Synchronises first. */
int mb_read_state(mb_handle *h, double *e, double *hfield, double *rho);

/* Device-time of all kernels enqueued by mb_run so far, in milliseconds
 * (HIP events around each mb_run call; synchronises). */
int mb_elapsed_ms(mb_handle *h, double *ms);

int mb_destroy(mb_handle *h);

/* ---- batches: many independent simulations in one launch sequence -------- */

/* All simulations share precision and variant; the blocked variant runs
 * every level count in its own kernel per chunk, or all chunks of a two- and
 * a three-level group in one work-queue persistent launch (the batched
 * parameter sweep; see mb_batch_run_mode).  Tables and state of all members
 * live in one device allocation. */
int mb_batch_setup(int hip_device, int32_t n, const mb_device_desc *devs,
                   const mb_scenario_desc *scens, mb_batch **out);
/* Runs every member to its own n_steps (uneven lengths allowed).  When
 * use_graph != 0 the chunk launches are captured once into a HIP graph and
 * replayed. */
int mb_batch_run(mb_batch *b, void *hip_stream, int32_t use_graph);
/* Restores every member's initial state and clears the records (as mb_reset). */
int mb_batch_reset(mb_batch *b, void *hip_stream);
/* How mb_batch_run would run the full chunks of the members' remaining steps:
 * 1 persistent launches with neighbour flags (one level-count group, every
 * tile resident at once), 2 work-queue persistent launches (weak coupling and
 * the exact field step, two- and/or three-level members, one wave per 64
 * cells on tiles of 128, 192 (FP32) or 256 cells: each workgroup takes
 * (chunk, tile) items in chunk-major order from a counter and waits for the
 * tile's and its neighbours' previous chunk, so the tiles need not all be
 * resident; taken when MB_QUEUE=1 is set in the environment at set-up), 0 one
 * launch per chunk and level count;
 * negative on error.  Uploads pending tables (synchronously). */
int mb_batch_run_mode(mb_batch *b);
/* Tile shape in use (as mb_shape; tuned over the whole batch). */
int mb_batch_shape(const mb_batch *b, int32_t *block, int32_t *depth, int32_t *regs, int32_t *lanes);
int mb_batch_record_shape(const mb_batch *b, int32_t sim, int record_id, int64_t *n_samples,
                          int64_t *width);
int mb_batch_read_records(mb_batch *b, int32_t sim, int record_id, double *out,
                          int64_t capacity, int64_t *n_out);
int mb_batch_elapsed_ms(mb_batch *b, double *ms);
int mb_batch_destroy(mb_batch *b);

/* ---- serving: continuous batching of solve requests --------------------- */

/* A server owns `hbm_budget` bytes of device memory and runs up to
 * `max_slots` solves at a time in FP32 (precision 32) or FP64 (64).  Solves
 * of one level count share an engine ("lane") with its own stream; each
 * chunk of a lane advances its solves by `chunk_steps` steps (or to their
 * end), and lanes advance independently.  Between a lane's chunks finished
 * solves are retired (records copied to the host, memory freed) and queued
 * requests whose arrival time has passed are admitted while slots and memory
 * allow.  The lanes use four streams created with the server; they overlap
 * on the GPU only when the process has enough hardware queues (HIP's
 * GPU_MAX_HW_QUEUES, read at HIP start-up: at least 8 is advised, with 4
 * some lanes can end up queued behind each other).  With the environment
 * variable MB_SERVER_TRACE=<file> each server appends one line per chunk
 * (times, lane, solves, cells, tile shape) to <file> when destroyed. */
int mb_server_create(int hip_device, size_t hbm_budget, int32_t max_slots, int32_t precision,
                     int32_t chunk_steps, mb_server **out);
/* Queues a request; `arrival_s` is its arrival time in seconds after the
 * server's clock start (mb_server_start).  Returns MB_ERR_BUDGET when the
 * request alone exceeds the budget. */
int mb_server_submit(mb_server *s, const mb_device_desc *dev, const mb_scenario_desc *scen,
                     double arrival_s, uint64_t *ticket);
/* Starts the clock and the worker thread that runs the chunk loop. */
int mb_server_start(mb_server *s);
/* Blocks until every submitted request is done (or timeout_s passes: returns
 * MB_ERR_STATE). */
int mb_server_drain(mb_server *s, double timeout_s);
/* Cancels a queued or running request; it is retired at the next chunk boundary. */
int mb_server_cancel(mb_server *s, uint64_t ticket);
/* Tickets of requests that reached a final state (done, cancelled or failed;
 * mb_server_status tells which) since the previous poll, oldest first: up to
 * `capacity` of them into done[], their count in *n_done; the rest stay for
 * the next poll.  Non-blocking. */
int mb_server_poll(mb_server *s, uint64_t *done, int32_t capacity, int32_t *n_done);
/* Status of a request: 0 queued, 1 running, 2 done, 3 cancelled, or a
 * negative error it ended with.  Times (seconds on the server clock) may be NULL. */
int mb_server_status(mb_server *s, uint64_t ticket, int32_t *state, double *t_arrival,
                     double *t_admit, double *t_done);
int mb_server_record_shape(mb_server *s, uint64_t ticket, int record_id, int64_t *n_samples,
                           int64_t *width);
int mb_server_read_records(mb_server *s, uint64_t ticket, int record_id, double *out,
                           int64_t capacity, int64_t *n_out);
/* Aggregate statistics: cell-updates done and busy wall time in seconds. */
int mb_server_stats(mb_server *s, double *cell_updates, double *busy_s, int64_t *chunks);
int mb_server_destroy(mb_server *s);

#ifdef __cplusplus
}
#endif
#endif /* MB_H */
