/*
 * fnlh.h -- C ABI of libfnlh, the MI355X (gfx950) solver for the shared-Jacobian,
 * frequency-shifted block-sparse linear systems of the implicit FNLH scheme
 * (Wang, Weber, Radford, di Mare, Meyer, "Convergence Acceleration of Favre-Averaged
 * Non-Linear Harmonic Method", arXiv 2404.01407).
 *
 * What is solved.  Section "Generalized RK Scheme for The Mean Flow" defines the
 * preconditioner matrix K = P/(eps sigma_CFL) + J (implicit) or K = P (explicit), with J
 * the first-order residual Jacobian (6x6 blocks: five flow variables plus the
 * Spalart-Allmaras variable) and P its block diagonal.  Section "Generalized RK Scheme
 * for Time-Linearized Harmonic Flows" adds i omega_l V I to the diagonal of K for
 * harmonic l; the sparsity pattern is shared by the mean flow and every harmonic.
 * Section "Solution Update" writes each RK stage as A x = B with A = K/(Gamma alpha_k)
 * and, for harmonic l, (A + i omega_l I V/(Gamma alpha_k)) x = B; multiplying by
 * Gamma alpha_k gives the canonical system solved here,
 *
 *       (K + i omega_{z(i),s} V_i I) x_s = b_s,      s = 0 .. n_sys-1,
 *
 * with b_s = Gamma alpha_k B_s supplied by the caller.  K is stored once; the shift
 * is applied on the fly, so matrix memory does not depend on the number of systems.
 * System s with omega row == 0 is the mean flow.
 *
 * How.  Each system is solved by preconditioned Richardson iteration
 * x <- x + M^-1 (b - K_s x), the paper's "ILU(0) used as a smoother, solved
 * iteratively and inexactly" (section "Solution Update"), with M one of
 *   FNLH_DILU    (D~ + L) D~^-1 (D~ + U) on a colour ordering (equals block ILU(0) when
 *                the cell graph has no triangles, e.g. every hex mesh),
 *   FNLH_SGS     (D + L) D^-1 (D + U),
 *   FNLH_JACOBI  block diagonal (the paper's explicit, point-by-point inversion),
 *   FNLH_PILU    ILU(0) inside each partition of fnlh_set_partitions, in the natural
 *                (cell id) order, the couplings between partitions left out (section
 *                "Parallel Implementation"; DILU on that order, which is ILU(0) when
 *                the cell graph has no triangles).
 * The stopping test is the paper's relative 2-norm of B - A x (section "Results",
 * key-parameter table: 1e-2 and 10 iterations there; any rtol / max here).
 *
 * Conventions for every call:
 *   - return value: FNLH_OK (0), a positive solver outcome, or a negative error code;
 *     no C++ exception crosses the ABI.  fnlh_last_error() gives a message.
 *   - "host" pointers are read during the call only; the caller keeps ownership.
 *   - "device" pointers are HIP device memory on the context's device (e.g. the data
 *     pointer of a torch tensor); the caller owns them.  The library owns its mesh
 *     copy, blocks, factor slots and scratch, all released by fnlh_destroy.
 *   - vectors cross the ABI in user cell order as interleaved complex128, [N][6]
 *     (12 doubles per cell: re0, im0, ..., re5, im5).
 *   - stream: a hipStream_t passed as void*; NULL is the default stream.  Work is
 *     stream-ordered; calls that return numbers to the host synchronise that stream.
 *   - call order: create -> (assemble_jacobian | set_blocks) -> set_harmonics ->
 *     (relax | residual)*.  Anything else returns FNLH_E_ORDER.  Re-assembly or new
 *     blocks invalidate all factors; set_harmonics invalidates the factors too.
 *   - a context is not thread-safe; use one context per host thread / stream.
 */
#ifndef FNLH_H
#define FNLH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fnlh_ctx_s* fnlh_ctx;

/* status codes.  Solver outcomes are > 0; the worst over several systems is reported
 * in the order OK < FELL_BACK < NOT_CONVERGED < DIVERGED. */
enum {
  FNLH_OK = 0,
  FNLH_NOT_CONVERGED = 1, /* max_sweeps reached above the tolerance            */
  FNLH_DIVERGED = 2,      /* NaN/Inf or ||r|| > div_factor ||r0||               */
  FNLH_FELL_BACK = 3,     /* FNLH_LEARNED: converged, but the network's corrections
                             were switched off for the system after three rejections
                             in a row (the plain sweeps finished the solve)          */
  FNLH_E_ARG = -1,        /* invalid argument                                   */
  FNLH_E_MESH = -2,       /* invalid mesh (ids, duplicates, volumes, colouring) */
  FNLH_E_SINGULAR = -3,   /* a diagonal block to invert is singular / not finite */
  FNLH_E_OOM = -4,        /* device allocation failed                           */
  FNLH_E_HIP = -5,        /* HIP runtime error (incl. no device)                */
  FNLH_E_ORDER = -6       /* call made in the wrong order                       */
};

/* block storage precision (matrix K and its shadow).  The factor inverses D~^-1 are FP64
 * with FP64 blocks and FP16 with a power-of-two scale per row otherwise: they only shape
 * the preconditioner, whose precision the FP64 outer residual makes irrelevant to the
 * converged result. */
enum { FNLH_F64 = 0, FNLH_F32 = 1, FNLH_BF16 = 2 };
/* operator of the outer (FP64) residual in reduced-precision modes:
 *   EXACT  - the FP64 operator: recomputed from the FP64 state and geometry after
 *            fnlh_assemble_jacobian, an FP64 copy of the blocks after fnlh_set_blocks;
 *            the iteration converges to the FP64 solution (defect correction).
 *   STORED - FP64 arithmetic on the upcast stored blocks: converges to the solution
 *            of the rounded system. */
enum { FNLH_OUTER_EXACT = 0, FNLH_OUTER_STORED = 1 };
/* colour ordering: AUTO = two colours when the cell graph is bipartite, else greedy */
enum { FNLH_ORDER_AUTO = 0, FNLH_ORDER_GREEDY = 1, FNLH_ORDER_BIPARTITE = 2, FNLH_ORDER_USER = 3 };
/* preconditioner */
enum { FNLH_DILU = 0, FNLH_SGS = 1, FNLH_JACOBI = 2, FNLH_LEARNED = 3, FNLH_PILU = 4 };
/* scheme of the preconditioner matrix (section "Generalized RK Scheme for The Mean Flow") */
enum { FNLH_IMPLICIT = 0, FNLH_EXPLICIT = 1 };

/* Mesh of node-centred control volumes as an edge list (section "Brief Description
 * of Hydra": edge-based finite volume).  All pointers are host memory. */
typedef struct {
  int64_t n_cells;            /* N > 0                                                */
  int64_t n_edges;            /* E >= 0 interior faces                                */
  int64_t n_bfaces;           /* B >= 0 boundary faces                                */
  int32_t n_zones;            /* >= 1; omega is given per zone (e.g. per blade row)   */
  int32_t pad_;
  const int32_t* edges;       /* [E][2] cell ids (a, b), a != b, no duplicate pairs   */
  const double* area;         /* [E][3] face area vector oriented from a to b         */
  const double* volume;       /* [N] control volumes, > 0                             */
  const int32_t* zone;        /* [N] zone of each cell in [0, n_zones), or NULL       */
  const int32_t* bface_cell;  /* [B] owning cell of each boundary face                */
  const double* bface_area;   /* [B][3] outward area vector                           */
} fnlh_mesh;

typedef struct {
  int32_t storage;            /* FNLH_F64 | FNLH_F32 | FNLH_BF16                        */
  int32_t outer;              /* FNLH_OUTER_EXACT | FNLH_OUTER_STORED                   */
  int32_t ordering;           /* FNLH_ORDER_*                                           */
  int32_t factor_slots;       /* D~^-1 slots kept at once; 0 = one per system           */
  const int32_t* user_colour; /* host [N] colour per cell if ordering == USER; classes
                                 must be independent sets, taken in ascending value    */
  int32_t device;             /* HIP device ordinal                                     */
  int32_t pad_;
} fnlh_options;

/* Create a context: validates and copies the mesh, builds the colour ordering, the
 * colour-major internal numbering (locality-ordered within each colour) and the
 * sliced-ELL block layout, and allocates the matrix on the device.
 * Errors: FNLH_E_ARG (null pointers, bad option values), FNLH_E_MESH (ids out of range,
 * self or duplicate edges, volume <= 0, zone out of range, invalid user colouring),
 * FNLH_E_HIP / FNLH_E_OOM (device).  *out is NULL on failure. */
int fnlh_create(fnlh_ctx* out, const fnlh_mesh* mesh, const fnlh_options* opts);
int fnlh_destroy(fnlh_ctx c);

/* Assemble K on the device from the FP64 state (section "Generalized RK Scheme for The
 * Mean Flow"): J from first-order Rusanov flux Jacobians with a frozen spectral radius
 * (stand-in for the paper's first-order approximate Jacobian), boundary faces against a
 * frozen far-field state, P = blockdiag(J), K = J + P/(eps sigma) (FNLH_IMPLICIT) or
 * K = P (FNLH_EXPLICIT); stored in the context's precision.
 *   state  device [N][6] conservative (rho, rho u, rho v, rho w, rho E, rho nu~), user order
 *   bstate device [B][6] far-field state per boundary face, or NULL (= owning cell's state)
 * Errors: FNLH_E_ARG (eps*sigma <= 0, null state), FNLH_E_HIP. */
int fnlh_assemble_jacobian(fnlh_ctx c, const double* state, const double* bstate, double eps,
                           double sigma, int32_t scheme, void* stream);

/* Set K from raw FP64 blocks instead (any matrix with the mesh's pattern).
 *   diag device [N][6][6]   K_ii, row-major, user order
 *   offd device [E][2][6][6] per edge e = (a, b): K_ab then K_ba, row-major */
int fnlh_set_blocks(fnlh_ctx c, const double* diag, const double* offd, void* stream);

/* Read back the stored blocks (upcast to FP64) in the layouts of fnlh_set_blocks. */
int fnlh_get_blocks(fnlh_ctx c, double* diag, double* offd, void* stream);

/* Frequencies: host [n_sys][n_zones] omega_{z,s} (section "Generalized RK Scheme for
 * Time-Linearized Harmonic Flows"; omega indexed per zone, cf. the harmonic series with
 * omega_{i,l}).  Invalidates factors.  1 <= n_sys <= 4096. */
int fnlh_set_harmonics(fnlh_ctx c, int32_t n_sys, const double* omega, void* stream);

/* Phase-lagged periodic couplings (section "Solution Update": on periodic boundaries each
 * harmonic carries its own inter-blade phase angle, which changes its left-hand side but
 * not the sparsity pattern).  edge_phase host [E]: 0 for an ordinary edge; +1 (-1) when
 * edge e = (a, b) couples a to the image of b one pitch above (below), whose value is
 * x_b e^{+i sigma} (e^{-i sigma}); row a's coupling K_ab is then applied to
 * x_b e^{i s sigma_s} and row b's K_ba to x_a e^{-i s sigma_s}.  sigma host [n_sys]: the
 * phase of every system (radians; 0 for the mean), n_sys as in fnlh_set_harmonics.
 * Applied on the fly in every sweep and residual; the DILU factors do not depend on it
 * (a coupling and its transpose carry conjugate phases), so no factor is invalidated.
 * edge_phase NULL removes the couplings' phases.  fnlh_set_harmonics resets every
 * system's phase to 0.  Errors: FNLH_E_ORDER before set_harmonics, FNLH_E_ARG for signs
 * outside {-1, 0, 1}, a wrong system count or non-finite phases. */
int fnlh_set_phase_lag(fnlh_ctx c, const int8_t* edge_phase, int32_t n_sys, const double* sigma);

/* r = b - K_s x with the outer FP64 operator (see FNLH_OUTER_*).
 *   x, b device [N][6] complex128 user order; r device [N][6] or NULL;
 *   norm2 host out: ||r||_2^2 over all 6N complex entries (may be NULL). */
int fnlh_residual(fnlh_ctx c, int32_t sys, const double* x, const double* b, double* r,
                  double* norm2, void* stream);

typedef struct {
  int32_t kind;          /* FNLH_DILU | FNLH_SGS | FNLH_JACOBI | FNLH_LEARNED | FNLH_PILU   */
  int32_t max_sweeps;    /* >= 0: total preconditioned sweeps per system                  */
  double rtol;           /* stop when ||b - K_s x|| <= rtol ||b - K_s x0||                 */
  int32_t check_every;   /* sweeps between host read-backs of the device stop flags (>=1) */
  int32_t inner_sweeps;  /* reduced precision: max inner sweeps per FP64 correction (0=auto) */
  double inner_rtol;     /* reduced precision: inner relative tolerance (0 = auto)          */
  double div_factor;     /* DIVERGED when ||r|| > div_factor ||r0|| (0 = 1e3)               */
  int32_t use_graph;     /* 1: replay check_every sweeps as one captured hipGraph            */
  int32_t learn_every;   /* FNLH_LEARNED, FP64 blocks: sweeps between learned corrections (0 = 16) */
  double* history;       /* host [n][history_len] or NULL: residual history per system (fnlh_relax) */
  int32_t history_len;   /* entries per system                                                */
  int32_t pad_;
} fnlh_relax_opts;

typedef struct {
  int32_t sweeps;        /* preconditioned sweeps applied                                 */
  int32_t outer;         /* FP64 outer corrections (reduced precision), else 0            */
  int32_t status;        /* FNLH_OK | FNLH_NOT_CONVERGED | FNLH_DIVERGED                  */
  int32_t fallbacks;     /* FNLH_LEARNED: learned corrections rejected (plain sweeps kept)   */
  double rel_res;        /* ||b - K_s x|| / ||b - K_s x0|| of the returned x, outer operator */
  double res0;           /* ||b - K_s x0||                                                 */
  double t_factor_ms;    /* time in factorisation (device events)                          */
  double t_sweep_ms;     /* time in sweeps and residuals (device events)                   */
  int32_t learned;       /* FNLH_LEARNED: learned corrections accepted                      */
  int32_t pad_;
} fnlh_sys_report;

/* FNLH_LEARNED runs the FNLH_DILU sweeps of this call and, every learn_every sweeps
 * (in reduced precision: after every FP64 correction, i.e. every inner solve, whose
 * length inner_sweeps / inner_rtol set), a correction by the network attached with
 * fnlh_nn_create: with r the FP64
 * residual of x and dx the network's output for r, x <- x + alpha dx with the complex
 * alpha minimising ||r - alpha K_s dx||.  The FP64 residual judges every correction:
 * one that is not finite or lowers ||r||^2 by less than 0.1% is rejected (counted in
 * fallbacks) and the sweeps go on from the unchanged x.  After three rejections in a row
 * a system gets no more corrections in this call (the network is not evaluated for it
 * any more; an accepted correction resets the run), and if it then converges its
 * status is FNLH_FELL_BACK.
 *
 * Solve n systems: sys[j] indexes the omega table, x[j] (in: x0, out: x) and b[j] are
 * device [N][6] complex128 user-order buffers (host arrays of n device pointers).
 * Returns the worst per-system status (FNLH_OK if all converged) or an error.
 * The tolerance test is evaluated on the residual of the previous iterate, computed
 * inside the sweep; the returned x is one sweep past the first iterate that met it and
 * rel_res is recomputed for it with the outer operator.
 * history (opts, optional): entry m of system j is ||b - K_s x^m|| after m sweeps as the
 * stop test measured it (entry 0 the initial residual; FP64 blocks: the FP64 residual of
 * every sweep; FP32/BF16 blocks: the FP64 residual after each outer correction and, in
 * between, the inner iteration's residual of the stored operator), entry sweeps the
 * returned x's (rel_res times res0), NaN beyond; at most history_len entries.  The
 * batched relax ignores it.
 * FNLH_PILU (section "Parallel Implementation"): each partition of fnlh_set_partitions
 * is factored and swept on its own by one workgroup, in the natural order of its cells
 * (level by level), with its y vector in LDS; FNLH_E_ORDER without partitions,
 * FNLH_E_ARG when the largest partition's y does not fit in a workgroup's LDS (the
 * device's limit less 1 KiB, 159 KiB on MI355X: at most 3392 cells with FP32/BF16
 * blocks, 1696 with FP64).  The first use after new
 * partitions builds the position layout on the host; the first factorisation after new
 * blocks copies the in-partition couplings into position order (device memory about
 * that of the off-diagonal blocks). */
int fnlh_relax(fnlh_ctx c, int32_t n, const int32_t* sys, double* const* x,
               const double* const* b, const fnlh_relax_opts* opts, fnlh_sys_report* rep,
               void* stream);

/* The residual of fnlh_residual without allocating: for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Computes r = b - K_s x with the same kernels and the same summation order
 * as fnlh_residual (bitwise the same r and norm), but its staging vectors, per-tile
 * partials and reduction state live in a file-scope device array of
 * fnlh_noalloc_scratch_bytes() bytes (64 MiB) that each device holds from the library's
 * first context on it until the process ends, instead of buffers the context allocates.
 * No hipMalloc, hipFree or allocating library call; no host synchronisation.
 *   x, b device [N][6] complex128 user order (caller-owned); r device [N][6] or NULL;
 *   norm2 DEVICE double [1] or NULL: receives ||r||_2^2 (stream-ordered).
 * The scratch holds 2 (3 with r) vectors of 96 x padded rows plus 8 bytes per 64-row
 * tile: at most about 233,000 cells with r; a larger mesh returns FNLH_E_ARG with the
 * needed size.  Every call on one device shares that device's array and leaves its
 * contents behind (nothing is read before it is written in the next call): calls that
 * overlap on one device (two streams, two host threads) race and give wrong results.
 * Needs matrix and harmonics (FNLH_E_ORDER). */
int fnlh_residual_noalloc(fnlh_ctx c, int32_t sys, const double* x, const double* b, double* r,
                          double* norm2, void* stream);
size_t fnlh_noalloc_scratch_bytes(void);

/* Ordering actually used: colour per cell (user order, host out [N]) and the count. */
int fnlh_get_ordering(fnlh_ctx c, int32_t* colour_of_cell, int32_t* n_colours);

/* Device bytes held: matrix (blocks, shadow, pattern), factor slots, vectors/scratch. */
int fnlh_memory(fnlh_ctx c, size_t* matrix_bytes, size_t* factor_bytes, size_t* vector_bytes);

/* Message of the last error on this context (or of the last failed fnlh_create when
 * c is NULL).  Valid until the next call on the same context. */
const char* fnlh_last_error(fnlh_ctx c);

/* Host-only helpers (no device needed): mesh validation and the ordering fnlh_create
 * would build.  colour [N] and perm [N] (internal position of each user cell) are host
 * outputs and may be NULL.  Same error codes as fnlh_create. */
int fnlh_order_mesh(const fnlh_mesh* mesh, const fnlh_options* opts, int32_t* colour,
                    int32_t* perm, int32_t* n_colours);

/* ---- batching: many independent instances (e.g. blade rows of different sizes, each
 * with its own mean + harmonics) solved together.  The harmonic systems are decoupled
 * (section "Favre-averaged Non-Linear Harmonic Method": cross-coupling of harmonics is
 * ignored) and so are the instances, so every sweep phase of every instance can run in
 * one launch.  Each instance keeps its own context (matrix, factors, stop state); the
 * batch groups the instances by system count and, per sweep, issues one launch per
 * group and colour phase over a concatenated (instance, tile) work list plus one
 * reduction for all (instance, system) pairs; check_every sweeps are replayed as one
 * captured hipGraph when use_graph is set.  Every system stops on its own tolerance.
 * Instances whose ordering is not two-coloured, or with more systems than one launch
 * handles (16, or fewer factor slots), are solved one by one with fnlh_relax. */
typedef struct fnlh_batch_s* fnlh_batch;
/* inst: n contexts on the same device with the same storage precision (host array);
 * the contexts must outlive the batch. */
int fnlh_batch_create(fnlh_batch* out, int32_t n, const fnlh_ctx* inst);
int fnlh_batch_destroy(fnlh_batch b);
/* Per instance i: n_sys[i] systems sys[i][j], vectors x[i][j] (in: x0, out: x) and
 * b[i][j] as in fnlh_relax.  rep has sum(n_sys) entries in instance order.
 * opts.kind is FNLH_DILU, FNLH_SGS or FNLH_LEARNED (every instance then needs a network
 * with weights; the learned corrections run per instance between batched chunks of
 * learn_every sweeps, or after every FP64 correction in reduced precision).  Returns
 * the worst status. */
int fnlh_batch_relax(fnlh_batch b, const int32_t* n_sys, const int32_t* const* sys, double* const* const* x,
                     const double* const* const* bvec, const fnlh_relax_opts* opts, fnlh_sys_report* rep,
                     void* stream);
const char* fnlh_batch_last_error(fnlh_batch b);
/* Batch scheduling: instances of at least loop_cells cells are iterated one after
 * another (each with its own sweep loop, as fnlh_relax does) instead of in the shared
 * launches; smaller instances stay batched.  An instance iterated alone keeps its blocks
 * largely cache-resident (MI355X's 256 MB Infinity Cache) from one sweep to the next,
 * while a batched sweep streams every instance through it; launch overhead favours
 * batching only for small instances.  Default 80,000 cells; loop_cells <= 0: every
 * eligible instance batched.  Results are the same either way (the batched and
 * per-instance sweeps are bitwise equal). */
int fnlh_batch_set_loop_cells(fnlh_batch b, int64_t loop_cells);
/* Batch autotuner: for each of the n_cand (1..64) candidate thresholds cand[k] (cells;
 * <= 0 batches every eligible instance) it runs fnlh_batch_relax with the arguments given
 * from a zero start, once to warm up and once timed with events on the stream (ms[k],
 * may be NULL), keeps the fastest threshold on the batch (*pick, may be NULL) and solves
 * once more with it: x is overwritten and holds that solve's result.  The instance
 * contexts' own settings (fnlh_autotune) are left as they are.  Returns the status of
 * the last solve. */
int fnlh_batch_autotune(fnlh_batch b, const int32_t* n_sys, const int32_t* const* sys, double* const* const* x,
                        const double* const* const* bvec, const fnlh_relax_opts* opts, int32_t n_cand,
                        const int64_t* cand, int64_t* pick, double* ms, void* stream);

/* Kernel timing of the sweep passes.  While enabled, every sweep-pass launch is
 * bracketed by HIP events on the caller's stream; durations and the algorithmic bytes
 * of each launch (blocks once per launch, per active system: D~^-1, own vectors, and
 * each distinct neighbour vector once) are accumulated per kernel kind. */
typedef struct {
  int64_t launches;  /* launches timed                     */
  double total_ms;   /* sum of event-measured durations    */
  double alg_bytes;  /* sum of algorithmic bytes           */
} fnlh_kernel_stats;
enum {
  FNLH_KSTAT_SWEEP_UPDATE = 0, /* two-colour pass over the second colour (reads K_ii) */
  FNLH_KSTAT_SWEEP_SET = 1,    /* two-colour pass over the first colour              */
  FNLH_KSTAT_FWD = 2,          /* general colouring, forward pass (all but the last colour) */
  FNLH_KSTAT_BWD = 3,          /* general colouring, backward pass                    */
  FNLH_KSTAT_JACOBI = 4,       /* block Jacobi pass                                   */
  FNLH_KSTAT_FWD_LAST = 5,     /* general colouring, forward pass of the last colour  */
  FNLH_KSTAT_REMAINDER = 6,    /* two colours plus remainder: the passes over the
                                  colours past the second and the correction of the
                                  second colour's rows coupled to them                */
  FNLH_KSTAT_PILU = 7,         /* partition-local ILU(0) sweep                          */
  FNLH_KSTAT_N = 8
};
/* on >= 1 resets the counters and starts timing the launches of every on-th sweep
 * (1 = every launch; a larger period bounds the event overhead); on = 0 stops.
 * While timing, sweeps are launched directly even if use_graph is set. */
int fnlh_stats_enable(fnlh_ctx c, int32_t on);
int fnlh_stats_get(fnlh_ctx c, int32_t which, fnlh_kernel_stats* out);

/* Tuning knobs (chosen by an autotuner or the caller; results do not depend on them
 * beyond floating-point summation order):
 *   FNLH_TUNE_SYS_PER_LANE  minimum systems a lane of the sweep kernels carries: 1, 2
 *                           or 4 (0 = automatic).
 *   FNLH_TUNE_LANES_PER_ROW lanes sharing one row in the two-colour pass: 1, 2 or 4
 *                           (0 = automatic: min(4, systems)).
 *   FNLH_TUNE_WAVE_GROUPS   two-colour pass workgroups: 1 = one wave per workgroup
 *                           (default; finer dispatch), 0 = one 64-row tile per
 *                           workgroup (its waves together); bitwise the same results.
 *   FNLH_TUNE_HYBRID        colourings with more than two colours whose colours past
 *                           the second hold at most a quarter of the rows (e.g. the
 *                           interface rows of a multi-row sector): 1 = sweep them as
 *                           the two-colour passes plus passes over the remainder
 *                           (default; each block of the first two colours read once per
 *                           sweep), 0 = the general forward/backward passes, 2 = the
 *                           hybrid passes for any colouring of three or more colours.
 *                           The same preconditioner either way (equal iterates up to
 *                           rounding).
 *   FNLH_TUNE_PILU_UNIT     FNLH_PILU: cells per work unit, the consecutive partitions
 *                           (by label) that one workgroup sweeps together, their levels
 *                           merged (a larger partition is a unit of its own); 0 =
 *                           automatic (N / 2048, between 64 and 1024).  More cells per
 *                           unit fill the wave's lanes on small partitions, fewer give
 *                           more workgroups.  Bitwise the same results.
 *   FNLH_TUNE_PILU_THREADS  FNLH_PILU: lanes of a sweep workgroup, four per row of a
 *                           level: 64, 128 or 256 (0 = automatic, after the units'
 *                           average level width).  Bitwise the same results.
 */
enum {
  FNLH_TUNE_SYS_PER_LANE = 0,
  FNLH_TUNE_LANES_PER_ROW = 1,
  FNLH_TUNE_WAVE_GROUPS = 2,
  FNLH_TUNE_HYBRID = 3,
  FNLH_TUNE_PILU_UNIT = 4,
  FNLH_TUNE_PILU_THREADS = 5
};
int fnlh_tune(fnlh_ctx c, int32_t param, int32_t value);

/* Autotuner: picks the sweep configuration by the time of whole solves.  For every
 * candidate (path: two-colour plus remainder or general passes when the ordering has
 * three or more colours; kernel shape: lanes per row 1/2/4 x systems per lane 1/2/4 or
 * automatic; one wave or one tile per workgroup) it solves the first n_sys systems
 * (right-hand side of ones, zero start, graph replay) to rtol with at most max_sweeps
 * sweeps (rtol 0: exactly max_sweeps sweeps), once to warm up (factors, graphs) and
 * twice timed with events on the stream, and keeps the fastest on the context (as
 * fnlh_tune would).  The candidates give the same iterates up to rounding (bitwise for
 * the kernel shape and workgroup mapping).  Requires harmonics; allocates two
 * n_sys-vector buffers for the call.  out (may be NULL) receives the choice, its time
 * and that of the first (default) candidate. */
typedef struct {
  int32_t lanes_per_row;   /* 0 = automatic */
  int32_t sys_per_lane;    /* 0 = automatic */
  int32_t wave_groups;     /* 1 = one wave per workgroup */
  int32_t hybrid;          /* path knob (FNLH_TUNE_HYBRID)  */
  double ms_best;          /* fastest solve of the pick (ms)  */
  double ms_default;       /* the default configuration's      */
  int32_t sweeps;          /* sweeps of the pick's solve, summed over the systems */
  int32_t candidates;      /* configurations timed */
} fnlh_tune_result;
int fnlh_autotune(fnlh_ctx c, int32_t n_sys, double rtol, int32_t max_sweeps, fnlh_tune_result* out,
                  void* stream);

/* ---- Krylov solve: restarted flexible GMRES around the same preconditioners (section
 * "Generalized RK Scheme for The Mean Flow": the ILU(0) approximation of K^-1 is used
 * either as a smoother, fnlh_relax, or as the preconditioner of a Newton-Krylov method;
 * the paper gives no Krylov algorithm, this is the textbook FGMRES(m) with right
 * preconditioning).  Per iteration j: z_j = M^-1 v_j, `inner_sweeps` preconditioned
 * Richardson sweeps from 0 (one sweep is exactly M^-1 of DILU, SGS or Jacobi; FP32/BF16
 * sweeps for reduced storage).  FNLH_LEARNED makes M^-1 nonlinear, which the flexible
 * method admits: z_j = alpha d + e, with d the attached network's correction for the
 * residual v_j (fnlh_nn_create), alpha the complex step minimising ||v_j - alpha K d||
 * (set to 0 where it is not finite or lowers ||v_j||^2 by less than 1e-3 of itself),
 * and e from `inner_sweeps` DILU sweeps from 0 on K e = v_j - alpha K d.  Then
 * w = (K + i omega V) z_j with the FP64 operator, orthogonalised against v_0..v_j by
 * classical Gram-Schmidt with a second pass where the norm falls below 1/sqrt(2) of
 * its value (DGKS), Givens rotations on the host; x += Z y at the end of each cycle of
 * `restart` iterations, and the next cycle starts from the true residual.  Inner products sum conj(u) v over all 6N complex
 * entries.  Stop when the residual norm (the least-squares one within a cycle, the true
 * one at a restart) is <= rtol ||r0||, after max_iters iterations, or on breakdown. */
typedef struct {
  int32_t kind;          /* FNLH_DILU, FNLH_SGS, FNLH_JACOBI, FNLH_LEARNED or FNLH_PILU: M */
  int32_t restart;       /* Krylov vectors per cycle, 1..256                               */
  int32_t max_iters;     /* total iterations (preconditioner applications) per system     */
  int32_t inner_sweeps;  /* sweeps per preconditioner application, >= 1                   */
  double rtol;           /* relative residual target                                        */
  int32_t use_graph;     /* replay the inner sweeps from HIP graphs                         */
  int32_t pad_;
} fnlh_gmres_opts;
typedef struct {
  int32_t iters, restarts, status;
  int32_t learned;       /* FNLH_LEARNED: preconditioner applications that kept the
                            network's correction (the others: iters - learned)             */
  double rel_res;        /* ||b - A x|| / ||b - A x0|| of the returned x (true residual, FP64) */
  double res0;           /* ||b - A x0||                                                     */
  double t_ms;           /* wall time of the call on the stream (all systems)               */
} fnlh_gmres_report;
/* n systems (1..16) of the set harmonics, solved together (each block read of the
 * preconditioner sweeps and operator products serves all of them): x[j], b[j] device
 * [N][6] complex128 (x in: x0, out: x), sys[j] their harmonic rows.  rep: host [n] or
 * NULL.  history: host [n][max_iters + 1] or NULL, the residual norm after each
 * iteration (index 0: ||r0||; least-squares norms within a cycle).  Device memory:
 * (2 restart + 2) vectors of 96 N n bytes besides the context's.  Frozen-turbulence and
 * phase-lagged systems are handled as in fnlh_relax (FNLH_LEARNED takes no
 * frozen-turbulence system).  Returns the worst status or an error (FNLH_E_ARG on bad
 * options, a frozen system with FNLH_LEARNED, or more systems than factor slots;
 * FNLH_E_ORDER for FNLH_LEARNED without a network with weights). */
int fnlh_gmres(fnlh_ctx c, int32_t n, const int32_t* sys, double* const* x, const double* const* b,
               const fnlh_gmres_opts* o, fnlh_gmres_report* rep, double* history, void* stream);

/* Partition-dropped couplings (section "Parallel Implementation": the LHS is split over
 * processors by a domain decomposition and the entries that couple two nodes of different
 * partitions are ignored, so each partition solves its own sub-system; convergence
 * degrades as the partitions shrink).  part [N] host, user order: the partition of each
 * cell (any int32 labels); NULL clears.  Every coupling (K_ab and K_ba) between cells of
 * different partitions is left out of the matrix the solves use: fnlh_relax, fnlh_gmres,
 * fnlh_residual and the stage solves of the RK driver work with that K (diagonal blocks
 * whole), while the RK residuals keep every coupling.  Applied at once to a matrix that
 * is present and to every later fnlh_assemble_jacobian / fnlh_set_blocks (the dropped
 * blocks are stored as zeros, and fnlh_get_blocks returns them so).  Changing or clearing
 * partitions that were already applied needs the matrix again (relax returns
 * FNLH_E_ORDER until fnlh_assemble_jacobian or fnlh_set_blocks).  Setting the same
 * couplings again is a no-op. */
int fnlh_set_partitions(fnlh_ctx c, const int32_t* part, void* stream);

/* Frozen turbulence (section "Brief Description of Hydra": the harmonic equations are
 * linearised with the turbulence model frozen, so the unit matrix of the frequency shift
 * in section "Generalized RK Scheme for Time-Linearized Harmonic Flows" is 5x5).
 * flags [n_sys] host, 1 = that system solves only the leading 5x5 sub-system of every
 * block with its sixth unknown held at zero, 0 = the full 6x6 system; NULL clears all.
 * For a frozen system fnlh_relax sets x's sixth component to 0 and keeps it there,
 * ignores b's, and leaves the sixth equation's residual out of every norm; fnlh_residual
 * takes x's sixth component as 0 and returns that residual component as 0.  Frozen
 * systems use the stored-factor kernels (not the two-colour fused pass) and cannot use
 * FNLH_LEARNED.  Cleared by fnlh_set_harmonics.  Errors: FNLH_E_ORDER before
 * set_harmonics, FNLH_E_ARG on a wrong count or a flag other than 0/1. */
int fnlh_set_frozen_turbulence(fnlh_ctx c, int32_t n_sys, const int8_t* flags);

/* ---- pseudo-time driver: the RK(5,3) scheme around the linear solve (section
 * "Generalized RK Scheme for The Mean Flow", eqn:rk and the hybrid RK(5,3) coefficient
 * table alpha = (1/4, 1/6, 3/8, 1/2, 1); section "Generalized RK Scheme for
 * Time-Linearized Harmonic Flows", eqn:rk_lin; section "Solution Update").  Per
 * pseudo-time step: Q^(0) = Q^n, Q^(k) = Q^(0) + x_k with K x_k = -Gamma alpha_k R^(k)
 * solved by fnlh_relax with the options lin (the paper's setting: rtol 1e-2, at most 10
 * sweeps), Gamma = 1/eps (implicit) or sigma (explicit).  The residual stand-in is the
 * first-order Rusanov residual (no viscous part, so the table's beta blending has no
 * effect).  Returns the worst stage-solve status (FNLH_NOT_CONVERGED is the normal
 * outcome of an inexact stage solve) or an error. */

/* R(Q) = sum over faces of 1/2 (F(Q_i) + F(Q_k)) - 1/2 lambda (Q_k - Q_i), lambda the
 * larger end spectral radius, boundary faces against bstate (device [B][6]) or the
 * cell's own state when NULL.  state device [N][6] user order; R device [N][6]; norm2
 * host ||R||^2 or NULL.  Needs only the mesh. */
int fnlh_rusanov_residual(fnlh_ctx c, const double* state, const double* bstate, double* R,
                          double* norm2, void* stream);
/* n_steps pseudo-time steps of the mean flow: state (device [N][6], in/out) is updated in
 * place; K is re-assembled at every step (fnlh_assemble_jacobian with eps, sigma,
 * scheme) and kept through its five stages.  sys: a system whose omega is 0 (the mean).
 * res_norm host [n_steps] or NULL: ||R(Q^n)|| at the start of each step. */
int fnlh_rk_mean(fnlh_ctx c, int32_t sys, double* state, const double* bstate, int32_t n_steps,
                 double eps, double sigma, int32_t scheme, const fnlh_relax_opts* lin,
                 double* res_norm, void* stream);
/* n_steps pseudo-time steps of harmonic sys about the assembled state: residual
 * R(q^) = (J + i omega V) q^ - f^ (J the residual Jacobian, matrix-free in FP64, with the
 * phase-lagged couplings if set), stage solves with K + i omega V; qhat device [N][6]
 * complex128 in/out (its sixth component set to 0 first for a frozen-turbulence system),
 * fhat device [N][6].  Its fixed point is the solution of
 * (J + i omega V) q^ = f^.  Needs fnlh_assemble_jacobian (Gamma from its eps, sigma,
 * scheme). */
int fnlh_rk_harmonic(fnlh_ctx c, int32_t sys, double* qhat, const double* fhat, int32_t n_steps,
                     const fnlh_relax_opts* lin, double* res_norm, void* stream);

/* ---- learned preconditioner (a project addition; the paper has no learned part).
 * A two-layer per-edge message-passing network on the context's cell graph maps the
 * residual r of system s to a correction dx ~ K_s^-1 r:
 *   sigma = sqrt(sum |r|^2 / (12 N)),  z_i = (K_ii + i omega V_i I)^-1 r_i,
 *   u_i = [r_i, z_i] / sigma (24 reals),  g_ij = K_ij z_j / sigma (12 reals),
 *   m_ij = relu(W1^T [u_i; u_j; g_ij]) (60 -> 64),  a_i = sum_j m_ij,
 *   h_i = relu(W2^T [u_i; a_i]) (88 -> 64),  p_ij = relu(W3^T [h_i; h_j]) (128 -> 64),
 *   c_i = sum_j p_ij,  q_i = relu(W4^T [h_i; c_i]) (128 -> 64),  d_i = W5^T q_i (64 -> 12),
 *   dx_i = sigma d_i;   complex values as (re, im) pairs; no biases, so dx(a r) = a dx(r).
 * Weights: FNLH_NN_PARAMS FP32 values W1..W5, each row-major [in][out]; the kernels use
 * BF16 copies with FP32 accumulation on the matrix cores.  Training loss of a pair
 * (r, e), e the error x* - x that left residual r: ||d - e/sigma||^2 / ||e/sigma||^2,
 * averaged over a batch; Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 master.
 * The network belongs to one context (its mesh, matrix and harmonics) and is freed with
 * it at the latest. */
typedef struct fnlh_nn_s* fnlh_nn;
enum { FNLH_NN_PARAMS = 26624 };
/* Attach a network to c (one per context; FNLH_E_ORDER if c has one).  Weights unset.
 * hidden: width of the hidden layers; the matrix-core tiles of the kernels are built for
 * 64 (0 also means 64), any other value is FNLH_E_ARG. */
int fnlh_nn_create(fnlh_nn* out, fnlh_ctx c, int32_t hidden);
int fnlh_nn_destroy(fnlh_nn nn);
/* host [FNLH_NN_PARAMS] FP32 weights in / out; setting them resets Adam.  Errors:
 * FNLH_E_ARG for non-finite values. */
int fnlh_nn_set_weights(fnlh_nn nn, const float* w);
int fnlh_nn_get_weights(fnlh_nn nn, float* w);
/* dx = network(r) for system sys: r, dx device [N][6] complex128 user order. */
int fnlh_nn_apply(fnlh_nn nn, int32_t sys, const double* r, double* dx, void* stream);
/* Workgroups of the backward (gradient) kernels: each sums the weight-gradient partials
 * of the 64-row tiles g, g + groups, g + 2 groups, ... and the partials are added in a
 * fixed order, so the gradient is deterministic for a given count.  1..512, or 0 for
 * the automatic min(512, tiles).  Changes only the summation order of the gradient. */
int fnlh_nn_set_grad_groups(fnlh_nn nn, int32_t groups);
/* Mean loss and its gradient over n pairs (device [N][6] user-order r[k], e[k]);
 * grad host [FNLH_NN_PARAMS] or NULL, loss host or NULL.  Synchronises the stream. */
int fnlh_nn_loss_grad(fnlh_nn nn, int32_t n, const int32_t* sys, const double* const* r,
                      const double* const* e, float* grad, double* loss, void* stream);
/* Keep n training pairs (r[k], e[k]) of system sys[k] on the device as BF16 copies in
 * the internal cell order (48 bytes per cell and pair; the caller's buffers may be
 * reused once the stream has run the call's work).  The pool grows by doubling;
 * fnlh_nn_reserve_pairs sizes it once for a known count.  n_pairs: count held. */
int fnlh_nn_add_pairs(fnlh_nn nn, int32_t n, const int32_t* sys, const double* const* r,
                      const double* const* e, void* stream);
int fnlh_nn_reserve_pairs(fnlh_nn nn, int64_t n_pairs, void* stream);
/* Training pairs from the plain solver, generated in the library and appended to the
 * pool (n * starts * snapshots pairs).  With b = 0 the solution is 0, so an iterate is
 * minus its own error and its residual is -K_s x: for each start k (0 <= k < starts),
 * the n systems sys[j] (1 <= n <= 16) start from x0 with the 12 N user-order values
 * 2u - 1, u = (mix(key + v) >> 11) 2^-53 for value v, key = mix(seed +
 * 0x9E3779B97F4A7C15 (j starts + k + 1)), mix the splitmix64 finaliser (Steele, Lea and
 * Flood 2014); then `snapshots` times: `every` sweeps of fnlh_relax over the n systems
 * together (FNLH_DILU, b = 0, rtol 0, check_every 16, graph replay), and for each j
 * r = fnlh_residual(sys[j], x, 0) = -K_s x and e = -x stored as one pair.  The pairs
 * are the ones that sequence of fnlh_relax, fnlh_residual and fnlh_nn_add_pairs calls
 * would store.  Allocates and frees n + 2 vectors of 96 N bytes; synchronises the stream.
 * Needs the matrix and harmonics, not weights. */
int fnlh_nn_generate(fnlh_nn nn, int32_t n, const int32_t* sys, int32_t starts, int32_t snapshots,
                     int32_t every, uint64_t seed, void* stream);
/* Read stored pair k back: sys host out (may be NULL), r and e device [N][6] complex128
 * user order (may be NULL), the BF16 values widened to FP64. */
int fnlh_nn_get_pair(fnlh_nn nn, int64_t k, int32_t* sys, double* r, double* e, void* stream);
int fnlh_nn_clear_pairs(fnlh_nn nn);
int fnlh_nn_pairs(fnlh_nn nn, int64_t* n_pairs);
/* steps Adam steps on batches of `batch` pairs drawn with replacement (splitmix64 from
 * seed); loss host [steps] (may be NULL) receives each step's batch loss before its
 * update.  Synchronises the stream. */
int fnlh_nn_train(fnlh_nn nn, int32_t steps, int32_t batch, float lr, uint64_t seed, float* loss,
                  void* stream);
/* Checkpoint of the network: a binary file with the tag "FNLHNN01", the hidden width
 * and parameter count (int32 each), the Adam step count (int64), then the FP32 master
 * weights, Adam's first and second moments (FNLH_NN_PARAMS float32 each), little-endian.
 * fnlh_nn_load restores all of it (weights, moments, step count), so training resumes
 * exactly where the saved network stopped.  The pair pool is not part of it.  Errors:
 * FNLH_E_ORDER (save before weights are set), FNLH_E_ARG (file cannot be opened, a
 * write fails, or the file is not a checkpoint of this network: tag, sizes, length,
 * non-finite values). */
int fnlh_nn_save(fnlh_nn nn, const char* path);
int fnlh_nn_load(fnlh_nn nn, const char* path);
/* The same state (FP32 weights, Adam moments and step count) copied device to device
 * from src to dst, networks of two contexts on one device (e.g. training one network
 * on pairs from several meshes, a round on each in turn).  src needs weights. */
int fnlh_nn_copy_state(fnlh_nn dst, fnlh_nn src);
/* Matrix-core check: out = A B for 64x64 BF16 operands (host a [64][64], host bt = B^T
 * [64][64], raw BF16 bits), FP32 out [64][64], computed by the network's tile routine. */
int fnlh_nn_selftest(fnlh_ctx c, const uint16_t* a, const uint16_t* bt, float* out);

/* Library version string. */
const char* fnlh_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FNLH_H */
