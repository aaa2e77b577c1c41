/*
 * wcmg — Wilson-clover multigrid on AMD MI355X (gfx950).
 *
 * C ABI of the library.  It follows the structure of the multigrid solver of
 * D. Richtmann, P. A. Boyle, T. Wettig, "Multigrid for Wilson Clover Fermions
 * in Grid" (LATTICE2018, arXiv:1904.08678):
 *   - Sec. 2.1: intergrid operators (restriction / prolongation), creation and
 *     application of the coarse-grid operator through its site-diagonal part
 *     (Mdiag) and single-direction hops (Mdir), recursion to more levels,
 *     initial setup (smoother iterated on random vectors), iterative
 *     refinement setup, MR / GMRES / flexible GMRES, double-precision outer
 *     solver with a single-precision preconditioner;
 *   - Sec. 2.2: the chirality-preserving prolongator
 *     P = [ (1+gamma5)/2 psi_i , (1-gamma5)/2 psi_i ];
 *   - Sec. 3: restriction owned per coarse site through a coarse-to-fine lookup
 *     table (no races), fine data linearised aggregate by aggregate.
 * The paper gives no formula for the Dirac operator; the conventions used are:
 * chiral Euclidean gamma basis (gamma5 = diag(1,1,-1,-1)), mass form
 *   D = (4+m0) + C - 1/2 sum_mu [(1-gamma_mu) U_mu(x) T_mu + (1+gamma_mu) U_mu(x-mu)^dag T_-mu],
 * Sheikholeslami-Wohlert clover C = c_sw (i/4) sum sigma_{mu nu} F_{mu nu}
 * with clover-leaf F = (Q - Q^dag)/8, antiperiodic t boundary as a sign on
 * t-hops crossing the boundary.
 *
 * Memory and execution
 *   - Every data pointer is a caller-owned DEVICE pointer unless named *_host.
 *     The library never frees caller memory; it copies what it keeps.
 *   - The context owns every internal buffer.  All work is enqueued on the HIP
 *     stream given at creation.  Calls that need a value on the host
 *     (setup, refine, solve, get_*) synchronise that stream before returning.
 *   - One context per host thread.
 *
 * Layouts at the ABI (interleaved complex, lexicographic sites with x fastest,
 * i = x + Lx*(y + Ly*(z + Lz*t))):
 *   gauge U          complex128 [V][4][3][3]   (direction mu = x,y,z,t; row, col)
 *   clover blocks    complex128 [V][2][6][6]   (chirality +, -; index 3*spin'+colour)
 *   fine field       [nrhs][V][4][3]            (spin, colour; spins 0,1 have gamma5 = +1)
 *   coarse field     [nrhs][Vc][Nb]             (b < Nb/2: sigma3 = +1, then sigma3 = -1)
 *   coarse operator  complex128 [Vc][9][Nb][Nb] (0 = site, then +x,-x,+y,-y,+z,-z,+t,-t;
 *                                                block d maps the field at the
 *                                                neighbour in direction d to site x)
 *   near-null vectors complex128 [nv][V_l][ns_l] (ns_0 = 12, ns_l = Nb_l)
 * The complex type of a field follows the precision argument: WCMG_F64 ->
 * complex128; WCMG_F32 and WCMG_BF16 -> complex64 (BF16 refers to the storage
 * of coarse-operator blocks only; vectors and accumulation stay FP32).
 *
 * Errors: every call returns a wcmg_status; nothing throws or aborts.
 * wcmg_last_error() gives a message for the last failing call on a context
 * (when no call has failed: the report of the last coarsest-GMRES solve that
 * was redone after a grid-barrier timeout, see wcmg_timers, or "").
 */
#ifndef WCMG_H
#define WCMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WCMG_OK = 0,
  WCMG_ERR_ARG = 1,        /* null pointer, bad enum, bad size */
  WCMG_ERR_DIMS = 2,       /* lattice not divisible by a block, coarse extent < 2 */
  WCMG_ERR_STATE = 3,      /* call out of order (e.g. solve before setup) */
  WCMG_ERR_HIP = 4,        /* a HIP runtime call failed */
  WCMG_ERR_NOMEM = 5,      /* device allocation failed */
  WCMG_ERR_BREAKDOWN = 6,  /* Gram-Schmidt breakdown: dependent near-null vectors */
  WCMG_ERR_NOCONV = 7,     /* solver reached its iteration limit; info and x are filled */
  WCMG_ERR_NAN = 8         /* NaN or Inf detected in a norm */
} wcmg_status;

typedef enum { WCMG_F64 = 0, WCMG_F32 = 1, WCMG_BF16 = 2 } wcmg_prec;

typedef struct {
  int32_t dims[4];         /* fine lattice extents x, y, z, t */
  double m0;               /* bare mass in D = (4 + m0) + ... */
  double c_sw;             /* clover coefficient */
  int32_t antiperiodic_t;  /* 1: antiperiodic fermion boundary in t */
  int32_t n_levels;        /* 1 (no multigrid) .. 3 */
  int32_t block[3][4];     /* aggregate extents from level l to l+1 */
  int32_t n_vec[3];        /* near-null vectors at level l; Nb_{l+1} = 2 n_vec[l] */
  int32_t relax_sweeps;    /* MR sweeps on D x = 0 in the initial setup */
  int32_t refine_iters;    /* iterative-setup iterations run by wcmg_setup */
  int32_t post_smooth;     /* MR post-smoothing steps in the cycle */
  int32_t coarse_restart, coarse_maxit, coarse_fixed_iters; /* coarsest GMRES; fixed > 0 disables early exit */
  double coarse_tol;       /* relative residual target of the coarsest GMRES */
  int32_t kcycle;          /* 1: K-cycle (FGMRES on intermediate levels), 0: V-cycle */
  int32_t kcycle_maxit;
  double kcycle_tol;
  int32_t outer_restart, outer_maxit;
  double outer_tol;        /* true relative residual ||b - D x|| / ||b|| */
  int32_t cycle_prec;      /* WCMG_F64 or WCMG_F32: arithmetic of the preconditioner */
  int32_t coarse_store_prec; /* storage of coarse blocks inside the cycle: F64, F32 or BF16 */
  int32_t setup_prec;      /* arithmetic of the relaxation in the setup: F64 or F32 */
  int32_t coarse_points;   /* blocks stored per coarse site: 9 (or 0) = Mdiag and all eight hops; 5 = Mdiag and
                              the forward hops, the backward hops applied as sigma3-conjugated adjoints of the
                              neighbours' forward blocks (Sec. 4: five independent stencil points; needs
                              Nb in {8, 12, 16, 24, 32}, else nine are stored) */
  int32_t smoother;        /* level-0 post-smoother: 0 = MR (post_smooth steps); 1 = SAP (post_smooth cycles of the
                              Schwarz alternating procedure, Sec. 2.1 and Sec. 4, on the level-0 aggregates as
                              domains; needs an even number of aggregates in every direction and at most 256
                              sites per aggregate).  Coarser levels always use MR. */
  int32_t sap_block_iters; /* MR steps per SAP domain solve (default 4) */
  int32_t even_odd;        /* 1: wcmg_solve runs the outer FGMRES on the even-odd Schur complement
                              Dhat = A_oo - H_oe A_ee^{-1} H_eo (Sec. 2.1 and Sec. 4 name red-black
                              preconditioning; see wcmg_apply_schur) with the MG cycle embedded as its
                              preconditioner, then reconstructs the even sites */
  int32_t reserved[1];     /* reserved[0]: flags selecting reference forms, for comparisons (default 0):
                              1 no host progress checks inside cycles; 2 the generic coarsest GMRES;
                              4 the coarsest GMRES as four kernels per Arnoldi step instead of one
                              persistent launch; 8 the outer Arnoldi step as classical Gram-Schmidt applied
                              twice instead of the single-reduction step; 16 the persistent launch's barrier
                              waits give up at once and every launch is checked before the next step (every
                              such solve then takes the four-kernel fallback: a test of that path); 32 the
                              fine Dslash reads neighbours from a table instead of site arithmetic; 64 full
                              3x3 links instead of two rows; 128 the first persistent launch's waits give up
                              at once and its failure is found at the next progress check (the launches in
                              between return x = 0: a test of the deferred check); 256 the persistent coarsest
                              GMRES launched through the cooperative-launch API (guaranteed co-residency, about
                              3 us more per launch on the benchmark) */
} wcmg_params;

typedef struct wcmg_ctx wcmg_ctx;

/* Fill *p with the defaults (two levels, 4^4 aggregates, 12 vectors, 20 sweeps,
 * MR(4), GMRES(20) to 0.05 / 100 on the coarsest level, FGMRES(20) to 1e-10,
 * FP64 everywhere). */
void wcmg_default_params(wcmg_params* p);

/* Create a context for the lattice in *p; stream is a hipStream_t (may be NULL
 * for the default stream).  Validates dimensions: WCMG_ERR_DIMS when a block
 * does not divide its level or a coarse extent falls below 2. */
int wcmg_create(const wcmg_params* p, void* stream, wcmg_ctx** out);
int wcmg_destroy(wcmg_ctx* ctx);
const char* wcmg_last_error(const wcmg_ctx* ctx);

/* Gauge field U (complex128 [V][4][3][3], device).  Copied.  Also builds the
 * clover term from U with c_sw (Sec. 2.1 names the operator; the clover-leaf
 * construction is the standard one). */
int wcmg_set_gauge(wcmg_ctx* ctx, const void* U);
/* Replace the clover term by caller blocks (complex128 [V][2][6][6], device,
 * Hermitian, without the 4+m0 mass term). */
int wcmg_set_clover(wcmg_ctx* ctx, const void* blocks);
/* Read the clover term back (complex128 [V][2][6][6], device). */
int wcmg_get_clover(wcmg_ctx* ctx, void* blocks);

/* Start vectors of the initial setup at level l: complex128 [nv][V_l][ns_l]. */
int wcmg_set_null_vectors(wcmg_ctx* ctx, int level, const void* v, int nv);
/* Current near-null vectors (normalised, before orthonormalisation). */
int wcmg_get_null_vectors(wcmg_ctx* ctx, int level, void* v);
/* The orthonormalised chirality halves defining P_l (Sec. 2.2), [nv][V_l][ns_l]. */
int wcmg_get_prolongator(wcmg_ctx* ctx, int level, void* v);

/* Initial setup of every level (Sec. 2.1) from the start vectors, then
 * refine_iters iterations of the iterative setup. */
int wcmg_setup(wcmg_ctx* ctx);
/* Iterative refinement setup (Sec. 2.1, DDalphaAMG-style): each vector is
 * replaced by the current preconditioner applied to it, then P and the coarse
 * operators are rebuilt. */
int wcmg_refine(wcmg_ctx* ctx, int iterations);
/* Replace the near-null vectors of level l (complex128 [nv][V_l][ns_l]) and
 * rebuild P_l, D_{l+1} and the Galerkin products below (down to the first
 * level not built yet).  Finer levels must be built.  Once every level has
 * been built (by wcmg_setup, a checkpoint import or these calls) the context
 * accepts cycles and solves. */
int wcmg_rebuild_from_vectors(wcmg_ctx* ctx, int level, const void* v);

/* Setup checkpoint (Sec. 2.1: a setup serves many solves, and more setup
 * iterations buy faster solves): the hierarchy after wcmg_setup (or
 * wcmg_setup_learned, wcmg_refine) as one host blob, to be loaded by a later
 * context instead of running the setup again.  Layout (little-endian):
 *   bytes   0..7    "WCMGSET1"
 *           8..15   uint32 version (1), uint32 n_levels
 *          16..31   int32 dims[4]
 *          32..79   int32 block[3][4]
 *          80..91   int32 n_vec[3]
 *          92..95   int32 antiperiodic_t
 *          96..111  double m0, double c_sw
 *         112..127  uint64 payload bytes, uint64 checksum of the payload
 *                   (64-bit FNV-1a over its 8-byte words)
 *         128..     per level l = 0 .. n_levels-2 the near-null vectors
 *                   complex128 [n_vec[l]][V_l][ns_l] (the layout of
 *                   wcmg_get_null_vectors)
 * Export: buf == NULL only reports the size in *bytes; otherwise buf (host,
 * capacity bytes, owned by the caller) receives the blob (WCMG_ERR_ARG if it
 * is too small; WCMG_ERR_STATE before the setup).  Import (host blob, read
 * only): the gauge field must be set; the header must match the context
 * (dims, levels, aggregates, n_vec, m0, c_sw, boundary) and the checksum the
 * payload, else WCMG_ERR_ARG and the context is unchanged; then P_l and
 * D_{l+1} are rebuilt level by level from the vectors (no relaxation, no
 * refinement; the setup timer reports this rebuild).  With the gauge field of the exporting context
 * the hierarchy, and every solve on it, is bit-identical to the exported one;
 * the blob does not identify the gauge field, so pairing them is the caller's
 * task. */
int wcmg_setup_export(wcmg_ctx* ctx, void* buf, size_t capacity, size_t* bytes);
int wcmg_setup_import(wcmg_ctx* ctx, const void* buf, size_t bytes);

/* Aggregation map of level l -> l+1: per site of level l (lexicographic),
 * the coarse site and the offset inside its aggregate.  Host int32 arrays of V_l. */
int wcmg_get_aggregate_map(wcmg_ctx* ctx, int level, int32_t* coarse_host, int32_t* offset_host);

/* Coarse operator of level l >= 1 (the Galerkin operator, Sec. 2.1: Mdiag and
 * the eight Mdir blocks per site) as [Vc][9][Nb][Nb] (device, caller-owned).
 * get: prec WCMG_F64 -> complex128 (the FP64 master); WCMG_F32 -> complex64
 * rounded from it; WCMG_BF16 -> complex64 holding the BF16-rounded values the
 * cycle's BF16 block storage uses (Nb divisible by 4).  set: prec WCMG_F64
 * (complex128) or WCMG_F32 (complex64, widened); the master and every stored
 * copy used by the cycle are replaced.  WCMG_ERR_ARG for other precisions. */
int wcmg_get_coarse_op(wcmg_ctx* ctx, int level, void* blocks, int prec);
int wcmg_set_coarse_op(wcmg_ctx* ctx, int level, const void* blocks, int prec);

/* out = D_l in for nrhs fields (level 0: Wilson-clover, Sec. 2.1 "Dirac
 * operator"; level >= 1: Mdiag + the eight Mdir blocks, Sec. 2.1).  prec: the
 * arithmetic, and the complex type of in/out; WCMG_BF16 only for level >= 1. */
int wcmg_apply_D(wcmg_ctx* ctx, int level, const void* in, void* out, int nrhs, int prec);
/* coarse = R_l fine = P_l^dag fine (Sec. 3 blockProject), fine at level l. */
int wcmg_restrict(wcmg_ctx* ctx, int level, const void* fine, void* coarse, int nrhs, int prec);
/* fine = P_l coarse. */
int wcmg_prolong(wcmg_ctx* ctx, int level, const void* coarse, void* fine, int nrhs, int prec);
/* x = K r: one application of the multigrid preconditioner rooted at level 0
 * (complex128 fields; arithmetic per cycle_prec). */
int wcmg_cycle(wcmg_ctx* ctx, const void* r, void* x);

typedef struct {
  int32_t outer_iters;
  int32_t converged;
  double true_rel_res;     /* ||b - D x|| / ||b||, recomputed in FP64 at exit */
  double t_solve_s;        /* wall time of the call */
  int64_t coarse_iters;    /* total coarsest-level GMRES iterations */
  int64_t cycles;          /* preconditioner applications */
} wcmg_solve_info;

/* Solve D x = b with FP64 flexible GMRES preconditioned by the MG cycle
 * (Sec. 2.1).  b, x: complex128 [nrhs][V][4][3]; x holds the initial guess.
 * info: host array of nrhs entries (may be NULL). */
int wcmg_solve(wcmg_ctx* ctx, const void* b, void* x, int nrhs, wcmg_solve_info* info);

/* Batched form of wcmg_solve: the right-hand sides are taken in groups of up
 * to 16, and each group is solved together, one FP64 FGMRES per right-hand
 * side advancing through shared launches (every Dslash, restrict, prolong and
 * coarse apply covers the group; with FP32/BF16 coarse storage and Nb in
 * {8,16,24,32,40} the coarse apply of a group of >= 4 runs on the matrix
 * cores).  A converged right-hand side is masked out of the group's launches.
 * Each solve is the method of wcmg_solve; results differ from it only by
 * rounding order.  b, x as in wcmg_solve (x holds the initial guesses).
 * flags: bit 0 (WCMG_BATCH_GRAPH) captures the preconditioner application in a
 *          HIP graph on its second use and replays it (the cycle then runs
 *          without host checks: inner solves run their iteration limits,
 *          predicated off once converged, and the coarsest GMRES is limited
 *          to one restart cycle, min(coarse_maxit, coarse_restart)
 *          iterations; the cycle must be FP32);
 *        bits 1-2: coarse apply kernel, 0 auto, 1 per-row vector kernel,
 *          2 matrix cores (WCMG_BATCH_VECTOR, WCMG_BATCH_MFMA);
 *        bit 3 (WCMG_BATCH_DSLASH_PER_RHS): FP32 Dslash launched per
 *          right-hand side instead of the shared-link multi-RHS kernel.
 * info: host array of nrhs entries (may be NULL); t_solve_s, coarse_iters and
 * cycles are those of the whole group.  Errors: WCMG_ERR_ARG for bad flags or
 * fields; WCMG_ERR_NOCONV / WCMG_ERR_NAN as wcmg_solve (x is written). */
#define WCMG_BATCH_GRAPH 1
#define WCMG_BATCH_VECTOR 2
#define WCMG_BATCH_MFMA 4
#define WCMG_BATCH_DSLASH_PER_RHS 8
int wcmg_solve_batched(wcmg_ctx* ctx, const void* b, void* x, int nrhs, int flags, wcmg_solve_info* info);

/* Ragged batched solve: nprob problems, each on its own context (its own
 * lattice, gauge field, hierarchy and tolerances), problem k solving
 * nrhs[k] right-hand sides b[k] -> x[k] (complex128 [nrhs[k]][V_k][4][3],
 * device, x[k] holding the initial guesses), solved together.  Each problem
 * runs the method of wcmg_solve_batched (one FP64 FGMRES per right-hand side
 * preconditioned by the two-level cycle, Sec. 2.1); the problems advance in
 * lock-step so that the coarse-grid GMRES of all of them is one batch whose
 * coarse-operator applies (Mdiag + Mdir, Sec. 2.1) are ONE matrix-core launch
 * over the sum of their coarse sites per Arnoldi step.  Results equal each
 * problem's own batched solve up to rounding order.  Requirements
 * (WCMG_ERR_ARG otherwise): 1..8 problems, 1..16 right-hand sides each,
 * every context set up (WCMG_ERR_STATE otherwise), two levels, FP32 cycle,
 * the same coarse block size Nb in {8,16,24,32,40} and the same coarse
 * storage (FP32 or BF16), the same outer_restart and coarse_restart, the
 * same stream, no even-odd outer solve, no context twice.  info: host array of
 * sum(nrhs) entries in problem order (may be NULL); t_solve_s is the whole
 * ragged solve's wall time, cycles the number of shared coarse-operator
 * launches.  WCMG_ERR_NOCONV / WCMG_ERR_NAN as wcmg_solve (x is written);
 * messages through wcmg_last_error(ctxs[0]). */
int wcmg_solve_ragged(wcmg_ctx* const* ctxs, int nprob, const void* const* b, void* const* x, const int* nrhs,
                      wcmg_solve_info* info);

/* ---------------------------------------------------------------------------
 * Learned near-null proposal (a setup accelerator; not part of the paper's
 * method).  A gauge-covariant network of three parallel-transport convolution
 * layers, n_vec -> channels -> channels -> n_vec channels, maps the n_vec start
 * vectors of a context (the Gaussian draws the plain setup relaxes) to n_vec
 * proposed near-null vectors of level 0.  Layer l:
 *   z_o(x) = sum_i sum_h W_l[h][o][i] (T_h a_i)(x),
 *   T_0 a = a(x), T_{2mu+1} a = U_mu(x) a(x+mu), T_{2mu+2} a = U_mu(x-mu)^dag a(x-mu)
 * (fermion boundary sign on t hops), then a = z / sqrt(1 + |z(x)|^2) per
 * channel and site except after the last layer.  Weights are FP32 complex,
 * activations BF16 (or FP32), accumulation FP32 on the matrix cores.
 * Loss against the context's current near-null vectors v_j (the targets):
 * per aggregate and chirality, c_j = argmin |v_j - Y c|, and
 *   L = sum |v_j - Y c_j|^2 / sum |v_j|^2.
 * Weights, host layout: layer 0, 1, 2, each [9][c_out][c_in] complex as
 * (re, im) float pairs; wcmg_nn_num_weights gives the float count.
 * Errors: WCMG_ERR_ARG for bad sizes (n_vec in {4, 8, 12, 16} and equal to the
 * context's, channels a multiple of 4 up to 32), WCMG_ERR_STATE when the
 * context lacks a gauge field, start vectors or (for the loss) near-null
 * vectors. */
typedef struct wcmg_nn wcmg_nn;
/* act_prec: WCMG_BF16 or WCMG_F32 activations; seed: initial weights (self
 * hop near the identity, other hops small Gaussian). */
int wcmg_nn_create(int n_vec, int channels, int act_prec, uint64_t seed, void* stream, wcmg_nn** out);
int wcmg_nn_destroy(wcmg_nn* nn);
const char* wcmg_nn_last_error(const wcmg_nn* nn);
int wcmg_nn_num_weights(const wcmg_nn* nn, int64_t* n_floats);
int wcmg_nn_get_weights(wcmg_nn* nn, float* host, int64_t n_floats);
int wcmg_nn_set_weights(wcmg_nn* nn, const float* host, int64_t n_floats);
/* out_dev: complex128 [n_vec][V][4][3] (lexicographic), the network applied to
 * the context's start vectors of level 0. */
int wcmg_nn_forward(wcmg_nn* nn, wcmg_ctx* ctx, void* out_dev);
/* Loss against the context's near-null vectors and its gradient with respect
 * to the real parameters (dL/dRe W, dL/dIm W in the weight layout) on the host;
 * grad_host may be NULL. */
int wcmg_nn_loss_grad(wcmg_nn* nn, wcmg_ctx* ctx, double* loss, float* grad_host, int64_t n_floats);
/* One Adam step (beta 0.9, 0.999) of learning rate lr on that loss; *loss is
 * the loss before the step. */
int wcmg_nn_train_step(wcmg_nn* nn, wcmg_ctx* ctx, float lr, double* loss);
/* Setup with the network's proposals as the level-0 near-null vectors: each
 * proposal is smoothed by relax_sweeps MR steps on D x = 0 (0: used as
 * proposed), P and D_c are built from them, deeper levels are relaxed as usual,
 * then refine_iters refinement iterations run.  Quality q = max_i |D y_i| /
 * |y_i| of the raw proposals; if q is not finite, exceeds threshold, or
 * Gram-Schmidt breaks down, the plain setup (wcmg_setup) runs instead and
 * *fell_back = 1.  Needs start vectors of every level that the plain setup
 * would. */
int wcmg_setup_learned(wcmg_ctx* ctx, wcmg_nn* nn, double threshold, int relax_sweeps, int* fell_back,
                       double* quality);

/* Kernel autotuner of the batched path.  For each launch configuration met
 * (operator, lattice or coarse-lattice size, block size, precision, number of
 * right-hand sides) the library times every applicable kernel variant once on
 * the live operands, keeps the fastest and reuses it; the result of a call
 * never depends on whether it tuned.  Configurations decided so far form a
 * table, exported as JSON text {"<configuration>": {"choice": v, "ms": [...]}}
 * and accepted back (entries loaded are used as given, without timing).
 *   wcmg_tune_enable: 0 = no timing (untuned configurations use the built-in
 *     defaults), 1 = tune (default).
 *   wcmg_tune_table: writes the JSON (NUL-terminated) to buf if it fits in len
 *     bytes; *needed receives the length including the NUL.  WCMG_ERR_ARG if
 *     it does not fit.
 *   wcmg_tune_load: merges a table produced by wcmg_tune_table; WCMG_ERR_ARG
 *     on malformed text. */
int wcmg_tune_enable(wcmg_ctx* ctx, int enable);
int wcmg_tune_table(wcmg_ctx* ctx, char* buf, int len, int* needed);
int wcmg_tune_load(wcmg_ctx* ctx, const char* json);

/* Per-phase timers in seconds: [0] setup total, [1] relaxation, [2] Gram-Schmidt,
 * [3] coarsening, [4] refinement, [5] last solve; [6] is a count: coarsest
 * GMRES solves that the single-launch form handed back to the multi-kernel
 * form after a grid-barrier timeout (0 in a healthy run); [7] the link rows
 * the fine Dslash reads per link: 2 when every link of the gauge field is
 * SU(3) to 1e-12 (the third row is rebuilt as the conjugated cross product of
 * the first two), else 3.  n entries (<= 8) are written. */
int wcmg_timers(wcmg_ctx* ctx, double* out_host, int n);

/* Kernel timing: when enabled, launches of the named kernel family are
 * bracketed by HIP events on the context stream.  Families:
 * "dslash_f64", "dslash_f32" (full fine operator), "wilson_term" (single
 * terms, coarsening), "coarse_apply_f64", "coarse_apply_f32",
 * "coarse_apply_bf16", "coarse_term", "coarse_mfma_f32", "coarse_mfma_bf16"
 * (batched coarse apply on the matrix cores), "coarse_gmres_step_f64",
 * "coarse_gmres_step_f32", "coarse_gmres_step_bf16" (apply step of the fused
 * coarsest GMRES), "coarse_gmres_persistent" (a whole coarsest GMRES solve
 * as one persistent launch), "restrict_f64", "restrict_f32", "prolong_f64",
 * "prolong_f32", "sap_f64", "sap_f32" (one SAP colour), "nn_forward",
 * "nn_backward" (network, on its own context).  Stats return the number of
 * timed launches and their total duration in milliseconds, then reset. */
int wcmg_profile_enable(wcmg_ctx* ctx, const char* family, int enable);
int wcmg_profile_stats(wcmg_ctx* ctx, const char* family, int64_t* launches, double* total_ms);

/* Even-odd Schur complement of the fine operator (Sec. 2.1 and Sec. 4 name
 * red-black preconditioning without writing it down).  Reading: sites are
 * even or odd by the parity of x+y+z+t; with A = (4 + m0) + C and the hopping
 * terms H_eo, H_oe between the parities, out = Dhat in with
 * Dhat = A_oo - H_oe A_ee^{-1} H_eo acting on the odd sites: the even part of
 * `in` is ignored and that of `out` set to zero.  FP64 fields [nrhs][V][4][3]
 * (complex128, canonical layout, device pointers).  WCMG_ERR_BREAKDOWN when a
 * chirality block of A is singular.  Synchronises the stream. */
int wcmg_apply_schur(wcmg_ctx* ctx, const void* in, void* out, int nrhs);

/* SAP on the fine operator (Sec. 2.1 and Sec. 4 name SAP, the smoother
 * DDalphaAMG normally uses, without defining it).  Reading: the domains are the
 * level-0 aggregates, coloured by the parity of their coarse coordinates; one
 * cycle visits colour 0 then colour 1, and for every domain B of the colour
 * forms r_B = b_B - (D x)_B with the current x, runs sap_block_iters MR steps
 * on D_B e = r_B from e = 0 (D_B: D with every coupling that leaves B dropped)
 * and sets x_B += e.  b and x: nrhs device fields [nrhs][V][4][3], complex128
 * (prec WCMG_F64) or complex64 (WCMG_F32), canonical layout; x holds the
 * initial guess and receives the result.  Needs the gauge field, n_levels >= 2,
 * even aggregate counts in every direction and aggregates of at most 256
 * sites (WCMG_ERR_DIMS / WCMG_ERR_ARG otherwise).  Synchronises the stream. */
int wcmg_sap(wcmg_ctx* ctx, const void* b, void* x, int nrhs, int cycles, int prec);

/* ---- standalone coarse operator (CoarsenedMatrix without a hierarchy) ---- */
typedef struct wcmg_coarse wcmg_coarse;
/* dims: coarse lattice extents (each >= 2); nb: block size (even);
 * store_prec: WCMG_F64, WCMG_F32 or WCMG_BF16 storage of the blocks. */
int wcmg_coarse_create(const int32_t dims[4], int nb, int store_prec, void* stream, wcmg_coarse** out);
int wcmg_coarse_destroy(wcmg_coarse* op);
/* Load blocks [Vc][9][Nb][Nb] from device memory: complex128 when src_prec is
 * WCMG_F64, complex64 when WCMG_F32.  Converted to the storage precision
 * (BF16: round to nearest even). */
int wcmg_coarse_set(wcmg_coarse* op, const void* blocks, int src_prec);
/* out = D_c in for nrhs fields [nrhs][Vc][Nb]: complex128 for F64 storage,
 * complex64 otherwise (FP32 accumulation).  With FP32/BF16 storage and several
 * right-hand sides the product runs on the matrix cores (each site and
 * direction is a complex [Nb x Nb] x [Nb x nrhs] GEMM), up to 16 per launch. */
int wcmg_coarse_apply(wcmg_coarse* op, const void* in, void* out, int nrhs);
/* wcmg_coarse_apply for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same result, bit for bit, but no
 * device allocation and no hipFree on any call.  Where the kernel needs a
 * scratch buffer (the scatter buffer of the five-point owner-computes apply,
 * kernel 3 on large lattices: 4 * nrhs * Vc * Nb complex values of the
 * storage's vector type) it uses a library-owned 64 MiB device array, one
 * per GPU, held until the process ends (its address is looked up on the
 * first call on a device).  WCMG_ERR_ARG when the scratch would exceed
 * 64 MiB (use fewer right-hand sides per call); WCMG_ERR_STATE when the
 * blocks of the chosen kernel's layout are not set.  Every call on a GPU
 * shares that GPU's scratch, so calls that overlap in time on one GPU (other
 * streams, other host threads) race; calls on one stream are ordered and
 * safe.  Nothing in the scratch needs clearing: each call writes every entry
 * it reads. */
int wcmg_coarse_apply_noalloc(wcmg_coarse* op, const void* in, void* out, int nrhs);
/* Kernel choice for wcmg_coarse_apply: 0 automatic (matrix cores from 4
 * right-hand sides on), 1 per-row vector kernel, 2 matrix cores (FP32/BF16
 * storage, Nb in {8, 16, 24, 32, 40}), 3 per-row kernel on five-point
 * storage (Nb in {8, 12, 16, 24, 32}): only Mdiag and the forward blocks of
 * wcmg_coarse_set's input are kept and the backward hops are applied as
 * Mdir_{-mu}(c) = s Mdir_{+mu}(c - mu)^dag s (s = +1 on the first Nb/2
 * components, -1 on the rest), which is the operator itself when it is
 * sigma3-hermitian as every Galerkin coarse operator of gamma5-hermitian D is
 * (Sec. 2.2, Sec. 4).  Switching to or from 3 must precede wcmg_coarse_set
 * (WCMG_ERR_STATE otherwise).  WCMG_ERR_ARG when unsupported. */
int wcmg_coarse_set_kernel(wcmg_coarse* op, int kernel);
/* Tile of the matrix-core kernel (kernel 2, or 0 with >= 4 right-hand sides):
 *   -1 (default) tuned: on the first apply of each batch width the operator
 *      times every tile that fits and keeps the fastest (identical results);
 *    0 one wave per coarse site, neighbour vectors read straight from memory;
 *    4, 8, 16 that many consecutive sites of one x-row per workgroup, the
 *      neighbour vectors of each direction staged once in LDS for all of them
 *      and the outputs written through LDS as whole rows;
 *    5, 9 4 or 8 sites per workgroup with the staged neighbour vectors and
 *      each wave storing its own outputs.
 * The site count must divide the lattice's x extent (WCMG_ERR_ARG otherwise,
 * or at apply time when the stage for that many right-hand sides exceeds
 * 160 KB).  Every tile gives the same result, bit for bit. */
int wcmg_coarse_set_tile(wcmg_coarse* op, int tile);
/* The operator's tile choices as JSON text (format of wcmg_tune_table, keys
 * "<arch> coarse_mfma_tile prec=.. Vc=.. Lx=.. nb=.. nrhs=..", choice =
 * index into the tiles {0, 4, 8, 16, 5, 9}, ms = measured mean per tile, -1
 * where it does not fit).  Same buffer contract as wcmg_tune_table. */
int wcmg_coarse_tune_table(wcmg_coarse* op, char* buf, int len, int* needed);
/* Time `reps` back-to-back applies between HIP events on the op's stream;
 * *avg_ms receives the mean launch duration. */
int wcmg_coarse_time(wcmg_coarse* op, const void* in, void* out, int nrhs, int reps, double* avg_ms);
const char* wcmg_coarse_last_error(const wcmg_coarse* op);

/* Ragged batch (multi-lattice form of the batched coarse apply): nprob
 * standalone coarse operators of equal Nb and storage precision (FP32 or BF16;
 * Nb in {8,16,24,32,40}), each with its own lattice, blocks and neighbours,
 * operator p applied to its nrhs[p] fields in[p] -> out[p] (complex64
 * [nrhs[p]][Vc_p][Nb], device), in ONE matrix-core launch over the sum of
 * their coarse sites, on ops[0]'s stream.  nprob in 1..8, nrhs[p] in 1..16.
 * Errors (WCMG_ERR_ARG for mismatched operators or sizes) are reported through
 * wcmg_coarse_last_error(ops[0]).  wcmg_coarse_time_ragged: reps launches,
 * mean milliseconds per launch by HIP events. */
int wcmg_coarse_apply_ragged(wcmg_coarse* const* ops, int nprob, const void* const* in, void* const* out,
                             const int* nrhs);
int wcmg_coarse_time_ragged(wcmg_coarse* const* ops, int nprob, const void* const* in, void* const* out,
                            const int* nrhs, int reps, double* avg_ms);

#ifdef __cplusplus
}
#endif
#endif /* WCMG_H */
