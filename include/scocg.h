/*
 * scocg — generalized shifted COCG Green's-function solver for MI355X (gfx950).
 *
 * The library solves the generalized shifted linear equations
 *
 *         (z_k S - H) x_j(z_k) = e_j,      k = 0..K-1,  j in a set of RHS,
 *
 * (Sec. 3, Eq. 2 of Hoshi et al., "Novel linear algebraic theory and
 * one-hundred-million-atom quantum material simulations on the K computer")
 * for a real symmetric H and a real symmetric positive definite S (Sec. 2;
 * S = NULL means S = I, the standard shifted problem of Sec. 3), and returns
 * the Green's-function elements G_ij(z_k) = e_i^T x_j(z_k) for requested
 * rows i (the Green's function as the analysis object, Sec. 2-3), or the
 * whole x_j(z_k).  The method is the generalized shifted conjugate
 * orthogonal CG (Sec. 3, item (i)): one Krylov subspace per RHS, built for a
 * seed shift; every other shift follows by scalar recurrences; the seed is
 * switched when it converges first.  In the order-N form each RHS may be
 * restricted to a local cluster of atoms (principal submatrices of H and S),
 * following the paper's order-N principle (Sec. 2).
 *
 * Conventions for every call:
 *   - Plain C types and pointers only.  "host" pointers are ordinary CPU
 *     memory; "device" pointers are HIP device memory on the current device.
 *   - Nothing here aborts or throws.  Negative return codes are hard errors,
 *     SCOCG_OK (0) is success, positive codes are warnings.  The message of
 *     the last failure on the calling thread is scocg_last_error().
 *   - Objects are owned by the library and released by their _free call,
 *     which accepts NULL.
 *   - A plan is bound to one device and is not safe to run from two threads
 *     or streams at once.
 */
#ifndef SCOCG_H
#define SCOCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes --------------------------------------------------------- */
typedef int32_t scocg_status;
#define SCOCG_OK                 0
#define SCOCG_W_PARTIAL          1   /* some (RHS, shift) pair did not converge */
#define SCOCG_W_S_DIAG           2   /* S has a diagonal element != 1 (accepted) */
#define SCOCG_E_ARG            (-1)  /* NULL / negative / out-of-range argument */
#define SCOCG_E_SHAPE          (-2)  /* malformed sparse structure */
#define SCOCG_E_NOT_SYMMETRIC  (-3)  /* block (a,b) != block (b,a)^T exactly */
#define SCOCG_E_DEVICE         (-4)  /* HIP runtime error (message says which) */
#define SCOCG_E_NOMEM          (-5)  /* device or host allocation failed */
#define SCOCG_E_UNSUPPORTED    (-6)  /* block size / shift count not compiled in */

/* ---- per-(RHS, shift) result codes ---------------------------------------- */
#define SCOCG_CONVERGED  0   /* recursive residual estimate < tol * ||b|| */
#define SCOCG_MAXITER    1   /* iteration limit reached; partial x returned */
#define SCOCG_BREAKDOWN  2   /* zero pivot (mu = 0, pi = 0 or gamma = 0) */
#define SCOCG_NONFINITE  3   /* NaN / Inf met in the recurrences */
#define SCOCG_ABORTED    4   /* team solver: a wait between the workgroups of a team
                                exceeded its bound and the run was abandoned (the
                                plan's stats call then fails with E_DEVICE) */

/* ---- precision of the vectors and stored blocks --------------------------- */
#define SCOCG_FP64        0  /* complex128 vectors, FP64 blocks */
#define SCOCG_FP32        1  /* complex64 vectors and SpMV, FP32 blocks; FP64
                                scalars; optional FP64 residual replacement;
                                FP64 audit and single-shift FP64 fallback */
#define SCOCG_FP32_BF16   2  /* as SCOCG_FP32 but blocks stored as bfloat16 */

/* ---- output modes --------------------------------------------------------- */
#define SCOCG_METHOD_COCG 0
#define SCOCG_METHOD_QMR 1
#define SCOCG_METHOD_COCG_LANCZOS 2
#define SCOCG_OUT_SELECTED_G  0  /* G_ij for the rows i listed per RHS */
#define SCOCG_OUT_FULL_X      1  /* the whole x_j(z_k) (cluster-local order) */

typedef struct { double re, im; } scocg_z;

typedef struct scocg_matrix  scocg_matrix;
typedef struct scocg_problem scocg_problem;
typedef struct scocg_plan    scocg_plan;

/* Thread-local message describing the last failing call ("" if none). */
const char* scocg_last_error(void);

/* Library version string. */
const char* scocg_version(void);

/* ---- matrices ------------------------------------------------------------- */
/*
 * A square block-sparse-row matrix over nbrows block rows of bdim x bdim
 * blocks (the LCAO orbital blocks of one atom pair, Sec. 8).
 *   rowptr  host int64[nbrows+1], rowptr[0] = 0, non-decreasing
 *   colidx  host int32[rowptr[nbrows]], strictly ascending within a row,
 *           each in [0, nbrows)
 *   vals    host double[rowptr[nbrows] * bdim * bdim], row-major per block:
 *           vals[(e*bdim + r)*bdim + c] = A(a*bdim + r, colidx[e]*bdim + c)
 * The arrays are copied; the caller keeps ownership of its buffers.  The
 * matrix must be exactly symmetric: for every block (a,b) the block (b,a)
 * must be present and equal to its transpose (SCOCG_E_NOT_SYMMETRIC).
 * bdim must be 1..16 (the solver runs bdim 1, 4 and 9; others give
 * SCOCG_E_UNSUPPORTED at plan creation).
 */
scocg_status scocg_matrix_from_bsr(int64_t nbrows, int32_t bdim, const int64_t* rowptr,
                                   const int32_t* colidx, const double* vals,
                                   scocg_matrix** out);

/*
 * Same from scalar CSR (n x n, host arrays, columns ascending per row),
 * regrouped into bdim x bdim blocks; n must be a multiple of bdim.
 */
scocg_status scocg_matrix_from_csr(int64_t n, const int64_t* rowptr, const int32_t* colidx,
                                   const double* vals, int32_t bdim, scocg_matrix** out);

/*
 * Same from a Matrix Market file (`%%MatrixMarket matrix coordinate real
 * symmetric|general`, 1-based entries; the form in which published
 * tight-binding matrix sets are distributed, cf. the matrix library of
 * Sec. 6).  A symmetric file's stored triangle is mirrored; duplicate
 * entries are summed; then as scocg_matrix_from_csr with the given bdim
 * (1 reads matrices with mixed orbital counts per atom).  Errors: E_ARG
 * (NULL, file cannot be opened), E_SHAPE (not a real coordinate matrix,
 * not square, bad or missing lines, index out of range), and those of the
 * CSR path (E_NOT_SYMMETRIC for a general file that is not symmetric).
 */
scocg_status scocg_matrix_from_mtx(const char* path, int32_t bdim, scocg_matrix** out);

/* Shape of a matrix: block rows, block dimension, stored blocks. */
scocg_status scocg_matrix_shape(const scocg_matrix* m, int64_t* nbrows, int32_t* bdim, int64_t* nblocks);

/* Copy the stored BSR arrays out (caller-allocated host arrays of the
 * sizes scocg_matrix_shape gives: nbrows+1, nblocks, nblocks*bdim*bdim). */
scocg_status scocg_matrix_export_bsr(const scocg_matrix* m, int64_t* rowptr, int32_t* colidx, double* vals);

void scocg_matrix_free(scocg_matrix* m);

/* ---- problem: H and S resident on the device ------------------------------ */
/*
 * Merges the block patterns of H and S and uploads the values to device
 * memory owned by the problem (FP64, plus FP32/BF16 copies on first use by
 * a plan that asks for them).  S may be NULL (S = I).  H and S must have the
 * same nbrows and bdim.  S's diagonal is checked: a diagonal element != 1 is
 * accepted with SCOCG_W_S_DIAG (the method only needs S SPD; a non-SPD S is
 * detected by the inner CG and reported as BREAKDOWN).
 */
scocg_status scocg_problem_create(const scocg_matrix* H, const scocg_matrix* S,
                                  scocg_problem** out);
void scocg_problem_free(scocg_problem* p);

/* ---- options -------------------------------------------------------------- */
typedef struct {
    double  tol;            /* converge when ||rho|| / |pi_k| < tol * ||b|| (> 0) */
    int32_t maxiter;        /* outer iterations; 0 = max(1000, 4*M_j) */
    int32_t precision;      /* SCOCG_FP64 / SCOCG_FP32 / SCOCG_FP32_BF16 */
    int32_t replace_every;  /* FP32 forms: FP64 residual replacement of the seed every
                               this many iterations; 0 = off (default).  A replacement is
                               taken only while the gap between the true and the recursive
                               residual is at most 0.1 of the latter (a seed taken over by a
                               switch can carry a larger gap, and replacing it would break
                               the recurrences).  It reaches the seeds only: the other
                               shifts keep their FP32 gap, which the audit and fallback fix */
    int32_t inner_maxiter;  /* inner CG iteration cap */
    double  inner_tol;      /* inner CG stop: ||res|| <= inner_tol * ||rho|| (FP64) */
    double  inner_tol_lo;   /* same for the FP32 inner CG */
    int32_t seed_index;     /* initial seed; -1 = rule: smallest |Im z|, then Re z
                               nearest the median of Re z, then lowest index */
    int32_t threads;        /* workgroup size 256/512/1024; 0 = default */
    int32_t slots;          /* resident workgroups; 0 = device CUs x occupancy */
    int32_t audit;          /* 0: off.  1: FP64 true-residual audit of every (RHS, shift);
                               for the FP32 forms every pair the audit finds above tol
                               is re-solved from its x by single-shift FP64 COCG.
                               2: as 1, with the FP64 re-solve for FP64 too.
                               With the audit on, resid holds the audited residual,
                               and a re-solved pair is CONVERGED only if its audited
                               residual is <= tol (MAXITER otherwise). */
    int32_t projected;      /* FP64 with SELECTED_G output: keep x_k, p_k only on the
                               requested rows and run the seed in the three-term form
                               (per-shift work O(rows) instead of O(M_j); no audit,
                               resid is the recursive estimate).  Default 1. */
    int32_t method;         /* SCOCG_METHOD_COCG (default): generalized shifted COCG
                               with seed switching (Sec. 3, item (i)).
                               SCOCG_METHOD_QMR: generalized shifted QMR (Sec. 3,
                               item (ii)) over the real S-Lanczos basis that real H,
                               S and b = e_j share across all shifts; FP64 with
                               SELECTED_G output only (E_UNSUPPORTED otherwise);
                               resid is the quasi-residual bound of the true
                               residual, iters the step at which it fell below tol.
                               SCOCG_METHOD_COCG_LANCZOS: the shifted COCG iterates
                               (those of the default method, in exact arithmetic)
                               computed on that real basis by an LDL^T of each
                               shift's tridiagonal, with no seed; resid is the
                               residual norm |zeta_n| ||t|| the recurrences give.
                               Same restrictions as QMR. */
    int32_t team_size;      /* the two real Lanczos-basis methods: workgroups that solve
                               one panel of right-hand sides together, splitting its
                               rows (1..32); 0 = chosen by the library; -1 = one
                               workgroup per right-hand side (the one-workgroup
                               solver).  Other methods ignore it. */
    int32_t panel_width;    /* right-hand sides solved together by one team, sharing
                               every block read of H and S: 1, 4 or 8 (4 and 8 need
                               4x4 blocks and every RHS on the whole system; with 4x4
                               blocks the block products then run on FP64 matrix
                               cores); 0 = chosen by the library. */
    int32_t team_registers; /* team solver with S != I, 4x4 blocks and a panel of 4 or 8:
                               1 (default) keeps the inner CG's direction, solution
                               and S-product in registers and its residual on the
                               workgroup's rows in LDS when a compiled instance
                               covers the workgroup's share of rows; 0 keeps them
                               in memory (the direction in LDS). */
} scocg_options;

/* Defaults: tol 1e-10, maxiter 0, FP64, replace_every 0, inner_maxiter 1000,
 * inner_tol 1e-13, inner_tol_lo 1e-6, seed_index -1, threads 0, slots 0, audit 1,
 * projected 1, method COCG, team_size 0, panel_width 0, team_registers 1. */
void scocg_options_default(scocg_options* opt);

/* ---- right-hand sides ----------------------------------------------------- */
/*
 * RHS number r (0..nrhs-1) is the unit vector e_j with j = rhs_index[r] (a
 * global orbital index).
 *   cluster_ptr/cluster_atoms  host CSR over RHS of global atom indices,
 *           strictly ascending per RHS; NULL = every RHS uses the whole
 *           system.  The atom of orbital j must be in RHS r's cluster.  The
 *           cluster system is the principal submatrix of (z S - H) on the
 *           cluster's orbitals, in ascending global order.
 *   out_mode SCOCG_OUT_SELECTED_G: out_ptr/out_rows (host CSR over RHS of
 *           global orbital indices, each inside the RHS's cluster) name the
 *           rows i of G_ij to return.  SCOCG_OUT_FULL_X: out_ptr/out_rows are
 *           ignored and the whole cluster-local x is returned.
 *   order   optional host permutation of 0..nrhs-1: the order in which RHS
 *           are handed to the GPU's work queue (a scheduler's choice; it
 *           changes timing only).  NULL = index order.
 * All arrays are read during the call only.
 */
typedef struct {
    const int64_t* cluster_ptr;
    const int32_t* cluster_atoms;
    int32_t        out_mode;
    const int64_t* out_ptr;
    const int32_t* out_rows;
    const int32_t* order;
} scocg_rhs_spec;

/* ---- plans ---------------------------------------------------------------- */
/*
 * Validates the shifts and RHS, builds the per-RHS local block maps (order-N
 * clusters) on the host and uploads everything the solve reads, plus the
 * per-workgroup working memory, to the device.  After this call a run reads
 * only device memory.
 *   nshift  K >= 1 (at most 512), shifts host scocg_z[K]
 *   nrhs    >= 0, rhs_index host int32[nrhs]
 */
scocg_status scocg_plan_create(scocg_problem* P, const scocg_options* opt, int32_t nshift,
                               const scocg_z* shifts, int32_t nrhs, const int32_t* rhs_index,
                               const scocg_rhs_spec* spec, scocg_plan** out);
void scocg_plan_free(scocg_plan* plan);

/*
 * Number of complex output values of a run: sum over RHS of K * n_out(r),
 * where n_out(r) is the length of RHS r's out_rows list (SELECTED_G) or its
 * cluster dimension (FULL_X).  The values of RHS r start at
 * K * out_offset(r) and are laid out [shift][row].
 */
int64_t scocg_plan_out_count(const scocg_plan* plan);
/*
 * Launch shape of a plan, host int64[SCOCG_NINFO]: [0] resident workgroups,
 * [1] threads per workgroup, [2] padded rows per workgroup slot, [3] bytes of
 * one slot, [4] initial seed index, [5] LDS bytes per workgroup,
 * [6] precision, [7] bit 0: every RHS uses the whole system; bit 1: projected;
 * bit 2: a real Lanczos-basis method; bit 3: its COCG (Galerkin) iterates;
 * bit 4: the inner CG's direction vector is kept in LDS (a Lanczos-basis
 * method with S != I, when M_j doubles fit beside the per-shift arrays);
 * bit 5: with bit 4 on a global system whose S has exactly-identity
 * diagonal blocks, S is applied as I plus a plan-held copy of its nonzero
 * off-diagonal blocks; bit 6: the team solver runs (then [0] is the number of
 * workgroups of all teams and [3] the bytes of one team's working memory);
 * bit 7: its block products run on FP64 matrix cores; bit 8: the inner CG
 * keeps its vectors in registers and LDS (team solver, or the one-workgroup
 * solver on ELL blocks at 512 threads); bit 9: with bit 5 in the
 * one-workgroup solver, the off-diagonal blocks are held in ELL form (every
 * block row padded to the same length).  [8] workgroups per
 * team (1 for the other solvers), [9] panel width (right-hand sides per team).
 */
#define SCOCG_NINFO 10
scocg_status scocg_plan_info(const scocg_plan* plan, int64_t* info);

/* out_offset(r) for every RHS (host int64[nrhs+1], prefix sums of n_out). */
scocg_status scocg_plan_out_offsets(const scocg_plan* plan, int64_t* offsets);

/*
 * Runs the whole solve on `stream` (a hipStream_t; NULL = default stream),
 * asynchronously.  All outputs are caller-owned DEVICE buffers:
 *   out    scocg_z[scocg_plan_out_count]     G_ij(z_k) or x
 *   iters  int32[nrhs*K]  iteration at which (r,k) converged (-1 if not)
 *   status int8[nrhs*K]   SCOCG_CONVERGED / MAXITER / BREAKDOWN / NONFINITE
 *   resid  double[nrhs*K] final residual estimate ||rho||/|pi_k| / ||b||;
 *                         for the FP32 forms with audit on, the audited FP64
 *                         true residual ||b - (z_k S - H) x|| / ||b||
 * Any output pointer may be NULL except out.  Returns after enqueueing.
 */
scocg_status scocg_plan_run(scocg_plan* plan, void* stream, scocg_z* out, int32_t* iters,
                            int8_t* status, double* resid);

/*
 * Records the whole run (queue reset and the persistent solver) on `stream`
 * (a non-default hipStream_t) into a HIP graph bound to these output
 * buffers, and instantiates it; scocg_plan_replay launches it again.  The
 * graph holds no memset nodes.  Replays on one plan must not overlap.
 */
scocg_status scocg_plan_capture(scocg_plan* plan, void* stream, scocg_z* out, int32_t* iters,
                                int8_t* status, double* resid);
scocg_status scocg_plan_replay(scocg_plan* plan, void* stream);

/*
 * Autotuner of the one-workgroup solvers: times one probe solve (every RHS
 * capped at probe_iters outer iterations, after a warm-up) for each
 * workgroup size in {256, 512, 1024} and each count of resident workgroups
 * per compute unit in {1, 2} (team_size -1), and returns the fastest pair
 * (threads, total resident workgroups) and its probe time in seconds.  The
 * arguments are those of scocg_plan_create; the caller caches the answer
 * (the Python binding keys a JSON file by GPU architecture and problem
 * shape).  The team solver's shape is searched by scocg_autotune_team.
 */
scocg_status scocg_autotune(scocg_problem* P, const scocg_options* opt, int32_t nshift,
                            const scocg_z* shifts, int32_t nrhs, const int32_t* rhs_index,
                            const scocg_rhs_spec* spec, int32_t probe_iters, int32_t* best_threads,
                            int32_t* best_slots, double* best_seconds);

/*
 * Autotuner of the team solver (the two real Lanczos-basis methods): times
 * one probe solve (every RHS capped at probe_iters outer iterations, after a
 * warm-up) for each candidate launch - panel width, workgroups per team and
 * workgroup size, and the one-workgroup solver - and writes the fastest into
 * *best: a copy of *opt with threads, slots, team_size and panel_width set
 * (maxiter as in *opt).  Candidates that do not fit the device are skipped;
 * E_UNSUPPORTED if none fits, E_ARG for another method.
 */
scocg_status scocg_autotune_team(scocg_problem* P, const scocg_options* opt, int32_t nshift,
                                 const scocg_z* shifts, int32_t nrhs, const int32_t* rhs_index,
                                 const scocg_rhs_spec* spec, int32_t probe_iters, scocg_options* best,
                                 double* best_seconds);

/* ---- learned RHS-cost predictor (for the work-queue order) ----------------- */
/*
 * 16 local-environment features of every RHS orbital j of a plan, computed
 * on the device from its cluster map and the FP64 blocks; device float
 * [nrhs][16], asynchronous on `stream`:
 *   0 cluster atoms n_j          1 block entries / n_j      2 neighbours of c(j)
 *   3 entries in the neighbours' rows                       4-6 orbital s / p / d
 *   7 H_jj                        8 ||H_cc||_F               9-10 Gershgorin
 *   bounds of the on-site block   11-13 mean / max / std of ||H_cb||_F over
 *   neighbours b                  14 sum_{i != j} |H_ji|     15 mean ||S_cb||_F
 */
scocg_status scocg_features(scocg_plan* plan, float* feats, void* stream);

/* Number of MLP parameters (5313): W1[64][16], b1[64], W2[64][64], b2[64], W3[64], b3. */
int64_t scocg_mlp_nparams(void);
/* Floats of the device work buffer a training step needs. */
int64_t scocg_mlp_work_floats(void);

/*
 * y[s] = MLP(x[s]) for s < n: 16 -> 64 -> 64 -> 1 with ReLU, FP32; all
 * device pointers (w float[5313], x float[n][16], y float[n]).
 */
scocg_status scocg_mlp_forward(const float* w, const float* x, int64_t n, float* y, void* stream);

/*
 * One training step on the batch idx[0..m) of (x, t) (idx NULL: samples
 * 0..m-1): loss = mean (y - t)^2 over the batch (device float scalar, may be
 * NULL), gradient (device float[5313], may be NULL), and, if lr > 0, one Adam
 * step (beta 0.9 / 0.999, eps 1e-8, bias-corrected with step >= 1) on w with
 * moments adam_m, adam_v.  work: device float[scocg_mlp_work_floats()].
 * Deterministic: per-wave partial gradients summed in a fixed order in FP64.
 */
scocg_status scocg_mlp_train_step(float* w, float* adam_m, float* adam_v, const float* x, const float* t,
                                  const int32_t* idx, int64_t m, float lr, int32_t step, float* loss,
                                  float* grad, float* work, void* stream);

/*
 * A whole training run of the cost network on host buffers (the learned
 * binning of the RHS queue; the network and its Adam steps run on the
 * current device through the two calls above).  feats: host float[n][16]
 * (raw features, as scocg_features writes them); log_iters: host float[n]
 * (targets, log outer iterations).  Every feature is z-scored with its
 * mean and standard deviation over the n samples (sd 1 where constant); a
 * fraction val_frac of the samples, drawn from the seeded stream, is held
 * out, the rest visited in a freshly shuffled order each epoch in batches
 * of `batch`; the weights of the epoch with the lowest validation loss are
 * returned (the last epoch's when val_frac = 0).  model_out: host float
 * [scocg_mlp_model_floats()] = the 5313 weights, then the 16 feature means,
 * then the 16 standard deviations; val_loss (may be NULL): the best
 * validation MSE (NaN when val_frac = 0).  Synchronous; allocates and frees
 * its own device buffers.  Deterministic for a given seed.  Errors: E_ARG
 * (NULL pointer, n < 2, non-finite target, epochs or batch < 1, lr <= 0,
 * val_frac outside [0, 1)), E_NOMEM, E_DEVICE.
 */
typedef struct {
    int32_t epochs;             /* default 200 */
    int32_t batch;              /* default 256 */
    float lr;                   /* Adam step size, default 1e-3 */
    float val_frac;             /* held-out fraction, default 0.2 */
    uint64_t seed;              /* initial weights and sample order (splitmix64 stream) */
    const float* init_weights;  /* host float[5313], or NULL: Kaiming-uniform weights (bound
                                   sqrt(6 / fan_in)) and zero biases drawn from seed */
} scocg_mlp_cfg;
void scocg_mlp_cfg_default(scocg_mlp_cfg* cfg);
/* Floats of a trained model: 5313 weights + 16 means + 16 standard deviations. */
int64_t scocg_mlp_model_floats(void);
scocg_status scocg_mlp_train(const float* feats, const float* log_iters, int64_t n, const scocg_mlp_cfg* cfg,
                             float* model_out, double* val_loss);
/*
 * pred[s] = network(z-scored feats[s]) for s < n with a model from
 * scocg_mlp_train; host buffers (model float[scocg_mlp_model_floats()],
 * feats float[n][16], pred float[n]); synchronous.  Errors: E_ARG (NULL
 * pointer, n < 0, a standard deviation <= 0 in the model), E_NOMEM, E_DEVICE.
 */
scocg_status scocg_mlp_predict(const float* model, const float* feats, int64_t n, float* pred);

/*
 * Replace the work-queue order of a plan (the permutation the plan was
 * created with, or index order): order is a host permutation of
 * 0..nrhs-1, NULL = index order.  The order changes timing only, never
 * results: each RHS's solve does not depend on when it runs.  With panels
 * of several RHS (panel_width > 1) the RHS that share a panel are the
 * consecutive entries of the order.  Synchronous (waits for the device,
 * so no launch of the plan still reads the old order; a captured graph
 * keeps working and sees the new order).  Errors: E_ARG (NULL plan, not a
 * permutation), E_DEVICE.
 */
scocg_status scocg_plan_set_order(scocg_plan* plan, const int32_t* order);

/*
 * Learned binning (the queue order of the persistent launch): computes the
 * 16 features of every RHS (scocg_features), predicts its log outer
 * iterations with a scocg_mlp_train model, takes as its cost the predicted
 * iterations times the block entries of its local pattern (features 0 x 1),
 * and sets the plan's order to decreasing cost (stable: ties keep index
 * order), so long solves start first and panels (panel_width > 1) group
 * RHS of similar predicted cost, which wait less for each other.  model
 * NULL: cost = block entries (by-size order).  order_out (host int32
 * [nrhs]) and cost_out (host float[nrhs]) may be NULL.  Synchronous.
 * Errors: E_ARG (NULL plan, a bad model, a non-finite cost), E_NOMEM,
 * E_DEVICE.
 */
scocg_status scocg_schedule(scocg_plan* plan, const float* model, int32_t* order_out, float* cost_out);

/* Energy integration of G (the density of states and the density matrix,
 * Sec. 2-3: the Green's function as the analysis object).  G is the output
 * buffer a previous scocg_plan_run of this plan wrote ([rhs][shift][row],
 * SELECTED_G or FULL_X).  For every output row o of RHS j:
 *   rho[o] = -(1/pi) sum_k weights[k] f(Re z_k) Im G_{row(o), j}(z_k),
 * with f(E) = 1/(1 + exp((E - mu)/kT)) (kT = 0: a step, 1/2 at E = mu), and,
 * if ldos is not NULL, ldos[j*nshift + k] = -(1/pi) Im G_jj(z_k) (NaN when
 * orbital j is not among RHS j's output rows).  weights: the caller's
 * quadrature weights on the real parts of the shifts (e.g. trapezoid for an
 * equally spaced mesh).  G, weights, rho (one double per output row: the
 * last of scocg_plan_out_offsets, i.e. scocg_plan_out_count / nshift) and
 * ldos (nrhs*nshift doubles) are device pointers owned by the caller; the call is
 * asynchronous on `stream`.  Errors: E_ARG (NULL pointer, non-finite mu,
 * negative or non-finite kT), E_DEVICE. */
scocg_status scocg_plan_integrate(scocg_plan* plan, void* stream, const scocg_z* G, const double* weights,
                                  double mu, double kT, double* rho, double* ldos);

/*
 * Integrated crystal-orbital Hamilton population (COHP) of every output
 * pair, the bond analysis the paper builds on G (Sec. 2: a COHP extension
 * based on the Green's function):
 *   cohp[o] = H_{row(o), j} rho[o]
 * for output row o of RHS j, with rho as scocg_plan_integrate of this plan
 * wrote it (device double[rows], rows = sum_j nout_j); cohp has the same
 * layout.  H_{row(o), j} is gathered once per output row when the plan is
 * built (0 where the atoms of row(o) and j share no block).  Summed over the
 * orbitals of an atom b, cohp is the population of the bond between orbital
 * j and atom b; summed over every row of a FULL_X output it is (H rho)_jj,
 * orbital j's part of the band energy tr(rho H).  Asynchronous on `stream`.
 * Errors: E_ARG (NULL pointer), E_DEVICE.
 */
scocg_status scocg_plan_cohp(scocg_plan* plan, void* stream, const double* rho, double* cohp);

/*
 * Per-RHS counters of the last run, copied to host int64[nrhs * SCOCG_NSTAT]
 * (synchronises the run's stream):
 *   [0] outer iterations   [1] sum over iterations of shifts updated
 *   [2] inner CG iterations [3] seed switches  [4] cluster dimension M_r
 *   [5] block entries of the local pattern     [6] residual replacements
 *   [7] fallback (FP64 re-solve) outer iterations
 */
#define SCOCG_NSTAT 8
scocg_status scocg_plan_stats(scocg_plan* plan, int64_t* stats);

/*
 * Convenience: plan_create + plan_run + copy back + plan_free, all on host
 * buffers (out sized as scocg_plan_out_count would report; iters, status,
 * resid sized nrhs*K; any of those three may be NULL).  Synchronous.
 * Returns SCOCG_W_PARTIAL if any pair did not converge.
 */
scocg_status scocg_solve(scocg_problem* P, const scocg_options* opt, int32_t nshift,
                         const scocg_z* shifts, int32_t nrhs, const int32_t* rhs_index,
                         const scocg_rhs_spec* spec, scocg_z* out, int32_t* iters,
                         int8_t* status, double* resid);

/*
 * The same solve on caller-owned DEVICE output buffers, asynchronous on
 * `stream` (a hipStream_t; NULL = the default stream): validates the inputs
 * and builds the plan exactly as scocg_plan_create (shifts, rhs_index and the
 * spec arrays are HOST arrays, because the per-RHS cluster maps are built on
 * the host), then enqueues the run as scocg_plan_run does and returns.  out:
 * device scocg_z[K * sum_j nout_j] in the [rhs][shift][row] layout of
 * scocg_plan_run (nout_j = out_ptr[j+1] - out_ptr[j] for SELECTED_G; M, or
 * bdim times the cluster's atom count, for FULL_X); iters, status, resid:
 * device [nrhs][K] or NULL.  The problem keeps the plan until scocg_sync.
 * Errors: those of scocg_plan_create and scocg_plan_run, returned before
 * anything is enqueued.
 */
scocg_status scocg_solve_device(scocg_problem* P, const scocg_options* opt, int32_t nshift,
                                const scocg_z* shifts, int32_t nrhs, const int32_t* rhs_index,
                                const scocg_rhs_spec* spec, scocg_z* out, int32_t* iters, int8_t* status,
                                double* resid, void* stream);
/*
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): the solve of scocg_solve_device with no
 * device allocation or release at all.  (It waits on `stream` once, for the
 * copies of its host arrays, so it is not a call to record into a graph.)  Every
 * piece of per-call device memory (shifts, RHS records, requested rows, queue,
 * counters and the workgroups' working memory) is carved from one fixed array
 * of 64 MiB per device that the library holds from its load until the process
 * ends.  The caller still passes the outputs (device buffers, as
 * scocg_solve_device).  Runs the one-workgroup solver of the two real
 * Lanczos-basis methods (opt->method COCG_LANCZOS or QMR, FP64, SELECTED_G
 * output, every RHS on the whole system; E_UNSUPPORTED otherwise) with S as
 * stored; as many workgroups run at once as the array holds (at most one per
 * RHS, the device's compute units times occupancy, and opt->slots if set).
 * E_ARG when one workgroup's working memory (roughly 64 M + 48 K n_out bytes
 * for M rows, K shifts, n_out requested rows) does not fit the array.  The
 * host arrays are copied before the call returns; the solve itself is then
 * enqueued on `stream` asynchronously.  All calls on one device share its
 * array, which keeps the last call's contents: calls that overlap on one
 * device (two host threads, or two streams whose solves run at once) race and
 * must be serialised by the caller.  No pending state is kept: synchronise
 * `stream` and read the status buffer (no scocg_sync).
 */
scocg_status scocg_solve_device_noalloc(scocg_problem* P, const scocg_options* opt, int32_t nshift,
                                        const scocg_z* shifts, int32_t nrhs, const int32_t* rhs_index,
                                        const scocg_rhs_spec* spec, scocg_z* out, int32_t* iters,
                                        int8_t* status, double* resid, void* stream);

/*
 * Waits for every scocg_solve_device of P still pending (on its stream) and
 * frees their plans.  Returns OK, W_PARTIAL if some pair of those solves
 * did not converge (read from their status buffers; a solve given status =
 * NULL is not checked), or E_DEVICE.  scocg_problem_free calls it.  One
 * problem per host thread: solves and syncs of one problem must not overlap.
 */
scocg_status scocg_sync(scocg_problem* P);

#ifdef __cplusplus
}
#endif
#endif /* SCOCG_H */
