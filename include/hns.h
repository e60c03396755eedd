/*
 * hns — preconditioned conjugate-gradient solves of the shallow-basin
 * projection step on AMD Instinct MI355X (gfx950).
 *
 * The paper (Besson & Straubhaar, "Wind driven 3D Navier-Stokes circulation
 * in the Atlantic") advances the anisotropic Navier-Stokes equations with a
 * velocity-correction projection method (Sec. 3).  Each time step solves
 *   - three velocity-prediction problems, one per component, whose matrix is
 *     mass / time step + anisotropic viscous stiffness (Sec. 4 eq.
 *     fofa_velo_pred, discretised in Sec. 5 eq. fofa_velo_pred_h), and
 *   - one pressure-increment problem with a pure-Neumann Laplacian whose
 *     solution is fixed up to a constant (eq. fofa_q_cor / fofa_q_cor_h),
 * all by preconditioned conjugate gradients (Remark 1 after Sec. 5).
 *
 * This library assembles those operators for linear (P1) tetrahedra and
 * solves them with Jacobi-preconditioned CG in hand-written HIP kernels.
 *
 * Conventions for every entry point:
 *   - Host pointers are read during the call only; the caller keeps them.
 *   - Device pointers (suffix _dev) are caller-owned device memory on the
 *     current HIP device; they must stay valid until the call returns.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *     Solver calls return only when the result is final (they synchronise on
 *     their own convergence reads).
 *   - A negative hns_status is an error; hns_last_error() then returns a
 *     thread-local message.  Outputs are unspecified after an error.
 *   - Nothing here is thread-safe for the *same* operator and the same
 *     stream; different streams may solve with one operator concurrently
 *     (each solve takes its own workspace).
 */
#ifndef HNS_H
#define HNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HNS_OK = 0,
    HNS_NOT_CONVERGED = 1,   /* max_iter reached; x holds the last iterate      */
    HNS_ERR_INVALID = -1,    /* bad argument, or non-finite right-hand side      */
    HNS_ERR_HIP = -2,        /* a HIP runtime call failed                        */
    HNS_ERR_OOM = -3,        /* device or host allocation failed                 */
    HNS_ERR_MESH = -4,       /* bad connectivity or a non-positive tetrahedron   */
    HNS_ERR_BREAKDOWN = -5   /* p^T A p <= 0 or a non-finite CG scalar           */
} hns_status;

typedef struct hns_operator hns_operator; /* opaque, device-resident */

/* Mesh of the shallow domain (Sec. 2): nodes, positively oriented linear
 * tetrahedra, per-node Dirichlet bits and (optionally) the surface triangles
 * on Gamma_s.  All arrays are host memory.
 *   xyz       n_nodes x 3, row-major, float64
 *   tets      n_tets x 4, int32, 0-based; det[v1-v0, v2-v0, v3-v0] > 0
 *   bc        n_nodes, uint8; bit c set = node is Dirichlet (value 0) for the
 *             solve that passes mask_bit = c (c = 0..7).  May be NULL (no
 *             Dirichlet nodes).
 *   surf_tris n_surf_tris x 3, int32 (may be NULL; needed only with
 *             HNS_STEP_AUX, for the wind-tension load on Gamma_s). */
typedef struct {
    int64_t n_nodes;
    const double *xyz;
    int64_t n_tets;
    const int32_t *tets;
    const uint8_t *bc;
    int64_t n_surf_tris;
    const int32_t *surf_tris;
} hns_mesh;

/* Operator kind (exactly one) */
#define HNS_POISSON   0x1u   /* A = K_nu  (pressure increment, eq. fofa_q_cor_h)      */
#define HNS_HELMHOLTZ 0x2u   /* A = M + dt*K_nu  (velocity prediction, eq.
                                fofa_velo_pred_h multiplied by dt; implicit Euler
                                first step, BDF2 uses dt' = 2 dt / 3)                */
/* Options */
#define HNS_KEEP_FP32 0x10u  /* also keep FP32 matrix/diagonal copies (HNS_MIXED)  */
#define HNS_KEEP_HOST 0x80u  /* keep a host copy of the assembled matrix (needed by
                                the IC(0) preconditioner, set_param "precond" = 2)   */
#define HNS_GPU_ASSEMBLY 0x40u /* build the operator on the device, bitwise the host
                                path's operator: without HNS_KEEP_HOST and
                                HNS_STEP_AUX, with the automatic or the diagonal
                                format, and when the element offsets fit the
                                unrolled diagonal storage (at most 16 upper
                                diagonals), everything (node incidence by counting
                                sort, offsets, values in diagonal storage, D^-1,
                                lumped mass); otherwise the values only (one lane
                                per row gathers its tetrahedra in order, as the host
                                loop does) on a pattern built on the host.  The
                                mesh is copied to the device for it; the transient
                                device memory is about twice the mesh arrays
                                (coordinates, tetrahedra, incidence lists)        */
#define HNS_MATRIX_FREE 0x800u /* bricks only (hns_assemble_hex): no stored matrix;
                                every product is computed element by element from
                                the mesh (sum factorisation over the tensor Gauss
                                points, trilinear geometry recomputed at each
                                point), element results summed into each node in
                                ascending element order (deterministic).  Only
                                the diagonal (Jacobi), the lumped mass and the
                                mesh are kept.  HNS_FP64 solves (point Jacobi or,
                                for order 1, the line preconditioner), per-slot
                                batch sessions and hns_apply; HNS_MIXED, block
                                multi-right-hand-side solves, IC(0) and the
                                allocation-free solve return HNS_ERR_INVALID.
                                hns_operator_format reports HNS_MATRIX_FREE       */
#define HNS_STEP_AUX  0x20u  /* also keep M, B_1..3, lumped mass, surface mass and
                                the mesh (coordinates, tetrahedra, node incidence)
                                for the step right-hand sides (hns_step_*)          */
/* Storage format of A on the device (default: chosen from the pattern) */
#define HNS_FMT_AUTO  0x000u
#define HNS_FMT_CSR   0x100u /* compressed sparse rows, 16 lanes per row            */
#define HNS_FMT_SELL  0x200u /* sliced ELLPACK, slice height 64 (one wavefront),
                                column-major inside a slice                          */
#define HNS_FMT_SDIA  0x400u /* symmetric diagonal storage: main + at most 64 upper
                                diagonals (zeros stored where a row lacks an
                                offset), no column indices, lower triangle read by
                                symmetry; needs a bitwise-symmetric matrix whose
                                pattern has few distinct offsets j - i (structured
                                meshes).  HNS_FMT_AUTO picks it for up to 16 offsets,
                                and for up to 64 when it stores fewer bytes than
                                CSR; else SELL when row lengths are even, else CSR  */

/* Solve modes */
#define HNS_FP64  0u         /* everything in FP64                                   */
#define HNS_MIXED 1u         /* FP32 matrix/vectors inside FP64 iterative refinement */

typedef struct {
    int32_t iterations;       /* CG iterations (all inner iterations in HNS_MIXED) */
    int32_t outer_iterations; /* refinement steps (HNS_MIXED), 1 otherwise         */
    double relres_true;       /* ||b - A x||_2 / ||b||_2 recomputed in FP64 at exit */
    double removed_mean;      /* mean of b removed in the pure-Neumann case        */
    int32_t status;           /* hns_status of this solve                           */
    int32_t reserved;
} hns_solve_info;

/* Assemble the operator of `flags` (one kind + options) on the device.
 * nu = diag(nu_h, nu_h, nu_v) is the anisotropic viscosity (Sec. 2); dt is
 * the time step (ignored for HNS_POISSON).  Assembly runs on the host (all
 * cores) and is uploaded once; the operator then stays resident.
 * Errors: HNS_ERR_INVALID (null/negative sizes, non-finite coefficients),
 * HNS_ERR_MESH (node index out of range, tetrahedron volume <= 0),
 * HNS_ERR_OOM, HNS_ERR_HIP. */
hns_status hns_assemble(const hns_mesh *mesh, double nu_h, double nu_v, double dt,
                        uint32_t flags, hns_operator **out);

/* Mesh of brick elements (the discretisation of Sec. 5: Q2 velocity, Q1
 * pressure).  All arrays are host memory.
 *   xyz       n_nodes x 3, row-major, float64
 *   order     1 (Q1: 8 nodes per element) or 2 (Q2: 27 nodes per element)
 *   hex       n_hex x (order+1)^3, int32, 0-based; local node (a, b, c), each
 *             in 0..order and standing for the reference point
 *             (-1 + 2a/order, -1 + 2b/order, -1 + 2c/order) of [-1,1]^3, at
 *             column a + (order+1) b + (order+1)^2 c.  The element is the
 *             trilinear image of the reference cube through its 8 corner
 *             nodes (a, b, c in {0, order}); the coordinates of the other Q2
 *             nodes are not used by the assembly.
 *   bc        n_nodes, uint8, Dirichlet bits as in hns_mesh (may be NULL). */
typedef struct {
    int64_t n_nodes;
    const double *xyz;
    int64_t n_hex;
    int32_t order;
    int32_t reserved;
    const int32_t *hex;
    const uint8_t *bc;
} hns_hex_mesh;

/* Assemble the operator of `flags` on a brick mesh (Sec. 5): A = K_nu
 * (HNS_POISSON) or M + dt*K_nu (HNS_HELMHOLTZ) for the Q1 or Q2 space of
 * `mesh->order`, integrated with the tensor Gauss rule of order+1 points per
 * direction.  The operator is used like one from hns_assemble (hns_solve,
 * batched sessions, IC(0), mixed precision); the line preconditioner
 * (set_param "precond" = 1) is offered for order 1 on a column-contiguous
 * numbering.  Accepted options: HNS_KEEP_FP32, HNS_KEEP_HOST and a storage
 * format, or HNS_MATRIX_FREE alone; HNS_GPU_ASSEMBLY and HNS_STEP_AUX are
 * HNS_ERR_INVALID here.
 * Errors: HNS_ERR_INVALID (null/negative sizes, order not 1 or 2, non-finite
 * coefficients, unsupported flags), HNS_ERR_MESH (node index out of range,
 * non-finite coordinate, Jacobian determinant <= 0 at a quadrature point),
 * HNS_ERR_OOM, HNS_ERR_HIP. */
hns_status hns_assemble_hex(const hns_hex_mesh *mesh, double nu_h, double nu_v, double dt,
                            uint32_t flags, hns_operator **out);

/* Solve A x = b by Jacobi-preconditioned conjugate gradients (Remark 1 after
 * Sec. 5; the diagonal preconditioner is the DIAG part of Remark 2).
 *   mask_bit  Dirichlet set: nodes with bit mask_bit of mesh.bc are fixed to 0
 *             (rows and columns eliminated symmetrically).  -1 = no Dirichlet
 *             node; with HNS_POISSON this is the pure-Neumann pressure problem:
 *             b is projected to zero sum (removed_mean reports the mean) and
 *             the answer is shifted to zero mass-weighted mean, standing in
 *             for the zero-mean constraint on q (Sec. 4, Remark 2).
 *   b_dev     n doubles (device).  Dirichlet entries are ignored.
 *   x_dev     n doubles (device): initial guess in, solution out (Dirichlet
 *             entries are returned as 0).
 *   tol       relative tolerance on the true residual: ||b - A x||_2 <= tol ||b||_2
 *   max_iter  cap on CG iterations (all inner iterations in HNS_MIXED)
 *   mode      HNS_FP64 or HNS_MIXED (needs HNS_KEEP_FP32)
 *   info      filled on every return (may be NULL)
 * b = 0 returns x = 0 after 0 iterations.  Non-finite b -> HNS_ERR_INVALID.
 * HNS_NOT_CONVERGED leaves the last iterate in x. */
hns_status hns_solve(hns_operator *op, int mask_bit, const double *b_dev, double *x_dev,
                     double tol, int max_iter, uint32_t mode, void *stream,
                     hns_solve_info *info);

/* Allocation-free variant of hns_solve, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, results and errors as hns_solve,
 * but the solve's workspace (CG vectors, partial sums, device scalars) lives
 * in a static device array of the library (hns_noalloc_scratch_bytes() =
 * 96 MiB; each GPU the library runs on holds its own copy until the process
 * ends), and the call allocates nothing: no hipMalloc, hipFree or pinned host
 * memory.  Every call on one GPU shares that array, which keeps the last
 * call's contents (each call initialises what it reads), so calls that
 * overlap on one GPU race: the caller serialises them.
 *   - point Jacobi only: an operator with set_param "precond" != 0 is
 *     HNS_ERR_INVALID;
 *   - where hns_solve would run the Jacobi-scaled recurrence, that recurrence
 *     runs if the operator already holds its scaled copy (built by a
 *     previous hns_solve), else the unscaled point-Jacobi recurrence (the
 *     same iterates in exact arithmetic, another rounding);
 *   - an operator whose workspace exceeds the scratch (hns_noalloc_bytes(op,
 *     mode) > hns_noalloc_scratch_bytes(): beyond about 3.1M rows in HNS_FP64
 *     and 2.5M in HNS_MIXED) is HNS_ERR_INVALID, with nothing run;
 *   - per-kernel timing (hns_profile_enable) is not recorded by these calls. */
hns_status hns_solve_noalloc(hns_operator *op, int mask_bit, const double *b_dev,
                             double *x_dev, double tol, int max_iter, uint32_t mode,
                             void *stream, hns_solve_info *info);

/* Scratch bytes hns_solve_noalloc needs for `op` in `mode`, and the size of
 * the static scratch (0 for a null operator). */
size_t hns_noalloc_bytes(const hns_operator *op, uint32_t mode);
size_t hns_noalloc_scratch_bytes(void);

/* Solve k independent systems A x_j = b_j sharing one read of A per iteration
 * (multi-right-hand-side CG; each column keeps its own CG scalars, reduced
 * deterministically, and stops on its own).  B_dev and X_dev are n x k
 * row-major (the k values of one node are contiguous), 1 <= k <= 1024.
 * mask_bits[j] is the Dirichlet bit of column j (-1 = none; with
 * HNS_POISSON a pure-Neumann column, projected and normalised as in
 * hns_solve).  X holds the initial guesses.  infos receives k entries
 * (outer_iterations = FP64 residual evaluations of the whole batch).
 * HNS_MIXED runs the FP32 recurrences with per-column FP64 residual
 * replacement as in hns_solve.  The host reads the columns' state after
 * chunks of at most "check_every" iterations: the first recurrence segment
 * runs whole chunks (HNS_MIXED: 8, 16, ... iterations), later ones the
 * longest segment so far plus 2
 * (so a residual replacement follows soon after the columns reach their
 * threshold), and a replacement waits up to 2 iterations for columns still
 * running; the chunking does not change any column's arithmetic.  With
 * "use_graph" = 1 each chunk length is captured once into a HIP graph (a few
 * kept per workspace) and replayed.
 * The return value is the worst column status (negative first). */
hns_status hns_solve_batched(hns_operator *op, int k, const int *mask_bits,
                             const double *B_dev, double *X_dev, double tol, int max_iter,
                             uint32_t mode, void *stream, hns_solve_info *infos);

/* ------------------------------------------------------------------------
 * Batch sessions (continuous batching).  A session owns `capacity` slots on
 * one operator.  Requests join free slots at any time (hns_batch_add),
 * advance together with the requests already running (hns_batch_advance),
 * and leave as soon as they finish (hns_batch_take), freeing the slot for
 * the next request.  Two forms, chosen at hns_batch_open by the operator's
 * "session_mode":
 *  - shared block: the slots are the columns of one multi-right-hand-side
 *    recurrence (all running slots share each operator read and each launch);
 *    per slot the arithmetic is that of hns_solve_batched (per-column
 *    scalars, tolerance and iteration cap; HNS_MIXED with FP64 residual
 *    replacement);
 *  - per slot: every slot runs hns_solve's own recurrence (HNS_MIXED as
 *    mixed_variant 0; the line preconditioner when "precond" is 1, point
 *    Jacobi otherwise, IC(0) included), its answer bitwise that of hns_solve
 *    with x0 = 0; an advance enqueues one chunk of every running slot and
 *    waits once.  With one or two slots sharing the operator read saves
 *    nothing next to the vector traffic, and a half-empty block still moves
 *    every column, so this is the default there.
 * Calls on one session must not overlap; sessions of different operators may
 * run on different streams concurrently.  Each call returns after its work on
 * `stream` has completed.
 * ------------------------------------------------------------------------ */
typedef struct hns_batch hns_batch;

/* Device bytes of a session (its workspace and right-hand-side block). */
size_t hns_batch_footprint(const hns_operator *op, int capacity, uint32_t mode);

/* Open a session of 1..1024 slots on `op` (mode HNS_FP64 or HNS_MIXED). */
hns_status hns_batch_open(hns_operator *op, int capacity, uint32_t mode, hns_batch **out);
void hns_batch_close(hns_batch *bt);

/* Put `count` requests into free slots: slot slots[q] solves A x = b_devs[q]
 * (device n-vector, copied) with Dirichlet bit mask_bits[q], relative
 * tolerance tols[q] and at most max_iters[q] iterations.  A right-hand side
 * with non-finite entries finishes at once with HNS_ERR_INVALID.
 * HNS_ERR_INVALID (nothing added) for a busy or repeated slot. */
hns_status hns_batch_add(hns_batch *bt, int count, const int *slots, const int *mask_bits,
                         const double *const *b_devs, const double *tols,
                         const int *max_iters, void *stream);

/* Run up to `iterations` CG iterations of every running slot (fewer when all
 * slots finish); *active_out (may be NULL) receives the slots still running. */
hns_status hns_batch_advance(hns_batch *bt, int iterations, void *stream, int *active_out);

/* states[slot] = 0 free, 1 running, 2 finished; infos (may be NULL) per slot. */
hns_status hns_batch_poll(hns_batch *bt, int *states, hns_solve_info *infos, void *stream);

/* Copy the result of a finished slot to x_dev (n doubles; pure-Neumann
 * results shifted to zero mass-weighted mean) and free the slot. */
hns_status hns_batch_take(hns_batch *bt, int slot, double *x_dev, hns_solve_info *info,
                          void *stream);

/* Autotuner of the multi-right-hand-side product of `hns_solve_batched` for
 * k columns in `mode` on this operator.  It times one launch of
 *   - the grid-stride product with 1, 2 and 4 consecutive columns per
 *     thread: times_us[0..2] (-1 where k is not a multiple of the width), and
 *   - on the narrow symmetric diagonal format, the LDS-tiled product in its
 *     three tile shapes (a block stages the rows its tile of consecutive rows
 *     reads, for a group of columns, then reads every term from LDS; FP64:
 *     16, 8, 16 columns by 64, 128, 32 rows, FP32: 32, 16, 16 columns by 64,
 *     128, 64 rows): times_us[3..5] (-1 where the shape does not apply),
 * so times_us holds 6 doubles.  *best_plan receives the plan later batched
 * solves of k columns in that mode use: V + 8 s, V the fastest width (also
 * the width of the vector updates) and s the tiled shape (1..3) when one is
 * faster than that width's product, else 0.  hns_solve_batched and the
 * shared-block sessions choose their plan the same way on first use of
 * (k, mode), unless "bspmm_vec" is set; plans are kept per process and in a
 * JSON file keyed by (GPU architecture, rows, nonzeros, k, precision,
 * format): $HNS_TUNE_CACHE, else $XDG_CACHE_HOME/hns/bspmm_plans.json
 * ($HOME/.cache when XDG_CACHE_HOME is unset); an unreadable or unwritable
 * file only means that the tuner runs again. */
hns_status hns_tune_batched(hns_operator *op, int k, uint32_t mode, void *stream,
                            double *times_us, int *best_plan);

/* Device bytes a solve of k right-hand sides in `mode` needs beyond the
 * resident operator (workspace: k = 1 for hns_solve, k > 1 for
 * hns_solve_batched), plus the operator's own bytes when include_operator
 * != 0.  Used for admission by HBM footprint. */
size_t hns_footprint_bytes(const hns_operator *op, int k, uint32_t mode, int include_operator);

/* Basic operator facts: rows, stored nonzeros of the full matrix, storage
 * format (HNS_FMT_CSR, _SELL or _SDIA), and for symmetric diagonal storage
 * the number of stored off-diagonals (upper ones; 0 for the other formats).
 * -1 (0 for the format) for a null operator. */
int64_t hns_operator_n(const hns_operator *op);
int64_t hns_operator_nnz(const hns_operator *op);
uint32_t hns_operator_format(const hns_operator *op);
int hns_operator_ndiag(const hns_operator *op);

/* Length of the water columns of the node numbering: nodes c L .. c L + L - 1
 * share their horizontal position (x, y) for every column c, as in the
 * vertical-first numbering of a terrain-following mesh; 0 when the numbering
 * is not made of such columns (the line preconditioner is then unavailable),
 * -1 for a null operator. */
int hns_operator_line_len(const hns_operator *op);

/* Where the operator was built: 0 on the host, 1 values on the device on a
 * host pattern, 2 entirely on the device (HNS_GPU_ASSEMBLY); -1 for a null
 * operator. */
int hns_operator_assembly(const hns_operator *op);

/* Tunables (returns HNS_ERR_INVALID for an unknown name or a bad value):
 *   "check_every"  CG iterations between host convergence reads (default 32;
 *                  see "small_n" for the single-workgroup path)
 *   "inner_tol"    relative tolerance of each FP32 inner solve (default 1e-5)
 *   "max_outer"    cap on refinement steps of the restarted variant (default 30)
 *   "mixed_variant" HNS_MIXED algorithm:
 *                  0 (default) one FP32 CG recurrence (FP32 matrix, vectors and
 *                    diagonal) whose residual is replaced by the FP64 true
 *                    residual, and whose iterate is added to the FP64
 *                    solution, each time it has dropped by "replace_drop";
 *                  1 classic refinement: a fresh FP32 CG to "inner_tol" per
 *                    FP64 correction x += |r| d;
 *                  2 FP32 matrix and diagonal with FP64 vectors, with the same
 *                    FP64 residual replacement as 0
 *   "replace_drop" residual drop between FP64 replacements, 0 < drop < 1
 *                  (default: 1e-3 where the FP32 recurrence of hns_solve runs
 *                  in one workgroup, up to "small_n" rows, since each
 *                  replacement costs two host round trips there; else 0.1)
 *   "use_graph"    1 = replay captured HIP graphs for the iteration chunks of
 *                  hns_solve_batched (default 0)
 *   "bspmm_vec"    columns per thread of the batched kernels: 0 = autotune
 *                  (default), or 1, 2, 4
 *   "bspmm_tile"   LDS-tiled batched product: -1 = the autotuner decides
 *                  (default), 0 = never, 1..3 = that tile shape (with
 *                  "bspmm_vec" set: always, where it applies; else the only
 *                  shape the autotuner tries); plans found with a value
 *                  other than -1 are not written to the plan file
 *   "spmv_it64"    launch shape of the single-vector diagonal-storage SpMV with
 *   "spmv_it32"    FP64 / FP32 vectors: workgroup-sized row passes per block
 *                  (integers 1..64; defaults 1, and 0 = by size for FP32: 1
 *                  below 500000 rows, 2 above)
 *   "spmv_rows64"  rows per lane of the FP64-vector diagonal-storage SpMV
 *                  (1 or 2; default 0 = by size: 1 below 250000 rows, where
 *                  the product is latency-bound and wants more workgroups,
 *                  else 2 with 16-byte loads)
 *   "vec_it"       16-byte packs per thread of the single-vector CG updates
 *                  (integers 1..64; default 0 = by size: 1 below 250000
 *                  rows, 2 below 1000000, 3 above).  The three change the
 *                  grid (and with it the summation order of the dot
 *                  products), not the arithmetic of a row or a pack; so
 *                  does "spmv_rows64".
 *   "small_n"      point-Jacobi FP64 / FP32 single right-hand-side solves of
 *                  operators with at most this many rows run each chunk of
 *                  iterations in one workgroup (one launch per chunk instead
 *                  of three per iteration; the same recurrence and stopping
 *                  rule, dot products summed over 1024 threads instead of
 *                  per-block partials; up to 4096 rows the vectors stay in
 *                  registers and LDS for the whole chunk).  The workgroup
 *                  stops by itself at the tolerance, so its chunks take up
 *                  to max(check_every, 1024) iterations (per-slot sessions:
 *                  the iterations of an advance).  Default 4096, 0 = never,
 *                  at most 1048576.  Not used while per-kernel timing is
 *                  enabled.
 *   "jacobi_scaling" 1 (default): point-Jacobi solves (precond 0) of an
 *                  operator in symmetric diagonal storage with at most 16
 *                  upper diagonals and more than "small_n" rows, HNS_FP64 or
 *                  HNS_MIXED with mixed_variant 0, run the Jacobi-PCG
 *                  recurrence of the paper's Sec. 5 remarks as plain CG on
 *                  D^-1/2 A D^-1/2 (D = diag(A)) with the vectors
 *                  D^1/2 x, D^-1/2 r, D^1/2 p: the same alpha, beta and
 *                  iterates in exact arithmetic, with a unit diagonal that is
 *                  not stored and no D^-1 reads per iteration.  Each segment
 *                  between FP64 true-residual checks starts from the true
 *                  residual, accumulates its correction in scaled form and
 *                  adds D^-1/2 times it to x; the stopping test still uses
 *                  |b - A x| (the recursive residual norm is weighted by
 *                  diag(A)).  The scaled operator (FP64, and FP32 when the
 *                  operator keeps FP32 values) is computed on the device on
 *                  first use and stays resident.  0 = the unscaled recurrence.
 *   "fuse_dir"     the Jacobi-scaled recurrence above in two launches per
 *                  iteration instead of three: the direction update of an
 *                  iteration rides in the product of the next, every
 *                  neighbour's r + beta p recomputed where the product reads
 *                  it, p alternating between two buffers (one more n-vector
 *                  of FP64 size per workspace).  The iterates, scalars and
 *                  iteration counts are bit for bit those of the three-launch
 *                  form.  -1 (default) while one vector of the recurrence
 *                  takes at most 4 MiB (524288 FP64 / 1048576 FP32 rows),
 *                  0 never, 1 always.  Per-kernel timing then times the
 *                  product (with the direction update) and the update.
 *   "session_mode" form of the batch sessions opened afterwards: 0 (default)
 *                  per-slot recurrences up to 2 slots, the shared block above;
 *                  1 always the shared block; 2 always per slot
 *   "precond"      0 = point Jacobi, the inverse diagonal (default; the
 *                  diagonal preconditioner of the paper's Sec. 5 remarks);
 *                  1 = vertical-line blocks: the inverse of the tridiagonal
 *                  block of each water column (the diagonal plus the
 *                  couplings between vertically adjacent nodes, Dirichlet
 *                  rows replaced by the identity), solved by the Thomas
 *                  recurrences with pivots factorised once per Dirichlet set
 *                  on first use (2 n doubles of device memory per set).  It
 *                  keeps CG's iteration count bounded on thin meshes whose
 *                  vertical couplings dwarf the horizontal ones, e.g. the
 *                  isotropic pressure operator of eq. fofa_q_cor_h.
 *                  Needs hns_operator_line_len >= 2; single right-hand
 *                  sides, HNS_FP64 or HNS_MIXED with mixed_variant 0 (FP32
 *                  factors, 2 n floats per set, in the FP32 iterations);
 *                  HNS_ERR_INVALID otherwise.
 *                  2 = incomplete Cholesky IC(0) (the velocity-system
 *                  preconditioner of the paper's Sec. 5 remarks) in a greedy
 *                  multicolour order: nodes coloured in node order with the
 *                  smallest colour no lower-numbered neighbour of the matrix
 *                  graph (Dirichlet rows and columns removed) has, then sorted
 *                  by (colour, node); L has the pattern of the lower triangle
 *                  of the reordered matrix and (L L^T)_ij matches it there.
 *                  Each triangular solve runs one launch per colour.
 *                  Factorised on the host per Dirichlet set on first use
 *                  (needs HNS_KEEP_HOST); HNS_FP64 single right-hand sides
 *                  with a Dirichlet set only; HNS_ERR_BREAKDOWN on a
 *                  non-positive pivot. */
hns_status hns_set_param(hns_operator *op, const char *name, double value);

/* y = A x on the device (FP64), with the rows of Dirichlet set mask_bit
 * zeroed and its columns ignored (mask_bit = -1: plain product). */
hns_status hns_apply(hns_operator *op, int mask_bit, const double *x_dev, double *y_dev,
                     void *stream);

/* ------------------------------------------------------------------------
 * Projection-step right-hand sides (Sec. 3 time discretisation, Sec. 4/5
 * weak forms), on a HNS_HELMHOLTZ operator assembled with HNS_STEP_AUX
 * (the mesh must carry its surface triangles).  The operator then also keeps
 *   M    mass matrix,  M_ij = int phi_i phi_j
 *   B_c  divergence coupling, (B_c)_ij = int phi_i d phi_j / d x_c, c = 1..3,
 *        and its transpose
 *   M_s  surface mass on Gamma_s, (M_s)_ij = int_{Gamma_s} phi_i phi_j ds
 *   m_L  lumped mass, (m_L)_i = sum_j M_ij
 * Velocity fields are 3 x n (component-major, one n-vector per component);
 * component c uses Dirichlet bit c-1 of mesh.bc.  All pointers are device.
 * The time step is the operator's dt (the implicit-Euler form of the
 * prediction step; a BDF2 step assembles with dt' = 2 dt / 3).
 * These calls use scratch memory of the operator: calls on one operator must
 * not overlap (different operators may run concurrently).  They return after
 * their work on `stream` has completed.
 * ------------------------------------------------------------------------ */

/* Velocity-prediction right-hand sides (eq. fofa_velo_pred_h multiplied by
 * dt, implicit-Euler form, advection left out):
 *   b_c = M u_c + dt (M_s theta_c + C_c + B_c^T p),
 * C_1 = M (f .* u_2), C_2 = -M (f .* u_1), C_3 = 0 (explicit Coriolis term
 * -2 omega x u with f = 2 omega_3), theta_3 = 0 (u_3 = 0 on Gamma_s).
 *   u_dev      3 x n, velocity at the previous step
 *   p_dev      n, pressure at the previous step (may be NULL: p = 0)
 *   theta_dev  2 x n, nodal wind tensions theta_1, theta_2 (may be NULL)
 *   f_dev      n, Coriolis parameter (may be NULL: no Coriolis term)
 *   b_dev      3 x n, output; entries on each component's Dirichlet set are 0 */
hns_status hns_step_velocity_rhs(hns_operator *helm, const double *u_dev, const double *p_dev,
                                 const double *theta_dev, const double *f_dev, double *b_dev,
                                 void *stream);

/* Pressure-increment right-hand side (eq. fofa_q_cor_h, implicit-Euler
 * form): b = -(1/dt) sum_c B_c u~_c for the predicted velocity ut_dev (3 x n). */
hns_status hns_step_pressure_rhs(hns_operator *helm, const double *ut_dev, double *b_dev,
                                 void *stream);

/* Pressure and velocity correction (eqs. fofa_pres_cor_h, fofa_velo_cor_h with
 * the lumped mass in place of M; u = u~ - dt grad q, the sign that follows
 * from the correction equations of Sec. 3):
 *   p += q;  u_c = u~_c - dt (B_c q) / m_L, set to 0 on the Dirichlet set of c.
 * ut_dev, u_dev: 3 x n (may alias); q_dev: n; p_dev: n, updated in place
 * (may be NULL). */
hns_status hns_step_correct(hns_operator *helm, const double *ut_dev, const double *q_dev,
                            double *p_dev, double *u_dev, void *stream);

/* ------------------------------------------------------------------------
 * Multi-step loop (Sec. 3 BDF2 scheme; Sec. 5 eqs. fofa_velo_pred_h,
 * fofa_q_cor_h, fofa_pres_cor_h, fofa_velo_cor_h).  Multiplying the BDF2
 * prediction by tau = 2 dt / 3 gives the operator M + tau K_nu (assemble a
 * HNS_HELMHOLTZ operator with dt = tau); the first step is implicit Euler
 * (tau = dt).  These calls use the auxiliary forms and the mesh kept by a
 * HNS_STEP_AUX operator `aux` (any dt); all vectors are device arrays, 3 x n
 * component-major for velocities; each call synchronises `stream`.
 * ------------------------------------------------------------------------ */

/* Explicit advection term: out_c[a] = int ((u . grad) u_c) phi_a dx for the P1
 * velocity u_dev (3 x n), c = 1..3.  u_dev and out_dev must not alias. */
hns_status hns_step_advection(hns_operator *aux, const double *u_dev, double *out_dev,
                              void *stream);

/* Prediction right-hand side of a BDF step:
 *   b_c = a1 M u_c + a2 M u'_c + tau (M_s theta_c + C_c(u) - adv_c + B_c^T p),
 * C_1 = M (f u_2), C_2 = -M (f u_1), C_3 = 0; zero on each component's
 * Dirichlet set.  BDF2: a1 = 4/3, a2 = -1/3 with u' = u^{k-1}; implicit Euler:
 * a1 = 1, a2 = 0 (uprev_dev may then be NULL).  p_dev, theta_dev (2 x n),
 * f_dev and adv_dev (3 x n, from hns_step_advection) may be NULL (term
 * absent). */
hns_status hns_step_velocity_rhs_bdf(hns_operator *aux, double tau, double a1,
                                     const double *u_dev, double a2, const double *uprev_dev,
                                     const double *p_dev, const double *theta_dev,
                                     const double *f_dev, const double *adv_dev, double *b_dev,
                                     void *stream);

/* Pressure-increment right-hand side b = -(1/tau) sum_c B_c u~_c. */
hns_status hns_step_pressure_rhs_tau(hns_operator *aux, double tau, const double *ut_dev,
                                     double *b_dev, void *stream);

/* Consistent-mass velocity correction (eq. fofa_velo_cor_h with the sign of
 * the correction equations): p += q when p_dev is not NULL, and
 *   rhs_c = M u~_c - tau B_c q, zero on the Dirichlet set of component c,
 * the right-hand side of M u_c = rhs_c, solved with hns_solve on a mass
 * operator (HNS_HELMHOLTZ assembled with nu_h = nu_v = dt = 0) and mask c. */
hns_status hns_step_correct_rhs(hns_operator *aux, double tau, const double *ut_dev,
                                const double *q_dev, double *p_dev, double *rhs_dev,
                                void *stream);

/* y = F x for one auxiliary form F of a HNS_STEP_AUX operator:
 * which = 0 M, 1..3 B_c, 4..6 B_c^T, 7 M_s (testing and diagnostics). */
hns_status hns_apply_aux(hns_operator *helm, int which, const double *x_dev, double *y_dev,
                         void *stream);

/* Kernel timing for measurement.  With period P > 0, every P-th CG
 * iteration of each chunk a solve runs on this operator (iterations P/2,
 * P/2 + P, ... of the chunk, counted from 0, so that with P > 1 a chunk's
 * first iteration is not sampled; a chunk shorter than P/2 + 1 iterations
 * samples none) records HIP events
 * around its three kernels on the solve's stream, and the durations of the
 * sampled iterations that did work (not the no-op launches after convergence
 * inside a chunk) are accumulated per kernel:
 *   kernel 0/1/2 = spmv / update / pupdate in FP64 vectors,
 *   kernel 3/4/5 = the same kernels in FP32 (inner iterations of HNS_MIXED).
 * hns_profile_read returns the summed milliseconds and the sampled launch
 * count; hns_profile_enable(op, P > 0) also clears the counters, P = 0 stops. */
hns_status hns_profile_enable(hns_operator *op, int period);
hns_status hns_profile_read(const hns_operator *op, int kernel, double *total_ms,
                            int64_t *launches);

void hns_operator_destroy(hns_operator *op);
const char *hns_status_string(hns_status s);
const char *hns_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HNS_H */
