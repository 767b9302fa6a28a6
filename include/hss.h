/*
 * hss.h -- C ABI of the MI355X (gfx950) HSS library: the HSS matrix x block
 * product and the implicit ULV factorization / solve of an HSS matrix given
 * by its generators on a balanced binary cluster tree.
 *
 * Definitions (Massei, Robol, Kressner, "hm-toolbox: Matlab software for HODLR
 * and HSS matrices"):
 *   - cluster tree: Def. 2.1; default splitting rule: Sec. 3.1;
 *   - HSS generators D_i, U_i, V_i, translation operators R (row) and W
 *     (column), core blocks B12/B21 stored at the parent: Sec. 2.2 and the
 *     nestedness equation "HSS_nestedness";
 *   - A * X: the four-step HSS product of Sec. 4.1;
 *   - ulv(A), A \ B: the implicit ULV factorization of Sec. 4.3 (Steps 1-4);
 *   - ||A||_2 by the power method on A^T A: Sec. 4.5;
 *   - backward error ||b - A x|| / (||A|| ||x|| + ||b||): Sec. 5.1.
 *
 * Conventions.  Indices are 0-based.  Heap numbering: node t has children
 * 2t+1 and 2t+2; the nodes of level l are t = 2^l - 1 .. 2^(l+1) - 2.  All
 * matrices are column-major.  Sizes are int64_t unless marked int32_t.
 * Streams are hipStream_t passed as void* (NULL = the null stream).
 *
 * Status codes: 0 = HSS_OK; a negative value -i means that argument i
 * (1-based) is invalid; positive values are the HSS_E* codes below.
 *
 * Threading: a handle must be externally synchronized.  Device work of a
 * call is enqueued on its stream; the product (op N) forks part of its work
 * to a stream the handle owns and joins it back with events, so it is
 * ordered after earlier work on the caller's stream and before later work
 * there, as if it ran on that stream alone.  Only the calls that create a
 * handle (hss_create, hss_hadamard, hss_compress), hss_get_generators and
 * hss_destroy synchronize; products, factorizations and solves (refined or not) are
 * stream-ordered, and their device-side outcome (backward errors, refinement
 * steps, singular pivots) is written to device-accessible memory that is
 * valid once the stream has reached the end of the call.
 *
 * Work buffers and graph capture: a handle's work buffers grow when a call
 * needs more right-hand-side columns than any earlier call; the buffers they
 * replace stay allocated until hss_destroy, so a HIP graph that captured an
 * earlier call stays valid when later calls are wider.  A graph must be
 * replayed while its handle exists, and replays of graphs that use the same
 * handle must not overlap each other or other calls on that handle.
 */
#ifndef HSS_H_
#define HSS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hss_status;

#define HSS_OK         0
#define HSS_ENOMEM     1   /* device allocation failed                          */
#define HSS_EHIP       2   /* HIP runtime error                                 */
#define HSS_ESTATE     3   /* call out of order, e.g. solve before factor       */
#define HSS_ESINGULAR  4   /* exact zero pivot in an L block or the root LU     */
#define HSS_ENOCONV    5   /* refinement reached max_refine above tol           */
#define HSS_EUNSUP     6   /* sizes beyond what the kernels support             */
#define HSS_ESCRATCH   7   /* beyond the fixed scratch of hss_matmul_noalloc    */

#define HSS_OP_N 0          /* Y = A X   */
#define HSS_OP_T 1          /* Y = A^T X */

#define HSS_F64 0
#define HSS_F32 1

typedef struct hss_handle hss_handle;

/* Cluster tree (Def. 2.1).  leaf_off has 2^p + 1 entries, leaf_off[0] = 0,
 * leaf_off[2^p] = n, strictly increasing (empty leaves are rejected).
 * ku / kv have 2^(p+1) - 1 entries in heap order: the number of columns of the
 * row / column basis of node t (entry 0, the root, is ignored).
 * Host memory, read during the call only. */
typedef struct {
  int64_t n;
  int32_t p;
  int32_t reserved;
  const int64_t *leaf_off;
  const int32_t *ku;
  const int32_t *kv;
} hss_tree_desc;

/* FP64 generators in the canonical packed layout, HOST memory.  Each array is
 * the concatenation, in heap order, of column-major blocks (ld = rows):
 *   D, U, V   leaves only:           m_t x m_t, m_t x ku_t, m_t x kv_t
 *   R, W      internal, not root:    (ku_c1+ku_c2) x ku_t, (kv_c1+kv_c2) x kv_t
 *   B12, B21  every internal node:   ku_c1 x kv_c2, ku_c2 x kv_c1
 * (Sec. 2.2: U_t = blkdiag(U_c1, U_c2) R_t, V_t = blkdiag(V_c1, V_c2) W_t;
 * A(I_c1, I_c2) = U_c1 B12_t V_c2^T and A(I_c2, I_c1) = U_c2 B21_t V_c1^T.)
 * The library copies them; the caller keeps ownership. */
typedef struct {
  const double *D, *U, *V, *R, *W, *B12, *B21;
} hss_gen_host;

/* Optional device allocator.  alloc returns NULL on failure (the calling
 * entry point then returns HSS_ENOMEM).  NULL hooks mean hipMalloc/hipFree. */
typedef struct {
  void *(*alloc)(size_t bytes, void *ctx);
  void (*free)(void *ptr, void *ctx);
  void *ctx;
} hss_alloc;

/* Solve options.  prec selects the factor set (HSS_F64 or HSS_F32; the root
 * block of either is factored in FP64).  tol > 0 asks for the normwise
 * backward error eta <= tol: the result is refined with FP64 residuals
 * (r = b - A x by the FP64 product) and corrections from the chosen factors,
 * at most max_refine times.  want_eta != 0 computes eta even when tol == 0. */
typedef struct {
  int32_t prec;
  int32_t max_refine;
  double tol;
  int32_t want_eta;
  int32_t reserved;
} hss_solve_opts;

/* Solve report, written by the device into memory that the caller provides
 * (device memory or pinned host memory from hipHostMalloc) and valid once
 * the stream has reached the end of the solve.  The block starts with this
 * header and continues with ncols doubles: the per-column backward errors
 * eta_j (0 when no backward error was computed).  Its size for nrhs
 * right-hand sides is HSS_SOLVE_INFO_BYTES(nrhs).
 *   eta_max        max_j eta_j (0 if not computed)
 *   norm2          the ||A||_2 estimate used in eta (power method, Sec. 4.5)
 *   iters          refinement steps applied
 *   status         HSS_OK, HSS_ENOCONV (tol not met after max_refine steps;
 *                  B holds the last iterate), HSS_ESINGULAR (an exact zero
 *                  pivot in the factors used) or HSS_EHIP (a bounded
 *                  device-side wait ran out)
 *   singular_node  heap id of a node whose factor has an exact zero pivot,
 *                  -1 if none
 *   ncols          nrhs of the solve (the number of eta_j that follow) */
typedef struct {
  double eta_max;
  double norm2;
  int32_t iters;
  int32_t status;
  int32_t singular_node;
  int32_t ncols;
} hss_solve_info;
#define HSS_SOLVE_INFO_BYTES(nrhs) (sizeof(hss_solve_info) + sizeof(double) * (size_t)(nrhs))

/* hss_create: validate the tree and generators, build the plan (node sizes,
 * offsets, level ranges), upload the generators to device memory, keep a
 * resident FP32 copy and estimate ||A||_2 by 16 steps of the power method on
 * A^T A (Sec. 4.5; a lower bound, so backward errors divided by it are
 * conservative) from a fixed start vector: v_i = the splitmix64 hash of
 * i + 0x5eed mapped to [-1, 1), normalized.  On success *out owns all device
 * memory of the matrix.
 * Errors: -1/-2/-3/-5 for invalid tree/generators/alloc/out, HSS_EUNSUP when a
 * node is larger than the kernels support (leaf size or merged size > 128, rank
 * > 64), HSS_ENOMEM, HSS_EHIP.  Synchronizes the stream. */
hss_status hss_create(const hss_tree_desc *tree, const hss_gen_host *gen,
                      const hss_alloc *alloc, void *stream, hss_handle **out);

/* hss_destroy: free everything the handle owns.  NULL is a no-op. */
hss_status hss_destroy(hss_handle *h);

/* hss_hadamard: the elementwise product C = A o B of two HSS matrices on the
 * same cluster tree (Sec. 4.4, eq. "hadamard" and the figure of its
 * pseudo-codes): D_C = D_A o D_B at the leaves; U_C = U_A .T U_B and
 * V_C = V_A .T V_B, the transpose Khatri-Rao products (row i is
 * kron(row i of U_A, row i of U_B), so column a kB + b is
 * U_A(:, a) o U_B(:, b)); R_C = R_A kron R_B for each child block of the
 * stacked R (likewise W), B12_C = B12_A kron B12_B, B21_C = B21_A kron B21_B.
 * Ranks multiply node by node.  The generators are formed on the device from
 * A's and B's resident FP64 generators (A and B are only read); *out is a new
 * handle, as from hss_create on those generators: resident FP32 copy,
 * ||C||_2 estimate, ready for products and factorizations.
 * Errors: -1/-2 for a NULL A or B, -2 when B's tree (n, leaf offsets)
 * differs from A's, -3 for incomplete allocator hooks, -5 for a NULL out;
 * HSS_EUNSUP when a product rank exceeds 64 or a merged block exceeds 128;
 * HSS_ENOMEM, HSS_EHIP.  Orders after earlier work on the stream, then
 * synchronizes it. */
hss_status hss_hadamard(const hss_handle *A, const hss_handle *B,
                        const hss_alloc *alloc, void *stream, hss_handle **out);

/* hss_compress: HSS recompression with truncation tolerance tau >= 0
 * (absolute; Sec. 4.5 and App. A): the generators of A are first brought
 * to proper form (orthonormal leaf bases and translation operators, by
 * Householder QR from the leaves up, the core blocks multiplied by the
 * triangular factors), then, level by level from the root down, every
 * child's block row [S | R diag(s)] and block column [S'^T | W diag(s')]
 * (s: the singular values kept at the parent) is replaced by its truncated
 * SVD, keeping the singular values > tau and at least one per node of
 * positive rank; core blocks, translation operators and leaf bases are
 * rotated into the kept singular vectors.  Both SVDs of a child use the
 * core blocks of its parent as they were before that level's updates.
 * The result, a new handle on A's tree with ranks <= A's (read them with
 * hss_ranks), satisfies ||A - C||_2 <= 2 (sqrt(2^p) - 1)/(sqrt(2) - 1) tau
 * (Prop. A.1); A is only read.  Device scratch of about
 * 2 (|U| + |V| + |R| + |W| + |B12| + |B21|) + 2 * 64^2 * nnodes doubles is
 * taken from alloc (or hipMalloc) for the call and released before it
 * returns.
 * Errors: -1 NULL A, -2 tau negative, NaN or infinite, -3 incomplete
 * allocator hooks, -5 NULL out; HSS_ENOMEM, HSS_EHIP.  Orders after earlier
 * work on the stream and synchronizes it. */
hss_status hss_compress(const hss_handle *A, double tau, const hss_alloc *alloc,
                        void *stream, hss_handle **out);

/* hss_construct_dense: the HSS approximation of a dense n x n FP64 matrix
 * (Sec. 3.2, the dense constructor: low-rank truncation of every HSS block
 * row and column from the leaves to the root, nested, by truncated SVD).
 * A: DEVICE memory, column-major, leading dimension lda >= n; only read, and
 * D is copied out of it.  The cluster tree is leaf_off (2^p + 1 entries,
 * host, as in hss_tree_desc; leaves of at most 128 rows); the ranks are
 * chosen here.  Level by level from the leaves up, on the matrix M of that
 * level (A at the leaves, then blkdiag(U^_t)^T A blkdiag(V^_t) over the
 * nodes t of the level below, the explicit nested bases U^_t, V^_t):
 *   leaf i:        U_i, V_i = the kept left singular vectors of the block
 *                  row A(I_i, I \ I_i) and of the block column
 *                  A(I \ I_i, I_i)^T; D_i = A(I_i, I_i);
 *   internal t:    R_t, W_t likewise from the block row and block column of
 *                  M formed by t's two children (both from M as it stands
 *                  at the start of the level); B12_t, B21_t = the blocks of
 *                  M coupling the two children.
 * A singular value is kept when it is > eps * sigma_1 of its block, at least
 * one per block (an exactly zero block keeps the first unit vector); the
 * bases come out orthonormal.  *out is a new handle (resident FP32 copy,
 * ||A||_2 estimate; read the ranks with hss_ranks).  Device scratch of about
 * n^2 + 2 (rows x ranks) doubles plus 2 * 128^2 doubles per node is taken
 * from alloc (or hipMalloc) for the call and released before it returns.
 * Errors: -1 NULL A, -2 lda < n, -3 n < 1, -4 p outside 0..30, -5 leaf
 * offsets invalid or NULL, -6 eps negative, NaN or infinite, -7 incomplete
 * allocator hooks, -9 NULL out; HSS_EUNSUP for a leaf above 128 rows or a
 * kept rank above 64; HSS_ENOMEM, HSS_EHIP.  Orders after earlier work on
 * the stream; synchronizes it once per level. */
hss_status hss_construct_dense(const double *A, int64_t lda, int64_t n, int32_t p,
                               const int64_t *leaf_off, double eps,
                               const hss_alloc *alloc, void *stream, hss_handle **out);

/* hss_ranks: the handle's ranks ku_t, kv_t in heap order (0 at the root)
 * into caller arrays of 2^(p+1) - 1 entries.  Host only; no device work.
 * Errors: -1 NULL h, -2 NULL ku, -3 NULL kv. */
hss_status hss_ranks(const hss_handle *h, int32_t *ku, int32_t *kv);

/* Destination of hss_get_generators: host buffers for the canonical packed
 * arrays (the layout and sizes hss_create reads; a pointer may be NULL only
 * when its array is empty, e.g. U, V, R, W when p = 0). */
typedef struct {
  double *D, *U, *V, *R, *W, *B12, *B21;
} hss_gen_out;

/* hss_get_generators: copy the handle's FP64 generators, in the canonical
 * packed layout, to host memory (the read-back of hss_hadamard's result and
 * of any handle).  Entry counts follow from the tree: leaves m^2, m ku, m kv;
 * internal non-root nodes (ku_c1 + ku_c2) ku, (kv_c1 + kv_c2) kv; internal
 * nodes ku_c1 kv_c2 and ku_c2 kv_c1.
 * Errors: -1 NULL h, -2 a missing buffer, HSS_EHIP.  Synchronizes the stream. */
hss_status hss_get_generators(const hss_handle *h, const hss_gen_out *g, void *stream);

/* hss_matmul: Y = op(A) X by the four steps of Sec. 4.1 (leaf projections,
 * upward pass with the column translations, core blocks, downward pass with
 * the row translations, leaf outputs plus D_i X_i).  X and Y are DEVICE
 * pointers to n x nrhs column-major blocks (ld >= n) of double (HSS_F64) or
 * float (HSS_F32, using the resident FP32 generators); they must not overlap.
 * nrhs == 0 is a no-op.  Asynchronous on stream. */
hss_status hss_matmul(hss_handle *h, int32_t op, int32_t prec, int64_t nrhs,
                      const void *X, int64_t ldx, void *Y, int64_t ldy, void *stream);

/* hss_matmul_noalloc: hss_matmul for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as hss_matmul, but
 * the product's work vectors (x^ and y^, 2 * ldm * max(nrhs, 8) elements,
 * ldm = sum over nodes of max(ku_t, kv_t)) live in a fixed 32 MiB device
 * array of the library instead of the handle's growable buffers, so the call
 * never allocates.  Each GPU holds its own copy of that array from library
 * load until the process ends.  Returns HSS_ESCRATCH (nothing enqueued) when
 * the product does not fit; hss_matmul_noalloc_max_rhs gives the largest nrhs
 * that fits (0 if none, -1 for invalid arguments).  The current device must
 * be the handle's.  Every call on a GPU shares that GPU's array: calls that
 * overlap in time on one GPU (on different streams or handles) race, so the
 * caller serializes them, e.g. on one stream. */
hss_status hss_matmul_noalloc(hss_handle *h, int32_t op, int32_t prec, int64_t nrhs,
                              const void *X, int64_t ldx, void *Y, int64_t ldy, void *stream);
int64_t hss_matmul_noalloc_max_rhs(hss_handle *h, int32_t prec);

/* hss_ulv_factor: implicit ULV factorization (Sec. 4.3, Step 1 on the leaves,
 * Step 3 merging siblings level by level, dense LU with partial pivoting of the
 * last merged block) in FP64 or FP32 (the root LU is FP64 in both).  Replaces
 * an earlier factorization of the same precision.  An exact zero pivot is
 * recorded on the device and reported by the next solve (HSS_ESINGULAR).
 * Asynchronous on stream. */
hss_status hss_ulv_factor(hss_handle *h, int32_t prec, void *stream);

/* hss_ulv_solve: B <- A^{-1} B in place (Steps 1, 2 and 4 applied to B with the
 * stored factors).  B is a DEVICE pointer to an n x nrhs FP64 block (ldb >= n).
 * o == NULL means {HSS_F64, 10, 0.0, 0}.  With o->tol > 0 the solve refines
 * B with FP64 residuals (the FP64 product) and corrections from the chosen
 * factors: up to o->max_refine steps are enqueued, each gated on the device
 * by the backward error of the step before it, so steps after convergence
 * do no work and the host never waits.  info (may be NULL) is device memory
 * or pinned host memory of HSS_SOLVE_INFO_BYTES(nrhs) bytes; the solve writes
 * it at its end on the stream.  Returns HSS_OK once the work is enqueued,
 * a negative code for an invalid argument, HSS_ESTATE if the requested
 * precision has not been factored, HSS_ENOMEM or HSS_EHIP; the outcome on the
 * device (HSS_ENOCONV, HSS_ESINGULAR) is info->status. */
hss_status hss_ulv_solve(hss_handle *h, int64_t nrhs, double *B, int64_t ldb,
                         const hss_solve_opts *o, hss_solve_info *info, void *stream);

/* hss_ulv_factor_solve: a fresh system in one call, hss_ulv_factor(h, o->prec)
 * followed by hss_ulv_solve(h, nrhs, B, ldb, o, info) (Sec. 4.3, Steps 1-4),
 * with the same kernels and the same results bit for bit.  In FP64 the
 * forward sweep of the first solve (Step 2 for level l) runs on the
 * handle's second stream as soon as level l is factored, beside the
 * factorization of the levels above it; in FP32 (shorter sweeps than the
 * hand-off costs) the sweep of each level runs right after its
 * factorization on the caller's stream.  The root solve, the backward sweep
 * and the refinement follow on the caller's stream.  Arguments, errors and report as
 * hss_ulv_solve (HSS_ESTATE does not arise).  Asynchronous on stream, which
 * the second stream forks from and joins back with events, so the call is
 * ordered on stream as if it ran there alone (and can be captured). */
hss_status hss_ulv_factor_solve(hss_handle *h, int64_t nrhs, double *B, int64_t ldb,
                                const hss_solve_opts *o, hss_solve_info *info, void *stream);

/* Query keys for hss_query (out is host memory of the stated type). */
#define HSS_Q_N              0   /* int64_t                                        */
#define HSS_Q_P              1   /* int32_t                                        */
#define HSS_Q_RESIDENT_BYTES 2   /* int64_t: device bytes owned by the handle     */
#define HSS_Q_NORM2          3   /* double: power-method ||A||_2 (taken at create) */
#define HSS_Q_GEN_ENTRIES    4   /* int64_t: generator entries (algorithmic size)  */
#define HSS_Q_FACTOR_ENTRIES 5   /* int64_t: entries of one factor set            */
hss_status hss_query(hss_handle *h, int32_t key, void *out, void *stream);

/* Host-only plan helpers (no device needed), used to check the plan against
 * independent implementations.
 * hss_plan_depth: depth p of the default tree (ceil-halving until the blocks
 *   have <= nmin indices, Sec. 3.1).
 * hss_plan_leaf_offsets: fills leaf_off[0 .. 2^p] for that tree.
 * hss_plan_node_ranges: for a tree description, fills start[t], size[t] of the
 *   index set of every node in heap order (2^(p+1)-1 entries each). */
int32_t hss_plan_depth(int64_t n, int64_t nmin);
hss_status hss_plan_leaf_offsets(int64_t n, int64_t nmin, int64_t *leaf_off, int64_t cap);
hss_status hss_plan_node_ranges(const hss_tree_desc *tree, int64_t *start, int64_t *size);

/* Batched calls: one launch per tree level across all handles (levels are
 * aligned at the leaves for upward passes and at the root for downward
 * passes).  Each result equals the single-handle call on the same stream,
 * bit for bit, except for products of 2 to 8 columns, which a batch runs on
 * the per-level kernels and a single call on the mailbox kernels (equal up
 * to the order of the sums).
 * hs: host array of count handles; the per-handle arrays are host arrays of
 * count entries; B / X / Y entries are device pointers.
 * Each call uploads small task tables (the handles' records, the per-level
 * node lists, the right-hand-side pointers) to device memory kept per
 * stream; a table equal byte for byte to one an earlier call on that stream
 * uploaded is reused.  Under HIP graph capture no upload can be recorded, so
 * a batched call is captured only after the same call (same handles, counts,
 * pointers and options) has run on that stream outside capture; otherwise it
 * returns HSS_ESTATE, and the capture (which may hold part of the call) is
 * to be discarded.  Tables used by a captured call are kept for the life of
 * the process. */
hss_status hss_batch_matmul(hss_handle *const *hs, int32_t count, int32_t op, int32_t prec,
                            const int64_t *nrhs, const void *const *X, const int64_t *ldx,
                            void *const *Y, const int64_t *ldy, void *stream);
hss_status hss_batch_ulv_factor(hss_handle *const *hs, int32_t count, int32_t prec,
                                void *stream);
/* hss_batch_ulv_solve: info is NULL or a host array of count pointers,
 * each NULL or a device / pinned block of HSS_SOLVE_INFO_BYTES(nrhs[i])
 * bytes.  Refinement is gated per instance: an instance whose backward error
 * meets tol takes no further corrections, and its iters counts its own. */
hss_status hss_batch_ulv_solve(hss_handle *const *hs, int32_t count, const int64_t *nrhs,
                               double *const *B, const int64_t *ldb, const hss_solve_opts *o,
                               hss_solve_info *const *info, void *stream);

/* Autotuning of launch choices.  The library chooses, per call, between
 * kernel variants that compute the same result: the product of 2 or more
 * columns on the mailbox climb or on the per-level wide kernels (Sec. 4.1,
 * the same four steps), and the number of right-hand-side columns a
 * wavefront carries through a solve sweep (1 or 4; Sec. 4.3 Steps 2 and 4).
 * Built-in rules pick them by default; hss_autotune times both variants of
 * each on h with nrhs columns in precision prec (HSS_F64 / HSS_F32; the
 * solve part needs that factorization and nrhs >= 4), on the stream, and
 * records the faster for every later single-matrix call on a matrix of the
 * same shape class (leaf block size, largest rank, depth, precision, column
 * bucket 1 | 2-3 | 4-7 | 8-15 | 16-31 | 32+), process-wide.  It allocates and
 * frees temporary blocks of n x nrhs through h's allocator and synchronizes
 * the stream.  report (NULL or cap bytes): a JSON object with the shape
 * class, the measured microseconds and the choices (HSS_ESCRATCH if cap is
 * too small).  Batched calls keep the built-in rules.
 * hss_tune_table writes the recorded choices as text, one line per shape
 * class (leaf_mp max_k depth prec bucket product_wide cpw and the four
 * times); hss_tune_load reads such text back (-1 on a malformed line, nothing
 * loaded); hss_tune_reset forgets every choice. */
hss_status hss_autotune(hss_handle *h, int64_t nrhs, int32_t prec, void *stream, char *report,
                        int64_t cap);
hss_status hss_tune_table(char *buf, int64_t cap);
hss_status hss_tune_load(const char *text);
hss_status hss_tune_reset(void);

/* Per-kernel timing (profiling aid).  hss_timing_enable(1) makes every
 * kernel launch of the library record a pair of HIP events on its stream;
 * hss_timing_report writes a JSON array [{"kernel", "launches", "total_ms"}]
 * aggregated since the last reset into buf (cap bytes, NUL-terminated;
 * HSS_EUNSUP if truncated), synchronizing on the recorded events.  Process
 * wide; not for concurrent use from several threads while enabled. */
hss_status hss_timing_enable(int32_t on);
hss_status hss_timing_report(char *buf, int64_t cap, int32_t reset);

/* Text for a status code (static storage). */
const char *hss_status_str(hss_status s);

#ifdef __cplusplus
}
#endif
#endif /* HSS_H_ */
