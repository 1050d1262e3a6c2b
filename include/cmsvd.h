/*
 * cmsvd -- incremental concatenated-SVD merge-error engine for MI355X (gfx950).
 *
 * C ABI of the HIP library libcmsvd.so.  It evaluates the incremental truncated-SVD
 * estimate of the optimal rank-r error of a horizontal concatenation
 * [A_1 ... A_K] (Lemma 1 and Corollary 3 of Shamrai, "Concatenated Matrix SVD:
 * Compression Bounds, Incremental Approximation, and Error-Constrained Clustering",
 * TMLR 2026: Methodology, incremental truncated SVD, and Appendix B) and the plug-in
 * error of Corollary 2, for single updates, for all requested candidate pairs, and
 * inside the greedy error-constrained clustering of Algorithm 3 (Appendix E); and
 * the residual certificate of Theorem 2 / Corollary 1 with the clustering of
 * Algorithm 2, and the Weyl-type certificate of Theorem 1 with the clustering of
 * Algorithm 1.
 *
 * Conventions shared by every call
 *   - Blocks A_i are real m x n_i matrices with a common row count m (Problem
 *     Formulation).  They are passed as cmsvd_block: a DEVICE pointer to a
 *     row-major matrix (element (i, c) at ptr[i * ld + c]), ld >= cols, dtype
 *     CMSVD_F32, CMSVD_BF16 or CMSVD_F64.  FP32 data is promoted to FP64 exactly;
 *     BF16 blocks are first widened to FP32 (exact) in a buffer of the handle, which
 *     holds 4 bytes per element of every BF16 block of the call until the next call
 *     that widens; all arithmetic is FP64 except the optional low-precision
 *     projections (cmsvd_set_projection).
 *   - A state of rank r (the state Algorithm 3 maintains) is a DEVICE basis U
 *     (m x r, row-major FP64, orthonormal or zero columns), DEVICE singular values
 *     S (r FP64, descending, zero-padded), and DEVICE accumulators
 *     acc[4] = {E_tot hi, E_tot lo, D hi, D lo}: the block energy sum_i ||A_i||_F^2
 *     and the energy discarded by truncation, each as a double-double.
 *   - The caller owns every input and output buffer; the handle owns only its
 *     workspace (grown on demand, freed by cmsvd_destroy), pinned staging buffers and
 *     one internal stream for uploads (default priority), whose work is ordered by
 *     events against the handle's stream in both directions.  Device memory comes
 *     from the allocator callbacks given to cmsvd_create_ex (for example PyTorch's
 *     caching allocator), else from hipMalloc; growing a workspace synchronises the
 *     handle's stream first.
 *   - All calls are ordered on the handle's HIP stream.  cmsvd_update,
 *     cmsvd_update_batch, cmsvd_merge_errors and cmsvd_sym_eigvals return once their
 *     work is enqueued (the host may block briefly while descriptor tables are
 *     uploaded, and cmsvd_merge_errors reads the block norms back once when its
 *     candidates are thin enough for the dense projection); results are valid after
 *     a stream synchronisation.  The other calls are synchronous.
 *   - Argument validation happens before any launch.  A non-OK status means no
 *     kernel was launched by that call, except CMSVD_EHIP (a HIP runtime failure),
 *     CMSVD_ENOMEM (a device or host allocation that failed part-way), and the
 *     widening of BF16 blocks, which follows the checks of the blocks themselves and
 *     precedes those of the other arguments (it writes only the handle's buffer).  No C++
 *     exception crosses the ABI: a failed host allocation returns CMSVD_ENOMEM, any
 *     other internal exception CMSVD_EUNSUPPORTED.  cmsvd_last_error() gives a
 *     thread-local message.
 *   - Every symmetric eigenproblem the library solves has order at most 2016: the
 *     core of an update (r_in + n_i), of a candidate merge (r + n_j), a block's or
 *     residual's Gram (n_j) and the explicit Gram of cmsvd_exact_tail (min(m, sum
 *     n_j)).  Larger orders return CMSVD_EUNSUPPORTED; append wider blocks as column
 *     panels (concatenation is associative, so the same matrix results).
 *     cmsvd_compress handles larger Grams by subspace iteration (its rank r_C is
 *     limited to 2016).
 *   - Reproducibility: a call repeated on the same data returns the same bits, except
 *     candidate evaluations whose core order r + n_j is 161..320 (their
 *     tridiagonalisation sums A v over several wavefronts with atomic adds, in an
 *     order that varies) and eigenproblems of order above 320; these agree from run to
 *     run to rounding, |d(err^2)| = O((r + n_j) u ||M||^2) with u = 2^-53.
 *   - NaN/Inf in the data propagate into the affected results; they are not errors.
 *     A rank-deficient residual is not an error either: its numerically absent
 *     directions are dropped (their energy stays in the error estimate).
 */
#ifndef CMSVD_H
#define CMSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cmsvd_ctx* cmsvd_handle;

typedef enum { CMSVD_F32 = 0, CMSVD_BF16 = 1, CMSVD_F64 = 2 } cmsvd_dtype;

/* Precision of the candidate projections Y = U_r^T A_j (see cmsvd_set_projection). */
typedef enum { CMSVD_PROJ_F64 = 0, CMSVD_PROJ_BF16 = 1, CMSVD_PROJ_BF16X3 = 2, CMSVD_PROJ_F32 = 3 } cmsvd_projection;

typedef enum {
    CMSVD_OK = 0,
    CMSVD_EINVAL = 1,      /* bad argument value (null pointer, r < 1, index out of range, ...) */
    CMSVD_ESHAPE = 2,      /* bad shapes (row counts differ, cols < 1, ld < cols, r > m, ...)  */
    CMSVD_ENOMEM = 3,      /* workspace allocation failed                                      */
    CMSVD_EHIP = 4,        /* a HIP runtime call failed                                        */
    CMSVD_EUNSUPPORTED = 5 /* dtype or size not supported by this library                      */
} cmsvd_status;

typedef struct {
    const void* ptr; /* device pointer, row-major                      */
    int64_t rows;    /* m                                               */
    int64_t cols;    /* n_i >= 1                                        */
    int64_t ld;      /* row stride in elements, >= cols                 */
    int32_t dtype;   /* cmsvd_dtype                                     */
} cmsvd_block;

/* Options of a handle (cmsvd_create_ex).  A zero-filled struct gives the defaults.
     projection   precision of the candidate projections (cmsvd_projection; see
                  cmsvd_set_projection, which can change it later)
     chol_tau     c in the pivot threshold c u ||B||_F^2 (u = 2^-52) of the first
                  Cholesky factorisation of CholeskyQR2 in every committed step (Lemma
                  1's thin QR of the residual): a pivot at or below it drops its
                  direction, whose energy stays in the error estimate.  0 = the block
                  width k (the default); at most 1e12.
     panel_cols   cmsvd_update and cmsvd_update_batch append a block wider than this as
                  consecutive column panels of this width (the last one narrower): the
                  same concatenation, truncated after every panel (Lemma 1 holds for any
                  blocking), so results depend on it.  0 = whole blocks (the default).
     graphs       nonzero: repeated cmsvd_merge_errors calls are replayed from a captured
                  HIP graph.  The first call with a given set of arguments (block
                  descriptors, pair list, r, output pointers, projection) runs eagerly and
                  sizes the workspaces; the second captures its launch sequence (kernel
                  nodes only: descriptor tables go to a buffer the graph owns, copied once
                  after the capture) and launches it; later ones launch the graph.  A graph
                  is dropped when a workspace it refers to is reallocated (it is then
                  captured again), and the four most recently used are kept.  A replay
                  reads the blocks' current contents.  Calls whose candidates take the
                  dense projection (thin blocks) are never captured.  Not used while stage
                  timing is on.  0 (the default): every call runs eagerly.
   CholeskyQR always takes two passes. */
typedef struct {
    int32_t projection;
    double chol_tau;
    int64_t panel_cols;
    int32_t graphs;
} cmsvd_options;

/* Creates a handle bound to a HIP stream (NULL = the default stream).  The current
   HIP device at creation time is the device used by every call on the handle.
   Default options; device memory from hipMalloc. */
cmsvd_status cmsvd_create(cmsvd_handle* handle, void* hip_stream);

/* cmsvd_create with options (NULL = defaults) and, optionally, the caller's device
   allocator: alloc(bytes, alloc_ctx) returns device memory of the handle's device (NULL
   on failure, reported as CMSVD_ENOMEM) and release(ptr, alloc_ctx) returns it; give
   both or neither (CMSVD_EINVAL).  The library calls them from the thread that makes
   the call, for its workspaces (grown on demand, released by cmsvd_destroy) and the
   per-call buffers of the synchronous calls (released before they return).  A buffer
   is released only after the work that reads it has completed or, for a grown
   workspace, after the handle's stream has been synchronised.  Out-of-range options
   give CMSVD_EINVAL. */
cmsvd_status cmsvd_create_ex(cmsvd_handle* handle, void* hip_stream, const cmsvd_options* options,
                             void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* alloc_ctx);
cmsvd_status cmsvd_destroy(cmsvd_handle handle);
cmsvd_status cmsvd_set_stream(cmsvd_handle handle, void* hip_stream);

/* Selects the precision of the projections Y = U_r^T A_j that candidate evaluations
   compute (Lemma 1; the off-diagonal block of the enlarged Gram of Corollary 3) in
   cmsvd_merge_errors and in the scan of cmsvd_cluster.
     CMSVD_PROJ_F64    (default) operands promoted to FP64 exactly, FP64 accumulation.
     CMSVD_PROJ_BF16   every element x of U_r and of A_j is rounded to FP32 (x32) and
                       then to BF16 (hi), both round-to-nearest-even; the products
                       hi_U hi_A are summed in FP32 on the matrix cores and widened to
                       FP64.
     CMSVD_PROJ_BF16X3 the same with lo = BF16(x32 - hi) staged too, summing
                       lo_U hi_A + hi_U lo_A + hi_U hi_A in FP32: three BF16 matrix-core
                       passes that carry about 16 significant bits per operand.
     CMSVD_PROJ_F32    every element of U_r and of A_j is rounded to FP32 (round-to-
                       nearest-even; FP32 data is unchanged) and the products are summed
                       in FP32 on the matrix cores (v_mfma_f32_16x16x4f32), then widened
                       to FP64.
   Everything else stays FP64: block norms and Grams A_j^T A_j, the anchors'
   truncations and every state update of the clustering (an accepted candidate is
   committed in FP64), the residual ordering of sort_mode 1, the core eigenvalues and
   the compensated plug-in subtraction.  The core is evaluated in Gram form
   [[S^2, S Y], [Y^T S, A_j^T A_j]], where an error in Y moves the top-r eigenvalue sum
   to first order, so the relative deviation of err from the FP64 path grows as
   err / ||[A_i, A_j]||_F shrinks.  Returns CMSVD_EINVAL for any other value; the
   setting applies to calls issued afterwards on this handle. */
cmsvd_status cmsvd_set_projection(cmsvd_handle handle, int32_t precision);
const char* cmsvd_last_error(void);

/* One incremental step: Lemma 1 (projection Y = U^T B, residual R = B - U Y, thin
   QR of R) and Corollary 3 (eigendecomposition of the enlarged Gram S_{t+1},
   truncation to the top r pairs), then the plug-in of Corollary 2.
     m            row count of the state and of B
     U, ldu       current basis, m x r_in row-major FP64 (ignored when r_in == 0)
     S            current singular values, r_in FP64 (ignored when r_in == 0)
     r_in         current state width (0 = empty state: the update then computes the
                  rank-r truncated SVD of B, Algorithm 3 step 1)
     B            the appended block (rows == m); wider than the handle's panel_cols
                  option, it is appended as consecutive column panels (cmsvd_options)
     r            target rank, 1 <= r <= m
     U_out, ldu_out  new basis, m x r row-major FP64 (must not alias U)
     S_out        new singular values, r FP64 (must not alias S)
     acc          state accumulators (see above), updated in place
     est          optional (may be NULL): est[0] = plug-in error sqrt(E_tot -
                  sum S_out^2) after the step, est[1] = sqrt(D) (the same quantity
                  from the discarded-energy tally; they agree to rounding).
   Directions whose eigenvalue is at rounding level get S_out = 0 and a zero column. */
cmsvd_status cmsvd_update(cmsvd_handle handle, int64_t m, const double* U, int64_t ldu, const double* S,
                          int64_t r_in, const cmsvd_block* B, int64_t r, double* U_out, int64_t ldu_out,
                          double* S_out, double* acc, double* est);

/* Several independent incremental steps at once (for example chains advanced in
   lockstep): step i takes state (U[i], S[i]) of width r_in, appends B[i] and writes
   (U_out[i], S_out[i]), updating acc[i] and est[i] (est may be NULL, or hold NULL
   entries).  Every argument means what it means for cmsvd_update; the pointer
   arguments are HOST arrays of count DEVICE pointers (U and S are ignored when
   r_in == 0), B is a host array of count block descriptors.  The steps share m, r,
   r_in and the leading dimensions; different steps must not share output buffers. */
cmsvd_status cmsvd_update_batch(cmsvd_handle handle, int64_t count, int64_t m, const double* const* U, int64_t ldu,
                                const double* const* S, int64_t r_in, const cmsvd_block* B, int64_t r,
                                double* const* U_out, int64_t ldu_out, double* const* S_out, double* const* acc,
                                double* const* est);

/* Merge errors for ordered candidate pairs (Corollary 2 applied to [A_i, A_j]: the
   anchor A_i is truncated to rank r first, then A_j is appended; order matters,
   Remark 3).
     blocks, nblocks   the collection (host array of descriptors of device data)
     pairs             HOST int32 array npairs x 2, (i, j) with 0 <= i, j < nblocks
     r                 target rank, 1 <= r <= m
     err               DEVICE npairs FP64: plug-in error sqrt(||A_i||^2 + ||A_j||^2 -
                       sum_{l<=r} sigma_l^2)
     rel               DEVICE npairs FP64 (may be NULL): err / ||[A_i, A_j]||_F
   nblocks and npairs are at most 2^31 - 1 (else CMSVD_EUNSUPPORTED).  Lists of a
   million pairs or more are checked and grouped on up to 16 host threads.  Thin candidates
   given as consecutive column ranges of one row-major matrix (in index order, one
   dtype and row stride) are read in place; others are first packed side by side. */
cmsvd_status cmsvd_merge_errors(cmsvd_handle handle, const cmsvd_block* blocks, int64_t nblocks,
                                const int32_t* pairs, int64_t npairs, int64_t r, double* err, double* rel);

/* Algorithm 3 (approximate clustering via incremental truncated SVD), pass-based:
   anchor = largest remaining block (ties: lower index); a pass orders the
   remaining candidates once (sort_mode 0: increasing ||A_j||_F; 1: increasing
   ||(I - Q_C Q_C^T) A_j||_F against the state at the pass start; ties: lower index)
   and scans them, accepting a candidate iff err / ||M_{C+j}||_F <= eps and then
   continuing the scan against the new state; passes repeat until one accepts
   nothing.
     labels       HOST nblocks int32: cluster id per block, ids in creation order
     nclusters    HOST out
     cluster_rel  HOST nblocks FP64 (may be NULL): final err/||M_C||_F per cluster
                  (first *nclusters entries) */
cmsvd_status cmsvd_cluster(cmsvd_handle handle, const cmsvd_block* blocks, int64_t nblocks, int64_t r,
                           double eps, int32_t sort_mode, int32_t* labels, int64_t* nclusters,
                           double* cluster_rel);

/* Autotuner of the scan schedule of Algorithm 3 (cmsvd_cluster): after an acceptance
   the scan evaluates the rest of the pass in chunks, the first of `chunk` candidates,
   doubling while none is feasible.  For candidates of width k (bucketed to the next
   power of two, at least 16) appended to rank-r states of m rows, with the handle's
   projection precision, it times one evaluation launch sequence of c synthetic
   candidates for c = 16, 32, .., 1024 (HIP events, best of three after a warm-up) and
   picks the largest c that costs at most 15 % more than c = 16: the candidates the
   device evaluates side by side for about the price of the smallest chunk.  When the
   cores (order r + k) exceed 320, the general eigen kernel's workgroup is measured the
   same way with 1024 and with 512 threads per problem, and the size with the lower time
   per candidate at its own chunk is kept for candidate evaluations (cmsvd_merge_errors
   and the scan) whose core order falls in the same power-of-two bucket as r + k.  The
   choices are kept in the handle (cmsvd_cluster uses the chunk of the median remaining
   width; shapes without one start at a quarter of the compute units) and in cache_path
   (may be NULL), a JSON object with one entry per line keyed "gfx950 m=.. k=.. r=..
   proj=..", holding the chosen chunk, the workgroup size (0: not applicable) and the
   measured times.  An entry already in the cache is
   loaded instead of measured unless force is nonzero.
     chunk_out   HOST out (may be NULL): the chunk chosen
   Synchronous; uses about (2 m k + m r + k^2) doubles of device memory while it runs. */
cmsvd_status cmsvd_autotune(cmsvd_handle handle, int64_t m, int64_t k, int64_t r, const char* cache_path,
                            int32_t force, int64_t* chunk_out);

/* The decisions of the last cmsvd_cluster call on this handle, for replaying them:
   for every cluster in creation order, its anchor and then the blocks it accepted, in
   the order of acceptance (each was evaluated against the state left by the previous
   entry of its cluster).  Every block appears once.
     order  HOST cap int32 (may be NULL with cap 0: *n is set and nothing copied)
     n      HOST out: the number of entries (nblocks of that call; 0 before any call)
   CMSVD_ESHAPE when cap < *n and order is given. */
cmsvd_status cmsvd_cluster_trace(cmsvd_handle handle, int32_t* order, int64_t cap, int64_t* n);

/* Algorithm 2 (residual-based clustering, Appendix E) with the certificate of
   Corollary 1: a cluster C keeps an orthonormal basis Q_C of the span of its blocks,
   its energy S_C and the r largest singular values mu of its concatenated residuals
   R_j = (I - Q Q^T) A_j, Q spanning the blocks accepted before j (Theorem 2).  The
   residual ranges are mutually orthogonal, so a candidate's certificate is
     b^2 = S_C + ||A_j||_F^2 - (sum of the r largest squares in mu u sigma(R_j)),
   which bounds the optimal rank-r error of M_{C+j} from above; the candidate joins
   iff b / ||M_{C+j}||_F <= eps (non-strict).  The loop is the pass-based one of
   cmsvd_cluster (same anchor choice, sort modes, tie rules and scan semantics), with
   the residual ordering ||(I - Q_C Q_C^T) A_j||_F taken against the full-span basis.
   Numerical span: the residual is projected twice and orthonormalised by
   CholeskyQR2; a direction whose squared singular value is below about
   k_j u ||A_j||_F^2 (u = 2^-52, the pivot threshold) is not added to Q_C.  Q_C takes
   m * min(m, sum_j n_j) doubles of device memory for the whole call.
     labels, nclusters   as cmsvd_cluster
     cluster_rel  HOST nblocks FP64 (may be NULL): the certified ratio
                  b / ||M_C||_F of each final cluster (first *nclusters entries)
   Synchronous. */
cmsvd_status cmsvd_cluster_residual(cmsvd_handle handle, const cmsvd_block* blocks, int64_t nblocks, int64_t r,
                                    double eps, int32_t sort_mode, int32_t* labels, int64_t* nclusters,
                                    double* cluster_rel);

/* Corollary 1 for a fixed order: the residual certificate of [A_1 ... A_K] with the
   blocks processed in the given order (the same state updates as
   cmsvd_cluster_residual, every block accepted).
     bound2   HOST out: S - sum_{l<=r} mu_l^2, clamped at 0 (an upper bound on the
              optimal rank-r error squared of the concatenation)
     mu       HOST r FP64 (may be NULL): the r largest residual singular values,
              descending, zero-padded
   Synchronous. */
cmsvd_status cmsvd_residual_bound(cmsvd_handle handle, const cmsvd_block* blocks, int64_t nblocks, int64_t r,
                                  double* bound2, double* mu);

/* Theorem 1 (Weyl-type bound) for a set of blocks: bound2 = S - max_j h_j, clamped at
   0, where S = sum_j ||A_j||_F^2 and h_j = sum_{l<=r} sigma_l(A_j)^2 is block j's
   r-head energy (its whole energy when it has at most r columns, else the sum of the r
   largest eigenvalues of its Gram A_j^T A_j).  An upper bound on the optimal rank-r
   error squared of the concatenation, for every r >= 1.
     bound2   HOST out
   Synchronous. */
cmsvd_status cmsvd_weyl_bound(cmsvd_handle handle, const cmsvd_block* blocks, int64_t nblocks, int64_t r,
                              double* bound2);

/* Algorithm 1 (Weyl-based max-norm clustering, Appendix E) with the certificate of
   Theorem 1: a cluster C keeps S_C and m_C = max_{j in C} h_j (h_j as in
   cmsvd_weyl_bound; when r covers every block's rank this is the largest block
   energy of the algorithm's step list); a candidate joins iff
   sqrt(max(0, S_C + ||A_j||^2 - max(m_C, h_j))) / sqrt(S_C + ||A_j||^2) <= eps.
   Anchor = largest remaining block by Frobenius norm; a pass scans the remaining
   blocks by increasing Frobenius norm (ties: lower index) and updates the state at
   each acceptance; passes repeat until one accepts nothing.
     labels, nclusters   as cmsvd_cluster
     cluster_rel  HOST nblocks FP64 (may be NULL): the certified ratio of each cluster
   Synchronous. */
cmsvd_status cmsvd_cluster_weyl(cmsvd_handle handle, const cmsvd_block* blocks, int64_t nblocks, int64_t r,
                                double eps, int32_t* labels, int64_t* nclusters, double* cluster_rel);

/* The optimal rank-r error squared of the concatenation, sum_{l>r} sigma_l^2 (Problem
   Formulation; Eckart-Young), from the eigenvalues of its explicit Gram (M^T M or
   M M^T, whichever is smaller): the reference value of the slack diagnostics.
   The workspace holds M in FP64.
     tail2    HOST out, clamped at 0
   Synchronous. */
cmsvd_status cmsvd_exact_tail(cmsvd_handle handle, const cmsvd_block* blocks, int64_t nblocks, int64_t r,
                              double* tail2);

/* Compression back-end (Problem Formulation, cluster-concatenate-SVD representation):
   the factors stored for one cluster M_C = [A_1 ... A_K] (the blocks given, in order),
   the rank-r_C truncated SVD with the singular values absorbed into the left factor,
   U~ = U S (m x r_C) and V (N_C x r_C), N_C = sum_j n_j, r_C = min(r, m, N_C).  Block j
   is recovered as U~ V_j^T with V_j its n_j rows of V; the error of the cluster is
   sum_{l > r_C} sigma_l^2 (Eckart-Young) and its memory r_C (m + N_C).  Computed from
   the eigenpairs of the explicit Gram (M^T M or M M^T, whichever is smaller, order
   n = min(m, N_C)); directions whose Gram eigenvalue is at most 8 n u lambda_1 (the
   Gram's resolution) are stored as zero columns.  For n above 2016 the top r_C
   eigenpairs come from subspace iteration on p = min(2016, max(2 r_C, r_C + 32))
   columns (CholeskyQR2 between products, Rayleigh-Ritz on X^T G X every step) until
   the sum of the top r_C Ritz values changes by at most 1e-14 relative, or after 60
   steps; the factors are then the Ritz projection, so tail2 is exactly their error and
   never below the optimum (Ky Fan), and the gap to it is the iteration's convergence.
   r_C above 2016 returns CMSVD_EUNSUPPORTED.
     Ut      DEVICE out, row-major m x r_C FP64, row stride ldu >= r_C: U S
     Vt      DEVICE out, row-major r_C x N_C FP64, row stride ldv >= N_C: V^T (block j
             occupies its n_j columns, in the order given)
     rank    HOST out: r_C
     tail2   HOST out: sum_{l > r_C} sigma_l^2 of M_C, clamped at 0
     energy  HOST out (may be NULL): ||M_C||_F^2
   The workspace holds M_C and its Gram in FP64.  Synchronous. */
cmsvd_status cmsvd_compress(cmsvd_handle handle, const cmsvd_block* blocks, int64_t nblocks, int64_t r, double* Ut,
                            int64_t ldu, double* Vt, int64_t ldv, int64_t* rank, double* tail2, double* energy);

/* The compression back-end over a whole partition (Problem Formulation; the
   compression ratio and realised error of the Experiments): for every cluster c =
   0 .. K-1 of labels (K = max label + 1; every id must have a block), cmsvd_compress
   of its blocks in index order, and the partition's summary
     ratio      = (sum over blocks of m n_i) / (sum over clusters of r_c (m + N_c)),
                  the stored entries of the blocks over those of the factors
     rel_error  = sqrt(sum_c tail2_c / sum_c ||M_c||_F^2)
     labels     HOST nblocks int32, cluster id per block (as the clustering calls return)
     Ut, ldu, Vt, ldv  HOST arrays of K entries (all four NULL: the factors are formed
                  in a scratch buffer and only the summary is returned): cluster c's
                  factors as in cmsvd_compress (Ut[c] m x r_c, Vt[c] r_c x N_c, DEVICE)
     ranks, tail2, energy  HOST arrays of K entries (each may be NULL): r_c, the
                  cluster's optimal rank-r_c error squared and ||M_c||_F^2
     nclusters, ratio, rel_error  HOST out
   Synchronous. */
cmsvd_status cmsvd_compress_partition(cmsvd_handle handle, const cmsvd_block* blocks, int64_t nblocks,
                                      const int32_t* labels, int64_t r, double* const* Ut, const int64_t* ldu,
                                      double* const* Vt, const int64_t* ldv, int64_t* ranks, double* tail2,
                                      double* energy, int64_t* nclusters, double* ratio, double* rel_error);

/* Tail energy of a chain and its gradient with respect to every block.
   The chain folds the blocks in order (the incremental state of Lemma 1 and
   Corollary 3, starting from the empty state); the tail energy is Corollary 2's
   plug-in f = E~_r^2 = sum_t ||A_t||_F^2 - sum_{l<=r} sigma_l^2 of the final state.
   The paper gives no gradient; the one computed here is the reverse mode through
   every truncation: with H_t the Gram of step t and W_t the derivative of the
   retained energy with respect to H_t, W_T projects onto the kept eigenvectors and
   W_t applies the Daleckii-Krein divided differences of the truncation to W_{t+1}
   (1 between kept eigenvalues, 0 between dropped ones, lam_i / (lam_i - lam_j)
   between a kept lam_i and a dropped lam_j); d f / d A_t = 2 A_t - 2 W_t A_t.  W_t is
   carried in factored form (m x r and r x r factors), so the reverse sweep costs
   GEMMs of the forward's sizes.
     blocks, nblocks   the chain, in order (device data, common row count m)
     r                 target rank, 1 <= r <= m
     checkpoint        steps between stored states (>= 1).  The forward keeps only
                       every checkpoint-th state; the backward recomputes the states
                       in between, and each step's residual basis and core
                       eigenvectors, instead of storing them.  Device memory:
                       about (nblocks / checkpoint + checkpoint + 6) m r doubles.
     f                 HOST out: the tail energy f
     grads             HOST array of nblocks DEVICE pointers, or NULL for the
                       forward only; grads[t] receives d f / d A_t as an m x n_t
                       row-major FP64 matrix with row stride n_t
     min_gap           HOST out (may be NULL): min over steps of
                       (lam_r - lam_{r+1}) / lam_1 of the step's core spectrum; the
                       gradient does not exist where this is 0 (a tie at the cut)
   Synchronous.  The device memory for states and factors is allocated per call (through
   the handle's allocator) and released before it returns. */
cmsvd_status cmsvd_tail_energy_grad(cmsvd_handle handle, const cmsvd_block* blocks, int64_t nblocks, int64_t r,
                                    int64_t checkpoint, double* f, double* const* grads, double* min_gap);

/* Building block exposed for testing and reuse: the largest nkeep eigenvalues of
   count symmetric matrices, each n x n column-major FP64 on the device (A + i*stride_a,
   lower triangle read, both triangles assumed equal), written descending to
   lam + i*nkeep (device).  Same kernel as the core step of the two calls above. */
cmsvd_status cmsvd_sym_eigvals(cmsvd_handle handle, const double* A, int64_t n, int64_t lda, int64_t stride_a,
                               int64_t count, int64_t nkeep, double* lam);

/* Size in bytes of the fixed device scratch of cmsvd_sym_eigvals_noalloc. */
#define CMSVD_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory: code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc.  The same computation and kernels as
   cmsvd_sym_eigvals (same arguments, layout, results and errors), but it calls no
   hipMalloc, hipFree, host staging copy or other allocating routine: the per-problem
   descriptors are written by a kernel, and they and the eigen kernel's tile slots live
   in a fixed array of CMSVD_NOALLOC_SCRATCH_BYTES in the library's code object (one
   copy per device, held until the process ends, its address looked up when a handle is
   created on that device).  Orders above 320 keep T (T + 1) / 2 tiles of 32 x 32
   doubles per workgroup slot (T = ceil(n / 32)); the call runs as many slots as fit
   beside the descriptors (at least one, so order 2016 runs on 3 workgroups: correct but
   slow).  A count or order whose descriptors and one slot do not fit returns
   CMSVD_EUNSUPPORTED before any launch.  Every call on a device shares that device's
   scratch and leaves its contents behind: calls that overlap on one device (several
   handles or streams) race and must be ordered by the caller.  Asynchronous on the
   handle's stream. */
cmsvd_status cmsvd_sym_eigvals_noalloc(cmsvd_handle handle, const double* A, int64_t n, int64_t lda,
                                       int64_t stride_a, int64_t count, int64_t nkeep, double* lam);

/* Graph use of the handle so far (cmsvd_options.graphs): sequences captured, graph
   replays, and the wall time of the last capture in milliseconds (capture,
   instantiation and the copy of its descriptor tables; excluded from the replays).
   Each output may be NULL. */
cmsvd_status cmsvd_graph_stats(cmsvd_handle handle, int64_t* captures, int64_t* replays, double* last_capture_ms);

/* Stage timing for measurement (off by default).  When enabled, every pipeline stage
   launched on the handle's stream is bracketed by HIP events recorded on that same
   stream.  Stages: 0 = block norms and Grams B^T B, 1 = commit pipeline (anchor
   initialisation and state updates), 2 = projection GEMM Y = U^T B of candidate
   evaluation, 3 = core eigenvalue kernel of candidate evaluation (tridiagonalisation,
   and for all but cores of order 161..320 also bisection and the plug-in error; one
   launch per evaluation chunk; cores of order 193..320 stop here after n - 192 column
   steps), 4 = the bisection kernel that finishes the evaluation of cores of order
   161..320 (eigenvalues of their tridiagonals, plug-in error), 5 = the
   tridiagonalisation of the trailing 192 x 192 matrices that cores of order 193..320
   hand over (three launches: four wavefronts per problem down to order 160 and to 64,
   then one wavefront per problem; two or more problems per compute unit).
   cmsvd_profile_read synchronises the handle's stream, writes for each of the 6
   stages the summed milliseconds and the number of bracketed launches, and resets
   the counters.  ms and count are HOST arrays of 6 entries. */
cmsvd_status cmsvd_profile(cmsvd_handle handle, int32_t enable);
cmsvd_status cmsvd_profile_read(cmsvd_handle handle, double* ms, int64_t* count);

/* Building block exposed for testing and reuse: one FP64 GEMM on the matrix cores,
   C = alpha op(A) op(B) + beta C, all column-major on the device.  op(A) is M x K,
   op(B) is K x N; trans_a / trans_b = 1 selects the transpose.  A and B may be FP32
   or FP64 (a_dtype / b_dtype); C is FP64.  Same kernel as the projections, Grams and
   rotations of the update (step (a) P = U^T B is trans_a = 0, trans_b = 1 on the
   column-major views of the row-major U and B). */
cmsvd_status cmsvd_gemm_f64(cmsvd_handle handle, int32_t trans_a, int32_t trans_b, int64_t M, int64_t N, int64_t K,
                            double alpha, const void* A, int64_t lda, int32_t a_dtype, const void* B, int64_t ldb,
                            int32_t b_dtype, double beta, double* C, int64_t ldc);

/* The same GEMM with BF16 operands, the kernel of CMSVD_PROJ_BF16 (passes = 1) and
   CMSVD_PROJ_BF16X3 (passes = 3): every element of op(A) and op(B) is rounded to FP32
   and then to BF16 (round-to-nearest-even) as it is staged, with the BF16 remainder as
   a second part when passes = 3; products are summed in FP32 on the matrix cores
   (v_mfma_f32_16x16x32_bf16), and alpha, beta and C are FP64.  Otherwise the same
   arguments and errors as cmsvd_gemm_f64; passes other than 1 or 3 give CMSVD_EINVAL. */
cmsvd_status cmsvd_gemm_bf16(cmsvd_handle handle, int32_t passes, int32_t trans_a, int32_t trans_b, int64_t M,
                             int64_t N, int64_t K, double alpha, const void* A, int64_t lda, int32_t a_dtype,
                             const void* B, int64_t ldb, int32_t b_dtype, double beta, double* C, int64_t ldc);

/* The same GEMM with FP32 operands, the kernel of CMSVD_PROJ_F32: every element of
   op(A) and op(B) is rounded to FP32 (round-to-nearest-even) as it is staged, products
   are summed in FP32 on the matrix cores (v_mfma_f32_16x16x4f32), and alpha, beta and C
   are FP64.  Otherwise the same arguments and errors as cmsvd_gemm_f64. */
cmsvd_status cmsvd_gemm_f32(cmsvd_handle handle, int32_t trans_a, int32_t trans_b, int64_t M, int64_t N, int64_t K,
                            double alpha, const void* A, int64_t lda, int32_t a_dtype, const void* B, int64_t ldb,
                            int32_t b_dtype, double beta, double* C, int64_t ldc);

#ifdef __cplusplus
}
#endif
#endif /* CMSVD_H */
