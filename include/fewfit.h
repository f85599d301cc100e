/*
 * fewfit -- multi-versioned single-precision GEMM with portability-tuned
 * variant sets, for AMD Instinct MI355X (gfx950).
 *
 * C ABI of libfewfit.so.  Every entry point returns an int status (0 or a
 * non-negative result on success, a negative FF_* code on failure), never
 * throws, and takes plain pointers and sizes.  Device pointers are HIP
 * device addresses; `stream` is a hipStream_t passed as void* (NULL = the
 * default stream).  The text of the last error of the calling thread is
 * available from fewfit_last_error().
 *
 * Method (arXiv 2507.15277, "A Few Fit Most"):
 *   - a GEMM kernel whose tuning parameters are compile-time constants is
 *     compiled ahead of time into a family of code variants (Sec. III-A,
 *     Sec. III-B: runtime recompilation costs far more than a run, and
 *     precompiling the whole space is too large);
 *   - PortabilityTune selects a small set kappa of variants that is best by
 *     a summary metric over a set of inputs (Sec. IV-B), scored by the
 *     library cost function of Eq. 1 (Sec. IV-D-1);
 *   - at run time one member of kappa is picked per input (Fig. 1, online
 *     inference).
 *
 * All matrices are row-major FP32 with no transposes:
 *   A is M x K with row stride lda >= max(1,K),
 *   B is K x N with row stride ldb >= max(1,N),
 *   C is M x N with row stride ldc >= max(1,N).
 * Sizes M, N, K must fit in int32 (else FF_ERR_TOO_LARGE).
 */
#ifndef FEWFIT_H
#define FEWFIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes.  -1 .. -11 name the invalid argument of sgemm() by
 * position, in the manner of reference BLAS xerbla. */
#define FF_OK 0
#define FF_ERR_M (-1)          /* M < 0 */
#define FF_ERR_N (-2)          /* N < 0 */
#define FF_ERR_K (-3)          /* K < 0 */
#define FF_ERR_A (-5)          /* A == NULL while A must be read */
#define FF_ERR_LDA (-6)        /* lda < max(1,K) */
#define FF_ERR_B (-7)          /* B == NULL while B must be read */
#define FF_ERR_LDB (-8)        /* ldb < max(1,N) */
#define FF_ERR_C (-10)         /* C == NULL while M*N > 0 */
#define FF_ERR_LDC (-11)       /* ldc < max(1,N) */
#define FF_ERR_NO_SET (-100)   /* no variant set loaded */
#define FF_ERR_VARIANT (-101)  /* unknown variant id */
#define FF_ERR_PARSE (-102)    /* malformed set file or manifest */
#define FF_ERR_ARCH (-103)     /* set or code object built for another GPU */
#define FF_ERR_HIP (-104)      /* a HIP runtime call failed */
#define FF_ERR_IO (-105)       /* file missing or unreadable */
#define FF_ERR_TOO_LARGE (-106)/* M, N or K above INT32_MAX, or pieces beyond the workspace */
#define FF_ERR_ARG (-107)      /* other invalid argument (tuning ABI) */

/* Precision forms: how the FP32 product is formed (accumulation and the
 * alpha/beta epilogue are FP32 in every form). */
#define FF_FORM_FP32 0    /* FP32 MFMA */
#define FF_FORM_BF16X3 1  /* split-bf16, 3 products: hi*hi + hi*lo + lo*hi */
#define FF_FORM_BF16X6 2  /* split-bf16 in 3 pieces, 6 products */
#define FF_FORM_FP16S 3   /* per-matrix power-of-two scaled fp16, 1 product */
#define FF_FORM_FP16X3 4  /* the same scaled fp16 in 2 pieces, 3 products */
/* Not a form of its own: the slot of a set whose members may be of any of
 * the forms above, chosen per shape for an accuracy target (portability
 * tuning over the variants whose measured normwise error meets the target,
 * the form being one more tuned parameter; Sec. IV-B, Eq. 1).  Each call
 * runs the chosen member in that member's own form. */
#define FF_FORM_MIXED 5

/* ---------------------------------------------------------------------
 * Hot path
 * ------------------------------------------------------------------- */

/*
 * C <- alpha * A * B + beta * C   (SGEMM; the operation the paper tunes,
 * title and Sec. V).
 *
 * Dispatches to the member of the loaded variant set that variant_select()
 * names for (M, N, K) and launches it on `stream`.  Asynchronous: returns
 * after the launch is enqueued; kernel faults surface at the caller's next
 * synchronisation.  Allocates nothing.
 *
 * Reference-BLAS semantics:
 *   - M == 0 or N == 0, or ((alpha == 0 or K == 0) and beta == 1): returns
 *     without touching C;
 *   - alpha == 0 or K == 0: A and B are not read, C <- beta * C;
 *   - beta == 0: C is not read (NaN or Inf in C does not propagate).
 * Arguments are validated in order before any HIP call; the first invalid
 * one is reported (FF_ERR_M ... FF_ERR_LDC).  Returns FF_ERR_NO_SET when no
 * set is loaded and the call would launch a GEMM kernel.
 *
 * Variants that split K over work-groups write their partial products to
 * one workspace per device (allocated when such a variant is first loaded)
 * and a second kernel sums them.  Calls that use that workspace (or the
 * other per-device buffers of sgemm_form()) are ordered across streams by
 * the library: a call on another stream than the previous such call first
 * waits for everything enqueued so far on that previous stream (an event
 * recorded there at that moment), so concurrent calls on several streams
 * give the same results as one stream; calls on one stream pay nothing
 * for it.  If the previous stream has been destroyed meanwhile, the call
 * synchronises the device instead.  A call made while its stream is being
 * captured into a HIP graph takes no part in that ordering (the library
 * cannot see when the graph is launched): replays of such a graph are
 * ordered with other calls on the device only by the stream they are
 * launched on.
 *
 * Each variant is deterministic: the same inputs give bitwise the same C.
 * Different variants may round differently.  The result of every variant
 * satisfies |C - C_exact| <= 4*K*2^-24*|alpha|*(|A||B|) elementwise, plus
 * 2*2^-24*(|alpha*A*B| + |beta*C|) when the epilogue rounds.
 */
int sgemm(int64_t M, int64_t N, int64_t K, float alpha,
          const float *A, int64_t lda, const float *B, int64_t ldb,
          float beta, float *C, int64_t ldc, void *stream);

/*
 * Load a variant set file (the output of portability tuning, Sec. IV-B):
 * the k member variants, their parameters, the GPU architecture they were
 * built for, its precision form (a "form" line; FP32 when absent; "mixed"
 * for FF_FORM_MIXED, whose members may be of any form), and the dispatch
 * table of training shapes.  Only the k code
 * objects of the set are loaded (Sec. III-B-3: pre-selection keeps the
 * number of shipped variants small).  Replaces any previously loaded set
 * of the same form.  At most 64 members.  The dispatch's wave correction is
 * tabulated for the current device at load.
 * Not safe to call concurrently with sgemm() on another thread.
 * Returns k on success; FF_ERR_IO, FF_ERR_PARSE, FF_ERR_ARCH, FF_ERR_HIP.
 */
int variant_set_load(const char *path);

/*
 * sgemm() in precision form `form` (FF_FORM_*), dispatched through the set
 * loaded for that form (FF_FORM_MIXED: through the mixed set, each call in
 * its chosen member's form).  The 16-bit forms split each FP32 operand into
 * bfloat16 or scaled float16 pieces inside the kernel and accumulate the
 * piece products in FP32 (not a paper method: an MI355X form of the same
 * operation).  Per-element error, as a multiple of |alpha|(|A||B|): about
 * 3.1*2^-16 (bf16x3), 4.2*2^-24 (bf16x6), 2.1*2^-11 (fp16s, for operands
 * within 2^25 of each matrix's largest magnitude), 3.1*2^-22 (fp16x3, for
 * operands within 2^18 of each matrix's largest magnitude; smaller ones
 * lose bits of their low piece to FP16 underflow), plus FP32 accumulation.
 * The fp16s and fp16x3 forms first reduce max|A| and max|B| on the device
 * into the per-device workspace and need finite inputs.  Pre-split variants
 * (LDS mode 2) first form the pieces of A and B into a 1 GiB per-device
 * pieces workspace (allocated when such a variant is loaded) and return
 * FF_ERR_TOO_LARGE when 2 * T * (Mp + Np) * Kp bytes exceed it (T pieces
 * per value, Mp, Np rounded up to the tile, Kp = K rounded up to 64).  Calls
 * on several streams are ordered on these buffers as described at sgemm().
 * Other semantics as sgemm(); FF_ERR_ARG for an unknown form.
 */
int sgemm_form(int form, int64_t M, int64_t N, int64_t K, float alpha,
               const float *A, int64_t lda, const float *B, int64_t ldb,
               float beta, float *C, int64_t ldc, void *stream);

/*
 * sgemm_form() for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same dispatch, split count and kernels as sgemm_form(), so the result is
 * bitwise equal to sgemm_form()'s on the same inputs; but every scratch
 * buffer the kernels use comes from one fixed device array of
 * FF_NOALLOC_SCRATCH_BYTES (256 MiB), which each device holds from this
 * entry point's first call on it until the process ends.  The call makes no
 * hipMalloc, hipFree or other allocating call (the variant set must be
 * loaded beforehand; variant_set_load() allocates).  Layout of the array:
 * 16 KiB of FP16 block maxima and exponents, then the pre-split pieces
 * (2 * T * (Mp + Np) * Kp bytes, as at sgemm_form(), rounded up to 256),
 * then the K-split slices (splits * M * N * 4 bytes); a call that needs
 * more than the array returns FF_ERR_TOO_LARGE before any launch.  Every
 * call on one device shares that device's array, which keeps the last
 * call's contents (nothing in it must start at zero: each call writes what
 * it reads).  Calls that overlap in time on one device race and give wrong
 * results: issue them on one stream, or order the streams.  Returns as
 * sgemm_form(); FF_ERR_HIP if the array's device address cannot be had.
 */
#define FF_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int sgemm_form_noalloc(int form, int64_t M, int64_t N, int64_t K, float alpha,
                       const float *A, int64_t lda, const float *B, int64_t ldb,
                       float beta, float *C, int64_t ldc, void *stream);

/*
 * Variant id that sgemm() would run for (M, N, K) under the loaded set.
 * Fig. 1 leaves the online picker open and Sec. V-I names unseen inputs as
 * a limitation; the rule used here (ptune_dispatch): find the training
 * shapes nearest to (M, N, K) in L1 distance over (log2 M, log2 N, log2 K),
 * sizes below 1 counted as 1, and take the member whose log-slowdowns
 * summed over them is smallest (ties to the member listed first), each
 * log-slowdown moved from the training shape to (M, N, K) by the member's
 * wave correction: log E(training launch) - log E(launch at (M, N, K)),
 * with E(g) = g / (ceil(g / cus) * cus) for a launch of g work-groups
 * (tiles times K splits) on the current device's cus compute units.  A
 * training shape therefore always gets its own winner.  Returns the id
 * (>= 0), FF_ERR_NO_SET, FF_ERR_HIP if the device cannot be queried, or an
 * argument error for negative sizes.
 */
int variant_select(int64_t M, int64_t N, int64_t K);

/* variant_select() for the set loaded for precision form `form`. */
int variant_select_form(int form, int64_t M, int64_t N, int64_t K);

/* Text of the calling thread's most recent error ("" if none). */
const char *fewfit_last_error(void);

/* ---------------------------------------------------------------------
 * Tuning ABI: variant inspection, timing and screening (Sec. V-C)
 * ------------------------------------------------------------------- */

/*
 * Load every variant listed in <dir>/manifest.txt (one descriptor line per
 * variant, code object <dir>/<name>.co).  Returns the number of variants
 * loaded; FF_ERR_IO, FF_ERR_PARSE, FF_ERR_HIP.
 */
int variant_manifest_load(const char *dir);

/* Number of variants currently registered (manifest and set members). */
int variant_count(void);

/*
 * Write variant `id`'s descriptor into buf (NUL-terminated, truncated to
 * len): "<id> <name> <MWG> <NWG> <KWG> <MI> <WM> <WN> <SK> <VW> <LDS> <GM> <SG>
 * <PREC> <PD>", PREC the precision form (FF_FORM_*), PD the prefetch depth.
 * Returns the full length, or FF_ERR_VARIANT.
 */
int variant_info(int id, char *buf, size_t len);

/* sgemm() with an explicit variant instead of dispatch; same semantics. */
int sgemm_variant(int id, int64_t M, int64_t N, int64_t K, float alpha,
                  const float *A, int64_t lda, const float *B, int64_t ldb,
                  float beta, float *C, int64_t ldc, void *stream);

/*
 * Work-groups of the GEMM kernel launch that sgemm_variant() makes for
 * variant `id` on (M, N, K) on the current device: the tiles of C times the
 * split count of K over work-groups (as many splits as the variant's SG
 * allows, no more than there are K slabs, every split non-empty, and no
 * more M x N FP32 slices than fit the K-split workspace).  0 when M or N is
 * 0.  These counts feed the dispatch's wave correction (variant_select()).
 * Writes *groups; returns 0, FF_ERR_M/N/K, FF_ERR_VARIANT or FF_ERR_ARG.
 */
int variant_work_groups(int id, int64_t M, int64_t N, int64_t K, int64_t *groups);

/*
 * Time variant `id` with HIP events on `stream`: `warmup` untimed launches,
 * then `trials` trials of `reps` back-to-back launches each, bracketed by
 * two events.  Writes the mean milliseconds per launch of each trial to
 * trial_ms[0..trials).  C is overwritten (it is read as well when beta != 0).
 * Synchronises the stream.  Returns 0, an sgemm() error or FF_ERR_HIP.
 */
int sgemm_time(int id, int64_t M, int64_t N, int64_t K, float alpha,
               const float *A, int64_t lda, const float *B, int64_t ldb,
               float beta, float *C, int64_t ldc, void *stream,
               int warmup, int reps, int trials, float *trial_ms);

/*
 * Correctness screen (Sec. V-C: variants whose results do not match the
 * reference kernels are dropped).  screen_reference() runs a plain
 * one-thread-per-element GPU kernel that forms, in FP64,
 *   ref[i][j] = alpha * sum_k A[i][k] B[k][j] + beta * C0[i][j]
 *   tol[i][j] = 4*K*2^-24*|alpha|*sum_k |A[i][k]||B[k][j]|
 *               (+ 2*2^-24*(|alpha*sum_k A B| + |beta*C0|) if alpha != 1 or beta != 0)
 * into caller-owned device arrays ref and tol (M*N doubles each, dense
 * row-major).  screen_compare() counts the elements of C (row stride ldc)
 * with |C - ref| > tol_scale*tol or non-finite C, and writes the largest
 * |C - ref| / (tol_scale*tol) and, if err2/ref2 are not NULL, the sums of
 * (C - ref)^2 and ref^2 (normwise relative error = sqrt(err2/ref2)).
 * tol_scale > 1 widens the bound for the 16-bit precision forms.
 * Both synchronise the stream.  Returns 0, FF_ERR_ARG or FF_ERR_HIP.
 */
int screen_reference(int64_t M, int64_t N, int64_t K, float alpha,
                     const float *A, int64_t lda, const float *B, int64_t ldb,
                     float beta, const float *C0, int64_t ldc0,
                     double *ref, double *tol, void *stream);
int screen_compare(int64_t M, int64_t N, const float *C, int64_t ldc,
                   const double *ref, const double *tol, double tol_scale,
                   int64_t *nbad, double *max_ratio, double *err2, double *ref2,
                   void *stream);

/* ---------------------------------------------------------------------
 * Batches of independent GEMMs in one grouped persistent launch
 * ------------------------------------------------------------------- */

/* One problem of a batch: C = alpha*A*B + beta*C with the batch's alpha,
 * beta; device pointers; `tiles` is filled in by sgemm_grouped_plan(). */
typedef struct ff_gemm_desc {
    const float *A;
    const float *B;
    float *C;
    int64_t lda, ldb, ldc;
    int32_t M, N, K, tiles;
} ff_gemm_desc;

/*
 * Host-side plan of a grouped launch of FP32 variant `id` over `count`
 * problems (descs in host memory): checks every problem (sizes >= 1,
 * lda >= K, ldb >= N, ldc >= N, non-null matrices), writes each problem's
 * tile count and prefix[g] = tiles before problem g, and *vec_ok = 1 if
 * every problem allows the variant's vector loads.  Returns the total tile
 * count, FF_ERR_ARG, FF_ERR_VARIANT or FF_ERR_TOO_LARGE.  No HIP call.
 */
int sgemm_grouped_plan(int id, int count, ff_gemm_desc *descs, int32_t *prefix, int *vec_ok);

/*
 * One persistent launch of variant `id` over a planned batch: descs and
 * prefix are the plan's arrays copied to device memory; the grid holds as
 * many work-groups as fit on the device at once and each walks the batch's
 * tile list with a fixed stride.  vec != 0 selects the vector-load kernel
 * (only if the plan allowed it).  Allocates nothing and does not
 * synchronise, so it can be captured in a HIP graph.  Returns 0,
 * FF_ERR_ARG, FF_ERR_VARIANT or FF_ERR_HIP.
 */
int sgemm_grouped(int id, int count, const ff_gemm_desc *descs, const int32_t *prefix,
                  int total, float alpha, float beta, int vec, void *stream);

/* ---------------------------------------------------------------------
 * Portability tuning on an execution-time table (host only, Sec. IV, V-C)
 *
 * A table is a dense row-major nv x ns array of doubles: t[v*ns + s] is the
 * time of variant v on shape s; +inf marks a failed or missing entry.
 * ------------------------------------------------------------------- */

/*
 * Post-processing pass (Sec. V-C; Table VI columns): per shape the best and
 * worst finite time and the lowest variant index attaining the best
 * (-1 if none); per entry slowdown = t / best and speedup = worst / t
 * (inf and 0 for failed entries).  Output arrays: best, worst, best_id of
 * length ns; slowdown, speedup of length nv*ns (either may be NULL).
 */
int ptune_postprocess(int nv, int ns, const double *t, double *best, double *worst,
                      int *best_id, double *slowdown, double *speedup);

/*
 * Library cost function, Eq. 1 (Sec. IV-D-1), with the minimum runtime over
 * the selected set in the numerator: the geometric mean over the chosen
 * shapes of min_{v in kappa} t[v][s] / best[s], where best[s] is the minimum
 * over all nv variants.  `shapes` lists nsel shape indices (NULL: all).
 * Writes the cost (>= 1; +inf if some shape has no finite member) to *cost.
 */
int ptune_cost(int nv, int ns, const double *t, int k, const int *kappa,
               int nsel, const int *shapes, double *cost);

/*
 * PortabilityTune (Sec. IV-B, Sec. IV-C-1): a set of min(k, nv) variants
 * minimising ptune_cost over the chosen shapes.
 *   method 0: exhaustive over all subsets of the variants left after
 *             dominance pruning (exact);
 *   method 1: greedy construction followed by single-swap local search;
 *   method -1: exhaustive if at most 2e8 subsets remain, else method 1.
 * Writes the set (ascending ids) to kappa_out[0..min(k,nv)), the cost to
 * *cost_out and the number of subsets scored to *evals_out (any of the
 * last two may be NULL).  Returns the set size or FF_ERR_ARG.
 */
int ptune_select(int nv, int ns, const double *t, int nsel, const int *shapes,
                 int k, int method, int *kappa_out, double *cost_out, int64_t *evals_out);

/*
 * Fleet objective (Sec. IV-D-2, Eq. 2) on one device: the fleet's task rate
 * is quantity(d) / sum_i y'(i) quantity(i), so maximising it minimises the
 * weighted total time sum_j weights[j] * min_{v in kappa} t[v][shapes[j]]
 * of one task.  Same search as ptune_select (dominance pruning keeps it
 * exact: a dominated variant never lowers the sum); writes the set and the
 * total.  weights has nsel positive entries (shapes must not be NULL).
 */
int ptune_select_total(int nv, int ns, const double *t, int nsel, const int *shapes,
                       const double *weights, int k, int method, int *kappa_out,
                       double *total_out, int64_t *evals_out);

/*
 * k-means selection (Sec. IV-C-2): every selected shape is a point in
 * nv-dimensional space, its relative performance best/t per variant (0
 * where failed); Lloyd's algorithm from the k initial centroids
 * init[0..k) (positions among the selected shapes; the caller draws them):
 * assign points to the nearest centroid (lowest index on ties), move
 * centroids to their points' mean (an empty cluster keeps its centroid),
 * until no assignment changes or max_iter.  Each final centroid contributes
 * its best variant (largest component, lowest id on ties; a variant already
 * taken is replaced by the centroid's next best).  Writes the sorted set
 * (returns its size <= k), the cluster of each point and the iterations.
 */
int ptune_kmeans(int nv, int ns, const double *t, int nsel, const int *shapes, int k,
                 const int *init, int max_iter, int *kappa_out, int *assign_out, int *iters_out);

/*
 * Decision-tree selection (Sec. IV-C-3): a regression tree from the shapes'
 * features (nfeat per selected shape, row-major) to their relative
 * performance vectors, grown best first to k leaves (each step splits the
 * leaf whose best axis split lowers the summed squared error most;
 * thresholds halfway between consecutive distinct values; ties to the lower
 * leaf, feature and threshold).  Each leaf's mean vector contributes its best
 * variant as in ptune_kmeans.  Writes the sorted set (returns its size) and
 * each shape's leaf; when node_feat, node_thr and node_child are given
 * (2k - 1 entries, node_child 2 per node), the tree as ptune_tree_route
 * reads it, and when leaf_variant is given (k entries), each leaf's variant.
 */
int ptune_tree(int nv, int ns, const double *t, int nsel, const int *shapes, int nfeat,
               const double *features, int k, int *kappa_out, int *leaf_out,
               int *node_feat, double *node_thr, int *node_child, int *leaf_variant);

/*
 * The tree of Sec. IV-C-3 estimates the performance vector of any
 * environment, so it also routes an unseen input to a leaf: the leaf of
 * feature vector x[0..nfeat) in the tree ptune_tree wrote (node_feat,
 * node_thr, node_child over nnodes = 2 * leaves - 1 nodes; node 0 the root;
 * an internal node n sends x[node_feat[n]] <= node_thr[n] to node
 * node_child[2n], else to node_child[2n + 1]; a leaf node has node_feat -1
 * and its leaf index in node_child[2n]).  With ptune_tree's leaf_variant
 * (the variant each leaf contributed), an unseen input gets its leaf's
 * variant.  Returns the leaf index, or FF_ERR_ARG for a malformed tree.
 */
int ptune_tree_route(int nnodes, const int *node_feat, const double *node_thr,
                     const int *node_child, int nfeat, const double *x);

/*
 * For each of the nsel shapes, the member of kappa with the lowest time
 * (ties to the lower id; -1 if none is finite): the dispatch table that a
 * set file records for its training shapes.
 */
int ptune_assign(int nv, int ns, const double *t, int k, const int *kappa,
                 int nsel, const int *shapes, int *winners);

/*
 * Index of the first training shape (ntrain triples M,N,K in train_mnk)
 * nearest to (M, N, K) in L1 distance over log2 sizes (sizes below 1 count
 * as 1).  Returns the index, or FF_ERR_ARG.
 */
int ptune_nearest(int ntrain, const int64_t *train_mnk, int64_t M, int64_t N, int64_t K);

/*
 * The dispatch rule of variant_select() on explicit data: members[0..k) are
 * the set's variant ids, cost[i*k + j] = log(t[members[j]][i] / best[i])
 * on training shape i (+inf where member j failed there).  Among the
 * training shapes at the smallest distance (as in ptune_nearest, equal
 * within 1e-9), returns the member id with the smallest sum over them of
 * cost[i*k + j] + (log E(groups_train[i*k + j]) - log E(groups_query[j])),
 * ties to the lower j, where E(g) = g / (ceil(g / cus) * cus) (1 for
 * g <= 0) and groups_* are work-group counts of member j's launch on
 * training shape i and on (M, N, K).  With groups_train or groups_query
 * NULL, or cus < 1, the correction is 0.  If every member's sum is +inf,
 * the member cheapest on the first nearest shape.  Returns the id, or
 * FF_ERR_ARG.
 */
int ptune_dispatch(int ntrain, const int64_t *train_mnk, int k, const int *members,
                   const double *cost, const int64_t *groups_train,
                   const int64_t *groups_query, int cus, int64_t M, int64_t N,
                   int64_t K);

#ifdef __cplusplus
}
#endif

#endif /* FEWFIT_H */
