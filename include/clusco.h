/*
 * clusco.h - C ABI of the gfx950 (MI355X) cRMSD library.
 *
 * The operation is the coordinate RMSD after optimal superposition
 * (Algorithms, Eq. 1) evaluated without a rotation matrix or an SVD through
 * Eq. 2:
 *
 *     cRMSD(A,B) = sqrt(R_A^2 + R_B^2 - 2 (sqrt(l1) + sqrt(l2) + S sqrt(l3)))
 *
 * where R_A is the radius of gyration of model A, M = (1/L) sum_i a_i b_i^T is
 * the 3x3 covariance of the centred models, l1 >= l2 >= l3 are the
 * eigenvalues of M^T M (roots of its characteristic cubic) and S is the sign
 * of det M (Algorithms, the paragraph after Eq. 2).  Over an ensemble of N
 * models the library produces the N(N-1)/2 all-versus-all scores the paper
 * counts (Background) or the scores of many models against references
 * (Results and Discussion: comparison with a reference model).
 *
 * Conventions shared by every entry point
 *  - Coordinates: device memory, float32, [models][L][3] row-major, models
 *    back to back, 4-byte aligned.  Units are Angstrom in and out.  Every
 *    model of one call has the same L and atom i of one model corresponds to
 *    atom i of every other (Eq. 1).
 *  - Packed output: device float32 [N(N-1)/2]; the score of the pair (i, j),
 *    i < j, is at k(i,j) = i(2N-i-1)/2 + (j-i-1) (row-major upper triangle,
 *    diagonal omitted; the same order as SciPy's condensed distance vector).
 *  - Workspace: device memory owned by the caller, at least the size the
 *    matching *_workspace_size call returns, 256-byte aligned.  Its contents
 *    need no initialisation and are scratch after the call returns
 *    (the fix-up counter excepted, see clusco_fixup_count).
 *  - stream: a hipStream_t passed as void* (NULL = the default stream).  All
 *    work is enqueued asynchronously; no call synchronises the host, except
 *    clusco_fixup_count.  Kernel faults surface at the caller's next sync.
 *  - Errors: every entry point returns a status and never aborts.  Argument
 *    errors are detected on the host before anything is enqueued.  A failed
 *    launch returns CLUSCO_ERR_HIP (text via clusco_last_error).
 *  - Non-finite coordinates propagate to NaN scores; they are not detected.
 *  - A handle is not thread-safe; use one per host thread.
 */
#ifndef CLUSCO_H
#define CLUSCO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CLUSCO_OK = 0,
    CLUSCO_ERR_INVALID_ARG = 1, /* null pointer, negative size, L < 1, bad alignment */
    CLUSCO_ERR_WORKSPACE = 2,   /* workspace null or smaller than required */
    CLUSCO_ERR_UNSUPPORTED = 3, /* precision or size this build does not handle */
    CLUSCO_ERR_HIP = 4          /* a HIP runtime call or launch failed */
} clusco_status;

/* Arithmetic of the covariance contraction.  The cubic solve and the final
 * combine of Eq. 2 always run in FP64; so does the fix-up of pairs whose
 * contraction error could exceed the mode's tolerance.
 *   FP32        FP32 MFMA products, FP32 accumulation.    tolerance 1e-4 A
 *   SPLIT_BF16  centred coordinates split a = hi + lo in bfloat16, three
 *               products hi*hi' + hi*lo' + lo*hi' on MFMA, FP32 accumulation.
 *                                                          tolerance 5e-4 A
 *   SPLIT_FP16  the same split in float16 (|coordinate| < 65504 A).
 *                                                          tolerance 1e-4 A
 *   FP64        FP64 products and accumulation.           tolerance 1e-6 A
 *   SPLIT_BF16X4  the bfloat16 split with the fourth product lo*lo' as well
 *               (no dropped term; fewer pairs need the fix-up).
 *                                                          tolerance 5e-4 A */
typedef enum {
    CLUSCO_FP32 = 0,
    CLUSCO_SPLIT_BF16 = 1,
    CLUSCO_SPLIT_FP16 = 2,
    CLUSCO_FP64 = 3,
    CLUSCO_SPLIT_BF16X4 = 4
} clusco_precision;

typedef struct clusco_ctx *clusco_handle;

/* Create a handle bound to HIP device `device`.  Owns host state only (device
 * properties, tolerances, cached plans); allocates no device memory. */
clusco_status clusco_create(clusco_handle *h, int device);
void clusco_destroy(clusco_handle h);
const char *clusco_status_string(clusco_status s);
/* Text of the last failure on this handle ("" if none).  Owned by the handle. */
const char *clusco_last_error(clusco_handle h);

/* Absolute tolerance (A) that decides which pairs the FP64 fix-up recomputes
 * for precision p.  tol <= 0 disables the fix-up (raw contraction results,
 * for error studies).  Defaults are the tolerances listed above. */
clusco_status clusco_set_tolerance(clusco_handle h, clusco_precision p, double tol);

/* The error model behind the fix-up (derived from Eq. 2: an error d of the
 * correlation moves L cRMSD^2 by 2d).  For precision p and models of L atoms,
 * *eps is the relative contraction error the library assumes: with W_i the
 * squared size of what the MFMAs contracted for model i (sum of squared
 * residuals from the reference in the reference frame, else its radius
 * E_i = L R_i^2), the score s of a pair is trusted when
 *     (eps (W_i + W_j) + 2e-10 (E_i + E_j)) / (L s) <= tol / 2
 * (the second term bounds the FP64 epilogue's root finding) and recomputed
 * in FP64 otherwise.  eps grows with the FP32 accumulation steps (sqrt of
 * the padded length) and, for three-product SPLIT_BF16, includes the dropped
 * lo*lo' products (use SPLIT_BF16X4 for the four-product value); it is 0 for
 * FP64. */
clusco_status clusco_flag_epsilon(clusco_handle h, clusco_precision p, int64_t L, double *eps);

/* ------------------------------------------------------ kernel configuration
 *
 * How the covariance contraction of one problem runs (the arithmetic and the
 * result's tolerance do not change with it; results may differ within the
 * precision's tolerance between configurations).  The paper's workloads are
 * decoy sets of very uneven size (Results and Discussion: 56 I-TASSER targets
 * of 12,500 to 32,000 models, Table 1), so the configuration is chosen per
 * (precision, N bucket, L bucket) from a tuning table measured on the device
 * by paper_1302_4000_amd/tune.py:
 *   products  split-BF16 only: 3 MFMA products per K-block (hi*hi' + hi*lo' +
 *             lo*hi') or 4 (+ lo*lo').  Four products cost a third more MFMA
 *             issue but leave far fewer pairs for the FP64 fix-up; the table
 *             holds whichever made the whole call faster.  Other precisions
 *             report 3 (4 for SPLIT_BF16X4).
 *   schedule  CLUSCO_SCHED_STAGED: one 64x64 tile per 4-wave workgroup with
 *             operands staged in LDS; CLUSCO_SCHED_PERSISTENT: persistent
 *             8-wave workgroups alternating contraction and FP64 epilogue,
 *             operands straight from global memory (never with the frame).
 *             Backward and threshold calls always use the staged schedule; a
 *             batched call uses the one most of its work prefers, the
 *             persistent one only when no ensemble of the batch uses the frame
 *             (so each ensemble's scores equal those of a single call with
 *             the configuration the batch gives it, clusco_get_config_batched).
 *   band      tile rows per band of the tile order (L2 reuse of operands).
 *   frame     1: every model is first superimposed onto a reference structure
 *             (of the ensemble's first eight models, of set A's in a cross
 *             comparison, the one whose squared cRMSDs to the others sum to
 *             the least) by its optimal rotation, and the MFMA contraction
 *             runs on the residuals from the reference; the large per-model
 *             terms of the correlation are added back in FP64.  Rotating a
 *             model leaves its scores unchanged (Eq. 1), while the
 *             contraction error shrinks with the residuals' size, so far
 *             fewer pairs need the FP64 fix-up.  0: the centred models are
 *             contracted directly.  FP64 and the backward never use it.
 * Without a table entry the built-in default is products 3, staged, band 16,
 * frame 1.
 * A cross comparison of Na x Nb models takes the bucket of the all-vs-all
 * size with as many pairs.
 *
 * The table is loaded by clusco_create from $CLUSCO_TUNING when that variable
 * is set (an empty value: no table), else from tuning/<arch>.json in the
 * directory of the library (arch from the device, e.g. gfx950); a missing or
 * malformed file leaves the built-in defaults.  File format (JSON object):
 *   "arch": "gfx950", "n_edges": [...], "l_edges": [...]  ascending lower
 *   bucket bounds (bucket i: edges[i] <= x < edges[i+1], the last is open),
 *   "entries": [{"precision": "fp32" | "split_bf16" | "split_fp16" |
 *   "split_bf16x4", "n_bucket": i, "l_bucket": j, "products": 3 | 4,
 *   "schedule": "staged" | "persistent", "band": 1..256, optionally
 *   "frame": 0 | 1 (default 1) and "call": "single" | "batched" (default
 *   "single"), ...}]
 * (other keys are ignored).  A "batched" entry is what an ensemble of its
 * bucket takes inside a batched call, where the per-call costs (the reference
 * pass, launches) are shared by all ensembles and the best choice can differ
 * from a single call's; a bucket without one uses its single-call entry. */
#define CLUSCO_SCHED_STAGED 0
#define CLUSCO_SCHED_PERSISTENT 1

typedef struct {
    int32_t products; /* 3 or 4 (see above) */
    int32_t schedule; /* CLUSCO_SCHED_STAGED or CLUSCO_SCHED_PERSISTENT */
    int32_t band;     /* 1..256 */
    int32_t frame;    /* 1: contract residuals in the reference frame, 0: the models */
    int32_t source;   /* out: 0 built-in default, 1 tuning table, 2 forced */
    int32_t bucket;   /* out: n_bucket * len(l_edges) + l_bucket of the table entry, else -1 */
} clusco_config;

/* Replace the handle's tuning table with the file at `path` (NULL: drop the
 * table, back to the built-in default).  On error (CLUSCO_ERR_INVALID_ARG:
 * unreadable or malformed; CLUSCO_ERR_UNSUPPORTED: made for another
 * architecture) the table is unchanged.  Host only; no device work. */
clusco_status clusco_load_tuning(clusco_handle h, const char *path);
/* Path of the loaded table ("" if none).  Owned by the handle. */
const char *clusco_tuning_path(clusco_handle h);
/* The configuration calls with these sizes and precision will use. */
clusco_status clusco_get_config(clusco_handle h, int64_t N, int64_t L, clusco_precision p,
                                clusco_config *cfg);
/* The configuration an ensemble of these sizes takes inside a batched call
 * (clusco_crmsd_batched): the bucket's "batched" entry when the table has
 * one, else the same as clusco_get_config.  Host only; no device work. */
clusco_status clusco_get_config_batched(clusco_handle h, int64_t N, int64_t L,
                                        clusco_precision p, clusco_config *cfg);
/* Use `cfg` (products, schedule, band) for every later call on this handle,
 * whatever the table says; NULL returns to the table.  For measurement (the
 * tuner times each candidate this way). */
clusco_status clusco_force_config(clusco_handle h, const clusco_config *cfg);

/* ----------------------------------------------------------- all-vs-all */

/* Workspace bytes for clusco_crmsd_matrix with these sizes (0 if invalid). */
size_t clusco_crmsd_workspace_size(clusco_handle h, int64_t N, int64_t L, clusco_precision p);

/* All-vs-all cRMSD of N models of L atoms (Eq. 2 for every pair i < j).
 * coords: device float32 [N][L][3].  out: device float32 [N(N-1)/2], packed.
 * N in {0, 1} returns CLUSCO_OK with nothing enqueued.  L = 1 gives zeros. */
clusco_status clusco_crmsd_matrix(clusco_handle h, const float *coords, int64_t N, int64_t L,
                                  clusco_precision p, float *out, void *ws, size_t ws_bytes,
                                  void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and result as clusco_crmsd_matrix, with the workspace taken
 * from a built-in device scratch array of CLUSCO_SCRATCH_BYTES instead of a
 * caller buffer.  The caller still passes coords and out.  Each device the
 * library runs on holds its own copy of the scratch from the first
 * clusco_create on that device until the process ends.  Sizes whose
 * workspace (clusco_crmsd_workspace_size) exceeds CLUSCO_SCRATCH_BYTES
 * return CLUSCO_ERR_UNSUPPORTED before anything is enqueued (64 MiB holds
 * N = 20,000 at L = 150 in every precision).  The call allocates nothing and
 * never synchronises.  All calls on one device share that device's scratch
 * and it keeps the last call's contents: calls that overlap on one device
 * (different streams, or different handles on concurrent streams) race and
 * must be ordered by the caller.  The prep kernel of every call clears the
 * counters the later kernels rely on, so no clearing is needed between
 * calls. */
#define CLUSCO_SCRATCH_BYTES (64u << 20)
clusco_status clusco_crmsd_matrix_noalloc(clusco_handle h, const float *coords, int64_t N,
                                          int64_t L, clusco_precision p, float *out, void *stream);

/* Pairs within a cRMSD cutoff (Results and Discussion: selecting the pairs of
 * models below a threshold, 3.2 A in the paper's example) without storing the
 * N(N-1)/2 matrix.  Every pair (i, j), i < j, whose score (computed exactly as
 * by clusco_crmsd_matrix, fix-up included) is below `cutoff` is appended to
 * out_i / out_j / out_score (device int32, int32, float32 arrays of
 * `capacity` entries) in no particular order.  *count (device uint64,
 * 8-byte aligned) receives the number of such pairs; when it exceeds
 * capacity only `capacity` of them are stored (call again with larger
 * arrays).  Pairs whose score lies within the precision's tolerance of the
 * cutoff may fall on either side. */
size_t clusco_crmsd_threshold_workspace_size(clusco_handle h, int64_t N, int64_t L,
                                             clusco_precision p);
clusco_status clusco_crmsd_threshold(clusco_handle h, const float *coords, int64_t N, int64_t L,
                                     clusco_precision p, float cutoff, int32_t *out_i,
                                     int32_t *out_j, float *out_score, int64_t capacity,
                                     uint64_t *count, void *ws, size_t ws_bytes, void *stream);

/* Number of 32x32 pair blocks the last forward call on this workspace sent to
 * the FP64 fix-up.  Synchronises `stream`.  For diagnostics only. */
clusco_status clusco_fixup_count(clusco_handle h, const void *ws, int64_t *count, void *stream);

/* Stage timing for measurement.  With max_calls > 0, the next max_calls
 * forward calls (all-vs-all, batched, cross) on this handle record HIP events
 * on their stream around their three stages: prep, contraction + epilogue,
 * and fix-up; backward calls (all-vs-all, cross) around prep, the pairs pass
 * (contraction + adjoint records) and the gradient pass.  Creates
 * 4 * max_calls events once; 0 disables and frees them. */
clusco_status clusco_stage_timing(clusco_handle h, int max_calls);

/* Sum of the recorded stage durations (ms) over the calls recorded since
 * timing was enabled or last read: ms[0] prep, ms[1] contraction + epilogue
 * (backward: pairs pass), ms[2] fix-up (backward: gradient pass); *calls =
 * how many calls were recorded.  Synchronises on the
 * last recorded event and restarts the recording. */
clusco_status clusco_stage_times(clusco_handle h, double ms[3], int *calls);

/* ------------------------------------------------------------- batched */

/* Workspace bytes for a batched call over E ensembles with host arrays
 * h_N[E], h_L[E] (0 if invalid). */
size_t clusco_crmsd_batched_workspace_size(clusco_handle h, int32_t E, const int64_t *h_N,
                                           const int64_t *h_L, clusco_precision p);

/* E independent ensembles in one launch sequence: Eq. 2 over several decoy
 * sets of uneven size (Results and Discussion: the I-TASSER benchmark of 56
 * targets, each clustered on its own; Table 1).  Ensemble e has h_N[e]
 * models of h_L[e] atoms starting at float element h_coord_off[e] of coords,
 * and its packed output (h_N[e](h_N[e]-1)/2 scores) starts at float element
 * h_out_off[e] of out.  h_* are HOST arrays read during the call; the plan
 * built from them is cached in the handle, so repeated calls with the same
 * shapes enqueue without host-side planning; outside a graph capture the
 * plan's launches are themselves replayed from a cached hipGraph.  Under the
 * caller's own stream capture the call allocates nothing: it needs a plan
 * cached by an earlier call with the same shapes (else
 * CLUSCO_ERR_UNSUPPORTED), and such a plan stays alive until clusco_destroy
 * because the caller's graph holds its device table.  Ensembles may not
 * overlap in out.  Each ensemble takes its configuration from
 * clusco_get_config_batched. */
clusco_status clusco_crmsd_batched(clusco_handle h, int32_t E, const int64_t *h_N,
                                   const int64_t *h_L, const int64_t *h_coord_off,
                                   const int64_t *h_out_off, const float *coords,
                                   clusco_precision p, float *out, void *ws, size_t ws_bytes,
                                   void *stream);

/* ------------------------------------------------------- many-vs-reference */

/* Workspace bytes for clusco_crmsd_cross. */
size_t clusco_crmsd_cross_workspace_size(clusco_handle h, int64_t Na, int64_t Nb, int64_t L,
                                         clusco_precision p);

/* Dense cRMSD between two sets: out[ia*Nb + ib] = cRMSD(A_ia, B_ib).
 * A: device float32 [Na][L][3], B: device float32 [Nb][L][3], out: device
 * float32 [Na][Nb].  Nb = 1 is the comparison of every model with one
 * reference structure (Results and Discussion, the -e mode). */
clusco_status clusco_crmsd_cross(clusco_handle h, const float *A, int64_t Na, const float *B,
                                 int64_t Nb, int64_t L, clusco_precision p, float *out,
                                 void *ws, size_t ws_bytes, void *stream);

/* --------------------------------------------------------------- backward */

/* Workspace bytes for clusco_crmsd_backward. */
size_t clusco_crmsd_backward_workspace_size(clusco_handle h, int64_t N, int64_t L,
                                            clusco_precision p);

/* Gradient of sum_{i<j} grad_out[k(i,j)] * cRMSD_ij with respect to coords
 * (derived from Eq. 1/Eq. 2: d cRMSD / d a_l = (a_l - Q b_l) / (L cRMSD) with
 * Q = U diag(1,1,S) V^T for M = U diag(s) V^T, and the mirror formula for b).
 * rmsd: the packed scores of a forward call on the same coords (device).
 * grad_out: device float32 packed.  grad_coords: device float32 [N][L][3],
 * overwritten.  Pairs whose score is 0 contribute nothing. */
clusco_status clusco_crmsd_backward(clusco_handle h, const float *coords, int64_t N, int64_t L,
                                    const float *rmsd, const float *grad_out,
                                    clusco_precision p, float *grad_coords, void *ws,
                                    size_t ws_bytes, void *stream);

/* Workspace bytes for clusco_crmsd_cross_backward. */
size_t clusco_crmsd_cross_backward_workspace_size(clusco_handle h, int64_t Na, int64_t Nb,
                                                  int64_t L, clusco_precision p);

/* Gradient of sum grad_out[ia*Nb+ib] * cRMSD(A_ia, B_ib): grad_A [Na][L][3]
 * and grad_B [Nb][L][3] (device float32, overwritten; grad_B may be NULL).
 * rmsd: the dense scores of a clusco_crmsd_cross call on the same inputs. */
clusco_status clusco_crmsd_cross_backward(clusco_handle h, const float *A, int64_t Na,
                                          const float *B, int64_t Nb, int64_t L,
                                          const float *rmsd, const float *grad_out,
                                          clusco_precision p, float *grad_A, float *grad_B,
                                          void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- dRMSD */

/* Workspace bytes for clusco_drmsd_matrix (0 if invalid).  It grows as
 * N * L(L-1)/2 * 4 bytes (the operand vectors) for the MFMA precisions. */
size_t clusco_drmsd_workspace_size(clusco_handle h, int64_t N, int64_t L, clusco_precision p);

/* All-vs-all distance RMSD (Algorithms, Eq. 5): for every pair i < j,
 *     dRMSD(i, j) = sqrt( (2 / (L(L-1))) sum_{p<q} (|x^i_p - x^i_q| - |x^j_p - x^j_q|)^2 ),
 * the RMS difference of the two models' intra-model distance matrices.  No
 * superposition is involved and mirror images score zero.  Same layouts,
 * packed output order, workspace and stream rules as clusco_crmsd_matrix.
 * The FP32 / split precisions take the product of the distance-deviation
 * vectors on MFMA (FP32 accumulation) and recompute in FP64 the pairs whose
 * accumulation error could exceed the precision's tolerance; FP64 evaluates
 * the definition in FP64 for every pair (slow: O(N^2 L^2)).  N in {0, 1}
 * returns CLUSCO_OK with nothing enqueued; L = 1 gives zeros.
 * L above 4096 returns CLUSCO_ERR_UNSUPPORTED. */
clusco_status clusco_drmsd_matrix(clusco_handle h, const float *coords, int64_t N, int64_t L,
                                  clusco_precision p, float *out, void *ws, size_t ws_bytes,
                                  void *stream);

/* ------------------------------------------------------------------ CMO */

/* Workspace bytes for clusco_cmo_matrix (0 if invalid): about
 * N * L(L-1)/2 bytes of contact bits plus small tables. */
size_t clusco_cmo_workspace_size(clusco_handle h, int64_t N, int64_t L);

/* All-vs-all contact map overlap (Algorithms, Eq. 6-7).  Atoms p < q of a
 * model are in contact when their distance is below `cutoff` (A; the paper
 * does not state its value), decided on d^2 < cutoff^2 in FP64 from the
 * float32 coordinates; the score of a pair is the Sorensen index of the two
 * contact sets,
 *     S = 100 * 2 n(A and B) / (n(A) + n(B))    in [0, 100],
 * and 0 when neither model has a contact.  The counts are exact integers
 * (an int8 Gram product on MFMA); S is their quotient rounded once to
 * float32.  Higher is more similar.  Same layouts, packed output order,
 * workspace and stream rules as clusco_crmsd_matrix; no precision choice.
 * N in {0, 1} returns CLUSCO_OK with nothing enqueued; L = 1 gives zeros;
 * L above 4096 returns CLUSCO_ERR_UNSUPPORTED; a negative or non-finite
 * cutoff CLUSCO_ERR_INVALID_ARG. */
clusco_status clusco_cmo_matrix(clusco_handle h, const float *coords, int64_t N, int64_t L,
                                float cutoff, float *out, void *ws, size_t ws_bytes, void *stream);

/* ----------------------------------------------------------- clustering */

/* Workspace bytes for clusco_kmedoids (0 if invalid): 256 + 8 N rounded up
 * to a multiple of 256. */
size_t clusco_cluster_workspace_size(clusco_handle h, int64_t N, int32_t k);

/* K-means clustering of a packed score matrix (Implementation; Results and
 * Discussion: K-means over the all-vs-all matrix, k clusters, and the
 * representative chosen by the smallest <R>/f).  Only the N(N-1)/2 scores
 * are used, so every cluster centre is one of its members (a medoid).
 * Alternating steps from the caller's k distinct initial medoids:
 *   assign  every model joins the cluster of its nearest medoid (float32
 *           comparison; ties to the lowest cluster index; a medoid always
 *           joins its own cluster);
 *   update  each cluster's new medoid is the member with the smallest sum of
 *           scores to the other members (ties to the lowest model index);
 * until no medoid changes or max_iter updates have run (then one more
 * assignment).  Each score is rounded once to a multiple of 2^-20 and summed
 * exactly in 64-bit integers, so results do not depend on summation order.
 * Scores must be finite, non-negative and below 2^22.
 *   D       device float32 [N(N-1)/2], the packed matrix of any entry point
 *   h_init  HOST int32 [k], distinct model indices in [0, N); copied on the
 *           stream before the call returns
 *   labels  device int32 [N]: cluster of each model
 *   medoids device int32 [k]: final medoids
 *   sizes   device int64 [k]: n_c
 *   mean_r  device float64 [k]: <R>_c, the mean score over the n_c(n_c-1)/2
 *           pairs of cluster c (0 when n_c = 1)
 *   info    device int64 [3]: the representative cluster (smallest
 *           <R>_c N / n_c over clusters with n_c >= 2; ties to the lowest
 *           index; -1 if none), updates run, 1 if converged
 * The representative model is medoids[info[0]].
 * check_every = 0: all max_iter steps are enqueued on the stream and the call
 *   returns without synchronising (steps after convergence return at once
 *   on the device, at a few microseconds of launch cost each).
 * check_every > 0: after every check_every steps the call synchronises the
 *   stream, reads the convergence flag and stops enqueuing once converged
 *   (not usable under stream capture).
 * 1 <= k <= N <= 2^20, 0 <= max_iter <= 100000, check_every >= 0. */
clusco_status clusco_kmedoids(clusco_handle h, const float *D, int64_t N, int32_t k,
                              const int32_t *h_init, int32_t max_iter, int32_t check_every,
                              int32_t *labels, int32_t *medoids, int64_t *sizes, double *mean_r,
                              int64_t *info, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CLUSCO_H */
