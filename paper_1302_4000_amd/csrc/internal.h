// Internal definitions shared by the gfx950 kernels and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/clusco.h"

namespace clusco {

// ---------------------------------------------------------------- layout
//
// The prep kernel writes centred coordinates in a fragment-native layout: for
// every block of 32 models (a "row block"), every K-block of atoms and every
// coordinate plane (x, y, z) there is one 1 KiB chunk holding exactly what the
// 64 lanes of a wave pass to one MFMA operand, lane-major.  A wave therefore
// loads an operand with one fully coalesced 16-byte-per-lane load, with no LDS
// staging and no swizzle in the contraction loop.  Both operands of the
// symmetric product Y Y^T use the same chunks.
//
//  FP32 (v_mfma_f32_32x32x2_f32, one value per lane per MFMA):
//      K-block = 8 atoms; lane l holds 4 floats = atoms 8kb + 4(l/32) + e,
//      e = 0..3, of model 32R + l%32.  Chunk index ((R*KB + kb)*3 + c).
//  SPLIT (v_mfma_f32_32x32x16_{bf16,f16}, 8 values per lane per MFMA):
//      K-block = 16 atoms; lane l holds 8 halves = atoms 16kb + 8(l/32) + e,
//      e = 0..7.  Chunk index (((R*KB + kb)*3 + c)*2 + part), part 0 = hi,
//      part 1 = lo.
//
// Rows are padded with zero models to a multiple of 64 (Np) and atoms with
// zeros to a multiple of the K-block (Lp).  Zero padding is exact because it
// is applied after centring and the scale 1/L uses the true L.

enum Mode { MODE_FP32 = 0, MODE_BF16 = 1, MODE_FP16 = 2, MODE_FP64 = 3, MODE_BF16X4 = 4 };
constexpr int NMODES = 5;

// split modes: hi/lo operand halves of bfloat16 (or float16) type
__host__ __device__ constexpr bool is_split(int mode)
{
    return mode == MODE_BF16 || mode == MODE_FP16 || mode == MODE_BF16X4;
}
__host__ __device__ constexpr bool is_bf16(int mode) { return mode == MODE_BF16 || mode == MODE_BF16X4; }

constexpr int ROWBLK = 32;   // models per MFMA row block
constexpr int TILE = 64;     // models per workgroup tile edge (2x2 waves)

__host__ __device__ constexpr int kblock(int mode) { return mode == MODE_FP32 ? 8 : 16; }

__host__ __device__ inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// packed upper-triangle index of (i, j), i < j
__host__ __device__ inline int64_t packed_index(int64_t i, int64_t j, int64_t N)
{
    return i * (2 * N - i - 1) / 2 + (j - i - 1);
}

// (row, column) of linear index t in the row-major upper triangle (diagonal
// included) of an nb x nb grid.
__host__ __device__ inline void tri_decode(int64_t t, int64_t nb, int64_t *bi, int64_t *bj)
{
    double B = 2.0 * (double)nb + 1.0;
    int64_t r = (int64_t)((B - sqrt(B * B - 8.0 * (double)t)) * 0.5);
    if (r < 0) r = 0;
    if (r > nb - 1) r = nb - 1;
    // start(r) = r*nb - r(r-1)/2
    while (r > 0 && r * nb - r * (r - 1) / 2 > t) --r;
    while (r + 1 < nb && (r + 1) * nb - (r + 1) * r / 2 <= t) ++r;
    *bi = r;
    *bj = r + (t - (r * nb - r * (r - 1) / 2));
}

__host__ __device__ inline int64_t tri_count(int64_t nb) { return nb * (nb + 1) / 2; }

// Banded order over the upper triangle of an nb x nb tile grid, for L2 reuse:
// bands of G tile rows, each swept column by column (rows inside a column),
// so consecutive tiles share a column of B and a band's rows of A stay
// resident.  A band first covers its own diagonal G x G triangle (column c
// holds rows 0..c), then every later column with all G rows.  Bijective onto
// {(bi, bj): 0 <= bi <= bj < nb}.
__host__ __device__ inline void band_decode(int64_t t, int64_t nb, int64_t G, int64_t *bi,
                                            int64_t *bj)
{
    int64_t r0 = 0;
    for (;;) {
        const int64_t g = nb - r0 < G ? nb - r0 : G;          // rows in this band
        const int64_t n = g * (g + 1) / 2 + g * (nb - r0 - g);
        if (t < n || r0 + g >= nb) {
            const int64_t d = g * (g + 1) / 2;
            if (t < d) {
                int64_t c = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
                while (c * (c + 1) / 2 > t) --c;
                while ((c + 1) * (c + 2) / 2 <= t) ++c;
                *bi = r0 + (t - c * (c + 1) / 2);
                *bj = r0 + c;
            } else {
                const int64_t u = t - d;
                *bi = r0 + u % g;
                *bj = r0 + g + u / g;
            }
            return;
        }
        t -= n;
        r0 += g;
    }
}

// Banded order over a full na x nb tile grid (bands of G rows, column-major).
__host__ __device__ inline void band_decode_rect(int64_t t, int64_t na, int64_t nb, int64_t G,
                                                 int64_t *bi, int64_t *bj)
{
    const int64_t band = t / (G * nb);
    const int64_t r0 = band * G;
    const int64_t g = na - r0 < G ? na - r0 : G;
    const int64_t u = t - band * G * nb;
    *bi = r0 + u % g;
    *bj = u / g;
}

__host__ inline size_t op_bytes_per_model(int mode, int64_t Lp)
{
    if (mode == MODE_FP32) return sizeof(float) * 3 * Lp;
    if (is_split(mode)) return 2 * 2 * 3 * Lp;
    return 0;
}

// ------------------------------------------------------------ problems
//
// A model set is a run of models of one length whose operands the prep pass
// writes.  A problem is one all-vs-all ensemble (A == B, packed output) or
// one cross comparison of two sets (dense Na x Nb output).  All offsets are
// relative to the bases passed at launch (coordinate arrays, workspace,
// output), so a table of sets or problems does not depend on the buffers.

// Reference frame.  With `frame` set, every model a of a set is first
// superimposed onto a reference structure r (a centred model of the
// problem's first set: of its first REF_CANDIDATES models the one with the
// smallest sum of squared cRMSD to the others, so that an outlier is not
// picked) by its optimal rotation R_a, and the contraction runs
// on the residuals d = R_a a - r instead of the coordinates.  For two models
// the correlation of the superimposed models is
//     H' = sum (r + d_A)(r + d_B)^T = G + P_A + P_B^T + D_AB,
//     G = sum r r^T,  P = sum d r^T,  D_AB = sum d_A d_B^T,
// and H' = R_A H R_B^T has the singular values and determinant sign of H, so
// Eq. 2 is unchanged.  Only D_AB (residuals of the size of the models'
// deviation from r, not of their radius of gyration) goes through the
// low-precision MFMA product; U = G + P and P^T are per-model FP64 terms the
// epilogue adds back.  Without `frame`, R = I and r = 0: U = P^T = 0 and
// d = a (the plain contraction).
struct ModelSet {
    int64_t X;            // float offset of the set's first coordinate
    int64_t N, Np, L, Lp, KB;
    int64_t model0;       // prefix of padded models over the launch
    int64_t ops;          // byte offset of the operand chunks in the workspace
    int64_t E;            // byte offset of the radii (double [Np])
    int64_t cen;          // byte offset of the centroids (double [Np][3])
    int64_t E64;          // byte offset of the exact FP64 radii of the raw coordinates
    int64_t U;            // byte offset of U = G + P (double [Np][9], row-major)
    int64_t PT;           // byte offset of P^T (double [Np][9])
    int64_t F;            // byte offset of the flag weights (double [Np], see Problem)
    int64_t ref_X;        // float offset of the reference candidates (models of L atoms)
    int64_t ref_N;        // models the candidates are taken from
    int64_t refinfo;      // byte offset of the candidates' moments (REF_INFO doubles)
    double fw, fe;        // flag weight F = fw W + fe E, W = sum |d|^2
    int32_t use_b;        // coordinates come from the second base pointer
    int32_t ref_b;        // the reference candidates come from the second base pointer
    int32_t frame;        // residuals from the reference frame (else R = I, r = 0)
    int32_t ref_own;      // this set's launch chooses the reference (else it shares one)
};

constexpr int REF_CANDIDATES = 8;
// Candidate moments of a set (doubles): L cRMSD^2 of every candidate pair,
// then each candidate's centroid (3) and G = sum r r^T (9).
constexpr int RI_PAIRS = REF_CANDIDATES * (REF_CANDIDATES - 1) / 2;
constexpr int RI_CEN = RI_PAIRS;
constexpr int RI_G = RI_CEN + 3 * REF_CANDIDATES;
constexpr int REF_INFO = RI_G + 9 * REF_CANDIDATES;

struct Problem {
    int64_t NA, NB, L, KB;
    int64_t nbA, nbB;     // 64-model tiles per side
    int64_t nrbA, nrbB;   // 32-model row blocks per side
    int64_t tile0;        // first 64x64 tile of this problem in the launch
    int64_t wtile0;       // first 32x32 block of this problem in the launch
    int64_t opsA, opsB, EA, EB, cenA, cenB;   // workspace byte offsets
    int64_t E64A, E64B;   // exact FP64 radii (fix-up)
    int64_t UA, PTB;      // reference-frame terms: U of the rows, P^T of the columns
    int64_t FA, FB;       // flag weights: a pair is recomputed when score < F_i + F_j
    int64_t XA, XB;       // float offsets into the first / second coordinate base
    int64_t out;          // float offset into the output base
    double flag_coef;     // > 0: the FP64 fix-up runs (flag weights in FA, FB); <= 0 never
    int32_t sym;          // 1: all-vs-all (packed, i < j); 0: dense NA x NB
    // kernel configuration chosen for this problem's (N, L) bucket
    int32_t x4;           // split-BF16: the fourth product lo*lo' is issued too
    int32_t band;         // tile rows per band of the tile order
    int32_t cfg;          // bucket of the tuning table the choice came from (-1: default)
    int32_t frame;        // the sets use the reference frame (epilogue adds U, P^T)
    int32_t pad2;
};

// Tile schedules (a tuning choice per problem bucket).
enum Schedule {
    SCHED_STAGED = 0,      // one 64x64 tile per 4-wave workgroup, operands staged in LDS
    SCHED_PERSISTENT = 1   // persistent 8-wave workgroups, contraction / epilogue ping-pong
                           // (operands from global memory, no reference frame)
};

// The fix-up flag of a pair: its score v is below F_i + F_j, the sum of the
// two models' flag weights, evaluated in FP32 (the weights rounded to float)
// by the tile epilogue and the fix-up's re-test alike, so that both take the
// same decision.  The weights bound the contraction error with a margin far
// above float rounding.
__device__ inline bool flag_pair(float v, float Fi, float Fj)
{
    return v < Fi + Fj;
}

__host__ __device__ inline int64_t problem_tiles(const Problem &p)
{
    return p.sym ? tri_count(p.nbA) : p.nbA * p.nbB;
}

__host__ __device__ inline int64_t problem_wtiles(const Problem &p)
{
    return p.sym ? tri_count(p.nrbA) : p.nrbA * p.nrbB;
}

// Fix-up list entry: problem index and the 32x32 block (row, column blocks).
struct FixEntry {
    uint32_t prob;
    uint32_t blk;         // (Ra << 16) | Rb
};

// Kernel launch descriptors.  Single problems travel inline; batched launches
// pass a device table (sorted by the host) plus its length.
struct PrepLaunch {
    const float *XA, *XB;
    char *ws;
    ModelSet set[2];      // inline sets (single / cross launches)
    const ModelSet *table;
    int32_t nset;
    int32_t mode;
    int64_t total;        // padded models over all sets
    int *counters;        // [0] fix-up list length, [1], [2] work counters (zeroed here)
    unsigned long long *zero64;   // zeroed here too when not null (emission count)
};

// Threshold emission: pairs (i, j), i < j, with score below `cutoff` are
// appended (in no particular order) to three arrays of `capacity` entries;
// *count receives how many there are (it may exceed capacity, in which case
// only the first `capacity` appended are stored).  Pairs the FP64 fix-up
// owns are marked in a per-block 32x32 bit mask instead and emitted there.
struct Emit {
    double cutoff;
    int32_t *i, *j;
    float *score;
    int64_t capacity;
    unsigned long long *count;
    uint32_t *masks;      // [list entry][32 rows] fix-up ownership bits
};

struct TileLaunch {
    char *ws;
    float *out;
    Problem prob;         // inline problem (single / cross launches)
    const Problem *table; // batched launches (prob unused)
    int32_t nprob;
    int32_t kind;         // TK_SYM, TK_RECT, TK_BATCH
    int64_t T;            // 64x64 tiles in the launch
    int32_t sched;        // SCHED_STAGED or SCHED_PERSISTENT (forward only)
    int32_t ctr;          // TK_BATCH persistent: index of its work counter in counters
    int64_t t0;           // TK_BATCH: first tile of this launch (tiles t0 .. t0 + T - 1)
    int *counters;
    FixEntry *list;
    // backward pass only: forward scores, incoming gradients, and the per-pair
    // record [w Q (9), w, 0, 0] written at 12 floats per output index
    const float *rmsd, *gout;
    float *wq;
    Emit emit;            // threshold pass only
};

enum TileKind { TK_SYM = 0, TK_RECT = 1, TK_BATCH = 2 };
enum TileOp { OP_FWD = 0, OP_BWD = 1, OP_THR = 2 };


// Gradient pass: for every model m of the row set, over all partners j,
//   grad_m = (sum_j w_mj) a_m - sum_j Q~_mj a_j
// with Q~ = Q of the record, or its transpose when m is the second model of
// the pair.
struct GradLaunch {
    const float *XR;          // raw coordinates of the row models
    const double *cenR;       // their centroids
    const float4 *P;          // centred partner coordinates, B fragment layout
    const float *wq;          // per-pair records
    float *grad;              // [NR][L][3]
    double *part;             // [nsplit][NR][L][3] partial G (nsplit > 1)
    double *wpart;            // [nsplit][NR] partial weight sums (nsplit > 1)
    int64_t NR, NC, L, Lp;
    int32_t kind;             // GK_SYM, GK_CROSS_A, GK_CROSS_B
    int32_t nsplit, bps;      // partner ranges and partner blocks per range
    int32_t pad;
};

struct GradSplit {
    int32_t nsplit, bps;
};

enum GradKind { GK_SYM = 0, GK_CROSS_A = 1, GK_CROSS_B = 2 };

struct FixupLaunch {
    const float *XA, *XB;
    const char *ws;
    float *out;
    Problem prob;
    const Problem *table;
    int32_t nprob;
    int32_t all;          // 1: recompute every pair of every block (FP64 precision)
    int64_t n_all;        // 32x32 blocks in the launch when all = 1
    const int *counters;
    FixEntry *list;       // the dense fix-up marks the entries it takes
    int32_t thr;          // 1: emit pairs below emit.cutoff instead of storing scores
    int32_t pad;
    Emit emit;
};

// All-vs-all dRMSD (Eq. 5) as a Gram matrix of distance-deviation vectors.
// Workspace regions (byte offsets): the reference distance vector c (double
// [Kp]), the atom pair of each distance index (uint32 p | q << 16, [Kp]), the
// radii E (double [Np]) and the operand chunks ([Np/32][KB][planes][64 lanes]
// as for one coordinate plane of the cRMSD layout).
struct DistLaunch {
    const float *X;       // raw coordinates [N][L][3]
    char *ws;
    float *out;           // packed [N(N-1)/2]
    int64_t N, Np, L;
    int64_t K, Kp, KB;    // distances per model, padded to the K-block, K-blocks
    int64_t nref;         // models averaged into the reference vector
    int64_t nb, T;        // 128-model tiles per side, tiles in the launch
    int64_t nrb;          // 32-model row blocks per side
    int64_t off_c, off_pq, off_E, off_ops;
    int *counters;        // [0] fix-up list length (zeroed by the prep pass)
    FixEntry *list;
    double flag_coef;     // flag a pair when score < flag_coef (E_i + E_j); <= 0 never
    int32_t all;          // 1: the fix-up recomputes every pair (FP64 precision)
    int32_t pad;
};

hipError_t launch_dist_prep(int mode, const DistLaunch &a, hipStream_t s);
hipError_t launch_dist_tile(int mode, const DistLaunch &a, hipStream_t s);
hipError_t launch_dist_fixup(const DistLaunch &a, hipStream_t s);

// All-vs-all contact map overlap (Eq. 6-7) as an integer Gram matrix.
// Workspace regions (byte offsets): the atom pair of each distance index
// (uint32 p | q << 16, [Kp]), the contact counts (int32 [Np]) and the int8
// contact bits ([Np/32][KB][64 lanes][16 bytes]).
struct CmoLaunch {
    const float *X;       // raw coordinates [N][L][3]
    char *ws;
    float *out;           // packed [N(N-1)/2]
    int64_t N, Np, L;
    int64_t K, Kp, KB;    // atom pairs, padded to the K-block of 32, K-blocks
    int64_t nb, T;        // 256-model tiles per side, tiles in the launch
    int64_t off_pq, off_n, off_ops;
    float cutoff;
    int32_t pad;
};

hipError_t launch_cmo(const CmoLaunch &a, hipStream_t s);

// Clustering of a packed score matrix (K-means with member centres).
struct ClusterLaunch {
    const float *D;       // packed scores [N(N-1)/2]
    int64_t N;
    int32_t k;
    int32_t pad;
    int32_t *medoid;      // [k], holds the initial medoids at launch
    int32_t *label;       // [N]
    long long *cost;      // [N] exact sums of rounded scores (workspace)
    int *state;           // [8] done, changed, iterations, converged, finished (workspace)
    long long *size;      // [k]
    double *mean_r;       // [k]
    long long *info;      // [3] representative cluster, iterations, converged
};

hipError_t launch_cluster_begin(const ClusterLaunch &a, hipStream_t s);
hipError_t launch_cluster_iters(const ClusterLaunch &a, int iters, hipStream_t s);
hipError_t launch_cluster_end(const ClusterLaunch &a, hipStream_t s);

// Workspace of one launch: counters, then per-set regions, then the list.
struct WsLayout {
    size_t total;
    size_t off_counters;  // 256 bytes
    size_t off_list;      // FixEntry [max_blocks]
    int64_t max_blocks;
};

hipError_t launch_prep(const PrepLaunch &a, hipStream_t s);   // also chooses the references
hipError_t launch_tile(int mode, const TileLaunch &a, hipStream_t s, int op = OP_FWD);
hipError_t launch_grad(const GradLaunch &a, hipStream_t s);
hipError_t launch_grad_planes(const float *X, const double *cen, float *P, int64_t N, int64_t L,
                              hipStream_t s);
int64_t grad_partners_padded(int64_t n);
GradSplit grad_split(int64_t NR, int64_t NC, int64_t L);
size_t grad_partial_bytes(int64_t NR, int64_t NC, int64_t L);
int64_t grad_atoms_padded(int64_t L);
hipError_t launch_zero(float *p, int64_t n, hipStream_t s);
hipError_t launch_fixup(const FixupLaunch &a, hipStream_t s);

// Device-side lookup of the entry of a prefix-sorted table holding index t.
template <typename T, typename F>
__device__ __forceinline__ int table_find(const T *tab, int n, int64_t t, F start)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start(tab[mid]) <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

} // namespace clusco
