// FP64 fix-up.  Pairs whose contraction error could exceed the tolerance are
// those with a small score relative to the models' radii: Eq. 2 subtracts
// 2(s1 + s2 + S s3) from R_A^2 + R_B^2, so an absolute error d in the
// correlation becomes an error of about d (E_A + E_B) / (L cRMSD) in cRMSD.
// The tile kernel lists every 32x32 block holding a pair whose stored score is
// below flag_coef (E_i + E_j); this kernel re-evaluates that test on the
// stored scores of each listed block, compacts the flagged pairs in LDS and
// recomputes each one from the raw float32 coordinates entirely in FP64
// (see pair_corr_span and pair_score), then the same Eq. 2 epilogue.  With `all` set (FP64 precision) every pair
// of every block is computed this way.  In threshold mode the candidates are
// the pairs the tile kernel marked in the block's ownership mask, and the
// recomputed pairs below the cutoff are appended to the output arrays.
#include "eq2.h"
#include "internal.h"

namespace clusco {

// Correlation of one pair entirely in FP64 from the raw float32 coordinates,
// H = sum_l x_l y_l^T (centred in pair_score), with the atoms split over
// FIX_SPAN lanes (lane sl takes atoms sl, sl + FIX_SPAN, ...: consecutive
// lanes read consecutive atoms) and the partial sums added by a fixed xor
// butterfly (reproducible); every lane of the group ends with the whole H.
constexpr int FIX_SPAN = 8;

__device__ __forceinline__ void pair_corr_span(const float *xi, const float *xj, int64_t L, int sl,
                                               double h[9])
{
#pragma unroll
    for (int u = 0; u < 9; ++u) h[u] = 0.0;
    for (int64_t l = sl; l < L; l += FIX_SPAN) {
        double a[3], b[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            a[u] = (double)xi[3 * l + u];
            b[u] = (double)xj[3 * l + u];
        }
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q) h[3 * p + q] = fma(a[p], b[q], h[3 * p + q]);
    }
#pragma unroll
    for (int off = FIX_SPAN / 2; off > 0; off >>= 1)
#pragma unroll
        for (int u = 0; u < 9; ++u) h[u] += __shfl_xor(h[u], off, FIX_SPAN);
}

// cRMSD from the uncentred correlation: H - L c_x c_y^T (the centred
// correlation; in FP64 the cancellation against translations of ~100 A costs
// about one digit) and the exact FP64 radii computed once per model by prep.
__device__ __forceinline__ float pair_score(double h[9], const double *ci, const double *cj,
                                            double ea, double eb, int64_t L)
{
    const double dl = (double)L;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) h[3 * p + q] = fma(-dl * ci[p], cj[q], h[3 * p + q]);
    const double lr2 = eq2_lrmsd2(h, ea, eb);
    return (float)sqrt(fmax(lr2 / dl, 0.0));
}

// One workgroup of FIX_THREADS per listed block at a time.
constexpr int FIX_THREADS = 256;

__global__ __launch_bounds__(FIX_THREADS) void fixup_kernel(FixupLaunch a)
{
    __shared__ uint16_t todo[ROWBLK * ROWBLK];
    __shared__ double hbuf[9][FIX_THREADS];
    __shared__ int cnt;
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t n = a.all ? a.n_all : (int64_t)a.counters[0];
    for (int64_t t = blockIdx.x; t < n; t += gridDim.x) {
        int e = 0;
        int64_t Ra, Rb;
        if (a.all) {
            if (a.table) e = table_find(a.table, a.nprob, t, [](const Problem &q) { return q.wtile0; });
        } else {
            e = (int)a.list[t].prob;
        }
        const Problem &p = a.table ? a.table[e] : a.prob;
        if (a.all) {
            const int64_t u = t - p.wtile0;
            if (p.sym) {
                tri_decode(u, p.nrbA, &Ra, &Rb);
            } else {
                Ra = u / p.nrbB;
                Rb = u - Ra * p.nrbB;
            }
        } else {
            const uint32_t b = a.list[t].blk;
            Ra = b >> 16;
            Rb = b & 0xFFFFu;
        }
        const int64_t NA = p.NA, NB = p.NB, L = p.L;
        const double *EA = (const double *)(a.ws + p.EA);
        const double *EB = (const double *)(a.ws + p.EB);
        float *out = a.out + p.out;
        if (tid == 0) cnt = 0;
        __syncthreads();
        for (int q = tid; q < ROWBLK * ROWBLK; q += FIX_THREADS) {
            const int64_t i = Ra * ROWBLK + (q >> 5), j = Rb * ROWBLK + (q & 31);
            const bool live = p.sym ? (i < j && j < NA) : (i < NA && j < NB);
            if (live) {
                bool need = true;
                if (a.all) {
                    need = true;
                } else if (a.thr) {
                    need = (a.emit.masks[32 * t + (q >> 5)] >> (q & 31)) & 1u;
                } else {
                    const int64_t k = p.sym ? packed_index(i, j, NA) : i * NB + j;
                    need = (double)out[k] < p.flag_coef * (EA[i] + EB[j]);
                }
                if (need) todo[atomicAdd(&cnt, 1)] = (uint16_t)q;
            }
        }
        __syncthreads();
        const int m = cnt;
        const float *XA = a.XA + p.XA, *XB = a.XB + p.XB;
        const double *cenA = (const double *)(a.ws + p.cenA);
        const double *cenB = (const double *)(a.ws + p.cenB);
        const double *E64A = (const double *)(a.ws + p.E64A);
        const double *E64B = (const double *)(a.ws + p.E64B);
        // per round of FIX_THREADS pairs: FIX_SPAN passes in which each
        // group of FIX_SPAN lanes computes one pair's correlation (all
        // groups at once) and parks it in LDS; then every thread finishes
        // one pair (one epilogue per pair, not one per lane of a group)
        const int grp = tid / FIX_SPAN, sl = tid % FIX_SPAN;
        for (int s0 = 0; s0 < m; s0 += FIX_THREADS) {   // uniform trip count (ballots below)
#pragma unroll 1
            for (int pass = 0; pass < FIX_SPAN; ++pass) {
                const int sp = s0 + pass * (FIX_THREADS / FIX_SPAN) + grp;
                if (sp < m) {     // uniform over each group of FIX_SPAN lanes
                    const int q = todo[sp];
                    const int64_t ip = Ra * ROWBLK + (q >> 5), jp = Rb * ROWBLK + (q & 31);
                    double h[9];
                    pair_corr_span(XA + ip * L * 3, XB + jp * L * 3, L, sl, h);
                    if (sl == 0) {
#pragma unroll
                        for (int u = 0; u < 9; ++u) hbuf[u][sp - s0] = h[u];
                    }
                }
            }
            __syncthreads();
            const int s = s0 + tid;
            int64_t i = 0, j = 0;
            float v = 0.0f;
            if (s < m) {
                const int q = todo[s];
                i = Ra * ROWBLK + (q >> 5);
                j = Rb * ROWBLK + (q & 31);
                double h[9];
#pragma unroll
                for (int u = 0; u < 9; ++u) h[u] = hbuf[u][tid];
                v = pair_score(h, cenA + 3 * i, cenB + 3 * j, E64A[i], E64B[j], L);
                if (!a.thr) out[p.sym ? packed_index(i, j, NA) : i * NB + j] = v;
            }
            __syncthreads();      // hbuf is rewritten by the next round
            if (a.thr) {
                const bool em = s < m && v < (float)a.emit.cutoff;
                const unsigned long long b = __ballot(em);
                if (b) {
                    unsigned long long base = 0;
                    if (lane == 0) base = atomicAdd(a.emit.count, (unsigned long long)__popcll(b));
                    base = __shfl(base, 0, 64);
                    if (em) {
                        const unsigned long long pos =
                            base + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
                        if (pos < (unsigned long long)a.emit.capacity) {
                            a.emit.i[pos] = (int32_t)i;
                            a.emit.j[pos] = (int32_t)j;
                            a.emit.score[pos] = v;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
}

hipError_t launch_fixup(const FixupLaunch &a, hipStream_t s)
{
    int64_t grid = a.all ? (a.n_all < 65536 ? a.n_all : 65536) : 4096;
    if (grid < 1) grid = 1;
    fixup_kernel<<<dim3((unsigned)grid), dim3(FIX_THREADS), 0, s>>>(a);
    return hipGetLastError();
}

} // namespace clusco
