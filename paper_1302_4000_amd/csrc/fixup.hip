// FP64 fix-up.  Pairs whose contraction error could exceed the tolerance are
// those with a small score relative to the size of what was contracted: Eq. 2
// subtracts 2(s1 + s2 + S s3) from R_A^2 + R_B^2, so an absolute error d in
// the correlation becomes an error of about d / (L cRMSD) in cRMSD, and d
// grows with the squared size of the contracted vectors (the models, or their
// residuals from the reference frame).  Prep folds that into one flag weight
// F per model; the tile kernel lists every 32x32 block holding a pair whose
// stored score is below F_i + F_j, and this kernel re-evaluates that test on the
// stored scores of each listed block, compacts the flagged pairs in LDS and
// recomputes each one from the raw float32 coordinates entirely in FP64
// (see pair_corr_span and pair_score), then the same Eq. 2 epilogue.  With
// `all` set (FP64 precision) every pair of every block is computed this way.
// Two kernels share the blocks: the dense kernel takes those with many pairs
// to recompute (staging the block's models in LDS), the sparse kernel the
// others.  In threshold mode the candidates are the pairs the tile kernel
// marked in the block's ownership mask, and the recomputed pairs below the
// cutoff are appended to the output arrays.
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

// Blocks with about FIX_DENSE or more pairs to recompute (estimated from a
// sample, see fixup_dense_kernel), and every block in `all` mode, go to the
// dense kernel: the block's 32 row and 32 column models are staged in LDS
// FIX_CHUNK atoms at a time, each model's chunk plane-major in FIX_STRIDE
// floats (odd, so that the 32 models of one side fall in distinct banks), and
// each thread accumulates one pair's correlation over the atoms in order from
// there.  A listed block the dense kernel took is marked (FIX_DONE in its
// problem word) and skipped by the sparse kernel, which runs after it.  A
// pair's value depends only on which kernel took its block, not on the order
// in which the block's pairs were compacted.
constexpr int FIX_CHUNK = 32;
constexpr int FIX_STRIDE = 3 * FIX_CHUNK + 1;
constexpr int FIX_DENSE = 96;
constexpr uint32_t FIX_DONE = 0x80000000u;
// The dense kernel's workgroup: FIX_DTHREADS threads, one pair each per round;
// its sample for the choice of kernel is every FIX_SAMPLE-th pair of a block.
constexpr int FIX_DTHREADS = 256;
constexpr int FIX_DWAVES = 3;
constexpr int FIX_SAMPLE = ROWBLK * ROWBLK / FIX_DTHREADS;
static_assert(2 * 3 * FIX_CHUNK <= FIX_DTHREADS, "one loader thread per float of two models");

// Word 3 of a raw (unswizzled, stride 0) buffer resource on gfx9: 32-bit data
// format, so out-of-range dword loads return zero.
constexpr int FIX_RSRC_WORD3 = 0x00020000;

// Buffer resource over [base, base + bytes): both are workgroup-uniform, made
// explicit so that the descriptor lives in scalar registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t side_rsrc(const float *base, int bytes)
{
    const uint64_t v = (uint64_t)base;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void *)(((uint64_t)hi << 32) | lo), (short)0,
                                             __builtin_amdgcn_readfirstlane(bytes), FIX_RSRC_WORD3);
}

// Accumulate atoms [0, cl) of one staged chunk into the pair's correlation
// (FULL: cl = FIX_CHUNK).
template <bool FULL>
__device__ __forceinline__ void chunk_corr(const float *xa, const float *xb, int cl, double h[9])
{
    const int n = FULL ? FIX_CHUNK : cl;
#pragma unroll 8
    for (int at = 0; at < n; ++at) {
        double va[3], vb[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            va[u] = (double)xa[u * FIX_CHUNK + at];
            vb[u] = (double)xb[u * FIX_CHUNK + at];
        }
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q) h[3 * p + q] = fma(va[p], vb[q], h[3 * p + q]);
    }
}

__global__ __launch_bounds__(FIX_THREADS) void fixup_kernel(FixupLaunch a)
{
    __shared__ uint16_t todo[ROWBLK * ROWBLK];
    __shared__ double hbuf[9][FIX_THREADS];
    __shared__ int cnt;
    const int tid = threadIdx.x, lane = tid & 63;
    if (a.all) return;                                // every block went to the dense kernel
    const int64_t n = (int64_t)a.counters[0];
    for (int64_t t = blockIdx.x; t < n; t += gridDim.x) {
        const uint32_t w = a.list[t].prob;
        if (w & FIX_DONE) continue;                   // taken by the dense kernel
        const Problem &p = a.table ? a.table[w] : a.prob;
        const uint32_t b = a.list[t].blk;
        const int64_t Ra = b >> 16, Rb = b & 0xFFFFu;
        const int64_t NA = p.NA, NB = p.NB, L = p.L;
        const double *FA = (const double *)(a.ws + p.FA);
        const double *FB = (const double *)(a.ws + p.FB);
        float *out = a.out + p.out;
        if (tid == 0) cnt = 0;
        __syncthreads();
        for (int q = tid; q < ROWBLK * ROWBLK; q += FIX_THREADS) {
            const int64_t i = Ra * ROWBLK + (q >> 5), j = Rb * ROWBLK + (q & 31);
            const bool live = p.sym ? (i < j && j < NA) : (i < NA && j < NB);
            if (live) {
                bool need;
                if (a.thr) {
                    need = (a.emit.masks[32 * t + (q >> 5)] >> (q & 31)) & 1u;
                } else {
                    const int64_t k = p.sym ? packed_index(i, j, NA) : i * NB + j;
                    need = flag_pair(out[k], (float)FA[i], (float)FB[j]);
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

__global__ __launch_bounds__(FIX_DTHREADS, FIX_DWAVES) void fixup_dense_kernel(FixupLaunch a)
{
    __shared__ uint16_t todo[ROWBLK * ROWBLK];
    __shared__ float xs[2 * ROWBLK * FIX_STRIDE];
    __shared__ int cnt;
    const int tid = threadIdx.x, lane = tid & 63;
    // staging: loader thread t (t < 2 x 3 FIX_CHUNK) holds float
    // t % (3 FIX_CHUNK) of the chunk of models t / (3 FIX_CHUNK), + 2, + 4,
    // ... (rows, then columns): a wave's loads are runs of consecutive floats
    // of one model.  Fetched into registers one chunk ahead of the products.
    const int lt = tid % (3 * FIX_CHUNK), lm = tid / (3 * FIX_CHUNK);
    const int lat = lt / 3, lu = lt - 3 * lat;
    const bool loader = tid < 2 * 3 * FIX_CHUNK;
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
        const double *FA = (const double *)(a.ws + p.FA);
        const double *FB = (const double *)(a.ws + p.FB);
        float *out = a.out + p.out;
        // which kernel takes a listed block: every block in `all` mode; in
        // threshold mode the count of candidates in the ownership mask; else
        // the count of flagged pairs among every fourth column (a sample, so
        // that blocks left to the sparse kernel cost a quarter of a scan)
        if (!a.all) {
            if (tid == 0) cnt = 0;
            __syncthreads();
            int c = 0;
            if (a.thr) {
                if (tid < ROWBLK) c = __popc(a.emit.masks[32 * t + tid]);
            } else {
                const int q = FIX_SAMPLE * tid;
                const int64_t i = Ra * ROWBLK + (q >> 5), j = Rb * ROWBLK + (q & 31);
                const bool live = p.sym ? (i < j && j < NA) : (i < NA && j < NB);
                if (live) {
                    const int64_t k = p.sym ? packed_index(i, j, NA) : i * NB + j;
                    c = flag_pair(out[k], (float)FA[i], (float)FB[j]) ? FIX_SAMPLE : 0;
                }
            }
            if (c) atomicAdd(&cnt, c);
            __syncthreads();
            const bool take = cnt >= FIX_DENSE;
            __syncthreads();                          // cnt is reset next
            if (!take) continue;
        }
        if (tid == 0) cnt = 0;
        __syncthreads();
        for (int q = tid; q < ROWBLK * ROWBLK; q += FIX_DTHREADS) {
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
                    need = flag_pair(out[k], (float)FA[i], (float)FB[j]);
                }
                if (need) todo[atomicAdd(&cnt, 1)] = (uint16_t)q;
            }
        }
        __syncthreads();
        const int m = cnt;
        if (!a.all && tid == 0) a.list[t].prob |= FIX_DONE;
        const float *XA = a.XA + p.XA, *XB = a.XB + p.XB;
        const double *cenA = (const double *)(a.ws + p.cenA);
        const double *cenB = (const double *)(a.ws + p.cenB);
        const double *E64A = (const double *)(a.ws + p.E64A);
        const double *E64B = (const double *)(a.ws + p.E64B);
        const int nA = (int)(NA - Ra * ROWBLK < ROWBLK ? NA - Ra * ROWBLK : ROWBLK);
        const int nB = (int)(NB - Rb * ROWBLK < ROWBLK ? NB - Rb * ROWBLK : ROWBLK);
        const int L3 = (int)(3 * L);
        // one buffer resource per side covering exactly its valid models:
        // reads past them (the last block row or column of a problem) return
        // zero, reads past the chunk's last atom land in the next model or
        // zero; neither slot is ever read
        const __amdgpu_buffer_rsrc_t rsA = side_rsrc(XA + Ra * ROWBLK * L * 3, nA * L3 * 4);
        const __amdgpu_buffer_rsrc_t rsB = side_rsrc(XB + Rb * ROWBLK * L * 3, nB * L3 * 4);
        float pre[ROWBLK];
        auto fetch = [&](int64_t c0) {
            if (!loader) return;
            const uint32_t v0 = 4u * (uint32_t)(lm * L3 + 3 * (int)c0 + lt), dk = 8u * (uint32_t)L3;
#pragma unroll
            for (int k = 0; k < ROWBLK / 2; ++k) {
                pre[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsA, (int)(v0 + k * dk), 0, 0));
                pre[ROWBLK / 2 + k] =
                    __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsB, (int)(v0 + k * dk), 0, 0));
            }
        };
        // per round of FIX_DTHREADS pairs each thread accumulates one pair's
        // correlation over the staged chunks, then finishes it
        for (int s0 = 0; s0 < m; s0 += FIX_DTHREADS) {   // uniform trip count (ballots below)
            const int s = s0 + tid;
            const int qs = s < m ? todo[s] : 0;
            const float *xa = xs + (qs >> 5) * FIX_STRIDE;
            const float *xb = xs + (ROWBLK + (qs & 31)) * FIX_STRIDE;
            double hc[9];
#pragma unroll
            for (int u = 0; u < 9; ++u) hc[u] = 0.0;
            fetch(0);
            for (int64_t c0 = 0; c0 < L; c0 += FIX_CHUNK) {
                const int cl = (int)(L - c0 < FIX_CHUNK ? L - c0 : FIX_CHUNK);
                __syncthreads();      // the previous chunk has been read
                if (loader) {         // into [model][plane][atom]
#pragma unroll
                    for (int k = 0; k < ROWBLK; ++k) xs[(lm + 2 * k) * FIX_STRIDE + lu * FIX_CHUNK + lat] = pre[k];
                }
                __syncthreads();
                if (c0 + FIX_CHUNK < L) fetch(c0 + FIX_CHUNK);
                if (s < m) {
                    if (cl == FIX_CHUNK) chunk_corr<true>(xa, xb, cl, hc);
                    else chunk_corr<false>(xa, xb, cl, hc);
                }
            }
            int64_t i = 0, j = 0;
            float v = 0.0f;
            if (s < m) {
                const int q = todo[s];
                i = Ra * ROWBLK + (q >> 5);
                j = Rb * ROWBLK + (q & 31);
                v = pair_score(hc, cenA + 3 * i, cenB + 3 * j, E64A[i], E64B[j], L);
                if (!a.thr) out[p.sym ? packed_index(i, j, NA) : i * NB + j] = v;
            }
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
    fixup_dense_kernel<<<dim3((unsigned)grid), dim3(FIX_DTHREADS), 0, s>>>(a);
    fixup_kernel<<<dim3((unsigned)grid), dim3(FIX_THREADS), 0, s>>>(a);
    return hipGetLastError();
}

} // namespace clusco
