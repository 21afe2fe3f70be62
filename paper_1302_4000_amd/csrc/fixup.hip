// FP64 fix-up.  Pairs whose contraction error could exceed the tolerance are
// those with a small score relative to the models' radii: Eq. 2 subtracts
// 2(s1 + s2 + S s3) from R_A^2 + R_B^2, so an absolute error d in the
// correlation becomes an error of about d (E_A + E_B) / (L cRMSD) in cRMSD.
// The tile kernel lists every 32x32 block holding a pair whose stored score is
// below flag_coef (E_i + E_j); this kernel re-evaluates that test on the
// stored scores of each listed block, compacts the flagged pairs in LDS and
// recomputes each one from the raw float32 coordinates entirely in FP64
// (centring with the FP64 centroids, H and both radii accumulated in FP64,
// then the same Eq. 2 epilogue).  With `all` set (FP64 precision) every pair
// of every block is computed this way.  In threshold mode the candidates are
// the pairs the tile kernel marked in the block's ownership mask, and the
// recomputed pairs below the cutoff are appended to the output arrays.
#include "eq2.h"
#include "internal.h"

namespace clusco {

__device__ __forceinline__ float pair_fp64(const float *xi, const float *xj, const double *ci,
                                           const double *cj, int64_t L)
{
    const double ci0 = ci[0], ci1 = ci[1], ci2 = ci[2];
    const double cj0 = cj[0], cj1 = cj[1], cj2 = cj[2];
    double h[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double ea = 0.0, eb = 0.0;
    for (int64_t l = 0; l < L; ++l) {
        const double a0 = (double)xi[3 * l] - ci0, a1 = (double)xi[3 * l + 1] - ci1,
                     a2 = (double)xi[3 * l + 2] - ci2;
        const double b0 = (double)xj[3 * l] - cj0, b1 = (double)xj[3 * l + 1] - cj1,
                     b2 = (double)xj[3 * l + 2] - cj2;
        h[0] += a0 * b0; h[1] += a0 * b1; h[2] += a0 * b2;
        h[3] += a1 * b0; h[4] += a1 * b1; h[5] += a1 * b2;
        h[6] += a2 * b0; h[7] += a2 * b1; h[8] += a2 * b2;
        ea += a0 * a0 + a1 * a1 + a2 * a2;
        eb += b0 * b0 + b1 * b1 + b2 * b2;
    }
    const double lr2 = eq2_lrmsd2(h, ea, eb);
    return (float)sqrt(fmax(lr2 / (double)L, 0.0));
}

__global__ __launch_bounds__(64) void fixup_kernel(FixupLaunch a)
{
    __shared__ uint16_t todo[ROWBLK * ROWBLK];
    __shared__ int cnt;
    const int lane = threadIdx.x;
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
        if (lane == 0) cnt = 0;
        __syncthreads();
        for (int q = lane; q < ROWBLK * ROWBLK; q += 64) {
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
        for (int s0 = 0; s0 < m; s0 += 64) {   // uniform trip count (ballots below)
            const int s = s0 + lane;
            int64_t i = 0, j = 0;
            float v = 0.0f;
            if (s < m) {
                const int q = todo[s];
                i = Ra * ROWBLK + (q >> 5);
                j = Rb * ROWBLK + (q & 31);
                v = pair_fp64(XA + i * L * 3, XB + j * L * 3, cenA + 3 * i, cenB + 3 * j, L);
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
    int64_t grid = a.all ? (a.n_all < 65536 ? a.n_all : 65536) : 2048;
    if (grid < 1) grid = 1;
    fixup_kernel<<<dim3((unsigned)grid), dim3(64), 0, s>>>(a);
    return hipGetLastError();
}

} // namespace clusco
