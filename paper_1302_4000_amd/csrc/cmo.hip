// All-vs-all contact map overlap (Algorithms, Eq. 6-7) as an integer Gram
// matrix on MFMA.
//
// A model's contact map over the atom pairs p < q is a 0/1 vector c_m of
// length K = L(L-1)/2 (contact: |x_p - x_q| < cutoff).  The Sorensen index of
// two maps needs n(A and B) = c_A . c_B and the counts n(A) = |c_A|, n(B):
//     S = 100 * 2 n(A and B) / (n(A) + n(B))   (0 when both counts are 0).
// The dot products of all pairs form the Gram matrix C C^T of 0/1 int8
// vectors, which v_mfma_i32_32x32x32_i8 computes exactly (int32
// accumulation; K < 2^31).
//
//  cmo_pairs    the atom pair (p, q) of every distance index k (row-major over
//               p < q), shared with nothing else
//  cmo_prep     one wave per model: contact bits as int8 in the fragment-native
//               chunk layout (K-blocks of 32) and the model's contact count.
//               Each contact is decided on d^2 = fma(u, u, fma(v, v, w w)) <
//               cutoff^2 in FP64 from the float32 coordinates
//  cmo_tile     256x256 pair tile per 8-wave workgroup, operand chunks
//               streamed into a 3-slot LDS ring, 64x128 pairs per wave;
//               epilogue S in FP64 (one correctly rounded division), packed
//               float32 store.  Everything is exact up to that one rounding.
#include "internal.h"

namespace clusco {

typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void cmo_pairs_kernel(CmoLaunch a)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.Kp) return;
    uint32_t *pq = (uint32_t *)(a.ws + a.off_pq);
    if (k >= a.K) {
        pq[k] = 0u;
        return;
    }
    int64_t p, q;
    tri_decode(k, a.L - 1, &p, &q);   // row p, column q - 1 of the strict triangle
    pq[k] = (uint32_t)p | ((uint32_t)(q + 1) << 16);
}

// One wave per padded model.  Lane l of chunk (R, kb) holds the 16 bytes of
// distance indices 32 kb + 16 (l / 32) + e, e = 0..15, of model 32 R + l % 32.
__global__ __launch_bounds__(64) void cmo_prep_kernel(CmoLaunch a)
{
    const int64_t m = blockIdx.x;
    const int lane = threadIdx.x;
    const bool real = m < a.N;
    const float *x = a.X + (real ? m : 0) * a.L * 3;
    const uint32_t *pq = (const uint32_t *)(a.ws + a.off_pq);
    int8_t *ops = (int8_t *)(a.ws + a.off_ops);
    const int64_t R = m / ROWBLK;
    const int r = (int)(m % ROWBLK);
    const double c2 = (double)a.cutoff * (double)a.cutoff;
    int cnt = 0;
    for (int64_t k = lane; k < a.Kp; k += 64) {
        int8_t bit = 0;
        if (real && k < a.K) {
            const uint32_t t = pq[k];
            const int p = (int)(t & 0xFFFFu), q = (int)(t >> 16);
            const double u = (double)x[3 * p] - (double)x[3 * q];
            const double v = (double)x[3 * p + 1] - (double)x[3 * q + 1];
            const double w = (double)x[3 * p + 2] - (double)x[3 * q + 2];
            bit = fma(u, u, fma(v, v, w * w)) < c2 ? 1 : 0;
        }
        cnt += bit;
        const int64_t kb = k >> 5, h = (k >> 4) & 1, e = k & 15;
        ops[((R * a.KB + kb) * 64 + r + 32 * h) * 16 + e] = bit;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if (lane == 0) ((int *)(a.ws + a.off_n))[m] = cnt;
}

constexpr int CT = 256;            // models per workgroup tile edge
constexpr int CB = CT / ROWBLK;    // 32-model blocks per tile edge

// s_waitcnt vmcnt(N) lgkmcnt(0) (expcnt left free), N <= 63.
template <int N>
__device__ __forceinline__ void cmo_wait_vm_lgkm()
{
    static_assert(N >= 0 && N < 64, "vmcnt field");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
}

// Operand chunks go straight from global memory into a 3-slot LDS ring
// (global_load_lds_dwordx4: load m of wave w moves chunk w + 8 m, lane l's
// 16 bytes landing at chunk base + 16 l), three K-blocks ahead, and each wave
// reads the next K-block's fragments into a second register set while the
// current K-block's products run.  Step s: loads of K-block s + 3 into the
// slot read at step s - 1, reads of slot s + 1, the products of K-block s,
// then a wait for the loads of K-block s + 2 only and a bare barrier.  The
// slots are separate LDS arrays in a loop unrolled by three, with the same
// number of loads in every step, so the compiler adds no waits of its own.
__global__ __launch_bounds__(512, 1) void cmo_tile_kernel(CmoLaunch a)
{
    constexpr int NCH = 2 * CB;    // chunks per K-block: A then B
    constexpr int PER = NCH / 8;   // chunk loads per wave
    __shared__ i32x4 slot0[NCH * 64], slot1[NCH * 64], slot2[NCH * 64];

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t per_xcd = gridDim.x >> 3;
    const int64_t t = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (t >= a.T) return;          // uniform over the workgroup
    int64_t bi, bj;
    band_decode(t, a.nb, 4, &bi, &bj);
    const int wy = w >> 1, wx = w & 1;
    const bool idle = bi == bj && 2 * wy >= 4 * wx + 4;   // wholly below the diagonal
    const int64_t KB = a.KB;
    const i32x4 *ops = (const i32x4 *)(a.ws + a.off_ops);
    int64_t src[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
        const int q = w + 8 * m;
        const int64_t R = (q < CB ? bi : bj) * CB + q % CB;
        src[m] = R * KB * 64;
    }
    // K-block kb into a slot; kb >= KB loads the first chunk of the operand
    // array (present, cached) into a slot nobody reads again
    auto dma = [&](int64_t kb, i32x4 *slot) {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const i32x4 *g = (kb < KB ? ops + src[m] + kb * 64 : ops) + lane;
            __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)g,
                                             (void __attribute__((address_space(3))) *)(slot + (w + 8 * m) * 64),
                                             16, 0, 0);
        }
    };
    struct Frag {
        i32x4 A[2], B[4];
    };
    auto read = [&](const i32x4 *slot, Frag &f) {
#pragma unroll
        for (int s = 0; s < 2; ++s) f.A[s] = slot[(2 * wy + s) * 64 + lane];
#pragma unroll
        for (int u = 0; u < 4; ++u) f.B[u] = slot[(CB + 4 * wx + u) * 64 + lane];
    };

    i32x16 acc[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[s][u][r] = 0;
    Frag cur;
    auto step = [&](int64_t s, i32x4 *sd, const i32x4 *sr) {
        dma(s + 3, sd);
        Frag nxt;
        read(sr, nxt);
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
            for (int u = 0; u < 4; ++u)
                acc[si][u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(cur.A[si], cur.B[u], acc[si][u], 0, 0, 0);
        // the loads of K-block s + 2 have landed (those of s + 3 stay in
        // flight) and this wave's reads of slot s + 1 are done before another
        // wave's loads may overwrite it
        __builtin_amdgcn_sched_barrier(0);
        cmo_wait_vm_lgkm<PER>();
        __builtin_amdgcn_s_barrier();
        cur = nxt;
    };

    dma(0, slot0);
    dma(1, slot1);
    dma(2, slot2);
    cmo_wait_vm_lgkm<PER>();       // K-blocks 0 and 1 have landed
    __builtin_amdgcn_s_barrier();
    read(slot0, cur);
    int64_t s = 0;
    for (; s + 3 <= KB; s += 3) {
        step(s, slot0, slot1);
        step(s + 1, slot1, slot2);
        step(s + 2, slot2, slot0);
    }
    if (s < KB) step(s, slot0, slot1);
    if (s + 1 < KB) step(s + 1, slot1, slot2);
    cmo_wait_vm_lgkm<0>();         // no load into LDS outlives the workgroup
    if (idle) return;

    // epilogue: lane holds column j = lane%32, rows 8(r/4) + 4(lane/32) + r%4;
    // contact counts of the wave's 64 rows (two per lane, shuffled to each
    // pair) and its lane's four columns, in one batch of loads
    const int *cnt = (const int *)(a.ws + a.off_n);
    const int64_t N = a.N;
    int nrow[2], ncol[4];
#pragma unroll
    for (int si = 0; si < 2; ++si) nrow[si] = cnt[(bi * CB + 2 * wy + si) * ROWBLK + (lane & 31)];
#pragma unroll
    for (int u = 0; u < 4; ++u) ncol[u] = cnt[(bj * CB + 4 * wx + u) * ROWBLK + (lane & 31)];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t j = (bj * CB + 4 * wx + u) * ROWBLK + (lane & 31);
        const int nj = ncol[u];
#pragma unroll
        for (int si = 0; si < 2; ++si) {
            const int64_t R = bi * CB + 2 * wy + si;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int64_t i0 = R * ROWBLK + 8 * g + 4 * (lane >> 5);
                int64_t base = i0 * (2 * N - i0 - 1) / 2 - i0 - 1;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t i = i0 + q;
                    const int den = __shfl(nrow[si], 8 * g + 4 * (lane >> 5) + q, 64) + nj;
                    const double sc = den > 0 ? (200.0 * (double)acc[si][u][4 * g + q]) / (double)den : 0.0;
                    if (i < j && j < N) a.out[base + j] = (float)sc;
                    base += N - i - 2;
                }
            }
        }
    }
}

hipError_t launch_cmo(const CmoLaunch &a, hipStream_t s)
{
    cmo_pairs_kernel<<<dim3((unsigned)((a.Kp + 255) / 256)), dim3(256), 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    cmo_prep_kernel<<<dim3((unsigned)a.Np), dim3(64), 0, s>>>(a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    cmo_tile_kernel<<<dim3((unsigned)round_up(a.T, 8)), dim3(512), 0, s>>>(a);
    return hipGetLastError();
}

} // namespace clusco
