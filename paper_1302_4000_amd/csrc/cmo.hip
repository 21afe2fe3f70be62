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
//  cmo_tile     256x256 pair tile per 8-wave workgroup, operand chunks staged
//               in LDS per K-block (double-buffered), 64x128 pairs per wave;
//               epilogue S in FP64 (one correctly rounded division), packed
//               float32 store.  Everything is exact up to that one rounding.
#include "internal.h"

namespace clusco {

typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void cmo_pin() { asm volatile("" ::: "memory"); }

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

__global__ __launch_bounds__(512, 1) void cmo_tile_kernel(CmoLaunch a)
{
    constexpr int NCH = 2 * CB;    // chunks per K-block: A then B
    constexpr int PER = NCH / 8;   // chunk loads per thread
    __shared__ i32x4 lds[2][NCH][64];

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
    const i32x4 *opl = ops + lane;
    i32x4 pre[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) pre[m] = opl[src[m]];
#pragma unroll
    for (int m = 0; m < PER; ++m) lds[0][w + 8 * m][lane] = pre[m];
    __syncthreads();

    i32x16 acc[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[s][u][r] = 0;

    for (int64_t kb = 0; kb < KB; ++kb) {
        const int buf = (int)(kb & 1);
        const bool more = kb + 1 < KB;
        if (more) {
#pragma unroll
            for (int m = 0; m < PER; ++m) pre[m] = opl[src[m] + (kb + 1) * 64];
        }
        cmo_pin();
        i32x4 A[2], B[4];
#pragma unroll
        for (int s = 0; s < 2; ++s) A[s] = lds[buf][2 * wy + s][lane];
#pragma unroll
        for (int u = 0; u < 4; ++u) B[u] = lds[buf][CB + 4 * wx + u][lane];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int u = 0; u < 4; ++u)
                acc[s][u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[s], B[u], acc[s][u], 0, 0, 0);
        if (more) {
#pragma unroll
            for (int m = 0; m < PER; ++m) lds[buf ^ 1][w + 8 * m][lane] = pre[m];
        }
        __syncthreads();
    }
    if (idle) return;

    // epilogue: lane holds column j = lane%32, rows 8(r/4) + 4(lane/32) + r%4
    const int *cnt = (const int *)(a.ws + a.off_n);
    const int64_t N = a.N;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t j = (bj * CB + 4 * wx + u) * ROWBLK + (lane & 31);
        const int nj = cnt[j];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int64_t R = bi * CB + 2 * wy + s;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int64_t i0 = R * ROWBLK + 8 * g + 4 * (lane >> 5);
                int64_t base = i0 * (2 * N - i0 - 1) / 2 - i0 - 1;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t i = i0 + q;
                    const int den = cnt[i] + nj;
                    const double sc = den > 0 ? (200.0 * (double)acc[s][u][4 * g + q]) / (double)den : 0.0;
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
