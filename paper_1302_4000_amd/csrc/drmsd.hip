// All-vs-all dRMSD (Algorithms, Eq. 5) as a Gram matrix on MFMA.
//
// With d_m the vector of model m's K = L(L-1)/2 intra-model distances (atom
// pairs p < q), dRMSD(i, j)^2 = |d_i - d_j|^2 / K, and for any reference
// vector c, |d_i - d_j|^2 = E_i + E_j - 2 G_ij with e_m = d_m - c,
// E_m = |e_m|^2 and G_ij = e_i . e_j.  Taking c as the mean distance vector
// of a sample of the ensemble shrinks e_m from distances (tens of A) to
// deviations (a few A), so E_i + E_j - 2 G_ij cancels far less.
//
//  dist_ref     c[k] = mean of d_m[k] over the first nref models, in FP64,
//               and the atom-pair table
//  dist_prep    e_m rounded to the operand format in the fragment-native
//               layout of the cRMSD kernels (one plane), E_m from exactly
//               the operand values (FP64)
//  dist_tile    symmetric product on MFMA: a 128x128 tile per workgroup,
//               64x64 per wave (2x2 MFMA blocks), operands straight from
//               L2 (waves of a workgroup share rows and columns through L1);
//               epilogue sqrt(max(E_i + E_j - 2G, 0) / K), packed store, and
//               the fix-up flag as in the cRMSD path
//  dist_fixup   flagged pairs recomputed from the raw coordinates entirely in
//               FP64 (distances and their differences, no Gram identity)
#include "internal.h"

namespace clusco {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double dist64(const float *x, int p, int q)
{
    const double u = (double)x[3 * p] - (double)x[3 * q];
    const double v = (double)x[3 * p + 1] - (double)x[3 * q + 1];
    const double w = (double)x[3 * p + 2] - (double)x[3 * q + 2];
    return sqrt(u * u + v * v + w * w);
}

// Atom pair of distance index k (row-major over p < q), and the reference.
__global__ __launch_bounds__(256) void dist_ref_kernel(DistLaunch a)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.Kp) return;
    double *c = (double *)(a.ws + a.off_c);
    uint32_t *pq = (uint32_t *)(a.ws + a.off_pq);
    if (k >= a.K) {
        c[k] = 0.0;
        pq[k] = 0u;
        return;
    }
    int64_t p, q;
    tri_decode(k, a.L - 1, &p, &q);   // rows p, columns q - 1 of the strict triangle
    q += 1;
    pq[k] = (uint32_t)p | ((uint32_t)q << 16);
    double s = 0.0;
    for (int64_t m = 0; m < a.nref; ++m) s += dist64(a.X + m * a.L * 3, (int)p, (int)q);
    c[k] = s / (double)a.nref;
}

__device__ __forceinline__ double wave_sum64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint16_t bf16_rn(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// One wave per padded model: e_m = d_m - c into the operand layout.
template <int MODE>
__global__ __launch_bounds__(64) void dist_prep_kernel(DistLaunch a)
{
    const int64_t m = blockIdx.x;
    const int lane = threadIdx.x;
    if (m == 0 && lane < 2) a.counters[lane] = 0;
    const bool real = m < a.N;
    const float *x = a.X + (real ? m : 0) * a.L * 3;
    const double *c = (const double *)(a.ws + a.off_c);
    const uint32_t *pq = (const uint32_t *)(a.ws + a.off_pq);
    double *E = (double *)(a.ws + a.off_E);
    const int64_t R = m / ROWBLK;
    const int r = (int)(m % ROWBLK);
    double e = 0.0;
    for (int64_t k = lane; k < a.Kp; k += 64) {
        double v = 0.0;
        if (real && k < a.K) {
            const uint32_t t = pq[k];
            v = dist64(x, (int)(t & 0xFFFFu), (int)(t >> 16)) - c[k];
        }
        if constexpr (MODE == MODE_FP32) {
            const float f = (float)v;
            e += (double)f * (double)f;
            const int64_t kb = k >> 3, h = (k >> 2) & 1, el = k & 3;
            ((float *)(a.ws + a.off_ops))[((R * a.KB + kb) * 64 + r + 32 * h) * 4 + el] = f;
        } else {
            const int64_t kb = k >> 4, h = (k >> 3) & 1, el = k & 7;
            const int64_t base = ((R * a.KB + kb) * 2) * 64;
            uint16_t *ops = (uint16_t *)(a.ws + a.off_ops);
            double hv, lv;
            uint16_t hb, lb;
            if constexpr (is_bf16(MODE)) {
                hb = bf16_rn((float)v);
                hv = (double)__uint_as_float((uint32_t)hb << 16);
                lb = bf16_rn((float)(v - hv));
                lv = (double)__uint_as_float((uint32_t)lb << 16);
            } else {
                const _Float16 hh = (_Float16)(float)v;
                hv = (double)(float)hh;
                const _Float16 ll = (_Float16)(float)(v - hv);
                lv = (double)(float)ll;
                hb = __builtin_bit_cast(uint16_t, hh);
                lb = __builtin_bit_cast(uint16_t, ll);
            }
            ops[(base + r + 32 * h) * 8 + el] = hb;
            ops[(base + 64 + r + 32 * h) * 8 + el] = lb;
            const double sv = hv + lv;
            e += sv * sv;
        }
    }
    e = wave_sum64(e);
    if (lane == 0) E[m] = e;
}

template <int MODE>
__device__ __forceinline__ f32x16 mfma16(u32x4 x, u32x4 y, f32x16 c)
{
    if constexpr (is_bf16(MODE))
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, x),
                                                       __builtin_bit_cast(bf16x8, y), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, x),
                                                      __builtin_bit_cast(f16x8, y), c, 0, 0, 0);
}

__device__ __forceinline__ void pin() { asm volatile("" ::: "memory"); }

constexpr int DT = 128;   // models per workgroup tile edge (2x2 waves of 64)

template <int MODE>
__global__ __launch_bounds__(256, 2) void dist_tile_kernel(DistLaunch a)
{
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t per_xcd = gridDim.x >> 3;
    const int64_t t = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (t >= a.T) return;
    int64_t bi, bj;
    band_decode(t, a.nb, 4, &bi, &bj);
    const int wy = w >> 1, wx = w & 1;
    if (bi == bj && wy > wx) return;
    const int64_t R0 = 4 * bi + 2 * wy, C0 = 4 * bj + 2 * wx;   // 32-row blocks
    if (R0 * ROWBLK >= a.N || C0 * ROWBLK >= a.N) return;

    f32x16 acc[2][2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[s][u][r] = 0.0f;
    const int64_t KB = a.KB;
    if constexpr (MODE == MODE_FP32) {
        const f32x4 *ops = (const f32x4 *)(a.ws + a.off_ops);
        f32x4 A[2], B[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            A[s] = ops[((R0 + s) * KB) * 64 + lane];
            B[s] = ops[((C0 + s) * KB) * 64 + lane];
        }
        for (int64_t kb = 0; kb < KB; ++kb) {
            const int64_t nx = kb + 1 < KB ? kb + 1 : kb;
            f32x4 An[2], Bn[2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                An[s] = ops[((R0 + s) * KB + nx) * 64 + lane];
                Bn[s] = ops[((C0 + s) * KB + nx) * 64 + lane];
            }
            pin();
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int u = 0; u < 2; ++u)
                        acc[s][u] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[s][e], B[u][e],
                                                                        acc[s][u], 0, 0, 0);
            pin();
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                A[s] = An[s];
                B[s] = Bn[s];
            }
        }
    } else {
        // chunk (R, kb, part) at ((R*KB + kb)*2 + part) * 64 lanes
        const u32x4 *ops = (const u32x4 *)(a.ws + a.off_ops);
        u32x4 Ah[2], Al[2], Bh[2], Bl[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            Ah[s] = ops[(((R0 + s) * KB) * 2) * 64 + lane];
            Al[s] = ops[(((R0 + s) * KB) * 2 + 1) * 64 + lane];
            Bh[s] = ops[(((C0 + s) * KB) * 2) * 64 + lane];
            Bl[s] = ops[(((C0 + s) * KB) * 2 + 1) * 64 + lane];
        }
        for (int64_t kb = 0; kb < KB; ++kb) {
            const int64_t nx = kb + 1 < KB ? kb + 1 : kb;
            u32x4 Ahn[2], Aln[2], Bhn[2], Bln[2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                Ahn[s] = ops[(((R0 + s) * KB + nx) * 2) * 64 + lane];
                Aln[s] = ops[(((R0 + s) * KB + nx) * 2 + 1) * 64 + lane];
                Bhn[s] = ops[(((C0 + s) * KB + nx) * 2) * 64 + lane];
                Bln[s] = ops[(((C0 + s) * KB + nx) * 2 + 1) * 64 + lane];
            }
            pin();
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int u = 0; u < 2; ++u) acc[s][u] = mfma16<MODE>(Ah[s], Bh[u], acc[s][u]);
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int u = 0; u < 2; ++u) acc[s][u] = mfma16<MODE>(Ah[s], Bl[u], acc[s][u]);
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int u = 0; u < 2; ++u) acc[s][u] = mfma16<MODE>(Al[s], Bh[u], acc[s][u]);
            if constexpr (MODE == MODE_BF16X4) {
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int u = 0; u < 2; ++u) acc[s][u] = mfma16<MODE>(Al[s], Bl[u], acc[s][u]);
            }
            pin();
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                Ah[s] = Ahn[s];
                Al[s] = Aln[s];
                Bh[s] = Bhn[s];
                Bl[s] = Bln[s];
            }
        }
    }

    // epilogue: lane holds column j = lane%32, rows 8(r/4) + 4(lane/32) + r%4
    const double *E = (const double *)(a.ws + a.off_E);
    const int64_t N = a.N;
    const double invK = 1.0 / (double)a.K;
    bool flagged[2][2] = {{false, false}, {false, false}};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int64_t j = (C0 + u) * ROWBLK + (lane & 31);
        const double Ej = E[j];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int64_t i0 = (R0 + s) * ROWBLK + 8 * g + 4 * (lane >> 5);
                int64_t base = i0 * (2 * N - i0 - 1) / 2 - i0 - 1;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t i = i0 + q;
                    const double Ei = E[i];
                    const double r2 = fma(-2.0, (double)acc[s][u][4 * g + q], Ei + Ej) * invK;
                    const float v = sqrtf((float)fmax(r2, 0.0));
                    const bool live = i < j && j < N;
                    if (live) a.out[base + j] = v;
                    flagged[s][u] |= live && (double)v < a.flag_coef * (Ei + Ej);
                    base += N - i - 2;
                }
            }
        }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int u = 0; u < 2; ++u)
            if (__any(flagged[s][u]) && lane == 0) {
                const int k = atomicAdd(&a.counters[0], 1);
                a.list[k] = FixEntry{0u, ((uint32_t)(R0 + s) << 16) | (uint32_t)(C0 + u)};
            }
}

// FP64 recomputation of flagged pairs straight from the definition.
__global__ __launch_bounds__(256) void dist_fixup_kernel(DistLaunch a)
{
    __shared__ uint16_t todo[ROWBLK * ROWBLK];
    __shared__ int cnt;
    const int tid = threadIdx.x;
    const int64_t n = a.all ? tri_count(a.nrb) : a.counters[0];
    const double *E = (const double *)(a.ws + a.off_E);
    const uint32_t *pq = (const uint32_t *)(a.ws + a.off_pq);
    const int64_t N = a.N;
    for (int64_t t = blockIdx.x; t < n; t += gridDim.x) {
        int64_t Ra, Rb;
        if (a.all) {
            tri_decode(t, a.nrb, &Ra, &Rb);
        } else {
            const uint32_t blk = a.list[t].blk;
            Ra = blk >> 16;
            Rb = blk & 0xFFFFu;
        }
        if (tid == 0) cnt = 0;
        __syncthreads();
        for (int q = tid; q < ROWBLK * ROWBLK; q += 256) {
            const int64_t i = Ra * ROWBLK + (q >> 5), j = Rb * ROWBLK + (q & 31);
            if (i < j && j < N &&
                (a.all || (double)a.out[packed_index(i, j, N)] < a.flag_coef * (E[i] + E[j])))
                todo[atomicAdd(&cnt, 1)] = (uint16_t)q;
        }
        __syncthreads();
        const int m = cnt;
        for (int s = tid; s < m; s += 256) {
            const int q = todo[s];
            const int64_t i = Ra * ROWBLK + (q >> 5), j = Rb * ROWBLK + (q & 31);
            const float *xi = a.X + i * a.L * 3, *xj = a.X + j * a.L * 3;
            double acc = 0.0;
            for (int64_t k = 0; k < a.K; ++k) {
                const uint32_t u = pq[k];
                const int p = (int)(u & 0xFFFFu), r = (int)(u >> 16);
                const double d = dist64(xi, p, r) - dist64(xj, p, r);
                acc = fma(d, d, acc);
            }
            a.out[packed_index(i, j, N)] = (float)sqrt(acc / (double)a.K);
        }
        __syncthreads();
    }
}

hipError_t launch_dist_prep(int mode, const DistLaunch &a, hipStream_t s)
{
    dist_ref_kernel<<<dim3((unsigned)((a.Kp + 255) / 256)), dim3(256), 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || mode == MODE_FP64) return e;   // FP64: the fix-up does all
    const dim3 pg((unsigned)a.Np), pb(64);
    switch (mode) {
    case MODE_FP32: dist_prep_kernel<MODE_FP32><<<pg, pb, 0, s>>>(a); break;
    case MODE_FP16: dist_prep_kernel<MODE_FP16><<<pg, pb, 0, s>>>(a); break;
    case MODE_BF16:
    case MODE_BF16X4: dist_prep_kernel<MODE_BF16><<<pg, pb, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dist_tile(int mode, const DistLaunch &a, hipStream_t s)
{
    const dim3 tg((unsigned)round_up(a.T, 8)), tb(256);
    switch (mode) {
    case MODE_FP32: dist_tile_kernel<MODE_FP32><<<tg, tb, 0, s>>>(a); break;
    case MODE_BF16: dist_tile_kernel<MODE_BF16><<<tg, tb, 0, s>>>(a); break;
    case MODE_FP16: dist_tile_kernel<MODE_FP16><<<tg, tb, 0, s>>>(a); break;
    case MODE_BF16X4: dist_tile_kernel<MODE_BF16X4><<<tg, tb, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dist_fixup(const DistLaunch &a, hipStream_t s)
{
    dist_fixup_kernel<<<dim3(2048), dim3(256), 0, s>>>(a);
    return hipGetLastError();
}

} // namespace clusco
