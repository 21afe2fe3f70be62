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
//  dist_tile    symmetric product on MFMA: a 256x256 tile per 8-wave
//               workgroup with the operand chunks staged in LDS per K-block
//               (double-buffered), 64x128 pairs per wave; epilogue
//               sqrt(max(E_i + E_j - 2G, 0) / K), packed store, and the
//               fix-up flag as in the cRMSD path
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

// e_m = d_m - c into the operand layout, one workgroup of PREP_T threads per
// row block of 32 padded models.  Thread (slot, kq) builds the 16 bytes of
// lane slot = r + 32 h of K-block kb = PREP_G i + kq (every i): the EL consecutive
// distance indices kb*KBW + EL h + el of model r, rounded to the operand
// format (FP32; or hi and lo halves in bf16 / fp16, both chunks), so each
// wave writes whole 1 KiB chunks.  E_m is summed from the same rounded
// values per thread, then over the model's 2 PREP_G threads in a fixed order.
constexpr int PREP_T = 1024;
constexpr int PREP_G = PREP_T / 64;   // K-block groups per workgroup

// Models of up to PREP_LDS_L atoms: the row block's 32 models are staged in
// LDS first (coalesced), so the six coordinates of each distance come from
// LDS instead of scattered cached global loads.
constexpr int PREP_LDS_L = 160;

template <int MODE, bool XL>
__global__ __launch_bounds__(PREP_T) void dist_prep_kernel(DistLaunch a)
{
    constexpr int KBW = MODE == MODE_FP32 ? 8 : 16;   // K-block width
    constexpr int EL = KBW / 2;                       // elements per lane slot
    __shared__ double red[PREP_T];
    __shared__ float xs[XL ? ROWBLK * PREP_LDS_L * 3 : 1];
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid < 2) a.counters[tid] = 0;
    const int64_t R = blockIdx.x;
    const int slot = tid & 63, kq = tid >> 6;
    const int r = slot & 31, h = slot >> 5;
    const int64_t m = R * ROWBLK + r;
    const bool real = m < a.N;
    const float *x;
    if constexpr (XL) {
        // the row block's models are contiguous: [R*32, R*32 + nr) x L x 3
        const int64_t nr = a.N - R * ROWBLK < ROWBLK ? a.N - R * ROWBLK : ROWBLK;
        const int64_t nf = (nr > 0 ? nr : 0) * a.L * 3;
        const float *src = a.X + R * ROWBLK * a.L * 3;
        for (int64_t f = tid; f < nf; f += PREP_T) xs[f] = src[f];
        __syncthreads();
        x = xs + (real ? r : 0) * a.L * 3;
    } else {
        x = a.X + (real ? m : 0) * a.L * 3;
    }
    const double *c = (const double *)(a.ws + a.off_c);
    const uint32_t *pq = (const uint32_t *)(a.ws + a.off_pq);
    double e = 0.0;
    for (int64_t kb = kq; kb < a.KB; kb += PREP_G) {
        const int64_t k0 = kb * KBW + EL * h;
        double v[EL];
#pragma unroll
        for (int el = 0; el < EL; ++el) {
            const int64_t k = k0 + el;
            v[el] = 0.0;
            if (real && k < a.K) {
                const uint32_t t = pq[k];
                v[el] = dist64(x, (int)(t & 0xFFFFu), (int)(t >> 16)) - c[k];
            }
        }
        if constexpr (MODE == MODE_FP32) {
            f32x4 f;
#pragma unroll
            for (int el = 0; el < EL; ++el) {
                f[el] = (float)v[el];
                e += (double)f[el] * (double)f[el];
            }
            ((f32x4 *)(a.ws + a.off_ops))[(R * a.KB + kb) * 64 + slot] = f;
        } else {
            uint16_t hb[EL], lb[EL];
#pragma unroll
            for (int el = 0; el < EL; ++el) {
                double hv, lv;
                if constexpr (is_bf16(MODE)) {
                    hb[el] = bf16_rn((float)v[el]);
                    hv = (double)__uint_as_float((uint32_t)hb[el] << 16);
                    lb[el] = bf16_rn((float)(v[el] - hv));
                    lv = (double)__uint_as_float((uint32_t)lb[el] << 16);
                } else {
                    const _Float16 hh = (_Float16)(float)v[el];
                    hv = (double)(float)hh;
                    const _Float16 ll = (_Float16)(float)(v[el] - hv);
                    lv = (double)(float)ll;
                    hb[el] = __builtin_bit_cast(uint16_t, hh);
                    lb[el] = __builtin_bit_cast(uint16_t, ll);
                }
                const double sv = hv + lv;
                e += sv * sv;
            }
            u32x4 hw, lw;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                hw[q] = (uint32_t)hb[2 * q] | ((uint32_t)hb[2 * q + 1] << 16);
                lw[q] = (uint32_t)lb[2 * q] | ((uint32_t)lb[2 * q + 1] << 16);
            }
            u32x4 *ops = (u32x4 *)(a.ws + a.off_ops) + (R * a.KB + kb) * 2 * 64;
            ops[slot] = hw;
            ops[64 + slot] = lw;
        }
    }
    red[tid] = e;
    __syncthreads();
    if (tid < ROWBLK) {
        double sum = 0.0;
        for (int q = 0; q < 2 * PREP_G; ++q) sum += red[tid + 32 * q];   // h = q & 1, kq = q >> 1
        ((double *)(a.ws + a.off_E))[R * ROWBLK + tid] = sum;
    }
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

// s_waitcnt vmcnt(N) lgkmcnt(0) (expcnt left free), N <= 63.
template <int N>
__device__ __forceinline__ void dist_wait_vm_lgkm()
{
    static_assert(N >= 0 && N < 64, "vmcnt field");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
}

constexpr int GT = 256;            // models per workgroup tile edge
constexpr int GB = GT / ROWBLK;    // 32-model blocks per tile edge

// One 256x256 pair tile per 8-wave workgroup; each wave multiplies 2 row
// blocks by 4 column blocks (64 x 128 pairs, eight 32x32 accumulators).  Per
// K-block the workgroup's operand chunks (its 8 row blocks and 8 column
// blocks) go straight from global memory into a 3-slot LDS ring
// (global_load_lds_dwordx4: load m of wave w moves chunk w + 8 m, lane l's 16
// bytes landing at chunk base + 16 l), issued three K-blocks ahead; every
// chunk reaches the CU once per K-block instead of once per wave that uses
// it.  A wave reads the next K-block's fragments from LDS into a second
// register set while the current K-block's MFMAs run.  Step s: loads of
// K-block s + 3 into the slot read at step s - 1, reads of slot s + 1, the
// MFMAs of K-block s, then a wait for the loads of K-block s + 2 only and a
// bare barrier.  The slots are separate LDS arrays used in a loop unrolled
// by three (slot fixed per step) with the same number of loads in every
// step, so the compiler adds no waits of its own.
template <int MODE>
__global__ __launch_bounds__(512, 1) void dist_tile_kernel(DistLaunch a)
{
    constexpr int P = is_split(MODE) ? 2 : 1;      // chunk parts (hi, lo)
    constexpr int NCH = 2 * GB * P;                // chunks per K-block, A then B
    constexpr int PER = NCH / 8;                   // chunk loads per wave
    __shared__ u32x4 slot0[NCH * 64], slot1[NCH * 64], slot2[NCH * 64];

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index, in scalars
    const int64_t per_xcd = gridDim.x >> 3;
    const int64_t t = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (t >= a.T) return;                          // uniform over the workgroup
    int64_t bi, bj;
    band_decode(t, a.nb, 4, &bi, &bj);
    const int wy = w >> 1, wx = w & 1;
    // on a diagonal tile, waves wholly below the diagonal multiply too (the
    // workgroup waits for its slowest wave anyway) but store nothing
    const bool idle = bi == bj && 2 * wy >= 4 * wx + 4;
    const int64_t KB = a.KB;
    const u32x4 *ops = (const u32x4 *)(a.ws + a.off_ops);
    int64_t src[PER];                              // wave's chunk bases (K-block 0)
#pragma unroll
    for (int m = 0; m < PER; ++m) {
        const int q = w + 8 * m;
        const int side = q / (GB * P), r = q % (GB * P);
        const int64_t R = (side ? bj : bi) * GB + r / P;
        src[m] = (R * KB * P + r % P) * 64;
    }
    // K-block kb into a slot; kb >= KB loads the first chunks of the operand
    // array (present, cached) into a slot nobody reads again
    auto dma = [&](int64_t kb, u32x4 *slot) {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const u32x4 *g = (kb < KB ? ops + src[m] + kb * P * 64 : ops) + lane;
            __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)g,
                                             (void __attribute__((address_space(3))) *)(slot + (w + 8 * m) * 64),
                                             16, 0, 0);
        }
    };
    struct Frag {
        u32x4 a[2 * P], b[4 * P];
    };
    auto read = [&](const u32x4 *slot, Frag &f) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int h = 0; h < P; ++h) f.a[s * P + h] = slot[((2 * wy + s) * P + h) * 64 + lane];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int h = 0; h < P; ++h) f.b[u * P + h] = slot[(GB * P + (4 * wx + u) * P + h) * 64 + lane];
    };

    f32x16 acc[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[s][u][r] = 0.0f;
    auto mma = [&](const Frag &f) {
        if constexpr (MODE == MODE_FP32) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        acc[s][u] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                            __builtin_bit_cast(f32x4, f.a[s])[e], __builtin_bit_cast(f32x4, f.b[u])[e],
                            acc[s][u], 0, 0, 0);
        } else {
            // hi*hi', hi*lo', lo*hi' (lo*lo' in x4 mode)
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[s][u] = mfma16<MODE>(f.a[2 * s], f.b[2 * u], acc[s][u]);
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[s][u] = mfma16<MODE>(f.a[2 * s], f.b[2 * u + 1], acc[s][u]);
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[s][u] = mfma16<MODE>(f.a[2 * s + 1], f.b[2 * u], acc[s][u]);
            if constexpr (MODE == MODE_BF16X4) {
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        acc[s][u] = mfma16<MODE>(f.a[2 * s + 1], f.b[2 * u + 1], acc[s][u]);
            }
        }
    };
    // one step: cur holds K-block s (read at the previous step) and gets
    // K-block s + 1 at the end; sd is the slot of K-block s (free: read last
    // step), sr the slot of K-block s + 1
    Frag cur;
    auto step = [&](int64_t s, u32x4 *sd, const u32x4 *sr) {
        dma(s + 3, sd);
        Frag nxt;
        read(sr, nxt);
        mma(cur);
        // both barriers' work: the loads of K-block s + 2 have landed (those
        // of s + 3 stay in flight) and this wave's reads of slot s + 1 are
        // done before another wave's loads may overwrite it
        __builtin_amdgcn_sched_barrier(0);
        dist_wait_vm_lgkm<PER>();
        __builtin_amdgcn_s_barrier();
        cur = nxt;
    };

    dma(0, slot0);
    dma(1, slot1);
    dma(2, slot2);
    dist_wait_vm_lgkm<PER>();          // K-blocks 0 and 1 have landed
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
    dist_wait_vm_lgkm<0>();            // no load into LDS outlives the workgroup

    // the epilogue's radii: E of the wave's 64 rows (two per lane, shuffled
    // to each pair) and of its lane's four columns, in one batch of loads
    const double *E = (const double *)(a.ws + a.off_E);
    double erow[2], ecol[4];
#pragma unroll
    for (int s = 0; s < 2; ++s) erow[s] = E[(bi * GB + 2 * wy + s) * ROWBLK + (lane & 31)];
#pragma unroll
    for (int u = 0; u < 4; ++u) ecol[u] = E[(bj * GB + 4 * wx + u) * ROWBLK + (lane & 31)];
    if (idle) return;

    // epilogue: lane holds column j = lane%32, rows 8(r/4) + 4(lane/32) + r%4
    const int64_t N = a.N;
    const double invK = 1.0 / (double)a.K;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t C = bj * GB + 4 * wx + u;
        const int64_t j = C * ROWBLK + (lane & 31);
        const double Ej = ecol[u];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int64_t R = bi * GB + 2 * wy + s;
            bool flagged = false;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int64_t i0 = R * ROWBLK + 8 * g + 4 * (lane >> 5);
                int64_t base = i0 * (2 * N - i0 - 1) / 2 - i0 - 1;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t i = i0 + q;
                    const double Ei = __shfl(erow[s], 8 * g + 4 * (lane >> 5) + q, 64);
                    const double r2 = fma(-2.0, (double)acc[s][u][4 * g + q], Ei + Ej) * invK;
                    const float v = sqrtf((float)fmax(r2, 0.0));
                    const bool live = i < j && j < N;
                    if (live) a.out[base + j] = v;
                    flagged |= live && (double)v < a.flag_coef * (Ei + Ej);
                    base += N - i - 2;
                }
            }
            if (__any(flagged) && lane == 0) {
                const int k = atomicAdd(&a.counters[0], 1);
                a.list[k] = FixEntry{0u, ((uint32_t)R << 16) | (uint32_t)C};
            }
        }
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
    const dim3 pg((unsigned)(a.Np / ROWBLK)), pb(PREP_T);
    const bool xl = a.L <= PREP_LDS_L;
    switch (mode) {
    case MODE_FP32:
        if (xl) dist_prep_kernel<MODE_FP32, true><<<pg, pb, 0, s>>>(a);
        else dist_prep_kernel<MODE_FP32, false><<<pg, pb, 0, s>>>(a);
        break;
    case MODE_FP16:
        if (xl) dist_prep_kernel<MODE_FP16, true><<<pg, pb, 0, s>>>(a);
        else dist_prep_kernel<MODE_FP16, false><<<pg, pb, 0, s>>>(a);
        break;
    case MODE_BF16:
    case MODE_BF16X4:
        if (xl) dist_prep_kernel<MODE_BF16, true><<<pg, pb, 0, s>>>(a);
        else dist_prep_kernel<MODE_BF16, false><<<pg, pb, 0, s>>>(a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dist_tile(int mode, const DistLaunch &a, hipStream_t s)
{
    const dim3 tg((unsigned)round_up(a.T, 8)), tb(512);
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
