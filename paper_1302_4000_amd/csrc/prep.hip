// Prep pass: centre every model, write the contraction operands in the
// fragment-native layout described in internal.h, and record each model's
// sum of squared centred coordinates (E = L R^2, Eq. 2) computed from exactly
// the operand values the contraction will use, plus its FP64 centroid for
// the fix-up.  One wave per (padded) model over all model sets of a launch;
// HBM-bound (reads 12 L bytes per model, writes the operands once).
#include "internal.h"

namespace clusco {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// round-to-nearest-even float -> bfloat16 bits (finite inputs)
__device__ __forceinline__ uint16_t bf16_bits_rn(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_bits_to_float(uint16_t b)
{
    return __uint_as_float((uint32_t)b << 16);
}

template <int MODE>
__global__ __launch_bounds__(64) void prep_kernel(PrepLaunch a)
{
    const int64_t g = blockIdx.x;
    const int lane = threadIdx.x;
    if (g == 0 && lane < 2) a.counters[lane] = 0;
    if (g == 0 && lane == 0 && a.zero64) *a.zero64 = 0ull;

    ModelSet s;
    if (a.table) {
        s = a.table[table_find(a.table, a.nset, g, [](const ModelSet &m) { return m.model0; })];
    } else {
        s = (a.nset > 1 && g >= a.set[1].model0) ? a.set[1] : a.set[0];
    }
    const int64_t m = g - s.model0;
    const int64_t L = s.L;
    const bool real = m < s.N;
    const float *x = (s.use_b ? a.XB : a.XA) + s.X + (real ? m : 0) * L * 3;
    double *E = (double *)(a.ws + s.E);
    double *cen = (double *)(a.ws + s.cen);
    double *E64 = (double *)(a.ws + s.E64);

    double c0 = 0.0, c1 = 0.0, c2 = 0.0;
    if (real) {
        for (int64_t l = lane; l < L; l += 64) {
            c0 += (double)x[3 * l];
            c1 += (double)x[3 * l + 1];
            c2 += (double)x[3 * l + 2];
        }
        const double inv = 1.0 / (double)L;
        c0 = wave_sum(c0) * inv;
        c1 = wave_sum(c1) * inv;
        c2 = wave_sum(c2) * inv;
    }
    if (lane == 0) {
        cen[3 * m] = c0;
        cen[3 * m + 1] = c1;
        cen[3 * m + 2] = c2;
    }
    // exact FP64 radius of the raw coordinates (used by the FP64 fix-up)
    double e64 = 0.0;
    if (real) {
        for (int64_t l = lane; l < L; l += 64) {
            const double d0 = (double)x[3 * l] - c0, d1 = (double)x[3 * l + 1] - c1,
                         d2 = (double)x[3 * l + 2] - c2;
            e64 += d0 * d0 + d1 * d1 + d2 * d2;
        }
        e64 = wave_sum(e64);
    }
    if (lane == 0) E64[m] = e64;
    if (MODE == MODE_FP64) {
        if (lane == 0) E[m] = 0.0;
        return;
    }

    const int64_t R = m / ROWBLK;
    const int r = (int)(m % ROWBLK);
    const int64_t KB = s.KB;
    const double cc[3] = {c0, c1, c2};
    double e = 0.0;
    for (int64_t l = lane; l < s.Lp; l += 64) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = (real && l < L) ? (double)x[3 * l + c] - cc[c] : 0.0;
            if (MODE == MODE_FP32) {
                const float f = (float)v;
                e += (double)f * (double)f;
                const int64_t kb = l >> 3, h = (l >> 2) & 1, el = l & 3;
                const int64_t idx = (((R * KB + kb) * 3 + c) * 64 + r + 32 * h) * 4 + el;
                ((float *)(a.ws + s.ops))[idx] = f;
            } else {
                const int64_t kb = l >> 4, h = (l >> 3) & 1, el = l & 7;
                const int64_t base = (((R * KB + kb) * 3 + c) * 2) * 64;
                const int64_t hi_idx = (base + r + 32 * h) * 8 + el;
                const int64_t lo_idx = (base + 64 + r + 32 * h) * 8 + el;
                uint16_t *ops = (uint16_t *)(a.ws + s.ops);
                double hv, lv;
                if (is_bf16(MODE)) {
                    const uint16_t hb = bf16_bits_rn((float)v);
                    hv = (double)bf16_bits_to_float(hb);
                    const uint16_t lb = bf16_bits_rn((float)(v - hv));
                    lv = (double)bf16_bits_to_float(lb);
                    ops[hi_idx] = hb;
                    ops[lo_idx] = lb;
                } else {
                    const _Float16 hh = (_Float16)(float)v;
                    hv = (double)(float)hh;
                    const _Float16 ll = (_Float16)(float)(v - hv);
                    lv = (double)(float)ll;
                    ops[hi_idx] = __builtin_bit_cast(uint16_t, hh);
                    ops[lo_idx] = __builtin_bit_cast(uint16_t, ll);
                }
                const double sv = hv + lv;   // exact in FP64
                e += sv * sv;
            }
        }
    }
    e = wave_sum(e);
    if (lane == 0) E[m] = e;
}

hipError_t launch_prep(const PrepLaunch &a, hipStream_t s)
{
    dim3 grid((unsigned)a.total), block(64);
    switch (a.mode) {
    case MODE_FP32: prep_kernel<MODE_FP32><<<grid, block, 0, s>>>(a); break;
    case MODE_BF16: prep_kernel<MODE_BF16><<<grid, block, 0, s>>>(a); break;
    case MODE_FP16: prep_kernel<MODE_FP16><<<grid, block, 0, s>>>(a); break;
    case MODE_BF16X4: prep_kernel<MODE_BF16><<<grid, block, 0, s>>>(a); break;
    default: prep_kernel<MODE_FP64><<<grid, block, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

} // namespace clusco
