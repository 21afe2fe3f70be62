// Prep pass: centre every model, write the contraction operands in the
// fragment-native layout described in internal.h, and record each model's
// sum of squared centred coordinates (E = L R^2, Eq. 2) computed from exactly
// the operand values the contraction will use, plus its FP64 centroid for
// the fix-up.  In the reference frame (see ModelSet) the model is first
// superimposed onto the reference structure by its optimal rotation, the
// operands are its residuals from the reference, and the per-model FP64
// terms U = G + P and P^T are recorded for the epilogue.  One wave per
// (padded) model over all model sets of a launch; HBM-bound (reads 12 L bytes
// per model, plus the reference's 12 L from L2 in the frame; writes the
// operands once).
#include "eq2.h"
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
    if (g == 0 && lane < 4) a.counters[lane] = 0;
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

    // Reference frame: the rotation rot taking this model onto the reference
    // (the proper rotation maximising sum r . (rot a), i.e. the transpose of
    // the trace-norm adjoint of sum a r^T), and G = sum r r^T.  A rotation
    // that is not orthonormal to 1e-12 (degenerate correlations) is replaced
    // by the identity: any rotation gives the same scores, only the size of
    // the residuals depends on it.
    const bool frame = s.frame != 0;
    double rot[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
    double G[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double cr[3] = {0.0, 0.0, 0.0};
    const float *xr = (s.ref_b ? a.XB : a.XA) + s.ref_X +
                      (frame ? (int64_t)*(const int *)(a.ws + s.refidx) * L * 3 : 0);
    if (frame && real) {
        for (int64_t l = lane; l < L; l += 64) {
            cr[0] += (double)xr[3 * l];
            cr[1] += (double)xr[3 * l + 1];
            cr[2] += (double)xr[3 * l + 2];
        }
        const double inv = 1.0 / (double)L;
#pragma unroll
        for (int c = 0; c < 3; ++c) cr[c] = wave_sum(cr[c]) * inv;
        double hm[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int64_t l = lane; l < L; l += 64) {
            const double av[3] = {(double)x[3 * l] - c0, (double)x[3 * l + 1] - c1,
                                  (double)x[3 * l + 2] - c2};
            const double rv[3] = {(double)xr[3 * l] - cr[0], (double)xr[3 * l + 1] - cr[1],
                                  (double)xr[3 * l + 2] - cr[2]};
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    hm[3 * p + q] = fma(av[p], rv[q], hm[3 * p + q]);
                    G[3 * p + q] = fma(rv[p], rv[q], G[3 * p + q]);
                }
        }
#pragma unroll
        for (int u = 0; u < 9; ++u) {
            hm[u] = wave_sum(hm[u]);
            G[u] = wave_sum(G[u]);
        }
        double q[9];
        eq2_adjoint(hm, q);
        double dev = 0.0;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const double d = q[p] * q[t] + q[3 + p] * q[3 + t] + q[6 + p] * q[6 + t];
                dev = fmax(dev, fabs(d - (p == t ? 1.0 : 0.0)));
            }
        const double det = q[0] * (q[4] * q[8] - q[5] * q[7]) - q[1] * (q[3] * q[8] - q[5] * q[6]) +
                           q[2] * (q[3] * q[7] - q[4] * q[6]);
        if (dev <= 1e-12 && det > 0.5) {
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int t = 0; t < 3; ++t) rot[3 * p + t] = q[3 * t + p];
        }
    }

    const int64_t R = m / ROWBLK;
    const int r = (int)(m % ROWBLK);
    const int64_t KB = s.KB;
    const double cc[3] = {c0, c1, c2};
    // e: radius of the model the contraction sees (reference + quantised
    // residual); w: of the quantised residual; pp: P = sum d r^T
    double e = 0.0, w = 0.0;
    double pp[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t l = lane; l < s.Lp; l += 64) {
        const bool in = real && l < L;
        double av[3], rv[3], dv[3], qv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            av[c] = in ? (double)x[3 * l + c] - cc[c] : 0.0;
            rv[c] = (in && frame) ? (double)xr[3 * l + c] - cr[c] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
            dv[c] = frame ? fma(rot[3 * c], av[0], fma(rot[3 * c + 1], av[1], fma(rot[3 * c + 2], av[2], -rv[c])))
                          : av[c];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = dv[c];
            if (MODE == MODE_FP32) {
                const float f = (float)v;
                qv[c] = (double)f;
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
                qv[c] = hv + lv;   // exact in FP64
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            w = fma(qv[c], qv[c], w);
            const double sv = rv[c] + qv[c];
            e = fma(sv, sv, e);
#pragma unroll
            for (int t = 0; t < 3; ++t) pp[3 * c + t] = fma(qv[c], rv[t], pp[3 * c + t]);
        }
    }
    e = wave_sum(e);
    w = wave_sum(w);
    if (frame) {
#pragma unroll
        for (int u = 0; u < 9; ++u) pp[u] = wave_sum(pp[u]);
    }
    if (lane == 0) {
        E[m] = e;
        ((double *)(a.ws + s.F))[m] = fma(s.fw, w, s.fe * e);
        double *U = (double *)(a.ws + s.U) + 9 * m;
        double *PT = (double *)(a.ws + s.PT) + 9 * m;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                U[3 * p + t] = (frame && real) ? G[3 * p + t] + pp[3 * p + t] : 0.0;
                PT[3 * p + t] = (frame && real) ? pp[3 * t + p] : 0.0;
            }
    }
}

// Reference choice, one workgroup per model set that owns a reference: of
// the first K = min(ref_N, REF_CANDIDATES) models, the one whose squared
// cRMSDs to the other K - 1 sum to the least (Eq. 2 in FP64 on the centred
// models; ties to the lowest index).  Its index goes to the workspace for
// prep.  Any choice gives the same scores; a central one gives the smallest
// residuals, hence the smallest contraction error.
__global__ __launch_bounds__(256) void ref_select_kernel(PrepLaunch a)
{
    __shared__ double cen[REF_CANDIDATES][3], rad[REF_CANDIDATES];
    __shared__ double lr2[REF_CANDIDATES * (REF_CANDIDATES - 1) / 2];
    const ModelSet &s = a.table ? a.table[blockIdx.x] : a.set[blockIdx.x];
    if (!s.frame || !s.ref_own) return;                  // uniform over the workgroup
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t L = s.L;
    const int K = (int)(s.ref_N < REF_CANDIDATES ? s.ref_N : REF_CANDIDATES);
    const float *x0 = (s.ref_b ? a.XB : a.XA) + s.ref_X;
    for (int k = w; k < K; k += 4) {
        const float *x = x0 + k * L * 3;
        double c[3] = {0.0, 0.0, 0.0};
        for (int64_t l = lane; l < L; l += 64)
#pragma unroll
            for (int u = 0; u < 3; ++u) c[u] += (double)x[3 * l + u];
#pragma unroll
        for (int u = 0; u < 3; ++u) c[u] = wave_sum(c[u]) / (double)L;
        double e = 0.0;
        for (int64_t l = lane; l < L; l += 64)
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const double d = (double)x[3 * l + u] - c[u];
                e = fma(d, d, e);
            }
        e = wave_sum(e);
        if (lane == 0) {
            cen[k][0] = c[0];
            cen[k][1] = c[1];
            cen[k][2] = c[2];
            rad[k] = e;
        }
    }
    __syncthreads();
    const int npair = K * (K - 1) / 2;
    for (int t = w; t < npair; t += 4) {
        int p = 0, q = t;
        while (q >= K - 1 - p) {
            q -= K - 1 - p;
            ++p;
        }
        q += p + 1;
        const float *xp = x0 + p * L * 3, *xq = x0 + q * L * 3;
        double h[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int64_t l = lane; l < L; l += 64) {
            double u[3], v[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                u[c] = (double)xp[3 * l + c] - cen[p][c];
                v[c] = (double)xq[3 * l + c] - cen[q][c];
            }
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) h[3 * i + j] = fma(u[i], v[j], h[3 * i + j]);
        }
#pragma unroll
        for (int u = 0; u < 9; ++u) h[u] = wave_sum(h[u]);
        if (lane == 0) lr2[t] = fmax(eq2_lrmsd2(h, rad[p], rad[q]), 0.0);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int best = 0;
        double bsum = 0.0;
        for (int k = 0; k < K; ++k) {
            double sum = 0.0;
            int t = 0;
            for (int p = 0; p < K; ++p)
                for (int q = p + 1; q < K; ++q, ++t)
                    if (p == k || q == k) sum += lr2[t];
            if (k == 0 || sum < bsum) {
                bsum = sum;
                best = k;
            }
        }
        *(int *)(a.ws + s.refidx) = best;
    }
}

hipError_t launch_prep(const PrepLaunch &a, hipStream_t s)
{
    bool frame = a.table != nullptr;     // a batch: some set may use the frame
    for (int k = 0; k < (a.table ? 0 : a.nset); ++k) frame |= a.set[k].frame != 0;
    if (frame && a.mode != MODE_FP64)
        ref_select_kernel<<<dim3((unsigned)a.nset), dim3(256), 0, s>>>(a);
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
