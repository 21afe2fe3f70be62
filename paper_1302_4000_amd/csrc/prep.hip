// Prep pass: centre every model, write the contraction operands in the
// fragment-native layout described in internal.h, and record each model's
// sum of squared centred coordinates (E = L R^2, Eq. 2) computed from exactly
// the operand values the contraction will use, plus its FP64 centroid for
// the fix-up.  In the reference frame (see ModelSet) the model is first
// superimposed onto the reference structure by its optimal rotation, the
// operands are its residuals from the reference, and the per-model FP64
// terms U = G + P and P^T are recorded for the epilogue.  A group of
// PREP_W lanes per (padded) model, 64 / PREP_W models per wave, over all
// model sets of a launch: the per-model work (reductions, the rotation)
// dominates at typical lengths, and a wave shares it over several models.
// Reads 12 L bytes per model (twice: two passes, the second from L2), plus
// the reference's 12 L from L2 in the frame; writes the operands once.
#include "eq2.h"
#include "internal.h"

namespace clusco {

constexpr int PREP_W = 8;
// atoms per lane whose loads a round of the atom loops issues together
constexpr int PREP_U = 4;
static_assert(REF_CANDIDATES <= PREP_W, "a group holds every reference candidate");
// The operand stores of pass 2 use that a round of a lane covers atoms
// sl + 8 i: the element within an 8-atom run is the lane's own, and every
// store of a round lies at a fixed offset from one base (see pass 2).
static_assert(PREP_W == 8 && PREP_U % 2 == 0, "pass 2 store addressing");

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

// Sums of N values over aligned groups of W lanes (W = 64: the wave), the N
// reductions interleaved (their cross-lane steps overlap instead of queueing
// behind one another).
template <int W = 64, int N>
__device__ __forceinline__ void wave_sums(double (&v)[N])
{
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) {
        double t[N];
#pragma unroll
        for (int k = 0; k < N; ++k) t[k] = __shfl_xor(v[k], o, 64);
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] += t[k];
    }
}

// Per model set that owns a reference (ModelSet::refinfo, doubles):
//   [0, RI_PAIRS)            L cRMSD^2 of candidate pairs (p, q), p < q, in
//                            row-major order over all REF_CANDIDATES slots
//   [RI_CEN, RI_CEN + 3 K)   the candidates' centroids
//   [RI_G, RI_G + 9 K)       their G = sum r r^T of the centred coordinates
constexpr int REF_WAVES = RI_PAIRS + REF_CANDIDATES;   // one wave per pair / candidate

// Reference candidates of every model set that owns a reference: the first
// K = min(ref_N, REF_CANDIDATES) models.  Grid: sets x (REF_WAVES / 4)
// workgroups of 4 waves; wave u < RI_PAIRS computes pair u's L cRMSD^2 by
// Eq. 2 in FP64 from one pass of moments (any choice of reference gives the
// same scores, so only its ranking matters), wave RI_PAIRS + k the centroid
// and G of candidate k.
__global__ __launch_bounds__(256) void ref_moments_kernel(PrepLaunch a)
{
    const int per = REF_WAVES / 4;
    const ModelSet &s = a.table ? a.table[blockIdx.x / per] : a.set[blockIdx.x / per];
    if (!s.frame || !s.ref_own) return;                  // uniform over the workgroup
    const int lane = threadIdx.x & 63;
    const int u = (int)(blockIdx.x % per) * 4 + (threadIdx.x >> 6);
    const int64_t L = s.L;
    const int K = (int)(s.ref_N < REF_CANDIDATES ? s.ref_N : REF_CANDIDATES);
    const float *x0 = (s.ref_b ? a.XB : a.XA) + s.ref_X;
    double *info = (double *)(a.ws + s.refinfo);
    const double inv = 1.0 / (double)L;
    if (u < RI_PAIRS) {
        int p = 0, q = u;
        while (q >= REF_CANDIDATES - 1 - p) {
            q -= REF_CANDIDATES - 1 - p;
            ++p;
        }
        q += p + 1;
        if (q >= K) return;
        const float *xp = x0 + p * L * 3, *xq = x0 + q * L * 3;
        // sum x_p, sum x_q, sum x_p x_q^T, sum |x_p|^2, sum |x_q|^2
        double m[17];
#pragma unroll
        for (int k = 0; k < 17; ++k) m[k] = 0.0;
        for (int64_t l = lane; l < L; l += 64) {
            double up[3], uq[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                up[c] = (double)xp[3 * l + c];
                uq[c] = (double)xq[3 * l + c];
                m[c] += up[c];
                m[3 + c] += uq[c];
                m[15] = fma(up[c], up[c], m[15]);
                m[16] = fma(uq[c], uq[c], m[16]);
            }
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) m[6 + 3 * i + j] = fma(up[i], uq[j], m[6 + 3 * i + j]);
        }
        wave_sums(m);
        if (lane == 0) {
            double h[9];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) h[3 * i + j] = m[6 + 3 * i + j] - m[i] * m[3 + j] * inv;
            const double ep = m[15] - (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) * inv;
            const double eq = m[16] - (m[3] * m[3] + m[4] * m[4] + m[5] * m[5]) * inv;
            info[u] = fmax(eq2_lrmsd2(h, ep, eq), 0.0);
        }
    } else {
        const int k = u - RI_PAIRS;
        if (k >= K) return;
        const float *x = x0 + k * L * 3;
        double c[3] = {0.0, 0.0, 0.0};
        for (int64_t l = lane; l < L; l += 64)
#pragma unroll
            for (int t = 0; t < 3; ++t) c[t] += (double)x[3 * l + t];
        wave_sums(c);
#pragma unroll
        for (int t = 0; t < 3; ++t) c[t] *= inv;
        double g[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) g[t] = 0.0;
        for (int64_t l = lane; l < L; l += 64) {
            const double r[3] = {(double)x[3 * l] - c[0], (double)x[3 * l + 1] - c[1],
                                 (double)x[3 * l + 2] - c[2]};
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) g[3 * i + j] = fma(r[i], r[j], g[3 * i + j]);
        }
        wave_sums(g);
        if (lane < 3) info[RI_CEN + 3 * k + lane] = c[lane];
        if (lane < 9) info[RI_G + 9 * k + lane] = g[lane];
    }
}

// The chosen reference of a set: of the K candidates, the one whose squared
// cRMSDs to the other K - 1 sum to the least (ties to the lowest index), so
// that an outlier model is not the reference.  Lane `base + k` of a group
// sums candidate k's row (k < K <= the group's width); every lane of the
// group returns the choice.
__device__ __forceinline__ int ref_choice(const double *info, int K, int sl, int base)
{
    // Pair (p, q), p < q, is entry p (2 REF_CANDIDATES - p - 1) / 2 + q - p - 1.
    // The row's entries are loaded without branches (all lie in the info
    // block; those past K are not used) and summed in ascending order of the
    // partner, which is ascending entry order.
    const int me = sl < REF_CANDIDATES ? sl : 0;
    double v[REF_CANDIDATES];
#pragma unroll
    for (int k = 0; k < REF_CANDIDATES; ++k) {
        const int p = k < me ? k : me, q = k < me ? me : k;
        v[k] = k == me ? 0.0 : info[p * (2 * REF_CANDIDATES - p - 1) / 2 + q - p - 1];
    }
    double sum = 0.0;
    if (sl < K) {
#pragma unroll
        for (int k = 0; k < REF_CANDIDATES; ++k)
            if (k != me && k < K) sum += v[k];
    }
    int best = 0;
    double bsum = __shfl(sum, base, 64);
    for (int k = 1; k < K; ++k) {
        const double v = __shfl(sum, base + k, 64);
        if (v < bsum) {
            bsum = v;
            best = k;
        }
    }
    return best;
}

template <int MODE>
__global__ __launch_bounds__(64) void prep_kernel(PrepLaunch a)
{
    // PREP_W lanes per model: a wave takes 64 / PREP_W consecutive models
    const int sl = (int)threadIdx.x % PREP_W;
    const int64_t g0 = (int64_t)blockIdx.x * (64 / PREP_W) + (int64_t)threadIdx.x / PREP_W;
    const bool live = g0 < a.total;                // groups past the last model write nothing
    const int64_t g = live ? g0 : a.total - 1;
    if (blockIdx.x == 0 && threadIdx.x < 4) a.counters[threadIdx.x] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.zero64) *a.zero64 = 0ull;

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
    const bool frame = MODE != MODE_FP64 && s.frame != 0;
    const double inv = 1.0 / (double)L;

    // the reference (frame): the chosen candidate's coordinates and
    // centroid from ref_moments_kernel (its G is read at the end)
    const float *xr = x;
    double cr[3] = {0.0, 0.0, 0.0};
    int kref = 0;
    if (frame) {
        const double *info = (const double *)(a.ws + s.refinfo);
        const int K = (int)(s.ref_N < REF_CANDIDATES ? s.ref_N : REF_CANDIDATES);
        const int k = ref_choice(info, K, sl, (int)threadIdx.x - sl);
        xr = (s.ref_b ? a.XB : a.XA) + s.ref_X + (int64_t)k * L * 3;
#pragma unroll
        for (int t = 0; t < 3; ++t) cr[t] = info[RI_CEN + 3 * k + t];
        kref = k;
    }

    // pass 1: the centroid and, in the frame, sum x r^T with r the centred
    // reference (= sum (x - c) r^T, since sum r = 0)
    // Both passes take the lane's atoms PREP_U at a time: the loads of a
    // round are issued together, without per-atom branches, before any is
    // used (one memory latency per round instead of one or two per atom).
    // Atoms past L of a real model load atom L - 1 (always there; xr is x
    // itself without the frame) and add exact zeros, so the sums are those of
    // one atom at a time in order.
    double m1[12];
#pragma unroll
    for (int t = 0; t < 12; ++t) m1[t] = 0.0;
    if (real) {
        for (int64_t l0 = sl; l0 < L; l0 += PREP_U * PREP_W) {
            float xs[PREP_U][3], rs[PREP_U][3];
#pragma unroll
            for (int u = 0; u < PREP_U; ++u) {
                const int64_t l = l0 + u * PREP_W, lc = l < L ? l : L - 1;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xs[u][c] = x[3 * lc + c];
                    rs[u][c] = xr[3 * lc + c];
                }
            }
#pragma unroll
            for (int u = 0; u < PREP_U; ++u) {
                const bool in = l0 + u * PREP_W < L;
                double xv[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xv[c] = in ? (double)xs[u][c] : 0.0;
                    m1[c] += xv[c];
                }
                if (frame) {
                    double rv[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) rv[c] = in ? (double)rs[u][c] - cr[c] : 0.0;
#pragma unroll
                    for (int p = 0; p < 3; ++p)
#pragma unroll
                        for (int q = 0; q < 3; ++q) m1[3 + 3 * p + q] = fma(xv[p], rv[q], m1[3 + 3 * p + q]);
                }
            }
        }
    }
    wave_sums<PREP_W>(m1);
    const double c0 = m1[0] * inv, c1 = m1[1] * inv, c2 = m1[2] * inv;
    if (sl == 0 && live) {
        cen[3 * m] = c0;
        cen[3 * m + 1] = c1;
        cen[3 * m + 2] = c2;
    }

    // Reference frame: the rotation rot taking this model onto the reference
    // (the proper rotation maximising sum r . (rot a), i.e. the transpose of
    // the trace-norm adjoint of sum a r^T).  A rotation that is not
    // orthonormal to 1e-12 (degenerate correlations) is replaced by the
    // identity: any rotation gives the same scores, only the size of the
    // residuals depends on it.
    double rot[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
    if (frame && real) {
        double hm[9], q[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) hm[t] = m1[3 + t];
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

    // pass 2: operands, and the sums m2 = [e64, e, w, P (9)]: e64 the exact
    // FP64 radius of the raw coordinates (the fix-up's), e the radius of the
    // model the contraction sees (reference + quantised residual), w that of
    // the quantised residual, P = sum d r^T
    const int64_t R = m / ROWBLK;
    const int r = (int)(m % ROWBLK);
    const int64_t KB = s.KB;
    const double cc[3] = {c0, c1, c2};
    double m2[12];
#pragma unroll
    for (int t = 0; t < 12; ++t) m2[t] = 0.0;
    const int64_t Lend = MODE == MODE_FP64 ? L : s.Lp;
    // Store addressing from the layout in internal.h with l = l0 + 8 u and
    // l0 = sl + 8 PREP_U j.  FP32 (K-block 8, runs of 4): kb = PREP_U j + u,
    // h = sl / 4, e = sl % 4, so (u, c) is at base + 768 u + 256 c floats.
    // 16-bit (K-block 16, runs of 8): kb = PREP_U j / 2 + u / 2, h = u % 2,
    // e = sl, so (u, c, part) is at base + 3072 (u / 2) + 256 (u % 2) +
    // 1024 c + 512 part halves.
    float *const ops32 = (float *)(a.ws + s.ops) + (R * KB * 3 * 64 + r + 32 * (sl >> 2)) * 4 + (sl & 3);
    uint16_t *const ops16 = (uint16_t *)(a.ws + s.ops) + (R * KB * 6 * 64 + r) * 8 + sl;
    for (int64_t l0 = sl; l0 < Lend; l0 += PREP_U * PREP_W) {
        float *const row32 = ops32 + (l0 - sl) / PREP_W * 768;
        uint16_t *const row16 = ops16 + (l0 - sl) / (2 * PREP_W) * 3072;
        // padding models (m >= N) load nothing: an empty ensemble has no
        // coordinates at all
        float xs[PREP_U][3] = {}, rs[PREP_U][3] = {};
        if (real) {
#pragma unroll
            for (int u = 0; u < PREP_U; ++u) {
                const int64_t l = l0 + u * PREP_W, lc = l < L ? l : L - 1;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xs[u][c] = x[3 * lc + c];
                    rs[u][c] = xr[3 * lc + c];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < PREP_U; ++u) {
            const int64_t l = l0 + u * PREP_W;
            if (l >= Lend) break;
            const bool in = real && l < L;
            double av[3], rv[3], dv[3], qv[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                av[c] = in ? (double)xs[u][c] - cc[c] : 0.0;
                rv[c] = (in && frame) ? (double)rs[u][c] - cr[c] : 0.0;
                m2[0] = fma(av[c], av[c], m2[0]);
            }
            if (MODE == MODE_FP64) continue;
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
                    if (live) row32[768 * u + 256 * c] = f;
                } else {
                    uint16_t *const hi = row16 + 3072 * (u >> 1) + 256 * (u & 1) + 1024 * c;
                    double hv, lv;
                    if (is_bf16(MODE)) {
                        const uint16_t hb = bf16_bits_rn((float)v);
                        hv = (double)bf16_bits_to_float(hb);
                        const uint16_t lb = bf16_bits_rn((float)(v - hv));
                        lv = (double)bf16_bits_to_float(lb);
                        if (live) {
                            hi[0] = hb;
                            hi[512] = lb;
                        }
                    } else {
                        const _Float16 hh = (_Float16)(float)v;
                        hv = (double)(float)hh;
                        const _Float16 ll = (_Float16)(float)(v - hv);
                        lv = (double)(float)ll;
                        if (live) {
                            hi[0] = __builtin_bit_cast(uint16_t, hh);
                            hi[512] = __builtin_bit_cast(uint16_t, ll);
                        }
                    }
                    qv[c] = hv + lv;   // exact in FP64
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                m2[2] = fma(qv[c], qv[c], m2[2]);
                const double sv = rv[c] + qv[c];
                m2[1] = fma(sv, sv, m2[1]);
#pragma unroll
                for (int t = 0; t < 3; ++t) m2[3 + 3 * c + t] = fma(qv[c], rv[t], m2[3 + 3 * c + t]);
            }
        }
    }
    wave_sums<PREP_W>(m2);
    if (sl == 0 && live) {
        E64[m] = m2[0];
        if (MODE == MODE_FP64) {
            E[m] = 0.0;
            return;
        }
        E[m] = m2[1];
        ((double *)(a.ws + s.F))[m] = fma(s.fw, m2[2], s.fe * m2[1]);
        double *U = (double *)(a.ws + s.U) + 9 * m;
        double *PT = (double *)(a.ws + s.PT) + 9 * m;
        const double *G = (const double *)(a.ws + s.refinfo) + RI_G + 9 * kref;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                U[3 * p + t] = (frame && real) ? G[3 * p + t] + m2[3 + 3 * p + t] : 0.0;
                PT[3 * p + t] = (frame && real) ? m2[3 + 3 * t + p] : 0.0;
            }
    }
}

hipError_t launch_prep(const PrepLaunch &a, hipStream_t s)
{
    bool frame = a.table != nullptr;     // a batch: some set may use the frame
    for (int k = 0; k < (a.table ? 0 : a.nset); ++k) frame |= a.set[k].frame != 0;
    if (frame && a.mode != MODE_FP64)
        ref_moments_kernel<<<dim3((unsigned)(a.nset * (REF_WAVES / 4))), dim3(256), 0, s>>>(a);
    dim3 grid((unsigned)((a.total + 64 / PREP_W - 1) / (64 / PREP_W))), block(64);
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
