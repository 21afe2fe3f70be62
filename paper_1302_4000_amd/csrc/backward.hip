// Gradient pass of the backward.  The pairs pass (tile kernel, OP_BWD) has
// stored, for every pair, w = g / (L cRMSD) and w Q, Q the adjoint of the
// pair's correlation (see eq2_adjoint).  Differentiating Eq. 2 (the optimum
// makes the derivative through the superposition vanish):
//     d cRMSD / d a_l = (a_l - Q b_l) / (L cRMSD),
//     d cRMSD / d b_l = (b_l - Q^T a_l) / (L cRMSD),
// so model m collects  (sum_j w_mj) a_m - sum_j Q~_mj b_j  with Q~ = Q when m
// is the pair's first model and Q^T when it is the second.  Both terms sum to
// zero over atoms (centred models), which is the centring Jacobian.
//
// The second term is one matrix product per workgroup of 16 models:
//     G[(c, m), l] = sum over (j, d) of  Q~_mj[c][d] * b_j[l][d],
// rows (coordinate c, model m), contraction over (partner j, coordinate d),
// columns atoms l.  It runs on v_mfma_f64_16x16x4_f64: FP64 products of the
// FP32 records and centred FP32 coordinates, FP64 accumulation in a fixed
// order (deterministic).  FP64 matters here: the two terms nearly cancel
// when the partners surround the model (a reference against many noisy
// copies of itself).
//
//  grad_planes  centred partner coordinates as float planes P[j][d][l] (atoms
//               padded with zeros to 16, partners to a multiple of 32), so
//               that the flattened contraction index k = 3j + d addresses row
//               k of a plain row-major matrix
//  grad_kernel  one workgroup = 16 models x 256 atoms x a range of partner
//               blocks (the whole range unless few row models), 8 waves, each owning
//               two 16-atom column tiles and all three coordinate row tiles
//               (6 accumulators).  Per block of 32 partners the 512 pair
//               records (one per thread) are staged to LDS as the A operand
//               (double-buffered, one barrier per block); B fragments come
//               straight from the planes into registers one block ahead.
//               The weights w are summed per model from the same staging.
//  grad_finish  with several partner ranges: FP64 partials summed in range
//               order (deterministic), then the gradient.
#include "internal.h"

namespace clusco {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int GBM = 16;               // models per workgroup (one MFMA row tile per coordinate)
constexpr int GBJ = 32;               // partners per staged block
constexpr int GKB = 3 * GBJ;          // contraction length of one block
constexpr int GKS = GKB / 4;          // MFMA steps per block
constexpr int GW = 8;                 // waves per workgroup
constexpr int GCT = 2;                // 16-atom column tiles per wave
constexpr int GLC = 16 * GW * GCT;    // atoms per workgroup (256)
constexpr int ARS = 3 * GBM + 1;      // LDS row stride of the staged weights
static_assert(GBM * GBJ == 64 * GW, "one pair record per thread per block");

__global__ __launch_bounds__(256) void grad_planes_kernel(const float *X, const double *cen,
                                                          float *P, int64_t N, int64_t Np,
                                                          int64_t L, int64_t Lp)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Np * Lp) return;
    const int64_t j = t / Lp, l = t % Lp;
    float v[3] = {0.0f, 0.0f, 0.0f};
    if (j < N && l < L) {
        const float *x = X + (j * L + l) * 3;
#pragma unroll
        for (int d = 0; d < 3; ++d) v[d] = (float)((double)x[d] - cen[3 * j + d]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) P[(j * 3 + d) * Lp + l] = v[d];
}

// The record of pair (m, j) seen from row model m: its index and whether the
// stored matrix must be transposed (m is the pair's second model).  Returns
// false when the pair does not exist.
__device__ __forceinline__ bool grad_pair(const GradLaunch &a, int64_t m, int64_t j, int64_t *k,
                                          bool *tr)
{
    if (m >= a.NR || j >= a.NC) return false;
    if (a.kind == GK_SYM) {
        if (m == j) return false;
        *tr = m > j;
        *k = *tr ? packed_index(j, m, a.NR) : packed_index(m, j, a.NR);
    } else if (a.kind == GK_CROSS_A) {
        *tr = false;
        *k = m * a.NC + j;
    } else {
        *tr = true;
        *k = j * a.NR + m;
    }
    return true;
}

__global__ __launch_bounds__(512, 1) void grad_kernel(GradLaunch a)
{
    __shared__ float As[2][GKB * ARS];    // A operand: [k = 3 j + d][row = 16 c + m]
    __shared__ float Ws[2][GBJ * GBM];    // weights w: [j][m]
    __shared__ double wfin[GBM];
    __shared__ double wred[64 * GW];

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t m0 = (int64_t)blockIdx.x * GBM;
    const int64_t l0 = (int64_t)blockIdx.y * GLC;
    const int64_t NC = a.NC, Lp = a.Lp;
    const int nblk = (int)((NC + GBJ - 1) / GBJ);
    const int split = (int)blockIdx.z;
    const int b0 = split * a.bps;
    const int b1 = min(nblk, b0 + a.bps);

    // column tiles of this wave (wave-uniform validity)
    bool colv[GCT];
    int64_t col[GCT];
#pragma unroll
    for (int ct = 0; ct < GCT; ++ct) {
        col[ct] = l0 + 16 * (w + GW * ct);
        colv[ct] = col[ct] < Lp;
    }
    const int g = lane >> 4, i16 = lane & 15;

    // staging: one pair per thread; the mapping keeps a wave's records
    // contiguous in memory (consecutive j for a row, or consecutive m when
    // the rows are the pairs' second models)
    auto stage_map = [&](int blk, int *ml, int *jl) {
        const int64_t j0 = (int64_t)blk * GBJ;
        const bool trblk = a.kind == GK_CROSS_B || (a.kind == GK_SYM && j0 + GBJ <= m0);
        if (trblk) {
            *ml = tid % GBM;
            *jl = tid / GBM;
        } else {
            *jl = tid % GBJ;
            *ml = tid / GBJ;
        }
    };
    auto stage_load = [&](int blk, int ml, int jl, float4 *r, bool *tr) -> bool {
        int64_t k;
        if (!grad_pair(a, m0 + ml, (int64_t)blk * GBJ + jl, &k, tr)) return false;
        const float4 *p = (const float4 *)(a.wq + 12 * k);
        r[0] = p[0];
        r[1] = p[1];
        r[2] = p[2];
        return true;
    };
    auto stage_store = [&](int buf, int ml, int jl, const float4 *r4, bool ok, bool tr) {
        float r[10];
        r[0] = r4[0].x; r[1] = r4[0].y; r[2] = r4[0].z; r[3] = r4[0].w;
        r[4] = r4[1].x; r[5] = r4[1].y; r[6] = r4[1].z; r[7] = r4[1].w;
        r[8] = r4[2].x; r[9] = r4[2].y;
        float *A = As[buf] + (3 * jl) * ARS + ml;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d)
                A[d * ARS + 16 * c] = ok ? (tr ? r[3 * d + c] : r[3 * c + d]) : 0.0f;
        Ws[buf][jl * GBM + ml] = ok ? r[9] : 0.0f;
    };
    auto load_b = [&](int blk, float (*bq)[GCT]) {
        const float *P = a.P + ((int64_t)blk * GKB + g) * Lp + i16;
#pragma unroll
        for (int s = 0; s < GKS; ++s)
#pragma unroll
            for (int ct = 0; ct < GCT; ++ct)
                bq[s][ct] = colv[ct] ? P[(int64_t)(4 * s) * Lp + col[ct]] : 0.0f;
    };

    f64x4 acc[3][GCT];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int ct = 0; ct < GCT; ++ct) acc[c][ct] = (f64x4){0.0, 0.0, 0.0, 0.0};
    double wpart = 0.0;

    float bcur[GKS][GCT], bnext[GKS][GCT];
    {
        int ml, jl;
        float4 r[3];
        bool tr = false;
        stage_map(b0, &ml, &jl);
        const bool ok = stage_load(b0, ml, jl, r, &tr);
        stage_store(0, ml, jl, r, ok, tr);
        load_b(b0, bcur);
    }
    __syncthreads();

    for (int blk = b0; blk < b1; ++blk) {
        const int buf = (blk - b0) & 1;
        const bool more = blk + 1 < b1;
        int ml = 0, jl = 0;
        float4 r[3];
        bool ok = false, tr = false;
        if (more) {
            stage_map(blk + 1, &ml, &jl);
            ok = stage_load(blk + 1, ml, jl, r, &tr);
            load_b(blk + 1, bnext);
        }
        const float *A = As[buf] + g * ARS + i16;
#pragma unroll
        for (int s = 0; s < GKS; ++s) {
            double af[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) af[c] = (double)A[(4 * s) * ARS + 16 * c];
#pragma unroll
            for (int ct = 0; ct < GCT; ++ct) {
                if (!colv[ct]) continue;
                const double bf = (double)bcur[s][ct];
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    acc[c][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[c], bf, acc[c][ct], 0, 0, 0);
            }
        }
        wpart += (double)Ws[buf][tid];
        if (more) stage_store(buf ^ 1, ml, jl, r, ok, tr);
        __syncthreads();
#pragma unroll
        for (int s = 0; s < GKS; ++s)
#pragma unroll
            for (int ct = 0; ct < GCT; ++ct) bcur[s][ct] = bnext[s][ct];
    }

    // sum of the weights per model, in a fixed order
    wred[tid] = wpart;
    __syncthreads();
    if (tid < GBM) {
        double sacc = 0.0;
        for (int q = 0; q < 64 * GW / GBM; ++q) sacc += wred[tid + GBM * q];
        wfin[tid] = sacc;
    }
    __syncthreads();

    // epilogue: accumulator element v of a lane is G row (c, m = lane / 16 + 4 v),
    // column l = col + lane % 16 (the f64 16x16x4 output layout).  With one
    // split the gradient is finished here; otherwise this split's weight sums
    // and G go to FP64 partials that grad_finish adds in split order.
    if (a.nsplit > 1 && tid < GBM && m0 + tid < a.NR)
        a.wpart[(int64_t)split * a.NR + m0 + tid] = wfin[tid];
#pragma unroll
    for (int ct = 0; ct < GCT; ++ct) {
        if (!colv[ct]) continue;
        const int64_t l = col[ct] + i16;
        if (l >= a.L) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int mm = g + 4 * v;
            const int64_t m = m0 + mm;
            if (m >= a.NR) continue;
            if (a.nsplit > 1) {
                double *pm = a.part + (((int64_t)split * a.NR + m) * a.L + l) * 3;
#pragma unroll
                for (int c = 0; c < 3; ++c) pm[c] = acc[c][ct][v];
                continue;
            }
            const float *xm = a.XR + (m * a.L + l) * 3;
            float *gm = a.grad + (m * a.L + l) * 3;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double am = (double)xm[c] - a.cenR[3 * m + c];
                gm[c] = (float)(wfin[mm] * am - acc[c][ct][v]);
            }
        }
    }
}

// Sum of the split partials in split order, then (sum w) a_m - G.
__global__ __launch_bounds__(256) void grad_finish_kernel(GradLaunch a)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.NR * a.L) return;
    const int64_t m = t / a.L;
    double ws = 0.0, gs[3] = {0.0, 0.0, 0.0};
    for (int sp = 0; sp < a.nsplit; ++sp) {
        ws += a.wpart[(int64_t)sp * a.NR + m];
        const double *pm = a.part + ((int64_t)sp * a.NR * a.L + t) * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) gs[c] += pm[c];
    }
    const float *xm = a.XR + t * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        a.grad[t * 3 + c] = (float)(ws * ((double)xm[c] - a.cenR[3 * m + c]) - gs[c]);
}

__global__ void zero_kernel(float *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

int64_t grad_partners_padded(int64_t n) { return round_up(n, GBJ); }
int64_t grad_atoms_padded(int64_t L) { return round_up(L, 16); }

hipError_t launch_grad_planes(const float *X, const double *cen, float *P, int64_t N,
                              int64_t L, hipStream_t s)
{
    const int64_t Np = grad_partners_padded(N), Lp = grad_atoms_padded(L);
    grad_planes_kernel<<<dim3((unsigned)((Np * Lp + 255) / 256)), dim3(256), 0, s>>>(X, cen, P, N, Np,
                                                                                     L, Lp);
    return hipGetLastError();
}

// Partner blocks per split: enough splits to give every compute unit a
// workgroup when there are few row models (a reference against many), one
// split otherwise.  Depends on the shapes only, so the workspace size does.
GradSplit grad_split(int64_t NR, int64_t NC, int64_t L)
{
    const int64_t work = ((NR + GBM - 1) / GBM) * ((L + GLC - 1) / GLC);
    const int64_t nblk = (NC + GBJ - 1) / GBJ;
    int64_t want = 256 / (work > 0 ? work : 1);
    if (want < 1) want = 1;
    if (want > nblk) want = nblk > 0 ? nblk : 1;
    GradSplit g;
    g.bps = (int32_t)((nblk + want - 1) / want);
    if (g.bps < 1) g.bps = 1;
    g.nsplit = (int32_t)((nblk + g.bps - 1) / g.bps);
    if (g.nsplit < 1) g.nsplit = 1;
    return g;
}

size_t grad_partial_bytes(int64_t NR, int64_t NC, int64_t L)
{
    const GradSplit g = grad_split(NR, NC, L);
    if (g.nsplit <= 1) return 0;
    return sizeof(double) * (size_t)g.nsplit * (size_t)NR * (size_t)(3 * L + 1);
}

hipError_t launch_grad(const GradLaunch &a, hipStream_t s)
{
    if (a.NR <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.NR + GBM - 1) / GBM), (unsigned)((a.L + GLC - 1) / GLC),
                    (unsigned)a.nsplit);
    grad_kernel<<<grid, dim3(64 * GW), 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.nsplit <= 1) return e;
    grad_finish_kernel<<<dim3((unsigned)((a.NR * a.L + 255) / 256)), dim3(256), 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_zero(float *p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    zero_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(p, n);
    return hipGetLastError();
}

} // namespace clusco
