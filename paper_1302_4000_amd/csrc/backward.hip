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
// columns atoms l.  It runs on v_mfma_f32_16x16x4_f32 over blocks of 32
// partners (96 contraction terms, FP32 accumulation from zero), and each
// block's result is added to FP64 accumulators in block order
// (deterministic).  The FP64 fold matters: the two terms nearly cancel when
// the partners surround the model (a reference against many noisy copies of
// itself), so the running sum must not carry FP32 rounding of its full
// magnitude; a block's FP32 sum carries only that of 1/128 of it (N = 4096).
//
//  grad_planes  centred partner coordinates in the B fragment layout (atoms
//               padded with zeros to 16, partners to a multiple of 32): per
//               partner block and 16-atom tile, 16-byte chunks holding a
//               lane's values for four consecutive steps, lane-major, so a
//               wave fetches four steps of a fragment with one coalesced
//               load.  Contraction index k = 3j + d (partner j, coordinate d)
//  grad_kernel  one workgroup = 16 models x 256 atoms x a range of partner
//               blocks (the whole range unless few row models), 8 waves, each owning
//               two 16-atom column tiles and all three coordinate row tiles
//               (6 accumulators).  Per block of 32 partners the 512 pair
//               records (one per thread) are staged to LDS as the A operand,
//               the three coordinate rows of a (k, m) entry side by side so
//               that a lane reads its three fragments with one 16-byte load
//               (double-buffered, one barrier per block); B fragments come
//               straight from the planes into registers half a block ahead.
//               Each thread also sums the weights w of the pairs it stages.
//  grad_finish  with several partner ranges: FP64 partials summed in range
//               order (deterministic), then the gradient.
#include "internal.h"

#include <type_traits>

namespace clusco {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int GBM = 16;               // models per workgroup (one MFMA row tile per coordinate)
constexpr int GBJ = 32;               // partners per staged block
constexpr int GKB = 3 * GBJ;          // contraction length of one block
constexpr int GKS = GKB / 4;          // MFMA steps per block
constexpr int GW = 8;                 // waves per workgroup
constexpr int GCT = 2;                // 16-atom column tiles per wave
constexpr int GLC = 16 * GW * GCT;    // atoms per workgroup (256)
constexpr int GQ = GKS / 4;           // 16-byte B chunks per lane per block and atom tile
static_assert(GBM * GBJ == 64 * GW, "one pair record per thread per block");
static_assert(GKS % 8 == 0, "two halves of whole 16-byte chunks");

// One thread per 16-byte chunk: chunk (blk, t, q, lane) holds, for lane
// (g, i) = (lane / 16, lane % 16), the B fragment values of steps s = 4q + e,
// e = 0..3, of partner block blk and atom tile t: contraction row k = 4s + g
// (partner 32 blk + k / 3, coordinate k % 3), atom 16 t + i.
__global__ __launch_bounds__(256) void grad_planes_kernel(const float *X, const double *cen,
                                                          float4 *P, int64_t N, int64_t nblk,
                                                          int64_t L, int64_t NT)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nblk * NT * GQ * 64) return;
    const int lane = (int)(t & 63);
    const int q = (int)((t >> 6) % GQ);
    const int64_t tile = (t / (64 * GQ)) % NT;
    const int64_t blk = t / (64 * GQ * NT);
    const int g = lane >> 4;
    const int64_t l = 16 * tile + (lane & 15);
    float v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int k = 4 * (4 * q + e) + g;
        const int64_t j = blk * GBJ + k / 3;
        const int d = k % 3;
        v[e] = (j < N && l < L) ? (float)((double)X[(j * L + l) * 3 + d] - cen[3 * j + d]) : 0.0f;
    }
    P[t] = make_float4(v[0], v[1], v[2], v[3]);
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
    __shared__ float4 As[2][GKB * GBM];   // A operand: [k = 3 j + d][m] -> (c = 0, 1, 2, pad)
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

    // column tiles of this wave: the first nct are inside the padded atoms
    // (wave-uniform); the others load column 0 and skip their products, so
    // that every load is unconditional and the waits stay exact
    int64_t col[GCT], colc[GCT];
    int nct = 0;
#pragma unroll
    for (int ct = 0; ct < GCT; ++ct) {
        col[ct] = l0 + 16 * (w + GW * ct);
        const bool in = col[ct] < Lp;
        colc[ct] = in ? col[ct] : 0;
        nct += in ? 1 : 0;
    }
    const int g = lane >> 4, i16 = lane & 15;

    // staging: one pair per thread, thread t = (pair model m = t % 16,
    // partner j = t / 16); a wave covers 4 consecutive partners of all 16
    // models, so its loads are 16 runs of 4 consecutive records (or 4 runs
    // of 16 when the rows are the pairs' second models) and its LDS stores
    // are contiguous.  Missing pairs load record 0 and store zeros.
    const int sml = tid % GBM, sjl = tid / GBM;
    struct Staged {
        float4 r[3];
        bool ok, tr;
    };
    auto stage_load = [&](int blk, Staged &st) {
        int64_t k = 0;
        st.tr = false;
        st.ok = grad_pair(a, m0 + sml, (int64_t)blk * GBJ + sjl, &k, &st.tr);
        const float4 *p = (const float4 *)(a.wq + 12 * (st.ok ? k : 0));
        st.r[0] = p[0];
        st.r[1] = p[1];
        st.r[2] = p[2];
    };
    // row c of the A operand at contraction index (j, d) is Q~[c][d]
    auto stage_store = [&](int buf, const Staged &st, double &wsum) {
        float r[10];
        r[0] = st.r[0].x; r[1] = st.r[0].y; r[2] = st.r[0].z; r[3] = st.r[0].w;
        r[4] = st.r[1].x; r[5] = st.r[1].y; r[6] = st.r[1].z; r[7] = st.r[1].w;
        r[8] = st.r[2].x; r[9] = st.r[2].y;
        float4 *A = As[buf] + (3 * sjl) * GBM + sml;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            float q[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) q[c] = st.ok ? (st.tr ? r[3 * d + c] : r[3 * c + d]) : 0.0f;
            A[d * GBM] = make_float4(q[0], q[1], q[2], 0.0f);
        }
        wsum += st.ok ? (double)r[9] : 0.0;
    };
    // B fragments of half a block (GKH steps) into registers: GQ / 2
    // coalesced 16-byte loads per column tile
    constexpr int GKH = GKS / 2;
    const int64_t NT = Lp / 16;
    auto load_half = [&](int blk, int h, float4 (*bq)[GCT]) {
#pragma unroll
        for (int ct = 0; ct < GCT; ++ct) {
            const float4 *P = a.P + (((int64_t)blk * NT + colc[ct] / 16) * GQ + h * (GQ / 2)) * 64 + lane;
#pragma unroll
            for (int q = 0; q < GQ / 2; ++q) bq[q][ct] = P[q * 64];
        }
    };

    // FP32 block accumulators and the FP64 running sums they are folded into
    f32x4 acc[3][GCT];
    double sum[3][GCT][4];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int ct = 0; ct < GCT; ++ct) {
            acc[c][ct] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int v = 0; v < 4; ++v) sum[c][ct][v] = 0.0;
        }
    double wpart = 0.0;

    // the unrolled contraction over half a block for the first NT column tiles
    auto kloop = [&](const float4 *A, const float4 (*bq)[GCT], auto NT) {
#pragma unroll
        for (int s = 0; s < GKH; ++s) {
            const float4 q = A[(4 * s) * GBM];
            const float af[3] = {q.x, q.y, q.z};
#pragma unroll
            for (int ct = 0; ct < decltype(NT)::value; ++ct) {
                const float4 b4 = bq[s / 4][ct];
                const float bf = s % 4 == 0 ? b4.x : s % 4 == 1 ? b4.y : s % 4 == 2 ? b4.z : b4.w;
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    acc[c][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[c], bf, acc[c][ct], 0, 0, 0);
            }
        }
    };
    auto khalf = [&](const float4 *A, const float4 (*bq)[GCT]) {
        if (nct == GCT) kloop(A, bq, std::integral_constant<int, GCT>{});
        else if (nct == 1) kloop(A, bq, std::integral_constant<int, 1>{});
    };

    // two register halves in fixed roles: b0h holds the first half of the
    // current block (fetched during the previous block), b1h its second half
    float4 b0h[GQ / 2][GCT], b1h[GQ / 2][GCT];
    {
        Staged st;
        stage_load(b0, st);
        stage_store(0, st, wpart);
        load_half(b0, 0, b0h);
    }
    __syncthreads();

    for (int blk = b0; blk < b1; ++blk) {
        const int buf = (blk - b0) & 1;
        // prefetch the next block (the last block refetches itself: every
        // load stays unconditional; its staging buffer is not read again)
        const int nxt = blk + 1 < b1 ? blk + 1 : blk;
        // second-half fragments first: waits on them then never wait on the
        // (older) record loads as well
        load_half(blk, 1, b1h);
        Staged st;
        stage_load(nxt, st);
        const float4 *A = As[buf] + g * GBM + i16;
        khalf(A, b0h);
        load_half(nxt, 0, b0h);
        khalf(A + 4 * GKH * GBM, b1h);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int ct = 0; ct < GCT; ++ct) {
#pragma unroll
                for (int v = 0; v < 4; ++v) sum[c][ct][v] += (double)acc[c][ct][v];
                acc[c][ct] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
            }
        double wdummy = 0.0;
        stage_store(buf ^ 1, st, blk + 1 < b1 ? wpart : wdummy);
        __syncthreads();
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

    // epilogue: accumulator element v of a lane is G row (c, m = 4 (lane / 16) + v),
    // column l = col + lane % 16 (the f32 16x16x4 output layout).  With one
    // split the gradient is finished here; otherwise this split's weight sums
    // and G go to FP64 partials that grad_finish adds in split order.
    if (a.nsplit > 1 && tid < GBM && m0 + tid < a.NR)
        a.wpart[(int64_t)split * a.NR + m0 + tid] = wfin[tid];
#pragma unroll
    for (int ct = 0; ct < GCT; ++ct) {
        if (ct >= nct) continue;
        const int64_t l = col[ct] + i16;
        if (l >= a.L) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int mm = 4 * g + v;
            const int64_t m = m0 + mm;
            if (m >= a.NR) continue;
            if (a.nsplit > 1) {
                double *pm = a.part + (((int64_t)split * a.NR + m) * a.L + l) * 3;
#pragma unroll
                for (int c = 0; c < 3; ++c) pm[c] = sum[c][ct][v];
                continue;
            }
            const float *xm = a.XR + (m * a.L + l) * 3;
            float *gm = a.grad + (m * a.L + l) * 3;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double am = (double)xm[c] - a.cenR[3 * m + c];
                gm[c] = (float)(wfin[mm] * am - sum[c][ct][v]);
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
#pragma unroll 4
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
    const int64_t nblk = grad_partners_padded(N) / GBJ, NT = grad_atoms_padded(L) / 16;
    const int64_t chunks = nblk * NT * GQ * 64;
    grad_planes_kernel<<<dim3((unsigned)((chunks + 255) / 256)), dim3(256), 0, s>>>(
        X, cen, (float4 *)P, N, nblk, L, NT);
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
