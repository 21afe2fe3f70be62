// K-means over the packed score matrix with member centres (medoids), and
// the representative cluster by the smallest <R>/f (Implementation; Results
// and Discussion: K-means clustering of the similarity matrix and selection
// of the representative model).
//
// Alternating steps from distinct initial medoids, as many as max_iter
// updates, each a few launches on the caller's stream: a device state word
// records convergence and every later launch returns at once (the host may
// also poll it and stop enqueuing).
//
//  km_assign   one thread per model: nearest medoid by exact float32
//              comparison (ties to the lowest cluster, a medoid joins its own
//              cluster); clears the model's cost
//  km_cost     one pass over the packed matrix in 64x64 pair tiles: for every
//              pair in one cluster, q = rint(score 2^20) is added to both
//              models' costs; row sums stay in registers along a run of
//              tiles, column sums are combined in LDS, and both reach HBM
//              through 64-bit integer atomics.  Integer sums are exact, so the
//              result does not depend on the order of the atomics
//  km_update   one workgroup per cluster: the member of smallest cost (ties to
//              the lowest index) becomes the medoid; the last workgroup to
//              finish closes the iteration (converged when nothing changed)
//  km_stats    one workgroup per cluster: size and the exact sum of costs
//              (twice the in-cluster pair sum), <R> = sum / (n (n - 1))
//  km_pick     the cluster of smallest <R> N / n among those with a pair
#include "internal.h"

namespace clusco {

enum { ST_DONE = 0, ST_CHANGED = 1, ST_ITERS = 2, ST_CONVERGED = 3, ST_FINISHED = 4 };

__device__ __forceinline__ float score_at(const float *D, int64_t N, int64_t i, int64_t j)
{
    if (i > j) {
        const int64_t t = i;
        i = j;
        j = t;
    }
    return D[packed_index(i, j, N)];
}

__device__ __forceinline__ long long quant(float d)
{
    return (long long)rint((double)d * 1048576.0);
}

// final = 1: the assignment after the last update when max_iter ran out.
__global__ __launch_bounds__(256) void km_assign(ClusterLaunch a, int final)
{
    const int *st = a.state;
    if (final ? st[ST_CONVERGED] != 0 : st[ST_DONE] != 0) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    int best = -1;
    for (int c = 0; c < a.k; ++c)
        if (a.medoid[c] == i) {
            best = c;
            break;
        }
    if (best < 0) {
        float bd = 0.0f;
        for (int c = 0; c < a.k; ++c) {
            const float d = score_at(a.D, a.N, i, a.medoid[c]);
            if (best < 0 || d < bd) {
                best = c;
                bd = d;
            }
        }
    }
    a.label[i] = best;
    a.cost[i] = 0;
}


// Sum of v over the 64 lanes of a wave (every lane gets the total).
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int KT = 64;   // pair tile edge of the cost pass

// Each workgroup takes a contiguous run of 64x64 tiles in row-major order,
// so a wave streams 16 packed rows along consecutive column tiles.  A thread
// owns one column of the tile and keeps its share of the 16 row sums in
// registers while the tile row is unchanged; the wave reduces them and one
// 64-bit atomic per row reaches HBM when the run leaves the row.  Column sums
// are combined over the four waves in LDS, one atomic per column and tile.
// The next tile's 16 scores per thread are loaded while the current tile is
// summed, and the labels of a wave's 16 rows are loaded once per tile row, so
// a tile waits on no load of its own.  (Atomics across the XCDs are the
// expensive part of a scattered design: one per scattered pair instead of one
// per column and tile is several times slower.)
__device__ __forceinline__ void cost_tile_load(const ClusterLaunch &a, int N, int64_t bi, int64_t bj,
                                               int g, int lane, float (&d)[16], int &lj)
{
    const int j = (int)(bj * KT) + lane;
    const int i0 = (int)(bi * KT) + g * 16;
    lj = j < N ? a.label[j] : -1;
    // packed row starts advance by N - i - 2
    int64_t base = (int64_t)i0 * (2 * (int64_t)N - i0 - 1) / 2 - i0 - 1;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = i0 + r;
        d[r] = (i < j && j < N) ? a.D[base + j] : 0.0f;
        base += N - i - 2;
    }
}

__global__ __launch_bounds__(256) void km_cost(ClusterLaunch a, int final)
{
    const int *st = a.state;
    if (final ? st[ST_CONVERGED] != 0 : st[ST_DONE] != 0) return;
    __shared__ unsigned long long cols[4][KT];
    const int64_t nt = (a.N + KT - 1) / KT;
    const int64_t T = tri_count(nt);
    const int64_t t0 = T * blockIdx.x / gridDim.x, t1 = T * (blockIdx.x + 1) / gridDim.x;
    if (t0 >= t1) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63, g = tid >> 6;
    const int N = (int)a.N;                     // N <= 2^20: indices fit 32 bits
    unsigned long long racc[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) racc[r] = 0;
    int64_t bi, bj;
    tri_decode(t0, nt, &bi, &bj);
    float d[16];
    int lj, lab[16];
    cost_tile_load(a, N, bi, bj, g, lane, d, lj);
    auto row_labels = [&](int64_t b) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t i = b * KT + g * 16 + r;
            lab[r] = i < N ? a.label[i] : -2;
        }
    };
    auto row_flush = [&](int64_t b) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const unsigned long long v = wave_sum_u64(racc[r]);
            racc[r] = 0;
            if (lane == 0 && v != 0) atomicAdd((unsigned long long *)&a.cost[b * KT + g * 16 + r], v);
        }
    };
    row_labels(bi);
    for (int64_t t = t0; t < t1; ++t) {
        int64_t ni = bi, nj = bj + 1;
        if (nj == nt) {
            ni = bi + 1;
            nj = ni;
        }
        float dn[16];
        int ljn = -1;
        if (t + 1 < t1) cost_tile_load(a, N, ni, nj, g, lane, dn, ljn);
        const int j = (int)(bj * KT) + lane;
        const int i0 = (int)(bi * KT) + g * 16;
        unsigned long long cs = 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = i0 + r;
            const unsigned long long q =
                (i < j && j < N && lab[r] == lj) ? (unsigned long long)quant(d[r]) : 0ull;
            cs += q;
            racc[r] += q;
        }
        cols[g][lane] = cs;
        __syncthreads();
        if (tid < KT) {
            const unsigned long long c = cols[0][tid] + cols[1][tid] + cols[2][tid] + cols[3][tid];
            if (c != 0) atomicAdd((unsigned long long *)&a.cost[bj * KT + tid], c);
        }
        __syncthreads();
        if (t + 1 < t1) {
            if (ni != bi) {                     // next tile row: flush the row sums
                row_flush(bi);
                row_labels(ni);
            }
            bi = ni;
            bj = nj;
            lj = ljn;
#pragma unroll
            for (int r = 0; r < 16; ++r) d[r] = dn[r];
        }
    }
    row_flush(bi);
}

// Block-wide lexicographic minimum of (key, index) over 256 threads.
__device__ __forceinline__ void block_min(long long &key, int64_t &idx)
{
    __shared__ long long sk[256];
    __shared__ int64_t si[256];
    const int tid = threadIdx.x;
    sk[tid] = key;
    si[tid] = idx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            const long long k2 = sk[tid + s];
            const int64_t i2 = si[tid + s];
            if (i2 >= 0 && (si[tid] < 0 || k2 < sk[tid] || (k2 == sk[tid] && i2 < si[tid]))) {
                sk[tid] = k2;
                si[tid] = i2;
            }
        }
        __syncthreads();
    }
    key = sk[0];
    idx = si[0];
    __syncthreads();
}

// One workgroup per cluster; the last workgroup to finish also closes the
// iteration (counts it; converged when no medoid changed).
__global__ __launch_bounds__(256) void km_update(ClusterLaunch a)
{
    int *st = a.state;
    if (st[ST_DONE] != 0) return;
    const int c = blockIdx.x;
    long long key = 0;
    int64_t idx = -1;
    // eight models per thread and round, their loads independent of the
    // comparisons (a scan with one dependent load pair per model waited on
    // every one); ascending i within a thread: ties keep the first
    constexpr int U = 8;
    for (int64_t i0 = threadIdx.x; i0 < a.N; i0 += U * (int64_t)blockDim.x) {
        int lab[U];
        long long cost[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * (int64_t)blockDim.x;
            lab[u] = i < a.N ? a.label[i] : -1;
            cost[u] = i < a.N ? a.cost[i] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (lab[u] == c && (idx < 0 || cost[u] < key)) {
                key = cost[u];
                idx = i0 + u * (int64_t)blockDim.x;
            }
    }
    block_min(key, idx);
    if (threadIdx.x == 0) {
        if (idx >= 0 && idx != a.medoid[c]) {
            a.medoid[c] = (int)idx;
            atomicOr(&st[ST_CHANGED], 1);
        }
        __threadfence();
        if (atomicAdd(&st[ST_FINISHED], 1) == a.k - 1) {
            __threadfence();
            const int changed = atomicOr(&st[ST_CHANGED], 0);
            st[ST_ITERS] += 1;
            if (changed == 0) {
                st[ST_DONE] = 1;
                st[ST_CONVERGED] = 1;
            }
            st[ST_CHANGED] = 0;
            st[ST_FINISHED] = 0;
        }
    }
}

__global__ void km_clear(ClusterLaunch a)
{
    if (threadIdx.x < 8) a.state[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void km_stats(ClusterLaunch a)
{
    __shared__ long long sn[256], ss[256];
    const int c = blockIdx.x;
    long long n = 0, s = 0;
    for (int64_t i = threadIdx.x; i < a.N; i += blockDim.x)
        if (a.label[i] == c) {
            ++n;
            s += a.cost[i];
        }
    sn[threadIdx.x] = n;
    ss[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            sn[threadIdx.x] += sn[threadIdx.x + k];
            ss[threadIdx.x] += ss[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        n = sn[0];
        a.size[c] = n;
        a.mean_r[c] = n > 1 ? ((double)ss[0] / 1048576.0) / ((double)n * (double)(n - 1)) : 0.0;
    }
}

__global__ __launch_bounds__(256) void km_pick(ClusterLaunch a)
{
    __shared__ double sv[256];
    __shared__ int si[256];
    double best = 0.0;
    int bc = -1;
    for (int c = threadIdx.x; c < a.k; c += blockDim.x) {
        const long long n = a.size[c];
        if (n > 1) {
            const double v = a.mean_r[c] * ((double)a.N / (double)n);
            if (bc < 0 || v < best) {
                best = v;
                bc = c;
            }
        }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const int c2 = si[threadIdx.x + s];
            const double v2 = sv[threadIdx.x + s];
            if (c2 >= 0 && (si[threadIdx.x] < 0 || v2 < sv[threadIdx.x] ||
                            (v2 == sv[threadIdx.x] && c2 < si[threadIdx.x]))) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = c2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.info[0] = si[0];
        a.info[1] = a.state[ST_ITERS];
        a.info[2] = a.state[ST_CONVERGED];
    }
}

static dim3 cost_grid(const ClusterLaunch &a)
{
    const int64_t nt = (a.N + KT - 1) / KT;
    const int64_t tiles = tri_count(nt);
    return dim3((unsigned)(tiles < 4096 ? tiles : 4096));
}

hipError_t launch_cluster_begin(const ClusterLaunch &a, hipStream_t s)
{
    km_clear<<<1, 64, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_cluster_iters(const ClusterLaunch &a, int iters, hipStream_t s)
{
    const dim3 b(256), gn((unsigned)((a.N + 255) / 256)), gk((unsigned)a.k), gc = cost_grid(a);
    for (int it = 0; it < iters; ++it) {
        km_assign<<<gn, b, 0, s>>>(a, 0);
        km_cost<<<gc, b, 0, s>>>(a, 0);
        km_update<<<gk, b, 0, s>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_cluster_end(const ClusterLaunch &a, hipStream_t s)
{
    const dim3 b(256), gn((unsigned)((a.N + 255) / 256)), gk((unsigned)a.k), gc = cost_grid(a);
    km_assign<<<gn, b, 0, s>>>(a, 1);
    km_cost<<<gc, b, 0, s>>>(a, 1);
    km_stats<<<gk, b, 0, s>>>(a);
    km_pick<<<1, b, 0, s>>>(a);
    return hipGetLastError();
}

} // namespace clusco
