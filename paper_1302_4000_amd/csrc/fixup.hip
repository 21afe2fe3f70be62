// FP64 fix-up.  Pairs whose contraction error could exceed the tolerance are
// those with a small score relative to the models' radii: Eq. 2 subtracts
// 2(s1 + s2 + S s3) from R_A^2 + R_B^2, so an absolute error d in the
// correlation becomes an error of about d (E_A + E_B) / (L cRMSD) in cRMSD.
// The tile kernel lists every 32x32 block holding a pair whose stored score is
// below flag_coef (E_i + E_j); this kernel re-evaluates that test on the
// stored scores of each listed block, compacts the flagged pairs in LDS and
// recomputes each one from the raw float32 coordinates entirely in FP64
// (centring with the FP64 centroids, H and both radii accumulated in FP64,
// then the same Eq. 2 epilogue).  With no list (FP64 precision) every pair of
// every block is computed this way.
#include "eq2.h"
#include "internal.h"

namespace clusco {

__device__ __forceinline__ float pair_fp64(const float *X, const double *cen, int64_t L,
                                           int64_t i, int64_t j)
{
    const float *xi = X + i * L * 3, *xj = X + j * L * 3;
    const double ci0 = cen[3 * i], ci1 = cen[3 * i + 1], ci2 = cen[3 * i + 2];
    const double cj0 = cen[3 * j], cj1 = cen[3 * j + 1], cj2 = cen[3 * j + 2];
    double h[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double ea = 0.0, eb = 0.0;
    for (int64_t l = 0; l < L; ++l) {
        const double a0 = (double)xi[3 * l] - ci0, a1 = (double)xi[3 * l + 1] - ci1,
                     a2 = (double)xi[3 * l + 2] - ci2;
        const double b0 = (double)xj[3 * l] - cj0, b1 = (double)xj[3 * l + 1] - cj1,
                     b2 = (double)xj[3 * l + 2] - cj2;
        h[0] += a0 * b0; h[1] += a0 * b1; h[2] += a0 * b2;
        h[3] += a1 * b0; h[4] += a1 * b1; h[5] += a1 * b2;
        h[6] += a2 * b0; h[7] += a2 * b1; h[8] += a2 * b2;
        ea += a0 * a0 + a1 * a1 + a2 * a2;
        eb += b0 * b0 + b1 * b1 + b2 * b2;
    }
    const double lr2 = eq2_lrmsd2(h, ea, eb);
    return (float)sqrt(fmax(lr2 / (double)L, 0.0));
}

__global__ __launch_bounds__(64) void fixup_kernel(FixupArgs a)
{
    __shared__ uint16_t todo[ROWBLK * ROWBLK];
    __shared__ int cnt;
    const int lane = threadIdx.x;
    const int64_t N = a.N;
    const int64_t n = a.counter ? (int64_t)*a.counter : a.n_all;
    for (int64_t t = blockIdx.x; t < n; t += gridDim.x) {
        int64_t Ra, Rb;
        if (a.counter) {
            const uint32_t v = a.list[t];
            Ra = v >> 16;
            Rb = v & 0xFFFFu;
        } else {
            tri_decode(t, a.nrb, &Ra, &Rb);
        }
        if (lane == 0) cnt = 0;
        __syncthreads();
        for (int p = lane; p < ROWBLK * ROWBLK; p += 64) {
            const int64_t i = Ra * ROWBLK + (p >> 5), j = Rb * ROWBLK + (p & 31);
            if (i < j && j < N) {
                bool need = true;
                if (a.counter)
                    need = (double)a.out[packed_index(i, j, N)] < a.flag_coef * (a.E[i] + a.E[j]);
                if (need) todo[atomicAdd(&cnt, 1)] = (uint16_t)p;
            }
        }
        __syncthreads();
        const int m = cnt;
        for (int s = lane; s < m; s += 64) {
            const int p = todo[s];
            const int64_t i = Ra * ROWBLK + (p >> 5), j = Rb * ROWBLK + (p & 31);
            a.out[packed_index(i, j, N)] = pair_fp64(a.X, a.cen, a.L, i, j);
        }
        __syncthreads();
    }
}

hipError_t launch_fixup(const FixupArgs &a, hipStream_t s)
{
    int64_t grid = a.counter ? 2048 : (a.n_all < 65536 ? a.n_all : 65536);
    if (grid < 1) grid = 1;
    fixup_kernel<<<dim3((unsigned)grid), dim3(64), 0, s>>>(a);
    return hipGetLastError();
}

} // namespace clusco
