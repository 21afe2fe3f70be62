// Gradient pass of the backward.  The pairs pass (tile kernel, OP_BWD) has
// stored, for every pair, w = g / (L cRMSD) and w Q, Q the adjoint of the
// pair's correlation (see eq2_adjoint).  Differentiating Eq. 2 (the optimum
// makes the derivative through the superposition vanish):
//     d cRMSD / d a_l = (a_l - Q b_l) / (L cRMSD),
//     d cRMSD / d b_l = (b_l - Q^T a_l) / (L cRMSD),
// so model m collects  (sum_j w_mj) a_m - sum_j Q~_mj a_j  with Q~ = Q when m
// is the pair's first model and Q^T when it is the second.  Both terms sum to
// zero over atoms (centred models), which is the centring Jacobian.
//
// One workgroup owns GM models and one thread one atom: each partner's
// centred coordinates are loaded once per workgroup and used for all GM
// models; the per-pair records are wave-uniform and come in through scalar
// loads.  Accumulation is FP64 in a fixed order (deterministic): the two
// terms nearly cancel when the partners surround the model (a reference
// against many noisy copies of itself), and FP64 FMA costs what FP32 FMA
// costs on this chip.
#include "internal.h"

namespace clusco {

constexpr int GM = 16;

__global__ __launch_bounds__(256) void grad_kernel(GradLaunch a)
{
    const int64_t m0 = (int64_t)blockIdx.x * GM;
    const int64_t NR = a.NR, NC = a.NC, L = a.L;
    for (int64_t l = threadIdx.x; l < L; l += blockDim.x) {
        double acc[GM][3], wsum[GM];
#pragma unroll
        for (int mm = 0; mm < GM; ++mm) {
            acc[mm][0] = acc[mm][1] = acc[mm][2] = 0.0;
            wsum[mm] = 0.0;
        }
        for (int64_t j = 0; j < NC; ++j) {
            const float *xj = a.XC + (j * L + l) * 3;
            const double b0 = (double)xj[0] - a.cenC[3 * j];
            const double b1 = (double)xj[1] - a.cenC[3 * j + 1];
            const double b2 = (double)xj[2] - a.cenC[3 * j + 2];
#pragma unroll
            for (int mm = 0; mm < GM; ++mm) {
                const int64_t m = m0 + mm;
                if (m >= NR || (a.kind == GK_SYM && m == j)) continue;
                bool tr;
                int64_t k;
                if (a.kind == GK_SYM) {
                    tr = m > j;
                    k = tr ? packed_index(j, m, NR) : packed_index(m, j, NR);
                } else if (a.kind == GK_CROSS_A) {
                    tr = false;
                    k = m * NC + j;
                } else {
                    tr = true;
                    k = j * NR + m;
                }
                const float *rk = a.wq + 12 * k;
                double r[10];
#pragma unroll
                for (int u = 0; u < 10; ++u) r[u] = (double)rk[u];
                wsum[mm] += r[9];
                if (!tr) {
                    acc[mm][0] += r[0] * b0 + r[1] * b1 + r[2] * b2;
                    acc[mm][1] += r[3] * b0 + r[4] * b1 + r[5] * b2;
                    acc[mm][2] += r[6] * b0 + r[7] * b1 + r[8] * b2;
                } else {
                    acc[mm][0] += r[0] * b0 + r[3] * b1 + r[6] * b2;
                    acc[mm][1] += r[1] * b0 + r[4] * b1 + r[7] * b2;
                    acc[mm][2] += r[2] * b0 + r[5] * b1 + r[8] * b2;
                }
            }
        }
#pragma unroll
        for (int mm = 0; mm < GM; ++mm) {
            const int64_t m = m0 + mm;
            if (m >= NR) continue;
            const float *xm = a.XR + (m * L + l) * 3;
            float *gm = a.grad + (m * L + l) * 3;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double am = (double)xm[c] - a.cenR[3 * m + c];
                gm[c] = (float)(wsum[mm] * am - acc[mm][c]);
            }
        }
    }
}

__global__ void zero_kernel(float *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

hipError_t launch_grad(const GradLaunch &a, hipStream_t s)
{
    if (a.NR <= 0) return hipSuccess;
    int64_t threads = round_up(a.L < 256 ? a.L : 256, 64);
    grad_kernel<<<dim3((unsigned)((a.NR + GM - 1) / GM)), dim3((unsigned)threads), 0, s>>>(a);
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
