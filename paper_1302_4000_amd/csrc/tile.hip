// Fused covariance contraction + Eq. 2 epilogue + packed store.
//
// The nine correlations H_cd[i][j] = sum_l X_c[i][l] X_d[j][l] of every pair
// of models (c, d in {x, y, z}) are the blocks of the symmetric product
// Y Y^T, Y = the centred coordinate planes.  One workgroup owns a 64x64 tile
// of model pairs in the upper triangle (tile rows <= tile columns); each of
// its four waves owns a 32x32 sub-tile and keeps nine MFMA accumulator sets,
// one per (c, d), so all nine entries of a pair's H sit in the same lane and
// register slot.  After the K loop each lane runs the FP64 Eq. 2 epilogue on
// its 16 pairs and stores them; for a fixed register slot the 64 lanes write
// two 128-byte runs of the packed row (consecutive j), so stores coalesce.
//
// Blocks are remapped so that each XCD (workgroups are dealt round-robin to
// the 8 XCDs) receives a contiguous range of tiles, which share operand rows
// in that XCD's L2.
#include "eq2.h"
#include "internal.h"

namespace clusco {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int MODE>
__device__ __forceinline__ f32x16 mfma_split(u32x4 a, u32x4 b, f32x16 c)
{
    if constexpr (MODE == MODE_BF16)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

// Contraction of one 32x32 wave tile: acc[3c+d] += X_c[Ra rows] X_d[Rb rows]^T
template <int MODE>
__device__ __forceinline__ void contract(const void *ops, int64_t Ra, int64_t Rb, int64_t KB,
                                         int lane, f32x16 acc[9])
{
    if constexpr (MODE == MODE_FP32) {
        const f32x4 *pa = (const f32x4 *)ops + Ra * KB * 3 * 64 + lane;
        const f32x4 *pb = (const f32x4 *)ops + Rb * KB * 3 * 64 + lane;
        f32x4 A[3], B[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            A[c] = pa[c * 64];
            B[c] = pb[c * 64];
        }
        for (int64_t kb = 0; kb < KB; ++kb) {
            f32x4 An[3], Bn[3];
            const bool more = kb + 1 < KB;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (more) {
                    An[c] = pa[((kb + 1) * 3 + c) * 64];
                    Bn[c] = pb[((kb + 1) * 3 + c) * 64];
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        acc[3 * c + d] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                            A[c][e], B[d][e], acc[3 * c + d], 0, 0, 0);
            if (more) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    A[c] = An[c];
                    B[c] = Bn[c];
                }
            }
        }
    } else {
        // chunk (kb, c, part) of row block R at ((R*KB + kb)*3 + c)*2 + part
        const u32x4 *pa = (const u32x4 *)ops + Ra * KB * 6 * 64 + lane;
        const u32x4 *pb = (const u32x4 *)ops + Rb * KB * 6 * 64 + lane;
        u32x4 A[6], B[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            A[q] = pa[q * 64];
            B[q] = pb[q * 64];
        }
        for (int64_t kb = 0; kb < KB; ++kb) {
            u32x4 An[6], Bn[6];
            const bool more = kb + 1 < KB;
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                if (more) {
                    An[q] = pa[((kb + 1) * 6 + q) * 64];
                    Bn[q] = pb[((kb + 1) * 6 + q) * 64];
                }
            }
            // hi*hi', then hi*lo', then lo*hi': each accumulator is touched
            // once per group of nine, so back-to-back MFMAs are independent
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    acc[3 * c + d] = mfma_split<MODE>(A[2 * c], B[2 * d], acc[3 * c + d]);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    acc[3 * c + d] = mfma_split<MODE>(A[2 * c], B[2 * d + 1], acc[3 * c + d]);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    acc[3 * c + d] = mfma_split<MODE>(A[2 * c + 1], B[2 * d], acc[3 * c + d]);
            if (more) {
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    A[q] = An[q];
                    B[q] = Bn[q];
                }
            }
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(256) void tile_kernel(TileArgs a)
{
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t per_xcd = gridDim.x >> 3;
    const int64_t t = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (t >= a.T) return;
    int64_t bi, bj;
    tri_decode(t, a.nb, &bi, &bj);
    const int wy = w >> 1, wx = w & 1;
    if (bi == bj && wy > wx) return;           // sub-tile entirely below the diagonal
    const int64_t Ra = 2 * bi + wy, Rb = 2 * bj + wx;
    const int64_t N = a.N;
    if (Ra * ROWBLK >= N || Rb * ROWBLK >= N) return;   // padding only

    f32x16 acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;

    contract<MODE>(a.ops, Ra, Rb, a.KB, lane, acc);

    // epilogue: lane holds column j = lane%32 and rows 8(r/4) + 4(lane/32) + r%4
    const double invL = 1.0 / (double)a.L;
    const int64_t j = Rb * ROWBLK + (lane & 31);
    const double Ej = a.E[j];
    bool flagged = false;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t i = Ra * ROWBLK + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (i < j && j < N) {
            double h[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) h[q] = (double)acc[q][r];
            const double Ei = a.E[i];
            const double lr2 = eq2_lrmsd2(h, Ei, Ej);
            const float v = sqrtf((float)fmax(lr2 * invL, 0.0));
            a.out[packed_index(i, j, N)] = v;
            flagged |= (double)v < a.flag_coef * (Ei + Ej);
        }
    }
    if (__any(flagged) && lane == 0) {
        const int s = atomicAdd(a.counter, 1);
        a.list[s] = ((uint32_t)Ra << 16) | (uint32_t)Rb;
    }
}

hipError_t launch_tile(int mode, const TileArgs &a, hipStream_t s)
{
    const int64_t grid = round_up(a.T, 8);
    dim3 g((unsigned)grid), b(256);
    switch (mode) {
    case MODE_FP32: tile_kernel<MODE_FP32><<<g, b, 0, s>>>(a); break;
    case MODE_BF16: tile_kernel<MODE_BF16><<<g, b, 0, s>>>(a); break;
    case MODE_FP16: tile_kernel<MODE_FP16><<<g, b, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace clusco
