// Internal definitions shared by the gfx950 kernels and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/clusco.h"

namespace clusco {

// ---------------------------------------------------------------- layout
//
// The prep kernel writes centred coordinates in a fragment-native layout: for
// every block of 32 models (a "row block"), every K-block of atoms and every
// coordinate plane (x, y, z) there is one 1 KiB chunk holding exactly what the
// 64 lanes of a wave pass to one MFMA operand, lane-major.  A wave therefore
// loads an operand with one fully coalesced 16-byte-per-lane load, with no LDS
// staging and no swizzle in the contraction loop.  Both operands of the
// symmetric product Y Y^T use the same chunks.
//
//  FP32 (v_mfma_f32_32x32x2_f32, one value per lane per MFMA):
//      K-block = 8 atoms; lane l holds 4 floats = atoms 8kb + 4(l/32) + e,
//      e = 0..3, of model 32R + l%32.  Chunk index ((R*KB + kb)*3 + c).
//  SPLIT (v_mfma_f32_32x32x16_{bf16,f16}, 8 values per lane per MFMA):
//      K-block = 16 atoms; lane l holds 8 halves = atoms 16kb + 8(l/32) + e,
//      e = 0..7.  Chunk index (((R*KB + kb)*3 + c)*2 + part), part 0 = hi,
//      part 1 = lo.
//
// Rows are padded with zero models to a multiple of 64 (Np) and atoms with
// zeros to a multiple of the K-block (Lp).  Zero padding is exact because it
// is applied after centring and the scale 1/L uses the true L.

enum Mode { MODE_FP32 = 0, MODE_BF16 = 1, MODE_FP16 = 2, MODE_FP64 = 3 };

constexpr int ROWBLK = 32;   // models per MFMA row block
constexpr int TILE = 64;     // models per workgroup tile edge (2x2 waves)

__host__ __device__ constexpr int kblock(int mode) { return mode == MODE_FP32 ? 8 : 16; }

__host__ __device__ inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// packed upper-triangle index of (i, j), i < j
__host__ __device__ inline int64_t packed_index(int64_t i, int64_t j, int64_t N)
{
    return i * (2 * N - i - 1) / 2 + (j - i - 1);
}

// Row of the upper triangle (diagonal included) that holds linear tile t,
// for an nb x nb grid of tiles in row-major order.
__host__ __device__ inline void tri_decode(int64_t t, int64_t nb, int64_t *bi, int64_t *bj)
{
    double B = 2.0 * (double)nb + 1.0;
    int64_t r = (int64_t)((B - sqrt(B * B - 8.0 * (double)t)) * 0.5);
    if (r < 0) r = 0;
    if (r > nb - 1) r = nb - 1;
    // start(r) = r*nb - r(r-1)/2
    while (r > 0 && r * nb - r * (r - 1) / 2 > t) --r;
    while (r + 1 < nb && (r + 1) * nb - (r + 1) * r / 2 <= t) ++r;
    *bi = r;
    *bj = r + (t - (r * nb - r * (r - 1) / 2));
}

__host__ __device__ inline int64_t tri_count(int64_t nb) { return nb * (nb + 1) / 2; }

// Workspace of one forward call (byte offsets, all 256-aligned).
struct FwdLayout {
    int mode;
    int64_t N, L, Np, Lp, KB;
    int64_t nrb;          // row blocks of 32
    int64_t n_wave_tiles; // 32x32 blocks in the upper triangle (diagonal included)
    size_t off_counter, off_E, off_cen, off_ops, off_list, total;
};

inline FwdLayout fwd_layout(int mode, int64_t N, int64_t L)
{
    FwdLayout f{};
    f.mode = mode;
    f.N = N;
    f.L = L;
    f.Np = round_up(N > 0 ? N : 1, TILE);
    f.Lp = round_up(L, kblock(mode));
    f.KB = f.Lp / kblock(mode);
    f.nrb = f.Np / ROWBLK;
    f.n_wave_tiles = tri_count(f.nrb);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += (size_t)round_up((int64_t)bytes, 256); return r; };
    f.off_counter = take(256);
    f.off_E = take(sizeof(double) * f.Np);
    f.off_cen = take(sizeof(double) * 3 * f.Np);
    size_t op_bytes = 0;
    if (mode == MODE_FP32) op_bytes = sizeof(float) * 3 * f.Np * f.Lp;
    else if (mode == MODE_BF16 || mode == MODE_FP16) op_bytes = 2 * 2 * 3 * f.Np * f.Lp;
    f.off_ops = take(op_bytes);
    f.off_list = take(sizeof(uint32_t) * f.n_wave_tiles);
    f.total = o;
    return f;
}

// ----------------------------------------------------- launch interfaces

struct PrepArgs {
    const float *X;    // [N][L][3]
    int64_t N, L, Np, Lp, KB;
    void *ops;         // operand chunks (null in FP64 mode)
    double *E;         // [Np] sum_i |a_i|^2 of the operand values
    double *cen;       // [Np][3] centroids (FP64)
    int *counter;      // zeroed here (fix-up list length)
};

struct TileArgs {
    const void *ops;
    const double *E;
    int64_t N, L, Np, KB;
    int64_t nb;        // 64-model tile rows
    int64_t T;         // tiles in the triangle
    float *out;        // packed
    double flag_coef;  // a pair is flagged when score < flag_coef * (E_i + E_j); <= 0: never
    int *counter;
    uint32_t *list;
};

struct FixupArgs {
    const float *X;      // raw coordinates [N][L][3]
    const double *cen;   // [Np][3]
    const double *E;     // operand radii (flag re-evaluation only)
    int64_t N, L, nrb;
    float *out;
    double flag_coef;
    const int *counter;  // list length (null: every 32x32 block of the triangle)
    const uint32_t *list;
    int64_t n_all;       // number of 32x32 blocks when counter is null
};

hipError_t launch_prep(int mode, const PrepArgs &a, hipStream_t s);
hipError_t launch_tile(int mode, const TileArgs &a, hipStream_t s);
hipError_t launch_fixup(const FixupArgs &a, hipStream_t s);

} // namespace clusco
