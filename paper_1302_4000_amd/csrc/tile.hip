// Fused covariance contraction + Eq. 2 epilogue + coalesced store.
//
// The nine correlations H_cd[i][j] = sum_l X_c[i][l] X_d[j][l] of every pair
// of models (c, d in {x, y, z}) are the blocks of the product Y_A Y_B^T,
// Y = the centred coordinate planes.  One workgroup owns a 64x64 tile of
// model pairs; each of its four waves owns a 32x32 sub-tile and keeps nine
// MFMA accumulator sets, one per (c, d), so all nine entries of a pair's H
// sit in the same lane and register slot.  After the K loop each lane runs
// the FP64 Eq. 2 epilogue on its 16 pairs and stores them; for a fixed
// register slot the 64 lanes write two 128-byte runs of consecutive j, so
// stores coalesce in both the packed and the dense output.
//
// Launch kinds:
//  TK_SYM    one all-vs-all ensemble; tiles of the upper triangle only (the
//            wave below the diagonal of a diagonal tile idles);
//  TK_RECT   one cross comparison, every tile of the NA x NB grid;
//  TK_BATCH  many all-vs-all ensembles in one launch.
// Two schedules, chosen per problem bucket by the tuning table: the staged
// kernel (one tile per 4-wave workgroup, operands staged in LDS; see
// staged_kernel) and the persistent ping-pong kernel (see tile_kernel).
// The order of tiles within a problem is banded (band_decode) with the
// problem's band width: a band's column sweep re-reads the column operands
// once per band, so wider bands fetch less until the band's row operands and
// the columns in flight outgrow the XCD's 4 MB L2 (at N = 20,000, L = 150,
// split-BF16: 8 rows fetched 0.77 GB per launch, 16 rows 0.44 GB).
#include "eq2.h"
#include "internal.h"

namespace clusco {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Keeps the compiler from sinking the next K-block's loads down to their
// first use, which would expose the full L2 latency on every K-block.
__device__ __forceinline__ void pin_order() { asm volatile("" ::: "memory"); }

template <int MODE>
__device__ __forceinline__ f32x16 mfma_split(u32x4 a, u32x4 b, f32x16 c)
{
    if constexpr (is_bf16(MODE))
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

// Contraction of one 32x32 wave tile: acc[3c+d] += X_c[Ra rows] X_d[Rb rows]^T
template <int MODE>
__device__ __forceinline__ void contract(const char *opsA, const char *opsB, int64_t Ra,
                                         int64_t Rb, int64_t KB, int lane, f32x16 acc[9])
{
    constexpr bool lolo = MODE == MODE_BF16X4;   // the fourth product lo*lo'
    if constexpr (MODE == MODE_FP32) {
        const f32x4 *pa = (const f32x4 *)opsA + Ra * KB * 3 * 64 + lane;
        const f32x4 *pb = (const f32x4 *)opsB + Rb * KB * 3 * 64 + lane;
        f32x4 A[3], B[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            A[c] = pa[c * 64];
            B[c] = pb[c * 64];
        }
        // the next K-block is always fetched (the last step re-reads its own
        // block) so the loop body has no branches
        for (int64_t kb = 0; kb < KB; ++kb) {
            const int64_t nx = (kb + 1 < KB ? kb + 1 : kb) * 3 * 64;
            f32x4 An[3], Bn[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                An[c] = pa[nx + c * 64];
                Bn[c] = pb[nx + c * 64];
            }
            pin_order();
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        acc[3 * c + d] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                            A[c][e], B[d][e], acc[3 * c + d], 0, 0, 0);
            pin_order();
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                A[c] = An[c];
                B[c] = Bn[c];
            }
        }
    } else {
        // chunk (kb, c, part) of row block R at ((R*KB + kb)*3 + c)*2 + part.
        // Only the hi parts are prefetched a whole K-block ahead; each lo part
        // is reloaded as soon as the last MFMA group reading it has issued,
        // which keeps the wave within 256 registers (two waves per SIMD).  The
        // last step re-reads its own block so the loop body has no branches.
        const u32x4 *pa = (const u32x4 *)opsA + Ra * KB * 6 * 64 + lane;
        const u32x4 *pb = (const u32x4 *)opsB + Rb * KB * 6 * 64 + lane;
        u32x4 Ah[3], Al[3], Bh[3], Bl[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Ah[c] = pa[(2 * c) * 64];
            Al[c] = pa[(2 * c + 1) * 64];
            Bh[c] = pb[(2 * c) * 64];
            Bl[c] = pb[(2 * c + 1) * 64];
        }
        for (int64_t kb = 0; kb < KB; ++kb) {
            const int64_t nx = (kb + 1 < KB ? kb + 1 : kb) * 6 * 64;
            u32x4 Ahn[3], Bhn[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Ahn[c] = pa[nx + (2 * c) * 64];
                Bhn[c] = pb[nx + (2 * c) * 64];
            }
            pin_order();
            // hi*hi', then hi*lo', then lo*hi': each accumulator is touched
            // once per group of nine, so back-to-back MFMAs are independent
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    acc[3 * c + d] = mfma_split<MODE>(Ah[c], Bh[d], acc[3 * c + d]);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    acc[3 * c + d] = mfma_split<MODE>(Ah[c], Bl[d], acc[3 * c + d]);
            if constexpr (lolo) {
                // fourth product lo*lo': the split then carries no dropped term
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        acc[3 * c + d] = mfma_split<MODE>(Al[c], Bl[d], acc[3 * c + d]);
            }
            pin_order();
#pragma unroll
            for (int d = 0; d < 3; ++d) Bl[d] = pb[nx + (2 * d + 1) * 64];
            pin_order();
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    acc[3 * c + d] = mfma_split<MODE>(Al[c], Bh[d], acc[3 * c + d]);
            pin_order();
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Al[c] = pa[nx + (2 * c + 1) * 64];
                Ah[c] = Ahn[c];
                Bh[c] = Bhn[c];
            }
            pin_order();
        }
    }
}

// Forward epilogue: one pair at a time per lane (two or four side by side
// measured no faster) and EPI_STEPS Newton steps on the largest root before
// the rare-lane continuation of eq2_largest_root.
#ifndef EPI_STEPS
#define EPI_STEPS 3
#endif

// A wave's share of one 64x64 tile: its 32x32 block and the problem.
struct WaveJob {
    int64_t Ra, Rb;
    int32_t pidx;
    int32_t active;
};

template <int KIND>
__device__ __forceinline__ const Problem &problem_of(const TileLaunch &a, int32_t pidx)
{
    if constexpr (KIND == TK_BATCH) return a.table[pidx];
    else return a.prob;
}

// Wave w's quarter of launch tile t (inactive past the end, below the
// diagonal of a diagonal tile, or entirely in padding).
template <int KIND>
__device__ __forceinline__ WaveJob decode_job(const TileLaunch &a, int64_t t, int w)
{
    WaveJob job{0, 0, 0, 0};
    if (t >= a.T) return job;
    int64_t bi, bj;
    int32_t e = 0;
    if constexpr (KIND == TK_BATCH) {
        const int64_t tg = a.t0 + t;
        e = table_find(a.table, a.nprob, tg, [](const Problem &q) { return q.tile0; });
        band_decode(tg - a.table[e].tile0, a.table[e].nbA, a.table[e].band, &bi, &bj);
    } else if constexpr (KIND == TK_SYM) {
        band_decode(t, a.prob.nbA, a.prob.band, &bi, &bj);
    } else {
        band_decode_rect(t, a.prob.nbA, a.prob.nbB, a.prob.band, &bi, &bj);
    }
    const Problem &p = problem_of<KIND>(a, e);
    const int wy = w >> 1, wx = w & 1;
    job.Ra = 2 * bi + wy;
    job.Rb = 2 * bj + wx;
    job.pidx = e;
    job.active = !(p.sym && bi == bj && wy > wx) && job.Ra * ROWBLK < p.NA &&
                 job.Rb * ROWBLK < p.NB;
    return job;
}

// The per-model values a wave's epilogue needs, loaded once (not once per
// pair, which would put a dependent memory round trip in front of every
// pair): the radius E and the flag weight F of the lane's column
// j = Rb*32 + lane%32, and of row Ra*32 + lane%32, from which each pair takes
// its row's values with a cross-lane shuffle.
struct EpiRadii {
    double ej, erow;
    float fj, frow;
};

__device__ __forceinline__ EpiRadii epi_radii(const TileLaunch &a, const Problem &p,
                                              const WaveJob &job, int lane)
{
    const double *EA = (const double *)(a.ws + p.EA);
    const double *EB = (const double *)(a.ws + p.EB);
    const double *FA = (const double *)(a.ws + p.FA);
    const double *FB = (const double *)(a.ws + p.FB);
    const int64_t j = job.Rb * ROWBLK + (lane & 31), i = job.Ra * ROWBLK + (lane & 31);
    return EpiRadii{EB[j], EA[i], (float)FB[j], (float)FA[i]};
}

// E of row Ra*32 + r (r < 32) from the lane that loaded it.
__device__ __forceinline__ double row_radius(const EpiRadii &er, int r)
{
    return __shfl(er.erow, r, 64);
}

// F of row Ra*32 + r (rounded to float: the flag test is flag_pair).
__device__ __forceinline__ float row_flag(const EpiRadii &er, int r)
{
    return __shfl(er.frow, r, 64);
}

// Correlation of the pair in accumulator slot r, in FP64: the contraction's
// value, plus in the reference frame U of the row (urow: its 9 values) and
// P^T of the column (pcol: its 9 values), in that order in every kernel.
template <bool FRAME>
__device__ __forceinline__ void pair_h(const f32x16 acc[9], int r, const double *urow,
                                       const double *pcol, double h[9])
{
#pragma unroll
    for (int u = 0; u < 9; ++u) {
        h[u] = (double)acc[u][r];
        if constexpr (FRAME) h[u] = (h[u] + urow[u]) + pcol[u];
    }
}

// The column's frame terms (P^T of column j = lane%32), read once and held
// in registers for the block's sixteen pairs (the empty asm stops the
// compiler from re-reading them per pair).
template <bool FRAME>
__device__ __forceinline__ void col_terms(const double *pcol, int lane, double (&pc)[9])
{
#pragma unroll
    for (int u = 0; u < 9; ++u) pc[u] = FRAME ? pcol[9 * (lane & 31) + u] : 0.0;
    if constexpr (FRAME) {
#pragma unroll
        for (int u = 0; u < 9; ++u) asm volatile("" : "+v"(pc[u]));
    }
}

// Row terms of the pair in accumulator slot k (row 8(k/4) + 4(lane/32) +
// k%4 of the block): U from LDS, E and F from the lane that loaded them.
// The epilogues request them one pair ahead, between the current pair's
// root and its square roots, so that their LDS latency is hidden.
template <bool FRAME>
__device__ __forceinline__ void row_terms(const double *urow, const EpiRadii &er, int lane, int k,
                                          double (&u)[9], double &e, float &f)
{
    const int rr = 8 * (k >> 2) + 4 * (lane >> 5) + (k & 3);
    if constexpr (FRAME) {
#pragma unroll
        for (int t = 0; t < 9; ++t) u[t] = urow[9 * rr + t];
    }
    e = row_radius(er, rr);
    f = row_flag(er, rr);
}

// Where the epilogue finds the reference-frame terms of its wave's block: U
// of its 32 rows and P^T of its 32 columns, 9 doubles per model (in LDS for
// the staged kernel, in the workspace for the persistent one).
struct FrameTerms {
    const double *urow, *pcol;
};

// FP64 Eq. 2 epilogue and store of one wave's 32x32 block.  The lane holds
// column j = lane%32 and rows 8(r/4) + 4(lane/32) + r%4 of accumulator slot r.
// Every slot is evaluated (padding rows and columns have H = 0 and E = 0,
// which is finite); only the store and the flag are predicated, so the FP64
// work runs without divergent branches.  urow: the U values of the wave's 32
// rows (reference frame).  A pair is listed for the FP64 fix-up when its
// score is below F_i + F_j and the problem runs the fix-up.
template <bool FRAME, bool SYM>
__device__ __forceinline__ void epilogue_t(const TileLaunch &a, const Problem &p,
                                           const WaveJob &job, int lane, const f32x16 acc[9],
                                           const EpiRadii &er, const FrameTerms &ft)
{
    const int64_t NA = p.NA, NB = p.NB;
    float *out = a.out + p.out;
    const double invL = 1.0 / (double)p.L;
    const bool fix = p.flag_coef > 0.0;
    const int64_t j = job.Rb * ROWBLK + (lane & 31);
    const double Ej = er.ej;
    const float Fj = er.fj;
    const bool jlive = j < (SYM ? NA : NB);
    double pc[9];
    col_terms<FRAME>(ft.pcol, lane, pc);
    double ur[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, ei;
    float fi;
    row_terms<FRAME>(ft.urow, er, lane, 0, ur, ei, fi);
    // the flag is folded in pair by pair into a wave-wide mask (scalar ALU):
    // the empty asm keeps the compiler from deferring all sixteen comparisons
    // to the end of the block, which would hold every score and row weight in
    // registers until then
    uint64_t flagged = 0;
    int64_t base = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int64_t i = job.Ra * ROWBLK + 8 * (k >> 2) + 4 * (lane >> 5) + (k & 3);
        // row base k(i, j) - j: packed rows advance by N - i - 2, dense by NB
        if ((k & 3) == 0) base = SYM ? i * (2 * NA - i - 1) / 2 - i - 1 : i * NB;
        double h[1][9], eiv[1] = {ei}, ejv[1] = {Ej}, lr2[1];
        const float fcur = fi;
        pair_h<FRAME>(acc, k, ur, pc, h[0]);
        Eq2Roots<1> st;
        eq2_roots_batch<1, EPI_STEPS>(h, st);
        if (k + 1 < 16) {
            __builtin_amdgcn_sched_barrier(0);
            row_terms<FRAME>(ft.urow, er, lane, k + 1, ur, ei, fi);
            __builtin_amdgcn_sched_barrier(0);
        }
        eq2_finish_batch<1>(st, eiv, ejv, lr2);
        // hardware square root (within 1 ulp): the score's tolerance is
        // orders of magnitude above float rounding
        const float v = __builtin_amdgcn_sqrtf((float)fmax(lr2[0] * invL, 0.0));
        const bool live = jlive && (SYM ? i < j : i < NA);
        if (live) out[base + j] = v;
        flagged |= __ballot(fix && live && flag_pair(v, fcur, Fj));
        asm volatile("" : "+s"(flagged));
        // the next row's base, kept incremental (the empty asm stops the
        // compiler from re-deriving it with a multiplication)
        base += SYM ? NA - i - 2 : NB;
        asm volatile("" : "+v"(base));
    }
    if (flagged != 0 && lane == 0) {
        const int s = atomicAdd(&a.counters[0], 1);
        a.list[s] = FixEntry{(uint32_t)job.pidx, ((uint32_t)job.Ra << 16) | (uint32_t)job.Rb};
    }
}

// SYM: the problem is one ensemble against itself (packed upper triangle);
// else a cross comparison (dense NA x NB).
template <bool SYM>
__device__ __forceinline__ void epilogue(const TileLaunch &a, const Problem &p,
                                         const WaveJob &job, int lane, const f32x16 acc[9],
                                         const EpiRadii &er, const FrameTerms &ft)
{
    if (p.frame) epilogue_t<true, SYM>(a, p, job, lane, acc, er, ft);
    else epilogue_t<false, SYM>(a, p, job, lane, acc, er, ft);
}

// Backward epilogue: per live pair, w = g / (L cRMSD) (0 where the score
// is 0 to within 1e-5 of the pair's mean radius, where cRMSD is not
// differentiable) and the adjoint Q of the pair's H; writes [w Q, w, 0, 0].
__device__ __forceinline__ void bwd_epilogue(const TileLaunch &a, const Problem &p,
                                             const WaveJob &job, int lane, const f32x16 acc[9],
                                             const EpiRadii &er)
{
    const int64_t NA = p.NA, NB = p.NB;
    const double L = (double)p.L;
    const int64_t j = job.Rb * ROWBLK + (lane & 31);
    const double Ej = er.ej;
    const bool jlive = j < (p.sym ? NA : NB);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int64_t i0 = job.Ra * ROWBLK + 8 * g + 4 * (lane >> 5);
        int64_t base = p.sym ? i0 * (2 * NA - i0 - 1) / 2 - i0 - 1 : i0 * NB;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 4 * g + q;
            const int64_t i = i0 + q;
            const bool live = jlive && (p.sym ? i < j : i < NA);
            if (live) {
                const int64_t k = base + j;
                const double sc = (double)a.rmsd[k], gk = (double)a.gout[k];
                const double floor_r = 1e-5 * sqrt((row_radius(er, 8 * g + 4 * (lane >> 5) + q) + Ej) / (2.0 * L));
                const double w = (gk != 0.0 && sc > floor_r) ? gk / (L * sc) : 0.0;
                float rec[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
                if (w != 0.0) {
                    double h[9], qm[9];
#pragma unroll
                    for (int u = 0; u < 9; ++u) h[u] = (double)acc[u][r];
                    eq2_adjoint(h, qm);
#pragma unroll
                    for (int u = 0; u < 9; ++u) rec[u] = (float)(w * qm[u]);
                    rec[9] = (float)w;
                }
                f32x4 *dst = (f32x4 *)(a.wq + 12 * k);
                dst[0] = f32x4{rec[0], rec[1], rec[2], rec[3]};
                dst[1] = f32x4{rec[4], rec[5], rec[6], rec[7]};
                dst[2] = f32x4{rec[8], rec[9], rec[10], rec[11]};
            }
            base += p.sym ? NA - i - 2 : NB;
        }
    }
}

// Number of lanes below this one whose bit is set in the wave-wide mask b.
__device__ __forceinline__ uint32_t lanes_below(unsigned long long b)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
}

// Threshold epilogue: scores as in the forward epilogue, but instead of the
// packed store, pairs below the cutoff are appended to the output arrays
// (one atomic for the whole 32x32 block, or for the workgroup's four blocks
// in the staged kernel, then each lane writes at its prefix position).  Pairs
// the fix-up will recompute are not emitted here; their bits go into the
// block's ownership mask with the list entry.  thr_scores does everything up
// to the count of the wave's pairs to emit; thr_write appends them at base.
struct ThrPairs {
    float vs[16];
    uint32_t emit;
    uint32_t total;   // pairs of the wave to emit
};

template <bool FRAME>
__device__ __forceinline__ void thr_scores_t(const TileLaunch &a, const Problem &p,
                                             const WaveJob &job, int lane, const f32x16 acc[9],
                                             const EpiRadii &er, const FrameTerms &ft,
                                             ThrPairs &tp)
{
    const int64_t NA = p.NA;
    const double invL = 1.0 / (double)p.L;
    const bool fix = p.flag_coef > 0.0;
    const float cutoff = (float)a.emit.cutoff;
    const int64_t j = job.Rb * ROWBLK + (lane & 31);
    const double Ej = er.ej;
    const float Fj = er.fj;
    const bool jlive = j < NA;
    // Column and row terms are read from LDS per pair: the sixteen scores
    // are held to the end here, and neither the column terms held in
    // registers nor a row-term prefetch fit beside them without spills.
    const double *pcol = ft.pcol + 9 * (lane & 31);
    uint32_t emit = 0, flag = 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t i = job.Ra * ROWBLK + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int rr = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        double h[1][9], eiv[1] = {row_radius(er, rr)}, ejv[1] = {Ej}, lr2[1];
        pair_h<FRAME>(acc, r, ft.urow + 9 * rr, pcol, h[0]);
        eq2_lrmsd2_batch<1, EPI_STEPS>(h, eiv, ejv, lr2);   // the forward's arithmetic
        const float v = __builtin_amdgcn_sqrtf((float)fmax(lr2[0] * invL, 0.0));
        const bool live = jlive && i < j;
        const bool fl = fix && live && flag_pair(v, row_flag(er, rr), Fj);
        tp.vs[r] = v;
        flag |= (uint32_t)fl << r;
        emit |= (uint32_t)(live && !fl && v < cutoff) << r;
    }
    if (__any(flag != 0)) {
        int s = 0;
        if (lane == 0) {
            s = atomicAdd(&a.counters[0], 1);
            a.list[s] = FixEntry{(uint32_t)job.pidx, ((uint32_t)job.Ra << 16) | (uint32_t)job.Rb};
        }
        s = __shfl(s, 0, 64);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const unsigned long long b = __ballot((flag >> r) & 1u);
            const int row = 8 * (r >> 2) + (r & 3);
            if (lane == 0) {
                a.emit.masks[32 * s + row] = (uint32_t)b;
                a.emit.masks[32 * s + row + 4] = (uint32_t)(b >> 32);
            }
        }
    }
    uint32_t total = 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) total += (uint32_t)__popcll(__ballot((emit >> r) & 1u));
    tp.emit = emit;
    tp.total = total;
}

__device__ __forceinline__ void thr_scores(const TileLaunch &a, const Problem &p, const WaveJob &job,
                                           int lane, const f32x16 acc[9], const EpiRadii &er,
                                           const FrameTerms &ft, ThrPairs &tp)
{
    if (p.frame) thr_scores_t<true>(a, p, job, lane, acc, er, ft, tp);
    else thr_scores_t<false>(a, p, job, lane, acc, er, ft, tp);
}

__device__ __forceinline__ void thr_write(const TileLaunch &a, const WaveJob &job, int lane,
                                          const ThrPairs &tp, unsigned long long base)
{
    const int64_t j = job.Rb * ROWBLK + (lane & 31);
    unsigned long long off = 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const unsigned long long b = __ballot((tp.emit >> r) & 1u);
        if ((tp.emit >> r) & 1u) {
            const unsigned long long pos = base + off + lanes_below(b);
            if (pos < (unsigned long long)a.emit.capacity) {
                a.emit.i[pos] = (int32_t)(job.Ra * ROWBLK + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3));
                a.emit.j[pos] = (int32_t)j;
                a.emit.score[pos] = tp.vs[r];
            }
        }
        off += (unsigned long long)__popcll(b);
    }
}

// One wave's block on its own: one atomic per wave.
__device__ __forceinline__ void thr_epilogue(const TileLaunch &a, const Problem &p,
                                             const WaveJob &job, int lane, const f32x16 acc[9],
                                             const EpiRadii &er, const FrameTerms &ft)
{
    ThrPairs tp;
    thr_scores_t<false>(a, p, job, lane, acc, er, ft, tp);
    if (tp.total == 0) return;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(a.emit.count, (unsigned long long)tp.total);
    base = __shfl(base, 0, 64);
    thr_write(a, job, lane, tp, base);
}

// Persistent ping-pong kernel.  A workgroup is two groups of four waves, one
// wave of each group per SIMD.  At phase ph the group of parity ph runs the
// MFMA contraction of the workgroup's tile ph while the other group runs the
// FP64 epilogue of tile ph-1 (which it contracted in the previous phase), so
// the matrix cores and the FP64 VALUs of every SIMD work at the same time.
// One barrier per phase keeps the groups in step; the tile index of each
// phase goes through a three-slot LDS ring, so a slot is never rewritten
// while a wave of the previous phase may still read it.
//
// Tile order: TK_SYM / TK_RECT follow the banded order, split into eight
// contiguous chunks, one per XCD (workgroups are dealt round-robin to the
// XCDs), whose workgroups take the chunk's tiles round-robin, one per phase.
// TK_BATCH takes tiles from a global counter in the host's order (most
// expensive tiles first), so uneven ensembles balance.
template <int MODE, int KIND, int OP>
__global__ __launch_bounds__(512, 1) void tile_kernel(TileLaunch a)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int grp = wave >> 2;
    const int w = wave & 3;
    __shared__ int64_t s_tile[3];
    const int64_t per = gridDim.x >> 3;
    const int64_t xcd = blockIdx.x & 7, jw = blockIdx.x >> 3;
    const int64_t c0 = a.T * xcd / 8, c1 = a.T * (xcd + 1) / 8;

    f32x16 acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
    WaveJob job{0, 0, 0, 0};
    for (int64_t ph = 0;; ++ph) {
        if (threadIdx.x == 0) {
            int64_t t;
            if constexpr (KIND == TK_BATCH) {
                t = atomicAdd(&a.counters[a.ctr], 1);
            } else {
                t = c0 + jw + per * ph;
                if (t >= c1) t = a.T;
            }
            s_tile[ph % 3] = t;
        }
        __syncthreads();
        const int64_t tk = s_tile[ph % 3];
        const int64_t te = ph > 0 ? s_tile[(ph + 2) % 3] : a.T;
        if (tk >= a.T && te >= a.T) break;
        if ((int)(ph & 1) == grp) {
            job = decode_job<KIND>(a, tk, w);
            if (job.active) {
#pragma unroll
                for (int q = 0; q < 9; ++q)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
                const Problem &p = problem_of<KIND>(a, job.pidx);
                contract<MODE>(a.ws + p.opsA, a.ws + p.opsB, job.Ra, job.Rb, p.KB, lane, acc);
            }
        } else if (job.active) {
            // the persistent schedule serves problems without the reference
            // frame only (the host never pairs the two)
            const Problem &pe = problem_of<KIND>(a, job.pidx);
            const EpiRadii er = epi_radii(a, pe, job, lane);
            const FrameTerms ft{nullptr, nullptr};
            if constexpr (OP == OP_FWD) epilogue_t<false, KIND != TK_RECT>(a, pe, job, lane, acc, er, ft);
            else if constexpr (OP == OP_BWD) bwd_epilogue(a, pe, job, lane, acc, er);
            else thr_epilogue(a, pe, job, lane, acc, er, ft);
            job.active = 0;
        }
    }
}

// ------------------------------------------------------ staged forward
//
// Forward pass of one problem (TK_SYM or TK_RECT): one 64x64 tile per 4-wave
// workgroup, two workgroups per CU.  The operand chunks of the tile's two
// row blocks of A and two of B for one K-block (24 KiB in the split modes)
// are staged in a 3-slot LDS ring: each chunk reaches the CU once instead of
// once per wave that reads it.  They travel straight from global memory to
// LDS (no registers) and are issued two K-blocks ahead, so a K-block's loads
// have a whole step of contraction to land.  Each wave then runs the FP64
// epilogue of its 32x32 block.  The two workgroups of a CU are independent,
// so one's MFMA contraction overlaps the other's FP64 epilogue.

template <int MODE>
struct StageGeom {
    static constexpr int P = is_split(MODE) ? 2 : 1;   // chunk parts (hi, lo)
    static constexpr int REGION = 3 * P * 64;           // u32x4 per (row block, K-block)
    static constexpr int SLOT = 4 * REGION;             // rows 0, 1 of A, rows 0, 1 of B
    static constexpr int PER = SLOT / 256;              // u32x4 loads per thread
};

// K-block kb (>= 0) of the tile whose first row blocks of A and B are rA
// and rB, sent straight from global memory to the LDS slot (no registers):
// wave w moves region w (row block rA + w of A for w < 2, rB + w - 2 of B
// otherwise; region R of K-block kb is chunks (R*KB + kb)*REGION onwards),
// load m carrying its chunks 64 m .. 64 m + 63, lane l's 16 bytes landing at
// slot + REGION w + 64 m + l.  The region's start is wave-uniform (kept in
// scalar registers, stage_base) and the lane's byte offset fixed, so a load
// needs no vector address arithmetic.
//
// kb < 0 issues the same number of loads into the same chunks, so that every
// step has the same count in flight: with kb = STAGE_FRAME, into chunks
// 0 .. 2 FRAME_CHUNKS - 1, the reference-frame terms of the tile (U of its 64
// rows, then P^T of its 64 columns, 9 doubles per model, contiguous in the
// workspace), the rest from the first chunks of A (always present, cached)
// like every other kb < 0; nothing reads a slot filled with the latter again.
constexpr int64_t STAGE_PAST = -1, STAGE_FRAME = -2;
constexpr int FRAME_CHUNKS = 2 * ROWBLK * 9 * 8 / 16;   // 16-byte chunks per 64 models

// Start of wave w's region in K-block 0 of the tile (wave-uniform).
template <int MODE>
__device__ __forceinline__ const char *stage_base(const Problem &p, const char *ws, int64_t rA,
                                                  int64_t rB, int w)
{
    using G = StageGeom<MODE>;
    const int64_t span = p.KB * G::REGION;           // chunks of one row block
    const u32x4 *src = w < 2 ? (const u32x4 *)(ws + p.opsA) + (rA + w) * span
                             : (const u32x4 *)(ws + p.opsB) + (rB + w - 2) * span;
    const uint64_t v = (uint64_t)src;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const char *)(((uint64_t)hi << 32) | lo);
}

template <int MODE>
__device__ __forceinline__ void stage_dma(const Problem &p, const char *ws, int64_t rA,
                                          int64_t rB, int64_t kb, int tid, int w,
                                          const char *base, u32x4 *slot)
{
    using G = StageGeom<MODE>;
    static_assert(2 * FRAME_CHUNKS <= G::SLOT, "frame terms fit a slot");
    static_assert(G::PER * 64 == G::REGION, "one region per wave");
    if (kb >= 0) {
        // The wave-uniform start of each load's chunks is held opaque in
        // scalar registers and the lane's 32-bit byte offset opaque in a
        // vector register, so that every address stays scalar base + 32-bit
        // offset (no 64-bit vector address arithmetic per load).
        uint32_t vo = (uint32_t)(tid & 63) * 16u;
        asm volatile("" : "+v"(vo));
#pragma unroll
        for (int m = 0; m < G::PER; ++m) {
            const char *row = base + (kb * G::REGION + 64 * m) * 16;
            asm volatile("" : "+s"(row));
            __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)(row + vo),
                                             (void __attribute__((address_space(3))) *)(slot + G::REGION * w + 64 * m),
                                             16, 0, 0);
        }
        return;
    }
    // once or twice per tile: chunk q of the slot from the frame terms or A
    const u32x4 *ops = (const u32x4 *)(ws + p.opsA);
    const u32x4 *fU = (const u32x4 *)(ws + p.UA) + rA * (ROWBLK * 9 * 8 / 16);
    const u32x4 *fP = (const u32x4 *)(ws + p.PTB) + rB * (ROWBLK * 9 * 8 / 16);
#pragma unroll
    for (int m = 0; m < G::PER; ++m) {
        const int q = G::REGION * w + 64 * m + (tid & 63);
        const u32x4 *src = ops + q;
        if (kb == STAGE_FRAME && q < 2 * FRAME_CHUNKS)
            src = q < FRAME_CHUNKS ? fU + q : fP + (q - FRAME_CHUNKS);
        __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)src,
                                         (void __attribute__((address_space(3))) *)(slot + G::REGION * w + 64 * m),
                                         16, 0, 0);
    }
}

// s_waitcnt vmcnt(N) alone (expcnt and lgkmcnt left free), N <= 63.
template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 64, "vmcnt field");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// One 64x64 tile t (launch-relative) by the workgroup's four waves, with
// the three ring slots of the workgroup.  The slots are separate arrays
// (fixed per unrolled step below), so that the compiler can tell the loads
// in flight into one slot from the reads of another and adds no wait for
// them.
template <int MODE, int KIND, int OP>
__device__ __forceinline__ void staged_tile(const TileLaunch &a, int64_t t, int tid, int lane, int w,
                                            u32x4 *slot0, u32x4 *slot1, u32x4 *slot2)
{
    using G = StageGeom<MODE>;
    const int wy = w >> 1, wx = w & 1;
    if constexpr (KIND == TK_BATCH) t += a.t0;
    int32_t e = 0;
    if constexpr (KIND == TK_BATCH)
        e = table_find(a.table, a.nprob, t, [](const Problem &q) { return q.tile0; });
    const Problem &p = problem_of<KIND>(a, e);
    int64_t bi, bj;
    if constexpr (KIND == TK_RECT) band_decode_rect(t, p.nbA, p.nbB, p.band, &bi, &bj);
    else band_decode(t - p.tile0, p.nbA, p.band, &bi, &bj);
    const int64_t KB = p.KB;
    constexpr bool lolo = MODE == MODE_BF16X4;     // the fourth product lo*lo'

    WaveJob job;
    job.Ra = 2 * bi + wy;
    job.Rb = 2 * bj + wx;
    job.pidx = e;
    job.active = !(p.sym && bi == bj && wy > wx) && job.Ra * ROWBLK < p.NA &&
                 job.Rb * ROWBLK < p.NB;
    // the epilogue's radii, loaded with the first K-blocks
    const EpiRadii er = epi_radii(a, p, job, lane);
    // In the reference frame the tile's frame terms travel like an operand
    // K-block, into the slot of K-block KB (the first step past the end, or
    // the prologue when KB = 1), which no step reads; they have landed once
    // the last step's wait and barrier have passed.
    const bool fterms = OP != OP_BWD && p.frame;
    const int64_t kb_frame = fterms ? STAGE_FRAME : STAGE_PAST;
    // the contraction runs at a raised wave priority: a SIMD's other wave is
    // usually in its FP64 epilogue, and the MFMA issue should not wait behind
    // that stream of VALU instructions
    __builtin_amdgcn_s_setprio(3);
    const char *const rbase = stage_base<MODE>(p, a.ws, 2 * bi, 2 * bj, w);
    stage_dma<MODE>(p, a.ws, 2 * bi, 2 * bj, 0, tid, w, rbase, slot0);
    stage_dma<MODE>(p, a.ws, 2 * bi, 2 * bj, KB > 1 ? 1 : kb_frame, tid, w, rbase, slot1);
    wait_vmcnt<0>();
    __builtin_amdgcn_s_barrier();

    f32x16 acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
    // One K-block from slot cur; the loads of K-block kb + 2 go into nxt
    // (the slot read one step earlier, released by that step's barrier) and
    // stay in flight across the next step: at the end of this step only the
    // loads of K-block kb + 1 (issued one step earlier) must have landed.
    // The barrier needs no memory fence: each wave's own waits order its
    // loads, and the LDS reads are complete once their MFMAs have issued.
    auto step = [&](int64_t kb, const u32x4 *cur, u32x4 *nxt) {
        stage_dma<MODE>(p, a.ws, 2 * bi, 2 * bj,
                        kb + 2 < KB ? kb + 2 : (kb + 2 == KB ? kb_frame : STAGE_PAST), tid, w, rbase,
                        nxt);
        pin_order();
        const u32x4 *sA = cur + wy * G::REGION + lane;
        const u32x4 *sB = cur + (2 + wx) * G::REGION + lane;
        if constexpr (MODE == MODE_FP32) {
            f32x4 A[3], B[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                A[c] = __builtin_bit_cast(f32x4, sA[c * 64]);
                B[c] = __builtin_bit_cast(f32x4, sB[c * 64]);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        acc[3 * c + d] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[c][e], B[d][e],
                                                                             acc[3 * c + d], 0, 0, 0);
        } else {
            // hi*hi', hi*lo', (lo*lo'), lo*hi': the order of the contraction
            // in the other kernels, so every path rounds identically; at most
            // three of the four operand sets are live at once
            u32x4 Ah[3], Bh[3], Al[3], Bl[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Ah[c] = sA[(2 * c) * 64];
                Bh[c] = sB[(2 * c) * 64];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) Bl[c] = sB[(2 * c + 1) * 64];
#pragma unroll
            for (int c = 0; c < 3; ++c) Al[c] = sA[(2 * c + 1) * 64];
            // the hi operands are read first and the first nine products
            // wait only for them; the lo operands land meanwhile
            __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    acc[3 * c + d] = mfma_split<MODE>(Ah[c], Bh[d], acc[3 * c + d]);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    acc[3 * c + d] = mfma_split<MODE>(Ah[c], Bl[d], acc[3 * c + d]);
            if constexpr (lolo) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        acc[3 * c + d] = mfma_split<MODE>(Al[c], Bl[d], acc[3 * c + d]);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    acc[3 * c + d] = mfma_split<MODE>(Al[c], Bh[d], acc[3 * c + d]);
        }
        // the wait and barrier stay behind the MFMAs (the scheduler would
        // otherwise hoist them, shortening the distance the loads get)
        __builtin_amdgcn_sched_barrier(0);
        wait_vmcnt<G::PER>();
        __builtin_amdgcn_s_barrier();
    };
    // whole rounds of three steps, then the remainder: every round ends with
    // the step into slot 2, so the compiler sees slot 0 complete at the top
    int64_t kb = 0;
    for (; kb + 3 <= KB; kb += 3) {
        step(kb, slot0, slot2);
        step(kb + 1, slot1, slot0);
        step(kb + 2, slot2, slot1);
    }
    if (kb < KB) step(kb, slot0, slot2);
    if (kb + 1 < KB) step(kb + 1, slot1, slot0);
    wait_vmcnt<0>();    // no load into LDS outlives the workgroup
    __builtin_amdgcn_s_setprio(0);
    const int fs = (int)(KB % 3);
    const double *fbase = (const double *)(fs == 0 ? slot0 : fs == 1 ? slot1 : slot2);
    const FrameTerms ft{fbase + 9 * ROWBLK * wy, fbase + 9 * ROWBLK * (2 + wx)};

    if constexpr (OP == OP_THR) {
        // the four waves' emission counts go to the output counter in one
        // atomic per workgroup (every wave, active or not, meets the barriers)
        __shared__ uint32_t wtot[4];
        __shared__ unsigned long long wbase;
        ThrPairs tp;
        tp.total = 0;
        if (job.active) thr_scores(a, p, job, lane, acc, er, ft, tp);
        if (lane == 0) wtot[w] = tp.total;
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t sum = wtot[0] + wtot[1] + wtot[2] + wtot[3];
            wbase = sum ? atomicAdd(a.emit.count, (unsigned long long)sum) : 0ull;
        }
        __syncthreads();
        if (tp.total) {
            unsigned long long base = wbase;
            for (int v = 0; v < w; ++v) base += wtot[v];
            thr_write(a, job, lane, tp, base);
        }
    } else if (job.active) {
        if constexpr (OP == OP_BWD) bwd_epilogue(a, p, job, lane, acc, er);
        else epilogue<KIND != TK_RECT>(a, p, job, lane, acc, er, ft);
    }
}

template <int MODE, int KIND, int OP>
__global__ __launch_bounds__(256, 2) void staged_kernel(TileLaunch a)
{
    using G = StageGeom<MODE>;
    __shared__ u32x4 slot0[G::SLOT], slot1[G::SLOT], slot2[G::SLOT];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    // Workgroups are dealt to the XCDs round-robin.  One problem: tiles in
    // banded order, one contiguous chunk per XCD.  A batch: the host's order
    // (most expensive tiles first, for balance) in runs of eight consecutive
    // tiles per XCD (within every 64 workgroups, XCD x takes tiles 8x..8x+7),
    // so neighbouring tiles of one problem share an L2.
    int64_t t;
    if constexpr (KIND == TK_BATCH) {
        const int64_t b = blockIdx.x;
        t = (b & ~(int64_t)63) + 8 * (b & 7) + ((b >> 3) & 7);
    } else {
        const int64_t per_xcd = gridDim.x >> 3;
        t = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    }
    if (t >= a.T) return;                          // uniform over the workgroup
    staged_tile<MODE, KIND, OP>(a, t, tid, lane, w, slot0, slot1, slot2);
}

template <int MODE>
static hipError_t launch_mode(const TileLaunch &a, hipStream_t s, int64_t grid, int op)
{
    dim3 g((unsigned)grid), b(512);
    // staged grids: a multiple of 8 (one chunk per XCD), or of 64 for a batch
    // (runs of 8 tiles per XCD); workgroups past the last tile return at once
    const dim3 sg((unsigned)round_up(a.T > 0 ? a.T : 1, a.kind == TK_BATCH ? 64 : 8)), sb(256);
    if (op == OP_THR) {
        if (a.kind != TK_SYM) return hipErrorInvalidValue;
        staged_kernel<MODE, TK_SYM, OP_THR><<<sg, sb, 0, s>>>(a);
        return hipGetLastError();
    }
    if (op == OP_BWD) {
        if (a.kind == TK_SYM) staged_kernel<MODE, TK_SYM, OP_BWD><<<sg, sb, 0, s>>>(a);
        else if (a.kind == TK_RECT) staged_kernel<MODE, TK_RECT, OP_BWD><<<sg, sb, 0, s>>>(a);
        else return hipErrorInvalidValue;
        return hipGetLastError();
    }
    const bool pers = a.sched == SCHED_PERSISTENT;
    switch (a.kind) {
    case TK_SYM:
        if (pers) tile_kernel<MODE, TK_SYM, OP_FWD><<<g, b, 0, s>>>(a);
        else staged_kernel<MODE, TK_SYM, OP_FWD><<<sg, sb, 0, s>>>(a);
        break;
    case TK_RECT:
        if (pers) tile_kernel<MODE, TK_RECT, OP_FWD><<<g, b, 0, s>>>(a);
        else staged_kernel<MODE, TK_RECT, OP_FWD><<<sg, sb, 0, s>>>(a);
        break;
    case TK_BATCH:
        if (pers) tile_kernel<MODE, TK_BATCH, OP_FWD><<<g, b, 0, s>>>(a);
        else staged_kernel<MODE, TK_BATCH, OP_FWD><<<sg, sb, 0, s>>>(a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tile(int mode, const TileLaunch &a, hipStream_t s, int op)
{
    // persistent: one workgroup (8 waves) per CU, a multiple of 8 so every
    // XCD gets the same number of workgroups; every workgroup leaves its
    // phase loop once both of its groups have run out of tiles
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t grid = round_up(cus, 8);
    const int64_t need = round_up(a.T > 0 ? a.T : 1, 8);
    if (grid > need) grid = need;
    switch (mode) {
    case MODE_FP32: return launch_mode<MODE_FP32>(a, s, grid, op);
    case MODE_BF16: return launch_mode<MODE_BF16>(a, s, grid, op);
    case MODE_FP16: return launch_mode<MODE_FP16>(a, s, grid, op);
    case MODE_BF16X4: return launch_mode<MODE_BF16X4>(a, s, grid, op);
    default: return hipErrorInvalidValue;
    }
}

} // namespace clusco
