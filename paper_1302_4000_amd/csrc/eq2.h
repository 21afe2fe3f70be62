// Per-pair epilogue of Eq. 2 (Algorithms): cRMSD from the 3x3 correlation of
// two centred models and their radii, with no SVD and no rotation matrix.
//
// Inputs are unnormalised: H = sum_i a_i b_i^T (so H = L M) and
// E_A = sum_i |a_i|^2 = L R_A^2.  With s1 >= s2 >= s3 the singular values of
// H and S = sign det H, Eq. 2 reads
//     L cRMSD^2 = E_A + E_B - 2 (s1 + s2 + S s3).
// The eigenvalues l_k = s_k^2 of H^T H are the roots of the cubic
//     l^3 - c2 l^2 + c1 l - c0,
//     c2 = |H|_F^2,  c1 = |cof H|_F^2 (sum of squared 2x2 minors),
//     c0 = (det H)^2.
// Both c2 and c1 are sums of squares here (no cancellation).  Only the
// largest root l1 is solved for, by FP64 Newton steps from an upper bound
// (see eq2_largest_root).  The other two roots enter
// only through their symmetric functions (Vieta on the deflated quadratic):
//     l2 + l3 = c2 - l1,   S s2 s3 = det H / s1,
// so  s2 + S s3 = sqrt(c2 - l1 + 2 det H / s1),
// which needs neither l2 nor l3 nor the square root of a tiny, noisy l3.
//
// Accuracy budget: the score needs s1 + s2 + S s3 to about 1e-10 relative,
// so the FP64 reciprocal and reciprocal square root come from the hardware
// estimates (v_rcp_f64, v_rsq_f64) refined by one Newton step each
// (relative error ~1e-14) instead of correctly rounded division and sqrt.
#pragma once

#include <hip/hip_runtime.h>

namespace clusco {

struct Eq2Coef {
    double c2, c1, det;
};

__device__ __forceinline__ Eq2Coef eq2_coefficients(const double h[9])
{
    // cofactors (2x2 minors) of H, row-major h[3p+q]
    double m00 = h[4] * h[8] - h[5] * h[7];
    double m01 = h[3] * h[8] - h[5] * h[6];
    double m02 = h[3] * h[7] - h[4] * h[6];
    double m10 = h[1] * h[8] - h[2] * h[7];
    double m11 = h[0] * h[8] - h[2] * h[6];
    double m12 = h[0] * h[7] - h[1] * h[6];
    double m20 = h[1] * h[5] - h[2] * h[4];
    double m21 = h[0] * h[5] - h[2] * h[3];
    double m22 = h[0] * h[4] - h[1] * h[3];
    Eq2Coef c;
    c.det = h[0] * m00 - h[1] * m01 + h[2] * m02;
    c.c2 = h[0] * h[0] + h[1] * h[1] + h[2] * h[2] + h[3] * h[3] + h[4] * h[4] + h[5] * h[5]
         + h[6] * h[6] + h[7] * h[7] + h[8] * h[8];
    c.c1 = m00 * m00 + m01 * m01 + m02 * m02 + m10 * m10 + m11 * m11 + m12 * m12
         + m20 * m20 + m21 * m21 + m22 * m22;
    return c;
}

// 1/sqrt(x) for x > 0: hardware estimate + one Newton step r(3 - x r^2)/2.
__device__ __forceinline__ double rsqrt_refined(double x)
{
    const double r = __builtin_amdgcn_rsq(x);
    const double hr = 0.5 * x * r;
    return fma(r, fma(-hr, r, 0.5), r);
}

// One Newton step on f(l) = l^3 - c2 l^2 + c1 l - c0.  With d = l - c2 and
// g = d l + c1 (so f = g l - c0), the slope is f'(l) = 3 l^2 - 2 c2 l + c1
// = g + l (l + d): five FP64 operations for f and f' together.  An
// approximate reciprocal of the slope only slows the contraction by its own
// relative error (~1e-8), far below the quadratic gain.  Returns the step
// taken.
__device__ __forceinline__ double eq2_newton(double &l, double c2, double c1, double c0)
{
    const double d = l - c2;
    const double g = fma(d, l, c1);
    const double f = fma(g, l, -c0);
    const double fp = fma(l, l + d, g);
    const double step = fp > 0.0 ? f * __builtin_amdgcn_rcp(fp) : 0.0;
    l -= step;
    return step;
}

// Largest root l1 of l^3 - c2 l^2 + c1 l - c0 (all roots real, >= 0).
//
// Start: x0 = c2 - c1 / c2 is an upper bound, since with s = l2 + l3,
//     x0 - l1 = (s^2 - l2 l3) / (l1 + s) >= 0,
// and it is tight when l1 dominates (the usual shape of protein models:
// relative excess (s / l1)^2).  Above l1 the cubic is increasing and convex
// (f'' = 6l - 2 c2 > 0 for l > c2/3), so Newton steps from x0 decrease
// monotonically to l1.  Four steps take a 3% excess to machine precision.
// Near a double root l1 = l2 Newton turns linear; lanes whose fourth step is
// still above 1e-9 relative continue (at most 60 more steps).
__device__ __forceinline__ double eq2_largest_root(double c2, double c1, double c0)
{
    double l = fma(-c1, __builtin_amdgcn_rcp(c2), c2);
    double step = 0.0;
#pragma unroll
    for (int it = 0; it < 4; ++it) step = eq2_newton(l, c2, c1, c0);
    if (fabs(step) > 1e-9 * l) {
        for (int it = 0; it < 60 && fabs(step) > 1e-15 * l; ++it) step = eq2_newton(l, c2, c1, c0);
    }
    return l;
}

// Sum s1 + s2 + S s3 of the signed singular values of H.
__device__ __forceinline__ double eq2_signed_sum(const double h[9])
{
    const Eq2Coef c = eq2_coefficients(h);
    if (!(c.c2 > 0.0)) return 0.0;
    double l1 = eq2_largest_root(c.c2, c.c1, c.det * c.det);
    l1 = fmax(l1, c.c2 * (1.0 / 3.0));             // l1 >= mean eigenvalue
    const double r1 = rsqrt_refined(l1);           // 1 / s1
    const double s1 = l1 * r1;
    const double t = fma(2.0 * c.det, r1, c.c2 - l1);   // (s2 + S s3)^2
    const double tp = fmax(t, 1e-300);
    const double s23 = (t > 0.0) ? tp * rsqrt_refined(tp) : 0.0;
    return s1 + s23;
}

// L * cRMSD^2 from H and the two radii (not clamped; may be slightly negative
// from rounding when the models coincide).
__device__ __forceinline__ double eq2_lrmsd2(const double h[9], double EA, double EB)
{
    return fma(-2.0, eq2_signed_sum(h), EA + EB);
}

// State between the two stages of eq2_lrmsd2_batch (per pair: the largest
// root l1, the coefficient c2, det H and the floored c2).
template <int NP>
struct Eq2Roots {
    double l[NP], c2[NP], det[NP], c2f[NP];
};

// First stage: coefficients and the largest root of every pair.
template <int NP, int STEPS>
__device__ __forceinline__ void eq2_roots_batch(const double (&h)[NP][9], Eq2Roots<NP> &st)
{
    double c1[NP], c0[NP], step[NP], floor_fp[NP];
    double (&c2)[NP] = st.c2, (&det)[NP] = st.det, (&l)[NP] = st.l, (&c2f)[NP] = st.c2f;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const Eq2Coef c = eq2_coefficients(h[p]);
        c2[p] = c.c2;
        c1[p] = c.c1;
        det[p] = c.det;
        c0[p] = c.det * c.det;
        c2f[p] = fmax(c.c2, 1e-300);
        floor_fp[p] = fmax(1e-30 * (c.c2 * c.c2), 1e-300);
        l[p] = fma(-c.c1, __builtin_amdgcn_rcp(c2f[p]), c.c2);
        step[p] = 0.0;
    }
#pragma unroll
    for (int it = 0; it < STEPS; ++it) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            // f and f' as in eq2_newton
            const double d = l[p] - c2[p];
            const double g = fma(d, l[p], c1[p]);
            const double f = fma(g, l[p], -c0[p]);
            const double fp = fma(l[p], l[p] + d, g);
            step[p] = f * __builtin_amdgcn_rcp(fmax(fp, floor_fp[p]));
            l[p] -= step[p];
        }
    }
    // A last step of relative size d leaves an error of about d^2 (quadratic
    // convergence at a simple root): below 1e-5 after three steps, 1e-9 after
    // four, the root is good to ~1e-10 or better; other lanes continue.
    constexpr double done_below = STEPS >= 4 ? 1e-9 : 1e-5;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        if (fabs(step[p]) > done_below * l[p]) {
            int it = 0;
#pragma clang loop unroll(disable)
            do {
                step[p] = eq2_newton(l[p], c2[p], c1[p], c0[p]);
            } while (++it < 60 && fabs(step[p]) > 1e-15 * l[p]);
        }
    }
}

// Second stage: s1 + s2 + S s3 from the root, and L cRMSD^2.
// The hardware reciprocal square roots (relative error below 6e-8 on
// gfx950) get one Newton step each: an error of that size in the sum
// s1 + s2 + S s3, whose magnitude is the radii E, would dominate the
// contraction error of the reference frame (proportional to the residual
// radii only).
template <int NP>
__device__ __forceinline__ void eq2_finish_batch(const Eq2Roots<NP> &st, const double (&ea)[NP],
                                                 const double (&eb)[NP], double (&out)[NP])
{
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const double l1 = fmax(st.l[p], st.c2f[p] * (1.0 / 3.0));
        const double r1 = rsqrt_refined(l1);
        const double t = fma(2.0 * st.det[p], r1, st.c2[p] - l1);   // (s2 + S s3)^2
        const double tp = fmax(t, 1e-300);
        const double sum = fma(l1, r1, tp * rsqrt_refined(tp));    // s1 + s2 + S s3
        out[p] = fma(-2.0, sum, ea[p] + eb[p]);
    }
}

// L * cRMSD^2 of NP independent pairs at once, for the tile epilogue: the
// arithmetic of eq2_lrmsd2 written with the fewest instructions.  The NP
// dependency chains sit side by side.  Instead of branches and selects on
// degenerate inputs, three floors keep every operation finite: the slope in
// the Newton step (at least 1e-30 c2^2, so a step at an exact double root is
// 0/tiny = 0), the root (at least max(c2, 1e-300)/3, so 1/sqrt never sees 0)
// and (s2 + S s3)^2 (at least 1e-300).  For H = 0 the sum then comes out as
// about 1e-150 instead of 0, far below the score's resolution.
template <int NP, int STEPS>
__device__ __forceinline__ void eq2_lrmsd2_batch(const double (&h)[NP][9], const double (&ea)[NP],
                                                 const double (&eb)[NP], double (&out)[NP])
{
    Eq2Roots<NP> st;
    eq2_roots_batch<NP, STEPS>(h, st);
    eq2_finish_batch<NP>(st, ea, eb, out);
}

// ------------------------------------------------------------ backward

// Unit vector spanning the null space of the symmetric 3x3 matrix M (given
// by its six distinct entries): the longest cross product of two of its
// rows.  Returns false when every cross product vanishes (rank < 2).
__device__ __forceinline__ bool null_vector(double m00, double m01, double m02, double m11,
                                            double m12, double m22, double v[3])
{
    const double r0[3] = {m00, m01, m02}, r1[3] = {m01, m11, m12}, r2[3] = {m02, m12, m22};
    double c[3][3];
    const double *pa[3] = {r0, r0, r1}, *pb[3] = {r1, r2, r2};
    double best = 0.0;
    int k = 0;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const double *a = pa[t], *b = pb[t];
        c[t][0] = a[1] * b[2] - a[2] * b[1];
        c[t][1] = a[2] * b[0] - a[0] * b[2];
        c[t][2] = a[0] * b[1] - a[1] * b[0];
        const double n = c[t][0] * c[t][0] + c[t][1] * c[t][1] + c[t][2] * c[t][2];
        if (n > best) {
            best = n;
            k = t;
        }
    }
    if (!(best > 0.0)) return false;
    const double inv = 1.0 / sqrt(best);
    v[0] = c[k][0] * inv;
    v[1] = c[k][1] * inv;
    v[2] = c[k][2] * inv;
    return true;
}

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Unit vector orthogonal to the unit vector a, any one.
__device__ __forceinline__ void any_orthogonal(const double a[3], double b[3])
{
    const double e[3] = {fabs(a[0]) < 0.57 ? 1.0 : 0.0, fabs(a[0]) < 0.57 ? 0.0 : 1.0, 0.0};
    cross3(a, e, b);
    const double inv = 1.0 / sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    b[0] *= inv;
    b[1] *= inv;
    b[2] *= inv;
}

// Removes the component of b along the unit vector a and normalises b;
// falls back to any unit vector orthogonal to a when little is left.
__device__ __forceinline__ void orthonormalise(const double a[3], double b[3], double floor_sq)
{
    const double d = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    b[0] -= d * a[0];
    b[1] -= d * a[1];
    b[2] -= d * a[2];
    const double n = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    if (n > floor_sq) {
        const double inv = 1.0 / sqrt(n);
        b[0] *= inv;
        b[1] *= inv;
        b[2] *= inv;
    } else {
        any_orthogonal(a, b);
    }
}

// Gradient of s1 + s2 + S s3 with respect to H (row-major q[3p+r]):
// Q = U V^T for H = U diag(s1, s2, S s3) V^T with U and V proper rotations,
// i.e. U diag(1,1,S) V^T of the SVD.  v1, v2 are eigenvectors of H^T H for
// l1, l2 (null vectors of H^T H - l I), v3 = v1 x v2; u_k = H v_k / s_k for
// k = 1, 2 and u3 = u1 x u2, so s3 is never divided by.  l2 comes from the
// deflated quadratic l^2 - (c2 - l1) l + c0 / l1.
__device__ __forceinline__ void eq2_adjoint(const double h[9], double q[9])
{
    const Eq2Coef c = eq2_coefficients(h);
#pragma unroll
    for (int t = 0; t < 9; ++t) q[t] = (t % 4 == 0) ? 1.0 : 0.0;
    if (!(c.c2 > 0.0)) return;
    const double l1 = fmax(eq2_largest_root(c.c2, c.c1, c.det * c.det), c.c2 * (1.0 / 3.0));
    const double sm = c.c2 - l1, pr = c.det * c.det / l1;
    const double l2 = 0.5 * (sm + sqrt(fmax(sm * sm - 4.0 * pr, 0.0)));
    // K = H^T H
    const double k00 = h[0] * h[0] + h[3] * h[3] + h[6] * h[6];
    const double k01 = h[0] * h[1] + h[3] * h[4] + h[6] * h[7];
    const double k02 = h[0] * h[2] + h[3] * h[5] + h[6] * h[8];
    const double k11 = h[1] * h[1] + h[4] * h[4] + h[7] * h[7];
    const double k12 = h[1] * h[2] + h[4] * h[5] + h[7] * h[8];
    const double k22 = h[2] * h[2] + h[5] * h[5] + h[8] * h[8];
    double v1[3], v2[3], v3[3], u1[3], u2[3], u3[3];
    if (!null_vector(k00 - l1, k01, k02, k11 - l1, k12, k22 - l1, v1)) {
        v1[0] = 1.0; v1[1] = 0.0; v1[2] = 0.0;
    }
    if (!null_vector(k00 - l2, k01, k02, k11 - l2, k12, k22 - l2, v2)) any_orthogonal(v1, v2);
    orthonormalise(v1, v2, 1e-6);
    cross3(v1, v2, v3);
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        u1[p] = h[3 * p] * v1[0] + h[3 * p + 1] * v1[1] + h[3 * p + 2] * v1[2];
        u2[p] = h[3 * p] * v2[0] + h[3 * p + 1] * v2[1] + h[3 * p + 2] * v2[2];
    }
    const double n1 = sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
    u1[0] /= n1; u1[1] /= n1; u1[2] /= n1;
    orthonormalise(u1, u2, 1e-24 * c.c2);
    cross3(u1, u2, u3);
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int r = 0; r < 3; ++r)
            q[3 * p + r] = u1[p] * v1[r] + u2[p] * v2[r] + u3[p] * v3[r];
}

} // namespace clusco
