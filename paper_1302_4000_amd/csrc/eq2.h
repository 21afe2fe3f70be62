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
// largest root l1 is solved for: a float32 trigonometric (Viete) estimate
// polished by two FP64 Newton steps on the cubic.  The other two roots enter
// only through their symmetric functions (Vieta on the deflated quadratic):
//     l2 + l3 = c2 - l1,   S s2 s3 = det H / s1,
// so  s2 + S s3 = sqrt(c2 - l1 + 2 det H / s1),
// which needs neither l2 nor l3 nor the square root of a tiny, noisy l3.
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

// Largest root of l^3 - c2 l^2 + c1 l - c0 (all roots real, >= 0).
__device__ __forceinline__ double eq2_largest_root(double c2, double c1, double c0)
{
    // float32 seed: l = m + 2a cos(phi/3), cos(phi) = -q / (2 a^3) for the
    // depressed cubic x^3 + p x + q (Viete's trigonometric form)
    float c2f = (float)c2, c1f = (float)c1, c0f = (float)c0;
    float m = c2f * (1.0f / 3.0f);
    float p = c1f - 3.0f * m * m;
    float q = (c1f - 2.0f * m * m) * m - c0f;
    float seed = m;
    if (p < 0.0f) {
        float a = sqrtf(-p * (1.0f / 3.0f));
        float t = -q / (2.0f * a * a * a);
        t = fminf(1.0f, fmaxf(-1.0f, t));
        seed = m + 2.0f * a * __cosf(acosf(t) * (1.0f / 3.0f));
    }
    double l = (double)seed;
    // Newton on the cubic; it is convex above its largest root, so a step
    // from either side lands on or above l1 and then decreases to it.
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        double f = ((l - c2) * l + c1) * l - c0;
        double fp = (3.0 * l - 2.0 * c2) * l + c1;
        if (fp > 0.0) l -= f / fp;
    }
    return l;
}

// L * cRMSD^2 from H and the two radii (not clamped; may be slightly negative
// from rounding when the models coincide).
__device__ __forceinline__ double eq2_lrmsd2(const double h[9], double EA, double EB)
{
    Eq2Coef c = eq2_coefficients(h);
    double sum = 0.0;
    if (c.c2 > 0.0) {
        double l1 = eq2_largest_root(c.c2, c.c1, c.det * c.det);
        l1 = fmax(l1, c.c2 * (1.0 / 3.0));          // l1 >= mean eigenvalue
        double s1 = sqrt(l1);
        double t = (c.c2 - l1) + 2.0 * (c.det / s1); // (s2 + S s3)^2
        sum = s1 + sqrt(fmax(t, 0.0));
    }
    return EA + EB - 2.0 * sum;
}

} // namespace clusco
