/*
 * FP64 CPU oracle for coordinate RMSD after optimal superposition.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the HIP library and never calls it.
 *
 * What it computes is the plain definition of cRMSD (Algorithms, Eq. 1):
 * the root-mean-square distance between corresponding atoms of two models
 * after the optimal rigid superposition (Background: Kabsch).  It does NOT
 * use the eigenvalue/cubic shortcut of Eq. 2; the GPU library does, and the
 * two meeting is what proves the shortcut.  Steps, for one pair (A, B):
 *
 *   1. centre each model on its arithmetic centroid (FP64 means);
 *   2. H = sum_i a_i b_i^T, a 3x3 matrix, FP64;
 *   3. H = U S V^T by one-sided (Hestenes) Jacobi rotations on the columns,
 *      swept cyclically until every column pair is orthogonal to 1e-15;
 *   4. d = sign det(V U^T) (+1 when zero), R = V diag(1,1,d) U^T, the proper
 *      rotation that maximises tr(R H), i.e. minimises sum |R a_i - b_i|^2;
 *   5. cRMSD = sqrt((1/L) sum_i |R a_i - b_i|^2), an explicit residual.
 *
 * Gradient (derived from Eq. 1 at the optimum, where the derivative through
 * R vanishes): d cRMSD / d a_i = (a_i - R^T b_i) / (L cRMSD) and
 * d cRMSD / d b_i = (b_i - R a_i) / (L cRMSD), then the centring Jacobian
 * (subtract the mean over atoms).  Defined as 0 when cRMSD is 0 (to within
 * 1e-12 of the models' joint radius, i.e. rounding of an exact zero).
 *
 * All coordinates are double [L][3] row-major (callers promote float32
 * exactly).  Packed all-vs-all output uses k(i,j) = i(2N-i-1)/2 + j-i-1 for
 * i < j, the order of N(N-1)/2 scores the paper counts (Background).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define JACOBI_TOL 1e-15
#define JACOBI_MAX_SWEEPS 100

static void centre(const double *x, int64_t L, double *a)
{
    double c[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < L; ++i)
        for (int k = 0; k < 3; ++k) c[k] += x[3 * i + k];
    for (int k = 0; k < 3; ++k) c[k] /= (double)L;
    for (int64_t i = 0; i < L; ++i)
        for (int k = 0; k < 3; ++k) a[3 * i + k] = x[3 * i + k] - c[k];
}

/* One-sided Jacobi SVD of a 3x3 matrix: H = U diag(s) V^T, s descending. */
static void svd3(const double H[3][3], double U[3][3], double s[3], double V[3][3])
{
    double W[3][3];
    memcpy(W, H, sizeof(W));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;

    static const int P[3] = {0, 0, 1}, Q[3] = {1, 2, 2};
    for (int sweep = 0; sweep < JACOBI_MAX_SWEEPS; ++sweep) {
        int rotated = 0;
        for (int r = 0; r < 3; ++r) {
            int p = P[r], q = Q[r];
            double alpha = 0, beta = 0, gamma = 0;
            for (int i = 0; i < 3; ++i) {
                alpha += W[i][p] * W[i][p];
                beta += W[i][q] * W[i][q];
                gamma += W[i][p] * W[i][q];
            }
            if (gamma == 0.0 || fabs(gamma) <= JACOBI_TOL * sqrt(alpha * beta)) continue;
            double zeta = (beta - alpha) / (2.0 * gamma);
            double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
            for (int i = 0; i < 3; ++i) {
                double wp = W[i][p], wq = W[i][q];
                W[i][p] = c * wp - sn * wq;
                W[i][q] = sn * wp + c * wq;
                double vp = V[i][p], vq = V[i][q];
                V[i][p] = c * vp - sn * vq;
                V[i][q] = sn * vp + c * vq;
            }
            rotated = 1;
        }
        if (!rotated) break;
    }

    /* singular values are the column norms; sort columns descending */
    double n[3];
    int ord[3] = {0, 1, 2};
    for (int k = 0; k < 3; ++k)
        n[k] = sqrt(W[0][k] * W[0][k] + W[1][k] * W[1][k] + W[2][k] * W[2][k]);
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (n[ord[b]] > n[ord[a]]) { int t = ord[a]; ord[a] = ord[b]; ord[b] = t; }
    double Vs[3][3];
    for (int k = 0; k < 3; ++k) {
        s[k] = n[ord[k]];
        for (int i = 0; i < 3; ++i) Vs[i][k] = V[i][ord[k]];
    }
    memcpy(V, Vs, sizeof(Vs));

    /* left singular vectors; complete an orthonormal basis where rank drops */
    double small = 1e-13 * s[0];
    double u[3][3];
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) u[k][i] = 0.0;
    if (s[0] > 0.0) {
        for (int i = 0; i < 3; ++i) u[0][i] = W[i][ord[0]] / s[0];
    } else {
        u[0][0] = 1.0;
    }
    if (s[1] > small && s[0] > 0.0) {
        for (int i = 0; i < 3; ++i) u[1][i] = W[i][ord[1]] / s[1];
    } else {
        /* any unit vector orthogonal to u0: cross with the least-aligned axis */
        int ax = 0;
        for (int i = 1; i < 3; ++i)
            if (fabs(u[0][i]) < fabs(u[0][ax])) ax = i;
        double e[3] = {0, 0, 0};
        e[ax] = 1.0;
        double c0 = u[0][1] * e[2] - u[0][2] * e[1];
        double c1 = u[0][2] * e[0] - u[0][0] * e[2];
        double c2 = u[0][0] * e[1] - u[0][1] * e[0];
        double m = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        u[1][0] = c0 / m; u[1][1] = c1 / m; u[1][2] = c2 / m;
    }
    if (s[2] > small && s[0] > 0.0) {
        for (int i = 0; i < 3; ++i) u[2][i] = W[i][ord[2]] / s[2];
    } else {
        u[2][0] = u[0][1] * u[1][2] - u[0][2] * u[1][1];
        u[2][1] = u[0][2] * u[1][0] - u[0][0] * u[1][2];
        u[2][2] = u[0][0] * u[1][1] - u[0][1] * u[1][0];
    }
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) U[i][k] = u[k][i];
}

static double det3(const double M[3][3])
{
    return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
         - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
         + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
}

/* Optimal proper rotation R (row-major 3x3) taking centred a onto centred b. */
static void kabsch_rotation(const double *a, const double *b, int64_t L, double R[3][3])
{
    double H[3][3] = {{0}};
    for (int64_t i = 0; i < L; ++i)
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) H[p][q] += a[3 * i + p] * b[3 * i + q];
    double U[3][3], s[3], V[3][3];
    svd3(H, U, s, V);
    double VUt[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            VUt[i][j] = V[i][0] * U[j][0] + V[i][1] * U[j][1] + V[i][2] * U[j][2];
    double d = det3(VUt) < 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            R[i][j] = V[i][0] * U[j][0] + V[i][1] * U[j][1] + d * V[i][2] * U[j][2];
}

/* cRMSD of two centred models with an explicit residual. */
static double rmsd_centred(const double *a, const double *b, int64_t L, double R[3][3])
{
    kabsch_rotation(a, b, L, R);
    double res = 0.0;
    for (int64_t i = 0; i < L; ++i) {
        for (int p = 0; p < 3; ++p) {
            double r = R[p][0] * a[3 * i] + R[p][1] * a[3 * i + 1] + R[p][2] * a[3 * i + 2]
                     - b[3 * i + p];
            res += r * r;
        }
    }
    return sqrt(res / (double)L);
}

/* ---------------------------------------------------------------- exports */

double oracle_crmsd_pair(const double *A, const double *B, int64_t L)
{
    if (L < 1) return 0.0;
    double *a = malloc(sizeof(double) * 6 * L), *b = a + 3 * L, R[3][3];
    centre(A, L, a);
    centre(B, L, b);
    double r = rmsd_centred(a, b, L, R);
    free(a);
    return r;
}

/* Optimal rotation (row-major) mapping centred A onto centred B. */
void oracle_kabsch_rotation(const double *A, const double *B, int64_t L, double *R9)
{
    double *a = malloc(sizeof(double) * 6 * L), *b = a + 3 * L, R[3][3];
    centre(A, L, a);
    centre(B, L, b);
    kabsch_rotation(a, b, L, R);
    memcpy(R9, R, sizeof(R));
    free(a);
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Centre every model once: out[N][L][3]. */
static double *centre_all(const double *X, int64_t N, int64_t L)
{
    double *C = malloc(sizeof(double) * 3 * L * (N > 0 ? N : 1));
    for (int64_t m = 0; m < N; ++m) centre(X + 3 * L * m, L, C + 3 * L * m);
    return C;
}

/* All-vs-all: out[k(i,j)] for i<j. */
int oracle_crmsd_matrix(const double *X, int64_t N, int64_t L, double *out, int nthreads)
{
    if (N < 0 || L < 1) return 1;
    set_threads(nthreads);
    double *C = centre_all(X, N, L);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < N; ++i) {
        double R[3][3];
        int64_t base = i * (2 * N - i - 1) / 2 - i - 1;
        for (int64_t j = i + 1; j < N; ++j)
            out[base + j] = rmsd_centred(C + 3 * L * i, C + 3 * L * j, L, R);
    }
    free(C);
    return 0;
}

/* Selected pairs (I[p], J[p]) of one ensemble. */
int oracle_crmsd_pairs(const double *X, int64_t N, int64_t L, const int64_t *I,
                       const int64_t *J, int64_t P, double *out, int nthreads)
{
    if (N < 0 || L < 1 || P < 0) return 1;
    for (int64_t p = 0; p < P; ++p)
        if (I[p] < 0 || I[p] >= N || J[p] < 0 || J[p] >= N) return 2;
    set_threads(nthreads);
#pragma omp parallel
    {
        double *a = malloc(sizeof(double) * 6 * L), *b = a + 3 * L, R[3][3];
#pragma omp for schedule(dynamic, 64)
        for (int64_t p = 0; p < P; ++p) {
            centre(X + 3 * L * I[p], L, a);
            centre(X + 3 * L * J[p], L, b);
            out[p] = rmsd_centred(a, b, L, R);
        }
        free(a);
    }
    return 0;
}

/* Dense cross matrix out[ia][ib] = cRMSD(A_ia, B_ib). */
int oracle_crmsd_cross(const double *A, int64_t Na, const double *B, int64_t Nb, int64_t L,
                       double *out, int nthreads)
{
    if (Na < 0 || Nb < 0 || L < 1) return 1;
    set_threads(nthreads);
    double *Ca = centre_all(A, Na, L), *Cb = centre_all(B, Nb, L);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < Na; ++i) {
        double R[3][3];
        for (int64_t j = 0; j < Nb; ++j)
            out[i * Nb + j] = rmsd_centred(Ca + 3 * L * i, Cb + 3 * L * j, L, R);
    }
    free(Ca);
    free(Cb);
    return 0;
}

/* Gradient of cRMSD(A,B) with respect to the raw coordinates of A (first
 * argument), scaled by g and added into gA.  a, b are the centred models. */
static void add_grad_first(const double *a, const double *b, int64_t L, double g, double *gA)
{
    double R[3][3];
    double r = rmsd_centred(a, b, L, R);
    /* cRMSD is not differentiable where it vanishes; the gradient is taken
     * as 0 there.  A residual at the rounding level of the radii counts as
     * zero (identical models leave ~1e-15 A, not an exact 0). */
    double e = 0.0;
    for (int64_t i = 0; i < 3 * L; ++i) e += a[i] * a[i] + b[i] * b[i];
    if (g == 0.0 || r <= 1e-12 * sqrt(e / (double)L)) return;
    double w = g / ((double)L * r);
    double mean[3] = {0, 0, 0};
    double *t = malloc(sizeof(double) * 3 * L);
    for (int64_t i = 0; i < L; ++i) {
        for (int p = 0; p < 3; ++p) {
            /* a_i - R^T b_i */
            double v = a[3 * i + p] - (R[0][p] * b[3 * i] + R[1][p] * b[3 * i + 1]
                                        + R[2][p] * b[3 * i + 2]);
            t[3 * i + p] = w * v;
            mean[p] += t[3 * i + p];
        }
    }
    for (int p = 0; p < 3; ++p) mean[p] /= (double)L;
    for (int64_t i = 0; i < L; ++i)
        for (int p = 0; p < 3; ++p) gA[3 * i + p] += t[3 * i + p] - mean[p];
    free(t);
}

/* Pair gradient: gA, gB (overwritten) = d cRMSD / d A, d cRMSD / d B. */
int oracle_crmsd_grad_pair(const double *A, const double *B, int64_t L, double *gA, double *gB,
                           double *rmsd)
{
    if (L < 1) return 1;
    double *a = malloc(sizeof(double) * 6 * L), *b = a + 3 * L, R[3][3];
    centre(A, L, a);
    centre(B, L, b);
    memset(gA, 0, sizeof(double) * 3 * L);
    memset(gB, 0, sizeof(double) * 3 * L);
    add_grad_first(a, b, L, 1.0, gA);
    add_grad_first(b, a, L, 1.0, gB);
    if (rmsd) *rmsd = rmsd_centred(a, b, L, R);
    free(a);
    return 0;
}

/* grad[N][L][3] = sum_{i<j} g[k(i,j)] d cRMSD_ij / d X  (overwritten).
 * Each model's row is gathered independently (every pair is visited from
 * both ends), so there are no write races. */
int oracle_crmsd_matrix_grad(const double *X, int64_t N, int64_t L, const double *g,
                             double *grad, int nthreads)
{
    if (N < 0 || L < 1) return 1;
    set_threads(nthreads);
    double *C = centre_all(X, N, L);
    memset(grad, 0, sizeof(double) * 3 * L * (N > 0 ? N : 0));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            int64_t lo = i < j ? i : j, hi = i < j ? j : i;
            double gk = g[lo * (2 * N - lo - 1) / 2 + hi - lo - 1];
            add_grad_first(C + 3 * L * i, C + 3 * L * j, L, gk, grad + 3 * L * i);
        }
    }
    free(C);
    return 0;
}

/* The same gradient for selected models only: out[r][L][3] is the row of
 * model rows[r] (for checking a large ensemble on a sample of models). */
int oracle_crmsd_matrix_grad_rows(const double *X, int64_t N, int64_t L, const double *g,
                                  const int64_t *rows, int64_t R, double *out, int nthreads)
{
    if (N < 0 || L < 1 || R < 0) return 1;
    for (int64_t r = 0; r < R; ++r)
        if (rows[r] < 0 || rows[r] >= N) return 2;
    set_threads(nthreads);
    memset(out, 0, sizeof(double) * 3 * L * R);
#pragma omp parallel
    {
        double *a = malloc(sizeof(double) * 6 * L), *b = a + 3 * L;
#pragma omp for schedule(dynamic, 16) collapse(2)
        for (int64_t r = 0; r < R; ++r) {
            for (int64_t j = 0; j < N; ++j) {
                const int64_t i = rows[r];
                if (j == i) continue;
                int64_t lo = i < j ? i : j, hi = i < j ? j : i;
                double gk = g[lo * (2 * N - lo - 1) / 2 + hi - lo - 1];
                double *tmp = calloc((size_t)(3 * L), sizeof(double));
                centre(X + 3 * L * i, L, a);
                centre(X + 3 * L * j, L, b);
                add_grad_first(a, b, L, gk, tmp);
#pragma omp critical
                for (int64_t t = 0; t < 3 * L; ++t) out[3 * L * r + t] += tmp[t];
                free(tmp);
            }
        }
        free(a);
    }
    return 0;
}

/* Cross gradient: gradA[Na][L][3], gradB[Nb][L][3] (overwritten) of
 * sum_{ia,ib} g[ia][ib] cRMSD(A_ia, B_ib). */
int oracle_crmsd_cross_grad(const double *A, int64_t Na, const double *B, int64_t Nb, int64_t L,
                            const double *g, double *gradA, double *gradB, int nthreads)
{
    if (Na < 0 || Nb < 0 || L < 1) return 1;
    set_threads(nthreads);
    double *Ca = centre_all(A, Na, L), *Cb = centre_all(B, Nb, L);
    memset(gradA, 0, sizeof(double) * 3 * L * Na);
    memset(gradB, 0, sizeof(double) * 3 * L * Nb);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < Na; ++i)
        for (int64_t j = 0; j < Nb; ++j)
            add_grad_first(Ca + 3 * L * i, Cb + 3 * L * j, L, g[i * Nb + j], gradA + 3 * L * i);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < Nb; ++j)
        for (int64_t i = 0; i < Na; ++i)
            add_grad_first(Cb + 3 * L * j, Ca + 3 * L * i, L, g[i * Nb + j], gradB + 3 * L * j);
    free(Ca);
    free(Cb);
    return 0;
}


/* ------------------------------------------------------------------ dRMSD
 * Distance RMSD (Algorithms, Eq. 5): the RMS difference of the two models'
 * intra-model distance matrices over the atom pairs i < j,
 *     dRMSD = sqrt( 2/(L(L-1)) sum_{i<j} (d^A_ij - d^B_ij)^2 ),
 * evaluated directly in FP64 (no Gram-matrix identity).  0 for L < 2. */
double oracle_drmsd_pair(const double *A, const double *B, int64_t L)
{
    if (L < 2) return 0.0;
    double s = 0.0;
    for (int64_t i = 0; i < L; ++i) {
        for (int64_t j = i + 1; j < L; ++j) {
            double da = 0.0, db = 0.0;
            for (int k = 0; k < 3; ++k) {
                double u = A[3 * i + k] - A[3 * j + k], v = B[3 * i + k] - B[3 * j + k];
                da += u * u;
                db += v * v;
            }
            double d = sqrt(da) - sqrt(db);
            s += d * d;
        }
    }
    return sqrt(2.0 * s / ((double)L * (double)(L - 1)));
}

int oracle_drmsd_matrix(const double *X, int64_t N, int64_t L, double *out, int nthreads)
{
    if (N < 0 || L < 1) return 1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < N; ++i) {
        int64_t base = i * (2 * N - i - 1) / 2 - i - 1;
        for (int64_t j = i + 1; j < N; ++j)
            out[base + j] = oracle_drmsd_pair(X + 3 * L * i, X + 3 * L * j, L);
    }
    return 0;
}

int oracle_drmsd_pairs(const double *X, int64_t N, int64_t L, const int64_t *I, const int64_t *J,
                       int64_t P, double *out, int nthreads)
{
    if (N < 0 || L < 1 || P < 0) return 1;
    for (int64_t p = 0; p < P; ++p)
        if (I[p] < 0 || I[p] >= N || J[p] < 0 || J[p] >= N) return 2;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < P; ++p)
        out[p] = oracle_drmsd_pair(X + 3 * L * I[p], X + 3 * L * J[p], L);
    return 0;
}

/* ------------------------------------------------------------- clustering
 * K-means over the all-vs-all matrix (Implementation; Results and
 * Discussion: K-means with k clusters, the representative chosen by the
 * smallest <R>/f).  Only the N(N-1)/2 scores are given, so a cluster centre
 * is one of its members (a medoid): the mean of models under cRMSD is not a
 * function of the matrix.  Alternating steps, from caller-given distinct
 * initial medoids:
 *   assign  every model joins the cluster of its nearest medoid (exact
 *           float32 comparison; ties to the lowest cluster index; a medoid
 *           always joins its own cluster);
 *   update  each cluster's new medoid is the member with the smallest sum of
 *           scores to the other members (ties to the lowest model index);
 * repeated until no medoid changes or max_iter updates have run (then one
 * more assignment).  The sums are plain FP64 sums of the float32 scores in
 * increasing model order.
 * Representative: n_c members, f = n_c / N, <R> = the mean score over the
 * n_c (n_c - 1) / 2 pairs of cluster c; the representative cluster minimises
 * <R> / f (clusters of one model are not eligible; ties to the lowest index)
 * and its medoid is the representative model.
 *
 * Diagnostic (not part of the method): tie_margin receives the smallest, over
 * every update and every cluster of n > 1 members, of (second smallest sum -
 * smallest sum) / (n - 1), i.e. how close any update came to a tie, per
 * summed score (+infinity when no update compared two members). */
static double packed_at(const float *D, int64_t N, int64_t i, int64_t j)
{
    if (i == j) return 0.0;
    if (i > j) { int64_t t = i; i = j; j = t; }
    return (double)D[i * (2 * N - i - 1) / 2 + (j - i - 1)];
}

static void km_assign(const float *D, int64_t N, int64_t k, const int32_t *med, int32_t *label)
{
    for (int64_t i = 0; i < N; ++i) {
        int64_t best = -1;
        for (int64_t c = 0; c < k; ++c)
            if (med[c] == i) { best = c; break; }
        if (best < 0) {
            double bd = 0.0;
            for (int64_t c = 0; c < k; ++c) {
                double d = packed_at(D, N, i, med[c]);
                if (best < 0 || d < bd) { best = c; bd = d; }
            }
        }
        label[i] = (int32_t)best;
    }
}

/* cost[i] = sum over the other members j of i's cluster of D(i, j). */
static void km_costs(const float *D, int64_t N, const int32_t *label, double *cost)
{
    for (int64_t i = 0; i < N; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < N; ++j)
            if (j != i && label[j] == label[i]) s += packed_at(D, N, i, j);
        cost[i] = s;
    }
}

int oracle_kmedoids(const float *D, int64_t N, int64_t k, const int32_t *init, int64_t max_iter,
                    int32_t *label, int32_t *medoid, int64_t *size, double *mean_r,
                    int64_t *info, double *tie_margin)
{
    if (N < 1 || k < 1 || k > N || max_iter < 0) return 1;
    for (int64_t c = 0; c < k; ++c) {
        if (init[c] < 0 || init[c] >= N) return 2;
        for (int64_t e = 0; e < c; ++e)
            if (init[e] == init[c]) return 3;
        medoid[c] = init[c];
    }
    double *cost = malloc(sizeof(double) * N);
    if (!cost) return 4;
    double margin = INFINITY;
    int64_t it = 0, converged = 0;
    while (it < max_iter) {
        km_assign(D, N, k, medoid, label);
        km_costs(D, N, label, cost);
        ++it;
        int changed = 0;
        for (int64_t c = 0; c < k; ++c) {
            int64_t best = -1, n = 0;
            for (int64_t i = 0; i < N; ++i)
                if (label[i] == c) {
                    ++n;
                    if (best < 0 || cost[i] < cost[best]) best = i;
                }
            if (n > 1) {
                double second = INFINITY;
                for (int64_t i = 0; i < N; ++i)
                    if (label[i] == c && i != best && cost[i] < second) second = cost[i];
                const double gap = (second - cost[best]) / (double)(n - 1);
                if (gap < margin) margin = gap;
            }
            if (best != medoid[c]) { medoid[c] = (int32_t)best; changed = 1; }
        }
        if (!changed) { converged = 1; break; }
    }
    if (!converged) {
        km_assign(D, N, k, medoid, label);
        km_costs(D, N, label, cost);
    }
    int64_t rep = -1;
    double rep_score = 0.0;
    for (int64_t c = 0; c < k; ++c) {
        int64_t n = 0;
        double s = 0.0;
        for (int64_t i = 0; i < N; ++i)
            if (label[i] == c) { ++n; s += cost[i]; }
        size[c] = n;
        mean_r[c] = n > 1 ? s / ((double)n * (double)(n - 1)) : 0.0;
        if (n > 1) {
            double score = mean_r[c] * ((double)N / (double)n);
            if (rep < 0 || score < rep_score) { rep = c; rep_score = score; }
        }
    }
    info[0] = rep;
    info[1] = it;
    info[2] = converged;
    if (tie_margin) *tie_margin = margin;
    free(cost);
    return 0;
}

/* -------------------------------------------------------------------- CMO
 * Contact map overlap (Algorithms, Eq. 6-7): atoms p < q of a model are in
 * contact when their distance is below the cut-off, C_pq = [|x_p - x_q| <
 * cutoff]; the score of two models is the Sorensen index of their contact
 * sets, S = 100 * 2 n(A and B) / (n(A) + n(B)), with n the number of
 * contacts.  Each contact is decided on the squared distance
 * u*u + v*v + w*w < cutoff^2 in FP64 (u, v, w the exact FP64 coordinate
 * differences; the library is built without floating-point contraction, so
 * every product and sum is rounded on its own); the counts are integers.
 * S = 0 when neither model has a contact. */
static int in_contact(const double *X, int64_t p, int64_t q, double c2)
{
    const double u = X[3 * p] - X[3 * q];
    const double v = X[3 * p + 1] - X[3 * q + 1];
    const double w = X[3 * p + 2] - X[3 * q + 2];
    return u * u + v * v + w * w < c2;
}

double oracle_cmo_pair(const double *A, const double *B, int64_t L, double cutoff)
{
    const double c2 = cutoff * cutoff;
    int64_t na = 0, nb = 0, nab = 0;
    for (int64_t p = 0; p < L; ++p)
        for (int64_t q = p + 1; q < L; ++q) {
            const int a = in_contact(A, p, q, c2), b = in_contact(B, p, q, c2);
            na += a;
            nb += b;
            nab += a & b;
        }
    if (na + nb == 0) return 0.0;
    return (200.0 * (double)nab) / (double)(na + nb);
}

int oracle_cmo_matrix(const double *X, int64_t N, int64_t L, double cutoff, double *out,
                      int nthreads)
{
    if (N < 0 || L < 1 || !(cutoff >= 0.0)) return 1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < N; ++i) {
        int64_t base = i * (2 * N - i - 1) / 2 - i - 1;
        for (int64_t j = i + 1; j < N; ++j)
            out[base + j] = oracle_cmo_pair(X + 3 * L * i, X + 3 * L * j, L, cutoff);
    }
    return 0;
}

int oracle_cmo_pairs(const double *X, int64_t N, int64_t L, double cutoff, const int64_t *I,
                     const int64_t *J, int64_t P, double *out, int nthreads)
{
    if (N < 0 || L < 1 || P < 0 || !(cutoff >= 0.0)) return 1;
    for (int64_t p = 0; p < P; ++p)
        if (I[p] < 0 || I[p] >= N || J[p] < 0 || J[p] >= N) return 2;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < P; ++p)
        out[p] = oracle_cmo_pair(X + 3 * L * I[p], X + 3 * L * J[p], L, cutoff);
    return 0;
}

/* Diagnostic for comparisons (not part of the method): per model, the number
 * of atom pairs whose squared distance lies within rel * cutoff^2 of
 * cutoff^2, where a differently rounded evaluation of the same squared
 * distance could take the other side of the strict cut-off. */
int oracle_cmo_near_ties(const double *X, int64_t N, int64_t L, double cutoff, double rel,
                         int64_t *count)
{
    if (N < 0 || L < 1 || !(cutoff >= 0.0) || !(rel >= 0.0)) return 1;
    const double c2 = cutoff * cutoff, band = rel * c2;
    for (int64_t m = 0; m < N; ++m) {
        const double *x = X + 3 * L * m;
        int64_t n = 0;
        for (int64_t p = 0; p < L; ++p)
            for (int64_t q = p + 1; q < L; ++q) {
                const double u = x[3 * p] - x[3 * q];
                const double v = x[3 * p + 1] - x[3 * q + 1];
                const double w = x[3 * p + 2] - x[3 * q + 2];
                const double d2 = u * u + v * v + w * w;
                n += fabs(d2 - c2) <= band;
            }
        count[m] = n;
    }
    return 0;
}
