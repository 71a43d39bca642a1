/*
 * sw_oracle.c -- plain FP64 CPU oracle for rigid alignment in sliced
 * 2-Wasserstein distance (Shi, Singer, Verbeke, "Fast rigid alignment of
 * heterogeneous images in sliced Wasserstein distance").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU path.
 *
 * Every step is the plain definition, written for a reader to check against
 * the paper by eye: direct hat-weighted line sums, a direct cumulative sum and
 * inversion, and a direct O(n^2 Q) scan over the rotation grid.  No FFT is
 * used anywhere; the FFT route of the paper reaches the same numbers up to
 * rounding order.  OpenMP is used only across independent images or pairs;
 * one image or one pair is always handled by one thread in a fixed order, so
 * results are deterministic.
 *
 * Conventions (the paper is silent on these; readings listed in the design
 * notes of the repository):
 *   pixel (i, j) of a row-major L x L image sits at (x_j, y_i) with
 *   x_j = (j - (L-1)/2) h, y_i = (i - (L-1)/2) h, h = 2/L   (App. A, pixel grid)
 *   only pixels with x^2 + y^2 <= (1-h)^2 are used; negative values are
 *   clipped to 0 (Sec. 4.4 keeps the positive part of noisy images)
 *   angles theta_k = 2 pi k / n                              (App. A)
 *   detector direction d_k = (cos theta_k, -sin theta_k), from the projection
 *   operator P_theta f(x) = int f(R_theta^T (x, y)) dy            (Sec. 2)
 *   detector bins b = 0..L-1, centres s_b = -1 + (b + 1/2) h, edges
 *   t_b = -1 + b h                                           (App. A, E3 part)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846264338327950288

/* per-result status codes (same meaning as the library's, written here
   independently) */
#define OR_STATUS_OK 0
#define OR_STATUS_ZERO_MASS 1
#define OR_STATUS_NONFINITE 2

/* Angle table: cos/sin of theta_k = 2 pi k / n.  Evaluated in FP64 on the
   first octant and completed by the exact symmetries of the circle, so that
   d_{k+n/4} is d_k turned by 90 degrees and d_{k+n/2} = -d_k bit for bit.
   For n not divisible by 8 only the quarter-turn symmetry is used. */
static void oracle_angles(int n, double *cs, double *sn)
{
    if (n % 4 != 0) {
        for (int k = 0; k < n; ++k) {
            double t = 2.0 * OR_PI * (double)k / (double)n;
            cs[k] = cos(t);
            sn[k] = sin(t);
        }
        return;
    }
    int q = n / 4;
    for (int k = 0; k < q; ++k) {
        if (n % 8 == 0 && k > n / 8) {
            /* theta_k = pi/2 - theta_{q-k} */
            double t = 2.0 * OR_PI * (double)(q - k) / (double)n;
            cs[k] = sin(t);
            sn[k] = cos(t);
        } else {
            double t = 2.0 * OR_PI * (double)k / (double)n;
            cs[k] = cos(t);
            sn[k] = sin(t);
        }
    }
    cs[0] = 1.0;
    sn[0] = 0.0;
    /* quarter turns: theta + pi/2 -> (cos, sin) = (-sin, cos) */
    for (int r = 1; r < 4; ++r)
        for (int k = 0; k < q; ++k) {
            cs[r * q + k] = -sn[(r - 1) * q + k];
            sn[r * q + k] = cs[(r - 1) * q + k];
        }
}

/* Disk mask in exact integer arithmetic: x^2 + y^2 <= (1-h)^2 with
   x = (2j - L + 1)/L, y = (2i - L + 1)/L and 1 - h = (L - 2)/L. */
static int oracle_in_disk(int L, int i, int j)
{
    long a = 2L * j - L + 1, b = 2L * i - L + 1, r = L - 2;
    return a * a + b * b <= r * r;
}

/* a1-a2: line projection by hat-weighted line sums (Sec. 2.3: columns of U
   are the 1-D projections at the n angles; projection operator of Sec. 2).
   P[k][b] = sum over masked pixels of F+(i,j) * max(0, 1 - |(p.d_k - s_b)/h|).
   Equivalently the pixel deposits into bins floor(tau) and floor(tau)+1 with
   tau = (p.d_k + 1)/h - 1/2, the two weights being 1 - frac and frac.
   img: [N][L][L] float (promoted to double), pmf: [N][n][L] double.
   nonfinite: [N] (nullable) set to 1 when the image holds a non-finite value. */
void oracle_project(const float *img, int64_t N, int L, int n, double *pmf, int32_t *nonfinite)
{
    double *cs = (double *)malloc(sizeof(double) * n);
    double *sn = (double *)malloc(sizeof(double) * n);
    oracle_angles(n, cs, sn);
    const double h = 2.0 / (double)L;
#pragma omp parallel for schedule(dynamic)
    for (int64_t g = 0; g < N; ++g) {
        const float *F = img + g * (int64_t)L * L;
        double *P = pmf + g * (int64_t)n * L;
        memset(P, 0, sizeof(double) * (size_t)n * L);
        int bad = 0;
        for (int64_t t = 0; t < (int64_t)L * L; ++t)
            if (!isfinite(F[t])) bad = 1;
        if (nonfinite) nonfinite[g] = bad;
        for (int k = 0; k < n; ++k) {
            double dx = cs[k], dy = -sn[k];
            for (int i = 0; i < L; ++i) {
                double y = ((double)i - 0.5 * (L - 1)) * h;
                for (int j = 0; j < L; ++j) {
                    if (!oracle_in_disk(L, i, j)) continue;
                    double v = (double)F[(int64_t)i * L + j];
                    if (!(v > 0.0)) continue; /* positive part; also drops NaN */
                    double x = ((double)j - 0.5 * (L - 1)) * h;
                    double tau = (x * dx + y * dy + 1.0) / h - 0.5;
                    double m = floor(tau);
                    double fr = tau - m;
                    int b = (int)m;
                    /* the mask keeps tau inside [1/2, L - 3/2]; the guards
                       only protect against rounding at the edge */
                    if (b >= 0 && b < L) P[(int64_t)k * L + b] += (1.0 - fr) * v;
                    if (b + 1 >= 0 && b + 1 < L) P[(int64_t)k * L + b + 1] += fr * v;
                }
            }
        }
    }
    free(cs);
    free(sn);
}

/* a3-a5: CDF by cumulative sum, quantiles by linear interpolation of the CDF,
   and the per-image scalars.  (Sec. 2.3, CDF and ICDF of each column; the
   1-D W2 closed form and the generalised inverse inf{t : F(t) >= z} of
   App. A.)
     m_k = sum_b P[k][b];  C[k][b] = (sum_{b' <= b} P[k][b']) / m_k,  C[k][-1] = 0
     levels z_j = (j + 1/2)/Q  (levels == 0)  or  z_j = j/Q  (levels == 1)
     b* = min{ b : C[k][b] >= z_j }   (L-1 if none)
     U[j][k] = t_{b*} + h (z_j - C[k][b*-1]) / (C[k][b*] - C[k][b*-1]),
               clamped to [t_{b*}, t_{b*+1}]
   aux[g][0] = image mass (sum of the clipped, masked pixels; NaN when the
               image holds a non-finite value)
   aux[g][1] = E = sum_{j,k} U[j][k]^2
   aux[g][2..3] = a = (1/n) sum_k ubar_k d_k, with ubar_k = (1/Q) sum_j U[j][k]
   pmf: [N][n][L], qt: [N][Q][n], aux: [N][4] (nullable). */
/* Quantiles of one nonnegative column P[0..L) at the Q levels, written to
   U[j * ldu] (j < Q); returns the column mass m.  C: L + 1 doubles of
   scratch (C[b+1] holds the CDF at the right edge of bin b). */
static double oracle_invert_column(const double *P, int L, int Q, int levels, double *U,
                                   int64_t ldu, double *C)
{
    const double h = 2.0 / (double)L;
    double m = 0.0;
    for (int b = 0; b < L; ++b) m += P[b];
    C[0] = 0.0;
    double run = 0.0;
    for (int b = 0; b < L; ++b) {
        run += P[b];
        C[b + 1] = (m > 0.0) ? run / m : 0.0;
    }
    for (int j = 0; j < Q; ++j) {
        double z = (levels == 1) ? (double)j / (double)Q : ((double)j + 0.5) / (double)Q;
        int bs = L - 1;
        for (int b = 0; b < L; ++b)
            if (C[b + 1] >= z) {
                bs = b;
                break;
            }
        double tl = -1.0 + (double)bs * h, tr = -1.0 + (double)(bs + 1) * h;
        double den = C[bs + 1] - C[bs];
        double u = (den > 0.0) ? tl + h * (z - C[bs]) / den : tl;
        if (u < tl) u = tl;
        if (u > tr) u = tr;
        U[(int64_t)j * ldu] = u;
    }
    return m;
}

/* E = sum of squares of a [rows][n] table and a = (1/n) sum_k ubar_k d_k with
   ubar_k the mean of column k over the rows. */
static void oracle_table_scalars(const double *U, int rows, int n, const double *cs,
                                 const double *sn, double *A)
{
    double E = 0.0, ar = 0.0, ai = 0.0;
    for (int j = 0; j < rows; ++j)
        for (int k = 0; k < n; ++k) E += U[(int64_t)j * n + k] * U[(int64_t)j * n + k];
    for (int k = 0; k < n; ++k) {
        double ub = 0.0;
        for (int j = 0; j < rows; ++j) ub += U[(int64_t)j * n + k];
        ub /= (double)rows;
        ar += ub * cs[k];
        ai += ub * (-sn[k]);
    }
    A[1] = E;
    A[2] = ar / (double)n;
    A[3] = ai / (double)n;
}

void oracle_quantiles(const double *pmf, int64_t N, int L, int n, int Q, int levels,
                      const int32_t *nonfinite, double *qt, double *aux)
{
    double *cs = (double *)malloc(sizeof(double) * n);
    double *sn = (double *)malloc(sizeof(double) * n);
    oracle_angles(n, cs, sn);
#pragma omp parallel for schedule(dynamic)
    for (int64_t g = 0; g < N; ++g) {
        const double *P = pmf + g * (int64_t)n * L;
        double *U = qt + g * (int64_t)Q * n;
        double *C = (double *)malloc(sizeof(double) * (L + 1));
        double mass0 = 0.0;
        for (int k = 0; k < n; ++k) {
            double m = oracle_invert_column(P + (int64_t)k * L, L, Q, levels, U + k, n, C);
            if (k == 0) mass0 = m;
        }
        free(C);
        if (aux) {
            double *A = aux + 4 * g;
            oracle_table_scalars(U, Q, n, cs, sn, A);
            A[0] = (nonfinite && nonfinite[g]) ? NAN : mass0;
        }
    }
    free(cs);
    free(sn);
}

/* Ramp filter (Sec. 2.2, optional high-pass step: the slice is multiplied by
   |xi| in the Fourier domain before the inverse transform).  Discretised as
   the filter |xi| sampled on the M = 2L point frequency grid of the detector
   (DC term zero) and applied to each column zero-padded to length M, i.e. the
   cyclic convolution with the kernel
     h[m] = (1/M) sum_{w=0}^{M-1} min(w, M - w) cos(2 pi w m / M)
   read on the L detector bins:
     Pf[k][b] = sum_{b'} h[(b - b') mod M] P[k][b'].
   Any positive scale of the filter drops out when each signed part is
   normalised.  pmf, out: [N][n][L]. */
void oracle_ramp(const double *pmf, int64_t N, int L, int n, double *out)
{
    const int M = 2 * L;
    double *hk = (double *)malloc(sizeof(double) * M);
    for (int m = 0; m < M; ++m) {
        double acc = 0.0;
        for (int w = 0; w < M; ++w) {
            int a = w < M - w ? w : M - w;
            acc += (double)a * cos(2.0 * OR_PI * (double)((int64_t)w * m % M) / (double)M);
        }
        hk[m] = acc / (double)M;
    }
#pragma omp parallel for schedule(dynamic)
    for (int64_t c = 0; c < N * (int64_t)n; ++c) {
        const double *P = pmf + c * L;
        double *R = out + c * L;
        for (int b = 0; b < L; ++b) {
            double acc = 0.0;
            for (int bp = 0; bp < L; ++bp) acc += hk[((b - bp) % M + M) % M] * P[bp];
            R[b] = acc;
        }
    }
    free(hk);
}

/* The filter kernel itself, for tests against its closed form. */
void oracle_ramp_kernel(int L, double *hk)
{
    const int M = 2 * L;
    for (int m = 0; m < M; ++m) {
        double acc = 0.0;
        for (int w = 0; w < M; ++w) {
            int a = w < M - w ? w : M - w;
            acc += (double)a * cos(2.0 * OR_PI * (double)((int64_t)w * m % M) / (double)M);
        }
        hk[m] = acc / (double)M;
    }
}

/* Quantile tables of ramp-filtered projections (ramp-filtered SW of Sec. 2.3
   and its appendix): each filtered column is split into its positive part
   max(Pf, 0) and its (absolute) negative part max(-Pf, 0), each part is
   normalised to unit mass and inverted like a plain projection.  The two
   tables are stacked: rows 0..Q-1 positive part, rows Q..2Q-1 negative part.
   aux[g][0] = the smallest part mass over all columns (0 when a part is empty
   somewhere; NaN for a non-finite image), aux[1..3] = E and a of the stacked
   [2Q][n] table.  pf: [N][n][L], qt: [N][2Q][n]. */
void oracle_quantiles_rf(const double *pf, int64_t N, int L, int n, int Q, int levels,
                         const int32_t *nonfinite, double *qt, double *aux)
{
    double *cs = (double *)malloc(sizeof(double) * n);
    double *sn = (double *)malloc(sizeof(double) * n);
    oracle_angles(n, cs, sn);
#pragma omp parallel for schedule(dynamic)
    for (int64_t g = 0; g < N; ++g) {
        const double *P = pf + g * (int64_t)n * L;
        double *U = qt + g * (int64_t)2 * Q * n;
        double *C = (double *)malloc(sizeof(double) * (L + 1));
        double *part = (double *)malloc(sizeof(double) * L);
        double mmin = INFINITY;
        for (int k = 0; k < n; ++k) {
            for (int sgn = 0; sgn < 2; ++sgn) {
                for (int b = 0; b < L; ++b) {
                    double v = P[(int64_t)k * L + b];
                    part[b] = sgn == 0 ? (v > 0.0 ? v : 0.0) : (v < 0.0 ? -v : 0.0);
                }
                double m = oracle_invert_column(part, L, Q, levels, U + (int64_t)sgn * Q * n + k,
                                                n, C);
                if (m < mmin) mmin = m;
            }
        }
        free(C);
        free(part);
        if (aux) {
            double *A = aux + 4 * g;
            oracle_table_scalars(U, 2 * Q, n, cs, sn, A);
            A[0] = (nonfinite && nonfinite[g]) ? NAN : mmin;
        }
    }
    free(cs);
    free(sn);
}

/* D(l, s) = (1/(nQ)) sum_k sum_j (U[j][k] - V[j][(k+l) mod n] - s.d_k)^2,
   the discrete SW2 of Sec. 2.3 between f and T_s R_{theta_l} g: a cyclic
   column shift is a rotation (Sec. 2.3, fast computation over rotations) and
   a translation adds s.d_k to every quantile of column k (proof of Thm 3.2,
   App. B).  j runs over the `rows` rows of the tables: Q for SW2, 2Q for the
   stacked tables of the ramp-filtered distance, whose objective is the sum
   of the two parts' objectives (each normalised by nQ). */
static double oracle_objective(const double *U, const double *V, int n, int Q, int rows, int l,
                               double sx, double sy, const double *cs, const double *sn)
{
    double acc = 0.0;
    for (int k = 0; k < n; ++k) {
        int kl = (k + l) % n;
        double shift = sx * cs[k] + sy * (-sn[k]);
        for (int j = 0; j < rows; ++j) {
            double r = U[(int64_t)j * n + k] - V[(int64_t)j * n + kl] - shift;
            acc += r * r;
        }
    }
    return acc / ((double)n * (double)Q);
}

/* Max-sliced objective at lag l (extended alignment results: the max-sliced
   W2 over the equispaced slices, the norm of U - V taken over columns):
     M(l) = max_k (1/Q) sum_j (U[j][k] - V[j][(k+l) mod n])^2,
   the largest per-angle W2^2 between f and R_{theta_l} g.  Rotation only:
   the shift that minimises a maximum has no closed form. */
static double oracle_max_sliced(const double *U, const double *V, int n, int Q, int rows, int l)
{
    double best = 0.0;
    for (int k = 0; k < n; ++k) {
        int kl = (k + l) % n;
        double acc = 0.0;
        for (int j = 0; j < rows; ++j) {
            double r = U[(int64_t)j * n + k] - V[(int64_t)j * n + kl];
            acc += r * r;
        }
        acc /= (double)Q;
        if (acc > best) best = acc;
    }
    return best;
}

/* a6-a10: exhaustive search over the rotation grid with the least-squares
   translation at every rotation, then the argmin (Sec. 2.3, discrete SW2
   over rotations; Thm 3.2 for the translation).
   For each lag l:
     b(l)  = (1/n) sum_k (ubar_k - vbar_{(k+l) mod n}) d_k
     s*(l) = 2 b(l)       (minimiser of D(l, .), using sum_k d_k d_k^T = (n/2) I)
     D*(l) = D(l, s*(l))  (mode 0, rotation + translation)
     D*(l) = D(l, 0)      (mode 1, rotation only: the paper's own objective)
     D*(l) = M(l)         (mode 2, max-sliced, rotation only, s* = 0)
   (With `rows` table rows and the 1/(nQ) normalisation,
   D(l, s) = D(l, 0) - (2 rows/Q) s.b(l) + (rows/(2Q)) |s|^2, so s*(l) = 2 b(l)
   for the stacked ramp-filtered tables as well.)
   l* = argmin D*(l), ties to the smallest l.
   Outputs per pair: out_l[p] = l*, out_s[p][2] = s*(l*) in pixels (x along
   +column, y along +row), out_d[p] = D*(l*), status[p], curve[p][n] = D*(.)
   (nullable), shift_curve[p][n][2] = s*(.) in pixels (nullable; zero in
   modes 1 and 2).  pairs: [P][2] (ref index, img index) or NULL for all ref x img
   in row-major order (p = r * n_img + g). */
void oracle_align_rows(const double *ref_qt, const double *ref_aux, int64_t n_ref,
                       const double *img_qt, const double *img_aux, int64_t n_img,
                       const int64_t *pairs, int64_t n_pairs, int L, int n, int Q, int rows,
                       int mode, int32_t *out_l, double *out_s, double *out_d, int32_t *status,
                       double *curve, double *shift_curve)
{
    double *cs = (double *)malloc(sizeof(double) * n);
    double *sn = (double *)malloc(sizeof(double) * n);
    oracle_angles(n, cs, sn);
    const double h = 2.0 / (double)L;
    int64_t P = pairs ? n_pairs : n_ref * n_img;
#pragma omp parallel for schedule(dynamic)
    for (int64_t p = 0; p < P; ++p) {
        int64_t r = pairs ? pairs[2 * p] : p / n_img;
        int64_t g = pairs ? pairs[2 * p + 1] : p % n_img;
        const double *U = ref_qt + r * (int64_t)rows * n;
        const double *V = img_qt + g * (int64_t)rows * n;
        double mr = ref_aux[4 * r], mg = img_aux[4 * g];
        int st = OR_STATUS_OK;
        if (isnan(mr) || isnan(mg)) st = OR_STATUS_NONFINITE;
        else if (!(mr > 0.0) || !(mg > 0.0)) st = OR_STATUS_ZERO_MASS;
        status[p] = st;
        if (st != OR_STATUS_OK) {
            out_l[p] = 0;
            out_s[2 * p] = out_s[2 * p + 1] = 0.0;
            out_d[p] = NAN;
            if (curve)
                for (int l = 0; l < n; ++l) curve[p * n + l] = NAN;
            continue;
        }
        double *ub = (double *)malloc(sizeof(double) * n);
        double *vb = (double *)malloc(sizeof(double) * n);
        for (int k = 0; k < n; ++k) {
            double su = 0.0, sv = 0.0;
            for (int j = 0; j < rows; ++j) {
                su += U[(int64_t)j * n + k];
                sv += V[(int64_t)j * n + k];
            }
            ub[k] = su / (double)rows;
            vb[k] = sv / (double)rows;
        }
        int best = -1;
        double bestd = 0.0, bsx = 0.0, bsy = 0.0;
        for (int l = 0; l < n; ++l) {
            double sx = 0.0, sy = 0.0;
            if (mode == 0) {
                double bx = 0.0, by = 0.0;
                for (int k = 0; k < n; ++k) {
                    double dd = ub[k] - vb[(k + l) % n];
                    bx += dd * cs[k];
                    by += dd * (-sn[k]);
                }
                sx = 2.0 * bx / (double)n;
                sy = 2.0 * by / (double)n;
            }
            double d = mode == 2 ? oracle_max_sliced(U, V, n, Q, rows, l)
                                 : oracle_objective(U, V, n, Q, rows, l, sx, sy, cs, sn);
            if (curve) curve[p * n + l] = d;
            if (shift_curve) {
                shift_curve[2 * (p * n + l)] = sx / h;
                shift_curve[2 * (p * n + l) + 1] = sy / h;
            }
            if (best < 0 || d < bestd) {
                best = l;
                bestd = d;
                bsx = sx;
                bsy = sy;
            }
        }
        free(ub);
        free(vb);
        out_l[p] = best;
        out_s[2 * p] = bsx / h;
        out_s[2 * p + 1] = bsy / h;
        out_d[p] = bestd;
    }
    free(cs);
    free(sn);
}

void oracle_align(const double *ref_qt, const double *ref_aux, int64_t n_ref,
                  const double *img_qt, const double *img_aux, int64_t n_img,
                  const int64_t *pairs, int64_t n_pairs, int L, int n, int Q, int mode,
                  int32_t *out_l, double *out_s, double *out_d, int32_t *status, double *curve)
{
    oracle_align_rows(ref_qt, ref_aux, n_ref, img_qt, img_aux, n_img, pairs, n_pairs, L, n, Q, Q,
                      mode, out_l, out_s, out_d, status, curve, NULL);
}

/* D(l, s) for one table pair at arbitrary (l, s), s in unit coordinates:
   exposed so that tests can minimise over s numerically and compare with the
   closed form above. */
double oracle_objective_at(const double *U, const double *V, int n, int Q, int rows, int l,
                           double sx, double sy)
{
    double *cs = (double *)malloc(sizeof(double) * n);
    double *sn = (double *)malloc(sizeof(double) * n);
    oracle_angles(n, cs, sn);
    double d = oracle_objective(U, V, n, Q, rows, l, sx, sy, cs, sn);
    free(cs);
    free(sn);
    return d;
}

/* The angle table itself, for tests of its symmetry. */
void oracle_angle_table(int n, double *cs, double *sn) { oracle_angles(n, cs, sn); }

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
