/*
 * oracle/dion_kernel.c -- TEST INFRASTRUCTURE (oracle side).  Only tests/,
 * the smoke check and the CPU-baseline leg of the benchmark may load this.
 * Nothing on the HIP product path links, loads or calls it.
 *
 * Two plain FP64 loops that are too slow in NumPy:
 *
 *  1. The universal vdW-DF kernel phi(d1,d2) that Eq. (Enl) integrates
 *     (its form is external to the paper, which only states that it depends
 *     on d1 = q1 r12 and d2 = q2 r12 and that it vanishes when integrated
 *     over a uniform density and decays as r^-6).  Reading used here (Dion
 *     et al. 2004, recalled, validated by the invariants the paper states):
 *
 *       phi(d1,d2) = (2/pi^2) Int_0^inf da Int_0^inf db a^2 b^2 W(a,b)
 *                    T(nu1(a), nu1(b), nu2(a), nu2(b))
 *       W(a,b)     = 2 [ S(a) F(b) + F(a) S(b) - 3 F(a) F(b) ]
 *                    with S(x) = sin x / x,  F(x) = (sin x - x cos x) / x^3
 *                    (algebraically identical to the usual
 *                    2[(3-a^2) b cos b sin a + ...]/(a^3 b^3) form, but free
 *                    of the cancellation at small a, b)
 *       T(w,x,y,z) = 1/2 [1/(w+x) + 1/(y+z)] [1/((w+y)(x+z)) + 1/((w+z)(y+x))]
 *       nu_i(y)    = y^2 / (2 h(y/d_i)),  h(t) = 1 - exp(-4 pi t^2 / 9)
 *
 *     The double integral is a plain weighted double sum over a quadrature
 *     mesh (nodes a_k, weights w_k) that the caller supplies.
 *
 *  2. The radial Fourier transform of a sampled radial function g(D)/D:
 *       out(kappa) = sum_i c_i g_i sin(kappa D_i),  D_i = i dD,
 *     with trapezoid weights c_i (1/2 at both ends); the caller scales it to
 *     4 pi Int D^2 j0(kappa D) Phi(D) dD = (4 pi / kappa) Int D sin(kappa D) Phi dD.
 */
#include <math.h>
#include <stdlib.h>

static const double kPi = 3.14159265358979323846;

/* F(x) = (sin x - x cos x)/x^3, by its Taylor series near 0:
 * sum_{n>=1} (-1)^(n+1) 2n x^(2n-2) / (2n+1)!  */
static double f_over_x3(double x)
{
    if (x < 0.5) {
        double x2 = x * x, term = 1.0 / 3.0, sum = term;
        for (int n = 1; n < 12; ++n) {
            /* ratio of term n+1 to term n */
            term *= -x2 * (double)(n + 1) / ((double)n * (2.0 * n + 2.0) * (2.0 * n + 3.0));
            sum += term;
        }
        return sum;
    }
    return (sin(x) - x * cos(x)) / (x * x * x);
}

static double sinc(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

/* nu(y) = y^2 / (2 h(y/d)) with h(t) = 1 - exp(-gamma t^2). */
static double nu_of(double y, double d)
{
    const double gamma = 4.0 * kPi / 9.0;
    if (d <= 0.0) return 0.5 * y * y; /* h = 1 */
    if (y == 0.0) return d * d / (2.0 * gamma);
    double t = y / d;
    double h = -expm1(-gamma * t * t);
    return y * y / (2.0 * h);
}

/* phi(d1[p], d2[p]) for p < npts, on the quadrature mesh (a, w) of na nodes. */
int oracle_dion_phi(int na, const double *a, const double *w,
                    int npts, const double *d1, const double *d2, double *out)
{
    if (na <= 0 || npts < 0) return -1;
    double *S = (double *)malloc(sizeof(double) * na);
    double *F = (double *)malloc(sizeof(double) * na);
    double *A = (double *)malloc(sizeof(double) * (size_t)na * na);
    if (!S || !F || !A) { free(S); free(F); free(A); return -2; }
    for (int i = 0; i < na; ++i) {
        S[i] = sinc(a[i]);
        F[i] = f_over_x3(a[i]);
    }
    /* A_ij = w_i w_j a_i^2 a_j^2 W(a_i, a_j): independent of d1, d2. */
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < na; ++j) {
            double W = 2.0 * (S[i] * F[j] + F[i] * S[j] - 3.0 * F[i] * F[j]);
            A[(size_t)i * na + j] = w[i] * w[j] * a[i] * a[i] * a[j] * a[j] * W;
        }

    #pragma omp parallel
    {
        double *n1 = (double *)malloc(sizeof(double) * na);
        double *n2 = (double *)malloc(sizeof(double) * na);
        #pragma omp for schedule(dynamic, 1)
        for (int p = 0; p < npts; ++p) {
            for (int i = 0; i < na; ++i) {
                n1[i] = nu_of(a[i], d1[p]);
                n2[i] = nu_of(a[i], d2[p]);
            }
            double total = 0.0;
            for (int i = 0; i < na; ++i) {
                const double wi = n1[i], yi = n2[i];
                const double *Ai = A + (size_t)i * na;
                double row = 0.0;
                /* T(w,x,y,z) with w = nu1(a_i), x = nu1(a_j), y = nu2(a_i), z = nu2(a_j) */
                for (int j = 0; j < na; ++j) {
                    const double xj = n1[j], zj = n2[j];
                    double T = 0.5 * (1.0 / (wi + xj) + 1.0 / (yi + zj)) *
                               (1.0 / ((wi + yi) * (xj + zj)) + 1.0 / ((wi + zj) * (yi + xj)));
                    row += Ai[j] * T;
                }
                total += row;
            }
            out[p] = 2.0 / (kPi * kPi) * total;
        }
        free(n1);
        free(n2);
    }
    free(S); free(F); free(A);
    return 0;
}

/* out[m] = sum_i c_i g[i] sin(kappa[m] D_i),  D_i = i dD,  i < nd, with
 * trapezoid weights c_0 = c_{nd-1} = 1/2, c_i = 1 otherwise.  sin(kappa D_i)
 * is advanced by a rotation and re-evaluated exactly every 64 steps; eight
 * kappa values are advanced together so the loop vectorises. */
int oracle_radial_sine_sum(int nd, double dD, const double *g,
                           int nk, const double *kappa, double *out)
{
    if (nd < 2 || nk < 0) return -1;
    const int nblk = (nk + 7) / 8;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < nblk; ++b) {
        double x[8], cx[8], sx[8], s[8], c[8], sum[8];
        for (int m = 0; m < 8; ++m) {
            int km = b * 8 + m;
            x[m] = (km < nk ? kappa[km] : 0.0) * dD;
            cx[m] = cos(x[m]); sx[m] = sin(x[m]);
            s[m] = 0.0; c[m] = 1.0; sum[m] = 0.0;
        }
        for (int i = 0; i < nd; ++i) {
            if ((i & 63) == 0)
                for (int m = 0; m < 8; ++m) { s[m] = sin(i * x[m]); c[m] = cos(i * x[m]); }
            const double gi = ((i == 0 || i == nd - 1) ? 0.5 : 1.0) * g[i];
            for (int m = 0; m < 8; ++m) {
                sum[m] += gi * s[m];
                double s2 = s[m] * cx[m] + c[m] * sx[m];
                c[m] = c[m] * cx[m] - s[m] * sx[m];
                s[m] = s2;
            }
        }
        for (int m = 0; m < 8; ++m)
            if (b * 8 + m < nk) out[b * 8 + m] = sum[m];
    }
    return 0;
}
