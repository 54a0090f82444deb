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
 *  3. The brute-force real-space double sum of Eq. (Enl) on a periodic grid
 *     with the soft kernel phi_s of Eq. (PhiSoft), no interpolation in q:
 *       sum_i sum_j sum_L n_i n_j phi_s(q_i r, q_j r),  r = |r_j - r_i + L|,
 *     0 < r < rcut, phi_s from a table over (angle, log D) supplied by the
 *     caller (see oracle/bruteforce.py), plus the continuum limit of the sum
 *     beyond rcut from the tabulated tail integral of phi_s along each ray.
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

/* ---------------------------------------------------------------- 3 */

/* cubic Lagrange weights for nodes 0, 1, 2, 3 at position t */
static void lag4w(double t, double w[4])
{
    w[0] = -(t - 1.0) * (t - 2.0) * (t - 3.0) / 6.0;
    w[1] = t * (t - 2.0) * (t - 3.0) / 2.0;
    w[2] = -t * (t - 1.0) * (t - 3.0) / 2.0;
    w[3] = t * (t - 1.0) * (t - 2.0) / 6.0;
}

/* first of 4 stencil nodes around fractional index x on n nodes, and the
 * position of x relative to it */
static int stencil(double x, int n, double *t)
{
    int i = (int)floor(x) - 1;
    if (i < 0) i = 0;
    if (i > n - 4) i = n - 4;
    *t = x - i;
    return i;
}

typedef struct {
    int nth, nu;
    double th0, dth, u0, du, dmax, ds, phi0, casym;
    const double *tab, *p2, *p4;   /* tab[k * nu + m]: phi at angle th0 + k dth, D = exp(u0 + m du) */
    const double *cum;             /* cum[k * nu + m]: 4 pi Int_{D_m}^inf D^2 phi_s dD on that ray */
} soft_table;

/* 4 pi Int_D^inf D'^2 phi_s(D') dD' on the ray of angle th (D >= d_s) */
static double tail_integral(const soft_table *T, double th, double D)
{
    double t, wt[4], s, wu[4];
    const int k = stencil((th - T->th0) / T->dth, T->nth, &t);
    lag4w(t, wt);
    const int m = stencil((log(D) - T->u0) / T->du, T->nu, &s);
    lag4w(s, wu);
    double v = 0.0;
    for (int a = 0; a < 4; ++a) {
        const double *row = T->cum + (size_t)(k + a) * T->nu + m;
        v += wt[a] * (wu[0] * row[0] + wu[1] * row[1] + wu[2] * row[2] + wu[3] * row[3]);
    }
    return v;
}

/* phi_s(d1, d2): soft polynomial below d_s (coefficients interpolated in the
 * angle), the table up to dmax, the asymptote beyond. */
static double phi_soft(const soft_table *T, double d1, double d2)
{
    const double D = sqrt(d1 * d1 + d2 * d2);
    if (D == 0.0) return T->phi0;
    const double lo = d1 < d2 ? d1 : d2, hi = d1 < d2 ? d2 : d1;
    if (D > T->dmax) return -T->casym / (d1 * d1 * d2 * d2 * (d1 * d1 + d2 * d2));
    const double th = atan2(lo, hi);   /* in [0, pi/4]: phi is symmetric */
    double t, wt[4];
    const int k = stencil((th - T->th0) / T->dth, T->nth, &t);
    lag4w(t, wt);
    if (D < T->ds) {
        double p2 = 0.0, p4 = 0.0;
        for (int a = 0; a < 4; ++a) { p2 += wt[a] * T->p2[k + a]; p4 += wt[a] * T->p4[k + a]; }
        const double D2 = D * D;
        return T->phi0 + p2 * D2 + p4 * D2 * D2;
    }
    double s, wu[4];
    const int m = stencil((log(D) - T->u0) / T->du, T->nu, &s);
    lag4w(s, wu);
    double v = 0.0;
    for (int a = 0; a < 4; ++a) {
        const double *row = T->tab + (size_t)(k + a) * T->nu + m;
        v += wt[a] * (wu[0] * row[0] + wu[1] * row[1] + wu[2] * row[2] + wu[3] * row[3]);
    }
    return v;
}

/* out[0] = sum over (i, j, L), 0 < r < rcut, of n_i n_j phi_s(q_i r, q_j r);
 * out[1] = sum_i n_i^2 phi_s(0, 0) (r = 0);
 * out[2] = the continuum limit beyond rcut:
 *          sum_{i,j} n_i n_j (1/Omega) Int_{r > rcut} 4 pi r^2 phi_s(q_i r, q_j r) dr
 *          = sum_{i,j} n_i n_j I(angle, rcut Q) / (Q^3 Omega),  Q = |(q_i, q_j)|,
 *          with I the tabulated tail integral along the ray (rcut Q >= d_s).
 * Grid [n1][n2][n3] (C order) in an orthorhombic cell. */
int oracle_bf_energy(int n1, int n2, int n3, const double *cell, const double *n, const double *q, double rcut,
                     int nth, double th0, double dth, int nu, double u0, double du, double dmax,
                     const double *tab, const double *p2, const double *p4, const double *cum, double ds,
                     double phi0, double casym, double *out)
{
    if (n1 < 1 || n2 < 1 || n3 < 1 || nth < 4 || nu < 4 || !(rcut > 0.0)) return -1;
    soft_table T = {nth, nu, th0, dth, u0, du, dmax, ds, phi0, casym, tab, p2, p4, cum};
    const int N = n1 * n2 * n3;
    const double h[3] = {cell[0] / n1, cell[1] / n2, cell[2] / n3};
    const int na[3] = {(int)ceil(rcut / cell[0]) + 1, (int)ceil(rcut / cell[1]) + 1, (int)ceil(rcut / cell[2]) + 1};
    const double omega = cell[0] * cell[1] * cell[2];
    const double r2c = rcut * rcut;
    double s_pair = 0.0, s_self = 0.0, s_tail = 0.0;
    #pragma omp parallel for schedule(dynamic, 8) reduction(+ : s_pair, s_self, s_tail)
    for (int i = 0; i < N; ++i) {
        const int i1 = i / (n2 * n3), i2 = (i / n3) % n2, i3 = i % n3;
        const double qi = q[i], ni = n[i];
        s_self += ni * ni * phi0;
        for (int j = i; j < N; ++j) {
            const int j1 = j / (n2 * n3), j2 = (j / n3) % n2, j3 = j % n3;
            const double qj = q[j], nj = n[j];
            const double mult = (j == i) ? 1.0 : 2.0;    /* (i, j) and (j, i) */
            const double dx = (j1 - i1) * h[0], dy = (j2 - i2) * h[1], dz = (j3 - i3) * h[2];
            double acc = 0.0;
            for (int a = -na[0]; a <= na[0]; ++a) {
                const double x = dx + a * cell[0];
                if (fabs(x) >= rcut) continue;
                for (int b = -na[1]; b <= na[1]; ++b) {
                    const double y = dy + b * cell[1];
                    const double xy = x * x + y * y;
                    if (xy >= r2c) continue;
                    for (int c = -na[2]; c <= na[2]; ++c) {
                        const double z = dz + c * cell[2];
                        const double r2 = xy + z * z;
                        if (r2 >= r2c || r2 == 0.0) continue;
                        const double r = sqrt(r2);
                        acc += phi_soft(&T, qi * r, qj * r);
                    }
                }
            }
            s_pair += mult * ni * nj * acc;
            const double Q = sqrt(qi * qi + qj * qj);
            const double th = atan2(qi < qj ? qi : qj, qi < qj ? qj : qi);
            s_tail += mult * ni * nj * tail_integral(&T, th, rcut * Q) / (Q * Q * Q * omega);
        }
    }
    out[0] = s_pair;
    out[1] = s_self;
    out[2] = s_tail;
    return 0;
}

/* phi_s(d1[p], d2[p]) from the same table (for the factorisation check) */
int oracle_phi_soft(int npts, const double *d1, const double *d2, int nth, double th0, double dth, int nu,
                    double u0, double du, double dmax, const double *tab, const double *p2, const double *p4,
                    double ds, double phi0, double casym, double *out)
{
    if (npts < 0 || nth < 4 || nu < 4) return -1;
    soft_table T = {nth, nu, th0, dth, u0, du, dmax, ds, phi0, casym, tab, p2, p4, 0};
    for (int p = 0; p < npts; ++p) out[p] = phi_soft(&T, d1[p], d2[p]);
    return 0;
}

