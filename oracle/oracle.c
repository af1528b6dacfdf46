/*
 * FP64 CPU oracle for periodic tricubic B-spline orbital evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * GPU library never includes, links or calls anything here, and this file
 * includes nothing from the library.
 *
 * What it computes (Mathuriya et al., SC'17):
 *  - Section 3: the Slater matrix A(i,j) = phi_i(r_j) needs every orbital at a
 *    proposed position r'_k, and the drift and local energy need its gradient
 *    and Laplacian (Algorithm 1, "ratio" and "derivatives" steps; the local
 *    energy equation).
 *  - Sections 2 and 3: the orbitals are 3D B-splines; the 1D functors are
 *    cubic B-splines.  Section 8.2: the table is a read-only 4-dimensional
 *    array (three grid axes and the orbital index), periodic over the
 *    supercell (Table 1 lists FFT grids of whole unit cells).
 *
 * The paper never writes the basis down.  The reading used here is the
 * uniform cubic tensor-product B-spline with coefficient c_j centred on grid
 * point j (stencil (1,4,1)/6 at the knots), periodic in each axis, with the
 * lower cell taken at knots.  Positions are reduced to the lattice in FP64.
 *
 * Everything below is plain loops in double precision, following the
 * definition term by term: no blocking, no separable shortcuts, no SIMD.
 */
#include <math.h>
#include <omp.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

/* 1D uniform cubic B-spline weights of the four coefficients that touch the
 * cell, at fractional offset t in [0,1], and their first and second
 * derivatives with respect to t. */
void oracle_basis(double t, double b[4], double db[4], double d2b[4])
{
    double s = 1.0 - t;
    b[0] = s * s * s / 6.0;
    b[1] = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
    b[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
    b[3] = t * t * t / 6.0;

    db[0] = -s * s / 2.0;
    db[1] = (3.0 * t * t - 4.0 * t) / 2.0;
    db[2] = (-3.0 * t * t + 2.0 * t + 1.0) / 2.0;
    db[3] = t * t / 2.0;

    d2b[0] = s;
    d2b[1] = 3.0 * t - 2.0;
    d2b[2] = 1.0 - 3.0 * t;
    d2b[3] = t;
}

/* Reduce one Cartesian coordinate to (cell index, fractional offset).
 * Periodic wrap, then the lower cell; u landing exactly on n is clamped to
 * the last cell with t = 1.  A non-finite coordinate yields cell 0 and t = NaN
 * so that the outputs are NaN and no index leaves the table. */
void oracle_reduce(double r, double cell, int32_t n, int32_t *i, double *t)
{
    if (!isfinite(r)) {
        *i = 0;
        *t = NAN;
        return;
    }
    double f = r / cell;
    f = f - floor(f);
    if (f >= 1.0)
        f = 0.0;
    double u = (double)n * f;
    double fl = floor(u);
    int32_t ii = (int32_t)fl;
    if (ii > n - 1)
        ii = n - 1;
    if (ii < 0)
        ii = 0;
    *i = ii;
    *t = u - (double)ii;
}

static int64_t wrap(int64_t j, int64_t n)
{
    j %= n;
    return j < 0 ? j + n : j;
}

/* Value, gradient and Laplacian of all norb orbitals at B positions.
 *   n[3], cell[3]   grid points and orthorhombic cell lengths per axis
 *   coefs           [n0][n1][n2][norb], orbital index fastest
 *   pos             [B][3]
 *   V [B][norb], G [B][3][norb], L [B][norb]   (outputs, overwritten)
 *   nthreads        OpenMP threads over positions (<= 0: runtime default)
 * Returns 0, or -1 on bad sizes. */
int oracle_eval_vgl(const int32_t n[3], const double cell[3], int32_t norb,
                    const double *coefs, int64_t B, const double *pos,
                    double *V, double *G, double *L, int32_t nthreads)
{
    if (norb <= 0 || B < 0 || n[0] <= 0 || n[1] <= 0 || n[2] <= 0)
        return -1;
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
    for (int64_t b = 0; b < B; ++b) {
        int32_t i[3];
        double t[3], a[3][4], da[3][4], d2a[3][4];
        for (int d = 0; d < 3; ++d) {
            oracle_reduce(pos[3 * b + d], cell[d], n[d], &i[d], &t[d]);
            oracle_basis(t[d], a[d], da[d], d2a[d]);
            double g = (double)n[d] / cell[d];
            for (int k = 0; k < 4; ++k) {
                da[d][k] *= g;
                d2a[d][k] *= g * g;
            }
        }
        double *v = V + b * norb;
        double *gx = G + (3 * b + 0) * norb;
        double *gy = G + (3 * b + 1) * norb;
        double *gz = G + (3 * b + 2) * norb;
        double *l = L + b * norb;
        for (int32_t m = 0; m < norb; ++m) {
            v[m] = 0.0;
            gx[m] = 0.0;
            gy[m] = 0.0;
            gz[m] = 0.0;
            l[m] = 0.0;
        }
        for (int k0 = 0; k0 < 4; ++k0)
            for (int k1 = 0; k1 < 4; ++k1)
                for (int k2 = 0; k2 < 4; ++k2) {
                    int64_t j0 = wrap((int64_t)i[0] + k0 - 1, n[0]);
                    int64_t j1 = wrap((int64_t)i[1] + k1 - 1, n[1]);
                    int64_t j2 = wrap((int64_t)i[2] + k2 - 1, n[2]);
                    const double *c = coefs + ((j0 * n[1] + j1) * n[2] + j2) * (int64_t)norb;
                    double wv = a[0][k0] * a[1][k1] * a[2][k2];
                    double wx = da[0][k0] * a[1][k1] * a[2][k2];
                    double wy = a[0][k0] * da[1][k1] * a[2][k2];
                    double wz = a[0][k0] * a[1][k1] * da[2][k2];
                    double wl = d2a[0][k0] * a[1][k1] * a[2][k2] +
                                a[0][k0] * d2a[1][k1] * a[2][k2] +
                                a[0][k0] * a[1][k1] * d2a[2][k2];
                    for (int32_t m = 0; m < norb; ++m) {
                        v[m] += wv * c[m];
                        gx[m] += wx * c[m];
                        gy[m] += wy * c[m];
                        gz[m] += wz * c[m];
                        l[m] += wl * c[m];
                    }
                }
    }
    return 0;
}

/* Value only at B positions (the quadrature-point evaluation of the
 * non-local pseudopotential, Section 3): V [B][norb]. */
int oracle_eval_v(const int32_t n[3], const double cell[3], int32_t norb,
                  const double *coefs, int64_t B, const double *pos, double *V,
                  int32_t nthreads)
{
    if (norb <= 0 || B < 0 || n[0] <= 0 || n[1] <= 0 || n[2] <= 0)
        return -1;
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
    for (int64_t b = 0; b < B; ++b) {
        int32_t i[3];
        double t[3], a[3][4], da[3][4], d2a[3][4];
        for (int d = 0; d < 3; ++d) {
            oracle_reduce(pos[3 * b + d], cell[d], n[d], &i[d], &t[d]);
            oracle_basis(t[d], a[d], da[d], d2a[d]);
        }
        double *v = V + b * norb;
        for (int32_t m = 0; m < norb; ++m)
            v[m] = 0.0;
        for (int k0 = 0; k0 < 4; ++k0)
            for (int k1 = 0; k1 < 4; ++k1)
                for (int k2 = 0; k2 < 4; ++k2) {
                    int64_t j0 = wrap((int64_t)i[0] + k0 - 1, n[0]);
                    int64_t j1 = wrap((int64_t)i[1] + k1 - 1, n[1]);
                    int64_t j2 = wrap((int64_t)i[2] + k2 - 1, n[2]);
                    const double *c = coefs + ((j0 * n[1] + j1) * n[2] + j2) * (int64_t)norb;
                    double wv = a[0][k0] * a[1][k1] * a[2][k2];
                    for (int32_t m = 0; m < norb; ++m)
                        v[m] += wv * c[m];
                }
    }
    return 0;
}

/* Round x to the nearest number with p significant bits whose leading-bit
 * exponent is at least emin (below that, a fixed spacing 2^(emin-p+1):
 * gradual underflow), ties to even.  Division by a power of two is exact, and
 * nearbyint rounds to nearest-even in the default rounding mode. */
double oracle_round_sig(double x, int32_t p, int32_t emin)
{
    if (x == 0.0 || !isfinite(x))
        return x;
    int e;
    frexp(x, &e); /* x = m 2^e, 0.5 <= |m| < 1: leading bit is 2^(e-1) */
    int lead = e - 1;
    if (lead < emin)
        lead = emin;
    double ulp = ldexp(1.0, lead - (p - 1));
    return nearbyint(x / ulp) * ulp;
}

/* Storage formats: 0 FP64, 1 FP32, 2 BF16, 3 FP16 (Section 7.2: reduced
 * precision for the table and its evaluation, precision-critical steps in
 * double).  16-bit formats store c / s_m with a power-of-two per-orbital
 * scale s_m = 2^ceil(log2 max_j |c_jm|) (1 for an all-zero orbital), so the
 * stored magnitudes lie in [0, 1].  Writes the dequantized table
 * s_m * q(c / s_m) into out (same shape as coefs) and s_m into scales. */
int oracle_dequantize(const double *coefs, int64_t npts, int32_t norb, int32_t fmt,
                      double *out, double *scales)
{
    if (npts < 0 || norb <= 0 || fmt < 0 || fmt > 3)
        return -1;
    for (int32_t m = 0; m < norb; ++m) {
        double s = 1.0;
        if (fmt >= 2) {
            double mx = 0.0;
            for (int64_t j = 0; j < npts; ++j) {
                double a = fabs(coefs[j * norb + m]);
                if (a > mx)
                    mx = a;
            }
            if (mx > 0.0) {
                /* smallest power of two >= mx */
                int e;
                double f = frexp(mx, &e);
                s = ldexp(1.0, f == 0.5 ? e - 1 : e);
            }
        }
        scales[m] = s;
    }
    for (int64_t j = 0; j < npts; ++j)
        for (int32_t m = 0; m < norb; ++m) {
            double c = coefs[j * norb + m];
            double q;
            switch (fmt) {
            case 0: q = c; break;
            case 1: q = oracle_round_sig(c, 24, -126); break;
            case 2: q = oracle_round_sig(c / scales[m], 8, -126) * scales[m]; break;
            default: q = oracle_round_sig(c / scales[m], 11, -14) * scales[m]; break;
            }
            out[j * norb + m] = q;
        }
    return 0;
}

/* Inverse of a 3x3 matrix by cofactors; returns the determinant (0 means
 * singular and inv is left unset). */
static double inverse3(const double m[9], double inv[9])
{
    double c00 = m[4] * m[8] - m[5] * m[7];
    double c01 = m[5] * m[6] - m[3] * m[8];
    double c02 = m[3] * m[7] - m[4] * m[6];
    double det = m[0] * c00 + m[1] * c01 + m[2] * c02;
    if (det == 0.0 || !isfinite(det))
        return 0.0;
    inv[0] = c00 / det;
    inv[1] = (m[2] * m[7] - m[1] * m[8]) / det;
    inv[2] = (m[1] * m[5] - m[2] * m[4]) / det;
    inv[3] = c01 / det;
    inv[4] = (m[0] * m[8] - m[2] * m[6]) / det;
    inv[5] = (m[2] * m[3] - m[0] * m[5]) / det;
    inv[6] = c02 / det;
    inv[7] = (m[1] * m[6] - m[0] * m[7]) / det;
    inv[8] = (m[0] * m[4] - m[1] * m[3]) / det;
    return det;
}

/* Value, gradient and full Hessian of all orbitals in a general (triclinic)
 * cell: the Bspline-vgh evaluation of Sections 3 and 8 (the paper's kernel
 * forms the Hessian, which a non-orthogonal cell needs for its Laplacian).
 *   lat[9]   row-major; row d is the Cartesian lattice vector a_d, along which
 *            the n[d] grid points run.  A position r = sum_d u_d a_d has
 *            fractional coordinates u = r Lat^-1; the spline is periodic in
 *            each u_d with period 1 and is evaluated at t_d = n_d frac(u_d).
 *   G [B][3][norb]: d/dr_c = sum_d Lat^-1[c][d] d/du_d
 *   H [B][6][norb]: xx, xy, xz, yy, yz, zz of
 *            d2/dr_c dr_e = sum_{d,d'} Lat^-1[c][d] Lat^-1[e][d'] d2/du_d du_d'
 * with d/du_d = n_d d/dt_d.  Returns 0, or -1 on bad sizes or a singular
 * lattice. */
int oracle_eval_vgh(const int32_t n[3], const double lat[9], int32_t norb,
                    const double *coefs, int64_t B, const double *pos,
                    double *V, double *G, double *H, int32_t nthreads)
{
    double inv[9];
    if (norb <= 0 || B < 0 || n[0] <= 0 || n[1] <= 0 || n[2] <= 0)
        return -1;
    if (inverse3(lat, inv) == 0.0)
        return -1;
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
    int fail = 0;
#pragma omp parallel num_threads(nt)
    {
        /* per-thread sums in the fractional frame: du[3][norb], duu[3][3][norb] */
        double *acc = (double *)malloc(sizeof(double) * 12 * (size_t)norb);
        if (!acc) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t b = 0; b < B; ++b) {
            if (!acc)
                continue;
            int32_t i[3];
            double t[3], a[3][4], da[3][4], d2a[3][4];
            for (int d = 0; d < 3; ++d) {
                double u = pos[3 * b + 0] * inv[0 * 3 + d] + pos[3 * b + 1] * inv[1 * 3 + d] +
                           pos[3 * b + 2] * inv[2 * 3 + d];
                oracle_reduce(u, 1.0, n[d], &i[d], &t[d]);
                oracle_basis(t[d], a[d], da[d], d2a[d]);
                for (int k = 0; k < 4; ++k) {
                    da[d][k] *= (double)n[d];
                    d2a[d][k] *= (double)n[d] * (double)n[d];
                }
            }
            double *v = V + b * norb;
            double *du = acc;             /* du[d][m] */
            double *duu = acc + 3 * norb; /* duu[d][e][m] */
            for (int32_t m = 0; m < norb; ++m)
                v[m] = 0.0;
            for (int64_t x = 0; x < 12 * (int64_t)norb; ++x)
                acc[x] = 0.0;
            for (int k0 = 0; k0 < 4; ++k0)
                for (int k1 = 0; k1 < 4; ++k1)
                    for (int k2 = 0; k2 < 4; ++k2) {
                        int64_t j0 = wrap((int64_t)i[0] + k0 - 1, n[0]);
                        int64_t j1 = wrap((int64_t)i[1] + k1 - 1, n[1]);
                        int64_t j2 = wrap((int64_t)i[2] + k2 - 1, n[2]);
                        const double *c = coefs + ((j0 * n[1] + j1) * n[2] + j2) * (int64_t)norb;
                        /* f[d][o]: the order-o basis factor of axis d (o = 0, 1, 2) */
                        const double f[3][3] = {{a[0][k0], da[0][k0], d2a[0][k0]},
                                                {a[1][k1], da[1][k1], d2a[1][k1]},
                                                {a[2][k2], da[2][k2], d2a[2][k2]}};
                        double w = f[0][0] * f[1][0] * f[2][0];
                        double w1[3], w2[3][3];
                        for (int d = 0; d < 3; ++d) {
                            int o[3] = {0, 0, 0};
                            o[d] = 1;
                            w1[d] = f[0][o[0]] * f[1][o[1]] * f[2][o[2]];
                            for (int e = 0; e < 3; ++e) {
                                int p[3] = {0, 0, 0};
                                p[d] += 1;
                                p[e] += 1;
                                w2[d][e] = f[0][p[0]] * f[1][p[1]] * f[2][p[2]];
                            }
                        }
                        for (int32_t m = 0; m < norb; ++m) {
                            v[m] += w * c[m];
                            for (int d = 0; d < 3; ++d) {
                                du[d * norb + m] += w1[d] * c[m];
                                for (int e = 0; e < 3; ++e)
                                    duu[(d * 3 + e) * norb + m] += w2[d][e] * c[m];
                            }
                        }
                    }
            /* chain rule to Cartesian */
            static const int hc[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
            for (int32_t m = 0; m < norb; ++m) {
                for (int c = 0; c < 3; ++c) {
                    double s = 0.0;
                    for (int d = 0; d < 3; ++d)
                        s += inv[c * 3 + d] * du[d * norb + m];
                    G[(3 * b + c) * norb + m] = s;
                }
                for (int h = 0; h < 6; ++h) {
                    int c = hc[h][0], e = hc[h][1];
                    double s = 0.0;
                    for (int d = 0; d < 3; ++d)
                        for (int d2 = 0; d2 < 3; ++d2)
                            s += inv[c * 3 + d] * inv[e * 3 + d2] * duu[(d * 3 + d2) * norb + m];
                    H[(6 * b + h) * norb + m] = s;
                }
            }
        }
        free(acc);
    }
    return fail ? -1 : 0;
}
