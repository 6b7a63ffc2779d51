/*
 * FP64 Ewald summation for point charges in a periodic cube.
 *
 * TEST INFRASTRUCTURE ONLY: this file belongs to the CPU oracle that checks the
 * GPU library.  Nothing in the product links or loads it.
 *
 * Convention: each sub-Hamiltonian of the paper (the periodic Coulomb sum over
 * all box shifts n, omitting only i=j at n=0) is taken as the Ewald energy with
 * tin-foil boundaries at infinity and a uniform neutralising background, so a
 * charged cell keeps a finite, alpha-independent energy.  The pair kernel is
 *   phi(r) = sum_n erfc(a|r+nL|)/|r+nL| + (4 pi/V) sum_{k!=0} e^{-k^2/4a^2} cos(k.r)/k^2
 *            - pi/(V a^2)
 * and its i=j value (self images only) is lim_{r->0} (phi(r) - 1/r).
 *
 * Entry points (all arrays row-major, double precision):
 *   ew_field : potential and field at target atoms from every charge
 *   ew_pair  : pair kernel phi(r) and G(r) = -grad phi(r) for given displacements
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define PI 3.14159265358979323846
#define TWO_OVER_SQRTPI 1.12837916709551257390

static double wrap1(double x, double L) {
    double w = x - L * floor(x / L);
    if (w >= L) w -= L;
    if (w < 0) w += L;
    return w;
}

typedef struct { int mx, my, mz; double coef; } kvec;

/* Half-space k-vectors with |m|^2 <= mmax^2, coef = 2 * (4 pi / V) exp(-k^2/4a^2)/k^2. */
static kvec *make_kvecs(double L, double alpha, int mmax, int64_t *nk_out) {
    int64_t cap = (int64_t)(2 * mmax + 1) * (2 * mmax + 1) * (mmax + 1);
    kvec *kv = (kvec *)malloc(sizeof(kvec) * (size_t)cap);
    int64_t nk = 0;
    double V = L * L * L;
    for (int mx = 0; mx <= mmax; ++mx)
        for (int my = -mmax; my <= mmax; ++my)
            for (int mz = -mmax; mz <= mmax; ++mz) {
                if (mx == 0 && (my < 0 || (my == 0 && mz <= 0))) continue;
                int m2 = mx * mx + my * my + mz * mz;
                if (m2 > mmax * mmax) continue;
                double k2 = (2 * PI / L) * (2 * PI / L) * m2;
                kv[nk].mx = mx; kv[nk].my = my; kv[nk].mz = mz;
                kv[nk].coef = 2.0 * (4.0 * PI / V) * exp(-k2 / (4 * alpha * alpha)) / k2;
                ++nk;
            }
    *nk_out = nk;
    return kv;
}

/* e^{i 2 pi m x / L} for m = 0..mmax, as (re, im) pairs, by direct cos/sin (no recurrence drift). */
static void phase_table(double x, double L, int mmax, double *t) {
    for (int m = 0; m <= mmax; ++m) {
        double a = 2 * PI * m * x / L;
        t[2 * m] = cos(a);
        t[2 * m + 1] = sin(a);
    }
}

static inline void cmul(double ar, double ai, double br, double bi, double *cr, double *ci) {
    *cr = ar * br - ai * bi;
    *ci = ar * bi + ai * br;
}

/* phase e^{i k.x} for k = (mx,my,mz) from per-axis tables (negative m via conjugation). */
static inline void phase_k(const double *tx, const double *ty, const double *tz, int mx, int my, int mz,
                           double *re, double *im) {
    double ar = tx[2 * mx], ai = tx[2 * mx + 1];
    int ay = my < 0 ? -my : my, az = mz < 0 ? -mz : mz;
    double br = ty[2 * ay], bi = (my < 0 ? -1.0 : 1.0) * ty[2 * ay + 1];
    double cr = tz[2 * az], ci = (mz < 0 ? -1.0 : 1.0) * tz[2 * az + 1];
    double dr, di;
    cmul(ar, ai, br, bi, &dr, &di);
    cmul(dr, di, cr, ci, re, im);
}

int ew_field(int64_t n, const double *x_in, const double *q, double L, double alpha, double rc, int mmax,
             int64_t nt, const int64_t *tgt, double *phi, double *field, int nthreads) {
    if (n <= 0 || L <= 0 || alpha <= 0 || rc <= 0 || mmax < 0) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    double V = L * L * L;
    double *x = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double Q = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) x[3 * i + d] = wrap1(x_in[3 * i + d], L);
        Q += q[i];
    }
    /* ---- real space: cell list ---- */
    int nc = (int)floor(L / rc);
    if (nc < 1) nc = 1;
    if (nc > 256) nc = 256;
    double cs = L / nc;
    int range = (int)ceil(rc / cs);
    int64_t ncell = (int64_t)nc * nc * nc;
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell + 1));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *cellof = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    memset(head, 0, sizeof(int64_t) * (size_t)(ncell + 1));
    for (int64_t i = 0; i < n; ++i) {
        int c[3];
        for (int d = 0; d < 3; ++d) {
            c[d] = (int)floor(x[3 * i + d] / cs);
            if (c[d] >= nc) c[d] = nc - 1;
            if (c[d] < 0) c[d] = 0;
        }
        cellof[i] = ((int64_t)c[0] * nc + c[1]) * nc + c[2];
        head[cellof[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) head[c + 1] += head[c];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
        memcpy(fill, head, sizeof(int64_t) * (size_t)ncell);
        for (int64_t i = 0; i < n; ++i) order[fill[cellof[i]]++] = i;
        free(fill);
    }
    double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = tgt[t];
        double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
        int ci[3] = {(int)(cellof[i] / ((int64_t)nc * nc)), (int)((cellof[i] / nc) % nc), (int)(cellof[i] % nc)};
        double p = 0, ex = 0, ey = 0, ez = 0;
        for (int dx = -range; dx <= range; ++dx)
            for (int dy = -range; dy <= range; ++dy)
                for (int dz = -range; dz <= range; ++dz) {
                    int u[3] = {ci[0] + dx, ci[1] + dy, ci[2] + dz}, w[3];
                    double sh[3];
                    for (int d = 0; d < 3; ++d) {
                        int s = (int)floor((double)u[d] / nc);
                        w[d] = u[d] - s * nc;
                        sh[d] = s * L;
                    }
                    int64_t c = ((int64_t)w[0] * nc + w[1]) * nc + w[2];
                    int self_img = (sh[0] == 0 && sh[1] == 0 && sh[2] == 0);
                    for (int64_t a = head[c]; a < head[c + 1]; ++a) {
                        int64_t j = order[a];
                        if (self_img && j == i) continue;
                        double rx = xi - (x[3 * j] + sh[0]);
                        double ry = yi - (x[3 * j + 1] + sh[1]);
                        double rz = zi - (x[3 * j + 2] + sh[2]);
                        double r2 = rx * rx + ry * ry + rz * rz;
                        if (r2 >= rc2) continue;
                        double r = sqrt(r2);
                        double e = erfc(alpha * r) / r;
                        p += q[j] * e;
                        double f = q[j] * (e + TWO_OVER_SQRTPI * alpha * exp(-alpha * alpha * r2)) / r2;
                        ex += f * rx; ey += f * ry; ez += f * rz;
                    }
                }
        phi[t] = p - TWO_OVER_SQRTPI * alpha * q[i] - PI * Q / (V * alpha * alpha);
        field[3 * t] = ex; field[3 * t + 1] = ey; field[3 * t + 2] = ez;
    }
    free(head); free(order); free(cellof);
    /* ---- reciprocal space ---- */
    int64_t nk;
    kvec *kv = make_kvecs(L, alpha, mmax, &nk);
    if (nk > 0) {
        int nth = omp_get_max_threads();
        double *Sp = (double *)calloc((size_t)nth * 2 * (size_t)nk, sizeof(double));
#pragma omp parallel
        {
            int th = omp_get_thread_num();
            double *S = Sp + (size_t)th * 2 * (size_t)nk;
            double *tx = (double *)malloc(sizeof(double) * 2 * (mmax + 1));
            double *ty = (double *)malloc(sizeof(double) * 2 * (mmax + 1));
            double *tz = (double *)malloc(sizeof(double) * 2 * (mmax + 1));
#pragma omp for schedule(static)
            for (int64_t j = 0; j < n; ++j) {
                phase_table(x[3 * j], L, mmax, tx);
                phase_table(x[3 * j + 1], L, mmax, ty);
                phase_table(x[3 * j + 2], L, mmax, tz);
                for (int64_t k = 0; k < nk; ++k) {
                    double re, im;
                    phase_k(tx, ty, tz, kv[k].mx, kv[k].my, kv[k].mz, &re, &im);
                    S[2 * k] += q[j] * re;
                    S[2 * k + 1] += q[j] * im;
                }
            }
            free(tx); free(ty); free(tz);
        }
        double *S = (double *)calloc(2 * (size_t)nk, sizeof(double));
        for (int th = 0; th < nth; ++th)
            for (int64_t k = 0; k < 2 * nk; ++k) S[k] += Sp[(size_t)th * 2 * (size_t)nk + k];
        free(Sp);
#pragma omp parallel
        {
            double *tx = (double *)malloc(sizeof(double) * 2 * (mmax + 1));
            double *ty = (double *)malloc(sizeof(double) * 2 * (mmax + 1));
            double *tz = (double *)malloc(sizeof(double) * 2 * (mmax + 1));
#pragma omp for schedule(static)
            for (int64_t t = 0; t < nt; ++t) {
                int64_t i = tgt[t];
                phase_table(x[3 * i], L, mmax, tx);
                phase_table(x[3 * i + 1], L, mmax, ty);
                phase_table(x[3 * i + 2], L, mmax, tz);
                double p = 0, ex = 0, ey = 0, ez = 0;
                for (int64_t k = 0; k < nk; ++k) {
                    double re, im;  /* e^{i k.x_i} */
                    phase_k(tx, ty, tz, kv[k].mx, kv[k].my, kv[k].mz, &re, &im);
                    /* e^{i k.x_i} conj(S) */
                    double ar = re * S[2 * k] + im * S[2 * k + 1];
                    double ai = im * S[2 * k] - re * S[2 * k + 1];
                    p += kv[k].coef * ar;
                    double g = kv[k].coef * ai * (2 * PI / L);
                    ex += g * kv[k].mx; ey += g * kv[k].my; ez += g * kv[k].mz;
                }
                phi[t] += p;
                field[3 * t] += ex; field[3 * t + 1] += ey; field[3 * t + 2] += ez;
            }
            free(tx); free(ty); free(tz);
        }
        free(S);
    }
    free(kv);
    free(x);
    return 0;
}

/* Pair kernel phi(r) and G(r) = -grad phi(r).  A zero displacement returns the
 * self-image value lim (phi(r) - 1/r) and G = 0. */
int ew_pair(double L, double alpha, double rc, int mmax, int64_t np, const double *r, double *phi, double *G,
            int nthreads) {
    if (L <= 0 || alpha <= 0 || rc <= 0 || mmax < 0) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    double V = L * L * L;
    int range = (int)ceil(rc / L) + 1;
    int64_t nk;
    kvec *kv = make_kvecs(L, alpha, mmax, &nk);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < np; ++t) {
        double r0[3];
        for (int d = 0; d < 3; ++d) r0[d] = r[3 * t + d] - L * floor(r[3 * t + d] / L + 0.5);  /* periodic */
        int is_zero = (r0[0] == 0 && r0[1] == 0 && r0[2] == 0);
        double p = 0, gx = 0, gy = 0, gz = 0;
        for (int a = -range; a <= range; ++a)
            for (int b = -range; b <= range; ++b)
                for (int c = -range; c <= range; ++c) {
                    if (is_zero && a == 0 && b == 0 && c == 0) continue;
                    double rx = r0[0] + a * L, ry = r0[1] + b * L, rz = r0[2] + c * L;
                    double d2 = rx * rx + ry * ry + rz * rz;
                    if (d2 >= rc * rc) continue;
                    double d = sqrt(d2);
                    double e = erfc(alpha * d) / d;
                    p += e;
                    double f = (e + TWO_OVER_SQRTPI * alpha * exp(-alpha * alpha * d2)) / d2;
                    gx += f * rx; gy += f * ry; gz += f * rz;
                }
        if (is_zero) p -= TWO_OVER_SQRTPI * alpha;
        for (int64_t k = 0; k < nk; ++k) {
            double kx = 2 * PI * kv[k].mx / L, ky = 2 * PI * kv[k].my / L, kz = 2 * PI * kv[k].mz / L;
            double ph = kx * r0[0] + ky * r0[1] + kz * r0[2];
            p += kv[k].coef * cos(ph);
            double s = kv[k].coef * sin(ph);
            gx += s * kx; gy += s * ky; gz += s * kz;
        }
        p -= PI / (V * alpha * alpha);
        phi[t] = p;
        G[3 * t] = gx; G[3 * t + 1] = gy; G[3 * t + 2] = gz;
    }
    free(kv);
    return 0;
}
