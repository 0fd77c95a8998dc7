/*
 * gavis_oracle.c -- plain, slow FP64 reference of the GAVIS visibility-field
 * path.  TEST INFRASTRUCTURE ONLY: nothing in the product library links,
 * loads or calls this file.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.
 *
 * What it computes (GAVIS, "Uncertainty-driven 3D Gaussian Splatting Active
 * Mapping via Anisotropic Visibility Field"):
 *   - real spherical harmonics and the vMF/SH constants   (Appendix, derivation
 *     of the vMF coefficients; eq. vmf_coeff, eq. vis_real)
 *   - single-view particle visibility                      (Appendix, Alg. 2)
 *   - visibility-field construction                        (Alg. 3, eq. vis_gamma)
 *   - visibility-field query with the AM-GM bound          (Alg. 1 / Alg. 4, eq. vis_bound)
 *   - exact multi-view visibility, the quantity the field  (eq. vis_all with eq. vis_p)
 *     and the bound approximate (validation mode)
 *   - per-Gaussian colour covariance from SH-coefficient   (Appendix, integration with FisherRF)
 *     variances, in place of the constant Q_c
 *   - expected depth per pixel under the same weights      (eq. id: the d_p^mn of f_corr)
 *   - uncertainty-quantification rasterisation             (Alg. 6, eq. alpha_comp, eq. huber)
 *   - view score and next-best-view argmax                 (eq. i_gain, eq. id with f_corr = 0)
 *
 * No tiling: every pixel gathers its own list of overlapping Gaussians, sorts
 * it by (depth, index) and composites it front to back.  Projection is the
 * EWA splatting used by 3D Gaussian Splatting (the paper builds on a modified
 * 3DGS rasteriser, Appendix on visibility-field construction).
 *
 * Readings where the paper is silent (kept identical on the GPU side):
 * alpha = o * exp(-m/2) with m the Mahalanobis distance
 * under the 2D covariance; "overlapping" means m <= cut (cut = 9, 3 sigma);
 * termination is T < eps_T tested after the update; depth is camera-space z,
 * and the depth order is decided on z rounded to FP32 (the kernels' sort-key
 * precision), ties by index; directions are camera centre -> particle; the SH
 * frame is the world frame.
 *
 * Parity flags.  Where an FP32 evaluation can take a different discrete
 * decision than this FP64 one (a pair near the overlap boundary, a
 * transmittance near eps_T, a depth that another FP64 evaluation order could
 * round to a neighbouring FP32 key), the oracle marks the
 * affected pixel (query) or Gaussian (build) so that the comparison can
 * leave it out and report how many were left out.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_LMAX 8

/* ------------------------------------------------------------------------ */
/* Special functions                                                        */
/* ------------------------------------------------------------------------ */

/* Modified spherical Bessel function of the first kind, i_l(x), from its
 * power series  i_l(x) = x^l * sum_k (x^2/2)^k / (k! (2l+2k+1)!!).
 * Used for the vMF expansion coefficients (eq. bl, eq. vmf_coeff). */
double ora_bessel_i(int l, double x)
{
    if (l < 0) return 0.0;
    double dfact = 1.0; /* (2l+1)!! */
    for (int j = 1; j <= 2 * l + 1; j += 2) dfact *= (double)j;
    double lead = pow(x, (double)l) / dfact;
    double term = 1.0, sum = 1.0, h = 0.5 * x * x;
    for (int k = 1; k < 400; ++k) {
        term *= h / ((double)k * (double)(2 * l + 2 * k + 1));
        sum += term;
        if (fabs(term) < 1e-18 * fabs(sum)) break;
    }
    return lead * sum;
}

/* Expansion constant a_l = 4 pi zeta i_l(kappa), zeta = exp(-kappa)
 * (Alg. 3 precomputation; eq. vis_gamma). */
double ora_a_l(int l, double kappa)
{
    return 4.0 * M_PI * exp(-kappa) * ora_bessel_i(l, kappa);
}

/* Associated Legendre function P_l^m(x), m >= 0, with the Condon-Shortley
 * phase (-1)^m included.  s = sqrt(1 - x^2) is passed in to keep accuracy
 * near the poles. */
static double assoc_legendre(int l, int m, double x, double s)
{
    double pmm = 1.0;
    double f = 1.0;
    for (int i = 1; i <= m; ++i) {
        pmm *= -f * s;
        f += 2.0;
    }
    if (l == m) return pmm;
    double pm1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pm1;
    double pl = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pl = ((2.0 * ll - 1.0) * x * pm1 - (ll + m - 1.0) * pmm) / (double)(ll - m);
        pmm = pm1;
        pm1 = pl;
    }
    return pl;
}

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return f;
}

/* Real spherical harmonics Y_lm(d) for l <= L, written exactly as the paper
 * defines them from the complex Y_l^m (Appendix, eq. vis_real and the real
 * basis that follows it):
 *   m < 0 : sqrt(2) (-1)^m Im[Y_l^{|m|}]
 *   m = 0 : Y_l^0
 *   m > 0 : sqrt(2) (-1)^m Re[Y_l^m]
 * with Y_l^m = N_lm P_l^m(cos theta) e^{i m phi}, theta the polar angle from
 * world +z and phi = atan2(y, x).  Output index k = l^2 + l + m. */
int ora_sh_real(int L, const double *dir, double *out)
{
    if (L < 0 || L > ORA_LMAX) return -1;
    double nrm = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    if (!(nrm > 0.0)) return -1;
    double x = dir[0] / nrm, y = dir[1] / nrm, z = dir[2] / nrm;
    double s = sqrt(x * x + y * y);
    double phi = atan2(y, x);
    for (int l = 0; l <= L; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double N = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
            double P = assoc_legendre(l, am, z, s);
            double sign = (am % 2) ? -1.0 : 1.0; /* (-1)^m, same for m and -m */
            double v;
            if (m < 0)
                v = sqrt(2.0) * sign * N * P * sin(am * phi);   /* Im[e^{i|m|phi}] */
            else if (m == 0)
                v = N * P;
            else
                v = sqrt(2.0) * sign * N * P * cos(am * phi);   /* Re[e^{i m phi}] */
            out[l * l + l + m] = v;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Camera and EWA projection                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    double R[9], t[3];   /* world -> camera, x_c = R x_w + t, row major */
    double fx, fy, cx, cy;
    int w, h;
    double C[3];         /* camera centre in world coordinates, -R^T t */
} ocam;

static void load_cam(ocam *c, const double *R, const double *t, const double *K, const int32_t *wh)
{
    memcpy(c->R, R, 9 * sizeof(double));
    memcpy(c->t, t, 3 * sizeof(double));
    c->fx = K[0]; c->fy = K[1]; c->cx = K[2]; c->cy = K[3];
    c->w = wh[0]; c->h = wh[1];
    for (int i = 0; i < 3; ++i)
        c->C[i] = -(R[0 * 3 + i] * t[0] + R[1 * 3 + i] * t[1] + R[2 * 3 + i] * t[2]);
}

typedef struct {
    int ok;
    double z, ux, uy;
    double ca, cb, cc;   /* conic = inverse 2D covariance [[ca, cb], [cb, cc]] */
    double sxx, syy;     /* 2D covariance diagonal (for the ellipse bounding box) */
} oproj;

/* EWA projection of one Gaussian: camera transform, 3D covariance
 * (R_q S)(R_q S)^T, Jacobian of the perspective map, 2D covariance plus a
 * low-pass dilation, and its inverse (the "conic" of Alg. 2 / Alg. 6). */
static void project_one(const double *mean, const double *scale, const double *quat,
                        const ocam *c, double lowpass, double znear, oproj *o)
{
    o->ok = 0;
    double p[3];
    for (int i = 0; i < 3; ++i)
        p[i] = c->R[i * 3 + 0] * mean[0] + c->R[i * 3 + 1] * mean[1] + c->R[i * 3 + 2] * mean[2] + c->t[i];
    double z = p[2];
    o->z = z;
    if (!(z > znear)) return;

    double qn = sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
    if (!(qn > 0.0)) return;
    double w = quat[0] / qn, x = quat[1] / qn, y = quat[2] / qn, zq = quat[3] / qn;
    double Rq[9] = {
        1 - 2 * (y * y + zq * zq), 2 * (x * y - w * zq),     2 * (x * zq + w * y),
        2 * (x * y + w * zq),     1 - 2 * (x * x + zq * zq), 2 * (y * zq - w * x),
        2 * (x * zq - w * y),     2 * (y * zq + w * x),     1 - 2 * (x * x + y * y)};
    double M[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i * 3 + j] = Rq[i * 3 + j] * scale[j];
    double S3[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += M[i * 3 + k] * M[j * 3 + k];
            S3[i * 3 + j] = acc;
        }
    double J[6] = {c->fx / z, 0.0, -c->fx * p[0] / (z * z),
                   0.0, c->fy / z, -c->fy * p[1] / (z * z)};
    double W[6]; /* J R */
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += J[i * 3 + k] * c->R[k * 3 + j];
            W[i * 3 + j] = acc;
        }
    double WS[6];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += W[i * 3 + k] * S3[k * 3 + j];
            WS[i * 3 + j] = acc;
        }
    double S2[4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += WS[i * 3 + k] * W[j * 3 + k];
            S2[i * 2 + j] = acc;
        }
    double a = S2[0] + lowpass, b = 0.5 * (S2[1] + S2[2]), cc = S2[3] + lowpass;
    double det = a * cc - b * b;
    if (!(det > 1e-12)) return;
    o->ca = cc / det;
    o->cb = -b / det;
    o->cc = a / det;
    o->sxx = a;
    o->syy = cc;
    o->ux = c->fx * p[0] / z + c->cx;
    o->uy = c->fy * p[1] / z + c->cy;
    o->ok = 1;
}

static inline double mahal2(const oproj *o, double qx, double qy)
{
    double dx = qx - o->ux, dy = qy - o->uy;
    return o->ca * dx * dx + 2.0 * o->cb * dx * dy + o->cc * dy * dy;
}

/* ------------------------------------------------------------------------ */
/* Per-pixel lists (no tiling)                                               */
/* ------------------------------------------------------------------------ */

/* A list entry: a Gaussian that overlaps the pixel (kind 0) or a "ghost" that
 * lies just outside the overlap boundary (kind 1, kept only so that the parity
 * flags know where a boundary flip would sit in depth order). */
typedef struct {
    double z;       /* depth, FP64 */
    double zk;      /* depth key: z rounded to FP32 (the precision the order is decided in) */
    double m;
    int32_t g;
    int32_t kind;   /* 0 real, 1 ghost */
    int32_t near;   /* 1 if |m - cut| is inside the FP32 error band */
    int32_t zamb;   /* 1 if z lies so close to an FP32 rounding midpoint that
                       another FP64 evaluation order may round it the other way */
} oentry;

/* The depth order "sorted by increasing z" is a discrete decision taken on a
 * floating-point value; it is taken here in the precision of the kernels'
 * sort keys (FP32 z, ties by index), so both sides order every pixel's list
 * identically.  The key is ambiguous only when z sits within 1e-12 |z| of a
 * rounding midpoint (a differently ordered FP64 evaluation may land on the
 * other side); such entries are flagged when a neighbour's key is equal or
 * adjacent. */
static void depth_key(double z, double *zk, int32_t *zamb)
{
    float f = (float)z;
    double d = z - (double)f;
    double mid = d >= 0.0 ? 0.5 * ((double)f + (double)nextafterf(f, INFINITY))
                          : 0.5 * ((double)f + (double)nextafterf(f, -INFINITY));
    *zk = (double)f;
    *zamb = fabs(z - mid) <= 1e-12 * fabs(z);
}

/* 1 if the FP32 keys of a and b may order them differently in another
 * evaluation: one key is ambiguous and they are equal or adjacent. */
static int depth_tie(const oentry *a, const oentry *b)
{
    if (!a->zamb && !b->zamb) return 0;
    float fa = (float)a->zk, fb = (float)b->zk;
    return fa == fb || nextafterf(fa, INFINITY) == fb || nextafterf(fb, INFINITY) == fa;
}

typedef struct {
    int64_t *start;  /* [npix + 1] */
    oentry *e;
} olists;

/* Work counts of one rasterisation, for the parity of the composited pair
 * count: every (pixel, Gaussian) pair composited before termination, the
 * list entries, and the same split by whether a near-tie decision touches
 * the pixel (there an FP32 evaluation may composite a different number of
 * pairs, at most the pixel's list length with its ghosts). */
typedef struct {
    int64_t pairs;            /* pairs composited */
    int64_t entries;          /* list entries (overlapping pairs, ghosts included) */
    int64_t pairs_clean;      /* pairs composited on pixels without a near-tie flag */
    int64_t entries_flagged;  /* list entries of flagged pixels */
    int64_t px_flagged;       /* pixels with a near-tie flag */
    int64_t px;               /* pixels */
} ocount;

static void count_add(ocount *a, const ocount *b)
{
    a->pairs += b->pairs; a->entries += b->entries; a->pairs_clean += b->pairs_clean;
    a->entries_flagged += b->entries_flagged; a->px_flagged += b->px_flagged; a->px += b->px;
}

static int cmp_entry(const void *pa, const void *pb)
{
    const oentry *a = (const oentry *)pa, *b = (const oentry *)pb;
    if (a->zk < b->zk) return -1;
    if (a->zk > b->zk) return 1;
    if (a->g < b->g) return -1;
    if (a->g > b->g) return 1;
    return 0;
}

/* FP32 error band on the Mahalanobis test, per (pixel, Gaussian) pair.  It
 * models a single-precision evaluation that keeps the centre relative to a
 * tile origin (|u_local| <= ORA_TILE_MAX + |d|) and evaluates m as a sum of
 * two squares of a rounded Cholesky factor of the conic:
 *   dm <= 2 sqrt(cut lambda_max) (ulp(u_local) + ulp(d)) + 2 cut (8 sqrt(cond) + 16) eps
 * with eps = 2^-24.  Pairs with |m - cut| below this band may be decided the
 * other way in FP32. */
#define ORA_TILE_MAX 32.0
#define ORA_EPS32 5.9604644775390625e-08

static double ulp32(double x)
{
    x = fabs(x);
    if (x < 1e-30) return 1e-45;
    int ex;
    frexp(x, &ex);                   /* x = f 2^ex, f in [0.5, 1) */
    return ldexp(1.0, ex - 24);
}

static void conic_eigs(const oproj *o, double *lmax, double *cond)
{
    double tr = o->ca + o->cc;
    double disc = sqrt((o->ca - o->cc) * (o->ca - o->cc) + 4 * o->cb * o->cb);
    double l1 = 0.5 * (tr + disc), l2 = 0.5 * (tr - disc);
    if (l2 < 1e-300) l2 = 1e-300;
    *lmax = l1;
    *cond = l1 / l2;
}

static double m_band_pair(const oproj *o, double cut, double dx, double dy)
{
    double lmax, cond;
    conic_eigs(o, &lmax, &cond);
    double d = fabs(dx) > fabs(dy) ? fabs(dx) : fabs(dy);
    return 2.0 * sqrt(cut * lmax) * (ulp32(ORA_TILE_MAX + d) + ulp32(d))
         + 2.0 * cut * (8.0 * sqrt(cond) + 16.0) * ORA_EPS32;
}

/* largest band over the ellipse, to size the ghost search box */
static double m_band_max(const oproj *o, double cut)
{
    double r = 3.0 * sqrt((o->sxx > o->syy ? o->sxx : o->syy) * (cut / 9.0)) + 2.0;
    return m_band_pair(o, cut, r, r);
}

/* Gather the per-pixel lists of one view.  mode 0: scatter each Gaussian over
 * the pixels of its ellipse bounding box (plus a one-pixel margin) and test
 * each; mode 1: brute force, every pixel tests every Gaussian.  Both apply the
 * same geometric predicate m <= cut, so they must agree exactly. */
static int gather(const oproj *P, int64_t n, const ocam *c, double cut, int mode, int with_ghosts, olists *L)
{
    int64_t npix = (int64_t)c->w * c->h;
    L->start = (int64_t *)calloc((size_t)npix + 1, sizeof(int64_t));
    if (!L->start) return -1;
    int64_t *cnt = L->start + 1;
    for (int pass = 0; pass < 2; ++pass) {
        int64_t *fill = NULL;
        if (pass == 1) {
            for (int64_t i = 0; i < npix; ++i) L->start[i + 1] += L->start[i];
            L->e = (oentry *)malloc(sizeof(oentry) * (size_t)(L->start[npix] > 0 ? L->start[npix] : 1));
            fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)npix);
            if (!L->e || !fill) { free(fill); return -1; }
            memcpy(fill, L->start, sizeof(int64_t) * (size_t)npix);
        }
        if (mode == 0) {
            for (int64_t g = 0; g < n; ++g) {
                const oproj *o = &P[g];
                if (!o->ok) continue;
                double bmax = with_ghosts ? m_band_max(o, cut) : 0.0;
                double rx = sqrt((cut + bmax) * o->sxx), ry = sqrt((cut + bmax) * o->syy);
                double fi0 = floor(o->ux - rx - 0.5) - 1, fi1 = ceil(o->ux + rx - 0.5) + 1;
                double fj0 = floor(o->uy - ry - 0.5) - 1, fj1 = ceil(o->uy + ry - 0.5) + 1;
                if (fi1 < 0 || fj1 < 0 || fi0 > c->w - 1 || fj0 > c->h - 1) continue;
                int i0 = fi0 < 0 ? 0 : (int)fi0, i1 = fi1 > c->w - 1 ? c->w - 1 : (int)fi1;
                int j0 = fj0 < 0 ? 0 : (int)fj0, j1 = fj1 > c->h - 1 ? c->h - 1 : (int)fj1;
                for (int j = j0; j <= j1; ++j)
                    for (int i = i0; i <= i1; ++i) {
                        double m = mahal2(o, i + 0.5, j + 0.5);
                        double band = with_ghosts ? m_band_pair(o, cut, i + 0.5 - o->ux, j + 0.5 - o->uy) : 0.0;
                        int real = m <= cut;
                        int near = fabs(m - cut) < band;
                        if (!real && !near) continue;
                        int64_t pix = (int64_t)j * c->w + i;
                        if (pass == 0) { cnt[pix]++; continue; }
                        oentry *e = &L->e[fill[pix]++];
                        e->z = o->z; depth_key(o->z, &e->zk, &e->zamb); e->m = m; e->g = (int32_t)g; e->kind = real ? 0 : 1; e->near = near;
                    }
            }
        } else {
            for (int64_t pix = 0; pix < npix; ++pix) {
                int i = (int)(pix % c->w), j = (int)(pix / c->w);
                for (int64_t g = 0; g < n; ++g) {
                    const oproj *o = &P[g];
                    if (!o->ok) continue;
                    double m = mahal2(o, i + 0.5, j + 0.5);
                    double band = with_ghosts ? m_band_pair(o, cut, i + 0.5 - o->ux, j + 0.5 - o->uy) : 0.0;
                    int real = m <= cut;
                    int near = fabs(m - cut) < band;
                    if (!real && !near) continue;
                    if (pass == 0) { cnt[pix]++; continue; }
                    oentry *e = &L->e[fill[pix]++];
                    e->z = o->z; depth_key(o->z, &e->zk, &e->zamb); e->m = m; e->g = (int32_t)g; e->kind = real ? 0 : 1; e->near = near;
                }
            }
        }
        if (pass == 1) free(fill);
    }
    /* sort every pixel's list by increasing depth, index as the tie break */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t pix = 0; pix < npix; ++pix) {
        int64_t s = L->start[pix], e = L->start[pix + 1];
        if (e - s > 1) qsort(&L->e[s], (size_t)(e - s), sizeof(oentry), cmp_entry);
    }
    return 0;
}

static void free_lists(olists *L)
{
    free(L->start);
    free(L->e);
    L->start = NULL;
    L->e = NULL;
}

/* relative band on the termination test */
#define ORA_TBAND 1e-4

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Projection of every Gaussian into one view, for per-Gaussian parity checks.
 * out[g*10 + ...] = ok, z, ux, uy, ca, cb, cc, sxx, syy, band. */
int ora_project_view(int64_t n, const double *means, const double *scales, const double *quats,
                     const double *camR, const double *camT, const double *camK, const int32_t *camWH,
                     double znear, double lowpass, double cut, double *out)
{
    ocam c;
    load_cam(&c, camR, camT, camK, camWH);
    for (int64_t g = 0; g < n; ++g) {
        oproj o;
        project_one(&means[3 * g], &scales[3 * g], &quats[4 * g], &c, lowpass, znear, &o);
        double *r = &out[10 * g];
        r[0] = o.ok; r[1] = o.z;
        r[2] = o.ok ? o.ux : 0; r[3] = o.ok ? o.uy : 0;
        r[4] = o.ok ? o.ca : 0; r[5] = o.ok ? o.cb : 0; r[6] = o.ok ? o.cc : 0;
        r[7] = o.ok ? o.sxx : 0; r[8] = o.ok ? o.syy : 0;
        r[9] = o.ok ? m_band_max(&o, cut) : 0;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Single-view particle visibility (Alg. 2) and VF construction (Alg. 3)     */
/* ------------------------------------------------------------------------ */

/* Alg. 2 for one view, with no tiling.  Per pixel, walk the depth-sorted list
 * of overlapping Gaussians: each reached Gaussian receives the current
 * transmittance and a count, then T <- T (1 - alpha); stop once T < eps_T.
 * Then v_g = (sum of T) / count where count > 0, else 0.
 *
 * Parity bookkeeping: pert[g] is a first-order bound on how far v_g can move
 * when an FP32 evaluation takes one of the near-tie decisions the other way:
 *   - own events (g's own pixel enters or leaves its count: a boundary pair,
 *     or the pixel's termination point): |dv| <= (T_x + v) / max(c - 1, 1);
 *   - downstream events (an earlier boundary flip or depth swap in the same
 *     pixel rescales the T that g receives): |dv| <= |dT| / c. */
static int single_view_visibility(const oproj *P, const double *opac, int64_t n, const ocam *c,
                                  double eps_T, double cut, int mode,
                                  double *v, int64_t *cnt, double *pert,
                                  ocount *counts, int32_t *pxpairs, uint8_t *pxflags)
{
    olists L = {0, 0};
    if (gather(P, n, c, cut, mode, 1, &L)) { free_lists(&L); return -1; }
    int64_t npix = (int64_t)c->w * c->h;
    int nth = ora_num_threads();
    size_t tot = (size_t)nth * (size_t)n + 1;
    double *sumT_t = (double *)calloc(tot, sizeof(double));
    double *dS_t = (double *)calloc(tot, sizeof(double));
    double *own_t = (double *)calloc(tot, sizeof(double));
    int64_t *cnt_t = (int64_t *)calloc(tot, sizeof(int64_t));
    int64_t *ownn_t = (int64_t *)calloc(tot, sizeof(int64_t));
    int64_t npairs = 0, nclean = 0, eflag = 0, pflag = 0;
    if (!sumT_t || !dS_t || !own_t || !cnt_t || !ownn_t) {
        free(sumT_t); free(dS_t); free(own_t); free(cnt_t); free(ownn_t); free_lists(&L);
        return -1;
    }
#pragma omp parallel reduction(+ : npairs, nclean, eflag, pflag)
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        double *sT = sumT_t + (size_t)tid * n;
        double *dd = dS_t + (size_t)tid * n;
        double *os = own_t + (size_t)tid * n;
        int64_t *cc = cnt_t + (size_t)tid * n;
        int64_t *on = ownn_t + (size_t)tid * n;
#pragma omp for schedule(static)
        for (int64_t pix = 0; pix < npix; ++pix) {
            int64_t s = L.start[pix], e = L.start[pix + 1];
            double T = 1.0;
            double rel = 0.0;        /* relative uncertainty of T from upstream flips */
            int flag_next = 0;       /* reaching the next real entry hinges on a near tie */
            int64_t last = -1;       /* last real entry processed */
            double T_last = 1.0, a_last = 0.0;   /* T received by, and alpha of, that entry */
            int flagged = 0;         /* a near-tie decision touches this pixel */
            int64_t k, np = 0;
            for (k = s; k < e; ++k) {
                const oentry *en = &L.e[k];
                int32_t g = en->g;
                if (en->kind == 1) {            /* ghost: FP32 may count this pixel */
                    double af = opac[g] * exp(-0.5 * cut);
                    os[g] += T;
                    on[g] += 1;
                    rel += af / (1.0 - af);
                    flagged = 1;
                    continue;
                }
                double alpha = opac[g] * exp(-0.5 * en->m);
                if (en->near) {                 /* real, but FP32 may drop this pixel */
                    os[g] += T;
                    on[g] += 1;
                    rel += alpha / (1.0 - alpha);
                    flagged = 1;
                }
                if (flag_next) { os[g] += T; on[g] += 1; flag_next = 0; flagged = 1; }
                if (last >= 0 && depth_tie(en, &L.e[last])) {
                    /* the two may swap: each one's T changes by T_last times the other's alpha */
                    dd[L.e[last].g] += T_last * alpha;
                    dd[g] += T_last * a_last;
                    flagged = 1;
                }
                sT[g] += T;
                cc[g] += 1;
                dd[g] += T * rel;
                np++;
                T_last = T;
                a_last = alpha;
                T *= (1.0 - alpha);
                last = k;
                if (fabs(T - eps_T) < (ORA_TBAND + 2.0 * rel) * eps_T) flag_next = 1;
                if (T < eps_T) break;
            }
            /* after a break, the next real entry is reached in FP32 if the break
             * decision flips, or if it swaps with the last one on a depth tie */
            if (k < e) {
                for (int64_t j = k + 1; j < e; ++j) {
                    if (L.e[j].kind != 0) continue;
                    if (flag_next) { os[L.e[j].g] += T; on[L.e[j].g] += 1; flagged = 1; }
                    if (last >= 0 && depth_tie(&L.e[j], &L.e[last])) {
                        os[L.e[j].g] += T_last;
                        on[L.e[j].g] += 1;
                        dd[L.e[last].g] += T_last;
                        flagged = 1;
                    }
                    break;
                }
            }
            npairs += np;
            if (flagged) { pflag++; eflag += e - s; }
            else nclean += np;
            if (pxpairs) pxpairs[pix] = (int32_t)np;
            if (pxflags) pxflags[pix] = (uint8_t)flagged;
        }
    }
    for (int64_t g = 0; g < n; ++g) {
        double s = 0.0, d = 0.0, ow = 0.0;
        int64_t cnum = 0, onum = 0;
        for (int t = 0; t < nth; ++t) {
            s += sumT_t[(size_t)t * n + g];
            d += dS_t[(size_t)t * n + g];
            ow += own_t[(size_t)t * n + g];
            cnum += cnt_t[(size_t)t * n + g];
            onum += ownn_t[(size_t)t * n + g];
        }
        v[g] = cnum > 0 ? s / (double)cnum : 0.0;
        cnt[g] = cnum;
        double p = 0.0;
        if (onum > 0) p += (ow + (double)onum * v[g]) / (double)(cnum > 1 ? cnum - 1 : 1);
        if (cnum > 0) p += d / (double)cnum;
        pert[g] = p;
    }
    if (counts) {
        ocount c1 = {npairs, L.start[npix], nclean, eflag, pflag, npix};
        count_add(counts, &c1);
    }
    free(sumT_t); free(dS_t); free(own_t); free(cnt_t); free(ownn_t);
    free_lists(&L);
    return 0;
}

/* Alg. 3: visibility-field construction.
 *   gamma[g][k] = sum_p v_p[g] * a_l * Y_k(d_p^g),  d_p^g = (x_g - x_p)/|x_g - x_p|
 * with a_l = 4 pi exp(-kappa) i_l(kappa) and v_p from Alg. 2 (eq. vis_gamma).
 * gamma is written for all n Gaussians ([n][K], K = (L+1)^2); virtual
 * particles (opacity 0) are measured like the others.
 *
 * Optional outputs:
 *   vview  [n_views][n]  per-view v_p[g]
 *   allow  [n][K]        first-order bound on |d gamma_gk| from near-tie decisions:
 *                        sum_p pert_p[g] |a_l Y_k(d_p^g)|
 *   stats  [8]           pairs composited, list entries, Gaussians with a
 *                        nonzero allowance, views processed, pairs composited
 *                        on pixels no near-tie decision touches, list entries
 *                        of the flagged pixels, flagged pixels, pixels
 * gather_mode: 0 = ellipse bounding-box scatter, 1 = brute force. */
int ora_vf_build(int64_t n, const double *means, const double *scales, const double *quats, const double *opac,
                 int32_t n_views, const double *camR, const double *camT, const double *camK, const int32_t *camWH,
                 int32_t L, double kappa, double eps_T, double znear, double lowpass, double cut, int32_t gather_mode,
                 double *gamma, double *vview, double *allow, int64_t *stats)
{
    if (n < 0 || n_views < 0 || L < 0 || L > ORA_LMAX) return -1;
    int K = (L + 1) * (L + 1);
    double al[ORA_LMAX + 1];
    for (int l = 0; l <= L; ++l) al[l] = ora_a_l(l, kappa);
    memset(gamma, 0, sizeof(double) * (size_t)n * K);
    if (allow) memset(allow, 0, sizeof(double) * (size_t)n * K);
    size_t nn = (size_t)(n > 0 ? n : 1);
    oproj *P = (oproj *)malloc(sizeof(oproj) * nn);
    double *v = (double *)malloc(sizeof(double) * nn);
    double *pert = (double *)malloc(sizeof(double) * nn);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * nn);
    uint8_t *touched = (uint8_t *)calloc(nn, 1);
    ocount counts = {0, 0, 0, 0, 0, 0};
    int rc = 0;
    if (!P || !v || !pert || !cnt || !touched) { rc = -1; goto done; }
    for (int32_t p = 0; p < n_views; ++p) {
        ocam c;
        load_cam(&c, &camR[9 * p], &camT[3 * p], &camK[4 * p], &camWH[2 * p]);
#pragma omp parallel for schedule(static)
        for (int64_t g = 0; g < n; ++g)
            project_one(&means[3 * g], &scales[3 * g], &quats[4 * g], &c, lowpass, znear, &P[g]);
        if (single_view_visibility(P, opac, n, &c, eps_T, cut, gather_mode, v, cnt, pert, &counts, NULL, NULL)) {
            rc = -1;
            goto done;
        }
#pragma omp parallel for schedule(static)
        for (int64_t g = 0; g < n; ++g) {
            if (vview) vview[(size_t)p * n + g] = v[g];
            if (pert[g] > 0.0) touched[g] = 1;
            if (v[g] == 0.0 && pert[g] == 0.0) continue;
            double d[3] = {means[3 * g] - c.C[0], means[3 * g + 1] - c.C[1], means[3 * g + 2] - c.C[2]};
            double Y[(ORA_LMAX + 1) * (ORA_LMAX + 1)];
            if (ora_sh_real(L, d, Y)) continue;   /* Gaussian at the camera centre */
            for (int l = 0; l <= L; ++l)
                for (int m = -l; m <= l; ++m) {
                    int k = l * l + l + m;
                    gamma[(size_t)g * K + k] += v[g] * al[l] * Y[k];
                    if (allow) allow[(size_t)g * K + k] += pert[g] * fabs(al[l] * Y[k]);
                }
        }
    }
    if (stats) {
        int64_t nt = 0;
        for (int64_t g = 0; g < n; ++g) nt += touched[g];
        stats[0] = counts.pairs; stats[1] = counts.entries; stats[2] = nt; stats[3] = n_views;
        stats[4] = counts.pairs_clean; stats[5] = counts.entries_flagged;
        stats[6] = counts.px_flagged; stats[7] = counts.px;
    }
done:
    free(P); free(v); free(pert); free(cnt); free(touched);
    return rc;
}

/* Per-view single-view visibility only (Alg. 2), for tests: v_out [n];
 * optional per-pixel outputs (row major): pairs composited and near-tie
 * flags; counts [6] (optional) as the ocount fields. */
int ora_single_view(int64_t n, const double *means, const double *scales, const double *quats, const double *opac,
                    const double *camR, const double *camT, const double *camK, const int32_t *camWH,
                    double eps_T, double znear, double lowpass, double cut, int32_t gather_mode,
                    double *v_out, int64_t *cnt_out, double *pert_out, int32_t *pxpairs, uint8_t *pxflags,
                    int64_t *counts_out)
{
    ocam c;
    load_cam(&c, camR, camT, camK, camWH);
    oproj *P = (oproj *)malloc(sizeof(oproj) * (size_t)(n > 0 ? n : 1));
    double *pert = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int rc = -1;
    if (P && pert && cnt) {
        for (int64_t g = 0; g < n; ++g)
            project_one(&means[3 * g], &scales[3 * g], &quats[4 * g], &c, lowpass, znear, &P[g]);
        ocount counts = {0, 0, 0, 0, 0, 0};
        rc = single_view_visibility(P, opac, n, &c, eps_T, cut, gather_mode, v_out, cnt, pert, &counts, pxpairs,
                                    pxflags);
        if (counts_out) {
            counts_out[0] = counts.pairs; counts_out[1] = counts.entries; counts_out[2] = counts.pairs_clean;
            counts_out[3] = counts.entries_flagged; counts_out[4] = counts.px_flagged; counts_out[5] = counts.px;
        }
        if (cnt_out) memcpy(cnt_out, cnt, sizeof(int64_t) * (size_t)n);
        if (pert_out) memcpy(pert_out, pert, sizeof(double) * (size_t)n);
    }
    free(P); free(pert); free(cnt);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* VF query (Alg. 1 / Alg. 4) and uncertainty rasterisation (Alg. 6)          */
/* ------------------------------------------------------------------------ */

/* Alg. 4 for one Gaussian: V~ = sum_k gamma_k Y_k(d), then the AM-GM lower
 * bound V = 1 - (1 - V~/|P|)^|P| (eq. vis_bound).  V~ is clamped to [0, |P|]
 * first, since the truncated expansion can leave that range; |P| = 0 gives 0. */
double ora_query_visibility(const double *gamma_g, int32_t L, int64_t n_train, const double *dir)
{
    if (n_train <= 0) return 0.0;
    double Y[(ORA_LMAX + 1) * (ORA_LMAX + 1)];
    if (ora_sh_real(L, dir, Y)) return 0.0;
    int K = (L + 1) * (L + 1);
    double Vt = 0.0;
    for (int k = 0; k < K; ++k) Vt += gamma_g[k] * Y[k];
    double P = (double)n_train;
    if (Vt < 0.0) Vt = 0.0;
    if (Vt > P) Vt = P;
    return 1.0 - pow(1.0 - Vt / P, P);
}

/* Multi-view visibility in direction d = x_g - C, exactly (eq. vis_all with
 * eq. vis_p): V = 1 - prod_p (1 - v_p nu(d; d_p)), nu = zeta exp(kappa d.d_p)
 * with zeta = exp(-kappa), unit d and d_p = x_g - C_p.  v_p = Phi T of view p
 * (the single-view visibility of Alg. 2), read as vtrain[p * stride].  A
 * Gaussian at a camera centre has no direction and gets 0 from that view
 * (and V = 0 when it sits at the querying centre). */
double ora_exact_visibility(int64_t n_train, const double *vtrain, int64_t stride, const double *trainC,
                            double kappa, const double *x, const double *C)
{
    double d[3] = {x[0] - C[0], x[1] - C[1], x[2] - C[2]};
    double nd = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!(nd > 0.0)) return 0.0;
    double prod = 1.0;
    for (int64_t p = 0; p < n_train; ++p) {
        double vp = vtrain[p * stride];
        if (vp == 0.0) continue;
        double e[3] = {x[0] - trainC[3 * p], x[1] - trainC[3 * p + 1], x[2] - trainC[3 * p + 2]};
        double ne = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        if (!(ne > 0.0)) continue;
        double cosang = (d[0] * e[0] + d[1] * e[1] + d[2] * e[2]) / (nd * ne);
        prod *= 1.0 - vp * exp(-kappa) * exp(kappa * cosang);
    }
    return 1.0 - prod;
}

/* Emitted-colour covariance of one Gaussian seen in direction d, from the
 * diagonal variances of its colour SH coefficients (Appendix, integration
 * with FisherRF): the colour is linear in the coefficients, so channel k has
 * variance Q_k(d) = sum over l <= Lc, m of Y_lm(d)^2 S_lmk, and with
 * independent channels |Q_c(d)| = prod_k Q_k.  S_lmk is read as
 * var[(k Kc + l^2 + l + m) stride], Kc = (Lc + 1)^2, k = 0..2.  Returns
 * 1/2 log|Q_c(d)|, each Q_k floored at 1e-30 (a zero variance would give
 * -infinity); 0 for a Gaussian without direction (at the camera centre). */
double ora_half_logdet_color(int32_t Lc, const double *var, int64_t stride, const double *d)
{
    double Y[(ORA_LMAX + 1) * (ORA_LMAX + 1)];
    if (Lc < 0 || Lc > ORA_LMAX || ora_sh_real(Lc, d, Y)) return 0.0;
    int Kc = (Lc + 1) * (Lc + 1);
    double h = 0.0;
    for (int k = 0; k < 3; ++k) {
        double Q = 0.0;
        for (int j = 0; j < Kc; ++j) Q += Y[j] * Y[j] * var[(int64_t)(k * Kc + j) * stride];
        h += 0.5 * log(Q > 1e-30 ? Q : 1e-30);
    }
    return h;
}

/* -x log x, with its limit 0 at x = 0 */
static inline double xlogx_neg(double x) { return x > 0.0 ? -x * log(x) : 0.0; }

/* Alg. 4 + Alg. 6 for every candidate view, then the per-view score
 * S_v = sum over pixels of the entropy bound (eq. id with f_corr = 0).
 *   alpha  = o exp(-m/2)
 *   alpha* = (v + beta (1 - v)) alpha + o0 (1 - beta) (1 - v)       (eq. alpha_comp)
 *   w*     = alpha* T;   H += -(w* v) log(w* v) + (w* v) c_c        (eq. huber, i >= 1)
 *   w0    += w* (1 - v); T <- T (1 - alpha*); stop once T < eps_T
 *   H     += -w0 log w0 + w0 c_0                                    (eq. huber, i = 0)
 * with c_c = half_logdet_Qc + 1.5 log(2 pi e), c_0 = half_logdet_Q0 + 1.5 log(2 pi e)
 * (D = 3 colour channels).  The last n_virtual Gaussians have V = 0.
 *
 * With color_var (optional, [3][Kc][n], Kc = (Lc + 1)^2) the constant c_c is
 * replaced per Gaussian and view by 1/2 log|Q_c(d)| + 1.5 log(2 pi e), Q_c(d)
 * from the SH-coefficient variances (ora_half_logdet_color).
 *
 * depth (optional, packed like maps) receives each pixel's expected depth
 * under the same compositing weights, D = sum w* z / sum w* (0 where no
 * Gaussian contributes): the d_p^mn that the spatial-correlation correction
 * of eq. id takes.
 *
 * gamma is [n][K].  maps (optional) is packed view after view, row major;
 * pflags (optional) likewise, 1 where a near-tie decision touches the pixel.
 * vq (optional) [n_views][n] receives the queried visibility.
 * absmaps (optional) receives per pixel the sum of the magnitudes of the
 * terms that make up H (the scale of its rounding error); pxpairs
 * (optional) the pairs composited per pixel.
 * stats [6]: pairs composited, list entries, flagged pixels, total pixels,
 * pairs composited on unflagged pixels, list entries of flagged pixels. */
static int vf_query_core(int64_t n, const double *means, const double *scales, const double *quats,
                         const double *opac, int64_t n_virtual, const double *gamma, int32_t L, int64_t n_train,
                         const double *vtrain, const double *trainC, double kappa,
                         const double *color_var, int32_t Lc, int32_t n_views, const double *camR, const double *camT, const double *camK,
                         const int32_t *camWH, double beta, double o0, double half_logdet_Q0,
                         double half_logdet_Qc, double eps_T, double znear, double lowpass, double cut,
                         int32_t gather_mode, double *maps, double *depth, double *scores, double *vq,
                         uint8_t *pflags, int64_t *stats, double *absmaps, int32_t *pxpairs)
{
    if (n < 0 || n_views < 0 || L < 0 || L > ORA_LMAX || n_virtual < 0 || n_virtual > n) return -1;
    int K = (L + 1) * (L + 1);
    const double c3 = 1.5 * log(2.0 * M_PI * M_E);
    const double cQc = half_logdet_Qc + c3, cQ0 = half_logdet_Q0 + c3;
    if (color_var && (Lc < 0 || Lc > ORA_LMAX)) return -1;
    oproj *P = (oproj *)malloc(sizeof(oproj) * (size_t)(n > 0 ? n : 1));
    double *v = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *cc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!P || !v || !cc) { free(P); free(v); free(cc); return -1; }
    int64_t pairs = 0, entries = 0, nflag = 0, npix_total = 0, pix_off = 0, pclean = 0, eflag = 0;
    int rc = 0;
    for (int32_t p = 0; p < n_views; ++p) {
        ocam c;
        load_cam(&c, &camR[9 * p], &camT[3 * p], &camK[4 * p], &camWH[2 * p]);
#pragma omp parallel for schedule(static)
        for (int64_t g = 0; g < n; ++g) {
            project_one(&means[3 * g], &scales[3 * g], &quats[4 * g], &c, lowpass, znear, &P[g]);
            double d[3] = {means[3 * g] - c.C[0], means[3 * g + 1] - c.C[1], means[3 * g + 2] - c.C[2]};
            if (g >= n - n_virtual) v[g] = 0.0;
            else if (vtrain) v[g] = ora_exact_visibility(n_train, &vtrain[g], n, trainC, kappa, &means[3 * g], c.C);
            else v[g] = ora_query_visibility(&gamma[(size_t)g * K], L, n_train, d);
            if (vq) vq[(size_t)p * n + g] = v[g];
            cc[g] = color_var ? ora_half_logdet_color(Lc, &color_var[g], n, d) + c3 : cQc;
        }
        olists Ls = {0, 0};
        if (gather(P, n, &c, cut, gather_mode, 1, &Ls)) { free_lists(&Ls); rc = -1; break; }
        int64_t npix = (int64_t)c.w * c.h;
        double score = 0.0;
        int64_t vpairs = 0, vflag = 0, vclean = 0, veflag = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : score, vpairs, vflag, vclean, veflag)
        for (int64_t pix = 0; pix < npix; ++pix) {
            int64_t s = Ls.start[pix], e = Ls.start[pix + 1];
            double T = 1.0, w0 = 0.0, H = 0.0, sw = 0.0, swz = 0.0;
            double Habs = 0.0;   /* sum of the magnitudes of the terms of H */
            int flag = 0;
            int64_t last = -1, k, np = 0;
            for (k = s; k < e; ++k) {
                const oentry *en = &Ls.e[k];
                if (en->kind == 1) { flag = 1; continue; }
                if (en->near) flag = 1;
                if (last >= 0 && depth_tie(en, &Ls.e[last])) flag = 1;
                int32_t g = en->g;
                double vg = v[g];
                double alpha = opac[g] * exp(-0.5 * en->m);
                double astar = (vg + beta * (1.0 - vg)) * alpha + o0 * (1.0 - beta) * (1.0 - vg);
                double w = astar * T;
                double x = w * vg;
                H += xlogx_neg(x) + x * cc[g];
                Habs += fabs(xlogx_neg(x)) + fabs(x * cc[g]);
                sw += w;
                swz += w * en->z;
                w0 += w * (1.0 - vg);
                T *= (1.0 - astar);
                np++;
                last = k;
                if (fabs(T - eps_T) < ORA_TBAND * eps_T) flag = 1;
                if (T < eps_T) break;
            }
            if (k < e) {
                for (int64_t j = k + 1; j < e; ++j) {
                    if (Ls.e[j].kind != 0) continue;
                    if (last >= 0 && depth_tie(&Ls.e[j], &Ls.e[last])) flag = 1;
                    break;
                }
            }
            H += xlogx_neg(w0) + w0 * cQ0;
            Habs += fabs(xlogx_neg(w0)) + fabs(w0 * cQ0);
            if (maps) maps[pix_off + pix] = H;
            if (absmaps) absmaps[pix_off + pix] = Habs;
            if (depth) depth[pix_off + pix] = sw > 0.0 ? swz / sw : 0.0;
            if (pflags) pflags[pix_off + pix] = (uint8_t)flag;
            if (pxpairs) pxpairs[pix_off + pix] = (int32_t)np;
            score += H;
            vflag += flag;
            vpairs += np;
            if (flag) veflag += e - s;
            else vclean += np;
        }
        entries += Ls.start[npix];
        free_lists(&Ls);
        scores[p] = score;
        pairs += vpairs;
        nflag += vflag;
        pclean += vclean;
        eflag += veflag;
        npix_total += npix;
        pix_off += npix;
    }
    if (stats) {
        stats[0] = pairs; stats[1] = entries; stats[2] = nflag; stats[3] = npix_total;
        stats[4] = pclean; stats[5] = eflag;
    }
    free(P); free(v); free(cc);
    return rc;
}

int ora_vf_query(int64_t n, const double *means, const double *scales, const double *quats, const double *opac,
                 int64_t n_virtual, const double *gamma, int32_t L, int64_t n_train,
                 int32_t n_views, const double *camR, const double *camT, const double *camK, const int32_t *camWH,
                 double beta, double o0, double half_logdet_Q0, double half_logdet_Qc,
                 double eps_T, double znear, double lowpass, double cut, int32_t gather_mode,
                 double *maps, double *scores, double *vq, uint8_t *pflags, int64_t *stats)
{
    return vf_query_core(n, means, scales, quats, opac, n_virtual, gamma, L, n_train, NULL, NULL, 0.0, NULL, 0,
                         n_views, camR, camT, camK, camWH, beta, o0, half_logdet_Q0, half_logdet_Qc, eps_T, znear,
                         lowpass, cut, gather_mode, maps, NULL, scores, vq, pflags, stats, NULL, NULL);
}

/* ora_vf_query with the per-pixel instrumentation: absmaps (sum of the
 * magnitudes of H's terms) and pxpairs (pairs composited), both optional. */
int ora_vf_query_instr(int64_t n, const double *means, const double *scales, const double *quats, const double *opac,
                       int64_t n_virtual, const double *gamma, int32_t L, int64_t n_train,
                       int32_t n_views, const double *camR, const double *camT, const double *camK,
                       const int32_t *camWH, double beta, double o0, double half_logdet_Q0, double half_logdet_Qc,
                       double eps_T, double znear, double lowpass, double cut, int32_t gather_mode,
                       double *maps, double *scores, double *vq, uint8_t *pflags, int64_t *stats,
                       double *absmaps, int32_t *pxpairs)
{
    return vf_query_core(n, means, scales, quats, opac, n_virtual, gamma, L, n_train, NULL, NULL, 0.0, NULL, 0,
                         n_views, camR, camT, camK, camWH, beta, o0, half_logdet_Q0, half_logdet_Qc, eps_T, znear,
                         lowpass, cut, gather_mode, maps, NULL, scores, vq, pflags, stats, absmaps, pxpairs);
}

/* ora_vf_query that also writes the expected-depth maps (packed like maps). */
int ora_vf_query_depth(int64_t n, const double *means, const double *scales, const double *quats, const double *opac,
                       int64_t n_virtual, const double *gamma, int32_t L, int64_t n_train,
                       int32_t n_views, const double *camR, const double *camT, const double *camK,
                       const int32_t *camWH, double beta, double o0, double half_logdet_Q0, double half_logdet_Qc,
                       double eps_T, double znear, double lowpass, double cut, int32_t gather_mode,
                       double *maps, double *depth, double *scores, uint8_t *pflags, int64_t *stats)
{
    return vf_query_core(n, means, scales, quats, opac, n_virtual, gamma, L, n_train, NULL, NULL, 0.0, NULL, 0,
                         n_views, camR, camT, camK, camWH, beta, o0, half_logdet_Q0, half_logdet_Qc, eps_T, znear,
                         lowpass, cut, gather_mode, maps, depth, scores, NULL, pflags, stats, NULL, NULL);
}

/* The same with the per-Gaussian colour covariance: color_var [3][Kc][n]
 * holds the variances of the colour SH coefficients of degree <= Lc. */
int ora_vf_query_color(int64_t n, const double *means, const double *scales, const double *quats, const double *opac,
                       int64_t n_virtual, const double *gamma, int32_t L, int64_t n_train, const double *color_var,
                       int32_t Lc, int32_t n_views, const double *camR, const double *camT, const double *camK,
                       const int32_t *camWH, double beta, double o0, double half_logdet_Q0, double eps_T,
                       double znear, double lowpass, double cut, int32_t gather_mode, double *maps, double *scores,
                       double *vq, uint8_t *pflags, int64_t *stats)
{
    if (!color_var && n > 0) return -1;
    return vf_query_core(n, means, scales, quats, opac, n_virtual, gamma, L, n_train, NULL, NULL, 0.0, color_var, Lc,
                         n_views, camR, camT, camK, camWH, beta, o0, half_logdet_Q0, 0.0, eps_T, znear,
                         lowpass, cut, gather_mode, maps, NULL, scores, vq, pflags, stats, NULL, NULL);
}

/* The same with the exact multi-view visibility in place of the SH query:
 * vtrain [n_train][n] holds v_p of every Gaussian in every training view,
 * trainC [n_train][3] the training camera centres. */
int ora_vf_query_exact(int64_t n, const double *means, const double *scales, const double *quats,
                       const double *opac, int64_t n_virtual, const double *vtrain, const double *trainC,
                       int64_t n_train, double kappa, int32_t n_views, const double *camR, const double *camT,
                       const double *camK, const int32_t *camWH, double beta, double o0, double half_logdet_Q0,
                       double half_logdet_Qc, double eps_T, double znear, double lowpass, double cut,
                       int32_t gather_mode, double *maps, double *scores, double *vq, uint8_t *pflags,
                       int64_t *stats)
{
    if (n_train < 0 || (n_train > 0 && (!vtrain || !trainC))) return -1;
    return vf_query_core(n, means, scales, quats, opac, n_virtual, NULL, 0, n_train, vtrain, trainC, kappa,
                         NULL, 0, n_views, camR, camT, camK, camWH, beta, o0, half_logdet_Q0, half_logdet_Qc, eps_T,
                         znear, lowpass, cut, gather_mode, maps, NULL, scores, vq, pflags, stats, NULL, NULL);
}

/* Next-best view (eq. i_gain): index of the largest score, lowest index on
 * exact ties; NaN scores never win.  Returns -1 when no score is a number. */
int32_t ora_argmax(const double *scores, int32_t n)
{
    int32_t best = -1;
    for (int32_t i = 0; i < n; ++i) {
        if (scores[i] != scores[i]) continue;
        if (best < 0 || scores[i] > scores[best]) best = i;
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Multi-view visibility for density control (Alg. 5)                        */
/* ------------------------------------------------------------------------ */

/* For every Gaussian: 1 - prod_p (1 - v_p[g]) with v_p from Alg. 2 over all
 * Gaussians of the scene (virtual particles carry opacity 0, so they are
 * measured but never occlude).  allow[g] (optional) bounds the change a
 * near-tie decision can cause: |d(1 - prod)| <= sum_p |d v_p|. */
int ora_multiview_visibility(int64_t n, const double *means, const double *scales, const double *quats,
                             const double *opac, int32_t n_views, const double *camR, const double *camT,
                             const double *camK, const int32_t *camWH, double eps_T, double znear, double lowpass,
                             double cut, int32_t gather_mode, double *vis, double *allow)
{
    size_t nn = (size_t)(n > 0 ? n : 1);
    oproj *P = (oproj *)malloc(sizeof(oproj) * nn);
    double *v = (double *)malloc(sizeof(double) * nn);
    double *pert = (double *)malloc(sizeof(double) * nn);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * nn);
    double *prod = (double *)malloc(sizeof(double) * nn);
    int rc = 0;
    if (!P || !v || !pert || !cnt || !prod) { rc = -1; goto done; }
    for (int64_t g = 0; g < n; ++g) { prod[g] = 1.0; if (allow) allow[g] = 0.0; }
    for (int32_t p = 0; p < n_views; ++p) {
        ocam c;
        load_cam(&c, &camR[9 * p], &camT[3 * p], &camK[4 * p], &camWH[2 * p]);
#pragma omp parallel for schedule(static)
        for (int64_t g = 0; g < n; ++g)
            project_one(&means[3 * g], &scales[3 * g], &quats[4 * g], &c, lowpass, znear, &P[g]);
        if (single_view_visibility(P, opac, n, &c, eps_T, cut, gather_mode, v, cnt, pert, NULL, NULL, NULL)) {
            rc = -1;
            goto done;
        }
        for (int64_t g = 0; g < n; ++g) {
            prod[g] *= (1.0 - v[g]);
            if (allow) allow[g] += pert[g];
        }
    }
    for (int64_t g = 0; g < n; ++g) vis[g] = 1.0 - prod[g];
done:
    free(P); free(v); free(pert); free(cnt); free(prod);
    return rc;
}

/* Virtual particles of the density control (Alg. 5): N_virt = floor(rho *
 * volume of the box [lo, hi]) particles; particle i sits at lo + u_i (hi - lo)
 * (u: the uniform draws, [n_draw][3], n_draw >= N_virt), isotropic scale s
 * with (4/3) pi s^3 rho = 1 + eta (each particle's 1-sigma ball holds 1 + eta
 * of the density's volume per particle), identity rotation and opacity 0.
 * Writes means_out [N_virt][3] if given; returns N_virt, or -1 if n_draw is
 * too small or the box is empty. */
int64_t ora_virtual_particles(const double *lo, const double *hi, double rho, double eta, const double *u,
                              int64_t n_draw, double *means_out, double *s_out)
{
    double vol = 1.0;
    for (int k = 0; k < 3; ++k) vol *= hi[k] - lo[k];
    if (!(vol > 0.0) || !(rho > 0.0)) return -1;
    const int64_t nv = (int64_t)floor(rho * vol);
    if (nv > n_draw) return -1;
    if (s_out) *s_out = cbrt(3.0 * (1.0 + eta) / (4.0 * M_PI * rho));
    if (means_out)
        for (int64_t i = 0; i < nv; ++i)
            for (int k = 0; k < 3; ++k) means_out[3 * i + k] = lo[k] + u[3 * i + k] * (hi[k] - lo[k]);
    return nv;
}

/* ------------------------------------------------------------------------ */
/* A single-precision evaluation of the same loops                          */
/* ------------------------------------------------------------------------ */

/* Parity bookkeeping only.  The near-tie flags and allowances above claim to
 * mark every pixel where a single-precision evaluation of Alg. 2 / Alg. 6 may
 * decide an overlap or a termination differently from this FP64 one.  The
 * functions below are such an evaluation, written independently of any GPU
 * code: the projection is the FP64 one above, rounded to float as a tile
 * rasteriser stores it (the centre as an integer anchor pixel plus a float
 * fraction, the conic as its float lower Cholesky factor, the depth as a
 * float key); per pixel, the centre is taken relative to the origin of the
 * pixel's 16 x 16 tile, m = (l11 ex + l21 ey)^2 + (l22 ey)^2, and every
 * quantity of the compositing recurrence (alpha, T, alpha*, w*, x, H) is a
 * float.  Sums over pixels (per-Gaussian visibility, scores) stay double so
 * that only the per-pixel decisions and arithmetic differ.  The test suite
 * checks that wherever the FP64 oracle raises no flag the two agree. */

typedef struct {
    int ok;
    int32_t ax, ay;        /* anchor pixel: the projected centre rounded to integers */
    float fx, fy;          /* centre minus anchor */
    float l11, l21, l22;   /* lower Cholesky factor of the conic (conic = L L^T) */
    float zk;              /* depth key */
    double ux, uy, sxx, syy;
} oproj32;

static void proj_to_f32(const oproj *o, oproj32 *r)
{
    r->ok = o->ok;
    if (!o->ok) return;
    double ax = rint(o->ux), ay = rint(o->uy);
    r->ax = (int32_t)ax; r->ay = (int32_t)ay;
    r->fx = (float)(o->ux - ax); r->fy = (float)(o->uy - ay);
    double l11 = sqrt(o->ca), l21 = o->cb / l11;
    double l22 = sqrt(fmax(o->cc - l21 * l21, 0.0));
    r->l11 = (float)l11; r->l21 = (float)l21; r->l22 = (float)l22;
    r->zk = (float)o->z;
    r->ux = o->ux; r->uy = o->uy; r->sxx = o->sxx; r->syy = o->syy;
}

static float mahal2_f32(const oproj32 *r, int i, int j)
{
    int ox = i & ~15, oy = j & ~15;
    float cx = (float)(r->ax - ox) + r->fx;
    float cy = (float)(r->ay - oy) + r->fy;
    float ex = cx - ((float)(i - ox) + 0.5f);
    float ey = cy - ((float)(j - oy) + 0.5f);
    float w1 = r->l11 * ex + r->l21 * ey;
    float w2 = r->l22 * ey;
    return w1 * w1 + w2 * w2;
}

typedef struct { float zk; float m; int32_t g; } oentry32;

static int cmp_entry32(const void *pa, const void *pb)
{
    const oentry32 *a = (const oentry32 *)pa, *b = (const oentry32 *)pb;
    if (a->zk < b->zk) return -1;
    if (a->zk > b->zk) return 1;
    return (a->g > b->g) - (a->g < b->g);
}

/* Per-pixel lists under the float predicate m <= cut, in (float depth, index)
 * order.  The search box is the FP64 ellipse's box widened by 1 % and two
 * pixels, far more than float rounding can move the boundary. */
static int gather_f32(const oproj32 *P, int64_t n, const ocam *c, float cut, int64_t **start_out, oentry32 **e_out)
{
    int64_t npix = (int64_t)c->w * c->h;
    int64_t *start = (int64_t *)calloc((size_t)npix + 1, sizeof(int64_t));
    if (!start) return -1;
    oentry32 *E = NULL;
    int64_t *fill = NULL;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            for (int64_t i = 0; i < npix; ++i) start[i + 1] += start[i];
            E = (oentry32 *)malloc(sizeof(oentry32) * (size_t)(start[npix] > 0 ? start[npix] : 1));
            fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(npix > 0 ? npix : 1));
            if (!E || !fill) { free(E); free(fill); free(start); return -1; }
            memcpy(fill, start, sizeof(int64_t) * (size_t)npix);
        }
        for (int64_t g = 0; g < n; ++g) {
            const oproj32 *o = &P[g];
            if (!o->ok) continue;
            double rx = 1.01 * sqrt((double)cut * o->sxx) + 2.0, ry = 1.01 * sqrt((double)cut * o->syy) + 2.0;
            double fi0 = floor(o->ux - rx - 0.5), fi1 = ceil(o->ux + rx - 0.5);
            double fj0 = floor(o->uy - ry - 0.5), fj1 = ceil(o->uy + ry - 0.5);
            if (fi1 < 0 || fj1 < 0 || fi0 > c->w - 1 || fj0 > c->h - 1) continue;
            int i0 = fi0 < 0 ? 0 : (int)fi0, i1 = fi1 > c->w - 1 ? c->w - 1 : (int)fi1;
            int j0 = fj0 < 0 ? 0 : (int)fj0, j1 = fj1 > c->h - 1 ? c->h - 1 : (int)fj1;
            for (int j = j0; j <= j1; ++j)
                for (int i = i0; i <= i1; ++i) {
                    float m = mahal2_f32(o, i, j);
                    if (!(m <= cut)) continue;
                    int64_t pix = (int64_t)j * c->w + i;
                    if (pass == 0) { start[pix + 1]++; continue; }
                    oentry32 *e = &E[fill[pix]++];
                    e->zk = o->zk; e->m = m; e->g = (int32_t)g;
                }
        }
    }
    free(fill);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t pix = 0; pix < npix; ++pix) {
        int64_t s = start[pix], e = start[pix + 1];
        if (e - s > 1) qsort(&E[s], (size_t)(e - s), sizeof(oentry32), cmp_entry32);
    }
    *start_out = start;
    *e_out = E;
    return 0;
}

/* Alg. 2 for one view in single precision: v[g] = (sum of T) / count. */
static int single_view_f32(const oproj32 *P, const double *opac, int64_t n, const ocam *c, float eps_T, float cut,
                           double *v, int32_t *pxpairs, int64_t *pairs_out)
{
    int64_t *start = NULL;
    oentry32 *E = NULL;
    if (gather_f32(P, n, c, cut, &start, &E)) return -1;
    int64_t npix = (int64_t)c->w * c->h;
    int nth = ora_num_threads();
    size_t tot = (size_t)nth * (size_t)n + 1;
    double *sT_t = (double *)calloc(tot, sizeof(double));
    int64_t *cc_t = (int64_t *)calloc(tot, sizeof(int64_t));
    if (!sT_t || !cc_t) { free(sT_t); free(cc_t); free(start); free(E); return -1; }
    int64_t npairs = 0;
#pragma omp parallel reduction(+ : npairs)
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        double *sT = sT_t + (size_t)tid * n;
        int64_t *cc = cc_t + (size_t)tid * n;
#pragma omp for schedule(static)
        for (int64_t pix = 0; pix < npix; ++pix) {
            float T = 1.0f;
            int32_t np = 0;
            for (int64_t k = start[pix]; k < start[pix + 1]; ++k) {
                const oentry32 *en = &E[k];
                float alpha = (float)opac[en->g] * expf(-0.5f * en->m);
                sT[en->g] += (double)T;
                cc[en->g] += 1;
                np++;
                T = T * (1.0f - alpha);
                if (T < eps_T) break;
            }
            npairs += np;
            if (pxpairs) pxpairs[pix] = np;
        }
    }
    for (int64_t g = 0; g < n; ++g) {
        double s = 0.0;
        int64_t k = 0;
        for (int t = 0; t < nth; ++t) { s += sT_t[(size_t)t * n + g]; k += cc_t[(size_t)t * n + g]; }
        v[g] = k > 0 ? (double)(float)(s / (double)k) : 0.0;
    }
    if (pairs_out) *pairs_out += npairs;
    free(sT_t); free(cc_t); free(start); free(E);
    return 0;
}

/* Alg. 3 with the single-precision Alg. 2 above: gamma [n][K]; pxpairs
 * (optional) per view and pixel, packed view after view; pairs (optional)
 * the total. */
int ora_vf_build_f32(int64_t n, const double *means, const double *scales, const double *quats, const double *opac,
                     int32_t n_views, const double *camR, const double *camT, const double *camK, const int32_t *camWH,
                     int32_t L, double kappa, double eps_T, double znear, double lowpass, double cut,
                     double *gamma, int32_t *pxpairs, int64_t *pairs)
{
    if (n < 0 || n_views < 0 || L < 0 || L > ORA_LMAX) return -1;
    int K = (L + 1) * (L + 1);
    double al[ORA_LMAX + 1];
    for (int l = 0; l <= L; ++l) al[l] = ora_a_l(l, kappa);
    memset(gamma, 0, sizeof(double) * (size_t)n * K);
    size_t nn = (size_t)(n > 0 ? n : 1);
    oproj *P = (oproj *)malloc(sizeof(oproj) * nn);
    oproj32 *P32 = (oproj32 *)malloc(sizeof(oproj32) * nn);
    double *v = (double *)malloc(sizeof(double) * nn);
    int64_t npairs = 0, off = 0;
    int rc = 0;
    if (!P || !P32 || !v) { rc = -1; goto done; }
    for (int32_t p = 0; p < n_views; ++p) {
        ocam c;
        load_cam(&c, &camR[9 * p], &camT[3 * p], &camK[4 * p], &camWH[2 * p]);
#pragma omp parallel for schedule(static)
        for (int64_t g = 0; g < n; ++g) {
            project_one(&means[3 * g], &scales[3 * g], &quats[4 * g], &c, lowpass, znear, &P[g]);
            proj_to_f32(&P[g], &P32[g]);
        }
        if (single_view_f32(P32, opac, n, &c, (float)eps_T, (float)cut, v, pxpairs ? pxpairs + off : NULL,
                            &npairs)) { rc = -1; goto done; }
        off += (int64_t)c.w * c.h;
        for (int64_t g = 0; g < n; ++g) {
            if (v[g] == 0.0) continue;
            double d[3] = {means[3 * g] - c.C[0], means[3 * g + 1] - c.C[1], means[3 * g + 2] - c.C[2]};
            double Y[(ORA_LMAX + 1) * (ORA_LMAX + 1)];
            if (ora_sh_real(L, d, Y)) continue;
            for (int l = 0; l <= L; ++l)
                for (int m = -l; m <= l; ++m) gamma[(size_t)g * K + l * l + l + m] += v[g] * al[l] * Y[l * l + l + m];
        }
    }
    if (pairs) *pairs = npairs;
done:
    free(P); free(P32); free(v);
    return rc;
}

/* Alg. 4 + Alg. 6 with every per-pixel quantity in single precision (the
 * per-Gaussian visibility of Alg. 4 is the FP64 one, rounded to float):
 * maps and pxpairs (optional) packed view after view, scores [n_views]. */
int ora_vf_query_f32(int64_t n, const double *means, const double *scales, const double *quats, const double *opac,
                     int64_t n_virtual, const double *gamma, int32_t L, int64_t n_train,
                     int32_t n_views, const double *camR, const double *camT, const double *camK, const int32_t *camWH,
                     double beta, double o0, double half_logdet_Q0, double half_logdet_Qc,
                     double eps_T, double znear, double lowpass, double cut,
                     double *maps, int32_t *pxpairs, double *scores)
{
    if (n < 0 || n_views < 0 || L < 0 || L > ORA_LMAX || n_virtual < 0 || n_virtual > n) return -1;
    int K = (L + 1) * (L + 1);
    const double c3 = 1.5 * log(2.0 * M_PI * M_E);
    const float cQc = (float)(half_logdet_Qc + c3), cQ0 = (float)(half_logdet_Q0 + c3);
    const float fb = (float)beta, fo0 = (float)o0, feps = (float)eps_T, fcut = (float)cut;
    size_t nn = (size_t)(n > 0 ? n : 1);
    oproj *P = (oproj *)malloc(sizeof(oproj) * nn);
    oproj32 *P32 = (oproj32 *)malloc(sizeof(oproj32) * nn);
    float *v = (float *)malloc(sizeof(float) * nn);
    int64_t off = 0;
    int rc = 0;
    if (!P || !P32 || !v) { rc = -1; goto done; }
    for (int32_t p = 0; p < n_views; ++p) {
        ocam c;
        load_cam(&c, &camR[9 * p], &camT[3 * p], &camK[4 * p], &camWH[2 * p]);
#pragma omp parallel for schedule(static)
        for (int64_t g = 0; g < n; ++g) {
            project_one(&means[3 * g], &scales[3 * g], &quats[4 * g], &c, lowpass, znear, &P[g]);
            proj_to_f32(&P[g], &P32[g]);
            double d[3] = {means[3 * g] - c.C[0], means[3 * g + 1] - c.C[1], means[3 * g + 2] - c.C[2]};
            v[g] = g >= n - n_virtual ? 0.0f : (float)ora_query_visibility(&gamma[(size_t)g * K], L, n_train, d);
        }
        int64_t *start = NULL;
        oentry32 *E = NULL;
        if (gather_f32(P32, n, &c, fcut, &start, &E)) { rc = -1; goto done; }
        int64_t npix = (int64_t)c.w * c.h;
        double score = 0.0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : score)
        for (int64_t pix = 0; pix < npix; ++pix) {
            float T = 1.0f, w0 = 0.0f, H = 0.0f;
            int32_t np = 0;
            for (int64_t k = start[pix]; k < start[pix + 1]; ++k) {
                const oentry32 *en = &E[k];
                float vg = v[en->g];
                float alpha = (float)opac[en->g] * expf(-0.5f * en->m);
                float astar = (vg + fb * (1.0f - vg)) * alpha + fo0 * (1.0f - fb) * (1.0f - vg);
                float w = astar * T;
                float x = w * vg;
                if (x > 0.0f) H += -x * logf(x);
                H += x * cQc;
                w0 += w * (1.0f - vg);
                T = T * (1.0f - astar);
                np++;
                if (T < feps) break;
            }
            if (w0 > 0.0f) H += -w0 * logf(w0);
            H += w0 * cQ0;
            if (maps) maps[off + pix] = (double)H;
            if (pxpairs) pxpairs[off + pix] = np;
            score += (double)H;
        }
        free(start); free(E);
        scores[p] = score;
        off += npix;
    }
done:
    free(P); free(P32); free(v);
    return rc;
}
