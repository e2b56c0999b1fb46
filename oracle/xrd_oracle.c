/*
 * Plain FP64 CPU oracle of the kinematical powder-XRD pipeline.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker for the GPU library:
 * only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code, header or table with the library.
 *
 * Every function is the textbook definition written out in double precision,
 * in the order the method states it (paper, Section 2: reciprocal-lattice
 * points inside the limiting sphere, structure factors as a sum over atoms for
 * each reflection, Lorentz-polarisation and Debye-Waller corrections, merging
 * of reflections within an angular tolerance).  The paper names these steps
 * but prints no formula; the formulas below are the standard kinematical ones:
 *
 *   G       metric tensor of (a, b, c, alpha, beta, gamma); G* = G^-1
 *   q       = h^T G* h = 1/d^2
 *   s^2     = q / 4           (s = sin(theta)/lambda)
 *   2theta  = 2 asin(lambda sqrt(q) / 2), degrees
 *   f_t(s)  = sum_{i=1..4} a_i exp(-b_i s^2) + c      (Cromer-Mann form)
 *   F(hkl)  = sum_j occ_j f_{t_j}(s) exp(-B_j s^2) exp(2 pi i (h x_j + k y_j + l z_j))
 *   LP      = (1 + cos^2 2theta) / (sin^2 theta cos theta)
 *   I       = |F|^2 LP
 *
 * Peaks: reflections sorted by (2theta, h, k, l); walking that order, a
 * reflection joins the open peak when its 2theta minus the 2theta of the
 * peak's first member is below the tolerance, otherwise it opens a new peak.
 * The peak sits at its first member's 2theta and carries the sum of member
 * intensities and the member count.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared xrd_oracle.c -lm
 * (no contraction, so every product and sum is rounded as written).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_AMBIG 1e-9 /* degrees: a comparison this close to its threshold is ambiguous */

/* ---- cell ------------------------------------------------------------- */

/* Metric tensor G and its inverse G* of a cell, both stored as
 * [11, 22, 33, 12, 13, 23].  Returns 0, or 1 when the cell is invalid:
 * non-positive lengths, angles outside (0, 180), or det(G)/(abc)^2 < 1e-3. */
int orc_cell(const double lat[6], double g[6], double gs[6], double *volume)
{
    double a = lat[0], b = lat[1], c = lat[2];
    if (!(a > 0.0) || !(b > 0.0) || !(c > 0.0)) return 1;
    for (int i = 3; i < 6; ++i)
        if (!(lat[i] > 0.0) || !(lat[i] < 180.0)) return 1;
    double ca = cos(lat[3] * ORC_PI / 180.0);
    double cb = cos(lat[4] * ORC_PI / 180.0);
    double cg = cos(lat[5] * ORC_PI / 180.0);
    double g11 = a * a, g22 = b * b, g33 = c * c;
    double g12 = a * b * cg, g13 = a * c * cb, g23 = b * c * ca;
    double c11 = g22 * g33 - g23 * g23;
    double c22 = g11 * g33 - g13 * g13;
    double c33 = g11 * g22 - g12 * g12;
    double c12 = g13 * g23 - g12 * g33;
    double c13 = g12 * g23 - g13 * g22;
    double c23 = g12 * g13 - g11 * g23;
    double det = g11 * c11 + g12 * c12 + g13 * c13;
    if (!(det / (g11 * g22 * g33) >= 1e-3)) return 1;
    if (g) { g[0] = g11; g[1] = g22; g[2] = g33; g[3] = g12; g[4] = g13; g[5] = g23; }
    if (gs) {
        gs[0] = c11 / det; gs[1] = c22 / det; gs[2] = c33 / det;
        gs[3] = c12 / det; gs[4] = c13 / det; gs[5] = c23 / det;
    }
    if (volume) *volume = sqrt(det);
    return 0;
}

/* q = h^T G* h, summed in this fixed order. */
double orc_q(const double gs[6], int h, int k, int l)
{
    double hh = (double)h * h, kk = (double)k * k, ll = (double)l * l;
    double hk = (double)h * k, hl = (double)h * l, kl = (double)k * l;
    return gs[0] * hh + gs[1] * kk + gs[2] * ll + 2.0 * (gs[3] * hk + gs[4] * hl + gs[5] * kl);
}

/* 2theta in degrees for q = 1/d^2; returns -1 when sin(theta) > 1. */
double orc_two_theta(double q, double lambda)
{
    double s = 0.5 * lambda * sqrt(q);
    if (s > 1.0) return -1.0;
    return 2.0 * asin(s) * (180.0 / ORC_PI);
}

/* Lorentz-polarisation factor at 2theta (degrees), unpolarised beam. */
double orc_lp(double two_theta)
{
    double th = 0.5 * two_theta * ORC_PI / 180.0;
    double c2 = cos(2.0 * th);
    double st = sin(th), ct = cos(th);
    return (1.0 + c2 * c2) / (st * st * ct);
}

/* orc_lp of each of n angles (a loop, for callers holding arrays). */
void orc_lp_many(long n, const double *two_theta, double *out)
{
    for (long i = 0; i < n; ++i) out[i] = orc_lp(two_theta[i]);
}

/* Cromer-Mann scattering factor at s^2 = (sin(theta)/lambda)^2. */
double orc_fsc(const double coeff[9], double s2)
{
    double f = coeff[8];
    for (int i = 0; i < 4; ++i) f += coeff[i] * exp(-coeff[4 + i] * s2);
    return f;
}

/* ---- enumeration -------------------------------------------------------- */

/* All integer (h, k, l) != 0 with tmin <= 2theta <= tmax, in lexicographic
 * order (h outermost).  The search box is generous on purpose:
 * |h| <= ceil(gmax |a|) + 1 and likewise for k, l, where gmax = 2 sin(theta_max)
 * / lambda, since h = g . a for a reciprocal vector g.  Writes at most
 * ``cap`` reflections and returns the total count (so cap = 0 only counts),
 * or -1 for an invalid cell or range.  ``amb`` (may be NULL) receives the
 * number of reflections whose 2theta lies within 1e-9 deg of a range bound. */
long orc_enumerate(const double lat[6], double lambda, double tmin, double tmax,
                   long cap, int *hkl, double *q, double *tt, long *amb)
{
    double gs[6];
    if (orc_cell(lat, NULL, gs, NULL)) return -1;
    if (!(lambda > 0.0) || !(tmin >= 0.0) || !(tmax > tmin) || !(tmax < 180.0)) return -1;
    double gmax = 2.0 * sin(0.5 * tmax * ORC_PI / 180.0) / lambda;
    int bh = (int)ceil(gmax * lat[0]) + 1;
    int bk = (int)ceil(gmax * lat[1]) + 1;
    int bl = (int)ceil(gmax * lat[2]) + 1;
    long n = 0, namb = 0;
    for (int h = -bh; h <= bh; ++h)
        for (int k = -bk; k <= bk; ++k)
            for (int l = -bl; l <= bl; ++l) {
                if (h == 0 && k == 0 && l == 0) continue;
                double qq = orc_q(gs, h, k, l);
                double t = orc_two_theta(qq, lambda);
                if (t < 0.0) continue;
                if (fabs(t - tmin) < ORC_AMBIG || fabs(t - tmax) < ORC_AMBIG) ++namb;
                if (t < tmin || t > tmax) continue;
                if (n < cap) {
                    hkl[3 * n] = h; hkl[3 * n + 1] = k; hkl[3 * n + 2] = l;
                    q[n] = qq; tt[n] = t;
                }
                ++n;
            }
    if (amb) *amb = namb;
    return n;
}

/* ---- structure factors -------------------------------------------------- */

/* F for each listed reflection: a direct sum over the crystal's atoms in
 * double precision with libm cos/sin/exp, no reduction of the phase.
 * ``absw`` (may be NULL) receives sum_j |w_j|, the size of the largest
 * possible |F|, which bounds the rounding error of the sum. */
void orc_structure_factors(long nr, const int *hkl, const double *q,
                           long na, const double *frac, const int *species,
                           const double *occ, const double *bfac, const double *coeff,
                           double *fr, double *fi, double *absw)
{
    for (long r = 0; r < nr; ++r) {
        double h = hkl[3 * r], k = hkl[3 * r + 1], l = hkl[3 * r + 2];
        double s2 = q[r] / 4.0;
        double re = 0.0, im = 0.0, aw = 0.0;
        for (long j = 0; j < na; ++j) {
            double f = orc_fsc(coeff + 9 * species[j], s2);
            double w = occ[j] * f * exp(-bfac[j] * s2);
            double t = h * frac[3 * j] + k * frac[3 * j + 1] + l * frac[3 * j + 2];
            double phi = 2.0 * ORC_PI * t;
            re += w * cos(phi);
            im += w * sin(phi);
            aw += fabs(w);
        }
        fr[r] = re; fi[r] = im;
        if (absw) absw[r] = aw;
    }
}

/* ---- sort and merge ----------------------------------------------------- */

typedef struct { double tt; int h, k, l; long idx; } orc_key;

static int orc_cmp(const void *pa, const void *pb)
{
    const orc_key *a = (const orc_key *)pa, *b = (const orc_key *)pb;
    if (a->tt < b->tt) return -1;
    if (a->tt > b->tt) return 1;
    if (a->h != b->h) return a->h < b->h ? -1 : 1;
    if (a->k != b->k) return a->k < b->k ? -1 : 1;
    if (a->l != b->l) return a->l < b->l ? -1 : 1;
    return 0;
}

/* perm[i] = index of the i-th reflection in (2theta, h, k, l) order. */
void orc_sort(long nr, const double *tt, const int *hkl, long *perm)
{
    orc_key *keys = (orc_key *)malloc(sizeof(orc_key) * (size_t)(nr > 0 ? nr : 1));
    for (long r = 0; r < nr; ++r) {
        keys[r].tt = tt[r];
        keys[r].h = hkl[3 * r]; keys[r].k = hkl[3 * r + 1]; keys[r].l = hkl[3 * r + 2];
        keys[r].idx = r;
    }
    qsort(keys, (size_t)nr, sizeof(orc_key), orc_cmp);
    for (long r = 0; r < nr; ++r) perm[r] = keys[r].idx;
    free(keys);
}

/* Anchor-rule merge of an ascending 2theta list.  Writes at most nr peaks
 * (position = anchor 2theta, summed intensity in list order, member count,
 * index of the first member) and returns their number.  ``amb`` receives the
 * number of anchor comparisons within 1e-9 deg of the tolerance. */
long orc_merge(long nr, const double *tt_sorted, const double *i_sorted, double tol,
               double *pk_tt, double *pk_i, int *pk_mult, long *pk_first, long *amb)
{
    long np = -1, namb = 0;
    double anchor = 0.0;
    for (long r = 0; r < nr; ++r) {
        int join = 0;
        if (np >= 0) {
            double d = tt_sorted[r] - anchor;
            if (fabs(d - tol) < ORC_AMBIG) ++namb;
            join = d < tol;
        }
        if (!join) {
            ++np;
            anchor = tt_sorted[r];
            pk_tt[np] = anchor; pk_i[np] = 0.0; pk_mult[np] = 0; pk_first[np] = r;
        }
        pk_i[np] += i_sorted[r];
        pk_mult[np] += 1;
    }
    if (amb) *amb = namb;
    return np + 1;
}

/* ---- broadening --------------------------------------------------------- */

/* y_g = sum_r I_r exp(-(x_g - t_r)^2 / (2 sigma^2)) / (sigma sqrt(2 pi)) over
 * the reflections with |x_g - t_r| <= window * sigma, x_g = t0 + g dt.
 * The loop visits, for each reflection, the grid points one step beyond its
 * window on each side and applies the window test to every one of them. */
void orc_broaden(long nr, const double *tt, const double *inten,
                 double t0, double dt, long npts, double sigma, double window, double *y)
{
    double half = window * sigma;
    double norm = 1.0 / (sigma * sqrt(2.0 * ORC_PI));
    for (long g = 0; g < npts; ++g) y[g] = 0.0;
    for (long r = 0; r < nr; ++r) {
        long glo = (long)floor((tt[r] - half - t0) / dt) - 1;
        long ghi = (long)ceil((tt[r] + half - t0) / dt) + 1;
        if (glo < 0) glo = 0;
        if (ghi > npts - 1) ghi = npts - 1;
        for (long g = glo; g <= ghi; ++g) {
            double x = t0 + (double)g * dt;
            double d = x - tt[r];
            if (fabs(d) > half) continue;
            y[g] += inten[r] * norm * exp(-(d * d) / (2.0 * sigma * sigma));
        }
    }
}

/* ---- whole pattern of one crystal, and a batch driver ------------------- */

typedef struct {
    long n_refl, n_peaks, amb_bound, amb_gap;
    int *hkl;                   /* [3 n_refl], enumeration (lexicographic) order */
    double *q, *tt, *lp, *fr, *fi, *absw, *inten; /* [n_refl] */
    long *perm;                 /* [n_refl], (2theta, h, k, l) order */
    double *pk_tt, *pk_i, *pk_y; /* [n_peaks] */
    int *pk_mult;
    long *pk_first;             /* position in perm of the peak's first member */
    int status;                 /* 0 ok, 1 invalid input, 2 out of memory */
} orc_crystal;

void orc_free_crystal(orc_crystal *c)
{
    free(c->hkl); free(c->q); free(c->tt); free(c->lp); free(c->fr); free(c->fi);
    free(c->absw); free(c->inten); free(c->perm);
    free(c->pk_tt); free(c->pk_i); free(c->pk_y); free(c->pk_mult); free(c->pk_first);
    memset(c, 0, sizeof(*c));
}

/* Full pattern of one crystal: enumerate, structure factors, LP, intensity,
 * sort, merge, scale to 0-100 (y = 100 I / max I, 0 when max I = 0), then
 * drop peaks with I < threshold * max I when threshold > 0. */
void orc_pattern(const double lat[6], double lambda, double tmin, double tmax, double tol,
                 double threshold, long na, const double *frac, const int *species,
                 const double *occ, const double *bfac, const double *coeff,
                 orc_crystal *out)
{
    memset(out, 0, sizeof(*out));
    long amb = 0;
    long n = orc_enumerate(lat, lambda, tmin, tmax, 0, NULL, NULL, NULL, NULL);
    if (n < 0 || !(tol > 0.0)) { out->status = 1; return; }
    size_t m = (size_t)(n > 0 ? n : 1);
    out->hkl = (int *)malloc(3 * m * sizeof(int));
    out->q = (double *)malloc(m * sizeof(double));
    out->tt = (double *)malloc(m * sizeof(double));
    out->lp = (double *)malloc(m * sizeof(double));
    out->fr = (double *)malloc(m * sizeof(double));
    out->fi = (double *)malloc(m * sizeof(double));
    out->absw = (double *)malloc(m * sizeof(double));
    out->inten = (double *)malloc(m * sizeof(double));
    out->perm = (long *)malloc(m * sizeof(long));
    out->pk_tt = (double *)malloc(m * sizeof(double));
    out->pk_i = (double *)malloc(m * sizeof(double));
    out->pk_y = (double *)malloc(m * sizeof(double));
    out->pk_mult = (int *)malloc(m * sizeof(int));
    out->pk_first = (long *)malloc(m * sizeof(long));
    double *ts = (double *)malloc(m * sizeof(double));
    double *is = (double *)malloc(m * sizeof(double));
    if (!out->hkl || !out->q || !out->tt || !out->lp || !out->fr || !out->fi || !out->absw ||
        !out->inten || !out->perm || !out->pk_tt || !out->pk_i || !out->pk_y ||
        !out->pk_mult || !out->pk_first || !ts || !is) {
        free(ts); free(is); orc_free_crystal(out); out->status = 2; return;
    }
    out->n_refl = orc_enumerate(lat, lambda, tmin, tmax, n, out->hkl, out->q, out->tt, &amb);
    out->amb_bound = amb;
    orc_structure_factors(n, out->hkl, out->q, na, frac, species, occ, bfac, coeff,
                          out->fr, out->fi, out->absw);
    for (long r = 0; r < n; ++r) {
        out->lp[r] = orc_lp(out->tt[r]);
        out->inten[r] = (out->fr[r] * out->fr[r] + out->fi[r] * out->fi[r]) * out->lp[r];
    }
    orc_sort(n, out->tt, out->hkl, out->perm);
    for (long r = 0; r < n; ++r) { ts[r] = out->tt[out->perm[r]]; is[r] = out->inten[out->perm[r]]; }
    long np = orc_merge(n, ts, is, tol, out->pk_tt, out->pk_i, out->pk_mult, out->pk_first, &amb);
    out->amb_gap = amb;
    free(ts); free(is);
    double mx = 0.0;
    for (long p = 0; p < np; ++p) if (out->pk_i[p] > mx) mx = out->pk_i[p];
    long kept = 0;
    for (long p = 0; p < np; ++p) {
        if (threshold > 0.0 && out->pk_i[p] < threshold * mx) continue;
        out->pk_tt[kept] = out->pk_tt[p];
        out->pk_i[kept] = out->pk_i[p];
        out->pk_mult[kept] = out->pk_mult[p];
        out->pk_first[kept] = out->pk_first[p];
        out->pk_y[kept] = mx > 0.0 ? 100.0 * out->pk_i[p] / mx : 0.0;
        ++kept;
    }
    out->n_peaks = kept;
}

/* Patterns of a CSR batch, crystals spread over ``nthreads`` OpenMP threads
 * (values below 1 mean one thread).  ``out`` has one entry per crystal; free each with
 * orc_free_crystal. */
void orc_pattern_batch(long nc, const double *lattice, const long *atom_offset,
                       const double *frac, const int *species, const double *occ,
                       const double *bfac, const double *coeff, double lambda,
                       const double *tmin, const double *tmax, double tol, double threshold,
                       int nthreads, orc_crystal *out)
{
    int nt = nthreads > 0 ? nthreads : 1;
    (void)nt;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (long c = 0; c < nc; ++c) {
        long a0 = atom_offset[c], a1 = atom_offset[c + 1];
        orc_pattern(lattice + 6 * c, lambda, tmin[c], tmax[c], tol, threshold, a1 - a0,
                    frac + 3 * a0, species + a0, occ + a0, bfac + a0, coeff, out + c);
    }
}

/* ---- augmentation of ML training patterns ------------------------------ */
/*
 * The paper's motivation (Section 1) is training data for ML models, built
 * from simulated patterns modified with experimental effects such as
 * preferred orientation and noise.  These are the plain definitions of two
 * such effects.
 */

/* u^T G* v with G* given as [11, 22, 33, 12, 13, 23]. */
static double orc_dot_gs(const double gs[6], const double u[3], const double v[3])
{
    return gs[0] * u[0] * v[0] + gs[1] * u[1] * v[1] + gs[2] * u[2] * v[2]
         + gs[3] * (u[0] * v[1] + u[1] * v[0]) + gs[4] * (u[0] * v[2] + u[2] * v[0])
         + gs[5] * (u[1] * v[2] + u[2] * v[1]);
}

/* March-Dollase preferred-orientation factor (Dollase, J. Appl. Cryst. 19
 * (1986) 267) of reflection h for the preferred direction hp (a reciprocal-
 * lattice vector in hkl components) and March parameter r:
 *   cos(alpha) = h^T G* hp / (|h| |hp|),  |v| = sqrt(v^T G* v),
 *   P = (r^2 cos^2(alpha) + sin^2(alpha) / r)^(-3/2).
 * r = 1 is a random powder (P = 1). */
double orc_march_dollase(const double gs[6], int h, int k, int l, const double hp[3], double r)
{
    const double hv[3] = {(double)h, (double)k, (double)l};
    const double c = orc_dot_gs(gs, hv, hp) / (sqrt(orc_dot_gs(gs, hv, hv)) * sqrt(orc_dot_gs(gs, hp, hp)));
    const double c2 = c * c;
    return pow(r * r * c2 + (1.0 - c2) / r, -1.5);
}

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the j-th output (j >= 1)
 * of the generator seeded with ``seed`` is mix(seed + j * 0x9e3779b97f4a7c15)
 * (arithmetic mod 2^64), mix being the generator's finaliser. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t j)
{
    uint64_t z = seed + j * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Standard normal variate number ``n`` of stream ``seed``: outputs 2n+1 and
 * 2n+2 of SplitMix64 give uniforms u = (top 53 bits + 1/2) 2^-53 in (0, 1),
 * and the Box-Muller transform sqrt(-2 ln u1) cos(2 pi u2). */
double orc_gauss(uint64_t seed, uint64_t n)
{
    const double u1 = ((double)(orc_splitmix64(seed, 2 * n + 1) >> 11) + 0.5) * 0x1p-53;
    const double u2 = ((double)(orc_splitmix64(seed, 2 * n + 2) >> 11) + 0.5) * 0x1p-53;
    return sqrt(-2.0 * log(u1)) * cos(2.0 * ORC_PI * u2);
}

/* Noise on broadened patterns y [n_c][n_pts], in place:
 *   y += (rel sqrt(max(y, 0)) + abs) z,  z = orc_gauss(seed, c n_pts + g)
 * (a counting-statistics term and a flat background term). */
void orc_noise(long n_c, long n_pts, uint64_t seed, double rel, double abs_, double *y)
{
    for (long c = 0; c < n_c; ++c)
        for (long g = 0; g < n_pts; ++g) {
            const long i = c * n_pts + g;
            const double v = y[i];
            y[i] = v + (rel * sqrt(v > 0.0 ? v : 0.0) + abs_) * orc_gauss(seed, (uint64_t)i);
        }
}

/* Broadening with 2theta-dependent widths (Caglioti, Paoletti and Ricci,
 * Nucl. Instrum. 3 (1958) 223) and pseudo-Voigt profiles: each reflection is
 *   eta L(d) + (1 - eta) G(d),  d = x - 2theta,
 * a unit-area Lorentzian L(d) = (2 / (pi Gam)) / (1 + (2 d / Gam)^2) and a
 * unit-area Gaussian G of the same full width at half maximum Gam,
 *   Gam^2 = U tan^2(theta) + V tan(theta) + W   (degrees^2, theta = 2theta / 2),
 *   sigma = Gam / (2 sqrt(2 ln 2)),
 * summed over the grid points with |d| <= window sigma (both components cut
 * there).  A reflection with Gam^2 <= 0 adds nothing.  eta = 0 is the
 * Gaussian broadening (with U = V = 0, orc_broaden with sigma =
 * sqrt(W) / (2 sqrt(2 ln 2))). */
void orc_broaden_caglioti(long nr, const double *tt, const double *inten, double t0, double dt, long npts,
                          double U, double V, double W, double eta, double window, double *y)
{
    for (long g = 0; g < npts; ++g) y[g] = 0.0;
    for (long r = 0; r < nr; ++r) {
        const double t = tan(0.5 * tt[r] * ORC_PI / 180.0);
        const double f2 = U * t * t + V * t + W;
        if (!(f2 > 0.0)) continue;
        const double gam = sqrt(f2);
        const double sigma = gam / (2.0 * sqrt(2.0 * log(2.0)));
        const double half = window * sigma;
        const double norm = 1.0 / (sigma * sqrt(2.0 * ORC_PI));
        long glo = (long)floor((tt[r] - half - t0) / dt) - 1;
        long ghi = (long)ceil((tt[r] + half - t0) / dt) + 1;
        if (glo < 0) glo = 0;
        if (ghi > npts - 1) ghi = npts - 1;
        for (long g = glo; g <= ghi; ++g) {
            const double x = t0 + (double)g * dt;
            const double d = x - tt[r];
            if (fabs(d) > half) continue;
            const double gauss = norm * exp(-(d * d) / (2.0 * sigma * sigma));
            const double u = 2.0 * d / gam;
            const double lorentz = 2.0 / (ORC_PI * gam) / (1.0 + u * u);
            y[g] += inten[r] * (eta * lorentz + (1.0 - eta) * gauss);
        }
    }
}

/* ---- families of symmetry-equivalent reflections ------------------------ */
/*
 * The paper lists, among the steps moved to compiled code (Section 2), the
 * grouping of symmetry-equivalent reflections, and its example output
 * (Section 3) gives each merged peak a list of families, each with a
 * multiplicity.  The input here carries no space group, so two equivalences
 * are defined (a reading: the paper states neither):
 *
 *   ORC_FAM_INDICES  equal multisets of absolute index values, taken in the
 *                    3-index form (h, k, l), or in the 4-index form
 *                    (h, k, -(h + k), l) on a hexagonal lattice; the usual
 *                    labelling convention of the Python calculator the paper
 *                    targets;
 *   ORC_FAM_LATTICE  related by a point operation of the lattice: an integer
 *                    matrix M with entries in {-1, 0, 1}, det M = +-1 and
 *                    M^T G* M = G*, acting as hkl -> M hkl (so q is kept).
 *
 * Metric equalities hold within ORC_FAM_TOL times the largest diagonal entry
 * of G*.  A lattice is hexagonal when G*11 = G*22, G*13 = G*23 = 0 and
 * G*12 = G*11 / 2 (a = b, alpha = beta = 90, gamma = 120 degrees).
 *
 * Within a peak, members are taken in the peak's member order; a member
 * joins the family of the earliest earlier member equivalent to it, or opens
 * a new family.  A family's label is its lexicographically largest (h, k, l)
 * member and its multiplicity the number of its members.
 */
#define ORC_FAM_INDICES 0
#define ORC_FAM_LATTICE 1
#define ORC_FAM_TOL 1e-6

static int orc_fam_close(double x, double y, double scale)
{
    return fabs(x - y) <= ORC_FAM_TOL * scale;
}

static double orc_fam_scale(const double gs[6])
{
    double s = gs[0];
    if (gs[1] > s) s = gs[1];
    if (gs[2] > s) s = gs[2];
    return s;
}

int orc_is_hexagonal(const double lat[6])
{
    double gs[6];
    if (orc_cell(lat, NULL, gs, NULL)) return 0;
    const double s = orc_fam_scale(gs);
    return orc_fam_close(gs[0], gs[1], s) && orc_fam_close(gs[4], 0.0, s) && orc_fam_close(gs[5], 0.0, s)
        && orc_fam_close(gs[3], 0.5 * gs[0], s);
}

/* Every point operation of the lattice, found by trying all 3^9 matrices with
 * entries in {-1, 0, 1}; ops[n][9] row-major.  Returns their number (at most
 * 48 for a lattice), or -1 if the cell is invalid or more than max_ops match. */
long orc_lattice_ops(const double lat[6], long max_ops, int *ops)
{
    double gs[6];
    if (orc_cell(lat, NULL, gs, NULL)) return -1;
    const double G[3][3] = {{gs[0], gs[3], gs[4]}, {gs[3], gs[1], gs[5]}, {gs[4], gs[5], gs[2]}};
    const double s = orc_fam_scale(gs);
    long n = 0;
    for (long code = 0; code < 19683; ++code) {
        int M[3][3];
        long c = code;
        for (int e = 0; e < 9; ++e) { M[e / 3][e % 3] = (int)(c % 3) - 1; c /= 3; }
        const long det = (long)M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
                       - (long)M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
                       + (long)M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
        if (det != 1 && det != -1) continue;
        int keep = 1;
        for (int i = 0; i < 3 && keep; ++i)
            for (int j = 0; j < 3 && keep; ++j) {
                double v = 0.0; /* (M^T G* M)_ij */
                for (int p = 0; p < 3; ++p)
                    for (int r = 0; r < 3; ++r) v += M[p][i] * G[p][r] * M[r][j];
                keep = orc_fam_close(v, G[i][j], s);
            }
        if (!keep) continue;
        if (n == max_ops) return -1;
        for (int e = 0; e < 9; ++e) ops[n * 9 + e] = M[e / 3][e % 3];
        ++n;
    }
    return n;
}

static int orc_fam_cmp_int(const void *a, const void *b)
{
    const int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* Whether reflections u and v are equivalent under the rule. */
static int orc_fam_equiv(int rule, int hex, long n_ops, const int *ops, const int *u, const int *v)
{
    if (rule == ORC_FAM_INDICES) {
        int a[4] = {abs(u[0]), abs(u[1]), abs(u[2]), abs(u[0] + u[1])};
        int b[4] = {abs(v[0]), abs(v[1]), abs(v[2]), abs(v[0] + v[1])};
        const int n = hex ? 4 : 3;
        qsort(a, n, sizeof(int), orc_fam_cmp_int);
        qsort(b, n, sizeof(int), orc_fam_cmp_int);
        for (int i = 0; i < n; ++i)
            if (a[i] != b[i]) return 0;
        return 1;
    }
    for (long o = 0; o < n_ops; ++o) {
        const int *M = ops + o * 9;
        int same = 1;
        for (int r = 0; r < 3 && same; ++r) same = M[r * 3] * u[0] + M[r * 3 + 1] * u[1] + M[r * 3 + 2] * u[2] == v[r];
        if (same) return 1;
    }
    return 0;
}

static int orc_hkl_greater(const int *u, const int *v)
{
    if (u[0] != v[0]) return u[0] > v[0];
    if (u[1] != v[1]) return u[1] > v[1];
    return u[2] > v[2];
}

/* Families of the peaks of one crystal with lattice ``lat``.  hkl[n][3] lists
 * the crystal's reflections in peak member order; peak p's members are
 * positions first[p] .. first[p] + mult[p] - 1.  Writes, for every member
 * position i, fam[i] = its family's number within its peak; for peak p,
 * n_fam[p] families whose labels and multiplicities sit at positions
 * first[p] + f of label[.][3] and fam_mult.  Returns 0, or 1 for an invalid
 * cell, rule, or more than 48 lattice operations. */
int orc_peak_families(const double lat[6], int rule, long n_peaks, const long *first, const long *mult,
                      const int *hkl, long *fam, long *n_fam, int *label, long *fam_mult)
{
    int ops[48 * 9];
    long n_ops = 0;
    int hex = 0;
    if (rule == ORC_FAM_LATTICE) {
        n_ops = orc_lattice_ops(lat, 48, ops);
        if (n_ops < 0) return 1;
    } else if (rule == ORC_FAM_INDICES) {
        double gs[6];
        if (orc_cell(lat, NULL, gs, NULL)) return 1;
        hex = orc_is_hexagonal(lat);
    } else {
        return 1;
    }
    for (long p = 0; p < n_peaks; ++p) {
        const long b = first[p], m = mult[p];
        long nf = 0;
        for (long i = 0; i < m; ++i) {
            const int *u = hkl + 3 * (b + i);
            long f = -1;
            for (long j = 0; j < i && f < 0; ++j)
                if (orc_fam_equiv(rule, hex, n_ops, ops, hkl + 3 * (b + j), u)) f = fam[b + j];
            if (f < 0) {
                f = nf++;
                fam_mult[b + f] = 0;
                memcpy(label + 3 * (b + f), u, 3 * sizeof(int));
            }
            fam[b + i] = f;
            fam_mult[b + f] += 1;
            if (orc_hkl_greater(u, label + 3 * (b + f))) memcpy(label + 3 * (b + f), u, 3 * sizeof(int));
        }
        n_fam[p] = nf;
    }
    return 0;
}
