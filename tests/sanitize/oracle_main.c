/* The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (the oracle is one translation unit, included here): whole patterns of
 * the rock-salt cell and of random triclinic cells, a batch, broadening,
 * noise, Caglioti profiles, lattice operations and families, with the
 * rock-salt counts checked. */
#include "../../oracle/xrd_oracle.c"

#include <stdio.h>

static int fails = 0;
static void expect(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAIL: %s\n", what);
        ++fails;
    }
}

static unsigned long long rng_state = 88172645463325252ull;
static double uni(double lo, double hi)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return lo + (hi - lo) * (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

int main(void)
{
    double coeff[2 * 9];
    for (int i = 0; i < 18; ++i) coeff[i] = (i % 9) < 4 ? uni(0.5, 6.0) : (i % 9) < 8 ? uni(0.5, 60.0) : uni(0, 1);
    /* rock salt: 586 reflections in 23 peaks (Section 3's worked cell shape) */
    double lat[6] = {5.64, 5.64, 5.64, 90, 90, 90};
    double frac[8 * 3] = {0, 0, 0, 0, .5, .5, .5, 0, .5, .5, .5, 0, .5, 0, 0, .5, .5, .5, 0, 0, .5, 0, .5, 0};
    int species[8] = {0, 0, 0, 0, 1, 1, 1, 1};
    double occ[8], bfac[8];
    for (int j = 0; j < 8; ++j) occ[j] = 1.0, bfac[j] = 0.5;
    orc_crystal c;
    orc_pattern(lat, 1.54184, 0.0, 90.0, 1e-5, 0.0, 8, frac, species, occ, bfac, coeff, &c);
    expect(c.status == 0 && c.n_refl == 586 && c.n_peaks == 23, "rock-salt counts");
    double *y = calloc(4001, sizeof(double));
    orc_broaden(c.n_refl, c.tt, c.inten, 10.0, 0.02, 4001, 0.1, 8.0, y);
    orc_broaden_caglioti(c.n_refl, c.tt, c.inten, 10.0, 0.02, 4001, 0.02, -0.005, 0.004, 0.3, 12.0, y);
    orc_noise(1, 4001, 7, 0.05, 0.01, y);
    long first[64], mult[64], n_fam[64];
    long *fam = malloc(sizeof(long) * c.n_refl), *fam_mult = malloc(sizeof(long) * c.n_refl);
    int *label = malloc(sizeof(int) * 3 * c.n_refl);
    long np = c.n_peaks < 64 ? c.n_peaks : 64;
    for (long p = 0; p < np; ++p) first[p] = c.pk_first[p], mult[p] = c.pk_mult[p];
    int *hkl_sorted = malloc(sizeof(int) * 3 * c.n_refl);
    for (long r = 0; r < c.n_refl; ++r)
        for (int d = 0; d < 3; ++d) hkl_sorted[3 * r + d] = c.hkl[3 * c.perm[r] + d];
    for (int rule = 0; rule < 2; ++rule)
        expect(orc_peak_families(lat, rule, np, first, mult, hkl_sorted, fam, n_fam, label, fam_mult) == 0,
               "families");
    expect(n_fam[0] == 1 && fam_mult[first[0]] == 6, "first peak: the six (100) reflections");
    int ops[48 * 9];
    expect(orc_lattice_ops(lat, 48, ops) == 48, "cubic point group");
    free(hkl_sorted);
    free(fam), free(fam_mult), free(label);
    free(y);
    orc_free_crystal(&c);
    /* random triclinic cells, one by one and as a batch */
    enum { NC = 12 };
    double lats[NC * 6], tmin[NC], tmax[NC];
    long off[NC + 1];
    off[0] = 0;
    for (int k = 0; k < NC; ++k) {
        for (int i = 0; i < 3; ++i) lats[6 * k + i] = uni(3.0, 12.0);
        for (int i = 3; i < 6; ++i) lats[6 * k + i] = uni(80.0, 100.0);
        off[k + 1] = off[k] + 1 + (long)uni(0, 40);
        tmin[k] = 10.0;
        tmax[k] = 90.0;
    }
    long na = off[NC];
    double *f = malloc(sizeof(double) * 3 * na), *o = malloc(sizeof(double) * na), *bf = malloc(sizeof(double) * na);
    int *sp = malloc(sizeof(int) * na);
    for (long j = 0; j < na; ++j) {
        for (int d = 0; d < 3; ++d) f[3 * j + d] = uni(0, 1);
        o[j] = uni(0.5, 1.0);
        bf[j] = uni(0, 2);
        sp[j] = (int)uni(0, 2) % 2;
    }
    orc_crystal out[NC];
    orc_pattern_batch(NC, lats, off, f, sp, o, bf, coeff, 1.54184, tmin, tmax, 1e-5, 1e-3, 1, out);
    for (int k = 0; k < NC; ++k) {
        expect(out[k].status == 0, "batch crystal");
        orc_crystal one;
        orc_pattern(lats + 6 * k, 1.54184, tmin[k], tmax[k], 1e-5, 1e-3, off[k + 1] - off[k], f + 3 * off[k],
                    sp + off[k], o + off[k], bf + off[k], coeff, &one);
        expect(one.n_refl == out[k].n_refl && one.n_peaks == out[k].n_peaks, "batch equals single");
        orc_free_crystal(&one);
        orc_free_crystal(&out[k]);
    }
    free(f), free(o), free(bf), free(sp);
    printf("oracle checks done, %d failures\n", fails);
    return fails == 0 ? 0 : 1;
}
