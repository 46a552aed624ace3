/* Host driver for the sanitizer test of the FP64 oracle: exercises the
 * tracer, projections (single line, sub-rays, PSF, attenuation, 3D), the
 * penalty, the objective and every preconditioner mode of the iteration on
 * small geometries.  Built with AddressSanitizer and UndefinedBehaviorSanitizer
 * by tests/test_oracle_sanitizers.py; any report fails the test. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

static double urand(unsigned* s) {
    *s = *s * 1664525u + 1013904223u;
    return (double)(*s >> 8) / 16777216.0;
}

static int run(orc_geom* g, unsigned seed) {
    const int nv = orc_n_voxels(g);
    const long nb = orc_n_bins(g);
    double* f = malloc(sizeof(double) * nv);
    double* f0 = malloc(sizeof(double) * nv);
    double* y = malloc(sizeof(double) * nb);
    double* r = malloc(sizeof(double) * nb);
    double* q = malloc(sizeof(double) * nb);
    double* b = malloc(sizeof(double) * nv);
    double* obj = malloc(sizeof(double) * 3);
    for (int j = 0; j < nv; ++j) f[j] = 0.5 + urand(&seed);
    orc_forward(g, f, 0, q);
    for (long i = 0; i < nb; ++i) {
        y[i] = floor(q[i] + 1.0 + urand(&seed));
        r[i] = 1.0;
    }
    orc_back(g, y, 1, b);
    orc_sensitivity(g, b);
    double phi = orc_objective(g, f, y, r, 0.3, 2.0, 1e-12);
    int bad = !isfinite(phi);
    for (int mode = 0; mode <= 4; ++mode) {
        orc_params p = {mode, 0.3, 2.0, 1e-12, 1e-4, 1e4, 1.0, 0.1, 3.0, 2.0, 2.0, 0.5, 2.0, 1, 3};
        for (int j = 0; j < nv; ++j) f0[j] = 1.0;
        if (orc_reconstruct(g, &p, f0, y, r, 2, obj) != 0) bad = 1;
        for (int k = 0; k < 3; ++k) bad |= !isfinite(obj[k]);
    }
    free(f); free(f0); free(y); free(r); free(q); free(b); free(obj);
    return bad;
}

int main(void) {
    int bad = 0;
    orc_geom g2 = {2, 12, 9, 1, 2.0, 2.5, 1.0, 10, 17, 1.7, 1, 0, 1.0, 0.0, 3, 1, 0.0, NULL};
    bad |= run(&g2, 1u);
    orc_geom gf = g2;
    gf.n_sub = 8;
    gf.psf_fwhm = 5.0;
    double* att = malloc(sizeof(double) * orc_n_bins(&gf));
    for (long i = 0; i < orc_n_bins(&gf); ++i) att[i] = 0.5 + 0.5 * (double)(i % 7) / 7.0;
    gf.att = att;
    bad |= run(&gf, 2u);
    orc_geom g3 = {3, 6, 5, 4, 2.0, 2.0, 3.0, 6, 9, 2.0, 4, 2, 3.0, 50.0, 2, 1, 0.0, NULL};
    bad |= run(&g3, 3u);
    free(att);
    printf(bad ? "oracle sanitize: FAILED\n" : "oracle sanitize: ok\n");
    return bad;
}
