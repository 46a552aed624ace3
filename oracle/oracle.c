/*
 * oracle.c -- plain FP64 CPU reference of SDP-BSREM (arXiv 2111.07886).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written to be read against the
 * paper: each routine names the equation or section it follows.  No blocking,
 * no fusion; the only parallelism is OpenMP over independent rays.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXAX 3

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of later parallel regions.  For timing: the back-projector
   adds thread-private images, so its last bits depend on the count. */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Geometry (Sec. IV-A set-up; readings listed in the header)          */
/* ------------------------------------------------------------------ */

int orc_n_planes(const orc_geom* g) {
    if (g->dim == 2) return 1;
    int R = g->n_rings, D = g->max_ring_diff, n = R;
    for (int d = 1; d <= D; ++d) n += 2 * (R - d);
    return n;
}

int orc_n_voxels(const orc_geom* g) { return g->nx * g->ny * (g->dim == 3 ? g->nz : 1); }

long orc_n_bins(const orc_geom* g) {
    return (long)orc_n_planes(g) * g->n_angles * g->n_radial;
}

/* span-1 plane order: d = 0, +1, -1, +2, -2, ...; ascending r1 within each d */
void orc_plane_rings(const orc_geom* g, int plane, int* r1, int* r2) {
    if (g->dim == 2) { *r1 = 0; *r2 = 0; return; }
    int R = g->n_rings;
    int left = plane;
    for (int m = 0; m <= 2 * g->max_ring_diff; ++m) {
        int d = (m == 0) ? 0 : ((m % 2) ? (m + 1) / 2 : -(m / 2));
        int lo = d < 0 ? -d : 0;
        int hi = d < 0 ? R - 1 : R - 1 - d;
        int cnt = hi - lo + 1;
        if (left < cnt) { *r1 = lo + left; *r2 = lo + left + d; return; }
        left -= cnt;
    }
    *r1 = -1; *r2 = -1;
}

void orc_angle(const orc_geom* g, int a, double* c, double* s) {
    if (a == 0) { *c = 1.0; *s = 0.0; return; }
    if (2 * a == g->n_angles) { *c = 0.0; *s = 1.0; return; }
    double th = (double)a * M_PI / (double)g->n_angles;
    *c = cos(th);
    *s = sin(th);
}

static double bin_pos(const orc_geom* g, int b) {
    return ((double)b - 0.5 * (double)(g->n_radial - 1)) * g->ds;
}

static long floor_div2(long v) { return (v >= 0) ? v / 2 : -((-v + 1) / 2); }

/* Cell of an axis-aligned ray lying at coordinate s_b on an axis with n cells
 * of size v: half-open cells, a ray on a cell's lower edge belongs to it.
 * When ds == v the position in cells is the exact integer/half-integer
 * (2b - (Nr-1) + n)/2, evaluated in integers. */
static int axis_cell(const orc_geom* g, int b, int n, double v) {
    if (g->ds == v) {
        long twice = 2L * b - (g->n_radial - 1) + n;
        return (int)floor_div2(twice);
    }
    return (int)floor((bin_pos(g, b) + 0.5 * n * v) / v);
}

/* LOR as P(u) = P0 + u D, u = transaxial path length; kappa = |D| */
typedef struct {
    double P0[MAXAX], D[MAXAX], kappa;
    int constcell[MAXAX];   /* cell index if D[k] == 0, else -2 */
} lor_t;

/* LOR of bin b moved by off [mm] along its normal (off = 0: the bin's line;
 * otherwise a sub-ray, 2D).  An axis-parallel sub-ray's cell follows the same
 * half-open rule, from its coordinate in FP64. */
static void make_lor(const orc_geom* g, int plane, int a, int b, double off, lor_t* L) {
    double c, s;
    orc_angle(g, a, &c, &s);
    double sb = bin_pos(g, b) + off;
    L->P0[0] = sb * c;
    L->P0[1] = sb * s;
    L->D[0] = -s;
    L->D[1] = c;
    if (off == 0.0) {
        L->constcell[0] = (s == 0.0) ? axis_cell(g, b, g->nx, g->vx) : -2;
        L->constcell[1] = (c == 0.0) ? axis_cell(g, b, g->ny, g->vy) : -2;
    } else {
        L->constcell[0] = (s == 0.0) ? (int)floor((sb + 0.5 * g->nx * g->vx) / g->vx) : -2;
        L->constcell[1] = (c == 0.0) ? (int)floor((sb + 0.5 * g->ny * g->vy) / g->vy) : -2;
    }
    if (g->dim == 2) {
        L->P0[2] = 0.0; L->D[2] = 0.0; L->constcell[2] = 0; L->kappa = 1.0;
        return;
    }
    int r1, r2;
    orc_plane_rings(g, plane, &r1, &r2);
    double R = g->n_rings;
    double z1 = ((double)r1 - 0.5 * (R - 1.0)) * g->ring_pitch;
    double z2 = ((double)r2 - 0.5 * (R - 1.0)) * g->ring_pitch;
    double h = sqrt(g->det_radius * g->det_radius - sb * sb);
    double mz = (z2 - z1) / (2.0 * h);
    L->P0[2] = z1 + mz * h;           /* z at u = 0 */
    L->D[2] = mz;
    L->constcell[2] = (r1 == r2) ? r1 : -2;   /* direct plane: slice centre */
    L->kappa = sqrt(1.0 + mz * mz);
}

static void axis_dims(const orc_geom* g, int n[MAXAX], double v[MAXAX], double lo[MAXAX]) {
    n[0] = g->nx; n[1] = g->ny; n[2] = (g->dim == 3) ? g->nz : 1;
    v[0] = g->vx; v[1] = g->vy; v[2] = (g->dim == 3) ? g->vz : 1.0;
    for (int k = 0; k < MAXAX; ++k) lo[k] = -0.5 * n[k] * v[k];
}

/* Siddon ray tracing: all plane crossings inside the image, merged in order;
 * each interval between successive crossings lies in one voxel, found from
 * its midpoint. */
int orc_trace(const orc_geom* g, int plane, int a, int b, int* vox, double* len, int cap) {
    return orc_trace_off(g, plane, a, b, 0.0, vox, len, cap);
}

int orc_trace_off(const orc_geom* g, int plane, int a, int b, double off, int* vox, double* len, int cap) {
    lor_t L;
    make_lor(g, plane, a, b, off, &L);
    int n[MAXAX]; double v[MAXAX], lo[MAXAX];
    axis_dims(g, n, v, lo);

    double ulo = -INFINITY, uhi = INFINITY;
    for (int k = 0; k < MAXAX; ++k) {
        if (L.D[k] == 0.0) {
            if (L.constcell[k] < 0 || L.constcell[k] >= n[k]) return 0;
            continue;
        }
        double u0 = (lo[k] - L.P0[k]) / L.D[k];
        double u1 = (lo[k] + n[k] * v[k] - L.P0[k]) / L.D[k];
        if (u0 > u1) { double t = u0; u0 = u1; u1 = t; }
        if (u0 > ulo) ulo = u0;
        if (u1 < uhi) uhi = u1;
    }
    if (!(uhi > ulo)) return 0;

    /* crossing parameters of each axis, ascending */
    int total = 2;
    for (int k = 0; k < MAXAX; ++k) if (L.D[k] != 0.0) total += n[k] + 1;
    double* cross = (double*)malloc(sizeof(double) * (size_t)total);
    double* axlist[MAXAX]; int axcnt[MAXAX];
    int used = 0;
    for (int k = 0; k < MAXAX; ++k) {
        axlist[k] = cross + used; axcnt[k] = 0;
        if (L.D[k] == 0.0) continue;
        for (int m = 0; m <= n[k]; ++m) {
            int mm = (L.D[k] > 0.0) ? m : n[k] - m;
            double u = (lo[k] + mm * v[k] - L.P0[k]) / L.D[k];
            if (u > ulo && u < uhi) axlist[k][axcnt[k]++] = u;
        }
        used += axcnt[k];
    }
    /* merge the three ascending lists between ulo and uhi */
    double* merged = (double*)malloc(sizeof(double) * (size_t)(used + 2));
    int nm = 0, pos[MAXAX] = {0, 0, 0};
    merged[nm++] = ulo;
    for (;;) {
        int best = -1; double bu = INFINITY;
        for (int k = 0; k < MAXAX; ++k)
            if (pos[k] < axcnt[k] && axlist[k][pos[k]] < bu) { bu = axlist[k][pos[k]]; best = k; }
        if (best < 0) break;
        merged[nm++] = bu;
        pos[best]++;
    }
    merged[nm++] = uhi;

    int out = 0;
    for (int m = 0; m + 1 < nm; ++m) {
        double du = merged[m + 1] - merged[m];
        if (!(du > 0.0)) continue;
        double mid = 0.5 * (merged[m] + merged[m + 1]);
        int idx[MAXAX];
        for (int k = 0; k < MAXAX; ++k) {
            if (L.D[k] == 0.0) { idx[k] = L.constcell[k]; continue; }
            double x = L.P0[k] + mid * L.D[k];
            int c = (int)floor((x - lo[k]) / v[k]);
            if (c < 0) c = 0;
            if (c >= n[k]) c = n[k] - 1;
            idx[k] = c;
        }
        if (out < cap) {
            vox[out] = (idx[2] * n[1] + idx[1]) * n[0] + idx[0];
            len[out] = du * L.kappa;
        }
        out++;
    }
    free(cross);
    free(merged);
    return out;
}

/* Chord of the LOR inside voxel (ix,iy,iz) by clipping against the three
 * slabs one at a time; an axis-parallel LOR is inside a slab iff its constant
 * coordinate lies in the half-open interval [lower, upper). */
double orc_chord_clip(const orc_geom* g, int plane, int a, int b, int ix, int iy, int iz) {
    return orc_chord_clip_off(g, plane, a, b, 0.0, ix, iy, iz);
}

double orc_chord_clip_off(const orc_geom* g, int plane, int a, int b, double off, int ix, int iy, int iz) {
    lor_t L;
    make_lor(g, plane, a, b, off, &L);
    int n[MAXAX]; double v[MAXAX], lo[MAXAX];
    axis_dims(g, n, v, lo);
    int id[MAXAX] = {ix, iy, iz};
    double ulo = -INFINITY, uhi = INFINITY;
    for (int k = 0; k < MAXAX; ++k) {
        double b0 = lo[k] + id[k] * v[k], b1 = b0 + v[k];
        if (L.D[k] == 0.0) {
            double x = L.P0[k];
            if (g->dim == 2 && k == 2) continue;
            if (!(x >= b0 && x < b1)) return 0.0;
            continue;
        }
        double u0 = (b0 - L.P0[k]) / L.D[k];
        double u1 = (b1 - L.P0[k]) / L.D[k];
        if (u0 > u1) { double t = u0; u0 = u1; u1 = t; }
        if (u0 > ulo) ulo = u0;
        if (u1 < uhi) uhi = u1;
    }
    return (uhi > ulo) ? (uhi - ulo) * L.kappa : 0.0;
}

/* ------------------------------------------------------------------ */
/* Projections                                                         */
/* ------------------------------------------------------------------ */

static int subset_angles(const orc_geom* g, int subset, int* angles) {
    int n = 0;
    for (int a = 0; a < g->n_angles; ++a)
        if (subset == 0 || a % g->n_subsets == subset - 1) angles[n++] = a;
    return n;
}

static int trace_cap(const orc_geom* g) {
    int nz = (g->dim == 3) ? g->nz : 1;
    return 2 * (g->nx + g->ny + nz) + 8;
}

static long nat_index(const orc_geom* g, int plane, int a, int b) {
    return ((long)plane * g->n_angles + a) * g->n_radial + b;
}

double orc_subray_offset(const orc_geom* g, int k) {
    int ns = g->n_sub > 1 ? g->n_sub : 1;
    return (((double)k + 0.5) / (double)ns - 0.5) * g->ds;
}

/* ------------------------------------------------------------------ */
/* PSF of Sec. IV-A: Gaussian, FWHM given, applied in image space      */
/* ------------------------------------------------------------------ */

int orc_psf_radius(const orc_geom* g, double v) {
    double sigma = g->psf_fwhm / (2.0 * sqrt(2.0 * log(2.0)));
    return (int)ceil(3.0 * sigma / v);
}

static void psf_taps(const orc_geom* g, double v, int K, double* w) {
    double sigma = g->psf_fwhm / (2.0 * sqrt(2.0 * log(2.0)));
    double sum = 0.0;
    for (int k = -K; k <= K; ++k) {
        double x = k * v;
        w[k + K] = exp(-x * x / (2.0 * sigma * sigma));
        sum += w[k + K];
    }
    for (int k = 0; k <= 2 * K; ++k) w[k] /= sum;
}

void orc_blur(const orc_geom* g, const double* in, double* out) {
    int nx = g->nx, ny = g->ny;
    int Kx = orc_psf_radius(g, g->vx), Ky = orc_psf_radius(g, g->vy);
    double* wx = (double*)malloc(sizeof(double) * (size_t)(2 * Kx + 1));
    double* wy = (double*)malloc(sizeof(double) * (size_t)(2 * Ky + 1));
    psf_taps(g, g->vx, Kx, wx);
    psf_taps(g, g->vy, Ky, wy);
    double* tmp = (double*)malloc(sizeof(double) * (size_t)nx * ny);
    for (int iy = 0; iy < ny; ++iy)          /* along x */
        for (int ix = 0; ix < nx; ++ix) {
            double acc = 0.0;
            for (int k = -Kx; k <= Kx; ++k) {
                int x = ix + k;
                if (x >= 0 && x < nx) acc += wx[k + Kx] * in[iy * nx + x];
            }
            tmp[iy * nx + ix] = acc;
        }
    for (int iy = 0; iy < ny; ++iy)          /* along y */
        for (int ix = 0; ix < nx; ++ix) {
            double acc = 0.0;
            for (int k = -Ky; k <= Ky; ++k) {
                int y = iy + k;
                if (y >= 0 && y < ny) acc += wy[k + Ky] * tmp[y * nx + ix];
            }
            out[iy * nx + ix] = acc;
        }
    free(tmp); free(wx); free(wy);
}

/* q = A_i f (sec. II-B), A = diag(att) P B: the image blurred by the PSF (if
 * any), then per ray of the subset the mean over its sub-rays of the Siddon
 * sums, times the ray's attenuation factor (if any) */
void orc_forward(const orc_geom* g, const double* f, int subset, double* q) {
    int* angles = (int*)malloc(sizeof(int) * (size_t)g->n_angles);
    int na = subset_angles(g, subset, angles);
    int ns = g->n_sub > 1 ? g->n_sub : 1;
    double* fb = NULL;
    if (g->psf_fwhm > 0.0) {
        fb = (double*)malloc(sizeof(double) * (size_t)orc_n_voxels(g));
        orc_blur(g, f, fb);
        f = fb;
    }
    int P = orc_n_planes(g), Nr = g->n_radial, cap = trace_cap(g);
    long nrays = (long)P * na * Nr;
#pragma omp parallel
    {
        int* vox = (int*)malloc(sizeof(int) * (size_t)cap);
        double* len = (double*)malloc(sizeof(double) * (size_t)cap);
#pragma omp for schedule(dynamic, 64)
        for (long ray = 0; ray < nrays; ++ray) {
            int b = (int)(ray % Nr);
            int al = (int)((ray / Nr) % na);
            int plane = (int)(ray / ((long)Nr * na));
            double acc = 0.0;
            for (int k = 0; k < ns; ++k) {
                double off = (ns > 1) ? orc_subray_offset(g, k) : 0.0;
                int cnt = orc_trace_off(g, plane, angles[al], b, off, vox, len, cap);
                double part = 0.0;
                for (int m = 0; m < cnt; ++m) part += len[m] * f[vox[m]];
                acc += part;
            }
            acc /= (double)ns;
            long i = nat_index(g, plane, angles[al], b);
            q[i] = g->att ? g->att[i] * acc : acc;
        }
        free(vox); free(len);
    }
    free(angles);
    free(fb);
}

/* out = A_i^T w = B^T P^T (att w): each ray of the subset scatters
 * att_i w_i a_ij into its voxels, every sub-ray with weight 1/n_sub
 * (thread-private images summed afterwards), then the PSF (symmetric) is
 * applied.  w == NULL means w = 1. */
void orc_back(const orc_geom* g, const double* w, int subset, double* out) {
    int* angles = (int*)malloc(sizeof(int) * (size_t)g->n_angles);
    int na = subset_angles(g, subset, angles);
    int ns = g->n_sub > 1 ? g->n_sub : 1;
    int P = orc_n_planes(g), Nr = g->n_radial, cap = trace_cap(g);
    int nv = orc_n_voxels(g);
    long nrays = (long)P * na * Nr;
    int nt = orc_num_threads();
    double* priv = (double*)calloc((size_t)nt * (size_t)nv, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* mine = priv + (size_t)tid * nv;
        int* vox = (int*)malloc(sizeof(int) * (size_t)cap);
        double* len = (double*)malloc(sizeof(double) * (size_t)cap);
#pragma omp for schedule(static)
        for (long ray = 0; ray < nrays; ++ray) {
            int b = (int)(ray % Nr);
            int al = (int)((ray / Nr) % na);
            int plane = (int)(ray / ((long)Nr * na));
            long i = nat_index(g, plane, angles[al], b);
            double wi = w ? w[i] : 1.0;
            if (g->att) wi *= g->att[i];
            if (wi == 0.0) continue;
            for (int k = 0; k < ns; ++k) {
                double off = (ns > 1) ? orc_subray_offset(g, k) : 0.0;
                int cnt = orc_trace_off(g, plane, angles[al], b, off, vox, len, cap);
                for (int m = 0; m < cnt; ++m) mine[vox[m]] += len[m] * wi / (double)ns;
            }
        }
        free(vox); free(len);
    }
    double* acc_img = (g->psf_fwhm > 0.0) ? (double*)malloc(sizeof(double) * (size_t)nv) : out;
    for (int j = 0; j < nv; ++j) {
        double acc = 0.0;
        for (int t = 0; t < nt; ++t) acc += priv[(size_t)t * nv + j];
        acc_img[j] = acc;
    }
    if (g->psf_fwhm > 0.0) {
        orc_blur(g, acc_img, out);
        free(acc_img);
    }
    free(priv);
    free(angles);
}

void orc_sensitivity(const orc_geom* g, double* s) { orc_back(g, NULL, 0, s); }

/* eq:pj -- p_j = (A^T 1)_j / M, or 1/M where the sensitivity is zero */
void orc_precond_norm(const orc_geom* g, const double* s, double* p) {
    int nv = orc_n_voxels(g);
    double M = g->n_subsets;
    for (int j = 0; j < nv; ++j) p[j] = (s[j] > 0.0) ? s[j] / M : 1.0 / M;
}

/* ------------------------------------------------------------------ */
/* Relative difference prior: eq:RDP, eqn:gradRD, eq:SecondDerivative  */
/* Neighbourhood: the 8 (2D) or 26 (3D) in-image neighbours, unit      */
/* weights, every ordered pair (j,k) counted.                          */
/* ------------------------------------------------------------------ */

typedef struct { int n; int dx[26], dy[26], dz[26]; } nbhd_t;

static void make_nbhd(const orc_geom* g, nbhd_t* N) {
    N->n = 0;
    int zr = (g->dim == 3) ? 1 : 0;
    for (int dz = -zr; dz <= zr; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy && !dz) continue;
                N->dx[N->n] = dx; N->dy[N->n] = dy; N->dz[N->n] = dz; N->n++;
            }
}

static int neighbour(const orc_geom* g, const nbhd_t* N, int m, int ix, int iy, int iz) {
    int nz = (g->dim == 3) ? g->nz : 1;
    int x = ix + N->dx[m], y = iy + N->dy[m], z = iz + N->dz[m];
    if (x < 0 || x >= g->nx || y < 0 || y >= g->ny || z < 0 || z >= nz) return -1;
    return (z * g->ny + y) * g->nx + x;
}

double orc_rdp_value(const orc_geom* g, const double* f, double gamma_R, double eps) {
    nbhd_t N; make_nbhd(g, &N);
    int nz = (g->dim == 3) ? g->nz : 1;
    double R = 0.0;
    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < g->ny; ++iy)
            for (int ix = 0; ix < g->nx; ++ix) {
                int j = (iz * g->ny + iy) * g->nx + ix;
                for (int m = 0; m < N.n; ++m) {
                    int k = neighbour(g, &N, m, ix, iy, iz);
                    if (k < 0) continue;
                    double d = f[j] - f[k];
                    R += d * d / (f[j] + f[k] + gamma_R * fabs(d) + eps);
                }
            }
    return R;
}

void orc_rdp_grad(const orc_geom* g, const double* f, double gamma_R, double eps, double* grad) {
    nbhd_t N; make_nbhd(g, &N);
    int nz = (g->dim == 3) ? g->nz : 1;
    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < g->ny; ++iy)
            for (int ix = 0; ix < g->nx; ++ix) {
                int j = (iz * g->ny + iy) * g->nx + ix;
                double acc = 0.0;
                for (int m = 0; m < N.n; ++m) {
                    int k = neighbour(g, &N, m, ix, iy, iz);
                    if (k < 0) continue;
                    double d = f[j] - f[k];
                    double den = f[j] + f[k] + gamma_R * fabs(d) + eps;
                    acc += d * (gamma_R * fabs(d) + f[j] + 3.0 * f[k] + 2.0 * eps) / (den * den);
                }
                grad[j] = 2.0 * acc;
            }
}

/* out = (Hessian of R at f) x, from eq:SecondDerivative */
void orc_rdp_hess_apply(const orc_geom* g, const double* f, double gamma_R, double eps,
                        const double* x, double* out) {
    nbhd_t N; make_nbhd(g, &N);
    int nz = (g->dim == 3) ? g->nz : 1;
    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < g->ny; ++iy)
            for (int ix = 0; ix < g->nx; ++ix) {
                int j = (iz * g->ny + iy) * g->nx + ix;
                double acc = 0.0;
                for (int m = 0; m < N.n; ++m) {
                    int k = neighbour(g, &N, m, ix, iy, iz);
                    if (k < 0) continue;
                    double den = f[j] + f[k] + gamma_R * fabs(f[j] - f[k]) + eps;
                    double den3 = den * den * den;
                    double hjj = 4.0 * (2.0 * f[k] + eps) * (2.0 * f[k] + eps) / den3;
                    double hjk = -4.0 * (4.0 * f[j] * f[k] + 2.0 * eps * (f[j] + f[k]) + eps * eps) / den3;
                    acc += hjj * x[j] + hjk * x[k];
                }
                out[j] = acc;
            }
}

/* Numerical image gradient magnitude (Sec. III-B): Matlab-style gradient
 * with unit spacing -- central differences inside, one-sided at the edges,
 * zero along an axis of length 1 -- then sqrt of the sum of squares. */
static double mgrad(const double* f, long j, long stride, int i, int n) {
    if (n < 2) return 0.0;
    if (i == 0) return f[j + stride] - f[j];
    if (i == n - 1) return f[j] - f[j - stride];
    return 0.5 * (f[j + stride] - f[j - stride]);
}

void orc_grad_mag(const orc_geom* g, const double* f, double* out) {
    int nz = (g->dim == 3) ? g->nz : 1;
    long sx = 1, sy = g->nx, sz = (long)g->nx * g->ny;
    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < g->ny; ++iy)
            for (int ix = 0; ix < g->nx; ++ix) {
                long j = (iz * sz) + iy * sy + ix;
                double gx = mgrad(f, j, sx, ix, g->nx);
                double gy = mgrad(f, j, sy, iy, g->ny);
                double gz = (g->dim == 3) ? mgrad(f, j, sz, iz, nz) : 0.0;
                out[j] = sqrt(gx * gx + gy * gy + gz * gz);
            }
}

/* ------------------------------------------------------------------ */
/* Objective: eq:FidelityTerm, eq:ObjectiveFunction                    */
/* ------------------------------------------------------------------ */

double orc_fidelity(const orc_geom* g, const double* f, const double* y, const double* r) {
    long nb = orc_n_bins(g);
    double* q = (double*)malloc(sizeof(double) * (size_t)nb);
    orc_forward(g, f, 0, q);
    double F = 0.0;
    for (long i = 0; i < nb; ++i) F += q[i] - y[i] * log(q[i] + r[i]);
    free(q);
    return F;
}

double orc_objective(const orc_geom* g, const double* f, const double* y, const double* r,
                     double beta, double gamma_R, double eps) {
    return orc_fidelity(g, f, y, r) + beta * orc_rdp_value(g, f, gamma_R, eps);
}

/* ------------------------------------------------------------------ */
/* Scalar sequences: relaxation (Sec. III, thm:SpecificSDPs),          */
/* preconditioner:Nesterov, preconditioner:KM                          */
/* ------------------------------------------------------------------ */

double orc_relax(const orc_params* p, long k) { return p->lambda0 / (p->a * (double)k + 1.0); }

double orc_nesterov_next(double t) { return 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t)); }

double orc_km_alpha(const orc_params* p, long J) {
    double n = (double)(J - 1);
    return (p->rho * n + p->delta2) / (n + p->delta1);
}

/* Upper bound U of the box B (eq:BoundedSet).  The paper only asserts that it
 * exists; this default is 1e3 times the larger of max f0 and the count
 * consistent mean activity (sum y - sum r)_+ / sum_j (A^T 1)_j. */
double orc_default_U(const orc_geom* g, const double* f0, const double* y, const double* r) {
    int nv = orc_n_voxels(g);
    long nb = orc_n_bins(g);
    double* s = (double*)malloc(sizeof(double) * (size_t)nv);
    orc_sensitivity(g, s);
    double ss = 0.0, sy = 0.0, sr = 0.0, fmax = 0.0;
    for (int j = 0; j < nv; ++j) { ss += s[j]; if (f0[j] > fmax) fmax = f0[j]; }
    for (long i = 0; i < nb; ++i) { sy += y[i]; sr += r[i]; }
    free(s);
    double chat = (sy - sr > 0.0 && ss > 0.0) ? (sy - sr) / ss : 0.0;
    return 1e3 * (fmax > chat ? fmax : chat);
}

void orc_state_init(orc_state* st) {
    st->k = 0; st->i = 1; st->t_nest = 1.0; st->have_frozen = 0;
}

/* ------------------------------------------------------------------ */
/* One SDP-BSREM subiteration, Table I:                                */
/*   f~ = f - lambda_k S^{k,i}(f) grad Phi_i(f),  f <- P_t(f~)         */
/* with S^{k,i} = diag(alpha_{k,i} nu^{k,i}) S(f) (Sec. III-B),         */
/* S from eq:preconditioner, P_t from eq:OperatorPt, nu from eq:nuki.   */
/* nu is computed from the iterate entering the subiteration.          */
/* ------------------------------------------------------------------ */

int orc_subiteration(const orc_geom* g, const orc_params* p, orc_state* st,
                     double* f, const double* y, const double* r,
                     const double* pnorm, double* nu_frozen, double* nu_out) {
    int M = g->n_subsets;
    if (M < 1 || st->i < 1 || st->i > M) return -1;
    int nv = orc_n_voxels(g);
    long J = st->k * (long)M + st->i;
    double lam = orc_relax(p, st->k);

    double alpha = 1.0;
    if (p->mode == ORC_M1 || p->mode == ORC_P1) {
        double t = st->t_nest, tn = orc_nesterov_next(t);
        alpha = 1.0 + (t - 1.0) / tn;
        st->t_nest = tn;
    } else if (p->mode == ORC_M2 || p->mode == ORC_P2) {
        alpha = orc_km_alpha(p, J);
    }

    /* gradient of the subset objective eq:SubObjFunc at f */
    long nb = orc_n_bins(g);
    double* q = (double*)malloc(sizeof(double) * (size_t)nb);
    double* w = (double*)calloc((size_t)nb, sizeof(double));
    orc_forward(g, f, st->i, q);
    int P = orc_n_planes(g);
    for (int plane = 0; plane < P; ++plane)
        for (int a = st->i - 1; a < g->n_angles; a += M)
            for (int b = 0; b < g->n_radial; ++b) {
                long n = nat_index(g, plane, a, b);
                w[n] = 1.0 - y[n] / (q[n] + r[n]);
            }
    double* bp = (double*)malloc(sizeof(double) * (size_t)nv);
    orc_back(g, w, st->i, bp);
    free(q); free(w);
    double* gR = (double*)malloc(sizeof(double) * (size_t)nv);
    orc_rdp_grad(g, f, p->gamma_R, p->eps, gR);

    /* nu^{k,i} (eq:nuki) */
    double* nu = (double*)malloc(sizeof(double) * (size_t)nv);
    int use_nu = (p->mode == ORC_P1 || p->mode == ORC_P2);
    if (!use_nu || J <= p->J0) {
        for (int j = 0; j < nv; ++j) nu[j] = 1.0;
    } else if (J <= p->J1) {
        double sf = 0.0;
        for (int j = 0; j < nv; ++j) sf += f[j];
        double meanf = sf / nv;
        double* mu = (double*)malloc(sizeof(double) * (size_t)nv);
        orc_grad_mag(g, f, mu);
        double smu = 0.0;
        for (int j = 0; j < nv; ++j) {
            double m = mu[j] / meanf;
            mu[j] = (m > 0.01) ? m : 0.01;
            smu += mu[j];
        }
        double meanmu = smu / nv;
        for (int j = 0; j < nv; ++j) {
            double v = meanmu / mu[j];
            if (v < p->nu1) v = p->nu1;
            if (v > p->nu2) v = p->nu2;
            nu[j] = v;
        }
        free(mu);
        if (J == p->J1) {
            memcpy(nu_frozen, nu, sizeof(double) * (size_t)nv);
            st->have_frozen = 1;
        }
    } else {
        for (int j = 0; j < nv; ++j) nu[j] = st->have_frozen ? nu_frozen[j] : 1.0;
    }
    if (nu_out) memcpy(nu_out, nu, sizeof(double) * (size_t)nv);

    double U = p->U, bm = p->beta / (double)M;
    for (int j = 0; j < nv; ++j) {
        double G = bp[j] + bm * gR[j];
        double S = (f[j] < 0.5 * U) ? f[j] / pnorm[j] : (U - f[j]) / pnorm[j];
        double ft = f[j] - lam * alpha * nu[j] * S * G;
        if (ft <= 0.0) f[j] = p->t_clip;
        else if (ft >= U) f[j] = U - p->t_clip;
        else f[j] = ft;
    }
    free(bp); free(gR); free(nu);

    st->i += 1;
    if (st->i > M) { st->i = 1; st->k += 1; }
    return 0;
}

int orc_reconstruct(const orc_geom* g, const orc_params* p, double* f,
                    const double* y, const double* r, int n_iter, double* obj) {
    int nv = orc_n_voxels(g);
    double* s = (double*)malloc(sizeof(double) * (size_t)nv);
    double* pn = (double*)malloc(sizeof(double) * (size_t)nv);
    double* frozen = (double*)calloc((size_t)nv, sizeof(double));
    orc_sensitivity(g, s);
    orc_precond_norm(g, s, pn);
    orc_state st;
    orc_state_init(&st);
    if (obj) obj[0] = orc_objective(g, f, y, r, p->beta, p->gamma_R, p->eps);
    int rc = 0;
    for (int k = 0; k < n_iter && rc == 0; ++k) {
        for (int i = 1; i <= g->n_subsets && rc == 0; ++i)
            rc = orc_subiteration(g, p, &st, f, y, r, pn, frozen, NULL);
        if (obj) obj[k + 1] = orc_objective(g, f, y, r, p->beta, p->gamma_R, p->eps);
    }
    free(s); free(pn); free(frozen);
    return rc;
}
