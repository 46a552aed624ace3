/*
 * oracle.h -- plain FP64 CPU reference of SDP-BSREM (Guo et al., arXiv 2111.07886).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this library; only the tests, the package smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the HIP path.
 *
 * Every routine is written for clarity, not speed: the system matrix A is the
 * classic Siddon ray tracer (sorted plane crossings, midpoint cell lookup),
 * back-projection is the same trace scattered ray by ray, and the iteration is
 * Table I (tab:SDPBSREM) step by step in double precision.  The full 2D model
 * of Sec. IV-A (sub-rays per bin, Gaussian PSF, attenuation factors) is the
 * same tracer applied per sub-ray, a plain separable convolution and a
 * per-bin product (orc_geom fields n_sub, psf_fwhm, att).
 *
 * Geometry conventions (the paper gives only the Matlab set-up of Sec. IV-A):
 *   pixel centres x = (ix - (nx-1)/2) vx, cells half-open [x0, x1);
 *   angles theta_a = a*pi/Na, with (cos,sin) snapped to (1,0) at a = 0 and to
 *   (0,1) at 2a = Na; bins s_b = (b - (Nr-1)/2) ds; ray (a,b) is the line
 *   x cos + y sin = s_b, direction (-sin, cos).
 *   3D: rings at slice centres z_r = (r - (R-1)/2) ring_pitch (R = nz, pitch = vz);
 *   LOR (a,b,r1,r2) runs from z_r1 at transaxial position u = -h to z_r2 at
 *   u = +h, h = sqrt(Rd^2 - s_b^2); span-1 plane order d = 0,+1,-1,...,+D,-D,
 *   ascending r1 within each d.
 *   Subset i (1-based) holds the angles a with a mod M == i-1.
 *   Sinograms are natural layout [plane][angle][bin]; images [z][y][x].
 */
#ifndef PET_ORACLE_H
#define PET_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int dim;                 /* 2 or 3 */
    int nx, ny, nz;          /* nz = 1 in 2D */
    double vx, vy, vz;       /* voxel size [mm] */
    int n_angles, n_radial;
    double ds;               /* radial bin spacing [mm] */
    int n_rings, max_ring_diff;
    double ring_pitch, det_radius;
    int n_subsets;
    /* full 2D system model of Sec. IV-A (all optional; 0 / NULL = off):
     * A = diag(att) P B with P the mean over n_sub parallel sub-rays per bin,
     * spread evenly over the bin width ds (offsets ((k + 1/2)/n_sub - 1/2) ds),
     * and B the image-space Gaussian PSF of FWHM psf_fwhm [mm]. */
    int n_sub;               /* sub-rays per bin (0 or 1: the single line s_b) */
    double psf_fwhm;         /* PSF FWHM [mm], 2D only */
    const double* att;       /* per-bin attenuation factors [n_bins], natural layout */
} orc_geom;

enum { ORC_BSREM = 0, ORC_M1 = 1, ORC_M2 = 2, ORC_P1 = 3, ORC_P2 = 4 };

typedef struct {
    int mode;
    double beta, gamma_R, eps, t_clip, U;
    double lambda0, a, rho, delta1, delta2, nu1, nu2;
    long J0, J1;
} orc_params;

/* iteration state carried between subiterations */
typedef struct {
    long k;              /* outer iteration (0-based) of the next subiteration */
    int i;               /* subset (1-based) of the next subiteration */
    double t_nest;       /* Nesterov t_{k,i} for the next subiteration */
    int have_frozen;     /* nu_frozen holds nu^{k1,i1} */
} orc_state;

int    orc_n_planes(const orc_geom* g);
int    orc_n_voxels(const orc_geom* g);
long   orc_n_bins(const orc_geom* g);
void   orc_plane_rings(const orc_geom* g, int plane, int* r1, int* r2);
void   orc_angle(const orc_geom* g, int a, double* c, double* s);

/* Siddon trace of one LOR; returns the number of (voxel, length) pairs written
 * (at most cap).  Lengths are in mm of the 3D segment inside each voxel. */
int    orc_trace(const orc_geom* g, int plane, int a, int b, int* vox, double* len, int cap);

/* chord length of the LOR inside one voxel by direct slab clipping (no trace) */
double orc_chord_clip(const orc_geom* g, int plane, int a, int b, int ix, int iy, int iz);
/* the same for the line x cos + y sin = s_b + off (a sub-ray; 2D) */
double orc_chord_clip_off(const orc_geom* g, int plane, int a, int b, double off, int ix, int iy, int iz);
/* Siddon trace of the line at offset off from bin b's centre line */
int    orc_trace_off(const orc_geom* g, int plane, int a, int b, double off, int* vox, double* len, int cap);
/* offset of sub-ray k of a bin */
double orc_subray_offset(const orc_geom* g, int k);
/* out = B in: separable Gaussian PSF (sigma = fwhm / (2 sqrt(2 ln 2)), taps at
 * whole-pixel distances up to ceil(3 sigma / v), normalised to sum 1 per axis,
 * zero outside the image: a symmetric operator).  2D. */
void   orc_blur(const orc_geom* g, const double* in, double* out);
int    orc_psf_radius(const orc_geom* g, double v);

/* q = A_i f for the rays of subset `subset` (1..M), or of all rays if subset == 0.
 * q is natural layout; entries of other subsets are left untouched. */
void   orc_forward(const orc_geom* g, const double* f, int subset, double* q);
/* out = A_i^T w using the rays of `subset` (0 = all); w natural layout */
void   orc_back(const orc_geom* g, const double* w, int subset, double* out);

void   orc_sensitivity(const orc_geom* g, double* s);                /* A^T 1 */
void   orc_precond_norm(const orc_geom* g, const double* s, double* p); /* eq:pj */

double orc_rdp_value(const orc_geom* g, const double* f, double gamma_R, double eps);
void   orc_rdp_grad(const orc_geom* g, const double* f, double gamma_R, double eps, double* grad);
void   orc_rdp_hess_apply(const orc_geom* g, const double* f, double gamma_R, double eps,
                          const double* x, double* out);
void   orc_grad_mag(const orc_geom* g, const double* f, double* out);

double orc_fidelity(const orc_geom* g, const double* f, const double* y, const double* r);
double orc_objective(const orc_geom* g, const double* f, const double* y, const double* r,
                     double beta, double gamma_R, double eps);

double orc_relax(const orc_params* p, long k);                       /* lambda_k */
double orc_nesterov_next(double t);                                  /* t -> t_next */
double orc_km_alpha(const orc_params* p, long J);                    /* eq. KM */
double orc_default_U(const orc_geom* g, const double* f0, const double* y, const double* r);

void   orc_state_init(orc_state* st);
/* One subiteration (Table I inner step) in place on f.  nu_frozen: q doubles
 * owned by the caller.  nu_out (optional, q doubles) receives nu^{k,i}.
 * Returns 0, or -1 on invalid arguments. */
int    orc_subiteration(const orc_geom* g, const orc_params* p, orc_state* st,
                        double* f, const double* y, const double* r,
                        const double* pnorm, double* nu_frozen, double* nu_out);
/* n_iter outer iterations from f (in/out).  obj: n_iter+1 doubles or NULL. */
int    orc_reconstruct(const orc_geom* g, const orc_params* p, double* f,
                       const double* y, const double* r, int n_iter, double* obj);

int    orc_num_threads(void);
void   orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
