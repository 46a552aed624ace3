// raygeom.h -- per-ray geometry of the forward (ray-driven) and back
// (voxel-driven) projectors.
//
// System model (Sec. IV-A): a_ij = length of LOR i inside voxel j.  A ray is
// walked along its "major" transaxial axis (rows when |cos| vx >= |sin| vy,
// else columns).  Over one major cell m the ray's coordinate on the other
// transaxial axis moves linearly, in grid units, from g(m) = P + Q m to
// g(m) + Q (|Q| <= 1), and its axial grid coordinate from z(m) = Pz + Qz m to
// z(m) + Qz.  With psi in [0,1] the position along that piece, the voxel
// (minor cell c, slice k) receives L * |psi-interval(c) /\ psi-interval(k)|,
// where L is the 3D length of the piece.  Axis-parallel rays (Q == 0) lie in
// cell floor(P): a ray on a cell's lower edge belongs to that cell.
//
// All positions are FP64, so that cell decisions agree with an FP64 reference
// up to rounding.  The 2D back-projector evaluates the same chord length in
// closed form for oblique rays (AngleK::e_out, inv_de, Lmax); the 3D one
// splits the transaxial piece among slices by the same axial coordinate.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace petos {

// Per-angle constants, computed on the host in FP64.
struct AngleK {
    double c, s;        // cos, sin of theta_a (snapped at 0 and pi/2)
    double Q, invQ;     // minor-coordinate step per major cell (invQ = 0 if Q == 0)
    double icv, K;      // P(b) = s_b * icv + K   (unused when Q == 0)
    double L;           // transaxial length of one major step
    double Au, Bu;      // u at major boundary 0: u0(b) = s_b * Au + Bu
    double du;          // du per major step
    double inv_du;      // 1 / du
    double wslope, wC;  // P(b) ~= wslope * b + wC (candidate windows only)
    double inv_wslope;  // 1 / wslope
    // chord length through one vx x vy cell as a function of the offset t of
    // the line from the cell centre (radially): Lmax for |t| <= e_in, falling
    // linearly to 0 at |t| = e_out (oblique angles only)
    double e_out;       // (vx |c| + vy |s|) / 2
    double inv_de;      // 1 / (e_out - e_in), e_in = |vx |c| - vy |s|| / 2
    double Lmax;        // min(vx / |s|, vy / |c|)
    double e_in;        // |vx |c| - vy |s|| / 2
    int row_major;      // 1: major axis = y (rows), minor = x
    int pad;
};

// Per-bin constants.
struct BinK {
    double sb;          // radial position of the bin
    double inv2h;       // 1 / (2 h), h = sqrt(Rd^2 - s_b^2)   (3D)
    double h;
    double axis_pos_x;  // exact grid position of an axis-parallel ray (x axis)
    double axis_pos_y;  // same on the y axis
};

// Geometry handed to kernels by value.
struct GeoK {
    int dim, nx, ny, nz;
    int n_angles, n_radial, n_subsets, n_planes;
    int n_rings, max_rd;
    int nvox;
    int pad;
    double vx, vy, vz, ds, det_radius;
    double h0;              // (n_radial - 1) / 2: s_b = (b - h0) ds
    const AngleK* ang;      // [n_angles]
    const BinK* bin;        // [n_radial]
    const int2* planes;     // [n_planes] (r1, d)
    const double* kappa;    // [n_radial][2D+1] 3D length per transaxial length
    const int* plane_base;  // [2D+1] first plane of ring difference d (index d + D)
    const double* inv_d;    // [2D+1] 1/d (0 for d = 0)
    // full 2D system model of Sec. IV-A (defaults: one line per bin, no PSF,
    // no attenuation)
    int n_sub;              // parallel sub-rays per bin, spread evenly over ds
    int psf_kx, psf_ky;     // PSF radius in pixels along x, y (0: no PSF)
    float sub_h;            // ds / n_sub: spacing of the sub-rays
    float inv_sub_h;        // n_sub / ds
    float sub_x0;           // offset of sub-ray 0 from the bin's line: sub_h/2 - ds/2
    float inv_nsub;         // 1 / n_sub
    double sub_half;        // largest |offset|: ds/2 - sub_h/2
    const float* att;       // per-bin attenuation factors [n_bins] (natural), or null
    const float* psf;       // PSF taps: [2 psf_kx + 1] along x, then [2 psf_ky + 1] along y
};

// The box B = {0 <= f <= U} of eq:BoundedSet as the FP32 update applies it.
// The branch of S (eq:preconditioner: f < U/2 or not) and of P_t
// (eq:OperatorPt: f~ >= U or not) is taken by comparing an FP32 value with
// U/2 and with U.  half_up and U_up are the smallest floats not below U/2 and
// U, so that for every float x, x < half_up exactly when x < U/2 and
// x >= U_up exactly when x >= U: both comparisons decide as they would
// against the FP64 bound (made on the host by make_box).
struct BoxK {
    float half_up;   // smallest float >= U/2
    float U_up;      // smallest float >= U
    float U;         // U rounded to nearest: the value in (U - f) / p
    float t_lo;      // t of P_t (0 < t < U)
    float t_hi;      // U - t, formed in FP64 and rounded once
};

// S_jj of eq:preconditioner, the relaxed step f~ = f - c nu S G of Table I
// (c = lambda_k alpha_{k,i}) and the projection P_t of eq:OperatorPt at one
// voxel: f~ <= 0 gives t, f~ >= U gives U - t, anything else is kept.
__device__ __forceinline__ float box_step(const BoxK& B, float fj, float pj, float c, float nu, float Gj) {
    const float S = (fj < B.half_up) ? fj / pj : (B.U - fj) / pj;
    const float ft = fj - c * nu * S * Gj;
    return (ft <= 0.0f) ? B.t_lo : ((ft >= B.U_up) ? B.t_hi : ft);
}

struct TxRay {
    double P, Q, invQ, L;
    int row_major;
};

__device__ __forceinline__ double bin_pos(const GeoK& g, int b) { return ((double)b - g.h0) * g.ds; }

__device__ __forceinline__ TxRay tx_ray(const GeoK& g, const AngleK& A, int b) {
    TxRay t;
    t.row_major = A.row_major;
    t.Q = A.Q;
    t.invQ = A.invQ;
    t.L = A.L;
    if (A.Q == 0.0) {
        t.P = A.row_major ? g.bin[b].axis_pos_x : g.bin[b].axis_pos_y;
    } else {
        t.P = __fma_rn(bin_pos(g, b), A.icv, A.K);
    }
    return t;
}

// axial part of the LOR in bin b: the axial grid position of plane (r1, d)
// at major boundary m is r1 + 1/2 + d (tau0 + tauQ m), tau = (u + h)/(2h) the
// fraction of the way from ring r1 to ring r1 + d (rings at slice centres).
struct ZBin {
    double tau0, tauQ, inv_tauQ;
};

__device__ __forceinline__ ZBin z_bin(const GeoK& g, const AngleK& A, int b) {
    const BinK& B = g.bin[b];
    ZBin zb;
    double u0 = __fma_rn(bin_pos(g, b), A.Au, A.Bu);
    zb.tau0 = (u0 + B.h) * B.inv2h;
    zb.tauQ = A.du * B.inv2h;
    zb.inv_tauQ = A.inv_du * (2.0 * B.h);
    return zb;
}

// psi-interval [lo, hi] of cell `cell` for a coordinate starting at g0 and
// moving by Q over psi in [0,1]; empty when hi <= lo.
__device__ __forceinline__ void cell_interval(double g0, double Q, double invQ, int cell,
                                              double& lo, double& hi) {
    if (Q == 0.0) {
        bool in = (floor(g0) == (double)cell);
        lo = 0.0;
        hi = in ? 1.0 : 0.0;
        return;
    }
    double t0 = ((double)cell - g0) * invQ;
    double t1 = ((double)cell + 1.0 - g0) * invQ;
    lo = fmax(0.0, fmin(t0, t1));
    hi = fmin(1.0, fmax(t0, t1));
}

// s_b - u_c for bin b and pixel (ix, iy): the bin's radial position minus
// that of the pixel centre (2D, oblique angles)
__device__ __forceinline__ double pixel_ts(const GeoK& g, const AngleK& A, int ix, int iy, int b) {
    const double xc = ((double)ix - 0.5 * (double)(g.nx - 1)) * g.vx;
    const double yc = ((double)iy - 0.5 * (double)(g.ny - 1)) * g.vy;
    const double uc = __fma_rn(xc, A.c, yc * A.s);
    return __fma_rn((double)b - g.h0, g.ds, -uc);
}

// Mean chord of the n_sub sub-rays of a bin through one pixel (oblique
// angle).  Sub-ray k sits at offset t_k = a + k h from the pixel centre
// (a = ts + sub_x0, h = sub_h); its chord through the vx x vy pixel is
// Lmax * T(t_k), T(t) = clamp((e_out - |t|) / (e_out - e_in), 0, 1), which is
// linear on (-e_out, -e_in], 1 on (-e_in, e_in], linear on (e_in, e_out] and
// 0 elsewhere.  The sum over k is taken piece by piece in closed form: the
// samples in a piece (lo, hi] are k0..k1 with k0 = floor((lo - a)/h) + 1,
// k1 = floor((hi - a)/h), and on a linear piece they add up to
// n v0 +- h n (n - 1) / 2 (times the slope), v0 the value at sample k0.
// Adjacent pieces share the boundary expression, so every sample is counted
// once.
__device__ __forceinline__ float subray_weight(const GeoK& g, const AngleK& A, double ts) {
    const float a = (float)ts + g.sub_x0;
    const float h = g.sub_h, ih = g.inv_sub_h;
    const int last = g.n_sub - 1;
    const float eo = (float)A.e_out, ei = (float)A.e_in, ide = (float)A.inv_de;
    const int b0 = (int)floorf((-eo - a) * ih);
    const int b1 = (int)floorf((-ei - a) * ih);
    const int b2 = (int)floorf((ei - a) * ih);
    const int b3 = (int)floorf((eo - a) * ih);
    float s = 0.0f;
    int k0 = max(b0 + 1, 0), k1 = min(b1, last);
    if (k1 >= k0) {                          // rising edge: (e_out + t) / de
        const float n = (float)(k1 - k0 + 1);
        const float c0 = eo + fmaf((float)k0, h, a);      // value at the first sample, times de
        s += ide * (n * c0 + h * 0.5f * n * (n - 1.0f));
    }
    k0 = max(b1 + 1, 0);
    k1 = min(b2, last);
    if (k1 >= k0) s += (float)(k1 - k0 + 1); // plateau
    k0 = max(b2 + 1, 0);
    k1 = min(b3, last);
    if (k1 >= k0) {                          // falling edge: (e_out - t) / de
        const float n = (float)(k1 - k0 + 1);
        const float c0 = eo - fmaf((float)k0, h, a);
        s += ide * (n * c0 - h * 0.5f * n * (n - 1.0f));
    }
    return (float)A.Lmax * s * g.inv_nsub;
}

// Axis-parallel angle: the number of sub-rays of bin b whose line lies in
// cell `cell` of the minor axis (n cells of size v; half-open cells, the
// position in FP64 as for a single line off the grid)
__device__ __forceinline__ int subray_axis_count(const GeoK& g, int b, int cell, int n, double v) {
    const double sb = bin_pos(g, b);
    int cnt = 0;
    for (int k = 0; k < g.n_sub; ++k) {
        const double off = (((double)k + 0.5) / (double)g.n_sub - 0.5) * g.ds;
        const int c = (int)floor((sb + off + 0.5 * n * v) / v);
        cnt += (c == cell) ? 1 : 0;
    }
    return cnt;
}

__device__ __forceinline__ float subray_axis_weight(const GeoK& g, const AngleK& A, int cnt) {
    return (float)A.L * (float)cnt * g.inv_nsub;
}

// range of major cells [m0, m1] on which the minor coordinate can be inside
// [0, n_minor); conservative by one cell on each side.
__device__ __forceinline__ void major_range(const TxRay& t, int n_major, int n_minor, int& m0, int& m1) {
    if (t.Q == 0.0) {
        double c = floor(t.P);
        if (c >= 0.0 && c < (double)n_minor) { m0 = 0; m1 = n_major - 1; }
        else { m0 = 0; m1 = -1; }
        return;
    }
    double B0 = (0.0 - t.P) * t.invQ;
    double B1 = ((double)n_minor - t.P) * t.invQ;
    double lo = fmin(B0, B1), hi = fmax(B0, B1);
    double flo = floor(lo) - 1.0, fhi = ceil(hi) + 1.0;
    if (flo < 0.0) flo = 0.0;
    if (fhi > (double)(n_major - 1)) fhi = (double)(n_major - 1);
    if (fhi < flo) { m0 = 0; m1 = -1; return; }
    m0 = (int)flo;
    m1 = (int)fhi;
}

}  // namespace petos
