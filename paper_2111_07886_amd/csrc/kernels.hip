// kernels.hip -- gfx950 kernels of one SDP-BSREM subiteration.
//
//   k_fp      ray-driven forward projection of a subset, fused with the
//             Poisson ratio w = 1 - y/(q + r) (or plain q, or the FP64
//             log-likelihood partials of eq:FidelityTerm)
//   k_bp      voxel-driven gather back-projection with the subset's sinogram
//             footprint staged in LDS (no atomics), fused with the RDP gradient
//             (eqn:gradRD), the smoothness measure mu (Sec. III-B) and
//             G = A_i^T w + (beta/M) grad R
//   k_update  nu of eq:nuki, S of eq:preconditioner, the relaxed step and
//             P_t of eq:OperatorPt, plus the FP64 sum of the new iterate
//   k_rdp     FP64 partials of R(f) (eq:RDP) for the objective
//
// FP64 sums are deterministic: fixed-order block trees, then the last block
// adds the per-block partials in index order (see Reduction).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>

#include "devutil.h"
#include "internal.h"

namespace petos {

__global__ __launch_bounds__(256) void k_finalize(Reduction R, int n) {
    __shared__ double s_red[4];
    double t = sum_partials(R.part, n, s_red);
    if (threadIdx.x == 0) *R.total = t;
}

// ------------------------------------------------------------------ forward projection

struct FPArgs {
    const float* f;
    const float* y;
    const float* r;
    float* out;
    const int* angles;
    int n_al;
    int mode;
    Reduction red;
    const float* att;        // per-bin attenuation factors (natural), or null
};

// Sub-ray model (Sec. IV-A): the bin's projection as the mean over its
// sub-rays, accumulated over major cells [s0, s1] of the ray.  Each pixel the
// strip of sub-rays can cross gets the same weight the back-projector gives
// it, so the two are an adjoint pair.
__device__ __forceinline__ float fp_subray_acc(const GeoK& g, const FPArgs& A, const AngleK& AK, int b, int s0,
                                               int s1) {
    const int row_major = AK.row_major;
    const int n_minor = row_major ? g.nx : g.ny;
    const int sx = row_major ? 1 : g.nx;
    const int sm = row_major ? g.nx : 1;
    float acc = 0.0f;
    if (AK.Q == 0.0) {
        // axis-parallel: the sub-rays stay in a few minor cells, the same in
        // every major cell
        const double v = row_major ? g.vx : g.vy;
        const double sb = bin_pos(g, b);
        const int c_lo = max((int)floor((sb - g.sub_half + 0.5 * n_minor * v) / v) - 1, 0);
        const int c_hi = min((int)floor((sb + g.sub_half + 0.5 * n_minor * v) / v) + 1, n_minor - 1);
        for (int c = c_lo; c <= c_hi; ++c) {
            const int cnt = subray_axis_count(g, b, c, n_minor, v);
            if (cnt == 0) continue;
            const float w = subray_axis_weight(g, AK, cnt);
            float part = 0.0f;
            for (int m = s0; m <= s1; ++m) {
                if (A.mode == FP_COUNT) { part += 1.0f; continue; }
                part = fmaf(w, img_at(A.f, m * sm + c * sx), part);
            }
            acc += part;
        }
        return acc;
    }
    const TxRay tx = tx_ray(g, AK, b);
    const double hsg = fabs(AK.icv) * g.sub_half;     // strip half-width in minor cells
    for (int m = s0; m <= s1; ++m) {
        const double g0 = __fma_rn(tx.Q, (double)m, tx.P), g1 = g0 + tx.Q;
        const int c0 = max((int)floor(fmin(g0, g1) - hsg) - 1, 0);
        const int c1 = min((int)floor(fmax(g0, g1) + hsg) + 1, n_minor - 1);
        for (int c = c0; c <= c1; ++c) {
            const int ix = row_major ? c : m, iy = row_major ? m : c;
            const float w = subray_weight(g, AK, pixel_ts(g, AK, ix, iy, b));
            if (w > 0.0f) {
                if (A.mode == FP_COUNT) { acc += 1.0f; continue; }
                acc = fmaf(w, img_at(A.f, m * sm + c * sx), acc);
            }
        }
    }
    return acc;
}

// One ray per (thread-row of the block); SEG threads split its major cells.
// The ray's sum does not depend on SEG: its major cells [m0, m1] are cut
// into 64 leaves of ceil(count / 64) consecutive cells, each leaf is summed
// in cell order, and the 64 leaf sums are added by a balanced binary tree.
// A thread takes 64 / SEG consecutive leaves and adds them by that tree's
// subtree (LeafTree); the SEG threads of a ray are adjacent lanes of one
// wave and add their subtrees by its top levels (group_sum_balanced).  So
// every SEG, and the batched kernels' choice of it, give the same bits.
template <int DIM, int SEG, bool SUB = false>
__device__ void fp_body(const GeoK& g, const FPArgs& A, long long vblock) {
    static_assert(DIM == 2, "the 3D forward projector is k_fp3");
    static_assert(SEG == 1 || (64 % SEG == 0), "segments of a ray stay in one wave");
    constexpr int RPB = NT / SEG;
    __shared__ double s_red[NT / 64];
    int lr = (SEG == 1) ? threadIdx.x : threadIdx.x / SEG;
    // one ray per wave: its index is wave-uniform, so that its decode, its
    // angle and bin records and its major range run once on the scalar unit
    if (SEG == 64) lr = __builtin_amdgcn_readfirstlane(lr);
    const int seg = (SEG == 1) ? 0 : threadIdx.x % SEG;
    const int P = g.n_planes, Nr = g.n_radial;
    const long long nrays = (long long)A.n_al * P * Nr;
    const long long ray = vblock * RPB + lr;
    const bool valid = ray < nrays;

    float acc = 0.0f;
    int b = 0, plane = 0, al = 0, a = 0;
    // the ray's y, r (and attenuation factor), loaded before the walk so that
    // their latency overlaps it
    const bool needs_data = A.mode == FP_RATIO || A.mode == FP_EM || A.mode == FP_OBJECTIVE;
    float yv = 0.0f, rv = 0.0f, atv = 1.0f;
    if (valid) {
        // a 2D pass holds fewer than 2^31 rays (checked with the descriptor):
        // 32-bit index arithmetic
        const int r32 = (int)ray;
        b = r32 % Nr;
        const int t = r32 / Nr;
        plane = t % P;
        al = t / P;
        a = A.angles[al];
        if (seg == 0) {
            const long long nat = ((long long)plane * g.n_angles + a) * Nr + b;
            if (needs_data) {
                yv = A.y[nat];
                rv = A.r[nat];
            }
            if (A.att != nullptr) atv = A.att[nat];
        }
        const AngleK& AK = g.ang[a];
        TxRay tx = tx_ray(g, AK, b);
        int n_major = tx.row_major ? g.ny : g.nx;
        int n_minor = tx.row_major ? g.nx : g.ny;
        int m0, m1;
        if (SUB) {
            // the major cells the strip of sub-rays can cross: the union of
            // the ranges of its two edge lines
            if (tx.Q == 0.0) {
                m0 = 0;
                m1 = n_major - 1;
            } else {
                const double hsg = fabs(AK.icv) * g.sub_half;
                TxRay e = tx;
                int a0, a1, c0, c1;
                e.P = tx.P - hsg;
                major_range(e, n_major, n_minor, a0, a1);
                e.P = tx.P + hsg;
                major_range(e, n_major, n_minor, c0, c1);
                if (a1 < a0) { a0 = c0; a1 = c1; }
                if (c1 < c0) { c0 = a0; c1 = a1; }
                m0 = min(a0, c0);
                m1 = max(a1, c1);
            }
        } else {
            major_range(tx, n_major, n_minor, m0, m1);
        }
        const int cnt = m1 - m0 + 1;
        const int per = (cnt + 63) / 64;              // cells per leaf
        constexpr int LPT = 64 / SEG;                 // leaves per thread
        const int sx = tx.row_major ? 1 : g.nx;       // stride along the minor cell index
        const int sm = tx.row_major ? g.nx : 1;       // stride along the major index
        const int qstep = (tx.Q > 0.0) ? 1 : -1;
        LeafTree<LPT> tree;
        for (int k = 0; k < LPT; ++k) {
            const int s0 = m0 + (seg * LPT + k) * per;
            const int s1 = min(m1, s0 + per - 1);
            float leaf = 0.0f;
            if (SUB) {
                if (s0 <= s1) leaf = fp_subray_acc(g, A, AK, b, s0, s1);
            } else {
                // Over major cell m the ray's minor coordinate runs from
                // gm = P + Q m to gm + Q (|Q| <= 1): it stays in cell c0 =
                // floor(gm), or crosses once into c0 + qstep at the fraction
                // t of the cell's length, t = (c0 + 1 - gm)/Q (Q > 0) or
                // (c0 - gm)/Q (Q < 0).  The cell and the crossing are decided
                // in FP64; t and the two lengths are formed in FP32 from the
                // FP64 distance to the crossed edge.
                const float Lf = (float)tx.L;
                const float invQf = (float)tx.invQ;
                const bool up = tx.Q >= 0.0;
                for (int m = s0; m <= s1; ++m) {
                    const double gm = __fma_rn(tx.Q, (double)m, tx.P);
                    const double cf = floor(gm);
                    const int c0 = (int)cf;
                    const double edge = up ? cf + 1.0 : cf;             // the edge the ray may cross
                    const double ge = gm + tx.Q;
                    const bool cross = up ? (ge > edge) : (ge < edge);
                    float a1 = Lf, a2 = 0.0f;
                    if (cross) {
                        a1 = Lf * ((float)(edge - gm) * invQf);
                        a2 = Lf - a1;
                    }
                    const int c1 = c0 + qstep;
                    const bool in0 = c0 >= 0 && c0 < n_minor && a1 > 0.0f;
                    const bool in1 = cross && c1 >= 0 && c1 < n_minor && a2 > 0.0f;
                    if (A.mode == FP_COUNT) {
                        leaf += (in0 ? 1.0f : 0.0f) + (in1 ? 1.0f : 0.0f);
                        continue;
                    }
                    // 24-bit signed products (full-rate multiplies; the
                    // descriptor check keeps nx, ny below 2^23)
                    const int base = __mul24(m, sm);
                    if (in0) leaf = fmaf(a1, img_at(A.f, base + __mul24(c0, sx)), leaf);
                    if (in1) leaf = fmaf(a2, img_at(A.f, base + __mul24(c1, sx)), leaf);
                }
            }
            tree.add(k, leaf);
        }
        acc = tree.sum;
    }
    // the subtrees of a ray's SEG threads (adjacent lanes; every lane of the
    // wave takes part), added by the tree's top levels, valid in each lane
    acc = group_sum_balanced<SEG>(acc);
    double term = 0.0;
    if (seg == 0 && valid) {
        long long nat = ((long long)plane * g.n_angles + a) * Nr + b;
        if (A.att != nullptr && A.mode != FP_COUNT && A.mode != FP_COMPACT) {
            // attenuated model: q = att (P f); the back-projected weights carry att too
            const float q = atv * acc;
            if (A.mode == FP_RATIO) A.out[ray] = atv * (1.0f - yv / (q + rv));
            else if (A.mode == FP_EM) A.out[ray] = atv * (yv / (q + rv));
            else if (A.mode == FP_PLAIN) A.out[nat] = q;
            else term = (double)q - (double)yv * log((double)q + (double)rv);
        } else if (A.mode == FP_RATIO) {
            float q = acc;
            A.out[ray] = 1.0f - yv / (q + rv);
        } else if (A.mode == FP_EM) {
            A.out[ray] = yv / (acc + rv);
        } else if (A.mode == FP_COUNT || A.mode == FP_COMPACT) {
            A.out[ray] = acc;
        } else if (A.mode == FP_PLAIN) {
            A.out[nat] = acc;
        } else {
            double q = (double)acc;
            term = q - (double)yv * log(q + (double)rv);
        }
    }
    if (A.mode == FP_OBJECTIVE) write_partial(term, A.red, s_red, vblock);
}

template <int DIM, int SEG, bool SUB>
__global__ __launch_bounds__(NT) void k_fp(GeoK g, FPArgs A) {
    fp_body<DIM, SEG, SUB>(g, A, blockIdx.x);
}

// ------------------------------------------------------------------ back projection

struct BPArgs {
    const float* w;          // null => unit weights (sensitivity)
    long long w_sp, w_sa;    // w index = plane * w_sp + angle_index * w_sa + b
    int w_natural;           // angle_index = natural angle (1) or position in the list (0)
    const int* angles;
    int n_al;
    float* out;
    const float* f;          // non-null => fused stencil, out = G
    float* mu;
    int want_mu;
    float beta_over_M, gamma_R, eps;
    const double* part_f;
    int n_part_f;
    Reduction red_mu;
    int nb_max;              // staged bins per angle
    int chunk;               // angles staged together
    // fused update of a 2D subiteration (fnew non-null): f is then the
    // snapshot of the entering iterate, G is not stored, and the new iterate
    // of the tile goes to fnew with the FP64 partials of its sum
    float* fnew;
    const float* pnorm;
    float* nu_frozen;
    int nu_mode;
    float step, nu1, nu2;
    BoxK box;
    const double* part_mu;
    int n_part_mu;
    Reduction red_f;
    const float* osem_sens;  // OSEM (fused): f <- f * (A_i^T w) / s_i with w = y/(q+r)
    const float* att;        // per-bin attenuation factors applied to natural-layout (or unit) w, or null
};

// nu of eq:nuki, S of eq:preconditioner, the relaxed step of Table I and P_t
// of eq:OperatorPt at one voxel; meanmu is mean(mu) when nu is recomputed,
// nu_in the frozen nu of the voxel when it is reused
__device__ __forceinline__ float sdp_update(float fj, float Gj, float pj, float muj, float meanmu, float nu_in,
                                            float* nu_frozen, long long j, int nu_mode, float step, float nu1,
                                            float nu2, const BoxK& box) {
    float nu = 1.0f;
    if (nu_mode == NU_COMPUTE || nu_mode == NU_COMPUTE_FREEZE) {
        nu = fminf(nu2, fmaxf(nu1, meanmu / muj));
        if (nu_mode == NU_COMPUTE_FREEZE) nu_frozen[j] = nu;
    } else if (nu_mode == NU_FROZEN) {
        nu = nu_in;
    }
    return box_step(box, fj, pj, step, nu, Gj);
}

// Per-pixel inputs of the update (p, mu, frozen nu, OSEM sensitivity), read
// by the owner thread of an inside pixel before the gather so that their
// latency overlaps it.
struct PixPre {
    float p, mu, nu, sens;
};

__device__ __forceinline__ PixPre pixel_prefetch(const BPArgs& A, bool active, long long j) {
    PixPre r{1.0f, 1.0f, 1.0f, 0.0f};
    if (!active || A.fnew == nullptr) return r;
    if (A.osem_sens != nullptr) {
        r.sens = A.osem_sens[j];
        return r;
    }
    r.p = A.pnorm[j];
    if (A.nu_mode == NU_COMPUTE || A.nu_mode == NU_COMPUTE_FREEZE) r.mu = A.mu[j];
    else if (A.nu_mode == NU_FROZEN) r.nu = A.nu_frozen[j];
    return r;
}

// Image-space part of a 2D subiteration at pixel (ix, iy), from the halo
// tile s_f of the snapshot (tile position lx, ly) and acc = the back-projected
// weights at the pixel: grad R, G = acc + (beta/M) grad R and either mu
// (Sec. III-B), the update of Table I, or the OSEM update.  Returns the
// pixel's share of the tile's FP64 partial (new f, or mu).
__device__ __forceinline__ double pixel_finish(const GeoK& g, const BPArgs& A, const float* s_f, int HX, int HY,
                                               int lx, int ly, int ix, int iy, float acc, float meanf,
                                               float meanmu, const PixPre& pre) {
    double part = 0.0;
    float gradR, gmag;
    stencil_at<2>(s_f, HX, HY, lx + 1, ly + 1, 0, ix, iy, 0, g, A.gamma_R, A.eps, gradR, gmag);
    const long long j = (long long)iy * g.nx + ix;
    const float Gj = fmaf(A.beta_over_M, gradR, acc);
    if (A.fnew != nullptr && A.osem_sens != nullptr) {
        // ordered-subsets EM (Hudson-Larkin): multiplicative update
        const float fj = s_f[(ly + 1) * HX + lx + 1];
        const float sj = pre.sens;
        const float fn = (sj > 0.0f) ? fj * acc / sj : fj;
        A.fnew[j] = fn;
        part = (double)fn;
    } else if (A.fnew != nullptr) {
        const float fj = s_f[(ly + 1) * HX + lx + 1];
        const float fn = sdp_update(fj, Gj, pre.p, pre.mu, meanmu, pre.nu, A.nu_frozen, j, A.nu_mode, A.step,
                                    A.nu1, A.nu2, A.box);
        A.fnew[j] = fn;
        part = (double)fn;
    } else {
        A.out[j] = Gj;
        if (A.want_mu) {
            const float mu = fmaxf(0.01f, gmag / meanf);
            A.mu[j] = mu;
            part = (double)mu;
        }
    }
    return part;
}

// Tile of the back-projector: X x Y pixels, AG threads per pixel (each takes
// every AG-th angle of the subset; partial sums added in group order).
template <int X_, int Y_, int AG_>
struct Tile {
    static constexpr int X = X_, Y = Y_, AG = AG_;
    static_assert(X_ * Y_ * AG_ == 256, "256 threads per block");
};
using Tile2L = Tile<16, 16, 1>;   // large images
using Tile2S = Tile<8, 8, 4>;     // small images: 4 angle groups

constexpr int MAXCH = 16;    // angles per staging chunk
constexpr int ANG_W = (int)(sizeof(AngleK) / sizeof(double));   // 8-byte words of an angle record
static_assert(sizeof(AngleK) % sizeof(double) == 0, "angle records are copied in 8-byte words");

// LEAN (the batched kernel, whose occupancy is register-bound) reads the
// angle records from the geometry table in the gather (only the axis-parallel
// and many-bin windows need them) and the pixel's update inputs after it;
// otherwise both are fetched before the gather.
template <class T, bool SUB = false, bool ATT = false, bool LEAN = false>
__device__ void bp_body(const GeoK& g, const BPArgs& A, int vblock) {
    constexpr int NV = T::X * T::Y;                 // pixels per tile
    constexpr int HX = T::X + 2, HY = T::Y + 2;
    extern __shared__ float s_w[];
    __shared__ float s_f[HX * HY];
    __shared__ int s_blo[MAXCH], s_nb[MAXCH], s_a[MAXCH], s_two[MAXCH];
    // oblique angles, per angle of the chunk: the tile's pixel (0, 0) centre
    // in bin units relative to blo, the steps per pixel in x and y, e_out in
    // bins, and the trapezoid's e_out, 1 / (e_out - e_in) and Lmax
    __shared__ float s_p0[MAXCH], s_dpx[MAXCH], s_dpy[MAXCH], s_E[MAXCH], s_eo[MAXCH], s_ide[MAXCH], s_lm[MAXCH];
    __shared__ AngleK s_ang[MAXCH];
    __shared__ double s_red[NT / 64];
    __shared__ float s_acc[T::AG > 1 ? T::AG * NV : 1];

    const int tiles_x = (g.nx + T::X - 1) / T::X;
    const int tx0 = (vblock % tiles_x) * T::X;
    const int ty0 = (vblock / tiles_x) * T::Y;
    const int vox = threadIdx.x % NV;               // pixel of the tile
    // angle group: a whole number of waves each, so the group index (and
    // with it the gather's angle loop) is wave-uniform and its index
    // arithmetic runs on the scalar unit
    static_assert(NV % 64 == 0, "angle groups of whole waves");
    const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / NV);
    const int lx = vox % T::X, ly = vox / T::X;
    const int ix = tx0 + lx, iy = ty0 + ly;
    const bool inside = ix < g.nx && iy < g.ny;
    const int Nr = g.n_radial;
    const int nb_max = A.nb_max;
    const double inv_ds = 1.0 / g.ds;
    // pixel centre in mm
    const double xc = ((double)ix - 0.5 * (double)(g.nx - 1)) * g.vx;
    const double yc = ((double)iy - 0.5 * (double)(g.ny - 1)) * g.vy;

    // tile box in mm
    const double X0 = ((double)tx0 - 0.5 * g.nx) * g.vx, X1 = X0 + T::X * g.vx;
    const double Y0 = ((double)ty0 - 0.5 * g.ny) * g.vy, Y1 = Y0 + T::Y * g.vy;

    // halo tile of f (fused stencil), the pixel's update inputs and mean f:
    // independent of the gather, so issued first; the halo goes to LDS once
    // the first chunk's angle records are on their way
    constexpr int HALO_PT = (HX * HY + NT - 1) / NT;
    float hv[HALO_PT];
    if (A.f != nullptr) {
#pragma unroll
        for (int k = 0; k < HALO_PT; ++k) {
            const int e = threadIdx.x + k * NT;
            const int hx = e % HX, hy = e / HX;
            const int gx = tx0 - 1 + hx, gy = ty0 - 1 + hy;
            float v = 0.0f;
            if (e < HX * HY && gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny) v = A.f[(long long)gy * g.nx + gx];
            hv[k] = v;
            if (LEAN && e < HX * HY) s_f[e] = v;
        }
    }
    const PixPre pre_early = LEAN ? PixPre{} : pixel_prefetch(A, inside && grp == 0, (long long)iy * g.nx + ix);
    float meanf = 1.0f;
    if (A.f != nullptr && A.want_mu) meanf = (float)(sum_partials(A.part_f, A.n_part_f, s_red) / (double)g.nvox);
    float meanmu = 1.0f;
    const bool want_meanmu = A.fnew != nullptr && (A.nu_mode == NU_COMPUTE || A.nu_mode == NU_COMPUTE_FREEZE);
    // the mu partials: with at most NT of them, loaded now and added after the
    // gather, so that the load overlaps the staging
    const bool mu_early = want_meanmu && A.n_part_mu <= NT;
    // With one wave of pixels (NV == 64) only wave 0 needs the totals: it
    // loads all the mu partials (lane l: partials l, l+64, l+128, l+192) and
    // adds them without the block's barriers, in block_sum's order.
    constexpr bool WAVE0_TOTALS = NV == 64 && !LEAN;
    double mu_q[WAVE0_TOTALS ? 4 : 1] = {};
    double mu_part = 0.0;
    if (mu_early) {
        if constexpr (WAVE0_TOTALS) {
            if (grp == 0) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int t = (int)threadIdx.x + 64 * k;
                    mu_q[k] = t < A.n_part_mu ? A.part_mu[t] : 0.0;
                }
            }
        } else {
            mu_part = partial_early(A.part_mu, A.n_part_mu);
        }
    }
    if (want_meanmu && !mu_early) meanmu = (float)(sum_partials(A.part_mu, A.n_part_mu, s_red) / (double)g.nvox);

    float acc = 0.0f;
    for (int c0 = 0; c0 < A.n_al; c0 += A.chunk) {
        const int nch = min(A.chunk, A.n_al - c0);
        // (1) the chunk's angle records into LDS and, with a sinogram, the
        // per-angle bin footprint of the tile (+1 bin margin)
        if (!LEAN) for (int e = threadIdx.x; e < nch * ANG_W; e += NT) {
            const int j = e / ANG_W, q = e - j * ANG_W;
            const unsigned long long* src = reinterpret_cast<const unsigned long long*>(&g.ang[A.angles[c0 + j]]);
            reinterpret_cast<unsigned long long*>(&s_ang[j])[q] = src[q];
        }
        if (threadIdx.x < nch) {
            const int j = threadIdx.x;
            const int a = A.angles[c0 + j];
            const AngleK& AK = g.ang[a];
            s_a[j] = a;
            if (A.w != nullptr) {
                double umin = 1e300, umax = -1e300;
                for (int k = 0; k < 4; ++k) {
                    const double x = (k & 1) ? X1 : X0, y = (k & 2) ? Y1 : Y0;
                    const double u = x * AK.c + y * AK.s;     // radial position
                    umin = fmin(umin, u);
                    umax = fmax(umax, u);
                }
                int blo = max((int)floor(umin / g.ds + g.h0) - 1, 0);
                int bhi = min((int)ceil(umax / g.ds + g.h0) + 1, Nr - 1);
                s_blo[j] = blo;
                s_nb[j] = max(0, min(bhi - blo + 1, nb_max));
                // a pixel's window holds at most two bins when e_out <= ds
                s_two[j] = (AK.Q != 0.0 && AK.e_out <= g.ds) ? 1 : 0;
                if (AK.Q != 0.0) {
                    const double xc0 = ((double)tx0 - 0.5 * (double)(g.nx - 1)) * g.vx;
                    const double yc0 = ((double)ty0 - 0.5 * (double)(g.ny - 1)) * g.vy;
                    const double u00 = __fma_rn(xc0, AK.c, yc0 * AK.s);
                    s_p0[j] = (float)(__fma_rn(u00, inv_ds, g.h0) - (double)blo);
                    s_dpx[j] = (float)(g.vx * AK.c * inv_ds);
                    s_dpy[j] = (float)(g.vy * AK.s * inv_ds);
                    s_E[j] = (float)(AK.e_out * inv_ds);
                    s_eo[j] = (float)AK.e_out;
                    s_ide[j] = (float)AK.inv_de;
                    s_lm[j] = (float)AK.Lmax;
                }
            }
        }
        if (!LEAN && c0 == 0 && A.f != nullptr) {
#pragma unroll
            for (int k = 0; k < HALO_PT; ++k) {
                const int e = threadIdx.x + k * NT;
                if (e < HX * HY) s_f[e] = hv[k];
            }
        }
        __syncthreads();
        if (A.w != nullptr) {
            // (2) stage the footprint rows into LDS
            const int nel = nch * nb_max;
            for (int e = threadIdx.x; e < nel; e += NT) {
                const int j = e / nb_max, col = e - j * nb_max;
                if (col < s_nb[j]) {
                    const int al = c0 + j;
                    const int aidx = A.w_natural ? s_a[j] : al;
                    const long long idx = (long long)aidx * A.w_sa + s_blo[j] + col;
                    s_w[e] = ATT ? A.w[idx] * A.att[idx] : A.w[idx];
                }
            }
            __syncthreads();
        }

        // (3) gather: every bin whose ray crosses this pixel.  Oblique angles
        // use the closed form of the chord length through the pixel (a
        // trapezoid in the radial offset t of the ray from the pixel centre),
        // so the window holds just the bins with |t| < e_out; axis-parallel
        // angles keep the half-open cell rule of the forward projector.
        if (inside) {
            for (int j = grp; j < nch; j += T::AG) {
                const int al = c0 + j;
                // from LDS (a global load per angle would stall the gather),
                // wave-uniform as j is
                const int a = __builtin_amdgcn_readfirstlane(s_a[j]);
                const AngleK& AK = LEAN ? g.ang[a] : s_ang[j];
                const int aidx = A.w_natural ? a : al;
                const int bst = s_blo[j], nbs = s_nb[j];
                auto wval = [&](int b) -> float {
                    if (A.w == nullptr) return ATT ? A.att[(long long)a * Nr + b] : 1.0f;
                    const int bcol = b - bst;
                    if (bcol >= 0 && bcol < nbs) return s_w[j * nb_max + bcol];
                    const long long idx = (long long)aidx * A.w_sa + b;
                    return ATT ? A.w[idx] * A.att[idx] : A.w[idx];
                };
                if (SUB) {
                    // sub-ray model: the weights of the forward projector's fp_subray_acc
                    if (AK.Q != 0.0) {
                        const double uc = __fma_rn(xc, AK.c, yc * AK.s);
                        const double reach = AK.e_out + g.sub_half;
                        const int b0 = max((int)ceil((uc - reach) * inv_ds + g.h0), 0);
                        const int b1 = min((int)floor((uc + reach) * inv_ds + g.h0), Nr - 1);
                        for (int b = b0; b <= b1; ++b) {
                            const float w = subray_weight(g, AK, pixel_ts(g, AK, ix, iy, b));
                            if (w > 0.0f) acc = fmaf(w, wval(b), acc);
                        }
                    } else {
                        const int mc = AK.row_major ? ix : iy;
                        const int n = AK.row_major ? g.nx : g.ny;
                        const double v = AK.row_major ? g.vx : g.vy;
                        const double pc = ((double)mc - 0.5 * (double)(n - 1)) * v;
                        const int b0 = max((int)floor((pc - 0.5 * v - g.sub_half) * inv_ds + g.h0) - 1, 0);
                        const int b1 = min((int)ceil((pc + 0.5 * v + g.sub_half) * inv_ds + g.h0) + 1, Nr - 1);
                        for (int b = b0; b <= b1; ++b) {
                            const int cnt = subray_axis_count(g, b, mc, n, v);
                            if (cnt > 0) acc = fmaf(subray_axis_weight(g, AK, cnt), wval(b), acc);
                        }
                    }
                } else if (A.w != nullptr && s_two[j]) {
                    // oblique, at most two bins per pixel: the pixel centre's
                    // position p in the staged window's bin units, in FP32 from
                    // the tile's reference (|p| within the window, its rounding
                    // near 1e-6 bins); bins k0 = the first above p - e_out/ds
                    // and k0 + 1, each weighted by the trapezoid of its radial
                    // offset (0 outside the window's reach)
                    const float p = fmaf((float)ly, s_dpy[j], fmaf((float)lx, s_dpx[j], s_p0[j]));
                    const int k0 = (int)floorf(p - s_E[j]) + 1;
                    const float dsf = (float)g.ds, eo = s_eo[j], ide = s_ide[j], lmax = s_lm[j];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int k = k0 + u;
                        const float tt = fabsf((p - (float)k) * dsf);
                        const float len = lmax * fminf(1.0f, (eo - tt) * ide);
                        if (len > 0.0f) {
                            if (k >= 0 && k < nbs) acc = fmaf(len, s_w[j * nb_max + k], acc);
                            else if (bst + k >= 0 && bst + k < Nr) acc = fmaf(len, wval(bst + k), acc);
                        }
                    }
                } else if (AK.Q != 0.0) {
                    const double uc = __fma_rn(xc, AK.c, yc * AK.s);
                    const int b0 = max((int)ceil((uc - AK.e_out) * inv_ds + g.h0), 0);
                    const int b1 = min((int)floor((uc + AK.e_out) * inv_ds + g.h0), Nr - 1);
                    // the radial offset of bin b0's line from the pixel centre
                    // in FP64, the window's later bins (|t| < e_out, at most
                    // three) in FP32 steps of ds from it
                    const float t0 = (float)__fma_rn((double)b0 - g.h0, g.ds, -uc);
                    const float dsf = (float)g.ds, eo = (float)AK.e_out, ide = (float)AK.inv_de;
                    const float lmax = (float)AK.Lmax;
                    for (int b = b0; b <= b1; ++b) {
                        const float tt = fabsf(fmaf((float)(b - b0), dsf, t0));
                        const float len = lmax * fminf(1.0f, (eo - tt) * ide);
                        if (len > 0.0f) acc = fmaf(len, wval(b), acc);
                    }
                } else {
                    const int m = AK.row_major ? iy : ix;
                    const int mc = AK.row_major ? ix : iy;
                    // axis-parallel: bins whose exact position falls in cell mc
                    const double base = AK.wC;
                    const double bA = ((double)mc - 1e-7 - base) * AK.inv_wslope;
                    const double bB = ((double)mc + 1.0 + 1e-7 - base) * AK.inv_wslope;
                    const int b0 = (int)fmax(floor(fmin(bA, bB)), 0.0);
                    const int b1 = (int)fmin(ceil(fmax(bA, bB)), (double)(Nr - 1));
                    for (int b = b0; b <= b1; ++b) {
                        const TxRay tx = tx_ray(g, AK, b);
                        double ax, bx;
                        cell_interval(__fma_rn(tx.Q, (double)m, tx.P), tx.Q, tx.invQ, mc, ax, bx);
                        if (bx > ax) acc = fmaf((float)(tx.L * (bx - ax)), wval(b), acc);
                    }
                }
            }
        }
        __syncthreads();
    }
    if (T::AG > 1) {
        s_acc[grp * NV + vox] = acc;
        __syncthreads();
        acc = 0.0f;
        for (int k = 0; k < T::AG; ++k) acc += s_acc[k * NV + vox];
    }
    const bool owner = grp == 0;

    if (A.f == nullptr) {
        if (inside && owner) A.out[(long long)iy * g.nx + ix] = acc;
        return;
    }

    if (mu_early) {
        if constexpr (WAVE0_TOTALS) {
            if (grp == 0) {
                double t = wave_sum(mu_q[0]);
#pragma unroll
                for (int k = 1; k < 4; ++k) t += wave_sum(mu_q[k]);
                meanmu = (float)(t / (double)g.nvox);
            }
        } else {
            meanmu = (float)(partials_total(mu_part, s_red) / (double)g.nvox);
        }
    }
    if (!LEAN && A.n_al <= 0) {
#pragma unroll
        for (int k = 0; k < HALO_PT; ++k) {
            const int e = threadIdx.x + k * NT;
            if (e < HX * HY) s_f[e] = hv[k];
        }
    }

    // (4) fused image-space part (the halo tile was loaded before the gather)
    __syncthreads();
    double part = 0.0;
    if (inside && owner) {
        const PixPre pre = LEAN ? pixel_prefetch(A, true, (long long)iy * g.nx + ix) : pre_early;
        part = pixel_finish(g, A, s_f, HX, HY, lx, ly, ix, iy, acc, meanf, meanmu, pre);
    }
    if (A.fnew == nullptr && !A.want_mu) return;
    const Reduction R = A.fnew != nullptr ? A.red_f : A.red_mu;
    if constexpr (WAVE0_TOTALS) {
        // waves 1..3 hold no pixel: the block's sum is wave 0's
        if (grp == 0) {
            const double bs = wave_sum(part);
            if (threadIdx.x == 0) R.part[vblock] = bs;
        }
    } else {
        write_partial(part, R, s_red, vblock);
    }
}

// Partials of sum f over the same tiles, threads and order as the fused
// update writes them (for an iterate handed in by the caller).
template <class T>
__global__ __launch_bounds__(NT) void k_sum_tiles(GeoK g, const float* f, Reduction R) {
    __shared__ double s_red[NT / 64];
    constexpr int NV = T::X * T::Y;
    const int tiles_x = (g.nx + T::X - 1) / T::X;
    const int vox = threadIdx.x % NV;
    const int ix = (blockIdx.x % tiles_x) * T::X + vox % T::X;
    const int iy = (blockIdx.x / tiles_x) * T::Y + vox / T::X;
    double v = 0.0;
    if ((int)threadIdx.x < NV && ix < g.nx && iy < g.ny) v = (double)f[(long long)iy * g.nx + ix];
    write_partial(v, R, s_red, blockIdx.x);
}

template <class T, bool SUB, bool ATT>
__global__ __launch_bounds__(NT) void k_bp(GeoK g, BPArgs A) {
    bp_body<T, SUB, ATT>(g, A, blockIdx.x);
}

// ------------------------------------------------------------------ PSF (Sec. IV-A)

constexpr int BLT = 16;         // output tile of the PSF blur

// out = B in: the separable Gaussian PSF, zero outside the image (so that B
// is symmetric).  One block per 16x16 output tile: the tile and its halo go
// to LDS, the pass along x into LDS, then the pass along y; taps are added in
// ascending order.
__global__ __launch_bounds__(NT) void k_blur2(GeoK g, const float* __restrict__ in, float* __restrict__ out) {
    __shared__ float s_in[(BLT + 2 * PSF_KMAX) * (BLT + 2 * PSF_KMAX)];
    __shared__ float s_x[(BLT + 2 * PSF_KMAX) * BLT];
    const int Kx = g.psf_kx, Ky = g.psf_ky;
    const int W = BLT + 2 * Kx, H = BLT + 2 * Ky;
    const int tiles_x = (g.nx + BLT - 1) / BLT;
    const int tx0 = ((int)blockIdx.x % tiles_x) * BLT, ty0 = ((int)blockIdx.x / tiles_x) * BLT;
    for (int e = threadIdx.x; e < W * H; e += NT) {
        const int hx = e % W, hy = e / W;
        const int x = tx0 - Kx + hx, y = ty0 - Ky + hy;
        s_in[e] = (x >= 0 && x < g.nx && y >= 0 && y < g.ny) ? in[(long long)y * g.nx + x] : 0.0f;
    }
    __syncthreads();
    const float* wx = g.psf;
    const float* wy = g.psf + 2 * Kx + 1;
    for (int e = threadIdx.x; e < BLT * H; e += NT) {
        const int lx = e % BLT, hy = e / BLT;
        float acc = 0.0f;
        for (int k = 0; k <= 2 * Kx; ++k) acc = fmaf(wx[k], s_in[hy * W + lx + k], acc);
        s_x[hy * BLT + lx] = acc;
    }
    __syncthreads();
    const int lx = threadIdx.x % BLT, ly = threadIdx.x / BLT;
    const int x = tx0 + lx, y = ty0 + ly;
    if (x < g.nx && y < g.ny) {
        float acc = 0.0f;
        for (int k = 0; k <= 2 * Ky; ++k) acc = fmaf(wy[k], s_x[(ly + k) * BLT + lx], acc);
        out[(long long)y * g.nx + x] = acc;
    }
}

// The image-space part of a 2D subiteration when the back-projection has to
// be blurred (PSF): Gb = A_i^T w, blurred here over the tile's halo (BLUR) or
// already blurred; the tiles, threads and partials are those of the fused
// back-projector k_bp<T>.
template <class T, bool BLUR>
__global__ __launch_bounds__(NT) void k_upd2(GeoK g, BPArgs A, const float* __restrict__ Gb) {
    constexpr int NV = T::X * T::Y;
    constexpr int HX = T::X + 2, HY = T::Y + 2;
    constexpr int BW = T::X + 2 * PSF_KMAX, BH = T::Y + 2 * PSF_KMAX;
    __shared__ float s_f[HX * HY];
    __shared__ float s_b[BLUR ? BW * BH : 1];
    __shared__ float s_bx[BLUR ? BH * T::X : 1];
    __shared__ double s_red[NT / 64];
    const int vblock = blockIdx.x;
    const int tiles_x = (g.nx + T::X - 1) / T::X;
    const int tx0 = (vblock % tiles_x) * T::X;
    const int ty0 = (vblock / tiles_x) * T::Y;
    const int vox = threadIdx.x % NV, grp = threadIdx.x / NV;
    const int lx = vox % T::X, ly = vox / T::X;
    const int ix = tx0 + lx, iy = ty0 + ly;
    const bool inside = ix < g.nx && iy < g.ny;
    const PixPre pre = pixel_prefetch(A, inside && grp == 0, (long long)iy * g.nx + ix);
    for (int e = threadIdx.x; e < HX * HY; e += NT) {
        const int hx = e % HX, hy = e / HX;
        const int gx = tx0 - 1 + hx, gy = ty0 - 1 + hy;
        s_f[e] = (gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny) ? A.f[(long long)gy * g.nx + gx] : 0.0f;
    }
    const int Kx = g.psf_kx, Ky = g.psf_ky;
    if (BLUR) {
        // the tile of A_i^T w with a PSF-radius halo (zero outside the image),
        // then the pass along x, as k_blur2 does
        const int W = T::X + 2 * Kx, H = T::Y + 2 * Ky;
        for (int e = threadIdx.x; e < W * H; e += NT) {
            const int hx = e % W, hy = e / W;
            const int x = tx0 - Kx + hx, y = ty0 - Ky + hy;
            s_b[e] = (x >= 0 && x < g.nx && y >= 0 && y < g.ny) ? Gb[(long long)y * g.nx + x] : 0.0f;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < T::X * H; e += NT) {
            const int bx = e % T::X, hy = e / T::X;
            float acc = 0.0f;
            for (int k = 0; k <= 2 * Kx; ++k) acc = fmaf(g.psf[k], s_b[hy * W + bx + k], acc);
            s_bx[hy * T::X + bx] = acc;
        }
    }
    float meanf = 1.0f;
    if (A.want_mu) meanf = (float)(sum_partials(A.part_f, A.n_part_f, s_red) / (double)g.nvox);
    float meanmu = 1.0f;
    if (A.fnew != nullptr && (A.nu_mode == NU_COMPUTE || A.nu_mode == NU_COMPUTE_FREEZE))
        meanmu = (float)(sum_partials(A.part_mu, A.n_part_mu, s_red) / (double)g.nvox);
    __syncthreads();
    double part = 0.0;
    if (inside && grp == 0) {
        float b;
        if (BLUR) {
            const float* wy = g.psf + 2 * Kx + 1;
            b = 0.0f;
            for (int k = 0; k <= 2 * Ky; ++k) b = fmaf(wy[k], s_bx[(ly + k) * T::X + lx], b);
        } else {
            b = Gb[(long long)iy * g.nx + ix];
        }
        part = pixel_finish(g, A, s_f, HX, HY, lx, ly, ix, iy, b, meanf, meanmu, pre);
    }
    if (A.fnew != nullptr) write_partial(part, A.red_f, s_red, vblock);
    else if (A.want_mu) write_partial(part, A.red_mu, s_red, vblock);
}

// ------------------------------------------------------------------ update

// Matlab-style gradient magnitude (unit spacing, central differences
// inside, one-sided at the edges) of a 2D image at pixel (ix, iy)
__device__ __forceinline__ float gmag2(const float* f, const GeoK& g, int ix, int iy, float fj) {
    const long long j = (long long)iy * g.nx + ix;
    float gx = 0.0f, gy = 0.0f;
    if (g.nx > 1) {
        if (ix == 0) gx = f[j + 1] - fj;
        else if (ix == g.nx - 1) gx = fj - f[j - 1];
        else gx = 0.5f * (f[j + 1] - f[j - 1]);
    }
    if (g.ny > 1) {
        if (iy == 0) gy = f[j + g.nx] - fj;
        else if (iy == g.ny - 1) gy = fj - f[j - g.nx];
        else gy = 0.5f * (f[j + g.nx] - f[j - g.nx]);
    }
    return sqrtf(gx * gx + gy * gy);
}

constexpr int PX_PER_BLOCK = 256;    // pixels per block of the 2D pixel pass
constexpr int PX_ITEM = 4;           // pixel blocks per batched work item

int px_grid(const pet_os_geom* G) { return (int)((G->n_vox + PX_PER_BLOCK - 1) / PX_PER_BLOCK); }
int px_items(const pet_os_geom* G) { return (px_grid(G) + PX_ITEM - 1) / PX_ITEM; }

struct PxArgs {
    const float* f;          // iterate entering the subiteration
    float* fsnap;            // its copy, read by the fused back-projection/update
    float* mu;
    int want_mu;
    const double* part_f;    // partials of sum f
    int n_part_f;
    Reduction red_mu;        // partials of sum mu, one per pixel block
};

// Pixel part of the first kernel of a 2D subiteration, PX_PER_BLOCK pixels
// per block: the snapshot of f and, when nu of eq:nuki is recomputed,
// mu = max(0.01, |grad f| / mean f) of Sec. III-B with its FP64 partial sums.
__device__ void px_body(const GeoK& g, const PxArgs& P, long long pblock) {
    __shared__ double s_red[NT / 64];
    constexpr int K = PX_PER_BLOCK / NT;
    float fv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const long long j = pblock * PX_PER_BLOCK + k * NT + threadIdx.x;
        fv[k] = j < g.nvox ? P.f[j] : 0.0f;
        if (j < g.nvox) P.fsnap[j] = fv[k];
    }
    if (!P.want_mu) return;
    const float meanf = (float)(sum_partials(P.part_f, P.n_part_f, s_red) / (double)g.nvox);
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const long long j = pblock * PX_PER_BLOCK + k * NT + threadIdx.x;
        if (j < g.nvox) {
            // (an image holds at most 2^30 pixels: 32-bit division)
            const int j32 = (int)j, iy = j32 / g.nx;
            const float mu = fmaxf(0.01f, gmag2(P.f, g, j32 - iy * g.nx, iy, fv[k]) / meanf);
            P.mu[j] = mu;
            part += (double)mu;
        }
    }
    write_partial(part, P.red_mu, s_red, pblock);
}

// First kernel of a 2D subiteration: blocks [0, n_fp) project the subset and
// form the Poisson ratio, the rest run the pixel pass.
template <int SEG, bool SUB>
__global__ __launch_bounds__(NT) void k_fp_px(GeoK g, FPArgs A, PxArgs P, int n_fp) {
    if ((int)blockIdx.x < n_fp) fp_body<2, SEG, SUB>(g, A, blockIdx.x);
    else px_body(g, P, (long long)blockIdx.x - n_fp);
}

__device__ void sum_body(const float* x, long long n, Reduction R, long long vblock) {
    __shared__ double s_red[NT / 64];
    const long long j = vblock * NT + threadIdx.x;
    write_partial(j < n ? (double)x[j] : 0.0, R, s_red, vblock);
}

__global__ __launch_bounds__(NT) void k_sum(const float* x, long long n, Reduction R) {
    sum_body(x, n, R, blockIdx.x);
}

__global__ __launch_bounds__(NT) void k_fill(float* x, long long n, float v) {
    const long long j = (long long)blockIdx.x * NT + threadIdx.x;
    if (j < n) x[j] = v;
}

// R(f) of eq:RDP, FP64 per voxel and per block
template <int DIM>
__global__ __launch_bounds__(NT) void k_rdp(GeoK g, const float* f, float gR, float eps, Reduction R) {
    __shared__ double s_red[NT / 64];
    const long long j = (long long)blockIdx.x * NT + threadIdx.x;
    double v = 0.0;
    if (j < g.nvox) {
        const int ix = (int)(j % g.nx), iy = (int)((j / g.nx) % g.ny), iz = (int)(j / ((long long)g.nx * g.ny));
        const double fj = f[j];
        const int zr = (DIM == 3) ? 1 : 0;
        for (int dz = -zr; dz <= zr; ++dz) {
            const int z = iz + dz;
            if (z < 0 || z >= (DIM == 3 ? g.nz : 1)) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                const int y = iy + dy;
                if (y < 0 || y >= g.ny) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    const int x = ix + dx;
                    if ((dx | dy | dz) == 0 || x < 0 || x >= g.nx) continue;
                    const double fk = f[((long long)z * g.ny + y) * g.nx + x];
                    const double d = fj - fk;
                    v += d * d / (fj + fk + (double)gR * fabs(d) + (double)eps);
                }
            }
        }
    }
    write_partial(v, R, s_red, blockIdx.x);
}

// ------------------------------------------------------------------ launchers

// threads per ray: enough rays x segments to fill the chip (~2^18 threads)
static int fp_seg_heuristic(long long nrays) {
    const long long target = 1LL << 18;
    if (nrays * 4 > target) return nrays >= target ? 1 : 4;
    if (nrays * 16 > target) return 16;
    return 64;
}

int fp_seg_for(const pet_os_geom* G, long long nrays, int requested) {
    if (requested > 0) return requested;
    (void)G;
    return fp_seg_heuristic(nrays);
}

int fp_grid_seg(const pet_os_geom* G, int n_al, int seg) {
    long long nrays = (long long)n_al * G->n_planes * G->d.n_radial;
    int rpb = NT / seg;
    return (int)((nrays + rpb - 1) / rpb);
}

int fp_grid(const pet_os_geom* G, int n_al) {
    if (G->d.dim == 3) return fp3_launch_grid(G, n_al);
    long long nrays = (long long)n_al * G->n_planes * G->d.n_radial;
    return fp_grid_seg(G, n_al, fp_seg_heuristic(nrays));
}

// 2D tile kinds 0: 16x16, 1: 8x8 with four angle groups; 3D geometries use
// kind 2, the column tiles of k_bp3
int bp_kind_default(const pet_os_geom* G) {
    if (G->d.dim == 3) return 2;
    long long tiles16 = (long long)((G->d.nx + 15) / 16) * ((G->d.ny + 15) / 16);
    return tiles16 < 1024 ? 1 : 0;
}

int bp_kind_of(const pet_os_geom* G) {
    if (G->d.dim == 2 && G->tuned_bp_kind >= 0) return G->tuned_bp_kind;
    return bp_kind_default(G);
}

int bp_grid_kind(const pet_os_geom* G, int kind) {
    if (kind == 2) return bp3_grid(G);
    const int T = kind == 0 ? 16 : 8;
    return ((G->d.nx + T - 1) / T) * ((G->d.ny + T - 1) / T);
}

int bp_grid(const pet_os_geom* G) { return bp_grid_kind(G, bp_kind_of(G)); }

int bp_grid_max(const pet_os_geom* G) {
    if (G->d.dim == 3) return bp3_grid_zb(G, 16);   // the most blocks any 3D shape launches
    return std::max(bp_grid_kind(G, 0), bp_grid_kind(G, 1));
}

int elem_grid(int64_t n) { return (int)((n + NT - 1) / NT); }

// the update leaves one partial of sum f per 3D update tile, or per 2D
// back-projection tile (the 2D update is fused into the back-projection)
int sumf_grid(const pet_os_geom* G) { return G->d.dim == 3 ? upd3_grid(G) : bp_grid(G); }

// partials of sum f of an image given by the caller, over the same blocks and
// in the same order as the update leaves them (3D: also its z-fastest copy)
int launch_sum_f(const pet_os_geom* G, const float* f, float* fz, Reduction red, hipStream_t s) {
    if (G->d.dim == 3) return launch_prep3(G, f, fz, red, s);
    const int grid = bp_grid(G);
    if (grid > red.cap) return fail(PET_OS_ERR_DEVICE, "sum partials too small");
    if (bp_kind_of(G) == 0) hipLaunchKernelGGL((k_sum_tiles<Tile2L>), dim3(grid), dim3(NT), 0, s, G->k, f, red);
    else hipLaunchKernelGGL((k_sum_tiles<Tile2S>), dim3(grid), dim3(NT), 0, s, G->k, f, red);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

template <int SEG, bool SUB>
static void fp_launch_t(const GeoK& k, const FPArgs& a, int grid, hipStream_t s) {
    petos_launch(k_fp<2, SEG, SUB>, dim3(grid), dim3(NT), 0, s, k, a);
}

template <bool SUB>
static void fp_launch_seg(int seg, const GeoK& k, const FPArgs& a, int grid, hipStream_t s) {
    if (seg == 64) fp_launch_t<64, SUB>(k, a, grid, s);
    else if (seg == 16) fp_launch_t<16, SUB>(k, a, grid, s);
    else if (seg == 4) fp_launch_t<4, SUB>(k, a, grid, s);
    else fp_launch_t<1, SUB>(k, a, grid, s);
}

template <bool SUB>
static void fp_px_launch_seg(int seg, dim3 blocks, const GeoK& k, const FPArgs& a, const PxArgs& P, int grid,
                             hipStream_t s) {
    if (seg == 64) petos_launch(k_fp_px<64, SUB>, blocks, dim3(NT), 0, s, k, a, P, grid);
    else if (seg == 16) petos_launch(k_fp_px<16, SUB>, blocks, dim3(NT), 0, s, k, a, P, grid);
    else if (seg == 4) petos_launch(k_fp_px<4, SUB>, blocks, dim3(NT), 0, s, k, a, P, grid);
    else petos_launch(k_fp_px<1, SUB>, blocks, dim3(NT), 0, s, k, a, P, grid);
}

int launch_fp(const pet_os_geom* G, const FPLaunch& L, hipStream_t s) {
    if (G->d.dim == 3) return launch_fp3(G, L, s);
    FPArgs a;
    a.f = L.f;
    a.y = L.y;
    a.r = L.r;
    a.out = L.out;
    a.angles = L.angles;
    a.n_al = L.n_al;
    a.mode = L.mode;
    a.red = L.red;
    a.att = L.raw ? nullptr : G->k.att;
    const bool sub = G->k.n_sub > 1;
    long long nrays = (long long)L.n_al * G->n_planes * G->d.n_radial;
    if (nrays == 0) return PET_OS_OK;
    int seg = fp_seg_for(G, nrays, L.seg);
    int grid = fp_grid_seg(G, L.n_al, seg);
    if (L.mode == FP_OBJECTIVE && grid > L.red.cap) return fail(PET_OS_ERR_DEVICE, "objective partials too small");
    if (L.px_fsnap != nullptr) {
        // 2D subiteration: the pixel pass rides in the same launch
        PxArgs P;
        P.f = L.px_f != nullptr ? L.px_f : L.f;
        P.fsnap = L.px_fsnap;
        P.mu = L.px_mu;
        P.want_mu = L.px_want_mu;
        P.part_f = L.px_part_f;
        P.n_part_f = L.px_n_part_f;
        P.red_mu = L.px_red_mu;
        const int npx = px_grid(G);
        if (P.want_mu && npx > P.red_mu.cap) return fail(PET_OS_ERR_DEVICE, "mu partials too small");
        const dim3 blocks(grid + npx);
        if (sub) fp_px_launch_seg<true>(seg, blocks, G->k, a, P, grid, s);
        else fp_px_launch_seg<false>(seg, blocks, G->k, a, P, grid, s);
        PETOS_HIP(hipGetLastError());
        return PET_OS_OK;
    }
    if (sub) fp_launch_seg<true>(seg, G->k, a, grid, s);
    else fp_launch_seg<false>(seg, G->k, a, grid, s);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

size_t bp_lds_budget(int kind) {
    (void)kind;
    return 4096 * sizeof(float);
}

// LDS footprint bounds of a 2D back-projection tile (host side, conservative)
void bp_stage_shape_kind(const pet_os_geom* G, int kind, int& nb_max, int& rows_max, int& chunk, size_t& lds) {
    const auto& d = G->d;
    const int T = kind == 0 ? 16 : 8;
    nb_max = (int)std::ceil(T * (d.vx + d.vy) / d.ds) + 4;
    if (nb_max > d.n_radial) nb_max = d.n_radial;
    rows_max = 1;
    const size_t budget_floats = bp_lds_budget(kind) / sizeof(float);
    chunk = (int)std::max<size_t>(1, budget_floats / (size_t)nb_max);
    if (chunk > MAXCH) chunk = MAXCH;
    lds = (size_t)chunk * nb_max * sizeof(float);
}

static void fill_bp_args(const pet_os_geom* G, const BPLaunch& L, BPArgs& a) {
    a.w = L.w;
    a.w_natural = L.w_natural;
    if (L.w_natural) {
        a.w_sa = G->d.n_radial;
        a.w_sp = (long long)G->d.n_angles * G->d.n_radial;
    } else {
        a.w_sp = G->d.n_radial;
        a.w_sa = (long long)G->n_planes * G->d.n_radial;
    }
    a.angles = L.angles;
    a.n_al = L.n_al;
    a.out = L.out;
    a.f = L.f;
    a.mu = L.mu;
    a.want_mu = L.want_mu;
    a.beta_over_M = L.beta_over_M;
    a.gamma_R = L.gamma_R;
    a.eps = L.eps;
    a.part_f = L.part_f;
    a.n_part_f = L.n_part_f;
    a.red_mu = L.red_mu;
    a.fnew = L.fnew;
    a.pnorm = L.pnorm;
    a.nu_frozen = L.nu_frozen;
    a.nu_mode = L.nu_mode;
    a.step = L.step;
    a.nu1 = L.nu1;
    a.nu2 = L.nu2;
    a.box = L.box;
    a.part_mu = L.part_mu;
    a.n_part_mu = L.n_part_mu;
    a.red_f = L.red_f;
    a.osem_sens = L.osem_sens;
    // compact subset weights already carry the attenuation (forward epilogue)
    a.att = (L.w == nullptr || L.w_natural) ? G->k.att : nullptr;
}

int launch_bp(const pet_os_geom* G, const BPLaunch& L, hipStream_t s) {
    if (G->d.dim == 3) return launch_bp3(G, L, s);
    BPArgs a{};
    fill_bp_args(G, L, a);
    size_t lds;
    int rows_unused;
    const int kind = bp_kind_of(G);
    bp_stage_shape_kind(G, kind, a.nb_max, rows_unused, a.chunk, lds);
    if (L.w == nullptr) lds = 0;
    int grid = bp_grid(G);
    if (L.want_mu && grid > L.red_mu.cap) return fail(PET_OS_ERR_DEVICE, "mu partials too small");
    if (L.fnew != nullptr && grid > L.red_f.cap) return fail(PET_OS_ERR_DEVICE, "sum partials too small");
    // the sub-ray gather and the attenuation of user or unit weights are
    // compiled only into the kernels that need them
    const bool sub = G->k.n_sub > 1, att = a.att != nullptr;
    const dim3 gr(grid), bl(NT);
    if (kind == 0) {
        if (sub && att) petos_launch(k_bp<Tile2L, true, true>, gr, bl, lds, s, G->k, a);
        else if (sub) petos_launch(k_bp<Tile2L, true, false>, gr, bl, lds, s, G->k, a);
        else if (att) petos_launch(k_bp<Tile2L, false, true>, gr, bl, lds, s, G->k, a);
        else petos_launch(k_bp<Tile2L, false, false>, gr, bl, lds, s, G->k, a);
    } else {
        if (sub && att) petos_launch(k_bp<Tile2S, true, true>, gr, bl, lds, s, G->k, a);
        else if (sub) petos_launch(k_bp<Tile2S, true, false>, gr, bl, lds, s, G->k, a);
        else if (att) petos_launch(k_bp<Tile2S, false, true>, gr, bl, lds, s, G->k, a);
        else petos_launch(k_bp<Tile2S, false, false>, gr, bl, lds, s, G->k, a);
    }
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

int launch_blur(const pet_os_geom* G, const float* in, float* out, hipStream_t s) {
    if (G->d.dim != 2 || G->k.psf_kx <= 0 || G->k.psf_ky <= 0) return fail(PET_OS_ERR_DEVICE, "no 2D PSF");
    if (G->k.psf_kx > PSF_KMAX || G->k.psf_ky > PSF_KMAX) return fail(PET_OS_ERR_DEVICE, "PSF radius too large");
    const int grid = ((G->d.nx + BLT - 1) / BLT) * ((G->d.ny + BLT - 1) / BLT);
    hipLaunchKernelGGL(k_blur2, dim3(grid), dim3(NT), 0, s, G->k, in, out);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

int launch_upd2(const pet_os_geom* G, const BPLaunch& L, const float* Gb, bool blur, hipStream_t s) {
    if (G->d.dim != 2) return fail(PET_OS_ERR_DEVICE, "2D only");
    if (L.f == nullptr) return fail(PET_OS_ERR_DEVICE, "update without the snapshot");
    BPArgs a{};
    fill_bp_args(G, L, a);
    const int grid = bp_grid(G);
    if (L.want_mu && grid > L.red_mu.cap) return fail(PET_OS_ERR_DEVICE, "mu partials too small");
    if (L.fnew != nullptr && grid > L.red_f.cap) return fail(PET_OS_ERR_DEVICE, "sum partials too small");
    if (blur && (G->k.psf_kx <= 0 || G->k.psf_kx > PSF_KMAX || G->k.psf_ky > PSF_KMAX))
        return fail(PET_OS_ERR_DEVICE, "no 2D PSF");
    const bool large = bp_kind_of(G) == 0;
    if (large && blur) hipLaunchKernelGGL((k_upd2<Tile2L, true>), dim3(grid), dim3(NT), 0, s, G->k, a, Gb);
    else if (large) hipLaunchKernelGGL((k_upd2<Tile2L, false>), dim3(grid), dim3(NT), 0, s, G->k, a, Gb);
    else if (blur) hipLaunchKernelGGL((k_upd2<Tile2S, true>), dim3(grid), dim3(NT), 0, s, G->k, a, Gb);
    else hipLaunchKernelGGL((k_upd2<Tile2S, false>), dim3(grid), dim3(NT), 0, s, G->k, a, Gb);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

// ------------------------------------------------------------------ data check
// The data of the problem statement (Sec. II-A): counts g >= 0, background
// gamma > 0 elementwise, and an initial image in the box B of eq:BoundedSet,
// every value finite.  Each block counts the entries that break a rule
// ([0] y, [1] r, [2] f) and the positive entries of f ([3]) over a
// grid-stride range; k_check_total adds the block counts in block order.
// f_lim is the smallest float above U (f <= U exactly when f < f_lim).
__global__ __launch_bounds__(NT) void k_check_data(const float* __restrict__ y, const float* __restrict__ r,
                                                   long long nb, const float* __restrict__ f, long long nv,
                                                   float f_lim, unsigned* __restrict__ part) {
    __shared__ unsigned s_c[4];
    if (threadIdx.x < 4) s_c[threadIdx.x] = 0u;
    __syncthreads();
    unsigned c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    const long long stride = (long long)gridDim.x * NT;
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < nb; i += stride) {
        const float yv = y[i], rv = r[i];
        c0 += (yv >= 0.0f && yv <= FLT_MAX) ? 0u : 1u;     // false for NaN
        c1 += (rv > 0.0f && rv <= FLT_MAX) ? 0u : 1u;
    }
    for (long long j = (long long)blockIdx.x * NT + threadIdx.x; j < nv; j += stride) {
        const float fv = f[j];
        c2 += (fv >= 0.0f && fv < f_lim && fv <= FLT_MAX) ? 0u : 1u;
        c3 += (fv > 0.0f) ? 1u : 0u;
    }
    atomicAdd(&s_c[0], c0);
    atomicAdd(&s_c[1], c1);
    atomicAdd(&s_c[2], c2);
    atomicAdd(&s_c[3], c3);
    __syncthreads();
    if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = s_c[threadIdx.x];
}

__global__ __launch_bounds__(NT) void k_check_total(const unsigned* __restrict__ part, int n_blocks,
                                                    unsigned long long* __restrict__ total) {
    __shared__ unsigned long long s_t[4];
    if (threadIdx.x < 4) s_t[threadIdx.x] = 0ull;
    __syncthreads();
    unsigned long long t[4] = {0ull, 0ull, 0ull, 0ull};
    for (int b = threadIdx.x; b < n_blocks; b += NT)
        for (int k = 0; k < 4; ++k) t[k] += part[b * 4 + k];
    for (int k = 0; k < 4; ++k) atomicAdd(&s_t[k], t[k]);
    __syncthreads();
    if (threadIdx.x < 4) total[threadIdx.x] = s_t[threadIdx.x];
}

int launch_check_data(const float* y, const float* r, int64_t nb, const float* f, int64_t nv, float f_lim,
                      unsigned* part, unsigned long long* total, hipStream_t s) {
    const int64_t n = std::max(nb, nv);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(CHECK_GRID, (n + NT - 1) / NT));
    hipLaunchKernelGGL(k_check_data, dim3(grid), dim3(NT), 0, s, y, r, (long long)nb, f, (long long)nv, f_lim,
                       part);
    hipLaunchKernelGGL(k_check_total, dim3(1), dim3(NT), 0, s, (const unsigned*)part, grid, total);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

__global__ __launch_bounds__(NT) void k_expneg(const float* __restrict__ x, float* __restrict__ y, long long n) {
    const long long j = (long long)blockIdx.x * NT + threadIdx.x;
    if (j < n) y[j] = expf(-x[j]);
}

int launch_expneg(const float* x, float* y, int64_t n, hipStream_t s) {
    if (n <= 0) return PET_OS_OK;
    hipLaunchKernelGGL(k_expneg, dim3(elem_grid(n)), dim3(NT), 0, s, x, y, (long long)n);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

// the separate update kernel serves 3D geometries; in 2D it is fused into
// the back-projection (BPLaunch::fnew)
int launch_update(const pet_os_geom* G, const UpdLaunch& L, hipStream_t s) {
    if (G->d.dim == 3) return launch_update3(G, L, s);
    return fail(PET_OS_ERR_DEVICE, "2D update is fused into the back-projection");
}

int launch_sum(const float* x, int64_t n, Reduction red, hipStream_t s) {
    int grid = elem_grid(n);
    if (grid > red.cap) return fail(PET_OS_ERR_DEVICE, "sum partials too small");
    hipLaunchKernelGGL(k_sum, dim3(grid), dim3(NT), 0, s, x, (long long)n, red);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

int launch_finalize(Reduction red, int n, hipStream_t s) {
    if (n > red.cap) return fail(PET_OS_ERR_DEVICE, "finalize beyond partial capacity");
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(NT), 0, s, red, n);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

int launch_fill(float* x, int64_t n, float v, hipStream_t s) {
    if (n == 0) return PET_OS_OK;
    hipLaunchKernelGGL(k_fill, dim3(elem_grid(n)), dim3(NT), 0, s, x, (long long)n, v);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

int launch_rdp_value(const pet_os_geom* G, const float* f, float gamma_R, float eps, Reduction red,
                     hipStream_t s) {
    int grid = elem_grid(G->n_vox);
    if (grid > red.cap) return fail(PET_OS_ERR_DEVICE, "rdp partials too small");
    if (G->d.dim == 3)
        hipLaunchKernelGGL((k_rdp<3>), dim3(grid), dim3(NT), 0, s, G->k, f, gamma_R, eps, red);
    else
        hipLaunchKernelGGL((k_rdp<2>), dim3(grid), dim3(NT), 0, s, G->k, f, gamma_R, eps, red);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

// ------------------------------------------------------------------ batched (persistent) kernels
// Every block walks a device-resident work list of (slot, block) items with a
// grid stride; the lists, their lengths and the slot table live in device
// memory, so one captured graph stays valid while requests come and go.

__device__ __forceinline__ bool slot_live(const SlotDev& d) { return d.active && d.J <= d.J_end; }

__device__ void fp_dispatch(const GeoK& g, const FPArgs& A, int seg, long long vblock) {
    switch (seg) {
        case 64: fp_body<2, 64>(g, A, vblock); break;
        case 16: fp_body<2, 16>(g, A, vblock); break;
        case 4: fp_body<2, 4>(g, A, vblock); break;
        default: fp_body<2, 1>(g, A, vblock); break;
    }
}

__global__ __launch_bounds__(NT) void k_fp_batch(const SlotDev* __restrict__ S, const Item* __restrict__ items, const int* __restrict__ count) {
    const int n = *count;
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const Item I = items[it];
        const SlotDev& d = S[I.slot];
        if (!slot_live(d)) continue;
        const int i = (d.J - 1) % d.g.n_subsets;
        if (I.block >= d.n_fp) {
            // pixel pass: snapshot of f and mu, PX_ITEM pixel blocks per item
            const int nu_mode = d.sched_nu[d.J - 1];
            PxArgs P;
            P.f = d.f;
            P.fsnap = d.fsnap;
            P.mu = d.mu;
            P.want_mu = (nu_mode == NU_COMPUTE || nu_mode == NU_COMPUTE_FREEZE) ? 1 : 0;
            P.part_f = d.part_f;
            P.n_part_f = d.n_part_f;
            P.red_mu.part = d.part_mu;
            P.red_mu.total = nullptr;
            P.red_mu.cap = d.n_part_mu;
            const int pb0 = (I.block - d.n_fp) * PX_ITEM;
            for (int pb = pb0; pb < min(pb0 + PX_ITEM, d.n_part_mu); ++pb) {
                px_body(d.g, P, pb);
                __syncthreads();
            }
        } else {
            FPArgs A{};
            A.f = d.f;
            A.y = d.y;
            A.r = d.r;
            A.out = d.w;
            A.angles = d.subset_lists + (long long)i * d.max_sub;
            A.n_al = d.subset_count[i];
            A.mode = FP_RATIO;
            fp_dispatch(d.g, A, d.fp_seg, I.block);
        }
        __syncthreads();
    }
}

// at most 96 VGPRs (5 waves per SIMD): the gather's per-angle tile
// references need more than 72 without spilling to scratch (6 waves: 80
// VGPRs and 7 spilled; 5 waves measured 1 % faster, with no scratch traffic)
template <class T>
__global__ __launch_bounds__(NT, 5) void k_bp_batch(const SlotDev* __restrict__ S, const Item* __restrict__ items, const int* __restrict__ count) {
    const int n = *count;
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const Item I = items[it];
        const SlotDev& d = S[I.slot];
        if (!slot_live(d)) continue;
        const int i = (d.J - 1) % d.g.n_subsets;
        const int nu_mode = d.sched_nu[d.J - 1];
        BPArgs A{};
        A.w = d.w;
        A.w_natural = 0;
        A.w_sp = d.g.n_radial;
        A.w_sa = (long long)d.g.n_planes * d.g.n_radial;
        A.angles = d.subset_lists + (long long)i * d.max_sub;
        A.n_al = d.subset_count[i];
        A.out = nullptr;
        A.f = d.fsnap;
        A.mu = d.mu;
        A.want_mu = 0;
        A.beta_over_M = d.beta_over_M;
        A.gamma_R = d.gamma_R;
        A.eps = d.eps;
        A.nb_max = d.nb_max;
        A.chunk = d.chunk;
        A.fnew = d.f;
        A.pnorm = d.pnorm;
        A.nu_frozen = d.nu_frozen;
        A.nu_mode = nu_mode;
        A.step = d.sched_step[d.J - 1];
        A.nu1 = d.nu1;
        A.nu2 = d.nu2;
        A.box = d.box;
        A.part_mu = d.part_mu;
        A.n_part_mu = d.n_part_mu;
        A.red_f.part = d.part_f;
        A.red_f.total = nullptr;
        A.red_f.cap = d.n_part_f;
        bp_body<T, false, false, true>(d.g, A, I.block);
        __syncthreads();
    }
}

// J += 1 for every live slot (one thread per slot, after the update)
__global__ __launch_bounds__(NT) void k_advance(SlotDev* S, int n_slots) {
    const int sidx = blockIdx.x * NT + threadIdx.x;
    if (sidx < n_slots && S[sidx].active && S[sidx].J <= S[sidx].J_end) S[sidx].J += 1;
}

int launch_batch_step(SlotDev* d_slots, int n_slots, Item* const lists[WL_COUNT], const int* d_counts,
                      const int grids[WL_COUNT], int live_mask, hipStream_t s) {
    auto live = [&](int k) { return (live_mask >> k) & 1; };
    if (live(WL_FP))
        hipLaunchKernelGGL(k_fp_batch, dim3(grids[WL_FP]), dim3(NT), 0, s, d_slots, lists[WL_FP], d_counts + WL_FP);
    if (live(WL_FP3)) launch_batch3_fp(d_slots, lists[WL_FP3], d_counts + WL_FP3, grids[WL_FP3], s);
    if (live(WL_BP0))
        hipLaunchKernelGGL((k_bp_batch<Tile2L>), dim3(grids[WL_BP0]), dim3(NT), bp_lds_budget(0), s, d_slots,
                           lists[WL_BP0], d_counts + WL_BP0);
    if (live(WL_BP1))
        hipLaunchKernelGGL((k_bp_batch<Tile2S>), dim3(grids[WL_BP1]), dim3(NT), bp_lds_budget(1), s, d_slots,
                           lists[WL_BP1], d_counts + WL_BP1);
    const int zbs[3] = {16, 32, 64};
    for (int k = 0; k < 6; ++k)
        if (live(WL_BP3 + k))
            launch_batch3_bp(d_slots, lists[WL_BP3 + k], d_counts + WL_BP3 + k, grids[WL_BP3 + k], zbs[k / 2],
                             (k & 1) ? 40 : 20, s);
    if (live(WL_PEN3)) launch_batch3_pen(d_slots, lists[WL_PEN3], d_counts + WL_PEN3, grids[WL_PEN3], s);
    if (live(WL_UPD3)) launch_batch3_upd(d_slots, lists[WL_UPD3], d_counts + WL_UPD3, grids[WL_UPD3], s);
    hipLaunchKernelGGL(k_advance, dim3((n_slots + NT - 1) / NT), dim3(NT), 0, s, d_slots, n_slots);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

}  // namespace petos
