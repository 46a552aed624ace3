// capi.cpp -- C ABI of the pet_os library: geometry tables, per-request state,
// the plain subiteration / reconstruct drivers, objective, checkpoints.
//
// Host side of SDP-BSREM (Table I): the FP64 scalar schedule (lambda_k of
// thm:SpecificSDPs, alpha_{k,i} of preconditioner:Nesterov / preconditioner:KM,
// the J-mode of eq:nuki) is evaluated here and handed to the kernels; every
// per-voxel and per-bin step runs on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "internal.h"

namespace petos {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

thread_local LaunchEvents g_launch_events;

int fail(int code, const std::string& msg) {
    set_error(msg);
    return code;
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// ---------------------------------------------------------------- geometry validation

int validate_desc(const pet_os_geom_desc* d) {
    if (!d) return fail(PET_OS_ERR_INVALID_ARG, "desc is NULL");
    if (d->dim != 2 && d->dim != 3) return fail(PET_OS_ERR_INVALID_ARG, "dim must be 2 or 3");
    if (d->nx < 1 || d->ny < 1) return fail(PET_OS_ERR_INVALID_ARG, "nx, ny must be >= 1");
    // the projectors form pixel offsets with 24-bit multiplies
    if (d->nx >= (1 << 23) || d->ny >= (1 << 23)) return fail(PET_OS_ERR_INVALID_ARG, "nx, ny must be below 2^23");
    if (!finite_pos(d->vx) || !finite_pos(d->vy) || !finite_pos(d->ds))
        return fail(PET_OS_ERR_INVALID_ARG, "vx, vy, ds must be finite and > 0");
    if (d->n_angles < 1 || d->n_radial < 1) return fail(PET_OS_ERR_INVALID_ARG, "n_angles, n_radial must be >= 1");
    if (d->n_subsets < 1 || d->n_subsets > d->n_angles)
        return fail(PET_OS_ERR_INVALID_ARG, "n_subsets must be in [1, n_angles]");
    if ((int64_t)d->nx * d->ny * (d->dim == 3 ? d->nz : 1) > (int64_t)1 << 30)
        return fail(PET_OS_ERR_INVALID_ARG, "image too large");
    if (d->n_subrays < 0 || d->n_subrays > 64) return fail(PET_OS_ERR_INVALID_ARG, "n_subrays must be in [0, 64]");
    // the projectors index one pass (all angles at most) in 32-bit integers:
    // 2D rays, and 3D forward work items (angle, bin, ring difference, ring chunk)
    {
        const int64_t D = d->dim == 3 ? std::max(0, d->max_ring_diff) : 0;
        const int64_t chunks = d->dim == 3 ? (std::max(1, d->n_rings) + 63) / 64 : 1;
        const int64_t per_pass = (int64_t)d->n_angles * d->n_radial * (2 * D + 1) * chunks;
        if (per_pass >= ((int64_t)1 << 31)) return fail(PET_OS_ERR_INVALID_ARG, "sinogram too large");
    }
    if (!(std::isfinite(d->psf_fwhm) && d->psf_fwhm >= 0.0))
        return fail(PET_OS_ERR_INVALID_ARG, "psf_fwhm must be finite and >= 0");
    if (d->dim == 3 && (d->n_subrays > 1 || d->psf_fwhm > 0.0))
        return fail(PET_OS_ERR_INVALID_ARG, "sub-rays and the PSF are 2D only");
    if (d->psf_fwhm > 0.0) {
        const double sigma = d->psf_fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
        if (std::ceil(3.0 * sigma / d->vx) > PSF_KMAX || std::ceil(3.0 * sigma / d->vy) > PSF_KMAX)
            return fail(PET_OS_ERR_INVALID_ARG, "PSF wider than 16 pixels (3 sigma)");
    }
    if (d->dim == 3) {
        if (d->nz < 1 || !finite_pos(d->vz)) return fail(PET_OS_ERR_INVALID_ARG, "nz >= 1 and vz > 0 required");
        if (d->n_rings != d->nz || d->ring_pitch != d->vz)
            return fail(PET_OS_ERR_INVALID_ARG, "rings must sit at slice centres: n_rings == nz, ring_pitch == vz");
        if (d->max_ring_diff < 0 || d->max_ring_diff > std::min(d->nz - 1, 31))
            return fail(PET_OS_ERR_INVALID_ARG, "max_ring_diff must be in [0, min(nz-1, 31)]");
        // the forward projector forms voxel offsets with 24-bit multiplies
        if ((int64_t)std::max(d->nx, d->ny) * d->nz >= ((int64_t)1 << 23))
            return fail(PET_OS_ERR_INVALID_ARG, "3D: nx*nz and ny*nz must be below 2^23");
        double half_diag = 0.5 * std::sqrt((double)d->nx * d->nx * d->vx * d->vx + (double)d->ny * d->ny * d->vy * d->vy);
        double smax = 0.5 * (d->n_radial - 1) * d->ds;
        if (!finite_pos(d->det_radius) || d->det_radius <= half_diag || d->det_radius <= smax)
            return fail(PET_OS_ERR_INVALID_ARG, "det_radius must exceed the image half-diagonal and the largest |s_b|");
        double hmin = std::sqrt(d->det_radius * d->det_radius - smax * smax);
        double step = std::sqrt(d->vx * d->vx + d->vy * d->vy);
        if (d->max_ring_diff * step / (2.0 * hmin) >= 1.0)
            return fail(PET_OS_ERR_INVALID_ARG, "LORs too oblique: more than one slice per transaxial voxel");
    }
    return PET_OS_OK;
}

static int n_planes_of(const pet_os_geom_desc* d) {
    if (d->dim == 2) return 1;
    int n = d->n_rings;
    for (int k = 1; k <= d->max_ring_diff; ++k) n += 2 * (d->n_rings - k);
    return n;
}

// exact grid position of an axis-parallel ray on an axis with n cells of size v
static double axis_pos(const pet_os_geom_desc* d, int b, int n, double v) {
    if (d->ds == v) return (double)(2L * b - (d->n_radial - 1) + n) / 2.0;
    double sb = ((double)b - 0.5 * (double)(d->n_radial - 1)) * d->ds;
    return (sb + 0.5 * n * v) / v;
}

static void build_angles(const pet_os_geom_desc* d, std::vector<AngleK>& out) {
    const double h0 = 0.5 * (double)(d->n_radial - 1);
    out.resize(d->n_angles);
    for (int a = 0; a < d->n_angles; ++a) {
        AngleK K{};
        double c, s;
        if (a == 0) { c = 1.0; s = 0.0; }
        else if (2 * a == d->n_angles) { c = 0.0; s = 1.0; }
        else {
            double th = (double)a * M_PI / (double)d->n_angles;
            c = std::cos(th);
            s = std::sin(th);
        }
        K.c = c;
        K.s = s;
        K.row_major = (std::fabs(c) * d->vx >= std::fabs(s) * d->vy) ? 1 : 0;
        if (K.row_major) {
            if (s == 0.0) {
                K.Q = 0.0; K.invQ = 0.0; K.icv = 0.0; K.K = 0.0;
                K.wslope = d->ds / d->vx;
                K.wC = 0.5 * d->nx - h0 * d->ds / d->vx;
            } else {
                double t = s / c;
                K.Q = -t * (d->vy / d->vx);
                K.invQ = 1.0 / K.Q;
                K.icv = 1.0 / (c * d->vx);
                K.K = 0.5 * d->nx + t * (d->vy / d->vx) * (0.5 * d->ny);
                K.wslope = d->ds * K.icv;
                K.wC = K.K - h0 * d->ds * K.icv;
            }
            K.L = d->vy / std::fabs(c);
            K.Au = -s / c;
            K.Bu = -0.5 * d->ny * d->vy / c;
            K.du = d->vy / c;
        } else {
            if (c == 0.0) {
                K.Q = 0.0; K.invQ = 0.0; K.icv = 0.0; K.K = 0.0;
                K.wslope = d->ds / d->vy;
                K.wC = 0.5 * d->ny - h0 * d->ds / d->vy;
            } else {
                double t = c / s;
                K.Q = -t * (d->vx / d->vy);
                K.invQ = 1.0 / K.Q;
                K.icv = 1.0 / (s * d->vy);
                K.K = 0.5 * d->ny + t * (d->vx / d->vy) * (0.5 * d->nx);
                K.wslope = d->ds * K.icv;
                K.wC = K.K - h0 * d->ds * K.icv;
            }
            K.L = d->vx / std::fabs(s);
            K.Au = c / s;
            K.Bu = 0.5 * d->nx * d->vx / s;
            K.du = -d->vx / s;
        }
        K.inv_du = 1.0 / K.du;
        K.inv_wslope = 1.0 / K.wslope;
        if (c != 0.0 && s != 0.0) {
            const double ex = 0.5 * d->vx * std::fabs(c), ey = 0.5 * d->vy * std::fabs(s);
            K.e_out = ex + ey;
            K.e_in = std::fabs(ex - ey);
            K.inv_de = 1.0 / (K.e_out - K.e_in);
            K.Lmax = std::min(d->vx / std::fabs(s), d->vy / std::fabs(c));
        }
        out[a] = K;
    }
}

}  // namespace petos

using namespace petos;

std::vector<int> pet_os_geom::subset_angles(int subset) const {
    std::vector<int> v;
    for (int a = 0; a < d.n_angles; ++a)
        if (subset == 0 || a % d.n_subsets == subset - 1) v.push_back(a);
    return v;
}

// device block layout helper
namespace {
struct Carver {
    size_t off = 0;
    template <typename T>
    size_t take(size_t n) {
        off = (off + 255) & ~(size_t)255;
        size_t at = off;
        off += n * sizeof(T);
        return at;
    }
};
}  // namespace


// The subset lists live inside dev_block right after the tables; keep their
// offsets in a side table keyed by the geometry.
#include <map>
#include <mutex>
static std::mutex g_geo_mu;
static std::map<const pet_os_geom*, GeomExtra> g_geo_extra;

GeomExtra* petos::extra_of(const pet_os_geom* g) {
    std::lock_guard<std::mutex> lk(g_geo_mu);
    auto it = g_geo_extra.find(g);
    return it == g_geo_extra.end() ? nullptr : &it->second;
}


extern "C" {

const char* pet_os_last_error(void) { return g_last_error.c_str(); }

const char* pet_os_version(void) { return "pet_os 0.1 (gfx950)"; }

// taps of the Gaussian PSF along one axis: exp(-x^2 / 2 sigma^2) at whole-pixel
// distances up to K = ceil(3 sigma / v), normalised to sum 1
static void psf_taps(double fwhm, double v, std::vector<float>& taps, int& K) {
    const double sigma = fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    K = (int)std::ceil(3.0 * sigma / v);
    std::vector<double> w(2 * K + 1);
    double sum = 0.0;
    for (int k = -K; k <= K; ++k) {
        const double x = k * v;
        w[k + K] = std::exp(-x * x / (2.0 * sigma * sigma));
        sum += w[k + K];
    }
    for (double& t : w) taps.push_back((float)(t / sum));
}

static int create_geometry(const pet_os_geom_desc* desc, const float* att_host, pet_os_geom** out);

int pet_os_create_geometry(const pet_os_geom_desc* desc, pet_os_geom** out) {
    return create_geometry(desc, nullptr, out);
}

int pet_os_create_geometry_attenuated(const pet_os_geom_desc* desc, const float* att, pet_os_geom** out) {
    if (!att) return fail(PET_OS_ERR_INVALID_ARG, "att is NULL");
    return create_geometry(desc, att, out);
}

static int create_geometry(const pet_os_geom_desc* desc, const float* att_host, pet_os_geom** out) {
    if (!out) return fail(PET_OS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int rc = validate_desc(desc);
    if (rc) return rc;
    if (att_host && desc->dim != 2) return fail(PET_OS_ERR_INVALID_ARG, "attenuation factors are 2D only");
    pet_os_geom_desc d = *desc;
    if (d.dim == 2) {
        d.nz = 1; d.vz = 1.0; d.n_rings = 1; d.max_ring_diff = 0; d.ring_pitch = 1.0;
    }
    auto* G = new pet_os_geom();
    G->d = d;
    G->n_planes = n_planes_of(&d);
    G->n_vox = (int64_t)d.nx * d.ny * d.nz;
    G->n_bins = (int64_t)G->n_planes * d.n_angles * d.n_radial;
    PETOS_HIP(hipGetDevice(&G->device));

    // host tables (FP64)
    std::vector<AngleK> ang;
    build_angles(&d, ang);
    std::vector<BinK> bins(d.n_radial);
    const int D = d.max_ring_diff, ND = 2 * D + 1;
    std::vector<double> kappa((size_t)d.n_radial * ND);
    for (int b = 0; b < d.n_radial; ++b) {
        BinK& B = bins[b];
        B.sb = ((double)b - 0.5 * (double)(d.n_radial - 1)) * d.ds;
        if (d.dim == 3) {
            B.h = std::sqrt(d.det_radius * d.det_radius - B.sb * B.sb);
            B.inv2h = 1.0 / (2.0 * B.h);
        } else {
            B.h = 1.0;
            B.inv2h = 0.5;
        }
        B.axis_pos_x = axis_pos(&d, b, d.nx, d.vx);
        B.axis_pos_y = axis_pos(&d, b, d.ny, d.vy);
        for (int k = -D; k <= D; ++k) {
            double mz = (double)k * d.ring_pitch / (2.0 * B.h);
            kappa[(size_t)b * ND + k + D] = (d.dim == 3) ? std::sqrt(1.0 + mz * mz) : 1.0;
        }
    }
    std::vector<int2> planes;
    std::vector<int> plane_base(ND);
    std::vector<double> inv_d(ND);
    for (int m = 0; m <= 2 * D; ++m) {
        int dd = (m == 0) ? 0 : ((m % 2) ? (m + 1) / 2 : -(m / 2));
        int lo = dd < 0 ? -dd : 0, hi = dd < 0 ? d.n_rings - 1 : d.n_rings - 1 - dd;
        plane_base[dd + D] = (int)planes.size();
        for (int r1 = lo; r1 <= hi; ++r1) planes.push_back(make_int2(r1, dd));
    }
    if (d.dim == 2) planes.assign(1, make_int2(0, 0));
    for (int k = -D; k <= D; ++k) inv_d[k + D] = (k == 0) ? 0.0 : 1.0 / (double)k;

    const int M = d.n_subsets;
    int max_sub = 0;
    std::vector<int> counts(M);
    for (int i = 1; i <= M; ++i) {
        counts[i - 1] = (int)G->subset_angles(i).size();
        max_sub = std::max(max_sub, counts[i - 1]);
    }
    G->max_sub_angles = max_sub;
    std::vector<int> lists((size_t)M * max_sub, 0);
    for (int i = 1; i <= M; ++i) {
        auto v = G->subset_angles(i);
        std::copy(v.begin(), v.end(), lists.begin() + (size_t)(i - 1) * max_sub);
    }
    std::vector<int> all(d.n_angles);
    for (int a = 0; a < d.n_angles; ++a) all[a] = a;
    // full 2D model: PSF taps (x then y) and attenuation factors
    std::vector<float> taps;
    int kx = 0, ky = 0;
    if (d.psf_fwhm > 0.0) {
        psf_taps(d.psf_fwhm, d.vx, taps, kx);
        psf_taps(d.psf_fwhm, d.vy, taps, ky);
    }
    if (att_host) {
        for (int64_t i = 0; i < G->n_bins; ++i)
            if (!(std::isfinite(att_host[i]) && att_host[i] > 0.0f)) {
                delete G;
                return fail(PET_OS_ERR_INVALID_ARG, "attenuation factors must be finite and > 0");
            }
    }

    Carver cv;
    size_t o_ang = cv.take<AngleK>(ang.size());
    size_t o_bin = cv.take<BinK>(bins.size());
    size_t o_pl = cv.take<int2>(planes.size());
    size_t o_kap = cv.take<double>(kappa.size());
    size_t o_pb = cv.take<int>(plane_base.size());
    size_t o_id = cv.take<double>(inv_d.size());
    size_t o_all = cv.take<int>(all.size());
    size_t o_lst = cv.take<int>(lists.size());
    size_t o_cnt = cv.take<int>(counts.size());
    size_t o_pn = cv.take<float>((size_t)G->n_vox);
    size_t o_sn = cv.take<float>((size_t)G->n_vox);
    size_t o_tap = cv.take<float>(std::max<size_t>(taps.size(), 1));
    size_t o_att = cv.take<float>(att_host ? (size_t)G->n_bins : 1);
    size_t o_tmp = cv.take<float>(d.psf_fwhm > 0.0 ? (size_t)G->n_vox : 1);
    size_t total = cv.off;
    char* blk = nullptr;
    if (hipMalloc(&blk, total) != hipSuccess) {
        delete G;
        return fail(PET_OS_ERR_OUT_OF_MEMORY, "hipMalloc of geometry tables failed");
    }
    G->dev_block = blk;
    auto up = [&](size_t off, const void* src, size_t bytes) {
        return hipMemcpy(blk + off, src, bytes, hipMemcpyHostToDevice);
    };
    if (up(o_ang, ang.data(), ang.size() * sizeof(AngleK)) != hipSuccess ||
        up(o_bin, bins.data(), bins.size() * sizeof(BinK)) != hipSuccess ||
        up(o_pl, planes.data(), planes.size() * sizeof(int2)) != hipSuccess ||
        up(o_kap, kappa.data(), kappa.size() * sizeof(double)) != hipSuccess ||
        up(o_pb, plane_base.data(), plane_base.size() * sizeof(int)) != hipSuccess ||
        up(o_id, inv_d.data(), inv_d.size() * sizeof(double)) != hipSuccess ||
        up(o_all, all.data(), all.size() * sizeof(int)) != hipSuccess ||
        up(o_lst, lists.data(), lists.size() * sizeof(int)) != hipSuccess ||
        up(o_cnt, counts.data(), counts.size() * sizeof(int)) != hipSuccess ||
        (!taps.empty() && up(o_tap, taps.data(), taps.size() * sizeof(float)) != hipSuccess) ||
        (att_host && up(o_att, att_host, (size_t)G->n_bins * sizeof(float)) != hipSuccess)) {
        (void)hipFree(blk);
        delete G;
        return fail(PET_OS_ERR_DEVICE, "upload of geometry tables failed");
    }
    GeoK& k = G->k;
    k.dim = d.dim; k.nx = d.nx; k.ny = d.ny; k.nz = d.nz;
    k.n_angles = d.n_angles; k.n_radial = d.n_radial; k.n_subsets = M; k.n_planes = G->n_planes;
    k.n_rings = d.n_rings; k.max_rd = D; k.nvox = (int)G->n_vox;
    k.vx = d.vx; k.vy = d.vy; k.vz = d.vz; k.ds = d.ds; k.det_radius = d.det_radius;
    k.h0 = 0.5 * (double)(d.n_radial - 1);
    k.ang = (const AngleK*)(blk + o_ang);
    k.bin = (const BinK*)(blk + o_bin);
    k.planes = (const int2*)(blk + o_pl);
    k.kappa = (const double*)(blk + o_kap);
    k.plane_base = (const int*)(blk + o_pb);
    k.inv_d = (const double*)(blk + o_id);
    k.n_sub = std::max(1, d.n_subrays);
    k.sub_h = (float)(d.ds / k.n_sub);
    k.inv_sub_h = (float)(k.n_sub / d.ds);
    k.sub_x0 = (float)(0.5 * d.ds / k.n_sub - 0.5 * d.ds);
    k.inv_nsub = (float)(1.0 / k.n_sub);
    k.sub_half = 0.5 * d.ds - 0.5 * d.ds / k.n_sub;
    k.psf_kx = kx;
    k.psf_ky = ky;
    k.psf = taps.empty() ? nullptr : (const float*)(blk + o_tap);
    k.att = att_host ? (const float*)(blk + o_att) : nullptr;
    G->full_model = k.n_sub > 1 || kx > 0 || att_host != nullptr;
    G->pnorm = (float*)(blk + o_pn);
    G->sens = (float*)(blk + o_sn);
    {
        std::lock_guard<std::mutex> lk(g_geo_mu);
        GeomExtra& e = g_geo_extra[G];
        e.all_angles = (int*)(blk + o_all);
        e.subset_lists = (int*)(blk + o_lst);
        e.d_subset_count = (int*)(blk + o_cnt);
        e.subset_count = counts;
    }

    // a0: sensitivity A^T 1 and p of eq:pj
    BPLaunch L{};
    L.w = nullptr;
    L.angles = (const int*)(blk + o_all);
    L.n_al = d.n_angles;
    L.out = d.psf_fwhm > 0.0 ? (float*)(blk + o_tmp) : G->sens;
    rc = launch_bp(G, L, nullptr);
    if (!rc && d.psf_fwhm > 0.0) rc = launch_blur(G, (float*)(blk + o_tmp), G->sens, nullptr);
    if (rc) { pet_os_destroy_geometry(G); return rc; }
    std::vector<float> s((size_t)G->n_vox);
    if (hipMemcpy(s.data(), G->sens, s.size() * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) {
        pet_os_destroy_geometry(G);
        return fail(PET_OS_ERR_DEVICE, "sensitivity read-back failed");
    }
    std::vector<float> p(s.size());
    double ssum = 0.0;
    for (size_t j = 0; j < s.size(); ++j) {
        ssum += s[j];
        p[j] = (s[j] > 0.0f) ? (float)((double)s[j] / (double)M) : (float)(1.0 / (double)M);
    }
    G->sens_sum = ssum;
    if (hipMemcpy(G->pnorm, p.data(), p.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        pet_os_destroy_geometry(G);
        return fail(PET_OS_ERR_DEVICE, "upload of p failed");
    }
    *out = G;
    return PET_OS_OK;
}

int pet_os_destroy_geometry(pet_os_geom* geom) {
    if (!geom) return fail(PET_OS_ERR_INVALID_ARG, "geom is NULL");
    {
        std::lock_guard<std::mutex> lk(g_geo_mu);
        g_geo_extra.erase(geom);
    }
    if (geom->dev_block) (void)hipFree(geom->dev_block);
    delete geom;
    return PET_OS_OK;
}

int pet_os_geometry_info(const pet_os_geom* g, int64_t* nv, int64_t* nb, int32_t* np) {
    if (!g) return fail(PET_OS_ERR_INVALID_ARG, "geom is NULL");
    if (nv) *nv = g->n_vox;
    if (nb) *nb = g->n_bins;
    if (np) *np = g->n_planes;
    return PET_OS_OK;
}

int pet_os_sensitivity(const pet_os_geom* g, float* out, pet_os_stream stream) {
    if (!g || !out) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    PETOS_HIP(hipMemcpyAsync(out, g->sens, (size_t)g->n_vox * sizeof(float), hipMemcpyDeviceToDevice,
                             (hipStream_t)stream));
    return PET_OS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- work buffers

namespace petos {

// Layout of one request's scratch in a single block: the offsets of every
// buffer from the block's start, and its size.
struct WorkLayout {
    size_t o_w, o_G, o_mu, o_nu, o_fz, o_snap, o_fb, o_red[RED_COUNT], o_tot, o_chk, o_chkt, bytes;
    int caps[RED_COUNT];
    bool need_nu, d3, psf;
};

static WorkLayout work_layout(const pet_os_geom* g, bool need_nu) {
    WorkLayout L{};
    Carver cv;
    size_t nv = (size_t)g->n_vox;
    L.need_nu = need_nu;
    L.d3 = g->d.dim == 3;
    L.psf = g->k.psf_kx > 0;
    // + 4 floats: the 3D back-projector's 16-byte staging loads may read up to
    // three bins past the last row
    L.o_w = cv.take<float>((size_t)g->max_sub_angles * g->n_planes * g->d.n_radial + 4);
    L.o_G = cv.take<float>(nv);
    L.o_mu = cv.take<float>(nv);
    L.o_nu = need_nu ? cv.take<float>(nv) : 0;
    L.o_fz = L.d3 ? cv.take<float>(nv) : 0;
    L.o_snap = cv.take<float>(nv);     // 2D: snapshot of f; 3D: penalty gradient
    L.o_fb = L.psf ? cv.take<float>(nv) : 0;
    L.caps[RED_SUMF] = std::max(std::max(sumf_grid(g), bp_grid_max(g)), elem_grid(g->n_vox));
    L.caps[RED_SUMMU] = std::max(std::max(bp_grid_max(g), elem_grid(g->n_vox)), g->d.dim == 3 ? pen3_grid(g) : 0);
    L.caps[RED_FID] = fp_grid(g, g->d.n_angles);
    L.caps[RED_RDP] = elem_grid(g->n_vox);
    L.caps[RED_SUMY] = elem_grid(g->n_bins);
    L.caps[RED_SUMR] = elem_grid(g->n_bins);
    L.caps[RED_SUMS] = 1;
    for (int r = 0; r < RED_COUNT; ++r) L.o_red[r] = cv.take<double>((size_t)L.caps[r]);
    L.o_tot = cv.take<double>(RED_COUNT);
    L.o_chk = cv.take<unsigned>((size_t)CHECK_GRID * 4);
    L.o_chkt = cv.take<unsigned long long>(4);
    L.bytes = cv.off;
    return L;
}

// point the buffers of w into the block at blk (laid out by L)
static void work_carve(const WorkLayout& L, char* blk, Work* w) {
    *w = Work{};
    w->bytes = L.bytes;
    w->red_block = (double*)blk;
    w->w = (float*)(blk + L.o_w);
    w->G = (float*)(blk + L.o_G);
    w->mu = (float*)(blk + L.o_mu);
    w->nu_frozen = L.need_nu ? (float*)(blk + L.o_nu) : nullptr;
    w->fz = L.d3 ? (float*)(blk + L.o_fz) : nullptr;
    w->fsnap = L.d3 ? nullptr : (float*)(blk + L.o_snap);
    w->gradR = L.d3 ? (float*)(blk + L.o_snap) : nullptr;
    w->fb = L.psf ? (float*)(blk + L.o_fb) : nullptr;
    w->check_part = (unsigned*)(blk + L.o_chk);
    w->check_total = (unsigned long long*)(blk + L.o_chkt);
    for (int r = 0; r < RED_COUNT; ++r) {
        w->red[r].part = (double*)(blk + L.o_red[r]);
        w->red[r].total = (double*)(blk + L.o_tot) + r;
        w->red[r].cap = L.caps[r];
    }
}

size_t work_bytes(const pet_os_geom* g, bool need_nu) { return work_layout(g, need_nu).bytes; }

int work_alloc(const pet_os_geom* g, bool need_nu, Work* w) {
    *w = Work{};
    const WorkLayout L = work_layout(g, need_nu);
    char* blk = nullptr;
    if (hipMalloc(&blk, L.bytes) != hipSuccess) return fail(PET_OS_ERR_OUT_OF_MEMORY, "hipMalloc of scratch failed");
    work_carve(L, blk, w);
    if (hipMemset(blk + L.o_tot, 0, RED_COUNT * sizeof(double)) != hipSuccess) {
        (void)hipFree(blk);
        *w = Work{};
        return fail(PET_OS_ERR_DEVICE, "scratch init failed");
    }
    return PET_OS_OK;
}

int work_place(const pet_os_geom* g, bool need_nu, void* base, size_t cap, Work* w, hipStream_t s) {
    *w = Work{};
    const WorkLayout L = work_layout(g, need_nu);
    if (L.bytes > cap)
        return fail(PET_OS_ERR_INVALID_ARG, "the reconstruction needs " + std::to_string(L.bytes) +
                                                " bytes of scratch; the static area holds " + std::to_string(cap));
    work_carve(L, (char*)base, w);
    // the totals start at zero, as in a fresh allocation (a fill kernel, so
    // that no memset is recorded if the caller captures the stream)
    int rc = launch_fill((float*)w->red[0].total, (int64_t)(RED_COUNT * sizeof(double) / sizeof(float)), 0.0f, s);
    if (rc) *w = Work{};
    return rc;
}

void work_free(Work* w) {
    if (w->red_block) (void)hipFree(w->red_block);
    *w = Work{};
}

}  // namespace petos

// ---------------------------------------------------------------- state


namespace petos {

int validate_params(const pet_os_params* p, const pet_os_geom* g) {
    if (!p) return fail(PET_OS_ERR_INVALID_ARG, "params is NULL");
    if (p->mode == PET_OS_OSEM) {
        // OSEM reads only what the objective needs
        if (!(std::isfinite(p->beta) && p->beta >= 0.0)) return fail(PET_OS_ERR_INVALID_ARG, "beta must be >= 0");
        if (!(std::isfinite(p->gamma_R) && p->gamma_R >= 0.0))
            return fail(PET_OS_ERR_INVALID_ARG, "gamma_R must be >= 0");
        if (!finite_pos(p->eps)) return fail(PET_OS_ERR_INVALID_ARG, "eps must be > 0");
        return PET_OS_OK;
    }
    if (p->mode < PET_OS_BSREM || p->mode > PET_OS_P2) return fail(PET_OS_ERR_INVALID_ARG, "unknown mode");
    if (!(std::isfinite(p->beta) && p->beta >= 0.0)) return fail(PET_OS_ERR_INVALID_ARG, "beta must be >= 0");
    if (!(std::isfinite(p->gamma_R) && p->gamma_R >= 0.0)) return fail(PET_OS_ERR_INVALID_ARG, "gamma_R must be >= 0");
    if (!finite_pos(p->eps)) return fail(PET_OS_ERR_INVALID_ARG, "eps must be > 0");
    if (!finite_pos(p->U)) return fail(PET_OS_ERR_INVALID_ARG, "U must be > 0");
    if (!(std::isfinite(p->t_clip) && p->t_clip > 0.0 && p->t_clip < p->U))
        return fail(PET_OS_ERR_INVALID_ARG, "t_clip must be in (0, U)");
    if (!finite_pos(p->lambda0) || !finite_pos(p->a)) return fail(PET_OS_ERR_INVALID_ARG, "lambda0, a must be > 0");
    if (p->mode == PET_OS_M2 || p->mode == PET_OS_P2) {
        if (!finite_pos(p->rho) || !finite_pos(p->delta1) || !finite_pos(p->delta2))
            return fail(PET_OS_ERR_INVALID_ARG, "rho, delta1, delta2 must be > 0");
    }
    if (p->mode == PET_OS_P1 || p->mode == PET_OS_P2) {
        if (!(finite_pos(p->nu1) && std::isfinite(p->nu2) && p->nu1 < p->nu2))
            return fail(PET_OS_ERR_INVALID_ARG, "need 0 < nu1 < nu2");
        if (p->J0 < 0 || p->J1 < p->J0) return fail(PET_OS_ERR_INVALID_ARG, "need 0 <= J0 <= J1");
    }
    (void)g;
    return PET_OS_OK;
}

// smallest float not below x (x finite, > 0)
static float float_at_or_above(double x) {
    float v = (float)x;
    if ((double)v < x) v = std::nextafter(v, std::numeric_limits<float>::infinity());
    return v;
}

BoxK make_box(double U, double t) {
    BoxK b;
    b.half_up = float_at_or_above(0.5 * U);
    b.U_up = float_at_or_above(U);
    b.U = (float)U;
    b.t_lo = (float)t;
    b.t_hi = (float)(U - t);
    return b;
}

// The data of the problem statement (Sec. II-A, eq:BoundedSet): counts
// y >= 0, background r > 0 (gamma in R^p_{++}), initial image f in
// B = [0, U]^q (OSEM: f >= 0), every entry finite; with the adaptive nu of
// eq:nuki from the first subiteration (P1/P2, J0 = 0) the mean of f must be
// > 0 (it divides the gradient magnitude in mu).
int check_data(const pet_os_geom* g, const pet_os_params* p, Work* w, const float* f, const float* y,
               const float* r, hipStream_t s) {
    float f_lim = std::numeric_limits<float>::infinity();
    if (p->mode != PET_OS_OSEM) {
        f_lim = (float)p->U;
        if ((double)f_lim <= p->U) f_lim = std::nextafter(f_lim, std::numeric_limits<float>::infinity());
    }
    int rc = launch_check_data(y, r, g->n_bins, f, g->n_vox, f_lim, w->check_part, w->check_total, s);
    if (rc) return rc;
    unsigned long long c[4] = {0, 0, 0, 0};
    PETOS_HIP(hipMemcpyAsync(c, w->check_total, sizeof(c), hipMemcpyDeviceToHost, s));
    PETOS_HIP(hipStreamSynchronize(s));
    if (c[0]) return fail(PET_OS_ERR_INVALID_ARG, "y: " + std::to_string(c[0]) + " entries negative or not finite");
    if (c[1])
        return fail(PET_OS_ERR_INVALID_ARG, "r: " + std::to_string(c[1]) + " entries not > 0 or not finite");
    if (c[2])
        return fail(PET_OS_ERR_INVALID_ARG, "f: " + std::to_string(c[2]) +
                                                (p->mode == PET_OS_OSEM ? " entries negative or not finite"
                                                                        : " entries outside [0, U] or not finite"));
    if ((p->mode == PET_OS_P1 || p->mode == PET_OS_P2) && p->J0 == 0 && c[3] == 0)
        return fail(PET_OS_ERR_INVALID_ARG, "f: mean must be > 0 when nu is adaptive from the first subiteration");
    return PET_OS_OK;
}

// FP64 scalar schedule of subiteration (k, i): lambda_k (thm:SpecificSDPs),
// alpha_{k,i} (preconditioner:Nesterov / preconditioner:KM) and the nu mode
// of eq:nuki; advances the Nesterov t.
Sched sched_next(const pet_os_params& p, int M, int64_t k, int i, double* t_nest, int have_frozen) {
    const int64_t J = k * (int64_t)M + i;
    Sched s;
    s.lam = p.lambda0 / (p.a * (double)k + 1.0);
    s.alpha = 1.0;
    if (p.mode == PET_OS_M1 || p.mode == PET_OS_P1) {
        double t = *t_nest;
        double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
        s.alpha = 1.0 + (t - 1.0) / tn;
        *t_nest = tn;
    } else if (p.mode == PET_OS_M2 || p.mode == PET_OS_P2) {
        double n = (double)(J - 1);
        s.alpha = (p.rho * n + p.delta2) / (n + p.delta1);
    }
    s.nu_mode = NU_ONE;
    if (p.mode == PET_OS_OSEM) {
        s.lam = 1.0;
        return s;
    }
    if (p.mode == PET_OS_P1 || p.mode == PET_OS_P2) {
        if (J <= p.J0) s.nu_mode = NU_ONE;
        else if (J < p.J1) s.nu_mode = NU_COMPUTE;
        else if (J == p.J1) s.nu_mode = NU_COMPUTE_FREEZE;
        else s.nu_mode = have_frozen ? NU_FROZEN : NU_ONE;
    }
    return s;
}

void schedule_table(const pet_os_params& p, int M, int64_t n_sub, std::vector<float>& step, std::vector<int>& nu) {
    step.resize((size_t)n_sub);
    nu.resize((size_t)n_sub);
    double t = 1.0;
    int have = 0;
    for (int64_t J = 1; J <= n_sub; ++J) {
        const int64_t k = (J - 1) / M;
        const int i = (int)((J - 1) % M) + 1;
        Sched sc = sched_next(p, M, k, i, &t, have);
        step[(size_t)(J - 1)] = (float)(sc.lam * sc.alpha);
        nu[(size_t)(J - 1)] = sc.nu_mode;
        if (sc.nu_mode == NU_COMPUTE_FREEZE) have = 1;
    }
}

static Sched schedule_step(pet_os_state* st) {
    return sched_next(st->p, st->g->d.n_subsets, st->k, st->i, &st->t_nest, st->have_frozen);
}

// events around launches of the profiled kernel
// Per-kernel profiling: a bracket of one launch hands its events to that
// launch (recorded by the dispatch: the kernel's own duration); a bracket of
// several launches records them around the launches.
static int prof_begin(pet_os_state* st, int kernel, hipStream_t s, hipEvent_t* end, bool single) {
    *end = nullptr;
    if (st->prof_kernel != kernel) return PET_OS_OK;
    if (st->prof_used == st->prof_ev.size()) {
        hipEvent_t a, b;
        PETOS_HIP(hipEventCreate(&a));
        PETOS_HIP(hipEventCreate(&b));
        st->prof_ev.emplace_back(a, b);
    }
    auto& pr = st->prof_ev[st->prof_used++];
    if (single) {
        g_launch_events = LaunchEvents{pr.first, pr.second};
    } else {
        PETOS_HIP(hipEventRecord(pr.first, s));
        *end = pr.second;
    }
    return PET_OS_OK;
}

static int prof_end(hipEvent_t end, hipStream_t s) {
    if (g_launch_events.start != nullptr) {
        // nothing was launched (an empty subset): a zero-length interval
        const LaunchEvents e = g_launch_events;
        g_launch_events = LaunchEvents{};
        PETOS_HIP(hipEventRecord(e.start, s));
        PETOS_HIP(hipEventRecord(e.stop, s));
    }
    if (end) PETOS_HIP(hipEventRecord(end, s));
    return PET_OS_OK;
}

// 3D: the bin-major copy of (y, r) that the staged forward projector reads
// (its y and r loads are then coalesced), made when the state first sees the
// pair of buffers, as the data check is.  A state that may not allocate (the
// static-scratch entry point), or whose allocation fails, reads y and r in
// their natural layout instead.
static int ensure_yr(pet_os_state* st, const float* y, const float* r, hipStream_t s) {
    const pet_os_geom* g = st->g;
    if (!st->may_allocate || !fp3_reads_yr(g)) return PET_OS_OK;
    if (st->yr != nullptr && st->yr_y == y && st->yr_r == r) return PET_OS_OK;
    if (st->yr == nullptr) {
        void* p = nullptr;
        if (hipMalloc(&p, (size_t)g->n_bins * sizeof(float2)) != hipSuccess) {
            (void)hipGetLastError();    // the natural layout serves
            return PET_OS_OK;
        }
        st->yr = (float2*)p;
    }
    st->yr_y = st->yr_r = nullptr;
    int rc = launch_yr3(g, y, r, st->yr, s);
    if (rc) return rc;
    st->yr_y = y;
    st->yr_r = r;
    return PET_OS_OK;
}

static int run_subiteration(pet_os_state* st, float* f, const float* y, const float* r, hipStream_t s,
                            bool sumf_current) {
    const pet_os_geom* g = st->g;
    GeomExtra* ex = extra_of(g);
    if (!ex) return fail(PET_OS_ERR_INVALID_ARG, "geometry was destroyed");
    const int M = g->d.n_subsets;
    Sched sc = schedule_step(st);
    const bool want_mu = sc.nu_mode == NU_COMPUTE || sc.nu_mode == NU_COMPUTE_FREEZE;
    int rc;
    // sum f of the entering iterate (mean f of the smoothness measure) and,
    // in 3D, its z-fastest copy, unless the previous update left them
    if ((want_mu || g->d.dim == 3) && !sumf_current) {
        rc = launch_sum_f(g, f, st->w.fz, st->w.red[RED_SUMF], s);
        if (rc) return rc;
    }
    const int* angles = ex->subset_lists + (size_t)(st->i - 1) * g->max_sub_angles;
    const int n_al = ex->subset_count[st->i - 1];
    const bool d3 = g->d.dim == 3;
    FPLaunch F{};
    F.f = f; F.fz = st->w.fz; F.y = y; F.r = r; F.out = st->w.w; F.angles = angles; F.n_al = n_al;
    if (d3 && (rc = ensure_yr(st, y, r, s))) return rc;
    F.yr = (d3 && st->yr != nullptr && st->yr_y == y && st->yr_r == r) ? st->yr : nullptr;
    const bool osem = st->p.mode == PET_OS_OSEM;
    const float* sens_i = osem ? st->osem_sens + (size_t)(st->i - 1) * g->n_vox : nullptr;
    F.mode = osem ? FP_EM : FP_RATIO;
    // threads per ray chosen for the largest subset, as the batched path does
    F.seg = fp_seg_for(g, (long long)g->max_sub_angles * g->n_planes * g->d.n_radial, g->tuned_seg);
    if (!d3) {
        // 2D: the pixel pass (snapshot of f, mu) rides in the forward launch
        F.px_fsnap = st->w.fsnap;
        F.px_mu = st->w.mu;
        F.px_want_mu = want_mu ? 1 : 0;
        F.px_part_f = st->w.red[RED_SUMF].part;
        F.px_n_part_f = sumf_grid(g);
        F.px_red_mu = st->w.red[RED_SUMMU];
    }
    const bool psf = !d3 && g->k.psf_kx > 0;
    hipEvent_t ev;
    if ((rc = prof_begin(st, 0, s, &ev, !psf))) return rc;
    if (psf) {
        // the projector sees the PSF-blurred iterate; the pixel pass the iterate
        rc = launch_blur(g, f, st->w.fb, s);
        F.f = st->w.fb;
        F.px_f = f;
    }
    if (!rc) rc = launch_fp(g, F, s);
    if (rc || (rc = prof_end(ev, s))) return rc;
    BPLaunch B{};
    B.w = st->w.w; B.w_natural = 0; B.angles = angles; B.n_al = n_al;
    B.beta_over_M = (float)(st->p.beta / (double)M);
    B.gamma_R = (float)st->p.gamma_R;
    B.eps = (float)st->p.eps;
    const float step = (float)(sc.lam * sc.alpha);
    if (!d3) {
        // 2D: back-projection, penalty gradient and update of each tile in one launch
        B.f = st->w.fsnap; B.out = nullptr; B.mu = st->w.mu; B.want_mu = 0;
        B.fnew = f; B.pnorm = g->pnorm; B.nu_frozen = st->w.nu_frozen; B.nu_mode = sc.nu_mode;
        B.step = step; B.nu1 = (float)st->p.nu1; B.nu2 = (float)st->p.nu2;
        B.box = make_box(st->p.U, st->p.t_clip);
        B.part_mu = st->w.red[RED_SUMMU].part; B.n_part_mu = px_grid(g);
        B.red_f = st->w.red[RED_SUMF];
        B.osem_sens = sens_i;
        if (osem) B.beta_over_M = 0.0f;
        if ((rc = prof_begin(st, 1, s, &ev, !psf))) return rc;
        if (psf) {
            // B A_i^T w needs the neighbouring tiles' back-projection: plain
            // back-projection, blur, then the image-space part per tile
            BPLaunch P{};
            P.w = st->w.w; P.w_natural = 0; P.angles = angles; P.n_al = n_al; P.out = st->w.G;
            rc = launch_bp(g, P, s);
            if (!rc) rc = launch_upd2(g, B, st->w.G, true, s);
        } else {
            rc = launch_bp(g, B, s);
        }
        if (rc || (rc = prof_end(ev, s))) return rc;
    } else {
        // 3D: the back-projection into G and (SDP-BSREM) in the same launch
        // the penalty gradient of f and mu, then the update, which adds the
        // penalty gradient to the back-projection
        B.out = st->w.G;
        if (!osem) {
            B.f = f; B.mu = st->w.mu; B.want_mu = want_mu ? 1 : 0;
            B.part_f = st->w.red[RED_SUMF].part;
            B.n_part_f = sumf_grid(g);
            B.red_mu = st->w.red[RED_SUMMU];
            B.gradR = st->w.gradR;
        }
        if ((rc = prof_begin(st, 1, s, &ev, true))) return rc;
        rc = launch_bp(g, B, s);
        if (rc || (rc = prof_end(ev, s))) return rc;
        UpdLaunch U{};
        if (!osem) {
            U.gradR = st->w.gradR;
            U.beta_over_M = B.beta_over_M;
        }
        U.osem_sens = sens_i;
        U.f = f; U.fz = st->w.fz; U.G = st->w.G; U.mu = st->w.mu; U.pnorm = g->pnorm; U.nu_frozen = st->w.nu_frozen;
        U.nu_mode = sc.nu_mode;
        U.step = step;
        U.nu1 = (float)st->p.nu1; U.nu2 = (float)st->p.nu2;
        U.box = make_box(st->p.U, st->p.t_clip);
        U.part_mu = st->w.red[RED_SUMMU].part;
        U.n_part_mu = pen3_grid(g);
        U.red_f = st->w.red[RED_SUMF];
        if ((rc = prof_begin(st, 2, s, &ev, true))) return rc;
        rc = launch_update(g, U, s);
        if (rc || (rc = prof_end(ev, s))) return rc;
    }
    if (sc.nu_mode == NU_COMPUTE_FREEZE) st->have_frozen = 1;
    st->i += 1;
    if (st->i > M) { st->i = 1; st->k += 1; }
    return PET_OS_OK;
}

// queue Phi(f) = fidelity + beta R into two device doubles (fid, R) at dst
static int queue_objective(const pet_os_geom* g, const pet_os_params* p, Work* w, const float* f,
                           const float* y, const float* r, double* dst, hipStream_t s) {
    GeomExtra* ex = extra_of(g);
    int rc = PET_OS_OK;
    if (g->d.dim == 3 && (rc = launch_prep3(g, f, w->fz, w->red[RED_SUMF], s))) return rc;
    FPLaunch F{};
    F.f = f; F.fz = w->fz; F.y = y; F.r = r; F.out = nullptr; F.angles = ex->all_angles; F.n_al = g->d.n_angles;
    F.mode = FP_OBJECTIVE; F.red = w->red[RED_FID];
    if (g->d.dim == 2 && g->k.psf_kx > 0) {
        if ((rc = launch_blur(g, f, w->fb, s))) return rc;
        F.f = w->fb;
    }
    rc = launch_fp(g, F, s);
    if (!rc) rc = launch_finalize(w->red[RED_FID], fp_grid(g, g->d.n_angles), s);
    if (!rc) rc = launch_rdp_value(g, f, (float)p->gamma_R, (float)p->eps, w->red[RED_RDP], s);
    if (!rc) rc = launch_finalize(w->red[RED_RDP], elem_grid(g->n_vox), s);
    if (rc) return rc;
    PETOS_HIP(hipMemcpyAsync(dst, w->red[RED_FID].total, sizeof(double), hipMemcpyDeviceToDevice, s));
    PETOS_HIP(hipMemcpyAsync(dst + 1, w->red[RED_RDP].total, sizeof(double), hipMemcpyDeviceToDevice, s));
    return PET_OS_OK;
}

}  // namespace petos

extern "C" {

int pet_os_state_create(const pet_os_geom* g, const pet_os_params* p, pet_os_state** out) {
    if (!out) return fail(PET_OS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!g || !extra_of(g)) return fail(PET_OS_ERR_INVALID_ARG, "invalid geometry");
    int rc = validate_params(p, g);
    if (rc) return rc;
    auto* st = new pet_os_state();
    st->g = g;
    st->p = *p;
    st->k = 0;
    st->i = 1;
    st->t_nest = 1.0;
    st->have_frozen = 0;
    const bool need_nu = p->mode == PET_OS_P1 || p->mode == PET_OS_P2;
    rc = work_alloc(g, need_nu, &st->w);
    if (rc) { delete st; return rc; }
    if (p->mode == PET_OS_OSEM) {
        // the M subset sensitivities A_i^T 1 of the EM update
        GeomExtra* ex = extra_of(g);
        const int M = g->d.n_subsets;
        if (hipMalloc(&st->osem_sens, sizeof(float) * (size_t)M * g->n_vox) != hipSuccess) {
            work_free(&st->w);
            delete st;
            return fail(PET_OS_ERR_OUT_OF_MEMORY, "hipMalloc of the subset sensitivities failed");
        }
        for (int i = 0; i < M && !rc; ++i) {
            BPLaunch L{};
            L.w = nullptr;
            L.angles = ex->subset_lists + (size_t)i * g->max_sub_angles;
            L.n_al = ex->subset_count[i];
            float* si = st->osem_sens + (size_t)i * g->n_vox;
            // with a PSF: B^T P^T att, the back-projection blurred from the state's scratch
            const bool psf = g->d.dim == 2 && g->k.psf_kx > 0;
            L.out = psf ? st->w.fb : si;
            rc = launch_bp(g, L, nullptr);
            if (!rc && psf) rc = launch_blur(g, st->w.fb, si, nullptr);
        }
        if (!rc && hipDeviceSynchronize() != hipSuccess) rc = fail(PET_OS_ERR_DEVICE, "subset sensitivities failed");
        if (rc) {
            (void)hipFree(st->osem_sens);
            work_free(&st->w);
            delete st;
            return rc;
        }
    }
    *out = st;
    return PET_OS_OK;
}

int pet_os_state_destroy(pet_os_state* st) {
    if (!st) return fail(PET_OS_ERR_INVALID_ARG, "state is NULL");
    work_free(&st->w);
    if (st->osem_sens) (void)hipFree(st->osem_sens);
    if (st->obj_dev) (void)hipFree(st->obj_dev);
    if (st->yr) (void)hipFree(st->yr);
    for (auto& pr : st->prof_ev) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    delete st;
    return PET_OS_OK;
}

int pet_os_state_position(const pet_os_state* st, int64_t* k, int32_t* i) {
    if (!st) return fail(PET_OS_ERR_INVALID_ARG, "state is NULL");
    if (k) *k = st->k;
    if (i) *i = st->i;
    return PET_OS_OK;
}

// the data check of a state's (f, y, r) buffers, made when they differ from
// the last ones it accepted
static int check_state_data(pet_os_state* st, const float* f, const float* y, const float* r, hipStream_t s) {
    if (st->checked_f == f && st->checked_y == y && st->checked_r == r) return PET_OS_OK;
    int rc = check_data(st->g, &st->p, &st->w, f, y, r, s);
    if (rc) return rc;
    st->checked_f = f;
    st->checked_y = y;
    st->checked_r = r;
    return PET_OS_OK;
}

int pet_os_subiteration(pet_os_state* st, float* f, const float* y, const float* r, pet_os_stream stream) {
    if (!st || !f || !y || !r) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    int rc = check_state_data(st, f, y, r, (hipStream_t)stream);
    if (rc) return rc;
    return run_subiteration(st, f, y, r, (hipStream_t)stream, false);
}

int pet_os_forward(const pet_os_geom* g, const float* f, int32_t subset, float* q, pet_os_stream stream) {
    if (!g || !f || !q) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    GeomExtra* ex = extra_of(g);
    if (!ex) return fail(PET_OS_ERR_INVALID_ARG, "invalid geometry");
    if (subset < 0 || subset > g->d.n_subsets) return fail(PET_OS_ERR_INVALID_ARG, "subset out of range");
    FPLaunch F{};
    F.f = f; F.out = q; F.mode = FP_PLAIN;
    F.angles = subset == 0 ? ex->all_angles : ex->subset_lists + (size_t)(subset - 1) * g->max_sub_angles;
    F.n_al = subset == 0 ? g->d.n_angles : ex->subset_count[subset - 1];
    if (g->d.dim == 2 && g->k.psf_kx > 0) {
        // the PSF-blurred image, in scratch released before returning
        hipStream_t s = (hipStream_t)stream;
        float* tmp = nullptr;
        if (hipMalloc(&tmp, sizeof(float) * (size_t)g->n_vox) != hipSuccess)
            return fail(PET_OS_ERR_OUT_OF_MEMORY, "hipMalloc failed");
        int rc = launch_blur(g, f, tmp, s);
        F.f = tmp;
        if (!rc) rc = launch_fp(g, F, s);
        if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = fail(PET_OS_ERR_DEVICE, "stream synchronize failed");
        (void)hipFree(tmp);
        return rc;
    }
    if (g->d.dim == 2) return launch_fp(g, F, (hipStream_t)stream);
    // 3D: the projector reads a z-fastest copy of f, made in scratch that is
    // released before returning (this call waits for the stream)
    hipStream_t s = (hipStream_t)stream;
    Work w;
    int rc = work_alloc(g, false, &w);
    if (rc) return rc;
    rc = launch_prep3(g, f, w.fz, w.red[RED_SUMF], s);
    F.fz = w.fz;
    if (!rc) rc = launch_fp(g, F, s);
    if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = fail(PET_OS_ERR_DEVICE, "stream synchronize failed");
    work_free(&w);
    return rc;
}

int pet_os_back(const pet_os_geom* g, const float* w, int32_t subset, float* out, pet_os_stream stream) {
    if (!g || !w || !out) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    GeomExtra* ex = extra_of(g);
    if (!ex) return fail(PET_OS_ERR_INVALID_ARG, "invalid geometry");
    if (subset < 0 || subset > g->d.n_subsets) return fail(PET_OS_ERR_INVALID_ARG, "subset out of range");
    BPLaunch B{};
    B.w = w; B.w_natural = 1; B.out = out;
    B.angles = subset == 0 ? ex->all_angles : ex->subset_lists + (size_t)(subset - 1) * g->max_sub_angles;
    B.n_al = subset == 0 ? g->d.n_angles : ex->subset_count[subset - 1];
    if (g->d.dim == 2 && g->k.psf_kx > 0) {
        // back-projection into scratch, then the (symmetric) PSF into out
        hipStream_t s = (hipStream_t)stream;
        float* tmp = nullptr;
        if (hipMalloc(&tmp, sizeof(float) * (size_t)g->n_vox) != hipSuccess)
            return fail(PET_OS_ERR_OUT_OF_MEMORY, "hipMalloc failed");
        B.out = tmp;
        int rc = launch_bp(g, B, s);
        if (!rc) rc = launch_blur(g, tmp, out, s);
        if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = fail(PET_OS_ERR_DEVICE, "stream synchronize failed");
        (void)hipFree(tmp);
        return rc;
    }
    return launch_bp(g, B, (hipStream_t)stream);
}

int pet_os_attenuation_factors(const pet_os_geom* g, const float* mu, float* att, pet_os_stream stream) {
    if (!g || !mu || !att) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    GeomExtra* ex = extra_of(g);
    if (!ex) return fail(PET_OS_ERR_INVALID_ARG, "invalid geometry");
    if (g->d.dim != 2) return fail(PET_OS_ERR_INVALID_ARG, "attenuation factors are 2D only");
    hipStream_t s = (hipStream_t)stream;
    // line integrals of mu through the sub-ray model, without PSF or attenuation
    FPLaunch F{};
    F.f = mu; F.out = att; F.mode = FP_PLAIN; F.raw = 1;
    F.angles = ex->all_angles; F.n_al = g->d.n_angles;
    int rc = launch_fp(g, F, s);
    if (!rc) rc = launch_expneg(att, att, g->n_bins, s);
    return rc;
}

int pet_os_objective(const pet_os_geom* g, const pet_os_params* p, const float* f, const float* y,
                     const float* r, double* phi, pet_os_stream stream) {
    if (!g || !p || !f || !y || !r || !phi) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    if (!extra_of(g)) return fail(PET_OS_ERR_INVALID_ARG, "invalid geometry");
    Work w;
    int rc = work_alloc(g, false, &w);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    double* dst = nullptr;
    if (hipMalloc(&dst, 2 * sizeof(double)) != hipSuccess) {
        work_free(&w);
        return fail(PET_OS_ERR_OUT_OF_MEMORY, "hipMalloc failed");
    }
    rc = queue_objective(g, p, &w, f, y, r, dst, s);
    double h[2] = {0, 0};
    if (!rc) {
        if (hipMemcpyAsync(h, dst, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = fail(PET_OS_ERR_DEVICE, "objective read-back failed");
    }
    (void)hipFree(dst);
    work_free(&w);
    if (rc) return rc;
    *phi = h[0] + p->beta * h[1];
    if (!std::isfinite(*phi)) return fail(PET_OS_ERR_NUMERIC, "objective is not finite");
    return PET_OS_OK;
}

int pet_os_default_U(const pet_os_geom* g, const float* f0, const float* y, const float* r, double* U,
                     pet_os_stream stream) {
    if (!g || !f0 || !y || !r || !U) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    Work w;
    int rc = work_alloc(g, false, &w);
    if (rc) return rc;
    rc = launch_sum(y, g->n_bins, w.red[RED_SUMY], s);
    if (!rc) rc = launch_finalize(w.red[RED_SUMY], elem_grid(g->n_bins), s);
    if (!rc) rc = launch_sum(r, g->n_bins, w.red[RED_SUMR], s);
    if (!rc) rc = launch_finalize(w.red[RED_SUMR], elem_grid(g->n_bins), s);
    double sy = 0, sr = 0;
    std::vector<float> fh((size_t)g->n_vox);
    if (!rc) {
        if (hipMemcpyAsync(&sy, w.red[RED_SUMY].total, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&sr, w.red[RED_SUMR].total, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(fh.data(), f0, fh.size() * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = fail(PET_OS_ERR_DEVICE, "default_U read-back failed");
    }
    work_free(&w);
    if (rc) return rc;
    double fmax = 0.0;
    for (float v : fh) fmax = std::max(fmax, (double)v);
    double chat = (sy - sr > 0.0 && g->sens_sum > 0.0) ? (sy - sr) / g->sens_sum : 0.0;
    *U = 1e3 * std::max(fmax, chat);
    return PET_OS_OK;
}

int pet_os_subset_gradient(const pet_os_geom* g, const pet_os_params* p, const float* f, const float* y,
                           const float* r, int32_t subset, float* grad, pet_os_stream stream) {
    if (!g || !p || !f || !y || !r || !grad) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    GeomExtra* ex = extra_of(g);
    if (!ex) return fail(PET_OS_ERR_INVALID_ARG, "invalid geometry");
    if (subset < 0 || subset > g->d.n_subsets) return fail(PET_OS_ERR_INVALID_ARG, "subset out of range");
    if (!(std::isfinite(p->beta) && p->beta >= 0.0 && std::isfinite(p->gamma_R) && p->gamma_R >= 0.0 &&
          std::isfinite(p->eps) && p->eps >= 0.0))
        return fail(PET_OS_ERR_INVALID_ARG, "beta, gamma_R and eps must be finite and >= 0");
    hipStream_t s = (hipStream_t)stream;
    const int* angles = subset == 0 ? ex->all_angles : ex->subset_lists + (size_t)(subset - 1) * g->max_sub_angles;
    const int n_al = subset == 0 ? g->d.n_angles : ex->subset_count[subset - 1];
    Work w;
    int rc = work_alloc(g, false, &w);
    if (rc) return rc;
    // the ratio sinogram of every ray does not fit the subset-sized scratch
    float* wsino = w.w;
    float* big = nullptr;
    if (n_al > g->max_sub_angles) {
        // + 4 floats of padding for the 3D back-projector's 16-byte staging loads
        if (hipMalloc(&big, sizeof(float) * ((size_t)n_al * g->n_planes * g->d.n_radial + 4)) != hipSuccess) {
            work_free(&w);
            return fail(PET_OS_ERR_OUT_OF_MEMORY, "hipMalloc of the ratio sinogram failed");
        }
        wsino = big;
    }
    if (g->d.dim == 3) rc = launch_prep3(g, f, w.fz, w.red[RED_SUMF], s);
    FPLaunch F{};
    F.f = f; F.fz = w.fz; F.y = y; F.r = r; F.out = wsino; F.angles = angles; F.n_al = n_al;
    F.mode = FP_RATIO;
    F.seg = fp_seg_for(g, (long long)n_al * g->n_planes * g->d.n_radial, g->tuned_seg);
    const bool psf = g->d.dim == 2 && g->k.psf_kx > 0;
    if (psf && !rc) {
        rc = launch_blur(g, f, w.fb, s);
        F.f = w.fb;
    }
    if (!rc) rc = launch_fp(g, F, s);
    BPLaunch B{};
    B.w = wsino; B.w_natural = 0; B.angles = angles; B.n_al = n_al;
    B.f = f; B.out = grad; B.mu = w.mu; B.want_mu = 0;
    B.beta_over_M = (float)(subset == 0 ? p->beta : p->beta / (double)g->d.n_subsets);
    B.gamma_R = (float)p->gamma_R;
    B.eps = (float)p->eps;
    B.part_f = w.red[RED_SUMF].part;
    B.n_part_f = sumf_grid(g);
    B.red_mu = w.red[RED_SUMMU];
    if (psf) {
        // B A_i^T w, then the penalty gradient per tile
        BPLaunch P{};
        P.w = wsino; P.w_natural = 0; P.angles = angles; P.n_al = n_al; P.out = w.G;
        if (!rc) rc = launch_bp(g, P, s);
        if (!rc) rc = launch_upd2(g, B, w.G, true, s);
    } else if (!rc && g->d.dim == 3) {
        // the back-projection into grad, then the penalty gradient added to it
        BPLaunch P = B;
        P.f = nullptr;
        rc = launch_bp(g, P, s);
        if (!rc) rc = launch_pen3(g, B, s);
    } else if (!rc) {
        rc = launch_bp(g, B, s);
    }
    if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = fail(PET_OS_ERR_DEVICE, "stream synchronize failed");
    if (big) (void)hipFree(big);
    work_free(&w);
    return rc;
}

static double angle_of(double ab, double aa, double bb) {
    if (!(aa > 0.0) || !(bb > 0.0)) return std::nan("");
    const double c = ab / std::sqrt(aa * bb);
    return std::acos(std::max(-1.0, std::min(1.0, c)));
}

int pet_os_gradient_angles(const pet_os_geom* g, const float* h_prev, const float* h_cur, const float* f,
                           double smooth_frac, double var_frac, double* theta, int64_t* count,
                           pet_os_stream stream) {
    if (!g || !h_prev || !h_cur || !f || !theta) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    if (!extra_of(g)) return fail(PET_OS_ERR_INVALID_ARG, "invalid geometry");
    if (!(std::isfinite(smooth_frac) && smooth_frac >= 0.0 && std::isfinite(var_frac) && var_frac >= 0.0))
        return fail(PET_OS_ERR_INVALID_ARG, "smooth_frac and var_frac must be finite and >= 0");
    hipStream_t s = (hipStream_t)stream;
    const size_t nd = angle_scratch_doubles(g->n_vox);
    double* blk = nullptr;
    if (hipMalloc(&blk, nd * sizeof(double)) != hipSuccess) return fail(PET_OS_ERR_OUT_OF_MEMORY, "hipMalloc failed");
    double* sums = blk + nd - 8;
    int rc = launch_gradient_angles(g, h_prev, h_cur, f, smooth_frac, var_frac, blk, s);
    double h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (!rc && (hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess))
        rc = fail(PET_OS_ERR_DEVICE, "angle read-back failed");
    (void)hipFree(blk);
    if (rc) return rc;
    theta[0] = angle_of(h[0], h[1], h[2]);
    theta[1] = angle_of(h[4], h[5], h[6]);
    if (count) {
        count[0] = (int64_t)h[3];
        count[1] = (int64_t)h[7];
    }
    return PET_OS_OK;
}

// n_iter iterations on a state; objective pairs (fid, R) after iteration j+1
// go to obj_dev[2 * (slot0 + j + 1)] when wanted.
static int run_iterations(pet_os_state* st, float* f, const float* y, const float* r, int n_iter, bool want_obj,
                          int every, int slot0, hipStream_t s, std::vector<char>& have) {
    const int M = st->g->d.n_subsets;
    bool sumf_current = false;
    int rc = PET_OS_OK;
    for (int j = 0; j < n_iter && !rc; ++j) {
        for (int i = 0; i < M && !rc; ++i) {
            rc = run_subiteration(st, f, y, r, s, sumf_current);
            sumf_current = true;     // the update kernel leaves sum(f) of the new iterate
        }
        if (!rc && want_obj && ((j + 1) % every == 0 || j + 1 == n_iter)) {
            rc = queue_objective(st->g, &st->p, &st->w, f, y, r, st->obj_dev + 2 * (size_t)(slot0 + j + 1), s);
            have[slot0 + j + 1] = 1;
        }
    }
    return rc;
}

}  // extern "C"

int petos::run_plain(pet_os_state* st, float* f, const float* y, const float* r, int n_iter, hipStream_t s) {
    std::vector<char> none;
    return run_iterations(st, f, y, r, n_iter, false, 1, 0, s, none);
}

extern "C" {

static int ensure_obj(pet_os_state* st, int n) {
    if (st->obj_cap >= n) return PET_OS_OK;
    if (st->obj_dev) {
        PETOS_HIP(hipDeviceSynchronize());
        (void)hipFree(st->obj_dev);
        st->obj_dev = nullptr;
        st->obj_cap = 0;
    }
    if (hipMalloc(&st->obj_dev, 2 * sizeof(double) * (size_t)n) != hipSuccess)
        return fail(PET_OS_ERR_OUT_OF_MEMORY, "hipMalloc of objective slots failed");
    st->obj_cap = n;
    return PET_OS_OK;
}

static int read_objectives(pet_os_state* st, int n, const std::vector<char>& have, double* out, int first,
                           hipStream_t s) {
    std::vector<double> h(2 * (size_t)n);
    PETOS_HIP(hipMemcpyAsync(h.data(), st->obj_dev, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    PETOS_HIP(hipStreamSynchronize(s));
    for (int k = first; k < n; ++k)
        out[k - first] = have[k] ? h[2 * k] + st->p.beta * h[2 * k + 1] : std::numeric_limits<double>::quiet_NaN();
    return PET_OS_OK;
}

int pet_os_run(pet_os_state* st, float* f, const float* y, const float* r, int32_t n_iter, double* obj,
               pet_os_stream stream) {
    if (!st || !f || !y || !r) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    if (n_iter < 0) return fail(PET_OS_ERR_INVALID_ARG, "n_iter must be >= 0");
    if (obj && st->p.objective_every < 1) return fail(PET_OS_ERR_INVALID_ARG, "objective_every must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    int rc = check_state_data(st, f, y, r, s);
    if (rc) return rc;
    if (obj && (rc = ensure_obj(st, n_iter + 1))) return rc;
    std::vector<char> have((size_t)n_iter + 1, 0);
    rc = run_iterations(st, f, y, r, n_iter, obj != nullptr, std::max(1, st->p.objective_every), 0, s, have);
    if (rc) return rc;
    if (obj) {
        std::vector<double> tmp((size_t)n_iter + 1);
        if ((rc = read_objectives(st, n_iter + 1, have, tmp.data(), 0, s))) return rc;
        for (int j = 0; j < n_iter; ++j) obj[j] = tmp[j + 1];
        if (n_iter > 0 && !std::isfinite(obj[n_iter - 1])) return fail(PET_OS_ERR_NUMERIC, "objective is not finite");
    }
    return PET_OS_OK;
}

int pet_os_reconstruct(const pet_os_geom* g, const pet_os_params* p, float* f, const float* y, const float* r,
                       int32_t n_iter, double* obj, pet_os_stream stream) {
    if (!g || !p || !f || !y || !r) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    if (n_iter < 0) return fail(PET_OS_ERR_INVALID_ARG, "n_iter must be >= 0");
    if (obj && p->objective_every < 1) return fail(PET_OS_ERR_INVALID_ARG, "objective_every must be >= 1");
    pet_os_state* st = nullptr;
    int rc = pet_os_state_create(g, p, &st);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = check_state_data(st, f, y, r, s))) {
        pet_os_state_destroy(st);
        return rc;
    }
    std::vector<char> have((size_t)n_iter + 1, 0);
    if (obj) {
        rc = ensure_obj(st, n_iter + 1);
        if (!rc) rc = queue_objective(g, p, &st->w, f, y, r, st->obj_dev, s);
        have[0] = 1;
    }
    if (!rc) rc = run_iterations(st, f, y, r, n_iter, obj != nullptr, p->objective_every, 0, s, have);
    if (!rc && obj) {
        rc = read_objectives(st, n_iter + 1, have, obj, 0, s);
        if (!rc && !std::isfinite(obj[n_iter])) rc = fail(PET_OS_ERR_NUMERIC, "objective is not finite");
    }
    // the state's scratch is released below: wait for the queued work first
    if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = fail(PET_OS_ERR_DEVICE, "stream synchronize failed");
    pet_os_state_destroy(st);
    return rc;
}

int pet_os_state_seek(pet_os_state* st, int64_t k, int32_t i, double t_nest, const float* nu_frozen) {
    if (!st) return fail(PET_OS_ERR_INVALID_ARG, "state is NULL");
    if (k < 0 || i < 1 || i > st->g->d.n_subsets) return fail(PET_OS_ERR_INVALID_ARG, "bad position");
    if (!(std::isfinite(t_nest) && t_nest >= 1.0)) return fail(PET_OS_ERR_INVALID_ARG, "t_nest must be >= 1");
    if (nu_frozen && !st->w.nu_frozen) return fail(PET_OS_ERR_INVALID_ARG, "state has no nu (mode is not P1/P2)");
    if (nu_frozen) {
        PETOS_HIP(hipDeviceSynchronize());
        PETOS_HIP(hipMemcpy(st->w.nu_frozen, nu_frozen, (size_t)st->g->n_vox * sizeof(float),
                            hipMemcpyDeviceToDevice));
        st->have_frozen = 1;
    }
    st->k = k;
    st->i = i;
    st->t_nest = t_nest;
    return PET_OS_OK;
}

int pet_os_state_profile(pet_os_state* st, int32_t kernel) {
    if (!st) return fail(PET_OS_ERR_INVALID_ARG, "state is NULL");
    if (kernel < -1 || kernel > 3) return fail(PET_OS_ERR_INVALID_ARG, "kernel must be -1..3");
    st->prof_kernel = kernel;
    return PET_OS_OK;
}

int pet_os_state_profile_read(pet_os_state* st, double* total_ms, int64_t* launches) {
    if (!st) return fail(PET_OS_ERR_INVALID_ARG, "state is NULL");
    double tot = 0.0;
    for (size_t k = 0; k < st->prof_used; ++k) {
        PETOS_HIP(hipEventSynchronize(st->prof_ev[k].second));
        float ms = 0.0f;
        PETOS_HIP(hipEventElapsedTime(&ms, st->prof_ev[k].first, st->prof_ev[k].second));
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = (int64_t)st->prof_used;
    st->prof_used = 0;
    return PET_OS_OK;
}

int pet_os_nnz(const pet_os_geom* g, int32_t subset, int64_t* nnz) {
    if (!g || !nnz) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    GeomExtra* ex = extra_of(g);
    if (!ex) return fail(PET_OS_ERR_INVALID_ARG, "invalid geometry");
    if (subset < 0 || subset > g->d.n_subsets) return fail(PET_OS_ERR_INVALID_ARG, "subset out of range");
    const int n_al = subset == 0 ? g->d.n_angles : ex->subset_count[subset - 1];
    const int64_t n = (int64_t)n_al * g->n_planes * g->d.n_radial;
    Work w;
    int rc = work_alloc(g, false, &w);
    if (rc) return rc;
    float* cnt = nullptr;
    if (hipMalloc(&cnt, (size_t)n * sizeof(float)) != hipSuccess) {
        work_free(&w);
        return fail(PET_OS_ERR_OUT_OF_MEMORY, "hipMalloc failed");
    }
    Reduction red = w.red[RED_SUMY];
    FPLaunch F{};
    F.out = cnt; F.mode = FP_COUNT; F.n_al = n_al;
    F.angles = subset == 0 ? ex->all_angles : ex->subset_lists + (size_t)(subset - 1) * g->max_sub_angles;
    rc = launch_fp(g, F, nullptr);
    if (!rc) rc = launch_sum(cnt, n, red, nullptr);
    if (!rc) rc = launch_finalize(red, elem_grid(n), nullptr);
    double tot = 0.0;
    if (!rc && (hipMemcpy(&tot, red.total, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess))
        rc = fail(PET_OS_ERR_DEVICE, "read-back failed");
    (void)hipDeviceSynchronize();
    (void)hipFree(cnt);
    work_free(&w);
    if (rc) return rc;
    *nnz = (int64_t)std::llround(tot);
    return PET_OS_OK;
}

// ---------------------------------------------------------------- checkpoints

struct CkptHeader {
    char magic[8];
    uint32_t version;
    uint32_t have_frozen;
    pet_os_geom_desc desc;
    pet_os_params params;
    int64_t k;
    int32_t i;
    int32_t pad;
    double t_nest;
    int64_t n_vox;
};

int pet_os_state_export(const pet_os_state* st, void* buf, size_t* len) {
    if (!st || !len) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    const size_t nv = (size_t)st->g->n_vox;
    const size_t need = sizeof(CkptHeader) + (st->w.nu_frozen ? nv * sizeof(float) : 0);
    if (!buf) { *len = need; return PET_OS_OK; }
    if (*len < need) return fail(PET_OS_ERR_INVALID_ARG, "buffer too small");
    CkptHeader h{};
    std::memcpy(h.magic, "PETOSCK1", 8);
    h.version = 1;
    h.have_frozen = (uint32_t)st->have_frozen;
    h.desc = st->g->d;
    h.params = st->p;
    h.k = st->k;
    h.i = st->i;
    h.t_nest = st->t_nest;
    h.n_vox = (int64_t)nv;
    std::memcpy(buf, &h, sizeof(h));
    if (st->w.nu_frozen) {
        PETOS_HIP(hipDeviceSynchronize());
        PETOS_HIP(hipMemcpy((char*)buf + sizeof(h), st->w.nu_frozen, nv * sizeof(float), hipMemcpyDeviceToHost));
    }
    *len = need;
    return PET_OS_OK;
}

int pet_os_state_import(pet_os_state* st, const void* buf, size_t len) {
    if (!st || !buf) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    if (len < sizeof(CkptHeader)) return fail(PET_OS_ERR_INVALID_ARG, "checkpoint too short");
    CkptHeader h;
    std::memcpy(&h, buf, sizeof(h));
    if (std::memcmp(h.magic, "PETOSCK1", 8) != 0 || h.version != 1)
        return fail(PET_OS_ERR_INVALID_ARG, "not a pet_os checkpoint");
    if (std::memcmp(&h.desc, &st->g->d, sizeof(pet_os_geom_desc)) != 0 || h.params.mode != st->p.mode ||
        h.n_vox != st->g->n_vox)
        return fail(PET_OS_ERR_STATE_MISMATCH, "checkpoint geometry or mode differs from the state");
    const size_t nv = (size_t)st->g->n_vox;
    const bool has_nu = st->w.nu_frozen != nullptr;
    if (len < sizeof(CkptHeader) + (has_nu ? nv * sizeof(float) : 0))
        return fail(PET_OS_ERR_INVALID_ARG, "checkpoint too short");
    if (h.i < 1 || h.i > st->g->d.n_subsets || h.k < 0) return fail(PET_OS_ERR_INVALID_ARG, "bad position");
    // every value is checked before any field of the state is written
    int rc = validate_params(&h.params, st->g);
    if (rc) return rc;
    if (!(std::isfinite(h.t_nest) && h.t_nest >= 1.0)) return fail(PET_OS_ERR_INVALID_ARG, "t_nest must be >= 1");
    if (h.have_frozen > 1 || (h.have_frozen && !has_nu))
        return fail(PET_OS_ERR_INVALID_ARG, "checkpoint marks a frozen nu the state cannot hold");
    if (has_nu) {
        PETOS_HIP(hipDeviceSynchronize());
        PETOS_HIP(hipMemcpy(st->w.nu_frozen, (const char*)buf + sizeof(h), nv * sizeof(float),
                            hipMemcpyHostToDevice));
    }
    st->p = h.params;
    st->k = h.k;
    st->i = h.i;
    st->t_nest = h.t_nest;
    st->have_frozen = (int)h.have_frozen;
    st->checked_f = st->checked_y = st->checked_r = nullptr;   // U may differ: check the data again
    return PET_OS_OK;
}

}  // extern "C"
