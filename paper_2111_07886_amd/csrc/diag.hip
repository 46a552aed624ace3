// diag.hip -- the gradient-consistency measure of Sec. IV-B (Fig. 2): the
// angle between two gradient images restricted to the smooth area
// I_s = {j : grad(f)_j < s mean(f)} and to the variable area
// I_v = {j : grad(f)_j > v mean(f)}, grad the Matlab-style gradient magnitude
// of the smoothness measure (Sec. III-B).
//
// One streaming pass over (h_prev, h_cur, f): 12 bytes per voxel plus the
// neighbours of f (from cache), after a pass that sums f (4 bytes per
// voxel).  The area decisions are taken in FP64 from the FP32 image; the
// eight sums (<a,b>, |a|^2, |b|^2, count per area) are FP64 block partials
// added in a fixed order by one finishing block per sum, so the result is
// bitwise reproducible for a given geometry.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "devutil.h"

namespace petos {

constexpr int ANG_Q = 8;            // sums per area pair
constexpr int ANG_MAX_GRID = 4096;  // blocks of the streaming pass (grid-stride beyond)
constexpr int ANG_U = 4;            // voxels per thread and pass: their loads are issued together

// about ANG_U voxels per thread on large images; at least min(n/NT, 1024)
// blocks so that small images still spread over the chip
int angle_grid(int64_t n) {
    const int64_t by_u = (n + (int64_t)NT * ANG_U - 1) / ((int64_t)NT * ANG_U);
    const int64_t spread = std::min<int64_t>((n + NT - 1) / NT, 1024);
    return (int)std::min<int64_t>(std::max<int64_t>(std::max(by_u, spread), 1), ANG_MAX_GRID);
}

// Grid-stride over the voxels with the stride's (x, y, z) decomposition
// carried incrementally, so that no thread divides per voxel.
struct AngleStride {
    int dx, dy, dz;     // (gridDim.x * NT) as a voxel offset in x, y, z
};

__device__ __forceinline__ void angle_advance(int& ix, int& iy, int& iz, const AngleStride& st, const GeoK& g) {
    ix += st.dx;
    iy += st.dy;
    iz += st.dz;
    if (ix >= g.nx) { ix -= g.nx; ++iy; }
    if (iy >= g.ny) { iy -= g.ny; ++iz; }
}

// one-sided at the edges, central inside, zero along an axis of length 1,
// from the loaded centre c and neighbours lo, hi
__device__ __forceinline__ double diff_of(float lo, float c, float hi, int i, int n) {
    if (n < 2) return 0.0;
    if (i == 0) return (double)hi - (double)c;
    if (i == n - 1) return (double)c - (double)lo;
    return 0.5 * ((double)hi - (double)lo);
}

__global__ __launch_bounds__(NT) void k_angle_terms(GeoK g, const float* __restrict__ hp,
                                                    const float* __restrict__ hc, const float* __restrict__ f,
                                                    const double* __restrict__ sumf, double smooth_frac,
                                                    double var_frac, AngleStride st, double* __restrict__ part) {
    __shared__ double sh[NT / 64];
    const int n = g.nvox;
    const double mean = sumf[0] / (double)n;
    const double ts = smooth_frac * mean, tv = var_frac * mean;
    const int sxy = g.nx * g.ny;
    const int stride = (int)gridDim.x * NT;
    double q[ANG_Q];
#pragma unroll
    for (int k = 0; k < ANG_Q; ++k) q[k] = 0.0;
    int j = (int)blockIdx.x * NT + (int)threadIdx.x;
    int ix = j % g.nx, iy = (j / g.nx) % g.ny, iz = j / sxy;
    for (; j < n; j += ANG_U * stride) {
        int cx[ANG_U], cy[ANG_U], cz[ANG_U];
        float c[ANG_U], xm[ANG_U], xp[ANG_U], ym[ANG_U], yp[ANG_U], zm[ANG_U], zp[ANG_U], a[ANG_U], b[ANG_U];
        // loads of the ANG_U voxels (neighbour indices clamped into the image;
        // a clamped value is never used)
#pragma unroll
        for (int u = 0; u < ANG_U; ++u) {
            const int jj = j + u * stride;
            cx[u] = ix; cy[u] = iy; cz[u] = iz;
            angle_advance(ix, iy, iz, st, g);
            const bool ok = jj < n;
            const int jc = ok ? jj : n - 1;
            c[u] = f[jc];
            xm[u] = f[max(jc - 1, 0)];
            xp[u] = f[min(jc + 1, n - 1)];
            ym[u] = f[max(jc - g.nx, 0)];
            yp[u] = f[min(jc + g.nx, n - 1)];
            zm[u] = (g.dim == 3) ? f[max(jc - sxy, 0)] : 0.0f;
            zp[u] = (g.dim == 3) ? f[min(jc + sxy, n - 1)] : 0.0f;
            a[u] = hp[jc];
            b[u] = hc[jc];
            if (!ok) cx[u] = -1;
        }
#pragma unroll
        for (int u = 0; u < ANG_U; ++u) {
            if (cx[u] < 0) continue;
            const double gx = diff_of(xm[u], c[u], xp[u], cx[u], g.nx);
            const double gy = diff_of(ym[u], c[u], yp[u], cy[u], g.ny);
            const double gz = (g.dim == 3) ? diff_of(zm[u], c[u], zp[u], cz[u], g.nz) : 0.0;
            const double gm = sqrt(gx * gx + gy * gy + gz * gz);
            const double av = (double)a[u], bv = (double)b[u];
            if (gm < ts) {
                q[0] += av * bv;
                q[1] += av * av;
                q[2] += bv * bv;
                q[3] += 1.0;
            }
            if (gm > tv) {
                q[4] += av * bv;
                q[5] += av * av;
                q[6] += bv * bv;
                q[7] += 1.0;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < ANG_Q; ++k) {
        const double bs = block_sum(q[k], sh);
        if (threadIdx.x == 0) part[(long long)k * gridDim.x + blockIdx.x] = bs;
    }
}

// block k adds the partials of sum k
__global__ __launch_bounds__(NT) void k_angle_finish(const double* __restrict__ part, int n,
                                                     double* __restrict__ out) {
    __shared__ double sh[NT / 64];
    const int k = blockIdx.x;
    const double t = sum_partials(part + (long long)k * n, n, sh);
    if (threadIdx.x == 0) out[k] = t;
}

int launch_angle_terms(const pet_os_geom* G, const float* hp, const float* hc, const float* f,
                       const double* sumf, double smooth_frac, double var_frac, double* part, int grid,
                       double* out, hipStream_t s) {
    if (grid != angle_grid(G->n_vox)) return fail(PET_OS_ERR_INVALID_ARG, "angle partials sized for another grid");
    if (G->n_vox > (int64_t)0x7fffffff - (int64_t)grid * NT * ANG_U)
        return fail(PET_OS_ERR_INVALID_ARG, "image too large");
    const int S = grid * NT, nx = G->d.nx, ny = G->d.ny;
    AngleStride st{S % nx, (S / nx) % ny, S / (nx * ny)};
    hipLaunchKernelGGL(k_angle_terms, dim3(grid), dim3(NT), 0, s, G->k, hp, hc, f, sumf, smooth_frac, var_frac, st,
                       part);
    PETOS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_angle_finish, dim3(ANG_Q), dim3(NT), 0, s, (const double*)part, grid, out);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

}  // namespace petos
