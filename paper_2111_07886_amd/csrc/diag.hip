// diag.hip -- the gradient-consistency measure of Sec. IV-B (Fig. 2): the
// angle between two gradient images restricted to the smooth area
// I_s = {j : grad(f)_j < s mean(f)} and to the variable area
// I_v = {j : grad(f)_j > v mean(f)}, grad the Matlab-style gradient magnitude
// of the smoothness measure (Sec. III-B).
//
// One streaming pass over (h_prev, h_cur, f): 12 bytes per voxel plus the
// neighbours of f (from cache), after a pass that sums f (4 bytes per
// voxel); both walk the image in the same XCD-grouped chunks.  The area decisions are taken in FP64 from the FP32 image; the
// eight sums (<a,b>, |a|^2, |b|^2, count per area) are FP64 block partials
// added in a fixed order by one finishing block per sum, so the result is
// bitwise reproducible for a given geometry.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "devutil.h"

namespace petos {

constexpr int ANG_Q = 8;            // sums per area pair
constexpr int ANG_MAX_GRID = 2048;  // blocks of the streaming pass

// contiguous chunks of NT-voxel rows per block: at most ANG_MAX_GRID blocks,
// a multiple of 8 so that the XCD grouping below is a permutation
int angle_grid(int64_t n) {
    const int64_t rows = (n + NT - 1) / NT;
    const int64_t g = std::min<int64_t>(rows, ANG_MAX_GRID);
    return (int)std::max<int64_t>(8, (g + 7) / 8 * 8);
}

struct AngleArgs {
    const float* hp;
    const float* hc;
    const float* f;
    const double* sumf;
    double smooth_frac, var_frac;
    double inv_nx, inv_ny;      // 1/nx, 1/ny for the exact quotient below
    int chunk;                  // voxels per block, a multiple of NT
    double* part;               // [ANG_Q][grid]
};

// floor(j / d) for 0 <= j < 2^31 from an FP64 reciprocal, corrected to exact
__device__ __forceinline__ int exact_div(int j, int d, double inv_d) {
    int q = (int)((double)j * inv_d);
    if (q * d > j) --q;
    else if ((q + 1) * d <= j) ++q;
    return q;
}

// Matlab-style difference along one axis from the centre value c and the
// values lo (index - stride) and hi (index + stride): one-sided at the edges,
// central inside, zero along an axis of length 1
__device__ __forceinline__ double axis_diff(float lo, float c, float hi, int i, int n) {
    if (n < 2) return 0.0;
    if (i == 0) return (double)hi - (double)c;
    if (i == n - 1) return (double)c - (double)lo;
    return 0.5 * ((double)hi - (double)lo);
}

// Block L (XCD-grouped: the blocks of one XCD take consecutive chunks, so
// the neighbouring slices they read sit in the same L2) streams voxels
// [L chunk, (L+1) chunk) in rows of NT consecutive voxels.  The x neighbours
// f[j -/+ 1] come from the adjacent lanes (a lane at the wave's edge loads
// its own), the y and z neighbours from cache.
__global__ __launch_bounds__(NT) void k_angle_terms(GeoK g, AngleArgs A) {
    __shared__ double sh[ANG_Q * NT];
    const int n = g.nvox;
    const int G = (int)gridDim.x;
    const int L = ((int)blockIdx.x % 8) * (G / 8) + (int)blockIdx.x / 8;
    const double mean = A.sumf[0] / (double)n;
    const double ts = A.smooth_frac * mean, tv = A.var_frac * mean;
    const int sxy = g.nx * g.ny;
    const int lane = threadIdx.x & 63;
    double q[ANG_Q];
#pragma unroll
    for (int k = 0; k < ANG_Q; ++k) q[k] = 0.0;
    const int j0 = L * A.chunk;
    const int j1 = min(n, j0 + A.chunk);
    for (int jb = j0; jb < j1; jb += NT) {
        const int j = jb + (int)threadIdx.x;
        const bool ok = j < j1;
        const int jc = ok ? j : j1 - 1;
        const float c = A.f[jc];
        const float a = A.hp[jc], b = A.hc[jc];
        // x neighbours from the adjacent lanes; the wave's edge lanes load
        float xm = __shfl_up(c, 1, 64), xp = __shfl_down(c, 1, 64);
        if (lane == 0) xm = A.f[max(jc - 1, 0)];
        if (lane == 63) xp = A.f[min(jc + 1, n - 1)];
        const float ym = A.f[max(jc - g.nx, 0)], yp = A.f[min(jc + g.nx, n - 1)];
        float zm = 0.0f, zp = 0.0f;
        if (g.dim == 3) {
            zm = A.f[max(jc - sxy, 0)];
            zp = A.f[min(jc + sxy, n - 1)];
        }
        if (!ok) continue;
        const int t = exact_div(j, g.nx, A.inv_nx);
        const int ix = j - t * g.nx;
        const int iz = exact_div(t, g.ny, A.inv_ny);
        const int iy = t - iz * g.ny;
        const double gx = axis_diff(xm, c, xp, ix, g.nx);
        const double gy = axis_diff(ym, c, yp, iy, g.ny);
        const double gz = (g.dim == 3) ? axis_diff(zm, c, zp, iz, g.nz) : 0.0;
        const double gm = sqrt(gx * gx + gy * gy + gz * gz);
        const double av = (double)a, bv = (double)b;
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
    // fixed-order tree over the block's threads, the eight sums side by side
#pragma unroll
    for (int k = 0; k < ANG_Q; ++k) sh[k * NT + threadIdx.x] = q[k];
    __syncthreads();
    for (int h = NT / 2; h >= 1; h >>= 1) {
        for (int e = threadIdx.x; e < ANG_Q * h; e += NT) {
            const int k = e / h, i = e % h;
            sh[k * NT + i] += sh[k * NT + i + h];
        }
        __syncthreads();
    }
    if (threadIdx.x < ANG_Q) A.part[(long long)threadIdx.x * G + blockIdx.x] = sh[threadIdx.x * NT];
}

// partials of sum f over the same chunks as k_angle_terms (the mean of f
// must be known before the area decisions)
__global__ __launch_bounds__(NT) void k_angle_sumf(GeoK g, const float* __restrict__ f, int chunk,
                                                   double* __restrict__ part) {
    __shared__ double sh[NT / 64];
    const int n = g.nvox;
    const int G = (int)gridDim.x;
    const int L = ((int)blockIdx.x % 8) * (G / 8) + (int)blockIdx.x / 8;
    const int j0 = L * chunk;
    const int j1 = min(n, j0 + chunk);
    double acc = 0.0;
    for (int j = j0 + (int)threadIdx.x; j < j1; j += NT) acc += (double)f[j];
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// block k adds the partials of sum k
__global__ __launch_bounds__(NT) void k_angle_finish(const double* __restrict__ part, int n,
                                                     double* __restrict__ out) {
    __shared__ double sh[NT / 64];
    const int k = blockIdx.x;
    const double t = sum_partials(part + (long long)k * n, n, sh);
    if (threadIdx.x == 0) out[k] = t;
}

size_t angle_scratch_doubles(int64_t n_vox) {
    const int grid = angle_grid(n_vox);
    return (size_t)grid + 1 + (size_t)ANG_Q * grid + ANG_Q;
}

int launch_gradient_angles(const pet_os_geom* G, const float* hp, const float* hc, const float* f,
                           double smooth_frac, double var_frac, double* scratch, hipStream_t s) {
    const int grid = angle_grid(G->n_vox);
    // every index formed in the kernels (chunk starts, +-nx, quotient checks) stays in int
    if (G->n_vox > (int64_t)0x7fffffff - (int64_t)(grid + 2) * NT - 2 * (int64_t)G->d.nx * G->d.ny)
        return fail(PET_OS_ERR_INVALID_ARG, "image too large");
    double* part_f = scratch;
    double* sumf = scratch + grid;
    double* part = sumf + 1;
    double* out = part + (size_t)ANG_Q * grid;
    const int64_t rows = (G->n_vox + NT - 1) / NT;
    const int chunk = (int)((rows + grid - 1) / grid) * NT;
    hipLaunchKernelGGL(k_angle_sumf, dim3(grid), dim3(NT), 0, s, G->k, f, chunk, part_f);
    PETOS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_angle_finish, dim3(1), dim3(NT), 0, s, (const double*)part_f, grid, sumf);
    PETOS_HIP(hipGetLastError());
    AngleArgs a;
    a.hp = hp;
    a.hc = hc;
    a.f = f;
    a.sumf = sumf;
    a.smooth_frac = smooth_frac;
    a.var_frac = var_frac;
    a.inv_nx = 1.0 / (double)G->d.nx;
    a.inv_ny = 1.0 / (double)G->d.ny;
    a.chunk = chunk;
    a.part = part;
    hipLaunchKernelGGL(k_angle_terms, dim3(grid), dim3(NT), 0, s, G->k, a);
    PETOS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_angle_finish, dim3(ANG_Q), dim3(NT), 0, s, (const double*)part, grid, out);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

}  // namespace petos
