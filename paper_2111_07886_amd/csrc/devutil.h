// devutil.h -- device helpers shared by the kernel files: fixed-order FP64
// block sums and partials, and the image-space stencil of the penalty.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

namespace petos {

constexpr int NT = 256;   // threads per block everywhere

// img[idx] of an image of at most 2^30 voxels (the geometry's limit): the
// base pointer is uniform and the byte offset fits 32 bits, so the load takes
// one 32-bit address add per lane instead of 64-bit index arithmetic
__device__ __forceinline__ float img_at(const float* img, int idx) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(img) + 4u * (unsigned)idx);
}

// ------------------------------------------------------------------ reductions

// Sums across lanes by DPP moves (no LDS crossbar): the partner lane of each
// step is i^1, i^2 (quad permutations), then the mirror within each half
// row and within each row of 16.  After step k every lane of its group of
// 2^(k+1) lanes holds the group's sum (the two addends of a step are the
// same pair on both sides, so the values agree exactly).
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
constexpr int DPP_XOR1 = 0xB1;          // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;          // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <-> 7 - i within each half row
constexpr int DPP_MIRROR = 0x140;       // lane i <-> 15 - i within each row

// Sum over aligned groups of W lanes (W = 1, 4, 16 or 64; every lane of the
// wave active), valid in every lane of the group.  W = 64 adds the four row
// sums, read from lanes 0, 16, 32, 48, in row order.
template <int W, class V>
__device__ __forceinline__ V group_sum(V v) {
    static_assert(W == 1 || W == 4 || W == 16 || W == 64, "group of 1, 4, 16 or 64 lanes");
    auto step = [](V x, auto ctrl) -> V {
        constexpr int C = decltype(ctrl)::value;
        if constexpr (sizeof(V) == 8) return x + dpp_f64<C>(x);
        else return x + dpp_f32<C>(x);
    };
    if constexpr (W >= 4) {
        v = step(v, std::integral_constant<int, DPP_XOR1>{});
        v = step(v, std::integral_constant<int, DPP_XOR2>{});
    }
    if constexpr (W >= 16) {
        v = step(v, std::integral_constant<int, DPP_HALF_MIRROR>{});
        v = step(v, std::integral_constant<int, DPP_MIRROR>{});
    }
    if constexpr (W == 64) {
        if constexpr (sizeof(V) == 8) {
            V r[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                r[k] = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 16 * k),
                                        __builtin_amdgcn_readlane(__double2loint(v), 16 * k));
            v = ((r[0] + r[1]) + r[2]) + r[3];
        } else {
            V r[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) r[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16 * k));
            v = ((r[0] + r[1]) + r[2]) + r[3];
        }
    }
    return v;
}

// Sum over aligned groups of W lanes by a balanced binary tree of the lanes
// (adjacent pairs, then pairs of pairs, ...): group_sum, except that W = 64
// adds its four row sums as (r0 + r1) + (r2 + r3).
template <int W>
__device__ __forceinline__ float group_sum_balanced(float v) {
    if constexpr (W < 64) {
        return group_sum<W>(v);
    } else {
        v = group_sum<16>(v);
        float r[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) r[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16 * k));
        return (r[0] + r[1]) + (r[2] + r[3]);
    }
}

// Balanced binary tree over L leaves (L a power of two) added in leaf order:
// add() takes leaves 0, 1, ..., L-1; after the last one total() holds
// (...((l0 + l1) + (l2 + l3)) + ...).  A pending left subtree is kept per
// level, so the association is that of the full tree whatever the leaves.
template <int L>
struct LeafTree {
    static constexpr int LOG = L >= 64 ? 6 : L >= 32 ? 5 : L >= 16 ? 4 : L >= 8 ? 3 : L >= 4 ? 2 : L >= 2 ? 1 : 0;
    static_assert((1 << LOG) == L, "a power of two of leaves");
    float pend[LOG > 0 ? LOG : 1];
    float sum = 0.0f;
    __device__ __forceinline__ void add(int k, float s) {
        bool carry = true;
#pragma unroll
        for (int l = 0; l < LOG; ++l) {
            if (carry) {
                if ((k >> l) & 1) {
                    s = pend[l] + s;
                } else {
                    pend[l] = s;
                    carry = false;
                }
            }
        }
        if (carry) sum = s;
    }
};

// Sum over the wave (every lane active), valid in every lane.
__device__ __forceinline__ double wave_sum(double v) { return group_sum<64>(v); }

// Sum of v over the block in a fixed order; valid in thread 0.
__device__ inline double block_sum(double v, double* sh /* >= NT/64 */) {
    v = wave_sum(v);
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    __syncthreads();
    return t;
}

// Every thread must call: the block's sum of v goes to R.part[vblock].
__device__ __forceinline__ void write_partial(double v, Reduction R, double* sh, long long vblock) {
    double bs = block_sum(v, sh);
    if (threadIdx.x == 0) R.part[vblock] = bs;
}

// Sum of part[0..n) in index-strided order, the same in every block; the
// result is returned to every thread.  The partials were written by an
// earlier kernel in the same stream.
__device__ inline double sum_partials(const double* part, int n, double* sh) {
    __shared__ double s_tot;
    // thread t adds part[t], part[t + NT], ... in that order; eight loads are
    // issued before they are added, so they wait for memory together
    double acc = 0.0;
    for (int base = threadIdx.x; base < n; base += 8 * NT) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = (base + k * NT < n) ? part[base + k * NT] : 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += v[k];
    }
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) s_tot = t;
    __syncthreads();
    return s_tot;
}

// sum_partials in two steps for n <= NT partials: the load, issued early so
// that its latency overlaps other work, and the block sum of the loaded
// values (the same order as sum_partials: thread t holds part[t]).
__device__ __forceinline__ double partial_early(const double* part, int n) {
    return ((int)threadIdx.x < n) ? part[threadIdx.x] : 0.0;
}

__device__ inline double partials_total(double v, double* sh) {
    __shared__ double s_tot;
    double t = block_sum(v, sh);
    if (threadIdx.x == 0) s_tot = t;
    __syncthreads();
    return s_tot;
}

// One neighbour pair's term of the RDP gradient (eqn:gradRD) at f_j, without
// the factor 2: (f_j - f_k)(gamma |f_j - f_k| + f_j + 3 f_k + 2 eps) /
// (f_j + f_k + gamma |f_j - f_k| + eps)^2, as numerator and 1 / denominator
// (the hardware reciprocal, 1 ulp, in place of a correctly rounded division:
// one instruction instead of about ten per pair).  fje = f_j + eps and fj2e =
// f_j + 2 eps are formed once per voxel.
struct RdpPair {
    float num, rden;
};
__device__ __forceinline__ RdpPair rdp_pair(float fj, float fje, float fj2e, float fk, float gR) {
    const float d = fj - fk;
    const float ad = fabsf(d);
    const float den = fmaf(gR, ad, fje + fk);
    RdpPair t;
    t.num = d * fmaf(3.0f, fk, fmaf(gR, ad, fj2e));
    t.rden = __builtin_amdgcn_rcpf(den * den);
    return t;
}
__device__ __forceinline__ float rdp_term(float fj, float fk, float gR, float eps) {
    const RdpPair t = rdp_pair(fj, fj + eps, fj + 2.0f * eps, fk, gR);
    return t.num * t.rden;
}

// Matlab-style derivative along one axis at index i of n (Sec. III-B):
// one-sided at the ends, central inside, 0 on an axis of length 1.
__device__ __forceinline__ float mat_der(int i, int n, float fp, float fj, float fm) {
    if (n < 2) return 0.0f;
    if (i == 0) return fp - fj;
    if (i == n - 1) return fj - fm;
    return 0.5f * (fp - fm);
}

// RDP gradient (eqn:gradRD; in-image 8/26 neighbours, unit weights) and the
// Matlab-style gradient magnitude of Sec. III-B at one voxel of the halo tile.
template <int DIM>
__device__ __forceinline__ void stencil_at(const float* sf, int HX, int HY, int hx, int hy, int hz, int ix,
                                           int iy, int iz, const GeoK& g, float gR, float eps, float& gradR,
                                           float& gmag) {
    auto at = [&](int dx, int dy, int dz) -> float {
        return sf[((hz + dz) * HY + (hy + dy)) * HX + (hx + dx)];
    };
    const float fj = at(0, 0, 0);
    float acc = 0.0f;
    const int zr = (DIM == 3) ? 1 : 0;
    for (int dz = -zr; dz <= zr; ++dz) {
        const int z = iz + dz;
        if (z < 0 || z >= g.nz) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int y = iy + dy;
            if (y < 0 || y >= g.ny) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                const int x = ix + dx;
                if ((dx | dy | dz) == 0 || x < 0 || x >= g.nx) continue;
                acc += rdp_term(fj, at(dx, dy, dz), gR, eps);
            }
        }
    }
    gradR = 2.0f * acc;
    auto der = [&](int i, int n, int dx, int dy, int dz) -> float {
        if (n < 2) return 0.0f;
        return mat_der(i, n, at(dx, dy, dz), fj, at(-dx, -dy, -dz));
    };
    const float gx = der(ix, g.nx, 1, 0, 0);
    const float gy = der(iy, g.ny, 0, 1, 0);
    const float gz = (DIM == 3) ? der(iz, g.nz, 0, 0, 1) : 0.0f;
    gmag = sqrtf(gx * gx + gy * gy + gz * gz);
}

}  // namespace petos
