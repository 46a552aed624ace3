// kernels3d.hip -- fully-3D (span-1) forward and back projection and update.
//
// Axial shift invariance.  Rings sit at slice centres, so the LOR of plane
// (r1, d) and that of plane (r1 + 1, d) (same angle and bin) cross the same
// transaxial cells with the same lengths, one slice apart: relative to its
// first ring the axial grid coordinate of a LOR over major cell m is
// zeta(m + psi) = 1/2 + d (tau0 + tauQ (m + psi)), independent of r1, and
// slice r1 + o is crossed exactly where zeta lies in [o, o + 1).  Both
// projectors are built on that:
//
//   k_fp3    one block per (angle, bin), a wave per ring difference in
//            turn; the lanes are the first rings r1.  The 64 lanes first walk
//            64 major cells in parallel and list the (transaxial cell, slice
//            offset o, length) pieces of that stretch in LDS; then every lane
//            adds length * f[cell, slice r1 + o] for every piece.  The image
//            columns of the stretch (a copy of the image with z fastest) are
//            staged in LDS once for all ring differences, so a piece costs
//            one conflict-free LDS read of 64 consecutive slices.  The
//            Poisson ratio (or the FP64 log-likelihood term) is the
//            epilogue, as in 2D.  k_fp3_wave (one wave per (angle, bin, ring
//            difference), the same pieces read from device memory) covers
//            more than 64 rings or 32 ring differences, and the batched path.
//   k_bp3    one block per 8x8 column tile and z-range.  A lane owns one
//            column; wave v takes ring differences v, v+4, ... of each
//            staged group.  Per angle a lane finds the bins whose ray crosses
//            its column's transaxial cell and, per ring difference, the one
//            or two slice offsets o1, o1+1 with their lengths a1, a2; these
//            apply to every slice of the column:
//                acc[iz] += a1 w[r1 = iz - o1] + a2 w[r1 = iz - o1 - 1],
//            with w staged in LDS as [d][row][bin] (bins fastest; row = r1
//            relative to the block, zero outside the valid rings), in a
//            staging area sized to the geometry's footprint (dynamic LDS in
//            the single-request kernel).  The four waves' partial sums are added in a
//            fixed order and the tile's back-projection is stored.  No
//            atomics.
//   k_pen3   the image-space part of a subiteration on 32 x 8 x 8 voxel
//            tiles with an LDS halo of f: G = A_i^T w + (beta/M) grad R(f)
//            (eqn:gradRD), mu (Sec. III-B) and FP64 partials of sum mu.
//            Apart from the back-projector, it runs at the occupancy of a
//            small kernel instead of at the end of every column tile.
//   k_upd3   the update of k_update on 64 x 32 (x, z) tiles, also writing
//            the z-fastest copy through LDS; FP64 partials of sum f.
//   k_prep3  the z-fastest copy and the sum-f partials of a caller's image
//            (the same tiles and summation order as k_upd3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "devutil.h"
#include "internal.h"

namespace petos {

// ------------------------------------------------------------------ forward projection

struct FP3Args {
    const float* fz;        // image with z fastest: fz[(iy * nx + ix) * nz + iz]
    const float* y;
    const float* r;
    const float2* yr;       // null, or (y, r) bin-major (read by the staged kernel instead)
    float* out;
    const int* angles;
    int n_al;
    int mode;
    Reduction red;
};

constexpr int FP3_W = NT / 64;      // waves per block: one (angle, bin, ring difference) each
constexpr int FP3_CAP = 3 * 64;     // pieces of a stretch of 64 major cells (<= 3 per cell)

struct Piece {
    int off;      // slice o of the voxel's column: in the z-fastest copy, or in the staged columns
    float len;    // 3D length
};

__host__ __device__ inline long long fp3_items(int n_al, int n_radial, int max_rd, int n_rings) {
    return (long long)n_al * n_radial * (2 * max_rd + 1) * ((n_rings + 63) / 64);
}

// memory ordering of LDS traffic between the lanes of one wave
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ void fp3_body(const GeoK& g, const FP3Args& A, long long vblock) {
    __shared__ Piece s_pc[FP3_W][FP3_CAP];
    __shared__ double s_red[NT / 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int D = g.max_rd, ND = 2 * D + 1, Nr = g.n_radial, R = g.n_rings;
    const int nch = (R + 63) / 64;
    const long long item = vblock * FP3_W + wave;
    bool live = item < fp3_items(A.n_al, Nr, D, R);
    int ch = 0, di = 0, b = 0, al = 0;
    if (live) {
        // fewer than 2^31 items per pass (checked with the descriptor): the
        // wave-uniform decode in 32-bit integers
        int t = (int)item;
        ch = t % nch;
        t /= nch;
        di = t % ND;
        t /= ND;
        b = t % Nr;
        al = t / Nr;
    }
    const int d = di - D;
    const int r1lo = max(0, -d), r1hi = min(R - 1, R - 1 - d);
    const int r1 = r1lo + ch * 64 + lane;
    live = live && (r1lo + ch * 64 <= r1hi);
    const bool lane_ok = live && r1 <= r1hi;
    const bool counting = A.mode == FP_COUNT;

    float acc = 0.0f;
    int a = 0;
    if (live) {
        a = A.angles[al];
        const AngleK& AK = g.ang[a];
        const TxRay tx = tx_ray(g, AK, b);
        const int n_major = tx.row_major ? g.ny : g.nx;
        const int n_minor = tx.row_major ? g.nx : g.ny;
        int m0, m1;
        major_range(tx, n_major, n_minor, m0, m1);
        const ZBin zb = z_bin(g, AK, b);
        const double zeta0 = __fma_rn((double)d, zb.tau0, 0.5);
        const double Qz = (double)d * zb.tauQ;
        const double invQz = (d == 0) ? 0.0 : g.inv_d[di] * zb.inv_tauQ;
        const double Lk = tx.L * g.kappa[(long long)b * ND + di];
        const int qstep = (tx.Q >= 0.0) ? 1 : -1;
        const int zstep = (Qz >= 0.0) ? 1 : -1;
        const float Lkf = (float)Lk, invQf = (float)tx.invQ, invQzf = (float)invQz;
        // a LOR between rings r1 and r1 + d stays in slices r1 + [min(0,d), max(0,d)]
        const int olo = min(0, d), ohi = max(0, d);
        // offset of voxel (minor cell c, major cell m, slice o) in the
        // z-fastest copy: m ms + c cs + o
        const int cs = tx.row_major ? g.nz : g.nx * g.nz;
        const int ms = tx.row_major ? g.nx * g.nz : g.nz;
        const int qcs = qstep * cs;
        for (int mb = m0; mb <= m1; mb += 64) {
            // (1) the lane's major cell: up to three pieces.  Over the cell
            // the ray's transaxial minor coordinate runs from gm to gm + Q
            // and its axial coordinate from zm to zm + Qz; each crosses at
            // most one edge, at the fraction tx or tz of the cell's length
            // (decided in FP64, the fractions formed in FP32 from the FP64
            // distances).  The pieces, in order along the ray: up to the
            // first crossing in (c0, o0), then up to the second in the cell
            // the first crossing leads to, then in (c0 + qstep, o0 + zstep).
            // (lanes past the last cell repeat it and keep no piece: no branch)
            const int m = min(mb + lane, m1);
            int off[3];
            float len[3];
            int present;
            {
                const double gm = __fma_rn(tx.Q, (double)m, tx.P);
                const double zm = __fma_rn(Qz, (double)m, zeta0);
                const double cf = floor(gm), of = floor(zm);
                const int c0 = (int)cf, o0 = (int)of;
                const double ce = (tx.Q >= 0.0) ? cf + 1.0 : cf;    // the edges the ray may cross
                const double oe = (Qz >= 0.0) ? of + 1.0 : of;
                const double ge = gm + tx.Q, ze = zm + Qz;
                const bool xc = (tx.Q >= 0.0) ? (ge > ce) : (ge < ce);
                const bool zc = (Qz >= 0.0) ? (ze > oe) : (ze < oe);
                const float tX = xc ? (float)(ce - gm) * invQf : 1.0f;
                const float tZ = zc ? (float)(oe - zm) * invQzf : 1.0f;
                const bool x_first = tX <= tZ;
                const float t1 = fminf(tX, tZ), t2 = fmaxf(tX, tZ);
                const int c1 = c0 + qstep, o1 = o0 + zstep;
                const int pc1 = x_first ? c1 : c0, po1 = x_first ? o0 : o1;
                const float f0 = t1, f1 = t2 - t1, f2 = 1.0f - t2;
                // a piece is kept when it exists, has a length and lies in the
                // image and in the LOR's slices; offset = m ms + c cs + o
                // (a cell index is in [0, n_minor) when it is below n_minor as unsigned)
                const bool v0 = f0 > 0.0f && (unsigned)c0 < (unsigned)n_minor && o0 >= olo && o0 <= ohi;
                const bool v1 = (xc || zc) && f1 > 0.0f && (unsigned)pc1 < (unsigned)n_minor && po1 >= olo && po1 <= ohi;
                const bool v2 = xc && zc && f2 > 0.0f && (unsigned)c1 < (unsigned)n_minor && o1 >= olo && o1 <= ohi;
                // 24-bit signed products (full-rate multiplies): the descriptor
                // check keeps the strides nx nz and ny nz below 2^23, and the
                // cell indices lie within a cell or two of the image
                const int offm = __mul24(m, ms);
                const int c0s = __mul24(c0, cs), c1s = c0s + qcs;
                off[0] = offm + c0s + o0;
                off[1] = offm + (x_first ? c1s : c0s) + po1;
                off[2] = offm + c1s + o1;
                len[0] = Lkf * f0;
                len[1] = Lkf * f1;
                len[2] = Lkf * f2;
                present = mb + lane <= m1 ? (v0 ? 1 : 0) | (v1 ? 2 : 0) | (v2 ? 4 : 0) : 0;
            }
            // (2) compact the pieces of the 64 cells, in cell order, into LDS
            // (each lane has 0..3 pieces: the exclusive prefix of the counts
            // is the sum over their two bits of 2^k x the lanes below with
            // bit k set, counted from the wave's ballots)
            const int cnt = __popc(present);
            int pos = 0, total = 0;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const unsigned long long m = __ballot((cnt >> k) & 1);
                pos += __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u)) << k;
                total += __popcll(m) << k;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (present & (1 << k)) {
                    s_pc[wave][pos] = Piece{off[k], len[k]};
                    ++pos;
                }
            }
            wave_lds_sync();
            // (3) every lane (first ring r1) applies every piece
            if (lane_ok) {
                if (counting) {
                    acc += (float)total;    // pieces of the LOR
                } else {
                    // eight pieces' image loads in flight per lane (sixteen cost
                    // more in occupancy than they hide in latency)
#pragma unroll 8
                    for (int j = 0; j < total; ++j) {
                        const Piece p = s_pc[wave][j];
                        acc = fmaf(p.len, img_at(A.fz, p.off + r1), acc);
                    }
                }
            }
            wave_lds_sync();
        }
    }

    double term = 0.0;
    if (lane_ok) {
        const int plane = g.plane_base[di] + (r1 - r1lo);
        const long long nat = ((long long)plane * g.n_angles + a) * Nr + b;
        const long long ray = ((long long)al * g.n_planes + plane) * Nr + b;
        if (A.mode == FP_RATIO) {
            A.out[ray] = 1.0f - A.y[nat] / (acc + A.r[nat]);
        } else if (A.mode == FP_EM) {
            A.out[ray] = A.y[nat] / (acc + A.r[nat]);
        } else if (A.mode == FP_COUNT || A.mode == FP_COMPACT) {
            A.out[ray] = acc;
        } else if (A.mode == FP_PLAIN) {
            A.out[nat] = acc;
        } else {
            const double q = (double)acc;
            term = q - (double)A.y[nat] * log(q + (double)A.r[nat]);
        }
    }
    if (A.mode == FP_OBJECTIVE) write_partial(term, A.red, s_red, vblock);
}

// Workgroups are dealt to the 8 XCDs round-robin by block index; renumber
// them so that each XCD (and its L2) takes a contiguous run of work: the ring
// differences of one bin read the same image columns, neighbouring tiles the
// same sinogram rows.  The grid is 8 * ceil(n / 8) blocks.
__device__ __forceinline__ long long xcd_block(long long block, long long n) {
    const long long per = (n + 7) / 8;
    return (block % 8) * per + block / 8;
}

// per-wave items (any ring count and ring difference range)
__global__ __launch_bounds__(NT) void k_fp3_wave(GeoK g, FP3Args A, long long n_blocks) {
    const long long vb = xcd_block(blockIdx.x, n_blocks);
    if (vb >= n_blocks) return;
    fp3_body(g, A, vb);
}

// Forward projection with the ray's image columns staged in LDS, used when
// the rings fit one chunk (nz <= 64) and there are at most 32 ring
// differences.  One block takes one (angle, bin); its eight waves take the
// ring differences w, w + 8, w + 16, w + 24.  The transaxial path of the ray
// is the same for every ring difference, so for each stretch of 64 major
// cells the columns it can enter (minor cells c0 and c0 + qstep of each major
// cell, all nz slices) are copied to LDS once, and every ring difference
// reads its pieces there instead of from device memory, where each piece
// cost a 256-byte wave load through the vector L1.  Pieces, their order and
// their arithmetic are those of fp3_body, so the results agree bit for bit.
constexpr int FPS_NT = 512;
constexpr int FPS_W = FPS_NT / 64;      // waves per block
constexpr int FPS_DPW = 4;              // ring differences per wave at most
constexpr int FPS_ZS = 64;              // floats per staged column (nz <= 64)
constexpr int FPS_SLOTS = 128;          // staged columns of a stretch: slot 2k (c0) and 2k + 1 (c0 + qstep) of cell mb + k

__host__ __device__ inline bool fp3_staged(int nz, int max_rd) {
    return nz <= FPS_ZS && 2 * max_rd + 1 <= FPS_W * FPS_DPW;
}

// Copy a stretch's columns into s_col: slot 2k holds minor cell c0 of major
// cell mb + k, slot 2k + 1 its neighbour c0 + qstep, all nz slices; columns
// outside the image or past m1 stay unwritten (no piece refers to them).
// With nz a multiple of 4 (column starts 16-byte aligned) a wave instruction
// copies four columns, sixteen lanes of 16 bytes each; else one column, a
// slice per lane.  Returns without waiting.
__device__ __forceinline__ void fp3s_stage(const float* fz, float* s_col, const TxRay& tx, int mb, int m1, int n_minor,
                                           int qstep, int ms, int cs, int nz, int wave, int lane) {
    if ((nz & 3) == 0) {
        const int sub = lane >> 4, q = (lane & 15) * 4;
        for (int s0 = wave * 4; s0 < FPS_SLOTS; s0 += FPS_W * 4) {
            const int slot = s0 + sub, m = mb + (slot >> 1);
            bool ok = m <= m1 && q < nz;
            int src = 0;
            if (ok) {
                const int c = (int)floor(__fma_rn(tx.Q, (double)m, tx.P)) + ((slot & 1) ? qstep : 0);
                ok = (unsigned)c < (unsigned)n_minor;
                src = __mul24(m, ms) + __mul24(c, cs) + q;
            }
            if (ok)
                __builtin_amdgcn_global_load_lds(fz + src, (__attribute__((address_space(3))) void*)(s_col + s0 * FPS_ZS),
                                                 16, 0, 0);
        }
    } else {
        for (int slot = wave; slot < FPS_SLOTS; slot += FPS_W) {
            const int m = mb + (slot >> 1);
            bool ok = m <= m1 && lane < nz;
            int src = 0;
            if (ok) {
                const int c = (int)floor(__fma_rn(tx.Q, (double)m, tx.P)) + ((slot & 1) ? qstep : 0);
                ok = (unsigned)c < (unsigned)n_minor;
                src = __mul24(m, ms) + __mul24(c, cs) + lane;
            }
            if (ok)
                __builtin_amdgcn_global_load_lds(fz + src, (__attribute__((address_space(3))) void*)(s_col + slot * FPS_ZS),
                                                 4, 0, 0);
        }
    }
}

__device__ void fp3s_body(const GeoK& g, const FP3Args& A, long long vblock) {
    __shared__ __attribute__((aligned(16))) float s_col[FPS_SLOTS * FPS_ZS];
    // the pieces as two arrays: length, and the byte offset (off + 16) * 4 of
    // slice o of the staged column, which fits 16 bits (o >= -15 here), so
    // that the broadcast reads of a batch of pieces move 6 bytes a piece
    __shared__ __attribute__((aligned(16))) unsigned short s_po[FPS_W][FP3_CAP];
    __shared__ __attribute__((aligned(16))) float s_pl[FPS_W][FP3_CAP];
    __shared__ double s_red[FPS_W];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int D = g.max_rd, ND = 2 * D + 1, Nr = g.n_radial, R = g.n_rings, nz = g.nz;
    const int b = (int)(vblock % Nr), al = (int)(vblock / Nr);
    const bool counting = A.mode == FP_COUNT;
    const int a = A.angles[al];
    const AngleK& AK = g.ang[a];
    // the ray's FP64 constants live in LDS (read where used) rather than in
    // registers across the loops
    __shared__ double s_ray[5];    // P, L, tau0, tauQ, inv_tauQ
    const TxRay tx0 = tx_ray(g, AK, b);
    const ZBin zb0 = z_bin(g, AK, b);
    if (threadIdx.x == 0) {
        s_ray[0] = tx0.P;
        s_ray[1] = tx0.L;
        s_ray[2] = zb0.tau0;
        s_ray[3] = zb0.tauQ;
        s_ray[4] = zb0.inv_tauQ;
    }
    TxRay tx = tx0;
    const int n_major = tx.row_major ? g.ny : g.nx;
    const int n_minor = tx.row_major ? g.nx : g.ny;
    int m0, m1;
    major_range(tx, n_major, n_minor, m0, m1);
    const int qstep = (tx.Q >= 0.0) ? 1 : -1;
    const float invQf = (float)tx.invQ;
    // offset of voxel (minor cell c, major cell m, slice o) in the z-fastest
    // copy: m ms + c cs + o (24-bit products, as in fp3_body)
    const int cs = tx.row_major ? nz : g.nx * nz;
    const int ms = tx.row_major ? g.nx * nz : nz;

    float acc[FPS_DPW];
#pragma unroll
    for (int j = 0; j < FPS_DPW; ++j) acc[j] = 0.0f;

    for (int mb = m0; mb <= m1; mb += 64) {
        // (1) stage the stretch's columns (counting reads no image, and is
        // given none)
        __syncthreads();    // the previous stretch's columns are read no more (and s_ray is written)
        tx.P = s_ray[0];
        if (!counting) fp3s_stage(A.fz, s_col, tx, mb, m1, n_minor, qstep, ms, cs, nz, wave, lane);
        __builtin_amdgcn_s_waitcnt(0);      // this wave's copies have landed
        __syncthreads();                    // and every other wave's

        // (2) the transaxial part of the lane's major cell, shared by the
        // wave's ring differences (lanes past the last cell repeat it and
        // keep no piece)
        const int mraw = mb + lane;
        const int m = min(mraw, m1);
        const double gm = __fma_rn(tx.Q, (double)m, tx.P);
        const double cf = floor(gm);
        const int c0 = (int)cf, c1 = c0 + qstep;
        const double ce = (tx.Q >= 0.0) ? cf + 1.0 : cf;
        const double ge = gm + tx.Q;
        const bool xc = (tx.Q >= 0.0) ? (ge > ce) : (ge < ce);
        const float tX = xc ? (float)(ce - gm) * invQf : 1.0f;
        const bool in0 = (unsigned)c0 < (unsigned)n_minor, in1 = (unsigned)c1 < (unsigned)n_minor;
        const int sl0 = 2 * (m - mb) * FPS_ZS, sl1 = sl0 + FPS_ZS;    // LDS offsets of the two columns

#pragma unroll
        for (int j = 0; j < FPS_DPW; ++j) {
            const int di = wave + FPS_W * j;
            if (di >= ND) break;
            const int d = di - D;
            // (3) the axial part and the pieces, as in fp3_body
            const double zeta0 = __fma_rn((double)d, s_ray[2], 0.5);
            const double Qz = (double)d * s_ray[3];
            const double invQz = (d == 0) ? 0.0 : g.inv_d[di] * s_ray[4];
            const float Lkf = (float)(s_ray[1] * g.kappa[(long long)b * ND + di]), invQzf = (float)invQz;
            const int zstep = (Qz >= 0.0) ? 1 : -1;
            const int olo = min(0, d), ohi = max(0, d);
            const double zm = __fma_rn(Qz, (double)m, zeta0);
            const double of = floor(zm);
            const int o0 = (int)of, o1 = o0 + zstep;
            const double oe = (Qz >= 0.0) ? of + 1.0 : of;
            const double ze = zm + Qz;
            const bool zc = (Qz >= 0.0) ? (ze > oe) : (ze < oe);
            const float tZ = zc ? (float)(oe - zm) * invQzf : 1.0f;
            const bool x_first = tX <= tZ;
            const float t1 = fminf(tX, tZ), t2 = fmaxf(tX, tZ);
            const int po1 = x_first ? o0 : o1;
            const bool pin1 = x_first ? in1 : in0;
            const float f0 = t1, f1 = t2 - t1, f2 = 1.0f - t2;
            const bool v0 = f0 > 0.0f && in0 && o0 >= olo && o0 <= ohi;
            const bool v1 = (xc || zc) && f1 > 0.0f && pin1 && po1 >= olo && po1 <= ohi;
            const bool v2 = xc && zc && f2 > 0.0f && in1 && o1 >= olo && o1 <= ohi;
            const int off[3] = {sl0 + o0, (x_first ? sl1 : sl0) + po1, sl1 + o1};
            const float len[3] = {Lkf * f0, Lkf * f1, Lkf * f2};
            const int present = mraw <= m1 ? (v0 ? 1 : 0) | (v1 ? 2 : 0) | (v2 ? 4 : 0) : 0;
            // (4) compact the pieces in cell order (as in fp3_body)
            const int cnt = __popc(present);
            int pos = 0, total = 0;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const unsigned long long bm = __ballot((cnt >> k) & 1);
                pos += __builtin_amdgcn_mbcnt_hi((unsigned)(bm >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bm, 0u)) << k;
                total += __popcll(bm) << k;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (present & (1 << k)) {
                    s_po[wave][pos] = (unsigned short)((off[k] + 16) * 4);
                    s_pl[wave][pos] = len[k];
                    ++pos;
                }
            }
            wave_lds_sync();
            // (5) every lane (first ring r1) applies every piece from LDS
            const int r1 = max(0, -d) + lane;
            if (r1 <= min(R - 1, R - 1 - d)) {
                if (counting) {
                    acc[j] += (float)total;
                } else {
                    // byte address of slice o of a piece's column for this
                    // lane: colb + (o + 16) * 4 with colb at ring r1 - 16
                    const char* colb = reinterpret_cast<const char*>(s_col) + 4 * r1 - 64;
                    int k = 0;
                    for (; k + 8 <= total; k += 8) {
                        // eight pieces: offsets in one 16-byte read, lengths in
                        // two, the eight column reads in flight together
                        const uint4 po4 = *reinterpret_cast<const uint4*>(&s_po[wave][k]);
                        const float4 l0 = *reinterpret_cast<const float4*>(&s_pl[wave][k]);
                        const float4 l1 = *reinterpret_cast<const float4*>(&s_pl[wave][k + 4]);
                        const unsigned po[4] = {po4.x, po4.y, po4.z, po4.w};
                        const float ln[8] = {l0.x, l0.y, l0.z, l0.w, l1.x, l1.y, l1.z, l1.w};
                        float x[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const unsigned ob = (u & 1) ? (po[u >> 1] >> 16) : (po[u >> 1] & 0xffffu);
                            x[u] = *reinterpret_cast<const float*>(colb + ob);
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u) acc[j] = fmaf(ln[u], x[u], acc[j]);
                    }
                    for (; k < total; ++k)
                        acc[j] = fmaf(s_pl[wave][k], *reinterpret_cast<const float*>(colb + s_po[wave][k]), acc[j]);
                }
            }
            wave_lds_sync();
        }
    }

    // (6) the rays' outputs, as in fp3_body
    double term = 0.0;
#pragma unroll
    for (int j = 0; j < FPS_DPW; ++j) {
        const int di = wave + FPS_W * j;
        if (di >= ND) break;
        const int d = di - D;
        const int r1lo = max(0, -d), r1 = r1lo + lane;
        if (r1 > min(R - 1, R - 1 - d)) continue;
        const int plane = g.plane_base[di] + (r1 - r1lo);
        const long long nat = ((long long)plane * g.n_angles + a) * Nr + b;
        const long long ray = ((long long)al * g.n_planes + plane) * Nr + b;
        if (A.mode == FP_RATIO || A.mode == FP_EM) {
            // y and r of the ray: from the bin-major copy the lanes' planes
            // are consecutive (one 512-byte wave load), in the natural layout
            // they lie n_angles * n_radial apart
            float yv, rv;
            if (A.yr != nullptr) {
                const float2 v = A.yr[((long long)a * Nr + b) * g.n_planes + plane];
                yv = v.x;
                rv = v.y;
            } else {
                yv = A.y[nat];
                rv = A.r[nat];
            }
            A.out[ray] = A.mode == FP_RATIO ? 1.0f - yv / (acc[j] + rv) : yv / (acc[j] + rv);
        } else if (A.mode == FP_COUNT || A.mode == FP_COMPACT) {
            A.out[ray] = acc[j];
        } else if (A.mode == FP_PLAIN) {
            A.out[nat] = acc[j];
        } else {
            const double q = (double)acc[j];
            term += q - (double)A.y[nat] * log(q + (double)A.r[nat]);
        }
    }
    if (A.mode == FP_OBJECTIVE) write_partial(term, A.red, s_red, vblock);
}

// six waves per SIMD: 44 KB of LDS per block lets three blocks share a CU
__global__ __launch_bounds__(FPS_NT, 6) void k_fp3(GeoK g, FP3Args A, long long n_blocks) {
    const long long vb = xcd_block(blockIdx.x, n_blocks);
    if (vb >= n_blocks) return;
    fp3s_body(g, A, vb);
}

// ------------------------------------------------------------------ back projection

// The image-space part of a 3D subiteration: grad R(f) (eqn:gradRD, 26
// in-image neighbours), either added after the back-projection b = A_i^T w
// as G = b + (beta/M) grad R(f) in place over b, or (gradR given) stored on
// its own for the update to add, so that it can run in the back-projector's
// launch; with want_mu the smoothness measure mu = max(0.01, |grad f| /
// mean f) (Sec. III-B) with the block's FP64 partial of sum mu.  One block
// per 32 (x) x 8 (y) x 8 (z) voxels (a thread per (x, y), eight slices
// each); f with a one-voxel halo in LDS.
constexpr int PEN3_X = 32, PEN3_Y = 8, PEN3_Z = 8;
constexpr int PEN3_HALO = (PEN3_X + 2) * (PEN3_Y + 2) * (PEN3_Z + 2);   // floats of the halo tile

struct Pen3Args {
    const float* f;
    float* G;                // in: b, out: G (gradR null)
    float* gradR;            // non-null: grad R(f) goes here and G is left alone
    float* mu;
    int want_mu;
    float beta_over_M, gamma_R, eps;
    const double* part_f;    // partials of sum f of the entering iterate (mean f)
    int n_part_f;
    Reduction red_mu;
};

__host__ __device__ inline int pen3_tiles(int n, int t) { return (n + t - 1) / t; }

__device__ void pen3_body(const GeoK& g, const Pen3Args& A, int vblock, float* s_f, double* s_red);


struct BP3Args {
    const float* w;          // null => unit weights (sensitivity)
    long long w_sp, w_sa;    // w index = plane * w_sp + angle_index * w_sa + b
    int w_natural;           // angle_index = natural angle (1) or position in the list (0)
    const int* angles;
    int n_al;
    float* out;              // the back-projection A_i^T w
    int nb;                  // staged bins per angle
    int zb;                  // slices per block: 16, 32 or 64
    int rw;                  // staged rows per (ring difference, bin)
    int dpg;                 // ring differences staged together: 4 or 8
    int half;                // floats of one staging buffer (>= dpg * row stride * rw)
    int lds;                 // floats of the staging area (two buffers; the finish reuses it)
    Pen3Args pen;            // the penalty blocks' arguments (gradR set) when n_pen > 0
    int n_pen;
};

constexpr int BP3_T = 8;         // columns per tile side
constexpr int BP3_ZMAX = 64;
constexpr int BP3_HMAX = 2;      // candidate bins of a column handled per pass
constexpr int BP3_LDS = 12288;   // floats of the largest staging area (48 KB)
constexpr int BP3_MAXND = 63;    // ring differences -31..31

// LDS row stride of the staged footprint: 20 bins (3 rows per wave load) or 40
__host__ __device__ inline int bp3_nbs(int nb) { return nb <= 20 ? 20 : 40; }
// The single-request kernel also has a 16-bin stride (one wave instruction
// then stages 16 rows, every lane used)
__host__ __device__ inline int bp3_nbs_single(int nb) { return nb <= 16 ? 16 : bp3_nbs(nb); }

// LDS shared by the back-projector's phases (declared once per kernel); the
// staging area is separate (dynamic in the single-request kernel, sized to
// the geometry's footprint).  Angles are taken in chunks of BP3_AMAX whose
// tile windows are found together, one thread per angle.
constexpr int BP3_AMAX = 16;
struct BP3Shared {
    int pbase[BP3_MAXND];    // plane of ring r1 = 0 of ring difference index di (plane_base - first ring)
    int ang[BP3_AMAX];       // the chunk's angles
    int blo[BP3_AMAX], nb[BP3_AMAX];    // the tile's staged bins of each angle
    double tau[BP3_AMAX][2];            // the tile's tau range of each angle
    double red[NT / 64];
};

// Slice-offset range (+1 margin) over the tile of ring difference d, from the
// tile's tau range of the angle.
__device__ __forceinline__ void bp3_orange(double tau0, double tau1, int d, int& omin, int& omax) {
    const double za = 0.5 + (double)d * tau0, zc = 0.5 + (double)d * tau1;
    omin = (int)floor(fmin(za, zc)) - 1;
    omax = (int)floor(fmax(za, zc)) + 1;
}

// acc[i] += a1 w(r1 = iz - o1) + a2 w(r1 = iz - o1 - 1) for the ZB slices
// of the block, with sp[(i + 1) * NBS] holding w(r1 = z0 + i - o1): the row
// of offset o1 + 1 for slice i is the row of offset o1 for slice i - 1, so
// the second term reuses the value loaded for the slice below and a column
// whose piece crosses a slice boundary costs one FMA more per slice, no LDS
// read (a2 = 0 elsewhere).  Loads go in batches of 16 to bound the live
// registers.
template <int ZB, int NBS>
__device__ __forceinline__ void bp3_apply(float (&acc)[BP3_ZMAX], const float* sp, float a1, float a2) {
    float below = sp[0];
#pragma unroll
    for (int c = 0; c < ZB; c += 16) {
        float v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = sp[(c + i + 1) * NBS];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            acc[c + i] = fmaf(a1, v[i], acc[c + i]);
            acc[c + i] = fmaf(a2, i == 0 ? below : v[i - 1], acc[c + i]);
        }
        below = v[15];
        __builtin_amdgcn_sched_barrier(0);
    }
}

// After all angles: add the four waves' partial sums in wave order into
// s_fin[lz][column] (top of the LDS area) and store the tile's
// back-projection.  The penalty gradient, mu and G of a subiteration follow
// in k_pen3.
template <int ZB>
__device__ void bp3_finish(const GeoK& g, const BP3Args& A, float (&acc)[BP3_ZMAX], float* s_w, int tx0, int ty0,
                           int z0) {
    constexpr int QS = ZB / 4;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float* s_fin = s_w + (A.lds - ZB * 64);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < QS; ++i) s_w[(wave * QS + i) * 64 + lane] = acc[q * QS + i];
        __syncthreads();
        if (wave == q) {
#pragma unroll 4
            for (int i = 0; i < QS; ++i) {
                float s = s_w[i * 64 + lane];
                s += s_w[(QS + i) * 64 + lane];
                s += s_w[(2 * QS + i) * 64 + lane];
                s += s_w[(3 * QS + i) * 64 + lane];
                s_fin[(q * QS + i) * 64 + lane] = s;
            }
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ZB * 64; e += NT) {
        const int c = e & 63, lz = e >> 6;
        const int ix = tx0 + (c & 7), iy = ty0 + (c >> 3), iz = z0 + lz;
        if (ix < g.nx && iy < g.ny && iz < g.nz) A.out[((long long)iz * g.ny + iy) * g.nx + ix] = s_fin[e];
    }
}

// Stage w of the calling wave's ring differences of group dg (slots ds =
// wave, wave + 4, ... < dpg: the ones it gathers) into buf as [ds][row][bin],
// row r of slot ds holding r1 = z0 - omax(d) + r - 1 (row 0 and invalid
// rings: zeros; unit weights: ones).  NBS is the row stride.  Per ring
// difference the rows of valid rings form one range [rlo, rhi]: the rows
// outside it are zero-filled by the wave, the range is copied straight from
// device memory into LDS, each lane moving four consecutive bins (16 bytes),
// 64 / (NBS / 4) rows per wave instruction; a caller's natural-layout w
// (whose last row may end at its allocation) moves one bin per lane.  A
// slot's rows are written and read by the same wave, so no block barrier
// orders them: the wave waits for its own loads.  Returns without waiting.
template <int NBS>
__device__ __forceinline__ void bp3_stage(const GeoK& g, const BP3Args& A, const BP3Shared& sh, float* buf, int dg,
                                          int z0, int aidx, int blo, int nbv, double tau0, double tau1) {
    constexpr int CPR = NBS / 4;                    // 16-byte chunks per row
    constexpr int RPI4 = 64 / CPR;                  // rows per wave instruction, 16-byte lanes
    constexpr int RPI1 = 64 / NBS;                  // rows per wave instruction, 4-byte lanes
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int D = g.max_rd, ND = 2 * D + 1, R = g.n_rings, rw = A.rw, dpg = A.dpg;
    const bool wide = !A.w_natural;
    // a lane's element of a chunk: row (chunk start + sub), bins from blo +
    // col; its offset from the chunk's first element is the same in every chunk
    const int sub = wide ? lane / CPR : lane / NBS;
    const int col = wide ? 4 * (lane - sub * CPR) : lane - sub * NBS;
    const int rpi = wide ? RPI4 : RPI1;
    const bool lane_ok = sub < rpi && col < nbv;
    const long long lane_off = (long long)sub * A.w_sp + col;
    for (int ds = wave; ds < dpg; ds += 4) {
        const int di = dg + ds;
        if (di >= ND) break;
        const int d = di - D;
        const int lo = max(0, -d), hi = min(R - 1, R - 1 - d);
        int omn, om;
        bp3_orange(tau0, tau1, d, omn, om);
        const int r1_row0 = z0 - om - 1;            // ring r1 of row 0
        // rows of valid rings (row 0 stays zero): [rlo, rhi], possibly empty
        const int rlo = max(1, lo - r1_row0), rhi = min(rw - 1, hi - r1_row0);
        float* bd = buf + ds * rw * NBS;
        // zeros below the range ([0, nzlo)) and above it ([top0, rw)), 16 bytes a lane
        const int nzlo = min(rlo, rw), top0 = max(rhi, rlo - 1) + 1, nzhi = max(rw - top0, 0);
        for (int e = lane; e < (nzlo + nzhi) * CPR; e += 64) {
            const int rr = e / CPR, cc = e - rr * CPR;
            const int row = rr < nzlo ? rr : top0 + (rr - nzlo);
            *reinterpret_cast<float4*>(bd + row * NBS + 4 * cc) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        if (rhi < rlo) continue;
        if (A.w == nullptr) {
            for (int e = lane; e < (rhi - rlo + 1) * NBS; e += 64) bd[rlo * NBS + e] = 1.0f;
            continue;
        }
        // (uniform) element of row rlo, bin blo: plane pbase[di] + r1
        const float* wr = A.w + ((long long)sh.pbase[di] + r1_row0 + rlo) * A.w_sp + (long long)aidx * A.w_sa + blo;
        const long long wstep = (long long)rpi * A.w_sp;
        if (wide) {
            // bins past the window (up to blo + nbv + 2) may be read: they lie
            // in the next row or in the scratch's padding, and are never gathered
            for (int r0 = rlo; r0 <= rhi; r0 += RPI4, wr += wstep) {
                if (lane_ok && r0 + sub <= rhi)
                    __builtin_amdgcn_global_load_lds(wr + lane_off, (__attribute__((address_space(3))) void*)(bd + r0 * NBS),
                                                     16, 0, 0);
            }
        } else {
            for (int r0 = rlo; r0 <= rhi; r0 += RPI1, wr += wstep) {
                if (lane_ok && r0 + sub <= rhi)
                    __builtin_amdgcn_global_load_lds(wr + lane_off, (__attribute__((address_space(3))) void*)(bd + r0 * NBS),
                                                     4, 0, 0);
            }
        }
    }
}

// Hits of one column for one angle: the transaxial psi-interval [ax, bx] of
// the column's cell in major cell m, for every bin b0..b1 whose ray crosses it,
// kept as tau at its smaller end (t0) and its tau extent (dt >= 0, from the
// FP64 difference), the transaxial length and the axial slope ck =
// ring_pitch / (2 h_b) per unit ring difference.  Over ring difference d the
// piece runs axially over zeta in 1/2 + d [t0, t0 + dt].  Slots take hits
// first .. first + BP3_HMAX - 1 (in bin order); returns the number of hits.
struct Hits {
    int b[BP3_HMAX];
    float t0[BP3_HMAX], dt[BP3_HMAX];
    float L[BP3_HMAX], ck[BP3_HMAX];
    bool v[BP3_HMAX];
};


// One candidate bin b of col_hits, with h and 1 / (2 h) of its table row
// already loaded.
__device__ __forceinline__ void col_hit_one(const GeoK& g, const AngleK& AK, double h, double inv2h, int m, int mc,
                                            int b, int first, float ck0, int& n, Hits& H) {
    double P;
    if (AK.Q == 0.0) P = AK.row_major ? g.bin[b].axis_pos_x : g.bin[b].axis_pos_y;
    else P = __fma_rn(bin_pos(g, b), AK.icv, AK.K);
    const double gm = __fma_rn(AK.Q, (double)m, P);
    double ax, bx;
    cell_interval(gm, AK.Q, AK.invQ, mc, ax, bx);
    if (!(bx > ax)) return;
    const int slot = n - first;
#pragma unroll
    for (int k = 0; k < BP3_HMAX; ++k) {
        if (slot == k) {
            // z_bin: tau at the start of major cell 0 and per major cell
            const double u0 = __fma_rn(bin_pos(g, b), AK.Au, AK.Bu);
            const double tau0 = (u0 + h) * inv2h, tauQ = AK.du * inv2h;
            const double tA = __fma_rn(tauQ, (double)m + ax, tau0);
            const double tB = __fma_rn(tauQ, (double)m + bx, tau0);
            H.b[k] = b;
            H.t0[k] = (float)fmin(tA, tB);
            H.dt[k] = (float)fabs(tB - tA);
            H.L[k] = (float)(AK.L * (bx - ax));
            H.ck[k] = ck0 * (float)inv2h;
            H.v[k] = true;
        }
    }
    ++n;
}

// The first two candidates of b0..b1 (of at most four when ds covers half a
// pixel's radial extent) load h and 1 / (2 h) together, clamped into the
// table so that the loads need no guard; the others follow one by one (two
// at once keep the register count at three waves per SIMD).
__device__ __forceinline__ int col_hits(const GeoK& g, const AngleK& AK, int m, int mc, int b0, int b1, int first,
                                        float ck0, Hits& H) {
#pragma unroll
    for (int k = 0; k < BP3_HMAX; ++k) {
        H.b[k] = 0;
        H.t0[k] = H.dt[k] = 0.0f;
        H.L[k] = H.ck[k] = 0.0f;
        H.v[k] = false;
    }
    constexpr int CMAX = 2;
    const int last = g.n_radial - 1;
    double h[CMAX], i2h[CMAX];
#pragma unroll
    for (int c = 0; c < CMAX; ++c) {
        const BinK& B = g.bin[min(max(b0 + c, 0), last)];
        h[c] = B.h;
        i2h[c] = B.inv2h;
    }
    int n = 0;
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
        if (b0 + c <= b1) col_hit_one(g, AK, h[c], i2h[c], m, mc, b0 + c, first, ck0, n, H);
    for (int b = b0 + CMAX; b <= b1; ++b) col_hit_one(g, AK, g.bin[b].h, g.bin[b].inv2h, m, mc, b, first, ck0, n, H);
    return n;
}

// One staging group of an angle: wait for this wave's copies into buf,
// issue the next group's copies into nxt, gather buf.  buf and nxt are
// distinct halves of the staging area; as restrict parameters they tell the
// compiler so, which lets the next group's copies stay in flight while buf
// is read (the compiler otherwise waits for every copy to LDS before an LDS
// read it cannot tell apart from their targets).
template <int ZB, int NBS>
__device__ __forceinline__ void bp3_group(const GeoK& g, const BP3Args& A, const BP3Shared& sh,
                                          float (&acc)[BP3_ZMAX], const Hits& H, const float* __restrict__ buf,
                                          float* __restrict__ nxt, bool stage_next, int dg, int z0, int aidx,
                                          int blo, int nbv, const double* tk) {
    const int wave = threadIdx.x >> 6;
    const int D = g.max_rd, ND = 2 * D + 1, rw = A.rw, dpg = A.dpg;
    // the angle's tau range in registers before any copy is in flight
    const double tau0 = tk[0], tau1 = tk[1];
    __builtin_amdgcn_s_waitcnt(0);      // this wave's copies (and zeros) into buf have landed
    if (stage_next) bp3_stage<NBS>(g, A, sh, nxt, dg + dpg, z0, aidx, blo, nbv, tau0, tau1);
    // (6) gather: wave v takes the group's ring differences v, v+4, ...
    for (int ds = wave; ds < dpg; ds += 4) {
        const int di = dg + ds;
        if (di >= ND) break;
        const int d = di - D;
        const float fd = (float)d, ad = fabsf(fd);
        int omin, omax;
        bp3_orange(tau0, tau1, d, omin, omax);
        const bool fits = omax - omin + ZB + 1 <= rw;
#pragma unroll
        for (int kk = 0; kk < BP3_HMAX; ++kk) {
            // the piece's axial range [zlo, zhi] in slice units (FP32:
            // |zeta| <= 1/2 + D, its rounding far below a slice); it
            // meets slice offsets o1 and, across boundary o2 = o1 + 1,
            // o2 (the host bounds the span below one slice)
            const float zref = fmaf(fd, H.t0[kk], 0.5f), span = ad * H.dt[kk];
            const float zlo = d >= 0 ? zref : zref - span;
            const float zhi = d >= 0 ? zref + span : zref;
            const float flo = floorf(zlo), fhi = floorf(zhi);
            const int o1 = (int)flo, o2 = (int)fhi;
            // 3D length per transaxial length of this (bin, d)
            const float x = fd * H.ck[kk];
            const float LK = H.L[kk] * __builtin_amdgcn_sqrtf(fmaf(x, x, 1.0f));
            const bool split = fhi != flo;
            // split in proportion to the axial lengths on either side
            const float frac = fminf(1.0f, fmaxf(0.0f, (fhi - zlo) * __builtin_amdgcn_rcpf(span)));
            const float a1 = split ? LK * frac : LK;
            const float a2 = LK - a1;
            // inside the staged footprint by construction: the tile's bin
            // window and tau range contain every hit of its columns, and
            // the host-side bounds on bins and slice-offset span hold; the
            // test only keeps LDS reads in range
            const int bcol = H.b[kk] - blo;
            const bool use = H.v[kk] && bcol >= 0 && bcol < nbv && o1 >= omin && o2 <= omax && fits;
            if (use) {
                // offset o1 with a1 and offset o2 = o1 + 1 (one row up
                // in the staging) with a2
                const float* sp = buf + (ds * rw + (omax - o1)) * NBS + bcol;
                bp3_apply<ZB, NBS>(acc, sp, a1, a2);
            }
        }
    }
}

template <int ZB, int NBS>
__device__ void bp3_body(const GeoK& g, const BP3Args& A, int vblock, BP3Shared& sh, float* s_w) {
    const int lane = threadIdx.x & 63;
    const int tiles_x = (g.nx + BP3_T - 1) / BP3_T, tiles_y = (g.ny + BP3_T - 1) / BP3_T;
    int t = vblock;
    const int tx0 = (t % tiles_x) * BP3_T;
    t /= tiles_x;
    const int ty0 = (t % tiles_y) * BP3_T;
    const int z0 = (t / tiles_y) * ZB;
    const int ix = tx0 + (lane & 7), iy = ty0 + (lane >> 3);
    const bool col_in = ix < g.nx && iy < g.ny;
    const int D = g.max_rd, ND = 2 * D + 1, Nr = g.n_radial;
    const int dpg = A.dpg;
    const float ck0 = (float)g.vz;      // ring pitch (== vz)

    float acc[BP3_ZMAX];
#pragma unroll
    for (int i = 0; i < BP3_ZMAX; ++i) acc[i] = 0.0f;
    // plane of ring 0 per ring difference, read by the staging (published by
    // the first barrier of the chunk loop)
    if ((int)threadIdx.x < ND) {
        const int d = (int)threadIdx.x - D;
        sh.pbase[threadIdx.x] = g.plane_base[threadIdx.x] - max(0, -d);
    }

    for (int c0 = 0; c0 < A.n_al; c0 += BP3_AMAX) {
        const int na = min(BP3_AMAX, A.n_al - c0);
        __syncthreads();    // the previous chunk's windows are read no more
        // (1) per angle of the chunk (one thread each): the tile's bins
        // [blo, blo + nb) (+1 bin margin) and tau range
        if ((int)threadIdx.x < na) {
            const int k = threadIdx.x;
            const int a = A.angles[c0 + k];
            const AngleK& AK = g.ang[a];
            const double X0 = ((double)tx0 - 0.5 * g.nx) * g.vx, X1 = X0 + BP3_T * g.vx;
            const double Y0 = ((double)ty0 - 0.5 * g.ny) * g.vy, Y1 = Y0 + BP3_T * g.vy;
            double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
            for (int q = 0; q < 4; ++q) {
                const double x = (q & 1) ? X1 : X0, y = (q & 2) ? Y1 : Y0;
                const double u = x * AK.c + y * AK.s;      // radial position
                const double v = -x * AK.s + y * AK.c;     // position along the ray
                umin = fmin(umin, u);
                umax = fmax(umax, u);
                vmin = fmin(vmin, v);
                vmax = fmax(vmax, v);
            }
            const int blo = max((int)floor(umin / g.ds + g.h0) - 1, 0);
            const int bhi = min((int)ceil(umax / g.ds + g.h0) + 1, Nr - 1);
            const int nb = max(0, min(bhi - blo + 1, min(A.nb, NBS)));
            double hmin = g.det_radius, hmax = g.det_radius;
            if (nb > 0) {
                const int bl = blo + nb - 1;
                hmin = fmin(g.bin[blo].h, g.bin[bl].h);
                hmax = ((double)blo <= g.h0 && (double)bl >= g.h0) ? g.det_radius : fmax(g.bin[blo].h, g.bin[bl].h);
            }
            sh.ang[k] = a;
            sh.blo[k] = blo;
            sh.nb[k] = nb;
            sh.tau[k][0] = 0.5 + vmin / (2.0 * (vmin < 0.0 ? hmin : hmax)) - 1e-9;
            sh.tau[k][1] = 0.5 + vmax / (2.0 * (vmax > 0.0 ? hmin : hmax)) + 1e-9;
        }
        __syncthreads();
        // (2) each wave goes through the chunk's angles on its own: the
        // staging slots it fills are the ones it gathers, so no barrier
        // orders the waves until the chunk ends
        for (int k = 0; k < na; ++k) {
            const int al = c0 + k;
            const int a = sh.ang[k];
            const AngleK& AK = g.ang[a];
            const int aidx = A.w_natural ? a : al;
            const int blo = sh.blo[k], nbv = sh.nb[k];
            const double* tk = sh.tau[k];    // read where used (registers are scarce)
            const int ngr = (ND + dpg - 1) / dpg;
            // the first group's loads run while the column's hits are found
            bp3_stage<NBS>(g, A, sh, s_w, 0, z0, aidx, blo, nbv, tk[0], tk[1]);
            // (3) candidate bins of the column: g(m) in [mc - max(Q,0), mc + 1 - min(Q,0)]
            const int m = AK.row_major ? iy : ix;
            const int mc = AK.row_major ? ix : iy;
            int b0 = 0, b1 = -1;
            if (col_in) {
                const double base = __fma_rn(AK.Q, (double)m, AK.wC);
                const double glo = (double)mc - fmax(AK.Q, 0.0) - 1e-7;
                const double ghi = (double)mc + 1.0 - fmin(AK.Q, 0.0) + 1e-7;
                const double bA = (glo - base) * AK.inv_wslope, bB = (ghi - base) * AK.inv_wslope;
                b0 = (int)fmax(floor(fmin(bA, bB)), 0.0);
                b1 = (int)fmin(ceil(fmax(bA, bB)), (double)(Nr - 1));
            }
            // (4) the column's hits: bins whose ray crosses its cell, in bin
            // order.  A pass takes BP3_HMAX of them; one pass covers any
            // column when ds is at least half the pixel's radial extent (e.g.
            // ds == vx == vy).  Every wave holds all the tile's columns, so
            // the passes (the wave's maximum) are the same in every wave.
            Hits H;
            const int nh = col_hits(g, AK, m, mc, b0, b1, 0, ck0, H);
            int npass = (nh + BP3_HMAX - 1) / BP3_HMAX;
#pragma unroll
            for (int sft = 1; sft < 64; sft <<= 1) npass = max(npass, __shfl_xor(npass, sft));
            npass = __builtin_amdgcn_readfirstlane(npass);
            for (int pass = 0; pass < npass; ++pass) {
                if (pass > 0) {
                    (void)col_hits(g, AK, m, mc, b0, b1, pass * BP3_HMAX, ck0, H);
                    bp3_stage<NBS>(g, A, sh, s_w, 0, z0, aidx, blo, nbv, tk[0], tk[1]);
                }
                // (5) w of ring differences in groups of dpg, double buffered:
                // the loads of group k+1 run while group k is gathered
                for (int gi = 0; gi < ngr; ++gi)
                    bp3_group<ZB, NBS>(g, A, sh, acc, H, s_w + (gi & 1) * A.half, s_w + ((gi + 1) & 1) * A.half,
                                       gi + 1 < ngr, gi * dpg, z0, aidx, blo, nbv, tk);
            }
            __builtin_amdgcn_s_waitcnt(0);      // no load of this angle is left in flight
        }
    }
    bp3_finish<ZB>(g, A, acc, s_w, tx0, ty0, z0);
}

// dynamic LDS: the staging area, A.lds floats.  Up to 32 slices per block the
// register budget is held to four waves per SIMD.  The first bp_blocks
// blocks back-project; A.n_pen more compute the penalty gradient and mu of
// the entering iterate (pen3_body, halo tile in the staging area): they need
// neither w nor b, and fill the CUs' spare slots and issue cycles while the
// latency-bound back-projection runs.
template <int ZB, int NBS>
__global__ __launch_bounds__(NT, ZB <= 32 ? 4 : 3) void k_bp3(GeoK g, BP3Args A, int n_tiles, int bp_blocks) {
    __shared__ BP3Shared sh;
    extern __shared__ __attribute__((aligned(16))) float bp3_stage_area[];
    if ((int)blockIdx.x >= bp_blocks) {
        pen3_body(g, A.pen, (int)blockIdx.x - bp_blocks, bp3_stage_area, sh.red);
        return;
    }
    const int tile = (int)xcd_block(blockIdx.x, n_tiles);
    if (tile >= n_tiles) return;
    bp3_body<ZB, NBS>(g, A, tile, sh, bp3_stage_area);
}

// ------------------------------------------------------------------ penalty gradient and mu


// s_f: PEN3_HALO floats of LDS, s_red: NT / 64 doubles
__device__ void pen3_body(const GeoK& g, const Pen3Args& A, int vblock, float* s_f, double* s_red) {
    constexpr int HX = PEN3_X + 2, HY = PEN3_Y + 2, HZ = PEN3_Z + 2;
    const int tx = pen3_tiles(g.nx, PEN3_X), ty = pen3_tiles(g.ny, PEN3_Y);
    const int x0 = (vblock % tx) * PEN3_X, y0 = ((vblock / tx) % ty) * PEN3_Y, z0 = (vblock / (tx * ty)) * PEN3_Z;
    for (int e = threadIdx.x; e < HX * HY * HZ; e += NT) {
        const int hx = e % HX, hy = (e / HX) % HY, hz = e / (HX * HY);
        const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
        float v = 0.0f;
        if (gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && gz >= 0 && gz < g.nz)
            v = A.f[((long long)gz * g.ny + gy) * g.nx + gx];
        s_f[e] = v;
    }
    float meanf = 1.0f;
    if (A.want_mu) meanf = (float)(sum_partials(A.part_f, A.n_part_f, s_red) / (double)g.nvox);
    __syncthreads();
    const int lx = threadIdx.x % PEN3_X, ly = threadIdx.x / PEN3_X;
    const int ix = x0 + lx, iy = y0 + ly;
    double mu_part = 0.0;
    if (ix < g.nx && iy < g.ny) {
        // The thread's column, slice by slice, with the 3x3 neighbourhood of
        // three slices in registers (one new slice read from LDS per step)
        // and the out-of-image neighbours masked instead of branched around
        // (the 26 in-image neighbours of eqn:gradRD, in stencil_at's order).
        const bool okx[3] = {ix > 0, true, ix < g.nx - 1};
        const bool oky[3] = {iy > 0, true, iy < g.ny - 1};
        const float gR = A.gamma_R, eps = A.eps;
        float pl[3][9];     // slices lz - 1, lz, lz + 1 of the halo tile (hz = lz .. lz + 2)
        auto load = [&](float (&p)[9], int hz) {
#pragma unroll
            for (int q = 0; q < 9; ++q) p[q] = s_f[(hz * HY + ly + q / 3) * HX + lx + q % 3];
        };
        load(pl[0], 0);
        load(pl[1], 1);
#pragma unroll
        for (int lz = 0; lz < PEN3_Z; ++lz) {
            const int iz = z0 + lz;
            if (iz >= g.nz) break;
            float (&pm)[9] = pl[lz % 3];
            float (&pc)[9] = pl[(lz + 1) % 3];
            float (&pp)[9] = pl[(lz + 2) % 3];
            load(pp, lz + 2);
            const bool okz[3] = {iz > 0, true, iz < g.nz - 1};
            const float fj = pc[4], fje = fj + eps, fj2e = fj + 2.0f * eps;
            float acc = 0.0f;
#pragma unroll
            for (int dz = 0; dz < 3; ++dz) {
                const float* p = dz == 0 ? pm : (dz == 1 ? pc : pp);
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    if (dz == 1 && q == 4) continue;
                    const RdpPair t = rdp_pair(fj, fje, fj2e, p[q], gR);
                    // an out-of-image neighbour adds 0
                    acc = fmaf(t.num, (okz[dz] && oky[q / 3] && okx[q % 3]) ? t.rden : 0.0f, acc);
                }
            }
            const float gradR = 2.0f * acc;
            const float gx = mat_der(ix, g.nx, pc[5], fj, pc[3]);
            const float gy = mat_der(iy, g.ny, pc[7], fj, pc[1]);
            const float gz = mat_der(iz, g.nz, pp[4], fj, pm[4]);
            const float gmag = sqrtf(gx * gx + gy * gy + gz * gz);
            const long long j = ((long long)iz * g.ny + iy) * g.nx + ix;
            if (A.gradR != nullptr) A.gradR[j] = gradR;
            else A.G[j] = fmaf(A.beta_over_M, gradR, A.G[j]);
            if (A.want_mu) {
                const float mu = fmaxf(0.01f, gmag / meanf);
                A.mu[j] = mu;
                mu_part += (double)mu;
            }
        }
    }
    if (A.want_mu) write_partial(mu_part, A.red_mu, s_red, vblock);
}

__global__ __launch_bounds__(NT) void k_pen3(GeoK g, Pen3Args A) {
    __shared__ float s_f[PEN3_HALO];
    __shared__ double s_red[NT / 64];
    pen3_body(g, A, blockIdx.x, s_f, s_red);
}

int pen3_grid(const pet_os_geom* G) {
    return pen3_tiles(G->d.nx, PEN3_X) * pen3_tiles(G->d.ny, PEN3_Y) * pen3_tiles(G->d.nz, PEN3_Z);
}

int launch_pen3(const pet_os_geom* G, const BPLaunch& L, hipStream_t s) {
    Pen3Args a{};
    a.f = L.f;
    a.G = L.out;
    a.mu = L.mu;
    a.want_mu = L.want_mu;
    a.beta_over_M = L.beta_over_M;
    a.gamma_R = L.gamma_R;
    a.eps = L.eps;
    a.part_f = L.part_f;
    a.n_part_f = L.n_part_f;
    a.red_mu = L.red_mu;
    const int grid = pen3_grid(G);
    if (L.want_mu && grid > L.red_mu.cap) return fail(PET_OS_ERR_DEVICE, "mu partials too small");
    petos_launch(k_pen3, dim3(grid), dim3(NT), 0, s, G->k, a);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

// ------------------------------------------------------------------ update and z-fastest copy

struct Upd3Args {
    float* f;
    float* fz;
    const float* G;
    const float* gradR;      // non-null: G = b + (beta/M) gradR, with b in G
    float beta_over_M;
    const float* mu;
    const float* pnorm;
    float* nu_frozen;
    int nu_mode;
    float step, nu1, nu2;
    BoxK box;
    const double* part_mu;
    int n_part_mu;
    Reduction red_f;
    int nx, ny, nz;
    const float* osem_sens;  // OSEM: f <- f * G / s_i (G = A_i^T (y/(q+r)))
};

constexpr int U3X = 64, U3Z = 32;

// update == false: only copy f into fz and write the partials of sum f
__device__ void upd3_body(const Upd3Args& A, long long vblock, bool update) {
    __shared__ float s_t[U3X * (U3Z + 1)];
    __shared__ double s_red[NT / 64];
    const int nxt = (A.nx + U3X - 1) / U3X;
    long long t = vblock;
    const int xt = (int)(t % nxt);
    t /= nxt;
    const int y = (int)(t % A.ny);
    const int z0 = (int)(t / A.ny) * U3Z, x0 = xt * U3X;
    const int lx = threadIdx.x & 63, zq = threadIdx.x >> 6;
    const int x = x0 + lx;
    const long long nvox = (long long)A.nx * A.ny * A.nz;
    const bool want_mu = update && (A.nu_mode == NU_COMPUTE || A.nu_mode == NU_COMPUTE_FREEZE);
    float meanmu = 1.0f;
    if (want_mu) meanmu = (float)(sum_partials(A.part_mu, A.n_part_mu, s_red) / (double)nvox);
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < U3Z / 4; ++k) {
        const int zz = zq + 4 * k, z = z0 + zz;
        float v = 0.0f;
        if (x < A.nx && z < A.nz) {
            const long long j = ((long long)z * A.ny + y) * A.nx + x;
            const float fj = A.f[j];
            if (update && A.osem_sens != nullptr) {
                // ordered-subsets EM (Hudson-Larkin): multiplicative update
                const float sj = A.osem_sens[j];
                const float fn = (sj > 0.0f) ? fj * A.G[j] / sj : fj;
                A.f[j] = fn;
                v = fn;
            } else if (update) {
                const float Gj = A.gradR != nullptr ? fmaf(A.beta_over_M, A.gradR[j], A.G[j]) : A.G[j];
                const float pj = A.pnorm[j];
                float nu = 1.0f;
                if (want_mu) {
                    nu = fminf(A.nu2, fmaxf(A.nu1, meanmu / A.mu[j]));
                    if (A.nu_mode == NU_COMPUTE_FREEZE) A.nu_frozen[j] = nu;
                } else if (A.nu_mode == NU_FROZEN) {
                    nu = A.nu_frozen[j];
                }
                const float fn = box_step(A.box, fj, pj, A.step, nu, Gj);
                A.f[j] = fn;
                v = fn;
            } else {
                v = fj;
            }
            part += (double)v;
        }
        s_t[lx * (U3Z + 1) + zz] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < U3Z * U3X / NT; ++k) {
        const int e = threadIdx.x + NT * k;
        const int xx = e / U3Z, zz = e % U3Z;
        const int xg = x0 + xx, z = z0 + zz;
        if (xg < A.nx && z < A.nz) A.fz[((long long)y * A.nx + xg) * A.nz + z] = s_t[xx * (U3Z + 1) + zz];
    }
    write_partial(part, A.red_f, s_red, vblock);
}

__global__ __launch_bounds__(NT) void k_upd3(Upd3Args A) { upd3_body(A, blockIdx.x, true); }
__global__ __launch_bounds__(NT) void k_prep3(Upd3Args A) { upd3_body(A, blockIdx.x, false); }

// ------------------------------------------------------------------ host side

int fp3_grid(const pet_os_geom* G, int n_al) {
    const long long n = fp3_items(n_al, G->d.n_radial, G->d.max_ring_diff, G->d.n_rings);
    return (int)((n + FP3_W - 1) / FP3_W);
}

// blocks of the single-request forward projection: one per (angle, bin) with
// staged columns, else the per-wave items of fp3_body
int fp3_launch_grid(const pet_os_geom* G, int n_al) {
    if (fp3_staged(G->d.nz, G->d.max_ring_diff)) return n_al * G->d.n_radial;
    return fp3_grid(G, n_al);
}

// Slices per block of the batched back-projector, and the default of the
// single-request one: the smallest of 16, 32, 64 that holds the volume's depth.
int bp3_zb(const pet_os_geom* G) { return G->d.nz <= 16 ? 16 : (G->d.nz <= 32 ? 32 : 64); }

int bp3_grid_zb(const pet_os_geom* G, int zb) {
    return ((G->d.nx + BP3_T - 1) / BP3_T) * ((G->d.ny + BP3_T - 1) / BP3_T) * ((G->d.nz + zb - 1) / zb);
}

// the single-request back-projector's slices per block: the autotuned value
// when there is one
static int bp3_zb_single(const pet_os_geom* G) { return G->tuned_zb > 0 ? G->tuned_zb : bp3_zb(G); }

int bp3_grid(const pet_os_geom* G) { return bp3_grid_zb(G, bp3_zb_single(G)); }
int bp3_grid_batch(const pet_os_geom* G) { return bp3_grid_zb(G, bp3_zb(G)); }

int upd3_grid(const pet_os_geom* G) {
    return ((G->d.nx + U3X - 1) / U3X) * G->d.ny * ((G->d.nz + U3Z - 1) / U3Z);
}

// Bins staged per angle (bound on an 8x8 tile's radial extent) and rows per
// (ring difference, bin) for zb slices: zb + slice-offset span + 1 pad row.
static int bp3_rows(const pet_os_geom* G, int zb, int& nb, int& rw) {
    const auto& d = G->d;
    // an 8x8 tile's projection onto the detector axis is at most
    // BP3_T sqrt(vx^2 + vy^2) wide; the window adds a bin of margin each side
    // and up to one for rounding at each end
    nb = (int)std::ceil(BP3_T * std::sqrt(d.vx * d.vx + d.vy * d.vy) / d.ds + 1e-6) + 4;
    if (nb > d.n_radial) nb = d.n_radial;
    if (nb > 40) return fail(PET_OS_ERR_INVALID_ARG, "3D geometry: more than 40 bins per 8x8 voxel tile (ds too small)");
    const double smax = 0.5 * (d.n_radial - 1) * d.ds;
    const double hmin = std::sqrt(d.det_radius * d.det_radius - smax * smax);
    const double hmax = d.det_radius;
    const double vhalf = 0.5 * std::sqrt((double)d.nx * d.nx * d.vx * d.vx + (double)d.ny * d.ny * d.vy * d.vy);
    const double dtau_tile = BP3_T * std::sqrt(d.vx * d.vx + d.vy * d.vy) / (2.0 * hmin);
    const double dtau_h = vhalf * (hmax - hmin) / (2.0 * hmin * hmin);
    const int span = (int)std::ceil(d.max_ring_diff * (dtau_tile + dtau_h) + 1e-9) + 3;
    rw = zb + span + 1;
    return PET_OS_OK;
}

// Staging shape of the batched back-projector (a fixed BP3_LDS-float area):
// the default slices per block and 8 ring differences staged together when
// two such buffers fit, else 4.  Fails if the footprint cannot fit in LDS.
int bp3_shape(const pet_os_geom* G, int& nb, int& zb, int& rw, int& dpg) {
    zb = bp3_zb(G);
    int rc = bp3_rows(G, zb, nb, rw);
    if (rc) return rc;
    const int nbs = bp3_nbs(nb);
    dpg = 8;
    if ((long long)dpg * nbs * rw > BP3_LDS / 2) dpg = 4;
    if ((long long)dpg * nbs * rw > BP3_LDS / 2)
        return fail(PET_OS_ERR_INVALID_ARG, "3D geometry: back-projection footprint does not fit in LDS");
    return PET_OS_OK;
}

// Shape of the single-request back-projector for zb slices per block and dpg
// ring differences per staging group (0: 8 if it fits, else 4): the staging
// area holds two buffers of dpg x row stride x rw floats and, for the finish,
// the halo tile of f and the block's sums; at most BP3_LDS floats.
int bp3_shape_single(const pet_os_geom* G, int zb, int dpg_req, int& nb, int& rw, int& dpg, int& half, int& lds) {
    int rc = bp3_rows(G, zb, nb, rw);
    if (rc) return rc;
    const long long nbs = bp3_nbs_single(nb);
    dpg = dpg_req > 0 ? dpg_req : ((8LL * nbs * rw <= BP3_LDS / 2) ? 8 : 4);
    const long long h = (long long)dpg * nbs * rw;
    const long long fin = 2LL * zb * 64;     // the finish: the waves' partial sums and their total
    const long long total = std::max(2 * h, fin);
    if (total > BP3_LDS)
        return fail(PET_OS_ERR_INVALID_ARG, "3D geometry: back-projection footprint does not fit in LDS");
    half = (int)h;
    lds = (int)total;
    return PET_OS_OK;
}

bool fp3_reads_yr(const pet_os_geom* G) { return G->d.dim == 3 && fp3_staged(G->d.nz, G->d.max_ring_diff); }

// yr[(a * n_radial + b) * n_planes + plane] = (y, r)[(plane * n_angles + a) *
// n_radial + b]: a transpose of [plane][angle-bin] by 64 x 64 tiles through
// LDS, both sides coalesced
__global__ __launch_bounds__(NT) void k_yr3(const float* __restrict__ y, const float* __restrict__ r,
                                            float2* __restrict__ yr, int n_ab, int n_planes) {
    __shared__ float2 t[64][65];
    const int ab0 = blockIdx.x * 64, p0 = blockIdx.y * 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = w; k < 64; k += NT / 64) {
        const int p = p0 + k, ab = ab0 + lane;
        if (p < n_planes && ab < n_ab) {
            const long long i = (long long)p * n_ab + ab;
            t[k][lane] = make_float2(y[i], r[i]);
        }
    }
    __syncthreads();
    for (int k = w; k < 64; k += NT / 64) {
        const int ab = ab0 + k, p = p0 + lane;
        if (p < n_planes && ab < n_ab) yr[(long long)ab * n_planes + p] = t[lane][k];
    }
}

int launch_yr3(const pet_os_geom* G, const float* y, const float* r, float2* yr, hipStream_t s) {
    const int n_ab = G->d.n_angles * G->d.n_radial;
    const dim3 grid((n_ab + 63) / 64, (G->n_planes + 63) / 64);
    if (grid.y > 65535) return fail(PET_OS_ERR_INVALID_ARG, "too many planes for the bin-major copy");
    petos_launch(k_yr3, grid, dim3(NT), 0, s, y, r, yr, n_ab, G->n_planes);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

int launch_fp3(const pet_os_geom* G, const FPLaunch& L, hipStream_t s) {
    FP3Args a;
    a.fz = L.fz;
    a.y = L.y;
    a.r = L.r;
    a.yr = L.yr;
    a.out = L.out;
    a.angles = L.angles;
    a.n_al = L.n_al;
    a.mode = L.mode;
    a.red = L.red;
    if (L.n_al == 0) return PET_OS_OK;
    if (L.mode != FP_COUNT && L.fz == nullptr) return fail(PET_OS_ERR_DEVICE, "3D forward projection without z copy");
    const int grid = fp3_launch_grid(G, L.n_al);
    if (L.mode == FP_OBJECTIVE && grid > L.red.cap) return fail(PET_OS_ERR_DEVICE, "objective partials too small");
    if (fp3_staged(G->d.nz, G->d.max_ring_diff))
        petos_launch(k_fp3, dim3(8 * ((grid + 7) / 8)), dim3(FPS_NT), 0, s, G->k, a, (long long)grid);
    else
        petos_launch(k_fp3_wave, dim3(8 * ((grid + 7) / 8)), dim3(NT), 0, s, G->k, a, (long long)grid);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

static void fill_bp3(const pet_os_geom* G, const BPLaunch& L, BP3Args& a) {
    a = BP3Args{};
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
}

int launch_bp3(const pet_os_geom* G, const BPLaunch& L, hipStream_t s) {
    if (2 * G->d.max_ring_diff + 1 > BP3_MAXND) return fail(PET_OS_ERR_INVALID_ARG, "max_ring_diff too large");
    BP3Args a;
    fill_bp3(G, L, a);
    a.zb = bp3_zb_single(G);
    int rc = bp3_shape_single(G, a.zb, G->tuned_dpg, a.nb, a.rw, a.dpg, a.half, a.lds);
    if (rc) return rc;
    // penalty blocks in the same launch when gradR is given (the penalty
    // gradient then goes there, and the update adds it to b)
    if ((L.f != nullptr) != (L.gradR != nullptr))
        return fail(PET_OS_ERR_DEVICE, "3D back-projection: the penalty blocks need both f and gradR");
    a.pen = Pen3Args{};
    a.n_pen = 0;
    if (L.gradR != nullptr) {
        a.pen.f = L.f;
        a.pen.G = nullptr;
        a.pen.gradR = L.gradR;
        a.pen.mu = L.mu;
        a.pen.want_mu = L.want_mu;
        a.pen.beta_over_M = L.beta_over_M;
        a.pen.gamma_R = L.gamma_R;
        a.pen.eps = L.eps;
        a.pen.part_f = L.part_f;
        a.pen.n_part_f = L.n_part_f;
        a.pen.red_mu = L.red_mu;
        a.n_pen = pen3_grid(G);
        if (L.want_mu && a.n_pen > L.red_mu.cap) return fail(PET_OS_ERR_DEVICE, "mu partials too small");
        a.lds = std::max(a.lds, PEN3_HALO);
    }
    const int grid = bp3_grid(G);
    const int nbs = bp3_nbs_single(a.nb);
    const int bp_blocks = 8 * ((grid + 7) / 8);
    const dim3 blocks(bp_blocks + a.n_pen);
    const size_t lds = (size_t)a.lds * sizeof(float);
    switch (a.zb) {
        case 16:
            if (nbs == 40) petos_launch(k_bp3<16, 40>, blocks, dim3(NT), lds, s, G->k, a, grid, bp_blocks);
            else if (nbs == 20) petos_launch(k_bp3<16, 20>, blocks, dim3(NT), lds, s, G->k, a, grid, bp_blocks);
            else petos_launch(k_bp3<16, 16>, blocks, dim3(NT), lds, s, G->k, a, grid, bp_blocks);
            break;
        case 32:
            if (nbs == 40) petos_launch(k_bp3<32, 40>, blocks, dim3(NT), lds, s, G->k, a, grid, bp_blocks);
            else if (nbs == 20) petos_launch(k_bp3<32, 20>, blocks, dim3(NT), lds, s, G->k, a, grid, bp_blocks);
            else petos_launch(k_bp3<32, 16>, blocks, dim3(NT), lds, s, G->k, a, grid, bp_blocks);
            break;
        case 64:
            if (nbs == 40) petos_launch(k_bp3<64, 40>, blocks, dim3(NT), lds, s, G->k, a, grid, bp_blocks);
            else if (nbs == 20) petos_launch(k_bp3<64, 20>, blocks, dim3(NT), lds, s, G->k, a, grid, bp_blocks);
            else petos_launch(k_bp3<64, 16>, blocks, dim3(NT), lds, s, G->k, a, grid, bp_blocks);
            break;
        default:
            return fail(PET_OS_ERR_DEVICE, "3D back-projector: slices per block must be 16, 32 or 64");
    }
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

static void fill_upd3(const pet_os_geom* G, const UpdLaunch& L, Upd3Args& a) {
    a.f = L.f;
    a.fz = L.fz;
    a.G = L.G;
    a.gradR = L.gradR;
    a.beta_over_M = L.beta_over_M;
    a.mu = L.mu;
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
    a.nx = G->d.nx;
    a.ny = G->d.ny;
    a.nz = G->d.nz;
    a.osem_sens = L.osem_sens;
}

int launch_update3(const pet_os_geom* G, const UpdLaunch& L, hipStream_t s) {
    Upd3Args a;
    fill_upd3(G, L, a);
    const int grid = upd3_grid(G);
    if (grid > L.red_f.cap) return fail(PET_OS_ERR_DEVICE, "sum partials too small");
    if (L.fz == nullptr) return fail(PET_OS_ERR_DEVICE, "3D update without z copy");
    petos_launch(k_upd3, dim3(grid), dim3(NT), 0, s, a);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

int launch_prep3(const pet_os_geom* G, const float* f, float* fz, Reduction red, hipStream_t s) {
    UpdLaunch L{};
    L.f = const_cast<float*>(f);    // read only when update == false
    L.fz = fz;
    L.red_f = red;
    Upd3Args a;
    fill_upd3(G, L, a);
    const int grid = upd3_grid(G);
    if (grid > red.cap) return fail(PET_OS_ERR_DEVICE, "sum partials too small");
    hipLaunchKernelGGL(k_prep3, dim3(grid), dim3(NT), 0, s, a);
    PETOS_HIP(hipGetLastError());
    return PET_OS_OK;
}

// ------------------------------------------------------------------ batched (persistent) kernels

__device__ __forceinline__ bool slot_live3(const SlotDev& d) { return d.active && d.J <= d.J_end; }

// Position of a persistent block in the item list: each XCD (blocks are
// dealt to the 8 XCDs round-robin) takes contiguous runs of items.  The grid
// is a multiple of 8.
__device__ __forceinline__ int xcd_item(int block, int grid) { return (block % 8) * (grid / 8) + block / 8; }

__global__ __launch_bounds__(NT) void k_fp3_batch(const SlotDev* __restrict__ S, const Item* __restrict__ items, const int* __restrict__ count) {
    const int n = *count;
    for (int it = xcd_item(blockIdx.x, gridDim.x); it < n; it += gridDim.x) {
        const Item I = items[it];
        const SlotDev& d = S[I.slot];
        if (!slot_live3(d)) continue;
        const int i = (d.J - 1) % d.g.n_subsets;
        FP3Args A{};
        A.fz = d.fz;
        A.y = d.y;
        A.r = d.r;
        A.out = d.w;
        A.angles = d.subset_lists + (long long)i * d.max_sub;
        A.n_al = d.subset_count[i];
        A.mode = FP_RATIO;
        fp3_body(d.g, A, I.block);
        __syncthreads();
    }
}

template <int ZB, int NBS>
__global__ __launch_bounds__(NT) void k_bp3_batch(const SlotDev* __restrict__ S, const Item* __restrict__ items, const int* __restrict__ count) {
    __shared__ BP3Shared sh;
    __shared__ __attribute__((aligned(16))) float s_w[BP3_LDS];
    const int n = *count;
    for (int it = xcd_item(blockIdx.x, gridDim.x); it < n; it += gridDim.x) {
        const Item I = items[it];
        const SlotDev& d = S[I.slot];
        if (!slot_live3(d) || d.zb != ZB) continue;
        const int i = (d.J - 1) % d.g.n_subsets;
        BP3Args A{};
        A.w = d.w;
        A.w_natural = 0;
        A.w_sp = d.g.n_radial;
        A.w_sa = (long long)d.g.n_planes * d.g.n_radial;
        A.angles = d.subset_lists + (long long)i * d.max_sub;
        A.n_al = d.subset_count[i];
        A.out = d.G;
        A.nb = d.nb_max;
        A.zb = d.zb;
        A.rw = d.rows_max;
        A.dpg = d.chunk;
        A.half = BP3_LDS / 2;
        A.lds = BP3_LDS;
        bp3_body<ZB, NBS>(d.g, A, I.block, sh, s_w);
        __syncthreads();
    }
}

__global__ __launch_bounds__(NT) void k_pen3_batch(const SlotDev* __restrict__ S, const Item* __restrict__ items, const int* __restrict__ count) {
    __shared__ float s_f[PEN3_HALO];
    __shared__ double s_red[NT / 64];
    const int n = *count;
    for (int it = xcd_item(blockIdx.x, gridDim.x); it < n; it += gridDim.x) {
        const Item I = items[it];
        const SlotDev& d = S[I.slot];
        if (!slot_live3(d)) continue;
        const int nu_mode = d.sched_nu[d.J - 1];
        Pen3Args A{};
        A.f = d.f;
        A.G = d.G;
        A.mu = d.mu;
        A.want_mu = (nu_mode == NU_COMPUTE || nu_mode == NU_COMPUTE_FREEZE) ? 1 : 0;
        A.beta_over_M = d.beta_over_M;
        A.gamma_R = d.gamma_R;
        A.eps = d.eps;
        A.part_f = d.part_f;
        A.n_part_f = d.n_part_f;
        A.red_mu.part = d.part_mu;
        A.red_mu.total = nullptr;
        A.red_mu.cap = d.n_part_mu;
        pen3_body(d.g, A, I.block, s_f, s_red);
        __syncthreads();
    }
}

__global__ __launch_bounds__(NT) void k_upd3_batch(const SlotDev* __restrict__ S, const Item* __restrict__ items, const int* __restrict__ count) {
    const int n = *count;
    for (int it = xcd_item(blockIdx.x, gridDim.x); it < n; it += gridDim.x) {
        const Item I = items[it];
        const SlotDev& d = S[I.slot];
        if (!slot_live3(d)) continue;
        Upd3Args A{};
        A.f = d.f;
        A.fz = d.fz;
        A.G = d.G;
        A.mu = d.mu;
        A.pnorm = d.pnorm;
        A.nu_frozen = d.nu_frozen;
        A.nu_mode = d.sched_nu[d.J - 1];
        A.step = d.sched_step[d.J - 1];
        A.nu1 = d.nu1;
        A.nu2 = d.nu2;
        A.box = d.box;
        A.part_mu = d.part_mu;
        A.n_part_mu = d.n_part_mu;
        A.red_f.part = d.part_f;
        A.red_f.total = nullptr;
        A.red_f.cap = d.n_part_f;
        A.nx = d.g.nx;
        A.ny = d.g.ny;
        A.nz = d.g.nz;
        upd3_body(A, I.block, true);
        __syncthreads();
    }
}

// the 3D part of one batched subiteration (lists WL_FP3, WL_BP3_*, WL_PEN3, WL_UPD3)
void launch_batch3_fp(const SlotDev* d_slots, const Item* list, const int* cnt, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_fp3_batch, dim3(grid), dim3(NT), 0, s, d_slots, list, cnt);
}

void launch_batch3_bp(const SlotDev* d_slots, const Item* list, const int* cnt, int grid, int zb, int nbs,
                      hipStream_t s) {
    if (zb == 16 && nbs == 20) hipLaunchKernelGGL((k_bp3_batch<16, 20>), dim3(grid), dim3(NT), 0, s, d_slots, list, cnt);
    else if (zb == 16) hipLaunchKernelGGL((k_bp3_batch<16, 40>), dim3(grid), dim3(NT), 0, s, d_slots, list, cnt);
    else if (zb == 32 && nbs == 20) hipLaunchKernelGGL((k_bp3_batch<32, 20>), dim3(grid), dim3(NT), 0, s, d_slots, list, cnt);
    else if (zb == 32) hipLaunchKernelGGL((k_bp3_batch<32, 40>), dim3(grid), dim3(NT), 0, s, d_slots, list, cnt);
    else if (nbs == 20) hipLaunchKernelGGL((k_bp3_batch<64, 20>), dim3(grid), dim3(NT), 0, s, d_slots, list, cnt);
    else hipLaunchKernelGGL((k_bp3_batch<64, 40>), dim3(grid), dim3(NT), 0, s, d_slots, list, cnt);
}

int bp3_nbs_of(const pet_os_geom* G) {
    int nb, zb, rw, dpg;
    if (bp3_shape(G, nb, zb, rw, dpg)) return 40;
    return bp3_nbs(nb);
}

void launch_batch3_pen(const SlotDev* d_slots, const Item* list, const int* cnt, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_pen3_batch, dim3(grid), dim3(NT), 0, s, d_slots, list, cnt);
}

void launch_batch3_upd(const SlotDev* d_slots, const Item* list, const int* cnt, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_upd3_batch, dim3(grid), dim3(NT), 0, s, d_slots, list, cnt);
}

}  // namespace petos
