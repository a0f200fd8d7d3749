// Device helpers shared by the LDS-staged ("tiled") kernels: the tile box
// and halo addressing, the per-entry table row, wave-uniform bit tests.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace pdk {

#define PD_SENTINEL_T ((int)0x80000000)
#define PD_TILE_WAVES 4
#define PD_TILE_THREADS (64 * PD_TILE_WAVES)

// one row of the per-entry table (pd_family_host.ktab)
struct KEnt {
    float m0, m1, m2, x;
    int soff;
    float ix;  // 1 / x
    int z0, z1;
};
static_assert(sizeof(KEnt) == 32, "ktab row is 8 words");
// one row of the second table (from word 1024): x M and the LDS offset
struct KEnt2 {
    float xm0, xm1, xm2;
    int soff;
};
static_assert(sizeof(KEnt2) == 16, "second ktab row is 4 words");
// one row of the third table (from word 1536), used by the single-precision
// kernels: M / x, x^2, x M and the neighbour's offset in their box; the
// third components last, so that a 2D row's used words are contiguous
struct KEnt1 {
    float mx0, mx1, x2, xm0, xm1;
    int soff;
    float mx2, xm2;
};
static_assert(sizeof(KEnt1) == 32, "third ktab row is 8 words");

// 64-bit words read through the scalar data cache (wave-uniform addresses)
typedef __attribute__((address_space(4))) const uint64_t cu64_t;

__device__ __forceinline__ double ext_canonical_t(double m1, double m2, double m3, double e1, double e2,
                                                  double e3) {
#pragma clang fp contract(off)
    double a = m1 * e1;
    double b = m2 * e2;
    double c = m3 * e3;
    return (a + b) + c;
}

__device__ __forceinline__ double shadow_scale_t(unsigned int mbits) {
    const float m = __uint_as_float(mbits);
    if (!(m > 0.0f) || !isfinite(m)) return ldexp(1.0, -100);
    const int e = ilogb((double)m);
    return ldexp(1.0, max(e - 27, -100));
}

__device__ __forceinline__ int quantise_t(double u, double invQ, bool &bad) {
    const double t = u * invQ;
    if (!(fabs(t) < 1073741824.0)) {
        bad = true;
        return 0;
    }
    return (int)rint(t);
}

__device__ __forceinline__ uint64_t uni64_t(uint64_t v) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// float of the 32-bit difference a - b (wrapping, never undefined)
__device__ __forceinline__ float idiff(int a, int b) { return (float)(int)((uint32_t)a - (uint32_t)b); }

// |v| if |v| >= 2^24 (a float that may hold a rounded integer), else 0
__device__ __forceinline__ float big_abs(float v) {
    const float m = fabsf(v);
    return m >= 16777216.0f ? m : 0.0f;
}

// Wave minimum of a non-negative breaking margin, merged into *key as
// ~(float bits) (a larger key is a smaller margin; zero means none yet).
// Called by every lane of the wave.
__device__ __forceinline__ void margin_merge(float m, unsigned int *key) {
    for (int o = 32; o > 0; o >>= 1) m = fminf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0 && m < __builtin_inff()) atomicMax(key, ~__float_as_uint(m));
}

// Wave maximum of non-negative floats, as their bits (which order the same
// way as int): a running maximum over lane shifts 1, 2, 4, 8 inside each
// 16-lane row (DPP moves, no LDS traffic), then the four row maxima read
// into scalars.  Called by every lane; the result is wave-uniform.
__device__ __forceinline__ unsigned int wave_max_bits(float v) {
    int b = (int)__float_as_uint(v);
    b = max(b, __builtin_amdgcn_update_dpp(0, b, 0x111, 0xf, 0xf, false));  // row_shr:1
    b = max(b, __builtin_amdgcn_update_dpp(0, b, 0x112, 0xf, 0xf, false));  // row_shr:2
    b = max(b, __builtin_amdgcn_update_dpp(0, b, 0x114, 0xf, 0xf, false));  // row_shr:4
    b = max(b, __builtin_amdgcn_update_dpp(0, b, 0x118, 0xf, 0xf, false));  // row_shr:8
    const int r0 = __builtin_amdgcn_readlane(b, 15), r1 = __builtin_amdgcn_readlane(b, 31);
    const int r2 = __builtin_amdgcn_readlane(b, 47), r3 = __builtin_amdgcn_readlane(b, 63);
    return (unsigned int)max(max(r0, r1), max(r2, r3));
}

// lane's bit of a wave-uniform 64-bit word, used as the condition mask as is
__device__ __forceinline__ bool lane_bit(uint64_t uniform_word) {
    return __builtin_amdgcn_inverse_ballot_w64(uniform_word);
}

// specimen of a tile: every row of a tile belongs to one specimen, padding
// rows carry id 0
__device__ __forceinline__ uint32_t tile_specimen(uint32_t aux) {
    const uint64_t b = __ballot((aux >> 8) != 0u);
    return b ? ((uint32_t)__builtin_amdgcn_readlane((int)aux, (int)__builtin_ctzll(b)) >> 8) : 0u;
}

struct Box {
    int T0, T1, R, Bx, Pz, nslot;
};

__device__ __forceinline__ Box make_box(const StepArgs &a, int dim) {
    Box b;
    int32_t B[4];
    pd_tile_box(a.tile, a.reach, dim, B);
    b.T0 = a.tile[0];
    b.T1 = a.tile[1];
    b.R = a.reach;
    b.Bx = B[0];
    b.Pz = B[3];
    b.nslot = B[3] * B[2];
    return b;
}

// LDS box slot of lane l of the tile (its own lattice point); tile edges
// are powers of two
template <int DIM>
__device__ __forceinline__ int own_slot(const Box &g, int lane) {
    const int s0 = __builtin_ctz((unsigned)g.T0), s1 = __builtin_ctz((unsigned)g.T1);
    const int l0 = lane & (g.T0 - 1), l1 = (lane >> s0) & (g.T1 - 1), l2 = lane >> (s0 + s1);
    return (l0 + g.R) + g.Bx * (l1 + g.R) + g.Pz * (DIM == 3 ? l2 + g.R : 0);
}

// slot of lane l's own point in the single-precision pass-1 box (pitches B
// from pd_tile_box1)
template <int DIM>
__device__ __forceinline__ int own_slot1(const int32_t *T, int R, const int32_t *B, int lane) {
    const int s0 = __builtin_ctz((unsigned)T[0]), s1 = __builtin_ctz((unsigned)T[1]);
    const int l0 = lane & (T[0] - 1), l1 = (lane >> s0) & (T[1] - 1), l2 = lane >> (s0 + s1);
    return (l0 + R) + B[0] * (l1 + R) + B[3] * (DIM == 3 ? l2 + R : 0);
}

// 1 / q for a power of two q (exact, no division)
__device__ __forceinline__ double inv_pow2(double q) { return ldexp(1.0, -ilogb(q)); }

// global row of a halo slot from its halo_map entry and the tile's
// neighbour table (-1: pitch padding or no tile in that direction)
__device__ __forceinline__ int64_t halo_row_of(int m, const int *tn) {
    if (m < 0) return -1;
    const int nt = tn[m >> 6];
    return nt < 0 ? -1 : (int64_t)nt * 64 + (m & 63);
}

// Barrier between the staging and the sweep of a tile.  With one tile per
// workgroup (TPW = 1) the four waves share the tile's LDS; with one tile per
// wave (TPW = 4) a wave reads only what it wrote itself, and its LDS
// operations complete in order, so a wavefront-scope fence suffices and the
// waves of a workgroup need not wait for each other.
template <int TPW>
__device__ __forceinline__ void tile_sync() {
    if constexpr (TPW <= 1) {  // one tile (TPW 1) or one super-tile (TPW 0) per workgroup
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

template <int TPW>
__device__ __forceinline__ bool tile_sync_or(bool p) {
    if constexpr (TPW <= 1) {
        return __syncthreads_or(p);
    } else {
        tile_sync<TPW>();
        return __ballot(p) != 0ull;
    }
}

// Workgroups are dealt round-robin to the 8 XCDs of the chip, each with its
// own L2.  Tile of workgroup b: every XCD gets a contiguous range of tiles,
// so neighbouring tiles, whose halo boxes overlap, are staged through the
// same L2.  A bijection of [0, n).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t n) {
    const int64_t q = n >> 3, r = n & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// slots per thread staged at once: 1280 slots in 3D, 512 in 2D
template <int DIM>
struct StageCap {
    static constexpr int value = DIM == 3 ? 5 : 2;
};

// How the four waves of a workgroup share the work: TPW tiles per workgroup.
//   TPW = 1: the four waves split the stencil of one tile in quarters and add
//            their partial sums in LDS (3D: a long stencil, a large halo box);
//   TPW = 4: every wave takes a whole tile of its own (2D: a short stencil,
//            whose quarters would leave each wave too little work per box);
//   TPW = 0: a super-tile, four tiles side by side (2 x 2 (x 1); 4x4x4 in
//            3D, 8x8 in 2D) that share one halo box staged by the whole
//            workgroup; every wave sweeps the whole stencil for its own tile.
// SPLIT waves share a tile; NT threads stage its box, MS slots each, so a box
// holds at most NT * MS slots (TPW = 4: 256).
template <int DIM, int TPW>
struct Grp {
    static constexpr int SPLIT = TPW == 0 ? 1 : PD_TILE_WAVES / TPW;
    static constexpr int NT = TPW == 0 ? PD_TILE_THREADS : 64 * SPLIT;
    static constexpr int MS = TPW == 0 ? (DIM == 3 ? 8 : 2) : (TPW == 1 ? StageCap<DIM>::value : 4);
    static constexpr int CAP = NT * MS;
};

// super-tile of this workgroup and the tile of this wave in it (quadrant
// 'sub'); a wave whose quadrant holds no tile reads the first tile of the
// super-tile and must not write
__device__ __forceinline__ int64_t super_tile(const StepArgs &a, int sub, int64_t &st, bool &valid) {
    st = xcd_tile(blockIdx.x, a.n_st);
    const int t = a.st_tiles[4 * st + sub];
    valid = t >= 0;
    if (valid) return t;
    for (int q = 0; q < 4; q++) {
        const int u = a.st_tiles[4 * st + q];
        if (u >= 0) return u;
    }
    return 0;
}

// first tile of a super-tile (the quadrant whose wave writes the box's
// shared reference point)
__device__ __forceinline__ int64_t first_st_tile(const StepArgs &a, int64_t st) {
    for (int q = 0; q < 4; q++) {
        const int u = a.st_tiles[4 * st + q];
        if (u >= 0) return u;
    }
    return 0;
}

// slot of lane l of quadrant q's tile in the super-tile box (reach R on
// every side; pitches 16 and 228 in 3D, x pitch 40 in 2D)
template <int DIM>
__device__ __forceinline__ int own_slot_st(int R, int sub, int lane) {
    if constexpr (DIM == 3)
        return ((lane & 3) + 4 * (sub & 1) + R) + 16 * (((lane >> 2) & 3) + 4 * (sub >> 1) + R) +
               228 * ((lane >> 4) + R);
    else
        return ((lane & 7) + 8 * (sub & 1) + R) + 40 * ((lane >> 3) + 8 * (sub >> 1) + R);
}

// tile of this wave; waves of the last workgroup past the last tile (TPW > 1)
// redo the last tile and must not write
template <int TPW>
__device__ __forceinline__ int64_t group_tile(int64_t n_tiles, int sub, bool &valid) {
    constexpr int P = TPW > 0 ? TPW : 1;  // (TPW = 0 never reaches here)
    const int64_t groups = (n_tiles + P - 1) / P;
    const int64_t t = xcd_tile(blockIdx.x, groups) * P + sub;
    valid = t < n_tiles;
    return valid ? t : n_tiles - 1;
}

// workgroup tiling the launchers choose: whole tiles per wave in 2D when the
// halo box (npoints points, unpadded) fits the per-wave staging capacity and
// the caller did not ask for one tile per workgroup
inline int tiles_per_group(const StepArgs &a, int npoints) {
    return (a.dim == 2 && !a.one_tile_per_group && npoints <= Grp<2, 4>::CAP) ? 4 : 1;
}

}  // namespace pdk
