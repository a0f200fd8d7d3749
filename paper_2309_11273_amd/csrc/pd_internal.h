// Internal declarations shared by the host and device sources of libpd.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "pd.h"

// Device control block (PD_CTL_BYTES bytes, caller-allocated, zeroed by
// pd_state_init).  Step counter: pass 1 of a step reads s2 and writes s1,
// pass 2 reads s1 and writes s2 = s1 + 1, so no kernel writes a slot that
// another wave of the same kernel reads.
#define PD_UMAX_SLOTS 64
#define PD_UMAX_STRIDE 32  // 4-byte words between slots (128 bytes)

struct pd_ctl {
    int64_t s1;
    int64_t s2;
    unsigned long long broken;    // directed bond-status bits cleared so far
    unsigned long long rechecks;  // FP64 rechecks made by the FP32 path
    unsigned int flags;           // bit 0: non-finite state, bit 1: shadow fallback used,
                                  // bit 2: a staged volume differs from vol_uniform
    unsigned int umax_bits[2];    // float bits of max |u| of shadow buffer k
    unsigned int margin_key;      // smallest |s - s_c| / s_c of a bond decided in double by
                                  // the FP32 path, stored as ~(float bits); 0 = none yet
    double qs[2];                 // fixed-point scale of shadow buffer k (power of two)
    unsigned long long fallbacks; // shadow entries that fell back to FP64
    double red[8];                // reductions (power iteration)
    unsigned long long dirty[2];  // rows marked for re-assembly, by step parity
    // FP32 path: the shadow, its scale and D_i are kept between calls.  They
    // describe uv[sh_cur] at step counter sh_step, built by the tile (1) or
    // gather (2) set-up (sh_kind; 0 = nothing valid).  Every other path that
    // advances the state advances s2 without sh_step, which invalidates them.
    int64_t sh_step;
    int32_t sh_kind;
    int32_t sh_cur;
    int32_t sh_skip;              // set-up of the current call skipped (shadow current)
    int32_t pad2;
    // energy checks of pd_step: kinetic and strain energy of the last check,
    // the total of the check before it, the step counter of the last check
    double en[4];
    unsigned long long pad1[6];
    // max |u| of shadow buffer k as written by the tile kernels: one slot per
    // tile class (tile mod PD_UMAX_SLOTS), each on its own 128-byte line, so
    // that the tiles' atomics do not queue on one address.  The maximum of
    // buffer k is that of umax_bits[k] and its slots.
    unsigned int umax_slot[2][PD_UMAX_SLOTS * PD_UMAX_STRIDE];
};
static_assert(offsetof(pd_ctl, umax_slot) % 128 == 0, "slots on their own lines");
static_assert(sizeof(pd_ctl) <= PD_CTL_BYTES, "control block too large");
static_assert(sizeof(pd_ctl) % 8 == 0, "control block is cleared in 8-byte words");

#define PD_CTL_NONFINITE 1u
#define PD_CTL_FALLBACK 2u
#define PD_CTL_VOLUME 4u  // a staged node volume differs from vol_uniform

// Padding stencil id.
#define PD_PAD_ID 127u

#ifdef __HIPCC__
#define PD_HD __host__ __device__
#else
#define PD_HD
#endif

#ifdef __HIPCC__
#include <hip/hip_runtime.h>

static_assert(PD_UMAX_SLOTS == 64, "one slot per lane of a wave64");
// Largest |u| bits of shadow buffer k: its word and its slots, read by one
// whole wave (lane l reads slot l).
__device__ __forceinline__ unsigned int umax_wave(const pd_ctl *ctl, int k, int lane) {
    unsigned int m = ctl->umax_slot[k][lane * PD_UMAX_STRIDE];
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned int t = (unsigned int)__shfl_xor((int)m, o);
        m = t > m ? t : m;
    }
    const unsigned int b = ctl->umax_bits[k];
    return m > b ? m : b;
}
// Clears the word and the slots of shadow buffer k (one whole wave).
__device__ __forceinline__ void umax_clear_wave(pd_ctl *ctl, int k, int lane) {
    ctl->umax_slot[k][lane * PD_UMAX_STRIDE] = 0u;
    if (lane == 0) ctl->umax_bits[k] = 0u;
}
// Per-row vectors kept with the problem's dimension (velocity, the row
// constants D_i and the carried force parts): a 3D row is three packed
// entries (x, y, z), a 2D row two (x, y), so no padding entry is moved.  The
// wave's rows are consecutive, so its accesses cover one contiguous range.
__device__ __forceinline__ double4 ldv(const double *p, int dim, int64_t r) {
    if (dim == 3) {
        const double *q = p + 3 * r;
        return make_double4(q[0], q[1], q[2], 0.0);
    }
    const double2 t = reinterpret_cast<const double2 *>(p)[r];
    return make_double4(t.x, t.y, 0.0, 0.0);
}
__device__ __forceinline__ void stv(double *p, int dim, int64_t r, double4 v) {
    if (dim == 3) {
        double *q = p + 3 * r;
        q[0] = v.x;
        q[1] = v.y;
        q[2] = v.z;
    } else {
        reinterpret_cast<double2 *>(p)[r] = make_double2(v.x, v.y);
    }
}
__device__ __forceinline__ float4 ldvf(const float *p, int dim, int64_t r) {
    if (dim == 3) {
        const float *q = p + 3 * r;
        return make_float4(q[0], q[1], q[2], 0.0f);
    }
    const float2 t = reinterpret_cast<const float2 *>(p)[r];
    return make_float4(t.x, t.y, 0.0f, 0.0f);
}
__device__ __forceinline__ void stvf(float *p, int dim, int64_t r, float4 v) {
    if (dim == 3) {
        float *q = p + 3 * r;
        q[0] = v.x;
        q[1] = v.y;
        q[2] = v.z;
    } else {
        reinterpret_cast<float2 *>(p)[r] = make_float2(v.x, v.y);
    }
}
#endif

// Bond word layout inside a 64-row slice whose words start at 'base' (a
// multiple of 256): words come in groups of four per lane, so that lane
// 'lane' reads words 4g..4g+3 of its row with one 16-byte load and the 64
// lanes of a wave read 1 KiB of consecutive memory.  Row lengths inside a
// slice are padded to a multiple of four.
PD_HD inline int64_t pd_widx(int64_t base, int64_t k, int lane) {
    return base + ((k >> 2) << 8) + ((int64_t)lane << 2) + (k & 3);
}

// LDS halo box of a 64-point tile T[0] x T[1] x T[2] with reach R: the tile
// plus R lattice points on every side; slot of box point (x, y, z) is
// x + B[0] y + B[3] z, and the box has B[3] * B[2] slots.  B[1] and B[2] are
// the y and z extents.  In 3D with 4x4x4 tiles the x pitch B[0] is padded up
// to 4 mod 8, which spreads each quarter-wave's 16-byte reads over the LDS
// banks.  (Padding the z pitch as well, up to 16 mod 32, removes the
// remaining bank conflicts of the wave-wide reads, but the larger box costs
// more in staging and occupancy than the conflicts do: measured slower.)
PD_HD inline void pd_tile_box(const int32_t *T, int R, int dim, int32_t *B) {
    B[0] = T[0] + 2 * R;
    if (dim == 3 && T[0] == 4) B[0] += (12 - B[0] % 8) % 8;
    B[1] = T[1] + 2 * R;
    B[2] = dim == 3 ? T[2] + 2 * R : 1;
    B[3] = B[0] * B[1];
}

// Points of the halo box itself (tile + R on every side, no padding).
PD_HD inline int pd_box_points(const int32_t *T, int R, int dim) {
    return (T[0] + 2 * R) * (T[1] + 2 * R) * (dim == 3 ? T[2] + 2 * R : 1);
}

// Fixed array stride (points) of the box the single-precision kernels
// stage as separate arrays: 3D (a multiple of 64, for the st64 reads); 2D
// boxes of at most 256 points (one wave per tile) or more (four waves per
// tile).
PD_HD inline int pd_box1_stride(int dim, int npoints) { return dim == 3 ? 1472 : (npoints <= 256 ? 336 : 1024); }

// Pitches of that box, laid out like pd_tile_box (B[0] x pitch, B[1] y
// pitch, B[2] z extent, B[3] = B[0] B[1] z pitch) but padded so that the 64
// lanes of a tile, reading one 4-byte element each at the same offset from
// their own points, hit 64 distinct LDS banks: x + B[0] y + B[3] z must be
// distinct mod 64 over the tile's positions, which pitches 12 and 144 give a
// 4x4x4 tile and an x pitch that is an odd multiple of 8 gives an 8x8 tile.
// Boxes the padding would push past the stride stay unpadded.
PD_HD inline void pd_tile_box1(const int32_t *T, int R, int dim, int32_t *B) {
    const int e0 = T[0] + 2 * R, e1 = T[1] + 2 * R, e2 = dim == 3 ? T[2] + 2 * R : 1;
    int p0 = e0, p1 = e1;
    if (dim == 3 && T[0] == 4 && T[1] == 4 && e0 <= 12) {
        p0 = 12;
        p1 = 12;
    } else if (dim == 2 && T[0] == 8 && e0 <= 24) {
        p0 = 24;
    }
    if (p0 * p1 * e2 > pd_box1_stride(dim, e0 * e1 * e2)) {
        p0 = e0;
        p1 = e1;
    }
    B[0] = p0;
    B[1] = p1;
    B[2] = e2;
    B[3] = p0 * p1;
}
