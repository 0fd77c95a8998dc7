// gv_device.hpp -- data layouts and device helpers shared by the HIP kernels
// of the visibility-field path (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gv {

// Raster tile: 16x16 pixels, one 256-thread workgroup (4 waves of 64), one
// pixel per lane.  Each wave covers an 8x8 quadrant of the tile.
constexpr int TILE = 16;
// Depth-sort values of the scanned emission: record index | min(tile count,
// PACK_SAT) << PACK_SHIFT (records below 2^PACK_SHIFT), so that the sort
// carries each record's tile count into depth order; a saturated count is
// read from the record's binning line.
constexpr int PACK_SHIFT = 24;
constexpr uint32_t PACK_SAT = 255u;
constexpr uint32_t PACK_RMASK = (1u << PACK_SHIFT) - 1u;
constexpr int TILE_SHIFT = 4;
constexpr int WG = 256;
constexpr int WAVES = WG / 64;

// LSD radix sort: 8-bit digits, a fixed number of blocks per pass.
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int RADIX_BLOCKS = 4096;

// Projection: PROJ_SPLIT threads per Gaussian, thread s of Gaussian g handles
// views s, s + PROJ_SPLIT, ...; records are numbered by (g, s, view), so a
// Gaussian's records stay contiguous.
constexpr int PROJ_SPLIT = 4;

// Device exclusive scan: elements per block.
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_BLOCK = WG * SCAN_ITEMS;

constexpr int MAX_K = 16;  // (L+1)^2 for L <= 3

// One camera as the kernels see it.  The projection reads it with uniform
// (scalar) loads, the raster with one lookup per workgroup.
struct ViewDev {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    float C[3];          // camera centre in world coordinates
    int32_t w, h;
    int32_t tiles_x, tiles_y;
    int32_t tile_base;   // first global tile id of this view
    int32_t pad0;
    int64_t pix_base;    // first pixel of this view in the packed maps
};
static_assert(sizeof(ViewDev) == 112, "ViewDev layout");

// One (Gaussian, view) record after projection: 32 bytes, gathered by the
// raster through the sorted tile lists.
//   uv        anchor pixel of the projected centre, int16 x | int16 y << 16
//   fx, fy    projected centre minus the anchor (|f| <= 0.5 unless clamped)
//   l11..l22  lower Cholesky factor of the 2D conic, times sqrt(log2(e)/2),
//             so that (l11 dx + l21 dy)^2 + (l22 dy)^2 = log2(e) m / 2
//   o         opacity
//   v         queried visibility (query path), unused by the build
struct Rec {
    int32_t uv;
    float fx, fy;
    float l11, l21, l22;
    float o;
    float v;
};
static_assert(sizeof(Rec) == 32, "Rec layout");

// What the binning needs of a record, in one 32-byte line: its tile
// rectangle (first global tile id, tiles per view row, rectangle width and
// height) and its ellipse relative to the rectangle's first tile.
//   tile0     global id of the rectangle's top-left tile
//   dims      tiles_x | (wx - 1) << 11 | (wy - 1) << 21 | live << 31
//   uvr       anchor pixel minus 16 x the rectangle's first tile column / row,
//             int16 x | int16 y << 16
//   fx, fy, l11, l21, l22   as in Rec
struct Bin {
    uint32_t tile0;
    uint32_t dims;
    int32_t uvr;
    float fx, fy;
    float l11, l21, l22;
};
static_assert(sizeof(Bin) == 32, "Bin layout");

__device__ __forceinline__ uint32_t bin_tiles_x(uint32_t dims) { return dims & 0x7FFu; }
__device__ __forceinline__ uint32_t bin_wx(uint32_t dims) { return ((dims >> 11) & 0x3FFu) + 1u; }
__device__ __forceinline__ uint32_t bin_wy(uint32_t dims) { return ((dims >> 21) & 0x3FFu) + 1u; }
__device__ __forceinline__ uint32_t bin_ntiles(uint32_t dims) { return (dims >> 31) ? bin_wx(dims) * bin_wy(dims) : 0u; }

// Status words at the start of every workspace.
struct Status {
    unsigned long long R_total;   // records produced by culling
    unsigned long long M_total;   // instances produced by binning
    uint32_t R_eff;               // min(R_total, capacity)
    uint32_t M_eff;
    uint32_t overflow;            // bit 0 records, bit 1 instances
    int32_t best;                 // argmax scratch
    uint32_t M_live;              // instances left after the tile sort drops dead ones
    uint32_t emit_ticket;         // next record block of the instance emission
    uint32_t tile_ticket[8];      // per XCD: next queue position of a persistent blend
    unsigned long long measure[4];
};

constexpr uint32_t DEAD_KEY = 0xFFFFFFFFu;

// Instance keys: global tile id in the low QMASK_SHIFT bits (sorted on), the
// record's quadrant mask for that tile in the bits above (carried along).
// Instances whose mask is empty get the tile id one past the last tile, so
// they sort behind every tile and no tile range contains them.
constexpr int QMASK_SHIFT = 28;
constexpr uint32_t TILE_KEY_MASK = (1u << QMASK_SHIFT) - 1u;

// ---------------------------------------------------------------- wave helpers

template <int CTRL, int ROWM = 0xF, int BANKM = 0xF>
__device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWM, BANKM, true));
}

// Sum of x over the 64 lanes of the wave; every lane must be active.  The
// total lands in lane 63 and is broadcast through a scalar register.
__device__ __forceinline__ float wave_sum(float x) {
    x += dpp_f<0x111>(x);                 // row_shr:1
    x += dpp_f<0x112>(x);                 // row_shr:2
    x += dpp_f<0x114>(x);                 // row_shr:4
    x += dpp_f<0x118>(x);                 // row_shr:8
    x += dpp_f<0x142, 0xA>(x);            // row_bcast:15 into rows 1, 3
    x += dpp_f<0x143, 0xC>(x);            // row_bcast:31 into rows 2, 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

__device__ __forceinline__ uint32_t lanes_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---------------------------------------------------------------- real SH, L <= 3

// Real spherical harmonics of a unit direction (x, y, z), index l^2 + l + m,
// in the basis built from the complex Y_l^m with the Condon-Shortley phase:
// sqrt(2) (-1)^m Im Y_l^|m| for m < 0, Y_l^0, sqrt(2) (-1)^m Re Y_l^m for m > 0.
template <int L>
__device__ __forceinline__ void sh_eval(float x, float y, float z, float *Y) {
    Y[0] = 0.28209479177387814f;
    if (L >= 1) {
        Y[1] = 0.4886025119029199f * y;
        Y[2] = 0.4886025119029199f * z;
        Y[3] = 0.4886025119029199f * x;
    }
    if (L >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = 1.0925484305920792f * x * y;
        Y[5] = 1.0925484305920792f * y * z;
        Y[6] = 0.31539156525252005f * (3.0f * zz - 1.0f);
        Y[7] = 1.0925484305920792f * x * z;
        Y[8] = 0.5462742152960396f * (xx - yy);
        if (L >= 3) {
            Y[9] = 0.5900435899266435f * y * (3.0f * xx - yy);
            Y[10] = 2.890611442640554f * x * y * z;
            Y[11] = 0.4570457994644658f * y * (5.0f * zz - 1.0f);
            Y[12] = 0.3731763325901154f * z * (5.0f * zz - 3.0f);
            Y[13] = 0.4570457994644658f * x * (5.0f * zz - 1.0f);
            Y[14] = 1.445305721320277f * z * (xx - yy);
            Y[15] = 0.5900435899266435f * x * (xx - 3.0f * yy);
        }
    }
}

// ---------------------------------------------------------------- storage types

__device__ __forceinline__ float load_f(const float *p, int64_t i) { return p[i]; }
__device__ __forceinline__ float load_f(const _Float16 *p, int64_t i) { return (float)p[i]; }
__device__ __forceinline__ float load_f(const uint16_t *p, int64_t i) {   // bfloat16 bits
    return __uint_as_float(((uint32_t)p[i]) << 16);
}


// ---------------------------------------------------------------- tile-local geometry

// Record -> tile-local form: centre relative to the tile origin, computed from
// the integer anchor and the FP32 fraction so that it keeps full precision.
__device__ __forceinline__ void local_centre(const Rec &R, int ox, int oy, float &ux, float &uy) {
    const int ax = (int)(int16_t)(R.uv & 0xFFFF);
    const int ay = R.uv >> 16;
    ux = (float)(ax - ox) + R.fx;
    uy = (float)(ay - oy) + R.fy;
}

// Quadrant test of the binning.  Bit q of the mask is set when the ellipse
// p <= qc reaches the rectangle spanned by the pixel centres of quadrant q of
// the tile (q = 2 row + column, quadrants of 8 x 8 pixels).  With the scaled
// Cholesky factor L = [[a, 0], [b, c]] of the conic, p = u^2 + w^2 with
// u = a ex + b ey, w = c ey, for the offset (ex, ey) = centre - point.  The
// points of the ellipse in a horizontal band of rows form a convex set whose
// x-extent comes from the extreme points of the ellipse: at offset ey the
// chord spans x = ux + (b ey +- s) / a, s = sqrt(qc - (c ey)^2); the
// rightmost point of the whole ellipse lies at ey_R = sqrt(qc) (b / c) / (c n),
// n = sqrt(1 + (b / c)^2), the leftmost at -ey_R, and over a band the extreme
// x are taken at ey_R and -ey_R clamped into the band.  The threshold and the
// x-extent are widened so that rounding never drops a quadrant holding a
// pixel the blend composites.
struct EllipseBands {
    float kx;    // b / a
    float ia;    // 1 / a
    float eyR;   // offset ey of the rightmost point
    float hy;    // half height sqrt(qc) / c
};

__device__ __forceinline__ float band_threshold(float qcut) { return fmaf(qcut, 1.001f, 0.01f); }

// The hardware reciprocal, square root and reciprocal square root (1 ulp)
// are used here and in the band tests below: their error is far inside the
// widening of the threshold and of the x-extent.
__device__ __forceinline__ EllipseBands ellipse_bands(float a, float b, float c, float sq) {
    EllipseBands E;
    E.ia = __builtin_amdgcn_rcpf(a);
    E.kx = b * E.ia;
    const float ic = __builtin_amdgcn_rcpf(c), bc = b * ic;
    E.eyR = sq * bc * ic * __builtin_amdgcn_rsqf(fmaf(bc, bc, 1.0f));
    E.hy = sq * ic;
    return E;
}

// The quadrant test in two parts.  band_extents (once per tile row of a
// record, from the centre's y offset uy in that row): per band j of eight
// pixel rows, the ellipse's x-extent as offsets from the centre's x before
// the margin, (a_j, b_j) = (xmax - ux, xmin - ux); a band no pixel row of
// which meets the ellipse gets (-inf, +inf).  quadrant_mask_ext (per tile of
// the row, from its ux): bit 2 j + i when the widened extent meets the pixel
// centres of column block i (x from 8 i + 0.5 to 8 i + 7.5).
__device__ __forceinline__ float4 band_extents(float uy, float kx, float ia, float c, float eyR, float hy, float qc) {
    float e[4];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const float lo = fmaxf(uy - (8.0f * j + 7.5f), -hy), hi = fminf(uy - (8.0f * j + 0.5f), hy);
        const float eR = __builtin_amdgcn_fmed3f(eyR, lo, hi), eL = __builtin_amdgcn_fmed3f(-eyR, lo, hi);
        const float tR = c * eR, tL = c * eL;
        const float sR = __builtin_amdgcn_sqrtf(fmaxf(fmaf(-tR, tR, qc), 0.0f));
        const float sL = __builtin_amdgcn_sqrtf(fmaxf(fmaf(-tL, tL, qc), 0.0f));
        const bool valid = lo <= hi;
        e[2 * j] = valid ? fmaf(sR, ia, kx * eR) : -__builtin_huge_valf();
        e[2 * j + 1] = valid ? fmaf(-sL, ia, kx * eL) : __builtin_huge_valf();
    }
    return make_float4(e[0], e[1], e[2], e[3]);
}

__device__ __forceinline__ uint32_t quadrant_mask_ext(float ux, const float4 &E) {
    const float mg = fmaf(1e-5f, fabsf(ux), 0.01f);
    const float xmax0 = (E.x + ux) + mg, xmin0 = (E.y + ux) - mg;
    const float xmax1 = (E.z + ux) + mg, xmin1 = (E.w + ux) - mg;
    uint32_t m = 0;
    m |= (xmax0 >= 0.5f && xmin0 <= 7.5f) ? 1u : 0u;
    m |= (xmax0 >= 8.5f && xmin0 <= 15.5f) ? 2u : 0u;
    m |= (xmax1 >= 0.5f && xmin1 <= 7.5f) ? 4u : 0u;
    m |= (xmax1 >= 8.5f && xmin1 <= 15.5f) ? 8u : 0u;
    return m;
}

// The same test for the sixteen 4 x 4 sub-blocks of the tile: bit 4 q + r is
// set when the ellipse reaches sub-block r (2 row + column inside the
// quadrant) of quadrant q, from four bands of four pixel rows and four blocks
// of four pixel columns, with the same widening.
__device__ __forceinline__ uint32_t subblock_mask_bands(float ux, float uy, float kx, float ia, float c, float eyR,
                                                        float hy, float qc) {
    const float mg = fmaf(1e-5f, fabsf(ux), 0.01f);
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float lo = fmaxf(uy - (4.0f * j + 3.5f), -hy), hi = fminf(uy - (4.0f * j + 0.5f), hy);
        const float eR = __builtin_amdgcn_fmed3f(eyR, lo, hi), eL = __builtin_amdgcn_fmed3f(-eyR, lo, hi);
        const float tR = c * eR, tL = c * eL;
        const float sR = __builtin_amdgcn_sqrtf(fmaxf(fmaf(-tR, tR, qc), 0.0f));
        const float sL = __builtin_amdgcn_sqrtf(fmaxf(fmaf(-tL, tL, qc), 0.0f));
        const float xmax = fmaf(sR, ia, fmaf(kx, eR, ux)) + mg;
        const float xmin = fmaf(-sL, ia, fmaf(kx, eL, ux)) - mg;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const bool in = lo <= hi && xmax >= 4.0f * i + 0.5f && xmin <= 4.0f * i + 3.5f;
            const int q = ((j >> 1) << 1) + (i >> 1), r = ((j & 1) << 1) + (i & 1);
            m |= in ? 1u << (4 * q + r) : 0u;
        }
    }
    return m;
}

}  // namespace gv
