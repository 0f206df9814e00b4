// Stencil walk shared by the pair kernels (rates and their adjoint): the
// rows of cells a particle's support sphere reaches, and the per-lane
// partner rings in LDS.
#pragma once

#include "csph_internal.h"

namespace csph {

// ---------------------------------------------------------------- partner queues
//
// A candidate test costs ~20 instructions, a pair interaction ~50.  Testing
// and interacting in the same loop would run the pair arithmetic whenever
// any lane of the wave accepts a candidate, with the other lanes idle (a
// particle accepts ~15-40 % of its candidates).  Instead each lane appends
// its accepted partners to a small ring in LDS while the wave walks the
// stencil in lock step, and as soon as some lane's ring is nearly full every
// lane pops one partner and the wave runs the pair arithmetic with (nearly)
// all lanes busy.  A lane's partners are summed in the order it popped them,
// which depends only on the input: results are reproducible.
//
// Each stencil row (cells cx-R..cx+R at fixed y, z) is clipped to the chord
// the support sphere of particle i cuts through it, with a safety margin,
// so that with cells smaller than the support the lanes test little more
// than the sphere.  The clipping only drops candidates that cannot be
// partners; membership is decided by the pair test itself.

constexpr int kQ = 8;  // ring slots per lane
constexpr int kU = 2;  // candidates tested per lock-step iteration

// Load base[idx] with a 32-bit byte offset from a wave-uniform base (records
// stay below 4 GiB), which keeps the address arithmetic in one VGPR.
template <typename T>
__device__ __forceinline__ T ld(const T *__restrict__ base, int idx) {
    return *(const T *)((const char *)base + (uint32_t)idx * (uint32_t)sizeof(T));
}

// Per-particle view of the stencil: cell, position in cell units, reach.
struct Stencil {
    int cx, cy, cz;
    float xc, yc, zc;  // (x - origin) / D
    float w2;          // (support/D)^2 with margin
    int R;
};

__device__ __forceinline__ Stencil make_stencil(const GridDev &g, double x, double y, double z,
                                                double H) {
    Stencil t;
    t.cx = cell_coord(x, g.ox, g.inv, g.dx);
    t.cy = cell_coord(y, g.oy, g.inv, g.dy);
    t.cz = cell_coord(z, g.oz, g.inv, g.dz);
    t.xc = (float)((x - g.ox) * g.inv);
    t.yc = (float)((y - g.oy) * g.inv);
    t.zc = (float)((z - g.oz) * g.inv);
    float hc = (float)(H * g.inv) * 1.0001f + 1e-3f;
    t.w2 = hc * hc;
    t.R = g.reach;
    return t;
}

// Stencil of the mirror image (x, y', z) of a particle across a wall plane
// normal to y (the kernels' y axis; see csph_internal.h): the image may lie
// off the mesh, so its y cell is not clamped (rows off the mesh are skipped);
// x, z, the chord centre and the reach are the particle's own.  Walking it
// visits every particle whose mirror image lies within the support of the
// particle, wherever the particles are relative to the wall.
__device__ __forceinline__ Stencil image_stencil(const GridDev &g, const Stencil &t,
                                                 double y_image) {
    Stencil s = t;
    const double f = floor((y_image - g.oy) * g.inv);
    s.cy = (int)fmin(fmax(f, -1048576.0), 1048576.0);
    s.yc = (float)((y_image - g.oy) * g.inv);
    return s;
}

// Periodic images (PairConst).  Faces of particle i: bit a set when axis a is periodic and i
// lies within the near-face band of one of its faces, bit 3 + a when that is the high face
// (shift k_a = -1) rather than the low one (k_a = +1).  An image is a non-empty mask m of
// such axes: the partners j at (x_j - k L) along the axes of m.
__device__ __forceinline__ int image_faces(const PairConst &pc, double x, double y, double z) {
    const double p[3] = {x, y, z};
    int f = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!((pc.per >> a) & 1)) continue;
        if (p[a] - pc.lo[a] < pc.hb)
            f |= 1 << a;
        else if (pc.hi[a] - p[a] < pc.hb)
            f |= 9 << a;
    }
    return f;
}

// k_a L_a of image m along axis a (0 when m does not shift axis a): the displacement to the
// image of j is d_a = (x_j,a - x_i,a) - k_a L_a, formed in that order.
__device__ __forceinline__ double image_shift(const PairConst &pc, int f, int m, int a) {
    return ((m >> a) & 1) ? (((f >> (3 + a)) & 1) ? -pc.L[a] : pc.L[a]) : 0.0;
}

// Cell index of coordinate v, not clamped to the mesh (an image point lies off it; rows off
// the mesh are skipped), bounded to keep the integer arithmetic finite.
__device__ __forceinline__ int free_cell(double v, double o, double inv) {
    return (int)fmin(fmax(floor((v - o) * inv), -1048576.0), 1048576.0);
}

// Stencil around the image point p = (x_i, y_i, z_i) + k L of image m, starting from stencil s
// (of i, or of its mirror image, whose y it keeps): the shifted axes take the point's own
// unclamped cells and chord centres.
__device__ __forceinline__ Stencil shifted_stencil(const GridDev &g, Stencil s, int m, double px,
                                                   double py, double pz) {
    if (m & 1) {
        s.cx = free_cell(px, g.ox, g.inv);
        s.xc = (float)((px - g.ox) * g.inv);
    }
    if (m & 2) {
        s.cy = free_cell(py, g.oy, g.inv);
        s.yc = (float)((py - g.oy) * g.inv);
    }
    if (m & 4) {
        s.cz = free_cell(pz, g.oz, g.inv);
        s.zc = (float)((pz - g.oz) * g.inv);
    }
    return s;
}

// Whether a particle at y can have mirror partners within support H: some
// particle's image 2 yw - y_j lies within H of it.  The images lie at or below
// yw + (yw - min_j y_j), so particles behind the wall widen the band in front of it.
__device__ __forceinline__ bool mirror_band(const GridDev &g, double y, double yw, double H) {
    const double ymin = g.yenc ? order_dec(*g.yenc) : g.ymin;
    return y - yw < H + fmax(yw - ymin, 0.0);
}

// Distance in cell units from coordinate c to the slab [k, k+1) (0 inside),
// shrunk by a margin.
__device__ __forceinline__ float slab_gap(float c, int k) {
    float d = fmaxf(fmaxf((float)k - c, c - (float)(k + 1)), 0.0f);
    return fmaxf(d - 1e-3f, 0.0f);
}

// Candidate range [j0, j0+len) of row (yy, zz) for a particle (or its
// image): the cells of the row within the chord its support sphere cuts
// through the row.  gz2 = squared z gap.  Branch-free per lane; a row off the
// mesh or missing the sphere gets len = 0, and when it does so for every lane
// of the wave the cell-range loads are skipped.
__device__ __forceinline__ void row_range(const int32_t *__restrict__ cs, const GridDev &g,
                                          const Stencil &t, bool on, int yy, int zz, float gz2,
                                          int &j0, int &len) {
    const bool inb = on && zz >= 0 && zz < g.dz && yy >= 0 && yy < g.dy;
    const float gy = slab_gap(t.yc, yy);
    const float rem = t.w2 - (gy * gy + gz2);
    // chord half-width; v_sqrt_f32 (1 ulp) is ample under the margins
    const float hw = __builtin_amdgcn_sqrtf(fmaxf(rem, 0.0f)) * 1.0001f + 1e-3f;
    const int xa = max(max((int)floorf(t.xc - hw), t.cx - t.R), 0);
    const int xb = min(min((int)floorf(t.xc + hw), t.cx + t.R), g.dx - 1);
    const bool ok = inb && rem > 0.0f && xb >= xa;
    j0 = 0;
    len = 0;
    if (__any(ok)) {
        const int row = (int)cell_key(g, 0, yy, zz);
        const int ia = ok ? row + xa : 0, ib = ok ? row + xb + 1 : 0;
        j0 = ld(cs, ia);
        len = ld(cs, ib) - j0;
    }
}

}  // namespace csph
