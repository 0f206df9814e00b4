// Verlet lists (sec. 4.2): for each particle, in cell order, the partners
// within the horizon R = (1 + beta) H, found on the chord-clipped stencil rows
// of the cell mesh with the exact FP64 test r^2 < R^2 (no contraction), plus
// mirror partners across the piston wall (sign bit set; the wall is normal to
// the kernels' y axis, and they are found on the stencil around the image of
// the particle).  A step then tests
// only the listed partners (r^2 < H^2), which gives N(i) exactly while no
// pair can have closed in from beyond R; the displacement kernel below feeds
// the caller's rebuild test.
#include "csph_internal.h"
#include "stencil.h"

namespace csph {

template <bool WALL>
__global__ __launch_bounds__(kBlock) void k_vlist(int64_t n, const double4 *__restrict__ A,
                                                  const int32_t *__restrict__ cs, GridDev g,
                                                  double R, double R2, double yw, int cap,
                                                  int32_t *__restrict__ count,
                                                  int32_t *__restrict__ idx,
                                                  unsigned long long *__restrict__ over) {
    // each lane gathers a chunk of 8 entries in LDS and stores it whole (two 16-byte stores)
    // instead of one scattered 4-byte store per entry
    __shared__ int stg[kBlock][kVlChunk];
    const int64_t s = xcd_block<64>(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const bool live = s < n;
    const double4 ai = live ? A[s] : make_double4(0.0, 0.0, 0.0, 0.0);
    const double xi = ai.x, yi = ai.y, zi = ai.z;
    const Stencil t = make_stencil(g, xi, yi, zi, R);
    const Stencil ti = WALL ? image_stencil(g, t, 2.0 * yw - yi) : t;
    const bool near = WALL && live && mirror_band(g, yi, yw, R);
    // blocked: entry c of particle s at idx[((c / 8) n + s) 8 + c % 8]; one lane fills whole
    // 32-byte chunks and a wave reading its lanes' entry c touches 16 cache lines
    static_assert(kVlChunk == 8, "a chunk is two int4");
    int4 *chunk = (int4 *)(idx + (live ? s * kVlChunk : 0));  // the lane's chunk c / 8
    const int64_t cstride = n * kVlChunk / 4;                   // int4s from one chunk to the next
    int *stage = stg[threadIdx.x];
    int c = 0;
    for (int pass = 0; pass < (WALL ? 2 : 1); ++pass) {
        const bool ghost = pass == 1;
        if (ghost && !__any(near)) break;
        const bool on = live && (!ghost || near);
        // mirror partners: the particles on the stencil around the image of i
        const Stencil &st = ghost ? ti : t;
        int oy = st.R, oz = -st.R - 1;
        int k = 0, j0 = 0, len = 0, jlast = 0;
        for (;;) {
            if (!__any(k < len)) {
                if (++oy > st.R) {
                    oy = -st.R;
                    if (++oz > st.R) break;
                }
                const int zz = st.cz + oz;
                const float gz = slab_gap(st.zc, zz);
                row_range(cs, g, st, on, st.cy + oy, zz, gz * gz, j0, len);
                jlast = len > 0 ? j0 + len - 1 : 0;
                k = 0;
                continue;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int j = min(j0 + k + u, jlast);
                const double4 aj = ld(A, j);
                const double yj = ghost ? 2.0 * yw - aj.y : aj.y;
                const double dx = aj.x - xi, dy = yj - yi, dz = aj.z - zi;
                const double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
                const bool acc = (k + u < len) && (ghost || j != (int)s) && r2 < R2;
                if (acc) {
                    stage[c & (kVlChunk - 1)] = ghost ? (j | (int)0x80000000) : j;
                    ++c;
                    if ((c & (kVlChunk - 1)) == 0) {  // chunk full: store it (within cap)
                        if (c <= cap) {
                            chunk[0] = make_int4(stage[0], stage[1], stage[2], stage[3]);
                            chunk[1] = make_int4(stage[4], stage[5], stage[6], stage[7]);
                        }
                        chunk += cstride;
                    }
                }
            }
            k += kU;
        }
    }
    if (live) {
        // the last, partly filled chunk (entries past the count are never read)
        if ((c & (kVlChunk - 1)) != 0 && c < cap) {
            chunk[0] = make_int4(stage[0], stage[1], stage[2], stage[3]);
            chunk[1] = make_int4(stage[4], stage[5], stage[6], stage[7]);
        }
        count[s] = c;
        if (c > cap) atomicMax(over, (unsigned long long)c);
    }
}

// max_i |r_i - r_ref,i| into *out (bits of a non-negative double; *out zeroed first).
__global__ __launch_bounds__(kBlock) void k_disp(int64_t n, const double *__restrict__ x,
                                                 const double *__restrict__ y,
                                                 const double *__restrict__ z,
                                                 const double *__restrict__ ref,
                                                 unsigned long long *__restrict__ out,
                                                 const int32_t *__restrict__ gate) {
    if (gate && *gate == 0) return;
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const double dx = x[i] - ref[i], dy = y[i] - ref[n + i], dz = z[i] - ref[2 * n + i];
        const double d = sqrt(((dx * dx) + (dy * dy)) + (dz * dz));
        m = d > m ? d : m;  // a NaN position leaves m as it is; positions are checked finite
    }
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    __shared__ double sh[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = sh[0];
        for (int q = 1; q < kBlock / 64; ++q) r = fmax(r, sh[q]);
        atomicMax(out, dbits(r));
    }
}

hipError_t launch_vlist(int64_t n, const double4 *A, const int32_t *cs, const GridDev &g,
                        double R, int wall, double yw, int cap, int32_t *count, int32_t *idx,
                        unsigned long long *over, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    const double R2 = R * R;
    if (wall)
        k_vlist<true><<<nb, kBlock, 0, st>>>(n, A, cs, g, R, R2, yw, cap, count, idx, over);
    else
        k_vlist<false><<<nb, kBlock, 0, st>>>(n, A, cs, g, R, R2, yw, cap, count, idx, over);
    return hipGetLastError();
}

hipError_t launch_disp(int64_t n, const double *x, const double *y, const double *z,
                       const double *ref, unsigned long long *out, hipStream_t st,
                       const int32_t *gate) {
    if (n <= 0) return hipSuccess;
    int64_t want = (n + kBlock - 1) / kBlock;
    unsigned nb = (unsigned)(want > kReduceBlocks ? kReduceBlocks : want);
    k_disp<<<nb, kBlock, 0, st>>>(n, x, y, z, ref, out, gate);
    return hipGetLastError();
}

// ---------------------------------------------------------------- list control block

__global__ void k_vl_init(csph_vlist_ctl *ctl, const double *t, double margin, double vw2) {
    ctl->t_build = t ? *t : 0.0;
    ctl->disp = 0.0;
    ctl->margin = margin;
    ctl->vw2 = vw2;
    ctl->pairs = 0;
    ctl->steps = 0;
    ctl->valid = 1;
}

// Before a list step: the lists give N(i) exactly while no pair can have entered the support
// from beyond the horizon, 2 max|r - r_ref| + 2 |v_wall| (t - t_build) < beta H (the first
// step after a build sees the build's own positions and wall); once that fails the lists stay
// stale until the next build.  A passing step's displacement is then taken afresh.
__global__ void k_vl_guard(csph_vlist_ctl *ctl, const double *t) {
    const double tt = t ? *t : ctl->t_build;
    const bool ok = ctl->valid != 0 &&
                    (ctl->steps == 0 ||
                     2.0 * ctl->disp + ctl->vw2 * (tt - ctl->t_build) < ctl->margin);
    ctl->valid = ok ? 1 : 0;
    if (ok) ctl->disp = 0.0;
}

hipError_t launch_vl_init(csph_vlist_ctl *ctl, const double *t, double margin, double vw2,
                          hipStream_t st) {
    k_vl_init<<<1, 1, 0, st>>>(ctl, t, margin, vw2);
    return hipGetLastError();
}

hipError_t launch_vl_guard(csph_vlist_ctl *ctl, const double *t, hipStream_t st) {
    k_vl_guard<<<1, 1, 0, st>>>(ctl, t);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_copy_i32(int32_t *__restrict__ dst,
                                                     const int32_t *__restrict__ src, int64_t n,
                                                     const int32_t *__restrict__ gate) {
    if (gate && *gate == 0) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

hipError_t launch_copy_i32(int32_t *dst, const int32_t *src, int64_t n, const int32_t *gate,
                           hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_copy_i32<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(dst, src, n, gate);
    return hipGetLastError();
}

}  // namespace csph
