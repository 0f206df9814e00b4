// Neighbour-set export N(i) = { j != i : |r_j - r_i|^2 < H_ij^2 } (sec. 4.1)
// as CSR over input indices, rows ascending.  Verification form only: the
// rate kernels gather partners on the fly and never materialise this list.
// The test is the FP64 expression ((dx*dx)+(dy*dy))+(dz*dz) < H*H without
// contraction, so membership is exact.  With periodic axes the partners
// include the periodic images, d = (r_j - r_i) - k L (each j appears once:
// the periods exceed twice the support).
#include "csph_internal.h"
#include "stencil.h"

namespace csph {

__global__ __launch_bounds__(kBlock) void k_gather_pos(int64_t n, const int32_t *__restrict__ perm,
                                                       const double *__restrict__ x,
                                                       const double *__restrict__ y,
                                                       const double *__restrict__ z,
                                                       const double *__restrict__ d,
                                                       double *__restrict__ xs,
                                                       double *__restrict__ ys,
                                                       double *__restrict__ zs,
                                                       double *__restrict__ ds) {
    int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    int i = perm[s];
    xs[s] = x[i];
    ys[s] = y[i];
    zs[s] = z[i];
    if (d) ds[s] = d[i];
}

hipError_t launch_gather_pos(int64_t n, const int32_t *perm, const double *x, const double *y,
                             const double *z, const double *d, const Ws &w, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_gather_pos<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        n, perm, x, y, z, d, w.srt[0], w.srt[1], w.srt[2], w.srt_d);
    return hipGetLastError();
}

// In-place heapsort of a[0..c) ascending (a max-heap, then the maximum moved to the end).
__device__ __forceinline__ void sift_down(int32_t *a, int root, int end) {
    const int v = a[root];
    for (;;) {
        int ch = 2 * root + 1;
        if (ch >= end) break;
        if (ch + 1 < end && a[ch + 1] > a[ch]) ++ch;
        if (a[ch] <= v) break;
        a[root] = a[ch];
        root = ch;
    }
    a[root] = v;
}

__device__ void heap_sort(int32_t *a, int c) {
    for (int r = c / 2 - 1; r >= 0; --r) sift_down(a, r, c);
    for (int e = c - 1; e > 0; --e) {
        const int t = a[0];
        a[0] = a[e];
        a[e] = t;
        sift_down(a, 0, e);
    }
}

template <bool PAIR, bool FILL, bool PER>
__global__ __launch_bounds__(kBlock) void k_nbr(int64_t n, GridDev g, PairConst pc,
                                                const double *__restrict__ x,
                                                const double *__restrict__ y,
                                                const double *__restrict__ z,
                                                const double *__restrict__ d,
                                                const int32_t *__restrict__ cs,
                                                const int32_t *__restrict__ perm,
                                                int32_t *__restrict__ count_orig,
                                                const int64_t *__restrict__ offsets,
                                                int32_t *__restrict__ idx) {
    int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    double xi = x[s], yi = y[s], zi = z[s];
    double di = PAIR ? d[s] : 0.0;
    const int R = g.reach;
    const int nf = PER ? image_faces(pc, xi, yi, zi) : 0;
    int i = perm[s];
    int64_t wpos = FILL ? offsets[i] : 0;
    int cnt = 0;
    // image m = 0: i itself; m > 0: the periodic image of i across the faces of mask m
    for (int m = 0; m < (PER ? 8 : 1); ++m) {
        if ((nf & m) != m) continue;
        const double shx = image_shift(pc, nf, m, 0), shy = image_shift(pc, nf, m, 1),
                     shz = image_shift(pc, nf, m, 2);
        const int cx = m & 1 ? free_cell(xi + shx, g.ox, g.inv) : cell_coord(xi, g.ox, g.inv, g.dx);
        const int cy = m & 2 ? free_cell(yi + shy, g.oy, g.inv) : cell_coord(yi, g.oy, g.inv, g.dy);
        const int cz = m & 4 ? free_cell(zi + shz, g.oz, g.inv) : cell_coord(zi, g.oz, g.inv, g.dz);
        const int x0 = max(cx - R, 0), x1 = min(cx + R, g.dx - 1);
        if (x0 > x1) continue;
        for (int oz = -R; oz <= R; ++oz) {
            int zz = cz + oz;
            if (zz < 0 || zz >= g.dz) continue;
            for (int oy = -R; oy <= R; ++oy) {
                int yy = cy + oy;
                if (yy < 0 || yy >= g.dy) continue;
                int row = (int)cell_key(g, 0, yy, zz);
                int j0 = cs[row + x0], j1 = cs[row + x1 + 1];
                for (int j = j0; j < j1; ++j) {
                    if (m == 0 && j == (int)s) continue;
                    double dx = x[j] - xi, dy = y[j] - yi, dz = z[j] - zi;
                    if (PER) {
                        dx = dx - shx;
                        dy = dy - shy;
                        dz = dz - shz;
                    }
                    double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
                    double H2;
                    if (PAIR) {
                        double H = pc.kappa * (0.5 * (di + d[j]));
                        H2 = H * H;
                    } else {
                        H2 = pc.H2;
                    }
                    if (r2 < H2) {
                        if (FILL) idx[wpos + cnt] = perm[j];
                        ++cnt;
                    }
                }
            }
        }
    }
    if (FILL) heap_sort(idx + wpos, cnt);  // the row ascending, O(c log c)
    if (!FILL) count_orig[i] = cnt;
}

hipError_t launch_nbr_count(int64_t n, const GridDev &g, const PairConst &pc, const double *x,
                            const double *y, const double *z, const double *d, const int32_t *cs,
                            const int32_t *perm, int32_t *count_orig, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
#define CSPH_NBR(P, X)                                                                    \
    if (!!pc.pair_mode == P && !!pc.per == X)                                             \
        k_nbr<P, false, X><<<nb, kBlock, 0, st>>>(n, g, pc, x, y, z, d, cs, perm, count_orig, \
                                                  nullptr, nullptr);
    CSPH_NBR(false, false)
    CSPH_NBR(true, false)
    CSPH_NBR(false, true)
    CSPH_NBR(true, true)
#undef CSPH_NBR
    return hipGetLastError();
}

hipError_t launch_nbr_fill(int64_t n, const GridDev &g, const PairConst &pc, const double *x,
                           const double *y, const double *z, const double *d, const int32_t *cs,
                           const int32_t *perm, const int64_t *offsets, int32_t *idx,
                           hipStream_t st) {
    if (n <= 0) return hipSuccess;
    unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
#define CSPH_NBR(P, X)                                                                    \
    if (!!pc.pair_mode == P && !!pc.per == X)                                             \
        k_nbr<P, true, X><<<nb, kBlock, 0, st>>>(n, g, pc, x, y, z, d, cs, perm, nullptr,    \
                                                 offsets, idx);
    CSPH_NBR(false, false)
    CSPH_NBR(true, false)
    CSPH_NBR(false, true)
    CSPH_NBR(true, true)
#undef CSPH_NBR
    return hipGetLastError();
}

}  // namespace csph
