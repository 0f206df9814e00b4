// Mesh bounds, cell keys, counting sort into cell order, cell ranges.
//
// Cell-ordered numbering is the GPU form of the linked-list cells and the
// locality renumbering of sec. 4.2: a counting sort by cell key.  Keys are
// histogrammed with integer atomics (each particle also gets a provisional
// rank inside its cell), an exclusive scan of the histogram gives the cell
// ranges, a scatter places every particle in its cell's segment, and each
// particle's final place in the segment is the number of the segment's
// particles with a smaller input index, so the order is exactly the stable
// order by (key, input index) whatever order the atomics ran in.
#include "csph_internal.h"
#include "hostsync.h"

namespace csph {

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// part[b*8 + {0..6}] = min x, min y, min z, max x, max y, max z, max d.
__global__ __launch_bounds__(kBlock) void k_bounds(const double *__restrict__ x,
                                                   const double *__restrict__ y,
                                                   const double *__restrict__ z,
                                                   const double *__restrict__ d, int64_t n,
                                                   double *__restrict__ part) {
    double v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        double a = x[i], b = y[i], c = z[i];
        v[0] = fmin(v[0], a); v[1] = fmin(v[1], b); v[2] = fmin(v[2], c);
        v[3] = fmax(v[3], a); v[4] = fmax(v[4], b); v[5] = fmax(v[5], c);
        if (d) v[6] = fmax(v[6], d[i]);
    }
    __shared__ double sh[kBlock / 64][7];
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = 0; k < 7; ++k) {
        double r = k < 3 ? wave_min(v[k]) : wave_max(v[k]);
        if (lane == 0) sh[wid][k] = r;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        int k = threadIdx.x;
        double r = sh[0][k];
        for (int q = 1; q < kBlock / 64; ++q) r = k < 3 ? fmin(r, sh[q][k]) : fmax(r, sh[q][k]);
        part[blockIdx.x * 8 + k] = r;
    }
}

__global__ __launch_bounds__(kBlock) void k_bounds_final(const double *__restrict__ part,
                                                         int nblocks, double *__restrict__ out) {
    double v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += kBlock)
        for (int k = 0; k < 7; ++k)
            v[k] = k < 3 ? fmin(v[k], part[b * 8 + k]) : fmax(v[k], part[b * 8 + k]);
    __shared__ double sh[kBlock / 64][7];
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = 0; k < 7; ++k) {
        double r = k < 3 ? wave_min(v[k]) : wave_max(v[k]);
        if (lane == 0) sh[wid][k] = r;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        int k = threadIdx.x;
        double r = sh[0][k];
        for (int q = 1; q < kBlock / 64; ++q) r = k < 3 ? fmin(r, sh[q][k]) : fmax(r, sh[q][k]);
        out[k] = r;
    }
}

// k_bounds_final, also writing the result to the host's pinned slot: each value with a
// system-scope fence, then (after the workgroup barrier) the sequence number with a
// system-scope release, which the host polls.
__global__ __launch_bounds__(kBlock) void k_bounds_final_host(const double *__restrict__ part,
                                                              int nblocks,
                                                              double *__restrict__ out,
                                                              HostBounds *hb,
                                                              unsigned long long seq) {
    double v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += kBlock)
        for (int k = 0; k < 7; ++k)
            v[k] = k < 3 ? fmin(v[k], part[b * 8 + k]) : fmax(v[k], part[b * 8 + k]);
    __shared__ double sh[kBlock / 64][7];
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = 0; k < 7; ++k) {
        double r = k < 3 ? wave_min(v[k]) : wave_max(v[k]);
        if (lane == 0) sh[wid][k] = r;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        int k = threadIdx.x;
        double r = sh[0][k];
        for (int q = 1; q < kBlock / 64; ++q) r = k < 3 ? fmin(r, sh[q][k]) : fmax(r, sh[q][k]);
        out[k] = r;
        hb->b[k] = r;
        __threadfence_system();
    }
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(&hb->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_bounds_host(const double *x, const double *y, const double *z,
                              const double *d, int64_t n, double *part, double *out,
                              HostBounds *hb, unsigned long long seq, hipStream_t st) {
    int64_t want = (n + kBlock - 1) / kBlock;
    int nb = (int)(want < 1 ? 1 : (want > kReduceBlocks ? kReduceBlocks : want));
    k_bounds<<<nb, kBlock, 0, st>>>(x, y, z, d, n, part);
    k_bounds_final_host<<<1, kBlock, 0, st>>>(part, nb, out, hb, seq);
    return hipGetLastError();
}

__global__ void k_word_host(const unsigned long long *__restrict__ src, HostBounds *hb,
                            unsigned long long seq) {
    if (threadIdx.x != 0) return;
    ((unsigned long long *)hb->b)[0] = *src;
    __hip_atomic_store(&hb->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_word_host(const unsigned long long *src, HostBounds *hb,
                            unsigned long long seq, hipStream_t st) {
    k_word_host<<<1, 64, 0, st>>>(src, hb, seq);
    return hipGetLastError();
}

hipError_t launch_bounds(const double *x, const double *y, const double *z, const double *d,
                         int64_t n, double *part, double *out, hipStream_t st) {
    int64_t want = (n + kBlock - 1) / kBlock;
    int nb = (int)(want < 1 ? 1 : (want > kReduceBlocks ? kReduceBlocks : want));
    k_bounds<<<nb, kBlock, 0, st>>>(x, y, z, d, n, part);
    k_bounds_final<<<1, kBlock, 0, st>>>(part, nb, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- exclusive scan

template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *lds, T &total) {
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T x = v;
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int k = 0; k < kBlock / 64; ++k) {
            T t = lds[k];
            lds[k] = run;
            run += t;
        }
        lds[kBlock / 64] = run;
    }
    __syncthreads();
    T excl = (x - v) + lds[wid];
    total = lds[kBlock / 64];
    __syncthreads();
    return excl;
}

template <typename TI>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const TI *__restrict__ in, int64_t len,
                                                        int64_t *__restrict__ tile_sum, int vec) {
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
    const int64_t own = base + (int64_t)threadIdx.x * kScanItems;  // the apply pass's layout
    if (sizeof(TI) == 4 && vec && own + kScanItems <= len) {
        const int4 a = ((const int4 *)(in + own))[0], b = ((const int4 *)(in + own))[1];
        s = (((int64_t)a.x + a.y) + ((int64_t)a.z + a.w)) + (((int64_t)b.x + b.y) + ((int64_t)b.z + b.w));
    } else {
        for (int k = 0; k < kScanItems; ++k) {
            int64_t i = own + k;
            if (i < len) s += (int64_t)in[i];
        }
    }
    __shared__ int64_t lds[kBlock / 64 + 1];
    int64_t total;
    block_exclusive_scan<int64_t>(s, lds, total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// Exclusive scan of the tile sums in one workgroup; out[len] = grand total.  Each thread
// takes a run of consecutive tiles, so one workgroup scan covers them all.
template <typename TO>
__global__ __launch_bounds__(kBlock) void k_scan_tops(int64_t *__restrict__ tile_sum,
                                                      int64_t ntiles, TO *__restrict__ out,
                                                      int64_t len) {
    __shared__ int64_t lds[kBlock / 64 + 1];
    const int64_t per = (ntiles + kBlock - 1) / kBlock;
    const int64_t a = (int64_t)threadIdx.x * per, b = a + per < ntiles ? a + per : ntiles;
    int64_t s = 0;
    for (int64_t i = a; i < b; ++i) s += tile_sum[i];
    int64_t total;
    int64_t run = block_exclusive_scan<int64_t>(s, lds, total);
    for (int64_t i = a; i < b; ++i) {
        const int64_t v = tile_sum[i];
        tile_sum[i] = run;
        run += v;
    }
    if (threadIdx.x == 0) out[len] = (TO)total;
}

// vec: in and out are 16-byte aligned 32-bit arrays; a thread's kScanItems = 8 values then move
// as two 16-byte loads and stores (the tail tile goes element by element).
template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_scan_apply(const TI *in, TO *out, int64_t len,
                                                       const int64_t *__restrict__ tile_off,
                                                       int vec) {
    static_assert(kScanItems == 8, "two 16-byte vectors per thread");
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    const bool wide = sizeof(TI) == 4 && sizeof(TO) == 4 && vec && base + kScanItems <= len;
    int64_t v[kScanItems];
    int64_t s = 0;
    if (wide) {
        const int4 a = ((const int4 *)(in + base))[0], b = ((const int4 *)(in + base))[1];
        const int w[kScanItems] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        for (int k = 0; k < kScanItems; ++k) v[k] = w[k];
    } else {
        for (int k = 0; k < kScanItems; ++k) {
            int64_t i = base + k;
            v[k] = i < len ? (int64_t)in[i] : 0;
        }
    }
    for (int k = 0; k < kScanItems; ++k) s += v[k];
    __shared__ int64_t lds[kBlock / 64 + 1];
    int64_t total;
    int64_t run = block_exclusive_scan<int64_t>(s, lds, total) + tile_off[blockIdx.x];
    if (wide) {
        int o[kScanItems];
        for (int k = 0; k < kScanItems; ++k) {
            o[k] = (int)run;
            run += v[k];
        }
        ((int4 *)(out + base))[0] = make_int4(o[0], o[1], o[2], o[3]);
        ((int4 *)(out + base))[1] = make_int4(o[4], o[5], o[6], o[7]);
    } else {
        for (int k = 0; k < kScanItems; ++k) {
            int64_t i = base + k;
            if (i < len) out[i] = (TO)run;
            run += v[k];
        }
    }
}

// out[0..len) = exclusive prefix sums of in[0..len), out[len] = total.
// in may alias out when TI == TO.  tmp holds ceil(len / kScanTile) int64.
template <typename TI, typename TO>
hipError_t launch_scan_exclusive(const TI *in, TO *out, int64_t len, int64_t *tmp,
                                 hipStream_t st) {
    int64_t ntiles = (len + kScanTile - 1) / kScanTile;
    const int vec = ((uintptr_t)in % 16 == 0) && ((uintptr_t)out % 16 == 0);
    if (ntiles > 0) k_scan_reduce<TI><<<(unsigned)ntiles, kBlock, 0, st>>>(in, len, tmp, vec);
    k_scan_tops<TO><<<1, kBlock, 0, st>>>(tmp, ntiles, out, len);
    if (ntiles > 0)
        k_scan_apply<TI, TO><<<(unsigned)ntiles, kBlock, 0, st>>>(in, out, len, tmp, vec);
    return hipGetLastError();
}

template hipError_t launch_scan_exclusive<int32_t, int32_t>(const int32_t *, int32_t *, int64_t,
                                                            int64_t *, hipStream_t);
template hipError_t launch_scan_exclusive<int32_t, int64_t>(const int32_t *, int64_t *, int64_t,
                                                            int64_t *, hipStream_t);

// ---------------------------------------------------------------- counting sort by cell

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t *p, int32_t v, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

// Whether coordinate v lies on the mesh axis (origin o, 1/D inv, dim cells), in the cell
// arithmetic of cell_coord.
__device__ __forceinline__ bool on_axis(double v, double o, double inv, int dim) {
    const double f = floor((v - o) * inv);
    return f >= 0.0 && f < (double)dim;
}

__global__ __launch_bounds__(kBlock) void k_keys(const double *__restrict__ x,
                                                 const double *__restrict__ y,
                                                 const double *__restrict__ z, int64_t n,
                                                 GridDev g, uint32_t *__restrict__ key,
                                                 uint32_t *__restrict__ rank,
                                                 int32_t *__restrict__ count,
                                                 uint32_t *__restrict__ key_out, BinCheck chk) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool live = i < n;
    double xi = 0.0, yi = 0.0, zi = 0.0;
    if (live) {
        xi = x[i];
        yi = y[i];
        zi = z[i];
        int cx = cell_coord(xi, g.ox, g.inv, g.dx);
        int cy = cell_coord(yi, g.oy, g.inv, g.dy);
        int cz = cell_coord(zi, g.oz, g.inv, g.dz);
        uint32_t k = g.morton ? morton_key(cx, cy, cz) : cell_key(g, cx, cy, cz);
        key[i] = k;
        rank[i] = (uint32_t)atomicAdd(&count[k], 1);
        if (key_out) key_out[i] = k;
    }
    if (chk.yenc) {  // the wave's minimum y, one atomic per wave
        unsigned long long e = live ? order_enc(yi) : ~0ull;
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long f = __shfl_xor(e, o, 64);
            e = f < e ? f : e;
        }
        if ((threadIdx.x & 63) == 0 && e != ~0ull) atomicMin(chk.yenc, e);
    }
    if (chk.outside) {
        bool out = live && !(on_axis(xi, g.ox, g.inv, g.dx) && on_axis(yi, g.oy, g.inv, g.dy) &&
                             on_axis(zi, g.oz, g.inv, g.dz));
        const double p[3] = {xi, yi, zi};
        for (int a = 0; a < 3; ++a)
            if (live && ((chk.per >> a) & 1) && !(p[a] >= chk.lo[a] && p[a] <= chk.hi[a]))
                out = true;
        const unsigned long long c = __popcll(__ballot(out));
        if ((threadIdx.x & 63) == 0 && c) atomicAdd(chk.outside, c);
    }
}

__global__ __launch_bounds__(kBlock) void k_scatter(const uint32_t *__restrict__ key,
                                                    const uint32_t *__restrict__ rank,
                                                    const int32_t *__restrict__ cs, int64_t n,
                                                    int32_t *__restrict__ tmp) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    tmp[cs[key[i]] + (int32_t)rank[i]] = (int32_t)i;
}

// Final place of the particle in slot s of the scattered order: its cell segment's start plus
// the number of the segment's particles with a smaller input index.  O(k) per particle for a
// cell of k particles, all particles in parallel (an in-cell sort by one thread per cell would
// cost O(k^2) for a dense cell).
__global__ __launch_bounds__(kBlock) void k_cell_rank(const uint32_t *__restrict__ key,
                                                      const int32_t *__restrict__ cs, int64_t n,
                                                      const int32_t *__restrict__ tmp,
                                                      int32_t *__restrict__ perm) {
    int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const int p = tmp[s];
    const uint32_t k = key[p];
    const int a = cs[k], b = cs[k + 1];
    int r = 0;
    for (int t = a; t < b; ++t) r += tmp[t] < p ? 1 : 0;
    perm[a + r] = p;
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_bin(const double *x, const double *y, const double *z, int64_t n,
                      const GridDev &g, const Ws &w, int32_t *perm, uint32_t *key_out,
                      int32_t *cell_start, hipStream_t st, const BinCheck *chk) {
    const BinCheck c = chk ? *chk : BinCheck{nullptr, nullptr, 0, {0, 0, 0}, {0, 0, 0}};
    const int64_t ncell = g.nkey;  // keys (cells, or the Morton key space)
    unsigned fb = blocks_for(ncell + 1);
    k_fill_i32<<<fb > 65535u ? 65535u : fb, kBlock, 0, st>>>(cell_start, 0, ncell + 1);
    if (n > 0)
        k_keys<<<blocks_for(n), kBlock, 0, st>>>(x, y, z, n, g, w.key, w.rank, cell_start,
                                                 key_out, c);
    hipError_t e = launch_scan_exclusive<int32_t, int32_t>(cell_start, cell_start, ncell,
                                                           w.scan_tmp, st);
    if (e != hipSuccess) return e;
    if (n > 0) {
        k_scatter<<<blocks_for(n), kBlock, 0, st>>>(w.key, w.rank, cell_start, n, w.bin_tmp);
        k_cell_rank<<<blocks_for(n), kBlock, 0, st>>>(w.key, cell_start, n, w.bin_tmp, perm);
    }
    return hipGetLastError();
}

}  // namespace csph
