// Voronoi load balancer (sec. 3): subdomain statistics and one generator move.
//
// Statistics (one pass over the particles, generators in LDS):
//   * particle and pair loads per subdomain (integers);
//   * geometric centres (eq. VoronoiGeomCenters) from fixed-point sums: each
//     particle adds round((x - g_k) * 2^32) (|x - g_k| < 2^24) to a 128-bit
//     integer per coordinate, so the sums are exact and do not depend on the
//     order in which the atomics run;
//   * which subdomains touch: a particle owned by k whose nearest other
//     generator l lies within D^sh of the k|l bisector plane marks (k, l) and
//     (l, k) in a K x K bit matrix (the same FP64 expressions as the CPU
//     reference, no contraction, so the bits are exact).
// Move (one workgroup, one thread per generator): two-body displacement
// (eq. BalancingOffset), three-body rotations about the circumcentre of each
// triplet of mutually touching subdomains (eqs. BalancingOffsetPlusRot,
// BalancingOffsetRot) with the shift capped at D^sh, and the cumulative
// movement (eq. TotalOffset); the sum of |g' - g| (eq. VDConvergence) is
// reduced in a fixed order.
#include "csph_internal.h"

namespace csph {

// defined with the Voronoi and binning kernels
__global__ void k_zero_u64(unsigned long long *p, int count);
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t count);

constexpr double kFix = 4294967296.0;  // 2^32: fixed-point scale of the centre sums
constexpr double kFixMax = 72057594037927936.0;  // 2^56: per-particle bound (|x - g| < 2^24)

// 128-bit two's-complement accumulator {lo, hi}: add a signed 64-bit value.
__device__ __forceinline__ void add128(unsigned long long *lo, unsigned long long *hi, long long v) {
    const unsigned long long u = (unsigned long long)v;
    const unsigned long long old = atomicAdd(lo, u);
    const unsigned long long carry = (old + u < old) ? 1ull : 0ull;
    const unsigned long long ext = v < 0 ? ~0ull : 0ull;
    const unsigned long long h = ext + carry;
    if (h) atomicAdd(hi, h);
}

__global__ __launch_bounds__(kBlock) void k_balance_stats(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    int64_t n, const int32_t *__restrict__ owner, const int32_t *__restrict__ nbr_count,
    const double *__restrict__ sites, int K, int W, double dsh,
    unsigned long long *__restrict__ g_part, unsigned long long *__restrict__ g_pairs,
    unsigned long long *__restrict__ g_sum, uint32_t *__restrict__ adj) {
    extern __shared__ double smem[];
    double *gs = smem;                                                   // 3K
    unsigned long long *s_lo = (unsigned long long *)(gs + 3 * K);       // 3K
    unsigned long long *s_hi = s_lo + 3 * K;                             // 3K
    unsigned long long *s_pairs = s_hi + 3 * K;                          // K
    unsigned int *s_part = (unsigned int *)(s_pairs + K);                // K
    for (int k = threadIdx.x; k < 3 * K; k += kBlock) {
        gs[k] = sites[k];
        s_lo[k] = 0ull;
        s_hi[k] = 0ull;
    }
    for (int k = threadIdx.x; k < K; k += kBlock) {
        s_pairs[k] = 0ull;
        s_part[k] = 0u;
    }
    __syncthreads();
    const double lim = 4.0 * (dsh * dsh);
    // wave-uniform grid-stride loop: every lane of a wave takes part in the shuffles
    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n;
         base += (int64_t)gridDim.x * kBlock) {
        const int64_t i = base + threadIdx.x;
        const int kr = i < n ? owner[i] : -1;
        const bool ok = kr >= 0 && kr < K;
        const int k = ok ? kr : 0;
        double p[3] = {0.0, 0.0, 0.0};
        long long v[3] = {0, 0, 0};
        unsigned long long pc = 0ull;
        if (ok) {
            p[0] = x[i];
            p[1] = y[i];
            p[2] = z[i];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                // |x - g| < 2^24: the value and any 64 of them fit in 63 bits
                const double f = fmin(fmax((p[d] - gs[3 * k + d]) * kFix, -kFixMax), kFixMax);
                v[d] = __double2ll_rn(f);
            }
            pc = nbr_count ? (unsigned long long)nbr_count[i] : 0ull;
        }
        const unsigned long long okm = __ballot(ok);
        if (okm == 0ull) continue;
        const int lead = __ffsll(okm) - 1;
        const int k0 = __shfl(k, lead, 64);
        if (__all(!ok || k == k0)) {
            // particles are in cell order, so a wave mostly shares one owner: sum the wave
            // in registers (exact integers; lanes without a particle add zeros) and let one
            // lane add the totals
            long long w0 = v[0], w1 = v[1], w2 = v[2];
            unsigned long long wp = pc;
            for (int o = 32; o > 0; o >>= 1) {
                w0 += __shfl_xor(w0, o, 64);
                w1 += __shfl_xor(w1, o, 64);
                w2 += __shfl_xor(w2, o, 64);
                wp += __shfl_xor(wp, o, 64);
            }
            if ((int)(threadIdx.x & 63) == lead) {
                atomicAdd(&s_part[k0], (unsigned)__popcll(okm));
                if (nbr_count) atomicAdd(&s_pairs[k0], wp);
                add128(&s_lo[3 * k0], &s_hi[3 * k0], w0);
                add128(&s_lo[3 * k0 + 1], &s_hi[3 * k0 + 1], w1);
                add128(&s_lo[3 * k0 + 2], &s_hi[3 * k0 + 2], w2);
            }
        } else if (ok) {
            atomicAdd(&s_part[k], 1u);
            if (nbr_count) atomicAdd(&s_pairs[k], pc);
#pragma unroll
            for (int d = 0; d < 3; ++d) add128(&s_lo[3 * k + d], &s_hi[3 * k + d], v[d]);
        }
        if (!ok) continue;
        if (K > 1) {
            // nearest other generator (ties to the smaller index) and the owner's distance
            double d2o = 0.0, bd = INFINITY;
            int best = -1;
            for (int l = 0; l < K; ++l) {
                const double ex = p[0] - gs[3 * l], ey = p[1] - gs[3 * l + 1],
                             ez = p[2] - gs[3 * l + 2];
                const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(ex, ex), __dmul_rn(ey, ey)),
                                            __dmul_rn(ez, ez));
                if (l == k) {
                    d2o = d2;
                } else if (d2 < bd) {
                    bd = d2;
                    best = l;
                }
            }
            if (best < 0) continue;  // no finite distance to another generator
            const double gx = gs[3 * best] - gs[3 * k], gy = gs[3 * best + 1] - gs[3 * k + 1],
                         gz = gs[3 * best + 2] - gs[3 * k + 2];
            const double gg = __dadd_rn(__dadd_rn(__dmul_rn(gx, gx), __dmul_rn(gy, gy)),
                                        __dmul_rn(gz, gz));
            const double q = __dsub_rn(bd, d2o);
            if (__dmul_rn(q, q) < __dmul_rn(lim, gg)) {
                uint32_t *w1 = adj + (size_t)k * W + (best >> 5);
                const uint32_t b1 = 1u << (best & 31);
                if (!(*w1 & b1)) atomicOr(w1, b1);
                uint32_t *w2 = adj + (size_t)best * W + (k >> 5);
                const uint32_t b2 = 1u << (k & 31);
                if (!(*w2 & b2)) atomicOr(w2, b2);
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kBlock) {
        if (s_part[k]) atomicAdd(&g_part[k], (unsigned long long)s_part[k]);
        if (s_pairs[k]) atomicAdd(&g_pairs[k], s_pairs[k]);
    }
    for (int k = threadIdx.x; k < 3 * K; k += kBlock) {
        const unsigned long long lo = s_lo[k], hi = s_hi[k];
        if (lo == 0ull && hi == 0ull) continue;
        // add the block's 128-bit value {lo, hi}
        const unsigned long long old = atomicAdd(&g_sum[k], lo);
        const unsigned long long carry = (old + lo < old) ? 1ull : 0ull;
        if (hi + carry) atomicAdd(&g_sum[3 * K + k], hi + carry);
    }
}

// centre = g + sum / (2^32 N) (the generator itself for an empty subdomain);
// counts to int64 outputs.
__global__ __launch_bounds__(kBlock) void k_balance_finish(
    const double *__restrict__ sites, int K, const unsigned long long *__restrict__ g_part,
    const unsigned long long *__restrict__ g_pairs, const unsigned long long *__restrict__ g_sum,
    int64_t *__restrict__ site_particles, int64_t *__restrict__ site_pairs,
    double *__restrict__ centre) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= K) return;
    const unsigned long long np = g_part[k];
    if (site_particles) site_particles[k] = (int64_t)np;
    if (site_pairs) site_pairs[k] = (int64_t)g_pairs[k];
    for (int d = 0; d < 3; ++d) {
        double c = sites[3 * k + d];
        if (np) {
            const unsigned long long lo = g_sum[3 * k + d];
            const long long hi = (long long)g_sum[3 * K + 3 * k + d];
            // hi 2^64 + lo with the first addition exact for |hi| < 2^20
            const double s = ((double)hi * 18446744073709551616.0 +
                              (double)(lo >> 32) * 4294967296.0) +
                             (double)(lo & 0xffffffffull);
            c += s / (kFix * (double)np);
        }
        centre[3 * k + d] = c;
    }
}

// ------------------------------------------------------------------ move

struct V3 {
    double x, y, z;
};
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// Rotate v by angle a about the axis along u (right hand), Rodrigues' form.
__device__ V3 rotate(V3 v, V3 u, double a) {
    const double inv = 1.0 / sqrt(dot(u, u));
    u = inv * u;
    double s, c;
    sincos(a, &s, &c);
    return c * v + s * cross(u, v) + (dot(u, v) * (1.0 - c)) * u;
}

__device__ __forceinline__ bool touch(const uint32_t *adj, int W, int a, int b) {
    return (adj[(size_t)a * W + (b >> 5)] >> (b & 31)) & 1u;
}

__global__ __launch_bounds__(1024) void k_balance_move(
    const double *__restrict__ sites, int K, int W, const int64_t *__restrict__ loads,
    const double *__restrict__ centre, const uint32_t *__restrict__ adj, double sigma,
    double theta, double gamma, double dsh, double *__restrict__ out, double *__restrict__ move_sum) {
    extern __shared__ double sm[];
    double *sg = sm;                         // 3K generators
    double *sL = sg + 3 * K;                 // K loads
    uint32_t *sa = (uint32_t *)(sL + K);     // K x W adjacency words
    __shared__ double red[1024];
    for (int q = threadIdx.x; q < 3 * K; q += blockDim.x) sg[q] = sites[q];
    for (int q = threadIdx.x; q < K; q += blockDim.x) sL[q] = (double)loads[q];
    for (int q = threadIdx.x; q < K * W; q += blockDim.x) sa[q] = adj[q];
    __syncthreads();
    const int k = threadIdx.x;
    double mv = 0.0;
    if (k < K) {
        const V3 gk{sg[3 * k], sg[3 * k + 1], sg[3 * k + 2]};
        const double Lk = sL[k];
        const uint32_t *rk = sa + (size_t)k * W;
        V3 two{0.0, 0.0, 0.0}, three{0.0, 0.0, 0.0};
        for (int wl = 0; wl < W; ++wl) {
            for (uint32_t bl = rk[wl] & ~(wl == (k >> 5) ? (1u << (k & 31)) : 0u); bl;
                 bl &= bl - 1) {
                const int l = wl * 32 + __ffs(bl) - 1;
                const V3 gl{sg[3 * l], sg[3 * l + 1], sg[3 * l + 2]};
                const double Ll = sL[l];
                const V3 gkl = gk - gl;
                const double nd = sqrt(dot(gkl, gkl));
                if (Lk + Ll != 0.0 && nd != 0.0)
                    two = two + (dsh * (Lk - Ll) / (Lk + Ll) / nd) * gkl;
                // m > l touching both k and l: the intersection of rows k and l
                const uint32_t *rl = sa + (size_t)l * W;
                for (int wm = l >> 5; wm < W; ++wm) {
                    uint32_t bm = rk[wm] & rl[wm];
                    if (wm == (l >> 5)) bm &= ~((2u << (l & 31)) - 1u);  // m > l
                    if (wm == (k >> 5)) bm &= ~(1u << (k & 31));         // m != k
                    for (; bm; bm &= bm - 1) {
                        const int m = wm * 32 + __ffs(bm) - 1;
                        const V3 gm{sg[3 * m], sg[3 * m + 1], sg[3 * m + 2]};
                        const double Lm = sL[m];
                        const double S = Lk + Ll + Lm;
                        // circumcentre of the triangle (g_k, g_l, g_m)
                        const V3 a = gl - gk, b = gm - gk;
                        const V3 nrm = cross(a, b);
                        const double n2 = dot(nrm, nrm);
                        if (S == 0.0 || !(n2 > 1e-24 * dot(a, a) * dot(b, b))) continue;
                        const V3 o = gk + (0.5 / n2) * cross(dot(a, a) * b - dot(b, b) * a, nrm);
                        const V3 ck = gk - o, cl = gl - o, cm = gm - o;
                        const V3 axl = cross(ck, cl), axm = cross(ck, cm);
                        if (dot(axl, axl) == 0.0 || dot(axm, axm) == 0.0) continue;
                        const double al = (M_PI / 3.0) * (Ll - Lk) / S;
                        const double am = (M_PI / 3.0) * (Lm - Lk) / S;
                        three = three + (rotate(rotate(ck, axl, al), axm, am) - ck);
                    }
                }
            }
        }
        const double nt = sqrt(dot(three, three));
        if (nt > dsh) three = (dsh / nt) * three;
        const V3 dg = (1.0 - sigma) * two + sigma * three;
        const V3 rc{centre[3 * k], centre[3 * k + 1], centre[3 * k + 2]};
        const V3 g2 = (1.0 - theta) * (gk + gamma * dg) + theta * rc;
        out[3 * k] = g2.x;
        out[3 * k + 1] = g2.y;
        out[3 * k + 2] = g2.z;
        const V3 d = g2 - gk;
        mv = sqrt(dot(d, d));
    }
    red[threadIdx.x] = mv;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *move_sum = red[0];
}

size_t balance_ws_bytes(int K) { return (size_t)K * 8 * sizeof(unsigned long long) + 256; }

hipError_t launch_balance_stats(const double *x, const double *y, const double *z, int64_t n,
                                const int32_t *owner, const int32_t *nbr_count,
                                const double *sites, int K, double dsh, int64_t *site_particles,
                                int64_t *site_pairs, double *centre, uint32_t *adj, void *ws,
                                hipStream_t st) {
    const int W = (K + 31) / 32;
    unsigned long long *g_part = (unsigned long long *)ws;   // K
    unsigned long long *g_pairs = g_part + K;                // K
    unsigned long long *g_sum = g_pairs + K;                 // 6K: lo[3K], hi[3K]
    const int nz = 8 * K;
    k_zero_u64<<<(unsigned)((nz + kBlock - 1) / kBlock), kBlock, 0, st>>>(g_part, nz);
    const int na = K * W;
    k_fill_i32<<<(unsigned)((na + kBlock - 1) / kBlock), kBlock, 0, st>>>((int32_t *)adj, 0, na);
    if (n > 0) {
        int64_t want = (n + kBlock - 1) / kBlock;
        unsigned nb = (unsigned)(want > kReduceBlocks ? kReduceBlocks : want);
        size_t shm = (size_t)K * (3 * sizeof(double) + 7 * sizeof(unsigned long long) +
                                  sizeof(unsigned int));
        k_balance_stats<<<nb, kBlock, shm, st>>>(x, y, z, n, owner, nbr_count, sites, K, W, dsh,
                                                 g_part, g_pairs, g_sum, adj);
    }
    k_balance_finish<<<(unsigned)((K + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        sites, K, g_part, g_pairs, g_sum, site_particles, site_pairs, centre);
    return hipGetLastError();
}

hipError_t launch_balance_move(const double *sites, int K, const int64_t *loads,
                               const double *centre, const uint32_t *adj, double sigma,
                               double theta, double gamma, double dsh, double *out,
                               double *move_sum, hipStream_t st) {
    const int W = (K + 31) / 32;
    // one thread per generator, rounded up to whole waves (block sums in a fixed tree)
    int nt = 64;
    while (nt < K) nt *= 2;
    const size_t shm = sizeof(double) * 4 * (size_t)K + sizeof(uint32_t) * (size_t)K * W;
    k_balance_move<<<1, nt, shm, st>>>(sites, K, W, loads, centre, adj, sigma, theta, gamma, dsh,
                                       out, move_sum);
    return hipGetLastError();
}

}  // namespace csph
