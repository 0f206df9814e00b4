// State renewal and global time step (Algorithm 1), compensated
// conservation totals, the return to input order, and the EOS inverse
// that builds E from (rho, p, v).
//
// Integrator: symplectic Euler with one rate evaluation per step,
//   v += dt dv/dt, E += dt dE/dt, rho += dt drho/dt, then r += dt v_new,
// dt = cfl * min_i h_i/s_i (a min is exact and order independent) or the
// caller's dt.  Totals use double-double (TwoSum) accumulation in a fixed
// reduction tree, so they are reproducible run to run.
#include "csph_internal.h"

namespace csph {

struct DD {
    double hi, lo;
};

// hi + b with the rounding error of the sum kept in lo (Knuth TwoSum).
__device__ __forceinline__ DD dd_add1(DD a, double b) {
    double s = a.hi + b;
    double bb = s - a.hi;
    double e = (a.hi - (s - bb)) + (b - bb);
    return DD{s, a.lo + e};
}

__device__ __forceinline__ DD dd_add(DD a, DD b) {
    double s = a.hi + b.hi;
    double bb = s - a.hi;
    double e = (a.hi - (s - bb)) + (b.hi - bb);
    e += a.lo + b.lo;
    double hi = s + e;
    double lo = e - (hi - s);
    return DD{hi, lo};
}

__global__ __launch_bounds__(kBlock) void k_fill_u64(unsigned long long *p, unsigned long long v,
                                                     int64_t count) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < count) p[i] = v;
}

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t count,
                           hipStream_t st) {
    if (count <= 0) return hipSuccess;
    k_fill_u64<<<(unsigned)((count + kBlock - 1) / kBlock), kBlock, 0, st>>>(p, v, count);
    return hipGetLastError();
}

__global__ void k_add_i64(int64_t *dst, const int64_t *src) { *dst += *src; }

hipError_t launch_add_i64(int64_t *dst, const int64_t *src, hipStream_t st) {
    k_add_i64<<<1, 1, 0, st>>>(dst, src);
    return hipGetLastError();
}

__device__ __forceinline__ double step_dt(const unsigned long long *dtmin, double cfl,
                                          double dt_in) {
    return cfl > 0.0 ? cfl * __longlong_as_double((long long)*dtmin) : dt_in;
}

struct State9 {
    double *f[9];
};

struct Rates5 {
    const double *f[5];
};

// Update in place (cell order) and accumulate block partial totals.  With the piston
// (a rigid wall that stops the particles, sec. 7.1), a particle whose new position lies
// behind the plane at the new time is reflected off it in the wall's frame: position and
// normal velocity mirrored, specific internal energy kept.  The wall is normal to the
// state's y array (the kernels' axes; see PairConst).
struct WallDev {
    int on;
    double y0, v;
    const double *t;  // time at the start of the step (device)
};

// Periodic axes (kernels' axes, bit a): a new position at or above hi moves down by the period,
// one below lo up by it (a particle moves less than a period per step).
struct PerDev {
    int mask;
    double lo[3], hi[3], L[3];
};

__device__ __forceinline__ double wrap_axis(const PerDev &p, int a, double v) {
    if (!((p.mask >> a) & 1)) return v;
    if (v >= p.hi[a]) return v - p.L[a];
    if (v < p.lo[a]) return v + p.L[a];
    return v;
}

// With VORO the kernel also assigns each particle's new position to its Voronoi generator
// (eq. VoronoiDefinition: FP64 argmin of ((dx dx) + (dy dy)) + (dz dz) without contraction,
// k scanned upwards with a strict comparison, so a tie keeps the smaller k) and counts
// particles and pairs per generator, as k_voronoi does: the VALU-bound scan overlaps the
// memory-bound update.  The generators come in the kernels' axes (x and y swapped with a
// wall), which leaves every squared distance unchanged (the sum of the x and y terms is
// commutative).
__global__ __launch_bounds__(kBlock) void k_integrate(int64_t n, State9 s, Rates5 r,
                                                      const unsigned long long *dtmin, double cfl,
                                                      double dt_in, WallDev wall, PerDev per,
                                                      VoroDev vo, ListGate lg,
                                                      double *__restrict__ part) {
    if (lg.gate && *lg.gate == 0) return;
    extern __shared__ double vsm[];
    double *gs = vsm;                                                   // 3K
    unsigned long long *hq = (unsigned long long *)(vsm + 3 * vo.K);    // K
    unsigned int *hp = (unsigned int *)(hq + vo.K);                     // K
    if (vo.K > 0) {
        for (int k = threadIdx.x; k < vo.K; k += kBlock) {
            gs[3 * k] = vo.sites[3 * k + (vo.swap ? 1 : 0)];
            gs[3 * k + 1] = vo.sites[3 * k + (vo.swap ? 0 : 1)];
            gs[3 * k + 2] = vo.sites[3 * k + 2];
            hp[k] = 0u;
            hq[k] = 0ull;
        }
        __syncthreads();
    }
    double dt = step_dt(dtmin, cfl, dt_in);
    const double yw = wall.on ? wall.y0 + wall.v * (*wall.t + dt) : 0.0;
    DD acc[5];
    for (int k = 0; k < 5; ++k) acc[k] = DD{0.0, 0.0};
    unsigned long long npairs = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        if (lg.pairs) npairs += (unsigned long long)lg.cnt[i];
        double vx = s.f[3][i] + dt * r.f[1][i];
        double vy = s.f[4][i] + dt * r.f[2][i];
        double vz = s.f[5][i] + dt * r.f[3][i];
        double E = s.f[7][i] + dt * r.f[4][i];
        double rho = s.f[6][i] + dt * r.f[0][i];
        double y = s.f[1][i] + dt * vy;
        if (wall.on && y < yw) {
            const double vr = 2.0 * wall.v - vy;
            E = E + 0.5 * ((vr * vr) - (vy * vy));
            vy = vr;
            y = 2.0 * yw - y;
        }
        double x = s.f[0][i] + dt * vx, z = s.f[2][i] + dt * vz;
        if (per.mask) {  // after the reflection, as the wall's axis is never periodic
            x = wrap_axis(per, 0, x);
            y = wrap_axis(per, 1, y);
            z = wrap_axis(per, 2, z);
        }
        s.f[0][i] = x;
        s.f[1][i] = y;
        s.f[2][i] = z;
        if (vo.K > 0) {
            int best = 0;
            double bd = INFINITY;
            for (int k = 0; k < vo.K; ++k) {
                const double dx = x - gs[3 * k], dy = y - gs[3 * k + 1], dz = z - gs[3 * k + 2];
                const double d2 = ((dx * dx) + (dy * dy)) + (dz * dz);
                if (d2 < bd) {
                    bd = d2;
                    best = k;
                }
            }
            vo.owner[vo.owner_at ? vo.owner_at[i] : (int)i] = best;
            atomicAdd(&hp[best], 1u);
            atomicAdd(&hq[best], (unsigned long long)vo.cnt[i]);
        }
        s.f[3][i] = vx;
        s.f[4][i] = vy;
        s.f[5][i] = vz;
        s.f[6][i] = rho;
        s.f[7][i] = E;
        double m = s.f[8][i];
        acc[0] = dd_add1(acc[0], m);
        acc[1] = dd_add1(acc[1], m * vx);
        acc[2] = dd_add1(acc[2], m * vy);
        acc[3] = dd_add1(acc[3], m * vz);
        acc[4] = dd_add1(acc[4], m * E);
    }
    __shared__ double sh[2][5][kBlock];
    for (int k = 0; k < 5; ++k) {
        sh[0][k][threadIdx.x] = acc[k].hi;
        sh[1][k][threadIdx.x] = acc[k].lo;
    }
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int k = 0; k < 5; ++k) {
                DD a{sh[0][k][threadIdx.x], sh[1][k][threadIdx.x]};
                DD b{sh[0][k][threadIdx.x + w], sh[1][k][threadIdx.x + w]};
                DD c = dd_add(a, b);
                sh[0][k][threadIdx.x] = c.hi;
                sh[1][k][threadIdx.x] = c.lo;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 5) {
        part[blockIdx.x * 10 + 2 * threadIdx.x] = sh[0][threadIdx.x][0];
        part[blockIdx.x * 10 + 2 * threadIdx.x + 1] = sh[1][threadIdx.x][0];
    }
    if (lg.pairs) {  // integer sums: exact in any order
        for (int o = 32; o > 0; o >>= 1) npairs += __shfl_xor(npairs, o, 64);
        if ((threadIdx.x & 63) == 0 && npairs) atomicAdd(lg.pairs, npairs);
    }
    if (vo.K > 0) {  // the reduction above ended with a barrier: every count is in LDS
        for (int k = threadIdx.x; k < vo.K; k += kBlock) {
            if (hp[k]) atomicAdd(&vo.site_part[k], (unsigned long long)hp[k]);
            if (hq[k] && vo.site_pairs) atomicAdd(&vo.site_pairs[k], hq[k]);
        }
    }
}

static int integrate_blocks(int64_t n) {
    int64_t want = (n + kBlock - 1) / kBlock;
    return (int)(want < 1 ? 1 : (want > kReduceBlocks ? kReduceBlocks : want));
}

hipError_t launch_integrate(int64_t n, double *const st8[9], const Ws &w, double cfl, double dt_in,
                            const PairConst &pc, const double *t, hipStream_t st,
                            const VoroDev *vo, const ListGate *lg) {
    State9 s;
    for (int k = 0; k < 9; ++k) s.f[k] = st8[k];
    Rates5 r{{w.rate[0], w.rate[1], w.rate[2], w.rate[3], w.rate[4]}};
    WallDev wall{pc.wall && t ? 1 : 0, pc.wall_y0, pc.wall_v, t};
    PerDev per{};
    per.mask = pc.per;
    for (int a = 0; a < 3; ++a) {
        per.lo[a] = pc.lo[a];
        per.hi[a] = pc.hi[a];
        per.L[a] = pc.L[a];
    }
    VoroDev v{};
    size_t shm = 0;
    if (vo && vo->K > 0) {
        v = *vo;
        launch_fill_u64(v.site_part, 0ull, v.K, st);
        if (v.site_pairs) launch_fill_u64(v.site_pairs, 0ull, v.K, st);
        shm = (size_t)v.K * (3 * sizeof(double) + sizeof(unsigned long long) + sizeof(unsigned));
    }
    const ListGate g = lg ? *lg : ListGate{nullptr, nullptr, nullptr, nullptr};
    int nb = integrate_blocks(n);
    k_integrate<<<nb, kBlock, shm, st>>>(n, s, r, w.dtmin, cfl, dt_in, wall, per, v, g,
                                         w.tot_part);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_finish(const double *__restrict__ part, int nblocks,
                                                   const unsigned long long *dtmin, double cfl,
                                                   double dt_in, double *t, double *dt_used,
                                                   double *totals, int swap_xy, ListGate lg) {
    if (lg.gate && *lg.gate == 0) return;
    __shared__ double sh[2][5][kBlock];
    DD acc[5];
    for (int k = 0; k < 5; ++k) acc[k] = DD{0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += kBlock)
        for (int k = 0; k < 5; ++k) acc[k] = dd_add(acc[k], DD{part[b * 10 + 2 * k], part[b * 10 + 2 * k + 1]});
    for (int k = 0; k < 5; ++k) {
        sh[0][k][threadIdx.x] = acc[k].hi;
        sh[1][k][threadIdx.x] = acc[k].lo;
    }
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int k = 0; k < 5; ++k) {
                DD a{sh[0][k][threadIdx.x], sh[1][k][threadIdx.x]};
                DD bb{sh[0][k][threadIdx.x + w], sh[1][k][threadIdx.x + w]};
                DD c = dd_add(a, bb);
                sh[0][k][threadIdx.x] = c.hi;
                sh[1][k][threadIdx.x] = c.lo;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 5 && totals) {
        // sums k = 1, 2 are the momenta along the state's x and y arrays, which are the
        // caller's y and x when the library swapped them
        const int k = threadIdx.x, o = swap_xy && (k == 1 || k == 2) ? 3 - k : k;
        totals[2 * o] = sh[0][k][0];
        totals[2 * o + 1] = sh[1][k][0];
    }
    if (threadIdx.x == 0) {
        double dt = step_dt(dtmin, cfl, dt_in);
        if (dt_used) *dt_used = dt;
        if (t) *t = *t + dt;
        if (lg.steps) *lg.steps += 1;
    }
}

hipError_t launch_finish_step(int64_t n, const Ws &w, double cfl, double dt_in, double *t,
                                double *dt_used, double *totals, int swap_xy, hipStream_t st,
                                const ListGate *lg) {
    const ListGate g = lg ? *lg : ListGate{nullptr, nullptr, nullptr, nullptr};
    k_finish<<<1, kBlock, 0, st>>>(w.tot_part, integrate_blocks(n), w.dtmin, cfl, dt_in, t,
                                   dt_used, totals, swap_xy, g);
    return hipGetLastError();
}

struct OutState {
    double *f[9];
    int32_t *mat;
    double *d;
    int64_t *id;
};

struct InState {
    const double *f[9];
    const int32_t *mat;
    const double *d;
    const int64_t *id;
};

__global__ __launch_bounds__(kBlock) void k_unpermute(int64_t n, const int32_t *__restrict__ perm,
                                                      InState src, const int32_t *src_cnt,
                                                      OutState dst, int32_t *out_cnt) {
    int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    int i = perm[s];
#pragma unroll
    for (int k = 0; k < 9; ++k) dst.f[k][i] = src.f[k][s];
    if (dst.mat && src.mat) dst.mat[i] = src.mat[s];
    if (dst.d && src.d) dst.d[i] = src.d[s];
    if (dst.id && src.id) dst.id[i] = src.id[s];
    if (out_cnt && src_cnt) out_cnt[i] = src_cnt[s];
}

hipError_t launch_unpermute(int64_t n, const int32_t *perm, double *const src[9],
                            const int32_t *src_mat, const double *src_d, const int64_t *src_id,
                            const int32_t *src_cnt, const csph_state &out, int32_t *out_cnt,
                            hipStream_t st) {
    if (n <= 0) return hipSuccess;
    InState a;
    for (int k = 0; k < 9; ++k) a.f[k] = src[k];
    a.mat = src_mat;
    a.d = src_d;
    a.id = src_id;
    OutState b{{out.x, out.y, out.z, out.vx, out.vy, out.vz, out.rho, out.E, out.m}, out.mat,
               out.d, out.id};
    k_unpermute<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, perm, a, src_cnt, b,
                                                                          out_cnt);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_init_energy(const double *__restrict__ rho,
                                                        const double *__restrict__ pres,
                                                        const double *__restrict__ vx,
                                                        const double *__restrict__ vy,
                                                        const double *__restrict__ vz,
                                                        const int32_t *__restrict__ mat, int64_t n,
                                                        EosDev eos, double *__restrict__ E) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int k = mat ? mat[i] : 0;
    if (k < 0 || k >= eos.n) k = 0;
    double e = eos_energy(eos, k, rho[i], pres[i]);
    E[i] = e + 0.5 * ((vx[i] * vx[i] + vy[i] * vy[i]) + vz[i] * vz[i]);
}

hipError_t launch_init_energy(const double *rho, const double *pres, const double *vx,
                              const double *vy, const double *vz, const int32_t *mat, int64_t n,
                              const EosDev &eos, double *E, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_init_energy<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(rho, pres, vx, vy, vz,
                                                                            mat, n, eos, E);
    return hipGetLastError();
}

}  // namespace csph
