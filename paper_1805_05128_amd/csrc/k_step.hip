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

// The workgroup's double-double sums (m, m vx, m vy, m vz, m E) reduced in a fixed tree into
// part[block * 10 ..] as (hi, lo) pairs; ends with a barrier.
__device__ __forceinline__ void block_totals(const DD acc[5], double *__restrict__ part) {
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
}

// The piston's reflection of a new position (normal axis y in the kernels' axes) in the
// wall's frame: y <- 2 yw - y, v_y <- 2 v_w - v_y, E changed by the kinetic-energy difference
// (the specific internal energy kept).
__device__ __forceinline__ void reflect(const WallDev &wall, double yw, double &y, double &vy,
                                        double &E) {
    if (wall.on && y < yw) {
        const double vr = 2.0 * wall.v - vy;
        E = E + 0.5 * ((vr * vr) - (vy * vy));
        vy = vr;
        y = 2.0 * yw - y;
    }
}

// With VORO the kernel also assigns each particle's new position to its Voronoi generator
// (eq. VoronoiDefinition: FP64 argmin of ((dx dx) + (dy dy)) + (dz dz) without contraction,
// k scanned upwards with a strict comparison, so a tie keeps the smaller k) and counts
// particles and pairs per generator, as k_voronoi does: the VALU-bound scan overlaps the
// memory-bound update.  The generators come in the kernels' axes (x and y exchanged when the
// library hands the kernels the caller's y as x), which leaves every squared distance
// unchanged (the sum of the x and y terms is commutative).
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
            gs[3 * k] = vo.sites[3 * k + vo.ax[0]];
            gs[3 * k + 1] = vo.sites[3 * k + vo.ax[1]];
            gs[3 * k + 2] = vo.sites[3 * k + vo.ax[2]];
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
        reflect(wall, yw, y, vy, E);
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
    block_totals(acc, part);
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

// Two-stage Runge-Kutta, first stage: U1 = U + dt F(U) with r1 = r + dt v (the old velocity),
// positions wrapped into a periodic box for the second evaluation; the first stage's neighbour
// counts are kept (the second evaluation overwrites them) and t + dt stored for the second
// evaluation's piston position.
struct Stage8 {
    double *f[8];  // x y z vx vy vz rho E
};

__global__ __launch_bounds__(kBlock) void k_rk2_predict(int64_t n, State9 s, Rates5 r,
                                                        const unsigned long long *dtmin,
                                                        double cfl, double dt_in, PerDev per,
                                                        const double *t, double *t2,
                                                        const int32_t *__restrict__ cnt,
                                                        int32_t *__restrict__ cnt_save,
                                                        Stage8 u1) {
    const double dt = step_dt(dtmin, cfl, dt_in);
    if (blockIdx.x == 0 && threadIdx.x == 0) *t2 = (t ? *t : 0.0) + dt;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const double vx = s.f[3][i], vy = s.f[4][i], vz = s.f[5][i];
        u1.f[0][i] = wrap_axis(per, 0, s.f[0][i] + dt * vx);
        u1.f[1][i] = wrap_axis(per, 1, s.f[1][i] + dt * vy);
        u1.f[2][i] = wrap_axis(per, 2, s.f[2][i] + dt * vz);
        u1.f[3][i] = vx + dt * r.f[1][i];
        u1.f[4][i] = vy + dt * r.f[2][i];
        u1.f[5][i] = vz + dt * r.f[3][i];
        u1.f[6][i] = s.f[6][i] + dt * r.f[0][i];
        u1.f[7][i] = s.f[7][i] + dt * r.f[4][i];
        cnt_save[i] = cnt[i];
    }
}

// Second stage: for slot q of the second evaluation's cell order (its particle i in the first
// stage's order, perm2[q] = i), U' = U/2 + (U1 + dt F(U1))/2 and r' = r/2 + (r1 + dt v1)/2, with
// r1 = r + dt v formed again exactly as the first stage formed it (unwrapped), then the
// piston's reflection at t + dt and the periodic wrap; written over U in place, with the block
// partial totals of the new state.
__global__ __launch_bounds__(kBlock) void k_rk2_combine(int64_t n, State9 s, Rates5 r2,
                                                        const unsigned long long *dtmin,
                                                        double cfl, double dt_in, WallDev wall,
                                                        PerDev per,
                                                        const int32_t *__restrict__ perm2,
                                                        Stage8 u1, double *__restrict__ part) {
    const double dt = step_dt(dtmin, cfl, dt_in);
    const double yw = wall.on ? wall.y0 + wall.v * (*wall.t + dt) : 0.0;
    DD acc[5];
    for (int k = 0; k < 5; ++k) acc[k] = DD{0.0, 0.0};
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kBlock) {
        const int i = perm2[q];
        const double x = s.f[0][i], y = s.f[1][i], z = s.f[2][i];
        const double vx = s.f[3][i], vy = s.f[4][i], vz = s.f[5][i];
        const double vx1 = u1.f[3][i], vy1 = u1.f[4][i], vz1 = u1.f[5][i];
        const double x1 = x + dt * vx, y1 = y + dt * vy, z1 = z + dt * vz;
        double nvx = 0.5 * vx + 0.5 * (vx1 + dt * r2.f[1][q]);
        double nvy = 0.5 * vy + 0.5 * (vy1 + dt * r2.f[2][q]);
        double nvz = 0.5 * vz + 0.5 * (vz1 + dt * r2.f[3][q]);
        double nE = 0.5 * s.f[7][i] + 0.5 * (u1.f[7][i] + dt * r2.f[4][q]);
        const double nrho = 0.5 * s.f[6][i] + 0.5 * (u1.f[6][i] + dt * r2.f[0][q]);
        double nx = 0.5 * x + 0.5 * (x1 + dt * vx1);
        double ny = 0.5 * y + 0.5 * (y1 + dt * vy1);
        double nz = 0.5 * z + 0.5 * (z1 + dt * vz1);
        reflect(wall, yw, ny, nvy, nE);
        if (per.mask) {
            nx = wrap_axis(per, 0, nx);
            ny = wrap_axis(per, 1, ny);
            nz = wrap_axis(per, 2, nz);
        }
        s.f[0][i] = nx;
        s.f[1][i] = ny;
        s.f[2][i] = nz;
        s.f[3][i] = nvx;
        s.f[4][i] = nvy;
        s.f[5][i] = nvz;
        s.f[6][i] = nrho;
        s.f[7][i] = nE;
        const double m = s.f[8][i];
        acc[0] = dd_add1(acc[0], m);
        acc[1] = dd_add1(acc[1], m * nvx);
        acc[2] = dd_add1(acc[2], m * nvy);
        acc[3] = dd_add1(acc[3], m * nvz);
        acc[4] = dd_add1(acc[4], m * nE);
    }
    block_totals(acc, part);
}

static PerDev per_dev(const PairConst &pc) {
    PerDev per{};
    per.mask = pc.per;
    for (int a = 0; a < 3; ++a) {
        per.lo[a] = pc.lo[a];
        per.hi[a] = pc.hi[a];
        per.L[a] = pc.L[a];
    }
    return per;
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
    const PerDev per = per_dev(pc);
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

hipError_t launch_rk2_predict(int64_t n, double *const st8[9], const Ws &w, double cfl,
                              double dt_in, const PairConst &pc, const double *t, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    State9 s;
    for (int k = 0; k < 9; ++k) s.f[k] = st8[k];
    Rates5 r{{w.rate[0], w.rate[1], w.rate[2], w.rate[3], w.rate[4]}};
    Stage8 u1;
    for (int k = 0; k < 8; ++k) u1.f[k] = w.stg[k];
    k_rk2_predict<<<integrate_blocks(n), kBlock, 0, st>>>(n, s, r, w.dtmin, cfl, dt_in,
                                                          per_dev(pc), t, w.t2, w.cnt, w.rk_cnt,
                                                          u1);
    return hipGetLastError();
}

hipError_t launch_rk2_combine(int64_t n, double *const st8[9], const Ws &w, double cfl,
                              double dt_in, const PairConst &pc, const double *t, hipStream_t st) {
    State9 s;
    for (int k = 0; k < 9; ++k) s.f[k] = st8[k];
    Rates5 r{{w.rate[0], w.rate[1], w.rate[2], w.rate[3], w.rate[4]}};
    Stage8 u1;
    for (int k = 0; k < 8; ++k) u1.f[k] = w.stg[k];
    WallDev wall{pc.wall && t ? 1 : 0, pc.wall_y0, pc.wall_v, t};
    k_rk2_combine<<<integrate_blocks(n), kBlock, 0, st>>>(n, s, r, w.dtmin, cfl, dt_in, wall,
                                                          per_dev(pc), w.perm2, u1, w.tot_part);
    return hipGetLastError();
}

// the caller's axis of each of the kernels' axes, by value
struct Ax3 {
    int k[3];
};

__global__ __launch_bounds__(kBlock) void k_finish(const double *__restrict__ part, int nblocks,
                                                   const unsigned long long *dtmin, double cfl,
                                                   double dt_in, double *t, double *dt_used,
                                                   double *totals, Ax3 ax, ListGate lg) {
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
        // sums k = 1, 2, 3 are the momenta along the state's x, y, z arrays, which are the
        // caller's axes ax.k[0], ax.k[1], ax.k[2]
        const int k = threadIdx.x, o = (k >= 1 && k <= 3) ? 1 + ax.k[k - 1] : k;
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
                                double *dt_used, double *totals, const int ax[3], hipStream_t st,
                                const ListGate *lg) {
    const ListGate g = lg ? *lg : ListGate{nullptr, nullptr, nullptr, nullptr};
    const Ax3 a3{{ax[0], ax[1], ax[2]}};
    k_finish<<<1, kBlock, 0, st>>>(w.tot_part, integrate_blocks(n), w.dtmin, cfl, dt_in, t,
                                   dt_used, totals, a3, g);
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
