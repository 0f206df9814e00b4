// Pair records and the CSPH rate kernels (eqs. SPH:Conti, SPH:Pulse,
// SPH:Energy of sec. 4.1), FP64 and mixed (FP32 pair arithmetic).
//
// Particles are in cell order; each thread owns one particle i and gathers
// over the (2R+1)^3 stencil of cells around its own.  Cells of one stencil
// row are contiguous in cell order, so a row is one index range.  Each
// particle sums its own partners (gather), so no floating-point atomics are
// used and results do not depend on scheduling.
#include "csph_internal.h"

namespace csph {

struct SrcState {
    const double *f[9];  // x y z vx vy vz rho E m
    const int32_t *mat;
    const double *d;
    const int64_t *id;
};

struct DstState {
    double *f[9];
    int32_t *mat;
    double *d;
    int64_t *id;
};

// ---------------------------------------------------------------- pack

// Gather particle perm[s] into slot s: sorted FP64 state copy, EOS
// (e = E - |v|^2/2; ideal or stiffened gas), pair record.
template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_pack(int64_t n, SrcState src,
                                                 const int32_t *__restrict__ perm, EosDev eos,
                                                 GridDev g, void *__restrict__ recA,
                                                 void *__restrict__ recB,
                                                 void *__restrict__ recC, DstState dst,
                                                 int64_t *__restrict__ nonphys) {
    int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    int i = perm[s];
    double v[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] = src.f[k][i];
#pragma unroll
    for (int k = 0; k < 9; ++k) dst.f[k][s] = v[k];
    int mt = src.mat ? src.mat[i] : 0;
    if (dst.mat) dst.mat[s] = mt;
    if (src.d && dst.d) dst.d[s] = src.d[i];
    if (src.id && dst.id) dst.id[s] = src.id[i];
    double x = v[0], y = v[1], z = v[2], vx = v[3], vy = v[4], vz = v[5], rho = v[6], E = v[7],
           m = v[8];
    int k = (mt >= 0 && mt < eos.n) ? mt : 0;
    double gm = eos.gamma[k], pinf = eos.pinf[k];
    double e = E - 0.5 * ((vx * vx + vy * vy) + vz * vz);
    double P, c2;
    if (eos.type[k] == CSPH_EOS_STIFFENED) {
        P = (gm - 1.0) * rho * e - gm * pinf;
        c2 = gm * (P + pinf) / rho;
    } else {
        P = (gm - 1.0) * rho * e;
        c2 = gm * P / rho;
    }
    bool bad = !(c2 >= 0.0);
    double c = bad ? 0.0 : sqrt(c2);
    if (bad && nonphys) atomicAdd((unsigned long long *)nonphys, 1ull);
    double Z = rho * c, V = m / rho;
    if (MIXED) {
        int cx = cell_coord(x, g.ox, g.inv, g.dx);
        int cy = cell_coord(y, g.oy, g.inv, g.dy);
        int cz = cell_coord(z, g.oz, g.inv, g.dz);
        float ox = (float)(x - (g.ox + (double)cx * g.cell));
        float oy = (float)(y - (g.oy + (double)cy * g.cell));
        float oz = (float)(z - (g.oz + (double)cz * g.cell));
        ((float4 *)recA)[s] = make_float4(ox, oy, oz, (float)V);
        ((float4 *)recB)[s] = make_float4((float)vx, (float)vy, (float)vz, (float)P);
        ((float2 *)recC)[s] = make_float2((float)Z, (float)c);
    } else {
        ((double4 *)recA)[s] = make_double4(x, y, z, V);
        ((double4 *)recB)[s] = make_double4(vx, vy, vz, P);
        ((double2 *)recC)[s] = make_double2(Z, c);
    }
}

hipError_t launch_pack(const csph_state &s, int64_t n, const int32_t *perm, const EosDev &eos,
                       int mixed, const GridDev &g, const Ws &w, double *const dst[9],
                       int32_t *dst_mat, double *dst_d, int64_t *dst_id, const int64_t *src_id,
                       int64_t *nonphys, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    SrcState src{{s.x, s.y, s.z, s.vx, s.vy, s.vz, s.rho, s.E, s.m}, s.mat, s.d, src_id};
    DstState ds;
    for (int k = 0; k < 9; ++k) ds.f[k] = dst[k];
    ds.mat = dst_mat;
    ds.d = dst_d;
    ds.id = dst_id;
    unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    if (mixed)
        k_pack<true><<<nb, kBlock, 0, st>>>(n, src, perm, eos, g, w.recA, w.recB, w.recC, ds,
                                            nonphys);
    else
        k_pack<false><<<nb, kBlock, 0, st>>>(n, src, perm, eos, g, w.recA, w.recB, w.recC, ds,
                                             nonphys);
    return hipGetLastError();
}

// ---------------------------------------------------------------- block min -> global

__device__ __forceinline__ void block_min_to(double v, unsigned long long *dst) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    __shared__ double sh[kBlock / 64];
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = sh[0];
        for (int q = 1; q < kBlock / 64; ++q) r = fmin(r, sh[q]);
        if (r >= 0.0) atomicMin(dst, dbits(r));
    }
}

struct RateOut {
    double *rho, *vx, *vy, *vz, *E, *sig;
    int32_t *cnt;
    unsigned long long *dtmin;
};

// ---------------------------------------------------------------- FP64 rates

// One partner of particle i: Riemann problem along e, kernel slope, sums.
__device__ __forceinline__ void pair64(double dx, double dy, double dz, double r2,
                                       const double4 &bi, const double2 &ci,
                                       double vxj, double vyj, double vzj, double Pj, double Zj,
                                       double cj, double Vj, double invH, double dwc,
                                       double &ar, double &avx, double &avy, double &avz,
                                       double &aE, double &sig) {
    if (r2 == 0.0) return;
    double r = sqrt(r2);
    double ir = 1.0 / r;
    double ex = dx * ir, ey = dy * ir, ez = dz * ir;
    double q = r * invH;
    double a1 = 1.0 - q;
    double dW = -dwc * q * (a1 * a1 * a1);
    double vL = (bi.x * ex + bi.y * ey) + bi.z * ez;
    double vR = (vxj * ex + vyj * ey) + vzj * ez;
    double Zi = ci.x, Pi = bi.w;
    double S = Zi + Zj;
    double vs, ps;
    if (S != 0.0) {
        double iS = 1.0 / S;
        vs = ((Zi * vL + Zj * vR) + (Pi - Pj)) * iS;
        ps = ((Zj * Pi + Zi * Pj) + Zi * Zj * (vL - vR)) * iS;
    } else {
        vs = 0.5 * (vL + vR);
        ps = 0.5 * (Pi + Pj);
    }
    double wgt = Vj * dW;
    ar += wgt * (vL - vs);
    double f = wgt * ps;
    avx += f * ex;
    avy += f * ey;
    avz += f * ez;
    aE += f * vs;
    double cl = vL - vR;
    double sp = fmax(ci.y, cj) + (cl > 0.0 ? cl : 0.0);
    sig = sp > sig ? sp : sig;
}

template <bool PAIR, bool WALL>
__global__ __launch_bounds__(kBlock) void k_rates64(int64_t n, const double4 *__restrict__ A,
                                                    const double4 *__restrict__ B,
                                                    const double2 *__restrict__ Cz,
                                                    const double *__restrict__ rho,
                                                    const double *__restrict__ dsz,
                                                    const int32_t *__restrict__ cs, GridDev g,
                                                    PairConst pc, const double *t_dev,
                                                    double t_host, RateOut o, int want_dt) {
    int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double dtv = INFINITY;
    if (s < n) {
        double4 a = A[s], b = B[s];
        double2 zc = Cz[s];
        double di = PAIR ? dsz[s] : 0.0;
        int cx = cell_coord(a.x, g.ox, g.inv, g.dx);
        int cy = cell_coord(a.y, g.oy, g.inv, g.dy);
        int cz = cell_coord(a.z, g.oz, g.inv, g.dz);
        double ar = 0.0, avx = 0.0, avy = 0.0, avz = 0.0, aE = 0.0, sig = zc.y;
        int cnt = 0;
        const int R = g.reach;
        const int x0 = max(cx - R, 0), x1 = min(cx + R, g.dx - 1);
        for (int oz = -R; oz <= R; ++oz) {
            int zz = cz + oz;
            if (zz < 0 || zz >= g.dz) continue;
            for (int oy = -R; oy <= R; ++oy) {
                int yy = cy + oy;
                if (yy < 0 || yy >= g.dy) continue;
                int row = (zz * g.dy + yy) * g.dx;
                int j0 = cs[row + x0], j1 = cs[row + x1 + 1];
                for (int j = j0; j < j1; ++j) {
                    if (j == (int)s) continue;
                    double4 aj = A[j];
                    double dx = aj.x - a.x, dy = aj.y - a.y, dz = aj.z - a.z;
                    double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
                    double invH, dwc;
                    if (PAIR) {
                        double H = pc.kappa * (0.5 * (di + dsz[j]));
                        if (!(r2 < H * H)) continue;
                        invH = 1.0 / H;
                        double i2 = invH * invH;
                        dwc = (210.0 / M_PI) * (i2 * i2);
                    } else {
                        if (!(r2 < pc.H2)) continue;
                        invH = pc.invH;
                        dwc = pc.dwc;
                    }
                    ++cnt;
                    double4 bj = B[j];
                    double2 zj = Cz[j];
                    pair64(dx, dy, dz, r2, b, zc, bj.x, bj.y, bj.z, bj.w, zj.x, zj.y, aj.w, invH,
                           dwc, ar, avx, avy, avz, aE, sig);
                }
            }
        }
        if (WALL) {
            double t = t_dev ? *t_dev : t_host;
            double xw = pc.wall_x0 + pc.wall_v * t;
            double vw2 = 2.0 * pc.wall_v;
            if (a.x - xw < pc.H) {
                for (int oz = -R; oz <= R; ++oz) {
                    int zz = cz + oz;
                    if (zz < 0 || zz >= g.dz) continue;
                    for (int oy = -R; oy <= R; ++oy) {
                        int yy = cy + oy;
                        if (yy < 0 || yy >= g.dy) continue;
                        int row = (zz * g.dy + yy) * g.dx;
                        int j0 = cs[row + x0], j1 = cs[row + x1 + 1];
                        for (int j = j0; j < j1; ++j) {
                            double4 aj = A[j];
                            double xg = 2.0 * xw - aj.x;
                            double dx = xg - a.x, dy = aj.y - a.y, dz = aj.z - a.z;
                            double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
                            double invH, dwc;
                            if (PAIR) {
                                double H = pc.kappa * (0.5 * (di + dsz[j]));
                                if (!(r2 < H * H)) continue;
                                invH = 1.0 / H;
                                double i2 = invH * invH;
                                dwc = (210.0 / M_PI) * (i2 * i2);
                            } else {
                                if (!(r2 < pc.H2)) continue;
                                invH = pc.invH;
                                dwc = pc.dwc;
                            }
                            double4 bj = B[j];
                            double2 zj = Cz[j];
                            pair64(dx, dy, dz, r2, b, zc, vw2 - bj.x, bj.y, bj.z, bj.w, zj.x, zj.y,
                                   aj.w, invH, dwc, ar, avx, avy, avz, aE, sig);
                        }
                    }
                }
            }
        }
        double ri = rho[s];
        double pre = 2.0 / ri;
        double drho = -2.0 * ri * ar;
        o.rho[s] = drho;
        o.vx[s] = pre * avx;
        o.vy[s] = pre * avy;
        o.vz[s] = pre * avz;
        o.E[s] = pre * aE;
        if (o.sig) o.sig[s] = sig;
        if (o.cnt) o.cnt[s] = cnt;
        // Courant limit and relative density-change limit of one explicit step
        dtv = fmin((PAIR ? di : pc.h_dt) / sig, ri / fabs(drho));
    }
    if (want_dt) block_min_to(dtv, o.dtmin);
}

// ---------------------------------------------------------------- mixed rates (FP32 pairs)

__device__ __forceinline__ void pair32(float dx, float dy, float dz, float r2, const float4 &bi,
                                       const float2 &ci, float vxj, float vyj, float vzj,
                                       float Pj, float Zj, float cj, float Vj, float invH,
                                       float dwc, float &ar, float &avx, float &avy, float &avz,
                                       float &aE, float &sig) {
    if (r2 == 0.0f) return;
    float ir = __builtin_amdgcn_rsqf(r2);
    float r = r2 * ir;
    float ex = dx * ir, ey = dy * ir, ez = dz * ir;
    float q = r * invH;
    float a1 = 1.0f - q;
    float dW = -dwc * q * (a1 * a1 * a1);
    // v_L - v_R from the velocity difference (no cancellation of bulk motion)
    float vrel = ((bi.x - vxj) * ex + (bi.y - vyj) * ey) + (bi.z - vzj) * ez;
    float vL = (bi.x * ex + bi.y * ey) + bi.z * ez;
    float Zi = ci.x, Pi = bi.w;
    float S = Zi + Zj;
    float dvl, ps;  // v_L - v*, P*
    if (S != 0.0f) {
        float iS = __builtin_amdgcn_rcpf(S);
        dvl = (Zj * vrel - (Pi - Pj)) * iS;
        ps = ((Zj * Pi + Zi * Pj) + Zi * Zj * vrel) * iS;
    } else {
        dvl = 0.5f * vrel;
        ps = 0.5f * (Pi + Pj);
    }
    float vs = vL - dvl;
    float wgt = Vj * dW;
    ar += wgt * dvl;
    float f = wgt * ps;
    avx += f * ex;
    avy += f * ey;
    avz += f * ez;
    aE += f * vs;
    float sp = fmaxf(ci.y, cj) + (vrel > 0.0f ? vrel : 0.0f);
    sig = sp > sig ? sp : sig;
}

template <bool PAIR, bool WALL>
__global__ __launch_bounds__(kBlock) void k_rates32(int64_t n, const float4 *__restrict__ A,
                                                    const float4 *__restrict__ B,
                                                    const float2 *__restrict__ Cz,
                                                    const double *__restrict__ xs,
                                                    const double *__restrict__ ys,
                                                    const double *__restrict__ zs,
                                                    const double *__restrict__ rho,
                                                    const double *__restrict__ dsz,
                                                    const int32_t *__restrict__ cs, GridDev g,
                                                    PairConst pc, const double *t_dev,
                                                    double t_host, RateOut o, int want_dt) {
    int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double dtv = INFINITY;
    if (s < n) {
        float4 a = A[s], b = B[s];
        float2 zc = Cz[s];
        double xi = xs[s];
        double di = PAIR ? dsz[s] : 0.0;
        int cx = cell_coord(xi, g.ox, g.inv, g.dx);
        int cy = cell_coord(ys[s], g.oy, g.inv, g.dy);
        int cz = cell_coord(zs[s], g.oz, g.inv, g.dz);
        float ar = 0.f, avx = 0.f, avy = 0.f, avz = 0.f, aE = 0.f, sig = zc.y;
        int cnt = 0;
        const int R = g.reach;
        const float Df = (float)g.cell;
        const float H2f = (float)pc.H2, invHf = (float)pc.invH, dwcf = (float)pc.dwc;
        bool wall_near = false;
        float wd = 0.f, vw2 = 0.f;
        if (WALL) {
            double t = t_dev ? *t_dev : t_host;
            double xw = pc.wall_x0 + pc.wall_v * t;
            wall_near = xi - xw < pc.H;
            wd = (float)(xw - xi);
            vw2 = (float)(2.0 * pc.wall_v);
        }
        for (int oz = -R; oz <= R; ++oz) {
            int zz = cz + oz;
            if (zz < 0 || zz >= g.dz) continue;
            float sz = (float)oz * Df;
            for (int oy = -R; oy <= R; ++oy) {
                int yy = cy + oy;
                if (yy < 0 || yy >= g.dy) continue;
                float sy = (float)oy * Df;
                int row = (zz * g.dy + yy) * g.dx;
                for (int ox = -R; ox <= R; ++ox) {
                    int xx = cx + ox;
                    if (xx < 0 || xx >= g.dx) continue;
                    float sx = (float)ox * Df;
                    int j0 = cs[row + xx], j1 = cs[row + xx + 1];
                    for (int j = j0; j < j1; ++j) {
                        float4 aj = A[j];
                        float dx = (aj.x + sx) - a.x, dy = (aj.y + sy) - a.y,
                              dz = (aj.z + sz) - a.z;
                        float H2, invH, dwc;
                        if (PAIR) {
                            double H = pc.kappa * (0.5 * (di + dsz[j]));
                            H2 = (float)(H * H);
                            invH = (float)(1.0 / H);
                            float i2 = invH * invH;
                            dwc = (float)(210.0 / M_PI) * (i2 * i2);
                        } else {
                            H2 = H2f;
                            invH = invHf;
                            dwc = dwcf;
                        }
                        if (j != (int)s) {
                            float r2 = (dx * dx + dy * dy) + dz * dz;
                            if (r2 < H2) {
                                ++cnt;
                                float4 bj = B[j];
                                float2 zj = Cz[j];
                                pair32(dx, dy, dz, r2, b, zc, bj.x, bj.y, bj.z, bj.w, zj.x, zj.y,
                                       aj.w, invH, dwc, ar, avx, avy, avz, aE, sig);
                            }
                        }
                        if (WALL && wall_near) {
                            float gx = 2.0f * wd - dx;
                            float r2 = (gx * gx + dy * dy) + dz * dz;
                            if (r2 < H2) {
                                float4 bj = B[j];
                                float2 zj = Cz[j];
                                pair32(gx, dy, dz, r2, b, zc, vw2 - bj.x, bj.y, bj.z, bj.w, zj.x,
                                       zj.y, aj.w, invH, dwc, ar, avx, avy, avz, aE, sig);
                            }
                        }
                    }
                }
            }
        }
        double ri = rho[s];
        double pre = 2.0 / ri;
        double drho = -2.0 * ri * (double)ar;
        o.rho[s] = drho;
        o.vx[s] = pre * (double)avx;
        o.vy[s] = pre * (double)avy;
        o.vz[s] = pre * (double)avz;
        o.E[s] = pre * (double)aE;
        if (o.sig) o.sig[s] = (double)sig;
        if (o.cnt) o.cnt[s] = cnt;
        dtv = fmin((PAIR ? di : pc.h_dt) / (double)sig, ri / fabs(drho));
    }
    if (want_dt) block_min_to(dtv, o.dtmin);
}

hipError_t launch_rates(int64_t n, int mixed, const GridDev &g, const PairConst &pc,
                        const Ws &w, double *const sorted[9], const double *d_sorted,
                        const double *t_dev, double t_host, int want_dt, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const double *rho_sorted = sorted[6];
    RateOut o{w.rate[0], w.rate[1], w.rate[2], w.rate[3], w.rate[4], w.sig, w.cnt, w.dtmin};
    unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    bool pair = pc.pair_mode != 0, wall = pc.wall != 0;
#define CSPH_RATES_CASE(P, W)                                                                  \
    if (pair == P && wall == W) {                                                              \
        if (mixed)                                                                             \
            k_rates32<P, W><<<nb, kBlock, 0, st>>>(n, (const float4 *)w.recA,                  \
                                                   (const float4 *)w.recB,                     \
                                                   (const float2 *)w.recC, sorted[0], sorted[1], \
                                                   sorted[2], rho_sorted, d_sorted, w.cs, g,    \
                                                   pc, t_dev, t_host, o, want_dt);             \
        else                                                                                   \
            k_rates64<P, W><<<nb, kBlock, 0, st>>>(n, (const double4 *)w.recA,                 \
                                                   (const double4 *)w.recB,                    \
                                                   (const double2 *)w.recC, rho_sorted,        \
                                                   d_sorted, w.cs, g, pc, t_dev, t_host, o,    \
                                                   want_dt);                                   \
    }
    CSPH_RATES_CASE(false, false)
    CSPH_RATES_CASE(false, true)
    CSPH_RATES_CASE(true, false)
    CSPH_RATES_CASE(true, true)
#undef CSPH_RATES_CASE
    return hipGetLastError();
}

// ---------------------------------------------------------------- back to input order

__global__ __launch_bounds__(kBlock) void k_unsort_rates(int64_t n,
                                                         const int32_t *__restrict__ perm,
                                                         RateOut src, csph_rates_out out,
                                                         double *__restrict__ signal,
                                                         int32_t *__restrict__ nbr_count) {
    int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    int i = perm[s];
    out.drho[i] = src.rho[s];
    out.dvx[i] = src.vx[s];
    out.dvy[i] = src.vy[s];
    out.dvz[i] = src.vz[s];
    out.dE[i] = src.E[s];
    if (signal) signal[i] = src.sig[s];
    if (nbr_count) nbr_count[i] = src.cnt[s];
}

hipError_t launch_unsort_rates(int64_t n, const int32_t *perm, const Ws &w, csph_rates_out out,
                               double *signal, int32_t *nbr_count, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    RateOut src{w.rate[0], w.rate[1], w.rate[2], w.rate[3], w.rate[4], w.sig, w.cnt, w.dtmin};
    k_unsort_rates<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, perm, src, out,
                                                                             signal, nbr_count);
    return hipGetLastError();
}

}  // namespace csph
