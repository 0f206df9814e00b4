// Hand-written adjoint (vector-Jacobian product) of the CSPH rates of
// eqs. SPH:Conti, SPH:Pulse, SPH:Energy (sec. 4.1), of the step, and of the
// EOS inverse that builds E from (rho, p, v).  FP64, fixed smoothing length.
//
// With cotangents a_i of the rates, J = sum_i a_i . R_i.  Writing
// b_rho = -2 rho_i a_rho, b_v = (2/rho_i) a_v, b_E = (2/rho_i) a_E,
// J = sum over unordered neighbour pairs of
//   Phi_ij = W'_ij [ V_j (b_rho,i (v_L - v*) + P* b_v,i.e + b_E,i P* v*)
//                  + V_i (b_rho,j (v* - v_R) - P* b_v,j.e - b_E,j P* v*) ]
// (e, v_L, v_R, v*, P* seen from i), plus the rho_i prefactors.  Because
// j in N(i) <=> i in N(j) for a fixed support, dJ/dq_i = sum_{j in N(i)}
// dPhi_ij/dq_i: every particle gathers its own gradient over its own
// neighbours, no atomics, fixed summation order.
//
// With the piston (sec. 7.1), a mirror pair (i, image of j) adds to J only i's side:
// Phi^m_ij = W'_ij V_j (b_rho,i (v_L - v*) + P* b_v,i.e + b_E,i P* v*), the image of j at
// (x_j, 2 y_w - y_j, z_j) with normal velocity 2 v_w - v_y,j (kernels' axes: the wall is normal
// to y).  Reflection is an isometry and an involution, so i's image lies within the support
// of j exactly when j's image lies within that of i: the walk around i's own image finds
// both the pairs (i, image of j), differentiated in q_i directly, and the pairs (j, image of
// i), differentiated in the image's q and mapped back (y and v_y change sign).  Each of the
// two is a member under the forward pass's own rounding of its offset.
#include "adjoint.h"
#include "csph_internal.h"
#include "stencil.h"

namespace csph {

struct VjpIn {
    const double4 *A;   // x y z V      (cell order)
    const double4 *B;   // vx vy vz P
    const double2 *C;   // Z c
    const double4 *Dw;  // b_rho b_vx b_vy b_vz
    const double *Ew;   // b_E
    const double *rho, *E, *m;  // sorted state
    const int32_t *mat;
    const double *a[5]; // rate cotangents (cell order): rho vx vy vz E
    const double *dsz;  // pair-h mode: particle sizes d (cell order, constants of the map)
};

// The piston at the time of the rates: position along the kernels' y, twice its velocity.
struct VjpWall {
    double yw, vw2;
    WallPass p;  // the rate sums of the first pass, or the band of the correction pass
};

struct VjpOut {
    double *g[8];       // x y z vx vy vz rho E, input order (perm)
    const double *gn[8];  // step VJP: cotangent of the next state (input order), or NULL
    double dt;          // step VJP: frozen time step
    int accumulate;     // 1: g += result (rates VJP); 0: g = result (+ identity terms)
    double *eos_part;   // [gridDim.x][2*CSPH_MAX_EOS]
};

// Rate cotangents and pair weights in cell order.  For a step VJP the
// cotangents follow from the next-state cotangent gn: a_rho = dt g_rho',
// a_v = dt (g_v' + dt g_r'), a_E = dt g_E'.
__global__ __launch_bounds__(kBlock) void k_vjp_weights(int64_t n,
                                                        const int32_t *__restrict__ perm,
                                                        const double *__restrict__ rho_s,
                                                        VjpOut o, const double *a_in0,
                                                        const double *a_in1, const double *a_in2,
                                                        const double *a_in3, const double *a_in4,
                                                        double *a0, double *a1, double *a2,
                                                        double *a3, double *a4,
                                                        double4 *__restrict__ Dw,
                                                        double *__restrict__ Ew) {
    int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    int i = perm[s];
    double ar, ax, ay, az, aE;
    if (o.gn[0]) {
        double dt = o.dt;
        ar = dt * o.gn[6][i];
        ax = dt * (o.gn[3][i] + dt * o.gn[0][i]);
        ay = dt * (o.gn[4][i] + dt * o.gn[1][i]);
        az = dt * (o.gn[5][i] + dt * o.gn[2][i]);
        aE = dt * o.gn[7][i];
    } else {
        ar = a_in0[i];
        ax = a_in1[i];
        ay = a_in2[i];
        az = a_in3[i];
        aE = a_in4[i];
    }
    a0[s] = ar;
    a1[s] = ax;
    a2[s] = ay;
    a3[s] = az;
    a4[s] = aE;
    double r = rho_s[s];
    double k = 2.0 / r;
    Dw[s] = make_double4(-2.0 * r * ar, k * ax, k * ay, k * az);
    Ew[s] = k * aE;
}

// A value with its partial derivatives in (rho, e, Gamma): forward-mode differentiation of
// the Mie-Grueneisen EOS, whose sound speed is too long an expression to differentiate by
// hand reliably.
struct Dual3 {
    double v, dr, de, dg;
};
__device__ __forceinline__ Dual3 operator+(Dual3 a, Dual3 b) {
    return {a.v + b.v, a.dr + b.dr, a.de + b.de, a.dg + b.dg};
}
__device__ __forceinline__ Dual3 operator-(Dual3 a, Dual3 b) {
    return {a.v - b.v, a.dr - b.dr, a.de - b.de, a.dg - b.dg};
}
__device__ __forceinline__ Dual3 operator*(Dual3 a, Dual3 b) {
    return {a.v * b.v, a.dr * b.v + a.v * b.dr, a.de * b.v + a.v * b.de, a.dg * b.v + a.v * b.dg};
}
__device__ __forceinline__ Dual3 operator/(Dual3 a, Dual3 b) {
    const double q = a.v / b.v, ib = 1.0 / b.v;
    return {q, (a.dr - q * b.dr) * ib, (a.de - q * b.de) * ib, (a.dg - q * b.dg) * ib};
}
__device__ __forceinline__ Dual3 cst(double c) { return {c, 0.0, 0.0, 0.0}; }

// Mie-Grueneisen (eqs. mie_gruneisen_eos, mie_gruneisen_reference) at (rho, e) with Gamma,
// each with its partials: x = rho0/rho, eta = 1 - x, D = 1 - s_a eta,
// P_r = rho0 c_a^2 eta / D^2, e_r = c_a^2 eta^2 / (2 D^2), P = P_r + Gamma rho (e - e_r),
// c^2 = c_a^2 x^2 (1 + s_a eta)/D^3 + Gamma (e - e_r) - Gamma c_a^2 eta x / D^3 + Gamma P / rho
// (the forward pass's sound speed: (dP/drho)_e + (P/rho^2)(dP/de)_rho).
__device__ __forceinline__ void mg_eos_dual(const EosDev &eos, int k, double rho_v, double e_v,
                                            Dual3 &P, Dual3 &c2) {
    const Dual3 rho{rho_v, 1.0, 0.0, 0.0}, e{e_v, 0.0, 1.0, 0.0}, g{eos.gamma[k], 0.0, 0.0, 1.0};
    const double rho0 = eos.rho0[k], ca2 = eos.ca[k] * eos.ca[k], sa = eos.sa[k];
    const Dual3 x = cst(rho0) / rho, eta = cst(1.0) - x;
    const Dual3 D = cst(1.0) - cst(sa) * eta, D2 = D * D, D3 = D2 * D;
    const Dual3 Pr = cst(rho0 * ca2) * eta / D2;
    const Dual3 er = cst(0.5 * ca2) * eta * eta / D2;
    P = Pr + g * rho * (e - er);
    const Dual3 dPr = cst(ca2) * x * x * (cst(1.0) + cst(sa) * eta) / D3;
    const Dual3 rder = cst(ca2) * eta * x / D3;
    c2 = dPr + g * (e - er) - g * rder + g * P / rho;
}

// Sums a particle gathers over its partners.
struct VjpAcc {
    double gr0 = 0, gr1 = 0, gr2 = 0, gv0 = 0, gv1 = 0, gv2 = 0, gP = 0, gZ = 0, gV = 0;
    double Sr = 0, Sv0 = 0, Sv1 = 0, Sv2 = 0, SE = 0;
};

// dPhi_ij/dq_i for one partner j (i's data: ai = x y z V, bi = v P, zi = Z c,
// di = b_rho b_v, bEi = b_E), plus the plain rate sums S* the prefactor terms
// need.  Branch-free: a lane without a partner (use = false) computes on
// placeholder data (r2 = 1) and keeps its sums.
__device__ __forceinline__ void vjp_pair(bool use, double dx, double dy, double dz, double r2,
                                         const double4 &ai, const double4 &bi, const double2 &zi,
                                         const double4 &di, double bEi, const double4 &aj,
                                         const double4 &bj, const double2 &zj, const double4 &dj,
                                         double bEj, double invH, double dwc, VjpAcc &A) {
#pragma clang fp contract(fast)
    const double Vi = ai.w, Pi = bi.w, Zi = zi.x;
    const double Vj = aj.w, Pj = bj.w, Zj = zj.x;
    const double r = sqrt(use ? r2 : 1.0), ir = 1.0 / r;
    const double ex = dx * ir, ey = dy * ir, ez = dz * ir;
    const double q = r * invH, a1 = 1.0 - q;
    const double Wp = -dwc * q * (a1 * a1 * a1);
    const double Wpp = -dwc * invH * (a1 * a1) * (1.0 - 4.0 * q);
    const double vL = (bi.x * ex + bi.y * ey) + bi.z * ez;
    const double vR = (bj.x * ex + bj.y * ey) + bj.z * ez;
    const double S = Zi + Zj;
    const bool sok = S != 0.0;
    const double iS = 1.0 / (sok ? S : 1.0);
    const double vs = sok ? ((Zi * vL + Zj * vR) + (Pi - Pj)) * iS : 0.5 * (vL + vR);
    const double ps = sok ? ((Zj * Pi + Zi * Pj) + Zi * Zj * (vL - vR)) * iS : 0.5 * (Pi + Pj);
    const double dvs_dvL = sok ? Zi * iS : 0.5;
    const double dvs_dvR = sok ? Zj * iS : 0.5;
    const double dps_dvL = sok ? Zi * Zj * iS : 0.0;
    const double dps_dvR = -dps_dvL;
    const double dvs_dP = sok ? iS : 0.0;
    const double dps_dP = sok ? Zj * iS : 0.5;
    const double dvs_dZ = sok ? (vL - vs) * iS : 0.0;
    const double dps_dZ = sok ? ((Pj + Zj * (vL - vR)) - ps) * iS : 0.0;
    const double bvie = (di.y * ex + di.z * ey) + di.w * ez;
    const double bvje = (dj.y * ex + dj.z * ey) + dj.w * ez;
    const double Gi = di.x * (vL - vs) + ps * bvie + bEi * ps * vs;
    const double Gj = dj.x * (vs - vR) - ps * bvje - bEj * ps * vs;
    const double G = Vj * Gi + Vi * Gj;
    const double Gvs = Vj * (bEi * ps - di.x) + Vi * (dj.x - bEj * ps);
    const double Gps = Vj * (bvie + bEi * vs) - Vi * (bvje + bEj * vs);
    const double dGdvL = Vj * di.x + Gvs * dvs_dvL + Gps * dps_dvL;
    const double dGdvR = -Vi * dj.x + Gvs * dvs_dvR + Gps * dps_dvR;
    const double wv = Wp * dGdvL;
    const double u0 = (dGdvL * bi.x + dGdvR * bj.x) + ps * (Vj * di.y - Vi * dj.y);
    const double u1 = (dGdvL * bi.y + dGdvR * bj.y) + ps * (Vj * di.z - Vi * dj.z);
    const double u2 = (dGdvL * bi.z + dGdvR * bj.z) + ps * (Vj * di.w - Vi * dj.w);
    const double ue = (u0 * ex + u1 * ey) + u2 * ez;
    const double k1 = Wpp * G, k2 = Wp * ir;
    const double w = Vj * Wp;
    const double f = w * ps;
    A.gV = use ? A.gV + Wp * Gj : A.gV;
    A.gP = use ? A.gP + Wp * (Gvs * dvs_dP + Gps * dps_dP) : A.gP;
    A.gZ = use ? A.gZ + Wp * (Gvs * dvs_dZ + Gps * dps_dZ) : A.gZ;
    A.gv0 = use ? A.gv0 + wv * ex : A.gv0;
    A.gv1 = use ? A.gv1 + wv * ey : A.gv1;
    A.gv2 = use ? A.gv2 + wv * ez : A.gv2;
    // dJ/dr_i = -dPhi/dd
    A.gr0 = use ? A.gr0 - (k1 * ex + k2 * (u0 - ue * ex)) : A.gr0;
    A.gr1 = use ? A.gr1 - (k1 * ey + k2 * (u1 - ue * ey)) : A.gr1;
    A.gr2 = use ? A.gr2 - (k1 * ez + k2 * (u2 - ue * ez)) : A.gr2;
    A.Sr = use ? A.Sr + w * (vL - vs) : A.Sr;
    A.Sv0 = use ? A.Sv0 + f * ex : A.Sv0;
    A.Sv1 = use ? A.Sv1 + f * ey : A.Sv1;
    A.Sv2 = use ? A.Sv2 + f * ez : A.Sv2;
    A.SE = use ? A.SE + f * vs : A.SE;
}

// The stencil walk of the FP64 rate kernel (lock-step rows clipped to the
// support chord, partners queued per lane in LDS, drained with all lanes
// busy); partners are j != i with 0 < r_ij^2 < H^2 in FP64 without
// contraction, as in the forward pass.  WALL: a second walk, around i's
// mirror image, for the lanes within the wall's band.  PER: walks around the
// periodic images i has (image_faces), with offsets (x_j - x_i) - k L formed
// as the forward pass forms them; j is a partner of i through shift k exactly
// when i is one of j through -k (the offset negates exactly), so the gather
// stays complete.  With both, the mirror image's periodic images too.  PAIR:
// each pair's support H_ij = kappa (d_i + d_j)/2 (symmetric to the bit; d
// held fixed), the walk testing candidates against the largest support and
// the pop deciding membership with the pair's own.  MIRONLY (with WALL): only the mirror
// walks, for the workgroups holding wall-band particles, their contributions added to the
// outputs of a gather without the wall (which keeps that gather's register budget, and its
// occupancy, for every other particle).
template <bool WALL, bool PER, bool PAIR, bool MIRONLY = false>
__global__ __launch_bounds__(kBlock) void k_vjp64(int64_t n, VjpIn in, VjpOut o,
                                                  const int32_t *__restrict__ perm,
                                                  const int32_t *__restrict__ cs, GridDev g,
                                                  PairConst pc, EosDev eos, int n_eos,
                                                  VjpWall wl) {
    __shared__ int qj[kQ][kBlock];
    const int tid = threadIdx.x;
    const int64_t blk = xcd_block_upto(blockIdx.x, gridDim.x, 256);  // as the FP64 rate kernel
    const int64_t s = blk * kBlock + tid;
    const bool live = s < n;
    double ge_gamma = 0.0, ge_pinf = 0.0;
    int mt = 0;
    double4 ai = make_double4(0.0, 0.0, 0.0, 0.0), bi = ai, di = ai;
    double2 zi = make_double2(0.0, 0.0);
    double bEi = 0.0;
    if (live) {
        ai = in.A[s];
        bi = in.B[s];
        di = in.Dw[s];
        zi = in.C[s];
        bEi = in.Ew[s];
    }
    if (wl.p.band) {
        // correction pass: a workgroup without a particle within the support of the band's
        // reach adds nothing (a NaN reach, no flagged particle, admits none)
        const double thr = order_dec(*wl.p.band) + pc.H * (1.0 + 1e-9);
        if (!__syncthreads_or(live && ai.y <= thr)) {
            if (!MIRONLY && (int)threadIdx.x < 2 * n_eos)
                o.eos_part[blk * 2 * CSPH_MAX_EOS + threadIdx.x] = 0.0;
            return;
        }
    }
    // the mirror-only gather: workgroups without a wall-band particle add nothing
    if (MIRONLY && !__syncthreads_or(live && mirror_band(g, ai.y, wl.yw, pc.H))) return;
    const Stencil t = make_stencil(g, ai.x, ai.y, ai.z, pc.H);
    const double H2 = pc.H2;  // the largest support (pair-h mode), squared
    const double dself = PAIR && live ? in.dsz[s] : 0.0;
    const int self = (int)s;
    // i's mirror image (its y, and its velocity record with the normal component mirrored),
    // zero weights for the side of a pair that has no rate
    const double yim = WALL ? 2.0 * wl.yw - ai.y : 0.0;
    const double4 bim = make_double4(bi.x, wl.vw2 - bi.y, bi.z, bi.w);
    const double4 d0 = make_double4(0.0, 0.0, 0.0, 0.0);
    VjpAcc acc, accm;  // accm: the pairs (j, image of i), in the image's q
    int qw = 0, qr = 0;
    // (sx, sy, sz): the walk's periodic shift k L (0 off the periodic walks)
    auto drain = [&](bool ghost, double sx, double sy, double sz) {
        const bool has = qr < qw;
        const int j = has ? qj[qr & (kQ - 1)][tid] : 0;
        qr += has ? 1 : 0;
        const double4 aj = ld(in.A, j), bj = ld(in.B, j), dj = ld(in.Dw, j);
        const double2 zj = ld(in.C, j);
        const double bEj = ld(in.Ew, j);
        double invH = pc.invH, dwc = pc.dwc, H2p = H2;
        if (PAIR) {  // the pair's own support, as the forward pass forms it
            const double H = pc.kappa * (0.5 * (dself + ld(in.dsz, j)));
            H2p = H * H;
            invH = 1.0 / (H > 0.0 ? H : 1.0);
            const double i2 = invH * invH;
            dwc = (210.0 / M_PI) * (i2 * i2);
        }
        double dx = aj.x - ai.x, dz = aj.z - ai.z;
        if (PER) {
            dx = dx - sx;
            dz = dz - sz;
        }
        if (!ghost) {
            double dy = aj.y - ai.y;
            if (PER) dy = dy - sy;
            const double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
            vjp_pair(has && (!PAIR || r2 < H2p), dx, dy, dz, r2, ai, bi, zi, di, bEi, aj, bj, zj,
                     dj, bEj, invH, dwc, acc);
            return;
        }
        // (i, image of j): offset (2 y_w - y_j) - y_i, as the forward pass forms it (the
        // wall's axis y is never periodic: no shift along it)
        const double dya = (2.0 * wl.yw - aj.y) - ai.y;
        const double r2a = ((dx * dx) + (dya * dya)) + (dz * dz);
        const double4 bjm = make_double4(bj.x, wl.vw2 - bj.y, bj.z, bj.w);
        vjp_pair(has && r2a < H2p && r2a != 0.0, dx, dya, dz, r2a, ai, bi, zi, di, bEi, aj,
                 bjm, zj, d0, 0.0, invH, dwc, acc);
        // (j, image of i): j's forward offset (2 y_w - y_i) - y_j, negated exactly
        const double dyb = aj.y - yim;
        const double r2b = ((dx * dx) + (dyb * dyb)) + (dz * dz);
        vjp_pair(has && r2b < H2p && r2b != 0.0, dx, dyb, dz, r2b, ai, bim, zi, d0, 0.0, aj,
                 bj, zj, dj, bEj, invH, dwc, accm);
    };
    // one walk over stencil st (ghost: the stencil around i's mirror image, whose partners
    // are tested as both kinds of mirror pair; img: around a periodic image point, shift
    // (sx, sy, sz)), every entry drained before it returns
    auto walk = [&](const Stencil &st, bool ghost, bool img, bool on, double sx, double sy,
                    double sz) {
        int oy = st.R, oz = -st.R - 1;
        int k = 0, j0 = 0, len = 0, jlast = 0;
        for (;;) {
            if (__any(qw - qr > kQ - kU)) {
                drain(ghost, sx, sy, sz);
                continue;
            }
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
            double4 aj[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) aj[u] = ld(in.A, min(j0 + k + u, jlast));
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int j = j0 + k + u;
                double dx = aj[u].x - ai.x, dz = aj[u].z - ai.z;
                if (PER) {
                    dx = dx - sx;
                    dz = dz - sz;
                }
                bool ok;
                if (!ghost) {
                    double dy = aj[u].y - ai.y;
                    if (PER) dy = dy - sy;
                    const double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
                    ok = (k + u < len) && (img || j != self) && r2 < H2 && r2 != 0.0;
                } else {
                    const double dya = (2.0 * wl.yw - aj[u].y) - ai.y, dyb = aj[u].y - yim;
                    const double dxz = (dx * dx);
                    const double r2a = (dxz + (dya * dya)) + (dz * dz);
                    const double r2b = (dxz + (dyb * dyb)) + (dz * dz);
                    ok = (k + u < len) && ((r2a < H2 && r2a != 0.0) || (r2b < H2 && r2b != 0.0));
                }
                qj[qw & (kQ - 1)][tid] = j;
                qw += ok ? 1 : 0;
            }
            k += kU;
        }
        while (__any(qr < qw)) drain(ghost, sx, sy, sz);
    };
    // the walks around the periodic images of point (px, py, pz) (i, or its mirror image) for
    // the lanes in `on`, stencil base st
    const int nf = PER ? image_faces(pc, ai.x, ai.y, ai.z) : 0;
    auto images = [&](const Stencil &base, bool ghost, bool on, double py) {
        for (int m = 1; m < 8; ++m) {
            const bool onm = on && (nf & m) == m;
            if (!__any(onm)) continue;
            const double sx = image_shift(pc, nf, m, 0), sy = image_shift(pc, nf, m, 1),
                         sz = image_shift(pc, nf, m, 2);
            const Stencil sm = shifted_stencil(g, base, m, ai.x + sx, py + sy, ai.z + sz);
            walk(sm, ghost, true, onm, sx, sy, sz);
        }
    };
    if (!MIRONLY) {
        walk(t, false, false, live, 0.0, 0.0, 0.0);
        if (PER) images(t, false, live, ai.y);
    }
    if (WALL) {
        const bool near = live && mirror_band(g, ai.y, wl.yw, pc.H);
        if (__any(near)) {
            const Stencil ti = image_stencil(g, t, yim);
            walk(ti, true, false, near, 0.0, 0.0, 0.0);
            if (PER) images(ti, true, near, yim);
        }
        // the image's q back to i's: y and v_y change sign, P, Z and V are i's own
        acc.gr0 += accm.gr0;
        acc.gr1 -= accm.gr1;
        acc.gr2 += accm.gr2;
        acc.gv0 += accm.gv0;
        acc.gv1 -= accm.gv1;
        acc.gv2 += accm.gv2;
        acc.gP += accm.gP;
        acc.gZ += accm.gZ;
        acc.gV += accm.gV;
    }
    if (live) {
        double gr0 = acc.gr0, gr1 = acc.gr1, gr2 = acc.gr2, gv0 = acc.gv0, gv1 = acc.gv1,
               gv2 = acc.gv2, gP = acc.gP, gZ = acc.gZ, gV = acc.gV;
        const double Sr = acc.Sr, Sv0 = acc.Sv0, Sv1 = acc.Sv1, Sv2 = acc.Sv2, SE = acc.SE;
        // prefactors rho_i: dJ/drho_i += (a_rho R_rho - a_v.R_v - a_E R_E)/rho_i
        double rho = in.rho[s], E = in.E[s], m = in.m[s];
        double ar = in.a[0][s], ax = in.a[1][s], ay = in.a[2][s], az = in.a[3][s],
               aE = in.a[4][s];
        double Rr = -2.0 * rho * Sr, pre = 2.0 / rho;
        double grho = (ar * Rr - pre * ((ax * Sv0 + ay * Sv1) + az * Sv2) - aE * pre * SE) / rho;
        // V = m/rho, Z = rho c
        grho += -gV * m / (rho * rho);
        double c = zi.y;
        grho += gZ * c;
        double gc = gZ * rho;
        double gc2 = c > 0.0 ? gc / (2.0 * c) : 0.0;
        // EOS: e = E - |v|^2/2, P and c^2 of the material
        mt = in.mat ? in.mat[s] : 0;
        if (mt < 0 || mt >= eos.n) mt = 0;
        double gm = eos.gamma[mt], pinf = eos.pinf[mt];
        double e = E - 0.5 * ((bi.x * bi.x + bi.y * bi.y) + bi.z * bi.z);
        double ge;
        if (eos.type[mt] == CSPH_EOS_MIE_GRUNEISEN) {
            // partial derivatives in (rho, e, Gamma) carried forward through the EOS
            Dual3 P, c2;
            mg_eos_dual(eos, mt, rho, e, P, c2);
            ge = gP * P.de + gc2 * c2.de;
            grho += gP * P.dr + gc2 * c2.dr;
            ge_gamma = gP * P.dg + gc2 * c2.dg;
        } else if (eos.type[mt] == CSPH_EOS_STIFFENED) {
            // P = (g-1) rho e - g pinf ;  c^2 = g (g-1) (e - pinf/rho)
            ge = gP * (gm - 1.0) * rho + gc2 * gm * (gm - 1.0);
            grho += gP * (gm - 1.0) * e + gc2 * gm * (gm - 1.0) * pinf / (rho * rho);
            ge_gamma = gP * (rho * e - pinf) + gc2 * (2.0 * gm - 1.0) * (e - pinf / rho);
            ge_pinf = -gP * gm - gc2 * gm * (gm - 1.0) / rho;
        } else {
            // P = (g-1) rho e ;  c^2 = g (g-1) e
            ge = gP * (gm - 1.0) * rho + gc2 * gm * (gm - 1.0);
            grho += gP * (gm - 1.0) * e;
            ge_gamma = gP * rho * e + gc2 * (2.0 * gm - 1.0) * e;
        }
        double gEo = ge;
        gv0 -= ge * bi.x;
        gv1 -= ge * bi.y;
        gv2 -= ge * bi.z;
        double res[8] = {gr0, gr1, gr2, gv0, gv1, gv2, grho, gEo};
        int i = perm[s];
        if (wl.p.svy) {  // this gather's part of the y-momentum rate sum (k_wall_flags)
            if (MIRONLY)
                wl.p.svy[s] += Sv1;
            else
                wl.p.svy[s] = Sv1;
        }
        if (!MIRONLY && o.gn[0]) {
            // identity part of the step: r' = r + dt v', v' = v + dt dv, ...
            double gnx = o.gn[0][i], gny = o.gn[1][i], gnz = o.gn[2][i];
            res[0] += gnx;
            res[1] += gny;
            res[2] += gnz;
            res[3] += o.gn[3][i] + o.dt * gnx;
            res[4] += o.gn[4][i] + o.dt * gny;
            res[5] += o.gn[5][i] + o.dt * gnz;
            res[6] += o.gn[6][i];
            res[7] += o.gn[7][i];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) o.g[k][i] = o.accumulate ? o.g[k][i] + res[k] : res[k];
    }
    // deterministic per-block sums of the EOS-parameter gradients: a butterfly within each
    // wave, then the waves' sums in a fixed order (a few hundred bytes of LDS, which leaves
    // the workgroups per CU to the register budget)
    __shared__ double sh[kBlock / 64][2 * CSPH_MAX_EOS];
    for (int k = 0; k < 2 * n_eos; ++k) {
        double v = (s < n && mt == (k >> 1)) ? ((k & 1) ? ge_pinf : ge_gamma) : 0.0;
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][k] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < 2 * n_eos) {
        const int k = threadIdx.x;
        static_assert(kBlock == 256, "four waves per workgroup");
        const double v = (sh[0][k] + sh[1][k]) + (sh[2][k] + sh[3][k]);
        double *e = o.eos_part + blk * 2 * CSPH_MAX_EOS + k;
        *e = MIRONLY ? *e + v : v;
    }
}

// g_eos[k] += sum over blocks of part[b][k], fixed order.
__global__ __launch_bounds__(kBlock) void k_eos_grad_final(const double *__restrict__ part,
                                                           int64_t nblocks, int nk,
                                                           double *__restrict__ g_eos) {
    __shared__ double sh[kBlock];
    for (int k = 0; k < nk; ++k) {
        double acc = 0.0;
        for (int64_t b = threadIdx.x; b < nblocks; b += kBlock) acc += part[b * 2 * CSPH_MAX_EOS + k];
        sh[threadIdx.x] = acc;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) g_eos[k] += sh[0];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ the CFL time step
struct State8c {
    const double *f[8];
};
struct Rates5c {
    const double *f[5];
};
// What the binding particle's direct terms need (k_dt_fix): the state in cell order, its
// sound speeds (C records), materials, sizes (pair h), the gradients (input order).
struct DtFix {
    const DtInfo *info;
    double cfl;
    const int32_t *perm, *cs;
    const double *srt[8];
    const int32_t *mat;
    const double2 *C;
    const double *dsz;
    double *g[8];
    double *g_eos;
    double yw, vw2;  // the piston at the rates' time (kernels' y), twice its velocity
    int wall;
};

// Adjoint of dt = cfl min_s tau_s, tau_s = min(h_s / sig_s, rho_s / |drho_s|), the FP64 rate
// kernel's own expression, recomputed bit for bit from the rates and signal speeds it wrote.
// J's cotangent of dt, g_dt, is a sum over all particles; dt's gradient is that of the one
// tau that binds: through the signal speed (the Courant limit: sig_s = max(c_s, max over the
// partners of max(c_s, c_j) + max(0, v_L - v_R)), whose maximum passes the gradient to the
// partner attaining it) or through rho_s / |drho_s| (the density-change limit: the rate's
// part enters the rate cotangent of that particle before the gather).

// The slot that sets the step: tau_s equal to the minimum the rate kernel found (the
// smallest such slot).
__global__ __launch_bounds__(kBlock) void k_dt_argmin(int64_t n, const double *__restrict__ rho_s,
                                                      const double *__restrict__ drho_s,
                                                      const double *__restrict__ sig_s,
                                                      const double *__restrict__ d_s, double h,
                                                      const unsigned long long *dtmin,
                                                      DtInfo *info) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const double tau = fmin((d_s ? d_s[s] : h) / sig_s[s], rho_s[s] / fabs(drho_s[s]));
    if (dbits(tau) == *dtmin) atomicMin(&info->arg, (unsigned long long)s);
}

// The binding particle's data, kept before the gather's weights overwrite the rates.
__global__ void k_dt_pick(const double *__restrict__ rho_s, const double *__restrict__ drho_s,
                          const double *__restrict__ sig_s, const double *__restrict__ d_s,
                          double h, DtInfo *info) {
    if (threadIdx.x != 0) return;
    const unsigned long long s = info->arg;
    info->courant = 0;
    if (s == ~0ull) return;
    info->rho = rho_s[s];
    info->drho = drho_s[s];
    info->sig = sig_s[s];
    info->h = d_s ? d_s[s] : h;
    info->courant = info->h / info->sig <= info->rho / fabs(info->drho) ? 1 : 2;
}

// g_dt = sum_i g_i . dU_i'/d dt over the Euler step v' = v + dt R_v, E' = E + dt R_E,
// rho' = rho + dt R_rho, r' = r + dt v' (dr'/d dt = v + 2 dt R_v), the reflection off the
// piston at yw1 = y_w(t + dt) transposed as in k_vjp_reflect, plus its explicit 2 v_w g_y''.
// Per-block partial sums (fixed order).
__global__ __launch_bounds__(kBlock) void k_dt_cot(int64_t n, const int32_t *__restrict__ perm,
                                                   State8c u, Rates5c r, VjpOut o, int wall,
                                                   double yw1, double vw,
                                                   double *__restrict__ part) {
    const double dt = o.dt;
    double acc = 0.0;
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * kBlock) {
        const int i = perm[s];
        const double Fr = r.f[0][s], Fx = r.f[1][s], Fy = r.f[2][s], Fz = r.f[3][s],
                     FE = r.f[4][s];
        double gy = o.gn[1][i], gvy = o.gn[4][i], extra = 0.0;
        const double gE = o.gn[7][i];
        if (wall && u.f[1][s] + dt * (u.f[4][s] + dt * Fy) < yw1) {
            extra = 2.0 * vw * gy;
            gvy = -gvy - 2.0 * vw * gE;
            gy = -gy;
        }
        acc += ((o.gn[0][i] * (u.f[3][s] + 2.0 * dt * Fx) + gy * (u.f[4][s] + 2.0 * dt * Fy)) +
                o.gn[2][i] * (u.f[5][s] + 2.0 * dt * Fz)) +
               ((o.gn[3][i] * Fx + gvy * Fy) + o.gn[5][i] * Fz) +
               (o.gn[6][i] * Fr + gE * FE) + extra;
    }
    __shared__ double sh[kBlock];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// info->gdt = sum of the partial sums, fixed order.
__global__ __launch_bounds__(kBlock) void k_dt_cot_final(const double *__restrict__ part, int nb,
                                                         DtInfo *info) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) acc += part[b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) info->gdt = sh[0];
}

// The density-change limit binds: d tau/d drho = -rho sgn(drho) / drho^2 joins the rate
// cotangent a_rho (and its pair weight b_rho = -2 rho a_rho) of the binding slot.
__global__ void k_dt_fix_weights(const DtInfo *info, double cfl, const double *__restrict__ rho_s,
                                 double *a0, double4 *Dw) {
    if (threadIdx.x != 0 || info->courant != 2) return;
    const unsigned long long s = info->arg;
    const double dr = info->drho;
    const double x = cfl * info->gdt * (-info->rho * (dr > 0.0 ? 1.0 : -1.0) / (dr * dr));
    a0[s] += x;
    Dw[s].x -= 2.0 * rho_s[s] * x;
}

// Partials of c^2 in (rho, e, gamma, p_inf) of material k.
__device__ void c2_partials(const EosDev &eos, int k, double rho, double e, double &dr,
                            double &de, double &dg, double &dpi) {
    const double g = eos.gamma[k];
    dpi = 0.0;
    if (eos.type[k] == CSPH_EOS_MIE_GRUNEISEN) {
        Dual3 P, c2;
        mg_eos_dual(eos, k, rho, e, P, c2);
        dr = c2.dr;
        de = c2.de;
        dg = c2.dg;
    } else if (eos.type[k] == CSPH_EOS_STIFFENED) {
        // c^2 = g (g-1) (e - p_inf/rho)
        const double pinf = eos.pinf[k];
        dr = g * (g - 1.0) * pinf / (rho * rho);
        de = g * (g - 1.0);
        dg = (2.0 * g - 1.0) * (e - pinf / rho);
        dpi = -g * (g - 1.0) / rho;
    } else {
        // c^2 = g (g-1) e
        dr = 0.0;
        de = g * (g - 1.0);
        dg = (2.0 * g - 1.0) * e;
    }
}

// gc (a cotangent of c_s) through the EOS: c = sqrt(c^2(rho, e)), e = E - |v|^2/2.
__device__ void c_chain(const DtFix &f, const EosDev &eos, int64_t s, double gc) {
    const double c = f.C[s].y;
    if (!(c > 0.0) || gc == 0.0) return;
    int k = f.mat ? f.mat[s] : 0;
    if (k < 0 || k >= eos.n) k = 0;
    const double rho = f.srt[6][s], E = f.srt[7][s];
    const double vx = f.srt[3][s], vy = f.srt[4][s], vz = f.srt[5][s];
    const double e = E - 0.5 * ((vx * vx + vy * vy) + vz * vz);
    double dr, de, dg, dpi;
    c2_partials(eos, k, rho, e, dr, de, dg, dpi);
    const double g2 = gc / (2.0 * c);
    const int i = f.perm[s];
    f.g[6][i] += g2 * dr;
    f.g[7][i] += g2 * de;
    f.g[3][i] -= g2 * de * vx;
    f.g[4][i] -= g2 * de * vy;
    f.g[5][i] -= g2 * de * vz;
    if (f.g_eos) {
        f.g_eos[2 * k] += g2 * dg;
        f.g_eos[2 * k + 1] += g2 * dpi;
    }
}

// After the gather: the binding particle's direct terms.  Density-change limit: d tau/d rho =
// 1/|drho|.  Courant limit: tau = h/sig, d tau/d sig = -h/sig^2; the signal speed's maximum
// is found again over the particle's partners (real, periodic images, mirror images; the
// forward pass's membership), and its gradient goes to the sound speed that attains
// max(c_s, c_j) and, when the pair closes, to both velocities and positions through
// v_L - v_R = (v_s - v_j).e (a mirror partner's y and v_y mapped back to j's).  The
// workgroup searches the partners: the candidates come in a fixed order (image m, then the
// real cells before the mirror ones, cells z-, y-, then x-major within the reach, slots
// ascending), each thread takes every kBlock-th (image, kind, cell) task, and the partner
// kept is the first in that order that attains the largest speed above c_s (the one a walk
// in that order with a strict comparison keeps).  Thread 0 applies the terms.
// Task tk of the search: its image m, kind (mirror or real) and shift, and the key of its
// cell (-1 when the image is not one i has, or the cell is off the mesh).
__device__ __forceinline__ void dt_task(const GridDev &g, const PairConst &pc, const DtFix &f,
                                        int nf, int NC, int W, int tk, double xi, double yi,
                                        double zi, int &m, bool &ghost, double &sx, double &sy,
                                        double &sz, int &key) {
    m = tk / (2 * NC);
    ghost = ((tk / NC) & 1) != 0;
    const int c = tk % NC;
    key = -1;
    if ((nf & m) != m || (ghost && !f.wall)) return;
    sx = image_shift(pc, nf, m, 0);
    sy = image_shift(pc, nf, m, 1);
    sz = image_shift(pc, nf, m, 2);
    // the wall's axis y is never periodic: the mirror point is 2 y_w - y_i
    const double px = xi + sx, py = ghost ? 2.0 * f.yw - yi : yi + sy, pz = zi + sz;
    const int zz = free_cell(pz, g.oz, g.inv) - g.reach + c / (W * W);
    const int yy = free_cell(py, g.oy, g.inv) - g.reach + (c / W) % W;
    const int xx = free_cell(px, g.ox, g.inv) - g.reach + c % W;
    if (zz < 0 || zz >= g.dz || yy < 0 || yy >= g.dy || xx < 0 || xx >= g.dx) return;
    key = (int)cell_key(g, xx, yy, zz);
}

__global__ __launch_bounds__(kBlock) void k_dt_fix(DtFix f, GridDev g, PairConst pc,
                                                   EosDev eos) {
    const DtInfo &in = *f.info;
    const int courant = in.courant;
    if (courant == 0) return;
    const int64_t s = (int64_t)in.arg;
    const int i = f.perm[s];
    const double G0 = f.cfl * in.gdt;
    if (courant == 2) {
        if (threadIdx.x == 0) f.g[6][i] += G0 / fabs(in.drho);
        return;
    }
    const double G = G0 * (-in.h / (in.sig * in.sig));
    const double xi = f.srt[0][s], yi = f.srt[1][s], zi = f.srt[2][s];
    const double vxi = f.srt[3][s], vyi = f.srt[4][s], vzi = f.srt[5][s];
    const double ci = f.C[s].y;
    const double di = f.dsz ? f.dsz[s] : 0.0;
    const int nf = pc.per ? image_faces(pc, xi, yi, zi) : 0;
    const int W = 2 * g.reach + 1, NC = W * W * W;
    // the offsets of candidate j in (image m, kind) as the forward pass forms them
    auto offsets = [&](int64_t j, bool ghost, double sx, double sy, double sz, double &dx,
                       double &dy, double &dz) {
        dx = (f.srt[0][j] - xi) - sx;
        dy = ghost ? (2.0 * f.yw - f.srt[1][j]) - yi : (f.srt[1][j] - yi) - sy;
        dz = (f.srt[2][j] - zi) - sz;
    };
    double best = ci;
    unsigned long long bkey = ~0ull;  // (task << 32) | slot of the kept candidate
    for (int tk = threadIdx.x; tk < 16 * NC; tk += kBlock) {
        int m, key;
        bool ghost;
        double sx = 0.0, sy = 0.0, sz = 0.0;
        dt_task(g, pc, f, nf, NC, W, tk, xi, yi, zi, m, ghost, sx, sy, sz, key);
        if (key < 0) continue;
        for (int j = f.cs[key]; j < f.cs[key + 1]; ++j) {
            double dx, dy, dz;
            offsets(j, ghost, sx, sy, sz, dx, dy, dz);
            double H2 = pc.H2;
            if (pc.pair_mode) {
                const double H = pc.kappa * (0.5 * (di + f.dsz[j]));
                H2 = H * H;
            }
            const double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
            if (!(r2 < H2) || r2 == 0.0 || (!ghost && j == s)) continue;
            const double vyj = ghost ? f.vw2 - f.srt[4][j] : f.srt[4][j];
            const double r = sqrt(r2);
            const double vrel =
                (((vxi - f.srt[3][j]) * dx + (vyi - vyj) * dy) + (vzi - f.srt[5][j]) * dz) / r;
            const double sp = fmax(ci, f.C[j].y) + (vrel > 0.0 ? vrel : 0.0);
            if (sp > best) {
                best = sp;
                bkey = ((unsigned long long)tk << 32) | (unsigned)j;
            }
        }
    }
    // the largest speed, first in the order among equals
    __shared__ double shs[kBlock];
    __shared__ unsigned long long shk[kBlock];
    shs[threadIdx.x] = best;
    shk[threadIdx.x] = bkey;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double a = shs[threadIdx.x], b = shs[threadIdx.x + w];
            const unsigned long long ka = shk[threadIdx.x], kb = shk[threadIdx.x + w];
            if (b > a || (b == a && kb < ka)) {
                shs[threadIdx.x] = b;
                shk[threadIdx.x] = kb;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const unsigned long long k = shk[0];
    if (k == ~0ull) {  // no partner exceeds c_s: sig = c_s
        c_chain(f, eos, s, G);
        return;
    }
    const int tk = (int)(k >> 32);
    const int64_t bj = (int64_t)(k & 0xffffffffull);
    int m, key;
    bool bghost;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    dt_task(g, pc, f, nf, NC, W, tk, xi, yi, zi, m, bghost, sx, sy, sz, key);
    double bd[3];
    offsets(bj, bghost, sx, sy, sz, bd[0], bd[1], bd[2]);
    const double cj = f.C[bj].y;
    if (ci >= cj)
        c_chain(f, eos, s, G);
    else
        c_chain(f, eos, bj, G);
    const double vyj = bghost ? f.vw2 - f.srt[4][bj] : f.srt[4][bj];
    const double dv[3] = {vxi - f.srt[3][bj], vyi - vyj, vzi - f.srt[5][bj]};
    const double r = sqrt(((bd[0] * bd[0]) + (bd[1] * bd[1])) + (bd[2] * bd[2]));
    const double vrel = ((dv[0] * bd[0] + dv[1] * bd[1]) + dv[2] * bd[2]) / r;
    if (!(vrel > 0.0)) return;
    const int jj = f.perm[bj];
    const double fy = bghost ? -1.0 : 1.0;  // j's y and v_y enter a mirror partner negated
    for (int a = 0; a < 3; ++a) {
        const double e = bd[a] / r;
        const double q = (dv[a] - vrel * e) / r;  // d vrel / d (offset)
        const double sj = a == 1 ? fy : 1.0;
        f.g[3 + a][i] += G * e;
        f.g[3 + a][jj] -= G * e * sj;
        f.g[a][i] -= G * q;
        f.g[a][jj] += G * q * sj;
    }
}

hipError_t launch_dt_adjoint(int64_t n, const int32_t *perm, double *const sorted[9],
                             const Ws &w, const double *d_sorted, double h,
                             const double *const gnext[8], double dt, int wall, double yw1,
                             double vw, DtInfo *info, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    k_dt_argmin<<<nb, kBlock, 0, st>>>(n, sorted[6], w.rate[0], w.sig, d_sorted, h, w.dtmin,
                                       info);
    k_dt_pick<<<1, 64, 0, st>>>(sorted[6], w.rate[0], w.sig, d_sorted, h, info);
    State8c u;
    for (int k = 0; k < 8; ++k) u.f[k] = sorted[k];
    Rates5c r;
    for (int k = 0; k < 5; ++k) r.f[k] = w.rate[k];
    VjpOut o;
    for (int k = 0; k < 8; ++k) {
        o.g[k] = nullptr;
        o.gn[k] = gnext[k];
    }
    o.dt = dt;
    o.accumulate = 0;
    o.eos_part = nullptr;
    const unsigned nr = (unsigned)kReduceBlocks;
    k_dt_cot<<<nr, kBlock, 0, st>>>(n, perm, u, r, o, wall, yw1, vw, w.bounds_part);
    k_dt_cot_final<<<1, kBlock, 0, st>>>(w.bounds_part, (int)nr, info);
    return hipGetLastError();
}

// The gather's launches.  With the piston: the gather without the wall for every particle,
// then the mirror walks for the workgroups holding wall-band particles, added to its outputs
// (the epilogue is linear in the walks' sums, so the two launches give the one-walk gather's
// result up to the order of the additions).  The wall's walks and state take some 60 more
// VGPRs, which in one kernel would hold every workgroup to two waves per SIMD instead of three.
static void vjp_gather(unsigned nb, int64_t n, const VjpIn &in, const VjpOut &o,
                       const int32_t *perm, const int32_t *cs, const GridDev &g,
                       const PairConst &pc, const EosDev &eos, bool wall, const VjpWall &wl,
                       hipStream_t st) {
    VjpOut om = o;  // the mirror-only gather adds to the first one's outputs
    om.accumulate = 1;
    const bool per = pc.per != 0, pair = pc.pair_mode != 0;
#define CSPH_VJP_CASE(X, Q)                                                                  \
    if (per == X && pair == Q) {                                                             \
        k_vjp64<false, X, Q><<<nb, kBlock, 0, st>>>(n, in, o, perm, cs, g, pc, eos, eos.n, wl); \
        if (wall)                                                                            \
            k_vjp64<true, X, Q, true><<<nb, kBlock, 0, st>>>(n, in, om, perm, cs, g, pc, eos, \
                                                             eos.n, wl);                      \
    }
    CSPH_VJP_CASE(false, false)
    CSPH_VJP_CASE(false, true)
    CSPH_VJP_CASE(true, false)
    CSPH_VJP_CASE(true, true)
#undef CSPH_VJP_CASE
}

hipError_t launch_vjp(int64_t n, const int32_t *perm, const int32_t *cs, const GridDev &g,
                      const PairConst &pc, const EosDev &eos, const Ws &w,
                      double *const sorted[9], const int32_t *mat_sorted,
                      const double *const a_in[5], double *const gout[8],
                      const double *const gnext[8], double dt, int accumulate, double *g_eos,
                      const double *d_sorted, int wall, double yw, double vw, hipStream_t st,
                      const DtAdj *dta) {
    if (n <= 0) return hipSuccess;
    unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    VjpOut o;
    for (int k = 0; k < 8; ++k) {
        o.g[k] = gout[k];
        o.gn[k] = gnext ? gnext[k] : nullptr;
    }
    o.dt = dt;
    o.accumulate = accumulate;
    o.eos_part = w.eos_part;
    k_vjp_weights<<<nb, kBlock, 0, st>>>(n, perm, sorted[6], o, a_in ? a_in[0] : nullptr,
                                         a_in ? a_in[1] : nullptr, a_in ? a_in[2] : nullptr,
                                         a_in ? a_in[3] : nullptr, a_in ? a_in[4] : nullptr,
                                         w.rate[0], w.rate[1], w.rate[2], w.rate[3], w.rate[4],
                                         (double4 *)w.recD, w.recE);
    if (dta)  // the density-change limit's term, in the rate cotangent of the binding particle
        k_dt_fix_weights<<<1, 64, 0, st>>>(dta->info, dta->cfl, sorted[6], w.rate[0],
                                           (double4 *)w.recD);
    VjpIn in;
    in.A = (const double4 *)w.recA;
    in.B = (const double4 *)w.recB;
    in.C = (const double2 *)w.recC;
    in.Dw = (const double4 *)w.recD;
    in.Ew = w.recE;
    in.rho = sorted[6];
    in.E = sorted[7];
    in.m = sorted[8];
    in.mat = mat_sorted;
    for (int k = 0; k < 5; ++k) in.a[k] = w.rate[k];
    in.dsz = d_sorted;
    const VjpWall wl{yw, 2.0 * vw, WallPass{nullptr, nullptr}};
    vjp_gather(nb, n, in, o, perm, cs, g, pc, eos, wall != 0, wl, st);
    if (g_eos) k_eos_grad_final<<<1, kBlock, 0, st>>>(w.eos_part, (int64_t)nb, 2 * eos.n, g_eos);
    if (dta) {
        DtFix f;
        f.info = dta->info;
        f.cfl = dta->cfl;
        f.perm = perm;
        f.cs = cs;
        for (int k = 0; k < 8; ++k) f.srt[k] = sorted[k];
        f.mat = mat_sorted;
        f.C = (const double2 *)w.recC;
        f.dsz = d_sorted;
        for (int k = 0; k < 8; ++k) f.g[k] = gout[k];
        f.g_eos = g_eos;
        f.yw = yw;
        f.vw2 = 2.0 * vw;
        f.wall = wall;
        k_dt_fix<<<1, kBlock, 0, st>>>(f, g, pc, eos);
    }
    return hipGetLastError();
}

hipError_t launch_vjp_wall(int64_t n, const int32_t *perm, const int32_t *cs, const GridDev &g,
                           const PairConst &pc, const EosDev &eos, const Ws &w,
                           double *const sorted[9], const int32_t *mat_sorted,
                           const double *const a_in[5], double *const gout[8],
                           const double *const gnext[8], double dt, int accumulate,
                           double *g_eos, const double *d_sorted, double yw, double vw,
                           const WallPass &wp, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    VjpOut o;
    for (int k = 0; k < 8; ++k) {
        o.g[k] = gout[k];
        o.gn[k] = gnext ? gnext[k] : nullptr;
    }
    o.dt = dt;
    o.accumulate = accumulate;
    o.eos_part = w.eos_part;
    k_vjp_weights<<<nb, kBlock, 0, st>>>(n, perm, sorted[6], o, a_in ? a_in[0] : nullptr,
                                         a_in ? a_in[1] : nullptr, a_in ? a_in[2] : nullptr,
                                         a_in ? a_in[3] : nullptr, a_in ? a_in[4] : nullptr,
                                         w.rate[0], w.rate[1], w.rate[2], w.rate[3], w.rate[4],
                                         (double4 *)w.recD, w.recE);
    VjpIn in;
    in.A = (const double4 *)w.recA;
    in.B = (const double4 *)w.recB;
    in.C = (const double2 *)w.recC;
    in.Dw = (const double4 *)w.recD;
    in.Ew = w.recE;
    in.rho = sorted[6];
    in.E = sorted[7];
    in.m = sorted[8];
    in.mat = mat_sorted;
    for (int k = 0; k < 5; ++k) in.a[k] = w.rate[k];
    in.dsz = d_sorted;
    const VjpWall wl{yw, 2.0 * vw, wp};
    vjp_gather(nb, n, in, o, perm, cs, g, pc, eos, true, wl, st);
    if (g_eos) k_eos_grad_final<<<1, kBlock, 0, st>>>(w.eos_part, (int64_t)nb, 2 * eos.n, g_eos);
    return hipGetLastError();
}

// The step's reflection test, y + dt (v_y + dt R_vy) < yw1 (kernels' y, cell order, R_vy =
// (2/rho) S_vy from the gathers' sums), flag[i] in input order, and reach = max(y, 2 y_w - y)
// over the flagged particles.
__global__ __launch_bounds__(kBlock) void k_wall_flags(int64_t n, const int32_t *__restrict__ perm,
                                                       const double *__restrict__ y_s,
                                                       const double *__restrict__ vy_s,
                                                       const double *__restrict__ rho_s,
                                                       const double *__restrict__ svy,
                                                       double dt, double yw1, double yw,
                                                       int32_t *__restrict__ flag,
                                                       unsigned long long *reach) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const double y = y_s[s];
    const double vy1 = vy_s[s] + dt * ((2.0 / rho_s[s]) * svy[s]);
    const bool f = y + dt * vy1 < yw1;
    flag[perm[s]] = f ? 1 : 0;
    if (f) atomicMax(reach, order_enc(fmax(y, 2.0 * yw - y)));
}

hipError_t launch_wall_flags(int64_t n, const int32_t *perm, double *const sorted[9],
                             const double *svy, double dt, double yw1, double yw, int32_t *flag,
                             unsigned long long *reach, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_wall_flags<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        n, perm, sorted[1], sorted[4], sorted[6], svy, dt, yw1, yw, flag, reach);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_reflect_delta(int64_t n,
                                                          const double *__restrict__ gy,
                                                          const double *__restrict__ gvy,
                                                          const double *__restrict__ gE,
                                                          double vw, double *__restrict__ dy,
                                                          double *__restrict__ dvy) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    dy[i] = -2.0 * gy[i];
    dvy[i] = -2.0 * gvy[i] - 2.0 * vw * gE[i];
}

__global__ __launch_bounds__(kBlock) void k_keep_flagged(int64_t n,
                                                         const int32_t *__restrict__ flag,
                                                         double *__restrict__ dy,
                                                         double *__restrict__ dvy) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n || flag[i] != 0) return;
    dy[i] = 0.0;
    dvy[i] = 0.0;
}

hipError_t launch_reflect_delta(int64_t n, const double *gy, const double *gvy, const double *gE,
                                double vw, double *dy, double *dvy, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_reflect_delta<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, gy, gvy, gE, vw,
                                                                             dy, dvy);
    return hipGetLastError();
}

hipError_t launch_keep_flagged(int64_t n, const int32_t *flag, double *dy, double *dvy,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_keep_flagged<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, flag, dy, dvy);
    return hipGetLastError();
}

// The step's reflection off the piston, transposed.  A particle whose new position y' =
// y + dt (v_y + dt R_vy) lies behind the wall at the step's end, yw1, left the step with
// y'' = 2 yw1 - y', v_y'' = 2 v_w - v_y', E'' = E' + ((v_y'')^2 - (v_y')^2)/2 = E' + 2 v_w^2
// - 2 v_w v_y'; the cotangents of (y', v_y') follow from those of the step's output:
// g_y' = -g_y'', g_vy' = -g_vy'' - 2 v_w g_E'' (g_E' = g_E'', the other fields unchanged).
// Slot s in cell order (state and rates there, formed as the step forms them); the
// cotangents in input order.
__global__ __launch_bounds__(kBlock) void k_vjp_reflect(
    int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ y_s,
    const double *__restrict__ vy_s, const double *__restrict__ dvy_s, double dt, double yw1,
    double vw, const double *__restrict__ gy, const double *__restrict__ gvy,
    const double *__restrict__ gE, double *__restrict__ gy_out, double *__restrict__ gvy_out) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const int i = perm[s];
    const double vy = vy_s[s] + dt * dvy_s[s];
    const double y = y_s[s] + dt * vy;
    const bool behind = y < yw1;
    gy_out[i] = behind ? -gy[i] : gy[i];
    gvy_out[i] = behind ? -gvy[i] - 2.0 * vw * gE[i] : gvy[i];
}

hipError_t launch_vjp_reflect(int64_t n, const int32_t *perm, const double *y_s,
                              const double *vy_s, const double *dvy_s, double dt, double yw1,
                              double vw, const double *gy, const double *gvy, const double *gE,
                              double *gy_out, double *gvy_out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    k_vjp_reflect<<<nb, kBlock, 0, st>>>(n, perm, y_s, vy_s, dvy_s, dt, yw1, vw, gy, gvy, gE,
                                         gy_out, gvy_out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ the RK2 step
// The two-stage step U1 = U + dt F(U, t), r1 = r + dt v; U' = U/2 + (U1 + dt F(U1, t + dt))/2,
// r' = r/2 + (r1 + dt v1)/2, then the reflection off the piston at t + dt and the wrap.  With
// g' the cotangent of (r', U') (the reflection transposed; the wrap is a translation):
//   g_U1 = (g'_r/2, g'_v/2 + (dt/2) g'_r, g'_rho/2, g'_E/2) + F(U1)^T (dt/2) g'_(rho, v, E)
//   g_U  = g'/2 + (g_U1,r, g_U1,v + dt g_U1,r, g_U1,rho, g_U1,E) + F(U)^T dt g_U1,(rho, v, E)
// The F^T terms are rate VJPs (the library's own); these kernels form the rest, elementwise
// in input order and the caller's axes (the piston is normal to x).
__device__ __forceinline__ double wrap_box(const Rk2Vjp &q, int a, double v) {
    if (!((q.per >> a) & 1)) return v;
    if (v >= q.hi[a]) return v - (q.hi[a] - q.lo[a]);
    if (v < q.lo[a]) return v + (q.hi[a] - q.lo[a]);
    return v;
}

// U1 (formed as the forward step forms it), g' (the reflection transposed, tested on
// x' = x/2 + (x1 + dt v1x)/2 as the step tests it), the direct part of g_U1 and the rate
// cotangents (dt/2) g'_(rho, v, E) of the second evaluation.
__global__ __launch_bounds__(kBlock) void k_rk2_vjp_stage2(int64_t n, Rk2Vjp q) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double dt = q.dt;
    double v1[3], r1[3];
    for (int a = 0; a < 3; ++a) {
        v1[a] = q.s[3 + a][i] + dt * q.F[1 + a][i];
        r1[a] = q.s[a][i] + dt * q.s[3 + a][i];
        q.u1[a][i] = wrap_box(q, a, r1[a]);
        q.u1[3 + a][i] = v1[a];
    }
    q.u1[6][i] = q.s[6][i] + dt * q.F[0][i];
    q.u1[7][i] = q.s[7][i] + dt * q.F[4][i];
    double g[8];
    for (int k = 0; k < 8; ++k) g[k] = q.gn[k][i];
    if (q.wall && 0.5 * q.s[0][i] + 0.5 * (r1[0] + dt * v1[0]) < q.xw1) {
        g[3] = -g[3] - 2.0 * q.vw * g[7];
        g[0] = -g[0];
    }
    q.gx[i] = g[0];
    q.gvx[i] = g[3];
    const double h = 0.5 * dt;
    for (int a = 0; a < 3; ++a) {
        q.gu1[a][i] = 0.5 * g[a];
        q.gu1[3 + a][i] = 0.5 * g[3 + a] + h * g[a];
        q.a[1 + a][i] = h * g[3 + a];
    }
    q.gu1[6][i] = 0.5 * g[6];
    q.gu1[7][i] = 0.5 * g[7];
    q.a[0][i] = h * g[6];
    q.a[4][i] = h * g[7];
}

// After the rate VJP at U1 has completed g_U1: the rate cotangents dt g_U1,(rho, v, E) of the
// first evaluation and g_U's direct part (gp may alias the output's cotangent: each element
// is read before it is written).
__global__ __launch_bounds__(kBlock) void k_rk2_vjp_stage1(int64_t n, Rk2Vjp q, double *gp0,
                                                           double *gp1, double *gp2,
                                                           double *gp3, double *gp4,
                                                           double *gp5, double *gp6,
                                                           double *gp7) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double dt = q.dt;
    double g[8], u[8];
    for (int k = 0; k < 8; ++k) {
        g[k] = q.gn[k][i];
        u[k] = q.gu1[k][i];
    }
    g[0] = q.gx[i];
    g[3] = q.gvx[i];
    double *gp[8] = {gp0, gp1, gp2, gp3, gp4, gp5, gp6, gp7};
    for (int a = 0; a < 3; ++a) {
        gp[a][i] = 0.5 * g[a] + u[a];
        gp[3 + a][i] = 0.5 * g[3 + a] + (u[3 + a] + dt * u[a]);
        q.a[1 + a][i] = dt * u[3 + a];
    }
    gp[6][i] = 0.5 * g[6] + u[6];
    gp[7][i] = 0.5 * g[7] + u[7];
    q.a[0][i] = dt * u[6];
    q.a[4][i] = dt * u[7];
}

hipError_t launch_rk2_vjp_stage2(int64_t n, const Rk2Vjp &q, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_rk2_vjp_stage2<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, q);
    return hipGetLastError();
}

hipError_t launch_rk2_vjp_stage1(int64_t n, const Rk2Vjp &q, double *const gp[8],
                                 hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_rk2_vjp_stage1<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        n, q, gp[0], gp[1], gp[2], gp[3], gp[4], gp[5], gp[6], gp[7]);
    return hipGetLastError();
}

// dE0/d(gamma, p_inf, v, rho) of E0 = e0(rho, p; gamma, p_inf) + |v|^2/2,
// e0 = p/((g-1) rho) (ideal), (p + g p_inf)/((g-1) rho) (stiffened), or
// e_r + (p - P_r)/(Gamma rho) (Mie-Grueneisen: d/dGamma in the gamma slot).
__global__ __launch_bounds__(kBlock) void k_init_energy_vjp(
    const double *__restrict__ rho, const double *__restrict__ pres, const double *__restrict__ vx,
    const double *__restrict__ vy, const double *__restrict__ vz, const int32_t *__restrict__ mat,
    int64_t n, EosDev eos, const double *__restrict__ gE, double *g_vx, double *g_vy,
    double *g_vz, double *g_rho, double *__restrict__ part) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double gg = 0.0, gp = 0.0;
    int k = 0;
    if (i < n) {
        k = mat ? mat[i] : 0;
        if (k < 0 || k >= eos.n) k = 0;
        double g = eos.gamma[k], pinf = eos.pinf[k], r = rho[i], p = pres[i], a = gE[i];
        double e0, de0;  // e0 and de0/drho
        if (eos.type[k] == CSPH_EOS_MIE_GRUNEISEN) {
            // e0 = e_r + (p - P_r)/(Gamma rho), with its partials in (rho, Gamma)
            const Dual3 rr{r, 1.0, 0.0, 0.0}, gd{g, 0.0, 0.0, 1.0};
            const double rho0 = eos.rho0[k], ca2 = eos.ca[k] * eos.ca[k], sa = eos.sa[k];
            const Dual3 x = cst(rho0) / rr, eta = cst(1.0) - x;
            const Dual3 D = cst(1.0) - cst(sa) * eta, D2 = D * D;
            const Dual3 Pr = cst(rho0 * ca2) * eta / D2;
            const Dual3 er = cst(0.5 * ca2) * eta * eta / D2;
            const Dual3 ed = er + (cst(p) - Pr) / (gd * rr);
            e0 = ed.v;
            de0 = ed.dr;
            gg = a * ed.dg;
        } else if (eos.type[k] == CSPH_EOS_STIFFENED) {
            e0 = (p + g * pinf) / ((g - 1.0) * r);
            de0 = -e0 / r;
            gg = a * (pinf / ((g - 1.0) * r) - e0 / (g - 1.0));
            gp = a * (g / ((g - 1.0) * r));
        } else {
            e0 = p / ((g - 1.0) * r);
            de0 = -e0 / r;
            gg = a * (-e0 / (g - 1.0));
        }
        if (g_vx) g_vx[i] += a * vx[i];
        if (g_vy) g_vy[i] += a * vy[i];
        if (g_vz) g_vz[i] += a * vz[i];
        if (g_rho) g_rho[i] += a * de0;
    }
    __shared__ double sh[2 * CSPH_MAX_EOS][kBlock];
    for (int q = 0; q < 2 * eos.n; ++q) sh[q][threadIdx.x] = 0.0;
    if (i < n) {
        sh[2 * k][threadIdx.x] = gg;
        sh[2 * k + 1][threadIdx.x] = gp;
    }
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 2 * eos.n; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        __syncthreads();
    }
    if ((int)threadIdx.x < 2 * eos.n)
        part[(int64_t)blockIdx.x * 2 * CSPH_MAX_EOS + threadIdx.x] = sh[threadIdx.x][0];
}

hipError_t launch_init_energy_vjp(const double *rho, const double *pres, const double *vx,
                                  const double *vy, const double *vz, const int32_t *mat,
                                  int64_t n, const EosDev &eos, const double *gE, double *g_vx,
                                  double *g_vy, double *g_vz, double *g_rho, double *g_eos,
                                  double *part, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    k_init_energy_vjp<<<nb, kBlock, 0, st>>>(rho, pres, vx, vy, vz, mat, n, eos, gE, g_vx, g_vy,
                                             g_vz, g_rho, part);
    if (g_eos) k_eos_grad_final<<<1, kBlock, 0, st>>>(part, (int64_t)nb, 2 * eos.n, g_eos);
    return hipGetLastError();
}

}  // namespace csph
