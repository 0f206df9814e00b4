// Internal declarations of the gfx950 contact-SPH library: device helpers,
// the workspace layout and the host-side launchers of each kernel file.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>

#include "csph.h"

namespace csph {

constexpr int kBlock = 256;           // threads per workgroup (4 wave64)
constexpr int kReduceBlocks = 1024;   // partial-reduction blocks (bounds, totals)
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;
constexpr int kMaxSites = 1024;       // Voronoi generators held in LDS (36 B each)
constexpr int kMaxBalanceSites = 512; // balancer generators held in LDS (84 B each)
constexpr int kXcd = 8;               // accelerator dies; workgroups go to them round robin
constexpr int kSlabShift = 4;         // cell order: y-slabs of 16 rows (see cell_key)
constexpr int kVlChunk = 8;           // Verlet-list entries per lane-owned 32-byte chunk
// The pair walks address per-particle records (up to 32 bytes) with 32-bit byte offsets.
constexpr int64_t kMaxPairN = (int64_t)1 << 27;

// Mesh as the kernels see it.
struct GridDev {
    double ox, oy, oz;  // origin
    double inv;         // 1/D
    double cell;        // D
    int dx, dy, dz;     // dims
    int reach;          // stencil half-width
    // cell order (cell_key): y-slabs of 2^ysh rows, z, then y in slab, then x
    int ysh, ymask, nfull;      // slab shift and mask; number of full slabs
    uint32_t sY, sZf, sZr;      // slab stride; z stride in a full / the last slab
    double ymin;                // minimum y of the particles (the origin may lie below it)
    int morton;                 // binning keys: 1 = Morton (csph_bin's export only)
    int64_t nkey;               // key space of the binning (cells, or 2^(3 bits) for Morton)
    // the minimum y found on the device by the binning (order_enc), for steps on a mesh the
    // caller gives; null: ymin
    const unsigned long long *yenc;
};

// A double as an unsigned integer of the same order (the sign bit set for v >= 0, every bit
// flipped for v < 0), so that integer atomics take minima of doubles.
__device__ __forceinline__ unsigned long long order_enc(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double order_dec(unsigned long long e) {
    const unsigned long long b = (e >> 63) ? (e & 0x7fffffffffffffffull) : ~e;
    return __longlong_as_double((long long)b);
}

// Checks the binning makes for a step on a mesh the caller gives (no bounds pass): the minimum
// y (yenc, reset to ~0 before), and the count of particles outside the mesh or, along a
// periodic axis (per, in the kernels' axes), outside the box [lo, hi].  Null pointers skip.
struct BinCheck {
    unsigned long long *yenc;
    unsigned long long *outside;
    int per;
    double lo[3], hi[3];
};

// Morton key: bit b of cx, cy, cz at key bits 3b, 3b+1, 3b+2 (10 bits each).  Each
// coordinate's bits are spread to every third position by shifts and masks.
__host__ __device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__host__ __device__ __forceinline__ uint32_t morton_key(int cx, int cy, int cz) {
    return spread3((uint32_t)cx) | (spread3((uint32_t)cy) << 1) | (spread3((uint32_t)cz) << 2);
}

// Key of cell (cx, cy, cz).  The mesh is cut along y into slabs of 2^ysh
// rows (the last one may be shorter); slabs come one after another, and in a
// slab the cells are ordered by z, then y, then x.  x is fastest, so a
// stencil row (fixed y, z) is one contiguous key range, while consecutive
// keys stay within a slab a few rows thick: the stencil neighbourhood of a
// stretch of particles is small.  With a single slab (ysh >= 31) this is the
// plain linear key (cz * dy + cy) * dx + cx.  Keys cover [0, dx*dy*dz).
__host__ __device__ __forceinline__ uint32_t cell_key(const GridDev &g, int cx, int cy, int cz) {
    const int sl = cy >> g.ysh;
    return (uint32_t)sl * g.sY + (uint32_t)cz * (sl < g.nfull ? g.sZf : g.sZr) +
           (uint32_t)(cy & g.ymask) * (uint32_t)g.dx + (uint32_t)cx;
}

// Workgroups are handed to the dies round robin.  Renumber them so that a die
// runs chunks of C consecutive workgroups (its L2 then holds the stencil
// neighbourhood of a stretch of cells instead of scattered pieces), the dies
// taking the chunks in turn, so that a region of costly particles (the wall
// band) is shared by all dies instead of falling on one.  Workgroups past the
// last whole round of chunks keep their number.
template <unsigned C>
__device__ __forceinline__ int64_t xcd_block(unsigned b, unsigned nb) {
    const unsigned round = kXcd * C, full = nb / round * round;
    if (b >= full) return b;
    const unsigned x = b % kXcd, t = b / kXcd;
    return ((int64_t)(t / C) * kXcd + x) * C + t % C;
}

// The same with chunks of at most C workgroups, smaller in a launch of fewer than four
// rounds of such chunks (whose groups would otherwise keep their numbers, spread over the
// dies): C' = min(C, nb / (4 kXcd)), at least 1.  Wave-uniform, so the compiler keeps it in
// scalar registers.
__device__ __forceinline__ int64_t xcd_block_upto(unsigned b, unsigned nb, unsigned C) {
    unsigned c = nb / (4u * kXcd);
    c = c < 1u ? 1u : (c < C ? c : C);
    const unsigned round = kXcd * c, full = nb / round * round;
    if (b >= full) return b;
    const unsigned x = b % kXcd, t = b / kXcd;
    return ((int64_t)(t / c) * kXcd + x) * c + t % c;
}

// Per-call constants of the pair interaction.
struct PairConst {
    double H;        // support (fixed mode)
    double H2;       // H*H (fixed mode)
    double invH;     // 1/H (fixed mode)
    double dwc;      // (210/pi)/H^4 (fixed mode)
    double kappa;    // pair mode: H_ij = kappa * (0.5*(d_i+d_j))
    double h_dt;     // h in the CFL rule (fixed mode)
    // Piston wall y = wall_y0 + wall_v t in the kernels' axes.  The wall of the
    // interface is normal to x; with a wall (and with a periodic x and an open y)
    // the library hands the kernels the x and y arrays (positions, velocities,
    // rates) swapped, so that the boundary's normal runs along the slab axis of
    // the cell order instead of its row axis: the particles within its support
    // then fill a few waves instead of a few lanes of every wave that starts a
    // row.  Squared distances ((dx dx + dy dy) + dz dz) do not change under the
    // swap, to the last bit.
    double wall_y0, wall_v;
    int pair_mode;
    int wall;
    // Periodic axes in the kernels' axes (bit a), the box [lo, hi) of each and its period
    // L = hi - lo; hb: the near-face band (the support with a relative margin of 1e-6).  A
    // particle within hb of the low face of a periodic axis has its image partners across that
    // face at x_j - L (shift k = +1), one within hb of the high face at x_j + L (k = -1); the
    // library requires L > 2 hb, so no particle is near both faces of an axis.
    int per;
    double hb;
    double lo[3], hi[3], L[3];
};

struct EosDev {
    int n;
    int type[CSPH_MAX_EOS];
    double gamma[CSPH_MAX_EOS];  // adiabatic index, or Grueneisen Gamma
    double pinf[CSPH_MAX_EOS];
    double rho0[CSPH_MAX_EOS], ca[CSPH_MAX_EOS], sa[CSPH_MAX_EOS];  // Mie-Grueneisen
};

// Mie-Grueneisen reference curves of the linear u_s - u_p Hugoniot
// (eq. mie_gruneisen_reference) at x = rho0/rho; returns D = 1 - s_a (1 - x).
__device__ __forceinline__ double mg_reference(const EosDev &eos, int k, double rho, double &Pr,
                                               double &er) {
    const double rho0 = eos.rho0[k], ca = eos.ca[k], sa = eos.sa[k];
    const double x = rho0 / rho;
    const double eta = 1.0 - x;
    const double D = 1.0 - sa * eta;
    const double D2 = D * D;
    Pr = rho0 * ca * ca * eta / D2;
    er = 0.5 * ca * ca * eta * eta / D2;
    return D;
}

// Pressure and squared sound speed of material k at (rho, e): ideal gas,
// stiffened gas, or Mie-Grueneisen (eq. mie_gruneisen_eos with the sound
// speed c^2 = (dP/drho)_e + (P/rho^2)(dP/de)_rho; -1 past the Hugoniot's
// compression limit).  FP64, no contraction.
__device__ __forceinline__ void eos_eval(const EosDev &eos, int k, double rho, double e,
                                         double &P, double &c2) {
    const double gm = eos.gamma[k];
    if (eos.type[k] == CSPH_EOS_MIE_GRUNEISEN) {
        const double ca = eos.ca[k], sa = eos.sa[k];
        double Pr, er;
        const double D = mg_reference(eos, k, rho, Pr, er);
        const double x = eos.rho0[k] / rho, eta = 1.0 - x, D3 = D * D * D;
        P = Pr + gm * rho * (e - er);
        const double dPr = ca * ca * x * x * (1.0 + sa * eta) / D3;
        const double rder = ca * ca * eta * x / D3;
        c2 = dPr + gm * (e - er) - gm * rder + gm * P / rho;
        if (!(D > 0.0)) c2 = -1.0;
    } else if (eos.type[k] == CSPH_EOS_STIFFENED) {
        const double pinf = eos.pinf[k];
        P = (gm - 1.0) * rho * e - gm * pinf;
        c2 = gm * (P + pinf) / rho;
    } else {
        P = (gm - 1.0) * rho * e;
        c2 = gm * P / rho;
    }
}

// Specific internal energy of material k at (rho, P): the EOS inverse.
__device__ __forceinline__ double eos_energy(const EosDev &eos, int k, double rho, double p) {
    const double g = eos.gamma[k];
    if (eos.type[k] == CSPH_EOS_MIE_GRUNEISEN) {
        double Pr, er;
        mg_reference(eos, k, rho, Pr, er);
        return er + (p - Pr) / (g * rho);
    }
    if (eos.type[k] == CSPH_EOS_STIFFENED) return (p + g * eos.pinf[k]) / ((g - 1.0) * rho);
    return p / ((g - 1.0) * rho);
}

// Cell coordinate min(floor((v - o) * inv), dim - 1), clamped at 0, FP64
// without contraction (the library is built with -ffp-contract=off).
__device__ __forceinline__ int cell_coord(double v, double o, double inv, int dim) {
    double f = floor((v - o) * inv);
    f = fmin(fmax(f, 0.0), (double)(dim - 1));
    return (int)f;
}

// Bit pattern of a non-negative double orders like the double itself.
__device__ __forceinline__ unsigned long long dbits(double v) {
    return (unsigned long long)__double_as_longlong(v);
}

// ---------------------------------------------------------------- device buffers
// Carved out of the caller's workspace, each region 256-byte aligned.
struct Ws {
    double *bounds_part;          // kReduceBlocks * 8
    double *bounds_out;           // 8
    uint32_t *key;                // n
    uint32_t *rank;               // n
    int32_t *cs;                  // ncell + 1
    int64_t *scan_tmp;            // scan tiles
    int32_t *perm;                // n
    int32_t *bin_tmp;             // n: cell order before the in-cell ranking (binning only)
    void *recA, *recB, *recC;     // pair records (FP64: 32+32+16 B; mixed: 16+16+8 B)
    void *recF;                   // FP64 stencil walks: cell-relative FP32 records (16 B)
    void *recD;                   // adjoint pair weights (32 B)
    double *recE;                 // adjoint energy weight
    double *eos_part;             // per-block EOS-parameter gradients, ceil(n/kBlock) * 16
    double *srt[9];               // sorted state copy x y z vx vy vz rho E m
    int32_t *srt_mat;
    double *srt_d;
    int64_t *srt_id;
    double *rate[5];              // drho dvx dvy dvz dE (cell order)
    double *sig;                  // signal speed (cell order)
    int32_t *cnt;                 // neighbour count (cell order)
    unsigned long long *dtmin;    // bits of min_i h_i/s_i
    unsigned long long *zflag;    // 0 once the pack meets a zero impedance Z = rho c
    int64_t *nonphys;             // scratch counter
    unsigned long long *yenc;     // steps on a caller's mesh: the particles' minimum y (order_enc)
    double *tot_part;             // kReduceBlocks * 10
    // two-stage Runge-Kutta steps only (ws_layout with rk2): the predicted state U1 in the
    // first stage's cell order (x, y, z wrapped into a periodic box; vx vy vz rho E), the
    // second stage's sorted copy, order and cell ranges, the first stage's neighbour counts
    // and the second stage's time t + dt
    double *stg[8];
    double *srt2[9];
    double *srt2_d;
    int32_t *perm2;
    int32_t *rk_cnt;
    double *t2;
    int32_t *cs2;                 // ncell2 + 1
    int64_t *scan_tmp2;           // scan tiles of the second mesh
    size_t bytes;
};

size_t ws_layout(Ws *w, void *base, int64_t n, int64_t ncell, bool rk2 = false,
                 int64_t ncell2 = 0);

// ---------------------------------------------------------------- launchers
// Every launcher enqueues on `st` and returns the HIP status of the launch.

// k_bin.hip
hipError_t launch_bounds(const double *x, const double *y, const double *z, const double *d,
                         int64_t n, double *part, double *out, hipStream_t st);
hipError_t launch_bin(const double *x, const double *y, const double *z, int64_t n,
                      const GridDev &g, const Ws &w, int32_t *perm, uint32_t *key_out,
                      int32_t *cell_start, hipStream_t st, const BinCheck *chk = nullptr);
template <typename TI, typename TO>
hipError_t launch_scan_exclusive(const TI *in, TO *out, int64_t len, int64_t *tmp, hipStream_t st);

// k_rates.hip
// gate (optional, device): the kernel does nothing while *gate == 0 (a Verlet-list step whose
// lists were found stale; csph_vlist_ctl::valid)
hipError_t launch_pack(const csph_state &s, int64_t n, const int32_t *perm, const EosDev &eos,
                       int mixed, const GridDev &g, const Ws &w, double *const dst[9],
                       int32_t *dst_mat, double *dst_d, int64_t *dst_id, const int64_t *src_id,
                       int64_t *nonphys, hipStream_t st, const int32_t *gate = nullptr);
// sorted: the cell-ordered FP64 state (x y z vx vy vz rho E m) the records were packed from.
hipError_t launch_rates(int64_t n, int mixed, const GridDev &g, const PairConst &pc,
                        const Ws &w, double *const sorted[9], const double *d_sorted,
                        const double *t_dev, double t_host, int want_dt, hipStream_t st,
                        const int32_t *vl_count = nullptr, const int32_t *vl_idx = nullptr,
                        int vl_cap = 0, const int32_t *gate = nullptr);
// Verlet-list control block: reset at a build; the per-step guard (csph_step_vlist).
hipError_t launch_vl_init(csph_vlist_ctl *ctl, const double *t, double margin, double vw2,
                          hipStream_t st);
hipError_t launch_vl_guard(csph_vlist_ctl *ctl, const double *t, hipStream_t st);
hipError_t launch_copy_i32(int32_t *dst, const int32_t *src, int64_t n, const int32_t *gate,
                           hipStream_t st);
// k_vlist.hip
hipError_t launch_vlist(int64_t n, const double4 *A, const int32_t *cs, const GridDev &g,
                        double R, int wall, double yw, int cap, int32_t *count, int32_t *idx,
                        unsigned long long *over, hipStream_t st);
hipError_t launch_disp(int64_t n, const double *x, const double *y, const double *z,
                       const double *ref, unsigned long long *out, hipStream_t st,
                       const int32_t *gate = nullptr);
hipError_t launch_unsort_rates(int64_t n, const int32_t *perm, const Ws &w, csph_rates_out out,
                               double *signal, int32_t *nbr_count, hipStream_t st);

// k_step.hip
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t count, hipStream_t st);
hipError_t launch_add_i64(int64_t *dst, const int64_t *src, hipStream_t st);  // *dst += *src
// Voronoi ownership computed by the step's update (csph_step_voronoi): K generators (K x 3,
// the caller's axes; swap = the kernels see x and y exchanged), owner written at i (cell
// order) or at owner_at[i], per-site particle and pair counts (cnt, cell order) overwritten.
struct VoroDev {
    const double *sites;
    int K;
    int ax[3];  // the caller's axis of each of the kernels' axes
    int32_t *owner;
    const int32_t *owner_at;
    const int32_t *cnt;
    unsigned long long *site_part, *site_pairs;
};
// A Verlet-list step's gate and counters: the update does nothing while *gate == 0; otherwise
// it adds sum_i cnt[i] to *pairs and the finishing kernel adds 1 to *steps.
struct ListGate {
    const int32_t *gate;
    const int32_t *cnt;
    unsigned long long *pairs;
    int32_t *steps;
};
// With pc.wall (and t, the device time at the step's start), particles behind the piston
// plane at the new time are reflected off it.  vo (optional): also the Voronoi ownership.
// Two-stage Runge-Kutta: the predicted state U1 (into w.stg, with the first stage's counts
// saved and t + dt) and the convex combination of the second stage (in place in st8, the first
// stage's cell order, with block partial totals).
hipError_t launch_rk2_predict(int64_t n, double *const st8[9], const Ws &w, double cfl,
                              double dt_in, const PairConst &pc, const double *t, hipStream_t st);
hipError_t launch_rk2_combine(int64_t n, double *const st8[9], const Ws &w, double cfl,
                              double dt_in, const PairConst &pc, const double *t, hipStream_t st);
hipError_t launch_integrate(int64_t n, double *const st8[9], const Ws &w, double cfl, double dt_in,
                            const PairConst &pc, const double *t, hipStream_t st,
                            const VoroDev *vo = nullptr, const ListGate *lg = nullptr);
hipError_t launch_finish_step(int64_t n, const Ws &w, double cfl, double dt_in, double *t, double *dt_used,
                              double *totals, const int ax[3], hipStream_t st,
                              const ListGate *lg = nullptr);
hipError_t launch_unpermute(int64_t n, const int32_t *perm, double *const src[9],
                            const int32_t *src_mat, const double *src_d, const int64_t *src_id,
                            const int32_t *src_cnt, const csph_state &out, int32_t *out_cnt,
                            hipStream_t st);
hipError_t launch_init_energy(const double *rho, const double *pres, const double *vx,
                              const double *vy, const double *vz, const int32_t *mat, int64_t n,
                              const EosDev &eos, double *E, hipStream_t st);

// k_adjoint.hip
// The CFL time step's adjoint (csph_step_vjp_cfl): the slot whose tau = min(h/sig,
// rho/|drho|) sets the step, which limit binds, and J's cotangent of dt.
struct DtInfo {
    unsigned long long arg;  // binding slot (cell order); ~0 before k_dt_argmin
    int courant;             // 1: the Courant limit binds, 2: the density-change limit
    int pad;
    double rho, drho, sig, h;  // the binding slot's density, density rate, signal speed, h
    double gdt;              // J's cotangent of dt
};
struct DtAdj {
    DtInfo *info;
    double cfl;
};
// Finds the binding slot (the FP64 rates and signal speeds of the step's state in w.rate,
// w.sig, the minimum in w.dtmin) and g_dt from the next state's cotangent (input order).
hipError_t launch_dt_adjoint(int64_t n, const int32_t *perm, double *const sorted[9],
                             const Ws &w, const double *d_sorted, double h,
                             const double *const gnext[8], double dt, int wall, double yw1,
                             double vw, DtInfo *info, hipStream_t st);
hipError_t launch_vjp(int64_t n, const int32_t *perm, const int32_t *cs, const GridDev &g,
                      const PairConst &pc, const EosDev &eos, const Ws &w,
                      double *const sorted[9], const int32_t *mat_sorted,
                      const double *const a_in[5], double *const gout[8],
                      const double *const gnext[8], double dt, int accumulate, double *g_eos,
                      const double *d_sorted, int wall, double yw, double vw, hipStream_t st,
                      const DtAdj *dta = nullptr);
// Step VJP with the piston: the cotangents of the pre-reflection y and v_y (input order) from
// the next state's (the state and its rates in cell order; yw1 the wall at the step's end).
// The RK2 step's VJP: its elementwise parts (k_adjoint.hip), in input order and the caller's
// axes.
struct Rk2Vjp {
    const double *s[8];   // U: x y z vx vy vz rho E
    const double *F[5];   // F(U): drho dvx dvy dvz dE
    const double *gn[8];  // the cotangent of the step's output
    double *u1[8];        // U1, its positions wrapped into the periodic box
    double *gx, *gvx;     // g' of x and v_x (the piston's reflection transposed)
    double *gu1[8];       // g_U1
    double *a[5];         // rate cotangents (rho vx vy vz E)
    double dt, xw1, vw;   // xw1: the piston at t + dt
    int wall, per;        // per: periodic axes (caller's), box [lo, hi)
    double lo[3], hi[3];
};
hipError_t launch_rk2_vjp_stage2(int64_t n, const Rk2Vjp &q, hipStream_t st);
hipError_t launch_rk2_vjp_stage1(int64_t n, const Rk2Vjp &q, double *const gp[8],
                                 hipStream_t st);
hipError_t launch_vjp_reflect(int64_t n, const int32_t *perm, const double *y_s,
                              const double *vy_s, const double *dvy_s, double dt, double yw1,
                              double vw, const double *gy, const double *gvy, const double *gE,
                              double *gy_out, double *gvy_out, hipStream_t st);
hipError_t launch_init_energy_vjp(const double *rho, const double *pres, const double *vx,
                                  const double *vy, const double *vz, const int32_t *mat,
                                  int64_t n, const EosDev &eos, const double *gE, double *g_vx,
                                  double *g_vy, double *g_vz, double *g_rho, double *g_eos,
                                  double *part, hipStream_t st);

// k_voronoi.hip
size_t balance_ws_bytes(int K);
hipError_t launch_balance_stats(const double *x, const double *y, const double *z, int64_t n,
                                const int32_t *owner, const int32_t *nbr_count,
                                const double *sites, int K, double dsh, int64_t *site_particles,
                                int64_t *site_pairs, double *centre, uint32_t *adj, void *ws,
                                hipStream_t st);
hipError_t launch_balance_move(const double *sites, int K, const int64_t *loads,
                               const double *centre, const uint32_t *adj, double sigma,
                               double theta, double gamma, double dsh, double *out,
                               double *move_sum, hipStream_t st);
hipError_t launch_voronoi(const double *x, const double *y, const double *z, int64_t n,
                          const double *sites, int K, const int32_t *nbr_count, int32_t *owner,
                          int64_t *site_particles, int64_t *site_pairs, hipStream_t st);

// k_neighbors.hip
hipError_t launch_gather_pos(int64_t n, const int32_t *perm, const double *x, const double *y,
                             const double *z, const double *d, const Ws &w, hipStream_t st);
hipError_t launch_nbr_count(int64_t n, const GridDev &g, const PairConst &pc, const double *x,
                            const double *y, const double *z, const double *d, const int32_t *cs,
                            const int32_t *perm, int32_t *count_orig, hipStream_t st);
hipError_t launch_nbr_fill(int64_t n, const GridDev &g, const PairConst &pc, const double *x,
                           const double *y, const double *z, const double *d, const int32_t *cs,
                           const int32_t *perm, const int64_t *offsets, int32_t *idx,
                           hipStream_t st);

}  // namespace csph
