// Pair records and the CSPH rate kernels (eqs. SPH:Conti, SPH:Pulse,
// SPH:Energy of sec. 4.1), FP64 and mixed (FP32 pair arithmetic).
//
// Particles are in cell order; each thread owns one particle i and gathers
// over the (2R+1)^3 stencil of cells around its own (and, with a piston
// wall, over the stencil around its mirror image).  Cells of one stencil
// row are contiguous in cell order, so a row is one index range.  Each
// particle sums its own partners (gather), so no floating-point atomics are
// used and results do not depend on scheduling.
#include "csph_internal.h"
#include "stencil.h"

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
// (e = E - |v|^2/2; ideal gas, stiffened gas or Mie-Grueneisen), pair record.
// Zero records after the n FP32 stencil records (cell-relative offsets, read by the candidate
// tests of both kernels): a walk loads up to kUS - 1 (kUS64 - 1) records past a row's last one
constexpr int kRecPad = 2;

template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_pack(int64_t n, SrcState src,
                                                 const int32_t *__restrict__ perm, EosDev eos,
                                                 GridDev g, void *__restrict__ recA,
                                                 void *__restrict__ recB,
                                                 void *__restrict__ recC, DstState dst,
                                                 int64_t *__restrict__ nonphys,
                                                 unsigned long long *__restrict__ zflag,
                                                 const int32_t *__restrict__ gate,
                                                 float4 *__restrict__ recF) {
    if (gate && *gate == 0) return;
    int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const int i = perm ? perm[s] : (int)s;  // no permutation: records of the state in place
    double v[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] = src.f[k][i];
    if (dst.f[0]) {
#pragma unroll
        for (int k = 0; k < 9; ++k) dst.f[k][s] = v[k];
    }
    int mt = src.mat ? src.mat[i] : 0;
    if (dst.mat) dst.mat[s] = mt;
    if (src.d && dst.d) dst.d[s] = src.d[i];
    if (src.id && dst.id) dst.id[s] = src.id[i];
    double x = v[0], y = v[1], z = v[2], vx = v[3], vy = v[4], vz = v[5], rho = v[6], E = v[7],
           m = v[8];
    int k = (mt >= 0 && mt < eos.n) ? mt : 0;
    double e = E - 0.5 * ((vx * vx + vy * vy) + vz * vz);
    double P, c2;
    eos_eval(eos, k, rho, e, P, c2);
    bool bad = !(c2 >= 0.0);
    double c = bad ? 0.0 : sqrt(c2);
    if (bad && nonphys) atomicAdd((unsigned long long *)nonphys, 1ull);
    double Z = rho * c, V = m / rho;
    // a zero impedance (in the precision the pairs use) needs the pair step's Z_i + Z_j = 0
    // branch; every writer stores the same value
    if ((MIXED ? (float)Z : Z) == 0.0 && zflag) *zflag = 0ull;
    if (MIXED && !perm) {  // list walks: FP64 position record
        ((double4 *)recA)[s] = make_double4(x, y, z, V);
        ((float4 *)recB)[s] = make_float4((float)vx, (float)vy, (float)vz, (float)P);
        ((float4 *)recC)[s] = make_float4((float)Z, (float)c, (float)V, 0.0f);
    } else {
        if (perm) {  // stencil walks: cell-relative FP32 offsets (the FP64 walk tests with them)
            int cx = cell_coord(x, g.ox, g.inv, g.dx);
            int cy = cell_coord(y, g.oy, g.inv, g.dy);
            int cz = cell_coord(z, g.oz, g.inv, g.dz);
            float ox = (float)(x - (g.ox + (double)cx * g.cell));
            float oy = (float)(y - (g.oy + (double)cy * g.cell));
            float oz = (float)(z - (g.oz + (double)cz * g.cell));
            // x offset, y, z offsets from the cell origin and the cell's x index
            float4 *F = MIXED ? (float4 *)recA : recF;
            F[s] = make_float4(ox, oy, oz, (float)cx);
            if (s == n - 1)
                for (int p = 1; p <= kRecPad; ++p) F[n - 1 + p] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        if (MIXED) {
            ((float4 *)recB)[s] = make_float4((float)vx, (float)vy, (float)vz, (float)P);
            ((float4 *)recC)[s] = make_float4((float)Z, (float)c, (float)V, 0.0f);
        } else {
            ((double4 *)recA)[s] = make_double4(x, y, z, V);
            ((double4 *)recB)[s] = make_double4(vx, vy, vz, P);
            ((double2 *)recC)[s] = make_double2(Z, c);
        }
    }
}

hipError_t launch_pack(const csph_state &s, int64_t n, const int32_t *perm, const EosDev &eos,
                       int mixed, const GridDev &g, const Ws &w, double *const dst[9],
                       int32_t *dst_mat, double *dst_d, int64_t *dst_id, const int64_t *src_id,
                       int64_t *nonphys, hipStream_t st, const int32_t *gate) {
    if (n <= 0) return hipSuccess;
    SrcState src{{s.x, s.y, s.z, s.vx, s.vy, s.vz, s.rho, s.E, s.m}, s.mat, s.d, src_id};
    DstState ds;
    for (int k = 0; k < 9; ++k) ds.f[k] = dst ? dst[k] : nullptr;
    ds.mat = dst_mat;
    ds.d = dst_d;
    ds.id = dst_id;
    // perm = NULL: records of the state as it is (Verlet steps); the A record then holds
    // the FP64 position in both precisions
    void *recA = w.recA;
    unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    if (mixed)
        k_pack<true><<<nb, kBlock, 0, st>>>(n, src, perm, eos, g, recA, w.recB, w.recC, ds,
                                            nonphys, w.zflag, gate, nullptr);
    else
        k_pack<false><<<nb, kBlock, 0, st>>>(n, src, perm, eos, g, recA, w.recB, w.recC, ds,
                                             nonphys, w.zflag, gate, (float4 *)w.recF);
    return hipGetLastError();
}

// ---------------------------------------------------------------- wave min -> global

// The FP32 rate kernel runs one wave per workgroup: its occupancy is bound by the LDS rings,
// and a wave's ring is released as soon as the wave ends (partner counts, hence wave run
// times, vary widely; a larger workgroup holds its rings until its slowest wave ends).  The
// FP64 kernel's occupancy is bound by registers; it keeps four-wave workgroups.
constexpr int kRate32Block = 64;
constexpr int kSlot = kRate32Block * (int)sizeof(float4);  // bytes per ring row
constexpr int kRing = kQ * kSlot;                        // bytes per wave's rings
constexpr int kRate64Block = kBlock;
constexpr int kSlot64 = kRate64Block * (int)sizeof(int);  // FP64 kernel: bytes per ring row
// most workgroups per die chunk (xcd_block_upto; measured on the porous shock's 100 steps,
// where the wall band's costly waves made one die the last to finish): ~131 k / ~65 k
// particles, fewer in launches too small for four rounds of such chunks.  The
// FP32 kernel's 2 048-wave chunks read 1.86 GB per launch beyond L2 (512: 2.31 GB, 1 024:
// 2.01 GB) in the same time; 4 096 leaves an eighth of the waves outside the whole rounds of
// chunks, unmapped, and reads 4.1 GB.  The FP64 kernel's 256 four-wave groups read 3.51 GB
// (64: 4.73 GB, 512: 3.22 GB), again in the same time.
constexpr unsigned kRate32Chunk = 2048;
constexpr unsigned kRate64Chunk = 256;

// min over the wave of v >= 0 into *dst (bits of a non-negative double); the atomic is
// skipped when it cannot lower the current value
__device__ __forceinline__ void wave_min_to(double v, unsigned long long *dst) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0 && v >= 0.0) {
        const unsigned long long b = dbits(v);
        if (b < __atomic_load_n(dst, __ATOMIC_RELAXED)) atomicMin(dst, b);
    }
}

// Verlet lists (sec. 4.2): entry k of particle s at idx[((k/8) n + s) 8 + k%8],
// k < count[s]; a mirror partner has the sign bit set.  Absent (idx = NULL) for
// stencil walks.  The list walks read two entries per 8-byte load.
static_assert(kU == 2, "list walks load kU = 2 entries at once");
constexpr int kUS = 3;  // candidates per lock-step iteration of the FP32 stencil walk (measured)
static_assert(kUS - 1 <= kRecPad, "the stencil walk reads up to kUS - 1 records past a row");
struct VList {
    const int32_t *count;
    const int32_t *idx;
    int cap;
    const int32_t *gate;  // list steps: nothing to do while *gate == 0
};

struct RateOut {
    double *rho, *vx, *vy, *vz, *E, *sig;
    int32_t *cnt;
    unsigned long long *dtmin;
    const unsigned long long *zflag;  // 0: some impedance is zero (see k_pack)
};

// Candidates whose FP32 squared distance lies within this relative band of
// the squared support are decided in FP64 from the FP64 positions (the mixed
// kernel re-tests them at the pop; the FP64 kernel queues them and decides
// every pop in FP64), so both accept exactly the FP64 neighbour set (the FP32
// error of r^2 is below 1e-6 relative for offsets within a few cells).
constexpr float kBand = 4e-5f;

// ---------------------------------------------------------------- FP64 rates
//
// The pair step is written without branches: a lane with no partner to
// evaluate (empty ring, coincident partner) runs the same instructions on
// placeholder data and keeps its sums by selection.  Divergent branches in
// the drain made the compiler shuffle the live sums between registers on
// every pop.

// 1/sqrt(x) and 1/x for x > 0 in FP64: the hardware estimate (v_rsq_f64, v_rcp_f64) refined
// by two Newton steps.  For 1/sqrt(x) the step is y <- y + (y/2)(1 - x y^2), for 1/x it is
// y <- y + y (1 - x y); each squares the relative error (up to a factor 3/2 for 1/sqrt), so
// two steps take the estimate to the last bits of FP64 (the result is within a few ulp, not
// correctly rounded: the rates are compared with a 1e-12 tolerance).  They replace the
// compiler's correctly rounded FP64 square root and divisions, which take several times the
// instructions.
__device__ __forceinline__ double rsqrt64(double x) {
#pragma clang fp contract(fast)
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double e = fma(-x * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

__device__ __forceinline__ double rcp64(double x) {
#pragma clang fp contract(fast)
    double y = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double e = fma(-x, y, 1.0);
        y = fma(y, e, y);
    }
    return y;
}

// One partner of particle i: Riemann problem along e, kernel slope, sums.
// The membership test that precedes it is exact; here contraction is allowed.
// ZS: some impedance may be zero, so Z_i + Z_j = 0 takes the mean state; otherwise that
// branch is left out.  As in the FP32 step, 1/(Z_i + Z_j) is folded into the weight, e is
// taken as the raw offsets times 1/r, and the energy flux sum_j f v* is accumulated as
// -sum_j f (v_L - v*): its sum_j f v_L part is v_i . sum_j f e_ij, added once from the
// momentum sums.
template <bool ZS>
__device__ __forceinline__ void pair64(bool use, double dx, double dy, double dz, double r2,
                                       const double4 &bi, const double2 &ci,
                                       double vxj, double vyj, double vzj, double Pj, double Zj,
                                       double cj, double Vj, double invH, double dwc,
                                       double &ar, double &avx, double &avy, double &avz,
                                       double &aE, double &sig) {
#pragma clang fp contract(fast)
    const double ir = rsqrt64(use ? r2 : 1.0);
    const double r = r2 * ir;
    const double q = r * invH;
    const double a1 = 1.0 - q;
    // a lane without a partner adds exact zeros: its kernel constant is selected to 0 and
    // every factor it multiplies is finite (placeholder offsets and r2 finite)
    const double dW = -(use ? dwc : 0.0) * q * (a1 * a1 * a1);
    // v_L - v_R from the velocity difference and the raw offsets
    const double vrel = (((bi.x - vxj) * dx + (bi.y - vyj) * dy) + (bi.z - vzj) * dz) * ir;
    const double Zi = ci.x, Pi = bi.w;
    const double S = Zi + Zj;
    // (v_L - v*) S and P* S; S = 0 takes the mean state, written as the same expressions
    // with Z_i = Z_j = 1 and the P and (v_L - v_R) terms dropped
    const bool sok = !ZS || S != 0.0;
    const double iS = rcp64(sok ? S : 2.0);
    const double Zjd = sok ? Zj : 1.0, Zid = sok ? Zi : 1.0;
    const double dP = sok ? Pi - Pj : 0.0, ZZ = sok ? Zi * Zj : 0.0;
    const double dvlS = Zjd * vrel - dP;
    const double psS = (Zjd * Pi + Zid * Pj) + ZZ * vrel;
    const double wS = (Vj * iS) * dW;  // V_j W' / S
    const double f = wS * psS;         // V_j W' P*
    const double fr = f * ir;
    const double sp = fmax(ci.y, cj) + (vrel > 0.0 ? vrel : 0.0);
    ar += wS * dvlS;
    avx += fr * dx;
    avy += fr * dy;
    avz += fr * dz;
    aE -= f * (dvlS * iS);
    sig = (use && sp > sig) ? sp : sig;
}

// FP64 stencil walk: candidates per lock-step iteration, pops per drain trigger (as in the
// FP32 kernel: the loop's copies of the live sums are paid once per two pops)
constexpr int kUS64 = 3;
constexpr int kPop64 = 2;
static_assert(kUS64 - 1 <= kRecPad, "the FP64 stencil walk reads up to kUS64 - 1 FP32 records past a row");

template <bool PAIR, bool WALL, bool PER>
struct Rates64 {
    const double4 *__restrict__ A;
    const double4 *__restrict__ B;
    const double2 *__restrict__ Cz;
    const float4 *__restrict__ F;  // stencil walks: cell-relative FP32 records (the test)
    const double *__restrict__ dsz;
    const int32_t *__restrict__ cs;
    GridDev g;
    PairConst pc;
    char *qb;         // the workgroup's rings: kQ rows of kRate64Block 4-byte slots
    int lane4;        // the lane's byte offset in a ring row
    uint32_t self32;  // byte offset of i's own 32-byte records
    bool live, near_wall;
    double4 a, b;
    double2 zc;
    double di, yw, vw2;  // wall position along y, twice its velocity
    Stencil t, ti;       // stencils of i and of its mirror image
    // the candidate test in FP32 from cell-relative records, as in the mixed kernel: i's
    // record (offsets and its cell's x index), D, the support bound (squared, with the band)
    // and the wall's distance
    float4 a32;
    float Df, hi32, wd;
    // periodic images: i's faces (image_faces), the image the walk is on (wave-uniform mask),
    // its stencil, i's FP32 offsets from the image point's cell origin and that cell's x index
    int nf = 0, im = 0;
    Stencil tm;
    float amx = 0.f, amy = 0.f, amz = 0.f, cxm = 0.f;
    double ar = 0.0, avx = 0.0, avy = 0.0, avz = 0.0, aE = 0.0, sig = 0.0;
    // ring counters in entries; an entry is the partner's 32-byte record offset, bit 0 set for
    // a mirror image, bits 1-3 the periodic image mask.  cnt: the exact members popped, |N(i)|
    int qw = 0, qr = 0, cnt = 0;

    __device__ __forceinline__ uint32_t &slot(int q) {
        return *(uint32_t *)(qb + (((q & (kQ - 1)) * kSlot64) | lane4));
    }

    // every lane pops its next partner, if it has one; MIR: the wave may hold mirror entries
    template <bool MIR, bool ZS>
    __device__ __forceinline__ void drain() {
        const bool has = qr < qw;
        const uint32_t e = slot(qr);
        qr += has ? 1 : 0;
        const uint32_t jo = has ? (MIR ? e & ~31u : e) : 0u;
        const bool ghost = MIR && (e & 1u);
        const int mm = PER && MIR ? (int)((e >> 1) & 7u) : 0;
        const int j = (int)(jo >> 5);
        const double4 aj = *(const double4 *)((const char *)A + jo);
        const double4 bj = *(const double4 *)((const char *)B + jo);
        const double2 zj = *(const double2 *)((const char *)Cz + (jo >> 1));
        const double yj = ghost ? 2.0 * yw - aj.y : aj.y;
        double dx = aj.x - a.x, dy = yj - a.y, dz = aj.z - a.z;
        if (PER) {  // image mm: d = (x_j - x_i) - k L
            dx = dx - image_shift(pc, nf, mm, 0);
            dy = dy - image_shift(pc, nf, mm, 1);
            dz = dz - image_shift(pc, nf, mm, 2);
        }
        // exact FP64 membership (the walk queued every candidate within the FP32 band of the
        // support), no contraction
        const double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
        double invH = pc.invH, dwc = pc.dwc, H2 = pc.H2;
        if (PAIR) {
            const double H = pc.kappa * (0.5 * (di + dsz[j]));
            H2 = H * H;
            invH = rcp64(H > 0.0 ? H : 1.0);
            const double i2 = invH * invH;
            dwc = (210.0 / M_PI) * (i2 * i2);
        }
        const bool in = has && r2 < H2;
        cnt += (in && !ghost) ? 1 : 0;
        pair64<ZS>(in && r2 != 0.0, dx, dy, dz, r2, b, zc, bj.x, ghost ? vw2 - bj.y : bj.y, bj.z,
               bj.w, zj.x, zj.y, aj.w, invH, dwc, ar, avx, avy, avz, aE, sig);
    }

    // one walk over the stencil: real partners, or mirror partners (GHOST); IMG: the walk
    // around periodic image im of i (or of its mirror image).  The candidates are tested in
    // FP32 from the cell-relative records, as in the mixed kernel, and every one within the
    // band of the support is queued: the pop decides membership exactly, in FP64.
    // One flat loop with wave-uniform branches (drain / next row / test a
    // chunk).
    template <bool GHOST, bool MIR, bool ZS, bool IMG>
    __device__ __forceinline__ void pass() {
#pragma clang fp contract(fast)
        const bool on = live && (!GHOST || near_wall) && (!IMG || (nf & im) == im);
        // mirror partners: the particles on the stencil around the image of i
        const Stencil &st = IMG ? tm : GHOST ? ti : t;
        const float ax0 = IMG ? amx : a32.x, az0 = IMG ? amz : a32.z, cx0 = IMG ? cxm : a32.w;
        const float ay0 = IMG && !GHOST ? amy : a32.y;
        const int cy0 = IMG && !GHOST ? tm.cy : t.cy;
        const uint32_t tag = (GHOST ? 1u : 0u) | (IMG ? (uint32_t)im << 1 : 0u);
        int oy = st.R, oz = -st.R - 1;  // advanced to (-R, -R) before the first row
        int k = 0, j0 = 0, len = 0, jlast = 0;
        float ay = 0.f, az = 0.f, gz2 = 0.f;
        for (;;) {
            if (__any(qw - qr > kQ - kUS64)) {  // keep every ring at <= kQ - kUS64 entries
#pragma unroll
                for (int p = 0; p < kPop64; ++p) drain<MIR, ZS>();
                continue;
            }
            if (!__any(k < len)) {
                if (++oy > st.R) {
                    oy = -st.R;
                    if (++oz > st.R) break;
                    const float gz = slab_gap(st.zc, st.cz + oz);  // per plane of rows
                    gz2 = gz * gz;
                    az = az0 - (float)oz * Df;
                }
                const int yy = st.cy + oy, zz = st.cz + oz;
                row_range(cs, g, st, on, yy, zz, gz2, j0, len);
                jlast = len > 0 ? j0 + len - 1 : 0;
                ay = ay0 - (float)(yy - cy0) * Df;
                k = 0;
                continue;
            }
            // the slots' records from j0 + k on, the start clamped to the row's last record
            // (the pack appends kUS64 - 1 zero records after the n records)
            const uint32_t jb = (uint32_t)min(j0 + k, jlast);
            const float4 *Fb = (const float4 *)((const char *)F + jb * (uint32_t)sizeof(float4));
            float4 aj[kUS64];
#pragma unroll
            for (int u = 0; u < kUS64; ++u) aj[u] = Fb[u];
#pragma unroll
            for (int u = 0; u < kUS64; ++u) {
                const int j = j0 + k + u;
                float dx = (aj[u].x + (aj[u].w - cx0) * Df) - ax0;
                float dy = aj[u].y - ay, dz = aj[u].z - az;
                if (GHOST) dy = 2.0f * wd - dy;
                const float r2 = (dx * dx + dy * dy) + dz * dz;
                float hj = hi32;
                if (PAIR) {
                    const double H = pc.kappa * (0.5 * (di + ld(dsz, j < jlast ? j : jlast)));
                    hj = (float)(H * H) * (1.0f + kBand);
                }
                // the entry's FP64 record offset (32 j for a slot that can be accepted)
                const uint32_t jo = (jb + (uint32_t)u) * (uint32_t)sizeof(double4);
                const bool acc = (k + u < len) & (GHOST || IMG || jo != self32) & (r2 < hj);
                // the ring slot qw is free: write always, advance on acceptance
                slot(qw) = jo | tag;
                qw += acc ? 1 : 0;
            }
            k += kUS64;
        }
    }

    // the walks around every periodic image some lane of the wave has (GHOST: around the
    // images of its mirror image)
    template <bool GHOST, bool ZS>
    __device__ __forceinline__ void images() {
        for (int m = 1; m < 8; ++m) {
            if (!__any(live && (!GHOST || near_wall) && (nf & m) == m)) continue;
            im = m;
            const double px = a.x + image_shift(pc, nf, m, 0);
            const double py = (GHOST ? 2.0 * yw - a.y : a.y) + image_shift(pc, nf, m, 1);
            const double pz = a.z + image_shift(pc, nf, m, 2);
            tm = shifted_stencil(g, GHOST ? ti : t, m, px, py, pz);
            amx = m & 1 ? (float)(px - (g.ox + (double)tm.cx * g.cell)) : a32.x;
            amy = m & 2 ? (float)(py - (g.oy + (double)tm.cy * g.cell)) : a32.y;
            amz = m & 4 ? (float)(pz - (g.oz + (double)tm.cz * g.cell)) : a32.z;
            cxm = (float)tm.cx;
            pass<GHOST, true, ZS, true>();
        }
    }

    // The whole walk: a Verlet list, or the stencil (and, for a wave with particles in the
    // wall band, the stencil around their images; for a wave with particles near periodic
    // faces, the stencils around their periodic images); every pop drained.  Returns |N(i)|.
    template <bool LIST, bool ZS>
    __device__ __forceinline__ int run(const int32_t *__restrict__ lst, int len, int64_t nl) {
        const bool anyw = WALL && __any(near_wall);
        if (LIST) {
            pass_list<ZS>(lst, len, nl);
            while (__any(qr < qw)) drain<WALL, ZS>();
        } else if (anyw || (PER && __any(nf != 0))) {
            pass<false, true, ZS, false>();
            if (PER) images<false, ZS>();
            if (anyw) {
                pass<true, true, ZS, false>();
                if (PER) images<true, ZS>();
            }
            while (__any(qr < qw)) drain<true, ZS>();
        } else {
            pass<false, false, ZS, false>();
            while (__any(qr < qw)) drain<false, ZS>();
        }
        return cnt;  // real partners (periodic images included), counted at the pops
    }

    // Verlet-list walk: the lane's own list in chunks of kU, exact FP64 membership
    // (mirror partners across the wall for flagged entries)
    template <bool ZS>
    __device__ __forceinline__ void pass_list(const int32_t *__restrict__ lst, int len,
                                              int64_t nl) {
        int k = 0;
        for (;;) {
            if (__any(qw - qr > kQ - kU)) {
                drain<WALL, ZS>();
                continue;
            }
            if (!__any(k < len)) break;
            const int2 ee = *(const int2 *)(lst + (int64_t)(k / kVlChunk) * nl * kVlChunk +
                                            (k % kVlChunk));
            int e[kU] = {k < len ? ee.x : 0, k + 1 < len ? ee.y : 0};
            double4 aj[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) aj[u] = ld(A, e[u] & 0x7fffffff);
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const bool ghost = WALL && e[u] < 0;
                const double yj = ghost ? 2.0 * yw - aj[u].y : aj[u].y;
                const double dx = aj[u].x - a.x, dy = yj - a.y, dz = aj[u].z - a.z;
                const double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
                const bool acc = (k + u < len) && r2 < pc.H2;
                // list entries carry the mirror flag in the sign bit
                const uint32_t eu = (uint32_t)e[u];
                slot(qw) = WALL ? (eu << 5) | (eu >> 31) : eu << 5;
                qw += acc ? 1 : 0;
            }
            k += kU;
        }
    }
};

// Occupancy hint of 4 waves per SIMD (up to 128 VGPRs): with the FP32 candidate test the
// kernel would spill at the 96 VGPRs of 5 waves (measured 9.22 against 7.72 ms on the porous
// shock's first 20 steps).
template <bool PAIR, bool WALL, bool LIST, bool PER>
__global__ __launch_bounds__(kRate64Block, 4) void k_rates64(int64_t n, const double4 *__restrict__ A,
                                                    const double4 *__restrict__ B,
                                                    const double2 *__restrict__ Cz,
                                                    const float4 *__restrict__ F,
                                                    const double *__restrict__ rho,
                                                    const double *__restrict__ dsz,
                                                    const int32_t *__restrict__ cs, GridDev g,
                                                    PairConst pc, const double *t_dev,
                                                    double t_host, RateOut o, int want_dt,
                                                    VList vl) {
    if (LIST && vl.gate && *vl.gate == 0) return;
    __shared__ int qj[kQ][kRate64Block];
    Rates64<PAIR, WALL, PER> k;
    k.qb = (char *)&qj[0][0];
    k.lane4 = threadIdx.x * (int)sizeof(int);
    k.A = A;
    k.B = B;
    k.Cz = Cz;
    k.F = F;
    k.dsz = dsz;
    k.cs = cs;
    k.g = g;
    k.pc = pc;
    const int64_t s =
        xcd_block_upto(blockIdx.x, gridDim.x, kRate64Chunk) * kRate64Block + threadIdx.x;
    k.self32 = (uint32_t)s * (uint32_t)sizeof(double4);
    k.live = s < n;
    k.a = make_double4(0.0, 0.0, 0.0, 0.0);
    k.b = k.a;
    k.zc = make_double2(0.0, 0.0);
    k.a32 = make_float4(0.f, 0.f, 0.f, 0.f);
    k.di = 0.0;
    if (k.live) {
        k.a = A[s];
        k.b = B[s];
        k.zc = Cz[s];
        if (!LIST) k.a32 = F[s];
        if (PAIR) k.di = dsz[s];
    }
    k.t = make_stencil(g, k.a.x, k.a.y, k.a.z, pc.H);
    k.ti = k.t;
    k.sig = k.zc.y;
    k.Df = (float)g.cell;
    k.hi32 = (float)pc.H2 * (1.0f + kBand);
    k.yw = 0.0;
    k.vw2 = 0.0;
    k.wd = 0.f;
    k.near_wall = false;
    if (WALL) {
        double tt = t_dev ? *t_dev : t_host;
        k.yw = pc.wall_y0 + pc.wall_v * tt;
        k.vw2 = 2.0 * pc.wall_v;
        k.near_wall = k.live && mirror_band(g, k.a.y, k.yw, pc.H);
        k.wd = (float)(k.yw - k.a.y);
        k.ti = image_stencil(g, k.t, 2.0 * k.yw - k.a.y);
    }
    k.tm = k.t;
    if (PER && k.live) k.nf = image_faces(pc, k.a.x, k.a.y, k.a.z);
    const int len = LIST && k.live ? min(vl.count[s], vl.cap) : 0;
    const int32_t *lst = LIST ? vl.idx + (k.live ? s * kVlChunk : 0) : nullptr;
    const int cnt = *o.zflag == 0 ? k.template run<LIST, true>(lst, len, n)
                                  : k.template run<LIST, false>(lst, len, n);
    double dtv = INFINITY;
    if (k.live) {
        double ri = rho[s];
        double pre = 2.0 / ri;
        double drho = -2.0 * ri * k.ar;
        o.rho[s] = drho;
        o.vx[s] = pre * k.avx;
        o.vy[s] = pre * k.avy;
        o.vz[s] = pre * k.avz;
        // sum_j f v* = v_i . sum_j f e_ij - sum_j f (v_L - v*)
        const double vf = (k.b.x * k.avx + k.b.y * k.avy) + k.b.z * k.avz;
        o.E[s] = pre * (k.aE + vf);
        if (o.sig) o.sig[s] = k.sig;
        if (o.cnt) o.cnt[s] = cnt;
        // Courant limit and relative density-change limit of one explicit step
        dtv = fmin((PAIR ? k.di : pc.h_dt) / k.sig, ri / fabs(drho));
    }
    if (want_dt) wave_min_to(dtv, o.dtmin);
}

// ---------------------------------------------------------------- mixed rates (FP32 pairs)

// max of two non-negative floats (sound and signal speeds): their bit patterns order like
// the values, so an integer max is exact, in one instruction (fmaxf quiets both inputs first)
__device__ __forceinline__ float fmax_nonneg(float a, float b) {
    return __int_as_float(max(__float_as_int(a), __float_as_int(b)));
}

template <bool ZS>
__device__ __forceinline__ void pair32(bool use, float dx, float dy, float dz, float r2,
                                       const float4 &bi, const float4 &ci, float vxj, float vyj,
                                       float vzj, float Pj, float Zj, float cj, float Vj,
                                       float invH, float dwch, float &ar, float &avx, float &avy,
                                       float &avz, float &aE, float &sig) {
#pragma clang fp contract(fast)
    // dwch = (210/pi)/H^5, so that dW/dr = -dwch r (1 - r/H)^3
    const float ir = __builtin_amdgcn_rsqf(use ? r2 : 1.0f);
    const float r = r2 * ir;
    const float a1 = 1.0f - r * invH;
    const float dWr = -(use ? dwch : 0.0f) * r * (a1 * a1 * a1);
    // v_L - v_R from the velocity difference and the raw offsets (no cancellation of bulk
    // motion); e = (dx, dy, dz) / r
    const float vrel = (((bi.x - vxj) * dx + (bi.y - vyj) * dy) + (bi.z - vzj) * dz) * ir;
    const float Zi = ci.x, Pi = bi.w;
    const float S = Zi + Zj;
    // (v_L - v*) S and P* S; S = 0 (both impedances zero) takes the mean state, written as
    // the same expressions with Z_i = Z_j = 1 and the P and (v_L - v_R) terms dropped
    const bool sok = !ZS || S != 0.0f;
    const float iS = __builtin_amdgcn_rcpf(sok ? S : 2.0f);
    const float Zjd = sok ? Zj : 1.0f, Zid = sok ? Zi : 1.0f;
    const float dP = sok ? Pi - Pj : 0.0f, ZZ = sok ? Zi * Zj : 0.0f;
    const float dvlS = Zjd * vrel - dP;
    const float psS = (Zjd * Pi + Zid * Pj) + ZZ * vrel;
    // a lane without a partner adds exact zeros: its weight is 0 (the kernel constant selected
    // to 0) and every factor it multiplies is finite (r2 = 1, finite offsets)
    const float wS = (Vj * iS) * dWr;  // V_j dW/dr / S
    const float f = wS * psS;          // V_j dW/dr P*
    const float fr = f * ir;
    const float sp = fmax_nonneg(ci.y, cj) + fmaxf(vrel, 0.0f);
    ar += wS * dvlS;
    avx += fr * dx;
    avy += fr * dy;
    avz += fr * dz;
    // energy flux f v* = f v_L - f (v_L - v*); the f v_L part sums to v_i . sum_j f e_ij, which
    // the kernel adds once from the momentum sums
    aE -= f * (dvlS * iS);
    sig = fmax_nonneg(sig, use ? sp : 0.0f);
}


// The exact FP64 membership test of a pair from its FP64 offsets, rounded as written (a
// product, a product, a sum, a product, a sum): this function lies outside the
// fast-contraction scope of the FP32 pair step, so none of it becomes a fused multiply-add
// when it is inlined there.
__device__ __forceinline__ bool member64(double ex, double ey, double ez, double H2) {
    return ((ex * ex) + (ey * ey)) + (ez * ez) < H2;
}

template <bool PAIR, bool WALL, bool LIST, bool PER>
struct Rates32 {
    const float4 *__restrict__ A;
    const float4 *__restrict__ B;
    const float4 *__restrict__ Cz;
    const double *__restrict__ xs;
    const double *__restrict__ ys;
    const double *__restrict__ zs;
    const double *__restrict__ dsz;
    const int32_t *__restrict__ cs;
    const double4 *__restrict__ P4;  // list walks: FP64 position record
    GridDev g;
    PairConst pc;
    char *qb;         // the wave's rings: kQ rows of kRate32Block float4 slots
    int lane16;       // the lane's byte offset in a ring row
    uint32_t self16;  // byte offset of i's own records
    bool live, near_wall;
    float4 a, b, c;
    double xi, yi, zi, di, yw;  // yw: wall position along y
    float wd, vw2, Df, cxf, lo, hi, dwch0;
    Stencil t, ti;               // stencils of i and of its mirror image
    // periodic images: i's faces (image_faces); the image the walk is on (wave-uniform mask),
    // its stencil, i's offsets from the image point's cell origin and that cell's x index
    int nf = 0, im = 0;
    Stencil tm;
    float amx = 0.f, amy = 0.f, amz = 0.f, cxm = 0.f;
    float ar = 0.f, avx = 0.f, avy = 0.f, avz = 0.f, aE = 0.f, sig = 0.f;
    // ring write and read counters in bytes, advancing one ring row (kSlot) per entry: a
    // slot's address is the counter masked to the ring, or'ed with the lane's offset;
    // unsigned, so that the fill level qw - qr stays exact if the counters wrap
    unsigned qw = 0, qr = 0;
    int cnt = 0;

    __device__ __forceinline__ float4 &slot(unsigned q) {
        return *(float4 *)(qb + ((q & (kRing - 1)) | (unsigned)lane16));
    }
    // A ring entry holds the partner's offsets and, in w, the byte offset of its 16-byte
    // records with bit 0 set for a mirror image and bits 1-3 holding the periodic image mask.

    // every lane pops its next partner, if it has one; MIR: the wave may hold mirror entries
    template <bool MIR, bool ZS>
    __device__ __forceinline__ void drain() {
#pragma clang fp contract(fast)
        const bool has = qr != qw;
        const float4 q = slot(qr);
        qr += has ? kSlot : 0;
        const uint32_t e = __float_as_uint(q.w);
        const uint32_t jo = has ? (MIR ? e & ~15u : e) : 0u;
        const bool ghost = MIR && (e & 1u);
        const int mm = PER && MIR ? (int)((e >> 1) & 7u) : 0;
        const int j = (int)(jo >> 4);
        const float4 bj = *(const float4 *)((const char *)B + jo);
        const float4 cj = *(const float4 *)((const char *)Cz + jo);
        float invH = (float)pc.invH, dwch = dwch0;
        float H2lo = lo;
        double H2d = pc.H2;
        if (PAIR) {
            const double H = pc.kappa * (0.5 * (di + dsz[j]));
            H2d = H * H;
            H2lo = (float)H2d * (1.0f - kBand);
            invH = (float)(1.0 / H);
            const float i2 = invH * invH;
            dwch = (float)(210.0 / M_PI) * (i2 * i2) * invH;
        }
        float qx = q.x, qy = q.y, qz = q.z;
        float r2 = (qx * qx + qy * qy) + qz * qz;
        // a list walk queues exact FP64 members only, with offsets rounded from FP64
        bool in = has && (LIST || r2 < H2lo);
        // (rare) near the support, decide membership in FP64; nearly coincident (r < H/100),
        // take the offsets from FP64 too: the cell-relative FP32 offsets carry ~1e-7 absolute
        // error, which would bend the direction e of so short a pair (and with it the
        // closing speed in the signal speed, which the kernel weight does not damp)
        if (!LIST && has && (!(r2 < H2lo) || r2 < H2lo * 1e-4f)) {
            const double yj = ghost ? 2.0 * yw - ys[j] : ys[j];
            double ex = xs[j] - xi, ey = yj - yi, ez = zs[j] - zi;
            if (PER) {  // image mm: d = (x_j - x_i) - k L
                ex = ex - image_shift(pc, nf, mm, 0);
                ey = ey - image_shift(pc, nf, mm, 1);
                ez = ez - image_shift(pc, nf, mm, 2);
            }
            in = member64(ex, ey, ez, H2d);
            qx = (float)ex;
            qy = (float)ey;
            qz = (float)ez;
            r2 = (qx * qx + qy * qy) + qz * qz;
        }
        cnt += (in && !ghost) ? 1 : 0;
        pair32<ZS>(in && r2 != 0.0f, qx, qy, qz, r2, b, c, bj.x, ghost ? vw2 - bj.y : bj.y,
                   bj.z, bj.w, cj.x, cj.y, cj.z, invH, dwch, ar, avx, avy, avz, aE, sig);
    }

    // flat loop as in the FP64 kernel.  IMG: the walk around image point im of i (or of its
    // mirror image), offsets relative to that point's cells; the wall axis y is never periodic,
    // so a mirror walk keeps i's own y offsets.
    template <bool GHOST, bool MIR, bool ZS, bool IMG>
    __device__ __forceinline__ void pass() {
#pragma clang fp contract(fast)
        const bool on = live && (!GHOST || near_wall) && (!IMG || (nf & im) == im);
        // mirror partners: the particles on the stencil around the image of i
        const Stencil &st = IMG ? tm : GHOST ? ti : t;
        const float ax0 = IMG ? amx : a.x, az0 = IMG ? amz : a.z, cx0 = IMG ? cxm : cxf;
        const float ay0 = IMG && !GHOST ? amy : a.y;
        const int cy0 = IMG && !GHOST ? tm.cy : t.cy;
        const uint32_t tag = (GHOST ? 1u : 0u) | (IMG ? (uint32_t)im << 1 : 0u);
        int oy = st.R, oz = -st.R - 1;
        int k = 0, j0 = 0, len = 0, jlast = 0;
        float ay = 0.f, az = 0.f, gz2 = 0.f;
        for (;;) {
            // two pops per trigger: some lane holds kQ - 1 entries, most lanes hold several,
            // and the loop's copies of the live sums are paid once per two pops
            if (__any(qw - qr > (kQ - kUS) * kSlot)) {
                drain<MIR, ZS>();
                drain<MIR, ZS>();
                continue;
            }
            if (!__any(k < len)) {
                if (++oy > st.R) {
                    oy = -st.R;
                    if (++oz > st.R) break;
                    // per plane of rows: squared z gap, i's z offset from the plane's cells
                    const float gz = slab_gap(st.zc, st.cz + oz);
                    gz2 = gz * gz;
                    az = az0 - (float)oz * Df;
                }
                const int yy = st.cy + oy, zz = st.cz + oz;
                row_range(cs, g, st, on, yy, zz, gz2, j0, len);
                jlast = len > 0 ? j0 + len - 1 : 0;
                // i's y offset from the row's cell origin (rows counted from i's own cell)
                ay = ay0 - (float)(yy - cy0) * Df;
                k = 0;
                continue;
            }
            // the slots' records from j0 + k on, the start clamped to the row's last record:
            // every load then reads a finite record (a lane with nothing left to pop reads the
            // slot written last), up to kUS - 1 past the row, which the zero records the pack
            // appends after the n records keep in bounds
            const uint32_t jbo = (uint32_t)min(j0 + k, jlast) * (uint32_t)sizeof(float4);
            const float4 *Ab = (const float4 *)((const char *)A + jbo);
            float4 aj[kUS];
#pragma unroll
            for (int u = 0; u < kUS; ++u) aj[u] = Ab[u];
#pragma unroll
            for (int u = 0; u < kUS; ++u) {
                const int j = j0 + k + u;
                float dx = (aj[u].x + (aj[u].w - cx0) * Df) - ax0;
                float dy = aj[u].y - ay, dz = aj[u].z - az;
                if (GHOST) dy = 2.0f * wd - dy;
                float r2 = (dx * dx + dy * dy) + dz * dz;
                float hj = hi;
                if (PAIR) {
                    double H = pc.kappa * (0.5 * (di + ld(dsz, j < jlast ? j : jlast)));
                    hj = (float)(H * H) * (1.0f + kBand);
                }
                // the entry's record offset (16 j for a slot that can be accepted); one select
                // per slot: the three tests combine as lane masks
                const uint32_t jo = jbo + (uint32_t)(u * sizeof(float4));
                const bool acc = (k + u < len) & (GHOST || IMG || jo != self16) & (r2 < hj);
                slot(qw) = make_float4(dx, dy, dz, __uint_as_float(jo | tag));
                qw += acc ? kSlot : 0;
            }
            k += kUS;
        }
    }

    // Point of image m of i (GHOST: of its mirror image) and its stencil and offsets.
    template <bool GHOST>
    __device__ __forceinline__ void set_image(int m) {
        im = m;
        const double px = xi + image_shift(pc, nf, m, 0);
        const double py = (GHOST ? 2.0 * yw - yi : yi) + image_shift(pc, nf, m, 1);
        const double pz = zi + image_shift(pc, nf, m, 2);
        tm = shifted_stencil(g, GHOST ? ti : t, m, px, py, pz);
        amx = m & 1 ? (float)(px - (g.ox + (double)tm.cx * g.cell)) : a.x;
        amy = m & 2 ? (float)(py - (g.oy + (double)tm.cy * g.cell)) : a.y;
        amz = m & 4 ? (float)(pz - (g.oz + (double)tm.cz * g.cell)) : a.z;
        cxm = (float)tm.cx;
    }

    // the walks around every periodic image some lane of the wave has
    template <bool GHOST, bool ZS>
    __device__ __forceinline__ void images() {
        for (int m = 1; m < 8; ++m) {
            if (!__any(live && (!GHOST || near_wall) && (nf & m) == m)) continue;
            set_image<GHOST>(m);
            pass<GHOST, true, ZS, true>();
        }
    }

    // The whole walk: a Verlet list, or the stencil (and, for a wave with particles in the
    // wall band, the stencil around their images; for a wave with particles near periodic
    // faces, the stencils around their periodic images); every pop drained.
    template <bool LIST_, bool ZS>
    __device__ __forceinline__ void run(const int32_t *__restrict__ lst, int len, int64_t nl) {
        const bool anyw = WALL && __any(near_wall);
        if (LIST_) {
            pass_list<ZS>(lst, len, nl);
            while (__any(qr != qw)) drain<WALL, ZS>();
        } else if (anyw || (PER && __any(nf != 0))) {
            pass<false, true, ZS, false>();
            if (PER) images<false, ZS>();
            if (anyw) {
                pass<true, true, ZS, false>();
                if (PER) images<true, ZS>();
            }
            while (__any(qr != qw)) drain<true, ZS>();
        } else {
            pass<false, false, ZS, false>();
            while (__any(qr != qw)) drain<false, ZS>();
        }
    }

    // Verlet-list walk: exact FP64 membership from the FP64 positions; the ring takes
    // the FP32 offsets (mirrored for flagged entries)
    template <bool ZS>
    __device__ __forceinline__ void pass_list(const int32_t *__restrict__ lst, int len,
                                              int64_t nl) {
        int k = 0;
        for (;;) {
            if (__any(qw - qr > (kQ - kU) * kSlot)) {
                drain<WALL, ZS>();
                continue;
            }
            if (!__any(k < len)) break;
            // entries k, k+1 share a chunk (k even): one 8-byte load
            const int2 ee = *(const int2 *)(lst + (int64_t)(k / kVlChunk) * nl * kVlChunk +
                                            (k % kVlChunk));
            int e[kU] = {k < len ? ee.x : 0, k + 1 < len ? ee.y : 0};
            double4 pj[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) pj[u] = ld(P4, e[u] & 0x7fffffff);
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const bool ghost = WALL && e[u] < 0;
                const double yj = ghost ? 2.0 * yw - pj[u].y : pj[u].y;
                const double dx = pj[u].x - xi, dy = yj - yi, dz = pj[u].z - zi;
                const double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
                const bool acc = (k + u < len) && r2 < pc.H2;
                // list entries carry the mirror flag in the sign bit
                const uint32_t eu = (uint32_t)e[u];
                slot(qw) = make_float4((float)dx, (float)dy, (float)dz,
                                       __uint_as_float(WALL ? (eu << 4) | (eu >> 31) : eu << 4));
                qw += acc ? kSlot : 0;
            }
            k += kU;
        }
    }
};

template <bool PAIR, bool WALL, bool LIST, bool PER>
__global__ __launch_bounds__(kRate32Block) void k_rates32(int64_t n, const float4 *__restrict__ A,
                                                    const float4 *__restrict__ B,
                                                    const float4 *__restrict__ Cz,
                                                    const double *__restrict__ xs,
                                                    const double *__restrict__ ys,
                                                    const double *__restrict__ zs,
                                                    const double *__restrict__ rho,
                                                    const double *__restrict__ dsz,
                                                    const int32_t *__restrict__ cs, GridDev g,
                                                    PairConst pc, const double *t_dev,
                                                    double t_host, RateOut o, int want_dt,
                                                    VList vl) {
    if (LIST && vl.gate && *vl.gate == 0) return;
    __shared__ float4 qd[kQ][kRate32Block];
    // finite placeholder offsets for lanes that pop from an empty ring
#pragma unroll
    for (int q = 0; q < kQ; ++q) qd[q][threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
    Rates32<PAIR, WALL, LIST, PER> k;
    k.A = A;
    k.P4 = (const double4 *)A;
    k.B = B;
    k.Cz = Cz;
    k.xs = xs;
    k.ys = ys;
    k.zs = zs;
    k.dsz = dsz;
    k.cs = cs;
    k.g = g;
    k.pc = pc;
    k.qb = (char *)&qd[0][0];
    k.lane16 = threadIdx.x * (int)sizeof(float4);
    const int64_t s =
        xcd_block_upto(blockIdx.x, gridDim.x, kRate32Chunk) * kRate32Block + threadIdx.x;
    k.self16 = (uint32_t)s * (uint32_t)sizeof(float4);
    k.live = s < n;
    k.a = make_float4(0.f, 0.f, 0.f, 0.f);
    k.b = k.a;
    k.c = k.a;
    k.xi = k.yi = k.zi = k.di = 0.0;
    if (k.live) {
        k.a = A[s];
        k.b = B[s];
        k.c = Cz[s];
        k.xi = xs[s];
        k.yi = ys[s];
        k.zi = zs[s];
        if (PAIR) k.di = dsz[s];
    }
    k.t = make_stencil(g, k.xi, k.yi, k.zi, pc.H);
    k.sig = k.c.y;
    k.Df = (float)g.cell;
    k.cxf = (float)k.t.cx;
    k.lo = (float)pc.H2 * (1.0f - kBand);
    k.hi = (float)pc.H2 * (1.0f + kBand);
    k.dwch0 = (float)(pc.dwc * pc.invH);
    k.ti = k.t;
    k.yw = 0.0;
    k.wd = 0.f;
    k.vw2 = 0.f;
    k.near_wall = false;
    if (WALL) {
        double tt = t_dev ? *t_dev : t_host;
        k.yw = pc.wall_y0 + pc.wall_v * tt;
        k.near_wall = k.live && mirror_band(g, k.yi, k.yw, pc.H);
        k.wd = (float)(k.yw - k.yi);
        k.vw2 = (float)(2.0 * pc.wall_v);
        k.ti = image_stencil(g, k.t, 2.0 * k.yw - k.yi);
    }
    k.tm = k.t;
    if (PER && k.live) k.nf = image_faces(pc, k.xi, k.yi, k.zi);
    const int len = LIST && k.live ? min(vl.count[s], vl.cap) : 0;
    const int32_t *lst = LIST ? vl.idx + (k.live ? s * kVlChunk : 0) : nullptr;
    if (*o.zflag == 0)
        k.template run<LIST, true>(lst, len, n);
    else
        k.template run<LIST, false>(lst, len, n);
    double dtv = INFINITY;
    if (k.live) {
        double ri = rho[s];
        double pre = 2.0 / ri;
        double drho = -2.0 * ri * (double)k.ar;
        o.rho[s] = drho;
        o.vx[s] = pre * (double)k.avx;
        o.vy[s] = pre * (double)k.avy;
        o.vz[s] = pre * (double)k.avz;
        const double vf = ((double)k.b.x * (double)k.avx + (double)k.b.y * (double)k.avy) +
                          (double)k.b.z * (double)k.avz;
        o.E[s] = pre * ((double)k.aE + vf);
        if (o.sig) o.sig[s] = (double)k.sig;
        if (o.cnt) o.cnt[s] = k.cnt;
        dtv = fmin((PAIR ? k.di : pc.h_dt) / (double)k.sig, ri / fabs(drho));
    }
    if (want_dt) wave_min_to(dtv, o.dtmin);
}

hipError_t launch_rates(int64_t n, int mixed, const GridDev &g, const PairConst &pc,
                        const Ws &w, double *const sorted[9], const double *d_sorted,
                        const double *t_dev, double t_host, int want_dt, hipStream_t st,
                        const int32_t *vl_count, const int32_t *vl_idx, int vl_cap,
                        const int32_t *gate) {
    if (n <= 0) return hipSuccess;
    const double *rho_sorted = sorted[6];
    RateOut o{w.rate[0], w.rate[1], w.rate[2], w.rate[3], w.rate[4], w.sig, w.cnt, w.dtmin,
              w.zflag};
    VList vl{vl_count, vl_idx, vl_cap, gate};
    const unsigned nb32 = (unsigned)((n + kRate32Block - 1) / kRate32Block);
    const unsigned nb64 = (unsigned)((n + kRate64Block - 1) / kRate64Block);
    const bool pair = pc.pair_mode != 0, wall = pc.wall != 0, list = vl_idx != nullptr;
    const bool per = pc.per != 0;
    if (list && (pair || per)) return hipErrorInvalidValue;
#define CSPH_RATES_CASE(P, W, L, X)                                                           \
    if (pair == P && wall == W && list == L && per == X) {                                    \
        if (mixed)                                                                            \
            k_rates32<P, W, L, X><<<nb32, kRate32Block, 0, st>>>(                             \
                n, (const float4 *)w.recA, (const float4 *)w.recB, (const float4 *)w.recC,    \
                sorted[0], sorted[1], sorted[2], rho_sorted, d_sorted, w.cs, g, pc, t_dev,    \
                t_host, o, want_dt, vl);                                                      \
        else                                                                                  \
            k_rates64<P, W, L, X><<<nb64, kRate64Block, 0, st>>>(                             \
                n, (const double4 *)w.recA, (const double4 *)w.recB,                          \
                (const double2 *)w.recC, (const float4 *)w.recF, rho_sorted, d_sorted, w.cs,  \
                g, pc, t_dev, t_host, o, want_dt, vl);                                        \
    }
    CSPH_RATES_CASE(false, false, false, false)
    CSPH_RATES_CASE(false, true, false, false)
    CSPH_RATES_CASE(true, false, false, false)
    CSPH_RATES_CASE(true, true, false, false)
    CSPH_RATES_CASE(false, false, true, false)
    CSPH_RATES_CASE(false, true, true, false)
    CSPH_RATES_CASE(false, false, false, true)
    CSPH_RATES_CASE(false, true, false, true)
    CSPH_RATES_CASE(true, false, false, true)
    CSPH_RATES_CASE(true, true, false, true)
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
    RateOut src{w.rate[0], w.rate[1], w.rate[2], w.rate[3], w.rate[4], w.sig, w.cnt, w.dtmin,
                w.zflag};
    k_unsort_rates<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, perm, src, out,
                                                                             signal, nbr_count);
    return hipGetLastError();
}

}  // namespace csph
