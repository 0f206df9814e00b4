// extern "C" entry points of libcsph: argument checks, mesh construction,
// workspace layout and the launch sequences of each call.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "adjoint.h"
#include "csph_internal.h"
#include "hostsync.h"

namespace csph {

static thread_local char g_err[512] = "";

static csph_status fail(csph_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

#define CSPH_HIP(expr)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(CSPH_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// ---------------------------------------------------------------- kernel timing

struct ProfRec {
    int group;
    hipEvent_t a, b;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static uint32_t g_prof_mask = ~0u;  // groups that record events while timing is on
static std::vector<ProfRec> g_prof_pending;
static std::vector<hipEvent_t> g_prof_pool;
static csph_profile g_prof_acc;

// Timing events only: no system-scope fence when one is recorded (the default fence writes
// back and invalidates the caches between the kernels it separates, which costs the stream
// ~10 us per event and the next kernel its warm L2).  csph_profile_read waits on each stop
// event and reads only the timestamps.
static hipError_t prof_event_create(hipEvent_t *e) {
    return hipEventCreateWithFlags(e, hipEventDisableSystemFence);
}

static hipEvent_t prof_event() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (prof_event_create(&e) != hipSuccess) return nullptr;
    return e;
}

// Records a start event on construction and a stop event on stop().
struct ProfScope {
    int group;
    hipStream_t st;
    hipEvent_t a = nullptr;
    // on = false: no event (the entry point that allocates nothing never creates events)
    ProfScope(int g, hipStream_t s, bool on = true) : group(g), st(s) {
        if (!on) return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof_on || !((g_prof_mask >> group) & 1u)) return;
        a = prof_event();
        if (a && hipEventRecord(a, st) != hipSuccess) {
            g_prof_pool.push_back(a);
            a = nullptr;
        }
    }
    void stop() {
        if (!a) return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        hipEvent_t b = prof_event();
        if (b && hipEventRecord(b, st) == hipSuccess) {
            g_prof_pending.push_back(ProfRec{group, a, b});
        } else {
            g_prof_pool.push_back(a);
            if (b) g_prof_pool.push_back(b);
        }
        a = nullptr;
    }
    ~ProfScope() { stop(); }
};

size_t ws_layout(Ws *w, void *base, int64_t n, int64_t ncell, bool rk2, int64_t ncell2) {
    size_t off = 0;
    char *b = (char *)base;
    auto take = [&](size_t bytes) -> void * {
        void *p = b ? (void *)(b + off) : nullptr;
        off += align256(bytes > 0 ? bytes : 1);
        return p;
    };
    size_t un = (size_t)(n > 0 ? n : 0);
    Ws t;
    t.bounds_part = (double *)take(sizeof(double) * 8 * kReduceBlocks);
    t.bounds_out = (double *)take(sizeof(double) * 8);
    t.dtmin = (unsigned long long *)take(2 * sizeof(unsigned long long));
    t.zflag = t.dtmin ? t.dtmin + 1 : nullptr;
    t.nonphys = (int64_t *)take(sizeof(int64_t));
    t.yenc = (unsigned long long *)take(sizeof(unsigned long long));
    t.tot_part = (double *)take(sizeof(double) * 10 * kReduceBlocks);
    int64_t scan_len = (n > ncell ? n : ncell) + 1;
    t.scan_tmp = (int64_t *)take(sizeof(int64_t) * (size_t)((scan_len + kScanTile - 1) / kScanTile + 1));
    t.key = (uint32_t *)take(sizeof(uint32_t) * un);
    t.rank = (uint32_t *)take(sizeof(uint32_t) * un);
    t.perm = (int32_t *)take(sizeof(int32_t) * un);
    t.bin_tmp = (int32_t *)take(sizeof(int32_t) * un);
    t.cnt = (int32_t *)take(sizeof(int32_t) * un);
    // A records: FP64 (32 B each) or FP32 (16 B), each followed by two zero records
    t.recA = take(32 * (un + 2));
    t.recB = take(32 * un);
    t.recC = take(16 * un);
    t.recF = take(16 * (un + 2));  // followed by two zero records, as the mixed A records
    t.recD = take(32 * un);
    t.recE = (double *)take(sizeof(double) * un);
    t.eos_part = (double *)take(sizeof(double) * 2 * CSPH_MAX_EOS * ((un + kBlock - 1) / kBlock + 1));
    for (int k = 0; k < 9; ++k) t.srt[k] = (double *)take(sizeof(double) * un);
    t.srt_mat = (int32_t *)take(sizeof(int32_t) * un);
    t.srt_d = (double *)take(sizeof(double) * un);
    t.srt_id = (int64_t *)take(sizeof(int64_t) * un);
    for (int k = 0; k < 5; ++k) t.rate[k] = (double *)take(sizeof(double) * un);
    t.sig = (double *)take(sizeof(double) * un);
    t.cs = (int32_t *)take(sizeof(int32_t) * (size_t)(ncell + 1));
    for (int k = 0; k < 8; ++k) t.stg[k] = nullptr;
    for (int k = 0; k < 9; ++k) t.srt2[k] = nullptr;
    t.srt2_d = nullptr;
    t.perm2 = t.rk_cnt = t.cs2 = nullptr;
    t.scan_tmp2 = nullptr;
    t.t2 = nullptr;
    if (rk2) {
        for (int k = 0; k < 8; ++k) t.stg[k] = (double *)take(sizeof(double) * un);
        for (int k = 0; k < 9; ++k) t.srt2[k] = (double *)take(sizeof(double) * un);
        t.srt2_d = (double *)take(sizeof(double) * un);
        t.perm2 = (int32_t *)take(sizeof(int32_t) * un);
        t.rk_cnt = (int32_t *)take(sizeof(int32_t) * un);
        t.t2 = (double *)take(sizeof(double));
        // last, so that laying the workspace out again with the second mesh's size moves
        // nothing the first stage wrote
        const int64_t nc2 = ncell2 > 0 ? ncell2 : ncell;
        t.cs2 = (int32_t *)take(sizeof(int32_t) * (size_t)(nc2 + 1));
        const int64_t len2 = (n > nc2 ? n : nc2) + 1;
        t.scan_tmp2 = (int64_t *)take(sizeof(int64_t) * (size_t)((len2 + kScanTile - 1) / kScanTile + 1));
    }
    t.bytes = off;
    if (w) *w = t;
    return off;
}

// Bytes of the workspace prefix used before the mesh is known (bounds).
static size_t ws_prefix() {
    return align256(sizeof(double) * 8 * kReduceBlocks) + align256(sizeof(double) * 8);
}

static csph_status check_params(const csph_params *p, bool need_pair_d, const double *d) {
    if (!p) return fail(CSPH_EINVAL, "params is NULL");
    if (p->precision != CSPH_FP64 && p->precision != CSPH_MIXED)
        return fail(CSPH_EINVAL, "precision %d unknown", p->precision);
    if (p->h_mode != CSPH_H_FIXED && p->h_mode != CSPH_H_PAIR)
        return fail(CSPH_EINVAL, "h_mode %d unknown", p->h_mode);
    if (!(p->kappa > 0.0) || !std::isfinite(p->kappa)) return fail(CSPH_EINVAL, "kappa must be > 0");
    if (p->h_mode == CSPH_H_FIXED && (!(p->h > 0.0) || !std::isfinite(p->h)))
        return fail(CSPH_EINVAL, "h must be > 0 in fixed-h mode");
    if (p->h_mode == CSPH_H_PAIR && need_pair_d && !d)
        return fail(CSPH_EINVAL, "pair-h mode needs the particle size array d");
    if (p->n_eos < 1 || p->n_eos > CSPH_MAX_EOS)
        return fail(CSPH_EINVAL, "n_eos must be in [1, %d]", CSPH_MAX_EOS);
    for (int k = 0; k < p->n_eos; ++k) {
        const csph_eos &e = p->eos[k];
        if (e.type != CSPH_EOS_IDEAL && e.type != CSPH_EOS_STIFFENED &&
            e.type != CSPH_EOS_MIE_GRUNEISEN)
            return fail(CSPH_EINVAL, "eos[%d].type %d unknown", k, e.type);
        if (e.type == CSPH_EOS_MIE_GRUNEISEN) {
            if (!(e.gamma > 0.0) || !std::isfinite(e.gamma))
                return fail(CSPH_EINVAL, "eos[%d].gamma (Grueneisen) must be > 0", k);
            if (!(e.rho0 > 0.0) || !std::isfinite(e.rho0) || !(e.c_a > 0.0) ||
                !std::isfinite(e.c_a) || !(e.s_a >= 0.0) || !std::isfinite(e.s_a))
                return fail(CSPH_EINVAL, "eos[%d]: need rho0 > 0, c_a > 0, s_a >= 0", k);
        } else if (!(e.gamma > 1.0) || !std::isfinite(e.gamma)) {
            return fail(CSPH_EINVAL, "eos[%d].gamma must be > 1", k);
        }
        if (!std::isfinite(e.p_inf)) return fail(CSPH_EINVAL, "eos[%d].p_inf not finite", k);
    }
    if (p->key_mode != CSPH_KEY_LINEAR && p->key_mode != CSPH_KEY_MORTON)
        return fail(CSPH_EINVAL, "key_mode %d unknown", p->key_mode);
    if (!std::isfinite(p->cell_size)) return fail(CSPH_EINVAL, "cell_size not finite");
    if (!std::isfinite(p->cfl)) return fail(CSPH_EINVAL, "cfl not finite");
    if (p->wall && (!std::isfinite(p->wall_x0) || !std::isfinite(p->wall_v)))
        return fail(CSPH_EINVAL, "wall position/velocity not finite");
    if (p->integrator != CSPH_INT_EULER && p->integrator != CSPH_INT_RK2)
        return fail(CSPH_EINVAL, "integrator %d unknown", p->integrator);
    if (p->periodic < 0 || p->periodic > 7) return fail(CSPH_EINVAL, "periodic mask %d unknown", p->periodic);
    if (p->wall && (p->periodic & 1)) return fail(CSPH_EINVAL, "the wall's axis x cannot be periodic");
    for (int a = 0; a < 3; ++a)
        if (((p->periodic >> a) & 1) &&
            !(std::isfinite(p->box_lo[a]) && std::isfinite(p->box_hi[a]) && p->box_hi[a] > p->box_lo[a]))
            return fail(CSPH_EINVAL, "periodic axis %d needs a finite box with box_hi > box_lo", a);
    return CSPH_OK;
}

// The caller's axis each of the kernels' axes takes (k[a] for kernel axis a).  The kernels walk
// stencil rows along their x axis and cut the cell order into slabs along y, so a boundary
// normal to their x axis puts particles within its support at both ends of every row, in a few
// lanes of most waves.  With a piston the wall normal (the caller's x) is handed over as y, so
// that the particles with mirror partners fill a few waves; without one a periodic x is handed
// over as y when y is open, so that the waves with periodic image walks are the few at the
// slab faces.  Only x and y are ever exchanged: the exact decisions sum squared offsets as
// ((x x) + (y y)) + (z z), whose rounding an exchange of the first two terms leaves unchanged.
struct Axes {
    int k[3];
};

static Axes kernel_axes(const csph_params *p) {
    if (p->wall || ((p->periodic & 1) && !(p->periodic & 2))) return Axes{{1, 0, 2}};
    return Axes{{0, 1, 2}};
}

// the kernels' axis that takes the caller's axis a
static int kernel_axis_of(const Axes &ax, int a) {
    return ax.k[0] == a ? 0 : ax.k[1] == a ? 1 : 2;
}

// Near-face band of the periodic image search: the support with a relative margin (a pair's
// FP64 offset carries a few ulp of the period).
static double periodic_band(double H) { return H * (1.0 + 1e-6); }

// Periodic boxes against the particle bounds (b: min x, y, z, max x, y, z in the kernels'
// axes, kernel_axes) and the maximum support: each period must
// exceed twice the near-face band (so a particle has images across one face per axis at most,
// and no pair of particles more than one image of each other) and the positions must lie in
// the box.
static csph_status check_box(const csph_params *p, const double b[6], double Hmax, int64_t n) {
    if (!p->periodic || n == 0) return CSPH_OK;
    const double hb = periodic_band(Hmax);
    for (int a = 0; a < 3; ++a) {
        if (!((p->periodic >> a) & 1)) continue;
        const int k = kernel_axis_of(kernel_axes(p), a);
        const double L = p->box_hi[a] - p->box_lo[a];
        if (!(L > 2.0 * hb))
            return fail(CSPH_EINVAL, "period %g of axis %d must exceed twice the support %g (1 + 1e-6)",
                        L, a, Hmax);
        if (!(b[k] >= p->box_lo[a] && b[3 + k] <= p->box_hi[a]))
            return fail(CSPH_EINVAL, "positions along periodic axis %d lie outside [%g, %g]", a,
                        p->box_lo[a], p->box_hi[a]);
    }
    return CSPH_OK;
}

static bool state_ok(const csph_state *s) {
    return s && s->n >= 0 &&
           (s->n == 0 || (s->x && s->y && s->z && s->vx && s->vy && s->vz && s->rho && s->E && s->m));
}

static EosDev eos_dev(const csph_params *p) {
    EosDev e;
    memset(&e, 0, sizeof(e));
    e.n = p->n_eos;
    for (int k = 0; k < p->n_eos; ++k) {
        e.type[k] = p->eos[k].type;
        e.gamma[k] = p->eos[k].gamma;
        e.pinf[k] = p->eos[k].p_inf;
        e.rho0[k] = p->eos[k].rho0;
        e.ca[k] = p->eos[k].c_a;
        e.sa[k] = p->eos[k].s_a;
    }
    return e;
}

static PairConst pair_const(const csph_params *p, double dmax) {
    PairConst c;
    memset(&c, 0, sizeof(c));
    c.pair_mode = p->h_mode == CSPH_H_PAIR;
    c.kappa = p->kappa;
    double H = c.pair_mode ? p->kappa * dmax : p->kappa * p->h;
    c.H = H;
    c.H2 = H * H;
    c.invH = 1.0 / H;
    double i2 = c.invH * c.invH;
    c.dwc = (210.0 / M_PI) * (i2 * i2);
    c.h_dt = p->h;
    c.wall = p->wall != 0;
    c.wall_y0 = p->wall_x0;  // the wall normal is the kernels' y axis (kernel_axes)
    c.wall_v = p->wall_v;
    c.per = 0;
    c.hb = periodic_band(H);
    const Axes ax = kernel_axes(p);
    for (int a = 0; a < 3; ++a) {
        const int k = kernel_axis_of(ax, a);
        if ((p->periodic >> a) & 1) {
            c.per |= 1 << k;
            c.lo[k] = p->box_lo[a];
            c.hi[k] = p->box_hi[a];
            c.L[k] = p->box_hi[a] - p->box_lo[a];
        }
    }
    return c;
}

// The arrays the kernels see: the caller's position, velocity and rate arrays in the kernels'
// axes (kernel_axes).
static csph_state kernel_view(const csph_state &s, const Axes &ax) {
    csph_state v = s;
    double *const pos[3] = {s.x, s.y, s.z}, *const vel[3] = {s.vx, s.vy, s.vz};
    v.x = pos[ax.k[0]];
    v.y = pos[ax.k[1]];
    v.z = pos[ax.k[2]];
    v.vx = vel[ax.k[0]];
    v.vy = vel[ax.k[1]];
    v.vz = vel[ax.k[2]];
    return v;
}

static csph_rates_out kernel_view(const csph_rates_out &o, const Axes &ax) {
    csph_rates_out v = o;
    double *const dv[3] = {o.dvx, o.dvy, o.dvz};
    v.dvx = dv[ax.k[0]];
    v.dvy = dv[ax.k[1]];
    v.dvz = dv[ax.k[2]];
    return v;
}

// slab = false: the plain linear cell key (the key csph_bin reports);
// slab = true: the y-slab order the internal passes sort by.
static GridDev grid_dev(const csph_grid &g, bool slab = true, double ymin = 0.0) {
    GridDev d;
    d.ymin = ymin;
    d.ox = g.origin[0];
    d.oy = g.origin[1];
    d.oz = g.origin[2];
    d.inv = g.inv_cell;
    d.cell = g.cell;
    d.dx = g.dims[0];
    d.dy = g.dims[1];
    d.dz = g.dims[2];
    d.reach = g.reach;
    const uint32_t dx = (uint32_t)d.dx, dy = (uint32_t)d.dy, dz = (uint32_t)d.dz;
    if (slab && dy > (1u << kSlabShift)) {
        const uint32_t rows = 1u << kSlabShift;
        d.ysh = kSlabShift;
        d.ymask = (int)rows - 1;
        d.nfull = (int)(dy >> kSlabShift);
        d.sZf = rows * dx;
        d.sZr = (dy & (rows - 1)) * dx;
        d.sY = dz * rows * dx;
    } else {
        d.ysh = 31;
        d.ymask = 0x7fffffff;
        d.nfull = 1;
        d.sZf = dy * dx;
        d.sZr = d.sZf;
        d.sY = 0;
    }
    d.morton = 0;
    d.nkey = (int64_t)d.dx * d.dy * d.dz;
    d.yenc = nullptr;
    return d;
}

// Bits per axis of the Morton key space of a mesh: ceil(log2(max dims)).
static int morton_bits(const int32_t dims[3]) {
    int m = dims[0] > dims[1] ? dims[0] : dims[1];
    m = m > dims[2] ? m : dims[2];
    int b = 0;
    while ((1 << b) < m) ++b;
    return b;
}

// ---------------------------------------------------------------- bounds to the host
//
// Each host thread keeps, per device, one pinned fine-grained slot that the bounds kernel
// writes, and a sequence number per call; make_grid is done with the slot before it returns,
// so a thread's calls never share it while in flight.  The host spins on the sequence
// number (asking the stream every ~1 000 spins whether it failed or drained without it),
// which returns a few microseconds after the kernel's store, where a copy to pageable
// memory and a stream synchronisation left the GPU idle for ~70 us per step.
constexpr int kPollDevices = 64;
struct PollSlots {
    HostBounds *host[kPollDevices] = {};
    HostBounds *dev[kPollDevices] = {};
    unsigned long long seq = 0;
};
static thread_local PollSlots g_poll;

// The calling thread's slot on the current device (allocated on first use), or nullptr when
// none can be had; *dev_slot receives its device address.
static HostBounds *host_slot(HostBounds **dev_slot) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kPollDevices) return nullptr;
    if (!g_poll.host[dev]) {
        void *hp = nullptr, *dp = nullptr;
        if (hipHostMalloc(&hp, sizeof(HostBounds), hipHostMallocCoherent) != hipSuccess ||
            !hp) {
            (void)hipGetLastError();
            return nullptr;
        }
        if (hipHostGetDevicePointer(&dp, hp, 0) != hipSuccess || !dp) {
            (void)hipGetLastError();
            (void)hipHostFree(hp);
            return nullptr;
        }
        __atomic_store_n(&((HostBounds *)hp)->seq, 0ull, __ATOMIC_RELEASE);
        g_poll.host[dev] = (HostBounds *)hp;
        g_poll.dev[dev] = (HostBounds *)dp;
    }
    *dev_slot = g_poll.dev[dev];
    return g_poll.host[dev];
}

// Spins until the slot holds sequence number `want` (asking the stream every ~1 000 spins
// whether it failed, or drained without it).
static csph_status poll_slot(HostBounds *hb, unsigned long long want, hipStream_t st,
                             const char *what) {
    for (unsigned it = 1; __atomic_load_n(&hb->seq, __ATOMIC_ACQUIRE) != want; ++it) {
        if ((it & 1023) == 0) {
            const hipError_t q = hipStreamQuery(st);
            if (q == hipSuccess) {
                if (__atomic_load_n(&hb->seq, __ATOMIC_ACQUIRE) == want) break;
                return fail(CSPH_EDEVICE, "%s: the stream drained without them", what);
            }
            if (q != hipErrorNotReady)
                return fail(CSPH_EDEVICE, "%s: %s", what, hipGetErrorString(q));
        }
        __builtin_ia32_pause();
    }
    return CSPH_OK;
}

// *done = false (nothing launched) when no slot can be had: the caller copies and
// synchronises instead.
static csph_status bounds_polled(const double *x, const double *y, const double *z,
                                 const double *d, int64_t n, double *part, double *out,
                                 hipStream_t st, double b[7], bool *done) {
    *done = false;
    HostBounds *dslot = nullptr, *hb = host_slot(&dslot);
    if (!hb) return CSPH_OK;
    const unsigned long long want = ++g_poll.seq;
    CSPH_HIP(launch_bounds_host(x, y, z, d, n, part, out, dslot, want, st));
    csph_status r = poll_slot(hb, want, st, "mesh bounds");
    if (r) return r;
    for (int k = 0; k < 7; ++k) b[k] = ((volatile const double *)hb->b)[k];
    *done = true;
    return CSPH_OK;
}

// A 64-bit device word to the host: through the thread's slot when it can be had (the word
// as b[0]'s bits), else a copy and a synchronisation.
static csph_status word_to_host(const unsigned long long *src, unsigned long long *out,
                                hipStream_t st) {
    HostBounds *dslot = nullptr, *hb = host_slot(&dslot);
    if (hb) {
        const unsigned long long want = ++g_poll.seq;
        CSPH_HIP(launch_word_host(src, dslot, want, st));
        csph_status r = poll_slot(hb, want, st, "device word");
        if (r) return r;
        *out = ((volatile const unsigned long long *)hb->b)[0];
        return CSPH_OK;
    }
    CSPH_HIP(hipMemcpyAsync(out, src, sizeof(*out), hipMemcpyDeviceToHost, st));
    CSPH_HIP(hipStreamSynchronize(st));
    return CSPH_OK;
}

// Mesh from device bounds (synchronises `st`); also returns max d and the minimum y.
// snap = false: the mesh of sec. 4.2 as csph_grid_build defines it (origin = the minimum
// position).  snap = true (the library's own passes): the origin is moved down to a whole
// multiple of D, so that the cells stay fixed in space from one step to the next while the
// particle set moves (a piston pushing the minimum along by a fraction of a cell per step
// would otherwise move every particle's cell index and scatter the next step's gather).
// Results do not depend on the mesh: membership is decided by exact FP64 distances.
// snap = true also checks the periodic box against the bounds (the arrays are then in the
// kernels' axes, x and y swapped when p has a wall).  poll: the bounds come through the
// calling thread's pinned slot (bounds_polled); the entry point that allocates nothing passes
// false and keeps the copy and the synchronisation.
static csph_status make_grid(const double *x, const double *y, const double *z, const double *d,
                             int64_t n, const csph_params *p, void *ws, size_t ws_bytes,
                             hipStream_t st, csph_grid *g, double *dmax, double *ymin,
                             bool snap, bool poll = true) {
    if (ws_bytes < ws_prefix() || !ws)
        return fail(CSPH_ECAPACITY, "workspace smaller than %zu bytes", ws_prefix());
    double b[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (n > 0) {
        Ws w;
        ws_layout(&w, ws, 0, 0);
        const double *dd = p->h_mode == CSPH_H_PAIR ? d : nullptr;
        bool done = false;
        if (poll) {
            csph_status r = bounds_polled(x, y, z, dd, n, w.bounds_part, w.bounds_out, st, b,
                                          &done);
            if (r) return r;
        }
        if (!done) {
            CSPH_HIP(launch_bounds(x, y, z, dd, n, w.bounds_part, w.bounds_out, st));
            CSPH_HIP(hipMemcpyAsync(b, w.bounds_out, sizeof(double) * 7, hipMemcpyDeviceToHost,
                                    st));
            CSPH_HIP(hipStreamSynchronize(st));
        }
    }
    for (int k = 0; k < 7; ++k)
        if (!std::isfinite(b[k])) return fail(CSPH_EINVAL, "non-finite particle positions or sizes");
    *dmax = b[6];
    *ymin = b[1];
    double Hmax = p->h_mode == CSPH_H_PAIR ? p->kappa * b[6] : p->kappa * p->h;
    if (snap) {
        csph_status r = check_box(p, b, Hmax, n);
        if (r) return r;
    }
    double D = p->cell_size > 0.0 ? p->cell_size : Hmax;
    if (!(D > 0.0)) D = 1.0;  // pair mode with all d = 0: any mesh works
    g->cell = D;
    g->inv_cell = 1.0 / D;
    if (snap) {
        for (int a = 0; a < 3; ++a) {
            const double o = floor(b[a] * g->inv_cell) * D;
            if (o <= b[a] && std::isfinite(o)) b[a] = o;  // else keep the minimum itself
        }
    }
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        g->origin[a] = b[a];
        double span = floor((b[3 + a] - b[a]) * g->inv_cell);
        if (!(span < 2.0e9)) return fail(CSPH_EINVAL, "mesh too fine for the particle extent");
        g->dims[a] = (int32_t)span + 1;
        ncell *= g->dims[a];
        if (ncell > 2000000000LL) return fail(CSPH_EINVAL, "mesh has more than 2e9 cells");
    }
    double r = ceil(Hmax / D);
    g->reach = r < 1.0 ? 1 : (int32_t)r;
    if (g->reach > 64) return fail(CSPH_EINVAL, "cell size below 1/64 of the support");
    g->ncell = ncell;
    g->key_mode = p->key_mode;
    g->pad = 0;
    g->nkey = ncell;
    if (p->key_mode == CSPH_KEY_MORTON) {
        if (g->dims[0] > 1024 || g->dims[1] > 1024 || g->dims[2] > 1024)
            return fail(CSPH_EINVAL, "Morton keys need at most 1024 cells per axis");
        g->nkey = (int64_t)1 << (3 * morton_bits(g->dims));
    }
    return CSPH_OK;
}

static csph_status need_ws(size_t have, int64_t n, int64_t ncell, size_t *ws_needed,
                           bool rk2 = false, int64_t ncell2 = 0) {
    size_t need = ws_layout(nullptr, nullptr, n, ncell, rk2, ncell2);
    if (ws_needed) *ws_needed = need;
    if (have < need) return fail(CSPH_ECAPACITY, "workspace needs %zu bytes, got %zu", need, have);
    return CSPH_OK;
}

// A mesh the caller gives for a step (csph_step_mesh): a positive cell, consistent dims and
// cell count, and a stencil reach covering the support H.
static csph_status check_mesh(const csph_grid *m, double H) {
    if (!m) return fail(CSPH_EINVAL, "mesh is NULL");
    if (!(m->cell > 0.0) || !std::isfinite(m->cell) || m->inv_cell != 1.0 / m->cell)
        return fail(CSPH_EINVAL, "mesh: need cell > 0 and inv_cell = 1/cell");
    int64_t nc = 1;
    for (int a = 0; a < 3; ++a) {
        if (m->dims[a] < 1 || !std::isfinite(m->origin[a]))
            return fail(CSPH_EINVAL, "mesh: dims must be >= 1 and the origin finite");
        nc *= m->dims[a];
        if (nc > 2000000000LL) return fail(CSPH_EINVAL, "mesh has more than 2e9 cells");
    }
    if (nc != m->ncell) return fail(CSPH_EINVAL, "mesh: ncell does not match dims");
    if (m->reach < 1 || m->reach > 64 || (double)m->reach * m->cell < H)
        return fail(CSPH_EINVAL, "mesh: reach * cell must cover the support (reach <= 64)");
    return CSPH_OK;
}

// The call's own non-physical count (counted into the workspace counter): added to the
// caller's counter, brought to the host (synchronises), CSPH_ENONPHYS when not 0.
static csph_status finish_nonphys(const Ws &w, int64_t *nonphys, hipStream_t st) {
    if (nonphys) CSPH_HIP(launch_add_i64(nonphys, w.nonphys, st));
    int64_t bad = 0;
    CSPH_HIP(hipMemcpyAsync(&bad, w.nonphys, sizeof(bad), hipMemcpyDeviceToHost, st));
    CSPH_HIP(hipStreamSynchronize(st));
    if (bad > 0) return fail(CSPH_ENONPHYS, "%lld particles in a non-physical state", (long long)bad);
    return CSPH_OK;
}

// ---------------------------------------------------------------- static scratch
//
// The workspace of csph_step_static, the entry point for callers that cannot allocate device
// memory: one array per GPU the library runs on, held from the code object's load until the
// process ends.  In host code the array's name is only a stand-in for the device symbol, so
// its device address is looked up once per device, with that device current, and that
// address is what the kernels receive.
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch[kMaxDevices];

static csph_status static_scratch(void **out) {
    int dev = 0;
    CSPH_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(CSPH_EDEVICE, "device %d: the static scratch serves devices 0..%d", dev,
                    kMaxDevices - 1);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        CSPH_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(CSPH_EDEVICE, "no device address for the static scratch");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return CSPH_OK;
}

// Voronoi outputs of csph_step_voronoi.
struct VoroArgs {
    const double *sites;
    int32_t K;
    int32_t *owner;
    int64_t *site_particles, *site_pairs;
};

// The body of csph_step, csph_step_static (prof = false: no timing events) and
// csph_step_voronoi (va: the ownership of the new positions).
static csph_status step_impl(const csph_state *s_in, csph_state *s_out, const csph_params *p,
                             double *t, double dt_in, double *dt_used, double *totals,
                             int32_t *nbr_count, int64_t *nonphys, void *ws, size_t ws_bytes,
                             size_t *ws_needed, hipStream_t st, bool prof,
                             const VoroArgs *va = nullptr, const csph_grid *mesh = nullptr,
                             int64_t *outside = nullptr);

}  // namespace csph

using namespace csph;

extern "C" {

const char *csph_status_string(csph_status s) {
    switch (s) {
        case CSPH_OK: return "CSPH_OK";
        case CSPH_EINVAL: return "CSPH_EINVAL: invalid argument";
        case CSPH_ECAPACITY: return "CSPH_ECAPACITY: output or workspace too small";
        case CSPH_EDEVICE: return "CSPH_EDEVICE: HIP runtime error";
        case CSPH_ENONPHYS: return "CSPH_ENONPHYS: non-physical state met (outputs written)";
        default: return "unknown csph status";
    }
}

const char *csph_last_error(void) { return g_err; }

const char *csph_version(void) { return "csph-gfx950 0.1"; }

size_t csph_workspace_size(int64_t n, int64_t ncell, const csph_params *p) {
    const bool rk2 = p && p->integrator == CSPH_INT_RK2;
    return ws_layout(nullptr, nullptr, n < 0 ? 0 : n, ncell < 1 ? 1 : ncell, rk2);
}

csph_status csph_grid_build(const double *x, const double *y, const double *z, int64_t n,
                            const csph_params *p, const double *d, csph_grid *grid, void *ws,
                            size_t ws_bytes, csph_stream stream) {
    g_err[0] = 0;
    if (n < 0 || !grid || (n > 0 && (!x || !y || !z))) return fail(CSPH_EINVAL, "bad arguments");
    csph_status s = check_params(p, n > 0, d);
    if (s) return s;
    double dmax, ymin;
    return make_grid(x, y, z, d, n, p, ws, ws_bytes, (hipStream_t)stream, grid, &dmax, &ymin,
                     false);
}

csph_status csph_bin(const double *x, const double *y, const double *z, int64_t n,
                     const csph_grid *grid, uint32_t *key, int32_t *perm, int32_t *cell_start,
                     int64_t cell_start_cap, void *ws, size_t ws_bytes, size_t *ws_needed,
                     csph_stream stream) {
    g_err[0] = 0;
    if (n < 0 || n >= INT32_MAX || !grid || !cell_start || (n > 0 && (!x || !y || !z || !perm)))
        return fail(CSPH_EINVAL, "bad arguments");
    if (!(grid->inv_cell > 0.0) || grid->dims[0] < 1 || grid->dims[1] < 1 || grid->dims[2] < 1)
        return fail(CSPH_EINVAL, "bad mesh");
    int64_t ncell = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
    if (ncell != grid->ncell) return fail(CSPH_EINVAL, "grid->ncell does not match dims");
    int64_t nkey = ncell;
    if (grid->key_mode == CSPH_KEY_MORTON) {
        if (grid->dims[0] > 1024 || grid->dims[1] > 1024 || grid->dims[2] > 1024)
            return fail(CSPH_EINVAL, "Morton keys need at most 1024 cells per axis");
        nkey = (int64_t)1 << (3 * morton_bits(grid->dims));
    } else if (grid->key_mode != CSPH_KEY_LINEAR) {
        return fail(CSPH_EINVAL, "grid->key_mode %d unknown", grid->key_mode);
    }
    if (nkey != grid->nkey) return fail(CSPH_EINVAL, "grid->nkey does not match dims and key_mode");
    if (cell_start_cap < nkey + 1)
        return fail(CSPH_ECAPACITY, "cell_start needs %lld entries", (long long)(nkey + 1));
    csph_status s = need_ws(ws_bytes, n, nkey, ws_needed);
    if (s) return s;
    Ws w;
    ws_layout(&w, ws, n, nkey);
    hipStream_t st = (hipStream_t)stream;
    ProfScope pb(CSPH_PROF_BIN, st);
    GridDev gd = grid_dev(*grid, false);
    gd.morton = grid->key_mode == CSPH_KEY_MORTON;
    gd.nkey = nkey;
    CSPH_HIP(launch_bin(x, y, z, n, gd, w, perm, key, cell_start, st));
    return CSPH_OK;
}

csph_status csph_neighbors(const csph_state *s, const csph_params *p, int64_t *offsets,
                           int32_t *idx, int64_t idx_cap, int64_t *nnz, void *ws, size_t ws_bytes,
                           size_t *ws_needed, csph_stream stream) {
    g_err[0] = 0;
    if (!s || s->n < 0 || s->n >= INT32_MAX || !offsets || !nnz ||
        (s->n > 0 && (!s->x || !s->y || !s->z)))
        return fail(CSPH_EINVAL, "bad arguments");
    csph_status r = check_params(p, s->n > 0, s->d);
    if (r) return r;
    hipStream_t st = (hipStream_t)stream;
    int64_t n = s->n;
    csph_grid g;
    double dmax, ymin;
    csph_params pn0 = *p;  // N(i) has no mirror partners: no wall
    pn0.wall = 0;
    p = &pn0;
    // positions in the kernels' axes (N(i) does not depend on them)
    const csph_state sv = kernel_view(*s, kernel_axes(p));
    r = make_grid(sv.x, sv.y, sv.z, s->d, n, p, ws, ws_bytes, st, &g, &dmax, &ymin, true);
    if (r) return r;
    r = need_ws(ws_bytes, n, g.ncell, ws_needed);
    if (r) return r;
    Ws w;
    ws_layout(&w, ws, n, g.ncell);
    GridDev gd = grid_dev(g, true, ymin);
    PairConst pc = pair_const(p, dmax);
    const double *dd = p->h_mode == CSPH_H_PAIR ? s->d : nullptr;
    ProfScope pn(CSPH_PROF_NEIGHBORS, st);
    CSPH_HIP(launch_bin(sv.x, sv.y, sv.z, n, gd, w, w.perm, nullptr, w.cs, st));
    CSPH_HIP(launch_gather_pos(n, w.perm, sv.x, sv.y, sv.z, dd, w, st));
    CSPH_HIP(launch_nbr_count(n, gd, pc, w.srt[0], w.srt[1], w.srt[2], w.srt_d, w.cs, w.perm,
                              w.cnt, st));
    pn.stop();
    CSPH_HIP((launch_scan_exclusive<int32_t, int64_t>(w.cnt, offsets, n, w.scan_tmp, st)));
    int64_t total = 0;
    CSPH_HIP(hipMemcpyAsync(&total, offsets + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    CSPH_HIP(hipStreamSynchronize(st));
    *nnz = total;
    if (!idx) return CSPH_OK;
    if (idx_cap < total)
        return fail(CSPH_ECAPACITY, "idx needs %lld entries", (long long)total);
    CSPH_HIP(launch_nbr_fill(n, gd, pc, w.srt[0], w.srt[1], w.srt[2], w.srt_d, w.cs, w.perm,
                             offsets, idx, st));
    return CSPH_OK;
}

csph_status csph_rates(const csph_state *s, const csph_params *p, double t, csph_rates_out out,
                       double *signal, int32_t *nbr_count, int64_t *nonphys, void *ws,
                       size_t ws_bytes, size_t *ws_needed, csph_stream stream) {
    g_err[0] = 0;
    if (!state_ok(s) || s->n >= INT32_MAX) return fail(CSPH_EINVAL, "bad state");
    if (s->n >= kMaxPairN) return fail(CSPH_EINVAL, "n >= 2^27 particles");
    if (s->n > 0 && (!out.drho || !out.dvx || !out.dvy || !out.dvz || !out.dE))
        return fail(CSPH_EINVAL, "rate outputs must not be NULL");
    if (!std::isfinite(t)) return fail(CSPH_EINVAL, "t not finite");
    csph_status r = check_params(p, s->n > 0, s->d);
    if (r) return r;
    hipStream_t st = (hipStream_t)stream;
    int64_t n = s->n;
    const Axes ax = kernel_axes(p);
    const csph_state sv = kernel_view(*s, ax);
    const csph_rates_out ov = kernel_view(out, ax);
    csph_grid g;
    double dmax, ymin;
    r = make_grid(sv.x, sv.y, sv.z, sv.d, n, p, ws, ws_bytes, st, &g, &dmax, &ymin, true);
    if (r) return r;
    r = need_ws(ws_bytes, n, g.ncell, ws_needed);
    if (r) return r;
    if (n == 0) return CSPH_OK;
    Ws w;
    ws_layout(&w, ws, n, g.ncell);
    GridDev gd = grid_dev(g, true, ymin);
    PairConst pc = pair_const(p, dmax);
    EosDev eos = eos_dev(p);
    int mixed = p->precision == CSPH_MIXED;
    bool pair = p->h_mode == CSPH_H_PAIR;
    {
        ProfScope pr(CSPH_PROF_BIN, st);
        CSPH_HIP(launch_bin(sv.x, sv.y, sv.z, n, gd, w, w.perm, nullptr, w.cs, st));
    }
    CSPH_HIP(launch_fill_u64(w.dtmin, 0x7ff0000000000000ull, 2, st));  // dt min, Z flag
    CSPH_HIP(launch_fill_u64((unsigned long long *)w.nonphys, 0ull, 1, st));
    {
        ProfScope pr(CSPH_PROF_PACK, st);
        CSPH_HIP(launch_pack(sv, n, w.perm, eos, mixed, gd, w, w.srt, w.srt_mat,
                             pair ? w.srt_d : nullptr, nullptr, nullptr, w.nonphys, st));
    }
    {
        ProfScope pr(CSPH_PROF_RATES, st);
        CSPH_HIP(launch_rates(n, mixed, gd, pc, w, w.srt, pair ? w.srt_d : nullptr, nullptr, t,
                              0, st));
    }
    {
        ProfScope pr(CSPH_PROF_REORDER, st);
        CSPH_HIP(launch_unsort_rates(n, w.perm, w, ov, signal, nbr_count, st));
    }
    return finish_nonphys(w, nonphys, st);
}

csph_status csph_step(const csph_state *s_in, csph_state *s_out, const csph_params *p, double *t,
                      double dt_in, double *dt_used, double *totals, int32_t *nbr_count,
                      int64_t *nonphys, void *ws, size_t ws_bytes, size_t *ws_needed,
                      csph_stream stream) {
    g_err[0] = 0;
    return step_impl(s_in, s_out, p, t, dt_in, dt_used, totals, nbr_count, nonphys, ws,
                     ws_bytes, ws_needed, (hipStream_t)stream, true);
}

csph_status csph_step_voronoi(const csph_state *s_in, csph_state *s_out, const csph_params *p,
                              double *t, double dt_in, double *dt_used, double *totals,
                              int32_t *nbr_count, int64_t *nonphys, const double *sites,
                              int32_t K, int32_t *owner, int64_t *site_particles,
                              int64_t *site_pairs, void *ws, size_t ws_bytes, size_t *ws_needed,
                              csph_stream stream) {
    g_err[0] = 0;
    if (K < 1 || K > kMaxSites || !sites || !site_particles ||
        (s_in && s_in->n > 0 && !owner))
        return fail(CSPH_EINVAL, "bad Voronoi arguments (1 <= K <= %d)", kMaxSites);
    const VoroArgs va{sites, K, owner, site_particles, site_pairs};
    return step_impl(s_in, s_out, p, t, dt_in, dt_used, totals, nbr_count, nonphys, ws,
                     ws_bytes, ws_needed, (hipStream_t)stream, true, &va);
}

csph_status csph_step_static(const csph_state *s_in, csph_state *s_out, const csph_params *p,
                             double *t, double dt_in, double *dt_used, double *totals,
                             int32_t *nbr_count, int64_t *nonphys, csph_stream stream) {
    g_err[0] = 0;
    void *ws = nullptr;
    csph_status r = static_scratch(&ws);
    if (r) return r;
    // sizes beyond the scratch are refused before any device work when the per-particle
    // part alone does not fit; the mesh part is checked once the mesh is known
    const int64_t n = s_in ? s_in->n : 0;
    if (n > 0 && ws_layout(nullptr, nullptr, n, 1) > kStaticScratchBytes)
        return fail(CSPH_ECAPACITY,
                    "csph_step_static: %lld particles need %zu bytes of scratch, more than its "
                    "%zu bytes", (long long)n, ws_layout(nullptr, nullptr, n, 1),
                    kStaticScratchBytes);
    size_t need = 0;
    r = step_impl(s_in, s_out, p, t, dt_in, dt_used, totals, nbr_count, nonphys, ws,
                  kStaticScratchBytes, &need, (hipStream_t)stream, false);
    if (r == CSPH_ECAPACITY)
        return fail(CSPH_ECAPACITY,
                    "csph_step_static: this step needs %zu bytes of scratch, more than its %zu "
                    "bytes", need, kStaticScratchBytes);
    return r;
}

csph_status csph_step_mesh(const csph_state *s_in, csph_state *s_out, const csph_params *p,
                           const csph_grid *mesh, double *t, double dt_in, double *dt_used,
                           double *totals, int32_t *nbr_count, int64_t *nonphys,
                           int64_t *outside, void *ws, size_t ws_bytes, size_t *ws_needed,
                           csph_stream stream) {
    g_err[0] = 0;
    if (!mesh) return fail(CSPH_EINVAL, "mesh is NULL");
    return step_impl(s_in, s_out, p, t, dt_in, dt_used, totals, nbr_count, nonphys, ws,
                     ws_bytes, ws_needed, (hipStream_t)stream, true, nullptr, mesh, outside);
}

}  // extern "C"

namespace csph {

static csph_status step_impl(const csph_state *s_in, csph_state *s_out, const csph_params *p,
                             double *t, double dt_in, double *dt_used, double *totals,
                             int32_t *nbr_count, int64_t *nonphys, void *ws, size_t ws_bytes,
                             size_t *ws_needed, hipStream_t st, bool prof, const VoroArgs *va,
                             const csph_grid *mesh, int64_t *outside) {
    if (!state_ok(s_in) || !state_ok(s_out) || s_in->n != s_out->n || s_in->n >= INT32_MAX)
        return fail(CSPH_EINVAL, "bad state");
    if (s_in->n >= kMaxPairN) return fail(CSPH_EINVAL, "n >= 2^27 particles");
    csph_status r = check_params(p, s_in->n > 0, s_in->d);
    if (r) return r;
    if (!(p->cfl > 0.0) && !(std::isfinite(dt_in) && dt_in >= 0.0))
        return fail(CSPH_EINVAL, "cfl <= 0 needs a finite dt_in >= 0");
    if (p->wall && !t) return fail(CSPH_EINVAL, "the wall position needs t");
    if (mesh) {
        if (p->h_mode != CSPH_H_FIXED)
            return fail(CSPH_EINVAL, "a step on a given mesh takes fixed-h mode");
        if (p->check_nonphys)
            return fail(CSPH_EINVAL, "a step on a given mesh does not wait: check_nonphys must be 0");
        r = check_mesh(mesh, p->kappa * p->h);
        if (r) return r;
    }
    const bool rk2 = p->integrator == CSPH_INT_RK2;
    if (rk2 && va) return fail(CSPH_EINVAL, "csph_step_voronoi takes the Euler step only");
    if ((s_in->mat && !s_out->mat) || (s_in->id && !s_out->id) ||
        (p->h_mode == CSPH_H_PAIR && !s_out->d))
        return fail(CSPH_EINVAL, "s_out must carry mat/id/d when s_in does");
    if (p->reorder && s_in->n > 0 &&
        (s_in->x == s_out->x || s_in->vx == s_out->vx || s_in->rho == s_out->rho ||
         s_in->E == s_out->E || s_in->m == s_out->m))
        return fail(CSPH_EINVAL, "reorder = 1 needs s_out distinct from s_in");
    int64_t n = s_in->n;
    const Axes ax = kernel_axes(p);
    const csph_state vin = kernel_view(*s_in, ax), vout = kernel_view(*s_out, ax);
    csph_grid g;
    double dmax = 0.0, ymin = 0.0;
    if (mesh) {  // the caller's mesh, in the kernels' axes
        g = *mesh;
        for (int a = 0; a < 3; ++a) {
            g.origin[a] = mesh->origin[ax.k[a]];
            g.dims[a] = mesh->dims[ax.k[a]];
        }
    } else {
        r = make_grid(vin.x, vin.y, vin.z, vin.d, n, p, ws, ws_bytes, st, &g, &dmax, &ymin, true,
                      prof);
        if (r) return r;
    }
    r = need_ws(ws_bytes, n, g.ncell, ws_needed, rk2);
    if (r) return r;
    Ws w;
    ws_layout(&w, ws, n, g.ncell, rk2);
    // the Euler step in cell order writes the neighbour counts where the caller wants them
    // (the output order is the rate kernel's), instead of copying them there at the end
    if (p->reorder && !rk2 && nbr_count) w.cnt = nbr_count;
    GridDev gd = grid_dev(g, true, ymin);
    // on a given mesh the binning finds the wall band's minimum y on the device and counts the
    // particles off the mesh (or outside a periodic box)
    BinCheck chk{nullptr, nullptr, 0, {0, 0, 0}, {0, 0, 0}};
    if (mesh) {
        if (p->wall) chk.yenc = w.yenc;
        chk.outside = (unsigned long long *)outside;
        gd.yenc = chk.yenc;
    }
    PairConst pc = pair_const(p, dmax);
    chk.per = mesh ? pc.per : 0;
    for (int a = 0; a < 3; ++a) {
        chk.lo[a] = pc.lo[a];
        chk.hi[a] = pc.hi[a];
    }
    EosDev eos = eos_dev(p);
    int mixed = p->precision == CSPH_MIXED;
    bool pair = p->h_mode == CSPH_H_PAIR;
    double *dst[9];
    int32_t *dmat;
    double *dd;
    int64_t *did;
    if (p->reorder) {
        double *o[9] = {vout.x, vout.y, vout.z, vout.vx, vout.vy, vout.vz,
                        vout.rho, vout.E, vout.m};
        for (int k = 0; k < 9; ++k) dst[k] = o[k];
        dmat = vout.mat;
        dd = pair ? vout.d : nullptr;
        did = vout.id;
    } else {
        for (int k = 0; k < 9; ++k) dst[k] = w.srt[k];
        dmat = w.srt_mat;
        dd = pair ? w.srt_d : nullptr;
        did = vin.id ? w.srt_id : nullptr;
    }
    // dt = cfl * min h/s (an empty set takes dt = 0); the pack clears the Z flag
    CSPH_HIP(launch_fill_u64(w.dtmin, n > 0 ? 0x7ff0000000000000ull : 0ull, 2, st));
    // checked: the pack counts into the workspace, read back at the end
    const bool check = p->check_nonphys != 0;
    if (check) CSPH_HIP(launch_fill_u64((unsigned long long *)w.nonphys, 0ull, 1, st));
    if (n > 0) {
        {
            ProfScope pr(CSPH_PROF_BIN, st, prof);
            if (chk.yenc) CSPH_HIP(launch_fill_u64(chk.yenc, ~0ull, 1, st));
            CSPH_HIP(launch_bin(vin.x, vin.y, vin.z, n, gd, w, w.perm, nullptr, w.cs, st,
                                mesh ? &chk : nullptr));
        }
        ProfScope pr(CSPH_PROF_PACK, st, prof);
        CSPH_HIP(launch_pack(vin, n, w.perm, eos, mixed, gd, w, dst, dmat, dd, did, vin.id,
                             check ? w.nonphys : nonphys, st));
    }
    if (n > 0) {
        ProfScope pr(CSPH_PROF_RATES, st, prof);
        CSPH_HIP(launch_rates(n, mixed, gd, pc, w, dst, dd, t, 0.0, p->cfl > 0.0, st));
    }
    const int32_t *cnt_out = w.cnt;  // the neighbour counts of U (in the first stage's order)
    if (rk2 && n > 0) {
        {
            ProfScope pr(CSPH_PROF_INTEGRATE, st, prof);
            CSPH_HIP(launch_rk2_predict(n, dst, w, p->cfl, dt_in, pc, t, st));
        }
        cnt_out = w.rk_cnt;
        // second evaluation, at U1: its own mesh, order and records
        double *d1 = pair ? dd : nullptr;
        csph_grid g2 = g;  // on a given mesh, the same mesh (no synchronisation)
        double dmax2 = dmax, ymin2 = ymin;
        if (!mesh) {
            r = make_grid(w.stg[0], w.stg[1], w.stg[2], d1, n, p, ws, ws_bytes, st, &g2, &dmax2,
                          &ymin2, true, prof);
            if (r) return r;
        }
        r = need_ws(ws_bytes, n, g.ncell, ws_needed, true, g2.ncell);
        if (r) return r;
        ws_layout(&w, ws, n, g.ncell, true, g2.ncell);
        Ws w2 = w;
        w2.cs = w.cs2;
        w2.scan_tmp = w.scan_tmp2;
        GridDev gd2 = grid_dev(g2, true, ymin2);
        gd2.yenc = gd.yenc;  // found again from U1 by the second binning
        BinCheck chk2 = chk;
        chk2.outside = nullptr;  // counted at U only
        PairConst pc2 = pair_const(p, dmax2);
        csph_state u1{n,       w.stg[0], w.stg[1], w.stg[2], w.stg[3], w.stg[4], w.stg[5],
                      w.stg[6], w.stg[7], dst[8],   dmat,     d1,       nullptr};
        {
            ProfScope pr(CSPH_PROF_BIN, st, prof);
            if (chk2.yenc) CSPH_HIP(launch_fill_u64(chk2.yenc, ~0ull, 1, st));
            CSPH_HIP(launch_bin(u1.x, u1.y, u1.z, n, gd2, w2, w.perm2, nullptr, w.cs2, st,
                                mesh ? &chk2 : nullptr));
        }
        {
            ProfScope pr(CSPH_PROF_PACK, st, prof);
            CSPH_HIP(launch_fill_u64(w.zflag, 0x7ff0000000000000ull, 1, st));
            CSPH_HIP(launch_pack(u1, n, w.perm2, eos, mixed, gd2, w2, w.srt2, nullptr,
                                 pair ? w.srt2_d : nullptr, nullptr, nullptr,
                                 check ? w.nonphys : nonphys, st));
        }
        {
            ProfScope pr(CSPH_PROF_RATES, st, prof);
            CSPH_HIP(launch_rates(n, mixed, gd2, pc2, w2, w.srt2, pair ? w.srt2_d : nullptr,
                                  w.t2, 0.0, 0, st));
        }
        ProfScope pr(CSPH_PROF_INTEGRATE, st, prof);
        CSPH_HIP(launch_rk2_combine(n, dst, w, p->cfl, dt_in, pc, t, st));
        CSPH_HIP(launch_finish_step(n, w, p->cfl, dt_in, t, dt_used, totals, ax.k, st));
    } else {
        ProfScope pr(CSPH_PROF_INTEGRATE, st, prof);
        VoroDev vd{};
        if (va) {
            vd.sites = va->sites;
            vd.K = va->K;
            for (int a = 0; a < 3; ++a) vd.ax[a] = ax.k[a];
            vd.owner = va->owner;
            vd.owner_at = p->reorder ? nullptr : w.perm;  // the output order
            vd.cnt = w.cnt;
            vd.site_part = (unsigned long long *)va->site_particles;
            vd.site_pairs = (unsigned long long *)va->site_pairs;
        }
        // n = 0 writes zero partials
        CSPH_HIP(launch_integrate(n, dst, w, p->cfl, dt_in, pc, t, st, va ? &vd : nullptr));
        CSPH_HIP(launch_finish_step(n, w, p->cfl, dt_in, t, dt_used, totals, ax.k, st));
    }
    ProfScope pro(CSPH_PROF_REORDER, st, prof);
    if (n > 0) {
        if (p->reorder) {
            if (nbr_count && cnt_out != nbr_count)
                CSPH_HIP(hipMemcpyAsync(nbr_count, cnt_out, sizeof(int32_t) * n,
                                        hipMemcpyDeviceToDevice, st));
        } else {
            csph_state o = vout;
            if (!pair) o.d = nullptr;
            CSPH_HIP(launch_unpermute(n, w.perm, w.srt, vin.mat ? w.srt_mat : nullptr, dd,
                                      did, cnt_out, o, nbr_count, st));
        }
    }
    pro.stop();
    return check ? finish_nonphys(w, nonphys, st) : CSPH_OK;
}

}  // namespace csph

extern "C" {


csph_status csph_vlist_build(const csph_state *s_in, csph_state *s_out, const csph_params *p,
                             const double *t, double beta, int32_t cap, int32_t *vl_count,
                             int32_t *vl_idx, double *x_ref, csph_vlist_ctl *ctl,
                             int32_t *max_count, void *ws, size_t ws_bytes, size_t *ws_needed,
                             csph_stream stream) {
    g_err[0] = 0;
    if (!state_ok(s_in) || !state_ok(s_out) || s_in->n != s_out->n || s_in->n >= INT32_MAX)
        return fail(CSPH_EINVAL, "bad state");
    if (s_in->n >= kMaxPairN) return fail(CSPH_EINVAL, "n >= 2^27 particles");
    csph_status r = check_params(p, false, nullptr);
    if (r) return r;
    if (p->h_mode != CSPH_H_FIXED) return fail(CSPH_EINVAL, "Verlet lists need fixed-h mode");
    if (p->periodic) return fail(CSPH_EINVAL, "Verlet lists do not support periodic boundaries");
    if (!(beta >= 0.0) || !std::isfinite(beta)) return fail(CSPH_EINVAL, "beta must be >= 0");
    if (cap < kVlChunk || cap % kVlChunk)
        return fail(CSPH_EINVAL, "cap must be a positive multiple of %d", kVlChunk);
    const int64_t n = s_in->n;
    if (n > 0 && (!vl_count || !vl_idx || !x_ref))
        return fail(CSPH_EINVAL, "vl_count, vl_idx and x_ref are required");
    if (((uintptr_t)vl_idx & 15) != 0) return fail(CSPH_EINVAL, "vl_idx must be 16-byte aligned");
    if (((uintptr_t)ctl & 7) != 0) return fail(CSPH_EINVAL, "ctl must be 8-byte aligned");
    if (n > 0 && (s_in->x == s_out->x || s_in->vx == s_out->vx || s_in->rho == s_out->rho ||
                  s_in->E == s_out->E || s_in->m == s_out->m))
        return fail(CSPH_EINVAL, "s_out must be distinct from s_in");
    if ((s_in->mat && !s_out->mat) || (s_in->id && !s_out->id))
        return fail(CSPH_EINVAL, "s_out must carry mat/id when s_in does");
    if (p->wall && !t) return fail(CSPH_EINVAL, "the wall position needs t");
    hipStream_t st = (hipStream_t)stream;
    // the mesh must reach the horizon (1 + beta) H
    csph_params ph = *p;
    ph.kappa = p->kappa * (1.0 + beta);
    csph_grid g;
    double dmax, ymin;
    const Axes ax = kernel_axes(p);
    const csph_state vin = kernel_view(*s_in, ax), vout = kernel_view(*s_out, ax);
    r = make_grid(vin.x, vin.y, vin.z, nullptr, n, &ph, ws, ws_bytes, st, &g, &dmax, &ymin, true);
    if (r) return r;
    r = need_ws(ws_bytes, n, g.ncell, ws_needed);
    if (r) return r;
    if (max_count) *max_count = 0;
    const double H = p->kappa * p->h;
    if (ctl)
        CSPH_HIP(launch_vl_init(ctl, t, beta * H, p->wall ? 2.0 * std::fabs(p->wall_v) : 0.0, st));
    if (n == 0) return CSPH_OK;
    Ws w;
    ws_layout(&w, ws, n, g.ncell);
    GridDev gd = grid_dev(g, true, ymin);
    EosDev eos = eos_dev(p);
    double *o[9] = {vout.x, vout.y, vout.z, vout.vx, vout.vy, vout.vz,
                    vout.rho, vout.E, vout.m};
    double twall = 0.0;
    if (p->wall) CSPH_HIP(hipMemcpyAsync(&twall, t, sizeof(double), hipMemcpyDeviceToHost, st));
    {
        ProfScope pr(CSPH_PROF_BIN, st);
        CSPH_HIP(launch_bin(vin.x, vin.y, vin.z, n, gd, w, w.perm, nullptr, w.cs, st));
        CSPH_HIP(launch_pack(vin, n, w.perm, eos, 0, gd, w, o, s_out->mat,
                             s_out->d && s_in->d ? s_out->d : nullptr, s_out->id, s_in->id,
                             nullptr, st));
    }
    CSPH_HIP(hipStreamSynchronize(st));  // twall
    const double R = (1.0 + beta) * H;
    const double yw = p->wall ? p->wall_x0 + p->wall_v * twall : 0.0;  // along the kernels' y
    unsigned long long over = 0;
    {
        ProfScope pr(CSPH_PROF_NEIGHBORS, st);
        CSPH_HIP(launch_fill_u64((unsigned long long *)w.nonphys, 0ull, 1, st));
        CSPH_HIP(launch_vlist(n, (const double4 *)w.recA, w.cs, gd, R, p->wall, yw, cap,
                              vl_count, vl_idx, (unsigned long long *)w.nonphys, st));
        const double *ref[3] = {s_out->x, s_out->y, s_out->z};  // the caller's axes
        for (int a = 0; a < 3; ++a)
            CSPH_HIP(hipMemcpyAsync(x_ref + a * n, ref[a], sizeof(double) * n,
                                    hipMemcpyDeviceToDevice, st));
        CSPH_HIP(hipMemcpyAsync(&over, w.nonphys, sizeof(over), hipMemcpyDeviceToHost, st));
    }
    CSPH_HIP(hipStreamSynchronize(st));
    if (max_count) *max_count = (int32_t)(over > (unsigned long long)cap ? over : 0);
    if (over > (unsigned long long)cap)
        return fail(CSPH_ECAPACITY, "a Verlet list holds %llu partners, cap is %d", over, cap);
    return CSPH_OK;
}

csph_status csph_step_vlist(csph_state *s, const csph_params *p, double *t, double dt_in,
                            double *dt_used, double *totals, int32_t *nbr_count,
                            int64_t *nonphys, const int32_t *vl_count, const int32_t *vl_idx,
                            int32_t cap, const double *x_ref, csph_vlist_ctl *ctl, void *ws,
                            size_t ws_bytes, size_t *ws_needed, csph_stream stream) {
    g_err[0] = 0;
    if (!state_ok(s) || s->n >= INT32_MAX) return fail(CSPH_EINVAL, "bad state");
    if (s->n >= kMaxPairN) return fail(CSPH_EINVAL, "n >= 2^27 particles");
    csph_status r = check_params(p, false, nullptr);
    if (r) return r;
    if (p->h_mode != CSPH_H_FIXED) return fail(CSPH_EINVAL, "Verlet lists need fixed-h mode");
    if (p->periodic) return fail(CSPH_EINVAL, "Verlet lists do not support periodic boundaries");
    if (p->integrator != CSPH_INT_EULER)
        return fail(CSPH_EINVAL, "Verlet-list steps take the Euler step only");
    if (!(p->cfl > 0.0) && !(std::isfinite(dt_in) && dt_in >= 0.0))
        return fail(CSPH_EINVAL, "cfl <= 0 needs a finite dt_in >= 0");
    if (p->wall && !t) return fail(CSPH_EINVAL, "the wall position needs t");
    const int64_t n = s->n;
    if (n > 0 && (!vl_count || !vl_idx || !x_ref || cap < kVlChunk || cap % kVlChunk))
        return fail(CSPH_EINVAL, "vl_count, vl_idx, x_ref and cap (a multiple of %d) are required",
                    kVlChunk);
    if (!ctl || ((uintptr_t)ctl & 7) != 0)
        return fail(CSPH_EINVAL, "ctl (the lists' control block, 8-byte aligned) is required");
    hipStream_t st = (hipStream_t)stream;
    r = need_ws(ws_bytes, n, 1, ws_needed);
    if (r) return r;
    Ws w;
    ws_layout(&w, ws, n, 1);
    GridDev gd;
    memset(&gd, 0, sizeof(gd));  // no mesh: the lists name the partners
    PairConst pc = pair_const(p, 0.0);
    EosDev eos = eos_dev(p);
    const int mixed = p->precision == CSPH_MIXED;
    const Axes ax = kernel_axes(p);
    const csph_state sv = kernel_view(*s, ax);
    double *cur[9] = {sv.x, sv.y, sv.z, sv.vx, sv.vy, sv.vz, sv.rho, sv.E, sv.m};
    // the lists' exactness bound, checked on the device; every kernel below does nothing once
    // the lists are stale
    CSPH_HIP(launch_vl_guard(ctl, t, st));
    const int32_t *gate = &ctl->valid;
    const ListGate lg{gate, w.cnt, (unsigned long long *)&ctl->pairs, &ctl->steps};
    // dt = cfl * min h/s (an empty set takes dt = 0); the pack clears the Z flag
    CSPH_HIP(launch_fill_u64(w.dtmin, n > 0 ? 0x7ff0000000000000ull : 0ull, 2, st));
    if (n > 0) {
        ProfScope pr(CSPH_PROF_PACK, st);
        CSPH_HIP(launch_pack(sv, n, nullptr, eos, mixed, gd, w, nullptr, nullptr, nullptr,
                             nullptr, nullptr, nonphys, st, gate));
    }
    if (n > 0) {
        ProfScope pr(CSPH_PROF_RATES, st);
        CSPH_HIP(launch_rates(n, mixed, gd, pc, w, cur, nullptr, t, 0.0, p->cfl > 0.0, st,
                              vl_count, vl_idx, cap, gate));
    }
    {
        ProfScope pr(CSPH_PROF_INTEGRATE, st);
        CSPH_HIP(launch_integrate(n, cur, w, p->cfl, dt_in, pc, t, st, nullptr, &lg));
        CSPH_HIP(launch_finish_step(n, w, p->cfl, dt_in, t, dt_used, totals, ax.k, st, &lg));
        CSPH_HIP(launch_disp(n, s->x, s->y, s->z, x_ref, (unsigned long long *)&ctl->disp, st,
                             gate));
    }
    if (n > 0 && nbr_count) CSPH_HIP(launch_copy_i32(nbr_count, w.cnt, n, gate, st));
    return CSPH_OK;
}

csph_status voronoi_assign(const double *x, const double *y, const double *z, int64_t n,
                           const double *sites, int32_t K, const int32_t *nbr_count,
                           int32_t *owner, int64_t *site_particles, int64_t *site_pairs,
                           csph_stream stream) {
    g_err[0] = 0;
    if (n < 0 || K < 1 || K > kMaxSites || !sites || !site_particles ||
        (n > 0 && (!x || !y || !z || !owner)))
        return fail(CSPH_EINVAL, "bad arguments (1 <= K <= %d)", kMaxSites);
    if (site_pairs && !nbr_count) return fail(CSPH_EINVAL, "site_pairs needs nbr_count");
    ProfScope pr(CSPH_PROF_VORONOI, (hipStream_t)stream);
    CSPH_HIP(launch_voronoi(x, y, z, n, sites, K, nbr_count, owner, site_particles, site_pairs,
                            (hipStream_t)stream));
    return CSPH_OK;
}

size_t csph_balance_workspace_size(int32_t K) {
    return K < 1 ? 0 : balance_ws_bytes(K);
}

csph_status csph_balance_stats(const double *x, const double *y, const double *z, int64_t n,
                               const int32_t *owner, const int32_t *nbr_count,
                               const double *sites, int32_t K, double dsh,
                               int64_t *site_particles, int64_t *site_pairs, double *centre,
                               uint32_t *adjacency, void *ws, size_t ws_bytes, size_t *ws_needed,
                               csph_stream stream) {
    g_err[0] = 0;
    if (n < 0 || K < 1 || K > kMaxBalanceSites || !sites || !site_particles || !centre ||
        !adjacency || (n > 0 && (!x || !y || !z || !owner)))
        return fail(CSPH_EINVAL, "bad arguments (1 <= K <= %d)", kMaxBalanceSites);
    if (site_pairs && !nbr_count) return fail(CSPH_EINVAL, "site_pairs needs nbr_count");
    if (!(dsh >= 0.0) || !std::isfinite(dsh)) return fail(CSPH_EINVAL, "dsh must be finite and >= 0");
    const size_t need = balance_ws_bytes(K);
    if (ws_needed) *ws_needed = need;
    if (!ws || ws_bytes < need) return fail(CSPH_ECAPACITY, "workspace needs %zu bytes", need);
    ProfScope pr(CSPH_PROF_BALANCE, (hipStream_t)stream);
    CSPH_HIP(launch_balance_stats(x, y, z, n, owner, site_pairs ? nbr_count : nullptr, sites, K,
                                  dsh, site_particles, site_pairs, centre, adjacency, ws,
                                  (hipStream_t)stream));
    return CSPH_OK;
}

csph_status csph_balance_move(const double *sites, int32_t K, const int64_t *loads,
                              const double *centre, const uint32_t *adjacency,
                              const csph_balance_params *bp, double *sites_out, double *move_sum,
                              csph_stream stream) {
    g_err[0] = 0;
    if (K < 1 || K > kMaxBalanceSites || !sites || !loads || !centre || !adjacency || !bp ||
        !sites_out || !move_sum)
        return fail(CSPH_EINVAL, "bad arguments (1 <= K <= %d)", kMaxBalanceSites);
    if (sites_out == sites) return fail(CSPH_EINVAL, "sites_out must not alias sites");
    const double v[4] = {bp->sigma, bp->theta, bp->gamma, bp->dsh};
    for (double a : v)
        if (!std::isfinite(a)) return fail(CSPH_EINVAL, "balance parameters must be finite");
    if (bp->dsh < 0.0) return fail(CSPH_EINVAL, "dsh must be >= 0");
    ProfScope pr(CSPH_PROF_BALANCE, (hipStream_t)stream);
    CSPH_HIP(launch_balance_move(sites, K, loads, centre, adjacency, bp->sigma, bp->theta,
                                 bp->gamma, bp->dsh, sites_out, move_sum, (hipStream_t)stream));
    return CSPH_OK;
}

csph_status csph_init_energy(const double *rho, const double *pres, const double *vx,
                             const double *vy, const double *vz, const int32_t *mat, int64_t n,
                             const csph_params *p, double *E, csph_stream stream) {
    g_err[0] = 0;
    if (n < 0 || (n > 0 && (!rho || !pres || !vx || !vy || !vz || !E)))
        return fail(CSPH_EINVAL, "bad arguments");
    csph_status r = check_params(p, false, nullptr);
    if (r) return r;
    CSPH_HIP(launch_init_energy(rho, pres, vx, vy, vz, mat, n, eos_dev(p), E, (hipStream_t)stream));
    return CSPH_OK;
}

static bool grad_ok(const csph_grad &g) {
    return g.x && g.y && g.z && g.vx && g.vy && g.vz && g.rho && g.E;
}

// A gradient struct in the kernels' axes (kernel_axes).
static csph_grad kernel_view(const csph_grad &gr, const Axes &ax) {
    csph_grad v = gr;
    double *const pos[3] = {gr.x, gr.y, gr.z}, *const vel[3] = {gr.vx, gr.vy, gr.vz};
    v.x = pos[ax.k[0]];
    v.y = pos[ax.k[1]];
    v.z = pos[ax.k[2]];
    v.vx = vel[ax.k[0]];
    v.vy = vel[ax.k[1]];
    v.vz = vel[ax.k[2]];
    return v;
}

// shared body of csph_rates_vjp / csph_step_vjp / csph_step_vjp_cfl (t: the time of the
// rates; cfl_dt: the step's dt is the CFL rule's, recomputed here and differentiated)
static csph_status vjp_common(const csph_state *s_in, const csph_params *p, double t,
                              const double *const a_in[5], const csph_grad *gnext_in, double dt,
                              csph_grad gout_in, int accumulate, double *g_eos, void *ws,
                              size_t ws_bytes, size_t *ws_needed, hipStream_t st,
                              bool cfl_dt = false, double *dt_used = nullptr) {
    const csph_state *s = s_in;
    if (!state_ok(s) || s->n >= INT32_MAX) return fail(CSPH_EINVAL, "bad state");
    if (s->n >= kMaxPairN) return fail(CSPH_EINVAL, "n >= 2^27 particles");
    csph_status r = check_params(p, s->n > 0, s->d);
    if (r) return r;
    int64_t n = s->n;
    if (n > 0 && !grad_ok(gout_in)) return fail(CSPH_EINVAL, "gradient outputs must not be NULL");
    if (!std::isfinite(t)) return fail(CSPH_EINVAL, "t not finite");
    // the kernels' axes: the state, the rate cotangents and the gradients swapped alike
    const Axes ax = kernel_axes(p);
    const csph_state sv = kernel_view(*s_in, ax);
    s = &sv;
    const csph_grad gout = kernel_view(gout_in, ax);
    csph_grad gnv;
    const csph_grad *gnext = nullptr;
    if (gnext_in) {
        gnv = kernel_view(*gnext_in, ax);
        gnext = &gnv;
    }
    const double *a[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    if (a_in) {
        const double *const av[3] = {a_in[1], a_in[2], a_in[3]};
        a[0] = a_in[0];
        a[1] = av[ax.k[0]];
        a[2] = av[ax.k[1]];
        a[3] = av[ax.k[2]];
        a[4] = a_in[4];
    }
    csph_grid g;
    double dmax, ymin;
    const bool pair = p->h_mode == CSPH_H_PAIR;
    r = make_grid(s->x, s->y, s->z, pair ? s->d : nullptr, n, p, ws, ws_bytes, st, &g, &dmax,
                  &ymin, true);
    if (r) return r;
    r = need_ws(ws_bytes, n, g.ncell, ws_needed);
    if (r) return r;
    if (n == 0) return CSPH_OK;
    Ws w;
    ws_layout(&w, ws, n, g.ncell);
    GridDev gd = grid_dev(g, true, ymin);
    PairConst pc = pair_const(p, dmax);
    EosDev eos = eos_dev(p);
    ProfScope pr(CSPH_PROF_ADJOINT, st);
    double *const dsrt = pair ? w.srt_d : nullptr;  // pair-h mode: the sizes in cell order
    // dt minimum and Z flag (the pack clears the flag where an impedance is zero)
    CSPH_HIP(launch_fill_u64(w.dtmin, 0x7ff0000000000000ull, 2, st));
    CSPH_HIP(launch_bin(s->x, s->y, s->z, n, gd, w, w.perm, nullptr, w.cs, st));
    CSPH_HIP(launch_pack(*s, n, w.perm, eos, 0, gd, w, w.srt, w.srt_mat, dsrt, nullptr,
                         nullptr, nullptr, st));
    double *go[8] = {gout.x, gout.y, gout.z, gout.vx, gout.vy, gout.vz, gout.rho, gout.E};
    const double *gn[8];
    if (gnext) {
        const double *tn[8] = {gnext->x, gnext->y, gnext->z, gnext->vx, gnext->vy, gnext->vz,
                               gnext->rho, gnext->E};
        for (int k = 0; k < 8; ++k) gn[k] = tn[k];
    }
    const bool wall = p->wall != 0;
    const double yw = wall ? p->wall_x0 + p->wall_v * t : 0.0;
    if (wall && gnext && !cfl_dt) {
        // the step's reflections, found from each particle's own rate sums that the gathers
        // form (first pass, the cotangent as given), then the gather of the change the
        // reflection's transpose makes to the flagged particles' cotangents, over the wall
        // band only
        const double yw1 = p->wall_x0 + p->wall_v * (t + dt);
        int32_t *flag = w.bin_tmp;             // free after the binning
        unsigned long long *reach = w.yenc;    // unused without a caller's mesh
        // the change a reflection would make, formed before the first pass writes g (which
        // may alias the cotangent), in the FP32 candidate records the adjoint does not read;
        // the signal-speed array (no rate evaluation here) takes the rate sums, then zeros
        double *dy = (double *)w.recF, *dvy = dy + n, *svy = w.sig;
        CSPH_HIP(launch_reflect_delta(n, gn[1], gn[4], gn[7], p->wall_v, dy, dvy, st));
        CSPH_HIP(launch_fill_u64(reach, 0ull, 1, st));
        CSPH_HIP(launch_vjp_wall(n, w.perm, w.cs, gd, pc, eos, w, w.srt, w.srt_mat, nullptr, go,
                                 gn, dt, 0, g_eos, dsrt, yw, p->wall_v,
                                 WallPass{svy, nullptr}, st));
        CSPH_HIP(launch_wall_flags(n, w.perm, w.srt, svy, dt, yw1, yw, flag, reach, st));
        // kept for the flagged particles; zeros for the other fields
        CSPH_HIP(launch_keep_flagged(n, flag, dy, dvy, st));
        CSPH_HIP(launch_fill_u64((unsigned long long *)svy, 0ull, n, st));
        const double *zero = svy;
        const double *dn[8] = {zero, dy, zero, zero, dvy, zero, zero, zero};
        CSPH_HIP(launch_vjp_wall(n, w.perm, w.cs, gd, pc, eos, w, w.srt, w.srt_mat, nullptr, go,
                                 dn, dt, 1, g_eos, dsrt, yw, p->wall_v,
                                 WallPass{nullptr, reach}, st));
        return CSPH_OK;
    }
    // the CFL step's FP64 rates at t: its signal speeds, dt and (with the piston) reflections
    if (gnext && cfl_dt)
        CSPH_HIP(launch_rates(n, 0, gd, pc, w, w.srt, dsrt, nullptr, t, 1, st));
    DtInfo *info = nullptr;
    if (cfl_dt) {
        unsigned long long bits = 0;
        r = word_to_host(w.dtmin, &bits, st);
        if (r) return r;
        double tau;
        memcpy(&tau, &bits, sizeof(tau));
        dt = p->cfl * tau;
        if (!(dt > 0.0) || !std::isfinite(dt))
            return fail(CSPH_EINVAL, "the CFL time step of this state is %g (not finite and > 0)",
                        dt);
        if (dt_used) *dt_used = dt;
        // the binding slot and J's cotangent of dt (from the next state's cotangent as given,
        // before the reflection's transpose below)
        info = (DtInfo *)w.tot_part;
        CSPH_HIP(launch_fill_u64(&info->arg, ~0ull, 1, st));
        CSPH_HIP(launch_dt_adjoint(n, w.perm, w.srt, w, dsrt, p->h, gn, dt, wall,
                                   p->wall_x0 + p->wall_v * (t + dt), p->wall_v, info, st));
    }
    if (wall && gnext) {
        // (the CFL step) the cotangents of the pre-reflection y and v_y go to the FP32
        // candidate records, which only the rate evaluation above reads (2 n + 4 doubles)
        double *gy = (double *)w.recF, *gvy = gy + n;
        const double yw1 = p->wall_x0 + p->wall_v * (t + dt);
        CSPH_HIP(launch_vjp_reflect(n, w.perm, w.srt[1], w.srt[4], w.rate[2], dt, yw1, p->wall_v,
                                    gn[1], gn[4], gn[7], gy, gvy, st));
        gn[1] = gy;
        gn[4] = gvy;
    }
    const DtAdj da{info, p->cfl};
    CSPH_HIP(launch_vjp(n, w.perm, w.cs, gd, pc, eos, w, w.srt, w.srt_mat, a, go,
                        gnext ? gn : nullptr, dt, accumulate, g_eos, dsrt, wall, yw, p->wall_v,
                        st, cfl_dt ? &da : nullptr));
    return CSPH_OK;
}

csph_status csph_rates_vjp(const csph_state *s, const csph_params *p, double t,
                           csph_rates_out a, csph_grad g_state, double *g_eos, void *ws,
                           size_t ws_bytes, size_t *ws_needed, csph_stream stream) {
    g_err[0] = 0;
    if (s && s->n > 0 && (!a.drho || !a.dvx || !a.dvy || !a.dvz || !a.dE))
        return fail(CSPH_EINVAL, "rate cotangents must not be NULL");
    const double *ai[5] = {a.drho, a.dvx, a.dvy, a.dvz, a.dE};
    return vjp_common(s, p, t, ai, nullptr, 0.0, g_state, 1, g_eos, ws, ws_bytes, ws_needed,
                      (hipStream_t)stream);
}

// The RK2 step's VJP (dt fixed), composed of the two evaluations' rate VJPs and the
// elementwise parts of launch_rk2_vjp_stage2/1 (whose comment gives the algebra): a forward
// FP64 rate evaluation at U gives U1; the rate VJP at U1 (time t + dt) completes g_U1; the one
// at U (time t) completes g_U.  Scratch arrays take the workspace's first 28 n doubles; the
// rate calls lay theirs out after them.
static csph_status step_vjp_rk2(const csph_state *s, const csph_params *p, double t, double dt,
                                csph_grad gn, csph_grad gp, double *g_eos, void *ws,
                                size_t ws_bytes, size_t *ws_needed, hipStream_t st) {
    if (!state_ok(s) || s->n >= INT32_MAX) return fail(CSPH_EINVAL, "bad state");
    csph_status r = check_params(p, s->n > 0, s->d);
    if (r) return r;
    const int64_t n = s->n;
    if (n > 0 && (!grad_ok(gp) || !grad_ok(gn)))
        return fail(CSPH_EINVAL, "gradient arrays must not be NULL");
    if (!std::isfinite(t)) return fail(CSPH_EINVAL, "t not finite");
    const size_t arr = align256(sizeof(double) * (size_t)(n > 0 ? n : 1));
    const size_t off = 28 * arr;
    if (ws_bytes < off) {
        const size_t need = off + ws_layout(nullptr, nullptr, n, 1);
        if (ws_needed) *ws_needed = need;
        return fail(CSPH_ECAPACITY, "workspace needs at least %zu bytes, got %zu", need, ws_bytes);
    }
    if (n == 0) {
        if (ws_needed) *ws_needed = off;
        return CSPH_OK;
    }
    char *b = (char *)ws;
    auto take = [&](int k) { return (double *)(b + (size_t)k * arr); };
    Rk2Vjp q;
    const double *sv[8] = {s->x, s->y, s->z, s->vx, s->vy, s->vz, s->rho, s->E};
    const double *gv[8] = {gn.x, gn.y, gn.z, gn.vx, gn.vy, gn.vz, gn.rho, gn.E};
    for (int k = 0; k < 8; ++k) {
        q.s[k] = sv[k];
        q.gn[k] = gv[k];
        q.u1[k] = take(k);
        q.gu1[k] = take(15 + k);
    }
    double *F[5];
    for (int k = 0; k < 5; ++k) {
        F[k] = take(8 + k);
        q.F[k] = F[k];
        q.a[k] = take(23 + k);
    }
    q.gx = take(13);
    q.gvx = take(14);
    q.dt = dt;
    q.wall = p->wall != 0;
    q.vw = p->wall_v;
    q.xw1 = p->wall_x0 + p->wall_v * (t + dt);
    q.per = p->periodic;
    for (int a = 0; a < 3; ++a) {
        q.lo[a] = p->box_lo[a];
        q.hi[a] = p->box_hi[a];
    }
    csph_params pf = *p;  // the FP64 map
    pf.precision = CSPH_FP64;
    pf.integrator = CSPH_INT_EULER;
    void *wr = b + off;
    const size_t wrb = ws_bytes - off;
    size_t need = 0;
    auto sized = [&](csph_status rs) {
        if (rs == CSPH_ECAPACITY && ws_needed) *ws_needed = off + need;
        return rs;
    };
    // F(U) at t
    r = csph_rates(s, &pf, t, csph_rates_out{F[0], F[1], F[2], F[3], F[4]}, nullptr, nullptr,
                   nullptr, wr, wrb, &need, st);
    if (r) return sized(r);
    CSPH_HIP(launch_rk2_vjp_stage2(n, q, st));
    // g_U1 += F(U1)^T (dt/2) g'_(rho, v, E), at t + dt with U1's wrapped positions
    const csph_state u1{n, q.u1[0], q.u1[1], q.u1[2], q.u1[3], q.u1[4], q.u1[5], q.u1[6],
                        q.u1[7], s->m, s->mat, s->d, nullptr};
    const csph_grad g1{q.gu1[0], q.gu1[1], q.gu1[2], q.gu1[3], q.gu1[4], q.gu1[5], q.gu1[6],
                       q.gu1[7]};
    const csph_rates_out a{q.a[0], q.a[1], q.a[2], q.a[3], q.a[4]};
    r = csph_rates_vjp(&u1, &pf, t + dt, a, g1, g_eos, wr, wrb, &need, st);
    if (r) return sized(r);
    double *gpv[8] = {gp.x, gp.y, gp.z, gp.vx, gp.vy, gp.vz, gp.rho, gp.E};
    CSPH_HIP(launch_rk2_vjp_stage1(n, q, gpv, st));
    // g_U += F(U)^T dt g_U1,(rho, v, E), at t
    r = csph_rates_vjp(s, &pf, t, a, gp, g_eos, wr, wrb, &need, st);
    if (r) return sized(r);
    if (ws_needed) *ws_needed = off + need;
    return CSPH_OK;
}

csph_status csph_step_vjp(const csph_state *s_n, const csph_params *p, double t, double dt,
                          csph_grad g_next, csph_grad g_prev, double *g_eos, void *ws,
                          size_t ws_bytes, size_t *ws_needed, csph_stream stream) {
    g_err[0] = 0;
    if (!std::isfinite(dt) || dt < 0.0) return fail(CSPH_EINVAL, "dt must be finite and >= 0");
    if (s_n && s_n->n > 0 && !grad_ok(g_next)) return fail(CSPH_EINVAL, "g_next has NULL arrays");
    if (p && p->integrator == CSPH_INT_RK2)
        return step_vjp_rk2(s_n, p, t, dt, g_next, g_prev, g_eos, ws, ws_bytes, ws_needed,
                            (hipStream_t)stream);
    return vjp_common(s_n, p, t, nullptr, &g_next, dt, g_prev, 0, g_eos, ws, ws_bytes,
                      ws_needed, (hipStream_t)stream);
}

csph_status csph_step_vjp_cfl(const csph_state *s_n, const csph_params *p, double t,
                              csph_grad g_next, csph_grad g_prev, double *g_eos, double *dt_used,
                              void *ws, size_t ws_bytes, size_t *ws_needed,
                              csph_stream stream) {
    g_err[0] = 0;
    if (s_n && s_n->n > 0 && !grad_ok(g_next)) return fail(CSPH_EINVAL, "g_next has NULL arrays");
    if (p && p->integrator != CSPH_INT_EULER)
        return fail(CSPH_EINVAL, "the step's adjoint is that of the Euler step only");
    if (p && !(p->cfl > 0.0))
        return fail(CSPH_EINVAL, "the CFL step's adjoint needs cfl > 0");
    if (dt_used) *dt_used = 0.0;
    return vjp_common(s_n, p, t, nullptr, &g_next, 0.0, g_prev, 0, g_eos, ws, ws_bytes,
                      ws_needed, (hipStream_t)stream, true, dt_used);
}

csph_status csph_init_energy_vjp(const double *rho, const double *pres, const double *vx,
                                 const double *vy, const double *vz, const int32_t *mat,
                                 int64_t n, const csph_params *p, const double *gE, double *g_vx,
                                 double *g_vy, double *g_vz, double *g_rho, double *g_eos,
                                 void *ws, size_t ws_bytes, size_t *ws_needed,
                                 csph_stream stream) {
    g_err[0] = 0;
    if (n < 0 || n >= INT32_MAX || (n > 0 && (!rho || !pres || !vx || !vy || !vz || !gE)))
        return fail(CSPH_EINVAL, "bad arguments");
    csph_status r = check_params(p, false, nullptr);
    if (r) return r;
    r = need_ws(ws_bytes, n, 1, ws_needed);
    if (r) return r;
    Ws w;
    ws_layout(&w, ws, n, 1);
    hipStream_t st = (hipStream_t)stream;
    ProfScope pr(CSPH_PROF_ADJOINT, st);
    CSPH_HIP(launch_init_energy_vjp(rho, pres, vx, vy, vz, mat, n, eos_dev(p), gE, g_vx, g_vy,
                                    g_vz, g_rho, g_eos, w.eos_part, st));
    return CSPH_OK;
}

csph_status csph_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    // create the events up front: first-use creation costs milliseconds
    while (g_prof_on && g_prof_pool.size() < 256) {
        hipEvent_t e = nullptr;
        if (prof_event_create(&e) != hipSuccess) return fail(CSPH_EDEVICE, "hipEventCreate failed");
        g_prof_pool.push_back(e);
    }
    return CSPH_OK;
}

csph_status csph_profile_groups(uint32_t mask) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_mask = mask;
    return CSPH_OK;
}

csph_status csph_profile_read(csph_profile *out) {
    g_err[0] = 0;
    std::vector<ProfRec> pend;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        pend.swap(g_prof_pending);
    }
    csph_status rc = CSPH_OK;
    for (const ProfRec &r : pend) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            rc = fail(CSPH_EDEVICE, "event timing failed");
        g_prof_acc.launches[r.group] += 1;
        g_prof_acc.ms[r.group] += ms;
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (const ProfRec &r : pend) {
        g_prof_pool.push_back(r.a);
        g_prof_pool.push_back(r.b);
    }
    if (out) *out = g_prof_acc;
    memset(&g_prof_acc, 0, sizeof(g_prof_acc));
    return rc;
}

}  // extern "C"
