/*
 * csph.h - C ABI of the MI355X (gfx950) contact-SPH hot-path library.
 *
 * The library computes the per-step particle interaction of the contact SPH
 * (CSPH) method of Egorova, Dyachkov, Parshikov & Zhakhovsky,
 * arXiv 1805.05128:
 *   - uniform cubic mesh binning and cell-ordered numbering (sec. 4.2,
 *     eq. Dcell and the linked-list cells / renumbering paragraphs);
 *   - neighbour sets inside the finite support radius (sec. 4.1);
 *   - the pairwise Riemann-solver rates of eqs. SPH:Conti, SPH:Pulse and
 *     SPH:Energy with the Wendland C2 kernel (sec. 4.1);
 *   - the state update and global time step (Algorithm 1, "renew particle
 *     positions and states and make global synchronization of SPH time
 *     step");
 *   - Voronoi ownership (eq. VoronoiDefinition, ties to the smaller index,
 *     sec. 3.1) and per-subdomain load counts;
 *   - hand-written adjoints (vector-Jacobian products) of the rates and of
 *     the step.
 *
 * Conventions shared by every entry point
 *   Pointers.   Array arguments are DEVICE pointers owned by the caller unless
 *               a comment says "host".  The library never allocates device
 *               memory: scratch comes from a caller-provided workspace
 *               (ws, ws_bytes).  When the workspace is too small the call
 *               returns CSPH_ECAPACITY and, if ws_needed is not NULL, writes
 *               the required size there (host).  Workspace contents do not
 *               persist between calls.
 *   Layout.     Structure of arrays, FP64, one entry per particle, particle
 *               count n < 2^31; particle indices are int32.  The calls that
 *               walk particle pairs (csph_rates, csph_step, csph_vlist_build,
 *               csph_step_vlist and the vector-Jacobian products) take
 *               n < 2^27 and return CSPH_EINVAL above: their kernels address
 *               per-particle records of up to 32 bytes with 32-bit offsets.
 *   Streams.    Work is enqueued on `stream` (a hipStream_t; NULL = default
 *               stream).  Calls that must learn a size on the host (mesh
 *               dimensions, neighbour count) wait for that stream; the
 *               others return as soon as the work is enqueued.  The mesh
 *               bounds (and the CFL step's minimum in its VJP) reach the
 *               host through a small pinned buffer per host thread and
 *               device, allocated on first use and held until the process
 *               ends, which the host polls (csph_step_static copies and
 *               synchronises instead).
 *   Errors.     Every call returns a csph_status.  CSPH_EINVAL: a bad
 *               argument (NULL where required, n < 0, bad parameters);
 *               CSPH_ECAPACITY: an output or workspace is too small;
 *               CSPH_EDEVICE: a HIP runtime error.  Nothing is written on
 *               EINVAL.  csph_last_error() returns a thread-local message.
 *               Non-physical states (negative or NaN squared sound speed,
 *               Mie-Grueneisen compression past its Hugoniot's limit) are
 *               counted on the device and never trapped: the particle's
 *               sound speed is taken as 0 and every output is written.
 *               csph_rates, and csph_step with params.check_nonphys = 1,
 *               then return CSPH_ENONPHYS after their closing
 *               synchronisation; an asynchronous csph_step only counts.
 */
#ifndef CSPH_H
#define CSPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t csph_status;
#define CSPH_OK 0
#define CSPH_EINVAL 1
#define CSPH_ECAPACITY 2
#define CSPH_EDEVICE 3
#define CSPH_ENONPHYS 4 /* outputs written; some particle's state was non-physical */

typedef void *csph_stream; /* hipStream_t */

#define CSPH_MAX_EOS 8
#define CSPH_EOS_IDEAL 0     /* P = (gamma-1) rho e,            c^2 = gamma P / rho          */
#define CSPH_EOS_STIFFENED 1 /* P = (gamma-1) rho e - gamma P_inf, c^2 = gamma (P+P_inf) / rho */
/* Mie-Grueneisen (eqs. mie_gruneisen_eos, mie_gruneisen_reference), gamma = Gamma:
 *   x = rho0/rho, eta = 1 - x, D = 1 - s_a eta,
 *   P_r = rho0 c_a^2 eta / D^2, e_r = c_a^2 eta^2 / (2 D^2), P = P_r + Gamma rho (e - e_r),
 *   c^2 = c_a^2 x^2 (1 + s_a eta)/D^3 + Gamma (e - e_r) - Gamma c_a^2 eta x / D^3 + Gamma P/rho
 *   (the sound speed (dP/drho)_s, derived; the paper prints none).  D <= 0 (compression
 *   beyond the Hugoniot's limit) or c^2 < 0 is non-physical: c = 0, counted. */
#define CSPH_EOS_MIE_GRUNEISEN 2

#define CSPH_FP64 0  /* every operation in FP64 */
#define CSPH_MIXED 1 /* pair arithmetic in FP32; positions, EOS, integration, totals FP64 */

#define CSPH_H_FIXED 0 /* support H = kappa*h for every pair */
#define CSPH_H_PAIR 1  /* H_ij = kappa*(d_i+d_j)/2, d_i given per particle (eq. SmoothingLengthDef) */

/* Cell keys csph_bin reports (sec. 4.2 cells, numbered for the renumbering of particles):
 * LINEAR (c_z dims_y + c_y) dims_x + c_x, over ncell keys; MORTON: the bits of c_x, c_y,
 * c_z interleaved (bit b of c_x at key bit 3b, of c_y at 3b+1, of c_z at 3b+2), over
 * 2^(3 bits) keys, bits = ceil(log2(max dims)), dims <= 1024 per axis. */
#define CSPH_KEY_LINEAR 0
#define CSPH_KEY_MORTON 1

/* Integrators of csph_step (Algorithm 1 renews the state; the paper names no integrator):
 * EULER: symplectic Euler, v, E, rho += dt F(U), then r += dt v_new (one rate evaluation).
 * RK2: two-stage strong-stability-preserving Runge-Kutta (Heun's method in Shu and Osher's
 * convex form), U1 = U + dt F(U, t) with r1 = r + dt v, U' = U/2 + (U1 + dt F(U1, t + dt))/2
 * with r' = r/2 + (r1 + dt v1)/2; dt from F(U) for both stages; the second evaluation takes
 * r1 wrapped into a periodic box and the piston at t + dt; the new state is reflected off the
 * piston and wrapped as the Euler step's.  Two rate evaluations (two binnings, two mesh
 * synchronisations); nbr_count is that of U, the non-physical count sums both evaluations. */
#define CSPH_INT_EULER 0
#define CSPH_INT_RK2 1

typedef struct {
    int32_t type;   /* CSPH_EOS_* */
    int32_t pad;
    double gamma;   /* adiabatic index (ideal, stiffened); Grueneisen Gamma (Mie-Grueneisen) */
    double p_inf;   /* stiffening pressure (stiffened gas only) */
    double rho0;    /* Mie-Grueneisen: reference density */
    double c_a;     /* Mie-Grueneisen: u_s = c_a + s_a u_p */
    double s_a;
} csph_eos;

typedef struct {
    int32_t precision; /* CSPH_FP64 | CSPH_MIXED */
    int32_t h_mode;    /* CSPH_H_FIXED | CSPH_H_PAIR */
    double h;          /* smoothing length (fixed mode); CFL length in both modes when > 0 */
    double kappa;      /* support radius in units of h (2 for the workloads, 1.936 in sec. 4.1) */
    double cell_size;  /* mesh cell D; <= 0 selects D = maximum support.  D may be smaller than
                          the support: the stencil then reaches ceil(H/D) cells each way */
    double cfl;        /* > 0: dt = cfl * min_i min(h_i / s_i, rho_i / |drho_i/dt|) (s_i the
                          pair signal speed; the second term bounds the relative density
                          change of one step); <= 0: the caller's dt is used */
    int32_t n_eos;     /* materials 0..n_eos-1; mat[i] selects eos[mat[i]] */
    int32_t wall;      /* 1: rigid piston plane x = wall_x0 + wall_v t, fluid at x > plane:
                          mirror partners in the rates (for any configuration, particles
                          behind the plane included), and csph_step reflects a particle
                          that crosses the plane */
    double wall_x0;
    double wall_v;
    csph_eos eos[CSPH_MAX_EOS];
    int32_t reorder;   /* csph_step: 1 = write the new state in cell order (renumbering of
                          sec. 4.2; `id` is carried along); 0 = keep the input order */
    int32_t key_mode;  /* CSPH_KEY_LINEAR | CSPH_KEY_MORTON: keys of csph_grid_build's mesh */
    int32_t check_nonphys; /* csph_step: 1 = wait for the step's kernels and return
                              CSPH_ENONPHYS if its EOS met a non-physical state */
    int32_t periodic;  /* periodic boundaries (secs. 6 and 7.1 run their plates periodic
                          across the impact direction): bit a (1 x, 2 y, 4 z) makes axis a
                          periodic on [box_lo[a], box_hi[a]) with period L_a = box_hi[a] -
                          box_lo[a].  The partners of i are the images (j, k) with
                          d_a = (x_j,a - x_i,a) - k_a L_a, k_a in {-1, 0, 1} (0 on the other
                          axes), |d| < H_ij, (j, k) != (i, 0); csph_step wraps a new position
                          x >= box_hi to x - L, x < box_lo to x + L.  Needs L_a > 2 H (1 +
                          1e-6) (H the maximum support), every position within [box_lo,
                          box_hi] on the periodic axes, and x not periodic with the wall;
                          else CSPH_EINVAL.  Not taken by the Verlet-list and adjoint calls
                          (CSPH_EINVAL).  0: open boundaries */
    double box_lo[3], box_hi[3]; /* the periodic box (read on the periodic axes only) */
    int32_t integrator; /* CSPH_INT_EULER | CSPH_INT_RK2 (csph_step, csph_step_static,
                           csph_step_mesh, csph_step_vjp; the Voronoi, Verlet-list and
                           CFL-adjoint steps take EULER only, else CSPH_EINVAL) */
    int32_t pad2;
} csph_params;

/* Particle state.  x..m: FP64 arrays of n entries.  mat: int32 material id
 * (NULL = material 0).  d: particle size d_i = (m_i/rho_i)^(1/3) used only
 * when h_mode = CSPH_H_PAIR (NULL otherwise).  id: optional int64 label
 * permuted together with the state when csph_step reorders. */
typedef struct {
    int64_t n;
    double *x, *y, *z;
    double *vx, *vy, *vz;
    double *rho;  /* density */
    double *E;    /* specific total energy E = e + |v|^2/2 (conservative form, eq. SPH:Energy) */
    double *m;    /* mass */
    int32_t *mat;
    double *d;
    int64_t *id;
} csph_state;

/* Uniform cubic mesh: origin = per-axis minimum of the positions,
 * inv_cell = 1/D (formed once on the host), dims_a = floor((max_a -
 * origin_a) * inv_cell) + 1, cell of a particle
 * c_a = min(floor((x_a - origin_a) * inv_cell), dims_a - 1), all in FP64
 * without contraction.  Keys: key_mode (see CSPH_KEY_*), over nkey keys. */
typedef struct {
    double origin[3];
    double cell;      /* D */
    double inv_cell;  /* 1.0 / D */
    int32_t dims[3];
    int32_t reach;    /* stencil half-width in cells: ceil(max support / D) */
    int64_t ncell;    /* dims[0] dims[1] dims[2] */
    int32_t key_mode; /* CSPH_KEY_LINEAR | CSPH_KEY_MORTON */
    int32_t pad;
    int64_t nkey;     /* key space: ncell (LINEAR) or 2^(3 bits) (MORTON) */
} csph_grid;

/* Rates of eqs. SPH:Conti, SPH:Pulse, SPH:Energy, one FP64 array each. */
typedef struct {
    double *drho, *dvx, *dvy, *dvz, *dE;
} csph_rates_out;

/* Human-readable name of a status code (static storage). */
const char *csph_status_string(csph_status s);
/* Thread-local message of the last failing call on this thread (static storage). */
const char *csph_last_error(void);
/* Library version string. */
const char *csph_version(void);

/* Workspace bytes the calls below need for n particles on a mesh of ncell
 * cells (host; no device work).  csph_bin, csph_neighbors, csph_rates and
 * csph_step each fit in this size (p->integrator = CSPH_INT_RK2 adds the second
 * stage's buffers; p may be NULL for the Euler step). */
size_t csph_workspace_size(int64_t n, int64_t ncell, const csph_params *p);

/* Mesh of sec. 4.2 for the given positions (see csph_grid).  Synchronises
 * the stream to bring the bounds to the host.  Cell size: p->cell_size, or
 * the maximum support when that is <= 0.  n = 0 gives a 1x1x1 mesh. */
csph_status csph_grid_build(const double *x, const double *y, const double *z, int64_t n,
                            const csph_params *p, const double *d, csph_grid *grid /* host out */,
                            void *ws, size_t ws_bytes, csph_stream stream);

/* Binning and cell-ordered numbering (sec. 4.2).  With *grid from
 * csph_grid_build (or any mesh that covers the positions), writes
 *   key[i]   cell key of particle i (input order, grid->key_mode), uint32;
 *   perm[s]  the input index of the s-th particle in cell order: the stable
 *            order by (key, input index);
 *   cell_start[c] = first s with key >= c, for c = 0..nkey
 *            (cell_start[nkey] = n); cell_start_cap >= nkey+1 entries.
 * key may be NULL.  Bit-exact: integer results of FP64 comparisons.
 * CSPH_EINVAL when grid->nkey does not match its dims and key_mode. */
csph_status csph_bin(const double *x, const double *y, const double *z, int64_t n,
                     const csph_grid *grid /* host */, uint32_t *key, int32_t *perm,
                     int32_t *cell_start, int64_t cell_start_cap, void *ws, size_t ws_bytes,
                     size_t *ws_needed, csph_stream stream);

/* Neighbour sets N(i) = { j != i : ((dx*dx)+(dy*dy))+(dz*dz) < H_ij^2 } in
 * FP64, H_ij = kappa*h or kappa*(0.5*(d_i+d_j)) (sec. 4.1: W > 0 only for
 * |r| < kappa h_ij), as CSR over input indices with each row ascending:
 * offsets[n+1] (int64, device), idx[nnz] (int32, device).  Builds its own
 * mesh (synchronises).  *nnz (host) receives the pair count.  idx may be
 * NULL (count only); if idx_cap < nnz the call returns CSPH_ECAPACITY with
 * offsets and *nnz filled.  A verification export: the rate kernels do not
 * need it. */
csph_status csph_neighbors(const csph_state *s, const csph_params *p, int64_t *offsets,
                           int32_t *idx, int64_t idx_cap, int64_t *nnz /* host */, void *ws,
                           size_t ws_bytes, size_t *ws_needed, csph_stream stream);

/* Rates of every particle at time t (t places the piston only), in the
 * input order: for each i and j in N(i), e = (r_j - r_i)/|r_j - r_i|,
 * v_L = v_i.e, v_R = v_j.e, acoustic Riemann solution
 *   v* = (Z_i v_L + Z_j v_R + P_i - P_j)/(Z_i+Z_j),
 *   P* = (Z_j P_i + Z_i P_j + Z_i Z_j (v_L - v_R))/(Z_i+Z_j),  Z = rho c,
 * W' = dW/dr of the Wendland C2 kernel with support H_ij, and
 *   drho_i = -2 rho_i sum_j (m_j/rho_j)(v_L - v*) W'
 *   dv_i   =  (2/rho_i) sum_j (m_j/rho_j) P* W' e
 *   dE_i   =  (2/rho_i) sum_j (m_j/rho_j) P* v* W'
 * (eqs. SPH:Conti, SPH:Pulse, SPH:Energy with grad_i W = -e W').  Coincident
 * particles count as neighbours and contribute nothing.  With a wall (sec. 7.1
 * rigid wall), every particle j (j = i included) whose mirror image
 * x' = 2 x_w - x_j lies within the support of i also acts through it, with
 * v_x' = 2 v_w - v_x,j and j's other fields, on either side of the wall.
 * signal (optional): s_i = max(c_i, max_j [max(c_i, c_j) + max(0, v_L - v_R)]).
 * nbr_count (optional): |N(i)| (real partners only).
 * nonphys (optional, device int64): incremented by the number of particles
 * whose squared sound speed is negative or NaN (their c is taken as 0).
 * Synchronises twice (mesh bounds; at the end, for the non-physical count):
 * returns CSPH_ENONPHYS, every output written, when that count is not 0. */
csph_status csph_rates(const csph_state *s, const csph_params *p, double t,
                       csph_rates_out out, double *signal, int32_t *nbr_count, int64_t *nonphys,
                       void *ws, size_t ws_bytes, size_t *ws_needed, csph_stream stream);

/* One step (Algorithm 1, state renewal and global time step):
 *   rates at (s_in, *t);  dt = cfl * min_i min(h/s_i, rho_i/|drho_i|)  (or dt_in
 *   when cfl <= 0);
 *   v += dt dv, E += dt dE, rho += dt drho, then r += dt v_new;  *t += dt.
 * s_out receives the new state (mat, m, d and id are carried); with
 * p->reorder = 1 in cell order, otherwise in the input order.  s_out may
 * alias s_in only when p->reorder = 0.  t (device, in/out), dt_used (device,
 * optional), totals (device, optional, 10 doubles): (hi, lo) compensated
 * FP64 sums of m, m vx, m vy, m vz, m E over the new state, in a fixed
 * reduction order.  nbr_count (optional) in the output order.  nonphys as
 * in csph_rates.  With a wall (p->wall; t is then required), a particle
 * whose new x lies behind the plane x_w(t + dt) is reflected off it, the
 * rigid wall of sec. 7.1 stopping it: x <- 2 x_w - x, v_x <- 2 v_w - v_x,
 * E <- E + (v_x'^2 - v_x^2)/2 (specific internal energy kept).
 * Synchronises once (mesh bounds); with p->check_nonphys also at the end,
 * returning CSPH_ENONPHYS (state written) if the EOS met a non-physical
 * state. */
csph_status csph_step(const csph_state *s_in, csph_state *s_out, const csph_params *p,
                      double *t, double dt_in, double *dt_used, double *totals,
                      int32_t *nbr_count, int64_t *nonphys, void *ws, size_t ws_bytes,
                      size_t *ws_needed, csph_stream stream);

/* csph_step fused with voronoi_assign of its result: the same step, and the Voronoi
 * ownership of the NEW positions (eq. VoronoiDefinition, ties to the smaller k, sec. 3.1)
 * with per-site loads, computed by the step's update kernel.  owner[i] (n, in s_out's
 * order), site_particles[k] and site_pairs[k] (K each, overwritten; site_pairs optional)
 * equal those of voronoi_assign(s_out positions, sites, K, nbr_count of this step) bit for
 * bit.  sites: K x 3 FP64, global coordinates, 1 <= K <= 1024.  Synchronises as csph_step. */
csph_status csph_step_voronoi(const csph_state *s_in, csph_state *s_out, const csph_params *p,
                              double *t, double dt_in, double *dt_used, double *totals,
                              int32_t *nbr_count, int64_t *nonphys, const double *sites,
                              int32_t K, int32_t *owner, int64_t *site_particles,
                              int64_t *site_pairs, void *ws, size_t ws_bytes, size_t *ws_needed,
                              csph_stream stream);

/* csph_step for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same step, same kernels and
 * results, with its workspace in a library-owned device array of 128 MiB per GPU
 * (enough for about 450 000 particles on a compact mesh) instead of a caller workspace.
 * The array is held on each GPU the library runs on until the process ends; the call
 * allocates nothing (no hipMalloc, no timing events: csph_profile_* does not see it).
 * The caller still passes the state, t and the outputs.  A step whose workspace exceeds
 * the array returns CSPH_ECAPACITY (the per-particle part is checked before any device
 * work, the mesh part after the bounds synchronisation), writing nothing.  Every call on
 * one GPU uses that GPU's one array: calls that overlap in time on one GPU (different
 * streams or host threads) race and must not be issued.  Synchronises as csph_step. */
csph_status csph_step_static(const csph_state *s_in, csph_state *s_out, const csph_params *p,
                             double *t, double dt_in, double *dt_used, double *totals,
                             int32_t *nbr_count, int64_t *nonphys, csph_stream stream);

/* csph_step on a mesh the caller gives, for callers that step many times over a known domain
 * and for graph capture (sec. 4.2's cells fixed over the domain instead of re-sized to the
 * particles each step): no bounds pass and no host synchronisation, so every kernel is
 * enqueued on `stream` and a caller may capture a sequence of these steps in a HIP graph and
 * replay it.  mesh (host): a csph_grid from csph_grid_build over points spanning the domain
 * (origin, cell, dims, reach in the caller's axes; its key_mode is not used); reach * cell
 * must cover the support (fixed-h mode only).  The results are those of csph_step while every
 * position lies on the mesh (and, along periodic axes, in the box): the binning counts the
 * particles that do not into *outside (device int64, optional, accumulated over calls, as
 * *nonphys); cells are clamped to the mesh, so nothing is read out of bounds for them, but
 * their partners may be missed.  With the piston the band of particles with mirror partners
 * is found on the device.  RK2 steps bin their second stage on the same mesh.
 * CSPH_EINVAL for pair-h mode, check_nonphys = 1 (it would synchronise) or a mesh whose reach
 * does not cover the support; otherwise as csph_step.  Capturing: size the workspace first
 * (an eager call), since a short one returns CSPH_ECAPACITY. */
csph_status csph_step_mesh(const csph_state *s_in, csph_state *s_out, const csph_params *p,
                           const csph_grid *mesh, double *t, double dt_in, double *dt_used,
                           double *totals, int32_t *nbr_count, int64_t *nonphys,
                           int64_t *outside, void *ws, size_t ws_bytes, size_t *ws_needed,
                           csph_stream stream);

/* Voronoi ownership (eq. VoronoiDefinition): owner[i] = the k minimising
 * ((x_i-g_kx)^2 + (y_i-g_ky)^2) + (z_i-g_kz)^2 in FP64 without contraction,
 * a tie going to the smaller k (sec. 3.1).  sites: K x 3 FP64, global
 * coordinates, 1 <= K <= 1024.  site_particles[k] (int64) = number of owned
 * particles; site_pairs[k] (int64, optional, needs nbr_count) = sum of
 * nbr_count over owned particles (interaction counts as the load measure,
 * sec. 1).  Both count arrays are overwritten.  Bit-exact (integers). */
csph_status voronoi_assign(const double *x, const double *y, const double *z, int64_t n,
                           const double *sites, int32_t K, const int32_t *nbr_count,
                           int32_t *owner, int64_t *site_particles, int64_t *site_pairs,
                           csph_stream stream);

/* Control block of a set of Verlet lists (device memory, caller-owned, 48 bytes, 8-byte
 * aligned).  csph_vlist_build fills it; each csph_step_vlist checks it on the device and
 * updates it, so a driver can issue list steps without waiting for them. */
typedef struct {
    double t_build; /* time of the build */
    double disp;    /* max_i |r_i - r_ref,i| of the current state */
    double margin;  /* beta H: the horizon margin of the lists */
    double vw2;     /* 2 |v_wall| (0 without a wall) */
    int64_t pairs;  /* directed pairs evaluated by the list steps since the build */
    int32_t steps;  /* list steps taken since the build */
    int32_t valid;  /* 1 while the lists give N(i) exactly; 0 once a step found them stale */
} csph_vlist_ctl;

/* Verlet lists (sec. 4.2): the partners of each particle within the horizon
 * R = (1 + beta) H, for reuse over several steps.  Fixed-h mode only.
 *   s_in -> s_out: the state renumbered into cell order (as csph_step with
 *     reorder = 1 does; s_out distinct from s_in; mat, id, d carried along).
 *     The lists index s_out's order.
 *   vl_count[n]: list lengths; vl_idx[cap * n] (device, 16-byte aligned; cap a multiple
 *     of 8): the partners of particle s in 8-entry chunks, entry k at
 *     vl_idx[((k/8) n + s) 8 + k%8], k < vl_count[s] (entries past the count in the last
 *     chunk are unspecified); j != s with r^2 < R^2 in FP64
 *     without contraction; a partner whose mirror image across the piston wall (at
 *     time *t, device) lies within R of s has the sign bit set.
 *   x_ref[3 n] (device): the positions at build, x..., y..., z....
 *   ctl (device, optional): reset for these lists (t_build = *t, steps = pairs = 0,
 *     valid = 1, margin = beta H, vw2 = 2 |wall_v|).
 *   *max_count (host, optional): 0, or the longest list when it exceeds cap; then the
 *     lists are truncated and the call returns CSPH_ECAPACITY.
 * Synchronises (mesh bounds, wall time, list overflow). */
csph_status csph_vlist_build(const csph_state *s_in, csph_state *s_out, const csph_params *p,
                             const double *t, double beta, int32_t cap, int32_t *vl_count,
                             int32_t *vl_idx, double *x_ref, csph_vlist_ctl *ctl,
                             int32_t *max_count, void *ws, size_t ws_bytes, size_t *ws_needed,
                             csph_stream stream);

/* One step from Verlet lists, in place on s (in the lists' order).  The rates take the
 * listed partners with r^2 < H^2 (FP64 test), which is N(i) exactly while no pair can
 * have entered the support from beyond the horizon, i.e. while
 * 2 max_i |r_i - r_ref,i| + 2 |v_wall| (t - t_build) < beta H.  The step checks that bound
 * on the device first (ctl->disp is the previous step's displacement; the first step after
 * a build always passes): when it fails, ctl->valid becomes 0 and this step and every later
 * one until the next csph_vlist_build leave s, t, dt_used, totals, nbr_count and nonphys
 * untouched.  Otherwise the update of csph_step (dt, totals, nbr_count, nonphys as there);
 * then ctl->disp = max_i |r_i - r_ref,i| of the new state, ctl->steps += 1 and
 * ctl->pairs += sum_i |N(i)|.  Asynchronous: a driver reads ctl when it synchronises. */
csph_status csph_step_vlist(csph_state *s, const csph_params *p, double *t, double dt_in,
                            double *dt_used, double *totals, int32_t *nbr_count,
                            int64_t *nonphys, const int32_t *vl_count, const int32_t *vl_idx,
                            int32_t cap, const double *x_ref, csph_vlist_ctl *ctl, void *ws,
                            size_t ws_bytes, size_t *ws_needed, csph_stream stream);

/* Voronoi load balancer (sec. 3).  Generators, centres: K x 3 row-major
 * FP64 (device); 1 <= K <= 512.  Adjacency: K rows of W = ceil(K/32)
 * uint32 words; bit (l % 32) of word [k W + l/32] set iff subdomains k and l
 * touch. */
typedef struct {
    double sigma;  /* weight of the three-body terms, eq. BalancingOffsetPlusRot */
    double theta;  /* weight of the material motion, eq. TotalOffset (0.25 in sec. 3.4) */
    double gamma;  /* scale of the balancing displacement, eq. TotalOffset */
    double dsh;    /* D^sh: half width of the exchange layer; length factor of the two-body
                      terms, cap of the three-body shift (sec. 3.2, 3.3) */
} csph_balance_params;

/* Workspace bytes csph_balance_stats needs for K generators. */
size_t csph_balance_workspace_size(int32_t K);

/* Subdomain statistics of the assignment owner[] (from voronoi_assign with
 * these generators; entries outside [0, K) are ignored):
 *   site_particles[k], site_pairs[k] (sum of nbr_count, optional, needs nbr_count);
 *   centre[k] = mean position of the particles owned by k (eq. VoronoiGeomCenters;
 *     the generator itself if there are none).  Exact fixed-point sums
 *     (resolution 2^-32 per coordinate, |x - g_k| < 2^24), deterministic;
 *   adjacency: k and l touch when some particle owned by one of them has the
 *     other as its nearest other generator (ties to the smaller index) and
 *     lies within dsh of their bisector plane, tested as
 *     (d2_l - d2_k)^2 < (4 dsh^2) |g_l - g_k|^2 in FP64 without contraction;
 *     bit-exact.
 * Asynchronous; ws from csph_balance_workspace_size (CSPH_ECAPACITY and
 * *ws_needed if too small). */
csph_status csph_balance_stats(const double *x, const double *y, const double *z, int64_t n,
                               const int32_t *owner, const int32_t *nbr_count,
                               const double *sites, int32_t K, double dsh,
                               int64_t *site_particles, int64_t *site_pairs, double *centre,
                               uint32_t *adjacency, void *ws, size_t ws_bytes, size_t *ws_needed,
                               csph_stream stream);

/* One generator move: loads[k] (particles or pairs) drive
 *   dg_k = (1 - sigma) sum_l dsh (L_k - L_l)/(L_k + L_l) (g_k - g_l)/|g_k - g_l|
 *        + sigma C( sum_{l<m} [M(c_k x c_m, a_m) M(c_k x c_l, a_l) c_k - c_k] ),
 * over touching l and mutually touching triplets (k, l, m), c_p = g_p - o_klm
 * (circumcentre), a_l = (pi/3)(L_l - L_k)/(L_k + L_l + L_m), C caps the
 * length at dsh (eqs. BalancingOffset, BalancingOffsetPlusRot,
 * BalancingOffsetRot); then g_k' = (1 - theta)(g_k + gamma dg_k) + theta centre_k
 * (eq. TotalOffset).  sites_out must not alias sites.  *move_sum (device) =
 * sum_k |g_k' - g_k| (eq. VDConvergence).  Zero-load pairs/triplets and
 * collinear triplets contribute nothing.  Asynchronous. */
csph_status csph_balance_move(const double *sites, int32_t K, const int64_t *loads,
                              const double *centre, const uint32_t *adjacency,
                              const csph_balance_params *bp, double *sites_out, double *move_sum,
                              csph_stream stream);

/* Specific total energy from the primitive state: e from the EOS inverse
 * (ideal: e = p/((gamma-1) rho); stiffened: e = (p + gamma P_inf)/((gamma-1) rho)),
 * E = e + |v|^2/2. */
csph_status csph_init_energy(const double *rho, const double *pres, const double *vx,
                             const double *vy, const double *vz, const int32_t *mat, int64_t n,
                             const csph_params *p, double *E, csph_stream stream);

/* Adjoint (vector-Jacobian products).  Both smoothing-length modes (in pair-h
 * mode the sizes d are constants of the map: no gradient is returned for them),
 * every boundary (open, the piston, periodic axes) and every material; FP64
 * arithmetic in both precisions (it differentiates the FP64 map).  A
 * gradient struct holds 8 FP64 arrays in the state's order.  The EOS-parameter
 * gradients are those of gamma and p_inf; for a Mie-Grueneisen material the
 * gamma slot holds d/dGamma and the p_inf slot stays 0 (rho0, c_a and s_a are
 * constants). */
typedef struct {
    double *x, *y, *z, *vx, *vy, *vz, *rho, *E;
} csph_grad;

/* VJP of csph_rates at time t (the piston's position; ignored without it):
 * with cotangents a of the five rate arrays (input order), g_state +=
 * (d rates / d state)^T a over the eight state arrays, and g_eos[2k] +=
 * dJ/d gamma_k, g_eos[2k+1] += dJ/d p_inf_k (device, 2*n_eos doubles,
 * optional).  The rates' dependence on (rho, E, v) through the EOS is
 * included; masses, materials and the piston's motion are constants.
 * Gather form: it relies on j in N(i) <=> i in N(j), with the piston on j's
 * mirror image lying within the support of i <=> i's within that of j
 * (sec. 7.1), and on periodic axes on j's image x_j - kL lying within the
 * support of i <=> i's image x_i + kL within that of j.  Where c = 0 the
 * derivative of c with respect to c^2 is taken as 0.  Synchronises once
 * (mesh bounds). */
csph_status csph_rates_vjp(const csph_state *s, const csph_params *p, double t,
                           csph_rates_out a, csph_grad g_state, double *g_eos, void *ws,
                           size_t ws_bytes, size_t *ws_needed, csph_stream stream);

/* VJP of one csph_step (either integrator) taken at time t with the time
 * step dt held fixed (the step's own dt, replayed): s_n is the state the step started
 * from, g_next the cotangent of the state after it (same particle order,
 * i.e. a step taken with reorder = 0), g_prev receives (d s_{n+1} / d s_n)^T
 * g_next (it may alias g_next), g_eos is accumulated as in csph_rates_vjp.
 * With the piston, the particles the step reflected off the wall at t + dt
 * are found again by the step's own test, x + dt (v_x + dt R_vx) < x_w(t + dt),
 * with R_vx in FP64 (the Euler step takes it from the sums its gather forms, in
 * another order than the rate kernel's: a particle ending within rounding of
 * the plane may be taken differently; the RK2 step evaluates the FP64 rates),
 * and the reflection's Jacobian is applied to their cotangents; the branch
 * itself is not differentiated.  The
 * periodic wrap is a translation (identity Jacobian).  The RK2 step's VJP is
 * composed of the rate VJPs of its two evaluations (U1 = U + dt F(U, t), the
 * second at U1 and t + dt) and an FP64 rate evaluation that forms U1; it takes
 * 28 n doubles of workspace beyond those calls' own (CSPH_ECAPACITY reports
 * the total) and synchronises three times. */
csph_status csph_step_vjp(const csph_state *s_n, const csph_params *p, double t, double dt,
                          csph_grad g_next, csph_grad g_prev, double *g_eos, void *ws,
                          size_t ws_bytes, size_t *ws_needed, csph_stream stream);

/* VJP of one Euler csph_step taken at time t whose time step came from the
 * CFL rule (p->cfl > 0; CSPH_EINVAL otherwise): dt = cfl min_i min(h_i/s_i,
 * rho_i/|drho_i|) is recomputed from s_n in FP64 (*dt_used, host, optional)
 * and its dependence on the state and the EOS parameters is included, so that
 * g_prev is the gradient of the step as csph_step takes it.  The minimum passes
 * dt's gradient to the particle that sets it: through its signal speed s_i
 * (the Courant limit; s_i is the maximum over its partners of max(c_i, c_j)
 * plus the closing speed, or c_i, and the maximum passes it on to the sound
 * speed, velocities and positions that attain it) or through rho_i/|drho_i|
 * (the density-change limit).  Arguments as in csph_step_vjp.  Synchronises
 * twice (mesh bounds, dt).  A state whose CFL step is not finite and positive
 * is CSPH_EINVAL. */
csph_status csph_step_vjp_cfl(const csph_state *s_n, const csph_params *p, double t,
                              csph_grad g_next, csph_grad g_prev, double *g_eos, double *dt_used,
                              void *ws, size_t ws_bytes, size_t *ws_needed, csph_stream stream);

/* VJP of csph_init_energy: with gE the cotangent of E, accumulates
 * g_vx/g_vy/g_vz += gE v, g_rho += gE de/drho (each optional) and
 * g_eos (2*n_eos, optional) += the gamma / p_inf parts. */
csph_status csph_init_energy_vjp(const double *rho, const double *pres, const double *vx,
                                 const double *vy, const double *vz, const int32_t *mat,
                                 int64_t n, const csph_params *p, const double *gE, double *g_vx,
                                 double *g_vy, double *g_vz, double *g_rho, double *g_eos,
                                 void *ws, size_t ws_bytes, size_t *ws_needed,
                                 csph_stream stream);

/* Kernel timing.  While enabled, every call records a pair of HIP events
 * on its stream around each kernel group below; csph_profile_read waits for
 * the recorded events, returns the summed durations and launch counts
 * since the previous read, and clears them.  Meant for benchmarks: the
 * events add a few microseconds per launch.  Not thread-safe across
 * concurrent callers. */
#define CSPH_PROF_BIN 0        /* bounds, keys, scan, scatter, per-cell order */
#define CSPH_PROF_PACK 1       /* gather into cell order + EOS + pair records */
#define CSPH_PROF_RATES 2      /* the pair-rate kernel */
#define CSPH_PROF_INTEGRATE 3  /* state update, dt, totals */
#define CSPH_PROF_VORONOI 4
#define CSPH_PROF_REORDER 5    /* return to input order */
#define CSPH_PROF_NEIGHBORS 6
#define CSPH_PROF_ADJOINT 7
#define CSPH_PROF_BALANCE 8    /* balancer statistics and generator moves */
#define CSPH_PROF_GROUPS 9
typedef struct {
    int64_t launches[CSPH_PROF_GROUPS];
    double ms[CSPH_PROF_GROUPS];
} csph_profile;

csph_status csph_profile_enable(int32_t on);
csph_status csph_profile_read(csph_profile *out /* host */);
/* Which groups record events while timing is enabled: bit g of mask for group g (default
 * all).  A benchmark that times only the pair-rate kernel inside its timed steps
 * (1 << CSPH_PROF_RATES) leaves the other groups' event records, and the idle stream
 * around them, out of those steps.  Never fails. */
csph_status csph_profile_groups(uint32_t mask);

#ifdef __cplusplus
}
#endif
#endif /* CSPH_H */
