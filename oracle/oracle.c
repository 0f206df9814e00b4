/*
 * Contact-SPH oracle: a plain, slow, FP64 CPU implementation of the per-step
 * particle interaction of Egorova, Dyachkov, Parshikov & Zhakhovsky,
 * "Parallel SPH modeling using dynamic domain decomposition and load
 * balancing displacement of Voronoi subdomains" (arXiv 1805.05128).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * checked against.  It shares no source, header, table or helper with the
 * GPU library, and the library never calls it.  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg load it.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared -pthread
 * (contraction off: every a*b+c below is a rounded product then a rounded sum).
 *
 * What each function follows:
 *   oracle_kernel_w / _dw   Wendland C2 kernel in 3D with support radius H
 *                           (sec. 4.1, the kernel of Dehnen & Aly cited there;
 *                           the paper prints only its radius kappa = 1.936).
 *   oracle_riemann          pairwise Riemann problem along e^R between left
 *                           particle i and right particle j (sec. 4.1); the
 *                           solver form is not printed, the linear acoustic
 *                           (impedance) solver is used.
 *   oracle_eos              e = E - v^2/2 (after eq. SPH:Energy); ideal and
 *                           stiffened-gas pressure and sound speed, and the
 *                           Mie-Grueneisen form (eqs. mie_gruneisen_eos,
 *                           mie_gruneisen_reference) with the sound speed
 *                           derived from it (not printed in the paper).
 *   oracle_neighbors        N(i) = { j != i : |r_j - r_i| < support }
 *                           (sec. 4.1, the support statement before sec. 4.2);
 *                           brute force over all j is the authority, a cell
 *                           list (sec. 4.2, eq. Dcell) gives the same sets.
 *                           With periodic axes (the PBC of the paper's static
 *                           and ejecta tests, secs. 6 and 7.1) partners are the
 *                           images of j: displacement (x_j - x_i) - k L per
 *                           periodic axis, k in {-1, 0, 1}.
 *   oracle_rates            eqs. SPH:Conti, SPH:Pulse, SPH:Energy.
 *   oracle_step             "renew particle positions and states" and the
 *                           global time step (Algorithm 1); symplectic Euler
 *                           with a Courant + density-change time step
 *                           (reading; the paper prints no time-step rule),
 *                           or a two-stage Runge-Kutta step (the paper names
 *                           no integrator).
 *   oracle_grid / _bin      uniform cubic mesh of cell size D (sec. 4.2) and
 *                           the cell-ordered particle numbering (sec. 4.2,
 *                           renumbering for locality).
 *   oracle_voronoi          eq. VoronoiDefinition with the boundary rule
 *                           "ties go to the smaller subdomain index"
 *                           (sec. 3.1); per-site particle and pair counts as
 *                           the load measure (interaction counts, sec. 1).
 *   oracle_totals           exact sums (Shewchuk expansions, correctly rounded).
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <sched.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ORACLE_MAX_EOS 8

typedef struct {
    double h;          /* smoothing length (fixed-h mode) */
    double kappa;      /* support radius in units of h */
    int32_t h_mode;    /* 0: support kappa*h for all pairs; 1: kappa*(d_i+d_j)/2 */
    int32_t n_eos;
    int32_t eos_type[ORACLE_MAX_EOS]; /* 0 ideal, 1 stiffened gas, 2 Mie-Grueneisen */
    double eos_gamma[ORACLE_MAX_EOS];
    double eos_pinf[ORACLE_MAX_EOS];
    int32_t wall;      /* 1: rigid piston plane x = wall_x0 + wall_v*t, normal +x */
    int32_t search;    /* 0: brute force over all j; 1: cell list */
    double wall_x0;
    double wall_v;
    double cfl;        /* >0: dt = cfl * min_i h_i/s_i */
    double cell_size;  /* cell-list mode: mesh size D (>= support) */
    int32_t nthreads;  /* 0: all cores this process may use */
    int32_t pad;
    /* Mie-Grueneisen materials (type 2; Gamma is eos_gamma) */
    double eos_rho0[ORACLE_MAX_EOS];
    double eos_ca[ORACLE_MAX_EOS];
    double eos_sa[ORACLE_MAX_EOS];
    /* periodic boundaries: bit a of `periodic` makes axis a periodic with period
     * box_hi[a] - box_lo[a] (every particle inside [box_lo, box_hi) along it) */
    int32_t periodic;
    int32_t pad2;
    double box_lo[3];
    double box_hi[3];
    /* 0: symplectic Euler; 1: two-stage strong-stability-preserving Runge-Kutta */
    int32_t integrator;
    int32_t pad3;
} oracle_cfg;

/* ------------------------------------------------------------------ */
/* threading: static split of [0, n) over worker threads               */

typedef void (*range_fn)(void *ctx, int64_t lo, int64_t hi);
typedef struct { range_fn fn; void *ctx; int64_t lo, hi; } range_job;

static void *range_thread(void *arg) {
    range_job *j = (range_job *)arg;
    j->fn(j->ctx, j->lo, j->hi);
    return NULL;
}

int oracle_num_threads(void) {
    cpu_set_t set;
    if (sched_getaffinity(0, sizeof(set), &set) == 0) {
        int c = CPU_COUNT(&set);
        if (c > 0) return c;
    }
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    return c > 0 ? (int)c : 1;
}

static void parallel_for(int nthreads, int64_t n, range_fn fn, void *ctx) {
    if (nthreads <= 0) nthreads = oracle_num_threads();
    if (nthreads > 256) nthreads = 256;
    if (n < 2048 || nthreads == 1) { fn(ctx, 0, n); return; }
    pthread_t th[256];
    range_job jobs[256];
    int64_t chunk = (n + nthreads - 1) / nthreads;
    int used = 0;
    for (int t = 0; t < nthreads; ++t) {
        int64_t lo = (int64_t)t * chunk, hi = lo + chunk;
        if (lo >= n) break;
        if (hi > n) hi = n;
        jobs[t] = (range_job){fn, ctx, lo, hi};
        pthread_create(&th[t], NULL, range_thread, &jobs[t]);
        ++used;
    }
    for (int t = 0; t < used; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------ */
/* kernel: Wendland C2 in 3D, support radius H, q = r/H                */

double oracle_kernel_w(double r, double H) {
    double q = r / H;
    if (!(q < 1.0)) return 0.0;
    double a = 1.0 - q;
    return (21.0 / (2.0 * M_PI * H * H * H)) * (a * a * a * a) * (1.0 + 4.0 * q);
}

/* dW/dr: d/dq[(1-q)^4 (1+4q)] = -20 q (1-q)^3, times 1/H. */
double oracle_kernel_dw(double r, double H) {
    double q = r / H;
    if (!(q < 1.0)) return 0.0;
    double a = 1.0 - q;
    return -(21.0 / (2.0 * M_PI * H * H * H)) * 20.0 * q * (a * a * a) / H;
}

/* ------------------------------------------------------------------ */
/* Riemann problem along e^R: left = particle i, right = particle j.   */
/* Acoustic waves: P* + Z_L v* = P_L + Z_L v_L (left-going wave) and   */
/* P* - Z_R v* = P_R - Z_R v_R (right-going wave).                     */

void oracle_riemann(double ZL, double ZR, double PL, double PR, double vL, double vR,
                    double *vstar, double *pstar) {
    double S = ZL + ZR;
    if (S == 0.0) {
        *vstar = 0.5 * (vL + vR);
        *pstar = 0.5 * (PL + PR);
        return;
    }
    *vstar = (ZL * vL + ZR * vR + (PL - PR)) / S;
    *pstar = (ZR * PL + ZL * PR + ZL * ZR * (vL - vR)) / S;
}

/* ------------------------------------------------------------------ */
/* equation of state                                                   */

/* Mie-Grueneisen reference curves of the linear u_s - u_p Hugoniot
 * (eq. mie_gruneisen_reference) at compression x = rho0/rho:
 *   P_r = rho0 c_a^2 (1 - x) / [1 - s_a (1 - x)]^2,
 *   e_r = (c_a^2 / 2) (1 - x)^2 / [1 - s_a (1 - x)]^2.
 * Returns D = 1 - s_a (1 - x) (the curves exist for D > 0). */
static double mg_reference(double rho0, double ca, double sa, double rho, double *Pr,
                           double *er) {
    double x = rho0 / rho;
    double eta = 1.0 - x;
    double D = 1.0 - sa * eta;
    double D2 = D * D;
    *Pr = rho0 * ca * ca * eta / D2;
    *er = 0.5 * ca * ca * eta * eta / D2;
    return D;
}

static int eos_eval(const oracle_cfg *cfg, int mat, double rho, double e, double *P, double *c) {
    int k = (mat >= 0 && mat < cfg->n_eos) ? mat : 0;
    double g = cfg->eos_gamma[k], pinf = cfg->eos_pinf[k];
    double p, c2;
    if (cfg->eos_type[k] == 2) {
        /* eq. mie_gruneisen_eos, P - P_r = Gamma rho (e - e_r), Gamma = eos_gamma.  The
         * paper prints no sound speed; c^2 = (dP/drho)_e + (P/rho^2)(dP/de)_rho, with
         * dP_r/drho = c_a^2 x^2 (1 + s_a eta)/D^3 and rho de_r/drho = c_a^2 eta x/D^3. */
        double rho0 = cfg->eos_rho0[k], ca = cfg->eos_ca[k], sa = cfg->eos_sa[k];
        double Pr, er;
        double D = mg_reference(rho0, ca, sa, rho, &Pr, &er);
        double x = rho0 / rho, eta = 1.0 - x, D3 = D * D * D;
        p = Pr + g * rho * (e - er);
        double dPr = ca * ca * x * x * (1.0 + sa * eta) / D3;
        double rder = ca * ca * eta * x / D3;
        c2 = dPr + g * (e - er) - g * rder + g * p / rho;
        if (!(D > 0.0)) c2 = -1.0; /* beyond the Hugoniot's compression limit */
    } else if (cfg->eos_type[k] == 1) {
        p = (g - 1.0) * rho * e - g * pinf;
        c2 = g * (p + pinf) / rho;
    } else {
        p = (g - 1.0) * rho * e;
        c2 = g * p / rho;
    }
    *P = p;
    int bad = !(c2 >= 0.0);
    *c = bad ? 0.0 : sqrt(c2);
    return bad;
}

static double specific_internal(double E, double vx, double vy, double vz) {
    return E - 0.5 * ((vx * vx + vy * vy) + vz * vz);
}

int64_t oracle_eos(const oracle_cfg *cfg, int64_t n, const double *rho, const double *E,
                   const double *vx, const double *vy, const double *vz, const int32_t *mat,
                   double *P, double *c) {
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        double e = specific_internal(E[i], vx[i], vy[i], vz[i]);
        bad += eos_eval(cfg, mat ? mat[i] : 0, rho[i], e, &P[i], &c[i]);
    }
    return bad;
}

/* E from (rho, p, v): invert the EOS for e, then E = e + v^2/2. */
void oracle_init_energy(const oracle_cfg *cfg, int64_t n, const double *rho, const double *p,
                        const double *vx, const double *vy, const double *vz, const int32_t *mat,
                        double *E) {
    for (int64_t i = 0; i < n; ++i) {
        int k = mat ? mat[i] : 0;
        if (k < 0 || k >= cfg->n_eos) k = 0;
        double g = cfg->eos_gamma[k];
        double e;
        if (cfg->eos_type[k] == 2) {
            double Pr, er;
            mg_reference(cfg->eos_rho0[k], cfg->eos_ca[k], cfg->eos_sa[k], rho[i], &Pr, &er);
            e = er + (p[i] - Pr) / (g * rho[i]);
        } else if (cfg->eos_type[k] == 1) {
            e = (p[i] + g * cfg->eos_pinf[k]) / ((g - 1.0) * rho[i]);
        } else {
            e = p[i] / ((g - 1.0) * rho[i]);
        }
        E[i] = e + 0.5 * ((vx[i] * vx[i] + vy[i] * vy[i]) + vz[i] * vz[i]);
    }
}

/* ------------------------------------------------------------------ */
/* mesh and cell-ordered numbering                                     */

/* origin = min coordinate, dims = floor((max - origin) / D) + 1 with 1/D
 * formed once; returns 0, or -1 when n == 0. */
int oracle_grid(int64_t n, const double *x, const double *y, const double *z, double D,
                double *origin, int32_t *dims) {
    if (n <= 0) return -1;
    const double *c[3] = {x, y, z};
    double inv = 1.0 / D;
    for (int d = 0; d < 3; ++d) {
        double lo = c[d][0], hi = c[d][0];
        for (int64_t i = 1; i < n; ++i) {
            if (c[d][i] < lo) lo = c[d][i];
            if (c[d][i] > hi) hi = c[d][i];
        }
        origin[d] = lo;
        dims[d] = (int32_t)floor((hi - lo) * inv) + 1;
    }
    return 0;
}

static int32_t cell_coord(double v, double o, double inv, int32_t dim) {
    int32_t c = (int32_t)floor((v - o) * inv);
    if (c < 0) c = 0;
    if (c > dim - 1) c = dim - 1;
    return c;
}

static int64_t morton_key(int32_t cx, int32_t cy, int32_t cz) {
    int64_t k = 0;
    for (int b = 0; b < 21; ++b) {
        k |= (int64_t)((cx >> b) & 1) << (3 * b);
        k |= (int64_t)((cy >> b) & 1) << (3 * b + 1);
        k |= (int64_t)((cz >> b) & 1) << (3 * b + 2);
    }
    return k;
}

typedef struct { int64_t key; int64_t idx; } key_idx;

static int cmp_key_idx(const void *a, const void *b) {
    const key_idx *p = (const key_idx *)a, *q = (const key_idx *)b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    return (p->idx > q->idx) - (p->idx < q->idx);
}

/* Cell triple, key (0: linear (cz*dy+cy)*dx+cx, 1: Morton), and the stable
 * order by (key, index): perm[s] = index of the s-th particle in cell order;
 * cell_start[c] = first s with key >= c, cell_start[ncell] = n. */
int oracle_bin(int64_t n, const double *x, const double *y, const double *z, double D,
               const double *origin, const int32_t *dims, int32_t key_mode,
               int32_t *cell, int64_t *key, int64_t *perm, int64_t *cell_start, int64_t ncell) {
    double inv = 1.0 / D;
    key_idx *ki = (key_idx *)malloc(sizeof(key_idx) * (size_t)(n > 0 ? n : 1));
    if (!ki) return -1;
    for (int64_t i = 0; i < n; ++i) {
        int32_t cx = cell_coord(x[i], origin[0], inv, dims[0]);
        int32_t cy = cell_coord(y[i], origin[1], inv, dims[1]);
        int32_t cz = cell_coord(z[i], origin[2], inv, dims[2]);
        if (cell) { cell[3 * i] = cx; cell[3 * i + 1] = cy; cell[3 * i + 2] = cz; }
        int64_t k = key_mode == 1 ? morton_key(cx, cy, cz)
                                  : ((int64_t)cz * dims[1] + cy) * dims[0] + cx;
        key[i] = k;
        ki[i].key = k;
        ki[i].idx = i;
    }
    qsort(ki, (size_t)n, sizeof(key_idx), cmp_key_idx);
    for (int64_t s = 0; s < n; ++s) perm[s] = ki[s].idx;
    if (cell_start) {
        int64_t s = 0;
        for (int64_t c = 0; c <= ncell; ++c) {
            while (s < n && ki[s].key < c) ++s;
            cell_start[c] = s;
        }
    }
    free(ki);
    return 0;
}

/* ------------------------------------------------------------------ */
/* neighbour sets                                                      */

typedef struct {
    const oracle_cfg *cfg;
    int64_t n;
    const double *x, *y, *z, *d;
    /* cell list (search == 1) */
    double origin[3], inv;
    int32_t dims[3], reach;
    int64_t *order;      /* particle indices in (cell, index) order */
    int64_t *cstart;     /* per linear cell */
} nbr_space;

static double support_sq(const nbr_space *sp, int64_t i, int64_t j) {
    const oracle_cfg *cfg = sp->cfg;
    double H = cfg->h_mode == 1 ? cfg->kappa * (0.5 * (sp->d[i] + sp->d[j])) : cfg->kappa * cfg->h;
    return H * H;
}

static double support_of(const nbr_space *sp, int64_t i, int64_t j) {
    const oracle_cfg *cfg = sp->cfg;
    return cfg->h_mode == 1 ? cfg->kappa * (0.5 * (sp->d[i] + sp->d[j])) : cfg->kappa * cfg->h;
}

/* Period of axis a, or 0 when it is not periodic. */
static double period(const oracle_cfg *cfg, int a) {
    return (cfg->periodic >> a) & 1 ? cfg->box_hi[a] - cfg->box_lo[a] : 0.0;
}

/* Component a of the displacement from i to image k of j: (x_j - x_i) - k L.  The difference
 * comes first, so swapping i and j (and k to -k) negates it exactly. */
static double disp(double xj, double xi, int k, double L) {
    double d = xj - xi;
    return k ? d - (double)k * L : d;
}

static int cmp_i64(const void *a, const void *b) {
    int64_t p = *(const int64_t *)a, q = *(const int64_t *)b;
    return (p > q) - (p < q);
}

/* Candidate j for particle i (all j, or the cells within reach), ascending. */
/* Candidates for partners of a point p (a particle, or the mirror image of one): all
 * particles (brute force), or those of the cells within the reach of p's cell, clamped to
 * the mesh (a point off the mesh then gets a superset of the particles within the support
 * of it).  Ascending j. */
static int64_t candidates_at(const nbr_space *sp, double px, double py, double pz,
                             int64_t *buf, int64_t cap) {
    int64_t cnt = 0;
    if (sp->cfg->search == 0) {
        for (int64_t j = 0; j < sp->n && cnt < cap; ++j) buf[cnt++] = j;
        return cnt;
    }
    int32_t ci[3];
    const double p[3] = {px, py, pz};
    for (int dd = 0; dd < 3; ++dd) {
        double f = floor((p[dd] - sp->origin[dd]) * sp->inv);
        if (f < 0.0) f = 0.0;
        if (f > (double)(sp->dims[dd] - 1)) f = (double)(sp->dims[dd] - 1);
        ci[dd] = (int32_t)f;
    }
    int R = sp->reach;
    for (int oz = -R; oz <= R; ++oz) {
        int cz = ci[2] + oz;
        if (cz < 0 || cz >= sp->dims[2]) continue;
        for (int oy = -R; oy <= R; ++oy) {
            int cy = ci[1] + oy;
            if (cy < 0 || cy >= sp->dims[1]) continue;
            for (int ox = -R; ox <= R; ++ox) {
                int cx = ci[0] + ox;
                if (cx < 0 || cx >= sp->dims[0]) continue;
                int64_t lc = ((int64_t)cz * sp->dims[1] + cy) * sp->dims[0] + cx;
                for (int64_t s = sp->cstart[lc]; s < sp->cstart[lc + 1] && cnt < cap; ++s)
                    buf[cnt++] = sp->order[s];
            }
        }
    }
    qsort(buf, (size_t)cnt, sizeof(int64_t), cmp_i64);
    return cnt;
}

/* Partners of particle i: the images (j, k) with |d| < H_ij, d_a = (x_j,a - x_i,a) - k_a L_a
 * (k_a = 0 on non-periodic axes), (j, k) != (i, 0); candidates are all j (brute force) or
 * the cells around the image point x_i + k L.  The partners go to s->pr with their image
 * shifts, ordered by j (each j appears at most once when every period exceeds twice the
 * support).  Returns the count. */
typedef struct { int64_t j; int k[3]; } partner;

static int cmp_partner(const void *a, const void *b) {
    const partner *p = (const partner *)a, *q = (const partner *)b;
    if (p->j != q->j) return p->j < q->j ? -1 : 1;
    for (int c = 0; c < 3; ++c)
        if (p->k[c] != q->k[c]) return p->k[c] < q->k[c] ? -1 : 1;
    return 0;
}

/* scratch of one worker: candidate indices, and the partners of one particle (grown on
 * demand) */
typedef struct { int64_t *buf; partner *pr; int64_t cap, pcap; } nbr_scratch;

static int64_t partners_of(const nbr_space *sp, int64_t i, nbr_scratch *s) {
    int64_t *buf = s->buf, cap = s->cap;
    const oracle_cfg *cfg = sp->cfg;
    const double L[3] = {period(cfg, 0), period(cfg, 1), period(cfg, 2)};
    int64_t cnt = 0;
    for (int kz = -1; kz <= 1; ++kz) {
        if (kz && !L[2]) continue;
        for (int ky = -1; ky <= 1; ++ky) {
            if (ky && !L[1]) continue;
            for (int kx = -1; kx <= 1; ++kx) {
                if (kx && !L[0]) continue;
                int64_t nc = candidates_at(sp, sp->x[i] + kx * L[0], sp->y[i] + ky * L[1],
                                           sp->z[i] + kz * L[2], buf, cap);
                for (int64_t q = 0; q < nc; ++q) {
                    int64_t j = buf[q];
                    if (j == i && !kx && !ky && !kz) continue;
                    double dx = disp(sp->x[j], sp->x[i], kx, L[0]);
                    double dy = disp(sp->y[j], sp->y[i], ky, L[1]);
                    double dz = disp(sp->z[j], sp->z[i], kz, L[2]);
                    double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
                    if (!(r2 < support_sq(sp, i, j))) continue;
                    if (cnt == s->pcap) {
                        s->pcap *= 2;
                        s->pr = (partner *)realloc(s->pr, sizeof(partner) * (size_t)s->pcap);
                        if (!s->pr) abort();
                    }
                    partner *out = s->pr;
                    out[cnt].j = j;
                    out[cnt].k[0] = kx;
                    out[cnt].k[1] = ky;
                    out[cnt].k[2] = kz;
                    ++cnt;
                }
            }
        }
    }
    qsort(s->pr, (size_t)cnt, sizeof(partner), cmp_partner);
    return cnt;
}

static double max_support(const oracle_cfg *cfg, int64_t n, const double *d) {
    if (cfg->h_mode != 1) return cfg->kappa * cfg->h;
    double dm = 0.0;
    for (int64_t i = 0; i < n; ++i) if (d[i] > dm) dm = d[i];
    return cfg->kappa * dm;
}

static int space_init(nbr_space *sp, const oracle_cfg *cfg, int64_t n, const double *x,
                      const double *y, const double *z, const double *d) {
    memset(sp, 0, sizeof(*sp));
    sp->cfg = cfg; sp->n = n; sp->x = x; sp->y = y; sp->z = z; sp->d = d;
    if (cfg->search != 1 || n == 0) return 0;
    double D = cfg->cell_size;
    double Hmax = max_support(cfg, n, d);
    if (!(D > 0.0)) D = Hmax;
    oracle_grid(n, x, y, z, D, sp->origin, sp->dims);
    sp->inv = 1.0 / D;
    sp->reach = (int32_t)ceil(Hmax / D);
    if (sp->reach < 1) sp->reach = 1;
    int64_t ncell = (int64_t)sp->dims[0] * sp->dims[1] * sp->dims[2];
    sp->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    sp->cstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell + 1));
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!sp->order || !sp->cstart || !key) { free(key); return -1; }
    oracle_bin(n, x, y, z, D, sp->origin, sp->dims, 0, NULL, key, sp->order, sp->cstart, ncell);
    free(key);
    return 0;
}

static void space_free(nbr_space *sp) {
    free(sp->order);
    free(sp->cstart);
}

typedef struct {
    nbr_space *sp;
    int64_t *count;       /* pass 1 output */
    const int64_t *offsets; int32_t *idx;  /* pass 2 */
} nbr_ctx;

static int scratch_init(nbr_scratch *s, int64_t n) {
    s->cap = n > 0 ? n : 1;
    s->pcap = 1024;
    s->buf = (int64_t *)malloc(sizeof(int64_t) * (size_t)s->cap);
    s->pr = (partner *)malloc(sizeof(partner) * (size_t)s->pcap);
    return s->buf && s->pr ? 0 : -1;
}

static void scratch_free(nbr_scratch *s) {
    free(s->buf);
    free(s->pr);
}

static void nbr_count_range(void *vctx, int64_t lo, int64_t hi) {
    nbr_ctx *ctx = (nbr_ctx *)vctx;
    nbr_space *sp = ctx->sp;
    nbr_scratch s;
    if (scratch_init(&s, sp->n) != 0) { scratch_free(&s); return; }
    for (int64_t i = lo; i < hi; ++i) ctx->count[i] = partners_of(sp, i, &s);
    scratch_free(&s);
}

static void nbr_fill_range(void *vctx, int64_t lo, int64_t hi) {
    nbr_ctx *ctx = (nbr_ctx *)vctx;
    nbr_space *sp = ctx->sp;
    nbr_scratch s;
    if (scratch_init(&s, sp->n) != 0) { scratch_free(&s); return; }
    for (int64_t i = lo; i < hi; ++i) {
        int64_t np = partners_of(sp, i, &s), w = ctx->offsets[i];
        for (int64_t q = 0; q < np; ++q) ctx->idx[w++] = (int32_t)s.pr[q].j;
    }
    scratch_free(&s);
}

/* CSR of N(i) = { j != i : ((dx*dx)+(dy*dy))+(dz*dz) < H_ij^2 }, rows ascending.
 * Returns nnz; if idx is NULL or idx_cap < nnz only offsets are written. */
int64_t oracle_neighbors(const oracle_cfg *cfg, int64_t n, const double *x, const double *y,
                         const double *z, const double *d, int64_t *offsets, int32_t *idx,
                         int64_t idx_cap) {
    nbr_space sp;
    if (space_init(&sp, cfg, n, x, y, z, d) != 0) return -1;
    int64_t *count = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    nbr_ctx ctx = {&sp, count, NULL, NULL};
    parallel_for(cfg->nthreads, n, nbr_count_range, &ctx);
    offsets[0] = 0;
    for (int64_t i = 0; i < n; ++i) offsets[i + 1] = offsets[i] + count[i];
    int64_t nnz = offsets[n];
    if (idx && idx_cap >= nnz) {
        ctx.offsets = offsets;
        ctx.idx = idx;
        parallel_for(cfg->nthreads, n, nbr_fill_range, &ctx);
    }
    free(count);
    space_free(&sp);
    return nnz;
}

/* ------------------------------------------------------------------ */
/* CSPH rates, eqs. SPH:Conti, SPH:Pulse, SPH:Energy                   */

typedef struct {
    nbr_space *sp;
    const double *vx, *vy, *vz, *rho, *m, *P, *c;
    double t;
    double *drho, *dvx, *dvy, *dvz, *dE, *signal;
    int64_t *nbr_count;
    const int64_t *sample; /* NULL: every particle; else output k is particle sample[k] */
} rates_ctx;

/* One interaction of particle i with a partner at displacement (dx, dy, dz)
 * from it, moving with (vxj, vyj, vzj), that carries j's P, Z = rho c, m/rho.
 * Adds to the three j-sums of eqs. SPH:Conti / SPH:Pulse / SPH:Energy:
 *   s_rho += (m_j/rho_j) (v_i^R - v*) e.gradW
 *   s_v   += (m_j/rho_j) P* gradW
 *   s_E   += (m_j/rho_j) P* v* e.gradW
 * with gradW = grad_i W_ij = -e^R W'_ij.  Also updates the signal speed. */
static void pair_term(double dx, double dy, double dz, double vxi, double vyi, double vzi,
                      double Pi, double Zi, double ci, double vxj, double vyj, double vzj,
                      double Pj, double Zj, double cj, double Vj, double H,
                      double *s_rho, double s_v[3], double *s_E, double *sig) {
    double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
    if (r2 == 0.0) return; /* coincident: e undefined, W'(0) = 0 */
    double r = sqrt(r2);
    double e[3] = {dx / r, dy / r, dz / r};
    double dW = oracle_kernel_dw(r, H);
    double gradW[3] = {-e[0] * dW, -e[1] * dW, -e[2] * dW};
    double e_dot_gradW = (e[0] * gradW[0] + e[1] * gradW[1]) + e[2] * gradW[2];
    double vL = (vxi * e[0] + vyi * e[1]) + vzi * e[2];
    double vR = (vxj * e[0] + vyj * e[1]) + vzj * e[2];
    double vs, ps;
    oracle_riemann(Zi, Zj, Pi, Pj, vL, vR, &vs, &ps);
    *s_rho += Vj * (vL - vs) * e_dot_gradW;
    for (int k = 0; k < 3; ++k) s_v[k] += Vj * ps * gradW[k];
    *s_E += Vj * ps * vs * e_dot_gradW;
    double cm = ci > cj ? ci : cj;
    double closing = vL - vR;
    double s = cm + (closing > 0.0 ? closing : 0.0);
    if (s > *sig) *sig = s;
}

static void rates_range(void *vctx, int64_t lo, int64_t hi) {
    rates_ctx *ctx = (rates_ctx *)vctx;
    nbr_space *sp = ctx->sp;
    const oracle_cfg *cfg = sp->cfg;
    nbr_scratch scr;
    if (scratch_init(&scr, sp->n) != 0) { scratch_free(&scr); return; }
    int64_t cap = scr.cap, *buf = scr.buf;
    const double L[3] = {period(cfg, 0), period(cfg, 1), period(cfg, 2)};
    double xw = cfg->wall_x0 + cfg->wall_v * ctx->t;
    for (int64_t o = lo; o < hi; ++o) {
        int64_t i = ctx->sample ? ctx->sample[o] : o;
        double Zi = ctx->rho[i] * ctx->c[i];
        double s_rho = 0.0, s_v[3] = {0.0, 0.0, 0.0}, s_E = 0.0, sig = ctx->c[i];
        /* real neighbours (periodic images included), ascending j */
        int64_t cnt = partners_of(sp, i, &scr);
        for (int64_t q = 0; q < cnt; ++q) {
            int64_t j = scr.pr[q].j;
            double Zj = ctx->rho[j] * ctx->c[j];
            double Vj = ctx->m[j] / ctx->rho[j];
            pair_term(disp(sp->x[j], sp->x[i], scr.pr[q].k[0], L[0]),
                      disp(sp->y[j], sp->y[i], scr.pr[q].k[1], L[1]),
                      disp(sp->z[j], sp->z[i], scr.pr[q].k[2], L[2]), ctx->vx[i], ctx->vy[i],
                      ctx->vz[i], ctx->P[i], Zi, ctx->c[i], ctx->vx[j], ctx->vy[j], ctx->vz[j],
                      ctx->P[j], Zj, ctx->c[j], Vj, support_of(sp, i, j),
                      &s_rho, s_v, &s_E, &sig);
        }
        /* mirror partners across the piston plane (j = i included): the particles whose
         * image lies within the support of i, i.e. those within the support of the image of
         * i; with periodic y or z, also the translated images of those (the wall's own axis
         * x is never periodic).  Ascending (k_z, k_y), then j. */
        if (cfg->wall) {
            for (int kz = -1; kz <= 1; ++kz) {
                if (kz && !L[2]) continue;
                for (int ky = -1; ky <= 1; ++ky) {
                    if (ky && !L[1]) continue;
                    int64_t nc = candidates_at(sp, 2.0 * xw - sp->x[i], sp->y[i] + ky * L[1],
                                               sp->z[i] + kz * L[2], buf, cap);
                    for (int64_t k = 0; k < nc; ++k) {
                        int64_t j = buf[k];
                        double xg = 2.0 * xw - sp->x[j];
                        double dx = xg - sp->x[i];
                        double dy = disp(sp->y[j], sp->y[i], ky, L[1]);
                        double dz = disp(sp->z[j], sp->z[i], kz, L[2]);
                        double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
                        if (!(r2 < support_sq(sp, i, j))) continue;
                        double Zj = ctx->rho[j] * ctx->c[j];
                        double Vj = ctx->m[j] / ctx->rho[j];
                        pair_term(dx, dy, dz, ctx->vx[i], ctx->vy[i], ctx->vz[i], ctx->P[i], Zi,
                                  ctx->c[i], 2.0 * cfg->wall_v - ctx->vx[j], ctx->vy[j],
                                  ctx->vz[j], ctx->P[j], Zj, ctx->c[j], Vj, support_of(sp, i, j),
                                  &s_rho, s_v, &s_E, &sig);
                    }
                }
            }
        }
        double rho_i = ctx->rho[i];
        ctx->drho[o] = 2.0 * rho_i * s_rho;
        ctx->dvx[o] = -(2.0 / rho_i) * s_v[0];
        ctx->dvy[o] = -(2.0 / rho_i) * s_v[1];
        ctx->dvz[o] = -(2.0 / rho_i) * s_v[2];
        ctx->dE[o] = -(2.0 / rho_i) * s_E;
        if (ctx->signal) ctx->signal[o] = sig;
        if (ctx->nbr_count) ctx->nbr_count[o] = cnt;
    }
    scratch_free(&scr);
}

/* Rates of every particle at time t (t only places the piston).  Returns the
 * number of particles with a non-physical (negative or NaN) squared sound
 * speed, or -1 on allocation failure. */
int64_t oracle_rates(const oracle_cfg *cfg, int64_t n, const double *x, const double *y,
                     const double *z, const double *vx, const double *vy, const double *vz,
                     const double *rho, const double *E, const double *m, const int32_t *mat,
                     const double *d, double t, double *drho, double *dvx, double *dvy,
                     double *dvz, double *dE, double *signal, int64_t *nbr_count) {
    double *P = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *c = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!P || !c) { free(P); free(c); return -1; }
    int64_t bad = oracle_eos(cfg, n, rho, E, vx, vy, vz, mat, P, c);
    nbr_space sp;
    if (space_init(&sp, cfg, n, x, y, z, d) != 0) { free(P); free(c); return -1; }
    rates_ctx ctx = {&sp, vx, vy, vz, rho, m, P, c, t, drho, dvx, dvy, dvz, dE, signal, nbr_count,
                     NULL};
    parallel_for(cfg->nthreads, n, rates_range, &ctx);
    space_free(&sp);
    free(P);
    free(c);
    return bad;
}

/* Rates of the listed particles only (outputs indexed like `sample`): the
 * same sums as oracle_rates, for spot checks of large particle sets. */
int64_t oracle_rates_sample(const oracle_cfg *cfg, int64_t n, const double *x, const double *y,
                            const double *z, const double *vx, const double *vy, const double *vz,
                            const double *rho, const double *E, const double *m,
                            const int32_t *mat, const double *d, double t, const int64_t *sample,
                            int64_t nsample, double *drho, double *dvx, double *dvy, double *dvz,
                            double *dE, double *signal, int64_t *nbr_count) {
    double *P = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *c = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!P || !c) { free(P); free(c); return -1; }
    int64_t bad = oracle_eos(cfg, n, rho, E, vx, vy, vz, mat, P, c);
    nbr_space sp;
    if (space_init(&sp, cfg, n, x, y, z, d) != 0) { free(P); free(c); return -1; }
    rates_ctx ctx = {&sp, vx, vy, vz, rho, m, P, c, t, drho, dvx, dvy, dvz, dE, signal, nbr_count,
                     sample};
    parallel_for(cfg->nthreads, nsample, rates_range, &ctx);
    space_free(&sp);
    free(P);
    free(c);
    return bad;
}

/* dt = cfl * min_i min(h_i / s_i, rho_i / |drho_i|), h_i = h (fixed) or
 * d_i (pair mode): the signal-speed (Courant) limit plus a limit on the
 * relative density change of one explicit step, which keeps rho > 0 where
 * free surfaces expand into vacuum.  drho may be NULL (Courant part only). */
double oracle_dt(const oracle_cfg *cfg, int64_t n, const double *signal, const double *d,
                 const double *rho, const double *drho) {
    double best = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double hi = cfg->h_mode == 1 ? d[i] : cfg->h;
        double v = hi / signal[i];
        if (v < best) best = v;
        if (drho && rho) {
            double w = rho[i] / fabs(drho[i]);
            if (w < best) best = w;
        }
    }
    return cfg->cfl * best;
}

/* The constraints on a new position (shared by both integrators): a particle behind the
 * piston plane xw is reflected off it in the wall's frame (x <- 2 xw - x, v_x <- 2 v_w - v_x,
 * E changed by the kinetic-energy difference), then periodic axes wrap it back into
 * [box_lo, box_hi) (a particle moves less than a period per step). */
static void constrain(const oracle_cfg *cfg, double xw, double *x, double *y, double *z,
                      double *vx, double *E) {
    if (cfg->wall && *x < xw) {
        double vr = 2.0 * cfg->wall_v - *vx;
        *E = *E + 0.5 * ((vr * vr) - (*vx * *vx));
        *vx = vr;
        *x = 2.0 * xw - *x;
    }
    double *pos[3] = {x, y, z};
    for (int a = 0; a < 3; ++a) {
        double Lp = period(cfg, a);
        if (!Lp) continue;
        if (*pos[a] >= cfg->box_hi[a]) *pos[a] = *pos[a] - Lp;
        else if (*pos[a] < cfg->box_lo[a]) *pos[a] = *pos[a] + Lp;
    }
}

/* Two-stage strong-stability-preserving Runge-Kutta step (Heun's method in Shu and Osher's
 * convex form; a reading: the paper names no integrator).  With F the rates of
 * (v, E, rho) and v the rate of r:
 *   U1 = U + dt F(U, t),                  r1 = r + dt v
 *   U' = U/2 + (U1 + dt F(U1, t + dt))/2, r' = r/2 + (r1 + dt v1)/2
 * (each product and sum rounded as written).  dt comes from the rates of U, as in the Euler
 * step, and serves both stages.  The second stage evaluates the rates at U1 with its
 * positions wrapped into the periodic box (and the piston at x_w(t + dt)); the combination
 * takes r1 unwrapped.  The new state is then constrained as the Euler step's.  nbr_count is
 * that of U; the non-physical count sums both evaluations. */
static int64_t step_rk2(const oracle_cfg *cfg, int64_t n, double *x, double *y, double *z,
                        double *vx, double *vy, double *vz, double *rho, double *E,
                        const double *m, const int32_t *mat, const double *d, double *t,
                        double dt_in, double *dt_used, int64_t *nbr_count) {
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    enum { NBUF = 23 };
    double *b[NBUF];
    int ok = 1;
    for (int k = 0; k < NBUF; ++k) ok &= (b[k] = (double *)malloc(sz)) != NULL;
    int64_t bad = -1;
    if (ok) {
        double *f0 = b[0], *f1 = b[1], *f2 = b[2], *f3 = b[3], *f4 = b[4], *sg = b[5];
        double *x1 = b[6], *y1 = b[7], *z1 = b[8], *vx1 = b[9], *vy1 = b[10], *vz1 = b[11];
        double *rho1 = b[12], *E1 = b[13], *xe = b[14], *ye = b[15], *ze = b[16];
        double *q0 = b[17], *q1 = b[18], *q2 = b[19], *q3 = b[20], *q4 = b[21];
        bad = oracle_rates(cfg, n, x, y, z, vx, vy, vz, rho, E, m, mat, d, *t, f0, f1, f2, f3,
                           f4, sg, nbr_count);
        double dt = cfg->cfl > 0.0 ? oracle_dt(cfg, n, sg, d, rho, f0) : dt_in;
        for (int64_t i = 0; i < n; ++i) {
            vx1[i] = vx[i] + dt * f1[i];
            vy1[i] = vy[i] + dt * f2[i];
            vz1[i] = vz[i] + dt * f3[i];
            E1[i] = E[i] + dt * f4[i];
            rho1[i] = rho[i] + dt * f0[i];
            x1[i] = x[i] + dt * vx[i];
            y1[i] = y[i] + dt * vy[i];
            z1[i] = z[i] + dt * vz[i];
            double pe[3] = {x1[i], y1[i], z1[i]};
            for (int a = 0; a < 3; ++a) {
                double Lp = period(cfg, a);
                if (!Lp) continue;
                if (pe[a] >= cfg->box_hi[a]) pe[a] = pe[a] - Lp;
                else if (pe[a] < cfg->box_lo[a]) pe[a] = pe[a] + Lp;
            }
            xe[i] = pe[0];
            ye[i] = pe[1];
            ze[i] = pe[2];
        }
        int64_t bad2 = bad < 0 ? -1
                               : oracle_rates(cfg, n, xe, ye, ze, vx1, vy1, vz1, rho1, E1, m, mat,
                                              d, *t + dt, q0, q1, q2, q3, q4, NULL, NULL);
        if (bad2 < 0) {
            bad = -1;
        } else {
            bad += bad2;
            double t_new = *t + dt;
            double xw = cfg->wall_x0 + cfg->wall_v * t_new;
            for (int64_t i = 0; i < n; ++i) {
                double nvx = 0.5 * vx[i] + 0.5 * (vx1[i] + dt * q1[i]);
                double nvy = 0.5 * vy[i] + 0.5 * (vy1[i] + dt * q2[i]);
                double nvz = 0.5 * vz[i] + 0.5 * (vz1[i] + dt * q3[i]);
                double nE = 0.5 * E[i] + 0.5 * (E1[i] + dt * q4[i]);
                double nrho = 0.5 * rho[i] + 0.5 * (rho1[i] + dt * q0[i]);
                double nx = 0.5 * x[i] + 0.5 * (x1[i] + dt * vx1[i]);
                double ny = 0.5 * y[i] + 0.5 * (y1[i] + dt * vy1[i]);
                double nz = 0.5 * z[i] + 0.5 * (z1[i] + dt * vz1[i]);
                constrain(cfg, xw, &nx, &ny, &nz, &nvx, &nE);
                x[i] = nx; y[i] = ny; z[i] = nz;
                vx[i] = nvx; vy[i] = nvy; vz[i] = nvz;
                E[i] = nE; rho[i] = nrho;
            }
            *t = t_new;
            if (dt_used) *dt_used = dt;
        }
    }
    for (int k = 0; k < NBUF; ++k) free(b[k]);
    return bad;
}

/* One step: rates at (state, t); dt from the CFL rule (cfl > 0) or dt_in;
 * v += dt dv/dt, E += dt dE/dt, rho += dt drho/dt, then r += dt v(new);
 * t += dt.  With the piston (the rigid wall of sec. 7.1, which stops the
 * particles at the wall), a particle whose new x lies behind the plane
 * x_w(t + dt) is reflected about it, as off a rigid wall in the wall's
 * frame: x <- 2 x_w - x, v_x <- 2 v_w - v_x, with its specific internal
 * energy kept (E changes by the kinetic-energy difference, the wall's work).
 * Periodic axes wrap the new positions back into the box.
 * integrator = 1 takes the two-stage Runge-Kutta step above instead.
 * State arrays are updated in place.  Returns the non-physical count from
 * the rate evaluation (or -1). */
int64_t oracle_step(const oracle_cfg *cfg, int64_t n, double *x, double *y, double *z,
                    double *vx, double *vy, double *vz, double *rho, double *E, const double *m,
                    const int32_t *mat, const double *d, double *t, double dt_in, double *dt_used,
                    int64_t *nbr_count) {
    if (cfg->integrator == 1)
        return step_rk2(cfg, n, x, y, z, vx, vy, vz, rho, E, m, mat, d, t, dt_in, dt_used,
                        nbr_count);
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *r0 = malloc(sz), *r1 = malloc(sz), *r2 = malloc(sz), *r3 = malloc(sz),
           *r4 = malloc(sz), *sg = malloc(sz);
    int64_t bad = -1;
    if (r0 && r1 && r2 && r3 && r4 && sg) {
        bad = oracle_rates(cfg, n, x, y, z, vx, vy, vz, rho, E, m, mat, d, *t, r0, r1, r2, r3,
                           r4, sg, nbr_count);
        double dt = cfg->cfl > 0.0 ? oracle_dt(cfg, n, sg, d, rho, r0) : dt_in;
        double t_new = *t + dt;
        double xw = cfg->wall_x0 + cfg->wall_v * t_new;
        for (int64_t i = 0; i < n; ++i) {
            vx[i] = vx[i] + dt * r1[i];
            vy[i] = vy[i] + dt * r2[i];
            vz[i] = vz[i] + dt * r3[i];
            E[i] = E[i] + dt * r4[i];
            rho[i] = rho[i] + dt * r0[i];
            x[i] = x[i] + dt * vx[i];
            y[i] = y[i] + dt * vy[i];
            z[i] = z[i] + dt * vz[i];
            constrain(cfg, xw, &x[i], &y[i], &z[i], &vx[i], &E[i]);
        }
        *t = t_new;
        if (dt_used) *dt_used = dt;
    }
    free(r0); free(r1); free(r2); free(r3); free(r4); free(sg);
    return bad;
}

/* ------------------------------------------------------------------ */
/* exact sums: Shewchuk's non-overlapping expansions, rounded as in     */
/* Python's math.fsum                                                   */

typedef struct { double *p; int64_t n, cap; } expansion;

static void exp_add(expansion *e, double x) {
    int64_t k = 0;
    for (int64_t i = 0; i < e->n; ++i) {
        double y = e->p[i];
        if (fabs(x) < fabs(y)) { double t = x; x = y; y = t; }
        double hi = x + y;
        double lo = y - (hi - x);
        if (lo != 0.0) e->p[k++] = lo;
        x = hi;
    }
    if (k >= e->cap) {
        e->cap = e->cap ? 2 * e->cap : 32;
        e->p = (double *)realloc(e->p, sizeof(double) * (size_t)e->cap);
    }
    e->p[k++] = x;
    e->n = k;
}

static double exp_round(const expansion *e) {
    int64_t n = e->n;
    if (n == 0) return 0.0;
    double hi = e->p[--n], lo = 0.0;
    while (n > 0) {
        double x = hi, y = e->p[--n];
        hi = x + y;
        double yr = hi - x;
        lo = y - yr;
        if (lo != 0.0) break;
    }
    if (n > 0 && ((lo < 0.0 && e->p[n - 1] < 0.0) || (lo > 0.0 && e->p[n - 1] > 0.0))) {
        double y = lo * 2.0, x = hi + y, yr = x - hi;
        if (y == yr) hi = x;
    }
    return hi;
}

/* out = exact sums of m_i, m_i vx_i, m_i vy_i, m_i vz_i, m_i E_i (each
 * product rounded once, the sum correctly rounded). */
void oracle_totals(int64_t n, const double *m, const double *vx, const double *vy,
                   const double *vz, const double *E, double *out) {
    expansion e[5];
    memset(e, 0, sizeof(e));
    for (int64_t i = 0; i < n; ++i) {
        exp_add(&e[0], m[i]);
        exp_add(&e[1], m[i] * vx[i]);
        exp_add(&e[2], m[i] * vy[i]);
        exp_add(&e[3], m[i] * vz[i]);
        exp_add(&e[4], m[i] * E[i]);
    }
    for (int k = 0; k < 5; ++k) { out[k] = exp_round(&e[k]); free(e[k].p); }
}

/* exact sum of a double array (for tests of compensated GPU sums) */
double oracle_exact_sum(int64_t n, const double *v) {
    expansion e = {0};
    for (int64_t i = 0; i < n; ++i) exp_add(&e, v[i]);
    double r = exp_round(&e);
    free(e.p);
    return r;
}

/* ------------------------------------------------------------------ */
/* Voronoi ownership and load counts                                   */

/* owner_i = the k minimising ((x-gx)^2 + (y-gy)^2) + (z-gz)^2 over all K
 * generators, a tie going to the smaller k.  site_particles[k] counts
 * owned particles, site_pairs[k] sums nbr_count over them (if given). */
void oracle_voronoi(int64_t n, const double *x, const double *y, const double *z, int32_t K,
                    const double *sites, const int64_t *nbr_count, int32_t *owner,
                    int64_t *site_particles, int64_t *site_pairs) {
    for (int32_t k = 0; k < K; ++k) { site_particles[k] = 0; site_pairs[k] = 0; }
    for (int64_t i = 0; i < n; ++i) {
        int32_t best = 0;
        double bd = INFINITY;
        for (int32_t k = 0; k < K; ++k) {
            double dx = x[i] - sites[3 * k], dy = y[i] - sites[3 * k + 1], dz = z[i] - sites[3 * k + 2];
            double d2 = ((dx * dx) + (dy * dy)) + (dz * dz);
            if (d2 < bd) { bd = d2; best = k; }
        }
        owner[i] = best;
        site_particles[best] += 1;
        if (nbr_count) site_pairs[best] += nbr_count[i];
    }
}
