/*
 * channel_oracle.c -- plain FP64 CPU oracle of the confined-channel TTCF example of
 * arxiv 2312.02990 (the second example system: a Lennard-Jones liquid between two walls
 * whose atoms are tethered to lattice sites; Eq. system2 and Eq. TTCF2).
 *
 * TEST INFRASTRUCTURE: only the test-suite and the benchmark's CPU-baseline leg use this
 * file. It shares no code with the GPU library.
 *
 * Build: part of libttcf_oracle.so (gcc -O2 -ffp-contract=off), one rounding per operation.
 *
 * System (reduced units, m = sigma = epsilon = k_B = 1):
 *   - atoms 0..n_fluid-1 are fluid, then n_wall/2 bottom-wall and n_wall/2 top-wall atoms;
 *   - x and z are periodic (edges lx, lz); y is bounded by the walls (no image in y);
 *   - pair potential phi = 4[(1/r)^12 - c (1/r)^6] - phi_c for r < rc, with c = c_ff for
 *     fluid-fluid and c_wf for wall-fluid pairs and the shift phi_c making phi(rc) = 0; wall
 *     atoms do not interact with each other (they are held by their tethers only: reading
 *     of the unspecified wall-wall interaction);
 *   - each wall atom is tethered to its lattice site by a spring of stiffness k;
 *   - the lattices move along x at +v/2 (top) and -v/2 (bottom), relative velocity v;
 *   - a Nose-Hoover thermostat acts on the wall atoms only (Eq. system2), with target
 *     temperature T_w and 3 N_w degrees of freedom.
 * Dissipation function (Eq. TTCF2, with the beta and the sign that the adiabatic energy
 * balance fixes): Omega = -beta sum_walls sum_i k (r^w_i - r^l_i) . u_wall
 *                       = -(k v / (2 T_w)) S,  S = sum_top (x^w - x^l) - sum_bottom (x^w - x^l).
 * Observables B(t): the wall-fluid shear stress at the interfaces (method of planes:
 * [sum_{fluid i, top j} F_x,ij - sum_{fluid i, bottom j} F_x,ij] / (2 A), A = lx lz) and the
 * streaming-momentum profile: per bin of y, sum p_x over fluid atoms / bin volume.
 */
#include "channel_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

static double min_image(double d, double l) { return d - l * rint(d / l); }

static int is_wall(const orc_channel* c, int32_t i) { return i >= c->n_fluid; }
static int is_top(const orc_channel* c, int32_t i) { return i >= c->n_fluid + c->n_wall / 2; }

/* energy shift of one pair type: phi(rc) = 0 */
static double pair_shift(double rc, double cw) {
    double s6 = 1.0 / (rc * rc * rc * rc * rc * rc);
    return -4.0 * (s6 * s6 - cw * s6);
}

int32_t orc_ch_forces(const orc_channel* c, const double* r, const double* rl, double* f,
                      double* out) {
    const int32_t n = c->n, nf = c->n_fluid, nw = c->n_wall;
    const double rc2 = c->rc * c->rc;
    const double sh_ff = pair_shift(c->rc, c->c_ff), sh_wf = pair_shift(c->rc, c->c_wf);
    const double* x = r;
    const double* y = r + n;
    const double* z = r + 2 * n;
    memset(f, 0, sizeof(double) * 3 * (size_t)n);
    double u_lj = 0.0, u_spring = 0.0, fx_top = 0.0, fx_bot = 0.0, s_obs = 0.0;
    /* every pair i < j with at least one fluid atom, by direct summation */
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t j = i + 1; j < n; ++j) {
            if (is_wall(c, i) && is_wall(c, j)) continue;
            double dx = min_image(x[i] - x[j], c->lx);
            double dy = y[i] - y[j];
            double dz = min_image(z[i] - z[j], c->lz);
            double r2 = dx * dx + dy * dy + dz * dz;
            if (!(r2 < rc2)) continue;
            const int wf = is_wall(c, i) || is_wall(c, j);
            const double cw = wf ? c->c_wf : c->c_ff;
            double s = 1.0 / r2;
            double s3 = s * s * s;
            double fs = (48.0 * s3 * s3 - 24.0 * cw * s3) * s;
            u_lj += 4.0 * (s3 * s3 - cw * s3) + (wf ? sh_wf : sh_ff);
            f[i] += fs * dx;
            f[n + i] += fs * dy;
            f[2 * n + i] += fs * dz;
            f[j] -= fs * dx;
            f[n + j] -= fs * dy;
            f[2 * n + j] -= fs * dz;
            if (wf) {
                /* x force on the fluid atom from the wall atom */
                const int32_t w = is_wall(c, i) ? i : j;
                const double fx_on_fluid = is_wall(c, i) ? -fs * dx : fs * dx;
                if (is_top(c, w))
                    fx_top += fx_on_fluid;
                else
                    fx_bot += fx_on_fluid;
            }
        }
    }
    /* tethers: F = -k (r^w - r^l), x and z by minimum image */
    for (int32_t q = 0; q < nw; ++q) {
        const int32_t i = nf + q;
        double dx = min_image(x[i] - rl[q], c->lx);
        double dy = y[i] - rl[nw + q];
        double dz = min_image(z[i] - rl[2 * nw + q], c->lz);
        f[i] -= c->k_spring * dx;
        f[n + i] -= c->k_spring * dy;
        f[2 * n + i] -= c->k_spring * dz;
        u_spring += 0.5 * c->k_spring * (dx * dx + dy * dy + dz * dz);
        s_obs += is_top(c, i) ? dx : -dx;
    }
    out[0] = u_lj;
    out[1] = u_spring;
    out[2] = fx_top;
    out[3] = fx_bot;
    out[4] = s_obs;
    return 0;
}

void orc_ch_observables(const orc_channel* c, const double* r, const double* p,
                        const double* fout, double* obs) {
    const int32_t n = c->n;
    const double area = c->lx * c->lz;
    obs[0] = (fout[2] - fout[3]) / (2.0 * area);
    const double w = (c->bin_hi - c->bin_lo) / (double)c->n_bins;
    for (int32_t b = 0; b < c->n_bins; ++b) obs[1 + b] = 0.0;
    for (int32_t i = 0; i < c->n_fluid; ++i) {
        const double y = r[n + i];
        if (!(y >= c->bin_lo) || !(y < c->bin_hi)) continue;
        int32_t b = (int32_t)floor((y - c->bin_lo) / w);
        if (b > c->n_bins - 1) b = c->n_bins - 1;
        obs[1 + b] += p[i];
    }
    for (int32_t b = 0; b < c->n_bins; ++b) obs[1 + b] /= area * w;
}

static void wrap_xz(const orc_channel* c, double* r) {
    const int32_t n = c->n;
    for (int32_t i = 0; i < n; ++i) {
        r[i] -= c->lx * floor(r[i] / c->lx);
        if (r[i] >= c->lx) r[i] = 0.0;
        r[2 * n + i] -= c->lz * floor(r[2 * n + i] / c->lz);
        if (r[2 * n + i] >= c->lz) r[2 * n + i] = 0.0;
    }
}

/* lattice sites at step k: x advanced by +-(v/2) k dt (top / bottom), y and z fixed */
static void lattice_at(const orc_channel* c, const double* rl0, double v, double dt, int64_t k,
                       double* rl) {
    const int32_t nw = c->n_wall;
    memcpy(rl, rl0, sizeof(double) * 3 * (size_t)nw);
    const double shift = 0.5 * v * ((double)k * dt);
    for (int32_t q = 0; q < nw; ++q) rl[q] += (q >= nw / 2) ? shift : -shift;
}

static double wall_p2(const orc_channel* c, const double* p) {
    const int32_t n = c->n;
    double s = 0.0;
    for (int32_t i = c->n_fluid; i < n; ++i)
        s += p[i] * p[i] + p[n + i] * p[n + i] + p[2 * n + i] * p[2 * n + i];
    return s;
}

int32_t orc_ch_run(const orc_channel* c, double t_wall, double q, double dt, double v,
                   double* r, double* p, double* zeta, const double* rl0, int64_t k0,
                   int64_t nsteps, double* obs_out, double* s_out, double* energy_out) {
    const int32_t n = c->n, nw = c->n_wall;
    const int nobs = 1 + c->n_bins;
    double* f = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* rl = (double*)malloc(sizeof(double) * 3 * (size_t)nw);
    if (!f || !rl) {
        free(f);
        free(rl);
        return -2;
    }
    const double nf_w = 3.0 * nw;
    const double h = dt;
    double fo[5];
    int64_t k = k0;
    lattice_at(c, rl0, v, dt, k, rl);
    orc_ch_forces(c, r, rl, f, fo);
    double z = *zeta;
    if (obs_out) orc_ch_observables(c, r, p, fo, obs_out);
    if (s_out) s_out[0] = fo[4];
    if (energy_out) {
        double ke = 0.0;
        for (int32_t a = 0; a < 3 * n; ++a) ke += 0.5 * p[a] * p[a];
        energy_out[0] = ke + fo[0] + fo[1];
    }
    for (int64_t s = 1; s <= nsteps; ++s) {
        /* thermostat half step on the wall atoms, then the velocity-Verlet step */
        if (q > 0.0) {
            z += 0.5 * h * (wall_p2(c, p) - nf_w * t_wall) / q;
            const double sc = exp(-z * 0.5 * h);
            for (int32_t i = c->n_fluid; i < n; ++i) {
                p[i] *= sc;
                p[n + i] *= sc;
                p[2 * n + i] *= sc;
            }
        }
        for (int32_t a = 0; a < 3 * n; ++a) p[a] += 0.5 * h * f[a];
        for (int32_t a = 0; a < 3 * n; ++a) r[a] += h * p[a];
        wrap_xz(c, r);
        k += 1;
        lattice_at(c, rl0, v, dt, k, rl);
        orc_ch_forces(c, r, rl, f, fo);
        for (int32_t a = 0; a < 3 * n; ++a) p[a] += 0.5 * h * f[a];
        if (q > 0.0) {
            const double sc = exp(-z * 0.5 * h);
            for (int32_t i = c->n_fluid; i < n; ++i) {
                p[i] *= sc;
                p[n + i] *= sc;
                p[2 * n + i] *= sc;
            }
            z += 0.5 * h * (wall_p2(c, p) - nf_w * t_wall) / q;
        }
        if (obs_out) orc_ch_observables(c, r, p, fo, obs_out + (size_t)s * nobs);
        if (s_out) s_out[s] = fo[4];
        if (energy_out) {
            double ke = 0.0;
            for (int32_t a = 0; a < 3 * n; ++a) ke += 0.5 * p[a] * p[a];
            energy_out[s] = ke + fo[0] + fo[1];
        }
    }
    *zeta = z;
    free(f);
    free(rl);
    return 0;
}

void orc_ch_map(const orc_channel* c, int32_t m, const double* r, const double* p, double zeta,
                const double* rl, double* r_out, double* p_out, double* zeta_out,
                double* rl_out) {
    const int32_t n = c->n, nw = c->n_wall;
    memcpy(r_out, r, sizeof(double) * 3 * (size_t)n);
    memcpy(p_out, p, sizeof(double) * 3 * (size_t)n);
    memcpy(rl_out, rl, sizeof(double) * 3 * (size_t)nw);
    *zeta_out = zeta;
    if (m == 1 || m == 3) {
        /* time reversal of momenta (and of the thermostat variable) */
        for (int32_t a = 0; a < 3 * n; ++a) p_out[a] = -p_out[a];
        *zeta_out = -zeta;
    }
    if (m == 2 || m == 3) {
        /* x reflection of atoms and lattice sites, x momenta change sign */
        for (int32_t i = 0; i < n; ++i) {
            r_out[i] = r[i] == 0.0 ? 0.0 : c->lx - r[i];
            p_out[i] = -p_out[i];
        }
        for (int32_t q = 0; q < nw; ++q) rl_out[q] = rl[q] == 0.0 ? 0.0 : c->lx - rl[q];
    }
}

/* ---- daughters in parallel ------------------------------------------------------------ */

typedef struct {
    const orc_channel* c;
    double t_wall, q, dt;
    const double *sr, *sp, *sz, *rl;
    const int32_t *state_of, *map_of;
    const double* v_of;
    int32_t nsteps, nd;
    double *obs, *s0;
    int32_t next;
    pthread_mutex_t mu;
} ch_job;

static void* ch_worker(void* arg) {
    ch_job* J = (ch_job*)arg;
    const orc_channel* c = J->c;
    const int32_t n = c->n, nw = c->n_wall;
    const int nobs = 1 + c->n_bins;
    double* r = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* p = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* rl = (double*)malloc(sizeof(double) * 3 * (size_t)nw);
    double* sser = (double*)malloc(sizeof(double) * ((size_t)J->nsteps + 1));
    for (;;) {
        pthread_mutex_lock(&J->mu);
        const int32_t d = J->next++;
        pthread_mutex_unlock(&J->mu);
        if (d >= J->nd) break;
        const int32_t st = J->state_of[d];
        double z;
        orc_ch_map(c, J->map_of[d], J->sr + (size_t)st * 3 * n, J->sp + (size_t)st * 3 * n,
                   J->sz[st], J->rl, r, p, &z, rl);
        orc_ch_run(c, J->t_wall, J->q, J->dt, J->v_of[d], r, p, &z, rl, 0, J->nsteps,
                   J->obs + (size_t)d * ((size_t)J->nsteps + 1) * nobs, sser, NULL);
        J->s0[d] = sser[0];
    }
    free(r);
    free(p);
    free(rl);
    free(sser);
    return NULL;
}

int32_t orc_ch_run_daughters(const orc_channel* c, double t_wall, double q, double dt,
                             const double* states_r, const double* states_p,
                             const double* states_zeta, const double* rl, const int32_t* state_of,
                             const int32_t* map_of, const double* v_of, int32_t n_daughters,
                             int32_t nsteps, double* obs, double* s0, int32_t nthreads) {
    ch_job J;
    J.c = c;
    J.t_wall = t_wall;
    J.q = q;
    J.dt = dt;
    J.sr = states_r;
    J.sp = states_p;
    J.sz = states_zeta;
    J.rl = rl;
    J.state_of = state_of;
    J.map_of = map_of;
    J.v_of = v_of;
    J.nsteps = nsteps;
    J.nd = n_daughters;
    J.obs = obs;
    J.s0 = s0;
    J.next = 0;
    pthread_mutex_init(&J.mu, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, ch_worker, &J);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.mu);
    return nthreads;
}
