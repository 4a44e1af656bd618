/*
 * ttcf_oracle.c -- plain FP64 CPU oracle for the TTCF daughter path of arxiv 2312.02990.
 *
 * TEST INFRASTRUCTURE: only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg use this file. It shares no code with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math, no vector intrinsics),
 * so every expression below is evaluated as written, one rounding per operation.
 *
 * What each part follows in the paper:
 *   - WCA / wetting-factor LJ pair potential: Example 1 (WCA equation, shift for continuity
 *     at r_c) and Example 2 (LJ with c_ij).
 *   - SLLOD equations of motion, Eq. (system1), under the sliding-brick (Lees-Edwards)
 *     boundaries that the paper equates with LAMMPS' box deformation (Example 1).
 *   - Equilibrium mother dynamics with a Nose-Hoover thermostat (Eq. system1 with
 *     gamma_dot = 0), sampled periodically (Mathematical Framework; Alg. LAMMPS SCRIPT).
 *   - The mappings of Eq. (mappings).
 *   - P_xy and the dissipation function of Eq. (TTCF1); Omega = -(V/T) gamma_dot P_xy in the
 *     pressure-tensor sign convention (the paper writes P_xy as a shear stress).
 *   - Planar elongational flow, a field the Introduction names as one TTCF extends to, with
 *     mappings of its own (Section Mathematical Framework: other fields need other mappings).
 * Where the paper does not fix a detail the chosen reading is stated at the spot.
 */
#include "ttcf_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------------ */
/* pair potential                                                                        */
/* ------------------------------------------------------------------------------------ */

/* phi(r) = 4[(1/r)^12 - c (1/r)^6] + shift, force on i from j = fscal * r_ij with
 * fscal = -phi'(r)/r = 48 r^-14 - 24 c r^-8. */
static void pair_eval(const orc_box* b, double r2, double* fscal, double* phi) {
    double s = 1.0 / r2;
    double s3 = s * s * s;
    double s6 = s3 * s3;
    *fscal = (48.0 * s6 - 24.0 * b->c_attr * s3) * s;
    *phi = 4.0 * (s6 - b->c_attr * s3) + b->u_shift;
}

/* Minimum-image separation r_i - r_j in the sliding-brick box with LE offset dxle:
 * the y image is chosen first; crossing it shifts x by the offset, then x and z are
 * wrapped periodically. */
static void min_image(const orc_box* b, double dxle, double xi, double yi, double zi,
                      double xj, double yj, double zj, double d[3]) {
    double dy = yi - yj;
    double ny = rint(dy / b->ly);
    dy = dy - ny * b->ly;
    double dx = xi - xj;
    dx = dx - ny * dxle;
    dx = dx - b->lx * rint(dx / b->lx);
    double dz = zi - zj;
    dz = dz - b->lz * rint(dz / b->lz);
    d[0] = dx;
    d[1] = dy;
    d[2] = dz;
}

/* ------------------------------------------------------------------------------------ */
/* cell list                                                                             */
/* ------------------------------------------------------------------------------------ */

int32_t orc_grid_dims(const orc_box* b, double side, int32_t dims[3]) {
    dims[0] = (int32_t)floor(b->lx / side);
    dims[1] = (int32_t)floor(b->ly / side);
    dims[2] = (int32_t)floor(b->lz / side);
    if (dims[0] < 4 || dims[1] < 3 || dims[2] < 3) return -1;
    return 0;
}

int32_t orc_cell_dims(const orc_box* b, int32_t dims[3]) { return orc_grid_dims(b, b->rc, dims); }

static int32_t cell_coord(double x, int32_t n, double inv_w) {
    int32_t c = (int32_t)floor(x * inv_w);
    if (c < 0) c = 0;
    if (c > n - 1) c = n - 1;
    return c;
}

int32_t orc_cell_list(const orc_box* b, const double* r, int32_t* cell_of, int32_t* order,
                      int32_t* start) {
    int32_t d[3];
    if (orc_cell_dims(b, d) != 0) return -1;
    return orc_cell_list_grid(b, d, r, cell_of, order, start);
}

int32_t orc_cell_list_grid(const orc_box* b, const int32_t d[3], const double* r,
                           int32_t* cell_of, int32_t* order, int32_t* start) {
    if (d[0] < 4 || d[1] < 3 || d[2] < 3) return -1;
    const int32_t n = b->n;
    const int32_t ncell = d[0] * d[1] * d[2];
    const double inv[3] = {(double)d[0] / b->lx, (double)d[1] / b->ly, (double)d[2] / b->lz};
    const double* x = r;
    const double* y = r + n;
    const double* z = r + 2 * n;
    for (int32_t c = 0; c <= ncell; ++c) start[c] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t cx = cell_coord(x[i], d[0], inv[0]);
        int32_t cy = cell_coord(y[i], d[1], inv[1]);
        int32_t cz = cell_coord(z[i], d[2], inv[2]);
        cell_of[i] = cx + d[0] * (cy + d[1] * cz);
        start[cell_of[i] + 1] += 1;
    }
    for (int32_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)ncell);
    if (!fill) return -2;
    for (int32_t c = 0; c < ncell; ++c) fill[c] = start[c];
    for (int32_t i = 0; i < n; ++i) order[fill[cell_of[i]]++] = i; /* ascending atom id */
    free(fill);
    return 0;
}

/* Visit every candidate j of atom i through the 27-cell neighbourhood. Rows of cells that
 * lie across the y boundary are images displaced by +-dxle in x, so for them the x range
 * is recomputed from the displaced image: all cells whose image overlaps
 * [cx*w - rc, (cx+1)*w + rc] (plus a tiny margin for rounding of the cell index). */
typedef void (*visit_fn)(void* ctx, int32_t i, int32_t j);

static void for_each_candidate(const orc_box* b, double dxle, const int32_t d[3],
                               const int32_t* cell_of, const int32_t* order,
                               const int32_t* start, int32_t i, double reach, visit_fn fn,
                               void* ctx) {
    const double wx = b->lx / (double)d[0];
    const int32_t c = cell_of[i];
    const int32_t cx = c % d[0];
    const int32_t cy = (c / d[0]) % d[1];
    const int32_t cz = c / (d[0] * d[1]);
    const double margin = 1e-9;
    for (int32_t dz = -1; dz <= 1; ++dz) {
        int32_t zz = (cz + dz + d[2]) % d[2];
        for (int32_t dy = -1; dy <= 1; ++dy) {
            int32_t yy = cy + dy;
            double img = 0.0;
            if (yy < 0) {
                yy += d[1];
                img = -1.0;
            } else if (yy >= d[1]) {
                yy -= d[1];
                img = 1.0;
            }
            double sh = img * dxle;
            int32_t lo = (int32_t)floor(((double)cx * wx - reach - margin - sh) / wx);
            int32_t hi = (int32_t)floor(((double)(cx + 1) * wx + reach + margin - sh) / wx);
            if (hi - lo + 1 > d[0]) hi = lo + d[0] - 1;
            for (int32_t xx = lo; xx <= hi; ++xx) {
                int32_t cxx = ((xx % d[0]) + d[0]) % d[0];
                int32_t cell = cxx + d[0] * (yy + d[1] * zz);
                for (int32_t s = start[cell]; s < start[cell + 1]; ++s) {
                    int32_t j = order[s];
                    if (j != i) fn(ctx, i, j);
                }
            }
        }
    }
}

typedef struct {
    const orc_box* b;
    double dxle;
    const double* r;
    double rc2;
    double fi[3];
    double u, w, npair;
} force_ctx;

static void force_visit(void* vctx, int32_t i, int32_t j) {
    force_ctx* c = (force_ctx*)vctx;
    const int32_t n = c->b->n;
    const double* r = c->r;
    double d[3];
    min_image(c->b, c->dxle, r[i], r[n + i], r[2 * n + i], r[j], r[n + j], r[2 * n + j], d);
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 < c->rc2) {
        double fs, phi;
        pair_eval(c->b, r2, &fs, &phi);
        c->fi[0] += fs * d[0];
        c->fi[1] += fs * d[1];
        c->fi[2] += fs * d[2];
        /* every unordered pair is visited twice: half of each contribution */
        c->u += 0.5 * phi;
        c->w += 0.5 * (d[0] * (fs * d[1]));
        c->npair += 0.5;
    }
}

int32_t orc_forces(const orc_box* b, double dxle, const double* r, double* f, double* out) {
    int32_t d[3];
    if (orc_cell_dims(b, d) != 0) return -1;
    const int32_t n = b->n;
    const int32_t ncell = d[0] * d[1] * d[2];
    int32_t* cell_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* start = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ncell + 1));
    if (!cell_of || !order || !start) {
        free(cell_of);
        free(order);
        free(start);
        return -2;
    }
    orc_cell_list(b, r, cell_of, order, start);
    force_ctx c;
    c.b = b;
    c.dxle = dxle;
    c.r = r;
    c.rc2 = b->rc * b->rc;
    c.u = 0.0;
    c.w = 0.0;
    c.npair = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        c.fi[0] = c.fi[1] = c.fi[2] = 0.0;
        for_each_candidate(b, dxle, d, cell_of, order, start, i, b->rc, force_visit, &c);
        f[i] = c.fi[0];
        f[n + i] = c.fi[1];
        f[2 * n + i] = c.fi[2];
    }
    out[0] = c.u;
    out[1] = c.w;
    out[2] = c.npair;
    free(cell_of);
    free(order);
    free(start);
    return 0;
}

int32_t orc_forces_brute(const orc_box* b, double dxle, const double* r, double* f,
                         double* out) {
    const int32_t n = b->n;
    const double rc2 = b->rc * b->rc;
    double u = 0.0, w = 0.0, npair = 0.0;
    for (int32_t k = 0; k < 3 * n; ++k) f[k] = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t j = i + 1; j < n; ++j) {
            /* every image of j: r_j + (mx*Lx + my*dxle, my*Ly, mz*Lz) */
            for (int32_t my = -2; my <= 2; ++my) {
                for (int32_t mx = -3; mx <= 3; ++mx) {
                    for (int32_t mz = -2; mz <= 2; ++mz) {
                        double dx = r[i] - (r[j] + (double)mx * b->lx + (double)my * dxle);
                        double dy = r[n + i] - (r[n + j] + (double)my * b->ly);
                        double dz = r[2 * n + i] - (r[2 * n + j] + (double)mz * b->lz);
                        double r2 = dx * dx + dy * dy + dz * dz;
                        if (r2 < rc2) {
                            double fs, phi;
                            pair_eval(b, r2, &fs, &phi);
                            f[i] += fs * dx;
                            f[n + i] += fs * dy;
                            f[2 * n + i] += fs * dz;
                            f[j] -= fs * dx;
                            f[n + j] -= fs * dy;
                            f[2 * n + j] -= fs * dz;
                            u += phi;
                            w += dx * (fs * dy);
                            npair += 1.0;
                        }
                    }
                }
            }
        }
    }
    out[0] = u;
    out[1] = w;
    out[2] = npair;
    return 0;
}

typedef struct {
    const orc_box* b;
    double dxle;
    const double* r;
    double rl2;
    int64_t cap, cnt;
    int32_t *pi, *pj;
} pair_ctx;

static void pair_visit(void* vctx, int32_t i, int32_t j) {
    pair_ctx* c = (pair_ctx*)vctx;
    if (j <= i) return;
    const int32_t n = c->b->n;
    const double* r = c->r;
    double d[3];
    min_image(c->b, c->dxle, r[i], r[n + i], r[2 * n + i], r[j], r[n + j], r[2 * n + j], d);
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 < c->rl2) {
        if (c->cnt < c->cap) {
            c->pi[c->cnt] = i;
            c->pj[c->cnt] = j;
        }
        c->cnt += 1;
    }
}

static int cmp_pair(const void* a, const void* b) {
    const int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

static void sort_pairs(int64_t cnt, int32_t* pi, int32_t* pj) {
    int64_t* key = (int64_t*)malloc(sizeof(int64_t) * (size_t)(cnt > 0 ? cnt : 1));
    for (int64_t k = 0; k < cnt; ++k) key[k] = ((int64_t)pi[k] << 32) | (int64_t)pj[k];
    qsort(key, (size_t)cnt, sizeof(int64_t), cmp_pair);
    for (int64_t k = 0; k < cnt; ++k) {
        pi[k] = (int32_t)(key[k] >> 32);
        pj[k] = (int32_t)(key[k] & 0xffffffff);
    }
    free(key);
}

/* Pair list of radius rlist. Up to rc it walks the canonical cell list; a Verlet list of a
 * larger radius (rc plus a skin) walks a grid whose cells are at least rlist wide, so that the
 * 27-cell neighbourhood still holds every candidate. */
int64_t orc_pairs(const orc_box* b, double dxle, const double* r, double rlist, int64_t cap,
                  int32_t* pi, int32_t* pj) {
    int32_t d[3];
    if (!(rlist > 0.0) || orc_grid_dims(b, rlist > b->rc ? rlist : b->rc, d) != 0) return -2;
    const int32_t n = b->n;
    const int32_t ncell = d[0] * d[1] * d[2];
    int32_t* cell_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* start = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ncell + 1));
    orc_cell_list_grid(b, d, r, cell_of, order, start);
    pair_ctx c = {b, dxle, r, rlist * rlist, cap, 0, pi, pj};
    for (int32_t i = 0; i < n; ++i)
        for_each_candidate(b, dxle, d, cell_of, order, start, i, rlist, pair_visit, &c);
    free(cell_of);
    free(order);
    free(start);
    if (c.cnt > cap) return -1;
    sort_pairs(c.cnt, pi, pj);
    return c.cnt;
}

int64_t orc_pairs_brute(const orc_box* b, double dxle, const double* r, double rlist,
                        int64_t cap, int32_t* pi, int32_t* pj) {
    const int32_t n = b->n;
    const double rl2 = rlist * rlist;
    int64_t cnt = 0;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t j = i + 1; j < n; ++j) {
            double d[3];
            min_image(b, dxle, r[i], r[n + i], r[2 * n + i], r[j], r[n + j], r[2 * n + j], d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < rl2) {
                if (cnt < cap) {
                    pi[cnt] = i;
                    pj[cnt] = j;
                }
                ++cnt;
            }
        }
    }
    return cnt > cap ? -1 : cnt;
}

/* ------------------------------------------------------------------------------------ */
/* observables and mappings                                                              */
/* ------------------------------------------------------------------------------------ */

static double kinetic(int32_t n, const double* p) {
    double s = 0.0;
    for (int32_t k = 0; k < 3 * n; ++k) s += p[k] * p[k];
    return 0.5 * s;
}

static double sum_pxpy(int32_t n, const double* p) {
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += p[i] * p[n + i];
    return s;
}

double orc_vpxy(const orc_box* b, double dxle, const double* r, const double* p) {
    double* f = (double*)malloc(sizeof(double) * 3 * (size_t)b->n);
    double out[3];
    orc_forces(b, dxle, r, f, out);
    free(f);
    return sum_pxpy(b->n, p) + out[1];
}

/* The pair parts of the pressure tensor's diagonal and the potential energy, for
 * orc_observables. Each unordered pair is visited twice, so each visit adds half. */
typedef struct {
    const orc_box* b;
    double dxle;
    const double* r;
    double rc2;
    double w[3];
    double u;
} obs_ctx;

static void obs_visit(void* vctx, int32_t i, int32_t j) {
    obs_ctx* c = (obs_ctx*)vctx;
    const int32_t n = c->b->n;
    const double* r = c->r;
    double d[3];
    min_image(c->b, c->dxle, r[i], r[n + i], r[2 * n + i], r[j], r[n + j], r[2 * n + j], d);
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 < c->rc2) {
        double fs, phi;
        pair_eval(c->b, r2, &fs, &phi);
        for (int a = 0; a < 3; ++a) c->w[a] += 0.5 * (d[a] * (fs * d[a]));
        c->u += 0.5 * phi;
    }
}

int32_t orc_observables(const orc_box* b, double dxle, const double* r, const double* p,
                        int32_t n_slabs, double* out) {
    int32_t d[3];
    if (n_slabs < 1 || orc_cell_dims(b, d) != 0) return -1;
    const int32_t n = b->n;
    const int32_t ncell = d[0] * d[1] * d[2];
    int32_t* cell_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* start = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ncell + 1));
    double* slab = (double*)calloc((size_t)n_slabs, sizeof(double));
    if (!cell_of || !order || !start || !slab) {
        free(cell_of);
        free(order);
        free(start);
        free(slab);
        return -2;
    }
    orc_cell_list(b, r, cell_of, order, start);
    obs_ctx c;
    c.b = b;
    c.dxle = dxle;
    c.r = r;
    c.rc2 = b->rc * b->rc;
    c.w[0] = c.w[1] = c.w[2] = 0.0;
    c.u = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for_each_candidate(b, dxle, d, cell_of, order, start, i, b->rc, obs_visit, &c);
    /* kinetic parts: sum_i p_a p_a (m = 1) */
    double kk[3] = {0.0, 0.0, 0.0};
    for (int32_t a = 0; a < 3; ++a)
        for (int32_t i = 0; i < n; ++i) kk[a] += p[a * n + i] * p[a * n + i];
    for (int32_t i = 0; i < n; ++i) {
        int32_t s = (int32_t)floor(r[n + i] * ((double)n_slabs / b->ly));
        if (s < 0) s = 0;
        if (s > n_slabs - 1) s = n_slabs - 1;
        slab[s] += p[i];
    }
    const double vol = b->lx * b->ly * b->lz;
    out[0] = ((kk[0] + c.w[0]) - (kk[1] + c.w[1])) / vol;
    out[1] = ((kk[1] + c.w[1]) - (kk[2] + c.w[2])) / vol;
    out[2] = (0.5 * (kk[0] + kk[1] + kk[2]) + c.u) / (double)n;
    for (int32_t s = 0; s < n_slabs; ++s) out[3 + s] = slab[s] / (vol / (double)n_slabs);
    free(cell_of);
    free(order);
    free(start);
    free(slab);
    return 0;
}

void orc_map(const orc_box* b, int32_t m, const double* r, const double* p, double* r_out,
             double* p_out) {
    const int32_t n = b->n;
    memcpy(r_out, r, sizeof(double) * 3 * (size_t)n);
    memcpy(p_out, p, sizeof(double) * 3 * (size_t)n);
    if (m == 1) {
        for (int32_t k = 0; k < 3 * n; ++k) p_out[k] = -p[k];
    } else if (m == 2 || m == 3) {
        for (int32_t i = 0; i < n; ++i) {
            /* x -> -x, brought back into [0, Lx) */
            r_out[i] = (r[i] == 0.0) ? 0.0 : b->lx - r[i];
        }
        if (m == 2) {
            for (int32_t i = 0; i < n; ++i) p_out[i] = -p[i];
        } else {
            for (int32_t i = 0; i < n; ++i) {
                p_out[n + i] = -p[n + i];
                p_out[2 * n + i] = -p[2 * n + i];
            }
        }
    }
}

/* Periodic wrap of one coordinate into [0, L). */
static double wrap1(double x, double l) {
    if (x >= l) {
        x -= l;
        if (x >= l) x -= l * floor(x / l);
    } else if (x < 0.0) {
        x += l;
        if (x < 0.0) x -= l * floor(x / l);
        if (x >= l) x = 0.0; /* x was a tiny negative number: x + L rounded to L */
    }
    return x;
}

/* Sliding-brick wrap: crossing the top (bottom) face moves x by -dxle (+dxle). */
static void wrap_le(const orc_box* b, double dxle, double* r) {
    const int32_t n = b->n;
    for (int32_t i = 0; i < n; ++i) {
        double x = r[i], y = r[n + i];
        if (y >= b->ly) {
            y -= b->ly;
            x -= dxle;
        } else if (y < 0.0) {
            y += b->ly;
            x += dxle;
            if (y >= b->ly) y = 0.0;
        }
        r[i] = wrap1(x, b->lx);
        r[n + i] = y;
        r[2 * n + i] = wrap1(r[2 * n + i], b->lz);
    }
}

/* ------------------------------------------------------------------------------------ */
/* mother: Nose-Hoover equilibrium dynamics                                              */
/* ------------------------------------------------------------------------------------ */

/* One symmetric step (h = dt):
 *   zeta += (h/2)(sum p^2 - nf T)/Q;  p *= exp(-zeta h/2);  p += (h/2) F;
 *   r += h p (wrap);  F = F(r);  p += (h/2) F;  p *= exp(-zeta h/2);
 *   zeta += (h/2)(sum p^2 - nf T)/Q.
 * The paper's thermostat equation (Eq. system1) gives the zeta dynamics; the mass Q is
 * not stated there and is a parameter here. */
int32_t orc_nh_run(const orc_box* b, double temperature, double q, double nf, double dt,
                   double* r, double* p, double* zeta, int64_t nsteps, double* vpxy_out,
                   double* ke_out, double* pe_out) {
    const int32_t n = b->n;
    double* f = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    if (!f) return -2;
    double out[3];
    if (orc_forces(b, 0.0, r, f, out) != 0) {
        free(f);
        return -1;
    }
    const double h = dt;
    double z = *zeta;
    if (vpxy_out) vpxy_out[0] = sum_pxpy(n, p) + out[1];
    if (ke_out) ke_out[0] = kinetic(n, p);
    if (pe_out) pe_out[0] = out[0];
    for (int64_t s = 1; s <= nsteps; ++s) {
        double p2 = 2.0 * kinetic(n, p);
        z += 0.5 * h * (p2 - nf * temperature) / q;
        double sc = exp(-z * 0.5 * h);
        for (int32_t k = 0; k < 3 * n; ++k) p[k] *= sc;
        for (int32_t k = 0; k < 3 * n; ++k) p[k] += 0.5 * h * f[k];
        for (int32_t k = 0; k < 3 * n; ++k) r[k] += h * p[k];
        wrap_le(b, 0.0, r);
        orc_forces(b, 0.0, r, f, out);
        for (int32_t k = 0; k < 3 * n; ++k) p[k] += 0.5 * h * f[k];
        sc = exp(-z * 0.5 * h);
        for (int32_t k = 0; k < 3 * n; ++k) p[k] *= sc;
        p2 = 2.0 * kinetic(n, p);
        z += 0.5 * h * (p2 - nf * temperature) / q;
        if (vpxy_out) vpxy_out[s] = sum_pxpy(n, p) + out[1];
        if (ke_out) ke_out[s] = kinetic(n, p);
        if (pe_out) pe_out[s] = out[0];
    }
    *zeta = z;
    free(f);
    return 0;
}

int32_t orc_mother_sample(const orc_box* b, double temperature, double q, double nf, double dt,
                          double* r, double* p, double* zeta, int64_t n_equil,
                          int32_t n_states, int64_t steps_between, double* states_r,
                          double* states_p) {
    return orc_mother_sample_zeta(b, temperature, q, nf, dt, r, p, zeta, n_equil, n_states,
                                  steps_between, states_r, states_p, 0);
}

int32_t orc_mother_sample_zeta(const orc_box* b, double temperature, double q, double nf,
                               double dt, double* r, double* p, double* zeta, int64_t n_equil,
                               int32_t n_states, int64_t steps_between, double* states_r,
                               double* states_p, double* states_zeta) {
    const size_t sz = 3 * (size_t)b->n;
    int32_t rc = orc_nh_run(b, temperature, q, nf, dt, r, p, zeta, n_equil, 0, 0, 0);
    if (rc) return rc;
    for (int32_t s = 0; s < n_states; ++s) {
        rc = orc_nh_run(b, temperature, q, nf, dt, r, p, zeta, steps_between, 0, 0, 0);
        if (rc) return rc;
        memcpy(states_r + (size_t)s * sz, r, sizeof(double) * sz);
        memcpy(states_p + (size_t)s * sz, p, sizeof(double) * sz);
        if (states_zeta) states_zeta[s] = *zeta;
    }
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* daughters: SLLOD with Lees-Edwards boundaries and a Gaussian isokinetic constraint    */
/* ------------------------------------------------------------------------------------ */

static double le_offset(const orc_box* b, double gamma_dot, double dt, int64_t k) {
    return fmod(gamma_dot * b->ly * ((double)k * dt), b->lx);
}

/* Exact flow, over a time tau, of the momentum equation dp/dt = F - alpha p with F held
 * fixed and alpha = (F.p)/(p.p) the Gaussian multiplier that keeps p.p constant
 * (closed form of Zhang, J. Chem. Phys. 106, 6102 (1997)):
 *   a = F.p/p.p, b = F.F/p.p, q = sqrt(b),
 *   s(tau) = (a/b)(cosh(q tau) - 1) + sinh(q tau)/q,  s'(tau) = (a/q) sinh(q tau) + cosh(q tau),
 *   p(tau) = (p(0) + F s(tau)) / s'(tau).
 * cosh - 1 is formed as 2 sinh^2(q tau/2) to avoid cancellation. */
void orc_iso_kick(int32_t n, double* p, const double* f, double tau) {
    double pp = 0.0, fp = 0.0, ff = 0.0;
    for (int32_t c = 0; c < 3 * n; ++c) {
        pp += p[c] * p[c];
        fp += f[c] * p[c];
        ff += f[c] * f[c];
    }
    double a = fp / pp;
    double b = ff / pp;
    double ch1_b, sh_q; /* (cosh(q tau) - 1)/b and sinh(q tau)/q */
    if (b > 0.0) {
        double q = sqrt(b);
        double hs = sinh(0.5 * q * tau) / q;
        ch1_b = 2.0 * hs * hs;
        sh_q = sinh(q * tau) / q;
    } else {
        ch1_b = 0.5 * tau * tau;
        sh_q = tau;
    }
    double s = a * ch1_b + sh_q;
    double sdot = a * sh_q + (1.0 + b * ch1_b);
    for (int32_t c = 0; c < 3 * n; ++c) p[c] = (p[c] + f[c] * s) / sdot;
}

/* Exact flow, over a time tau, of dpx/dt = -gamma_dot py - alpha px, dpy/dt = -alpha py,
 * dpz/dt = -alpha pz with alpha = -gamma_dot (sum px py)/(p.p): alpha multiplies every
 * component, so the solution is the unconstrained shear flow px -> px - gamma_dot tau py
 * scaled back to the initial p.p. */
void orc_iso_shear(int32_t n, double* p, double gamma_dot, double tau) {
    double pp0 = 0.0, pp1 = 0.0;
    for (int32_t c = 0; c < 3 * n; ++c) pp0 += p[c] * p[c];
    for (int32_t i = 0; i < n; ++i) p[i] -= tau * gamma_dot * p[n + i];
    for (int32_t c = 0; c < 3 * n; ++c) pp1 += p[c] * p[c];
    double g = sqrt(pp0 / pp1);
    for (int32_t c = 0; c < 3 * n; ++c) p[c] *= g;
}

/* One step (h = dt) of Eq. (system1) with the Nose-Hoover term replaced by the Gaussian
 * isokinetic multiplier alpha = (sum F.p - gamma_dot sum px py)/(sum p.p) (reading: the
 * daughters are isokinetic). Symmetric splitting of the vector field into a shear part S,
 * a force part K and a streaming part D, each integrated exactly:
 *   S(h/2) K(h/2) D(h) [k += 1, new LE offset, sliding-brick wrap, F = F(r)] K(h/2) S(h/2)
 * with
 *   S: dpx/dt = -gamma_dot py (- alpha_S p under the constraint)
 *   K: dp/dt = F (- alpha_K p under the constraint)
 *   D: dx/dt = px + gamma_dot y, dy/dt = py, dz/dt = pz:
 *      x += h px + h gamma_dot (y + (h/2) py); y += h py; z += h pz.
 * Each constrained part keeps p.p fixed, so the step is second order, time reversible and
 * isokinetic; a final rescale to K0 only removes round-off drift (its factor is 1 to
 * within a few ulps). gik = 0 gives the adiabatic SLLOD step (no multiplier). */
static int32_t sllod_run(const orc_box* b, double gamma_dot, double dt, int32_t gik, double k0,
                         double* r, double* p, int64_t* kstep, int64_t nsteps, double* vpxy_out,
                         double* ke_out, double* pe_out, int32_t n_slabs, double* obs_out) {
    const int32_t n = b->n;
    const size_t nobs = 3 + (size_t)(n_slabs > 0 ? n_slabs : 0);
    double* f = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    if (!f) return -2;
    double* x = r;
    double* y = r + n;
    double* z = r + 2 * n;
    double* px = p;
    double* py = p + n;
    double* pz = p + 2 * n;
    double out[3];
    int64_t k = *kstep;
    double dxle = le_offset(b, gamma_dot, dt, k);
    if (orc_forces(b, dxle, r, f, out) != 0) {
        free(f);
        return -1;
    }
    if (k0 <= 0.0) k0 = kinetic(n, p);
    const double h = dt;
    if (vpxy_out) vpxy_out[0] = sum_pxpy(n, p) + out[1];
    if (ke_out) ke_out[0] = kinetic(n, p);
    if (pe_out) pe_out[0] = out[0];
    if (obs_out) orc_observables(b, dxle, r, p, n_slabs, obs_out);
    for (int64_t s = 1; s <= nsteps; ++s) {
        if (gik) {
            orc_iso_shear(n, p, gamma_dot, 0.5 * h);
            orc_iso_kick(n, p, f, 0.5 * h);
        } else {
            for (int32_t i = 0; i < n; ++i) px[i] -= 0.5 * h * gamma_dot * py[i];
            for (int32_t c = 0; c < 3 * n; ++c) p[c] += 0.5 * h * f[c];
        }
        for (int32_t i = 0; i < n; ++i) {
            x[i] += h * px[i] + h * gamma_dot * (y[i] + 0.5 * h * py[i]);
            y[i] += h * py[i];
            z[i] += h * pz[i];
        }
        k += 1;
        dxle = le_offset(b, gamma_dot, dt, k);
        wrap_le(b, dxle, r);
        orc_forces(b, dxle, r, f, out);
        if (gik) {
            orc_iso_kick(n, p, f, 0.5 * h);
            orc_iso_shear(n, p, gamma_dot, 0.5 * h);
            double lam = sqrt(k0 / kinetic(n, p));
            for (int32_t c = 0; c < 3 * n; ++c) p[c] *= lam;
        } else {
            for (int32_t c = 0; c < 3 * n; ++c) p[c] += 0.5 * h * f[c];
            for (int32_t i = 0; i < n; ++i) px[i] -= 0.5 * h * gamma_dot * py[i];
        }
        if (vpxy_out) vpxy_out[s] = sum_pxpy(n, p) + out[1];
        if (ke_out) ke_out[s] = kinetic(n, p);
        if (pe_out) pe_out[s] = out[0];
        if (obs_out) orc_observables(b, dxle, r, p, n_slabs, obs_out + (size_t)s * nobs);
    }
    *kstep = k;
    free(f);
    return 0;
}

int32_t orc_sllod_run(const orc_box* b, double gamma_dot, double dt, int32_t gik, double k0,
                      double* r, double* p, int64_t* kstep, int64_t nsteps, double* vpxy_out,
                      double* ke_out, double* pe_out) {
    return sllod_run(b, gamma_dot, dt, gik, k0, r, p, kstep, nsteps, vpxy_out, ke_out, pe_out, 0,
                     0);
}

/* One step of Eq. (system1) with its Nose-Hoover multiplier alpha = zeta. Each part is
 * integrated exactly:
 *   Z: d zeta/dt = (sum p^2 - nf T)/Q with p fixed;
 *   T: dp/dt = -zeta p with zeta fixed, p *= exp(-zeta tau);
 *   S: dpx/dt = -gamma_dot py (py fixed);
 *   K: dp/dt = F (F fixed);
 *   D: the streaming of orc_sllod_run.
 * T and S commute (T scales every component). The sequence
 * Z T S K D K S T Z over half steps is symmetric, so the step is second order and time
 * reversible under (p, zeta, gamma_dot) -> (-p, -zeta, -gamma_dot). */
static int32_t nh_sllod_run(const orc_box* b, double gamma_dot, double dt, double temperature,
                            double q, double nf, double* r, double* p, double* zeta,
                            int64_t* kstep, int64_t nsteps, double* vpxy_out, double* ke_out,
                            double* pe_out, double* zeta_out, int32_t n_slabs, double* obs_out) {
    const int32_t n = b->n;
    const size_t nobs = 3 + (size_t)(n_slabs > 0 ? n_slabs : 0);
    double* f = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    if (!f) return -2;
    double* x = r;
    double* y = r + n;
    double* z = r + 2 * n;
    double* px = p;
    double* py = p + n;
    double* pz = p + 2 * n;
    double out[3];
    int64_t k = *kstep;
    double dxle = le_offset(b, gamma_dot, dt, k);
    if (orc_forces(b, dxle, r, f, out) != 0) {
        free(f);
        return -1;
    }
    const double h = dt, tau = 0.5 * dt;
    double zt = *zeta;
    if (vpxy_out) vpxy_out[0] = sum_pxpy(n, p) + out[1];
    if (ke_out) ke_out[0] = kinetic(n, p);
    if (pe_out) pe_out[0] = out[0];
    if (zeta_out) zeta_out[0] = zt;
    if (obs_out) orc_observables(b, dxle, r, p, n_slabs, obs_out);
    for (int64_t s = 1; s <= nsteps; ++s) {
        zt += tau * (2.0 * kinetic(n, p) - nf * temperature) / q;
        double sc = exp(-zt * tau);
        for (int32_t c = 0; c < 3 * n; ++c) p[c] *= sc;
        for (int32_t i = 0; i < n; ++i) px[i] -= tau * gamma_dot * py[i];
        for (int32_t c = 0; c < 3 * n; ++c) p[c] += tau * f[c];
        for (int32_t i = 0; i < n; ++i) {
            x[i] += h * px[i] + h * gamma_dot * (y[i] + tau * py[i]);
            y[i] += h * py[i];
            z[i] += h * pz[i];
        }
        k += 1;
        dxle = le_offset(b, gamma_dot, dt, k);
        wrap_le(b, dxle, r);
        orc_forces(b, dxle, r, f, out);
        for (int32_t c = 0; c < 3 * n; ++c) p[c] += tau * f[c];
        for (int32_t i = 0; i < n; ++i) px[i] -= tau * gamma_dot * py[i];
        sc = exp(-zt * tau);
        for (int32_t c = 0; c < 3 * n; ++c) p[c] *= sc;
        zt += tau * (2.0 * kinetic(n, p) - nf * temperature) / q;
        if (vpxy_out) vpxy_out[s] = sum_pxpy(n, p) + out[1];
        if (ke_out) ke_out[s] = kinetic(n, p);
        if (pe_out) pe_out[s] = out[0];
        if (zeta_out) zeta_out[s] = zt;
        if (obs_out) orc_observables(b, dxle, r, p, n_slabs, obs_out + (size_t)s * nobs);
    }
    *zeta = zt;
    *kstep = k;
    free(f);
    return 0;
}

int32_t orc_nh_sllod_run(const orc_box* b, double gamma_dot, double dt, double temperature,
                         double q, double nf, double* r, double* p, double* zeta,
                         int64_t* kstep, int64_t nsteps, double* vpxy_out, double* ke_out,
                         double* pe_out, double* zeta_out) {
    return nh_sllod_run(b, gamma_dot, dt, temperature, q, nf, r, p, zeta, kstep, nsteps,
                        vpxy_out, ke_out, pe_out, zeta_out, 0, 0);
}

/* ------------------------------------------------------------------------------------ */
/* colour field                                                                          */
/* ------------------------------------------------------------------------------------ */

/* Colour charge of atom i: +1 for even i, -1 for odd i. */
static double colour_charge(int32_t i) { return (i & 1) ? -1.0 : 1.0; }

/* f_tot = f + c_i F_e along x */
static void colour_total(int32_t n, const double* f, double fe, double* ft) {
    memcpy(ft, f, sizeof(double) * 3 * (size_t)n);
    for (int32_t i = 0; i < n; ++i) ft[i] += colour_charge(i) * fe;
}

static double colour_current(int32_t n, const double* p) {
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += colour_charge(i) * p[i];
    return s;
}

int32_t orc_colour_run(const orc_box* b, double fe, double dt, int32_t gik, double k0, double* r,
                       double* p, int64_t nsteps, double* jx_out, double* ke_out,
                       double* pe_out) {
    const int32_t n = b->n;
    double* f = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* ft = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    if (!f || !ft) {
        free(f);
        free(ft);
        return -2;
    }
    double out[3];
    if (orc_forces(b, 0.0, r, f, out) != 0) {
        free(f);
        free(ft);
        return -1;
    }
    colour_total(n, f, fe, ft);
    if (k0 <= 0.0) k0 = kinetic(n, p);
    const double h = dt;
    if (jx_out) jx_out[0] = colour_current(n, p);
    if (ke_out) ke_out[0] = kinetic(n, p);
    if (pe_out) pe_out[0] = out[0];
    for (int64_t s = 1; s <= nsteps; ++s) {
        if (gik)
            orc_iso_kick(n, p, ft, 0.5 * h);
        else
            for (int32_t c = 0; c < 3 * n; ++c) p[c] += 0.5 * h * ft[c];
        for (int32_t c = 0; c < 3 * n; ++c) r[c] += h * p[c];
        wrap_le(b, 0.0, r);
        orc_forces(b, 0.0, r, f, out);
        colour_total(n, f, fe, ft);
        if (gik) {
            orc_iso_kick(n, p, ft, 0.5 * h);
            double lam = sqrt(k0 / kinetic(n, p));
            for (int32_t c = 0; c < 3 * n; ++c) p[c] *= lam;
        } else {
            for (int32_t c = 0; c < 3 * n; ++c) p[c] += 0.5 * h * ft[c];
        }
        if (jx_out) jx_out[s] = colour_current(n, p);
        if (ke_out) ke_out[s] = kinetic(n, p);
        if (pe_out) pe_out[s] = out[0];
    }
    free(f);
    free(ft);
    return 0;
}

/* The colour field with the Nose-Hoover multiplier of Eq. (system1) in place of the Gaussian
 * one: dp/dt = F + c F_e x_hat - zeta p, d zeta/dt = (sum p^2 - nf T)/q. The splitting of
 * nh_sllod_run without its shear part, each part exact:
 *   Z(h/2) T(h/2) K(h/2) D(h) [F(r)] K(h/2) T(h/2) Z(h/2)
 * with K the kick under the total force F + c F_e x_hat. */
int32_t orc_nh_colour_run(const orc_box* b, double fe, double dt, double temperature, double q,
                          double nf, double* r, double* p, double* zeta, int64_t nsteps,
                          double* jx_out, double* ke_out, double* pe_out, double* zeta_out) {
    const int32_t n = b->n;
    double* f = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* ft = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    if (!f || !ft) {
        free(f);
        free(ft);
        return -2;
    }
    double out[3];
    if (orc_forces(b, 0.0, r, f, out) != 0) {
        free(f);
        free(ft);
        return -1;
    }
    colour_total(n, f, fe, ft);
    const double h = dt, tau = 0.5 * dt;
    double zt = *zeta;
    if (jx_out) jx_out[0] = colour_current(n, p);
    if (ke_out) ke_out[0] = kinetic(n, p);
    if (pe_out) pe_out[0] = out[0];
    if (zeta_out) zeta_out[0] = zt;
    for (int64_t s = 1; s <= nsteps; ++s) {
        zt += tau * (2.0 * kinetic(n, p) - nf * temperature) / q;
        double sc = exp(-zt * tau);
        for (int32_t c = 0; c < 3 * n; ++c) p[c] *= sc;
        for (int32_t c = 0; c < 3 * n; ++c) p[c] += tau * ft[c];
        for (int32_t c = 0; c < 3 * n; ++c) r[c] += h * p[c];
        wrap_le(b, 0.0, r);
        orc_forces(b, 0.0, r, f, out);
        colour_total(n, f, fe, ft);
        for (int32_t c = 0; c < 3 * n; ++c) p[c] += tau * ft[c];
        sc = exp(-zt * tau);
        for (int32_t c = 0; c < 3 * n; ++c) p[c] *= sc;
        zt += tau * (2.0 * kinetic(n, p) - nf * temperature) / q;
        if (jx_out) jx_out[s] = colour_current(n, p);
        if (ke_out) ke_out[s] = kinetic(n, p);
        if (pe_out) pe_out[s] = out[0];
        if (zeta_out) zeta_out[s] = zt;
    }
    *zeta = zt;
    free(f);
    free(ft);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* batch of daughters on a thread pool (one daughter per thread at a time)               */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    const orc_box* b;
    double dt;
    const double *states_r, *states_p;
    int32_t n_daughters;
    const int32_t *state_of, *map_of;
    const double* gamma_of;
    int64_t nsteps;
    double *vpxy_out, *r_out, *p_out;
    int32_t tid, nthreads;
    int32_t status;
    /* Nose-Hoover daughters when states_zeta is not NULL */
    const double* states_zeta;
    double temperature, q, nf;
    /* per-step observables of orc_observables when obs_out is not NULL */
    int32_t n_slabs;
    double* obs_out;
    /* colour-field daughters (gamma_of holds F_e, vpxy_out receives V J_x) */
    int32_t colour;
} batch_job;

static void* batch_worker(void* arg) {
    batch_job* jb = (batch_job*)arg;
    const size_t sz = 3 * (size_t)jb->b->n;
    double* r = (double*)malloc(sizeof(double) * sz);
    double* p = (double*)malloc(sizeof(double) * sz);
    jb->status = 0;
    for (int32_t d = jb->tid; d < jb->n_daughters; d += jb->nthreads) {
        const int32_t s = jb->state_of[d];
        orc_map(jb->b, jb->map_of[d], jb->states_r + (size_t)s * sz, jb->states_p + (size_t)s * sz,
                r, p);
        int64_t k = 0;
        int32_t rc;
        double* vp = jb->vpxy_out + (size_t)d * (size_t)(jb->nsteps + 1);
        double* ob = jb->obs_out ? jb->obs_out + (size_t)d * (size_t)(jb->nsteps + 1) *
                                                     (size_t)(3 + jb->n_slabs)
                                 : 0;
        if (jb->colour && jb->states_zeta) {
            double zt = (jb->map_of[d] & 1) ? -jb->states_zeta[s] : jb->states_zeta[s];
            rc = orc_nh_colour_run(jb->b, jb->gamma_of[d], jb->dt, jb->temperature, jb->q, jb->nf,
                                   r, p, &zt, jb->nsteps, vp, 0, 0, 0);
        } else if (jb->colour) {
            rc = orc_colour_run(jb->b, jb->gamma_of[d], jb->dt, 1, 0.0, r, p, jb->nsteps, vp, 0,
                                0);
        } else if (jb->states_zeta) {
            /* the mappings that reverse the momenta (m = 1, 3) reverse the thermostat too */
            double zt = (jb->map_of[d] & 1) ? -jb->states_zeta[s] : jb->states_zeta[s];
            rc = nh_sllod_run(jb->b, jb->gamma_of[d], jb->dt, jb->temperature, jb->q, jb->nf, r,
                              p, &zt, &k, jb->nsteps, vp, 0, 0, 0, jb->n_slabs, ob);
        } else {
            rc = sllod_run(jb->b, jb->gamma_of[d], jb->dt, 1, 0.0, r, p, &k, jb->nsteps, vp, 0, 0,
                           jb->n_slabs, ob);
        }
        if (rc) jb->status = rc;
        if (jb->r_out) memcpy(jb->r_out + (size_t)d * sz, r, sizeof(double) * sz);
        if (jb->p_out) memcpy(jb->p_out + (size_t)d * sz, p, sizeof(double) * sz);
    }
    free(r);
    free(p);
    return 0;
}

static int32_t run_batch(const orc_box* b, double dt, const double* states_r,
                         const double* states_p, const double* states_zeta, double temperature,
                         double q, double nf, int32_t n_daughters, const int32_t* state_of,
                         const int32_t* map_of, const double* gamma_of, int64_t nsteps,
                         int32_t nthreads, double* vpxy_out, double* r_out, double* p_out,
                         int32_t n_slabs, double* obs_out, int32_t colour);

int32_t orc_run_daughters(const orc_box* b, double dt, const double* states_r,
                          const double* states_p, int32_t n_daughters, const int32_t* state_of,
                          const int32_t* map_of, const double* gamma_of, int64_t nsteps,
                          int32_t nthreads, double* vpxy_out, double* r_out, double* p_out) {
    return run_batch(b, dt, states_r, states_p, 0, 0.0, 0.0, 0.0, n_daughters, state_of, map_of,
                     gamma_of, nsteps, nthreads, vpxy_out, r_out, p_out, 0, 0, 0);
}

int32_t orc_run_daughters_nh(const orc_box* b, double dt, double temperature, double q,
                             double nf, const double* states_r, const double* states_p,
                             const double* states_zeta, int32_t n_daughters,
                             const int32_t* state_of, const int32_t* map_of,
                             const double* gamma_of, int64_t nsteps, int32_t nthreads,
                             double* vpxy_out, double* r_out, double* p_out) {
    if (!states_zeta) return -1;
    return run_batch(b, dt, states_r, states_p, states_zeta, temperature, q, nf, n_daughters,
                     state_of, map_of, gamma_of, nsteps, nthreads, vpxy_out, r_out, p_out, 0, 0,
                     0);
}

int32_t orc_run_daughters_obs(const orc_box* b, double dt, double temperature, double q,
                              double nf, const double* states_r, const double* states_p,
                              const double* states_zeta, int32_t n_daughters,
                              const int32_t* state_of, const int32_t* map_of,
                              const double* gamma_of, int64_t nsteps, int32_t nthreads,
                              double* vpxy_out, int32_t n_slabs, double* obs_out) {
    if (n_slabs < 1 || !obs_out) return -1;
    return run_batch(b, dt, states_r, states_p, states_zeta, temperature, q, nf, n_daughters,
                     state_of, map_of, gamma_of, nsteps, nthreads, vpxy_out, 0, 0, n_slabs,
                     obs_out, 0);
}

int32_t orc_run_daughters_colour(const orc_box* b, double dt, const double* states_r,
                                 const double* states_p, const double* states_zeta,
                                 double temperature, double q, double nf, int32_t n_daughters,
                                 const int32_t* state_of, const int32_t* map_of,
                                 const double* fe_of, int64_t nsteps, int32_t nthreads,
                                 double* jx_out, double* r_out, double* p_out) {
    return run_batch(b, dt, states_r, states_p, states_zeta, temperature, q, nf, n_daughters,
                     state_of, map_of, fe_of, nsteps, nthreads, jx_out, r_out, p_out, 0, 0, 1);
}

static int32_t run_batch(const orc_box* b, double dt, const double* states_r,
                         const double* states_p, const double* states_zeta, double temperature,
                         double q, double nf, int32_t n_daughters, const int32_t* state_of,
                         const int32_t* map_of, const double* gamma_of, int64_t nsteps,
                         int32_t nthreads, double* vpxy_out, double* r_out, double* p_out,
                         int32_t n_slabs, double* obs_out, int32_t colour) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > n_daughters) nthreads = n_daughters > 0 ? n_daughters : 1;
    batch_job* jobs = (batch_job*)calloc((size_t)nthreads, sizeof(batch_job));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int32_t t = 0; t < nthreads; ++t) {
        batch_job j = {b,      dt,     states_r, states_p, n_daughters, state_of, map_of,
                       gamma_of, nsteps, vpxy_out, r_out,  p_out,       t,        nthreads, 0,
                       states_zeta, temperature, q, nf, n_slabs, obs_out, colour};
        jobs[t] = j;
        pthread_create(&th[t], 0, batch_worker, &jobs[t]);
    }
    int32_t status = 0;
    for (int32_t t = 0; t < nthreads; ++t) {
        pthread_join(th[t], 0);
        if (jobs[t].status) status = jobs[t].status;
    }
    free(jobs);
    free(th);
    return status ? status : nthreads;
}

/* ------------------------------------------------------------------------------------ */
/* planar elongational flow (PEF)                                                        */
/* ------------------------------------------------------------------------------------ */
/* The Introduction names elongational flow as a field TTCF extends to, and Section
 * Mathematical Framework notes that another field needs its own mappings. Reading used
 * here: the SLLOD equations of Eq. (system1) with the velocity gradient
 * grad u = diag(rate, -rate, 0) in place of the shear,
 *   dr/dt = p + r . grad u,  dp/dt = F - p . grad u - alpha p,
 * the Gaussian isokinetic alpha, and an orthorhombic box that deforms with the flow:
 *   L_x = L_x0 exp(e), L_y = L_y0 exp(-e), L_z = L_z0, e = e0 + rate (k dt)
 * (the volume is conserved). Daughters are short transients, so no reproducible
 * (Kraynik-Reinelt) lattice is needed; the box must keep every edge above 2 r_c.
 * B = P_xx - P_yy and Omega = -(V/T) grad u : P = -(V/T) rate (P_xx - P_yy). */

static void pef_box(const orc_box* b0, double e, orc_box* bk) {
    *bk = *b0;
    bk->lx = b0->lx * exp(e);
    bk->ly = b0->ly * exp(-e);
}

/* Forces by a plain sum over all pairs i < j with the minimum image of the orthorhombic box
 * (valid while every edge exceeds 2 r_c). out[0] = U, out[1] = W_xx - W_yy =
 * sum_{i<j} (x_ij F_x,ij - y_ij F_y,ij), out[2] = interacting pairs. */
int32_t orc_pef_forces(const orc_box* b, const double* r, double* f, double* out) {
    const int32_t n = b->n;
    if (!(b->lx > 2.0 * b->rc && b->ly > 2.0 * b->rc && b->lz > 2.0 * b->rc)) return -1;
    const double rc2 = b->rc * b->rc;
    double u = 0.0, w = 0.0, npair = 0.0;
    for (int32_t k = 0; k < 3 * n; ++k) f[k] = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t j = i + 1; j < n; ++j) {
            double dx = r[i] - r[j];
            double dy = r[n + i] - r[n + j];
            double dz = r[2 * n + i] - r[2 * n + j];
            dx -= b->lx * rint(dx / b->lx);
            dy -= b->ly * rint(dy / b->ly);
            dz -= b->lz * rint(dz / b->lz);
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rc2) {
                double fs, phi;
                pair_eval(b, r2, &fs, &phi);
                f[i] += fs * dx;
                f[n + i] += fs * dy;
                f[2 * n + i] += fs * dz;
                f[j] -= fs * dx;
                f[n + j] -= fs * dy;
                f[2 * n + j] -= fs * dz;
                u += phi;
                w += dx * (fs * dx) - dy * (fs * dy);
                npair += 1.0;
            }
        }
    }
    out[0] = u;
    out[1] = w;
    out[2] = npair;
    return 0;
}

/* Mappings for PEF (reading): bit 0 reverses the momenta (time reversal), bit 1 exchanges
 * the x and y axes of positions and momenta (a symmetry of the cubic box). P_xx - P_yy, and
 * so Omega(0), keeps its sign under time reversal and changes it under the exchange: over
 * m = 0..3 the signs are +, +, -, -. */
void orc_map_pef(const orc_box* b, int32_t m, const double* r, const double* p, double* r_out,
                 double* p_out) {
    const int32_t n = b->n;
    const int32_t sw = (m & 2) ? 1 : 0;
    const double sg = (m & 1) ? -1.0 : 1.0;
    for (int32_t i = 0; i < n; ++i) {
        r_out[i] = r[(sw ? n : 0) + i];
        r_out[n + i] = r[(sw ? 0 : n) + i];
        r_out[2 * n + i] = r[2 * n + i];
        p_out[i] = sg * p[(sw ? n : 0) + i];
        p_out[n + i] = sg * p[(sw ? 0 : n) + i];
        p_out[2 * n + i] = sg * p[2 * n + i];
    }
}

/* (1 - exp(-u)) / u, the time integral of exp(-u s/h) over one step divided by h */
static double pef_phi(double u) { return u == 0.0 ? 1.0 : -expm1(-u) / u; }

/* One PEF trajectory of nsteps steps of h = dt. Symmetric splitting into a flow part E, the
 * force part K and the streaming part D, each exact:
 *   E(h/2) K(h/2) D(h) [k += 1, new box, wrap, F = F(r)] K(h/2) E(h/2)
 * with
 *   E: dp_x/dt = -rate p_x, dp_y/dt = +rate p_y (- alpha_E p under the constraint): the
 *      unconstrained solution p_x e^{-rate tau}, p_y e^{rate tau} scaled back to the initial
 *      p.p;
 *   K: dp/dt = F (- alpha_K p), orc_iso_kick;
 *   D: dx/dt = p_x + rate x, dy/dt = p_y - rate y, dz/dt = p_z with p fixed:
 *      x -> e^{rate h} (x + h p_x phi(rate h)), y -> e^{-rate h} (y + h p_y phi(-rate h)),
 *      phi(u) = (1 - e^{-u})/u, so that x / L_x advances by h p_x phi(rate h) / L_x(t).
 * The isokinetic run ends each step with a rescale to K0 (round-off only); gik = 0 gives the
 * adiabatic step (E without the multiplier, K a plain kick). vn1_out[s] = V (P_xx - P_yy)
 * after step s (s = 0: the start). *e0 is the strain at the start; it is advanced. */
int32_t orc_pef_run(const orc_box* b0, double rate, double dt, int32_t gik, double k0,
                    double* e0, double* r, double* p, int64_t nsteps, double* vn1_out,
                    double* ke_out, double* pe_out) {
    const int32_t n = b0->n;
    double* f = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    if (!f) return -2;
    double* x = r;
    double* y = r + n;
    double* z = r + 2 * n;
    double* px = p;
    double* py = p + n;
    const double h = dt;
    const double e_start = *e0;
    orc_box bk;
    pef_box(b0, e_start, &bk);
    double out[3];
    if (orc_pef_forces(&bk, r, f, out) != 0) {
        free(f);
        return -1;
    }
    if (k0 <= 0.0) k0 = kinetic(n, p);
    const double ex = exp(-0.5 * rate * h), ey = exp(0.5 * rate * h);
    const double dx_scale = exp(rate * h), dy_scale = exp(-rate * h);
    const double phx = pef_phi(rate * h), phy = pef_phi(-rate * h);
    double s0 = 0.0;
    for (int32_t i = 0; i < n; ++i) s0 += px[i] * px[i] - py[i] * py[i];
    if (vn1_out) vn1_out[0] = s0 + out[1];
    if (ke_out) ke_out[0] = kinetic(n, p);
    if (pe_out) pe_out[0] = out[0];
    for (int64_t s = 1; s <= nsteps; ++s) {
        for (int half = 0; half < 2; ++half) {
            if (half == 1) {
                /* streaming, then the new box, wrap and forces */
                for (int32_t i = 0; i < n; ++i) {
                    x[i] = dx_scale * (x[i] + h * px[i] * phx);
                    y[i] = dy_scale * (y[i] + h * py[i] * phy);
                    z[i] += h * p[2 * n + i];
                }
                pef_box(b0, e_start + rate * ((double)s * h), &bk);
                for (int32_t i = 0; i < n; ++i) {
                    x[i] = wrap1(x[i], bk.lx);
                    y[i] = wrap1(y[i], bk.ly);
                    z[i] = wrap1(z[i], bk.lz);
                }
                if (orc_pef_forces(&bk, r, f, out) != 0) {
                    free(f);
                    return -1;
                }
            }
            /* E then K in the first half step, K then E in the second */
            for (int part = 0; part < 2; ++part) {
                const int do_e = (half == 0) ? (part == 0) : (part == 1);
                if (do_e) {
                    double pp0 = 0.0, pp1 = 0.0;
                    if (gik)
                        for (int32_t c = 0; c < 3 * n; ++c) pp0 += p[c] * p[c];
                    for (int32_t i = 0; i < n; ++i) {
                        px[i] *= ex;
                        py[i] *= ey;
                    }
                    if (gik) {
                        for (int32_t c = 0; c < 3 * n; ++c) pp1 += p[c] * p[c];
                        const double g = sqrt(pp0 / pp1);
                        for (int32_t c = 0; c < 3 * n; ++c) p[c] *= g;
                    }
                } else if (gik) {
                    orc_iso_kick(n, p, f, 0.5 * h);
                } else {
                    for (int32_t c = 0; c < 3 * n; ++c) p[c] += 0.5 * h * f[c];
                }
            }
        }
        if (gik) {
            const double lam = sqrt(k0 / kinetic(n, p));
            for (int32_t c = 0; c < 3 * n; ++c) p[c] *= lam;
        }
        double sk = 0.0;
        for (int32_t i = 0; i < n; ++i) sk += px[i] * px[i] - py[i] * py[i];
        if (vn1_out) vn1_out[s] = sk + out[1];
        if (ke_out) ke_out[s] = kinetic(n, p);
        if (pe_out) pe_out[s] = out[0];
    }
    *e0 = e_start + rate * ((double)nsteps * h);
    free(f);
    return 0;
}

typedef struct {
    const orc_box* b;
    double dt;
    const double *states_r, *states_p;
    int32_t n_daughters;
    const int32_t *state_of, *map_of;
    const double* rate_of;
    int64_t nsteps;
    double *vn1_out, *r_out, *p_out;
    int32_t tid, nthreads, status;
    /* Nose-Hoover daughters when states_zeta is not NULL */
    const double* states_zeta;
    double temperature, q, nf;
} pef_job;

static void* pef_worker(void* arg) {
    pef_job* jb = (pef_job*)arg;
    const size_t sz = 3 * (size_t)jb->b->n;
    double* r = (double*)malloc(sizeof(double) * sz);
    double* p = (double*)malloc(sizeof(double) * sz);
    jb->status = 0;
    for (int32_t d = jb->tid; d < jb->n_daughters; d += jb->nthreads) {
        const int32_t s = jb->state_of[d];
        orc_map_pef(jb->b, jb->map_of[d], jb->states_r + (size_t)s * sz,
                    jb->states_p + (size_t)s * sz, r, p);
        double e = 0.0;
        double* vn = jb->vn1_out + (size_t)d * (size_t)(jb->nsteps + 1);
        int32_t rc;
        if (jb->states_zeta) {
            /* the mappings that reverse the momenta (m = 1, 3) reverse the thermostat too */
            double zt = (jb->map_of[d] & 1) ? -jb->states_zeta[s] : jb->states_zeta[s];
            rc = orc_nh_pef_run(jb->b, jb->rate_of[d], jb->dt, jb->temperature, jb->q, jb->nf,
                                &e, r, p, &zt, jb->nsteps, vn, 0, 0, 0);
        } else {
            rc = orc_pef_run(jb->b, jb->rate_of[d], jb->dt, 1, 0.0, &e, r, p, jb->nsteps, vn, 0,
                             0);
        }
        if (rc) jb->status = rc;
        if (jb->r_out) memcpy(jb->r_out + (size_t)d * sz, r, sizeof(double) * sz);
        if (jb->p_out) memcpy(jb->p_out + (size_t)d * sz, p, sizeof(double) * sz);
    }
    free(r);
    free(p);
    return 0;
}

static int32_t run_pef_batch(const orc_box* b, double dt, const double* states_r,
                             const double* states_p, const double* states_zeta,
                             double temperature, double q, double nf, int32_t n_daughters,
                             const int32_t* state_of, const int32_t* map_of,
                             const double* rate_of, int64_t nsteps, int32_t nthreads,
                             double* vn1_out, double* r_out, double* p_out) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > n_daughters) nthreads = n_daughters > 0 ? n_daughters : 1;
    pef_job* jobs = (pef_job*)calloc((size_t)nthreads, sizeof(pef_job));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int32_t t = 0; t < nthreads; ++t) {
        pef_job j = {b,      dt,      states_r, states_p, n_daughters, state_of, map_of, rate_of,
                     nsteps, vn1_out, r_out,    p_out,    t,           nthreads, 0,
                     states_zeta, temperature, q, nf};
        jobs[t] = j;
        pthread_create(&th[t], 0, pef_worker, &jobs[t]);
    }
    int32_t status = 0;
    for (int32_t t = 0; t < nthreads; ++t) {
        pthread_join(th[t], 0);
        if (jobs[t].status) status = jobs[t].status;
    }
    free(jobs);
    free(th);
    return status ? status : nthreads;
}

/* Planar elongation with the Nose-Hoover multiplier of Eq. (system1) in place of the
 * Gaussian one: dp/dt = F - p . grad u - zeta p, d zeta/dt = (sum p^2 - nf T)/q. The
 * splitting of nh_sllod_run with the elongation's flow part E in place of the shear part,
 * each part exact over half steps:
 *   Z T E K D(h) [new box, wrap, F] K E T Z
 * with Z: zeta += tau (sum p^2 - nf T)/q; T: p *= exp(-zeta tau); E: p_x e^{-rate tau},
 * p_y e^{rate tau}; K: p += F tau; D the streaming of orc_pef_run. The sequence is
 * symmetric: second order and time reversible under (p, zeta, rate) -> (-p, -zeta, -rate)
 * from the final strain. zeta_out[s] holds zeta after step s. */
int32_t orc_nh_pef_run(const orc_box* b0, double rate, double dt, double temperature, double q,
                       double nf, double* e0, double* r, double* p, double* zeta, int64_t nsteps,
                       double* vn1_out, double* ke_out, double* pe_out, double* zeta_out) {
    const int32_t n = b0->n;
    double* f = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    if (!f) return -2;
    double* x = r;
    double* y = r + n;
    double* z = r + 2 * n;
    double* px = p;
    double* py = p + n;
    const double h = dt, tau = 0.5 * dt;
    const double e_start = *e0;
    orc_box bk;
    pef_box(b0, e_start, &bk);
    double out[3];
    if (orc_pef_forces(&bk, r, f, out) != 0) {
        free(f);
        return -1;
    }
    const double ex = exp(-rate * tau), ey = exp(rate * tau);
    const double dx_scale = exp(rate * h), dy_scale = exp(-rate * h);
    const double phx = pef_phi(rate * h), phy = pef_phi(-rate * h);
    double zt = *zeta;
    double s0 = 0.0;
    for (int32_t i = 0; i < n; ++i) s0 += px[i] * px[i] - py[i] * py[i];
    if (vn1_out) vn1_out[0] = s0 + out[1];
    if (ke_out) ke_out[0] = kinetic(n, p);
    if (pe_out) pe_out[0] = out[0];
    if (zeta_out) zeta_out[0] = zt;
    for (int64_t s = 1; s <= nsteps; ++s) {
        zt += tau * (2.0 * kinetic(n, p) - nf * temperature) / q;
        double sc = exp(-zt * tau);
        for (int32_t c = 0; c < 3 * n; ++c) p[c] *= sc;
        for (int32_t i = 0; i < n; ++i) {
            px[i] *= ex;
            py[i] *= ey;
        }
        for (int32_t c = 0; c < 3 * n; ++c) p[c] += tau * f[c];
        for (int32_t i = 0; i < n; ++i) {
            x[i] = dx_scale * (x[i] + h * px[i] * phx);
            y[i] = dy_scale * (y[i] + h * py[i] * phy);
            z[i] += h * p[2 * n + i];
        }
        pef_box(b0, e_start + rate * ((double)s * h), &bk);
        for (int32_t i = 0; i < n; ++i) {
            x[i] = wrap1(x[i], bk.lx);
            y[i] = wrap1(y[i], bk.ly);
            z[i] = wrap1(z[i], bk.lz);
        }
        if (orc_pef_forces(&bk, r, f, out) != 0) {
            free(f);
            return -1;
        }
        for (int32_t c = 0; c < 3 * n; ++c) p[c] += tau * f[c];
        for (int32_t i = 0; i < n; ++i) {
            px[i] *= ex;
            py[i] *= ey;
        }
        sc = exp(-zt * tau);
        for (int32_t c = 0; c < 3 * n; ++c) p[c] *= sc;
        zt += tau * (2.0 * kinetic(n, p) - nf * temperature) / q;
        double sk = 0.0;
        for (int32_t i = 0; i < n; ++i) sk += px[i] * px[i] - py[i] * py[i];
        if (vn1_out) vn1_out[s] = sk + out[1];
        if (ke_out) ke_out[s] = kinetic(n, p);
        if (pe_out) pe_out[s] = out[0];
        if (zeta_out) zeta_out[s] = zt;
    }
    *zeta = zt;
    *e0 = e_start + rate * ((double)nsteps * h);
    free(f);
    return 0;
}

int32_t orc_run_daughters_pef(const orc_box* b, double dt, const double* states_r,
                              const double* states_p, int32_t n_daughters,
                              const int32_t* state_of, const int32_t* map_of,
                              const double* rate_of, int64_t nsteps, int32_t nthreads,
                              double* vn1_out, double* r_out, double* p_out) {
    return run_pef_batch(b, dt, states_r, states_p, 0, 0.0, 0.0, 0.0, n_daughters, state_of,
                         map_of, rate_of, nsteps, nthreads, vn1_out, r_out, p_out);
}

int32_t orc_run_daughters_pef_nh(const orc_box* b, double dt, double temperature, double q,
                                 double nf, const double* states_r, const double* states_p,
                                 const double* states_zeta, int32_t n_daughters,
                                 const int32_t* state_of, const int32_t* map_of,
                                 const double* rate_of, int64_t nsteps, int32_t nthreads,
                                 double* vn1_out, double* r_out, double* p_out) {
    if (!states_zeta) return -1;
    return run_pef_batch(b, dt, states_r, states_p, states_zeta, temperature, q, nf, n_daughters,
                         state_of, map_of, rate_of, nsteps, nthreads, vn1_out, r_out, p_out);
}

/* ------------------------------------------------------------------------------------ */
/* mixed flow: shear and planar elongation together                                      */
/* ------------------------------------------------------------------------------------ */
/* The Introduction names mixed flows among those TTCF extends to. Reading used here: SLLOD
 * with u_x = erate x + srate y, u_y = -erate y, i.e. dr/dt = p + A r, dp/dt = F - A p
 * - alpha p with A = [[erate, srate, 0], [0, -erate, 0], [0, 0, 0]], Gaussian isokinetic
 * (or Nose-Hoover) alpha, in the box that the flow carries: columns of
 * H(t) = exp(A t) diag(L_x0, L_y0, L_z0), i.e.
 *   H_xx = L_x0 e^{erate t}, H_yy = L_y0 e^{-erate t}, H_xy = L_y0 srate t sinhc(erate t)
 * (sinhc x = sinh x / x), a triclinic cell of constant volume. Positions are wrapped by their
 * fractional coordinates s = H^-1 r. The dissipative flux is grad u : P = erate (P_xx - P_yy)
 * + srate P_xy; the daughters record V J with J = (grad u : P) / |rate|,
 * |rate| = sqrt(erate^2 + srate^2), so that Omega(0) = -(V/T) |rate| J(0). */

static double sinhc(double x) { return x == 0.0 ? 1.0 : sinh(x) / x; }

static void mix_box(const orc_box* b0, double er, double sr, double t, double h[3]) {
    h[0] = b0->lx * exp(er * t);
    h[1] = b0->ly * sr * t * sinhc(er * t);
    h[2] = b0->ly * exp(-er * t);
}

/* Forces in the triclinic cell (columns (h0, 0, 0), (h1, h2, 0), (0, 0, L_z)) by a plain sum
 * over pairs i < j, each through the image that rounds its fractional separation: when every
 * perpendicular width of the cell exceeds 2 r_c, that image is the only one within r_c
 * (else -1). out = {U, W_xx - W_yy, W_xy, pairs}. */
int32_t orc_mix_forces(const orc_box* b0, const double h[3], const double* r, double* f,
                       double* out) {
    const int32_t n = b0->n;
    const double wx = h[0] * h[2] / sqrt(h[1] * h[1] + h[2] * h[2]);
    if (!(wx > 2.0 * b0->rc && h[2] > 2.0 * b0->rc && b0->lz > 2.0 * b0->rc)) return -1;
    const double rc2 = b0->rc * b0->rc;
    double u = 0.0, wn = 0.0, wxy = 0.0, npair = 0.0;
    for (int32_t k = 0; k < 3 * n; ++k) f[k] = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t j = i + 1; j < n; ++j) {
            /* fractional separation: s = H^-1 (r_i - r_j) */
            double dx = r[i] - r[j];
            double dy = r[n + i] - r[n + j];
            double dz = r[2 * n + i] - r[2 * n + j];
            double sy = dy / h[2];
            double sx = (dx - h[1] * sy) / h[0];
            double sz = dz / b0->lz;
            sx -= rint(sx);
            sy -= rint(sy);
            sz -= rint(sz);
            dx = h[0] * sx + h[1] * sy;
            dy = h[2] * sy;
            dz = b0->lz * sz;
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rc2) {
                double fs, phi;
                pair_eval(b0, r2, &fs, &phi);
                f[i] += fs * dx;
                f[n + i] += fs * dy;
                f[2 * n + i] += fs * dz;
                f[j] -= fs * dx;
                f[n + j] -= fs * dy;
                f[2 * n + j] -= fs * dz;
                u += phi;
                wn += dx * (fs * dx) - dy * (fs * dy);
                wxy += dx * (fs * dy);
                npair += 1.0;
            }
        }
    }
    out[0] = u;
    out[1] = wn;
    out[2] = wxy;
    out[3] = npair;
    return 0;
}

/* Mappings for mixed flow (reading): bit 1 exchanges the x and y axes of positions and
 * momenta, then bit 0 reflects x (x -> L_x - x, p_x -> -p_x). P_xx - P_yy changes sign under
 * the exchange and P_xy under the reflection, so over m = 0..3 the flux J(0) takes
 * erate N1 (+, +, -, -) + srate P_xy (+, -, +, -) and averages to zero. */
void orc_map_mix(const orc_box* b, int32_t m, const double* r, const double* p, double* r_out,
                 double* p_out) {
    const int32_t n = b->n;
    orc_map_pef(b, m & 2, r, p, r_out, p_out);
    if (m & 1) {
        for (int32_t i = 0; i < n; ++i) {
            r_out[i] = (r_out[i] == 0.0) ? 0.0 : b->lx - r_out[i];
            p_out[i] = -p_out[i];
        }
    }
}

/* wrap r into the cell H through its fractional coordinates */
static void mix_wrap(int32_t n, const double h[3], double lz, double* r) {
    for (int32_t i = 0; i < n; ++i) {
        double sy = r[n + i] / h[2];
        double sx = (r[i] - h[1] * sy) / h[0];
        double sz = r[2 * n + i] / lz;
        sx -= floor(sx);
        sy -= floor(sy);
        sz -= floor(sz);
        if (sx >= 1.0) sx = 0.0;
        if (sy >= 1.0) sy = 0.0;
        if (sz >= 1.0) sz = 0.0;
        r[i] = h[0] * sx + h[1] * sy;
        r[n + i] = h[2] * sy;
        r[2 * n + i] = lz * sz;
    }
}

/* p -> exp(-A tau) p: p_x e^{-erate tau} - srate tau sinhc(erate tau) p_y, p_y e^{erate tau} */
static void mix_flow(int32_t n, double* p, double er, double sr, double tau) {
    const double a = exp(-er * tau), d = exp(er * tau), c = -sr * tau * sinhc(er * tau);
    for (int32_t i = 0; i < n; ++i) {
        const double px = p[i], py = p[n + i];
        p[i] = a * px + c * py;
        p[n + i] = d * py;
    }
}

/* One mixed-flow trajectory, steps of h = dt from time t0 = *t (advanced by the run).
 * Isokinetic: E(h/2) K(h/2) D(h) [new cell, wrap, F] K(h/2) E(h/2), rescale to K0, with
 *   E: p -> exp(-A tau) p scaled back to its p.p;
 *   K: orc_iso_kick;
 *   D: r -> exp(A h) (r + N p), N = int_0^h exp(-A u) du
 *      = [[h phi(erate h), -srate (h^2/2) sinhc(erate h/2)^2], [0, h phi(-erate h)]]
 *      (phi(u) = (1 - e^-u)/u), the exact streaming with p fixed.
 * gik = 0: the adiabatic step. thermo = 1 (gik ignored): Nose-Hoover, Z T E K D K E T Z.
 * vj_out[s] = V J after step s; comp_out[2 s], comp_out[2 s + 1] = V (P_xx - P_yy) and V P_xy
 * (NULL to skip). */
int32_t orc_mix_run(const orc_box* b0, double er, double sr, double dt, int32_t gik,
                    int32_t thermo, double temperature, double q, double nf, double* t,
                    double* r, double* p, double* zeta, int64_t nsteps, double* vj_out,
                    double* ke_out, double* pe_out, double* comp_out) {
    const int32_t n = b0->n;
    double* f = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    if (!f) return -2;
    const double h = dt, tau = 0.5 * dt;
    const double t0 = *t;
    const double rn = sqrt(er * er + sr * sr);
    double hb[3];
    mix_box(b0, er, sr, t0, hb);
    double out[4];
    if (orc_mix_forces(b0, hb, r, f, out) != 0) {
        free(f);
        return -1;
    }
    double k0 = kinetic(n, p);
    double zt = zeta ? *zeta : 0.0;
    /* exp(A h) and N */
    const double ea = exp(er * h), ed = exp(-er * h), eb = sr * h * sinhc(er * h);
    const double nxx = h * pef_phi(er * h), nyy = h * pef_phi(-er * h);
    const double hs = sinhc(0.5 * er * h);
    const double nxy = -sr * 0.5 * h * h * hs * hs;
#define MIX_VJ(KS)                                                                    \
    do {                                                                              \
        double s1 = 0.0, s2 = 0.0;                                                    \
        for (int32_t i = 0; i < n; ++i) {                                             \
            s1 += p[i] * p[i] - p[n + i] * p[n + i];                                  \
            s2 += p[i] * p[n + i];                                                    \
        }                                                                             \
        if (vj_out) vj_out[KS] = rn > 0.0 ? (er * (s1 + out[1]) + sr * (s2 + out[2])) / rn : 0.0; \
        if (comp_out) {                                                               \
            comp_out[2 * (KS)] = s1 + out[1];                                         \
            comp_out[2 * (KS) + 1] = s2 + out[2];                                     \
        }                                                                             \
    } while (0)
    MIX_VJ(0);
    if (ke_out) ke_out[0] = kinetic(n, p);
    if (pe_out) pe_out[0] = out[0];
    for (int64_t s = 1; s <= nsteps; ++s) {
        if (thermo) {
            zt += tau * (2.0 * kinetic(n, p) - nf * temperature) / q;
            const double sc = exp(-zt * tau);
            for (int32_t c = 0; c < 3 * n; ++c) p[c] *= sc;
        }
        {
            const double pp0 = 2.0 * kinetic(n, p);
            mix_flow(n, p, er, sr, tau);
            if (gik && !thermo) {
                const double g = sqrt(pp0 / (2.0 * kinetic(n, p)));
                for (int32_t c = 0; c < 3 * n; ++c) p[c] *= g;
            }
        }
        if (gik && !thermo)
            orc_iso_kick(n, p, f, tau);
        else
            for (int32_t c = 0; c < 3 * n; ++c) p[c] += tau * f[c];
        for (int32_t i = 0; i < n; ++i) {
            const double x = r[i] + nxx * p[i] + nxy * p[n + i];
            const double y = r[n + i] + nyy * p[n + i];
            r[i] = ea * x + eb * y;
            r[n + i] = ed * y;
            r[2 * n + i] += h * p[2 * n + i];
        }
        mix_box(b0, er, sr, t0 + (double)s * h, hb);
        mix_wrap(n, hb, b0->lz, r);
        if (orc_mix_forces(b0, hb, r, f, out) != 0) {
            free(f);
            return -1;
        }
        if (gik && !thermo)
            orc_iso_kick(n, p, f, tau);
        else
            for (int32_t c = 0; c < 3 * n; ++c) p[c] += tau * f[c];
        {
            const double pp0 = 2.0 * kinetic(n, p);
            mix_flow(n, p, er, sr, tau);
            if (gik && !thermo) {
                const double g = sqrt(pp0 / (2.0 * kinetic(n, p)));
                for (int32_t c = 0; c < 3 * n; ++c) p[c] *= g;
            }
        }
        if (thermo) {
            const double sc = exp(-zt * tau);
            for (int32_t c = 0; c < 3 * n; ++c) p[c] *= sc;
            zt += tau * (2.0 * kinetic(n, p) - nf * temperature) / q;
        } else if (gik) {
            const double lam = sqrt(k0 / kinetic(n, p));
            for (int32_t c = 0; c < 3 * n; ++c) p[c] *= lam;
        }
        MIX_VJ(s);
        if (ke_out) ke_out[s] = kinetic(n, p);
        if (pe_out) pe_out[s] = out[0];
    }
#undef MIX_VJ
    if (zeta) *zeta = zt;
    *t = t0 + (double)nsteps * h;
    free(f);
    return 0;
}

typedef struct {
    const orc_box* b;
    double dt;
    const double *states_r, *states_p, *states_zeta;
    int32_t n_daughters;
    const int32_t *state_of, *map_of;
    const double *er_of, *sr_of;
    int64_t nsteps;
    double *vj_out, *r_out, *p_out, *comp_out;
    double temperature, q, nf;
    int32_t tid, nthreads, status;
} mix_job;

static void* mix_worker(void* arg) {
    mix_job* jb = (mix_job*)arg;
    const size_t sz = 3 * (size_t)jb->b->n;
    double* r = (double*)malloc(sizeof(double) * sz);
    double* p = (double*)malloc(sizeof(double) * sz);
    jb->status = 0;
    for (int32_t d = jb->tid; d < jb->n_daughters; d += jb->nthreads) {
        const int32_t s = jb->state_of[d];
        orc_map_mix(jb->b, jb->map_of[d], jb->states_r + (size_t)s * sz,
                    jb->states_p + (size_t)s * sz, r, p);
        double t = 0.0;
        /* none of the mixed-flow mappings reverses time: zeta is carried unchanged */
        double zt = jb->states_zeta ? jb->states_zeta[s] : 0.0;
        int32_t rc = orc_mix_run(jb->b, jb->er_of[d], jb->sr_of[d], jb->dt, 1,
                                 jb->states_zeta ? 1 : 0, jb->temperature, jb->q, jb->nf, &t, r,
                                 p, &zt, jb->nsteps,
                                 jb->vj_out + (size_t)d * (size_t)(jb->nsteps + 1), 0, 0,
                                 jb->comp_out ? jb->comp_out + (size_t)d * 2 * (size_t)(jb->nsteps + 1)
                                              : 0);
        if (rc) jb->status = rc;
        if (jb->r_out) memcpy(jb->r_out + (size_t)d * sz, r, sizeof(double) * sz);
        if (jb->p_out) memcpy(jb->p_out + (size_t)d * sz, p, sizeof(double) * sz);
    }
    free(r);
    free(p);
    return 0;
}

int32_t orc_run_daughters_mix(const orc_box* b, double dt, const double* states_r,
                              const double* states_p, const double* states_zeta,
                              double temperature, double q, double nf, int32_t n_daughters,
                              const int32_t* state_of, const int32_t* map_of,
                              const double* er_of, const double* sr_of, int64_t nsteps,
                              int32_t nthreads, double* vj_out, double* r_out, double* p_out,
                              double* comp_out) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > n_daughters) nthreads = n_daughters > 0 ? n_daughters : 1;
    mix_job* jobs = (mix_job*)calloc((size_t)nthreads, sizeof(mix_job));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int32_t t = 0; t < nthreads; ++t) {
        mix_job j = {b,     dt,       states_r, states_p,    states_zeta, n_daughters,
                     state_of, map_of, er_of,   sr_of,       nsteps,      vj_out,
                     r_out, p_out,    comp_out, temperature, q,       nf,
                     t,     nthreads, 0};
        jobs[t] = j;
        pthread_create(&th[t], 0, mix_worker, &jobs[t]);
    }
    int32_t status = 0;
    for (int32_t t = 0; t < nthreads; ++t) {
        pthread_join(th[t], 0);
        if (jobs[t].status) status = jobs[t].status;
    }
    free(jobs);
    free(th);
    return status ? status : nthreads;
}
