/*
 * ttcf_oracle.h -- plain FP64 CPU oracle for the TTCF daughter path of
 * arxiv 2312.02990 (TTCF4LAMMPS).
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg load this library. The GPU library shares no code with it and
 * never calls it.
 *
 * Conventions (LJ reduced units, m = sigma = epsilon = k_B = 1):
 *   - state arrays are structure-of-arrays: r = [x(0..n-1) | y(..) | z(..)], same for p, f;
 *   - p is the peculiar momentum (thermal part only; the streaming velocity gamma_dot*y
 *     is carried by the SLLOD position equation);
 *   - P_xy is the pressure-tensor component, V*P_xy = sum_i px_i py_i + sum_{i<j} x_ij F_y,ij.
 *
 * Parity status of each entry point is listed in the test-suite; every function here is
 * pinned by at least one independent check (brute force, closed form or invariant).
 */
#ifndef TTCF_ORACLE_H
#define TTCF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n;        /* atoms                                                   */
    int32_t pad_;
    double  lx, ly, lz;  /* box edges                                            */
    double  rc;       /* cutoff radius; pairs interact when r^2 < rc*rc           */
    double  c_attr;   /* attraction factor c: phi = 4[(1/r)^12 - c (1/r)^6] + shift */
    double  u_shift;  /* energy shift making phi(rc) = 0 (WCA: +1)               */
} orc_box;

/* Cell grid: n_a = floor(L_a / rc); returns 0 or -1 if any n_a < 3 or n_x < 4. */
int32_t orc_cell_dims(const orc_box* b, int32_t dims[3]);
/* Grid of cells at least `side` wide: n_a = floor(L_a / side); same conditions. */
int32_t orc_grid_dims(const orc_box* b, double side, int32_t dims[3]);

/* Canonical cell list of positions r (SoA, every coordinate in [0, L)):
 * cell_of[i] = cx + nx*(cy + ny*cz) with c_a = floor(r_a * (n_a / L_a)) clamped to [0, n_a-1];
 * order[] lists atom ids sorted by (cell id, atom id); start[c]..start[c+1] is cell c's range. */
int32_t orc_cell_list(const orc_box* b, const double* r, int32_t* cell_of, int32_t* order,
                      int32_t* start);
/* The same on a given grid d (c_a = floor(r_a * (d_a / L_a)), clamped). */
int32_t orc_cell_list_grid(const orc_box* b, const int32_t d[3], const double* r,
                           int32_t* cell_of, int32_t* order, int32_t* start);

/* Pair forces through the cell list, Lees-Edwards offset dxle.
 * f: SoA forces; out[0] = U (potential energy), out[1] = W_xy = sum_{i<j} x_ij F_y,ij,
 * out[2] = number of interacting pairs. */
int32_t orc_forces(const orc_box* b, double dxle, const double* r, double* f, double* out);

/* Same quantities by an O(N^2) sum over explicit periodic / sliding-brick images. */
int32_t orc_forces_brute(const orc_box* b, double dxle, const double* r, double* f, double* out);

/* Pairs i<j with squared minimum-image separation < rlist^2 (FP64, dx*dx + dy*dy + dz*dz
 * without contraction), returned sorted by (i, j). Up to rlist = rc they are found through the
 * canonical cell list; a Verlet list of radius rlist > rc (rc plus a skin) through the grid
 * of cells at least rlist wide. Returns the count, -1 if the capacity is too small, -2 if the
 * box is too small for that grid. */
int64_t orc_pairs(const orc_box* b, double dxle, const double* r, double rlist, int64_t cap,
                  int32_t* pi, int32_t* pj);
/* Same set by testing every pair i<j. */
int64_t orc_pairs_brute(const orc_box* b, double dxle, const double* r, double rlist,
                        int64_t cap, int32_t* pi, int32_t* pj);

/* V*P_xy of a state at LE offset dxle. */
double orc_vpxy(const orc_box* b, double dxle, const double* r, const double* p);

/* The four phase-space mappings of a start state (m = 0 identity, 1 p->-p,
 * 2 x-reflection (x,px)->(-x,-px), 3 (x,py,pz)->(-x,-py,-pz)); reflected x is wrapped
 * back into [0, Lx). */
void orc_map(const orc_box* b, int32_t m, const double* r, const double* p, double* r_out,
             double* p_out);

/* Nose-Hoover equilibrium run (gamma_dot = 0, plain periodic box), symmetric splitting.
 * q = thermostat mass, nf = degrees of freedom. Per-step outputs may be NULL:
 * vpxy_out[k], ke_out[k], pe_out[k] for k = 0..nsteps. */
int32_t orc_nh_run(const orc_box* b, double temperature, double q, double nf, double dt,
                   double* r, double* p, double* zeta, int64_t nsteps, double* vpxy_out,
                   double* ke_out, double* pe_out);

/* Exact isokinetic sub-flows (sum p.p preserved): force kick over tau with F fixed, and
 * the shear flow dpx/dt = -gamma_dot py, both with the Gaussian multiplier. */
void orc_iso_kick(int32_t n, double* p, const double* f, double tau);
void orc_iso_shear(int32_t n, double* p, double gamma_dot, double tau);

/* SLLOD run under Lees-Edwards boundaries, step counter k (LE offset
 * dx = fmod(gamma_dot * ly * (k*dt), lx)); gik != 0 integrates the Gaussian isokinetic
 * equations (kinetic energy held at k0; k0 <= 0: the kinetic energy of the initial p).
 * Per-step outputs (k = 0..nsteps) may be NULL: vpxy_out, ke_out, pe_out. */
int32_t orc_sllod_run(const orc_box* b, double gamma_dot, double dt, int32_t gik, double k0,
                      double* r, double* p, int64_t* k, int64_t nsteps, double* vpxy_out,
                      double* ke_out, double* pe_out);

/* Mother sampling: starting from (r, p, zeta) run n_equil NH steps, then n_states times
 * {run steps_between NH steps; copy (r, p) into states_r/p[s]}. The thermostat state is
 * carried through. states_r, states_p: n_states * 3n each. */
int32_t orc_mother_sample(const orc_box* b, double temperature, double q, double nf, double dt,
                          double* r, double* p, double* zeta, int64_t n_equil,
                          int32_t n_states, int64_t steps_between, double* states_r,
                          double* states_p);

/* SLLOD of Eq. (system1) as printed, with the Nose-Hoover multiplier: d zeta/dt =
 * (sum p^2 - nf T)/q. Symmetric splitting, each part exact:
 *   Z(h/2) T(h/2) S(h/2) K(h/2) D(h) [k += 1, LE offset, wrap, F = F(r)] K(h/2) S(h/2) T(h/2) Z(h/2)
 * Z: zeta += (h/2)(sum p^2 - nf T)/q; T: p *= exp(-zeta h/2); S: px -= (h/2) gamma_dot py;
 * K: p += (h/2) F; D: the streaming part of orc_sllod_run. Per-step outputs (k = 0..nsteps)
 * may be NULL: vpxy_out, ke_out, pe_out, zeta_out. */
int32_t orc_nh_sllod_run(const orc_box* b, double gamma_dot, double dt, double temperature,
                         double q, double nf, double* r, double* p, double* zeta, int64_t* k,
                         int64_t nsteps, double* vpxy_out, double* ke_out, double* pe_out,
                         double* zeta_out);

/* orc_mother_sample that also saves the thermostat variable of every state (states_zeta,
 * n_states doubles). */
int32_t orc_mother_sample_zeta(const orc_box* b, double temperature, double q, double nf,
                               double dt, double* r, double* p, double* zeta, int64_t n_equil,
                               int32_t n_states, int64_t steps_between, double* states_r,
                               double* states_p, double* states_zeta);

/* Batch of Nose-Hoover SLLOD daughters (orc_nh_sllod_run): as orc_run_daughters, each start
 * state with its thermostat variable states_zeta[s], reversed by the mappings that reverse
 * time (m = 1 and 3). */
int32_t orc_run_daughters_nh(const orc_box* b, double dt, double temperature, double q,
                             double nf, const double* states_r, const double* states_p,
                             const double* states_zeta, int32_t n_daughters,
                             const int32_t* state_of, const int32_t* map_of,
                             const double* gamma_of, int64_t nsteps, int32_t nthreads,
                             double* vpxy_out, double* r_out, double* p_out);

/* Observables of a state beyond P_xy (m = 1; V = Lx Ly Lz; pair sums over r^2 < rc^2):
 *   out[0] = P_xx - P_yy, out[1] = P_yy - P_zz, with
 *            V P_aa = sum_i p_a,i^2 + sum_{i<j} r_ij,a F_ij,a (r_ij the minimum image);
 *   out[2] = (K + U) / N, K = sum_i p_i^2 / 2 (peculiar), U = sum_{i<j} phi(r_ij);
 *   out[3 + s], s = 0..n_slabs-1: sum of p_x over the atoms with
 *            floor(y n_slabs / Ly) = s (clamped), divided by the slab volume V / n_slabs.
 * dxle is the Lees-Edwards offset of the positions. Returns 0, or -1 (n_slabs < 1 or a
 * box too small for the cell grid). */
int32_t orc_observables(const orc_box* b, double dxle, const double* r, const double* p,
                        int32_t n_slabs, double* out);

/* Batch of daughters as orc_run_daughters (states_zeta == NULL: GIK) or orc_run_daughters_nh
 * (Nose-Hoover), that also records orc_observables after every step:
 * obs_out[(d (nsteps + 1) + k) (3 + n_slabs) + c]. */
int32_t orc_run_daughters_obs(const orc_box* b, double dt, double temperature, double q,
                              double nf, const double* states_r, const double* states_p,
                              const double* states_zeta, int32_t n_daughters,
                              const int32_t* state_of, const int32_t* map_of,
                              const double* gamma_of, int64_t nsteps, int32_t nthreads,
                              double* vpxy_out, int32_t n_slabs, double* obs_out);

/* Colour field (the colour-conductivity field of Evans and Morriss): atom i carries the
 * colour charge c_i = +1 for even i and -1 for odd i, and the field F_e adds c_i F_e along x:
 *   dr/dt = p,  dp/dt = F + c F_e x_hat - alpha p   (no streaming term, no box shear).
 * The adiabatic energy changes at dH/dt = F_e sum_i c_i p_x,i = F_e V J_x, so the dissipation
 * function is Omega = (V/T) F_e J_x and the response is the colour current J_x.
 * gik = 1: alpha = p.(F + c F_e x_hat)/p.p (kinetic energy held at k0, k0 <= 0: that of the
 * initial p), each half kick the exact isokinetic flow under the fixed total force, then a
 * rescale to k0 (round-off only); gik = 0: alpha = 0. Steps K(h/2) D(h) [F(r)] K(h/2).
 * Per-step outputs (k = 0..nsteps, may be NULL): jx_out = V J_x = sum_i c_i p_x,i, ke_out,
 * pe_out. */
int32_t orc_colour_run(const orc_box* b, double fe, double dt, int32_t gik, double k0, double* r,
                       double* p, int64_t nsteps, double* jx_out, double* ke_out,
                       double* pe_out);

/* The colour field with the Nose-Hoover multiplier of Eq. (system1): dp/dt = F + c F_e x_hat
 * - zeta p, d zeta/dt = (sum p^2 - nf T)/q; steps Z T K D K T Z over half steps (the
 * splitting of orc_nh_sllod_run without its shear part). Outputs as orc_nh_sllod_run, with
 * jx_out = V J_x in place of V P_xy. */
int32_t orc_nh_colour_run(const orc_box* b, double fe, double dt, double temperature, double q,
                          double nf, double* r, double* p, double* zeta, int64_t nsteps,
                          double* jx_out, double* ke_out, double* pe_out, double* zeta_out);

/* Batch of colour-field daughters, as orc_run_daughters with the field strength fe_of[d] in
 * place of the shear rate and V J_x in place of V P_xy: isokinetic (orc_colour_run) when
 * states_zeta is NULL, else Nose-Hoover (orc_nh_colour_run) from each state's zeta, reversed
 * by the mappings that reverse the momenta (m = 1, 3). */
int32_t orc_run_daughters_colour(const orc_box* b, double dt, const double* states_r,
                                 const double* states_p, const double* states_zeta,
                                 double temperature, double q, double nf, int32_t n_daughters,
                                 const int32_t* state_of, const int32_t* map_of,
                                 const double* fe_of, int64_t nsteps, int32_t nthreads,
                                 double* jx_out, double* r_out, double* p_out);

/* Planar elongational flow (Introduction: TTCF extends to elongational flows): SLLOD with
 * grad u = diag(rate, -rate, 0) in a box deforming as L_x0 e^e, L_y0 e^-e, L_z0,
 * e = e0 + rate t, Gaussian isokinetic or adiabatic (gik = 0).
 * orc_pef_forces: all-pairs forces with the orthorhombic minimum image (every edge must
 * exceed 2 r_c, else -1); out = {U, W_xx - W_yy, pairs}.
 * orc_map_pef: mapping m (bit 0 reverses p, bit 1 exchanges the x and y axes).
 * orc_pef_run: one trajectory in place; *e0 is the start strain (advanced by the run);
 * vn1_out = V (P_xx - P_yy), ke_out, pe_out: nsteps + 1 values each (NULL to skip).
 * orc_run_daughters_pef: as orc_run_daughters with rate_of[d] and V (P_xx - P_yy) series. */
int32_t orc_pef_forces(const orc_box* b, const double* r, double* f, double* out);
void orc_map_pef(const orc_box* b, int32_t m, const double* r, const double* p, double* r_out,
                 double* p_out);
int32_t orc_pef_run(const orc_box* b0, double rate, double dt, int32_t gik, double k0,
                    double* e0, double* r, double* p, int64_t nsteps, double* vn1_out,
                    double* ke_out, double* pe_out);
/* Nose-Hoover planar elongation (splitting Z T E K D K E T Z over half steps); outputs as
 * orc_pef_run plus zeta_out (nsteps + 1 values, NULL to skip); *zeta is advanced.
 * orc_run_daughters_pef_nh: as orc_run_daughters_pef from each state's zeta, reversed by the
 * mappings that reverse the momenta (m = 1, 3). */
int32_t orc_nh_pef_run(const orc_box* b0, double rate, double dt, double temperature, double q,
                       double nf, double* e0, double* r, double* p, double* zeta, int64_t nsteps,
                       double* vn1_out, double* ke_out, double* pe_out, double* zeta_out);
int32_t orc_run_daughters_pef_nh(const orc_box* b, double dt, double temperature, double q,
                                 double nf, const double* states_r, const double* states_p,
                                 const double* states_zeta, int32_t n_daughters,
                                 const int32_t* state_of, const int32_t* map_of,
                                 const double* rate_of, int64_t nsteps, int32_t nthreads,
                                 double* vn1_out, double* r_out, double* p_out);
int32_t orc_run_daughters_pef(const orc_box* b, double dt, const double* states_r,
                              const double* states_p, int32_t n_daughters,
                              const int32_t* state_of, const int32_t* map_of,
                              const double* rate_of, int64_t nsteps, int32_t nthreads,
                              double* vn1_out, double* r_out, double* p_out);

/* Mixed flow (Introduction: TTCF extends to mixed flows): SLLOD with u_x = erate x + srate y,
 * u_y = -erate y in the triclinic cell carried by the flow, H(t) = exp(A t) diag(L0):
 * H_xx = L_x0 e^{erate t}, H_xy = L_y0 srate t sinhc(erate t), H_yy = L_y0 e^{-erate t}.
 * orc_mix_forces: h = {H_xx, H_xy, H_yy}; every pair through the image that rounds its
 * fractional separation (the only one within r_c while every perpendicular width exceeds
 * 2 r_c, else -1); out = {U, W_xx - W_yy, W_xy, pairs}.
 * orc_map_mix: bit 1 exchanges the x and y axes, then bit 0 reflects x.
 * orc_mix_run: one trajectory from time *t (advanced); gik = 0 adiabatic; thermo = 1
 * Nose-Hoover from *zeta (advanced); vj_out = V J, J = (erate (P_xx - P_yy) + srate P_xy) /
 * sqrt(erate^2 + srate^2); ke_out, pe_out: nsteps + 1 values each; comp_out: 2 (nsteps + 1)
 * values, V (P_xx - P_yy) and V P_xy per step (each NULL to skip).
 * orc_run_daughters_mix: isokinetic daughters, or Nose-Hoover when states_zeta is given
 * (no mapping reverses time, so zeta is carried unchanged). */
int32_t orc_mix_forces(const orc_box* b0, const double h[3], const double* r, double* f,
                       double* out);
void orc_map_mix(const orc_box* b, int32_t m, const double* r, const double* p, double* r_out,
                 double* p_out);
int32_t orc_mix_run(const orc_box* b0, double er, double sr, double dt, int32_t gik,
                    int32_t thermo, double temperature, double q, double nf, double* t,
                    double* r, double* p, double* zeta, int64_t nsteps, double* vj_out,
                    double* ke_out, double* pe_out, double* comp_out);
int32_t orc_run_daughters_mix(const orc_box* b, double dt, const double* states_r,
                              const double* states_p, const double* states_zeta,
                              double temperature, double q, double nf, int32_t n_daughters,
                              const int32_t* state_of, const int32_t* map_of,
                              const double* er_of, const double* sr_of, int64_t nsteps,
                              int32_t nthreads, double* vj_out, double* r_out, double* p_out,
                              double* comp_out);

/* Batch of independent GIK-SLLOD daughters on a pool of nthreads threads.
 * Daughter d starts from start state state_of[d] under mapping map_of[d] with shear rate
 * gamma_of[d] and runs nsteps steps; its series V*P_xy(t_k), k = 0..nsteps, goes to
 * vpxy_out[d*(nsteps+1) + k]. Final states (may be NULL) go to r_out/p_out[d*3n].
 * Returns the number of threads used, or a negative error. */
int32_t orc_run_daughters(const orc_box* b, double dt, const double* states_r,
                          const double* states_p, int32_t n_daughters, const int32_t* state_of,
                          const int32_t* map_of, const double* gamma_of, int64_t nsteps,
                          int32_t nthreads, double* vpxy_out, double* r_out, double* p_out);

#ifdef __cplusplus
}
#endif
#endif
