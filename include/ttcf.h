/*
 * ttcf.h -- C ABI of the MI355X (gfx950) TTCF daughter library.
 *
 * The library integrates many SLLOD "daughter" trajectories branched from an equilibrium
 * "mother" trajectory and turns them into a transient-time correlation function (TTCF)
 * response, following arxiv 2312.02990 (TTCF4LAMMPS):
 *   - Eq. (TTCF):      <B(t)> = <B(0)> + int_0^t <Omega(0) B(s)> ds
 *   - Eq. (integrand): <Omega(0) B(s)> = (1/N) sum_i Omega(0)_i B(s)_i over N daughters
 *   - Eq. (mappings):  every start state Gamma spawns Gamma, Gamma', Gamma'', Gamma'''
 *   - Eq. (system1):   SLLOD equations of motion (Lees-Edwards sliding-brick boundaries)
 *   - Eq. (TTCF1):     Omega = -(V/T) gamma_dot P_xy for the bulk shear field, with P_xy the
 *                      pressure-tensor component (the paper writes +gamma_dot V P_xy / k_B T with
 *                      P_xy read as the shear stress)
 *   - Alg. LAMMPS SCRIPT: initialise, run the mother, save a state every N_s steps, map it,
 *                      switch the field on, run N_d daughter steps, record the response.
 * The five calls ttcf_init_mother, ttcf_spawn_daughters, ttcf_step, ttcf_accumulate and
 * ttcf_response follow that algorithm; the remaining calls are inspection hooks.
 *
 * Conventions
 *   - LJ reduced units (m = sigma = epsilon = k_B = 1).
 *   - Every call returns an int32 status (TTCF_OK = 0, negative on error); out-parameters
 *     are written only on success; ttcf_last_error(ctx) gives a message. No exception and no
 *     C++ type crosses this interface.
 *   - Host arrays are caller-owned and are read or written during the call only.
 *     Position and momentum arrays are structure-of-arrays FP64: [x_0..x_{n-1}, y_0.., z_0..].
 *     Momenta are peculiar momenta (the streaming part gamma_dot*y is not included).
 *   - The context owns all device memory; allocations go through hipMalloc unless
 *     ttcf_set_allocator installed other functions (before the first context was created).
 *   - A context is single-threaded and stream-ordered: work is enqueued on the stream given
 *     at creation; calls that return host data synchronise that stream.
 *   - There is no CPU fallback: every call that computes runs HIP kernels and fails with
 *     TTCF_EDEVICE when no gfx950 device is usable.
 */
#ifndef TTCF_H
#define TTCF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ttcf_ctx ttcf_ctx; /* opaque, owned by the library */

enum {
    TTCF_OK = 0,
    TTCF_EINVAL = -1,    /* bad argument (sizes, box too small for the cell grid, ...)    */
    TTCF_ENOMEM = -2,    /* device or host allocation failed                              */
    TTCF_EDEVICE = -3,   /* a HIP call failed, or no usable gfx950 device                 */
    TTCF_ESTATE = -4,    /* call out of order (e.g. a response before any accumulation)   */
    TTCF_EUNSTABLE = -5, /* every daughter group failed its health check                  */
    TTCF_ESCRATCH = -6   /* ttcf_pair_forces_static: the input needs more than its static
                            device scratch of TTCF_STATIC_SCRATCH_BYTES                      */
};

enum { TTCF_WCA = 0, TTCF_LJ = 1 };

/* Arithmetic of the pair forces. Positions, momenta, the thermostat multiplier, P_xy and
 * every accumulated sum are FP64 in both forms. */
enum { TTCF_PREC_FP64 = 0, TTCF_PREC_FP32_FORCES = 1 };

/* Observables: P_xy (bulk); for the channel, the wall shear stress and the momentum
 * profile (n_bins values per time point); for the bulk, when recorded
 * (ttcf_record_observables), the normal-stress differences P_xx - P_yy and P_yy - P_zz, the
 * energy per atom (K + U)/N with K the peculiar kinetic energy, and the momentum profile over
 * TTCF_BULK_SLABS slabs of y (per slab: sum of p_x over its atoms / slab volume; slab s holds
 * floor(y TTCF_BULK_SLABS / L_y) = s; TTCF_BULK_SLABS values per time point). */
enum {
    TTCF_OBS_PXY = 0,
    TTCF_OBS_WALL_STRESS = 1,
    TTCF_OBS_VPROFILE = 2,
    TTCF_OBS_N1 = 3,
    TTCF_OBS_N2 = 4,
    TTCF_OBS_ENERGY = 5,
    TTCF_OBS_SLAB_PX = 6,
    TTCF_OBS_JX = 7,     /* colour-field daughters (ttcf_spawn_colour): the colour current J_x */
    TTCF_OBS_PEF_N1 = 8, /* planar-elongation daughters (ttcf_spawn_elongational): P_xx - P_yy */
    TTCF_OBS_MIX_J = 9,  /* mixed-flow daughters (ttcf_spawn_mixed): the flux J */
    TTCF_OBS_MIX_N1 = 10,  /* mixed-flow daughters: P_xx - P_yy */
    TTCF_OBS_MIX_PXY = 11  /* mixed-flow daughters: P_xy */
};
enum { TTCF_BULK_SLABS = 8 };

/* One simulated system (Example 1 of the paper: WCA fluid in a cubic periodic box). */
typedef struct {
    int32_t n_atoms;
    int32_t potential;     /* TTCF_WCA or TTCF_LJ (phi = 4[(1/r)^12 - c_attr (1/r)^6] + shift)  */
    double  box[3];        /* box edges Lx, Ly, Lz                                              */
    double  temperature;   /* target T: mother thermostat and the Omega normalisation           */
    double  dt;            /* time step                                                         */
    double  r_cut;         /* cutoff; pairs interact when r^2 < r_cut^2 (WCA: 2^(1/6))          */
    double  c_attr;        /* attraction factor c (WCA: 1)                                      */
    double  u_shift;       /* energy shift (NaN: the library's, making phi(r_cut) = 0; WCA: 1)  */
    double  nh_tau;        /* mother Nose-Hoover time constant: Q = (3N-3) T nh_tau^2           */
    int32_t precision;     /* TTCF_PREC_*                                                       */
    int32_t block_threads; /* threads per workgroup for this system (0: chosen by the library)  */
    int32_t daughter_thermostat; /* TTCF_DAUGHTER_GIK or TTCF_DAUGHTER_NH                       */
} ttcf_system;

/* Thermostat of the daughters. GIK: the Gaussian isokinetic multiplier (kinetic energy held
 * at its start value). NH: Eq. (system1) as printed, the Nose-Hoover variable of the mother
 * (same Q = (3N-3) T nh_tau^2 and target (3N-3) T) carried from the start state and reversed
 * by the mappings that reverse the momenta (1 and 3). */
enum { TTCF_DAUGHTER_GIK = 0, TTCF_DAUGHTER_NH = 1 };

/* Optional allocator (e.g. a framework's caching allocator). Process-wide; must be set
 * before the first context exists. NULL restores hipMalloc/hipFree. */
typedef void* (*ttcf_alloc_fn)(uint64_t bytes, void* stream, void* user);
typedef void (*ttcf_free_fn)(void* ptr, void* user);
int32_t ttcf_set_allocator(ttcf_alloc_fn alloc, ttcf_free_fn release, void* user);

/* ---- the five calls ----------------------------------------------------------------- */

/* Alg. LAMMPS SCRIPT, "initialize system (null ext. field)" and "run N_t timestep".
 * Creates a context when *ctx == NULL (stream: a hipStream_t, or NULL for the default
 * stream), otherwise adds another mother to *ctx (systems of different size may share one
 * context; their daughters then run in one batch). r0, p0: host, 3*n_atoms doubles each,
 * every coordinate inside [0, L). Runs n_melt Nose-Hoover steps at t_melt (0 steps to skip)
 * and then n_equil steps at sys->temperature, on the GPU. *out_mother receives the mother id. */
int32_t ttcf_init_mother(ttcf_ctx** ctx, const ttcf_system* sys, const double* r0,
                         const double* p0, int64_t n_melt, double t_melt, int64_t n_equil,
                         void* stream, int32_t* out_mother);

/* Alg. LAMMPS SCRIPT, the outer loop: for each of n_states start states "run N_s timestep,
 * save system state", then for each mapping "load, apply mapping, switch on ext. field".
 * steps_between > 0: the mother advances steps_between steps before each saved state (the
 *   new states replace the mother's stored set);
 * steps_between == 0: the mother's stored states are reused (n_states must equal their
 *   count), so several shear rates can share one set of start states.
 * mapping_mask: bit m selects mapping m of Eq. (mappings) (0xF: all four).
 * gamma_dot: n_gamma == 1 (one rate for all) or n_gamma == n_states (one per state, shared by
 *   its mapped daughters).
 * n_steps: daughter length N_d >= 1 (B(0) is recorded by the first step call, so a daughter
 * of no steps would have nothing to accumulate). Daughters are numbered state-major from
 * *out_first.
 * Omega(0) and B(0) are taken on the mapped start state. */
int32_t ttcf_spawn_daughters(ttcf_ctx* ctx, int32_t mother, int32_t n_states,
                             int64_t steps_between, uint32_t mapping_mask,
                             const double* gamma_dot, int32_t n_gamma, int32_t n_steps,
                             int64_t* out_first);

/* Section Mathematical Framework: the method holds for other external fields with their
 * own dissipation function. The colour field (the colour-conductivity field of Evans and
 * Morriss; the paper names no second field): atom i carries the colour charge +1 (even i)
 * or -1 (odd i), and the field adds charge * F_e along x; no streaming term, no box shear.
 * Daughters follow the mother system's daughter thermostat: isokinetic, dp/dt = F + c F_e x_hat
 * - alpha p with alpha keeping p.p fixed, or Nose-Hoover (alpha = zeta of Eq. system1, carried
 * from the start state and reversed by mappings 1 and 3);
 * B(t) = J_x = (1/V) sum_i c_i p_x,i, Omega(0) = (V/T) F_e J_x(0) (from dH/dt = F_e V J_x).
 * The four mappings of Eq. (mappings) apply unchanged: J_x(0) takes the signs (+, -, -, +).
 * Arguments as ttcf_spawn_daughters, with the field strengths F_e in place of the shear
 * rates. The recorded series (ttcf_export_series) holds V J_x(t_k); ttcf_accumulate folds
 * these groups and ttcf_response(ctx, TTCF_OBS_JX, F_e, ...) returns <J_x(t)> (per unit
 * field, the colour conductivity, when the filter is <= 0). Neighbour-list form with the lists
 * in LDS only: TTCF_EINVAL for FP64 forces, an odd atom count, or with the extra observables
 * switched on; stepping them in the cell form or with global lists also fails (TTCF_EINVAL). */
int32_t ttcf_spawn_colour(ttcf_ctx* ctx, int32_t mother, int32_t n_states,
                          int64_t steps_between, uint32_t mapping_mask, const double* field,
                          int32_t n_field, int32_t n_steps, int64_t* out_first);

/* Introduction: TTCF extends to elongational flows; Section Mathematical Framework: a field
 * other than shear needs its own mappings. Planar elongational flow (the paper prints no
 * equations for it): SLLOD of Eq. (system1) with grad u = diag(rate, -rate, 0), with the
 * mother system's daughter thermostat (isokinetic: alpha keeps p.p fixed; Nose-Hoover:
 * alpha = zeta of Eq. system1, carried from the start state and reversed by mappings 1 and
 * 3), in an orthorhombic box deforming as L_x e^e, L_y e^-e, L_z with
 * e = rate t (volume conserved); no reproducible lattice, as daughters are short.
 * B(t) = P_xx - P_yy, Omega(0) = -(V/T) rate (P_xx - P_yy)(0) (from dH/dt = -V grad u : P).
 * Mappings (bit m of mapping_mask): 0 identity, 1 reversed momenta, 2 x and y axes exchanged
 * (positions and momenta), 3 both; P_xx - P_yy takes the signs (+, +, -, -), so <Omega(0)>
 * vanishes over the four. Arguments as ttcf_spawn_daughters, with the elongation rates in
 * place of the shear rates. The recorded series holds V (P_xx - P_yy)(t_k); the final
 * states (ttcf_export_daughter) are in the coordinates of the deformed box. ttcf_accumulate
 * folds these groups and ttcf_response(ctx, TTCF_OBS_PEF_N1, rate, ...) returns
 * <P_xx - P_yy>(t) (-4 times the elongational viscosity times the rate in the linear regime).
 * Forces are FP64 whatever the system's precision. TTCF_EINVAL for N > 2048, L_x != L_y,
 * the extra observables switched on, or a rate and length that would shrink a box edge below
 * 3 r_c before the daughter ends. */
int32_t ttcf_spawn_elongational(ttcf_ctx* ctx, int32_t mother, int32_t n_states,
                                int64_t steps_between, uint32_t mapping_mask, const double* rate,
                                int32_t n_rate, int32_t n_steps, int64_t* out_first);

/* Introduction: TTCF extends to mixed flows. Mixed flow (the paper prints no equations for
 * it): SLLOD of Eq. (system1) with u_x = erate x + srate y, u_y = -erate y, i.e.
 * dr/dt = p + A r, dp/dt = F - A p - alpha p with A = [[erate, srate, 0], [0, -erate, 0],
 * [0, 0, 0]], with the mother system's daughter thermostat, in the triclinic cell the flow
 * carries, H(t) = exp(A t) diag(L): H_xx = L e^{erate t}, H_xy = L srate t sinh(erate t) /
 * (erate t), H_yy = L e^{-erate t} (volume conserved; no cell flips, as daughters are short).
 * B(t) = J = (erate (P_xx - P_yy) + srate P_xy) / |rate|, |rate| = sqrt(erate^2 + srate^2),
 * the flux conjugate to the flow (grad u : P / |rate|); Omega(0) = -(V/T) |rate| J(0).
 * Mappings (bit m of mapping_mask): bit 1 exchanges the x and y axes (positions and
 * momenta), then bit 0 reflects x (x -> L - x, p_x -> -p_x); P_xx - P_yy takes the signs
 * (+, +, -, -) and P_xy (+, -, +, -), so <Omega(0)> vanishes over the four. None reverses
 * time, so Nose-Hoover daughters carry zeta unchanged.
 * erate, srate: n_rate == 1 or n_states values each (one pair per start state). The series
 * holds V J(t_k); ttcf_response(ctx, TTCF_OBS_MIX_J, |rate|, ...) returns <J>(t) (for a
 * Newtonian fluid -eta (4 erate^2 + srate^2) / |rate|), and TTCF_OBS_MIX_N1 and
 * TTCF_OBS_MIX_PXY the TTCF of each component under the same Omega (-4 eta erate and
 * -eta srate in the linear regime); ttcf_export_observables exports them as columns 0 and 1
 * of the extra-observable layout (the other columns hold zeros). Final states are in the coordinates
 * of the carried cell. Forces are FP64. TTCF_EINVAL for N > 2048, L_x != L_y, both rates
 * zero, the extra observables switched on, or rates and a length that would narrow a
 * perpendicular width of the cell below 3 r_c before the daughter ends. */
int32_t ttcf_spawn_mixed(ttcf_ctx* ctx, int32_t mother, int32_t n_states, int64_t steps_between,
                         uint32_t mapping_mask, const double* erate, const double* srate,
                         int32_t n_rate, int32_t n_steps, int64_t* out_first);

/* Alg. LAMMPS SCRIPT, "run N_d timestep": advances every live daughter by up to n_steps
 * steps (never past its own N_d) in one persistent kernel launch per kernel form, recording
 * B(t_k) = P_xy (J_x for colour-field daughters, P_xx - P_yy for planar-elongation ones) after
 * every step. Asynchronous on the context's stream.
 * TTCF_EINVAL when a daughter needs a kernel form its system cannot run (see
 * ttcf_record_observables, ttcf_spawn_colour and ttcf_set_step_shape). */
int32_t ttcf_step(ttcf_ctx* ctx, int32_t n_steps);

/* Eq. (integrand) and Alg. SHELL SCRIPT "perform partial average and TTCF integration":
 * folds every finished daughter into per-start-state sums (the trapezoid-rule integral of
 * P_xy(0) B(s) and the direct average of B, compensated FP64) and frees its slot. A group
 * whose daughters failed the health check (non-finite or drifting values) is kept out of
 * every average as a whole, since dropping single mappings would break <Omega(0)> = 0.
 * *out_groups (may be NULL) receives the number of healthy groups added. */
int32_t ttcf_accumulate(ttcf_ctx* ctx, int64_t* out_groups);

/* Eq. (TTCF) and Alg. SHELL SCRIPT "gather total averages, total TTCF integration,
 * statistics". For k = 0..n_t-1 writes (any pointer may be NULL; n_t doubles each):
 *   ttcf_mean[k] = <B(0)> + int_0^{t_k} <Omega(0) B(s)> ds   (trapezoid rule)
 *   dav_mean[k]  = <B(t_k)>                                  (direct average)
 *   *_se[k]      = block standard error over start states (std, ddof=1, / sqrt(count)).
 * gamma_dot_filter > 0: only groups whose shear rate equals it exactly;
 * gamma_dot_filter <= 0: every group, each divided by its own shear rate (the response per
 *   unit shear rate; -ttcf_mean is then the transient viscosity of Eq. (visc)).
 * Synchronises the stream. TTCF_ESTATE if no group matches or n_t exceeds the recorded
 * length of a matching group. */
int32_t ttcf_response(ttcf_ctx* ctx, int32_t observable, double gamma_dot_filter, int32_t n_t,
                      double* ttcf_mean, double* ttcf_se, double* dav_mean, double* dav_se,
                      int64_t* out_n_states);
/* observable: TTCF_OBS_PXY, or one of TTCF_OBS_N1, _N2, _ENERGY, _SLAB_PX (Eq. TTCF with that
 * B and Omega(0) still -(V/T) gamma_dot P_xy(0); every matching group must have recorded
 * them, else TTCF_ESTATE). TTCF_OBS_SLAB_PX writes n_t x TTCF_BULK_SLABS values (slab
 * fastest) per array. */

/* Section Mathematical Framework: B(t) may be any phase function. Sets whether daughters
 * spawned from now on also record the extra bulk observables (TTCF_OBS_N1 .. _SLAB_PX) after
 * every step, beside V*P_xy; ttcf_accumulate folds them like P_xy. on: 0 or 1. They are
 * recorded by the neighbour-list form with its lists in LDS only: spawning them on a system
 * with FP64 forces fails with TTCF_EINVAL, and so does stepping them in the cell form or with
 * lists in global scratch (a system whose lists do not fit in LDS). Captured graphs record
 * P_xy only: with graphs alive, switching on
 * fails with TTCF_ESTATE, and ttcf_graph_create fails while it is on. The recording costs a
 * second kernel build with the extra pair sums and one more workgroup reduction per step. */
int32_t ttcf_record_observables(ttcf_ctx* ctx, int32_t on);

/* Inspection: the extra observables of live daughters first..first+count-1 that record them:
 * out[(q n_t + k) * (3 + TTCF_BULK_SLABS) + c], c = 0: P_xx - P_yy, 1: P_yy - P_zz,
 * 2: (K + U)/N, 3 + s: slab s of the momentum profile. */
int32_t ttcf_export_observables(ttcf_ctx* ctx, int64_t first, int32_t count, int32_t n_t,
                                double* out);

/* Eq. (corr_modified): the response with the integrand <Omega(0)B(s)> - <Omega(0)><B(s)>,
 * which corrects a finite sample whose <Omega(0)> is not zero (e.g. daughters spawned without
 * all four mappings; with all four it equals ttcf_response's TTCF). B = P_xy. Over the
 * healthy groups at shear rate gamma_dot_filter (> 0; they must share V/T, dt and the number
 * of mapped daughters per group, so that every daughter weighs the same), for
 * k = 0..n_t-1: mean[k] = <B(0)> + trapezoid integral to t_k of the modified integrand, the
 * averages over all their daughters; se[k] = jackknife standard error over the groups (start
 * states). Either pointer may be NULL. Errors: TTCF_EINVAL, TTCF_ESTATE (no matching group,
 * n_t too long). */
int32_t ttcf_response_modified(ttcf_ctx* ctx, double gamma_dot_filter, int32_t n_t, double* mean,
                               double* se, int64_t* out_n_states);
/* ttcf_response_modified for any observable of ttcf_response (TTCF_OBS_SLAB_PX: n_t x
 * TTCF_BULK_SLABS values per array, slab fastest). */
int32_t ttcf_observable_response_modified(ttcf_ctx* ctx, int32_t observable,
                                          double gamma_dot_filter, int32_t n_t, double* mean,
                                          double* se, int64_t* out_n_states);

/* ---- lifetime and errors ------------------------------------------------------------ */

void ttcf_destroy(ttcf_ctx* ctx);              /* NULL-safe; frees all device memory */
const char* ttcf_strerror(int32_t code);       /* static string                      */
const char* ttcf_last_error(const ttcf_ctx* ctx); /* valid until the next call on ctx  */

/* ---- inspection hooks (tests and benchmarks) ---------------------------------------- */

/* Alg. LAMMPS SCRIPT, "run N_s timestep, save system state" alone: the mother advances
 * steps_between steps before each of n_states saved states (replacing the stored set);
 * no daughter is spawned. */
int32_t ttcf_sample_states(ttcf_ctx* ctx, int32_t mother, int32_t n_states,
                           int64_t steps_between);
/* Replace the mother's stored start states by host data (n_states * 3n doubles each for
 * r and p, state-major), so that a daughter batch can start from given states. */
int32_t ttcf_import_states(ttcf_ctx* ctx, int32_t mother, int32_t n_states, const double* r,
                           const double* p);
/* Copy the mother's stored start states to host arrays of the same layout. */
int32_t ttcf_export_states(ttcf_ctx* ctx, int32_t mother, int32_t n_states, double* r,
                           double* p);
/* The thermostat variable of every stored start state (n_states doubles): sampling records
 * the mother's (or its copy's) at each saved state, ttcf_import_states sets 0, and
 * ttcf_import_states_zeta sets given values for the first n_states stored states. Nose-Hoover
 * daughters start from it (TTCF_DAUGHTER_NH). */
int32_t ttcf_import_states_zeta(ttcf_ctx* ctx, int32_t mother, int32_t n_states,
                                const double* zeta);
int32_t ttcf_export_states_zeta(ttcf_ctx* ctx, int32_t mother, int32_t n_states, double* zeta);
/* Beside Alg. LAMMPS SCRIPT's one serial mother: n_replicas copies of the mother's current state,
 * copy q with the momentum kick kicks[q*3n ..] added as given (may be NULL; kicks should sum to
 * zero per copy), run decorrelate_steps Nose-Hoover steps together (one launch), then save
 * states_per_replica states each steps_between steps apart. The stored set is replaced by the
 * n_replicas * states_per_replica states, copy-major. The mother itself does not move. */
int32_t ttcf_sample_states_replicated(ttcf_ctx* ctx, int32_t mother, int32_t n_replicas,
                                      const double* kicks, int64_t decorrelate_steps,
                                      int32_t states_per_replica, int64_t steps_between);
/* Mother's current state: r, p (3n each), the Nose-Hoover variable and the step count. */
int32_t ttcf_export_mother(ttcf_ctx* ctx, int32_t mother, double* r, double* p, double* zeta,
                           int64_t* steps);
/* Sec. Mathematical Framework: the delay T_s between saved states must exceed the time over
 * which the mother's states stay correlated. Autocorrelation of a series x[0..n) (host data,
 * ttcf_acf) or of the mother's recorded V*P_xy series (ttcf_mother_acf), computed on the GPU:
 *   acf[k] = C(k)/C(0), C(k) = sum_{i < n-k} (x_i - m)(x_{i+k} - m) / (n - k), m the mean,
 * for 0 <= k < max_lag (max_lag <= n; compensated FP64 sums). *first_below (may be NULL): the
 * smallest k >= 1 with acf[k] < threshold, -1 if none; *tau_int (may be NULL): the
 * integrated correlation time in steps, 1/2 + sum of acf[k] over 1 <= k < k0, k0 the first
 * lag with acf[k] <= 0 (max_lag if none). A choice of T_s: first_below for a small threshold,
 * or a few tau_int. Errors: TTCF_EINVAL (sizes), TTCF_ESTATE (no recorded series). */
int32_t ttcf_acf(ttcf_ctx* ctx, const double* series, int64_t n, int32_t max_lag,
                 double threshold, double* acf, int32_t* first_below, double* tau_int);
int32_t ttcf_mother_acf(ttcf_ctx* ctx, int32_t mother, int32_t max_lag, double threshold,
                        double* acf, int32_t* first_below, double* tau_int);
/* Mother series: V*P_xy after every step of the last ttcf_init_mother/ttcf_spawn_daughters
 * run on this mother when recording was enabled with ttcf_record_mother (n values). */
int32_t ttcf_record_mother(ttcf_ctx* ctx, int32_t mother, int64_t capacity);
int32_t ttcf_export_mother_series(ttcf_ctx* ctx, int32_t mother, int64_t n, double* vpxy,
                                  int64_t* out_count);
/* A live (not yet accumulated) daughter: r, p (3n each) and its step counter. */
int32_t ttcf_export_daughter(ttcf_ctx* ctx, int64_t daughter, double* r, double* p,
                             int64_t* k);
/* Recorded series of live daughters first..first+count-1: vpxy[d*n_t + k] = V*P_xy(t_k). */
int32_t ttcf_export_series(ttcf_ctx* ctx, int64_t first, int32_t count, int32_t n_t,
                           double* vpxy);
/* Health word of a live daughter (0 = healthy). */
int32_t ttcf_daughter_health(ttcf_ctx* ctx, int64_t daughter, int32_t* health);
/* Failure injection: writes NaN into momentum component 0 of atom 0 of a live daughter. */
int32_t ttcf_debug_poison(ttcf_ctx* ctx, int64_t daughter);

/* Grids of a system (no device work): cells[3] (may be NULL) the canonical cell grid
 * floor(L_a / r_cut) of ttcf_debug_cell_list and the cell form; list_cells[3] (may be NULL)
 * the list grid floor(L_a / (r_cut + skin)) of the pair-list form for skin `skin` (<= 0:
 * automatic), all zero when the box is too small for it; *list_skin (may be NULL) the skin
 * used (the automatic one, or `skin`). TTCF_EINVAL for a system the library refuses. */
int32_t ttcf_cell_grid(const ttcf_system* sys, double skin, int32_t* cells, int32_t* list_cells,
                       double* list_skin);

/* Stateless kernels on given host positions (SoA, inside the box), run on `stream`:
 * the canonical cell list (cell_of[n], order[n], start[n_cells+1]; cell id
 * cx + nx (cy + ny cz), c_a = floor(r_a * (n_a / L_a)), n_a = floor(L_a / r_cut)) ... */
int32_t ttcf_debug_cell_list(const ttcf_system* sys, const double* r, int32_t* dims,
                             int32_t* cell_of, int32_t* order, int32_t* start, void* stream);
/* ... the pairs i<j with squared minimum-image separation < rlist^2 (rlist <= r_cut), found
 * through the cell list at Lees-Edwards offset dxle, sorted by (i, j); *count receives the
 * number found (-1 if cap is too small) ... */
int32_t ttcf_debug_pairs(const ttcf_system* sys, double dxle, const double* r, double rlist,
                         int64_t cap, int32_t* pi, int32_t* pj, int64_t* count, void* stream);
/* ... and one force evaluation: f (3n, SoA), out[0] = U, out[1] = W_xy = sum_{i<j} x_ij F_y,ij,
 * computed in sys->precision. */
int32_t ttcf_debug_forces(const ttcf_system* sys, double dxle, const double* r, double* f,
                          double* out, void* stream);
/* The pair-list form's own list build and force pass (the device functions ttcf_step runs)
 * on given host positions r (SoA, inside the box), at the Lees-Edwards offset of strain step
 * kstep at shear rate gamma_dot (fmod(gamma_dot L_y (kstep dt), L_x), Example 1's sliding
 * brick), list skin `skin` (<= 0: automatic) and pair capacity kcap per atom (<= 0:
 * automatic), FP32 forces whatever sys->precision says. Writes:
 *   dims[3] (may be NULL): the list grid lc_a = floor(L_a / (r_cut + skin));
 *   cell_of[n]: list-grid cell of every atom, cx + lc_x (cy + lc_y cz), c_a = floor(r_a (lc_a /
 *     L_a)) clamped; order[n]: atom ids in the build's order (by cell, then id);
 *     start[cells + 1]: each cell's first position in that order;
 *   pi, pj (capacity cap): the listed pairs as atom ids, pi < pj, sorted; *count their number
 *     (-1 when cap is too small) -- the pairs whose FP32 fixed-point separation is below
 *     r_cut + skin;
 *   f[3n]: the forces the integrator uses; out[0] = W_xy; out[1] = the offset used;
 *   out[2] = r_cut + skin; out[3] = 1 if a pair came closer than the fixed-point force range
 *   allows.
 * Returns TTCF_EUNSTABLE (outputs written, the pair list incomplete) when the capacity
 * overflowed; TTCF_EINVAL for more than 4096 atoms or a box too small for the list grid. */
int32_t ttcf_debug_pair_form(const ttcf_system* sys, double gamma_dot, int64_t kstep, double skin,
                             int32_t kcap, const double* r, int32_t* dims, int32_t* cell_of,
                             int32_t* order, int32_t* start, int64_t cap, int32_t* pi, int32_t* pj,
                             int64_t* count, double* f, double* out, void* stream);

/* For callers that cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): the list build and force pass of
 * ttcf_debug_pair_form (the same kernel) with no allocation of any kind on the device. The
 * pair lists and the build's other by-products go to a static device array of
 * TTCF_STATIC_SCRATCH_BYTES (1 MiB) that every GPU the library runs on holds from the first
 * call there until the process ends; an input that needs more (pair words
 * 64 ceil(n / 256 or 512) * apt * kcap, plus the cells and atoms) returns TTCF_ESCRATCH.
 * Liquids of up to 4096 atoms at the automatic capacity (kcap near 10) fit, and any system of
 * up to 2048 atoms at the largest, kcap = 64.
 *   r:   DEVICE positions (3n FP64, SoA), inside the box (not checked: positions outside
 *        are binned into the edge cells and give meaningless forces, never an access out of
 *        bounds);
 *   f:   DEVICE output, 3n FP64 forces (the ones ttcf_debug_pair_form returns);
 *   out: DEVICE output, 4 FP64: W_xy, 1 if a pair came closer than the fixed-point force
 *        range allows, the Lees-Edwards offset used, 1 if the capacity kcap overflowed (the
 *        forces then miss pairs).
 * Other arguments as for ttcf_debug_pair_form. Enqueued on `stream`, no synchronisation;
 * r, f and out must stay valid until the stream has run it. Calls on one GPU share that
 * GPU's scratch: calls that can overlap on one GPU (other streams, other threads) race and
 * must be ordered by the caller. Nothing in the scratch needs to start at zero. */
int32_t ttcf_pair_forces_static(const ttcf_system* sys, double gamma_dot, int64_t kstep,
                                double skin, int32_t kcap, const double* r, double* f,
                                double* out, void* stream);
enum { TTCF_STATIC_SCRATCH_BYTES = 1 << 20 };

/* Shape of the daughter step kernel (the knobs a tuner searches). variant: 0 automatic,
 * 1 cell list rebuilt every step (FP64 or FP32 forces), 2 pair list of radius r_cut + skin
 * rebuilt when needed (FP32 forces, at most 4096 atoms: every pair within the radius stored
 * once in per-workgroup global scratch, four atoms per thread, pair forces summed in 32-bit
 * fixed point by LDS integer atomics), 3 the same as 2; threads: workgroup size of the cell
 * form (0: the system's block_threads, else the library's choice; the pair form always uses
 * 64 ceil(n / 256) threads per daughter); skin <= 0 selects the automatic skin (the list-cell
 * grid of a 0.2 sigma skin, with the skin widened to fill those cells); kmax: pair capacity
 * per atom of the pair form, at most 64 (<= 0: 1.5 times half the ideal-gas count within the
 * list radius, plus two); a daughter whose list outgrows it is marked unhealthy (list
 * overflow). Affects the following ttcf_step calls; results do not depend on the skin,
 * capacity or rebuild schedule (integer force sums do not depend on their order, and pairs
 * beyond r_cut contribute nothing). */
int32_t ttcf_set_step_shape(ttcf_ctx* ctx, int32_t variant, int32_t threads, double skin,
                            int32_t kmax);

/* Launch-shape autotuner for the batched step of many independent daughters (Sec. Software
 * methodology: the daughter runs are split into independent jobs, one per core). Times the
 * step kernel on probe daughters spawned from the first n_states stored start states of
 * `mother` (0: all; all four mappings, shear rate gamma_dot; the set repeated until there
 * are four daughters per compute unit, so that throughput is measured), over a short untimed
 * warm-up and probe_steps timed steps (they should span several list rebuilds, e.g. the
 * daughter length, or the pick favours short lists), for each candidate shape: the cell form
 * at 256, 512 and 1024 threads, and (FP32 forces) the neighbour-list form at those sizes and
 * at the skins that fill list cells one coarser, equal to and one finer than the automatic
 * grid, its list capacity raised while the probe overflows. Probe daughters are discarded
 * (never accumulated) and live daughters are not advanced. The fastest shape (list capacity
 * plus a margin of 4 where it fits) is stored in the context's cache under (device
 * architecture, N, round(1000 N/V), round(10000 r_cut), precision), replacing an older entry,
 * and written to *out (may be NULL). While no explicit shape is set (ttcf_set_step_shape(ctx,
 * 0, 0, 0, 0), the default), ttcf_step uses the cached shape of each daughter's system, the
 * list grid of its skin and, per launch, the workgroup size of the largest system. Synchronises
 * the context's stream. Errors: TTCF_EINVAL (no stored states, bad arguments, no shape fits),
 * TTCF_EDEVICE (probe daughters unhealthy other than by list overflow, or a HIP error). */
typedef struct ttcf_shape {
    int32_t variant;       /* 1 cell form, 2 neighbour-list form                              */
    int32_t threads;       /* workgroup size                                                  */
    int32_t kmax;          /* neighbour-list capacity per atom (list form)                    */
    double skin;           /* list skin, sigma (list form)                                    */
    double ms_per_step;    /* probe batch, device milliseconds per step                       */
    int32_t candidates;    /* shapes timed                                                    */
} ttcf_shape;
int32_t ttcf_autotune(ttcf_ctx* ctx, int32_t mother, int32_t n_states, double gamma_dot,
                      int32_t probe_steps, ttcf_shape* out);
/* The context's cache of tuned shapes as JSON text: an array of objects with keys arch, n,
 * rho_key, rc_key, precision, variant, threads, kmax, skin, ms_per_step. *len receives the
 * text length (without the terminating NUL); buf (may be NULL) receives at most cap - 1
 * characters and a NUL (TTCF_EINVAL when cap <= len). */
int32_t ttcf_autotune_export(ttcf_ctx* ctx, char* buf, int64_t cap, int64_t* len);
/* Adds the entries of such a text to the cache (replacing equal keys). Entries of other
 * architectures are kept but never used on this device. TTCF_EINVAL on a malformed entry
 * (nothing is added then). */
int32_t ttcf_autotune_import(ttcf_ctx* ctx, const char* text);

/* Device time of the daughter step kernel: total milliseconds and launch count since the
 * last reset (timing events are recorded on the context's stream around every launch). */
int32_t ttcf_step_timing(ttcf_ctx* ctx, double* total_ms, int64_t* launches, int32_t reset);

/* ---- captured batch cycles -----------------------------------------------------------
 * One cycle of Alg. SHELL SCRIPT and Alg. LAMMPS SCRIPT for one mother, recorded once as a
 * HIP graph and replayed without host work: the mother (or its parallel copies) advances and
 * saves start states, the mapped daughters of every state are spawned, run n_steps steps and
 * folded into per-start-state rows, as ttcf_sample_states / ttcf_sample_states_replicated,
 * ttcf_spawn_daughters, ttcf_step and ttcf_accumulate would do them, with the same kernels
 * and launch shapes (the shape is resolved when the graph is created). Every node is a
 * kernel (no memset or copy nodes). */
typedef struct ttcf_graph ttcf_graph;
typedef struct ttcf_graph_desc {
    int32_t mother;
    int32_t n_replicas;          /* 0: the mother itself saves the states; R > 0: R copies of it
                                  * (made at creation with optional momentum kicks, then
                                  * decorrelated) run in parallel and persist across replays */
    const double* kicks;         /* R*3n zero-sum momentum kicks (SoA per copy) or NULL      */
    int64_t decorrelate_steps;   /* copies: steps run once at creation                        */
    int32_t states_per_replica;  /* states saved per copy per replay (R = 0: per replay)      */
    int64_t steps_between;       /* mother steps before each saved state (> 0)                */
    uint32_t mapping_mask;       /* as ttcf_spawn_daughters                                   */
    const double* gamma_dot;     /* n_gamma == 1, or one rate per saved state                 */
    int32_t n_gamma;
    int32_t n_steps;             /* daughter length N_d                                       */
    int32_t max_replays;         /* accumulator rows are reserved for this many replays       */
} ttcf_graph_desc;
/* Records the cycle. Start states are saved copy-major (copy r's states together), groups are
 * numbered state-major as in ttcf_spawn_daughters. Reserves max_replays * (number of saved
 * states) accumulator rows (they count in ttcf_response once written) plus room for 4096
 * rows of ordinary ttcf_accumulate calls: while a graph exists the accumulator cannot grow
 * beyond that (TTCF_ESTATE). The context's mother is advanced by replays in stream order with
 * the context's other work. Errors: TTCF_EINVAL (bad description, shape does not fit),
 * TTCF_ENOMEM, TTCF_EDEVICE (capture or instantiation failed). */
int32_t ttcf_graph_create(ttcf_ctx* ctx, const ttcf_graph_desc* desc, ttcf_graph** out);
/* One cycle over several mothers, for a batch of uneven N (Sec. Software methodology: Alg.
 * SHELL SCRIPT's independent jobs, here one graph): descs[k] describes mother k's part as
 * for ttcf_graph_create (distinct mothers; every part the same n_steps and max_replays, every
 * mother the same force precision). A replay runs each part's mothers and spawns, then steps
 * all daughters together in the persistent launches of their kernel form and thermostat,
 * largest systems first, exactly as ttcf_step steps such a mix, and folds every group; groups
 * are numbered part by part, state-major, as the same ttcf_spawn_daughters calls in part
 * order would number them, and rows are reserved for max_replays times all saved states.
 * Errors as ttcf_graph_create; TTCF_EINVAL for n_desc <= 0 or > 4096. */
int32_t ttcf_graph_create_multi(ttcf_ctx* ctx, const ttcf_graph_desc* descs, int32_t n_desc,
                                ttcf_graph** out);
/* Replays the cycle n_replays times on the context's stream (asynchronous). TTCF_ESTATE when
 * that would exceed max_replays. */
int32_t ttcf_graph_launch(ttcf_graph* graph, int32_t n_replays);
/* Replays so far. */
int32_t ttcf_graph_replays(const ttcf_graph* graph, int32_t* out_replays);
/* Waits for the context's stream and frees the graph and its buffers; rows it has written
 * stay in the accumulator. ttcf_destroy destroys the graphs of its context. */
void ttcf_graph_destroy(ttcf_graph* graph);

/* ---- learned control variate for Eq. (TTCF) ------------------------------------------
 * Not part of the paper's method: a variance-reduction layer over its estimator. A network
 * g(x) predicts B(t_1..t_K) of a daughter from 64 features x of its mapped start state
 * (P_xy(0), Omega(0) of Eq. (TTCF1); per slab of 20 equal slabs in y the sums of p_x, of
 * p_x p_y and of half the pair virials x_ij F_y,ij of its atoms; and the two parts of
 * d(V P_xy)/dt at t = 0 without force derivatives, sum_i (F_x,i p_y,i + p_x,i F_y,i) and
 * sum_{i<j} (p_x,i - p_x,j) F_y,ij; systems up to about 2200 atoms). Each daughter gets h(t_k) = Omega(0) int_0^{t_k} g ds (trapezoid rule on the
 * step grid, g(0) = B(0)); a start state's H_n is the mean of h over its mappings. The
 * estimate is mean_n [G_n(t) - H_n(t)] + mu_H(t), with G_n the start state's Eq. (TTCF)
 * series and mu_H = E[H] over equilibrium start states, estimated from independent mother
 * samples. For any fixed network the estimate is unbiased; a zero network gives Eq. (TTCF).
 *
 * Network: y = W3 gelu(W2 gelu(W1 x' + b1) + b2) + b3 with 256 hidden units, GELU in its
 * erf form, x' the standardised features and y the standardised targets (column mean and
 * standard deviation over the training set, fixed when training starts). Parameters are FP32,
 * laid out flat as W1[64][256], b1[256], W2[256][256], b2[256], W3[256][K], b3[K] (row-major,
 * input index first); 64*256 + 256 + 256*256 + 256 + 256*K + K values. The products run on
 * the bfloat16 matrix cores (operands rounded to nearest even, FP32 accumulation). */

/* (Re)create the network with K = n_out outputs from host weights (n_weights FP32 values in
 * the layout above); clears the Adam moments, the training set and the mean term. */
int32_t ttcf_cv_init(ttcf_ctx* ctx, int32_t n_out, const float* weights, int64_t n_weights);
/* Copy the current parameters to a host array of n_weights floats. */
int32_t ttcf_cv_export_weights(ttcf_ctx* ctx, float* weights, int64_t n_weights);
/* Append live daughters first..first+count-1 (all of one mother, each stepped at least K
 * steps, start states still stored on the mother) to the training set: their features and
 * the targets B(t_1..t_K) = P_xy from their recorded series. */
int32_t ttcf_cv_add_training(ttcf_ctx* ctx, int64_t first, int32_t count);
/* Training rows first_row..first_row+count-1 as stored (raw, not standardised): features
 * x[count][64] and targets t[count][K] (either pointer may be NULL). */
int32_t ttcf_cv_export_training(ttcf_ctx* ctx, int64_t first_row, int32_t count, float* x,
                                float* t);
/* Adam (beta 0.9/0.999, eps 1e-8) on the mean squared error of the standardised targets,
 * batches of `batch` rows, steps = floor(rows / batch) per epoch. order (may be NULL: rows in
 * stored order) holds epochs * rows training-row indices, one permutation per epoch; rows
 * past the last full batch are skipped. loss_out (may be NULL) receives each epoch's loss on
 * its last batch (epochs doubles). */
int32_t ttcf_cv_train(ttcf_ctx* ctx, int32_t epochs, int32_t batch, double lr,
                      const int32_t* order, double* loss_out);
/* Roles of daughters that carry the control variate. */
enum { TTCF_CV_ESTIMATE = 1, TTCF_CV_CALIBRATE = 2 };

/* Give live daughters first..first+count-1 (consecutive ids, one mother, stepped at least
 * once, start states still stored on the mother) their h series from the current network;
 * ttcf_accumulate then carries H_n beside G_n for every group whose daughters all have one in
 * the same role. role TTCF_CV_ESTIMATE: the groups enter ttcf_cv_response; TTCF_CV_CALIBRATE:
 * they only enter ttcf_cv_calibrate. h is zero past t_K. */
int32_t ttcf_cv_attach(ttcf_ctx* ctx, int64_t first, int32_t count, int32_t role);
/* mu_H at shear rate gamma_dot from mother samples that no daughter of the estimate used:
 * n_replicas copies of the mother's current state, copy q with the host momentum kick
 * kicks[q*3n ..] added as given (may be NULL: no kicks; kicks let the copies decorrelate and
 * should sum to zero per copy, so that the total momentum stays zero), run
 * decorrelate_steps Nose-Hoover steps, then `rounds` times: states_per_replica states each
 * steps_between steps apart, all four mappings of each, h from the network, added to the
 * running compensated sums. The mother itself does not move. *out_samples (may be NULL) gets
 * the total number of start states in the mean term. */
int32_t ttcf_cv_mean_term(ttcf_ctx* ctx, int32_t mother, int32_t n_replicas, const double* kicks,
                          int64_t decorrelate_steps, int32_t rounds, int32_t states_per_replica,
                          int64_t steps_between, double gamma_dot, int64_t* out_samples);
/* Control-variate coefficient beta(t_k) = Cov(G_n, H_n) / Var(H_n), k = 0..n_t-1, over the
 * healthy calibration groups at shear rate gamma_dot_filter (0 where H does not vary); kept by
 * the context and used by ttcf_cv_response at that rate. Fitted on groups that the estimate
 * does not use, it leaves the estimate unbiased while never letting a poor network add
 * variance (to within the calibration's own sampling error). beta (may be NULL): n_t doubles. */
int32_t ttcf_cv_calibrate(ttcf_ctx* ctx, double gamma_dot_filter, int32_t n_t, double* beta);
/* Control-variate estimate at k = 0..n_t-1 (n_t <= K + 1) over the healthy estimate groups at
 * shear rate gamma_dot_filter (which must equal the mean term's):
 *   cv_mean = mean_n [G_n - beta H_n] + beta mu_H, beta from ttcf_cv_calibrate (else 1);
 * cv_se, its block standard error over start states (without the mean term's error);
 * plain_mean/plain_se, the Eq. (TTCF) estimate over the same groups; mu_h/mu_h_se, the added
 * term beta mu_H and its standard error (samples taken as independent). Any pointer may be
 * NULL. */
int32_t ttcf_cv_response(ttcf_ctx* ctx, double gamma_dot_filter, int32_t n_t, double* cv_mean,
                         double* cv_se, double* plain_mean, double* plain_se, double* mu_h,
                         double* mu_h_se, int64_t* out_n_states);
/* The network alone (tests): forward pass on host rows x[rows][64] (fed to W1 unstandardised)
 * into y[rows][K] ... */
int32_t ttcf_mlp_forward(ttcf_ctx* ctx, const float* x, int32_t rows, float* y);
/* ... and the gradient of mean((y - target)^2) over all rows*K elements with respect to the
 * parameters, in the flat layout (n_weights floats into grad). */
int32_t ttcf_mlp_gradient(ttcf_ctx* ctx, const float* x, const float* target, int32_t rows,
                          float* grad);

/* ---- the confined channel (the paper's second example) -------------------------------
 * Eq. system2: a Lennard-Jones liquid between two walls; wall atoms are tethered by springs
 * of stiffness k to lattice sites, the lattices move along x at +v/2 (top) and -v/2 (bottom),
 * and a Nose-Hoover thermostat acts on the wall atoms only. Pairs interact by
 * 4[(1/r)^12 - c (1/r)^6] (shifted to vanish at r_cut) with c = c_ff (fluid-fluid) or c_wf
 * (wall-fluid); wall atoms do not interact with each other. x and z are periodic; y is
 * bounded by the walls. Integration: velocity Verlet with the thermostat's half steps around
 * it (time reversible). FP32 pair forces, FP64 tethers, positions, momenta and sums.
 * Dissipation function (Eq. TTCF2 with beta = 1/T and the sign of the adiabatic energy
 * balance): Omega(0) = -(k v / (2 T)) S(0), S = sum_top (x^w - x^l) - sum_bottom (x^w - x^l).
 * Observables B(t): TTCF_OBS_WALL_STRESS, [sum_{fluid i, top j} F_x,ij -
 * sum_{fluid i, bottom j} F_x,ij] / (2 lx lz) (the method-of-planes stress at the
 * interfaces); TTCF_OBS_VPROFILE, per bin of y in [bin_lo, bin_hi), the fluid's summed p_x
 * over the bin volume.
 * Mappings (Eq. mappings, applied to atoms and lattice sites): 1 reverses p and the
 * thermostat variable; 2 reflects x and reverses p_x; 3 reflects x and reverses p_y, p_z and
 * the thermostat variable. Arrays are SoA over all atoms: fluid first, then the bottom wall,
 * then the top wall; lattice arrays are SoA over the wall atoms (bottom then top).
 * Results are deterministic for a given sequence of calls. */
typedef struct ttcf_channel_ctx ttcf_channel_ctx; /* opaque, owned by the library */

typedef struct {
    int32_t n_fluid;      /* fluid atoms                                                   */
    int32_t n_wall;       /* wall atoms of both walls (even; the first half is the bottom) */
    int32_t n_bins;       /* momentum-profile bins, 1..256                                 */
    int32_t kmax;         /* neighbour-list capacity per atom (<= 0: 160)                  */
    double lx, lz;        /* periodic edges                                                */
    double y_extent;      /* every atom stays inside [0, y_extent)                         */
    double r_cut, c_ff, c_wf, k_spring;
    double temperature;   /* wall thermostat target                                        */
    double dt, nh_tau;    /* thermostat mass Q = 3 N_w T nh_tau^2                          */
    double bin_lo, bin_hi;
    double skin;          /* neighbour-list skin (<= 0: 0.4, less where a small box needs
                           * it for 3 list cells across x and z and 4 along y; at least 0.1) */
} ttcf_channel;

/* Alg. LAMMPS SCRIPT "initialise": a context holding the mother (positions r0, momenta p0,
 * 3 n each; lattice sites, 3 n_wall; thermostat variable 0) on `stream`. */
int32_t ttcf_channel_create(ttcf_channel_ctx** ctx, const ttcf_channel* ch, const double* r0,
                            const double* p0, const double* lattice, void* stream);
void ttcf_channel_destroy(ttcf_channel_ctx* ctx);
const char* ttcf_channel_last_error(const ttcf_channel_ctx* ctx);
/* "run N_t timestep": the equilibrium mother (lattices at rest) advances n_steps. */
int32_t ttcf_channel_run_mother(ttcf_channel_ctx* ctx, int64_t n_steps);
/* "run N_s timestep, save system state", n_states times: replaces the stored start states. */
int32_t ttcf_channel_sample_states(ttcf_channel_ctx* ctx, int32_t n_states,
                                   int64_t steps_between);
/* Beside the one serial mother (as ttcf_sample_states_replicated for the bulk): n_replicas
 * copies of the mother's current state, copy q with the momentum kick kicks[q*3n ..] added
 * (may be NULL; kicks let the copies decorrelate and should sum to zero per component), run
 * the mother's dynamics in one persistent launch: decorrelate_steps steps, then
 * states_per_replica states each steps_between steps apart. The stored set is replaced by
 * the n_replicas * states_per_replica states, copy-major, with each copy's wall thermostat
 * variable. The mother itself does not move. TTCF_EUNSTABLE if a copy fails its health
 * check (the stored set is then empty). */
int32_t ttcf_channel_sample_states_replicated(ttcf_channel_ctx* ctx, int32_t n_replicas,
                                              const double* kicks, int64_t decorrelate_steps,
                                              int32_t states_per_replica,
                                              int64_t steps_between);
/* Stored start states from / to host arrays: r, p (n_states x 3n), zeta (n_states). */
int32_t ttcf_channel_import_states(ttcf_channel_ctx* ctx, int32_t n_states, const double* r,
                                   const double* p, const double* zeta);
int32_t ttcf_channel_export_states(ttcf_channel_ctx* ctx, int32_t n_states, double* r, double* p,
                                   double* zeta);
int32_t ttcf_channel_export_mother(ttcf_channel_ctx* ctx, double* r, double* p, double* zeta,
                                   int64_t* steps);
/* Map the first n_states stored states (mapping_mask as for the bulk), set the lattice speed
 * v (n_v == 1, or one per state), daughters of n_steps >= 1 steps, numbered state-major from
 * *out_first. */
int32_t ttcf_channel_spawn(ttcf_channel_ctx* ctx, int32_t n_states, uint32_t mapping_mask,
                           const double* v, int32_t n_v, int32_t n_steps, int64_t* out_first);
/* "run N_d timestep": every live daughter advances up to n_steps (one launch per batch),
 * recording the observables after every step. Asynchronous. */
int32_t ttcf_channel_step(ttcf_channel_ctx* ctx, int32_t n_steps);
/* Fold finished batches into per-start-state rows (mapping means of B(t) and of
 * int_0^t S(0) B(s) ds, compensated FP64); a group with an unhealthy daughter is excluded. */
int32_t ttcf_channel_accumulate(ttcf_channel_ctx* ctx, int64_t* out_groups);
/* Eq. TTCF and the direct average of one observable at lattice speed v_filter (exact match),
 * k = 0..n_t-1; TTCF_OBS_VPROFILE writes n_t x n_bins values (bin fastest) per array. Block
 * standard errors over start states. Any pointer may be NULL. */
int32_t ttcf_channel_response(ttcf_channel_ctx* ctx, int32_t observable, double v_filter,
                              int32_t n_t, double* ttcf_mean, double* ttcf_se, double* dav_mean,
                              double* dav_se, int64_t* out_n_states);
/* Inspection: recorded observables of live daughters (count x n_t x (1 + n_bins)) and their
 * S(0); a daughter's state; its health word; one force evaluation of a configuration at the
 * lattice sites given (f: 3n, out[0..2] = x force on the fluid from the top and from the
 * bottom wall and S, out[3] = list overflow, out[4] = an atom outside [0, y_extent)); the
 * device time of the step kernel. */
int32_t ttcf_channel_export_series(ttcf_channel_ctx* ctx, int64_t first, int32_t count,
                                   int32_t n_t, double* obs, double* s0);
int32_t ttcf_channel_export_daughter(ttcf_channel_ctx* ctx, int64_t daughter, double* r,
                                     double* p, double* zeta);
int32_t ttcf_channel_daughter_health(ttcf_channel_ctx* ctx, int64_t daughter, int32_t* health);
int32_t ttcf_channel_debug_forces(const ttcf_channel* ch, const double* r, const double* lattice,
                                  double* f, double* out, void* stream);
int32_t ttcf_channel_step_timing(ttcf_channel_ctx* ctx, double* total_ms, int64_t* launches,
                                 int32_t reset);

#ifdef __cplusplus
}
#endif
#endif
