/*
 * channel_oracle.h -- FP64 CPU oracle of the confined-channel example (Eq. system2,
 * Eq. TTCF2 of arxiv 2312.02990). TEST INFRASTRUCTURE; shares no code with the GPU library.
 *
 * Layout: positions and momenta are SoA over all atoms (fluid, then bottom wall, then top
 * wall): r = [x(0..n-1) | y | z]. Lattice sites rl are SoA over the wall atoms only.
 */
#ifndef TTCF_CHANNEL_ORACLE_H
#define TTCF_CHANNEL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n;        /* all atoms                                                      */
    int32_t n_fluid;  /* atoms 0..n_fluid-1                                             */
    int32_t n_wall;   /* both walls; the first half is the bottom wall                  */
    int32_t n_bins;   /* momentum-profile bins                                          */
    double lx, lz;    /* periodic edges                                                 */
    double rc;        /* cutoff of every pair type                                      */
    double c_ff, c_wf;/* wetting factors: fluid-fluid, wall-fluid                        */
    double k_spring;  /* tether stiffness                                               */
    double bin_lo, bin_hi; /* y range of the profile bins                              */
} orc_channel;

/* Forces (LJ pairs with at least one fluid atom, plus tethers to the lattice sites rl).
 * out[0] = LJ energy, out[1] = spring energy, out[2] = x force on the fluid from the top
 * wall, out[3] = same from the bottom wall, out[4] = S = sum_top dx - sum_bottom dx of the
 * tether extensions (minimum image). */
int32_t orc_ch_forces(const orc_channel* c, const double* r, const double* rl, double* f,
                      double* out);
/* Observables from a force evaluation's out[]: obs[0] wall shear stress, obs[1..n_bins] the
 * x-momentum density per bin. */
void orc_ch_observables(const orc_channel* c, const double* r, const double* p,
                        const double* fout, double* obs);
/* Velocity Verlet with a Nose-Hoover thermostat on the wall atoms (q <= 0: none), lattices
 * moving at +-v/2 along x from rl0 (their position at step k is rl0 +- (v/2) k dt), starting
 * at step k0. Per-step outputs (steps 0..nsteps, any may be NULL): obs_out[(1+n_bins) per
 * step], s_out (the S observable), energy_out (kinetic + LJ + spring energy). */
int32_t orc_ch_run(const orc_channel* c, double t_wall, double q, double dt, double v,
                   double* r, double* p, double* zeta, const double* rl0, int64_t k0,
                   int64_t nsteps, double* obs_out, double* s_out, double* energy_out);
/* Mappings: 0 identity, 1 (p, zeta) -> -(p, zeta), 2 x-reflection of atoms and lattice
 * sites with p_x -> -p_x, 3 both (x reflected, p_y and p_z and zeta reversed). */
void orc_ch_map(const orc_channel* c, int32_t m, const double* r, const double* p, double zeta,
                const double* rl, double* r_out, double* p_out, double* zeta_out,
                double* rl_out);
/* Mapped daughters of stored states (rl: the mother's lattice sites) at lattice speeds v_of,
 * one per thread at a time. obs: n_daughters x (nsteps+1) x (1+n_bins); s0: S(0) of each. */
int32_t orc_ch_run_daughters(const orc_channel* c, double t_wall, double q, double dt,
                             const double* states_r, const double* states_p,
                             const double* states_zeta, const double* rl, const int32_t* state_of,
                             const int32_t* map_of, const double* v_of, int32_t n_daughters,
                             int32_t nsteps, double* obs, double* s0, int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
