// ttcf_internal.h -- device-side parameter blocks and kernel launchers shared by the
// gfx950 kernels (ttcf_kernels.hip) and the host runtime behind the C ABI (ttcf_capi.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ttcf {

constexpr int kMaxThreads = 1024;
constexpr int kMaxWaves = kMaxThreads / 64;
constexpr int kRedSlots = 12;       // doubles reduced per block reduction
constexpr int kMaxCells1D = 1023;   // packed cell coordinates use 10 bits each
constexpr int kMaxAtoms = 65535;    // sorted atom ids are stored as uint16
constexpr int kPefMaxAtoms = 2048;  // planar-elongation daughters: two atoms per thread

// Constants of one simulated system, uniform inside a workgroup.
struct SysDev {
    int32_t n;          // atoms
    int32_t nc[3];      // cell grid, n_a = floor(L_a / r_cut)
    double box[3];      // L_a
    double w[3];        // cell widths L_a / n_a
    double inv_w[3];    // n_a / L_a (one FP64 division on the host, as the cell index needs)
    double rc, rc2;     // cutoff and its square
    double c_attr;      // attraction factor c
    double u_shift;     // energy shift
    double dt;
    double volume;
    // neighbour-list form: list-build grid with cells of width >= rc + skin, and the
    // 32-bit fixed-point map of the box (coordinate * 2^32 / L, so integer differences are
    // minimum-image separations)
    int32_t lc[3];
    double lw[3];
    double l_inv_w[3];
    double skin;
    double fix_scale[3];   // 2^32 / L_a
    float fix_unit[3];     // L_a / 2^32
    float rc2_f;           // cutoff^2 and list radius^2 in FP32
    float rl2_f;
    // pair-list form: pairs closer than this (squared, FP32) have a force that could leave
    // the range of the fixed-point force accumulators; meeting one marks the daughter
    float rg2_f;
};

// Observables recorded beside V*P_xy when a daughter has an extra series (kObsCols per time
// point): P_xx - P_yy, P_yy - P_zz, (K + U)/N, and kObsSlabs values of the y-slab profile
// sum(p_x)/(slab volume), slab s holding floor(y kObsSlabs / L_y) = s.
constexpr int kObsSlabs = 8;
constexpr int kObsCols = 3 + kObsSlabs;

// Pair-list form: largest system (eight atoms per thread, 512 threads; pair words hold
// 14-bit atom ranks), the largest pair capacity per atom, and the force magnitude whose
// pairs are flagged (the fixed-point accumulators hold +-4096 force units).
constexpr int kPairMaxAtoms = 4096;
constexpr int kPairMaxCap = 64;
constexpr double kPairForceGuard = 1024.0;

// One daughter trajectory. Owned by the host runtime; the kernel updates k, done, health.
struct DaughterDesc {
    double* state;      // 6n doubles: x | y | z | px | py | pz
    double* series;     // n_steps + 1 doubles: V * P_xy(t_k)
    SysDev sys;
    double gamma_dot;
    double k0;          // kinetic energy held by the isokinetic constraint
    int64_t k;          // strain counter: LE offset = fmod(gamma_dot Ly (k dt), Lx)
    int32_t n_steps;    // daughter length N_d
    int32_t done;       // steps completed so far
    int32_t health;     // 0 healthy; bit 0 non-finite, bit 1 kinetic-energy drift
    int32_t group;      // start-state group (accumulator slot)
    int32_t map;        // mapping 0..3
    int32_t block;      // threads per workgroup the launcher was sized for
    int32_t kmax;       // pair-list form: pair capacity per atom (a wave's segment holds
                        // kmax * 256 pairs)
    double* hseries;    // n_steps + 1 doubles: learned control variate h(t_k), or null
    // thermostat of the daughter: 0 Gaussian isokinetic, 1 Nose-Hoover (zeta carried from the
    // start state; d zeta/dt = (sum p^2 - nh_target)/nh_q)
    int32_t thermo;
    int32_t field;      // kFieldShear, or kFieldColour (gamma_dot 0, fe the field strength)
    double zeta;
    double nh_q;
    double nh_target;
    double* xseries;    // (n_steps + 1) x kObsCols extra observables, or null
    double fe;          // colour field strength F_e (kFieldColour)
    int32_t pad2_;
    int32_t pad3_;
    // mixed flow (kFieldMixed): u_x = erate x + srate y, u_y = -erate y; gamma_dot holds
    // sqrt(erate^2 + srate^2)
    double erate, srate;
};

// External field of a daughter: SLLOD shear at gamma_dot, the colour field (charge +1 on
// even atoms, -1 on odd ones, force charge * F_e along x; series V J_x = sum charge p_x), or
// planar elongational flow at rate gamma_dot (grad u = diag(rate, -rate, 0) in a deforming
// box; series V (P_xx - P_yy); k counts the steps that set the box strain rate k dt).
// Mixed flow: shear and planar elongation together (erate, srate), series V J with
// J = (erate (P_xx - P_yy) + srate P_xy) / sqrt(erate^2 + srate^2).
enum Field : int32_t { kFieldShear = 0, kFieldColour = 1, kFieldElong = 2, kFieldMixed = 3 };

enum Health : int32_t {
    kHealthNonFinite = 1,
    kHealthDrift = 2,
    kHealthListOverflow = 4,
    kHealthForceRange = 8  // a pair came closer than the fixed-point force range allows
};

// Daughter step kernels: the cell-list form rebuilds a canonical cell list every step and
// evaluates pairs over the 27-cell stencil (FP64 or FP32 forces); the pair-list form (FP32
// forces) keeps every pair within rc + skin once in a list in global scratch, rebuilt only
// when the atoms have moved far enough to require it.
enum Variant : int32_t { kVariantCells = 0, kVariantNeighbourList = 1 };

// Launch configuration of the persistent daughter kernel.
struct BatchLaunch {
    DaughterDesc* descs;   // device array
    const int32_t* order;  // device: job order (largest systems first)
    int32_t n_jobs;
    int32_t* queue;        // device counter (zeroed by the launcher)
    int32_t max_steps;     // steps this call (each daughter stops at its own N_d)
    int32_t threads;       // workgroup size
    int32_t apt;           // atoms per thread (template selector: 1, 2, 4 or 8)
    int32_t precision;     // 0 FP64 forces, 1 FP32 forces
    int32_t grid;          // workgroups (persistent)
    int32_t nmax, cmax;    // largest system / cell grid in the batch (LDS sizing)
    int32_t variant;       // Variant
    int32_t kmax;          // pair capacity per atom (pair-list form)
    int32_t thermo;        // daughter thermostat of every job (0 isokinetic, 1 Nose-Hoover)
    int32_t obs;           // 1: some job records the extra observables (list form only)
    int32_t field;         // 1: some job is a colour-field daughter (list form)
    int32_t pairs_lds;     // pair-list form: 1 if each job's pair words live in LDS after its
                           // layout (lds_bytes covers lds_bytes_pairs_lds of every job)
    uint32_t* pairs;       // pair-list form otherwise: grid x pair_stride pair words
    int64_t pair_stride;   // >= job_threads(n) / 64 * 256 * kmax of every job
    size_t lds_bytes;
};

// Planar-elongation daughters (ttcf_elongation.hip): one workgroup per job, two atoms per
// thread, FP64 forces over a cell grid rebuilt every step from the deformed box; one launch
// per daughter thermostat.
struct PefLaunch {
    DaughterDesc* descs;   // device array
    const int32_t* order;  // device: desc index of each job
    int32_t n_jobs;
    int32_t max_steps;     // steps this call (each daughter stops at its own N_d)
    int32_t threads;       // pef_threads(nmax)
    int32_t nmax;          // largest system
    int32_t cmax;          // >= the cell count of any job's box at any step
    int32_t thermo;        // daughter thermostat of every job (0 isokinetic, 1 Nose-Hoover)
    int32_t mix;           // 1: mixed-flow daughters (k_daughters_mix)
    size_t lds_bytes;      // lds_bytes_pef(nmax, cmax)
};

struct MotherLaunch {
    SysDev sys;
    double* state;         // 6n doubles
    double* zeta;          // device scalar: Nose-Hoover variable
    double temperature;    // target
    double q;              // thermostat mass
    double nf;             // degrees of freedom
    int64_t n_chunks;      // snapshots to take (0: just run steps_per_chunk)
    int64_t steps_per_chunk;
    double* snapshots;     // n_chunks * 6n doubles, or nullptr
    double* snap_zeta;     // n_chunks doubles: the thermostat variable at each snapshot, or nullptr
    double* series;        // V*P_xy after every step (n_chunks*steps_per_chunk), or nullptr
    int32_t threads, apt, precision;
    size_t lds_bytes;
};

struct AccumLaunch {
    const DaughterDesc* descs;   // device
    const int32_t* first_of;     // device: first desc index of each group (n_groups + 1)
    double* d_out;               // n_groups rows of stride n_t: mean over mappings of P_xy(t_k)
    double* i_out;               // same: mean over mappings of int_0^t P_xy(0) P_xy(s) ds
    int32_t* health_out;         // n_groups
    double* gamma_out;           // n_groups
    double* h_out;               // same layout: mean over mappings of h(t_k) (0 without CV)
    int32_t n_groups, n_t;
    int32_t row_stride;          // doubles between output rows (0: n_t)
    const int32_t* row_step;     // device counter or null: outputs start (*row_step) * n_groups
                                 // rows further on (a replayed graph writes fresh rows each time)
};

struct ResponseLaunch {
    const double* d_all;         // groups' direct-average series (row stride n_t_stride)
    const double* i_all;         // groups' integral series
    const double* gamma;         // per group shear rate
    const double* coef;          // per group V gamma / T (Omega(0) = -coef P_xy(0))
    const int32_t* health;       // per group health
    const int32_t* rows;         // selected group rows
    int32_t n_rows, n_t, n_t_stride;
    int32_t normalise;           // divide each group by its own shear rate
    const double* h_all;         // groups' control-variate series, or null (plain TTCF)
    const double* mu_h;          // control-variate mean term per time point, or null
    const double* beta;          // control-variate coefficient per time point, or null (1)
    double* out;                 // 4 * n_t: ttcf mean, ttcf se, dav mean, dav se
    int32_t* used;               // number of healthy rows
};

// ---- learned control variate ---------------------------------------------------------
constexpr int kCvIn = 64;       // features per start state
constexpr int kCvSlabs = 20;    // y slabs of the binned features (3 per slab, then 2 rates)
constexpr int kCvHidden = 256;  // hidden width of both hidden layers

struct GemmArgs {
    const float* A;
    int64_t sam, sak;            // A(m, k) = A[m sam + k sak]
    const float* B;
    int64_t sbk, sbn;            // B(k, n) = B[k sbk + n sbn]
    float* C;
    int ldc;
    const float* bias;           // epilogue 0/1
    float* Z;                    // epilogue 1: pre-activation output
    const float* Zin;            // epilogue 2: pre-activation input
    int M, N, K;
    int epi;                     // 0 C = AB + bias; 1 Z = AB + bias, C = gelu(Z); 2 C = AB gelu'(Zin)
};

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s);
hipError_t launch_colsum(const float* X, int M, int N, int ld, float* out, hipStream_t s);
hipError_t launch_mse_grad(const float* Y, const float* Tg, int64_t count, float scale, float* dY,
                           hipStream_t s);
hipError_t launch_mse_loss(const float* Y, const float* Tg, int64_t count, double* loss,
                           hipStream_t s);
hipError_t launch_adam(float* P, const float* G, float* Mo, float* Vo, int64_t n, float lr,
                       int64_t step, hipStream_t s);
hipError_t launch_gather_norm(const float* src, const int32_t* idx, int rows, int cols,
                              const float* mu, const float* inv, float* dst, hipStream_t s);
hipError_t launch_col_stats(const float* X, int64_t rows, int cols, float* mu, float* inv,
                            hipStream_t s);
hipError_t launch_cv_gather_series(const double* const* series, int32_t count, int32_t n_out,
                                   double inv_volume, float* targets, double* vpxy0, hipStream_t s);
hipError_t launch_cv_scatter_h(const double* h, int32_t stride, int32_t count, double* const* dst,
                               const int32_t* lens, hipStream_t s);
hipError_t launch_cv_beta(const ResponseLaunch& r, double* beta, hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, int64_t count, hipStream_t s);
size_t lds_bytes_cv_features(int32_t n);
size_t lds_bytes_cv_features_maps(int32_t n);
// the features of rows 4 s + m (m = 0..3, the four mappings) of each of n_states states, the
// pair sums done once per state; vpxy0 by state, vsign by mapping
hipError_t launch_cv_features_maps(const double* states, int32_t n, int32_t n_states,
                                   const double* vpxy0, const double* vsign, const double* box,
                                   double rc2, double c_attr, double volume, double temperature,
                                   double gamma_dot, float* out, double* b0_out, double* om_out,
                                   hipStream_t s);
hipError_t launch_cv_features(const double* states, int32_t n, const int32_t* state_of,
                              const int32_t* map_of, const double* vpxy0, const double* vsign,
                              int32_t rows, const double* box, double rc2, double c_attr,
                              double volume, double temperature, double gamma_dot, float* out,
                              double* b0_out, double* om_out, hipStream_t s);
hipError_t launch_cv_h(const float* pred, int rows, int n_out, const float* ymu, const float* yinv,
                       const double* b0, const double* omega, double dt, double* out,
                       int64_t out_stride, hipStream_t s);
// part: cv_mu_scratch_doubles(nt) doubles of device scratch for the partial sums
size_t cv_mu_scratch_doubles(int nt);
hipError_t launch_cv_mu_accum(const double* h, int groups, int maps, int nt, double* sum,
                              double* comp, double* sumsq, double* compsq, double* part,
                              hipStream_t s);
hipError_t launch_states_vpxy(const SysDev& sys, const double* states, int32_t count, double* out,
                              hipStream_t s);

// Host-side choice of the per-daughter kernel shape.
int pick_threads(int n, int requested);
int pick_apt(int n, int threads);
size_t lds_bytes_for(int nmax, int cmax, int threads, int precision);
// Pair-list form (ttcf_pairs.hip): LDS of one job of n atoms and `cells` list cells (a launch
// needs the largest over its daughters), the threads that own a job's atoms (four each), and
// the pair words of its segments per workgroup for a capacity of kcap pairs per atom.
size_t lds_bytes_pairs(int n, int cells);
int pair_job_threads(int n);
int pair_job_apt(int n);
int pair_small_apt();  // atoms per thread of the systems whose pair words can sit in LDS
// a launch runs every job with `apt` atoms per thread (the largest job's), so a job's wave
// segments hold 64 apt kcap words each
inline int64_t pair_words(int n, int kcap, int apt) {
    return (int64_t)pair_job_threads(n) * apt * kcap;
}
// LDS of one job with its pair words in LDS too (after the job's layout)
inline size_t lds_bytes_pairs_lds(int n, int cells, int kcap, int apt) {
    return lds_bytes_pairs(n, cells) + sizeof(uint32_t) * (size_t)pair_words(n, kcap, apt);
}
hipError_t launch_pairs(const BatchLaunch& b, hipStream_t s);
// The pair form's list build and one force pass on given positions (inspection): per atom its
// list-grid cell and rank, the cell starts (cells + 1), the pair words of each wave segment
// (kcap * 64 * apt per wave) and their counts, the forces (3n), out[0] = W_xy, out[1] = 1 if
// a pair fell inside the guard radius, out[2] = the Lees-Edwards offset used, out[3] = 1 if
// a wave's pair list outgrew its segment (the list then incomplete).
hipError_t launch_debug_pair_form(const SysDev& S, double gamma_dot, int64_t kstep, const double* r,
                                  int32_t kcap, uint32_t* pairs, int32_t* seg_count,
                                  int32_t* cell_of, int32_t* rank_of, int32_t* start, double* f,
                                  double* out, hipStream_t s);

hipError_t launch_daughters(const BatchLaunch& b, hipStream_t s);
hipError_t launch_mothers(const MotherLaunch* dev_ms, int count, const MotherLaunch& shape,
                          hipStream_t s);
hipError_t launch_replicate(const double* src, const double* zsrc, int32_t n, const double* kicks,
                            int32_t count, double* dst, double* zdst, hipStream_t s);
hipError_t launch_accumulate(const AccumLaunch& a, hipStream_t s);
// dst[i] = src[i], i < count (64-bit words)
hipError_t launch_copy_words(const uint64_t* src, uint64_t* dst, int64_t count, hipStream_t s);
// descs[d].zeta = zeta[state_of[d]], reversed for the time-reversing mappings (map_of odd)
hipError_t launch_desc_zeta(DaughterDesc* descs, const double* zeta, const int32_t* state_of,
                            const int32_t* map_of, int32_t count, hipStream_t s);
// Autocorrelation of x[0..n) at lags 0..max_lag-1 (normalised by C(0)), the first lag below
// threshold and the integrated correlation time; scratch: 1 double (the mean)
hipError_t launch_acf(const double* x, int64_t n, int32_t max_lag, double threshold,
                      double* scratch, double* acf, int32_t* first_below, double* tau_int,
                      hipStream_t s);
// Eq. (corr_modified) over selected accumulator rows sharing coef and dt (ttcf_estimators.hip)
struct ModifiedLaunch {
    const double* d_all;   // accumulator rows of B: D_n(t), I_n(t), row stride `stride`
    const double* i_all;
    int32_t stride;
    const double* p_all;   // P_xy direct-average rows (their t = 0 value gives <Omega(0)>),
    int32_t p_stride;      // row stride p_stride (B = P_xy: p_all = d_all)
    const int32_t* rows;   // selected rows
    int32_t n_rows, n_t;
    double coef;           // V gamma_dot / T of every selected row
    double dt;             // time step of every selected row
    double* j_rows;        // n_rows x n_t scratch
    double* out;           // [0, n_t): estimate, [n_t, 2 n_t): jackknife standard error
};
hipError_t launch_response_modified(const ModifiedLaunch& a, hipStream_t s);

// Accumulation of the extra observables: per group and column c, the mapping means
// D_n,c(t_k) of B_c(t_k) and I_n,c(t_k) of int_0^t P_xy(0) B_c(s) ds (trapezoid rule).
// Output row of group g, column c: d_out + g * row_stride + c * stride (n_t values).
struct AccumObsLaunch {
    const DaughterDesc* descs;   // device: every daughter has an xseries
    const int32_t* first_of;     // device: n_groups + 1
    double* d_out;
    double* i_out;
    int32_t n_groups, n_t;
    int64_t stride, row_stride;
};
hipError_t launch_accumulate_obs(const AccumObsLaunch& a, hipStream_t s);
// *counter += 1 (one thread)
hipError_t launch_increment(int32_t* counter, hipStream_t s);
hipError_t launch_response(const ResponseLaunch& r, hipStream_t s);
int pef_threads(int nmax);
int pef_max_cells(double volume, double rc);
size_t lds_bytes_pef(int nmax, int cmax);
hipError_t launch_pef(const PefLaunch& L, hipStream_t s);
hipError_t launch_spawn_pef(const double* states, int32_t n, const int32_t* state_of,
                            const int32_t* map_of, double* const* dst, int32_t n_daughters,
                            int32_t mix, double lx, hipStream_t s);
hipError_t launch_spawn(const double* states, int32_t n, int32_t n_states, const int32_t* state_of,
                        const int32_t* map_of, double* const* dst, int32_t n_daughters, double lx,
                        hipStream_t s);
hipError_t launch_debug_cells(const SysDev& sys, const double* r, int32_t* cell_of, int32_t* order,
                              int32_t* start, hipStream_t s);
hipError_t launch_debug_pairs(const SysDev& sys, double dxle, const double* r, double rlist,
                              int64_t cap, int32_t* pi, int32_t* pj, unsigned long long* count,
                              hipStream_t s);
hipError_t launch_debug_forces(const SysDev& sys, int precision, double dxle, const double* r,
                               double* f, double* out, hipStream_t s);

}  // namespace ttcf
