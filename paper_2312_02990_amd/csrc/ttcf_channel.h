// ttcf_channel.h -- parameter blocks and launchers of the confined-channel kernels
// (ttcf_channel.hip) shared with their host runtime (ttcf_channel_capi.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ttcf_internal.h"

namespace ttcf {

constexpr int kChThreads = 1024;  // loops over atoms
constexpr int kChWavesPerSimd = 4;  // register budget of the step kernel: 128 VGPRs per lane
constexpr int kChMaxWaves = kChThreads / 64;
constexpr int kChRed = 4;          // doubles per block reduction
constexpr int kChMaxBins = 256;

// Constants of one channel system (uniform in a workgroup).
struct ChannelDev {
    int32_t n, n_fluid, n_wall, n_bins;
    int32_t lc[3];          // list grid: cells at least r_c + skin wide (y: over [0, y_extent))
    int32_t kmax;           // list capacity per atom
    double lx, lz, y_extent;
    double rc, skin;
    double c_ff, c_wf, k_spring;
    double temperature, q, nf_w, dt;
    double bin_lo, bin_hi, bin_w;
    double fix_scale[3];    // 2^32 / (lx, y_extent, lz)
    float fix_unit[3];      // (lx, y_extent, lz) / 2^32
    float rc2_f, rl2_f;
};

// One trajectory (a daughter, or the mother with series == null and v == 0).
struct ChannelDesc {
    double* r;              // 3n, SoA
    double* p;              // 3n
    float* f;               // 3n, forces at the current positions
    double* latx;           // n_wall lattice x at step 0 (mapped for reflected daughters)
    const double* laty;     // n_wall (shared with the mother)
    const double* latz;
    double* series;         // (n_steps + 1) x (1 + n_bins) observables, or null
    double v;               // relative lattice speed (top +v/2, bottom -v/2)
    double zeta;            // wall thermostat variable
    double pw2;             // sum of wall p^2 of the current state
    double s0;              // S at step 0 (written by the kernel)
    int64_t k;              // step counter (lattice position)
    int32_t n_steps, done, health, state, map, pad_;
};

struct ChannelLaunch {
    ChannelDev sys;
    ChannelDesc* descs;
    const int32_t* order;   // job order (null: 0..n_jobs-1)
    int32_t n_jobs, grid, cmax, max_steps;
    int32_t* queue;
    char* scratch;          // grid x scratch_stride bytes
    size_t scratch_stride;
};

struct ChannelAccum {
    const ChannelDesc* descs;  // the groups' daughters, consecutive
    const int32_t* first_of;   // n_groups + 1
    double* d_out;             // n_groups rows of row_stride doubles, each n_t x n_obs used
    double* i_out;
    int32_t n_groups, n_t, n_obs;
    double dt;
    size_t row_stride;         // >= n_t * n_obs
};

struct ChannelResponse {
    const double* d_all;
    const double* i_all;
    const double* coef;        // per row: k v / (2 T)
    const int32_t* rows;
    int32_t n_rows, n_t, n_obs, col0, n_cols;
    size_t row_stride;         // doubles per row (n_t_max x n_obs)
    double* out;               // 4 planes of n_t x n_cols
};

size_t channel_lds_bytes(int nmax, int cmax);
// replicas of the mother (momenta plus optional kicks) and snapshots of replicas into the
// stored start states (slot q * per + slot of replica q)
hipError_t launch_channel_replicate(const double* r, const double* p, const double* kicks,
                                    int32_t n, ChannelDesc* descs, int32_t count, hipStream_t s);
hipError_t launch_channel_snapshot(const ChannelDesc* descs, int32_t count, int32_t n,
                                   double* states, int32_t per, int32_t slot, hipStream_t s);
size_t channel_scratch_bytes(int nmax, int kmax);
hipError_t launch_channel(const ChannelLaunch& b, hipStream_t s);
hipError_t launch_channel_debug_forces(const ChannelLaunch& b, double* out, hipStream_t s);
hipError_t launch_channel_spawn(const double* states, int32_t n, int32_t n_wall, double lx,
                                const double* latx0, ChannelDesc* descs, int32_t count,
                                hipStream_t s);
hipError_t launch_channel_accumulate(const ChannelAccum& a, hipStream_t s);
hipError_t launch_channel_response(const ChannelResponse& r, hipStream_t s);

// device memory through the allocator shared with the bulk runtime
void* rt_alloc(size_t bytes, hipStream_t s);
void rt_free(void* p);

}  // namespace ttcf
