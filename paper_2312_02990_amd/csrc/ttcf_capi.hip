// ttcf_capi.hip -- host runtime behind the C ABI of include/ttcf.h.
//
// Owns the mothers, the daughter descriptors and the per-start-state accumulators of one
// context; every computing call enqueues gfx950 kernels from ttcf_kernels.hip on the
// context's stream. There is no host fallback for any computation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ttcf.h"
#include "ttcf_internal.h"

using namespace ttcf;

namespace {

ttcf_alloc_fn g_alloc = nullptr;
ttcf_free_fn g_free = nullptr;
void* g_user = nullptr;
int g_live_contexts = 0;

void* dev_alloc(size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 8;
    if (g_alloc) return g_alloc((uint64_t)bytes, (void*)s, g_user);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void dev_free(void* p) {
    if (!p) return;
    if (g_free)
        g_free(p, g_user);
    else
        (void)hipFree(p);
}

}  // namespace

namespace ttcf {
void* rt_alloc(size_t bytes, hipStream_t s) { return dev_alloc(bytes, s); }
void rt_free(void* p) { dev_free(p); }
}  // namespace ttcf

namespace {

// Device buffers of one call, freed on every return path (stream-ordered like dev_alloc).
struct Scratch {
    hipStream_t s;
    std::vector<void*> held;
    explicit Scratch(hipStream_t st) : s(st) {}
    Scratch(const Scratch&) = delete;
    Scratch& operator=(const Scratch&) = delete;
    template <typename T>
    T* get(size_t count) {
        void* p = dev_alloc(sizeof(T) * count + 64, s);
        if (p) held.push_back(p);
        return (T*)p;
    }
    ~Scratch() {
        for (void* p : held) dev_free(p);
    }
};

struct Mother {
    ttcf_system sys{};
    SysDev dev{};
    int threads = 0, apt = 0;
    double* state = nullptr;     // 6n
    double* zeta = nullptr;      // 1
    int64_t steps = 0;
    double* states = nullptr;    // n_states * 6n
    int32_t n_states = 0, states_cap = 0;
    double* series = nullptr;    // recorded V*P_xy
    int64_t series_cap = 0, series_count = 0;
};

// Stored start states: states_cap blocks of 6n doubles (r, p), then states_cap doubles with
// the thermostat variable of each state.
inline double* zetas_of(const Mother& m) {
    return m.states ? m.states + 6 * (size_t)m.dev.n * (size_t)m.states_cap : nullptr;
}

inline size_t state_buffer_bytes(int n, int count) {
    return sizeof(double) * (6 * (size_t)n + 1) * (size_t)count;
}

struct Batch {
    int32_t mother = -1;
    int32_t n_daughters = 0;
    int32_t n_steps = 0;
    int64_t first_id = 0;
    double* states = nullptr;    // n_daughters * 6n
    double* series = nullptr;    // n_daughters * (n_steps + 1)
    double* hseries = nullptr;   // learned control variate, same layout (allocated on demand)
    double* xseries = nullptr;   // extra observables: n_daughters * (n_steps + 1) * kObsCols
    void* scratch = nullptr;     // spawn index arrays
    int32_t remaining = 0;       // daughters not yet accumulated
};

struct StepShape {              // knobs of the daughter step kernel (0: automatic)
    int32_t variant = 0;        // 1 cell form, 2 pair-list form (3: the same as 2)
    int32_t threads = 0;
    int32_t kmax = 0;           // pair capacity per atom (0: auto_pair_cap)
    double skin = 0.0;          // list skin (<= 0: auto_skin)
};

struct TunedShape {             // one autotuner result
    std::string arch;           // device architecture name
    int32_t n = 0;              // atoms
    int32_t rho_key = 0;        // round(1000 n / V)
    int32_t rc_key = 0;         // round(10000 r_cut)
    int32_t precision = 0;
    StepShape shape;
    double ms_per_step = 0.0;   // probe batch, per step
};

struct Live {                   // host view of one live daughter
    int64_t id;
    int32_t batch;
    int32_t index;              // within its batch
    int32_t group;
    int32_t state;              // index of its start state in the mother's stored set
    int32_t cv_role = 0;        // learned control variate: 0 none, 1 estimate, 2 calibration
};

}  // namespace

struct ttcf_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    int num_cu = 0;
    size_t max_lds = 0;
    std::string err;
    std::vector<Mother> mothers;
    std::vector<Batch> batches;
    // live daughters: host mirror and device copy of their descriptors
    std::vector<DaughterDesc> descs;
    std::vector<Live> live;
    DaughterDesc* d_descs = nullptr;
    size_t d_descs_cap = 0;
    bool device_newer = false;  // kernels have advanced the device descriptors
    int32_t* d_order = nullptr;
    size_t d_order_cap = 0;
    int32_t* d_queue = nullptr;
    int64_t next_id = 0;
    int32_t next_group = 0;
    // accumulated start-state groups
    double* acc_d = nullptr;
    double* acc_i = nullptr;
    int64_t acc_rows = 0, acc_cap = 0;
    int32_t acc_stride = 0;
    std::vector<double> row_gamma, row_coef, row_dt;
    std::vector<int32_t> row_nt, row_health, row_maps;  // row_maps: daughters in the group
    double* d_row_gamma = nullptr;
    double* d_row_coef = nullptr;
    int32_t* d_row_health = nullptr;
    // mother launch blocks (device array)
    MotherLaunch* d_mlaunch = nullptr;
    int32_t mlaunch_cap = 0;
    // accumulated control-variate series (same rows as acc_d)
    double* acc_h = nullptr;
    std::vector<int32_t> row_cv;
    // extra observables: recorded by daughters spawned while record_obs is set; accumulated
    // rows of kObsCols columns of acc_stride values (allocated with the first such spawn)
    bool record_obs = false;
    // some spawned daughters record extra columns on their own (mixed flow: its components)
    bool own_x = false;
    double* acc_xd = nullptr;
    double* acc_xi = nullptr;
    std::vector<char> row_x;
    // external field of each accumulated row (kFieldShear or kFieldColour)
    std::vector<int32_t> row_field;
    // pair-list form: the pair lists of the persistent workgroups (global scratch)
    uint32_t* nl_scratch = nullptr;
    size_t nl_scratch_bytes = 0;
    // learned control variate
    int32_t cv_out = 0;          // outputs (time points t_1..t_nout)
    int64_t cv_nparam = 0;
    float* cv_p = nullptr;       // parameters, gradients, Adam moments (4 x nparam)
    float* cv_g = nullptr;
    float* cv_m = nullptr;
    float* cv_v = nullptr;
    int64_t cv_adam_steps = 0;
    float* cv_x = nullptr;       // training features (raw)
    float* cv_t = nullptr;       // training targets (raw)
    int64_t cv_rows = 0, cv_cap = 0;
    float* cv_stats = nullptr;   // x mean, x 1/std (kCvIn each), y mean, y 1/std (cv_out each)
    bool cv_stats_ready = false;
    double* cv_mu = nullptr;     // mean term: sum, comp, sumsq, compsq (4 x (cv_out + 1))
    int64_t cv_mu_count = 0;
    double cv_mu_dt = 0.0;
    double cv_mu_gamma = 0.0;
    std::vector<double> cv_beta;  // calibrated control-variate coefficient per time point
    double cv_beta_gamma = 0.0;
    // shape of the daughter step kernel: set explicitly, or looked up per system among the
    // tuned shapes (when none is set), else the library's defaults
    StepShape shape;
    bool shape_explicit = false;
    std::vector<TunedShape> tuned;
    std::string arch;
    // captured batch cycles (they pin the accumulator arrays while they exist)
    std::vector<ttcf_graph*> graphs;
    bool graph_rows_dirty = false;  // graphs have written row health since the last download
    int32_t last_variant = -1;
    // timing of the step kernel
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending_events;
    double step_ms = 0.0;
    int64_t step_launches = 0;
};

namespace {

int32_t fail(ttcf_ctx* c, int32_t code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

#define HIPCHECK(ctx, expr)                                                                   \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail((ctx), TTCF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Separation below which a pair's force exceeds kPairForceGuard (bisection on the repulsive
// branch of 24 (2 r^-13 - c r^-7), which falls monotonically up to its zero (2/c)^(1/6)).
double guard_radius(const SysDev& d) {
    auto force = [&](double r) {
        const double s = 1.0 / (r * r), s3 = s * s * s;
        return 24.0 * s3 * (2.0 * s3 - d.c_attr) / r;
    };
    double lo = 0.01, hi = d.c_attr > 0.0 ? std::pow(2.0 / d.c_attr, 1.0 / 6.0) : d.rc;
    hi = std::min(hi, d.rc);
    if (force(hi) >= kPairForceGuard) return hi;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        (force(mid) > kPairForceGuard ? lo : hi) = mid;
    }
    return lo;
}

int32_t build_sysdev(const ttcf_system* s, SysDev* d, std::string* why) {
    if (s->n_atoms < 2 || s->n_atoms > kMaxAtoms) {
        *why = "n_atoms must be in [2, 65535]";
        return TTCF_EINVAL;
    }
    if (!(s->r_cut > 0.0) || !(s->dt > 0.0) || !(s->temperature > 0.0)) {
        *why = "r_cut, dt and temperature must be positive";
        return TTCF_EINVAL;
    }
    d->n = s->n_atoms;
    for (int a = 0; a < 3; ++a) {
        if (!(s->box[a] > 0.0)) {
            *why = "box edges must be positive";
            return TTCF_EINVAL;
        }
        d->nc[a] = (int32_t)std::floor(s->box[a] / s->r_cut);
        d->box[a] = s->box[a];
        d->w[a] = s->box[a] / (double)d->nc[a];
        d->inv_w[a] = (double)d->nc[a] / s->box[a];
    }
    if (d->nc[0] < 4 || d->nc[1] < 3 || d->nc[2] < 3 || d->nc[0] > kMaxCells1D ||
        d->nc[1] > kMaxCells1D || d->nc[2] > kMaxCells1D) {
        *why = "box too small for the cell grid (need floor(Lx/rc) >= 4, floor(Ly/rc), "
               "floor(Lz/rc) >= 3)";
        return TTCF_EINVAL;
    }
    d->rc = s->r_cut;
    d->rc2 = s->r_cut * s->r_cut;
    d->c_attr = s->c_attr;
    // NaN: the shift that makes phi vanish at the cutoff (Example 1: continuity at r_c)
    if (std::isnan(s->u_shift)) {
        const double s6 = 1.0 / std::pow(s->r_cut, 6.0);
        d->u_shift = -4.0 * (s6 * s6 - s->c_attr * s6);
    } else {
        d->u_shift = s->u_shift;
    }
    d->dt = s->dt;
    d->volume = s->box[0] * s->box[1] * s->box[2];
    for (int a = 0; a < 3; ++a) {
        d->fix_scale[a] = 4294967296.0 / s->box[a];
        d->fix_unit[a] = (float)(s->box[a] / 4294967296.0);
    }
    d->rc2_f = (float)d->rc2;
    const double rg = guard_radius(*d);  // depends on the potential only
    d->rg2_f = (float)(rg * rg);
    return TTCF_OK;
}

// List-build grid of the pair-list form for a given skin; false if the box is too small for
// a 27-cell stencil of that reach.
// Automatic skin: the list grid of a 0.2 sigma skin, with the skin widened to fill its cells
// (cell width minus the cutoff, in the narrowest direction). Fewer rebuilds for the same
// candidate count per rebuild. (At N = 2048, rho = 0.8442: 10 cells a side, skin 0.22.)
double auto_skin(const SysDev& d) {
    const double base = d.rc + 0.2;
    double w = d.box[0];
    for (int a = 0; a < 3; ++a) {
        const double n = std::floor(d.box[a] / base);
        if (n >= 1.0) w = std::min(w, d.box[a] / n);
    }
    return std::max(0.2, w * (1.0 - 1e-9) - d.rc);
}

bool set_list_grid(SysDev* d, double skin) {
    if (!(skin > 0.0)) skin = auto_skin(*d);
    const double reach = d->rc + skin;
    d->skin = skin;
    for (int a = 0; a < 3; ++a) {
        d->lc[a] = (int32_t)std::floor(d->box[a] / reach);
        d->lw[a] = d->box[a] / (double)d->lc[a];
        d->l_inv_w[a] = (double)d->lc[a] / d->box[a];
    }
    d->rl2_f = (float)(reach * reach);
    return d->lc[0] >= 4 && d->lc[1] >= 3 && d->lc[2] >= 3 && d->lc[0] <= kMaxCells1D &&
           d->lc[1] <= kMaxCells1D && d->lc[2] <= kMaxCells1D;
}

// Default pair capacity per atom of the pair-list form: half the ideal-gas count within the
// list radius, with half again as margin (a wave's segment covers 256 atoms, so its total
// count varies little), plus two.
int32_t auto_pair_cap(const SysDev& d) {
    const double reach = d.rc + d.skin;
    const double half = 2.0943951023931953 * reach * reach * reach * (d.n / d.volume);
    return std::min<int32_t>(kPairMaxCap, (int32_t)std::ceil(1.5 * half + 2.0));
}

int32_t check_shape(ttcf_ctx* c, const ttcf_system* s, const SysDev& d, int* threads, int* apt) {
    const int t = pick_threads(d.n, s->block_threads);
    if (t % 64 != 0 || t < 64 || t > kMaxThreads)
        return fail(c, TTCF_EINVAL, "block_threads must be a multiple of 64 in [64, 1024]");
    const int a = pick_apt(d.n, t);
    if (a < 0) return fail(c, TTCF_EINVAL, "too many atoms for the chosen block size (max 4/thread)");
    *threads = t;
    *apt = a;
    return TTCF_OK;
}

size_t lds_for(const SysDev& d, int precision) {
    return lds_bytes_for(d.n, d.nc[0] * d.nc[1] * d.nc[2], 0, precision);
}

// Pull the device descriptors back when kernels have advanced them.
int32_t sync_descs(ttcf_ctx* c) {
    if (!c->device_newer || c->descs.empty()) return TTCF_OK;
    HIPCHECK(c, hipMemcpyAsync(c->descs.data(), c->d_descs, sizeof(DaughterDesc) * c->descs.size(),
                               hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    c->device_newer = false;
    return TTCF_OK;
}

int32_t push_descs(ttcf_ctx* c) {
    if (c->descs.empty()) return TTCF_OK;
    if (c->d_descs_cap < c->descs.size()) {
        dev_free(c->d_descs);
        size_t cap = std::max<size_t>(c->descs.size(), 2 * c->d_descs_cap);
        c->d_descs = (DaughterDesc*)dev_alloc(sizeof(DaughterDesc) * cap, c->stream);
        if (!c->d_descs) return fail(c, TTCF_ENOMEM, "descriptor allocation failed");
        c->d_descs_cap = cap;
    }
    HIPCHECK(c, hipMemcpyAsync(c->d_descs, c->descs.data(), sizeof(DaughterDesc) * c->descs.size(),
                               hipMemcpyHostToDevice, c->stream));
    // pageable source: complete the copy before the host vector can change
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return TTCF_OK;
}

int32_t upload_mother_launches(ttcf_ctx* c, const MotherLaunch* ls, int32_t count) {
    if (c->mlaunch_cap < count) {
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        dev_free(c->d_mlaunch);
        c->d_mlaunch = (MotherLaunch*)dev_alloc(sizeof(MotherLaunch) * count, c->stream);
        if (!c->d_mlaunch) return fail(c, TTCF_ENOMEM, "mother launch allocation failed");
        c->mlaunch_cap = count;
    }
    HIPCHECK(c, hipMemcpyAsync(c->d_mlaunch, ls, sizeof(MotherLaunch) * count, hipMemcpyHostToDevice,
                               c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return TTCF_OK;
}

int32_t run_mother(ttcf_ctx* c, Mother& m, double temperature, int64_t n_chunks,
                   int64_t steps_per_chunk, double* snapshots, double* snap_zeta = nullptr) {
    if (steps_per_chunk <= 0 && n_chunks <= 0) return TTCF_OK;
    MotherLaunch L{};
    L.sys = m.dev;
    L.state = m.state;
    L.zeta = m.zeta;
    L.temperature = temperature;
    const double nf = 3.0 * m.dev.n - 3.0;
    L.nf = nf;
    L.q = nf * temperature * m.sys.nh_tau * m.sys.nh_tau;
    L.n_chunks = n_chunks;
    L.steps_per_chunk = steps_per_chunk;
    L.snapshots = snapshots;
    L.snap_zeta = snap_zeta;
    const int64_t total = (n_chunks > 0 ? n_chunks : 1) * steps_per_chunk;
    L.series = nullptr;
    if (m.series && m.series_count + total <= m.series_cap) {
        L.series = m.series + m.series_count;
        m.series_count += total;
    }
    L.threads = m.threads;
    L.apt = m.apt;
    L.precision = m.sys.precision;
    L.lds_bytes = lds_for(m.dev, m.sys.precision);
    int32_t rc = upload_mother_launches(c, &L, 1);
    if (rc != TTCF_OK) return rc;
    HIPCHECK(c, launch_mothers(c->d_mlaunch, 1, L, c->stream));
    m.steps += total;
    return TTCF_OK;
}

// The extra-column accumulator at the current capacity and stride, if the accumulator exists
// without it (a later growth copies it along).
int32_t ensure_acc_x(ttcf_ctx* c) {
    if (c->acc_xd || c->acc_cap == 0) return TTCF_OK;
    double* xd = (double*)dev_alloc(sizeof(double) * (size_t)c->acc_cap * kObsCols * c->acc_stride,
                                    c->stream);
    double* xi = (double*)dev_alloc(sizeof(double) * (size_t)c->acc_cap * kObsCols * c->acc_stride,
                                    c->stream);
    if (!xd || !xi) {
        dev_free(xd);
        dev_free(xi);
        return fail(c, TTCF_ENOMEM, "accumulator allocation failed");
    }
    c->acc_xd = xd;
    c->acc_xi = xi;
    return TTCF_OK;
}

int32_t grow_acc(ttcf_ctx* c, int64_t rows_needed, int32_t n_t) {
    const int32_t stride = std::max(c->acc_stride, n_t);
    // groups with extra columns need their accumulator too, even where the rows would fit
    if ((c->record_obs || c->own_x) && !c->acc_xd) {
        const int32_t rc = ensure_acc_x(c);
        if (rc != TTCF_OK) return rc;
    }
    if (rows_needed <= c->acc_cap && stride == c->acc_stride) return TTCF_OK;
    if (!c->graphs.empty())
        return fail(c, TTCF_ESTATE, "accumulator capacity is pinned by a captured graph: destroy "
                                    "it before accumulating beyond the rows reserved for it");
    const int64_t cap = std::max<int64_t>(rows_needed, 2 * c->acc_cap);
    double* nd = (double*)dev_alloc(sizeof(double) * (size_t)cap * stride, c->stream);
    double* ni = (double*)dev_alloc(sizeof(double) * (size_t)cap * stride, c->stream);
    double* nh = (double*)dev_alloc(sizeof(double) * (size_t)cap * stride, c->stream);
    double* ng = (double*)dev_alloc(sizeof(double) * (size_t)cap, c->stream);
    double* nc = (double*)dev_alloc(sizeof(double) * (size_t)cap, c->stream);
    int32_t* nhl = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)cap, c->stream);
    if (!nd || !ni || !nh || !ng || !nc || !nhl)
        return fail(c, TTCF_ENOMEM, "accumulator allocation failed");
    double* nxd = nullptr;
    double* nxi = nullptr;
    const bool with_x = c->record_obs || c->own_x || c->acc_xd;
    if (with_x) {
        nxd = (double*)dev_alloc(sizeof(double) * (size_t)cap * kObsCols * stride, c->stream);
        nxi = (double*)dev_alloc(sizeof(double) * (size_t)cap * kObsCols * stride, c->stream);
        if (!nxd || !nxi) return fail(c, TTCF_ENOMEM, "accumulator allocation failed");
    }
    if (c->acc_rows > 0) {
        HIPCHECK(c, hipMemcpy2DAsync(nd, sizeof(double) * stride, c->acc_d,
                                     sizeof(double) * c->acc_stride, sizeof(double) * c->acc_stride,
                                     (size_t)c->acc_rows, hipMemcpyDeviceToDevice, c->stream));
        HIPCHECK(c, hipMemcpy2DAsync(ni, sizeof(double) * stride, c->acc_i,
                                     sizeof(double) * c->acc_stride, sizeof(double) * c->acc_stride,
                                     (size_t)c->acc_rows, hipMemcpyDeviceToDevice, c->stream));
        HIPCHECK(c, hipMemcpy2DAsync(nh, sizeof(double) * stride, c->acc_h,
                                     sizeof(double) * c->acc_stride, sizeof(double) * c->acc_stride,
                                     (size_t)c->acc_rows, hipMemcpyDeviceToDevice, c->stream));
        if (with_x && c->acc_xd) {
            // a row is kObsCols columns of the stride: copy column by column
            HIPCHECK(c, hipMemcpy2DAsync(nxd, sizeof(double) * stride, c->acc_xd,
                                         sizeof(double) * c->acc_stride,
                                         sizeof(double) * c->acc_stride,
                                         (size_t)c->acc_rows * kObsCols, hipMemcpyDeviceToDevice,
                                         c->stream));
            HIPCHECK(c, hipMemcpy2DAsync(nxi, sizeof(double) * stride, c->acc_xi,
                                         sizeof(double) * c->acc_stride,
                                         sizeof(double) * c->acc_stride,
                                         (size_t)c->acc_rows * kObsCols, hipMemcpyDeviceToDevice,
                                         c->stream));
        }
        HIPCHECK(c, hipStreamSynchronize(c->stream));
    }
    if (with_x) {
        dev_free(c->acc_xd);
        dev_free(c->acc_xi);
        c->acc_xd = nxd;
        c->acc_xi = nxi;
    }
    dev_free(c->acc_d);
    dev_free(c->acc_i);
    dev_free(c->acc_h);
    dev_free(c->d_row_gamma);
    dev_free(c->d_row_coef);
    dev_free(c->d_row_health);
    c->acc_d = nd;
    c->acc_i = ni;
    c->acc_h = nh;
    c->d_row_gamma = ng;
    c->d_row_coef = nc;
    c->d_row_health = nhl;
    c->acc_cap = cap;
    c->acc_stride = stride;
    return TTCF_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------

extern "C" {

int32_t ttcf_set_allocator(ttcf_alloc_fn alloc, ttcf_free_fn release, void* user) {
    if (g_live_contexts > 0) return TTCF_ESTATE;
    if ((alloc == nullptr) != (release == nullptr)) return TTCF_EINVAL;
    g_alloc = alloc;
    g_free = release;
    g_user = user;
    return TTCF_OK;
}

const char* ttcf_strerror(int32_t code) {
    switch (code) {
        case TTCF_OK: return "ok";
        case TTCF_EINVAL: return "invalid argument";
        case TTCF_ENOMEM: return "out of memory";
        case TTCF_EDEVICE: return "device error";
        case TTCF_ESTATE: return "call out of order";
        case TTCF_EUNSTABLE: return "every daughter group failed its health check";
        case TTCF_ESCRATCH:
            return "the input needs more than the static scratch of the allocation-free call";
    }
    return "unknown error";
}

const char* ttcf_last_error(const ttcf_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

void ttcf_destroy(ttcf_ctx* c) {
    if (!c) return;
    while (!c->graphs.empty()) ttcf_graph_destroy(c->graphs.back());
    (void)hipStreamSynchronize(c->stream);
    for (auto& ev : c->pending_events) {
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    for (auto& m : c->mothers) {
        dev_free(m.state);
        dev_free(m.zeta);
        dev_free(m.states);
        dev_free(m.series);
    }
    for (auto& b : c->batches) {
        dev_free(b.states);
        dev_free(b.series);
        dev_free(b.scratch);
        dev_free(b.hseries);
        dev_free(b.xseries);
    }
    dev_free(c->acc_xd);
    dev_free(c->acc_xi);
    dev_free(c->nl_scratch);
    dev_free(c->d_descs);
    dev_free(c->d_order);
    dev_free(c->d_queue);
    dev_free(c->acc_d);
    dev_free(c->acc_i);
    dev_free(c->d_row_gamma);
    dev_free(c->d_row_coef);
    dev_free(c->d_row_health);
    dev_free(c->d_mlaunch);
    dev_free(c->acc_h);
    dev_free(c->cv_p);
    dev_free(c->cv_x);
    dev_free(c->cv_t);
    dev_free(c->cv_stats);
    dev_free(c->cv_mu);
    --g_live_contexts;
    delete c;
}

int32_t ttcf_init_mother(ttcf_ctx** pctx, const ttcf_system* sys, const double* r0,
                         const double* p0, int64_t n_melt, double t_melt, int64_t n_equil,
                         void* stream, int32_t* out_mother) {
    if (!pctx || !sys || !r0 || !p0 || n_melt < 0 || n_equil < 0) return TTCF_EINVAL;
    if (sys->precision != TTCF_PREC_FP64 && sys->precision != TTCF_PREC_FP32_FORCES)
        return TTCF_EINVAL;
    if (n_melt > 0 && !(t_melt > 0.0)) return TTCF_EINVAL;
    ttcf_ctx* c = *pctx;
    bool created = false;
    if (!c) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return TTCF_EDEVICE;
        c = new ttcf_ctx();
        created = true;
        ++g_live_contexts;
        c->stream = (hipStream_t)stream;
        if (hipGetDevice(&c->device) != hipSuccess) {
            ttcf_destroy(c);
            return TTCF_EDEVICE;
        }
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) {
            ttcf_destroy(c);
            return TTCF_EDEVICE;
        }
        c->num_cu = prop.multiProcessorCount;
        c->max_lds = prop.sharedMemPerBlock;
        c->arch = prop.gcnArchName;
        c->d_queue = (int32_t*)dev_alloc(sizeof(int32_t) * 4, c->stream);
        if (!c->d_queue) {
            ttcf_destroy(c);
            return TTCF_ENOMEM;
        }
    }
    if (sys->daughter_thermostat != TTCF_DAUGHTER_GIK && sys->daughter_thermostat != TTCF_DAUGHTER_NH) {
        if (created) ttcf_destroy(c);
        else c->err = "daughter_thermostat must be TTCF_DAUGHTER_GIK or TTCF_DAUGHTER_NH";
        return TTCF_EINVAL;
    }
    Mother m;
    m.sys = *sys;
    std::string why;
    int32_t rc = build_sysdev(sys, &m.dev, &why);
    if (rc == TTCF_OK) rc = check_shape(c, sys, m.dev, &m.threads, &m.apt);
    else c->err = why;
    if (rc == TTCF_OK && lds_for(m.dev, sys->precision) > c->max_lds)
        rc = fail(c, TTCF_EINVAL, "system too large for one workgroup's LDS");
    if (rc != TTCF_OK) {
        if (created) ttcf_destroy(c);
        return rc;
    }
    const int n = sys->n_atoms;
    for (int k = 0; k < 3 * n; ++k) {
        const int a = k / n;
        if (!(r0[k] >= 0.0 && r0[k] < sys->box[a]) || !std::isfinite(p0[k])) {
            if (created) ttcf_destroy(c);
            else c->err = "initial positions must lie in [0, L) and momenta be finite";
            return TTCF_EINVAL;
        }
    }
    m.state = (double*)dev_alloc(sizeof(double) * 6 * n, c->stream);
    m.zeta = (double*)dev_alloc(sizeof(double), c->stream);
    if (!m.state || !m.zeta) {
        dev_free(m.state);
        dev_free(m.zeta);
        if (created) ttcf_destroy(c);
        return TTCF_ENOMEM;
    }
    const double zero = 0.0;
    HIPCHECK(c, hipMemcpyAsync(m.state, r0, sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipMemcpyAsync(m.state + 3 * n, p0, sizeof(double) * 3 * n, hipMemcpyHostToDevice,
                               c->stream));
    HIPCHECK(c, hipMemcpyAsync(m.zeta, &zero, sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    c->mothers.push_back(m);
    Mother& mm = c->mothers.back();
    rc = run_mother(c, mm, t_melt, 0, n_melt, nullptr);
    if (rc == TTCF_OK) rc = run_mother(c, mm, sys->temperature, 0, n_equil, nullptr);
    if (rc != TTCF_OK) return rc;
    *pctx = c;
    if (out_mother) *out_mother = (int32_t)c->mothers.size() - 1;
    return TTCF_OK;
}

int32_t ttcf_record_mother(ttcf_ctx* c, int32_t mother, int64_t capacity) {
    if (!c || mother < 0 || mother >= (int32_t)c->mothers.size() || capacity < 0) return TTCF_EINVAL;
    Mother& m = c->mothers[mother];
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    dev_free(m.series);
    m.series = capacity > 0 ? (double*)dev_alloc(sizeof(double) * capacity, c->stream) : nullptr;
    if (capacity > 0 && !m.series) return fail(c, TTCF_ENOMEM, "series allocation failed");
    m.series_cap = capacity;
    m.series_count = 0;
    return TTCF_OK;
}

int32_t ttcf_export_mother_series(ttcf_ctx* c, int32_t mother, int64_t n, double* vpxy,
                                  int64_t* out_count) {
    if (!c || mother < 0 || mother >= (int32_t)c->mothers.size() || n < 0) return TTCF_EINVAL;
    Mother& m = c->mothers[mother];
    const int64_t cnt = std::min(n, m.series_count);
    if (cnt > 0 && vpxy)
        HIPCHECK(c, hipMemcpyAsync(vpxy, m.series, sizeof(double) * cnt, hipMemcpyDeviceToHost,
                                   c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    if (out_count) *out_count = m.series_count;
    return TTCF_OK;
}

namespace {
// Autocorrelation of a device series; results to host.
int32_t acf_device(ttcf_ctx* c, const double* d_x, int64_t n, int32_t max_lag, double threshold,
                   double* acf, int32_t* first_below, double* tau_int) {
    if (n < 2 || max_lag < 1 || max_lag > n || !acf)
        return fail(c, TTCF_EINVAL, "acf needs 2 <= n, 1 <= max_lag <= n and an output array");
    Scratch sc(c->stream);
    double* d = sc.get<double>((size_t)max_lag + 4);
    if (!d) return fail(c, TTCF_ENOMEM, "acf scratch allocation failed");
    double* d_acf = d + 4;
    int32_t* d_fb = (int32_t*)(d + 1);
    HIPCHECK(c, launch_acf(d_x, n, max_lag, threshold, d, d_acf, d_fb, d + 2, c->stream));
    double tail[2];
    int32_t fb = -1;
    HIPCHECK(c, hipMemcpyAsync(acf, d_acf, sizeof(double) * max_lag, hipMemcpyDeviceToHost,
                               c->stream));
    HIPCHECK(c, hipMemcpyAsync(&fb, d_fb, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipMemcpyAsync(tail, d + 2, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    if (first_below) *first_below = fb;
    if (tau_int) *tau_int = tail[0];
    return TTCF_OK;
}
}  // namespace

int32_t ttcf_acf(ttcf_ctx* c, const double* series, int64_t n, int32_t max_lag, double threshold,
                 double* acf, int32_t* first_below, double* tau_int) {
    if (!c || !series || n < 2) return TTCF_EINVAL;
    Scratch sc(c->stream);
    double* d_x = sc.get<double>((size_t)n);
    if (!d_x) return fail(c, TTCF_ENOMEM, "acf series allocation failed");
    HIPCHECK(c, hipMemcpyAsync(d_x, series, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    return acf_device(c, d_x, n, max_lag, threshold, acf, first_below, tau_int);
}

int32_t ttcf_mother_acf(ttcf_ctx* c, int32_t mother, int32_t max_lag, double threshold,
                        double* acf, int32_t* first_below, double* tau_int) {
    if (!c || mother < 0 || mother >= (int32_t)c->mothers.size()) return TTCF_EINVAL;
    Mother& m = c->mothers[mother];
    if (!m.series || m.series_count < 2)
        return fail(c, TTCF_ESTATE, "no recorded mother series (ttcf_record_mother, then run)");
    return acf_device(c, m.series, m.series_count, max_lag, threshold, acf, first_below, tau_int);
}

int32_t ttcf_import_states(ttcf_ctx* c, int32_t mother, int32_t n_states, const double* r,
                           const double* p) {
    if (!c || mother < 0 || mother >= (int32_t)c->mothers.size() || n_states <= 0 || !r || !p)
        return TTCF_EINVAL;
    Mother& m = c->mothers[mother];
    const size_t n = (size_t)m.dev.n;
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    if (m.states_cap < n_states) {
        dev_free(m.states);
        m.states = (double*)dev_alloc(state_buffer_bytes((int)n, n_states), c->stream);
        if (!m.states) return fail(c, TTCF_ENOMEM, "state buffer allocation failed");
        m.states_cap = n_states;
    }
    HIPCHECK(c, launch_fill_f64(zetas_of(m), 0.0, n_states, c->stream));
    for (int32_t s = 0; s < n_states; ++s) {
        HIPCHECK(c, hipMemcpyAsync(m.states + 6 * n * s, r + 3 * n * s, sizeof(double) * 3 * n,
                                   hipMemcpyHostToDevice, c->stream));
        HIPCHECK(c, hipMemcpyAsync(m.states + 6 * n * s + 3 * n, p + 3 * n * s,
                                   sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream));
    }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    m.n_states = n_states;
    return TTCF_OK;
}

int32_t ttcf_export_states(ttcf_ctx* c, int32_t mother, int32_t n_states, double* r, double* p) {
    if (!c || mother < 0 || mother >= (int32_t)c->mothers.size() || n_states <= 0) return TTCF_EINVAL;
    Mother& m = c->mothers[mother];
    if (n_states > m.n_states) return fail(c, TTCF_EINVAL, "fewer stored states than requested");
    const size_t n = (size_t)m.dev.n;
    for (int32_t s = 0; s < n_states; ++s) {
        if (r)
            HIPCHECK(c, hipMemcpyAsync(r + 3 * n * s, m.states + 6 * n * s, sizeof(double) * 3 * n,
                                       hipMemcpyDeviceToHost, c->stream));
        if (p)
            HIPCHECK(c, hipMemcpyAsync(p + 3 * n * s, m.states + 6 * n * s + 3 * n,
                                       sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return TTCF_OK;
}

int32_t ttcf_import_states_zeta(ttcf_ctx* c, int32_t mother, int32_t n_states,
                                const double* zeta) {
    if (!c || mother < 0 || mother >= (int32_t)c->mothers.size() || n_states <= 0 || !zeta)
        return TTCF_EINVAL;
    Mother& m = c->mothers[mother];
    if (n_states > m.n_states) return fail(c, TTCF_EINVAL, "fewer stored states than given");
    HIPCHECK(c, hipMemcpyAsync(zetas_of(m), zeta, sizeof(double) * n_states,
                               hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return TTCF_OK;
}

int32_t ttcf_export_states_zeta(ttcf_ctx* c, int32_t mother, int32_t n_states, double* zeta) {
    if (!c || mother < 0 || mother >= (int32_t)c->mothers.size() || n_states <= 0 || !zeta)
        return TTCF_EINVAL;
    Mother& m = c->mothers[mother];
    if (n_states > m.n_states) return fail(c, TTCF_EINVAL, "fewer stored states than requested");
    HIPCHECK(c, hipMemcpyAsync(zeta, zetas_of(m), sizeof(double) * n_states,
                               hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return TTCF_OK;
}

int32_t ttcf_export_mother(ttcf_ctx* c, int32_t mother, double* r, double* p, double* zeta,
                           int64_t* steps) {
    if (!c || mother < 0 || mother >= (int32_t)c->mothers.size()) return TTCF_EINVAL;
    Mother& m = c->mothers[mother];
    const size_t n = (size_t)m.dev.n;
    if (r) HIPCHECK(c, hipMemcpyAsync(r, m.state, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->stream));
    if (p)
        HIPCHECK(c, hipMemcpyAsync(p, m.state + 3 * n, sizeof(double) * 3 * n, hipMemcpyDeviceToHost,
                                   c->stream));
    if (zeta) HIPCHECK(c, hipMemcpyAsync(zeta, m.zeta, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    if (steps) *steps = m.steps;
    return TTCF_OK;
}

int32_t ttcf_sample_states(ttcf_ctx* c, int32_t mother, int32_t n_states, int64_t steps_between) {
    if (!c || mother < 0 || mother >= (int32_t)c->mothers.size() || n_states <= 0 ||
        steps_between <= 0)
        return TTCF_EINVAL;
    Mother& m = c->mothers[mother];
    const size_t n = (size_t)m.dev.n;
    if (m.states_cap < n_states) {
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        dev_free(m.states);
        m.states = (double*)dev_alloc(state_buffer_bytes((int)n, n_states), c->stream);
        if (!m.states) return fail(c, TTCF_ENOMEM, "state buffer allocation failed");
        m.states_cap = n_states;
    }
    int32_t rc = run_mother(c, m, m.sys.temperature, n_states, steps_between, m.states,
                            zetas_of(m));
    if (rc != TTCF_OK) return rc;
    m.n_states = n_states;
    return TTCF_OK;
}

namespace {
int32_t spawn_impl(ttcf_ctx* c, int32_t mother, int32_t n_states, int64_t steps_between,
                   uint32_t mapping_mask, const double* gamma_dot, int32_t n_gamma, int32_t n_steps,
                   bool prefix_ok, int64_t* out_first, int32_t field = kFieldShear,
                   const double* erate = nullptr, const double* srate = nullptr);
}

int32_t ttcf_spawn_daughters(ttcf_ctx* c, int32_t mother, int32_t n_states, int64_t steps_between,
                             uint32_t mapping_mask, const double* gamma_dot, int32_t n_gamma,
                             int32_t n_steps, int64_t* out_first) {
    return spawn_impl(c, mother, n_states, steps_between, mapping_mask, gamma_dot, n_gamma, n_steps,
                      false, out_first);
}

int32_t ttcf_spawn_colour(ttcf_ctx* c, int32_t mother, int32_t n_states, int64_t steps_between,
                          uint32_t mapping_mask, const double* field, int32_t n_field,
                          int32_t n_steps, int64_t* out_first) {
    return spawn_impl(c, mother, n_states, steps_between, mapping_mask, field, n_field, n_steps,
                      false, out_first, kFieldColour);
}

int32_t ttcf_spawn_mixed(ttcf_ctx* c, int32_t mother, int32_t n_states, int64_t steps_between,
                         uint32_t mapping_mask, const double* erate, const double* srate,
                         int32_t n_rate, int32_t n_steps, int64_t* out_first) {
    if (!c) return TTCF_EINVAL;
    if (!erate || !srate || n_rate < 1 || n_rate > (1 << 24))
        return fail(c, TTCF_EINVAL, "bad mixed-flow rates");
    // the field strength |rate| sets Omega's coefficient and the response filter
    std::vector<double> rn(n_rate);
    for (int32_t g = 0; g < n_rate; ++g) {
        rn[g] = std::sqrt(erate[g] * erate[g] + srate[g] * srate[g]);
        if (!std::isfinite(rn[g]) || !(rn[g] > 0.0))
            return fail(c, TTCF_EINVAL, "mixed-flow rates must be finite and not both zero");
    }
    return spawn_impl(c, mother, n_states, steps_between, mapping_mask, rn.data(), n_rate,
                      n_steps, false, out_first, kFieldMixed, erate, srate);
}

int32_t ttcf_spawn_elongational(ttcf_ctx* c, int32_t mother, int32_t n_states,
                                int64_t steps_between, uint32_t mapping_mask, const double* rate,
                                int32_t n_rate, int32_t n_steps, int64_t* out_first) {
    return spawn_impl(c, mother, n_states, steps_between, mapping_mask, rate, n_rate, n_steps,
                      false, out_first, kFieldElong);
}

namespace {
// prefix_ok: with steps_between == 0, the first n_states stored states may be used
int32_t spawn_impl(ttcf_ctx* c, int32_t mother, int32_t n_states, int64_t steps_between,
                   uint32_t mapping_mask, const double* gamma_dot, int32_t n_gamma, int32_t n_steps,
                   bool prefix_ok, int64_t* out_first, int32_t field, const double* erate,
                   const double* srate) {
    if (!c) return TTCF_EINVAL;
    if (mother < 0 || mother >= (int32_t)c->mothers.size() || n_states <= 0 || steps_between < 0 ||
        (mapping_mask & 0xFu) == 0 || (mapping_mask & ~0xFu) != 0 || !gamma_dot ||
        !(n_gamma == 1 || n_gamma == n_states) || n_steps < 1)
        return fail(c, TTCF_EINVAL, "bad spawn arguments");
    for (int32_t g = 0; g < n_gamma; ++g)
        if (!std::isfinite(gamma_dot[g])) return fail(c, TTCF_EINVAL, "shear rates must be finite");
    Mother& m = c->mothers[mother];
    const size_t n = (size_t)m.dev.n;
    if (c->record_obs && m.sys.precision != TTCF_PREC_FP32_FORCES)
        return fail(c, TTCF_EINVAL, "the extra observables are recorded by the list form only "
                                    "(FP32 forces)");
    if (field == kFieldColour) {
        if (c->record_obs)
            return fail(c, TTCF_EINVAL, "colour-field daughters record V J_x only: switch the "
                                        "extra observables off");
        if (m.sys.precision != TTCF_PREC_FP32_FORCES)
            return fail(c, TTCF_EINVAL, "colour-field daughters run in the list form (FP32 forces)");
        if (m.dev.n % 2 != 0)
            return fail(c, TTCF_EINVAL, "the colour field needs an even number of atoms");
    }
    if (field == kFieldMixed) {
        if (c->record_obs)
            return fail(c, TTCF_EINVAL, "mixed-flow daughters record their flux only: switch "
                                        "the extra observables off");
        if (m.dev.n > kPefMaxAtoms)
            return fail(c, TTCF_EINVAL, "mixed-flow daughters hold at most 2048 atoms");
        if (m.dev.box[0] != m.dev.box[1])
            return fail(c, TTCF_EINVAL, "the mixed-flow mappings exchange x and y: the box must "
                                        "have L_x = L_y");
        // the carried cell keeps every perpendicular width at 3 r_c or more, step by step
        for (int32_t g = 0; g < n_gamma; ++g) {
            const double er = erate[g], sr = srate[g], l = m.dev.box[0];
            for (int32_t k = 0; k <= n_steps; ++k) {
                const double t = (double)k * m.dev.dt, x = er * t;
                const double hxx = l * std::exp(x), hyy = l * std::exp(-x);
                const double hxy = l * sr * t * (x == 0.0 ? 1.0 : std::sinh(x) / x);
                const double wx = hxx * hyy / std::sqrt(hxy * hxy + hyy * hyy);
                if (wx < 3.0 * m.dev.rc || hyy < 3.0 * m.dev.rc)
                    return fail(c, TTCF_EINVAL, "the mixed flow would narrow the cell below "
                                                "3 r_c before the daughter ends (lower the rates "
                                                "or the length, or use a larger system)");
            }
        }
    }
    if (field == kFieldElong) {
        if (c->record_obs)
            return fail(c, TTCF_EINVAL, "planar-elongation daughters record V (P_xx - P_yy) "
                                        "only: switch the extra observables off");
        if (m.dev.n > kPefMaxAtoms)
            return fail(c, TTCF_EINVAL, "planar-elongation daughters hold at most 2048 atoms");
        if (m.dev.box[0] != m.dev.box[1])
            return fail(c, TTCF_EINVAL, "planar elongation exchanges x and y: the box must "
                                        "have L_x = L_y");
        // every edge stays at 3 r_c or more over the whole daughter (the cell stencil)
        for (int32_t g = 0; g < n_gamma; ++g) {
            const double shrink = std::exp(-std::fabs(gamma_dot[g]) * (double)n_steps * m.dev.dt);
            if (m.dev.box[0] * shrink < 3.0 * m.dev.rc)
                return fail(c, TTCF_EINVAL, "the elongation would shrink a box edge below 3 r_c "
                                            "before the daughter ends (lower the rate or the "
                                            "length, or use a larger system)");
        }
    }
    if (steps_between > 0) {
        int32_t rc = ttcf_sample_states(c, mother, n_states, steps_between);
        if (rc != TTCF_OK) return rc;
    } else if (m.n_states != n_states && !(prefix_ok && n_states <= m.n_states)) {
        return fail(c, TTCF_EINVAL, "steps_between == 0 needs n_states equal to the stored count");
    }
    int32_t rc = sync_descs(c);
    if (rc != TTCF_OK) return rc;
    std::vector<int32_t> maps;
    for (int q = 0; q < 4; ++q)
        if (mapping_mask & (1u << q)) maps.push_back(q);
    const int32_t nm = (int32_t)maps.size();
    const int32_t nd = n_states * nm;
    Batch b;
    b.mother = mother;
    b.n_daughters = nd;
    b.n_steps = n_steps;
    b.first_id = c->next_id;
    b.remaining = nd;
    b.states = (double*)dev_alloc(sizeof(double) * 6 * n * nd, c->stream);
    b.series = (double*)dev_alloc(sizeof(double) * (size_t)(n_steps + 1) * nd, c->stream);
    const size_t scratch_bytes = sizeof(int32_t) * 2 * nd + sizeof(double*) * nd + 64;
    b.scratch = dev_alloc(scratch_bytes, c->stream);
    // mixed-flow daughters always record their flux components (columns 0 and 1); their
    // accumulator columns exist from here on (a captured graph may pin the other arrays)
    const bool with_x = c->record_obs || field == kFieldMixed;
    if (field == kFieldMixed) {
        c->own_x = true;
        rc = ensure_acc_x(c);
        if (rc != TTCF_OK) return rc;
    }
    if (with_x)
        b.xseries = (double*)dev_alloc(sizeof(double) * (size_t)(n_steps + 1) * kObsCols * nd,
                                       c->stream);
    if (!b.states || !b.series || !b.scratch || (with_x && !b.xseries)) {
        dev_free(b.states);
        dev_free(b.series);
        dev_free(b.scratch);
        dev_free(b.xseries);
        return fail(c, TTCF_ENOMEM, "daughter allocation failed");
    }
    // Nose-Hoover daughters start from their state's thermostat variable
    const bool nh = m.sys.daughter_thermostat == TTCF_DAUGHTER_NH;
    std::vector<double> hz;
    if (nh) {
        hz.resize(n_states);
        HIPCHECK(c, hipMemcpyAsync(hz.data(), zetas_of(m), sizeof(double) * n_states,
                                   hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(c, hipStreamSynchronize(c->stream));
    }
    const double nf = 3.0 * (double)m.dev.n - 3.0;
    std::vector<char> host(scratch_bytes);
    double** dst = (double**)host.data();
    int32_t* state_of = (int32_t*)(host.data() + sizeof(double*) * nd);
    int32_t* map_of = state_of + nd;
    const int32_t bidx = (int32_t)c->batches.size();
    for (int32_t s = 0; s < n_states; ++s) {
        const int32_t group = c->next_group++;
        const double g = gamma_dot[n_gamma == 1 ? 0 : s];
        for (int32_t q = 0; q < nm; ++q) {
            const int32_t d = s * nm + q;
            dst[d] = b.states + 6 * n * d;
            state_of[d] = s;
            map_of[d] = maps[q];
            DaughterDesc ds{};
            ds.state = dst[d];
            ds.series = b.series + (size_t)(n_steps + 1) * d;
            ds.xseries = b.xseries ? b.xseries + (size_t)(n_steps + 1) * kObsCols * d : nullptr;
            ds.sys = m.dev;
            ds.gamma_dot = field == kFieldColour ? 0.0 : g;  // the elongation rate for kFieldElong
            if (field == kFieldMixed) {
                ds.erate = erate[n_gamma == 1 ? 0 : s];
                ds.srate = srate[n_gamma == 1 ? 0 : s];
            }
            ds.field = field;
            ds.fe = field == kFieldColour ? g : 0.0;
            ds.k0 = 0.0;
            ds.k = 0;
            ds.n_steps = n_steps;
            ds.done = 0;
            ds.health = 0;
            ds.group = group;
            ds.map = maps[q];
            ds.block = m.threads;
            if (nh) {
                ds.thermo = 1;
                // mappings 1 and 3 reverse time, except for mixed flow (they reflect x there)
                ds.zeta = ((maps[q] & 1) && field != kFieldMixed) ? -hz[s] : hz[s];
                ds.nh_q = nf * m.sys.temperature * m.sys.nh_tau * m.sys.nh_tau;
                ds.nh_target = nf * m.sys.temperature;
            }
            c->descs.push_back(ds);
            c->live.push_back(Live{c->next_id + d, bidx, d, group, s});
        }
    }
    HIPCHECK(c, hipMemcpyAsync(b.scratch, host.data(), scratch_bytes, hipMemcpyHostToDevice, c->stream));
    {
        const int32_t* d_state_of = (const int32_t*)((char*)b.scratch + sizeof(double*) * nd);
        if (field == kFieldElong || field == kFieldMixed)
            HIPCHECK(c, launch_spawn_pef(m.states, m.dev.n, d_state_of, d_state_of + nd,
                                         (double* const*)b.scratch, nd,
                                         field == kFieldMixed ? 1 : 0, m.dev.box[0], c->stream));
        else
            HIPCHECK(c, launch_spawn(m.states, m.dev.n, n_states, d_state_of, d_state_of + nd,
                                     (double* const*)b.scratch, nd, m.dev.box[0], c->stream));
    }
    // the host copy of the index arrays must outlive the asynchronous copy
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    c->batches.push_back(b);
    c->next_id += nd;
    rc = push_descs(c);
    if (rc != TTCF_OK) return rc;
    if (out_first) *out_first = b.first_id;
    return TTCF_OK;
}

// Launch shape of one group of daughters in one kernel form. threads_req > 0 fixes the
// workgroup size; kmax is the list capacity of the neighbour-list form.
// block_explicit: some member's system fixes its workgroup size (block_threads > 0).
int32_t plan_group(ttcf_ctx* c, const std::vector<const DaughterDesc*>& group, bool block_explicit,
                   int variant, int precision, int32_t n_steps, int threads_req, BatchLaunch* L) {
    int nmax = 0, cmax = 0, lcmax = 0, threads = 0, kmax = 0;
    size_t nl_lds = 0;
    int64_t pair_stride = 0;
    const bool nlf = variant == kVariantNeighbourList;
    for (const DaughterDesc* dp : group) {
        const DaughterDesc& d = *dp;
        kmax = std::max(kmax, d.kmax);
        nmax = std::max(nmax, d.sys.n);
        cmax = std::max(cmax, d.sys.nc[0] * d.sys.nc[1] * d.sys.nc[2]);
        lcmax = std::max(lcmax, d.sys.lc[0] * d.sys.lc[1] * d.sys.lc[2]);
        if (nlf) {
            nl_lds = std::max(nl_lds, lds_bytes_pairs(d.sys.n, d.sys.lc[0] * d.sys.lc[1] * d.sys.lc[2]));
            threads = std::max(threads, pair_job_threads(d.sys.n));
        } else {
            threads = std::max(threads, d.block);
        }
    }
    // the pair-list form: four atoms per thread of each job, the workgroup as large as the
    // largest job needs (the thread count of a job does not depend on the launch)
    if (!nlf && threads_req > 0) threads = threads_req;
    (void)block_explicit;
    const int apt = nlf ? pair_job_apt(nmax) : pick_apt(nmax, threads);
    if (apt < 0) return fail(c, TTCF_EINVAL, "batch needs more than 4 atoms per thread");
    // pair words in LDS when every job's fit beside its layout (four atoms per thread only),
    // else in global scratch
    size_t nl_lds_pl = 0;
    if (nlf)
        for (const DaughterDesc* dp : group) {
            pair_stride = std::max<int64_t>(pair_stride, pair_words(dp->sys.n, dp->kmax, apt));
            nl_lds_pl = std::max(nl_lds_pl, lds_bytes_pairs_lds(dp->sys.n, dp->sys.lc[0] * dp->sys.lc[1] *
                                                                   dp->sys.lc[2], dp->kmax, apt));
        }
    const bool pairs_lds = nlf && apt == pair_small_apt() && nl_lds_pl <= c->max_lds;
    *L = BatchLaunch{};
    L->descs = c->d_descs;
    L->n_jobs = (int32_t)group.size();
    L->queue = c->d_queue;
    L->max_steps = n_steps;
    L->threads = threads;
    L->apt = apt;
    L->precision = precision;
    L->nmax = nmax;
    L->cmax = variant == kVariantNeighbourList ? lcmax : cmax;
    L->variant = variant;
    L->kmax = kmax;
    L->thermo = group.empty() ? 0 : group[0]->thermo;
    for (const DaughterDesc* dp : group) {
        L->obs = L->obs || dp->xseries != nullptr;
        L->field = L->field || dp->field != kFieldShear;
    }
    if (L->field && L->obs)
        return fail(c, TTCF_EINVAL, "colour-field daughters cannot share a step call with "
                                    "daughters recording the extra observables");
    L->pair_stride = pair_stride;
    L->pairs_lds = pairs_lds ? 1 : 0;
    L->lds_bytes = nlf ? (pairs_lds ? nl_lds_pl : nl_lds) : lds_bytes_for(nmax, cmax, threads, precision);
    if (L->lds_bytes > c->max_lds) return fail(c, TTCF_EINVAL, "batch exceeds the LDS of one workgroup");
    const int per_cu_lds = (int)(c->max_lds / L->lds_bytes);
    // the pair-list kernel is compiled for 512-thread workgroups (256 registers: 2 waves per
    // SIMD); the cell form allows 8 waves per SIMD
    const int per_cu_waves = (nlf ? 8 : 32) / (threads / 64);
    const int per_cu = std::max(1, std::min(per_cu_lds, per_cu_waves));
    L->grid = std::min<int>(L->n_jobs, per_cu * c->num_cu);
    return TTCF_OK;
}

int32_t rho_key_of(const SysDev& d) { return (int32_t)std::lround(1000.0 * d.n / d.volume); }
int32_t rc_key_of(const SysDev& d) { return (int32_t)std::lround(10000.0 * d.rc); }

const TunedShape* find_tuned(const ttcf_ctx* c, const SysDev& d, int precision) {
    const int32_t rk = rho_key_of(d), ck = rc_key_of(d);
    for (const TunedShape& t : c->tuned)
        if (t.n == d.n && t.rho_key == rk && t.rc_key == ck && t.precision == precision &&
            t.arch == c->arch)
            return &t;
    return nullptr;
}

// Shape a daughter of system d runs with: `force`, else the explicit shape, else the tuned
// shape of its system, else the defaults.
StepShape resolve_shape(const ttcf_ctx* c, const SysDev& d, int precision, const StepShape* force) {
    StepShape e;
    if (force) {
        e = *force;
    } else if (c->shape_explicit) {
        e = c->shape;
    } else if (const TunedShape* t = find_tuned(c, d, precision)) {
        e = t->shape;
    }
    return e;
}

// Writes the list grid and pair capacity of shape e into a descriptor; *nl tells whether it
// runs in the pair-list form (FP32 forces, at most kPairMaxAtoms atoms, not forced to cells,
// and its LDS fits).
int32_t apply_shape(ttcf_ctx* c, const StepShape& e, int precision, DaughterDesc* d, bool* nl) {
    *nl = false;
    d->kmax = 0;
    if (precision == TTCF_PREC_FP32_FORCES && e.variant != 1 && d->sys.n <= kPairMaxAtoms &&
        e.kmax <= kPairMaxCap && set_list_grid(&d->sys, e.skin)) {
        const int cells = d->sys.lc[0] * d->sys.lc[1] * d->sys.lc[2];
        if (lds_bytes_pairs(d->sys.n, cells) <= c->max_lds) {
            *nl = true;
            d->kmax = e.kmax > 0 ? e.kmax : auto_pair_cap(d->sys);
        }
    }
    if ((e.variant == 2 || e.variant == 3) && !*nl)
        return fail(c, TTCF_EINVAL, "pair-list form does not fit this batch");
    return TTCF_OK;
}

// The context's pair-list scratch, grown (after the stream drains) to `bytes`.
int32_t ensure_nl_scratch(ttcf_ctx* c, size_t bytes) {
    if (bytes <= c->nl_scratch_bytes) return TTCF_OK;
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    dev_free(c->nl_scratch);
    c->nl_scratch = (uint32_t*)dev_alloc(bytes, c->stream);
    c->nl_scratch_bytes = c->nl_scratch ? bytes : 0;
    if (!c->nl_scratch) return fail(c, TTCF_ENOMEM, "list scratch allocation failed");
    return TTCF_OK;
}

// Advances the live daughters selected by `only` (all when null) by up to n_steps. `force`
// (may be null) overrides every other shape. With timing, the launches are bracketed by
// events that ttcf_step_timing reads.
int32_t step_impl(ttcf_ctx* c, int32_t n_steps, const std::vector<char>* only,
                  const StepShape* force, bool timing) {
    if (c->descs.empty() || n_steps == 0) return TTCF_OK;
    int32_t rc = sync_descs(c);
    if (rc != TTCF_OK) return rc;
    // daughters still to run; each goes to the pair-list form when it may, else to the cell
    // form; each (form, thermostat) is one persistent launch, largest systems first.
    // groups[2 form + thermo], form 0 pair lists (4 atoms per thread), 1 cells, 2 pair lists
    // (8 atoms per thread: more than 2048 atoms)
    std::vector<int32_t> groups[6];
    // planar-elongation (0, 1) and mixed-flow (2, 3) daughters by thermostat: own kernels, FP64
    std::vector<int32_t> pef[4];
    std::vector<StepShape> eff(c->descs.size());
    int precision = -1;
    for (size_t i = 0; i < c->descs.size(); ++i) {
        DaughterDesc& d = c->descs[i];
        if (d.health != 0 || d.done >= d.n_steps || (only && !(*only)[i])) continue;
        if (d.field == kFieldElong || d.field == kFieldMixed) {
            pef[(d.field == kFieldMixed ? 2 : 0) + (d.thermo ? 1 : 0)].push_back((int32_t)i);
            continue;
        }
        const Mother& m = c->mothers[c->batches[c->live[i].batch].mother];
        if (precision < 0)
            precision = m.sys.precision;
        else if (precision != m.sys.precision)
            return fail(c, TTCF_EINVAL, "live daughters mix force precisions");
        const StepShape e = resolve_shape(c, d.sys, precision, force);
        eff[i] = e;
        bool nl = false;
        rc = apply_shape(c, e, precision, &d, &nl);
        if (rc != TTCF_OK) return rc;
        if (d.xseries && !nl)
            return fail(c, TTCF_EINVAL, "daughters recording the extra observables need the "
                                        "neighbour-list form, and this system runs in cells");
        if (d.field != kFieldShear && !nl)
            return fail(c, TTCF_EINVAL, "colour-field daughters need the neighbour-list form, "
                                        "and this system runs in cells");
        const int form = !nl ? 1 : (pair_job_apt(d.sys.n) == pair_small_apt() ? 0 : 2);
        groups[2 * form + (d.thermo ? 1 : 0)].push_back((int32_t)i);
    }
    const bool any_nl = !groups[0].empty() || !groups[1].empty() || !groups[4].empty() ||
                        !groups[5].empty();
    const bool any_cell = !groups[2].empty() || !groups[3].empty();
    if (!any_nl && !any_cell && pef[0].empty() && pef[1].empty() && pef[2].empty() &&
        pef[3].empty())
        return TTCF_OK;
    if (any_nl) {
        rc = push_descs(c);  // the list grids were just written into the descriptors
        if (rc != TTCF_OK) return rc;
    }
    auto by_size = [&](int32_t a, int32_t b) { return c->descs[a].sys.n > c->descs[b].sys.n; };
    std::vector<int32_t> order;
    for (auto& g : groups) {
        std::stable_sort(g.begin(), g.end(), by_size);
        order.insert(order.end(), g.begin(), g.end());
    }
    for (auto& g : pef) {
        std::stable_sort(g.begin(), g.end(), by_size);
        order.insert(order.end(), g.begin(), g.end());
    }
    if (c->d_order_cap < order.size()) {
        dev_free(c->d_order);
        c->d_order = (int32_t*)dev_alloc(sizeof(int32_t) * order.size() * 2, c->stream);
        if (!c->d_order) return fail(c, TTCF_ENOMEM, "order allocation failed");
        c->d_order_cap = order.size() * 2;
    }
    HIPCHECK(c, hipMemcpyAsync(c->d_order, order.data(), sizeof(int32_t) * order.size(),
                               hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    if (any_nl || any_cell)
        c->last_variant = !any_nl ? kVariantCells : (!any_cell ? kVariantNeighbourList : 3);
    size_t offset = 0;
    for (int gi = 0; gi < 6; ++gi) {
        const int form = gi / 2;
        const std::vector<int32_t>& group = groups[gi];
        if (group.empty()) continue;
        // the largest system's shape sets the workgroup size
        std::vector<const DaughterDesc*> ds;
        bool block_explicit = false;
        for (int32_t i : group) {
            ds.push_back(&c->descs[i]);
            block_explicit = block_explicit ||
                             c->mothers[c->batches[c->live[i].batch].mother].sys.block_threads > 0;
        }
        BatchLaunch L{};
        rc = plan_group(c, ds, block_explicit, form == 1 ? kVariantCells : kVariantNeighbourList,
                        precision, n_steps, eff[group[0]].threads, &L);
        if (rc != TTCF_OK) return rc;
        if (form != 1 && !L.pairs_lds) {
            rc = ensure_nl_scratch(c, sizeof(uint32_t) * (size_t)L.grid * (size_t)L.pair_stride);
            if (rc != TTCF_OK) return rc;
            L.pairs = c->nl_scratch;
        }
        L.order = c->d_order + offset;
        offset += group.size();
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timing) {
            HIPCHECK(c, hipEventCreate(&e0));
            HIPCHECK(c, hipEventCreate(&e1));
            HIPCHECK(c, hipEventRecord(e0, c->stream));
        }
        HIPCHECK(c, launch_daughters(L, c->stream));
        if (timing) {
            HIPCHECK(c, hipEventRecord(e1, c->stream));
            c->pending_events.emplace_back(e0, e1);
        }
    }
    for (int th = 0; th < 4; ++th) {
        if (pef[th].empty()) continue;
        PefLaunch P{};
        P.descs = c->d_descs;
        P.order = c->d_order + offset;
        offset += pef[th].size();
        P.n_jobs = (int32_t)pef[th].size();
        P.max_steps = n_steps;
        P.thermo = th & 1;
        P.mix = th >> 1;
        for (int32_t i : pef[th]) {
            const SysDev& sd = c->descs[i].sys;
            P.nmax = std::max(P.nmax, sd.n);
            // no cell grid of a box of this volume exceeds volume / r_c^3 cells
            P.cmax = std::max(P.cmax, pef_max_cells(sd.volume, sd.rc) + 8);
        }
        P.threads = pef_threads(P.nmax);
        P.lds_bytes = lds_bytes_pef(P.nmax, P.cmax);
        if (P.lds_bytes > c->max_lds)
            return fail(c, TTCF_EINVAL, "planar-elongation batch exceeds the LDS of one workgroup");
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timing) {
            HIPCHECK(c, hipEventCreate(&e0));
            HIPCHECK(c, hipEventCreate(&e1));
            HIPCHECK(c, hipEventRecord(e0, c->stream));
        }
        HIPCHECK(c, launch_pef(P, c->stream));
        if (timing) {
            HIPCHECK(c, hipEventRecord(e1, c->stream));
            c->pending_events.emplace_back(e0, e1);
        }
    }
    c->device_newer = true;
    return TTCF_OK;
}

// Removes the live daughters of batch `bidx` without accumulating them and frees the batch.
int32_t discard_batch(ttcf_ctx* c, int32_t bidx) {
    int32_t rc = sync_descs(c);
    if (rc != TTCF_OK) return rc;
    std::vector<DaughterDesc> nd;
    std::vector<Live> nl;
    for (size_t q = 0; q < c->descs.size(); ++q) {
        if (c->live[q].batch != bidx) {
            nd.push_back(c->descs[q]);
            nl.push_back(c->live[q]);
        }
    }
    c->descs.swap(nd);
    c->live.swap(nl);
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    Batch& b = c->batches[bidx];
    dev_free(b.states);
    dev_free(b.series);
    dev_free(b.scratch);
    dev_free(b.hseries);
    dev_free(b.xseries);
    b.states = nullptr;
    b.series = nullptr;
    b.scratch = nullptr;
    b.hseries = nullptr;
    b.xseries = nullptr;
    b.remaining = 0;
    return push_descs(c);
}

}  // namespace

int32_t ttcf_step(ttcf_ctx* c, int32_t n_steps) {
    if (!c || n_steps < 0) return TTCF_EINVAL;
    return step_impl(c, n_steps, nullptr, nullptr, true);
}

int32_t ttcf_set_step_shape(ttcf_ctx* c, int32_t variant, int32_t threads, double skin,
                            int32_t kmax) {
    if (!c || variant < 0 || variant > 3 || threads < 0 || threads > kMaxThreads ||
        (threads > 0 && threads % 64 != 0) || kmax > kPairMaxCap)
        return fail(c, TTCF_EINVAL, "bad step shape (kmax is at most 64)");
    c->shape.variant = variant;
    c->shape.threads = threads;
    c->shape.skin = skin > 0.0 ? skin : 0.0;
    c->shape.kmax = kmax > 0 ? kmax : 0;
    c->shape_explicit = variant != 0 || threads != 0 || skin > 0.0 || kmax > 0;
    return TTCF_OK;
}

int32_t ttcf_autotune(ttcf_ctx* c, int32_t mother, int32_t n_states, double gamma_dot,
                      int32_t probe_steps, ttcf_shape* out) {
    if (!c) return TTCF_EINVAL;
    if (mother < 0 || mother >= (int32_t)c->mothers.size() || n_states < 0 || probe_steps < 1 ||
        !std::isfinite(gamma_dot))
        return fail(c, TTCF_EINVAL, "bad autotune arguments");
    Mother& m = c->mothers[mother];
    if (m.n_states < 1) return fail(c, TTCF_EINVAL, "autotune needs stored start states");
    if (n_states == 0 || n_states > m.n_states) n_states = m.n_states;
    const SysDev& d = m.dev;
    const int precision = m.sys.precision;
    // candidate shapes: the cell form at 256, 512 and 1024 threads; the pair-list form (four
    // atoms per thread) at the skins that fill list cells one coarser, equal to and one finer
    // than the automatic grid
    std::vector<StepShape> cand;
    for (int t : {256, 512, 1024}) {
        if (pick_apt(d.n, t) < 0) continue;
        if (lds_bytes_for(d.n, d.nc[0] * d.nc[1] * d.nc[2], t, precision) <= c->max_lds)
            cand.push_back(StepShape{1, t, 0, 0.0});
    }
    std::vector<double> skins;
    if (precision == TTCF_PREC_FP32_FORCES) {
        const double lmin = std::min(d.box[0], std::min(d.box[1], d.box[2]));
        const int n0 = (int)std::floor(lmin / (d.rc + 0.2));
        for (int lc = n0 - 1; lc <= n0 + 1; ++lc) {
            if (lc < 3) continue;
            const double skin = lmin / lc * (1.0 - 1e-9) - d.rc;
            SysDev probe = d;
            if (skin >= 0.1 && set_list_grid(&probe, skin)) skins.push_back(skin);
        }
    }
    // the automatic capacity at each skin is tried first; a capacity that overflows on the
    // probe is raised and the shape timed again
    if (d.n <= kPairMaxAtoms)
        for (double skin : skins) {
            SysDev probe = d;
            set_list_grid(&probe, skin);
            cand.push_back(StepShape{2, pair_job_threads(d.n), auto_pair_cap(probe), skin});
        }
    int32_t rc = sync_descs(c);
    if (rc != TTCF_OK) return rc;
    const int warm = std::max(1, probe_steps / 5);
    double best = 1e300;
    StepShape best_shape;
    int timed = 0;
    for (size_t ci = 0; ci < cand.size(); ++ci) {
        StepShape sh = cand[ci];
        for (int attempt = 0; attempt < 4; ++attempt) {
            if (sh.variant == 2) {
                SysDev probe = d;
                set_list_grid(&probe, sh.skin);
                if (lds_bytes_pairs(d.n, probe.lc[0] * probe.lc[1] * probe.lc[2]) > c->max_lds)
                    break;
            }
            // enough copies of the probe states to give every compute unit four daughters,
            // so that the probe measures throughput, not the latency of a few daughters
            const int32_t copies = std::max(1, (c->num_cu + n_states - 1) / n_states);
            const int32_t bfirst = (int32_t)c->batches.size();
            for (int32_t k = 0; k < copies && rc == TTCF_OK; ++k) {
                int64_t first = -1;
                rc = spawn_impl(c, mother, n_states, 0, 0xF, &gamma_dot, 1, warm + probe_steps,
                                true, &first);
            }
            const int32_t bend = (int32_t)c->batches.size();
            auto discard_probe = [&]() {
                int32_t r2 = TTCF_OK;
                for (int32_t b = bfirst; b < bend && r2 == TTCF_OK; ++b) r2 = discard_batch(c, b);
                return r2;
            };
            if (rc != TTCF_OK) {
                (void)discard_probe();
                return rc;
            }
            std::vector<char> only(c->descs.size(), 0);
            for (size_t q = 0; q < c->descs.size(); ++q)
                only[q] = c->live[q].batch >= bfirst && c->live[q].batch < bend;
            rc = step_impl(c, warm, &only, &sh, false);
            hipEvent_t e0 = nullptr, e1 = nullptr;
            float ms = 0.0f;
            if (rc == TTCF_OK) {
                HIPCHECK(c, hipEventCreate(&e0));
                HIPCHECK(c, hipEventCreate(&e1));
                HIPCHECK(c, hipEventRecord(e0, c->stream));
                rc = step_impl(c, probe_steps, &only, &sh, false);
                HIPCHECK(c, hipEventRecord(e1, c->stream));
                HIPCHECK(c, hipEventSynchronize(e1));
                HIPCHECK(c, hipEventElapsedTime(&ms, e0, e1));
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
            }
            if (rc != TTCF_OK) {
                (void)discard_probe();
                return rc;
            }
            rc = sync_descs(c);
            if (rc != TTCF_OK) return rc;
            int32_t health = 0;
            for (size_t q = 0; q < c->descs.size(); ++q)
                if (only[q]) health |= c->descs[q].health;
            rc = discard_probe();
            if (rc != TTCF_OK) return rc;
            if (health & ~kHealthListOverflow)
                return fail(c, TTCF_EDEVICE, "probe daughters failed the health check");
            if (health & kHealthListOverflow) {
                if (sh.kmax >= kPairMaxCap) break;
                sh.kmax = std::min(kPairMaxCap, sh.kmax + 4);
                continue;
            }
            ++timed;
            const double per_step = ms / probe_steps;
            if (per_step < best) {
                best = per_step;
                best_shape = sh;
            }
            break;
        }
    }
    if (timed == 0) return fail(c, TTCF_EINVAL, "no step shape fits this system");
    // a margin over the capacity the probe needed
    if (best_shape.variant == 2) best_shape.kmax = std::min(kPairMaxCap, best_shape.kmax + 2);
    TunedShape t;
    t.arch = c->arch;
    t.n = d.n;
    t.rho_key = rho_key_of(d);
    t.rc_key = rc_key_of(d);
    t.precision = precision;
    t.shape = best_shape;
    t.ms_per_step = best;
    bool replaced = false;
    for (TunedShape& u : c->tuned)
        if (u.arch == t.arch && u.n == t.n && u.rho_key == t.rho_key && u.rc_key == t.rc_key &&
            u.precision == t.precision) {
            u = t;
            replaced = true;
        }
    if (!replaced) c->tuned.push_back(t);
    if (out) {
        out->variant = best_shape.variant;
        out->threads = best_shape.threads;
        out->kmax = best_shape.kmax;
        out->skin = best_shape.skin;
        out->ms_per_step = best;
        out->candidates = timed;
    }
    return TTCF_OK;
}

int32_t ttcf_autotune_export(ttcf_ctx* c, char* buf, int64_t cap, int64_t* len) {
    if (!c || cap < 0) return TTCF_EINVAL;
    std::string js = "[\n";
    char line[512];
    for (size_t i = 0; i < c->tuned.size(); ++i) {
        const TunedShape& t = c->tuned[i];
        std::snprintf(line, sizeof line,
                      "{\"arch\": \"%s\", \"n\": %d, \"rho_key\": %d, \"rc_key\": %d, "
                      "\"precision\": %d, \"variant\": %d, \"threads\": %d, \"kmax\": %d, "
                      "\"skin\": %.17g, \"ms_per_step\": %.9g}%s\n",
                      t.arch.c_str(), t.n, t.rho_key, t.rc_key, t.precision, t.shape.variant,
                      t.shape.threads, t.shape.kmax, t.shape.skin, t.ms_per_step,
                      i + 1 < c->tuned.size() ? "," : "");
        js += line;
    }
    js += "]\n";
    if (len) *len = (int64_t)js.size();
    if (buf && cap > 0) {
        const size_t n = std::min<size_t>(js.size(), (size_t)cap - 1);
        std::memcpy(buf, js.data(), n);
        buf[n] = '\0';
        if (js.size() + 1 > (size_t)cap) return fail(c, TTCF_EINVAL, "buffer too small");
    }
    return TTCF_OK;
}

namespace {
// Value of "key": in the object text [b, e); strings without escapes, numbers via strtod.
bool json_field(const char* b, const char* e, const char* key, std::string* str, double* num) {
    const std::string pat = std::string("\"") + key + "\"";
    const std::string obj(b, e);
    size_t at = obj.find(pat);
    if (at == std::string::npos) return false;
    at = obj.find(':', at + pat.size());
    if (at == std::string::npos) return false;
    ++at;
    while (at < obj.size() && (obj[at] == ' ' || obj[at] == '\t')) ++at;
    if (at >= obj.size()) return false;
    if (str) {
        if (obj[at] != '"') return false;
        const size_t end = obj.find('"', at + 1);
        if (end == std::string::npos) return false;
        *str = obj.substr(at + 1, end - at - 1);
        return true;
    }
    char* stop = nullptr;
    *num = std::strtod(obj.c_str() + at, &stop);
    return stop != obj.c_str() + at;
}
}  // namespace

int32_t ttcf_autotune_import(ttcf_ctx* c, const char* text) {
    if (!c || !text) return TTCF_EINVAL;
    std::vector<TunedShape> got;
    const char* p = text;
    while ((p = std::strchr(p, '{')) != nullptr) {
        const char* e = std::strchr(p, '}');
        if (!e) return fail(c, TTCF_EINVAL, "autotune cache: unterminated object");
        TunedShape t;
        double v[9];
        const char* keys[9] = {"n", "rho_key", "rc_key", "precision", "variant",
                               "threads", "kmax", "skin", "ms_per_step"};
        if (!json_field(p, e, "arch", &t.arch, nullptr))
            return fail(c, TTCF_EINVAL, "autotune cache: missing arch");
        for (int k = 0; k < 9; ++k)
            if (!json_field(p, e, keys[k], nullptr, &v[k]))
                return fail(c, TTCF_EINVAL, std::string("autotune cache: missing ") + keys[k]);
        t.n = (int32_t)v[0];
        t.rho_key = (int32_t)v[1];
        t.rc_key = (int32_t)v[2];
        t.precision = (int32_t)v[3];
        t.shape.variant = (int32_t)v[4];
        t.shape.threads = (int32_t)v[5];
        t.shape.kmax = (int32_t)v[6];
        t.shape.skin = v[7];
        t.ms_per_step = v[8];
        if (t.shape.variant < 1 || t.shape.variant > 2 || t.shape.threads % 64 != 0 ||
            t.shape.threads < 64 || t.shape.threads > kMaxThreads || t.shape.kmax < 0 ||
            t.shape.kmax > (t.shape.variant == 2 ? kPairMaxCap : 255) || !(t.shape.skin >= 0.0) ||
            t.n < 2)
            return fail(c, TTCF_EINVAL, "autotune cache: shape out of range");
        got.push_back(t);
        p = e + 1;
    }
    for (const TunedShape& t : got) {
        bool replaced = false;
        for (TunedShape& u : c->tuned)
            if (u.arch == t.arch && u.n == t.n && u.rho_key == t.rho_key && u.rc_key == t.rc_key &&
                u.precision == t.precision) {
                u = t;
                replaced = true;
            }
        if (!replaced) c->tuned.push_back(t);
    }
    return TTCF_OK;
}

int32_t ttcf_step_timing(ttcf_ctx* c, double* total_ms, int64_t* launches, int32_t reset) {
    if (!c) return TTCF_EINVAL;
    for (auto& ev : c->pending_events) {
        HIPCHECK(c, hipEventSynchronize(ev.second));
        float ms = 0.0f;
        HIPCHECK(c, hipEventElapsedTime(&ms, ev.first, ev.second));
        c->step_ms += ms;
        c->step_launches += 1;
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    c->pending_events.clear();
    if (total_ms) *total_ms = c->step_ms;
    if (launches) *launches = c->step_launches;
    if (reset) {
        c->step_ms = 0.0;
        c->step_launches = 0;
    }
    return TTCF_OK;
}

int32_t ttcf_accumulate(ttcf_ctx* c, int64_t* out_groups) {
    if (!c) return TTCF_EINVAL;
    int32_t rc = sync_descs(c);
    if (rc != TTCF_OK) return rc;
    // ready groups: every daughter finished or failed; groups are contiguous in descs
    std::vector<int32_t> first_of;
    std::vector<char> take(c->descs.size(), 0);
    size_t i = 0;
    std::vector<std::pair<size_t, size_t>> ready;
    while (i < c->descs.size()) {
        size_t j = i;
        bool done = true;
        while (j < c->descs.size() && c->descs[j].group == c->descs[i].group) {
            const DaughterDesc& d = c->descs[j];
            if (d.health == 0 && d.done < d.n_steps) done = false;
            ++j;
        }
        if (done) ready.emplace_back(i, j);
        i = j;
    }
    if (ready.empty()) {
        if (out_groups) *out_groups = 0;
        return TTCF_OK;
    }
    // groups with equal series length go in one launch; lengths may differ between batches
    std::vector<int32_t> lens;
    for (auto& r : ready) lens.push_back(c->descs[r.first].n_steps + 1);
    int32_t maxlen = *std::max_element(lens.begin(), lens.end());
    rc = grow_acc(c, c->acc_rows + (int64_t)ready.size(), maxlen);
    if (rc != TTCF_OK) return rc;
    int64_t added_healthy = 0;
    std::vector<int32_t> uniq = lens;
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    int32_t* d_first = (int32_t*)dev_alloc(sizeof(int32_t) * (ready.size() + 1), c->stream);
    if (!d_first) return fail(c, TTCF_ENOMEM, "index allocation failed");
    for (int32_t len : uniq) {
        first_of.clear();
        std::vector<size_t> which;
        for (size_t g = 0; g < ready.size(); ++g)
            if (lens[g] == len) which.push_back(g);
        // the kernel reads each group's daughters as a contiguous desc range
        // (group k: descs [first_of[k], first_of[k+1]) ); build a compacted desc array
        std::vector<DaughterDesc> sub;
        for (size_t g : which) {
            first_of.push_back((int32_t)sub.size());
            for (size_t q = ready[g].first; q < ready[g].second; ++q) sub.push_back(c->descs[q]);
        }
        first_of.push_back((int32_t)sub.size());
        DaughterDesc* d_sub = (DaughterDesc*)dev_alloc(sizeof(DaughterDesc) * sub.size(), c->stream);
        if (!d_sub) {
            dev_free(d_first);
            return fail(c, TTCF_ENOMEM, "descriptor allocation failed");
        }
        HIPCHECK(c, hipMemcpyAsync(d_sub, sub.data(), sizeof(DaughterDesc) * sub.size(),
                                   hipMemcpyHostToDevice, c->stream));
        HIPCHECK(c, hipMemcpyAsync(d_first, first_of.data(), sizeof(int32_t) * first_of.size(),
                                   hipMemcpyHostToDevice, c->stream));
        AccumLaunch A{};
        A.descs = d_sub;
        A.first_of = d_first;
        A.d_out = c->acc_d + (size_t)c->acc_rows * c->acc_stride;
        A.i_out = c->acc_i + (size_t)c->acc_rows * c->acc_stride;
        A.health_out = c->d_row_health + c->acc_rows;
        A.gamma_out = c->d_row_gamma + c->acc_rows;
        A.h_out = c->acc_h + (size_t)c->acc_rows * c->acc_stride;
        A.n_groups = (int32_t)which.size();
        A.n_t = len;
        A.row_stride = c->acc_stride;  // rows are written with the context's stride
        HIPCHECK(c, launch_accumulate(A, c->stream));
        // extra observables: one launch per run of consecutive groups that recorded them
        std::vector<char> has_x(which.size(), 1);
        for (size_t q = 0; q < which.size(); ++q)
            for (size_t d = ready[which[q]].first; d < ready[which[q]].second; ++d)
                has_x[q] = has_x[q] && c->descs[d].xseries != nullptr;
        for (size_t q0 = 0; q0 < which.size();) {
            if (!has_x[q0]) {
                ++q0;
                continue;
            }
            size_t q1 = q0;
            while (q1 < which.size() && has_x[q1]) ++q1;
            if (!c->acc_xd) {
                dev_free(d_sub);
                dev_free(d_first);
                return fail(c, TTCF_ESTATE, "no accumulator for the extra observables");
            }
            AccumObsLaunch X{};
            X.descs = d_sub;
            X.first_of = d_first + q0;
            X.stride = c->acc_stride;
            X.row_stride = (int64_t)kObsCols * c->acc_stride;
            X.d_out = c->acc_xd + (size_t)(c->acc_rows + (int64_t)q0) * X.row_stride;
            X.i_out = c->acc_xi + (size_t)(c->acc_rows + (int64_t)q0) * X.row_stride;
            X.n_groups = (int32_t)(q1 - q0);
            X.n_t = len;
            HIPCHECK(c, launch_accumulate_obs(X, c->stream));
            q0 = q1;
        }
        std::vector<int32_t> hh(which.size());
        HIPCHECK(c, hipMemcpyAsync(hh.data(), A.health_out, sizeof(int32_t) * which.size(),
                                   hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        dev_free(d_sub);
        for (size_t q = 0; q < which.size(); ++q) {
            const DaughterDesc& d0 = c->descs[ready[which[q]].first];
            const double temp =
                c->mothers[c->batches[c->live[ready[which[q]].first].batch].mother].sys.temperature;
            const bool colour = d0.field == kFieldColour;
            // the row's field strength and coef, Omega(0) = -coef * (series(0) / V): the
            // series is V P_xy for shear (Omega = -(V/T) gamma_dot P_xy), V J_x for the
            // colour field (Omega = +(V/T) F_e J_x) and V (P_xx - P_yy) for planar
            // elongation (Omega = -(V/T) rate (P_xx - P_yy), the shear form)
            c->row_gamma.push_back(colour ? d0.fe : d0.gamma_dot);
            c->row_field.push_back(d0.field);
            c->row_dt.push_back(d0.sys.dt);
            c->row_maps.push_back((int32_t)(ready[which[q]].second - ready[which[q]].first));
            c->row_coef.push_back(colour ? -d0.sys.volume * d0.fe / temp
                                         : d0.sys.volume * d0.gamma_dot / temp);
            c->row_nt.push_back(len);
            c->row_health.push_back(hh[q]);
            c->row_x.push_back(has_x[q]);
            {
                // a group carries the control variate when all its daughters do, in one role
                int role = c->live[ready[which[q]].first].cv_role;
                for (size_t d = ready[which[q]].first; d < ready[which[q]].second; ++d)
                    if (c->descs[d].hseries == nullptr || c->live[d].cv_role != role) role = 0;
                c->row_cv.push_back(role);
            }
            if (hh[q] == 0) ++added_healthy;
        }
        c->acc_rows += (int64_t)which.size();
        for (size_t g : which)
            for (size_t q = ready[g].first; q < ready[g].second; ++q) take[q] = 1;
    }
    dev_free(d_first);
    HIPCHECK(c, hipMemcpyAsync(c->d_row_coef, c->row_coef.data(), sizeof(double) * c->row_coef.size(),
                               hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipMemcpyAsync(c->d_row_gamma, c->row_gamma.data(),
                               sizeof(double) * c->row_gamma.size(), hipMemcpyHostToDevice, c->stream));
    // drop accumulated daughters; free batches with nothing left
    std::vector<DaughterDesc> nd;
    std::vector<Live> nl;
    for (size_t q = 0; q < c->descs.size(); ++q) {
        if (take[q]) {
            c->batches[c->live[q].batch].remaining -= 1;
        } else {
            nd.push_back(c->descs[q]);
            nl.push_back(c->live[q]);
        }
    }
    c->descs.swap(nd);
    c->live.swap(nl);
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    for (auto& b : c->batches) {
        if (b.remaining == 0 && b.states) {
            dev_free(b.states);
            dev_free(b.series);
            dev_free(b.scratch);
            dev_free(b.hseries);
            dev_free(b.xseries);
            b.states = nullptr;
            b.series = nullptr;
            b.scratch = nullptr;
            b.hseries = nullptr;
            b.xseries = nullptr;
        }
    }
    rc = push_descs(c);
    if (rc != TTCF_OK) return rc;
    if (out_groups) *out_groups = added_healthy;
    if (added_healthy == 0) return fail(c, TTCF_EUNSTABLE, "every finished group failed its health check");
    return TTCF_OK;
}

namespace {
// Rows that replayed graphs wrote carry their health on the device only: fetch it.
int32_t refresh_row_health(ttcf_ctx* c) {
    if (!c->graph_rows_dirty || c->acc_rows == 0) return TTCF_OK;
    HIPCHECK(c, hipMemcpyAsync(c->row_health.data(), c->d_row_health,
                               sizeof(int32_t) * (size_t)c->acc_rows, hipMemcpyDeviceToHost,
                               c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    c->graph_rows_dirty = false;
    return TTCF_OK;
}
}  // namespace

namespace {
// Columns of an observable in the accumulator: P_xy has its own arrays (acc_d, acc_i); the
// extra observables are columns of acc_xd, acc_xi. Returns false for an unknown observable.
static_assert(kObsSlabs == TTCF_BULK_SLABS, "slab count of the ABI");
bool obs_columns(int32_t observable, int* col0, int* ncol) {
    switch (observable) {
        case TTCF_OBS_PXY: *col0 = -1; *ncol = 1; return true;
        case TTCF_OBS_JX: *col0 = -1; *ncol = 1; return true;  // colour rows hold V J_x there
        case TTCF_OBS_PEF_N1: *col0 = -1; *ncol = 1; return true;  // elongation: V (P_xx - P_yy)
        case TTCF_OBS_MIX_J: *col0 = -1; *ncol = 1; return true;   // mixed flow: V J
        case TTCF_OBS_MIX_N1: *col0 = 0; *ncol = 1; return true;   // mixed flow: P_xx - P_yy
        case TTCF_OBS_MIX_PXY: *col0 = 1; *ncol = 1; return true;  // mixed flow: P_xy
        case TTCF_OBS_N1: *col0 = 0; *ncol = 1; return true;
        case TTCF_OBS_N2: *col0 = 1; *ncol = 1; return true;
        case TTCF_OBS_ENERGY: *col0 = 2; *ncol = 1; return true;
        case TTCF_OBS_SLAB_PX: *col0 = 3; *ncol = kObsSlabs; return true;
    }
    return false;
}

// the field whose rows carry an observable
int32_t field_of_observable(int32_t observable) {
    switch (observable) {
        case TTCF_OBS_JX: return kFieldColour;
        case TTCF_OBS_PEF_N1: return kFieldElong;
        case TTCF_OBS_MIX_J:
        case TTCF_OBS_MIX_N1:
        case TTCF_OBS_MIX_PXY: return kFieldMixed;
    }
    return kFieldShear;
}

// accumulator arrays and row stride of column `col` (-1: P_xy)
void obs_arrays(const ttcf_ctx* c, int col, const double** d, const double** i, int64_t* stride) {
    if (col < 0) {
        *d = c->acc_d;
        *i = c->acc_i;
        *stride = c->acc_stride;
    } else {
        *d = c->acc_xd + (size_t)col * c->acc_stride;
        *i = c->acc_xi + (size_t)col * c->acc_stride;
        *stride = (int64_t)kObsCols * c->acc_stride;
    }
}
}  // namespace

int32_t ttcf_response(ttcf_ctx* c, int32_t observable, double gamma_dot_filter, int32_t n_t,
                      double* ttcf_mean, double* ttcf_se, double* dav_mean, double* dav_se,
                      int64_t* out_n_states) {
    int col0 = 0, ncol = 0;
    if (!c || n_t <= 0 || !obs_columns(observable, &col0, &ncol)) return TTCF_EINVAL;
    int32_t rc0 = refresh_row_health(c);
    if (rc0 != TTCF_OK) return rc0;
    const int32_t want_field = field_of_observable(observable);
    std::vector<int32_t> rows;
    for (int64_t r = 0; r < c->acc_rows; ++r) {
        if (c->row_field[r] != want_field) continue;
        if (gamma_dot_filter > 0.0 && c->row_gamma[r] != gamma_dot_filter) continue;
        if (c->row_health[r] != 0) continue;
        if (gamma_dot_filter <= 0.0 && c->row_gamma[r] == 0.0) continue;
        rows.push_back((int32_t)r);
    }
    if (rows.empty()) return fail(c, TTCF_ESTATE, "no accumulated group matches the filter");
    for (int32_t r : rows) {
        if (c->row_nt[r] < n_t) return fail(c, TTCF_ESTATE, "n_t exceeds a matching group's length");
        if (col0 >= 0 && !c->row_x[r])
            return fail(c, TTCF_ESTATE, "a matching group did not record the extra observables");
    }
    const size_t plane = (size_t)n_t * ncol;
    const size_t bytes = sizeof(int32_t) * rows.size() + sizeof(double) * 4 * plane + 64;
    char* scratch = (char*)dev_alloc(bytes, c->stream);
    if (!scratch) return fail(c, TTCF_ENOMEM, "response scratch allocation failed");
    double* d_out = (double*)scratch;
    int32_t* d_used = (int32_t*)(scratch + sizeof(double) * 4 * plane);
    int32_t* d_rows = d_used + 4;
    HIPCHECK(c, hipMemcpyAsync(d_rows, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice,
                               c->stream));
    std::vector<int32_t> hh = c->row_health;
    HIPCHECK(c, hipMemcpyAsync(c->d_row_health, hh.data(), sizeof(int32_t) * hh.size(),
                               hipMemcpyHostToDevice, c->stream));
    for (int q = 0; q < ncol; ++q) {
        const double* da = nullptr;
        const double* ia = nullptr;
        int64_t stride = 0;
        obs_arrays(c, col0 < 0 ? -1 : col0 + q, &da, &ia, &stride);
        ResponseLaunch R{};
        R.d_all = da;
        R.i_all = ia;
        R.gamma = c->d_row_gamma;
        R.coef = c->d_row_coef;
        R.health = c->d_row_health;
        R.rows = d_rows;
        R.n_rows = (int32_t)rows.size();
        R.n_t = n_t;
        R.n_t_stride = (int32_t)stride;
        R.normalise = gamma_dot_filter <= 0.0 ? 1 : 0;
        R.out = d_out + (size_t)q * 4 * n_t;
        R.used = d_used;
        HIPCHECK(c, launch_response(R, c->stream));
    }
    std::vector<double> out(4 * plane);
    int32_t used = 0;
    HIPCHECK(c, hipMemcpyAsync(out.data(), d_out, sizeof(double) * 4 * plane, hipMemcpyDeviceToHost,
                               c->stream));
    HIPCHECK(c, hipMemcpyAsync(&used, d_used, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    dev_free(scratch);
    // column q's block holds mean, se, dav, dav se (n_t each); the outputs put the columns
    // fastest
    double* dst[4] = {ttcf_mean, ttcf_se, dav_mean, dav_se};
    for (int w = 0; w < 4; ++w) {
        if (!dst[w]) continue;
        for (int32_t k = 0; k < n_t; ++k)
            for (int q = 0; q < ncol; ++q)
                dst[w][(size_t)k * ncol + q] = out[((size_t)q * 4 + w) * n_t + k];
    }
    if (out_n_states) *out_n_states = used;
    return TTCF_OK;
}

// ---------------------------------------------------------------------------------------
// captured batch cycles
// ---------------------------------------------------------------------------------------
struct ttcf_graph {
    ttcf_ctx* ctx = nullptr;
    hipStream_t cap = nullptr;        // private stream the cycle was captured on
    std::vector<hipStream_t> side;    // branches of the capture (the parts' mothers and spawns)
    std::vector<hipEvent_t> events;   // fork and join points of the branches
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void*> bufs;          // device buffers owned by the graph
    int32_t n_states = 0, max_replays = 0, replays = 0;
    // (mother, steps the context's own mother advances per replay) of every part
    std::vector<std::pair<int32_t, int64_t>> mother_steps;
    void* get(size_t bytes) {
        void* p = dev_alloc(bytes + 64, ctx->stream);
        if (p) bufs.push_back(p);
        return p;
    }
};

namespace {

constexpr int32_t kRowPending = 1 << 30;  // reserved row not yet written by a replay

void free_graph(ttcf_graph* g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    for (hipStream_t s : g->side) (void)hipStreamDestroy(s);
    for (hipEvent_t e : g->events) (void)hipEventDestroy(e);
    for (void* p : g->bufs) dev_free(p);
    delete g;
}

// One mother's share of a captured cycle.
struct GraphPart {
    const ttcf_graph_desc* gd = nullptr;
    int32_t n = 0;                      // atoms
    size_t sz = 0;                      // doubles per state
    int32_t n_states = 0, nm = 0, nd = 0, n_copies = 0;
    std::vector<int32_t> maps;
    int32_t st0 = 0, d0 = 0;            // its first state (group) and daughter in the cycle
    size_t dstate0 = 0;                 // its daughters' first double in the state buffer
    double* states = nullptr;           // saved start states
    double* szeta = nullptr;            // their thermostat variables
    MotherLaunch* d_ml = nullptr;
    std::vector<MotherLaunch> ml;
    bool nh = false;
    StepShape shape;
};

// Records one cycle over the mothers of `gds` (every part as ttcf_graph_create describes):
// each part's mothers save their states and their daughters are spawned, then all daughters
// run in the persistent step launches of their (form, thermostat), largest systems first, as
// ttcf_step would run them, and every group is folded into the reserved rows.
int32_t graph_create_impl(ttcf_ctx* c, const ttcf_graph_desc* gds, int32_t n_desc,
                          ttcf_graph** out) {
    if (!c || !gds || n_desc <= 0 || !out) return TTCF_EINVAL;
    if (c->record_obs)
        return fail(c, TTCF_ESTATE, "captured cycles record P_xy only: switch the extra "
                                    "observables off first");
    std::vector<GraphPart> parts(n_desc);
    int64_t states64 = 0;
    int32_t nd = 0;
    int precision = -1;
    size_t dstate_total = 0;
    const int32_t n_steps = gds[0].n_steps;
    const int32_t max_replays = gds[0].max_replays;
    for (int32_t k = 0; k < n_desc; ++k) {
        const ttcf_graph_desc* gd = &gds[k];
        if (gd->mother < 0 || gd->mother >= (int32_t)c->mothers.size() || gd->n_replicas < 0 ||
            gd->states_per_replica <= 0 || gd->steps_between <= 0 || gd->decorrelate_steps < 0 ||
            (gd->mapping_mask & 0xFu) == 0 || (gd->mapping_mask & ~0xFu) != 0 || !gd->gamma_dot ||
            gd->n_steps <= 0 || gd->max_replays <= 0)
            return fail(c, TTCF_EINVAL, "bad graph description");
        if (gd->n_steps != n_steps || gd->max_replays != max_replays)
            return fail(c, TTCF_EINVAL, "the parts of a cycle share n_steps and max_replays");
        for (int32_t j = 0; j < k; ++j)
            if (gds[j].mother == gd->mother)
                return fail(c, TTCF_EINVAL, "a mother appears in two parts of a cycle");
        const Mother& m = c->mothers[gd->mother];
        if (precision < 0)
            precision = m.sys.precision;
        else if (precision != m.sys.precision)
            return fail(c, TTCF_EINVAL, "the mothers of a cycle mix force precisions");
        GraphPart& P = parts[k];
        P.gd = gd;
        P.n = m.dev.n;
        P.sz = 6 * (size_t)P.n;
        P.n_copies = std::max(1, gd->n_replicas);
        const int64_t ns64 = (int64_t)P.n_copies * gd->states_per_replica;
        if (ns64 > (1 << 22)) return fail(c, TTCF_EINVAL, "too many start states per replay");
        P.n_states = (int32_t)ns64;
        if (!(gd->n_gamma == 1 || gd->n_gamma == P.n_states))
            return fail(c, TTCF_EINVAL, "n_gamma must be 1 or the number of saved states");
        for (int32_t q = 0; q < gd->n_gamma; ++q)
            if (!std::isfinite(gd->gamma_dot[q]))
                return fail(c, TTCF_EINVAL, "shear rates must be finite");
        for (int q = 0; q < 4; ++q)
            if (gd->mapping_mask & (1u << q)) P.maps.push_back(q);
        P.nm = (int32_t)P.maps.size();
        P.nd = P.n_states * P.nm;
        P.st0 = (int32_t)states64;
        P.d0 = nd;
        P.dstate0 = dstate_total;
        P.nh = m.sys.daughter_thermostat == TTCF_DAUGHTER_NH;
        states64 += P.n_states;
        if (states64 > (1 << 22)) return fail(c, TTCF_EINVAL, "too many start states per replay");
        nd += P.nd;
        dstate_total += P.sz * P.nd;
    }
    const int32_t n_states = (int32_t)states64;
    const int32_t n_t = n_steps + 1;
    const int64_t reserve = (int64_t)max_replays * n_states;
    // accumulator rows: grow (while nothing pins it) to hold the reserved rows and headroom
    int32_t rc = grow_acc(c, c->acc_rows + reserve + 4096, n_t);
    if (rc != TTCF_OK) return rc;

    ttcf_graph* g = new ttcf_graph();
    g->ctx = c;
    g->n_states = n_states;
    g->max_replays = max_replays;
    auto bail = [&](int32_t code, const std::string& msg) {
        (void)hipStreamSynchronize(c->stream);
        free_graph(g);
        return fail(c, code, msg);
    };
    double* dstates = (double*)g->get(sizeof(double) * dstate_total);
    double* series = (double*)g->get(sizeof(double) * (size_t)n_t * nd);
    DaughterDesc* descs = (DaughterDesc*)g->get(sizeof(DaughterDesc) * nd);
    DaughterDesc* templ = (DaughterDesc*)g->get(sizeof(DaughterDesc) * nd);
    int32_t* ints = (int32_t*)g->get(sizeof(int32_t) * ((size_t)3 * nd + n_states + 8));
    double** dst = (double**)g->get(sizeof(double*) * nd);
    if (!dstates || !series || !descs || !templ || !ints || !dst)
        return bail(TTCF_ENOMEM, "graph allocation failed");
    int32_t* order = ints;
    int32_t* state_of = order + nd;         // the part's own state index
    int32_t* map_of = state_of + nd;
    int32_t* first_of = map_of + nd;        // n_states + 1
    int32_t* queue = first_of + n_states + 1;
    int32_t* replay = queue + 4;

    // mothers of the cycle: each part's mother itself, or persistent copies of it
    for (GraphPart& P : parts) {
        const ttcf_graph_desc* gd = P.gd;
        Mother& m = c->mothers[gd->mother];
        const int n = P.n;
        P.states = (double*)g->get(sizeof(double) * P.sz * P.n_states);
        P.szeta = (double*)g->get(sizeof(double) * P.n_states);
        P.d_ml = (MotherLaunch*)g->get(sizeof(MotherLaunch) * P.n_copies);
        if (!P.states || !P.szeta || !P.d_ml) return bail(TTCF_ENOMEM, "graph allocation failed");
        P.ml.assign(P.n_copies, MotherLaunch{});
        const double nf = 3.0 * n - 3.0;
        double* rep = nullptr;
        if (gd->n_replicas > 0) {
            rep = (double*)g->get(sizeof(double) * (P.sz * P.n_copies + P.n_copies));
            double* kick_d = gd->kicks
                                 ? (double*)g->get(sizeof(double) * 3 * (size_t)n * P.n_copies)
                                 : nullptr;
            if (!rep || (gd->kicks && !kick_d)) return bail(TTCF_ENOMEM, "graph allocation failed");
            if (gd->kicks &&
                hipMemcpyAsync(kick_d, gd->kicks, sizeof(double) * 3 * (size_t)n * P.n_copies,
                               hipMemcpyHostToDevice, c->stream) != hipSuccess)
                return bail(TTCF_EDEVICE, "kick upload failed");
            if (launch_replicate(m.state, m.zeta, n, kick_d, P.n_copies, rep,
                                 rep + P.sz * P.n_copies, c->stream) != hipSuccess)
                return bail(TTCF_EDEVICE, "replica launch failed");
        }
        for (int r = 0; r < P.n_copies; ++r) {
            MotherLaunch& L = P.ml[r];
            L.sys = m.dev;
            L.state = rep ? rep + P.sz * r : m.state;
            L.zeta = rep ? rep + P.sz * P.n_copies + r : m.zeta;
            L.temperature = m.sys.temperature;
            L.nf = nf;
            L.q = nf * m.sys.temperature * m.sys.nh_tau * m.sys.nh_tau;
            L.threads = m.threads;
            L.apt = m.apt;
            L.precision = m.sys.precision;
            L.lds_bytes = lds_for(m.dev, m.sys.precision);
            L.series = nullptr;
        }
        if (rep && gd->decorrelate_steps > 0) {
            // once, outside the graph, through the context's own launch block
            for (auto& L : P.ml) {
                L.n_chunks = 0;
                L.steps_per_chunk = gd->decorrelate_steps;
                L.snapshots = nullptr;
            }
            rc = upload_mother_launches(c, P.ml.data(), P.n_copies);
            if (rc != TTCF_OK) return bail(rc, c->err);
            if (launch_mothers(c->d_mlaunch, P.n_copies, P.ml[0], c->stream) != hipSuccess)
                return bail(TTCF_EDEVICE, "decorrelation launch failed");
        }
        for (int r = 0; r < P.n_copies; ++r) {
            P.ml[r].n_chunks = gd->states_per_replica;
            P.ml[r].steps_per_chunk = gd->steps_between;
            P.ml[r].snapshots = P.states + P.sz * (size_t)r * gd->states_per_replica;
            P.ml[r].snap_zeta = P.szeta + (size_t)r * gd->states_per_replica;
        }
        g->mother_steps.emplace_back(
            gd->mother, rep ? 0 : (int64_t)gd->states_per_replica * gd->steps_between);
    }

    // daughter descriptors (state-major groups per part, parts in order, as the same
    // ttcf_spawn_daughters calls would number them), their shapes and their step launches
    std::vector<DaughterDesc> hd(nd);
    std::vector<double*> hdst(nd);
    std::vector<int32_t> hints(3 * (size_t)nd + n_states + 1);
    std::vector<char> nl_of(nd, 0);
    bool block_explicit = false;
    for (GraphPart& P : parts) {
        const ttcf_graph_desc* gd = P.gd;
        const Mother& m = c->mothers[gd->mother];
        block_explicit = block_explicit || m.sys.block_threads > 0;
        P.shape = resolve_shape(c, m.dev, precision, nullptr);
        const double nf = 3.0 * P.n - 3.0;
        for (int32_t st = 0; st < P.n_states; ++st) {
            const int32_t group = c->next_group++;
            const double gdot = gd->gamma_dot[gd->n_gamma == 1 ? 0 : st];
            for (int32_t q = 0; q < P.nm; ++q) {
                const int32_t d = P.d0 + st * P.nm + q;
                DaughterDesc& ds = hd[d];
                ds = DaughterDesc{};
                ds.state = dstates + P.dstate0 + P.sz * (size_t)(st * P.nm + q);
                ds.series = series + (size_t)n_t * d;
                ds.sys = m.dev;
                ds.gamma_dot = gdot;
                ds.n_steps = n_steps;
                ds.group = group;
                ds.map = P.maps[q];
                ds.block = m.threads;
                if (P.nh) {  // zeta itself is written by a kernel at every replay
                    ds.thermo = 1;
                    ds.nh_q = nf * m.sys.temperature * m.sys.nh_tau * m.sys.nh_tau;
                    ds.nh_target = nf * m.sys.temperature;
                }
                bool nl = false;
                rc = apply_shape(c, P.shape, precision, &ds, &nl);
                if (rc != TTCF_OK) return bail(rc, c->err);
                nl_of[d] = nl ? 1 : 0;
                hdst[d] = ds.state;
                hints[nd + d] = st;                   // state_of (the part's own index)
                hints[2 * (size_t)nd + d] = P.maps[q];  // map_of
            }
            hints[3 * (size_t)nd + P.st0 + st] = P.d0 + st * P.nm;  // first_of
        }
    }
    hints[3 * (size_t)nd + n_states] = nd;
    // launch groups as in ttcf_step: (form, thermostat), form 0 pair lists at four atoms per
    // thread, 1 cells, 2 pair lists at eight; largest systems first inside each
    std::vector<int32_t> groups[6];
    for (int32_t d = 0; d < nd; ++d) {
        const int form = !nl_of[d] ? 1 : (pair_job_apt(hd[d].sys.n) == pair_small_apt() ? 0 : 2);
        groups[2 * form + (hd[d].thermo ? 1 : 0)].push_back(d);
    }
    std::vector<BatchLaunch> launches;
    size_t offset = 0;
    for (int gi = 0; gi < 6; ++gi) {
        std::vector<int32_t>& grp = groups[gi];
        if (grp.empty()) continue;
        std::stable_sort(grp.begin(), grp.end(),
                         [&](int32_t a, int32_t b) { return hd[a].sys.n > hd[b].sys.n; });
        std::vector<const DaughterDesc*> hp;
        for (int32_t d : grp) {
            hp.push_back(&hd[d]);
            hints[offset + hp.size() - 1] = d;   // order
        }
        const int form = gi / 2;
        const StepShape& sh = parts[0].shape;
        int threads_req = sh.threads;
        for (const GraphPart& P : parts)
            if (grp[0] >= P.d0 && grp[0] < P.d0 + P.nd) threads_req = P.shape.threads;
        BatchLaunch B{};
        rc = plan_group(c, hp, block_explicit, form == 1 ? kVariantCells : kVariantNeighbourList,
                        precision, n_steps, threads_req, &B);
        if (rc != TTCF_OK) return bail(rc, c->err);
        if (form != 1 && !B.pairs_lds) {
            // the graph owns the pair-list scratch its replays use
            B.pairs = (uint32_t*)g->get(sizeof(uint32_t) * (size_t)B.grid * (size_t)B.pair_stride);
            if (!B.pairs) return bail(TTCF_ENOMEM, "pair-list scratch allocation failed");
        }
        B.descs = descs;
        B.order = order + offset;
        B.queue = queue;
        launches.push_back(B);
        offset += grp.size();
    }

    // reserved rows: metadata on the host and the device; pending until a replay writes them
    const int64_t row0 = c->acc_rows;
    for (int64_t r = 0; r < reserve; ++r) {
        const int32_t st = (int32_t)(r % n_states);
        const GraphPart* P = &parts[0];
        for (const GraphPart& Q : parts)
            if (st >= Q.st0 && st < Q.st0 + Q.n_states) P = &Q;
        const DaughterDesc& d0 = hd[P->d0 + (size_t)(st - P->st0) * P->nm];
        const Mother& m = c->mothers[P->gd->mother];
        c->row_gamma.push_back(d0.gamma_dot);
        c->row_dt.push_back(d0.sys.dt);
        c->row_maps.push_back(P->nm);
        c->row_coef.push_back(d0.sys.volume * d0.gamma_dot / m.sys.temperature);
        c->row_nt.push_back(n_t);
        c->row_health.push_back(kRowPending);
        c->row_cv.push_back(0);
        c->row_x.push_back(0);
        c->row_field.push_back(kFieldShear);
    }
    c->acc_rows += reserve;
    auto undo_rows = [&]() {
        c->acc_rows = row0;
        c->row_gamma.resize(row0);
        c->row_dt.resize(row0);
        c->row_maps.resize(row0);
        c->row_coef.resize(row0);
        c->row_nt.resize(row0);
        c->row_health.resize(row0);
        c->row_cv.resize(row0);
        c->row_x.resize(row0);
        c->row_field.resize(row0);
    };
    const int32_t zero = 0;
    bool ok = hipMemcpyAsync(templ, hd.data(), sizeof(DaughterDesc) * nd, hipMemcpyHostToDevice,
                             c->stream) == hipSuccess &&
              hipMemcpyAsync(dst, hdst.data(), sizeof(double*) * nd, hipMemcpyHostToDevice,
                             c->stream) == hipSuccess &&
              hipMemcpyAsync(ints, hints.data(), sizeof(int32_t) * hints.size(),
                             hipMemcpyHostToDevice, c->stream) == hipSuccess &&
              hipMemcpyAsync(replay, &zero, sizeof(int32_t), hipMemcpyHostToDevice, c->stream) ==
                  hipSuccess;
    for (GraphPart& P : parts)
        ok = ok && hipMemcpyAsync(P.d_ml, P.ml.data(), sizeof(MotherLaunch) * P.n_copies,
                                  hipMemcpyHostToDevice, c->stream) == hipSuccess;
    ok = ok &&
         hipMemcpyAsync(c->d_row_gamma, c->row_gamma.data(), sizeof(double) * c->row_gamma.size(),
                        hipMemcpyHostToDevice, c->stream) == hipSuccess &&
         hipMemcpyAsync(c->d_row_coef, c->row_coef.data(), sizeof(double) * c->row_coef.size(),
                        hipMemcpyHostToDevice, c->stream) == hipSuccess &&
         hipMemcpyAsync(c->d_row_health + row0, c->row_health.data() + row0,
                        sizeof(int32_t) * (size_t)reserve, hipMemcpyHostToDevice, c->stream) ==
             hipSuccess &&
         hipStreamSynchronize(c->stream) == hipSuccess;
    if (!ok) {
        undo_rows();
        return bail(TTCF_EDEVICE, "graph upload failed");
    }
    AccumLaunch A{};
    A.descs = descs;
    A.first_of = first_of;
    A.d_out = c->acc_d + (size_t)row0 * c->acc_stride;
    A.i_out = c->acc_i + (size_t)row0 * c->acc_stride;
    A.health_out = c->d_row_health + row0;
    A.gamma_out = c->d_row_gamma + row0;
    A.h_out = c->acc_h + (size_t)row0 * c->acc_stride;
    A.n_groups = n_states;
    A.n_t = n_t;
    A.row_stride = c->acc_stride;
    A.row_step = replay;

    // the cycle: mothers -> spawn -> descriptor reset -> step -> accumulate -> next row block.
    // With several parts, each part's mothers and spawn form a branch of the graph (up to
    // kBranches branches, parts dealt round robin), so small mother launches run side by side.
    constexpr int kBranches = 8;
    const int n_branch = n_desc > 1 ? std::min<int>(n_desc, kBranches) : 0;
    bool made = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking) == hipSuccess;
    for (int b = 0; made && b < n_branch; ++b) {
        hipStream_t st = nullptr;
        made = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (made) g->side.push_back(st);
    }
    for (int b = 0; made && b < (n_branch ? n_branch + 1 : 0); ++b) {
        hipEvent_t ev = nullptr;
        made = hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        if (made) g->events.push_back(ev);
    }
    if (!made) {
        undo_rows();
        return bail(TTCF_EDEVICE, "stream creation failed");
    }
    hipError_t e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        hipError_t e1 = hipSuccess;
        if (n_branch > 0) e1 = hipEventRecord(g->events[0], g->cap);
        for (int b = 0; b < n_branch && e1 == hipSuccess; ++b)
            e1 = hipStreamWaitEvent(g->side[b], g->events[0], 0);
        for (int32_t k = 0; k < n_desc && e1 == hipSuccess; ++k) {
            GraphPart& P = parts[k];
            hipStream_t st = n_branch ? g->side[k % n_branch] : g->cap;
            e1 = launch_mothers(P.d_ml, P.n_copies, P.ml[0], st);
            if (e1 == hipSuccess)
                e1 = launch_spawn(P.states, P.n, P.n_states, state_of + P.d0, map_of + P.d0,
                                  dst + P.d0, P.nd, c->mothers[P.gd->mother].dev.box[0], st);
        }
        for (int b = 0; b < n_branch && e1 == hipSuccess; ++b) {
            e1 = hipEventRecord(g->events[1 + b], g->side[b]);
            if (e1 == hipSuccess) e1 = hipStreamWaitEvent(g->cap, g->events[1 + b], 0);
        }
        if (e1 == hipSuccess)
            e1 = launch_copy_words((const uint64_t*)templ, (uint64_t*)descs,
                                   (int64_t)(sizeof(DaughterDesc) / 8) * nd, g->cap);
        for (GraphPart& P : parts)
            if (e1 == hipSuccess && P.nh)
                e1 = launch_desc_zeta(descs + P.d0, P.szeta, state_of + P.d0, map_of + P.d0, P.nd,
                                      g->cap);
        for (const BatchLaunch& B : launches)
            if (e1 == hipSuccess) e1 = launch_daughters(B, g->cap);
        if (e1 == hipSuccess) e1 = launch_accumulate(A, g->cap);
        if (e1 == hipSuccess) e1 = launch_increment(replay, g->cap);
        e = hipStreamEndCapture(g->cap, &g->graph);
        if (e1 != hipSuccess) e = e1;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        undo_rows();
        return bail(TTCF_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
    }
    static_assert(sizeof(DaughterDesc) % 8 == 0, "descriptors are copied as 64-bit words");
    c->graphs.push_back(g);
    *out = g;
    return TTCF_OK;
}

}  // namespace

int32_t ttcf_graph_create(ttcf_ctx* c, const ttcf_graph_desc* gd, ttcf_graph** out) {
    return graph_create_impl(c, gd, 1, out);
}

int32_t ttcf_graph_create_multi(ttcf_ctx* c, const ttcf_graph_desc* gds, int32_t n_desc,
                                ttcf_graph** out) {
    if (n_desc <= 0 || n_desc > 4096) return TTCF_EINVAL;
    return graph_create_impl(c, gds, n_desc, out);
}

int32_t ttcf_graph_launch(ttcf_graph* g, int32_t n_replays) {
    if (!g || n_replays < 0) return TTCF_EINVAL;
    ttcf_ctx* c = g->ctx;
    if (g->replays + (int64_t)n_replays > g->max_replays)
        return fail(c, TTCF_ESTATE, "replays beyond the rows reserved for this graph");
    for (int32_t r = 0; r < n_replays; ++r) {
        HIPCHECK(c, hipGraphLaunch(g->exec, c->stream));
        ++g->replays;
        for (const auto& ms : g->mother_steps) c->mothers[ms.first].steps += ms.second;
        c->graph_rows_dirty = true;
    }
    return TTCF_OK;
}

int32_t ttcf_graph_replays(const ttcf_graph* g, int32_t* out) {
    if (!g || !out) return TTCF_EINVAL;
    *out = g->replays;
    return TTCF_OK;
}

void ttcf_graph_destroy(ttcf_graph* g) {
    if (!g) return;
    ttcf_ctx* c = g->ctx;
    (void)hipStreamSynchronize(c->stream);
    auto it = std::find(c->graphs.begin(), c->graphs.end(), g);
    if (it != c->graphs.end()) c->graphs.erase(it);
    free_graph(g);
}

namespace {
int32_t response_modified_impl(ttcf_ctx* c, int32_t observable, double gamma_dot_filter,
                               int32_t n_t, double* mean, double* se, int64_t* out_n_states) {
    int col0 = 0, ncol = 0;
    if (!c || !(gamma_dot_filter > 0.0) || n_t <= 0 || !obs_columns(observable, &col0, &ncol))
        return TTCF_EINVAL;
    int32_t rc = refresh_row_health(c);
    if (rc != TTCF_OK) return rc;
    const int32_t want_field = field_of_observable(observable);
    std::vector<int32_t> rows;
    for (int64_t r = 0; r < c->acc_rows; ++r)
        if (c->row_field[r] == want_field && c->row_gamma[r] == gamma_dot_filter &&
            c->row_health[r] == 0)
            rows.push_back((int32_t)r);
    if (rows.empty()) return fail(c, TTCF_ESTATE, "no accumulated group matches the filter");
    for (int32_t r : rows) {
        if (c->row_nt[r] < n_t) return fail(c, TTCF_ESTATE, "n_t exceeds a matching group's length");
        if (c->row_coef[r] != c->row_coef[rows[0]] || c->row_dt[r] != c->row_dt[rows[0]] ||
            c->row_maps[r] != c->row_maps[rows[0]])
            return fail(c, TTCF_EINVAL, "matching groups differ in V/T, dt or mapping count");
        if (col0 >= 0 && !c->row_x[r])
            return fail(c, TTCF_ESTATE, "a matching group did not record the extra observables");
    }
    Scratch sc(c->stream);
    int32_t* d_rows = sc.get<int32_t>(rows.size());
    double* d_j = sc.get<double>(rows.size() * (size_t)n_t);
    double* d_out = sc.get<double>(2 * (size_t)n_t * ncol);
    if (!d_rows || !d_j || !d_out) return fail(c, TTCF_ENOMEM, "response scratch allocation failed");
    HIPCHECK(c, hipMemcpyAsync(d_rows, rows.data(), sizeof(int32_t) * rows.size(),
                               hipMemcpyHostToDevice, c->stream));
    for (int q = 0; q < ncol; ++q) {
        const double* da = nullptr;
        const double* ia = nullptr;
        int64_t stride = 0;
        obs_arrays(c, col0 < 0 ? -1 : col0 + q, &da, &ia, &stride);
        ModifiedLaunch A{};
        A.d_all = da;
        A.i_all = ia;
        A.stride = (int32_t)stride;
        A.p_all = c->acc_d;
        A.p_stride = c->acc_stride;
        A.rows = d_rows;
        A.n_rows = (int32_t)rows.size();
        A.n_t = n_t;
        A.coef = c->row_coef[rows[0]];
        A.dt = c->row_dt[rows[0]];
        A.j_rows = d_j;  // columns run in stream order, so one scratch serves them all
        A.out = d_out + (size_t)q * 2 * n_t;
        HIPCHECK(c, launch_response_modified(A, c->stream));
    }
    std::vector<double> out(2 * (size_t)n_t * ncol);
    HIPCHECK(c, hipMemcpyAsync(out.data(), d_out, sizeof(double) * out.size(), hipMemcpyDeviceToHost,
                               c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    for (int32_t k = 0; k < n_t; ++k)
        for (int q = 0; q < ncol; ++q) {
            if (mean) mean[(size_t)k * ncol + q] = out[(size_t)q * 2 * n_t + k];
            if (se) se[(size_t)k * ncol + q] = out[(size_t)q * 2 * n_t + n_t + k];
        }
    if (out_n_states) *out_n_states = (int64_t)rows.size();
    return TTCF_OK;
}
}  // namespace

int32_t ttcf_response_modified(ttcf_ctx* c, double gamma_dot_filter, int32_t n_t, double* mean,
                               double* se, int64_t* out_n_states) {
    return response_modified_impl(c, TTCF_OBS_PXY, gamma_dot_filter, n_t, mean, se,
                                  out_n_states);
}

int32_t ttcf_observable_response_modified(ttcf_ctx* c, int32_t observable, double gamma_dot_filter,
                                          int32_t n_t, double* mean, double* se,
                                          int64_t* out_n_states) {
    return response_modified_impl(c, observable, gamma_dot_filter, n_t, mean, se, out_n_states);
}

int32_t ttcf_record_observables(ttcf_ctx* c, int32_t on) {
    if (!c || (on != 0 && on != 1)) return TTCF_EINVAL;
    if (on && !c->graphs.empty())
        return fail(c, TTCF_ESTATE, "captured graphs exist; they record P_xy only");
    if (on) {
        // the accumulator exists without the extra columns: give it them now
        const int32_t rc = ensure_acc_x(c);
        if (rc != TTCF_OK) return rc;
    }
    c->record_obs = on != 0;
    return TTCF_OK;
}

// live daughters are kept in increasing id order (spawned in order, removed in place)
static int32_t find_live(ttcf_ctx* c, int64_t id) {
    auto it = std::lower_bound(c->live.begin(), c->live.end(), id,
                               [](const Live& l, int64_t v) { return l.id < v; });
    if (it == c->live.end() || it->id != id) return -1;
    return (int32_t)(it - c->live.begin());
}

int32_t ttcf_export_observables(ttcf_ctx* c, int64_t first, int32_t count, int32_t n_t,
                                double* out) {
    if (!c || count <= 0 || n_t <= 0 || !out) return TTCF_EINVAL;
    int32_t rc = sync_descs(c);
    if (rc != TTCF_OK) return rc;
    for (int32_t q = 0; q < count; ++q) {
        const int32_t i = find_live(c, first + q);
        if (i < 0) return fail(c, TTCF_EINVAL, "no live daughter with that id");
        const DaughterDesc& d = c->descs[i];
        if (!d.xseries) return fail(c, TTCF_ESTATE, "that daughter does not record them");
        if (n_t > d.n_steps + 1) return fail(c, TTCF_EINVAL, "n_t exceeds the daughter's length");
        HIPCHECK(c, hipMemcpyAsync(out + (size_t)q * n_t * kObsCols, d.xseries,
                                   sizeof(double) * (size_t)n_t * kObsCols, hipMemcpyDeviceToHost,
                                   c->stream));
    }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return TTCF_OK;
}

int32_t ttcf_export_daughter(ttcf_ctx* c, int64_t daughter, double* r, double* p, int64_t* k) {
    if (!c) return TTCF_EINVAL;
    int32_t rc = sync_descs(c);
    if (rc != TTCF_OK) return rc;
    const int32_t i = find_live(c, daughter);
    if (i < 0) return fail(c, TTCF_EINVAL, "no such live daughter");
    const DaughterDesc& d = c->descs[i];
    const size_t n = (size_t)d.sys.n;
    if (r) HIPCHECK(c, hipMemcpyAsync(r, d.state, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->stream));
    if (p)
        HIPCHECK(c, hipMemcpyAsync(p, d.state + 3 * n, sizeof(double) * 3 * n, hipMemcpyDeviceToHost,
                                   c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    if (k) *k = d.k;
    return TTCF_OK;
}

int32_t ttcf_export_series(ttcf_ctx* c, int64_t first, int32_t count, int32_t n_t, double* vpxy) {
    if (!c || count <= 0 || n_t <= 0 || !vpxy) return TTCF_EINVAL;
    int32_t rc = sync_descs(c);
    if (rc != TTCF_OK) return rc;
    for (int32_t q = 0; q < count; ++q) {
        const int32_t i = find_live(c, first + q);
        if (i < 0) return fail(c, TTCF_EINVAL, "no such live daughter");
        const DaughterDesc& d = c->descs[i];
        if (n_t > d.n_steps + 1) return fail(c, TTCF_EINVAL, "n_t exceeds the daughter length");
        HIPCHECK(c, hipMemcpyAsync(vpxy + (size_t)q * n_t, d.series, sizeof(double) * n_t,
                                   hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return TTCF_OK;
}

int32_t ttcf_daughter_health(ttcf_ctx* c, int64_t daughter, int32_t* health) {
    if (!c || !health) return TTCF_EINVAL;
    int32_t rc = sync_descs(c);
    if (rc != TTCF_OK) return rc;
    const int32_t i = find_live(c, daughter);
    if (i < 0) return fail(c, TTCF_EINVAL, "no such live daughter");
    *health = c->descs[i].health;
    return TTCF_OK;
}

int32_t ttcf_debug_poison(ttcf_ctx* c, int64_t daughter) {
    if (!c) return TTCF_EINVAL;
    int32_t rc = sync_descs(c);
    if (rc != TTCF_OK) return rc;
    const int32_t i = find_live(c, daughter);
    if (i < 0) return fail(c, TTCF_EINVAL, "no such live daughter");
    const DaughterDesc& d = c->descs[i];
    const double nan = std::nan("");
    HIPCHECK(c, hipMemcpyAsync(d.state + 3 * (size_t)d.sys.n, &nan, sizeof(double),
                               hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return TTCF_OK;
}

}  // extern "C"

// ---- replicas of a mother ---------------------------------------------------------------

namespace {

// Copies of a mother's current state (and thermostat variable), each with its own optional
// momentum kick, advanced together by one launch of the mother kernel (one workgroup per
// copy). The mother itself is not changed.
struct Replicas {
    Scratch* sc = nullptr;
    std::vector<MotherLaunch> ls;
    double* rep = nullptr;
    int32_t count = 0;
    ~Replicas() { delete sc; }

    int32_t start(ttcf_ctx* c, Mother& m, int32_t n_rep, const double* kicks, int64_t decorrelate) {
        const int n = m.dev.n;
        const size_t sz = 6 * (size_t)n;
        sc = new Scratch(c->stream);
        rep = sc->get<double>(sz * n_rep + n_rep);
        double* kick_d = kicks ? sc->get<double>(3 * (size_t)n * n_rep) : nullptr;
        if (!rep || (kicks && !kick_d)) return fail(c, TTCF_ENOMEM, "replica allocation failed");
        double* zrep = rep + sz * n_rep;
        if (kicks)
            HIPCHECK(c, hipMemcpyAsync(kick_d, kicks, sizeof(double) * 3 * (size_t)n * n_rep,
                                       hipMemcpyHostToDevice, c->stream));
        HIPCHECK(c, launch_replicate(m.state, m.zeta, n, kick_d, n_rep, rep, zrep, c->stream));
        count = n_rep;
        ls.assign(n_rep, MotherLaunch{});
        const double nf = 3.0 * n - 3.0;
        for (int r = 0; r < n_rep; ++r) {
            MotherLaunch& L = ls[r];
            L.sys = m.dev;
            L.state = rep + sz * r;
            L.zeta = zrep + r;
            L.temperature = m.sys.temperature;
            L.nf = nf;
            L.q = nf * m.sys.temperature * m.sys.nh_tau * m.sys.nh_tau;
            L.threads = m.threads;
            L.apt = m.apt;
            L.precision = m.sys.precision;
            L.lds_bytes = lds_for(m.dev, m.sys.precision);
        }
        if (decorrelate > 0) return run(c, 0, decorrelate, nullptr);
        return TTCF_OK;
    }

    // every copy: n_chunks times {steps steps; snapshot into snaps (copy-major), and its
    // thermostat variable into zsnaps}
    int32_t run(ttcf_ctx* c, int64_t n_chunks, int64_t steps, double* snaps,
                double* zsnaps = nullptr) {
        const size_t sz = 6 * (size_t)ls[0].sys.n;
        for (int r = 0; r < count; ++r) {
            ls[r].n_chunks = n_chunks;
            ls[r].steps_per_chunk = steps;
            ls[r].snapshots = snaps ? snaps + sz * (size_t)r * (size_t)n_chunks : nullptr;
            ls[r].snap_zeta = zsnaps ? zsnaps + (size_t)r * (size_t)n_chunks : nullptr;
        }
        int32_t rc = upload_mother_launches(c, ls.data(), count);
        if (rc != TTCF_OK) return rc;
        HIPCHECK(c, launch_mothers(c->d_mlaunch, count, ls[0], c->stream));
        return TTCF_OK;
    }

    int32_t sample(ttcf_ctx* c, int32_t per_copy, int64_t between, double* snaps,
                   double* zsnaps = nullptr) {
        return run(c, per_copy, between, snaps, zsnaps);
    }
};

}  // namespace

extern "C" int32_t ttcf_sample_states_replicated(ttcf_ctx* c, int32_t mother, int32_t n_replicas,
                                                 const double* kicks, int64_t decorrelate_steps,
                                                 int32_t states_per_replica, int64_t steps_between) {
    if (!c || mother < 0 || mother >= (int32_t)c->mothers.size() || n_replicas <= 0 ||
        states_per_replica <= 0 || steps_between <= 0 || decorrelate_steps < 0)
        return TTCF_EINVAL;
    Mother& m = c->mothers[mother];
    const int64_t total = (int64_t)n_replicas * states_per_replica;
    if (total > (int64_t)1 << 24) return fail(c, TTCF_EINVAL, "too many states");
    const size_t n = (size_t)m.dev.n;
    if (m.states_cap < total) {
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        dev_free(m.states);
        m.states = (double*)dev_alloc(state_buffer_bytes((int)n, (int)total), c->stream);
        m.states_cap = m.states ? total : 0;
        m.n_states = 0;
        if (!m.states) return fail(c, TTCF_ENOMEM, "state buffer allocation failed");
    }
    Replicas R;
    int32_t rc = R.start(c, m, n_replicas, kicks, decorrelate_steps);
    if (rc == TTCF_OK) rc = R.sample(c, states_per_replica, steps_between, m.states, zetas_of(m));
    if (rc != TTCF_OK) return rc;
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    m.n_states = (int32_t)total;
    return TTCF_OK;
}

// ---- learned control variate -------------------------------------------------------------

namespace {

// parameter offsets: W1 [kCvIn x H], b1 [H], W2 [H x H], b2 [H], W3 [H x n_out], b3 [n_out]
struct CvLayout {
    int64_t w1, b1, w2, b2, w3, b3, total;
};

CvLayout cv_layout(int n_out) {
    CvLayout l;
    const int64_t H = kCvHidden;
    l.w1 = 0;
    l.b1 = l.w1 + (int64_t)kCvIn * H;
    l.w2 = l.b1 + H;
    l.b2 = l.w2 + H * H;
    l.w3 = l.b2 + H;
    l.b3 = l.w3 + H * n_out;
    l.total = l.b3 + n_out;
    return l;
}

// Scratch of one forward/backward pass over `rows` samples.
struct CvWork {
    float *x, *t, *z1, *a1, *z2, *a2, *y, *dy, *dz2, *dz1;
    double* loss;
    void* base = nullptr;
};

int32_t cv_work_alloc(ttcf_ctx* c, int rows, CvWork* w) {
    const int H = kCvHidden, O = c->cv_out;
    const size_t f = (size_t)rows * (kCvIn + O + 4 * H + 2 * O + 2 * H) + 64;
    w->base = dev_alloc(sizeof(float) * f + 64, c->stream);
    if (!w->base) return fail(c, TTCF_ENOMEM, "network scratch allocation failed");
    float* p = (float*)w->base;
    w->x = p; p += (size_t)rows * kCvIn;
    w->t = p; p += (size_t)rows * O;
    w->z1 = p; p += (size_t)rows * H;
    w->a1 = p; p += (size_t)rows * H;
    w->z2 = p; p += (size_t)rows * H;
    w->a2 = p; p += (size_t)rows * H;
    w->y = p; p += (size_t)rows * O;
    w->dy = p; p += (size_t)rows * O;
    w->dz2 = p; p += (size_t)rows * H;
    w->dz1 = p; p += (size_t)rows * H;
    w->loss = (double*)(((uintptr_t)p + 15) & ~(uintptr_t)15);
    return TTCF_OK;
}

GemmArgs gemm(const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk, int64_t sbn,
              float* C, int ldc, int M, int N, int K, int epi, const float* bias = nullptr,
              float* Z = nullptr, const float* Zin = nullptr) {
    GemmArgs g{};
    g.A = A;
    g.sam = sam;
    g.sak = sak;
    g.B = B;
    g.sbk = sbk;
    g.sbn = sbn;
    g.C = C;
    g.ldc = ldc;
    g.bias = bias;
    g.Z = Z;
    g.Zin = Zin;
    g.M = M;
    g.N = N;
    g.K = K;
    g.epi = epi;
    return g;
}

// y = W3 gelu(W2 gelu(W1 x + b1) + b2) + b3 for w.x (rows x kCvIn)
int32_t cv_forward(ttcf_ctx* c, const float* P, CvWork& w, int rows) {
    const int H = kCvHidden, O = c->cv_out;
    const CvLayout l = cv_layout(O);
    HIPCHECK(c, launch_gemm(gemm(w.x, kCvIn, 1, P + l.w1, H, 1, w.a1, H, rows, H, kCvIn, 1, P + l.b1, w.z1),
                            c->stream));
    HIPCHECK(c, launch_gemm(gemm(w.a1, H, 1, P + l.w2, H, 1, w.a2, H, rows, H, H, 1, P + l.b2, w.z2),
                            c->stream));
    HIPCHECK(c, launch_gemm(gemm(w.a2, H, 1, P + l.w3, O, 1, w.y, O, rows, O, H, 0, P + l.b3),
                            c->stream));
    return TTCF_OK;
}

// gradient of mean((y - t)^2) over every element into G
int32_t cv_backward(ttcf_ctx* c, const float* P, float* G, CvWork& w, int rows) {
    const int H = kCvHidden, O = c->cv_out;
    const CvLayout l = cv_layout(O);
    const int64_t cnt = (int64_t)rows * O;
    HIPCHECK(c, launch_mse_grad(w.y, w.t, cnt, 2.0f / (float)cnt, w.dy, c->stream));
    // W3: a2^T dy; b3: column sums of dy; dz2 = (dy W3^T) gelu'(z2)
    HIPCHECK(c, launch_gemm(gemm(w.a2, 1, H, w.dy, O, 1, G + l.w3, O, H, O, rows, 0), c->stream));
    HIPCHECK(c, launch_colsum(w.dy, rows, O, O, G + l.b3, c->stream));
    HIPCHECK(c, launch_gemm(gemm(w.dy, O, 1, P + l.w3, 1, O, w.dz2, H, rows, H, O, 2, nullptr, nullptr, w.z2),
                            c->stream));
    HIPCHECK(c, launch_gemm(gemm(w.a1, 1, H, w.dz2, H, 1, G + l.w2, H, H, H, rows, 0), c->stream));
    HIPCHECK(c, launch_colsum(w.dz2, rows, H, H, G + l.b2, c->stream));
    HIPCHECK(c, launch_gemm(gemm(w.dz2, H, 1, P + l.w2, 1, H, w.dz1, H, rows, H, H, 2, nullptr, nullptr, w.z1),
                            c->stream));
    HIPCHECK(c, launch_gemm(gemm(w.x, 1, kCvIn, w.dz1, H, 1, G + l.w1, H, kCvIn, H, rows, 0), c->stream));
    HIPCHECK(c, launch_colsum(w.dz1, rows, H, H, G + l.b1, c->stream));
    return TTCF_OK;
}

int32_t cv_check(ttcf_ctx* c) {
    if (!c) return TTCF_EINVAL;
    if (!c->cv_p) return fail(c, TTCF_ESTATE, "the control-variate network is not initialised");
    return TTCF_OK;
}

// Features, P_xy(0) and Omega(0) of live daughters [first, first + count): rows of kCvIn
// floats; with d_targets != null also B(t_1..t_nout) of each daughter (FP32). Returns the
// index of the first daughter in the live list through *i0_out.
int32_t cv_features_of(ttcf_ctx* c, int64_t first, int32_t count, float* d_feat, double* d_b0,
                       double* d_om, float* d_targets, int32_t n_out, int32_t* i0_out) {
    int32_t rc = sync_descs(c);
    if (rc != TTCF_OK) return rc;
    const int32_t i0 = find_live(c, first);
    if (i0 < 0 || i0 + count > (int32_t)c->live.size() ||
        c->live[i0 + count - 1].id != first + count - 1)
        return fail(c, TTCF_EINVAL, "the daughters must be live and consecutive");
    const int mother = c->batches[c->live[i0].batch].mother;
    Mother& m = c->mothers[mother];
    std::vector<int32_t> idx(2 * (size_t)count);
    std::vector<const double*> ser(count);
    for (int32_t q = 0; q < count; ++q) {
        const int32_t i = i0 + q;
        if (c->batches[c->live[i].batch].mother != mother)
            return fail(c, TTCF_EINVAL, "daughters of one call must share a mother");
        const DaughterDesc& d = c->descs[i];
        if (d.field != kFieldShear)
            return fail(c, TTCF_EINVAL, "the learned control variate serves shear daughters");
        if (d.done < std::max(1, n_out))
            return fail(c, TTCF_ESTATE, "the daughters have not been stepped far enough");
        if (c->live[i].state >= m.n_states)
            return fail(c, TTCF_ESTATE, "the mother's stored states were replaced");
        idx[q] = c->live[i].state;
        idx[count + q] = d.map;
        ser[q] = d.series;
    }
    Scratch sc(c->stream);
    double* d_vp = sc.get<double>(count);
    int32_t* d_idx = sc.get<int32_t>(2 * (size_t)count);
    const double** d_ser = sc.get<const double*>(count);
    if (!d_vp || !d_idx || !d_ser) return fail(c, TTCF_ENOMEM, "feature scratch allocation failed");
    HIPCHECK(c, hipMemcpyAsync(d_idx, idx.data(), sizeof(int32_t) * idx.size(), hipMemcpyHostToDevice,
                               c->stream));
    HIPCHECK(c, hipMemcpyAsync(d_ser, ser.data(), sizeof(double*) * count, hipMemcpyHostToDevice,
                               c->stream));
    HIPCHECK(c, launch_cv_gather_series(d_ser, count, n_out, 1.0 / m.dev.volume, d_targets, d_vp,
                                        c->stream));
    if (lds_bytes_cv_features(m.dev.n) > c->max_lds)
        return fail(c, TTCF_EINVAL, "system too large for the control-variate features");
    HIPCHECK(c, launch_cv_features(m.states, m.dev.n, d_idx, d_idx + count, d_vp, nullptr, count,
                                   m.dev.box, m.dev.rc2, m.dev.c_attr, m.dev.volume,
                                   m.sys.temperature, c->descs[i0].gamma_dot, d_feat, d_b0, d_om,
                                   c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    if (i0_out) *i0_out = i0;
    return TTCF_OK;
}

// Standardised-network predictions of B(t_1..t_nout) for raw feature rows, then h rows.
int32_t cv_predict_h(ttcf_ctx* c, const float* d_feat, const double* d_b0, const double* d_om,
                     int rows, double dt, double* d_h, int64_t h_stride) {
    const int O = c->cv_out;
    const float* xs = c->cv_stats;
    const float* ys = c->cv_stats + 2 * kCvIn;
    const int chunk = 65536;
    CvWork w;
    int32_t rc = cv_work_alloc(c, std::min(rows, chunk), &w);
    if (rc != TTCF_OK) return rc;
    for (int r0 = 0; r0 < rows; r0 += chunk) {
        const int nr = std::min(chunk, rows - r0);
        HIPCHECK(c, launch_gather_norm(d_feat + (size_t)r0 * kCvIn, nullptr, nr, kCvIn, xs, xs + kCvIn,
                                       w.x, c->stream));
        rc = cv_forward(c, c->cv_p, w, nr);
        if (rc != TTCF_OK) return rc;
        HIPCHECK(c, launch_cv_h(w.y, nr, O, ys, ys + O, d_b0 + r0, d_om + r0, dt,
                                d_h + (size_t)r0 * h_stride, h_stride, c->stream));
    }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    dev_free(w.base);
    return TTCF_OK;
}

}  // namespace

extern "C" {

int32_t ttcf_cv_init(ttcf_ctx* c, int32_t n_out, const float* weights, int64_t n_weights) {
    if (!c || n_out <= 0 || n_out > 4096 || !weights) return TTCF_EINVAL;
    const CvLayout l = cv_layout(n_out);
    if (n_weights != l.total) return fail(c, TTCF_EINVAL, "weight count does not match the network");
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    dev_free(c->cv_p);
    dev_free(c->cv_stats);
    dev_free(c->cv_mu);
    c->cv_out = n_out;
    c->cv_nparam = l.total;
    c->cv_p = (float*)dev_alloc(sizeof(float) * 4 * l.total, c->stream);
    c->cv_stats = (float*)dev_alloc(sizeof(float) * (2 * kCvIn + 2 * n_out), c->stream);
    c->cv_mu = (double*)dev_alloc(sizeof(double) * 4 * (n_out + 1), c->stream);
    if (!c->cv_p || !c->cv_stats || !c->cv_mu) return fail(c, TTCF_ENOMEM, "network allocation failed");
    c->cv_g = c->cv_p + l.total;
    c->cv_m = c->cv_g + l.total;
    c->cv_v = c->cv_m + l.total;
    HIPCHECK(c, hipMemcpyAsync(c->cv_p, weights, sizeof(float) * l.total, hipMemcpyHostToDevice, c->stream));
    std::vector<float> zeros(2 * l.total, 0.0f);
    HIPCHECK(c, hipMemcpyAsync(c->cv_m, zeros.data(), sizeof(float) * 2 * l.total, hipMemcpyHostToDevice,
                               c->stream));
    std::vector<float> st(2 * kCvIn + 2 * n_out);
    for (int i = 0; i < kCvIn; ++i) st[i] = 0.f, st[kCvIn + i] = 1.f;
    for (int i = 0; i < n_out; ++i) st[2 * kCvIn + i] = 0.f, st[2 * kCvIn + n_out + i] = 1.f;
    HIPCHECK(c, hipMemcpyAsync(c->cv_stats, st.data(), sizeof(float) * st.size(), hipMemcpyHostToDevice,
                               c->stream));
    std::vector<double> mz(4 * (n_out + 1), 0.0);
    HIPCHECK(c, hipMemcpyAsync(c->cv_mu, mz.data(), sizeof(double) * mz.size(), hipMemcpyHostToDevice,
                               c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    c->cv_adam_steps = 0;
    c->cv_stats_ready = false;
    c->cv_mu_count = 0;
    c->cv_rows = 0;
    c->cv_beta.clear();
    c->cv_beta_gamma = 0.0;
    return TTCF_OK;
}

int32_t ttcf_cv_export_weights(ttcf_ctx* c, float* weights, int64_t n_weights) {
    int32_t rc = cv_check(c);
    if (rc != TTCF_OK) return rc;
    if (!weights || n_weights != c->cv_nparam) return TTCF_EINVAL;
    HIPCHECK(c, hipMemcpyAsync(weights, c->cv_p, sizeof(float) * n_weights, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return TTCF_OK;
}

int32_t ttcf_mlp_forward(ttcf_ctx* c, const float* x, int32_t rows, float* y) {
    int32_t rc = cv_check(c);
    if (rc != TTCF_OK) return rc;
    if (!x || !y || rows <= 0) return TTCF_EINVAL;
    CvWork w;
    rc = cv_work_alloc(c, rows, &w);
    if (rc != TTCF_OK) return rc;
    HIPCHECK(c, hipMemcpyAsync(w.x, x, sizeof(float) * rows * kCvIn, hipMemcpyHostToDevice, c->stream));
    rc = cv_forward(c, c->cv_p, w, rows);
    if (rc != TTCF_OK) return rc;
    HIPCHECK(c, hipMemcpyAsync(y, w.y, sizeof(float) * rows * c->cv_out, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    dev_free(w.base);
    return TTCF_OK;
}

int32_t ttcf_mlp_gradient(ttcf_ctx* c, const float* x, const float* target, int32_t rows,
                          float* grad) {
    int32_t rc = cv_check(c);
    if (rc != TTCF_OK) return rc;
    if (!x || !target || !grad || rows <= 0) return TTCF_EINVAL;
    CvWork w;
    rc = cv_work_alloc(c, rows, &w);
    if (rc != TTCF_OK) return rc;
    HIPCHECK(c, hipMemcpyAsync(w.x, x, sizeof(float) * rows * kCvIn, hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipMemcpyAsync(w.t, target, sizeof(float) * rows * c->cv_out, hipMemcpyHostToDevice,
                               c->stream));
    rc = cv_forward(c, c->cv_p, w, rows);
    if (rc == TTCF_OK) rc = cv_backward(c, c->cv_p, c->cv_g, w, rows);
    if (rc != TTCF_OK) return rc;
    HIPCHECK(c, hipMemcpyAsync(grad, c->cv_g, sizeof(float) * c->cv_nparam, hipMemcpyDeviceToHost,
                               c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    dev_free(w.base);
    return TTCF_OK;
}

int32_t ttcf_cv_add_training(ttcf_ctx* c, int64_t first, int32_t count) {
    int32_t rc = cv_check(c);
    if (rc != TTCF_OK) return rc;
    if (count <= 0) return TTCF_EINVAL;
    const int O = c->cv_out;
    if (c->cv_rows + count > c->cv_cap) {
        const int64_t cap = std::max<int64_t>(c->cv_rows + count, 2 * c->cv_cap);
        float* nx = (float*)dev_alloc(sizeof(float) * cap * kCvIn, c->stream);
        float* nt = (float*)dev_alloc(sizeof(float) * cap * O, c->stream);
        if (!nx || !nt) {
            dev_free(nx);
            dev_free(nt);
            return fail(c, TTCF_ENOMEM, "training-set allocation failed");
        }
        if (c->cv_rows > 0) {
            HIPCHECK(c, hipMemcpyAsync(nx, c->cv_x, sizeof(float) * c->cv_rows * kCvIn,
                                       hipMemcpyDeviceToDevice, c->stream));
            HIPCHECK(c, hipMemcpyAsync(nt, c->cv_t, sizeof(float) * c->cv_rows * O,
                                       hipMemcpyDeviceToDevice, c->stream));
        }
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        dev_free(c->cv_x);
        dev_free(c->cv_t);
        c->cv_x = nx;
        c->cv_t = nt;
        c->cv_cap = cap;
    }
    Scratch sc(c->stream);
    double* tmp = sc.get<double>(2 * (size_t)count);
    if (!tmp) return fail(c, TTCF_ENOMEM, "scratch allocation failed");
    rc = cv_features_of(c, first, count, c->cv_x + c->cv_rows * kCvIn, tmp, tmp + count,
                        c->cv_t + c->cv_rows * O, O, nullptr);
    if (rc != TTCF_OK) return rc;
    c->cv_rows += count;
    c->cv_stats_ready = false;
    return TTCF_OK;
}

int32_t ttcf_cv_export_training(ttcf_ctx* c, int64_t first_row, int32_t count, float* x, float* t) {
    int32_t rc = cv_check(c);
    if (rc != TTCF_OK) return rc;
    if (first_row < 0 || count <= 0 || first_row + count > c->cv_rows) return TTCF_EINVAL;
    if (x)
        HIPCHECK(c, hipMemcpyAsync(x, c->cv_x + first_row * kCvIn, sizeof(float) * count * kCvIn,
                                   hipMemcpyDeviceToHost, c->stream));
    if (t)
        HIPCHECK(c, hipMemcpyAsync(t, c->cv_t + first_row * c->cv_out,
                                   sizeof(float) * count * c->cv_out, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return TTCF_OK;
}

int32_t ttcf_cv_train(ttcf_ctx* c, int32_t epochs, int32_t batch, double lr, const int32_t* order,
                      double* loss_out) {
    int32_t rc = cv_check(c);
    if (rc != TTCF_OK) return rc;
    if (epochs < 0 || batch <= 0 || !(lr > 0.0)) return TTCF_EINVAL;
    if (c->cv_rows < batch) return fail(c, TTCF_ESTATE, "fewer training samples than one batch");
    const int O = c->cv_out;
    const int64_t n = c->cv_rows;
    if (order)
        for (int64_t q = 0; q < (int64_t)epochs * n; ++q)
            if (order[q] < 0 || order[q] >= n) return fail(c, TTCF_EINVAL, "order index out of range");
    float* xs = c->cv_stats;
    float* ys = c->cv_stats + 2 * kCvIn;
    if (!c->cv_stats_ready) {
        HIPCHECK(c, launch_col_stats(c->cv_x, n, kCvIn, xs, xs + kCvIn, c->stream));
        HIPCHECK(c, launch_col_stats(c->cv_t, n, O, ys, ys + O, c->stream));
        c->cv_stats_ready = true;
    }
    CvWork w;
    rc = cv_work_alloc(c, batch, &w);
    if (rc != TTCF_OK) return rc;
    int32_t* d_idx = (int32_t*)dev_alloc(sizeof(int32_t) * n, c->stream);
    if (!d_idx) return fail(c, TTCF_ENOMEM, "index allocation failed");
    std::vector<int32_t> nat;
    if (!order) {
        nat.resize(n);
        for (int64_t q = 0; q < n; ++q) nat[q] = (int32_t)q;
    }
    const int64_t steps = n / batch;
    for (int32_t e = 0; e < epochs; ++e) {
        const int32_t* ord = order ? order + (int64_t)e * n : nat.data();
        HIPCHECK(c, hipMemcpyAsync(d_idx, ord, sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream));
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        for (int64_t s = 0; s < steps; ++s) {
            const int32_t* bi = d_idx + s * batch;
            HIPCHECK(c, launch_gather_norm(c->cv_x, bi, batch, kCvIn, xs, xs + kCvIn, w.x, c->stream));
            HIPCHECK(c, launch_gather_norm(c->cv_t, bi, batch, O, ys, ys + O, w.t, c->stream));
            rc = cv_forward(c, c->cv_p, w, batch);
            if (rc == TTCF_OK) rc = cv_backward(c, c->cv_p, c->cv_g, w, batch);
            if (rc != TTCF_OK) return rc;
            c->cv_adam_steps += 1;
            HIPCHECK(c, launch_adam(c->cv_p, c->cv_g, c->cv_m, c->cv_v, c->cv_nparam, (float)lr,
                                    c->cv_adam_steps, c->stream));
            if (s == steps - 1 && loss_out) {
                HIPCHECK(c, launch_mse_loss(w.y, w.t, (int64_t)batch * O, w.loss, c->stream));
                HIPCHECK(c, hipMemcpyAsync(loss_out + e, w.loss, sizeof(double), hipMemcpyDeviceToHost,
                                           c->stream));
            }
        }
    }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    dev_free(d_idx);
    dev_free(w.base);
    return TTCF_OK;
}

int32_t ttcf_cv_attach(ttcf_ctx* c, int64_t first, int32_t count, int32_t role) {
    int32_t rc = cv_check(c);
    if (rc != TTCF_OK) return rc;
    if (count <= 0 || (role != TTCF_CV_ESTIMATE && role != TTCF_CV_CALIBRATE)) return TTCF_EINVAL;
    if (!c->cv_stats_ready) return fail(c, TTCF_ESTATE, "train the network before attaching it");
    const int O = c->cv_out;
    Scratch sc(c->stream);
    float* feat = sc.get<float>((size_t)count * kCvIn);
    double* b0 = sc.get<double>(2 * (size_t)count);
    double* hrow = sc.get<double>((size_t)count * (O + 1));
    double** dst = sc.get<double*>(count);
    int32_t* nk = sc.get<int32_t>(count);
    if (!feat || !b0 || !hrow || !dst || !nk) return fail(c, TTCF_ENOMEM, "feature allocation failed");
    double* om = b0 + count;
    int32_t i0 = 0;
    rc = cv_features_of(c, first, count, feat, b0, om, nullptr, 0, &i0);
    if (rc != TTCF_OK) return rc;
    rc = cv_predict_h(c, feat, b0, om, count, c->descs[i0].sys.dt, hrow, O + 1);
    if (rc != TTCF_OK) return rc;
    // each daughter's h series lives in its batch's buffer, laid out like the B series; h is
    // zero past t_K
    std::vector<double*> dh(count);
    std::vector<int32_t> nh(count);
    for (int32_t q = 0; q < count; ++q) {
        const int32_t i = i0 + q;
        Batch& b = c->batches[c->live[i].batch];
        const size_t len = (size_t)b.n_steps + 1;
        if (!b.hseries) {
            b.hseries = (double*)dev_alloc(sizeof(double) * len * b.n_daughters, c->stream);
            if (!b.hseries) return fail(c, TTCF_ENOMEM, "h series allocation failed");
            HIPCHECK(c, launch_fill_f64(b.hseries, 0.0, (int64_t)len * b.n_daughters, c->stream));
        }
        dh[q] = b.hseries + len * c->live[i].index;
        nh[q] = std::min(b.n_steps, O) + 1;
        c->descs[i].hseries = dh[q];
        c->live[i].cv_role = role;
    }
    HIPCHECK(c, hipMemcpyAsync(dst, dh.data(), sizeof(double*) * count, hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipMemcpyAsync(nk, nh.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, launch_cv_scatter_h(hrow, O + 1, count, dst, nk, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return push_descs(c);
}

int32_t ttcf_cv_mean_term(ttcf_ctx* c, int32_t mother, int32_t n_replicas, const double* kicks,
                          int64_t decorrelate_steps, int32_t rounds, int32_t states_per_replica,
                          int64_t steps_between, double gamma_dot, int64_t* out_samples) {
    int32_t rc = cv_check(c);
    if (rc != TTCF_OK) return rc;
    if (mother < 0 || mother >= (int32_t)c->mothers.size() || n_replicas <= 0 || rounds <= 0 ||
        states_per_replica <= 0 || steps_between <= 0 || decorrelate_steps < 0 ||
        !std::isfinite(gamma_dot))
        return TTCF_EINVAL;
    if (!c->cv_stats_ready) return fail(c, TTCF_ESTATE, "train the network before the mean term");
    if (c->cv_mu_count > 0 && gamma_dot != c->cv_mu_gamma)
        return fail(c, TTCF_EINVAL, "the mean term already holds samples at another shear rate");
    Mother& m = c->mothers[mother];
    const int n = m.dev.n, O = c->cv_out;
    if (lds_bytes_cv_features_maps(n) > c->max_lds)
        return fail(c, TTCF_EINVAL, "system too large for the control-variate features");
    const int64_t per_round = (int64_t)n_replicas * states_per_replica;
    if (per_round * 4 > (1 << 22)) return fail(c, TTCF_EINVAL, "too many samples per round");
    Scratch sc(c->stream);
    const size_t sz = 6 * (size_t)n;
    double* snaps = sc.get<double>(sz * per_round);
    double* vp = sc.get<double>(per_round);
    const int rows = (int)(4 * per_round);
    float* feat = sc.get<float>((size_t)rows * kCvIn);
    double* b0 = sc.get<double>(2 * (size_t)rows);
    double* hh = sc.get<double>((size_t)rows * (O + 1));
    double* sgn = sc.get<double>(4);
    double* mu_part = sc.get<double>(cv_mu_scratch_doubles(O + 1));
    if (!snaps || !vp || !feat || !b0 || !hh || !sgn || !mu_part)
        return fail(c, TTCF_ENOMEM, "mean-term allocation failed");
    const double sgn_h[4] = {1.0, 1.0, -1.0, -1.0};  // sign of P_xy(0) under each mapping
    HIPCHECK(c, hipMemcpyAsync(sgn, sgn_h, sizeof(sgn_h), hipMemcpyHostToDevice, c->stream));
    Replicas R;
    rc = R.start(c, m, n_replicas, kicks, decorrelate_steps);
    if (rc != TTCF_OK) return rc;
    for (int32_t round = 0; round < rounds; ++round) {
        rc = R.sample(c, states_per_replica, steps_between, snaps);
        if (rc != TTCF_OK) return rc;
        HIPCHECK(c, launch_states_vpxy(m.dev, snaps, (int32_t)per_round, vp, c->stream));
        HIPCHECK(c, launch_cv_features_maps(snaps, n, (int32_t)per_round, vp, sgn, m.dev.box,
                                            m.dev.rc2, m.dev.c_attr, m.dev.volume,
                                            m.sys.temperature, gamma_dot, feat, b0, b0 + rows,
                                            c->stream));
        rc = cv_predict_h(c, feat, b0, b0 + rows, rows, m.dev.dt, hh, O + 1);
        if (rc != TTCF_OK) return rc;
        HIPCHECK(c, launch_cv_mu_accum(hh, (int)per_round, 4, O + 1, c->cv_mu, c->cv_mu + (O + 1),
                                       c->cv_mu + 2 * (O + 1), c->cv_mu + 3 * (O + 1), mu_part,
                                       c->stream));
    }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    c->cv_mu_count += per_round * rounds;
    c->cv_mu_dt = m.dev.dt;
    c->cv_mu_gamma = gamma_dot;
    if (out_samples) *out_samples = c->cv_mu_count;
    return TTCF_OK;
}

int32_t ttcf_cv_calibrate(ttcf_ctx* c, double gamma_dot_filter, int32_t n_t, double* beta) {
    int32_t rc = cv_check(c);
    if (rc != TTCF_OK) return rc;
    rc = refresh_row_health(c);
    if (rc != TTCF_OK) return rc;
    if (n_t <= 0 || n_t > c->cv_out + 1) return fail(c, TTCF_EINVAL, "n_t beyond the network's grid");
    std::vector<int32_t> rows;
    for (int64_t r = 0; r < c->acc_rows; ++r) {
        if (c->row_cv[r] != TTCF_CV_CALIBRATE || c->row_health[r] != 0) continue;
        if (c->row_gamma[r] != gamma_dot_filter || c->row_nt[r] < n_t) continue;
        rows.push_back((int32_t)r);
    }
    if (rows.size() < 2) return fail(c, TTCF_ESTATE, "fewer than two calibration groups");
    Scratch sc(c->stream);
    double* d_beta = sc.get<double>(n_t);
    int32_t* d_rows = sc.get<int32_t>(rows.size());
    if (!d_beta || !d_rows) return fail(c, TTCF_ENOMEM, "calibration scratch allocation failed");
    HIPCHECK(c, hipMemcpyAsync(d_rows, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice,
                               c->stream));
    HIPCHECK(c, hipMemcpyAsync(c->d_row_health, c->row_health.data(), sizeof(int32_t) * c->row_health.size(),
                               hipMemcpyHostToDevice, c->stream));
    ResponseLaunch R{};
    R.d_all = c->acc_d;
    R.i_all = c->acc_i;
    R.gamma = c->d_row_gamma;
    R.coef = c->d_row_coef;
    R.health = c->d_row_health;
    R.rows = d_rows;
    R.n_rows = (int32_t)rows.size();
    R.n_t = n_t;
    R.n_t_stride = c->acc_stride;
    R.h_all = c->acc_h;
    HIPCHECK(c, launch_cv_beta(R, d_beta, c->stream));
    std::vector<double> bb(n_t);
    HIPCHECK(c, hipMemcpyAsync(bb.data(), d_beta, sizeof(double) * n_t, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    c->cv_beta = bb;
    c->cv_beta_gamma = gamma_dot_filter;
    if (beta) std::memcpy(beta, bb.data(), sizeof(double) * n_t);
    return TTCF_OK;
}

int32_t ttcf_cv_response(ttcf_ctx* c, double gamma_dot_filter, int32_t n_t, double* cv_mean,
                         double* cv_se, double* plain_mean, double* plain_se, double* mu_h,
                         double* mu_h_se, int64_t* out_n_states) {
    int32_t rc = cv_check(c);
    if (rc != TTCF_OK) return rc;
    rc = refresh_row_health(c);
    if (rc != TTCF_OK) return rc;
    if (n_t <= 0 || n_t > c->cv_out + 1) return fail(c, TTCF_EINVAL, "n_t beyond the network's grid");
    if (c->cv_mu_count < 2) return fail(c, TTCF_ESTATE, "no mean term: call ttcf_cv_mean_term");
    if (!(gamma_dot_filter > 0.0) || gamma_dot_filter != c->cv_mu_gamma)
        return fail(c, TTCF_EINVAL, "the filter must be the shear rate of the mean term");
    std::vector<int32_t> rows;
    for (int64_t r = 0; r < c->acc_rows; ++r) {
        if (c->row_cv[r] != TTCF_CV_ESTIMATE || c->row_health[r] != 0) continue;
        if (c->row_gamma[r] != gamma_dot_filter) continue;
        if (c->row_nt[r] < n_t) continue;
        rows.push_back((int32_t)r);
    }
    if (rows.size() < 2) return fail(c, TTCF_ESTATE, "fewer than two groups carry the control variate");
    const bool calibrated = c->cv_beta_gamma == gamma_dot_filter && (int32_t)c->cv_beta.size() >= n_t;
    // mean term per time point from its compensated sums
    const int K = c->cv_out + 1;
    std::vector<double> mu(4 * (size_t)K);
    HIPCHECK(c, hipMemcpyAsync(mu.data(), c->cv_mu, sizeof(double) * mu.size(), hipMemcpyDeviceToHost,
                               c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    std::vector<double> muv(K), muse(K);
    const double cnt = (double)c->cv_mu_count;
    for (int k = 0; k < K; ++k) {
        const double sm = mu[k] + mu[K + k], s2 = mu[2 * K + k] + mu[3 * K + k];
        muv[k] = sm / cnt;
        const double var = (s2 - sm * sm / cnt) / (cnt - 1.0);
        muse[k] = std::sqrt(std::max(var, 0.0) / cnt);
    }
    if (calibrated)
        for (int k = 0; k < n_t; ++k) {
            muv[k] *= c->cv_beta[k];
            muse[k] *= std::fabs(c->cv_beta[k]);
        }
    Scratch sc(c->stream);
    double* d_mu = sc.get<double>(K);
    double* d_beta = sc.get<double>(K);
    double* d_out = sc.get<double>(8 * (size_t)n_t);
    int32_t* d_used = sc.get<int32_t>(2);
    int32_t* d_rows = sc.get<int32_t>(rows.size());
    if (!d_mu || !d_beta || !d_out || !d_used || !d_rows)
        return fail(c, TTCF_ENOMEM, "response scratch allocation failed");
    // the kernel adds beta * mu: pass mu_H itself and beta (1 when uncalibrated)
    {
        std::vector<double> bb(K, 1.0), mraw(K);
        for (int k = 0; k < K; ++k) mraw[k] = mu[k] + mu[K + k];
        for (int k = 0; k < K; ++k) mraw[k] /= cnt;
        if (calibrated)
            for (int k = 0; k < n_t; ++k) bb[k] = c->cv_beta[k];
        HIPCHECK(c, hipMemcpyAsync(d_mu, mraw.data(), sizeof(double) * K, hipMemcpyHostToDevice, c->stream));
        HIPCHECK(c, hipMemcpyAsync(d_beta, bb.data(), sizeof(double) * K, hipMemcpyHostToDevice, c->stream));
        HIPCHECK(c, hipStreamSynchronize(c->stream));
    }
    HIPCHECK(c, hipMemcpyAsync(d_rows, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice,
                               c->stream));
    HIPCHECK(c, hipMemcpyAsync(c->d_row_health, c->row_health.data(), sizeof(int32_t) * c->row_health.size(),
                               hipMemcpyHostToDevice, c->stream));
    ResponseLaunch R{};
    R.d_all = c->acc_d;
    R.i_all = c->acc_i;
    R.gamma = c->d_row_gamma;
    R.coef = c->d_row_coef;
    R.health = c->d_row_health;
    R.rows = d_rows;
    R.n_rows = (int32_t)rows.size();
    R.n_t = n_t;
    R.n_t_stride = c->acc_stride;
    R.normalise = 0;
    // the plain estimate over the same groups, then the control-variate one
    R.out = d_out + 4 * (size_t)n_t;
    R.used = d_used + 1;
    HIPCHECK(c, launch_response(R, c->stream));
    R.h_all = c->acc_h;
    R.mu_h = d_mu;
    R.beta = d_beta;
    R.out = d_out;
    R.used = d_used;
    HIPCHECK(c, launch_response(R, c->stream));
    std::vector<double> out(8 * (size_t)n_t);
    int32_t used = 0;
    HIPCHECK(c, hipMemcpyAsync(out.data(), d_out, sizeof(double) * out.size(), hipMemcpyDeviceToHost,
                               c->stream));
    HIPCHECK(c, hipMemcpyAsync(&used, d_used, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    if (cv_mean) std::memcpy(cv_mean, out.data(), sizeof(double) * n_t);
    if (cv_se) std::memcpy(cv_se, out.data() + n_t, sizeof(double) * n_t);
    if (plain_mean) std::memcpy(plain_mean, out.data() + 4 * n_t, sizeof(double) * n_t);
    if (plain_se) std::memcpy(plain_se, out.data() + 5 * n_t, sizeof(double) * n_t);
    if (mu_h) std::memcpy(mu_h, muv.data(), sizeof(double) * n_t);
    if (mu_h_se) std::memcpy(mu_h_se, muse.data(), sizeof(double) * n_t);
    if (out_n_states) *out_n_states = used;
    return TTCF_OK;
}

}  // extern "C"

extern "C" {

// ---- stateless inspection kernels ---------------------------------------------------------

static int32_t debug_setup(const ttcf_system* sys, const double* r, SysDev* S, double** d_r,
                           hipStream_t s, int lds_precision) {
    std::string why;
    int32_t rc = build_sysdev(sys, S, &why);
    if (rc != TTCF_OK) return rc;
    if (pick_apt(S->n, pick_threads(S->n, 0)) < 0) return TTCF_EINVAL;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return TTCF_EDEVICE;
    if (lds_bytes_for(S->n, S->nc[0] * S->nc[1] * S->nc[2], 0, lds_precision) > prop.sharedMemPerBlock)
        return TTCF_EINVAL;
    for (int k = 0; k < 3 * S->n; ++k)
        if (!(r[k] >= 0.0 && r[k] < S->box[k / S->n])) return TTCF_EINVAL;
    *d_r = (double*)dev_alloc(sizeof(double) * 3 * S->n, s);
    if (!*d_r) return TTCF_ENOMEM;
    if (hipMemcpyAsync(*d_r, r, sizeof(double) * 3 * S->n, hipMemcpyHostToDevice, s) != hipSuccess)
        return TTCF_EDEVICE;
    return TTCF_OK;
}

int32_t ttcf_debug_cell_list(const ttcf_system* sys, const double* r, int32_t* dims,
                             int32_t* cell_of, int32_t* order, int32_t* start, void* stream) {
    if (!sys || !r || !cell_of || !order || !start) return TTCF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    SysDev S{};
    double* d_r = nullptr;
    int32_t rc = debug_setup(sys, r, &S, &d_r, s, TTCF_PREC_FP32_FORCES);
    if (rc != TTCF_OK) {
        dev_free(d_r);
        return rc;
    }
    const int C = S.nc[0] * S.nc[1] * S.nc[2];
    int32_t* buf = (int32_t*)dev_alloc(sizeof(int32_t) * (2 * S.n + C + 1), s);
    if (!buf) {
        dev_free(d_r);
        return TTCF_ENOMEM;
    }
    hipError_t e = launch_debug_cells(S, d_r, buf, buf + S.n, buf + 2 * S.n, s);
    if (e == hipSuccess) e = hipMemcpyAsync(cell_of, buf, sizeof(int32_t) * S.n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(order, buf + S.n, sizeof(int32_t) * S.n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(start, buf + 2 * S.n, sizeof(int32_t) * (C + 1), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dev_free(buf);
    dev_free(d_r);
    if (e != hipSuccess) return TTCF_EDEVICE;
    if (dims) {
        dims[0] = S.nc[0];
        dims[1] = S.nc[1];
        dims[2] = S.nc[2];
    }
    return TTCF_OK;
}

int32_t ttcf_debug_pairs(const ttcf_system* sys, double dxle, const double* r, double rlist,
                         int64_t cap, int32_t* pi, int32_t* pj, int64_t* count, void* stream) {
    if (!sys || !r || !pi || !pj || !count || cap < 0 || !(rlist > 0.0) || rlist > sys->r_cut)
        return TTCF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    SysDev S{};
    double* d_r = nullptr;
    int32_t rc = debug_setup(sys, r, &S, &d_r, s, TTCF_PREC_FP32_FORCES);
    if (rc != TTCF_OK) {
        dev_free(d_r);
        return rc;
    }
    const size_t cap_sz = (size_t)std::max<int64_t>(cap, 1);
    int32_t* buf = (int32_t*)dev_alloc(sizeof(int32_t) * 2 * cap_sz + 16, s);
    if (!buf) {
        dev_free(d_r);
        return TTCF_ENOMEM;
    }
    unsigned long long* d_cnt = (unsigned long long*)(buf + 2 * cap_sz);
    const unsigned long long zero = 0;
    hipError_t e = hipMemcpyAsync(d_cnt, &zero, sizeof(zero), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_debug_pairs(S, dxle, d_r, rlist, cap, buf, buf + cap_sz, d_cnt, s);
    unsigned long long cnt = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&cnt, d_cnt, sizeof(cnt), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && (int64_t)cnt <= cap) {
        std::vector<int32_t> a(cnt), b(cnt);
        e = hipMemcpyAsync(a.data(), buf, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(b.data(), buf + cap_sz, sizeof(int32_t) * cnt,
                                                hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        // the kernel emits pairs in arrival order; present them sorted by (i, j)
        std::vector<int64_t> key(cnt);
        for (size_t q = 0; q < cnt; ++q) key[q] = ((int64_t)a[q] << 32) | (int64_t)(uint32_t)b[q];
        std::sort(key.begin(), key.end());
        for (size_t q = 0; q < cnt; ++q) {
            pi[q] = (int32_t)(key[q] >> 32);
            pj[q] = (int32_t)(key[q] & 0xffffffff);
        }
    }
    dev_free(buf);
    dev_free(d_r);
    if (e != hipSuccess) return TTCF_EDEVICE;
    *count = (int64_t)cnt <= cap ? (int64_t)cnt : -1;
    return TTCF_OK;
}

int32_t ttcf_debug_forces(const ttcf_system* sys, double dxle, const double* r, double* f,
                          double* out, void* stream) {
    if (!sys || !r || !f || !out) return TTCF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    SysDev S{};
    double* d_r = nullptr;
    int32_t rc = debug_setup(sys, r, &S, &d_r, s, sys->precision);
    if (rc != TTCF_OK) {
        dev_free(d_r);
        return rc;
    }
    double* buf = (double*)dev_alloc(sizeof(double) * (3 * S.n + 2), s);
    if (!buf) {
        dev_free(d_r);
        return TTCF_ENOMEM;
    }
    hipError_t e = launch_debug_forces(S, sys->precision, dxle, d_r, buf, buf + 3 * S.n, s);
    if (e == hipSuccess) e = hipMemcpyAsync(f, buf, sizeof(double) * 3 * S.n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, buf + 3 * S.n, sizeof(double) * 2, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dev_free(buf);
    dev_free(d_r);
    return e == hipSuccess ? TTCF_OK : TTCF_EDEVICE;
}

int32_t ttcf_debug_pair_form(const ttcf_system* sys, double gamma_dot, int64_t kstep, double skin,
                             int32_t kcap, const double* r, int32_t* dims, int32_t* cell_of,
                             int32_t* order, int32_t* start, int64_t cap, int32_t* pi, int32_t* pj,
                             int64_t* count, double* f, double* out, void* stream) {
    if (!sys || !r || !cell_of || !order || !start || !pi || !pj || !count || !f || !out ||
        cap < 0 || kcap > kPairMaxCap || !std::isfinite(gamma_dot) || !std::isfinite(skin))
        return TTCF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    SysDev S{};
    std::string why;
    int32_t rc = build_sysdev(sys, &S, &why);
    if (rc != TTCF_OK) return rc;
    if (S.n > kPairMaxAtoms || !set_list_grid(&S, skin)) return TTCF_EINVAL;
    if (kcap <= 0) kcap = auto_pair_cap(S);
    const int C = S.lc[0] * S.lc[1] * S.lc[2];
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return TTCF_EDEVICE;
    if (lds_bytes_pairs(S.n, C) > prop.sharedMemPerBlock) return TTCF_EINVAL;
    for (int k = 0; k < 3 * S.n; ++k)
        if (!(r[k] >= 0.0 && r[k] < S.box[k / S.n])) return TTCF_EINVAL;
    const int n = S.n;
    const int waves = pair_job_threads(n) / 64;
    const int apt = pair_job_apt(n);
    const int64_t words = pair_words(n, kcap, apt);
    // device layout: r (3n doubles), f (3n), out (4); pairs (words), seg counts (waves),
    // cell_of, rank_of (n each), start (C + 1)
    const size_t dbytes = sizeof(double) * (6 * (size_t)n + 4);
    const size_t ibytes = sizeof(uint32_t) * ((size_t)words + waves + 2 * (size_t)n + C + 1);
    char* buf = (char*)dev_alloc(dbytes + ibytes, s);
    if (!buf) return TTCF_ENOMEM;
    double* d_r = (double*)buf;
    double* d_f = d_r + 3 * n;
    double* d_out = d_f + 3 * n;
    uint32_t* d_pairs = (uint32_t*)(buf + dbytes);
    int32_t* d_seg = (int32_t*)(d_pairs + words);
    int32_t* d_cell = d_seg + waves;
    int32_t* d_rank = d_cell + n;
    int32_t* d_start = d_rank + n;
    std::vector<uint32_t> words_h((size_t)words);
    std::vector<int32_t> seg(waves), rank(n);
    hipError_t e = hipMemcpyAsync(d_r, r, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_debug_pair_form(S, gamma_dot, kstep, d_r, kcap, d_pairs, d_seg, d_cell, d_rank,
                                   d_start, d_f, d_out, s);
    if (e == hipSuccess) e = hipMemcpyAsync(f, d_f, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s);
    double o3[3] = {0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(o3, d_out, sizeof(o3), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(words_h.data(), d_pairs, sizeof(uint32_t) * words, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(seg.data(), d_seg, sizeof(int32_t) * waves, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(cell_of, d_cell, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(rank.data(), d_rank, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(start, d_start, sizeof(int32_t) * (C + 1), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dev_free(buf);
    if (e != hipSuccess) return TTCF_EDEVICE;
    // ranks to atom ids: the build's order
    std::vector<int32_t> atom_of(n, -1);
    for (int a = 0; a < n; ++a) {
        if (rank[a] < 0 || rank[a] >= n || atom_of[rank[a]] != -1) return TTCF_EDEVICE;
        atom_of[rank[a]] = a;
    }
    for (int q = 0; q < n; ++q) order[q] = atom_of[q];
    const int64_t seg_cap = (int64_t)kcap * 64 * apt;
    bool overflow = false;
    std::vector<int64_t> key;
    for (int w = 0; w < waves; ++w) {
        if (seg[w] > seg_cap) overflow = true;
        const int64_t used = std::min<int64_t>(seg[w], seg_cap);
        for (int64_t q = 0; q < used; ++q) {
            const uint32_t word = words_h[(size_t)(w * seg_cap + q)];
            const int a = atom_of[word & 0x3FFFu], b = atom_of[(word >> 14) & 0x3FFFu];
            const int i = std::min(a, b), j = std::max(a, b);
            key.push_back(((int64_t)i << 32) | (int64_t)j);
        }
    }
    std::sort(key.begin(), key.end());
    if ((int64_t)key.size() <= cap)
        for (size_t q = 0; q < key.size(); ++q) {
            pi[q] = (int32_t)(key[q] >> 32);
            pj[q] = (int32_t)(key[q] & 0xffffffff);
        }
    *count = (int64_t)key.size() <= cap ? (int64_t)key.size() : -1;
    out[0] = o3[0];
    out[1] = o3[2];
    out[2] = S.rc + S.skin;
    out[3] = o3[1];
    if (dims) {
        dims[0] = S.lc[0];
        dims[1] = S.lc[1];
        dims[2] = S.lc[2];
    }
    return overflow ? TTCF_EUNSTABLE : TTCF_OK;
}

int32_t ttcf_cell_grid(const ttcf_system* sys, double skin, int32_t* cells, int32_t* list_cells,
                       double* list_skin) {
    if (!sys || !std::isfinite(skin)) return TTCF_EINVAL;
    SysDev S{};
    std::string why;
    int32_t rc = build_sysdev(sys, &S, &why);
    if (rc != TTCF_OK) return rc;
    if (cells)
        for (int a = 0; a < 3; ++a) cells[a] = S.nc[a];
    const bool ok = set_list_grid(&S, skin);
    if (list_cells)
        for (int a = 0; a < 3; ++a) list_cells[a] = ok ? S.lc[a] : 0;
    if (list_skin) *list_skin = ok ? S.skin : 0.0;
    return TTCF_OK;
}

}  // extern "C"

// ---- allocation-free pair-form forces ---------------------------------------------------

// The device scratch of ttcf_pair_forces_static: the pair lists and the build's by-products,
// one copy on every GPU the library runs on, held until the process ends. Host code uses it
// only through the address hipGetSymbolAddress returns on each device (the array's own name
// is a host-side stand-in, not a device address).
static __device__ __align__(256) uint32_t scratch[TTCF_STATIC_SCRATCH_BYTES / 4];

namespace {

constexpr int kStaticMaxDevices = 64;

struct StaticScratch {
    uint32_t* ptr = nullptr;  // this device's copy of `scratch`
    size_t lds = 0;           // its LDS per workgroup
};

std::mutex g_static_mu;
StaticScratch g_static[kStaticMaxDevices];

// The current device's scratch, looked up once per device (with that device current).
int32_t static_scratch(StaticScratch* out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kStaticMaxDevices)
        return TTCF_EDEVICE;
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticScratch& d = g_static[dev];
    if (!d.ptr) {
        void* ptr = nullptr;
        int lds = 0;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr ||
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess)
            return TTCF_EDEVICE;
        d.lds = (size_t)lds;
        d.ptr = (uint32_t*)ptr;
    }
    *out = d;
    return TTCF_OK;
}

inline int64_t words256(int64_t words) { return (words + 63) & ~int64_t(63); }

}  // namespace

extern "C" {

int32_t ttcf_pair_forces_static(const ttcf_system* sys, double gamma_dot, int64_t kstep,
                                double skin, int32_t kcap, const double* r, double* f,
                                double* out, void* stream) {
    if (!sys || !r || !f || !out || kcap > kPairMaxCap || !std::isfinite(gamma_dot) ||
        !std::isfinite(skin))
        return TTCF_EINVAL;
    SysDev S{};
    std::string why;
    int32_t rc = build_sysdev(sys, &S, &why);
    if (rc != TTCF_OK) return rc;
    if (S.n > kPairMaxAtoms || !set_list_grid(&S, skin)) return TTCF_EINVAL;
    if (kcap <= 0) kcap = auto_pair_cap(S);
    const int n = S.n;
    const int C = S.lc[0] * S.lc[1] * S.lc[2];
    const int waves = pair_job_threads(n) / 64;
    // scratch layout (each part 256-byte aligned): pair words, wave counts, cell and rank of
    // every atom, cell starts
    const int64_t w_pairs = words256(pair_words(n, kcap, pair_job_apt(n)));
    const int64_t w_seg = words256(waves), w_atoms = words256(n);
    const int64_t need = w_pairs + w_seg + 2 * w_atoms + words256(C + 1);
    if (need * 4 > TTCF_STATIC_SCRATCH_BYTES) return TTCF_ESCRATCH;
    StaticScratch d;
    rc = static_scratch(&d);
    if (rc != TTCF_OK) return rc;
    if (lds_bytes_pairs(n, C) > d.lds) return TTCF_EINVAL;
    uint32_t* pairs = d.ptr;
    int32_t* seg = (int32_t*)(pairs + w_pairs);
    int32_t* cell_of = seg + w_seg;
    int32_t* rank_of = cell_of + w_atoms;
    int32_t* start = rank_of + w_atoms;
    const hipError_t e = launch_debug_pair_form(S, gamma_dot, kstep, r, kcap, pairs, seg,
                                                cell_of, rank_of, start, f, out,
                                                (hipStream_t)stream);
    return e == hipSuccess ? TTCF_OK : TTCF_EDEVICE;
}

}  // extern "C"
