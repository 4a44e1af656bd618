// ttcf_channel_capi.hip -- host runtime and C ABI of the confined-channel example
// (ttcf_channel_* in include/ttcf.h). The calls follow the same algorithm as the bulk ones
// (Alg. LAMMPS SCRIPT): a mother trajectory is run and sampled, each start state spawns
// its mapped daughters with the lattices moving, the daughters are stepped in one
// persistent launch per batch, and finished groups are folded into per-start-state rows from
// which Eq. TTCF (with Omega of Eq. TTCF2) is formed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ttcf.h"
#include "ttcf_channel.h"

using namespace ttcf;

namespace {

struct ChBatch {
    int32_t n_states = 0, n_daughters = 0, n_steps = 0;
    int64_t first_id = 0;
    double* r = nullptr;       // n_daughters x 3n
    double* p = nullptr;
    float* f = nullptr;
    double* latx = nullptr;    // n_daughters x n_wall
    double* series = nullptr;  // n_daughters x (n_steps + 1) x n_obs
    ChannelDesc* d_descs = nullptr;
    std::vector<ChannelDesc> descs;
    bool live = true;
};

}  // namespace

struct ttcf_channel_ctx {
    hipStream_t stream = nullptr;
    std::string err;
    ttcf_channel ch{};
    ChannelDev dev{};
    int num_cu = 0;
    size_t max_lds = 0;
    // mother
    double* m_r = nullptr;
    double* m_p = nullptr;
    float* m_f = nullptr;
    double* lat = nullptr;     // 3 x n_wall (x, y, z rows)
    ChannelDesc* d_mdesc = nullptr;
    ChannelDesc mdesc{};
    int64_t m_steps = 0;
    // stored start states: per state [r (3n) | p (3n) | zeta]
    double* states = nullptr;
    int32_t n_states = 0, states_cap = 0;
    // daughters
    std::vector<ChBatch> batches;
    int64_t next_id = 0;
    // accumulated start-state rows
    double* acc_d = nullptr;
    double* acc_i = nullptr;
    int64_t acc_rows = 0, acc_cap = 0;
    int32_t acc_nt = 0;        // time points per row (the stride's t extent)
    std::vector<double> row_v, row_coef;
    std::vector<int32_t> row_nt, row_health;
    // launch resources
    char* scratch = nullptr;
    size_t scratch_bytes = 0;
    int32_t* queue = nullptr;
    // timing of the step kernel
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    double step_ms = 0.0;
    int64_t launches = 0;
};

namespace {

thread_local std::string g_free_err;  // message of the last failed call without a context

int32_t cfail(ttcf_channel_ctx* c, int32_t code, const std::string& msg) {
    if (c)
        c->err = msg;
    else
        g_free_err = msg;
    return code;
}

#define CHK(ctx, expr)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return cfail((ctx), TTCF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

int32_t build_dev(const ttcf_channel* ch, ChannelDev* d, std::string* why) {
    const int64_t n = (int64_t)ch->n_fluid + ch->n_wall;
    if (ch->n_fluid < 1 || ch->n_wall < 2 || (ch->n_wall % 2) != 0 || n > kMaxAtoms) {
        *why = "need n_fluid >= 1, an even n_wall >= 2 and at most 65535 atoms";
        return TTCF_EINVAL;
    }
    if (ch->n_bins < 1 || ch->n_bins > kChMaxBins || !(ch->bin_hi > ch->bin_lo)) {
        *why = "bad profile bins";
        return TTCF_EINVAL;
    }
    if (!(ch->r_cut > 0.0) || !(ch->dt > 0.0) || !(ch->temperature > 0.0) ||
        !(ch->nh_tau > 0.0) || !(ch->k_spring >= 0.0) || !(ch->lx > 0.0) || !(ch->lz > 0.0) ||
        !(ch->y_extent > 0.0)) {
        *why = "non-positive length, cutoff, time step, temperature or thermostat time";
        return TTCF_EINVAL;
    }
    std::memset(d, 0, sizeof(*d));
    d->n = (int32_t)n;
    d->n_fluid = ch->n_fluid;
    d->n_wall = ch->n_wall;
    d->n_bins = ch->n_bins;
    d->kmax = ch->kmax > 0 ? ch->kmax : 160;
    if (d->kmax > 1024) {
        *why = "kmax must be at most 1024";
        return TTCF_EINVAL;
    }
    d->lx = ch->lx;
    d->lz = ch->lz;
    d->y_extent = ch->y_extent;
    d->rc = ch->r_cut;
    if (ch->skin > 0.0) {
        d->skin = ch->skin;
    } else {
        // 0.4 (the fastest on the full-size channel), narrowed where a small box needs it to
        // keep three list cells across x and z and four along y
        const double room = std::min(std::min(ch->lx, ch->lz) / 3.0, ch->y_extent / 4.0);
        d->skin = std::max(0.1, std::min(0.4, (room - ch->r_cut) * (1.0 - 1e-9)));
    }
    d->c_ff = ch->c_ff;
    d->c_wf = ch->c_wf;
    d->k_spring = ch->k_spring;
    d->temperature = ch->temperature;
    d->nf_w = 3.0 * ch->n_wall;
    d->q = d->nf_w * ch->temperature * ch->nh_tau * ch->nh_tau;
    d->dt = ch->dt;
    d->bin_lo = ch->bin_lo;
    d->bin_hi = ch->bin_hi;
    d->bin_w = (ch->bin_hi - ch->bin_lo) / (double)ch->n_bins;
    const double reach = d->rc + d->skin;
    const double ext[3] = {ch->lx, ch->y_extent, ch->lz};
    for (int a = 0; a < 3; ++a) {
        d->lc[a] = (int32_t)std::floor(ext[a] / reach);
        d->fix_scale[a] = 4294967296.0 / ext[a];
        d->fix_unit[a] = (float)(ext[a] / 4294967296.0);
    }
    d->rc2_f = (float)(d->rc * d->rc);
    d->rl2_f = (float)(reach * reach);
    // x and z periodic with three distinct neighbour columns; in y two cells must span at
    // most half the extent so that fixed-point differences of neighbours stay in int32
    if (d->lc[0] < 3 || d->lc[2] < 3 || d->lc[1] < 4 || d->lc[0] * d->lc[1] * d->lc[2] > 65536) {
        *why = "box too small for the list grid (need 3 cells in x and z, 4 in y)";
        return TTCF_EINVAL;
    }
    if (ch->lx < 2.0 * reach || ch->lz < 2.0 * reach) {
        *why = "periodic edges must exceed twice r_cut + skin";
        return TTCF_EINVAL;
    }
    return TTCF_OK;
}

int32_t ensure_scratch(ttcf_channel_ctx* c, int grid) {
    const size_t stride = channel_scratch_bytes(c->dev.n, c->dev.kmax);
    const size_t need = stride * (size_t)grid;
    if (need <= c->scratch_bytes) return TTCF_OK;
    CHK(c, hipStreamSynchronize(c->stream));
    rt_free(c->scratch);
    c->scratch = (char*)rt_alloc(need, c->stream);
    c->scratch_bytes = c->scratch ? need : 0;
    if (!c->scratch) return cfail(c, TTCF_ENOMEM, "scratch allocation failed");
    return TTCF_OK;
}

int32_t launch(ttcf_channel_ctx* c, ChannelDesc* d_descs, int32_t n_jobs, int32_t max_steps,
               bool timed) {
    const size_t lds = channel_lds_bytes(c->dev.n, c->dev.lc[0] * c->dev.lc[1] * c->dev.lc[2]);
    if (lds > c->max_lds) return cfail(c, TTCF_EINVAL, "system exceeds the LDS of one workgroup");
    // resident workgroups per CU: the LDS and the register budget (4 SIMDs per CU)
    const int per_cu = std::max(
        1, std::min<int>((int)(c->max_lds / lds), 4 * kChWavesPerSimd / (kChThreads / 64)));
    const int grid = std::max(1, std::min(n_jobs, per_cu * c->num_cu));
    int32_t rc = ensure_scratch(c, grid);
    if (rc != TTCF_OK) return rc;
    ChannelLaunch L{};
    L.sys = c->dev;
    L.descs = d_descs;
    L.order = nullptr;
    L.n_jobs = n_jobs;
    L.grid = grid;
    L.cmax = c->dev.lc[0] * c->dev.lc[1] * c->dev.lc[2];
    L.max_steps = max_steps;
    L.queue = c->queue;
    L.scratch = c->scratch;
    L.scratch_stride = channel_scratch_bytes(c->dev.n, c->dev.kmax);
    const int32_t zero = 0;
    (void)hipGetLastError();
    CHK(c, hipMemcpyAsync(c->queue, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        CHK(c, hipEventCreate(&e0));
        CHK(c, hipEventCreate(&e1));
        CHK(c, hipEventRecord(e0, c->stream));
    }
    CHK(c, launch_channel(L, c->stream));
    if (timed) {
        CHK(c, hipEventRecord(e1, c->stream));
        c->events.emplace_back(e0, e1);
    }
    return TTCF_OK;
}

void free_batch(ChBatch& b) {
    rt_free(b.r);
    rt_free(b.p);
    rt_free(b.f);
    rt_free(b.latx);
    rt_free(b.series);
    rt_free(b.d_descs);
    b.r = b.p = b.latx = b.series = nullptr;
    b.f = nullptr;
    b.d_descs = nullptr;
    b.live = false;
}

int32_t pull_mother(ttcf_channel_ctx* c) {
    CHK(c, hipMemcpyAsync(&c->mdesc, c->d_mdesc, sizeof(ChannelDesc), hipMemcpyDeviceToHost,
                          c->stream));
    CHK(c, hipStreamSynchronize(c->stream));
    return TTCF_OK;
}

int32_t run_mother(ttcf_channel_ctx* c, int64_t n_steps) {
    while (n_steps > 0) {
        const int32_t chunk = (int32_t)std::min<int64_t>(n_steps, 1 << 30);
        c->mdesc.n_steps = c->mdesc.done + chunk;
        CHK(c, hipMemcpyAsync(c->d_mdesc, &c->mdesc, sizeof(ChannelDesc), hipMemcpyHostToDevice,
                              c->stream));
        int32_t rc = launch(c, c->d_mdesc, 1, chunk, false);
        if (rc != TTCF_OK) return rc;
        rc = pull_mother(c);
        if (rc != TTCF_OK) return rc;
        if (c->mdesc.health != 0) return cfail(c, TTCF_EUNSTABLE, "the mother trajectory failed its health check");
        c->m_steps += chunk;
        n_steps -= chunk;
    }
    return TTCF_OK;
}

int32_t grow_states(ttcf_channel_ctx* c, int32_t n_states) {
    if (c->states_cap >= n_states) return TTCF_OK;
    CHK(c, hipStreamSynchronize(c->stream));
    rt_free(c->states);
    c->states = (double*)rt_alloc(sizeof(double) * ((size_t)6 * c->dev.n + 1) * n_states, c->stream);
    c->states_cap = c->states ? n_states : 0;
    c->n_states = 0;
    if (!c->states) return cfail(c, TTCF_ENOMEM, "state buffer allocation failed");
    return TTCF_OK;
}

int32_t grow_acc(ttcf_channel_ctx* c, int64_t rows, int32_t n_t) {
    const int nobs = 1 + c->dev.n_bins;
    const int32_t nt = std::max(c->acc_nt, n_t);
    if (rows <= c->acc_cap && nt == c->acc_nt) return TTCF_OK;
    const int64_t cap = std::max<int64_t>(rows, 2 * c->acc_cap);
    const size_t row = (size_t)nt * nobs;
    double* nd = (double*)rt_alloc(sizeof(double) * row * cap, c->stream);
    double* ni = (double*)rt_alloc(sizeof(double) * row * cap, c->stream);
    if (!nd || !ni) {
        rt_free(nd);
        rt_free(ni);
        return cfail(c, TTCF_ENOMEM, "accumulator allocation failed");
    }
    if (c->acc_rows > 0) {
        const size_t old = (size_t)c->acc_nt * nobs;
        CHK(c, hipMemcpy2DAsync(nd, sizeof(double) * row, c->acc_d, sizeof(double) * old,
                                sizeof(double) * old, (size_t)c->acc_rows, hipMemcpyDeviceToDevice,
                                c->stream));
        CHK(c, hipMemcpy2DAsync(ni, sizeof(double) * row, c->acc_i, sizeof(double) * old,
                                sizeof(double) * old, (size_t)c->acc_rows, hipMemcpyDeviceToDevice,
                                c->stream));
    }
    CHK(c, hipStreamSynchronize(c->stream));
    rt_free(c->acc_d);
    rt_free(c->acc_i);
    c->acc_d = nd;
    c->acc_i = ni;
    c->acc_cap = cap;
    c->acc_nt = nt;
    return TTCF_OK;
}

int32_t find_daughter(ttcf_channel_ctx* c, int64_t id, int* bi, int* di) {
    for (size_t b = 0; b < c->batches.size(); ++b) {
        const ChBatch& B = c->batches[b];
        if (B.live && id >= B.first_id && id < B.first_id + B.n_daughters) {
            *bi = (int)b;
            *di = (int)(id - B.first_id);
            return TTCF_OK;
        }
    }
    return cfail(c, TTCF_EINVAL, "no such live daughter");
}

int32_t pull_batch(ttcf_channel_ctx* c, ChBatch& b) {
    CHK(c, hipMemcpyAsync(b.descs.data(), b.d_descs, sizeof(ChannelDesc) * b.descs.size(),
                          hipMemcpyDeviceToHost, c->stream));
    CHK(c, hipStreamSynchronize(c->stream));
    return TTCF_OK;
}

}  // namespace

extern "C" {

int32_t ttcf_channel_create(ttcf_channel_ctx** out, const ttcf_channel* ch, const double* r0,
                            const double* p0, const double* lattice, void* stream) {
    if (!out || !ch || !r0 || !p0 || !lattice) return TTCF_EINVAL;
    *out = nullptr;
    ChannelDev dev;
    std::string why;
    int32_t rc = build_dev(ch, &dev, &why);
    if (rc != TTCF_OK) return cfail(nullptr, rc, why);
    int devid = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&devid);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, devid);
    if (e != hipSuccess)
        return cfail(nullptr, TTCF_EDEVICE, std::string("device query: ") + hipGetErrorString(e));
    ttcf_channel_ctx* c = new ttcf_channel_ctx();
    c->stream = (hipStream_t)stream;
    c->ch = *ch;
    c->dev = dev;
    c->num_cu = prop.multiProcessorCount;
    c->max_lds = prop.sharedMemPerBlock;
    const size_t n = (size_t)dev.n, nw = (size_t)dev.n_wall;
    c->m_r = (double*)rt_alloc(sizeof(double) * 3 * n, c->stream);
    c->m_p = (double*)rt_alloc(sizeof(double) * 3 * n, c->stream);
    c->m_f = (float*)rt_alloc(sizeof(float) * 3 * n, c->stream);
    c->lat = (double*)rt_alloc(sizeof(double) * 3 * nw, c->stream);
    c->d_mdesc = (ChannelDesc*)rt_alloc(sizeof(ChannelDesc), c->stream);
    c->queue = (int32_t*)rt_alloc(64, c->stream);
    if (!c->m_r || !c->m_p || !c->m_f || !c->lat || !c->d_mdesc || !c->queue) {
        ttcf_channel_destroy(c);
        return TTCF_ENOMEM;
    }
    if (hipMemcpyAsync(c->m_r, r0, sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->m_p, p0, sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->lat, lattice, sizeof(double) * 3 * nw, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
        ttcf_channel_destroy(c);
        return TTCF_EDEVICE;
    }
    ChannelDesc& m = c->mdesc;
    m = ChannelDesc{};
    m.r = c->m_r;
    m.p = c->m_p;
    m.f = c->m_f;
    m.latx = c->lat;
    m.laty = c->lat + nw;
    m.latz = c->lat + 2 * nw;
    m.series = nullptr;
    m.v = 0.0;
    if (hipMemcpyAsync(c->d_mdesc, &m, sizeof(ChannelDesc), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        ttcf_channel_destroy(c);
        return TTCF_EDEVICE;
    }
    *out = c;
    return TTCF_OK;
}

void ttcf_channel_destroy(ttcf_channel_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& b : c->batches) free_batch(b);
    for (auto& e : c->events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    rt_free(c->m_r);
    rt_free(c->m_p);
    rt_free(c->m_f);
    rt_free(c->lat);
    rt_free(c->d_mdesc);
    rt_free(c->states);
    rt_free(c->acc_d);
    rt_free(c->acc_i);
    rt_free(c->scratch);
    rt_free(c->queue);
    delete c;
}

const char* ttcf_channel_last_error(const ttcf_channel_ctx* c) {
    return c ? c->err.c_str() : g_free_err.c_str();
}

int32_t ttcf_channel_run_mother(ttcf_channel_ctx* c, int64_t n_steps) {
    if (!c || n_steps < 0) return TTCF_EINVAL;
    return run_mother(c, n_steps);
}

int32_t ttcf_channel_sample_states(ttcf_channel_ctx* c, int32_t n_states, int64_t steps_between) {
    if (!c || n_states <= 0 || steps_between <= 0) return TTCF_EINVAL;
    int32_t rc = grow_states(c, n_states);
    if (rc != TTCF_OK) return rc;
    const size_t n = (size_t)c->dev.n, sz = 6 * n + 1;
    for (int32_t s = 0; s < n_states; ++s) {
        rc = run_mother(c, steps_between);
        if (rc != TTCF_OK) return rc;
        double* dst = c->states + sz * s;
        CHK(c, hipMemcpyAsync(dst, c->m_r, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, c->stream));
        CHK(c, hipMemcpyAsync(dst + 3 * n, c->m_p, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice,
                              c->stream));
        CHK(c, hipMemcpyAsync(dst + 6 * n, &c->mdesc.zeta, sizeof(double), hipMemcpyHostToDevice,
                              c->stream));
        CHK(c, hipStreamSynchronize(c->stream));
    }
    c->n_states = n_states;
    return TTCF_OK;
}

int32_t ttcf_channel_sample_states_replicated(ttcf_channel_ctx* c, int32_t n_replicas,
                                              const double* kicks, int64_t decorrelate_steps,
                                              int32_t states_per_replica,
                                              int64_t steps_between) {
    if (!c || n_replicas <= 0 || decorrelate_steps < 0 || states_per_replica <= 0 ||
        steps_between <= 0)
        return TTCF_EINVAL;
    const int64_t total = decorrelate_steps + (int64_t)states_per_replica * steps_between;
    const int64_t n_out = (int64_t)n_replicas * states_per_replica;
    if (total > (1 << 30) || n_out > (1 << 22))
        return cfail(c, TTCF_EINVAL, "too many replica steps or states");
    int32_t rc = grow_states(c, (int32_t)n_out);
    if (rc != TTCF_OK) return rc;
    const size_t n = (size_t)c->dev.n, R = (size_t)n_replicas;
    double* rr = (double*)rt_alloc(sizeof(double) * 3 * n * R, c->stream);
    double* pp = (double*)rt_alloc(sizeof(double) * 3 * n * R, c->stream);
    float* ff = (float*)rt_alloc(sizeof(float) * 3 * n * R, c->stream);
    double* dk = kicks ? (double*)rt_alloc(sizeof(double) * 3 * n * R, c->stream) : nullptr;
    ChannelDesc* dd = (ChannelDesc*)rt_alloc(sizeof(ChannelDesc) * R, c->stream);
    auto release = [&]() {
        (void)hipStreamSynchronize(c->stream);
        rt_free(rr);
        rt_free(pp);
        rt_free(ff);
        rt_free(dk);
        rt_free(dd);
    };
    if (!rr || !pp || !ff || !dd || (kicks && !dk)) {
        release();
        return cfail(c, TTCF_ENOMEM, "replica allocation failed");
    }
    // every replica: the mother's dynamics (lattice at rest), its own copy of the state
    std::vector<ChannelDesc> hd(R);
    for (size_t q = 0; q < R; ++q) {
        ChannelDesc& D = hd[q];
        D = c->mdesc;
        D.r = rr + 3 * n * q;
        D.p = pp + 3 * n * q;
        D.f = ff + 3 * n * q;
        D.series = nullptr;
        D.v = 0.0;
        D.done = 0;  // the first launch computes forces and the wall p^2 of the kicked state
        D.n_steps = (int32_t)total;
        D.health = 0;
    }
    auto chk = [&](hipError_t e, const char* what) -> int32_t {
        if (e == hipSuccess) return TTCF_OK;
        release();
        return cfail(c, TTCF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    if ((rc = chk(hipMemcpyAsync(dd, hd.data(), sizeof(ChannelDesc) * R, hipMemcpyHostToDevice,
                                 c->stream), "descriptors")) != TTCF_OK)
        return rc;
    if (kicks &&
        (rc = chk(hipMemcpyAsync(dk, kicks, sizeof(double) * 3 * n * R, hipMemcpyHostToDevice,
                                 c->stream), "kicks")) != TTCF_OK)
        return rc;
    if ((rc = chk(launch_channel_replicate(c->m_r, c->m_p, dk, c->dev.n, dd, n_replicas,
                                           c->stream), "replicate")) != TTCF_OK)
        return rc;
    // one persistent launch per stretch: decorrelation, then one per saved state
    if (decorrelate_steps > 0) {
        rc = launch(c, dd, n_replicas, (int32_t)decorrelate_steps, false);
        if (rc != TTCF_OK) {
            release();
            return rc;
        }
    }
    for (int32_t st = 0; st < states_per_replica; ++st) {
        rc = launch(c, dd, n_replicas, (int32_t)steps_between, false);
        if (rc != TTCF_OK) {
            release();
            return rc;
        }
        if ((rc = chk(launch_channel_snapshot(dd, n_replicas, c->dev.n, c->states,
                                              states_per_replica, st, c->stream),
                      "snapshot")) != TTCF_OK)
            return rc;
    }
    if ((rc = chk(hipMemcpyAsync(hd.data(), dd, sizeof(ChannelDesc) * R, hipMemcpyDeviceToHost,
                                 c->stream), "descriptors")) != TTCF_OK)
        return rc;
    release();
    for (size_t q = 0; q < R; ++q)
        if (hd[q].health != 0 || hd[q].done != (int32_t)total) {
            c->n_states = 0;
            return cfail(c, TTCF_EUNSTABLE, "a mother replica failed its health check");
        }
    c->n_states = (int32_t)n_out;
    return TTCF_OK;
}

int32_t ttcf_channel_import_states(ttcf_channel_ctx* c, int32_t n_states, const double* r,
                                   const double* p, const double* zeta) {
    if (!c || n_states <= 0 || !r || !p || !zeta) return TTCF_EINVAL;
    int32_t rc = grow_states(c, n_states);
    if (rc != TTCF_OK) return rc;
    const size_t n = (size_t)c->dev.n, sz = 6 * n + 1;
    for (int32_t s = 0; s < n_states; ++s) {
        double* dst = c->states + sz * s;
        CHK(c, hipMemcpyAsync(dst, r + 3 * n * s, sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream));
        CHK(c, hipMemcpyAsync(dst + 3 * n, p + 3 * n * s, sizeof(double) * 3 * n, hipMemcpyHostToDevice,
                              c->stream));
        CHK(c, hipMemcpyAsync(dst + 6 * n, zeta + s, sizeof(double), hipMemcpyHostToDevice, c->stream));
    }
    CHK(c, hipStreamSynchronize(c->stream));
    c->n_states = n_states;
    return TTCF_OK;
}

int32_t ttcf_channel_export_states(ttcf_channel_ctx* c, int32_t n_states, double* r, double* p,
                                   double* zeta) {
    if (!c || n_states <= 0 || n_states > c->n_states) return TTCF_EINVAL;
    const size_t n = (size_t)c->dev.n, sz = 6 * n + 1;
    for (int32_t s = 0; s < n_states; ++s) {
        const double* src = c->states + sz * s;
        if (r) CHK(c, hipMemcpyAsync(r + 3 * n * s, src, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->stream));
        if (p)
            CHK(c, hipMemcpyAsync(p + 3 * n * s, src + 3 * n, sizeof(double) * 3 * n,
                                  hipMemcpyDeviceToHost, c->stream));
        if (zeta) CHK(c, hipMemcpyAsync(zeta + s, src + 6 * n, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    CHK(c, hipStreamSynchronize(c->stream));
    return TTCF_OK;
}

int32_t ttcf_channel_export_mother(ttcf_channel_ctx* c, double* r, double* p, double* zeta,
                                   int64_t* steps) {
    if (!c) return TTCF_EINVAL;
    const size_t n = (size_t)c->dev.n;
    if (r) CHK(c, hipMemcpyAsync(r, c->m_r, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->stream));
    if (p) CHK(c, hipMemcpyAsync(p, c->m_p, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->stream));
    CHK(c, hipStreamSynchronize(c->stream));
    if (zeta) *zeta = c->mdesc.zeta;
    if (steps) *steps = c->m_steps;
    return TTCF_OK;
}

int32_t ttcf_channel_spawn(ttcf_channel_ctx* c, int32_t n_states, uint32_t mapping_mask,
                           const double* v, int32_t n_v, int32_t n_steps, int64_t* out_first) {
    if (!c || n_states <= 0 || !v || !(n_v == 1 || n_v == n_states) || n_steps < 1 ||
        (mapping_mask & 0xFu) == 0 || (mapping_mask & ~0xFu) != 0)
        return cfail(c, TTCF_EINVAL, "bad spawn arguments");
    if (n_states > c->n_states) return cfail(c, TTCF_ESTATE, "fewer stored start states than asked for");
    for (int32_t i = 0; i < n_v; ++i)
        if (!std::isfinite(v[i])) return cfail(c, TTCF_EINVAL, "lattice speeds must be finite");
    std::vector<int32_t> maps;
    for (int m = 0; m < 4; ++m)
        if (mapping_mask & (1u << m)) maps.push_back(m);
    const int nm = (int)maps.size();
    const size_t n = (size_t)c->dev.n, nw = (size_t)c->dev.n_wall;
    const int nobs = 1 + c->dev.n_bins;
    ChBatch b;
    b.n_states = n_states;
    b.n_daughters = n_states * nm;
    b.n_steps = n_steps;
    b.first_id = c->next_id;
    const size_t nd = (size_t)b.n_daughters;
    b.r = (double*)rt_alloc(sizeof(double) * 3 * n * nd, c->stream);
    b.p = (double*)rt_alloc(sizeof(double) * 3 * n * nd, c->stream);
    b.f = (float*)rt_alloc(sizeof(float) * 3 * n * nd, c->stream);
    b.latx = (double*)rt_alloc(sizeof(double) * nw * nd, c->stream);
    b.series = (double*)rt_alloc(sizeof(double) * ((size_t)n_steps + 1) * nobs * nd, c->stream);
    b.d_descs = (ChannelDesc*)rt_alloc(sizeof(ChannelDesc) * nd, c->stream);
    if (!b.r || !b.p || !b.f || !b.latx || !b.series || !b.d_descs) {
        free_batch(b);
        return cfail(c, TTCF_ENOMEM, "daughter allocation failed");
    }
    b.descs.resize(nd);
    for (size_t d = 0; d < nd; ++d) {
        ChannelDesc& D = b.descs[d];
        D = ChannelDesc{};
        D.r = b.r + 3 * n * d;
        D.p = b.p + 3 * n * d;
        D.f = b.f + 3 * n * d;
        D.latx = b.latx + nw * d;
        D.laty = c->lat + nw;
        D.latz = c->lat + 2 * nw;
        D.series = b.series + ((size_t)n_steps + 1) * nobs * d;
        D.state = (int32_t)(d / nm);
        D.map = maps[d % nm];
        D.v = v[n_v == 1 ? 0 : D.state];
        D.n_steps = n_steps;
    }
    CHK(c, hipMemcpyAsync(b.d_descs, b.descs.data(), sizeof(ChannelDesc) * nd, hipMemcpyHostToDevice,
                          c->stream));
    CHK(c, launch_channel_spawn(c->states, c->dev.n, c->dev.n_wall, c->dev.lx, c->lat, b.d_descs,
                                b.n_daughters, c->stream));
    CHK(c, hipStreamSynchronize(c->stream));
    c->next_id += b.n_daughters;
    if (out_first) *out_first = b.first_id;
    c->batches.push_back(std::move(b));
    return TTCF_OK;
}

int32_t ttcf_channel_step(ttcf_channel_ctx* c, int32_t n_steps) {
    if (!c || n_steps < 0) return TTCF_EINVAL;
    if (n_steps == 0) return TTCF_OK;
    for (auto& b : c->batches) {
        if (!b.live) continue;
        int32_t rc = launch(c, b.d_descs, b.n_daughters, n_steps, true);
        if (rc != TTCF_OK) return rc;
    }
    return TTCF_OK;
}

int32_t ttcf_channel_accumulate(ttcf_channel_ctx* c, int64_t* out_groups) {
    if (!c) return TTCF_EINVAL;
    const int nobs = 1 + c->dev.n_bins;
    int64_t added = 0;
    for (auto& b : c->batches) {
        if (!b.live) continue;
        int32_t rc = pull_batch(c, b);
        if (rc != TTCF_OK) return rc;
        bool finished = true;
        for (const auto& d : b.descs) finished = finished && (d.health != 0 || d.done >= d.n_steps);
        if (!finished) continue;
        const int nm = b.n_daughters / b.n_states;
        const int32_t n_t = b.n_steps + 1;
        rc = grow_acc(c, c->acc_rows + b.n_states, n_t);
        if (rc != TTCF_OK) return rc;
        std::vector<int32_t> first_of(b.n_states + 1);
        for (int32_t g = 0; g <= b.n_states; ++g) first_of[g] = g * nm;
        int32_t* d_first = (int32_t*)rt_alloc(sizeof(int32_t) * first_of.size(), c->stream);
        if (!d_first) return cfail(c, TTCF_ENOMEM, "allocation failed");
        CHK(c, hipMemcpyAsync(d_first, first_of.data(), sizeof(int32_t) * first_of.size(),
                              hipMemcpyHostToDevice, c->stream));
        // one thread per (group, observable), every group's row at the context's stride
        const size_t row = (size_t)c->acc_nt * nobs;
        ChannelAccum A{};
        A.descs = b.d_descs;
        A.first_of = d_first;
        A.d_out = c->acc_d + row * (size_t)c->acc_rows;
        A.i_out = c->acc_i + row * (size_t)c->acc_rows;
        A.n_groups = b.n_states;
        A.n_t = n_t;
        A.n_obs = nobs;
        A.dt = c->dev.dt;
        A.row_stride = row;
        CHK(c, launch_channel_accumulate(A, c->stream));
        CHK(c, hipStreamSynchronize(c->stream));
        rt_free(d_first);
        for (int32_t g = 0; g < b.n_states; ++g) {
            int32_t h = 0;
            for (int m = 0; m < nm; ++m) h |= b.descs[(size_t)g * nm + m].health;
            const double vv = b.descs[(size_t)g * nm].v;
            c->row_v.push_back(vv);
            c->row_coef.push_back(c->dev.k_spring * vv / (2.0 * c->dev.temperature));
            c->row_nt.push_back(n_t);
            c->row_health.push_back(h);
            if (h == 0) ++added;
        }
        c->acc_rows += b.n_states;
        free_batch(b);
    }
    if (out_groups) *out_groups = added;
    return TTCF_OK;
}

int32_t ttcf_channel_response(ttcf_channel_ctx* c, int32_t observable, double v_filter, int32_t n_t,
                              double* ttcf_mean, double* ttcf_se, double* dav_mean, double* dav_se,
                              int64_t* out_n_states) {
    if (!c || n_t <= 0 || (observable != TTCF_OBS_WALL_STRESS && observable != TTCF_OBS_VPROFILE))
        return TTCF_EINVAL;
    std::vector<int32_t> rows;
    for (int64_t r = 0; r < c->acc_rows; ++r) {
        if (c->row_health[r] != 0 || c->row_v[r] != v_filter) continue;
        if (c->row_nt[r] < n_t) return cfail(c, TTCF_ESTATE, "n_t exceeds a matching group's length");
        rows.push_back((int32_t)r);
    }
    if (rows.empty()) return cfail(c, TTCF_ESTATE, "no accumulated group at this lattice speed");
    const int nobs = 1 + c->dev.n_bins;
    const int col0 = observable == TTCF_OBS_WALL_STRESS ? 0 : 1;
    const int ncol = observable == TTCF_OBS_WALL_STRESS ? 1 : c->dev.n_bins;
    const size_t plane = (size_t)n_t * ncol;
    double* d_out = (double*)rt_alloc(sizeof(double) * 4 * plane, c->stream);
    int32_t* d_rows = (int32_t*)rt_alloc(sizeof(int32_t) * rows.size(), c->stream);
    double* d_coef = (double*)rt_alloc(sizeof(double) * c->row_coef.size(), c->stream);
    if (!d_out || !d_rows || !d_coef) {
        rt_free(d_out);
        rt_free(d_rows);
        rt_free(d_coef);
        return cfail(c, TTCF_ENOMEM, "allocation failed");
    }
    CHK(c, hipMemcpyAsync(d_rows, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice, c->stream));
    CHK(c, hipMemcpyAsync(d_coef, c->row_coef.data(), sizeof(double) * c->row_coef.size(),
                          hipMemcpyHostToDevice, c->stream));
    ChannelResponse R{};
    R.d_all = c->acc_d;
    R.i_all = c->acc_i;
    R.coef = d_coef;
    R.rows = d_rows;
    R.n_rows = (int32_t)rows.size();
    R.n_t = n_t;
    R.n_obs = nobs;
    R.col0 = col0;
    R.n_cols = ncol;
    R.row_stride = (size_t)c->acc_nt * nobs;
    R.out = d_out;
    CHK(c, launch_channel_response(R, c->stream));
    std::vector<double> out(4 * plane);
    CHK(c, hipMemcpyAsync(out.data(), d_out, sizeof(double) * out.size(), hipMemcpyDeviceToHost, c->stream));
    CHK(c, hipStreamSynchronize(c->stream));
    rt_free(d_out);
    rt_free(d_rows);
    rt_free(d_coef);
    if (ttcf_mean) std::memcpy(ttcf_mean, out.data(), sizeof(double) * plane);
    if (ttcf_se) std::memcpy(ttcf_se, out.data() + plane, sizeof(double) * plane);
    if (dav_mean) std::memcpy(dav_mean, out.data() + 2 * plane, sizeof(double) * plane);
    if (dav_se) std::memcpy(dav_se, out.data() + 3 * plane, sizeof(double) * plane);
    if (out_n_states) *out_n_states = (int64_t)rows.size();
    return TTCF_OK;
}

int32_t ttcf_channel_export_series(ttcf_channel_ctx* c, int64_t first, int32_t count, int32_t n_t,
                                   double* obs, double* s0) {
    if (!c || count <= 0 || n_t <= 0) return TTCF_EINVAL;
    const int nobs = 1 + c->dev.n_bins;
    for (int32_t q = 0; q < count; ++q) {
        int bi = 0, di = 0;
        int32_t rc = find_daughter(c, first + q, &bi, &di);
        if (rc != TTCF_OK) return rc;
        ChBatch& b = c->batches[bi];
        if (n_t > b.n_steps + 1) return cfail(c, TTCF_EINVAL, "n_t beyond the daughter's length");
        rc = pull_batch(c, b);
        if (rc != TTCF_OK) return rc;
        if (obs)
            CHK(c, hipMemcpyAsync(obs + (size_t)q * n_t * nobs, b.descs[di].series,
                                  sizeof(double) * (size_t)n_t * nobs, hipMemcpyDeviceToHost, c->stream));
        if (s0) s0[q] = b.descs[di].s0;
    }
    CHK(c, hipStreamSynchronize(c->stream));
    return TTCF_OK;
}

int32_t ttcf_channel_export_daughter(ttcf_channel_ctx* c, int64_t id, double* r, double* p,
                                     double* zeta) {
    if (!c) return TTCF_EINVAL;
    int bi = 0, di = 0;
    int32_t rc = find_daughter(c, id, &bi, &di);
    if (rc != TTCF_OK) return rc;
    ChBatch& b = c->batches[bi];
    rc = pull_batch(c, b);
    if (rc != TTCF_OK) return rc;
    const size_t n = (size_t)c->dev.n;
    if (r) CHK(c, hipMemcpyAsync(r, b.descs[di].r, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->stream));
    if (p) CHK(c, hipMemcpyAsync(p, b.descs[di].p, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->stream));
    CHK(c, hipStreamSynchronize(c->stream));
    if (zeta) *zeta = b.descs[di].zeta;
    return TTCF_OK;
}

int32_t ttcf_channel_daughter_health(ttcf_channel_ctx* c, int64_t id, int32_t* health) {
    if (!c || !health) return TTCF_EINVAL;
    int bi = 0, di = 0;
    int32_t rc = find_daughter(c, id, &bi, &di);
    if (rc != TTCF_OK) return rc;
    rc = pull_batch(c, c->batches[bi]);
    if (rc != TTCF_OK) return rc;
    *health = c->batches[bi].descs[di].health;
    return TTCF_OK;
}

int32_t ttcf_channel_debug_forces(const ttcf_channel* ch, const double* r, const double* lattice,
                                  double* f, double* out, void* stream) {
    if (!ch || !r || !lattice || !f || !out) return TTCF_EINVAL;
    ChannelDev dev;
    std::string why;
    int32_t rc = build_dev(ch, &dev, &why);
    if (rc != TTCF_OK) return cfail(nullptr, rc, why);
    hipStream_t s = (hipStream_t)stream;
    int devid = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&devid);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, devid);
    if (e != hipSuccess)
        return cfail(nullptr, TTCF_EDEVICE, std::string("device query: ") + hipGetErrorString(e));
    const int cmax = dev.lc[0] * dev.lc[1] * dev.lc[2];
    if (channel_lds_bytes(dev.n, cmax) > prop.sharedMemPerBlock)
        return cfail(nullptr, TTCF_EINVAL, "system exceeds the LDS of one workgroup");
    const size_t n = (size_t)dev.n, nw = (size_t)dev.n_wall;
    const size_t sbytes = channel_scratch_bytes(dev.n, dev.kmax);
    char* buf = (char*)rt_alloc(sizeof(double) * (3 * n + 3 * nw + 8) + sizeof(float) * 3 * n +
                                    sizeof(ChannelDesc) + sbytes + 1024, s);
    if (!buf) return cfail(nullptr, TTCF_ENOMEM, "allocation failed");
    double* d_r = (double*)buf;
    double* d_lat = d_r + 3 * n;
    double* d_out = d_lat + 3 * nw;
    float* d_f = (float*)(d_out + 8);
    ChannelDesc* d_desc = (ChannelDesc*)(((uintptr_t)(d_f + 3 * n) + 255) & ~(uintptr_t)255);
    char* d_scr = (char*)(((uintptr_t)(d_desc + 1) + 255) & ~(uintptr_t)255);
    ChannelDesc D{};
    D.r = d_r;
    D.f = d_f;
    D.latx = d_lat;
    D.laty = d_lat + nw;
    D.latz = d_lat + 2 * nw;
    D.v = 0.0;
    D.k = 0;
    ChannelLaunch L{};
    L.sys = dev;
    L.descs = d_desc;
    L.n_jobs = 1;
    L.grid = 1;
    L.cmax = cmax;
    L.scratch = d_scr;
    L.scratch_stride = sbytes;
    std::vector<float> fh(3 * n);
    auto step = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && g_free_err.empty()) g_free_err = std::string(what) + ": " + hipGetErrorString(e);
        return e == hipSuccess;
    };
    g_free_err.clear();
    (void)hipGetLastError();
    bool ok = step(hipMemcpyAsync(d_r, r, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s), "copy r") &&
              step(hipMemcpyAsync(d_lat, lattice, sizeof(double) * 3 * nw, hipMemcpyHostToDevice, s),
                   "copy lattice") &&
              step(hipMemcpyAsync(d_desc, &D, sizeof(D), hipMemcpyHostToDevice, s), "copy descriptor") &&
              step(launch_channel_debug_forces(L, d_out, s), "force kernel launch") &&
              step(hipMemcpyAsync(fh.data(), d_f, sizeof(float) * 3 * n, hipMemcpyDeviceToHost, s),
                   "copy forces") &&
              step(hipMemcpyAsync(out, d_out, sizeof(double) * 5, hipMemcpyDeviceToHost, s), "copy out") &&
              step(hipStreamSynchronize(s), "synchronise");
    rt_free(buf);
    if (!ok) return TTCF_EDEVICE;
    for (size_t i = 0; i < 3 * n; ++i) f[i] = fh[i];
    return TTCF_OK;
}

int32_t ttcf_channel_step_timing(ttcf_channel_ctx* c, double* total_ms, int64_t* launches,
                                 int32_t reset) {
    if (!c) return TTCF_EINVAL;
    for (auto& e : c->events) {
        CHK(c, hipEventSynchronize(e.second));
        float ms = 0.f;
        CHK(c, hipEventElapsedTime(&ms, e.first, e.second));
        c->step_ms += ms;
        c->launches += 1;
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    c->events.clear();
    if (total_ms) *total_ms = c->step_ms;
    if (launches) *launches = c->launches;
    if (reset) {
        c->step_ms = 0.0;
        c->launches = 0;
    }
    return TTCF_OK;
}

}  // extern "C"
