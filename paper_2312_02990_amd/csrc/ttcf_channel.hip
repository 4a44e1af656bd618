// ttcf_channel.hip -- gfx950 kernels of the confined-channel example (Eq. system2,
// Eq. TTCF2): a Lennard-Jones liquid between two walls whose atoms are tethered to lattice
// sites moving at +-v/2 along x, with a Nose-Hoover thermostat on the wall atoms.
//
// One workgroup integrates one trajectory at a time. The state (FP64 r and p, FP32 forces)
// stays in global memory: 18000 atoms do not fit in LDS. A step is a few coalesced passes
// over the atoms. Pair separations come from 32-bit fixed-point coordinates (periodic in x
// and z, so wrapped integer differences are minimum images; plain in y). Verlet lists of
// radius r_c + skin live in global scratch, rebuilt through an LDS counting sort when the
// largest path length since the last build reaches skin / 2. All reductions have a fixed
// order, and the momentum profile is summed as 64-bit fixed point: results are
// deterministic.
#include <hip/hip_runtime.h>

#include "ttcf_channel.h"

namespace ttcf {

namespace {

constexpr double kProfileScale = 1099511627776.0;  // 2^40: fixed point of the profile sums
constexpr int kChUnroll = 8;                         // list entries per trip of the force loop
constexpr int kChScanUnroll = 8;                     // candidates per trip of the list build

__device__ __forceinline__ uint32_t fixp(double v, double scale) {
    return (uint32_t)(int64_t)rint(v * scale);
}

__device__ __forceinline__ int cell_of(uint32_t q, int nc) {
    return (int)(((uint64_t)q * (uint64_t)nc) >> 32);
}

__device__ __forceinline__ double min_image(double d, double l) { return d - l * rint(d / l); }

template <int K>
__device__ __forceinline__ void ch_block_sum(double (&v)[K], double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double x = v[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        v[k] = x;
    }
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) red[wave * K + k] = v[k];
    __syncthreads();
    if (threadIdx.x < K) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w * K + threadIdx.x];
        red[kChMaxWaves * K + threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = red[kChMaxWaves * K + k];
    __syncthreads();
}

__device__ __forceinline__ float ch_block_max(float v, float* wmax) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
    __syncthreads();
    float m = 0.f;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, wmax[w]);
    __syncthreads();
    return m;
}

// Exclusive scan of cnt[0..C) into start[0..C) and into cnt (placement cursors).
__device__ void ch_scan(int32_t* cnt, int32_t* start, int C, int32_t* ws) {
    const int T = blockDim.x, t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6, nw = T >> 6;
    const int chunk = (C + T - 1) / T;
    const int b = min(t * chunk, C), e = min(b + chunk, C);
    int local = 0;
    for (int c = b; c < e; ++c) local += cnt[c];
    int x = local;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) ws[wave] = x;
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int w = 0; w < nw; ++w) {
            const int v = ws[w];
            ws[w] = run;
            run += v;
        }
    }
    __syncthreads();
    int run = ws[wave] + x - local;
    for (int c = b; c < e; ++c) {
        const int v = cnt[c];
        start[c] = run;
        cnt[c] = run;
        run += v;
    }
    __syncthreads();
}

struct ChLds {
    ChannelDev* sys;
    int32_t* cnt;      // [cmax]
    int32_t* start;    // [cmax + 1]
    uint16_t* sid;     // [nmax + 4]
    double* red;       // block reductions
    int32_t* ws;       // [kChMaxWaves]
    float* wmax;       // [kChMaxWaves]
    unsigned long long* bins;  // [kChMaxBins] profile sums (fixed point)
    int32_t* misc;     // [4]: job, list overflow, out of range
};

__host__ __device__ inline size_t ch_align(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct ChPlan {
    size_t sys, cnt, start, sid, red, ws, wmax, bins, misc, total;
};

__host__ __device__ inline ChPlan ch_plan(int nmax, int cmax) {
    ChPlan p;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = ch_align(off, 16);
        const size_t at = off;
        off += bytes;
        return at;
    };
    p.sys = take(sizeof(ChannelDev));
    p.cnt = take(4 * (size_t)cmax);
    p.start = take(4 * ((size_t)cmax + 1));
    p.sid = take(2 * ((size_t)nmax + 4));
    p.red = take(sizeof(double) * (kChMaxWaves + 1) * kChRed);
    p.ws = take(4 * kChMaxWaves);
    p.wmax = take(4 * kChMaxWaves);
    p.bins = take(8 * kChMaxBins);
    p.misc = take(16);
    p.total = ch_align(off, 128);
    return p;
}

__device__ inline ChLds ch_carve(char* base, int nmax, int cmax) {
    const ChPlan p = ch_plan(nmax, cmax);
    ChLds L;
    L.sys = (ChannelDev*)(base + p.sys);
    L.cnt = (int32_t*)(base + p.cnt);
    L.start = (int32_t*)(base + p.start);
    L.sid = (uint16_t*)(base + p.sid);
    L.red = (double*)(base + p.red);
    L.ws = (int32_t*)(base + p.ws);
    L.wmax = (float*)(base + p.wmax);
    L.bins = (unsigned long long*)(base + p.bins);
    L.misc = (int32_t*)(base + p.misc);
    return L;
}

// Per-workgroup global scratch: fixed-point positions in atom order and in list-grid order,
// lists, list lengths, path lengths. Lists and list lengths are indexed by list-grid slot
// (the position of the atom in the counting sort) and hold slots, so that the force pass
// walks the atoms cell by cell and a wave's gathers stay in a few neighbouring cells.
struct ChScratch {
    uint4* posq;       // [n] by atom  (X, Y, Z, type: 0 fluid, 1 bottom wall, 2 top wall)
    uint4* posq_s;     // [n] by slot: posq_s[i] = posq[sid[i]]
    uint16_t* nbr;     // [(kmax + 1) n] by slot, row kmax is a sink for rejected candidates
    uint16_t* ncnt;    // [n] by slot
    float* path;       // [n] by atom
};

__host__ __device__ inline size_t ch_scratch_bytes(int nmax, int kmax) {
    return 2 * ch_align(16 * (size_t)nmax, 256) + ch_align(2 * ((size_t)kmax + 1) * nmax, 256) +
           ch_align(2 * (size_t)nmax, 256) + ch_align(4 * (size_t)nmax, 256);
}

__device__ inline ChScratch ch_scratch(char* base, int nmax, int kmax) {
    ChScratch s;
    size_t off = 0;
    s.posq = (uint4*)(base + off);
    off += ch_align(16 * (size_t)nmax, 256);
    s.posq_s = (uint4*)(base + off);
    off += ch_align(16 * (size_t)nmax, 256);
    s.nbr = (uint16_t*)(base + off);
    off += ch_align(2 * ((size_t)kmax + 1) * nmax, 256);
    s.ncnt = (uint16_t*)(base + off);
    off += ch_align(2 * (size_t)nmax, 256);
    s.path = (float*)(base + off);
    return s;
}

__device__ __forceinline__ uint32_t atom_type(const ChannelDev& S, int a) {
    return a < S.n_fluid ? 0u : (a < S.n_fluid + S.n_wall / 2 ? 1u : 2u);
}

// fixed-point positions of every atom; flags atoms that left [0, y_extent)
__device__ void ch_publish(const ChannelDev& S, const double* r, const ChScratch& G,
                           const ChLds& L) {
    const int n = S.n;
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        const double y = r[n + a];
        if (!(y >= 0.0) || !(y < S.y_extent)) L.misc[2] = 1;
        const double yc = fmin(fmax(y, 0.0), S.y_extent * (1.0 - 1e-15));
        G.posq[a] = make_uint4(fixp(r[a], S.fix_scale[0]), fixp(yc, S.fix_scale[1]),
                               fixp(r[2 * n + a], S.fix_scale[2]), atom_type(S, a));
    }
}

// positions in list-grid order for the slots of the last list build (sid stays in LDS)
__device__ __forceinline__ void ch_gather_sorted(const ChannelDev& S, const ChScratch& G,
                                                 const ChLds& L) {
    for (int i = threadIdx.x; i < S.n; i += blockDim.x) G.posq_s[i] = G.posq[L.sid[i]];
}

__device__ __forceinline__ void ch_sep(const uint4& qa, const uint4& qb, const ChannelDev& S,
                                       float& dx, float& dy, float& dz) {
    dx = (float)(int32_t)(qa.x - qb.x) * S.fix_unit[0];
    dy = (float)(int32_t)(qa.y - qb.y) * S.fix_unit[1];
    dz = (float)(int32_t)(qa.z - qb.z) * S.fix_unit[2];
}

// Counting sort into the list grid (LDS), then every atom collects the atoms within
// r_c + skin over its 27-cell neighbourhood (no images in y). Wall-wall pairs are left out.
__device__ void ch_rebuild(const ChannelDev& S, const ChScratch& G, const ChLds& L) {
    const int n = S.n, T = blockDim.x, t = threadIdx.x;
    const int nc0 = S.lc[0], nc1 = S.lc[1], nc2 = S.lc[2];
    const int C = nc0 * nc1 * nc2;
    for (int c = t; c < C; c += T) L.cnt[c] = 0;
    if (t == 0) L.misc[1] = 0;
    __syncthreads();
    for (int a = t; a < n; a += T) {
        const uint4 q = G.posq[a];
        const int c = cell_of(q.x, nc0) + nc0 * (cell_of(q.y, nc1) + nc1 * cell_of(q.z, nc2));
        atomicAdd(&L.cnt[c], 1);
    }
    __syncthreads();
    ch_scan(L.cnt, L.start, C, L.ws);
    if (t == 0) L.start[C] = n;
    for (int a = t; a < n; a += T) {
        const uint4 q = G.posq[a];
        const int c = cell_of(q.x, nc0) + nc0 * (cell_of(q.y, nc1) + nc1 * cell_of(q.z, nc2));
        const int idx = atomicAdd(&L.cnt[c], 1);
        L.sid[idx] = (uint16_t)a;
    }
    __syncthreads();
    // the atoms of a cell in ascending id order: list order, and so every force sum, then does
    // not depend on the order in which the placement atomics ran
    for (int c = t; c < C; c += T) {
        const int b = L.start[c], e = L.start[c + 1];
        for (int i = b + 1; i < e; ++i) {
            const uint16_t v = L.sid[i];
            int q = i - 1;
            while (q >= b && L.sid[q] > v) {
                L.sid[q + 1] = L.sid[q];
                --q;
            }
            L.sid[q + 1] = v;
        }
    }
    __syncthreads();
    ch_gather_sorted(S, G, L);
    for (int a = t; a < n; a += T) G.path[a] = 0.f;
    __syncthreads();
    const float rl2 = S.rl2_f;
    const int kmax = S.kmax;
    bool over = false;
    for (int i = t; i < n; i += T) {
        const uint4 qa = G.posq_s[i];
        const int cx = cell_of(qa.x, nc0), cy = cell_of(qa.y, nc1), cz = cell_of(qa.z, nc2);
        const bool wall_a = qa.w != 0u;
        int count = 0;
        int slot = i;
        const int sink = kmax * n + i;
        auto scan = [&](int lo, int hi) {
            for (int tt = lo; tt < hi; tt += kChScanUnroll) {
                int jn[kChScanUnroll];
                uint4 q[kChScanUnroll];
#pragma unroll
                for (int u = 0; u < kChScanUnroll; ++u) jn[u] = tt + u < hi ? tt + u : i;
#pragma unroll
                for (int u = 0; u < kChScanUnroll; ++u) q[u] = G.posq_s[jn[u]];
#pragma unroll
                for (int u = 0; u < kChScanUnroll; ++u) {
                    float dx, dy, dz;
                    ch_sep(qa, q[u], S, dx, dy, dz);
                    const bool both_wall = wall_a & (q[u].w != 0u);
                    const bool hit = (jn[u] != i) & !both_wall &
                                     (dx * dx + dy * dy + dz * dz < rl2);
                    const bool room = hit & (count < kmax);
                    G.nbr[room ? slot : sink] = (uint16_t)jn[u];
                    slot += room ? n : 0;
                    count += hit ? 1 : 0;
                }
            }
        };
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = cy + dy;
            if (yy < 0 || yy >= nc1) continue;
            for (int dz = -1; dz <= 1; ++dz) {
                int zz = cz + dz;
                zz = zz < 0 ? zz + nc2 : (zz >= nc2 ? zz - nc2 : zz);
                const int base = nc0 * (yy + nc1 * zz);
                int x0 = cx - 1;
                if (x0 < 0) x0 += nc0;
                const int xe = x0 + 3;
                scan(L.start[base + x0], L.start[base + (xe < nc0 ? xe : nc0)]);
                if (xe > nc0) scan(L.start[base], L.start[base + xe - nc0]);
            }
        }
        if (count > kmax) {
            over = true;
            count = kmax;
        }
        G.ncnt[i] = (uint16_t)count;
    }
    if (over) L.misc[1] = 1;
    __syncthreads();
}

// Forces (LJ through the lists in FP32, tethers in FP64, the sum rounded once to FP32),
// walked in list-grid order: positions come from posq_s (filled for this step), forces go
// to the atom's own index. Partial sums of this thread: [0] x force on fluid from the top
// wall, [1] from the bottom wall, [2] S = sum_top dx - sum_bottom dx of the tether extensions.
__device__ void ch_forces(const ChannelDev& S, const double* r, float* f, const double* latx,
                          const double* laty, const double* latz, double v, int64_t k,
                          const ChScratch& G, const ChLds& L, double (&part)[3]) {
    const int n = S.n, nf = S.n_fluid;
    const float rc2 = S.rc2_f;
    const float cff = (float)S.c_ff, cwf = (float)S.c_wf;
    const double shift = 0.5 * v * ((double)k * S.dt);
    part[0] = part[1] = part[2] = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int a = L.sid[i];
        const uint4 qa = G.posq_s[i];
        const bool fluid_a = qa.w == 0u;
        const int cnt = G.ncnt[i];
        float gx = 0.f, gy = 0.f, gz = 0.f, wt = 0.f, wb = 0.f;
        // kChUnroll list entries per trip: their index loads, then their position gathers, are
        // issued together; entries past the list length read row 0 and add nothing
        for (int kk = 0; kk < cnt; kk += kChUnroll) {
            int j[kChUnroll];
            uint4 qb[kChUnroll];
#pragma unroll
            for (int u = 0; u < kChUnroll; ++u) j[u] = G.nbr[(kk + u < cnt ? kk + u : 0) * n + i];
#pragma unroll
            for (int u = 0; u < kChUnroll; ++u) qb[u] = G.posq_s[j[u]];
#pragma unroll
            for (int u = 0; u < kChUnroll; ++u) {
                float dx, dy, dz;
                ch_sep(qa, qb[u], S, dx, dy, dz);
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float cw = (fluid_a & (qb[u].w == 0u)) ? cff : cwf;
                const float inv = 1.0f / r2;
                const float s3 = inv * inv * inv;
                const bool in = (kk + u < cnt) & (r2 < rc2);
                const float fs = in ? s3 * (48.f * s3 - 24.f * cw) * inv : 0.f;
                gx += fs * dx;
                gy += fs * dy;
                gz += fs * dz;
                wt += (fluid_a & (qb[u].w == 2u)) ? fs * dx : 0.f;
                wb += (fluid_a & (qb[u].w == 1u)) ? fs * dx : 0.f;
            }
        }
        if (fluid_a) {
            f[a] = gx;
            f[n + a] = gy;
            f[2 * n + a] = gz;
            part[0] += (double)wt;
            part[1] += (double)wb;
        } else {
            const int q = a - nf;
            const bool top = qa.w == 2u;
            const double xl = latx[q] + (top ? shift : -shift);
            const double ex = min_image(r[a] - xl, S.lx);
            const double ey = r[n + a] - laty[q];
            const double ez = min_image(r[2 * n + a] - latz[q], S.lz);
            f[a] = (float)((double)gx - S.k_spring * ex);
            f[n + a] = (float)((double)gy - S.k_spring * ey);
            f[2 * n + a] = (float)((double)gz - S.k_spring * ez);
            part[2] += top ? ex : -ex;
        }
    }
}

__device__ void ch_write_observables(const ChannelDev& S, double fxt, double fxb, const ChLds& L,
                                     double* row) {
    const double area = S.lx * S.lz;
    for (int b = threadIdx.x; b <= S.n_bins; b += blockDim.x) {
        if (b == 0)
            row[0] = (fxt - fxb) / (2.0 * area);
        else
            row[b] = ((double)(long long)L.bins[b - 1] / kProfileScale) / (area * S.bin_w);
    }
}

__device__ __forceinline__ void ch_bin(const ChannelDev& S, double y, double px, const ChLds& L) {
    if (!(y >= S.bin_lo) || !(y < S.bin_hi)) return;
    int b = (int)floor((y - S.bin_lo) / S.bin_w);
    if (b > S.n_bins - 1) b = S.n_bins - 1;
    atomicAdd(&L.bins[b], (unsigned long long)llrint(px * kProfileScale));
}

__device__ void run_channel(ChannelDesc* d, int steps_cap, const ChScratch& G, const ChLds& L) {
    const ChannelDev& S = *L.sys;
    const int n = S.n, nf = S.n_fluid, T = blockDim.x, t = threadIdx.x;
    double* r = d->r;
    double* p = d->p;
    float* f = d->f;
    const double v = d->v;
    int64_t k = d->k;
    int done = d->done;
    int health = d->health;
    double zeta = d->zeta;
    double pw2 = d->pw2;
    const int todo = health != 0 ? 0 : min(steps_cap, d->n_steps - done);
    if (todo <= 0 && done > 0) return;
    const int nobs = 1 + S.n_bins;
    const double h = S.dt, tau = 0.5 * S.dt;
    if (t == 0) L.misc[2] = 0;
    __syncthreads();
    ch_publish(S, r, G, L);
    __syncthreads();
    ch_rebuild(S, G, L);
    if (L.misc[1] != 0) health |= kHealthListOverflow;
    if (done == 0) {
        // forces, S(0), sum of wall p^2 and the observables of the start state
        double part[3];
        ch_forces(S, r, f, d->latx, d->laty, d->latz, v, k, G, L, part);
        double w2 = 0.0;
        for (int b = t; b < S.n_bins; b += T) L.bins[b] = 0ull;
        __syncthreads();
        for (int a = t; a < n; a += T) {
            if (a >= nf)
                w2 += p[a] * p[a] + p[n + a] * p[n + a] + p[2 * n + a] * p[2 * n + a];
            else
                ch_bin(S, r[n + a], p[a], L);
        }
        double red4[4] = {part[0], part[1], part[2], w2};
        ch_block_sum<4>(red4, L.red);
        pw2 = red4[3];
        if (t == 0) d->s0 = red4[2];
        if (d->series) ch_write_observables(S, red4[0], red4[1], L, d->series);
        __syncthreads();
    }
    if (health != 0) {
        if (t == 0) d->health = health;
        return;
    }
    const float skin = (float)S.skin;
    for (int step = 0; step < todo; ++step) {
        // thermostat half step (walls), half kick, drift, periodic wrap in x and z
        zeta += tau * (pw2 - S.nf_w * S.temperature) / S.q;
        const double c1 = exp(-zeta * tau);
        float pmax = 0.f;
        for (int a = t; a < n; a += T) {
            double px = p[a], py = p[n + a], pz = p[2 * n + a];
            if (a >= nf) {
                px *= c1;
                py *= c1;
                pz *= c1;
            }
            px += tau * (double)f[a];
            py += tau * (double)f[n + a];
            pz += tau * (double)f[2 * n + a];
            double x = r[a] + h * px, y = r[n + a] + h * py, z = r[2 * n + a] + h * pz;
            x -= S.lx * floor(x / S.lx);
            if (x >= S.lx) x = 0.0;
            z -= S.lz * floor(z / S.lz);
            if (z >= S.lz) z = 0.0;
            r[a] = x;
            r[n + a] = y;
            r[2 * n + a] = z;
            p[a] = px;
            p[n + a] = py;
            p[2 * n + a] = pz;
            const float pl = G.path[a] + (float)(h * sqrt(px * px + py * py + pz * pz));
            G.path[a] = pl;
            pmax = fmaxf(pmax, pl);
        }
        k += 1;
        __syncthreads();
        ch_publish(S, r, G, L);
        const float dmax = ch_block_max(pmax, L.wmax);
        if (2.f * dmax * 1.0001f >= skin) {
            ch_rebuild(S, G, L);
            if (L.misc[1] != 0) {
                health |= kHealthListOverflow;
                break;
            }
        } else {
            ch_gather_sorted(S, G, L);
            __syncthreads();
        }
        double part[3];
        ch_forces(S, r, f, d->latx, d->laty, d->latz, v, k, G, L, part);
        for (int b = t; b < S.n_bins; b += T) L.bins[b] = 0ull;
        __syncthreads();
        // half kick, thermostat half step, observables
        const double c2 = exp(-zeta * tau);
        double w2 = 0.0;
        for (int a = t; a < n; a += T) {
            double px = p[a] + tau * (double)f[a];
            double py = p[n + a] + tau * (double)f[n + a];
            double pz = p[2 * n + a] + tau * (double)f[2 * n + a];
            if (a >= nf) {
                px *= c2;
                py *= c2;
                pz *= c2;
                w2 += px * px + py * py + pz * pz;
            } else {
                ch_bin(S, r[n + a], px, L);
            }
            p[a] = px;
            p[n + a] = py;
            p[2 * n + a] = pz;
        }
        double red3[3] = {part[0], part[1], w2};
        ch_block_sum<3>(red3, L.red);
        pw2 = red3[2];
        zeta += tau * (pw2 - S.nf_w * S.temperature) / S.q;
        done += 1;
        if (d->series) ch_write_observables(S, red3[0], red3[1], L, d->series + (size_t)done * nobs);
        if (!isfinite(pw2) || !isfinite(zeta)) {
            health |= kHealthNonFinite;
            break;
        }
        if (L.misc[2] != 0) {
            health |= kHealthNonFinite;
            break;
        }
        __syncthreads();
    }
    __syncthreads();
    if (t == 0) {
        d->k = k;
        d->done = done;
        d->health = health;
        d->zeta = zeta;
        d->pw2 = pw2;
    }
    __syncthreads();
}

// Four waves per SIMD (128 VGPRs, a 64-byte spill), two workgroups per CU: the gathers of the
// force loop need the waves to hide their latency. On 1024 daughters this measured 19% faster
// than the unconstrained 160-VGPR build (one workgroup per CU); three workgroups per CU leave
// a two-thirds-empty second round on such batches.
__global__ __launch_bounds__(kChThreads, kChWavesPerSimd) void k_channel(ChannelLaunch b) {
    extern __shared__ __align__(16) char smem[];
    const ChLds L = ch_carve(smem, b.sys.n, b.cmax);
    if (threadIdx.x == 0) *L.sys = b.sys;
    const ChScratch G = ch_scratch(b.scratch + (size_t)blockIdx.x * b.scratch_stride, b.sys.n,
                                   b.sys.kmax);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) L.misc[0] = atomicAdd(b.queue, 1);
        __syncthreads();
        const int j = __builtin_amdgcn_readfirstlane(L.misc[0]);
        if (j >= b.n_jobs) break;
        run_channel(&b.descs[b.order ? b.order[j] : j], b.max_steps, G, L);
    }
}

// ---- spawn: mapped copies of stored start states -----------------------------------------
// states: per state [r (3n) | p (3n) | zeta]; mapping 1 reverses p and zeta, 2 reflects x of
// atoms and lattice sites and reverses p_x, 3 does both (p_x unchanged).
__global__ void k_channel_spawn(const double* states, int32_t n, int32_t n_wall, double lx,
                                const double* latx0, ChannelDesc* descs, int32_t count) {
    const int d = blockIdx.x;
    if (d >= count) return;
    ChannelDesc& D = descs[d];
    const double* st = states + (size_t)D.state * ((size_t)6 * n + 1);
    const int m = D.map;
    const bool rev = m == 1 || m == 3, refl = m == 2 || m == 3;
    for (int i = threadIdx.x; i < 3 * n; i += blockDim.x) {
        double x = st[i];
        double pv = st[3 * n + i];
        const bool is_x = i < n;
        if (refl && is_x) x = x == 0.0 ? 0.0 : lx - x;
        if (rev) pv = -pv;
        if (refl && is_x) pv = -pv;
        D.r[i] = x;
        D.p[i] = pv;
    }
    for (int q = threadIdx.x; q < n_wall; q += blockDim.x) {
        const double x = latx0[q];
        D.latx[q] = refl ? (x == 0.0 ? 0.0 : lx - x) : x;
    }
    if (threadIdx.x == 0) {
        const double z = st[6 * (size_t)n];
        D.zeta = rev ? -z : z;
    }
}

// Replica q of the mother: its positions, and its momenta plus kick q (kicks may be null).
__global__ void k_channel_replicate(const double* r, const double* p, const double* kicks,
                                    int32_t n, ChannelDesc* descs, int32_t count) {
    const int q = blockIdx.x;
    if (q >= count) return;
    ChannelDesc& D = descs[q];
    const double* kq = kicks ? kicks + (size_t)q * 3 * n : nullptr;
    for (int i = threadIdx.x; i < 3 * n; i += blockDim.x) {
        D.r[i] = r[i];
        D.p[i] = kq ? p[i] + kq[i] : p[i];
    }
}

// Stored start state q * per + s: replica q's positions, momenta and thermostat variable.
__global__ void k_channel_snapshot(const ChannelDesc* descs, int32_t count, int32_t n,
                                   double* states, int32_t per, int32_t s) {
    const int q = blockIdx.x;
    if (q >= count) return;
    const ChannelDesc& D = descs[q];
    double* dst = states + ((size_t)q * per + s) * ((size_t)6 * n + 1);
    for (int i = threadIdx.x; i < 3 * n; i += blockDim.x) {
        dst[i] = D.r[i];
        dst[3 * n + i] = D.p[i];
    }
    if (threadIdx.x == 0) dst[6 * (size_t)n] = D.zeta;
}

// ---- accumulate and response (several observables per time point) ------------------------
// One thread per (group, observable): D(t) = mean_m B_m(t); I(t) = mean_m int_0^t S_m(0)
// B_m(s) ds (trapezoid, compensated); the start state's TTCF series is D(0) - coef I(t).
__global__ void k_channel_accumulate(ChannelAccum a) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= a.n_groups * a.n_obs) return;
    const int g = id / a.n_obs, o = id % a.n_obs;
    const int b = a.first_of[g], e = a.first_of[g + 1];
    const int nm = min(e - b, 4);
    double s0[4], sum[4], comp[4], prev[4];
    const double* ser[4];
    for (int m = 0; m < nm; ++m) {
        const ChannelDesc& d = a.descs[b + m];
        ser[m] = d.series;
        s0[m] = d.s0;
        prev[m] = d.series[o];
        sum[m] = 0.0;
        comp[m] = 0.0;
    }
    const double inm = 1.0 / (double)nm;
    double* dout = a.d_out + (size_t)g * a.row_stride;
    double* iout = a.i_out + (size_t)g * a.row_stride;
    double d0 = 0.0;
    for (int m = 0; m < nm; ++m) d0 += prev[m];
    dout[o] = d0 * inm;
    iout[o] = 0.0;
    for (int k = 1; k < a.n_t; ++k) {
        double dsum = 0.0, isum = 0.0;
        for (int m = 0; m < nm; ++m) {
            const double cur = ser[m][(size_t)k * a.n_obs + o];
            const double add = 0.5 * a.dt * (s0[m] * prev[m] + s0[m] * cur);
            const double ts = sum[m] + add;
            comp[m] += fabs(sum[m]) >= fabs(add) ? (sum[m] - ts) + add : (add - ts) + sum[m];
            sum[m] = ts;
            prev[m] = cur;
            dsum += cur;
            isum += sum[m] + comp[m];
        }
        dout[(size_t)k * a.n_obs + o] = dsum * inm;
        iout[(size_t)k * a.n_obs + o] = isum * inm;
    }
}

// One thread per (t, observable column): mean and block standard error over the rows.
__global__ void k_channel_response(ChannelResponse r) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= r.n_t * r.n_cols) return;
    const int k = id / r.n_cols, o = r.col0 + id % r.n_cols;
    auto neu = [](double& s, double& c, double v) {
        const double ts = s + v;
        c += fabs(s) >= fabs(v) ? (s - ts) + v : (v - ts) + s;
        s = ts;
    };
    double gs = 0, gc = 0, ds = 0, dc = 0;
    for (int i = 0; i < r.n_rows; ++i) {
        const int row = r.rows[i];
        const double* dd = r.d_all + (size_t)row * r.row_stride;
        const double* ii = r.i_all + (size_t)row * r.row_stride;
        neu(gs, gc, dd[o] - r.coef[row] * ii[(size_t)k * r.n_obs + o]);
        neu(ds, dc, dd[(size_t)k * r.n_obs + o]);
    }
    const double gm = (gs + gc) / r.n_rows, dm = (ds + dc) / r.n_rows;
    double gv = 0, gvc = 0, dv = 0, dvc = 0;
    for (int i = 0; i < r.n_rows; ++i) {
        const int row = r.rows[i];
        const double* dd = r.d_all + (size_t)row * r.row_stride;
        const double* ii = r.i_all + (size_t)row * r.row_stride;
        const double g = dd[o] - r.coef[row] * ii[(size_t)k * r.n_obs + o] - gm;
        const double x = dd[(size_t)k * r.n_obs + o] - dm;
        neu(gv, gvc, g * g);
        neu(dv, dvc, x * x);
    }
    const double denom = r.n_rows > 1 ? (double)(r.n_rows - 1) * (double)r.n_rows : 1.0;
    const size_t out = (size_t)k * r.n_cols + (o - r.col0);
    const size_t plane = (size_t)r.n_t * r.n_cols;
    r.out[out] = gm;
    r.out[plane + out] = r.n_rows > 1 ? sqrt((gv + gvc) / denom) : 0.0;
    r.out[2 * plane + out] = dm;
    r.out[3 * plane + out] = r.n_rows > 1 ? sqrt((dv + dvc) / denom) : 0.0;
}

// Forces of one configuration (tests): the list build and force passes of the step kernel.
__global__ __launch_bounds__(kChThreads) void k_channel_debug_forces(ChannelLaunch b,
                                                                     double* out) {
    extern __shared__ __align__(16) char smem[];
    const ChLds L = ch_carve(smem, b.sys.n, b.cmax);
    if (threadIdx.x == 0) {
        *L.sys = b.sys;
        L.misc[2] = 0;
    }
    __syncthreads();
    const ChannelDev& S = *L.sys;
    const ChScratch G = ch_scratch(b.scratch, S.n, S.kmax);
    ChannelDesc& d = b.descs[0];
    ch_publish(S, d.r, G, L);
    __syncthreads();
    ch_rebuild(S, G, L);
    double part[3];
    ch_forces(S, d.r, d.f, d.latx, d.laty, d.latz, d.v, d.k, G, L, part);
    ch_block_sum<3>(part, L.red);
    if (threadIdx.x == 0) {
        out[0] = part[0];
        out[1] = part[1];
        out[2] = part[2];
        out[3] = (double)L.misc[1];
        out[4] = (double)L.misc[2];
    }
}

}  // namespace

size_t channel_lds_bytes(int nmax, int cmax) { return ch_plan(nmax, cmax).total; }
size_t channel_scratch_bytes(int nmax, int kmax) { return ch_scratch_bytes(nmax, kmax); }

hipError_t launch_channel(const ChannelLaunch& b, hipStream_t s) {
    const size_t lds = ch_plan(b.sys.n, b.cmax).total;
    (void)hipFuncSetAttribute((const void*)k_channel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    hipLaunchKernelGGL(k_channel, dim3(b.grid), dim3(kChThreads), lds, s, b);
    return hipGetLastError();
}

hipError_t launch_channel_debug_forces(const ChannelLaunch& b, double* out, hipStream_t s) {
    const size_t lds = ch_plan(b.sys.n, b.cmax).total;
    (void)hipFuncSetAttribute((const void*)k_channel_debug_forces,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_channel_debug_forces, dim3(1), dim3(kChThreads), lds, s, b, out);
    return hipGetLastError();
}

hipError_t launch_channel_spawn(const double* states, int32_t n, int32_t n_wall, double lx,
                                const double* latx0, ChannelDesc* descs, int32_t count,
                                hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_channel_spawn, dim3(count), dim3(256), 0, s, states, n, n_wall, lx, latx0,
                       descs, count);
    return hipGetLastError();
}

hipError_t launch_channel_replicate(const double* r, const double* p, const double* kicks,
                                    int32_t n, ChannelDesc* descs, int32_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_channel_replicate, dim3(count), dim3(256), 0, s, r, p, kicks, n, descs,
                       count);
    return hipGetLastError();
}

hipError_t launch_channel_snapshot(const ChannelDesc* descs, int32_t count, int32_t n,
                                   double* states, int32_t per, int32_t slot, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_channel_snapshot, dim3(count), dim3(256), 0, s, descs, count, n, states,
                       per, slot);
    return hipGetLastError();
}

hipError_t launch_channel_accumulate(const ChannelAccum& a, hipStream_t s) {
    const int total = a.n_groups * a.n_obs;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_channel_accumulate, dim3((total + 63) / 64), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_channel_response(const ChannelResponse& r, hipStream_t s) {
    const int total = r.n_t * r.n_cols;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_channel_response, dim3((total + 63) / 64), dim3(64), 0, s, r);
    return hipGetLastError();
}

}  // namespace ttcf
