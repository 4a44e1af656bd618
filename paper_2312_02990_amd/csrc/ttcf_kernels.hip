// ttcf_kernels.hip -- gfx950 kernels of the TTCF daughter path (arxiv 2312.02990).
//
// One workgroup owns one trajectory (a daughter, or the mother). Positions and momenta live
// in FP64 registers of their owner thread (atom a belongs to thread a % T); the cell list is
// rebuilt in LDS every step (counting sort, canonical (cell, atom id) order), and the pair
// forces are evaluated one sorted slot per thread over the 27-cell neighbourhood, whose rows
// across the y boundary are displaced by the Lees-Edwards offset. Pair separations are
// formed from coordinates relative to the owning cell's corner, so the FP32 force form loses
// no precision to the absolute coordinate. All reductions are fixed-order wavefront butterflies
// followed by a fixed-order sum over waves: results are deterministic.
#include <hip/hip_runtime.h>

#include "ttcf_internal.h"

namespace ttcf {

// ---------------------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------------------

template <typename Real> struct Vec4;
template <> struct Vec4<float> { using T = float4; };
template <> struct Vec4<double> { using T = double4; };

__device__ __forceinline__ float pack_cell(float, int v) { return __int_as_float(v); }
__device__ __forceinline__ double pack_cell(double, int v) { return (double)v; }
__device__ __forceinline__ int unpack_cell(float w) { return __float_as_int(w); }
__device__ __forceinline__ int unpack_cell(double w) { return (int)w; }

// Reciprocal: hardware estimate refined by Newton steps to (near) correct rounding.
__device__ __forceinline__ float recip(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    float e = __builtin_fmaf(-x, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// Cell coordinate of one FP64 coordinate: floor(v * (n / L)), clamped. A lone product,
// so nothing can be contracted and the result is bit-identical to any IEEE evaluation.
__device__ __forceinline__ int cell_coord(double v, double inv_w, int nc) {
    int c = (int)floor(v * inv_w);
    return c < 0 ? 0 : (c > nc - 1 ? nc - 1 : c);
}

__device__ __forceinline__ double wrap1(double x, double l) {
    if (x >= l) {
        x -= l;
        if (x >= l) x -= l * floor(x / l);
    } else if (x < 0.0) {
        x += l;
        if (x < 0.0) x -= l * floor(x / l);
        if (x >= l) x = 0.0;
    }
    return x;
}

// Lees-Edwards offset fmod(gamma_dot L_y (k dt), L_x), from the integer step counter. The
// remainder v - q L_x of the right integer q is exactly representable, so one fused
// multiply-add gives it exactly (the same bits as fmod); q from the rounded quotient can be
// off by one, which the two checks correct.
__device__ __forceinline__ double le_offset(const SysDev& S, double gamma_dot, int64_t k) {
    const double v = gamma_dot * S.box[1] * ((double)k * S.dt);
    const double lx = S.box[0];
    const double av = fabs(v);
    if (av < lx) return v;
    const double q = floor(av / lx);
    double r = __builtin_fma(-lx, q, av);
    if (r < 0.0)
        r = __builtin_fma(-lx, q - 1.0, av);
    else if (r >= lx)
        r = __builtin_fma(-lx, q + 1.0, av);
    return v < 0.0 ? -r : r;
}

// Sliding-brick wrap of one atom after a move (y crossing shifts x by -+ dxle).
__device__ __forceinline__ void wrap_le(const SysDev& S, double dxle, double& x, double& y,
                                        double& z) {
    if (y >= S.box[1]) {
        y -= S.box[1];
        x -= dxle;
    } else if (y < 0.0) {
        y += S.box[1];
        x += dxle;
        if (y >= S.box[1]) y = 0.0;
    }
    x = wrap1(x, S.box[0]);
    z = wrap1(z, S.box[2]);
}

// ---------------------------------------------------------------------------------------
// LDS layout
// ---------------------------------------------------------------------------------------

template <typename Real>
struct Lds {
    typename Vec4<Real>::T* spos;  // [nmax] sorted cell-relative positions, .w = packed cell
    Real* ax;                      // [nmax] per atom id: relative x, later F_x
    Real* ay;
    Real* az;
    double* red;                   // block-reduction scratch
    Real* shx;                     // [3 rows][5] x shift of each stencil column
    Real* shyz;                    // [6]: y shifts (dy = -1,0,1), z shifts
    int32_t* rowinfo;              // [3 rows][2]: first column offset mod nx, column count
    int32_t* cnt;                  // [cmax] counts, then placement cursors
    int32_t* start;                // [cmax + 1]
    uint16_t* sid;                 // [nmax] atom ids in canonical order
    int32_t* scan;                 // [kMaxWaves]
    int32_t* misc;                 // [4]
    SysDev* sys;                   // the trajectory's system constants (read from LDS, so
                                   // they do not occupy registers across the step loop)
};

struct LdsPlan {
    size_t spos, ax, ay, az, red, shx, shyz, rowinfo, cnt, start, sid, scan, misc, sys, total;
};

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) & ~(a - 1); }

__host__ __device__ inline LdsPlan plan_lds(int nmax, int cmax, size_t real_bytes) {
    LdsPlan p;
    size_t off = 0;
    auto take = [&](size_t bytes, size_t al) {
        off = align_up(off, al);
        size_t at = off;
        off += bytes;
        return at;
    };
    p.spos = take(4 * real_bytes * (size_t)nmax, 32);
    p.ax = take(real_bytes * (size_t)nmax, 16);
    p.ay = take(real_bytes * (size_t)nmax, 16);
    p.az = take(real_bytes * (size_t)nmax, 16);
    p.red = take(sizeof(double) * (kMaxWaves * kRedSlots + kRedSlots), 16);
    p.shx = take(real_bytes * 16, 16);
    p.shyz = take(real_bytes * 8, 16);
    p.rowinfo = take(sizeof(int32_t) * 8, 16);
    p.cnt = take(sizeof(int32_t) * (size_t)cmax, 16);
    p.start = take(sizeof(int32_t) * (size_t)(cmax + 1), 16);
    p.sid = take(sizeof(uint16_t) * (size_t)nmax, 16);
    p.scan = take(sizeof(int32_t) * kMaxWaves, 16);
    p.misc = take(sizeof(int32_t) * 4, 16);
    p.sys = take(sizeof(SysDev), 16);
    p.total = align_up(off, 128);
    return p;
}

template <typename Real>
__device__ inline Lds<Real> carve(char* base, int nmax, int cmax) {
    LdsPlan p = plan_lds(nmax, cmax, sizeof(Real));
    Lds<Real> L;
    L.spos = (typename Vec4<Real>::T*)(base + p.spos);
    L.ax = (Real*)(base + p.ax);
    L.ay = (Real*)(base + p.ay);
    L.az = (Real*)(base + p.az);
    L.red = (double*)(base + p.red);
    L.shx = (Real*)(base + p.shx);
    L.shyz = (Real*)(base + p.shyz);
    L.rowinfo = (int32_t*)(base + p.rowinfo);
    L.cnt = (int32_t*)(base + p.cnt);
    L.start = (int32_t*)(base + p.start);
    L.sid = (uint16_t*)(base + p.sid);
    L.scan = (int32_t*)(base + p.scan);
    L.misc = (int32_t*)(base + p.misc);
    L.sys = (SysDev*)(base + p.sys);
    return L;
}

// ---------------------------------------------------------------------------------------
// block-level collectives
// ---------------------------------------------------------------------------------------

// One 32-bit DPP move (lanes without a source keep `old`).
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp32(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xf, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = dpp32<CTRL, ROWS>(0u, (uint32_t)u);
    const uint32_t hi = dpp32<CTRL, ROWS>(0u, (uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Inclusive sum over the wave with row shifts (1, 2, 4, 8 inside rows of 16) and row
// broadcasts (15, 31): lane 63 ends with the wave total. VALU data-parallel moves, no LDS.
__device__ __forceinline__ double wave_total_dpp(double x) {
    x += dpp_f64<0x111, 0xf>(x);  // row_shr:1
    x += dpp_f64<0x112, 0xf>(x);  // row_shr:2
    x += dpp_f64<0x114, 0xf>(x);  // row_shr:4
    x += dpp_f64<0x118, 0xf>(x);  // row_shr:8
    x += dpp_f64<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
    x += dpp_f64<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
    return x;
}

// The same for the maximum of non-negative floats (0 is the identity).
__device__ __forceinline__ float wave_max_dpp(float x) {
    auto step = [](float a, uint32_t b) { return fmaxf(a, __builtin_bit_cast(float, b)); };
    x = step(x, dpp32<0x111, 0xf>(0u, __builtin_bit_cast(uint32_t, x)));
    x = step(x, dpp32<0x112, 0xf>(0u, __builtin_bit_cast(uint32_t, x)));
    x = step(x, dpp32<0x114, 0xf>(0u, __builtin_bit_cast(uint32_t, x)));
    x = step(x, dpp32<0x118, 0xf>(0u, __builtin_bit_cast(uint32_t, x)));
    x = step(x, dpp32<0x142, 0xa>(0u, __builtin_bit_cast(uint32_t, x)));
    x = step(x, dpp32<0x143, 0xc>(0u, __builtin_bit_cast(uint32_t, x)));
    return x;
}

// Sum K doubles over the workgroup; every thread receives the totals. Fixed order: a scan
// inside each wave (its total in lane 63), then wave 0..W-1 in sequence.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_total_dpp(v[k]);
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[wave * K + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < K) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w * K + threadIdx.x];
        red[kMaxWaves * kRedSlots + threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = red[kMaxWaves * kRedSlots + k];
}

// Exclusive scan of cnt[0..C) into start[0..C) (and into cnt as placement cursors).
__device__ __forceinline__ void scan_cells(int32_t* cnt, int32_t* start, int C, int32_t* ws) {
    const int T = blockDim.x, t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6, nw = T >> 6;
    const int chunk = (C + T - 1) / T;
    const int b = t * chunk;
    const int e = min(C, b + chunk);
    int local = 0;
    for (int c = b; c < e; ++c) local += cnt[c];
    int x = local;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) ws[wave] = x;
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int w = 0; w < nw; ++w) {
            int v = ws[w];
            ws[w] = acc;
            acc += v;
        }
    }
    __syncthreads();
    int run = ws[wave] + x - local;
    for (int c = b; c < e; ++c) {
        int v = cnt[c];
        start[c] = run;
        cnt[c] = run;
        run += v;
    }
}

// ---------------------------------------------------------------------------------------
// cell list (steps 1-4) and pair forces (step 5)
// ---------------------------------------------------------------------------------------

// Shift tables of the stencil. Row 1: columns cx-1..cx+1 of a row that does not cross the y
// boundary. Rows 0/2: the row below/above the box, an image displaced by -dxle/+dxle in x;
// its columns are every cell whose image overlaps [cx w - rc, (cx+1) w + rc] (plus a margin
// that covers the FP32 cutoff test), which is cx + off .. cx + off + nq - 1, independent of cx.
// Column q of a row has x shift S = -(off + q) w - sh, with sh the row's image displacement
// reduced to [-Lx/2, Lx/2]; the separation is then d_x = (u_i - u_j) + S.
template <typename Real>
__device__ void build_shift_tables(const SysDev& S, double dxle, const Lds<Real>& L) {
    const double wx = S.w[0];
    const double margin = 1e-6 * S.rc;
    for (int row = 0; row < 3; ++row) {
        int off, nq;
        double sh;
        if (row == 1) {
            off = -1;
            nq = 3;
            sh = 0.0;
        } else {
            double img = row == 0 ? -1.0 : 1.0;
            sh = img * dxle;
            sh -= S.box[0] * rint(sh / S.box[0]);
            off = (int)floor((-S.rc - margin - sh) / wx);
            int hi = (int)floor((wx + S.rc + margin - sh) / wx);
            nq = hi - off + 1;
            if (nq > 5) nq = 5;
            if (nq > S.nc[0]) nq = S.nc[0];
        }
        int offm = ((off % S.nc[0]) + S.nc[0]) % S.nc[0];
        L.rowinfo[2 * row] = offm;
        L.rowinfo[2 * row + 1] = nq;
        for (int q = 0; q < 5; ++q) L.shx[row * 5 + q] = (Real)(-(double)(off + q) * wx - sh);
    }
    for (int d = 0; d < 3; ++d) {
        L.shyz[d] = (Real)(-(double)(d - 1) * S.w[1]);
        L.shyz[3 + d] = (Real)(-(double)(d - 1) * S.w[2]);
    }
}

// Steps 1-4: cell of every atom, relative coordinates, counting sort into canonical order,
// sorted positions. Leaves cnt[] zeroed. cell_out (may be null) receives each owned atom's cell.
template <typename Real, int APT>
__device__ void build_cells(const SysDev& S, double dxle, const double (&x)[APT],
                            const double (&y)[APT], const double (&z)[APT], const Lds<Real>& L,
                            int (&cell)[APT]) {
    const int T = blockDim.x, t = threadIdx.x, n = S.n;
    const int nc0 = S.nc[0], nc1 = S.nc[1], nc2 = S.nc[2];
    const int C = nc0 * nc1 * nc2;
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        cell[j] = -1;
        if (a < n) {
            const int cx = cell_coord(x[j], S.inv_w[0], nc0);
            const int cy = cell_coord(y[j], S.inv_w[1], nc1);
            const int cz = cell_coord(z[j], S.inv_w[2], nc2);
            cell[j] = cx + nc0 * (cy + nc1 * cz);
            L.ax[a] = (Real)(x[j] - (double)cx * S.w[0]);
            L.ay[a] = (Real)(y[j] - (double)cy * S.w[1]);
            L.az[a] = (Real)(z[j] - (double)cz * S.w[2]);
            atomicAdd(&L.cnt[cell[j]], 1);
        }
    }
    if (t == 0) build_shift_tables<Real>(S, dxle, L);
    __syncthreads();
    scan_cells(L.cnt, L.start, C, L.scan);
    if (t == 0) L.start[C] = n;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        if (cell[j] >= 0) {
            const int idx = atomicAdd(&L.cnt[cell[j]], 1);
            L.sid[idx] = (uint16_t)(t + j * T);
        }
    }
    __syncthreads();
    for (int c = t; c < C; c += T) {
        const int b = L.start[c], e = L.start[c + 1];
        for (int i = b + 1; i < e; ++i) {  // insertion sort: cells hold a handful of atoms
            const uint16_t v = L.sid[i];
            int k = i - 1;
            while (k >= b && L.sid[k] > v) {
                L.sid[k + 1] = L.sid[k];
                --k;
            }
            L.sid[k + 1] = v;
        }
        const int cx = c % nc0, cy = (c / nc0) % nc1, cz = c / (nc0 * nc1);
        const int pk = cx | (cy << 10) | (cz << 20);
        for (int i = b; i < e; ++i) {
            const int a = L.sid[i];
            typename Vec4<Real>::T v;
            v.x = L.ax[a];
            v.y = L.ay[a];
            v.z = L.az[a];
            v.w = pack_cell(Real(0), pk);
            L.spos[i] = v;
        }
        L.cnt[c] = 0;
    }
    __syncthreads();
}

// Step 5: forces of every sorted slot, written per atom id into ax/ay/az; returns this
// thread's share of W_xy = sum_{i<j} x_ij F_y,ij (and U when want_u).
template <typename Real, bool WantU>
__device__ void pair_forces(const SysDev& S, const Lds<Real>& L, double& wpart, double& upart) {
    const int T = blockDim.x, t = threadIdx.x, n = S.n;
    const int nc0 = S.nc[0], nc1 = S.nc[1], nc2 = S.nc[2];
    const Real rc2 = (Real)S.rc2;
    const Real ca = (Real)S.c_attr;
    const Real ush = (Real)S.u_shift;
    double wacc = 0.0, uacc = 0.0;
    for (int s = t; s < n; s += T) {
        const typename Vec4<Real>::T ui = L.spos[s];
        const int pk = unpack_cell(ui.w);
        const int cx = pk & 1023, cy = (pk >> 10) & 1023, cz = pk >> 20;
        Real fx = 0, fy = 0, fz = 0, wxy = 0, ue = 0;
#pragma unroll 1
        for (int dz = 0; dz < 3; ++dz) {
            int zz = cz + dz - 1;
            zz = zz < 0 ? zz + nc2 : (zz >= nc2 ? zz - nc2 : zz);
            const Real sz = L.shyz[3 + dz];
#pragma unroll 1
            for (int dy = 0; dy < 3; ++dy) {
                int yy = cy + dy - 1;
                int row = 1;
                if (yy < 0) {
                    yy += nc1;
                    row = 0;
                } else if (yy >= nc1) {
                    yy -= nc1;
                    row = 2;
                }
                const Real sy = L.shyz[dy];
                const int nq = L.rowinfo[2 * row + 1];
                int xx = cx + L.rowinfo[2 * row];
                if (xx >= nc0) xx -= nc0;
                const int base = nc0 * (yy + nc1 * zz);
#pragma unroll 1
                for (int q = 0; q < nq; ++q) {
                    const Real sx = L.shx[row * 5 + q];
                    const int c = base + xx;
                    const int e = L.start[c + 1];
                    for (int tt = L.start[c]; tt < e; ++tt) {
                        if (tt == s) continue;
                        const typename Vec4<Real>::T uj = L.spos[tt];
                        const Real dx = (ui.x - uj.x) + sx;
                        const Real dyv = (ui.y - uj.y) + sy;
                        const Real dzv = (ui.z - uj.z) + sz;
                        const Real r2 = dx * dx + dyv * dyv + dzv * dzv;
                        if (r2 < rc2) {
                            const Real inv = recip(r2);
                            const Real s3 = inv * inv * inv;
                            const Real fs = s3 * (Real(48) * s3 - Real(24) * ca) * inv;
                            fx += fs * dx;
                            fy += fs * dyv;
                            fz += fs * dzv;
                            wxy += dx * (fs * dyv);
                            if (WantU) ue += Real(4) * s3 * (s3 - ca) + ush;
                        }
                    }
                    ++xx;
                    if (xx >= nc0) xx -= nc0;
                }
            }
        }
        const int i = L.sid[s];
        L.ax[i] = fx;
        L.ay[i] = fy;
        L.az[i] = fz;
        wacc += (double)wxy;
        if (WantU) uacc += (double)ue;
    }
    wpart = 0.5 * wacc;  // every unordered pair was visited from both sides
    upart = 0.5 * uacc;
    __syncthreads();
}

// Full force evaluation for the owned atoms.
template <typename Real, int APT, bool WantU>
__device__ void compute_forces(const SysDev& S, double dxle, const double (&x)[APT],
                               const double (&y)[APT], const double (&z)[APT], double (&fx)[APT],
                               double (&fy)[APT], double (&fz)[APT], double& wpart, double& upart,
                               const Lds<Real>& L) {
    int cell[APT];
    build_cells<Real, APT>(S, dxle, x, y, z, L, cell);
    pair_forces<Real, WantU>(S, L, wpart, upart);
    const int T = blockDim.x, t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        if (a < S.n) {
            fx[j] = (double)L.ax[a];
            fy[j] = (double)L.ay[a];
            fz[j] = (double)L.az[a];
        } else {
            fx[j] = fy[j] = fz[j] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------------------
// isokinetic integrator coefficients
// ---------------------------------------------------------------------------------------

// Exact flow over tau of dp/dt = F - (F.p/p.p) p with F fixed: p -> (p + F s)/sdot,
// s = (a/b)(cosh(q tau) - 1) + sinh(q tau)/q, sdot = (a/q) sinh(q tau) + cosh(q tau),
// a = F.p/p.p, b = F.F/p.p, q = sqrt(b) (Zhang, J. Chem. Phys. 106, 6102 (1997)).
// With u = b tau^2 = (q tau)^2 the two combinations needed are power series in u:
//   (cosh(q tau) - 1)/b = tau^2 (1/2 + u/24 + u^2/720 + ...)
//   sinh(q tau)/q       = tau   (1 + u/6 + u^2/120 + ...)
// Seven terms reach double precision for u < 0.04 (q tau < 0.2, the usual regime: the
// first omitted term is below 1e-17 of the sum); larger arguments use the library sinh.
__device__ __forceinline__ void iso_kick_coeffs(double a, double b, double tau, double& s,
                                                double& sdot) {
    double ch1_b, sh_q;
    const double u = b * tau * tau;
    if (u < 0.04) {
        // Horner forms of the two series, coefficients 2/(2k+2)! and 1/(2k+1)!
        double c = 1.0 / 87178291200.0;  // 1/14!
        c = c * u + 1.0 / 479001600.0;   // 1/12!
        c = c * u + 1.0 / 3628800.0;     // 1/10!
        c = c * u + 1.0 / 40320.0;       // 1/8!
        c = c * u + 1.0 / 720.0;         // 1/6!
        c = c * u + 1.0 / 24.0;          // 1/4!
        c = c * u + 0.5;                 // 1/2!
        double d = 1.0 / 1307674368000.0;  // 1/15!
        d = d * u + 1.0 / 6227020800.0;    // 1/13!
        d = d * u + 1.0 / 39916800.0;      // 1/11!
        d = d * u + 1.0 / 362880.0;        // 1/9!
        d = d * u + 1.0 / 5040.0;          // 1/7!
        d = d * u + 1.0 / 120.0;           // 1/5!
        d = d * u + 1.0 / 6.0;             // 1/3!
        d = d * u + 1.0;
        ch1_b = tau * tau * c;
        sh_q = tau * d;
    } else {
        const double q = sqrt(b);
        const double hs = sinh(0.5 * q * tau) / q;
        ch1_b = 2.0 * hs * hs;
        sh_q = sinh(q * tau) / q;
    }
    s = a * ch1_b + sh_q;
    sdot = a * sh_q + (1.0 + b * ch1_b);
}

// ---------------------------------------------------------------------------------------
// daughter: isokinetic SLLOD under Lees-Edwards boundaries
// ---------------------------------------------------------------------------------------
//
// Step (h = dt, tau = h/2, tg = tau gamma_dot), the symmetric splitting
//   S(tau) K(tau) D(h) [forces] K(tau) S(tau)
// with S the shear flow px -= tg py and K the force kick, both carrying the Gaussian
// multiplier (so both keep sum p.p), and D the streaming flow x += h px + h gamma_dot (y +
// tau py), y += h py, z += h pz. S under the constraint is the plain shear scaled back to the
// old p.p; K is the closed-form kick above. The scalars each part needs are moments of (p, F):
// the moments reduced once after the force pass give, in closed form, those of the second
// half and of the next step's first half, so the step needs a single block reduction.
template <typename Real, int APT, bool NH>
__device__ void run_daughter(DaughterDesc* dsc, int steps_cap, const Lds<Real>& L) {
    const int T = blockDim.x, t = threadIdx.x;
    if (t == 0) *L.sys = dsc->sys;
    __syncthreads();
    const SysDev& S = *L.sys;
    const int n = S.n;
    double* st = dsc->state;
    const double gd = dsc->gamma_dot;
    int64_t k = dsc->k;
    int done = dsc->done;
    const int n_steps = dsc->n_steps;
    double k0 = dsc->k0;
    int health = dsc->health;
    // Nose-Hoover daughters (Eq. system1 as printed): zeta from the mapped start state
    constexpr bool nh = NH;  // the descriptor's thermo selects the instantiation
    double zt = dsc->zeta;
    const double nh_iq = nh ? 1.0 / dsc->nh_q : 0.0, nh_tgt = dsc->nh_target;
    int todo = min(steps_cap, n_steps - done);
    if (health != 0) todo = 0;
    if (todo <= 0 && done > 0) return;

    double x[APT], y[APT], z[APT], px[APT], py[APT], pz[APT], fx[APT], fy[APT], fz[APT];
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        const bool v = a < n;
        x[j] = v ? st[a] : 0.0;
        y[j] = v ? st[n + a] : 0.0;
        z[j] = v ? st[2 * n + a] : 0.0;
        px[j] = v ? st[3 * n + a] : 0.0;
        py[j] = v ? st[4 * n + a] : 0.0;
        pz[j] = v ? st[5 * n + a] : 0.0;
    }
    double dxle = le_offset(S, gd, k);
    double wpart, upart;
    compute_forces<Real, APT, false>(S, dxle, x, y, z, fx, fy, fz, wpart, upart, L);

    // prologue moments: pp, pxpy, pypy, fp, fxpy, ff, W
    double m0[7] = {0, 0, 0, 0, 0, 0, wpart};
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        m0[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
        m0[1] += px[j] * py[j];
        m0[2] += py[j] * py[j];
        m0[3] += fx[j] * px[j] + fy[j] * py[j] + fz[j] * pz[j];
        m0[4] += fx[j] * py[j];
        m0[5] += fx[j] * fx[j] + fy[j] * fy[j] + fz[j] * fz[j];
    }
    block_sum<7>(m0, L.red);
    if (done == 0) {
        if (k0 <= 0.0) k0 = 0.5 * m0[0];
        if (t == 0) dsc->series[0] = m0[1] + m0[6];
    }
    double pp = m0[0], pxpy = m0[1], pypy = m0[2], fp = m0[3], fxpy = m0[4], ff = m0[5];
    const double h = S.dt, tau = 0.5 * S.dt, tg = tau * gd;

    for (int step = 0; step < todo; ++step) {
        if (nh) {
            // ---- first half: Z(tau) T(tau) S(tau) K(tau); pp = sum p^2 of the current p
            zt += tau * (pp - nh_tgt) * nh_iq;
            const double c1 = exp(-zt * tau);
#pragma unroll
            for (int j = 0; j < APT; ++j) {
                const double qy = c1 * py[j];
                px[j] = c1 * px[j] - tg * qy + tau * fx[j];
                py[j] = qy + tau * fy[j];
                pz[j] = c1 * pz[j] + tau * fz[j];
            }
        } else {
        // ---- first half: S(tau) then K(tau)
        const double ppt = pp - 2.0 * tg * pxpy + tg * tg * pypy;
        const double g1 = sqrt(pp / ppt);
        const double fp1 = g1 * (fp - tg * fxpy);
        double s1, sd1;
        iso_kick_coeffs(fp1 / pp, ff / pp, tau, s1, sd1);
        const double isd1 = 1.0 / sd1;
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            const double qx = g1 * (px[j] - tg * py[j]);
            const double qy = g1 * py[j];
            const double qz = g1 * pz[j];
            px[j] = (qx + fx[j] * s1) * isd1;
            py[j] = (qy + fy[j] * s1) * isd1;
            pz[j] = (qz + fz[j] * s1) * isd1;
        }
        }
        // ---- streaming D(h), new strain, sliding-brick wrap
        k += 1;
        dxle = le_offset(S, gd, k);
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            x[j] += h * px[j] + h * gd * (y[j] + tau * py[j]);
            y[j] += h * py[j];
            z[j] += h * pz[j];
            wrap_le(S, dxle, x[j], y[j], z[j]);
        }
        compute_forces<Real, APT, false>(S, dxle, x, y, z, fx, fy, fz, wpart, upart, L);
        if (nh) {
            // ---- second half: K(tau) S(tau) T(tau), then Z(tau) on the new sum p^2
            const double c2 = exp(-zt * tau);
            double m4[4] = {0, 0, wpart, 0};  // pp, pxpy, W, position sum
#pragma unroll
            for (int j = 0; j < APT; ++j) {
                const double qy = py[j] + tau * fy[j];
                px[j] = c2 * (px[j] + tau * fx[j] - tg * qy);
                py[j] = c2 * qy;
                pz[j] = c2 * (pz[j] + tau * fz[j]);
                m4[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                m4[1] += px[j] * py[j];
                m4[3] += x[j] + y[j] + z[j];
            }
            block_sum<4>(m4, L.red);
            pp = m4[0];
            zt += tau * (pp - nh_tgt) * nh_iq;
            const double vpxy = m4[1] + m4[2];
            done += 1;
            if (t == 0) dsc->series[done] = vpxy;
            if (!isfinite(vpxy) || !isfinite(zt) || !isfinite(m4[3])) {
                health |= kHealthNonFinite;
                break;
            }
            continue;
        }
        // ---- moments of (p'', F): pp, pxpy, pypy, fp, fxpy, fypx, fxfy, fypy, fyfy, ff, W, pos
        double m[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, wpart, 0};
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            m[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
            m[1] += px[j] * py[j];
            m[2] += py[j] * py[j];
            m[3] += fx[j] * px[j] + fy[j] * py[j] + fz[j] * pz[j];
            m[4] += fx[j] * py[j];
            m[5] += fy[j] * px[j];
            m[6] += fx[j] * fy[j];
            m[7] += fy[j] * py[j];
            m[8] += fy[j] * fy[j];
            m[9] += fx[j] * fx[j] + fy[j] * fy[j] + fz[j] * fz[j];
            m[11] += x[j] + y[j] + z[j];
        }
        block_sum<12>(m, L.red);
        // ---- second half: K(tau) then S(tau), then the exact K0 rescale
        double s2, sd2;
        iso_kick_coeffs(m[3] / m[0], m[9] / m[0], tau, s2, sd2);
        const double isd2 = 1.0 / sd2;
        const double pp3 = (m[0] + 2.0 * s2 * m[3] + s2 * s2 * m[9]) * isd2 * isd2;
        const double pxpy3 = (m[1] + s2 * (m[4] + m[5]) + s2 * s2 * m[6]) * isd2 * isd2;
        const double pypy3 = (m[2] + 2.0 * s2 * m[7] + s2 * s2 * m[8]) * isd2 * isd2;
        const double fp3 = (m[3] + s2 * m[9]) * isd2;
        const double fxpy3 = (m[4] + s2 * m[6]) * isd2;
        const double ppt2 = pp3 - 2.0 * tg * pxpy3 + tg * tg * pypy3;
        const double pxpyt = pxpy3 - tg * pypy3;
        const double c = sqrt(2.0 * k0 / ppt2);
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            const double qx = (px[j] + fx[j] * s2) * isd2;
            const double qy = (py[j] + fy[j] * s2) * isd2;
            const double qz = (pz[j] + fz[j] * s2) * isd2;
            px[j] = c * (qx - tg * qy);
            py[j] = c * qy;
            pz[j] = c * qz;
        }
        pp = c * c * ppt2;
        pxpy = c * c * pxpyt;
        pypy = c * c * pypy3;
        fp = c * (fp3 - tg * fxpy3);
        fxpy = c * fxpy3;
        ff = m[9];
        const double vpxy = pxpy + m[10];
        done += 1;
        if (t == 0) dsc->series[done] = vpxy;
        if (!isfinite(vpxy) || !isfinite(c) || !isfinite(m[11])) {
            health |= kHealthNonFinite;
            break;
        }
        if (fabs(pp3 / m[0] - 1.0) > 1e-10) {
            health |= kHealthDrift;
            break;
        }
    }
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        if (a < n) {
            st[a] = x[j];
            st[n + a] = y[j];
            st[2 * n + a] = z[j];
            st[3 * n + a] = px[j];
            st[4 * n + a] = py[j];
            st[5 * n + a] = pz[j];
        }
    }
    if (t == 0) {
        dsc->k = k;
        dsc->done = done;
        dsc->k0 = k0;
        dsc->health = health;
        dsc->zeta = zt;
    }
    __syncthreads();
}

template <typename Real, int APT, int MAXT, bool NH>
__global__ __launch_bounds__(MAXT) void k_daughters(BatchLaunch b) {
    extern __shared__ __align__(32) char smem[];
    const Lds<Real> L = carve<Real>(smem, b.nmax, b.cmax);
    for (int c = threadIdx.x; c < b.cmax; c += blockDim.x) L.cnt[c] = 0;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) L.misc[0] = atomicAdd(b.queue, 1);
        __syncthreads();
        // the job index is the same in every lane: make that visible so the descriptor is
        // read with scalar loads and its fields stay in scalar registers
        const int j = __builtin_amdgcn_readfirstlane(L.misc[0]);
        if (j >= b.n_jobs) break;
        run_daughter<Real, APT, NH>(&b.descs[b.order[j]], b.max_steps, L);
    }
}

__global__ void k_zero_int(int32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------------------
// mother: Nose-Hoover equilibrium dynamics (gamma_dot = 0, plain periodic box)
// ---------------------------------------------------------------------------------------
// zeta += tau (p.p - nf T)/Q; p = exp(-zeta tau) p + tau F; r += h p; F = F(r); p += tau F;
// p *= exp(-zeta tau); zeta += tau (p.p - nf T)/Q. The p.p of the last update is c^2 times
// the reduced p.p before the scaling, so one reduction per step suffices.
template <typename Real, int APT>
__global__ __launch_bounds__(kMaxThreads) void k_mother(const MotherLaunch* ms, int nmax, int cmax) {
    extern __shared__ __align__(32) char smem[];
    const MotherLaunch& m = ms[blockIdx.x];  // one workgroup per mother
    const Lds<Real> L = carve<Real>(smem, nmax, cmax);
    if (threadIdx.x == 0) *L.sys = m.sys;
    __syncthreads();
    const SysDev& S = *L.sys;
    const int T = blockDim.x, t = threadIdx.x, n = S.n;
    for (int c = t; c < S.nc[0] * S.nc[1] * S.nc[2]; c += T) L.cnt[c] = 0;
    double x[APT], y[APT], z[APT], px[APT], py[APT], pz[APT], fx[APT], fy[APT], fz[APT];
    double* st = m.state;
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        const bool v = a < n;
        x[j] = v ? st[a] : 0.0;
        y[j] = v ? st[n + a] : 0.0;
        z[j] = v ? st[2 * n + a] : 0.0;
        px[j] = v ? st[3 * n + a] : 0.0;
        py[j] = v ? st[4 * n + a] : 0.0;
        pz[j] = v ? st[5 * n + a] : 0.0;
    }
    __syncthreads();
    double wpart, upart;
    compute_forces<Real, APT, false>(S, 0.0, x, y, z, fx, fy, fz, wpart, upart, L);
    double m0[1] = {0.0};
#pragma unroll
    for (int j = 0; j < APT; ++j) m0[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
    block_sum<1>(m0, L.red);
    double pp = m0[0];
    double zeta = *m.zeta;
    const double h = S.dt, tau = 0.5 * S.dt, gT = m.nf * m.temperature, iq = 1.0 / m.q;
    const int64_t chunks = m.n_chunks > 0 ? m.n_chunks : 1;
    int64_t rec = 0;
    for (int64_t ch = 0; ch < chunks; ++ch) {
        for (int64_t s = 0; s < m.steps_per_chunk; ++s) {
            zeta += tau * (pp - gT) * iq;
            const double c1 = exp(-zeta * tau);
#pragma unroll
            for (int j = 0; j < APT; ++j) {
                px[j] = c1 * px[j] + tau * fx[j];
                py[j] = c1 * py[j] + tau * fy[j];
                pz[j] = c1 * pz[j] + tau * fz[j];
                x[j] += h * px[j];
                y[j] += h * py[j];
                z[j] += h * pz[j];
                wrap_le(S, 0.0, x[j], y[j], z[j]);
            }
            compute_forces<Real, APT, false>(S, 0.0, x, y, z, fx, fy, fz, wpart, upart, L);
            double mm[3] = {0.0, 0.0, wpart};
#pragma unroll
            for (int j = 0; j < APT; ++j) {
                px[j] += tau * fx[j];
                py[j] += tau * fy[j];
                pz[j] += tau * fz[j];
                mm[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                mm[1] += px[j] * py[j];
            }
            block_sum<3>(mm, L.red);
            const double c2 = exp(-zeta * tau);
#pragma unroll
            for (int j = 0; j < APT; ++j) {
                px[j] *= c2;
                py[j] *= c2;
                pz[j] *= c2;
            }
            pp = c2 * c2 * mm[0];
            zeta += tau * (pp - gT) * iq;
            if (m.series != nullptr && t == 0) m.series[rec] = c2 * c2 * mm[1] + mm[2];
            ++rec;
        }
        if (m.snap_zeta != nullptr && t == 0) m.snap_zeta[ch] = zeta;
        if (m.snapshots != nullptr) {
            double* dst = m.snapshots + (size_t)ch * 6 * (size_t)n;
#pragma unroll
            for (int j = 0; j < APT; ++j) {
                const int a = t + j * T;
                if (a < n) {
                    dst[a] = x[j];
                    dst[n + a] = y[j];
                    dst[2 * n + a] = z[j];
                    dst[3 * n + a] = px[j];
                    dst[4 * n + a] = py[j];
                    dst[5 * n + a] = pz[j];
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        if (a < n) {
            st[a] = x[j];
            st[n + a] = y[j];
            st[2 * n + a] = z[j];
            st[3 * n + a] = px[j];
            st[4 * n + a] = py[j];
            st[5 * n + a] = pz[j];
        }
    }
    if (t == 0) *m.zeta = zeta;
}

// ---------------------------------------------------------------------------------------
// spawn: the mappings of the start states
// ---------------------------------------------------------------------------------------
// m = 0 identity; 1 p -> -p; 2 (x, px) -> (-x, -px); 3 (x, py, pz) -> (-x, -py, -pz); the
// reflected x is brought back into [0, Lx) as Lx - x (0 stays 0).
__global__ void k_spawn(const double* states, int32_t n, const int32_t* state_of,
                        const int32_t* map_of, double* const* dst, double lx) {
    const int d = blockIdx.x;
    const double* src = states + (size_t)state_of[d] * 6 * (size_t)n;
    double* out = dst[d];
    const int m = map_of[d];
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        double x = src[a], y = src[n + a], z = src[2 * n + a];
        double px = src[3 * n + a], py = src[4 * n + a], pz = src[5 * n + a];
        if (m == 1) {
            px = -px;
            py = -py;
            pz = -pz;
        } else if (m == 2 || m == 3) {
            x = (x == 0.0) ? 0.0 : lx - x;
            if (m == 2) {
                px = -px;
            } else {
                py = -py;
                pz = -pz;
            }
        }
        out[a] = x;
        out[n + a] = y;
        out[2 * n + a] = z;
        out[3 * n + a] = px;
        out[4 * n + a] = py;
        out[5 * n + a] = pz;
    }
}

// ---------------------------------------------------------------------------------------
// accumulate: per start-state group, the direct average and the integral of P(0)P(s)
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ void neumaier_add(double& sum, double& comp, double v) {
    const double tsum = sum + v;
    if (fabs(sum) >= fabs(v))
        comp += (sum - tsum) + v;
    else
        comp += (v - tsum) + sum;
    sum = tsum;
}

constexpr int kMaxMaps = 4;

__global__ void k_accumulate(AccumLaunch a) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n_groups) return;
    const int b = a.first_of[g], e = a.first_of[g + 1];
    // output row of this group
    const size_t row = (size_t)g + (a.row_step ? (size_t)(*a.row_step) * (size_t)a.n_groups : 0);
    const size_t stride = a.row_stride > 0 ? (size_t)a.row_stride : (size_t)a.n_t;
    const int nm = min(e - b, kMaxMaps);
    int health = 0;
    double p0[kMaxMaps], sum[kMaxMaps], comp[kMaxMaps], prev[kMaxMaps];
    const double* ser[kMaxMaps];
    double inv_v = 1.0, dt = 0.0;
    for (int m = 0; m < nm; ++m) {
        const DaughterDesc& d = a.descs[b + m];
        health |= d.health;
        ser[m] = d.series;
        inv_v = 1.0 / d.sys.volume;
        dt = d.sys.dt;
        p0[m] = d.series[0] * inv_v;
        prev[m] = p0[m];
        sum[m] = 0.0;
        comp[m] = 0.0;
    }
    a.health_out[row] = health;
    a.gamma_out[row] = a.descs[b].gamma_dot;
    const double inm = 1.0 / (double)nm;
    double* dout = a.d_out + row * stride;
    double* iout = a.i_out + row * stride;
    if (a.h_out) {
        // mapping mean of the learned control variate (0 where a daughter has none)
        double* hout = a.h_out + row * stride;
        for (int k = 0; k < a.n_t; ++k) {
            double hs = 0.0;
            for (int m = 0; m < nm; ++m) {
                const double* hh = a.descs[b + m].hseries;
                hs += hh ? hh[k] : 0.0;
            }
            hout[k] = hs * inm;
        }
    }
    {
        double dsum = 0.0;
        for (int m = 0; m < nm; ++m) dsum += p0[m];
        dout[0] = dsum * inm;
        iout[0] = 0.0;
    }
    for (int k = 1; k < a.n_t; ++k) {
        double dsum = 0.0, isum = 0.0;
        for (int m = 0; m < nm; ++m) {
            const double cur = ser[m][k] * inv_v;
            neumaier_add(sum[m], comp[m], 0.5 * dt * (p0[m] * prev[m] + p0[m] * cur));
            prev[m] = cur;
            dsum += cur;
            isum += sum[m] + comp[m];
        }
        dout[k] = dsum * inm;
        iout[k] = isum * inm;
    }
}

// ---------------------------------------------------------------------------------------
// response: mean and block standard error over the selected groups, per time point
// ---------------------------------------------------------------------------------------
// G_n(t) = D_n(0) - coef_n I_n(t), coef_n = V gamma_n / T, is the start state's TTCF estimate
// (Eq. TTCF with Omega(0) = -(V/T) gamma_n P_xy(0)); D_n(t) its direct average. Two passes (mean, then the
// squared deviations), each a compensated sum in a fixed row order.
__global__ void k_response(ResponseLaunch r) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= r.n_t) return;
    double gs = 0, gc = 0, ds = 0, dc = 0;
    int used = 0;
    const double beta = r.beta ? r.beta[k] : 1.0;
    for (int i = 0; i < r.n_rows; ++i) {
        const int row = r.rows[i];
        if (r.health[row] != 0) continue;
        const double* dser = r.d_all + (size_t)row * r.n_t_stride;
        const double* iser = r.i_all + (size_t)row * r.n_t_stride;
        const double gam = r.gamma[row];
        double g = dser[0] - r.coef[row] * iser[k];
        if (r.h_all) g -= beta * r.h_all[(size_t)row * r.n_t_stride + k];
        double dv = dser[k];
        if (r.normalise) {
            g /= gam;
            dv /= gam;
        }
        neumaier_add(gs, gc, g);
        neumaier_add(ds, dc, dv);
        ++used;
    }
    const double gm = (gs + gc) / (double)used;
    const double dm = (ds + dc) / (double)used;
    double gv = 0, gvc = 0, dvv = 0, dvc = 0;
    for (int i = 0; i < r.n_rows; ++i) {
        const int row = r.rows[i];
        if (r.health[row] != 0) continue;
        const double* dser = r.d_all + (size_t)row * r.n_t_stride;
        const double* iser = r.i_all + (size_t)row * r.n_t_stride;
        const double gam = r.gamma[row];
        double g = dser[0] - r.coef[row] * iser[k];
        if (r.h_all) g -= beta * r.h_all[(size_t)row * r.n_t_stride + k];
        double dv = dser[k];
        if (r.normalise) {
            g /= gam;
            dv /= gam;
        }
        neumaier_add(gv, gvc, (g - gm) * (g - gm));
        neumaier_add(dvv, dvc, (dv - dm) * (dv - dm));
    }
    const double denom = used > 1 ? (double)(used - 1) * (double)used : 1.0;
    r.out[k] = gm + (r.mu_h ? beta * r.mu_h[k] : 0.0);
    r.out[r.n_t + k] = used > 1 ? sqrt((gv + gvc) / denom) : 0.0;
    r.out[2 * r.n_t + k] = dm;
    r.out[3 * r.n_t + k] = used > 1 ? sqrt((dvv + dvc) / denom) : 0.0;
    if (k == 0) *r.used = used;
}

// Control-variate coefficient beta(t) = Cov(G, H) / Var(H) over the selected healthy groups
// (the variance-minimising multiple of H), two compensated passes in a fixed row order;
// beta = 0 where H does not vary.
__global__ void k_cv_beta(ResponseLaunch r, double* beta) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= r.n_t) return;
    double gs = 0, gc = 0, hs = 0, hc = 0;
    int used = 0;
    for (int i = 0; i < r.n_rows; ++i) {
        const int row = r.rows[i];
        if (r.health[row] != 0) continue;
        const double* dser = r.d_all + (size_t)row * r.n_t_stride;
        const double g = dser[0] - r.coef[row] * r.i_all[(size_t)row * r.n_t_stride + k];
        neumaier_add(gs, gc, g);
        neumaier_add(hs, hc, r.h_all[(size_t)row * r.n_t_stride + k]);
        ++used;
    }
    if (used < 2) {
        beta[k] = 0.0;
        return;
    }
    const double gm = (gs + gc) / used, hm = (hs + hc) / used;
    double cs = 0, cc = 0, vs = 0, vc = 0;
    for (int i = 0; i < r.n_rows; ++i) {
        const int row = r.rows[i];
        if (r.health[row] != 0) continue;
        const double* dser = r.d_all + (size_t)row * r.n_t_stride;
        const double g = dser[0] - r.coef[row] * r.i_all[(size_t)row * r.n_t_stride + k] - gm;
        const double h = r.h_all[(size_t)row * r.n_t_stride + k] - hm;
        neumaier_add(cs, cc, g * h);
        neumaier_add(vs, vc, h * h);
    }
    const double var = vs + vc;
    beta[k] = var > 0.0 ? (cs + cc) / var : 0.0;
}

// ---------------------------------------------------------------------------------------
// V*P_xy of many stored states (6n doubles each), one workgroup per state at a time
// ---------------------------------------------------------------------------------------

template <int APT>
__global__ __launch_bounds__(kMaxThreads) void k_states_vpxy(SysDev S, const double* states,
                                                             int32_t count, double* out) {
    extern __shared__ __align__(32) char smem[];
    const int C = S.nc[0] * S.nc[1] * S.nc[2];
    const Lds<double> L = carve<double>(smem, S.n, C);
    const int T = blockDim.x, t = threadIdx.x, n = S.n;
    for (int c = t; c < C; c += T) L.cnt[c] = 0;
    for (int sidx = blockIdx.x; sidx < count; sidx += gridDim.x) {
        const double* st = states + (size_t)sidx * 6 * (size_t)n;
        double x[APT], y[APT], z[APT], fx[APT], fy[APT], fz[APT];
        double kin = 0.0;
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            const int a = t + j * T;
            const bool v = a < n;
            x[j] = v ? st[a] : 0.0;
            y[j] = v ? st[n + a] : 0.0;
            z[j] = v ? st[2 * n + a] : 0.0;
            kin += v ? st[3 * n + a] * st[4 * n + a] : 0.0;
        }
        __syncthreads();
        double wpart, upart;
        compute_forces<double, APT, false>(S, 0.0, x, y, z, fx, fy, fz, wpart, upart, L);
        double m[2] = {kin, wpart};
        block_sum<2>(m, L.red);
        if (t == 0) out[sidx] = m[0] + m[1];
    }
}

// ---------------------------------------------------------------------------------------
// inspection kernels (single workgroup, positions given)
// ---------------------------------------------------------------------------------------

template <typename Real, int APT>
__global__ __launch_bounds__(kMaxThreads) void k_debug_cells(SysDev S, const double* r,
                                                             int32_t* cell_of, int32_t* order,
                                                             int32_t* start) {
    extern __shared__ __align__(32) char smem[];
    const int C = S.nc[0] * S.nc[1] * S.nc[2];
    const Lds<Real> L = carve<Real>(smem, S.n, C);
    const int T = blockDim.x, t = threadIdx.x, n = S.n;
    for (int c = t; c < C; c += T) L.cnt[c] = 0;
    double x[APT], y[APT], z[APT];
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        x[j] = a < n ? r[a] : 0.0;
        y[j] = a < n ? r[n + a] : 0.0;
        z[j] = a < n ? r[2 * n + a] : 0.0;
    }
    __syncthreads();
    int cell[APT];
    build_cells<Real, APT>(S, 0.0, x, y, z, L, cell);
#pragma unroll
    for (int j = 0; j < APT; ++j)
        if (cell[j] >= 0) cell_of[t + j * T] = cell[j];
    for (int i = t; i < n; i += T) order[i] = L.sid[i];
    for (int c = t; c <= C; c += T) start[c] = L.start[c];
}

template <typename Real, int APT>
__global__ __launch_bounds__(kMaxThreads) void k_debug_forces(SysDev S, double dxle,
                                                              const double* r, double* f,
                                                              double* out) {
    extern __shared__ __align__(32) char smem[];
    const int C = S.nc[0] * S.nc[1] * S.nc[2];
    const Lds<Real> L = carve<Real>(smem, S.n, C);
    const int T = blockDim.x, t = threadIdx.x, n = S.n;
    for (int c = t; c < C; c += T) L.cnt[c] = 0;
    double x[APT], y[APT], z[APT], fx[APT], fy[APT], fz[APT];
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        x[j] = a < n ? r[a] : 0.0;
        y[j] = a < n ? r[n + a] : 0.0;
        z[j] = a < n ? r[2 * n + a] : 0.0;
    }
    __syncthreads();
    double wpart, upart;
    compute_forces<Real, APT, true>(S, dxle, x, y, z, fx, fy, fz, wpart, upart, L);
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        if (a < n) {
            f[a] = fx[j];
            f[n + a] = fy[j];
            f[2 * n + a] = fz[j];
        }
    }
    double m[2] = {upart, wpart};
    block_sum<2>(m, L.red);
    if (t == 0) {
        out[0] = m[0];
        out[1] = m[1];
    }
}

// Minimum-image separation exactly as a plain FP64 evaluation gives it: y image first (its
// crossing shifts x by the offset), then periodic x and z. No contraction into FMAs, so the
// pair set below is bit-identical to any IEEE evaluation of the same expressions.
__device__ void min_image_exact(const SysDev& S, double dxle, double xi, double yi, double zi,
                                double xj, double yj, double zj, double& dx, double& dy,
                                double& dz) {
#pragma clang fp contract(off)
    dy = yi - yj;
    const double ny = rint(dy / S.box[1]);
    dy = dy - ny * S.box[1];
    dx = xi - xj;
    dx = dx - ny * dxle;
    dx = dx - S.box[0] * rint(dx / S.box[0]);
    dz = zi - zj;
    dz = dz - S.box[2] * rint(dz / S.box[2]);
}

__device__ double dist2_exact(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    return dx * dx + dy * dy + dz * dz;
}

// Pairs i<j closer than rlist, found through the same cell list and stencil as the forces
// (FP32 shift tables are not used: the test is done on FP64 absolute positions).
template <int APT>
__global__ __launch_bounds__(kMaxThreads) void k_debug_pairs(SysDev S, double dxle,
                                                             const double* r, double rlist,
                                                             int64_t cap, int32_t* pi,
                                                             int32_t* pj,
                                                             unsigned long long* count) {
    extern __shared__ __align__(32) char smem[];
    const int C = S.nc[0] * S.nc[1] * S.nc[2];
    const Lds<float> L = carve<float>(smem, S.n, C);
    const int T = blockDim.x, t = threadIdx.x, n = S.n;
    const int nc0 = S.nc[0], nc1 = S.nc[1], nc2 = S.nc[2];
    for (int c = t; c < C; c += T) L.cnt[c] = 0;
    double x[APT], y[APT], z[APT];
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        x[j] = a < n ? r[a] : 0.0;
        y[j] = a < n ? r[n + a] : 0.0;
        z[j] = a < n ? r[2 * n + a] : 0.0;
    }
    __syncthreads();
    int cell[APT];
    build_cells<float, APT>(S, dxle, x, y, z, L, cell);
    const double rl2 = rlist * rlist;
    for (int s = t; s < n; s += T) {
        const int i = L.sid[s];
        const int pk = unpack_cell(L.spos[s].w);
        const int cx = pk & 1023, cy = (pk >> 10) & 1023, cz = pk >> 20;
        for (int dz = 0; dz < 3; ++dz) {
            int zz = cz + dz - 1;
            zz = zz < 0 ? zz + nc2 : (zz >= nc2 ? zz - nc2 : zz);
            for (int dy = 0; dy < 3; ++dy) {
                int yy = cy + dy - 1;
                int row = 1;
                if (yy < 0) {
                    yy += nc1;
                    row = 0;
                } else if (yy >= nc1) {
                    yy -= nc1;
                    row = 2;
                }
                const int nq = L.rowinfo[2 * row + 1];
                int xx = cx + L.rowinfo[2 * row];
                if (xx >= nc0) xx -= nc0;
                for (int q = 0; q < nq; ++q) {
                    const int c = xx + nc0 * (yy + nc1 * zz);
                    for (int tt = L.start[c]; tt < L.start[c + 1]; ++tt) {
                        const int j = L.sid[tt];
                        if (j <= i) continue;
                        double ddx, ddy, ddz;
                        min_image_exact(S, dxle, r[i], r[n + i], r[2 * n + i], r[j], r[n + j],
                                        r[2 * n + j], ddx, ddy, ddz);
                        if (dist2_exact(ddx, ddy, ddz) < rl2) {
                            const unsigned long long at = atomicAdd(count, 1ull);
                            if ((int64_t)at < cap) {
                                pi[at] = i;
                                pj[at] = j;
                            }
                        }
                    }
                    ++xx;
                    if (xx >= nc0) xx -= nc0;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// neighbour-list form of the daughter step (FP32 pair forces)
// ---------------------------------------------------------------------------------------
//
// Pair separations come from 32-bit fixed-point coordinates X = rint(x 2^32 / L): the box
// is exactly 2^32 units wide, so the wrapped integer difference X_i - X_j is the periodic
// minimum image. The y difference tells whether the pair reaches across the sliding
// boundary (n_y = +-1); then the Lees-Edwards offset, also in fixed point, is subtracted
// from the x difference. The result is converted to FP32 once, so the separation carries
// one rounding of a number no larger than the cutoff.
//
// Every atom keeps a list of the atoms within rc + skin, sorted by atom id, in LDS. A pair's
// relative displacement since the list was built is at most
//   2 d + |gamma_dot| t (rc + 2 d),
// with d the largest peculiar path length of any atom and t the time since the build (the
// second term is the shear flow between the two atoms; across the y boundary the drifting
// offset compensates the images' streaming). The lists are rebuilt as soon as that bound
// reaches the skin, so every pair inside rc is always listed. Because each list is sorted
// and pairs outside rc add nothing, the forces do not depend on when rebuilds happen.

// Entries per trip of the force loop and candidates per trip of the list build: their loads
// are issued together, so that LDS latency overlaps within a wave.
constexpr int kNlPairsPerTrip = 2;
constexpr int kNlScanPerTrip = 4;

struct NlLds {
    uint4* posq;       // [nmax] fixed-point positions (X, Y, Z, unused)
    uint16_t* nbr;     // [kmax][nmax] neighbour ids, column a = atom a
    uint32_t* ncnt;    // [nmax] list lengths
    int32_t* cnt;      // [cmax] list-grid cell counts / cursors
    int32_t* start;    // [cmax + 1]
    uint16_t* sid;     // [nmax + kNlScanPerTrip] atoms grouped by list-grid cell, then padding
    int32_t* rowinfo;  // [3 rows][2]: first column offset mod nx, column count
    double* red;       // block-reduction scratch
    int32_t* scan;     // [kMaxWaves]
    float* wmax;       // [2 kMaxWaves] per-wave maxima of the two path lengths
    int32_t* misc;     // [4]: [0] job, [1] list overflow
    SysDev* sys;
};

struct NlPlan {
    size_t posq, nbr, ncnt, cnt, start, sid, rowinfo, red, scan, wmax, misc, sys, total;
};

// global_lists: the lists live in per-workgroup global scratch instead (systems whose lists
// do not fit in LDS); everything else stays in LDS.
__host__ __device__ inline NlPlan plan_nl(int nmax, int cmax, int kmax, bool global_lists = false) {
    NlPlan p;
    size_t off = 0;
    auto take = [&](size_t bytes, size_t al) {
        off = align_up(off, al);
        size_t at = off;
        off += bytes;
        return at;
    };
    p.posq = take(16 * (size_t)nmax, 16);
    // row kmax: sink for rejected candidates
    p.nbr = global_lists ? 0 : take(2 * (size_t)(kmax + 1) * nmax, 16);
    p.ncnt = take(4 * (size_t)nmax, 16);
    p.cnt = take(4 * (size_t)cmax, 16);
    p.start = take(4 * (size_t)(cmax + 1), 16);
    // padding: the reads of a trip past the end of a range stay inside
    p.sid = take(2 * (size_t)(nmax + kNlScanPerTrip), 16);
    p.rowinfo = take(4 * 8, 16);
    p.red = take(sizeof(double) * (kMaxWaves * kRedSlots + kRedSlots), 16);
    p.scan = take(4 * kMaxWaves, 16);
    p.wmax = take(8 * kMaxWaves, 16);
    p.misc = take(4 * 4, 16);
    p.sys = take(sizeof(SysDev), 16);
    p.total = align_up(off, 128);
    return p;
}

__device__ inline NlLds carve_nl(char* base, int nmax, int cmax, int kmax,
                                 uint16_t* global_nbr = nullptr) {
    NlPlan p = plan_nl(nmax, cmax, kmax, global_nbr != nullptr);
    NlLds L;
    L.posq = (uint4*)(base + p.posq);
    L.nbr = global_nbr ? global_nbr : (uint16_t*)(base + p.nbr);
    L.ncnt = (uint32_t*)(base + p.ncnt);
    L.cnt = (int32_t*)(base + p.cnt);
    L.start = (int32_t*)(base + p.start);
    L.sid = (uint16_t*)(base + p.sid);
    L.rowinfo = (int32_t*)(base + p.rowinfo);
    L.red = (double*)(base + p.red);
    L.scan = (int32_t*)(base + p.scan);
    L.wmax = (float*)(base + p.wmax);
    L.misc = (int32_t*)(base + p.misc);
    L.sys = (SysDev*)(base + p.sys);
    return L;
}

__device__ __forceinline__ uint32_t fix32(double v, double scale) {
    return (uint32_t)(int64_t)rint(v * scale);
}

// Separation (FP32) of fixed-point positions i and j; dxq is the LE offset in fixed point.
__device__ __forceinline__ void fix_sep(uint32_t xi, uint32_t yi, uint32_t zi, const uint4& q,
                                        uint32_t dxq, const SysDev& S, float& dx, float& dy,
                                        float& dz) {
    const uint32_t uy = yi - q.y;
    const int32_t iy = (int32_t)uy;
    // n_y = +1 when y_i - y_j > L/2 (the image above is nearer), -1 when < -L/2, else 0:
    // n_y = (sign bit of the wrapped difference) - (borrow of the unsigned subtraction);
    // the x difference then loses n_y times the offset
    const uint32_t sgn = uy >> 31;
    const uint32_t brw = yi < q.y ? 1u : 0u;
    const uint32_t shift = ((0u - sgn) & dxq) - ((0u - brw) & dxq);
    const int32_t ix = (int32_t)(xi - q.x - shift);
    const int32_t iz = (int32_t)(zi - q.z);
    dx = (float)ix * S.fix_unit[0];
    dy = (float)iy * S.fix_unit[1];
    dz = (float)iz * S.fix_unit[2];
}

// Rebuild the lists: counting sort of the atoms into the list grid (cells >= rc + skin wide),
// then every owner collects its atoms' neighbours within rc + skin over the 27-cell stencil
// (LE-displaced x range for rows across the y boundary) and sorts them by id.
template <int APT>
__device__ __forceinline__ void nl_rebuild(const SysDev& S, double dxle, uint32_t dxq, const double (&x)[APT],
                           const double (&y)[APT], const double (&z)[APT],
                           const uint32_t (&qx)[APT], const uint32_t (&qy)[APT],
                           const uint32_t (&qz)[APT], const NlLds& L, int kmax, int nmax) {
    const int T = blockDim.x, t = threadIdx.x, n = S.n;
    const int nc0 = S.lc[0], nc1 = S.lc[1], nc2 = S.lc[2];
    const int C = nc0 * nc1 * nc2;
    int cell[APT];
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        cell[j] = -1;
        if (a < n) {
            const int cx = cell_coord(x[j], S.l_inv_w[0], nc0);
            const int cy = cell_coord(y[j], S.l_inv_w[1], nc1);
            const int cz = cell_coord(z[j], S.l_inv_w[2], nc2);
            cell[j] = cx + nc0 * (cy + nc1 * cz);
            atomicAdd(&L.cnt[cell[j]], 1);
        }
    }
    if (t == 0) {
        L.misc[1] = 0;
        const double reach = S.rc + S.skin;
        const double wx = S.lw[0];
        const double margin = 1e-6 * reach;
        for (int row = 0; row < 3; ++row) {
            int off, nq;
            if (row == 1) {
                off = -1;
                nq = 3;
            } else {
                double sh = (row == 0 ? -1.0 : 1.0) * dxle;
                sh -= S.box[0] * rint(sh / S.box[0]);
                off = (int)floor((-reach - margin - sh) / wx);
                const int hi = (int)floor((wx + reach + margin - sh) / wx);
                nq = hi - off + 1;
                if (nq > 5) nq = 5;
                if (nq > nc0) nq = nc0;
            }
            L.rowinfo[2 * row] = ((off % nc0) + nc0) % nc0;
            L.rowinfo[2 * row + 1] = nq;
        }
    }
    __syncthreads();
    scan_cells(L.cnt, L.start, C, L.scan);
    if (t == 0) L.start[C] = n;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        if (cell[j] >= 0) {
            const int idx = atomicAdd(&L.cnt[cell[j]], 1);
            L.sid[idx] = (uint16_t)(t + j * T);
        }
    }
    __syncthreads();
    const float rl2 = S.rl2_f;
    const float ux = S.fix_unit[0], uy = S.fix_unit[1], uz = S.fix_unit[2];
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        if (a >= n) continue;
        const int c0 = cell[j];
        const int cx = c0 % nc0, cy = (c0 / nc0) % nc1, cz = c0 / (nc0 * nc1);
        int count = 0;
        // the cells of one stencil row are consecutive cell ids, so their atoms form one
        // contiguous range of the sorted order (two when the row wraps around in x)
        // branch-free: every candidate is written, rejected ones into the sink row kmax
        const int sink = kmax * nmax + a;
        int slot = a;  // count * nmax + a while count < kmax
        // rsh: the Lees-Edwards x shift of the row's y image (+offset for a row wrapped from
        // the top, -offset from the bottom, 0 otherwise). A candidate within the list radius is
        // nearer than half the box in y, so its minimum image is the row's image; for the others
        // the test fails with either shift.
        auto scan = [&](int lo, int hi, uint32_t rsh) {
#pragma unroll 1
            for (int tt = lo; tt < hi; tt += kNlScanPerTrip) {
                int jn[kNlScanPerTrip];
                uint4 q[kNlScanPerTrip];
#pragma unroll
                for (int u = 0; u < kNlScanPerTrip; ++u) {
                    // unconditional load (the array is padded); a value past the range is
                    // replaced before it is used as an index
                    const int raw = L.sid[tt + u];
                    jn[u] = tt + u < hi ? raw : a;
                }
#pragma unroll
                for (int u = 0; u < kNlScanPerTrip; ++u) q[u] = L.posq[jn[u]];
#pragma unroll
                for (int u = 0; u < kNlScanPerTrip; ++u) {
                    const float ddx = (float)(int32_t)(qx[j] - q[u].x - rsh) * ux;
                    const float ddy = (float)(int32_t)(qy[j] - q[u].y) * uy;
                    const float ddz = (float)(int32_t)(qz[j] - q[u].z) * uz;
                    const bool hit = (jn[u] != a) & (ddx * ddx + ddy * ddy + ddz * ddz < rl2);
                    const bool room = hit & (count < kmax);
                    L.nbr[room ? slot : sink] = (uint16_t)jn[u];
                    slot += room ? nmax : 0;
                    count += hit ? 1 : 0;
                }
            }
        };
#pragma unroll 1
        for (int r9 = 0; r9 < 9; ++r9) {
            int zz = cz + r9 / 3 - 1;
            zz = zz < 0 ? zz + nc2 : (zz >= nc2 ? zz - nc2 : zz);
            int yy = cy + r9 % 3 - 1;
            int row = 1;
            if (yy < 0) {
                yy += nc1;
                row = 0;
            } else if (yy >= nc1) {
                yy -= nc1;
                row = 2;
            }
            const int nq = L.rowinfo[2 * row + 1];
            int x0 = cx + L.rowinfo[2 * row];
            if (x0 >= nc0) x0 -= nc0;
            const int base = nc0 * (yy + nc1 * zz);
            const int xe = x0 + nq;
            const uint32_t rsh = row == 2 ? dxq : (row == 0 ? 0u - dxq : 0u);
            scan(L.start[base + x0], L.start[base + (xe < nc0 ? xe : nc0)], rsh);
            if (xe > nc0) scan(L.start[base], L.start[base + xe - nc0], rsh);
        }
        if (count > kmax) {
            L.misc[1] = 1;
            count = kmax;
        }
        // ascending ids: a fixed summation order for the forces
        for (int i = 1; i < count; ++i) {
            const uint16_t v = L.nbr[i * nmax + a];
            int k = i - 1;
            while (k >= 0 && L.nbr[k * nmax + a] > v) {
                L.nbr[(k + 1) * nmax + a] = L.nbr[k * nmax + a];
                --k;
            }
            L.nbr[(k + 1) * nmax + a] = v;
        }
        L.ncnt[a] = (uint32_t)count;
    }
    for (int c = t; c < C; c += T) L.cnt[c] = 0;
    __syncthreads();
}

// Forces on the owned atoms from their lists; returns this thread's share of W_xy.
// Marks, for every owned atom, the list entries within the inner radius (bit k: entry k);
// entries beyond it cannot reach r_c before the next refresh.
// PER: list entries per trip (their loads issued together).
template <int APT, int PER>
__device__ __forceinline__ void nl_inner(const SysDev& S, uint32_t dxq, const uint32_t (&qx)[APT],
                                         const uint32_t (&qy)[APT], const uint32_t (&qz)[APT],
                                         const NlLds& L, int nmax, uint32_t (&imask)[APT]) {
    const int T = blockDim.x, t = threadIdx.x, n = S.n;
    const float ri2 = S.ri2_f;
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        uint32_t m = 0u;
        if (a < n) {
            const int c = L.ncnt[a];
            // PER entries per trip: their id loads, then their position loads, are issued
            // together; entries past the count reread entry k and set no bit
            for (int k = 0; k < c; k += PER) {
                int id[PER];
                uint4 q[PER];
#pragma unroll
                for (int u = 0; u < PER; ++u) id[u] = L.nbr[(k + u < c ? k + u : k) * nmax + a];
#pragma unroll
                for (int u = 0; u < PER; ++u) q[u] = L.posq[id[u]];
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    float dx, dy, dz;
                    fix_sep(qx[j], qy[j], qz[j], q[u], dxq, S, dx, dy, dz);
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    m |= ((k + u < c) & (r2 < ri2)) ? 1u << ((k + u) & 31) : 0u;
                }
            }
        }
        imask[j] = m;
    }
}

// OBS: also this thread's halves of the pair sums W_xx, W_yy, W_zz and U (xw).
template <int APT, bool OBS>
__device__ __forceinline__ double nl_forces(const SysDev& S, uint32_t dxq,
                                            const uint32_t (&qx)[APT], const uint32_t (&qy)[APT],
                                            const uint32_t (&qz)[APT], const uint32_t (&imask)[APT],
                                            float (&fx)[APT], float (&fy)[APT], float (&fz)[APT],
                                            const NlLds& L, int nmax, double (&xw)[4]) {
    const int T = blockDim.x, t = threadIdx.x;
    const float rc2 = S.rc2_f;
    const float ca = (float)S.c_attr;
    const float ushift = (float)S.u_shift;
    double wacc = 0.0;
    if (OBS) xw[0] = xw[1] = xw[2] = xw[3] = 0.0;
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        float gx = 0.f, gy = 0.f, gz = 0.f, w = 0.f;
        float vxx = 0.f, vyy = 0.f, vzz = 0.f, uu = 0.f;
        {
            // the inner entries in list order (ascending ids): a fixed summation order, and
            // every skipped entry lies beyond r_c, where a pair adds an exact zero
            // one pair, added in list order; `live` false adds exact zeros
            auto pair = [&](const uint4& q, bool live) {
                float dx, dy, dz;
                fix_sep(qx[j], qy[j], qz[j], q, dxq, S, dx, dy, dz);
                const float r2 = dx * dx + dy * dy + dz * dz;
                // listed pairs beyond the cutoff contribute an exact zero (no branch)
                const float inv = recip(r2);
                const float s3 = inv * inv * inv;
                const bool in = live & (r2 < rc2);
                const float fs = in ? s3 * (48.f * s3 - 24.f * ca) * inv : 0.f;
                gx += fs * dx;
                gy += fs * dy;
                gz += fs * dz;
                w += dx * (fs * dy);
                if (OBS) {
                    vxx += dx * (fs * dx);
                    vyy += dy * (fs * dy);
                    vzz += dz * (fs * dz);
                    uu += in ? 4.f * s3 * (s3 - ca) + ushift : 0.f;
                }
            };
            // P inner entries per trip: their id loads, then their position loads, are issued
            // before the arithmetic; missing entries at the end repeat the first one and add
            // nothing. The build with the extra pair sums keeps one entry per trip: with two
            // it outgrows the register budget.
            constexpr int P = OBS ? 1 : kNlPairsPerTrip;
            uint32_t mk = imask[j];
            while (mk != 0u) {
                int kk[P];
                bool live[P];
                kk[0] = __builtin_ctz(mk);
                live[0] = true;
                mk &= mk - 1u;
#pragma unroll
                for (int u = 1; u < P; ++u) {
                    live[u] = mk != 0u;
                    kk[u] = live[u] ? __builtin_ctz(mk) : kk[0];
                    mk &= mk - 1u;
                }
                int id[P];
                uint4 q[P];
#pragma unroll
                for (int u = 0; u < P; ++u) id[u] = L.nbr[kk[u] * nmax + a];
#pragma unroll
                for (int u = 0; u < P; ++u) q[u] = L.posq[id[u]];
#pragma unroll
                for (int u = 0; u < P; ++u) pair(q[u], live[u]);
            }
        }
        fx[j] = gx;
        fy[j] = gy;
        fz[j] = gz;
        wacc += (double)w;
        if (OBS) {
            xw[0] += 0.5 * (double)vxx;
            xw[1] += 0.5 * (double)vyy;
            xw[2] += 0.5 * (double)vzz;
            xw[3] += 0.5 * (double)uu;
        }
    }
    return 0.5 * wacc;
}

// The extra observables of the owned atoms at one time point (momenta p, positions in
// [0, L), pair halves xw of the last force pass), reduced over the workgroup and written by
// thread 0 to row `row` of the daughter's extra series.
template <int APT>
__device__ __forceinline__ void nl_record_obs(const SysDev& S, const double (&y)[APT],
                                              const double (&px)[APT], const double (&py)[APT],
                                              const double (&pz)[APT], const double (&xw)[4],
                                              double* xs, int row, const NlLds& L) {
    double o[kObsCols];
#pragma unroll
    for (int c = 0; c < kObsCols; ++c) o[c] = 0.0;
    const double slab_scale = (double)kObsSlabs / S.box[1];
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        // lanes past n hold zero momenta and add nothing
        const double xx = px[j] * px[j], yy = py[j] * py[j], zz = pz[j] * pz[j];
        o[0] += xx - yy;
        o[1] += yy - zz;
        o[2] += 0.5 * (xx + yy + zz);
        int sl = (int)floor(y[j] * slab_scale);
        sl = sl < 0 ? 0 : (sl > kObsSlabs - 1 ? kObsSlabs - 1 : sl);
#pragma unroll
        for (int q = 0; q < kObsSlabs; ++q) o[3 + q] += sl == q ? px[j] : 0.0;
    }
    o[0] += xw[0] - xw[1];
    o[1] += xw[1] - xw[2];
    o[2] += xw[3];
    block_sum<kObsCols>(o, L.red);
    if (threadIdx.x == 0) {
        double* out = xs + (size_t)row * kObsCols;
        const double iv = 1.0 / S.volume;
        out[0] = o[0] * iv;
        out[1] = o[1] * iv;
        out[2] = o[2] / (double)S.n;
#pragma unroll
        for (int q = 0; q < kObsSlabs; ++q) out[3 + q] = o[3 + q] * ((double)kObsSlabs * iv);
    }
}

// Publish the fixed-point positions of the owned atoms and the wave maxima of the path
// lengths; after the barrier every thread reads the workgroup maximum.
template <int APT>
__device__ __forceinline__ float2 nl_publish(const SysDev& S, const double (&x)[APT],
                                             const double (&y)[APT], const double (&z)[APT],
                                             uint32_t (&qx)[APT], uint32_t (&qy)[APT],
                                             uint32_t (&qz)[APT], const float (&path)[APT],
                                             const float (&path_in)[APT], const NlLds& L) {
    const int T = blockDim.x, t = threadIdx.x, n = S.n;
    float pm = 0.f, pi = 0.f;
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        qx[j] = fix32(x[j], S.fix_scale[0]);
        qy[j] = fix32(y[j], S.fix_scale[1]);
        qz[j] = fix32(z[j], S.fix_scale[2]);
        if (a < n) {
            L.posq[a] = make_uint4(qx[j], qy[j], qz[j], 0u);
            pm = fmaxf(pm, path[j]);
            pi = fmaxf(pi, path_in[j]);
        }
    }
    pm = wave_max_dpp(pm);
    pi = wave_max_dpp(pi);
    if ((t & 63) == 63) {
        L.wmax[2 * (t >> 6)] = pm;
        L.wmax[2 * (t >> 6) + 1] = pi;
    }
    __syncthreads();
    float2 m = make_float2(0.f, 0.f);
    for (int w = 0; w < (T >> 6); ++w) {
        m.x = fmaxf(m.x, L.wmax[2 * w]);
        m.y = fmaxf(m.y, L.wmax[2 * w + 1]);
    }
    return m;
}

// COL: the build that also runs colour-field daughters (either thermostat): atom a carries
// the colour charge +1 (even a) or -1 (odd a), the field adds charge * F_e to its x force in
// FP64, there is no shear, and the series records V J_x = sum_a charge p_x,a.
template <int APT, bool NH, bool OBS, bool COL>
__device__ void run_daughter_nl(DaughterDesc* dsc, int steps_cap, const NlLds& L, int kmax,
                                int nmax) {
    const int T = blockDim.x, t = threadIdx.x;
    if (t == 0) *L.sys = dsc->sys;
    __syncthreads();
    const SysDev& S = *L.sys;
    const int n = S.n;
    double* st = dsc->state;
    const bool col = COL && dsc->field == kFieldColour;  // uniform per job
    const double gd = col ? 0.0 : dsc->gamma_dot;
    int64_t k = dsc->k;
    int done = dsc->done;
    const int n_steps = dsc->n_steps;
    double k0 = dsc->k0;
    int health = dsc->health;
    // Nose-Hoover daughters (Eq. system1 as printed): zeta from the mapped start state
    constexpr bool nh = NH;  // the descriptor's thermo selects the instantiation
    double zt = dsc->zeta;
    const double nh_iq = nh ? 1.0 / dsc->nh_q : 0.0, nh_tgt = dsc->nh_target;
    int todo = min(steps_cap, n_steps - done);
    if (health != 0) todo = 0;
    if (todo <= 0 && done > 0) return;

    double x[APT], y[APT], z[APT], px[APT], py[APT], pz[APT];
    float fx[APT], fy[APT], fz[APT];  // FP32 pair forces; every use below promotes them to FP64
    uint32_t qx[APT], qy[APT], qz[APT];
    float path[APT], path_in[APT];  // path lengths since the last rebuild / inner refresh
    uint32_t imask[APT];
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        const bool v = a < n;
        x[j] = v ? st[a] : 0.0;
        y[j] = v ? st[n + a] : 0.0;
        z[j] = v ? st[2 * n + a] : 0.0;
        px[j] = v ? st[3 * n + a] : 0.0;
        py[j] = v ? st[4 * n + a] : 0.0;
        pz[j] = v ? st[5 * n + a] : 0.0;
        path[j] = 0.f;
        path_in[j] = 0.f;
    }
    // colour charges (zero past n and for shear daughters) and the field's x force in FP64
    double cq[APT], ce[APT];
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        cq[j] = (COL && col && a < n) ? ((a & 1) ? -1.0 : 1.0) : 0.0;
        ce[j] = COL ? cq[j] * dsc->fe : 0.0;
    }
    auto fxd = [&](int j) -> double {
        if constexpr (COL)
            return (double)fx[j] + ce[j];
        else
            return (double)fx[j];
    };
    double dxle = le_offset(S, gd, k);
    uint32_t dxq = fix32(dxle, S.fix_scale[0]);
    nl_publish<APT>(S, x, y, z, qx, qy, qz, path, path_in, L);
    nl_rebuild<APT>(S, dxle, dxq, x, y, z, qx, qy, qz, L, kmax, nmax);
    if (L.misc[1] != 0) health |= kHealthListOverflow;
    // the build with the extra pair sums keeps one entry per trip (register budget)
    constexpr int kInnerPer = OBS ? 1 : 4;
    nl_inner<APT, kInnerPer>(S, dxq, qx, qy, qz, L, nmax, imask);
    double xw[4];
    double wpart = nl_forces<APT, OBS>(S, dxq, qx, qy, qz, imask, fx, fy, fz, L, nmax, xw);
    double* const xs = OBS ? dsc->xseries : nullptr;

    double m0[7] = {0, 0, 0, 0, 0, 0, wpart};
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        m0[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
        m0[1] += (COL && col) ? cq[j] * px[j] : px[j] * py[j];
        m0[2] += py[j] * py[j];
        m0[3] += fxd(j) * px[j] + (double)fy[j] * py[j] + (double)fz[j] * pz[j];
        m0[4] += fxd(j) * py[j];
        m0[5] += fxd(j) * fxd(j) + (double)fy[j] * (double)fy[j] +
                 (double)fz[j] * (double)fz[j];
    }
    block_sum<7>(m0, L.red);
    if (done == 0) {
        if (k0 <= 0.0) k0 = 0.5 * m0[0];
        if (t == 0) dsc->series[0] = (COL && col) ? m0[1] : m0[1] + m0[6];
        if (OBS && xs) nl_record_obs<APT>(S, y, px, py, pz, xw, xs, 0, L);
    }
    if (health != 0) todo = 0;
    double pp = m0[0], pxpy = m0[1], pypy = m0[2], fp = m0[3], fxpy = m0[4], ff = m0[5];
    const double h = S.dt, tau = 0.5 * S.dt, tg = tau * gd;
    const float reach = (float)S.rc;
    const float skin = (float)S.skin;
    const float skin_in = (float)S.skin_in;
    const float agd = (float)fabs(gd);
    int since = 0, since_in = 0;

    for (int step = 0; step < todo; ++step) {
        if (nh) {
            // ---- first half: Z(tau) T(tau) S(tau) K(tau); pp = sum p^2 of the current p
            zt += tau * (pp - nh_tgt) * nh_iq;
            const double c1 = exp(-zt * tau);
#pragma unroll
            for (int j = 0; j < APT; ++j) {
                const double qy = c1 * py[j];
                px[j] = c1 * px[j] - tg * qy + tau * fxd(j);
                py[j] = qy + tau * (double)fy[j];
                pz[j] = c1 * pz[j] + tau * (double)fz[j];
            }
        } else {
        // ---- first half: S(tau) then K(tau)
        const double ppt = pp - 2.0 * tg * pxpy + tg * tg * pypy;
        const double g1 = sqrt(pp / ppt);
        const double fp1 = g1 * (fp - tg * fxpy);
        double s1, sd1;
        iso_kick_coeffs(fp1 / pp, ff / pp, tau, s1, sd1);
        const double isd1 = 1.0 / sd1;
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            const double qxp = g1 * (px[j] - tg * py[j]);
            const double qyp = g1 * py[j];
            const double qzp = g1 * pz[j];
            px[j] = (qxp + fxd(j) * s1) * isd1;
            py[j] = (qyp + (double)fy[j] * s1) * isd1;
            pz[j] = (qzp + (double)fz[j] * s1) * isd1;
        }
        }
        // ---- streaming D(h), new strain, sliding-brick wrap, peculiar path length
        k += 1;
        dxle = le_offset(S, gd, k);
        dxq = fix32(dxle, S.fix_scale[0]);
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            const double vx = px[j] + tg * py[j];
            const float dl = (float)h * sqrtf((float)(vx * vx + py[j] * py[j] + pz[j] * pz[j]));
            path[j] += dl;
            path_in[j] += dl;
            x[j] += h * px[j] + h * gd * (y[j] + tau * py[j]);
            y[j] += h * py[j];
            z[j] += h * pz[j];
            wrap_le(S, dxle, x[j], y[j], z[j]);
        }
        const float2 dm = nl_publish<APT>(S, x, y, z, qx, qy, qz, path, path_in, L);
        ++since;
        ++since_in;
        const float tsince = (float)(since * h), tin = (float)(since_in * h);
        // the same displacement bound guards the lists (skin) and the inner set (skin_in)
        const bool rebuild = 2.f * dm.x + agd * tsince * (reach + 2.f * dm.x) >= skin;
        if (rebuild) {
            nl_rebuild<APT>(S, dxle, dxq, x, y, z, qx, qy, qz, L, kmax, nmax);
            if (L.misc[1] != 0) {
                health |= kHealthListOverflow;
                break;
            }
#pragma unroll
            for (int j = 0; j < APT; ++j) path[j] = 0.f;
            since = 0;
        }
        if (rebuild || 2.f * dm.y + agd * tin * (reach + 2.f * dm.y) >= skin_in) {
            nl_inner<APT, kInnerPer>(S, dxq, qx, qy, qz, L, nmax, imask);
#pragma unroll
            for (int j = 0; j < APT; ++j) path_in[j] = 0.f;
            since_in = 0;
        }
        wpart = nl_forces<APT, OBS>(S, dxq, qx, qy, qz, imask, fx, fy, fz, L, nmax, xw);
        if (nh) {
            // ---- second half: K(tau) S(tau) T(tau), then Z(tau) on the new sum p^2
            const double c2 = exp(-zt * tau);
            double m4[4] = {0, 0, wpart, 0};  // pp, pxpy, W, position sum
#pragma unroll
            for (int j = 0; j < APT; ++j) {
                const double qy = py[j] + tau * (double)fy[j];
                px[j] = c2 * (px[j] + tau * fxd(j) - tg * qy);
                py[j] = c2 * qy;
                pz[j] = c2 * (pz[j] + tau * (double)fz[j]);
                m4[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                m4[1] += (COL && col) ? cq[j] * px[j] : px[j] * py[j];
                m4[3] += x[j] + y[j] + z[j];
            }
            block_sum<4>(m4, L.red);
            pp = m4[0];
            zt += tau * (pp - nh_tgt) * nh_iq;
            const double vpxy = (COL && col) ? m4[1] : m4[1] + m4[2];
            done += 1;
            if (t == 0) dsc->series[done] = vpxy;
            if (OBS && xs) nl_record_obs<APT>(S, y, px, py, pz, xw, xs, done, L);
            if (!isfinite(vpxy) || !isfinite(zt) || !isfinite(m4[3])) {
                health |= kHealthNonFinite;
                break;
            }
            continue;
        }
        // ---- moments of (p'', F): pp, pxpy, pypy, fp, fxpy, fypx, fxfy, fypy, fyfy, ff, W, pos
        double m[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, wpart, 0};
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            m[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
            m[1] += (COL && col) ? cq[j] * px[j] : px[j] * py[j];
            m[2] += py[j] * py[j];
            m[3] += fxd(j) * px[j] + (double)fy[j] * py[j] + (double)fz[j] * pz[j];
            m[4] += (COL && col) ? cq[j] * fxd(j) : fxd(j) * py[j];
            m[5] += (double)fy[j] * px[j];
            m[6] += fxd(j) * (double)fy[j];
            m[7] += (double)fy[j] * py[j];
            m[8] += (double)fy[j] * (double)fy[j];
            m[9] += fxd(j) * fxd(j) + (double)fy[j] * (double)fy[j] +
                    (double)fz[j] * (double)fz[j];
            m[11] += x[j] + y[j] + z[j];
        }
        block_sum<12>(m, L.red);
        double s2, sd2;
        iso_kick_coeffs(m[3] / m[0], m[9] / m[0], tau, s2, sd2);
        const double isd2 = 1.0 / sd2;
        const double pp3 = (m[0] + 2.0 * s2 * m[3] + s2 * s2 * m[9]) * isd2 * isd2;
        const double pxpy3 = (m[1] + s2 * (m[4] + m[5]) + s2 * s2 * m[6]) * isd2 * isd2;
        const double pypy3 = (m[2] + 2.0 * s2 * m[7] + s2 * s2 * m[8]) * isd2 * isd2;
        const double fp3 = (m[3] + s2 * m[9]) * isd2;
        const double fxpy3 = (m[4] + s2 * m[6]) * isd2;
        const double ppt2 = pp3 - 2.0 * tg * pxpy3 + tg * tg * pypy3;
        const double pxpyt = pxpy3 - tg * pypy3;
        const double c = sqrt(2.0 * k0 / ppt2);
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            const double qxp = (px[j] + fxd(j) * s2) * isd2;
            const double qyp = (py[j] + (double)fy[j] * s2) * isd2;
            const double qzp = (pz[j] + (double)fz[j] * s2) * isd2;
            px[j] = c * (qxp - tg * qyp);
            py[j] = c * qyp;
            pz[j] = c * qzp;
        }
        pp = c * c * ppt2;
        pxpy = c * c * pxpyt;
        pypy = c * c * pypy3;
        fp = c * (fp3 - tg * fxpy3);
        fxpy = c * fxpy3;
        ff = m[9];
        // colour: V J_x of the final momenta c (p + s2 F) / sd2 from the charge moments
        const double vpxy = (COL && col) ? c * (m[1] + s2 * m[4]) * isd2 : pxpy + m[10];
        done += 1;
        if (t == 0) dsc->series[done] = vpxy;
        if (OBS && xs) nl_record_obs<APT>(S, y, px, py, pz, xw, xs, done, L);
        if (!isfinite(vpxy) || !isfinite(c) || !isfinite(m[11])) {
            health |= kHealthNonFinite;
            break;
        }
        if (fabs(pp3 / m[0] - 1.0) > 1e-10) {
            health |= kHealthDrift;
            break;
        }
    }
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * T;
        if (a < n) {
            st[a] = x[j];
            st[n + a] = y[j];
            st[2 * n + a] = z[j];
            st[3 * n + a] = px[j];
            st[4 * n + a] = py[j];
            st[5 * n + a] = pz[j];
        }
    }
    if (t == 0) {
        dsc->k = k;
        dsc->done = done;
        dsc->k0 = k0;
        dsc->health = health;
        dsc->zeta = zt;
    }
    __syncthreads();
}

// The job slot sits at the start of the LDS; behind it the LDS is laid out per job for that
// daughter's own size, list grid and capacity, so a launch needs only the largest single
// footprint among its daughters.
constexpr int kNlJobBytes = 128;

// GL: the lists of each workgroup in global scratch (b.nbr, b.nbr_stride entries apart).
template <int APT, int MAXT, bool NH, bool OBS, bool COL, bool GL>
__global__ __launch_bounds__(MAXT) void k_daughters_nl(BatchLaunch b) {
    extern __shared__ __align__(32) char smem[];
    int32_t* job = (int32_t*)smem;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) *job = atomicAdd(b.queue, 1);
        __syncthreads();
        const int j = __builtin_amdgcn_readfirstlane(*job);
        if (j >= b.n_jobs) break;
        DaughterDesc* d = &b.descs[b.order[j]];
        const int n = d->sys.n, kmax = d->kmax;
        const int cells = d->sys.lc[0] * d->sys.lc[1] * d->sys.lc[2];
        const NlLds L = carve_nl(smem + kNlJobBytes, n, cells, kmax,
                                 GL ? b.nbr + (size_t)blockIdx.x * b.nbr_stride : nullptr);
        for (int c = threadIdx.x; c < cells; c += blockDim.x) L.cnt[c] = 0;
        // run_daughter_nl synchronises before its first use of the counts
        run_daughter_nl<APT, NH, OBS, COL>(d, b.max_steps, L, kmax, n);
    }
}

// ---------------------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------------------

template <int APT>
static hipError_t states_vpxy_t(const SysDev& S, const double* states, int32_t count, double* out,
                                int threads, hipStream_t s) {
    const size_t lds = plan_lds(S.n, S.nc[0] * S.nc[1] * S.nc[2], sizeof(double)).total;
    (void)hipFuncSetAttribute((const void*)k_states_vpxy<APT>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int grid = count < 2048 ? count : 2048;
    hipLaunchKernelGGL((k_states_vpxy<APT>), dim3(grid), dim3(threads), lds, s, S, states, count,
                       out);
    return hipGetLastError();
}

hipError_t launch_states_vpxy(const SysDev& S, const double* states, int32_t count, double* out,
                              hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int threads = pick_threads(S.n, 0);
    switch (pick_apt(S.n, threads)) {
        case 1: return states_vpxy_t<1>(S, states, count, out, threads, s);
        case 2: return states_vpxy_t<2>(S, states, count, out, threads, s);
        case 4: return states_vpxy_t<4>(S, states, count, out, threads, s);
    }
    return hipErrorInvalidValue;
}

int pick_threads(int n, int requested) {
    if (requested > 0) return requested;
    int t = ((n + 63) / 64) * 64;
    if (t > kMaxThreads) t = kMaxThreads;
    if (t < 64) t = 64;
    return t;
}

int pick_apt(int n, int threads) {
    const int need = (n + threads - 1) / threads;
    if (need <= 1) return 1;
    if (need <= 2) return 2;
    if (need <= 4) return 4;
    return -1;
}

size_t lds_bytes_nl(int n, int cells, int kmax, bool global_lists) {
    return kNlJobBytes + plan_nl(n, cells, kmax, global_lists).total;
}

size_t lds_bytes_for(int nmax, int cmax, int threads, int precision) {
    (void)threads;
    return plan_lds(nmax, cmax, precision == 0 ? sizeof(double) : sizeof(float)).total;
}

template <typename Real, int APT, int MAXT, bool NH>
static hipError_t launch_daughters_t(const BatchLaunch& b, hipStream_t s) {
    if (b.threads > MAXT) return hipErrorInvalidValue;
    (void)hipFuncSetAttribute((const void*)k_daughters<Real, APT, MAXT, NH>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)b.lds_bytes);
    hipLaunchKernelGGL((k_daughters<Real, APT, MAXT, NH>), dim3(b.grid), dim3(b.threads),
                       b.lds_bytes, s, b);
    return hipGetLastError();
}

template <typename Real, bool NH>
static hipError_t launch_daughters_r(const BatchLaunch& b, hipStream_t s) {
    // workgroups of up to 512 threads get a 256-register budget, 1024-thread ones 128
    if (b.threads <= 512) {
        switch (b.apt) {
            case 1: return launch_daughters_t<Real, 1, 512, NH>(b, s);
            case 2: return launch_daughters_t<Real, 2, 512, NH>(b, s);
            case 4: return launch_daughters_t<Real, 4, 512, NH>(b, s);
        }
    } else {
        switch (b.apt) {
            case 1: return launch_daughters_t<Real, 1, 1024, NH>(b, s);
            case 2: return launch_daughters_t<Real, 2, 1024, NH>(b, s);
            case 4: return launch_daughters_t<Real, 4, 1024, NH>(b, s);
        }
    }
    return hipErrorInvalidValue;
}

template <int APT, int MAXT, bool NH, bool OBS, bool COL, bool GL>
static hipError_t launch_nl_t(const BatchLaunch& b, hipStream_t s) {
    if (b.threads > MAXT) return hipErrorInvalidValue;
    (void)hipFuncSetAttribute((const void*)k_daughters_nl<APT, MAXT, NH, OBS, COL, GL>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)b.lds_bytes);
    hipLaunchKernelGGL((k_daughters_nl<APT, MAXT, NH, OBS, COL, GL>), dim3(b.grid),
                       dim3(b.threads), b.lds_bytes, s, b);
    return hipGetLastError();
}

template <bool NH, bool OBS, bool COL, bool GL = false>
static hipError_t launch_nl(const BatchLaunch& b, hipStream_t s) {
    if (b.threads <= 512) {
        switch (b.apt) {
            case 1: return launch_nl_t<1, 512, NH, OBS, COL, GL>(b, s);
            case 2: return launch_nl_t<2, 512, NH, OBS, COL, GL>(b, s);
            case 4: return launch_nl_t<4, 512, NH, OBS, COL, GL>(b, s);
        }
    } else {
        switch (b.apt) {
            case 1: return launch_nl_t<1, 1024, NH, OBS, COL, GL>(b, s);
            case 2: return launch_nl_t<2, 1024, NH, OBS, COL, GL>(b, s);
            case 4: return launch_nl_t<4, 1024, NH, OBS, COL, GL>(b, s);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_daughters(const BatchLaunch& b, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, b.queue, 1);
    // one instantiation per daughter thermostat: the isokinetic build does not carry the
    // Nose-Hoover branch's registers (10% on the list form)
    if (b.variant == kVariantNeighbourList) {
        if (b.precision != 1) return hipErrorInvalidValue;
        // the extra observables have their own instantiations, so the plain build carries
        // none of their registers
        // lists in global scratch: shear daughters of either thermostat, P_xy only
        if (b.global_lists) {
            if (b.obs || b.field || !b.nbr) return hipErrorInvalidValue;
            return b.thermo ? launch_nl<true, false, false, true>(b, s)
                            : launch_nl<false, false, false, true>(b, s);
        }
        // colour-field daughters: isokinetic, without the extra observables
        if (b.field) {
            if (b.obs) return hipErrorInvalidValue;
            return b.thermo ? launch_nl<true, false, true>(b, s) : launch_nl<false, false, true>(b, s);
        }
        if (b.obs)
            return b.thermo ? launch_nl<true, true, false>(b, s)
                            : launch_nl<false, true, false>(b, s);
        return b.thermo ? launch_nl<true, false, false>(b, s) : launch_nl<false, false, false>(b, s);
    }
    if (b.obs || b.field) return hipErrorInvalidValue;  // the cell form: shear and P_xy only
    if (b.thermo)
        return b.precision == 0 ? launch_daughters_r<double, true>(b, s)
                                : launch_daughters_r<float, true>(b, s);
    return b.precision == 0 ? launch_daughters_r<double, false>(b, s)
                            : launch_daughters_r<float, false>(b, s);
}

template <typename Real, int APT>
static hipError_t launch_mother_t(const MotherLaunch* dev_ms, int count, int threads, int nmax,
                                  int cmax, size_t lds, hipStream_t s) {
    (void)hipFuncSetAttribute((const void*)k_mother<Real, APT>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_mother<Real, APT>), dim3(count), dim3(threads), lds, s, dev_ms, nmax, cmax);
    return hipGetLastError();
}

// dev_ms: device array of `count` mothers sharing one launch shape (threads, apt, precision)
hipError_t launch_mothers(const MotherLaunch* dev_ms, int count, const MotherLaunch& shape,
                          hipStream_t s) {
    const int nmax = shape.sys.n, cmax = shape.sys.nc[0] * shape.sys.nc[1] * shape.sys.nc[2];
    if (shape.precision == 0) {
        switch (shape.apt) {
            case 1: return launch_mother_t<double, 1>(dev_ms, count, shape.threads, nmax, cmax, shape.lds_bytes, s);
            case 2: return launch_mother_t<double, 2>(dev_ms, count, shape.threads, nmax, cmax, shape.lds_bytes, s);
            case 4: return launch_mother_t<double, 4>(dev_ms, count, shape.threads, nmax, cmax, shape.lds_bytes, s);
        }
    } else {
        switch (shape.apt) {
            case 1: return launch_mother_t<float, 1>(dev_ms, count, shape.threads, nmax, cmax, shape.lds_bytes, s);
            case 2: return launch_mother_t<float, 2>(dev_ms, count, shape.threads, nmax, cmax, shape.lds_bytes, s);
            case 4: return launch_mother_t<float, 4>(dev_ms, count, shape.threads, nmax, cmax, shape.lds_bytes, s);
        }
    }
    return hipErrorInvalidValue;
}

// replica r of a mother: state = src + (0 | kicks[r]) on the momenta, zeta copied
__global__ void k_replicate(const double* src, const double* zsrc, int32_t n, const double* kicks,
                            double* dst, double* zdst) {
    const int r = blockIdx.x;
    double* d = dst + (size_t)r * 6 * n;
    const double* k = kicks ? kicks + (size_t)r * 3 * n : nullptr;
    for (int i = threadIdx.x; i < 6 * n; i += blockDim.x)
        d[i] = src[i] + ((k && i >= 3 * n) ? k[i - 3 * n] : 0.0);
    if (threadIdx.x == 0) zdst[r] = *zsrc;
}

hipError_t launch_replicate(const double* src, const double* zsrc, int32_t n, const double* kicks,
                            int32_t count, double* dst, double* zdst, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_replicate, dim3(count), dim3(256), 0, s, src, zsrc, n, kicks, dst, zdst);
    return hipGetLastError();
}

hipError_t launch_accumulate(const AccumLaunch& a, hipStream_t s) {
    if (a.n_groups <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_accumulate, dim3((a.n_groups + 63) / 64), dim3(64), 0, s, a);
    return hipGetLastError();
}

__global__ void k_copy_words(const uint64_t* src, uint64_t* dst, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_desc_zeta(DaughterDesc* descs, const double* zeta, const int32_t* state_of,
                            const int32_t* map_of, int32_t count) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= count) return;
    const double z = zeta[state_of[d]];
    descs[d].zeta = (map_of[d] & 1) ? -z : z;
}

hipError_t launch_desc_zeta(DaughterDesc* descs, const double* zeta, const int32_t* state_of,
                            const int32_t* map_of, int32_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_desc_zeta, dim3((count + 255) / 256), dim3(256), 0, s, descs, zeta,
                       state_of, map_of, count);
    return hipGetLastError();
}

// ---- autocorrelation of a series (choice of the sampling interval T_s) ----------------
// out[0] = mean of x[0..n) (one workgroup, fixed order: strided partial sums, then a block sum)
__global__ void k_series_mean(const double* x, int64_t n, double* out) {
    __shared__ double red[kMaxWaves * kRedSlots + kRedSlots];
    double v[1] = {0.0};
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) v[0] += x[i];
    block_sum<1>(v, red);
    if (threadIdx.x == 0) out[0] = v[0] / (double)n;
}

// acf[k] = C(k) / C(0), C(k) = sum_{i < n-k} (x_i - m)(x_{i+k} - m) / (n - k): one thread
// per lag; lanes of a wave read consecutive x_{i+k} and share x_i.
__global__ void k_acf(const double* x, int64_t n, const double* mean, int32_t max_lag,
                      double* acf) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const double m = mean[0];
    double c0 = 0.0, ck = 0.0, comp0 = 0.0, compk = 0.0;
    const bool live = k < max_lag && (int64_t)k < n;
    for (int64_t i = 0; i < n; ++i) {
        const double a = x[i] - m;
        // Neumaier sums: the lag-0 sum (each thread forms it, for its own normalisation)
        neumaier_add(c0, comp0, a * a);
        if (live && i + k < n) neumaier_add(ck, compk, a * (x[i + k] - m));
    }
    if (live) {
        const double cz = (c0 + comp0) / (double)n;
        acf[k] = ((ck + compk) / (double)(n - k)) / cz;
    }
}

// first lag k >= 1 with acf[k] < threshold (-1 if none), and the integrated correlation
// time 1/2 + sum_{1 <= k < k0} acf[k], k0 the first lag with acf[k] <= 0 (max_lag if none)
__global__ void k_acf_summary(const double* acf, int32_t max_lag, double threshold,
                              int32_t* first_below, double* tau_int) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int32_t fb = -1;
    for (int32_t k = 1; k < max_lag; ++k)
        if (acf[k] < threshold) {
            fb = k;
            break;
        }
    double tau = 0.5;
    for (int32_t k = 1; k < max_lag && acf[k] > 0.0; ++k) tau += acf[k];
    first_below[0] = fb;
    tau_int[0] = tau;
}

hipError_t launch_acf(const double* x, int64_t n, int32_t max_lag, double threshold,
                      double* scratch, double* acf, int32_t* first_below, double* tau_int,
                      hipStream_t s) {
    if (n < 2 || max_lag < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_series_mean, dim3(1), dim3(1024), 0, s, x, n, scratch);
    hipLaunchKernelGGL(k_acf, dim3((max_lag + 63) / 64), dim3(64), 0, s, x, n, scratch, max_lag,
                       acf);
    hipLaunchKernelGGL(k_acf_summary, dim3(1), dim3(64), 0, s, acf, max_lag, threshold,
                       first_below, tau_int);
    return hipGetLastError();
}

__global__ void k_increment(int32_t* counter) {
    if (threadIdx.x == 0) counter[0] = counter[0] + 1;
}

hipError_t launch_copy_words(const uint64_t* src, uint64_t* dst, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t want = (count + 255) / 256;
    const int64_t blocks = want < 1024 ? want : 1024;
    hipLaunchKernelGGL(k_copy_words, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, count);
    return hipGetLastError();
}

hipError_t launch_increment(int32_t* counter, hipStream_t s) {
    hipLaunchKernelGGL(k_increment, dim3(1), dim3(64), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_response(const ResponseLaunch& r, hipStream_t s) {
    hipLaunchKernelGGL(k_response, dim3((r.n_t + 63) / 64), dim3(64), 0, s, r);
    return hipGetLastError();
}

hipError_t launch_cv_beta(const ResponseLaunch& r, double* beta, hipStream_t s) {
    hipLaunchKernelGGL(k_cv_beta, dim3((r.n_t + 63) / 64), dim3(64), 0, s, r, beta);
    return hipGetLastError();
}

hipError_t launch_spawn(const double* states, int32_t n, int32_t n_states,
                        const int32_t* state_of, const int32_t* map_of, double* const* dst,
                        int32_t n_daughters, double lx, hipStream_t s) {
    (void)n_states;
    if (n_daughters <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_spawn, dim3(n_daughters), dim3(256), 0, s, states, n, state_of, map_of,
                       dst, lx);
    return hipGetLastError();
}

template <typename Real, int APT>
static hipError_t debug_cells_t(const SysDev& S, const double* r, int32_t* cell_of,
                                int32_t* order, int32_t* start, int threads, hipStream_t s) {
    const size_t lds = plan_lds(S.n, S.nc[0] * S.nc[1] * S.nc[2], sizeof(Real)).total;
    (void)hipFuncSetAttribute((const void*)k_debug_cells<Real, APT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_debug_cells<Real, APT>), dim3(1), dim3(threads), lds, s, S, r, cell_of,
                       order, start);
    return hipGetLastError();
}

hipError_t launch_debug_cells(const SysDev& S, const double* r, int32_t* cell_of, int32_t* order,
                              int32_t* start, hipStream_t s) {
    const int threads = pick_threads(S.n, 0);
    switch (pick_apt(S.n, threads)) {
        case 1: return debug_cells_t<float, 1>(S, r, cell_of, order, start, threads, s);
        case 2: return debug_cells_t<float, 2>(S, r, cell_of, order, start, threads, s);
        case 4: return debug_cells_t<float, 4>(S, r, cell_of, order, start, threads, s);
    }
    return hipErrorInvalidValue;
}

template <typename Real, int APT>
static hipError_t debug_forces_t(const SysDev& S, double dxle, const double* r, double* f,
                                 double* out, int threads, hipStream_t s) {
    const size_t lds = plan_lds(S.n, S.nc[0] * S.nc[1] * S.nc[2], sizeof(Real)).total;
    (void)hipFuncSetAttribute((const void*)k_debug_forces<Real, APT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_debug_forces<Real, APT>), dim3(1), dim3(threads), lds, s, S, dxle, r,
                       f, out);
    return hipGetLastError();
}

hipError_t launch_debug_forces(const SysDev& S, int precision, double dxle, const double* r,
                               double* f, double* out, hipStream_t s) {
    const int threads = pick_threads(S.n, 0);
    const int apt = pick_apt(S.n, threads);
    if (precision == 0) {
        switch (apt) {
            case 1: return debug_forces_t<double, 1>(S, dxle, r, f, out, threads, s);
            case 2: return debug_forces_t<double, 2>(S, dxle, r, f, out, threads, s);
            case 4: return debug_forces_t<double, 4>(S, dxle, r, f, out, threads, s);
        }
    } else {
        switch (apt) {
            case 1: return debug_forces_t<float, 1>(S, dxle, r, f, out, threads, s);
            case 2: return debug_forces_t<float, 2>(S, dxle, r, f, out, threads, s);
            case 4: return debug_forces_t<float, 4>(S, dxle, r, f, out, threads, s);
        }
    }
    return hipErrorInvalidValue;
}

template <int APT>
static hipError_t debug_pairs_t(const SysDev& S, double dxle, const double* r, double rlist,
                                int64_t cap, int32_t* pi, int32_t* pj,
                                unsigned long long* count, int threads, hipStream_t s) {
    const size_t lds = plan_lds(S.n, S.nc[0] * S.nc[1] * S.nc[2], sizeof(float)).total;
    (void)hipFuncSetAttribute((const void*)k_debug_pairs<APT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_debug_pairs<APT>), dim3(1), dim3(threads), lds, s, S, dxle, r, rlist,
                       cap, pi, pj, count);
    return hipGetLastError();
}

hipError_t launch_debug_pairs(const SysDev& S, double dxle, const double* r, double rlist,
                              int64_t cap, int32_t* pi, int32_t* pj, unsigned long long* count,
                              hipStream_t s) {
    const int threads = pick_threads(S.n, 0);
    switch (pick_apt(S.n, threads)) {
        case 1: return debug_pairs_t<1>(S, dxle, r, rlist, cap, pi, pj, count, threads, s);
        case 2: return debug_pairs_t<2>(S, dxle, r, rlist, cap, pi, pj, count, threads, s);
        case 4: return debug_pairs_t<4>(S, dxle, r, rlist, cap, pi, pj, count, threads, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace ttcf
