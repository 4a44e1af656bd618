// ttcf_elongation.hip -- planar elongational flow (PEF) daughters on gfx950.
//
// The Introduction names elongational flow among the fields TTCF extends to, and Section
// Mathematical Framework notes that a field other than shear needs mappings of its own. The
// paper prints no PEF equations; the dynamics here is SLLOD (Eq. system1 with the velocity
// gradient grad u = diag(rate, -rate, 0) in place of the shear) with the Gaussian isokinetic
// multiplier, in an orthorhombic box that deforms with the flow:
//   L_x = L_x0 e^e, L_y = L_y0 e^-e, L_z = L_z0, e = rate (k dt)   (volume conserved).
// Daughters are short transients, so the box needs no reproducible (Kraynik-Reinelt)
// lattice; the host refuses a daughter whose box edges would fall below 3 r_c.
//
// Positions are held as fractions s of the current box. Under the flow, ds/dt = p / L(t),
// which over a step with p fixed integrates exactly to s += h p phi(rate h) / L(t_k),
// phi(u) = (1 - e^-u) / u (and phi(-rate h) along y). One step of h = dt:
//   E(h/2) K(h/2) D(h) [k += 1, new box, cell list, forces] K(h/2) E(h/2), rescale to K0,
// E: p_x e^{-rate tau}, p_y e^{rate tau}, scaled back to the step's p.p (the multiplier's
// share of the flow term); K: the exact constrained kick under fixed forces (Zhang, J. Chem.
// Phys. 106, 6102 (1997)). B = P_xx - P_yy, recorded as V (P_xx - P_yy) after every step;
// Omega(0) = -(V/T) grad u : P = -(V/T) rate (P_xx - P_yy).
//
// Layout: one workgroup per daughter, two atoms per thread, momenta and forces in
// registers, fractional positions in LDS by atom id. The cell grid is rebuilt every step
// from the current box (n_a = floor(L_a / r_c) >= 3) with each cell's members in ascending
// atom id, and every pair is evaluated from both sides (FP64), so each force, virial and
// reduction has a fixed summation order: results are deterministic.

#include <math.h>

#include "ttcf_internal.h"

namespace ttcf {
namespace {

constexpr int kPefApt = 2;  // atoms per thread

constexpr int kPefMaxHits = 24;  // pairs within r_c per atom held between the two passes
constexpr int kPefScan = 3;      // candidates per lane per trip of the first pass

struct PefPlan {
    size_t sx, sy, sz, red, start, cnt, ws, sid, hits, total;
};

__host__ __device__ inline size_t pef_align(size_t v) { return (v + 15) & ~(size_t)15; }

__host__ __device__ inline PefPlan pef_plan(int nmax, int cmax) {
    PefPlan p;
    size_t o = 0;
    p.sx = o;
    o = pef_align(o + sizeof(double) * (size_t)nmax);
    p.sy = o;
    o = pef_align(o + sizeof(double) * (size_t)nmax);
    p.sz = o;
    o = pef_align(o + sizeof(double) * (size_t)nmax);
    p.red = o;
    o = pef_align(o + sizeof(double) * (size_t)(kMaxWaves * kRedSlots + kRedSlots));
    p.start = o;
    o = pef_align(o + sizeof(int32_t) * (size_t)(cmax + 1));
    p.cnt = o;
    o = pef_align(o + sizeof(int32_t) * (size_t)cmax);
    p.ws = o;
    o = pef_align(o + sizeof(int32_t) * (size_t)kMaxWaves);
    p.sid = o;
    o = pef_align(o + sizeof(uint16_t) * (size_t)nmax);
    p.hits = o;
    o = pef_align(o + sizeof(uint16_t) * (size_t)kPefMaxHits * kMaxThreads);
    p.total = o;
    return p;
}

struct PefShared {
    double *sx, *sy, *sz;  // [nmax] fractional positions by atom id
    double* red;           // reduction scratch
    int32_t* start;        // [cells + 1] first sorted slot of each cell
    int32_t* cnt;          // [cells] counts, then placement cursors
    int32_t* ws;           // [waves] scan scratch
    uint16_t* sid;         // [nmax] atom ids sorted by (cell, id)
    uint16_t* hits;        // [kPefMaxHits][threads] each lane's pairs within r_c (row, range, id)
};

// Sum of K doubles over the workgroup, the same total in every thread. Fixed order: an xor
// butterfly inside each wave (lane 0's result is used), then the waves in sequence.
template <int K>
__device__ __forceinline__ void pef_sum(double (&v)[K], double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    }
    if (lane == 0) {
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

__device__ __forceinline__ double pef_wrap(double s) {
    s -= floor(s);
    return s >= 1.0 ? 0.0 : s;
}

// (1 - e^-u) / u
__device__ __forceinline__ double pef_phi(double u) { return u == 0.0 ? 1.0 : -expm1(-u) / u; }

// Exact flow of dp/dt = F - alpha p over tau with F fixed and alpha = F.p / p.p:
// a = F.p/p.p, b = F.F/p.p, q = sqrt(b), s = a (cosh(q tau) - 1)/b + sinh(q tau)/q,
// sdot = a sinh(q tau)/q + cosh(q tau), p -> (p + F s) / sdot.
__device__ __forceinline__ void pef_kick_coeffs(double a, double b, double tau, double& s,
                                                double& sdot) {
    double ch1_b, sh_q;
    if (b > 0.0) {
        const double q = sqrt(b);
        const double hs = sinh(0.5 * q * tau) / q;
        ch1_b = 2.0 * hs * hs;
        sh_q = sinh(q * tau) / q;
    } else {
        ch1_b = 0.5 * tau * tau;
        sh_q = tau;
    }
    s = a * ch1_b + sh_q;
    sdot = a * sh_q + (1.0 + b * ch1_b);
}

__device__ __forceinline__ int pef_cell(double s, int nc) {
    const int c = (int)(s * (double)nc);
    return c > nc - 1 ? nc - 1 : c;
}

// Reciprocal: the hardware estimate refined by two Newton steps (within an ulp of 1/x).
__device__ __forceinline__ double pef_recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// Force on atom i in two passes over the 27-cell stencil of the current cell list. Pass 1
// runs its nine rows (dz, dy), each the rank range of the row's three x cells (two ranges
// where the row wraps in x), kPefScan candidates per lane per trip, and keeps the members
// within r_c in the lane's hit list as (row, range, atom id); pass 2 evaluates the listed
// pairs with every lane busy until the longest list is done, so the force arithmetic runs
// once per pair rather than once per candidate slot of the wave. Members keep the fixed
// (row, rank) order, so each force and virial sum has a fixed order. A stencil cell across
// the box edge is the image shifted by one box length (see pef_atom_force). SEP(ax, ay, az,
// m, d) sets the separation d of atom i at fractional (ax, ay, az) from member m; ACC(fs, d)
// adds a pair with force factor fs. A list longer than kPefMaxHits makes the force NaN
// (the daughter then fails its health check).
template <class SEP, class ACC>
__device__ __forceinline__ void pef_rows_force(const PefShared& S, int i, int ncx, int ncy,
                                               int ncz, double rc2, double ca, double& fx,
                                               double& fy, double& fz, SEP sep, ACC acc) {
    const int T = blockDim.x, t = threadIdx.x;
    const bool own = i >= 0;
    const double six = own ? S.sx[i] : 0.0, siy = own ? S.sy[i] : 0.0, siz = own ? S.sz[i] : 0.0;
    const int cx = pef_cell(six, ncx), cy = pef_cell(siy, ncy), cz = pef_cell(siz, ncz);
    // the second range of a row wrapping in x: cell ncx - 1 at +1 (cx = 0) or cell 0 at -1
    const double shx1 = cx == 0 ? 1.0 : -1.0;
    // image shifts of row r in y and z, and the first rank of its cell row
    auto row = [&](int r, double& shy, double& shz, int& rowb) {
        const int dz = r / 3 - 1, dy = r % 3 - 1;
        int zz = cz + dz, yy = cy + dy;
        shz = zz < 0 ? 1.0 : (zz >= ncz ? -1.0 : 0.0);
        zz += zz < 0 ? ncz : (zz >= ncz ? -ncz : 0);
        shy = yy < 0 ? 1.0 : (yy >= ncy ? -1.0 : 0.0);
        yy += yy < 0 ? ncy : (yy >= ncy ? -ncy : 0);
        rowb = ncx * (yy + ncy * zz);
    };
    int nh = 0;
#pragma unroll 1
    for (int r = 0; r < 9; ++r) {
        double shy, shz;
        int rowb;
        row(r, shy, shz, rowb);
        int lo0, hi0, lo1 = 0, hi1 = 0;
        if (cx >= 1 && cx <= ncx - 2) {
            lo0 = S.start[rowb + cx - 1];
            hi0 = S.start[rowb + cx + 2];
        } else if (cx == 0) {
            lo0 = S.start[rowb];
            hi0 = S.start[rowb + 2];
            lo1 = S.start[rowb + ncx - 1];
            hi1 = S.start[rowb + ncx];
        } else {
            lo0 = S.start[rowb + ncx - 2];
            hi0 = S.start[rowb + ncx];
            lo1 = S.start[rowb];
            hi1 = S.start[rowb + 1];
        }
        const int len0 = own ? hi0 - lo0 : 0;
        const int len = len0 + (own ? hi1 - lo1 : 0);
        const int off1 = lo1 - len0;
        const double ay = siy + shy, az = siz + shz;
        for (int v = 0; __builtin_amdgcn_ballot_w64(v < len) != 0; v += kPefScan) {
            int m[kPefScan];
#pragma unroll
            for (int u = 0; u < kPefScan; ++u) {
                const int vv = v + u;
                m[u] = S.sid[vv < len ? vv + (vv < len0 ? lo0 : off1) : 0];
            }
#pragma unroll
            for (int u = 0; u < kPefScan; ++u) {
                const int vv = v + u;
                const bool r1 = vv >= len0;
                double d[3];
                sep(six + (r1 ? shx1 : 0.0), ay, az, m[u], d);
                const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if ((vv < len) & (m[u] != i) & (r2 < rc2)) {
                    if (nh < kPefMaxHits)
                        S.hits[nh * T + t] = (uint16_t)((r << 12) | ((r1 ? 1 : 0) << 11) | m[u]);
                    ++nh;
                }
            }
        }
    }
    for (int k = 0; __builtin_amdgcn_ballot_w64(k < nh) != 0; ++k) {
        if (k < nh && k < kPefMaxHits) {
            const uint32_t e = S.hits[k * T + t];
            double shy, shz;
            int rowb;
            row((int)(e >> 12), shy, shz, rowb);
            double d[3];
            sep(six + ((e >> 11) & 1u ? shx1 : 0.0), siy + shy, siz + shz, (int)(e & 0x7FFu), d);
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            const double inv = pef_recip(r2);
            const double s3 = inv * inv * inv;
            const double fs = (48.0 * s3 * s3 - 24.0 * ca * s3) * inv;
            fx += fs * d[0];
            fy += fs * d[1];
            fz += fs * d[2];
            acc(fs, d);
        }
    }
    if (nh > kPefMaxHits) fx = __builtin_nan("");
}

// Force on atom i from the 27-cell stencil of the current cell list (cells in a fixed
// order, members in ascending id), and its half of the pair virial. A stencil cell across
// the box edge is the image shifted by one box length, so the separation of a member is
// (s_i - shift) - s_j: with cells at least r_c wide, every pair within r_c is found through
// its minimum image, and any other image is at least r_c away (every edge holds 3 cells).
__device__ __forceinline__ void pef_atom_force(const PefShared& S, int i, int ncx, int ncy,
                                               int ncz, double lx, double ly, double lz,
                                               double rc2, double ca, double& fx, double& fy,
                                               double& fz, double& w) {
    const double six = S.sx[i], siy = S.sy[i], siz = S.sz[i];
    const int cx = pef_cell(six, ncx), cy = pef_cell(siy, ncy), cz = pef_cell(siz, ncz);
#pragma unroll 1
    for (int dz = -1; dz <= 1; ++dz) {
        int zz = cz + dz;
        double az = siz;
        if (zz < 0) {
            zz += ncz;
            az += 1.0;
        } else if (zz >= ncz) {
            zz -= ncz;
            az -= 1.0;
        }
#pragma unroll 1
        for (int dy = -1; dy <= 1; ++dy) {
            int yy = cy + dy;
            double ay = siy;
            if (yy < 0) {
                yy += ncy;
                ay += 1.0;
            } else if (yy >= ncy) {
                yy -= ncy;
                ay -= 1.0;
            }
            for (int dx = -1; dx <= 1; ++dx) {
                int xx = cx + dx;
                double ax = six;
                if (xx < 0) {
                    xx += ncx;
                    ax += 1.0;
                } else if (xx >= ncx) {
                    xx -= ncx;
                    ax -= 1.0;
                }
                const int c = xx + ncx * (yy + ncy * zz);
                const int e = S.start[c + 1];
                for (int q = S.start[c]; q < e; ++q) {
                    const int m = S.sid[q];
                    if (m == i) continue;
                    const double ddx = (ax - S.sx[m]) * lx;
                    const double ddy = (ay - S.sy[m]) * ly;
                    const double ddz = (az - S.sz[m]) * lz;
                    const double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                    if (r2 < rc2) {
                        const double inv = pef_recip(r2);
                        const double s3 = inv * inv * inv;
                        const double fs = (48.0 * s3 * s3 - 24.0 * ca * s3) * inv;
                        fx += fs * ddx;
                        fy += fs * ddy;
                        fz += fs * ddz;
                        w += 0.5 * (fs * (ddx * ddx - ddy * ddy));
                    }
                }
            }
        }
    }
}

// Canonical cell list of the fractional positions in LDS: every thread calls it; it begins
// and ends with a barrier.
__device__ void pef_build_cells(const PefShared& S, int n, int ncx, int ncy, int ncz) {
    const int T = blockDim.x, t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6, nw = T >> 6;
    const int C = ncx * ncy * ncz;
    __syncthreads();
    for (int c = t; c < C; c += T) S.cnt[c] = 0;
    __syncthreads();
    int cell[kPefApt];
#pragma unroll
    for (int j = 0; j < kPefApt; ++j) {
        const int a = t + j * T;
        cell[j] = -1;
        if (a < n) {
            cell[j] = pef_cell(S.sx[a], ncx) +
                      ncx * (pef_cell(S.sy[a], ncy) + ncy * pef_cell(S.sz[a], ncz));
            atomicAdd(&S.cnt[cell[j]], 1);
        }
    }
    __syncthreads();
    // exclusive scan of the counts: contiguous chunks per thread, then waves in order
    {
        const int chunk = (C + T - 1) / T;
        const int b = t * chunk;
        const int e = min(C, b + chunk);
        int local = 0;
        for (int c = b; c < e; ++c) local += S.cnt[c];
        int x = local;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) S.ws[wave] = x;
        __syncthreads();
        if (t == 0) {
            int acc = 0;
            for (int v = 0; v < nw; ++v) {
                const int q = S.ws[v];
                S.ws[v] = acc;
                acc += q;
            }
            S.start[C] = acc;
        }
        __syncthreads();
        int run = S.ws[wave] + x - local;
        for (int c = b; c < e; ++c) {
            const int q = S.cnt[c];
            S.start[c] = run;
            S.cnt[c] = run;
            run += q;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPefApt; ++j)
        if (cell[j] >= 0) S.sid[atomicAdd(&S.cnt[cell[j]], 1)] = (uint16_t)(t + j * T);
    __syncthreads();
    // members of each cell in ascending atom id (insertion sort; a few atoms per cell)
    for (int c = t; c < C; c += T) {
        const int b = S.start[c], e = S.start[c + 1];
        for (int q = b + 1; q < e; ++q) {
            const uint16_t v = S.sid[q];
            int r = q - 1;
            while (r >= b && S.sid[r] > v) {
                S.sid[r + 1] = S.sid[r];
                --r;
            }
            S.sid[r + 1] = v;
        }
    }
    __syncthreads();
}

// The cell list, then the forces on the thread's atoms and its share of the pair virial
// W_xx - W_yy (each pair is seen from both sides, so each side adds half).
__device__ void pef_forces(const PefShared& S, int n, int ncx, int ncy, int ncz, double lx,
                           double ly, double lz, double rc2, double ca, double (&fx)[kPefApt],
                           double (&fy)[kPefApt], double (&fz)[kPefApt], double& w) {
    const int T = blockDim.x, t = threadIdx.x;
    pef_build_cells(S, n, ncx, ncy, ncz);
    w = 0.0;
    auto sep = [&](double ax, double ay, double az, int m, double (&d)[3]) {
        d[0] = (ax - S.sx[m]) * lx;
        d[1] = (ay - S.sy[m]) * ly;
        d[2] = (az - S.sz[m]) * lz;
    };
    auto acc = [&](double fs, const double (&d)[3]) {
        w += 0.5 * (fs * (d[0] * d[0] - d[1] * d[1]));
    };
    for (int j = 0; j < kPefApt; ++j) {
        const int i = t + j * T;
        double ax = 0.0, ay = 0.0, az = 0.0;
        pef_rows_force(S, i < n ? i : -1, ncx, ncy, ncz, rc2, ca, ax, ay, az, sep, acc);
        fx[j] = ax;
        fy[j] = ay;
        fz[j] = az;
    }
}

// NH: Nose-Hoover daughters (dp/dt gains -zeta p, d zeta/dt = (sum p^2 - nf T)/Q), stepped
// Z T E K D K E T Z over half steps with each part exact, in place of the isokinetic
// E K D K E and rescale.
template <bool NH>
__global__ void __launch_bounds__(1024) k_daughters_pef(PefLaunch L) {
    extern __shared__ __align__(16) char smem[];
    const PefPlan plan = pef_plan(L.nmax, L.cmax);
    PefShared S;
    S.sx = (double*)(smem + plan.sx);
    S.sy = (double*)(smem + plan.sy);
    S.sz = (double*)(smem + plan.sz);
    S.red = (double*)(smem + plan.red);
    S.start = (int32_t*)(smem + plan.start);
    S.cnt = (int32_t*)(smem + plan.cnt);
    S.ws = (int32_t*)(smem + plan.ws);
    S.sid = (uint16_t*)(smem + plan.sid);
    S.hits = (uint16_t*)(smem + plan.hits);

    DaughterDesc* dp = L.descs + L.order[blockIdx.x];
    const int T = blockDim.x, t = threadIdx.x;
    const int n = dp->sys.n;
    const int32_t done0 = dp->done;
    if (dp->health != 0 || done0 >= dp->n_steps) return;  // uniform over the workgroup
    const int steps = min(L.max_steps, dp->n_steps - done0);
    const double rate = dp->gamma_dot, h = dp->sys.dt;
    const double l0x = dp->sys.box[0], l0y = dp->sys.box[1], lz = dp->sys.box[2];
    const double rc = dp->sys.rc, rc2 = dp->sys.rc2, ca = dp->sys.c_attr;
    double* st = dp->state;
    double* series = dp->series;
    int64_t k = dp->k;
    int health = 0;
    if (n > T * kPefApt || n > L.nmax) health = kHealthNonFinite;  // the host sizes launches
    double e = rate * ((double)k * h);
    double lx = l0x * exp(e), ly = l0y * exp(-e);
    int ncx = (int)floor(lx / rc), ncy = (int)floor(ly / rc), ncz = (int)floor(lz / rc);
    if (ncx < 3 || ncy < 3 || ncz < 3 || ncx * ncy * ncz > L.cmax) health = kHealthNonFinite;
    if (health) {
        if (t == 0) dp->health = health;
        return;
    }
    const double ex = exp(-0.5 * rate * h), ey = exp(0.5 * rate * h), tau = 0.5 * h;
    double zeta = dp->zeta;
    const double nh_q = dp->nh_q, nh_target = dp->nh_target;
    const double phx = pef_phi(rate * h), phy = pef_phi(-rate * h);

    double px[kPefApt], py[kPefApt], pz[kPefApt];
    double fx[kPefApt], fy[kPefApt], fz[kPefApt];
#pragma unroll
    for (int j = 0; j < kPefApt; ++j) {
        const int a = t + j * T;
        px[j] = py[j] = pz[j] = 0.0;
        if (a < n) {
            S.sx[a] = pef_wrap(st[a] / lx);
            S.sy[a] = pef_wrap(st[n + a] / ly);
            S.sz[a] = pef_wrap(st[2 * n + a] / lz);
            px[j] = st[3 * n + a];
            py[j] = st[4 * n + a];
            pz[j] = st[5 * n + a];
        }
    }
    double w;
    pef_forces(S, n, ncx, ncy, ncz, lx, ly, lz, rc2, ca, fx, fy, fz, w);
    double k0 = dp->k0;
    {
        double v[3] = {0.0, 0.0, w};
#pragma unroll
        for (int j = 0; j < kPefApt; ++j) {
            v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
            v[1] += px[j] * px[j] - py[j] * py[j];
        }
        pef_sum<3>(v, S.red);
        if (done0 == 0) {
            k0 = 0.5 * v[0];
            if (t == 0) series[0] = v[1] + v[2];
        }
    }
    int it = 0;
    for (; it < steps; ++it) {
        if constexpr (NH) {
            // Z(h/2) T(h/2) E(h/2) K(h/2)
            {
                double v[1] = {0.0};
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                pef_sum<1>(v, S.red);
                zeta += tau * (v[0] - nh_target) / nh_q;
                const double sc = exp(-zeta * tau);
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    px[j] = (px[j] * sc) * ex + tau * fx[j];
                    py[j] = (py[j] * sc) * ey + tau * fy[j];
                    pz[j] = pz[j] * sc + tau * fz[j];
                }
            }
        } else {
            // E(h/2)
            {
                double v[2] = {0.0, 0.0};
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                    px[j] *= ex;
                    py[j] *= ey;
                    v[1] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                }
                pef_sum<2>(v, S.red);
                const double g = sqrt(v[0] / v[1]);
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    px[j] *= g;
                    py[j] *= g;
                    pz[j] *= g;
                }
            }
            // K(h/2)
            {
                double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                    v[1] += fx[j] * px[j] + fy[j] * py[j] + fz[j] * pz[j];
                    v[2] += fx[j] * fx[j] + fy[j] * fy[j] + fz[j] * fz[j];
                }
                pef_sum<3>(v, S.red);
                double s, sd;
                pef_kick_coeffs(v[1] / v[0], v[2] / v[0], 0.5 * h, s, sd);
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    px[j] = (px[j] + fx[j] * s) / sd;
                    py[j] = (py[j] + fy[j] * s) / sd;
                    pz[j] = (pz[j] + fz[j] * s) / sd;
                }
            }
        }
        // D(h) in fractional coordinates, then the box of step k + 1. Every thread has
        // passed the barriers of the two sums above, so no thread still reads S.sx, and
        // each thread moves only its own atoms.
        {
            const double ax = h * phx / lx, ay = h * phy / ly, az = h / lz;
#pragma unroll
            for (int j = 0; j < kPefApt; ++j) {
                const int a = t + j * T;
                if (a < n) {
                    S.sx[a] = pef_wrap(S.sx[a] + px[j] * ax);
                    S.sy[a] = pef_wrap(S.sy[a] + py[j] * ay);
                    S.sz[a] = pef_wrap(S.sz[a] + pz[j] * az);
                }
            }
            k += 1;
            e = rate * ((double)k * h);
            lx = l0x * exp(e);
            ly = l0y * exp(-e);
            ncx = (int)floor(lx / rc);
            ncy = (int)floor(ly / rc);
            if (ncx < 3 || ncy < 3 || ncx * ncy * ncz > L.cmax) {
                health = kHealthNonFinite;  // uniform: every thread stops here
                break;
            }
        }
        pef_forces(S, n, ncx, ncy, ncz, lx, ly, lz, rc2, ca, fx, fy, fz, w);
        if constexpr (NH) {
            // K(h/2) E(h/2) T(h/2) Z(h/2), with V (P_xx - P_yy) in the same sum
            {
                const double sc = exp(-zeta * tau);
                double v[3] = {0.0, 0.0, w};
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    px[j] = ((px[j] + tau * fx[j]) * ex) * sc;
                    py[j] = ((py[j] + tau * fy[j]) * ey) * sc;
                    pz[j] = (pz[j] + tau * fz[j]) * sc;
                    v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                    v[1] += px[j] * px[j] - py[j] * py[j];
                }
                pef_sum<3>(v, S.red);
                zeta += tau * (v[0] - nh_target) / nh_q;
                const double vn1 = v[1] + v[2];
                if (t == 0) series[done0 + it + 1] = vn1;
                if (!isfinite(vn1)) {
                    health = kHealthNonFinite;  // uniform: every thread holds the same sum
                    ++it;
                    break;
                }
            }
        } else {
            // K(h/2), with the virial of the new positions in the same sum
            {
                double v[4] = {0.0, 0.0, 0.0, w};
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                    v[1] += fx[j] * px[j] + fy[j] * py[j] + fz[j] * pz[j];
                    v[2] += fx[j] * fx[j] + fy[j] * fy[j] + fz[j] * fz[j];
                }
                pef_sum<4>(v, S.red);
                w = v[3];
                double s, sd;
                pef_kick_coeffs(v[1] / v[0], v[2] / v[0], 0.5 * h, s, sd);
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    px[j] = (px[j] + fx[j] * s) / sd;
                    py[j] = (py[j] + fy[j] * s) / sd;
                    pz[j] = (pz[j] + fz[j] * s) / sd;
                }
            }
            // E(h/2)
            {
                double v[2] = {0.0, 0.0};
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                    px[j] *= ex;
                    py[j] *= ey;
                    v[1] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                }
                pef_sum<2>(v, S.red);
                const double g = sqrt(v[0] / v[1]);
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    px[j] *= g;
                    py[j] *= g;
                    pz[j] *= g;
                }
            }
            // rescale to K0 (round-off only) and record V (P_xx - P_yy)
            {
                double v[2] = {0.0, 0.0};
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                    v[1] += px[j] * px[j] - py[j] * py[j];
                }
                pef_sum<2>(v, S.red);
                const double lam = sqrt(k0 / (0.5 * v[0]));
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    px[j] *= lam;
                    py[j] *= lam;
                    pz[j] *= lam;
                }
                const double vn1 = lam * lam * v[1] + w;
                if (t == 0) series[done0 + it + 1] = vn1;
                if (!isfinite(vn1)) {
                    health = kHealthNonFinite;  // uniform: every thread holds the same sum
                    ++it;
                    break;
                }
            }
        }
    }
    // the state in the coordinates of the current box
#pragma unroll
    for (int j = 0; j < kPefApt; ++j) {
        const int a = t + j * T;
        if (a < n) {
            st[a] = S.sx[a] * lx;
            st[n + a] = S.sy[a] * ly;
            st[2 * n + a] = S.sz[a] * lz;
            st[3 * n + a] = px[j];
            st[4 * n + a] = py[j];
            st[5 * n + a] = pz[j];
        }
    }
    if (t == 0) {
        dp->k = k;
        dp->done = done0 + it;
        dp->k0 = k0;
        if (NH) dp->zeta = zeta;
        dp->health = health;
    }
}

// ---- mixed flow: shear and planar elongation together ---------------------------------
// u_x = erate x + srate y, u_y = -erate y: dr/dt = p + A r, dp/dt = F - A p - alpha p with
// A = [[erate, srate, 0], [0, -erate, 0], [0, 0, 0]] (the Introduction names mixed flows
// among those TTCF extends to). The cell is the one the flow carries, H(t) = exp(A t)
// diag(L): H_xx = L e^{erate t}, H_xy = L srate t sinhc(erate t), H_yy = L e^{-erate t}.
// Positions are fractions s = H^-1 r; the streaming with p fixed gives exactly
// s += H(t)^-1 N p, N = int_0^h exp(-A u) du; the flow part E is p -> exp(-A tau) p. The
// cell grid uses the perpendicular widths of the tilted cell (n_x from L^2 / |b|, b its
// second edge), so the 27-cell stencil with image shifts finds every pair within r_c.
// The recorded flux is V J, J = (erate (P_xx - P_yy) + srate P_xy) / |rate|, and
// Omega(0) = -(V/T) |rate| J(0).

__device__ __forceinline__ double mix_sinhc(double x) { return x == 0.0 ? 1.0 : sinh(x) / x; }

struct MixCell {
    double hxx, hxy, hyy;
    int ncx, ncy;
};

__device__ __forceinline__ MixCell mix_cell(double l0x, double l0y, double er, double sr,
                                            double t, double rc) {
    MixCell c;
    const double x = er * t;
    c.hxx = l0x * exp(x);
    c.hxy = l0y * sr * t * mix_sinhc(x);
    c.hyy = l0y * exp(-x);
    const double wx = c.hxx * c.hyy / sqrt(c.hxy * c.hxy + c.hyy * c.hyy);
    c.ncx = (int)floor(wx / rc);
    c.ncy = (int)floor(c.hyy / rc);
    return c;
}

// Force on atom i in the tilted cell, and its halves of W_xx - W_yy and W_xy.
__device__ __forceinline__ void mix_atom_force(const PefShared& S, int i, int ncx, int ncy,
                                               int ncz, const MixCell& H, double lz,
                                               double rc2, double ca, double& fx, double& fy,
                                               double& fz, double& wn, double& wxy) {
    const double six = S.sx[i], siy = S.sy[i], siz = S.sz[i];
    const int cx = pef_cell(six, ncx), cy = pef_cell(siy, ncy), cz = pef_cell(siz, ncz);
#pragma unroll 1
    for (int dz = -1; dz <= 1; ++dz) {
        int zz = cz + dz;
        double az = siz;
        if (zz < 0) {
            zz += ncz;
            az += 1.0;
        } else if (zz >= ncz) {
            zz -= ncz;
            az -= 1.0;
        }
#pragma unroll 1
        for (int dy = -1; dy <= 1; ++dy) {
            int yy = cy + dy;
            double ay = siy;
            if (yy < 0) {
                yy += ncy;
                ay += 1.0;
            } else if (yy >= ncy) {
                yy -= ncy;
                ay -= 1.0;
            }
            for (int dx = -1; dx <= 1; ++dx) {
                int xx = cx + dx;
                double ax = six;
                if (xx < 0) {
                    xx += ncx;
                    ax += 1.0;
                } else if (xx >= ncx) {
                    xx -= ncx;
                    ax -= 1.0;
                }
                const int c = xx + ncx * (yy + ncy * zz);
                const int e = S.start[c + 1];
                for (int q = S.start[c]; q < e; ++q) {
                    const int m = S.sid[q];
                    if (m == i) continue;
                    const double fsx = ax - S.sx[m], fsy = ay - S.sy[m];
                    const double ddx = fsx * H.hxx + fsy * H.hxy;
                    const double ddy = fsy * H.hyy;
                    const double ddz = (az - S.sz[m]) * lz;
                    const double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                    if (r2 < rc2) {
                        const double inv = pef_recip(r2);
                        const double s3 = inv * inv * inv;
                        const double fs = (48.0 * s3 * s3 - 24.0 * ca * s3) * inv;
                        fx += fs * ddx;
                        fy += fs * ddy;
                        fz += fs * ddz;
                        wn += 0.5 * (fs * (ddx * ddx - ddy * ddy));
                        wxy += 0.5 * (fs * (ddx * ddy));
                    }
                }
            }
        }
    }
}

__device__ void mix_forces(const PefShared& S, int n, int ncz, const MixCell& H, double lz,
                           double rc2, double ca, double (&fx)[kPefApt], double (&fy)[kPefApt],
                           double (&fz)[kPefApt], double& wn, double& wxy) {
    const int T = blockDim.x, t = threadIdx.x;
    pef_build_cells(S, n, H.ncx, H.ncy, ncz);
    wn = 0.0;
    wxy = 0.0;
    auto sep = [&](double ax, double ay, double az, int m, double (&d)[3]) {
        const double fsx = ax - S.sx[m], fsy = ay - S.sy[m];
        d[0] = fsx * H.hxx + fsy * H.hxy;
        d[1] = fsy * H.hyy;
        d[2] = (az - S.sz[m]) * lz;
    };
    auto acc = [&](double fs, const double (&d)[3]) {
        wn += 0.5 * (fs * (d[0] * d[0] - d[1] * d[1]));
        wxy += 0.5 * (fs * (d[0] * d[1]));
    };
    for (int j = 0; j < kPefApt; ++j) {
        const int i = t + j * T;
        double ax = 0.0, ay = 0.0, az = 0.0;
        pef_rows_force(S, i < n ? i : -1, H.ncx, H.ncy, ncz, rc2, ca, ax, ay, az, sep, acc);
        fx[j] = ax;
        fy[j] = ay;
        fz[j] = az;
    }
}

// NH: Nose-Hoover daughters (Z T E K D K E T Z over half steps), else isokinetic
// (E K D K E with E and K constrained, then a rescale to K0).
template <bool NH>
__global__ void __launch_bounds__(1024) k_daughters_mix(PefLaunch L) {
    extern __shared__ __align__(16) char smem[];
    const PefPlan plan = pef_plan(L.nmax, L.cmax);
    PefShared S;
    S.sx = (double*)(smem + plan.sx);
    S.sy = (double*)(smem + plan.sy);
    S.sz = (double*)(smem + plan.sz);
    S.red = (double*)(smem + plan.red);
    S.start = (int32_t*)(smem + plan.start);
    S.cnt = (int32_t*)(smem + plan.cnt);
    S.ws = (int32_t*)(smem + plan.ws);
    S.sid = (uint16_t*)(smem + plan.sid);
    S.hits = (uint16_t*)(smem + plan.hits);

    DaughterDesc* dp = L.descs + L.order[blockIdx.x];
    const int T = blockDim.x, t = threadIdx.x;
    const int n = dp->sys.n;
    const int32_t done0 = dp->done;
    if (dp->health != 0 || done0 >= dp->n_steps) return;  // uniform over the workgroup
    const int steps = min(L.max_steps, dp->n_steps - done0);
    const double er = dp->erate, sr = dp->srate, rn = dp->gamma_dot, h = dp->sys.dt;
    const double l0x = dp->sys.box[0], l0y = dp->sys.box[1], lz = dp->sys.box[2];
    const double rc = dp->sys.rc, rc2 = dp->sys.rc2, ca = dp->sys.c_attr;
    double* st = dp->state;
    double* series = dp->series;
    // the flux components P_xx - P_yy and P_xy (columns 0 and 1 of kObsCols per time point)
    double* xs = dp->xseries;
    const double inv_v = 1.0 / dp->sys.volume;
    int64_t k = dp->k;
    int health = 0;
    if (n > T * kPefApt || n > L.nmax || !(rn > 0.0)) health = kHealthNonFinite;
    MixCell H = mix_cell(l0x, l0y, er, sr, (double)k * h, rc);
    const int ncz = (int)floor(lz / rc);
    if (H.ncx < 3 || H.ncy < 3 || ncz < 3 || H.ncx * H.ncy * ncz > L.cmax)
        health = kHealthNonFinite;
    if (health) {
        if (t == 0) dp->health = health;
        return;
    }
    const double tau = 0.5 * h;
    // Per-daughter constants live in LDS and are read where they are used, which keeps them
    // out of the registers that the force loop needs: exp(-A tau) (fa, fc, fd),
    // N = int_0^h exp(-A u) du (nxx, nxy, nyy), the rates, the thermostat, 1/V and K0.
    __shared__ double kc[16];
    enum { kFa, kFc, kFd, kNxx, kNxy, kNyy, kEr, kSr, kRn, kQ, kTarget, kInvV, kK0, kL0x, kL0y };
    if (t == 0) {
        kc[kFa] = exp(-er * tau);
        kc[kFd] = exp(er * tau);
        kc[kFc] = -sr * tau * mix_sinhc(er * tau);
        kc[kNxx] = h * pef_phi(er * h);
        kc[kNyy] = h * pef_phi(-er * h);
        const double hs = mix_sinhc(0.5 * er * h);
        kc[kNxy] = -sr * 0.5 * h * h * hs * hs;
        kc[kEr] = er;
        kc[kSr] = sr;
        kc[kRn] = rn;
        kc[kQ] = dp->nh_q;
        kc[kTarget] = dp->nh_target;
        kc[kInvV] = inv_v;
        kc[kL0x] = l0x;
        kc[kL0y] = l0y;
    }
    double zeta = dp->zeta;

    double px[kPefApt], py[kPefApt], pz[kPefApt];
    double fx[kPefApt], fy[kPefApt], fz[kPefApt];
#pragma unroll
    for (int j = 0; j < kPefApt; ++j) {
        const int a = t + j * T;
        px[j] = py[j] = pz[j] = 0.0;
        if (a < n) {
            const double sy = st[n + a] / H.hyy;
            S.sx[a] = pef_wrap((st[a] - H.hxy * sy) / H.hxx);
            S.sy[a] = pef_wrap(sy);
            S.sz[a] = pef_wrap(st[2 * n + a] / lz);
            px[j] = st[3 * n + a];
            py[j] = st[4 * n + a];
            pz[j] = st[5 * n + a];
        }
    }
    double wn, wxy;
    mix_forces(S, n, ncz, H, lz, rc2, ca, fx, fy, fz, wn, wxy);
    double k0 = dp->k0;
    {
        double v[5] = {0.0, 0.0, 0.0, wn, wxy};
#pragma unroll
        for (int j = 0; j < kPefApt; ++j) {
            v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
            v[1] += px[j] * px[j] - py[j] * py[j];
            v[2] += px[j] * py[j];
        }
        pef_sum<5>(v, S.red);
        if (done0 == 0) {
            k0 = 0.5 * v[0];
            if (t == 0) {
                series[0] = (er * (v[1] + v[3]) + sr * (v[2] + v[4])) / rn;
                if (xs) {
                    xs[0] = (v[1] + v[3]) * inv_v;
                    xs[1] = (v[2] + v[4]) * inv_v;
                    for (int c = 2; c < kObsCols; ++c) xs[c] = 0.0;
                }
            }
        }
    }
    if (t == 0) kc[kK0] = k0;
    __syncthreads();
    int it = 0;
    for (; it < steps; ++it) {
        if constexpr (NH) {
            // Z(h/2) T(h/2) E(h/2) K(h/2)
            double v[1] = {0.0};
#pragma unroll
            for (int j = 0; j < kPefApt; ++j) v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
            pef_sum<1>(v, S.red);
            zeta += tau * (v[0] - kc[kTarget]) / kc[kQ];
            const double sc = exp(-zeta * tau);
#pragma unroll
            for (int j = 0; j < kPefApt; ++j) {
                const double qx = px[j] * sc, qy = py[j] * sc;
                px[j] = (kc[kFa] * qx + kc[kFc] * qy) + tau * fx[j];
                py[j] = kc[kFd] * qy + tau * fy[j];
                pz[j] = pz[j] * sc + tau * fz[j];
            }
        } else {
            // E(h/2), constrained
            {
                double v[2] = {0.0, 0.0};
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                    const double qx = kc[kFa] * px[j] + kc[kFc] * py[j];
                    py[j] = kc[kFd] * py[j];
                    px[j] = qx;
                    v[1] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                }
                pef_sum<2>(v, S.red);
                const double g = sqrt(v[0] / v[1]);
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    px[j] *= g;
                    py[j] *= g;
                    pz[j] *= g;
                }
            }
            // K(h/2)
            {
                double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                    v[1] += fx[j] * px[j] + fy[j] * py[j] + fz[j] * pz[j];
                    v[2] += fx[j] * fx[j] + fy[j] * fy[j] + fz[j] * fz[j];
                }
                pef_sum<3>(v, S.red);
                double s1, sd;
                pef_kick_coeffs(v[1] / v[0], v[2] / v[0], tau, s1, sd);
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    px[j] = (px[j] + fx[j] * s1) / sd;
                    py[j] = (py[j] + fy[j] * s1) / sd;
                    pz[j] = (pz[j] + fz[j] * s1) / sd;
                }
            }
        }
        // D(h): s += H(t)^-1 N p (every thread has passed the barriers of the sums above, so
        // no thread still reads S.sx; each thread moves only its own atoms), then the cell
        // of step k + 1
        {
#pragma unroll
            for (int j = 0; j < kPefApt; ++j) {
                const int a = t + j * T;
                if (a < n) {
                    const double uy = kc[kNyy] * py[j];
                    const double dsy = uy / H.hyy;
                    const double dsx = ((kc[kNxx] * px[j] + kc[kNxy] * py[j]) - H.hxy * dsy) / H.hxx;
                    S.sx[a] = pef_wrap(S.sx[a] + dsx);
                    S.sy[a] = pef_wrap(S.sy[a] + dsy);
                    S.sz[a] = pef_wrap(S.sz[a] + h * pz[j] / lz);
                }
            }
            k += 1;
            H = mix_cell(kc[kL0x], kc[kL0y], kc[kEr], kc[kSr], (double)k * h, rc);
            if (H.ncx < 3 || H.ncy < 3 || H.ncx * H.ncy * ncz > L.cmax) {
                health = kHealthNonFinite;  // uniform: every thread stops here
                break;
            }
        }
        mix_forces(S, n, ncz, H, lz, rc2, ca, fx, fy, fz, wn, wxy);
        double vj, cn, cxy;  // flux, V (P_xx - P_yy), V P_xy
        if constexpr (NH) {
            // K(h/2) E(h/2) T(h/2) Z(h/2), with the flux in the same sum
            const double sc = exp(-zeta * tau);
            double v[5] = {0.0, 0.0, 0.0, wn, wxy};
#pragma unroll
            for (int j = 0; j < kPefApt; ++j) {
                const double qx = px[j] + tau * fx[j], qy = py[j] + tau * fy[j];
                px[j] = (kc[kFa] * qx + kc[kFc] * qy) * sc;
                py[j] = (kc[kFd] * qy) * sc;
                pz[j] = (pz[j] + tau * fz[j]) * sc;
                v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                v[1] += px[j] * px[j] - py[j] * py[j];
                v[2] += px[j] * py[j];
            }
            pef_sum<5>(v, S.red);
            zeta += tau * (v[0] - kc[kTarget]) / kc[kQ];
            cn = v[1] + v[3];
            cxy = v[2] + v[4];
            vj = (kc[kEr] * cn + kc[kSr] * cxy) / kc[kRn];
        } else {
            // K(h/2)
            {
                double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                    v[1] += fx[j] * px[j] + fy[j] * py[j] + fz[j] * pz[j];
                    v[2] += fx[j] * fx[j] + fy[j] * fy[j] + fz[j] * fz[j];
                }
                pef_sum<3>(v, S.red);
                double s1, sd;
                pef_kick_coeffs(v[1] / v[0], v[2] / v[0], tau, s1, sd);
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    px[j] = (px[j] + fx[j] * s1) / sd;
                    py[j] = (py[j] + fy[j] * s1) / sd;
                    pz[j] = (pz[j] + fz[j] * s1) / sd;
                }
            }
            // E(h/2), constrained
            {
                double v[2] = {0.0, 0.0};
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                    const double qx = kc[kFa] * px[j] + kc[kFc] * py[j];
                    py[j] = kc[kFd] * py[j];
                    px[j] = qx;
                    v[1] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                }
                pef_sum<2>(v, S.red);
                const double g = sqrt(v[0] / v[1]);
#pragma unroll
                for (int j = 0; j < kPefApt; ++j) {
                    px[j] *= g;
                    py[j] *= g;
                    pz[j] *= g;
                }
            }
            // rescale to K0 (round-off only), with the flux in the same sum
            double v[5] = {0.0, 0.0, 0.0, wn, wxy};
#pragma unroll
            for (int j = 0; j < kPefApt; ++j) {
                v[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
                v[1] += px[j] * px[j] - py[j] * py[j];
                v[2] += px[j] * py[j];
            }
            pef_sum<5>(v, S.red);
            const double lam = sqrt(kc[kK0] / (0.5 * v[0]));
#pragma unroll
            for (int j = 0; j < kPefApt; ++j) {
                px[j] *= lam;
                py[j] *= lam;
                pz[j] *= lam;
            }
            cn = lam * lam * v[1] + v[3];
            cxy = lam * lam * v[2] + v[4];
            vj = (kc[kEr] * cn + kc[kSr] * cxy) / kc[kRn];
        }
        if (t == 0) {
            series[done0 + it + 1] = vj;
            if (xs) {
                double* row = xs + (size_t)(done0 + it + 1) * kObsCols;
                row[0] = cn * kc[kInvV];
                row[1] = cxy * kc[kInvV];
                for (int c = 2; c < kObsCols; ++c) row[c] = 0.0;
            }
        }
        if (!isfinite(vj)) {
            health = kHealthNonFinite;  // uniform: every thread holds the same sum
            ++it;
            break;
        }
    }
    // the state in the coordinates of the current cell
#pragma unroll
    for (int j = 0; j < kPefApt; ++j) {
        const int a = t + j * T;
        if (a < n) {
            st[a] = H.hxx * S.sx[a] + H.hxy * S.sy[a];
            st[n + a] = H.hyy * S.sy[a];
            st[2 * n + a] = lz * S.sz[a];
            st[3 * n + a] = px[j];
            st[4 * n + a] = py[j];
            st[5 * n + a] = pz[j];
        }
    }
    if (t == 0) {
        dp->k = k;
        dp->done = done0 + it;
        dp->k0 = k0;
        if (NH) dp->zeta = zeta;
        dp->health = health;
    }
}

// Start states of planar-elongation daughters under their mappings: bit 1 of map exchanges
// the x and y axes of positions and momenta (the box is cubic), bit 0 reverses the momenta.
// Mixed-flow daughters (mix): bit 1 exchanges the axes, then bit 0 reflects x
// (x -> L_x - x, p_x -> -p_x).
__global__ void k_spawn_pef(const double* states, int32_t n, const int32_t* state_of,
                            const int32_t* map_of, double* const* dst, int32_t mix, double lx) {
    const int d = blockIdx.x;
    const double* src = states + (size_t)state_of[d] * 6 * (size_t)n;
    double* out = dst[d];
    const int m = map_of[d];
    const bool sw = (m & 2) != 0;
    const bool rev = !mix && (m & 1) != 0;
    const bool refl = mix && (m & 1) != 0;
    const double sg = rev ? -1.0 : 1.0;
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        const double x = src[a], y = src[n + a], z = src[2 * n + a];
        const double px = src[3 * n + a], py = src[4 * n + a], pz = src[5 * n + a];
        const double xs = sw ? y : x;
        out[a] = refl ? (xs == 0.0 ? 0.0 : lx - xs) : xs;
        out[n + a] = sw ? x : y;
        out[2 * n + a] = z;
        out[3 * n + a] = (refl ? -1.0 : sg) * (sw ? py : px);
        out[4 * n + a] = sg * (sw ? px : py);
        out[5 * n + a] = sg * pz;
    }
}

}  // namespace

int pef_threads(int nmax) {
    const int half = (nmax + kPefApt - 1) / kPefApt;
    const int t = ((half + 63) / 64) * 64;
    return t < 64 ? 64 : t;
}

int pef_max_cells(double volume, double rc) {
    return (int)floor(volume / (rc * rc * rc));
}

size_t lds_bytes_pef(int nmax, int cmax) { return pef_plan(nmax, cmax).total; }

hipError_t launch_pef(const PefLaunch& L, hipStream_t s) {
    if (L.n_jobs <= 0) return hipSuccess;
    if (L.threads < 64 || L.threads > kMaxThreads || L.threads % 64 != 0 ||
        L.nmax > L.threads * kPefApt || L.cmax < 27)
        return hipErrorInvalidValue;
    if (L.mix) {
        if (L.thermo) {
            (void)hipFuncSetAttribute((const void*)k_daughters_mix<true>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_bytes);
            hipLaunchKernelGGL(k_daughters_mix<true>, dim3(L.n_jobs), dim3(L.threads),
                               L.lds_bytes, s, L);
        } else {
            (void)hipFuncSetAttribute((const void*)k_daughters_mix<false>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_bytes);
            hipLaunchKernelGGL(k_daughters_mix<false>, dim3(L.n_jobs), dim3(L.threads),
                               L.lds_bytes, s, L);
        }
    } else if (L.thermo) {
        (void)hipFuncSetAttribute((const void*)k_daughters_pef<true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_bytes);
        hipLaunchKernelGGL(k_daughters_pef<true>, dim3(L.n_jobs), dim3(L.threads), L.lds_bytes, s,
                           L);
    } else {
        (void)hipFuncSetAttribute((const void*)k_daughters_pef<false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_bytes);
        hipLaunchKernelGGL(k_daughters_pef<false>, dim3(L.n_jobs), dim3(L.threads), L.lds_bytes,
                           s, L);
    }
    return hipGetLastError();
}

hipError_t launch_spawn_pef(const double* states, int32_t n, const int32_t* state_of,
                            const int32_t* map_of, double* const* dst, int32_t n_daughters,
                            int32_t mix, double lx, hipStream_t s) {
    if (n_daughters <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_spawn_pef, dim3(n_daughters), dim3(256), 0, s, states, n, state_of,
                       map_of, dst, mix, lx);
    return hipGetLastError();
}

}  // namespace ttcf
