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

#include "ttcf_device.h"

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

// s + e = a + b exactly (Knuth's branch-free two-sum)
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    const double bp = s - a;
    e = (a - (s - bp)) + (b - bp);
}

// Inclusive prefix sum over the 64 lanes of a wave, compensated: on return s + c is the sum
// of the lane's and all lower lanes' v, each partial carried as a two-sum pair (a fixed
// combination order, so the result does not depend on timing).
__device__ __forceinline__ void wave_scan_comp(double v, double& s, double& c) {
    const int lane = threadIdx.x & 63;
    s = v;
    c = 0.0;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double ls = __shfl_up(s, d, 64), lc = __shfl_up(c, d, 64);
        if (lane >= d) {
            double t, e;
            two_sum(ls, s, t, e);
            s = t;
            c = lc + c + e;
        }
    }
}

// One wave per group; its lanes take 64 consecutive time points at a time. The trapezoid
// terms of int_0^t P(0) P(s) ds are summed by a compensated prefix scan over the lanes, with
// the total so far carried from one block of 64 points to the next.
__global__ __launch_bounds__(64) void k_accumulate(AccumLaunch a) {
    const int g = blockIdx.x, lane = threadIdx.x;
    const int b = a.first_of[g], e = a.first_of[g + 1];
    // output row of this group
    const size_t row = (size_t)g + (a.row_step ? (size_t)(*a.row_step) * (size_t)a.n_groups : 0);
    const size_t stride = a.row_stride > 0 ? (size_t)a.row_stride : (size_t)a.n_t;
    const int nm = min(e - b, kMaxMaps);
    int health = 0;
    double p0[kMaxMaps], cs[kMaxMaps], cc[kMaxMaps];
    const double* ser[kMaxMaps];
    double inv_v = 1.0, dt = 0.0;
    for (int m = 0; m < nm; ++m) {
        const DaughterDesc& d = a.descs[b + m];
        health |= d.health;
        ser[m] = d.series;
        inv_v = 1.0 / d.sys.volume;
        dt = d.sys.dt;
        p0[m] = d.series[0] * inv_v;
        cs[m] = 0.0;
        cc[m] = 0.0;
    }
    if (lane == 0) {
        a.health_out[row] = health;
        a.gamma_out[row] = a.descs[b].gamma_dot;
    }
    const double inm = 1.0 / (double)nm;
    double* dout = a.d_out + row * stride;
    double* iout = a.i_out + row * stride;
    if (a.h_out) {
        // mapping mean of the learned control variate (0 where a daughter has none)
        double* hout = a.h_out + row * stride;
        for (int k = lane; k < a.n_t; k += 64) {
            double hs = 0.0;
            for (int m = 0; m < nm; ++m) {
                const double* hh = a.descs[b + m].hseries;
                hs += hh ? hh[k] : 0.0;
            }
            hout[k] = hs * inm;
        }
    }
    for (int k0 = 0; k0 < a.n_t; k0 += 64) {
        const int k = k0 + lane;
        const bool live = k < a.n_t;
        double dsum = 0.0, isum = 0.0;
        for (int m = 0; m < nm; ++m) {
            const double cur = live ? ser[m][k] * inv_v : 0.0;
            const double prev = live && k > 0 ? ser[m][k - 1] * inv_v : 0.0;
            // the trapezoid over [t_{k-1}, t_k] (none at k = 0)
            const double term = live && k > 0 ? 0.5 * dt * (p0[m] * prev + p0[m] * cur) : 0.0;
            double s, c;
            wave_scan_comp(term, s, c);
            double t, err;
            two_sum(cs[m], s, t, err);
            const double tc = cc[m] + c + err;
            dsum += cur;
            isum += t + tc;
            cs[m] = __shfl(t, 63, 64);
            cc[m] = __shfl(tc, 63, 64);
        }
        if (live) {
            dout[k] = dsum * inm;
            iout[k] = isum * inm;
        }
    }
}

// ---------------------------------------------------------------------------------------
// response: mean and block standard error over the selected groups, per time point
// ---------------------------------------------------------------------------------------
// G_n(t) = D_n(0) - coef_n I_n(t), coef_n = V gamma_n / T, is the start state's TTCF estimate
// (Eq. TTCF with Omega(0) = -(V/T) gamma_n P_xy(0)); D_n(t) its direct average. Two passes
// (mean, then the squared deviations). A workgroup takes 64 time points, one per lane; its
// kRespWaves waves split the rows (wave w takes rows w, w + kRespWaves, ...), each a
// compensated sum, and the wave partials are combined in wave order: a fixed order.
constexpr int kRespWaves = 16;

__device__ __forceinline__ void resp_values(const ResponseLaunch& r, int row, int k,
                                            double beta, double& g, double& dv) {
    const double* dser = r.d_all + (size_t)row * r.n_t_stride;
    const double* iser = r.i_all + (size_t)row * r.n_t_stride;
    g = dser[0] - r.coef[row] * iser[k];
    if (r.h_all) g -= beta * r.h_all[(size_t)row * r.n_t_stride + k];
    dv = dser[k];
    if (r.normalise) {
        const double gam = r.gamma[row];
        g /= gam;
        dv /= gam;
    }
}

// the block-wide compensated sums of two per-thread (sum, comp) pairs, per lane, in wave
// order; every thread receives its lane's totals
__device__ __forceinline__ void resp_combine(double (*part)[kRespWaves][64], double& a_s,
                                             double& a_c, double& b_s, double& b_c) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    part[0][w][lane] = a_s;
    part[1][w][lane] = a_c;
    part[2][w][lane] = b_s;
    part[3][w][lane] = b_c;
    __syncthreads();
    double as = 0, ac = 0, bs = 0, bc = 0;
    for (int v = 0; v < kRespWaves; ++v) {
        neumaier_add(as, ac, part[0][v][lane]);
        neumaier_add(as, ac, part[1][v][lane]);
        neumaier_add(bs, bc, part[2][v][lane]);
        neumaier_add(bs, bc, part[3][v][lane]);
    }
    __syncthreads();  // the partials may be overwritten after this
    a_s = as;
    a_c = ac;
    b_s = bs;
    b_c = bc;
}

__global__ __launch_bounds__(64 * kRespWaves) void k_response(ResponseLaunch r) {
    __shared__ double part[4][kRespWaves][64];
    __shared__ int cnt[kRespWaves];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int k0 = blockIdx.x * 64 + lane;
    const bool live = k0 < r.n_t;
    const int k = live ? k0 : 0;
    double gs = 0, gc = 0, ds = 0, dc = 0;
    int used = 0;
    const double beta = r.beta ? r.beta[k] : 1.0;
    for (int i = w; i < r.n_rows; i += kRespWaves) {
        const int row = r.rows[i];
        if (r.health[row] != 0) continue;
        double g, dv;
        resp_values(r, row, k, beta, g, dv);
        neumaier_add(gs, gc, g);
        neumaier_add(ds, dc, dv);
        ++used;
    }
    if (lane == 0) cnt[w] = used;
    resp_combine(part, gs, gc, ds, dc);  // (its first barrier also publishes cnt)
    used = 0;
    for (int v = 0; v < kRespWaves; ++v) used += cnt[v];
    const double gm = (gs + gc) / (double)used;
    const double dm = (ds + dc) / (double)used;
    double gv = 0, gvc = 0, dvv = 0, dvc = 0;
    for (int i = w; i < r.n_rows; i += kRespWaves) {
        const int row = r.rows[i];
        if (r.health[row] != 0) continue;
        double g, dv;
        resp_values(r, row, k, beta, g, dv);
        neumaier_add(gv, gvc, (g - gm) * (g - gm));
        neumaier_add(dvv, dvc, (dv - dm) * (dv - dm));
    }
    resp_combine(part, gv, gvc, dvv, dvc);
    if (w != 0 || !live) return;
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

hipError_t launch_daughters(const BatchLaunch& b, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, b.queue, 1);
    // one instantiation per daughter thermostat: the isokinetic build does not carry the
    // Nose-Hoover branch's registers (10% on the list form)
    if (b.variant == kVariantNeighbourList) return launch_pairs(b, s);
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
    hipLaunchKernelGGL(k_accumulate, dim3(a.n_groups), dim3(64), 0, s, a);
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
    hipLaunchKernelGGL(k_response, dim3((r.n_t + 63) / 64), dim3(64 * kRespWaves), 0, s, r);
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
