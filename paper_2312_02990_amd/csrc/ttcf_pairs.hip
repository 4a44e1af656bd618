// ttcf_pairs.hip -- pair-list form of the daughter step kernel on gfx950 (FP32 pair forces,
// FP64 integration, thermostat and sums).
//
// One workgroup integrates one daughter at a time (persistent, jobs from a queue), four atoms
// per thread: atom a belongs to thread a mod T_job, T_job = 64 ceil(n / 256), so a daughter's
// arithmetic does not depend on the launch's workgroup size. Positions and momenta stay in
// FP64 registers of their owner for the whole call.
//
// Pair list. Every pair closer than the list radius r_l = r_c + skin is stored once, as one
// 32-bit word (two 14-bit atom ranks and whether the pair crosses the y boundary), in a
// segment that belongs to one wave: in LDS after the job's layout when all segments fit
// there, else in per-workgroup global scratch. The list is built from a cell grid whose cells
// are at least r_l wide: the atoms are counting-sorted into canonical (cell, atom id) order
// (their rank), and the atom of rank s scans the half of the 27-cell neighbourhood that lies
// after it (its own cell past s, the next cell in x, the row above in y, and the three rows
// of the next layer in z; rows across the y boundary are the Lees-Edwards images, displaced
// by the offset). It is rebuilt when the atoms may have moved far enough for an unlisted pair
// to reach r_c (the bound of the previous list form: 2 d + |gamma_dot| t (r_c + 2 d) >= skin,
// d the largest peculiar path length since the build).
//
// Forces. The 64-pair chunks of all segments are dealt round robin to the waves, every lane
// busy. Each pair's force is truncated to 32-bit fixed point (a multiple of 2^-19 force
// units) and added to both atoms with LDS integer atomics (+ to one, - to the other). Integer
// sums do not depend on their order, so every atom's force is independent of the list's
// order, of the skin and grid, of which lane or wave evaluated a pair, and of the rebuild
// schedule; the total force is exactly zero. The virial x_ij F_y,ij of each pair (and the
// extra observables' pair terms) is rounded to a multiple of 2^-19 and summed as an exact
// 64-bit integer, so W_xy has the same independence.
//
// Separations come from 32-bit fixed-point positions X = round(x 2^32 / L) (the box is 2^32
// units wide, so integer differences wrap to the minimum image). Between rebuilds the
// published positions are unwrapped: an atom that crossed the y boundary c times keeps
// X + c offset(t) in x, so each pair keeps the y image it was built with. A pair whose j
// image lies above i is stored as (i, j) with the shift flag, one whose image lies below as
// (j, i) with the flag, so the separation is X_i - X_j, or X_i - (X_j + offset(t)) when
// flagged; every atom publishes both x values.
#include "ttcf_device.h"

namespace ttcf {
namespace {

constexpr int kPairThreads = 512;            // largest workgroup (256 registers per lane)
constexpr int kSmallApt = 4;                 // atoms per thread up to kSmallApt kPairThreads atoms
constexpr int kLargeApt = 8;                 // atoms per thread of larger systems
constexpr int kLargeThreads = 512;           // workgroup limit of the kLargeApt build
constexpr int kJobBytes = 128;               // job slot in front of the per-job LDS
constexpr int kScanPerTrip = 3;              // list build: candidates per lane per trip
constexpr int kPfRed = 16;                   // doubles per thread in one block reduction
constexpr float kForceUnits = 524288.0f;     // 2^19 fixed-point units per force unit
constexpr float kForceStep = 1.0f / 524288.0f;
constexpr float kSumUnits = 524288.0f;       // 2^19 units per virial or energy unit
constexpr double kSumStep = 1.0 / 524288.0;
constexpr double kTwo52 = 4503599627370496.0;    // 2^52

struct PairLds {
    uint4* pos;        // [n] by rank: fixed-point x, y, z, and x + the Lees-Edwards offset
                       // (the x of the image a pair across the y boundary uses); then the two
                       // dummy entries (0, 0, 0, 0) and 2^31 (L/2) in every component
    unsigned long long* fxy;  // [n] by rank: fixed-point force accumulators, x and y packed
                              // in one 64-bit integer y 2^32 + x
    int32_t* fz;              // [n] by rank: the same for z (separate arrays of 8- and 4-byte
                              // stride spread random ranks over more LDS banks)
    uint32_t* fcell;          // [n] by rank: list-grid cell cx | cy << 10 | cz << 20 (each build)
    int32_t* cnt;      // [cells] counts, then placement cursors
    int32_t* start;    // [cells + 1]
    int32_t* rowinfo;  // [3 rows][2]: first x cell offset mod lc_x, cell count
    double* red;       // [kMaxWaves * kPfRed] wave partials of the step's reduction
    double* red2;      // the same for the extra-observable reduction
    int32_t* scan;     // [kMaxWaves]
    float* wmax;       // [kMaxWaves] wave maxima of the path length
    int32_t* flags;    // [kMaxWaves] per wave: its pair list overflowed
    int32_t* wcnt;     // [kMaxWaves] pairs in each wave's segment (at most its capacity)
    double* ktab;      // [16] series coefficients of the isokinetic kick
    SysDev* sys;
    // during a rebuild the fxy area holds the sorted atom ids (u16 [n]) and the rank of
    // every atom id (u16 [n])
};

struct PairPlan {
    size_t pos, fxy, fz, fcell, cnt, start, rowinfo, red, red2, scan, wmax, flags, wcnt, ktab, sys,
        total;
};

__host__ __device__ inline size_t pf_align(size_t v, size_t a) { return (v + a - 1) & ~(a - 1); }

__host__ __device__ inline PairPlan plan_pairs(int n, int cells) {
    PairPlan p;
    size_t off = 0;
    auto take = [&](size_t bytes, size_t al) {
        off = pf_align(off, al);
        const size_t at = off;
        off += bytes;
        return at;
    };
    p.pos = take(16 * (size_t)(n + 2), 16);  // and the two dummy entries of the no-pair word
    p.fxy = take(8 * (size_t)n, 16);
    p.fz = take(4 * (size_t)n, 16);
    p.fcell = take(4 * (size_t)n, 16);
    p.cnt = take(4 * (size_t)cells, 16);
    p.start = take(4 * (size_t)(cells + 1), 16);
    p.rowinfo = take(4 * 8, 16);
    p.red = take(sizeof(double) * kMaxWaves * kPfRed, 16);
    p.red2 = take(sizeof(double) * kMaxWaves * kPfRed, 16);
    p.scan = take(4 * kMaxWaves, 16);
    p.wmax = take(4 * kMaxWaves, 16);
    p.flags = take(4 * kMaxWaves, 16);
    p.wcnt = take(4 * kMaxWaves, 16);
    p.ktab = take(sizeof(double) * 16, 16);
    p.sys = take(sizeof(SysDev), 16);
    p.total = pf_align(off, 128);
    return p;
}

__device__ inline PairLds carve_pairs(char* base, int n, int cells) {
    const PairPlan p = plan_pairs(n, cells);
    PairLds L;
    L.pos = (uint4*)(base + p.pos);
    L.fxy = (unsigned long long*)(base + p.fxy);
    L.fz = (int32_t*)(base + p.fz);
    L.fcell = (uint32_t*)(base + p.fcell);
    L.cnt = (int32_t*)(base + p.cnt);
    L.start = (int32_t*)(base + p.start);
    L.rowinfo = (int32_t*)(base + p.rowinfo);
    L.red = (double*)(base + p.red);
    L.red2 = (double*)(base + p.red2);
    L.scan = (int32_t*)(base + p.scan);
    L.wmax = (float*)(base + p.wmax);
    L.flags = (int32_t*)(base + p.flags);
    L.wcnt = (int32_t*)(base + p.wcnt);
    L.ktab = (double*)(base + p.ktab);
    L.sys = (SysDev*)(base + p.sys);
    return L;
}

// Atoms per thread of a daughter of n atoms (4 up to 2048 atoms, else 8), and the threads that
// own its atoms: a multiple of 64 up to 512.
__host__ __device__ inline int job_apt(int n) {
    return n <= kSmallApt * kPairThreads ? kSmallApt : kLargeApt;
}
__host__ __device__ inline int job_threads(int n) {
    const int per_wave = 64 * job_apt(n);
    return ((n + per_wave - 1) / per_wave) * 64;
}

// round(v 2^32 / L) mod 2^32 for v in [0, L): one fused multiply-add puts the rounded value in
// the low mantissa bits of 2^52 + v scale.
__device__ __forceinline__ uint32_t fixq(double v, double scale) {
    return (uint32_t)__double2loint(__builtin_fma(v, scale, kTwo52));
}

// The fixed-point force of an accumulator: x and y from the packed 64-bit sum y 2^32 + x.
__device__ __forceinline__ int3 unpack_force(unsigned long long xy, int z) {
    const long long v = (long long)xy;
    const int lo = (int)(uint32_t)v;
    return make_int3(lo, (int)((v - (long long)lo) >> 32), z);
}

// Pair words: rank i (bits 0-13), rank j (14-27); kShiftBit: j is taken at its image across
// the y boundary, x_j + the Lees-Edwards offset (a pair whose image lies the other way is
// stored as (j, i)); no pair (lanes past a segment's end): the word of the two dummy entries
// after the n atoms' positions, (n, n + 1), which lie half a box apart along every axis, so that
// the force pass needs no test of its own for them.
constexpr uint32_t kShiftBit = 1u << 28;
__device__ __forceinline__ uint32_t no_pair_word(int n) {
    return (uint32_t)n | ((uint32_t)(n + 1) << 14);
}

// The series coefficients of iso_kick_coeffs_tab, written to the job's LDS by one thread:
// tab[k] = 1/(2k+2)! (k = 0..6), tab[7 + k] = 1/(2k+1)! (k = 0..7).
__device__ __forceinline__ void write_kick_table(double* tab) {
    double f = 1.0;  // running factorial
    for (int m = 1; m <= 15; ++m) {
        f *= (double)m;
        if (m % 2 == 0) tab[m / 2 - 1] = 1.0 / f;
        else tab[7 + m / 2] = 1.0 / f;
    }
}

// iso_kick_coeffs with the series coefficients read from LDS where they are used (as
// literals the compiler hoists them into registers for the whole step loop), and, for
// q tau beyond the series' range, the argument halved until it is in range and the
// doubling formulas sinh 2x = 2 sinh x cosh x, cosh 2x - 1 = 2 sinh^2 x applied back.
// Returns s and sdot of the exact constrained kick over tau.
__device__ __forceinline__ void iso_kick_coeffs_tab(double a, double b, double tau,
                                                    const double* tab, double& s,
                                                    double& sdot) {
    double ch1_b, sh_q;
    const double u = b * tau * tau;
    if (u < 0.04) {
        // Estrin's scheme: the same polynomials in fewer dependent steps
        const double u2 = u * u, u4 = u2 * u2;
        const double c = (tab[0] + tab[1] * u) + u2 * (tab[2] + tab[3] * u) +
                         u4 * ((tab[4] + tab[5] * u) + u2 * tab[6]);
        const double d = (tab[7] + tab[8] * u) + u2 * (tab[9] + tab[10] * u) +
                         u4 * ((tab[11] + tab[12] * u) + u2 * (tab[13] + tab[14] * u));
        ch1_b = tau * tau * c;
        sh_q = tau * d;
    } else {
        int m = 0;
        double v = u;
        while (v >= 0.04) {
            v *= 0.25;
            ++m;
        }
        double c = tab[6];
        for (int k = 5; k >= 0; --k) c = c * v + tab[k];
        double d = tab[14];
        for (int k = 6; k >= 0; --k) d = d * v + tab[7 + k];
        const double th = sqrt(v);
        double c1 = v * c, sh = th * d;  // cosh x - 1, sinh x at x = q tau / 2^m
        for (int i = 0; i < m; ++i) {
            const double nsh = 2.0 * sh * (1.0 + c1);
            c1 = 2.0 * sh * sh;
            sh = nsh;
        }
        const double q = sqrt(b);
        ch1_b = c1 / b;
        sh_q = sh / q;
    }
    s = a * ch1_b + sh_q;
    sdot = a * sh_q + (1.0 + b * ch1_b);
}

// 1/x to about an ulp for x of normal size: the hardware reciprocal and two Newton steps
// (the step's scalars are one dependent chain that every wave waits on, so the short chain
// pays where a correctly rounded division would not).
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// 1/sqrt(x) to about an ulp for positive x of normal size: the hardware estimate and two
// Newton steps y <- y (1 + (1 - x y^2) / 2).
__device__ __forceinline__ double rsq_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double e = __builtin_fma(-(x * y), y, 1.0);
        y = __builtin_fma(0.5 * y, e, y);
    }
    return y;
}

// le_offset without branches (the same value: the remainder of |v| by L_x is exact whichever
// of the neighbouring multiples the estimate q lands on, and the fused multiply-adds
// compute it from q - 1, q or q + 1 exactly); ilx = 1 / L_x.
__device__ __forceinline__ double le_offset_nb(const SysDev& S, double gamma_dot, int64_t k,
                                               double ilx) {
    const double v = gamma_dot * S.box[1] * ((double)k * S.dt);
    const double lx = S.box[0];
    const double av = fabs(v);
    const double q = floor(av * ilx);
    const double r0 = __builtin_fma(-lx, q, av);
    const double rm = __builtin_fma(-lx, q - 1.0, av);
    const double rp = __builtin_fma(-lx, q + 1.0, av);
    const double r = r0 < 0.0 ? rm : (r0 >= lx ? rp : r0);
    const double sr = v < 0.0 ? -r : r;
    return av < lx ? v : sr;
}

// One DPP move of a double from the lane the control selects (every lane has a source).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo =
        (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// The value of lane ^ D (D = 16: lanes of rows 0 and 2; D = 32: lanes 0..31) from gfx950's
// row and half swaps (the second result of a swap of x with itself holds, in those lanes, the
// other row's or half's values).
template <int D>
__device__ __forceinline__ double swap_partner(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
    uint32_t plo, phi;
    if constexpr (D == 16) {
        plo = __builtin_amdgcn_permlane16_swap(lo, lo, false, false)[1];
        phi = __builtin_amdgcn_permlane16_swap(hi, hi, false, false)[1];
    } else {
        plo = __builtin_amdgcn_permlane32_swap(lo, lo, false, false)[1];
        phi = __builtin_amdgcn_permlane32_swap(hi, hi, false, false)[1];
    }
    return __builtin_bit_cast(double, ((uint64_t)phi << 32) | plo);
}

// Sum of red[w kPfRed] over waves w = 0..nw-1 in that order, the loads issued together (a
// wave past nw adds an exact zero).
__device__ __forceinline__ double waves_sum(const double* red, int nw) {
    double v[kPairThreads / 64];
#pragma unroll
    for (int w = 0; w < kPairThreads / 64; ++w) v[w] = w < nw ? red[w * kPfRed] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kPairThreads / 64; ++w) s += v[w];
    return s;
}

// One stage of a transposed reduction: a lane with `upper` set keeps a[H..2H) and hands
// a[0..H) to the lane the control selects, the others keep a[0..H) and hand a[H..2H); the
// kept half adds what arrives. The control must pair every lane with one of the other kind
// holding the same value subsets (an exchange, or a rotation that flips one lane bit).
template <int H, int CTRL>
__device__ __forceinline__ void xstage(double* a, bool upper) {
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const double keep = upper ? a[H + i] : a[i];
        const double send = upper ? a[i] : a[H + i];
        a[i] = keep + dpp_move<CTRL>(send);
    }
}

// The 12-value sum of the step over the first nw waves; every thread receives the totals.
// Inside a wave a transposed reduction: lane bit 0 (exchange with lane ^ 1) splits 12 values
// into 6, bit 1 (lane ^ 2) into 3, bit 2 (rotation by 4 in a row of 16) into 2 of 3 plus a
// zero, bit 3 (rotation by 8) into 1; two cross-row sums (lane ^ 16, lane ^ 32) complete the
// wave totals, 16 slots of which 12 hold values. Then waves 0..nw-1 in sequence, as in
// pf_block_sum below. Fixed order throughout; one barrier, and the same rule for `red`.
__device__ __forceinline__ void pf_block_sum12(double (&v)[12], double* red, int nw) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4, b3 = lane & 8;
    double a[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) a[k] = v[k];
    xstage<6, 0xB1>(a, b0);  // quad_perm [1, 0, 3, 2]
    xstage<3, 0x4E>(a, b1);  // quad_perm [2, 3, 0, 1]
    a[3] = 0.0;
    xstage<2, 0x124>(a, b2);  // row_ror:4
    xstage<1, 0x128>(a, b3);  // row_ror:8
    // cross-row sums without LDS: in rows 0 and 2 the lane of row + 1, then in lanes 0..31
    // the lane 32 above (the swaps' second results; only row 0 is used)
    a[0] += swap_partner<16>(a[0]);
    a[0] += swap_partner<32>(a[0]);
    // value held by this lane: 6 b0 + 3 b1 + (0, 1 or 2 from b2, b3; none if both are set)
    const int idx = 6 * (int)b0 + 3 * (int)b1 + (b2 ? 2 : (int)b3);
    if (lane < 16 && !(b2 && b3) && wave < nw) red[wave * kPfRed + idx] = a[0];
    __syncthreads();
    const double s = lane < 12 ? waves_sum(red + lane, nw) : 0.0;
    const uint64_t u = __builtin_bit_cast(uint64_t, s);
    const int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const uint32_t l = (uint32_t)__builtin_amdgcn_readlane(lo, k);
        const uint32_t h = (uint32_t)__builtin_amdgcn_readlane(hi, k);
        v[k] = __builtin_bit_cast(double, ((uint64_t)h << 32) | l);
    }
}

// Sum K doubles over the first nw waves; every thread receives the totals. Fixed order: a
// scan inside each wave (total in lane 63), then waves 0..nw-1 in sequence, done by lanes
// 0..K-1 of every wave and broadcast from them. One barrier; `red` may be written again
// only after a later barrier.
template <int K>
__device__ __forceinline__ void pf_block_sum(double (&v)[K], double* red, int nw) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_total_dpp(v[k]);
    if (lane == 63 && wave < nw) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[wave * kPfRed + k] = v[k];
    }
    __syncthreads();
    const double s = lane < K ? waves_sum(red + lane, nw) : 0.0;
    const uint64_t u = __builtin_bit_cast(uint64_t, s);
    const int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t l = (uint32_t)__builtin_amdgcn_readlane(lo, k);
        const uint32_t h = (uint32_t)__builtin_amdgcn_readlane(hi, k);
        v[k] = __builtin_bit_cast(double, ((uint64_t)h << 32) | l);
    }
}

// The dynamic LDS of the kernels below: a job slot, then the running job's layout.
extern __shared__ __align__(32) char pf_smem[];

__device__ __forceinline__ PairLds job_lds(int n, int cells) {
    return carve_pairs(pf_smem + kJobBytes, n, cells);
}

typedef __attribute__((address_space(1))) uint32_t gu32;  // pair words in global scratch
typedef __attribute__((address_space(1))) double gf64;    // series in global memory
typedef __attribute__((address_space(3))) uint32_t lu32;  // pair words in LDS

// ---------------------------------------------------------------------------------------
// list build
// ---------------------------------------------------------------------------------------

// Pairs of the 64-rank groups this wave takes (rank s tests the half neighbourhood after it)
// into `seg` (capacity seg_cap; gu32* or lu32*). Returns the number found (wave-uniform; may
// exceed the capacity).
template <int APT, typename P>
__device__ __forceinline__ int pf_gen_pairs(int n, int cells, uint32_t dxq, P seg, int seg_cap,
                                            int tj) {
    const PairLds L = job_lds(n, cells);
    const SysDev& S = *L.sys;
    const int nc0 = S.lc[0], nc1 = S.lc[1], nc2 = S.lc[2];
    const int t = threadIdx.x, lane = t & 63;
    int base = 0;  // wave-uniform: pairs found so far by this wave
    if (t >= tj) return 0;
    // r_l^2 and the y and z fixed-point steps in units of the x step
    const float ux = S.fix_unit[0];
    const float rl2u = S.rl2_f / (ux * ux);
    const float ryx = S.fix_unit[1] / ux, rzx = S.fix_unit[2] / ux;
    // groups of 64 consecutive ranks go to the waves as they ask (a counter in LDS), so that
    // a wave whose rows were short takes more of them; forces do not depend on which wave
    // lists a pair
#pragma unroll 1
    for (;;) {
        int grp = 0;
        if (lane == 0) grp = atomicAdd(&L.scan[0], 1);
        const int r0 = __builtin_amdgcn_readfirstlane(grp) * 64;
        if (r0 >= n) break;  // wave-uniform
        const int s = r0 + lane;
        const bool own = s < n;
        const uint3 qi = *(const uint3*)&L.pos[own ? s : 0];
        const uint32_t cc = L.fcell[own ? s : 0];
        const int cx = (int)(cc & 1023u), cy = (int)((cc >> 10) & 1023u), cz = (int)(cc >> 20);
#pragma unroll 1
        for (int r = 0; r < 5; ++r) {
            // row r: (dz, dy) = (0, 0) own cell past s and the next cell in x; (0, +1);
            // (+1, -1), (+1, 0), (+1, +1) -- the 3-cell x window, or for a row across the y
            // boundary the window of its displaced image
            int lo0, hi0, lo1 = 0, hi1 = 0, ny = 0;
            if (r == 0) {
                const int rowb = nc0 * (cy + nc1 * cz);
                lo0 = s + 1;
                if (cx + 1 < nc0) {
                    hi0 = L.start[rowb + cx + 2];
                } else {
                    hi0 = L.start[rowb + cx + 1];
                    lo1 = L.start[rowb];
                    hi1 = L.start[rowb + 1];
                }
            } else {
                const int dz = r == 1 ? 0 : 1;
                const int dy = r == 1 ? 1 : r - 3;
                int zz = cz + dz;
                if (zz >= nc2) zz -= nc2;
                int yy = cy + dy;
                if (yy < 0) {
                    yy += nc1;
                    ny = -1;
                } else if (yy >= nc1) {
                    yy -= nc1;
                    ny = 1;
                }
                int x0, nq;
                if (ny == 0) {
                    x0 = cx == 0 ? nc0 - 1 : cx - 1;
                    nq = 3;
                } else {
                    const int row = ny > 0 ? 2 : 0;
                    x0 = cx + L.rowinfo[2 * row];
                    if (x0 >= nc0) x0 -= nc0;
                    nq = L.rowinfo[2 * row + 1];
                }
                // cells x0 .. x0 + nq - 1 (mod lc_x): one or two rank ranges (the start of
                // cell lc_x of a row is the end of the row)
                const int xe = x0 + nq;
                const int rowb = nc0 * (yy + nc1 * zz);
                lo0 = L.start[rowb + x0];
                if (xe <= nc0) {
                    hi0 = L.start[rowb + xe];
                } else {
                    hi0 = L.start[rowb + nc0];
                    lo1 = L.start[rowb];
                    hi1 = L.start[rowb + xe - nc0];
                }
            }
            const uint32_t rsh = ny > 0 ? dxq : (ny < 0 ? 0u - dxq : 0u);
            const int len0 = own ? max(hi0 - lo0, 0) : 0;
            const int len = len0 + (own ? max(hi1 - lo1, 0) : 0);
            // the pair word: (s, k), or (k, s) for an image below, flagged when shifted
            const int shs = ny < 0 ? 14 : 0;
            const uint32_t wfix = ((uint32_t)s << shs) | (ny != 0 ? kShiftBit : 0u);
            // candidate vv of the row: rank lo0 + vv in the first range, lo1 + (vv - len0)
            // in the second
            const int off1 = lo1 - len0;
            // kScanPerTrip candidates per lane per trip, their loads issued together; trips
            // until the wave's longest row is done
            for (int v = 0; __builtin_amdgcn_ballot_w64(v < len) != 0; v += kScanPerTrip) {
                int k[kScanPerTrip];
                uint3 q[kScanPerTrip];
#pragma unroll
                for (int u = 0; u < kScanPerTrip; ++u) {
                    const int vv = v + u;
                    const int kk = vv + (vv < len0 ? lo0 : off1);
                    k[u] = vv < len ? kk : 0;  // (len is 0 past n)
                }
#pragma unroll
                for (int u = 0; u < kScanPerTrip; ++u) q[u] = *(const uint3*)&L.pos[k[u]];
#pragma unroll
                for (int u = 0; u < kScanPerTrip; ++u) {
                    // the squared distance in units of the x fixed-point step
                    const float ddx = (float)(int32_t)(qi.x - q[u].x - rsh);
                    const float ddy = (float)(int32_t)(qi.y - q[u].y) * ryx;
                    const float ddz = (float)(int32_t)(qi.z - q[u].z) * rzx;
                    // one compare against a limit that no square reaches past the row's end,
                    // so that the ballot is that compare's mask
                    const float lim = v + u < len ? rl2u : -1.f;
                    const bool hit = ddx * ddx + ddy * ddy + ddz * ddz < lim;
                    const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
                    const int below = (int)__builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    // past the capacity every hit lands in the last slot (the count reports
                    // the overflow)
                    const int at = min(base + below, seg_cap - 1);
                    if (hit) seg[at] = wfix | ((uint32_t)k[u] << (14 - shs));
                    base += (int)__builtin_popcountll(m);
                }
            }
        }
    }
    return base;
}

// Rebuild at Lees-Edwards offset dxle (dxq in fixed point) from the owners' FP64 positions:
// canonical (cell, id) ranks on the list grid, positions published (crossing counts reset),
// this wave's pairs in `seg`. Returns the wave's pair count (may exceed seg_cap); *overflow
// receives whether any wave's list overflowed (the same in every thread). cell: the list-grid
// cell of each owned atom (-1 past n). Every thread of the workgroup calls it.
template <int APT, typename P>
__device__ __forceinline__ int pf_rebuild(const SysDev& S, double dxle, uint32_t dxq,
                                          const double (&x)[APT], const double (&y)[APT],
                                          const double (&z)[APT], int (&rank)[APT],
                                          int (&cr)[APT], const PairLds& L, P seg, int seg_cap,
                                          int tj, int (&cell)[APT], bool* overflow) {
    const int T = blockDim.x, t = threadIdx.x, n = S.n;
    const int nc0 = S.lc[0], nc1 = S.lc[1], nc2 = S.lc[2];
    const int C = nc0 * nc1 * nc2;
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * tj;
        cell[j] = -1;
        if (t < tj && a < n) {
            const int cx = cell_coord(x[j], S.l_inv_w[0], nc0);
            const int cy = cell_coord(y[j], S.l_inv_w[1], nc1);
            const int cz = cell_coord(z[j], S.l_inv_w[2], nc2);
            cell[j] = cx + nc0 * (cy + nc1 * cz);
            atomicAdd(&L.cnt[cell[j]], 1);
        }
    }
    if (t == 0) {
        // x windows of the rows across the y boundary: every cell whose image (displaced by
        // -+dxle) overlaps [cx w - r_l, (cx + 1) w + r_l], plus a margin for the FP32 test
        const double reach = S.rc + S.skin;
        const double wx = S.lw[0];
        const double margin = 1e-6 * reach;
        for (int row = 0; row < 3; row += 2) {
            double sh = (row == 0 ? -1.0 : 1.0) * dxle;
            sh -= S.box[0] * rint(sh / S.box[0]);
            const int off = (int)floor((-reach - margin - sh) / wx);
            const int hi = (int)floor((wx + reach + margin - sh) / wx);
            int nq = hi - off + 1;
            if (nq > nc0) nq = nc0;
            L.rowinfo[2 * row] = ((off % nc0) + nc0) % nc0;
            L.rowinfo[2 * row + 1] = nq;
        }
    }
    __syncthreads();
    scan_cells(L.cnt, L.start, C, L.scan);
    if (t == 0) L.start[C] = n;
    __syncthreads();
    uint16_t* sid = (uint16_t*)L.fxy;
    uint16_t* rk = sid + n;
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        if (cell[j] >= 0) {
            const int idx = atomicAdd(&L.cnt[cell[j]], 1);
            sid[idx] = (uint16_t)(t + j * tj);
        }
    }
    __syncthreads();
    // canonical order inside each cell (ascending id), the rank of every atom, cursors reset
    for (int c = t; c < C; c += T) {
        const int lo = L.start[c], hi = L.start[c + 1];
        for (int i = lo + 1; i < hi; ++i) {
            const uint16_t v = sid[i];
            int k = i - 1;
            while (k >= lo && sid[k] > v) {
                sid[k + 1] = sid[k];
                --k;
            }
            sid[k + 1] = v;
        }
        for (int i = lo; i < hi; ++i) rk[sid[i]] = (uint16_t)i;
        L.cnt[c] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * tj;
        cr[j] = 0;
        rank[j] = 0;
        if (cell[j] >= 0) {
            rank[j] = rk[a];
            const int c = cell[j];
            const uint32_t cx = (uint32_t)(c % nc0), cy = (uint32_t)((c / nc0) % nc1),
                           cz = (uint32_t)(c / (nc0 * nc1));
            L.pos[rank[j]] = make_uint4(fixq(x[j], S.fix_scale[0]), fixq(y[j], S.fix_scale[1]),
                                        fixq(z[j], S.fix_scale[2]), cx | (cy << 10) | (cz << 20));
        }
    }
    __syncthreads();
    // the scratch is free again: clear the force accumulators for the next force pass and
    // move each rank's cell there; the shifted x in its place
    for (int i = t; i < n; i += T) {
        const uint4 q = L.pos[i];
        L.fxy[i] = 0ull;
        L.fz[i] = 0;
        L.fcell[i] = q.w;
        L.pos[i].w = q.x + dxq;
    }
    if (t == 0) L.scan[0] = 0;  // the list build's group counter (the scan is done with it)
    __syncthreads();
    const int count = pf_gen_pairs<APT>(n, C, dxq, seg, seg_cap, tj);
    const int wave = t >> 6, nwb = T >> 6;
    if ((t & 63) == 0) {
        L.flags[wave] = count > seg_cap ? 1 : 0;
        L.wcnt[wave] = min(count, seg_cap);
    }
    __syncthreads();
    int any = 0;
#pragma unroll
    for (int w = 0; w < kPairThreads / 64; ++w) any |= w < nwb ? L.flags[w] : 0;
    *overflow = any != 0;
    return count;
}

// ---------------------------------------------------------------------------------------
// force pass
// ---------------------------------------------------------------------------------------

// Lane shares of the pair sums of one force pass, in units of 2^-19 (exact integers): W_xy,
// and (OBS) W_xx, W_yy, W_zz and U; close: a pair came inside the guard radius.
struct PfSums {
    double w, xx, yy, zz, u;
    int close;
};

// Forces of the pairs of every wave segment into the fixed-point accumulators. The segments'
// 64-pair chunks, taken in order (segment 0 first), go round robin to the waves of the
// workgroup: wave w forces chunks w, w + W, w + 2W, ... of W waves, so every wave gets the
// same share whatever its own list held. Called by every thread; the pair counts come from
// the last build (L.wcnt). Out of line, so that the step loop's registers and these do not
// add up.
template <bool OBS, typename P>
__device__ __forceinline__ PfSums pf_forces(int n, int cells, uint32_t dxq, P pair_base,
                                            int seg_cap) {
    const PairLds L = job_lds(n, cells);
    const SysDev& S = *L.sys;
    const int lane = threadIdx.x & 63, nwb = blockDim.x >> 6;
    const float rc2 = S.rc2_f, rg2 = S.rg2_f;
    const float ca = (float)S.c_attr;
    const float ushift = (float)S.u_shift;
    const float ux = S.fix_unit[0], uy = S.fix_unit[1], uz = S.fix_unit[2];
    // force factor in force units: 2^19 (48 s3 - 24 c) s3 / r^2
    const float f48 = 48.f * kForceUnits, f24 = 24.f * kForceUnits * ca;
    // lane shares of the sums in 2^-19 units (exact 64-bit integers)
    long long aw = 0, axx = 0, ayy = 0, azz = 0, au = 0;
    bool close = false;
    // lane s < W: pairs of segment s and the chunks before it; lanes from W on: the total
    int seg_pairs = 0, seg_first = 0;
#pragma unroll
    for (int s = 0; s < kPairThreads / 64; ++s) {
        const int c = s < nwb ? L.wcnt[s] : 0;
        if (s == lane) seg_pairs = c;
        if (s < lane) seg_first += (c + 63) >> 6;
    }
    const int chunks = __builtin_amdgcn_readlane(seg_first, kPairThreads / 64);
    const uint32_t nopair = no_pair_word(n);
    // the word of chunk g in this lane: segment s is the last one starting at or before g
    auto word_of = [&](int g) -> uint32_t {
        if (g >= chunks) return nopair;
        const int s = __popcll(__ballot(seg_first <= g)) - 1;
        const int first = __builtin_amdgcn_readlane(seg_first, s);
        const int cnt = __builtin_amdgcn_readlane(seg_pairs, s);
        const int at = (g - first) * 64 + lane;
        return at < cnt ? pair_base[(size_t)s * seg_cap + at] : nopair;
    };
    // software pipeline: the pair words two chunks ahead and the positions one chunk ahead
    // are loaded before this chunk's atomics (LDS operations complete in order, so loads
    // issued after the atomics would wait for them)
    const int g0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t w_next = word_of(g0);
    uint32_t w_after = word_of(g0 + nwb);
    uint3 pi_next = *(const uint3*)&L.pos[w_next & 0x3FFFu];
    uint4 pj_next = L.pos[(w_next >> 14) & 0x3FFFu];
    for (int g = g0; g < chunks; g += nwb) {
        const uint32_t word = w_next;
        const uint3 qi = pi_next;
        const uint4 qj = pj_next;
        w_next = w_after;
        w_after = word_of(g + 2 * nwb);
        pi_next = *(const uint3*)&L.pos[w_next & 0x3FFFu];
        pj_next = L.pos[(w_next >> 14) & 0x3FFFu];
        const int si = (int)(word & 0x3FFFu), sj = (int)((word >> 14) & 0x3FFFu);
        const uint32_t xj = (word & kShiftBit) ? qj.w : qj.x;
        const float dx = (float)(int32_t)(qi.x - xj) * ux;
        const float dy = (float)(int32_t)(qi.y - qj.y) * uy;
        const float dz = (float)(int32_t)(qi.z - qj.z) * uz;
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < rc2) {
            const float inv = __builtin_amdgcn_rcpf(r2);  // within 1 ulp
            const float s3 = inv * inv * inv;
            const float fs = s3 * (f48 * s3 - f24) * inv;
            const float gx = fs * dx, gy = fs * dy, gz = fs * dz;  // in force units
            close |= r2 < rg2;
            // truncated to a whole unit: odd in the separation, so a pair gives the same
            // increments whichever atom it lists first; atom j gets exactly the negation
            // (a plain conversion: v_cvt_i32_f32 rounds toward zero)
            const int qx = (int)gx, qy = (int)gy, qz = (int)gz;
            // x and y share one 64-bit integer, V = qy 2^32 + qx: sums of such values are
            // exact, and each component stays within +-2^31, so both decode exactly
            const unsigned long long v = (unsigned long long)(((long long)qy << 32) + (long long)qx);
            // (LDS atomics without return; j's through the subtracting form, so that no
            // negated copies are needed)
            __hip_atomic_fetch_add(&L.fxy[si], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(&L.fz[si], qz, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_sub(&L.fxy[sj], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_sub(&L.fz[sj], qz, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            // pair sums: the FP32 products rounded to the nearest 2^-19 unit, ties to even
            // (odd, so that mirrored configurations give exactly opposite sums)
            aw += __float2int_rn(dx * gy);
            if (OBS) {
                axx += __float2int_rn(dx * gx);
                ayy += __float2int_rn(dy * gy);
                azz += __float2int_rn(dz * gz);
                au += __float2int_rn((4.f * s3 * (s3 - ca) + ushift) * kSumUnits);
            }
        }
    }
    PfSums o;
    o.w = (double)aw;
    o.xx = (double)axx;
    o.yy = (double)ayy;
    o.zz = (double)azz;
    o.u = (double)au;
    o.close = close ? 1 : 0;
    return o;
}

// ---------------------------------------------------------------------------------------
// extra observables
// ---------------------------------------------------------------------------------------

// The extra observables at one time point: kinetic parts from the owned atoms' momenta p,
// pair parts (exact integers in units of 2^-19) of the force pass, reduced over the
// workgroup (kinetic and pair sums in separate slots) and written by thread 0 to row `row`.
template <int APT>
__device__ __forceinline__ void pf_record_obs(const SysDev& S, const double (&y)[APT],
                                              const double (&px)[APT], const double (&py)[APT],
                                              const double (&pz)[APT], const PfSums& ps,
                                              gf64* xs, int row, const PairLds& L, int nw) {
    double o[kObsCols + 4];
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
    o[kObsCols] = ps.xx;
    o[kObsCols + 1] = ps.yy;
    o[kObsCols + 2] = ps.zz;
    o[kObsCols + 3] = ps.u;
    pf_block_sum<kObsCols + 4>(o, L.red2, nw);
    if (threadIdx.x == 0) {
        const double wxx = o[kObsCols] * kSumStep, wyy = o[kObsCols + 1] * kSumStep,
                     wzz = o[kObsCols + 2] * kSumStep, u = o[kObsCols + 3] * kSumStep;
        gf64* out = xs + (size_t)row * kObsCols;
        const double iv = 1.0 / S.volume;
        out[0] = (o[0] + (wxx - wyy)) * iv;
        out[1] = (o[1] + (wyy - wzz)) * iv;
        out[2] = (o[2] + u) / (double)S.n;
#pragma unroll
        for (int q = 0; q < kObsSlabs; ++q) out[3 + q] = o[3 + q] * ((double)kObsSlabs * iv);
    }
}

// ---------------------------------------------------------------------------------------
// one daughter
// ---------------------------------------------------------------------------------------

// Publish the owned atoms' fixed-point positions (unwrapped by their crossing counts) and
// return the workgroup maximum of their path lengths since the last build (one barrier).
template <int APT>
__device__ __forceinline__ float pf_publish(const SysDev& S, uint32_t dxq, const double (&x)[APT],
                                            const double (&y)[APT], const double (&z)[APT],
                                            const int (&rank)[APT], const int (&cr)[APT],
                                            const float (&path)[APT], const PairLds& L, int tj,
                                            int nw) {
    const int t = threadIdx.x, n = S.n;
    float pm = 0.f;
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * tj;
        if (t < tj && a < n) {
            // x, y, z only: w keeps the cell of the last build
            const uint32_t qx = fixq(x[j], S.fix_scale[0]) + (uint32_t)cr[j] * dxq;
            L.pos[rank[j]] =
                make_uint4(qx, fixq(y[j], S.fix_scale[1]), fixq(z[j], S.fix_scale[2]), qx + dxq);
            pm = fmaxf(pm, path[j]);
        }
    }
    pm = wave_max_dpp(pm);
    if ((t & 63) == 63) L.wmax[t >> 6] = pm;
    __syncthreads();
    float v[kPairThreads / 64];
#pragma unroll
    for (int w = 0; w < kPairThreads / 64; ++w) v[w] = w < nw ? L.wmax[w] : 0.f;
    float m = 0.f;
#pragma unroll
    for (int w = 0; w < kPairThreads / 64; ++w) m = fmaxf(m, v[w]);
    return m;
}

// Daughter step, h = dt, tau = h/2, tg = tau gamma_dot. Both thermostats split the step as
//   [first half] D(h) [forces] [second half],
// isokinetic: first half S(tau) K(tau), second half K(tau) S(tau) and the rescale to K0 (the
// exact constrained flows, closed forms from the moments of (p, F)); Nose-Hoover (Eq.
// system1 as printed): first half Z(tau) T(tau) S(tau) K(tau), second half K(tau) S(tau)
// T(tau) Z(tau). Either half maps p to a p + b F + c p_y x_hat + d F_y x_hat (y, z: a p + b F)
// with scalars from the moments reduced once per step, so the second half of one step and the
// first half of the next are applied together as one update of the momenta; the end-of-step
// moments that B(t) and the next first half need follow in closed form.
// COL: the build that also runs colour-field daughters (either thermostat): atom a carries
// the colour charge +1 (even a) or -1 (odd a), the field adds charge * F_e to its x force in
// FP64, there is no shear, and the series records V J_x = sum_a charge p_x,a.
template <int APT, bool NH, bool OBS, bool COL, typename P>
__device__ void run_daughter_pairs(DaughterDesc* dsc, int steps_cap, const PairLds& L,
                                   P pair_base) {
    const int t = threadIdx.x;
    if (t == 0) {
        *L.sys = dsc->sys;
        write_kick_table(L.ktab);
    }
    __syncthreads();
    const SysDev& S = *L.sys;
    const int n = S.n;
    const int cells = S.lc[0] * S.lc[1] * S.lc[2];
    const int tj = job_threads(n);
    const int nw = blockDim.x >> 6;  // waves of the workgroup (the owners and any others)
    const int wave = t >> 6;
    double* st = dsc->state;
    const bool col = COL && dsc->field == kFieldColour;  // uniform per job
    const double gd = col ? 0.0 : dsc->gamma_dot;
    int64_t k = dsc->k;
    int done = dsc->done;
    const int n_steps = dsc->n_steps;
    double k0 = dsc->k0;
    int health = dsc->health;
    double zt = dsc->zeta;
    const double nh_iq = NH ? 1.0 / dsc->nh_q : 0.0, nh_tgt = dsc->nh_target;
    int todo = min(steps_cap, n_steps - done);
    if (health != 0) todo = 0;
    if (todo <= 0 && done > 0) return;
    // this wave's pair segment
    const int seg_cap = dsc->kmax * 64 * APT;
    const P seg = pair_base + (size_t)wave * seg_cap;

    double x[APT], y[APT], z[APT], px[APT], py[APT], pz[APT];
    float fx[APT], fy[APT], fz[APT];  // FP32 forces; every use promotes them to FP64
    int rank[APT], cr[APT], cell[APT];
    float path[APT];
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * tj;
        const bool v = t < tj && a < n;
        x[j] = v ? st[a] : 0.0;
        y[j] = v ? st[n + a] : 0.0;
        z[j] = v ? st[2 * n + a] : 0.0;
        px[j] = v ? st[3 * n + a] : 0.0;
        py[j] = v ? st[4 * n + a] : 0.0;
        pz[j] = v ? st[5 * n + a] : 0.0;
        path[j] = 0.f;
        fx[j] = fy[j] = fz[j] = 0.f;
    }
    // colour charges (zero past n and for shear daughters) and the field's x force in FP64
    double ce[APT];
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * tj;
        const double cq = (COL && col && t < tj && a < n) ? ((a & 1) ? -1.0 : 1.0) : 0.0;
        ce[j] = COL ? cq * dsc->fe : 0.0;
    }
    auto charge = [&](int j) -> double { return ((t + j * tj) & 1) ? -1.0 : 1.0; };
    auto fxd = [&](int j) -> double {
        if constexpr (COL)
            return (double)fx[j] + ce[j];
        else
            return (double)fx[j];
    };
    double dxle = le_offset(S, gd, k);
    uint32_t dxq = fix32(dxle, S.fix_scale[0]);
    PfSums ps{0.0, 0.0, 0.0, 0.0, 0.0, 0};
    bool ovf = false;
    // forces of the start state
    pf_rebuild<APT>(S, dxle, dxq, x, y, z, rank, cr, L, seg, seg_cap, tj, cell, &ovf);
    if (ovf) health |= kHealthListOverflow;
    ps = pf_forces<OBS>(n, cells, dxq, pair_base, seg_cap);
    __syncthreads();
    auto readback = [&]() {
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            const int a = t + j * tj;
            if (t < tj && a < n) {
                const int3 q = unpack_force(L.fxy[rank[j]], L.fz[rank[j]]);
                fx[j] = (float)q.x * kForceStep;
                fy[j] = (float)q.y * kForceStep;
                fz[j] = (float)q.z * kForceStep;
                L.fxy[rank[j]] = 0ull;
                L.fz[rank[j]] = 0;
            }
        }
    };
    readback();
    // the series as global pointers held for the whole call: a generic store would make the
    // next barrier wait for it, and a store through the descriptor's pointer would make the
    // compiler reload that pointer every step
    gf64* const xs = OBS ? (gf64*)dsc->xseries : nullptr;
    gf64* const series = (gf64*)dsc->series;

    double m0[8] = {0, 0, 0, 0, 0, 0, ps.w, (double)ps.close};
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        // one multiply-add with a selected factor, so that shear daughters get the same
        // contractions in every build
        const double w1 = (COL && col) ? charge(j) : py[j];
        m0[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j];
        m0[1] += w1 * px[j];
        m0[2] += py[j] * py[j];
        m0[3] += fxd(j) * px[j] + (double)fy[j] * py[j] + (double)fz[j] * pz[j];
        m0[4] += fxd(j) * py[j];
        m0[5] += fxd(j) * fxd(j) + (double)fy[j] * (double)fy[j] +
                 (double)fz[j] * (double)fz[j];
    }
    pf_block_sum<8>(m0, L.red, nw);
    if (m0[7] != 0.0) health |= kHealthForceRange;
    if (done == 0) {
        if (k0 <= 0.0) k0 = 0.5 * m0[0];
        if (t == 0) dsc->k0 = k0;
        if (t == 0) series[0] = (COL && col) ? m0[1] : m0[1] + m0[6] * kSumStep;
        if (OBS && xs) pf_record_obs<APT>(S, y, px, py, pz, ps, xs, 0, L, nw);
    }
    if (health != 0) todo = 0;
    const double sqrt2k0 = sqrt(2.0 * k0);
    const double h = S.dt, tau = 0.5 * S.dt, tg = tau * gd;
    const float hpath = (float)h * (1.f + 0x1p-20f);
    const float reach = (float)S.rc;
    const float skin = (float)S.skin;
    const float agd = (float)fabs(gd);
    int since = 0;
    // First half of a step from the end-of-step moments pp, pxpy, pypy, fp, fxpy, ff (F the
    // current forces): p -> e p + g p_y x_hat + hh F.
    double pp = m0[0], pxpy = m0[1], pypy = m0[2], fp = m0[3], fxpy = m0[4], ff = m0[5];
    auto first_half = [&](double& e, double& g, double& hh) {
        if (NH) {
            zt += tau * (pp - nh_tgt) * nh_iq;
            const double c1 = exp(-zt * tau);
            e = c1;
            g = -tg * c1;
            hh = tau;
        } else {
            const double ppt = pp - 2.0 * tg * pxpy + tg * tg * pypy;
            const double g1 = pp * rsq_nr(pp * ppt);  // sqrt(pp / ppt)
            const double ipp = rcp_nr(pp);
            const double fp1 = g1 * (fp - tg * fxpy);
            double s1, sd1;
            iso_kick_coeffs_tab(fp1 * ipp, ff * ipp, tau, L.ktab, s1, sd1);
            const double isd1 = rcp_nr(sd1);
            e = g1 * isd1;
            g = -tg * e;
            hh = s1 * isd1;
        }
    };
    if (todo > 0) {
        double e, g, hh;
        first_half(e, g, hh);
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            const double qx = e * px[j] + g * py[j] + hh * fxd(j);
            py[j] = e * py[j] + hh * (double)fy[j];
            pz[j] = e * pz[j] + hh * (double)fz[j];
            px[j] = qx;
        }
    }

    // the offset of the next step, computed a step ahead where its dependent chain overlaps
    // the kick scalars' chain
    const double ilx = 1.0 / S.box[0];
    double dxle_n = le_offset_nb(S, gd, k + 1, ilx);
    uint32_t dxq_n = fix32(dxle_n, S.fix_scale[0]);
    for (int step = 0; step < todo; ++step) {
        // ---- streaming D(h), new strain, sliding-brick wrap (crossings counted), path length
        k += 1;
        dxle = dxle_n;
        dxq = dxq_n;
        const double lx = S.box[0], ly = S.box[1], lz = S.box[2];
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            const double vx = px[j] + tg * py[j];
            // the hardware square root (about an ulp) with the step scaled up by 2^-20, so
            // that the path length stays an upper bound
            path[j] += hpath * __builtin_amdgcn_sqrtf((float)(vx * vx + py[j] * py[j] + pz[j] * pz[j]));
            x[j] += h * px[j] + h * gd * (y[j] + tau * py[j]);
            y[j] += h * py[j];
            z[j] += h * pz[j];
        }
        // sliding-brick wrap of the atoms of slot j, only in a wave where one of them left the
        // box (a few percent of the steps, and one slot at a time, so that the waves reach the
        // next barrier together): a step moves an atom far less than a box edge, so each axis
        // needs at most one image shift (the same operations as wrap_le in that case); a y
        // crossing shifts x by -+ the offset
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            const bool out = (x[j] < 0.0) | (x[j] >= lx) | (y[j] < 0.0) | (y[j] >= ly) |
                             (z[j] < 0.0) | (z[j] >= lz);
            if (__builtin_amdgcn_ballot_w64(out) != 0) {
                const bool up = y[j] >= ly, dn = y[j] < 0.0;
                cr[j] += up ? 1 : (dn ? -1 : 0);
                y[j] += up ? -ly : (dn ? ly : 0.0);
                y[j] = y[j] >= ly ? 0.0 : y[j];  // a tiny negative y plus L rounded up to L
                x[j] += up ? -dxle : (dn ? dxle : 0.0);
                x[j] += x[j] >= lx ? -lx : (x[j] < 0.0 ? lx : 0.0);
                x[j] = x[j] >= lx ? 0.0 : x[j];
                z[j] += z[j] >= lz ? -lz : (z[j] < 0.0 ? lz : 0.0);
                z[j] = z[j] >= lz ? 0.0 : z[j];
            }
        }
        const float dm = pf_publish<APT>(S, dxq, x, y, z, rank, cr, path, L, tj, nw);
        ++since;
        const float tsince = (float)(since * h);
        if (2.f * dm + agd * tsince * (reach + 2.f * dm) >= skin) {
            pf_rebuild<APT>(S, dxle, dxq, x, y, z, rank, cr, L, seg, seg_cap, tj, cell, &ovf);
            if (ovf) {  // the same in every thread
                health |= kHealthListOverflow;
                break;
            }
#pragma unroll
            for (int j = 0; j < APT; ++j) path[j] = 0.f;
            since = 0;
        }
        ps = pf_forces<OBS>(n, cells, dxq, pair_base, seg_cap);
        __syncthreads();
        readback();
        // ---- moments of (p, F): pp, pxpy, pypy, fp, fxpy, fypx, fxfy, fypy, fyfy, ff, W,
        // range flag; a non-finite position makes pp non-finite (0 times it)
        double m[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, ps.w, (double)ps.close};
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            const double w1 = (COL && col) ? charge(j) : py[j];  // as for m0
            m[0] += px[j] * px[j] + py[j] * py[j] + pz[j] * pz[j] + 0.0 * (x[j] + y[j] + z[j]);
            m[1] += w1 * px[j];
            m[2] += py[j] * py[j];
            m[3] += fxd(j) * px[j] + (double)fy[j] * py[j] + (double)fz[j] * pz[j];
            m[4] += w1 * fxd(j);
            m[5] += (double)fy[j] * px[j];
            m[6] += fxd(j) * (double)fy[j];
            m[7] += (double)fy[j] * py[j];
            m[8] += (double)fy[j] * (double)fy[j];
            m[9] += fxd(j) * fxd(j) + (double)fy[j] * (double)fy[j] +
                    (double)fz[j] * (double)fz[j];
        }
        pf_block_sum12(m, L.red, nw);
        // ---- second half: p_end = A p + B F + (C p_y + D F_y) x_hat, end-of-step moments
        double A, B, C, D, vpxy;
        bool drift = false;
        if (NH) {
            const double c2 = exp(-zt * tau);
            A = c2;
            B = c2 * tau;
            C = -c2 * tg;
            D = C * tau;
            pp = A * A * m[0] + 2.0 * A * B * m[3] + B * B * m[9] + C * C * m[2] +
                 2.0 * C * D * m[7] + D * D * m[8] + 2.0 * A * C * m[1] + 2.0 * A * D * m[5] +
                 2.0 * B * C * m[4] + 2.0 * B * D * m[6];
            pxpy = A * A * m[1] + A * B * (m[5] + m[4]) + B * B * m[6] + A * C * m[2] +
                   (B * C + A * D) * m[7] + B * D * m[8];
            zt += tau * (pp - nh_tgt) * nh_iq;
        } else {
            double s2, sd2;
            const double im0 = rcp_nr(m[0]);
            iso_kick_coeffs_tab(m[3] * im0, m[9] * im0, tau, L.ktab, s2, sd2);
            const double isd2 = rcp_nr(sd2);
            const double pp3 = (m[0] + 2.0 * s2 * m[3] + s2 * s2 * m[9]) * isd2 * isd2;
            const double pxpy3 = (m[1] + s2 * (m[4] + m[5]) + s2 * s2 * m[6]) * isd2 * isd2;
            const double pypy3 = (m[2] + 2.0 * s2 * m[7] + s2 * s2 * m[8]) * isd2 * isd2;
            const double fp3 = (m[3] + s2 * m[9]) * isd2;
            const double fxpy3 = (m[4] + s2 * m[6]) * isd2;
            const double ppt2 = pp3 - 2.0 * tg * pxpy3 + tg * tg * pypy3;
            const double c = sqrt2k0 * rsq_nr(ppt2);  // sqrt(2 k0 / ppt2)
            A = c * isd2;
            B = A * s2;
            C = -tg * A;
            D = -tg * B;
            pp = c * c * ppt2;
            pxpy = c * c * (pxpy3 - tg * pypy3);
            pypy = c * c * pypy3;
            fp = c * (fp3 - tg * fxpy3);
            fxpy = c * fxpy3;
            ff = m[9];
            drift = fabs(pp3 * im0 - 1.0) > 1e-10;
        }
        // colour: V J_x of the final momenta from the charge moments (no shear: C = D = 0)
        vpxy = (COL && col) ? A * m[1] + B * m[4] : pxpy + m[10] * kSumStep;
        done += 1;
        if (t == 0) series[done] = vpxy;
        if (m[11] != 0.0) health |= kHealthForceRange;
        if (!isfinite(vpxy) || !isfinite(pp) || !isfinite(zt)) health |= kHealthNonFinite;
        if (drift) health |= kHealthDrift;
        const bool last = step + 1 == todo || health != 0;
        if (OBS && xs) {
            double qx[APT], qy[APT], qz[APT];
#pragma unroll
            for (int j = 0; j < APT; ++j) {
                qx[j] = A * px[j] + B * fxd(j) + C * py[j] + D * (double)fy[j];
                qy[j] = A * py[j] + B * (double)fy[j];
                qz[j] = A * pz[j] + B * (double)fz[j];
            }
            pf_record_obs<APT>(S, y, qx, qy, qz, ps, xs, done, L, nw);
        }
        if (last) {
#pragma unroll
            for (int j = 0; j < APT; ++j) {
                const double qx = A * px[j] + B * fxd(j) + C * py[j] + D * (double)fy[j];
                py[j] = A * py[j] + B * (double)fy[j];
                pz[j] = A * pz[j] + B * (double)fz[j];
                px[j] = qx;
            }
            break;
        }
        // ---- the next step's first half, applied together with this second half
        dxle_n = le_offset_nb(S, gd, k + 1, ilx);
        dxq_n = fix32(dxle_n, S.fix_scale[0]);
        double e, g, hh;
        first_half(e, g, hh);
        const double K1 = e * A, K2 = e * C + g * A, K3 = e * B + hh, K4 = e * D + g * B;
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            const double qx = K1 * px[j] + K2 * py[j] + K3 * fxd(j) + K4 * (double)fy[j];
            py[j] = K1 * py[j] + K3 * (double)fy[j];
            pz[j] = K1 * pz[j] + K3 * (double)fz[j];
            px[j] = qx;
        }
    }
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * tj;
        if (t < tj && a < n) {
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
        dsc->health = health;
        dsc->zeta = zt;
    }
    // the accumulators must be zero for the next job (a call that stopped after a force pass
    // without reading it back would leave forces in them)
    for (int i = t; i < n; i += blockDim.x) {
        L.fxy[i] = 0ull;
        L.fz[i] = 0;
    }
    __syncthreads();
}

// PL: the pair words of every job live in LDS after its layout (b.lds_bytes covers them),
// else in the workgroup's slice of b.pairs.
template <int APT, bool NH, bool OBS, bool COL, bool PL>
__global__ __launch_bounds__(APT == kLargeApt ? kLargeThreads : kPairThreads) void k_daughters_pairs(
    BatchLaunch b) {
    int32_t* job = (int32_t*)pf_smem;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) *job = atomicAdd(b.queue, 1);
        __syncthreads();
        const int j = __builtin_amdgcn_readfirstlane(*job);
        if (j >= b.n_jobs) break;
        DaughterDesc* d = &b.descs[b.order[j]];
        const int n = d->sys.n;
        const int cells = d->sys.lc[0] * d->sys.lc[1] * d->sys.lc[2];
        const PairLds L = job_lds(n, cells);
        for (int c = threadIdx.x; c < cells; c += blockDim.x) L.cnt[c] = 0;
        if (threadIdx.x == 0) {
            L.pos[n] = make_uint4(0u, 0u, 0u, 0u);
            L.pos[n + 1] = make_uint4(1u << 31, 1u << 31, 1u << 31, 1u << 31);
        }
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            L.fxy[i] = 0ull;
            L.fz[i] = 0;
        }
        // run_daughter_pairs synchronises before its first use of the counts
        if constexpr (PL)
            run_daughter_pairs<APT, NH, OBS, COL>(
                d, b.max_steps, L, (lu32*)(pf_smem + kJobBytes + plan_pairs(n, cells).total));
        else
            run_daughter_pairs<APT, NH, OBS, COL>(
                d, b.max_steps, L, (gu32*)(b.pairs + (size_t)blockIdx.x * b.pair_stride));
    }
}

// The list build and one force pass on given positions, with the step kernel's own
// functions (one workgroup): list-grid cell and rank of every atom, the cell starts, the
// pair words of every wave segment (translated to atom ids by the host), the forces the
// integrator would use, W_xy, and flags.
template <int APT>
__global__ __launch_bounds__(APT == kLargeApt ? kLargeThreads : kPairThreads) void k_debug_pair_form(
    SysDev Sg, double gamma_dot, int64_t kstep, const double* r, int32_t kcap, uint32_t* pairs,
    int32_t* seg_count, int32_t* cell_of, int32_t* rank_of, int32_t* start, double* f,
    double* out) {
    const int cells = Sg.lc[0] * Sg.lc[1] * Sg.lc[2];
    const PairLds L = job_lds(Sg.n, cells);
    const int t = threadIdx.x;
    if (t == 0) *L.sys = Sg;
    for (int c = t; c < cells; c += blockDim.x) L.cnt[c] = 0;
    if (t == 0) {
        L.pos[Sg.n] = make_uint4(0u, 0u, 0u, 0u);
        L.pos[Sg.n + 1] = make_uint4(1u << 31, 1u << 31, 1u << 31, 1u << 31);
    }
    for (int i = t; i < Sg.n; i += blockDim.x) {
        L.fxy[i] = 0ull;
        L.fz[i] = 0;
    }
    __syncthreads();
    const SysDev& S = *L.sys;
    const int n = S.n, tj = job_threads(n), wave = t >> 6;
    double x[APT], y[APT], z[APT];
    int rank[APT], cr[APT], cell[APT];
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * tj;
        const bool v = t < tj && a < n;
        x[j] = v ? r[a] : 0.0;
        y[j] = v ? r[n + a] : 0.0;
        z[j] = v ? r[2 * n + a] : 0.0;
    }
    const double dxle = le_offset(S, gamma_dot, kstep);
    const uint32_t dxq = fix32(dxle, S.fix_scale[0]);
    const int seg_cap = kcap * 64 * APT;
    gu32* seg = (gu32*)(pairs + (size_t)wave * seg_cap);
    bool ovf = false;
    const int count = pf_rebuild<APT>(S, dxle, dxq, x, y, z, rank, cr, L, seg, seg_cap, tj, cell, &ovf);
    PfSums ps{0.0, 0.0, 0.0, 0.0, 0.0, 0};
    ps = pf_forces<false>(n, cells, dxq, (const gu32*)pairs, seg_cap);
    if ((t & 63) == 0 && t < tj) seg_count[wave] = count;
    __syncthreads();
    double m[2] = {ps.w, (double)ps.close};
    pf_block_sum<2>(m, L.red, blockDim.x >> 6);
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int a = t + j * tj;
        if (t < tj && a < n) {
            const int3 q = unpack_force(L.fxy[rank[j]], L.fz[rank[j]]);
            f[a] = (double)((float)q.x * kForceStep);
            f[n + a] = (double)((float)q.y * kForceStep);
            f[2 * n + a] = (double)((float)q.z * kForceStep);
            cell_of[a] = cell[j];
            rank_of[a] = rank[j];
        }
    }
    for (int c = t; c <= cells; c += blockDim.x) start[c] = L.start[c];
    if (t == 0) {
        out[0] = m[0] * kSumStep;
        out[1] = m[1];
        out[2] = dxle;
        out[3] = ovf ? 1.0 : 0.0;
    }
}

}  // namespace

int pair_job_threads(int n) { return job_threads(n); }
int pair_job_apt(int n) { return job_apt(n); }
int pair_small_apt() { return kSmallApt; }

size_t lds_bytes_pairs(int n, int cells) { return kJobBytes + plan_pairs(n, cells).total; }

template <int APT, bool NH, bool OBS, bool COL, bool PL>
static hipError_t launch_pairs_t(const BatchLaunch& b, hipStream_t s) {
    (void)hipFuncSetAttribute((const void*)k_daughters_pairs<APT, NH, OBS, COL, PL>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)b.lds_bytes);
    hipLaunchKernelGGL((k_daughters_pairs<APT, NH, OBS, COL, PL>), dim3(b.grid), dim3(b.threads),
                       b.lds_bytes, s, b);
    return hipGetLastError();
}

template <bool NH, bool OBS, bool COL>
static hipError_t launch_pairs_a(const BatchLaunch& b, hipStream_t s) {
    // the atoms per thread of the largest job; every job of the launch runs with it. Pair
    // words in LDS only fit next to systems of four atoms per thread.
    if (b.apt == kSmallApt)
        return b.pairs_lds ? launch_pairs_t<kSmallApt, NH, OBS, COL, true>(b, s)
                           : launch_pairs_t<kSmallApt, NH, OBS, COL, false>(b, s);
    if (b.pairs_lds) return hipErrorInvalidValue;
    return launch_pairs_t<kLargeApt, NH, OBS, COL, false>(b, s);
}

hipError_t launch_pairs(const BatchLaunch& b, hipStream_t s) {
    if (b.precision != 1 || (!b.pairs && !b.pairs_lds) || b.threads > kPairThreads ||
        b.threads % 64 != 0 ||
        (b.apt != kSmallApt && b.apt != kLargeApt))
        return hipErrorInvalidValue;
    // colour-field daughters do not record the extra observables
    if (b.field) {
        if (b.obs) return hipErrorInvalidValue;
        return b.thermo ? launch_pairs_a<true, false, true>(b, s)
                        : launch_pairs_a<false, false, true>(b, s);
    }
    if (b.obs)
        return b.thermo ? launch_pairs_a<true, true, false>(b, s)
                        : launch_pairs_a<false, true, false>(b, s);
    return b.thermo ? launch_pairs_a<true, false, false>(b, s)
                    : launch_pairs_a<false, false, false>(b, s);
}

hipError_t launch_debug_pair_form(const SysDev& S, double gamma_dot, int64_t kstep, const double* r,
                                  int32_t kcap, uint32_t* pairs, int32_t* seg_count,
                                  int32_t* cell_of, int32_t* rank_of, int32_t* start, double* f,
                                  double* out, hipStream_t s) {
    const int threads = job_threads(S.n);
    const size_t lds = lds_bytes_pairs(S.n, S.lc[0] * S.lc[1] * S.lc[2]);
    if (job_apt(S.n) == kSmallApt) {
        (void)hipFuncSetAttribute((const void*)k_debug_pair_form<kSmallApt>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_debug_pair_form<kSmallApt>, dim3(1), dim3(threads), lds, s, S,
                           gamma_dot, kstep, r, kcap, pairs, seg_count, cell_of, rank_of, start, f,
                           out);
    } else {
        (void)hipFuncSetAttribute((const void*)k_debug_pair_form<kLargeApt>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_debug_pair_form<kLargeApt>, dim3(1), dim3(threads), lds, s, S, gamma_dot,
                           kstep, r, kcap, pairs, seg_count, cell_of, rank_of, start, f, out);
    }
    return hipGetLastError();
}

}  // namespace ttcf
