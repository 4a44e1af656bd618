// ttcf_device.h -- device helpers shared by the gfx950 kernel files: the reciprocal, cell
// coordinates, the Lees-Edwards offset and wrap, wavefront and workgroup reductions, the
// cell-count scan, the closed-form isokinetic kick and the 32-bit fixed-point map.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "ttcf_internal.h"

namespace ttcf {

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


__device__ __forceinline__ uint32_t fix32(double v, double scale) {
    return (uint32_t)(int64_t)rint(v * scale);
}

}  // namespace ttcf
