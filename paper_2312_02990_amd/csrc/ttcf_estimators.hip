// ttcf_estimators.hip -- the TTCF response with the modified integrand of Eq. (corr_modified),
// <Omega(0)B(s)> - <Omega(0)><B(s)>, from the per-start-state accumulator rows; and the
// accumulation of the extra observables (Eq. TTCF and Eq. integrand with B another phase
// function, Omega(0) still from P_xy(0)).
//
// With Omega_d(0) = -coef P_xy,d(0) (coef = V gamma_dot / T, Eq. TTCF1), a row n holds
// D_n(t) (mapping mean of B(t)) and I_n(t) (mapping mean of int_0^t P_xy(0) B(s) ds), and
// its P_xy row holds P_n(0), the mapping mean of P_xy(0). Over N rows of equal size the
// estimate is
//   theta(t) = <D(0)> - coef <I(t)> + coef <P(0)> J(t),   J(t) = int_0^t <D(s)> ds,
// the last term being -int <Omega(0)><B(s)> ds (for B = P_xy, P = D). Its standard error is
// the jackknife over the rows (start states), in FP64 with compensated sums.
#include <hip/hip_runtime.h>

#include "ttcf_internal.h"

namespace ttcf {
namespace {

__device__ __forceinline__ void comp_add(double& sum, double& comp, double v) {
    const double t = sum + v;
    comp += fabs(sum) >= fabs(v) ? (sum - t) + v : (v - t) + sum;
    sum = t;
}

// one thread per selected row: J_n(t_k), the trapezoid integral of D_n on the step grid
__global__ void k_row_trapz(ModifiedLaunch a) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_rows) return;
    const double* d = a.d_all + (size_t)a.rows[r] * a.stride;
    double* j = a.j_rows + (size_t)r * a.n_t;
    double s = 0.0, c = 0.0;
    j[0] = 0.0;
    for (int k = 1; k < a.n_t; ++k) {
        comp_add(s, c, 0.5 * a.dt * (d[k - 1] + d[k]));
        j[k] = s + c;
    }
}

// one thread per time point: the estimate and its jackknife error
__global__ void k_response_modified(ModifiedLaunch a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n_t) return;
    const int n = a.n_rows;
    double sd0 = 0.0, cd0 = 0.0, sp0 = 0.0, cp0 = 0.0, si = 0.0, ci = 0.0, sj = 0.0, cj = 0.0;
    for (int r = 0; r < n; ++r) {
        const size_t row = (size_t)a.rows[r] * a.stride;
        comp_add(sd0, cd0, a.d_all[row]);
        comp_add(sp0, cp0, a.p_all[(size_t)a.rows[r] * a.p_stride]);
        comp_add(si, ci, a.i_all[row + k]);
        comp_add(sj, cj, a.j_rows[(size_t)r * a.n_t + k]);
    }
    sd0 += cd0;
    sp0 += cp0;
    si += ci;
    sj += cj;
    const double inv_n = 1.0 / (double)n;
    const double md0 = sd0 * inv_n, mp0 = sp0 * inv_n, mi = si * inv_n, mj = sj * inv_n;
    a.out[k] = md0 - a.coef * mi + a.coef * mp0 * mj;
    double se = nan("");
    if (n > 1) {
        const double inv = 1.0 / (double)(n - 1);
        auto leave_out = [&](int r) {
            const size_t row = (size_t)a.rows[r] * a.stride;
            const double d0 = (sd0 - a.d_all[row]) * inv;
            const double p0 = (sp0 - a.p_all[(size_t)a.rows[r] * a.p_stride]) * inv;
            const double ii = (si - a.i_all[row + k]) * inv;
            const double jj = (sj - a.j_rows[(size_t)r * a.n_t + k]) * inv;
            return d0 - a.coef * ii + a.coef * p0 * jj;
        };
        double sm = 0.0, cm = 0.0;
        for (int r = 0; r < n; ++r) comp_add(sm, cm, leave_out(r));
        const double mean = (sm + cm) * inv_n;
        double sq = 0.0, cq = 0.0;
        for (int r = 0; r < n; ++r) {
            const double e = leave_out(r) - mean;
            comp_add(sq, cq, e * e);
        }
        se = sqrt((double)(n - 1) * inv_n * (sq + cq));
    }
    a.out[a.n_t + k] = se;
}

// one thread per (group, extra column): mapping means of B_c(t_k) and of the trapezoid
// integral of P_xy(0) B_c(s), compensated per daughter as in the P_xy accumulation
__global__ void k_accumulate_obs(AccumObsLaunch a) {
    constexpr int kMaps = 4;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= a.n_groups * kObsCols) return;
    const int g = id / kObsCols, col = id % kObsCols;
    const int b = a.first_of[g], e = a.first_of[g + 1];
    const int nm = min(e - b, kMaps);
    double p0[kMaps], sum[kMaps], comp[kMaps], prev[kMaps];
    const double* ser[kMaps];
    double dt = 0.0;
    for (int m = 0; m < nm; ++m) {
        const DaughterDesc& d = a.descs[b + m];
        ser[m] = d.xseries;
        dt = d.sys.dt;
        p0[m] = d.series[0] / d.sys.volume;
        prev[m] = d.xseries[col];
        sum[m] = 0.0;
        comp[m] = 0.0;
    }
    const double inm = 1.0 / (double)nm;
    double* dout = a.d_out + (size_t)g * a.row_stride + (size_t)col * a.stride;
    double* iout = a.i_out + (size_t)g * a.row_stride + (size_t)col * a.stride;
    double d0 = 0.0;
    for (int m = 0; m < nm; ++m) d0 += prev[m];
    dout[0] = d0 * inm;
    iout[0] = 0.0;
    for (int k = 1; k < a.n_t; ++k) {
        double dsum = 0.0, isum = 0.0;
        for (int m = 0; m < nm; ++m) {
            const double cur = ser[m][(size_t)k * kObsCols + col];
            comp_add(sum[m], comp[m], 0.5 * dt * (p0[m] * prev[m] + p0[m] * cur));
            prev[m] = cur;
            dsum += cur;
            isum += sum[m] + comp[m];
        }
        dout[k] = dsum * inm;
        iout[k] = isum * inm;
    }
}

}  // namespace

hipError_t launch_accumulate_obs(const AccumObsLaunch& a, hipStream_t s) {
    const int total = a.n_groups * kObsCols;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_accumulate_obs, dim3((total + 63) / 64), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_response_modified(const ModifiedLaunch& a, hipStream_t s) {
    if (a.n_rows <= 0 || a.n_t <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_row_trapz, dim3((a.n_rows + 63) / 64), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_response_modified, dim3((a.n_t + 63) / 64), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace ttcf
