// ttcf_mlp.hip -- gfx950 kernels of the learned control variate: start-state features, a
// bfloat16 matrix-core GEMM with FP32 accumulation (forward and backward passes of the MLP),
// Adam, and the integral h = Omega(0) int g ds of the predicted response.
#include <hip/hip_runtime.h>

#include "ttcf_internal.h"

namespace ttcf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even
__device__ __forceinline__ short f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ---------------------------------------------------------------------------------------
// GEMM: C(m, n) = sum_k A(m, k) B(k, n), A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn]
// Operands are rounded to bfloat16 as they are staged into LDS; gfx950's
// v_mfma_f32_16x16x32_bf16 accumulates in FP32. Workgroup tile 64 x 64 (four waves of
// 32 x 32, each 2 x 2 MFMA tiles), K step 32: one matrix instruction per tile and step.
// Operand layout of the 16x16x32 instruction: lane l holds A[l % 16][8 (l / 16) + i] and
// B[8 (l / 16) + i][l % 16] (i = 0..7); the result D[4 (l / 16) + i][l % 16].
// Epilogues: 0 C = acc + bias; 1 Z = acc + bias, C = gelu(Z); 2 C = acc * gelu'(Zin).
// The K loop runs in a fixed order: results are deterministic.
// ---------------------------------------------------------------------------------------

constexpr int kBM = 64, kBN = 64, kBK = 32;

__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
    __shared__ short As[kBM][kBK + 4];
    __shared__ short Bs[kBK][kBN + 4];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += kBK) {
        for (int e = t; e < kBM * kBK; e += 256) {
            const int r = e / kBK, c = e % kBK;
            const int m = m0 + r, k = k0 + c;
            const float v = (m < g.M && k < g.K) ? g.A[(int64_t)m * g.sam + (int64_t)k * g.sak] : 0.f;
            As[r][c] = f2bf(v);
        }
        for (int e = t; e < kBK * kBN; e += 256) {
            const int r = e / kBN, c = e % kBN;
            const int k = k0 + r, n = n0 + c;
            const float v = (k < g.K && n < g.N) ? g.B[(int64_t)k * g.sbk + (int64_t)n * g.sbn] : 0.f;
            Bs[r][c] = f2bf(v);
        }
        __syncthreads();
        {
            const int kb = (lane >> 4) * 8;
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int row = wm + i * 16 + (lane & 15);
#pragma unroll
                for (int e = 0; e < 8; ++e) a[i][e] = __builtin_bit_cast(__bf16, As[row][kb + e]);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int col = wn + j * 16 + (lane & 15);
#pragma unroll
                for (int e = 0; e < 8; ++e) b[j][e] = __builtin_bit_cast(__bf16, Bs[kb + e][col]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
                const int n = n0 + wn + j * 16 + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][r];
                const int64_t o = (int64_t)m * g.ldc + n;
                if (g.epi == 0) {
                    if (g.bias) v += g.bias[n];
                    g.C[o] = v;
                } else if (g.epi == 1) {
                    if (g.bias) v += g.bias[n];
                    g.Z[o] = v;
                    g.C[o] = gelu_f(v);
                } else {
                    g.C[o] = v * gelu_grad_f(g.Zin[o]);
                }
            }
}

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0) return hipSuccess;
    dim3 grid((g.N + kBN - 1) / kBN, (g.M + kBM - 1) / kBM);
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// small element-wise and reduction kernels (fixed-order sums)
// ---------------------------------------------------------------------------------------

// out[n] = sum over the M rows of X(m, n): 64 columns per workgroup, its 16 waves taking
// every 16th row, the wave partials added in wave order (a fixed order)
__global__ __launch_bounds__(1024) void k_colsum(const float* X, int M, int N, int ld,
                                                 float* out) {
    __shared__ float part[16][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + lane;
    float s = 0.f;
    if (n < N)
        for (int m = w; m < M; m += 16) s += X[(int64_t)m * ld + n];
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && n < N) {
        float t = 0.f;
        for (int v = 0; v < 16; ++v) t += part[v][lane];
        out[n] = t;
    }
}

// dY = 2 (Y - T) / (M N); loss (one value) = mean (Y - T)^2 when loss != null
__global__ void k_mse_grad(const float* Y, const float* Tg, int64_t count, float scale, float* dY) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dY[i] = scale * (Y[i] - Tg[i]);
}

__global__ void k_mse_loss(const float* Y, const float* Tg, int64_t count, double* loss) {
    __shared__ double part[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 256) {
        const double d = (double)Y[i] - (double)Tg[i];
        s += d * d;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int i = 0; i < 256; ++i) tot += part[i];
        *loss = tot / (double)count;
    }
}

__global__ void k_adam(float* P, const float* G, float* Mo, float* Vo, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = G[i];
    const float m = b1 * Mo[i] + (1.f - b1) * g;
    const float v = b2 * Vo[i] + (1.f - b2) * g * g;
    Mo[i] = m;
    Vo[i] = v;
    P[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// dst[r][c] = (src[idx[r]][c] - mu[c]) * inv[c] (mu, inv may be null: plain gather)
__global__ void k_gather_norm(const float* src, const int32_t* idx, int rows, int cols,
                              const float* mu, const float* inv, float* dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    const int64_t sr = idx ? idx[r] : r;
    float v = src[sr * cols + c];
    if (mu) v = (v - mu[c]) * inv[c];
    dst[e] = v;
}

// mean and 1/std of every column (two passes in FP64; std floor 1e-12)
__global__ void k_col_stats(const float* X, int64_t rows, int cols, float* mu, float* inv) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    double s = 0.0;
    for (int64_t r = 0; r < rows; ++r) s += X[r * cols + c];
    const double m = s / (double)rows;
    double q = 0.0;
    for (int64_t r = 0; r < rows; ++r) {
        const double d = X[r * cols + c] - m;
        q += d * d;
    }
    const double sd = sqrt(q / (double)(rows > 1 ? rows - 1 : 1));
    mu[c] = (float)m;
    inv[c] = (float)(1.0 / (sd > 1e-12 ? sd : 1e-12));
}

hipError_t launch_colsum(const float* X, int M, int N, int ld, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3((N + 63) / 64), dim3(1024), 0, s, X, M, N, ld, out);
    return hipGetLastError();
}
hipError_t launch_mse_grad(const float* Y, const float* Tg, int64_t count, float scale, float* dY,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_mse_grad, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, Y, Tg,
                       count, scale, dY);
    return hipGetLastError();
}
hipError_t launch_mse_loss(const float* Y, const float* Tg, int64_t count, double* loss,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_mse_loss, dim3(1), dim3(256), 0, s, Y, Tg, count, loss);
    return hipGetLastError();
}
hipError_t launch_adam(float* P, const float* G, float* Mo, float* Vo, int64_t n, float lr,
                       int64_t step, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P, G, Mo, Vo, n,
                       lr, b1, b2, 1e-8f, c1, c2);
    return hipGetLastError();
}
hipError_t launch_gather_norm(const float* src, const int32_t* idx, int rows, int cols,
                              const float* mu, const float* inv, float* dst, hipStream_t s) {
    const int64_t n = (int64_t)rows * cols;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_norm, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, idx,
                       rows, cols, mu, inv, dst);
    return hipGetLastError();
}
hipError_t launch_col_stats(const float* X, int64_t rows, int cols, float* mu, float* inv,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_col_stats, dim3((cols + 63) / 64), dim3(64), 0, s, X, rows, cols, mu, inv);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// features of mapped start states
// ---------------------------------------------------------------------------------------
// Row layout (kCvIn = 64): [P_xy(0), Omega(0); per slab k of kCvSlabs = 20 in y (k = floor(y
// 20 / Ly) clamped): sum p_x, sum p_x p_y, and half the pair virial x_ij F_y,ij of each of the
// slab's atoms; then sum_i (F_x,i p_y,i + p_x,i F_y,i) and sum_{i<j} (p_x,i - p_x,j) F_y,ij],
// all of the mapped start state (Eq. (mappings): x -> -x for mappings 2 and 3, p_x and p_y
// signs as below). One workgroup of 64 threads per row: the mapped state is staged in LDS,
// thread q computes the pair terms of atoms q, q + 64, ... against every other atom (each
// pair seen from both sides, so no atomics), then thread q < 62 forms one sum in atom order
// (deterministic). FP64 throughout; LDS 9 n doubles.
__global__ __launch_bounds__(64) void k_cv_features(
    const double* states, int32_t n, const int32_t* state_of, const int32_t* map_of,
    const double* vpxy0, const double* vsign, int32_t rows, double lx, double ly, double lz,
    double rc2, double c_attr, double volume, double temperature, double gamma_dot, float* out,
    double* b0_out, double* om_out) {
    extern __shared__ double cvs[];
    double* X = cvs;
    double* Y = X + n;
    double* Z = Y + n;
    double* PX = Z + n;
    double* PY = PX + n;
    double* FX = PY + n;
    double* FY = FX + n;
    double* VIR = FY + n;
    double* D2 = VIR + n;
    const int row = blockIdx.x;
    if (row >= rows) return;
    const double* st = states + (size_t)state_of[row] * 6 * (size_t)n;
    const int m = map_of[row];
    // mapping signs: p -> -p (m=1); (x, px) -> (-x, -px) (m=2); (x, py, pz) -> -(...) (m=3)
    const double sx = (m == 1 || m == 2) ? -1.0 : 1.0;
    const double sy = (m == 1 || m == 3) ? -1.0 : 1.0;
    const double sr = (m == 2 || m == 3) ? -1.0 : 1.0;  // x of the positions
    const int q = threadIdx.x;
    for (int a = q; a < n; a += blockDim.x) {
        X[a] = sr * st[a];
        Y[a] = st[n + a];
        Z[a] = st[2 * n + a];
        PX[a] = sx * st[3 * n + a];
        PY[a] = sy * st[4 * n + a];
    }
    __syncthreads();
    // minimum image with the reciprocal edges (the image chosen differs from a division's
    // only for separations within rounding of half a box, far beyond r_c)
    const double ilx = 1.0 / lx, ily = 1.0 / ly, ilz = 1.0 / lz;
    for (int i = q; i < n; i += blockDim.x) {
        const double xi = X[i], yi = Y[i], zi = Z[i], pxi = PX[i];
        double fx = 0.0, fy = 0.0, vir = 0.0, d2 = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = xi - X[j], dy = yi - Y[j], dz = zi - Z[j];
            dx -= lx * rint(dx * ilx);
            dy -= ly * rint(dy * ily);
            dz -= lz * rint(dz * ilz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rc2) {
                const double inv2 = 1.0 / r2;
                const double inv6 = inv2 * inv2 * inv2;
                const double fs = 24.0 * inv6 * (2.0 * inv6 - c_attr) * inv2;
                fx += fs * dx;
                fy += fs * dy;
                vir += 0.5 * dx * (fs * dy);
                d2 += 0.5 * (pxi - PX[j]) * (fs * dy);
            }
        }
        FX[i] = fx;
        FY[i] = fy;
        VIR[i] = vir;
        D2[i] = d2;
    }
    __syncthreads();
    float* o = out + (size_t)row * kCvIn;
    if (q < 3 * kCvSlabs) {
        const int slab = q % kCvSlabs;
        const int kind = q / kCvSlabs;  // 0 p_x, 1 p_x p_y, 2 virial
        const double inv = (double)kCvSlabs / ly;
        double acc = 0.0;
        for (int a = 0; a < n; ++a) {
            int k = (int)floor(Y[a] * inv);
            k = k < 0 ? 0 : (k > kCvSlabs - 1 ? kCvSlabs - 1 : k);
            if (k != slab) continue;
            acc += kind == 0 ? PX[a] : (kind == 1 ? PX[a] * PY[a] : VIR[a]);
        }
        o[2 + q] = (float)acc;
    } else if (q == 3 * kCvSlabs) {
        double acc = 0.0;
        for (int a = 0; a < n; ++a) acc += FX[a] * PY[a] + PX[a] * FY[a];
        o[2 + q] = (float)acc;
    } else if (q == 3 * kCvSlabs + 1) {
        double acc = 0.0;
        for (int a = 0; a < n; ++a) acc += D2[a];
        o[2 + q] = (float)acc;
    }
    if (q == 0) {
        // vpxy0 indexed by row (vsign null) or by state with the mapping's sign of P_xy
        const double vp = vsign ? vpxy0[state_of[row]] * vsign[m] : vpxy0[row];
        const double pxy = vp / volume;
        const double om = -(volume / temperature) * gamma_dot * pxy;
        o[0] = (float)pxy;
        o[1] = (float)om;
        if (b0_out) b0_out[row] = pxy;
        if (om_out) om_out[row] = om;
    }
}

// The same features for the four mapped rows of each of n_states start states (row
// 4 s + m), the pair sums done once per state: every feature of mapping m is the unmapped one
// times a sign (p_x sums and the two force-momentum sums by s_x, p_x p_y by s_x s_y, the virial
// by s_r, the sign of x), and the per-row kernel's operations give exactly those negations,
// so both kernels write the same bits.
__global__ __launch_bounds__(64) void k_cv_features_maps(
    const double* states, int32_t n, int32_t n_states, const double* vpxy0, const double* vsign,
    double lx, double ly, double lz, double rc2, double c_attr, double volume,
    double temperature, double gamma_dot, float* out, double* b0_out, double* om_out) {
    extern __shared__ double cvs[];
    double* X = cvs;
    double* Y = X + n;
    double* Z = Y + n;
    double* PX = Z + n;
    double* PY = PX + n;
    double* FX = PY + n;
    double* FY = FX + n;
    double* VIR = FY + n;
    double* D2 = VIR + n;
    double* feat = D2 + n;  // [3 kCvSlabs + 2] the unmapped features
    const int st_i = blockIdx.x;
    if (st_i >= n_states) return;
    const double* st = states + (size_t)st_i * 6 * (size_t)n;
    const int q = threadIdx.x;
    for (int a = q; a < n; a += blockDim.x) {
        X[a] = st[a];
        Y[a] = st[n + a];
        Z[a] = st[2 * n + a];
        PX[a] = st[3 * n + a];
        PY[a] = st[4 * n + a];
    }
    __syncthreads();
    const double ilx = 1.0 / lx, ily = 1.0 / ly, ilz = 1.0 / lz;
    for (int i = q; i < n; i += blockDim.x) {
        const double xi = X[i], yi = Y[i], zi = Z[i], pxi = PX[i];
        double fx = 0.0, fy = 0.0, vir = 0.0, d2 = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = xi - X[j], dy = yi - Y[j], dz = zi - Z[j];
            dx -= lx * rint(dx * ilx);
            dy -= ly * rint(dy * ily);
            dz -= lz * rint(dz * ilz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rc2) {
                const double inv2 = 1.0 / r2;
                const double inv6 = inv2 * inv2 * inv2;
                const double fs = 24.0 * inv6 * (2.0 * inv6 - c_attr) * inv2;
                fx += fs * dx;
                fy += fs * dy;
                vir += 0.5 * dx * (fs * dy);
                d2 += 0.5 * (pxi - PX[j]) * (fs * dy);
            }
        }
        FX[i] = fx;
        FY[i] = fy;
        VIR[i] = vir;
        D2[i] = d2;
    }
    __syncthreads();
    if (q < 3 * kCvSlabs) {
        const int slab = q % kCvSlabs;
        const int kind = q / kCvSlabs;  // 0 p_x, 1 p_x p_y, 2 virial
        const double inv = (double)kCvSlabs / ly;
        double acc = 0.0;
        for (int a = 0; a < n; ++a) {
            int k = (int)floor(Y[a] * inv);
            k = k < 0 ? 0 : (k > kCvSlabs - 1 ? kCvSlabs - 1 : k);
            if (k != slab) continue;
            acc += kind == 0 ? PX[a] : (kind == 1 ? PX[a] * PY[a] : VIR[a]);
        }
        feat[q] = acc;
    } else if (q == 3 * kCvSlabs) {
        double acc = 0.0;
        for (int a = 0; a < n; ++a) acc += FX[a] * PY[a] + PX[a] * FY[a];
        feat[q] = acc;
    } else if (q == 3 * kCvSlabs + 1) {
        double acc = 0.0;
        for (int a = 0; a < n; ++a) acc += D2[a];
        feat[q] = acc;
    }
    __syncthreads();
    // row 4 st_i + m: mapping signs p -> -p (m=1); (x, px) -> (-x, -px) (m=2);
    // (x, py, pz) -> -(...) (m=3)
    for (int e = q; e < 4 * (3 * kCvSlabs + 2); e += blockDim.x) {
        const int m = e / (3 * kCvSlabs + 2), f = e % (3 * kCvSlabs + 2);
        const double sx = (m == 1 || m == 2) ? -1.0 : 1.0;
        const double sy = (m == 1 || m == 3) ? -1.0 : 1.0;
        const double sr = (m == 2 || m == 3) ? -1.0 : 1.0;
        const int kind = f < 3 * kCvSlabs ? f / kCvSlabs : 3;
        const double sg = kind == 0 ? sx : (kind == 1 ? sx * sy : (kind == 2 ? sr : sx));
        out[(size_t)(4 * st_i + m) * kCvIn + 2 + f] = (float)(sg * feat[f]);
    }
    if (q < 4) {
        const int row = 4 * st_i + q;
        const double vp = vpxy0[st_i] * vsign[q];
        const double pxy = vp / volume;
        const double om = -(volume / temperature) * gamma_dot * pxy;
        out[(size_t)row * kCvIn] = (float)pxy;
        out[(size_t)row * kCvIn + 1] = (float)om;
        if (b0_out) b0_out[row] = pxy;
        if (om_out) om_out[row] = om;
    }
}

size_t lds_bytes_cv_features(int32_t n) { return sizeof(double) * 9 * (size_t)n; }
size_t lds_bytes_cv_features_maps(int32_t n) {
    return lds_bytes_cv_features(n) + sizeof(double) * (3 * kCvSlabs + 2);
}

hipError_t launch_cv_features(const double* states, int32_t n, const int32_t* state_of,
                              const int32_t* map_of, const double* vpxy0, const double* vsign,
                              int32_t rows, const double* box, double rc2, double c_attr,
                              double volume, double temperature, double gamma_dot, float* out,
                              double* b0_out, double* om_out, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    const size_t lds = lds_bytes_cv_features(n);
    (void)hipFuncSetAttribute((const void*)k_cv_features,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_cv_features, dim3(rows), dim3(64), lds, s, states, n, state_of, map_of,
                       vpxy0, vsign, rows, box[0], box[1], box[2], rc2, c_attr, volume,
                       temperature, gamma_dot, out, b0_out, om_out);
    return hipGetLastError();
}

hipError_t launch_cv_features_maps(const double* states, int32_t n, int32_t n_states,
                                   const double* vpxy0, const double* vsign, const double* box,
                                   double rc2, double c_attr, double volume, double temperature,
                                   double gamma_dot, float* out, double* b0_out, double* om_out,
                                   hipStream_t s) {
    if (n_states <= 0) return hipSuccess;
    const size_t lds = lds_bytes_cv_features_maps(n);
    (void)hipFuncSetAttribute((const void*)k_cv_features_maps,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_cv_features_maps, dim3(n_states), dim3(64), lds, s, states, n, n_states,
                       vpxy0, vsign, box[0], box[1], box[2], rc2, c_attr, volume, temperature,
                       gamma_dot, out, b0_out, om_out);
    return hipGetLastError();
}

// P_xy(0) (as V P_xy) and, when targets != null, B(t_1..t_nout) = P_xy of each daughter's
// recorded series, one workgroup per daughter.
__global__ void k_cv_gather_series(const double* const* series, int32_t count, int32_t n_out,
                                   double inv_volume, float* targets, double* vpxy0) {
    const int row = blockIdx.x;
    if (row >= count) return;
    const double* s = series[row];
    if (targets)
        for (int k = threadIdx.x; k < n_out; k += blockDim.x)
            targets[(size_t)row * n_out + k] = (float)(s[k + 1] * inv_volume);
    if (threadIdx.x == 0) vpxy0[row] = s[0];
}

hipError_t launch_cv_gather_series(const double* const* series, int32_t count, int32_t n_out,
                                   double inv_volume, float* targets, double* vpxy0, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cv_gather_series, dim3(count), dim3(64), 0, s, series, count, n_out,
                       inv_volume, targets, vpxy0);
    return hipGetLastError();
}

// h rows (stride values apart) into each daughter's own h series, the first lens[r] values
__global__ void k_cv_scatter_h(const double* h, int32_t stride, int32_t count, double* const* dst,
                               const int32_t* lens) {
    const int row = blockIdx.x;
    if (row >= count) return;
    double* d = dst[row];
    for (int k = threadIdx.x; k < lens[row]; k += blockDim.x) d[k] = h[(size_t)row * stride + k];
}

hipError_t launch_cv_scatter_h(const double* h, int32_t stride, int32_t count, double* const* dst,
                               const int32_t* lens, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cv_scatter_h, dim3(count), dim3(64), 0, s, h, stride, count, dst, lens);
    return hipGetLastError();
}

__global__ void k_fill_f64(double* p, double v, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

hipError_t launch_fill_f64(double* p, double v, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}

// h(t_k) = Omega(0) int_0^{t_k} g ds (trapezoid, g(0) = B(0)) of each row, FP64; pred holds
// the standardised predictions, B(t_k) = pred / yinv[k] + ymu[k]. out rows (n_out + 1 values)
// are out_stride apart.
__global__ void k_cv_h(const float* pred, int rows, int n_out, const float* ymu, const float* yinv,
                       const double* b0, const double* omega, double dt, double* out,
                       int64_t out_stride) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const float* p = pred + (size_t)r * n_out;
    double* h = out + (size_t)r * out_stride;
    double prev = b0[r], acc = 0.0;
    const double om = omega[r];
    h[0] = 0.0;
    for (int k = 0; k < n_out; ++k) {
        const double cur = (double)p[k] / (double)yinv[k] + (double)ymu[k];
        acc += 0.5 * dt * (prev + cur);
        prev = cur;
        h[k + 1] = om * acc;
    }
}

hipError_t launch_cv_h(const float* pred, int rows, int n_out, const float* ymu, const float* yinv,
                       const double* b0, const double* omega, double dt, double* out,
                       int64_t out_stride, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cv_h, dim3((rows + 63) / 64), dim3(64), 0, s, pred, rows, n_out, ymu, yinv,
                       b0, omega, dt, out, out_stride);
    return hipGetLastError();
}

// mean-term accumulation: for every t, add the mapping means of h over the groups of this
// chunk (group = `maps` consecutive rows) into compensated sums of H and H^2. First pass:
// workgroup (t block, partition p) takes the groups of partition p (contiguous ranges), its
// wave w every kMuWaves-th of them, and writes the wave's compensated partial sums; second
// pass: per t, the partials are added to the running sums in (p, w) order. The result does not
// depend on timing.
constexpr int kMuParts = 32;
constexpr int kMuWaves = 8;

__device__ __forceinline__ void mu_neumaier(double& sum, double& comp, double v) {
    const double t = sum + v;
    comp += fabs(sum) >= fabs(v) ? (sum - t) + v : (v - t) + sum;
    sum = t;
}

__global__ __launch_bounds__(64 * kMuWaves) void k_cv_mu_partial(const double* h, int groups,
                                                                  int maps, int nt,
                                                                  double* part) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int k = blockIdx.x * 64 + lane, p = blockIdx.y;
    if (k >= nt) return;
    const int per = (groups + kMuParts - 1) / kMuParts;
    const int g0 = p * per, g1 = min(groups, g0 + per);
    double s = 0.0, c = 0.0, s2 = 0.0, c2 = 0.0;
    for (int g = g0 + w; g < g1; g += kMuWaves) {
        double v = 0.0;
        for (int m = 0; m < maps; ++m) v += h[((size_t)g * maps + m) * nt + k];
        v /= (double)maps;
        mu_neumaier(s, c, v);
        mu_neumaier(s2, c2, v * v);
    }
    double* out = part + (size_t)(p * kMuWaves + w) * 4 * nt;
    out[k] = s;
    out[nt + k] = c;
    out[2 * nt + k] = s2;
    out[3 * nt + k] = c2;
}

__global__ void k_cv_mu_combine(const double* part, int nt, double* sum, double* comp,
                                double* sumsq, double* compsq) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    double s = sum[k], c = comp[k], s2 = sumsq[k], c2 = compsq[k];
    for (int i = 0; i < kMuParts * kMuWaves; ++i) {
        const double* q = part + (size_t)i * 4 * nt;
        mu_neumaier(s, c, q[k]);
        mu_neumaier(s, c, q[nt + k]);
        mu_neumaier(s2, c2, q[2 * nt + k]);
        mu_neumaier(s2, c2, q[3 * nt + k]);
    }
    sum[k] = s;
    comp[k] = c;
    sumsq[k] = s2;
    compsq[k] = c2;
}

size_t cv_mu_scratch_doubles(int nt) { return (size_t)kMuParts * kMuWaves * 4 * (size_t)nt; }

hipError_t launch_cv_mu_accum(const double* h, int groups, int maps, int nt, double* sum,
                              double* comp, double* sumsq, double* compsq, double* part,
                              hipStream_t s) {
    if (groups <= 0 || nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cv_mu_partial, dim3((nt + 63) / 64, kMuParts), dim3(64 * kMuWaves), 0, s,
                       h, groups, maps, nt, part);
    hipLaunchKernelGGL(k_cv_mu_combine, dim3((nt + 63) / 64), dim3(64), 0, s, part, nt, sum, comp,
                       sumsq, compsq);
    return hipGetLastError();
}

}  // namespace ttcf
