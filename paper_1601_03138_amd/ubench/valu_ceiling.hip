// Instruction-throughput ceilings of gfx950 for the force kernels' arithmetic (packed FP32
// disabled, as in the library): FP32 and FP64 FMA rates, v_rsq_f32 and v_rsq_f64 rates, and
// the quadrupole particle-cell interaction with its j-record broadcast from LDS (no global
// memory in the loop), in FP32 and in FP64 (hardware estimate + one Newton step, as in the
// library).  A second FP32 form takes the linear part Q r = Q x_i - Q X from 4x4x1 FP32
// MFMAs (the alternative that was measured and not adopted); it prints how far its results
// are from the VALU form's.  Prints one line per measurement; used to derive the force
// kernels' rooflines.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#define CK(x)                                                                        \
    do {                                                                             \
        hipError_t e_ = (x);                                                         \
        if (e_ != hipSuccess) {                                                      \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                                \
        }                                                                            \
    } while (0)

__global__ void __launch_bounds__(256) k_fma(float *out, int iters, float a, float b) {
    float x[8];
    for (int k = 0; k < 8; k++) x[k] = threadIdx.x * 0.001f + k;
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int k = 0; k < 8; k++) x[k] = fmaf(x[k], a, b);
    }
    float s = 0;
    for (int k = 0; k < 8; k++) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_rsq(float *out, int iters, float a) {
    float x[8];
    for (int k = 0; k < 8; k++) x[k] = 1.0f + threadIdx.x * 0.001f + k;
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int k = 0; k < 8; k++) x[k] = __builtin_amdgcn_rsqf(x[k]) + a;
    }
    float s = 0;
    for (int k = 0; k < 8; k++) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// the library's quadrupole particle-cell interaction, j from a 64-entry LDS table
__global__ void __launch_bounds__(256) k_pc(float4 *out4, int iters, const float4 *tab) {
    __shared__ float4 t[3 * 64];
    for (int k = threadIdx.x; k < 3 * 64; k += blockDim.x) t[k] = tab[k];
    __syncthreads();
    const float xi = threadIdx.x * 1e-3f, yi = 0.5f - xi, zi = 0.25f + xi, e2 = 1e-6f;
    float ax = 0, ay = 0, az = 0, ph = 0;
    for (int i = 0; i < iters; i++) {
        const int j = i & 63;
        const float4 A = t[3 * j], B = t[3 * j + 1], C = t[3 * j + 2];
        const float rx = xi - A.x, ry = yi - A.y, rz = zi - A.z;
        const float R2 = fmaf(rz, rz, fmaf(ry, ry, fmaf(rx, rx, e2)));
        const float Ri = __builtin_amdgcn_rsqf(R2), Ri2 = Ri * Ri, MRi = A.w * Ri;
        const float qx = fmaf(B.w, ry, fmaf(C.x, rz, B.x * rx));
        const float qy = fmaf(B.w, rx, fmaf(C.y, rz, B.y * ry));
        const float qz = fmaf(C.x, rx, fmaf(C.y, ry, B.z * rz));
        const float rqr = fmaf(rx, qx, fmaf(ry, qy, rz * qz));
        const float Ri5 = Ri * Ri2 * Ri2, tt = rqr * Ri5, u = Ri2 * fmaf(2.5f, tt, MRi);
        ax = fmaf(-u, rx, fmaf(Ri5, qx, ax));
        ay = fmaf(-u, ry, fmaf(Ri5, qy, ay));
        az = fmaf(-u, rz, fmaf(Ri5, qz, az));
        ph -= fmaf(0.5f, tt, MRi);
    }
    out4[blockIdx.x * blockDim.x + threadIdx.x] = make_float4(ax, ay, az, ph);
}

// The same interaction with Q r from three 4x4x1 FP32 MFMAs.  Per j six float4 in LDS: (X, M),
// (-(Q X), 0), and the rows (Q[r][0..2], 0) for r = 0..3 (row 3 zero).  The four lanes of a
// 4-lane block share the j-entry (here every lane does); lane l supplies A = Q[l % 4][k] and
// B = its own coordinate k, so after k = 0, 1, 2 its accumulator holds (Q x_i - Q X)_r,
// r = 0..3, for its own particle; the accumulator starts at -(Q X).
__global__ void __launch_bounds__(256) k_pc_mfma(float4 *out4, int iters, const float4 *tab) {
    __shared__ float4 t[6 * 64];
    for (int k = threadIdx.x; k < 6 * 64; k += blockDim.x) t[k] = tab[k];
    __syncthreads();
    const float xi = threadIdx.x * 1e-3f, yi = 0.5f - xi, zi = 0.25f + xi, e2 = 1e-6f;
    const int row = threadIdx.x & 3;
    float ax = 0, ay = 0, az = 0, ph = 0;
    typedef float f4 __attribute__((ext_vector_type(4)));
    for (int i = 0; i < iters; i++) {
        const int j = i & 63;
        const float4 XM = t[6 * j], nqx = t[6 * j + 1], Ar = t[6 * j + 2 + row];
        f4 acc = {nqx.x, nqx.y, nqx.z, nqx.w};
        acc = __builtin_amdgcn_mfma_f32_4x4x1f32(Ar.x, xi, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_4x4x1f32(Ar.y, yi, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_4x4x1f32(Ar.z, zi, acc, 0, 0, 0);
        const float qx = acc[0], qy = acc[1], qz = acc[2];
        const float rx = xi - XM.x, ry = yi - XM.y, rz = zi - XM.z;
        const float R2 = fmaf(rz, rz, fmaf(ry, ry, fmaf(rx, rx, e2)));
        const float Ri = __builtin_amdgcn_rsqf(R2), Ri2 = Ri * Ri, MRi = XM.w * Ri;
        const float rqr = fmaf(rx, qx, fmaf(ry, qy, rz * qz));
        const float Ri5 = Ri * Ri2 * Ri2, tt = rqr * Ri5, u = Ri2 * fmaf(2.5f, tt, MRi);
        ax = fmaf(-u, rx, fmaf(Ri5, qx, ax));
        ay = fmaf(-u, ry, fmaf(Ri5, qy, ay));
        az = fmaf(-u, rz, fmaf(Ri5, qz, az));
        ph -= fmaf(0.5f, tt, MRi);
    }
    out4[blockIdx.x * blockDim.x + threadIdx.x] = make_float4(ax, ay, az, ph);
}

__global__ void __launch_bounds__(256) k_fma64(double *out, int iters, double a, double b) {
    double x[8];
    for (int k = 0; k < 8; k++) x[k] = threadIdx.x * 0.001 + k;
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int k = 0; k < 8; k++) x[k] = fma(x[k], a, b);
    }
    double s = 0;
    for (int k = 0; k < 8; k++) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_rsq64(double *out, int iters, double a) {
    double x[8];
    for (int k = 0; k < 8; k++) x[k] = 1.0 + threadIdx.x * 0.001 + k;
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int k = 0; k < 8; k++) x[k] = __builtin_amdgcn_rsq(x[k]) + a;
    }
    double s = 0;
    for (int k = 0; k < 8; k++) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__device__ __forceinline__ double rsqrt_nr1(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double r = fma(-(x * y), y, 1.0);
    return fma(y * r, 0.5, y);
}

// the library's FP64 quadrupole particle-cell interaction, j from a 64-entry LDS table
__global__ void __launch_bounds__(256) k_pc64(double *out, int iters, const double4 *tab) {
    __shared__ double4 t[3 * 64];
    for (int k = threadIdx.x; k < 3 * 64; k += blockDim.x) t[k] = tab[k];
    __syncthreads();
    const double xi = threadIdx.x * 1e-3, yi = 0.5 - xi, zi = 0.25 + xi, e2 = 1e-6;
    double ax = 0, ay = 0, az = 0, ph = 0;
    for (int i = 0; i < iters; i++) {
        const int j = i & 63;
        const double4 A = t[3 * j], B = t[3 * j + 1], C = t[3 * j + 2];
        const double rx = xi - A.x, ry = yi - A.y, rz = zi - A.z;
        const double R2 = fma(rz, rz, fma(ry, ry, fma(rx, rx, e2)));
        const double Ri = rsqrt_nr1(R2), Ri2 = Ri * Ri, MRi = A.w * Ri;
        const double qx = fma(B.w, ry, fma(C.x, rz, B.x * rx));
        const double qy = fma(B.w, rx, fma(C.y, rz, B.y * ry));
        const double qz = fma(C.x, rx, fma(C.y, ry, B.z * rz));
        const double rqr = fma(rx, qx, fma(ry, qy, rz * qz));
        const double Ri5 = Ri * Ri2 * Ri2, tt = rqr * Ri5, u = Ri2 * fma(2.5, tt, MRi);
        ax = fma(-u, rx, fma(Ri5, qx, ax));
        ay = fma(-u, ry, fma(Ri5, qy, ay));
        az = fma(-u, rz, fma(Ri5, qz, az));
        ph -= fma(0.5, tt, MRi);
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = ax + ay + az + ph;
}

int main() {
    const int blocks = 256 * 16, threads = 256, iters = 4096;
    float *out = nullptr;
    float4 *tab = nullptr;
    double *out64 = nullptr;
    double4 *tab64 = nullptr;
    CK(hipMalloc(&out64, sizeof(double) * blocks * threads));
    CK(hipMalloc(&tab64, sizeof(double4) * 3 * 64));
    std::vector<double4> h64(3 * 64);
    for (int k = 0; k < 3 * 64; k++)
        h64[k] = make_double4(0.1 * (k % 7) + 1, 0.2 * (k % 5) + 1, 0.3 * (k % 3) + 1, 1e-3);
    CK(hipMemcpy(tab64, h64.data(), sizeof(double4) * h64.size(), hipMemcpyHostToDevice));
    CK(hipMalloc(&out, sizeof(float) * blocks * threads));
    // FP32 superparticle table: 64 entries (X, M, Q), in the VALU layout (A = (X, M),
    // B = (Qxx, Qyy, Qzz, Qxy), C = (Qxz, Qyz, 0, 0)) and in the MFMA layout
    float4 *tab_m = nullptr, *out4 = nullptr, *out4_m = nullptr;
    const size_t nlane = (size_t)blocks * threads;
    CK(hipMalloc(&tab, sizeof(float4) * 3 * 64));
    CK(hipMalloc(&tab_m, sizeof(float4) * 6 * 64));
    CK(hipMalloc(&out4, sizeof(float4) * nlane));
    CK(hipMalloc(&out4_m, sizeof(float4) * nlane));
    std::vector<float4> h(3 * 64), hm(6 * 64);
    for (int j = 0; j < 64; j++) {
        const float X = 1.0f + 0.1f * (j % 7), Y = 1.0f + 0.2f * (j % 5), Z = 1.0f + 0.3f * (j % 3);
        const float qxx = 1e-4f * (1 + j % 3), qyy = 2e-4f * (1 + j % 5), qzz = 1.5e-4f,
                    qxy = 3e-5f * (j % 4), qxz = -2e-5f * (j % 3), qyz = 1e-5f * (j % 5);
        h[3 * j] = make_float4(X, Y, Z, 1e-3f);
        h[3 * j + 1] = make_float4(qxx, qyy, qzz, qxy);
        h[3 * j + 2] = make_float4(qxz, qyz, 0, 0);
        const float Q[3][3] = {{qxx, qxy, qxz}, {qxy, qyy, qyz}, {qxz, qyz, qzz}};
        hm[6 * j] = h[3 * j];
        float qX[3];
        for (int r = 0; r < 3; r++) qX[r] = Q[r][0] * X + Q[r][1] * Y + Q[r][2] * Z;
        hm[6 * j + 1] = make_float4(-qX[0], -qX[1], -qX[2], 0);
        for (int r = 0; r < 3; r++) hm[6 * j + 2 + r] = make_float4(Q[r][0], Q[r][1], Q[r][2], 0);
        hm[6 * j + 5] = make_float4(0, 0, 0, 0);
    }
    CK(hipMemcpy(tab, h.data(), sizeof(float4) * h.size(), hipMemcpyHostToDevice));
    CK(hipMemcpy(tab_m, hm.data(), sizeof(float4) * hm.size(), hipMemcpyHostToDevice));
    hipEvent_t a, b;
    CK(hipEventCreate(&a));
    CK(hipEventCreate(&b));
    float ms = 0;
    for (int rep = 0; rep < 2; rep++) {           // the second repetition is reported warm
        CK(hipEventRecord(a));
        hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(threads), 0, 0, out, iters, 1.0001f, 0.5f);
        CK(hipEventRecord(b));
        CK(hipEventSynchronize(b));
        CK(hipEventElapsedTime(&ms, a, b));
        const double fmas = (double)blocks * threads * iters * 8;
        std::printf("rep %d fma: %.3f ms, %.2f TFLOP/s (FMA = 2)\n", rep, ms, 2 * fmas / ms / 1e9);
        CK(hipEventRecord(a));
        hipLaunchKernelGGL(k_rsq, dim3(blocks), dim3(threads), 0, 0, out, iters, 0.25f);
        CK(hipEventRecord(b));
        CK(hipEventSynchronize(b));
        CK(hipEventElapsedTime(&ms, a, b));
        const double rs = (double)blocks * threads * iters * 8;
        std::printf("rep %d rsq+add: %.3f ms, %.2f T rsq/s\n", rep, ms, rs / ms / 1e9);
        CK(hipEventRecord(a));
        hipLaunchKernelGGL(k_pc, dim3(blocks), dim3(threads), 0, 0, out4, iters * 4, tab);
        CK(hipEventRecord(b));
        CK(hipEventSynchronize(b));
        CK(hipEventElapsedTime(&ms, a, b));
        const double pcs = (double)blocks * threads * iters * 4;
        std::printf("rep %d quadrupole pc (LDS j): %.3f ms, %.3e interactions/s, %.1f TFLOP/s at 54\n",
                    rep, ms, pcs / (ms * 1e-3), pcs * 54 / (ms * 1e-3) / 1e12);
        CK(hipEventRecord(a));
        hipLaunchKernelGGL(k_pc_mfma, dim3(blocks), dim3(threads), 0, 0, out4_m, iters * 4, tab_m);
        CK(hipEventRecord(b));
        CK(hipEventSynchronize(b));
        CK(hipEventElapsedTime(&ms, a, b));
        std::printf("rep %d quadrupole pc, Q r on 4x4x1 MFMA (LDS j): %.3f ms, %.3e interactions/s\n",
                    rep, ms, pcs / (ms * 1e-3));
        CK(hipEventRecord(a));
        hipLaunchKernelGGL(k_fma64, dim3(blocks), dim3(threads), 0, 0, out64, iters, 1.0001, 0.5);
        CK(hipEventRecord(b));
        CK(hipEventSynchronize(b));
        CK(hipEventElapsedTime(&ms, a, b));
        std::printf("rep %d fma f64: %.3f ms, %.2f TFLOP/s (FMA = 2)\n", rep, ms, 2 * fmas / ms / 1e9);
        CK(hipEventRecord(a));
        hipLaunchKernelGGL(k_rsq64, dim3(blocks), dim3(threads), 0, 0, out64, iters, 0.25);
        CK(hipEventRecord(b));
        CK(hipEventSynchronize(b));
        CK(hipEventElapsedTime(&ms, a, b));
        std::printf("rep %d rsq f64+add: %.3f ms, %.2f T rsq/s\n", rep, ms, rs / ms / 1e9);
        CK(hipEventRecord(a));
        hipLaunchKernelGGL(k_pc64, dim3(blocks), dim3(threads), 0, 0, out64, iters, tab64);
        CK(hipEventRecord(b));
        CK(hipEventSynchronize(b));
        CK(hipEventElapsedTime(&ms, a, b));
        const double pcs64 = (double)blocks * threads * iters;
        std::printf("rep %d quadrupole pc f64 (LDS j): %.3f ms, %.3e interactions/s, %.1f TFLOP/s at 54\n",
                    rep, ms, pcs64 / (ms * 1e-3), pcs64 * 54 / (ms * 1e-3) / 1e12);
    }
    {   // the two FP32 forms on the first workgroup's lanes (the other workgroups repeat them)
        std::vector<float4> r1(threads), r2(threads);
        CK(hipMemcpy(r1.data(), out4, sizeof(float4) * threads, hipMemcpyDeviceToHost));
        CK(hipMemcpy(r2.data(), out4_m, sizeof(float4) * threads, hipMemcpyDeviceToHost));
        double da = 0, dp = 0;
        for (int t = 0; t < threads; t++) {
            const double ex = r2[t].x - r1[t].x, ey = r2[t].y - r1[t].y, ez = r2[t].z - r1[t].z;
            const double n = std::sqrt((double)r1[t].x * r1[t].x + (double)r1[t].y * r1[t].y +
                                       (double)r1[t].z * r1[t].z);
            da = std::fmax(da, std::sqrt(ex * ex + ey * ey + ez * ez) / n);
            dp = std::fmax(dp, std::fabs((double)r2[t].w - r1[t].w) / std::fabs((double)r1[t].w));
        }
        std::printf("MFMA form vs VALU form: max rel acceleration diff %.2e, potential %.2e\n", da, dp);
    }
    CK(hipFree(tab_m));
    CK(hipFree(out4));
    CK(hipFree(out4_m));
    CK(hipFree(out64));
    CK(hipFree(tab64));
    CK(hipFree(out));
    CK(hipFree(tab));
    return 0;
}
