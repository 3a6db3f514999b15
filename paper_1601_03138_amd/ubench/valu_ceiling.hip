// Instruction-throughput ceilings of gfx950 for the force kernel's arithmetic (packed FP32
// disabled, as in the library): FP32 FMA rate, v_rsq_f32 rate, and the quadrupole
// particle-cell interaction with its j-record broadcast from LDS (no global memory in the
// loop).  Prints one line per measurement; used to derive the force kernel's roofline.
#include <hip/hip_runtime.h>

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
__global__ void __launch_bounds__(256) k_pc(float *out, int iters, const float4 *tab) {
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
        const float Ri = __builtin_amdgcn_rsqf(R2), Ri2 = Ri * Ri, MRi = A.w * Ri, MRi3 = MRi * Ri2;
        const float qx = fmaf(B.w, ry, fmaf(C.x, rz, B.x * rx));
        const float qy = fmaf(B.w, rx, fmaf(C.y, rz, B.y * ry));
        const float qz = fmaf(C.x, rx, fmaf(C.y, ry, B.z * rz));
        const float rqr = fmaf(rx, qx, fmaf(ry, qy, rz * qz));
        const float Ri5 = Ri * Ri2 * Ri2, tt = rqr * Ri5, u = fmaf(2.5f * tt, Ri2, MRi3);
        ax = fmaf(-u, rx, fmaf(Ri5, qx, ax));
        ay = fmaf(-u, ry, fmaf(Ri5, qy, ay));
        az = fmaf(-u, rz, fmaf(Ri5, qz, az));
        ph -= fmaf(0.5f, tt, MRi);
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = ax + ay + az + ph;
}

int main() {
    const int blocks = 256 * 16, threads = 256, iters = 4096;
    float *out = nullptr;
    float4 *tab = nullptr;
    CK(hipMalloc(&out, sizeof(float) * blocks * threads));
    CK(hipMalloc(&tab, sizeof(float4) * 3 * 64));
    std::vector<float4> h(3 * 64);
    for (int k = 0; k < 3 * 64; k++)
        h[k] = make_float4(0.1f * (k % 7) + 1, 0.2f * (k % 5) + 1, 0.3f * (k % 3) + 1, 1e-3f);
    CK(hipMemcpy(tab, h.data(), sizeof(float4) * h.size(), hipMemcpyHostToDevice));
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
        hipLaunchKernelGGL(k_pc, dim3(blocks), dim3(threads), 0, 0, out, iters * 4, tab);
        CK(hipEventRecord(b));
        CK(hipEventSynchronize(b));
        CK(hipEventElapsedTime(&ms, a, b));
        const double pcs = (double)blocks * threads * iters * 4;
        std::printf("rep %d quadrupole pc (LDS j): %.3f ms, %.3e interactions/s, %.1f TFLOP/s at 54\n",
                    rep, ms, pcs / (ms * 1e-3), pcs * 54 / (ms * 1e-3) / 1e12);
    }
    CK(hipFree(out));
    CK(hipFree(tab));
    return 0;
}
