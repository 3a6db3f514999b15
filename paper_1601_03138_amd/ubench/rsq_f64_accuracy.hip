// Accuracy of the FP64 reciprocal square root used by the force kernels: the hardware
// estimate (v_rsq_f64) alone, after one Newton step (what the library uses) and after two,
// each against 1/sqrt(x) computed with the correctly rounded FP64 square root and division.
// Arguments: 2^22 values, mantissas spread over [1, 4) and exponents -30..30.  Prints the
// maximum and rms relative error of each.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cmath>
#include <vector>
__global__ void k(int n, double *e0, double *e1, double *e2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ex = (i % 61) - 30;                       // exponents -30..30
    const double x = ldexp(1.0 + (double)(i / 61) / (double)(n / 61 + 1) * 3.0, ex);
    const double r = 1.0 / sqrt(x);
    double y = __builtin_amdgcn_rsq(x);
    e0[i] = fabs(y - r) / r;
    double t = fma(-(x * y), y, 1.0);
    y = fma(y * t, 0.5, y);
    e1[i] = fabs(y - r) / r;
    t = fma(-(x * y), y, 1.0);
    y = fma(y * t, 0.5, y);
    e2[i] = fabs(y - r) / r;
}
int main() {
    const int n = 1 << 22;
    double *d0, *d1, *d2;
    if (hipMalloc(&d0, n * 8) || hipMalloc(&d1, n * 8) || hipMalloc(&d2, n * 8)) return 1;
    hipLaunchKernelGGL(k, dim3((n + 255) / 256), dim3(256), 0, 0, n, d0, d1, d2);
    std::vector<double> h0(n), h1(n), h2(n);
    if (hipMemcpy(h0.data(), d0, n * 8, hipMemcpyDeviceToHost) || hipMemcpy(h1.data(), d1, n * 8, hipMemcpyDeviceToHost) ||
        hipMemcpy(h2.data(), d2, n * 8, hipMemcpyDeviceToHost)) return 2;
    double m0 = 0, m1 = 0, m2 = 0, s0 = 0, s1 = 0, s2 = 0;
    for (int i = 0; i < n; i++) {
        m0 = fmax(m0, h0[i]); m1 = fmax(m1, h1[i]); m2 = fmax(m2, h2[i]);
        s0 += h0[i] * h0[i]; s1 += h1[i] * h1[i]; s2 += h2[i] * h2[i];
    }
    printf("estimate: max rel %.3e rms %.3e\none Newton step: max rel %.3e rms %.3e\ntwo Newton steps: max rel %.3e rms %.3e\n",
           m0, sqrt(s0 / n), m1, sqrt(s1 / n), m2, sqrt(s2 / n));
    return 0;
}
