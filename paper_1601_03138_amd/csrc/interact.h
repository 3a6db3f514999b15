// Softened-gravity interaction functions shared by the force kernels (k_force.hip) and the
// one-launch walk + force kernel (k_fused.hip).
//
// Particle term (equation ParticleParticleNbody, G = 1):
//   a_i += m_j (r_j - r_i) / (|r_j - r_i|^2 + eps_i^2)^{3/2},  phi_i -= m_j / (...)^{1/2}
// Superparticle term (equation ParticleSuperparticleNbody with the superparticle at r'_j,
// extended to the quadrupole; r = r_i - X, R^2 = |r|^2 + eps_i^2):
//   phi_i -= M/R + (1/2) r.Q.r / R^5
//   a_i   += -M r / R^3 + Q r / R^5 - (5/2) (r.Q.r) r / R^7
// FP32: hardware reciprocal square root; FP64: the hardware estimate refined by one
// Newton-Raphson step.
#pragma once

#include <hip/hip_runtime.h>

namespace fdx {

template <class T> struct V4;
template <> struct V4<float> { using t = float4; };
template <> struct V4<double> { using t = double4; };

__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
// Newton-Raphson for y = x^{-1/2}: y <- y + y (1 - x y^2) / 2, once from the hardware
// estimate.  Measured over 2^22 arguments spanning 60 binades, the estimate errs by at most
// 5.2e-8 relative and one step leaves at most 4.1e-15 (rms 3.2e-16; a second step gives
// 2.5e-16): far below the rounding of a force sum over thousands of list entries.
__device__ __forceinline__ double rsqrt_t(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double r = fma(-(x * y), y, 1.0);
    return fma(y * r, 0.5, y);
}

// Tree part of TreePM (cutoff kernel, monopole): the Newtonian pair force times
// g(xi), xi = 2 r / r_cut, the complement of the force between two S2 clouds of diameter
// r_cut (Hockney & Eastwood):
//   g = 1 - xi^3 (224 - 224 xi^2 + 70 xi^3 + 48 xi^4 - 21 xi^5) / 140,              xi <= 1
//   g = 1 - (12 - 224 xi^2 + 896 xi^3 - 840 xi^4 + 224 xi^5 + 70 xi^6 - 48 xi^7 + 7 xi^8)/140,
//                                                                            1 < xi < 2
//   g = 0 beyond; r unsoftened, softening in the Newtonian factor only; no potential.
// The division by 140 is folded into the coefficients (Horner form), so no divide is issued.
template <class T>
__device__ __forceinline__ T s2_cutoff(T xi) {
    if (xi >= (T)2) return (T)0;
    if (xi <= (T)1) {
        // (224 - 224 xi^2 + 70 xi^3 + 48 xi^4 - 21 xi^5) / 140
        const T p = fma(xi, fma(xi, fma(xi, fma(xi, (T)(-21.0 / 140.0), (T)(48.0 / 140.0)),
                                        (T)0.5), (T)-1.6), (T)0);
        return (T)1 - xi * xi * xi * fma(xi, p, (T)1.6);
    }
    // (12 - 224 xi^2 + 896 xi^3 - 840 xi^4 + 224 xi^5 + 70 xi^6 - 48 xi^7 + 7 xi^8) / 140
    const T q = fma(xi, fma(xi, fma(xi, fma(xi, fma(xi, fma(xi, fma(xi, (T)0.05,
                                                                     (T)(-48.0 / 140.0)),
                                                             (T)0.5), (T)1.6), (T)-6.0),
                                    (T)6.4), (T)-1.6), (T)0);
    return (T)1 - fma(xi, q, (T)(12.0 / 140.0));
}

// unsoftened |r| for the cutoff argument: FP32 from the hardware reciprocal square root
// (a separation whose square is below the smallest normal float gives g = 1 either way);
// FP64 the correctly rounded square root
__device__ __forceinline__ float cut_dist(float r2) {
    return r2 >= 1.17549435e-38f ? r2 * __builtin_amdgcn_rsqf(r2) : 0.0f;
}
__device__ __forceinline__ double cut_dist(double r2) { return sqrt(r2); }

template <class T, bool CUT = false>
__device__ __forceinline__ void pp(const typename V4<T>::t &J, T xi, T yi, T zi, T e2, T &ax,
                                   T &ay, T &az, T &ph, T cut_s = (T)0) {
    const T dx = J.x - xi, dy = J.y - yi, dz = J.z - zi;
    if (CUT) {
        const T r2u = fma(dz, dz, fma(dy, dy, dx * dx));
        const T ri = rsqrt_t(r2u + e2);
        const T f = J.w * ri * ri * ri * s2_cutoff<T>(cut_dist(r2u) * cut_s);
        ax = fma(f, dx, ax);
        ay = fma(f, dy, ay);
        az = fma(f, dz, az);
        return;
    }
    const T r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
    const T ri = rsqrt_t(r2);
    const T mri = J.w * ri;
    const T mri3 = mri * (ri * ri);
    ax = fma(mri3, dx, ax);
    ay = fma(mri3, dy, ay);
    az = fma(mri3, dz, az);
    ph -= mri;
}

template <class T, bool QUAD, bool CUT = false>
__device__ __forceinline__ void pc(const typename V4<T>::t &A, const typename V4<T>::t &B,
                                   const typename V4<T>::t &C, T xi, T yi, T zi, T e2, T &ax,
                                   T &ay, T &az, T &ph, T cut_s = (T)0) {
    const T rx = xi - A.x, ry = yi - A.y, rz = zi - A.z;
    if (CUT) {                                       // monopole with cutoff
        const T r2u = fma(rz, rz, fma(ry, ry, rx * rx));
        const T Ri = rsqrt_t(r2u + e2);
        const T f = A.w * Ri * Ri * Ri * s2_cutoff<T>(cut_dist(r2u) * cut_s);
        ax = fma(-f, rx, ax);
        ay = fma(-f, ry, ay);
        az = fma(-f, rz, az);
        return;
    }
    const T R2 = fma(rz, rz, fma(ry, ry, fma(rx, rx, e2)));
    const T Ri = rsqrt_t(R2);
    const T Ri2 = Ri * Ri;
    const T MRi = A.w * Ri;
    if (!QUAD) {
        const T MRi3 = MRi * Ri2;
        ax = fma(-MRi3, rx, ax);
        ay = fma(-MRi3, ry, ay);
        az = fma(-MRi3, rz, az);
        ph -= MRi;
    } else {
        // B = {Qxx, Qyy, Qzz, Qxy}, C = {Qxz, Qyz, -, -}
        const T qx = fma(B.w, ry, fma(C.x, rz, B.x * rx));
        const T qy = fma(B.w, rx, fma(C.y, rz, B.y * ry));
        const T qz = fma(C.x, rx, fma(C.y, ry, B.z * rz));
        const T rqr = fma(rx, qx, fma(ry, qy, rz * qz));
        const T Ri5 = Ri * Ri2 * Ri2;
        const T t = rqr * Ri5;                       // r.Q.r / R^5
        const T u = Ri2 * fma((T)2.5, t, MRi);       // M/R^3 + (5/2) r.Q.r / R^7
        ax = fma(-u, rx, fma(Ri5, qx, ax));
        ay = fma(-u, ry, fma(Ri5, qy, ay));
        az = fma(-u, rz, fma(Ri5, qz, az));
        ph -= fma((T)0.5, t, MRi);
    }
}

}  // namespace fdx
