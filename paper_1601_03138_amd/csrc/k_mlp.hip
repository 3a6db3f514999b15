// Learned interaction-list length predictor: per-group features, an MLP 8 -> 64 -> 64 -> 1
// with SiLU activations in FP32, and its training kernels (forward + backward with a
// deterministic gradient reduction, Adam).
//
// The paper models the mean list length in closed form (equation nlist_long, section "Tree
// traverse and interaction calculation"); the network predicts each group's own length from
// cheap group features so list memory can be sized before a single walk.  Forces never
// depend on it: groups whose list does not fit are re-walked exactly.
//
// Parameter layout (4801 floats): W1[8][64], b1[64], W2[64][64], b2[64], W3[64], b3.
#include "dev_util.h"
#include "fdx_internal.h"
#include "mlp.h"

namespace fdx {

namespace {

constexpr int kH = kMlpHidden;
constexpr int kIn = kMlpIn;
constexpr int OW1 = 0, OB1 = kIn * kH, OW2 = OB1 + kH, OB2 = OW2 + kH * kH, OW3 = OB2 + kH,
              OB3 = OW3 + kH;
static_assert(OB3 + 1 == kMlpParams, "parameter layout");

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// Group features (raw, before standardisation):
//   0 ln n_i                         1 ln(largest extent of the group box, grid units)
//   2 ln(1 + distance of the box centre to the root centre, grid units)
//   3 ln(parent mass / system mass)  4 ln(parent side / root side)
//   5 depth of the group's cell      6 ln(parent count / parent volume in root units)
//   7 log2 N of the system
__global__ void k_features(const uint32_t *ngroups_c, Groups g, Cells c, const int64_t *sys_off,
                           const float *mu, const float *sd, float *X) {
    const uint32_t G = *ngroups_c;
    for (size_t gi = gtid(); gi < G; gi += gstride()) {
        const uint32_t *bx = g.box + 6 * gi;
        const uint32_t cell = g.cell[gi];
        const uint32_t par = c.parent[cell] == kNone ? cell : c.parent[cell];
        const uint32_t s = g.sys[gi];
        const float ext = (float)max(max(bx[3] - bx[0], bx[4] - bx[1]), bx[5] - bx[2]) + 1.0f;
        const float half = 1048576.0f;   // root centre in grid units: 2^20
        const float dx = 0.5f * ((float)bx[0] + (float)bx[3] + 1.0f) - half;
        const float dy = 0.5f * ((float)bx[1] + (float)bx[4] + 1.0f) - half;
        const float dz = 0.5f * ((float)bx[2] + (float)bx[5] + 1.0f) - half;
        const float dist = sqrtf(dx * dx + dy * dy + dz * dz);
        const double msys = c.mom[10 * (size_t)s];
        const double mpar = c.mom[10 * (size_t)par];
        const float plev = (float)c.level[par];
        const float nsys = (float)(sys_off[s + 1] - sys_off[s]);
        float f[kIn];
        f[0] = logf((float)g.count[gi]);
        f[1] = logf(ext);
        f[2] = logf(1.0f + dist);
        f[3] = (float)log(fmax(mpar, 1e-300) / fmax(msys, 1e-300));
        f[4] = -plev * 0.69314718f;
        f[5] = (float)c.level[cell];
        f[6] = logf((float)c.count[par]) + 3.0f * plev * 0.69314718f;
        f[7] = log2f(fmaxf(nsys, 1.0f));
#pragma unroll
        for (int k = 0; k < kIn; k++) X[gi * kIn + k] = (f[k] - mu[k]) / sd[k];
    }
}

// inference: one thread per sample; parameters staged in LDS.  The second layer runs over
// blocks of 8 units (8 accumulators, their weights read as vectors), which keeps the register
// budget near 100 and several waves per SIMD; every sum is taken in the same order as a
// plain unit-by-unit evaluation (bias first, then inputs ascending; the output over units
// ascending).  At least 4 waves per SIMD (128 registers).
__global__ void __launch_bounds__(256, 4)
k_mlp_infer(size_t n, const uint32_t *n_dev, const float *X, const float *P, float *y) {
    __shared__ float w[kMlpParams];
    for (int k = threadIdx.x; k < kMlpParams; k += blockDim.x) w[k] = P[k];
    __syncthreads();
    const size_t nn = n_dev ? *n_dev : n;
    for (size_t s = gtid(); s < nn; s += gstride()) {
        // the weights are read from LDS where they are used: without this compiler barrier
        // the first layer's 576 loop-invariant reads are hoisted out of the sample loop and
        // spill
        __asm__ volatile("" ::: "memory");
        float x[kIn], h1[kH];
#pragma unroll
        for (int k = 0; k < kIn; k++) x[k] = X[s * kIn + k];
#pragma unroll
        for (int u = 0; u < kH; u++) {
            float z = w[OB1 + u];
#pragma unroll
            for (int k = 0; k < kIn; k++) z = fmaf(x[k], w[OW1 + k * kH + u], z);
            h1[u] = silu(z);
        }
        float out = w[OB3];
#pragma unroll 1
        for (int u0 = 0; u0 < kH; u0 += 8) {
            float z[8];
#pragma unroll
            for (int j = 0; j < 8; j++) z[j] = w[OB2 + u0 + j];
#pragma unroll
            for (int k = 0; k < kH; k++) {
#pragma unroll
                for (int j = 0; j < 8; j++) z[j] = fmaf(h1[k], w[OW2 + k * kH + u0 + j], z[j]);
            }
#pragma unroll
            for (int j = 0; j < 8; j++) out = fmaf(silu(z[j]), w[OW3 + u0 + j], out);
        }
        y[s] = out;
    }
}

// Training forward + backward for one block of kSB samples (rows idx[b*kSB ...] of X, t):
// writes the block's partial gradient (sum over its samples of d loss / d param, with
// loss = mean over the whole batch of (y - t)^2) and its partial loss.
constexpr int kSB = 32;
constexpr int kTT = 256;

__global__ void __launch_bounds__(kTT)
k_mlp_train(size_t nb, const uint32_t *idx, const float *X, const float *T, const float *P,
            float inv_batch, float *gpart, float *lpart) {
    __shared__ float w[kMlpParams];
    __shared__ float xs[kSB][kIn];
    __shared__ float z1[kSB][kH], h1[kSB][kH], z2[kSB][kH], h2[kSB][kH];
    __shared__ float dy[kSB];
    __shared__ float red[kTT / kWave];
    const int tid = threadIdx.x;
    const size_t b = blockIdx.x;
    for (int k = tid; k < kMlpParams; k += kTT) w[k] = P[k];
    const size_t s0 = b * kSB;
    for (int k = tid; k < kSB * kIn; k += kTT) {
        const size_t s = s0 + k / kIn;
        xs[k / kIn][k % kIn] = s < nb ? X[(size_t)idx[s] * kIn + k % kIn] : 0.0f;
    }
    __syncthreads();
    // layer 1
    for (int k = tid; k < kSB * kH; k += kTT) {
        const int s = k / kH, u = k % kH;
        float z = w[OB1 + u];
#pragma unroll
        for (int i = 0; i < kIn; i++) z = fmaf(xs[s][i], w[OW1 + i * kH + u], z);
        z1[s][u] = z;
        h1[s][u] = silu(z);
    }
    __syncthreads();
    // layer 2
    for (int k = tid; k < kSB * kH; k += kTT) {
        const int s = k / kH, u = k % kH;
        float z = w[OB2 + u];
        for (int i = 0; i < kH; i++) z = fmaf(h1[s][i], w[OW2 + i * kH + u], z);
        z2[s][u] = z;
        h2[s][u] = silu(z);
    }
    __syncthreads();
    // output, loss, dy
    float lsum = 0.0f;
    if (tid < kSB) {
        const size_t s = s0 + tid;
        float out = w[OB3];
        for (int i = 0; i < kH; i++) out = fmaf(h2[tid][i], w[OW3 + i], out);
        const float e = s < nb ? out - T[idx[s]] : 0.0f;
        dy[tid] = 2.0f * e * inv_batch;
        lsum = e * e;
    }
    __syncthreads();
    float *g = gpart + b * kMlpParams;
    // dW3, db3
    if (tid < kH) {
        float a = 0.0f;
        for (int s = 0; s < kSB; s++) a = fmaf(h2[s][tid], dy[s], a);
        g[OW3 + tid] = a;
    }
    if (tid == kH) {
        float a = 0.0f;
        for (int s = 0; s < kSB; s++) a += dy[s];
        g[OB3] = a;
    }
    __syncthreads();
    // dz2 (in place of h2): dy * W3 * silu'(z2)
    for (int k = tid; k < kSB * kH; k += kTT) {
        const int s = k / kH, u = k % kH;
        h2[s][u] = dy[s] * w[OW3 + u] * silu_grad(z2[s][u]);
    }
    __syncthreads();
    // dW2[i][u] = sum_s h1[s][i] dz2[s][u];  db2[u] = sum_s dz2[s][u]
    for (int k = tid; k < kH * kH; k += kTT) {
        const int i = k / kH, u = k % kH;
        float a = 0.0f;
        for (int s = 0; s < kSB; s++) a = fmaf(h1[s][i], h2[s][u], a);
        g[OW2 + k] = a;
    }
    if (tid < kH) {
        float a = 0.0f;
        for (int s = 0; s < kSB; s++) a += h2[s][tid];
        g[OB2 + tid] = a;
    }
    __syncthreads();
    // dz1 (in place of z1): (dz2 W2^T) * silu'(z1)
    for (int k = tid; k < kSB * kH; k += kTT) {
        const int s = k / kH, i = k % kH;
        float a = 0.0f;
        for (int u = 0; u < kH; u++) a = fmaf(h2[s][u], w[OW2 + i * kH + u], a);
        h1[s][i] = a * silu_grad(z1[s][i]);
    }
    __syncthreads();
    // dW1[i][u] = sum_s x[s][i] dz1[s][u];  db1[u] = sum_s dz1[s][u]
    for (int k = tid; k < kIn * kH; k += kTT) {
        const int i = k / kH, u = k % kH;
        float a = 0.0f;
        for (int s = 0; s < kSB; s++) a = fmaf(xs[s][i], h1[s][u], a);
        g[OW1 + k] = a;
    }
    if (tid < kH) {
        float a = 0.0f;
        for (int s = 0; s < kSB; s++) a += h1[s][tid];
        g[OB1 + tid] = a;
    }
    // partial loss (sum of squared errors of this block)
    float v = lsum;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    if (lane_id() == 0) red[tid / kWave] = v;
    __syncthreads();
    if (tid == 0) {
        float a = 0.0f;
        for (int k = 0; k < kTT / kWave; k++) a += red[k];
        lpart[b] = a;
    }
}

// grad[p] = sum over blocks in block order (deterministic); loss = sum(lpart) / batch
__global__ void k_mlp_reduce(size_t nblocks, const float *gpart, const float *lpart,
                             float inv_batch, float *grad, float *loss) {
    for (size_t p = gtid(); p < (size_t)kMlpParams; p += gstride()) {
        float a = 0.0f;
        for (size_t b = 0; b < nblocks; b++) a += gpart[b * kMlpParams + p];
        grad[p] = a;
    }
    if (gtid() == 0) {
        float a = 0.0f;
        for (size_t b = 0; b < nblocks; b++) a += lpart[b];
        *loss = a * inv_batch;
    }
}

// Adam (Kingma & Ba): m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
// w <- w - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
__global__ void k_adam(float *P, const float *grad, float *m, float *v, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    for (size_t p = gtid(); p < (size_t)kMlpParams; p += gstride()) {
        const float gr = grad[p];
        const float mm = b1 * m[p] + (1.0f - b1) * gr;
        const float vv = b2 * v[p] + (1.0f - b2) * gr * gr;
        m[p] = mm;
        v[p] = vv;
        P[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
}

// capacity of each group's list from the prediction (log length) and a margin
__global__ void k_pred_caps(const uint32_t *ngroups_c, const float *y, float margin,
                            uint32_t cap_max, uint32_t *cap) {
    const uint32_t G = *ngroups_c;
    for (size_t gi = gtid(); gi < G; gi += gstride()) {
        const float c = ceilf(__expf(fminf(y[gi] + margin, 30.0f)));
        cap[gi] = (uint32_t)fminf(fmaxf(c, 1.0f), (float)cap_max);
    }
}

// Re-walk of overflowed groups: exact sizes into new segments appended after `base_total`.
__global__ void k_ovf_caps(const uint32_t *nsel, const uint32_t *sel, const uint32_t *cnt_e,
                           const uint32_t *cnt_s, uint32_t *ocap) {
    const uint32_t K = *nsel;
    for (size_t k = gtid(); k < K; k += gstride()) ocap[k] = cnt_e[sel[k]] + cnt_s[sel[k]];
}
__global__ void k_ovf_seg(const uint32_t *nsel, const uint32_t *sel, const uint32_t *ocap,
                          const uint64_t *ooff, const uint64_t *base_total, uint64_t *seg,
                          uint32_t *cap) {
    const uint32_t K = *nsel;
    for (size_t k = gtid(); k < K; k += gstride()) {
        const uint32_t gi = sel[k];
        seg[gi] = *base_total + ooff[k];
        cap[gi] = ocap[k];
    }
}

inline unsigned grid_for(size_t n, unsigned cap = 8192) {
    size_t b = (n + 255) / 256;
    b = b < 1 ? 1 : (b > cap ? cap : b);
    return (unsigned)b;
}

}  // namespace

hipError_t mlp_features(size_t gmax, const Groups g, const Cells c, const int64_t *sys_off,
                        const float *mu, const float *sd, float *X, DevStatus *st, hipStream_t s) {
    hipLaunchKernelGGL(k_features, dim3(grid_for(gmax)), dim3(256), 0, s, &st->n_groups_c, g, c,
                       sys_off, mu, sd, X);
    return hipGetLastError();
}

hipError_t mlp_infer(size_t n, const uint32_t *n_dev, const float *X, const float *P, float *y,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_infer, dim3(grid_for(n, 4096)), dim3(256), 0, s, n, n_dev, X, P, y);
    return hipGetLastError();
}

size_t mlp_train_blocks(size_t batch) { return (batch + kSB - 1) / kSB; }

hipError_t mlp_grad(size_t batch, const uint32_t *idx, const float *X, const float *T,
                    const float *P, float *gpart, float *lpart, float *grad, float *loss,
                    hipStream_t s) {
    const size_t nb = mlp_train_blocks(batch);
    const float inv = 1.0f / (float)batch;
    hipLaunchKernelGGL(k_mlp_train, dim3((unsigned)nb), dim3(kTT), 0, s, batch, idx, X, T, P, inv,
                       gpart, lpart);
    hipLaunchKernelGGL(k_mlp_reduce, dim3(grid_for(kMlpParams)), dim3(256), 0, s, nb, gpart, lpart,
                       inv, grad, loss);
    return hipGetLastError();
}

hipError_t mlp_adam(float *P, const float *grad, float *m, float *v, int step, float lr,
                    hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(kMlpParams)), dim3(256), 0, s, P, grad, m, v, lr, b1,
                       b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t pred_caps(size_t gmax, const float *y, float margin, uint32_t cap_max, uint32_t *cap,
                     DevStatus *st, hipStream_t s) {
    hipLaunchKernelGGL(k_pred_caps, dim3(grid_for(gmax)), dim3(256), 0, s, &st->n_groups_c, y,
                       margin, cap_max, cap);
    return hipGetLastError();
}

hipError_t ovf_caps(size_t gmax, const uint32_t *nsel, const uint32_t *sel, const uint32_t *cnt_e,
                    const uint32_t *cnt_s, uint32_t *ocap, hipStream_t s) {
    hipLaunchKernelGGL(k_ovf_caps, dim3(grid_for(gmax)), dim3(256), 0, s, nsel, sel, cnt_e, cnt_s,
                       ocap);
    return hipGetLastError();
}

hipError_t ovf_seg(size_t gmax, const uint32_t *nsel, const uint32_t *sel, const uint32_t *ocap,
                   const uint64_t *ooff, const uint64_t *base_total, uint64_t *seg, uint32_t *cap,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_ovf_seg, dim3(grid_for(gmax)), dim3(256), 0, s, nsel, sel, ocap, ooff,
                       base_total, seg, cap);
    return hipGetLastError();
}

}  // namespace fdx
