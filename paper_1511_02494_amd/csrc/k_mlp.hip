// Learned selector: MLP 12 -> 64 -> 64 -> 6 in FP32 (inference and training).
//
// Inference fixes the order of every operation so that its outputs are
// reproducible bit for bit on any implementation that follows it:
//   g_k = plog2(1 + f_k) (k < 8) or f_k, plog2(v) = (e - 1) + (2m - 1) for
//   (m, e) = frexp(v);  z_k = fl32(fl32(fl32(g_k) - mu_k) * rho_k);
//   each unit: acc = 0; acc = fl32(acc + fl32(w_k * in_k)) in input order;
//   out = fl32(acc + b); ReLU on hidden units (v > 0 ? v : +0).
// Decision: infeasible variants skipped, first maximal logit wins,
// margin = fl32(top1 - top2) (+inf with one feasible variant), fallback when
// margin < tau or some |z_k| > 8.
//
// Training: one workgroup runs a whole minibatch (forward, masked softmax
// cross-entropy, backward); every output element is summed by one thread in
// a fixed order, so gradients are deterministic.
#include <math.h>

#include "dev.h"
#include "feat_acc.h"
#include "internal.h"

namespace spmvsel {

namespace {
constexpr int D0 = 12, D1 = 64, D2 = 64, D3 = 6;
constexpr int OW1 = 0, OB1 = OW1 + D1 * D0, OW2 = OB1 + D1, OB2 = OW2 + D2 * D1,
              OW3 = OB2 + D2, OB3 = OW3 + D3 * D2, NP = OB3 + D3;
static_assert(NP == 5382, "parameter count");

struct Feat12 {
    double f[12];
};

}  // namespace

using feat::plog2;

// The network and decision for features f (LDS or registers), 64 threads.
__device__ __forceinline__ void mlp_infer_body(const float *__restrict__ P,
                                               const float *__restrict__ norm, const double *f,
                                               uint32_t feas, float tau, float *__restrict__ out) {
    __shared__ float z[D0], h1[D1], h2[D2], lg[D3];
    const int t = threadIdx.x;
    if (t < D0) {
        const double g = t < 8 ? plog2(1.0 + f[t]) : f[t];
        z[t] = __fmul_rn(__fsub_rn((float)g, norm[t]), norm[D0 + t]);
    }
    __syncthreads();
    {
        float acc = 0.f;
        for (int k = 0; k < D0; ++k) acc = __fadd_rn(acc, __fmul_rn(P[OW1 + t * D0 + k], z[k]));
        const float v = __fadd_rn(acc, P[OB1 + t]);
        h1[t] = v > 0.f ? v : 0.f;
    }
    __syncthreads();
    {
        float acc = 0.f;
        for (int k = 0; k < D1; ++k) acc = __fadd_rn(acc, __fmul_rn(P[OW2 + t * D1 + k], h1[k]));
        const float v = __fadd_rn(acc, P[OB2 + t]);
        h2[t] = v > 0.f ? v : 0.f;
    }
    __syncthreads();
    if (t < D3) {
        float acc = 0.f;
        for (int k = 0; k < D2; ++k) acc = __fadd_rn(acc, __fmul_rn(P[OW3 + t * D2 + k], h2[k]));
        lg[t] = __fadd_rn(acc, P[OB3 + t]);
    }
    __syncthreads();
    if (t == 0) {
        int best = -1, second = -1;
        for (int v = 0; v < D3; ++v) {
            if (!((feas >> v) & 1u)) continue;
            if (best < 0 || lg[v] > lg[best]) {
                second = best;
                best = v;
            } else if (second < 0 || lg[v] > lg[second]) {
                second = v;
            }
        }
        float margin = 0.f;
        bool fb = true;
        if (best >= 0) {
            margin = second >= 0 ? __fsub_rn(lg[best], lg[second]) : __int_as_float(0x7f800000);
            bool ood = false;
            for (int k = 0; k < D0; ++k) ood = ood || fabsf(z[k]) > 8.0f;
            fb = margin < tau || ood;
        }
        out[0] = __int_as_float(best);
        out[1] = margin;
        out[2] = fb ? 1.f : 0.f;
        for (int v = 0; v < D3; ++v) out[3 + v] = lg[v];
        for (int k = 0; k < D0; ++k) out[9 + k] = z[k];
    }
}

__global__ __launch_bounds__(64) void k_mlp_infer(const float *__restrict__ P,
                                                  const float *__restrict__ norm, Feat12 F,
                                                  uint32_t feas, float tau, float *__restrict__ out) {
    mlp_infer_body(P, norm, F.f, feas, tau, out);
}

// ---------------------------------------------------------------- selection in one pass
// partials: the nparts partial records of the one-pass selection kernel
// (feature sums, and the delta16 block spans in words 12 (height H0) and 13
// (H1; meaningful when two_heights)); feas_base: the variants feasible
// whatever the spans.  out (kRecBytes, pinned host memory or device): the
// inference record of k_mlp_infer in floats 0..31, then the common part
// (feasibility bits, features, reduced record; see select_store_common).
__global__ __launch_bounds__(64) void k_mlp_select(const float *__restrict__ P,
                                                   const float *__restrict__ norm,
                                                   const uint64_t *__restrict__ partials,
                                                   int nparts, int64_t n, int64_t m, int64_t nnz,
                                                   int vb, int xb, int two_heights,
                                                   uint32_t feas_base, float tau,
                                                   float *__restrict__ out) {
    __shared__ uint64_t w[16];
    __shared__ double f[12];
    __shared__ uint32_t feas;
    feat::select_prologue(nparts, partials, n, m, nnz, vb, xb, two_heights, feas_base, w, f, &feas);
    if (threadIdx.x == 0) feat::select_store_common(reinterpret_cast<char *>(out), f, feas, w);
    mlp_infer_body(P, norm, f, feas, tau, out);
}

hipError_t launch_mlp_select(const float *d_params, const float *d_norm, const uint64_t *d_partials,
                             int nparts, int64_t n, int64_t m, int64_t nnz, int vb, int xb,
                             int two_heights, uint32_t feas_base, float tau, float *out,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_select, dim3(1), dim3(64), 0, s, d_params, d_norm, d_partials, nparts,
                       n, m, nnz, vb, xb, two_heights, feas_base, tau, out);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const float *d_params, const float *d_norm, const double *feats,
                            uint32_t feasible, float tau, float *d_out, hipStream_t s) {
    Feat12 F;
    for (int i = 0; i < 12; ++i) F.f[i] = feats[i];
    hipLaunchKernelGGL(k_mlp_infer, dim3(1), dim3(64), 0, s, d_params, d_norm, F, feasible, tau,
                       d_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- training
constexpr int kTrainThreads = 1024;

// workspace (floats): a1[B*64], a2[B*64], dl[B*6], da2[B*64], da1[B*64], lb[B]
// Loss per sample: -log of the softmax mass of its target set A (feasible
// logits only): A = {lab[b]} (cross-entropy) when accept is null, else the
// feasible variants with accept[b*6+j] != 0 (every variant close enough to
// the fastest).  d loss / d logit_j = p_j - p_j [j in A] / sum_A p.
__global__ __launch_bounds__(kTrainThreads) void k_mlp_fwd_bwd(
    const float *__restrict__ P, const float *__restrict__ Z, const int32_t *__restrict__ lab,
    const uint8_t *__restrict__ accept, const uint8_t *__restrict__ mask, int B,
    float *__restrict__ G, float *__restrict__ loss, float *__restrict__ ws) {
    float *a1 = ws, *a2 = a1 + B * D1, *dl = a2 + B * D2, *da2 = dl + B * D3, *da1 = da2 + B * D2,
          *lb = da1 + B * D1;
    const int t = threadIdx.x;
    // forward
    for (int q = t; q < B * D1; q += kTrainThreads) {
        const int b = q / D1, j = q % D1;
        float acc = P[OB1 + j];
        for (int k = 0; k < D0; ++k) acc += P[OW1 + j * D0 + k] * Z[b * D0 + k];
        a1[q] = acc;
    }
    __syncthreads();
    for (int q = t; q < B * D2; q += kTrainThreads) {
        const int b = q / D2, j = q % D2;
        float acc = P[OB2 + j];
        for (int k = 0; k < D1; ++k) acc += P[OW2 + j * D1 + k] * fmaxf(a1[b * D1 + k], 0.f);
        a2[q] = acc;
    }
    __syncthreads();
    for (int b = t; b < B; b += kTrainThreads) {
        float lg[D3];
        float mx = -INFINITY;
        for (int j = 0; j < D3; ++j) {
            float acc = P[OB3 + j];
            for (int k = 0; k < D2; ++k) acc += P[OW3 + j * D2 + k] * fmaxf(a2[b * D2 + k], 0.f);
            lg[j] = acc;
            if (mask[b * D3 + j] && acc > mx) mx = acc;
        }
        float se = 0.f, sa = 0.f;
        bool in[D3];
        for (int j = 0; j < D3; ++j) {
            const float e = mask[b * D3 + j] ? expf(lg[j] - mx) : 0.f;
            in[j] = accept ? accept[b * D3 + j] != 0 && mask[b * D3 + j] : j == lab[b];
            se += e;
            sa += in[j] ? e : 0.f;
        }
        lb[b] = -(logf(sa) - logf(se));
        for (int j = 0; j < D3; ++j) {
            const float e = mask[b * D3 + j] ? expf(lg[j] - mx) : 0.f;
            const float sm = e / se;
            dl[b * D3 + j] = (sm - (in[j] ? e / sa : 0.f)) / (float)B;
        }
    }
    __syncthreads();
    // backward through layer 3 and 2
    for (int q = t; q < B * D2; q += kTrainThreads) {
        const int b = q / D2, k = q % D2;
        float acc = 0.f;
        for (int j = 0; j < D3; ++j) acc += dl[b * D3 + j] * P[OW3 + j * D2 + k];
        da2[q] = a2[q] > 0.f ? acc : 0.f;
    }
    __syncthreads();
    for (int q = t; q < B * D1; q += kTrainThreads) {
        const int b = q / D1, k = q % D1;
        float acc = 0.f;
        for (int j = 0; j < D2; ++j) acc += da2[b * D2 + j] * P[OW2 + j * D1 + k];
        da1[q] = a1[q] > 0.f ? acc : 0.f;
    }
    __syncthreads();
    // parameter gradients: sums over the batch in sample order
    for (int q = t; q < NP; q += kTrainThreads) {
        float acc = 0.f;
        if (q < OB1) {
            const int j = q / D0, k = q % D0;
            for (int b = 0; b < B; ++b) acc += da1[b * D1 + j] * Z[b * D0 + k];
        } else if (q < OW2) {
            const int j = q - OB1;
            for (int b = 0; b < B; ++b) acc += da1[b * D1 + j];
        } else if (q < OB2) {
            const int j = (q - OW2) / D1, k = (q - OW2) % D1;
            for (int b = 0; b < B; ++b) acc += da2[b * D2 + j] * fmaxf(a1[b * D1 + k], 0.f);
        } else if (q < OW3) {
            const int j = q - OB2;
            for (int b = 0; b < B; ++b) acc += da2[b * D2 + j];
        } else if (q < OB3) {
            const int j = (q - OW3) / D2, k = (q - OW3) % D2;
            for (int b = 0; b < B; ++b) acc += dl[b * D3 + j] * fmaxf(a2[b * D2 + k], 0.f);
        } else {
            const int j = q - OB3;
            for (int b = 0; b < B; ++b) acc += dl[b * D3 + j];
        }
        G[q] = acc;
    }
    if (t == 0) {
        float s = 0.f;
        for (int b = 0; b < B; ++b) s += lb[b];
        loss[0] = s / (float)B;
    }
}

hipError_t launch_mlp_fwd_bwd(const float *params, const float *Z, const int32_t *labels,
                              const uint8_t *accept, const uint8_t *mask, int B, float *grads,
                              float *loss, hipStream_t s) {
    static float *ws[64] = {nullptr};  // per-device workspace for B <= 1024
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (!ws[dev]) {
        e = hipMalloc(&ws[dev], (size_t)1024 * (4 * 64 + 6 + 1) * sizeof(float));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3(1), dim3(kTrainThreads), 0, s, params, Z, labels, accept,
                       mask, B, grads, loss, ws[dev]);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_adam(float *__restrict__ p, const float *__restrict__ g,
                                                 float *__restrict__ m, float *__restrict__ v,
                                                 int n, float lr, float b1, float b2, float eps,
                                                 float c1, float c2) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_mlp_adam(float *p, const float *g, float *m, float *v, int n, int step, float lr,
                           float b1, float b2, float eps, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const float c1 = (float)(1.0 - pow((double)b1, step));
    const float c2 = (float)(1.0 - pow((double)b2, step));
    hipLaunchKernelGGL(k_adam, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, p, g, m, v, n,
                       lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace spmvsel
