// Learned preconditioner: a per-|G+k|-shell network (3 -> 64 -> 64 -> 1, tanh) that
// scales the paper's M(G) by exp(f) inside the folded CG, with hand-written
// FP32 inference, loss/gradient and Adam kernels, and the kernels that turn solver
// snapshots into training tables.
//
//   x_si = (T_s / Ecut, T_i / Ecut, E_ref / Ecut)
//   h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), r = W3 h2 + b3, f = 8 tanh(r / 8)
//   loss (per band, per snapshot): 1 - sum_s w A / (sqrt(sum_s w^2 B) sqrt(E)), w = exp(f)
// with A_si = sum_{G in s} Re(conj e_i . K0 g_i), B_si = sum_{G in s} |K0 g_i|^2,
// E_i = ||e_i||^2, e_i = (I - Psi* Psi*^H) psi_i the band's error outside the converged
// subspace (the CG steps along -K g, so K g should point along e).  Parameters:
// W1[64][3], b1[64], W2[64][64], b2[64], W3[64], b3 (4481 floats).
#include "kernels.h"

namespace pw {

constexpr int MH = 64;
constexpr int NPAR = MH * 3 + MH + MH * MH + MH + MH + 1;
constexpr int OW1 = 0, OB1 = OW1 + MH * 3, OW2 = OB1 + MH, OB2 = OW2 + MH * MH, OW3 = OB2 + MH, OB3 = OW3 + MH;

__device__ inline void load_params(float *s, const float *__restrict__ w) {
    for (int i = threadIdx.x; i < NPAR; i += blockDim.x) s[i] = w[i];
    __syncthreads();
}

// forward for one input; h1, h2 returned for the backward pass
__device__ inline float mlp_forward(const float *P, const float x[3], float h1[MH], float h2[MH], float &t) {
#pragma unroll 8
    for (int o = 0; o < MH; ++o)
        h1[o] = tanhf(P[OW1 + 3 * o] * x[0] + P[OW1 + 3 * o + 1] * x[1] + P[OW1 + 3 * o + 2] * x[2] + P[OB1 + o]);
    float r = P[OB3];
    for (int o = 0; o < MH; ++o) {
        float a = P[OB2 + o];
#pragma unroll 16
        for (int i = 0; i < MH; ++i) a += P[OW2 + MH * o + i] * h1[i];
        h2[o] = tanhf(a);
        r += P[OW3 + o] * h2[o];
    }
    t = tanhf(r * 0.125f);
    return 8.0f * t;
}

// the same forward without the hidden states (inference): h1 indexed only by
// unrolled constants stays in registers; sums in the order of mlp_forward
__device__ inline float mlp_eval(const float *P, const float x[3]) {
    float h1[MH];
#pragma unroll
    for (int o = 0; o < MH; ++o)
        h1[o] = tanhf(P[OW1 + 3 * o] * x[0] + P[OW1 + 3 * o + 1] * x[1] + P[OW1 + 3 * o + 2] * x[2] + P[OB1 + o]);
    float r = P[OB3];
#pragma unroll 1
    for (int o = 0; o < MH; ++o) {
        const float *w2 = P + OW2 + MH * o;
        float a = P[OB2 + o];
#pragma unroll
        for (int i = 0; i < MH; ++i) a += w2[i] * h1[i];
        r += P[OW3 + o] * tanhf(a);
    }
    return 8.0f * tanhf(r * 0.125f);
}

// f[s][i] for one snapshot (inference inside the solver)
__global__ __launch_bounds__(256) void k_mlp_infer(int nshell, int nb, const double *__restrict__ shell_t,
                                                   const double *__restrict__ tband, double e_ref, double ecut,
                                                   const float *__restrict__ w, float *__restrict__ f) {
    __shared__ float P[NPAR];
    load_params(P, w);
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nshell * nb) return;
    const int s = idx / nb, i = idx - s * nb;
    const float x[3] = {(float)(shell_t[s] / ecut), (float)(tband[i] / ecut), (float)(e_ref / ecut)};
    f[idx] = mlp_eval(P, x);
}

void mlp_infer(int nshell, int nb, const double *shell_t, const double *tband, double e_ref, double ecut,
               const float *w, float *f, hipStream_t st) {
    const int n = nshell * nb;
    hipLaunchKernelGGL(k_mlp_infer, dim3((n + 255) / 256), dim3(256), 0, st, nshell, nb, shell_t, tband, e_ref,
                       ecut, w, f);
    PW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// training.  Tables of snapshot k: tabs[k][0][s][i] = A, [1] = B, [2] = C with
// E_i = sum_s C_si.  Pass 1: per (k, i) the sums u = sum_s w A, q = sum_s w^2 B,
// E and the band loss.  Pass 2: per sample dL/dr and the weight gradients,
// reduced inside each workgroup by small GEMMs over 64-sample sub-batches.
// Pass 3: fixed-order sum of the workgroup partials.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_bandsums(int nshell, int nb, const double *__restrict__ shell_t,
                                                      const double *__restrict__ tband,
                                                      const double *__restrict__ e_ref, double ecut,
                                                      const double *__restrict__ tabs, const float *__restrict__ w,
                                                      double *__restrict__ sums) {
    __shared__ float P[NPAR];
    __shared__ double red[3][256];
    load_params(P, w);
    const int i = blockIdx.x, k = blockIdx.y;
    const double *A = tabs + (int64_t)k * 3 * nshell * nb;
    const double *B = A + (int64_t)nshell * nb;
    const double *Cc = B + (int64_t)nshell * nb;
    double u = 0, q = 0, e = 0;
    const float xt = (float)(tband[(int64_t)k * nb + i] / ecut), xe = (float)(e_ref[k] / ecut);
    for (int s = threadIdx.x; s < nshell; s += blockDim.x) {
        const float x[3] = {(float)(shell_t[s] / ecut), xt, xe};
        float h1[MH], h2[MH], t;
        const double wf = exp((double)mlp_forward(P, x, h1, h2, t));
        const int64_t o = (int64_t)s * nb + i;
        u += wf * A[o];
        q += wf * wf * B[o];
        e += Cc[o];
    }
    red[0][threadIdx.x] = u;
    red[1][threadIdx.x] = q;
    red[2][threadIdx.x] = e;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *o = sums + ((int64_t)k * nb + i) * 4;
        o[0] = red[0][0];
        o[1] = red[1][0];
        o[2] = red[2][0];
        const double den = sqrt(red[1][0]) * sqrt(red[2][0]);
        o[3] = den > 0 ? 1.0 - red[0][0] / den : 0.0;    // band loss
    }
}

constexpr int SB = 64;    // samples per sub-batch (one wave)

__global__ __launch_bounds__(64) void k_mlp_backward(int nshell, int nb, int nsnap, const double *__restrict__ shell_t,
                                                     const double *__restrict__ tband,
                                                     const double *__restrict__ e_ref, double ecut,
                                                     const double *__restrict__ tabs, const float *__restrict__ w,
                                                     const double *__restrict__ sums, int64_t chunk,
                                                     float *__restrict__ partial) {
    extern __shared__ unsigned char smem_raw[];
    float *P = reinterpret_cast<float *>(smem_raw);
    float *sh1 = P + NPAR + 3;              // [SB][MH]
    float *sd2 = sh1 + SB * MH;             // [SB][MH]
    float *sd1 = sd2 + SB * MH;             // [SB][MH]
    float *sh2 = sd1 + SB * MH;             // [SB][MH]
    float *sx = sh2 + SB * MH;              // [SB][3]
    float *sd3 = sx + SB * 3;               // [SB]
    load_params(P, w);
    const int lane = threadIdx.x;
    const int64_t nsamp = (int64_t)nsnap * nb * nshell;
    const int64_t s0 = (int64_t)blockIdx.x * chunk;
    const int64_t s1 = min(nsamp, s0 + chunk);
    const double inv_nk = 1.0 / ((double)nsnap * nb);
    // per-thread gradient accumulators: W2 row `lane` (64), W1 row `lane` (3), b1, b2, W3 entries `lane`
    float gw2[MH], gw1[3] = {0, 0, 0}, gb1 = 0, gb2 = 0, gw3 = 0, gb3 = 0;
#pragma unroll
    for (int j = 0; j < MH; ++j) gw2[j] = 0;
    for (int64_t base = s0; base < s1; base += SB) {
        const int64_t smp = base + lane;
        float x[3] = {0, 0, 0}, h1[MH], h2[MH], d3 = 0.0f;
        if (smp < s1) {
            // sample order: (k, i, s) with s fastest
            const int s = (int)(smp % nshell);
            const int64_t ki = smp / nshell;
            const int i = (int)(ki % nb), k = (int)(ki / nb);
            x[0] = (float)(shell_t[s] / ecut);
            x[1] = (float)(tband[(int64_t)k * nb + i] / ecut);
            x[2] = (float)(e_ref[k] / ecut);
            float t;
            const float f = mlp_forward(P, x, h1, h2, t);
            const double wf = exp((double)f);
            const double *sm = sums + ((int64_t)k * nb + i) * 4;
            const double u = sm[0], q = sm[1], E = sm[2];
            const double n = sqrt(q), se = sqrt(E);
            const int64_t o = (int64_t)k * 3 * nshell * nb + (int64_t)s * nb + i;
            const double a = tabs[o], b = tabs[o + (int64_t)nshell * nb];
            double dldw = 0.0;
            if (n > 0 && se > 0) dldw = (-a / (n * se) + u * wf * b / (n * n * n * se)) * inv_nk;
            d3 = (float)(dldw * wf) * (1.0f - t * t);
        } else {
#pragma unroll
            for (int j = 0; j < MH; ++j) { h1[j] = 0; h2[j] = 0; }
        }
        // backward to the hidden layers
        float d2[MH];
#pragma unroll
        for (int o = 0; o < MH; ++o) d2[o] = d3 * P[OW3 + o] * (1.0f - h2[o] * h2[o]);
        for (int j = 0; j < MH; ++j) {
            float a = 0.0f;
#pragma unroll 16
            for (int o = 0; o < MH; ++o) a += d2[o] * P[OW2 + MH * o + j];
            sd1[lane * MH + j] = a * (1.0f - h1[j] * h1[j]);
        }
#pragma unroll
        for (int j = 0; j < MH; ++j) {
            sh1[lane * MH + j] = h1[j];
            sd2[lane * MH + j] = d2[j];
            sh2[lane * MH + j] = h2[j];
        }
        sx[lane * 3 + 0] = x[0];
        sx[lane * 3 + 1] = x[1];
        sx[lane * 3 + 2] = x[2];
        sd3[lane] = d3;
        __syncthreads();
        // reduce the sub-batch: thread `lane` owns output unit o = lane
        const int o = lane;
        for (int n = 0; n < SB; ++n) {
            const float dn = sd2[n * MH + o];
#pragma unroll 16
            for (int j = 0; j < MH; ++j) gw2[j] += dn * sh1[n * MH + j];
            gb2 += dn;
            const float d1n = sd1[n * MH + o];
            gw1[0] += d1n * sx[n * 3 + 0];
            gw1[1] += d1n * sx[n * 3 + 1];
            gw1[2] += d1n * sx[n * 3 + 2];
            gb1 += d1n;
            gw3 += sd3[n] * sh2[n * MH + o];
            if (o == 0) gb3 += sd3[n];
        }
        __syncthreads();
    }
    float *out = partial + (int64_t)blockIdx.x * NPAR;
    const int o = lane;
    for (int j = 0; j < MH; ++j) out[OW2 + MH * o + j] = gw2[j];
    out[OW1 + 3 * o] = gw1[0];
    out[OW1 + 3 * o + 1] = gw1[1];
    out[OW1 + 3 * o + 2] = gw1[2];
    out[OB1 + o] = gb1;
    out[OB2 + o] = gb2;
    out[OW3 + o] = gw3;
    if (o == 0) out[OB3] = gb3;
}

// grad = sum over workgroups (fixed order); loss = mean band loss
__global__ void k_mlp_reduce(int nwg, const float *__restrict__ partial, int nk, const double *__restrict__ sums,
                             float *__restrict__ grad, float *__restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < NPAR) {
        double s = 0;
        for (int g = 0; g < nwg; ++g) s += partial[(int64_t)g * NPAR + p];
        grad[p] = (float)s;
    }
    if (p == 0 && loss) {
        double l = 0;
        for (int k = 0; k < nk; ++k) l += sums[4 * k + 3];
        loss[0] = (float)(l / nk);
    }
}

__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPAR) return;
    const float gg = g[p];
    const float mm = b1 * m[p] + (1.0f - b1) * gg;
    const float vv = b2 * v[p] + (1.0f - b2) * gg * gg;
    m[p] = mm;
    v[p] = vv;
    w[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

constexpr int kTrainWG = 512;

size_t mlp_work_bytes(int nshell, int nb, int nsnap) {
    return (size_t)nsnap * nb * 4 * sizeof(double) + (size_t)kTrainWG * NPAR * sizeof(float) + 256;
}

void mlp_loss_grad(int nshell, int nb, int nsnap, const double *shell_t, const double *tband, const double *e_ref,
                   double ecut, const double *tabs, const float *w, float *grad, float *loss, void *work,
                   hipStream_t st) {
    double *sums = (double *)work;
    float *partial = (float *)((char *)work + (size_t)nsnap * nb * 4 * sizeof(double));
    hipLaunchKernelGGL(k_mlp_bandsums, dim3(nb, nsnap), dim3(256), 0, st, nshell, nb, shell_t, tband, e_ref, ecut,
                       tabs, w, sums);
    PW_LAUNCH_CHECK();
    const int64_t nsamp = (int64_t)nsnap * nb * nshell;
    int64_t chunk = (nsamp + kTrainWG - 1) / kTrainWG;
    chunk = ((chunk + SB - 1) / SB) * SB;
    const int nwg = (int)((nsamp + chunk - 1) / chunk);
    const size_t lds = sizeof(float) * (NPAR + 3 + 4 * SB * MH + SB * 3 + SB);
    static size_t attr = 64 * 1024;
    if (lds > attr) {
        PW_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_mlp_backward),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr = lds;
    }
    hipLaunchKernelGGL(k_mlp_backward, dim3(nwg), dim3(64), lds, st, nshell, nb, nsnap, shell_t, tband, e_ref, ecut,
                       tabs, w, sums, chunk, partial);
    PW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NPAR + 255) / 256), dim3(256), 0, st, nwg, partial, nsnap * nb, sums,
                       grad, loss);
    PW_LAUNCH_CHECK();
}

void mlp_adam(float *w, const float *g, float *m, float *v, int step, float lr, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((NPAR + 255) / 256), dim3(256), 0, st, w, g, m, v, lr, b1, b2, 1e-8f, c1, c2);
    PW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// harvest: shell sums of one snapshot.  E = (I - P*) X (band-major, [nb][npw]),
// Z = K0 o g.  tabs[0][s][i] = sum Re(conj E . Z), [1] = sum |Z|^2, [2] = sum |E|^2,
// summed over the plane waves of shell s listed in shell_pw[shell_off[s] ..].
// delta >= 0: every sum of shell s is weighted by (T_s - e_ref)^2 + delta^2, the
// plane-wave diagonal of (H - E)^2 without the potential, so that the loss
// compares K g and E in that approximate A-norm instead of the Euclidean one.
// ---------------------------------------------------------------------------
__global__ void k_shell_tables(int nshell, int nb, int npw, const int32_t *__restrict__ shell_off,
                               const int32_t *__restrict__ shell_pw, const double2 *__restrict__ E,
                               const double2 *__restrict__ Z, int64_t ld, const double *__restrict__ shell_t,
                               double e_ref, double delta, double *__restrict__ tabs) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nshell * nb) return;
    const int s = (int)(idx / nb), i = (int)(idx % nb);
    double a = 0, b = 0, c = 0;
    for (int t = shell_off[s]; t < shell_off[s + 1]; ++t) {
        const int g = shell_pw[t];
        const double2 e = E[(int64_t)i * ld + g], z = Z[(int64_t)i * ld + g];
        a += e.x * z.x + e.y * z.y;
        b += z.x * z.x + z.y * z.y;
        c += e.x * e.x + e.y * e.y;
    }
    if (delta >= 0.0) {
        const double dt = shell_t[s] - e_ref, w = dt * dt + delta * delta;
        a *= w;
        b *= w;
        c *= w;
    }
    tabs[idx] = a;
    tabs[(int64_t)nshell * nb + idx] = b;
    tabs[2 * (int64_t)nshell * nb + idx] = c;
}

void shell_tables(int nshell, int nb, int npw, const int32_t *shell_off, const int32_t *shell_pw, const void *E,
                  const void *Z, int64_t ld, const double *shell_t, double e_ref, double delta, double *tabs,
                  hipStream_t st) {
    const int64_t n = (int64_t)nshell * nb;
    hipLaunchKernelGGL(k_shell_tables, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, nshell, nb, npw, shell_off,
                       shell_pw, (const double2 *)E, (const double2 *)Z, ld, shell_t, e_ref, delta, tabs);
    PW_LAUNCH_CHECK();
}

int mlp_nparam() { return NPAR; }

}  // namespace pw
