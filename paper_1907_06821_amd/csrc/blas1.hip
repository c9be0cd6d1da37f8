// Band-wise vector kernels of the folded-spectrum CG: fused gradient and
// preconditioner, conjugation, line-search inner products, per-band updates and
// residual norms.  All blocks are band-major complex128 [nb][ld]; every
// reduction is two-stage (per-workgroup partials, then a fixed-order sum), so
// results do not depend on scheduling.
#include "kernels.h"

namespace pw {

constexpr int RT = 256;          // threads per reduction workgroup
constexpr int RCHUNK = RT * 8;   // plane waves per reduction workgroup

int band_splits(int npw) { return (npw + RCHUNK - 1) / RCHUNK; }

// kVec plane waves per thread, strided by the workgroup so that each load stays
// coalesced, loads issued ahead of the stores
constexpr int kVec = 4;
inline dim3 vec_grid(int npw, int nb) { return dim3((unsigned)((npw + 256 * kVec - 1) / (256 * kVec)), nb); }


__device__ inline double tpa_k(double x) {
    // Teter-Payne-Allan kinetic preconditioner
    const double num = 27.0 + x * (18.0 + x * (12.0 + 8.0 * x));
    return num / (num + 16.0 * x * x * x * x);
}

__device__ inline double prec_weight(const PrecArgs &pa, int b, int g) {
    const double t = pa.kin[g];
    if (pa.kind == 0) {
        const double k = tpa_k(t / pa.tband[b]);
        return k * k;
    }
    // the paper's M(G); the learned preconditioner scales it by exp(f)
    const double d = t - pa.e_ref;
    double w = 1.0 / (d * d + pa.de2);
    if (pa.kind == 2) w *= exp((double)pa.ftab[(int64_t)pa.shell[g] * pa.nb + b]);
    return w;
}

template <int NQ>
__device__ inline void block_store(double (&acc)[NQ], double *partial, int nb, int nsplit, int b, int split) {
    __shared__ double red[NQ][RT];
#pragma unroll
    for (int q = 0; q < NQ; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = RT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) partial[((int64_t)q * nb + b) * nsplit + split] = red[q][0];
    }
}

// out[q * nb + b] = sum_split partial[q][b][split]
__device__ __forceinline__ void finish_body(int nsplit, const double *__restrict__ partial, double *__restrict__ out,
                                            int i) {
    double s = 0;
    for (int k = 0; k < nsplit; ++k) s += partial[(int64_t)i * nsplit + k];
    out[i] = s;
}

__global__ void finish_red(int nq, int nb, int nsplit, const double *__restrict__ partial, double *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nq * nb) finish_body(nsplit, partial, out, i);
}

static void finish(int nq, int nb, const BandRed &r, double *out, hipStream_t st) {
    hipLaunchKernelGGL(finish_red, dim3((nq * nb + 255) / 256), dim3(256), 0, st, nq, nb, r.nsplit, r.partial, out);
    PW_LAUNCH_CHECK();
}

// the plane waves of reduction workgroup `split` of band b (bodies below take
// (b, split) so that single and batched kernels share them)
#define BAND_LOOP(npw)                                                     \
    const int g0 = split * RCHUNK;                                         \
    const int g1 = min(npw, g0 + RCHUNK);                                  \
    for (int g = g0 + threadIdx.x; g < g1; g += RT)

// ---------------------------------------------------------------------------
__device__ __forceinline__ void mu_tband_body(int nb, int npw, const double2 *__restrict__ Y,
                                              const double2 *__restrict__ X, int64_t ld,
                                              const double *__restrict__ kin, double *partial, int nsplit, int b,
                                              int split) {
    double acc[2] = {0, 0};
    BAND_LOOP(npw) {
        const double2 y = Y[(int64_t)b * ld + g], x = X[(int64_t)b * ld + g];
        acc[0] += y.x * y.x + y.y * y.y;
        acc[1] += kin[g] * (x.x * x.x + x.y * x.y);
    }
    block_store<2>(acc, partial, nb, nsplit, b, split);
}

__global__ __launch_bounds__(RT) void k_mu_tband(int nb, int npw, const double2 *__restrict__ Y,
                                                 const double2 *__restrict__ X, int64_t ld,
                                                 const double *__restrict__ kin, double *partial, int nsplit) {
    mu_tband_body(nb, npw, Y, X, ld, kin, partial, nsplit, blockIdx.y, blockIdx.x);
}

void red_mu_tband(int nb, int npw, const void *Y, const void *X, int64_t ld, const double *kin, double *mu,
                  double *tband, BandRed r, hipStream_t st) {
    hipLaunchKernelGGL(k_mu_tband, dim3(r.nsplit, nb), dim3(RT), 0, st, nb, npw, (const double2 *)Y,
                       (const double2 *)X, ld, kin, r.partial, r.nsplit);
    PW_LAUNCH_CHECK();
    // mu -> out[0:nb], tband -> out[nb:2nb] requires contiguous outputs
    PW_CHECK(tband == mu + nb, PW_EINVAL, "mu and tband must be adjacent");
    finish(2, nb, r, mu, st);
}

// G = AX - mu X ; Z = K o G ; gz = Re<G, Z> ; gzo = Re<Gold, Z> ; Gold <- G
__device__ __forceinline__ void grad_body(int nb, int npw, const double2 *__restrict__ X,
                                          const double2 *__restrict__ AX, double2 *__restrict__ Gold,
                                          double2 *__restrict__ Z, int64_t ld, const double *__restrict__ mu,
                                          const PrecArgs &pa, double *partial, int nsplit, int b, int split) {
    double acc[2] = {0, 0};
    const int g0 = split * RCHUNK, g1 = min(npw, g0 + RCHUNK);
    const double m = mu[b];
    // four plane waves per pass, their loads ahead of the arithmetic (the sums keep
    // the order of one plane wave at a time)
    for (int gb = g0 + threadIdx.x; gb < g1; gb += RT * 4) {
        double2 x[4], ax[4], go[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int g = gb + RT * j;
            if (g < g1) {
                const int64_t i = (int64_t)b * ld + g;
                x[j] = X[i];
                ax[j] = AX[i];
                go[j] = Gold[i];
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int g = gb + RT * j;
            if (g < g1) {
                const int64_t i = (int64_t)b * ld + g;
                const double2 gr = make_double2(ax[j].x - m * x[j].x, ax[j].y - m * x[j].y);
                const double w = prec_weight(pa, b, g);
                const double2 z = make_double2(w * gr.x, w * gr.y);
                acc[0] += gr.x * z.x + gr.y * z.y;
                acc[1] += go[j].x * z.x + go[j].y * z.y;
                Gold[i] = gr;
                Z[i] = z;
            }
        }
    }
    block_store<2>(acc, partial, nb, nsplit, b, split);
}

__global__ __launch_bounds__(RT) void k_grad(int nb, int npw, const double2 *__restrict__ X,
                                             const double2 *__restrict__ AX, double2 *__restrict__ Gold,
                                             double2 *__restrict__ Z, int64_t ld, const double *__restrict__ mu,
                                             PrecArgs pa, double *partial, int nsplit) {
    grad_body(nb, npw, X, AX, Gold, Z, ld, mu, pa, partial, nsplit, blockIdx.y, blockIdx.x);
}

void red_grad(int nb, int npw, const void *X, const void *AX, void *Gold, void *Z, int64_t ld, const double *mu,
              PrecArgs pa, double *gz, double *gzo, BandRed r, hipStream_t st) {
    hipLaunchKernelGGL(k_grad, dim3(r.nsplit, nb), dim3(RT), 0, st, nb, npw, (const double2 *)X,
                       (const double2 *)AX, (double2 *)Gold, (double2 *)Z, ld, mu, pa, r.partial, r.nsplit);
    PW_LAUNCH_CHECK();
    PW_CHECK(gzo == gz + nb, PW_EINVAL, "gz and gzo must be adjacent");
    finish(2, nb, r, gz, st);
}

__device__ __forceinline__ void gzold_body(int nb, int npw, const double2 *__restrict__ G, int64_t ld,
                                           const PrecArgs &pa, double *partial, int nsplit, int b, int split) {
    double acc[1] = {0};
    BAND_LOOP(npw) {
        const double2 v = G[(int64_t)b * ld + g];
        acc[0] += prec_weight(pa, b, g) * (v.x * v.x + v.y * v.y);
    }
    block_store<1>(acc, partial, nb, nsplit, b, split);
}

__global__ __launch_bounds__(RT) void k_gzold(int nb, int npw, const double2 *__restrict__ G, int64_t ld,
                                              PrecArgs pa, double *partial, int nsplit) {
    gzold_body(nb, npw, G, ld, pa, partial, nsplit, blockIdx.y, blockIdx.x);
}

void red_gzold(int nb, int npw, const void *G, int64_t ld, PrecArgs pa, double *gz_old, BandRed r, hipStream_t st) {
    hipLaunchKernelGGL(k_gzold, dim3(r.nsplit, nb), dim3(RT), 0, st, nb, npw, (const double2 *)G, ld, pa,
                       r.partial, r.nsplit);
    PW_LAUNCH_CHECK();
    finish(1, nb, r, gz_old, st);
}

// P = -Z + beta P with Polak-Ribiere beta = max(0, (gz - gzo) / gz_old); the
// first workgroup of each band also stores gz as the next gz_old.
__device__ __forceinline__ void pupdate_body(int npw, const double2 *__restrict__ Z, double2 *__restrict__ P,
                                             int64_t ld, const double *__restrict__ gz,
                                             const double *__restrict__ gzo, const double *__restrict__ gz_old, int b,
                                             int g) {
    const double den = gz_old[b];
    double beta = den > 0.0 ? (gz[b] - gzo[b]) / den : 0.0;
    if (!(beta > 0.0)) beta = 0.0;
    if (g < npw) {
        const int64_t i = (int64_t)b * ld + g;
        const double2 z = Z[i], p = P[i];
        P[i] = make_double2(-z.x + beta * p.x, -z.y + beta * p.y);
    }
}

__global__ __launch_bounds__(256) void k_pupdate(int nb, int npw, const double2 *__restrict__ Z,
                                                 double2 *__restrict__ P, int64_t ld, const double *__restrict__ gz,
                                                 const double *__restrict__ gzo, double *__restrict__ gz_old) {
    const int g0 = blockIdx.x * 256 * kVec + threadIdx.x;
#pragma unroll
    for (int j = 0; j < kVec; ++j) pupdate_body(npw, Z, P, ld, gz, gzo, gz_old, blockIdx.y, g0 + 256 * j);
}

__global__ void k_store_gzold(int nb, const double *gz, double *gz_old) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) gz_old[b] = gz[b];
}

void pupdate(int nb, int npw, const void *Z, void *P, int64_t ld, const double *gz, const double *gzo,
             double *gz_old, hipStream_t st) {
    hipLaunchKernelGGL(k_pupdate, vec_grid(npw, nb), dim3(256), 0, st, nb, npw, (const double2 *)Z,
                       (double2 *)P, ld, gz, gzo, gz_old);
    PW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_store_gzold, dim3((nb + 255) / 256), dim3(256), 0, st, nb, gz, gz_old);
    PW_LAUNCH_CHECK();
}

// <Y, YP> (re, im), ||YP||^2, ||P||^2
__device__ __forceinline__ void line_body(int nb, int npw, const double2 *__restrict__ Y,
                                          const double2 *__restrict__ YP, const double2 *__restrict__ P, int64_t ld,
                                          double *partial, int nsplit, int b, int split) {
    double acc[4] = {0, 0, 0, 0};
    BAND_LOOP(npw) {
        const int64_t i = (int64_t)b * ld + g;
        const double2 y = Y[i], yp = YP[i], p = P[i];
        acc[0] += y.x * yp.x + y.y * yp.y;
        acc[1] += y.x * yp.y - y.y * yp.x;
        acc[2] += yp.x * yp.x + yp.y * yp.y;
        acc[3] += p.x * p.x + p.y * p.y;
    }
    block_store<4>(acc, partial, nb, nsplit, b, split);
}

__global__ __launch_bounds__(RT) void k_line(int nb, int npw, const double2 *__restrict__ Y,
                                             const double2 *__restrict__ YP, const double2 *__restrict__ P,
                                             int64_t ld, double *partial, int nsplit) {
    line_body(nb, npw, Y, YP, P, ld, partial, nsplit, blockIdx.y, blockIdx.x);
}

void red_line(int nb, int npw, const void *Y, const void *YP, const void *P, int64_t ld, double *out4, BandRed r,
              hipStream_t st) {
    hipLaunchKernelGGL(k_line, dim3(r.nsplit, nb), dim3(RT), 0, st, nb, npw, (const double2 *)Y,
                       (const double2 *)YP, (const double2 *)P, ld, r.partial, r.nsplit);
    PW_LAUNCH_CHECK();
    finish(4, nb, r, out4, st);
}

// Exact minimum of the Rayleigh quotient of A on span{psi, p} (p orthogonal to
// psi): lowest eigenvector of [[a11, a12], [conj a12, a22]] in the basis
// {psi, p/|p|}, computed without cancellation.  coef[b] = (alpha re, alpha im,
// beta re, beta im) with psi' = alpha psi + beta p.
__device__ __forceinline__ void line_coef_body(int nb, const double *__restrict__ mu, const double *__restrict__ l4,
                                               double *__restrict__ coef, int b) {
    const double pn2 = l4[3 * nb + b];
    double ar = 1, ai = 0, br = 0, bi = 0;
    if (pn2 > 0.0) {
        const double pn = sqrt(pn2);
        const double a11 = mu[b];
        const double cr = l4[b] / pn, ci = l4[nb + b] / pn;   // a12 = <Y, YP>/|p|
        const double a22 = l4[2 * nb + b] / pn2;
        const double d = 0.5 * (a22 - a11);
        const double r = sqrt(d * d + cr * cr + ci * ci);
        if (r > 0.0) {
            if (d >= 0) { ar = d + r; ai = 0; br = -cr; bi = ci; }          // (d + r, -conj a12)
            else { ar = cr; ai = ci; br = d - r; bi = 0; }                  // (a12, d - r)
            const double nrm = sqrt(ar * ar + ai * ai + br * br + bi * bi);
            ar /= nrm; ai /= nrm; br /= nrm * pn; bi /= nrm * pn;
        }
    }
    coef[4 * b + 0] = ar;
    coef[4 * b + 1] = ai;
    coef[4 * b + 2] = br;
    coef[4 * b + 3] = bi;
}

__global__ void k_line_coef(int nb, const double *__restrict__ mu, const double *__restrict__ l4,
                            double *__restrict__ coef) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) line_coef_body(nb, mu, l4, coef, b);
}

void line_coef(int nb, const double *mu, const double *l4, double *coef, hipStream_t st) {
    hipLaunchKernelGGL(k_line_coef, dim3((nb + 255) / 256), dim3(256), 0, st, nb, mu, l4, coef);
    PW_LAUNCH_CHECK();
}

__device__ inline double2 lin2(double2 a, double2 x, double2 b, double2 y) {
    return make_double2(a.x * x.x - a.y * x.y + b.x * y.x - b.y * y.y, a.x * x.y + a.y * x.x + b.x * y.y + b.y * y.x);
}

__device__ __forceinline__ void combine3_body(int npw, double2 *__restrict__ X, double2 *__restrict__ Y,
                                              double2 *__restrict__ AX, const double2 *__restrict__ P,
                                              const double2 *__restrict__ YP, const double2 *__restrict__ AP,
                                              int64_t ld, const double *__restrict__ coef, int b, int g) {
    if (g >= npw) return;
    const double2 al = make_double2(coef[4 * b], coef[4 * b + 1]);
    const double2 be = make_double2(coef[4 * b + 2], coef[4 * b + 3]);
    const int64_t i = (int64_t)b * ld + g;
    X[i] = lin2(al, X[i], be, P[i]);
    Y[i] = lin2(al, Y[i], be, YP[i]);
    AX[i] = lin2(al, AX[i], be, AP[i]);
}

__global__ __launch_bounds__(256) void k_combine3(int nb, int npw, double2 *__restrict__ X, double2 *__restrict__ Y,
                                                  double2 *__restrict__ AX, const double2 *__restrict__ P,
                                                  const double2 *__restrict__ YP, const double2 *__restrict__ AP,
                                                  int64_t ld, const double *__restrict__ coef) {
    const int g0 = blockIdx.x * 256 * kVec + threadIdx.x;
#pragma unroll
    for (int j = 0; j < kVec; ++j) combine3_body(npw, X, Y, AX, P, YP, AP, ld, coef, blockIdx.y, g0 + 256 * j);
}

void combine3(int nb, int npw, void *X, void *Y, void *AX, const void *P, const void *YP, const void *AP,
              int64_t ld, const double *coef, hipStream_t st) {
    hipLaunchKernelGGL(k_combine3, vec_grid(npw, nb), dim3(256), 0, st, nb, npw, (double2 *)X,
                       (double2 *)Y, (double2 *)AX, (const double2 *)P, (const double2 *)YP, (const double2 *)AP,
                       ld, coef);
    PW_LAUNCH_CHECK();
}

// res[b] = || Y_b - w_b X_b ||
__device__ __forceinline__ void resid_body(int nb, int npw, const double2 *__restrict__ Y,
                                           const double2 *__restrict__ X, int64_t ld, const double *__restrict__ w,
                                           double *partial, int nsplit, int b, int split) {
    double acc[1] = {0};
    BAND_LOOP(npw) {
        const int64_t i = (int64_t)b * ld + g;
        const double2 y = Y[i], x = X[i];
        const double wb = w[b];
        const double rx = y.x - wb * x.x, ry = y.y - wb * x.y;
        acc[0] += rx * rx + ry * ry;
    }
    block_store<1>(acc, partial, nb, nsplit, b, split);
}

__global__ __launch_bounds__(RT) void k_resid(int nb, int npw, const double2 *__restrict__ Y,
                                              const double2 *__restrict__ X, int64_t ld, const double *__restrict__ w,
                                              double *partial, int nsplit) {
    resid_body(nb, npw, Y, X, ld, w, partial, nsplit, blockIdx.y, blockIdx.x);
}

__global__ void k_sqrt(int n, double *x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = sqrt(x[i]);
}

void red_resid(int nb, int npw, const void *Y, const void *X, int64_t ld, const double *w, double *res, BandRed r,
               hipStream_t st) {
    hipLaunchKernelGGL(k_resid, dim3(r.nsplit, nb), dim3(RT), 0, st, nb, npw, (const double2 *)Y,
                       (const double2 *)X, ld, w, r.partial, r.nsplit);
    PW_LAUNCH_CHECK();
    finish(1, nb, r, res, st);
    hipLaunchKernelGGL(k_sqrt, dim3((nb + 255) / 256), dim3(256), 0, st, nb, res);
    PW_LAUNCH_CHECK();
}

__global__ __launch_bounds__(RT) void k_norm2(int nb, int npw, const double2 *__restrict__ X, int64_t ld,
                                              double *partial, int nsplit) {
    const int b = blockIdx.y, split = blockIdx.x;
    double acc[1] = {0};
    BAND_LOOP(npw) {
        const double2 x = X[(int64_t)b * ld + g];
        acc[0] += x.x * x.x + x.y * x.y;
    }
    block_store<1>(acc, partial, nb, nsplit, b, split);
}

void band_norms(int nb, int npw, const void *X, int64_t ld, double *out, BandRed r, hipStream_t st) {
    hipLaunchKernelGGL(k_norm2, dim3(r.nsplit, nb), dim3(RT), 0, st, nb, npw, (const double2 *)X, ld, r.partial,
                       r.nsplit);
    PW_LAUNCH_CHECK();
    finish(1, nb, r, out, st);
    hipLaunchKernelGGL(k_sqrt, dim3((nb + 255) / 256), dim3(256), 0, st, nb, out);
    PW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Batched band kernels: the problems of a batched folded-CG run (one BandProb
// each, all with nb bands) in one launch, blockIdx.y = problem x nb + band (or the
// problem alone); problems whose mask entry is 0 and workgroups beyond a problem's
// own extent return at once.  They run the bodies of the kernels above with each
// problem's arguments, so every problem's numbers are those of its own launches.
// ---------------------------------------------------------------------------
#define BATCH_BAND(nb)                                                     \
    const int q = blockIdx.y / (nb), b = blockIdx.y % (nb);               \
    if (!mask[q]) return;                                                  \
    const BandProb &p = probs[q];

__global__ __launch_bounds__(RT) void kb_mu_tband(const BandProb *__restrict__ probs, const int *__restrict__ mask,
                                                  int nb) {
    BATCH_BAND(nb)
    if ((int)blockIdx.x >= p.nsplit) return;
    mu_tband_body(nb, p.npw, p.blk[kBY], p.blk[kBX], p.ld, p.pa.kin, p.red, p.nsplit, b, blockIdx.x);
}

__global__ __launch_bounds__(RT) void kb_grad(const BandProb *__restrict__ probs, const int *__restrict__ mask,
                                              int nb) {
    BATCH_BAND(nb)
    if ((int)blockIdx.x >= p.nsplit) return;
    grad_body(nb, p.npw, p.blk[kBX], p.blk[kBAX], p.blk[kBG], p.blk[kBZ], p.ld, p.vec, p.pa, p.red, p.nsplit, b,
              blockIdx.x);
}

__global__ __launch_bounds__(RT) void kb_gzold(const BandProb *__restrict__ probs, const int *__restrict__ mask,
                                               int nb) {
    BATCH_BAND(nb)
    if ((int)blockIdx.x >= p.nsplit) return;
    gzold_body(nb, p.npw, p.blk[kBG], p.ld, p.pa, p.red, p.nsplit, b, blockIdx.x);
}

__global__ __launch_bounds__(RT) void kb_line(const BandProb *__restrict__ probs, const int *__restrict__ mask,
                                              int nb) {
    BATCH_BAND(nb)
    if ((int)blockIdx.x >= p.nsplit) return;
    line_body(nb, p.npw, p.blk[kBY], p.blk[kBYP], p.blk[kBP], p.ld, p.red, p.nsplit, b, blockIdx.x);
}

__global__ __launch_bounds__(RT) void kb_resid(const BandProb *__restrict__ probs, const int *__restrict__ mask,
                                               int nb, int iy, int ix) {
    BATCH_BAND(nb)
    if ((int)blockIdx.x >= p.nsplit) return;
    resid_body(nb, p.npw, p.blk[iy], p.blk[ix], p.ld, p.vec + 13 * nb, p.red, p.nsplit, b, blockIdx.x);
}

__global__ void kb_pupdate(const BandProb *__restrict__ probs, const int *__restrict__ mask, int nb) {
    BATCH_BAND(nb)
    pupdate_body(p.npw, p.blk[kBZ], p.blk[kBP], p.ld, p.vec + 2 * nb, p.vec + 3 * nb, p.vec + 4 * nb, b,
                 blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void kb_combine3(const BandProb *__restrict__ probs, const int *__restrict__ mask, int nb) {
    BATCH_BAND(nb)
    combine3_body(p.npw, p.blk[kBX], p.blk[kBY], p.blk[kBAX], p.blk[kBP], p.blk[kBYP], p.blk[kBAP], p.ld,
                  p.vec + 9 * nb, b, blockIdx.x * blockDim.x + threadIdx.x);
}

// blockIdx.y = problem: out = vec + off nb, nq quantities of nb bands
__global__ void kb_finish(const BandProb *__restrict__ probs, const int *__restrict__ mask, int nb, int nq, int off) {
    if (!mask[blockIdx.y]) return;
    const BandProb &p = probs[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nq * nb) finish_body(p.nsplit, p.red, p.vec + off * nb, i);
}

__global__ void kb_scalars(const BandProb *__restrict__ probs, const int *__restrict__ mask, int nb, int what) {
    if (!mask[blockIdx.y]) return;
    const BandProb &p = probs[blockIdx.y];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    if (what == 0) p.vec[4 * nb + b] = p.vec[2 * nb + b];                 // gz_old <- gz
    else if (what == 1) line_coef_body(nb, p.vec, p.vec + 5 * nb, p.vec + 9 * nb, b);
    else p.vec[14 * nb + b] = sqrt(p.vec[14 * nb + b]);                   // res <- sqrt(res)
}

// blk[dst[k]] <- blk[src[k]], k < n (blockIdx.z)
__global__ void kb_copy(const BandProb *__restrict__ probs, const int *__restrict__ mask, int nb, int4 src, int4 dst) {
    BATCH_BAND(nb)
    const int k = blockIdx.z;
    const int si = k == 0 ? src.x : k == 1 ? src.y : k == 2 ? src.z : src.w;
    const int di = k == 0 ? dst.x : k == 1 ? dst.y : k == 2 ? dst.z : dst.w;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < p.npw) p.blk[di][(int64_t)b * p.ld + g] = p.blk[si][(int64_t)b * p.ld + g];
}
__global__ void kb_save(const BandProb *__restrict__ probs, const int *__restrict__ mask, int nb) {
    BATCH_BAND(nb)
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < p.npw) p.psi[(int64_t)b * p.ldpsi + g] = p.blk[kBX][(int64_t)b * p.ld + g];
}
#undef BATCH_BAND

__global__ void kb_gather(const BandProb *__restrict__ probs, int nb, double *__restrict__ out,
                          int *__restrict__ sout) {
    const BandProb &p = probs[blockIdx.x];
    for (int i = threadIdx.x; i < 2 * nb; i += blockDim.x) out[(int64_t)blockIdx.x * 2 * nb + i] = p.vec[13 * nb + i];
    if (threadIdx.x < 8) sout[blockIdx.x * 8 + threadIdx.x] = p.status[threadIdx.x];
}

void band_batch_save(const BandProb *probs, const int *mask, int nprob, int nb, int maxnpw, hipStream_t st) {
    hipLaunchKernelGGL(kb_save, dim3((maxnpw + 255) / 256, nprob * nb), dim3(256), 0, st, probs, mask, nb);
    PW_LAUNCH_CHECK();
}

void band_batch_gather(const BandProb *probs, int nprob, int nb, double *out, int *sout, hipStream_t st) {
    hipLaunchKernelGGL(kb_gather, dim3(nprob), dim3(256), 0, st, probs, nb, out, sout);
    PW_LAUNCH_CHECK();
}

void band_batch(BandOp op, const BandProb *probs, const int *mask, int nprob, int nb, int maxsplit, int maxnpw,
                hipStream_t st, int a0, int a1) {
    const dim3 red(maxsplit, nprob * nb), vec((maxnpw + 255) / 256, nprob * nb);
    const dim3 fin((4 * nb + 255) / 256, nprob), sc((nb + 255) / 256, nprob);
    switch (op) {
        case BandOp::MuTband:
            hipLaunchKernelGGL(kb_mu_tband, red, dim3(RT), 0, st, probs, mask, nb);
            PW_LAUNCH_CHECK();
            hipLaunchKernelGGL(kb_finish, fin, dim3(256), 0, st, probs, mask, nb, 2, 0);   // mu, tband
            break;
        case BandOp::Grad:
            hipLaunchKernelGGL(kb_grad, red, dim3(RT), 0, st, probs, mask, nb);
            PW_LAUNCH_CHECK();
            hipLaunchKernelGGL(kb_finish, fin, dim3(256), 0, st, probs, mask, nb, 2, 2);   // gz, gzo
            break;
        case BandOp::GzOld:
            hipLaunchKernelGGL(kb_gzold, red, dim3(RT), 0, st, probs, mask, nb);
            PW_LAUNCH_CHECK();
            hipLaunchKernelGGL(kb_finish, fin, dim3(256), 0, st, probs, mask, nb, 1, 4);   // gz_old
            break;
        case BandOp::PUpdate:
            hipLaunchKernelGGL(kb_pupdate, vec, dim3(256), 0, st, probs, mask, nb);
            PW_LAUNCH_CHECK();
            hipLaunchKernelGGL(kb_scalars, sc, dim3(256), 0, st, probs, mask, nb, 0);
            break;
        case BandOp::Line:
            hipLaunchKernelGGL(kb_line, red, dim3(RT), 0, st, probs, mask, nb);
            PW_LAUNCH_CHECK();
            hipLaunchKernelGGL(kb_finish, fin, dim3(256), 0, st, probs, mask, nb, 4, 5);   // line4
            PW_LAUNCH_CHECK();
            hipLaunchKernelGGL(kb_scalars, sc, dim3(256), 0, st, probs, mask, nb, 1);       // coef
            break;
        case BandOp::Combine3:
            hipLaunchKernelGGL(kb_combine3, vec, dim3(256), 0, st, probs, mask, nb);
            break;
        case BandOp::Resid:   // res = ||blk[a0] - lam blk[a1]||
            hipLaunchKernelGGL(kb_resid, red, dim3(RT), 0, st, probs, mask, nb, a0, a1);
            PW_LAUNCH_CHECK();
            hipLaunchKernelGGL(kb_finish, fin, dim3(256), 0, st, probs, mask, nb, 1, 14);
            PW_LAUNCH_CHECK();
            hipLaunchKernelGGL(kb_scalars, sc, dim3(256), 0, st, probs, mask, nb, 2);
            break;
    }
    PW_LAUNCH_CHECK();
}

void band_batch_copy(const BandProb *probs, const int *mask, int nprob, int nb, int maxnpw, int n, const int *src,
                     const int *dst, hipStream_t st) {
    PW_CHECK(n >= 1 && n <= 4, PW_EINVAL, "batched copy of 1..4 blocks");
    int4 s4{src[0], n > 1 ? src[1] : 0, n > 2 ? src[2] : 0, n > 3 ? src[3] : 0};
    int4 d4{dst[0], n > 1 ? dst[1] : 0, n > 2 ? dst[2] : 0, n > 3 ? dst[3] : 0};
    hipLaunchKernelGGL(kb_copy, dim3((maxnpw + 255) / 256, nprob * nb, n), dim3(256), 0, st, probs, mask, nb, s4, d4);
    PW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Column-wise PCG of the folded linear equation (H - E)^2 x = (H - E) w.  Every
// column (right-hand side) has its own alpha and beta; the scalars stay on the
// device, each written by one thread per column.

// alpha = rz / <p, A p> with <p, A p> = ||YP||^2 (YP = (H - E) p)
__global__ void k_lin_alpha(int nb, int nsplit, const double *__restrict__ partial, const double *__restrict__ rz,
                            double *__restrict__ alpha) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double pap = 0;
    for (int k = 0; k < nsplit; ++k) pap += partial[(int64_t)b * nsplit + k];
    alpha[b] = pap > 0.0 ? rz[b] / pap : 0.0;
}

void lin_alpha(int nb, int npw, const void *YP, int64_t ld, const double *rz, double *alpha, BandRed r,
               hipStream_t st) {
    hipLaunchKernelGGL(k_norm2, dim3(r.nsplit, nb), dim3(RT), 0, st, nb, npw, (const double2 *)YP, ld, r.partial,
                       r.nsplit);
    PW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_lin_alpha, dim3((nb + 255) / 256), dim3(256), 0, st, nb, r.nsplit, r.partial, rz, alpha);
    PW_LAUNCH_CHECK();
}

// X += alpha P, Y += alpha YP, R -= alpha AP
__global__ void k_lin_update(int nb, int npw, double2 *__restrict__ X, double2 *__restrict__ Y,
                             double2 *__restrict__ R, const double2 *__restrict__ P, const double2 *__restrict__ YP,
                             const double2 *__restrict__ AP, int64_t ld, const double *__restrict__ alpha) {
    const int b = blockIdx.y;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npw) return;
    const double a = alpha[b];
    const int64_t i = (int64_t)b * ld + g;
    const double2 p = P[i], yp = YP[i], ap = AP[i];
    double2 x = X[i], y = Y[i], r = R[i];
    x.x += a * p.x;  x.y += a * p.y;
    y.x += a * yp.x; y.y += a * yp.y;
    r.x -= a * ap.x; r.y -= a * ap.y;
    X[i] = x;
    Y[i] = y;
    R[i] = r;
}

void lin_update(int nb, int npw, void *X, void *Y, void *R, const void *P, const void *YP, const void *AP, int64_t ld,
                const double *alpha, hipStream_t st) {
    hipLaunchKernelGGL(k_lin_update, dim3((npw + 255) / 256, nb), dim3(256), 0, st, nb, npw, (double2 *)X,
                       (double2 *)Y, (double2 *)R, (const double2 *)P, (const double2 *)YP, (const double2 *)AP, ld,
                       alpha);
    PW_LAUNCH_CHECK();
}

// Z = M o (R - U) with the paper's M(G) (U may be null); partial sums of Re<R, Z>
__global__ __launch_bounds__(RT) void k_lin_mdiag(int nb, int npw, const double2 *__restrict__ R,
                                                  const double2 *__restrict__ U, double2 *__restrict__ Z, int64_t ld,
                                                  const double *__restrict__ kin, double e_ref, double de2,
                                                  double *partial, int nsplit) {
    const int b = blockIdx.y, split = blockIdx.x;
    double acc[1] = {0};
    BAND_LOOP(npw) {
        const int64_t i = (int64_t)b * ld + g;
        const double2 r = R[i];
        double2 v = r;
        if (U) {
            const double2 u = U[i];
            v.x -= u.x;
            v.y -= u.y;
        }
        const double d = kin[g] - e_ref;
        const double m = 1.0 / (d * d + de2);
        const double2 z = make_double2(m * v.x, m * v.y);
        acc[0] += r.x * z.x + r.y * z.y;
        Z[i] = z;
    }
    block_store<1>(acc, partial, nb, nsplit, b, split);
}

__global__ __launch_bounds__(RT) void k_lin_rz(int nb, int npw, const double2 *__restrict__ R,
                                               const double2 *__restrict__ Z, int64_t ld, double *partial,
                                               int nsplit) {
    const int b = blockIdx.y, split = blockIdx.x;
    double acc[1] = {0};
    BAND_LOOP(npw) {
        const int64_t i = (int64_t)b * ld + g;
        const double2 r = R[i], z = Z[i];
        acc[0] += r.x * z.x + r.y * z.y;
    }
    block_store<1>(acc, partial, nb, nsplit, b, split);
}

// rz_new = sum of partials; beta = rz_new / rz (0 on the first call); rz <- rz_new
__global__ void k_lin_beta(int nb, int nsplit, const double *__restrict__ partial, double *__restrict__ rz,
                           double *__restrict__ beta, int first) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double s = 0;
    for (int k = 0; k < nsplit; ++k) s += partial[(int64_t)b * nsplit + k];
    const double old = rz[b];
    beta[b] = (!first && old > 0.0) ? s / old : 0.0;
    rz[b] = s;
}

void lin_mdiag(int nb, int npw, const void *R, const void *U, void *Z, int64_t ld, const double *kin, double e_ref,
               double de2, double *rz, double *beta, bool first, bool with_rz, BandRed r, hipStream_t st) {
    hipLaunchKernelGGL(k_lin_mdiag, dim3(r.nsplit, nb), dim3(RT), 0, st, nb, npw, (const double2 *)R,
                       (const double2 *)U, (double2 *)Z, ld, kin, e_ref, de2, r.partial, r.nsplit);
    PW_LAUNCH_CHECK();
    if (with_rz) {
        hipLaunchKernelGGL(k_lin_beta, dim3((nb + 255) / 256), dim3(256), 0, st, nb, r.nsplit, r.partial, rz, beta,
                           first ? 1 : 0);
        PW_LAUNCH_CHECK();
    }
}

void lin_rz_beta(int nb, int npw, const void *R, const void *Z, int64_t ld, double *rz, double *beta, bool first,
                 BandRed r, hipStream_t st) {
    hipLaunchKernelGGL(k_lin_rz, dim3(r.nsplit, nb), dim3(RT), 0, st, nb, npw, (const double2 *)R,
                       (const double2 *)Z, ld, r.partial, r.nsplit);
    PW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_lin_beta, dim3((nb + 255) / 256), dim3(256), 0, st, nb, r.nsplit, r.partial, rz, beta,
                       first ? 1 : 0);
    PW_LAUNCH_CHECK();
}

// P = Z + beta P
__global__ void k_lin_pupdate(int nb, int npw, const double2 *__restrict__ Z, double2 *__restrict__ P, int64_t ld,
                              const double *__restrict__ beta) {
    const int b = blockIdx.y;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npw) return;
    const double be = beta[b];
    const int64_t i = (int64_t)b * ld + g;
    const double2 z = Z[i], p = P[i];
    P[i] = make_double2(z.x + be * p.x, z.y + be * p.y);
}

void lin_pupdate(int nb, int npw, const void *Z, void *P, int64_t ld, const double *beta, hipStream_t st) {
    hipLaunchKernelGGL(k_lin_pupdate, dim3((npw + 255) / 256, nb), dim3(256), 0, st, nb, npw, (const double2 *)Z,
                       (double2 *)P, ld, beta);
    PW_LAUNCH_CHECK();
}

// E[l][i] = C[l][i] / d_i - D[l][i]   (coefficients of the eigenstate part of M')
__global__ void k_lin_coef(int n, int nev, const double2 *__restrict__ C, const double2 *__restrict__ D,
                           const double *__restrict__ invd, double2 *__restrict__ E) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n * nev) return;
    const double s = invd[k % nev];
    const double2 c = C[k], d = D[k];
    E[k] = make_double2(c.x * s - d.x, c.y * s - d.y);
}

void lin_coef(int nrhs, int nev, const void *C, const void *D, const double *invd, void *E, hipStream_t st) {
    const int n = nrhs * nev;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_lin_coef, dim3((n + 255) / 256), dim3(256), 0, st, nrhs, nev, (const double2 *)C,
                       (const double2 *)D, invd, (double2 *)E);
    PW_LAUNCH_CHECK();
}

// err[b] = ||Y_b - W_b||
__global__ __launch_bounds__(RT) void k_lin_err(int nb, int npw, const double2 *__restrict__ Y, int64_t ldy,
                                                const double2 *__restrict__ W, int64_t ldw, double *partial,
                                                int nsplit) {
    const int b = blockIdx.y, split = blockIdx.x;
    double acc[1] = {0};
    BAND_LOOP(npw) {
        const double2 y = Y[(int64_t)b * ldy + g], w = W[(int64_t)b * ldw + g];
        const double rx = y.x - w.x, ry = y.y - w.y;
        acc[0] += rx * rx + ry * ry;
    }
    block_store<1>(acc, partial, nb, nsplit, b, split);
}

void lin_err(int nb, int npw, const void *Y, int64_t ldy, const void *W, int64_t ldw, double *err, BandRed r,
             hipStream_t st) {
    hipLaunchKernelGGL(k_lin_err, dim3(r.nsplit, nb), dim3(RT), 0, st, nb, npw, (const double2 *)Y, ldy,
                       (const double2 *)W, ldw, r.partial, r.nsplit);
    PW_LAUNCH_CHECK();
    finish(1, nb, r, err, st);
    hipLaunchKernelGGL(k_sqrt, dim3((nb + 255) / 256), dim3(256), 0, st, nb, err);
    PW_LAUNCH_CHECK();
}

// R -= AX
__global__ void k_lin_sub(int nb, int npw, double2 *__restrict__ R, const double2 *__restrict__ AX, int64_t ld) {
    const int b = blockIdx.y;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npw) return;
    const int64_t i = (int64_t)b * ld + g;
    const double2 r = R[i], a = AX[i];
    R[i] = make_double2(r.x - a.x, r.y - a.y);
}

void lin_sub(int nb, int npw, void *R, const void *AX, int64_t ld, hipStream_t st) {
    hipLaunchKernelGGL(k_lin_sub, dim3((npw + 255) / 256, nb), dim3(256), 0, st, nb, npw, (double2 *)R,
                       (const double2 *)AX, ld);
    PW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Chebyshev filter: U_{k+1} = s (H - c) U_k - U_{k-1} with T = (H - c) U_k given;
// the new vector overwrites U_{k-1} (first: U_1 = s T, U_0 untouched) and
// Y += gamma U_{k+1}.
__global__ void k_cheb_step(int nb, int npw, const double2 *__restrict__ T, double2 *__restrict__ Uprev,
                            double2 *__restrict__ Y, int64_t ld, double s, double gamma, int first) {
    const int b = blockIdx.y;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npw) return;
    const int64_t i = (int64_t)b * ld + g;
    const double2 t = T[i];
    double2 u = make_double2(s * t.x, s * t.y);
    if (!first) {
        const double2 p = Uprev[i];
        u.x -= p.x;
        u.y -= p.y;
    }
    Uprev[i] = u;
    double2 y = Y[i];
    y.x += gamma * u.x;
    y.y += gamma * u.y;
    Y[i] = y;
}

void cheb_step(int nb, int npw, const void *T, void *Uprev, void *Y, int64_t ld, double s, double gamma, bool first,
               hipStream_t st) {
    hipLaunchKernelGGL(k_cheb_step, dim3((npw + 255) / 256, nb), dim3(256), 0, st, nb, npw, (const double2 *)T,
                       (double2 *)Uprev, (double2 *)Y, ld, s, gamma, first ? 1 : 0);
    PW_LAUNCH_CHECK();
}

// dst = s * src
__global__ void k_scale_copy(int nb, int npw, const double2 *__restrict__ src, int64_t lds, double2 *__restrict__ dst,
                             int64_t ldd, double s) {
    const int b = blockIdx.y;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npw) return;
    const double2 v = src[(int64_t)b * lds + g];
    dst[(int64_t)b * ldd + g] = make_double2(s * v.x, s * v.y);
}

void scale_copy(int nb, int npw, const void *src, int64_t lds, void *dst, int64_t ldd, double s, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_copy, dim3((npw + 255) / 256, nb), dim3(256), 0, st, nb, npw, (const double2 *)src, lds,
                       (double2 *)dst, ldd, s);
    PW_LAUNCH_CHECK();
}

// Lanczos: W -= alpha V + beta Vprev (one vector)
__global__ void k_lanczos(int npw, double2 *__restrict__ W, const double2 *__restrict__ V,
                          const double2 *__restrict__ Vp, double alpha, double beta) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npw) return;
    const double2 v = V[g], p = Vp[g];
    double2 w = W[g];
    w.x -= alpha * v.x + beta * p.x;
    w.y -= alpha * v.y + beta * p.y;
    W[g] = w;
}

void lanczos_update(int npw, void *W, const void *V, const void *Vp, double alpha, double beta, hipStream_t st) {
    hipLaunchKernelGGL(k_lanczos, dim3((npw + 255) / 256), dim3(256), 0, st, npw, (double2 *)W, (const double2 *)V,
                       (const double2 *)Vp, alpha, beta);
    PW_LAUNCH_CHECK();
}

// out[b] = Re <A_b, B_b>
void red_dot_re(int nb, int npw, const void *A, const void *B, int64_t ld, double *out, BandRed r, hipStream_t st) {
    hipLaunchKernelGGL(k_lin_rz, dim3(r.nsplit, nb), dim3(RT), 0, st, nb, npw, (const double2 *)A, (const double2 *)B,
                       ld, r.partial, r.nsplit);
    PW_LAUNCH_CHECK();
    finish(1, nb, r, out, st);
}

// ---------------------------------------------------------------------------
// Wave-function interpolation between k-points.

// dst[b][g] = src[b][map[g]] (0 where map[g] < 0): coefficients onto another sphere
__global__ void k_gather_pw(int nb, int npw_to, const double2 *__restrict__ src, int64_t lds,
                            const int32_t *__restrict__ map, double2 *__restrict__ dst, int64_t ldd) {
    const int b = blockIdx.y;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npw_to) return;
    const int32_t m = map[g];
    dst[(int64_t)b * ldd + g] = m >= 0 ? src[(int64_t)b * lds + m] : make_double2(0.0, 0.0);
}

void gather_pw(int nb, int npw_to, const void *src, int64_t lds, const int32_t *map, void *dst, int64_t ldd,
               hipStream_t st) {
    hipLaunchKernelGGL(k_gather_pw, dim3((npw_to + 255) / 256, nb), dim3(256), 0, st, nb, npw_to, (const double2 *)src,
                       lds, map, (double2 *)dst, ldd);
    PW_LAUNCH_CHECK();
}

// Hk[i][j] = alpha e1[i] delta_ij + (1 - alpha) sum_m conj(U[i][m]) U[j][m] e2[m]
__global__ void k_kinterp_hk(int n, double alpha, const double *__restrict__ e1, const double *__restrict__ e2,
                             const double2 *__restrict__ U, double2 *__restrict__ Hk) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n * n) return;
    const int i = k / n, j = k % n;
    double re = 0.0, im = 0.0;
    for (int m = 0; m < n; ++m) {
        const double2 a = U[(int64_t)i * n + m], b = U[(int64_t)j * n + m];
        const double w = e2[m];
        re += w * (a.x * b.x + a.y * b.y);        // conj(a) b
        im += w * (a.x * b.y - a.y * b.x);
    }
    re *= 1.0 - alpha;
    im *= 1.0 - alpha;
    if (i == j) re += alpha * e1[i];
    Hk[k] = make_double2(re, im);
}

void kinterp_hk(int n, double alpha, const double *e1, const double *e2, const void *U, void *Hk, hipStream_t st) {
    hipLaunchKernelGGL(k_kinterp_hk, dim3((n * n + 255) / 256), dim3(256), 0, st, n, alpha, e1, e2,
                       (const double2 *)U, (double2 *)Hk);
    PW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
__global__ void k_fill_zero(uint4 *p, size_t n16) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) p[i] = make_uint4(0, 0, 0, 0);
}

void fill_zero(void *p, size_t bytes, hipStream_t st) {
    PW_CHECK(bytes % 16 == 0 && ((uintptr_t)p % 16) == 0, PW_EINVAL, "fill_zero needs 16-byte aligned sizes");
    const size_t n16 = bytes / 16;
    if (!n16) return;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, st, (uint4 *)p, n16);
    PW_LAUNCH_CHECK();
}

template <typename S, typename D>
__global__ __launch_bounds__(256) void k_convert(int npw, const S *__restrict__ src, int64_t lds, D *__restrict__ dst,
                                                 int64_t ldd) {
    const int b = blockIdx.y;
    const int g0 = blockIdx.x * 256 * kVec + threadIdx.x;
    S v[kVec];
#pragma unroll
    for (int j = 0; j < kVec; ++j) {
        const int g = g0 + 256 * j;
        if (g < npw) v[j] = src[(int64_t)b * lds + g];
    }
#pragma unroll
    for (int j = 0; j < kVec; ++j) {
        const int g = g0 + 256 * j;
        if (g < npw) {
            D o;
            o.x = v[j].x;
            o.y = v[j].y;
            dst[(int64_t)b * ldd + g] = o;
        }
    }
}

void copy_block(int nb, int npw, const void *src, int64_t lds, void *dst, int64_t ldd, hipStream_t st) {
    if (nb <= 0) return;
    hipLaunchKernelGGL((k_convert<double2, double2>), vec_grid(npw, nb), dim3(256), 0, st, npw,
                       (const double2 *)src, lds, (double2 *)dst, ldd);
    PW_LAUNCH_CHECK();
}

void c64_to_c128(int nb, int npw, const void *src, int64_t lds, void *dst, int64_t ldd, hipStream_t st) {
    if (nb <= 0) return;
    hipLaunchKernelGGL((k_convert<float2, double2>), vec_grid(npw, nb), dim3(256), 0, st, npw,
                       (const float2 *)src, lds, (double2 *)dst, ldd);
    PW_LAUNCH_CHECK();
}

void c128_to_c64(int nb, int npw, const void *src, int64_t lds, void *dst, int64_t ldd, hipStream_t st) {
    if (nb <= 0) return;
    hipLaunchKernelGGL((k_convert<double2, float2>), vec_grid(npw, nb), dim3(256), 0, st, npw,
                       (const double2 *)src, lds, (float2 *)dst, ldd);
    PW_LAUNCH_CHECK();
}

__global__ void k_nan_check(size_t n, const double *x, int *flag) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(x[i])) flag[0] = 1;
}

void nan_check(size_t n, const double *x, int *flag, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_nan_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, x, flag);
    PW_LAUNCH_CHECK();
}

}  // namespace pw
