// Complex FP64 GEMMs on gfx950 matrix cores (v_mfma_f64_16x16x4f64).
//
// Two shapes cover the whole path:
//   NT (split-K):  C[m][n] = sum_k op(A[m][k]) B[n][k],   K = npw (huge), M, N small
//                  -> projections <beta_p|psi_b>, Gram Psi^H Psi, Psi^H Y, Psi^H P
//   NN:            Out[m][j] = alpha sum_k W[m][k] X[k][j] + beta Out[m][j],  j over npw
//                  -> back-projection sum_p beta_p D_p c_pb, block rotations Psi Q
// Complex products are four real MFMAs into separate real/imaginary accumulators.
// Operand tiles are staged in LDS (rows padded by one element against bank
// conflicts); split-K partial sums are reduced by a second deterministic kernel,
// so results are bitwise reproducible (no floating-point atomics).
#include "kernels.h"

namespace pw {

typedef double v4d __attribute__((ext_vector_type(4)));

// Lane layout of v_mfma_f64_16x16x4f64 (wave64):
//   A operand: lane l holds A[i = l % 16][k = l / 16]
//   B operand: lane l holds B[k = l / 16][j = l % 16]
//   D:         lane l, item v holds D[i = l / 16 + 4 v][j = l % 16]  (checked on gfx950)
__device__ inline v4d mfma16(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int KT = 16;       // k-depth of one LDS stage (complex elements)

// ---------------------------------------------------------------------------
// NT split-K partials: partial[s][m][n] = sum_{k in chunk s} op(A[m][k]) * B[n][k]
// op = conj when CONJA.  Tile 64 x 64, 4 waves each 32 x 32.
// ---------------------------------------------------------------------------
template <bool CONJA>
__global__ __launch_bounds__(256) void zgemm_nt_partial(int M, int N, int K, const double2 *__restrict__ A,
                                                        int64_t lda, const double2 *__restrict__ B, int64_t ldb,
                                                        int kchunk, double2 *__restrict__ partial) {
    __shared__ double2 As[64][KT + 1];
    __shared__ double2 Bs[64][KT + 1];
    const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64, s = blockIdx.z;
    const int kbeg = s * kchunk;
    const int kend = min(K, kbeg + kchunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    v4d accr[2][2], acci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) { accr[i][j] = v4d{0, 0, 0, 0}; acci[i][j] = v4d{0, 0, 0, 0}; }
    for (int k0 = kbeg; k0 < kend; k0 += KT) {
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int e = tid + it * 256;
            const int r = e / KT, kk = e % KT;
            const int gk = k0 + kk;
            const int gm = m0 + r, gn = n0 + r;
            As[r][kk] = (gm < M && gk < kend) ? A[(int64_t)gm * lda + gk] : make_double2(0.0, 0.0);
            Bs[r][kk] = (gn < N && gk < kend) ? B[(int64_t)gn * ldb + gk] : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int kq = 0; kq < KT / 4; ++kq) {
            const int k = kq * 4 + (lane >> 4);
            double2 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = As[wm * 32 + i * 16 + (lane & 15)][k];
                if (CONJA) a[i].y = -a[i].y;
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[wn * 32 + j * 16 + (lane & 15)][k];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    accr[i][j] = mfma16(a[i].x, b[j].x, accr[i][j]);
                    accr[i][j] = mfma16(-a[i].y, b[j].y, accr[i][j]);
                    acci[i][j] = mfma16(a[i].x, b[j].y, acci[i][j]);
                    acci[i][j] = mfma16(a[i].y, b[j].x, acci[i][j]);
                }
        }
        __syncthreads();
    }
    double2 *P = partial + (int64_t)s * M * N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 32 + i * 16 + (lane >> 4) + 4 * v;
                const int col = n0 + wn * 32 + j * 16 + (lane & 15);
                if (row < M && col < N) P[(int64_t)row * N + col] = make_double2(accr[i][j][v], acci[i][j][v]);
            }
}

// out = alpha * rowscale[m] * sum_s partial[s][m][n] (+ beta * out); TRANS writes out[n][m]
template <bool TRANS>
__global__ void reduce_partial(int M, int N, int nsplit, const double2 *__restrict__ partial, double alpha,
                               const double *__restrict__ rowscale, double beta, double2 *__restrict__ out,
                               int64_t ldo) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)M * N) return;
    const int m = (int)(idx / N), n = (int)(idx % N);
    double re = 0, im = 0;
    for (int s = 0; s < nsplit; ++s) {
        const double2 v = partial[(int64_t)s * M * N + idx];
        re += v.x;
        im += v.y;
    }
    double sc = alpha * (rowscale ? rowscale[m] : 1.0);
    double2 *o = TRANS ? out + (int64_t)n * ldo + m : out + (int64_t)m * ldo + n;
    if (beta != 0.0) {
        *o = make_double2(sc * re + beta * o->x, sc * im + beta * o->y);
    } else {
        *o = make_double2(sc * re, sc * im);
    }
}

// ---------------------------------------------------------------------------
// NN: Out[m][j] = alpha * sum_k W[m][k] X[k][j] + beta * Out[m][j]
// Tile 64 (m) x 64 (j), 4 waves each 32 x 32.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void zgemm_nn(int M, int J, int K, const double2 *__restrict__ W, int64_t ldw,
                                                const double2 *__restrict__ X, int64_t ldx, double alpha,
                                                double beta, double2 *__restrict__ Out, int64_t ldo) {
    __shared__ double2 Ws[64][KT + 1];
    __shared__ double2 Xs[KT][64 + 1];
    const int j0 = blockIdx.x * 64, m0 = blockIdx.y * 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wj = wave >> 1;
    v4d accr[2][2], acci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) { accr[i][j] = v4d{0, 0, 0, 0}; acci[i][j] = v4d{0, 0, 0, 0}; }
    for (int k0 = 0; k0 < K; k0 += KT) {
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int e = tid + it * 256;
            {   // W tile 64 x KT
                const int r = e / KT, kk = e % KT;
                const int gm = m0 + r, gk = k0 + kk;
                Ws[r][kk] = (gm < M && gk < K) ? W[(int64_t)gm * ldw + gk] : make_double2(0.0, 0.0);
            }
            {   // X tile KT x 64
                const int kk = e / 64, c = e % 64;
                const int gk = k0 + kk, gj = j0 + c;
                Xs[kk][c] = (gk < K && gj < J) ? X[(int64_t)gk * ldx + gj] : make_double2(0.0, 0.0);
            }
        }
        __syncthreads();
#pragma unroll
        for (int kq = 0; kq < KT / 4; ++kq) {
            const int k = kq * 4 + (lane >> 4);
            double2 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = Ws[wm * 32 + i * 16 + (lane & 15)][k];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Xs[k][wj * 32 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    accr[i][j] = mfma16(a[i].x, b[j].x, accr[i][j]);
                    accr[i][j] = mfma16(-a[i].y, b[j].y, accr[i][j]);
                    acci[i][j] = mfma16(a[i].x, b[j].y, acci[i][j]);
                    acci[i][j] = mfma16(a[i].y, b[j].x, acci[i][j]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 32 + i * 16 + (lane >> 4) + 4 * v;
                const int col = j0 + wj * 32 + j * 16 + (lane & 15);
                if (row < M && col < J) {
                    double2 *o = Out + (int64_t)row * ldo + col;
                    double re = alpha * accr[i][j][v], im = alpha * acci[i][j][v];
                    if (beta != 0.0) { re += beta * o->x; im += beta * o->y; }
                    *o = make_double2(re, im);
                }
            }
}

// ---------------------------------------------------------------------------
// host wrappers
// ---------------------------------------------------------------------------
// Number of K-splits so that the grid holds >= ~1024 workgroups and each chunk
// keeps at least a few LDS stages.
int nt_splits(int M, int N, int K) {
    const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
    int s = (1024 + tiles - 1) / tiles;
    const int maxs = (K + 4 * KT - 1) / (4 * KT);
    if (s > maxs) s = maxs;
    if (s < 1) s = 1;
    return s;
}

size_t nt_partial_bytes(int M, int N, int K) {
    return (size_t)nt_splits(M, N, K) * M * N * sizeof(double2);
}

// C (M x N, ldc) = alpha * rowscale o (op(A) B^T) (+ beta C); trans: write C^T (N x M)
void zgemm_nt(int M, int N, int K, bool conja, const void *A, int64_t lda, const void *B, int64_t ldb,
              double alpha, const double *rowscale, double beta, void *C, int64_t ldc, bool trans, void *partial,
              hipStream_t st) {
    if (M <= 0 || N <= 0) return;
    const int ns = nt_splits(M, N, K);
    int kchunk = (K + ns - 1) / ns;
    kchunk = ((kchunk + KT - 1) / KT) * KT;
    const int nsplit = (K + kchunk - 1) / kchunk;
    dim3 grid((M + 63) / 64, (N + 63) / 64, nsplit > 0 ? nsplit : 1);
    if (K <= 0) {
        fill_zero(partial, (size_t)M * N * sizeof(double2), st);
    } else if (conja) {
        hipLaunchKernelGGL((zgemm_nt_partial<true>), grid, dim3(256), 0, st, M, N, K,
                           (const double2 *)A, lda, (const double2 *)B, ldb, kchunk, (double2 *)partial);
    } else {
        hipLaunchKernelGGL((zgemm_nt_partial<false>), grid, dim3(256), 0, st, M, N, K,
                           (const double2 *)A, lda, (const double2 *)B, ldb, kchunk, (double2 *)partial);
    }
    PW_LAUNCH_CHECK();
    const int64_t tot = (int64_t)M * N;
    const int nblk = (int)((tot + 255) / 256);
    const int ns_eff = K <= 0 ? 1 : nsplit;
    if (trans)
        hipLaunchKernelGGL((reduce_partial<true>), dim3(nblk), dim3(256), 0, st, M, N, ns_eff,
                           (const double2 *)partial, alpha, rowscale, beta, (double2 *)C, ldc);
    else
        hipLaunchKernelGGL((reduce_partial<false>), dim3(nblk), dim3(256), 0, st, M, N, ns_eff,
                           (const double2 *)partial, alpha, rowscale, beta, (double2 *)C, ldc);
    PW_LAUNCH_CHECK();
}

// Out (M x J, ldo) = alpha * W (M x K, ldw) . X (K x J, ldx) + beta * Out
void zgemm_nn_launch(int M, int J, int K, const void *W, int64_t ldw, const void *X, int64_t ldx, double alpha,
                     double beta, void *Out, int64_t ldo, hipStream_t st) {
    if (M <= 0 || J <= 0) return;
    dim3 grid((J + 63) / 64, (M + 63) / 64);
    hipLaunchKernelGGL(zgemm_nn, grid, dim3(256), 0, st, M, J, K, (const double2 *)W, ldw, (const double2 *)X,
                       ldx, alpha, beta, (double2 *)Out, ldo);
    PW_LAUNCH_CHECK();
}

}  // namespace pw
