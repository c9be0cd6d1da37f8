// Mixed-precision projector GEMMs: BF16 operands, FP32 accumulation on gfx950
// matrix cores (v_mfma_f32_16x16x32_bf16), complex64 wave functions.
//
//   projection      projT[b][p] = D_p sum_G conj(beta_p(G)) psi_b(G)     (split-K)
//   back-projection out[b][G]  += sum_p projT[b][p] beta_p(G)
// The projector table is stored once as two BF16 planes (real, imaginary),
// [nproj][ldb] with ldb a multiple of 64 and zero padding.  Wave functions and
// projections are rounded to BF16 (nearest even) as they are staged into LDS.
#include "kernels.h"

namespace pw {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Lane layout of v_mfma_f32_16x16x32_bf16 (wave64):
//   A: lane l holds A[i = l % 16][k = 8 (l / 16) + 0..7]
//   B: lane l holds B[k = 8 (l / 16) + 0..7][j = l % 16]
//   D: lane l, item v holds D[i = 4 (l / 16) + v][j = l % 16]
__device__ inline v4f mfma_bf16(bf16x8 a, bf16x8 b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline bf16x8 neg8(bf16x8 v) {
    union { bf16x8 b; uint4 u; } x;
    x.b = v;
    x.u.x ^= 0x80008000u; x.u.y ^= 0x80008000u; x.u.z ^= 0x80008000u; x.u.w ^= 0x80008000u;
    return x.b;
}

constexpr int KB = 64;          // k-depth per LDS stage
constexpr int LP = KB + 8;      // padded LDS row (bf16 elements)

// ---------------------------------------------------------------------------
// projection partials: partial[s][p][b] over K chunk s
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void proj_bf16_partial(int M, int N, int K, const uint16_t *__restrict__ Br,
                                                         const uint16_t *__restrict__ Bi, int64_t ldb,
                                                         const float2 *__restrict__ psi, int64_t ld, int kchunk,
                                                         float2 *__restrict__ partial) {
    __shared__ __attribute__((aligned(16))) uint16_t Ar[64][LP], Ai[64][LP], Pr[64][LP], Pi[64][LP];
    const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64, s = blockIdx.z;
    const int kbeg = s * kchunk;
    const int kend = min(K, kbeg + kchunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    v4f accr[2][2], acci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) { accr[i][j] = v4f{0, 0, 0, 0}; acci[i][j] = v4f{0, 0, 0, 0}; }
    for (int k0 = kbeg; k0 < kend; k0 += KB) {
        // projector planes: 64 rows x 64 bf16, 16-byte pieces
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int e = tid + it * 256;          // 0..511
            const int r = e >> 3, c8 = (e & 7) * 8;
            const int gm = m0 + r;
            uint4 vr = make_uint4(0, 0, 0, 0), vi = make_uint4(0, 0, 0, 0);
            if (gm < M) {
                vr = *reinterpret_cast<const uint4 *>(Br + (int64_t)gm * ldb + k0 + c8);
                vi = *reinterpret_cast<const uint4 *>(Bi + (int64_t)gm * ldb + k0 + c8);
            }
            *reinterpret_cast<uint4 *>(&Ar[r][c8]) = vr;
            *reinterpret_cast<uint4 *>(&Ai[r][c8]) = vi;
        }
        // wave functions: 64 bands x 64 complex64, rounded to bf16
#pragma unroll
        for (int it = 0; it < 16; ++it) {
            const int e = tid + it * 256;          // 0..4095
            const int r = e >> 6, c = e & 63;
            const int gn = n0 + r, gk = k0 + c;
            float2 v = make_float2(0.f, 0.f);
            if (gn < N && gk < kend) v = psi[(int64_t)gn * ld + gk];
            Pr[r][c] = f2bf(v.x);
            Pi[r][c] = f2bf(v.y);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KB / 32; ++ks) {
            const int kk = ks * 32 + 8 * (lane >> 4);
            bf16x8 ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int row = wm * 32 + i * 16 + (lane & 15);
                ar[i] = *reinterpret_cast<const bf16x8 *>(&Ar[row][kk]);
                ai[i] = *reinterpret_cast<const bf16x8 *>(&Ai[row][kk]);
                nai[i] = neg8(ai[i]);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int row = wn * 32 + j * 16 + (lane & 15);
                br[j] = *reinterpret_cast<const bf16x8 *>(&Pr[row][kk]);
                bi[j] = *reinterpret_cast<const bf16x8 *>(&Pi[row][kk]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    // conj(beta) psi: re = br pr + bi pi, im = br pi - bi pr
                    accr[i][j] = mfma_bf16(ar[i], br[j], accr[i][j]);
                    accr[i][j] = mfma_bf16(ai[i], bi[j], accr[i][j]);
                    acci[i][j] = mfma_bf16(ar[i], bi[j], acci[i][j]);
                    acci[i][j] = mfma_bf16(nai[i], br[j], acci[i][j]);
                }
        }
        __syncthreads();
    }
    float2 *P = partial + (int64_t)s * M * N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
                const int col = n0 + wn * 32 + j * 16 + (lane & 15);
                if (row < M && col < N) P[(int64_t)row * N + col] = make_float2(accr[i][j][v], acci[i][j][v]);
            }
}

// projT[b][p] = d[p] * sum_s partial[s][p][b]
__global__ void proj_bf16_reduce(int M, int N, int nsplit, const float2 *__restrict__ partial,
                                 const float *__restrict__ d, float2 *__restrict__ projT) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)M * N) return;
    const int m = (int)(idx / N), n = (int)(idx % N);
    double re = 0, im = 0;
    for (int s = 0; s < nsplit; ++s) {
        const float2 v = partial[(int64_t)s * M * N + idx];
        re += v.x;
        im += v.y;
    }
    const double sc = d ? d[m] : 1.0;
    projT[(int64_t)n * M + m] = make_float2((float)(re * sc), (float)(im * sc));
}

static int bf16_splits(int M, int N, int K) {
    const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
    int s = (1024 + tiles - 1) / tiles;
    const int maxs = (K + 4 * KB - 1) / (4 * KB);
    if (s > maxs) s = maxs;
    if (s < 1) s = 1;
    return s;
}

size_t cnt_partial_bytes(int M, int N, int K) { return (size_t)bf16_splits(M, N, K) * M * N * sizeof(float2); }

void proj_bf16(int nproj, int nb, int npw, const void *beta_bf16, const void *psi, int64_t ld, const float *d,
               void *projT, void *partial, hipStream_t st) {
    // ldb: planes are [nproj][ldb] with ldb = npw rounded up to 64
    const int64_t ldb = ((npw + 63) / 64) * 64;
    const uint16_t *Br = (const uint16_t *)beta_bf16;
    const uint16_t *Bi = Br + (int64_t)nproj * ldb;
    const int ns = bf16_splits(nproj, nb, npw);
    int kchunk = (npw + ns - 1) / ns;
    kchunk = ((kchunk + KB - 1) / KB) * KB;
    const int nsplit = (npw + kchunk - 1) / kchunk;
    dim3 grid((nproj + 63) / 64, (nb + 63) / 64, nsplit);
    hipLaunchKernelGGL(proj_bf16_partial, grid, dim3(256), 0, st, nproj, nb, npw, Br, Bi, ldb, (const float2 *)psi,
                       ld, kchunk, (float2 *)partial);
    PW_LAUNCH_CHECK();
    const int64_t tot = (int64_t)nproj * nb;
    hipLaunchKernelGGL(proj_bf16_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, nproj, nb, nsplit,
                       (const float2 *)partial, d, (float2 *)projT);
    PW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// back-projection: out[b][G] += sum_p W[b][p] beta_p(G), W = projT (complex64)
// tile 64 bands x 64 plane waves
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void backproj_bf16_kernel(int M, int J, int K, const float2 *__restrict__ W,
                                                            const uint16_t *__restrict__ Br,
                                                            const uint16_t *__restrict__ Bi, int64_t ldb,
                                                            float2 *__restrict__ out, int64_t ldo) {
    __shared__ __attribute__((aligned(16))) uint16_t Wr[64][LP], Wi[64][LP], Tr[64][LP], Ti[64][LP];
    const int j0 = blockIdx.x * 64, m0 = blockIdx.y * 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wj = wave >> 1;
    v4f accr[2][2], acci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) { accr[i][j] = v4f{0, 0, 0, 0}; acci[i][j] = v4f{0, 0, 0, 0}; }
    for (int k0 = 0; k0 < K; k0 += KB) {
        // W tile: 64 bands x 64 projectors
#pragma unroll
        for (int it = 0; it < 16; ++it) {
            const int e = tid + it * 256;
            const int r = e >> 6, c = e & 63;
            const int gm = m0 + r, gk = k0 + c;
            float2 v = make_float2(0.f, 0.f);
            if (gm < M && gk < K) v = W[(int64_t)gm * K + gk];
            Wr[r][c] = f2bf(v.x);
            Wi[r][c] = f2bf(v.y);
        }
        // projector tile, transposed into LDS: T[j][k] = beta[k0 + k][j0 + j]
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int e = tid + it * 256;          // 0..511: 64 k-rows x 8 pieces of 8 plane waves
            const int kr = e >> 3, c8 = (e & 7) * 8;
            const int gk = k0 + kr;
            uint4 vr = make_uint4(0, 0, 0, 0), vi = make_uint4(0, 0, 0, 0);
            if (gk < K && j0 + c8 < ldb) {
                vr = *reinterpret_cast<const uint4 *>(Br + (int64_t)gk * ldb + j0 + c8);
                vi = *reinterpret_cast<const uint4 *>(Bi + (int64_t)gk * ldb + j0 + c8);
            }
            const uint16_t *pr = reinterpret_cast<const uint16_t *>(&vr);
            const uint16_t *pi = reinterpret_cast<const uint16_t *>(&vi);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                Tr[c8 + q][kr] = pr[q];
                Ti[c8 + q][kr] = pi[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KB / 32; ++ks) {
            const int kk = ks * 32 + 8 * (lane >> 4);
            bf16x8 ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int row = wm * 32 + i * 16 + (lane & 15);
                ar[i] = *reinterpret_cast<const bf16x8 *>(&Wr[row][kk]);
                ai[i] = *reinterpret_cast<const bf16x8 *>(&Wi[row][kk]);
                nai[i] = neg8(ai[i]);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int row = wj * 32 + j * 16 + (lane & 15);
                br[j] = *reinterpret_cast<const bf16x8 *>(&Tr[row][kk]);
                bi[j] = *reinterpret_cast<const bf16x8 *>(&Ti[row][kk]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    // W beta: re = wr br - wi bi, im = wr bi + wi br
                    accr[i][j] = mfma_bf16(ar[i], br[j], accr[i][j]);
                    accr[i][j] = mfma_bf16(nai[i], bi[j], accr[i][j]);
                    acci[i][j] = mfma_bf16(ar[i], bi[j], acci[i][j]);
                    acci[i][j] = mfma_bf16(ai[i], br[j], acci[i][j]);
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
                const int row = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
                const int col = j0 + wj * 32 + j * 16 + (lane & 15);
                if (row < M && col < J) {
                    float2 *o = out + (int64_t)row * ldo + col;
                    const float2 old = *o;
                    *o = make_float2(old.x + accr[i][j][v], old.y + acci[i][j][v]);
                }
            }
}

void backproj_bf16(int nb, int npw, int nproj, const void *projT, const void *beta_bf16, void *out, int64_t ldo,
                   hipStream_t st) {
    const int64_t ldb = ((npw + 63) / 64) * 64;
    const uint16_t *Br = (const uint16_t *)beta_bf16;
    const uint16_t *Bi = Br + (int64_t)nproj * ldb;
    dim3 grid((npw + 63) / 64, (nb + 63) / 64);
    hipLaunchKernelGGL(backproj_bf16_kernel, grid, dim3(256), 0, st, nb, npw, nproj, (const float2 *)projT, Br, Bi,
                       ldb, (float2 *)out, ldo);
    PW_LAUNCH_CHECK();
}

}  // namespace pw
