// Complex FP64 GEMMs on gfx950 matrix cores (v_mfma_f64_16x16x4f64).
//
// Two shapes cover the whole path:
//   NT (split-K):  C[m][n] = sum_k op(A[m][k]) B[n][k],   K = npw (huge), M, N small
//                  -> projections <beta_p|psi_b>, Gram Psi^H Psi, Psi^H Y, Psi^H P
//   NN:            Out[m][j] = alpha sum_k W[m][k] X[k][j] + beta Out[m][j],  j over npw
//                  -> back-projection sum_p beta_p D_p c_pb, block rotations Q . Psi
// Complex products are four real MFMAs into separate real/imaginary accumulators.
// Operand tiles are staged in LDS (rows padded against bank conflicts); the next
// k-stage is fetched into registers while the current one is multiplied.
// Split-K partial sums are reduced by a second kernel in a fixed order, so
// results are bitwise reproducible (no floating-point atomics).
#include "kernels.h"

namespace pw {

typedef double v4d __attribute__((ext_vector_type(4)));

// Lane layout of v_mfma_f64_16x16x4f64 (wave64), checked on gfx950:
//   A operand: lane l holds A[i = l % 16][k = l / 16]
//   B operand: lane l holds B[k = l / 16][j = l % 16]
//   D:         lane l, item v holds D[i = l / 16 + 4 v][j = l % 16]
__device__ inline v4d mfma16(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int KT = 16;       // k-depth of one LDS stage (complex elements)

// Complex products of a wave's 16 x 16 blocks, two forms.  Four real products:
// c1 += Re(a b), c2 += Im(a b).  Three (Gauss), for waves of at most four blocks in
// workgroups of at most eight waves, whose third accumulator still fits the
// register file without spilling: c1 += ar br, c2 += ai bi,
// c3 += (ar + ai)(br + bi), with sa = ar + ai and sb = br + bi formed once per
// operand fragment; then Re(sum a b) = c1 - c2 and Im(sum a b) = c3 - c1 - c2.
// The three-product form does three quarters of the matrix-core work; its error
// stays within a few units of roundoff of (|ar| + |ai|)(|br| + |bi|) summed over k.
template <bool G3>
__device__ inline void cmfma_blk(const double2 a, const double2 b, double sa, double sb, v4d &c1, v4d &c2,
                                 v4d &c3) {
    if constexpr (G3) {
        c1 = mfma16(a.x, b.x, c1);
        c2 = mfma16(a.y, b.y, c2);
        c3 = mfma16(sa, sb, c3);
    } else {
        c1 = mfma16(a.x, b.x, c1);
        c1 = mfma16(-a.y, b.y, c1);
        c2 = mfma16(a.x, b.y, c2);
        c2 = mfma16(a.y, b.x, c2);
    }
}
template <bool G3> __device__ inline double2 cmfma_result(const v4d &c1, const v4d &c2, const v4d &c3, int v) {
    if constexpr (G3) return make_double2(c1[v] - c2[v], c3[v] - c1[v] - c2[v]);
    else return make_double2(c1[v], c2[v]);
}

// ---------------------------------------------------------------------------
// NT split-K partials: partial[s][m][n] = sum_{k in chunk s} op(A[m][k]) * B[n][k]
// op = conj when CONJA.  Waves WM x WN, each BM x BN blocks of 16 x 16.
// ---------------------------------------------------------------------------
// TAG only separates the projector launches from the block-algebra ones in profiles
// one tile (bm, bn) of split s; the batched kernel below runs the same body
template <int WM, int WN, int BM, int BN, bool CONJA, bool G3OK>
__device__ __forceinline__ void nt_partial_tile(int M, int N, int K, const double2 *__restrict__ A, int64_t lda,
                                                const double2 *__restrict__ B, int64_t ldb, int kchunk,
                                                double2 *__restrict__ partial, int herm, int bm, int bn, int s) {
    constexpr int NT = WM * WN * 64;
    constexpr int TM = WM * BM * 16, TN = WN * BN * 16;
    constexpr int LA = (TM * KT + NT - 1) / NT, LB = (TN * KT + NT - 1) / NT;   // loads per thread per stage
    __shared__ double2 As[TM][KT + 1];
    __shared__ double2 Bs[TN][KT + 1];
    const int m0 = bm * TM, n0 = bn * TN;
    // herm (A = B): the result is Hermitian, so tiles wholly above the diagonal are left
    // to the reduction, which takes them from their mirror images
    if (herm && n0 > m0 + TM - 1) return;
    const int kbeg = s * kchunk;
    const int kend = min(K, kbeg + kchunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    // Gram matrices A^H A keep the four-product form: identical columns then give
    // identical entries (an exactly singular matrix for dependent bands, which the
    // Cholesky factorisation must see as such)
    constexpr bool G3 = G3OK && BM * BN <= 4 && NT <= 512;
    constexpr int NC3 = G3 ? BN : 1;
    v4d c1[BM][BN], c2[BM][BN], c3[BM][NC3];
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
            c1[i][j] = c2[i][j] = v4d{0, 0, 0, 0};
            if (j < NC3) c3[i][j] = v4d{0, 0, 0, 0};
        }
    double2 ra[LA], rb[LB];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int it = 0; it < LA; ++it) {
            const int e = tid + it * NT, r = e / KT, kk = e % KT, gk = k0 + kk, gm = m0 + r;
            ra[it] = (e < TM * KT && gm < M && gk < kend) ? A[(int64_t)gm * lda + gk] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int it = 0; it < LB; ++it) {
            const int e = tid + it * NT, r = e / KT, kk = e % KT, gk = k0 + kk, gn = n0 + r;
            rb[it] = (e < TN * KT && gn < N && gk < kend) ? B[(int64_t)gn * ldb + gk] : make_double2(0.0, 0.0);
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int it = 0; it < LA; ++it) {
            const int e = tid + it * NT;
            if (e < TM * KT) As[e / KT][e % KT] = ra[it];
        }
#pragma unroll
        for (int it = 0; it < LB; ++it) {
            const int e = tid + it * NT;
            if (e < TN * KT) Bs[e / KT][e % KT] = rb[it];
        }
    };
    if (kbeg < kend) {
        fetch(kbeg);
        stash();
    }
    __syncthreads();
    for (int k0 = kbeg; k0 < kend; k0 += KT) {
        const bool more = k0 + KT < kend;
        if (more) fetch(k0 + KT);
#pragma unroll
        for (int kq = 0; kq < KT / 4; ++kq) {
            const int k = kq * 4 + (lane >> 4);
            double2 a[BM], b[BN];
            double sa[BM], sb[BN];
#pragma unroll
            for (int i = 0; i < BM; ++i) {
                a[i] = As[(wm * BM + i) * 16 + (lane & 15)][k];
                if (CONJA) a[i].y = -a[i].y;
                sa[i] = a[i].x + a[i].y;
            }
#pragma unroll
            for (int j = 0; j < BN; ++j) {
                b[j] = Bs[(wn * BN + j) * 16 + (lane & 15)][k];
                sb[j] = b[j].x + b[j].y;
            }
#pragma unroll
            for (int i = 0; i < BM; ++i)
#pragma unroll
                for (int j = 0; j < BN; ++j)
                    cmfma_blk<G3>(a[i], b[j], sa[i], sb[j], c1[i][j], c2[i][j], c3[i][G3 ? j : 0]);
        }
        __syncthreads();
        if (more) {
            stash();
            __syncthreads();
        }
    }
    double2 *P = partial + (int64_t)s * M * N;
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + (wm * BM + i) * 16 + (lane >> 4) + 4 * v;
                const int col = n0 + (wn * BN + j) * 16 + (lane & 15);
                if (row < M && col < N)
                    P[(int64_t)row * N + col] = cmfma_result<G3>(c1[i][j], c2[i][j], c3[i][G3 ? j : 0], v);
            }
}

template <int WM, int WN, int BM, int BN, bool CONJA, int TAG>
__global__ __launch_bounds__(WM * WN * 64) void zgemm_nt_partial(int M, int N, int K, const double2 *__restrict__ A,
                                                                 int64_t lda, const double2 *__restrict__ B,
                                                                 int64_t ldb, int kchunk,
                                                                 double2 *__restrict__ partial, int herm) {
    nt_partial_tile<WM, WN, BM, BN, CONJA, true>(M, N, K, A, lda, B, ldb, kchunk, partial, herm, blockIdx.x, blockIdx.y,
                                           blockIdx.z);
}

// A Gram matrix A^H A on a one-dimensional grid over the live tiles (on and below the
// diagonal) of every split, live tile fastest.  Workgroups reach the eight XCDs round
// robin in dispatch order, so each XCD gets an equal share of the live tiles; on the
// (tile column, tile row, split) grid XCD x took tile column x, whose live tiles grow
// with x (the last XCD eight times the first's at 1024 bands), and the whole launch
// waited for it.  Each tile and split is the same computation as on that grid.
template <int WM, int WN, int BM, int BN>
__global__ __launch_bounds__(WM * WN * 64) void zgemm_nt_herm(int M, int N, int K, const double2 *__restrict__ A,
                                                              int64_t lda, int kchunk, double2 *__restrict__ partial,
                                                              int live) {
    constexpr int TM = WM * BM * 16, TN = WN * BN * 16;
    const int ntl = (N + TN - 1) / TN;
    const int s = blockIdx.x / live;
    int t = blockIdx.x % live, i = 0;
    for (;; ++i) {
        const int c = min(ntl, (i * TM + TM - 1) / TN + 1);   // live tiles of tile row i
        if (t < c) break;
        t -= c;
    }
    nt_partial_tile<WM, WN, BM, BN, true, false>(M, N, K, A, lda, A, lda, kchunk, partial, 1, i, t, s);
}

// Several independent problems in one launch (one job each, blockIdx.z = job x
// maxsplit + split; jobs whose mask entry is 0 and tiles beyond a job's own
// extent return at once).  Every tile runs the body of the single-problem kernel
// with that job's arguments, so each job's result is bit for bit the same.
template <int WM, int WN, int BM, int BN, bool CONJA, int TAG, bool G3OK>
__global__ __launch_bounds__(WM * WN * 64) void zgemm_nt_partial_jobs(const NtJob *__restrict__ jobs,
                                                                      const int *__restrict__ mask, int maxsplit) {
    constexpr int TM = WM * BM * 16, TN = WN * BN * 16;
    const int q = blockIdx.z / maxsplit, s = blockIdx.z % maxsplit;
    if (!mask[q]) return;
    const NtJob &j = jobs[q];
    if (s >= j.nsplit || (int)blockIdx.x * TM >= j.M || (int)blockIdx.y * TN >= j.N) return;
    nt_partial_tile<WM, WN, BM, BN, CONJA, G3OK>(j.M, j.N, j.K, j.A, j.lda, j.B, j.ldb, j.kchunk, j.partial, j.herm,
                                           blockIdx.x, blockIdx.y, s);
}

// out = alpha * rowscale[m] * sum_s partial[s][m][n] (+ beta * out); TRANS writes out[n][m].
// A workgroup of 256 threads takes 64 consecutive elements: wave g sums the
// splits s = g (mod 4) for each, then wave 0 adds the four sums in order (fixed
// summation order, so the result does not depend on scheduling).  herm: only the
// partials on and below the diagonal exist; an element above it is the conjugate
// of its mirror.
constexpr int kRedElems = 64, kRedGroups = 4;

template <bool TRANS>
__device__ __forceinline__ void reduce_block(int M, int N, int nsplit, const double2 *__restrict__ partial,
                                             double alpha, const double *__restrict__ rowscale, double beta,
                                             double2 *__restrict__ out, int64_t ldo, int herm, int blk) {
    __shared__ double2 sum[kRedGroups][kRedElems];
    const int e = threadIdx.x % kRedElems, g = threadIdx.x / kRedElems;
    const int64_t tot = (int64_t)M * N;
    const int64_t idx = (int64_t)blk * kRedElems + e;
    const int m_ = (int)(idx / N), n_ = (int)(idx % N);
    const bool mirror = herm && n_ > m_;
    const int64_t src = mirror ? (int64_t)n_ * N + m_ : idx;
    double re = 0, im = 0;
    if (idx < tot)
        for (int s = g; s < nsplit; s += kRedGroups) {
            const double2 v = partial[(int64_t)s * tot + src];
            re += v.x;
            im += v.y;
        }
    if (mirror) im = -im;
    sum[g][e] = make_double2(re, im);
    __syncthreads();
    if (g != 0 || idx >= tot) return;
    re = 0;
    im = 0;
#pragma unroll
    for (int q = 0; q < kRedGroups; ++q) {
        re += sum[q][e].x;
        im += sum[q][e].y;
    }
    const int m = (int)(idx / N), n = (int)(idx % N);
    double sc = alpha * (rowscale ? rowscale[m] : 1.0);
    double2 *o = TRANS ? out + (int64_t)n * ldo + m : out + (int64_t)m * ldo + n;
    if (beta != 0.0) {
        *o = make_double2(sc * re + beta * o->x, sc * im + beta * o->y);
    } else {
        *o = make_double2(sc * re, sc * im);
    }
}

template <bool TRANS>
__global__ __launch_bounds__(kRedElems * kRedGroups) void reduce_partial(int M, int N, int nsplit,
                                                                         const double2 *__restrict__ partial,
                                                                         double alpha,
                                                                         const double *__restrict__ rowscale,
                                                                         double beta, double2 *__restrict__ out,
                                                                         int64_t ldo, int herm) {
    reduce_block<TRANS>(M, N, nsplit, partial, alpha, rowscale, beta, out, ldo, herm, blockIdx.x);
}

template <bool TRANS>
__global__ __launch_bounds__(kRedElems * kRedGroups) void reduce_partial_jobs(const NtJob *__restrict__ jobs,
                                                                              const int *__restrict__ mask) {
    if (!mask[blockIdx.y]) return;
    const NtJob &j = jobs[blockIdx.y];
    if ((int64_t)blockIdx.x * kRedElems >= (int64_t)j.M * j.N) return;
    reduce_block<TRANS>(j.M, j.N, j.nsplit, j.partial, j.alpha, j.rowscale, j.beta, j.C, j.ldc, j.herm, blockIdx.x);
}

// ---------------------------------------------------------------------------
// NN: Out_z[m][j] = alpha * sum_k W[m][k] X_z[k][j] + beta * Out_z[m][j]
// for up to 4 (X_z, Out_z) pairs sharing W (blockIdx.z).  Waves WM x WJ, each
// BM x BJ blocks of 16 x 16; KD-deep LDS stages (a multiple of 4).
// ---------------------------------------------------------------------------
struct NNBatch {
    const double2 *X[4];
    double2 *Out[4];
};

template <int WM, int WJ, int BM, int BJ, int KD>
__device__ __forceinline__ void nn_tile(int M, int J, int K, const double2 *__restrict__ W, int64_t ldw,
                                        const double2 *__restrict__ X, double2 *__restrict__ Out, int64_t ldx,
                                        double alpha, double beta, int64_t ldo, int lower, int bj, int bm) {
    constexpr int NT = WM * WJ * 64;
    constexpr int TM = WM * BM * 16, TJ = WJ * BJ * 16;
    constexpr int LW = (TM * KD + NT - 1) / NT, LX = (KD * TJ + NT - 1) / NT;
    __shared__ double2 Ws[TM][KD + 1];
    __shared__ double2 Xs[KD][TJ + 1];
    const int j0 = bj * TJ, m0 = bm * TM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wj = wave / WM;
    constexpr bool G3 = BM * BJ <= 4 && NT <= 512;
    constexpr int NC3 = G3 ? BJ : 1;
    v4d c1[BM][BJ], c2[BM][BJ], c3[BM][NC3];
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j) {
            c1[i][j] = c2[i][j] = v4d{0, 0, 0, 0};
            if (j < NC3) c3[i][j] = v4d{0, 0, 0, 0};
        }
    double2 rw[LW], rx[LX];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int it = 0; it < LW; ++it) {
            const int e = tid + it * NT, r = e / KD, kk = e % KD, gm = m0 + r, gk = k0 + kk;
            rw[it] = (e < TM * KD && gm < M && gk < K) ? W[(int64_t)gm * ldw + gk] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int it = 0; it < LX; ++it) {
            const int e = tid + it * NT, kk = e / TJ, c = e % TJ, gk = k0 + kk, gj = j0 + c;
            rx[it] = (e < KD * TJ && gk < K && gj < J) ? X[(int64_t)gk * ldx + gj] : make_double2(0.0, 0.0);
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int it = 0; it < LW; ++it) {
            const int e = tid + it * NT;
            if (e < TM * KD) Ws[e / KD][e % KD] = rw[it];
        }
#pragma unroll
        for (int it = 0; it < LX; ++it) {
            const int e = tid + it * NT;
            if (e < KD * TJ) Xs[e / TJ][e % TJ] = rx[it];
        }
    };
    // lower: W is lower triangular (zero above the diagonal), so this row tile's
    // products end at its last row; the skipped terms are exact zeros
    const int kend = lower ? min(K, m0 + TM) : K;
    if (kend > 0) {
        fetch(0);
        stash();
    }
    __syncthreads();
    for (int k0 = 0; k0 < kend; k0 += KD) {
        const bool more = k0 + KD < kend;
        if (more) fetch(k0 + KD);
#pragma unroll
        for (int kq = 0; kq < KD / 4; ++kq) {
            const int k = kq * 4 + (lane >> 4);
            double2 a[BM], b[BJ];
            double sa[BM], sb[BJ];
#pragma unroll
            for (int i = 0; i < BM; ++i) {
                a[i] = Ws[(wm * BM + i) * 16 + (lane & 15)][k];
                sa[i] = a[i].x + a[i].y;
            }
#pragma unroll
            for (int j = 0; j < BJ; ++j) {
                b[j] = Xs[k][(wj * BJ + j) * 16 + (lane & 15)];
                sb[j] = b[j].x + b[j].y;
            }
#pragma unroll
            for (int i = 0; i < BM; ++i)
#pragma unroll
                for (int j = 0; j < BJ; ++j)
                    cmfma_blk<G3>(a[i], b[j], sa[i], sb[j], c1[i][j], c2[i][j], c3[i][G3 ? j : 0]);
        }
        __syncthreads();
        if (more) {
            stash();
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + (wm * BM + i) * 16 + (lane >> 4) + 4 * v;
                const int col = j0 + (wj * BJ + j) * 16 + (lane & 15);
                if (row < M && col < J) {
                    double2 *o = Out + (int64_t)row * ldo + col;
                    const double2 r = cmfma_result<G3>(c1[i][j], c2[i][j], c3[i][G3 ? j : 0], v);
                    double re = alpha * r.x, im = alpha * r.y;
                    if (beta != 0.0) { re += beta * o->x; im += beta * o->y; }
                    *o = make_double2(re, im);
                }
            }
}

template <int WM, int WJ, int BM, int BJ, int TAG, int KD>
__global__ __launch_bounds__(WM * WJ * 64) void zgemm_nn_kernel(int M, int J, int K, const double2 *__restrict__ W,
                                                                int64_t ldw, NNBatch bt, int64_t ldx, double alpha,
                                                                double beta, int64_t ldo, int lower) {
    nn_tile<WM, WJ, BM, BJ, KD>(M, J, K, W, ldw, bt.X[blockIdx.z], bt.Out[blockIdx.z], ldx, alpha, beta, ldo, lower,
                                blockIdx.x, blockIdx.y);
}

// several problems in one launch: blockIdx.z = job x 4 + block of the job
template <int WM, int WJ, int BM, int BJ, int TAG, int KD>
__global__ __launch_bounds__(WM * WJ * 64) void zgemm_nn_jobs(const NnJob *__restrict__ jobs,
                                                             const int *__restrict__ mask) {
    constexpr int TM = WM * BM * 16, TJ = WJ * BJ * 16;
    const int q = blockIdx.z / 4, z = blockIdx.z % 4;
    if (!mask[q]) return;
    const NnJob &j = jobs[q];
    if (z >= j.nz || (int)blockIdx.x * TJ >= j.J || (int)blockIdx.y * TM >= j.M) return;
    nn_tile<WM, WJ, BM, BJ, KD>(j.M, j.J, j.K, j.W, j.ldw, j.X[z], j.Out[z], j.ldx, j.alpha, j.beta, j.ldo, j.lower,
                                blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// host wrappers
// ---------------------------------------------------------------------------
// NT tiles: TN = 16 (N <= 16), 32 (N <= 32), 64 (N <= 64), 128 (N <= 128) or 144
// (N <= 144, for 128 wanted bands plus buffer bands), else 128 for a Gram matrix and
// 64 for other products (their four blocks per wave take the three-product form); TM = 128
// rows of A when A is tall (the projector table: B is then re-read half as often)
// or of a square band-by-band product of up to 128 (Gram matrices: one tile); 48
// for square products of 129..144 (three waves of 3 x 3 blocks, 48 x 144 tiles),
// else 64.  The narrow tiles serve a few right-hand sides against the whole table,
// where a 64-wide tile would spend most of its matrix-core work on padding.
static int nt_tn(int M, int N, bool herm) {
    // beyond 144 bands, products other than Gram matrices: tiles 64 columns wide, whose four
    // blocks per wave take the three-product form
    if (!herm && N > 144) return 64;
    // square products of at most 128 bands (the block algebra of up to 128 bands): 64 x 64
    // tiles, whose four blocks per wave take the three-product form outside Gram matrices
    if (M == N && N > 64 && N <= 128) return 64;
    // tall products of 128 bands (the projection of 128 bands onto 512 or more projectors)
    if (!herm && M >= 512 && N == 128) return 64;
    return N <= 16 ? 16 : (N <= 32 ? 32 : (N <= 64 ? 64 : (N <= 128 ? 128 : (N <= 144 ? 144 : 128))));
}
static int nt_tm(int M, int N) {
    if (N <= 32) return M >= 512 ? 128 : 64;
    if (M == N && M > 128 && M <= 144) return 48;
    return (M >= 256 && N > 64) ? 128 : 64;
}

// tile shape of an NT product (batched NT jobs of one launch must share it)
int nt_tile_id(int M, int N, bool herm) { return nt_tm(M, N) * 1024 + nt_tn(M, N, herm); }

// tiles of a Gram matrix's tile grid that reach the diagonal
static int nt_live_tiles(int M, int N) {
    const int tn = nt_tn(M, N, true), tm = nt_tm(M, N);
    const int mt = (M + tm - 1) / tm, ntl = (N + tn - 1) / tn;
    int live = 0;
    for (int i = 0; i < mt; ++i) live += std::min(ntl, (i * tm + tm - 1) / tn + 1);
    return live;
}

// K-splits: enough workgroups to cover the chip (~512, two per compute unit) while
// keeping at least four LDS stages per chunk and the partial sums under 64 MiB
// (128 MiB for a Gram matrix).  Other than for a Gram matrix the count is the one
// with the least time per split in rounds of 512 workgroups: a split count just
// past a whole round leaves a short last round (96 tiles x 6 splits = 576
// workgroups ran at about half the speed of 96 x 5).
int nt_splits(int M, int N, int K, bool herm) {
    const int tn = nt_tn(M, N, herm), tm = nt_tm(M, N);
    const int mt = (M + tm - 1) / tm, ntl = (N + tn - 1) / tn;
    const int tiles = mt * ntl;
    int s = (512 + tiles - 1) / tiles;
    if (!herm) {
        const int64_t cap = ((int64_t)64 << 20) / ((int64_t)M * N * (int64_t)sizeof(double2));
        const int hi = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)s, (K + 4 * KT - 1) / (4 * KT), cap}));
        int best = 1;
        double bcost = 2.0;
        for (int c = 1; c <= hi; ++c) {
            const double cost = (double)(((int64_t)tiles * c + 511) / 512) / c;
            if (cost < bcost * (1.0 - 1e-9)) {
                bcost = cost;
                best = c;
            }
        }
        return best;
    }
    {
        // a Gram matrix computes only the tiles that reach the diagonal: as many
        // splits as fill the 256 compute units once (a second workgroup on a unit
        // halves the speed of both)
        const int live = nt_live_tiles(M, N);
        if (live * 2 <= 256) s = std::min(s, std::max(1, 256 / live));
        else s = std::min(s, std::max(1, 512 / live));
    }
    const int maxs = (K + 4 * KT - 1) / (4 * KT);
    if (s > maxs) s = maxs;
    const int64_t cap = ((int64_t)(herm ? 128 : 64) << 20) / ((int64_t)M * N * (int64_t)sizeof(double2));
    if (s > cap) s = (int)cap;
    if (s < 1) s = 1;
    return s;
}

size_t nt_partial_bytes(int M, int N, int K) {
    const int s = std::max(nt_splits(M, N, K, false), M == N ? nt_splits(M, N, K, true) : 1);
    return (size_t)s * M * N * sizeof(double2);
}

template <int WM, int WN, int BM, int BN>
static void nt_go(dim3 grid, bool conja, bool proj, hipStream_t st, int M, int N, int K, const void *A, int64_t lda,
                  const void *B, int64_t ldb, int kchunk, void *partial, int herm) {
    const dim3 blk(WM * WN * 64);
    if (herm) {
        const int live = nt_live_tiles(M, N);
        hipLaunchKernelGGL((zgemm_nt_herm<WM, WN, BM, BN>), dim3((unsigned)(live * grid.z)), blk, 0, st, M, N, K,
                           (const double2 *)A, lda, kchunk, (double2 *)partial, live);
    } else if (conja && proj)
        hipLaunchKernelGGL((zgemm_nt_partial<WM, WN, BM, BN, true, 1>), grid, blk, 0, st, M, N, K, (const double2 *)A,
                           lda, (const double2 *)B, ldb, kchunk, (double2 *)partial, herm);
    else if (conja)
        hipLaunchKernelGGL((zgemm_nt_partial<WM, WN, BM, BN, true, 0>), grid, blk, 0, st, M, N, K, (const double2 *)A,
                           lda, (const double2 *)B, ldb, kchunk, (double2 *)partial, herm);
    else
        hipLaunchKernelGGL((zgemm_nt_partial<WM, WN, BM, BN, false, 0>), grid, blk, 0, st, M, N, K,
                           (const double2 *)A, lda, (const double2 *)B, ldb, kchunk, (double2 *)partial, herm);
}

// C (M x N, ldc) = alpha * rowscale o (op(A) B^T) (+ beta C); trans: write C^T (N x M)
void zgemm_nt(int M, int N, int K, bool conja, const void *A, int64_t lda, const void *B, int64_t ldb,
              double alpha, const double *rowscale, double beta, void *C, int64_t ldc, bool trans, void *partial,
              hipStream_t st, bool proj, bool herm_in) {
    if (M <= 0 || N <= 0) return;
    // a Gram matrix A^H A: half the tiles (alpha real, no row scale)
    const int herm = (herm_in && conja && A == B && lda == ldb && M == N && !rowscale) ? 1 : 0;
    const int ns = nt_splits(M, N, K, herm != 0);
    int kchunk = (K + ns - 1) / ns;
    kchunk = ((kchunk + KT - 1) / KT) * KT;
    const int nsplit = K > 0 ? (K + kchunk - 1) / kchunk : 1;
    const int tn = nt_tn(M, N, herm != 0), tm = nt_tm(M, N);
    dim3 grid((M + tm - 1) / tm, (N + tn - 1) / tn, nsplit);
    if (K <= 0) fill_zero(partial, (size_t)M * N * sizeof(double2), st);
    else if (tn == 16 && tm == 128) nt_go<4, 1, 2, 1>(grid, conja, proj, st, M, N, K, A, lda, B, ldb, kchunk, partial, herm);
    else if (tn == 16) nt_go<4, 1, 1, 1>(grid, conja, proj, st, M, N, K, A, lda, B, ldb, kchunk, partial, herm);
    else if (tn == 32 && tm == 128) nt_go<4, 1, 2, 2>(grid, conja, proj, st, M, N, K, A, lda, B, ldb, kchunk, partial, herm);
    else if (tn == 32) nt_go<4, 1, 1, 2>(grid, conja, proj, st, M, N, K, A, lda, B, ldb, kchunk, partial, herm);
    else if (tn == 64 && tm == 128) nt_go<4, 2, 2, 2>(grid, conja, proj, st, M, N, K, A, lda, B, ldb, kchunk, partial, herm);
    else if (tn == 64) nt_go<2, 2, 2, 2>(grid, conja, proj, st, M, N, K, A, lda, B, ldb, kchunk, partial, herm);
    else if (tm == 48) nt_go<1, 3, 3, 3>(grid, conja, proj, st, M, N, K, A, lda, B, ldb, kchunk, partial, herm);
    else if (tm == 128 && tn == 128) nt_go<4, 2, 2, 4>(grid, conja, proj, st, M, N, K, A, lda, B, ldb, kchunk, partial, herm);
    else if (tm == 128) nt_go<4, 3, 2, 3>(grid, conja, proj, st, M, N, K, A, lda, B, ldb, kchunk, partial, herm);
    else if (tn == 128) nt_go<2, 2, 2, 4>(grid, conja, proj, st, M, N, K, A, lda, B, ldb, kchunk, partial, herm);
    else nt_go<2, 3, 2, 3>(grid, conja, proj, st, M, N, K, A, lda, B, ldb, kchunk, partial, herm);
    PW_LAUNCH_CHECK();
    const int64_t tot = (int64_t)M * N;
    const int nblk = (int)((tot + kRedElems - 1) / kRedElems);
    const dim3 rblk(kRedElems * kRedGroups);
    if (trans)
        hipLaunchKernelGGL((reduce_partial<true>), dim3(nblk), rblk, 0, st, M, N, nsplit, (const double2 *)partial,
                           alpha, rowscale, beta, (double2 *)C, ldc, herm);
    else
        hipLaunchKernelGGL((reduce_partial<false>), dim3(nblk), rblk, 0, st, M, N, nsplit, (const double2 *)partial,
                           alpha, rowscale, beta, (double2 *)C, ldc, herm);
    PW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Batched launches over independent problems (one job each): the tile shape and
// split-K chunking of every job are those zgemm_nt / zgemm_nn_batch would pick for
// it alone, so each job's result is bit for bit that of its own call.
// ---------------------------------------------------------------------------
NtJob nt_job(int M, int N, int K, bool conja, const void *A, int64_t lda, const void *B, int64_t ldb, double alpha,
             const double *rowscale, double beta, void *C, int64_t ldc, void *partial, bool herm_in) {
    PW_CHECK(M > 0 && N > 0 && K > 0, PW_EINVAL, "batched NT GEMM needs positive sizes");
    NtJob j{};
    j.M = M; j.N = N; j.K = K;
    j.herm = (herm_in && conja && A == B && lda == ldb && M == N && !rowscale) ? 1 : 0;
    const int ns = nt_splits(M, N, K, j.herm != 0);
    j.kchunk = ((K + ns - 1) / ns + KT - 1) / KT * KT;
    j.nsplit = (K + j.kchunk - 1) / j.kchunk;
    j.A = (const double2 *)A; j.lda = lda;
    j.B = (const double2 *)B; j.ldb = ldb;
    j.alpha = alpha; j.beta = beta; j.rowscale = rowscale;
    j.C = (double2 *)C; j.ldc = ldc;
    j.partial = (double2 *)partial;
    return j;
}

template <int WM, int WN, int BM, int BN>
static void nt_jobs_go(dim3 grid, bool conja, bool proj, bool herm, hipStream_t st, const NtJob *jobs,
                       const int *mask, int maxsplit) {
    const dim3 blk(WM * WN * 64);
    if (herm)
        hipLaunchKernelGGL((zgemm_nt_partial_jobs<WM, WN, BM, BN, true, 0, false>), grid, blk, 0, st, jobs, mask,
                           maxsplit);
    else if (conja && proj)
        hipLaunchKernelGGL((zgemm_nt_partial_jobs<WM, WN, BM, BN, true, 1, true>), grid, blk, 0, st, jobs, mask,
                           maxsplit);
    else if (conja)
        hipLaunchKernelGGL((zgemm_nt_partial_jobs<WM, WN, BM, BN, true, 0, true>), grid, blk, 0, st, jobs, mask,
                           maxsplit);
    else
        hipLaunchKernelGGL((zgemm_nt_partial_jobs<WM, WN, BM, BN, false, 0, true>), grid, blk, 0, st, jobs, mask,
                           maxsplit);
}

void zgemm_nt_jobs(const std::vector<NtJob> &h, const NtJob *d_jobs, const int *d_mask, bool conja, bool trans,
                   bool proj, hipStream_t st) {
    // jobs with M = 0 are placeholders (a problem without such a product): skipped
    const NtJob *first = nullptr;
    for (const NtJob &j : h)
        if (j.M > 0 && !first) first = &j;
    if (!first) return;
    const int tn = nt_tn(first->M, first->N, first->herm != 0), tm = nt_tm(first->M, first->N);
    int maxsplit = 1, mt = 1, ntl = 1;
    int64_t maxel = 1;
    for (const NtJob &j : h) {
        if (j.M <= 0) continue;
        PW_CHECK(nt_tn(j.M, j.N, j.herm != 0) == tn && nt_tm(j.M, j.N) == tm, PW_EINVAL,
                 "batched NT jobs need one tile shape");
        maxsplit = std::max(maxsplit, j.nsplit);
        mt = std::max(mt, (j.M + tm - 1) / tm);
        ntl = std::max(ntl, (j.N + tn - 1) / tn);
        maxel = std::max(maxel, (int64_t)j.M * j.N);
    }
    // the jobs of one call are all Gram matrices or none (the same product in every problem)
    bool herm = false;
    for (const NtJob &j : h)
        if (j.M > 0) {
            PW_CHECK(j.herm == first->herm, PW_EINVAL, "batched NT jobs mix Gram and other products");
            herm = j.herm != 0;
        }
    dim3 grid(mt, ntl, (unsigned)(h.size() * maxsplit));
    if (tn == 16 && tm == 128) nt_jobs_go<4, 1, 2, 1>(grid, conja, proj, herm, st, d_jobs, d_mask, maxsplit);
    else if (tn == 16) nt_jobs_go<4, 1, 1, 1>(grid, conja, proj, herm, st, d_jobs, d_mask, maxsplit);
    else if (tn == 32 && tm == 128) nt_jobs_go<4, 1, 2, 2>(grid, conja, proj, herm, st, d_jobs, d_mask, maxsplit);
    else if (tn == 32) nt_jobs_go<4, 1, 1, 2>(grid, conja, proj, herm, st, d_jobs, d_mask, maxsplit);
    else if (tn == 64 && tm == 128) nt_jobs_go<4, 2, 2, 2>(grid, conja, proj, herm, st, d_jobs, d_mask, maxsplit);
    else if (tn == 64) nt_jobs_go<2, 2, 2, 2>(grid, conja, proj, herm, st, d_jobs, d_mask, maxsplit);
    else if (tm == 48) nt_jobs_go<1, 3, 3, 3>(grid, conja, proj, herm, st, d_jobs, d_mask, maxsplit);
    else if (tm == 128 && tn == 128) nt_jobs_go<4, 2, 2, 4>(grid, conja, proj, herm, st, d_jobs, d_mask, maxsplit);
    else if (tm == 128) nt_jobs_go<4, 3, 2, 3>(grid, conja, proj, herm, st, d_jobs, d_mask, maxsplit);
    else if (tn == 128) nt_jobs_go<2, 2, 2, 4>(grid, conja, proj, herm, st, d_jobs, d_mask, maxsplit);
    else nt_jobs_go<2, 3, 2, 3>(grid, conja, proj, herm, st, d_jobs, d_mask, maxsplit);
    PW_LAUNCH_CHECK();
    const dim3 rgrid((unsigned)((maxel + kRedElems - 1) / kRedElems), (unsigned)h.size());
    const dim3 rblk(kRedElems * kRedGroups);
    if (trans) hipLaunchKernelGGL((reduce_partial_jobs<true>), rgrid, rblk, 0, st, d_jobs, d_mask);
    else hipLaunchKernelGGL((reduce_partial_jobs<false>), rgrid, rblk, 0, st, d_jobs, d_mask);
    PW_LAUNCH_CHECK();
}

template <int WM, int WJ, int BM, int BJ, int KD = KT>
static void nn_go(int nz, bool proj, hipStream_t st, int M, int J, int K, const void *W, int64_t ldw,
                  const NNBatch &bt, int64_t ldx, double alpha, double beta, int64_t ldo, int lower) {
    static_assert(KD % 4 == 0, "LDS stage depth");
    constexpr int TM = WM * BM * 16, TJ = WJ * BJ * 16;
    dim3 grid((J + TJ - 1) / TJ, (M + TM - 1) / TM, nz);
    const dim3 blk(WM * WJ * 64);
    if (proj)
        hipLaunchKernelGGL((zgemm_nn_kernel<WM, WJ, BM, BJ, 1, KD>), grid, blk, 0, st, M, J, K, (const double2 *)W, ldw,
                           bt, ldx, alpha, beta, ldo, lower);
    else
        hipLaunchKernelGGL((zgemm_nn_kernel<WM, WJ, BM, BJ, 0, KD>), grid, blk, 0, st, M, J, K, (const double2 *)W, ldw,
                           bt, ldx, alpha, beta, ldo, lower);
}

// Out_z (M x J, ldo) = alpha * W (M x K, ldw) . X_z (K x J, ldx) + beta * Out_z, z < nz <= 4
// Default tiles: 16 x 64 (M <= 16), 32 x 32 (M <= 32), 64 (M <= 64), 144 (128 < M <= 144), else 128 rows.
// NN tile configurations (waves over rows x columns, 16 x 16 blocks per wave)
// the autotuner chooses between; id: {WM, WJ, BM, BJ, KD}, tile (16 WM BM) x
// (16 WJ BJ), KD-deep stages.  A workgroup of 9 waves leaves one SIMD with three
// waves and the others with two; the 12-wave 144-row tiles spread evenly.  Tiles
// 12 and 13 (16 x 64 and 32 x 32, one 16 x 16 block per wave) serve a few
// right-hand sides against the table: many small workgroups keep every CU
// streaming it (8 bands: 134 us against 446 us for the 64-row tile and 222 us
// for a 16 x 256 tile on the 0.79 GB table).
static const int kNnCfg[kNnCfgs][5] = {{2, 2, 2, 2, 16}, {4, 1, 2, 4, 16}, {9, 1, 1, 4, 16}, {4, 2, 2, 2, 16},
                                       {8, 1, 1, 4, 16}, {4, 1, 2, 2, 16}, {2, 4, 2, 2, 16}, {9, 1, 1, 4, 8},
                                       {3, 2, 3, 2, 8},  {8, 1, 1, 4, 8},  {3, 4, 3, 2, 8},  {3, 4, 3, 1, 8},
                                       {1, 4, 1, 1, 16}, {2, 2, 1, 1, 16}};

int nn_default_cfg(int M) { return M <= 16 ? 12 : M <= 32 ? 13 : M <= 64 ? 0 : (M > 128 && M <= 144) ? 11 : 9; }

void nn_cfg_shape(int id, int &tm, int &tj, int &nthr) {
    PW_CHECK(id >= 0 && id < kNnCfgs, PW_EINVAL, "NN tile %d unknown", id);
    const int *c = kNnCfg[id];
    tm = 16 * c[0] * c[2];
    tj = 16 * c[1] * c[3];
    nthr = 64 * c[0] * c[1];
}

void zgemm_nn_batch(int nz, int M, int J, int K, const void *W, int64_t ldw, const void *const *X, int64_t ldx,
                    double alpha, double beta, void *const *Out, int64_t ldo, hipStream_t st, bool proj, int cfg,
                    bool lower) {
    const int lw = lower ? 1 : 0;
    if (M <= 0 || J <= 0 || nz <= 0) return;
    PW_CHECK(nz <= 4, PW_EINVAL, "at most 4 blocks per batched rotation");
    NNBatch bt{};
    for (int z = 0; z < nz; ++z) {
        bt.X[z] = (const double2 *)X[z];
        bt.Out[z] = (double2 *)Out[z];
    }
    if (cfg < 0) cfg = nn_default_cfg(M);
    switch (cfg) {
        case 0: nn_go<2, 2, 2, 2>(nz, proj, st, M, J, K, W, ldw, bt, ldx, alpha, beta, ldo, lw); break;
        case 1: nn_go<4, 1, 2, 4>(nz, proj, st, M, J, K, W, ldw, bt, ldx, alpha, beta, ldo, lw); break;
        case 2: nn_go<9, 1, 1, 4>(nz, proj, st, M, J, K, W, ldw, bt, ldx, alpha, beta, ldo, lw); break;
        case 3: nn_go<4, 2, 2, 2>(nz, proj, st, M, J, K, W, ldw, bt, ldx, alpha, beta, ldo, lw); break;
        case 4: nn_go<8, 1, 1, 4>(nz, proj, st, M, J, K, W, ldw, bt, ldx, alpha, beta, ldo, lw); break;
        case 5: nn_go<4, 1, 2, 2>(nz, proj, st, M, J, K, W, ldw, bt, ldx, alpha, beta, ldo, lw); break;
        case 6: nn_go<2, 4, 2, 2>(nz, proj, st, M, J, K, W, ldw, bt, ldx, alpha, beta, ldo, lw); break;
        case 7: nn_go<9, 1, 1, 4, 8>(nz, proj, st, M, J, K, W, ldw, bt, ldx, alpha, beta, ldo, lw); break;
        case 8: nn_go<3, 2, 3, 2, 8>(nz, proj, st, M, J, K, W, ldw, bt, ldx, alpha, beta, ldo, lw); break;
        case 9: nn_go<8, 1, 1, 4, 8>(nz, proj, st, M, J, K, W, ldw, bt, ldx, alpha, beta, ldo, lw); break;
        case 10: nn_go<3, 4, 3, 2, 8>(nz, proj, st, M, J, K, W, ldw, bt, ldx, alpha, beta, ldo, lw); break;
        case 11: nn_go<3, 4, 3, 1, 8>(nz, proj, st, M, J, K, W, ldw, bt, ldx, alpha, beta, ldo, lw); break;
        case 12: nn_go<1, 4, 1, 1>(nz, proj, st, M, J, K, W, ldw, bt, ldx, alpha, beta, ldo, lw); break;
        case 13: nn_go<2, 2, 1, 1>(nz, proj, st, M, J, K, W, ldw, bt, ldx, alpha, beta, ldo, lw); break;
        default: PW_CHECK(false, PW_EINVAL, "NN tile %d unknown", cfg);
    }
    PW_LAUNCH_CHECK();
}

template <int WM, int WJ, int BM, int BJ, int KD = KT>
static void nn_jobs_go(int njobs, int maxM, int maxJ, bool proj, hipStream_t st, const NnJob *jobs, const int *mask) {
    constexpr int TM = WM * BM * 16, TJ = WJ * BJ * 16;
    dim3 grid((maxJ + TJ - 1) / TJ, (maxM + TM - 1) / TM, 4 * njobs);
    const dim3 blk(WM * WJ * 64);
    if (proj) hipLaunchKernelGGL((zgemm_nn_jobs<WM, WJ, BM, BJ, 1, KD>), grid, blk, 0, st, jobs, mask);
    else hipLaunchKernelGGL((zgemm_nn_jobs<WM, WJ, BM, BJ, 0, KD>), grid, blk, 0, st, jobs, mask);
}

void zgemm_nn_jobs_launch(const std::vector<NnJob> &h, const NnJob *d_jobs, const int *d_mask, int cfg, bool proj,
                          hipStream_t st) {
    // jobs with nz = 0 are placeholders: skipped
    int maxM = 0, maxJ = 0, m0 = 0;
    for (const NnJob &j : h) {
        if (j.nz == 0) continue;
        PW_CHECK(j.nz <= 4 && j.M > 0 && j.J > 0, PW_EINVAL, "bad batched NN job");
        if (!maxM) m0 = j.M;
        PW_CHECK(nn_default_cfg(j.M) == nn_default_cfg(m0), PW_EINVAL, "NN jobs differ in tile");
        maxM = std::max(maxM, j.M);
        maxJ = std::max(maxJ, j.J);
    }
    if (!maxM) return;
    if (cfg < 0) cfg = nn_default_cfg(m0);
    const int n = (int)h.size();
    switch (cfg) {
        case 0: nn_jobs_go<2, 2, 2, 2>(n, maxM, maxJ, proj, st, d_jobs, d_mask); break;
        case 1: nn_jobs_go<4, 1, 2, 4>(n, maxM, maxJ, proj, st, d_jobs, d_mask); break;
        case 2: nn_jobs_go<9, 1, 1, 4>(n, maxM, maxJ, proj, st, d_jobs, d_mask); break;
        case 3: nn_jobs_go<4, 2, 2, 2>(n, maxM, maxJ, proj, st, d_jobs, d_mask); break;
        case 4: nn_jobs_go<8, 1, 1, 4>(n, maxM, maxJ, proj, st, d_jobs, d_mask); break;
        case 5: nn_jobs_go<4, 1, 2, 2>(n, maxM, maxJ, proj, st, d_jobs, d_mask); break;
        case 6: nn_jobs_go<2, 4, 2, 2>(n, maxM, maxJ, proj, st, d_jobs, d_mask); break;
        case 7: nn_jobs_go<9, 1, 1, 4, 8>(n, maxM, maxJ, proj, st, d_jobs, d_mask); break;
        case 8: nn_jobs_go<3, 2, 3, 2, 8>(n, maxM, maxJ, proj, st, d_jobs, d_mask); break;
        case 9: nn_jobs_go<8, 1, 1, 4, 8>(n, maxM, maxJ, proj, st, d_jobs, d_mask); break;
        case 10: nn_jobs_go<3, 4, 3, 2, 8>(n, maxM, maxJ, proj, st, d_jobs, d_mask); break;
        case 11: nn_jobs_go<3, 4, 3, 1, 8>(n, maxM, maxJ, proj, st, d_jobs, d_mask); break;
        case 12: nn_jobs_go<1, 4, 1, 1>(n, maxM, maxJ, proj, st, d_jobs, d_mask); break;
        case 13: nn_jobs_go<2, 2, 1, 1>(n, maxM, maxJ, proj, st, d_jobs, d_mask); break;
        default: PW_CHECK(false, PW_EINVAL, "NN tile %d unknown", cfg);
    }
    PW_LAUNCH_CHECK();
}

void zgemm_nn_launch(int M, int J, int K, const void *W, int64_t ldw, const void *X, int64_t ldx, double alpha,
                     double beta, void *Out, int64_t ldo, hipStream_t st, bool proj, int cfg, bool lower) {
    const void *xs[1] = {X};
    void *os[1] = {Out};
    zgemm_nn_batch(1, M, J, K, W, ldw, xs, ldx, alpha, beta, os, ldo, st, proj, cfg, lower);
}

}  // namespace pw
