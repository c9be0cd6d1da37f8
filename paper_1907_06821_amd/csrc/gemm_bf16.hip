// Mixed-precision projector GEMMs: BF16 operands, FP32 accumulation on gfx950
// matrix cores (v_mfma_f32_16x16x32_bf16), complex64 wave functions.
//
//   projection      projT[b][p] = D_p sum_G conj(beta_p(G)) psi_b(G)     (split-K)
//   back-projection out[b][G]  += sum_p projT[b][p] beta_p(G)
//
// Tables (built once per context, zero padded):
//   beta   planes nproj x ldg   (ldg = npw rounded up to 64)   projection operand
//   betaT  planes ldg x ldp     (ldp = nproj rounded up to 64) back-projection operand
// Per H psi the wave functions are rounded once to BF16 planes nb x ldg, and the
// projection's reduction writes D . C directly as BF16 planes nb x ldp.
//
// Contexts of up to 144 bands keep every plane row-major, so that each MFMA
// operand fragment (8 consecutive k of one row) is one 16-byte load; workgroup
// tiles span all bands of the call, each table is read once per H psi, the band
// operand is staged in LDS and the table fragments go straight into registers.
// Contexts of more than 144 bands store every plane in 16-row panels
// (bf16_panel_index): 16 rows by 32 k as one 1 KB fragment in the matrix cores'
// lane order, a panel's fragments in k order.  Their kernels (the ring kernels
// below) copy whole fragments from memory into LDS, tiles of 256 bands, so each
// table is read once per 256 bands.  Rounding is to nearest even.
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

__device__ inline bf16x8 load8(const uint16_t *p) { return *reinterpret_cast<const bf16x8 *>(p); }
__device__ inline bf16x8 zero8() {
    union { bf16x8 b; uint4 u; } x;
    x.u = make_uint4(0, 0, 0, 0);
    return x.b;
}

constexpr int KS = 64;          // k-depth per LDS stage
constexpr int LPAD = KS + 8;    // padded LDS row (bf16 elements, 144 bytes)
constexpr int MAXNB = 144;      // largest band tile (9 blocks of 16)

int64_t bf16_ld(int n) { return ((int64_t)n + 63) / 64 * 64; }

// ---------------------------------------------------------------------------
// complex64 rows -> row-major BF16 planes of rows x ldp, zero beyond n
// ---------------------------------------------------------------------------
__global__ void k_c64_to_planes(int rows, int n, const float2 *__restrict__ src, int64_t lds, int64_t ldp,
                                uint16_t *__restrict__ re, uint16_t *__restrict__ im) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (g >= ldp) return;
    const float2 v = g < n ? src[(int64_t)r * lds + g] : make_float2(0.f, 0.f);
    const int64_t o = (int64_t)r * ldp + g;
    re[o] = f2bf(v.x);
    im[o] = f2bf(v.y);
}

// complex64 rows -> BF16 planes in 16-row panels: a workgroup takes 16 rows x 256
// columns, converts them through LDS (row reads coalesced) and writes its eight 1 KB
// panel blocks per plane as whole 16-byte runs (consecutive threads, consecutive
// runs); zero beyond n, rows beyond `rows` left alone
__global__ __launch_bounds__(256) void k_c64_to_panels(int rows, int n, const float2 *__restrict__ src, int64_t lds,
                                                       int64_t ldp, uint16_t *__restrict__ re,
                                                       uint16_t *__restrict__ im) {
    __shared__ uint4 tre[16][32], tim[16][32];            // [row][run of 8 columns]
    uint16_t *lre = reinterpret_cast<uint16_t *>(&tre[0][0]), *lim = reinterpret_cast<uint16_t *>(&tim[0][0]);
    const int t = threadIdx.x, r0 = blockIdx.y * 16;
    const int64_t k0 = (int64_t)blockIdx.x * 256, k = k0 + t;
#pragma unroll 4
    for (int i = 0; i < 16; ++i) {
        const int r = r0 + i;
        const float2 v = r < rows && k < n ? src[(int64_t)r * lds + k] : make_float2(0.f, 0.f);
        lre[i * 256 + t] = f2bf(v.x);
        lim[i * 256 + t] = f2bf(v.y);
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int id = t + 256 * h, q = id & 63;
        const int i = q & 15, run = (id >> 6) * 4 + (q >> 4);   // panel block id >> 6, run q within it
        const int r = r0 + i;
        const int64_t kk = k0 + run * 8;
        if (r >= rows || kk >= ldp) continue;
        const int64_t o = bf16_panel_index(r, kk, ldp);
        *reinterpret_cast<uint4 *>(re + o) = tre[i][run];
        *reinterpret_cast<uint4 *>(im + o) = tim[i][run];
    }
}

// complex128 table rows [r_off, r_off + rows) ([rows][n]) -> columns of the transposed BF16 planes
// ldn x ldr (row-major or 16-row panels); columns from r_off + rows up to r_end are written as
// zeros (padding)
__global__ void k_c128_to_planes_t(int rows, int n, const double2 *__restrict__ src, int64_t ldr, int64_t ldn,
                                   uint16_t *__restrict__ re, uint16_t *__restrict__ im, int r_off, int64_t r_end,
                                   int panel) {
    __shared__ double2 tile[32][33];
    const int r0 = r_off + blockIdx.y * 32, g0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 32 x 8
    for (int y = ty; y < 32; y += 8) {
        const int r = r0 + y - r_off, g = g0 + tx;
        tile[y][tx] = (r < rows && g < n) ? src[(int64_t)r * n + g] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int g = g0 + y, r = r0 + tx;
        if (g < ldn && r < r_end) {
            const double2 v = tile[tx][y];
            const int64_t o = panel ? bf16_panel_index(g, r, ldr) : (int64_t)g * ldr + r;
            re[o] = f2bf((float)v.x);
            im[o] = f2bf((float)v.y);
        }
    }
}

void beta_to_bf16_t(int nproj, int npw, const void *beta64, void *tr, void *ti, hipStream_t st, bool panel) {
    beta_to_bf16_t_rows(nproj, 0, nproj, npw, beta64, tr, ti, st, panel);
}

// rows [p0, p0 + rows) of an nproj-row table (beta64 holds just those rows); the
// chunk that ends the table also writes the zero columns up to the padded width
void beta_to_bf16_t_rows(int nproj, int p0, int rows, int npw, const void *beta64, void *tr, void *ti,
                         hipStream_t st, bool panel) {
    const int64_t ldr = bf16_ld(nproj), ldn = bf16_ld(npw);
    PW_CHECK(p0 % 32 == 0 && p0 + rows <= nproj, PW_EINVAL, "table chunk must start on a 32-row boundary");
    const int64_t r_end = p0 + rows == nproj ? ldr : p0 + rows;
    dim3 grid((unsigned)((ldn + 31) / 32), (unsigned)((r_end - p0 + 31) / 32));
    hipLaunchKernelGGL(k_c128_to_planes_t, grid, dim3(256), 0, st, rows, npw, (const double2 *)beta64, ldr, ldn,
                       (uint16_t *)tr, (uint16_t *)ti, p0, r_end, panel ? 1 : 0);
    PW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// projection partials: partial[s][b][p] = sum over G chunk s of conj(beta) psi.
// Workgroup: NW*16 projectors (16 per wave) x NBLK*16 bands; grid (M tiles,
// splits).  The next stage's projector fragments and band pieces are loaded into
// registers while the current stage is multiplied.
// ---------------------------------------------------------------------------
template <int NBLK, int NW>
__global__ __launch_bounds__(NW * 64) void proj16_partial(int M, int N, const uint16_t *__restrict__ Br,
                                                          const uint16_t *__restrict__ Bi, int64_t ldg,
                                                          const uint16_t *__restrict__ Pr,
                                                          const uint16_t *__restrict__ Pi, int kchunk,
                                                          float2 *__restrict__ partial) {
    constexpr int NB = NBLK * 16, NT = NW * 64;
    constexpr int PPT = (NB * (KS / 8) + NT - 1) / NT;   // 16-byte band pieces per thread and plane
    __shared__ __attribute__((aligned(16))) uint16_t sPr[NB][LPAD], sPi[NB][LPAD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * (NW * 16) + wave * 16;
    const int s = blockIdx.y;
    const int kbeg = s * kchunk;
    const int kend = (int)min((int64_t)kbeg + kchunk, ldg);
    v4f ar_[NBLK], ai_[NBLK];
#pragma unroll
    for (int j = 0; j < NBLK; ++j) { ar_[j] = v4f{0, 0, 0, 0}; ai_[j] = v4f{0, 0, 0, 0}; }
    const int64_t rowA = m0 + (lane & 15);
    const bool okA = rowA < M;
    bf16x8 fa_r[2], fa_i[2];
    uint4 pr_n[PPT], pi_n[PPT];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int64_t off = rowA * ldg + k0 + ks * 32 + 8 * (lane >> 4);
            fa_r[ks] = okA ? load8(Br + off) : zero8();
            fa_i[ks] = okA ? load8(Bi + off) : zero8();
        }
#pragma unroll
        for (int t = 0; t < PPT; ++t) {
            const int e = tid + t * NT, r = e >> 3, c8 = (e & 7) * 8;
            pr_n[t] = make_uint4(0, 0, 0, 0);
            pi_n[t] = make_uint4(0, 0, 0, 0);
            if (e < NB * (KS / 8) && r < N) {
                pr_n[t] = *reinterpret_cast<const uint4 *>(Pr + (int64_t)r * ldg + k0 + c8);
                pi_n[t] = *reinterpret_cast<const uint4 *>(Pi + (int64_t)r * ldg + k0 + c8);
            }
        }
    };
    if (kbeg < kend) fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += KS) {
#pragma unroll
        for (int t = 0; t < PPT; ++t) {
            const int e = tid + t * NT, r = e >> 3, c8 = (e & 7) * 8;
            if (e < NB * (KS / 8)) {
                *reinterpret_cast<uint4 *>(&sPr[r][c8]) = pr_n[t];
                *reinterpret_cast<uint4 *>(&sPi[r][c8]) = pi_n[t];
            }
        }
        const bf16x8 ca_r[2] = {fa_r[0], fa_r[1]}, ca_i[2] = {fa_i[0], fa_i[1]};
        __syncthreads();
        if (k0 + KS < kend) fetch(k0 + KS);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int kk = ks * 32 + 8 * (lane >> 4);
            const bf16x8 nai = neg8(ca_i[ks]);
#pragma unroll
            for (int j = 0; j < NBLK; ++j) {
                const int row = j * 16 + (lane & 15);
                const bf16x8 br = load8(&sPr[row][kk]), bi = load8(&sPi[row][kk]);
                // conj(beta) psi: re = br pr + bi pi, im = br pi - bi pr
                ar_[j] = mfma_bf16(ca_r[ks], br, ar_[j]);
                ar_[j] = mfma_bf16(ca_i[ks], bi, ar_[j]);
                ai_[j] = mfma_bf16(ca_r[ks], bi, ai_[j]);
                ai_[j] = mfma_bf16(nai, br, ai_[j]);
            }
        }
        __syncthreads();
    }
    float2 *P = partial + (int64_t)s * M * N;
#pragma unroll
    for (int j = 0; j < NBLK; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = m0 + 4 * (lane >> 4) + v;
            const int col = j * 16 + (lane & 15);
            if (row < M && col < N) P[(int64_t)col * M + row] = make_float2(ar_[j][v], ai_[j][v]);
        }
}

// W planes N x ldp (row-major or 16-row panels) = bf16(d[p] * sum_s partial[s][b][p]),
// zero for p >= M
__global__ void proj16_reduce(int M, int N, int nsplit, const float2 *__restrict__ partial,
                              const float *__restrict__ d, int64_t ldp, uint16_t *__restrict__ Wr,
                              uint16_t *__restrict__ Wi, int panel) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)N * ldp) return;
    const int n = (int)(idx / ldp), m = (int)(idx % ldp);
    float re = 0.f, im = 0.f;
    if (m < M) {
        double sr = 0, si = 0;
        for (int s = 0; s < nsplit; ++s) {
            const float2 v = partial[(int64_t)s * M * N + (int64_t)n * M + m];
            sr += v.x;
            si += v.y;
        }
        const double sc = d ? d[m] : 1.0;
        re = (float)(sr * sc);
        im = (float)(si * sc);
    }
    const int64_t o = panel ? bf16_panel_index(n, m, ldp) : idx;
    Wr[o] = f2bf(re);
    Wi[o] = f2bf(im);
}

// ---------------------------------------------------------------------------
// back-projection: out[b][G] += sum_p W[b][p] beta_p(G), W from the BF16 planes.
// Workgroup: NBLK*16 bands x NW*16 plane waves (16 per wave); grid: G tiles.  The
// next stage's table fragments and W pieces are loaded into registers while the
// current stage is multiplied.
// ---------------------------------------------------------------------------
template <int NBLK, int NW>
__global__ __launch_bounds__(NW * 64) void backproj16(int N, int J, int64_t ldp, const uint16_t *__restrict__ Wr,
                                                      const uint16_t *__restrict__ Wi,
                                                      const uint16_t *__restrict__ Tr,
                                                      const uint16_t *__restrict__ Ti, float2 *__restrict__ out,
                                                      int64_t ldo) {
    constexpr int NB = NBLK * 16, NT = NW * 64;
    constexpr int WPT = (NB * (KS / 8) + NT - 1) / NT;   // 16-byte W pieces per thread and plane
    __shared__ __attribute__((aligned(16))) uint16_t sWr[NB][LPAD], sWi[NB][LPAD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t gcol = (int64_t)blockIdx.x * (NW * 16) + wave * 16 + (lane & 15);
    const bool okB = gcol < J;
    v4f ar_[NBLK], ai_[NBLK];
#pragma unroll
    for (int i = 0; i < NBLK; ++i) { ar_[i] = v4f{0, 0, 0, 0}; ai_[i] = v4f{0, 0, 0, 0}; }
    bf16x8 fb_r[2], fb_i[2];
    uint4 wr_n[WPT], wi_n[WPT];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int64_t off = gcol * ldp + k0 + ks * 32 + 8 * (lane >> 4);
            fb_r[ks] = okB ? load8(Tr + off) : zero8();
            fb_i[ks] = okB ? load8(Ti + off) : zero8();
        }
#pragma unroll
        for (int t = 0; t < WPT; ++t) {
            const int e = tid + t * NT, r = e >> 3, c8 = (e & 7) * 8;
            wr_n[t] = make_uint4(0, 0, 0, 0);
            wi_n[t] = make_uint4(0, 0, 0, 0);
            if (e < NB * (KS / 8) && r < N) {
                wr_n[t] = *reinterpret_cast<const uint4 *>(Wr + (int64_t)r * ldp + k0 + c8);
                wi_n[t] = *reinterpret_cast<const uint4 *>(Wi + (int64_t)r * ldp + k0 + c8);
            }
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < ldp; k0 += KS) {
#pragma unroll
        for (int t = 0; t < WPT; ++t) {
            const int e = tid + t * NT, r = e >> 3, c8 = (e & 7) * 8;
            if (e < NB * (KS / 8)) {
                *reinterpret_cast<uint4 *>(&sWr[r][c8]) = wr_n[t];
                *reinterpret_cast<uint4 *>(&sWi[r][c8]) = wi_n[t];
            }
        }
        const bf16x8 cb_r[2] = {fb_r[0], fb_r[1]}, cb_i[2] = {fb_i[0], fb_i[1]};
        __syncthreads();
        if (k0 + KS < ldp) fetch(k0 + KS);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int kk = ks * 32 + 8 * (lane >> 4);
#pragma unroll
            for (int i = 0; i < NBLK; ++i) {
                const int row = i * 16 + (lane & 15);
                const bf16x8 wr = load8(&sWr[row][kk]), wi = load8(&sWi[row][kk]);
                // W beta: re = wr br - wi bi, im = wr bi + wi br
                ar_[i] = mfma_bf16(wr, cb_r[ks], ar_[i]);
                ar_[i] = mfma_bf16(neg8(wi), cb_i[ks], ar_[i]);
                ai_[i] = mfma_bf16(wr, cb_i[ks], ai_[i]);
                ai_[i] = mfma_bf16(wi, cb_r[ks], ai_[i]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < NBLK; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int b = i * 16 + 4 * (lane >> 4) + v;
            if (b < N && okB) {
                float2 *o = out + (int64_t)b * ldo + gcol;
                const float2 old = *o;
                *o = make_float2(old.x + ar_[i][v], old.y + ai_[i][v]);
            }
        }
}

// Workgroups go to the eight XCDs (each with its own L2) round robin in dispatch
// order.  wide_tile renumbers them so that each XCD takes one contiguous run of
// tile indices, band tile fastest: the workgroups running together on an XCD are
// then a few row tiles by every band tile of one split and share their table rows
// and band planes in that XCD's L2 (the table is read from memory about once per
// call instead of once per band tile).  A bijection of the grid, so every tile is
// computed exactly as before.
struct WideTile {
    int x, y, z;
};
__device__ inline WideTile wide_tile() {
    const int X = gridDim.x, Y = gridDim.y;
    const int T = X * Y * gridDim.z;
    const int id = blockIdx.x + X * (blockIdx.y + Y * blockIdx.z);
    const int xcd = id % 8, q = T / 8, r = T % 8;
    const int L = xcd * q + min(xcd, r) + id / 8;
    return WideTile{(L / Y) % X, L % Y, L / (X * Y)};
}

// ---------------------------------------------------------------------------
// Wide band blocks (contexts of more than MAXNB bands, operands in 16-row
// panels).  A workgroup of WM x WN waves covers WM*RB*16 table rows (projection)
// or plane waves (back-projection) by WN*NBLK*16 = 256 bands; each wave takes RB
// row blocks by NBLK band blocks, so a band fragment read from LDS feeds RB
// complex products and a table fragment NBLK of them.  Both operands of a
// 32-deep stage go from memory straight into LDS through
// global_load_lds_dwordx4 (no registers on the way), kRingStages stages deep: a
// workgroup keeps two stages (96 KB) of loads in flight while it multiplies a
// third.  Each copy moves one whole 1 KB fragment of a panel, contiguous in
// memory and already in the MFMA's lane order (lane l: row l % 16, k 8 (l / 16)
// + 0..7), into one 1 KB block of LDS, so every fragment read is one linear
// ds_read_b128; a workgroup streams a few dozen panels, each sequentially along
// k.  (Row-major planes, where each copy gathers 64 bytes from each of 16 rows
// 1.5 MB apart, ran the same copies at less than half the rate: every row is
// its own stream and page.)  Row blocks beyond an operand are read as its last
// block: their products only reach outputs that are not stored.  The copies
// are issued in inline assembly because the compiler, not knowing which stage a
// DMA fills, would wait for all of them before any LDS read; here each wave
// waits for its own copies of the stage it is about to use (s_waitcnt vmcnt
// counts them in issue order) and the barrier then publishes every wave's part.
// ---------------------------------------------------------------------------
constexpr int kRingStages = 3;

// 16 bytes per lane from g (per lane) into LDS at lds + 16 lane (lds wave-uniform);
// m0 carries the LDS address and is restored afterwards
__device__ inline void lds_dma16(const void *g, uint32_t lds) {
    uint32_t keep;
    asm volatile(
        "s_mov_b32 %0, m0\n\t"
        "s_mov_b32 m0, %1\n\t"
        "global_load_lds_dwordx4 %2, off\n\t"
        "s_mov_b32 m0, %0"
        : "=&s"(keep)
        : "s"(lds), "v"(g)
        : "memory");
}

// at most N of this wave's copies still in flight, its LDS reads done, then the barrier
template <int N>
__device__ inline void ring_barrier() {
    asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}

__device__ inline uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}

// projection: partial[s][b][m] = sum over split s of conj(beta_m) psi_b; tiles of
// WM RB 16 table rows by WN NBLK 16 bands, each wave RB x NBLK fragments
template <int RB, int NBLK, int WM, int WN>
__global__ __launch_bounds__(WM * WN * 64) void proj_ring(int M, int N, const uint16_t *__restrict__ Br,
                                                          const uint16_t *__restrict__ Bi, int64_t ldg,
                                                          const uint16_t *__restrict__ Pr,
                                                          const uint16_t *__restrict__ Pi, int kchunk,
                                                          float2 *__restrict__ partial) {
    constexpr int NW = WM * WN, TB = WM * RB, BB = WN * NBLK;
    constexpr int BLK = 2 * (TB + BB), PW = BLK / NW, STAGE = BLK * 1024;
    static_assert(BLK % NW == 0, "DMA blocks must divide evenly over the waves");
    __shared__ __attribute__((aligned(1024))) uint8_t ring[kRingStages][STAGE];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave % WM, wn = wave / WM;
    const WideTile tile = wide_tile();
    const int m0 = tile.x * (TB * 16), n0 = tile.y * (BB * 16);
    const int kbeg = tile.z * kchunk;
    const int nst = (int)((std::min((int64_t)kbeg + kchunk, ldg) - kbeg) / 32);
    const uint16_t *src[PW];
    const int64_t kb0 = ((int64_t)(ldg >> 5) << 9), kfirst = (int64_t)(kbeg >> 5) << 9;
#pragma unroll
    for (int i = 0; i < PW; ++i) {
        const int b = wave * PW + i;
        if (b < 2 * TB) {
            const int rb = std::min(m0 / 16 + b % TB, (M - 1) >> 4);
            src[i] = (b < TB ? Br : Bi) + rb * kb0 + kfirst + lane * 8;
        } else {
            const int c = b - 2 * TB;
            const int nb = std::min(n0 / 16 + c % BB, (N - 1) >> 4);
            src[i] = (c < BB ? Pr : Pi) + nb * kb0 + kfirst + lane * 8;
        }
    }
    const uint32_t base = __builtin_amdgcn_readfirstlane(lds_addr(&ring[0][0]));
    auto issue = [&](int s) {
        const uint32_t slot = base + (uint32_t)((s % kRingStages) * STAGE + wave * PW * 1024);
#pragma unroll
        for (int i = 0; i < PW; ++i) lds_dma16(src[i] + 512 * s, slot + (uint32_t)(i * 1024));
    };
    v4f ar_[RB][NBLK], ai_[RB][NBLK];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int j = 0; j < NBLK; ++j) { ar_[r][j] = v4f{0, 0, 0, 0}; ai_[r][j] = v4f{0, 0, 0, 0}; }
#pragma unroll
    for (int s = 0; s < kRingStages - 1; ++s)
        if (s < nst) issue(s);
    for (int t = 0; t < nst; ++t) {
        // stage t landed (stage t + 1 may still be in flight)
        if (t + 1 < nst) ring_barrier<PW>();
        else ring_barrier<0>();
        if (t + kRingStages - 1 < nst) issue(t + kRingStages - 1);    // into the slot stage t - 1 left
        const uint8_t *S = &ring[t % kRingStages][0] + lane * 16;
        bf16x8 tr[RB], ti[RB], tn[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            tr[r] = *reinterpret_cast<const bf16x8 *>(S + (wm * RB + r) * 1024);
            ti[r] = *reinterpret_cast<const bf16x8 *>(S + (TB + wm * RB + r) * 1024);
            tn[r] = neg8(ti[r]);
        }
#pragma unroll
        for (int j = 0; j < NBLK; ++j) {
            const bf16x8 pr = *reinterpret_cast<const bf16x8 *>(S + (2 * TB + wn * NBLK + j) * 1024);
            const bf16x8 pi = *reinterpret_cast<const bf16x8 *>(S + (2 * TB + BB + wn * NBLK + j) * 1024);
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                // conj(beta) psi: re = br pr + bi pi, im = br pi - bi pr
                ar_[r][j] = mfma_bf16(tr[r], pr, ar_[r][j]);
                ar_[r][j] = mfma_bf16(ti[r], pi, ar_[r][j]);
                ai_[r][j] = mfma_bf16(tr[r], pi, ai_[r][j]);
                ai_[r][j] = mfma_bf16(tn[r], pr, ai_[r][j]);
            }
        }
    }
    float2 *P = partial + (int64_t)tile.z * M * N;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int j = 0; j < NBLK; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + (wm * RB + r) * 16 + 4 * (lane >> 4) + v;
                const int col = n0 + (wn * NBLK + j) * 16 + (lane & 15);
                if (row < M && col < N) P[(int64_t)col * M + row] = make_float2(ar_[r][j][v], ai_[r][j][v]);
            }
}

// back-projection: out[b][g] += sum_p W[b][p] beta_p(g); tiles of WM GB 16 plane
// waves by WN NBLK 16 bands, each wave NBLK x GB fragments, all ldp projectors
template <int GB, int NBLK, int WM, int WN>
__global__ __launch_bounds__(WM * WN * 64) void backproj_ring(int N, int J, int64_t ldp,
                                                              const uint16_t *__restrict__ Wr,
                                                              const uint16_t *__restrict__ Wi,
                                                              const uint16_t *__restrict__ Tr,
                                                              const uint16_t *__restrict__ Ti,
                                                              float2 *__restrict__ out, int64_t ldo) {
    constexpr int NW = WM * WN, TB = WM * GB, BB = WN * NBLK;
    constexpr int BLK = 2 * (TB + BB), PW = BLK / NW, STAGE = BLK * 1024;
    static_assert(BLK % NW == 0, "DMA blocks must divide evenly over the waves");
    __shared__ __attribute__((aligned(1024))) uint8_t ring[kRingStages][STAGE];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave % WM, wn = wave / WM;
    const WideTile tile = wide_tile();
    const int g0 = tile.x * (TB * 16), b0 = tile.y * (BB * 16);
    const int nst = (int)(ldp / 32);
    const uint16_t *src[PW];
    const int64_t kb0 = (int64_t)(ldp >> 5) << 9;
#pragma unroll
    for (int i = 0; i < PW; ++i) {
        const int b = wave * PW + i;
        if (b < 2 * TB) {
            const int gb = std::min(g0 / 16 + b % TB, (J - 1) >> 4);
            src[i] = (b < TB ? Tr : Ti) + gb * kb0 + lane * 8;
        } else {
            const int c = b - 2 * TB;
            const int nb = std::min(b0 / 16 + c % BB, (N - 1) >> 4);
            src[i] = (c < BB ? Wr : Wi) + nb * kb0 + lane * 8;
        }
    }
    const uint32_t base = __builtin_amdgcn_readfirstlane(lds_addr(&ring[0][0]));
    auto issue = [&](int s) {
        const uint32_t slot = base + (uint32_t)((s % kRingStages) * STAGE + wave * PW * 1024);
#pragma unroll
        for (int i = 0; i < PW; ++i) lds_dma16(src[i] + 512 * s, slot + (uint32_t)(i * 1024));
    };
    v4f ar_[NBLK][GB], ai_[NBLK][GB];
#pragma unroll
    for (int i = 0; i < NBLK; ++i)
#pragma unroll
        for (int g = 0; g < GB; ++g) { ar_[i][g] = v4f{0, 0, 0, 0}; ai_[i][g] = v4f{0, 0, 0, 0}; }
#pragma unroll
    for (int s = 0; s < kRingStages - 1; ++s)
        if (s < nst) issue(s);
    for (int t = 0; t < nst; ++t) {
        if (t + 1 < nst) ring_barrier<PW>();
        else ring_barrier<0>();
        if (t + kRingStages - 1 < nst) issue(t + kRingStages - 1);
        const uint8_t *S = &ring[t % kRingStages][0] + lane * 16;
        bf16x8 tr[GB], ti[GB];
#pragma unroll
        for (int g = 0; g < GB; ++g) {
            tr[g] = *reinterpret_cast<const bf16x8 *>(S + (wm * GB + g) * 1024);
            ti[g] = *reinterpret_cast<const bf16x8 *>(S + (TB + wm * GB + g) * 1024);
        }
#pragma unroll
        for (int i = 0; i < NBLK; ++i) {
            const bf16x8 wr = *reinterpret_cast<const bf16x8 *>(S + (2 * TB + wn * NBLK + i) * 1024);
            const bf16x8 wi = *reinterpret_cast<const bf16x8 *>(S + (2 * TB + BB + wn * NBLK + i) * 1024);
            const bf16x8 nwi = neg8(wi);
#pragma unroll
            for (int g = 0; g < GB; ++g) {
                // W beta: re = wr br - wi bi, im = wr bi + wi br
                ar_[i][g] = mfma_bf16(wr, tr[g], ar_[i][g]);
                ar_[i][g] = mfma_bf16(nwi, ti[g], ar_[i][g]);
                ai_[i][g] = mfma_bf16(wr, ti[g], ai_[i][g]);
                ai_[i][g] = mfma_bf16(wi, tr[g], ai_[i][g]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NBLK; ++i)
#pragma unroll
        for (int g = 0; g < GB; ++g)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int b = b0 + (wn * NBLK + i) * 16 + 4 * (lane >> 4) + v;
                const int gc = g0 + (wm * GB + g) * 16 + (lane & 15);
                if (b < N && gc < J) {
                    float2 *o = out + (int64_t)b * ldo + gc;
                    const float2 old = *o;
                    *o = make_float2(old.x + ar_[i][g][v], old.y + ai_[i][g][v]);
                }
            }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int band_blocks(int nb) { return nb <= 64 ? 4 : nb <= 128 ? 8 : 9; }
static int band_chunk(int nb) { return nb <= MAXNB ? nb : 128; }

bool bf16_panels(int max_bands) { return max_bands > MAXNB; }
int64_t bf16_rows(int rows, int max_bands) { return bf16_panels(max_bands) ? ((int64_t)rows + 15) / 16 * 16 : rows; }

constexpr int kB16ProjNW = 4;   // waves (16 projectors each) per projection workgroup

static int proj_splits(int M, int64_t ldg) {
    const int mt = (M + 16 * kB16ProjNW - 1) / (16 * kB16ProjNW);
    int s = (512 + mt - 1) / mt;
    const int maxs = (int)((ldg + 2 * KS - 1) / (2 * KS));      // at least two stages per split
    return std::max(1, std::min(s, maxs));
}

// wide kernels: launch variants {RB (row blocks per wave), NBLK (band blocks per
// wave), WM x WN waves}; every variant spans 256 bands.  1 and 2 give each of
// four waves 64 x 128 or 32 x 256 outputs, so every LDS fragment feeds more
// products; 3 reads the fewest fragments per wave of the eight-wave tiles.
static const int kWide[kBf16WideVariants][4] = {{2, 8, 4, 2}, {4, 8, 2, 2}, {2, 16, 4, 1}, {4, 4, 2, 4}};
constexpr int kWideBands = 256;
static int wide_rows(int v) { return kWide[v][2] * kWide[v][0] * 16; }

// split-K of the wide projection: about 512 workgroups, at least four 32-deep stages per split
static int wide_splits(int v, int M, int N, int64_t ldg) {
    const int tiles = ((M + wide_rows(v) - 1) / wide_rows(v)) * ((N + kWideBands - 1) / kWideBands);
    const int s = (512 + tiles - 1) / tiles;
    const int maxs = (int)std::max<int64_t>(1, ldg / (4 * 32));
    return std::max(1, std::min(s, maxs));
}

size_t cnt_partial_bytes(int M, int N, int K, int max_bands) {
    if (bf16_panels(max_bands)) {
        int s = 1;
        for (int v = 0; v < kBf16WideVariants; ++v) s = std::max(s, wide_splits(v, M, N, bf16_ld(K)));
        return (size_t)s * M * N * sizeof(float2);
    }
    return (size_t)proj_splits(M, bf16_ld(K)) * M * band_chunk(N) * sizeof(float2);
}

template <int RB, int NBLK, int WM, int WN>
static void proj_ring_go(int v, int M, int N, const uint16_t *Br, const uint16_t *Bi, int64_t ldg,
                         const uint16_t *Pr, const uint16_t *Pi, float2 *partial, int &nsplit, hipStream_t st) {
    const int ns = wide_splits(v, M, N, ldg);
    int kchunk = (int)((ldg + ns - 1) / ns);
    kchunk = (kchunk + 31) / 32 * 32;
    nsplit = (int)((ldg + kchunk - 1) / kchunk);
    constexpr int rows = WM * RB * 16;
    dim3 grid((M + rows - 1) / rows, (N + kWideBands - 1) / kWideBands, nsplit);
    hipLaunchKernelGGL((proj_ring<RB, NBLK, WM, WN>), grid, dim3(64 * WM * WN), 0, st, M, N, Br, Bi, ldg, Pr, Pi,
                       kchunk, partial);
    PW_LAUNCH_CHECK();
}

template <int GB, int NBLK, int WM, int WN>
static void back_ring_go(int N, int J, int64_t ldp, const uint16_t *Wr, const uint16_t *Wi, const uint16_t *Tr,
                         const uint16_t *Ti, float2 *out, int64_t ldo, hipStream_t st) {
    constexpr int cols = WM * GB * 16;
    dim3 grid((unsigned)((J + cols - 1) / cols), (N + kWideBands - 1) / kWideBands);
    hipLaunchKernelGGL((backproj_ring<GB, NBLK, WM, WN>), grid, dim3(64 * WM * WN), 0, st, N, J, ldp, Wr, Wi, Tr,
                       Ti, out, ldo);
    PW_LAUNCH_CHECK();
}

size_t bf16_scratch_bytes(int nproj, int npw, int max_bands) {
    return (size_t)2 * bf16_rows(max_bands, max_bands) * (bf16_ld(npw) + bf16_ld(nproj)) * sizeof(uint16_t);
}

template <int NBLK>
static void proj_go(int M, int N, const uint16_t *Br, const uint16_t *Bi, int64_t ldg, const uint16_t *Pr,
                    const uint16_t *Pi, float2 *partial, int &nsplit, hipStream_t st) {
    const int ns = proj_splits(M, ldg);
    int kchunk = (int)((ldg + ns - 1) / ns);
    kchunk = (kchunk + KS - 1) / KS * KS;
    nsplit = (int)((ldg + kchunk - 1) / kchunk);
    dim3 grid((M + 16 * kB16ProjNW - 1) / (16 * kB16ProjNW), nsplit);
    hipLaunchKernelGGL((proj16_partial<NBLK, kB16ProjNW>), grid, dim3(64 * kB16ProjNW), 0, st, M, N, Br, Bi, ldg, Pr, Pi,
                       kchunk, partial);
    PW_LAUNCH_CHECK();
}

constexpr int kB16BackNW = 4;   // waves (16 plane waves each) per back-projection workgroup

template <int NBLK>
static void back_go(int N, int J, int64_t ldp, const uint16_t *Wr, const uint16_t *Wi, const uint16_t *Tr,
                    const uint16_t *Ti, float2 *out, int64_t ldo, hipStream_t st) {
    hipLaunchKernelGGL((backproj16<NBLK, kB16BackNW>), dim3((J + 16 * kB16BackNW - 1) / (16 * kB16BackNW)),
                       dim3(64 * kB16BackNW), 0, st, N, J, ldp, Wr, Wi, Tr, Ti, out, ldo);
    PW_LAUNCH_CHECK();
}

// Scratch (bf16_scratch_bytes): Pr, Pi (rows x ldg) then Wr, Wi (rows x ldp), rows =
// bf16_rows(max_bands), each plane row-major or in 16-row panels as the tables.
struct Bf16Scratch {
    uint16_t *Pr, *Pi, *Wr, *Wi;
    Bf16Scratch(void *p, int max_bands, int64_t ldg, int64_t ldp) {
        const int64_t rows = bf16_rows(max_bands, max_bands);
        Pr = (uint16_t *)p;
        Pi = Pr + rows * ldg;
        Wr = Pi + rows * ldg;
        Wi = Wr + rows * ldp;
    }
};

// W = bf16(D o (B^H psi)) for the bands of a complex64 block (into the scratch)
void proj_bf16(int nproj, int nb, int npw, int max_bands, const void *beta16, const float *d, const void *psi,
               int64_t ld, void *scratch, void *partial, hipStream_t st, int variant) {
    const int64_t ldg = bf16_ld(npw), ldp = bf16_ld(nproj);
    const bool panel = bf16_panels(max_bands);
    const uint16_t *Br = (const uint16_t *)beta16, *Bi = Br + bf16_rows(nproj, max_bands) * ldg;
    Bf16Scratch S(scratch, max_bands, ldg, ldp);
    if (panel)
        hipLaunchKernelGGL(k_c64_to_panels, dim3((unsigned)((ldg + 255) / 256), (nb + 15) / 16), dim3(256), 0, st, nb,
                           npw, (const float2 *)psi, ld, ldg, S.Pr, S.Pi);
    else
        hipLaunchKernelGGL(k_c64_to_planes, dim3((unsigned)((ldg + 255) / 256), nb), dim3(256), 0, st, nb, npw,
                           (const float2 *)psi, ld, ldg, S.Pr, S.Pi);
    PW_LAUNCH_CHECK();
    if (panel) {
        // every band in one launch of 256-band tiles, split over the plane waves
        PW_CHECK(variant >= 0 && variant < kBf16WideVariants, PW_EINVAL, "BF16 tile variant %d unknown", variant);
        int nsplit = 1;
        float2 *part = (float2 *)partial;
        switch (variant) {
            case 0: proj_ring_go<2, 8, 4, 2>(0, nproj, nb, Br, Bi, ldg, S.Pr, S.Pi, part, nsplit, st); break;
            case 1: proj_ring_go<4, 8, 2, 2>(1, nproj, nb, Br, Bi, ldg, S.Pr, S.Pi, part, nsplit, st); break;
            case 2: proj_ring_go<2, 16, 4, 1>(2, nproj, nb, Br, Bi, ldg, S.Pr, S.Pi, part, nsplit, st); break;
            default: proj_ring_go<4, 4, 2, 4>(3, nproj, nb, Br, Bi, ldg, S.Pr, S.Pi, part, nsplit, st); break;
        }
        const int64_t tot = (int64_t)nb * ldp;
        hipLaunchKernelGGL(proj16_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, nproj, nb, nsplit,
                           (const float2 *)partial, d, ldp, S.Wr, S.Wi, 1);
        PW_LAUNCH_CHECK();
        return;
    }
    for (int b0 = 0; b0 < nb; b0 += band_chunk(nb)) {
        const int n = std::min(band_chunk(nb), nb - b0);
        const uint16_t *Pr = S.Pr + (int64_t)b0 * ldg, *Pi = S.Pi + (int64_t)b0 * ldg;
        int nsplit = 1;
        float2 *part = (float2 *)partial;
        switch (band_blocks(n)) {
            case 4: proj_go<4>(nproj, n, Br, Bi, ldg, Pr, Pi, part, nsplit, st); break;
            case 8: proj_go<8>(nproj, n, Br, Bi, ldg, Pr, Pi, part, nsplit, st); break;
            default: proj_go<9>(nproj, n, Br, Bi, ldg, Pr, Pi, part, nsplit, st); break;
        }
        const int64_t tot = (int64_t)n * ldp;
        hipLaunchKernelGGL(proj16_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, nproj, n, nsplit,
                           (const float2 *)part, d, ldp, S.Wr + (int64_t)b0 * ldp, S.Wi + (int64_t)b0 * ldp, 0);
        PW_LAUNCH_CHECK();
    }
}

// out[b] += B . W[b] with W from proj_bf16's scratch
void backproj_bf16(int nproj, int nb, int npw, int max_bands, const void *betaT16, const void *scratch, void *out,
                   int64_t ldo, hipStream_t st, int variant) {
    const int64_t ldg = bf16_ld(npw), ldp = bf16_ld(nproj);
    const uint16_t *Tr = (const uint16_t *)betaT16, *Ti = Tr + ldg * ldp;
    Bf16Scratch S(const_cast<void *>(scratch), max_bands, ldg, ldp);
    if (bf16_panels(max_bands)) {
        PW_CHECK(variant >= 0 && variant < kBf16WideVariants, PW_EINVAL, "BF16 tile variant %d unknown", variant);
        const uint16_t *Wr = S.Wr, *Wi = S.Wi;
        float2 *o = (float2 *)out;
        switch (variant) {
            case 0: back_ring_go<2, 8, 4, 2>(nb, npw, ldp, Wr, Wi, Tr, Ti, o, ldo, st); break;
            case 1: back_ring_go<4, 8, 2, 2>(nb, npw, ldp, Wr, Wi, Tr, Ti, o, ldo, st); break;
            case 2: back_ring_go<2, 16, 4, 1>(nb, npw, ldp, Wr, Wi, Tr, Ti, o, ldo, st); break;
            default: back_ring_go<4, 4, 2, 4>(nb, npw, ldp, Wr, Wi, Tr, Ti, o, ldo, st); break;
        }
        return;
    }
    for (int b0 = 0; b0 < nb; b0 += band_chunk(nb)) {
        const int n = std::min(band_chunk(nb), nb - b0);
        const uint16_t *Wr = S.Wr + (int64_t)b0 * ldp, *Wi = S.Wi + (int64_t)b0 * ldp;
        float2 *po = (float2 *)out + (int64_t)b0 * ldo;
        switch (band_blocks(n)) {
            case 4: back_go<4>(n, npw, ldp, Wr, Wi, Tr, Ti, po, ldo, st); break;
            case 8: back_go<8>(n, npw, ldp, Wr, Wi, Tr, Ti, po, ldo, st); break;
            default: back_go<9>(n, npw, ldp, Wr, Wi, Tr, Ti, po, ldo, st); break;
        }
    }
}

}  // namespace pw
