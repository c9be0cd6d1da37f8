// Sphere <-> grid 3D FFT passes of the H psi path (gfx950).
//
//   z pass (inverse):  sphere coefficients of CB columns -> LDS -> length-N2 FFTs
//                      -> column grid cols[b][z][c]          (c over touched columns)
//   xy pass:           one (band, z) plane: scatter its columns into an N0 x N1 LDS
//                      plane, 2D inverse FFT (y only on the x rows the sphere
//                      touches), multiply by V(., ., z), 2D forward FFT, gather
//                      the columns back in place
//   z pass (forward):  column grid -> LDS -> FFTs -> (1/N) . gather onto the
//                      sphere, fused with the kinetic term (T_G - shift) c(G)
// Only the z-columns that touch the sphere travel through HBM.  Common grid
// lengths are compiled with their radices built in (CtLen); other lengths use the
// run-time plan (RtLen).  Planes of 16, 32, 48 or 64 points a side take the
// four-lane xy kernel (xy_quad) by default: each 1D transform lives in the
// registers of four lanes, exchanging through DPP quad permutes.  A context can carry per-pass launch choices (kernel
// kind, radix schedule, threads) picked by the autotuner at the end of this file.
#include "fft_core.h"
#include "kernels.h"
#include <vector>
#include <tuple>
#include <mutex>
#include <map>
#include <deque>
#include <memory>

namespace pw {

constexpr int kZpf = 4;    // sphere coefficients per thread loaded ahead in the inverse z pass
constexpr int kZcb = 16;   // columns per z-pass workgroup (pw_ctx::cb)

struct ZArgs {
    FftPlan plan;             // length N2
    int n2, ncols, cb, nb;
    const int32_t *colstart;  // [ncols + 1]
    const int32_t *zmap;      // [npw]: (c % cb) * (n2 + 1) + (n2_of_g mod n2)
    const void *tw;           // [n2] exp(-2 pi i t / n2)
};

struct XYArgs {
    FftPlan plan0, plan1;     // lengths N0 and N1
    int n0, n1, n2, ncols;
    int rowlo, nrows;         // x rows that hold columns: (rowlo + r) mod n0, r < nrows
    const int32_t *colpos;    // [ncols]: i0 * (n1 + 1) + i1 (padded plane index)
    const int32_t *colslot;   // [ncols]: place of (slot (i0 - rowlo) mod n0, column i1) in the
                              // four-lane kernel's plane of touched rows (quad_rs, quad_pad)
    const void *tw0, *tw1;
    const void *vz;           // [n2][n0][n1] potential, z-major (or null)
};

// one problem of a batched H psi (hpsi_batch below): its FFT arguments and blocks
struct FftJob {
    ZArgs z;
    XYArgs xy;
    int prob;                 // index into the problems' mask
    const void *in;           // sphere block (z inverse input, kinetic term of the z forward pass)
    int64_t ld;
    void *cols;               // the problem's column grid
    const double *kin;
    double shift, scale;
    void *out;
    int64_t ldo;
};

template <typename T> __device__ inline void load_tw(cplx<T> *dst, const cplx<T> *src, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// z pass, inverse: sphere -> column grid
// ---------------------------------------------------------------------------
template <typename T, int NTHR, typename LZ>
__device__ __forceinline__ void zinv_body(const ZArgs &a, const cplx<T> *__restrict__ psi, int64_t ld,
                                          cplx<T> *__restrict__ cols, int cb, int b) {
    extern __shared__ unsigned char smem_raw[];
    const int n2 = LZ::N > 0 ? LZ::N : a.n2;
    cplx<T> *tw = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *buf = tw + n2;
    const int c0 = cb * a.cb;
    const int c1 = min(c0 + a.cb, a.ncols);
    const int nc = c1 - c0;
    const int rs = n2 + 1;
    // the first kZpf coefficients per thread are loaded before the zero fill, so
    // that their latency overlaps it
    const int g0 = a.colstart[c0], g1 = a.colstart[c1];
    const cplx<T> *src = psi + (int64_t)b * ld;
    cplx<T> pv[kZpf];
    int pz[kZpf];
#pragma unroll
    for (int j = 0; j < kZpf; ++j) {
        const int g = g0 + threadIdx.x + j * NTHR;
        const bool in = g < g1;
        pv[j] = in ? src[g] : cmake<T>(0, 0);
        pz[j] = in ? a.zmap[g] : -1;
    }
    load_tw<T>(tw, reinterpret_cast<const cplx<T> *>(a.tw), n2);
    for (int i = threadIdx.x; i < nc * rs; i += NTHR) buf[i] = cmake<T>(0, 0);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kZpf; ++j)
        if (pz[j] >= 0) buf[pz[j]] = pv[j];
    for (int g = g0 + threadIdx.x + kZpf * NTHR; g < g1; g += NTHR) buf[a.zmap[g]] = src[g];
    __syncthreads();
    FftGeom geo{n2, nc, 1, rs, 0, nc};
    LZ::template fft<T, NTHR, 0>(buf, a.plan, geo, tw, +1);
    cplx<T> *dst = cols + (int64_t)b * n2 * a.ncols + c0;
    for (int e = threadIdx.x; e < nc * n2; e += NTHR) {
        const int z = e / nc, ci = e - z * nc;
        dst[(int64_t)z * a.ncols + ci] = buf[ci * rs + z];
    }
}

template <typename T, int NTHR, typename LZ>
__global__ __launch_bounds__(NTHR) void zpass_inv(ZArgs a, const cplx<T> *__restrict__ psi, int64_t ld,
                                                  cplx<T> *__restrict__ cols) {
    zinv_body<T, NTHR, LZ>(a, psi, ld, cols, blockIdx.x, blockIdx.y);
}

// Batched launches over independent problems (one FftJob each, blockIdx.y = job x
// nb + band; masked jobs and blocks beyond a job's extent return at once): the
// bodies of the single-problem kernels with each job's arguments.
template <typename T, int NTHR, typename LZ>
__global__ __launch_bounds__(NTHR) void zpass_inv_jobs(const FftJob *__restrict__ jobs, const int *__restrict__ mask,
                                                       int nb) {
    const FftJob &j = jobs[blockIdx.y / nb];
    if (!mask[j.prob] || (int)blockIdx.x * j.z.cb >= j.z.ncols) return;
    zinv_body<T, NTHR, LZ>(j.z, reinterpret_cast<const cplx<T> *>(j.in), j.ld, reinterpret_cast<cplx<T> *>(j.cols),
                           blockIdx.x, blockIdx.y % nb);
}

// ---------------------------------------------------------------------------
// z pass, forward: column grid -> sphere, with (1/N) and the kinetic epilogue
//   out[g] = scale * FFT(cols)[g] + (kin[g] - shift) * psi[g]   (kin may be null)
// ---------------------------------------------------------------------------
template <typename T, int NTHR, typename LZ>
__device__ __forceinline__ void zfwd_body(const ZArgs &a, const cplx<T> *__restrict__ cols,
                                          const cplx<T> *__restrict__ psi, int64_t ld,
                                          const double *__restrict__ kin, double shift, double scale,
                                          cplx<T> *__restrict__ out, int64_t ldo, int cb, int b) {
    extern __shared__ unsigned char smem_raw[];
    const int n2 = LZ::N > 0 ? LZ::N : a.n2;
    cplx<T> *tw = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *buf = tw + n2;
    const int c0 = cb * a.cb;
    const int c1 = min(c0 + a.cb, a.ncols);
    const int nc = c1 - c0;
    const int rs = n2 + 1;
    load_tw<T>(tw, reinterpret_cast<const cplx<T> *>(a.tw), n2);
    const cplx<T> *src = cols + (int64_t)b * n2 * a.ncols + c0;
    if constexpr (LZ::N > 0) {
        // compile-time length: every load of the block is issued before the first
        // LDS store (nc <= kZcb, checked on the host)
        constexpr int PER = (kZcb * LZ::N + NTHR - 1) / NTHR;
        cplx<T> v[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + q * NTHR;
            const int z = e / nc, ci = e - z * nc;
            v[q] = e < nc * n2 ? src[(int64_t)z * a.ncols + ci] : cmake<T>(0, 0);
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + q * NTHR;
            const int z = e / nc, ci = e - z * nc;
            if (e < nc * n2) buf[ci * rs + z] = v[q];
        }
    } else {
        for (int e = threadIdx.x; e < nc * n2; e += NTHR) {
            const int z = e / nc, ci = e - z * nc;
            buf[ci * rs + z] = src[(int64_t)z * a.ncols + ci];
        }
    }
    __syncthreads();
    FftGeom geo{n2, nc, 1, rs, 0, nc};
    LZ::template fft<T, NTHR, 0>(buf, a.plan, geo, tw, -1);
    const int g0 = a.colstart[c0], g1 = a.colstart[c1];
    cplx<T> *o = out + (int64_t)b * ldo;
    const T sc = (T)scale;
    if (kin) {
        const cplx<T> *p = psi + (int64_t)b * ld;
        for (int g = g0 + threadIdx.x; g < g1; g += NTHR) {
            const cplx<T> v = buf[a.zmap[g]];
            const cplx<T> c = p[g];
            const T t = (T)(kin[g] - shift);
            o[g] = cmake<T>(v.x * sc + t * c.x, v.y * sc + t * c.y);
        }
    } else {
        for (int g = g0 + threadIdx.x; g < g1; g += NTHR) o[g] = cscale<T>(buf[a.zmap[g]], sc);
    }
}

template <typename T, int NTHR, typename LZ>
__global__ __launch_bounds__(NTHR) void zpass_fwd(ZArgs a, const cplx<T> *__restrict__ cols,
                                                  const cplx<T> *__restrict__ psi, int64_t ld,
                                                  const double *__restrict__ kin, double shift, double scale,
                                                  cplx<T> *__restrict__ out, int64_t ldo) {
    zfwd_body<T, NTHR, LZ>(a, cols, psi, ld, kin, shift, scale, out, ldo, blockIdx.x, blockIdx.y);
}

template <typename T, int NTHR, typename LZ>
__global__ __launch_bounds__(NTHR) void zpass_fwd_jobs(const FftJob *__restrict__ jobs, const int *__restrict__ mask,
                                                       int nb) {
    const FftJob &j = jobs[blockIdx.y / nb];
    if (!mask[j.prob] || (int)blockIdx.x * j.z.cb >= j.z.ncols) return;
    zfwd_body<T, NTHR, LZ>(j.z, reinterpret_cast<const cplx<T> *>(j.cols), reinterpret_cast<const cplx<T> *>(j.in),
                           j.ld, j.kin, j.shift, j.scale, reinterpret_cast<cplx<T> *>(j.out), j.ldo, blockIdx.x,
                           blockIdx.y % nb);
}

// ---------------------------------------------------------------------------
// xy pass.  MODE 0: columns -> plane -> x V -> columns (in place)
//           MODE 1: columns -> plane -> grid out [b][x][y][z]
//           MODE 2: grid in [b][x][y][z] -> plane -> columns
// ---------------------------------------------------------------------------
template <typename T, int NTHR, int MODE, typename L0, typename L1>
__device__ __forceinline__ void xy_pass_body(const XYArgs &a, cplx<T> *__restrict__ cols, cplx<T> *__restrict__ grid,
                                             int z, int b) {
    extern __shared__ unsigned char smem_raw[];
    const int n0 = L0::N > 0 ? L0::N : a.n0;
    const int n1 = L1::N > 0 ? L1::N : a.n1;
    cplx<T> *tw0 = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *tw1 = tw0 + n0;
    cplx<T> *pl = tw1 + n1;
    const int rs = n1 + 1;
    const int npl = n0 * n1;
    load_tw<T>(tw0, reinterpret_cast<const cplx<T> *>(a.tw0), n0);
    load_tw<T>(tw1, reinterpret_cast<const cplx<T> *>(a.tw1), n1);
    cplx<T> *crow = cols + ((int64_t)b * a.n2 + z) * a.ncols;
    const FftGeom gy{n1, a.nrows, 1, rs, a.rowlo, n0};    // y transforms on the touched x rows
    const FftGeom gx{n0, n1, rs, 1, 0, n1};                // x transforms on every y
    if (MODE != 2) {
        for (int i = threadIdx.x; i < n0 * rs; i += NTHR) pl[i] = cmake<T>(0, 0);
        __syncthreads();
        for (int c = threadIdx.x; c < a.ncols; c += NTHR) pl[a.colpos[c]] = crow[c];
        __syncthreads();
        L1::template fft<T, NTHR, 0>(pl, a.plan1, gy, tw1, +1);
        L0::template fft<T, NTHR, L1::N>(pl, a.plan0, gx, tw0, +1);
    } else {
        const cplx<T> *gin = grid + (int64_t)b * npl * a.n2;
        for (int i = threadIdx.x; i < npl; i += NTHR) {
            const int x = i / n1, y = i - x * n1;
            pl[x * rs + y] = gin[(int64_t)i * a.n2 + z];
        }
        __syncthreads();
    }
    if (MODE == 1) {
        cplx<T> *gout = grid + (int64_t)b * npl * a.n2;
        for (int i = threadIdx.x; i < npl; i += NTHR) {
            const int x = i / n1, y = i - x * n1;
            gout[(int64_t)i * a.n2 + z] = pl[x * rs + y];
        }
        return;
    }
    if (MODE == 0) {
        const T *vzt = reinterpret_cast<const T *>(a.vz) + (int64_t)z * npl;
        for (int i = threadIdx.x; i < npl; i += NTHR) {
            const int x = i / n1, y = i - x * n1;
            pl[x * rs + y] = cscale<T>(pl[x * rs + y], vzt[i]);
        }
        __syncthreads();
    }
    L0::template fft<T, NTHR, L1::N>(pl, a.plan0, gx, tw0, -1);
    L1::template fft<T, NTHR, 0>(pl, a.plan1, gy, tw1, -1);
    for (int c = threadIdx.x; c < a.ncols; c += NTHR) crow[c] = pl[a.colpos[c]];
}

template <typename T, int NTHR, int MODE, typename L0, typename L1>
__global__ __launch_bounds__(NTHR) void xy_pass(XYArgs a, cplx<T> *__restrict__ cols, cplx<T> *__restrict__ grid) {
    xy_pass_body<T, NTHR, MODE, L0, L1>(a, cols, grid, blockIdx.x, blockIdx.y);
}

template <typename T, int NTHR, typename L0, typename L1>
__global__ __launch_bounds__(NTHR) void xy_pass_jobs(const FftJob *__restrict__ jobs, const int *__restrict__ mask,
                                                     int nb) {
    const FftJob &j = jobs[blockIdx.y / nb];
    if (!mask[j.prob]) return;
    xy_pass_body<T, NTHR, 0, L0, L1>(j.xy, reinterpret_cast<cplx<T> *>(j.cols), nullptr, blockIdx.x, blockIdx.y % nb);
}

// ---------------------------------------------------------------------------
// xy pass with four lanes per transform (MODE 0, n0 == n1 == L = 4 M, M in
// {4, 8, 12, 16, 24, 32}).  A length-L DFT splits as L = 4 x M:
//   quad_a: lane q holds x[q + 4 m] (m < M): M-point DFT over m in registers,
//           twiddle exp(s 2 pi i q k / L), 4-point DFT across the quad (DPP
//           exchanges, decimation in frequency); lane q then holds
//           X[k + M rho(q)], rho = the 2-bit reversal.
//   quad_b: lane q holds x[n + M rho(q)] (n < M): 4-point DFT across the quad
//           (decimation in time), twiddle exp(s 2 pi i n q / L), M-point DFT in
//           registers; lane q then holds X[q + 4 k].
// quad_a's output layout is quad_b's input layout, so the x transforms run
// inverse -> V(r) -> forward in registers.  Per plane: zero the touched rows,
// scatter the columns, y inverse on the touched rows, x inverse . V . x forward
// per y, y forward on the touched rows, gather: five barriers in all.  LDS holds
// only the nrows x rows the sphere touches (slot r is row rowlo + r mod L): the
// x transforms read the other rows as zeros and keep only the touched rows of
// their output, which is all the y forward transforms and the gather use.  So a
// 128-point complex128 plane of the 4000-atom wire (71 touched rows) fits LDS.
// ---------------------------------------------------------------------------
template <int N> struct CosTab;
template <> struct CosTab<12> {
    static constexpr double c[12] = {1.0, 0.86602540378443864676, 0.5, 0.0, -0.5, -0.86602540378443864676,
                                     -1.0, -0.86602540378443864676, -0.5, 0.0, 0.5, 0.86602540378443864676};
};
template <> struct CosTab<16> {
    static constexpr double c[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                                     0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                                     -1.0, -0.92387953251128675613, -0.70710678118654752440,
                                     -0.38268343236508977173, 0.0, 0.38268343236508977173, 0.70710678118654752440,
                                     0.92387953251128675613};
};

template <> struct CosTab<24> {
    static constexpr double c[24] = {
        1.0, 0.96592582628906828675, 0.86602540378443864676, 0.70710678118654752440, 0.5,
        0.25881904510252076235, 0.0, -0.25881904510252076235, -0.5, -0.70710678118654752440,
        -0.86602540378443864676, -0.96592582628906828675, -1.0, -0.96592582628906828675,
        -0.86602540378443864676, -0.70710678118654752440, -0.5, -0.25881904510252076235, 0.0,
        0.25881904510252076235, 0.5, 0.70710678118654752440, 0.86602540378443864676, 0.96592582628906828675};
};
template <> struct CosTab<32> {
    static constexpr double c[32] = {
        1.0, 0.98078528040323044913, 0.92387953251128675613, 0.83146961230254523708, 0.70710678118654752440,
        0.55557023301960222474, 0.38268343236508977173, 0.19509032201612826785, 0.0, -0.19509032201612826785,
        -0.38268343236508977173, -0.55557023301960222474, -0.70710678118654752440, -0.83146961230254523708,
        -0.92387953251128675613, -0.98078528040323044913, -1.0, -0.98078528040323044913, -0.92387953251128675613,
        -0.83146961230254523708, -0.70710678118654752440, -0.55557023301960222474, -0.38268343236508977173,
        -0.19509032201612826785, 0.0, 0.19509032201612826785, 0.38268343236508977173, 0.55557023301960222474,
        0.70710678118654752440, 0.83146961230254523708, 0.92387953251128675613, 0.98078528040323044913};
};

// exp(S 2 pi i t / N)
template <typename T, int N, int S> __device__ inline cplx<T> wconst(int t) {
    return cmake<T>((T)CosTab<N>::c[t % N], (T)(S * CosTab<N>::c[(t + 3 * N / 4) % N]));
}

// in-register DFT of length P Q: index b + P a in, c + Q d out
template <typename T, int P, int Q, int S> __device__ inline void dft_pq(cplx<T> *v) {
    constexpr int M = P * Q;
    cplx<T> t[P][Q];
#pragma unroll
    for (int b = 0; b < P; ++b) {
        cplx<T> u[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) u[a] = v[b + P * a];
        Dft<T, Q>::run(u, S);
#pragma unroll
        for (int c = 0; c < Q; ++c) t[b][c] = (b > 0 && c > 0) ? cmul<T>(u[c], wconst<T, M, S>(b * c)) : u[c];
    }
#pragma unroll
    for (int c = 0; c < Q; ++c) {
        cplx<T> u[P];
#pragma unroll
        for (int b = 0; b < P; ++b) u[b] = t[b][c];
        Dft<T, P>::run(u, S);
#pragma unroll
        for (int d = 0; d < P; ++d) v[c + Q * d] = u[d];
    }
}

template <typename T, int M, int S> __device__ inline void reg_dft(cplx<T> *v) {
    if constexpr (M == 4) Dft<T, 4>::run(v, S);
    else if constexpr (M == 8) Dft<T, 8>::run(v, S);
    else if constexpr (M == 12) dft_pq<T, 3, 4, S>(v);
    else if constexpr (M == 16) dft_pq<T, 4, 4, S>(v);
    else if constexpr (M == 24) dft_pq<T, 3, 8, S>(v);
    else {
        static_assert(M == 32, "register DFT length");
        dft_pq<T, 4, 8, S>(v);
    }
}

// value of lane (this lane's quad position permuted by quad_perm CTRL)
// (every lane of a quad is active wherever these run, so no lane reads an inactive one)
template <int CTRL> __device__ inline float quad_mov(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ inline double quad_mov(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kQuadXor1 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;   // quad_perm [2, 3, 0, 1]

// radix-2 step across lane pairs q, q ^ BIT: the lane with BIT clear keeps
// own + partner, the other partner - own
template <typename T, int M, int CTRL, int BIT> __device__ inline void quad_bfly(cplx<T> *v, int q) {
    const T sg = (q & BIT) ? (T)-1 : (T)1;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const T px = quad_mov<CTRL>(v[k].x), py = quad_mov<CTRL>(v[k].y);
        v[k] = cmake<T>(px + sg * v[k].x, py + sg * v[k].y);
    }
}

// lane 3 of the quad multiplies by exp(S 2 pi i / 4) = S i
template <typename T, int M, int S> __device__ inline void quad_w4(cplx<T> *v, int q) {
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = q == 3 ? mul_si<T>(v[k], S) : v[k];
}

// v[k] *= exp(S 2 pi i q k / L) from the table tw[t] = exp(-2 pi i t / L)
template <typename T, int M, int S> __device__ inline void quad_tw(cplx<T> *v, const cplx<T> *tw, int q) {
#pragma unroll
    for (int k = 1; k < M; ++k) {
        const cplx<T> w = tw[q * k];
        v[k] = S > 0 ? cmulc<T>(v[k], w) : cmul<T>(v[k], w);
    }
}

template <typename T, int M, int S> __device__ inline void quad_a(cplx<T> *v, const cplx<T> *tw, int q) {
    reg_dft<T, M, S>(v);
    quad_tw<T, M, S>(v, tw, q);
    quad_bfly<T, M, kQuadXor2, 2>(v, q);
    quad_w4<T, M, S>(v, q);
    quad_bfly<T, M, kQuadXor1, 1>(v, q);
}

template <typename T, int M, int S> __device__ inline void quad_b(cplx<T> *v, const cplx<T> *tw, int q) {
    quad_bfly<T, M, kQuadXor1, 1>(v, q);
    quad_w4<T, M, S>(v, q);
    quad_bfly<T, M, kQuadXor2, 2>(v, q);
    quad_tw<T, M, S>(v, tw, q);
    reg_dft<T, M, S>(v);
}

template <typename T, int M, int NTHR, bool VPF = sizeof(T) == 4>
__device__ __forceinline__ void xy_quad_body(const XYArgs &a, cplx<T> *__restrict__ cols, int z, int b) {
    constexpr int L = 4 * M, RS = quad_rs(M), PD = quad_pad(M), MB = M + PD, NQ = NTHR / 4;
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *tw = reinterpret_cast<cplx<T> *>(smem_raw);   // [L]
    cplx<T> *pl = tw + L;                                   // [nrows][RS], touched x rows only
    const int tid = threadIdx.x, q = tid & 3, quad = tid >> 2;
    const int rq = ((q & 1) << 1) | (q >> 1);
    const int nrows = a.nrows, rowlo = a.rowlo;
    cplx<T> *crow = cols + ((int64_t)b * a.n2 + z) * a.ncols;
    // the first CPF columns per thread are loaded before the zeroing, so that their
    // latency overlaps it
    constexpr int CPF = 4;
    cplx<T> cv[CPF];
#pragma unroll
    for (int j = 0; j < CPF; ++j) {
        const int c = tid + j * NTHR;
        if (c < a.ncols) cv[j] = crow[c];
    }
    load_tw<T>(tw, reinterpret_cast<const cplx<T> *>(a.tw0), L);
    for (int i = tid; i < nrows * RS; i += NTHR) pl[i] = cmake<T>(0, 0);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < CPF; ++j) {
        const int c = tid + j * NTHR;
        if (c < a.ncols) pl[a.colslot[c]] = cv[j];
    }
    for (int c = tid + CPF * NTHR; c < a.ncols; c += NTHR) pl[a.colslot[c]] = crow[c];
    __syncthreads();
    for (int f = quad; f < nrows; f += NQ) {                 // y inverse, touched rows
        cplx<T> *p = pl + f * RS;
        cplx<T> v[M];
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] = p[q + 4 * m + (4 * m / M) * PD];
        quad_a<T, M, 1>(v, tw, q);
#pragma unroll
        for (int k = 0; k < M; ++k) p[k + MB * rq] = v[k];
    }
    __syncthreads();
    const T *vz = reinterpret_cast<const T *>(a.vz) + (int64_t)z * L * L;
    // V(r) loaded ahead of the x transforms (VPF; always for complex64), or at its
    // use (fewer VGPRs: complex128 on 64-point planes 182 against 208 at 256 threads)
    for (int y = quad; y < L; y += NQ) {                     // x inverse, V, x forward
        const int yc = y + (y / M) * PD;
        T vv[M];
        if constexpr (VPF) {
#pragma unroll
            for (int k = 0; k < M; ++k) vv[k] = vz[(k + M * rq) * L + y];
        }
        cplx<T> v[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            int dx = q + 4 * m - rowlo;
            if (dx < 0) dx += L;
            v[m] = dx < nrows ? pl[dx * RS + yc] : cmake<T>(0, 0);
        }
        quad_a<T, M, 1>(v, tw, q);
#pragma unroll
        for (int k = 0; k < M; ++k) v[k] = cscale<T>(v[k], VPF ? vv[k] : vz[(k + M * rq) * L + y]);
        quad_b<T, M, -1>(v, tw, q);
#pragma unroll
        for (int k = 0; k < M; ++k) {
            int dx = q + 4 * k - rowlo;
            if (dx < 0) dx += L;
            if (dx < nrows) pl[dx * RS + yc] = v[k];
        }
    }
    __syncthreads();
    for (int f = quad; f < nrows; f += NQ) {                 // y forward, touched rows
        cplx<T> *p = pl + f * RS;
        cplx<T> v[M];
#pragma unroll
        for (int k = 0; k < M; ++k) v[k] = p[k + MB * rq];
        quad_b<T, M, -1>(v, tw, q);
#pragma unroll
        for (int k = 0; k < M; ++k) p[q + 4 * k + (4 * k / M) * PD] = v[k];
    }
    __syncthreads();
    for (int c = tid; c < a.ncols; c += NTHR) crow[c] = pl[a.colslot[c]];
}

template <typename T, int M, int NTHR, bool VPF>
__global__ __launch_bounds__(NTHR) void xy_quad(XYArgs a, cplx<T> *__restrict__ cols) {
    xy_quad_body<T, M, NTHR, VPF>(a, cols, blockIdx.x, blockIdx.y);
}

template <typename T, int M, int NTHR>
__global__ __launch_bounds__(NTHR) void xy_quad_jobs(const FftJob *__restrict__ jobs, const int *__restrict__ mask,
                                                     int nb) {
    const FftJob &j = jobs[blockIdx.y / nb];
    if (!mask[j.prob]) return;
    xy_quad_body<T, M, NTHR>(j.xy, reinterpret_cast<cplx<T> *>(j.cols), blockIdx.x, blockIdx.y % nb);
}

// timing input of the autotuner: values in [-1, 1) from an integer hash of the index
__global__ void k_fill_tune(float2 *__restrict__ p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t h = (uint32_t)i * 2654435761u;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    p[i] = make_float2((float)(h & 0xffff) / 32768.0f - 1.0f, (float)(h >> 16) / 32768.0f - 1.0f);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <typename T> static int pick_threads(const FftPlan &p, int howmany) {
    for (int t : {256, 512, 1024})
        if (fft_fits<T>(p, howmany, t)) return t;
    return 0;
}

template <typename T>
static ZArgs zargs(pw_ctx *ctx, int nb) {
    ZArgs a;
    a.plan = ctx->plan[2];
    a.n2 = ctx->cell.n[2];
    a.ncols = ctx->basis.ncols;
    a.cb = ctx->cb;
    a.nb = nb;
    a.colstart = ctx->d_colstart.as<int32_t>();
    a.zmap = ctx->d_zmap.as<int32_t>();
    a.tw = sizeof(T) == 8 ? ctx->d_tw64[2].p : ctx->d_tw32[2].p;
    return a;
}

template <typename T>
static XYArgs xyargs(pw_ctx *ctx) {
    XYArgs a;
    a.plan0 = ctx->plan[0];
    a.plan1 = ctx->plan[1];
    a.n0 = ctx->cell.n[0];
    a.n1 = ctx->cell.n[1];
    a.n2 = ctx->cell.n[2];
    a.ncols = ctx->basis.ncols;
    a.rowlo = ((ctx->basis.n0min % a.n0) + a.n0) % a.n0;
    a.nrows = ctx->basis.n0max - ctx->basis.n0min + 1;
    a.colpos = ctx->d_colpos.as<int32_t>();
    a.colslot = ctx->d_colslot.as<int32_t>();
    a.tw0 = sizeof(T) == 8 ? ctx->d_tw64[0].p : ctx->d_tw32[0].p;
    a.tw1 = sizeof(T) == 8 ? ctx->d_tw64[1].p : ctx->d_tw32[1].p;
    a.vz = sizeof(T) == 8 ? ctx->d_vz64.p : ctx->d_vz32.p;
    return a;
}

// kernels asking for more than 64 KiB of dynamic LDS must say so first
template <typename F> static void allow_lds(F *kernel, size_t lds) {
    PW_CHECK(lds <= 160 * 1024, PW_EUNSUPPORTED, "kernel needs %zu bytes of LDS", lds);
    if (lds > 64 * 1024)
        PW_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
}

// z passes: launch with a compile-time length when one is built for n2
template <typename T, typename LZ, int NTHR>
static void zinv_go(const ZArgs &a, int ncb, int nb, size_t lds, hipStream_t s, const void *psi, int64_t ld,
                    void *cols) {
    allow_lds(zpass_inv<T, NTHR, LZ>, lds);
    hipLaunchKernelGGL((zpass_inv<T, NTHR, LZ>), dim3(ncb, nb), dim3(NTHR), lds, s, a,
                       reinterpret_cast<const cplx<T> *>(psi), ld, reinterpret_cast<cplx<T> *>(cols));
}

template <typename T, typename LZ, int NTHR>
static void zfwd_go(const ZArgs &a, int ncb, int nb, size_t lds, hipStream_t s, const void *cols, const void *psi,
                    int64_t ld, const double *kin, double shift, double scale, void *out, int64_t ldo) {
    allow_lds(zpass_fwd<T, NTHR, LZ>, lds);
    hipLaunchKernelGGL((zpass_fwd<T, NTHR, LZ>), dim3(ncb, nb), dim3(NTHR), lds, s, a,
                       reinterpret_cast<const cplx<T> *>(cols), reinterpret_cast<const cplx<T> *>(psi), ld, kin,
                       shift, scale, reinterpret_cast<cplx<T> *>(out), ldo);
}


template <typename T> static FftChoice &choice_of(pw_ctx *ctx, int pass) {
    FftTune &t = ctx->tune[sizeof(T) == 8 ? 0 : 1];
    return pass == 0 ? t.zinv : pass == 1 ? t.xy : t.zfwd;
}

static bool z_has_ct(int n2) {
    switch (n2) {
        case 16: case 20: case 32: case 40: case 48: case 64: case 96: case 128: case 192: case 384: case 512:
            return true;
        default: return false;
    }
}

// dispatch a functor on (length policy, threads) for a z-pass length: the
// compile-time length unless `runtime`, else the runtime plan with nthr_rt threads
template <typename T, typename F> static void with_zlen(int n2, int nthr_rt, bool runtime, F &&f) {
#define PW_ZCASE(L)                                                                   \
    case L: {                                                                         \
        constexpr int t = ct_threads<T>(L, kZcb);                                     \
        static_assert(t > 0, "z length does not fit");                              \
        f.template operator()<CtLen<L>, t>();                                         \
        return;                                                                       \
    }
    if (!runtime) {
        switch (n2) {
            PW_ZCASE(16) PW_ZCASE(20) PW_ZCASE(32) PW_ZCASE(40) PW_ZCASE(48) PW_ZCASE(64) PW_ZCASE(96)
            PW_ZCASE(128) PW_ZCASE(192) PW_ZCASE(384) PW_ZCASE(512)
            default: break;
        }
    }
#undef PW_ZCASE
    switch (nthr_rt) {
        case 256: f.template operator()<RtLen, 256>(); return;
        case 512: f.template operator()<RtLen, 512>(); return;
        case 1024: f.template operator()<RtLen, 1024>(); return;
        default: PW_CHECK(false, PW_EUNSUPPORTED, "FFT length %d does not fit the register budget", n2);
    }
}

template <typename T> struct ZinvGo {
    const ZArgs &a; int ncb, nb; size_t lds; hipStream_t s; const void *psi; int64_t ld; void *cols;
    template <typename LZ, int NT> void operator()() { zinv_go<T, LZ, NT>(a, ncb, nb, lds, s, psi, ld, cols); }
};

template <typename T> struct ZfwdGo {
    const ZArgs &a; int ncb, nb; size_t lds; hipStream_t s; const void *cols, *psi; int64_t ld;
    const double *kin; double shift, scale; void *out; int64_t ldo;
    template <typename LZ, int NT> void operator()() {
        zfwd_go<T, LZ, NT>(a, ncb, nb, lds, s, cols, psi, ld, kin, shift, scale, out, ldo);
    }
};

// z passes honour the context's launch choice (autotuner) for their pass
template <typename T> static int z_setup(pw_ctx *ctx, int pass, ZArgs &a, bool &runtime) {
    const FftChoice &c = choice_of<T>(ctx, pass);
    runtime = c.kind == 2;
    if (runtime) {
        a.plan = c.p0;
        return c.nthr;
    }
    return pick_threads<T>(a.plan, a.cb);
}

template <typename T>
void launch_zinv(pw_ctx *ctx, int nb, const void *psi, int64_t ld, void *cols, hipStream_t s) {
    ZArgs a = zargs<T>(ctx, nb);
    PW_CHECK(a.cb == kZcb, PW_EINVAL, "column block mismatch");
    const int ncb = (a.ncols + a.cb - 1) / a.cb;
    const size_t lds = sizeof(cplx<T>) * (a.n2 + (size_t)a.cb * (a.n2 + 1));
    bool runtime;
    const int nthr = z_setup<T>(ctx, 0, a, runtime);
    ZinvGo<T> go{a, ncb, nb, lds, s, psi, ld, cols};
    with_zlen<T>(a.n2, nthr, runtime, go);
    PW_LAUNCH_CHECK();
}

template <typename T>
void launch_zfwd(pw_ctx *ctx, int nb, const void *cols, const void *psi, int64_t ld, const double *kin,
                 double shift, double scale, void *out, int64_t ldo, hipStream_t s) {
    ZArgs a = zargs<T>(ctx, nb);
    PW_CHECK(a.cb == kZcb, PW_EINVAL, "column block mismatch");
    const int ncb = (a.ncols + a.cb - 1) / a.cb;
    const size_t lds = sizeof(cplx<T>) * (a.n2 + (size_t)a.cb * (a.n2 + 1));
    bool runtime;
    const int nthr = z_setup<T>(ctx, 2, a, runtime);
    ZfwdGo<T> go{a, ncb, nb, lds, s, cols, psi, ld, kin, shift, scale, out, ldo};
    with_zlen<T>(a.n2, nthr, runtime, go);
    PW_LAUNCH_CHECK();
}

static bool xy_has_quad(int n0, int n1) {
    return n0 == n1 && (n0 == 16 || n0 == 32 || n0 == 48 || n0 == 64 || n0 == 96 || n0 == 128);
}

// LDS of the four-lane kernel: twiddles and the touched rows of one plane
template <typename T> static size_t quad_lds(const XYArgs &a) {
    return sizeof(cplx<T>) * ((size_t)a.n0 + (size_t)a.nrows * quad_rs(std::max(1, a.n1 / 4)));
}

template <typename T, int M, int NTHR, bool VPF>
static void quad_go(const XYArgs &a, int nb, hipStream_t s, void *cols) {
    const size_t lds = quad_lds<T>(a);
    allow_lds(xy_quad<T, M, NTHR, VPF>, lds);
    hipLaunchKernelGGL((xy_quad<T, M, NTHR, VPF>), dim3(a.n2, nb), dim3(NTHR), lds, s, a,
                       reinterpret_cast<cplx<T> *>(cols));
}

// vpf: complex128 with V(r) loaded ahead (planes of at most 64 points; complex64
// always loads it ahead)
template <typename T, int NTHR>
static void quad_len(const XYArgs &a, int nb, hipStream_t s, void *cols, bool vpf) {
    constexpr bool D = sizeof(T) == 8;
    if (D && vpf) {
        if constexpr (D) {
            switch (a.n0) {
                case 16: quad_go<T, 4, NTHR, true>(a, nb, s, cols); return;
                case 32: quad_go<T, 8, NTHR, true>(a, nb, s, cols); return;
                case 48: quad_go<T, 12, NTHR, true>(a, nb, s, cols); return;
                case 64: quad_go<T, 16, NTHR, true>(a, nb, s, cols); return;
                default: PW_CHECK(false, PW_EUNSUPPORTED, "no V-prefetch xy kernel for %d x %d", a.n0, a.n1);
            }
        }
        return;
    }
    switch (a.n0) {
        case 16: quad_go<T, 4, NTHR, !D>(a, nb, s, cols); break;
        case 32: quad_go<T, 8, NTHR, !D>(a, nb, s, cols); break;
        case 48: quad_go<T, 12, NTHR, !D>(a, nb, s, cols); break;
        case 64: quad_go<T, 16, NTHR, !D>(a, nb, s, cols); break;
        case 96: quad_go<T, 24, NTHR, !D>(a, nb, s, cols); break;
        case 128: quad_go<T, 32, NTHR, !D>(a, nb, s, cols); break;
        default: PW_CHECK(false, PW_EUNSUPPORTED, "no four-lane xy kernel for %d x %d", a.n0, a.n1);
    }
}

template <typename T, int MODE, typename L0, typename L1, int NTHR>
static void xy_go(const XYArgs &a, int nb, size_t lds, hipStream_t s, void *cols, void *grid) {
    allow_lds(xy_pass<T, NTHR, MODE, L0, L1>, lds);
    hipLaunchKernelGGL((xy_pass<T, NTHR, MODE, L0, L1>), dim3(a.n2, nb), dim3(NTHR), lds, s, a,
                       reinterpret_cast<cplx<T> *>(cols), reinterpret_cast<cplx<T> *>(grid));
}

template <typename T, int MODE>
void launch_xy(pw_ctx *ctx, int nb, void *cols, void *grid, hipStream_t s) {
    XYArgs a = xyargs<T>(ctx);
    const FftChoice &c = choice_of<T>(ctx, 1);
    // default for the V(r) pass on 16/32/48/64/96/128-point planes: the four-lane kernel
    if (MODE == 0 && (c.kind == 3 || (c.kind == 0 && xy_has_quad(a.n0, a.n1) && quad_lds<T>(a) <= 160 * 1024))) {
        PW_CHECK(xy_has_quad(a.n0, a.n1), PW_EUNSUPPORTED, "no four-lane xy kernel for %d x %d", a.n0, a.n1);
        const int nthr = c.kind == 3 ? c.nthr : (sizeof(T) == 8 || a.n0 > 64 ? 256 : 192);
        const bool vpf = c.kind == 3 && c.vpf;
        switch (nthr) {
            case 128: quad_len<T, 128>(a, nb, s, cols, vpf); break;
            case 192: quad_len<T, 192>(a, nb, s, cols, vpf); break;
            case 256: quad_len<T, 256>(a, nb, s, cols, vpf); break;
            case 512: quad_len<T, 512>(a, nb, s, cols, vpf); break;
            default: PW_CHECK(false, PW_EUNSUPPORTED, "four-lane xy kernel with %d threads", nthr);
        }
        PW_LAUNCH_CHECK();
        return;
    }
    const size_t lds = sizeof(cplx<T>) * (a.n0 + a.n1 + (size_t)a.n0 * (a.n1 + 1));
    PW_CHECK(lds <= 160 * 1024, PW_EUNSUPPORTED, "xy plane %dx%d does not fit LDS", a.n0, a.n1);
    if (c.kind != 2 && a.n0 == a.n1) {
#define PW_XYCASE(L)                                                                        \
    case L: {                                                                               \
        constexpr int t1 = ct_threads<T>(L, L), t = t1;                                    \
        if constexpr (t > 0) {                                                              \
            xy_go<T, MODE, CtLen<L>, CtLen<L>, t>(a, nb, lds, s, cols, grid);                \
            PW_LAUNCH_CHECK();                                                              \
            return;                                                                         \
        }                                                                                   \
        break;                                                                              \
    }
        switch (a.n0) {
            PW_XYCASE(16) PW_XYCASE(32) PW_XYCASE(40) PW_XYCASE(48) PW_XYCASE(64) PW_XYCASE(96) PW_XYCASE(128)
            default: break;
        }
#undef PW_XYCASE
    }
    int nthr = 0;
    if (c.kind == 2) {
        a.plan0 = c.p0;
        a.plan1 = c.p1;
        nthr = c.nthr;
    } else {
        for (int t : {256, 512, 1024})
            if (fft_fits<T>(a.plan1, a.n0, t) && fft_fits<T>(a.plan0, a.n1, t)) { nthr = t; break; }
    }
    switch (nthr) {
        case 256: xy_go<T, MODE, RtLen, RtLen, 256>(a, nb, lds, s, cols, grid); break;
        case 512: xy_go<T, MODE, RtLen, RtLen, 512>(a, nb, lds, s, cols, grid); break;
        case 1024: xy_go<T, MODE, RtLen, RtLen, 1024>(a, nb, lds, s, cols, grid); break;
        default: PW_CHECK(false, PW_EUNSUPPORTED, "xy FFT does not fit the register budget");
    }
    PW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Batched complex128 H psi over independent problems (contexts) with the same
// band count: the three FFT passes once per group of equal grids and the two
// projector GEMMs once for all problems, each problem's mask entry deciding at
// run time whether its blocks are touched.  Every problem sees the kernels,
// launch shapes and split-K chunking of its own pw_hpsi call (default launch
// choices, all its bands in one FFT chunk), so its result is bit for bit that of
// its own call.
// ---------------------------------------------------------------------------
struct HpsiGroup {
    std::vector<FftJob> h;
    DevBuf d;
    pw_ctx *rep;              // a context of the group (grid, launch choices)
    size_t quad_lds = 0;
};
struct HpsiBatch {
    int nb = 0, nprob = 0;
    std::deque<HpsiGroup> groups;
    // projector GEMM jobs, one per problem, per launch of proj_band_split's band ranges
    std::vector<std::vector<NtJob>> nt;
    std::vector<std::vector<NnJob>> nn;
    std::deque<DevBuf> d_nt, d_nn;
    const int *mask = nullptr;
    int nn_cfg = -1;
};

template <typename T, int NTHR, typename LZ>
static void zinv_jobs_go(const HpsiGroup &g, int nb, size_t lds, const int *mask, hipStream_t s) {
    allow_lds(zpass_inv_jobs<T, NTHR, LZ>, lds);
    int ncb = 1;
    for (const FftJob &j : g.h) ncb = std::max(ncb, (j.z.ncols + j.z.cb - 1) / j.z.cb);
    hipLaunchKernelGGL((zpass_inv_jobs<T, NTHR, LZ>), dim3(ncb, (unsigned)(g.h.size() * nb)), dim3(NTHR), lds, s,
                       g.d.as<FftJob>(), mask, nb);
}
template <typename T, int NTHR, typename LZ>
static void zfwd_jobs_go(const HpsiGroup &g, int nb, size_t lds, const int *mask, hipStream_t s) {
    allow_lds(zpass_fwd_jobs<T, NTHR, LZ>, lds);
    int ncb = 1;
    for (const FftJob &j : g.h) ncb = std::max(ncb, (j.z.ncols + j.z.cb - 1) / j.z.cb);
    hipLaunchKernelGGL((zpass_fwd_jobs<T, NTHR, LZ>), dim3(ncb, (unsigned)(g.h.size() * nb)), dim3(NTHR), lds, s,
                       g.d.as<FftJob>(), mask, nb);
}
template <typename T> struct ZJobsGo {
    const HpsiGroup &g; int nb; size_t lds; const int *mask; hipStream_t s; bool fwd;
    template <typename LZ, int NT> void operator()() {
        if (fwd) zfwd_jobs_go<T, NT, LZ>(g, nb, lds, mask, s);
        else zinv_jobs_go<T, NT, LZ>(g, nb, lds, mask, s);
    }
};
template <typename T, int M, int NTHR>
static void quad_jobs_go(const HpsiGroup &g, int nb, const int *mask, hipStream_t s) {
    allow_lds(xy_quad_jobs<T, M, NTHR>, g.quad_lds);
    hipLaunchKernelGGL((xy_quad_jobs<T, M, NTHR>), dim3(g.rep->cell.n[2], (unsigned)(g.h.size() * nb)), dim3(NTHR),
                       g.quad_lds, s, g.d.as<FftJob>(), mask, nb);
}
template <typename T, typename L0, typename L1, int NTHR>
static void xy_jobs_go(const HpsiGroup &g, int nb, size_t lds, const int *mask, hipStream_t s) {
    allow_lds(xy_pass_jobs<T, NTHR, L0, L1>, lds);
    hipLaunchKernelGGL((xy_pass_jobs<T, NTHR, L0, L1>), dim3(g.rep->cell.n[2], (unsigned)(g.h.size() * nb)),
                       dim3(NTHR), lds, s, g.d.as<FftJob>(), mask, nb);
}

// the xy pass of pw_hpsi's default choice for this group's grid (complex128)
static void xy_jobs(const HpsiGroup &g, int nb, const int *mask, hipStream_t s) {
    using T = double;
    const XYArgs &a = g.h[0].xy;
    if (xy_has_quad(a.n0, a.n1) && g.quad_lds <= 160 * 1024) {
        switch (a.n0) {
            case 16: quad_jobs_go<T, 4, 256>(g, nb, mask, s); break;
            case 32: quad_jobs_go<T, 8, 256>(g, nb, mask, s); break;
            case 48: quad_jobs_go<T, 12, 256>(g, nb, mask, s); break;
            case 64: quad_jobs_go<T, 16, 256>(g, nb, mask, s); break;
            case 96: quad_jobs_go<T, 24, 256>(g, nb, mask, s); break;
            default: quad_jobs_go<T, 32, 256>(g, nb, mask, s); break;
        }
        PW_LAUNCH_CHECK();
        return;
    }
    const size_t lds = sizeof(cplx<T>) * (a.n0 + a.n1 + (size_t)a.n0 * (a.n1 + 1));
    PW_CHECK(lds <= 160 * 1024, PW_EUNSUPPORTED, "xy plane %dx%d does not fit LDS", a.n0, a.n1);
    if (a.n0 == a.n1) {
#define PW_XYJCASE(L)                                                                       \
    case L: {                                                                               \
        constexpr int t = ct_threads<T>(L, L);                                              \
        if constexpr (t > 0) {                                                              \
            xy_jobs_go<T, CtLen<L>, CtLen<L>, t>(g, nb, lds, mask, s);                      \
            PW_LAUNCH_CHECK();                                                              \
            return;                                                                         \
        }                                                                                   \
        break;                                                                              \
    }
        switch (a.n0) {
            PW_XYJCASE(16) PW_XYJCASE(32) PW_XYJCASE(40) PW_XYJCASE(48) PW_XYJCASE(64) PW_XYJCASE(96) PW_XYJCASE(128)
            default: break;
        }
#undef PW_XYJCASE
    }
    int nthr = 0;
    for (int t : {256, 512, 1024})
        if (fft_fits<T>(a.plan1, a.n0, t) && fft_fits<T>(a.plan0, a.n1, t)) { nthr = t; break; }
    switch (nthr) {
        case 256: xy_jobs_go<T, RtLen, RtLen, 256>(g, nb, lds, mask, s); break;
        case 512: xy_jobs_go<T, RtLen, RtLen, 512>(g, nb, lds, mask, s); break;
        case 1024: xy_jobs_go<T, RtLen, RtLen, 1024>(g, nb, lds, mask, s); break;
        default: PW_CHECK(false, PW_EUNSUPPORTED, "xy FFT does not fit the register budget");
    }
    PW_LAUNCH_CHECK();
}

static bool default_choices(pw_ctx *c) {
    const FftTune &t = c->tune[0];
    return t.zinv.kind == 0 && t.xy.kind == 0 && t.zfwd.kind == 0;
}

bool hpsi_batch_ok(int n, pw_ctx *const *ctx, int nb, std::string *why) {
    // the projection of every problem in one launch per band range: one NT tile shape
    // (it follows the projector count)
    const int nb1 = proj_band_split(nb);
    int tile0 = -1, tile1 = -1;
    for (int p = 0; p < n; ++p) {
        pw_ctx *c = ctx[p];
        const char *w = nullptr;
        const int t0 = c->nproj ? nt_tile_id(c->nproj, nb1, false) : -1;
        const int t1 = c->nproj && nb > nb1 ? nt_tile_id(c->nproj, nb - nb1, false) : -1;
        if (!c->d_beta64.p && c->nproj) w = "no stored complex128 projector table";
        else if (!default_choices(c)) w = "autotuned FFT launch choices";
        else if (c->cols_bands < nb || c->max_bands < nb) w = "bands beyond one FFT chunk";
        else if (c->nn_tune.get(nb) >= 0 || c->rot_tune.get(nb) >= 0) w = "autotuned GEMM tiles";
        else if ((t0 >= 0 && tile0 >= 0 && t0 != tile0) || (t1 >= 0 && tile1 >= 0 && t1 != tile1))
            w = "projector counts that take different GEMM tiles";
        if (t0 >= 0) tile0 = t0;
        if (t1 >= 0) tile1 = t1;
        if (w) {
            if (why) *why = w;
            return false;
        }
    }
    return true;
}

HpsiBatch *hpsi_batch_create(int n, pw_ctx *const *ctx, int nb, void *const *in, const int64_t *ld,
                             void *const *out, const int64_t *ldo, const double *shift, const int *mask) {
    std::unique_ptr<HpsiBatch> B(new HpsiBatch);
    B->nb = nb;
    B->nprob = n;
    B->mask = mask;
    std::map<std::tuple<int, int, int>, int> gid;
    const int nb1 = proj_band_split(nb), nlaunch = (nb + nb1 - 1) / nb1;
    B->nt.resize(nlaunch);
    B->nn.resize(nlaunch);
    for (int p = 0; p < n; ++p) {
        pw_ctx *c = ctx[p];
        const auto key = std::make_tuple(c->cell.n[0], c->cell.n[1], c->cell.n[2]);
        auto it = gid.find(key);
        if (it == gid.end()) {
            it = gid.emplace(key, (int)B->groups.size()).first;
            B->groups.emplace_back();
            B->groups.back().rep = c;
        }
        HpsiGroup &g = B->groups[it->second];
        FftJob j{};
        j.z = zargs<double>(c, nb);
        j.xy = xyargs<double>(c);
        j.prob = p;
        j.in = in[p];
        j.ld = ld[p];
        j.cols = c->d_cols.p;
        j.kin = c->d_kin.as<double>();
        j.shift = shift[p];
        j.scale = 1.0 / ((double)c->cell.n[0] * c->cell.n[1] * c->cell.n[2]);
        j.out = out[p];
        j.ldo = ldo[p];
        g.quad_lds = std::max(g.quad_lds, quad_lds<double>(j.xy));
        g.h.push_back(j);
        for (int l = 0; l < nlaunch; ++l) {
            const int b0 = l * nb1, nbl = std::min(nb1, nb - b0);
            if (c->nproj) {
                double2 *proj = c->d_proj.as<double2>() + (size_t)b0 * c->nproj;
                B->nt[l].push_back(nt_job(c->nproj, nbl, c->basis.npw, true, c->d_beta64.p, c->basis.npw,
                                          (const double2 *)in[p] + (size_t)b0 * ld[p], ld[p], 1.0,
                                          c->d_dproj.as<double>(), 0.0, proj, c->nproj, c->d_partial.p, false));
                NnJob q{};
                q.M = nbl; q.J = c->basis.npw; q.K = c->nproj; q.nz = 1; q.lower = 0;
                q.W = proj; q.ldw = c->nproj;
                q.X[0] = c->d_beta64.as<double2>(); q.Out[0] = (double2 *)out[p] + (size_t)b0 * ldo[p];
                q.ldx = c->basis.npw; q.ldo = ldo[p]; q.alpha = 1.0; q.beta = 1.0;
                B->nn[l].push_back(q);
            } else {
                // keep the job index equal to the problem index: an empty job the kernels skip
                NtJob e{};
                e.M = 0; e.N = 0; e.nsplit = 0;
                B->nt[l].push_back(e);
                NnJob q{};
                B->nn[l].push_back(q);
            }
        }
    }
    for (HpsiGroup &g : B->groups) {
        g.d.alloc(g.h.size() * sizeof(FftJob));
        PW_HIP(hipMemcpy(g.d.p, g.h.data(), g.h.size() * sizeof(FftJob), hipMemcpyHostToDevice));
    }
    for (int l = 0; l < nlaunch; ++l) {
        B->d_nt.emplace_back();
        B->d_nt.back().alloc(B->nt[l].size() * sizeof(NtJob));
        PW_HIP(hipMemcpy(B->d_nt.back().p, B->nt[l].data(), B->nt[l].size() * sizeof(NtJob), hipMemcpyHostToDevice));
        B->d_nn.emplace_back();
        B->d_nn.back().alloc(B->nn[l].size() * sizeof(NnJob));
        PW_HIP(hipMemcpy(B->d_nn.back().p, B->nn[l].data(), B->nn[l].size() * sizeof(NnJob), hipMemcpyHostToDevice));
    }
    return B.release();
}

void hpsi_batch_destroy(HpsiBatch *b) { delete b; }

void hpsi_batch_run(HpsiBatch *B, hipStream_t s) {
    using T = double;
    const int nb = B->nb;
    for (const HpsiGroup &g : B->groups) {
        const ZArgs &a = g.h[0].z;
        const size_t lds = sizeof(cplx<T>) * (a.n2 + (size_t)a.cb * (a.n2 + 1));
        const int nthr = pick_threads<T>(a.plan, a.cb);
        ZJobsGo<T> inv{g, nb, lds, B->mask, s, false};
        with_zlen<T>(a.n2, nthr, false, inv);
        PW_LAUNCH_CHECK();
        xy_jobs(g, nb, B->mask, s);
        ZJobsGo<T> fwd{g, nb, lds, B->mask, s, true};
        with_zlen<T>(a.n2, nthr, false, fwd);
        PW_LAUNCH_CHECK();
    }
    bool any = false;
    for (size_t q = 0; q < B->nt[0].size(); ++q) any = any || B->nt[0][q].M > 0;
    if (!any) return;
    for (size_t l = 0; l < B->nt.size(); ++l)
        zgemm_nt_jobs(B->nt[l], B->d_nt[l].as<NtJob>(), B->mask, true, true, true, s);
    for (size_t l = 0; l < B->nn.size(); ++l)
        zgemm_nn_jobs_launch(B->nn[l], B->d_nn[l].as<NnJob>(), B->mask, -1, true, s);
}

// ---------------------------------------------------------------------------
// Autotuner: for each pass (z inverse, xy with V, z forward) time every launch
// variant that fits this grid -- the compile-time length kernel and the
// runtime-plan kernel for each radix schedule and thread count -- on nb bands
// and keep the fastest; for complex128 also the tiles of the back-projection GEMM
// and of the block-rotation GEMM.
// Results are cached per (grid, sphere, dtype, nb).
// ---------------------------------------------------------------------------
template <typename T> static bool xy_has_ct(int n) {
    switch (n) {
#define PW_XYH(L) \
    case L: return ct_threads<T>(L, L) > 0;
        PW_XYH(16) PW_XYH(32) PW_XYH(40) PW_XYH(48) PW_XYH(64) PW_XYH(96) PW_XYH(128)
#undef PW_XYH
        default: return false;
    }
}

static bool same_plan(const FftPlan &a, const FftPlan &b) {
    if (a.n != b.n || a.nstages != b.nstages) return false;
    for (int i = 0; i < a.nstages; ++i)
        if (a.radix[i] != b.radix[i]) return false;
    return true;
}

// the choice a candidate record stands for; false if it does not fit
template <typename T> static bool choice_from(pw_ctx *ctx, const pw_fft_cand &r, FftChoice &c) {
    const int n0 = ctx->cell.n[0], n1 = ctx->cell.n[1], n2 = ctx->cell.n[2];
    c = FftChoice{};
    c.kind = r.kind;
    if (r.kind == 0) return true;
    if (r.kind == 1) return r.pass == 1 ? (n0 == n1 && xy_has_ct<T>(n0)) : z_has_ct(n2);
    if (r.kind == 3) {
        c.nthr = r.nthr;
        // sched 1: complex128 with V(r) loaded ahead, on planes of at most 64 points
        c.vpf = r.sched == 1;
        if (r.sched != 0 && !(r.sched == 1 && sizeof(T) == 8 && n0 <= 64)) return false;
        // (512 threads would spill the complex128 96- and 128-point kernels: not offered)
        return r.pass == 1 && xy_has_quad(n0, n1) && quad_lds<T>(xyargs<T>(ctx)) <= 160 * 1024 &&
               (c.nthr == 128 || c.nthr == 192 || c.nthr == 256 || (c.nthr == 512 && (sizeof(T) == 4 || n0 <= 64)));
    }
    if (r.kind != 2 || r.sched < 0 || r.sched > 2) return false;
    c.nthr = r.nthr;
    if (c.nthr != 256 && c.nthr != 512 && c.nthr != 1024) return false;
    if (r.pass == 1) {
        c.p0 = make_plan_sched(n0, r.sched);
        c.p1 = make_plan_sched(n1, r.sched);
        return fft_fits<T>(c.p1, n0, c.nthr) && fft_fits<T>(c.p0, n1, c.nthr);
    }
    c.p0 = make_plan_sched(n2, r.sched);
    return fft_fits<T>(c.p0, kZcb, c.nthr);
}

template <typename T> static std::vector<pw_fft_cand> candidates(pw_ctx *ctx, int pass) {
    std::vector<pw_fft_cand> out;
    pw_fft_cand r{};
    r.pass = pass;
    FftChoice c;
    r.kind = 1;
    if (choice_from<T>(ctx, r, c)) out.push_back(r);
    for (int vpf = 0; vpf < 2; ++vpf)
        for (int t : {128, 192, 256, 512}) {
            r = pw_fft_cand{};
            r.pass = pass;
            r.kind = 3;
            r.nthr = t;
            r.sched = vpf;
            if (choice_from<T>(ctx, r, c)) out.push_back(r);
        }
    std::vector<FftChoice> seen;
    for (int sched = 0; sched < 3; ++sched) {
        for (int t : {256, 512, 1024}) {
            r = pw_fft_cand{};
            r.pass = pass;
            r.kind = 2;
            r.sched = sched;
            r.nthr = t;
            if (!choice_from<T>(ctx, r, c)) continue;
            bool dup = false;
            for (const FftChoice &o : seen)
                if (o.nthr == t && same_plan(o.p0, c.p0) && (pass != 1 || same_plan(o.p1, c.p1))) dup = true;
            if (dup) continue;
            seen.push_back(c);
            r.nradix = c.p0.nstages;
            for (int i = 0; i < c.p0.nstages; ++i) r.radix[i] = c.p0.radix[i];
            out.push_back(r);
        }
    }
    return out;
}

template <typename T>
static void run_pass(pw_ctx *ctx, int pass, int nb, void *in, void *out, hipStream_t s) {
    const int64_t ld = ctx->basis.npw;
    if (pass == 0) launch_zinv<T>(ctx, nb, in, ld, ctx->d_cols.p, s);
    else if (pass == 1) launch_xy<T, 0>(ctx, nb, ctx->d_cols.p, nullptr, s);
    else launch_zfwd<T>(ctx, nb, ctx->d_cols.p, in, ld, ctx->d_kin.as<double>(), 0.0, 1.0, out, ld, s);
}

namespace {
struct TuneKey {
    int n[3], ncols, npw, dbl, nb, nproj, max_bands;
    bool operator<(const TuneKey &o) const {
        return std::tie(n[0], n[1], n[2], ncols, npw, dbl, nb, nproj, max_bands) <
               std::tie(o.n[0], o.n[1], o.n[2], o.ncols, o.npw, o.dbl, o.nb, o.nproj, o.max_bands);
    }
};
struct TuneVal {
    FftTune tune;
    int nn = -1, rot = -1;
    std::vector<pw_fft_cand> recs;
    int bf16 = -1;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune_cache;
}  // namespace

template <typename T>
void autotune_fft(pw_ctx *ctx, int nb, int reps, std::vector<pw_fft_cand> &recs, hipStream_t s) {
    PW_CHECK(nb >= 1 && nb <= ctx->max_bands && reps >= 1, PW_EINVAL, "bad autotune sizes");
    PW_CHECK(nb <= ctx->cols_bands, PW_EINVAL, "autotune on %d bands: the column grid holds %d", nb, ctx->cols_bands);
    FftTune &tune = ctx->tune[sizeof(T) == 8 ? 0 : 1];
    const TuneKey key{{ctx->cell.n[0], ctx->cell.n[1], ctx->cell.n[2]}, ctx->basis.ncols, ctx->basis.npw,
                      sizeof(T) == 8, nb, ctx->nproj, ctx->max_bands};
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            tune = it->second.tune;
            if (it->second.nn >= 0) ctx->nn_tune.set(nb, it->second.nn);
            if (it->second.rot >= 0) ctx->rot_tune.set(nb, it->second.rot);
            if (it->second.bf16 >= 0) ctx->bf16_variant = it->second.bf16;
            recs = it->second.recs;
            return;
        }
    }
    const size_t bytes = (size_t)nb * ctx->basis.npw * sizeof(cplx<T>);
    DevBuf in, out;
    in.alloc(bytes);
    out.alloc(bytes);
    fill_zero(in.p, bytes, s);
    fill_zero(out.p, bytes, s);
    tune = FftTune{};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PW_HIP(hipEventCreate(&e0));
    struct Ev {
        hipEvent_t &a, &b;
        ~Ev() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } guard{e0, e1};
    PW_HIP(hipEventCreate(&e1));
    recs.clear();
    int nn_best = -1, rot_best = -1;
    run_pass<T>(ctx, 0, nb, in.p, out.p, s);              // column grid for the xy timings
    for (int pass = 0; pass < 3; ++pass) {
        std::vector<pw_fft_cand> cs = candidates<T>(ctx, pass);
        const size_t first = recs.size();
        int best = -1;
        for (size_t k = 0; k < cs.size(); ++k) {
            FftChoice c;
            choice_from<T>(ctx, cs[k], c);
            choice_of<T>(ctx, pass) = c;
            run_pass<T>(ctx, pass, nb, in.p, out.p, s);   // warm-up (and LDS attribute)
            PW_HIP(hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r) run_pass<T>(ctx, pass, nb, in.p, out.p, s);
            PW_HIP(hipEventRecord(e1, s));
            PW_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            PW_HIP(hipEventElapsedTime(&ms, e0, e1));
            cs[k].ms = ms / reps;
            if (best < 0 || cs[k].ms < cs[best].ms) best = (int)k;
            recs.push_back(cs[k]);
        }
        PW_CHECK(best >= 0, PW_EUNSUPPORTED, "no FFT launch variant fits pass %d", pass);
        recs[first + best].chosen = 1;
        FftChoice c;
        choice_from<T>(ctx, cs[best], c);
        choice_of<T>(ctx, pass) = c;
        if (pass == 0) run_pass<T>(ctx, 0, nb, in.p, out.p, s);
    }
    // complex128 back-projection GEMM tiles (pass 4) for this band count
    if (sizeof(T) == 8 && ctx->nproj > 0 && ctx->d_beta64.p) {
        const int npw = ctx->basis.npw, K = ctx->nproj;
        fill_zero(ctx->d_proj.p, (size_t)nb * K * sizeof(double2), s);
        const size_t first = recs.size();
        int best = -1;
        for (int id = 0; id < kNnCfgs; ++id) {
            pw_fft_cand r{};
            r.pass = 4;
            r.kind = 3;
            r.sched = id;
            r.nradix = 3;
            nn_cfg_shape(id, r.radix[0], r.radix[1], r.nthr);
            r.radix[2] = nb;
            auto go = [&]() {
                zgemm_nn_launch(nb, npw, K, ctx->d_proj.p, K, ctx->d_beta64.p, npw, 1.0, 0.0, out.p, npw, s, true, id);
            };
            go();
            PW_HIP(hipEventRecord(e0, s));
            for (int k = 0; k < reps; ++k) go();
            PW_HIP(hipEventRecord(e1, s));
            PW_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            PW_HIP(hipEventElapsedTime(&ms, e0, e1));
            r.ms = ms / reps;
            if (best < 0 || r.ms < recs[first + best].ms) best = id;
            recs.push_back(r);
        }
        recs[first + best].chosen = 1;
        nn_best = best;
        ctx->nn_tune.set(nb, best);
    }
    // complex128 block-rotation GEMM tiles (pass 5): Out = W . X with W nb x nb
    if (sizeof(T) == 8) {
        const int npw = ctx->basis.npw;
        DevBuf w;
        w.alloc((size_t)nb * nb * sizeof(double2));
        fill_zero(w.p, (size_t)nb * nb * sizeof(double2), s);
        const size_t first = recs.size();
        int best = -1;
        for (int id = 0; id < kNnCfgs; ++id) {
            pw_fft_cand r{};
            r.pass = 5;
            r.kind = 3;
            r.sched = id;
            r.nradix = 3;
            nn_cfg_shape(id, r.radix[0], r.radix[1], r.nthr);
            r.radix[2] = nb;
            auto go = [&]() { zgemm_nn_launch(nb, npw, nb, w.p, nb, in.p, npw, 1.0, 0.0, out.p, npw, s, false, id); };
            go();
            PW_HIP(hipEventRecord(e0, s));
            for (int k = 0; k < reps; ++k) go();
            PW_HIP(hipEventRecord(e1, s));
            PW_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            PW_HIP(hipEventElapsedTime(&ms, e0, e1));
            r.ms = ms / reps;
            if (best < 0 || r.ms < recs[first + best].ms) best = id;
            recs.push_back(r);
        }
        recs[first + best].chosen = 1;
        rot_best = best;
        ctx->rot_tune.set(nb, best);
        PW_HIP(hipStreamSynchronize(s));
    }
    // complex64 BF16 projector GEMMs beyond 144 bands (pass 6): every launch variant of the
    // projection and back-projection pair, timed on max_bands bands of nonzero values (the
    // matrix cores' power, and with it the clock, depends on the data)
    int bf16_best = -1;
    if (sizeof(T) == 4 && ctx->nproj > 0 && ctx->max_bands > 144 && ctx->d_beta_bf16.p) {
        const int nbw = ctx->max_bands, npw = ctx->basis.npw;
        DevBuf win, wout;
        win.alloc((size_t)nbw * npw * 8);
        wout.alloc((size_t)nbw * npw * 8);
        const size_t nval = (size_t)nbw * npw;
        hipLaunchKernelGGL(k_fill_tune, dim3((unsigned)((nval + 255) / 256)), dim3(256), 0, s,
                           (float2 *)win.p, nval);
        PW_LAUNCH_CHECK();
        fill_zero(wout.p, (size_t)nbw * npw * 8, s);
        const size_t first = recs.size();
        for (int v = 0; v < kBf16WideVariants; ++v) {
            pw_fft_cand r{};
            r.pass = 6;
            r.kind = 3;
            r.sched = v;
            r.radix[2] = nbw;
            auto go = [&]() {
                proj_bf16(ctx->nproj, nbw, npw, ctx->max_bands, ctx->d_beta_bf16.p, ctx->d_dproj32.as<float>(),
                          win.p, npw, ctx->d_bf16_ws.p, ctx->d_partial.p, s, v);
                backproj_bf16(ctx->nproj, nbw, npw, ctx->max_bands, ctx->d_betaT_bf16.p, ctx->d_bf16_ws.p, wout.p,
                              npw, s, v);
            };
            go();
            PW_HIP(hipEventRecord(e0, s));
            for (int k = 0; k < reps; ++k) go();
            PW_HIP(hipEventRecord(e1, s));
            PW_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            PW_HIP(hipEventElapsedTime(&ms, e0, e1));
            r.ms = ms / reps;
            if (bf16_best < 0 || r.ms < recs[first + bf16_best].ms) bf16_best = v;
            recs.push_back(r);
        }
        recs[first + bf16_best].chosen = 1;
        ctx->bf16_variant = bf16_best;
        PW_HIP(hipStreamSynchronize(s));
    }
    PW_HIP(hipStreamSynchronize(s));
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[key] = TuneVal{tune, nn_best, rot_best, recs, bf16_best};
}

template <typename T> void fft_choose(pw_ctx *ctx, const pw_fft_cand &r) {
    if (r.pass == 6) {
        PW_CHECK(sizeof(T) == 4, PW_EUNSUPPORTED, "BF16 GEMM variants are chosen for complex64 only");
        PW_CHECK(r.kind == 0 || (r.kind == 3 && r.sched >= 0 && r.sched < kBf16WideVariants), PW_EUNSUPPORTED,
                 "BF16 GEMM variant unknown");
        ctx->bf16_variant = r.kind == 0 ? 0 : r.sched;
        return;
    }
    if (r.pass == 4 || r.pass == 5) {
        PW_CHECK(sizeof(T) == 8, PW_EUNSUPPORTED, "GEMM tiles are chosen for complex128 only");
        PW_CHECK(r.kind == 0 || (r.kind == 3 && r.sched >= 0 && r.sched < kNnCfgs), PW_EUNSUPPORTED,
                 "GEMM tile candidate unknown");
        PW_CHECK(r.radix[2] >= 1, PW_EINVAL, "GEMM tile candidate needs its band count in radix[2]");
        (r.pass == 4 ? ctx->nn_tune : ctx->rot_tune).set(r.radix[2], r.kind == 0 ? -1 : r.sched);
        return;
    }
    PW_CHECK(r.pass >= 0 && r.pass <= 2, PW_EINVAL, "FFT pass %d unknown", r.pass);
    FftChoice c;
    PW_CHECK(choice_from<T>(ctx, r, c), PW_EUNSUPPORTED, "FFT launch variant does not fit this grid");
    choice_of<T>(ctx, r.pass) = c;
}

template void autotune_fft<double>(pw_ctx *, int, int, std::vector<pw_fft_cand> &, hipStream_t);
template void autotune_fft<float>(pw_ctx *, int, int, std::vector<pw_fft_cand> &, hipStream_t);
template void fft_choose<double>(pw_ctx *, const pw_fft_cand &);
template void fft_choose<float>(pw_ctx *, const pw_fft_cand &);

// explicit instantiations used by api.cpp
template void launch_zinv<double>(pw_ctx *, int, const void *, int64_t, void *, hipStream_t);
template void launch_zinv<float>(pw_ctx *, int, const void *, int64_t, void *, hipStream_t);
template void launch_zfwd<double>(pw_ctx *, int, const void *, const void *, int64_t, const double *, double,
                                  double, void *, int64_t, hipStream_t);
template void launch_zfwd<float>(pw_ctx *, int, const void *, const void *, int64_t, const double *, double,
                                 double, void *, int64_t, hipStream_t);
template void launch_xy<double, 0>(pw_ctx *, int, void *, void *, hipStream_t);
template void launch_xy<double, 1>(pw_ctx *, int, void *, void *, hipStream_t);
template void launch_xy<double, 2>(pw_ctx *, int, void *, void *, hipStream_t);
template void launch_xy<float, 0>(pw_ctx *, int, void *, void *, hipStream_t);
template void launch_xy<float, 1>(pw_ctx *, int, void *, void *, hipStream_t);
template void launch_xy<float, 2>(pw_ctx *, int, void *, void *, hipStream_t);

}  // namespace pw
