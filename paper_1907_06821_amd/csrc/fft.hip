// Sphere <-> grid 3D FFT of the H psi path, staged in LDS, for gfx950.
//
// The local potential is applied as FFT^-1 (V(r) . FFT psi): coefficients on the
// cutoff sphere go to real space with exp(+iG.r), are multiplied by V(r_j) and
// come back with (1/N) exp(-iG.r).  The transform is split in two kinds of pass so
// that only the z-columns that touch the sphere are ever moved through HBM:
//
//   z pass (inverse):  sphere coefficients of CB columns -> LDS -> length-N2 FFTs
//                      -> column grid cols[b][z][c]          (c over touched columns)
//   xy pass:           one (band, z) plane: scatter its columns into an N0 x N1 LDS
//                      plane, 2D inverse FFT, multiply by V(., ., z), 2D forward FFT,
//                      gather the columns back (in place)
//   z pass (forward):  column grid -> LDS -> FFTs -> (1/N) . gather onto the sphere,
//                      fused with the kinetic term (T_G - shift) c(G)
//
// Every 1D transform is a mixed-radix (8, 4, 2, 3, 5) Stockham FFT on LDS data: a
// thread loads its butterflies' inputs into registers, all threads synchronise,
// then write the outputs, so one LDS buffer suffices.  Twiddles exp(-2 pi i t/n)
// come from a table computed on the host in extended precision.
#include "common.h"

namespace pw {

// ---------------------------------------------------------------------------
// small DFTs on registers; sign = -1 forward, +1 inverse
// ---------------------------------------------------------------------------
template <typename T> __device__ inline cplx<T> mul_si(cplx<T> a, int sign) {
    // a * (sign * i)
    return sign > 0 ? cmake<T>(-a.y, a.x) : cmake<T>(a.y, -a.x);
}

template <typename T, int R> struct Dft;

template <typename T> struct Dft<T, 2> {
    __device__ static inline void run(cplx<T> *v, int) {
        cplx<T> a = v[0], b = v[1];
        v[0] = cadd<T>(a, b);
        v[1] = csub<T>(a, b);
    }
};

template <typename T> struct Dft<T, 4> {
    __device__ static inline void run(cplx<T> *v, int s) {
        cplx<T> t0 = cadd<T>(v[0], v[2]), t1 = csub<T>(v[0], v[2]);
        cplx<T> t2 = cadd<T>(v[1], v[3]), t3 = mul_si<T>(csub<T>(v[1], v[3]), s);
        v[0] = cadd<T>(t0, t2);
        v[2] = csub<T>(t0, t2);
        v[1] = cadd<T>(t1, t3);
        v[3] = csub<T>(t1, t3);
    }
};

template <typename T> struct Dft<T, 8> {
    __device__ static inline void run(cplx<T> *v, int s) {
        const T h = (T)0.70710678118654752440084436210485;
        cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
        cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
        Dft<T, 4>::run(e, s);
        Dft<T, 4>::run(o, s);
        // w8^k = exp(s * 2 pi i k / 8)
        cplx<T> w1 = cmake<T>(h, s * h), w3 = cmake<T>(-h, s * h);
        cplx<T> o1 = cmul<T>(o[1], w1), o2 = mul_si<T>(o[2], s), o3 = cmul<T>(o[3], w3);
        v[0] = cadd<T>(e[0], o[0]);
        v[4] = csub<T>(e[0], o[0]);
        v[1] = cadd<T>(e[1], o1);
        v[5] = csub<T>(e[1], o1);
        v[2] = cadd<T>(e[2], o2);
        v[6] = csub<T>(e[2], o2);
        v[3] = cadd<T>(e[3], o3);
        v[7] = csub<T>(e[3], o3);
    }
};

template <typename T> struct Dft<T, 3> {
    __device__ static inline void run(cplx<T> *v, int s) {
        const T c = (T)-0.5, sn = (T)0.86602540378443864676372317075294;
        cplx<T> t = cadd<T>(v[1], v[2]);
        cplx<T> d = mul_si<T>(cscale<T>(csub<T>(v[1], v[2]), sn), s);
        cplx<T> m = cadd<T>(v[0], cscale<T>(t, c));
        v[0] = cadd<T>(v[0], t);
        v[1] = cadd<T>(m, d);
        v[2] = csub<T>(m, d);
    }
};

template <typename T> struct Dft<T, 5> {
    __device__ static inline void run(cplx<T> *v, int s) {
        const T c1 = (T)0.30901699437494742410229341718282;    // cos(2 pi/5)
        const T c2 = (T)-0.80901699437494742410229341718282;   // cos(4 pi/5)
        const T s1 = (T)0.95105651629515357211643933337938;    // sin(2 pi/5)
        const T s2 = (T)0.58778525229247312916870595463907;    // sin(4 pi/5)
        cplx<T> t1 = cadd<T>(v[1], v[4]), t2 = cadd<T>(v[2], v[3]);
        cplx<T> t3 = csub<T>(v[1], v[4]), t4 = csub<T>(v[2], v[3]);
        cplx<T> a = cadd<T>(v[0], cadd<T>(cscale<T>(t1, c1), cscale<T>(t2, c2)));
        cplx<T> b = cadd<T>(v[0], cadd<T>(cscale<T>(t1, c2), cscale<T>(t2, c1)));
        cplx<T> p = mul_si<T>(cadd<T>(cscale<T>(t3, s1), cscale<T>(t4, s2)), s);
        cplx<T> q = mul_si<T>(csub<T>(cscale<T>(t3, s2), cscale<T>(t4, s1)), s);
        v[0] = cadd<T>(v[0], cadd<T>(t1, t2));
        v[1] = cadd<T>(a, p);
        v[4] = csub<T>(a, p);
        v[2] = cadd<T>(b, q);
        v[3] = csub<T>(b, q);
    }
};

// ---------------------------------------------------------------------------
// one Stockham stage on LDS data.
// howmany transforms of length n; element e of transform f sits at
// buf[((f + f0) % fmod) * ds + e * es].  Ns = product of earlier radices.
// ---------------------------------------------------------------------------
struct FftGeom {
    int n, howmany, es, ds, f0, fmod;
};

template <typename T, int R, int NIT, int NTHR>
__device__ inline void fft_stage(cplx<T> *buf, const FftGeom &g, int Ns, const cplx<T> *tw, int sign) {
    const int nbf = g.n / R;
    const int total = g.howmany * nbf;
    const int tws = g.n / (Ns * R);
    const int tid = threadIdx.x;
    cplx<T> v[NIT][R];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = tid + it * NTHR;
        if (idx < total) {
            int f, j;
            if (g.es == 1) { f = idx / nbf; j = idx - f * nbf; }
            else { j = idx / g.howmany; f = idx - j * g.howmany; }
            int row = f + g.f0;
            if (row >= g.fmod) row -= g.fmod;
            const cplx<T> *src = buf + row * g.ds;
            const int k = j % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = src[(j + r * nbf) * g.es];
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cplx<T> w = tw[k * r * tws];
                    if (sign > 0) w.y = -w.y;
                    v[it][r] = cmul<T>(v[it][r], w);
                }
            }
            Dft<T, R>::run(v[it], sign);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = tid + it * NTHR;
        if (idx < total) {
            int f, j;
            if (g.es == 1) { f = idx / nbf; j = idx - f * nbf; }
            else { j = idx / g.howmany; f = idx - j * g.howmany; }
            int row = f + g.f0;
            if (row >= g.fmod) row -= g.fmod;
            cplx<T> *dst = buf + row * g.ds;
            const int k = j % Ns;
            const int o = (j / Ns) * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[(o + r * Ns) * g.es] = v[it][r];
        }
    }
    __syncthreads();
}

// registers per thread per stage: MAXV complex values
template <typename T> struct FftRegs { static constexpr int MAXV = 16; };
template <> struct FftRegs<float> { static constexpr int MAXV = 24; };

template <typename T, int NTHR>
__device__ void lds_fft(cplx<T> *buf, const FftPlan &plan, const FftGeom &g, const cplx<T> *tw, int sign) {
    constexpr int MAXV = FftRegs<T>::MAXV;
    int Ns = 1;
    for (int s = 0; s < plan.nstages; ++s) {
        const int R = plan.radix[s];
        switch (R) {
            case 8: fft_stage<T, 8, MAXV / 8, NTHR>(buf, g, Ns, tw, sign); break;
            case 4: fft_stage<T, 4, MAXV / 4, NTHR>(buf, g, Ns, tw, sign); break;
            case 2: fft_stage<T, 2, MAXV / 2, NTHR>(buf, g, Ns, tw, sign); break;
            case 3: fft_stage<T, 3, MAXV / 3, NTHR>(buf, g, Ns, tw, sign); break;
            case 5: fft_stage<T, 5, MAXV / 5, NTHR>(buf, g, Ns, tw, sign); break;
            default: break;
        }
        Ns *= R;
    }
}

// host check that every stage fits the per-thread register budget
template <typename T> static bool fft_fits(const FftPlan &plan, int howmany, int nthr) {
    constexpr int MAXV = FftRegs<T>::MAXV;
    for (int s = 0; s < plan.nstages; ++s) {
        const int R = plan.radix[s];
        const long total = (long)howmany * (plan.n / R);
        const long nit = (total + nthr - 1) / nthr;
        if (nit > MAXV / R) return false;
    }
    return true;
}

// ---------------------------------------------------------------------------
// kernel parameters
// ---------------------------------------------------------------------------
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
    const void *tw0, *tw1;
    const void *vz;           // [n2][n0][n1] potential, z-major (or null)
};

template <typename T> __device__ inline void load_tw(cplx<T> *dst, const cplx<T> *src, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// z pass, inverse: sphere -> column grid
// ---------------------------------------------------------------------------
template <typename T, int NTHR>
__global__ __launch_bounds__(NTHR) void zpass_inv(ZArgs a, const cplx<T> *__restrict__ psi, int64_t ld,
                                                  cplx<T> *__restrict__ cols) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *tw = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *buf = tw + a.n2;
    const int cb = blockIdx.x, b = blockIdx.y;
    const int c0 = cb * a.cb;
    const int c1 = min(c0 + a.cb, a.ncols);
    const int nc = c1 - c0;
    const int rs = a.n2 + 1;
    load_tw<T>(tw, reinterpret_cast<const cplx<T> *>(a.tw), a.n2);
    for (int i = threadIdx.x; i < nc * rs; i += NTHR) buf[i] = cmake<T>(0, 0);
    __syncthreads();
    const int g0 = a.colstart[c0], g1 = a.colstart[c1];
    const cplx<T> *src = psi + (int64_t)b * ld;
    for (int g = g0 + threadIdx.x; g < g1; g += NTHR) buf[a.zmap[g]] = src[g];
    __syncthreads();
    FftGeom geo{a.n2, nc, 1, rs, 0, nc};
    lds_fft<T, NTHR>(buf, a.plan, geo, tw, +1);
    cplx<T> *dst = cols + (int64_t)b * a.n2 * a.ncols + c0;
    for (int e = threadIdx.x; e < nc * a.n2; e += NTHR) {
        const int z = e / nc, ci = e - z * nc;
        dst[(int64_t)z * a.ncols + ci] = buf[ci * rs + z];
    }
}

// ---------------------------------------------------------------------------
// z pass, forward: column grid -> sphere, with (1/N) and the kinetic epilogue
//   out[g] = scale * FFT(cols)[g] + (kin[g] - shift) * psi[g]   (kin may be null)
// ---------------------------------------------------------------------------
template <typename T, int NTHR>
__global__ __launch_bounds__(NTHR) void zpass_fwd(ZArgs a, const cplx<T> *__restrict__ cols,
                                                  const cplx<T> *__restrict__ psi, int64_t ld,
                                                  const double *__restrict__ kin, double shift, double scale,
                                                  cplx<T> *__restrict__ out, int64_t ldo) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *tw = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *buf = tw + a.n2;
    const int cb = blockIdx.x, b = blockIdx.y;
    const int c0 = cb * a.cb;
    const int c1 = min(c0 + a.cb, a.ncols);
    const int nc = c1 - c0;
    const int rs = a.n2 + 1;
    load_tw<T>(tw, reinterpret_cast<const cplx<T> *>(a.tw), a.n2);
    const cplx<T> *src = cols + (int64_t)b * a.n2 * a.ncols + c0;
    for (int e = threadIdx.x; e < nc * a.n2; e += NTHR) {
        const int z = e / nc, ci = e - z * nc;
        buf[ci * rs + z] = src[(int64_t)z * a.ncols + ci];
    }
    __syncthreads();
    FftGeom geo{a.n2, nc, 1, rs, 0, nc};
    lds_fft<T, NTHR>(buf, a.plan, geo, tw, -1);
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

// ---------------------------------------------------------------------------
// xy pass.  MODE 0: columns -> plane -> x V -> columns (in place)
//           MODE 1: columns -> plane -> grid out [b][x][y][z]
//           MODE 2: grid in [b][x][y][z] -> plane -> columns
// ---------------------------------------------------------------------------
template <typename T, int NTHR, int MODE>
__global__ __launch_bounds__(NTHR) void xy_pass(XYArgs a, cplx<T> *__restrict__ cols, cplx<T> *__restrict__ grid) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *tw0 = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *tw1 = tw0 + a.n0;
    cplx<T> *pl = tw1 + a.n1;
    const int z = blockIdx.x, b = blockIdx.y;
    const int rs = a.n1 + 1;
    const int64_t npl = (int64_t)a.n0 * a.n1;
    load_tw<T>(tw0, reinterpret_cast<const cplx<T> *>(a.tw0), a.n0);
    load_tw<T>(tw1, reinterpret_cast<const cplx<T> *>(a.tw1), a.n1);
    cplx<T> *crow = cols + ((int64_t)b * a.n2 + z) * a.ncols;
    if (MODE != 2) {
        for (int i = threadIdx.x; i < a.n0 * rs; i += NTHR) pl[i] = cmake<T>(0, 0);
        __syncthreads();
        for (int c = threadIdx.x; c < a.ncols; c += NTHR) pl[a.colpos[c]] = crow[c];
        __syncthreads();
        // inverse along y on the rows that hold columns, then along x everywhere
        FftGeom gy{a.n1, a.nrows, 1, rs, a.rowlo, a.n0};
        lds_fft<T, NTHR>(pl, a.plan1, gy, tw1, +1);
        FftGeom gx{a.n0, a.n1, rs, 1, 0, a.n1};
        lds_fft<T, NTHR>(pl, a.plan0, gx, tw0, +1);
    } else {
        const cplx<T> *gin = grid + (int64_t)b * npl * a.n2;
        for (int i = threadIdx.x; i < npl; i += NTHR) {
            const int x = i / a.n1, y = i - x * a.n1;
            pl[x * rs + y] = gin[(int64_t)i * a.n2 + z];
        }
        __syncthreads();
    }
    if (MODE == 1) {
        cplx<T> *gout = grid + (int64_t)b * npl * a.n2;
        for (int i = threadIdx.x; i < npl; i += NTHR) {
            const int x = i / a.n1, y = i - x * a.n1;
            gout[(int64_t)i * a.n2 + z] = pl[x * rs + y];
        }
        return;
    }
    if (MODE == 0) {
        const double *vz = reinterpret_cast<const double *>(a.vz);
        const T *vzt = reinterpret_cast<const T *>(a.vz) + (int64_t)z * npl;
        for (int i = threadIdx.x; i < npl; i += NTHR) {
            const int x = i / a.n1, y = i - x * a.n1;
            pl[x * rs + y] = cscale<T>(pl[x * rs + y], vzt[i]);
        }
        (void)vz;
        __syncthreads();
    }
    // forward along x everywhere, then along y on the rows that hold columns
    FftGeom gx{a.n0, a.n1, rs, 1, 0, a.n1};
    lds_fft<T, NTHR>(pl, a.plan0, gx, tw0, -1);
    FftGeom gy{a.n1, a.nrows, 1, rs, a.rowlo, a.n0};
    lds_fft<T, NTHR>(pl, a.plan1, gy, tw1, -1);
    for (int c = threadIdx.x; c < a.ncols; c += NTHR) crow[c] = pl[a.colpos[c]];
}

// ---------------------------------------------------------------------------
// host launchers
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

#define PW_LAUNCH_BY_THREADS(nthr, KERNEL, T, grid, lds, stream, ...)                           \
    do {                                                                                       \
        switch (nthr) {                                                                        \
            case 256: allow_lds(KERNEL<T, 256>, lds); hipLaunchKernelGGL((KERNEL<T, 256>), grid, dim3(256), lds, stream, __VA_ARGS__); break; \
            case 512: allow_lds(KERNEL<T, 512>, lds); hipLaunchKernelGGL((KERNEL<T, 512>), grid, dim3(512), lds, stream, __VA_ARGS__); break; \
            case 1024: allow_lds(KERNEL<T, 1024>, lds); hipLaunchKernelGGL((KERNEL<T, 1024>), grid, dim3(1024), lds, stream, __VA_ARGS__); break; \
            default: PW_CHECK(false, PW_EUNSUPPORTED, "FFT does not fit the register budget"); \
        }                                                                                      \
        PW_LAUNCH_CHECK();                                                                     \
    } while (0)

template <typename T>
void launch_zinv(pw_ctx *ctx, int nb, const void *psi, int64_t ld, void *cols, hipStream_t s) {
    ZArgs a = zargs<T>(ctx, nb);
    const int ncb = (a.ncols + a.cb - 1) / a.cb;
    const int nthr = pick_threads<T>(a.plan, a.cb);
    const size_t lds = sizeof(cplx<T>) * (a.n2 + (size_t)a.cb * (a.n2 + 1));
    PW_LAUNCH_BY_THREADS(nthr, zpass_inv, T, dim3(ncb, nb), lds, s, a,
                         reinterpret_cast<const cplx<T> *>(psi), ld, reinterpret_cast<cplx<T> *>(cols));
}

template <typename T>
void launch_zfwd(pw_ctx *ctx, int nb, const void *cols, const void *psi, int64_t ld, const double *kin,
                 double shift, double scale, void *out, int64_t ldo, hipStream_t s) {
    ZArgs a = zargs<T>(ctx, nb);
    const int ncb = (a.ncols + a.cb - 1) / a.cb;
    const int nthr = pick_threads<T>(a.plan, a.cb);
    const size_t lds = sizeof(cplx<T>) * (a.n2 + (size_t)a.cb * (a.n2 + 1));
    PW_LAUNCH_BY_THREADS(nthr, zpass_fwd, T, dim3(ncb, nb), lds, s, a,
                         reinterpret_cast<const cplx<T> *>(cols), reinterpret_cast<const cplx<T> *>(psi), ld,
                         kin, shift, scale, reinterpret_cast<cplx<T> *>(out), ldo);
}

template <typename T, int MODE>
void launch_xy(pw_ctx *ctx, int nb, void *cols, void *grid, hipStream_t s) {
    XYArgs a = xyargs<T>(ctx);
    int nthr = 0;
    for (int t : {256, 512, 1024})
        if (fft_fits<T>(a.plan1, a.n0, t) && fft_fits<T>(a.plan0, a.n1, t)) { nthr = t; break; }
    const size_t lds = sizeof(cplx<T>) * (a.n0 + a.n1 + (size_t)a.n0 * (a.n1 + 1));
    PW_CHECK(lds <= 160 * 1024, PW_EUNSUPPORTED, "xy plane %dx%d does not fit LDS", a.n0, a.n1);
    cplx<T> *c = reinterpret_cast<cplx<T> *>(cols);
    cplx<T> *g = reinterpret_cast<cplx<T> *>(grid);
    dim3 gr(a.n2, nb);
    switch (nthr) {
        case 256: allow_lds(xy_pass<T, 256, MODE>, lds); hipLaunchKernelGGL((xy_pass<T, 256, MODE>), gr, dim3(256), lds, s, a, c, g); break;
        case 512: allow_lds(xy_pass<T, 512, MODE>, lds); hipLaunchKernelGGL((xy_pass<T, 512, MODE>), gr, dim3(512), lds, s, a, c, g); break;
        case 1024: allow_lds(xy_pass<T, 1024, MODE>, lds); hipLaunchKernelGGL((xy_pass<T, 1024, MODE>), gr, dim3(1024), lds, s, a, c, g); break;
        default: PW_CHECK(false, PW_EUNSUPPORTED, "xy FFT does not fit the register budget");
    }
    PW_LAUNCH_CHECK();
}

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
