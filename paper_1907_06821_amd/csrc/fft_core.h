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
#pragma once
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
// Consecutive threads take consecutive transforms at the same butterfly, so the
// 16 lanes that share an LDS cycle touch 16 rows of odd stride ds (distinct banks
// for the usual padded row lengths); with consecutive butterflies of one
// transform per lane instead, a stage's strided writes hit the same banks (five
// conflict cycles per LDS instruction on 512-point columns).
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
            j = idx / g.howmany;
            f = idx - j * g.howmany;
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
            j = idx / g.howmany;
            f = idx - j * g.howmany;
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
template <typename T> inline bool fft_fits(const FftPlan &plan, int howmany, int nthr) {
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
// compile-time lengths: the same factorisation as make_plan, resolved by the
// compiler so that every index division is by a constant.
// ---------------------------------------------------------------------------
struct RadixList {
    int n;
    int r[kMaxStages];
};

constexpr RadixList ct_plan(int n) {
    RadixList p{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
    int m = n, e2 = 0;
    while (m % 2 == 0) { m /= 2; ++e2; }
    int c2 = 0, c3 = 0, c4 = 0, c5 = 0, c8 = e2 / 3;
    const int rem = e2 % 3;
    if (rem == 1 && c8 > 0) { --c8; c4 += 2; }
    else if (rem == 1) c2 += 1;
    else if (rem == 2) c4 += 1;
    while (m % 3 == 0) { m /= 3; ++c3; }
    while (m % 5 == 0) { m /= 5; ++c5; }
    for (int i = 0; i < c8; ++i) p.r[p.n++] = 8;
    for (int i = 0; i < c5; ++i) p.r[p.n++] = 5;
    for (int i = 0; i < c4; ++i) p.r[p.n++] = 4;
    for (int i = 0; i < c3; ++i) p.r[p.n++] = 3;
    for (int i = 0; i < c2; ++i) p.r[p.n++] = 2;
    return p;
}

constexpr int ct_radix(int n, int s) { return s < ct_plan(n).n ? ct_plan(n).r[s] : 0; }

// threads per workgroup so that `howmany` transforms of length n fit the
// per-thread register budget in every stage (0 if none does)
template <typename T> constexpr int ct_threads(int n, int howmany) {
    const RadixList p = ct_plan(n);
    for (int t = 256; t <= 1024; t *= 2) {
        bool ok = true;
        for (int s = 0; s < p.n; ++s) {
            const int R = p.r[s];
            const long total = (long)howmany * (n / R);
            if ((total + t - 1) / t > FftRegs<T>::MAXV / R) ok = false;
        }
        if (ok) return t;
    }
    return 0;
}

// HM > 0: the transform count is the compile-time constant HM
template <typename T, int N, int R, int NS, int NTHR, int HM>
__device__ inline void ct_stage(cplx<T> *buf, const FftGeom &g, const cplx<T> *tw, int sign) {
    constexpr int nbf = N / R;
    constexpr int tws = N / (NS * R);
    constexpr int NIT = FftRegs<T>::MAXV / R;
    const int howmany = HM > 0 ? HM : g.howmany;
    const int total = howmany * nbf;
    const int tid = threadIdx.x;
    cplx<T> v[NIT][R];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = tid + it * NTHR;
        if (idx < total) {
            int f, j;
            j = idx / howmany;
            f = idx - j * howmany;
            int row = f + g.f0;
            if (row >= g.fmod) row -= g.fmod;
            const cplx<T> *src = buf + row * g.ds;
            const int k = j % NS;
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = src[(j + r * nbf) * g.es];
            if (NS > 1) {
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
            j = idx / howmany;
            f = idx - j * howmany;
            int row = f + g.f0;
            if (row >= g.fmod) row -= g.fmod;
            cplx<T> *dst = buf + row * g.ds;
            const int k = j % NS;
            const int o = (j / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[(o + r * NS) * g.es] = v[it][r];
        }
    }
    __syncthreads();
}

template <typename T, int N, int S, int NS, int NTHR, int HM>
__device__ inline void ct_fft(cplx<T> *buf, const FftGeom &g, const cplx<T> *tw, int sign) {
    constexpr int R = ct_radix(N, S);
    if constexpr (R > 0) {
        ct_stage<T, N, R, NS, NTHR, HM>(buf, g, tw, sign);
        ct_fft<T, N, S + 1, NS * R, NTHR, HM>(buf, g, tw, sign);
    }
}

// Length policies for the kernels: RtLen reads the plan at run time, CtLen<N>
// has the length and radices built in.
struct RtLen {
    static constexpr int N = 0;
    template <typename T, int NTHR, int HM>
    __device__ static inline void fft(cplx<T> *buf, const FftPlan &plan, const FftGeom &g, const cplx<T> *tw,
                                      int sign) {
        lds_fft<T, NTHR>(buf, plan, g, tw, sign);
    }
};

template <int LEN> struct CtLen {
    static constexpr int N = LEN;
    template <typename T, int NTHR, int HM>
    __device__ static inline void fft(cplx<T> *buf, const FftPlan &, const FftGeom &g, const cplx<T> *tw, int sign) {
        ct_fft<T, LEN, 0, 1, NTHR, HM>(buf, g, tw, sign);
    }
};

}  // namespace pw
