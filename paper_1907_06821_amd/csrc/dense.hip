// Small dense FP64 linear algebra on the GPU for the block solver.
//
//   chol_inv_*         : S = L L^H (Cholesky), T = conj(L^{-1}), so that the band-major
//                        block Psi' = T . Psi is orthonormal (Gram/Cholesky step).
//   tridiag_ql_*_kernel + backtransform_kernel: Hermitian eigensolver for the
//                        Rayleigh-Ritz subspace step (Householder tridiagonalisation,
//                        implicit QL); outputs the eigenvalues and the band-major
//                        rotation R with Psi' = R . Psi.
// The factorisations run as one workgroup; they are O(N^3) on N x N matrices and
// off the O(N^2 npw) critical path.
#include "common.h"

#include <algorithm>
#include <cfloat>

namespace pw {

__device__ inline double2 zmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 zmulc(double2 a, double2 b) { return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }   // a conj(b)
__device__ inline double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double2 zfma(double2 a, double2 b, double2 c) {   // a b + c
    return make_double2(c.x + a.x * b.x - a.y * b.y, c.y + a.x * b.y + a.y * b.x);
}

// ---------------------------------------------------------------------------
// Cholesky + triangular inverse.  W: work copy of S (N x N, ld N), overwritten
// with L in its lower triangle.  T (N x N): conj(L^{-1}).  status[0] = 0 ok,
// j + 1 if pivot j is not positive.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void chol_inv_kernel(int N, const double2 *__restrict__ S, int64_t lds,
                                                        double2 *__restrict__ W, double2 *__restrict__ T,
                                                        int *__restrict__ status) {
    __shared__ double piv;
    __shared__ int bad;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < N * N; e += nt) {
        const int i = e / N, k = e % N;
        W[e] = S[(int64_t)i * lds + k];
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < N; ++j) {
        if (tid == 0) {
            const double d = W[(int64_t)j * N + j].x;
            if (!(d > 0.0) || !isfinite(d)) { bad = j + 1; piv = 1.0; }
            else piv = sqrt(d);
        }
        __syncthreads();
        if (bad) break;
        const double inv = 1.0 / piv;
        for (int i = j + 1 + tid; i < N; i += nt) {
            double2 v = W[(int64_t)i * N + j];
            W[(int64_t)i * N + j] = make_double2(v.x * inv, v.y * inv);
        }
        if (tid == 0) W[(int64_t)j * N + j] = make_double2(piv, 0.0);
        __syncthreads();
        const int m = N - j - 1;
        for (int e = tid; e < m * m; e += nt) {
            const int i = j + 1 + e / m, k = j + 1 + e % m;
            if (k <= i) {
                const double2 lij = W[(int64_t)i * N + j], lkj = W[(int64_t)k * N + j];
                const double2 u = zmulc(lij, lkj);
                double2 w = W[(int64_t)i * N + k];
                W[(int64_t)i * N + k] = make_double2(w.x - u.x, w.y - u.y);
            }
        }
        __syncthreads();
    }
    if (tid == 0 && bad) status[0] = bad;   // sticky: callers clear it
    if (bad) return;
    // Linv by rows: Linv[i][c] = (delta_ic - sum_{c<=k<i} L[i][k] Linv[k][c]) / L[i][i]; stored conj in T
    for (int e = tid; e < N * N; e += nt) T[e] = make_double2(0.0, 0.0);
    __syncthreads();
    for (int i = 0; i < N; ++i) {
        const double dinv = 1.0 / W[(int64_t)i * N + i].x;
        for (int c = tid; c <= i; c += nt) {
            double re = (c == i) ? 1.0 : 0.0, im = 0.0;
            for (int k = c; k < i; ++k) {
                const double2 l = W[(int64_t)i * N + k];
                const double2 x = zconj(T[(int64_t)k * N + c]);   // Linv[k][c]
                re -= l.x * x.x - l.y * x.y;
                im -= l.x * x.y + l.y * x.x;
            }
            T[(int64_t)i * N + c] = make_double2(re * dinv, -im * dinv);   // conj(Linv[i][c])
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Same result for N <= 128 with the packed lower triangle held in LDS
// (N (N + 1) / 2 complex values, 132 KiB at N = 128): Cholesky by columns, then
// L^{-1} in place from the last column backwards.
// ---------------------------------------------------------------------------
__device__ inline int tri(int i, int k) { return i * (i + 1) / 2 + k; }

// largest matrix whose packed triangle (N (N + 1) / 2 complex128) fits in LDS
constexpr int kLdsMaxN = 136;

// (row, column) of entry q of a packed lower triangle
__device__ inline void tri_rc(int q, int &i, int &k) {
    int r = (int)((sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
    while (r * (r + 1) / 2 > q) --r;
    while ((r + 1) * (r + 2) / 2 <= q) ++r;
    i = r;
    k = q - r * (r + 1) / 2;
}

template <int NT>
__global__ __launch_bounds__(NT) void chol_inv_lds_kernel(int N, const double2 *__restrict__ S, int64_t lds,
                                                          double2 *__restrict__ T, int *__restrict__ status) {
    extern __shared__ unsigned char smem_raw[];
    double2 *L = reinterpret_cast<double2 *>(smem_raw);
    __shared__ double piv;
    __shared__ int bad;
    const int tid = threadIdx.x;
    for (int q = tid; q < N * (N + 1) / 2; q += NT) {   // every load in flight at once
        int i, k;
        tri_rc(q, i, k);
        L[q] = S[(int64_t)i * lds + k];
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < N; ++j) {
        if (tid == 0) {
            const double d = L[tri(j, j)].x;
            if (!(d > 0.0) || !isfinite(d)) { bad = j + 1; piv = 1.0; }
            else { piv = sqrt(d); L[tri(j, j)] = make_double2(piv, 0.0); }
        }
        __syncthreads();
        if (bad) break;
        const double inv = 1.0 / piv;
        for (int i = j + 1 + tid; i < N; i += NT) {
            const double2 v = L[tri(i, j)];
            L[tri(i, j)] = make_double2(v.x * inv, v.y * inv);
        }
        __syncthreads();
        // trailing update L[i][k] -= L[i][j] conj(L[k][j]): a row per group of G
        // threads, the group's lanes striding over the row's columns
        {
            constexpr int G = NT / 128;
            const int sub = tid % G;
            for (int i = j + 1 + tid / G; i < N; i += NT / G) {
                const double2 lij = L[tri(i, j)];
                const int base = tri(i, 0);
                for (int k = j + 1 + sub; k <= i; k += G) {
                    const double2 lkj = L[tri(k, j)];
                    const double2 u = zmulc(lij, lkj);
                    const double2 w = L[base + k];
                    L[base + k] = make_double2(w.x - u.x, w.y - u.y);
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0 && bad) status[0] = bad;
    if (bad) return;
    // in-place inverse: column j of L^{-1} from columns > j (already inverted);
    // each row's dot product is split over a group of G lanes and summed by shuffles
    for (int j = N - 1; j >= 0; --j) {
        constexpr int G = NT / 128;
        const double djj = 1.0 / L[tri(j, j)].x;
        const int sub = tid % G;
        double rr[2], ri[2];
        // rows j+1+tid/G and j+1+tid/G+128 (N <= 256)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            double ar = 0.0, ai = 0.0;
            const int i = j + 1 + tid / G + h * (NT / G);
            if (i < N) {
                for (int k = j + 1 + sub; k <= i; k += G) {
                    const double2 a = L[tri(i, k)], b = L[tri(k, j)];   // Linv[i][k], L[k][j]
                    ar += a.x * b.x - a.y * b.y;
                    ai += a.x * b.y + a.y * b.x;
                }
            }
#pragma unroll
            for (int o = G / 2; o > 0; o >>= 1) {
                ar += __shfl_xor(ar, o, G);
                ai += __shfl_xor(ai, o, G);
            }
            rr[h] = ar;
            ri[h] = ai;
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = j + 1 + tid / G + h * (NT / G);
            if (i < N && sub == 0) L[tri(i, j)] = make_double2(-rr[h] * djj, -ri[h] * djj);
        }
        if (tid == 0) L[tri(j, j)] = make_double2(djj, 0.0);
        __syncthreads();
    }
    for (int e = tid; e < N * N; e += NT) {
        const int i = e / N, c = e % N;
        const double2 v = c <= i ? L[tri(i, c)] : make_double2(0.0, 0.0);
        T[e] = make_double2(v.x, -v.y);
    }
}

// ---------------------------------------------------------------------------
// Hermitian eigensolver: A = Q T Q^H, T = Z diag(d) Z^T, eigenvectors Q Z.
//
// 1. Householder reduction to a real symmetric tridiagonal T,
//    Q = H_0 H_1 ... H_{N-2}.  H_k = I - tau_k v_k v_k^H acts on rows k+1..N-1
//    with v_k[k+1] = 1 and H_k^H sending column k below the diagonal to
//    beta_k e_1, beta_k real (complex reflectors in the convention of LAPACK's
//    zlarfg).  The two-sided update A22 <- H^H A22 H is the rank-2 form
//    A22 - v w^H - w v^H with w = tau A22 v - (tau/2) ((tau A22 v)^H v) v.
//    v_k (entries k+1..N-1) is stored at hv + k(N-1) - k(k-1)/2, tau_k at
//    hv + N(N-1)/2 + k.
// 2. Implicit QL with Wilkinson's shift on T (the tql2 algorithm of Bowdler,
//    Martin, Reinsch and Wilkinson, 1968).  Wave 0 runs the scalar recurrence
//    of the next sweep while the other waves apply the Givens rotations of the
//    previous one to the rows of Z (double-buffered rotation lists).
// 3. Eigenvalues ordered by key into lam; Z column m is zg[m N + r], its rank
//    rank[m]; info = largest QL iteration count of one eigenvalue, -1 if one
//    needed more than kQlMaxIter.
// The back-transformation (second launch) writes Q Z[:, m] as row rank[m] of R,
// so that R . Psi rotates a band-major block.
//
// tridiag_ql_lds_kernel (N <= kLdsMaxN): A as a packed lower triangle in LDS,
// then Z in the same LDS.  tridiag_ql_global_kernel (N <= kEigMaxN): full A in
// global memory (rows coalesced), Z in global memory over the dead A.
// ---------------------------------------------------------------------------
constexpr int kQlMaxIter = 60;
constexpr int kEigNT = 1024;
constexpr int kEigMaxN = 1024;

__device__ inline double2 lds_get(const double2 *L, int i, int k) {
    return i >= k ? L[tri(i, k)] : zconj(L[tri(k, i)]);
}
__device__ inline double wave_sum(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}
__device__ inline double2 wave_sum2(double2 x) { return make_double2(wave_sum(x.x), wave_sum(x.y)); }
__host__ __device__ inline int refl_off(int k, int N) { return k * (N - 1) - k * (k - 1) / 2; }

// Reflector for x = (alpha, x2) with s2 = |x2|^2: tau, beta, 1/(alpha - beta).
__device__ inline void householder(double2 al, double s2, double2 &tau, double &beta, double2 &scl) {
    tau = make_double2(0.0, 0.0);
    scl = make_double2(0.0, 0.0);
    beta = al.x;
    if (s2 > 0.0 || al.y != 0.0) {
        const double nrm = sqrt(al.x * al.x + al.y * al.y + s2);
        beta = al.x >= 0.0 ? -nrm : nrm;
        tau = make_double2((beta - al.x) / beta, -al.y / beta);
        const double2 den = make_double2(al.x - beta, al.y);
        const double dd = den.x * den.x + den.y * den.y;
        scl = make_double2(den.x / dd, -den.y / dd);
    }
}

// r = sqrt(f^2 + g^2) and 1/r: hardware reciprocal square root refined by two
// Goldschmidt steps and a final Newton correction of r; library hypot outside
// the range where f^2 + g^2 neither overflows nor underflows.  Returns 0 if
// r == 0.  Every lane of the wave holds the same f and g, so the rare cases are
// taken as scalar branches.
__device__ __forceinline__ int givens_norm(double f, double g, double &r, double &rinv) {
    const double x = f * f + g * g;
    if (__builtin_amdgcn_readfirstlane((int)!(x >= 1e-290 && x <= 1e290))) {
        r = hypot(f, g);
        rinv = 1.0 / r;
        return __builtin_amdgcn_readfirstlane((int)(r != 0.0));
    }
    const double y = __builtin_amdgcn_rsq(x);
    double h = 0.5 * y, q = x * y;
    double t = fma(-q, h, 0.5);
    q = fma(q, t, q);
    h = fma(h, t, h);
    t = fma(-q, h, 0.5);
    q = fma(q, t, q);
    h = fma(h, t, h);
    r = fma(fma(-q, q, x), h, q);
    rinv = 2.0 * h;
    return 1;
}

// One implicit QL sweep of the tridiagonal (d, e), run uniformly by all 64 lanes
// of a wave.  (l, iter, maxiter, fail) carry over between calls.  Records the
// rotations (c_t, s_t) acting on columns (msweep-1-t, msweep-t) and returns
// msweep, or -1 once every eigenvalue has converged.
__device__ __forceinline__ int ql_sweep(int N, double *d, double *e, double *cs, double *sn, int &l, int &iter,
                                        int &maxiter, bool &fail, int lane, int &nrot) {
    nrot = 0;
    while (l < N) {
        int m = N - 1;
        for (int base = l; base < N - 1; base += 64) {
            const int idx = base + lane;
            bool small = false;
            if (idx < N - 1) small = fabs(e[idx]) <= DBL_EPSILON * (fabs(d[idx]) + fabs(d[idx + 1]));
            const unsigned long long bal = __ballot(small);
            if (bal) {
                m = base + __ffsll((long long)bal) - 1;
                break;
            }
        }
        if (m == l) {
            maxiter = max(maxiter, iter);
            ++l;
            iter = 0;
            continue;
        }
        if (iter == kQlMaxIter) {
            fail = true;
            ++l;
            iter = 0;
            continue;
        }
        ++iter;
        const double dl = d[l], el = e[l];
        double g = (d[l + 1] - dl) / (2.0 * el);
        double r = hypot(g, 1.0);
        g = d[m] - dl + el / (g + copysign(r, g));
        double s = 1.0, c = 1.0, p = 0.0;
        double dip1 = d[m];                     // d[i+1] as it was before this sweep
        double ei = e[m - 1], di = d[m - 1];
        bool split = false;
        for (int i = m - 1; i >= l; --i) {
            // next step's operands, loaded ahead (index clamped on the last step)
            const int ip = i > l ? i - 1 : i;
            const double en = e[ip], dn = d[ip];
            const double f = s * ei, b = c * ei;
            double rinv;
            if (!givens_norm(f, g, r, rinv)) {  // T splits: the next search restarts on the shorter block
                if (lane == 0) {
                    d[i + 1] = dip1 - p;
                    e[i + 1] = 0.0;
                    e[m] = 0.0;
                }
                split = true;
                break;
            }
            s = f * rinv;
            c = g * rinv;
            g = dip1 - p;
            const double rr = (di - g) * s + 2.0 * c * b;
            p = s * rr;
            if (lane == 0) {
                e[i + 1] = r;
                d[i + 1] = g + p;
                cs[nrot] = c;
                sn[nrot] = s;
            }
            r = rr;
            g = c * rr - b;
            ++nrot;
            dip1 = di;
            ei = en;
            di = dn;
        }
        if (!split && lane == 0) {
            d[l] = dip1 - p;
            e[l] = g;
            e[m] = 0.0;
        }
        __builtin_amdgcn_wave_barrier();   // lane 0's stores stay ahead of the next sweep's loads
        return m;
    }
    return -1;
}

// Rotation list of one sweep applied to row `row` of Z (Zt[i N + row] = Z[row][i]).
__device__ __forceinline__ void ql_apply(double *Zt, int N, int row, int msweep, int nrot, const double *cs,
                                         const double *sn) {
    double carry = Zt[(int64_t)msweep * N + row];       // column i+1 of the current rotation
#pragma unroll 4
    for (int t = 0; t < nrot; ++t) {
        const int i = msweep - 1 - t;
        const double zi = Zt[(int64_t)i * N + row];
        Zt[(int64_t)(i + 1) * N + row] = sn[t] * zi + cs[t] * carry;
        carry = cs[t] * zi - sn[t] * carry;
    }
    Zt[(int64_t)(msweep - nrot) * N + row] = carry;
}

// QL on (d, e) with Z (identity on entry) by the whole block, then eigenvalue
// order.  NMAX sizes the rotation lists.
template <int NT, int NMAX>
__device__ __forceinline__ void ql_block(int N, double *d, double *e, double (*cs)[NMAX], double (*sn)[NMAX],
                                         int (*ctl)[2], double *Zt, double *lam, int *rank, int key, double ref,
                                         int *info) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) {
        ctl[1][0] = -2;                                 // nothing to apply yet
        ctl[1][1] = 0;
    }
    __syncthreads();
    int l = 0, iter = 0, maxiter = 0;
    bool fail = false;
    for (int b = 0;; b ^= 1) {
        if (wid == 0) {
            int nrot;
            const int ms = ql_sweep(N, d, e, cs[b], sn[b], l, iter, maxiter, fail, lane, nrot);
            if (lane == 0) {
                ctl[b][0] = ms;
                ctl[b][1] = nrot;
            }
        } else {
            const int pm = ctl[b ^ 1][0], pn = ctl[b ^ 1][1];
            if (pm >= 0 && pn > 0)
                for (int row = tid - 64; row < N; row += NT - 64) ql_apply(Zt, N, row, pm, pn, cs[b ^ 1], sn[b ^ 1]);
        }
        __syncthreads();
        if (ctl[b][0] < 0) break;
    }
    for (int i = tid; i < N; i += NT) {
        const double li = d[i];
        const double ki = key ? fabs(li - ref) : li;
        int rk = 0;
        for (int j = 0; j < N; ++j) {
            const double lj = d[j];
            const double kj = key ? fabs(lj - ref) : lj;
            if (kj < ki || (kj == ki && (lj < li || (lj == li && j < i)))) ++rk;
        }
        lam[rk] = li;
        rank[i] = rk;
    }
    if (tid == 0 && info) info[0] = fail ? -1 : maxiter;
}

template <int NT>
__global__ __launch_bounds__(NT) void tridiag_ql_lds_kernel(int N, const double2 *__restrict__ Ain, int64_t lda,
                                                            double2 *__restrict__ hv, double *__restrict__ zg,
                                                            int *__restrict__ rank, double *__restrict__ lam, int key,
                                                            double ref, int *__restrict__ info) {
    extern __shared__ unsigned char smem_raw[];
    double2 *L = reinterpret_cast<double2 *>(smem_raw);     // packed lower triangle of A
    double *Zt = reinterpret_cast<double *>(smem_raw);      // afterwards: Zt[i N + r] = Z[r][i]
    __shared__ double2 v[kLdsMaxN], w[kLdsMaxN];
    __shared__ double d[kLdsMaxN], e[kLdsMaxN], cs[2][kLdsMaxN], sn[2][kLdsMaxN];
    __shared__ double2 sc[3][2];                            // tau, 1/(alpha - beta), w correction; by parity of k
    __shared__ int ctl[2][2];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int ntri = N * (N + 1) / 2;
    const int tau_off = N * (N - 1) / 2;
    for (int q = tid; q < ntri; q += NT) {
        int i, k;
        tri_rc(q, i, k);
        const double2 a = Ain[(int64_t)i * lda + k], b = Ain[(int64_t)k * lda + i];
        L[q] = make_double2(0.5 * (a.x + b.x), i == k ? 0.0 : 0.5 * (a.y - b.y));
    }
    __syncthreads();
    for (int k = 0; k + 1 < N; ++k) {
        const int par = k & 1, m = N - 1 - k;
        if (wid == 0) {
            double s2 = 0.0;
            for (int i = k + 2 + lane; i < N; i += 64) {
                const double2 a = L[tri(i, k)];
                s2 += a.x * a.x + a.y * a.y;
            }
            s2 = wave_sum(s2);
            if (lane == 0) {
                double2 tau, scl;
                double beta;
                householder(L[tri(k + 1, k)], s2, tau, beta, scl);
                d[k] = L[tri(k, k)].x;
                e[k] = beta;
                sc[0][par] = tau;
                sc[1][par] = scl;
                hv[tau_off + k] = tau;
            }
        }
        __syncthreads();
        const double2 tau = sc[0][par], scl = sc[1][par];
        if (tau.x == 0.0 && tau.y == 0.0) continue;        // H_k = I: nothing to update
        const int off = refl_off(k, N);
        for (int i = k + 1 + tid; i < N; i += NT) {
            const double2 x = i == k + 1 ? make_double2(1.0, 0.0) : zmul(L[tri(i, k)], scl);
            v[i] = x;
            hv[off + (i - k - 1)] = x;
        }
        __syncthreads();
        {   // w = tau A22 v, eight lanes per row
            const int g = tid >> 3, s = tid & 7;
            for (int r = g; r < m; r += NT / 8) {
                const int i = k + 1 + r;
                double2 acc = make_double2(0.0, 0.0);
                for (int j = k + 1 + s; j < N; j += 8) acc = zfma(lds_get(L, i, j), v[j], acc);
                for (int o = 4; o > 0; o >>= 1) {
                    acc.x += __shfl_xor(acc.x, o);
                    acc.y += __shfl_xor(acc.y, o);
                }
                if (s == 0) w[i] = zmul(tau, acc);
            }
        }
        __syncthreads();
        if (wid == 0) {
            double2 t = make_double2(0.0, 0.0);             // w^H v
            for (int i = k + 1 + lane; i < N; i += 64) t = zfma(zconj(w[i]), v[i], t);
            t = wave_sum2(t);
            if (lane == 0) {
                const double2 h = zmul(tau, t);
                sc[2][par] = make_double2(-0.5 * h.x, -0.5 * h.y);
            }
        }
        __syncthreads();
        const double2 a2 = sc[2][par];
        for (int q = tid; q < m * (m + 1) / 2; q += NT) {
            int ii, jj;
            tri_rc(q, ii, jj);
            const int i = k + 1 + ii, j = k + 1 + jj;
            const double2 vi = v[i], vj = v[j];
            const double2 wi = zfma(a2, vi, w[i]), wj = zfma(a2, vj, w[j]);
            const double2 t1 = zmulc(vi, wj), t2 = zmulc(wi, vj);
            double2 a = L[tri(i, j)];
            a.x -= t1.x + t2.x;
            a.y = i == j ? 0.0 : a.y - (t1.y + t2.y);
            L[tri(i, j)] = a;
        }
        __syncthreads();
    }
    if (tid == 0) {
        d[N - 1] = L[tri(N - 1, N - 1)].x;
        e[N - 1] = 0.0;
    }
    __syncthreads();
    for (int q = tid; q < N * N; q += NT) Zt[q] = (q / N == q % N) ? 1.0 : 0.0;
    ql_block<NT, kLdsMaxN>(N, d, e, cs, sn, ctl, Zt, lam, rank, key, ref, info);
    for (int q = tid; q < N * N; q += NT) zg[q] = Zt[q];
}

// Same algorithm for N <= kEigMaxN.  Ag: N x N work copy of A (full Hermitian,
// rows coalesced); Z overwrites it once the reduction is done (zg == Ag).
template <int NT>
__global__ __launch_bounds__(NT) void tridiag_ql_global_kernel(int N, const double2 *__restrict__ Ain, int64_t lda,
                                                               double2 *__restrict__ Ag, double2 *__restrict__ hv,
                                                               int *__restrict__ rank, double *__restrict__ lam,
                                                               int key, double ref, int *__restrict__ info) {
    __shared__ double2 v[kEigMaxN], w[kEigMaxN];
    __shared__ double d[kEigMaxN], e[kEigMaxN], cs[2][kEigMaxN], sn[2][kEigMaxN];
    __shared__ double2 sc[3][2];
    __shared__ int ctl[2][2];
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int tau_off = N * (N - 1) / 2;
    for (int i = wid; i < N; i += NW)
        for (int j = lane; j < N; j += 64) {
            const double2 a = Ain[(int64_t)i * lda + j], b = Ain[(int64_t)j * lda + i];
            Ag[(int64_t)i * N + j] = make_double2(0.5 * (a.x + b.x), i == j ? 0.0 : 0.5 * (a.y - b.y));
        }
    __syncthreads();
    for (int k = 0; k + 1 < N; ++k) {
        const int par = k & 1, m = N - 1 - k;
        const double2 *rowk = Ag + (int64_t)k * N;          // A[k][i] = conj(A[i][k])
        if (wid == 0) {
            double s2 = 0.0;
            for (int i = k + 2 + lane; i < N; i += 64) {
                const double2 a = rowk[i];
                s2 += a.x * a.x + a.y * a.y;
            }
            s2 = wave_sum(s2);
            if (lane == 0) {
                double2 tau, scl;
                double beta;
                householder(zconj(rowk[k + 1]), s2, tau, beta, scl);
                d[k] = rowk[k].x;
                e[k] = beta;
                sc[0][par] = tau;
                sc[1][par] = scl;
                hv[tau_off + k] = tau;
            }
        }
        __syncthreads();
        const double2 tau = sc[0][par], scl = sc[1][par];
        if (tau.x == 0.0 && tau.y == 0.0) continue;
        const int off = refl_off(k, N);
        for (int i = k + 1 + tid; i < N; i += NT) {
            const double2 x = i == k + 1 ? make_double2(1.0, 0.0) : zmul(zconj(rowk[i]), scl);
            v[i] = x;
            hv[off + (i - k - 1)] = x;
        }
        __syncthreads();
        for (int r = wid; r < m; r += NW) {                 // w = tau A22 v, one wave per row
            const int i = k + 1 + r;
            const double2 *row = Ag + (int64_t)i * N;
            double2 acc = make_double2(0.0, 0.0);
            for (int j = k + 1 + lane; j < N; j += 64) acc = zfma(row[j], v[j], acc);
            acc = wave_sum2(acc);
            if (lane == 0) w[i] = zmul(tau, acc);
        }
        __syncthreads();
        if (wid == 0) {
            double2 t = make_double2(0.0, 0.0);
            for (int i = k + 1 + lane; i < N; i += 64) t = zfma(zconj(w[i]), v[i], t);
            t = wave_sum2(t);
            if (lane == 0) {
                const double2 h = zmul(tau, t);
                sc[2][par] = make_double2(-0.5 * h.x, -0.5 * h.y);
            }
        }
        __syncthreads();
        const double2 a2 = sc[2][par];
        for (int r = wid; r < m; r += NW) {
            const int i = k + 1 + r;
            double2 *row = Ag + (int64_t)i * N;
            const double2 vi = v[i], wi = zfma(a2, vi, w[i]);
            for (int j = k + 1 + lane; j < N; j += 64) {
                const double2 vj = v[j], wj = zfma(a2, vj, w[j]);
                const double2 t1 = zmulc(vi, wj), t2 = zmulc(wi, vj);
                double2 a = row[j];
                a.x -= t1.x + t2.x;
                a.y = i == j ? 0.0 : a.y - (t1.y + t2.y);
                row[j] = a;
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        d[N - 1] = Ag[(int64_t)(N - 1) * N + (N - 1)].x;
        e[N - 1] = 0.0;
    }
    __syncthreads();
    double *Zt = reinterpret_cast<double *>(Ag);
    for (int q = tid; q < N * N; q += NT) Zt[q] = (q / N == q % N) ? 1.0 : 0.0;
    __syncthreads();
    ql_block<NT, kEigMaxN>(N, d, e, cs, sn, ctl, Zt, lam, rank, key, ref, info);
}

// Back-transformation, one wave per eigenvector, NW waves per workgroup.
// LDS_V: all reflectors staged in LDS (N <= kLdsMaxN); otherwise read from
// global memory one reflector ahead.
template <int NW, int NMAX, bool LDS_V>
__global__ __launch_bounds__(64 * NW) void backtransform_kernel(int N, const double2 *__restrict__ hv,
                                                                const double *__restrict__ zg,
                                                                const int *__restrict__ rank,
                                                                double2 *__restrict__ R) {
    extern __shared__ unsigned char smem_raw[];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int tau_off = N * (N - 1) / 2;
    const double2 *sv = hv;
    if constexpr (LDS_V) {
        double2 *s = reinterpret_cast<double2 *>(smem_raw);
        for (int q = tid; q < tau_off + N - 1; q += 64 * NW) s[q] = hv[q];
        __syncthreads();
        sv = s;
    }
    constexpr int Q = (NMAX + 63) / 64;
    const int m = blockIdx.x * NW + wid;
    if (m >= N) return;
    double2 y[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int r = lane + 64 * q;
        y[q] = make_double2(r < N ? zg[(int64_t)m * N + r] : 0.0, 0.0);
    }
    for (int k = N - 2; k >= 0; --k) {
        const double2 tk = sv[tau_off + k];
        if (tk.x == 0.0 && tk.y == 0.0) continue;
        const int off = refl_off(k, N) - (k + 1);           // v_k[r] = sv[off + r], r > k
        double2 vk[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int r = lane + 64 * q;
            vk[q] = (r > k && r < N) ? sv[off + r] : make_double2(0.0, 0.0);
        }
        double2 s = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < Q; ++q) s = zfma(zconj(vk[q]), y[q], s);
        s = wave_sum2(s);
        const double2 ts = zmul(tk, s);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const double2 u = zmul(ts, vk[q]);
            y[q].x -= u.x;
            y[q].y -= u.y;
        }
    }
    const int64_t row = (int64_t)rank[m] * N;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int r = lane + 64 * q;
        if (r < N) R[row + r] = y[q];
    }
}

// ---------------------------------------------------------------------------
// host wrappers
// ---------------------------------------------------------------------------
namespace {
// raise a kernel's dynamic LDS limit to the bytes it is launched with
void lds_limit(const void *fn, size_t bytes, size_t &have) {
    if (bytes > have) {
        PW_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
        have = bytes;
    }
}
constexpr int kBackNW = 4;
}  // namespace

void chol_inv(int N, const void *S, int64_t lds, void *work, void *T, int *status, hipStream_t st) {
    if (N <= kLdsMaxN) {
        PW_CHECK(N > 0 && N < 4096, PW_EINVAL, "bad Cholesky size");   // inverse keeps one band per thread
        const size_t bytes = (size_t)N * (N + 1) / 2 * sizeof(double2);
        static size_t attr_bytes = 64 * 1024;   // default dynamic LDS limit
        lds_limit(reinterpret_cast<const void *>(chol_inv_lds_kernel<1024>), bytes, attr_bytes);
        hipLaunchKernelGGL(chol_inv_lds_kernel<1024>, dim3(1), dim3(1024), bytes, st, N, (const double2 *)S, lds,
                           (double2 *)T, status);
    } else {
        hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(1024), 0, st, N, (const double2 *)S, lds,
                           (double2 *)work, (double2 *)T, status);
    }
    PW_LAUNCH_CHECK();
}

size_t dense_eigh_work_bytes(int N) { return (size_t)32 * N * N; }

void dense_eigh(int N, const void *A, int64_t lda, void *work, double *lam, void *R, int key, double ref, int *info,
                hipStream_t st) {
    PW_CHECK(N >= 1 && N <= kEigMaxN, PW_EUNSUPPORTED, "dense eigensolver limited to 1 <= N <= 1024");
    // work: reflectors and taus, then Z (N^2 real; for N > kLdsMaxN the N x N
    // complex copy of A that Z overwrites), then the ranks: 24 N^2 + 12 N bytes at most
    const bool lds = N <= kLdsMaxN;
    double2 *hv = (double2 *)work;
    double2 *zbuf = hv + ((size_t)N * (N - 1) / 2 + N);
    int *rank = (int *)((char *)zbuf + (size_t)N * N * (lds ? 8 : 16));
    static size_t attr1 = 64 * 1024, attr2 = 64 * 1024;
    if (lds) {
        const size_t b1 = std::max((size_t)N * (N + 1) / 2 * sizeof(double2), (size_t)N * N * sizeof(double));
        lds_limit(reinterpret_cast<const void *>(tridiag_ql_lds_kernel<kEigNT>), b1, attr1);
        hipLaunchKernelGGL(tridiag_ql_lds_kernel<kEigNT>, dim3(1), dim3(kEigNT), b1, st, N, (const double2 *)A, lda,
                           hv, (double *)zbuf, rank, lam, key, ref, info);
        PW_LAUNCH_CHECK();
        const size_t b2 = std::max<size_t>(1, (size_t)N * (N - 1) / 2 + N - 1) * sizeof(double2);
        lds_limit(reinterpret_cast<const void *>(backtransform_kernel<kBackNW, kLdsMaxN, true>), b2, attr2);
        hipLaunchKernelGGL((backtransform_kernel<kBackNW, kLdsMaxN, true>), dim3((N + kBackNW - 1) / kBackNW),
                           dim3(64 * kBackNW), b2, st, N, (const double2 *)hv, (const double *)zbuf,
                           (const int *)rank, (double2 *)R);
    } else {
        hipLaunchKernelGGL(tridiag_ql_global_kernel<kEigNT>, dim3(1), dim3(kEigNT), 0, st, N, (const double2 *)A,
                           lda, zbuf, hv, rank, lam, key, ref, info);
        PW_LAUNCH_CHECK();
        hipLaunchKernelGGL((backtransform_kernel<kBackNW, kEigMaxN, false>), dim3((N + kBackNW - 1) / kBackNW),
                           dim3(64 * kBackNW), 0, st, N, (const double2 *)hv, (const double *)zbuf, (const int *)rank,
                           (double2 *)R);
    }
    PW_LAUNCH_CHECK();
}

}  // namespace pw
