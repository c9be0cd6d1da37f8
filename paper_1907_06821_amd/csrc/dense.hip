// Small dense FP64 linear algebra on the GPU for the block solver.
//
//   chol_inv_*         : S = L L^H (Cholesky), T = conj(L^{-1}), so that the band-major
//                        block Psi' = T . Psi is orthonormal (Gram/Cholesky step).
//   tridiag_ql_*_kernel + backtransform_kernel: Hermitian eigensolver for the
//                        Rayleigh-Ritz subspace step (Householder tridiagonalisation,
//                        divide and conquer with implicit QL on the leaves); outputs
//                        the eigenvalues and the band-major rotation R with
//                        Psi' = R . Psi.
// The factorisations run as one workgroup; they are O(N^3) on N x N matrices and
// off the O(N^2 npw) critical path.
#include "kernels.h"

#include <algorithm>
#include <cfloat>
#include <mutex>

namespace pw {

__device__ inline double2 zmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 zmulc(double2 a, double2 b) { return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }   // a conj(b)
__device__ inline double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double2 zfma(double2 a, double2 b, double2 c) {   // a b + c
    return make_double2(c.x + a.x * b.x - a.y * b.y, c.y + a.x * b.y + a.y * b.x);
}

// ---------------------------------------------------------------------------
// Cholesky + triangular inverse: S = L L^H, T = conj(L^{-1}) (N x N, zero above
// the diagonal); status[0] = j + 1 for the first pivot j that is not positive
// (callers clear it).  N <= kLdsMaxN: one workgroup (chol_inv_lds_kernel);
// larger N: blocked, below.
// ---------------------------------------------------------------------------
__device__ inline int tri(int i, int k) { return i * (i + 1) / 2 + k; }

// v_mfma_f64_16x16x4f64 (wave64): lane l holds A[l % 16][k = l / 16] and
// B[k = l / 16][l % 16]; item v of D at lane l is D[l / 16 + 4 v][l % 16]
typedef double v4d __attribute__((ext_vector_type(4)));
__device__ inline v4d mfma_f64(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

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

// N <= kLdsMaxN.  The packed lower triangle lives in LDS.  Factorisation: right-
// looking without square roots during the sweep, by panels of 16 columns: step j
// subtracts L_ij conj(L_kj) / L_jj (rows i > j) from the panel's later columns only
// and leaves column j unscaled, one barrier per column (column j is read, never
// written, in step j); after the panel, the rest of its rank-16 update (columns k
// past the panel) runs on the FP64 matrix cores.  Then every column k is divided by
// sqrt(L_kk), which turns the diagonal into sqrt(L_kk) as well.  Inverse in place:
// the diagonal blocks of 16 first, all at once, then the block rows below on the
// matrix cores (see the inverse below).
template <int NT>
__device__ __forceinline__ void chol_inv_lds_body(int N, const double2 *__restrict__ S, int64_t lds,
                                                  double2 *__restrict__ T, int64_t ldt, int pivot_base,
                                                  int *__restrict__ status) {
    extern __shared__ unsigned char smem_raw[];
    double2 *L = reinterpret_cast<double2 *>(smem_raw);
    __shared__ double sd[kLdsMaxN];
    __shared__ double rdp[16];                           // 1 / d_j of the panel's columns
    const int tid = threadIdx.x;
    for (int q = tid; q < N * (N + 1) / 2; q += NT) {   // every load in flight at once
        int i, k;
        tri_rc(q, i, k);
        L[q] = S[(int64_t)i * lds + k];
    }
    __syncthreads();
    constexpr int G = NT / 128;
    constexpr int PB = 16;                               // panel width
    const int sub = tid % G, lane = tid & 63, wave = tid >> 6, lr = lane & 15, lk = lane >> 4;
    for (int p0 = 0; p0 < N; p0 += PB) {
        const int pe = min(p0 + PB, N);
        // the panel's columns one by one, each step updating only the panel's columns
        for (int j = p0; j < pe; ++j) {
            const double d = L[tri(j, j)].x;             // the same value in every thread
            if (!(d > 0.0) || !isfinite(d)) {
                if (tid == 0 && status[0] == 0) status[0] = pivot_base + j + 1;   // the first failure is kept
                return;
            }
            const double rd = 1.0 / d;
            if (tid == 0) rdp[j - p0] = rd;
            // a row per group of G threads, the group's lanes striding over the row's panel columns
            for (int i = j + 1 + tid / G; i < N; i += NT / G) {
                const double2 lij = L[tri(i, j)];
                const double2 s_ = make_double2(lij.x * rd, lij.y * rd);
                const int base = tri(i, 0), ke = min(i, pe - 1);
                for (int k = j + 1 + sub; k <= ke; k += G) {
                    const double2 u = zmulc(s_, L[tri(k, j)]);
                    const double2 w = L[base + k];
                    L[base + k] = make_double2(w.x - u.x, w.y - u.y);
                }
            }
            __syncthreads();
        }
        // the rest of the rank-PB update, L[i][k] -= sum_j (L[i][j] / d_j) conj(L[k][j]) for
        // i >= k >= pe, on the FP64 matrix cores: one wave per 16 x 16 tile of the lower
        // triangle, four 4-deep steps over the panel's columns
        const int nt = (N - pe + 15) / 16;
        for (int t = wave; t < nt * (nt + 1) / 2; t += NT / 64) {
            int ti = 0;
            while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
            const int tk = t - ti * (ti + 1) / 2;
            const int ia = pe + 16 * ti + lr, kb = pe + 16 * tk + lr;
            v4d c1 = {0.0, 0.0, 0.0, 0.0}, c2 = c1;
#pragma unroll
            for (int k4 = 0; k4 < PB; k4 += 4) {
                const int j = p0 + k4 + lk;
                double2 a = make_double2(0.0, 0.0), b = a;
                if (j < pe) {
                    if (ia < N) {
                        const double2 x = L[tri(ia, j)];
                        a = make_double2(x.x * rdp[j - p0], x.y * rdp[j - p0]);
                    }
                    if (kb < N) {
                        const double2 y = L[tri(kb, j)];
                        b = make_double2(y.x, -y.y);
                    }
                }
                c1 = mfma_f64(a.x, b.x, c1);
                c1 = mfma_f64(-a.y, b.y, c1);
                c2 = mfma_f64(a.x, b.y, c2);
                c2 = mfma_f64(a.y, b.x, c2);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = pe + 16 * ti + lk + 4 * v, k = pe + 16 * tk + lr;
                if (i < N && k <= i) {
                    const double2 w = L[tri(i, k)];
                    L[tri(i, k)] = make_double2(w.x - c1[v], w.y - c2[v]);
                }
            }
        }
        __syncthreads();
    }
    for (int k = tid; k < N; k += NT) sd[k] = 1.0 / sqrt(L[tri(k, k)].x);
    __syncthreads();
    for (int q = tid; q < N * (N + 1) / 2; q += NT) {
        int i, k;
        tri_rc(q, i, k);
        const double f = sd[k];
        L[q] = make_double2(L[q].x * f, L[q].y * f);
    }
    __syncthreads();
    // in-place inverse X = L^{-1} by block rows of BS.  First every diagonal block
    // X_II = inv(L_II) at once, in place (16 threads per block, one per column,
    // forward substitution): no later step reads L_II.  Then for block row I, with the
    // rows above already holding X,
    //   X_Ic = -X_II sum_{k = c}^{r0 - 1} L[r0 + ., k] X[k][c]   for every column c < r0
    // both products on the FP64 matrix cores, one wave per 16-column tile of X_I.: the
    // sums as (L_I. rows, 4-deep k steps) x (X rows, zero above the diagonal), then
    // -X_II times them, whose B operand for k step v is item v of the sums' own
    // accumulator.  The results wait in registers until every read of the block row
    // is done.
    {
        constexpr int BS = 16;
        static_assert(NT / 64 * BS >= kLdsMaxN, "a wave per 16-column tile left of the last block row");
        static_assert(NT / BS * BS >= kLdsMaxN, "16 threads per diagonal block");
        {
            const int r0 = (tid / BS) * BS, c = tid % BS, nr = min(BS, N - r0);
            double2 col[BS];
            if (r0 < N) {                            // column c of inv(L_II), unrolled so that the
#pragma unroll                                       // block's loads issue ahead of the sums
                for (int i = 0; i < BS; ++i) {
                    double2 acc = make_double2(i == c ? 1.0 : 0.0, 0.0);
                    if (i < nr) {
#pragma unroll
                        for (int q = 0; q < i; ++q)
                            if (q >= c) {
                                const double2 u = zmul(L[tri(r0 + i, r0 + q)], col[q]);
                                acc = make_double2(acc.x - u.x, acc.y - u.y);
                            }
                        const double inv = 1.0 / L[tri(r0 + i, r0 + i)].x;
                        acc = make_double2(acc.x * inv, acc.y * inv);
                    }
                    col[i] = i < c ? make_double2(0.0, 0.0) : acc;
                }
            }
            __syncthreads();
            if (r0 < N && c < nr) {
#pragma unroll
                for (int i = 0; i < BS; ++i)
                    if (i >= c && i < nr) L[tri(r0 + i, r0 + c)] = col[i];
            }
            __syncthreads();
        }
        for (int r0 = BS; r0 < N; r0 += BS) {
            const int nr = min(BS, N - r0);
            const int c0 = wave * BS;                // this wave's column tile
            const bool act = c0 < r0;                // the same for the whole wave
            v4d x1 = {0.0, 0.0, 0.0, 0.0}, x2 = x1;
            if (act) {
                v4d s1 = x1, s2 = x1;
                const int ar = r0 + lr, bc = c0 + lr;
                for (int k4 = c0; k4 < r0; k4 += 4) {
                    const int k = k4 + lk;
                    const double2 a = lr < nr ? L[tri(ar, k)] : make_double2(0.0, 0.0);
                    const double2 b = bc <= k ? L[tri(k, bc)] : make_double2(0.0, 0.0);
                    s1 = mfma_f64(a.x, b.x, s1);
                    s1 = mfma_f64(-a.y, b.y, s1);
                    s2 = mfma_f64(a.x, b.y, s2);
                    s2 = mfma_f64(a.y, b.x, s2);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q = 4 * v + lk;        // X_II[lr][q], zero above the diagonal
                    const double2 a = q <= lr && lr < nr ? L[tri(r0 + lr, r0 + q)] : make_double2(0.0, 0.0);
                    x1 = mfma_f64(a.x, s1[v], x1);
                    x1 = mfma_f64(-a.y, s2[v], x1);
                    x2 = mfma_f64(a.x, s2[v], x2);
                    x2 = mfma_f64(a.y, s1[v], x2);
                }
            }
            __syncthreads();
            if (act) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = lk + 4 * v;
                    if (r < nr) L[tri(r0 + r, c0 + lr)] = make_double2(-x1[v], -x2[v]);
                }
            }
            __syncthreads();
        }
    }
    for (int e = tid; e < N * N; e += NT) {
        const int i = e / N, c = e % N;
        const double2 v = c <= i ? L[tri(i, c)] : make_double2(0.0, 0.0);
        T[(int64_t)i * ldt + c] = make_double2(v.x, -v.y);
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void chol_inv_lds_kernel(int N, const double2 *__restrict__ S, int64_t lds,
                                                          double2 *__restrict__ T, int64_t ldt, int pivot_base,
                                                          int *__restrict__ status) {
    chol_inv_lds_body<NT>(N, S, lds, T, ldt, pivot_base, status);
}

// one problem per workgroup (batched folded-CG runs); masked problems return at once
template <int NT>
__global__ __launch_bounds__(NT) void chol_inv_lds_jobs(const DenseJob *__restrict__ jobs,
                                                        const int *__restrict__ mask) {
    if (!mask[blockIdx.x]) return;
    const DenseJob &j = jobs[blockIdx.x];
    chol_inv_lds_body<NT>(j.N, j.A, j.lda, j.T, j.ldt, 0, j.status);
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
// 2. T = Z diag(d) Z^T by divide and conquer (see dc_block below); its leaves
//    use implicit QL with Wilkinson's shift (the tql2 algorithm of Bowdler,
//    Martin, Reinsch and Wilkinson, 1968), one wave per leaf.
// 3. Eigenvalues ordered by key into lam; Z column m is zg[m N + r], its rank
//    rank[m]; info = largest QL iteration count of one eigenvalue, -1 if one
//    needed more than kQlMaxIter.
// The back-transformation (second launch) writes Q Z[:, m] as row rank[m] of R,
// so that R . Psi rotates a band-major block.
//
// tridiag_ql_lds_kernel (N <= kLdsMaxN): A as a packed lower triangle in LDS,
// whose space then holds the divide and conquer's scratch; Z, V and the
// product's temporary in global work memory.  kLdsMaxN < N <= kEigMaxN: the same
// steps as launches over the whole GPU (hh_* and dc_*_kernel below), full A in
// global memory, Z and the rest over the dead A.
// ---------------------------------------------------------------------------
constexpr int kQlMaxIter = 60;
constexpr int kEigNT = 512;
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

// ---------------------------------------------------------------------------
// Divide and conquer on the tridiagonal (Cuppen's rank-one tearing, eigenvectors
// by the Gu-Eisenstat formula).  T is torn at the boundaries of P = 2^k leaves of
// at most kDcLeaf rows: T = diag(T_1', ..., T_P') + sum of rank-one terms
// |beta| w w^T, w = e_{b-1} + sign(beta) e_b, with T_i' = T_i minus |beta| on the
// torn corners.  Each leaf is solved by the QL sweeps above (one wave per leaf,
// concurrently); pairs of solved blocks are then merged level by level:
// diag(D) + rho z z^T with z the last row of the left block's eigenvectors and
// sign(beta) times the first row of the right block's.  A merge sorts D,
// deflates (rho |z_j| below tol, or a Givens rotation folding z_j into a nearly
// equal neighbour), solves the secular equation 1 + rho sum z_j^2/(d_j - x) = 0
// for each remaining root (one thread per root, safeguarded Newton in the
// coordinate tau = x - d_origin of the nearer pole, so that d_j - x keeps full
// relative accuracy), recomputes z from the roots (Gu-Eisenstat) for
// orthogonal eigenvectors, and forms the block's new eigenvectors Z V.
// Z (Zt[i N + r] = Z[r][i]), V and the product's temporary are in global memory.
// ---------------------------------------------------------------------------
constexpr int kDcLeaf = 16;

// LDS scratch of the divide and conquer for n rows (carved from `base`)
struct DcLds {
    double *sD, *sz, *kd, *kz, *tau, *zh, *lamv, *rc, *rs, *beta;
    double *gz, *gv;        // dc_kc(n)-deep chunks of Z_kept and V for the product
    int *perm, *flag, *kept, *org, *ri, *rj, *ctl;
    double *wcs, *wsn;      // per-wave rotation lists of the leaf QL sweeps
    double *dbl;
    int kc;                 // depth of the product's k chunks
};
// depth of the product's k chunks: each chunk holds dc_kc(n) n <= 2048 doubles
__host__ __device__ inline int dc_kc(int n) { return min(16, 2048 / n); }
// chunks: whether the scratch also holds the two product chunks
__host__ __device__ inline size_t dc_lds_bytes(int n, int nwaves, bool chunks) {
    return (size_t)n * (9 * sizeof(double) + 6 * sizeof(int)) + (chunks ? (size_t)2 * dc_kc(n) * n * sizeof(double) : 0) +
           64 * sizeof(double) + 16 * sizeof(int) +
           (size_t)nwaves * 2 * kDcLeaf * sizeof(double) + 16 * sizeof(double) + 64;
}
// gz, gv: the product chunks if they live elsewhere, else null (carved here)
__device__ inline DcLds dc_carve(unsigned char *base, int n, int nwaves, double *gz, double *gv) {
    DcLds t;
    double *p = reinterpret_cast<double *>(base);
    t.sD = p; p += n;
    t.sz = p; p += n;
    t.kd = p; p += n;
    t.kz = p; p += n;
    t.tau = p; p += n;
    t.zh = p; p += n;
    t.lamv = p; p += n;
    t.rc = p; p += n;
    t.rs = p; p += n;
    t.beta = p; p += 64;
    if (gz) {
        t.gz = gz;
        t.gv = gv;
    } else {
        t.gz = p; p += dc_kc(n) * n;
        t.gv = p; p += dc_kc(n) * n;
    }
    t.wcs = p; p += nwaves * kDcLeaf;
    t.wsn = p; p += nwaves * kDcLeaf;
    t.dbl = p; p += 16;
    int *q = reinterpret_cast<int *>(p);
    t.perm = q; q += n;
    t.flag = q; q += n;
    t.kept = q; q += n;
    t.org = q; q += n;
    t.ri = q; q += n;
    t.rj = q; q += n;
    t.ctl = q;
    t.kc = dc_kc(n);
    return t;
}

// Levels of the divide and conquer whose merges are at most kDcWaveSpan leaves wide
// run their merges concurrently, one wave each, with scratch of their own behind
// the workgroup's (LDS kernel only).
constexpr int kDcWaveSpan = 4;
__host__ __device__ inline int dc_leaves(int n) {
    int P = 1;
    while ((n + P - 1) / P > kDcLeaf) P *= 2;
    return P;
}
__host__ __device__ inline size_t dc_round(size_t b) { return (b + 255) / 256 * 256; }
// bytes of one wave's merge scratch at a level of merges `span` leaves wide
__host__ __device__ inline size_t dc_wave_merge_bytes(int N, int span) {
    const int P = dc_leaves(N);
    return dc_round(dc_lds_bytes((span * N + P - 1) / P + 1, 1, true));
}
// all of the waves' scratch (the largest level)
__host__ __device__ inline size_t dc_wave_bytes(int N, int nwaves) {
    const int P = dc_leaves(N);
    size_t m = 0;
    for (int span = 2; span <= kDcWaveSpan && span <= P; span *= 2) {
        const int nm = P / span;
        if (nm < 2) break;
        const size_t b = (size_t)(nm < nwaves ? nm : nwaves) * dc_wave_merge_bytes(N, span);
        m = b > m ? b : m;
    }
    return m;
}

// workgroup-wide or (NT = 64) wave-wide barrier of the merges
template <int NT> __device__ __forceinline__ void dc_sync() {
    if constexpr (NT == 64) {
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
    } else {
        __syncthreads();
    }
}

// 1/x: hardware reciprocal estimate refined by two Newton steps (about 1 ulp)
__device__ inline double rcp64(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// sum over the G consecutive lanes of a group
template <int G> __device__ inline double group_sum(double x) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, G);
    return x;
}

// root i of 1 + rho sum_j z_j^2 / (d_j - x) (d ascending, z_j != 0) by a group of
// G lanes (lane `sub` sums the terms j = sub mod G): the nearer pole's index in
// *org, tau = x - d[*org] returned.  Newton on h(tau) = (d_org - x) g(x), which has
// no pole at the origin, safeguarded by the bracket; the first iterate is h's
// linearisation at tau = 0.
template <int G>
__device__ inline double secular_root(int i, int K, const double *d, const double *z, double rho, int sub, int *org) {
    double lo, hi;
    int o;
    if (i < K - 1) {
        const double mid = 0.5 * (d[i] + d[i + 1]);
        double f = 0.0;
        for (int j = sub; j < K; j += G) f += rho * z[j] * z[j] * rcp64(d[j] - mid);
        f = 1.0 + group_sum<G>(f);
        if (f > 0.0) {
            o = i;
            lo = 0.0;
            hi = mid - d[i];
        } else {
            o = i + 1;
            lo = mid - d[i + 1];
            hi = 0.0;
        }
    } else {
        o = K - 1;
        double zz = 0.0;
        for (int j = sub; j < K; j += G) zz += z[j] * z[j];
        lo = 0.0;
        hi = rho * group_sum<G>(zz);
    }
    const double dorg = d[o], rzo = rho * z[o] * z[o];
    double s0 = 0.0;
    for (int j = sub; j < K; j += G)
        if (j != o) s0 += rho * z[j] * z[j] * rcp64(d[j] - dorg);
    s0 = 1.0 + group_sum<G>(s0);
    double tau = s0 != 0.0 ? rzo / s0 : 0.5 * (lo + hi);
    if (!(tau > lo && tau < hi)) tau = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        double sv = 0.0, sp = 0.0;
        for (int j = sub; j < K; j += G) {
            if (j == o) continue;
            const double inv = rcp64((d[j] - dorg) - tau);
            const double t = rho * z[j] * z[j] * inv;
            sv += t;
            sp += t * inv;
        }
        sv = 1.0 + group_sum<G>(sv);
        sp = group_sum<G>(sp);
        const double h = rzo - tau * sv, hp = -sv - tau * sp;
        const bool below = tau > 0.0 ? h > 0.0 : (tau < 0.0 && h < 0.0);   // g(tau) < 0: root above tau
        if (below) lo = tau;
        else hi = tau;
        double tn = hp != 0.0 ? tau - h / hp : 0.5 * (lo + hi);
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        const bool done = fabs(tn - tau) <= 2.0 * DBL_EPSILON * fabs(tn) ||
                          hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi));
        tau = tn;
        if (done) break;
    }
    *org = o;
    return tau;
}

// merge of the solved blocks [a, b) and [b, c), first part (whole workgroup): order and
// deflation (its rotations applied to Z); the kept poles and weights in t.kd, t.kz, their
// count in t.ctl[0], rho |z|^2 in t.dbl[0]
template <int NT>
__device__ void dc_merge_deflate(int N, int a, int b, int c, double beta, double *d, double *Zt, const DcLds &t) {
    const int tid = threadIdx.x % NT;
    const int n = c - a;
    const double rho = fabs(beta), sg = beta >= 0.0 ? 1.0 : -1.0;
    // z and the ascending order of the block's eigenvalues
    for (int j = tid; j < n; j += NT) {
        const int col = a + j;
        const double zj = col < b ? Zt[(int64_t)col * N + (b - 1)] : sg * Zt[(int64_t)col * N + b];
        const double dj = d[col];
        int rk = 0;
        for (int k = 0; k < n; ++k) {
            const double dk = d[a + k];
            if (dk < dj || (dk == dj && k < j)) ++rk;
        }
        t.sD[rk] = dj;
        t.sz[rk] = zj;
        t.perm[rk] = col;
    }
    dc_sync<NT>();
    // deflation (one thread, in ascending order)
    if (tid == 0) {
        double nz = 0.0, dmax = 0.0;
        for (int j = 0; j < n; ++j) {
            nz += t.sz[j] * t.sz[j];
            dmax = fmax(dmax, fabs(t.sD[j]));
        }
        nz = sqrt(nz);
        const double rhon = rho * nz * nz;
        const double tol = 8.0 * DBL_EPSILON * fmax(dmax, rhon);
        for (int j = 0; j < n; ++j) t.sz[j] /= nz;
        int pj = -1, nrot = 0;
        for (int j = 0; j < n; ++j) {
            t.flag[j] = 0;
            if (rhon * fabs(t.sz[j]) <= tol) {
                t.flag[j] = 1;
                continue;
            }
            if (pj < 0) {
                pj = j;
                continue;
            }
            const double h = hypot(t.sz[pj], t.sz[j]);
            const double cc = t.sz[j] / h, ss = t.sz[pj] / h;
            if (fabs((t.sD[j] - t.sD[pj]) * cc * ss) <= tol) {
                t.ri[nrot] = pj;
                t.rj[nrot] = j;
                t.rc[nrot] = cc;
                t.rs[nrot] = ss;
                ++nrot;
                const double dp = t.sD[pj], dq = t.sD[j];
                t.sD[pj] = dp * cc * cc + dq * ss * ss;
                t.sD[j] = dp * ss * ss + dq * cc * cc;
                t.sz[pj] = 0.0;
                t.sz[j] = h;
                t.flag[pj] = 1;
            }
            pj = j;
        }
        int K = 0;
        for (int j = 0; j < n; ++j)
            if (!t.flag[j]) {
                t.kept[K] = j;
                t.kd[K] = t.sD[j];
                t.kz[K] = t.sz[j];
                ++K;
            }
        t.ctl[0] = K;
        t.ctl[1] = nrot;
        t.dbl[0] = rhon;
    }
    dc_sync<NT>();
    const int nrot = t.ctl[1];
    // the deflation's rotations act on the block's eigenvector columns, row by row
    for (int r = a + tid; r < c; r += NT)
        for (int q = 0; q < nrot; ++q) {
            double *zp = Zt + (int64_t)t.perm[t.ri[q]] * N + r;
            double *zq = Zt + (int64_t)t.perm[t.rj[q]] * N + r;
            const double x = *zp, y = *zq;
            *zp = t.rc[q] * x - t.rs[q] * y;
            *zq = t.rs[q] * x + t.rc[q] * y;
        }
    dc_sync<NT>();
}

// second part: secular roots, the merged eigenvalues in t.lamv and the kept block's
// eigenvectors V (K x K, row i for root i)
template <int NT>
__device__ void dc_merge_roots(int N, int a, int b, int c, double beta, double *d, double *Zt, double *V,
                               const DcLds &t) {
    dc_merge_deflate<NT>(N, a, b, c, beta, d, Zt, t);
    const int tid = threadIdx.x % NT;
    const int n = c - a, K = t.ctl[0];
    const double rhon = t.dbl[0];
    // roots of the secular equation, four lanes each; flag of a kept position = -(root + 1)
    {
        constexpr int G = 4;
        const int sub = tid % G;
        for (int i = tid / G; i < K; i += NT / G) {
            int o;
            const double tv = secular_root<G>(i, K, t.kd, t.kz, rhon, sub, &o);
            if (sub == 0) {
                t.tau[i] = tv;
                t.org[i] = o;
                t.flag[t.kept[i]] = -(i + 1);
            }
        }
    }
    dc_sync<NT>();
    // z recomputed from the roots: zh_j^2 = prod_i (x_i - d_j) / (rho prod_{i != j} (d_i - d_j))
    for (int j = tid; j < K; j += NT) {
        double w = 1.0;
        for (int i = 0; i < K; ++i) {
            const double xi = (t.kd[t.org[i]] - t.kd[j]) + t.tau[i];
            w *= i == j ? xi : xi * rcp64(t.kd[i] - t.kd[j]);
        }
        t.zh[j] = copysign(sqrt(fmax(w, 0.0) / rhon), t.kz[j]);
    }
    // eigenvalues in ascending (sorted) position; deflated ones keep their D
    for (int j = tid; j < n; j += NT) t.lamv[j] = t.sD[j];
    dc_sync<NT>();
    for (int i = tid; i < K; i += NT) t.lamv[t.kept[i]] = t.kd[t.org[i]] + t.tau[i];
    // eigenvectors of diag(D) + rho z z^T on the kept set: V[i][j] = zh_j / (d_j - x_i), normalised
    for (int i = tid; i < K; i += NT) {
        const int o = t.org[i];
        const double ti = t.tau[i], dorg = t.kd[o];
        double nrm = 0.0;
        for (int j = 0; j < K; ++j) {
            const double v = t.zh[j] * rcp64((t.kd[j] - dorg) - ti);
            V[(int64_t)i * K + j] = v;
            nrm += v * v;
        }
        const double inv = 1.0 / sqrt(nrm);
        for (int j = 0; j < K; ++j) V[(int64_t)i * K + j] *= inv;
    }
    dc_sync<NT>();
}

// second part: the block's new eigenvector columns and eigenvalues
template <int NT>
__device__ void dc_merge_update(int N, int a, int c, double *d, double *Zt, const double *V, double *Ztmp,
                                const DcLds &t) {
    const int tid = threadIdx.x % NT;
    const int n = c - a, K = t.ctl[0];
    // new columns in ascending order: deflated ones copied, kept ones (Z_kept V^T):
    // k chunks of Z_kept (rows of the block) and V staged in LDS, each thread
    // accumulating 4 x 4 tiles of the product
    for (int e = tid; e < n * n; e += NT) {
        const int tcol = e / n;
        if (t.flag[tcol] > 0) Ztmp[e] = Zt[(int64_t)t.perm[tcol] * N + a + e % n];
    }
    {
        constexpr int RT = 4;
        const int KC = t.kc;
        double *zc = t.gz, *vc = t.gv;                    // [KC][n], [KC][K]
        const int nr = (n + RT - 1) / RT, nc = (K + RT - 1) / RT;
        for (int k0 = 0; k0 < K; k0 += KC) {
            const int kc = min(KC, K - k0);
            for (int e = tid; e < kc * n; e += NT) {
                const int jj = e / n, r = e % n;
                zc[jj * n + r] = Zt[(int64_t)t.perm[t.kept[k0 + jj]] * N + a + r];
            }
            for (int e = tid; e < K * kc; e += NT) {
                const int i = e / kc, jj = e % kc;
                vc[jj * K + i] = V[(int64_t)i * K + k0 + jj];
            }
            dc_sync<NT>();
            for (int tile = tid; tile < nr * nc; tile += NT) {
                const int r0 = (tile % nr) * RT, c0 = (tile / nr) * RT;
                double acc[RT][RT];
#pragma unroll
                for (int x = 0; x < RT; ++x)
#pragma unroll
                    for (int y = 0; y < RT; ++y) acc[x][y] = 0.0;
                if (k0 > 0) {
#pragma unroll
                    for (int x = 0; x < RT; ++x)
#pragma unroll
                        for (int y = 0; y < RT; ++y)
                            if (r0 + x < n && c0 + y < K) acc[x][y] = Ztmp[(int64_t)t.kept[c0 + y] * n + r0 + x];
                }
                for (int jj = 0; jj < kc; ++jj) {
                    double zr[RT], vr[RT];
#pragma unroll
                    for (int x = 0; x < RT; ++x) zr[x] = r0 + x < n ? zc[jj * n + r0 + x] : 0.0;
#pragma unroll
                    for (int y = 0; y < RT; ++y) vr[y] = c0 + y < K ? vc[jj * K + c0 + y] : 0.0;
#pragma unroll
                    for (int x = 0; x < RT; ++x)
#pragma unroll
                        for (int y = 0; y < RT; ++y) acc[x][y] = fma(zr[x], vr[y], acc[x][y]);
                }
#pragma unroll
                for (int x = 0; x < RT; ++x)
#pragma unroll
                    for (int y = 0; y < RT; ++y)
                        if (r0 + x < n && c0 + y < K) Ztmp[(int64_t)t.kept[c0 + y] * n + r0 + x] = acc[x][y];
            }
            dc_sync<NT>();
        }
    }
    for (int e = tid; e < n * n; e += NT) {
        const int tcol = e / n, r = e % n;
        Zt[(int64_t)(a + tcol) * N + a + r] = Ztmp[e];
    }
    for (int j = tid; j < n; j += NT) d[a + j] = t.lamv[j];
    dc_sync<NT>();
}

template <int NT>
__device__ void dc_merge(int N, int a, int b, int c, double beta, double *d, double *Zt, double *V, double *Ztmp,
                         const DcLds &t) {
    dc_merge_roots<NT>(N, a, b, c, beta, d, Zt, V, t);
    dc_merge_update<NT>(N, a, c, d, Zt, V, Ztmp, t);
}

// Eigen-decomposition of the tridiagonal (d, e) into d (eigenvalues) and Zt
// (global), then eigenvalue order.  e is overwritten.
template <int NT>
__device__ void dc_block(int N, double *d, double *e, double *Zt, double *V, double *Ztmp, unsigned char *scratch,
                         double *gz, double *gv, bool wave_merges, double *lam, int *rank, int key, double ref,
                         int *info) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const DcLds t = dc_carve(scratch, N, NW, gz, gv);
    const int P = dc_leaves(N);
    for (int q = tid; q < N * N; q += NT) Zt[q] = (q / N == q % N) ? 1.0 : 0.0;
    if (tid == 0) {
        for (int i = 1; i < P; ++i) {
            const int bb = (int)((int64_t)i * N / P);
            const double be = e[bb - 1];
            t.beta[i] = be;
            d[bb - 1] -= fabs(be);
            d[bb] -= fabs(be);
            e[bb - 1] = 0.0;
        }
        t.ctl[2] = 0;                                       // largest QL iteration count
        t.ctl[3] = 0;                                       // a leaf failed to converge
    }
    __syncthreads();
    // leaves: implicit QL, one wave per leaf
    for (int leaf = wid; leaf < P; leaf += NW) {
        const int a = (int)((int64_t)leaf * N / P), b = (int)((int64_t)(leaf + 1) * N / P);
        const int n = b - a;
        double *cs = t.wcs + wid * kDcLeaf, *sn = t.wsn + wid * kDcLeaf;
        int l = 0, iter = 0, maxiter = 0;
        bool fail = false;
        for (;;) {
            int nrot;
            const int ms = ql_sweep(n, d + a, e + a, cs, sn, l, iter, maxiter, fail, lane, nrot);
            if (ms < 0) break;
            if (lane < n && nrot > 0) ql_apply(Zt + (int64_t)a * N + a, N, lane, ms, nrot, cs, sn);
            __builtin_amdgcn_wave_barrier();
        }
        if (lane == 0) {
            atomicMax(&t.ctl[2], maxiter);
            if (fail) t.ctl[3] = 1;
        }
    }
    __syncthreads();
    // merges, level by level; narrow levels one wave per merge, each in its own
    // scratch and in the rows [a, c) of V and Ztmp
    for (int span = 2; span <= P; span *= 2) {
        const int nm = P / span;
        if (wave_merges && span <= kDcWaveSpan && nm >= 2) {
            const size_t wb = dc_wave_merge_bytes(N, span);
            const int maxn = (span * N + P - 1) / P + 1;
            unsigned char *mine = scratch + dc_round(dc_lds_bytes(N, NW, gz == nullptr)) + (size_t)wid * wb;
            for (int m = wid; m < nm; m += NW) {
                const int k = m * span;
                const int a = (int)((int64_t)k * N / P), b = (int)((int64_t)(k + span / 2) * N / P);
                const int c = (int)((int64_t)(k + span) * N / P);
                const double be = t.beta[k + span / 2];
                if (be != 0.0) {
                    const DcLds tw = dc_carve(mine, maxn, 1, nullptr, nullptr);
                    dc_merge<64>(N, a, b, c, be, d, Zt, V + (int64_t)a * N, Ztmp + (int64_t)a * N, tw);
                }
            }
            __syncthreads();
            continue;
        }
        for (int k = 0; k < P; k += span) {
            const int a = (int)((int64_t)k * N / P), b = (int)((int64_t)(k + span / 2) * N / P);
            const int c = (int)((int64_t)(k + span) * N / P);
            const double be = t.beta[k + span / 2];
            if (be != 0.0) dc_merge<NT>(N, a, b, c, be, d, Zt, V, Ztmp, t);
        }
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
    if (tid == 0 && info) info[0] = t.ctl[3] ? -1 : t.ctl[2];
}

template <int NT>
__device__ __forceinline__ void tridiag_ql_lds_body(int N, const double2 *__restrict__ Ain, int64_t lda,
                                                    double2 *__restrict__ hv, double *__restrict__ zg,
                                                    int *__restrict__ rank, double *__restrict__ lam, int key,
                                                    double ref, int *__restrict__ info) {
    extern __shared__ unsigned char smem_raw[];
    double2 *L = reinterpret_cast<double2 *>(smem_raw);     // packed lower triangle of A
    __shared__ double2 v[kLdsMaxN], w[kLdsMaxN];
    __shared__ double d[kLdsMaxN], e[kLdsMaxN];
    __shared__ double2 sc[3][2];                            // tau, 1/(alpha - beta), w correction; by parity of k
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
    // the triangle is dead: its LDS becomes the divide and conquer's scratch
    dc_block<NT>(N, d, e, zg, zg + (size_t)N * N, zg + 2 * (size_t)N * N, smem_raw, nullptr, nullptr, true, lam, rank,
                 key, ref, info);
}

template <int NT>
__global__ __launch_bounds__(NT) void tridiag_ql_lds_kernel(int N, const double2 *__restrict__ Ain, int64_t lda,
                                                            double2 *__restrict__ hv, double *__restrict__ zg,
                                                            int *__restrict__ rank, double *__restrict__ lam, int key,
                                                            double ref, int *__restrict__ info) {
    tridiag_ql_lds_body<NT>(N, Ain, lda, hv, zg, rank, lam, key, ref, info);
}

template <int NT>
__global__ __launch_bounds__(NT) void tridiag_ql_lds_jobs(const DenseJob *__restrict__ jobs,
                                                          const int *__restrict__ mask) {
    if (!mask[blockIdx.x]) return;
    const DenseJob &j = jobs[blockIdx.x];
    tridiag_ql_lds_body<NT>(j.N, j.A, j.lda, j.hv, j.zbuf, j.rank, j.lam, 0, 0.0, j.info);
}

// ---------------------------------------------------------------------------
// Householder reduction for kLdsMaxN < N <= kEigMaxN over the whole GPU, two
// launches per step.  Step k's rank-two update A22 -= v w'^H + w' v^H (w' = w -
// (tau/2)(w^H v) v, w = tau A22 v) is applied to row k + 1 by one workgroup, which
// then forms reflector k + 1 from that row (hh_rowstep); a second launch applies it
// to the rows below, one wave per row, and forms w of step k + 1 from each updated
// row in the same pass (hh_fused), so the trailing matrix streams through every CU
// once per step.  The same reflectors as the one-workgroup kernel above, stored in
// the same places (hv); Ag is the N x N work copy of A (full Hermitian, rows
// coalesced), whose storage Z takes once the reduction is done; v, w and the
// step's scalars (two of each, by step parity) live in the part of the work
// region that V takes later, d and e in the divide and conquer's DcGlobal.
// ---------------------------------------------------------------------------
constexpr int kHhWaves = 8;          // rows (waves) per workgroup of the row kernels

struct HhScratch {
    double2 *v, *w, *sc;             // step 0's v, w and scalars (sc[0] tau)
    double *d, *e;                   // the tridiagonal
};
// per step parity: v, w (N each) and the scalars tau, a2 = -(tau/2) w^H v
struct HhBufs {
    double2 *v[2], *w[2], *sc[2];
    double *d, *e;
};

__global__ __launch_bounds__(256) void hh_symmetrize(int N, const double2 *__restrict__ Ain, int64_t lda,
                                                     double2 *__restrict__ Ag) {
    const int i = blockIdx.x;
    for (int j = threadIdx.x; j < N; j += 256) {
        const double2 a = Ain[(int64_t)i * lda + j], b = Ain[(int64_t)j * lda + i];
        Ag[(int64_t)i * N + j] = make_double2(0.5 * (a.x + b.x), i == j ? 0.0 : 0.5 * (a.y - b.y));
    }
}

// w[i] = tau sum_j A[i][j] v[j], rows i > k, one wave per row
__global__ __launch_bounds__(64 * kHhWaves) void hh_matvec(int N, int k, const double2 *__restrict__ Ag,
                                                           HhScratch s) {
    const double2 tau = s.sc[0];
    if (tau.x == 0.0 && tau.y == 0.0) return;
    const int lane = threadIdx.x & 63;
    const int i = k + 1 + blockIdx.x * kHhWaves + (threadIdx.x >> 6);
    if (i >= N) return;
    const double2 *row = Ag + (int64_t)i * N;
    double2 acc = make_double2(0.0, 0.0);
    for (int j = k + 1 + lane; j < N; j += 64) acc = zfma(row[j], s.v[j], acc);
    acc = wave_sum2(acc);
    if (lane == 0) s.w[i] = zmul(tau, acc);
}

// row r = k + 1: step k's update (k >= 0, its tau nonzero; a2 of step k formed here
// and kept in sck[1]), then, if r < N - 1, reflector r from the updated row
// (A[r][i] = conj(A[i][r]); v[r + 1] = 1) into vr, scr[0], hv, d[r] and e[r]
constexpr int kHhRowT = 256;
__global__ __launch_bounds__(kHhRowT) void hh_rowstep(int N, int k, double2 *__restrict__ Ag, double2 *__restrict__ hv,
                                                      const double2 *__restrict__ vk, const double2 *__restrict__ wk,
                                                      double2 *__restrict__ sck, double2 *__restrict__ vr,
                                                      double2 *__restrict__ scr, double *__restrict__ d,
                                                      double *__restrict__ e) {
    __shared__ double2 red[kHhRowT / 64];
    __shared__ double sred[kHhRowT / 64];
    __shared__ double2 bc[4];                 // a2, tau, scale, A[r][r + 1]
    __shared__ double dg;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, r = k + 1;
    const double2 tauk = k >= 0 ? sck[0] : make_double2(0.0, 0.0);
    const bool upd = !(tauk.x == 0.0 && tauk.y == 0.0);
    double2 a2 = make_double2(0.0, 0.0);
    if (upd) {
        double2 t = make_double2(0.0, 0.0);
        for (int i = r + tid; i < N; i += kHhRowT) t = zfma(zconj(wk[i]), vk[i], t);
        t = wave_sum2(t);
        if (lane == 0) red[wid] = t;
        __syncthreads();
        if (tid == 0) {
            double2 tt = make_double2(0.0, 0.0);
            for (int q = 0; q < kHhRowT / 64; ++q) tt = make_double2(tt.x + red[q].x, tt.y + red[q].y);
            const double2 h = zmul(tauk, tt);
            bc[0] = make_double2(-0.5 * h.x, -0.5 * h.y);
            sck[1] = bc[0];
        }
        __syncthreads();
        a2 = bc[0];
    }
    double2 *row = Ag + (int64_t)r * N;
    constexpr int RJ = kEigMaxN / kHhRowT;
    double2 a[RJ];
    double s2 = 0.0;
    const double2 vi = upd ? vk[r] : make_double2(0.0, 0.0);
    const double2 wi = upd ? zfma(a2, vi, wk[r]) : make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < RJ; ++q) {
        const int j = r + tid + q * kHhRowT;
        a[q] = make_double2(0.0, 0.0);
        if (j < N) {
            double2 x = row[j];
            if (upd) {
                const double2 vj = vk[j], wj = zfma(a2, vj, wk[j]);
                const double2 t1 = zmulc(vi, wj), t2 = zmulc(wi, vj);
                x.x -= t1.x + t2.x;
                x.y = j == r ? 0.0 : x.y - (t1.y + t2.y);
                row[j] = x;
            }
            a[q] = x;
            if (j == r) dg = x.x;
            if (j == r + 1) bc[3] = x;
            if (j >= r + 2) s2 += x.x * x.x + x.y * x.y;
        }
    }
    if (r >= N - 1) return;
    s2 = wave_sum(s2);
    if (lane == 0) sred[wid] = s2;
    __syncthreads();
    if (tid == 0) {
        double ss = 0.0;
        for (int q = 0; q < kHhRowT / 64; ++q) ss += sred[q];
        double2 tau, scl;
        double beta;
        householder(zconj(bc[3]), ss, tau, beta, scl);
        d[r] = dg;
        e[r] = beta;
        scr[0] = tau;
        hv[N * (N - 1) / 2 + r] = tau;
        bc[1] = tau;
        bc[2] = scl;
    }
    __syncthreads();
    const double2 tau = bc[1], scl = bc[2];
    if (tau.x == 0.0 && tau.y == 0.0) return;
    const int off = refl_off(r, N);
#pragma unroll
    for (int q = 0; q < RJ; ++q) {
        const int j = r + tid + q * kHhRowT;
        if (j >= r + 1 && j < N) {
            const double2 x = j == r + 1 ? make_double2(1.0, 0.0) : zmul(zconj(a[q]), scl);
            vr[j] = x;
            hv[off + (j - r - 1)] = x;
        }
    }
}

// rows i > k + 1: step k's update (if its tau is nonzero), then w of step k + 1,
// tau_r sum_{j > k + 1} A'[i][j] vr[j], from the updated row (one wave per row)
__global__ __launch_bounds__(64 * kHhWaves) void hh_fused(int N, int k, double2 *__restrict__ Ag,
                                                          const double2 *__restrict__ vk,
                                                          const double2 *__restrict__ wk,
                                                          const double2 *__restrict__ sck,
                                                          const double2 *__restrict__ vr, double2 *__restrict__ wr,
                                                          const double2 *__restrict__ scr) {
    const double2 tauk = sck[0], taur = scr[0];
    const bool upd = !(tauk.x == 0.0 && tauk.y == 0.0);
    const int lane = threadIdx.x & 63;
    const int i = k + 2 + blockIdx.x * kHhWaves + (threadIdx.x >> 6);
    if (i >= N) return;
    const double2 a2 = upd ? sck[1] : make_double2(0.0, 0.0);
    double2 *row = Ag + (int64_t)i * N;
    const double2 vi = upd ? vk[i] : make_double2(0.0, 0.0);
    const double2 wi = upd ? zfma(a2, vi, wk[i]) : make_double2(0.0, 0.0);
    double2 acc = make_double2(0.0, 0.0);
    for (int j = k + 1 + lane; j < N; j += 64) {
        double2 x = row[j];
        if (upd) {
            const double2 vj = vk[j], wj = zfma(a2, vj, wk[j]);
            const double2 t1 = zmulc(vi, wj), t2 = zmulc(wi, vj);
            x.x -= t1.x + t2.x;
            x.y = i == j ? 0.0 : x.y - (t1.y + t2.y);
            row[j] = x;
        }
        if (j >= k + 2) acc = zfma(x, vr[j], acc);
    }
    acc = wave_sum2(acc);
    if (lane == 0) wr[i] = zmul(taur, acc);
}

// ---------------------------------------------------------------------------
// Divide and conquer for kLdsMaxN < N <= kEigMaxN over the whole GPU: the tears,
// leaves and merges of dc_block, in launches.  The tears; Z = I; the leaves (one
// wave each, its d, e and rotation lists in LDS); then per level of merges one
// workgroup per merge for the order and deflation (its scratch in LDS), the secular
// roots, the recomputed z and the rows of V each over all of the level's merges, a
// tiled product Z_kept V^T, and the copy of the new columns back into Z; last the
// eigenvalue order.  The product sums over the kept columns in the same order as
// dc_merge_update.  d, e, beta and what the launches of a merge hand on (per row of
// the merge: the order, the deflation flags, the ordered D; per root: the kept
// position, pole, weight, root and recomputed z; per merge, at its first row: the
// kept count and rho |z|^2) stay in global memory.
// ---------------------------------------------------------------------------
struct DcGlobal {
    double *d, *e, *beta;
    double *sd, *kd, *kz, *tau, *zh; // per row of a merge: ordered D; per root: kept pole, weight, root, z
    double *rho;                     // per merge (at its first row): rho |z|^2
    int *perm, *flag, *kept, *kcount, *org;
    int *ctl;                        // [0] largest QL iteration count, [1] a leaf failed
};
// bytes of DcGlobal for N rows (after 256-byte alignment)
__host__ __device__ constexpr size_t dc_global_bytes(int N) { return (size_t)92 * N + 64; }

// eigensolver work bytes: reflectors and taus, then 3 N^2 doubles (Z, V, the
// product's temporary; or the N x N complex copy of A followed by V), the ranks,
// then (256-byte aligned) the divide and conquer's DcGlobal
constexpr size_t eigh_work_bytes(int N) {
    return ((size_t)N * (N - 1) / 2 + N) * sizeof(double2) + (size_t)24 * N * N + (size_t)4 * N + 256 +
           dc_global_bytes(N) + 256;
}

constexpr int kDcLeafWaves = 4;      // leaves (waves) per workgroup
constexpr int kDcTile = 64;          // rows and columns of a product tile
constexpr int kDcKc = 16;            // kept columns per staged chunk of the product

// merge m of the level whose merges are `span` leaves wide: rows [a, c), split at b
__device__ inline double dc_level_merge(int N, int span, int m, const DcGlobal &g, int &a, int &b, int &c) {
    const int P = dc_leaves(N), k = m * span;
    a = (int)((int64_t)k * N / P);
    b = (int)((int64_t)(k + span / 2) * N / P);
    c = (int)((int64_t)(k + span) * N / P);
    return g.beta[k + span / 2];
}

__global__ void dc_tear_kernel(int N, const double2 *__restrict__ Ag, DcGlobal g) {
    if (threadIdx.x != 0) return;
    g.d[N - 1] = Ag[(int64_t)(N - 1) * N + (N - 1)].x;
    g.e[N - 1] = 0.0;
    const int P = dc_leaves(N);
    for (int i = 1; i < P; ++i) {
        const int bb = (int)((int64_t)i * N / P);
        const double be = g.e[bb - 1];
        g.beta[i] = be;
        g.d[bb - 1] -= fabs(be);
        g.d[bb] -= fabs(be);
        g.e[bb - 1] = 0.0;
    }
    g.ctl[0] = 0;
    g.ctl[1] = 0;
}

__global__ __launch_bounds__(256) void dc_identity_kernel(int N, double *__restrict__ Zt) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q < (int64_t)N * N) Zt[q] = (q / N == q % N) ? 1.0 : 0.0;
}

__global__ __launch_bounds__(64 * kDcLeafWaves) void dc_leaf_kernel(int N, double *__restrict__ Zt, DcGlobal g) {
    __shared__ double sd[kDcLeafWaves][kDcLeaf], se[kDcLeafWaves][kDcLeaf];
    __shared__ double scs[kDcLeafWaves][kDcLeaf], ssn[kDcLeafWaves][kDcLeaf];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int P = dc_leaves(N), leaf = blockIdx.x * kDcLeafWaves + wid;
    if (leaf >= P) return;
    const int a = (int)((int64_t)leaf * N / P), n = (int)((int64_t)(leaf + 1) * N / P) - a;
    double *d = sd[wid], *e = se[wid];
    if (lane < n) {
        d[lane] = g.d[a + lane];
        e[lane] = g.e[a + lane];
    }
    dc_sync<64>();
    int l = 0, iter = 0, maxiter = 0;
    bool fail = false;
    for (;;) {
        int nrot;
        const int ms = ql_sweep(n, d, e, scs[wid], ssn[wid], l, iter, maxiter, fail, lane, nrot);
        if (ms < 0) break;
        if (lane < n && nrot > 0) ql_apply(Zt + (int64_t)a * N + a, N, lane, ms, nrot, scs[wid], ssn[wid]);
        __builtin_amdgcn_wave_barrier();
    }
    dc_sync<64>();
    if (lane < n) g.d[a + lane] = d[lane];
    if (lane == 0) {
        atomicMax(&g.ctl[0], maxiter);
        if (fail) atomicMax(&g.ctl[1], 1);
    }
}

// one workgroup per merge of the level: order, deflation and its rotations of Z; hands
// on the order, the deflation flags, the ordered D, the kept positions, poles and
// weights, their count and rho |z|^2
template <int NT>
__global__ __launch_bounds__(NT) void dc_deflate_kernel(int N, int span, double *__restrict__ Zt, DcGlobal g) {
    extern __shared__ unsigned char smem_raw[];
    int a, b, c;
    const double be = dc_level_merge(N, span, blockIdx.x, g, a, b, c);
    if (be == 0.0) return;
    const int n = c - a;
    double *no_chunks = reinterpret_cast<double *>(smem_raw);   // non-null: the product runs elsewhere
    const DcLds t = dc_carve(smem_raw, n, NT / 64, no_chunks, no_chunks);
    dc_merge_deflate<NT>(N, a, b, c, be, g.d, Zt, t);
    const int K = t.ctl[0];
    for (int j = threadIdx.x; j < n; j += NT) {
        g.perm[a + j] = t.perm[j];
        g.flag[a + j] = t.flag[j];
        g.sd[a + j] = t.sD[j];
    }
    for (int i = threadIdx.x; i < K; i += NT) {
        g.kept[a + i] = t.kept[i];
        g.kd[a + i] = t.kd[i];
        g.kz[a + i] = t.kz[i];
    }
    if (threadIdx.x == 0) {
        g.kcount[a] = K;
        g.rho[a] = t.dbl[0];
    }
}

// secular roots of every merge of the level over the whole GPU: kDcRootLanes lanes per
// root, the merge's poles and weights staged in LDS (a workgroup of the one-workgroup
// merge solves its roots in turn, its waves waiting for their slowest root each time)
constexpr int kDcRootLanes = 16;
constexpr int kDcRootsPerBlock = 256 / kDcRootLanes;
__global__ __launch_bounds__(256) void dc_secular_kernel(int N, int span, DcGlobal g) {
    __shared__ double sd[kEigMaxN], sz[kEigMaxN];
    int a, b, c;
    if (dc_level_merge(N, span, blockIdx.y, g, a, b, c) == 0.0) return;
    const int K = g.kcount[a], i0 = blockIdx.x * kDcRootsPerBlock;
    if (i0 >= K) return;
    for (int j = threadIdx.x; j < K; j += 256) {
        sd[j] = g.kd[a + j];
        sz[j] = g.kz[a + j];
    }
    __syncthreads();
    const int sub = threadIdx.x % kDcRootLanes, i = i0 + threadIdx.x / kDcRootLanes;
    if (i < K) {
        int o;
        const double tv = secular_root<kDcRootLanes>(i, K, sd, sz, g.rho[a], sub, &o);
        if (sub == 0) {
            g.tau[a + i] = tv;
            g.org[a + i] = o;
        }
    }
}

// z recomputed from the roots (one thread per kept pole) and the merged eigenvalues
// into d: roots at the kept positions, the deflated positions keep their D
__global__ __launch_bounds__(256) void dc_zh_kernel(int N, int span, DcGlobal g) {
    __shared__ double sd[kEigMaxN], st[kEigMaxN];
    __shared__ int so[kEigMaxN];
    int a, b, c;
    if (dc_level_merge(N, span, blockIdx.y, g, a, b, c) == 0.0) return;
    const int n = c - a, K = g.kcount[a], x = blockIdx.x * 256 + threadIdx.x;
    if ((int)blockIdx.x * 256 >= n) return;
    for (int j = threadIdx.x; j < K; j += 256) {
        sd[j] = g.kd[a + j];
        st[j] = g.tau[a + j];
        so[j] = g.org[a + j];
    }
    __syncthreads();
    if (x < K) {
        double w = 1.0;
        for (int i = 0; i < K; ++i) {
            const double xi = (sd[so[i]] - sd[x]) + st[i];
            w *= i == x ? xi : xi * rcp64(sd[i] - sd[x]);
        }
        g.zh[a + x] = copysign(sqrt(fmax(w, 0.0) / g.rho[a]), g.kz[a + x]);
        g.d[a + g.kept[a + x]] = sd[so[x]] + st[x];
    }
    if (x < n && g.flag[a + x] > 0) g.d[a + x] = g.sd[a + x];
}

// V of every merge of the level (at V + a N, row i for root i): one wave per row,
// V[i][j] = zh_j / (d_j - x_i), normalised
constexpr int kDcVWaves = 4;
__global__ __launch_bounds__(64 * kDcVWaves) void dc_vmat_kernel(int N, int span, double *__restrict__ V, DcGlobal g) {
    __shared__ double sd[kEigMaxN], sz[kEigMaxN];
    int a, b, c;
    if (dc_level_merge(N, span, blockIdx.y, g, a, b, c) == 0.0) return;
    const int K = g.kcount[a], i0 = blockIdx.x * kDcVWaves;
    if (i0 >= K) return;
    for (int j = threadIdx.x; j < K; j += 64 * kDcVWaves) {
        sd[j] = g.kd[a + j];
        sz[j] = g.zh[a + j];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, i = i0 + (threadIdx.x >> 6);
    if (i >= K) return;
    const double ti = g.tau[a + i], dorg = sd[g.org[a + i]];
    constexpr int J = kEigMaxN / 64;
    double v[J];
    double nrm = 0.0;
#pragma unroll
    for (int q = 0; q < J; ++q) {
        const int j = lane + 64 * q;
        v[q] = j < K ? sz[j] * rcp64((sd[j] - dorg) - ti) : 0.0;
        nrm += v[q] * v[q];
    }
    const double inv = 1.0 / sqrt(wave_sum(nrm));
    double *row = V + (int64_t)a * N + (int64_t)i * K;
#pragma unroll
    for (int q = 0; q < J; ++q) {
        const int j = lane + 64 * q;
        if (j < K) row[j] = v[q] * inv;
    }
}

// new columns of every merge of the level into its temporary (Ztmp + a N, column j
// at j n): deflated ones copied, kept ones Z_kept V^T in 64 x 64 tiles, 4 x 4 per
// thread, over kDcKc-deep chunks of the kept columns staged in LDS
__global__ __launch_bounds__(256) void dc_product_kernel(int N, int span, int tiles, const double *__restrict__ Zt,
                                                         const double *__restrict__ V, double *__restrict__ Ztmp,
                                                         DcGlobal g) {
    __shared__ double zs[kDcKc][kDcTile], vs[kDcKc][kDcTile];
    int a, b, c;
    if (dc_level_merge(N, span, blockIdx.y, g, a, b, c) == 0.0) return;
    const int n = c - a;
    const int r0 = (blockIdx.x % tiles) * kDcTile, c0 = (blockIdx.x / tiles) * kDcTile;
    if (r0 >= n || c0 >= n) return;
    const int tid = threadIdx.x, K = g.kcount[a];
    const int *perm = g.perm + a, *flag = g.flag + a, *kept = g.kept + a;
    double *Zm = Ztmp + (int64_t)a * N;
    const double *Vm = V + (int64_t)a * N;
    for (int e = tid; e < kDcTile * kDcTile; e += 256) {
        const int tc = c0 + e / kDcTile, r = r0 + e % kDcTile;
        if (tc < n && r < n && flag[tc] > 0) Zm[(int64_t)tc * n + r] = Zt[(int64_t)perm[tc] * N + a + r];
    }
    if (c0 >= K) return;
    const int tr = (tid & 15) * 4, tq = (tid >> 4) * 4;
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
    for (int j0 = 0; j0 < K; j0 += kDcKc) {
        const int kc = min(kDcKc, K - j0);
        __syncthreads();
        for (int e = tid; e < kDcKc * kDcTile; e += 256) {
            const int jj = e / kDcTile, x = e % kDcTile;           // Z: rows contiguous
            zs[jj][x] = jj < kc && r0 + x < n ? Zt[(int64_t)perm[kept[j0 + jj]] * N + a + r0 + x] : 0.0;
            const int cy = e / kDcKc, ji = e % kDcKc;              // V: kept index contiguous
            vs[ji][cy] = ji < kc && c0 + cy < K ? Vm[(int64_t)(c0 + cy) * K + j0 + ji] : 0.0;
        }
        __syncthreads();
        for (int jj = 0; jj < kc; ++jj) {
            double zr[4], vr[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) zr[x] = zs[jj][tr + x];
#pragma unroll
            for (int y = 0; y < 4; ++y) vr[y] = vs[jj][tq + y];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = fma(zr[x], vr[y], acc[x][y]);
        }
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int r = r0 + tr + x, cc = c0 + tq + y;
            if (r < n && cc < K) Zm[(int64_t)kept[cc] * n + r] = acc[x][y];
        }
}

// the level's new columns back into Z (block x: column x of each merge)
__global__ __launch_bounds__(256) void dc_write_kernel(int N, int span, double *__restrict__ Zt,
                                                       const double *__restrict__ Ztmp, DcGlobal g) {
    int a, b, c;
    if (dc_level_merge(N, span, blockIdx.y, g, a, b, c) == 0.0) return;
    const int n = c - a, col = blockIdx.x;
    if (col >= n) return;
    const double *src = Ztmp + (int64_t)a * N + (int64_t)col * n;
    double *dst = Zt + (int64_t)(a + col) * N + a;
    for (int r = threadIdx.x; r < n; r += 256) dst[r] = src[r];
}

// eigenvalues ordered by key (ties by value, then index) into lam, ranks, info
__global__ __launch_bounds__(256) void dc_order_kernel(int N, DcGlobal g, int *__restrict__ rank,
                                                       double *__restrict__ lam, int key, double ref,
                                                       int *__restrict__ info) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i == 0 && info) info[0] = g.ctl[1] ? -1 : g.ctl[0];
    if (i >= N) return;
    const double li = g.d[i];
    const double ki = key ? fabs(li - ref) : li;
    int rk = 0;
    for (int j = 0; j < N; ++j) {
        const double lj = g.d[j];
        const double kj = key ? fabs(lj - ref) : lj;
        if (kj < ki || (kj == ki && (lj < li || (lj == li && j < i)))) ++rk;
    }
    lam[rk] = li;
    rank[i] = rk;
}

// Back-transformation, one wave per eigenvector, NW waves per workgroup.
// LDS_V: all reflectors staged in LDS (N <= kLdsMaxN); otherwise read from
// global memory one reflector ahead.
template <int NW, int NMAX, bool LDS_V>
__device__ __forceinline__ void backtransform_body(int N, const double2 *__restrict__ hv,
                                                   const double *__restrict__ zg, const int *__restrict__ rank,
                                                   double2 *__restrict__ R, int bx) {
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
    const int m = bx * NW + wid;
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

template <int NW, int NMAX, bool LDS_V>
__global__ __launch_bounds__(64 * NW) void backtransform_kernel(int N, const double2 *__restrict__ hv,
                                                                const double *__restrict__ zg,
                                                                const int *__restrict__ rank,
                                                                double2 *__restrict__ R) {
    backtransform_body<NW, NMAX, LDS_V>(N, hv, zg, rank, R, blockIdx.x);
}

template <int NW, int NMAX>
__global__ __launch_bounds__(64 * NW) void backtransform_lds_jobs(const DenseJob *__restrict__ jobs,
                                                                  const int *__restrict__ mask) {
    if (!mask[blockIdx.y]) return;
    const DenseJob &j = jobs[blockIdx.y];
    if ((int)blockIdx.x * NW >= j.N) return;
    backtransform_body<NW, NMAX, true>(j.N, j.hv, j.zbuf, j.rank, j.R, blockIdx.x);
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

// ---------------------------------------------------------------------------
// Blocked Cholesky and inverse for N > kLdsMaxN (right-looking, blocks of kCholB):
// for each diagonal block, the one-workgroup LDS kernel factors it and writes
// T_kk = conj(L_kk^-1) into T's diagonal block; the panel below becomes
// L_ik = A_ik L_kk^-H = A_ik T_kk^T and the trailing matrix A -= L_p L_p^H, both
// multi-workgroup FP64 MFMA products.  Then T by block rows (T = conj(X),
// X = L^-1): T_ij = -T_ii sum_{m = j}^{i-1} conj(L_im) T_mj, i.e. one product
// with T's rows above and one with T_ii.  Work: W (N x N) holding L, then the
// transposed diagonal inverse (B x B), the panel (N x B) and its conjugate
// transpose (B x N), reused for conj(L)'s block row and the sums in the inverse.
// ---------------------------------------------------------------------------
constexpr int kCholB = 128;

__global__ void k_transpose_block(int rows, int cols, const double2 *__restrict__ src, int64_t lds,
                                  double2 *__restrict__ dst, int64_t ldd, int conjugate) {
    __shared__ double2 tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 32 x 8
    for (int y = ty; y < 32; y += 8) {
        const int r = r0 + y, c = c0 + tx;
        if (r < rows && c < cols) tile[y][tx] = src[(int64_t)r * lds + c];
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int c = c0 + y, r = r0 + tx;
        if (r < rows && c < cols) {
            const double2 v = tile[tx][y];
            dst[(int64_t)c * ldd + r] = conjugate ? make_double2(v.x, -v.y) : v;
        }
    }
}

__global__ void k_conj_copy(int rows, int cols, const double2 *__restrict__ src, int64_t lds,
                            double2 *__restrict__ dst, int64_t ldd) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (c < cols) {
        const double2 v = src[(int64_t)r * lds + c];
        dst[(int64_t)r * ldd + c] = make_double2(v.x, -v.y);
    }
}

static void transpose_block(int rows, int cols, const double2 *src, int64_t lds, double2 *dst, int64_t ldd, bool cj,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_transpose_block, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, st, rows, cols, src,
                       lds, dst, ldd, cj ? 1 : 0);
    PW_LAUNCH_CHECK();
}

size_t chol_inv_work_bytes(int N) {
    if (N <= kLdsMaxN) return (size_t)N * N * sizeof(double2);
    return ((size_t)N * N + (size_t)kCholB * kCholB + (size_t)2 * N * kCholB) * sizeof(double2);
}

static void chol_diag(int b, const double2 *A, int64_t lda, double2 *T, int64_t ldt, int pivot_base, int *status,
                      hipStream_t st) {
    const size_t bytes = (size_t)b * (b + 1) / 2 * sizeof(double2);
    static size_t attr_bytes = 64 * 1024;   // default dynamic LDS limit
    lds_limit(reinterpret_cast<const void *>(chol_inv_lds_kernel<1024>), bytes, attr_bytes);
    hipLaunchKernelGGL(chol_inv_lds_kernel<1024>, dim3(1), dim3(1024), bytes, st, b, A, lda, T, ldt, pivot_base,
                       status);
    PW_LAUNCH_CHECK();
}

void chol_inv(int N, const void *S_, int64_t lds, void *work, void *T_, int *status, hipStream_t st) {
    PW_CHECK(N > 0 && N <= 8192, PW_EINVAL, "bad Cholesky size %d", N);
    const double2 *S = (const double2 *)S_;
    double2 *T = (double2 *)T_;
    if (N <= kLdsMaxN) {
        chol_diag(N, S, lds, T, N, 0, status, st);
        return;
    }
    constexpr int B = kCholB;
    double2 *W = (double2 *)work;
    double2 *TkT = W + (size_t)N * N, *P = TkT + (size_t)B * B, *PH = P + (size_t)N * B;
    copy_block(N, N, S, lds, W, N, st);
    fill_zero(T, (size_t)N * N * sizeof(double2), st);
    for (int k0 = 0; k0 < N; k0 += B) {
        const int b = std::min(B, N - k0), r0 = k0 + b, rows = N - r0;
        chol_diag(b, W + (size_t)k0 * N + k0, N, T + (size_t)k0 * N + k0, N, k0, status, st);
        if (rows == 0) break;
        transpose_block(b, b, T + (size_t)k0 * N + k0, N, TkT, b, false, st);                // T_kk^T = L_kk^-H
        zgemm_nn_launch(rows, b, b, W + (size_t)r0 * N + k0, N, TkT, b, 1.0, 0.0, P, b, st);  // L_ik
        copy_block(rows, b, P, b, W + (size_t)r0 * N + k0, N, st);
        transpose_block(rows, b, P, b, PH, rows, true, st);                                  // L_p^H
        zgemm_nn_launch(rows, rows, b, P, b, PH, rows, -1.0, 1.0, W + (size_t)r0 * N + r0, N, st);
    }
    for (int i0 = B; i0 < N; i0 += B) {
        const int b = std::min(B, N - i0);
        hipLaunchKernelGGL(k_conj_copy, dim3((i0 + 255) / 256, b), dim3(256), 0, st, b, i0,
                           (const double2 *)(W + (size_t)i0 * N), (int64_t)N, P, (int64_t)i0);
        PW_LAUNCH_CHECK();
        zgemm_nn_launch(b, i0, i0, P, i0, T, N, 1.0, 0.0, PH, i0, st);                         // sums
        zgemm_nn_launch(b, i0, b, T + (size_t)i0 * N + i0, N, PH, i0, -1.0, 0.0, T + (size_t)i0 * N, N, st);
    }
}

// Batched small dense kernels (N <= kLdsMaxN, one workgroup per problem) for
// batched folded-CG runs: the bodies of chol_inv's and dense_eigh's one-workgroup
// path with each job's arguments (key 0).
DenseJob dense_job(int N, const void *A, int64_t lda, void *work, double *lam, void *R, int *info, void *T,
                   int *status) {
    PW_CHECK(N >= 1 && N <= kLdsMaxN, PW_EUNSUPPORTED, "batched dense kernels need N <= %d", kLdsMaxN);
    DenseJob j{};
    j.N = N;
    j.A = (const double2 *)A;
    j.lda = lda;
    j.T = (double2 *)T;
    j.ldt = N;
    j.status = status;
    j.hv = (double2 *)work;
    j.zbuf = (double *)(j.hv + ((size_t)N * (N - 1) / 2 + N));
    j.rank = (int *)((char *)j.zbuf + (size_t)24 * N * N);
    j.lam = lam;
    j.R = (double2 *)R;
    j.info = info;
    return j;
}

void chol_inv_jobs(int N, const DenseJob *jobs, const int *mask, int njobs, hipStream_t st) {
    PW_CHECK(N >= 1 && N <= kLdsMaxN, PW_EUNSUPPORTED, "batched Cholesky needs N <= %d", kLdsMaxN);
    const size_t bytes = (size_t)N * (N + 1) / 2 * sizeof(double2);
    static size_t attr_bytes = 64 * 1024;
    lds_limit(reinterpret_cast<const void *>(chol_inv_lds_jobs<1024>), bytes, attr_bytes);
    hipLaunchKernelGGL(chol_inv_lds_jobs<1024>, dim3(njobs), dim3(1024), bytes, st, jobs, mask);
    PW_LAUNCH_CHECK();
}

void dense_eigh_jobs(int N, const DenseJob *jobs, const int *mask, int njobs, hipStream_t st) {
    PW_CHECK(N >= 1 && N <= kLdsMaxN, PW_EUNSUPPORTED, "batched eigensolver needs N <= %d", kLdsMaxN);
    const size_t dcb = dc_round(dc_lds_bytes(N, kEigNT / 64, true)) + dc_wave_bytes(N, kEigNT / 64);
    const size_t b1 = std::max((size_t)N * (N + 1) / 2 * sizeof(double2), dcb);
    static size_t attr1 = 64 * 1024, attr2 = 64 * 1024;
    lds_limit(reinterpret_cast<const void *>(tridiag_ql_lds_jobs<kEigNT>), b1, attr1);
    hipLaunchKernelGGL(tridiag_ql_lds_jobs<kEigNT>, dim3(njobs), dim3(kEigNT), b1, st, jobs, mask);
    PW_LAUNCH_CHECK();
    const size_t b2 = std::max<size_t>(1, (size_t)N * (N - 1) / 2 + N - 1) * sizeof(double2);
    lds_limit(reinterpret_cast<const void *>(backtransform_lds_jobs<kBackNW, kLdsMaxN>), b2, attr2);
    hipLaunchKernelGGL((backtransform_lds_jobs<kBackNW, kLdsMaxN>), dim3((N + kBackNW - 1) / kBackNW, njobs),
                       dim3(64 * kBackNW), b2, st, jobs, mask);
    PW_LAUNCH_CHECK();
}

size_t dense_eigh_work_bytes(int N) { return eigh_work_bytes(N); }

void dense_eigh(int N, const void *A, int64_t lda, void *work, double *lam, void *R, int key, double ref, int *info,
                hipStream_t st) {
    PW_CHECK(N >= 1 && N <= kEigMaxN, PW_EUNSUPPORTED, "dense eigensolver limited to 1 <= N <= 1024");
    const bool lds = N <= kLdsMaxN;
    double2 *hv = (double2 *)work;
    double2 *zbuf = hv + ((size_t)N * (N - 1) / 2 + N);
    int *rank = (int *)((char *)zbuf + (size_t)24 * N * N);
    const size_t dcb = lds ? dc_round(dc_lds_bytes(N, kEigNT / 64, true)) + dc_wave_bytes(N, kEigNT / 64)
                           : dc_lds_bytes(N, kEigNT / 64, false);
    static size_t attr1 = 64 * 1024, attr2 = 64 * 1024, attr3 = 64 * 1024;
    if (lds) {
        const size_t b1 = std::max((size_t)N * (N + 1) / 2 * sizeof(double2), dcb);
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
        // the reduction over the whole GPU (the matrix copy in the first 16 N^2 bytes of
        // zbuf; v, w and the step's scalars in the next 8 N^2, which V takes later),
        // then the divide and conquer (d, e and the merges' hand-over after the ranks)
        double2 *Ag = (double2 *)zbuf;
        char *ext = (char *)(((uintptr_t)(rank + N) + 255) & ~(uintptr_t)255);
        DcGlobal g;
        g.d = (double *)ext;
        g.e = g.d + N;
        g.beta = g.e + N;
        g.sd = g.beta + N;
        g.kd = g.sd + N;
        g.kz = g.kd + N;
        g.tau = g.kz + N;
        g.zh = g.tau + N;
        g.rho = g.zh + N;
        g.perm = (int *)(g.rho + N);
        g.flag = g.perm + N;
        g.kept = g.flag + N;
        g.kcount = g.kept + N;
        g.org = g.kcount + N;
        g.ctl = g.org + N;
        HhBufs hb;
        hb.v[0] = (double2 *)((char *)zbuf + (size_t)16 * N * N);
        hb.v[1] = hb.v[0] + N;
        hb.w[0] = hb.v[1] + N;
        hb.w[1] = hb.w[0] + N;
        hb.sc[0] = hb.w[1] + N;
        hb.sc[1] = hb.sc[0] + 2;
        hb.d = g.d;
        hb.e = g.e;
        hipLaunchKernelGGL(hh_symmetrize, dim3(N), dim3(256), 0, st, N, (const double2 *)A, lda, Ag);
        // reflector 0, w of step 0; then per step k: row k + 1 and reflector k + 1, the rows
        // below with w of step k + 1; last, row N - 1 with the update of step N - 2
        hipLaunchKernelGGL(hh_rowstep, dim3(1), dim3(kHhRowT), 0, st, N, -1, Ag, hv, (const double2 *)hb.v[1],
                           (const double2 *)hb.w[1], hb.sc[1], hb.v[0], hb.sc[0], hb.d, hb.e);
        HhScratch s0;
        s0.v = hb.v[0];
        s0.w = hb.w[0];
        s0.sc = hb.sc[0];
        s0.d = hb.d;
        s0.e = hb.e;
        hipLaunchKernelGGL(hh_matvec, dim3((N - 1 + kHhWaves - 1) / kHhWaves), dim3(64 * kHhWaves), 0, st, N, 0,
                           (const double2 *)Ag, s0);
        PW_LAUNCH_CHECK();
        for (int k = 0; k + 1 < N; ++k) {
            const int p = k & 1, q = p ^ 1;
            hipLaunchKernelGGL(hh_rowstep, dim3(1), dim3(kHhRowT), 0, st, N, k, Ag, hv, (const double2 *)hb.v[p],
                               (const double2 *)hb.w[p], hb.sc[p], hb.v[q], hb.sc[q], hb.d, hb.e);
            if (k + 2 < N)
                hipLaunchKernelGGL(hh_fused, dim3((N - k - 2 + kHhWaves - 1) / kHhWaves), dim3(64 * kHhWaves), 0, st,
                                   N, k, Ag, (const double2 *)hb.v[p], (const double2 *)hb.w[p],
                                   (const double2 *)hb.sc[p], (const double2 *)hb.v[q], hb.w[q],
                                   (const double2 *)hb.sc[q]);
        }
        PW_LAUNCH_CHECK();
        double *Zt = (double *)zbuf, *Ztmp = Zt + (size_t)N * N, *V = Zt + 2 * (size_t)N * N;
        hipLaunchKernelGGL(dc_tear_kernel, dim3(1), dim3(64), 0, st, N, (const double2 *)Ag, g);
        hipLaunchKernelGGL(dc_identity_kernel, dim3((unsigned)(((int64_t)N * N + 255) / 256)), dim3(256), 0, st, N,
                           Zt);
        const int P = dc_leaves(N);
        hipLaunchKernelGGL(dc_leaf_kernel, dim3((P + kDcLeafWaves - 1) / kDcLeafWaves), dim3(64 * kDcLeafWaves), 0,
                           st, N, Zt, g);
        PW_LAUNCH_CHECK();
        for (int span = 2; span <= P; span *= 2) {
            const int nm = P / span;
            const int nmax = (int)(((int64_t)span * N + P - 1) / P) + 1;   // no merge of the level is larger
            const size_t lb = dc_lds_bytes(nmax, kEigNT / 64, false);
            lds_limit(reinterpret_cast<const void *>(dc_deflate_kernel<kEigNT>), lb, attr3);
            hipLaunchKernelGGL(dc_deflate_kernel<kEigNT>, dim3(nm), dim3(kEigNT), lb, st, N, span, Zt, g);
            hipLaunchKernelGGL(dc_secular_kernel, dim3((nmax + kDcRootsPerBlock - 1) / kDcRootsPerBlock, nm),
                               dim3(256), 0, st, N, span, g);
            hipLaunchKernelGGL(dc_zh_kernel, dim3((nmax + 255) / 256, nm), dim3(256), 0, st, N, span, g);
            hipLaunchKernelGGL(dc_vmat_kernel, dim3((nmax + kDcVWaves - 1) / kDcVWaves, nm), dim3(64 * kDcVWaves), 0,
                               st, N, span, V, g);
            const int tiles = (nmax + kDcTile - 1) / kDcTile;
            hipLaunchKernelGGL(dc_product_kernel, dim3(tiles * tiles, nm), dim3(256), 0, st, N, span, tiles,
                               (const double *)Zt, (const double *)V, Ztmp, g);
            hipLaunchKernelGGL(dc_write_kernel, dim3(nmax, nm), dim3(256), 0, st, N, span, Zt, (const double *)Ztmp,
                               g);
            PW_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(dc_order_kernel, dim3((N + 255) / 256), dim3(256), 0, st, N, g, rank, lam, key, ref, info);
        PW_LAUNCH_CHECK();
        hipLaunchKernelGGL((backtransform_kernel<kBackNW, kEigMaxN, false>), dim3((N + kBackNW - 1) / kBackNW),
                           dim3(64 * kBackNW), 0, st, N, (const double2 *)hv, (const double *)zbuf, (const int *)rank,
                           (double2 *)R);
    }
    PW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// The eigensolver without allocation (pw_dense_eigh_noalloc): its work memory is
// the file-scope device array `scratch`, one copy per GPU for the life of the
// process.  In host code the array's name only stands for the symbol, so host
// code never hands it to a kernel or a copy: it uses the device address that
// hipGetSymbolAddress returns, looked up once per device with that device current
// and kept per device.  Sized for N <= kNoAllocMaxN: the eigensolver's work, then
// 256 bytes for the QL iteration count.
// ---------------------------------------------------------------------------
constexpr int kNoAllocMaxN = 512;
constexpr size_t kNoAllocWork = (eigh_work_bytes(kNoAllocMaxN) + 255) / 256 * 256;
constexpr size_t kScratchBytes = kNoAllocWork + 256;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// device address of `scratch` on the current device (looked up on its first use there)
static void *scratch_on_current_device() {
    int dev = 0;
    PW_HIP(hipGetDevice(&dev));
    PW_CHECK(dev >= 0 && dev < kMaxDevices, PW_EUNSUPPORTED, "device ordinal %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        PW_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        PW_CHECK(ptr != nullptr, PW_EHIP, "no device address for the eigensolver scratch");
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace pw

extern "C" pw_status pw_dense_eigh_noalloc(int32_t n, const void *A, int64_t lda, double *w, void *R, int32_t key,
                                           double ref, int32_t *sweeps, void *stream) {
    try {
        PW_CHECK(n >= 1 && n <= pw::kNoAllocMaxN && lda >= n && A && w && R, PW_EINVAL,
                 "bad pw_dense_eigh_noalloc arguments (1 <= n <= %d)", pw::kNoAllocMaxN);
        PW_CHECK(key == 0 || key == 1, PW_EINVAL, "key must be 0 or 1");
        PW_CHECK(pw::dense_eigh_work_bytes(n) <= pw::kNoAllocWork, PW_EUNSUPPORTED, "scratch too small for n = %d", n);
        hipStream_t st = (hipStream_t)stream;
        char *base = (char *)pw::scratch_on_current_device();
        int *info = (int *)(base + pw::kNoAllocWork);
        pw::fill_zero(info, 16, st);                 // the array keeps the last call's contents
        pw::dense_eigh(n, A, lda, base, w, R, key, ref, info, st);
        int h = 0;
        PW_HIP(hipMemcpyAsync(&h, info, sizeof(int), hipMemcpyDeviceToHost, st));
        PW_HIP(hipStreamSynchronize(st));
        if (sweeps) *sweeps = h;
        PW_CHECK(h >= 0, PW_ENOCONV, "tridiagonal QL iteration did not converge");
        return PW_OK;
    } catch (const pw::Fail &f) {
        return f.st;
    } catch (...) {
        pw::set_error("unexpected exception in pw_dense_eigh_noalloc");
        return PW_EINVAL;
    }
}
