// Small dense FP64 linear algebra on the GPU for the block solver.
//
//   chol_inv_*         : S = L L^H (Cholesky), T = conj(L^{-1}), so that the band-major
//                        block Psi' = T . Psi is orthonormal (Gram/Cholesky step).
//   tridiag_ql_kernel + backtransform_kernel (N <= 136) and jacobi_kernel (larger N):
//                        Hermitian eigensolver for the Rayleigh-Ritz subspace step;
//                        outputs the eigenvalues and the band-major rotation R with
//                        Psi' = R . Psi.
// The factorisations run as one workgroup; they are O(N^3) on N x N matrices and
// off the O(N^2 npw) critical path.
#include "common.h"

#include <algorithm>
#include <cfloat>

namespace pw {

__device__ inline double2 zmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 zmulc(double2 a, double2 b) { return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }   // a conj(b)
__device__ inline double2 zconj(double2 a) { return make_double2(a.x, -a.y); }

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

template <int NT>
__global__ __launch_bounds__(NT) void chol_inv_lds_kernel(int N, const double2 *__restrict__ S, int64_t lds,
                                                          double2 *__restrict__ T, int *__restrict__ status) {
    extern __shared__ unsigned char smem_raw[];
    double2 *L = reinterpret_cast<double2 *>(smem_raw);
    __shared__ double piv;
    __shared__ int bad;
    const int tid = threadIdx.x;
    for (int i = 0; i < N; ++i)
        for (int k = tid; k <= i; k += NT) L[tri(i, k)] = S[(int64_t)i * lds + k];
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
// Hermitian Jacobi.  A (N x N, ld N) is overwritten; V accumulates eigenvectors
// as columns.  Output: lam[b] (sorted by key), R[b][j] = V[j][perm b] so that
// new band b = sum_j R[b][j] old_j.  key: 0 ascending lam, 1 ascending |lam - ref|
// (ties by lam).  Odd N is handled by a dummy index that never rotates.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void jacobi_kernel(int N, const double2 *__restrict__ Ain, int64_t lda,
                                                      double2 *__restrict__ A, double2 *__restrict__ V,
                                                      double *__restrict__ lam, double2 *__restrict__ R,
                                                      int key, double ref, int max_sweeps, double tol,
                                                      int *__restrict__ info) {
    extern __shared__ unsigned char smem_raw[];
    // per pair: p, q, c, s (real), phase (complex)
    int *pp = reinterpret_cast<int *>(smem_raw);
    int *qq = pp + 512;
    double *cs = reinterpret_cast<double *>(qq + 512);
    double *sn = cs + 512;
    double2 *ph = reinterpret_cast<double2 *>(sn + 512);
    __shared__ double red[1024];
    __shared__ int sweeps_done;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int Ne = N + (N & 1);        // even player count
    const int npair = Ne / 2;
    for (int e = tid; e < N * N; e += nt) {
        const int i = e / N, k = e % N;
        double2 a = Ain[(int64_t)i * lda + k];
        const double2 b = Ain[(int64_t)k * lda + i];
        A[e] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));   // Hermitian part
        V[e] = make_double2(i == k ? 1.0 : 0.0, 0.0);
    }
    if (tid == 0) sweeps_done = 0;
    __syncthreads();
    double prev_offs = INFINITY;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        // convergence: off-diagonal Frobenius norm vs diagonal
        double off = 0.0, dia = 0.0;
        for (int e = tid; e < N * N; e += nt) {
            const int i = e / N, k = e % N;
            const double2 a = A[e];
            if (i != k) off += a.x * a.x + a.y * a.y;
            else dia += a.x * a.x;
        }
        red[tid] = off;
        __syncthreads();
        for (int s = nt / 2; s > 0; s >>= 1) { if (tid < s) red[tid] += red[tid + s]; __syncthreads(); }
        const double offs = red[0];
        __syncthreads();
        red[tid] = dia;
        __syncthreads();
        for (int s = nt / 2; s > 0; s >>= 1) { if (tid < s) red[tid] += red[tid + s]; __syncthreads(); }
        const double dias = red[0];
        __syncthreads();
        // converged: relative off-diagonal Frobenius norm below tol, or at the
        // rounding floor (no further decrease once already below 1e-10)
        const double tot = dias + offs;
        if (offs <= tol * tol * tot || offs == 0.0) break;
        if (sweep > 0 && offs <= 1e-28 * tot && offs >= 0.5 * prev_offs) break;   // rounding floor
        prev_offs = offs;
        if (tid == 0) sweeps_done = sweep + 1;
        for (int r = 0; r < Ne - 1; ++r) {
            // pairs of this round (circle method)
            for (int k = tid; k < npair; k += nt) {
                int p, q;
                if (k == 0) { p = r; q = Ne - 1; }
                else { p = (r + k) % (Ne - 1); q = (r - k + Ne - 1) % (Ne - 1); }
                if (p > q) { int t = p; p = q; q = t; }
                pp[k] = p; qq[k] = q;
                double c = 1.0, s = 0.0;
                double2 e = make_double2(1.0, 0.0);
                if (q < N) {
                    const double app = A[(int64_t)p * N + p].x, aqq = A[(int64_t)q * N + q].x;
                    const double2 apq = A[(int64_t)p * N + q];
                    const double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
                    if (mag > 0.0) {
                        const double tau = (aqq - app) / (2.0 * mag);
                        const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                        e = make_double2(apq.x / mag, -apq.y / mag);    // exp(-i phi)
                    }
                }
                cs[k] = c; sn[k] = s; ph[k] = e;
            }
            __syncthreads();
            // U = [[c, s], [-e s, e c]] with e = exp(-i phi); rows: A <- U^H A
            for (int w = tid; w < npair * N; w += nt) {
                const int k = w / N, col = w % N;
                const int p = pp[k], q = qq[k];
                if (q >= N || sn[k] == 0.0) continue;
                const double c = cs[k], s = sn[k];
                const double2 e = ph[k];
                const double2 ap = A[(int64_t)p * N + col], aq = A[(int64_t)q * N + col];
                // new_p = c ap - s conj(e) aq ; new_q = s ap + c conj(e) aq
                const double2 ea = zmul(zconj(e), aq);
                A[(int64_t)p * N + col] = make_double2(c * ap.x - s * ea.x, c * ap.y - s * ea.y);
                A[(int64_t)q * N + col] = make_double2(s * ap.x + c * ea.x, s * ap.y + c * ea.y);
            }
            __syncthreads();
            // columns: A <- A U, V <- V U
            for (int w = tid; w < npair * N; w += nt) {
                const int k = w / N, row = w % N;
                const int p = pp[k], q = qq[k];
                if (q >= N || sn[k] == 0.0) continue;
                const double c = cs[k], s = sn[k];
                const double2 e = ph[k];
                {
                    const double2 ap = A[(int64_t)row * N + p], aq = A[(int64_t)row * N + q];
                    // new_p = c ap - s e aq ; new_q = s ap + c e aq
                    const double2 ea = zmul(e, aq);
                    A[(int64_t)row * N + p] = make_double2(c * ap.x - s * ea.x, c * ap.y - s * ea.y);
                    A[(int64_t)row * N + q] = make_double2(s * ap.x + c * ea.x, s * ap.y + c * ea.y);
                }
                {
                    const double2 vp = V[(int64_t)row * N + p], vq = V[(int64_t)row * N + q];
                    const double2 ev = zmul(e, vq);
                    V[(int64_t)row * N + p] = make_double2(c * vp.x - s * ev.x, c * vp.y - s * ev.y);
                    V[(int64_t)row * N + q] = make_double2(s * vp.x + c * ev.x, s * vp.y + c * ev.y);
                }
            }
            __syncthreads();
            for (int k = tid; k < npair; k += nt) {
                const int p = pp[k], q = qq[k];
                if (q < N && sn[k] != 0.0) {
                    A[(int64_t)p * N + q] = make_double2(0.0, 0.0);
                    A[(int64_t)q * N + p] = make_double2(0.0, 0.0);
                    A[(int64_t)p * N + p].y = 0.0;
                    A[(int64_t)q * N + q].y = 0.0;
                }
            }
            __syncthreads();
        }
    }
    // sort by key: rank of each eigenvalue
    double *dval = reinterpret_cast<double *>(red);     // reuse (N <= 1024)
    __syncthreads();
    for (int i = tid; i < N; i += nt) dval[i] = A[(int64_t)i * N + i].x;
    __syncthreads();
    for (int i = tid; i < N; i += nt) {
        const double li = dval[i];
        const double ki = key ? fabs(li - ref) : li;
        int rank = 0;
        for (int j = 0; j < N; ++j) {
            const double lj = dval[j];
            const double kj = key ? fabs(lj - ref) : lj;
            if (kj < ki || (kj == ki && (lj < li || (lj == li && j < i)))) ++rank;
        }
        lam[rank] = li;
        for (int j = 0; j < N; ++j) R[(int64_t)rank * N + j] = V[(int64_t)j * N + i];
    }
    if (tid == 0 && info) info[0] = sweeps_done;
}

// ---------------------------------------------------------------------------
// Hermitian eigensolver for N <= kLdsMaxN in two launches.
//
// tridiag_ql_kernel (one workgroup, A in LDS as a packed lower triangle):
//   1. Householder reduction A = Q T Q^H, T real symmetric tridiagonal,
//      Q = H_0 H_1 ... H_{N-2}.  H_k = I - tau_k v_k v_k^H acts on rows k+1..N-1
//      with v_k[k+1] = 1 and H_k^H sending column k below the diagonal to
//      beta_k e_1, beta_k real (complex reflectors in the convention of LAPACK's
//      zlarfg; the two-sided update A22 <- H^H A22 H is the rank-2 form
//      A22 - v w^H - w v^H with w = tau A22 v - (tau/2)(tau A22 v)^H v v).
//      v_k (entries k+1..N-1) is stored at hv + k(N-1) - k(k-1)/2, tau_k at
//      hv + N(N-1)/2 + k.
//   2. T = Z diag(d) Z^T by implicit QL with Wilkinson's shift (the tql2
//      algorithm of Bowdler, Martin, Reinsch and Wilkinson, 1968).  One lane
//      runs the scalar recurrence of a QL sweep and records its Givens
//      rotations; every lane then applies them to its own row of Z (held
//      column-major in the LDS the triangle used).
//   3. Eigenvalues ordered by key into lam; Z column m to zg[m N + r] and its
//      rank to rank[m].  info = largest QL iteration count of an eigenvalue,
//      -1 if one needed more than kQlMaxIter.
// backtransform_kernel: eigenvector m of A is Q Z[:, m]; written as row rank[m]
//   of R (R . Psi rotates a band-major block, as for jacobi_kernel).
// ---------------------------------------------------------------------------
constexpr int kQlMaxIter = 60;

__device__ inline double2 zfma(double2 a, double2 b, double2 c) {
    return make_double2(c.x + a.x * b.x - a.y * b.y, c.y + a.x * b.y + a.y * b.x);
}
__device__ inline double2 lds_get(const double2 *L, int i, int k) {
    return i >= k ? L[tri(i, k)] : zconj(L[tri(k, i)]);
}
__device__ inline double wave_sum(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}
// (row, column) of entry q of a packed lower triangle
__device__ inline void tri_rc(int q, int &i, int &k) {
    int r = (int)((sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
    while (r * (r + 1) / 2 > q) --r;
    while ((r + 1) * (r + 2) / 2 <= q) ++r;
    i = r;
    k = q - r * (r + 1) / 2;
}
__host__ __device__ inline int refl_off(int k, int N) { return k * (N - 1) - k * (k - 1) / 2; }

template <int NT>
__global__ __launch_bounds__(NT) void tridiag_ql_kernel(int N, const double2 *__restrict__ Ain, int64_t lda,
                                                        double2 *__restrict__ hv, double *__restrict__ zg,
                                                        int *__restrict__ rank, double *__restrict__ lam, int key,
                                                        double ref, int *__restrict__ info) {
    extern __shared__ unsigned char smem_raw[];
    double2 *L = reinterpret_cast<double2 *>(smem_raw);     // packed lower triangle of A
    double *Zt = reinterpret_cast<double *>(smem_raw);      // afterwards: Zt[i N + r] = Z[r][i]
    __shared__ double2 v[kLdsMaxN], w[kLdsMaxN];
    __shared__ double d[kLdsMaxN], e[kLdsMaxN], cs[kLdsMaxN], sn[kLdsMaxN];
    __shared__ double2 sc[3][2];                            // tau, 1/(alpha - beta), w correction; by parity of k
    __shared__ int ctl[2];
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

    // 1. Householder reduction
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
                const double2 al = L[tri(k + 1, k)];
                double2 tau = make_double2(0.0, 0.0), scl = make_double2(0.0, 0.0);
                double beta = al.x;
                if (s2 > 0.0 || al.y != 0.0) {
                    const double nrm = sqrt(al.x * al.x + al.y * al.y + s2);
                    beta = al.x >= 0.0 ? -nrm : nrm;
                    tau = make_double2((beta - al.x) / beta, -al.y / beta);
                    const double2 den = make_double2(al.x - beta, al.y);
                    const double dd = den.x * den.x + den.y * den.y;
                    scl = make_double2(den.x / dd, -den.y / dd);
                }
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
        // w = tau A22 v, eight lanes per row
        {
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
            t.x = wave_sum(t.x);
            t.y = wave_sum(t.y);
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
    __syncthreads();

    // 2. implicit QL; lane 0 carries (l, iter) from sweep to sweep
    int l = 0, iter = 0, maxiter = 0;
    bool fail = false;
    for (;;) {
        if (tid == 0) {
            int msweep = -1, nrot = 0;
            while (l < N) {
                int m = l;
                for (; m < N - 1; ++m) {
                    const double dd = fabs(d[m]) + fabs(d[m + 1]);
                    if (fabs(e[m]) <= DBL_EPSILON * dd) break;
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
                double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                double r = hypot(g, 1.0);
                g = d[m] - d[l] + e[l] / (g + copysign(r, g));
                double s = 1.0, c = 1.0, p = 0.0;
                bool split = false;
                for (int i = m - 1; i >= l; --i) {
                    const double f = s * e[i], b = c * e[i];
                    r = hypot(f, g);
                    e[i + 1] = r;
                    if (r == 0.0) {                          // T splits: restart on the shorter block
                        d[i + 1] -= p;
                        e[m] = 0.0;
                        split = true;
                        break;
                    }
                    s = f / r;
                    c = g / r;
                    g = d[i + 1] - p;
                    r = (d[i] - g) * s + 2.0 * c * b;
                    p = s * r;
                    d[i + 1] = g + p;
                    g = c * r - b;
                    cs[nrot] = c;
                    sn[nrot] = s;
                    ++nrot;
                }
                if (!split) {
                    d[l] -= p;
                    e[l] = g;
                    e[m] = 0.0;
                }
                msweep = m;
                break;
            }
            ctl[0] = msweep;
            ctl[1] = nrot;
        }
        __syncthreads();
        const int msweep = ctl[0], nrot = ctl[1];
        if (msweep < 0) break;
        if (tid < N && nrot > 0) {
            // rotation t mixes columns (i, i+1), i = msweep - 1 - t; carry holds column i+1
            double carry = Zt[msweep * N + tid];
            for (int t = 0; t < nrot; ++t) {
                const int i = msweep - 1 - t;
                const double zi = Zt[i * N + tid];
                Zt[(i + 1) * N + tid] = sn[t] * zi + cs[t] * carry;
                carry = cs[t] * zi - sn[t] * carry;
            }
            Zt[(msweep - nrot) * N + tid] = carry;
        }
        __syncthreads();
    }

    // 3. order, eigenvalues, tridiagonal eigenvectors
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
    for (int q = tid; q < N * N; q += NT) zg[q] = Zt[q];
    if (tid == 0 && info) info[0] = fail ? -1 : maxiter;
}

// One wave per eigenvector, NW waves per workgroup; all reflectors staged in LDS.
template <int NW>
__global__ __launch_bounds__(64 * NW) void backtransform_kernel(int N, const double2 *__restrict__ hv,
                                                                const double *__restrict__ zg,
                                                                const int *__restrict__ rank,
                                                                double2 *__restrict__ R) {
    extern __shared__ unsigned char smem_raw[];
    double2 *sv = reinterpret_cast<double2 *>(smem_raw);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int tau_off = N * (N - 1) / 2;
    for (int q = tid; q < tau_off + N - 1; q += 64 * NW) sv[q] = hv[q];
    __syncthreads();
    constexpr int Q = (kLdsMaxN + 63) / 64;
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
        double2 s = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int r = lane + 64 * q;
            if (r > k && r < N) s = zfma(zconj(sv[off + r]), y[q], s);
        }
        s.x = wave_sum(s.x);
        s.y = wave_sum(s.y);
        const double2 ts = zmul(tk, s);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int r = lane + 64 * q;
            if (r > k && r < N) {
                const double2 u = zmul(ts, sv[off + r]);
                y[q].x -= u.x;
                y[q].y -= u.y;
            }
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

void dense_eigh(int N, const void *A, int64_t lda, void *work_a, void *work_v, double *lam, void *R, int key,
                double ref, int *info, hipStream_t st) {
    PW_CHECK(N >= 1 && N <= 1024, PW_EUNSUPPORTED, "dense eigensolver limited to 1 <= N <= 1024");
    if (N <= kLdsMaxN) {
        // work_a: reflectors and taus (N (N + 1) / 2 complex); work_v: Z (N^2 real) then the ranks
        double2 *hv = (double2 *)work_a;
        double *zg = (double *)work_v;
        int *rank = (int *)(zg + (size_t)N * N);
        const size_t b1 = std::max((size_t)N * (N + 1) / 2 * sizeof(double2), (size_t)N * N * sizeof(double));
        static size_t attr1 = 64 * 1024, attr2 = 64 * 1024;
        lds_limit(reinterpret_cast<const void *>(tridiag_ql_kernel<1024>), b1, attr1);
        hipLaunchKernelGGL(tridiag_ql_kernel<1024>, dim3(1), dim3(1024), b1, st, N, (const double2 *)A, lda, hv,
                           zg, rank, lam, key, ref, info);
        PW_LAUNCH_CHECK();
        const size_t b2 = std::max<size_t>(1, (size_t)N * (N - 1) / 2 + N - 1) * sizeof(double2);
        lds_limit(reinterpret_cast<const void *>(backtransform_kernel<kBackNW>), b2, attr2);
        hipLaunchKernelGGL(backtransform_kernel<kBackNW>, dim3((N + kBackNW - 1) / kBackNW), dim3(64 * kBackNW), b2,
                           st, N, (const double2 *)hv, (const double *)zg, (const int *)rank, (double2 *)R);
        PW_LAUNCH_CHECK();
        return;
    }
    const size_t lds = 512 * (2 * sizeof(int) + 2 * sizeof(double) + sizeof(double2));
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(1024), lds, st, N, (const double2 *)A, lda, (double2 *)work_a,
                       (double2 *)work_v, lam, (double2 *)R, key, ref, 25, 1e-13, info);
    PW_LAUNCH_CHECK();
}

}  // namespace pw
