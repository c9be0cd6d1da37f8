// Small dense FP64 linear algebra on the GPU for the block solver.
//
//   chol_inv_kernel : S = L L^H (Cholesky), T = conj(L^{-1}), so that the band-major
//                     block Psi' = T . Psi is orthonormal (Gram/Cholesky step).
//   jacobi_kernel   : Hermitian eigensolver (cyclic Jacobi, round-robin parallel
//                     ordering) for the Rayleigh-Ritz subspace step; outputs the
//                     eigenvalues and the band-major rotation R with Psi' = R . Psi.
// Both run as one workgroup on matrices held in global memory (N <= 1024); they
// are O(N^3) on N x N matrices and off the O(N^2 npw) critical path.
#include "common.h"

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
constexpr int kLdsPairs = kLdsMaxN / 2;

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
// Hermitian Jacobi for N <= 128 with the packed lower triangle of A in LDS and
// the eigenvectors as rows of Vt (Vt[i][r] = V[r][i]) in global memory.  In a
// round the N/2 disjoint rotations J act at once, A <- J^H A J: every 2 x 2 block
// of A between two pairs (r, s) x (p, q) becomes U_rs^H B U_pq, so one pass over
// the blocks does both sides.  Same outputs as jacobi_kernel.
// ---------------------------------------------------------------------------
__device__ inline double2 lds_get(const double2 *L, int i, int k) {
    return i >= k ? L[tri(i, k)] : zconj(L[tri(k, i)]);
}
__device__ inline void lds_put(double2 *L, int i, int k, double2 v) {
    if (i >= k) L[tri(i, k)] = v;
    else L[tri(k, i)] = zconj(v);
}

template <int NT>
__global__ __launch_bounds__(NT) void jacobi_lds_kernel(int N, const double2 *__restrict__ Ain, int64_t lda,
                                                        double2 *__restrict__ Vt, double *__restrict__ lam,
                                                        double2 *__restrict__ R, int key, double ref, int max_sweeps,
                                                        double tol, int *__restrict__ info) {
    extern __shared__ unsigned char smem_raw[];
    double2 *L = reinterpret_cast<double2 *>(smem_raw);            // packed lower triangle
    __shared__ int pp[kLdsPairs], qq[kLdsPairs];
    __shared__ double cs[kLdsPairs], sn[kLdsPairs];
    __shared__ double2 ph[kLdsPairs];
    __shared__ double red[NT];
    __shared__ int sweeps_done;
    const int tid = threadIdx.x;
    const int Ne = N + (N & 1);
    const int npair = Ne / 2;
    for (int i = 0; i < N; ++i)
        for (int k = tid; k <= i; k += NT) {
            const double2 a = Ain[(int64_t)i * lda + k], b = Ain[(int64_t)k * lda + i];
            L[tri(i, k)] = make_double2(0.5 * (a.x + b.x), i == k ? 0.0 : 0.5 * (a.y - b.y));
        }
    for (int e = tid; e < N * N; e += NT) Vt[e] = make_double2((e / N) == (e % N) ? 1.0 : 0.0, 0.0);
    if (tid == 0) sweeps_done = 0;
    __syncthreads();
    double prev_offs = INFINITY;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int e = tid; e < N * (N + 1) / 2; e += NT) {
            // row of packed index e
            int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
            while (i * (i + 1) / 2 > e) --i;
            while ((i + 1) * (i + 2) / 2 <= e) ++i;
            const int k = e - i * (i + 1) / 2;
            const double2 a = L[e];
            if (k != i) off += 2.0 * (a.x * a.x + a.y * a.y);
            else dia += a.x * a.x;
        }
        red[tid] = off;
        __syncthreads();
        for (int s = NT / 2; s > 0; s >>= 1) { if (tid < s) red[tid] += red[tid + s]; __syncthreads(); }
        const double offs = red[0];
        __syncthreads();
        red[tid] = dia;
        __syncthreads();
        for (int s = NT / 2; s > 0; s >>= 1) { if (tid < s) red[tid] += red[tid + s]; __syncthreads(); }
        const double dias = red[0];
        __syncthreads();
        const double tot = dias + offs;
        if (offs <= tol * tol * tot || offs == 0.0) break;
        if (sweep > 0 && offs <= 1e-28 * tot && offs >= 0.5 * prev_offs) break;   // rounding floor
        prev_offs = offs;
        if (tid == 0) sweeps_done = sweep + 1;
        for (int r = 0; r < Ne - 1; ++r) {
            if (tid < npair) {
                const int k = tid;
                int p, q;
                if (k == 0) { p = r; q = Ne - 1; }
                else { p = (r + k) % (Ne - 1); q = (r - k + Ne - 1) % (Ne - 1); }
                if (p > q) { int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                double2 e = make_double2(1.0, 0.0);
                if (q < N) {
                    const double app = L[tri(p, p)].x, aqq = L[tri(q, q)].x;
                    const double2 apq = zconj(L[tri(q, p)]);
                    const double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
                    if (mag > 0.0) {
                        const double tau = (aqq - app) / (2.0 * mag);
                        const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                        e = make_double2(apq.x / mag, -apq.y / mag);    // exp(-i phi)
                    }
                }
                pp[k] = p; qq[k] = q; cs[k] = c; sn[k] = s; ph[k] = e;
            }
            __syncthreads();
            // eigenvector rows, first half: Vt[p] <- c Vt[p] - s e Vt[q], Vt[q] <- s Vt[p] + c e Vt[q].
            // Each element is touched once per round, so every load is issued here,
            // ahead of the LDS block updates, and the stores follow them.
            constexpr int MAXIT = (kLdsPairs * kLdsMaxN + NT - 1) / NT;
            double2 vp[MAXIT], vq[MAXIT];
#pragma unroll
            for (int it = 0; it < MAXIT; ++it) {
                const int w = tid + it * NT;
                vp[it] = vq[it] = make_double2(0.0, 0.0);
                if (w < npair * N) {
                    const int k = w / N, row = w - k * N;
                    const int p = pp[k], q = qq[k];
                    if (q < N && sn[k] != 0.0) {
                        vp[it] = Vt[(int64_t)p * N + row];
                        vq[it] = Vt[(int64_t)q * N + row];
                    }
                }
            }
            // blocks (k1 <= k2): B = A[{r1, s1}][{p2, q2}] <- U1^H B U2, U = [[c, s], [-e s, e c]]
            for (int w = tid; w < npair * npair; w += NT) {
                const int k1 = w / npair, k2 = w - k1 * npair;
                if (k1 > k2) continue;
                const int i0 = pp[k1], i1 = qq[k1], j0 = pp[k2], j1 = qq[k2];
                const double c1 = cs[k1], s1 = sn[k1], c2 = cs[k2], s2 = sn[k2];
                const double2 e1 = ph[k1], e2 = ph[k2];
                if (s1 == 0.0 && s2 == 0.0) continue;
                const bool v1 = i1 < N, v2 = j1 < N;
                double2 b00 = lds_get(L, i0, j0);
                double2 b01 = v2 ? lds_get(L, i0, j1) : make_double2(0.0, 0.0);
                double2 b10 = v1 ? lds_get(L, i1, j0) : make_double2(0.0, 0.0);
                double2 b11 = (v1 && v2) ? lds_get(L, i1, j1) : make_double2(0.0, 0.0);
                // left: rows (i0, i1) <- U1^H rows: new0 = c1 b0 - s1 conj(e1) b1 ; new1 = s1 b0 + c1 conj(e1) b1
                const double2 ce1 = zconj(e1);
                double2 t00 = zmul(ce1, b10), t01 = zmul(ce1, b11);
                double2 l00 = make_double2(c1 * b00.x - s1 * t00.x, c1 * b00.y - s1 * t00.y);
                double2 l01 = make_double2(c1 * b01.x - s1 * t01.x, c1 * b01.y - s1 * t01.y);
                double2 l10 = make_double2(s1 * b00.x + c1 * t00.x, s1 * b00.y + c1 * t00.y);
                double2 l11 = make_double2(s1 * b01.x + c1 * t01.x, s1 * b01.y + c1 * t01.y);
                // right: cols (j0, j1) <- cols U2: new0 = c2 a0 - s2 e2 a1 ; new1 = s2 a0 + c2 e2 a1
                double2 u0 = zmul(e2, l01), u1 = zmul(e2, l11);
                double2 r00 = make_double2(c2 * l00.x - s2 * u0.x, c2 * l00.y - s2 * u0.y);
                double2 r01 = make_double2(s2 * l00.x + c2 * u0.x, s2 * l00.y + c2 * u0.y);
                double2 r10 = make_double2(c2 * l10.x - s2 * u1.x, c2 * l10.y - s2 * u1.y);
                double2 r11 = make_double2(s2 * l10.x + c2 * u1.x, s2 * l10.y + c2 * u1.y);
                if (k1 == k2) {
                    // diagonal block: the rotation zeroes the off-diagonal pair
                    L[tri(i0, i0)] = make_double2(r00.x, 0.0);
                    if (v1) {
                        L[tri(i1, i1)] = make_double2(r11.x, 0.0);
                        L[tri(i1, i0)] = make_double2(0.0, 0.0);
                    }
                } else {
                    lds_put(L, i0, j0, r00);
                    if (v2) lds_put(L, i0, j1, r01);
                    if (v1) lds_put(L, i1, j0, r10);
                    if (v1 && v2) lds_put(L, i1, j1, r11);
                }
            }
            // eigenvector rows, second half: combine and store
#pragma unroll
            for (int it = 0; it < MAXIT; ++it) {
                const int w = tid + it * NT;
                if (w < npair * N) {
                    const int k = w / N, row = w - k * N;
                    const int p = pp[k], q = qq[k];
                    if (q < N && sn[k] != 0.0) {
                        const double c = cs[k], s = sn[k];
                        const double2 ev = zmul(ph[k], vq[it]);
                        Vt[(int64_t)p * N + row] = make_double2(c * vp[it].x - s * ev.x, c * vp[it].y - s * ev.y);
                        Vt[(int64_t)q * N + row] = make_double2(s * vp[it].x + c * ev.x, s * vp[it].y + c * ev.y);
                    }
                }
            }
            __syncthreads();
        }
    }
    double *dval = red;
    for (int i = tid; i < N; i += NT) dval[i] = L[tri(i, i)].x;
    __syncthreads();
    for (int i = tid; i < N; i += NT) {
        const double li = dval[i];
        const double ki = key ? fabs(li - ref) : li;
        int rank = 0;
        for (int j = 0; j < N; ++j) {
            const double lj = dval[j];
            const double kj = key ? fabs(lj - ref) : lj;
            if (kj < ki || (kj == ki && (lj < li || (lj == li && j < i)))) ++rank;
        }
        lam[rank] = li;
        for (int j = 0; j < N; ++j) R[(int64_t)rank * N + j] = Vt[(int64_t)i * N + j];
    }
    if (tid == 0 && info) info[0] = sweeps_done;
}

// ---------------------------------------------------------------------------
// host wrappers
// ---------------------------------------------------------------------------
void chol_inv(int N, const void *S, int64_t lds, void *work, void *T, int *status, hipStream_t st) {
    if (N <= kLdsMaxN) {
        PW_CHECK(N > 0 && N < 4096, PW_EINVAL, "bad Cholesky size");   // inverse keeps one band per thread
        const size_t bytes = (size_t)N * (N + 1) / 2 * sizeof(double2);
        static size_t attr_bytes = 64 * 1024;   // default dynamic LDS limit
        if (bytes > attr_bytes) {
            PW_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(chol_inv_lds_kernel<1024>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
            attr_bytes = bytes;
        }
        hipLaunchKernelGGL(chol_inv_lds_kernel<1024>, dim3(1), dim3(1024), bytes, st, N, (const double2 *)S, lds,
                           (double2 *)T, status);
    } else {
        hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(1024), 0, st, N, (const double2 *)S, lds,
                           (double2 *)work, (double2 *)T, status);
    }
    PW_LAUNCH_CHECK();
}

void jacobi_eigh(int N, const void *A, int64_t lda, void *work_a, void *work_v, double *lam, void *R, int key,
                 double ref, int *info, hipStream_t st) {
    PW_CHECK(N <= 1024, PW_EUNSUPPORTED, "Jacobi eigensolver limited to N <= 1024");
    if (N <= kLdsMaxN) {
        const size_t bytes = (size_t)N * (N + 1) / 2 * sizeof(double2);
        static size_t attr_bytes = 64 * 1024;
        if (bytes > attr_bytes) {
            PW_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(jacobi_lds_kernel<512>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
            attr_bytes = bytes;
        }
        hipLaunchKernelGGL(jacobi_lds_kernel<512>, dim3(1), dim3(512), bytes, st, N, (const double2 *)A, lda,
                           (double2 *)work_v, lam, (double2 *)R, key, ref, 25, 1e-13, info);
        PW_LAUNCH_CHECK();
        return;
    }
    const size_t lds = 512 * (2 * sizeof(int) + 2 * sizeof(double) + sizeof(double2));
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(1024), lds, st, N, (const double2 *)A, lda, (double2 *)work_a,
                       (double2 *)work_v, lam, (double2 *)R, key, ref, 25, 1e-13, info);
    PW_LAUNCH_CHECK();
}

}  // namespace pw
