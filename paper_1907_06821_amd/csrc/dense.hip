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
        if (offs <= tol * tol * dias || offs == 0.0) break;
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
// host wrappers
// ---------------------------------------------------------------------------
void chol_inv(int N, const void *S, int64_t lds, void *work, void *T, int *status, hipStream_t st) {
    hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(1024), 0, st, N, (const double2 *)S, lds, (double2 *)work,
                       (double2 *)T, status);
    PW_LAUNCH_CHECK();
}

void jacobi_eigh(int N, const void *A, int64_t lda, void *work_a, void *work_v, double *lam, void *R, int key,
                 double ref, int *info, hipStream_t st) {
    PW_CHECK(N <= 1024, PW_EUNSUPPORTED, "Jacobi eigensolver limited to N <= 1024");
    const size_t lds = 512 * (2 * sizeof(int) + 2 * sizeof(double) + sizeof(double2));
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(1024), lds, st, N, (const double2 *)A, lda, (double2 *)work_a,
                       (double2 *)work_v, lam, (double2 *)R, key, ref, 30, 1e-15, info);
    PW_LAUNCH_CHECK();
}

}  // namespace pw
