// Wave-function interpolation between two k-points (host control, arithmetic on the GPU).
//
// Sec. II.C: with orthonormal eigenstates psi_i(k1), psi_i(k2) and their energies,
// H(k) ~ alpha H(k1) + (1 - alpha) H(k2), alpha = (k - k2) / (k1 - k2), and in the
// basis psi_i(k1)
//   H_ij(k) = alpha eps_i(k1) delta_ij + (1 - alpha) sum_m conj(U_im) U_jm eps_m(k2),
// U the row-wise Gram-Schmidt orthonormalisation of S_ij = <psi_j(k2)|psi_i(k1)>.
// Its eigenvectors c give psi(k) = alpha sum_j c_j psi_j(k1) + (1 - alpha) sum_jl c_j U_jl psi_l(k2).
//
// On the GPU: psi(k2) is gathered onto the k1 sphere (coefficients missing there are
// zero), S is one split-K NT GEMM over the plane waves, the Gram-Schmidt is the
// Cholesky factorisation of the rows' Gram matrix (U = L^-1 S, the same triangular
// recurrence), H(k) is built by a small kernel and diagonalised by the dense
// eigensolver, and psi(k) takes two NN GEMMs after gathering both blocks onto the
// sphere of k.
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "kernels.h"

namespace pw {

// for each plane wave of `to`, its index in `from` (-1 if outside that sphere)
static std::vector<int32_t> sphere_map(const Basis &from, const Basis &to) {
    auto key = [](const int32_t *m) {
        return ((uint64_t)(uint32_t)(m[0] + (1 << 20)) << 42) | ((uint64_t)(uint32_t)(m[1] + (1 << 20)) << 21) |
               (uint64_t)(uint32_t)(m[2] + (1 << 20));
    };
    std::unordered_map<uint64_t, int32_t> idx;
    idx.reserve((size_t)from.npw * 2);
    for (int g = 0; g < from.npw; ++g) idx[key(&from.miller[3 * (size_t)g])] = g;
    std::vector<int32_t> map(to.npw);
    for (int g = 0; g < to.npw; ++g) {
        auto it = idx.find(key(&to.miller[3 * (size_t)g]));
        map[g] = it == idx.end() ? -1 : it->second;
    }
    return map;
}

static bool same_cell(const pw_cell &a, const pw_cell &b) {
    for (int i = 0; i < 3; ++i)
        if (a.n[i] != b.n[i] || a.cell[i] != b.cell[i]) return false;
    return a.ecut == b.ecut;
}

}  // namespace pw

using namespace pw;

extern "C" {

pw_status pw_kinterp(pw_ctx *ctx1, pw_ctx *ctx2, pw_ctx *ctxk, double alpha, int32_t n, const void *psi1, int64_t ld1,
                     const double *eps1, const void *psi2, int64_t ld2, const double *eps2, double *eps_out,
                     void *psi_out, int64_t ldo, void *stream) {
    try {
        PW_CHECK(ctx1 && ctx2 && ctxk && psi1 && psi2 && eps1 && eps2 && eps_out, PW_EINVAL, "null argument");
        PW_CHECK(same_cell(ctx1->cell, ctx2->cell) && same_cell(ctx1->cell, ctxk->cell), PW_EINVAL,
                 "the three contexts must share cell, grid and cutoff");
        const int np1 = ctx1->basis.npw, np2 = ctx2->basis.npw, npk = ctxk->basis.npw;
        PW_CHECK(n >= 1 && n <= 1024 && n <= np1 && n <= np2, PW_EINVAL, "n %d must be in [1, min(1024, npw)]", n);
        PW_CHECK(ld1 >= np1 && ld2 >= np2, PW_EINVAL, "ld1 or ld2 smaller than its sphere");
        PW_CHECK(!psi_out || ldo >= npk, PW_EINVAL, "ldo < npw of the k context");
        PW_CHECK(psi_out != psi1 && psi_out != psi2, PW_EINVAL, "psi_out must not alias psi1 or psi2");
        PW_CHECK(std::isfinite(alpha), PW_ENAN, "non-finite alpha");
        for (int i = 0; i < n; ++i)
            PW_CHECK(std::isfinite(eps1[i]) && std::isfinite(eps2[i]), PW_ENAN, "non-finite energy %d", i);
        hipStream_t st = (hipStream_t)stream;
        const size_t nn = (size_t)n * n;
        // device work: maps, gathered blocks, n x n matrices, eigensolver work, split-K partials
        const std::vector<int32_t> m21 = sphere_map(ctx2->basis, ctx1->basis);
        DevBuf dmap, P2, mats, work, part, vec;
        dmap.alloc((size_t)(np1 + 2 * npk) * 4);
        P2.alloc((size_t)n * np1 * 16);
        mats.alloc(7 * nn * 16 + 256);
        work.alloc(std::max(dense_eigh_work_bytes(n), chol_inv_work_bytes(n)));
        part.alloc(std::max(nt_partial_bytes(n, n, np1), nt_partial_bytes(n, n, n)));
        vec.alloc((size_t)3 * n * 8);
        double2 *S = mats.as<double2>(), *G = S + nn, *T = G + nn, *U = T + nn, *Hk = U + nn, *R = Hk + nn,
                *RU = R + nn;
        int *d_status = (int *)(RU + nn);
        double *d_e1 = vec.as<double>(), *d_e2 = d_e1 + n, *d_lam = d_e2 + n;
        int32_t *d_m21 = dmap.as<int32_t>();
        PW_HIP(hipMemcpyAsync(d_m21, m21.data(), (size_t)np1 * 4, hipMemcpyHostToDevice, st));
        PW_HIP(hipMemcpyAsync(d_e1, eps1, (size_t)n * 8, hipMemcpyHostToDevice, st));
        PW_HIP(hipMemcpyAsync(d_e2, eps2, (size_t)n * 8, hipMemcpyHostToDevice, st));
        fill_zero(d_status, 256, st);
        // S[i][j] = <psi_j(k2)|psi_i(k1)> on the k1 sphere
        gather_pw(n, np1, psi2, ld2, d_m21, P2.p, np1, st);
        zgemm_nt(n, n, np1, true, P2.p, np1, psi1, ld1, 1.0, nullptr, 0.0, S, n, true, part.p, st);
        // Gram-Schmidt of the rows of S: G[a][b] = sum_j conj(S_aj) S_bj = L L^H, U = conj(L^-1) . S
        zgemm_nt(n, n, n, true, S, n, S, n, 1.0, nullptr, 0.0, G, n, false, part.p, st);
        chol_inv(n, G, n, work.p, T, d_status, st);   // the eigensolver's work is free here
        int chol = 0;
        PW_HIP(hipMemcpyAsync(&chol, d_status, sizeof(int), hipMemcpyDeviceToHost, st));
        PW_HIP(hipStreamSynchronize(st));
        PW_CHECK(!chol, PW_ENOTPD, "the overlap rows are linearly dependent (pivot %d)", chol - 1);
        zgemm_nn_launch(n, n, n, T, n, S, n, 1.0, 0.0, U, n, st);
        kinterp_hk(n, alpha, d_e1, d_e2, U, Hk, st);
        dense_eigh(n, Hk, n, work.p, d_lam, R, 0, 0.0, d_status + 4, st);
        if (psi_out) {
            const std::vector<int32_t> m1k = sphere_map(ctx1->basis, ctxk->basis);
            const std::vector<int32_t> m2k = sphere_map(ctx2->basis, ctxk->basis);
            int32_t *d_m1k = d_m21 + np1, *d_m2k = d_m1k + npk;
            PW_HIP(hipMemcpyAsync(d_m1k, m1k.data(), (size_t)npk * 4, hipMemcpyHostToDevice, st));
            PW_HIP(hipMemcpyAsync(d_m2k, m2k.data(), (size_t)npk * 4, hipMemcpyHostToDevice, st));
            DevBuf Q1, Q2;
            Q1.alloc((size_t)n * npk * 16);
            Q2.alloc((size_t)n * npk * 16);
            gather_pw(n, npk, psi1, ld1, d_m1k, Q1.p, npk, st);
            gather_pw(n, npk, psi2, ld2, d_m2k, Q2.p, npk, st);
            zgemm_nn_launch(n, n, n, R, n, U, n, 1.0, 0.0, RU, n, st);
            zgemm_nn_launch(n, npk, n, R, n, Q1.p, npk, alpha, 0.0, psi_out, ldo, st);
            zgemm_nn_launch(n, npk, n, RU, n, Q2.p, npk, 1.0 - alpha, 1.0, psi_out, ldo, st);
            PW_HIP(hipStreamSynchronize(st));          // the maps and gathered blocks are freed on return
        }
        PW_HIP(hipMemcpyAsync(eps_out, d_lam, (size_t)n * 8, hipMemcpyDeviceToHost, st));
        PW_HIP(hipStreamSynchronize(st));
        return PW_OK;
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PW_ENOMEM;
    } catch (...) {
        set_error("unexpected exception in pw_kinterp");
        return PW_EINVAL;
    }
}

}  // extern "C"
