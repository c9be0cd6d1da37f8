// Chebyshev filter diagonalisation of an energy window (host control, arithmetic on the GPU).
//
// The paper generates the eigenstates near E with ChebFD (Sec. II.B, ChebFD paragraph):
// a polynomial p(H) in Chebyshev polynomials imitates a window around E, is applied to
// a block of vectors (each band independently), and a subspace diagonalisation of
// <phi_i|H|phi_j> follows; the step is repeated.  The paper gives no formulas; the
// textbook ones are used:
//   x = (H - c) / h, c = (emax + emin) / 2, h = (emax - emin) / 2 ([emin, emax] holds the spectrum)
//   window [E - w, E + w] -> [a, b]; coefficients of its indicator
//     mu_0 = (acos a - acos b) / pi, mu_k = 2 (sin(k acos a) - sin(k acos b)) / (k pi)
//   Jackson damping g_k = ((M - k + 1) cos(k q) + sin(k q) cot q) / (M + 1), q = pi / (M + 1)
//     (kernel polynomial method, Weisse et al., Rev. Mod. Phys. 78, 275 (2006))
//   p(H) v = sum_k g_k mu_k T_k(x) v, T_{k+1} = 2 x T_k - T_{k-1}: one H psi per degree.
// A step then orthonormalises the filtered block (Gram/Cholesky), diagonalises
// <phi_i|H|phi_j> (Householder + divide and conquer) and returns the Ritz values
// ascending with their residuals ||H phi_i - eps_i phi_i||.
//
// The spectral interval comes from the caller, or from pw_spectral_bounds: k steps of
// Lanczos on H from a caller-supplied start vector; the extreme Ritz values of the
// k x k tridiagonal (diagonalised by the library's dense kernel), widened by twice
// their residual bounds |beta_k s_k| and by 1% of the width.
#include <cmath>
#include <vector>

#include "kernels.h"

namespace pw {

void hpsi_any(pw_ctx *ctx, pw_dtype dt, int nb, const void *psi, int64_t ld, void *out, int64_t ldo, double shift,
              hipStream_t st);
void orthonormalize_c128(pw_ctx *ctx, int nb, void *psi, int64_t ld, void *ws, void *small, int *d_status,
                         hipStream_t st);

static std::vector<double> window_coef(double e, double w, double emin, double emax, int degree) {
    const double c = 0.5 * (emax + emin), h = 0.5 * (emax - emin);
    const double a = std::fmin(1.0, std::fmax(-1.0, (e - w - c) / h));
    const double b = std::fmin(1.0, std::fmax(-1.0, (e + w - c) / h));
    const double ta = std::acos(a), tb = std::acos(b);
    const double pi = 3.14159265358979323846;
    const double q = pi / (degree + 1);
    std::vector<double> coef(degree + 1);
    for (int k = 0; k <= degree; ++k) {
        const double mu = k == 0 ? (ta - tb) / pi : 2.0 * (std::sin(k * ta) - std::sin(k * tb)) / (k * pi);
        const double g = ((degree - k + 1) * std::cos(k * q) + std::sin(k * q) / std::tan(q)) / (degree + 1);
        coef[k] = g * mu;
    }
    return coef;
}

struct ChebBufs {
    DevBuf U, Up, T, Y;
    explicit ChebBufs(size_t blk) {
        U.alloc(blk);
        Up.alloc(blk);
        T.alloc(blk);
        Y.alloc(blk);
    }
};

// Y = p(H) psi (internal leading dimension npw); U, Up and T are scratch
static void cheb_filter(pw_ctx *ctx, int nb, const void *psi, int64_t ld, const std::vector<double> &coef, double emin,
                        double emax, ChebBufs &b, hipStream_t st) {
    const int npw = ctx->basis.npw;
    const int64_t L = npw;
    const double c = 0.5 * (emax + emin), h = 0.5 * (emax - emin);
    void *U = b.U.p, *Up = b.Up.p;
    copy_block(nb, npw, psi, ld, U, L, st);
    scale_copy(nb, npw, U, L, b.Y.p, L, coef[0], st);
    const int degree = (int)coef.size() - 1;
    for (int k = 1; k <= degree; ++k) {
        hpsi_any(ctx, PW_C128, nb, U, L, b.T.p, L, c, st);              // T = (H - c) U_k-1
        cheb_step(nb, npw, b.T.p, Up, b.Y.p, L, (k == 1 ? 1.0 : 2.0) / h, coef[k], k == 1, st);
        std::swap(U, Up);                                                // U = U_k, Up = U_k-1
    }
}

static void check_window(double e, double w, int degree, double emin, double emax) {
    PW_CHECK(std::isfinite(e) && std::isfinite(w) && std::isfinite(emin) && std::isfinite(emax), PW_ENAN,
             "non-finite window or bounds");
    PW_CHECK(emax > emin, PW_EINVAL, "emax must exceed emin");
    PW_CHECK(w > 0.0, PW_EINVAL, "half width must be positive");
    PW_CHECK(e + w > emin && e - w < emax, PW_EINVAL, "window outside [emin, emax]");
    PW_CHECK(degree >= 0 && degree <= 100000, PW_EINVAL, "degree %d outside [0, 100000]", degree);
}

}  // namespace pw

using namespace pw;

extern "C" {

pw_status pw_cheb_filter(pw_ctx *ctx, int32_t nb, const void *psi, int64_t ld, void *out, int64_t ldo, double e,
                         double half_width, int32_t degree, double emin, double emax, void *stream) {
    try {
        PW_CHECK(ctx && psi && out, PW_EINVAL, "null argument");
        PW_CHECK(ctx->flags & PW_PREP_C128, PW_EUNSUPPORTED, "the filter needs a complex128 context");
        PW_CHECK(nb >= 1 && nb <= ctx->max_bands, PW_EINVAL, "nb %d must be in [1, max_bands]", nb);
        PW_CHECK(ld >= ctx->basis.npw && ldo >= ctx->basis.npw, PW_EINVAL, "ld or ldo < npw");
        PW_CHECK(psi != out, PW_EINVAL, "psi and out must not alias");
        check_window(e, half_width, degree, emin, emax);
        hipStream_t st = (hipStream_t)stream;
        const int npw = ctx->basis.npw;
        ChebBufs b((size_t)nb * npw * 16);
        cheb_filter(ctx, nb, psi, ld, window_coef(e, half_width, emin, emax, degree), emin, emax, b, st);
        copy_block(nb, npw, b.Y.p, npw, out, ldo, st);
        PW_HIP(hipStreamSynchronize(st));
        return PW_OK;
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PW_ENOMEM;
    } catch (...) {
        set_error("unexpected exception in pw_cheb_filter");
        return PW_EINVAL;
    }
}

pw_status pw_chebfd_step(pw_ctx *ctx, int32_t nb, void *psi, int64_t ld, double e, double half_width, int32_t degree,
                         double emin, double emax, double *eig, double *resid, void *stream) {
    try {
        PW_CHECK(ctx && psi, PW_EINVAL, "null argument");
        PW_CHECK(ctx->flags & PW_PREP_C128, PW_EUNSUPPORTED, "ChebFD needs a complex128 context");
        PW_CHECK(nb >= 1 && nb <= ctx->max_bands && nb <= 1024 && nb <= ctx->basis.npw, PW_EINVAL,
                 "nb %d must be in [1, min(max_bands, 1024, npw)]", nb);
        PW_CHECK(ld >= ctx->basis.npw, PW_EINVAL, "ld < npw");
        check_window(e, half_width, degree, emin, emax);
        hipStream_t st = (hipStream_t)stream;
        const int npw = ctx->basis.npw;
        const int64_t L = npw;
        const size_t nn = (size_t)nb * nb * 16;
        ChebBufs b((size_t)nb * npw * 16);
        DevBuf small, work, vec;
        small.alloc(5 * nn + 256);
        work.alloc(dense_eigh_work_bytes(nb));
        const int nsplit = band_splits(npw);
        vec.alloc((size_t)nb * 16 + (size_t)nb * nsplit * 8);
        double *lam = vec.as<double>(), *res = lam + nb;
        const BandRed br{res + nb, nsplit};
        double2 *S = small.as<double2>(), *R = S + (size_t)nb * nb, *osmall = R + (size_t)nb * nb;
        int *d_status = (int *)((char *)small.p + 5 * nn);
        fill_zero(d_status, 256, st);
        cheb_filter(ctx, nb, psi, ld, window_coef(e, half_width, emin, emax, degree), emin, emax, b, st);
        nan_check((size_t)nb * npw * 2, b.Y.as<double>(), d_status + 8, st);
        int nan_flag = 0;
        PW_HIP(hipMemcpyAsync(&nan_flag, d_status + 8, sizeof(int), hipMemcpyDeviceToHost, st));
        PW_HIP(hipStreamSynchronize(st));
        PW_CHECK(!nan_flag, PW_ENAN, "the filtered block is not finite (is [emin, emax] the whole spectrum?)");
        // orthonormalise (T as scratch), then Rayleigh-Ritz in H
        orthonormalize_c128(ctx, nb, b.Y.p, L, b.T.p, osmall, d_status, st);
        hpsi_any(ctx, PW_C128, nb, b.Y.p, L, b.T.p, L, 0.0, st);
        zgemm_nt(nb, nb, npw, true, b.Y.p, L, b.T.p, L, 1.0, nullptr, 0.0, S, nb, false, ctx->d_partial.p, st);
        dense_eigh(nb, S, nb, work.p, lam, R, 0, 0.0, d_status + 4, st);
        zgemm_nn_launch(nb, npw, nb, R, nb, b.Y.p, L, 1.0, 0.0, b.U.p, L, st, false, ctx->rot_tune.get(nb));
        zgemm_nn_launch(nb, npw, nb, R, nb, b.T.p, L, 1.0, 0.0, b.Up.p, L, st, false, ctx->rot_tune.get(nb));
        red_resid(nb, npw, b.Up.p, b.U.p, L, lam, res, br, st);
        int h_status[12] = {0};
        std::vector<double> h_lam(nb), h_res(nb);
        PW_HIP(hipMemcpyAsync(h_status, d_status, sizeof h_status, hipMemcpyDeviceToHost, st));
        PW_HIP(hipMemcpyAsync(h_lam.data(), lam, (size_t)nb * 8, hipMemcpyDeviceToHost, st));
        PW_HIP(hipMemcpyAsync(h_res.data(), res, (size_t)nb * 8, hipMemcpyDeviceToHost, st));
        PW_HIP(hipStreamSynchronize(st));
        PW_CHECK(!h_status[0], PW_ENOTPD,
                 "the filtered block lost rank (pivot %d): too few states in the window for nb bands, or too low a "
                 "degree", h_status[0] - 1);
        copy_block(nb, npw, b.U.p, L, psi, ld, st);
        PW_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < nb; ++i) {
            if (eig) eig[i] = h_lam[i];
            if (resid) resid[i] = h_res[i];
        }
        return PW_OK;
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PW_ENOMEM;
    } catch (...) {
        set_error("unexpected exception in pw_chebfd_step");
        return PW_EINVAL;
    }
}

pw_status pw_spectral_bounds(pw_ctx *ctx, const void *v0, int32_t steps, double *emin, double *emax, void *stream) {
    try {
        PW_CHECK(ctx && v0 && emin && emax, PW_EINVAL, "null argument");
        PW_CHECK(ctx->flags & PW_PREP_C128, PW_EUNSUPPORTED, "needs a complex128 context");
        PW_CHECK(steps >= 2 && steps <= 1024 && steps <= ctx->basis.npw, PW_EINVAL,
                 "steps %d must be in [2, min(1024, npw)]", steps);
        hipStream_t st = (hipStream_t)stream;
        const int npw = ctx->basis.npw;
        const size_t vb = (size_t)npw * 16;
        DevBuf bV, bVp, bW, vec, mats, work;
        bV.alloc(vb);
        bVp.alloc(vb);
        bW.alloc(vb);
        const int nsplit = band_splits(npw);
        vec.alloc(64 + (size_t)nsplit * 8 + (size_t)steps * 8);
        double *d_s = vec.as<double>(), *d_lam = d_s + 4;
        const BandRed br{d_lam + steps, nsplit};
        auto read = [&](const double *p) {
            double v = 0;
            PW_HIP(hipMemcpyAsync(&v, p, 8, hipMemcpyDeviceToHost, st));
            PW_HIP(hipStreamSynchronize(st));
            return v;
        };
        void *V = bV.p, *Vp = bVp.p, *W = bW.p;
        band_norms(1, npw, v0, npw, d_s, br, st);
        const double n0 = read(d_s);
        PW_CHECK(n0 > 0.0 && std::isfinite(n0), PW_EINVAL, "start vector is zero or not finite");
        scale_copy(1, npw, v0, npw, V, npw, 1.0 / n0, st);
        fill_zero(Vp, vb, st);
        std::vector<double> al, be;               // be[j] couples v_j and v_j+1
        double beta = 0.0;
        for (int j = 0; j < steps; ++j) {
            hpsi_any(ctx, PW_C128, 1, V, npw, W, npw, 0.0, st);
            red_dot_re(1, npw, V, W, npw, d_s, br, st);
            const double alpha = read(d_s);
            lanczos_update(npw, W, V, Vp, alpha, beta, st);
            band_norms(1, npw, W, npw, d_s, br, st);
            beta = read(d_s);
            PW_CHECK(std::isfinite(alpha) && std::isfinite(beta), PW_ENAN, "non-finite Lanczos step %d", j);
            al.push_back(alpha);
            be.push_back(beta);
            if (beta <= 1e-12 * std::fabs(alpha) + 1e-300) break;         // invariant subspace found
            std::swap(Vp, V);
            scale_copy(1, npw, W, npw, V, npw, 1.0 / beta, st);
        }
        // Ritz values of the tridiagonal, on the GPU's dense eigensolver
        const int m = (int)al.size();
        std::vector<double> T((size_t)2 * m * m, 0.0);
        for (int i = 0; i < m; ++i) {
            T[2 * ((size_t)i * m + i)] = al[i];
            if (i + 1 < m) {
                T[2 * ((size_t)i * m + i + 1)] = be[i];
                T[2 * ((size_t)(i + 1) * m + i)] = be[i];
            }
        }
        mats.alloc((size_t)2 * m * m * 16 + 64);
        work.alloc(dense_eigh_work_bytes(m));
        double2 *dT = mats.as<double2>(), *dR = dT + (size_t)m * m;
        int *info = (int *)(dR + (size_t)m * m);
        PW_HIP(hipMemcpyAsync(dT, T.data(), T.size() * 8, hipMemcpyHostToDevice, st));
        fill_zero(info, 16, st);
        dense_eigh(m, dT, m, work.p, d_lam, dR, 0, 0.0, info, st);
        std::vector<double> lam(m), R((size_t)2 * m * m);
        PW_HIP(hipMemcpyAsync(lam.data(), d_lam, (size_t)m * 8, hipMemcpyDeviceToHost, st));
        PW_HIP(hipMemcpyAsync(R.data(), dR, R.size() * 8, hipMemcpyDeviceToHost, st));
        PW_HIP(hipStreamSynchronize(st));
        // residual bound of a Ritz pair: |beta_m| times the last component of its vector
        const double bm = be[m - 1];
        auto rb = [&](int i) { return bm * std::hypot(R[2 * ((size_t)i * m + m - 1)], R[2 * ((size_t)i * m + m - 1) + 1]); };
        const double width = lam[m - 1] - lam[0];
        *emin = lam[0] - 2.0 * rb(0) - 0.01 * width;
        *emax = lam[m - 1] + 2.0 * rb(m - 1) + 0.01 * width;
        return PW_OK;
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PW_ENOMEM;
    } catch (...) {
        set_error("unexpected exception in pw_spectral_bounds");
        return PW_EINVAL;
    }
}

}  // extern "C"
