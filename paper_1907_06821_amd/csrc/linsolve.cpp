// Folded linear equation of the system states (host control, all arithmetic on the GPU).
//
// The system states obey (H - E) psi = w (Sec. II.A); H - E is indefinite, so the
// equation is folded to (H - E)^2 psi = (H - E) w and solved by PCG (Sec. II.B,
// folded equation and functional F).  Each column (source) runs its own PCG:
//   YP = (H - E) P, AP = (H - E) YP                  (two H psi)
//   alpha = <r, z> / ||YP||^2                        (||YP||^2 = <p, A p>)
//   X += alpha P, Y += alpha YP, R -= alpha AP       (Y = (H - E) X carried along)
//   Z = K R, beta = <r', z'> / <r, z>, P = Z + beta P
// The paper's error ||(H - E) x - w|| is ||Y - W||, read by the host every
// check_every iterations; the final value comes from a fresh H psi.  The
// check_every iterations between two reads are recorded once into a HIP graph and
// replayed (the step lengths live on the device and the blocks never move).
//
// K is the paper's M(G) or the eigenstate-augmented M' (Sec. II.B, M' equation)
// in its Hermitian form
//   M' r = (1 - P) M (1 - P) r + sum_i phi_i <phi_i|r> / d_i,  d_i = (eps_i - E)^2 + Delta_i^2,
// applied as C = Phi^H R (split-K NT GEMM), U = Phi C (NN GEMM), Z = M o (R - U),
// D = Phi^H Z, E = C / d - D, Z += Phi E: the two projections of (1 - P) M (1 - P)
// share the first product with the eigenstate term.
#include <chrono>
#include <cmath>
#include <vector>

#include "kernels.h"

namespace pw {

namespace {
struct SegmentGraph {
    hipStream_t cap = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    ~SegmentGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (g) (void)hipGraphDestroy(g);
        if (cap) (void)hipStreamDestroy(cap);
    }
};
}  // namespace

void hpsi_any(pw_ctx *ctx, pw_dtype dt, int nb, const void *psi, int64_t ld, void *out, int64_t ldo, double shift,
              hipStream_t st);

pw_status folded_linsolve(pw_ctx *ctx, double E, int nrhs, const void *w, int64_t ldw, void *psi, int64_t ld,
                          int nev, const void *phi, int64_t ldphi, const double *eps, const double *delta,
                          double *resid, const pw_lin_opts &o, pw_lin_stats *stats, hipStream_t st) {
    const auto t0 = std::chrono::steady_clock::now();
    const int npw = ctx->basis.npw;
    const int64_t L = npw;
    const size_t blk = (size_t)nrhs * npw * 16;
    DevBuf bX, bY, bR, bP, bYP, bAP, bZ, bU;
    DevBuf *blocks[] = {&bX, &bY, &bR, &bP, &bYP, &bAP, &bZ, &bU};
    for (DevBuf *d : blocks) d->alloc(blk);
    void *X = bX.p, *Y = bY.p, *R = bR.p, *P = bP.p, *YP = bYP.p, *AP = bAP.p, *Z = bZ.p, *U = bU.p;
    const int nsplit = band_splits(npw);
    DevBuf red, vec;
    red.alloc((size_t)nrhs * nsplit * 8);
    vec.alloc((size_t)nrhs * 4 * 8);
    double *rz = vec.as<double>(), *alpha = rz + nrhs, *beta = rz + 2 * nrhs, *err = rz + 3 * nrhs;
    const BandRed br{red.as<double>(), nsplit};
    const double *kin = ctx->d_kin.as<double>();
    const double de2 = o.delta_e * o.delta_e;

    const bool aug = o.precond == 1;
    DevBuf coefs, part, invd;
    double2 *Cm = nullptr, *Dm = nullptr, *Em = nullptr;
    if (aug) {
        const size_t nc = (size_t)nrhs * nev;
        coefs.alloc(3 * nc * 16);
        Cm = coefs.as<double2>();
        Dm = Cm + nc;
        Em = Dm + nc;
        part.alloc(nt_partial_bytes(nev, nrhs, npw));
        std::vector<double> h_invd(nev);
        for (int i = 0; i < nev; ++i) {
            const double d = (eps[i] - E) * (eps[i] - E) + delta[i] * delta[i];
            PW_CHECK(d > 0.0 && std::isfinite(d), PW_EINVAL,
                     "eigenpair %d: (eps - E)^2 + Delta^2 must be positive and finite", i);
            h_invd[i] = 1.0 / d;
        }
        invd.alloc((size_t)nev * 8);
        PW_HIP(hipMemcpyAsync(invd.p, h_invd.data(), (size_t)nev * 8, hipMemcpyHostToDevice, st));
        PW_HIP(hipStreamSynchronize(st));
    }
    hipStream_t cur = st;   // the launch stream: st, or the capture stream while a segment is recorded
    // Z = K R, then rz <- <R, Z> and beta = rz_new / rz_old
    auto precondition = [&](bool first) {
        const hipStream_t st = cur;
        if (!aug) {
            lin_mdiag(nrhs, npw, R, nullptr, Z, L, kin, E, de2, rz, beta, first, true, br, st);
            return;
        }
        zgemm_nt(nev, nrhs, npw, true, phi, ldphi, R, L, 1.0, nullptr, 0.0, Cm, nev, true, part.p, st);
        zgemm_nn_launch(nrhs, npw, nev, Cm, nev, phi, ldphi, 1.0, 0.0, U, L, st);
        lin_mdiag(nrhs, npw, R, U, Z, L, kin, E, de2, rz, beta, first, false, br, st);
        zgemm_nt(nev, nrhs, npw, true, phi, ldphi, Z, L, 1.0, nullptr, 0.0, Dm, nev, true, part.p, st);
        lin_coef(nrhs, nev, Cm, Dm, invd.as<double>(), Em, st);
        zgemm_nn_launch(nrhs, npw, nev, Em, nev, phi, ldphi, 1.0, 1.0, Z, L, st);
        lin_rz_beta(nrhs, npw, R, Z, L, rz, beta, first, br, st);
    };

    auto hm = [&](const void *in, int64_t ldi, void *out) { hpsi_any(ctx, PW_C128, nrhs, in, ldi, out, L, E, cur); };
    // set-up: R = (H - E) w - (H - E)^2 x0, Y = (H - E) x0, P = Z = K R
    copy_block(nrhs, npw, psi, ld, X, L, st);
    hm(X, L, Y);
    hm(Y, L, U);
    hm(w, ldw, R);
    lin_sub(nrhs, npw, R, U, L, st);
    precondition(true);
    copy_block(nrhs, npw, Z, L, P, L, st);

    std::vector<double> h_err(nrhs);
    const int check = std::max(1, o.check_every);
    int it = 0, nhist = 0;
    bool converged = false;
    // one segment: `len` PCG iterations and the device side of the check that ends it
    auto segment = [&](int len) {
        const hipStream_t st = cur;
        for (int k = 0; k < len; ++k) {
            hm(P, L, YP);
            hm(YP, L, AP);
            lin_alpha(nrhs, npw, YP, L, rz, alpha, br, st);
            lin_update(nrhs, npw, X, Y, R, P, YP, AP, L, alpha, st);
            precondition(false);
            lin_pupdate(nrhs, npw, Z, P, L, beta, st);
        }
        lin_err(nrhs, npw, Y, L, w, ldw, err, br, st);
    };
    // a full segment is pure device work with fixed pointers: it is recorded once into a graph and
    // replayed (not while per-stage profiling is on, whose events are recorded on the host's side)
    SegmentGraph graph;
    const bool use_graph = o.use_graph && !ctx->prof_on;
    while (it < o.maxit) {
        const int len = std::min(check, o.maxit - it);
        if (use_graph && len == check) {
            if (!graph.exec) {
                PW_HIP(hipStreamCreateWithFlags(&graph.cap, hipStreamNonBlocking));
                PW_HIP(hipStreamBeginCapture(graph.cap, hipStreamCaptureModeThreadLocal));
                cur = graph.cap;
                try {
                    segment(len);
                } catch (...) {
                    cur = st;
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(graph.cap, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                cur = st;
                PW_HIP(hipStreamEndCapture(graph.cap, &graph.g));
                PW_HIP(hipGraphInstantiate(&graph.exec, graph.g, nullptr, nullptr, 0));
            }
            PW_HIP(hipGraphLaunch(graph.exec, st));
        } else {
            segment(len);
        }
        it += len;
        {
            PW_HIP(hipMemcpyAsync(h_err.data(), err, (size_t)nrhs * 8, hipMemcpyDeviceToHost, st));
            PW_HIP(hipStreamSynchronize(st));
            double mx = 0.0;
            bool finite = true;
            for (double v : h_err) {
                if (!std::isfinite(v)) finite = false;
                mx = std::max(mx, v);
            }
            PW_CHECK(finite, PW_ENAN, "non-finite error at iteration %d", it);
            if (stats && stats->hist && nhist < stats->n_hist) {
                stats->hist[2 * nhist] = it;
                stats->hist[2 * nhist + 1] = mx;
                ++nhist;
            }
            if (o.verbose) fprintf(stderr, "[pw] lin it %6d  max error %.3e\n", it, mx);
            if (mx <= o.tol) {
                converged = true;
                break;
            }
        }
    }
    // final error from a fresh (H - E) x
    hm(X, L, Y);
    lin_err(nrhs, npw, Y, L, w, ldw, err, br, st);
    copy_block(nrhs, npw, X, L, psi, ld, st);
    PW_HIP(hipMemcpyAsync(h_err.data(), err, (size_t)nrhs * 8, hipMemcpyDeviceToHost, st));
    PW_HIP(hipStreamSynchronize(st));
    double mx = 0.0;
    for (int l = 0; l < nrhs; ++l) {
        if (resid) resid[l] = h_err[l];
        mx = std::max(mx, h_err[l]);
    }
    const int64_t n_hpsi = (int64_t)(3 + 2 * it + 1) * nrhs;    // set-up, two per iteration, final check
    if (stats) {
        stats->iters = it;
        stats->converged = converged ? 1 : 0;
        stats->n_hpsi = n_hpsi;
        stats->max_resid = mx;
        stats->n_hist = nhist;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!converged) {
        set_error("folded linear solve did not reach tol %.3e in %d iterations (max error %.3e)", o.tol, o.maxit, mx);
        return PW_ENOCONV;
    }
    return PW_OK;
}

}  // namespace pw

extern "C" {

void pw_lin_opts_default(pw_lin_opts *o) {
    if (!o) return;
    o->tol = 1e-8;
    o->maxit = 20000;
    o->precond = 0;
    o->delta_e = 1.0;
    o->check_every = 10;
    o->verbose = 0;
    o->use_graph = 1;
}

pw_status pw_folded_linear_solve(pw_ctx *ctx, double e, int32_t nrhs, const void *w, int64_t ldw, void *psi,
                                 int64_t ld, int32_t nev, const void *phi, int64_t ldphi, const double *eps,
                                 const double *delta, double *resid, const pw_lin_opts *opts, pw_lin_stats *stats,
                                 void *stream) {
    try {
        PW_CHECK(ctx && w && psi, PW_EINVAL, "null argument");
        PW_CHECK(ctx->flags & PW_PREP_C128, PW_EUNSUPPORTED, "the linear solve needs a complex128 context");
        PW_CHECK(nrhs >= 1 && nrhs <= ctx->max_bands, PW_EINVAL, "nrhs %d must be in [1, max_bands %d]", nrhs,
                 ctx->max_bands);
        PW_CHECK(ld >= ctx->basis.npw && ldw >= ctx->basis.npw, PW_EINVAL, "ld or ldw < npw");
        PW_CHECK(psi != w, PW_EINVAL, "psi and w must not alias");
        PW_CHECK(std::isfinite(e), PW_ENAN, "non-finite energy");
        pw_lin_opts o;
        pw_lin_opts_default(&o);
        if (opts) o = *opts;
        PW_CHECK(o.tol > 0 && o.maxit >= 1 && o.check_every >= 1 && o.delta_e > 0, PW_EINVAL,
                 "bad linear-solve options");
        PW_CHECK(o.precond == 0 || o.precond == 1, PW_EINVAL, "preconditioner %d unknown", o.precond);
        if (o.precond == 1) {
            PW_CHECK(nev >= 1 && nev <= ctx->basis.npw, PW_EINVAL, "M' needs 1 <= nev <= npw eigenpairs (nev %d)", nev);
            PW_CHECK(phi && eps && delta, PW_EINVAL, "M' needs phi, eps and delta");
            PW_CHECK(ldphi >= ctx->basis.npw, PW_EINVAL, "ldphi < npw");
        }
        return pw::folded_linsolve(ctx, e, nrhs, w, ldw, psi, ld, o.precond == 1 ? nev : 0, phi, ldphi, eps, delta,
                                   resid, o, stats, (hipStream_t)stream);
    } catch (const pw::Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        pw::set_error("host allocation failed");
        return PW_ENOMEM;
    } catch (...) {
        pw::set_error("unexpected exception in pw_folded_linear_solve");
        return PW_EINVAL;
    }
}

}  // extern "C"
