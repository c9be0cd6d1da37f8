// Folded-spectrum preconditioned CG driver (host control, all arithmetic on the GPU).
//
// Finds the nb eigenpairs of H nearest E by minimising tr(Psi^H A Psi), A = (H - E)^2,
// over orthonormal Psi: the folded operator and its positivity are the paper's folded
// equation (Sec. II.B), the CG functional is the paper's F with the eigenvector in place
// of the scattering source (Sec. II.B), the G-diagonal preconditioner is M(G) of Sec.
// II.B (or the folded Teter-Payne-Allan form), and convergence is the eigen-residual
// Delta_i = ||H psi_i - theta_i psi_i|| of Sec. II.B.
//
// One iteration (band-major blocks [nb][npw], Y = (H - E) X, AX = (H - E) Y):
//   mu = ||Y||^2, T_i            -> G = AX - mu X, Z = K o G, Polak-Ribiere P
//   P -= X (X^H P)               -> YP = (H - E) P, AP = (H - E) YP   (two H psi)
//   per-band exact 2x2 minimum   -> X, Y, AX updated together
//   S = X^H X = L L^H            -> X, Y, AX <- conj(L^-1) . (X, Y, AX)
// Every check_every iterations: Y and AX recomputed from X, Rayleigh-Ritz in A
// (bands ordered by folded value, directions turned with them), and the residuals
// Delta_i of a Rayleigh-Ritz in H taken on copies; the host syncs only here.
#include <algorithm>
#include <chrono>
#include <memory>
#include <cmath>
#include <utility>

#include "kernels.h"

namespace pw {

void hpsi_any(pw_ctx *ctx, pw_dtype dt, int nb, const void *psi, int64_t ld, void *out, int64_t ldo, double shift,
              hipStream_t st);

struct Solver {
    int nbmax = 0, npw = 0;
    DevBuf X, Y, AX, P, YP, AP, G, Z, T1, T2, T3;
    DevBuf small;                  // N x N work matrices
    DevBuf vec;                    // per-band vectors
    DevBuf red;                    // reduction partials
    DevBuf status;                 // ints
    DevBuf ftab;                   // learned preconditioner scaling [nshell][nb] (float)
    int nsplit = 0;
};

void solver_destroy(Solver *s) { delete s; }

static Solver *solver_get(pw_ctx *ctx, int nb, bool mixed) {
    Solver *s = ctx->solver;
    const int npw = ctx->basis.npw;
    if (!s || s->nbmax < nb) {
        delete s;
        ctx->solver = nullptr;
        s = new Solver();
        s->nbmax = ctx->max_bands;
        s->npw = npw;
        const size_t blk = (size_t)s->nbmax * npw * 16;
        DevBuf *blocks[] = {&s->X, &s->Y, &s->AX, &s->P, &s->YP, &s->AP, &s->G, &s->Z, &s->T1, &s->T2, &s->T3};
        for (DevBuf *d : blocks) d->alloc(blk);
        const size_t nn = (size_t)s->nbmax * s->nbmax * 16;
        // Sm, Wm, Tm, Rm, then the eigensolver's work, which the Cholesky inverse borrows
        s->small.alloc(4 * nn + std::max(dense_eigh_work_bytes(s->nbmax), chol_inv_work_bytes(s->nbmax)));
        s->vec.alloc((size_t)s->nbmax * 8 * 24);
        s->nsplit = band_splits(npw);
        s->red.alloc((size_t)4 * s->nbmax * s->nsplit * 8);
        s->status.alloc(256);
        s->ftab.alloc((size_t)ctx->basis.shell_t.size() * s->nbmax * sizeof(float));
        ctx->solver = s;
        ctx->device_bytes += (int64_t)(11 * blk + s->small.bytes + s->vec.bytes + s->red.bytes + 256);
    }
    (void)mixed;   // the complex64 staging of mixed H psi lives in the rotation temporaries
    return s;
}

// One folded-CG solve as a resumable object: setup(), then segments of
// iterations each ending in the device part of a check (check_device), the host
// decisions (check_host), and finish().  Segments are pure device work, so they
// can be recorded into a graph; with swap_free set, rotations copy back into the
// blocks instead of exchanging block pointers, so a recorded segment leaves the
// pointers as it found them and can be replayed.
struct FcgRun {
    pw_ctx *ctx;
    double E;
    int nb;
    void *psi;
    int64_t ld;
    double *eig, *resid;
    pw_cg_opts o;
    pw_cg_stats *stats;
    hipStream_t st;
    bool swap_free = false;

    std::chrono::steady_clock::time_point t_start;
    int npw = 0, nshell = 0, check = 1, nwant = 0;
    bool mixed = false, use_mixed = false;
    Solver *s = nullptr;
    int64_t L = 0;
    void *X, *Y, *AX, *P, *YP, *AP, *G, *Z, *T1, *T2, *T3;
    double2 *Sm, *Wm, *Tm, *Rm, *Aw;
    double *mu, *tband, *gz, *gzo, *gz_old, *line4, *coef, *lam, *res;
    int *d_status;
    BandRed br;
    PrecArgs pa{};
    int64_t n_hpsi = 0;
    std::vector<double> h_lam, h_res;
    int h_status[8] = {0};
    int it = 0, stall = 0, nhist = 0, nsnap = 0;
    bool converged = false;
    double best = INFINITY;
    int lstall = 0, switch_it = -1, recoveries = 0, nchecks = 0;
    double lbest = INFINITY;
    pw_status result = PW_OK;

    FcgRun(pw_ctx *c, double e, int n, void *p, int64_t l, double *ev, double *rv, const pw_cg_opts &opt,
           pw_cg_stats *sta, hipStream_t stream)
        : ctx(c), E(e), nb(n), psi(p), ld(l), eig(ev), resid(rv), o(opt), stats(sta), st(stream) {
        t_start = std::chrono::steady_clock::now();
        npw = ctx->basis.npw;
        mixed = use_mixed = o.precision == 1;
        s = solver_get(ctx, nb, mixed);
        L = npw;   // internal leading dimension
        X = s->X.p; Y = s->Y.p; AX = s->AX.p; P = s->P.p; YP = s->YP.p; AP = s->AP.p;
        G = s->G.p; Z = s->Z.p; T1 = s->T1.p; T2 = s->T2.p; T3 = s->T3.p;
        const size_t nn = (size_t)nb * nb;
        Sm = (double2 *)s->small.p; Wm = Sm + nn; Tm = Wm + nn; Rm = Tm + nn; Aw = Rm + nn;
        double *v = (double *)s->vec.p;
        mu = v; tband = v + nb; gz = v + 2 * nb; gzo = v + 3 * nb; gz_old = v + 4 * nb;
        line4 = v + 5 * nb; coef = v + 9 * nb; lam = v + 13 * nb; res = v + 14 * nb;
        d_status = (int *)s->status.p;
        br = BandRed{(double *)s->red.p, s->nsplit};
        pa.kind = o.precond;
        pa.ftab = s->ftab.as<float>();
        pa.kin = ctx->d_kin.as<double>();
        pa.tband = tband;
        pa.e_ref = E;
        pa.de2 = o.delta_e * o.delta_e;
        pa.shell = ctx->d_shell.as<int32_t>();
        pa.nb = nb;
        h_lam.assign(nb, 0.0);
        h_res.assign(nb, 0.0);
        // largest residual among the nconv Ritz values (theta - E) nearest zero
        nwant = (o.nconv > 0 && o.nconv < nb) ? o.nconv : nb;
        check = std::max(1, o.check_every);
        nshell = (int)ctx->basis.shell_t.size();
    }

    void fold(void *in, void *y, void *ay, bool low) {
        if (low) {
            // complex64 staging in the rotation temporaries, which hold nothing live during a
            // fold: T1 = [P32 | Q32] (each nb x npw complex64 fits half a block), T2 = [R32]
            void *P32 = T1, *Q32 = (char *)T1 + (size_t)nb * npw * 8, *R32 = T2;
            c128_to_c64(nb, npw, in, L, P32, L, st);
            hpsi_any(ctx, PW_C64, nb, P32, L, Q32, L, E, st);
            hpsi_any(ctx, PW_C64, nb, Q32, L, R32, L, E, st);
            c64_to_c128(nb, npw, Q32, L, y, L, st);
            c64_to_c128(nb, npw, R32, L, ay, L, st);
        } else {
            hpsi_any(ctx, PW_C128, nb, in, L, y, L, E, st);
            hpsi_any(ctx, PW_C128, nb, y, L, ay, L, E, st);
        }
        n_hpsi += 2 * nb;
    }
    // the rotated block takes tmp's storage, or (swap_free) is copied back
    void settle(void *&blk, void *&tmp) {
        if (swap_free) copy_block(nb, npw, tmp, L, blk, L, st);
        else std::swap(blk, tmp);
    }
    void rotate(const double2 *M, void *&blk, void *&tmp, bool lower = false) {
        {
            ProfScope p(ctx, 7, st);
            zgemm_nn_launch(nb, npw, nb, M, nb, blk, L, 1.0, 0.0, tmp, L, st, false, ctx->rot_tune.get(nb), lower);
        }
        settle(blk, tmp);
    }
    // S (nb x nb) = A^H B over the plane waves
    void gram(const void *A, const void *B, double alpha, double2 *S, bool trans) {
        ProfScope p(ctx, A == B ? 8 : 6, st);
        // A == B: a Gram matrix, Hermitian, so half its tiles
        zgemm_nt(nb, nb, npw, true, A, L, B, L, alpha, nullptr, 0.0, S, nb, trans, ctx->d_partial.p, st, false,
                 A == B);
    }
    // (X, Y, AX) <- M . (X, Y, AX) in one batched launch (lower: M lower triangular)
    void rotate3(const double2 *M, bool lower = false) {
        const void *in[3] = {X, Y, AX};
        void *out[3] = {T1, T2, T3};
        {
            ProfScope p(ctx, 5, st);
            zgemm_nn_batch(3, nb, npw, nb, M, nb, in, L, 1.0, 0.0, out, L, st, false, ctx->rot_tune.get(nb), lower);
        }
        settle(X, T1);
        settle(Y, T2);
        settle(AX, T3);
    }
    void orth() {
        gram(X, X, 1.0, Sm, false);
        chol_inv(nb, Sm, nb, Aw, Tm, d_status, st);
        rotate3(Tm, true);                    // conj(L^-1) is lower triangular
    }
    // Rayleigh-Ritz in A = (H - E)^2 on the iterate (Y, AX exact): Ritz values of
    // Y^H Y ascending; the search directions and gradients turn with the bands.
    void a_rr(bool rotate_dirs) {
        gram(Y, Y, 1.0, Sm, false);
        dense_eigh(nb, Sm, nb, Aw, lam, Rm, 0, 0.0, d_status + 4, st);
        rotate3(Rm);
        if (rotate_dirs) {
            const void *in[2] = {P, G};
            void *out[2] = {T1, T2};
            zgemm_nn_batch(2, nb, npw, nb, Rm, nb, in, L, 1.0, 0.0, out, L, st, false, ctx->rot_tune.get(nb));
            settle(P, T1);
            settle(G, T2);
        }
    }
    // Rayleigh-Ritz in H on copies of the block: lam = theta - E ascending and the
    // residuals Delta_i of the H-Ritz vectors (the iterate itself is left alone)
    void h_resid() {
        gram(X, Y, 1.0, Sm, false);
        dense_eigh(nb, Sm, nb, Aw, lam, Rm, 0, 0.0, d_status + 4, st);
        {
            ProfScope p(ctx, 7, st);
            zgemm_nn_launch(nb, npw, nb, Rm, nb, X, L, 1.0, 0.0, T1, L, st, false, ctx->rot_tune.get(nb));
        }
        {
            ProfScope p(ctx, 7, st);
            zgemm_nn_launch(nb, npw, nb, Rm, nb, Y, L, 1.0, 0.0, T2, L, st, false, ctx->rot_tune.get(nb));
        }
        red_resid(nb, npw, T2, T1, L, lam, res, br, st);
    }
    // band kinetic energies, then (learned preconditioner) the per-shell scaling table
    void band_stats() {
        red_mu_tband(nb, npw, Y, X, L, ctx->d_kin.as<double>(), mu, tband, br, st);
        if (pa.kind == 2)
            mlp_infer(nshell, nb, ctx->d_shell_t.as<double>(), tband, E, ctx->cell.ecut, ctx->d_mlp.as<float>(),
                      s->ftab.as<float>(), st);
    }
    double wanted_max() const {
        std::vector<int> idx(nb);
        for (int b = 0; b < nb; ++b) idx[b] = b;
        std::stable_sort(idx.begin(), idx.end(),
                         [&](int a, int c) { return std::fabs(h_lam[a]) < std::fabs(h_lam[c]); });
        double m = 0.0;
        for (int r = 0; r < nwant; ++r) m = std::max(m, h_res[idx[r]]);
        return m;
    }

    // this solve as one problem of a fused batch (blocks fixed: swap_free)
    BandProb band_prob() const {
        BandProb b{};
        b.npw = npw;
        b.nsplit = br.nsplit;
        b.ld = L;
        void *const blk[kBlocks] = {X, Y, AX, P, YP, AP, G, Z, T1, T2, T3};
        for (int i = 0; i < kBlocks; ++i) b.blk[i] = (double2 *)blk[i];
        b.vec = mu;
        b.red = br.partial;
        b.pa = pa;
        b.psi = (double2 *)psi;
        b.ldpsi = ld;
        b.status = d_status;
        return b;
    }

    void setup() {
        fill_zero(s->status.p, 256, st);
        copy_block(nb, npw, psi, ld, X, L, st);
        fill_zero(P, (size_t)nb * npw * 16, st);
        fill_zero(G, (size_t)nb * npw * 16, st);
        fill_zero(gz_old, ((size_t)nb * 8 + 15) / 16 * 16, st);
        // initial orthonormalisation (Y, AX are garbage here but get overwritten)
        gram(X, X, 1.0, Sm, false);
        chol_inv(nb, Sm, nb, Aw, Tm, d_status, st);
        rotate(Tm, X, T1, true);
        fold(X, Y, AX, false);
        a_rr(false);
        fill_zero(gz_old, ((size_t)nb * 8 + 15) / 16 * 16, st);
    }
    // iterations left before the next check
    int segment_length() const { return std::min(check - it % check, o.maxit - it); }
    void iteration() {
        ++it;
        band_stats();
        red_grad(nb, npw, X, AX, G, Z, L, mu, pa, gz, gzo, br, st);
        pupdate(nb, npw, Z, P, L, gz, gzo, gz_old, st);
        // P -= X (X^H P): W[b][j] = -<x_j|p_b>
        gram(X, P, -1.0, Wm, true);
        {
            ProfScope p(ctx, 7, st);
            zgemm_nn_launch(nb, npw, nb, Wm, nb, X, L, 1.0, 1.0, P, L, st, false, ctx->rot_tune.get(nb));
        }
        fold(P, YP, AP, use_mixed);
        red_line(nb, npw, Y, YP, P, L, line4, br, st);
        line_coef(nb, mu, line4, coef, st);
        combine3(nb, npw, X, Y, AX, P, YP, AP, L, coef, st);
        orth();
        if (o.snap_every > 0 && o.snap_buf && it % o.snap_every == 0 && nsnap < o.snap_cap) {
            copy_block(nb, npw, X, L, (char *)o.snap_buf + (size_t)nsnap * nb * npw * 16, npw, st);
            ++nsnap;
        }
    }
    // After a lost Gram factorisation: back to the iterate of the last check (in psi;
    // the start block before the first check), band `bad` replaced by a seeded random
    // vector, directions cleared, then the set-up again (orthonormalisation, Y, AX,
    // Rayleigh-Ritz in A).
    void restart(int bad) {
        ++recoveries;
        if (o.verbose) fprintf(stderr, "[pw] it %6d  Gram factorisation lost at band %d: restart\n", it, bad);
        std::vector<double2> v(npw);
        uint64_t x = 0x9E3779B97F4A7C15ull * (uint64_t)(recoveries + 1) ^ (uint64_t)it;
        auto unif = [&]() {       // splitmix64 to (0, 1)
            x += 0x9E3779B97F4A7C15ull;
            uint64_t z = x;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            return ((z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        };
        for (int g = 0; g < npw; ++g) v[g] = make_double2(unif() - 0.5, unif() - 0.5);
        const int b = std::min(std::max(bad, 0), nb - 1);
        PW_HIP(hipMemcpyAsync((char *)psi + (size_t)b * ld * 16, v.data(), (size_t)npw * 16, hipMemcpyHostToDevice,
                              st));
        PW_HIP(hipStreamSynchronize(st));
        setup();
    }
    void check_device() {
        fold(X, Y, AX, false);
        a_rr(true);
        h_resid();
        // PR denominator for the rotated gradients
        band_stats();
        red_gzold(nb, npw, G, L, pa, gz_old, br, st);
    }
    // the host side of a check; false once the solve stops (converged or failed)
    bool check_host() {
        PW_HIP(hipMemcpyAsync(h_lam.data(), lam, nb * 8, hipMemcpyDeviceToHost, st));
        PW_HIP(hipMemcpyAsync(h_res.data(), res, nb * 8, hipMemcpyDeviceToHost, st));
        PW_HIP(hipMemcpyAsync(h_status, d_status, sizeof h_status, hipMemcpyDeviceToHost, st));
        PW_HIP(hipStreamSynchronize(st));
        return decide();
    }
    // the decisions of a check from h_lam, h_res and h_status; defer_save: the
    // caller saves X to psi itself when this returns true with restarted unchanged
    bool restarted = false;
    bool decide(bool defer_save = false) {
        restarted = false;
        ++nchecks;
        if (o.fault_check > 0 && nchecks == o.fault_check) h_status[0] = nb / 2 + 1;   // forced by the host
        if (h_status[0]) {
            if (o.recover && recoveries < 3) {
                restart(h_status[0] - 1);
                restarted = true;
                return it < o.maxit;
            }
            set_error("Gram matrix lost positive definiteness (pivot %d) before iteration %d", h_status[0] - 1, it);
            result = PW_ENOTPD;
            return false;
        }
        bool finite = true;
        for (int b = 0; b < nb; ++b)
            if (!std::isfinite(h_res[b]) || !std::isfinite(h_lam[b])) finite = false;
        if (!finite) {
            set_error("non-finite residual at iteration %d", it);
            result = PW_ENAN;
            return false;
        }
        const double mx = wanted_max();
        if (stats && stats->hist && nhist < stats->n_hist) {
            stats->hist[2 * nhist] = it;
            stats->hist[2 * nhist + 1] = mx;
            ++nhist;
        }
        if (o.verbose) fprintf(stderr, "[pw] it %6d  max resid %.3e%s\n", it, mx, use_mixed ? "  (mixed)" : "");
        if (mx <= o.tol) {
            converged = true;
            return false;
        }
        // the iterate of this check is the one a restart goes back to
        if (o.recover && !defer_save) copy_block(nb, npw, X, L, psi, ld, st);
        // the learned preconditioner gives way to the paper's M(G) once the best residual
        // has not halved over learned_stall checks
        if (pa.kind == 2 && o.learned_stall > 0) {
            if (mx < 0.5 * lbest) {
                lbest = mx;
                lstall = 0;
            } else if (++lstall >= o.learned_stall) {
                pa.kind = 1;
                switch_it = it;
                if (o.verbose) fprintf(stderr, "[pw] it %6d  learned preconditioner stalled: M(G) from here\n", it);
            }
        }
        // precision ladder: leave the low-precision operator below mixed_switch, or
        // once the best residual has not improved by 2x over stall_checks checks
        // while within 20 x mixed_switch (a stall higher up is the search for the
        // last wanted states, which the operator's precision does not limit), or
        // over 10 x stall_checks checks anywhere
        if (use_mixed) {
            if (mx < 0.5 * best) {
                best = mx;
                stall = 0;
            } else if (o.stall_checks > 0) {
                ++stall;
                if ((stall >= o.stall_checks && best < 20.0 * o.mixed_switch) || stall >= 10 * o.stall_checks)
                    use_mixed = false;
            }
            if (mx < o.mixed_switch) use_mixed = false;
            if (!use_mixed && o.verbose) fprintf(stderr, "[pw] it %6d  switching to FP64 H psi\n", it);
        }
        return it < o.maxit;
    }
    // final Rayleigh-Ritz in H, ascending energies, FP64 residuals
    pw_status finish() {
        if (result == PW_OK || result == PW_ENOCONV) {
            hpsi_any(ctx, PW_C128, nb, X, L, Y, L, E, st);
            n_hpsi += nb;
            gram(X, Y, 1.0, Sm, false);
            dense_eigh(nb, Sm, nb, Aw, lam, Rm, 0, 0.0, d_status + 4, st);
            rotate(Rm, X, T1);
            rotate(Rm, Y, T2);
            red_resid(nb, npw, Y, X, L, lam, res, br, st);
            copy_block(nb, npw, X, L, psi, ld, st);
            PW_HIP(hipMemcpyAsync(h_lam.data(), lam, nb * 8, hipMemcpyDeviceToHost, st));
            PW_HIP(hipMemcpyAsync(h_res.data(), res, nb * 8, hipMemcpyDeviceToHost, st));
            PW_HIP(hipStreamSynchronize(st));
            for (int b = 0; b < nb; ++b) {
                if (eig) eig[b] = h_lam[b] + E;
                if (resid) resid[b] = h_res[b];
            }
            const double mx = wanted_max();
            if (!converged) {
                converged = mx <= o.tol;
                if (!converged) {
                    set_error("folded CG did not reach tol %.3e in %d iterations (max residual %.3e)", o.tol, o.maxit,
                              mx);
                    result = PW_ENOCONV;
                }
            }
            if (stats) stats->max_resid = mx;
        }
        // the solver's scratch blocks may have been swapped: keep them in the struct
        s->X.p = X; s->Y.p = Y; s->AX.p = AX; s->P.p = P; s->YP.p = YP; s->AP.p = AP;
        s->G.p = G; s->Z.p = Z; s->T1.p = T1; s->T2.p = T2; s->T3.p = T3;
        if (stats) {
            stats->iters = it;
            stats->converged = converged ? 1 : 0;
            stats->n_hpsi = n_hpsi;
            stats->n_hist = nhist;
            stats->n_snap = nsnap;
            stats->precond_switch_it = switch_it;
            stats->recoveries = recoveries;
            stats->fused = 0;
            stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        }
        return result;
    }
};

namespace {
// HIP events on the solver's stream around the phases of a solve (set-up, iteration
// segments, checks, final Rayleigh-Ritz); elapsed times are read after the host has
// synchronised anyway
struct PhaseClock {
    hipEvent_t ev[6] = {};
    double ms[4] = {0, 0, 0, 0};
    PhaseClock() {
        for (hipEvent_t &e : ev) PW_HIP(hipEventCreate(&e));
    }
    ~PhaseClock() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    void mark(int i, hipStream_t st) { PW_HIP(hipEventRecord(ev[i], st)); }
    void add(int phase, int a, int b) {
        float t = 0.f;
        PW_HIP(hipEventElapsedTime(&t, ev[a], ev[b]));
        ms[phase] += t;
    }
};
}  // namespace

pw_status folded_cg(pw_ctx *ctx, double E, int nb, void *psi, int64_t ld, double *eig, double *resid,
                    const pw_cg_opts &o, pw_cg_stats *stats, hipStream_t st) {
    FcgRun r(ctx, E, nb, psi, ld, eig, resid, o, stats, st);
    PhaseClock clk;
    // per-stage profiling (pw_profile_begin) records the iterations only
    struct Pause {
        pw_ctx *c;
        ~Pause() { c->prof_pause = false; }
    } pause{ctx};
    ctx->prof_pause = true;
    clk.mark(0, st);
    r.setup();
    clk.mark(1, st);
    bool first = true;
    for (;;) {
        const int n = r.segment_length();
        clk.mark(2, st);
        ctx->prof_pause = false;
        for (int k = 0; k < n; ++k) r.iteration();
        ctx->prof_pause = true;
        clk.mark(3, st);
        r.check_device();
        clk.mark(4, st);
        const bool more = r.check_host();     // synchronises the stream
        if (first) clk.add(0, 0, 1);
        first = false;
        clk.add(1, 2, 3);
        clk.add(2, 3, 4);
        if (!more) break;
    }
    clk.mark(5, st);
    const pw_status res = r.finish();         // synchronises the stream
    {
        float t = 0.f;
        PW_HIP(hipEventRecord(clk.ev[4], st));
        PW_HIP(hipEventSynchronize(clk.ev[4]));
        PW_HIP(hipEventElapsedTime(&t, clk.ev[5], clk.ev[4]));
        clk.ms[3] = t;
    }
    if (stats)
        for (int k = 0; k < 4; ++k) stats->ms[k] = clk.ms[k];
    return res;
}

// ---------------------------------------------------------------------------
// Batched solves: independent problems (one context each) advance together.
// Each problem's segment (check_every iterations and the device side of the
// check) is recorded once per (length, H psi precision) into a graph.  Each
// check round then either launches every running problem's instantiated segment
// back to back on the caller's stream (batch_launch = 1), or launches one graph
// whose independent child graphs are those segments (batch_launch = 0; rebuilt
// and instantiated again whenever a problem finishes or changes precision).
// Between rounds the host reads every problem's residuals.  Per problem, the
// kernels and their order are those of the unbatched solve.
// ---------------------------------------------------------------------------
namespace {
struct SegGraph {
    int len = 0;
    bool low = false;
    int kind = 0;          // preconditioner the segment was recorded with
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t hpsi = 0;
};
struct BatchItem {
    std::unique_ptr<FcgRun> run;
    std::vector<SegGraph> segs;
    bool active = true;
    hipGraph_t cur = nullptr;
    int len = 0;
    int64_t hpsi = 0;
};
struct BatchRes {
    std::vector<BatchItem> items;
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    ~BatchRes() {
        if (exec) (void)hipGraphExecDestroy(exec);
        for (auto &b : items)
            for (auto &g : b.segs) {
                if (g.exec) (void)hipGraphExecDestroy(g.exec);
                if (g.g) (void)hipGraphDestroy(g.g);
            }
        if (cap) (void)hipStreamDestroy(cap);
    }
};

SegGraph record_segment(FcgRun &r, int len, hipStream_t cap) {
    SegGraph sg;
    sg.len = len;
    sg.low = r.use_mixed;
    sg.kind = r.pa.kind;
    const hipStream_t keep = r.st;
    const int it0 = r.it;
    const int64_t h0 = r.n_hpsi;
    r.st = cap;
    PW_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    try {
        for (int k = 0; k < len; ++k) r.iteration();
        r.check_device();
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(cap, &g);
        if (g) (void)hipGraphDestroy(g);
        r.st = keep;
        throw;
    }
    r.st = keep;
    PW_HIP(hipStreamEndCapture(cap, &sg.g));
    sg.hpsi = r.n_hpsi - h0;
    r.it = it0;          // recording does not advance the solve
    r.n_hpsi = h0;
    return sg;
}
}  // namespace

// ---------------------------------------------------------------------------
// Fused batch (batch_launch = 2): every step of an iteration and of a check is
// one launch (or one per group of equal FFT grids) over all problems, each
// problem's kernels, tiles and split-K chunking being those of its own solve, so
// each problem's numbers are bit for bit those of its own solve.  A device mask
// says which problems still run: kernels of finished problems return at once,
// so the recorded round (segment of iterations and the device part of a check)
// is replayed unchanged while problems drop out.  FP64 H psi, preconditioners 0
// and 1, at most 136 bands, default launch choices, projector counts whose
// projection takes one GEMM tile shape.
// ---------------------------------------------------------------------------
namespace {
struct FusedJobs {
    std::vector<NtJob> h;
    DevBuf d;
    void up() {
        d.alloc(h.size() * sizeof(NtJob));
        PW_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(NtJob), hipMemcpyHostToDevice));
    }
};
struct FusedNn {
    std::vector<NnJob> h;
    DevBuf d;
    void up() {
        d.alloc(h.size() * sizeof(NnJob));
        PW_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(NnJob), hipMemcpyHostToDevice));
    }
};
struct FusedDense {
    std::vector<DenseJob> h;
    DevBuf d;
    void up() {
        d.alloc(h.size() * sizeof(DenseJob));
        PW_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(DenseJob), hipMemcpyHostToDevice));
    }
};
struct HpsiHandle {
    HpsiBatch *b = nullptr;
    ~HpsiHandle() { if (b) hpsi_batch_destroy(b); }
};

NnJob nn_job(int nb, int npw, const double2 *W, const std::vector<void *> &x, const std::vector<void *> &out,
             int64_t L, double beta, bool lower) {
    NnJob j{};
    j.M = nb; j.J = npw; j.K = nb; j.nz = (int)x.size(); j.lower = lower ? 1 : 0;
    j.W = W; j.ldw = nb;
    for (size_t z = 0; z < x.size(); ++z) {
        j.X[z] = (const double2 *)x[z];
        j.Out[z] = (double2 *)out[z];
    }
    j.ldx = L; j.ldo = L; j.alpha = 1.0; j.beta = beta;
    return j;
}
}  // namespace

static bool fused_ok(int nprob, pw_ctx *const *ctxs, int nb, const pw_cg_opts &o, std::string *why) {
    if (o.precision != 0) { *why = "mixed precision"; return false; }
    if (o.precond != 0 && o.precond != 1) { *why = "learned preconditioner"; return false; }
    if (nb > 136) { *why = "more than 136 bands"; return false; }
    if (o.snap_every > 0 && o.snap_buf) { *why = "snapshots"; return false; }
    return hpsi_batch_ok(nprob, ctxs, nb, why);
}

static void fused_solve(std::vector<FcgRun *> &runs, const pw_cg_opts &o, hipStream_t st) {
    const int n = (int)runs.size(), nb = runs[0]->nb;
    int maxsplit = 1, maxnpw = 1;
    std::vector<BandProb> hp(n);
    std::vector<pw_ctx *> ctx(n);
    std::vector<double> shift(n);
    std::vector<void *> X(n), Y(n), AX(n), P(n), YP(n), AP(n);
    for (int p = 0; p < n; ++p) {
        FcgRun &r = *runs[p];
        hp[p] = r.band_prob();
        ctx[p] = r.ctx;
        shift[p] = r.E;
        X[p] = r.X; Y[p] = r.Y; AX[p] = r.AX; P[p] = r.P; YP[p] = r.YP; AP[p] = r.AP;
        maxsplit = std::max(maxsplit, r.br.nsplit);
        maxnpw = std::max(maxnpw, r.npw);
    }
    DevBuf d_probs, d_mask, d_save, d_out, d_sout;
    d_probs.alloc(n * sizeof(BandProb));
    PW_HIP(hipMemcpy(d_probs.p, hp.data(), n * sizeof(BandProb), hipMemcpyHostToDevice));
    std::vector<int> mask(n, 1), save(n, 0);
    d_mask.alloc(n * sizeof(int));
    d_save.alloc(n * sizeof(int));
    PW_HIP(hipMemcpy(d_mask.p, mask.data(), n * sizeof(int), hipMemcpyHostToDevice));
    d_out.alloc((size_t)n * 2 * nb * sizeof(double));
    d_sout.alloc((size_t)n * 8 * sizeof(int));
    const int *dm = d_mask.as<int>();
    const BandProb *dp = d_probs.as<BandProb>();
    // H psi of the four fold inputs (internal leading dimension L = npw)
    std::vector<int64_t> Ls(n);
    for (int p = 0; p < n; ++p) Ls[p] = runs[p]->L;
    HpsiHandle h_p, h_yp, h_x, h_y;
    h_p.b = hpsi_batch_create(n, ctx.data(), nb, P.data(), Ls.data(), YP.data(), Ls.data(), shift.data(), dm);
    h_yp.b = hpsi_batch_create(n, ctx.data(), nb, YP.data(), Ls.data(), AP.data(), Ls.data(), shift.data(), dm);
    h_x.b = hpsi_batch_create(n, ctx.data(), nb, X.data(), Ls.data(), Y.data(), Ls.data(), shift.data(), dm);
    h_y.b = hpsi_batch_create(n, ctx.data(), nb, Y.data(), Ls.data(), AX.data(), Ls.data(), shift.data(), dm);
    // block products of an iteration and of a check
    FusedJobs nt_xp, nt_xx, nt_yy, nt_xy;
    FusedNn nn_px, nn_orth, nn_rr3, nn_pg, nn_x, nn_y;
    FusedDense chol, eig;
    for (int p = 0; p < n; ++p) {
        FcgRun &r = *runs[p];
        const int npw = r.npw;
        const int64_t L = r.L;
        void *part = r.ctx->d_partial.p;
        nt_xp.h.push_back(nt_job(nb, nb, npw, true, r.X, L, r.P, L, -1.0, nullptr, 0.0, r.Wm, nb, part, false));
        nt_xx.h.push_back(nt_job(nb, nb, npw, true, r.X, L, r.X, L, 1.0, nullptr, 0.0, r.Sm, nb, part, true));
        nt_yy.h.push_back(nt_job(nb, nb, npw, true, r.Y, L, r.Y, L, 1.0, nullptr, 0.0, r.Sm, nb, part, true));
        nt_xy.h.push_back(nt_job(nb, nb, npw, true, r.X, L, r.Y, L, 1.0, nullptr, 0.0, r.Sm, nb, part, false));
        nn_px.h.push_back(nn_job(nb, npw, r.Wm, {r.X}, {r.P}, L, 1.0, false));
        nn_orth.h.push_back(nn_job(nb, npw, r.Tm, {r.X, r.Y, r.AX}, {r.T1, r.T2, r.T3}, L, 0.0, true));
        nn_rr3.h.push_back(nn_job(nb, npw, r.Rm, {r.X, r.Y, r.AX}, {r.T1, r.T2, r.T3}, L, 0.0, false));
        nn_pg.h.push_back(nn_job(nb, npw, r.Rm, {r.P, r.G}, {r.T1, r.T2}, L, 0.0, false));
        nn_x.h.push_back(nn_job(nb, npw, r.Rm, {r.X}, {r.T1}, L, 0.0, false));
        nn_y.h.push_back(nn_job(nb, npw, r.Rm, {r.Y}, {r.T2}, L, 0.0, false));
        chol.h.push_back(dense_job(nb, r.Sm, nb, r.Aw, nullptr, nullptr, nullptr, r.Tm, r.d_status));
        eig.h.push_back(dense_job(nb, r.Sm, nb, r.Aw, r.lam, r.Rm, r.d_status + 4, nullptr, nullptr));
    }
    for (FusedJobs *j : {&nt_xp, &nt_xx, &nt_yy, &nt_xy}) j->up();
    for (FusedNn *j : {&nn_px, &nn_orth, &nn_rr3, &nn_pg, &nn_x, &nn_y}) j->up();
    chol.up();
    eig.up();
    const int c_xyax[3] = {kBT1, kBT2, kBT3}, d_xyax[3] = {kBX, kBY, kBAX};
    const int c_pg[2] = {kBT1, kBT2}, d_pg[2] = {kBP, kBG};
    auto band = [&](BandOp op, int a0 = 0, int a1 = 0) {
        band_batch(op, dp, dm, n, nb, maxsplit, maxnpw, st, a0, a1);
    };
    auto iteration = [&]() {
        band(BandOp::MuTband);
        band(BandOp::Grad);
        band(BandOp::PUpdate);
        zgemm_nt_jobs(nt_xp.h, nt_xp.d.as<NtJob>(), dm, true, true, false, st);
        zgemm_nn_jobs_launch(nn_px.h, nn_px.d.as<NnJob>(), dm, -1, false, st);
        hpsi_batch_run(h_p.b, st);
        hpsi_batch_run(h_yp.b, st);
        band(BandOp::Line);
        band(BandOp::Combine3);
        zgemm_nt_jobs(nt_xx.h, nt_xx.d.as<NtJob>(), dm, true, false, false, st);
        chol_inv_jobs(nb, chol.d.as<DenseJob>(), dm, n, st);
        zgemm_nn_jobs_launch(nn_orth.h, nn_orth.d.as<NnJob>(), dm, -1, false, st);
        band_batch_copy(dp, dm, n, nb, maxnpw, 3, c_xyax, d_xyax, st);
    };
    auto check_device = [&]() {
        hpsi_batch_run(h_x.b, st);
        hpsi_batch_run(h_y.b, st);
        zgemm_nt_jobs(nt_yy.h, nt_yy.d.as<NtJob>(), dm, true, false, false, st);
        dense_eigh_jobs(nb, eig.d.as<DenseJob>(), dm, n, st);
        zgemm_nn_jobs_launch(nn_rr3.h, nn_rr3.d.as<NnJob>(), dm, -1, false, st);
        band_batch_copy(dp, dm, n, nb, maxnpw, 3, c_xyax, d_xyax, st);
        zgemm_nn_jobs_launch(nn_pg.h, nn_pg.d.as<NnJob>(), dm, -1, false, st);
        band_batch_copy(dp, dm, n, nb, maxnpw, 2, c_pg, d_pg, st);
        zgemm_nt_jobs(nt_xy.h, nt_xy.d.as<NtJob>(), dm, true, false, false, st);
        dense_eigh_jobs(nb, eig.d.as<DenseJob>(), dm, n, st);
        zgemm_nn_jobs_launch(nn_x.h, nn_x.d.as<NnJob>(), dm, -1, false, st);
        zgemm_nn_jobs_launch(nn_y.h, nn_y.d.as<NnJob>(), dm, -1, false, st);
        band(BandOp::Resid, kBT2, kBT1);
        band(BandOp::MuTband);
        band(BandOp::GzOld);
        band_batch_gather(dp, n, nb, d_out.as<double>(), d_sout.as<int>(), st);
    };
    // one recorded round per segment length
    struct Round {
        int len;
        hipGraph_t g = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<Round> rounds;
    struct Guard {
        std::vector<Round> &r;
        hipStream_t cap = nullptr;
        ~Guard() {
            for (Round &x : r) {
                if (x.exec) (void)hipGraphExecDestroy(x.exec);
                if (x.g) (void)hipGraphDestroy(x.g);
            }
            if (cap) (void)hipStreamDestroy(cap);
        }
    } guard{rounds};
    PW_HIP(hipStreamCreateWithFlags(&guard.cap, hipStreamNonBlocking));
    std::vector<double> out((size_t)n * 2 * nb);
    std::vector<int> sout((size_t)n * 8);
    for (;;) {
        int len = 0;
        for (int p = 0; p < n; ++p)
            if (mask[p]) { len = runs[p]->segment_length(); break; }
        if (!len) break;
        Round *rd = nullptr;
        for (Round &x : rounds)
            if (x.len == len) rd = &x;
        if (!rd) {
            rounds.push_back(Round{len});
            rd = &rounds.back();
            const hipStream_t keep = st;
            st = guard.cap;
            PW_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            try {
                for (int k = 0; k < len; ++k) iteration();
                check_device();
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(st, &g);
                if (g) (void)hipGraphDestroy(g);
                st = keep;
                throw;
            }
            PW_HIP(hipStreamEndCapture(st, &rd->g));
            st = keep;
            PW_HIP(hipGraphInstantiate(&rd->exec, rd->g, nullptr, nullptr, 0));
        }
        PW_HIP(hipGraphLaunch(rd->exec, st));
        PW_HIP(hipMemcpyAsync(out.data(), d_out.p, out.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        PW_HIP(hipMemcpyAsync(sout.data(), d_sout.p, sout.size() * sizeof(int), hipMemcpyDeviceToHost, st));
        PW_HIP(hipStreamSynchronize(st));
        bool changed = false, any_save = false;
        for (int p = 0; p < n; ++p) {
            save[p] = 0;
            if (!mask[p]) continue;
            FcgRun &r = *runs[p];
            r.it += len;
            r.n_hpsi += (int64_t)2 * nb * len + 2 * nb;
            std::copy(out.begin() + (size_t)p * 2 * nb, out.begin() + (size_t)p * 2 * nb + nb, r.h_lam.begin());
            std::copy(out.begin() + (size_t)p * 2 * nb + nb, out.begin() + (size_t)(p + 1) * 2 * nb, r.h_res.begin());
            for (int k = 0; k < 8; ++k) r.h_status[k] = sout[(size_t)p * 8 + k];
            const bool more = r.decide(true);
            if (!more) {
                mask[p] = 0;
                changed = true;
            } else if (o.recover && !r.restarted) {
                save[p] = 1;
                any_save = true;
            }
        }
        if (any_save) {
            PW_HIP(hipMemcpyAsync(d_save.p, save.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
            band_batch_save(dp, d_save.as<int>(), n, nb, maxnpw, st);
        }
        if (changed) PW_HIP(hipMemcpyAsync(d_mask.p, mask.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
        PW_HIP(hipStreamSynchronize(st));   // the host vectors outlive the copies
    }
}

pw_status batch_solve(int nprob, pw_ctx *const *ctxs, const double *e_ref, int nb, void *const *psi,
                      const int64_t *ld, double *const *eig, double *const *resid, const pw_cg_opts &o,
                      pw_cg_stats *stats, int32_t *status, hipStream_t st) {
    std::string why;
    const bool fused = o.batch_launch == 2 && fused_ok(nprob, ctxs, nb, o, &why);
    const bool each = o.batch_launch != 0;   // launch each problem's recorded segment, or one graph of them all
    if (o.batch_launch == 2 && !fused && o.verbose) fprintf(stderr, "[pw] batch: not fused (%s)\n", why.c_str());
    BatchRes R;
    R.items.resize(nprob);
    PW_HIP(hipStreamCreateWithFlags(&R.cap, hipStreamNonBlocking));
    for (int p = 0; p < nprob; ++p) {
        BatchItem &b = R.items[p];
        b.run.reset(new FcgRun(ctxs[p], e_ref[p], nb, psi[p], ld[p], eig ? eig[p] : nullptr,
                               resid ? resid[p] : nullptr, o, stats ? &stats[p] : nullptr, st));
        b.run->swap_free = true;
        b.run->setup();
    }
    if (fused) {
        std::vector<FcgRun *> runs;
        for (BatchItem &b : R.items) runs.push_back(b.run.get());
        fused_solve(runs, o, st);
    }
    for (; !fused;) {
        bool any = false, changed = false;
        for (BatchItem &b : R.items) {
            hipGraph_t want = nullptr;
            if (b.active) {
                FcgRun &r = *b.run;
                const int len = r.segment_length();
                SegGraph *sg = nullptr;
                for (SegGraph &c : b.segs)
                    if (c.len == len && c.low == r.use_mixed && c.kind == r.pa.kind) sg = &c;
                if (!sg) {
                    b.segs.push_back(record_segment(r, len, R.cap));
                    sg = &b.segs.back();
                    if (each) PW_HIP(hipGraphInstantiate(&sg->exec, sg->g, nullptr, nullptr, 0));
                }
                if (each) PW_HIP(hipGraphLaunch(sg->exec, st));
                want = sg->g;
                b.len = len;
                b.hpsi = sg->hpsi;
                any = true;
            }
            if (want != b.cur) changed = true;
            b.cur = want;
        }
        if (!any) break;
        if (!each && (changed || !R.exec)) {
            if (R.exec) {
                PW_HIP(hipGraphExecDestroy(R.exec));
                R.exec = nullptr;
            }
            hipGraph_t parent = nullptr;
            PW_HIP(hipGraphCreate(&parent, 0));
            try {
                for (BatchItem &b : R.items) {
                    if (!b.cur) continue;
                    hipGraphNode_t node;
                    PW_HIP(hipGraphAddChildGraphNode(&node, parent, nullptr, 0, b.cur));
                }
                PW_HIP(hipGraphInstantiate(&R.exec, parent, nullptr, nullptr, 0));
            } catch (...) {
                (void)hipGraphDestroy(parent);
                throw;
            }
            PW_HIP(hipGraphDestroy(parent));
        }
        if (!each) PW_HIP(hipGraphLaunch(R.exec, st));
        for (BatchItem &b : R.items) {
            if (!b.active) continue;
            b.run->it += b.len;
            b.run->n_hpsi += b.hpsi;
        }
        for (BatchItem &b : R.items)
            if (b.active && !b.run->check_host()) b.active = false;
    }
    pw_status worst = PW_OK;
    for (int p = 0; p < nprob; ++p) {
        const pw_status r = R.items[p].run->finish();
        if (status) status[p] = r;
        if (r != PW_OK && (worst == PW_OK || worst == PW_ENOCONV)) worst = r;
    }
    if (fused && stats)
        for (int p = 0; p < nprob; ++p) stats[p].fused = 1;
    return worst;
}

// Training tables of one snapshot (see pw_mlp_harvest in pw.h), using the solver's
// blocks as scratch.
void mlp_harvest(pw_ctx *ctx, double E, int nb, const void *xs, const void *xc, int64_t ld, double delta_e,
                 double delta, double *tabs, double *tband_out, hipStream_t st) {
    const int npw = ctx->basis.npw;
    Solver *s = solver_get(ctx, nb, false);
    const int64_t L = npw;
    void *X = s->X.p, *Y = s->Y.p, *AX = s->AX.p, *G = s->G.p, *Z = s->Z.p, *T1 = s->T1.p, *Xc = s->T2.p;
    double *v = (double *)s->vec.p;
    double *mu = v, *tband = v + nb, *gz = v + 2 * nb, *gzo = v + 3 * nb;
    double2 *Wm = (double2 *)s->small.p;
    BandRed br{(double *)s->red.p, s->nsplit};
    copy_block(nb, npw, xs, ld, X, L, st);
    copy_block(nb, npw, xc, ld, Xc, L, st);
    hpsi_any(ctx, PW_C128, nb, X, L, Y, L, E, st);
    hpsi_any(ctx, PW_C128, nb, Y, L, AX, L, E, st);
    red_mu_tband(nb, npw, Y, X, L, ctx->d_kin.as<double>(), mu, tband, br, st);
    PrecArgs pa{};
    pa.kind = 1;                                                    // K0 = the paper's M(G)
    pa.kin = ctx->d_kin.as<double>();
    pa.e_ref = E;
    pa.de2 = delta_e * delta_e;
    pa.tband = tband;
    pa.nb = nb;
    fill_zero(G, (size_t)nb * npw * 16, st);
    red_grad(nb, npw, X, AX, G, Z, L, mu, pa, gz, gzo, br, st);     // G = A x - mu x, Z = K0 o G
    // E = X - W . Xc with W[i][j] = <xc_j | x_i>: the part of x_i outside span(Xc)
    zgemm_nt(nb, nb, npw, true, Xc, L, X, L, 1.0, nullptr, 0.0, Wm, nb, true, ctx->d_partial.p, st);
    copy_block(nb, npw, X, L, T1, L, st);
    zgemm_nn_launch(nb, npw, nb, Wm, nb, Xc, L, -1.0, 1.0, T1, L, st, false, ctx->rot_tune.get(nb));
    shell_tables((int)ctx->basis.shell_t.size(), nb, npw, ctx->d_shell_off.as<int32_t>(),
                 ctx->d_shell_pw.as<int32_t>(), T1, Z, L, ctx->d_shell_t.as<double>(), E, delta, tabs, st);
    PW_HIP(hipMemcpyAsync(tband_out, tband, nb * sizeof(double), hipMemcpyDeviceToDevice, st));
}

}  // namespace pw

extern "C" {

pw_status pw_mlp_harvest(pw_ctx *ctx, double e_ref, int32_t nb, const void *x_snap, const void *x_conv, int64_t ld,
                         double delta_e, double weight_delta, double *tabs, double *tband, void *stream) {
    try {
        PW_CHECK(ctx && x_snap && x_conv && tabs && tband, PW_EINVAL, "null argument");
        PW_CHECK(ctx->flags & PW_PREP_C128, PW_EUNSUPPORTED, "harvest needs a complex128 context");
        PW_CHECK(nb >= 1 && nb <= ctx->max_bands && nb <= 1024 && ld >= ctx->basis.npw, PW_EINVAL,
                 "bad harvest sizes");
        PW_CHECK(delta_e > 0.0, PW_EINVAL, "delta_e must be positive");
        pw::mlp_harvest(ctx, e_ref, nb, x_snap, x_conv, ld, delta_e, weight_delta, tabs, tband, (hipStream_t)stream);
        return PW_OK;
    } catch (const pw::Fail &f) {
        return f.st;
    }
}

void pw_cg_opts_default(pw_cg_opts *o) {
    if (!o) return;
    o->tol = 1e-6;
    o->maxit = 20000;
    o->precond = 0;
    o->delta_e = 1.0;
    o->precision = 0;
    o->check_every = 20;
    o->verbose = 0;
    o->mixed_switch = 5e-4;
    o->stall_checks = 5;
    o->snap_buf = nullptr;
    o->snap_every = 0;
    o->snap_cap = 0;
    o->nconv = 0;
    o->batch_launch = 2;
    o->learned_stall = 25;
    o->recover = 1;
    o->fault_check = 0;
}

pw_status pw_folded_cg_solve(pw_ctx *ctx, double e_ref, int32_t nb, void *psi, int64_t ld, double *eig,
                             double *resid, const pw_cg_opts *opts, pw_cg_stats *stats, void *stream) {
    try {
        PW_CHECK(ctx && psi, PW_EINVAL, "null argument");
        PW_CHECK(ctx->flags & PW_PREP_C128, PW_EUNSUPPORTED, "the solver needs a complex128 context");
        PW_CHECK(nb >= 1 && nb <= ctx->max_bands && nb <= 1024, PW_EINVAL, "nb %d must be in [1, min(max_bands, 1024)]",
                 nb);
        PW_CHECK(nb <= ctx->basis.npw, PW_EINVAL, "more bands than plane waves");
        PW_CHECK(ld >= ctx->basis.npw, PW_EINVAL, "ld < npw");
        PW_CHECK(std::isfinite(e_ref), PW_ENAN, "non-finite e_ref");
        pw_cg_opts o;
        pw_cg_opts_default(&o);
        if (opts) o = *opts;
        PW_CHECK(o.tol > 0 && o.maxit >= 1 && o.check_every >= 1, PW_EINVAL, "bad solver options");
        PW_CHECK(o.precond >= 0 && o.precond <= 2, PW_EINVAL, "preconditioner %d unknown", o.precond);
        PW_CHECK(o.precond != 2 || ctx->d_mlp.p, PW_EUNSUPPORTED, "precond 2 needs pw_mlp_set first");
        PW_CHECK(o.snap_every <= 0 || (o.snap_buf && o.snap_cap >= 0), PW_EINVAL, "snapshots need a buffer");
        PW_CHECK(o.precision == 0 || o.precision == 1, PW_EINVAL, "precision must be 0 or 1");
        if (o.precision == 1)
            PW_CHECK(ctx->flags & PW_PREP_C64, PW_EUNSUPPORTED, "mixed precision needs PW_PREP_C64");
        return pw::folded_cg(ctx, e_ref, nb, psi, ld, eig, resid, o, stats, (hipStream_t)stream);
    } catch (const pw::Fail &f) {
        return f.st;
    } catch (...) {
        pw::set_error("unexpected exception in pw_folded_cg_solve");
        return PW_EINVAL;
    }
}

pw_status pw_batch_solve(int32_t nprob, pw_ctx *const *ctx, const double *e_ref, int32_t nb, void *const *psi,
                         const int64_t *ld, double *const *eig, double *const *resid, const pw_cg_opts *opts,
                         pw_cg_stats *stats, int32_t *status, void *stream) {
    try {
        PW_CHECK(nprob >= 1 && ctx && e_ref && psi && ld, PW_EINVAL, "null argument or nprob < 1");
        pw_cg_opts o;
        pw_cg_opts_default(&o);
        if (opts) o = *opts;
        PW_CHECK(o.tol > 0 && o.maxit >= 1 && o.check_every >= 1, PW_EINVAL, "bad solver options");
        PW_CHECK(o.precond >= 0 && o.precond <= 2, PW_EINVAL, "preconditioner %d unknown", o.precond);
        PW_CHECK(o.snap_every <= 0, PW_EINVAL, "snapshots are not taken in batched solves");
        PW_CHECK(o.precision == 0 || o.precision == 1, PW_EINVAL, "precision must be 0 or 1");
        for (int p = 0; p < nprob; ++p) {
            pw_ctx *c = ctx[p];
            PW_CHECK(c && psi[p], PW_EINVAL, "problem %d: null context or block", p);
            for (int q = 0; q < p; ++q) PW_CHECK(ctx[q] != c, PW_EINVAL, "problems %d and %d share a context", q, p);
            PW_CHECK(c->flags & PW_PREP_C128, PW_EUNSUPPORTED, "problem %d: the solver needs a complex128 context", p);
            PW_CHECK(nb >= 1 && nb <= c->max_bands && nb <= 1024 && nb <= c->basis.npw, PW_EINVAL,
                     "problem %d: bad nb %d", p, nb);
            PW_CHECK(ld[p] >= c->basis.npw, PW_EINVAL, "problem %d: ld < npw", p);
            PW_CHECK(std::isfinite(e_ref[p]), PW_ENAN, "problem %d: non-finite e_ref", p);
            PW_CHECK(o.precond != 2 || c->d_mlp.p, PW_EUNSUPPORTED, "problem %d: precond 2 needs pw_mlp_set", p);
            PW_CHECK(o.precision == 0 || (c->flags & PW_PREP_C64), PW_EUNSUPPORTED,
                     "problem %d: mixed precision needs PW_PREP_C64", p);
        }
        return pw::batch_solve(nprob, ctx, e_ref, nb, psi, ld, eig, resid, o, stats, status, (hipStream_t)stream);
    } catch (const pw::Fail &f) {
        return f.st;
    } catch (...) {
        pw::set_error("unexpected exception in pw_batch_solve");
        return PW_EINVAL;
    }
}

}  // extern "C"
