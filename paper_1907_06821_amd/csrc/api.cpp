// C ABI of libpw: contexts, H psi, wave <-> grid transforms, orthonormalisation.
#include <cmath>
#include <cstring>
#include <memory>

#include "kernels.h"

namespace pw {
const char *last_error();
void build_projectors(int npw, int natom, int nl, const int32_t *d_miller, const pw_cell &c, const double *d_pos,
                      double sigma, void *beta, hipStream_t st);
void build_vz(int n0, int n1, int n2, const double *v, double *vz64, float *vz32, hipStream_t st);
void beta_to_bf16(int rows, int npw, int64_t ldp, const void *src, void *re, void *im, hipStream_t st, bool panel);
void solver_destroy(Solver *s);

void DevBuf::alloc(size_t b) {
    free_();
    if (b == 0) return;
    b = (b + 255) & ~size_t(255);
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
        p = nullptr;
        set_error("hipMalloc(%zu bytes) failed: %s", b, hipGetErrorString(e));
        throw Fail{PW_ENOMEM};
    }
    bytes = b;
}

void DevBuf::free_() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

template <typename T> static void upload(DevBuf &d, const std::vector<T> &h, int64_t &acct) {
    d.alloc(h.size() * sizeof(T));
    acct += (int64_t)d.bytes;
    if (!h.empty()) PW_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}

static void twiddles(int n, std::vector<double> &t64, std::vector<float> &t32) {
    t64.resize(2 * n);
    t32.resize(2 * n);
    for (int t = 0; t < n; ++t) {
        const long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)t / (long double)n;
        const double c = (double)cosl(ang), s = (double)-sinl(ang);
        t64[2 * t] = c;
        t64[2 * t + 1] = s;
        t32[2 * t] = (float)cosl(ang);
        t32[2 * t + 1] = (float)-sinl(ang);
    }
}

// Largest split-K scratch any call can need: the split count grows as the output
// shrinks, so take the maximum over every band count up to max_bands.
size_t hpsi_partial_bytes(const pw_ctx *ctx) {
    size_t b = 0;
    const int npw = ctx->basis.npw;
    const bool c128 = ctx->flags & PW_PREP_C128, c64 = ctx->flags & PW_PREP_C64;
    for (int n = 1; n <= ctx->max_bands; ++n) {
        if (ctx->nproj && c128) {
            b = std::max(b, nt_partial_bytes(ctx->nproj, n, npw));
            if (ctx->beta_otf) {
                // the chunk of rows and the last, shorter one
                b = std::max(b, nt_partial_bytes(ctx->otf_atoms * ctx->nl, n, npw));
                const int tail = ctx->natom % ctx->otf_atoms;
                if (tail) b = std::max(b, nt_partial_bytes(tail * ctx->nl, n, npw));
            }
        }
        if (ctx->nproj && c64) b = std::max(b, cnt_partial_bytes(ctx->nproj, n, npw, ctx->max_bands));
        if (c128) b = std::max(b, nt_partial_bytes(n, n, npw));
    }
    return b;
}

// The local and kinetic part of (H - shift) psi: the three FFT passes, cols_bands bands per launch
template <typename T>
static void hpsi_local(pw_ctx *ctx, int nb, const void *psi, int64_t ld, void *out, int64_t ldo, double shift,
                       hipStream_t st) {
    const double scale = 1.0 / ((double)ctx->cell.n[0] * ctx->cell.n[1] * ctx->cell.n[2]);
    const size_t es = 2 * sizeof(T);
    for (int b0 = 0; b0 < nb; b0 += ctx->cols_bands) {
        const int n = std::min(ctx->cols_bands, nb - b0);
        const char *pi = (const char *)psi + (size_t)b0 * ld * es;
        char *po = (char *)out + (size_t)b0 * ldo * es;
        { ProfScope p(ctx, 0, st); launch_zinv<T>(ctx, n, pi, ld, ctx->d_cols.p, st); }
        { ProfScope p(ctx, 1, st); launch_xy<T, 0>(ctx, n, ctx->d_cols.p, nullptr, st); }
        {
            ProfScope p(ctx, 2, st);
            launch_zfwd<T>(ctx, n, ctx->d_cols.p, pi, ld, ctx->d_kin.as<double>(), shift, scale, po, ldo, st);
        }
    }
}

// Nonlocal term with projector rows generated per call: for each chunk of otf_atoms
// atoms, the rows beta_p(G) of its projectors are written to the chunk buffer, then
// projT[b][p] = D_p <beta_p|psi_b> and out += projT . beta over that chunk's rows.
static void nonlocal_otf(pw_ctx *ctx, int nb, const void *psi, int64_t ld, void *out, int64_t ldo, hipStream_t st) {
    const int npw = ctx->basis.npw, nl = ctx->nl;
    double2 *proj = ctx->d_proj.as<double2>();
    for (int a0 = 0; a0 < ctx->natom; a0 += ctx->otf_atoms) {
        const int na = std::min(ctx->otf_atoms, ctx->natom - a0), p0 = a0 * nl, rows = na * nl;
        build_projectors(npw, na, nl, ctx->d_miller.as<int32_t>(), ctx->cell, ctx->d_pos.as<double>() + 3 * a0,
                         ctx->sigma, ctx->d_beta_chunk.p, st);
        {
            ProfScope p(ctx, 3, st);
            zgemm_nt(rows, nb, npw, true, ctx->d_beta_chunk.p, npw, psi, ld, 1.0, ctx->d_dproj.as<double>() + p0, 0.0,
                     proj + p0, ctx->nproj, true, ctx->d_partial.p, st, true);
        }
        ProfScope p(ctx, 4, st);
        zgemm_nn_launch(nb, npw, rows, proj + p0, ctx->nproj, ctx->d_beta_chunk.p, npw, 1.0, 1.0, out, ldo, st, true);
    }
}

// (H - shift) psi for one chunk of at most max_bands bands, complex128
static void hpsi_c128(pw_ctx *ctx, int nb, const void *psi, int64_t ld, void *out, int64_t ldo, double shift,
                      hipStream_t st) {
    const int npw = ctx->basis.npw;
    hpsi_local<double>(ctx, nb, psi, ld, out, ldo, shift, st);
    if (ctx->nproj && ctx->beta_otf) {
        nonlocal_otf(ctx, nb, psi, ld, out, ldo, st);
    } else if (ctx->nproj) {
        // projT[b][p] = D_p <beta_p | psi_b>, then out += projT . beta; band counts just past
        // 128 as the first 128 bands (tiles of the three-product form) and the rest
        const int nb1 = proj_band_split(nb);
        double2 *proj = ctx->d_proj.as<double2>();
        {
            ProfScope p(ctx, 3, st);
            for (int b0 = 0; b0 < nb; b0 += nb1)
                zgemm_nt(ctx->nproj, std::min(nb1, nb - b0), npw, true, ctx->d_beta64.p, npw,
                         (const double2 *)psi + (size_t)b0 * ld, ld, 1.0, ctx->d_dproj.as<double>(), 0.0,
                         proj + (size_t)b0 * ctx->nproj, ctx->nproj, true, ctx->d_partial.p, st, true);
        }
        ProfScope p(ctx, 4, st);
        for (int b0 = 0; b0 < nb; b0 += nb1) {
            const int n = std::min(nb1, nb - b0);
            zgemm_nn_launch(n, npw, ctx->nproj, proj + (size_t)b0 * ctx->nproj, ctx->nproj, ctx->d_beta64.p, npw, 1.0,
                            1.0, (double2 *)out + (size_t)b0 * ldo, ldo, st, true, ctx->nn_tune.get(n));
        }
    }
}

static void hpsi_c64(pw_ctx *ctx, int nb, const void *psi, int64_t ld, void *out, int64_t ldo, double shift,
                     hipStream_t st) {
    const int npw = ctx->basis.npw;
    hpsi_local<float>(ctx, nb, psi, ld, out, ldo, shift, st);
    if (ctx->nproj) {
        {
            ProfScope p(ctx, 3, st);
            proj_bf16(ctx->nproj, nb, npw, ctx->max_bands, ctx->d_beta_bf16.p, ctx->d_dproj32.as<float>(), psi, ld,
                      ctx->d_bf16_ws.p, ctx->d_partial.p, st, ctx->bf16_variant);
        }
        ProfScope p(ctx, 4, st);
        backproj_bf16(ctx->nproj, nb, npw, ctx->max_bands, ctx->d_betaT_bf16.p, ctx->d_bf16_ws.p, out, ldo, st,
                      ctx->bf16_variant);
    }
}

void hpsi_any(pw_ctx *ctx, pw_dtype dt, int nb, const void *psi, int64_t ld, void *out, int64_t ldo, double shift,
              hipStream_t st) {
    const size_t es = dt == PW_C128 ? 16 : 8;
    for (int b0 = 0; b0 < nb; b0 += ctx->max_bands) {
        const int nbc = std::min(ctx->max_bands, nb - b0);
        const char *pi = (const char *)psi + (size_t)b0 * ld * es;
        char *po = (char *)out + (size_t)b0 * ldo * es;
        if (dt == PW_C128) hpsi_c128(ctx, nbc, pi, ld, po, ldo, shift, st);
        else hpsi_c64(ctx, nbc, pi, ld, po, ldo, shift, st);
    }
}

// pw_orthonormalize's small work: S and T (nb x nb each), then the Cholesky work
static size_t ortho_small_bytes(int nb) {
    return ((size_t)2 * nb * nb * 16 + chol_inv_work_bytes(nb) + 255) / 256 * 256;
}

// Psi <- Psi L^{-H} for a complex128 block, using ws (>= nb*npw complex128) as scratch
void orthonormalize_c128(pw_ctx *ctx, int nb, void *psi, int64_t ld, void *ws, void *small, int *d_status,
                         hipStream_t st) {
    const int npw = ctx->basis.npw;
    double2 *S = (double2 *)small;
    double2 *T = S + (size_t)nb * nb;
    double2 *W = T + (size_t)nb * nb;     // chol_inv_work_bytes(nb)
    zgemm_nt(nb, nb, npw, true, psi, ld, psi, ld, 1.0, nullptr, 0.0, S, nb, false, ctx->d_partial.p, st, false, true);
    chol_inv(nb, S, nb, W, T, d_status, st);
    zgemm_nn_launch(nb, npw, nb, T, nb, psi, ld, 1.0, 0.0, ws, npw, st, false, ctx->rot_tune.get(nb), true);
    copy_block(nb, npw, ws, npw, psi, ld, st);
}

}  // namespace pw

using namespace pw;

#define PW_API_BEGIN try {
#define PW_API_END                                                       \
    }                                                                    \
    catch (const Fail &f) { return f.st; }                               \
    catch (const std::bad_alloc &) { set_error("host allocation failed"); return PW_ENOMEM; } \
    catch (...) { set_error("unexpected exception"); return PW_EINVAL; } \
    return PW_OK;

extern "C" {

const char *pw_last_error(void) { return pw::last_error(); }

pw_status pw_basis_size(const pw_cell *cell, int32_t *npw) {
    PW_API_BEGIN
    PW_CHECK(cell && npw, PW_EINVAL, "null argument");
    std::vector<int32_t> m;
    enumerate_miller(*cell, m);
    *npw = (int32_t)(m.size() / 3);
    PW_API_END
}

pw_status pw_basis_miller(const pw_cell *cell, int32_t *miller, int32_t npw) {
    PW_API_BEGIN
    PW_CHECK(cell && miller, PW_EINVAL, "null argument");
    std::vector<int32_t> m;
    enumerate_miller(*cell, m);
    PW_CHECK((int64_t)m.size() == 3 * (int64_t)npw, PW_EINVAL, "npw %d does not match the basis (%zu)", npw,
             m.size() / 3);
    std::memcpy(miller, m.data(), m.size() * sizeof(int32_t));
    PW_API_END
}

pw_status pw_ctx_create(const pw_cell *cell, const pw_potential *pot, int32_t max_bands, int32_t flags, void *stream,
                        pw_ctx **out) {
    PW_API_BEGIN
    PW_CHECK(cell && pot && out, PW_EINVAL, "null argument");
    PW_CHECK(max_bands >= 1 && max_bands <= 8192, PW_EINVAL, "max_bands %d out of range", max_bands);
    PW_CHECK(pot->v_r, PW_EINVAL, "v_r is null");
    PW_CHECK(pot->natom >= 0 && (pot->natom == 0 || (pot->pos && pot->d)), PW_EINVAL, "bad atom arrays");
    PW_CHECK(pot->nl == 0 || pot->nl == 1 || pot->nl == 4, PW_EINVAL, "nl must be 0, 1 or 4");
    PW_CHECK(!(flags & ~(PW_PREP_C128 | PW_PREP_C64 | PW_PREP_C128_OTF)), PW_EINVAL, "unknown context flags %d",
             flags);
    if (flags & PW_PREP_C128_OTF) flags |= PW_PREP_C128;
    if (!(flags & (PW_PREP_C128 | PW_PREP_C64))) flags |= PW_PREP_C128;
    PW_CHECK(pot->natom == 0 || pot->nl == 0 || std::isfinite(pot->sigma), PW_ENAN, "non-finite projector width");
    *out = nullptr;
    std::unique_ptr<pw_ctx> c(new pw_ctx());
    hipStream_t st = (hipStream_t)stream;
    c->cell = *cell;
    for (int a = 0; a < 3; ++a) c->plan[a] = make_plan(cell->n[a]);
    c->basis = build_basis(*cell);
    c->max_bands = max_bands;
    c->flags = flags;
    c->natom = pot->nl ? pot->natom : 0;
    c->nl = pot->nl;
    c->nproj = c->natom * c->nl;
    PW_HIP(hipGetDevice(&c->device));
    const Basis &b = c->basis;
    const int n0 = cell->n[0], n1 = cell->n[1], n2 = cell->n[2];
    int64_t acct = 0;
    upload(c->d_kin, b.kin, acct);
    upload(c->d_colstart, b.col_start, acct);
    std::vector<int32_t> zmap(b.npw), colpos(b.ncols), colslot(b.ncols);
    const int rowlo = ((b.n0min % n0) + n0) % n0;
    const int qm = std::max(1, n1 / 4);      // the four-lane xy kernel's plane layout (square planes)
    for (int col = 0; col < b.ncols; ++col) {
        colpos[col] = b.col_i0[col] * (n1 + 1) + b.col_i1[col];
        const int i1 = b.col_i1[col];
        colslot[col] = ((b.col_i0[col] - rowlo + n0) % n0) * quad_rs(qm) + i1 + (i1 / qm) * quad_pad(qm);
        for (int g = b.col_start[col]; g < b.col_start[col + 1]; ++g) {
            const int n2v = b.miller[3 * g + 2];
            zmap[g] = (col % c->cb) * (n2 + 1) + ((n2v % n2) + n2) % n2;
        }
    }
    upload(c->d_zmap, zmap, acct);
    upload(c->d_colpos, colpos, acct);
    upload(c->d_colslot, colslot, acct);
    upload(c->d_shell, b.shell, acct);
    upload(c->d_shell_t, b.shell_t, acct);
    {
        // plane waves grouped by shell (CSR), for the learned preconditioner's tables
        const int ns = (int)b.shell_t.size();
        std::vector<int32_t> off(ns + 1, 0), pws(b.npw);
        for (int g = 0; g < b.npw; ++g) ++off[b.shell[g] + 1];
        for (int s = 0; s < ns; ++s) off[s + 1] += off[s];
        std::vector<int32_t> fill(off.begin(), off.end() - 1);
        for (int g = 0; g < b.npw; ++g) pws[fill[b.shell[g]]++] = g;
        upload(c->d_shell_off, off, acct);
        upload(c->d_shell_pw, pws, acct);
    }
    for (int a = 0; a < 3; ++a) {
        std::vector<double> t64;
        std::vector<float> t32;
        twiddles(cell->n[a], t64, t32);
        upload(c->d_tw64[a], t64, acct);
        upload(c->d_tw32[a], t32, acct);
    }
    // V(r) is checked for NaN/Inf on the host (one copy), then kept z-major per prepared precision
    const int64_t ngrid = (int64_t)n0 * n1 * n2;
    {
        std::vector<double> hv(ngrid);
        PW_HIP(hipMemcpy(hv.data(), pot->v_r, ngrid * sizeof(double), hipMemcpyDeviceToHost));
        for (double v : hv) PW_CHECK(std::isfinite(v), PW_ENAN, "non-finite local potential sample");
    }
    if (flags & PW_PREP_C128) c->d_vz64.alloc(ngrid * 8);
    if (flags & PW_PREP_C64) c->d_vz32.alloc(ngrid * 4);
    acct += c->d_vz64.bytes + c->d_vz32.bytes;
    build_vz(n0, n1, n2, pot->v_r, c->d_vz64.as<double>(), c->d_vz32.as<float>(), st);
    if (c->nproj) {
        c->dproj.assign(pot->d, pot->d + c->nproj);
        for (double d : c->dproj) PW_CHECK(std::isfinite(d), PW_ENAN, "non-finite KB strength");
        upload(c->d_dproj, c->dproj, acct);
        std::vector<float> d32(c->dproj.begin(), c->dproj.end());
        upload(c->d_dproj32, d32, acct);
        std::vector<int32_t> mil(b.miller);
        DevBuf d_mil, d_pos;
        int64_t tmp = 0;
        upload(d_mil, mil, tmp);
        std::vector<double> pos(pot->pos, pot->pos + 3 * c->natom);
        upload(d_pos, pos, tmp);
        c->beta_otf = flags & PW_PREP_C128_OTF;
        const bool c128 = (flags & PW_PREP_C128) && !c->beta_otf;   // a stored complex128 table
        if (c->beta_otf) {
            // rows of otf_atoms atoms per chunk: about kOtfBytes of scratch, at least one atom
            constexpr size_t kOtfBytes = size_t(4) << 30;
            const size_t per_atom = (size_t)c->nl * b.npw * 16;
            c->otf_atoms = (int)std::max<size_t>(1, std::min<size_t>(c->natom, kOtfBytes / per_atom));
            c->sigma = pot->sigma;
            c->d_beta_chunk.alloc((size_t)c->otf_atoms * per_atom);
            upload(c->d_miller, mil, acct);
            upload(c->d_pos, pos, acct);
            acct += c->d_beta_chunk.bytes;
        }
        if (c128) {
            c->d_beta64.alloc((size_t)c->nproj * b.npw * 16);
            build_projectors(b.npw, c->natom, c->nl, d_mil.as<int32_t>(), *cell, d_pos.as<double>(), pot->sigma,
                             c->d_beta64.p, st);
        }
        if (flags & PW_PREP_C64) {
            c->ldb16 = ((b.npw + 63) / 64) * 64;
            // contexts of more than 144 bands keep the planes in 16-row panels (rows padded to 16)
            const bool panel = bf16_panels(max_bands);
            const size_t prow = (size_t)bf16_rows(c->nproj, max_bands);
            c->d_beta_bf16.alloc((size_t)2 * prow * c->ldb16 * 2);
            char *br = (char *)c->d_beta_bf16.p, *bi = br + prow * c->ldb16 * 2;
            if (prow > (size_t)c->nproj) fill_zero(c->d_beta_bf16.p, c->d_beta_bf16.bytes, st);
            const size_t tplane = (size_t)bf16_ld(b.npw) * bf16_ld(c->nproj) * 2;
            c->d_betaT_bf16.alloc(2 * tplane);
            char *tr = (char *)c->d_betaT_bf16.p, *ti = tr + tplane;
            if (c128) {
                beta_to_bf16(c->nproj, b.npw, c->ldb16, c->d_beta64.p, br, bi, st, panel);
                beta_to_bf16_t(c->nproj, b.npw, c->d_beta64.p, tr, ti, st, panel);
            } else {
                // complex64 only: the FP64 rows are built and rounded 64 atoms at a time, so the FP64
                // table (16 nproj npw bytes) never exists whole; the BF16 planes are the same bits
                constexpr int kAtomChunk = 64;
                DevBuf chunk;
                chunk.alloc((size_t)std::min(c->natom, kAtomChunk) * c->nl * b.npw * 16);
                for (int a0 = 0; a0 < c->natom; a0 += kAtomChunk) {
                    const int na = std::min(kAtomChunk, c->natom - a0), p0 = a0 * c->nl, rows = na * c->nl;
                    build_projectors(b.npw, na, c->nl, d_mil.as<int32_t>(), *cell, d_pos.as<double>() + 3 * a0,
                                     pot->sigma, chunk.p, st);
                    beta_to_bf16(rows, b.npw, c->ldb16, chunk.p, br + (size_t)p0 * c->ldb16 * 2,
                                 bi + (size_t)p0 * c->ldb16 * 2, st, panel);
                    beta_to_bf16_t_rows(c->nproj, p0, rows, b.npw, chunk.p, tr, ti, st, panel);
                }
                PW_HIP(hipStreamSynchronize(st));     // the chunk buffer dies here
            }
            c->d_bf16_ws.alloc(bf16_scratch_bytes(c->nproj, b.npw, max_bands));
            if (panel) fill_zero(c->d_bf16_ws.p, c->d_bf16_ws.bytes, st);   // padding rows of the last panel
            acct += c->d_beta_bf16.bytes + c->d_betaT_bf16.bytes + c->d_bf16_ws.bytes;
        }
        acct += c->d_beta64.bytes;
        PW_HIP(hipStreamSynchronize(st));   // d_mil, d_pos die here
    }
    // column grid for cols_bands bands of the widest prepared dtype: all max_bands bands up to
    // kColsBytes, else the FFT passes run that many bands per launch
    {
        constexpr size_t kColsBytes = size_t(4) << 30;
        const size_t per_band = (size_t)n2 * b.ncols * ((flags & PW_PREP_C128) ? 16 : 8);
        c->cols_bands = (int)std::max<size_t>(1, std::min<size_t>(max_bands, kColsBytes / per_band));
        c->d_cols.alloc((size_t)c->cols_bands * per_band);
    }
    c->d_proj.alloc((size_t)max_bands * std::max(1, c->nproj) * 16);
    c->d_partial.alloc(hpsi_partial_bytes(c.get()));
    // pw_orthonormalize's block scratch: complex128 contexts with a stored table only (a
    // PW_PREP_C128_OTF context allocates it on its first pw_orthonormalize call)
    if ((flags & PW_PREP_C128) && !c->beta_otf) c->d_ortho_ws.alloc((size_t)max_bands * b.npw * 16);
    c->d_ortho_small.alloc(ortho_small_bytes(max_bands) + 256);
    acct += c->d_cols.bytes + c->d_proj.bytes + c->d_partial.bytes + c->d_ortho_ws.bytes + c->d_ortho_small.bytes;
    c->device_bytes = acct;
    PW_HIP(hipStreamSynchronize(st));
    *out = c.release();
    PW_API_END
}

pw_status pw_ctx_destroy(pw_ctx *ctx) {
    PW_API_BEGIN
    if (!ctx) return PW_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->solver) solver_destroy(ctx->solver);
    for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
    ctx->prof_pool.clear();
    DevBuf *bufs[] = {&ctx->d_kin, &ctx->d_zmap, &ctx->d_colpos, &ctx->d_colstart, &ctx->d_vz64, &ctx->d_vz32,
                      &ctx->d_tw64[0], &ctx->d_tw64[1], &ctx->d_tw64[2], &ctx->d_tw32[0], &ctx->d_tw32[1],
                      &ctx->d_tw32[2], &ctx->d_beta64, &ctx->d_beta_bf16, &ctx->d_betaT_bf16, &ctx->d_bf16_ws, &ctx->d_dproj, &ctx->d_dproj32,
                      &ctx->d_shell, &ctx->d_cols, &ctx->d_proj, &ctx->d_partial, &ctx->d_ortho_ws,
                      &ctx->d_colslot, &ctx->d_miller, &ctx->d_pos, &ctx->d_beta_chunk,
                      &ctx->d_ortho_small};
    for (DevBuf *d : bufs) d->free_();
    (void)hipSetDevice(cur);
    delete ctx;
    PW_API_END
}

pw_status pw_ctx_set_otf_atoms(pw_ctx *ctx, int32_t atoms) {
    PW_API_BEGIN
    PW_CHECK(ctx, PW_EINVAL, "null context");
    PW_CHECK(ctx->beta_otf, PW_EUNSUPPORTED, "context has a stored projector table");
    PW_CHECK(atoms >= 1, PW_EINVAL, "atoms per chunk must be positive");
    atoms = std::min(atoms, ctx->natom);
    PW_HIP(hipDeviceSynchronize());
    const size_t old = ctx->d_beta_chunk.bytes;
    ctx->d_beta_chunk.alloc((size_t)atoms * ctx->nl * ctx->basis.npw * 16);
    ctx->otf_atoms = atoms;
    ctx->device_bytes += (int64_t)ctx->d_beta_chunk.bytes - (int64_t)old;
    const size_t need = hpsi_partial_bytes(ctx);
    if (need > ctx->d_partial.bytes) ctx->d_partial.alloc(need);
    PW_API_END
}

pw_status pw_ctx_get_info(const pw_ctx *ctx, pw_ctx_info *info) {
    PW_API_BEGIN
    PW_CHECK(ctx && info, PW_EINVAL, "null argument");
    info->npw = ctx->basis.npw;
    info->ncols = ctx->basis.ncols;
    info->nshell = (int32_t)ctx->basis.shell_t.size();
    info->nproj = ctx->nproj;
    for (int a = 0; a < 3; ++a) info->grid[a] = ctx->cell.n[a];
    info->max_bands = ctx->max_bands;
    info->device_bytes = ctx->device_bytes;
    info->cols_bands = ctx->cols_bands;
    PW_API_END
}

pw_status pw_ctx_kinetic(const pw_ctx *ctx, double *kin) {
    PW_API_BEGIN
    PW_CHECK(ctx && kin, PW_EINVAL, "null argument");
    std::memcpy(kin, ctx->basis.kin.data(), sizeof(double) * ctx->basis.npw);
    PW_API_END
}

pw_status pw_ctx_shells(const pw_ctx *ctx, int32_t *shell, double *shell_t) {
    PW_API_BEGIN
    PW_CHECK(ctx, PW_EINVAL, "null argument");
    if (shell) std::memcpy(shell, ctx->basis.shell.data(), sizeof(int32_t) * ctx->basis.npw);
    if (shell_t) std::memcpy(shell_t, ctx->basis.shell_t.data(), sizeof(double) * ctx->basis.shell_t.size());
    PW_API_END
}

static void check_block_args(const pw_ctx *ctx, pw_dtype dt, int nb, const void *a, int64_t lda) {
    PW_CHECK(ctx, PW_EINVAL, "null context");
    PW_CHECK(dt == PW_C128 || dt == PW_C64, PW_EINVAL, "unknown dtype %d", (int)dt);
    PW_CHECK(nb >= 0, PW_EINVAL, "negative band count");
    PW_CHECK(nb == 0 || a, PW_EINVAL, "null block");
    PW_CHECK(lda >= ctx->basis.npw, PW_EINVAL, "leading dimension %lld < npw %d", (long long)lda, ctx->basis.npw);
    if (dt == PW_C64) PW_CHECK(ctx->flags & PW_PREP_C64, PW_EUNSUPPORTED, "context built without PW_PREP_C64");
    if (dt == PW_C128) PW_CHECK(ctx->flags & PW_PREP_C128, PW_EUNSUPPORTED, "context built without PW_PREP_C128");
}

pw_status pw_hpsi(pw_ctx *ctx, pw_dtype dtype, int32_t nb, const void *psi, int64_t ld, void *hpsi, int64_t ldh,
                  double shift, void *stream) {
    PW_API_BEGIN
    check_block_args(ctx, dtype, nb, psi, ld);
    check_block_args(ctx, dtype, nb, hpsi, ldh);
    PW_CHECK(nb == 0 || psi != hpsi, PW_EINVAL, "psi and hpsi must not alias");
    PW_CHECK(std::isfinite(shift), PW_ENAN, "non-finite shift");
    if (nb == 0) return PW_OK;
    hpsi_any(ctx, dtype, nb, psi, ld, hpsi, ldh, shift, (hipStream_t)stream);
    PW_API_END
}

pw_status pw_wave_to_grid(pw_ctx *ctx, pw_dtype dtype, int32_t nb, const void *psi, int64_t ld, void *grid,
                          void *stream) {
    PW_API_BEGIN
    check_block_args(ctx, dtype, nb, psi, ld);
    PW_CHECK(nb == 0 || grid, PW_EINVAL, "null grid");
    hipStream_t st = (hipStream_t)stream;
    const size_t es = dtype == PW_C128 ? 16 : 8;
    const size_t ng = (size_t)ctx->cell.n[0] * ctx->cell.n[1] * ctx->cell.n[2];
    for (int b0 = 0; b0 < nb; b0 += ctx->cols_bands) {
        const int nbc = std::min(ctx->cols_bands, nb - b0);
        const char *pi = (const char *)psi + (size_t)b0 * ld * es;
        char *go = (char *)grid + (size_t)b0 * ng * es;
        if (dtype == PW_C128) {
            launch_zinv<double>(ctx, nbc, pi, ld, ctx->d_cols.p, st);
            launch_xy<double, 1>(ctx, nbc, ctx->d_cols.p, go, st);
        } else {
            launch_zinv<float>(ctx, nbc, pi, ld, ctx->d_cols.p, st);
            launch_xy<float, 1>(ctx, nbc, ctx->d_cols.p, go, st);
        }
    }
    PW_API_END
}

pw_status pw_grid_to_wave(pw_ctx *ctx, pw_dtype dtype, int32_t nb, const void *grid, void *psi, int64_t ld,
                          void *stream) {
    PW_API_BEGIN
    check_block_args(ctx, dtype, nb, psi, ld);
    PW_CHECK(nb == 0 || grid, PW_EINVAL, "null grid");
    hipStream_t st = (hipStream_t)stream;
    const size_t es = dtype == PW_C128 ? 16 : 8;
    const size_t ng = (size_t)ctx->cell.n[0] * ctx->cell.n[1] * ctx->cell.n[2];
    const double scale = 1.0 / (double)ng;
    for (int b0 = 0; b0 < nb; b0 += ctx->cols_bands) {
        const int nbc = std::min(ctx->cols_bands, nb - b0);
        char *po = (char *)psi + (size_t)b0 * ld * es;
        const char *gi = (const char *)grid + (size_t)b0 * ng * es;
        if (dtype == PW_C128) {
            launch_xy<double, 2>(ctx, nbc, ctx->d_cols.p, (void *)gi, st);
            launch_zfwd<double>(ctx, nbc, ctx->d_cols.p, nullptr, 0, nullptr, 0.0, scale, po, ld, st);
        } else {
            launch_xy<float, 2>(ctx, nbc, ctx->d_cols.p, (void *)gi, st);
            launch_zfwd<float>(ctx, nbc, ctx->d_cols.p, nullptr, 0, nullptr, 0.0, scale, po, ld, st);
        }
    }
    PW_API_END
}

pw_status pw_dense_eigh(int32_t n, const void *A, int64_t lda, double *w, void *R, int32_t key, double ref,
                        int32_t *sweeps, void *stream) {
    PW_API_BEGIN
    PW_CHECK(n >= 1 && n <= 1024 && lda >= n && A && w && R, PW_EINVAL, "bad pw_dense_eigh arguments");
    PW_CHECK(key == 0 || key == 1, PW_EINVAL, "key must be 0 or 1");
    hipStream_t st = (hipStream_t)stream;
    DevBuf work;
    const size_t wb = (dense_eigh_work_bytes(n) + 255) / 256 * 256;
    work.alloc(wb + 256);
    int *info = (int *)((char *)work.p + wb);
    dense_eigh(n, A, lda, work.p, w, R, key, ref, info, st);
    int h = 0;
    PW_HIP(hipMemcpyAsync(&h, info, sizeof(int), hipMemcpyDeviceToHost, st));
    PW_HIP(hipStreamSynchronize(st));
    if (sweeps) *sweeps = h;
    PW_CHECK(h >= 0, PW_ENOCONV, "tridiagonal QL iteration did not converge");
    PW_API_END
}

pw_status pw_dense_chol_inv(int32_t n, const void *S, int64_t lds, void *T, void *stream) {
    PW_API_BEGIN
    PW_CHECK(n >= 1 && n <= 8192 && lds >= n && S && T, PW_EINVAL, "bad pw_dense_chol_inv arguments");
    hipStream_t st = (hipStream_t)stream;
    DevBuf work;
    const size_t wb = (chol_inv_work_bytes(n) + 255) / 256 * 256;
    work.alloc(wb + 256);
    int *status = (int *)((char *)work.p + wb);
    fill_zero(status, 16, st);
    chol_inv(n, S, lds, work.p, T, status, st);
    int h = 0;
    PW_HIP(hipMemcpyAsync(&h, status, sizeof(int), hipMemcpyDeviceToHost, st));
    PW_HIP(hipStreamSynchronize(st));
    PW_CHECK(h == 0, PW_ENOTPD, "matrix not positive definite at pivot %d", h - 1);
    PW_API_END
}

pw_status pw_mlp_set(pw_ctx *ctx, const float *weights) {
    PW_API_BEGIN
    PW_CHECK(ctx && weights, PW_EINVAL, "null argument");
    PW_CHECK(mlp_nparam() == PW_MLP_NPARAM, PW_EINVAL, "parameter count mismatch");
    // validate a host copy first: rejected weights never reach the context, which
    // keeps the network it had (or none)
    std::vector<float> h(PW_MLP_NPARAM);
    PW_HIP(hipMemcpy(h.data(), weights, PW_MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost));
    for (float x : h) PW_CHECK(std::isfinite(x), PW_ENAN, "non-finite network weight");
    if (!ctx->d_mlp.p) ctx->d_mlp.alloc(PW_MLP_NPARAM * sizeof(float));
    PW_HIP(hipMemcpy(ctx->d_mlp.p, h.data(), PW_MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice));
    PW_API_END
}

pw_status pw_mlp_forward(int32_t nshell, int32_t nb, const double *shell_t, const double *tband, double e_ref,
                         double ecut, const float *weights, float *f, void *stream) {
    PW_API_BEGIN
    PW_CHECK(nshell >= 1 && nb >= 1 && shell_t && tband && weights && f && ecut > 0, PW_EINVAL,
             "bad pw_mlp_forward arguments");
    mlp_infer(nshell, nb, shell_t, tband, e_ref, ecut, weights, f, (hipStream_t)stream);
    PW_API_END
}

int64_t pw_mlp_work_bytes(int32_t nshell, int32_t nb, int32_t nsnap) {
    if (nshell < 1 || nb < 1 || nsnap < 1) return -1;
    return (int64_t)mlp_work_bytes(nshell, nb, nsnap);
}

pw_status pw_mlp_loss_grad(int32_t nshell, int32_t nb, int32_t nsnap, const double *shell_t, const double *tband,
                           const double *e_ref, double ecut, const double *tabs, const float *weights, float *grad,
                           float *loss, void *work, int64_t work_bytes, void *stream) {
    PW_API_BEGIN
    PW_CHECK(nshell >= 1 && nb >= 1 && nsnap >= 1 && shell_t && tband && e_ref && tabs && weights && grad && work &&
                 ecut > 0, PW_EINVAL, "bad pw_mlp_loss_grad arguments");
    PW_CHECK(work_bytes >= (int64_t)mlp_work_bytes(nshell, nb, nsnap), PW_EINVAL, "work buffer too small");
    mlp_loss_grad(nshell, nb, nsnap, shell_t, tband, e_ref, ecut, tabs, weights, grad, loss, work,
                  (hipStream_t)stream);
    PW_API_END
}

pw_status pw_mlp_adam(float *weights, const float *grad, float *m, float *v, int32_t step, float lr, void *stream) {
    PW_API_BEGIN
    PW_CHECK(weights && grad && m && v && step >= 1 && lr > 0, PW_EINVAL, "bad pw_mlp_adam arguments");
    mlp_adam(weights, grad, m, v, step, lr, (hipStream_t)stream);
    PW_API_END
}

pw_status pw_mlp_train(int32_t nshell, int32_t nb, int32_t nsnap, const double *shell_t, const double *tband,
                       const double *e_ref, double ecut, const double *tabs, float *weights, float *grad, float *m,
                       float *v, int32_t step0, int32_t nsteps, float lr, float *loss_hist, void *work,
                       int64_t work_bytes, void *stream) {
    PW_API_BEGIN
    PW_CHECK(nshell >= 1 && nb >= 1 && nsnap >= 1 && nsteps >= 0 && step0 >= 0 && lr > 0 && shell_t && tband &&
                 e_ref && tabs && weights && grad && m && v && work, PW_EINVAL, "bad pw_mlp_train arguments");
    PW_CHECK(work_bytes >= (int64_t)mlp_work_bytes(nshell, nb, nsnap) + (int64_t)sizeof(float) * (nsteps + 64),
             PW_EINVAL, "work buffer too small (needs pw_mlp_work_bytes + 4 (nsteps + 64) bytes)");
    hipStream_t st = (hipStream_t)stream;
    float *losses = (float *)((char *)work + mlp_work_bytes(nshell, nb, nsnap));
    for (int t = 0; t < nsteps; ++t) {
        mlp_loss_grad(nshell, nb, nsnap, shell_t, tband, e_ref, ecut, tabs, weights, grad, losses + t, work, st);
        mlp_adam(weights, grad, m, v, step0 + t + 1, lr, st);
    }
    if (loss_hist && nsteps > 0)
        PW_HIP(hipMemcpyAsync(loss_hist, losses, sizeof(float) * nsteps, hipMemcpyDeviceToHost, st));
    PW_HIP(hipStreamSynchronize(st));
    PW_API_END
}

pw_status pw_profile_begin(pw_ctx *ctx, int32_t max_records) {
    PW_API_BEGIN
    PW_CHECK(ctx && max_records >= 1 && max_records <= (1 << 22), PW_EINVAL, "bad profile arguments");
    for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
    ctx->prof_pool.clear();
    ctx->prof_rec.clear();
    ctx->prof_rec.reserve(max_records);
    ctx->prof_pool.resize(2 * (size_t)max_records, nullptr);
    for (auto &e : ctx->prof_pool) PW_HIP(hipEventCreate(&e));
    ctx->prof_next = 0;
    ctx->prof_on = true;
    PW_API_END
}

pw_status pw_profile_end(pw_ctx *ctx, double *ms, int64_t *launches) {
    PW_API_BEGIN
    PW_CHECK(ctx && ms && launches, PW_EINVAL, "null argument");
    for (int k = 0; k < PW_PROF_NKINDS; ++k) { ms[k] = 0.0; launches[k] = 0; }
    for (const ProfRec &r : ctx->prof_rec) {
        PW_HIP(hipEventSynchronize(r.b));
        float t = 0.f;
        PW_HIP(hipEventElapsedTime(&t, r.a, r.b));
        if (r.kind >= 0 && r.kind < PW_PROF_NKINDS) {
            ms[r.kind] += t;
            launches[r.kind] += 1;
        }
    }
    ctx->prof_on = false;
    for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
    ctx->prof_pool.clear();
    ctx->prof_rec.clear();
    ctx->prof_next = 0;
    PW_API_END
}

pw_status pw_ctx_autotune(pw_ctx *ctx, pw_dtype dtype, int32_t nb, int32_t reps, pw_fft_cand *cands, int32_t cap,
                          int32_t *ncand, void *stream) {
    PW_API_BEGIN
    PW_CHECK(ctx && (cands || cap == 0) && cap >= 0, PW_EINVAL, "bad autotune arguments");
    PW_CHECK(dtype == PW_C128 || dtype == PW_C64, PW_EINVAL, "unknown dtype");
    PW_CHECK(ctx->flags & (dtype == PW_C128 ? PW_PREP_C128 : PW_PREP_C64), PW_EUNSUPPORTED,
             "context not prepared for this dtype");
    std::vector<pw_fft_cand> recs;
    if (dtype == PW_C128) autotune_fft<double>(ctx, nb, reps, recs, (hipStream_t)stream);
    else autotune_fft<float>(ctx, nb, reps, recs, (hipStream_t)stream);
    for (int i = 0; i < (int)recs.size() && i < cap; ++i) cands[i] = recs[i];
    if (ncand) *ncand = (int32_t)recs.size();
    PW_API_END
}

pw_status pw_ctx_fft_choose(pw_ctx *ctx, pw_dtype dtype, const pw_fft_cand *cand) {
    PW_API_BEGIN
    PW_CHECK(ctx && cand, PW_EINVAL, "null argument");
    PW_CHECK(dtype == PW_C128 || dtype == PW_C64, PW_EINVAL, "unknown dtype");
    if (dtype == PW_C128) fft_choose<double>(ctx, *cand);
    else fft_choose<float>(ctx, *cand);
    PW_API_END
}

pw_status pw_orthonormalize(pw_ctx *ctx, int32_t nb, void *psi, int64_t ld, void *stream) {
    PW_API_BEGIN
    check_block_args(ctx, PW_C128, nb, psi, ld);
    PW_CHECK(nb <= ctx->max_bands, PW_EINVAL, "nb %d > max_bands %d", nb, ctx->max_bands);
    if (nb == 0) return PW_OK;
    hipStream_t st = (hipStream_t)stream;
    if (!ctx->d_ortho_ws.p) ctx->d_ortho_ws.alloc((size_t)ctx->max_bands * ctx->basis.npw * 16);
    int *d_status = (int *)((char *)ctx->d_ortho_small.p + ortho_small_bytes(ctx->max_bands));
    fill_zero(d_status, 16, st);
    orthonormalize_c128(ctx, nb, psi, ld, ctx->d_ortho_ws.p, ctx->d_ortho_small.p, d_status, st);
    int status = 0;
    PW_HIP(hipMemcpyAsync(&status, d_status, sizeof(int), hipMemcpyDeviceToHost, st));
    PW_HIP(hipStreamSynchronize(st));
    PW_CHECK(status == 0, PW_ENOTPD, "Gram matrix not positive definite at pivot %d", status - 1);
    PW_API_END
}

}  // extern "C"
