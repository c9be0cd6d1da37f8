// Host-side launchers of the libpw kernels (declarations).
#pragma once
#include "common.h"

namespace pw {

// fft.hip
template <typename T> void launch_zinv(pw_ctx *, int nb, const void *psi, int64_t ld, void *cols, hipStream_t);
template <typename T>
void launch_zfwd(pw_ctx *, int nb, const void *cols, const void *psi, int64_t ld, const double *kin, double shift,
                 double scale, void *out, int64_t ldo, hipStream_t);
template <typename T, int MODE> void launch_xy(pw_ctx *, int nb, void *cols, void *grid, hipStream_t);

// LDS plane of the four-lane xy kernel for planes of L = 4 m points a side: the
// element of row slot r, column c sits at r quad_rs(m) + c + (c / m) quad_pad(m).
// Its accesses (lane q of a quad at column q + 4 k, or at k + m q', or four lanes
// on consecutive rows of one column) then fall into distinct banks among the 16
// lanes that share an LDS cycle: rows are 4 mod 16 elements apart and each of the
// four column blocks of m is shifted by one more element mod 16.
constexpr int quad_pad(int m) {
    int p = 1;
    while ((m + p) % 16 != 1) ++p;
    return p;
}
constexpr int quad_rs(int m) {
    int r = 4 * m + 3 * quad_pad(m);
    while (r % 16 != 4) ++r;
    return r;
}

// gemm.hip (complex128)
int nt_splits(int M, int N, int K, bool herm = false);
size_t nt_partial_bytes(int M, int N, int K);
int nt_tile_id(int M, int N, bool herm);
// bands per projector GEMM launch of the stored-table FP64 H psi: 129-144 bands go as
// the first 128 (tiles of the three-product form) and the rest, others in one launch
inline int proj_band_split(int nb) { return nb > 128 && nb <= 144 ? 128 : nb; }
// herm: A == B (a Gram matrix A^H B): only the tiles on and below the diagonal are computed
void zgemm_nt(int M, int N, int K, bool conja, const void *A, int64_t lda, const void *B, int64_t ldb,
              double alpha, const double *rowscale, double beta, void *C, int64_t ldc, bool trans, void *partial,
              hipStream_t, bool proj = false, bool herm = false);
// NN GEMM tile configurations: cfg < 0 picks by M, else one of kNnCfgs (autotuner)
constexpr int kNnCfgs = 14;
void nn_cfg_shape(int id, int &tm, int &tj, int &nthr);
// lower: W is lower triangular (zeros above its diagonal are skipped; same results)
void zgemm_nn_launch(int M, int J, int K, const void *W, int64_t ldw, const void *X, int64_t ldx, double alpha,
                     double beta, void *Out, int64_t ldo, hipStream_t, bool proj = false, int cfg = -1,
                     bool lower = false);
void zgemm_nn_batch(int nz, int M, int J, int K, const void *W, int64_t ldw, const void *const *X, int64_t ldx,
                    double alpha, double beta, void *const *Out, int64_t ldo, hipStream_t, bool proj = false, int cfg = -1,
                    bool lower = false);

// Batched launches over independent problems: one job per problem in a device
// array, mask[q] = 0 skips job q (device-side, so a recorded launch stays valid as
// problems finish).  Each job's tiles and split-K chunking are those of its own
// single call, so its result is bit for bit the same.
struct NtJob {                // C = alpha rowscale o (op(A) B^T) + beta C, split-K over K
    int M, N, K, kchunk, nsplit, herm;
    const double2 *A, *B;
    int64_t lda, ldb;
    double alpha, beta;
    const double *rowscale;
    double2 *C;
    int64_t ldc;
    double2 *partial;
};
struct NnJob {                // Out_z = alpha W X_z + beta Out_z, z < nz
    int M, J, K, nz, lower;
    const double2 *W;
    int64_t ldw;
    const double2 *X[4];
    double2 *Out[4];
    int64_t ldx, ldo;
    double alpha, beta;
};
NtJob nt_job(int M, int N, int K, bool conja, const void *A, int64_t lda, const void *B, int64_t ldb, double alpha,
             const double *rowscale, double beta, void *C, int64_t ldc, void *partial, bool herm);
// jobs: host copy (tile shape, grid) and device copy; all with one tile shape
void zgemm_nt_jobs(const std::vector<NtJob> &h, const NtJob *d_jobs, const int *d_mask, bool conja, bool trans,
                   bool proj, hipStream_t);
int nn_default_cfg(int M);
void zgemm_nn_jobs_launch(const std::vector<NnJob> &h, const NnJob *d_jobs, const int *d_mask, int cfg, bool proj,
                          hipStream_t);

// Batched one-workgroup dense kernels (N <= 136) over problems (dense.hip)
struct DenseJob {
    int N;
    const double2 *A;         // Gram (Cholesky) or the Hermitian matrix (eigensolver)
    int64_t lda;
    double2 *T;               // Cholesky: conj(L^-1), N x N
    int64_t ldt;
    int *status;              // Cholesky: first failing pivot + 1
    double2 *hv;              // eigensolver work (dense_eigh's layout) and outputs
    double *zbuf;
    int *rank;
    double *lam;
    double2 *R;
    int *info;
};
DenseJob dense_job(int N, const void *A, int64_t lda, void *work, double *lam, void *R, int *info, void *T,
                   int *status);
void chol_inv_jobs(int N, const DenseJob *jobs, const int *mask, int njobs, hipStream_t);
void dense_eigh_jobs(int N, const DenseJob *jobs, const int *mask, int njobs, hipStream_t);

// Batched complex128 (H - shift) psi over problems with the same band count (fft.hip):
// in[p] -> out[p] for every problem p whose mask entry is set, bit for bit each
// problem's own hpsi_any.  hpsi_batch_ok says whether the contexts allow it (stored
// FP64 table, default launch choices, all bands in one FFT chunk).
struct HpsiBatch;
bool hpsi_batch_ok(int n, pw_ctx *const *ctx, int nb, std::string *why);
HpsiBatch *hpsi_batch_create(int n, pw_ctx *const *ctx, int nb, void *const *in, const int64_t *ld,
                             void *const *out, const int64_t *ldo, const double *shift, const int *mask);
void hpsi_batch_run(HpsiBatch *, hipStream_t);
void hpsi_batch_destroy(HpsiBatch *);

// gemm_bf16.hip (complex64 blocks, BF16 projector table, FP32 accumulation)
// BF16 planes of contexts of more than 144 bands (bf16_panels) are stored in
// 16-row panels: rows 16 q .. 16 q + 15 of 32 consecutive k as one 1 KB fragment,
// element (r, k) at lane r % 16 + 16 ((k % 32) / 8), position k % 8 (the matrix
// cores' operand order), the fragments of a panel in k order; ld (the padded row
// length, a multiple of 64) columns per row.  Rows are padded to a multiple of 16
// (bf16_rows), and a panel of rows r0 .. starts at r0 ld for r0 a multiple of 16.
__host__ __device__ inline int64_t bf16_panel_index(int64_t r, int64_t k, int64_t ld) {
    return ((((r >> 4) * (ld >> 5) + (k >> 5)) << 6) + (r & 15) + (((k & 31) >> 3) << 4)) * 8 + (k & 7);
}
bool bf16_panels(int max_bands);
int64_t bf16_rows(int rows, int max_bands);
size_t cnt_partial_bytes(int M, int N, int K, int max_bands);
int64_t bf16_ld(int n);
size_t bf16_scratch_bytes(int nproj, int npw, int max_bands);
void beta_to_bf16_t(int nproj, int npw, const void *beta64, void *tr, void *ti, hipStream_t st, bool panel);
void beta_to_bf16_t_rows(int nproj, int p0, int rows, int npw, const void *beta64, void *tr, void *ti,
                         hipStream_t st, bool panel);
// variant: launch variant of the kernels for more than 144 bands (autotuner pass 6)
constexpr int kBf16WideVariants = 4;
void proj_bf16(int nproj, int nb, int npw, int max_bands, const void *beta16, const float *d, const void *psi,
               int64_t ld, void *scratch, void *partial, hipStream_t st, int variant = 0);
void backproj_bf16(int nproj, int nb, int npw, int max_bands, const void *betaT16, const void *scratch, void *out,
                   int64_t ldo, hipStream_t st, int variant = 0);

// dense.hip
// S = L L^H, T = conj(L^-1); work: chol_inv_work_bytes(N) device bytes
size_t chol_inv_work_bytes(int N);
void chol_inv(int N, const void *S, int64_t lds, void *work, void *T, int *status, hipStream_t);
// Hermitian eigensolver (1 <= N <= 1024); work: dense_eigh_work_bytes(N) device bytes.
size_t dense_eigh_work_bytes(int N);
void dense_eigh(int N, const void *A, int64_t lda, void *work, double *lam, void *R, int key, double ref, int *info,
                hipStream_t);

// mlp.hip
int mlp_nparam();
void mlp_infer(int nshell, int nb, const double *shell_t, const double *tband, double e_ref, double ecut,
               const float *w, float *f, hipStream_t);
size_t mlp_work_bytes(int nshell, int nb, int nsnap);
void mlp_loss_grad(int nshell, int nb, int nsnap, const double *shell_t, const double *tband, const double *e_ref,
                   double ecut, const double *tabs, const float *w, float *grad, float *loss, void *work, hipStream_t);
void mlp_adam(float *w, const float *g, float *m, float *v, int step, float lr, hipStream_t);
void shell_tables(int nshell, int nb, int npw, const int32_t *shell_off, const int32_t *shell_pw, const void *E,
                  const void *Z, int64_t ld, const double *shell_t, double e_ref, double delta, double *tabs,
                  hipStream_t);

// blas1.hip -------------------------------------------------------------------
struct PrecArgs {
    int kind;                 // 0 TPA^2, 1 paper M(G), 2 M(G) * exp(f[shell][band])
    const double *kin;        // [npw]
    const double *tband;      // [nb] band kinetic energies (TPA)
    double e_ref, de2;        // M(G)
    const float *ftab;        // [nshell][nb] learned log-scaling
    const int32_t *shell;     // [npw]
    int nb;
};

// One problem of a batched folded-CG run (all problems with the same band count
// nb): its solver blocks, its per-band vectors (mu, tband, gz, gzo, gz_old, line4
// (4 nb), coef (4 nb), lam, res, nb each, in that order) and reduction scratch.
enum { kBX = 0, kBY, kBAX, kBP, kBYP, kBAP, kBG, kBZ, kBT1, kBT2, kBT3, kBlocks };
struct BandProb {
    int npw, nsplit;
    int64_t ld;
    double2 *blk[kBlocks];
    double *vec;
    double *red;
    PrecArgs pa;
    double2 *psi;             // the caller's block (the iterate a restart goes back to)
    int64_t ldpsi;
    int *status;              // the solver's status ints (Cholesky pivot, eigensolver info)
};
enum class BandOp { MuTband, Grad, GzOld, PUpdate, Line, Combine3, Resid };
// one batched launch (or two, for reductions) of a band-wise step of FcgRun over
// every problem whose mask entry is set; Resid: res = ||blk[a0] - lam blk[a1]||
void band_batch(BandOp op, const BandProb *probs, const int *mask, int nprob, int nb, int maxsplit, int maxnpw,
                hipStream_t st, int a0 = 0, int a1 = 0);
void band_batch_copy(const BandProb *probs, const int *mask, int nprob, int nb, int maxnpw, int n, const int *src,
                     const int *dst, hipStream_t st);
// psi <- X for every masked-in problem
void band_batch_save(const BandProb *probs, const int *mask, int nprob, int nb, int maxnpw, hipStream_t st);
// out[p] = (lam[0..nb), res[0..nb)), sout[p] = status[0..8) for every problem (masked-out ones too)
void band_batch_gather(const BandProb *probs, int nprob, int nb, double *out, int *sout, hipStream_t st);

struct BandRed {              // scratch for two-stage band reductions
    double *partial;          // [nq][nb][nsplit]
    int nsplit;
};
int band_splits(int npw);

void fill_zero(void *p, size_t bytes, hipStream_t);
template <typename T>
void autotune_fft(pw_ctx *ctx, int nb, int reps, std::vector<pw_fft_cand> &recs, hipStream_t s);
template <typename T> void fft_choose(pw_ctx *ctx, const pw_fft_cand &r);
void copy_block(int nb, int npw, const void *src, int64_t lds, void *dst, int64_t ldd, hipStream_t);
void red_mu_tband(int nb, int npw, const void *Y, const void *X, int64_t ld, const double *kin, double *mu,
                  double *tband, BandRed, hipStream_t);
void red_grad(int nb, int npw, const void *X, const void *AX, void *Gold, void *Z, int64_t ld, const double *mu,
              PrecArgs pa, double *gz, double *gzo, BandRed, hipStream_t);
void red_gzold(int nb, int npw, const void *G, int64_t ld, PrecArgs pa, double *gz_old, BandRed, hipStream_t);
void pupdate(int nb, int npw, const void *Z, void *P, int64_t ld, const double *gz, const double *gzo,
             double *gz_old, hipStream_t);
void red_line(int nb, int npw, const void *Y, const void *YP, const void *P, int64_t ld, double *out4,
              BandRed, hipStream_t);
void line_coef(int nb, const double *mu, const double *line4, double *coef, hipStream_t);
void combine3(int nb, int npw, void *X, void *Y, void *AX, const void *P, const void *YP, const void *AP,
              int64_t ld, const double *coef, hipStream_t);
void red_resid(int nb, int npw, const void *Y, const void *X, int64_t ld, const double *w, double *res,
               BandRed, hipStream_t);
void band_norms(int nb, int npw, const void *X, int64_t ld, double *out, BandRed, hipStream_t);
void c64_to_c128(int nb, int npw, const void *src, int64_t lds, void *dst, int64_t ldd, hipStream_t);
void c128_to_c64(int nb, int npw, const void *src, int64_t lds, void *dst, int64_t ldd, hipStream_t);
void nan_check(size_t n, const double *x, int *flag, hipStream_t);
// folded linear equation, column-wise PCG (per-column scalars on the device)
void lin_alpha(int nb, int npw, const void *YP, int64_t ld, const double *rz, double *alpha, BandRed, hipStream_t);
void lin_update(int nb, int npw, void *X, void *Y, void *R, const void *P, const void *YP, const void *AP, int64_t ld,
                const double *alpha, hipStream_t);
void lin_mdiag(int nb, int npw, const void *R, const void *U, void *Z, int64_t ld, const double *kin, double e_ref,
               double de2, double *rz, double *beta, bool first, bool with_rz, BandRed, hipStream_t);
void lin_rz_beta(int nb, int npw, const void *R, const void *Z, int64_t ld, double *rz, double *beta, bool first,
                 BandRed, hipStream_t);
void lin_pupdate(int nb, int npw, const void *Z, void *P, int64_t ld, const double *beta, hipStream_t);
void lin_coef(int nrhs, int nev, const void *C, const void *D, const double *invd, void *E, hipStream_t);
void lin_err(int nb, int npw, const void *Y, int64_t ldy, const void *W, int64_t ldw, double *err, BandRed,
             hipStream_t);
void lin_sub(int nb, int npw, void *R, const void *AX, int64_t ld, hipStream_t);
// Chebyshev filter and Lanczos bounds
void cheb_step(int nb, int npw, const void *T, void *Uprev, void *Y, int64_t ld, double s, double gamma, bool first,
               hipStream_t);
void scale_copy(int nb, int npw, const void *src, int64_t lds, void *dst, int64_t ldd, double s, hipStream_t);
void lanczos_update(int npw, void *W, const void *V, const void *Vp, double alpha, double beta, hipStream_t);
void red_dot_re(int nb, int npw, const void *A, const void *B, int64_t ld, double *out, BandRed, hipStream_t);
// wave-function interpolation
void gather_pw(int nb, int npw_to, const void *src, int64_t lds, const int32_t *map, void *dst, int64_t ldd,
               hipStream_t);
void kinterp_hk(int n, double alpha, const double *e1, const double *e2, const void *U, void *Hk, hipStream_t);

}  // namespace pw
