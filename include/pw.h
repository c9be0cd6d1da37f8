/*
 * pw.h -- C ABI of libpw: folded-spectrum plane-wave eigensolver for gfx950.
 *
 * The library finds the Kohn-Sham states of a plane-wave Hamiltonian nearest a
 * reference energy E by minimising <psi|(H - E)^2|psi> with preconditioned
 * conjugate gradients.  The folded operator (H - E)^2 and its positivity are
 * the paper's folded equation (Sec. II.B); the few-states-near-E use is the
 * folded-spectrum method the paper names in Sec. II.B; the G-diagonal
 * preconditioner M(G) and the eigen-residual Delta_i = ||H phi_i - eps_i phi_i||
 * are defined under the paper's M' equation (Sec. II.B).  Around the eigensolve:
 * the folded linear equation of the system states with the eigenstate-augmented
 * preconditioner M' (Sec. II.B), Chebyshev filter diagonalisation of an energy
 * window (Sec. II.B) and wave-function interpolation between k-points (Sec. II.C).
 *
 * Conventions shared by every entry point
 *   - Cell: orthorhombic, lengths L = (L0, L1, L2) bohr, axis 2 is z.
 *     Reciprocal vectors G = 2 pi (n0/L0, n1/L1, n2/L2), Miller triple n.
 *   - Basis: every n with (1/2)|G + k|^2 <= ecut (Ha).  Coefficient order is
 *     lexicographic in the signed triple (n0, n1, n2); pw_basis_miller returns
 *     it.  Every n must land on a distinct grid point: 2 max|n_i| + 1 <= N_i.
 *   - Wave-function blocks are band-major: band b, plane wave g at
 *     psi[b * ld + g], interleaved complex (re, im), complex128 or complex64.
 *   - Real space: grid point r_j = (j0 L0/N0, j1 L1/N1, j2 L2/N2), arrays
 *     [N0][N1][N2] C order.  G -> r is the unnormalised sum
 *     f(r_j) = sum_G c(G) exp(+i G.r_j); r -> G is
 *     c(G) = (1/N) sum_j f(r_j) exp(-i G.r_j), N = N0 N1 N2.  With V given by
 *     its grid samples this makes the FFT application of V equal to the
 *     plane-wave matrix element Vt(G - G') exactly.
 *   - Nonlocal term: Kleinman-Bylander sum_p |beta_p> D_p <beta_p|, 4 per atom
 *     (s, px, py, pz) with q = G + k:
 *       beta_{a,j}(G) = sqrt(8 pi^1.5 s^3) Y_j(q) exp(-|q|^2 s^2/2) exp(-i q.R_a) / sqrt(Omega),
 *       Y_s = 1, Y_{p,m} = sqrt(3) q_m/|q| (0 at q = 0).
 *   - Pointers marked "device" are HIP device memory owned by the caller; the
 *     library never frees them.  Pointers marked "host" are read (or written)
 *     before the call returns.  `stream` is a hipStream_t (NULL = default).
 *   - Errors: every call returns a pw_status and never aborts; the text of the
 *     last error on the calling thread is pw_last_error().  On PW_ENOCONV the
 *     outputs hold the best iterate; on any other error outputs are
 *     unspecified.
 */
#ifndef PW_H
#define PW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PW_OK = 0,
    PW_EINVAL = -1,       /* bad argument (size, stride, null pointer, grid too small) */
    PW_ENOMEM = -2,       /* device allocation failed */
    PW_EHIP = -3,         /* a HIP runtime call failed */
    PW_ENOTPD = -4,       /* Gram matrix not positive definite (dependent bands) */
    PW_ENOCONV = -5,      /* solver hit maxit before tol */
    PW_ENAN = -6,         /* NaN/Inf met in an input or a convergence scalar */
    PW_EUNSUPPORTED = -7  /* combination not built (e.g. dtype without its tables) */
} pw_status;

typedef enum {
    PW_C128 = 0,          /* complex128 everywhere */
    PW_C64 = 1            /* complex64 FFT/pointwise, BF16 x BF16 -> FP32 projector GEMMs */
} pw_dtype;

typedef struct pw_ctx pw_ctx;

/* Cell, grid and cutoff of one plane-wave problem. */
typedef struct {
    int32_t n[3];         /* FFT grid N0, N1, N2; each a product of 2, 3, 5, at most 1024 */
    double cell[3];       /* L0, L1, L2 (bohr) */
    double kpt[3];        /* Bloch vector k, Cartesian (1/bohr) */
    double ecut;          /* kinetic cutoff (Ha) */
} pw_cell;

/* Potential: local part sampled on the grid plus KB projectors.
 * v_r    device, float64 [N0][N1][N2], Ha; copied into the context.
 * natom  number of projector centres (0 = local only)
 * pos    host [natom][3] bohr
 * nl     projectors per atom: 0, 1 (s) or 4 (s, px, py, pz)
 * sigma  projector Gaussian width (bohr)
 * d      host [natom * nl] KB strengths D_p (Ha), order per atom s, px, py, pz */
typedef struct {
    const double *v_r;
    int32_t natom;
    const double *pos;
    int32_t nl;
    double sigma;
    const double *d;
} pw_potential;

/* Context flags: which precisions to prepare tables for. */
#define PW_PREP_C128 1    /* complex128 projector table [nproj][npw] */
#define PW_PREP_C64  2    /* BF16 projector table and complex64 potential */
#define PW_PREP_C128_OTF 4 /* complex128 H psi without a stored table: each H psi generates the
                              complex128 projector rows from their closed form a chunk of atoms at a
                              time (a few GB of scratch) and applies them chunk by chunk; for cells
                              whose table (16 nproj npw bytes) does not fit.  Implies PW_PREP_C128. */

typedef struct {
    int32_t npw;          /* plane waves in the sphere */
    int32_t ncols;        /* (n0, n1) columns that touch the sphere */
    int32_t nshell;       /* distinct |G + k| shells */
    int32_t nproj;        /* natom * nl */
    int32_t grid[3];
    int32_t max_bands;
    int64_t device_bytes; /* workspace + tables owned by the context */
    int32_t cols_bands;   /* bands per FFT launch (the column grid holds that many; H psi loops) */
} pw_ctx_info;

/* Number of plane waves in the sphere (host only, no GPU). */
pw_status pw_basis_size(const pw_cell *cell, int32_t *npw);

/* Miller triples of the basis in coefficient order: host int32 [npw][3]. */
pw_status pw_basis_miller(const pw_cell *cell, int32_t *miller, int32_t npw);

/* Build a context on the current device: basis, z-column tables, kinetic
 * energies, shells, V (z-major copy), projector tables per `flags`, and a
 * workspace for hpsi on up to `max_bands` bands.  All device memory is
 * allocated here (and by the first folded-CG solve); hot calls allocate
 * nothing.  Returns PW_EINVAL if the sphere does not fit the grid.
 * A context is not safe for overlapping calls: its scratch (column grid,
 * split-K partials, BF16 planes, solver workspace) serves every call on it, so
 * calls on one context from several streams or threads race.  Calls on
 * different contexts may overlap; the autotuner's process-wide result cache is
 * guarded by a mutex. */
pw_status pw_ctx_create(const pw_cell *cell, const pw_potential *pot, int32_t max_bands,
                        int32_t flags, void *stream, pw_ctx **out);
pw_status pw_ctx_destroy(pw_ctx *ctx);
pw_status pw_ctx_get_info(const pw_ctx *ctx, pw_ctx_info *info);

/* Atoms per chunk of a PW_PREP_C128_OTF context (default: as many as fit 4 GB of
 * complex128 rows).  Reallocates the chunk buffer (allocates; synchronises).
 * Results do not depend on it beyond the order in which chunks are summed.
 * PW_EUNSUPPORTED for a context with a stored table. */
pw_status pw_ctx_set_otf_atoms(pw_ctx *ctx, int32_t atoms);

/* Host copies of per-plane-wave tables: kinetic energy (1/2)|G+k|^2 (float64
 * [npw]) and shell index (int32 [npw], shells ascending in energy). */
pw_status pw_ctx_kinetic(const pw_ctx *ctx, double *kin_host);
pw_status pw_ctx_shells(const pw_ctx *ctx, int32_t *shell_host, double *shell_t_host);

/* hpsi = (H - shift) psi for nb bands.  psi, hpsi: device, [nb][ld] / [nb][ldh]
 * of the dtype's complex type, ld, ldh >= npw, no overlap.  Any nb >= 0 (the
 * call loops over chunks of max_bands).  PW_C64 needs a context built with
 * PW_PREP_C64.  Asynchronous on `stream`. */
pw_status pw_hpsi(pw_ctx *ctx, pw_dtype dtype, int32_t nb, const void *psi, int64_t ld,
                  void *hpsi, int64_t ldh, double shift, void *stream);

/* Wave <-> grid transforms of the hpsi path (no potential).
 * to_grid:   out[b][j] = sum_G c_b(G) exp(+i G.r_j)        (device [nb][N])
 * from_grid: c_b(G) = (1/N) sum_j f_b(r_j) exp(-i G.r_j)   (device [nb][ld])
 * Grid arrays are [nb][N0][N1][N2] contiguous complex of the dtype. */
pw_status pw_wave_to_grid(pw_ctx *ctx, pw_dtype dtype, int32_t nb, const void *psi, int64_t ld,
                          void *grid, void *stream);
pw_status pw_grid_to_wave(pw_ctx *ctx, pw_dtype dtype, int32_t nb, const void *grid,
                          void *psi, int64_t ld, void *stream);

/* Orthonormalise a complex128 block in place: S = Psi^H Psi, S = L L^H,
 * Psi <- Psi L^{-H} (the Gram/Cholesky step of the solver).  Returns
 * PW_ENOTPD (synchronising) if a Cholesky pivot is not positive. */
pw_status pw_orthonormalize(pw_ctx *ctx, int32_t nb, void *psi, int64_t ld, void *stream);

/* FFT launch autotuner.  A candidate is one launch variant of one pass of
 * pw_hpsi's FFT: pass 0 the z inverse pass, 1 the xy planes with V(r), 2 the
 * z forward pass with the kinetic term; kind 1 the kernel built for this
 * length at compile time, kind 2 the runtime-plan kernel with nthr threads
 * (256, 512 or 1024) and radix schedule sched (0: radices 8 first, 1: radix 4
 * at most, 2: the radices of 0 in ascending order; radix[] lists the z plan or
 * the xy axis-0 plan), for pass 1 on planes of 16, 32, 48, 64, 96 or 128
 * points a side kind 3 the four-lane register kernel with nthr threads (128,
 * 192, 256 or 512; the default there; sched 1, complex128 planes of at most 64
 * points only: V(r) loaded ahead of the x transforms), kind 0 the built-in
 * default.  Pass 4 (complex128 only)
 * is the back-projection GEMM: kind 3, sched the tile id, radix[0..1] the tile's
 * rows and columns, radix[2] the band count it was timed at (the choice applies
 * to calls with that many bands), nthr its threads.  Pass 5 (complex128 only),
 * in the same form, is the block-rotation GEMM of the solver (an nb x nb matrix
 * times the nb-band block).  Pass 6 (complex64, contexts of more than 144
 * bands) is the BF16 projection and back-projection pair timed together at
 * max_bands: kind 3, sched the launch variant 0-3 (four tile shapes of 256
 * bands, fed by LDS DMA three stages deep from the 16-row panels such contexts
 * keep their BF16 planes in). */
typedef struct {
    int32_t pass;
    int32_t kind;
    int32_t nthr;
    int32_t sched;
    int32_t nradix;
    int32_t radix[12];
    double ms;            /* out: time per launch on nb bands */
    int32_t chosen;       /* out: 1 for the fastest of its pass */
} pw_fft_cand;

/* Times every candidate that fits this context's grid (and projector table) on
 * nb (<= max_bands) bands of dtype, reps launches each, and installs the fastest
 * of each pass for later pw_hpsi calls of that dtype.  The records (at most cap) go to
 * cands (host), their number to *ncand.  Results are cached per (grid, sphere,
 * dtype, nb) for the process, so equal cells are timed once.  Allocates
 * scratch; synchronises. */
pw_status pw_ctx_autotune(pw_ctx *ctx, pw_dtype dtype, int32_t nb, int32_t reps, pw_fft_cand *cands, int32_t cap,
                          int32_t *ncand, void *stream);
/* Installs one candidate (pass, kind, nthr, sched of *cand) for dtype; kind 0
 * restores the default.  PW_EUNSUPPORTED if it does not fit the grid. */
pw_status pw_ctx_fft_choose(pw_ctx *ctx, pw_dtype dtype, const pw_fft_cand *cand);

/* Small dense FP64 kernels of the block algebra, exposed for direct use and
 * testing (device pointers, complex128, row-major).
 *
 * pw_dense_eigh: eigen-decomposition of the Hermitian part of A (n x n, ld lda):
 *   w (device, n) eigenvalues ordered by key (0: ascending, 1: ascending
 *   |w - ref|), R (device, n x n) with row b the eigenvector of w[b] in the input
 *   basis (so a band-major block rotates as Psi' = R . Psi).  Householder
 *   tridiagonalisation, then divide and conquer on the tridiagonal (leaves of at
 *   most 16 rows by implicit QL, rank-one merges); sweeps (host, optional) gets
 *   the largest QL iteration count of one leaf eigenvalue, and PW_ENOCONV is
 *   returned if one exceeds 60.  Synchronises.
 * pw_dense_chol_inv: S = L L^H for Hermitian positive definite S (n x n, lds,
 *   n <= 8192), T = conj(L^{-1}) (n x n, zero above the diagonal) so that
 *   Psi' = T . Psi has Psi'^H Psi' = I when S = Psi^H Psi.  n <= 136: one
 *   workgroup with the packed triangle in LDS; larger n: blocked by 128 (that
 *   kernel on the diagonal blocks, matrix-core products for the panels, the
 *   trailing updates and the inverse).  Returns PW_ENOTPD, naming the first
 *   pivot that is not positive.  Synchronises.
 * Both are the Rayleigh-Ritz and Gram/Cholesky steps of the solver. */
/* pw_dense_eigh: n <= 1024.  n <= 136 in one workgroup (A as a packed triangle in
 * LDS); larger n as launches over the whole GPU (two per Householder step, then
 * per level of merges one workgroup per merge for the order and deflation, and
 * the secular roots, eigenvector weights and a tiled product each over all of the
 * level's merges). */
pw_status pw_dense_eigh(int32_t n, const void *A, int64_t lda, double *w, void *R, int32_t key, double ref,
                        int32_t *sweeps, void *stream);
pw_status pw_dense_chol_inv(int32_t n, const void *S, int64_t lds, void *T, void *stream);

/* pw_dense_eigh for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * eigensolver, kernels and results, with its work memory in a device array
 * inside the library (about 8.4 MB on each GPU it runs on, held until the
 * process ends) instead of a per-call allocation, so n <= 512 (PW_EINVAL above).
 * The array keeps the last call's contents and every call on one GPU shares it:
 * calls that overlap on one GPU (other streams or threads) race.  Arguments,
 * outputs and errors as pw_dense_eigh; synchronises `stream`. */
pw_status pw_dense_eigh_noalloc(int32_t n, const void *A, int64_t lda, double *w, void *R, int32_t key, double ref,
                                int32_t *sweeps, void *stream);

/* Solver options. */
typedef struct {
    double tol;           /* stop when max_i Delta_i <= tol (Ha); paper's accuracy 1e-6 */
    int32_t maxit;        /* CG iterations cap */
    int32_t precond;      /* 0 folded Teter-Payne-Allan, 1 paper M(G), 2 learned (network set) */
    double delta_e;       /* dE of M(G) (Ha) */
    int32_t precision;    /* 0 FP64 throughout; 1 mixed (complex64 H psi, FP64 block algebra) */
    int32_t check_every;  /* iterations between exact residual checks */
    int32_t verbose;      /* print the residual at each check to stderr */
    double mixed_switch;  /* mixed: use FP64 H psi once max Delta < mixed_switch (default 5e-4, above
                             the level where BF16 projector products slow the 256-atom wire) */
    int32_t stall_checks; /* mixed: also switch after this many checks (default 5) without a 2x gain of
                             the best residual once it is below 20 x mixed_switch, or after 10 x this
                             many anywhere (0 = never) */
    void *snap_buf;       /* optional device complex128 [snap_cap][nb][npw]: iterate snapshots for training */
    int32_t snap_every;   /* store X after every snap_every-th iteration (0 = never) */
    int32_t snap_cap;     /* capacity of snap_buf in snapshots */
    int32_t nconv;        /* only the nconv Ritz pairs nearest e_ref must reach tol (0 = all nb); the
                             other nb - nconv bands are buffer bands that widen the folded gap */
    int32_t batch_launch; /* pw_batch_solve only: 2 (default) fuses the problems: every step of an
                             iteration or check is one launch over all problems (one per group of equal
                             FFT grids for the FFT passes), a device mask skipping finished problems,
                             the round of check_every iterations and its check recorded once as a graph
                             and replayed; it applies when every problem has FP64 H psi (precision 0),
                             preconditioner 0 or 1, at most 136 bands, a stored FP64 projector table,
                             projector counts whose projection takes one GEMM tile shape (the row
                             tile follows the count: 64 rows below 256 projectors, 128 from there
                             at more than 64 bands), default launch choices and no snapshots, else
                             mode 1 runs.  1 launches each
                             problem's recorded segment graph in turn every check round; 0 launches one
                             graph holding all running problems' segments as child graphs (rebuilt when
                             a problem finishes or changes precision).  Every mode runs each problem's
                             own kernels, tiles and reduction order: results are bit for bit those of
                             solving the problems one by one. */
    int32_t learned_stall;/* precond 2: fall back to the paper's M(G) after this many checks without the
                             best residual halving (default 25; 0 = never).  A folded solve normally
                             spends a few hundred iterations on a plateau where the residual falls
                             slowly whatever the preconditioner, so the count must outlast it */
    int32_t recover;      /* 1 (default): when the Gram matrix loses positive definiteness, restart from
                             the iterate of the last check (kept in psi) with the failing band replaced by
                             a seeded random vector, up to three times; 0: return PW_ENOTPD */
    int32_t fault_check;  /* tests of the recovery: at this check (1-based) the host marks the Gram
                             factorisation as failed at band nb / 2 before reading its status (0 = never) */
} pw_cg_opts;

typedef struct {
    int32_t iters;        /* CG iterations done */
    int32_t converged;    /* 1 if max Delta <= tol */
    int64_t n_hpsi;       /* band-H psi applications */
    double max_resid;     /* final max_i Delta_i, from an FP64 H psi */
    double seconds;       /* wall time of the solve */
    int32_t n_hist;       /* in: capacity of hist; out: entries written */
    double *hist;         /* host, optional: [n_hist][2] = (iteration, max Delta) */
    int32_t n_snap;       /* out: snapshots written to snap_buf */
    int32_t precond_switch_it; /* out: iteration at which precond 2 fell back to M(G), -1 if it did not */
    int32_t recoveries;   /* out: restarts after a lost Gram factorisation */
    int32_t fused;        /* out (pw_batch_solve): 1 when the problem ran in the fused batch */
    double ms[4];         /* out: GPU time (HIP events on the stream) of the set-up (first orthonormalisation,
                             two H psi, Rayleigh-Ritz), the CG iterations, the checks (residuals and
                             Rayleigh-Ritz every check_every iterations) and the final Rayleigh-Ritz in H;
                             zeros from pw_batch_solve */
} pw_cg_stats;

void pw_cg_opts_default(pw_cg_opts *opts);

/* Folded-spectrum PCG for the nb states nearest e_ref.
 * psi   device complex128 [nb][ld]: in, start block (any full-rank block);
 *       out, Ritz vectors of H ascending in energy, orthonormal.
 * eig   host [nb]: Ritz values theta_i (Ha), ascending.
 * resid host [nb]: Delta_i = ||H psi_i - theta_i psi_i|| from an FP64 H psi.
 * The solver synchronises `stream` once per check_every iterations. */
pw_status pw_folded_cg_solve(pw_ctx *ctx, double e_ref, int32_t nb, void *psi, int64_t ld,
                             double *eig, double *resid, const pw_cg_opts *opts,
                             pw_cg_stats *stats, void *stream);

/* Batched folded-spectrum solves of nprob independent problems (many cells of
 * uneven grid size and many E_ref values), each with its own context ctx[p]
 * (distinct), start/result block psi[p] (device complex128 [nb][ld[p]]) and
 * e_ref[p]; eig[p], resid[p] (host [nb] each; eig/resid may be NULL) as for
 * pw_folded_cg_solve, stats (host [nprob], optional), status (host [nprob],
 * optional) the per-problem result.  Every problem runs the kernels of its own
 * pw_folded_cg_solve in the same order (same results); the check_every
 * iterations between checks are recorded once per problem into a graph, and every
 * check round replays the running problems' graphs on `stream` (one after another,
 * or as one graph of child graphs: opts->batch_launch), with one host read of every
 * problem's residuals in between.  Snapshots are not supported.  Returns PW_OK
 * if every problem converged, PW_ENOCONV if some did not, else the first other
 * error.  Synchronises. */
pw_status pw_batch_solve(int32_t nprob, pw_ctx *const *ctx, const double *e_ref, int32_t nb, void *const *psi,
                         const int64_t *ld, double *const *eig, double *const *resid, const pw_cg_opts *opts,
                         pw_cg_stats *stats, int32_t *status, void *stream);

/* ---------------------------------------------------------------------------
 * Folded linear equation of the system states (Sec. II.A system-state equation,
 * Sec. II.B folded equation, functional F and preconditioner M').
 *
 * Solves (H - E)^2 psi_l = (H - E) w_l for nrhs sources at once by column-wise
 * preconditioned CG (each column its own step lengths); the error of a column
 * is the paper's ||(H - E) psi_l - w_l||, and the solve stops when its maximum
 * over the columns is <= tol.  Preconditioner:
 *   precond 0: the paper's G-diagonal M(G) = 1 / ((T_G - E)^2 + delta_e^2);
 *   precond 1: M' built from nev approximate eigenpairs (phi_i, eps_i, Delta_i),
 *     applied in its Hermitian form
 *       M' = (1 - P) M (1 - P) + sum_i |phi_i><phi_i| / ((eps_i - E)^2 + Delta_i^2),
 *     P = sum_i |phi_i><phi_i| (the paper prints M (1 - P) + ..., which is not
 *     Hermitian unless M commutes with P; both agree on span{phi_i}).
 * ------------------------------------------------------------------------- */
typedef struct {
    double tol;           /* stop when max_l ||(H - E) psi_l - w_l|| <= tol (paper: 1e-8 a.u.) */
    int32_t maxit;        /* PCG iterations cap */
    int32_t precond;      /* 0 M(G), 1 M' (needs nev >= 1 eigenpairs) */
    double delta_e;       /* dE of M(G) (Ha), > 0 */
    int32_t check_every;  /* iterations between reads of the error by the host */
    int32_t verbose;      /* print the error at each check to stderr */
    int32_t use_graph;    /* 1 (default): record the check_every iterations between two error reads
                             once into a HIP graph and replay it (same kernels in the same order);
                             0: launch them one by one.  Not used while per-stage profiling is on. */
} pw_lin_opts;

typedef struct {
    int32_t iters;        /* PCG iterations done */
    int32_t converged;    /* 1 if the error reached tol at a check */
    int64_t n_hpsi;       /* band-H psi applications */
    double max_resid;     /* final max_l ||(H - E) psi_l - w_l|| from a fresh H psi */
    double seconds;       /* wall time of the solve */
    int32_t n_hist;       /* in: capacity of hist; out: entries written */
    double *hist;         /* host, optional: [n_hist][2] = (iteration, max error) */
} pw_lin_stats;

void pw_lin_opts_default(pw_lin_opts *opts);

/* ctx    complex128 context; nrhs in [1, max_bands].
 * w      device complex128 [nrhs][ldw], the sources (read only).
 * psi    device complex128 [nrhs][ld]: in, the start guess (zeros for psi_0 = 0);
 *        out, the solution.
 * phi    device complex128 [nev][ldphi], orthonormal approximate eigenvectors
 *        (e.g. pw_folded_cg_solve's output); used when precond = 1, may be NULL
 *        with nev = 0 otherwise.
 * eps, delta  host [nev]: their energies eps_i (Ha) and errors Delta_i =
 *        ||H phi_i - eps_i phi_i|| (pw_folded_cg_solve's eig and resid).
 * resid  host [nrhs] (optional): final ||(H - E) psi_l - w_l|| from a fresh H psi.
 * Allocates its workspace (8 blocks of nrhs x npw complex128, and for M' an
 * nrhs x nev coefficient set) for the call and frees it at the end.  Returns
 * PW_ENOCONV (solution and residuals still written) if maxit is reached first.
 * Synchronises `stream` once per check_every iterations. */
pw_status pw_folded_linear_solve(pw_ctx *ctx, double e, int32_t nrhs, const void *w, int64_t ldw, void *psi,
                                 int64_t ld, int32_t nev, const void *phi, int64_t ldphi, const double *eps,
                                 const double *delta, double *resid, const pw_lin_opts *opts, pw_lin_stats *stats,
                                 void *stream);

/* ---------------------------------------------------------------------------
 * Chebyshev filter diagonalisation of an energy window (Sec. II.B, ChebFD
 * paragraph: a Chebyshev polynomial p(H) imitating a window around E, applied to
 * a block of vectors, then a subspace diagonalisation; repeated).
 *
 * The filter is p(H) = sum_{k<=degree} g_k mu_k T_k((H - c)/h) with c, h the
 * centre and half width of [emin, emax], mu_k the Chebyshev coefficients of the
 * indicator of [e - half_width, e + half_width] and g_k Jackson's damping
 * factors; one complex128 H psi per degree.  [emin, emax] must contain the whole
 * spectrum of H (else the recurrence grows without bound); pw_spectral_bounds
 * estimates it.  All three synchronise `stream`; blocks are device complex128
 * band-major [nb][ld], 1 <= nb <= max_bands; each call allocates its scratch
 * (four nb x npw blocks) and frees it before returning.
 * ------------------------------------------------------------------------- */

/* out = p(H) psi (psi and out must not alias).  PW_EINVAL for degree outside
 * [0, 100000], emax <= emin, half_width <= 0 or a window outside [emin, emax]. */
pw_status pw_cheb_filter(pw_ctx *ctx, int32_t nb, const void *psi, int64_t ld, void *out, int64_t ldo, double e,
                         double half_width, int32_t degree, double emin, double emax, void *stream);

/* One ChebFD step in place: psi <- Rayleigh-Ritz vectors of H on span p(H) psi
 * (Gram/Cholesky orthonormalisation, then <phi_i|H|phi_j> diagonalised), with
 * eig (host [nb], optional) the Ritz values ascending and resid (host [nb],
 * optional) ||H phi_i - eps_i phi_i||.  nb <= 1024.  PW_ENOTPD if the filtered
 * block lost rank (more bands than the filter keeps), PW_ENAN if it is not
 * finite (bounds that miss part of the spectrum). */
pw_status pw_chebfd_step(pw_ctx *ctx, int32_t nb, void *psi, int64_t ld, double e, double half_width, int32_t degree,
                         double emin, double emax, double *eig, double *resid, void *stream);

/* Estimate of an interval holding the spectrum of H: `steps` (2..1024) Lanczos
 * steps from the start vector v0 (device complex128 [npw], not zero; the caller
 * draws it), the extreme Ritz values of the tridiagonal widened by twice their
 * residual bounds and by 1% of their spread.  An estimate, not a proof: a start
 * vector orthogonal to an extreme eigenvector misses it. */
pw_status pw_spectral_bounds(pw_ctx *ctx, const void *v0, int32_t steps, double *emin, double *emax, void *stream);

/* Wave-function interpolation between two k-points (Sec. II.C): from n
 * orthonormal eigenstates psi1 (device complex128 [n][ld1] on ctx1's sphere) with
 * energies eps1 (host [n]) at k1, and psi2/eps2 likewise at k2, the energies
 * eps_out (host [n], ascending) at k = k2 + alpha (k1 - k2) from
 *   H_ij(k) = alpha eps1_i delta_ij + (1 - alpha) sum_m conj(U_im) U_jm eps2_m,
 * U the row-wise Gram-Schmidt of S_ij = <psi_j(k2)|psi_i(k1)>; and, if psi_out is
 * not NULL, the interpolated states alpha sum_j c_j psi1_j + (1 - alpha)
 * sum_jl c_j U_jl psi2_l on ctxk's sphere (device complex128 [n][ldo]; not
 * renormalised).  The three contexts (at k1, k2 and k) must share cell, grid and
 * cutoff; coefficients are matched by Miller triple, one missing from a sphere
 * counting as zero.  n <= 1024; psi_out must not alias psi1 or psi2.  PW_ENOTPD
 * if the overlap rows are linearly dependent.  Allocates its scratch for the
 * call; synchronises `stream`. */
pw_status pw_kinterp(pw_ctx *ctx1, pw_ctx *ctx2, pw_ctx *ctxk, double alpha, int32_t n, const void *psi1, int64_t ld1,
                     const double *eps1, const void *psi2, int64_t ld2, const double *eps2, double *eps_out,
                     void *psi_out, int64_t ldo, void *stream);

/* ---------------------------------------------------------------------------
 * Learned preconditioner (precond = 2).  Not in the paper: a network standing in
 * for the diagonal preconditioner (the paper's is M(G), Sec. II.B).  Per |G+k|
 * shell s and band i, f_si = MLP(T_s/Ecut, T_i/Ecut, E_ref/Ecut), a 3-64-64-1 tanh
 * network with output 8 tanh(r/8); the CG uses K_i(G) = M(G) exp(f), M(G) the
 * paper's preconditioner with the solve's delta_e.
 * Parameters (float32, PW_MLP_NPARAM): W1[64][3], b1[64], W2[64][64], b2[64],
 * W3[64], b3.  Training loss per band and snapshot: 1 - Re<K g, e>/(|K g| |e|),
 * e = (I - Psi* Psi*^H) psi the band's error outside the converged subspace (the
 * CG steps along -K g, so K g should point along e); it
 * depends on a snapshot only through shell tables A_si = sum_{G in s} Re(conj e
 * K0 g), B_si = sum |K0 g|^2, C_si = sum |e|^2 (doubles, [3][nshell][nb]).
 * All pointers below are device pointers unless stated.
 * ------------------------------------------------------------------------- */
#define PW_MLP_NPARAM 4481

/* Install the network used by precond = 2 (weights copied into the context). */
pw_status pw_mlp_set(pw_ctx *ctx, const float *weights);

/* f [nshell][nb] for shell energies shell_t [nshell], band kinetic energies
 * tband [nb] (both float64, Ha) at one e_ref; ecut scales the inputs. */
pw_status pw_mlp_forward(int32_t nshell, int32_t nb, const double *shell_t, const double *tband, double e_ref,
                         double ecut, const float *weights, float *f, void *stream);

/* Shell tables of one snapshot: x_snap [nb][ld] an iterate of a solve at e_ref,
 * x_conv [nb][ld] the converged orthonormal block.  Recomputes the gradient
 * g = A x - <x|A|x> x with two FP64 H psi, the weights K0 = M(G) with delta_e
 * (> 0, Ha) and the band kinetic energies (written to tband [nb]), and writes
 * tabs [3][nshell][nb]: per shell s
 * and band i, the sums over the shell of Re(conj(e) K0 g), |K0 g|^2 and |e|^2 with
 * e = (I - X* X*^H) x.  weight_delta >= 0 multiplies the sums of shell s by
 * (T_s - e_ref)^2 + weight_delta^2 (an approximate A-norm for the cosine loss);
 * weight_delta < 0 leaves them unweighted. */
pw_status pw_mlp_harvest(pw_ctx *ctx, double e_ref, int32_t nb, const void *x_snap, const void *x_conv, int64_t ld,
                         double delta_e, double weight_delta, double *tabs, double *tband, void *stream);

/* Scratch bytes needed by pw_mlp_loss_grad (host function). */
int64_t pw_mlp_work_bytes(int32_t nshell, int32_t nb, int32_t nsnap);

/* Mean loss over nsnap snapshots x nb bands and its gradient (float32 [NPARAM]).
 * tband [nsnap][nb], e_ref [nsnap], tabs [nsnap][3][nshell][nb]; loss: one float;
 * work: caller-allocated, >= pw_mlp_work_bytes.  Deterministic (no atomics). */
pw_status pw_mlp_loss_grad(int32_t nshell, int32_t nb, int32_t nsnap, const double *shell_t, const double *tband,
                           const double *e_ref, double ecut, const double *tabs, const float *weights, float *grad,
                           float *loss, void *work, int64_t work_bytes, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8); step counts from 1. */
pw_status pw_mlp_adam(float *weights, const float *grad, float *m, float *v, int32_t step, float lr, void *stream);

/* nsteps full-batch training steps (loss/gradient, then Adam at steps step0+1 ..
 * step0+nsteps) on the device.  grad [NPARAM] and m, v (Adam moments) are
 * caller-owned device float32; loss_hist (host, optional, [nsteps]) receives the
 * loss before each step.  Synchronises once at the end. */
pw_status pw_mlp_train(int32_t nshell, int32_t nb, int32_t nsnap, const double *shell_t, const double *tband,
                       const double *e_ref, double ecut, const double *tabs, float *weights, float *grad, float *m,
                       float *v, int32_t step0, int32_t nsteps, float lr, float *loss_hist, void *work,
                       int64_t work_bytes, void *stream);

/* Per-stage timing with HIP events recorded on the stream each stage is
 * launched on.  pw_profile_begin allocates room for max_records stage launches
 * (allocation happens here, not in the timed calls); pw_profile_end waits for
 * the recorded events and returns, per stage kind, the summed milliseconds and
 * the launch count.  Kinds: 0 z pass inverse, 1 xy pass (2D FFTs and V),
 * 2 z pass forward + kinetic, 3 projection <beta|psi>, 4 back-projection
 * (for generated rows: per chunk, the row generation counted with neither), and
 * the folded-CG solver's FP64 block products: 5 the rotation of X, Y and AX by
 * one nb x nb matrix (three products of 8 npw nb^2 flops in one launch), 6 the nb x nb
 * products A^H B of two different blocks (8 npw nb^2 flops), 7 the other single
 * rotations nb x nb times nb x npw (8 npw nb^2 flops; the P update, the Ritz
 * rotations), 8 the Hermitian Gram matrices X^H X (the tiles on and below the
 * diagonal; 4 npw nb (nb + 1) flops determine the matrix).
 * Inside pw_folded_cg_solve only the CG iterations are recorded, not the set-up,
 * the checks or the final Rayleigh-Ritz. */
#define PW_PROF_NKINDS 9
pw_status pw_profile_begin(pw_ctx *ctx, int32_t max_records);
pw_status pw_profile_end(pw_ctx *ctx, double *ms, int64_t *launches);

const char *pw_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PW_H */
