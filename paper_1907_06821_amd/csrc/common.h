// Shared definitions of libpw: complex types, error plumbing, context layout.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/pw.h"

namespace pw {

// ---------------------------------------------------------------------------
// complex arithmetic on HIP vector types (interleaved re, im)
// ---------------------------------------------------------------------------
template <typename T> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename T> using cplx = typename cvec<T>::type;

template <typename T> __host__ __device__ inline cplx<T> cmake(T re, T im) {
    cplx<T> z; z.x = re; z.y = im; return z;
}
template <typename T> __host__ __device__ inline cplx<T> cadd(cplx<T> a, cplx<T> b) {
    return cmake<T>(a.x + b.x, a.y + b.y);
}
template <typename T> __host__ __device__ inline cplx<T> csub(cplx<T> a, cplx<T> b) {
    return cmake<T>(a.x - b.x, a.y - b.y);
}
template <typename T> __host__ __device__ inline cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return cmake<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T> __host__ __device__ inline cplx<T> cmulc(cplx<T> a, cplx<T> b) {
    return cmake<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T> __host__ __device__ inline cplx<T> cscale(cplx<T> a, T s) {
    return cmake<T>(a.x * s, a.y * s);
}

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);
struct Fail {
    pw_status st;
};

#define PW_HIP(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            ::pw::set_error("%s:%d: %s -> %s", __FILE__, __LINE__, #call,                  \
                            hipGetErrorString(e_));                                       \
            throw ::pw::Fail{PW_EHIP};                                                    \
        }                                                                                 \
    } while (0)

#define PW_CHECK(cond, status, ...)                                                       \
    do {                                                                                  \
        if (!(cond)) {                                                                    \
            ::pw::set_error(__VA_ARGS__);                                                 \
            throw ::pw::Fail{status};                                                     \
        }                                                                                 \
    } while (0)

#define PW_LAUNCH_CHECK() PW_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// FFT plans
// ---------------------------------------------------------------------------
constexpr int kMaxStages = 12;
struct FftPlan {
    int n;
    int nstages;
    int radix[kMaxStages];
};
FftPlan make_plan(int n);   // factor n into radices 8, 4, 2, 3, 5
// radix schedules the autotuner tries: 0 make_plan, 1 radices 4 (2) 3 5 only,
// 2 make_plan's radices in ascending order
FftPlan make_plan_sched(int n, int sched);

// Launch choice of one FFT pass: kind 0 built-in default, 1 the compile-time
// length kernel, 2 the runtime-plan kernel with nthr threads and plans p0 (and
// p1 for the xy pass).
struct FftChoice {
    int kind = 0;
    int nthr = 0;
    bool vpf = false;       // four-lane xy kernel, complex128: V(r) loaded ahead
    FftPlan p0{}, p1{};
};
// back-projection GEMM tile per band count (complex128); -1: chosen by band count
struct GemmTune {
    static constexpr int kSlots = 8;
    int nb[kSlots] = {0, 0, 0, 0, 0, 0, 0, 0};
    int id[kSlots] = {-1, -1, -1, -1, -1, -1, -1, -1};
    int get(int n) const {
        for (int i = 0; i < kSlots; ++i)
            if (nb[i] == n) return id[i];
        return -1;
    }
    void set(int n, int v) {
        int slot = -1;
        for (int i = 0; i < kSlots && slot < 0; ++i)
            if (nb[i] == n || nb[i] == 0) slot = i;
        if (slot < 0) slot = kSlots - 1;
        nb[slot] = n;
        id[slot] = v;
    }
};
struct FftTune {
    FftChoice zinv, xy, zfwd;
};

// ---------------------------------------------------------------------------
// basis (host)
// ---------------------------------------------------------------------------
struct Basis {
    int npw = 0;
    std::vector<int32_t> miller;     // [npw][3]
    std::vector<double> kin;         // [npw]
    // z-columns: runs of consecutive n2 at fixed (n0, n1), in coefficient order
    int ncols = 0;
    std::vector<int32_t> col_start;  // [ncols + 1]
    std::vector<int32_t> col_i0;     // n0 mod N0
    std::vector<int32_t> col_i1;     // n1 mod N1
    std::vector<int32_t> col_n2lo;   // first n2 of the run
    std::vector<int32_t> shell;      // [npw]
    std::vector<double> shell_t;     // [nshell]
    int n0min = 0, n0max = 0;
};
void enumerate_miller(const pw_cell &c, std::vector<int32_t> &miller);
Basis build_basis(const pw_cell &c);

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { free_(); }
    void alloc(size_t b);
    void free_();
    template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

struct Solver;   // folded-CG workspace (solver.cpp)

// optional per-stage timing with HIP events on the launch stream
struct ProfRec {
    int kind;
    hipEvent_t a, b;
};

}  // namespace pw

struct pw_ctx {
    pw_cell cell;
    pw::Basis basis;
    int max_bands = 0;
    int flags = 0;
    int natom = 0, nl = 0, nproj = 0;
    std::vector<double> dproj;       // host copy [nproj]
    int device = 0;
    int64_t device_bytes = 0;
    pw::FftPlan plan[3];
    pw::FftTune tune[2];             // FFT launch choices: [0] complex128, [1] complex64
    pw::GemmTune nn_tune;            // back-projection GEMM tiles by band count (autotuner)
    pw::GemmTune rot_tune;           // block-rotation GEMM tiles (M = K = bands) by band count (autotuner)
    int bf16_variant = 0;            // launch variant of the BF16 projector GEMMs beyond 144 bands (autotuner)
    int cb = 16;                     // z-columns per workgroup in the z passes
    // device tables
    pw::DevBuf d_kin, d_zmap, d_colpos, d_colstart, d_vz64, d_vz32, d_tw64[3], d_tw32[3];
    pw::DevBuf d_colslot;            // [ncols]: column's place in a plane that holds only the touched x rows
    pw::DevBuf d_beta64, d_beta_bf16, d_dproj, d_dproj32, d_shell;
    pw::DevBuf d_betaT_bf16;         // BF16 planes of the transposed table [ldg][ldp] (back-projection)
    // complex128 projector rows generated per H psi, otf_atoms atoms at a time, instead of a stored
    // table (PW_PREP_C128_OTF): Miller triples and atom centres on the device, one chunk of rows
    bool beta_otf = false;
    int otf_atoms = 0;
    double sigma = 0.0;
    pw::DevBuf d_miller, d_pos, d_beta_chunk;
    pw::DevBuf d_bf16_ws;            // per-call BF16 planes of psi and of D . C
    int64_t ldb16 = 0;               // row length of the BF16 projector planes
    // hpsi workspace
    pw::DevBuf d_cols;               // [cols_bands][N2][ncols] of the widest prepared dtype
    int cols_bands = 0;              // bands per FFT launch (the column grid holds that many)
    pw::DevBuf d_proj;               // projections [nproj][max_bands] complex128
    pw::DevBuf d_partial;            // split-K partial sums
    pw::DevBuf d_ortho_ws, d_ortho_small;   // pw_orthonormalize scratch
    pw::DevBuf d_shell_t, d_shell_off, d_shell_pw;   // shell energies and plane waves grouped by shell
    pw::DevBuf d_mlp;                // learned-preconditioner weights (float32), empty until pw_mlp_set
    pw::Solver *solver = nullptr;
    // profiling (pw_profile_begin / pw_profile_end)
    bool prof_on = false;
    bool prof_pause = false;         // set by the folded-CG solver outside its iterations
    std::vector<hipEvent_t> prof_pool;
    std::vector<pw::ProfRec> prof_rec;
    size_t prof_next = 0;
};

namespace pw {
// Records a pair of events around a launch sequence when profiling is on.
struct ProfScope {
    pw_ctx *c;
    hipStream_t st;
    hipEvent_t b = nullptr;
    ProfScope(pw_ctx *ctx, int kind, hipStream_t s) : c(ctx), st(s) {
        if (c->prof_on && !c->prof_pause && c->prof_next + 2 <= c->prof_pool.size() &&
            c->prof_rec.size() < c->prof_rec.capacity()) {
            hipEvent_t a = c->prof_pool[c->prof_next++];
            b = c->prof_pool[c->prof_next++];
            c->prof_rec.push_back(ProfRec{kind, a, b});
            (void)hipEventRecord(a, st);
        }
    }
    ~ProfScope() {
        if (b) (void)hipEventRecord(b, st);
    }
};
}  // namespace pw
