// Per-context device tables: Kleinman-Bylander projectors on the sphere, the
// z-major potential copy, and precision conversions of them.
#include "kernels.h"

namespace pw {

// beta_{a,j}(G) = sqrt(8 pi^1.5 s^3) Y_j(q) exp(-|q|^2 s^2 / 2) exp(-i q.R_a) / sqrt(Omega),
// q = G + k, Y_s = 1, Y_{p,m} = sqrt(3) q_m / |q| (0 at q = 0); rows a*nl + j.
__global__ void k_projectors(int npw, int natom, int nl, const int32_t *__restrict__ miller, double c0, double c1,
                             double c2, double k0, double k1, double k2, const double *__restrict__ pos,
                             double sigma, double norm, double2 *__restrict__ beta) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int a = blockIdx.y;
    if (g >= npw) return;
    const double tp = 6.283185307179586476925286766559;
    const double q0 = tp * miller[3 * g] / c0 + k0;
    const double q1 = tp * miller[3 * g + 1] / c1 + k1;
    const double q2 = tp * miller[3 * g + 2] / c2 + k2;
    const double qq = q0 * q0 + q1 * q1 + q2 * q2;
    const double qn = sqrt(qq);
    const double rad = norm * exp(-0.5 * qq * sigma * sigma);
    const double ph = q0 * pos[3 * a] + q1 * pos[3 * a + 1] + q2 * pos[3 * a + 2];
    double sn, cs;
    sincos(ph, &sn, &cs);
    const double2 e = make_double2(cs, -sn);
    double2 *row = beta + (int64_t)a * nl * npw;
    row[g] = make_double2(rad * e.x, rad * e.y);
    if (nl == 4) {
        const double s3 = 1.7320508075688772935274463415059;
        const double qs[3] = {q0, q1, q2};
        for (int m = 0; m < 3; ++m) {
            const double y = qn > 0.0 ? s3 * qs[m] / qn : 0.0;
            row[(int64_t)(m + 1) * npw + g] = make_double2(rad * y * e.x, rad * y * e.y);
        }
    }
}

void build_projectors(int npw, int natom, int nl, const int32_t *d_miller, const pw_cell &c, const double *d_pos,
                      double sigma, void *beta, hipStream_t st) {
    const double omega = c.cell[0] * c.cell[1] * c.cell[2];
    const double norm = std::sqrt(8.0 * std::pow(M_PI, 1.5) * sigma * sigma * sigma) / std::sqrt(omega);
    hipLaunchKernelGGL(k_projectors, dim3((npw + 255) / 256, natom), dim3(256), 0, st, npw, natom, nl, d_miller,
                       c.cell[0], c.cell[1], c.cell[2], c.kpt[0], c.kpt[1], c.kpt[2], d_pos, sigma, norm,
                       (double2 *)beta);
    PW_LAUNCH_CHECK();
}

// vz[z][x][y] = v[x][y][z], float64 and float32 copies
__global__ void k_vtranspose(int n0, int n1, int n2, const double *__restrict__ v, double *__restrict__ vz64,
                             float *__restrict__ vz32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)n0 * n1 * n2;
    if (i >= n) return;
    const int z = (int)(i % n2);
    const int64_t xy = i / n2;
    const double val = v[i];
    if (vz64) vz64[(int64_t)z * n0 * n1 + xy] = val;
    if (vz32) vz32[(int64_t)z * n0 * n1 + xy] = (float)val;
}

void build_vz(int n0, int n1, int n2, const double *v, double *vz64, float *vz32, hipStream_t st) {
    const int64_t n = (int64_t)n0 * n1 * n2;
    hipLaunchKernelGGL(k_vtranspose, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n0, n1, n2, v, vz64, vz32);
    PW_LAUNCH_CHECK();
}

// split complex128 rows into BF16 real and imaginary planes (round to nearest even)
__device__ inline uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

__global__ void k_to_bf16_planes(int rows, int npw, int64_t ldp, const double2 *__restrict__ src,
                                 uint16_t *__restrict__ re, uint16_t *__restrict__ im, int panel) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (r >= rows) return;
    if (g < ldp) {
        const double2 v = g < npw ? src[(int64_t)r * npw + g] : make_double2(0.0, 0.0);
        const int64_t o = panel ? bf16_panel_index(r, g, ldp) : (int64_t)r * ldp + g;
        re[o] = to_bf16((float)v.x);
        im[o] = to_bf16((float)v.y);
    }
}

// rows x npw complex128 -> BF16 planes of ldp columns, row-major or in 16-row panels
// (re and im then start on a panel boundary)
void beta_to_bf16(int rows, int npw, int64_t ldp, const void *src, void *re, void *im, hipStream_t st, bool panel) {
    hipLaunchKernelGGL(k_to_bf16_planes, dim3((unsigned)((ldp + 255) / 256), rows), dim3(256), 0, st, rows, npw, ldp,
                       (const double2 *)src, (uint16_t *)re, (uint16_t *)im, panel ? 1 : 0);
    PW_LAUNCH_CHECK();
}

}  // namespace pw
