// Plane-wave basis, z-column tables, shells and FFT factorisation (host side).
//
// The basis is every Miller triple n with (1/2)|G + k|^2 <= Ecut, G = 2 pi n_i / L_i
// (plane-wave cutoff, Sec. II computational details), ordered lexicographically in
// (n0, n1, n2).  At fixed (n0, n1) the kept n2 form one run of consecutive integers
// (the sphere's chord), which is what the z pass of the FFT consumes.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <numeric>

#include "common.h"

namespace pw {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

const char *last_error() { return g_err.c_str(); }

static inline double kinetic_of(const pw_cell &c, int n0, int n1, int n2) {
    const double tp = 2.0 * M_PI;
    double q0 = tp * n0 / c.cell[0] + c.kpt[0];
    double q1 = tp * n1 / c.cell[1] + c.kpt[1];
    double q2 = tp * n2 / c.cell[2] + c.kpt[2];
    return 0.5 * (q0 * q0 + q1 * q1 + q2 * q2);
}

void enumerate_miller(const pw_cell &c, std::vector<int32_t> &miller) {
    PW_CHECK(c.ecut > 0 && c.cell[0] > 0 && c.cell[1] > 0 && c.cell[2] > 0, PW_EINVAL,
             "cell lengths and ecut must be positive");
    const double gmax = std::sqrt(2.0 * c.ecut);
    int nmax[3];
    for (int a = 0; a < 3; ++a)
        nmax[a] = (int)std::ceil((gmax + std::fabs(c.kpt[a])) * c.cell[a] / (2.0 * M_PI)) + 1;
    miller.clear();
    for (int n0 = -nmax[0]; n0 <= nmax[0]; ++n0)
        for (int n1 = -nmax[1]; n1 <= nmax[1]; ++n1)
            for (int n2 = -nmax[2]; n2 <= nmax[2]; ++n2)
                if (kinetic_of(c, n0, n1, n2) <= c.ecut) {
                    miller.push_back(n0);
                    miller.push_back(n1);
                    miller.push_back(n2);
                }
}

Basis build_basis(const pw_cell &c) {
    Basis b;
    enumerate_miller(c, b.miller);
    b.npw = (int)(b.miller.size() / 3);
    PW_CHECK(b.npw > 0, PW_EINVAL, "empty basis");
    int mx[3] = {0, 0, 0};
    for (int g = 0; g < b.npw; ++g)
        for (int a = 0; a < 3; ++a) mx[a] = std::max(mx[a], std::abs(b.miller[3 * g + a]));
    for (int a = 0; a < 3; ++a)
        PW_CHECK(2 * mx[a] + 1 <= c.n[a], PW_EINVAL,
                 "cutoff sphere does not fit the grid on axis %d: 2*%d+1 > %d", a, mx[a], c.n[a]);
    b.kin.resize(b.npw);
    for (int g = 0; g < b.npw; ++g)
        b.kin[g] = kinetic_of(c, b.miller[3 * g], b.miller[3 * g + 1], b.miller[3 * g + 2]);
    // z-columns
    b.col_start.clear();
    b.n0min = b.miller[0];
    b.n0max = b.miller[0];
    for (int g = 0; g < b.npw; ++g) {
        const int n0 = b.miller[3 * g], n1 = b.miller[3 * g + 1], n2 = b.miller[3 * g + 2];
        bool fresh = (g == 0) || n0 != b.miller[3 * (g - 1)] || n1 != b.miller[3 * (g - 1) + 1];
        if (!fresh) PW_CHECK(n2 == b.miller[3 * (g - 1) + 2] + 1, PW_EINVAL, "non-contiguous column");
        if (fresh) {
            b.col_start.push_back(g);
            b.col_i0.push_back(((n0 % c.n[0]) + c.n[0]) % c.n[0]);
            b.col_i1.push_back(((n1 % c.n[1]) + c.n[1]) % c.n[1]);
            b.col_n2lo.push_back(n2);
        }
        b.n0min = std::min(b.n0min, n0);
        b.n0max = std::max(b.n0max, n0);
    }
    b.ncols = (int)b.col_start.size();
    b.col_start.push_back(b.npw);
    // shells: sort T ascending, new shell when consecutive values differ by > 1e-9 Ha
    std::vector<int> order(b.npw);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b.kin[x] < b.kin[y]; });
    b.shell.assign(b.npw, 0);
    int sid = -1;
    for (int i = 0; i < b.npw; ++i) {
        const int g = order[i];
        if (i == 0 || b.kin[g] - b.kin[order[i - 1]] > 1e-9) {
            ++sid;
            b.shell_t.push_back(b.kin[g]);
        }
        b.shell[g] = sid;
    }
    return b;
}

FftPlan make_plan(int n) {
    FftPlan p{};
    p.n = n;
    PW_CHECK(n >= 1 && n <= 4096, PW_EINVAL, "FFT length %d out of range", n);
    int m = n, e2 = 0;
    while (m % 2 == 0) { m /= 2; ++e2; }
    std::vector<int> r;
    int n8 = e2 / 3, rem = e2 % 3;
    if (rem == 1 && n8 > 0) { --n8; r.push_back(4); r.push_back(4); }
    else if (rem == 1) r.push_back(2);
    else if (rem == 2) r.push_back(4);
    for (int i = 0; i < n8; ++i) r.push_back(8);
    while (m % 3 == 0) { m /= 3; r.push_back(3); }
    while (m % 5 == 0) { m /= 5; r.push_back(5); }
    PW_CHECK(m == 1, PW_EINVAL, "FFT length %d has a prime factor other than 2, 3, 5", n);
    PW_CHECK((int)r.size() <= kMaxStages, PW_EINVAL, "FFT length %d needs too many stages", n);
    // larger radices first
    std::sort(r.begin(), r.end(), [](int a, int b) { return a > b; });
    p.nstages = (int)r.size();
    for (int i = 0; i < p.nstages; ++i) p.radix[i] = r[i];
    return p;
}

FftPlan make_plan_sched(int n, int sched) {
    FftPlan p = make_plan(n);
    if (sched == 1) {
        int m = n;
        std::vector<int> r;
        while (m % 4 == 0) { m /= 4; r.push_back(4); }
        if (m % 2 == 0) { m /= 2; r.push_back(2); }
        while (m % 3 == 0) { m /= 3; r.push_back(3); }
        while (m % 5 == 0) { m /= 5; r.push_back(5); }
        PW_CHECK((int)r.size() <= kMaxStages, PW_EINVAL, "FFT length %d needs too many stages", n);
        std::sort(r.begin(), r.end(), [](int a, int b) { return a > b; });
        p.nstages = (int)r.size();
        for (int i = 0; i < p.nstages; ++i) p.radix[i] = r[i];
    } else if (sched == 2) {
        std::reverse(p.radix, p.radix + p.nstages);
    }
    return p;
}

}  // namespace pw
