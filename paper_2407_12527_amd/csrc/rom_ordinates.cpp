// rom_ordinates.cpp -- ordinate sets of librom (host, double precision).
//
// ROM sets (Sec. 3.1 steps 1-2; Sec. 4.2): the first-quadrant (zeta, theta) rectangle
// [0,1] x [0,pi/2] is split into nz x nt equal cells (zeta bands from the pole down, theta bands
// from 0 up); each cell receives one point drawn uniformly and independently; the other three
// quadrants are the exact mirror images of eq. (3.5); all weights are 1/n (eq. (3.4)).
// Deterministic quadratures: the uniform and Gaussian sets of Appendix A.
//
// Random numbers come from SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the state advances by
// 0x9e3779b97f4a7c15 and each output is the advanced state through the xor-shift-multiply
// finalizer; u = (x >> 11) * 2^-53.  Sample s of a seed uses the stream seeded with output s+1
// of the master generator.  These formulas are the published definitions and are evaluated
// exactly as written (no fused multiply-add), so generated sets are reproducible bit for bit.
#include <cmath>
#include <cstdint>
#include <vector>

#include "rom_host.h"

#pragma clang fp contract(off)

namespace rom {

namespace {

constexpr uint64_t kGolden = 0x9e3779b97f4a7c15ULL;
constexpr double kPi = 3.14159265358979323846;

inline uint64_t mix64(uint64_t x)
{
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ULL;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebULL;
    x ^= x >> 31;
    return x;
}

struct SplitMix64 {
    uint64_t state;
    explicit SplitMix64(uint64_t s) : state(s) {}
    uint64_t next()
    {
        state += kGolden;
        return mix64(state);
    }
    double uniform() { return double(next() >> 11) * 0x1.0p-53; }
};

inline uint64_t stream_seed(uint64_t seed, int64_t sample)
{
    // output number sample+1 of SplitMix64(seed), reached directly
    return mix64(seed + uint64_t(sample + 1) * kGolden);
}

inline void store(double* dirs, int l, double c, double s, double z)
{
    dirs[3 * l] = c;
    dirs[3 * l + 1] = s;
    dirs[3 * l + 2] = z;
}

void mirror(double* dirs, int m, int l, double c, double s, double z)
{
    store(dirs, l, c, s, z);
    store(dirs, l + m, -c, s, z);
    store(dirs, l + 2 * m, -c, -s, z);
    store(dirs, l + 3 * m, c, -s, z);
}

// Legendre polynomial of degree n and its derivative at x (Bonnet recursion).
void legendre_pd(int n, double x, double& p, double& dp)
{
    double pm1 = 1.0, pn = x;
    if (n == 0) {
        p = 1.0;
        dp = 0.0;
        return;
    }
    for (int k = 2; k <= n; ++k) {
        const double pk = ((2 * k - 1) * x * pn - (k - 1) * pm1) / k;
        pm1 = pn;
        pn = pk;
    }
    p = pn;
    dp = n * (x * pn - pm1) / ((x - 1.0) * (x + 1.0));
}

// Positive roots of P_{2N} in decreasing order, by Newton's method.
std::vector<double> positive_legendre_roots(int deg, int count)
{
    std::vector<double> r(count);
    for (int i = 0; i < count; ++i) {
        double x = std::cos(kPi * (i + 0.75) / (deg + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre_pd(deg, x, p, dp);
            const double step = p / dp;
            x -= step;
            if (std::fabs(step) < 1e-16) break;
        }
        r[i] = x;
    }
    return r;
}

}  // namespace

int zeta_bands(int m)
{
    int nz = 1;
    for (int d = 1; int64_t(d) * d <= m; ++d)
        if (m % d == 0) nz = d;
    return nz;
}

int ordinate_count(const rom_ord_spec& sp)
{
    switch (sp.kind) {
    case ROM_ORD_STRATIFIED: return (sp.p1 > 0 && sp.p2 > 0) ? 4 * sp.p1 * sp.p2 : -1;
    case ROM_ORD_IID_SPHERE: return sp.p1 > 0 ? sp.p1 : -1;
    case ROM_ORD_UNIFORM2D: return sp.p1 > 0 ? 4 * sp.p1 * sp.p1 : -1;
    case ROM_ORD_GAUSS2D: return sp.p1 > 0 ? 2 * sp.p1 * (sp.p1 + 1) : -1;
    default: return -1;
    }
}

int generate_ordinates(const rom_ord_spec& sp, uint64_t seed, int64_t sample, double* dirs, double* w)
{
    const int n = ordinate_count(sp);
    if (n <= 0) return ROM_E_ARG;
    switch (sp.kind) {
    case ROM_ORD_STRATIFIED: {
        const int nz = sp.p1, nt = sp.p2, m = nz * nt;
        SplitMix64 rng(stream_seed(seed, sample));
        for (int i = 0; i < nz; ++i) {
            for (int j = 0; j < nt; ++j) {
                const double uz = rng.uniform();
                const double ut = rng.uniform();
                const double zeta = 1.0 - (double(i) + uz) / double(nz);
                const double theta = (double(j) + ut) * (0.5 * kPi) / double(nt);
                const double rho = std::sqrt((1.0 - zeta) * (1.0 + zeta));
                mirror(dirs, m, i * nt + j, rho * std::cos(theta), rho * std::sin(theta), zeta);
            }
        }
        for (int l = 0; l < n; ++l) w[l] = 1.0 / double(n);
        return ROM_OK;
    }
    case ROM_ORD_IID_SPHERE: {
        SplitMix64 rng(stream_seed(seed, sample));
        for (int l = 0; l < n; ++l) {
            const double uz = rng.uniform();
            const double ut = rng.uniform();
            const double zeta = 2.0 * uz - 1.0;
            const double theta = ut * (2.0 * kPi);
            const double rho = std::sqrt((1.0 - zeta) * (1.0 + zeta));
            store(dirs, l, rho * std::cos(theta), rho * std::sin(theta), zeta);
            w[l] = 1.0 / double(n);
        }
        return ROM_OK;
    }
    case ROM_ORD_UNIFORM2D: {
        // eq. (A.5): zeta_i = (2N-2i+1)/(2N), theta_j = (2j-1) pi / (4N), weight 1/(4N^2)
        const int N = sp.p1, m = N * N;
        for (int i = 1; i <= N; ++i)
            for (int j = 1; j <= N; ++j) {
                const double zeta = double(2 * N - 2 * i + 1) / double(2 * N);
                const double theta = double(2 * j - 1) * kPi / double(4 * N);
                const double rho = std::sqrt((1.0 - zeta) * (1.0 + zeta));
                mirror(dirs, m, (i - 1) * N + (j - 1), rho * std::cos(theta), rho * std::sin(theta), zeta);
            }
        for (int l = 0; l < n; ++l) w[l] = 1.0 / double(n);
        return ROM_OK;
    }
    case ROM_ORD_GAUSS2D: {
        // Appendix A: level i = 1..N at the i-th largest positive root of P_{2N}, azimuths
        // (2j-1) pi / (4i), j = 1..i, weight 1 / (2 i (1 - zeta^2) P'_{2N}(zeta)^2)
        const int N = sp.p1, m = N * (N + 1) / 2;
        const std::vector<double> roots = positive_legendre_roots(2 * N, N);
        for (int i = 1; i <= N; ++i) {
            const double zeta = roots[i - 1];
            double p, dp;
            legendre_pd(2 * N, zeta, p, dp);
            const double wi = 1.0 / (2.0 * i * ((1.0 - zeta) * (1.0 + zeta)) * dp * dp);
            const double rho = std::sqrt((1.0 - zeta) * (1.0 + zeta));
            for (int j = 1; j <= i; ++j) {
                const double theta = double(2 * j - 1) * kPi / double(4 * i);
                const int l = i * (i - 1) / 2 + (j - 1);
                mirror(dirs, m, l, rho * std::cos(theta), rho * std::sin(theta), zeta);
                w[l] = w[l + m] = w[l + 2 * m] = w[l + 3 * m] = wi;
            }
        }
        return ROM_OK;
    }
    default: return ROM_E_ARG;
    }
}

// Slab ordinates (Sec. 4.1), weights normalized to sum 1 (the paper's 2/n with the 1/2 of the
// slab average folded in).  RANDOM: [-1, 1] in n equal cells (n even), one uniform draw in each
// cell of [-1, 0] (in order from -1, sample's own stream), the cells of [0, 1] receive the mirror
// images mu_l = -mu_{n+1-l}.  GAUSS: Gauss-Legendre nodes in decreasing order.  UNIFORM: the
// midpoints of n equal cells.
int slab_ordinates(int kind, int n, uint64_t seed, int64_t sample, double* mu, double* w)
{
    if (n <= 0 || !mu || !w) return ROM_E_ARG;
    switch (kind) {
    case ROM_SLAB_RANDOM: {
        if (n & 1) return ROM_E_ARG;
        SplitMix64 rng(stream_seed(seed, sample));
        const double width = 2.0 / double(n);
        for (int l = 0; l < n / 2; ++l) {
            const double u = rng.uniform();
            mu[l] = -1.0 + double(l) * width + u * width;
        }
        for (int l = n / 2; l < n; ++l) mu[l] = -mu[n - 1 - l];
        for (int l = 0; l < n; ++l) w[l] = 1.0 / double(n);
        return ROM_OK;
    }
    case ROM_SLAB_GAUSS: {
        // roots of P_n: the positive ones (decreasing), then their negatives, then 0 for odd n
        const std::vector<double> pos = positive_legendre_roots(n, n / 2);
        int l = 0;
        for (int i = 0; i < n / 2; ++i) mu[l++] = pos[i];
        if (n & 1) mu[l++] = 0.0;
        for (int i = n / 2 - 1; i >= 0; --i) mu[l++] = -pos[i];
        for (int k = 0; k < n; ++k) {
            double p, dp;
            legendre_pd(n, mu[k], p, dp);
            w[k] = 1.0 / (((1.0 - mu[k]) * (1.0 + mu[k])) * dp * dp);  // Gauss weight 2/(...) halved
        }
        return ROM_OK;
    }
    case ROM_SLAB_UNIFORM:
        for (int l = 0; l < n; ++l) {
            mu[l] = -1.0 + (2.0 * l + 1.0) / double(n);
            w[l] = 1.0 / double(n);
        }
        return ROM_OK;
    default: return ROM_E_ARG;
    }
}

// Scattering phase function of the cosine between two 3-D directions, folded over +-zeta':
// X-Y solutions are even in zeta, so each stored ordinate stands for the pair (c, s, +-zeta).
double phase_folded(int kind, double g, const double* u, const double* v)
{
    const double planar = u[0] * v[0] + u[1] * v[1];
    const double zz = u[2] * v[2];
    auto P = [&](double mu) -> double {
        if (kind == ROM_SCAT_LINEAR) return 1.0 + g * mu;  // eq. (2.1)
        if (kind == ROM_SCAT_HG) {
            const double d = 1.0 + g * g - 2.0 * g * mu;
            return (1.0 - g * g) / (d * std::sqrt(d));
        }
        return 1.0;
    };
    return 0.5 * (P(planar + zz) + P(planar - zz));
}

}  // namespace rom
