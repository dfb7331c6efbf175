/*
 * rom_oracle.c -- plain FP64 CPU oracle for discrete-ordinate (DOM) and random-ordinate (ROM)
 * source iteration of the steady radiative transport equation in X-Y geometry.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  This is the independent reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or helper with the GPU
 * library, and it never calls it.
 *
 * Paper: L. Li, M. Tang, Y. Yang, "Random ordinate method for mitigating the ray effect in
 * radiative transport equation simulations", arXiv:2407.12527.
 *
 * Everything is written for clarity, not speed: double precision throughout, textbook loop
 * orders, one ordinate sweep at a time (ordinates may run on separate OpenMP threads, since
 * they are independent once the source is fixed), and sums taken in index order.
 *
 * Readings of points the paper leaves open:
 *   - spatial scheme: first-order upwind ("step") on the main path; the paper's own diamond
 *     difference (Sec. 2) is available as ORC_SCHEME_DD;
 *   - source iteration starts from phi^0 = 0 (the Neumann series of Sec. 3.2, eq. (3.10)) and
 *     stops when max|phi^k - phi^{k-1}| <= tol * max|phi^k|;
 *   - random ordinates: one independent uniform draw per (zeta, theta) cell of the first
 *     quadrant (Sec. 3.1 steps 1-2; Sec. 4.2), mirrored into the other quadrants by exact sign
 *     flips (eq. (3.5));
 *   - random numbers: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), u = (x >> 11) * 2^-53;
 *   - anisotropic kernels are folded over +-zeta' because the X-Y solution is even in zeta.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_EARG (-1)
#define ORC_ENOMEM (-2)

#define ORC_SCHEME_STEP 0
#define ORC_SCHEME_DD 1

#define ORC_SCAT_ISO 0
#define ORC_SCAT_LINEAR 1
#define ORC_SCAT_HG 2
#define ORC_SCAT_DENSE 3
#define ORC_SCAT_NORMALIZE 0x10 /* flag: rescale P so that sum_l w_l P_l'l = 1 (remark, Sec. 3.1) */

#define ORC_ORD_STRATIFIED 0
#define ORC_ORD_IID_SPHERE 1
#define ORC_ORD_UNIFORM2D 2
#define ORC_ORD_GAUSS2D 3

typedef struct {
    int32_t nx, ny;
    double x0, x1, y0, y1;
} orc_grid;

/* Inflow data, eq. (1.2) and its X-Y form in Appendix A.  Isotropic arrays hold one value per
 * boundary cell (left/right: [ny], bottom/top: [nx]); angular arrays hold one value per
 * (ordinate, boundary cell), ordinate-major ([n][ny] or [n][nx]) and take precedence.
 * NULL means vacuum for that face. */
typedef struct {
    const double *left, *right, *bottom, *top;
    const double *aleft, *aright, *abottom, *atop;
} orc_inflow;

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------------------------ */
/* SplitMix64, from its published definition (Steele, Lea, Flood 2014): the state advances by  */
/* the golden gamma and each output is the state passed through the 64-bit finalizer.          */
/* ------------------------------------------------------------------------------------------ */
#define SM64_GAMMA 0x9e3779b97f4a7c15ULL

static uint64_t sm64_finalize(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix64_next(uint64_t *state)
{
    *state += SM64_GAMMA;
    return sm64_finalize(*state);
}

double orc_u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

/* Seed of the stream for sample s: the (s+1)-th output of a SplitMix64 generator seeded with
 * the master seed.  Output k of such a generator is finalize(seed + k * gamma), so any sample's
 * stream is reachable directly. */
uint64_t orc_sample_seed(uint64_t seed, int64_t sample)
{
    return sm64_finalize(seed + (uint64_t)(sample + 1) * SM64_GAMMA);
}

/* ------------------------------------------------------------------------------------------ */
/* Ordinate sets.  dirs is [n][3] = (c, s, zeta) with (c, s) = sqrt(1 - zeta^2)(cos, sin)theta,  */
/* the projection of a unit-sphere direction onto the x-y plane (Appendix A).                 */
/* ------------------------------------------------------------------------------------------ */

/* Largest divisor of m that does not exceed sqrt(m): the number of zeta bands used when the
 * per-quadrant ordinate count is not a perfect square (the paper only uses N x N, Sec. 4.2). */
int orc_zeta_bands(int m)
{
    int best = 1;
    for (int d = 1; (long)d * d <= m; ++d)
        if (m % d == 0) best = d;
    return best;
}

static void put_dir(double *dirs, int l, double c, double s, double z)
{
    dirs[3 * l + 0] = c;
    dirs[3 * l + 1] = s;
    dirs[3 * l + 2] = z;
}

/* ROM ordinates in X-Y geometry (Sec. 3.1 steps 1-2; Sec. 4.2): the first-quadrant (zeta,
 * theta) rectangle [0,1] x [0,pi/2] is cut into nz x nt equal cells, zeta bands counted from
 * the pole (zeta_i = (N-i+1)/N) and theta bands from theta = 0; one point is drawn uniformly in
 * every cell, independently, with index l = i*nt + j.  The other quadrants are the mirror images
 * of eq. (3.5): l+m -> (-c, s), l+2m -> (-c, -s), l+3m -> (c, -s), same zeta.  Weights are the
 * cell areas over the total, 1/n (eq. (3.4)). */
int orc_ordinates_stratified(int nz, int nt, uint64_t seed, int64_t sample, double *dirs, double *w)
{
    if (nz <= 0 || nt <= 0 || !dirs || !w) return ORC_EARG;
    const int m = nz * nt, n = 4 * m;
    uint64_t st = orc_sample_seed(seed, sample);
    for (int i = 0; i < nz; ++i) {
        for (int j = 0; j < nt; ++j) {
            double uz = orc_u01(orc_splitmix64_next(&st));
            double ut = orc_u01(orc_splitmix64_next(&st));
            double zeta = 1.0 - ((double)i + uz) / (double)nz;
            double theta = ((double)j + ut) * (0.5 * M_PI) / (double)nt;
            double rho = sqrt((1.0 - zeta) * (1.0 + zeta));
            double c = rho * cos(theta);
            double s = rho * sin(theta);
            int l = i * nt + j;
            put_dir(dirs, l, c, s, zeta);
            put_dir(dirs, l + m, -c, s, zeta);
            put_dir(dirs, l + 2 * m, -c, -s, zeta);
            put_dir(dirs, l + 3 * m, c, -s, zeta);
        }
    }
    for (int l = 0; l < n; ++l) w[l] = 1.0 / (double)n;
    return ORC_OK;
}

/* n directions drawn independently and uniformly on the whole unit sphere (zeta = 2u-1,
 * theta = 2 pi u'), projected to the x-y plane, equal weights 1/n.  Not stratified and not
 * mirror-symmetric: the plain Monte-Carlo quadrature. */
int orc_ordinates_iid_sphere(int n, uint64_t seed, int64_t sample, double *dirs, double *w)
{
    if (n <= 0 || !dirs || !w) return ORC_EARG;
    uint64_t st = orc_sample_seed(seed, sample);
    for (int l = 0; l < n; ++l) {
        double uz = orc_u01(orc_splitmix64_next(&st));
        double ut = orc_u01(orc_splitmix64_next(&st));
        double zeta = 2.0 * uz - 1.0;
        double theta = ut * (2.0 * M_PI);
        double rho = sqrt((1.0 - zeta) * (1.0 + zeta));
        put_dir(dirs, l, rho * cos(theta), rho * sin(theta), zeta);
        w[l] = 1.0 / (double)n;
    }
    return ORC_OK;
}

/* Legendre polynomial P_n and its derivative at x by the three-term recurrence. */
static void legendre(int n, double x, double *p, double *dp)
{
    double p0 = 1.0, p1 = x;
    if (n == 0) {
        *p = 1.0;
        *dp = 0.0;
        return;
    }
    for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / (double)k;
        p0 = p1;
        p1 = pk;
    }
    *p = p1;
    *dp = (double)n * (x * p1 - p0) / ((x - 1.0) * (x + 1.0));
}

/* Gauss-Legendre nodes (descending) and weights 2/((1-x^2) P_n'(x)^2) on [-1,1] (Appendix A),
 * nodes found by Newton's method from the usual cosine guess. */
int orc_gauss_legendre(int n, double *x, double *w)
{
    if (n <= 0 || !x || !w) return ORC_EARG;
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        double p, dp;
        for (int it = 0; it < 100; ++it) {
            legendre(n, z, &p, &dp);
            double dz = p / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        legendre(n, z, &p, &dp);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z) * (1.0 + z) * dp * dp);
    }
    return ORC_OK;
}

/* "2D uniform quadrature" of Appendix A, eq. (A.5): N x N first-quadrant nodes
 * zeta_i = (2N-2i+1)/(2N), theta_j = (2j-1) pi/(4N), l = (i-1)N + j, weight 1/(4N^2), other
 * quadrants by the mirror symmetry.  4N^2 ordinates. */
int orc_quadrature_uniform2d(int N, double *dirs, double *w)
{
    if (N <= 0 || !dirs || !w) return ORC_EARG;
    const int m = N * N, n = 4 * m;
    for (int i = 1; i <= N; ++i) {
        for (int j = 1; j <= N; ++j) {
            double zeta = (double)(2 * N - 2 * i + 1) / (double)(2 * N);
            double theta = (double)(2 * j - 1) * M_PI / (double)(4 * N);
            double rho = sqrt((1.0 - zeta) * (1.0 + zeta));
            double c = rho * cos(theta), s = rho * sin(theta);
            int l = (i - 1) * N + (j - 1);
            put_dir(dirs, l, c, s, zeta);
            put_dir(dirs, l + m, -c, s, zeta);
            put_dir(dirs, l + 2 * m, -c, -s, zeta);
            put_dir(dirs, l + 3 * m, c, -s, zeta);
        }
    }
    for (int l = 0; l < n; ++l) w[l] = 1.0 / (double)n;
    return ORC_OK;
}

/* "2D Gaussian quadrature" of Appendix A: zeta_1 > ... > zeta_N are the positive roots of
 * L_{2N}; level i carries i azimuths theta_{i,j} = (2j-1) pi/(4i), j = 1..i, each with weight
 * 1/(2 i (1-zeta_i^2) L'_{2N}(zeta_i)^2); l = i(i-1)/2 + j.  Other quadrants by mirror
 * symmetry.  2N(N+1) ordinates. */
int orc_quadrature_gauss2d(int N, double *dirs, double *w)
{
    if (N <= 0 || !dirs || !w) return ORC_EARG;
    const int m = N * (N + 1) / 2;
    double *x = (double *)malloc(sizeof(double) * 2 * N);
    double *gw = (double *)malloc(sizeof(double) * 2 * N);
    if (!x || !gw) {
        free(x);
        free(gw);
        return ORC_ENOMEM;
    }
    orc_gauss_legendre(2 * N, x, gw); /* descending: x[0..N-1] are the positive roots */
    for (int i = 1; i <= N; ++i) {
        double zeta = x[i - 1];
        double p, dp;
        legendre(2 * N, zeta, &p, &dp);
        double wi = 1.0 / (2.0 * i * ((1.0 - zeta) * (1.0 + zeta)) * dp * dp);
        double rho = sqrt((1.0 - zeta) * (1.0 + zeta));
        for (int j = 1; j <= i; ++j) {
            double theta = (double)(2 * j - 1) * M_PI / (double)(4 * i);
            double c = rho * cos(theta), s = rho * sin(theta);
            int l = i * (i - 1) / 2 + (j - 1);
            put_dir(dirs, l, c, s, zeta);
            put_dir(dirs, l + m, -c, s, zeta);
            put_dir(dirs, l + 2 * m, -c, -s, zeta);
            put_dir(dirs, l + 3 * m, c, -s, zeta);
            w[l] = w[l + m] = w[l + 2 * m] = w[l + 3 * m] = wi;
        }
    }
    free(x);
    free(gw);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Scattering: W[l'][l] = w_l' * P(u_l', u_l), eq. (3.4), self term included; optionally with */
/* each row of P renormalized (the remark of Sec. 3.1).                                        */
/* ------------------------------------------------------------------------------------------ */

/* Phase functions of the cosine mu between two 3-D directions.  LINEAR is the kernel
 * 1 + g cos(xi) of eq. (2.1); HG is Henyey-Greenstein (1-g^2)/(1+g^2-2 g mu)^{3/2}, whose
 * sphere average is 1 as eq. (1.1) requires of P. */
static double phase(int kind, double g, double mu)
{
    switch (kind) {
    case ORC_SCAT_ISO:
        return 1.0;
    case ORC_SCAT_LINEAR:
        return 1.0 + g * mu;
    case ORC_SCAT_HG: {
        double d = 1.0 + g * g - 2.0 * g * mu;
        return (1.0 - g * g) / (d * sqrt(d));
    }
    default:
        return 0.0;
    }
}

/* Build W.  With fold = 1, each stored ordinate (c, s, zeta) stands for the pair (c, s, +zeta)
 * and (c, s, -zeta): X-Y solutions are even in zeta, so the sphere integral of eq. (1.1) over
 * the mirrored lower hemisphere gives P_eff = (P(mu+) + P(mu-))/2 with mu+- = cc' + ss' +- zz'.
 * With fold = 0 the raw 3-D cosine cc' + ss' + zz' is used.  DENSE copies the caller's P. */
int orc_build_W(int n, const double *dirs, const double *w, int kind, double g, int fold,
                const double *P, double *W)
{
    const int normalize = (kind & ORC_SCAT_NORMALIZE) != 0;
    kind &= ~ORC_SCAT_NORMALIZE;
    if (n <= 0 || !dirs || !w || !W) return ORC_EARG;
    if (kind == ORC_SCAT_DENSE && !P) return ORC_EARG;
    double *row = (double *)malloc(sizeof(double) * n);
    if (!row) return ORC_ENOMEM;
    for (int lp = 0; lp < n; ++lp) {
        for (int l = 0; l < n; ++l) {
            if (kind == ORC_SCAT_DENSE) {
                row[l] = P[(size_t)lp * n + l];
            } else {
                double cc = dirs[3 * lp] * dirs[3 * l] + dirs[3 * lp + 1] * dirs[3 * l + 1];
                double zz = dirs[3 * lp + 2] * dirs[3 * l + 2];
                if (fold)
                    row[l] = 0.5 * (phase(kind, g, cc + zz) + phase(kind, g, cc - zz));
                else
                    row[l] = phase(kind, g, cc + zz);
            }
        }
        /* Normalized: the remark after eq. (3.5) asks that everything scattered out of the
         * incoming direction l' arrives somewhere, sum over outgoing l of w_l P_l'l = 1; the
         * row l' of P is divided by that sum r_l'. */
        double r = 1.0;
        if (normalize) {
            r = 0.0;
            for (int l = 0; l < n; ++l) r += w[l] * row[l];
            if (!(r > 0.0)) {
                free(row);
                return ORC_EARG;
            }
        }
        for (int l = 0; l < n; ++l) W[(size_t)lp * n + l] = w[lp] * (row[l] / r);
    }
    free(row);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Transport sweep: psi_l = L_l^{-1} S_l for every ordinate (the inversion of the streaming +   */
/* collision operator of Sec. 3.2), on the uniform cell-centred grid of Sec. 2.                 */
/* ------------------------------------------------------------------------------------------ */

static double inflow_x(const orc_inflow *in, int l, int ny, int j, int from_left)
{
    if (!in) return 0.0;
    if (from_left) {
        if (in->aleft) return in->aleft[(size_t)l * ny + j];
        return in->left ? in->left[j] : 0.0;
    }
    if (in->aright) return in->aright[(size_t)l * ny + j];
    return in->right ? in->right[j] : 0.0;
}

static double inflow_y(const orc_inflow *in, int l, int nx, int i, int from_bottom)
{
    if (!in) return 0.0;
    if (from_bottom) {
        if (in->abottom) return in->abottom[(size_t)l * nx + i];
        return in->bottom ? in->bottom[i] : 0.0;
    }
    if (in->atop) return in->atop[(size_t)l * nx + i];
    return in->top ? in->top[i] : 0.0;
}

/* One ordinate.  The characteristic direction (c, s) enters through the faces it points away
 * from: c >= 0 sweeps i upward from the left face, c < 0 downward from the right face, and the
 * same for s and j (inflow faces as in the X-Y boundary conditions of Appendix A).
 *
 * STEP (first-order upwind): the upwind face value is the upstream cell's value, so the cell
 * balance  c (psi - psi_in_x)/dx + s (psi - psi_in_y)/dy + sigma_t psi = S  gives
 *     psi = (S + a psi_in_x + b psi_in_y) / (sigma_t + a + b),  a = |c|/dx, b = |s|/dy.
 * DD (diamond difference, Sec. 2): the centre value is the mean of the in/out face values,
 *     psi = (S + 2a psi_in_x + 2b psi_in_y) / (sigma_t + 2a + 2b),  psi_out = 2 psi - psi_in. */
static void sweep_one(const orc_grid *g, const double *sigma_t, int l, const double *dir,
                      const double *S, const orc_inflow *in, int scheme, double *psi)
{
    const int nx = g->nx, ny = g->ny;
    const double dx = (g->x1 - g->x0) / nx, dy = (g->y1 - g->y0) / ny;
    const double c = dir[0], s = dir[1];
    const double a = fabs(c) / dx, b = fabs(s) / dy;
    const int xpos = (c >= 0.0), ypos = (s >= 0.0);
    double *yface = (double *)malloc(sizeof(double) * nx); /* y-face values along the front */
    for (int ii = 0; ii < nx; ++ii) {
        int i = xpos ? ii : nx - 1 - ii;
        yface[i] = inflow_y(in, l, nx, i, ypos);
    }
    for (int jj = 0; jj < ny; ++jj) {
        int j = ypos ? jj : ny - 1 - jj;
        double xface = inflow_x(in, l, ny, j, xpos);
        for (int ii = 0; ii < nx; ++ii) {
            int i = xpos ? ii : nx - 1 - ii;
            size_t cell = (size_t)j * nx + i;
            double v;
            if (scheme == ORC_SCHEME_DD) {
                v = (S[cell] + 2.0 * a * xface + 2.0 * b * yface[i]) / (sigma_t[cell] + 2.0 * a + 2.0 * b);
                xface = 2.0 * v - xface;
                yface[i] = 2.0 * v - yface[i];
            } else {
                v = (S[cell] + a * xface + b * yface[i]) / (sigma_t[cell] + a + b);
                xface = v;
                yface[i] = v;
            }
            psi[cell] = v;
        }
    }
    free(yface);
}

/* All ordinates.  src is either one source per cell shared by every ordinate (src_per_ordinate
 * = 0) or one per (ordinate, cell) ([n][cells]).  psi is [n][cells]. */
int orc_sweep(const orc_grid *g, const double *sigma_t, int n, const double *dirs, const double *src,
              int src_per_ordinate, const orc_inflow *in, int scheme, double *psi)
{
    if (!g || g->nx <= 0 || g->ny <= 0 || !sigma_t || n <= 0 || !dirs || !src || !psi) return ORC_EARG;
    const size_t cells = (size_t)g->nx * g->ny;
#pragma omp parallel for schedule(dynamic, 1)
    for (int l = 0; l < n; ++l) {
        const double *S = src_per_ordinate ? src + (size_t)l * cells : src;
        sweep_one(g, sigma_t, l, dirs + 3 * l, S, in, scheme, psi + (size_t)l * cells);
    }
    return ORC_OK;
}

/* Scalar flux phi = sum_l w_l psi_l (the average density of Sec. 2), summed in index order. */
void orc_scalar_flux(size_t cells, int n, const double *w, const double *psi, double *phi)
{
    for (size_t k = 0; k < cells; ++k) phi[k] = 0.0;
    for (int l = 0; l < n; ++l)
        for (size_t k = 0; k < cells; ++k) phi[k] += w[l] * psi[(size_t)l * cells + k];
}

/* ------------------------------------------------------------------------------------------ */
/* Source iteration (the classical iteration whose iterates are the partial sums of the Neumann */
/* series eq. (3.10)):  psi^k = L^{-1}( sigma_s sum_l' W[l'][l] psi^{k-1}_l' + q ),  psi^0 = 0.  */
/* For isotropic scattering the source reduces to sigma_s phi^{k-1} + q.                        */
/* ------------------------------------------------------------------------------------------ */

/* Relative change max|phi - phi_old| / max|phi| (0 when phi is identically zero). */
static double rel_change(size_t cells, const double *phi, const double *old)
{
    double dmax = 0.0, pmax = 0.0;
    for (size_t k = 0; k < cells; ++k) {
        double d = fabs(phi[k] - old[k]);
        if (d > dmax) dmax = d;
        if (fabs(phi[k]) > pmax) pmax = fabs(phi[k]);
    }
    return pmax > 0.0 ? dmax / pmax : 0.0;
}

int orc_source_iterate(const orc_grid *g, const double *sigma_t, const double *sigma_s, const double *q,
                       const orc_inflow *in, int n, const double *dirs, const double *w, const double *W,
                       int scheme, double tol, int max_iter, double *phi, double *psi_out, int *iters,
                       double *final_r, double *r_hist)
{
    if (!g || g->nx <= 0 || g->ny <= 0 || !sigma_t || !sigma_s || !q || n <= 0 || !dirs || !w || !phi ||
        max_iter <= 0)
        return ORC_EARG;
    const size_t cells = (size_t)g->nx * g->ny;
    double *psi = (double *)calloc((size_t)n * cells, sizeof(double));
    double *old = (double *)calloc(cells, sizeof(double));
    double *src = (double *)calloc(W ? (size_t)n * cells : cells, sizeof(double));
    if (!psi || !old || !src) {
        free(psi);
        free(old);
        free(src);
        return ORC_ENOMEM;
    }
    for (size_t k = 0; k < cells; ++k) phi[k] = 0.0;
    int status = ORC_NOT_CONVERGED, k;
    double r = 0.0;
    for (k = 1; k <= max_iter; ++k) {
        /* scattering source from the previous iterate, eq. (3.1) right-hand side */
        if (W) {
#pragma omp parallel for schedule(static)
            for (size_t cell = 0; cell < cells; ++cell) {
                for (int l = 0; l < n; ++l) {
                    double acc = 0.0;
                    for (int lp = 0; lp < n; ++lp) acc += W[(size_t)lp * n + l] * psi[(size_t)lp * cells + cell];
                    src[(size_t)l * cells + cell] = sigma_s[cell] * acc + q[cell];
                }
            }
        } else {
            for (size_t cell = 0; cell < cells; ++cell) src[cell] = sigma_s[cell] * phi[cell] + q[cell];
        }
        memcpy(old, phi, sizeof(double) * cells);
        orc_sweep(g, sigma_t, n, dirs, src, W != NULL, in, scheme, psi);
        orc_scalar_flux(cells, n, w, psi, phi);
        r = rel_change(cells, phi, old);
        if (r_hist) r_hist[k - 1] = r;
        if (r <= tol) {
            status = ORC_OK;
            break;
        }
    }
    if (iters) *iters = (k <= max_iter) ? k : max_iter;
    if (final_r) *final_r = r;
    if (psi_out) memcpy(psi_out, psi, sizeof(double) * (size_t)n * cells);
    free(psi);
    free(old);
    free(src);
    return status;
}

/* Ordinate set of one sample for the generator kinds (deterministic kinds ignore seed/sample). */
int orc_ordinate_count(int kind, int p1, int p2)
{
    switch (kind) {
    case ORC_ORD_STRATIFIED: return 4 * p1 * p2;
    case ORC_ORD_IID_SPHERE: return p1;
    case ORC_ORD_UNIFORM2D: return 4 * p1 * p1;
    case ORC_ORD_GAUSS2D: return 2 * p1 * (p1 + 1);
    default: return -1;
    }
}

int orc_generate(int kind, int p1, int p2, uint64_t seed, int64_t sample, double *dirs, double *w)
{
    switch (kind) {
    case ORC_ORD_STRATIFIED: return orc_ordinates_stratified(p1, p2, seed, sample, dirs, w);
    case ORC_ORD_IID_SPHERE: return orc_ordinates_iid_sphere(p1, seed, sample, dirs, w);
    case ORC_ORD_UNIFORM2D: return orc_quadrature_uniform2d(p1, dirs, w);
    case ORC_ORD_GAUSS2D: return orc_quadrature_gauss2d(p1, dirs, w);
    default: return ORC_EARG;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Ensemble (Sec. 4.1, eq. (4.6)): t independent ordinate samples s = 0..t-1, each solved to    */
/* convergence; mean = (1/t) sum_s phi_s and the unbiased variance sum_s (phi_s - mean)^2/(t-1),   */
/* both by two plain passes over the stored per-sample solutions.                               */
/* ------------------------------------------------------------------------------------------ */
int orc_ensemble(const orc_grid *g, const double *sigma_t, const double *sigma_s, const double *q,
                 const orc_inflow *in, int ord_kind, int p1, int p2, uint64_t seed, int t, int scat_kind,
                 double gpar, int fold, int scheme, double tol, int max_iter, double *mean, double *var,
                 double *phis, int *iters)
{
    if (!g || t <= 0 || !mean) return ORC_EARG;
    const int n = orc_ordinate_count(ord_kind, p1, p2);
    if (n <= 0) return ORC_EARG;
    const size_t cells = (size_t)g->nx * g->ny;
    double *dirs = (double *)malloc(sizeof(double) * 3 * n);
    double *w = (double *)malloc(sizeof(double) * n);
    double *W = (scat_kind & ~ORC_SCAT_NORMALIZE) == ORC_SCAT_ISO ? NULL : (double *)malloc(sizeof(double) * (size_t)n * n);
    double *all = phis ? phis : (double *)malloc(sizeof(double) * cells * (size_t)t);
    if (!dirs || !w || !all || ((scat_kind & ~ORC_SCAT_NORMALIZE) != ORC_SCAT_ISO && !W)) {
        free(dirs);
        free(w);
        free(W);
        if (!phis) free(all);
        return ORC_ENOMEM;
    }
    int status = ORC_OK;
    for (int s = 0; s < t; ++s) {
        orc_generate(ord_kind, p1, p2, seed, s, dirs, w);
        if (W) orc_build_W(n, dirs, w, scat_kind, gpar, fold, NULL, W);
        int it = 0;
        int st = orc_source_iterate(g, sigma_t, sigma_s, q, in, n, dirs, w, W, scheme, tol, max_iter,
                                    all + (size_t)s * cells, NULL, &it, NULL, NULL);
        if (st < 0) {
            status = st;
            break;
        }
        if (st == ORC_NOT_CONVERGED) status = ORC_NOT_CONVERGED;
        if (iters) iters[s] = it;
    }
    if (status >= 0) {
        for (size_t k = 0; k < cells; ++k) {
            double acc = 0.0;
            for (int s = 0; s < t; ++s) acc += all[(size_t)s * cells + k];
            mean[k] = acc / (double)t;
        }
        if (var) {
            for (size_t k = 0; k < cells; ++k) {
                double acc = 0.0;
                for (int s = 0; s < t; ++s) {
                    double d = all[(size_t)s * cells + k] - mean[k];
                    acc += d * d;
                }
                var[k] = t > 1 ? acc / (double)(t - 1) : 0.0;
            }
        }
    }
    free(dirs);
    free(w);
    free(W);
    if (!phis) free(all);
    return status;
}

/* ------------------------------------------------------------------------------------------ */
/* Slab geometry (Sec. 4.1, Example 4.1): mu psi_x + sigma_t psi = sigma_s phi + q on [x0, x1], */
/* phi = (1/2) int psi dmu, isotropic scattering P = 1.                                         */
/*                                                                                            */
/* Readings (the paper's second-order scheme [ShiA] is not given in its text): unknowns at the */
/* grid points x_i = x0 + i dx, i = 0..nx, as the paper's slab error norm uses; diamond        */
/* difference on each cell [x_i, x_{i+1}] with the cell's sigma_t the mean of its end values    */
/* and the cell source the mean of its end sources,                                            */
/*   |mu| (psi_out - psi_in) / dx + sigma_c (psi_in + psi_out) / 2 = (S_i + S_{i+1}) / 2;       */
/* weights normalized to sum 1 (the paper's 2/n together with the 1/2 of the slab average), so */
/* phi = sum_l w_l psi_l.                                                                      */
/* ------------------------------------------------------------------------------------------ */

/* ROM slab ordinates: [-1, 1] cut into n equal cells (n even); one uniform draw in each cell of
 * [-1, 0], the cells of [0, 1] get the mirror images mu_l = -mu_{n+1-l}; weights 1/n.  The
 * draws use sample `sample`'s SplitMix64 stream, cells in increasing order. */
int orc_slab_ordinates_rom(int n, uint64_t seed, int64_t sample, double *mu, double *w)
{
    if (n <= 0 || (n & 1) || !mu || !w) return ORC_EARG;
    uint64_t st = orc_sample_seed(seed, sample);
    const int m = n / 2;
    const double width = 2.0 / (double)n;
    for (int l = 0; l < m; ++l) {
        const double u = orc_u01(orc_splitmix64_next(&st));
        mu[l] = -1.0 + (double)l * width + u * width;  /* cell l of [-1, 0], counted from -1 */
    }
    for (int l = m; l < n; ++l) mu[l] = -mu[n - 1 - l];
    for (int l = 0; l < n; ++l) w[l] = 1.0 / (double)n;
    return ORC_OK;
}

/* DOM slab quadratures: kind 0 Gauss-Legendre on [-1, 1] (weights halved), kind 1 the uniform
 * midpoint rule of n equal cells. */
int orc_slab_quadrature(int kind, int n, double *mu, double *w)
{
    if (n <= 0 || !mu || !w) return ORC_EARG;
    if (kind == 0) {
        int rc = orc_gauss_legendre(n, mu, w);
        if (rc) return rc;
        for (int l = 0; l < n; ++l) w[l] *= 0.5;
        return ORC_OK;
    }
    if (kind == 1) {
        for (int l = 0; l < n; ++l) {
            mu[l] = -1.0 + (2.0 * l + 1.0) / (double)n;
            w[l] = 1.0 / (double)n;
        }
        return ORC_OK;
    }
    return ORC_EARG;
}

/* One slab sweep of every ordinate for the node source S [nx+1]: psi [n][nx+1].  inflow[l] is
 * psi at the entry boundary of ordinate l (x0 when mu_l > 0, x1 when mu_l < 0). */
int orc_slab_sweep(int nx, double x0, double x1, const double *sigma_t, int n, const double *mu,
                   const double *inflow, const double *S, double *psi)
{
    if (nx <= 0 || !(x1 > x0) || !sigma_t || n <= 0 || !mu || !inflow || !S || !psi) return ORC_EARG;
    const double dx = (x1 - x0) / (double)nx;
    for (int l = 0; l < n; ++l) {
        if (mu[l] == 0.0) return ORC_EARG;
        const double a = fabs(mu[l]) / dx;
        double *p = psi + (size_t)l * (nx + 1);
        if (mu[l] > 0.0) {
            p[0] = inflow[l];
            for (int i = 0; i < nx; ++i) {
                const double sc = 0.5 * (sigma_t[i] + sigma_t[i + 1]);
                const double sbar = 0.5 * (S[i] + S[i + 1]);
                p[i + 1] = ((a - 0.5 * sc) * p[i] + sbar) / (a + 0.5 * sc);
            }
        } else {
            p[nx] = inflow[l];
            for (int i = nx - 1; i >= 0; --i) {
                const double sc = 0.5 * (sigma_t[i] + sigma_t[i + 1]);
                const double sbar = 0.5 * (S[i] + S[i + 1]);
                p[i] = ((a - 0.5 * sc) * p[i + 1] + sbar) / (a + 0.5 * sc);
            }
        }
    }
    return ORC_OK;
}

/* Slab source iteration from phi^0 = 0 with the same stopping rule as the X-Y case. */
int orc_slab_source_iterate(int nx, double x0, double x1, const double *sigma_t, const double *sigma_s,
                            const double *q, int n, const double *mu, const double *w, const double *inflow,
                            double tol, int max_iter, double *phi, int *iters, double *final_r)
{
    if (nx <= 0 || !sigma_s || !q || !w || !phi || max_iter <= 0) return ORC_EARG;
    const size_t nn = (size_t)nx + 1;
    double *psi = (double *)malloc(sizeof(double) * (size_t)n * nn);
    double *S = (double *)malloc(sizeof(double) * nn);
    double *old = (double *)malloc(sizeof(double) * nn);
    if (!psi || !S || !old) {
        free(psi);
        free(S);
        free(old);
        return ORC_ENOMEM;
    }
    for (size_t i = 0; i < nn; ++i) phi[i] = 0.0;
    int status = ORC_NOT_CONVERGED, k;
    double r = 0.0;
    for (k = 1; k <= max_iter; ++k) {
        for (size_t i = 0; i < nn; ++i) S[i] = sigma_s[i] * phi[i] + q[i];
        memcpy(old, phi, sizeof(double) * nn);
        int rc = orc_slab_sweep(nx, x0, x1, sigma_t, n, mu, inflow, S, psi);
        if (rc) {
            status = rc;
            break;
        }
        for (size_t i = 0; i < nn; ++i) {
            double acc = 0.0;
            for (int l = 0; l < n; ++l) acc += w[l] * psi[(size_t)l * nn + i];
            phi[i] = acc;
        }
        r = rel_change(nn, phi, old);
        if (r <= tol) {
            status = ORC_OK;
            break;
        }
    }
    if (iters) *iters = (k <= max_iter) ? k : max_iter;
    if (final_r) *final_r = r;
    free(psi);
    free(S);
    free(old);
    return status;
}
