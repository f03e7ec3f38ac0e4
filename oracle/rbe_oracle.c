/*
 * Plain FP64 CPU oracle for the random batch Ewald (RBE) k-space path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code with the HIP path.
 *
 * Every function is the textbook definition written out, in FP64, with the
 * sums taken in index order and Neumaier-compensated.  No blocking, fusion or
 * reordering beyond what the definitions state.  Loops over independent
 * outputs (one wave vector, one particle) may run on several OpenMP threads;
 * each output is still computed by one thread in a fixed order, so the
 * results do not depend on the thread count.
 *
 * Conventions (paper, Sec. 2.2, Gaussian units, prefactor 1):
 *   wave vector     k_l = 2 pi m_l / L,  m_l integer triple, V = L^3
 *   structure factor  rho(k) = sum_i q_i exp(i k . r_i)              (Sec. 2.2, definition of rho)
 *   per-k weight    w_l: Q/P for the RBE estimator (Eq. frbe),
 *                   exp(-k^2/4 alpha) for the full Ewald sum (Eq. long)
 *   c_l = w_l 4 pi / (V k_l^2)
 *   force           F_i = -sum_l c_l q_i k_l Im(exp(-i k_l . r_i) rho(k_l))   (Eq. frbe / Eq. long)
 *   energy          U   = sum_l (c_l / 2) |rho(k_l)|^2   (long-range energy term of the
 *                   split Ewald energy, Sec. 2.2, with the same importance weights)
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double s, c; } nsum;   /* Neumaier running sum */

static void nsum_add(nsum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else                       a->c += (v - t) + a->s;
    a->s = t;
}
static double nsum_get(const nsum *a) { return a->s + a->c; }

static const double PI = 3.14159265358979323846264338327950288;
static const double TWO_PI = 6.283185307179586476925286766559;
static const double FOUR_PI = 12.566370614359172953850573533118;

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of later OpenMP loops (for timing on a stated number of cores; the
   results do not depend on it). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* k_l = 2 pi m_l / L */
static void wave_vector(const int32_t *m, int64_t l, double L, double k[3]) {
    for (int d = 0; d < 3; ++d) k[d] = TWO_PI * (double)m[3 * l + d] / L;
}

/* rho(k_l) = sum_i q_i exp(i k_l . r_i); out rho[2l] = Re, rho[2l+1] = Im. */
void oracle_rho(int64_t n, const double *x, const double *y, const double *z, const double *q,
                int64_t p, const int32_t *m, double L, double *rho)
{
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < p; ++l) {
        double k[3];
        wave_vector(m, l, L, k);
        nsum re = {0, 0}, im = {0, 0};
        for (int64_t i = 0; i < n; ++i) {
            double th = k[0] * x[i] + k[1] * y[i] + k[2] * z[i];
            nsum_add(&re, q[i] * cos(th));
            nsum_add(&im, q[i] * sin(th));
        }
        rho[2 * l] = nsum_get(&re);
        rho[2 * l + 1] = nsum_get(&im);
    }
}

/* c_l = w_l 4 pi / (V k_l^2); zero for the (excluded) k = 0 term. */
static double coef(const int32_t *m, int64_t l, const double *w, double L) {
    double k[3];
    wave_vector(m, l, L, k);
    double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    if (k2 == 0.0) return 0.0;
    double V = L * L * L;
    return w[l] * FOUR_PI / (V * k2);
}

/*
 * Forces (SoA: F[0..n) x, F[n..2n) y, F[2n..3n) z) and energy U from a given rho.
 *   F_i = -q_i sum_l c_l k_l Im(exp(-i theta_il) rho_l),
 *   Im(exp(-i theta) (C + i S)) = cos(theta) S - sin(theta) C.
 */
void oracle_force_from_rho(int64_t n, const double *x, const double *y, const double *z,
                           const double *q, int64_t p, const int32_t *m, const double *w,
                           double L, const double *rho, double *F, double *U)
{
    nsum u = {0, 0};
    for (int64_t l = 0; l < p; ++l) {
        double c = coef(m, l, w, L);
        nsum_add(&u, 0.5 * c * (rho[2 * l] * rho[2 * l] + rho[2 * l + 1] * rho[2 * l + 1]));
    }
    *U = nsum_get(&u);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        nsum f[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t l = 0; l < p; ++l) {
            double k[3];
            wave_vector(m, l, L, k);
            double c = coef(m, l, w, L);
            double th = k[0] * x[i] + k[1] * y[i] + k[2] * z[i];
            double im = cos(th) * rho[2 * l + 1] - sin(th) * rho[2 * l];
            for (int d = 0; d < 3; ++d) nsum_add(&f[d], c * k[d] * im);
        }
        for (int d = 0; d < 3; ++d) F[(int64_t)d * n + i] = -q[i] * nsum_get(&f[d]);
    }
}

/* Full evaluation: rho, F and U for one system. rho may be NULL. */
void oracle_force_energy(int64_t n, const double *x, const double *y, const double *z,
                         const double *q, int64_t p, const int32_t *m, const double *w,
                         double L, double *rho_out, double *F, double *U)
{
    double stack_rho[2 * 256];
    double *rho = rho_out;
    if (rho == NULL) {
        if (p > 256) return;   /* callers pass a buffer for large p */
        rho = stack_rho;
    }
    oracle_rho(n, x, y, z, q, p, m, L, rho);
    oracle_force_from_rho(n, x, y, z, q, p, m, w, L, rho, F, U);
}

/*
 * Forces for a subset of particles only (sampled checks at large n): F_sel is
 * SoA over the nsel selected indices; rho must be the full structure factor.
 */
void oracle_force_subset(int64_t n, const double *x, const double *y, const double *z,
                         const double *q, int64_t p, const int32_t *m, const double *w,
                         double L, const double *rho, int64_t nsel, const int64_t *sel,
                         double *F_sel)
{
    (void)n;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < nsel; ++s) {
        int64_t i = sel[s];
        nsum f[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t l = 0; l < p; ++l) {
            double k[3];
            wave_vector(m, l, L, k);
            double c = coef(m, l, w, L);
            double th = k[0] * x[i] + k[1] * y[i] + k[2] * z[i];
            double im = cos(th) * rho[2 * l + 1] - sin(th) * rho[2 * l];
            for (int d = 0; d < 3; ++d) nsum_add(&f[d], c * k[d] * im);
        }
        for (int d = 0; d < 3; ++d) F_sel[(int64_t)d * nsel + s] = -q[i] * nsum_get(&f[d]);
    }
}

/*
 * Vector-Jacobian product of (U, F) with respect to positions and charges.
 *
 * Upstream gradients: gU (scalar) on U and GF (SoA, 3n) on F.  With
 * a_l = c_l / 2, g_il = GF_i . k_l, C + iS = rho, the linearised loss is
 *   Lin = sum_l a_l [ gU (C_l^2 + S_l^2) - 2 (X_l S_l - Y_l C_l) ],
 *   X_l = sum_i q_i g_il cos(theta_il),  Y_l = sum_i q_i g_il sin(theta_il).
 * Differentiating through theta_il = k_l . r_i and q_i:
 *   Chat_l = 2 a_l (gU C_l + Y_l),  Shat_l = 2 a_l (gU S_l - X_l)
 *   dL/dr_i = q_i sum_l k_l [Shat_l cos - Chat_l sin + 2 a_l g_il (C_l cos + S_l sin)]
 *   dL/dq_i = sum_l [Chat_l cos + Shat_l sin - 2 a_l g_il (S_l cos - C_l sin)]
 * (derived from the energy and force definitions above; the paper has no adjoint).
 */
void oracle_vjp(int64_t n, const double *x, const double *y, const double *z, const double *q,
                int64_t p, const int32_t *m, const double *w, double L, double gU,
                const double *GF, double *gr, double *gq, double *work /* 6p doubles */)
{
    double *rho = work, *XY = work + 2 * p, *hat = work + 4 * p;
    oracle_rho(n, x, y, z, q, p, m, L, rho);
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < p; ++l) {
        double k[3];
        wave_vector(m, l, L, k);
        nsum X = {0, 0}, Y = {0, 0};
        for (int64_t i = 0; i < n; ++i) {
            double th = k[0] * x[i] + k[1] * y[i] + k[2] * z[i];
            double g = GF[i] * k[0] + GF[n + i] * k[1] + GF[2 * n + i] * k[2];
            nsum_add(&X, q[i] * g * cos(th));
            nsum_add(&Y, q[i] * g * sin(th));
        }
        XY[2 * l] = nsum_get(&X);
        XY[2 * l + 1] = nsum_get(&Y);
    }
    for (int64_t l = 0; l < p; ++l) {
        double a = 0.5 * coef(m, l, w, L);
        hat[2 * l] = 2.0 * a * (gU * rho[2 * l] + XY[2 * l + 1]);
        hat[2 * l + 1] = 2.0 * a * (gU * rho[2 * l + 1] - XY[2 * l]);
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        nsum r[3] = {{0, 0}, {0, 0}, {0, 0}}, qq = {0, 0};
        for (int64_t l = 0; l < p; ++l) {
            double k[3];
            wave_vector(m, l, L, k);
            double a = 0.5 * coef(m, l, w, L);
            double C = rho[2 * l], S = rho[2 * l + 1];
            double Ch = hat[2 * l], Sh = hat[2 * l + 1];
            double th = k[0] * x[i] + k[1] * y[i] + k[2] * z[i];
            double cs = cos(th), sn = sin(th);
            double g = GF[i] * k[0] + GF[n + i] * k[1] + GF[2 * n + i] * k[2];
            double sr = Sh * cs - Ch * sn + 2.0 * a * g * (C * cs + S * sn);
            for (int d = 0; d < 3; ++d) nsum_add(&r[d], k[d] * sr);
            nsum_add(&qq, Ch * cs + Sh * sn - 2.0 * a * g * (S * cs - C * sn));
        }
        for (int d = 0; d < 3; ++d) gr[(int64_t)d * n + i] = q[i] * nsum_get(&r[d]);
        gq[i] = nsum_get(&qq);
    }
}

/*
 * k-space virial tensor: the negative derivative of the long-range energy term with
 * respect to a symmetric affine strain of the box at fixed fractional coordinates
 * (the pressure of the NPT variant the paper cites in Sec. 2.2).  With
 * U_l = (c_l / 2) |rho_l|^2,
 *   W_ab = sum_l U_l (delta_ab - 2 k_la k_lb (1/k_l^2 + 1/(4 alpha))).
 * The 1/(4 alpha) part comes from the k-dependence of the Ewald kernel
 * exp(-k^2/4 alpha); with RBE weights w_l = S/P the same sum is the importance-
 * sampled estimate of the Ewald k-space virial.  W[6] = xx, yy, zz, xy, xz, yz.
 */
void oracle_virial(int64_t p, const int32_t *m, const double *w, double L, double alpha,
                   const double *rho, double *W)
{
    nsum acc[6] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
    static const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int64_t l = 0; l < p; ++l) {
        double k[3];
        wave_vector(m, l, L, k);
        double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        if (k2 == 0.0) continue;
        double u = 0.5 * coef(m, l, w, L) * (rho[2 * l] * rho[2 * l] + rho[2 * l + 1] * rho[2 * l + 1]);
        double g = 2.0 * (1.0 / k2 + 1.0 / (4.0 * alpha));
        for (int c = 0; c < 6; ++c) {
            double t = (ia[c] == ib[c] ? 1.0 : 0.0) - g * k[ia[c]] * k[ib[c]];
            nsum_add(&acc[c], u * t);
        }
    }
    for (int c = 0; c < 6; ++c) W[c] = nsum_get(&acc[c]);
}

/*
 * Real-space and self parts of the Ewald energy (Sec. 2.2, split energy):
 *   U_real = 1/2 sum_{i,j} sum'_{|n_d| <= nmax} q_i q_j erfc(sqrt(alpha) |r_ij + n L|) / |r_ij + n L|
 *   U_self = -sqrt(alpha / pi) sum_i q_i^2
 * (the prime drops n = 0 when i = j).  Used only for the Madelung check.
 */
void oracle_ewald_real_self(int64_t n, const double *x, const double *y, const double *z,
                            const double *q, double L, double alpha, int32_t nmax,
                            double *U_real, double *U_self)
{
    double sa = sqrt(alpha);
    nsum ur = {0, 0}, us = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            for (int a = -nmax; a <= nmax; ++a)
                for (int b = -nmax; b <= nmax; ++b)
                    for (int c = -nmax; c <= nmax; ++c) {
                        if (i == j && a == 0 && b == 0 && c == 0) continue;
                        double dx = x[i] - x[j] + a * L;
                        double dy = y[i] - y[j] + b * L;
                        double dz = z[i] - z[j] + c * L;
                        double r = sqrt(dx * dx + dy * dy + dz * dz);
                        nsum_add(&ur, 0.5 * q[i] * q[j] * erfc(sa * r) / r);
                    }
        }
        nsum_add(&us, q[i] * q[i]);
    }
    *U_real = nsum_get(&ur);
    *U_self = -sqrt(alpha / PI) * nsum_get(&us);
}
