/*
 * Plain FP64 CPU oracle for the random batch list (RBL) short-range force.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code with the HIP path.  Brute force over all
 * pairs with the minimum image (the outer cutoff is below L/2), FP64, no
 * neighbour lists.
 *
 * Definitions (paper, Sec. 2.1-2.3, Eqs. (lj), (fshort), (short), (fshell);
 * Algorithm 2), Gaussian units with prefactor 1:
 *   pair force on i from j, d = r_i - r_j (minimum image), r = |d|:
 *     LJ       24 eps_ij (2 (s/r)^12 - (s/r)^6) d / r^2,
 *              eps_ij = sqrt(eps_i eps_j), s = (sig_i + sig_j) / 2    (Lorentz-Berthelot)
 *     Coulomb  q_i q_j (erfc(sqrt(alpha) r) / r^2 + 2 sqrt(alpha / pi) exp(-alpha r^2) / r) d / r
 *   core  C(i) = {j != i : r < r_c},  shell S(i) = {j : r_c <= r <= r_s}
 *   F_i^core  = sum over C(i);  F_i^shell* = (N_s / p) sum over the batch B(i)
 *   F^corr    = -(1/N) sum_i (F_i^core + F_i^shell*);  F_i = F_i^core + F_i^shell* + F^corr
 *
 * Readings (the paper does not fix them):
 *   batch    systematic sampling in the traversal order of S(i): with the particle's
 *            uniform u_i, positions floor((b + u_i) N_s / p), b = 0..p-1, each weighted
 *            N_s / p (every shell particle is in the batch with probability p / N_s); if
 *            N_s <= p the batch is the whole shell with weight 1;
 *   order    cells of side h = L / nc, nc = floor(L / r_c); stencil reach R = ceil(r_s / h);
 *            per axis the offsets -R..R (all nc cells, offsets 0..nc-1, when 2R + 1 > nc),
 *            x outermost, z innermost; within a cell, ascending particle index;
 *   cells    cell_d = min(floor((x_d / L - floor(x_d / L)) nc), nc - 1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static const double RBL_PI = 3.14159265358979323846264338327950288;

typedef struct { double s, c; } rsum;   /* Neumaier running sum */

static void rsum_add(rsum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else                       a->c += (v - t) + a->s;
    a->s = t;
}

/* minimum-image difference of one coordinate, |d| <= L/2 */
static double min_image(double d, double L) { return d - L * rint(d / L); }

/* wrapped fractional coordinate in [0, 1) */
static double frac(double x, double L) {
    double s = x / L;
    return s - floor(s);
}

/* force on i from j given d = r_i - r_j and r2 = |d|^2 (the three components into f) */
static void pair_force(double qi, double qj, double ei, double ej, double si, double sj, double alpha,
                       const double d[3], double r2, double f[3]) {
    const double r = sqrt(r2);
    double g = 0.0;   /* F = g d */
    const double eps = sqrt(ei * ej);
    if (eps != 0.0) {
        const double s = 0.5 * (si + sj);
        const double s2 = s * s / r2;
        const double s6 = s2 * s2 * s2;
        g += 24.0 * eps * (2.0 * s6 * s6 - s6) / r2;
    }
    if (qi != 0.0 && qj != 0.0 && alpha >= 0.0) {
        const double sa = sqrt(alpha);
        const double kern = erfc(sa * r) / r2 + 2.0 * sqrt(alpha / RBL_PI) * exp(-alpha * r2) / r;
        g += qi * qj * kern / r;
    }
    for (int k = 0; k < 3; ++k) f[k] = g * d[k];
}

/* the cell grid of the traversal order */
typedef struct { int64_t nc; int64_t R; int64_t span; int wrap; } grid;

static grid make_grid(double L, double rc, double rs) {
    grid g;
    g.nc = (int64_t)floor(L / rc);
    if (g.nc < 1) g.nc = 1;
    const double h = L / (double)g.nc;
    g.R = (int64_t)ceil(rs / h);
    g.wrap = (2 * g.R + 1 > g.nc);
    g.span = g.wrap ? g.nc : 2 * g.R + 1;
    return g;
}

static int64_t cell_of(double x, double L, int64_t nc) {
    int64_t c = (int64_t)floor(frac(x, L) * (double)nc);
    return c < nc - 1 ? c : nc - 1;
}

/* position of cell cj along one axis in the stencil of ci */
static int64_t stencil_pos(int64_t ci, int64_t cj, const grid *g) {
    if (g->wrap) return ((cj - ci) % g->nc + g->nc) % g->nc;
    return ((cj - ci + g->R) % g->nc + g->nc) % g->nc;
}

typedef struct { int64_t key; int64_t j; } shell_entry;

static int cmp_entry(const void *a, const void *b) {
    const int64_t ka = ((const shell_entry *)a)->key, kb = ((const shell_entry *)b)->key;
    return (ka > kb) - (ka < kb);
}

/*
 * Raw RBL force of particle i, F_i^core + F_i^shell* (Eqs. short, fshell), by brute force
 * over all particles; sh: scratch for n entries.  Returns N_s.
 */
static int64_t rbl_raw_one(int64_t i, int64_t n, const double *x, const double *y, const double *z, const double *q,
                           const double *eps, const double *sig, double L, double alpha, double rc2, double rs2,
                           int32_t p, double u, const grid *g, shell_entry *sh, double out[3]) {
    const double pi_[3] = {x[i], y[i], z[i]};
    const int64_t ci[3] = {cell_of(x[i], L, g->nc), cell_of(y[i], L, g->nc), cell_of(z[i], L, g->nc)};
    rsum core[3] = {{0, 0}, {0, 0}, {0, 0}};
    int64_t ns = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        const double pj[3] = {x[j], y[j], z[j]};
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = min_image(pi_[k] - pj[k], L);
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (r2 < rc2) {
            double f[3];
            pair_force(q[i], q[j], eps[i], eps[j], sig[i], sig[j], alpha, d, r2, f);
            for (int k = 0; k < 3; ++k) rsum_add(&core[k], f[k]);
        } else if (r2 <= rs2) {
            const int64_t cj[3] = {cell_of(x[j], L, g->nc), cell_of(y[j], L, g->nc), cell_of(z[j], L, g->nc)};
            const int64_t s = (stencil_pos(ci[0], cj[0], g) * g->span + stencil_pos(ci[1], cj[1], g)) * g->span +
                              stencil_pos(ci[2], cj[2], g);
            sh[ns].key = s * n + j;
            sh[ns].j = j;
            ++ns;
        }
    }
    qsort(sh, (size_t)ns, sizeof(shell_entry), cmp_entry);
    rsum shell[3] = {{0, 0}, {0, 0}, {0, 0}};
    const double wgt = ns > p ? (double)ns / (double)p : 1.0;
    const int64_t nb = ns > p ? p : ns;
    for (int64_t b = 0; b < nb; ++b) {
        int64_t pos = ns > p ? (int64_t)floor(((double)b + u) * (double)ns / (double)p) : b;
        /* b + u < p, so the exact position is at most N_s - 1; the rounding of b + u can
           reach p, and the clamp restores the exact value there */
        if (pos > ns - 1) pos = ns - 1;
        const int64_t j = sh[pos].j;
        const double pj[3] = {x[j], y[j], z[j]};
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = min_image(pi_[k] - pj[k], L);
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double f[3];
        pair_force(q[i], q[j], eps[i], eps[j], sig[i], sig[j], alpha, d, r2, f);
        for (int k = 0; k < 3; ++k) rsum_add(&shell[k], f[k]);
    }
    for (int k = 0; k < 3; ++k) out[k] = (core[k].s + core[k].c) + wgt * (shell[k].s + shell[k].c);
    return ns;
}

static int valid(double L, double rc, double rs, int32_t p) { return rc > 0.0 && rc <= rs && rs < 0.5 * L && p >= 1; }

/*
 * RBL short-range force (Algorithm 2).  u: N uniforms in [0, 1) (the batch offsets).
 * F: 3N doubles, F[d N + i].  ns_out (may be NULL): N_s of every particle.
 * Returns 0, or -1 for invalid cutoffs (need 0 < r_c <= r_s < L/2, p >= 1).
 */
int oracle_rbl_short_force(int64_t n, const double *x, const double *y, const double *z, const double *q,
                           const double *eps, const double *sig, double L, double alpha, double rc, double rs,
                           int32_t p, const double *u, double *F, int64_t *ns_out) {
    if (!valid(L, rc, rs, p)) return -1;
    const grid g = make_grid(L, rc, rs);
    double *raw = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    int bad = (raw == NULL);
#pragma omp parallel
    {
        shell_entry *sh = (shell_entry *)malloc(sizeof(shell_entry) * (size_t)(n > 0 ? n : 1));
        if (sh == NULL) bad = 1;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            if (bad) continue;
            double f[3];
            const int64_t ns = rbl_raw_one(i, n, x, y, z, q, eps, sig, L, alpha, rc * rc, rs * rs, p, u[i], &g, sh, f);
            for (int k = 0; k < 3; ++k) raw[k * n + i] = f[k];
            if (ns_out) ns_out[i] = ns;
        }
        free(sh);
    }
    if (bad) { free(raw); return -2; }
    /* F^corr = -(1/N) sum_i (F^core_i + F^shell*_i), index order */
    for (int k = 0; k < 3; ++k) {
        rsum t = {0, 0};
        for (int64_t i = 0; i < n; ++i) rsum_add(&t, raw[k * n + i]);
        const double corr = n > 0 ? -(t.s + t.c) / (double)n : 0.0;
        for (int64_t i = 0; i < n; ++i) F[k * n + i] = raw[k * n + i] + corr;
    }
    free(raw);
    return 0;
}

/*
 * Raw forces F_i^core + F_i^shell* (no momentum correction) of the selected particles
 * sel[0..m-1], each by brute force over all n particles; u: their batch offsets (m).
 * out: 3m doubles, out[d m + s]; ns_out (may be NULL): their N_s.  Returns 0 or -1.
 */
int oracle_rbl_raw_subset(int64_t n, const double *x, const double *y, const double *z, const double *q,
                          const double *eps, const double *sig, double L, double alpha, double rc, double rs,
                          int32_t p, int64_t m, const int64_t *sel, const double *u, double *out, int64_t *ns_out) {
    if (!valid(L, rc, rs, p)) return -1;
    const grid g = make_grid(L, rc, rs);
    int bad = 0;
#pragma omp parallel
    {
        shell_entry *sh = (shell_entry *)malloc(sizeof(shell_entry) * (size_t)(n > 0 ? n : 1));
        if (sh == NULL) bad = 1;
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < m; ++s) {
            if (bad) continue;
            double f[3];
            const int64_t ns = rbl_raw_one(sel[s], n, x, y, z, q, eps, sig, L, alpha, rc * rc, rs * rs, p, u[s], &g,
                                           sh, f);
            for (int k = 0; k < 3; ++k) out[k * m + s] = f[k];
            if (ns_out) ns_out[s] = ns;
        }
        free(sh);
    }
    return bad ? -2 : 0;
}

/*
 * Short-range energy with every pair inside r_s (no batch):
 *   U = (1/2) sum_i sum_{j != i, r < r_s} [4 eps_ij ((s/r)^12 - (s/r)^6) + q_i q_j erfc(sqrt(alpha) r) / r]
 * (Eqs. (lj) and the real-space term of the split Coulomb energy, truncated at r_s).
 */
double oracle_short_energy(int64_t n, const double *x, const double *y, const double *z, const double *q,
                           const double *eps, const double *sig, double L, double alpha, double rs) {
    const double rs2 = rs * rs;
    rsum t = {0, 0};
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double d[3] = {min_image(x[i] - x[j], L), min_image(y[i] - y[j], L), min_image(z[i] - z[j], L)};
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 > rs2) continue;
            const double r = sqrt(r2);
            double e = 0.0;
            const double ee = sqrt(eps[i] * eps[j]);
            if (ee != 0.0) {
                const double s = 0.5 * (sig[i] + sig[j]);
                const double s6 = pow(s / r, 6.0);
                e += 4.0 * ee * (s6 * s6 - s6);
            }
            e += q[i] * q[j] * erfc(sqrt(alpha) * r) / r;
            rsum_add(&t, 0.5 * e);
        }
    return t.s + t.c;
}
