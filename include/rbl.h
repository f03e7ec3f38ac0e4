/*
 * rbl.h -- C ABI of the random batch list (RBL) short-range force on MI355X (gfx950).
 *
 * The short-range part of the nonbonded force (arXiv 2407.09315, Sec. 2.3 and
 * Algorithm 2): around particle i the core C(i) = {j != i : r_ij < r_c} is summed
 * exactly and the shell S(i) = {j : r_c <= r_ij <= r_s} is estimated from a batch,
 *
 *   F_i^core   = sum_{j in C(i)} F_ij                                  (Eq. short)
 *   F_i^shell* = (N_s / p) sum_{j in B(i)} F_ij,  N_s = |S(i)|          (Eq. fshell)
 *   F^corr     = -(1/N) sum_i (F_i^core + F_i^shell*)   (momentum correction)
 *   F_i        = F_i^core + F_i^shell* + F^corr,
 *
 * with the pair force on i from j, d = r_i - r_j at the minimum image, r = |d|:
 *   Lennard-Jones (Eq. lj, Lorentz-Berthelot mixing eps_ij = sqrt(eps_i eps_j),
 *     s_ij = (sig_i + sig_j) / 2):   24 eps_ij (2 (s_ij/r)^12 - (s_ij/r)^6) d / r^2;
 *   real-space Ewald Coulomb (Eq. fshort, prefactor 1):
 *     q_i q_j (erfc(sqrt(alpha) r) / r^2 + 2 sqrt(alpha / pi) exp(-alpha r^2) / r) d / r.
 *
 * The batch (the paper fixes no scheme): systematic sampling of the shell in a fixed
 * traversal order.  Particle i draws u_i in [0, 1) -- word 0 of Philox4x64-10 (Salmon
 * et al., SC'11) with key (seed, step) and counter (i, 0, 3, 0), top 53 bits -- and
 * takes the shell members at positions min(floor((b + u_i) N_s / p), N_s - 1), b = 0..p-1
 * (the minimum is the exact value where the rounding of b + u_i reaches p), each with
 * weight N_s / p; when N_s <= p the batch is the whole shell with weight 1.  Every
 * shell particle is in the batch with probability p / N_s, so the estimate is unbiased.
 * Traversal order: cells of side h = L / nc, nc = floor(L / r_c); stencil reach
 * R = ceil(r_s / h); per axis the cell offsets -R..R (all nc cells, offsets 0..nc-1, when
 * 2R + 1 > nc), x outermost, z innermost; within a cell, ascending particle index; a
 * particle's cell is min(floor((x / L - floor(x / L)) nc), nc - 1) per axis.
 *
 * Layouts: x, y, z, q, eps, sig are (dev) FP64 arrays of N; F is (dev) 3N FP64,
 * F[d N + i]; all arithmetic is FP64.  Scratch lives in a caller workspace of
 * rbl_plan_workspace_bytes() bytes, 256-byte aligned; work is enqueued on `stream`
 * without synchronisation.  Results are bitwise reproducible for the same inputs.
 * Positions may lie outside [0, L) (they are wrapped); a non-finite position gives NaN
 * forces, which the momentum correction carries to every particle.
 *
 * Work split: the fast path holds a cell's stencil of up to `stencil_positions` particles
 * in on-chip memory and up to `pairs_per_particle` core and batch pairs per particle in the
 * workspace (rbl_plan_capacity; sized from the mean density N / L^3 with a wide Poisson
 * allowance, a multiple of 4, at most 4096).  Particles beyond either take a slower path
 * with the same result; the sum order of a particle's pairs differs between the two, by
 * rounding only.
 */
#ifndef RBL_H
#define RBL_H

#include "rbe.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t N;       /* particles, >= 0 (below 2^31) */
    double L;        /* cubic box edge, > 0 */
    double alpha;    /* Ewald splitting of the real-space Coulomb term, >= 0 */
    double r_c;      /* core radius, > 0 */
    double r_s;      /* outer cutoff, r_c <= r_s < L / 2 */
    int32_t p;       /* shell batch size, >= 1 */
} rbl_params;

typedef struct rbl_plan rbl_plan;   /* opaque; host memory owned by the library */

/* Validate the parameters and fix the cell grid.  RBE_EINVAL for parameters out of range
   (also a grid of more than 2^28 cells). */
rbe_status rbl_plan_create(const rbl_params *params, rbl_plan **out);
size_t rbl_plan_workspace_bytes(const rbl_plan *plan);
/* The cell grid: cells per axis, stencil reach R (in cells) and cells per stencil axis. */
rbe_status rbl_plan_grid(const rbl_plan *plan, int32_t *cells_per_axis, int32_t *reach, int32_t *stencil_span);
/* Events (hipEvent_t, created and owned by the caller) that rbl_short_force records on its
   stream just before and after the selection kernel and the pair kernel, for timing those two
   kernels; NULL clears a slot.  RBE_EINVAL for a NULL plan. */
rbe_status rbl_plan_set_timing_events(rbl_plan *plan, void *select_begin, void *select_end, void *pair_begin,
                                      void *pair_end);
/* The fast path's limits: pair slots per particle and stencil positions per cell. */
rbe_status rbl_plan_capacity(const rbl_plan *plan, int32_t *pairs_per_particle, int32_t *stencil_positions);
void rbl_plan_destroy(rbl_plan *plan);

/*
 * The RBL short-range force of every particle (Algorithm 2: cell list, core sum and shell
 * batch, momentum correction), enqueued on `stream`.  ns (dev, may be NULL) receives N_s of
 * every particle (int32).  RBE_EINVAL for NULL arrays with N > 0, RBE_EWORKSPACE for a
 * NULL or misaligned workspace, RBE_ENODEV without a device, RBE_EHIP on a launch error.
 */
rbe_status rbl_short_force(const rbl_plan *plan, const double *x, const double *y, const double *z,
                           const double *q, const double *eps, const double *sig, uint64_t seed,
                           uint64_t step, double *F, int32_t *ns, void *ws, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RBL_H */
