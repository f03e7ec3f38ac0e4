/*
 * rbe.h -- C ABI of the MI355X (gfx950) random batch Ewald k-space library.
 *
 * The library evaluates the Fourier-space (k-space) part of the Coulomb force
 * for N point charges in a periodic cubic box with the random batch Ewald
 * (RBE) estimator (arXiv 2407.09315, Sec. 2.2 and Algorithm 1):
 *
 *   wave vectors     k_l = 2 pi m_l / L,  m_l in Z^3 \ {0},  l = 1..P,
 *                    drawn from exp(-k^2 / 4 alpha) / S      (Sec. 2.2; Alg. 1 step 1)
 *   structure factor rho(k) = sum_j q_j exp(i k . r_j)       (Sec. 2.2; Alg. 1 steps 2-3)
 *   force            F_i = -sum_l c_l q_i k_l Im(exp(-i k_l . r_i) rho(k_l))
 *                                                           (Eq. frbe; Alg. 1 step 4)
 *   energy           U   = sum_l (c_l / 2) |rho(k_l)|^2
 *   with             c_l = w_l 4 pi / (V k_l^2),  V = L^3,
 *                    w_l = S / P for the RBE estimator (Eq. frbe, Q = S),
 *                    w_l = exp(-k_l^2 / 4 alpha) for the full Ewald sum (Eq. long).
 *   S = (sum_{m in Z} exp(-pi^2 m^2 / (alpha L^2)))^3 - 1 is the normalisation
 *   of the sampling density (the paper's Q).
 *
 * Units: Gaussian, prefactor 1 (energy in e^2/A for charges in e and lengths
 * in A); the caller multiplies by its Coulomb constant.  No neutralising
 * background term is added for non-neutral systems.
 *
 * Batches.  Every device call works on a batch of B independent systems whose
 * particles and wave vectors are concatenated: system b owns particles
 * [sys_off[b], sys_off[b+1]) and wave vectors [k_off[b], k_off[b+1]).  A single
 * system is the batch B = 1; there is one code path.
 *
 * Memory.  (dev) = caller-owned device memory, (host) = caller-owned host
 * memory.  The library never allocates or frees device memory: all scratch
 * lives in a caller-provided workspace of rbe_plan_workspace_bytes() bytes,
 * 256-byte aligned.  Its only allocation is the host-side plan object.
 * Device work is enqueued asynchronously on `stream` (a hipStream_t; NULL is
 * the default stream) and the call returns without synchronising.
 *
 * Layouts.  Positions and charges: four FP64 arrays x, y, z, q of N_total
 * elements (structure of arrays).  Positions may lie anywhere; results are
 * periodic in each coordinate with period L.  Wave vectors m: int32, P_total
 * rows of (m_x, m_y, m_z).  rho: FP64 pairs (Re, Im), P_total rows.  Forces:
 * three planes of N_total values, F[d * N_total + i], in FP64 (RBE_FP64) or
 * FP32 (RBE_FP32_MIXED, RBE_FP32).  U: one FP64 value per system.
 *
 * Errors.  Every call returns an rbe_status.  Arguments are checked on the
 * host before anything is enqueued; on failure nothing is launched and
 * rbe_last_error() (thread-local) holds a message.  Nothing aborts.
 * Non-finite positions or charges are not rejected; they propagate as NaN into rho
 * and from there into every force, the energy, the virial and the VJP outputs.
 *
 * Wave vectors.  The sampler never draws m = (0, 0, 0), but a caller-supplied list may
 * hold it (k = 0 is excluded from the Ewald sum): such a row gets rho_l = sum_j q_j
 * (to the rounding of the precision) and the weight c_l = 0, so it adds nothing to F,
 * U, the virial or the VJP, whatever its w_l.
 *
 * Determinism.  Every reduction runs in a fixed order, so results are
 * bitwise reproducible for the same inputs, plan parameters and device.
 */
#ifndef RBE_H
#define RBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RBE_ABI_VERSION 3

typedef enum {
    RBE_OK = 0,
    RBE_EINVAL = -1,          /* invalid argument (host-side check) */
    RBE_ENODEV = -2,          /* no usable HIP device */
    RBE_EHIP = -3,            /* a HIP runtime call or kernel launch failed */
    RBE_EWORKSPACE = -4,      /* workspace missing, misaligned or too small */
    RBE_EUNSUPPORTED = -5     /* valid request this build does not implement */
} rbe_status;

typedef enum {
    RBE_FP64 = 0,             /* FP64 phases, sin/cos and sums throughout */
    RBE_FP32_MIXED = 1,       /* exact fixed-point phases, FP32 sin/cos and per-wave sums,
                                 FP64 cross-block sums and energy; FP32 forces */
    RBE_FP32 = 2              /* as RBE_FP32_MIXED, but the phase m.r/L is formed in FP32
                                 from fractional coordinates in [-1/2, 1/2]: fewer operations,
                                 with a phase error that grows with |m| (about |m|_1 2^-25
                                 turns).  Plans are refused (RBE_EUNSUPPORTED) for systems
                                 with L sqrt(2 alpha) / (2 pi) > 16, the spread of sampled
                                 m per component; caller-supplied m needs
                                 |m_x| + |m_y| + |m_z| <= 510 (the hardware sine takes at
                                 most 256 turns).  No phase cache */
} rbe_precision;

typedef enum {
    RBE_PHASE_AUTO = 0,       /* the measured choice for this shape (currently recompute) */
    RBE_PHASE_RECOMPUTE = 1,  /* the force pass recomputes every phase */
    RBE_PHASE_CACHED = 2      /* the rho pass stores (cos, sin) of every (i, l) in the
                                 workspace (8 B per term, FP32_MIXED only) and the force
                                 pass reads them */
} rbe_phase_mode;

/* Device sampler of a plan (rbe_plan_set_sampler). */
typedef enum {
    RBE_SAMPLER_EXACT = 0,       /* exact i.i.d. draws (rbe_sample_k), the default */
    RBE_SAMPLER_METROPOLIS = 1   /* the paper's Metropolis procedure (rbe_sample_k_metropolis) */
} rbe_sampler;

/*
 * A batch of B independent periodic cubic systems (all host memory, read only by
 * rbe_plan_create, which copies what it needs).  System b owns particles
 * [sys_off[b], sys_off[b+1]) and wave vectors [k_off[b], k_off[b+1]) of the
 * concatenated arrays; L[b] is its box edge (A) and alpha[b] its Ewald splitting
 * parameter (A^-2), both finite and > 0.
 */
typedef struct {
    int32_t B;                /* number of systems, > 0 */
    const int64_t *sys_off;   /* B + 1 non-decreasing particle offsets, sys_off[0] = 0 */
    const int64_t *k_off;     /* B + 1 non-decreasing wave-vector offsets, k_off[0] = 0 */
    const double *L;          /* B box edges */
    const double *alpha;      /* B splitting parameters */
} rbe_batch_desc;

typedef struct rbe_plan rbe_plan;   /* opaque; host memory owned by the library */
typedef struct rbe_graph rbe_graph; /* opaque; an instantiated HIP graph of one evaluation */

/* ---------------------------------------------------------------- host-only calls */

/*
 * Draw P wave-vector index triples m (Sec. 2.2; Alg. 1 step 1): i.i.d. from
 * exp(-k^2 / 4 alpha) with k = 2 pi m / L and m != 0.  Each component is a
 * 1-D discrete Gaussian exp(-pi^2 m_d^2 / (alpha L^2)) drawn by inverse CDF on
 * |m_d| <= ceil(9 L sqrt(alpha/2) / pi) + 1; a zero vector is redrawn.
 * Uniforms come from Philox4x64-10 (Salmon et al., SC'11) with key
 * (seed, stream_id) and counter (l, attempt, 0, 0); word d gives
 * u_d = (word_d >> 11) * 2^-53.  m_out: (host) P*3 int32.  w_out (host, P
 * doubles, may be NULL) receives S/P; S_out (host, may be NULL) receives S.
 * Returns RBE_EINVAL for L <= 0, alpha <= 0, P < 0, NULL m_out with P > 0,
 * or if the zero vector is drawn 1024 times in a row.
 */
rbe_status rbe_sample_k(uint64_t seed, uint64_t stream_id, double L, double alpha, int32_t P,
                        int32_t *m_out, double *w_out, double *S_out);

/*
 * Draw P wave-vector index triples with the Metropolis procedure the paper names
 * for this step (Sec. 2.2; Alg. 1 step 1).  The paper fixes no proposal, start or
 * burn-in; this chain (one per wave vector, the P chains independent):
 *   target   exp(-pi^2 |m|^2 / (alpha L^2)) on Z^3 \ {0};
 *   start    m = (1, 0, 0);
 *   proposal m' = m + d, each d_j uniform on {-D..D}, D = max(1, ceil(1.5 sigma)),
 *            sigma = L sqrt(alpha/2) / pi;
 *   accept   m' != 0 and (|m'|^2 <= |m|^2 or u < exp(-pi^2 (|m'|^2 - |m|^2) / (alpha L^2)));
 *   output   the state after burn_in steps.
 * Step t of chain l draws Philox4x64-10 with key (seed, stream_id) and counter
 * (l, t, 1, 0): d_j = min(floor(u_j (2D + 1)), 2D) - D from words 0..2, u from
 * word 3 (u = (word >> 11) * 2^-53).  After a finite burn-in the draws are only
 * approximately distributed as the target (64 steps reach it within the noise
 * of 10^5 samples for the boxes of this library's workloads).  Outputs as for
 * rbe_sample_k.  RBE_EINVAL for L <= 0, alpha <= 0, P < 0, burn_in < 0 or a
 * NULL m_out with P > 0.
 */
rbe_status rbe_sample_k_metropolis(uint64_t seed, uint64_t stream_id, double L, double alpha, int32_t P,
                                   int32_t burn_in, int32_t *m_out, double *w_out, double *S_out);

/* S = (sum_m exp(-pi^2 m^2 / (alpha L^2)))^3 - 1 (the paper's Q). */
rbe_status rbe_normalization(double L, double alpha, double *S_out);

/*
 * Full-Ewald weights w_l = exp(-k_l^2 / 4 alpha) (Eq. long) for given m (host,
 * P*3 int32) into w_out (host, P doubles).  With these weights the library
 * evaluates the deterministic Ewald k-space sum over the listed vectors.
 */
rbe_status rbe_ewald_weights(double L, double alpha, int32_t P, const int32_t *m, double *w_out);

/*
 * Create a plan for the batch `batch` (host; see rbe_batch_desc).  precision:
 * rbe_precision; phase_mode: rbe_phase_mode.  The plan copies everything it needs;
 * the descriptor and its arrays may be freed afterwards.  Tile parameters come from
 * the built-in defaults or from rbe_plan_set_tiles.  RBE_EINVAL for a NULL
 * descriptor or array, B <= 0, offsets that do not start at 0 or decrease, a
 * system of 2^30 or more particles or wave vectors, L or alpha not finite and
 * > 0, or an unknown enum; RBE_EUNSUPPORTED for the combinations noted at
 * rbe_precision and rbe_phase_mode.  *out is NULL on failure.
 */
rbe_status rbe_plan_create(const rbe_batch_desc *batch, int32_t precision, int32_t phase_mode,
                           rbe_plan **out);

/* Bytes of device workspace the plan needs (a multiple of 256). */
size_t rbe_plan_workspace_bytes(const rbe_plan *plan);

/*
 * Select kernel variants (autotuner hook).  rho_variant and force_variant
 * index the variant tables reported by rbe_plan_num_variants; -1 keeps the
 * current choice.  The workspace size covers every variant, but its contents
 * change: call rbe_plan_upload again before the next device call.
 */
rbe_status rbe_plan_set_tiles(rbe_plan *plan, int32_t rho_variant, int32_t force_variant);
rbe_status rbe_plan_num_variants(const rbe_plan *plan, int32_t *n_rho, int32_t *n_force);
rbe_status rbe_plan_get_tiles(const rbe_plan *plan, int32_t *rho_variant, int32_t *force_variant);

/*
 * Layout of rho variant `variant` of the plan's precision (0 <= variant < n_rho of
 * rbe_plan_num_variants), written to the six host int32 outputs:
 *   particles_per_lane: the per-wave layouts' tile is 64 x this many particles;
 *   vectors_per_chunk: wave vectors per inner-loop chunk (per lane in the k-lane layout);
 *   vectors_per_item: at most this many wave vectors per work item;
 *   waves_per_block: 4 (one item per wave), 16 (one block per CU sharing single-chunk
 *     items) or 1 (k-lane layout: one item per 256-thread block, wave vectors across
 *     the lanes);
 *   particles_per_tile: particles per tile (64 x particles_per_lane, or for a k-lane
 *     variant its own size; with the phase cache a k-lane variant uses 64 x
 *     particles_per_lane);
 *   compensated: 1 if the forward rho pass of the FP32 forms sums in compensated FP32
 *     (runs of 16 terms per lane added into (hi, lo) pairs by TwoSum, pairs combined
 *     within the block, FP64 only across tiles), 0 for plain FP32 per-lane sums of at
 *     most 43 terms combined in FP64.  The adjoint pass B1 and the phase cache use the
 *     plain sums.
 * RBE_EINVAL for a NULL pointer or a variant out of range.
 */
rbe_status rbe_plan_rho_variant_info(const rbe_plan *plan, int32_t variant, int32_t *particles_per_lane,
                                     int32_t *vectors_per_chunk, int32_t *vectors_per_item,
                                     int32_t *waves_per_block, int32_t *particles_per_tile,
                                     int32_t *compensated);

/*
 * Persistent grids.  The rho-shaped passes run one wave per work item, four
 * waves per block (the k-lane rho variants: one four-wave block per item);
 * rho_cap > 0 launches at most rho_cap waves (rounded up to whole blocks).
 * The force-shaped passes run one 256-thread block per work item;
 * force_cap > 0 launches at most force_cap blocks.  Wave (block) j of a
 * capped grid of G takes items j, j + G, j + 2G, ...  0 (the default) launches
 * one wave (block) per item.  Results do not depend on the caps (each item
 * writes its own partial-sum slots).
 */
rbe_status rbe_plan_set_grid_caps(rbe_plan *plan, int32_t rho_cap, int32_t force_cap);
rbe_status rbe_plan_get_grid_caps(const rbe_plan *plan, int32_t *rho_cap, int32_t *force_cap);

/*
 * Occupancy clamp of the rho-shaped passes (on by default): each single-wave block
 * reserves unused LDS so that a CU holds at most its even share of the pass's
 * blocks (4 x ceil(blocks / (4 x CUs))), whatever the state the previous kernel
 * left the CUs in.  The autotuner measures both settings.
 */
rbe_status rbe_plan_set_occupancy_clamp(rbe_plan *plan, int32_t on);
rbe_status rbe_plan_get_occupancy_clamp(const rbe_plan *plan, int32_t *on);

/*
 * Kernel timing hook: when set (non-NULL hipEvent_t handles), every later call
 * records rho_begin / rho_end on its stream right before / after the rho-pass
 * kernel (the cross-tile reduction is outside the pair) and force_begin /
 * force_end around the force-pass kernel.  NULL clears a slot.  The events
 * belong to the caller.
 */
rbe_status rbe_plan_set_timing_events(rbe_plan *plan, void *rho_begin, void *rho_end,
                                      void *force_begin, void *force_end);

/* Release the plan (host memory only). */
void rbe_plan_destroy(rbe_plan *plan);

/* ---------------------------------------------------------------- device calls */

/*
 * Copy the plan's metadata (system table, work lists, sampler tables) into
 * the workspace ws (dev, rbe_plan_workspace_bytes bytes, 256-byte aligned)
 * and wait for the copy.  Call once per workspace, before any other device
 * call with that workspace and before any graph capture.
 */
rbe_status rbe_plan_upload(const rbe_plan *plan, void *ws, void *stream);

/*
 * rho(k_l) for every wave vector of every system (Sec. 2.2; Alg. 1 steps 2-3).
 * x, y, z, q: (dev) N_total FP64 each.  m: (dev) P_total*3 int32.
 * rho: (dev) P_total*2 FP64 (Re, Im).  ws: the uploaded workspace.
 * In RBE_PHASE_CACHED mode this call also fills the phase cache in ws.
 */
rbe_status rbe_structure_factor(const rbe_plan *plan, const double *x, const double *y,
                                const double *z, const double *q, const int32_t *m,
                                double *rho, void *ws, void *stream);

/*
 * Forces and energies from rho (Eq. frbe with per-k weights; Alg. 1 step 4).
 * w: (dev) P_total FP64 weights (S/P for RBE, exp(-k^2/4 alpha) for Ewald).
 * rho: (dev) the output of rbe_structure_factor for the same inputs.
 * F: (dev) 3*N_total values, FP64 for RBE_FP64, FP32 for RBE_FP32_MIXED and RBE_FP32.
 * U: (dev) B FP64 values.  In RBE_PHASE_CACHED mode the phase cache in ws
 * must come from rbe_structure_factor on the same positions.  In the FP32
 * precisions the call first writes one 32-byte row per wave vector (m, c_l
 * times rho) into ws with a small kernel; rbe_evaluate and the graph have the
 * cross-tile reduction write these rows instead.
 */
rbe_status rbe_kspace_force(const rbe_plan *plan, const double *x, const double *y,
                            const double *z, const double *q, const int32_t *m,
                            const double *w, const double *rho, void *F, double *U, void *ws,
                            void *stream);

/*
 * k-space virial tensor of every system (the pressure term of the NPT variant the
 * paper cites in Sec. 2.2): the negative derivative of the long-range energy
 * term under a symmetric affine strain of the box at fixed fractional
 * coordinates,
 *   W_ab = sum_l U_l (delta_ab - 2 k_la k_lb (1/k_l^2 + 1/(4 alpha))),
 *   U_l = (c_l / 2) |rho_l|^2.
 * The 1/(4 alpha) part is the strain derivative of the Ewald kernel
 * exp(-k^2/4 alpha); with RBE weights w = S/P the sum is the importance-sampled
 * estimate of the Ewald k-space virial.  m, w, rho: (dev) as for
 * rbe_kspace_force.  W: (dev) 6 FP64 values per system, in the order xx, yy,
 * zz, xy, xz, yz.  Summed in a fixed order in FP64 for every precision.
 */
rbe_status rbe_kspace_virial(const rbe_plan *plan, const int32_t *m, const double *w,
                             const double *rho, double *W, void *ws, void *stream);

/*
 * Vector-Jacobian product of (U, F) (derived from the definitions above; the
 * paper has no adjoint).  Upstream gradients: gU (dev, B FP64) on U and gF
 * (dev, 3*N_total, dtype of F) on F.  Outputs (dev, FP64 in every precision): gr
 * (3*N_total, dL/dr, three planes like F) and gq (N_total, dL/dq).  The FP32
 * forms accumulate in FP32 and write doubles.  rho must be the forward
 * structure factor.  Phases are recomputed (no phase cache is used).
 */
rbe_status rbe_kspace_vjp(const rbe_plan *plan, const double *x, const double *y,
                          const double *z, const double *q, const int32_t *m, const double *w,
                          const double *rho, const double *gU, const void *gF, double *gr,
                          double *gq, void *ws, void *stream);

/*
 * Choose the plan's device sampler: RBE_SAMPLER_EXACT (default) or
 * RBE_SAMPLER_METROPOLIS with `burn_in` steps per chain (default 64).  Used by
 * rbe_sample_k_device, rbe_evaluate, rbe_evaluate_static and graphs created
 * afterwards.  RBE_EINVAL for another value or burn_in < 0.
 */
rbe_status rbe_plan_set_sampler(rbe_plan *plan, int32_t sampler, int32_t burn_in);

/*
 * Draw the wave vectors of every system on the device: system b uses the
 * plan's sampler with key (seed + b, stream_id), so its rows of m equal
 * rbe_sample_k(seed + b, stream_id, L_b, alpha_b, P_b) (or
 * rbe_sample_k_metropolis with the plan's burn-in).  m: (dev) P_total*3 int32;
 * w: (dev) P_total FP64 receives S_b / P_b.  The plan rejects systems whose
 * zero-vector probability exceeds 1/2.
 */
rbe_status rbe_sample_k_device(const rbe_plan *plan, uint64_t seed, uint64_t stream_id,
                               int32_t *m, double *w, void *ws, void *stream);

/*
 * Autotuner: time every rho-pass variant and every force-pass variant on the
 * caller's inputs, in the order an evaluation runs them (rbe_structure_factor
 * then rbe_kspace_force, reps timed rounds after one warm-up, HIP events on
 * `stream` right around each kernel), the rho variants with and without the
 * occupancy clamp; keep the fastest of each with one block per work item,
 * upload the plan again and report the choice and its mean kernel times in ms
 * (any output pointer may be NULL).  Arguments as for the calls it times; rho,
 * F and U are overwritten.  Synchronises `stream`.  On failure the plan keeps the
 * variants it had and is uploaded to ws again, so it stays usable.
 */
rbe_status rbe_plan_tune(rbe_plan *plan, const double *x, const double *y, const double *z,
                         const double *q, const int32_t *m, const double *w, double *rho, void *F,
                         double *U, void *ws, void *stream, int32_t reps, int32_t *rho_variant,
                         int32_t *force_variant, int32_t *rho_grid_cap, double *rho_ms,
                         double *force_ms);

/*
 * One whole evaluation of every system of the plan (Alg. 1 steps 2-4), enqueued
 * on `stream` without host synchronisation: device sampling
 * (rbe_sample_k_device), rbe_structure_factor and rbe_kspace_force.  Arguments
 * and step_counter as for rbe_graph_create below; m and w are outputs (the drawn
 * wave vectors and weights).  Back-to-back calls keep the device busy without
 * the per-launch cost of a graph replay.
 */
rbe_status rbe_evaluate(const rbe_plan *plan, uint64_t seed, uint64_t stream_base,
                        uint64_t *step_counter, const double *x, const double *y, const double *z,
                        const double *q, int32_t *m, double *w, double *rho, void *F, double *U,
                        void *ws, void *stream);

/*
 * Capture one whole evaluation of every system of the plan -- device sampling
 * (rbe_sample_k_device), rbe_structure_factor and rbe_kspace_force -- into a
 * HIP graph, for replay with rbe_graph_launch at the cost of one launch.
 * The graph records the pointers given here; replays read the buffers' current
 * contents (update positions in place between replays).  step_counter (dev, one
 * uint64, may be NULL): the sampler of system b uses stream id
 * stream_base + *step_counter and the force pass adds 1 to it, so every replay
 * draws new wave vectors (NULL: every replay uses stream_base).  The plan and
 * the workspace must stay alive and uploaded while the graph is used.
 */
rbe_status rbe_graph_create(const rbe_plan *plan, uint64_t seed, uint64_t stream_base,
                            uint64_t *step_counter, const double *x, const double *y,
                            const double *z, const double *q, int32_t *m, double *w, double *rho,
                            void *F, double *U, void *ws, rbe_graph **out);
rbe_status rbe_graph_launch(const rbe_graph *graph, void *stream);
void rbe_graph_destroy(rbe_graph *graph);

/*
 * rbe_evaluate without a workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same kernels and results as rbe_evaluate (bitwise), with the
 * workspace replaced by a library-owned device scratch array of 64 MiB, one per
 * device, alive until the process ends.  The call allocates nothing and frees
 * nothing; the caller still passes every input and output.
 *   Limit: the plan's current layout must fit the scratch; a larger one (about
 *   10M charges at P = 200, or the phase cache of all but small systems) returns
 *   RBE_EWORKSPACE before anything is enqueued -- use rbe_evaluate then.
 *   Sharing: all calls on one device share its scratch.  The first call with a
 *   plan (or after rbe_plan_set_tiles / rbe_plan_tune changed its layout, or after
 *   another plan used the scratch) enqueues an upload of the plan's tables ahead
 *   of the kernels.  Calls that may overlap on one device -- concurrent host
 *   threads, or different streams without synchronisation between them -- race on
 *   the scratch and must be serialised by the caller.
 *   Errors: as rbe_evaluate; RBE_EUNSUPPORTED for device ordinals >= 64.
 */
rbe_status rbe_evaluate_static(const rbe_plan *plan, uint64_t seed, uint64_t stream_base,
                               uint64_t *step_counter, const double *x, const double *y,
                               const double *z, const double *q, int32_t *m, double *w,
                               double *rho, void *F, double *U, void *stream);

/* ---------------------------------------------------------------- diagnostics */

const char *rbe_status_string(rbe_status status);
const char *rbe_last_error(void);   /* thread-local text of the last failure on this thread */
int32_t rbe_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RBE_H */
