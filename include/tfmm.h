/*
 * tfmm.h -- C ABI of libtfmm, an MI355X (gfx950) implementation of the
 * angular-momentum-conserving Fast Multipole Method of Korobkin et al.,
 * "Conservation of Angular Momentum in the Fast Multipole Method"
 * (arXiv:2107.07166).
 *
 * What is computed (paper Sec. 2, notation kept): N particles at X_a with
 * masses m_a; gravitational forces F_a = m_a a_a with G a parameter.  Pairs of
 * tree nodes A, B that pass the multipole acceptance criterion
 * (Eq. mac_criterion: (r_A,max + r_B,max) / R <= theta, theta = tan of the
 * MAC angle, 0 <= theta < 1) interact through the Taylor series of Eq. taylor
 * truncated at total degree p about the two centres of mass; all other pairs
 * of leaves interact exactly (Eq. jia).  Both directions of every pair use
 * the same expression (mutual interactions), so linear momentum is conserved
 * (Eq. netforce).  Three variants:
 *   TFMM_STANDARD   -- the symmetric expansion itself (leaves the spurious
 *                      torques of Eq. total_torque);
 *   TFMM_CONSERVING -- each far-field pair force re-projected onto the line
 *                      joining the two particles (Eq. realign), with the
 *                      projection scalar expanded in (x_a - y_b) to degree
 *                      p-1 (Eqs. nab-expansion, abnab-expansion; equal to
 *                      Eq. aaB1 at p = 2): no spurious torque;
 *   TFMM_CONSERVING_R2 -- zeroth order only (p must be 1): each far-field pair
 *                      force is the zeroth-order magnitude along the line
 *                      joining the particles (Eq. realign2), that line
 *                      expanded to first order in (x_a - y_b)/|R|
 *                      (Eq. nab-expansion); summed over a node this is
 *                      Eq. aaB0, which needs the node quadrupoles.  With
 *                      softening the magnitude is |R| (R^2 + eps^2)^(-3/2).
 * Softening: the kernel is -(r^2 + eps^2)^(-1/2) in the near and far field.
 *
 * Conventions for every entry point:
 *  - return value: TFMM_OK (0) or a negative tfmm_status; on error the
 *    context keeps a message, see tfmm_last_error();
 *  - device pointers are HIP device addresses (e.g. torch.Tensor.data_ptr()
 *    of a CUDA/HIP tensor); they stay owned by the caller and must outlive
 *    the stream work that reads or writes them;
 *  - `stream` is a hipStream_t (NULL = the null stream); work is enqueued on
 *    it in order.  Calls return after enqueueing, except where noted as
 *    "synchronising" (they wait for the work queued on the stream so far:
 *    the host polls a pinned word that a kernel writes after that work, for
 *    at most 20 ms, then blocks in the runtime);
 *  - a context is not thread-safe: use one per host thread;
 *  - after TFMM_EDEVICE the context is unusable and must be destroyed.
 */
#ifndef TFMM_H
#define TFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TFMM_OK = 0,
    TFMM_EINVAL = -1,  /* invalid argument; nothing was enqueued */
    TFMM_ENOMEM = -2,  /* the context's device-memory budget would be exceeded */
    TFMM_EDEVICE = -3, /* a HIP call failed; the context is now unusable */
    TFMM_ESTATE = -4   /* object used out of order (e.g. lists before a walk) */
} tfmm_status;

typedef enum { TFMM_STANDARD = 0, TFMM_CONSERVING = 1, TFMM_CONSERVING_R2 = 2 } tfmm_variant;

/* TFMM_FP64: every step in FP64.  TFMM_MIXED32: near field (P2P) and M2L in
 * FP32 with FP64 accumulation across source leaves / per node; tree, centres
 * of mass, r_max, moments (P2M, M2M), L2L, L2P and all reductions in FP64. */
typedef enum { TFMM_FP64 = 0, TFMM_MIXED32 = 1 } tfmm_precision;

typedef struct tfmm_ctx tfmm_ctx;   /* device, memory budget, error state */
typedef struct tfmm_tree tfmm_tree; /* one particle set: keys, octree, lists, expansions */

typedef struct {
    int p;            /* expansion order, 1..8 (Eq. taylor truncated at degree p) */
    double theta;     /* tan(theta_MAC) of Eq. mac_criterion, 0 <= theta < 1 */
    double softening; /* Plummer softening eps >= 0 */
    double G;         /* gravitational constant */
    int variant;      /* tfmm_variant */
    int precision;    /* tfmm_precision */
    int scalar_degree; /* TFMM_CONSERVING only: degree K of the projection
                          scalar (a.u)/|u|^2 of Eq. abnab-expansion, which
                          Sec. 3.2 allows to keep more terms; 0 = the default
                          p-1; otherwise p-1 <= K <= min(p+1, 6).  The order-p
                          standard force is realigned (Eq. realign) with the
                          scalar's Taylor polynomial of degree K in
                          x_a - y_b: still central, no net torque, closer to
                          the direct sum; moments and locals of order K+1. */
} tfmm_params;

/* Create a context on HIP device `device` that may hold at most
 * `hbm_budget_bytes` of library-owned device memory (0 = no limit).
 * Errors: EINVAL (bad device or NULL out), EDEVICE. */
int tfmm_ctx_create(int device, size_t hbm_budget_bytes, tfmm_ctx **out);

/* Destroy a context; every tree created from it must be destroyed first.
 * Synchronises the device.  NULL is ignored. */
int tfmm_ctx_destroy(tfmm_ctx *ctx);

/* Message of the last failed call on this context ("" if none).  Valid until
 * the next call on the context. */
const char *tfmm_last_error(const tfmm_ctx *ctx);

/* Device memory currently held by the context's trees and scratch.  Buffers
 * released by destroyed or resized trees stay with the context for reuse by
 * later trees (they count against hbm_budget_bytes, and are given back to the
 * device when a new allocation would exceed the budget or fail, and when the
 * context is destroyed); they are not included here. */
size_t tfmm_ctx_bytes_in_use(const tfmm_ctx *ctx);

/* All device memory the context holds: the buffers counted by
 * tfmm_ctx_bytes_in_use plus the released blocks it keeps for reuse (the
 * amount charged against hbm_budget_bytes).  0 for NULL. */
size_t tfmm_ctx_bytes_held(const tfmm_ctx *ctx);

/* Change the context's device-memory budget (0 = no limit) for later
 * allocations; released blocks kept for reuse are given back first if the
 * context holds more than the new budget.  Memory already in use by trees is
 * not touched (later growth beyond the budget fails with ENOMEM).  Errors:
 * EINVAL (NULL), EDEVICE. */
int tfmm_ctx_set_budget(tfmm_ctx *ctx, size_t hbm_budget_bytes);

/* Give every released block the context keeps for reuse back to the device
 * (tfmm_ctx_bytes_held then equals tfmm_ctx_bytes_in_use).  Synchronises the
 * device.  Errors: EINVAL (NULL). */
int tfmm_ctx_trim(tfmm_ctx *ctx);

/* Build the tree for n particles.  pos: device, n x 3 FP64 row-major (x, y, z
 * of particle a at pos[3a..3a+2]); mass: device, n FP64 (> 0).  n_leaf: a
 * node with more than n_leaf particles is split (1..4096).  Keys: 21 bits per
 * axis over the bounding cube, stable sort, octree numbered level by level in
 * Morton order; per node FP64 mass, centre of mass and r_max (the exact
 * largest particle distance from the centre of mass, Eq. mac_criterion).
 * Synchronising (reads the level boundaries back once).  The tree keeps its
 * own sorted copy of pos and mass.  Errors: EINVAL, ENOMEM, EDEVICE. */
int tfmm_build_tree(tfmm_ctx *ctx, int64_t n, const double *pos, const double *mass,
                    int n_leaf, void *stream, tfmm_tree **out);

/* Rebuild an existing tree in place for a particle set of n particles (n may
 * differ from the previous build; pos and mass as in tfmm_build_tree).  Device
 * buffers are grow-only, so a tree reused for sets of similar size allocates
 * nothing.  Synchronising.  Errors: EINVAL, ENOMEM, EDEVICE. */
int tfmm_tree_rebuild(tfmm_tree *tree, int64_t n, const double *pos, const double *mass, void *stream);

/* Run the mutual dual-tree walk for `theta` (Eq. mac_criterion) and build the
 * per-target interaction lists.  tfmm_evaluate_forces calls it when theta
 * changed; exposed for list export.  Synchronising.  Errors: EINVAL, ENOMEM,
 * EDEVICE. */
int tfmm_tree_walk(tfmm_tree *tree, double theta, void *stream);

/* Forces on every particle: force (device, n x 3 FP64 row-major, original
 * particle order) = G m_a (near + far) for the tree's particles.
 * potential: NULL, or device n FP64 (original order) that receives
 * G phi(X_a): the exact softened near-field potential of the other particles
 * -sum m_b (r^2 + eps^2)^(-1/2) plus the far field from the standard
 * expansion of Eq. taylor (potential coefficient L_0 included) truncated at
 * degree p, for every variant (the realigned variants change the forces,
 * not this potential).  It costs an extra far-field pass after the forces.  Asynchronous except for the walk
 * when params->theta differs from the tree's last walk.  Part of the work
 * runs on a second stream owned by the tree, forked from `stream` at the call
 * and joined back into it before the forces are written, so the call is
 * ordered on `stream` like a single kernel.
 * Errors: EINVAL (p outside 1..8, theta outside [0,1), eps < 0, bad variant
 * or precision, TFMM_CONSERVING_R2 with p != 1, scalar_degree set for another
 * variant or outside its range, NULL force), ENOMEM, EDEVICE. */
int tfmm_evaluate_forces(tfmm_tree *tree, const tfmm_params *params, double *force,
                         double *potential, void *stream);

/* Forests: several independent particle sets solved by one set of launches
 * (for serving many small requests at once).  Set k is particles
 * offsets[k] .. offsets[k+1]-1 of pos and mass (device, laid out as in
 * tfmm_build_tree); offsets is a host array of n_sets + 1 ascending values
 * with offsets[0] = 0 and every set non-empty (1 <= n_sets <= 4096, at most
 * 2^30 particles in all).  Every set gets what tfmm_build_tree would build
 * for it alone -- its own bounding cube, keys, octree under its own root
 * (node k is the root of set k; nodes are numbered level by level across the
 * sets, in set order inside a level), moments and r_max (Eq.
 * mac_criterion) -- and the walk starts from the pair (root k, root k) of
 * every set, so nodes of different sets never interact: the forces of a set
 * are bit for bit those of the set solved alone with the same parameters.
 * Synchronising.  Errors: EINVAL (bad offsets or n_leaf, NULL pointers),
 * ENOMEM, EDEVICE. */
int tfmm_build_forest(tfmm_ctx *ctx, int n_sets, const int64_t *offsets, const double *pos,
                      const double *mass, int n_leaf, void *stream, tfmm_tree **out);

/* Rebuild any tree in place as a forest of n_sets sets (arguments as in
 * tfmm_build_forest; n_sets = 1 is tfmm_tree_rebuild, and tfmm_tree_rebuild
 * turns a forest back into one set).  Synchronising.  Errors: as
 * tfmm_build_forest. */
int tfmm_forest_rebuild(tfmm_tree *tree, int n_sets, const int64_t *offsets, const double *pos,
                        const double *mass, void *stream);

/* tfmm_evaluate_forces on a forest with one MAC parameter per set: theta is
 * a host array of n_sets values in [0, 1) (Eq. mac_criterion for the pairs of
 * set k uses theta[k]), or NULL for params->theta everywhere.  p, softening,
 * G, variant, precision and scalar_degree are shared by all sets.  force and
 * potential are laid out like pos (set after set, input order inside a set).
 * tfmm_evaluate_forces on a forest equals this call with theta = NULL.
 * Errors: as tfmm_evaluate_forces, and EINVAL for a theta outside [0, 1). */
int tfmm_evaluate_forest(tfmm_tree *tree, const tfmm_params *params, const double *theta,
                         double *force, double *potential, void *stream);

/* Build + evaluate in one call (tree is built, used and destroyed).
 * Synchronising.  Errors: as tfmm_build_tree and tfmm_evaluate_forces. */
int tfmm_evaluate_forces_oneshot(tfmm_ctx *ctx, int64_t n, const double *pos, const double *mass,
                                 int n_leaf, const tfmm_params *params, double *force, void *stream);

/* nsteps kick-drift-kick leapfrog steps on resident state (gravity-only
 * analogue of the paper's star evolution, Sec. 4): v += (F/m) dt/2;
 * x += v dt; rebuild the tree and walk it; F = force(x); v += (F/m) dt/2.
 * pos, vel, force: device n x 3 FP64 (updated in place); mass: device n FP64,
 * the masses the tree was built with.  force must hold the forces at pos on
 * entry when force_valid != 0, otherwise they are evaluated first; on return
 * it holds the forces at the final positions.  The tree must have been built
 * for n particles, as one set (not a forest).  Synchronising (each rebuild
 * reads sizes).
 * Errors: EINVAL (bad pointers, nsteps < 0, non-finite dt, bad params),
 * ENOMEM, EDEVICE. */
int tfmm_leapfrog(tfmm_tree *tree, const tfmm_params *params, double *pos, double *vel,
                  const double *mass, double *force, double dt, int nsteps, int force_valid,
                  void *stream);

/* Momentum diagnostics in FP64 (Eqs. netforce, total_torque summed over all
 * particles, about the system centre of mass).  pos, mass, force: device, as
 * above; vel: device n x 3 or NULL.  out: host, 20 doubles:
 *   [0..2] sum F, [3] sum |F|, [4..6] sum (X - Xcm) x F, [7] sum |X - Xcm||F|,
 *   [8..10] P = sum m v, [11..13] L = sum m (X - Xcm) x v, [14] sum m,
 *   [15..17] Xcm, [18] |sum F| / sum |F|, [19] |sum (X-Xcm) x F| / sum |X-Xcm||F|.
 * Deterministic fixed-order reduction.  Synchronising.  Errors: EINVAL, EDEVICE. */
int tfmm_momentum_diagnostics(tfmm_ctx *ctx, int64_t n, const double *pos, const double *vel,
                              const double *mass, const double *force, void *stream, double *out);

/* tfmm_momentum_diagnostics without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops): the
 * same kernels and the same 20 values, written asynchronously to out (device,
 * 20 FP64, caller-owned) on `stream`; no synchronisation, no hipMalloc, no
 * memset.  The partial sums live in a fixed static device array of 82 KiB per
 * GPU (set up when the first context is created on that GPU, held until the
 * process ends) that every call on that GPU shares: calls that overlap on one
 * GPU (different streams, or different host threads) race and must be
 * serialised by the caller.  Nothing in it has to start at zero.  Limit:
 * 1 <= n <= 2^30.  Errors: EINVAL (n out of range, NULL pos, mass, force or
 * out), EDEVICE. */
int tfmm_momentum_diagnostics_noalloc(tfmm_ctx *ctx, int64_t n, const double *pos, const double *vel,
                                      const double *mass, const double *force, double *out, void *stream);

/* Sizes of a tree: out[0] n, [1] nodes, [2] leaves, [3] deepest level,
 * [4] far (M2L) unordered pairs, [5] near (P2P) unordered pairs, [6] directed
 * near particle interactions (sum over directed leaf pairs of n_target *
 * n_source, self pairs n(n-1)), [7] directed far pairs.  [4..7] are -1 before
 * the first walk.  Host output.  [6] is counted on the device on the first
 * request after a walk; that request waits for the device to be idle.
 * Errors: EINVAL, EDEVICE. */
int tfmm_tree_info(const tfmm_tree *tree, int64_t *out);

/* Copy the tree to host buffers (each may be NULL; caller-allocated):
 * keys: n uint64 in original particle order; order: n int32, sorted position
 * -> original index; and per node (sizes from tfmm_tree_info): level (int32),
 * prefix (uint64, key >> 3(21 - level)), first / count (int32, sorted range),
 * child_first (int32, -1 for leaves), nchild (int32), parent (int32, -1 for
 * the root), com (3 FP64 per node), mass (FP64), rmax (FP64).  Synchronising.
 * Errors: EINVAL, EDEVICE. */
int tfmm_tree_export(tfmm_tree *tree, uint64_t *keys, int32_t *order, int32_t *level,
                     uint64_t *prefix, int32_t *first, int32_t *count, int32_t *child_first,
                     int32_t *nchild, int32_t *parent, double *com, double *mass, double *rmax);

/* Copy the last walk's unordered pairs to host buffers (int32 pairs, lower
 * node index first, in the walk's emission order): far (M2L) and near (P2P,
 * self pairs (L, L) included).  Synchronising.  Errors: EINVAL, ESTATE (no
 * walk yet), EDEVICE. */
int tfmm_lists_export(tfmm_tree *tree, int32_t *m2l_pairs, int32_t *p2p_pairs);

/* Destroy a tree and release its device memory.  Synchronises the device.
 * NULL is ignored. */
int tfmm_tree_destroy(tfmm_tree *tree);

/* Estimate of the device bytes a tree of n particles at order p needs (for
 * admission control; a forest: n = all its particles).  The interaction
 * lists grow as theta falls: on the serving workloads (theta >= 0.4, Plummer,
 * ball and disk sets) a fresh tree holds at most 0.9 of it.  A tree reused
 * for another particle set keeps its grow-only buffers, so it can hold more.
 * Pure host computation. */
size_t tfmm_footprint_bytes(int64_t n, int p, int n_leaf, int precision);

/* Per-phase device times (milliseconds), averaged over the evaluations
 * (tfmm_evaluate_forces) and rebuilds (tfmm_tree_rebuild) run on this tree
 * since timing was last switched on or off with tfmm_tree_set_timing, which
 * also clears the averages.  Measured with HIP events on the stream each
 * phase runs on.  out: host, 10 doubles: [0] M2L, [1] P2P, [2] L2L, [3] L2P,
 * [4] moments (moments, M2L and L2L run on the tree's second stream beside
 * P2P, which runs on the caller's; L2P runs on the caller's stream after the
 * two join), [5] whole evaluation (including a walk if one was needed),
 * [6] rebuild (keys, sort, octree, geometry; 0 if no timed rebuild),
 * [7] walk (frontier passes and both list chains, averaged over the timed
 * evaluations that walked; 0 if none), [8] the walk's frontier passes alone,
 * [9] the interaction pass: from the first start to the last end of P2P and
 * M2L, which run side by side.
 * While timing is on, each evaluation records up to eleven events and each
 * rebuild two; an evaluation reads the previous evaluation's times and a
 * rebuild the previous rebuild's.  tfmm_tree_phase_times synchronises with
 * the last timed evaluation and rebuild.  Errors: EINVAL, ESTATE (no timed
 * evaluation), EDEVICE. */
int tfmm_tree_set_timing(tfmm_tree *tree, int enable);
int tfmm_tree_phase_times(tfmm_tree *tree, double *out);

#ifdef __cplusplus
}
#endif

#endif /* TFMM_H */
