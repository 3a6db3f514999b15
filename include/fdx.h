/*
 * fdx.h -- C ABI of the MI355X (gfx950) Barnes-Hut gravity library.
 *
 * The calls follow the way Iwasawa et al. ("Implementation and Performance of FDPS",
 * section "An example -- gravitational N-body problem") state a gravitational N-body
 * problem: initialise, hand over the particles, build the tree, compute the long-range
 * force from particles (EPJ) and superparticles (SPJ) under an opening angle theta, and
 * advance the particles with the leapfrog of the sample program; then finalise.  The
 * interaction is fixed to softened Newtonian gravity with G = 1:
 *   a_i   = sum_j m_j (r_j - r_i) / (|r_j - r_i|^2 + eps_i^2)^{3/2}      (j != i)
 *   phi_i = -sum_j m_j / (|r_j - r_i|^2 + eps_i^2)^{1/2}                  (j != i)
 * approximated by the tree (equations ParticleParticleNbody, ParticleSuperparticleNbody
 * and geqL), with superparticles up to the quadrupole moment.
 *
 * Conventions for every call:
 *   - returns FDX_OK (0) on success or a negative FDX_E* code; no C++ exception crosses
 *     this boundary (a host allocation failure inside a call returns FDX_ENOMEM, any other
 *     exception FDX_EINVAL); fdx_last_error() then holds a message for that context;
 *   - all GPU work is issued on the stream bound at fdx_create, in order, asynchronously;
 *     calls that return data to host memory synchronise that stream first;
 *   - the library owns its tree, list and scratch buffers (device memory it allocates);
 *     the caller owns every pointer it passes;
 *   - particle arrays are structure-of-arrays FP64 of length n; several independent systems
 *     may be laid end to end (sys_off), and particles never interact across systems;
 *   - results are deterministic: the same input gives bit-identical keys, cells, lists and
 *     forces on every run;
 *   - one context must not be used from two host threads at once.
 */
#ifndef FDX_H
#define FDX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdx_ctx fdx_ctx;

/* status codes */
#define FDX_OK 0
#define FDX_EINVAL -1   /* an argument is out of range, null or non-finite */
#define FDX_ENOMEM -2   /* a device or host allocation failed */
#define FDX_EHIP -3     /* a HIP runtime call failed, or a kernel reported an error */
#define FDX_ESTATE -4   /* calls made in the wrong order (e.g. force before particles) */

/* where a pointer lives */
#define FDX_MEM_HOST 0
#define FDX_MEM_DEVICE 1

/* fdx_calc_force / fdx_integrate flags (bitwise or) */
#define FDX_QUAD 1        /* superparticles carry the quadrupole moment (else monopole) */
#define FDX_FP32REL 2     /* FP32 force kernels on group-relative coordinates with
                             compensated accumulation (else FP64 kernels); a group too wide
                             for that -- 9 u min(S / eps_min, 2^d) > 1e-4 with u = 2^-24,
                             S its cell side, eps_min its smallest softening, d the depth of
                             its deepest leaf below its cell -- is evaluated in FP64 */
#define FDX_PREDICTOR 4   /* size interaction lists from the learned list-length predictor
                             (single walk; overflowing groups are re-walked exactly, so
                             forces never depend on it) */
#define FDX_PERSISTENT 8  /* one persistent force launch: the groups, in tree order, are cut
                             into one contiguous queue per XCD; a workgroup pops its own
                             XCD's queue, then takes slots from the others' */
#define FDX_GRAPH 16      /* fdx_integrate: capture one step as a HIP graph and replay it */
#define FDX_TIMING 32     /* record per-phase times (fdx_get_stats) */
#define FDX_FUSED 64      /* walk and force in one persistent launch (the paper's multiwalk,
                             section "Design concept of FDPS"): each wave pops a group, walks
                             the tree for it and evaluates the entries in tiles of 64 as the
                             walk emits them, so no interaction list is stored (lists and the
                             opening test are those of the separate walk; forces agree within
                             rounding).  The groups, in tree order, are cut into one queue per
                             XCD at equal cumulative cost: members x the learned predictor's
                             list length with FDX_PREDICTOR (nothing precedes the kernel that
                             knows the lengths), else members.  n_group <= 256; FDX_PERSISTENT
                             is implied.  fdx_get_lists returns the counts only unless
                             fdx_set_list_capture is on. */

/* Create a context on HIP device `device`, issuing work on `hip_stream` (a hipStream_t;
 * NULL = the library creates its own stream).  Corresponds to FDPS's Initialize.
 * *out receives the handle.  FDX_EINVAL if out is null or the device does not exist. */
int fdx_create(fdx_ctx **out, int device, void *hip_stream);

/* Free every buffer the library owns and the handle.  Corresponds to FDPS's Finalize.
 * A null ctx is accepted and ignored. */
int fdx_destroy(fdx_ctx *ctx);

/* Hand over n particles (the ParticleSystem of the sample program): positions x,y,z,
 * velocities vx,vy,vz and masses m, each an FP64 array of length n; eps = per-particle
 * softening (length n, or null to use the eps argument of fdx_calc_force); sys_off = n_sys+1
 * ascending int64 offsets that split [0, n) into independent systems (null with n_sys = 1
 * for a single system).
 * mem_kind FDX_MEM_HOST: the arrays are copied to device memory before the call returns.
 * mem_kind FDX_MEM_DEVICE: the arrays are device pointers that the library borrows: it
 *   reads them, and fdx_integrate updates x..vz in place; the caller keeps them alive and
 *   unchanged by others until fdx_destroy or the next fdx_set_particles.  sys_off is always
 *   a host pointer.
 * Masses must be finite and >= 0, eps finite and > 0 (checked on the host for host memory
 * and on the device, reported by the next fdx_calc_force, for device memory).  When all eps
 * of each system are one value (checked once here), evaluations take it from the system's
 * first particle instead of reading the array per particle; the results are the same.
 * FDX_EINVAL: n < 0, n >= 2^31, a null array, n_sys < 1, offsets not ascending from 0 to n,
 * or an invalid value. */
int fdx_set_particles(fdx_ctx *ctx, int64_t n, const double *x, const double *y,
                      const double *z, const double *vx, const double *vy, const double *vz,
                      const double *m, const double *eps, const int64_t *sys_off,
                      int32_t n_sys, int32_t mem_kind);

/* Build the tree of the current positions: root cube and 63-bit Morton keys per system,
 * stable radix sort by (system, key), octree cells (split while a cell holds more than
 * n_leaf particles, up to level 21), multipole moments up to the quadrupole, and i-particle
 * groups (maximal cells of at most n_group particles; modified tree algorithm, section
 * "Tree traverse and interaction calculation").  fdx_calc_force does this itself; this call
 * exists to inspect or time the tree alone.  FDX_EINVAL: n_leaf < 1 or n_group < 1;
 * FDX_ESTATE: no particles. */
int fdx_build_tree(fdx_ctx *ctx, int32_t n_leaf, int32_t n_group);

/* One force evaluation (calcForceAllAndWriteBack of the sample program): rebuilds the tree,
 * walks each group from its system's root with opening angle theta (a cell of side S whose
 * centre lies at distance D from the group's box is a superparticle iff S^2 < theta^2 D^2,
 * otherwise it is opened; opened leaves give particles), and evaluates accelerations and
 * potentials.  Results stay in device memory in the caller's original particle order
 * (fdx_get_forces).  eps is the softening used when fdx_set_particles got no eps array.
 * flags: FDX_QUAD, FDX_FP32REL, FDX_PREDICTOR, FDX_PERSISTENT, FDX_TIMING.
 * FDX_EINVAL: theta not in (0, 1], n_leaf < 1, n_group < 1 or > 512, eps not finite > 0
 * when it is used, or non-finite particle data; FDX_ESTATE: no particles. */
int fdx_calc_force(fdx_ctx *ctx, double theta, int32_t n_leaf, int32_t n_group, double eps,
                   int32_t flags);

/* Advance n_steps leapfrog steps of size dt (predict: v += dt/2 a, x += dt v; force;
 * correct: v += dt/2 a), with the theta, n_leaf, n_group, eps and flags of the last
 * fdx_calc_force (or fdx_calc_force_cutoff), which must have been called first (the sample
 * program evaluates the force once before its loop); fdx_build_tree, fdx_calc_density,
 * fdx_build_exchange_lists and fdx_autotune in between do not change them.  flags may add
 * FDX_GRAPH: the step is captured once as a HIP graph and replayed.  FDX_ESTATE: no prior
 * force evaluation; FDX_EINVAL: dt not finite or n_steps < 0. */
int fdx_integrate(fdx_ctx *ctx, double dt, int32_t n_steps, int32_t flags);

/* List sizing of FDX_GRAPH steps with several systems.  A group's list has at most as many
 * entries as its system has particles (its entries cover disjoint sets of them), so the
 * captured step can size every group's list segment by its system, min(particles of the
 * system, percent / 100 x the longest list the system had in the evaluation before the
 * capture + 64), and fill the lists in one walk, without a count walk, when all segments fit
 * a 16 GiB budget.  A list that outgrows its segment is moved to the buffer's spare quarter
 * inside the walk (fdx_stats.list_spills); a replay where that space ran out is redone
 * eagerly (fdx_stats.graph_recoveries) and the percentage doubles for the next capture.
 * percent = 0 sizes the segments by a count walk in every step.  Default 200.  FDX_EINVAL:
 * percent < 0. */
int fdx_set_graph_list_margin(fdx_ctx *ctx, int32_t percent);

/* List capture for FDX_FUSED evaluations (for checks): when on, an eager FDX_FUSED evaluation
 * first sizes every group's list by a counting walk and the fused kernel also writes the
 * entries it evaluates into them, so fdx_get_lists returns them (graph-captured steps never
 * capture).  Default off. */
int fdx_set_list_capture(fdx_ctx *ctx, int32_t on);

/* Copy positions and velocities (caller's order) into x..vz (length n each, memory of
 * kind mem_kind).  Any pointer may be null to skip that array. */
int fdx_get_particles(fdx_ctx *ctx, double *x, double *y, double *z, double *vx, double *vy,
                      double *vz, int32_t mem_kind);

/* Copy the last forces (caller's order) into ax, ay, az, pot (length n each; null skips).
 * FDX_ESTATE if no force has been evaluated. */
int fdx_get_forces(fdx_ctx *ctx, double *ax, double *ay, double *az, double *pot,
                   int32_t mem_kind);

/* Sizes and counters of the last tree / force evaluation. */
typedef struct {
    int64_t n, n_sys;
    int64_t n_cells, n_groups, depth;
    int64_t n_epj, n_spj;              /* list entries summed over groups */
    int64_t n_interactions_pp;         /* sum over groups of n_i * |EPJ| (self pairs included) */
    int64_t n_interactions_pc;         /* sum over groups of n_i * |SPJ| */
    int64_t overflow_groups;           /* predictor path: groups whose list outgrew its
                                          predicted capacity (walked again in spare space, or
                                          re-walked exactly by a second pass) */
    int64_t list_capacity;             /* list entries allocated in the last walk */
    int32_t n_leaf, n_group, flags;
    int32_t shape;                     /* force-kernel shape used (see fdx_autotune_shapes) */
    double theta;
    /* phase times in milliseconds (FDX_TIMING): keys, sort, tree, moments, groups, walk,
       force, unsort, predict, total; with FDX_PREDICTOR, predict = features, network and
       capacities and walk = the walk after them (predict = 0 otherwise); with FDX_FUSED,
       predict = features, network and queue boundaries, walk = 0 and force = the one
       walk + force launch */
    double t_keys, t_sort, t_tree, t_moments, t_groups, t_walk, t_force, t_unsort, t_predict,
        t_total;
    /* FP32 evaluations: groups evaluated by the FP64 kernel instead, because FP32 rounding of
       coordinates relative to the group centre could move a close pair's force by more than
       1e-4 of itself (see FDX_FP32REL) */
    int64_t fp64_groups;
    int64_t graph_recoveries;   /* graph-replayed steps redone eagerly (a capacity overflowed) */
    int64_t list_spills;        /* lists that outgrew a predicted or per-system segment and were
                                   moved to the list buffer's spare space inside the walk
                                   (cumulative over the context) */
} fdx_stats;

int fdx_get_stats(fdx_ctx *ctx, fdx_stats *out);

/* Debug views for parity checks (host memory, sizes from fdx_get_stats; null skips).
 * cube[4 s] = {origin x, y, z, side} of system s; key[r] and perm[r] = key and original
 * index of the particle at sorted rank r; cell arrays in breadth-first order;
 * mom[10 c] = {M, X, Y, Z, Qxx, Qyy, Qzz, Qxy, Qxz, Qyz}. */
int fdx_get_tree(fdx_ctx *ctx, double *cube, uint64_t *key, uint32_t *perm, int32_t *level,
                 uint64_t *prefix, uint32_t *begin, uint32_t *count, uint32_t *first_child,
                 uint32_t *nchild, uint32_t *parent, double *mom);

/* Groups in ascending order of their first sorted particle: cell, begin, count, integer
 * box qmin[3 g], qmax[3 g] (grid units) and the geometric centre of the group's cell. */
int fdx_get_groups(fdx_ctx *ctx, uint32_t *cell, uint32_t *begin, uint32_t *count,
                   uint32_t *qmin, uint32_t *qmax, double *centre);

/* Interaction lists of the last walk: n_epj[g], n_spj[g]; epj = the EPJ entries (sorted
 * particle ranks) of all groups concatenated, spj = the SPJ entries (cell ids) likewise
 * (each group's entries in the library's emission order).  Null epj and spj copy the
 * counts only. */
int fdx_get_lists(fdx_ctx *ctx, uint32_t *n_epj, uint32_t *n_spj, uint32_t *epj,
                  uint32_t *spj);

/* ---- Autotuner (n_group and force-kernel workgroup shape) ----------------------------
 * The paper finds an optimal group size from the trade-off between list construction and
 * force cost (section "Tree traverse and interaction calculation"); the autotuner measures
 * it instead.  fdx_autotune_shapes() = number of force-kernel shapes (threads per workgroup x
 * i-particles per thread x j-entries per LDS tile, with or without the next tile's loads issued
 * early; the name gives each: nt512_ipl1_w8_jt128 = 512 threads, one i-particle per thread,
 * 8 waves per SIMD, tiles of 128 entries; without _jt the tile is the workgroup size).
 * fdx_autotune times fdx_calc_force (median of `reps` calls after
 * one warm-up) for each of the n_cand candidate group sizes and every shape that can hold
 * them, keeps the fastest shape for later calls of the same precision (FDX_FP32REL set or
 * not in `flags`; the other precision keeps its shape) and returns it with its group size;
 * times_ms[k * shapes + v] receives each time (NaN where the shape cannot hold the group
 * size; null skips).  With FDX_GRAPH in `flags` it times graph-captured leapfrog steps of
 * dt = 0 (which leave the particles unchanged) instead of eager evaluations, with the
 * persistent kernel.  Shapes whose kernel spills registers to scratch memory are not timed
 * (NaN) when a shape that does not spill can hold the group size.  When the context had a
 * force evaluation before the call, it is evaluated again at the end with its own
 * parameters (and the chosen shape), so forces, lists and the parameters of fdx_integrate
 * are the caller's; otherwise the context is left without a force.
 * fdx_set_shape fixes the shape of both precisions (-1 = default).
 * FDX_EINVAL: no candidates, reps < 1, or a shape out of range. */
int fdx_autotune_shapes(void);
const char *fdx_shape_name(int32_t shape);   /* e.g. "nt512_ipl1_pf"; "" if out of range */
int fdx_set_shape(fdx_ctx *ctx, int32_t shape);
int fdx_autotune(fdx_ctx *ctx, double theta, int32_t n_leaf, double eps, int32_t flags,
                 const int32_t *n_group_cand, int32_t n_cand, int32_t reps, double *times_ms,
                 int32_t *best_n_group, int32_t *best_shape);
/* fdx_autotune_cached: the same search, with its result recorded in the text file `path`
 * (one JSON object per line: {"key": "...", "n_group": g, "shape": v}); the key holds the
 * device architecture, floor(log2 n), floor(log2 n_sys), theta, n_leaf, the QUAD / FP32REL /
 * PERSISTENT / GRAPH flags, the candidate list and reps.  A recorded key is applied without timing
 * (*from_cache = 1: the shape is kept for later calls and the group size returned); otherwise
 * fdx_autotune runs and one line is appended (*from_cache = 0).  Lines that do not parse, or
 * name a shape that cannot hold their group size, are ignored.  FDX_EINVAL: null path, no
 * candidates, reps < 1, or the file cannot be written; FDX_ESTATE: no particles. */
int fdx_autotune_cached(fdx_ctx *ctx, const char *path, double theta, int32_t n_leaf,
                        double eps, int32_t flags, const int32_t *n_group_cand, int32_t n_cand,
                        int32_t reps, int32_t *best_n_group, int32_t *best_shape,
                        int32_t *from_cache);

/* ---- Learned interaction-list length predictor -----------------------------------------
 * A small network (8 inputs -> 64 -> 64 -> 1, SiLU, FP32; fdx_mlp_params() = 4801 weights)
 * predicts ln(|EPJ| + |SPJ|) of each group from cheap group features, so FDX_PREDICTOR can
 * size every list before one single walk (a closed-form model of the mean length is the
 * paper's equation nlist_long).  Lists that outgrow their predicted capacity are walked
 * again exactly, so forces never depend on the predictor.  All arrays are host memory.
 * fdx_predictor_features: raw features of every group of the last tree, X[8 g + k]:
 *   ln n_i, ln box extent, ln(1 + distance of the box centre to the root centre), ln(parent
 *   mass / system mass), ln(parent side / root side), depth, ln(parent density), log2 N_sys.
 * fdx_mlp_forward / fdx_mlp_grad: the network's forward pass and the full-batch gradient of
 *   the mean squared error on given weights P[4801] and standardised inputs (for checks).
 * fdx_mlp_adam: n_steps steps of the training's Adam kernel (Kingma & Ba, beta1 0.9, beta2
 *   0.999, eps 1e-8, learning rate lr) on P, m, v (4801 each, updated in place) with the
 *   gradient grads[4801 k ...] at step number step0 + k + 1 (for checks).
 * fdx_predictor_train: trains on n samples (raw features, ln length) with the library's own
 *   forward/backward/Adam kernels: seeded 90/10 split, standardisation from the training
 *   part, `epochs` passes of minibatches of `batch`, learning rate lr; the capacity margin is
 *   the 99th percentile of the held-out residual; losses[e] = mean loss of epoch e.
 * fdx_predictor_margin: set the margin (ln factor; NaN keeps it) and read it back.
 * fdx_predictor_save / load: weights, normalisation and margin to / from a binary file.
 * FDX_ESTATE: predictor not trained or loaded (margin, save, FDX_PREDICTOR). */
int fdx_mlp_params(void);
int fdx_predictor_features(fdx_ctx *ctx, float *X);
int fdx_mlp_forward(fdx_ctx *ctx, const float *P, const float *X, int64_t n, float *y);
int fdx_mlp_grad(fdx_ctx *ctx, const float *P, const float *X, const float *t, int64_t n,
                 float *grad, float *loss);
int fdx_mlp_adam(fdx_ctx *ctx, float *P, float *m, float *v, const float *grads, int32_t n_steps,
                 int32_t step0, double lr);
int fdx_predictor_train(fdx_ctx *ctx, const float *X, const float *t, int64_t n, int32_t epochs,
                        int32_t batch, double lr, int64_t seed, float *losses);
int fdx_predictor_margin(fdx_ctx *ctx, double margin, double *out);
int fdx_predictor_save(fdx_ctx *ctx, const char *path);
int fdx_predictor_load(fdx_ctx *ctx, const char *path);

/* ---- Tree part of TreePM -----------------------------------------------------------------
 * The paper's cosmological run splits gravity into a mesh part and a tree part with a
 * monopole-only kernel and a cutoff of three mesh widths, with the S2 cloud profile of
 * Hockney & Eastwood (section "Cosmological simulation").  fdx_calc_force_cutoff evaluates
 * the tree part: cells whose cube lies farther than r_cut from a group's box are dropped, the
 * rest follow the opening angle theta, superparticles are monopoles, and every pair force is
 * Newton's times g(2 r / r_cut), the complement of the force between two S2 clouds of
 * diameter r_cut (g = 1 at r = 0, 0 for r >= r_cut; r unsoftened, eps_i in the Newtonian
 * factor).  The potential is not computed (returned as 0).  Same arguments as fdx_calc_force
 * plus r_cut (finite > 0); flags: FDX_FP32REL, FDX_PERSISTENT, FDX_TIMING.  fdx_integrate then
 * steps with this force (not with FDX_GRAPH).  FDX_EINVAL: r_cut, FDX_QUAD, FDX_PREDICTOR or
 * FDX_GRAPH, or a parameter fdx_calc_force rejects. */
int fdx_calc_force_cutoff(fdx_ctx *ctx, double theta, int32_t n_leaf, int32_t n_group, double eps,
                          double r_cut, int32_t flags);

/* ---- Exchange lists between domains ----------------------------------------------------
 * Before the force step every process sends every other process the particles and
 * superparticles it needs, found by the usual tree traversal of its own local tree with the
 * fixed opening angle theta (section "Exchange of particles and superparticles", long-range
 * mode; the total length per domain is modelled by equation n_list_long).  Here the domains
 * are the systems of the particle set (sys_off), each with its own local tree, as virtual
 * processes on one GPU.  The receiving domain enters the traversal as the exact bounding box
 * of its particles mapped into the sender's integer grid (floor((x - o) * 2^21 / Lr) per
 * axis, clamped to [-2^24, 2^24]); a cell of side S whose centre lies at distance D from that
 * box is sent as a superparticle iff S^2 < theta^2 D^2, otherwise opened, and an opened leaf
 * sends its particles.  Pairs (sender s, receiver r != s) are ordered by sender, then
 * receiver: pair k = s * (n_sys - 1) + (r < s ? r : r - 1).
 * fdx_build_exchange_lists: builds the local trees (keys, sort, cells, moments) and every
 *   pair's list; theta in (0, 1], n_leaf >= 1.  FDX_EINVAL: fewer than two domains, an empty
 *   domain or a parameter out of range; FDX_ESTATE: no particles.
 * fdx_get_exchange_counts: n_epj[s * n_sys + r], n_spj[s * n_sys + r] (host, n_sys^2 each,
 *   zero on the diagonal; null skips).
 * fdx_get_exchange_lists: all pairs' entries concatenated in pair order (host memory):
 *   epj = caller's particle indices, spj = cell ids of fdx_get_tree (whose mom rows are the
 *   superparticles), each pair's entries in an order of the library's choosing (null
 *   skips).
 * fdx_get_exchange_stats: sizes, list memory and the device time of the two parts.
 * The getters return FDX_ESTATE if no lists were built since the last fdx_set_particles. */
typedef struct {
    int64_t n_domains, n_pairs;
    int64_t n_epj, n_spj;              /* entries over all pairs */
    int64_t list_capacity;             /* entries allocated: (n_sys - 1) n, the per-sender
                                          bound, while that fits 16 GiB (one fill walk);
                                          else the exact total from a count walk */
    double ms_tree;                    /* keys, sort, cells and moments of all local trees */
    double ms_lists;                   /* pair boxes, count walk, offsets, fill walk */
} fdx_exchange_stats;

int fdx_build_exchange_lists(fdx_ctx *ctx, double theta, int32_t n_leaf);
int fdx_get_exchange_counts(fdx_ctx *ctx, uint32_t *n_epj, uint32_t *n_spj);
int fdx_get_exchange_lists(fdx_ctx *ctx, uint32_t *epj, uint32_t *spj);
int fdx_get_exchange_stats(fdx_ctx *ctx, fdx_exchange_stats *out);

/* ---- Short-range neighbour lists and SPH density ---------------------------------------
 * The same tree is traversed for short-range interactions with four kinds of cutoff
 * (section "Interaction calculation"): fixed (pairs with r < r_cut), j-dependent
 * (FDX_CUT_SCATTER: r < h_j), i-dependent (FDX_CUT_GATHER: r < h_i) and symmetric
 * (r < max(h_i, h_j)); equation nlist_short models the list length.  For every group the walk
 * keeps the particles of each leaf whose cube lies within the search radius of the group's
 * box (r_cut, the group's largest h, the cell's largest h, or the larger of the two), and the
 * density kernel evaluates, for every particle,
 *   rho_i = sum_j m_j W(|r_ij|, H) over pairs with |r_ij| < H (j = i included),
 *   H = r_cut (fixed), h_j (scatter), h_i (gather); symmetric: the mean of the gather and
 *   the scatter sums; n_ngb_i = number of such j (symmetric: |r_ij| < max(h_i, h_j)),
 * with the Wendland C6 kernel of the paper's SPH application (section "Giant impact
 * simulation"), q = r/H < 1: W = 1365/(64 pi H^3) (1-q)^8 (1 + 8q + 25q^2 + 32q^3).  FP64;
 * neighbour counts are exact.
 * fdx_calc_density: mode FDX_CUT_*; r_cut (fixed mode, finite > 0); h = support radius of
 *   every particle, caller's order, length n, in host or device memory (mem_kind; ignored in
 *   fixed mode); n_leaf, n_group as for the tree; flags: FDX_TIMING (phase times in
 *   fdx_get_stats: t_walk = walk, t_force = density).  The candidate lists stay readable with
 *   fdx_get_lists (no superparticles).  FDX_EINVAL: bad mode, r_cut, h (null, non-positive or
 *   non-finite), n_leaf or n_group; FDX_ESTATE: no particles.
 * fdx_get_density: rho and n_ngb (length n each, caller's order, null skips).  FDX_ESTATE if
 *   none was computed since the last fdx_set_particles. */
#define FDX_CUT_FIXED 0
#define FDX_CUT_SCATTER 1
#define FDX_CUT_GATHER 2
#define FDX_CUT_SYMMETRIC 3
int fdx_calc_density(fdx_ctx *ctx, int32_t mode, double r_cut, const double *h, int32_t mem_kind,
                     int32_t n_leaf, int32_t n_group, int32_t flags);
int fdx_get_density(fdx_ctx *ctx, double *rho, uint32_t *n_ngb, int32_t mem_kind);

/* ---- Domain decomposition: multisection with cost-weighted sampling ---------------------
 * Section "Domain decomposition": the domains are n_x n_y n_z boxes found by dividing once
 * per axis -- n_x slabs along x, each slab into n_y columns along y, each column into n_z
 * domains along z -- so that sample particles are equally divided; each current domain (a
 * system of the particle set, standing in for a process) samples its own particles at a rate
 * proportional to its cost per particle, so that every sample stands for the same work.
 * Then every particle is sent to the domain whose box holds it (the exchange of particles).
 *   Samples: current domain p with n_p particles draws
 *     k_p = floor(n_sample * T_p / sum_q T_q)   (FP64, the sum in domain order; 0 if n_p = 0)
 *   samples; T_p = cost[p] when given, else the count of members times list length summed
 *   over p's groups in the last walk (FDX_DD_COST_LISTS), else n_p (uniform sampling).
 *   Sample s (numbered over the domains in order) is particle
 *   off_p + floor(r_s n_p / 2^64), r_s = output number s of SplitMix64 seeded with seed.
 *   Division: each segment's samples sorted by coordinate (ties by sample number) are cut
 *   into n runs, run i = sorted ranks [floor(i m / n), floor((i+1) m / n)) of its m samples;
 *   a cut lies at the midpoint (a + b) * 0.5 of the samples on either side; the outer faces
 *   are -inf and +inf.  Domain (ix, iy, iz) is number (ix n_y + iy) n_z + iz and holds the
 *   particles with bx[ix] <= x < bx[ix+1], by[ix][iy] <= y < by[ix][iy+1],
 *   bz[ix][iy][iz] <= z < bz[ix][iy][iz+1].
 *   Exchange: the new order lists the particles grouped by destination, within one
 *   destination in their current order (that is, by source domain, then position).
 * fdx_dd_factor: (n_x, n_y, n_z) for n domains, integers close to n^(1/3): among the
 *   factorisations n_x >= n_y >= n_z, the smallest n_x - n_z, then the smallest n_x - n_y.
 *   Host only.  FDX_EINVAL: n < 1 or a null pointer.
 * fdx_decompose: n_x, n_y, n_z >= 1; n_sample in [1, 2^31); cost = host array of n_sys
 *   finite non-negative values or null; flags FDX_DD_COST_LISTS (needs cost == null and a walk
 *   on the current particles).  Work is enqueued on the stream (FDX_DD_COST_LISTS reads the
 *   costs back first).  FDX_EINVAL: a size out of range, more than 2^24 (source, destination)
 *   pairs, a bad cost, a zero total cost, or fewer samples than domains; FDX_ESTATE: no
 *   particles, or no walk for FDX_DD_COST_LISTS.
 * fdx_get_decomposition: faces bx[n_x+1], by[n_x][n_y+1], bz[n_x][n_y][n_z+1], the send
 *   counts [source p][destination d] (n_sys x n_domains) and the new domain offsets
 *   dom_off[n_domains+1]; host memory, null skips.
 * fdx_get_dd_samples: k_p per current domain (n_sys), the particle of every sample and the
 *   domain its division put it in (K = sum k_p each; fdx_get_dd_stats gives K); host, null
 *   skips.
 * fdx_get_dd_destinations: dest[i] for every particle (current order) and order[r] = the
 *   current index of the particle at new position r (length n each), host or device memory.
 * fdx_exchange_particles: applies the last decomposition: the context's particles are
 *   reordered into the new order on the device (into library-owned memory, also when they
 *   were borrowed) and the domains become the systems (n_sys = n_domains, sys_off =
 *   dom_off).  Afterwards every getter's "caller's order" is the new order; earlier forces
 *   and lists are dropped.
 * fdx_get_dd_stats: sizes, n_moved = particles whose destination number differs from their
 *   current domain number, and the device time of each part.
 * The getters and fdx_exchange_particles return FDX_ESTATE without a decomposition of the
 * current particles (fdx_set_particles drops it; the exchange keeps it readable). */
#define FDX_DD_COST_LISTS 1
typedef struct {
    int32_t nx, ny, nz, n_domains, n_src;
    int64_t n_samples;                 /* K */
    int64_t n_moved;
    double ms_sample;                  /* costs (if from lists), samples */
    double ms_divide;                  /* three sorts of the samples and their cuts */
    double ms_assign;                  /* destinations, partition sort, send counts */
    double ms_exchange;                /* reorder of the particle arrays (0 if not applied) */
} fdx_dd_stats;

int fdx_dd_factor(int32_t n, int32_t *nx, int32_t *ny, int32_t *nz);
int fdx_decompose(fdx_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int64_t n_sample,
                  const double *cost, uint64_t seed, int32_t flags);
int fdx_get_decomposition(fdx_ctx *ctx, double *bx, double *by, double *bz,
                          int64_t *send_counts, int64_t *dom_off);
int fdx_get_dd_samples(fdx_ctx *ctx, int64_t *k_per_domain, uint32_t *sample_idx,
                       uint32_t *sample_domain);
int fdx_get_dd_destinations(fdx_ctx *ctx, uint32_t *dest, uint32_t *order, int32_t mem_kind);
int fdx_exchange_particles(fdx_ctx *ctx);
int fdx_get_dd_stats(fdx_ctx *ctx, fdx_dd_stats *out);

/* ---- Direct summation (the reference for the tree's error) -----------------------------
 * The exact quantity the tree approximates, equation ParticleParticleNbody (section "An
 * example -- gravitational N-body problem") with G = 1, for selected target particles:
 *   a_i   =  sum_{j != i} m_j (x_j - x_i) / (|x_j - x_i|^2 + eps_i^2)^{3/2}
 *   phi_i = -sum_{j != i} m_j / (|x_j - x_i|^2 + eps_i^2)^{1/2}
 * over the particles j of i's system, at the context's current positions, in FP64 with
 * compensated sums; O(n_targets x system size) work.
 * fdx_direct_forces: targets = host array of n_targets indices in [0, n) (caller's order);
 *   out = host array of 4 n_targets values (ax, ay, az, phi per target); eps = the softening
 *   when the particles carry none (finite, > 0; ignored otherwise).  Synchronous.
 *   FDX_EINVAL: n_targets outside [0, 2^24], a null pointer, an index out of range or a bad
 *   eps; FDX_ESTATE: no particles. */
int fdx_direct_forces(fdx_ctx *ctx, const int64_t *targets, int64_t n_targets, double eps,
                      double *out);

/* ---- One force evaluation that allocates nothing ---------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid the allocator).  The same evaluation as fdx_calc_force on one
 * system, without a context: every buffer the library would own (keys, sort scratch, sorted
 * particles, cells, moments, groups, interaction lists, device status) is carved from one
 * 128 MiB array in device memory that the library declares statically; each device holds its
 * own copy from the first call on it until the process ends.  The call issues no device or
 * host allocation.
 * device: HIP device; hip_stream: the hipStream_t to work on (NULL: the null stream); the call
 *   returns after the evaluation finished on it.
 * x, y, z, m, eps (or null), ax, ay, az, pot: device arrays of length n (the caller owns them;
 *   eps null uses eps_all); results in the caller's order, as fdx_get_forces.
 * theta, n_leaf, n_group: as fdx_calc_force; flags: FDX_QUAD, FDX_FP32REL, FDX_PERSISTENT.
 * err (optional, err_len bytes): the message of a failure ("" on success).
 * Limits: n <= 131072 (2^17); the interaction lists get what the array has left after the
 * other buffers (about 80 MiB at n = 2^17, 2e7 entries).
 * Every call on a device shares its array and leaves its contents there: calls that overlap on
 * one device (two host threads, or two streams) race and must not be issued.
 * FDX_EINVAL: n outside [0, 2^17], other flags, a null array, a bad parameter (as
 * fdx_calc_force), or non-finite particle data; FDX_ENOMEM: the lists or cells do not fit the
 * array (nothing is allocated instead); FDX_EHIP: a HIP call failed. */
int fdx_calc_force_noalloc(int device, void *hip_stream, int64_t n, const double *x,
                           const double *y, const double *z, const double *m, const double *eps,
                           double eps_all, double theta, int32_t n_leaf, int32_t n_group,
                           int32_t flags, double *ax, double *ay, double *az, double *pot,
                           char *err, int32_t err_len);

/* Message of the last failed call on ctx (never null; "" when none). */
const char *fdx_last_error(const fdx_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* FDX_H */
