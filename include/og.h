/*
 * og.h — C ABI of the MI355X short-range TreePM tree force.
 *
 * The library builds an octree over particles in a (periodic) box and
 * evaluates, per target particle, the short-range part of the TreePM
 * gravitational force with a Barnes-Hut walk.  The operations follow the
 * paper's "Gravity Solver" section:
 *   - tree construction ("Tree construction": root cube covering the domain,
 *     recursive 8-way subdivision, particles in space-filling-curve order,
 *     bottom-up pass for node mass and centre of mass, two-pointer
 *     first-child/sibling traversal order);
 *   - tree walk ("Tree walk": one walk per target from the root, Barnes-Hut
 *     opening criterion plus a boundary check, accepted nodes act as a point
 *     mass at their centre of mass, the sibling pointer skips the subtree);
 *   - force evaluation ("Force evaluation" and "Particle Mesh": the tree
 *     carries the short-range term of the split 1/r = erfc(r/2A)/r +
 *     erf(r/2A)/r, A = r_s).
 * Where the paper leaves a choice open this library uses: Plummer softening
 * (r^2+eps^2)^(-3/2); 63-bit Morton keys; a cutoff r < r_cut with the
 * periodic minimum image; a node is skipped when on some axis its cube lies
 * farther than r_cut from the target; open iff side^2 > theta^2 |COM-x|^2 or
 * the target lies inside the node cube enlarged 1.2x; leaves hold up to
 * leaf_max particles.  Per target, acceleration
 *   a_i = sum_j G m_j d_ij (r^2+eps^2)^(-3/2) [erfc(u) + 2u/sqrt(pi) e^(-u^2)]
 *   phi_i = -sum_j G m_j erfc(u) / sqrt(r^2+eps^2),   u = r/(2 r_s),
 * summed over the particles and accepted nodes of the walk.
 *
 * Conventions for every call:
 *   - return value: OG_OK (0) or a negative OG_E* code; output handles are
 *     written only on success; nothing aborts or throws across the ABI;
 *     og_last_error() returns a thread-local detail string.
 *   - every array argument is a DEVICE pointer (HIP device memory) unless
 *     stated as host; a host pointer where a device one is required gives
 *     OG_EINVAL.
 *   - work is enqueued on the stream given in og_params.stream (a
 *     hipStream_t; NULL = the default stream).  Inputs must stay valid and
 *     unchanged until that stream has passed the call; outputs are valid
 *     once it has.  The tree copies what it needs and keeps no caller
 *     pointer beyond the call.
 *   - a built tree is read-only: og_tree_force calls on it may run
 *     concurrently on different streams; og_tree_free must not overlap any
 *     other use of the tree.
 */
#ifndef OG_H
#define OG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    OG_OK = 0,
    OG_EINVAL = -1,       /* invalid argument */
    OG_ERANGE = -2,       /* a position outside [0,box) (periodic) or not finite */
    OG_ENOMEM = -3,       /* device allocation failed or workspace too small */
    OG_EDEVICE = -4,      /* a HIP runtime error */
    OG_EBUSY = -5,        /* server: over budget and queue full */
    OG_EUNSUPPORTED = -6, /* valid request the library does not handle */
    OG_ENOTFOUND = -7,    /* server: unknown ticket */
    OG_ECORRUPT = -8      /* og_tree_validate: a tree invariant does not hold */
};

/* Arithmetic of the walk.  FP64: every step in double precision.  MIXED:
 * positions are turned into node-relative offsets in FP64 (at build time
 * for particles and node centres of mass, per target at walk start); the
 * opening tests and the interactions then run in FP32 on those offsets and
 * every contribution is accumulated per target in FP64. */
enum { OG_PREC_FP64 = 0, OG_PREC_MIXED = 1 };

/* Softening kernel (paper, "Force evaluation").  PLUMMER: the factors
 * (r^2+eps^2)^(-3/2) and (r^2+eps^2)^(-1/2).  SPLINE: the point mass is
 * spread with the cubic spline density of compact support h = 2.8 eps (eps
 * is the Plummer-equivalent length): with u = r/h,
 *   u < 1/2: 1/r^3 -> (32/3 - 192/5 u^2 + 32 u^3)/h^3,
 *            1/r   -> (14/5 - 16/3 u^2 + 48/5 u^4 - 32/5 u^5)/h,
 *   u < 1:   1/r^3 -> (64/3 - 48 u + 192/5 u^2 - 32/3 u^3 - 1/(15 u^3))/h^3,
 *            1/r   -> (16/5 - 1/(15 u) - 32/3 u^2 + 16 u^3 - 48/5 u^4
 *                      + 32/15 u^5)/h,
 *   u >= 1:  unsoftened.
 * The short-range factors (erfc split) multiply either kernel. */
enum { OG_SOFT_PLUMMER = 0, OG_SOFT_SPLINE = 1 };

/* Opening criterion for nodes beyond the boundary check (paper, "Tree
 * walk").  BH: open iff side^2 > theta^2 r^2.  RELATIVE: open iff
 * G M side^2 > alpha |a_old| r^4, with a_old the target's previous
 * acceleration (og_force_opts.a_old); r = |COM - x| (minimum image). */
enum { OG_OPEN_BH = 0, OG_OPEN_RELATIVE = 1 };

/* Space-filling curve of the particle order and of the children of every
 * node (paper, "Tree construction": insertion in Peano-Hilbert order).
 * MORTON: 63-bit key, bit 3b+2 = x bit b, 3b+1 = y, 3b = z.  HILBERT: the
 * cell coordinates are first mapped to the transposed Hilbert index
 * (Skilling 2004) and then interleaved the same way.  The nodes (cells) are
 * the same for both; only their order, hence the summation order, differs. */
enum { OG_CURVE_MORTON = 0, OG_CURVE_HILBERT = 1 };

/* Interaction lists (paper, "Neighbour search": nearby particles are grouped
 * and served by one search).  TARGET: every target follows its own walk;
 * the result does not depend on the grouping.  GROUP: one walk per group of
 * group_max consecutive targets in curve order; a node is pruned when it is
 * pruned for every target of the group, accepted for all when none of the
 * targets that keep it would open it, and opened otherwise; every target
 * then adds the same monopoles and leaf particles in traversal order, each
 * with its own cutoff and self test.  The result depends on the grouping
 * (more nodes opened: more interactions, smaller error). */
enum { OG_LISTS_TARGET = 0, OG_LISTS_GROUP = 1 };

typedef struct og_params {
    uint32_t struct_size;   /* = sizeof(og_params) (ABI check) */
    double G;               /* gravitational constant (default 1) */
    double eps;             /* Plummer softening length, >= 0 */
    double r_s;             /* split scale A_smth; <= 0: plain Newtonian force,
                               no cutoff (then periodic must be 0) */
    double r_cut;           /* cutoff radius; 0 => 4.5 r_s; periodic: < box/2 */
    double theta;           /* opening angle, >= 0 (0 opens every node) */
    double alpha;           /* relative criterion tolerance, > 0 when used */
    int32_t periodic;       /* 1: positions in [0,box)^3 with minimum image;
                               0: open boundaries, root = bounding cube */
    int32_t leaf_max;       /* max particles per leaf (default 8), 1..4096;
                               the result depends on it */
    int32_t precision;      /* OG_PREC_FP64 or OG_PREC_MIXED (default MIXED) */
    int32_t group_max;      /* targets per wavefront group, 1..64, 0 = 64;
                               the result does not depend on it (except
                               with OG_LISTS_GROUP) */
    int32_t walk_list_cap;  /* mixed walk: accepted partners buffered per
                               target before evaluation, 4, 8, 16 or 32; 0 =
                               default (4); the result does not depend on it */
    int32_t softening;      /* OG_SOFT_PLUMMER (default) or OG_SOFT_SPLINE
                               (needs eps > 0) */
    int32_t criterion;      /* OG_OPEN_BH (default) or OG_OPEN_RELATIVE */
    int32_t curve;          /* OG_CURVE_MORTON (default) or OG_CURVE_HILBERT */
    int32_t lists;          /* OG_LISTS_TARGET (default) or OG_LISTS_GROUP */
    const double *eps_particle; /* device [N] FP64, caller order: every
                               particle's own (Plummer-equivalent) softening
                               length, or NULL (all use eps).  A pair uses
                               the larger of its two lengths; a node's
                               monopole the larger of the target's and the
                               node's largest; a node holding different
                               lengths whose largest, e_max, exceeds the
                               target's is opened when the target lies
                               within 2.8 e_max of its centre of mass (the
                               paper's mixed-softening check, "Tree walk").
                               A length <= 0 or not finite gives OG_ERANGE
                               from og_tree_status.  Not with
                               OG_LISTS_GROUP (OG_EUNSUPPORTED). */
    void *stream;           /* hipStream_t, NULL = default stream */
    void *workspace;        /* optional caller device buffer for the tree */
    size_t workspace_bytes; /* its size; must be >= og_tree_workspace_bound */
} og_params;

/* Defaults: G 1, eps 0, r_s 0, r_cut 0, theta 0.5, alpha 0, periodic 1,
 * leaf_max 8, MIXED, group_max 0, walk_list_cap 0, PLUMMER, BH, MORTON,
 * TARGET lists, no stream, no workspace. */
void og_params_default(og_params *p);

/* Device bytes one tree over N particles needs (upper bound, independent of
 * the particle distribution); 0 for invalid arguments.  Used for HBM
 * admission before the build. */
size_t og_tree_workspace_bound(int64_t N, const og_params *p);

typedef struct og_tree og_tree;

/* Build the octree (keys, sort, topology, moments) of N particles.
 *   pos:  device, [N][3] FP64, row-major, caller order
 *   mass: device, [N] FP64, > 0
 *   box:  periodic box side (> 0); with periodic = 0 it is not used
 * Enqueued on params->stream; returns without waiting for the device.  A
 * periodic coordinate outside [0,box) (or a non-finite one) is found on the
 * device: the tree is then marked and og_tree_status reports OG_ERANGE;
 * the keys of such particles are clamped so that every kernel stays in
 * bounds.  Errors: OG_EINVAL (N < 1 or > 2^27-1, box <= 0, eps < 0,
 * theta < 0, leaf_max outside 1..4096, group_max outside 0..64,
 * walk_list_cap not 0, 4, 8, 16 or 32, periodic
 * with r_s <= 0 or r_cut >= box/2, unknown softening, criterion, curve or lists, SPLINE
 * with eps = 0, RELATIVE with alpha <= 0, null pointers, host pointers),
 * OG_ENOMEM, OG_EDEVICE. */
int og_tree_build(const double *pos, const double *mass, int64_t N, double box,
                  const og_params *params, og_tree **out);

/* Targets of a force evaluation: caller-order particle indices (device,
 * int64, each in [0,N); repeats allowed) or idx = NULL for all N particles
 * in caller order.  An index outside [0,N) is found on the device: its
 * entry receives particle 0's result, and the tree is marked so that
 * og_tree_status reports OG_ERANGE from then on. */
typedef struct og_targets {
    const int64_t *idx;
    int64_t M;
} og_targets;

/* Short-range force on the targets, with the tree's parameters.
 *   targets: NULL or {NULL, N} = all particles;
 *   acc: device [M][3] FP64, pot: device [M] FP64 or NULL, in target order.
 * Enqueued on the tree's stream.  A tree built with OG_OPEN_RELATIVE needs
 * a_old (og_tree_force_ex); here it gives OG_EINVAL. */
int og_tree_force(const og_tree *tree, const og_targets *targets, double *acc, double *pot);

/* Allocation-free variant of og_tree_force, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, precision, stream and
 * results (bitwise) as og_tree_force; the caller passes the inputs and
 * outputs, and the call makes no hipMalloc, hipFree or other allocating
 * call.  A target list's sort scratch lives in a fixed device array inside
 * the library (about 25 MB, for up to OG_NOALLOC_MAX_TARGETS targets),
 * which each GPU the library runs on holds until the process ends; a walk
 * over all N particles (targets NULL or idx NULL) needs none.  Every call on
 * a GPU shares that GPU's array: calls that overlap on one GPU (on other
 * streams or threads) race, so serialise them.  Errors: as og_tree_force,
 * and OG_EINVAL when targets->M > OG_NOALLOC_MAX_TARGETS. */
#define OG_NOALLOC_MAX_TARGETS 1048576
int og_tree_force_noalloc(const og_tree *tree, const og_targets *targets, double *acc, double *pot);

typedef struct og_force_opts {
    uint32_t struct_size;   /* = sizeof(og_force_opts) */
    int32_t precision;      /* -1: the tree's; else OG_PREC_* */
    void *stream;           /* NULL: the tree's stream */
    int64_t *n_inter;       /* device [M] or NULL: per-target count of
                               contributions that passed the cutoff */
    const double *a_old;    /* device [N][3] FP64, caller order: previous
                               accelerations for OG_OPEN_RELATIVE (required
                               then, ignored otherwise) */
} og_force_opts;

/* As og_tree_force, with a precision, stream and interaction counts. */
int og_tree_force_ex(const og_tree *tree, const og_targets *targets, const og_force_opts *opts,
                     double *acc, double *pot);

/* Forces on the active particles only (paper, "Code structure": particles
 * move on individual power-of-two time steps; at a step, those on the
 * current time-step level and below are active).  The tree stays resident
 * and is walked only for them.
 *   bin:   device [N] int8, caller order: each particle's time-step level
 *   level: particle i is active iff bin[i] <= level
 *   opts:  as og_tree_force_ex (NULL: the tree's precision and stream);
 *          n_inter, when given, is [N] in caller order
 *   acc:   device [N][3] FP64, pot: device [N] FP64 or NULL, caller order;
 *          only the active particles' entries are written
 *   n_active: device int64 [1] or NULL: receives the number of active
 *          particles
 * Nothing is read back to the host: the active list is compacted on the
 * device, in curve order, and the walk reads its length there.  Errors as
 * og_tree_force_ex. */
int og_tree_force_active(const og_tree *tree, const int8_t *bin, int32_t level, const og_force_opts *opts,
                         double *acc, double *pot, int64_t *n_active);

/* Synchronise the tree's stream and report the device-side status of the
 * build: OG_OK or OG_ERANGE. */
int og_tree_status(const og_tree *tree);

/* Synchronise and report node count, deepest level and device bytes held. */
int og_tree_stats(const og_tree *tree, int64_t *n_nodes, int32_t *depth, size_t *bytes);

/* Copy the tree to HOST buffers (synchronises); any pointer may be NULL.
 *   keys[N]   Morton keys in sorted order      perm[N]  sorted -> caller index
 *   first, count, skip, parent [n_nodes]      level [n_nodes]
 *   node_m_com [n_nodes][4] = (mass, com_x, com_y, com_z)
 * Node arrays must hold og_tree_stats' n_nodes entries. */
int og_tree_export(const og_tree *tree, uint64_t *keys, uint32_t *perm, uint32_t *first,
                   uint32_t *count, uint8_t *level, uint32_t *skip, uint32_t *parent,
                   double *node_m_com);

/* Check a built tree's invariants on the host (synchronises; copies the
 * tree's arrays to host memory, O(N + n_nodes) work and host memory, so it
 * is a test and audit tool, not part of a time step).  The invariants are
 * those of the paper's "Tree construction" (particles in space-filling-
 * curve order, the recursive 8-way cube hierarchy in pre-order with
 * first-child / sibling links, mass and centre of mass from the bottom-up
 * pass) and of this library's derived records:
 *   - keys sorted; perm a permutation of [0,N); every particle's key is the
 *     key of its position; periodic positions inside [0,box);
 *   - node 0 is the root: level 0, particles [0,N), no parent, skip = the
 *     node count;
 *   - every node holds a non-empty particle range whose keys share the
 *     node's prefix, and its corner is aligned to its level; a node is a
 *     leaf iff it holds at most leaf_max particles or is at the finest
 *     level (21);
 *   - an internal node's children (node+1, then along skip) are 1..8 nodes
 *     one level down, in distinct octants of its cube, with parent links to
 *     it, whose particle ranges tile its range in order; a leaf's skip is
 *     the next node;
 *   - a node's mass is the sum of its particles' (children's) masses and
 *     its centre of mass is theirs, inside its cube; FP32 copies, softening
 *     ranges and walk records agree with the FP64 values.
 * Returns OG_OK, OG_ERANGE (the build reported out-of-range positions),
 * OG_ECORRUPT (og_last_error() names the first violation), OG_EINVAL (NULL
 * tree) or OG_EDEVICE. */
int og_tree_validate(const og_tree *tree);

/* Free the tree and its device memory (not a caller workspace).  Waits for
 * the tree's stream first. */
int og_tree_free(og_tree *tree);

/* ---------------------------------------------------------------- batch --
 * Many independent boxes, each with its own particles and parameters, built
 * and walked by the same kernels in one set of launches (a box index is part
 * of every sort key and every walk group).  Each box's result equals the
 * result of building and walking that box alone. */
typedef struct og_box {
    const double *pos;   /* device [N][3] */
    const double *mass;  /* device [N] */
    int64_t N;
    double box;
    og_params params;    /* per box; stream/workspace fields ignored;
                            precision, group_max, walk_list_cap and lists
                            must equal box 0's; OG_OPEN_RELATIVE is not
                            available here (OG_EUNSUPPORTED) */
    double *acc;         /* device [N][3] output, caller order */
    double *pot;         /* device [N] output or NULL */
} og_box;

typedef struct og_batch og_batch;

/* Build all B boxes' trees on `stream` (hipStream_t or NULL). */
int og_batch_build(const og_box *boxes, int32_t B, void *stream, og_batch **out);
/* Walk every box's particles and write each box's acc/pot. */
int og_batch_force(og_batch *b);
/* Capture og_batch_build's kernels + og_batch_force for the same boxes into
 * a HIP graph owned by the batch, and replay it: positions and masses are
 * re-read from the same device pointers on every replay. */
int og_batch_graph_replay(og_batch *b);
int og_batch_status(const og_batch *b);
int og_batch_free(og_batch *b);

/* -------------------------------------------------------------- serving --
 * Continuous batching: requests (one box each) are admitted when their
 * tree's device footprint fits the HBM budget and a slot is free, built on
 * their own stream as soon as admitted, and walked while other requests
 * build or walk; a request that arrives while others are on the device is
 * admitted as soon as memory and a slot free up.  Trees stay resident until
 * the caller releases the ticket. */
typedef struct og_server og_server;

int og_server_create(size_t hbm_budget_bytes, int32_t max_slots, og_server **out);
/* Submit a request; its pos/mass/acc/pot are device buffers owned by the
 * caller and must stay valid until the ticket is released.  The request's
 * params.stream (hipStream_t, NULL = the null stream) is the stream its
 * inputs are written on: submit records an event there and the request's
 * build waits for it, so the caller need not synchronise before submitting.
 * The request itself runs on a slot stream of the server's; acc/pot are
 * valid once og_server_poll reports done or og_server_wait returns.
 * OG_EBUSY when the request can never fit the budget or the pending queue
 * is full.  A request that fails after submission (a launch error, a
 * position outside the box, a forced fault) is reported by poll/wait with
 * its error code; the server keeps serving the others. */
int og_server_submit(og_server *s, const og_box *req, uint64_t *ticket);
/* Progress the server (admit, launch, retire) without blocking. */
int og_server_progress(og_server *s);
/* done = 1 once acc/pot are written; times in seconds on the server's
 * monotonic clock (arrival = submit call, done = completion observed). */
int og_server_poll(og_server *s, uint64_t ticket, int32_t *done, double *t_arrive, double *t_done);
/* Block until the ticket is done (progressing the server meanwhile).  May
 * run concurrently with calls on other threads, including a release of the
 * same ticket (the wait then returns OG_ENOTFOUND or the request's result). */
int og_server_wait(og_server *s, uint64_t ticket);
/* Free the request's resident tree and its arena range (waiting for a
 * request still on the device). */
int og_server_release(og_server *s, uint64_t ticket);
/* Bytes currently reserved by admitted requests, and counts. */
int og_server_stats(const og_server *s, size_t *reserved, int32_t *in_flight, int32_t *pending);
int og_server_destroy(og_server *s);

/* ------------------------------------------------------- particle mesh --
 * Long-range part of the TreePM force (paper, "Particle Mesh"): the split
 * 1/r = erfc(r/2A)/r + erf(r/2A)/r gives the tree the erfc term and the
 * mesh the erf term.  On an n^3 periodic mesh of a box of side L:
 *   1. cloud-in-cell assignment of the masses to the nodes j L/n;
 *   2. FFT of the density rho;
 *   3. phi_k = -4 pi G exp(-k^2 r_s^2) / k^2 / W(k)^2 rho_k, with W the CIC
 *      window prod_a sinc^2(pi m_a/n) (assignment and interpolation
 *      deconvolved) and phi_0 = 0 (periodic, mean density removed);
 *      a_k = -i k phi_k, the Nyquist wavenumber's derivative set to 0;
 *   4. inverse FFTs and CIC interpolation at the particles; the potential
 *      drops the particle's own long-range term, -G m/(sqrt(pi) r_s).
 * The mesh sum is deterministic (fixed-point deposit).  Positions outside
 * [0, L) are wrapped. */
typedef struct og_pm og_pm;

/* Device bytes an n_grid^3 mesh holds: 32 n^3 + 256, plus 24 n bytes of
 * FFT and deconvolution tables and (n/8)^3 + 1 words of block starts, each
 * rounded up to 256 bytes; 0 if n_grid invalid. */
size_t og_pm_workspace_bound(int32_t n_grid);
/* n_grid: power of two in 8..1024; box > 0; r_s > 0 (the split scale of
 * the tree); stream: hipStream_t or NULL.  Allocates the mesh.  Errors:
 * OG_EINVAL, OG_ENOMEM. */
int og_pm_create(int32_t n_grid, double box, double G, double r_s, void *stream, og_pm **out);
/* Long-range acceleration and potential of N particles.
 *   pos: device [N][3] FP64, mass: device [N] FP64 (caller order)
 *   acc: device [N][3] FP64, pot: device [N] FP64 or NULL (caller order)
 *   accumulate: 0 overwrite, 1 add (e.g. onto og_tree_force's short-range
 *   result, giving the full TreePM force).
 * Enqueued on the mesh's stream.  Errors: OG_EINVAL, OG_EDEVICE. */
int og_pm_force(og_pm *pm, const double *pos, const double *mass, int64_t N, double *acc, double *pot,
                int32_t accumulate);
/* As og_pm_force for the particles of a built periodic tree whose box side
 * equals the mesh's, with the same result to the bit.  The tree's curve
 * order makes every block of 8^3 mesh cells a contiguous run of its
 * particles, so each block is deposited and interpolated by one workgroup
 * through a tile of its 9^3 nodes in LDS (the block's nodes are written
 * once, without atomics; blocks of more than 2048 particles hand the rest
 * to per-particle kernels).  acc/pot (device, [N][3] and [N] or NULL) are
 * written in caller order.  Ordered after the tree's build on its stream.
 * Errors: OG_EINVAL, OG_EDEVICE. */
int og_pm_force_tree(og_pm *pm, const og_tree *tree, double *acc, double *pot, int32_t accumulate);
/* Waits for the mesh's stream and frees it. */
int og_pm_free(og_pm *pm);

const char *og_strerror(int code);
const char *og_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* OG_H */
