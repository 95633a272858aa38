/*
 * ORACLE — test infrastructure only.
 *
 * Plain, slow, obviously-correct FP64 CPU implementation of the short-range
 * Barnes-Hut octree force of the TreePM scheme (paper: "Gravity Solver",
 * subsections "Oct-Tree", "Tree construction", "Tree walk", "Force
 * evaluation", "Particle Mesh").  Only the test-suite, the smoke entry and the
 * CPU-baseline leg of the benchmark may load this file's library.  It shares
 * no code, header, table or helper with the HIP path of the package.
 *
 * Readings of points the paper leaves open (numbered as in the design notes):
 *   R1  Plummer softening (r^2+eps^2)^(-3/2) instead of the paper's spline.
 *   R2  short-range force factor S(u) = erfc(u) + 2u/sqrt(pi) exp(-u^2),
 *       u = r/(2 r_s), which is -r^2 d/dr[erfc(r/2r_s)/r] of the split
 *       potential of the "Particle Mesh" subsection; potential -Gm erfc(u)/
 *       sqrt(r^2+eps^2).
 *   R3  contribution iff r^2 < r_cut^2 (strict), only when r_s > 0.
 *   R4  node skipped when on some axis |minimg(centre - x)| > r_cut + side/2.
 *   R5  Barnes-Hut test: open iff side^2 > theta^2 |COM - x|^2.
 *   R6  also open iff |minimg(centre - x)| < 0.6 side on all three axes.
 *   R8  leaves hold up to leaf_max particles (unlimited at level 21); a leaf
 *       may be accepted as a monopole like any node.
 *   R10 key quantisation, R11 Morton bit order, R12 pre-order node order,
 *   R13 one-step minimum image, R14 self excluded by index.
 *   R24 spline softening (switch): the point mass is replaced by the cubic
 *       spline density of compact support h = 2.8 eps, and the short-range
 *       factors of R2 multiply that softened force and potential.
 *   R25 relative opening criterion (switch): open iff
 *       G M side^2 > alpha |a_old| r^4 (r = |COM - x|), or by R6.
 *   R31 group-shared interaction lists (separate entry): for a group of
 *       targets the walk opens a node when any target for which the node is
 *       not pruned (R4) would open it (R5/R6 or R25); a node pruned for
 *       every target is skipped; otherwise every target of the group adds
 *       the node's monopole, or each particle of an opened leaf, subject to
 *       its own cutoff and self test.
 *   R32 per-particle softening (optional array): a pair is softened with
 *       the larger of its two lengths, a node's monopole with the larger of
 *       the target's and the node's largest; the mixed-softening check
 *       opens a node that holds different softenings, whose largest exceeds
 *       the target's, when the target lies within 2.8 times that largest
 *       length of the node's centre of mass.
 *   R26 Peano-Hilbert keys (switch): the cell's three 21-bit coordinates
 *       are turned into the transposed Hilbert index of Skilling (2004,
 *       "Programming the Hilbert curve") and interleaved as in R11.  The
 *       set of cells, hence of nodes, is the Morton one; children are
 *       ordered along the curve.
 *
 * Every function cites the passage it follows.  Summation order: the walk
 * adds contributions in traversal order; moments are summed particle by
 * particle in sorted order relative to the node centre.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OGO_LEVELS 21
#define OGO_GRID 2097152.0 /* 2^21 cells per axis at the deepest level */

/* ---------------------------------------------------------------- frame --
 * Root cube (paper, "Tree construction": the root covers the whole domain).
 * Periodic: [0, box)^3.  Open boundaries: lower corner = per-axis minimum,
 * side = largest per-axis extent (1 when all points coincide).
 * Returns 0, or -2 when a periodic coordinate lies outside [0, box) or is
 * not finite.                                                              */
int ogo_frame(const double *pos, int64_t n, double box, int periodic,
              double *lo3, double *side_out)
{
    if (periodic) {
        for (int64_t i = 0; i < 3 * n; ++i) {
            double v = pos[i];
            if (!(v >= 0.0 && v < box)) return -2;
        }
        lo3[0] = lo3[1] = lo3[2] = 0.0;
        *side_out = box;
        return 0;
    }
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) { lo[k] = pos[k]; hi[k] = pos[k]; }
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            double v = pos[3 * i + k];
            if (!isfinite(v)) return -2;
            if (v < lo[k]) lo[k] = v;
            if (v > hi[k]) hi[k] = v;
        }
    double L = 0.0;
    for (int k = 0; k < 3; ++k) {
        double e = hi[k] - lo[k];
        if (e > L) L = e;
        lo3[k] = lo[k];
    }
    if (!(L > 0.0)) L = 1.0;
    *side_out = L;
    return 0;
}

/* ----------------------------------------------------------------- keys --
 * 63-bit Morton key per particle (R10, R11).  Integer cell per axis:
 *   c = min(trunc((x - lo) * (2^21 / L)), 2^21 - 1)
 * with one FP64 division for the scale and one FP64 multiply per axis.
 * Bit 3b+2 of the key is bit b of cx, 3b+1 of cy, 3b of cz.               */
static uint32_t ogo_cell(double x, double lo, double scale)
{
    double v = (x - lo) * scale;
    if (v >= OGO_GRID - 1.0) return (uint32_t)(OGO_GRID - 1.0);
    return (uint32_t)v; /* v >= 0: truncation toward zero */
}

/* R26: Skilling's transform of cell coordinates into the "transposed"
 * Hilbert index (paper, "Tree construction" and "Domain decomposition":
 * particles follow the Peano-Hilbert curve).  Going from the top bit down,
 * at bit q the lower bits are either inverted (when coordinate i has bit q
 * set) or exchanged between coordinate 0 and i; then the result is Gray
 * coded.  Interleaving the three outputs, coordinate 0 first, gives the
 * index along the curve.                                                   */
static void ogo_hilbert(uint32_t c[3])
{
    for (uint32_t q = 1u << (OGO_LEVELS - 1); q > 1; q >>= 1) {
        uint32_t low = q - 1;
        for (int i = 0; i < 3; ++i) {
            if (c[i] & q) {
                c[0] ^= low;
            } else {
                uint32_t t = (c[0] ^ c[i]) & low;
                c[0] ^= t;
                c[i] ^= t;
            }
        }
    }
    c[1] ^= c[0];
    c[2] ^= c[1];
    uint32_t flip = 0;
    for (uint32_t q = 1u << (OGO_LEVELS - 1); q > 1; q >>= 1)
        if (c[2] & q) flip ^= q - 1;
    for (int i = 0; i < 3; ++i) c[i] ^= flip;
}

/* curve: 0 Morton (R11), 1 Peano-Hilbert (R26). */
void ogo_keys(const double *pos, int64_t n, const double *lo3, double L, int curve,
              uint64_t *keys)
{
    double scale = OGO_GRID / L;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t c[3];
        for (int k = 0; k < 3; ++k) c[k] = ogo_cell(pos[3 * i + k], lo3[k], scale);
        if (curve == 1) ogo_hilbert(c);
        uint64_t key = 0;
        for (int b = 0; b < OGO_LEVELS; ++b) {
            key |= (uint64_t)((c[0] >> b) & 1u) << (3 * b + 2);
            key |= (uint64_t)((c[1] >> b) & 1u) << (3 * b + 1);
            key |= (uint64_t)((c[2] >> b) & 1u) << (3 * b);
        }
        keys[i] = key;
    }
}

/* ----------------------------------------------------------------- sort --
 * Particles ordered along the space-filling curve (paper, "Tree
 * construction": insertion follows the curve order).  Ties between equal
 * keys are broken by the original index, so the order is unique.          */
static const uint64_t *ogo_sort_keys;
static int ogo_cmp(const void *a, const void *b)
{
    uint32_t i = *(const uint32_t *)a, j = *(const uint32_t *)b;
    uint64_t ki = ogo_sort_keys[i], kj = ogo_sort_keys[j];
    if (ki != kj) return ki < kj ? -1 : 1;
    return i < j ? -1 : (i > j ? 1 : 0);
}

void ogo_sort(const uint64_t *keys, int64_t n, uint32_t *perm)
{
    for (int64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    ogo_sort_keys = keys;
    qsort(perm, (size_t)n, sizeof(uint32_t), ogo_cmp);
    ogo_sort_keys = NULL;
}

/* ------------------------------------------------------------- topology --
 * Recursive 8-way subdivision of the root cube (paper, "Oct-Tree"), written
 * as the recursion itself: a node holding `count` sorted particles at
 * `level` is emitted, then, if count > leaf_max and level < 21, each
 * non-empty sub-cube (ascending 3-bit digit) is emitted in turn.  The
 * emission order is the pre-order of R12; skip (the paper's "sibling"
 * pointer) is the index of the first node emitted after the subtree.      */
typedef struct {
    const uint64_t *skeys;
    int leaf_max;
    int64_t cap, n_nodes;
    uint32_t *first, *count, *skip, *parent;
    uint8_t *level;
    int overflow;
} ogo_topo_ctx;

static void ogo_emit(ogo_topo_ctx *t, uint32_t first, uint32_t count, int level,
                     uint32_t parent)
{
    if (t->n_nodes >= t->cap) { t->overflow = 1; return; }
    int64_t me = t->n_nodes++;
    t->first[me] = first;
    t->count[me] = count;
    t->level[me] = (uint8_t)level;
    t->parent[me] = parent;
    if ((int)count > t->leaf_max && level < OGO_LEVELS) {
        int shift = 3 * (OGO_LEVELS - level - 1); /* digit of the child level */
        uint32_t j = first, end = first + count;
        while (j < end) {
            uint64_t d = (t->skeys[j] >> shift) & 7u;
            uint32_t k = j;
            while (k < end && ((t->skeys[k] >> shift) & 7u) == d) ++k;
            ogo_emit(t, j, k - j, level + 1, (uint32_t)me);
            j = k;
        }
    }
    t->skip[me] = (uint32_t)t->n_nodes;
}

/* Returns the node count, or -1 when more than `cap` nodes would be made. */
int64_t ogo_topology(const uint64_t *skeys, int64_t n, int leaf_max, int64_t cap,
                     uint32_t *first, uint32_t *count, uint8_t *level,
                     uint32_t *skip, uint32_t *parent)
{
    ogo_topo_ctx t = {skeys, leaf_max, cap, 0, first, count, skip, parent, level, 0};
    ogo_emit(&t, 0, (uint32_t)n, 0, 0xffffffffu);
    return t.overflow ? -1 : t.n_nodes;
}

/* ------------------------------------------------------------- geometry --
 * Cube of a node (paper, "Tree construction": cubic cell centre and side).
 * Corner cell c = the node's first particle's cell (as for its key) with
 * the low (21 - level) bits cleared; side = L 2^-level;
 * centre = lo + (c + 2^(20-level)) L 2^-21.  spos: sorted positions.      */
static void ogo_node_geometry(const double *x, int level, const double *lo3,
                              double L, double centre[3], double *side)
{
    double scale = OGO_GRID / L;
    int drop = OGO_LEVELS - level;
    double h = ldexp(L, -OGO_LEVELS);
    double half = ldexp(1.0, drop - 1);
    for (int k = 0; k < 3; ++k) {
        uint32_t c = ogo_cell(x[k], lo3[k], scale);
        uint32_t corner = (c >> drop) << drop;
        centre[k] = lo3[k] + ((double)corner + half) * h;
    }
    *side = ldexp(L, -level);
}

void ogo_node_centres(const double *spos, int64_t n_nodes, const uint32_t *first,
                      const uint8_t *level, const double *lo3, double L,
                      double *centre3, double *side)
{
    for (int64_t r = 0; r < n_nodes; ++r)
        ogo_node_geometry(spos + 3 * (int64_t)first[r], level[r], lo3, L, centre3 + 3 * r,
                          side + r);
}

/* -------------------------------------------------------------- moments --
 * Mass and centre of mass of every node (paper, "Tree construction": the
 * bottom-up pass computes total mass and centre of mass).  Written as the
 * definition: for each node, sum over its own particles in sorted order,
 *   M = sum m_j,   COM = centre + (sum m_j (x_j - centre)) / M.
 * spos is [n][3] in sorted order, smass [n] in sorted order.               */
void ogo_moments(const double *spos, const double *smass, int64_t n_nodes,
                 const uint32_t *first, const uint32_t *count,
                 const double *centre3, double *mass_out, double *com3)
{
    for (int64_t r = 0; r < n_nodes; ++r) {
        const double *c = centre3 + 3 * r;
        double M = 0.0, s[3] = {0.0, 0.0, 0.0};
        for (uint32_t j = first[r]; j < first[r] + count[r]; ++j) {
            double m = smass[j];
            M += m;
            for (int k = 0; k < 3; ++k) s[k] += m * (spos[3 * j + k] - c[k]);
        }
        mass_out[r] = M;
        for (int k = 0; k < 3; ++k) com3[3 * r + k] = c[k] + s[k] / M;
    }
}

/* ------------------------------------------------------- pair and walk --
 * Pair term (paper, "Force evaluation" and "Particle Mesh"; readings R1-R3)
 * added for a partner of mass m at minimum-image offset d = x_partner - x_i.
 */
typedef struct {
    double G, eps2, r_s, rcut, rc2, theta2, box;
    int periodic, cutoff;
    int spline;      /* R24: 0 Plummer, 1 cubic spline of support h */
    double h;        /* spline support, 2.8 eps */
    int relative;    /* R25: 0 Barnes-Hut (R5), 1 relative criterion */
    double alpha;    /* relative criterion tolerance */
    double eps;      /* softening length when no per-particle lengths */
    const double *seps, *emax, *emin; /* R32: per-particle (sorted) and per-node */
} ogo_walk_params;

static double ogo_minimg(double d, const ogo_walk_params *p)
{
    /* R13: one step into [-box/2, box/2]; exactly +-box/2 is kept. */
    if (!p->periodic) return d;
    if (d > 0.5 * p->box) return d - p->box;
    if (d < -0.5 * p->box) return d + p->box;
    return d;
}

static const double OGO_TWO_OVER_SQRTPI = 1.1283791670955126; /* 2/sqrt(pi) */

/* R24: softened 1/r^3 (force) and 1/r (potential) of a unit point mass
 * spread with the cubic spline density
 *   rho(s) = 8/(pi h^3) (1 - 6q^2 + 6q^3)  for q = s/h < 1/2,
 *            8/(pi h^3) 2 (1 - q)^3         for 1/2 <= q < 1,   0 beyond,
 * (paper, "Force evaluation": spline kernel of compact support h, the
 * Plummer-equivalent eps = h/2.8).  With u = r/h and M(u) the enclosed mass,
 * the force factor is M(u)/r^3 and the potential factor M(u)/r plus
 * 4 pi int_r^h s rho(s) ds; written out as polynomials in u:
 *   u < 1/2:  g h^3 = 32/3 - 192/5 u^2 + 32 u^3
 *             w h   = 14/5 - 16/3 u^2 + 48/5 u^4 - 32/5 u^5
 *   u < 1:    g h^3 = 64/3 - 48 u + 192/5 u^2 - 32/3 u^3 - 1/(15 u^3)
 *             w h   = 16/5 - 1/(15 u) - 32/3 u^2 + 16 u^3 - 48/5 u^4 + 32/15 u^5
 *   u >= 1:   g = 1/r^3, w = 1/r.                                         */
static void ogo_spline(double r, double h, double *g, double *w)
{
    if (r >= h) {
        *g = 1.0 / (r * r * r);
        *w = 1.0 / r;
        return;
    }
    double u = r / h, u2 = u * u, h3 = h * h * h;
    if (u < 0.5) {
        *g = (32.0 / 3.0 - 192.0 / 5.0 * u2 + 32.0 * u2 * u) / h3;
        *w = (14.0 / 5.0 - 16.0 / 3.0 * u2 + 48.0 / 5.0 * u2 * u2 - 32.0 / 5.0 * u2 * u2 * u) / h;
    } else {
        *g = (64.0 / 3.0 - 48.0 * u + 192.0 / 5.0 * u2 - 32.0 / 3.0 * u2 * u
              - 1.0 / (15.0 * u2 * u)) / h3;
        *w = (16.0 / 5.0 - 1.0 / (15.0 * u) - 32.0 / 3.0 * u2 + 16.0 * u2 * u
              - 48.0 / 5.0 * u2 * u2 + 32.0 / 15.0 * u2 * u2 * u) / h;
    }
}

/* Pair term with softening length e (the pair's, R32; else the global one). */
static int ogo_pair(const double d[3], double m, double e, const ogo_walk_params *p,
                    double acc[3], double *pot)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (p->cutoff && !(r2 < p->rc2)) return 0;
    double g, w; /* softened 1/r^3 and 1/r */
    if (p->spline) {
        ogo_spline(sqrt(r2), 2.8 * e, &g, &w);
    } else {
        double rinv = 1.0 / sqrt(r2 + e * e);
        g = rinv * rinv * rinv;
        w = rinv;
    }
    double S = 1.0, pf = 1.0;
    if (p->cutoff) {
        double r = sqrt(r2);
        double u = r / (2.0 * p->r_s);
        double e = erfc(u);
        S = e + OGO_TWO_OVER_SQRTPI * u * exp(-u * u);
        pf = e;
    }
    double f = p->G * m * g * S;
    acc[0] += f * d[0];
    acc[1] += f * d[1];
    acc[2] += f * d[2];
    *pot -= p->G * m * pf * w;
    return 1;
}

/* R32: largest and smallest softening length of every node's particles
 * (written into one allocation, returned for freeing; NULL without
 * per-particle lengths).                                                   */
static double *ogo_node_eps(const double *seps, int64_t n_nodes, const uint32_t *first,
                            const uint32_t *count, ogo_walk_params *p)
{
    p->seps = seps;
    p->emax = p->emin = NULL;
    if (!seps) return NULL;
    double *buf = (double *)malloc(sizeof(double) * 2 * (size_t)(n_nodes > 0 ? n_nodes : 1));
    for (int64_t r = 0; r < n_nodes; ++r) {
        double hi = seps[first[r]], lo = hi;
        for (uint32_t j = first[r]; j < first[r] + count[r]; ++j) {
            if (seps[j] > hi) hi = seps[j];
            if (seps[j] < lo) lo = seps[j];
        }
        buf[r] = hi;
        buf[n_nodes + r] = lo;
    }
    p->emax = buf;
    p->emin = buf + n_nodes;
    return buf;
}

/* Per-target tree walk (paper, "Tree walk"): one target per invocation,
 * starting at the root, moving to the first child (index + 1 in pre-order)
 * when a node is opened and to `skip` when it is accepted or pruned.      */
static int64_t ogo_walk_one(uint32_t ps, const double *spos, const double *smass,
                            int64_t n_nodes, const uint32_t *first,
                            const uint32_t *count, const uint8_t *is_leaf,
                            const uint32_t *skip, const double *centre3,
                            const double *side, const double *nmass,
                            const double *com3, const ogo_walk_params *p,
                            double aold, double acc[3], double *pot)
{
    const double *xi = spos + 3 * (int64_t)ps;
    const double ei = p->seps ? p->seps[ps] : p->eps;
    int64_t nint = 0;
    int64_t n = 0;
    acc[0] = acc[1] = acc[2] = 0.0;
    *pot = 0.0;
    while (n < n_nodes) {
        double s = side[n], dc[3], d[3];
        for (int k = 0; k < 3; ++k) dc[k] = ogo_minimg(centre3[3 * n + k] - xi[k], p);
        if (p->cutoff) {
            double reach = p->rcut + 0.5 * s;
            if (fabs(dc[0]) > reach || fabs(dc[1]) > reach || fabs(dc[2]) > reach) {
                n = skip[n];
                continue;
            }
        }
        for (int k = 0; k < 3; ++k) d[k] = ogo_minimg(com3[3 * n + k] - xi[k], p);
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double near = 0.6 * s;
        int far_open = p->relative ? (p->G * nmass[n] * s * s > p->alpha * aold * r2 * r2)
                                   : (s * s > p->theta2 * r2);
        int open = far_open ||
                   (fabs(dc[0]) < near && fabs(dc[1]) < near && fabs(dc[2]) < near);
        if (p->seps && p->emin[n] < p->emax[n] && p->emax[n] > ei) {
            /* R32: mixed-softening check */
            double hm = 2.8 * p->emax[n];
            if (r2 < hm * hm) open = 1;
        }
        if (!open) {
            double e = p->seps ? (ei > p->emax[n] ? ei : p->emax[n]) : p->eps;
            nint += ogo_pair(d, nmass[n], e, p, acc, pot);
            n = skip[n];
        } else if (!is_leaf[n]) {
            n = n + 1;
        } else {
            for (uint32_t j = first[n]; j < first[n] + count[n]; ++j) {
                if (j == ps) continue; /* R14 */
                double dj[3];
                for (int k = 0; k < 3; ++k) dj[k] = ogo_minimg(spos[3 * j + k] - xi[k], p);
                double e = p->seps ? (ei > p->seps[j] ? ei : p->seps[j]) : p->eps;
                nint += ogo_pair(dj, smass[j], e, p, acc, pot);
            }
            n = skip[n];
        }
    }
    return nint;
}

/* Tree walk for the targets given as sorted positions `tpos[M]`; outputs in
 * the same order.  Targets run in parallel; each target's own sum is
 * sequential in traversal order, so results do not depend on threads.
 * softening: 0 Plummer, 1 spline (R24).  criterion: 0 Barnes-Hut, 1
 * relative (R25) with tolerance alpha and the targets' previous
 * accelerations aold3[M][3] (target order).                               */
void ogo_walk(const double *spos, const double *smass, int64_t n_nodes,
              const uint32_t *first, const uint32_t *count, const uint8_t *level,
              const uint32_t *skip, const double *centre3, const double *side,
              const double *nmass, const double *com3, int leaf_max,
              double G, double eps, double r_s, double r_cut, double theta,
              int periodic, double box, int softening, int criterion, double alpha,
              const double *aold3, const double *seps, const uint32_t *tpos, int64_t M,
              double *acc3, double *pot, int64_t *nint)
{
    ogo_walk_params p;
    p.G = G;
    p.eps2 = eps * eps;
    p.r_s = r_s;
    p.cutoff = r_s > 0.0;
    p.rcut = r_cut;
    p.rc2 = r_cut * r_cut;
    p.theta2 = theta * theta;
    p.periodic = periodic;
    p.box = box;
    p.spline = softening == 1;
    p.h = 2.8 * eps;
    p.relative = criterion == 1;
    p.alpha = alpha;
    p.eps = eps;
    double *eminmax = ogo_node_eps(seps, n_nodes, first, count, &p);
    uint8_t *is_leaf = (uint8_t *)malloc((size_t)(n_nodes > 0 ? n_nodes : 1));
    for (int64_t r = 0; r < n_nodes; ++r)
        is_leaf[r] = !((int)count[r] > leaf_max && level[r] < OGO_LEVELS);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < M; ++t) {
        double a[3], ph, ao = 0.0;
        if (p.relative) {
            const double *v = aold3 + 3 * t;
            ao = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        }
        int64_t c = ogo_walk_one(tpos[t], spos, smass, n_nodes, first, count, is_leaf,
                                 skip, centre3, side, nmass, com3, &p, ao, a, &ph);
        acc3[3 * t] = a[0];
        acc3[3 * t + 1] = a[1];
        acc3[3 * t + 2] = a[2];
        pot[t] = ph;
        if (nint) nint[t] = c;
    }
    free(eminmax);
    free(is_leaf);
}

/* ------------------------------------------------- group-shared walk --
 * R31 (paper, "Neighbour search": nearby particles are grouped and served
 * by one search; "Tree walk" for the per-node rules).  Groups are given as
 * ranges goff[g]..goff[g+1] of the target list tpos (sorted positions);
 * every target of a group sees the same node sequence and adds the same
 * partners in the same order, each with its own cutoff and self test.     */
void ogo_walk_groups(const double *spos, const double *smass, int64_t n_nodes,
                     const uint32_t *first, const uint32_t *count, const uint8_t *level,
                     const uint32_t *skip, const double *centre3, const double *side,
                     const double *nmass, const double *com3, int leaf_max,
                     double G, double eps, double r_s, double r_cut, double theta,
                     int periodic, double box, int softening, int criterion, double alpha,
                     const double *aold3, const double *seps, const uint32_t *tpos,
                     const int64_t *goff, int64_t n_groups, double *acc3, double *pot,
                     int64_t *nint)
{
    ogo_walk_params p;
    p.G = G;
    p.eps2 = eps * eps;
    p.r_s = r_s;
    p.cutoff = r_s > 0.0;
    p.rcut = r_cut;
    p.rc2 = r_cut * r_cut;
    p.theta2 = theta * theta;
    p.periodic = periodic;
    p.box = box;
    p.spline = softening == 1;
    p.h = 2.8 * eps;
    p.relative = criterion == 1;
    p.alpha = alpha;
    p.eps = eps;
    double *eminmax = ogo_node_eps(seps, n_nodes, first, count, &p);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < n_groups; ++g) {
        const int64_t t0 = goff[g], t1 = goff[g + 1];
        for (int64_t t = t0; t < t1; ++t) {
            acc3[3 * t] = acc3[3 * t + 1] = acc3[3 * t + 2] = 0.0;
            pot[t] = 0.0;
            nint[t] = 0;
        }
        int64_t n = 0;
        while (n < n_nodes) {
            const double s = side[n];
            const int leaf = !((int)count[n] > leaf_max && level[n] < OGO_LEVELS);
            int any_live = 0, any_open = 0;
            for (int64_t t = t0; t < t1; ++t) {
                const double *xi = spos + 3 * (int64_t)tpos[t];
                double dc[3], d[3];
                for (int k = 0; k < 3; ++k) dc[k] = ogo_minimg(centre3[3 * n + k] - xi[k], &p);
                if (p.cutoff) {
                    double reach = p.rcut + 0.5 * s;
                    if (fabs(dc[0]) > reach || fabs(dc[1]) > reach || fabs(dc[2]) > reach) continue;
                }
                any_live = 1;
                for (int k = 0; k < 3; ++k) d[k] = ogo_minimg(com3[3 * n + k] - xi[k], &p);
                double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                double near = 0.6 * s, ao = 0.0;
                if (p.relative) {
                    const double *v = aold3 + 3 * t;
                    ao = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                }
                int far_open = p.relative ? (p.G * nmass[n] * s * s > p.alpha * ao * r2 * r2)
                                          : (s * s > p.theta2 * r2);
                if (far_open || (fabs(dc[0]) < near && fabs(dc[1]) < near && fabs(dc[2]) < near))
                    any_open = 1;
                if (p.seps) { /* R32 */
                    double ei = p.seps[tpos[t]], hm = 2.8 * p.emax[n];
                    if (p.emin[n] < p.emax[n] && p.emax[n] > ei && r2 < hm * hm) any_open = 1;
                }
            }
            if (!any_live) {
                n = skip[n];
            } else if (!any_open) {
                for (int64_t t = t0; t < t1; ++t) {
                    const double *xi = spos + 3 * (int64_t)tpos[t];
                    double d[3];
                    for (int k = 0; k < 3; ++k) d[k] = ogo_minimg(com3[3 * n + k] - xi[k], &p);
                    double ei = p.seps ? p.seps[tpos[t]] : p.eps;
                    double e = p.seps ? (ei > p.emax[n] ? ei : p.emax[n]) : p.eps;
                    nint[t] += ogo_pair(d, nmass[n], e, &p, acc3 + 3 * t, pot + t);
                }
                n = skip[n];
            } else if (!leaf) {
                n = n + 1;
            } else {
                for (uint32_t j = first[n]; j < first[n] + count[n]; ++j) {
                    for (int64_t t = t0; t < t1; ++t) {
                        if (j == tpos[t]) continue; /* R14 */
                        const double *xi = spos + 3 * (int64_t)tpos[t];
                        double dj[3];
                        for (int k = 0; k < 3; ++k) dj[k] = ogo_minimg(spos[3 * j + k] - xi[k], &p);
                        double ei = p.seps ? p.seps[tpos[t]] : p.eps;
                        double e = p.seps ? (ei > p.seps[j] ? ei : p.seps[j]) : p.eps;
                        nint[t] += ogo_pair(dj, smass[j], e, &p, acc3 + 3 * t, pot + t);
                    }
                }
                n = skip[n];
            }
        }
    }
    free(eminmax);
}
