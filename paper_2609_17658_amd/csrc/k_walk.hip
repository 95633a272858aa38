// Tree walk kernels for CDNA4 (gfx950, wave64).
//
// Paper, "Tree walk": one walk per target from the root; at each node the
// opening criterion decides between the first child (next node in
// pre-order) and the sibling pointer (skip); a leaf's particles contribute
// directly.  Paper, "Force evaluation" / "Particle Mesh": every accepted
// node or particle adds the short-range (erfc) part of the split force.
//
// GPU mapping: a persistent grid; each wavefront pops a group of up to 64
// consecutive targets in curve order (spatial neighbours) from an atomic
// queue and walks the tree once for the whole group.  Lane i owns target i
// and keeps `next`, the next node of ITS OWN per-target walk.  At node n
// the lanes with next == n apply the per-target rules; the wave goes to
// n + 1 when any lane opened n (ballot), otherwise to skip(n).  A lane
// therefore sees exactly the node sequence of its own walk, in the same
// order, so its result does not depend on the group it was placed in.
// Node records are wave-uniform: they are read with scalar loads, one per
// visit, once the wave has chosen the node (requesting both possible
// successors ahead of the decision costs more vector work to select between
// them than the load latency it hides).
#include <cstdlib>
#include <type_traits>

#include "og_kernels.h"

namespace og {

namespace {

// 2/sqrt(pi)
constexpr double kTwoOverSqrtPi = 1.1283791670955126;

// Abramowitz & Stegun 7.1.26: erfc(x) ~ t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) e^(-x^2),
// t = 1/(1 + p x), x >= 0, |error| <= 1.5e-7.
constexpr float kAsP = 0.3275911f;
constexpr float kAsA1 = 0.254829592f;
constexpr float kAsA2 = -0.284496736f;
constexpr float kAsA3 = 1.421413741f;
constexpr float kAsA4 = -1.453152027f;
constexpr float kAsA5 = 1.061405429f;
// The FP32 walk evaluates with v = x sqrt(log2 e) (exp(-x^2) = 2^(-v^2)):
// p and 2/sqrt(pi) divided by sqrt(log2 e) = 1.2011224087864498.
constexpr float kSqrtLog2e = 1.2011224087864498f;
constexpr float kAsPv = 0.2727374808792225f;
constexpr float kTwoOverSqrtPiV = 0.9394372786996513f;

// Read-only tree data is read through the constant address space: the
// compiler may then use scalar (SMEM) loads for wave-uniform addresses.  The
// walk never writes these arrays.
template <class T>
__device__ inline const __attribute__((address_space(4))) T *cptr(const T *p) {
  return (const __attribute__((address_space(4))) T *)(uintptr_t)p;
}
__device__ inline Topo ld(const Topo *p) {
  const auto q = cptr(p);
  Topo t;
  t.corner = q->corner;
  t.a = q->a;
  t.b = q->b;
  return t;
}
__device__ inline double4 ld(const double4 *p) {
  const auto q = cptr(p);
  return make_double4(q->x, q->y, q->z, q->w);
}
__device__ inline Mom64 ld(const Mom64 *p) {
  const auto q = cptr(p);
  return Mom64{q->cx, q->cy, q->cz, q->m};
}
__device__ inline BoxDev ld(const BoxDev *p) {
  const auto q = cptr(p);
  BoxDev b;
  b.pos = q->pos;
  b.mass = q->mass;
  b.acc = q->acc;
  b.pot = q->pot;
  b.lo[0] = q->lo[0];
  b.lo[1] = q->lo[1];
  b.lo[2] = q->lo[2];
  b.L = q->L;
  b.scale = q->scale;
  b.box = q->box;
  b.G = q->G;
  b.eps2 = q->eps2;
  b.r_s = q->r_s;
  b.rcut = q->rcut;
  b.rc2 = q->rc2;
  b.theta2 = q->theta2;
  b.Gf = q->Gf;
  b.eps2f = q->eps2f;
  b.inv2rsf = q->inv2rsf;
  b.rcutf = q->rcutf;
  b.rc2f = q->rc2f;
  b.theta2f = q->theta2f;
  b.Lf = q->Lf;
  b.h22f = q->h22f;
  b.p_off = q->p_off;
  b.n = q->n;
  b.root = q->root;
  b.node_end = q->node_end;
  b.periodic = q->periodic;
  b.cutoff = q->cutoff;
  b.leaf_max = q->leaf_max;
  b.g_off = q->g_off;
  b.spline = q->spline;
  b.relative = q->relative;
  b.hs = q->hs;
  b.alpha = q->alpha;
  b.hsf = q->hsf;
  b.hinvf = q->hinvf;
  b.curve = q->curve;
  b.epsp = q->epsp;
  b.eps = q->eps;
  return b;
}

__device__ inline double rdl(double v, uint32_t j) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), (int)j);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), (int)j);
  return __longlong_as_double(((long long)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Group g: box and target range.  Every particle a target: the targets of box
// b are cut into chunks of `chunk` consecutive sorted particles, box b's
// chunks numbered from g_off.  A target list: chunks of that list (box 0).
struct GroupRef {
  uint32_t box, tstart, tcount;
};
__device__ inline GroupRef group_of(const WalkArgs &A, uint32_t g) {
  GroupRef r;
  if (A.tkey) {
    r.box = 0;
    r.tstart = g * A.chunk;
    r.tcount = min(A.chunk, A.n_targets - r.tstart);
    return r;
  }
  int lo = 0, hi = A.B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cptr(A.boxes + mid)->g_off <= g) lo = mid; else hi = mid - 1;
  }
  const uint32_t off = cptr(A.boxes + lo)->g_off, p0 = cptr(A.boxes + lo)->p_off, nb = cptr(A.boxes + lo)->n;
  r.box = (uint32_t)lo;
  r.tstart = p0 + (g - off) * A.chunk;
  r.tcount = min(A.chunk, p0 + nb - r.tstart);
  return r;
}

// Target of lane `lane`: sorted particle position and output slot.
__device__ inline bool lane_target(const WalkArgs &A, const GroupRef &gr, const BoxDev &bx, uint32_t lane,
                                   uint32_t &p, uint32_t &slot) {
  if (lane >= gr.tcount) return false;
  if (A.tkey) {
    p = (uint32_t)A.tkey[gr.tstart + lane];
    slot = A.tval[gr.tstart + lane];
  } else {
    p = gr.tstart + lane;
    slot = A.perm[p] - bx.p_off;
  }
  return true;
}

__device__ inline void write_out(const WalkArgs &A, const BoxDev &bx, uint32_t slot, double ax, double ay,
                                 double az, double ph, uint32_t ni) {
  double *acc = A.acc ? A.acc : bx.acc;
  double *pot = A.pot_override ? A.pot : bx.pot;
  acc[3ull * slot] = ax;
  acc[3ull * slot + 1] = ay;
  acc[3ull * slot + 2] = az;
  if (pot) pot[slot] = ph;
  if (A.nint) A.nint[slot] = (int64_t)ni;
}

// Group queues.  Workgroups are dispatched round-robin over the chip's
// kQueues XCDs, each with its own L2, so the groups (consecutive in curve
// order) are split into kQueues contiguous ranges and workgroup b starts on
// range b % kQueues: the waves of one XCD sweep one region of space and
// share its tree nodes in their L2.  A wave whose range is exhausted moves
// on to the next range, so every group is processed exactly once and every
// wave leaves the loop once all ranges are exhausted.
struct GroupQueue {
  uint32_t *counters;
  uint32_t n_groups;
  uint32_t q, tried;
};
__device__ inline uint32_t range_begin(uint32_t n_groups, uint32_t q) {
  return (uint32_t)(((uint64_t)n_groups * q) / kQueues);
}
// Next group for this wave, or n_groups when all are taken.
__device__ inline uint32_t pop_group(GroupQueue &Q, uint32_t lane) {
  while (Q.tried < kQueues) {
    const uint32_t b = range_begin(Q.n_groups, Q.q), e = range_begin(Q.n_groups, Q.q + 1);
    uint32_t i = 0;
    if (lane == 0) i = atomicAdd(&Q.counters[Q.q], 1u);
    i = __builtin_amdgcn_readlane(i, 0);  // wave-uniform
    if (b + i < e) return b + i;
    Q.q = (Q.q + 1) % kQueues;
    ++Q.tried;
  }
  return Q.n_groups;
}
// Target and group counts produced on the device (active targets).
__device__ inline void device_counts(WalkArgs &A) {
  if (A.dev_count) {
    A.n_targets = cptr(A.dev_count)[0];
    A.n_groups = cptr(A.dev_count)[1];
  }
}
__device__ inline GroupQueue make_queue(const WalkArgs &A) {
  GroupQueue Q;
  Q.counters = A.counter;
  Q.n_groups = A.n_groups;
  Q.q = blockIdx.x % kQueues;
  Q.tried = 0;
  return Q;
}

// ------------------------------------------------------------ FP64 form --
__device__ inline double minimg(double d, bool periodic, double box) {
  const double hi = d > 0.5 * box ? d - box : d;
  const double w = d < -0.5 * box ? d + box : hi;
  return periodic ? w : d;
}

// The minimum image of three offsets, applied only when the (wave-uniform)
// flag says it can change one: a branch, not a select, so groups that need
// no wrap skip the work.
__device__ inline void minimg3(double &x, double &y, double &z, bool wrap, double box) {
  if (wrap) {
    x = minimg(x, true, box);
    y = minimg(y, true, box);
    z = minimg(z, true, box);
  }
}

// Spline-softened 1/r^3 (g) and 1/r (w) of a unit mass spread with the
// cubic spline density of support h (paper, "Force evaluation"); u = r/h.
__device__ inline void spline64(double r, double h, double &g, double &w) {
#pragma clang fp contract(off)
  if (r >= h) {
    g = 1.0 / (r * r * r);
    w = 1.0 / r;
    return;
  }
  const double u = r / h, u2 = u * u, h3 = h * h * h;
  if (u < 0.5) {
    g = (32.0 / 3.0 - 192.0 / 5.0 * u2 + 32.0 * u2 * u) / h3;
    w = (14.0 / 5.0 - 16.0 / 3.0 * u2 + 48.0 / 5.0 * u2 * u2 - 32.0 / 5.0 * u2 * u2 * u) / h;
  } else {
    g = (64.0 / 3.0 - 48.0 * u + 192.0 / 5.0 * u2 - 32.0 / 3.0 * u2 * u - 1.0 / (15.0 * u2 * u)) / h3;
    w = (16.0 / 5.0 - 1.0 / (15.0 * u) - 32.0 / 3.0 * u2 + 16.0 * u2 * u - 48.0 / 5.0 * u2 * u2 +
         32.0 / 15.0 * u2 * u2 * u) /
        h;
  }
}

// erfc(u) = exp(-u^2) erfcx(u).  erfcx on 0 <= u <= 3 (r < 6 r_s) is a
// polynomial of degree 25 in t = 2u/3 - 1 (coefficients from
// gen_erfcx64.py, relative error below 1e-15), so the pair term needs one
// exponential; larger u falls back to the library erfc.
__constant__ double kErfcx64[26] = {
    -1.9285526545026629e-09, 5.7920154915414246e-09, -4.6119752723685525e-09,
    1.2374418534053267e-08, -6.8302916092557606e-08, 1.8960282584894505e-07,
    -4.5725982227457081e-07, 1.2076614734008636e-06, -3.1901620317342984e-06,
    8.1102004120020287e-06, -2.0126549072150048e-05, 4.8905112127983934e-05,
    -0.00011601010087456714, 0.00026818449435352847, -0.00060331955090763077,
    0.0013184708553075387, -0.0027932530866193999, 0.0057231897175237054,
    -0.011309695741544485, 0.021484255075844793, -0.039077115130126794,
    0.06772278857525682, -0.11114180538602185, 0.17133983967481778,
    -0.2454343765988401, 0.32158541645431754,
};
__device__ inline double erfcx64(double u) {
  // The coefficients are read with scalar loads at each use: kept in
  // registers across the walk they would cost 52 of them and halve the
  // number of resident waves.
  const double *c = kErfcx64;
  asm volatile("" : "+s"(c));
  const auto q = cptr(c);
  const double t = fma(u, 2.0 / 3.0, -1.0);
  double y = q[0];
  // y * t + c_i as one three-operand FMA with the coefficient read from the
  // scalar registers (the compiler's two-operand form first copies every
  // coefficient into vector registers: two moves per step)
#pragma unroll
  for (int i = 1; i < 26; ++i) {
    const double ci = q[i];
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(y) : "v"(y), "v"(t), "s"(ci));
  }
  return y;
}

// exp(x) for the pair term's x = -u^2 <= 0.  Cody and Waite's reduction:
// x = k ln2 + r with k = rint(x / ln2), |r| <= ln2/2, and ln2 in two parts
// whose first has 29 significant bits, so k ln2_hi is exact.  exp(r) is
// its Taylor series to r^13 (the truncation is below 5e-18 relative), one
// three-operand FMA per term with the coefficient as a scalar operand, and
// the result is scaled by 2^k (underflowing to 0 far below the doubles the
// walk can reach; the clamp keeps r finite there).
__constant__ double kExpTaylor[14] = {
    1.6059043836821613e-10, 2.08767569878681e-09, 2.505210838544172e-08, 2.755731922398589e-07,
    2.7557319223985893e-06, 2.48015873015873e-05, 0.0001984126984126984, 0.001388888888888889,
    0.008333333333333333,   0.041666666666666664, 0.16666666666666666,   0.5,
    1.0,                    1.0,
};  // 1/13!, 1/12!, ..., 1/1!, 1/0!
constexpr double kLn2Hi = 0x1.62e42ff000000p-1, kLn2Lo = -0x1.718432a1b0e26p-35, kLog2e = 1.4426950408889634;
__device__ inline double exp_nonpos(double x) {
  x = fmax(x, -1100.0);
  const double kd = rint(x * kLog2e);
  double r = fma(-kd, kLn2Hi, x);
  r = fma(-kd, kLn2Lo, r);
  const double *c = kExpTaylor;
  asm volatile("" : "+s"(c));
  const auto q = cptr(c);
  double y = q[0];
#pragma unroll
  for (int i = 1; i < 14; ++i) {
    const double ci = q[i];
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(y) : "v"(y), "v"(r), "s"(ci));
  }
  return ldexp(y, (int)kd);
}

// e: the pair's softening length (used by the kExt variants; the others
// take the box's).
// kTail: some pair may have u = r / (2 r_s) > 3 (r_cut > 6 r_s), past the
// erfcx polynomial; without it the kernel carries no library erfc, whose
// constants would otherwise hold vector registers for the whole walk.
template <bool kExt, bool kTail = true>
__device__ inline bool pair64_terms(double dx, double dy, double dz, double m, double e, const BoxDev &bx,
                                    double4 &t) {
#pragma clang fp contract(off)
  const double r2 = dx * dx + dy * dy + dz * dz;
  if (bx.cutoff && !(r2 < bx.rc2)) return false;
  double g, w;  // softened 1/r^3 and 1/r
  if (kExt && bx.spline) {
    spline64(sqrt(r2), 2.8 * e, g, w);
  } else {
    const double rinv = rsqrt(r2 + (kExt ? e * e : bx.eps2));  // within an ulp or two of 1/sqrt
    g = rinv * rinv * rinv;
    w = rinv;
  }
  double S = 1.0, pf = 1.0;
  if (bx.cutoff) {
    const double r = sqrt(r2);
    const double u = r * (0.5 / bx.r_s);
    const double eu = exp_nonpos(-u * u);
    const double e = (!kTail || u <= 3.0) ? eu * erfcx64(u) : erfc(u);
    S = e + kTwoOverSqrtPi * u * eu;
    pf = e;
  }
  const double f = bx.G * m * g * S;
  t = make_double4(f * dx, f * dy, f * dz, bx.G * m * pf * w);
  return true;
}

// The pair term added to one target's sums: the force terms and the
// potential term of pair64_terms, each rounded once and then added.
template <bool kExt, bool kTail = true>
__device__ inline void pair64(double dx, double dy, double dz, double m, double e, const BoxDev &bx,
                              double &ax, double &ay, double &az, double &ph, uint32_t &ni) {
#pragma clang fp contract(off)
  double4 t;
  if (!pair64_terms<kExt, kTail>(dx, dy, dz, m, e, bx, t)) return;
  ax += t.x;
  ay += t.y;
  az += t.z;
  ph -= t.w;
  ++ni;
}

// Plain FP64 walk: every quantity in double precision, with the same
// expressions (and no contraction) as a direct reading of the walk rules.
// The decisions are taken at the node; an accepted monopole (FP64 offset and
// mass) or an opened leaf (its particle range) goes to the lane's own list
// in LDS, and the lists are evaluated when one is full and at the end of
// the walk, with the pair terms spread over all lanes (flush64).  Each
// target still sums its partners in traversal order, but the costly FP64
// pair terms run with the lanes of many nodes at once instead of only the
// lanes that accepted or opened the current node.
// kExt: the spline softening and the relative criterion are read from each
// box.
constexpr int kWalk64Waves = 4;  // waves per workgroup
// List entries per lane: 4, or 3 for the instances with per-entry
// softening lengths (kExt), so that lists, lengths and the evaluation slots
// stay within 40 KB per workgroup (four workgroups, 16 waves, per CU).
template <bool kExt>
constexpr int walk64_cap() { return kExt ? 3 : 4; }

// List entries: a monopole is (offset, mass), mass >= 0; a leaf has w = -1
// and, in the bits of x, its first particle (bits 0..31), count (32..62)
// and whether its particles' offsets need the minimum image (bit 63).
__device__ inline uint32_t entry_items64(const double4 &q) {
  return q.w >= 0.0 ? 1u : (uint32_t)((uint64_t)__double_as_longlong(q.x) >> 32) & 0x7fffffffu;
}

__device__ inline uint32_t lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Evaluate and empty every lane's list with the pair terms computed by all
// lanes.  A lane's items are its partners in list order (a monopole entry is
// one item, a leaf entry one item per particle).  Row k holds the k-th item
// of every lane that has more than k items; whole rows are laid out one
// after another in steps of at most 64 slots.  In each step the owners write their items'
// descriptors into the slots, every lane computes the pair terms of one
// slot (pair64_terms, the arithmetic of an evaluation by the owner), and the
// owners add the terms of their items in row order, which is their list
// order.  So each target sums its partners in traversal order with the same
// FP64 operations, while the costly pair terms run on every lane instead of
// only on the lanes whose lists are longest.  `slots` holds a step's
// descriptors (x: owner lane | entry << 8, y: particle within the entry,
// z: the owner's target) and then, in the same place, its terms; a ballot
// marks the slots whose pair contributes.
// The row machinery of the evaluation, for any list layout: items(e) is
// the number of items of this lane's entry e (e < nent), and
// term(l, e, j, po, t) computes the terms t of item j of lane l's entry e
// for target po and says whether the pair contributes.
constexpr uint32_t kOwnerRows = 48;  // lanes with an item from which a row is evaluated in place
template <int kCap, class Items, class Term>
__device__ inline void flush_rows64(double4 *slots, uint32_t lane, uint32_t p, uint32_t nent, Items items, Term term,
                                    double &ax, double &ay, double &az, double &ph, uint32_t &ni) {
#pragma clang fp contract(off)
  // this lane's entry sizes (in items) and their total
  uint32_t sz[kCap];
  uint32_t P = 0;
#pragma unroll
  for (int e = 0; e < kCap; ++e) {
    sz[e] = (uint32_t)e < nent ? items((uint32_t)e) : 0u;
    P += sz[e];
  }
  uint32_t ce = 0, cj = 0;  // entry and particle of this lane's next item
  uint32_t k = 0;           // next row (wave-uniform)
  // Rows that nearly every lane takes part in are evaluated by their owners
  // in place (no slots): the same terms, added in the same order.
  uint64_t row = __ballot(P > 0);
  while ((uint32_t)__popcll(row) >= kOwnerRows) {
    if (P > k) {
      double4 t = make_double4(0.0, 0.0, 0.0, 0.0);
      if (term(lane, ce, cj, p, t)) {
        ax += t.x;
        ay += t.y;
        az += t.z;
        ph -= t.w;
        ++ni;
      }
      uint32_t n = sz[0];
#pragma unroll
      for (int e = 1; e < kCap; ++e) n = ce == (uint32_t)e ? sz[e] : n;
      ++cj;
      const bool next_entry = cj == n;
      ce += next_entry ? 1u : 0u;
      cj = next_entry ? 0u : cj;
    }
    ++k;
    row = __ballot(P > k);
  }
  while (row) {
    // fill the step with whole rows k, k + 1, ... while they fit
    const uint32_t k0 = k;
    uint32_t f = 0;
    do {
      const uint32_t c = (uint32_t)__popcll(row);
      if (f + c > 64u) break;
      if (P > k) {
        const uint32_t at = f + lane_rank(row);
        *reinterpret_cast<uint4 *>(slots + at) = make_uint4(lane | (ce << 8), cj, p, 0u);
        uint32_t n = sz[0];
  #pragma unroll
        for (int e = 1; e < kCap; ++e) n = ce == (uint32_t)e ? sz[e] : n;
        ++cj;
        const bool next_entry = cj == n;
        ce += next_entry ? 1u : 0u;
        cj = next_entry ? 0u : cj;
      }
      f += c;
      ++k;
      row = __ballot(P > k);
    } while (row);
    __builtin_amdgcn_wave_barrier();
    // every lane computes the terms of one slot; a ballot marks the slots
    // that contribute (a partner other than the target, within the cutoff)
    double4 t = make_double4(0.0, 0.0, 0.0, 0.0);
    bool contributes = false;
    if (lane < f) {
      const uint4 d = *reinterpret_cast<const uint4 *>(slots + lane);
      contributes = term(d.x & 63u, d.x >> 8, d.y, d.z, t);
    }
    const uint64_t used = __ballot(contributes);
    __builtin_amdgcn_wave_barrier();
    slots[lane] = t;
    __builtin_amdgcn_wave_barrier();
    // the owners add their terms, row by row (the rows of the fill)
    uint32_t g = 0;
    for (uint32_t kk = k0; kk < k; ++kk) {
      const uint64_t rr = __ballot(P > kk);
      if (P > kk) {
        const uint32_t at = g + lane_rank(rr);
        if ((used >> at) & 1u) {
          const double4 u = slots[at];
          ax += u.x;
          ay += u.y;
          az += u.z;
          ph -= u.w;
          ++ni;
        }
      }
      g += (uint32_t)__popcll(rr);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

template <bool kExt, bool kTail>
__device__ inline void flush64(const WalkArgs &A, double4 (*list)[64], double (*lsoft)[64], double4 *slots,
                               uint32_t lane, uint32_t p, bool soft, const BoxDev &bx, uint32_t &cnt, double &ax,
                               double &ay, double &az, double &ph, uint32_t &ni) {
  constexpr int kCap = walk64_cap<kExt>();
  flush_rows64<kCap>(
      slots, lane, p, cnt, [&](uint32_t e) __attribute__((always_inline)) { return entry_items64(list[e][lane]); },
      [&](uint32_t l, uint32_t e, uint32_t j, uint32_t po, double4 &t) __attribute__((always_inline)) {
#pragma clang fp contract(off)
        const double4 q = list[e][l];
        double dx = q.x, dy = q.y, dz = q.z, m = q.w, es = bx.eps;
        bool use = true;
        if (q.w >= 0.0) {
          if (soft) es = lsoft[e][l];
        } else {
          const uint64_t bits = (uint64_t)__double_as_longlong(q.x);
          const uint32_t i = (uint32_t)bits + j;
          use = i != po;
          const double4 xo = A.part64[po], sp = A.part64[i];
          dx = sp.x - xo.x;
          dy = sp.y - xo.y;
          dz = sp.z - xo.z;
          // a branch: leaves of interior groups (below level 1) need no image
          minimg3(dx, dy, dz, (bits >> 63) != 0, bx.box);
          m = sp.w;
          if (soft) {
            const double ej = A.seps[i], eo = A.seps[po];
            es = eo > ej ? eo : ej;
          }
        }
        return use && pair64_terms<kExt, kTail>(dx, dy, dz, m, es, bx, t);
      },
      ax, ay, az, ph, ni);
  cnt = 0;
}

// Four waves per SIMD: the instance for boxes with r_cut < 6 r_s needs 97
// vector registers and no scratch; the one with the library erfc tail needs
// 128 and spills a few values to scratch.
template <bool kExt, bool kTail>
__global__ __launch_bounds__(64 * kWalk64Waves) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_walk64(WalkArgs A) {
#pragma clang fp contract(off)
  constexpr int kCap = walk64_cap<kExt>();
  __shared__ double4 lists[kWalk64Waves][kCap][64];
  __shared__ double lsofts[kExt ? kWalk64Waves : 1][kExt ? kCap : 1][64];
  __shared__ double4 slotss[kWalk64Waves][64];
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double4(*list)[64] = lists[wv];
  double(*lsoft)[64] = lsofts[kExt ? wv : 0];
  double4 *slots = slotss[wv];
  device_counts(A);
  GroupQueue Q = make_queue(A);
  while (true) {
    const uint32_t g = pop_group(Q, lane);
    if (g >= A.n_groups) break;
    const GroupRef gr = group_of(A, g);
    const BoxDev bx = ld(A.boxes + gr.box);
    uint32_t p = 0, slot = 0;
    const bool valid = lane_target(A, gr, bx, lane, p, slot);
    double4 xi = make_double4(0.0, 0.0, 0.0, 0.0);
    if (valid) xi = A.part64[p];
    double aold = 0.0;  // |previous acceleration| for the relative criterion
    const bool relative = kExt && bx.relative;
    if (valid && relative) {
      const double *v = A.a_old + 3ull * (A.perm[p] - bx.p_off);
      aold = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    }
    // softening: the target's own length (per-particle lengths) or the box's
    const bool soft = kExt && A.seps != nullptr && bx.epsp != nullptr;
    const double ei = soft && valid ? A.seps[p] : bx.eps;
    const bool periodic = bx.periodic;
    const double box = bx.box;
    // A group whose targets all lie farther than r_cut from every face of
    // the periodic box (r_cut below a quarter of the box) needs no minimum
    // image below level 1: a node of side <= box/4 within reach of such a
    // target is within half a box of it, and so are its centre of mass and
    // particles, while any other node is pruned in either image.  The
    // offsets, and so every decision and term, are those of the minimum
    // image.
    bool interior = false;
    if (periodic) {
      const double m = bx.rcut + 0x1p-40 * box;
      const bool inside = !valid || (xi.x >= m && xi.x <= box - m && xi.y >= m && xi.y <= box - m &&
                                     xi.z >= m && xi.z <= box - m);
      interior = bx.rcut <= 0.24 * box && __ballot(!inside) == 0;
    }
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    uint32_t ni = 0, cnt = 0;
    uint32_t n = bx.root;
    const uint32_t nend = bx.node_end;
    uint32_t next = valid ? n : nend;
    while (n < nend) {
      // room for this visit's entry
      if (__ballot(cnt >= (uint32_t)kCap))
        flush64<kExt, kTail>(A, list, lsoft, slots, lane, p, soft, bx, cnt, ax, ay, az, ph, ni);
      const Topo t = ld(A.topo + n);
      const Mom64 mm = ld(A.mom64 + n);
      const bool leaf = (t.corner & kLeafBit) != 0;
      const uint32_t ns = leaf ? n + 1 : t.a;
      const int lev = (int)(t.b >> kCountBits);
      const bool wrap = periodic && !(interior && lev >= 2);
      // cube centre and side, computed once per build
      const double4 cs = ld(A.cen64 + n);
      const double side = cs.w, c0 = cs.x, c1 = cs.y, c2 = cs.z;
      bool open_int = false;
      if (next == n) {
        double dcx = c0 - xi.x, dcy = c1 - xi.y, dcz = c2 - xi.z;
        minimg3(dcx, dcy, dcz, wrap, box);
        bool pruned = false;
        if (bx.cutoff) {
          const double reach = bx.rcut + 0.5 * side;
          pruned = fabs(dcx) > reach || fabs(dcy) > reach || fabs(dcz) > reach;
        }
        if (pruned) {
          next = ns;
        } else {
          double dx = mm.cx - xi.x, dy = mm.cy - xi.y, dz = mm.cz - xi.z;
          minimg3(dx, dy, dz, wrap, box);
          const double r2 = dx * dx + dy * dy + dz * dz;
          const double near = 0.6 * side;
          const bool far_open = relative ? (bx.G * mm.m * side * side > bx.alpha * aold * r2 * r2)
                                            : (side * side > bx.theta2 * r2);
          bool open = far_open || (fabs(dcx) < near && fabs(dcy) < near && fabs(dcz) < near);
          double e = bx.eps;
          if (soft) {
            // the node's softening range; mixed-softening check
            const double emax = *cptr(A.semax + n), emin = *cptr(A.semin + n);
            if (emin < emax && emax > ei) {
              const double hm = 2.8 * emax;
              if (r2 < hm * hm) open = true;
            }
            e = ei > emax ? ei : emax;
          }
          if (!open) {
            // the monopole, if within the cutoff (the test the pair term makes)
            if (!bx.cutoff || r2 < bx.rc2) {
              list[cnt][lane] = make_double4(dx, dy, dz, mm.m);
              if (kExt) lsoft[cnt][lane] = e;
              ++cnt;
            }
            next = ns;
          } else if (!leaf) {
            open_int = true;
            next = n + 1;
          } else {
            const uint64_t range = (uint64_t)t.a | ((uint64_t)(t.b & kCountMask) << 32) | ((uint64_t)wrap << 63);
            list[cnt][lane] = make_double4(__longlong_as_double((long long)range), 0.0, 0.0, -1.0);
            ++cnt;
            next = n + 1;
          }
        }
      }
      // a leaf's skip is n + 1; a skip always moves forward
      n = (leaf || __ballot(open_int) || t.a <= n) ? n + 1 : t.a;
    }
    flush64<kExt, kTail>(A, list, lsoft, slots, lane, p, soft, bx, cnt, ax, ay, az, ph, ni);
    if (valid) write_out(A, bx, slot, ax, ay, az, ph, ni);
  }
}

// ----------------------------------------------------------- mixed form --
// Every lane works in FP32 offsets from its own origin, the centre of the
// level-21 cell holding its target.  Cell indices (in half-cells, < 2^23)
// are exact, so a node centre relative to a lane's origin is one exact
// integer difference times the half-cell size; in a periodic box that
// difference is the minimum image (reduced once per node on the scalar unit
// for compact groups, per lane otherwise).  A node's centre of mass is its
// centre plus the node's FP32 offset, a particle is its leaf's centre plus
// its FP32 offset (both offsets formed in FP64 at build time), and the
// target is FP64 (x - origin) rounded once.  Node data comes from 48-byte
// walk records read with scalar loads.
//
// Accepted partners are not evaluated at the node: each lane appends
// (offset, mass) to its own list in LDS, in traversal order, and the lists
// are evaluated lane-parallel when one of them is full and at the end of
// the walk.  The per-target summation order is thus the traversal order,
// and a lane evaluates only its own partners, so the interaction arithmetic
// runs with the lanes of many nodes at once even though the lanes'
// decisions at a node differ.  The per-lane decisions are computed without
// branches.
constexpr int kWalk32Threads = 64;       // one wavefront per workgroup

struct Consts32 {
  float G, eps2, inv2rs, rc2, theta2, h22, half_box, box;  // inv2rs: sqrt(log2 e) / (2 r_s)
  float hs2, hinv;  // spline support squared and inverse
  bool cutoff, periodic, spline;
  bool soft;        // per-particle softening lengths: each pair brings its own
};

__device__ inline WNode ldw(const WNode *p) {
  const auto q = cptr(p);
  WNode w;
  w.c[0] = q->c[0];
  w.c[1] = q->c[1];
  w.c[2] = q->c[2];
  w.side2 = q->side2;
  w.o[0] = q->o[0];
  w.o[1] = q->o[1];
  w.o[2] = q->o[2];
  w.m = q->m;
  w.reach = q->reach;
  w.near = q->near;
  w.a = q->a;
  w.cf = q->cf;
  return w;
}

// Spline-softened 1/r^3 (g) and 1/r (w) inside the support, u = r/h < 1.
__device__ inline void spline32(float u, float hinv, float &g, float &w) {
#pragma clang fp contract(fast)
  const float u2 = u * u, h3 = hinv * hinv * hinv;
  if (u < 0.5f) {
    g = (32.0f / 3.0f + u2 * (-192.0f / 5.0f + 32.0f * u)) * h3;
    w = (14.0f / 5.0f + u2 * (-16.0f / 3.0f + u2 * (48.0f / 5.0f - 32.0f / 5.0f * u))) * hinv;
  } else {
    const float iu = __builtin_amdgcn_rcpf(u);
    g = (64.0f / 3.0f + u * (-48.0f + u * (192.0f / 5.0f - 32.0f / 3.0f * u)) - (1.0f / 15.0f) * iu * iu * iu) * h3;
    w = (16.0f / 5.0f - (1.0f / 15.0f) * iu + u2 * (-32.0f / 3.0f + u * (16.0f + u * (-48.0f / 5.0f + 32.0f / 15.0f * u)))) *
        hinv;
  }
}

// One partner at offset (dx, dy, dz) with r2 = |d|^2, mass m: FP32 pair
// term, accumulated in FP64.
// e: the pair's softening length when k.soft (kExt variants only).
template <bool kExt>
// gm: the partner's G times mass (walk records and FP32 particle copies hold
// it so).
__device__ inline void eval32(float dx, float dy, float dz, float r2, float gm, const Consts32 &k, double &ax,
                              double &ay, double &az, double &ph, float e = 0.0f) {
#pragma clang fp contract(fast)
  float g, wv;  // softened 1/r^3 and 1/r
  if (kExt && k.spline) {
    float hs2 = k.hs2, hinv = k.hinv;
    if (k.soft) {
      const float h = 2.8f * e;
      hs2 = h * h;
      hinv = __builtin_amdgcn_rcpf(h);
    }
    const float ri = __builtin_amdgcn_rsqf(r2);
    if (r2 < hs2) {
      const float r = r2 > 0.0f ? r2 * ri : 0.0f;
      spline32(r * hinv, hinv, g, wv);
    } else {
      g = ri * ri * ri;
      wv = ri;
    }
  } else {
    wv = __builtin_amdgcn_rsqf(r2 + (kExt && k.soft ? e * e : k.eps2));
    g = 0.0f;  // Plummer: formed below as wv^3, sharing G m wv with the potential
  }
  float S = 1.0f, pf = 1.0f;
  if (k.cutoff) {
    // the hardware square root (about 1 ulp); r2 = 0 (coincident partners)
    // gives r = 0
    const float r = __builtin_amdgcn_sqrtf(r2);
    // v = u sqrt(log2 e) with u = r / (2 r_s) (k.inv2rs holds the product), so
    // that exp(-u^2) = 2^(-v^2) is one exp2; the constants in u are rescaled
    const float v = r * k.inv2rs;
    const float e = __builtin_amdgcn_exp2f(-(v * v));
    const float t = __builtin_amdgcn_rcpf(1.0f + kAsPv * v);
    const float ec = t * (kAsA1 + t * (kAsA2 + t * (kAsA3 + t * (kAsA4 + t * kAsA5)))) * e;
    S = ec + kTwoOverSqrtPiV * v * e;
    pf = ec;
  }
  float fs, ps;  // G m (1/r^3) S and G m (1/r) erfc, softened
  if (kExt && k.spline) {
    fs = gm * g * S;
    ps = gm * wv * pf;
  } else {
    const float gw = gm * wv;
    ps = gw * pf;
    fs = gw * (wv * wv) * S;
  }
  const double f = (double)fs;
  ax = fma(f, (double)dx, ax);
  ay = fma(f, (double)dy, ay);
  az = fma(f, (double)dz, az);
  ph -= (double)ps;
}

// 2^23 + a as a float, exactly, for 0 <= a < 2^23.
__device__ inline float biased(int a) { return __int_as_float(0x4B000000 | a); }

__device__ inline int wrap_cells(int d) {
  // the periodic box is 2^22 half-cells long
  const int hi = d > (1 << 21) ? d - (1 << 22) : d;
  return d < -(1 << 21) ? d + (1 << 22) : hi;
}

__device__ inline float wrap_box(float d, const Consts32 &k) {
  const float hi = d > k.half_box ? d - k.box : d;
  return d < -k.half_box ? d + k.box : hi;
}

__device__ inline int wave_max_i32(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return __builtin_amdgcn_readfirstlane(v);
}

__device__ inline int wave_min_i32(int v) { return -wave_max_i32(-v); }

// List entries (float4).  A monopole: (offset, mass), mass >= 0, already
// known to pass the cutoff.  A leaf: (offset of the leaf's centre of mass, tag), the
// tag's bits as laid out by leaf_tag_bits.
__device__ inline float leaf_tag(uint32_t first, uint32_t n, bool wrap) {
  return __uint_as_float(leaf_tag_bits(first, n, wrap));
}

// Evaluate and empty every lane's list, lane-parallel: each step every lane
// takes the next partner of its own list (a monopole, or the next particle
// of a leaf entry, read with a per-lane load), in list order.
// A lane's list position is kept as the byte offset of its slot in `list`
// (row * kListRow + lane * 16), which is the LDS address the slot's load or
// store takes, so that no address is formed per entry.
constexpr uint32_t kListRow = kWalk32Threads * sizeof(float4);
__device__ inline float4 &list_at(float4 (*list)[kWalk32Threads], uint32_t off) {
  return *reinterpret_cast<float4 *>(reinterpret_cast<char *>(list) + off);
}

template <int kCap, bool kExt, bool kSoft>
__device__ inline void flush(const WalkArgs &A, float4 (*list)[kWalk32Threads], float (*lsoft)[kWalk32Threads],
                             float eif, uint32_t lane, uint32_t p, uint32_t &cnt, const Consts32 &k, double &ax,
                             double &ay, double &az, double &ph, uint32_t &ni) {
#pragma clang fp contract(fast)
  // cnt: this lane's next free slot (byte offset); e: the entry being read
  uint32_t e = lane * (uint32_t)sizeof(float4), j = 0;
  while (__ballot(e < cnt)) {
    if (e < cnt) {
      const float4 q = list_at(list, e);
      const uint32_t tag = __float_as_uint(q.w);
      float dx = q.x, dy = q.y, dz = q.z, m = q.w;
      float r2 = fmaf(dz, dz, fmaf(dx, dx, dy * dy));
      bool use = true;
      float es = 0.0f;                    // the pair's softening length (k.soft)
      if (kSoft && k.soft && !(tag & kTagLeaf)) es = lsoft[e / kListRow][lane];
      if (tag & kTagLeaf) {
        const uint32_t first = tag & kTagFirst, n = ((tag >> 27) & 7u) + 1u;
        const float4 pq = A.part32[first + j];
        dx += pq.x;
        dy += pq.y;
        dz += pq.z;
        if (tag & kTagWrap) {
          dx = wrap_box(dx, k);
          dy = wrap_box(dy, k);
          dz = wrap_box(dz, k);
        }
        m = pq.w;
        r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        use = (first + j != p) && (!k.cutoff || r2 < k.rc2);
        if (kSoft && k.soft) {
          const float ej = (float)A.seps[first + j];
          es = eif > ej ? eif : ej;
        }
        ++j;
        if (j == n) {
          j = 0;
          e += kListRow;
        }
      } else {
        e += kListRow;
      }
      if (use) {
        eval32<kExt>(dx, dy, dz, r2, m, k, ax, ay, az, ph, es);
        ++ni;
      }
    }
  }
  cnt = lane * (uint32_t)sizeof(float4);
}

// kMode: 0 = cutoff and periodicity read from each box; 1 = cutoff, open
// boundaries; 2 = cutoff, periodic; 3 = plain Newtonian, open boundaries.
// kExt: the spline softening and the relative criterion are read from each
// box (only with kMode 0); kSoft (with kExt): per-particle softening lengths.
// kWide: node records addressed with 64-bit offsets (forests whose records
// exceed 4 GiB); otherwise a record's byte offset is one 32-bit scalar
// product, which the scalar load takes as its offset register.
template <int kCap, int kMode, bool kExt, bool kSoft = false, bool kWide = false>
// With 4-deep lists every variant fits 8 waves per SIMD (64 vector and at
// most 96 scalar registers, no spills), which hides more latency than the
// 7 that the scalar registers would otherwise allow.
__global__ __launch_bounds__(kWalk32Threads)
__attribute__((amdgpu_waves_per_eu(kCap == 4 ? 8 : 1, 8))) void k_walk32(WalkArgs A) {
#pragma clang fp contract(fast)
  __shared__ float4 list[kCap][kWalk32Threads];
  __shared__ float lsoft[kSoft ? kCap : 1][kWalk32Threads];  // monopoles' softening lengths
  const uint32_t lane = threadIdx.x;
  device_counts(A);
  GroupQueue Q = make_queue(A);
  while (true) {
    const uint32_t g = pop_group(Q, lane);
    if (g >= A.n_groups) break;
    const GroupRef gr = group_of(A, g);
    const BoxDev bx = ld(A.boxes + gr.box);
    const bool kCut = kMode == 0 ? bx.cutoff != 0 : kMode != 3;
    const bool kPer = kMode == 0 ? bx.periodic != 0 : kMode == 2;
    Consts32 k;
    k.G = bx.Gf;
    k.eps2 = bx.eps2f;
    k.inv2rs = bx.inv2rsf * kSqrtLog2e;
    k.rc2 = bx.rc2f;
    k.theta2 = bx.theta2f;
    k.h22 = bx.h22f;
    k.box = bx.Lf;
    k.half_box = 0.5f * bx.Lf;
    k.cutoff = kCut;
    k.periodic = kPer;
    k.spline = kExt && bx.spline;
    k.hs2 = bx.hsf * bx.hsf;
    k.hinv = bx.hinvf;
    k.soft = kSoft && A.seps != nullptr && bx.epsp != nullptr;  // this box has per-particle lengths
    const bool relative = kExt && bx.relative;
    uint32_t p = 0, slot = 0;
    const bool valid = lane_target(A, gr, bx, lane, p, slot);
    const float eif = k.soft && valid ? (float)A.seps[p] : 0.0f;  // the target's softening length
    // relative criterion: open iff G M side^2 > alpha |a_old| r^4 (the
    // record's mass is G M)
    float aol = 0.0f;
    if (relative && valid) {
      const double *v = A.a_old + 3ull * (A.perm[p] - bx.p_off);
      aol = (float)(bx.alpha * sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
    }
    // lane origin: centre of the target's level-21 cell, in half-cells
    int o0 = 0, o1 = 0, o2 = 0;
    float xr = 0.0f, yr = 0.0f, zr = 0.0f;
    if (valid) {
      uint32_t cc[3];
      key_cell(A.skeys[p], bx.curve, cc);
      o0 = 2 * (int)cc[0] + 1;
      o1 = 2 * (int)cc[1] + 1;
      o2 = 2 * (int)cc[2] + 1;
      const double h22 = bx.L * 0x1p-22;
      const double4 q = A.part64[p];
      xr = (float)(q.x - (bx.lo[0] + (double)o0 * h22));
      yr = (float)(q.y - (bx.lo[1] + (double)o1 * h22));
      zr = (float)(q.z - (bx.lo[2] + (double)o2 * h22));
    }
    // Offsets between a lane's origin o and a node centre c, in half-cells.
    // Periodic box (2^22 half-cells): with g the first lane's origin and
    // E = max |o - g| over the group's lanes, the scalar unit reduces c - g
    // modulo 2^22 into [-2^21, 2^21) once per node, and each lane subtracts
    // its o - g.  For the root (centre at half the box) that is c - o
    // itself.  For every other node (at most half a box wide) it is the
    // minimum image whenever the node is within reach of the lane, as long
    // as r_cut + E stays below a quarter of the box; a node out of reach is
    // pruned in either image.  Wider groups (also those that straddle the
    // box boundary) take the minimum image per lane.
    // Groups whose targets all lie farther than r_cut from every face of the
    // box take c - o as it is: a node for which that is not the minimum
    // image lies beyond the face nearest the target, so none of its points
    // is within r_cut of it in either image.  Such a node is pruned in the
    // raw image (it is more than a quarter box away); in the minimum image it
    // may be visited, but it contributes nothing, so the contributions and
    // their order are the same.
    const int g0 = __builtin_amdgcn_readfirstlane(o0), g1 = __builtin_amdgcn_readfirstlane(o1),
              g2 = __builtin_amdgcn_readfirstlane(o2);
    constexpr int kHalf = 1 << 21, kMask = (1 << 22) - 1;
    const int gq0 = g0 - kHalf, gq1 = g1 - kHalf, gq2 = g2 - kHalf;
    // per-lane term subtracted from the reduced node centre: (o - g) + 2^21
    const int q0 = o0 - gq0, q1 = o1 - gq1, q2 = o2 - gq2;
    bool lane_wrap = false, interior = false;
    if (kPer) {
      const float rc = sqrtf(k.rc2);
      const int e = valid ? max(abs(o0 - g0), max(abs(o1 - g1), abs(o2 - g2))) : 0;
      lane_wrap = !((float)wave_max_i32(e) + rc / k.h22 < (float)((1 << 20) - (1 << 16)));
      // half-cells from the lane origin to the nearest face; the target is
      // within one half-cell of its origin
      const int df = valid ? min(min(min(o0, o1), o2), (1 << 22) - max(max(o0, o1), o2)) : (1 << 22);
      interior = !A.no_interior && (float)(wave_min_i32(df) - 2) * k.h22 > rc;
    }
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    // cnt: the byte offset of this lane's next free list slot (see list_at)
    uint32_t ni = 0, cnt = lane * (uint32_t)sizeof(float4);
    const uint32_t cfull = cnt + kCap * kListRow;
    const uint32_t nend = bx.node_end;
    // A lane is active at node n while next <= n: an opening lane keeps its
    // value and so stays active in the subtree; a lane that prunes or accepts
    // n moves next to skip(n).
    uint32_t next = valid ? bx.root : nend;
    // kForm: 0 = c - o as it is (open boxes, interior groups); 1 = reduced
    // against the first lane; 2 = the minimum image per lane
    auto walk = [&](auto form_t) {
      constexpr int kForm = decltype(form_t)::value;
      // Offsets in half-cells become floats exactly without a per-lane
      // conversion: for 0 <= a, b < 2^23 the float with bit pattern
      // 0x4B000000 | a is 2^23 + a, and (2^23 + a) - (2^23 + b) = a - b
      // exactly.  The node's term is a scalar OR, the lane's is fixed.
      const float qb0 = biased(kForm == 1 ? q0 : o0), qb1 = biased(kForm == 1 ? q1 : o1),
                  qb2 = biased(kForm == 1 ? q2 : o2);
      // A leaf of more than 8 particles takes one list entry per 8 of its
      // particles: the wave stays on it (pend = the next particle offset)
      // until the lanes that opened it have appended every entry.  While the
      // wave stays, those are exactly the lanes with next <= n (an opening
      // lane keeps next, every other lane is past n).
      uint32_t pend = 0;
      // the next node's record is read after the decision (the wave's other
      // work and the other waves on the SIMD cover the scalar load)
      for (uint32_t n = bx.root; n < nend;) {
        const WNode w = kWide ? ldw(A.wnode + n)
                              : ldw((const WNode *)((const char *)A.wnode + n * (uint32_t)sizeof(WNode)));
        const uint32_t cf = w.cf;
        // room for this visit's entry
        if (__ballot(cnt >= cfull)) flush<kCap, kExt, kSoft>(A, list, lsoft, eif, lane, p, cnt, k, ax, ay, az, ph, ni);
        float f0, f1, f2;  // node centre minus lane origin, in half-cells (exact)
        if (kPer && kForm == 1) {
          f0 = biased((w.c[0] - gq0) & kMask) - qb0;
          f1 = biased((w.c[1] - gq1) & kMask) - qb1;
          f2 = biased((w.c[2] - gq2) & kMask) - qb2;
        } else if (kPer && kForm == 2) {
          f0 = (float)wrap_cells((w.c[0] & kMask) - o0);
          f1 = (float)wrap_cells((w.c[1] & kMask) - o1);
          f2 = (float)wrap_cells((w.c[2] & kMask) - o2);
        } else {  // the record holds the node's term already
          f0 = __int_as_float(w.c[0]) - qb0;
          f1 = __int_as_float(w.c[1]) - qb1;
          f2 = __int_as_float(w.c[2]) - qb2;
        }
        const float dcx = f0 * k.h22 - xr, dcy = f1 * k.h22 - yr, dcz = f2 * k.h22 - zr;
        const float mdc = fmaxf(fmaxf(fabsf(dcx), fabsf(dcy)), fabsf(dcz));
        // a leaf's record holds its list tag (sign bit set) where an internal
        // node's holds its skip (node indices stay below 2^31)
        const uint32_t ns = (int32_t)w.a < 0 ? n + 1 : w.a;
        // the rare cases (a big leaf, offsets that may need the minimum
        // image) take the general path; the common visit below has no
        // branch of its own
        if (pend | (cf & (kWBig | (kPer ? kWWrap : 0u)))) {
          const uint32_t lc = cf & kWCount;
          const bool wrapd = kPer && (cf & kWWrap) != 0;
          if (pend) {
            if (next <= n) {
              list_at(list, cnt) = make_float4(dcx + w.o[0], dcy + w.o[1], dcz + w.o[2],
                                               leaf_tag((w.a & kTagFirst) + pend, min(8u, lc - pend), wrapd));
              cnt += kListRow;
            }
            pend += 8;
            if (pend >= lc) {
              pend = 0;
              ++n;
            }
            continue;
          }
          float dx = dcx + w.o[0], dy = dcy + w.o[1], dz = dcz + w.o[2];
          if (wrapd) {
            dx = wrap_box(dx, k);
            dy = wrap_box(dy, k);
            dz = wrap_box(dz, k);
          }
          const float r2 = fmaf(dz, dz, fmaf(dx, dx, dy * dy));
          const bool act = next <= n;
          const bool live = act && !(kCut && mdc > w.reach);
          const bool far_open = relative ? (w.m * w.side2 > aol * (r2 * r2)) : (w.side2 > r2);
          bool open = far_open || (mdc < w.near);
          float emono = 0.0f;
          if (kSoft && k.soft) {
            const float emax = (float)*cptr(A.semax + n), emin = (float)*cptr(A.semin + n);
            const float hm = 2.8f * emax;
            if (emin < emax && emax > eif && r2 < hm * hm) open = true;
            emono = eif > emax ? eif : emax;
          }
          const bool contrib = live && !open && (!kCut || r2 < k.rc2);
          const bool open_here = live && open;
          list_at(list, cnt) = make_float4(dx, dy, dz, open_here ? leaf_tag(w.a & kTagFirst, min(8u, lc), wrapd) : w.m);
          if (kSoft) lsoft[cnt / kListRow][lane] = emono;
          cnt += (contrib || (open_here && (cf & kWLeaf) != 0)) ? kListRow : 0u;
          if (act && !open_here) next = ns;
          const bool opened = __ballot(open_here) != 0;
          if ((cf & kWBig) && opened) {
            pend = 8;
          } else {
            n = opened ? n + 1 : max(ns, n + 1);
          }
          continue;
        }
        const bool act = next <= n;
        const bool live = act && !(kCut && mdc > w.reach);
        // every active lane prunes n: the wave skips its subtree (the lanes'
        // next stays at or before n, which is where the walk resumes)
        if (kCut && !__ballot(live)) {
          n = max(ns, n + 1);
          continue;
        }
        const float dx = dcx + w.o[0], dy = dcy + w.o[1], dz = dcz + w.o[2];
        const float r2 = fmaf(dz, dz, fmaf(dx, dx, dy * dy));
        const bool far_open = relative ? (w.m * w.side2 > aol * (r2 * r2)) : (w.side2 > r2);
        bool open = far_open || (mdc < w.near);
        float emono = 0.0f;  // the monopole's softening length (k.soft)
        if (kSoft && k.soft) {
          const float emax = (float)*cptr(A.semax + n), emin = (float)*cptr(A.semin + n);
          const float hm = 2.8f * emax;
          if (emin < emax && emax > eif && r2 < hm * hm) open = true;
          emono = eif > emax ? eif : emax;
        }
        const bool contrib = live && !open && (!kCut || r2 < k.rc2);
        const bool open_here = live && open;
        // one entry: the offset of n's centre of mass and either its mass
        // (an accepted monopole) or, at an opened leaf, the leaf's tag (its
        // particles' offsets are stored from that centre of mass).  Every
        // lane writes its next slot; only a real entry advances it.
        const float4 entry = make_float4(dx, dy, dz, open_here ? __uint_as_float(w.a) : w.m);
        list_at(list, cnt) = entry;
        if (kSoft) lsoft[cnt / kListRow][lane] = emono;
        cnt += (contrib || (open_here && (cf & kWLeaf) != 0)) ? kListRow : 0u;
        // a lane past n is past all of n's subtree, so max() leaves it as
        // it is, and moves an active lane that did not open n to skip(n)
        next = open_here ? next : max(next, ns);
        // the lanes still at or before n are exactly those that opened it; a
        // leaf's skip is n + 1; a skip always moves forward
        n = __ballot(next <= n) ? n + 1 : max(ns, n + 1);
      }
    };
    if (kPer && lane_wrap) walk(std::integral_constant<int, 2>{});
    else if (kPer && !interior) walk(std::integral_constant<int, 1>{});
    else walk(std::integral_constant<int, 0>{});
    flush<kCap, kExt, kSoft>(A, list, lsoft, eif, lane, p, cnt, k, ax, ay, az, ph, ni);
    if (valid) write_out(A, bx, slot, ax, ay, az, ph, ni);
  }
}

// ------------------------------------------------- screened FP64 walk --
// The FP64 walk's decisions compare FP64 quantities with per-node
// thresholds: the largest centre offset max|dc| with r_cut + side/2 (prune)
// and 0.6 side (near), r^2 with side^2/theta^2 (open) and r_cut^2 (cutoff).
// This walk forms the same quantities in FP32 the way the mixed walk does
// (node centres exact in half-cells, each target's offset from its cell
// centre rounded once, centre-of-mass offsets rounded once) and takes a
// comparison's outcome from the FP32 value when it lies outside a band
// around the threshold that the FP32 error cannot cross.  With h half a
// level-21 cell, the FP32 max|dc| is within 2^-22.4 (max|dc| + h) +
// 2^-51 (|lo| + L) of the FP64 one, and near a threshold max|dc| >= 1.2 h;
// r^2 is within 2^-18.5 r^2 of the FP64 value near either r^2 threshold
// when theta <= 1 (there |offset| <= 1.5 r and h <= r/2).  With the
// thresholds' own FP32 rounding (at most 5 x 2^-24) the distance tests need
// under 2^-20.4 and the r^2 tests under 2^-18.3 relative; the bands are
// 64 ulps (at least 2^-18) and 1024 ulps (at least 2^-14).  The relative
// criterion, G M side^2 > alpha |a_old| r^4, has no theta to bound r by the
// side; but where the near test is certainly false the centre of mass is at
// least 0.1 side from the target (it lies within side/2 of the centre on the
// axis where |dc| >= 0.6 side), so r^2 is within 2^-16.3 r^2 and the
// comparison within 2^-15.2 of its FP64 value; its band is 4096 ulps (at
// least 2^-12).  Where the near test is certainly true the node is opened
// whatever the criterion says.  With per-particle lengths a node is also
// opened when r^2 < (2.8 emax)^2 (its lengths differing and its largest
// above the target's, comparisons made in FP64): the same r^2 bound with a
// 1024-ulp band.
// A lane with a value inside a band, every lane at a node whose offsets may
// need the minimum image (kWWrap, which includes the two top levels of a
// periodic box), and every lane of a box outside the bounds above (theta >
// 1 with the geometric criterion, a root corner beyond 64 root sides from
// the origin, periodic without a cutoff) takes the FP64 walk's tests in its
// own expressions (tests64).
// List entries are references, a node (monopole) or a leaf's particle
// range, with the FP64 walk's image flag, and the evaluation forms each FP64
// offset from the FP64 centre of mass or particle and the target as the
// FP64 walk does.  Decisions, offsets, pair terms and summation order are
// those of k_walk64, so the results are the same to the bit.

// Entry: x = node (monopole) or first particle (leaf); y = item count |
// kELeaf | kEWrap (the offsets take the minimum image).
constexpr uint32_t kELeaf = 0x80000000u, kEWrap = 0x40000000u;
constexpr uint32_t kScreenRow = kWalk32Threads * sizeof(uint2);
constexpr uint32_t kBandC = 64, kBandR = 1024, kBandRel = 4096;  // bands, in ulps of the FP32 value
constexpr int kScreenCap = 4;  // list entries per lane

// |bits(v) - bits(t)| < band for non-negative v and positive t, given
// lo = bits(t) - band: one unsigned comparison
__device__ inline bool in_band(float v, uint32_t lo, uint32_t band) { return __float_as_uint(v) - lo < 2u * band; }

// |a_old| of a target, in the FP64 walk's expression.
__device__ inline double norm3_64(const double *v) {
#pragma clang fp contract(off)
  return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

// The FP64 walk's tests of a node (cube centre and side cs, moments mm) for a
// target at xi, in its expressions: the cutoff prune, the opening criterion
// (geometric, or relative with the target's |a_old| aold) and the cutoff
// test of the monopole.
// soft: per-particle lengths, with the node's length range (emin, emax) and
// the target's length ei (the mixed-softening opening test).
__device__ inline void tests64(const double4 &cs, const Mom64 &mm, const double4 &xi, bool wrap, const BoxDev &bx,
                               bool relative, double aold, bool soft, double emin, double emax, double ei,
                               bool &pruned, bool &open, bool &within) {
#pragma clang fp contract(off)
  const double side = cs.w, box = bx.box;
  double dcx = cs.x - xi.x, dcy = cs.y - xi.y, dcz = cs.z - xi.z;
  minimg3(dcx, dcy, dcz, wrap, box);
  pruned = false;
  if (bx.cutoff) {
    const double reach = bx.rcut + 0.5 * side;
    pruned = fabs(dcx) > reach || fabs(dcy) > reach || fabs(dcz) > reach;
  }
  double dx = mm.cx - xi.x, dy = mm.cy - xi.y, dz = mm.cz - xi.z;
  minimg3(dx, dy, dz, wrap, box);
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double near = 0.6 * side;
  const bool far_open = relative ? (bx.G * mm.m * side * side > bx.alpha * aold * r2 * r2) : (side * side > bx.theta2 * r2);
  open = far_open || (fabs(dcx) < near && fabs(dcy) < near && fabs(dcz) < near);
  if (soft && emin < emax && emax > ei) {
    const double hm = 2.8 * emax;
    if (r2 < hm * hm) open = true;
  }
  within = !bx.cutoff || r2 < bx.rc2;
}

// (2.8 emax)^2 in the FP64 walk's expression.
__device__ inline double hm2_64(double emax) {
#pragma clang fp contract(off)
  const double hm = 2.8 * emax;
  return hm * hm;
}

// kMode as for k_walk32; kTail as for k_walk64; kCap: list entries per lane;
// kExt: the softening kernel, the opening criterion and per-particle lengths
// are read from each box (spline, relative-criterion and per-particle-length
// boxes).
// Seven waves per SIMD (at most 72 vector registers, a few bytes of
// scratch; the target's FP64 position is reloaded by the lanes that take the
// FP64 tests instead of being kept across the walk); the instance for the
// variant boxes takes six (80, some scratch: faster than five without) and
// the instances with the library erfc tail four (128, a few values in
// scratch, like the FP64 walk's instances with the tail).
template <int kMode, bool kTail, int kCap, bool kExt = false>
__global__ __launch_bounds__(kWalk32Threads) __attribute__((amdgpu_waves_per_eu(kTail ? 4 : (kExt ? 6 : 7), 8))) void k_walk64s(WalkArgs A) {
#pragma clang fp contract(fast)
  __shared__ uint2 list[kCap][kWalk32Threads];
  __shared__ double4 slots[kWalk32Threads];
  const uint32_t lane = threadIdx.x;
  device_counts(A);
  GroupQueue Q = make_queue(A);
  while (true) {
    const uint32_t g = pop_group(Q, lane);
    if (g >= A.n_groups) break;
    const GroupRef gr = group_of(A, g);
    const BoxDev bx = ld(A.boxes + gr.box);
    const bool kCut = kMode == 0 ? bx.cutoff != 0 : kMode != 3;
    const bool kPer = kMode == 0 ? bx.periodic != 0 : kMode == 2;
    uint32_t p = 0, slot = 0;
    const bool valid = lane_target(A, gr, bx, lane, p, slot);
    double4 xi = make_double4(0.0, 0.0, 0.0, 0.0);
    if (valid) xi = A.part64[p];
    // the FP64 walk's interior groups (no minimum image below level 1)
    bool interior = false;
    if (kPer) {
      const double box = bx.box, m = bx.rcut + 0x1p-40 * box;
      const bool inside = !valid || (xi.x >= m && xi.x <= box - m && xi.y >= m && xi.y <= box - m &&
                                     xi.z >= m && xi.z <= box - m);
      interior = bx.rcut <= 0.24 * box && __ballot(!inside) == 0;
    }
    // lane origin (the centre of the target's level-21 cell, in half-cells)
    // and the target's FP32 offset from it, as in the mixed walk
    int o0 = 0, o1 = 0, o2 = 0;
    float xr = 0.0f, yr = 0.0f, zr = 0.0f;
    if (valid) {
      uint32_t cc[3];
      key_cell(A.skeys[p], bx.curve, cc);
      o0 = 2 * (int)cc[0] + 1;
      o1 = 2 * (int)cc[1] + 1;
      o2 = 2 * (int)cc[2] + 1;
      const double h22 = bx.L * 0x1p-22;
      xr = (float)(xi.x - (bx.lo[0] + (double)o0 * h22));
      yr = (float)(xi.y - (bx.lo[1] + (double)o1 * h22));
      zr = (float)(xi.z - (bx.lo[2] + (double)o2 * h22));
    }
    const float h22f = bx.h22f, rc2f = bx.rc2f;
    // the relative criterion: the target's |a_old| (FP64, and alpha |a_old|
    // in FP32 for the screen; the record's mass is G M, its side2 side^2)
    const bool relative = kExt && bx.relative;
    double aold = 0.0;
    float aol = 0.0f;
    if (relative && valid) {
      aold = norm3_64(A.a_old + 3ull * (A.perm[p] - bx.p_off));
      aol = (float)(bx.alpha * aold);
    }
    // per-particle lengths: the target's (FP64, as the FP64 walk reads it)
    const bool soft = kExt && A.seps != nullptr && bx.epsp != nullptr;
    const double ei = soft && valid ? A.seps[p] : bx.eps;
    const double lim = 64.0 * bx.L;
    const bool screened = (relative || bx.theta2 <= 1.0) && fabs(bx.lo[0]) <= lim && fabs(bx.lo[1]) <= lim &&
                          fabs(bx.lo[2]) <= lim && (!kPer || kCut);
    // a target farther than its cell from the cell's centre (not one inside
    // the root cube) is not screened either
    const bool lane_exact = !screened || fmaxf(fmaxf(fabsf(xr), fabsf(yr)), fabsf(zr)) > 1.5f * h22f;
    const int g0 = __builtin_amdgcn_readfirstlane(o0), g1 = __builtin_amdgcn_readfirstlane(o1),
              g2 = __builtin_amdgcn_readfirstlane(o2);
    constexpr int kHalf = 1 << 21, kMask = (1 << 22) - 1;
    const int gq0 = g0 - kHalf, gq1 = g1 - kHalf, gq2 = g2 - kHalf;
    const int q0 = o0 - gq0, q1 = o1 - gq1, q2 = o2 - gq2;
    bool lane_wrap = false;
    if (kPer) {
      const float rc = sqrtf(rc2f);
      const int e = valid ? max(abs(o0 - g0), max(abs(o1 - g1), abs(o2 - g2))) : 0;
      lane_wrap = !((float)wave_max_i32(e) + rc / h22f < (float)((1 << 20) - (1 << 16)));
    }
    // the FP64 walk's image flag below level 1
    const uint32_t gwrap = kPer && !interior ? kEWrap : 0u;
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    // cnt: byte offset of this lane's next free list slot
    uint32_t ni = 0, cnt = lane * (uint32_t)sizeof(uint2);
    const uint32_t cfull = cnt + kCap * kScreenRow;
    const uint32_t nend = bx.node_end;
    uint32_t next = valid ? bx.root : nend;
    auto flush = [&]() __attribute__((always_inline)) {
      const uint32_t nent = (cnt - lane * (uint32_t)sizeof(uint2)) / kScreenRow;
      flush_rows64<kCap>(
          slots, lane, p, nent,
          [&](uint32_t e) __attribute__((always_inline)) {
            const uint32_t y = list[e][lane].y;
            return (y & kELeaf) ? (y & kCountMask) : 1u;
          },
          [&](uint32_t l, uint32_t e, uint32_t j, uint32_t po, double4 &t) __attribute__((always_inline)) {
#pragma clang fp contract(off)
            const uint2 q = list[e][l];
            const double4 xo = A.part64[po];
            double dx, dy, dz, m, es = bx.eps;
            bool use = true;
            if (q.y & kELeaf) {
              const uint32_t i = q.x + j;
              use = i != po;
              const double4 sp = A.part64[i];
              dx = sp.x - xo.x;
              dy = sp.y - xo.y;
              dz = sp.z - xo.z;
              m = sp.w;
              if (soft) {
                const double ej = A.seps[i], eo = A.seps[po];
                es = eo > ej ? eo : ej;
              }
            } else {
              const Mom64 mm = A.mom64[q.x];
              dx = mm.cx - xo.x;
              dy = mm.cy - xo.y;
              dz = mm.cz - xo.z;
              m = mm.m;
              if (soft) {
                // the monopole's length: the larger of the target's and the node's largest
                const double eo = A.seps[po], emax = A.semax[q.x];
                es = eo > emax ? eo : emax;
              }
            }
            minimg3(dx, dy, dz, (q.y & kEWrap) != 0, bx.box);
            return use && pair64_terms<kExt, kTail>(dx, dy, dz, m, es, bx, t);
          },
          ax, ay, az, ph, ni);
      cnt = lane * (uint32_t)sizeof(uint2);
    };
    // kForm as in the mixed walk: 0 = c - o as it is (open boxes, the FP64
    // walk's interior groups), 1 = reduced against the first lane, 2 = the
    // minimum image per lane
    auto walk = [&](auto form_t) {
      constexpr int kForm = decltype(form_t)::value;
      const float qb0 = biased(kForm == 1 ? q0 : o0), qb1 = biased(kForm == 1 ? q1 : o1),
                  qb2 = biased(kForm == 1 ? q2 : o2);
      for (uint32_t n = bx.root; n < nend;) {
        const WNode w = ldw((const WNode *)((const char *)A.wnode + n * (uint32_t)sizeof(WNode)));
        if (__ballot(cnt >= cfull)) flush();
        float f0, f1, f2;
        if (kPer && kForm == 1) {
          f0 = biased((w.c[0] - gq0) & kMask) - qb0;
          f1 = biased((w.c[1] - gq1) & kMask) - qb1;
          f2 = biased((w.c[2] - gq2) & kMask) - qb2;
        } else if (kPer && kForm == 2) {
          f0 = (float)wrap_cells((w.c[0] & kMask) - o0);
          f1 = (float)wrap_cells((w.c[1] & kMask) - o1);
          f2 = (float)wrap_cells((w.c[2] & kMask) - o2);
        } else {
          f0 = __int_as_float(w.c[0]) - qb0;
          f1 = __int_as_float(w.c[1]) - qb1;
          f2 = __int_as_float(w.c[2]) - qb2;
        }
        const float dcx = f0 * h22f - xr, dcy = f1 * h22f - yr, dcz = f2 * h22f - zr;
        const float mdc = fmaxf(fmaxf(fabsf(dcx), fabsf(dcy)), fabsf(dcz));
        const uint32_t cf = w.cf;
        const bool leaf = (cf & kWLeaf) != 0;
        const uint32_t ns = leaf ? n + 1 : w.a;
        const bool act = next <= n;
        const bool amb_w = lane_exact || (kPer && (cf & kWWrap) != 0);
        const bool amb_c = amb_w || (kCut && in_band(mdc, __float_as_uint(w.reach) - kBandC, kBandC));
        // every active lane certainly prunes n: the wave skips its subtree
        if (kCut && !__ballot(act && (amb_c || !(mdc > w.reach)))) {
          n = max(ns, n + 1);
          continue;
        }
        const float dx = dcx + w.o[0], dy = dcy + w.o[1], dz = dcz + w.o[2];
        const float r2 = fmaf(dz, dz, fmaf(dx, dx, dy * dy));
        bool live = act && !(kCut && mdc > w.reach);
        const float gms2 = w.m * w.side2, ar4 = aol * (r2 * r2);  // relative: G M side^2, alpha |a_old| r^4
        bool open = (relative ? gms2 > ar4 : w.side2 > r2) || mdc < w.near;
        bool within = !kCut || r2 < rc2f;
        // per-particle lengths: the node is also opened when its lengths
        // differ, its largest exceeds the target's and r < 2.8 emax (the
        // length comparisons are made in FP64, exactly; r^2 is screened)
        bool amb_s = false;
        double emin = 0.0, emax = 0.0;
        if (kExt && soft) {
          emax = *cptr(A.semax + n);
          emin = *cptr(A.semin + n);
          if (emin < emax && emax > ei) {
            const float hm2 = (float)hm2_64(emax);
            open = open || r2 < hm2;
            amb_s = in_band(r2, __float_as_uint(hm2) - kBandR, kBandR);
          }
        }
        const bool amb = amb_c || amb_s || in_band(mdc, __float_as_uint(w.near) - kBandC, kBandC) ||
                         (relative ? in_band(ar4, __float_as_uint(gms2) - kBandRel, kBandRel)
                                   : in_band(r2, __float_as_uint(w.side2) - kBandR, kBandR)) ||
                         (kCut && in_band(r2, __float_as_uint(rc2f) - kBandR, kBandR));
        uint32_t ewrap = gwrap;
        if (__ballot(act && amb)) {
          const Topo t = ld(A.topo + n);
          const double4 cs = ld(A.cen64 + n);
          const Mom64 mm = ld(A.mom64 + n);
          if (act && amb) {
            const bool wrap = kPer && !(interior && (int)(t.b >> kCountBits) >= 2);
            bool pruned;
            const double4 xq = A.part64[p];  // reloaded: not kept in registers across the walk
            tests64(cs, mm, xq, wrap, bx, relative, aold, kExt && soft, emin, emax, ei, pruned, open, within);
            live = !pruned;
            ewrap = wrap ? kEWrap : 0u;
          }
        }
        const bool open_here = live && open;
        const bool take = live && (open ? leaf : within);
        // every lane writes its next slot; only a real entry advances it
        *reinterpret_cast<uint2 *>(reinterpret_cast<char *>(list) + cnt) =
            open_here ? make_uint2(w.a & kTagFirst, (cf & kWCount) | kELeaf | ewrap) : make_uint2(n, 1u | ewrap);
        cnt += take ? kScreenRow : 0u;
        next = open_here ? next : max(next, ns);
        n = __ballot(next <= n) ? n + 1 : max(ns, n + 1);
      }
    };
    if (kPer && !interior && lane_wrap) walk(std::integral_constant<int, 2>{});
    else if (kPer && !interior) walk(std::integral_constant<int, 1>{});
    else walk(std::integral_constant<int, 0>{});
    flush();
    if (valid) write_out(A, bx, slot, ax, ay, az, ph, ni);
  }
}

// ------------------------------------------- group-shared interaction lists --
// One walk per group of targets (the paper's grouped neighbour search
// applied to the tree walk): at a visited node every lane applies the
// per-target pruning and opening tests to its own target; the node is
// skipped when it is pruned for every lane, accepted for the whole group
// when no lane that keeps it would open it, and opened when one would.
// Accepted monopoles and the particles of opened leaves go to one list per
// wave, and every lane evaluates the whole list for its own target (with
// its own cutoff and self test), in traversal order.  Evaluation is thus
// uniform across the wave, at the price of more interactions per target;
// the result depends on the grouping.

// FP64: the same arithmetic as the per-target FP64 walk, evaluated at the node.
template <bool kExt, bool kTail>
__global__ __launch_bounds__(256) void k_walkg64(WalkArgs A) {
#pragma clang fp contract(off)
  const uint32_t lane = threadIdx.x & 63;
  device_counts(A);
  GroupQueue Q = make_queue(A);
  while (true) {
    const uint32_t g = pop_group(Q, lane);
    if (g >= A.n_groups) break;
    const GroupRef gr = group_of(A, g);
    const BoxDev bx = ld(A.boxes + gr.box);
    uint32_t p = 0, slot = 0;
    const bool valid = lane_target(A, gr, bx, lane, p, slot);
    double4 xi = make_double4(0.0, 0.0, 0.0, 0.0);
    if (valid) xi = A.part64[p];
    double aold = 0.0;
    const bool relative = kExt && bx.relative;
    if (valid && relative) {
      const double *v = A.a_old + 3ull * (A.perm[p] - bx.p_off);
      aold = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    }
    const bool periodic = bx.periodic;
    const double box = bx.box;
    // as in the per-target FP64 walk: a group farther than r_cut from every
    // periodic face needs the minimum image only for the nodes of levels 0
    // and 1, and never for particle offsets (a particle more than half a box
    // away is beyond the cutoff in either image)
    bool interior = false;
    if (periodic) {
      const double m = bx.rcut + 0x1p-40 * box;
      const bool inside = !valid || (xi.x >= m && xi.x <= box - m && xi.y >= m && xi.y <= box - m &&
                                     xi.z >= m && xi.z <= box - m);
      interior = bx.rcut <= 0.24 * box && __ballot(!inside) == 0;
    }
    const bool pwrap = periodic && !interior;
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    uint32_t ni = 0;
    uint32_t n = bx.root;
    const uint32_t nend = bx.node_end;
    while (n < nend) {
      const Topo t = ld(A.topo + n);
      const Mom64 mm = ld(A.mom64 + n);
      const bool leaf = (t.corner & kLeafBit) != 0;
      const uint32_t ns = leaf ? n + 1 : t.a;
      const int lev = (int)(t.b >> kCountBits);
      const bool wrap = periodic && !(interior && lev >= 2);
      // cube centre and side, computed once per build
      const double4 cs = ld(A.cen64 + n);
      const double side = cs.w, c0 = cs.x, c1 = cs.y, c2 = cs.z;
      bool live = false, open = false;
      double dx = 0.0, dy = 0.0, dz = 0.0;
      if (valid) {
        double dcx = c0 - xi.x, dcy = c1 - xi.y, dcz = c2 - xi.z;
        minimg3(dcx, dcy, dcz, wrap, box);
        bool pruned = false;
        if (bx.cutoff) {
          const double reach = bx.rcut + 0.5 * side;
          pruned = fabs(dcx) > reach || fabs(dcy) > reach || fabs(dcz) > reach;
        }
        dx = mm.cx - xi.x;
        dy = mm.cy - xi.y;
        dz = mm.cz - xi.z;
        minimg3(dx, dy, dz, wrap, box);
        if (!pruned) {
          live = true;
          const double r2 = dx * dx + dy * dy + dz * dz;
          const double near = 0.6 * side;
          const bool far_open = relative ? (bx.G * mm.m * side * side > bx.alpha * aold * r2 * r2)
                                         : (side * side > bx.theta2 * r2);
          open = far_open || (fabs(dcx) < near && fabs(dcy) < near && fabs(dcz) < near);
        }
      }
      const uint32_t nskip = ns > n ? ns : n + 1;  // a skip always moves forward
      uint32_t nn;
      if (!__ballot(live)) {
        nn = nskip;
      } else if (!__ballot(open)) {
        if (valid) pair64<kExt, kTail>(dx, dy, dz, mm.m, bx.eps, bx, ax, ay, az, ph, ni);
        nn = nskip;
      } else if (leaf) {
        const uint32_t f = t.a, cnt = t.b & kCountMask;
        for (uint32_t base = 0; base < cnt; base += 64) {
          double4 q = make_double4(0.0, 0.0, 0.0, 0.0);
          if (base + lane < cnt) q = A.part64[f + base + lane];
          const uint32_t m = min(64u, cnt - base);
          for (uint32_t j = 0; j < m; ++j) {
            const double qx = rdl(q.x, j), qy = rdl(q.y, j), qz = rdl(q.z, j), qm = rdl(q.w, j);
            if (valid && f + base + j != p) {
              double ex = qx - xi.x, ey = qy - xi.y, ez = qz - xi.z;
              minimg3(ex, ey, ez, pwrap, box);
              pair64<kExt, kTail>(ex, ey, ez, qm, bx.eps, bx, ax, ay, az, ph, ni);
            }
          }
        }
        nn = n + 1;
      } else {
        nn = n + 1;
      }
      n = nn;
    }
    if (valid) write_out(A, bx, slot, ax, ay, az, ph, ni);
  }
}

// Mixed: list entries hold a node centre and an FP32 offset from it (centre
// of mass, or particle), so each lane forms its own offset exactly as the
// per-target mixed walk does.  The centre is stored as the scalar term of
// that walk's exact half-cell offset (2^23 plus the centre reduced against
// the group's first lane), or, for open boxes and for groups that take the
// minimum image per lane, as the node record holds it (2^23 plus the
// centre, as float bits).
struct __attribute__((aligned(16))) GEntry {
  float c[3];
  uint32_t tag;  // bit 31: offsets may need the minimum image; bits 0..30: particle, or kGNoSelf
  float o[3];
  float m;
};
constexpr uint32_t kGWrap = 0x80000000u, kGNoSelf = 0x7fffffffu;
constexpr uint32_t kGroupCap = 128;

// 128 entries (4 KB of LDS per wave) leave room for 8 waves per SIMD, which
// pays for the extra flushes.
// kWide as for the per-target mixed walk: 64-bit node record offsets.
template <int kMode, bool kExt, bool kWide = false>
__global__ __launch_bounds__(kWalk32Threads) __attribute__((amdgpu_waves_per_eu(kExt ? 1 : 8, 8))) void k_walkg32(WalkArgs A) {
#pragma clang fp contract(fast)
  __shared__ GEntry list[kGroupCap];
  const uint32_t lane = threadIdx.x;
  device_counts(A);
  GroupQueue Q = make_queue(A);
  while (true) {
    const uint32_t g = pop_group(Q, lane);
    if (g >= A.n_groups) break;
    const GroupRef gr = group_of(A, g);
    const BoxDev bx = ld(A.boxes + gr.box);
    const bool kCut = kMode == 0 ? bx.cutoff != 0 : kMode != 3;
    const bool kPer = kMode == 0 ? bx.periodic != 0 : kMode == 2;
    Consts32 k;
    k.G = bx.Gf;
    k.eps2 = bx.eps2f;
    k.inv2rs = bx.inv2rsf * kSqrtLog2e;
    k.rc2 = bx.rc2f;
    k.theta2 = bx.theta2f;
    k.h22 = bx.h22f;
    k.box = bx.Lf;
    k.half_box = 0.5f * bx.Lf;
    k.cutoff = kCut;
    k.periodic = kPer;
    k.spline = kExt && bx.spline;
    k.hs2 = bx.hsf * bx.hsf;
    k.hinv = bx.hinvf;
    k.soft = false;  // per-particle softening is not offered with group lists
    const bool relative = kExt && bx.relative;
    uint32_t p = 0, slot = 0;
    const bool valid = lane_target(A, gr, bx, lane, p, slot);
    float aol = 0.0f;
    if (relative && valid) {
      const double *v = A.a_old + 3ull * (A.perm[p] - bx.p_off);
      aol = (float)(bx.alpha * sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));  // against G M
    }
    int o0 = 0, o1 = 0, o2 = 0;
    float xr = 0.0f, yr = 0.0f, zr = 0.0f;
    if (valid) {
      uint32_t cc[3];
      key_cell(A.skeys[p], bx.curve, cc);
      o0 = 2 * (int)cc[0] + 1;
      o1 = 2 * (int)cc[1] + 1;
      o2 = 2 * (int)cc[2] + 1;
      const double h22 = bx.L * 0x1p-22;
      const double4 q = A.part64[p];
      xr = (float)(q.x - (bx.lo[0] + (double)o0 * h22));
      yr = (float)(q.y - (bx.lo[1] + (double)o1 * h22));
      zr = (float)(q.z - (bx.lo[2] + (double)o2 * h22));
    }
    // node centre minus lane origin in half-cells, as in the per-target
    // mixed walk: a scalar reduction against the first lane's origin g, and a
    // fixed per-lane term; groups wider than r_cut + |o - g| allows take the
    // minimum image per lane
    const int g0 = __builtin_amdgcn_readfirstlane(o0), g1 = __builtin_amdgcn_readfirstlane(o1),
              g2 = __builtin_amdgcn_readfirstlane(o2);
    constexpr int kHalf = 1 << 21, kMask = (1 << 22) - 1;
    const int gq0 = g0 - kHalf, gq1 = g1 - kHalf, gq2 = g2 - kHalf;
    const float qb0 = biased(kPer ? o0 - gq0 : o0), qb1 = biased(kPer ? o1 - gq1 : o1),
                qb2 = biased(kPer ? o2 - gq2 : o2);
    bool lane_wrap = false;
    if (kPer) {
      const int e = valid ? max(abs(o0 - g0), max(abs(o1 - g1), abs(o2 - g2))) : 0;
      const float rc_cells = sqrtf(k.rc2) / k.h22;
      lane_wrap = !((float)wave_max_i32(e) + rc_cells < (float)((1 << 20) - (1 << 16)));
    }
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    uint32_t ni = 0, cnt = 0;
    auto walk = [&](auto lane_wrap_t) {
      constexpr bool kLaneWrap = decltype(lane_wrap_t)::value;
      // the stored form of a node centre (uniform over the wave)
      auto centre = [&](const int *c, float *f) {
        if (kPer && !kLaneWrap) {
          f[0] = biased((c[0] - gq0) & kMask);
          f[1] = biased((c[1] - gq1) & kMask);
          f[2] = biased((c[2] - gq2) & kMask);
        } else {  // the record's form: 2^23 + c as float bits
          f[0] = __int_as_float(c[0]);
          f[1] = __int_as_float(c[1]);
          f[2] = __int_as_float(c[2]);
        }
      };
      // this lane's offset to a stored centre, in half-cells (exact)
      auto offset = [&](const float *f, float &f0, float &f1, float &f2) {
        if (kPer && kLaneWrap) {
          f0 = (float)wrap_cells((__float_as_int(f[0]) & kMask) - o0);
          f1 = (float)wrap_cells((__float_as_int(f[1]) & kMask) - o1);
          f2 = (float)wrap_cells((__float_as_int(f[2]) & kMask) - o2);
        } else {
          f0 = f[0] - qb0;
          f1 = f[1] - qb1;
          f2 = f[2] - qb2;
        }
      };
      // every lane evaluates every entry for its own target, in list order
      auto flush = [&]() __attribute__((always_inline)) {
        __syncthreads();
        for (uint32_t e = 0; e < cnt; ++e) {
          const GEntry q = list[e];
          float f0, f1, f2;
          offset(q.c, f0, f1, f2);
          float dx = (f0 * k.h22 - xr) + q.o[0];
          float dy = (f1 * k.h22 - yr) + q.o[1];
          float dz = (f2 * k.h22 - zr) + q.o[2];
          if (kPer && (q.tag & kGWrap)) {
            dx = wrap_box(dx, k);
            dy = wrap_box(dy, k);
            dz = wrap_box(dz, k);
          }
          const float r2 = fmaf(dz, dz, fmaf(dx, dx, dy * dy));
          const bool use = valid && (!kCut || r2 < k.rc2) && (q.tag & kGNoSelf) != p;
          if (use) {
            eval32<kExt>(dx, dy, dz, r2, q.m, k, ax, ay, az, ph);
            ++ni;
          }
        }
        __syncthreads();
        cnt = 0;
      };
      uint32_t n = bx.root;
      const uint32_t nend = bx.node_end;
      while (n < nend) {
        const WNode w = kWide ? ldw(A.wnode + n)
                              : ldw((const WNode *)((const char *)A.wnode + n * (uint32_t)sizeof(WNode)));
        const bool leaf = (w.cf & kWLeaf) != 0;
        const uint32_t ns = leaf ? n + 1 : w.a;
        const uint32_t lc = w.cf & kWCount;
        float fc[3], f0, f1, f2;
        centre(w.c, fc);
        offset(fc, f0, f1, f2);
        const float dcx = f0 * k.h22 - xr, dcy = f1 * k.h22 - yr, dcz = f2 * k.h22 - zr;
        const float mdc = fmaxf(fmaxf(fabsf(dcx), fabsf(dcy)), fabsf(dcz));
        const bool wrapd = kPer && (w.cf & kWWrap) != 0;
        float dx = dcx + w.o[0], dy = dcy + w.o[1], dz = dcz + w.o[2];
        if (wrapd) {
          dx = wrap_box(dx, k);
          dy = wrap_box(dy, k);
          dz = wrap_box(dz, k);
        }
        const float r2 = fmaf(dz, dz, fmaf(dx, dx, dy * dy));
        const bool live = valid && !(kCut && mdc > w.reach);
        const bool far_open = relative ? (w.m * w.side2 > aol * (r2 * r2)) : (w.side2 > r2);
        const bool open = live && (far_open || mdc < w.near);
        const uint32_t nskip = ns > n ? ns : n + 1;  // a skip always moves forward
        uint32_t nn;
        if (!__ballot(live)) {
          nn = nskip;
        } else if (!__ballot(open)) {
          if (cnt == kGroupCap) flush();
          if (lane == 0) {
            GEntry q;
            q.c[0] = fc[0];
            q.c[1] = fc[1];
            q.c[2] = fc[2];
            q.tag = kGNoSelf | (wrapd ? kGWrap : 0u);
            q.o[0] = w.o[0];
            q.o[1] = w.o[1];
            q.o[2] = w.o[2];
            q.m = w.m;
            list[cnt] = q;
          }
          ++cnt;
          nn = nskip;
        } else {
          if (leaf) {
            for (uint32_t j0 = 0; j0 < lc; j0 += 64) {
              const uint32_t m = min(64u, lc - j0);
              if (cnt + m > kGroupCap) flush();
              if (lane < m) {
                const uint32_t j = (w.a & kTagFirst) + j0 + lane;
                const float4 pq = A.part32[j];
                GEntry q;
                q.c[0] = fc[0];
                q.c[1] = fc[1];
                q.c[2] = fc[2];
                q.tag = j | (wrapd ? kGWrap : 0u);
                q.o[0] = w.o[0] + pq.x;  // leaf offsets are stored from the leaf's centre of mass
                q.o[1] = w.o[1] + pq.y;
                q.o[2] = w.o[2] + pq.z;
                q.m = pq.w;
                list[cnt + lane] = q;
              }
              cnt += m;
            }
          }
          nn = n + 1;
        }
        n = nn;
      }
      flush();
    };
    if (kPer && lane_wrap) walk(std::true_type{});
    else walk(std::false_type{});
    if (valid) write_out(A, bx, slot, ax, ay, az, ph, ni);
  }
}

}  // namespace

int walk_list_capacity() {
  static int cap = -1;
  if (cap < 0) {
    const char *e = getenv("OG_WALK_LIST_CAP");
    const int v = e ? atoi(e) : 0;
    cap = (v == 4 || v == 8 || v == 16 || v == 32) ? v : 4;
  }
  return cap;
}

// OG_WIDE_NODES=1 takes the 64-bit record offsets for every forest, and
// OG_NO_INTERIOR=1 the reduced periodic offsets for every group (the tests
// compare both forms on small inputs); read at each launch.
static bool env_flag(const char *name) {
  const char *e = getenv(name);
  return e && atoi(e) == 1;
}
static bool wide_nodes_forced() { return env_flag("OG_WIDE_NODES"); }

void launch_walk(const WalkArgs &W0, int precision, hipStream_t s) {
  const TraceRange trace_range(precision == 0 ? "walk: fp64" : "walk: mixed");
  WalkArgs W = W0;
  W.no_interior = env_flag("OG_NO_INTERIOR") ? 1 : 0;
  const uint32_t cus = (uint32_t)device_cu_count();
  const uint32_t groups = W.n_groups > 0 ? W.n_groups : 1;
  launch_reset_n(W.counter, kQueues, s);
  if (W.group_lists) {
    if (precision == 0) {
      const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(3u * cus, (groups + 3) / 4));
      if (W.ext && W.erfc_tail) k_walkg64<true, true><<<blocks, 256, 0, s>>>(W);
      else if (W.ext) k_walkg64<true, false><<<blocks, 256, 0, s>>>(W);
      else if (W.erfc_tail) k_walkg64<false, true><<<blocks, 256, 0, s>>>(W);
      else k_walkg64<false, false><<<blocks, 256, 0, s>>>(W);
    } else {
      // one wave per workgroup, 4 KB of list each, 8 waves per SIMD
      const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(32u * cus, groups));
      const int mode = W.box_kind;
      if (W.wide_nodes || wide_nodes_forced()) k_walkg32<0, true, true><<<blocks, kWalk32Threads, 0, s>>>(W);
      else if (W.ext) k_walkg32<0, true><<<blocks, kWalk32Threads, 0, s>>>(W);
      else if (mode == 2) k_walkg32<2, false><<<blocks, kWalk32Threads, 0, s>>>(W);
      else if (mode == 1) k_walkg32<1, false><<<blocks, kWalk32Threads, 0, s>>>(W);
      else if (mode == 3) k_walkg32<3, false><<<blocks, kWalk32Threads, 0, s>>>(W);
      else k_walkg32<0, false><<<blocks, kWalk32Threads, 0, s>>>(W);
    }
    return;
  }
  if (precision == 0 && !W.wide_nodes && !wide_nodes_forced() && !env_flag("OG_WALK64_PLAIN")) {
    // screened FP64 walk: one wave per workgroup, 7 waves per SIMD
    const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(28u * cus, groups));
    if (W.ext && W.erfc_tail) k_walk64s<0, true, kScreenCap, true><<<blocks, kWalk32Threads, 0, s>>>(W);
    else if (W.ext) k_walk64s<0, false, kScreenCap, true><<<blocks, kWalk32Threads, 0, s>>>(W);
    else if (W.erfc_tail) k_walk64s<0, true, kScreenCap><<<blocks, kWalk32Threads, 0, s>>>(W);
    else if (W.box_kind == 2) k_walk64s<2, false, kScreenCap><<<blocks, kWalk32Threads, 0, s>>>(W);
    else k_walk64s<0, false, kScreenCap><<<blocks, kWalk32Threads, 0, s>>>(W);
  } else if (precision == 0) {
    // 4 waves per workgroup, 4 waves per SIMD
    const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(4u * cus, (groups + 3) / 4));
    if (W.ext && W.erfc_tail) k_walk64<true, true><<<blocks, 64 * kWalk64Waves, 0, s>>>(W);
    else if (W.ext) k_walk64<true, false><<<blocks, 64 * kWalk64Waves, 0, s>>>(W);
    else if (W.erfc_tail) k_walk64<false, true><<<blocks, 64 * kWalk64Waves, 0, s>>>(W);
    else k_walk64<false, false><<<blocks, 64 * kWalk64Waves, 0, s>>>(W);
  } else {
    // one wave per workgroup; LDS per wave = cap x 1 KB of lists
    const int cap = W.list_cap > 0 ? W.list_cap : walk_list_capacity();
    const uint32_t per_cu = std::min<uint32_t>(32u, 160u / (uint32_t)cap);
    const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(per_cu * cus, groups));
    const int mode = W.box_kind;
    const bool wide = W.wide_nodes || wide_nodes_forced();
#define OG_WALK32(C)                                                                 \
  do {                                                                               \
    if (wide && W.seps) k_walk32<4, 0, true, true, true><<<blocks, kWalk32Threads, 0, s>>>(W); \
    else if (wide) k_walk32<4, 0, true, false, true><<<blocks, kWalk32Threads, 0, s>>>(W); \
    else if (W.seps) k_walk32<C, 0, true, true><<<blocks, kWalk32Threads, 0, s>>>(W); \
    else if (W.ext) k_walk32<C, 0, true><<<blocks, kWalk32Threads, 0, s>>>(W);       \
    else if (mode == 2) k_walk32<C, 2, false><<<blocks, kWalk32Threads, 0, s>>>(W);  \
    else if (mode == 1) k_walk32<C, 1, false><<<blocks, kWalk32Threads, 0, s>>>(W);  \
    else if (mode == 3) k_walk32<C, 3, false><<<blocks, kWalk32Threads, 0, s>>>(W);  \
    else k_walk32<C, 0, false><<<blocks, kWalk32Threads, 0, s>>>(W);                 \
  } while (0)
    if (cap == 8) OG_WALK32(8);
    else if (cap == 4) OG_WALK32(4);
    else if (cap == 32) OG_WALK32(32);
    else OG_WALK32(16);
#undef OG_WALK32
  }
}

}  // namespace og
