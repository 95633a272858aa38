// Tree walk kernels for CDNA4 (gfx950, wave64).
//
// Paper, "Tree walk": one walk per target from the root; at each node the
// opening criterion decides between the first child (next node in
// pre-order) and the sibling pointer (skip); a leaf's particles contribute
// directly.  Paper, "Force evaluation" / "Particle Mesh": every accepted
// node or particle adds the short-range (erfc) part of the split force.
//
// GPU mapping: a persistent grid; each wavefront pops a group of <= 64
// spatially adjacent targets (one node of the tree) from an atomic queue
// and walks the tree once for the whole group.  Lane i owns target i and
// keeps `next`, the next node of ITS OWN per-target walk.  At node n the
// lanes with next == n apply the per-target rules; the wave goes to n + 1
// when any lane opened n, otherwise to skip(n).  A lane therefore sees
// exactly the node sequence of its own walk, in the same order, so its
// result does not depend on the group it was placed in.  Node records are
// wave-uniform (scalar loads); a leaf's particles are loaded once,
// coalesced, and broadcast lane by lane with readlane.
#include "og_kernels.h"

namespace og {

namespace {

constexpr int kThreads = 256;

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

__device__ inline float rdl(float v, uint32_t j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), (int)j));
}
__device__ inline double rdl(double v, uint32_t j) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), (int)j);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), (int)j);
  return __longlong_as_double(((long long)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Target of lane `lane` in group gr: sorted particle position and output slot.
__device__ inline bool lane_target(const WalkArgs &A, const Group &gr, const BoxDev &bx, uint32_t lane,
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

// ------------------------------------------------------------ FP64 form --
__device__ inline double minimg(double d, bool periodic, double box) {
  if (!periodic) return d;
  if (d > 0.5 * box) return d - box;
  if (d < -0.5 * box) return d + box;
  return d;
}

__device__ inline void pair64(double dx, double dy, double dz, double m, const BoxDev &bx, double &ax,
                              double &ay, double &az, double &ph, uint32_t &ni) {
#pragma clang fp contract(off)
  const double r2 = dx * dx + dy * dy + dz * dz;
  if (bx.cutoff && !(r2 < bx.rc2)) return;
  const double rinv = 1.0 / sqrt(r2 + bx.eps2);
  double S = 1.0, pf = 1.0;
  if (bx.cutoff) {
    const double r = sqrt(r2);
    const double u = r / (2.0 * bx.r_s);
    const double e = erfc(u);
    S = e + kTwoOverSqrtPi * u * exp(-u * u);
    pf = e;
  }
  const double f = bx.G * m * rinv * rinv * rinv * S;
  ax += f * dx;
  ay += f * dy;
  az += f * dz;
  ph -= bx.G * m * pf * rinv;
  ++ni;
}

__global__ __launch_bounds__(kThreads) void k_walk64(WalkArgs A) {
#pragma clang fp contract(off)
  const uint32_t lane = threadIdx.x & 63;
  while (true) {
    uint32_t g = 0;
    if (lane == 0) g = atomicAdd(A.counter, 1u);
    g = __shfl(g, 0, 64);
    if (g >= *A.n_groups) break;
    const Group gr = A.groups[g];
    const BoxDev &bx = A.boxes[gr.box];
    uint32_t p = 0, slot = 0;
    const bool valid = lane_target(A, gr, bx, lane, p, slot);
    double4 xi = make_double4(0.0, 0.0, 0.0, 0.0);
    if (valid) xi = A.part64[p];
    const bool periodic = bx.periodic, cutoff = bx.cutoff;
    const double box = bx.box, h = bx.L * 0x1p-21;
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    uint32_t ni = 0;
    uint32_t n = bx.root;
    const uint32_t nend = bx.node_end;
    uint32_t next = valid ? n : nend;
    while (n < nend) {
      const Topo t = A.topo[n];
      const Mom64 mm = A.mom64[n];
      const bool leaf = (t.corner & kLeafBit) != 0;
      const int lev = (int)(t.b >> kCountBits);
      const double side = ldexp(bx.L, -lev);
      const double half = ldexp(1.0, 20 - lev);
      const double c0 = bx.lo[0] + ((double)(uint32_t)(t.corner & 0x1fffffull) + half) * h;
      const double c1 = bx.lo[1] + ((double)(uint32_t)((t.corner >> 21) & 0x1fffffull) + half) * h;
      const double c2 = bx.lo[2] + ((double)(uint32_t)((t.corner >> 42) & 0x1fffffull) + half) * h;
      bool open_int = false, open_leaf = false;
      if (next == n) {
        const double dcx = minimg(c0 - xi.x, periodic, box);
        const double dcy = minimg(c1 - xi.y, periodic, box);
        const double dcz = minimg(c2 - xi.z, periodic, box);
        bool pruned = false;
        if (cutoff) {
          const double reach = bx.rcut + 0.5 * side;
          pruned = fabs(dcx) > reach || fabs(dcy) > reach || fabs(dcz) > reach;
        }
        if (pruned) {
          next = leaf ? n + 1 : t.a;
        } else {
          const double dx = minimg(mm.cx - xi.x, periodic, box);
          const double dy = minimg(mm.cy - xi.y, periodic, box);
          const double dz = minimg(mm.cz - xi.z, periodic, box);
          const double r2 = dx * dx + dy * dy + dz * dz;
          const double near = 0.6 * side;
          const bool open = (side * side > bx.theta2 * r2) ||
                            (fabs(dcx) < near && fabs(dcy) < near && fabs(dcz) < near);
          if (!open) {
            pair64(dx, dy, dz, mm.m, bx, ax, ay, az, ph, ni);
            next = leaf ? n + 1 : t.a;
          } else if (!leaf) {
            open_int = true;
            next = n + 1;
          } else {
            open_leaf = true;
            next = n + 1;
          }
        }
      }
      if (leaf) {
        if (__ballot(open_leaf)) {
          const uint32_t f = t.a, cnt = t.b & kCountMask;
          for (uint32_t base = 0; base < cnt; base += 64) {
            double4 q = make_double4(0.0, 0.0, 0.0, 0.0);
            if (base + lane < cnt) q = A.part64[f + base + lane];
            const uint32_t m = min(64u, cnt - base);
            for (uint32_t j = 0; j < m; ++j) {
              const double qx = rdl(q.x, j), qy = rdl(q.y, j), qz = rdl(q.z, j), qm = rdl(q.w, j);
              if (open_leaf && f + base + j != p) {
                const double dx = minimg(qx - xi.x, periodic, box);
                const double dy = minimg(qy - xi.y, periodic, box);
                const double dz = minimg(qz - xi.z, periodic, box);
                pair64(dx, dy, dz, qm, bx, ax, ay, az, ph, ni);
              }
            }
          }
        }
        n = n + 1;
      } else {
        n = (__ballot(open_int) || t.a <= n) ? n + 1 : t.a;
      }
    }
    if (valid) write_out(A, bx, slot, ax, ay, az, ph, ni);
  }
}

// ----------------------------------------------------------- mixed form --
// Every lane works in FP32 offsets from its own origin `ref`, the centre of
// the level-21 cell holding its target.  Node centres relative to ref come
// from exact integer cell arithmetic (periodic minimum image on integers,
// the box being 2^22 half-cells long); a node's centre of mass is its centre
// plus the node's FP32 offset, a particle is its leaf centre plus its FP32
// offset (both offsets formed in FP64 at build time); the target itself is
// FP64 (x - ref) rounded once.  The origin depends on the target only, so
// results do not depend on how targets are grouped.
struct Consts32 {
  float G, eps2, inv2rs, rcut, rc2, theta2, h22, L, half_box, box;
  bool cutoff, periodic;
};

__device__ inline void pair32(float dx, float dy, float dz, float r2, float m, const Consts32 &k, double &ax,
                              double &ay, double &az, double &ph, uint32_t &ni) {
  const float rinv = __builtin_amdgcn_rsqf(r2 + k.eps2);
  float S = 1.0f, pf = 1.0f;
  if (k.cutoff) {
    const float r = r2 > 0.0f ? r2 * __builtin_amdgcn_rsqf(r2) : 0.0f;
    const float u = r * k.inv2rs;
    const float e = __expf(-u * u);
    const float t = __builtin_amdgcn_rcpf(1.0f + kAsP * u);
    const float ec = t * (kAsA1 + t * (kAsA2 + t * (kAsA3 + t * (kAsA4 + t * kAsA5)))) * e;
    S = ec + (float)kTwoOverSqrtPi * u * e;
    pf = ec;
  }
  const float mr = k.G * m * rinv;
  const float f = mr * rinv * rinv * S;
  ax += (double)(f * dx);
  ay += (double)(f * dy);
  az += (double)(f * dz);
  ph -= (double)(mr * pf);
  ++ni;
}

__device__ inline int wrap_half_cells(int d, bool periodic) {
  // the periodic box is 2^22 half-cells long
  if (periodic) {
    if (d > (1 << 21)) d -= (1 << 22);
    else if (d < -(1 << 21)) d += (1 << 22);
  }
  return d;
}

__device__ inline float wrap_box(float d, const Consts32 &k) {
  if (d > k.half_box) return d - k.box;
  if (d < -k.half_box) return d + k.box;
  return d;
}

__global__ __launch_bounds__(kThreads) void k_walk32(WalkArgs A) {
#pragma clang fp contract(fast)
  const uint32_t lane = threadIdx.x & 63;
  while (true) {
    uint32_t g = 0;
    if (lane == 0) g = atomicAdd(A.counter, 1u);
    g = __shfl(g, 0, 64);
    if (g >= *A.n_groups) break;
    const Group gr = A.groups[g];
    const BoxDev &bx = A.boxes[gr.box];
    Consts32 k;
    k.G = bx.Gf;
    k.eps2 = bx.eps2f;
    k.inv2rs = bx.inv2rsf;
    k.rcut = bx.rcutf;
    k.rc2 = bx.rc2f;
    k.theta2 = bx.theta2f;
    k.h22 = bx.h22f;
    k.L = bx.Lf;
    k.box = bx.Lf;
    k.half_box = 0.5f * bx.Lf;
    k.cutoff = bx.cutoff;
    k.periodic = bx.periodic;
    uint32_t p = 0, slot = 0;
    const bool valid = lane_target(A, gr, bx, lane, p, slot);
    // lane origin: centre of the target's level-21 cell, in half-cells
    int r0 = 0, r1 = 0, r2i = 0;
    float xr = 0.0f, yr = 0.0f, zr = 0.0f;
    if (valid) {
      const uint64_t key = A.skeys[p];
      r0 = 2 * (int)compact3(key >> 2) + 1;
      r1 = 2 * (int)compact3(key >> 1) + 1;
      r2i = 2 * (int)compact3(key) + 1;
      const double h22 = bx.L * 0x1p-22;
      const double4 q = A.part64[p];
      xr = (float)(q.x - (bx.lo[0] + (double)r0 * h22));
      yr = (float)(q.y - (bx.lo[1] + (double)r1 * h22));
      zr = (float)(q.z - (bx.lo[2] + (double)r2i * h22));
    }
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    uint32_t ni = 0;
    uint32_t n = bx.root;
    const uint32_t nend = bx.node_end;
    uint32_t next = valid ? n : nend;
    while (n < nend) {
      const Topo t = A.topo[n];
      const Mom32 mm = A.mom32[n];
      const bool leaf = (t.corner & kLeafBit) != 0;
      const int lev = (int)(t.b >> kCountBits);
      const int hc = 1 << (kLevels - lev);
      const float side = ldexpf(k.L, -lev);
      // offsets may need the minimum image once the node can reach half a box
      const bool wrapd = k.periodic && (k.rcut + side >= k.half_box);
      bool open_int = false, open_leaf = false;
      float dcx = 0.0f, dcy = 0.0f, dcz = 0.0f;
      if (next == n || leaf) {
        const int d0 = wrap_half_cells(2 * (int)(t.corner & 0x1fffffull) + hc - r0, k.periodic);
        const int d1 = wrap_half_cells(2 * (int)((t.corner >> 21) & 0x1fffffull) + hc - r1, k.periodic);
        const int d2 = wrap_half_cells(2 * (int)((t.corner >> 42) & 0x1fffffull) + hc - r2i, k.periodic);
        dcx = (float)d0 * k.h22 - xr;
        dcy = (float)d1 * k.h22 - yr;
        dcz = (float)d2 * k.h22 - zr;
      }
      if (next == n) {
        bool pruned = false;
        if (k.cutoff) {
          const float reach = k.rcut + 0.5f * side;
          pruned = fabsf(dcx) > reach || fabsf(dcy) > reach || fabsf(dcz) > reach;
        }
        if (pruned) {
          next = leaf ? n + 1 : t.a;
        } else {
          float dx = dcx + mm.ox, dy = dcy + mm.oy, dz = dcz + mm.oz;
          if (wrapd) {
            dx = wrap_box(dx, k);
            dy = wrap_box(dy, k);
            dz = wrap_box(dz, k);
          }
          const float r2 = dx * dx + dy * dy + dz * dz;
          const float near = 0.6f * side;
          const bool open = (side * side > k.theta2 * r2) ||
                            (fabsf(dcx) < near && fabsf(dcy) < near && fabsf(dcz) < near);
          if (!open) {
            if (!k.cutoff || r2 < k.rc2) pair32(dx, dy, dz, r2, mm.m, k, ax, ay, az, ph, ni);
            next = leaf ? n + 1 : t.a;
          } else if (!leaf) {
            open_int = true;
            next = n + 1;
          } else {
            open_leaf = true;
            next = n + 1;
          }
        }
      }
      if (leaf) {
        if (__ballot(open_leaf)) {
          const uint32_t f = t.a, cnt = t.b & kCountMask;
          for (uint32_t base = 0; base < cnt; base += 64) {
            float4 q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (base + lane < cnt) q = A.part32[f + base + lane];
            const uint32_t m = min(64u, cnt - base);
            for (uint32_t j = 0; j < m; ++j) {
              const float qx = rdl(q.x, j), qy = rdl(q.y, j), qz = rdl(q.z, j), qm = rdl(q.w, j);
              if (open_leaf && f + base + j != p) {
                float dx = dcx + qx, dy = dcy + qy, dz = dcz + qz;
                if (wrapd) {
                  dx = wrap_box(dx, k);
                  dy = wrap_box(dy, k);
                  dz = wrap_box(dz, k);
                }
                const float r2 = dx * dx + dy * dy + dz * dz;
                if (!k.cutoff || r2 < k.rc2) pair32(dx, dy, dz, r2, qm, k, ax, ay, az, ph, ni);
              }
            }
          }
        }
        n = n + 1;
      } else {
        n = (__ballot(open_int) || t.a <= n) ? n + 1 : t.a;
      }
    }
    if (valid) write_out(A, bx, slot, ax, ay, az, ph, ni);
  }
}

int g_blocks[2] = {0, 0};

}  // namespace

void launch_walk(const WalkArgs &W, int precision, uint32_t max_groups, hipStream_t s) {
  const int which = precision == 0 ? 0 : 1;
  if (g_blocks[which] == 0) {
    int per_cu = 0;
    hipError_t e = which == 0
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_walk64, kThreads, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_walk32, kThreads, 0);
    if (e != hipSuccess || per_cu <= 0) per_cu = 2;
    g_blocks[which] = per_cu * device_cu_count();
  }
  uint32_t waves_needed = max_groups > 0 ? max_groups : 1;
  uint32_t blocks = std::min<uint32_t>((uint32_t)g_blocks[which], (waves_needed + 3) / 4);
  if (blocks == 0) blocks = 1;
  launch_reset(W.counter, s);
  if (which == 0)
    k_walk64<<<blocks, kThreads, 0, s>>>(W);
  else
    k_walk32<<<blocks, kThreads, 0, s>>>(W);
}

}  // namespace og
