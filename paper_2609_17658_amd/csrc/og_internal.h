// Internal device-side data layout of the tree force library (HIP, gfx950).
//
// A "forest" holds B >= 1 independent boxes whose particles are concatenated
// in one global index space; box b owns global particle indices
// [p_off, p_off + n) both in caller order and after the sort (the sort key
// is (box, Morton key, index)), and the nodes [root, node_end) of its
// pre-order tree.  A single tree is a forest with B = 1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace og {

constexpr int kLevels = 21;                 // deepest level; 2^21 cells per axis
constexpr uint32_t kGrid = 1u << kLevels;
constexpr int kCountBits = 27;              // node particle count field width
constexpr uint32_t kCountMask = (1u << kCountBits) - 1u;
constexpr uint64_t kLeafBit = 1ull << 63;   // in Topo::corner

// Host-side stage ranges for profilers (roctx), the analogue of the paper's
// code timers: with OG_TRACE=1 in the environment every API call and build
// stage pushes a named range around the work it enqueues (host enqueue
// intervals; the kernels they enqueue appear beside them in a marker trace,
// e.g. rocprofv3 --marker-trace --kernel-trace).  Off by default.
bool trace_on();
struct TraceRange {
  bool on;
  explicit TraceRange(const char *name);
  ~TraceRange();
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};

// Status bits written by kernels (read by the host at sync points).
constexpr uint32_t kStatusRange = 1u;       // a position outside the box
constexpr uint32_t kStatusNodes = 2u;       // node bound exceeded (never expected)
constexpr uint32_t kStatusTarget = 4u;      // a target index outside [0, N)

// Per-box descriptor, device resident.
struct BoxDev {
  const double *pos;     // caller [n][3]
  const double *mass;    // caller [n]
  double *acc;           // batch output [n][3] (caller order) or null
  double *pot;           // batch output [n] or null
  double lo[3];          // root cube lower corner
  double L;              // root cube side
  double scale;          // 2^21 / L
  double box;            // periodic box side
  double G, eps2, r_s, rcut, rc2, theta2;
  float Gf, eps2f, inv2rsf, rcutf, rc2f, theta2f, Lf, h22f;
  uint32_t p_off, n;     // particle range
  uint32_t root, node_end;  // node range, written on the device
  int32_t periodic, cutoff, leaf_max;
  uint32_t g_off;          // first walk group of this box
  int32_t spline, relative;  // softening kernel, opening criterion
  double hs, alpha;          // spline support 2.8 eps; relative tolerance
  float hsf, hinvf;          // FP32 support and its inverse
  int32_t curve;             // 0 Morton, 1 Peano-Hilbert keys
  const double *epsp;        // caller [n] per-particle softening lengths, or null
  double eps;                // softening length of particles without their own
};

// Walk-order node record, 16 bytes.
//   corner: cx | cy << 21 | cz << 42 (cube corner in level-21 cells), bit 63 = leaf
//   a:      leaf ? first particle : skip (next node after the subtree)
//   b:      count | level << 27
struct __attribute__((aligned(16))) Topo {
  uint64_t corner;
  uint32_t a;
  uint32_t b;
};

// Node moments: FP64 absolute centre of mass + mass; FP32 offset of the
// centre of mass from the cube centre + mass.
struct __attribute__((aligned(32))) Mom64 {
  double cx, cy, cz, m;
};
struct __attribute__((aligned(16))) Mom32 {
  float ox, oy, oz, m;
};

// Walk record of a node for the mixed-precision walk, 48 bytes (scalar
// loads): everything the per-node decisions need, precomputed in FP32.
//   c[3]:   cube centre c in half-cells of the level-21 grid, stored as
//           0x4B000000 | c: the bits of the float 2^23 + c, a multiple of
//           2^22 above c (so c modulo 2^22 is unchanged)
//   side2:  side^2 / theta^2, the squared distance inside which the
//           geometric criterion opens the node (infinite at theta = 0); in a
//           box with the relative criterion, side^2
//   reach:  r_cut + side/2;  near: 0.6 side
//   o[3]:   centre of mass minus cube centre;  m: G times the mass
//   a:      internal node: skip (the next node after the subtree);
//           leaf: its interaction-list tag (below), whose low bits hold
//           the leaf's first particle
//   cf:     particle count | kWBig (a leaf of more than 8 particles) |
//           kWLeaf | kWWrap (offsets inside the node may need the minimum
//           image)
constexpr uint32_t kWBig = 1u << 29, kWLeaf = 1u << 30, kWWrap = 1u << 31, kWCount = kCountMask;
// Leaf tag, as stored in interaction lists (the float bits of the entry's
// fourth component): sign bit set, bits 0..26 the first particle, bits
// 27..29 the number of particles minus one (at most 8 per entry), bit 30
// set when particle offsets may need the minimum image.
constexpr uint32_t kTagLeaf = 0x80000000u, kTagWrap = 0x40000000u, kTagFirst = (1u << 27) - 1u;
__host__ __device__ inline uint32_t leaf_tag_bits(uint32_t first, uint32_t n, bool wrap) {
  return kTagLeaf | (wrap ? kTagWrap : 0u) | ((n - 1u) << 27) | first;
}
struct __attribute__((aligned(16))) WNode {
  int32_t c[3];
  float side2;
  float o[3];
  float m;
  float reach, near;
  uint32_t a, cf;
};

// ---- bit helpers ------------------------------------------------------
__host__ __device__ inline uint64_t spread3(uint32_t v) {
  // bits b of v (b < 21) -> bit 3b of the result
  uint64_t x = v & 0x1fffffull;
  x = (x | (x << 32)) & 0x001f00000000ffffull;
  x = (x | (x << 16)) & 0x001f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}
__host__ __device__ inline uint32_t compact3(uint64_t x) {
  // bit 3b of x -> bit b of the result
  x &= 0x1249249249249249ull;
  x = (x | (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x | (x >> 4)) & 0x100f00f00f00f00full;
  x = (x | (x >> 8)) & 0x001f0000ff0000ffull;
  x = (x | (x >> 16)) & 0x001f00000000ffffull;
  x = (x | (x >> 32)) & 0x00000000001fffffull;
  return (uint32_t)x;
}
__host__ __device__ inline uint64_t morton3(uint32_t cx, uint32_t cy, uint32_t cz) {
  return (spread3(cx) << 2) | (spread3(cy) << 1) | spread3(cz);
}

// Peano-Hilbert order of level-21 cells (Skilling 2004, "Programming the
// Hilbert curve"): the coordinates are mapped to the transposed Hilbert
// index and interleaved like Morton coordinates.  Encoding walks the bits
// from the top: at bit q, the bits below q of coordinate 0 are inverted
// when coordinate i has bit q set, otherwise the bits below q are swapped
// between coordinate 0 and i; a Gray code finishes it.  Every level-l cell
// is a run of 8^(21-l) consecutive keys whose top 3l bits name the cell.
__host__ __device__ inline uint64_t hilbert3(uint32_t x, uint32_t y, uint32_t z) {
  uint32_t c[3] = {x, y, z};
  for (uint32_t q = 1u << (kLevels - 1); q > 1; q >>= 1) {
    const uint32_t low = q - 1;
    for (int i = 0; i < 3; ++i) {
      if (c[i] & q) {
        c[0] ^= low;
      } else {
        const uint32_t t = (c[0] ^ c[i]) & low;
        c[0] ^= t;
        c[i] ^= t;
      }
    }
  }
  c[1] ^= c[0];
  c[2] ^= c[1];
  uint32_t flip = 0;
  for (uint32_t q = 1u << (kLevels - 1); q > 1; q >>= 1)
    if (c[2] & q) flip ^= q - 1;
  return morton3(c[0] ^ flip, c[1] ^ flip, c[2] ^ flip);
}
// Inverse of hilbert3: the cell of a key.
__host__ __device__ inline void hilbert3_cell(uint64_t key, uint32_t c[3]) {
  c[0] = compact3(key >> 2);
  c[1] = compact3(key >> 1);
  c[2] = compact3(key);
  // undo the Gray code
  const uint32_t t = c[2] >> 1;
  c[2] ^= c[1];
  c[1] ^= c[0];
  c[0] ^= t;
  // undo the per-bit inversions and swaps, from the lowest bit up
  for (uint32_t q = 2; q != (1u << kLevels); q <<= 1) {
    const uint32_t low = q - 1;
    for (int i = 2; i >= 0; --i) {
      if (c[i] & q) {
        c[0] ^= low;
      } else {
        const uint32_t u = (c[0] ^ c[i]) & low;
        c[0] ^= u;
        c[i] ^= u;
      }
    }
  }
}
// Cell of a key on either curve (curve 0 Morton, 1 Peano-Hilbert).
__host__ __device__ inline void key_cell(uint64_t key, int curve, uint32_t c[3]) {
  if (curve) {
    hilbert3_cell(key, c);
  } else {
    c[0] = compact3(key >> 2);
    c[1] = compact3(key >> 1);
    c[2] = compact3(key);
  }
}

// Number of leading 3-bit digits two keys share (0..21); keys < 2^63.
__device__ inline int shared_levels(uint64_t a, uint64_t b) {
  uint64_t x = a ^ b;
  if (x == 0) return kLevels;
  return (__clzll((long long)x) - 1) / 3;
}

// Box that owns global particle index g (offsets ascending, B entries).
__device__ inline int box_of(const BoxDev *boxes, int B, uint32_t g) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (boxes[mid].p_off <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace og
