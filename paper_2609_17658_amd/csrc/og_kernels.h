// Host-side launchers of the library's HIP kernels.  All take a stream and
// enqueue only; none allocates or synchronises.
#pragma once

#include "og_internal.h"

namespace og {

// Exclusive scan of n = *n_dev (device scalar, <= cap) uint32 values:
// out[0..n] with out[n] = total.  `partial` holds cap/kScanTile + 2 words.
constexpr uint32_t kScanTile = 4096;
void scan_u32(const uint32_t *in, uint32_t *out, const uint32_t *n_dev, uint32_t cap,
              uint32_t *partial, hipStream_t s);

// LSD radix sort of (key, val) pairs, 8-bit digits.  Key passes
// [pass_lo, pass_hi) on the 64-bit key, then `box_passes` passes on the box
// of each value (global particle index).  Ping-pongs between a and b;
// returns true when the result ends in b.
constexpr uint32_t kSortTile = 4096;
bool radix_sort(uint64_t *keys_a, uint32_t *vals_a, uint64_t *keys_b, uint32_t *vals_b,
                uint32_t n, int pass_lo, int pass_hi, int box_passes, const BoxDev *boxes,
                int B, uint32_t *hist, uint32_t *digit_tot, hipStream_t s);
size_t radix_hist_words(uint32_t n);

struct BuildArrays {
  BoxDev *boxes;
  int B;
  uint32_t n;                 // total particles
  uint32_t node_cap;          // node capacity
  uint64_t *minmax;           // [B][6] ordered-bits min/max for open boxes
  uint64_t *keys_a, *keys_b;
  uint32_t *vals_a, *vals_b;
  uint32_t *hist, *digit_tot;
  uint32_t *perm, *inv;
  double4 *part64;
  float4 *part32;
  int8_t *lcp;
  uint8_t *depth;
  uint32_t *nstart, *S, *scan_partial;
  Topo *topo;
  Mom64 *mom64;
  Mom32 *mom32;
  WNode *wnode;
  double4 *cen64;  // per node: FP64 cube centre (x, y, z) and side (w), for the FP64 walks
  uint32_t *first, *skip, *parent;
  uint32_t *top_cnt;          // [0] top nodes [2] deepest top level
  uint32_t *top_buf;          // TopArrays' lists, kTopWords per top node (top_cap)
  uint32_t *top_id;           // per node: index of a top node in the top list
  uint32_t top_cap;           // bound on the top nodes (top_node_bound)
  uint32_t *scalars;          // [0] status [3] n_nodes [4] n [8..15] walk queues
                              // [5] deepest level (stats)
  int any_open;               // some box has periodic = 0
  int leaf_max;               // largest leaf_max of the boxes
  double *seps;               // sorted per-particle softening lengths (null: none given)
  double *semax, *semin;      // per node: largest and smallest of its particles' lengths
};

// The moment kernels sum subtrees of up to kSegNodes nodes per workgroup;
// the nodes with larger subtrees ("top" nodes) are summed by one workgroup.
// Top nodes of one level have disjoint subtrees of more than kSegNodes
// nodes each, so there are fewer than node_cap / kSegNodes + 1 per level.
constexpr uint32_t kSegNodes = 768;
inline uint32_t top_node_bound(uint32_t node_cap) { return 2 * (((kLevels + 1) * (node_cap / kSegNodes + 1) + 1) / 2); }

// The top-node list the moment kernels pass to the top-node kernel.
struct TopArrays {
  uint32_t *cnt;    // [0] top nodes [2] deepest level of a top node
  uint4 *list;      // top nodes (cap): node, level, cube corner (low, high word)
  uint64_t *slot;   // per top node: eight child slots by octant (8 cap)
  uint32_t *id;     // per node (node_cap): its class (a top node: with its index in `list`)
  uint32_t cap;
};
constexpr size_t kTopWords = 20;  // words of top_buf per top node

void launch_build(BuildArrays &A, hipStream_t s);
void launch_max_level(const BuildArrays &A, uint32_t *out, hipStream_t s);

// Targets given as caller-order indices (box 0 only): the target list
// sorted by tree position (so that consecutive targets are neighbours).
struct TargetArrays {
  const int64_t *idx;
  uint32_t M;
  uint64_t *tkey_a, *tkey_b;
  uint32_t *tval_a, *tval_b;
  uint32_t *hist, *digit_tot;
  uint32_t *scalars;          // [0] status [8..15] walk queues
  const uint64_t *tkey;       // result (points at a or b)
  const uint32_t *tval;
};
void launch_targets(const BuildArrays &A, TargetArrays &T, hipStream_t s);

// Active targets of one tree: the particles whose time-step level bin[i]
// (caller order) is <= level, in curve order, compacted on the device.
// counts[0] = number of active targets, counts[1] = walk groups of `chunk`;
// n_active (optional) receives counts[0] as int64.
struct ActiveArrays {
  const int8_t *bin;
  int32_t level;
  uint32_t *flags, *offs, *partial;
  uint64_t *tkey;
  uint32_t *tval;
  uint32_t *counts;           // [0] active, [1] groups, [8..15] walk queues
  int64_t *n_active;
};
void launch_active(const BuildArrays &A, ActiveArrays &T, uint32_t chunk, hipStream_t s);
size_t scan_partial_words(uint32_t n);

struct WalkArgs {
  const BoxDev *boxes;
  const Topo *topo;
  const Mom32 *mom32;
  const WNode *wnode;
  const double4 *cen64;
  const Mom64 *mom64;
  const float4 *part32;
  const double4 *part64;
  const uint32_t *perm;
  const uint64_t *skeys;      // sorted Morton keys
  uint32_t n_groups;          // walk groups (chunks of `chunk` targets)
  uint32_t chunk;             // targets per group, <= 64
  int list_cap;               // mixed walk list entries per lane (0 = default)
  uint32_t n_targets;         // length of the target list (tkey != null)
  int B;                      // boxes
  int box_kind;               // shared by all boxes: 1 cutoff+open, 2 cutoff+periodic,
                              // 3 Newtonian+open; 0 mixed
  uint32_t *counter;          // kQueues group counters
  const uint64_t *tkey;       // sorted target positions, or null: all particles
  const uint32_t *tval;       // target slots
  double *acc;                // non-null: outputs by slot; null: per-box acc/pot
  double *pot;
  int64_t *nint;
  int pot_override;           // 1: use `pot` (possibly null) instead of the box's
  int ext;                    // some box uses spline softening or the relative criterion
  const uint32_t *dev_count;  // non-null: n_targets = [0], n_groups = [1], read on the device
  const double *seps, *semax, *semin;  // per-particle softening (null: the boxes' eps)
  int group_lists;            // 1: group-shared interaction lists, 0: per-target walk
  const double *a_old;        // relative criterion: previous accelerations [n][3], caller order
  int wide_nodes;             // the node records span more than 4 GiB (64-bit record offsets)
  int no_interior;            // mixed walk: reduce every periodic offset (no raw form for interior groups)
  int erfc_tail;              // FP64 walks: some box has r_cut / (2 r_s) >= 3 (library erfc past the polynomial)
};
void launch_walk(const WalkArgs &W, int precision, hipStream_t s);
void launch_reset(uint32_t *word, hipStream_t s);
void launch_reset_n(uint32_t *words, int n, hipStream_t s);

// Walk group queues: one per XCD (see k_walk.hip).
constexpr uint32_t kQueues = 8;

int device_cu_count();

}  // namespace og
