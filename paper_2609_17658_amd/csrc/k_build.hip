// Tree construction kernels for CDNA4 (gfx950, wave64): root frame, Morton
// keys, LSD radix sort, gather into sorted SoA/AoS, pre-order topology,
// bottom-up moments and walk groups.
//
// Paper, "Tree construction": the root covers the domain; particles are
// placed in space-filling-curve order; the cube hierarchy is the recursive
// 8-way subdivision; a bottom-up pass gives node mass and centre of mass;
// traversal uses a first-child ("nextnode") and a sibling pointer.  Here the
// hierarchy is built without insertion: from the sorted keys every particle
// knows at which levels it starts a node, so node ranks come from one scan.
//
// Compiled with -ffp-contract=off: keys and node geometry are rounded
// exactly as written, which makes them bit-identical to any other IEEE
// evaluation of the same expressions.
#include "og_kernels.h"

namespace og {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ inline uint32_t lane_id() { return threadIdx.x & 63; }

// Barrier that orders LDS only: the global stores still in flight are not
// waited for (use where the workgroup exchanges data through LDS alone).
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Block-wide exclusive scan of one value per thread (256 threads).
template <bool kLdsOnly = false>
__device__ inline uint32_t block_exscan(uint32_t v, uint32_t *tmp4, uint32_t *total) {
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t t = __shfl_up(x, off, 64);
    if (lane >= (uint32_t)off) x += t;
  }
  if (lane == 63) tmp4[w] = x;
  if (kLdsOnly) lds_barrier();
  else __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    uint32_t t = tmp4[i];
    if (i < (int)w) base += t;
    tot += t;
  }
  if (kLdsOnly) lds_barrier();
  else __syncthreads();
  *total = tot;
  return base + x - v;
}

// ---------------------------------------------------------------- scan --
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t *in, const uint32_t *n_dev,
                                                          uint32_t *partial) {
  __shared__ uint32_t tmp[kWaves];
  const uint32_t n = *n_dev;
  const uint32_t base = blockIdx.x * kScanTile;
  if (base >= n) return;
  uint32_t s = 0;
  for (uint32_t i = threadIdx.x; i < kScanTile; i += kThreads) {
    uint32_t e = base + i;
    if (e < n) s += in[e];
  }
  uint32_t tot;
  block_exscan(s, tmp, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kThreads) void k_scan_partials(uint32_t *partial, const uint32_t *n_dev) {
  __shared__ uint32_t tmp[kWaves];
  const uint32_t n = *n_dev;
  const uint32_t nb = (n + kScanTile - 1) / kScanTile;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nb; base += kThreads) {
    uint32_t e = base + threadIdx.x;
    uint32_t v = e < nb ? partial[e] : 0u;
    uint32_t tot;
    uint32_t ex = block_exscan(v, tmp, &tot);
    if (e < nb) partial[e] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) partial[nb] = carry;  // grand total
}

__global__ __launch_bounds__(kThreads) void k_scan_down(const uint32_t *in, uint32_t *out,
                                                        const uint32_t *n_dev, const uint32_t *partial) {
  __shared__ uint32_t buf[kScanTile];
  __shared__ uint32_t tmp[kWaves];
  const uint32_t n = *n_dev;
  const uint32_t base = blockIdx.x * kScanTile;
  const uint32_t nb = (n + kScanTile - 1) / kScanTile;
  if (base > n) return;
  if (base == n) {  // n is a multiple of the tile: this block only writes the total
    if (threadIdx.x == 0) out[n] = partial[nb];
    return;
  }
  for (uint32_t i = threadIdx.x; i < kScanTile; i += kThreads) {
    uint32_t e = base + i;
    buf[i] = e < n ? in[e] : 0u;
  }
  __syncthreads();
  constexpr uint32_t per = kScanTile / kThreads;  // 16 consecutive values per thread
  uint32_t loc[per];
  uint32_t s = 0;
#pragma unroll
  for (uint32_t k = 0; k < per; ++k) {
    loc[k] = buf[threadIdx.x * per + k];
    s += loc[k];
  }
  uint32_t tot;
  uint32_t ex = block_exscan(s, tmp, &tot) + partial[blockIdx.x];
#pragma unroll
  for (uint32_t k = 0; k < per; ++k) {
    buf[threadIdx.x * per + k] = ex;
    ex += loc[k];
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kScanTile; i += kThreads) {
    uint32_t e = base + i;
    if (e < n) out[e] = buf[i];
  }
  if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = partial[nb];
}

// --------------------------------------------------------------- frame --
// Order-preserving map of doubles to unsigned 64-bit integers.
__device__ inline uint64_t d2ord(double v) {
  uint64_t u = (uint64_t)__double_as_longlong(v);
  return (u >> 63) ? ~u : (u | (1ull << 63));
}
__device__ inline double ord2d(uint64_t u) {
  u = (u >> 63) ? (u & ~(1ull << 63)) : ~u;
  return __longlong_as_double((long long)u);
}

__global__ __launch_bounds__(kThreads) void k_frame_init(int B, uint64_t *minmax) {
  int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < 6 * B) minmax[i] = (i % 6) < 3 ? ~0ull : 0ull;
}

__global__ __launch_bounds__(kThreads) void k_frame_reduce(const BoxDev *boxes, int B, uint32_t n,
                                                           uint64_t *minmax, uint32_t *status) {
  uint32_t g = blockIdx.x * kThreads + threadIdx.x;
  if (g >= n) return;
  int b = box_of(boxes, B, g);
  const BoxDev &bx = boxes[b];
  if (bx.periodic) return;
  uint32_t i = g - bx.p_off;
  const double *x = bx.pos + 3ull * i;
  bool ok = true;
  uint64_t o[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double v = x[k];
    ok = ok && isfinite(v);
    o[k] = d2ord(v);
  }
  if (!ok) {
    atomicOr(status, kStatusRange);
    return;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    atomicMin((unsigned long long *)&minmax[6 * b + k], (unsigned long long)o[k]);
    atomicMax((unsigned long long *)&minmax[6 * b + 3 + k], (unsigned long long)o[k]);
  }
}

__global__ void k_frame_finalize(BoxDev *boxes, int B, const uint64_t *minmax) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  BoxDev &bx = boxes[b];
  if (bx.periodic) return;
  double L = 0.0;
  for (int k = 0; k < 3; ++k) {
    double lo = ord2d(minmax[6 * b + k]);
    double hi = ord2d(minmax[6 * b + 3 + k]);
    if (minmax[6 * b + k] == ~0ull) { lo = 0.0; hi = 0.0; }  // no finite point
    double e = hi - lo;
    if (e > L) L = e;
    bx.lo[k] = lo;
  }
  if (!(L > 0.0)) L = 1.0;
  bx.L = L;
  bx.scale = 2097152.0 / L;
  bx.Lf = (float)L;
  bx.h22f = (float)(L * 0x1p-22);
}

// ---------------------------------------------------------------- keys --
__device__ inline uint32_t cell_of(double x, double lo, double scale, bool &bad) {
  double v = (x - lo) * scale;
  if (!(v >= 0.0)) {  // below the root cube or NaN
    bad = true;
    return 0u;
  }
  if (v >= 2097151.0) return 2097151u;
  return (uint32_t)v;
}

__global__ __launch_bounds__(kThreads) void k_keys(const BoxDev *boxes, int B, uint32_t n,
                                                   uint64_t *keys, uint32_t *vals, uint32_t *status) {
  uint32_t g = blockIdx.x * kThreads + threadIdx.x;
  if (g >= n) return;
  const BoxDev &bx = boxes[box_of(boxes, B, g)];
  uint32_t i = g - bx.p_off;
  const double *x = bx.pos + 3ull * i;
  bool bad = false;
  uint32_t c[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double v = x[k];
    if (bx.periodic && !(v < bx.box)) bad = true;  // v >= box or NaN
    c[k] = cell_of(v, bx.lo[k], bx.scale, bad);
  }
  if (bad) atomicOr(status, kStatusRange);
  keys[g] = bx.curve ? hilbert3(c[0], c[1], c[2]) : morton3(c[0], c[1], c[2]);
  vals[g] = g;
}

// ---------------------------------------------------------------- sort --
constexpr int kSortItems = kSortTile / kThreads;  // 16 per thread

__device__ inline uint32_t sort_digit(uint64_t key, uint32_t val, int pass, const BoxDev *boxes,
                                      int B) {
  if (pass < 8) return (uint32_t)(key >> (8 * pass)) & 255u;
  return ((uint32_t)box_of(boxes, B, val) >> (8 * (pass - 8))) & 255u;
}

__global__ __launch_bounds__(kThreads) void k_sort_hist(const uint64_t *keys, const uint32_t *vals,
                                                        uint32_t n, int pass, const BoxDev *boxes,
                                                        int B, uint32_t *hist, uint32_t ntiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kSortTile;
#pragma unroll 4
  for (int r = 0; r < kSortItems; ++r) {
    uint32_t e = base + r * kThreads + threadIdx.x;
    // the key passes need no value
    if (e < n) atomicAdd(&h[sort_digit(keys[e], pass < 8 ? 0u : vals[e], pass, boxes, B)], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// One block per digit: exclusive scan of that digit's per-tile counts.
__global__ __launch_bounds__(kThreads) void k_sort_rowscan(uint32_t *hist, uint32_t ntiles,
                                                           uint32_t *digit_tot) {
  __shared__ uint32_t tmp[kWaves];
  uint32_t *row = hist + (size_t)blockIdx.x * ntiles;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < ntiles; base += kThreads) {
    uint32_t e = base + threadIdx.x;
    uint32_t v = e < ntiles ? row[e] : 0u;
    uint32_t tot;
    uint32_t ex = block_exscan(v, tmp, &tot);
    if (e < ntiles) row[e] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) digit_tot[blockIdx.x] = carry;
}

// Stable scatter of one tile.  Wave w owns tile elements
// [w*1024, (w+1)*1024) in 16 rounds of 64; ranks among equal digits come
// from ballot-matched peer masks, per-wave running counts, a scan over
// waves and a scan over digits.  The tile is reordered in LDS first so that
// the global writes of each digit run are contiguous.
__global__ __launch_bounds__(kThreads) void k_sort_scatter(const uint64_t *keys_in, const uint32_t *vals_in,
                                                           uint64_t *keys_out, uint32_t *vals_out,
                                                           uint32_t n, int pass, const BoxDev *boxes,
                                                           int B, const uint32_t *hist,
                                                           const uint32_t *digit_tot, uint32_t ntiles) {
  __shared__ uint64_t skeys[kSortTile];
  __shared__ uint32_t svals[kSortTile];
  __shared__ uint32_t wcnt[kWaves][256];
  __shared__ uint32_t gbase[256];    // global base of each digit for this tile
  __shared__ uint32_t tbase[256];    // base of each digit inside the tile
  __shared__ uint32_t tmp[kWaves];

  const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
  const uint32_t base = blockIdx.x * kSortTile;
  const uint32_t tile_n = min(kSortTile, n - base);

  // digit bases over the whole array: exclusive scan of the digit totals
  {
    uint32_t tot;
    uint32_t ex = block_exscan(digit_tot[tid], tmp, &tot);
    gbase[tid] = ex + hist[tid * ntiles + blockIdx.x];
  }
#pragma unroll
  for (int k = 0; k < kWaves; ++k) wcnt[k][tid] = 0;
  __syncthreads();

  uint64_t key[kSortItems];
  uint32_t val[kSortItems];
  uint32_t dig[kSortItems];
  uint32_t off[kSortItems];
  const uint32_t wbase = w * (kSortItems * 64);
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    uint32_t le = wbase + r * 64 + lane;
    bool valid = le < tile_n;
    key[r] = valid ? keys_in[base + le] : 0ull;
    val[r] = valid ? vals_in[base + le] : 0u;
    dig[r] = valid ? sort_digit(key[r], val[r], pass, boxes, B) : 0u;
  }
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    uint32_t le = wbase + r * 64 + lane;
    bool valid = le < tile_n;
    uint64_t peers = __ballot(valid);
    const uint32_t d = dig[r];
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      uint64_t bb = __ballot((d >> bit) & 1u);
      peers &= ((d >> bit) & 1u) ? bb : ~bb;
    }
    uint32_t leader = __ffsll((unsigned long long)peers) - 1;
    uint32_t rank = __popcll(peers & ((1ull << lane) - 1ull));
    uint32_t old = 0;
    if (valid && lane == leader) {
      old = wcnt[w][d];
      wcnt[w][d] = old + (uint32_t)__popcll(peers);
    }
    old = __shfl(old, valid ? leader : lane, 64);
    off[r] = old + rank;
  }
  __syncthreads();
  // per digit: exclusive scan over waves, then over digits
  {
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
      uint32_t t = wcnt[k][tid];
      wcnt[k][tid] = acc;
      acc += t;
    }
    uint32_t tot;
    tbase[tid] = block_exscan(acc, tmp, &tot);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    uint32_t le = wbase + r * 64 + lane;
    if (le < tile_n) {
      uint32_t lp = tbase[dig[r]] + wcnt[w][dig[r]] + off[r];
      skeys[lp] = key[r];
      svals[lp] = val[r];
    }
  }
  __syncthreads();
#pragma unroll 4
  for (int r = 0; r < kSortItems; ++r) {
    uint32_t e = r * kThreads + tid;
    if (e < tile_n) {
      uint64_t k = skeys[e];
      uint32_t v = svals[e];
      uint32_t d = sort_digit(k, v, pass, boxes, B);
      uint32_t gp = gbase[d] + (e - tbase[d]);
      keys_out[gp] = k;
      vals_out[gp] = v;
    }
  }
}

// -------------------------------------------------------------- gather --
__global__ __launch_bounds__(kThreads) void k_gather(const BoxDev *boxes, int B, uint32_t n,
                                                     const uint32_t *vals, uint32_t *perm,
                                                     uint32_t *inv, double4 *part64, double *seps,
                                                     uint32_t *status) {
  uint32_t p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  uint32_t g = vals[p];
  const BoxDev &bx = boxes[box_of(boxes, B, g)];
  uint32_t i = g - bx.p_off;
  const double *x = bx.pos + 3ull * i;
  part64[p] = make_double4(x[0], x[1], x[2], bx.mass[i]);
  perm[p] = g;
  inv[g] = p;
  if (seps) {
    const double e = bx.epsp ? bx.epsp[i] : bx.eps;
    if (!(e > 0.0 && e < INFINITY)) atomicOr(status, kStatusRange);
    seps[p] = e;
  }
}

// ------------------------------------------------------------ topology --
// lcp(p): levels shared by sorted keys p-1 and p inside one box; -1 at a
// box's first particle and past its last one.
// depth(p): the level of the leaf holding p = the smallest level whose node
// around p holds <= leaf_max particles (21 at most).  The node at level L
// around p holds 1 + #{neighbours q within leaf_max places with
// lcp-range-min >= L}, so depth = 1 + the leaf_max-th largest of the
// running minima of lcp to the right and to the left (merged, both
// sequences are non-increasing).  nstart(p) = nodes whose first particle
// is p = levels lcp(p)+1 .. depth(p).
// The block's lcp values, with a halo of lmax on each side, are formed once
// in LDS from the keys: lcp(q) = shared levels of keys q-1 and q, -1 at the
// first particle of a box and outside [0, n).  A particle's running minima
// pass through its box's first particle (left) or the next box's first
// particle (right) before they could leave its box, so values beyond
// contribute min(-1, .) = -1, as when each is evaluated against the box.
__global__ __launch_bounds__(kThreads) void k_lcp_depth(const BoxDev *boxes, int B, uint32_t n, int lmax,
                                                        const uint64_t *skeys, int8_t *lcp,
                                                        uint8_t *depth, uint32_t *nstart) {
  extern __shared__ int8_t sl[];  // lcp of particles lo .. lo + kThreads + 2 lmax
  const int64_t p0 = (int64_t)blockIdx.x * kThreads, lo = p0 - lmax;
  const int cnt = kThreads + 2 * lmax + 1;
  for (int i = threadIdx.x; i < cnt; i += kThreads) {
    const int64_t q = lo + i;
    int v = -1;
    if (q > 0 && q < (int64_t)n && (B == 1 || (uint32_t)q != boxes[box_of(boxes, B, (uint32_t)q)].p_off))
      v = shared_levels(skeys[q - 1], skeys[q]);
    sl[i] = (int8_t)v;
  }
  __syncthreads();
  const uint32_t p = (uint32_t)p0 + threadIdx.x;
  if (p >= n) return;
  const int lm = boxes[box_of(boxes, B, p)].leaf_max;
  const int8_t *L = sl + (p - lo);  // L[j] = lcp(p + j)
  const int own = L[0];
  int ri = 1, li = 1;
  int rv = L[1];
  int lv = own;
  int v = -1;
  for (int k = 0; k < lm; ++k) {
    if (rv >= lv) {
      v = rv;
      ++ri;
      rv = ri <= lm ? min(rv, (int)L[ri]) : -2;
    } else {
      v = lv;
      ++li;
      lv = (li <= lm && p + 1 >= (uint32_t)li) ? min(lv, (int)L[1 - li]) : -2;
    }
  }
  int d = min(kLevels, v + 1);
  lcp[p] = (int8_t)own;
  depth[p] = (uint8_t)d;
  nstart[p] = (uint32_t)max(0, d - own);
}

// Per box: node range [S[p_off], S[p_off+n]).
// Node range of each box; a box's root has no parent.
__global__ void k_box_nodes(BoxDev *boxes, int B, const uint32_t *S, uint32_t n, uint32_t node_cap,
                            uint32_t *scalars, uint32_t *parent) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) {
    const uint32_t root = min(S[boxes[b].p_off], node_cap);
    boxes[b].root = root;
    boxes[b].node_end = min(S[boxes[b].p_off + boxes[b].n], node_cap);
    if (root < node_cap) parent[root] = 0xffffffffu;
  }
  if (b == 0) {
    uint32_t tot = S[n];
    scalars[3] = min(tot, node_cap);
    if (tot > node_cap) atomicOr(&scalars[0], kStatusNodes);
  }
}

// End (exclusive) of the level-L node that starts at p: first q in (p, b1]
// whose key leaves the node's prefix; exponential then binary search.
__device__ inline uint32_t node_end(const uint64_t *skeys, uint32_t p, int L, uint32_t b1) {
  if (L == 0) return b1;
  const int sh = 63 - 3 * L;
  const uint64_t pre = skeys[p] >> sh;
  uint32_t lo = p, step = 1;  // lo: last index known inside the node
  while (true) {
    uint32_t q = lo + step;
    if (q >= b1 || (skeys[q] >> sh) != pre) break;
    lo = q;
    step <<= 1;
  }
  uint32_t hi = min(lo + step, b1);  // first index known outside (or b1)
  while (hi - lo > 1) {
    uint32_t mid = lo + ((hi - lo) >> 1);
    if ((skeys[mid] >> sh) == pre) lo = mid; else hi = mid;
  }
  return hi;
}

__global__ __launch_bounds__(kThreads) void k_emit(const BoxDev *boxes, int B, uint32_t n,
                                                   const uint64_t *skeys, const int8_t *lcp,
                                                   const uint8_t *depth, const uint32_t *S,
                                                   uint32_t node_cap, Topo *topo, uint32_t *first,
                                                   uint32_t *skip) {
  uint32_t p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  const int l0 = lcp[p], d = depth[p];
  if (d <= l0) return;
  const BoxDev &bx = boxes[box_of(boxes, B, p)];
  const uint32_t b1 = bx.p_off + bx.n;
  const uint64_t key = skeys[p];
  uint32_t cc[3];
  key_cell(key, bx.curve, cc);
  const uint32_t cx = cc[0], cy = cc[1], cz = cc[2];
  uint32_t rank = S[p];
  for (int L = l0 + 1; L <= d; ++L, ++rank) {
    if (rank >= node_cap) return;
    const uint32_t e = node_end(skeys, p, L, b1);
    const int drop = kLevels - L;
    const uint64_t corner = (uint64_t)((cx >> drop) << drop) | ((uint64_t)((cy >> drop) << drop) << 21) |
                            ((uint64_t)((cz >> drop) << drop) << 42);
    const bool leaf = (L == d);
    const uint32_t sk = S[e];
    Topo t;
    t.corner = corner | (leaf ? kLeafBit : 0ull);
    t.a = leaf ? p : sk;
    t.b = ((e - p) & kCountMask) | ((uint32_t)L << kCountBits);
    topo[rank] = t;
    first[rank] = p;
    skip[rank] = sk;
  }
}

// Parent links: every child of an internal node points at it.
__global__ __launch_bounds__(kThreads) void k_links(const Topo *topo, const uint32_t *skip,
                                                    const uint32_t *scalars, uint32_t node_cap,
                                                    uint32_t *parent) {
  const uint32_t tot = min(scalars[3], node_cap);
  for (uint32_t r = blockIdx.x * kThreads + threadIdx.x; r < tot; r += gridDim.x * kThreads) {
    const Topo t = topo[r];
    if (t.corner & kLeafBit) continue;
    const uint32_t end = min(t.a, tot);
    for (uint32_t c = r + 1; c < end;) {
      parent[c] = r;
      const uint32_t nx = skip[c];
      if (nx <= c) break;  // never taken for a well-formed tree
      c = nx;
    }
  }
}

// Cube centre of a node in FP64: lo + (corner + 2^(20-level)) L 2^-21.
__device__ inline void node_centre(const BoxDev &bx, uint64_t corner, int level, double c[3]) {
  const double h = bx.L * 0x1p-21;
  const double half = ldexp(1.0, 20 - level);
  c[0] = bx.lo[0] + ((double)(uint32_t)(corner & 0x1fffffull) + half) * h;
  c[1] = bx.lo[1] + ((double)(uint32_t)((corner >> 21) & 0x1fffffull) + half) * h;
  c[2] = bx.lo[2] + ((double)(uint32_t)((corner >> 42) & 0x1fffffull) + half) * h;
}

// Walk record (see WNode) and FP64 cube centre and side of node r.
__device__ inline void walk_records(const BoxDev &bx, const Topo &t, const Mom32 &m, uint32_t r, WNode *wn,
                                    double4 *cen64) {
  const int lev = (int)(t.b >> kCountBits);
  const int hc = 1 << (kLevels - lev);
  const bool leaf = (t.corner & kLeafBit) != 0;
  const float side = ldexpf(bx.Lf, -lev);
  WNode w;
  w.c[0] = 0x4B000000 | (2 * (int)(t.corner & 0x1fffffull) + hc);
  w.c[1] = 0x4B000000 | (2 * (int)((t.corner >> 21) & 0x1fffffull) + hc);
  w.c[2] = 0x4B000000 | (2 * (int)((t.corner >> 42) & 0x1fffffull) + hc);
  // the geometric criterion side^2 > theta^2 r^2 as one comparison with r^2
  w.side2 = bx.relative ? side * side : (bx.theta2f > 0.0f ? side * side / bx.theta2f : INFINITY);
  w.o[0] = m.ox;
  w.o[1] = m.oy;
  w.o[2] = m.oz;
  w.m = bx.Gf * m.m;  // G M: the FP32 pair term's factor
  w.reach = bx.rcutf + 0.5f * side;
  w.near = 0.6f * side;
  const uint32_t count = t.b & kCountMask;
  const bool wrap = bx.periodic && bx.rcutf + side >= 0.5f * bx.Lf;
  w.a = leaf ? leaf_tag_bits(t.a, min(count, 8u), wrap) : t.a;
  w.cf = count | (leaf && count > 8u ? kWBig : 0u) | (leaf ? kWLeaf : 0u) | (wrap ? kWWrap : 0u);
  wn[r] = w;
  // the FP64 walks' cube centre and side, in the expressions they used to
  // evaluate at every visit (so the values are the same to the bit)
  const double h = bx.L * 0x1p-21, half = ldexp(1.0, 20 - lev);
  cen64[r] = make_double4(bx.lo[0] + ((double)(uint32_t)(t.corner & 0x1fffffull) + half) * h,
                          bx.lo[1] + ((double)(uint32_t)((t.corner >> 21) & 0x1fffffull) + half) * h,
                          bx.lo[2] + ((double)(uint32_t)((t.corner >> 42) & 0x1fffffull) + half) * h,
                          ldexp(bx.L, -lev));
}

// Mass and centre of mass of node r from its mass M and first moments s
// about the cube centre c; FP64 and FP32 forms, then the walk records.
__device__ inline Mom64 store_node(const BoxDev &bx, const Topo &t, uint32_t r, const double c[3], double M,
                                   double s0, double s1, double s2, Mom64 *mom64, Mom32 *mom32, WNode *wn,
                                   double4 *cen64) {
  const Mom64 m{c[0] + s0 / M, c[1] + s1 / M, c[2] + s2 / M, M};
  mom64[r] = m;
  const Mom32 m32{(float)(m.cx - c[0]), (float)(m.cy - c[1]), (float)(m.cz - c[2]), (float)M};
  mom32[r] = m32;
  walk_records(bx, t, m32, r, wn, cen64);
  return m;
}

// One particle q of a leaf with cube centre c: its mass and first moments
// added.
__device__ inline void leaf_add(const double4 q, const double c[3], double &M, double &s0, double &s1, double &s2) {
  const double dx = q.x - c[0], dy = q.y - c[1], dz = q.z - c[2];
  M += q.w;
  s0 += q.w * dx;
  s1 += q.w * dy;
  s2 += q.w * dz;
}

// A leaf particle's FP32 offset from the leaf's centre of mass m (the mixed
// walk adds it to the target's offset from that centre) and its G times
// mass (the product the FP32 pair term would form, rounded the same way).
__device__ inline float4 leaf_offset(const double4 q, const Mom64 &m, float Gf) {
  return make_float4((float)(q.x - m.cx), (float)(q.y - m.cy), (float)(q.z - m.cz), Gf * (float)q.w);
}

// Sums of an internal node over its children's moments, in child order.
struct ChildSums {
  double c[3];
  double M = 0.0, q0 = 0.0, q1 = 0.0, q2 = 0.0, hi = 0.0, lo = INFINITY;
  __device__ void add(const Mom64 &m) {
    M += m.m;
    q0 += m.m * (m.cx - c[0]);
    q1 += m.m * (m.cy - c[1]);
    q2 += m.m * (m.cz - c[2]);
  }
  __device__ void add_lengths(double h, double l) {
    hi = h > hi ? h : hi;
    lo = l < lo ? l : lo;
  }
};

// Node after the last node of r's subtree (pre-order).
__device__ inline uint32_t subtree_end(const Topo &t, uint32_t r, uint32_t tot) {
  return (t.corner & kLeafBit) ? r + 1 : max(r + 1, min(t.a, tot));
}

__device__ inline const BoxDev &node_box(const BoxDev *boxes, int B, const uint32_t *first, uint32_t r) {
  return boxes[B == 1 ? 0 : box_of(boxes, B, first[r])];
}

// Bottom-up moments (paper, "Tree construction": a bottom-up pass computes
// each node's mass and centre of mass).  Leaves sum their particles about
// the cube centre (and write each particle's FP32 offset from it); an
// internal node sums its children in child order.  Every node is summed
// once, in that fixed order, so the result is deterministic.  Every node
// also gets its walk records (WNode, FP64 centre), and with per-particle
// softening lengths (seps non-null) the largest and smallest length of its
// particles (semax, semin).
// The order of work, in three launches:
//  - k_moments_leaves sums every leaf and classifies every node: a node
//    whose subtree holds more than kSegNodes nodes is a top node; one with
//    at most kSegNodes whose parent is a top node (or which has no parent)
//    roots a segment, a contiguous pre-order range of nodes.  Top nodes
//    are listed, each with eight empty child slots.
//  - k_moments_segments: a workgroup takes the segments whose roots lie in
//    its chunk of kSegChunk node indices and sums their internal nodes
//    level by level, deepest first, with the moments in LDS; each child of
//    a top node in the chunk takes its octant slot in its parent's entry.
//  - k_moments_top: one workgroup sums the top nodes level by level.
constexpr uint32_t kSegChunk = kThreads;               // one chunk node per thread
constexpr uint32_t kSegRange = kSegChunk + kSegNodes;  // nodes a chunk's segments can span
constexpr uint32_t kSegPer = kSegRange / kThreads;     // range positions per thread
static_assert(kSegRange % kThreads == 0 && kSegRange < 0xffffu, "segment range in whole rounds, 16-bit");
constexpr int kLeafStage = 1024;                       // leaf particles staged per round (32 KB)
constexpr uint32_t kNone = 0xffffffffu;
constexpr uint32_t kTopRef = 0x80000000u;              // in a child slot: a top node's index in the top list
constexpr uint32_t kClsRoot = 1u;                      // node class: roots a segment
constexpr uint32_t kClsTop = 0x80000000u;              // node class: top node (| its index in the top list)

// Octant of a node's cube in its parent (the cell parity at its own level).
__device__ inline uint32_t octant(const Topo &t) {
  const int sh = kLevels - (int)(t.b >> kCountBits);
  return (uint32_t)((t.corner >> sh) & 1u) | (uint32_t)((t.corner >> (21 + sh)) & 1u) << 1 |
         (uint32_t)((t.corner >> (42 + sh)) & 1u) << 2;
}

__global__ __launch_bounds__(kThreads) void k_moments_leaves(const BoxDev *boxes, int B, const Topo *topo,
                                                             const uint32_t *parent, const double4 *part64,
                                                             float4 *part32, Mom64 *mom64, Mom32 *mom32,
                                                             WNode *wn, double4 *cen64, uint32_t *scalars,
                                                             uint32_t node_cap, TopArrays T, const double *seps,
                                                             double *semax, double *semin) {
  // the round's leaf particles, loaded coalesced (a leaf's thread would
  // otherwise read its particles with a stride of a leaf between lanes)
  __shared__ double4 stage[kLeafStage];
  __shared__ uint32_t prange[2], s_ntop, s_tlev, s_tbase;
  const uint32_t tot = min(scalars[3], node_cap);
  for (uint32_t r0 = blockIdx.x * kThreads; r0 < tot; r0 += gridDim.x * kThreads) {
    const uint32_t r = r0 + threadIdx.x;
    if (threadIdx.x == 0) {
      prange[0] = 0xffffffffu;
      prange[1] = 0u;
      s_ntop = 0;
      s_tlev = 0;
    }
    lds_barrier();
    Topo t{};
    uint32_t top_slot = kNone;
    const bool in = r < tot;
    if (in) {
      t = topo[r];
      const uint32_t p = parent[r];
      const bool has_p = p < tot;
      const bool ptop = has_p && subtree_end(topo[p], p, tot) - p > kSegNodes;
      if (subtree_end(t, r, tot) - r > kSegNodes) {
        top_slot = atomicAdd(&s_ntop, 1u);
        atomicMax(&s_tlev, t.b >> kCountBits);
      } else {
        T.id[r] = !has_p || ptop ? kClsRoot : 0u;
      }
      if (t.corner & kLeafBit) {
        atomicMin(&prange[0], t.a);
        atomicMax(&prange[1], t.a + (t.b & kCountMask));
      }
    }
    lds_barrier();
    if (threadIdx.x == 0) {  // one reservation per workgroup and round in the top lists
      if (s_ntop) {
        s_tbase = atomicAdd(&T.cnt[0], s_ntop);
        atomicMax(&T.cnt[2], s_tlev);
      }
    }
    const uint32_t pa = prange[0], pn = prange[1] > pa ? prange[1] - pa : 0u;
    const bool staged = pn <= (uint32_t)kLeafStage;
    if (staged)
      for (uint32_t i = threadIdx.x; i < pn; i += kThreads) stage[i] = part64[pa + i];
    lds_barrier();
    if (top_slot != kNone) {
      const uint32_t k = s_tbase + top_slot;
      if (k < T.cap) {
        T.list[k] = make_uint4(r, t.b >> kCountBits, (uint32_t)t.corner, (uint32_t)(t.corner >> 32));
#pragma unroll
        for (int q = 0; q < 8; ++q) T.slot[8 * k + q] = ~0ull;
        T.id[r] = kClsTop | k;
      } else {
        T.id[r] = 0u;
        atomicOr(&scalars[0], kStatusNodes);
      }
    }
    if (in && (t.corner & kLeafBit)) {
      const uint32_t f = t.a, cnt = t.b & kCountMask;
      const BoxDev &bx = boxes[B == 1 ? 0 : box_of(boxes, B, f)];
      double c[3];
      node_centre(bx, t.corner, (int)(t.b >> kCountBits), c);
      double M = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
      // (two loops: a select between an LDS and a global pointer is not
      // formed, which this compiler mishandles)
      if (staged) {
        for (uint32_t j = f; j < f + cnt; ++j) leaf_add(stage[j - pa], c, M, s0, s1, s2);
      } else {
        for (uint32_t j = f; j < f + cnt; ++j) leaf_add(part64[j], c, M, s0, s1, s2);
      }
      const Mom64 m = store_node(bx, t, r, c, M, s0, s1, s2, mom64, mom32, wn, cen64);
      if (staged) {
        for (uint32_t j = f; j < f + cnt; ++j) part32[j] = leaf_offset(stage[j - pa], m, bx.Gf);
      } else {
        for (uint32_t j = f; j < f + cnt; ++j) part32[j] = leaf_offset(part64[j], m, bx.Gf);
      }
      if (seps) {
        double hi = seps[f], lo = hi;
        for (uint32_t j = f + 1; j < f + cnt; ++j) {
          hi = seps[j] > hi ? seps[j] : hi;
          lo = seps[j] < lo ? seps[j] : lo;
        }
        semax[r] = hi;
        semin[r] = lo;
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_moments_segments(const BoxDev *boxes, int B, const Topo *topo,
                                                               const uint32_t *first, const uint32_t *parent,
                                                               const uint32_t *cls, Mom64 *mom64, Mom32 *mom32,
                                                               WNode *wn, double4 *cen64, const uint32_t *scalars,
                                                               uint32_t node_cap, TopArrays T, double *semax,
                                                               double *semin) {
  __shared__ Mom64 smom[kSegRange];
  __shared__ uint16_t send[kSegRange];  // per position: the position after its subtree
  __shared__ int32_t mark[kSegRange];   // +1 at segment roots, -1 at their ends; then prefix sums
  __shared__ uint32_t tmp4[kWaves], s_end, s_lo, s_hi;
  const uint32_t tot = min(scalars[3], node_cap);
  for (uint32_t base = blockIdx.x * kSegChunk; base < tot; base += gridDim.x * kSegChunk) {
    lds_barrier();  // the previous chunk is done with the shared arrays
    for (uint32_t i = threadIdx.x; i < kSegRange; i += kThreads) mark[i] = 0;
    if (threadIdx.x == 0) {
      s_end = base;
      s_lo = kLevels + 1;
      s_hi = 0;
    }
    lds_barrier();
    // range position i = threadIdx.x + k kThreads is node base + i
    Topo t[kSegPer];
    bool mine[kSegPer];
    const uint32_t x = base + threadIdx.x;
    uint32_t xcls = 0;
    if (x < tot) {
      t[0] = topo[x];
      xcls = cls[x];
      if (xcls == kClsRoot) {
        const uint32_t e = subtree_end(t[0], x, tot);  // e - base < kSegRange (at most kSegNodes nodes)
        atomicAdd(&mark[threadIdx.x], 1);
        atomicSub(&mark[e - base], 1);
        atomicMax(&s_end, e);
        atomicMin(&s_lo, t[0].b >> kCountBits);
      }
    }
    lds_barrier();
    // a segment root or top node with a parent: the parent is a top node;
    // the child takes its slot there as (node << 32 | ref), ref its top-list
    // index with kTopRef or, for a segment root, the node
    if (x < tot && xcls != 0u) {
      const uint32_t p = parent[x];
      if (p < tot) {
        const uint32_t pc = cls[p];
        if ((pc & kClsTop) && (pc & ~kClsTop) < T.cap) {
          const uint32_t ref = (xcls & kClsTop) ? kTopRef | (xcls & ~kClsTop) : x;
          T.slot[8 * (pc & ~kClsTop) + octant(t[0])] = (uint64_t)x << 32 | ref;
        }
      }
    }
    const uint32_t rlen = s_end - base;  // this chunk's segments lie in [base, s_end)
    if (rlen == 0) continue;
    {  // inclusive prefix sums of the marks: 1 inside a segment, 0 elsewhere
      int32_t v[kSegPer];
      uint32_t run = 0, total;
#pragma unroll
      for (uint32_t k = 0; k < kSegPer; ++k) {
        v[k] = mark[threadIdx.x * kSegPer + k];
        run += (uint32_t)v[k];
      }
      int32_t acc = (int32_t)block_exscan<true>(run, tmp4, &total);
#pragma unroll
      for (uint32_t k = 0; k < kSegPer; ++k) {
        acc += v[k];
        mark[threadIdx.x * kSegPer + k] = acc;
      }
    }
    lds_barrier();
    // the leaves' moments and every node's subtree end into LDS
#pragma unroll
    for (uint32_t k = 0; k < kSegPer; ++k) {
      const uint32_t i = threadIdx.x + k * kThreads;
      mine[k] = i < rlen && mark[i] > 0;
      if (!mine[k]) continue;
      if (k > 0) t[k] = topo[base + i];
      send[i] = (uint16_t)(min(subtree_end(t[k], base + i, tot), base + rlen) - base);
      if (t[k].corner & kLeafBit) smom[i] = mom64[base + i];
      else atomicMax(&s_hi, t[k].b >> kCountBits);
    }
    lds_barrier();  // slots, leaf moments and s_hi complete
    // internal nodes, deepest level first
    for (int L = (int)s_hi; L >= (int)s_lo; --L) {
      if (semax) __syncthreads();  // children's lengths written (global memory)
      else if (L != (int)s_hi) lds_barrier();
      // positions of this level as a bit mask; one copy of the body (the
      // position's topology picked by selects, not by indexing)
      uint32_t todo = 0;
#pragma unroll
      for (uint32_t k = 0; k < kSegPer; ++k)
        if (mine[k] && !(t[k].corner & kLeafBit) && (int)(t[k].b >> kCountBits) == L) todo |= 1u << k;
      while (todo) {
        const uint32_t k = __builtin_ctz(todo);
        todo &= todo - 1;
        Topo tk = t[0];
#pragma unroll
        for (uint32_t q = 1; q < kSegPer; ++q)
          if (k == q) tk = t[q];
        const uint32_t i = threadIdx.x + k * kThreads, r = base + i;
        const BoxDev &bx = node_box(boxes, B, first, r);
        ChildSums cs;
        node_centre(bx, tk.corner, L, cs.c);
        // children in child order: the first follows r, each next one
        // follows the previous one's subtree
        const uint32_t pend = send[i];
        for (uint32_t c = i + 1; c < pend;) {
          cs.add(smom[c]);
          if (semax) cs.add_lengths(semax[base + c], semin[base + c]);
          const uint32_t nx = send[c];
          if (nx <= c) break;  // never taken for a well-formed tree
          c = nx;
        }
        smom[i] = store_node(bx, tk, r, cs.c, cs.M, cs.q0, cs.q1, cs.q2, mom64, mom32, wn, cen64);
        if (semax) {
          semax[r] = cs.hi;
          semin[r] = cs.lo;
        }
      }
    }
  }
}

// The top nodes (subtrees of more than kSegNodes nodes), summed by one
// workgroup after the segments, level by level, deepest first.  A top
// node's slots hold its children (top nodes and segment roots) by octant
// as (node << 32 | ref); sorted, they give child order.  With at most
// kTopThreads top nodes every thread holds one, its slots and its segment
// -root children's moments in registers, and the top nodes' moments stay
// in LDS, so the levels cost no memory round trip; larger sets read slots
// and moments from global memory at every level.  FP32 moments and walk
// records follow.
constexpr int kTopThreads = 1024;

// A node's slots in child order (empty slots, all ones, sort last).
__device__ inline void sort_slots(uint64_t sl[8]) {
#pragma unroll
  for (int q = 1; q < 8; ++q)
#pragma unroll
    for (int j = q; j > 0; --j)
      if (sl[j] < sl[j - 1]) {
        const uint64_t u = sl[j];
        sl[j] = sl[j - 1];
        sl[j - 1] = u;
      }
}

__device__ inline Mom64 top_mom(const ChildSums &cs) {
  return Mom64{cs.c[0] + cs.q0 / cs.M, cs.c[1] + cs.q1 / cs.M, cs.c[2] + cs.q2 / cs.M, cs.M};
}

__device__ inline void top_records(const BoxDev &bx, const Topo &t, uint32_t r, const double c[3],
                                   const Mom64 &m, Mom32 *mom32, WNode *wn, double4 *cen64) {
  const Mom32 m32{(float)(m.cx - c[0]), (float)(m.cy - c[1]), (float)(m.cz - c[2]), (float)m.m};
  mom32[r] = m32;
  walk_records(bx, t, m32, r, wn, cen64);
}

__global__ __launch_bounds__(kTopThreads) void k_moments_top(const BoxDev *boxes, int B, const Topo *topo,
                                                             const uint32_t *first, Mom64 *mom64, Mom32 *mom32,
                                                             WNode *wn, double4 *cen64, TopArrays T,
                                                             double *semax, double *semin) {
  __shared__ Mom64 smt[kTopThreads];
  const uint32_t ntop = min(T.cnt[0], T.cap);
  if (ntop == 0) return;
  const int hi = (int)min(T.cnt[2], (uint32_t)kLevels);
  if (ntop <= (uint32_t)kTopThreads && semax == nullptr) {
    // one top node per thread, everything it needs in registers
    const uint32_t i = threadIdx.x;
    const bool own = i < ntop;
    int lev = -1;
    uint32_t r = 0;
    uint64_t sl[8];
    Mom64 m[8];
    ChildSums cs;
    Topo t{};
    if (own) {
      const uint4 e = T.list[i];
      r = e.x;
      lev = (int)min(e.y, (uint32_t)kLevels);
      t = topo[r];
      node_centre(node_box(boxes, B, first, r), (uint64_t)e.z | (uint64_t)e.w << 32, lev, cs.c);
#pragma unroll
      for (int q = 0; q < 8; ++q) sl[q] = T.slot[8 * i + q];
      sort_slots(sl);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (sl[q] != ~0ull && !((uint32_t)sl[q] & kTopRef)) m[q] = mom64[(uint32_t)(sl[q] >> 32)];
    }
    for (int L = hi; L >= 0; --L) {
      lds_barrier();  // deeper levels summed
      if (lev != L) continue;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (sl[q] == ~0ull) continue;
        if ((uint32_t)sl[q] & kTopRef) m[q] = smt[(uint32_t)sl[q] & ~kTopRef];
        cs.add(m[q]);
      }
      const Mom64 mr = top_mom(cs);
      smt[i] = mr;
      mom64[r] = mr;
      top_records(node_box(boxes, B, first, r), t, r, cs.c, mr, mom32, wn, cen64);
    }
    return;
  }
  for (int L = hi; L >= 0; --L) {
    __syncthreads();  // deeper levels summed (global memory)
    for (uint32_t i = threadIdx.x; i < ntop; i += kTopThreads) {
      const uint4 e = T.list[i];
      if ((int)e.y != L) continue;
      const uint32_t r = e.x;
      uint64_t sl[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) sl[q] = T.slot[8 * i + q];
      sort_slots(sl);
      Mom64 m[8];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (sl[q] != ~0ull) m[q] = mom64[(uint32_t)(sl[q] >> 32)];
      const BoxDev &bx = node_box(boxes, B, first, r);
      ChildSums cs;
      node_centre(bx, (uint64_t)e.z | (uint64_t)e.w << 32, L, cs.c);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (sl[q] != ~0ull) cs.add(m[q]);
      const Mom64 mr = top_mom(cs);
      mom64[r] = mr;
      if (semax) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (sl[q] != ~0ull) {
            const uint32_t node = (uint32_t)(sl[q] >> 32);
            cs.add_lengths(semax[node], semin[node]);
          }
        semax[r] = cs.hi;
        semin[r] = cs.lo;
      }
      top_records(bx, topo[r], r, cs.c, mr, mom32, wn, cen64);
    }
  }
}

// --------------------------------------------------- targets (subsets) --
__global__ __launch_bounds__(kThreads) void k_targets_map(const BoxDev *boxes, const int64_t *idx,
                                                          uint32_t M, const uint32_t *inv,
                                                          uint64_t *tkey, uint32_t *tval,
                                                          uint32_t *status) {
  uint32_t t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= M) return;
  int64_t i = idx[t];
  const uint32_t n = boxes[0].n;
  if (i < 0 || i >= (int64_t)n) {  // reported through the tree's status word
    atomicOr(status, kStatusTarget);
    i = 0;
  }
  tkey[t] = inv[(uint32_t)i];
  tval[t] = t;
}

__global__ __launch_bounds__(kThreads) void k_max_level(const Topo *topo, const uint32_t *scalars,
                                                        uint32_t node_cap, uint32_t *out) {
  __shared__ uint32_t m;
  if (threadIdx.x == 0) m = 0;
  __syncthreads();
  const uint32_t tot = min(scalars[3], node_cap);
  uint32_t v = 0;
  for (uint32_t r = blockIdx.x * kThreads + threadIdx.x; r < tot; r += gridDim.x * kThreads)
    v = max(v, topo[r].b >> kCountBits);
  atomicMax(&m, v);
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(out, m);
}

__global__ void k_reset(uint32_t *w) { *w = 0; }
__global__ void k_reset_n(uint32_t *w, int n) {
  if ((int)threadIdx.x < n) w[threadIdx.x] = 0;
}
// Status word cleared, particle count for the device-side scans, counters
// of the top-node lists cleared.
__global__ void k_init_scalars(uint32_t *sc, uint32_t n, uint32_t *top_cnt) {
  if (threadIdx.x == 0) {
    sc[0] = 0u;
    sc[4] = n;
  }
  if (threadIdx.x < 4) top_cnt[threadIdx.x] = 0;
}

inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

int g_cu = 0;

}  // namespace

int device_cu_count() {
  if (g_cu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0)
      cu = 256;
    g_cu = cu;
  }
  return g_cu;
}

void launch_reset(uint32_t *word, hipStream_t s) { k_reset<<<1, 1, 0, s>>>(word); }
void launch_reset_n(uint32_t *words, int n, hipStream_t s) { k_reset_n<<<1, 64, 0, s>>>(words, n); }

void launch_max_level(const BuildArrays &A, uint32_t *out, hipStream_t s) {
  k_reset<<<1, 1, 0, s>>>(out);
  const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>(cdiv(A.node_cap, kThreads), 1024));
  k_max_level<<<g, kThreads, 0, s>>>(A.topo, A.scalars, A.node_cap, out);
}

void scan_u32(const uint32_t *in, uint32_t *out, const uint32_t *n_dev, uint32_t cap,
              uint32_t *partial, hipStream_t s) {
  const uint32_t nb = cdiv((uint64_t)cap + 1, kScanTile);
  k_scan_reduce<<<nb, kThreads, 0, s>>>(in, n_dev, partial);
  k_scan_partials<<<1, kThreads, 0, s>>>(partial, n_dev);
  k_scan_down<<<nb, kThreads, 0, s>>>(in, out, n_dev, partial);
}

size_t radix_hist_words(uint32_t n) { return (size_t)256 * cdiv(n > 0 ? n : 1, kSortTile); }

bool radix_sort(uint64_t *keys_a, uint32_t *vals_a, uint64_t *keys_b, uint32_t *vals_b, uint32_t n,
                int pass_lo, int pass_hi, int box_passes, const BoxDev *boxes, int B,
                uint32_t *hist, uint32_t *digit_tot, hipStream_t s) {
  const uint32_t ntiles = cdiv(n, kSortTile);
  uint64_t *ki = keys_a, *ko = keys_b;
  uint32_t *vi = vals_a, *vo = vals_b;
  bool in_b = false;
  for (int pass = pass_lo; pass < pass_hi + box_passes; ++pass) {
    const int pp = pass < pass_hi ? pass : 8 + (pass - pass_hi);
    k_sort_hist<<<ntiles, kThreads, 0, s>>>(ki, vi, n, pp, boxes, B, hist, ntiles);
    k_sort_rowscan<<<256, kThreads, 0, s>>>(hist, ntiles, digit_tot);
    k_sort_scatter<<<ntiles, kThreads, 0, s>>>(ki, vi, ko, vo, n, pp, boxes, B, hist, digit_tot, ntiles);
    std::swap(ki, ko);
    std::swap(vi, vo);
    in_b = !in_b;
  }
  return in_b;
}

void launch_build(BuildArrays &A, hipStream_t s) {
  const uint32_t n = A.n;
  const uint32_t nb = cdiv(n, kThreads);
  k_init_scalars<<<1, 64, 0, s>>>(A.scalars, n, A.top_cnt);
  if (A.any_open) {
    k_frame_init<<<cdiv(6 * (uint64_t)A.B, kThreads), kThreads, 0, s>>>(A.B, A.minmax);
    k_frame_reduce<<<nb, kThreads, 0, s>>>(A.boxes, A.B, n, A.minmax, &A.scalars[0]);
    k_frame_finalize<<<cdiv(A.B, 64), 64, 0, s>>>(A.boxes, A.B, A.minmax);
  }
  // Start in the buffer pair that makes the sorted result land in *_a.
  const int box_passes = A.B <= 1 ? 0 : (A.B <= 256 ? 1 : 2);
  const bool odd = ((8 + box_passes) & 1) != 0;
  uint64_t *k0 = odd ? A.keys_b : A.keys_a, *k1 = odd ? A.keys_a : A.keys_b;
  uint32_t *v0 = odd ? A.vals_b : A.vals_a, *v1 = odd ? A.vals_a : A.vals_b;
  {
    const TraceRange r("build: keys");
    k_keys<<<nb, kThreads, 0, s>>>(A.boxes, A.B, n, k0, v0, &A.scalars[0]);
  }
  {
    const TraceRange r("build: radix sort");
    radix_sort(k0, v0, k1, v1, n, 0, 8, box_passes, A.boxes, A.B, A.hist, A.digit_tot, s);
  }
  const uint64_t *skeys = A.keys_a;
  {
    const TraceRange r("build: gather");
    k_gather<<<nb, kThreads, 0, s>>>(A.boxes, A.B, n, A.vals_a, A.perm, A.inv, A.part64, A.seps, &A.scalars[0]);
  }
  const uint32_t gnodes = std::max<uint32_t>(1, std::min<uint32_t>(cdiv(A.node_cap, kThreads), 8192));
  {
    const TraceRange r("build: topology");
    k_lcp_depth<<<nb, kThreads, kThreads + 2 * A.leaf_max + 1, s>>>(A.boxes, A.B, n, A.leaf_max, skeys, A.lcp,
                                                                    A.depth, A.nstart);
    scan_u32(A.nstart, A.S, &A.scalars[4], n, A.scan_partial, s);
    k_box_nodes<<<cdiv(A.B, 64), 64, 0, s>>>(A.boxes, A.B, A.S, n, A.node_cap, A.scalars, A.parent);
    k_emit<<<nb, kThreads, 0, s>>>(A.boxes, A.B, n, skeys, A.lcp, A.depth, A.S, A.node_cap, A.topo,
                                   A.first, A.skip);
    k_links<<<gnodes, kThreads, 0, s>>>(A.topo, A.skip, A.scalars, A.node_cap, A.parent);
  }
  {
    const TraceRange r("build: moments");
    const size_t c = A.top_cap;
    const TopArrays T{A.top_cnt, reinterpret_cast<uint4 *>(A.top_buf), reinterpret_cast<uint64_t *>(A.top_buf + 4 * c),
                      A.top_id, A.top_cap};
    // grid-stride over nodes (the node count is known on the device only)
    const uint32_t gleaf = std::max<uint32_t>(1, std::min<uint32_t>(cdiv(A.node_cap, kThreads), 4096));
    k_moments_leaves<<<gleaf, kThreads, 0, s>>>(A.boxes, A.B, A.topo, A.parent, A.part64, A.part32, A.mom64,
                                                A.mom32, A.wnode, A.cen64, A.scalars, A.node_cap, T, A.seps,
                                                A.semax, A.semin);
    const uint32_t gseg = std::max<uint32_t>(1, std::min<uint32_t>(cdiv(A.node_cap, kSegChunk), 4096));
    k_moments_segments<<<gseg, kThreads, 0, s>>>(A.boxes, A.B, A.topo, A.first, A.parent, A.top_id, A.mom64,
                                                 A.mom32, A.wnode, A.cen64, A.scalars, A.node_cap, T, A.semax,
                                                 A.semin);
    k_moments_top<<<1, kTopThreads, 0, s>>>(A.boxes, A.B, A.topo, A.first, A.mom64, A.mom32, A.wnode, A.cen64, T,
                                            A.semax, A.semin);
  }
}


// Active targets (see ActiveArrays).  Flags and the compaction run over the
// sorted order, so the active list keeps the curve order of the tree.
__global__ __launch_bounds__(kThreads) void k_active_flags(const uint32_t *perm, const int8_t *bin,
                                                           int32_t level, uint32_t n, uint32_t *flags) {
  const uint32_t p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  flags[p] = (int32_t)bin[perm[p]] <= level ? 1u : 0u;
}

__global__ __launch_bounds__(kThreads) void k_active_scatter(const uint32_t *flags, const uint32_t *offs,
                                                             const uint32_t *perm, uint32_t n, uint32_t chunk,
                                                             uint64_t *tkey, uint32_t *tval, uint32_t *counts,
                                                             int64_t *n_active) {
  const uint32_t p = blockIdx.x * kThreads + threadIdx.x;
  if (p == 0) {
    const uint32_t m = offs[n];
    counts[0] = m;
    counts[1] = (m + chunk - 1) / chunk;
    if (n_active) *n_active = (int64_t)m;
  }
  if (p >= n || !flags[p]) return;
  const uint32_t o = offs[p];
  tkey[o] = p;
  tval[o] = perm[p];
}

size_t scan_partial_words(uint32_t n) { return cdiv((uint64_t)n + 1, kScanTile) + 1; }

void launch_active(const BuildArrays &A, ActiveArrays &T, uint32_t chunk, hipStream_t s) {
  const uint32_t n = A.n;
  k_active_flags<<<cdiv(n, kThreads), kThreads, 0, s>>>(A.perm, T.bin, T.level, n, T.flags);
  scan_u32(T.flags, T.offs, &A.scalars[4], n, T.partial, s);
  k_active_scatter<<<cdiv(n, kThreads), kThreads, 0, s>>>(T.flags, T.offs, A.perm, n, chunk, T.tkey, T.tval,
                                                         T.counts, T.n_active);
}

void launch_targets(const BuildArrays &A, TargetArrays &T, hipStream_t s) {
  const uint32_t M = T.M;
  k_reset<<<1, 1, 0, s>>>(&T.scalars[0]);
  k_targets_map<<<cdiv(M, kThreads), kThreads, 0, s>>>(A.boxes, T.idx, M, A.inv, T.tkey_a, T.tval_a,
                                                      &A.scalars[0]);
  int passes = 1;
  while (passes < 4 && (A.n >> (8 * passes)) != 0) ++passes;
  bool in_b = radix_sort(T.tkey_a, T.tval_a, T.tkey_b, T.tval_b, M, 0, passes, 0, A.boxes, 1, T.hist,
                         T.digit_tot, s);
  T.tkey = in_b ? T.tkey_b : T.tkey_a;
  T.tval = in_b ? T.tval_b : T.tval_a;
}

}  // namespace og
