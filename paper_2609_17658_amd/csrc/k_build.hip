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

// Block-wide exclusive scan of one value per thread (256 threads).
__device__ inline uint32_t block_exscan(uint32_t v, uint32_t *tmp4, uint32_t *total) {
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t t = __shfl_up(x, off, 64);
    if (lane >= (uint32_t)off) x += t;
  }
  if (lane == 63) tmp4[w] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    uint32_t t = tmp4[i];
    if (i < (int)w) base += t;
    tot += t;
  }
  __syncthreads();
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
__device__ inline int lcp_at(const uint64_t *skeys, uint32_t q, uint32_t b0, uint32_t b1) {
  if (q <= b0 || q >= b1) return -1;
  return shared_levels(skeys[q - 1], skeys[q]);
}

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

// Parent links and child counts; counts the internal nodes of each level.
__global__ __launch_bounds__(kThreads) void k_links(const Topo *topo, const uint32_t *skip,
                                                    const uint32_t *scalars, uint32_t node_cap,
                                                    uint32_t *parent, uint32_t *nchild,
                                                    uint32_t *lvl_cnt) {
  __shared__ uint32_t h[kLevels + 1];
  if (threadIdx.x <= kLevels) h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t tot = min(scalars[3], node_cap);
  for (uint32_t r = blockIdx.x * kThreads + threadIdx.x; r < tot; r += gridDim.x * kThreads) {
    const Topo t = topo[r];
    uint32_t nc = 0;
    if (!(t.corner & kLeafBit)) {
      const uint32_t end = min(t.a, tot);
      for (uint32_t c = r + 1; c < end;) {
        parent[c] = r;
        ++nc;
        const uint32_t nx = skip[c];
        if (nx <= c) break;  // never taken for a well-formed tree
        c = nx;
      }
      atomicAdd(&h[t.b >> kCountBits], 1u);
    }
    nchild[r] = nc;
  }
  __syncthreads();
  if (threadIdx.x <= kLevels && h[threadIdx.x]) atomicAdd(&lvl_cnt[threadIdx.x], h[threadIdx.x]);
}

// Particles staged in LDS per round of the leaf-moment kernel (32 KB).
constexpr int kLeafStage = 1024;

// Cube centre of a node in FP64: lo + (corner + 2^(20-level)) L 2^-21.
__device__ inline void node_centre(const BoxDev &bx, uint64_t corner, int level, double c[3]) {
  const double h = bx.L * 0x1p-21;
  const double half = ldexp(1.0, 20 - level);
  c[0] = bx.lo[0] + ((double)(uint32_t)(corner & 0x1fffffull) + half) * h;
  c[1] = bx.lo[1] + ((double)(uint32_t)((corner >> 21) & 0x1fffffull) + half) * h;
  c[2] = bx.lo[2] + ((double)(uint32_t)((corner >> 42) & 0x1fffffull) + half) * h;
}

// Bottom-up moments, level by level (paper, "Tree construction": a
// bottom-up pass computes each node's mass and centre of mass).  Leaves sum
// their particles relative to the cube centre (and write each particle's
// FP32 offset from that centre); internal nodes are bucketed by level and
// each level, deepest first, sums its children in child order.  Every
// node is summed once in a fixed order, so the result is deterministic, and
// levels are separated by kernel boundaries only.
// With per-particle softening lengths (seps non-null) every node also gets
// the largest and smallest length of its particles (semax, semin).
__global__ __launch_bounds__(kThreads) void k_leaves_and_buckets(
    const BoxDev *boxes, int B, const Topo *topo, const double4 *part64, float4 *part32, Mom64 *mom64,
    Mom32 *mom32, const uint32_t *scalars, uint32_t node_cap, const uint32_t *lvl_cnt, uint32_t *lvl_fill,
    uint32_t *lvl_nodes, const double *seps, double *semax, double *semin) {
  __shared__ uint32_t base[kLevels + 1], lcount[kLevels + 1], lres[kLevels + 1];
  // the round's leaf particles, loaded coalesced (a leaf's thread would
  // otherwise read its particles with a stride of a leaf between lanes)
  __shared__ double4 stage[kLeafStage];
  __shared__ uint32_t prange[2];
  if (threadIdx.x <= kLevels) {
    uint32_t o = 0;
    for (int l = 0; l < (int)threadIdx.x; ++l) o += lvl_cnt[l];
    base[threadIdx.x] = o;
  }
  const uint32_t tot = min(scalars[3], node_cap);
  const uint32_t stride = gridDim.x * kThreads;
  // round-based so that each block reserves bucket slots once per round
  for (uint32_t r0 = blockIdx.x * kThreads; r0 < tot; r0 += stride) {
    const uint32_t r = r0 + threadIdx.x;
    if (threadIdx.x <= kLevels) lcount[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
      prange[0] = 0xffffffffu;
      prange[1] = 0u;
    }
    __syncthreads();
    Topo t{};
    const bool is_leaf = r < tot && ((t = topo[r]).corner & kLeafBit) != 0;
    if (is_leaf) {
      atomicMin(&prange[0], t.a);
      atomicMax(&prange[1], t.a + (t.b & kCountMask));
    }
    __syncthreads();
    const uint32_t pa = prange[0], pn = prange[1] > pa ? prange[1] - pa : 0u;
    const bool staged = pn <= (uint32_t)kLeafStage;
    if (staged)
      for (uint32_t i = threadIdx.x; i < pn; i += kThreads) stage[i] = part64[pa + i];
    __syncthreads();
    int lvl = -1;
    uint32_t slot = 0;
    if (r < tot) {
      if (is_leaf) {
        const uint32_t f = t.a, cnt = t.b & kCountMask;
        const BoxDev &bx = boxes[box_of(boxes, B, f)];
        double c[3];
        node_centre(bx, t.corner, (int)(t.b >> kCountBits), c);
        double M = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (uint32_t j = f; j < f + cnt; ++j) {
          const double4 q = staged ? stage[j - pa] : part64[j];
          const double dx = q.x - c[0], dy = q.y - c[1], dz = q.z - c[2];
          M += q.w;
          s0 += q.w * dx;
          s1 += q.w * dy;
          s2 += q.w * dz;
          part32[j] = make_float4((float)dx, (float)dy, (float)dz, (float)q.w);
        }
        const double com[3] = {c[0] + s0 / M, c[1] + s1 / M, c[2] + s2 / M};
        mom64[r] = Mom64{com[0], com[1], com[2], M};
        mom32[r] = Mom32{(float)(com[0] - c[0]), (float)(com[1] - c[1]), (float)(com[2] - c[2]), (float)M};
        if (seps) {
          double hi = seps[f], lo = hi;
          for (uint32_t j = f + 1; j < f + cnt; ++j) {
            hi = seps[j] > hi ? seps[j] : hi;
            lo = seps[j] < lo ? seps[j] : lo;
          }
          semax[r] = hi;
          semin[r] = lo;
        }
      } else {
        lvl = (int)(t.b >> kCountBits);
        slot = atomicAdd(&lcount[lvl], 1u);
      }
    }
    __syncthreads();
    if (threadIdx.x <= kLevels && lcount[threadIdx.x])
      lres[threadIdx.x] = atomicAdd(&lvl_fill[threadIdx.x], lcount[threadIdx.x]);
    __syncthreads();
    if (lvl >= 0) lvl_nodes[base[lvl] + lres[lvl] + slot] = r;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void k_moments_level(const BoxDev *boxes, int B, int level,
                                                            const Topo *topo, const uint32_t *first,
                                                            const uint32_t *skip, const uint32_t *lvl_cnt,
                                                            const uint32_t *lvl_nodes, const uint32_t *scalars,
                                                            uint32_t node_cap, Mom64 *mom64, Mom32 *mom32,
                                                            double *semax, double *semin) {
  uint32_t o = 0;
  for (int l = 0; l < level; ++l) o += lvl_cnt[l];
  const uint32_t cnt = lvl_cnt[level];
  const uint32_t tot = min(scalars[3], node_cap);
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < cnt; i += gridDim.x * kThreads) {
    const uint32_t par = lvl_nodes[o + i];
    const Topo tp = topo[par];
    const BoxDev &bx = boxes[box_of(boxes, B, first[par])];
    double cp[3];
    node_centre(bx, tp.corner, level, cp);
    double Mp = 0.0, q0 = 0.0, q1 = 0.0, q2 = 0.0;
    double hi = 0.0, lo = INFINITY;
    const uint32_t pend = min(tp.a, tot);
    for (uint32_t ch = par + 1; ch < pend;) {
      const Mom64 m = mom64[ch];
      Mp += m.m;
      q0 += m.m * (m.cx - cp[0]);
      q1 += m.m * (m.cy - cp[1]);
      q2 += m.m * (m.cz - cp[2]);
      if (semax) {
        hi = semax[ch] > hi ? semax[ch] : hi;
        lo = semin[ch] < lo ? semin[ch] : lo;
      }
      const uint32_t nx = skip[ch];
      if (nx <= ch) break;  // never taken for a well-formed tree
      ch = nx;
    }
    const double cm[3] = {cp[0] + q0 / Mp, cp[1] + q1 / Mp, cp[2] + q2 / Mp};
    mom64[par] = Mom64{cm[0], cm[1], cm[2], Mp};
    mom32[par] = Mom32{(float)(cm[0] - cp[0]), (float)(cm[1] - cp[1]), (float)(cm[2] - cp[2]), (float)Mp};
    if (semax) {
      semax[par] = hi;
      semin[par] = lo;
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

// Walk records for the mixed-precision walk (see WNode).
__global__ __launch_bounds__(kThreads) void k_wnodes(const BoxDev *boxes, int B, const Topo *topo,
                                                     const Mom32 *mom32, const uint32_t *first,
                                                     const uint32_t *scalars, uint32_t node_cap, WNode *wn,
                                                     double4 *cen64) {
  const uint32_t tot = min(scalars[3], node_cap);
  for (uint32_t r = blockIdx.x * kThreads + threadIdx.x; r < tot; r += gridDim.x * kThreads) {
    const Topo t = topo[r];
    const Mom32 m = mom32[r];
    const BoxDev &bx = boxes[box_of(boxes, B, first[r])];
    const int lev = (int)(t.b >> kCountBits);
    const int hc = 1 << (kLevels - lev);
    const bool leaf = (t.corner & kLeafBit) != 0;
    const float side = ldexpf(bx.Lf, -lev);
    WNode w;
    w.c[0] = 0x4B000000 | (2 * (int)(t.corner & 0x1fffffull) + hc);
    w.c[1] = 0x4B000000 | (2 * (int)((t.corner >> 21) & 0x1fffffull) + hc);
    w.c[2] = 0x4B000000 | (2 * (int)((t.corner >> 42) & 0x1fffffull) + hc);
    w.side2 = side * side;
    w.o[0] = m.ox;
    w.o[1] = m.oy;
    w.o[2] = m.oz;
    w.m = m.m;
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
// Status word cleared, particle count for the device-side scans, level
// counters of the moment buckets cleared.
__global__ void k_init_scalars(uint32_t *sc, uint32_t n, uint32_t *lvl_cnt, uint32_t *lvl_fill) {
  if (threadIdx.x == 0) {
    sc[0] = 0u;
    sc[4] = n;
  }
  if (threadIdx.x <= kLevels) {
    lvl_cnt[threadIdx.x] = 0;
    lvl_fill[threadIdx.x] = 0;
  }
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
  k_init_scalars<<<1, 64, 0, s>>>(A.scalars, n, A.lvl_cnt, A.lvl_fill);
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
    k_links<<<gnodes, kThreads, 0, s>>>(A.topo, A.skip, A.scalars, A.node_cap, A.parent, A.nchild, A.lvl_cnt);
  }
  {
    const TraceRange r("build: moments");
    k_leaves_and_buckets<<<gnodes, kThreads, 0, s>>>(A.boxes, A.B, A.topo, A.part64, A.part32, A.mom64,
                                                     A.mom32, A.scalars, A.node_cap, A.lvl_cnt, A.lvl_fill,
                                                     A.lvl_nodes, A.seps, A.semax, A.semin);
    // internal nodes at level L number at most n / (leaf_max + 1) <= n / 2; most
    // levels hold few, so a small grid (grid-stride) keeps the launches short
    const uint32_t glev = std::max<uint32_t>(1, std::min<uint32_t>(cdiv(n / 2 + 1, kThreads), 512));
    for (int L = kLevels - 1; L >= 0; --L)
      k_moments_level<<<glev, kThreads, 0, s>>>(A.boxes, A.B, L, A.topo, A.first, A.skip, A.lvl_cnt,
                                                A.lvl_nodes, A.scalars, A.node_cap, A.mom64, A.mom32, A.semax,
                                                A.semin);
  }
  const TraceRange r("build: walk records");
  k_wnodes<<<gnodes, kThreads, 0, s>>>(A.boxes, A.B, A.topo, A.mom32, A.first, A.scalars, A.node_cap,
                                       A.wnode, A.cen64);
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
