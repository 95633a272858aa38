// Particle-mesh long-range force for CDNA4 (gfx950).
//
// Paper, "Particle Mesh": the particles' mass is assigned to a periodic
// mesh, the density is Fourier transformed, multiplied by the Green's
// function of the Poisson equation with the Gaussian filter
// exp(-k^2 A_smth^2), and transformed back; the tree carries the erfc part
// of the split, the mesh the erf part.
//
// Layout: an n^3 mesh of complex FP64 values (double2), index (x*n + y)*n + z.
//   1. deposit: cloud-in-cell weights onto the nodes j*L/n, summed in
//      64-bit fixed point (a power-of-two scale fitted to N * max m), so
//      the mesh does not depend on the order of the additions.  Caller
//      order: atomics onto the mesh.  A tree's curve order: one workgroup
//      per block of 8^3 cells sums its particles in LDS and stores its
//      nodes (plus a halo for the blocks above);
//   2. forward 3-D FFT of the density: length-n transforms along z (the
//      pass that reads the fixed-point sums), y and x; each workgroup
//      transforms a tile of neighbouring lines in LDS, so every pass reads
//      and writes whole cache lines;
//   3. per wave vector, in the x pass: phi_k = -4 pi G exp(-k^2 r_s^2) /
//      k^2 / W(k)^2 rho_k, W the CIC window, and a_k = -i k phi_k; two
//      inverse transforms carry (a_x + i a_y) and (a_z + i phi), each a
//      pair of real fields, and their x passes run in the same workgroup;
//   4. the inverse y and z passes, then CIC interpolation at the particles.
#include <climits>
#include <cmath>
#include <cstdlib>

#include "og_internal.h"
#include "og_pm.h"

namespace og {

namespace {

constexpr int kPmThreads = 256;
constexpr int kFftThreads = 256;

__device__ inline void cic(double x, int n, double inv_d, int &i0, double &f) {
  const double u = x * inv_d;
  const double fl = floor(u);
  f = u - fl;
  // periodic wrap; n is a power of two, so two's complement masking is the
  // non-negative remainder
  i0 = (int)((long long)fl & (long long)(n - 1));
}

__global__ __launch_bounds__(kPmThreads) void k_fill_u64(unsigned long long *p, uint64_t count) {
  for (uint64_t i = blockIdx.x * (uint64_t)kPmThreads + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * kPmThreads)
    p[i] = 0ull;
}

// Particle i: caller arrays, or a tree's particles in curve order.
struct PartRef {
  const double *pos, *mass;
  const double4 *part;
  __device__ inline double4 get(uint32_t i) const {
    if (part) return part[i];
    return make_double4(pos[3ull * i], pos[3ull * i + 1], pos[3ull * i + 2], mass[i]);
  }
};

// Largest mass (positive doubles order like their bit patterns).
__global__ __launch_bounds__(kPmThreads) void k_mass_max(PartRef P, uint32_t N, unsigned long long *mmax) {
  __shared__ unsigned long long red[kPmThreads / 64];
  unsigned long long v = 0ull;
  for (uint32_t i = blockIdx.x * kPmThreads + threadIdx.x; i < N; i += gridDim.x * kPmThreads) {
    const double m = P.part ? P.part[i].w : P.mass[i];
    const unsigned long long b = m > 0.0 ? (unsigned long long)__double_as_longlong(m) : 0ull;
    v = b > v ? b : v;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kPmThreads / 64; ++w) v = red[w] > v ? red[w] : v;
    atomicMax(mmax, v);
  }
}

// Fixed-point scale: 2^(62 - e) with N * max m < 2^e, so no node overflows.
__device__ inline double fixed_scale(const unsigned long long *mmax, uint32_t N) {
  const double m = __longlong_as_double((long long)*mmax);
  int e = 0;
  frexp((double)N * m, &e);
  return ldexp(1.0, 62 - e);
}

__global__ __launch_bounds__(kPmThreads) void k_deposit(PartRef P, uint32_t N, int n, double inv_d,
                                                        const unsigned long long *mmax,
                                                        unsigned long long *acc_mesh) {
  const uint32_t i = blockIdx.x * kPmThreads + threadIdx.x;
  if (i >= N) return;
  const double scale = fixed_scale(mmax, N);
  const double4 q = P.get(i);
  int ix, iy, iz;
  double fx, fy, fz;
  cic(q.x, n, inv_d, ix, fx);
  cic(q.y, n, inv_d, iy, fy);
  cic(q.z, n, inv_d, iz, fz);
  const double m = q.w * scale;
  const int jx[2] = {ix, ix + 1 == n ? 0 : ix + 1};
  const int jy[2] = {iy, iy + 1 == n ? 0 : iy + 1};
  const int jz[2] = {iz, iz + 1 == n ? 0 : iz + 1};
  const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const unsigned long long q = (unsigned long long)llrint(m * wx[a] * wy[b] * wz[c]);
        atomicAdd(acc_mesh + ((uint64_t)jx[a] * n + jy[b]) * n + jz[c], q);
      }
}

// Deposit of particles in curve order: the 256 particles of a workgroup
// are neighbours in space, so their 8 x 256 node weights are first summed in
// an LDS tile spanning the workgroup's box of nodes, then the tile is added
// to the mesh (one global atomic per touched node).  Integer sums: the
// result is the same as adding every weight to the mesh directly, which is
// what a workgroup whose box exceeds the tile (straddling the periodic edge,
// or spread out) does.
constexpr int kDepositTile = 4096;  // nodes (32 KB)

// ------------------------------------------------------ mesh blocks --
// Tree order (a periodic tree whose root cube is the mesh box, n = 2^k):
// the mesh cell of a particle is the top k bits of its level-21 tree cell,
// so the particles of a block of 8^3 cells (a cube of the tree at level
// k - 3) are one contiguous run of the sorted keys, starting at
// bstart[h] for the block whose key prefix is h.  A block's particles
// touch the 9^3 nodes lo .. lo + 8 of each axis: its own 8^3 (which no
// other block's interior holds) and 217 halo nodes shared with the blocks
// above it.
constexpr int kBlk = 8;                                        // cells per block edge
constexpr int kTile = kBlk + 1;                                // nodes per tile edge
constexpr int kTile3 = kTile * kTile * kTile;                  // 729
constexpr int kHalo = kTile3 - kBlk * kBlk * kBlk;             // 217
constexpr uint32_t kBlockChunk = 2048;  // particles a block's own workgroup takes

// Workgroups are dealt to the 8 XCDs in turn (g % 8), each XCD with its
// own L2.  Giving XCD j the j-th contiguous share of the work units keeps
// neighbouring units (which share mesh nodes) in one L2.  A bijection of
// [0, G) for any G.
constexpr uint32_t kXcds = 8;
__device__ inline uint32_t xcd_unit(uint32_t g, uint32_t G) {
  const uint32_t q = G / kXcds, r = G % kXcds, j = g % kXcds, i = g / kXcds;
  return j * q + min(j, r) + i;
}

struct BlockRef {
  const uint64_t *keys;
  const uint32_t *bstart;
  int shift3;   // key bits below the block prefix: 3 (21 - (k - 3))
  int curve;
  double tscale;  // 2^21 / L, the tree's cell scale
};

// A particle beyond the first kBlockChunk of its block (handled by the
// per-particle kernels).
__device__ inline bool block_extra(const BlockRef &R, uint32_t i) {
  return i - R.bstart[(uint32_t)(R.keys[i] >> R.shift3)] >= kBlockChunk;
}

__global__ __launch_bounds__(kPmThreads) void k_block_starts(BlockRef R, uint32_t N, uint32_t nblocks,
                                                             uint32_t *bstart) {
  const uint32_t h = blockIdx.x * kPmThreads + threadIdx.x;
  if (h > nblocks) return;
  uint32_t lo = 0, hi = N;  // first particle whose prefix is >= h
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if ((R.keys[mid] >> R.shift3) < (uint64_t)h) lo = mid + 1;
    else hi = mid;
  }
  bstart[h] = lo;
}

// Lower mesh corner (in cells) of block h: the cell of its first key.
__device__ inline void block_corner(const BlockRef &R, uint32_t h, int logn, int g0[3]) {
  uint32_t c[3];
  key_cell((uint64_t)h << R.shift3, R.curve, c);
  const int sh = kLevels - logn + 3;
  for (int k = 0; k < 3; ++k) g0[k] = (int)(c[k] >> sh) * kBlk;
}

// A particle's CIC node offsets inside its block's tile (0..7) and
// fractions.  The cell is the tree's (the key was formed from it); the
// fraction is x n / L minus that cell, as cic() forms it (the two differ
// only where x n / L rounds up to n, where both put the whole weight on
// node n = node 0).
__device__ inline void tile_cic(const double4 &q, const BlockRef &R, int logn, double inv_d, const int g0[3],
                                int r[3], double f[3]) {
  const double xs[3] = {q.x, q.y, q.z};
  const int sh = kLevels - logn;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double v = xs[k] * R.tscale;
    const uint32_t cell = !(v >= 0.0) ? 0u : (v >= 2097151.0 ? 2097151u : (uint32_t)v);
    const int ix = (int)(cell >> sh);
    r[k] = min(max(ix - g0[k], 0), kBlk - 1);
    f[k] = xs[k] * inv_d - (double)ix;
  }
}

__device__ inline int halo_index(int tx, int ty, int tz) {
  // faces x = 8 (9 x 9), y = 8 (8 x 9), z = 8 (8 x 8)
  return tx == kBlk ? ty * kTile + tz : (ty == kBlk ? 81 + tx * kTile + tz : 153 + tx * kBlk + ty);
}

// One workgroup per block: the block's first kBlockChunk particles summed
// in an LDS tile, then its 8^3 own nodes stored to the mesh (every node of
// the mesh is some block's own node, so the mesh needs no clearing) and
// its halo to halo[block] (added by k_density_blocks).
__global__ __launch_bounds__(kPmThreads) void k_deposit_blocks(const double4 *part, BlockRef R, uint32_t N, int n,
                                                               int logn, double inv_d,
                                                               const unsigned long long *mmax,
                                                               unsigned long long *mesh,
                                                               unsigned long long *halo) {
  __shared__ unsigned long long tile[kTile3];
  const uint32_t h = xcd_unit(blockIdx.x, gridDim.x);
  const uint32_t s = R.bstart[h], e = min(R.bstart[h + 1], s + kBlockChunk);
  int g0[3];
  block_corner(R, h, logn, g0);
  for (int c = threadIdx.x; c < kTile3; c += kPmThreads) tile[c] = 0ull;
  __syncthreads();
  const double scale = fixed_scale(mmax, N);
  for (uint32_t p = s + threadIdx.x; p < e; p += kPmThreads) {
    const double4 q = part[p];
    int r[3];
    double f[3];
    tile_cic(q, R, logn, inv_d, g0, r, f);
    const double m = q.w * scale;
    const double w[3][2] = {{1.0 - f[0], f[0]}, {1.0 - f[1], f[1]}, {1.0 - f[2], f[2]}};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const unsigned long long qv = (unsigned long long)llrint(m * w[0][a] * w[1][b] * w[2][c]);
          atomicAdd(&tile[((r[0] + a) * kTile + r[1] + b) * kTile + r[2] + c], qv);
        }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < kBlk * kBlk * kBlk; c += kPmThreads) {
    const int lx = c >> 6, ly = (c >> 3) & 7, lz = c & 7;
    mesh[((uint64_t)(g0[0] + lx) * n + (g0[1] + ly)) * n + (g0[2] + lz)] = tile[(lx * kTile + ly) * kTile + lz];
  }
  const uint32_t nb = (uint32_t)n / kBlk;
  unsigned long long *hb =
      halo + (((uint64_t)(g0[0] / kBlk) * nb + (uint32_t)(g0[1] / kBlk)) * nb + (uint32_t)(g0[2] / kBlk)) * kHalo;
  for (int c = threadIdx.x; c < kHalo; c += kPmThreads) {
    int tx, ty, tz;
    if (c < 81) {
      tx = kBlk;
      ty = c / kTile;
      tz = c % kTile;
    } else if (c < 153) {
      tx = (c - 81) / kTile;
      ty = kBlk;
      tz = (c - 81) % kTile;
    } else {
      tx = (c - 153) / kBlk;
      ty = (c - 153) % kBlk;
      tz = kBlk;
    }
    hb[c] = tile[(tx * kTile + ty) * kTile + tz];
  }
}

// A node's fixed-point sum: the mesh entry plus, with block halos, the
// halo entries of the blocks below it that touch it (up to 7, for a block
// corner).  Unsigned sums: the same value as any other order of adding the
// same weights.
__device__ inline unsigned long long node_sum(const unsigned long long *mesh, const unsigned long long *halo,
                                              uint64_t i, int gx, int gy, int gz, int n) {
  unsigned long long v = mesh[i];
  if (halo == nullptr) return v;
  const int lx = gx & (kBlk - 1), ly = gy & (kBlk - 1), lz = gz & (kBlk - 1);
  const int nb = n / kBlk, bm = nb - 1;
  const int bx = gx / kBlk, by = gy / kBlk, bz = gz / kBlk;
  // the block (bx - dx, by - dy, bz - dz) holds this node as tile node
  // (lx + 8 dx, ly + 8 dy, lz + 8 dz) when every shifted axis has l = 0
  auto from = [&](int dx, int dy, int dz) {
    const uint64_t blk = ((uint64_t)((bx - dx) & bm) * nb + ((by - dy) & bm)) * nb + ((bz - dz) & bm);
    return halo[blk * kHalo + halo_index(lx + kBlk * dx, ly + kBlk * dy, lz + kBlk * dz)];
  };
  if (lz == 0) v += from(0, 0, 1);
  if (ly == 0) {
    v += from(0, 1, 0);
    if (lz == 0) v += from(0, 1, 1);
  }
  if (lx == 0) {
    v += from(1, 0, 0);
    if (lz == 0) v += from(1, 0, 1);
    if (ly == 0) {
      v += from(1, 1, 0);
      if (lz == 0) v += from(1, 1, 1);
    }
  }
  return v;
}

__global__ __launch_bounds__(kPmThreads) void k_deposit_tiled(PartRef P, uint32_t N, int n, double inv_d,
                                                              const unsigned long long *mmax,
                                                              unsigned long long *acc_mesh, BlockRef R) {
  __shared__ unsigned long long tile[kDepositTile];
  __shared__ int red[6][kPmThreads / 64];
  const uint32_t i = xcd_unit(blockIdx.x, gridDim.x) * kPmThreads + threadIdx.x;
  // with block starts: only the particles the block workgroups left
  const bool ok = i < N && (R.bstart == nullptr || block_extra(R, i));
  if (R.bstart != nullptr && __syncthreads_or(ok) == 0) return;
  const double scale = fixed_scale(mmax, N);
  int ix = 0, iy = 0, iz = 0;
  double fx = 0.0, fy = 0.0, fz = 0.0, m = 0.0;
  if (ok) {
    const double4 q = P.get(i);
    cic(q.x, n, inv_d, ix, fx);
    cic(q.y, n, inv_d, iy, fy);
    cic(q.z, n, inv_d, iz, fz);
    m = q.w * scale;
  }
  // the workgroup's box of lower nodes (the upper node is +1, unwrapped)
  int v[6] = {ok ? ix : INT_MAX, ok ? iy : INT_MAX, ok ? iz : INT_MAX,
              ok ? ix : INT_MIN, ok ? iy : INT_MIN, ok ? iz : INT_MIN};
  for (int off = 32; off > 0; off >>= 1)
    for (int a = 0; a < 6; ++a) {
      const int o = __shfl_xor(v[a], off, 64);
      v[a] = a < 3 ? min(v[a], o) : max(v[a], o);
    }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int a = 0; a < 6; ++a) red[a][wv] = v[a];
  __syncthreads();
  int lo[3], ext[3];
  for (int a = 0; a < 3; ++a) {
    int l = red[a][0], h = red[a + 3][0];
    for (int w = 1; w < kPmThreads / 64; ++w) {
      l = min(l, red[a][w]);
      h = max(h, red[a + 3][w]);
    }
    lo[a] = l;
    ext[a] = h - l + 2;  // nodes lo .. h + 1
  }
  const long long vol = (long long)ext[0] * ext[1] * ext[2];
  const int wx[2] = {0, 1};
  const double wgt[3][2] = {{1.0 - fx, fx}, {1.0 - fy, fy}, {1.0 - fz, fz}};
  if (vol <= kDepositTile) {
    for (int c = threadIdx.x; c < (int)vol; c += kPmThreads) tile[c] = 0ull;
    __syncthreads();
    if (ok) {
      const int rx = ix - lo[0], ry = iy - lo[1], rz = iz - lo[2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const unsigned long long qv = (unsigned long long)llrint(m * wgt[0][a] * wgt[1][b] * wgt[2][c]);
            atomicAdd(&tile[((rx + wx[a]) * ext[1] + ry + wx[b]) * ext[2] + rz + wx[c]], qv);
          }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < (int)vol; c += kPmThreads) {
      const unsigned long long qv = tile[c];
      if (!qv) continue;
      const int cz = c % ext[2], cy = (c / ext[2]) % ext[1], cx = c / (ext[2] * ext[1]);
      int gx = lo[0] + cx, gy = lo[1] + cy, gz = lo[2] + cz;
      gx = gx >= n ? gx - n : gx;
      gy = gy >= n ? gy - n : gy;
      gz = gz >= n ? gz - n : gz;
      atomicAdd(acc_mesh + ((uint64_t)gx * n + gy) * n + gz, qv);
    }
  } else if (ok) {
    const int jx[2] = {ix, ix + 1 == n ? 0 : ix + 1};
    const int jy[2] = {iy, iy + 1 == n ? 0 : iy + 1};
    const int jz[2] = {iz, iz + 1 == n ? 0 : iz + 1};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const unsigned long long qv = (unsigned long long)llrint(m * wgt[0][a] * wgt[1][b] * wgt[2][c]);
          atomicAdd(acc_mesh + ((uint64_t)jx[a] * n + jy[b]) * n + jz[c], qv);
        }
  }
}

// ----------------------------------------------------------------- FFT --
// Length-n transforms along one axis, radix 2, decimation in time (input in
// bit-reversed order).  kSign = -1: forward e^{-2 pi i jk/n}; +1: inverse
// without the 1/n.  A workgroup transforms a tile of `tl` lines.  Axis 2
// (z, contiguous): `tl` consecutive lines; axes 1 and 0: `tl` lines with
// consecutive z, so element j of the tile is `tl` contiguous values, and
// the neighbouring tiles (the rest of those cache lines) go to the same
// XCD (xcd_unit), so that a line fetched for one tile serves the next.
struct LineTile {
  int n, logn, axis, tl;
  uint32_t g, a, z0;
  __device__ LineTile(int n_, int logn_, int axis_, int tl_, uint32_t g_) : n(n_), logn(logn_), axis(axis_), tl(tl_), g(g_) {
    const uint32_t per = (uint32_t)(n / tl);
    a = g / per;
    z0 = (g % per) * tl;
  }
  // tile element idx -> line t, position j along the line
  __device__ void split(int idx, int &t, int &j) const {
    if (axis == 2) {
      t = idx >> logn;
      j = idx & (n - 1);
    } else {
      t = idx % tl;
      j = idx / tl;
    }
  }
  __device__ uint64_t addr(int t, int j) const {
    const uint64_t nn = (uint64_t)n;
    if (axis == 2) return ((uint64_t)g * tl + t) * nn + j;
    if (axis == 1) return ((uint64_t)a * nn + j) * nn + z0 + t;
    return ((uint64_t)j * nn + a) * nn + z0 + t;
  }
  // mesh coordinates of element (t, j)
  __device__ void coords(int t, int j, int &x, int &y, int &z) const {
    if (axis == 2) {
      const uint32_t line = g * tl + t;
      x = (int)(line >> logn);
      y = (int)(line & (n - 1));
      z = j;
    } else if (axis == 1) {
      x = (int)a;
      y = j;
      z = (int)z0 + t;
    } else {
      x = j;
      y = (int)a;
      z = (int)z0 + t;
    }
  }
};

__device__ inline int brev(int j, int logn) { return (int)(__brev((uint32_t)j) >> (32 - logn)); }

// LDS position of tile element i: one 16-byte pad after every 16 elements,
// so that the bit-reversed scatter of the loads and the short-stride
// butterflies of the first stages fall into different banks.
__host__ __device__ inline int lp(int i) { return i + (i >> 4); }
// LDS elements of a padded tile of m elements.
__host__ __device__ inline int lp_size(int m) { return lp(m - 1) + 1; }

// Tables of one mesh, computed once per force call (k_pm_tables) and
// copied into LDS by each workgroup: forward twiddles e^{-2 pi i k / n} and
// inverse twiddles e^{+2 pi i k / n}, k < n/2, and per axis index j (signed
// wave number m) the factor exp(-(2 pi m / L)^2 r_s^2) / sinc(pi m / n)^4:
// the Gaussian filter exp(-k^2 r_s^2) and the CIC deconvolution 1 / W(k)^2
// are both products over the three axes.
struct PmTables {
  double2 *twf, *twi;
  double *wax;
};

__device__ inline double sinc(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

__global__ __launch_bounds__(kPmThreads) void k_pm_tables(PmTables Tb, int n, double L, double r_s) {
  const int k = blockIdx.x * kPmThreads + threadIdx.x;
  if (k < n / 2) {
    double sn, cs;
    sincospi(2.0 * k / n, &sn, &cs);
    Tb.twf[k] = make_double2(cs, -sn);
    Tb.twi[k] = make_double2(cs, sn);
  }
  if (k < n) {
    const int m = k < n / 2 ? k : k - n;
    const double sj = sinc(M_PI * m / n), s2 = sj * sj;
    const double km = 2.0 * M_PI / L * m;
    Tb.wax[k] = exp(-(km * r_s) * (km * r_s)) / (s2 * s2);
  }
}

template <int kT = kFftThreads, typename T>
__device__ inline void copy_to_lds(T *dst, const T *src, int count) {
  for (int k = threadIdx.x; k < count; k += kT) dst[k] = src[k];
}

// The radix-2 stages of `total / n` lines held in LDS (bit-reversed input,
// natural-order output).  Callers synchronise before and after.
// kConj: `tw` holds the opposite sign's twiddles (e^{-sign ...}), used
// conjugated.
template <int kSign, bool kConj = false>
__device__ inline void fft_stages(double2 *buf, const double2 *tw, int n, int logn, int total) {
  // complex products as fused multiply-adds (deterministic, and one
  // rounding fewer per product)
#pragma clang fp contract(fast)
  const int tid = threadIdx.x;
  int s = 1;
  if (logn & 1) {
    // one radix-2 stage (len 2, twiddle 1) when log2 n is odd
    for (int b = tid; b < total / 2; b += kFftThreads) {
      const int i0 = 2 * b;
      const double2 u = buf[lp(i0)], v = buf[lp(i0 + 1)];
      buf[lp(i0)] = make_double2(u.x + v.x, u.y + v.y);
      buf[lp(i0 + 1)] = make_double2(u.x - v.x, u.y - v.y);
    }
    __syncthreads();
    s = 2;
  }
  // two radix-2 stages (s and s + 1) per pass over the LDS lines: each
  // thread takes the four elements i0 + {0, h, 2h, 3h} of one group of 4h
  for (; s < logn; s += 2) {
    const int h = 1 << (s - 1), step1 = n >> s, step2 = n >> (s + 1);
    for (int b = tid; b < total / 4; b += kFftThreads) {
      const int t = b >> (logn - 2), r = b & (n / 4 - 1);
      const int pos = r & (h - 1), grp = r >> (s - 1);
      const int i0 = t * n + grp * 4 * h + pos;
      double2 w1 = tw[pos * step1], w2 = tw[pos * step2];
      if (kConj) {
        w1.y = -w1.y;
        w2.y = -w2.y;
      }
      // the second stage's twiddle for the odd pair is w2 exp(sign i pi/2)
      const double2 w3 = make_double2(-kSign * w2.y, kSign * w2.x);
      const double2 a = buf[lp(i0)], b0 = buf[lp(i0 + h)], c = buf[lp(i0 + 2 * h)], d0 = buf[lp(i0 + 3 * h)];
      const double2 vb = make_double2(b0.x * w1.x - b0.y * w1.y, b0.x * w1.y + b0.y * w1.x);
      const double2 vd = make_double2(d0.x * w1.x - d0.y * w1.y, d0.x * w1.y + d0.y * w1.x);
      const double2 a1 = make_double2(a.x + vb.x, a.y + vb.y), b1 = make_double2(a.x - vb.x, a.y - vb.y);
      const double2 c1 = make_double2(c.x + vd.x, c.y + vd.y), d1 = make_double2(c.x - vd.x, c.y - vd.y);
      const double2 vc = make_double2(c1.x * w2.x - c1.y * w2.y, c1.x * w2.y + c1.y * w2.x);
      const double2 ve = make_double2(d1.x * w3.x - d1.y * w3.y, d1.x * w3.y + d1.y * w3.x);
      buf[lp(i0)] = make_double2(a1.x + vc.x, a1.y + vc.y);
      buf[lp(i0 + 2 * h)] = make_double2(a1.x - vc.x, a1.y - vc.y);
      buf[lp(i0 + h)] = make_double2(b1.x + ve.x, b1.y + ve.y);
      buf[lp(i0 + 3 * h)] = make_double2(b1.x - ve.x, b1.y - ve.y);
    }
    __syncthreads();
  }
}

template <int kSign>
__global__ __launch_bounds__(kFftThreads) void k_fft_axis(double2 *data, const double2 *twg, int n, int logn, int axis,
                                                          int tl) {
  extern __shared__ double2 sm[];
  double2 *buf = sm;
  double2 *tw = sm + lp_size(tl * n);
  copy_to_lds(tw, twg, n / 2);
  const LineTile T(n, logn, axis, tl, xcd_unit(blockIdx.x, gridDim.x));
  const int total = tl * n;
  for (int idx = threadIdx.x; idx < total; idx += kFftThreads) {
    int t, j;
    T.split(idx, t, j);
    buf[lp(t * n + brev(j, logn))] = data[T.addr(t, j)];
  }
  __syncthreads();
  fft_stages<kSign>(buf, tw, n, logn, total);
  for (int idx = threadIdx.x; idx < total; idx += kFftThreads) {
    int t, j;
    T.split(idx, t, j);
    data[T.addr(t, j)] = buf[lp(t * n + j)];
  }
}

// The forward z pass of the density: each node's fixed-point sum (with the
// block halos, when given) becomes mass / cell volume, the real part of the
// input, as it is read.
__global__ __launch_bounds__(kFftThreads) void k_fft_z_density(const unsigned long long *mesh,
                                                               const unsigned long long *halo, uint32_t N,
                                                               const unsigned long long *mmax, double inv_vol,
                                                               const double2 *twg, double2 *rho, int n, int logn,
                                                               int tl) {
  extern __shared__ double2 sm[];
  double2 *buf = sm;
  double2 *tw = sm + lp_size(tl * n);
  copy_to_lds(tw, twg, n / 2);
  const double f = inv_vol / fixed_scale(mmax, N);
  const LineTile T(n, logn, 2, tl, xcd_unit(blockIdx.x, gridDim.x));
  const int total = tl * n;
  for (int idx = threadIdx.x; idx < total; idx += kFftThreads) {
    int t, j, x, y, z;
    T.split(idx, t, j);
    T.coords(t, j, x, y, z);
    const unsigned long long v = node_sum(mesh, halo, T.addr(t, j), x, y, z, n);
    buf[lp(t * n + brev(j, logn))] = make_double2((double)v * f, 0.0);
  }
  __syncthreads();
  fft_stages<-1>(buf, tw, n, logn, total);
  for (int idx = threadIdx.x; idx < total; idx += kFftThreads) {
    int t, j;
    T.split(idx, t, j);
    rho[T.addr(t, j)] = buf[lp(t * n + j)];
  }
}

// Green's function, Gaussian filter, CIC deconvolution and gradient at wave
// vector (ix, iy, iz): phi_k = -4 pi G exp(-k^2 r_s^2) / k^2 / W(k)^2 rho_k
// and a_k = -i k phi_k; returns (a_x + i a_y)_k in *pa and (a_z + i phi)_k
// in *pb.  wax: the per-axis factors of the filter and the deconvolution.
__device__ inline void green(double2 rho, int ix, int iy, int iz, int n, double kf, double G, const double *wax,
                             double2 *pa, double2 *pb) {
  const int mx = ix < n / 2 ? ix : ix - n, my = iy < n / 2 ? iy : iy - n, mz = iz < n / 2 ? iz : iz - n;
  const double kx = kf * mx, ky = kf * my, kz = kf * mz;
  const double k2 = kx * kx + ky * ky + kz * kz;
  if (k2 == 0.0) {
    *pa = make_double2(0.0, 0.0);
    *pb = make_double2(0.0, 0.0);
    return;
  }
  const double g = -4.0 * M_PI * G / k2 * (wax[ix] * wax[iy] * wax[iz]);
  const double pr = g * rho.x, pi = g * rho.y;  // phi_k
  // derivative wavenumbers, the Nyquist one dropped
  const double dx = mx == -n / 2 ? 0.0 : kx, dy = my == -n / 2 ? 0.0 : ky, dz = mz == -n / 2 ? 0.0 : kz;
  // a_k = -i k phi_k = k (phi_i, -phi_r)
  const double axr = dx * pi, axi = -dx * pr;
  const double ayr = dy * pi, ayi = -dy * pr;
  const double azr = dz * pi, azi = -dz * pr;
  *pa = make_double2(axr - ayi, axi + ayr);
  *pb = make_double2(azr - pi, azi + pr);
}

// The forward x pass, Green's function and the inverse x passes of both
// output fields in one workgroup: B holds the y-z transformed density on
// entry; on exit A holds (a_x + i a_y) and B (a_z + i phi), transformed
// back along x.  The x lines stay in LDS between the steps; the spectrum,
// in natural order after the forward stages, goes back in bit-reversed
// order for the inverse stages through registers (each thread holds at
// most kXgPer tile elements: tl n <= kXgPer kFftThreads, as fft_lines
// picks for this kernel).
constexpr int kXgPer = 8;
__global__ __launch_bounds__(kFftThreads) void k_fft_x_green(double2 *B, double2 *A, PmTables Tb, int n, int logn,
                                                             int tl, double L, double G) {
  extern __shared__ double2 sm[];
  double2 *bb = sm;
  double2 *ba = sm + lp_size(tl * n);
  double2 *tw = ba + lp_size(tl * n);
  double *wax = reinterpret_cast<double *>(tw + n / 2);
  copy_to_lds(tw, Tb.twf, n / 2);
  copy_to_lds(wax, Tb.wax, n);
  const LineTile T(n, logn, 0, tl, xcd_unit(blockIdx.x, gridDim.x));
  const int total = tl * n;
  for (int idx = threadIdx.x; idx < total; idx += kFftThreads) {
    int t, j;
    T.split(idx, t, j);
    bb[lp(t * n + brev(j, logn))] = B[T.addr(t, j)];
  }
  __syncthreads();
  fft_stages<-1>(bb, tw, n, logn, total);
  const double kf = 2.0 * M_PI / L;
  {
    double2 oa[kXgPer], ob[kXgPer];
    int dst[kXgPer];
#pragma unroll
    for (int k = 0; k < kXgPer; ++k) {
      const int idx = threadIdx.x + k * kFftThreads;
      dst[k] = -1;
      if (idx < total) {
        int t, j, x, y, z;
        T.split(idx, t, j);
        T.coords(t, j, x, y, z);
        green(bb[lp(t * n + j)], x, y, z, n, kf, G, wax, &oa[k], &ob[k]);
        dst[k] = lp(t * n + brev(j, logn));
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kXgPer; ++k)
      if (dst[k] >= 0) {
        ba[dst[k]] = oa[k];
        bb[dst[k]] = ob[k];
      }
  }
  __syncthreads();
  fft_stages<1, true>(ba, tw, n, logn, total);
  fft_stages<1, true>(bb, tw, n, logn, total);
  for (int idx = threadIdx.x; idx < total; idx += kFftThreads) {
    int t, j;
    T.split(idx, t, j);
    const uint64_t k = T.addr(t, j);
    A[k] = ba[lp(t * n + j)];
    B[k] = bb[lp(t * n + j)];
  }
}

// ------------------------------------------ register-staged FFT (n >= 64) --
// The same radix-2 decimation-in-time transform, with its first three and
// last three stages done in registers.  A thread owns a column i < n/8 of a
// line: the elements i + k n/8, k = 0..7.  Loaded in that order, they are
// the eight bit-reversed-order inputs of the LDS group 8 brev(i) .. + 7, so
// the thread runs stages 1-3 on them (twiddles 1, +-i and (+-1 +- i)/sqrt 2)
// and writes the group contiguously; stages 4 .. log2 n - 3 run in LDS as
// before; and the last three stages combine exactly the elements i + k n/8
// again, which the thread reads, transforms and stores in natural order.
// No bit-reversed scatter, one LDS sweep at n = 256.  LDS holds one pad
// element per 8 (lq), which spreads the groups' contiguous writes over the
// banks.
__host__ __device__ inline int lq(int p) { return p + (p >> 3); }
__host__ __device__ inline int lq_size(int m) { return lq(m - 1) + 1; }

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cmul(double2 a, double2 w) {
#pragma clang fp contract(fast)
  return make_double2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}
// times e^{sign i pi / 2} = sign i
template <int kSign>
__device__ inline double2 mul_si(double2 a) { return make_double2(-kSign * a.y, kSign * a.x); }

// Stages 1-3 on one group of eight, in LDS order (u[r] = input brev3(r)).
template <int kSign>
__device__ inline void dft8_first(double2 u[8]) {
#pragma clang fp contract(fast)
  constexpr double c = 0.70710678118654752440;  // cos pi/4
#pragma unroll
  for (int p = 0; p < 8; p += 2) {
    const double2 a = u[p], b = u[p + 1];
    u[p] = cadd(a, b);
    u[p + 1] = csub(a, b);
  }
#pragma unroll
  for (int q = 0; q < 8; q += 4) {
    double2 a = u[q], b = u[q + 2];
    u[q] = cadd(a, b);
    u[q + 2] = csub(a, b);
    a = u[q + 1];
    b = mul_si<kSign>(u[q + 3]);
    u[q + 1] = cadd(a, b);
    u[q + 3] = csub(a, b);
  }
  const double2 x5 = u[5], x7 = u[7];
  const double2 b[4] = {u[4], make_double2(c * (x5.x - kSign * x5.y), c * (x5.y + kSign * x5.x)), mul_si<kSign>(u[6]),
                        make_double2(c * (-x7.x - kSign * x7.y), c * (kSign * x7.x - x7.y))};
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double2 a = u[r];
    u[r] = cadd(a, b[r]);
    u[r + 4] = csub(a, b[r]);
  }
}

// The last three stages on the elements i + k n/8 (natural order in e[k]
// on exit).  tw: e^{sign 2 pi i k / n} (kConj: the opposite sign's table,
// conjugated).
template <bool kConj>
__device__ inline double2 twid(const double2 *tw, int k) {
  double2 w = tw[k];
  if (kConj) w.y = -w.y;
  return w;
}
template <bool kConj>
__device__ inline void dft8_last(double2 e[8], int i, int n, const double2 *tw) {
  const double2 w = twid<kConj>(tw, 4 * i);
#pragma unroll
  for (int p = 0; p < 8; p += 2) {
    const double2 a = e[p], b = cmul(e[p + 1], w);
    e[p] = cadd(a, b);
    e[p + 1] = csub(a, b);
  }
  const double2 w0 = twid<kConj>(tw, 2 * i), w1 = twid<kConj>(tw, 2 * i + n / 4);
#pragma unroll
  for (int q = 0; q < 8; q += 4) {
    double2 a = e[q], b = cmul(e[q + 2], w0);
    e[q] = cadd(a, b);
    e[q + 2] = csub(a, b);
    a = e[q + 1];
    b = cmul(e[q + 3], w1);
    e[q + 1] = cadd(a, b);
    e[q + 3] = csub(a, b);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double2 a = e[k], b = cmul(e[k + 4], twid<kConj>(tw, i + k * (n / 8)));
    e[k] = cadd(a, b);
    e[k + 4] = csub(a, b);
  }
}

// Stages 4 .. log2 n - 3 of `total / n` lines in LDS (lq layout): one
// radix-2 stage first when their number is odd, then two stages per sweep.
// Callers synchronise before; every sweep ends with a barrier.
template <int kSign, bool kConj, int kT = kFftThreads>
__device__ inline void fft_middle(double2 *buf, const double2 *tw, int n, int logn, int total) {
#pragma clang fp contract(fast)
  const int tid = threadIdx.x;
  const int s_end = logn - 3;  // last middle stage
  int s = 4;
  if ((s_end - s + 1) & 1) {
    const int h = 1 << (s - 1), step = n >> s;
    for (int b = tid; b < total / 2; b += kT) {
      const int t = b >> (logn - 1), r = b & (n / 2 - 1);
      const int pos = r & (h - 1), grp = r >> (s - 1);
      const int i0 = t * n + grp * 2 * h + pos;
      const double2 a = buf[lq(i0)], v = cmul(buf[lq(i0 + h)], twid<kConj>(tw, pos * step));
      buf[lq(i0)] = cadd(a, v);
      buf[lq(i0 + h)] = csub(a, v);
    }
    __syncthreads();
    ++s;
  }
  for (; s < s_end; s += 2) {
    const int h = 1 << (s - 1), step1 = n >> s, step2 = n >> (s + 1);
    for (int b = tid; b < total / 4; b += kT) {
      const int t = b >> (logn - 2), r = b & (n / 4 - 1);
      const int pos = r & (h - 1), grp = r >> (s - 1);
      const int i0 = t * n + grp * 4 * h + pos;
      const double2 w1 = twid<kConj>(tw, pos * step1), w2 = twid<kConj>(tw, pos * step2);
      const double2 w3 = mul_si<kSign>(w2);
      const double2 a = buf[lq(i0)], b0 = buf[lq(i0 + h)], c = buf[lq(i0 + 2 * h)], d0 = buf[lq(i0 + 3 * h)];
      const double2 vb = cmul(b0, w1), vd = cmul(d0, w1);
      const double2 a1 = cadd(a, vb), b1 = csub(a, vb), c1 = cadd(c, vd), d1 = csub(c, vd);
      const double2 vc = cmul(c1, w2), ve = cmul(d1, w3);
      buf[lq(i0)] = cadd(a1, vc);
      buf[lq(i0 + 2 * h)] = csub(a1, vc);
      buf[lq(i0 + h)] = cadd(b1, ve);
      buf[lq(i0 + 3 * h)] = csub(b1, ve);
    }
    __syncthreads();
  }
}

// Column c of a tile: line t and column i < n/8 (consecutive c run along the
// contiguous direction of the global rows).
__device__ inline void tile_col(const LineTile &T, int c, int &t, int &i) {
  if (T.axis == 2) {
    t = c >> (T.logn - 3);
    i = c & (T.n / 8 - 1);
  } else {
    t = c & (T.tl - 1);
    i = c / T.tl;
  }
}

__device__ inline int brev3(int r) { return ((r & 1) << 2) | (r & 2) | ((r >> 2) & 1); }

template <int kSign>
__global__ __launch_bounds__(kFftThreads) void k_fft8_axis(double2 *data, const double2 *twg, int n, int logn,
                                                           int axis, int tl) {
  extern __shared__ double2 sm[];
  double2 *buf = sm;
  double2 *tw = sm + lq_size(tl * n);
  copy_to_lds(tw, twg, n / 2);
  const LineTile T(n, logn, axis, tl, xcd_unit(blockIdx.x, gridDim.x));
  const int cols = tl * n / 8, n8 = n / 8;
  for (int c = threadIdx.x; c < cols; c += kFftThreads) {
    int t, i;
    tile_col(T, c, t, i);
    double2 u[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) u[brev3(k)] = data[T.addr(t, i + k * n8)];
    dft8_first<kSign>(u);
    const int base = t * n + 8 * brev(i, logn - 3);
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[lq(base + r)] = u[r];
  }
  __syncthreads();
  fft_middle<kSign, false>(buf, tw, n, logn, tl * n);
  for (int c = threadIdx.x; c < cols; c += kFftThreads) {
    int t, i;
    tile_col(T, c, t, i);
    double2 e[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) e[k] = buf[lq(t * n + i + k * n8)];
    dft8_last<false>(e, i, n, tw);
#pragma unroll
    for (int k = 0; k < 8; ++k) data[T.addr(t, i + k * n8)] = e[k];
  }
}

// The fused x pass (see k_fft_x_green) with register stages: a thread's
// column leaves the forward transform in natural order, i + k n/8, which
// is exactly the column the inverse transforms' first stages need, so the
// Green's function and those stages run in registers.  One LDS tile serves
// the forward transform and then each output field in turn (the other
// field waits in registers).  At most one column per thread (tl n <= 8
// kT, as fft_lines picks; kT = 512 on the large meshes gives tiles of
// eight lines there, whose rows along the contiguous axis are whole 128-byte
// lines).
template <int kT>
__global__ __launch_bounds__(kT) void k_fft8_x_green(double2 *B, double2 *A, PmTables Tb, int n, int logn, int tl,
                                                     double L, double G) {
  extern __shared__ double2 sm[];
  double2 *bb = sm;
  double2 *tw = sm + lq_size(tl * n);
  double *wax = reinterpret_cast<double *>(tw + n / 2);
  copy_to_lds<kT>(tw, Tb.twf, n / 2);
  copy_to_lds<kT>(wax, Tb.wax, n);
  const LineTile T(n, logn, 0, tl, xcd_unit(blockIdx.x, gridDim.x));
  const int cols = tl * n / 8, n8 = n / 8;
  const int c = threadIdx.x;
  int t = 0, i = 0, base = 0;
  if (c < cols) {
    tile_col(T, c, t, i);
    base = t * n + 8 * brev(i, logn - 3);
    double2 u[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) u[brev3(k)] = B[T.addr(t, i + k * n8)];
    dft8_first<-1>(u);
#pragma unroll
    for (int r = 0; r < 8; ++r) bb[lq(base + r)] = u[r];
  }
  __syncthreads();
  fft_middle<-1, false, kT>(bb, tw, n, logn, tl * n);
  double2 ua[8], ub[8];
  if (c < cols) {
    double2 e[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) e[k] = bb[lq(t * n + i + k * n8)];
    dft8_last<false>(e, i, n, tw);
    const double kf = 2.0 * M_PI / L;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      int x, y, z;
      T.coords(t, i + k * n8, x, y, z);
      green(e[k], x, y, z, n, kf, G, wax, &ua[brev3(k)], &ub[brev3(k)]);
    }
    dft8_first<1>(ua);
    dft8_first<1>(ub);
  }
  // each output field in turn through the tile
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    __syncthreads();  // every read of the tile is done
    if (c < cols) {
#pragma unroll
      for (int r = 0; r < 8; ++r) bb[lq(base + r)] = f == 0 ? ua[r] : ub[r];
    }
    __syncthreads();
    fft_middle<1, true, kT>(bb, tw, n, logn, tl * n);
    if (c < cols) {
      double2 e[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) e[k] = bb[lq(t * n + i + k * n8)];
      dft8_last<true>(e, i, n, tw);
      double2 *out = f == 0 ? A : B;
#pragma unroll
      for (int k = 0; k < 8; ++k) out[T.addr(t, i + k * n8)] = e[k];
    }
  }
}

// Write one particle's interpolated mesh force (slot i, caller order).
__device__ inline void put_out(uint32_t i, double ax, double ay, double az, double ph, double *acc, double *pot,
                               int accumulate) {
  if (accumulate) {
    acc[3ull * i] += ax;
    acc[3ull * i + 1] += ay;
    acc[3ull * i + 2] += az;
    if (pot) pot[i] += ph;
  } else {
    acc[3ull * i] = ax;
    acc[3ull * i + 1] = ay;
    acc[3ull * i + 2] = az;
    if (pot) pot[i] = ph;
  }
}

// One workgroup per block: the 9^3 tile nodes of both fields staged in LDS
// once, then the block's first kBlockChunk particles interpolated from
// them, with the arithmetic of k_interp.
__global__ __launch_bounds__(kPmThreads) void k_interp_blocks(const double2 *A, const double2 *B, const double4 *part,
                                                              BlockRef R, const uint32_t *perm, int n, int logn,
                                                              double inv_d, double norm, double self, double *acc,
                                                              double *pot, int accumulate) {
  __shared__ double2 ta[kTile3], tb[kTile3];
  const uint32_t h = xcd_unit(blockIdx.x, gridDim.x);
  const uint32_t s = R.bstart[h], e = min(R.bstart[h + 1], s + kBlockChunk);
  if (s == e) return;
  int g0[3];
  block_corner(R, h, logn, g0);
  const int mask = n - 1;
  for (int c = threadIdx.x; c < kTile3; c += kPmThreads) {
    const int tx = c / (kTile * kTile), ty = (c / kTile) % kTile, tz = c % kTile;
    const uint64_t k = ((uint64_t)((g0[0] + tx) & mask) * n + ((g0[1] + ty) & mask)) * n + ((g0[2] + tz) & mask);
    ta[c] = A[k];
    tb[c] = B[k];
  }
  __syncthreads();
  for (uint32_t p = s + threadIdx.x; p < e; p += kPmThreads) {
    const double4 q = part[p];
    int r[3];
    double f[3];
    tile_cic(q, R, logn, inv_d, g0, r, f);
    const double wx[2] = {1.0 - f[0], f[0]}, wy[2] = {1.0 - f[1], f[1]}, wz[2] = {1.0 - f[2], f[2]};
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int k = ((r[0] + a) * kTile + r[1] + b) * kTile + r[2] + c;
          const double w = wx[a] * wy[b] * wz[c];
          const double2 u = ta[k], v = tb[k];
          ax += w * u.x;
          ay += w * u.y;
          az += w * v.x;
          ph += w * v.y;
        }
    ax *= norm;
    ay *= norm;
    az *= norm;
    ph = ph * norm + self * q.w;
    put_out(perm[p], ax, ay, az, ph, acc, pot, accumulate);
  }
}

__global__ __launch_bounds__(kPmThreads) void k_interp(const double2 *A, const double2 *B, PartRef P,
                                                       const uint32_t *perm, uint32_t N, int n, double inv_d,
                                                       double norm, double self, double *acc, double *pot,
                                                       int accumulate, BlockRef R) {
  const uint32_t t = xcd_unit(blockIdx.x, gridDim.x) * kPmThreads + threadIdx.x;
  if (t >= N) return;
  if (R.bstart != nullptr && !block_extra(R, t)) return;
  const double4 q = P.get(t);
  const uint32_t i = perm ? perm[t] : t;  // output slot: caller index
  int ix, iy, iz;
  double fx, fy, fz;
  cic(q.x, n, inv_d, ix, fx);
  cic(q.y, n, inv_d, iy, fy);
  cic(q.z, n, inv_d, iz, fz);
  const int jx[2] = {ix, ix + 1 == n ? 0 : ix + 1};
  const int jy[2] = {iy, iy + 1 == n ? 0 : iy + 1};
  const int jz[2] = {iz, iz + 1 == n ? 0 : iz + 1};
  const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
  double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const uint64_t k = ((uint64_t)jx[a] * n + jy[b]) * n + jz[c];
        const double w = wx[a] * wy[b] * wz[c];
        const double2 u = A[k], v = B[k];
        ax += w * u.x;
        ay += w * u.y;
        az += w * v.x;
        ph += w * v.y;
      }
  ax *= norm;
  ay *= norm;
  az *= norm;
  ph = ph * norm + self * q.w;
  put_out(i, ax, ay, az, ph, acc, pot, accumulate);
}

inline uint32_t blocks_for(uint64_t work, uint32_t threads, uint32_t cap) {
  const uint64_t b = (work + threads - 1) / threads;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(b, cap));
}

}  // namespace

// Meshes from 64 points per axis take the register-staged passes.
inline bool fft_regs(int n) { return n >= 64; }

// LDS bytes of a workgroup of `tl` lines: the padded tile and the forward
// or inverse twiddles; fused (the x pass with the Green's function): its
// padded tile (two for the small meshes' kernel), the forward twiddles and
// the per-axis Green factors.
size_t fft_lds_bytes(int n, int tl, bool fused) {
  const size_t tile = (size_t)(fft_regs(n) ? lq_size(tl * n) : lp_size(tl * n)) * sizeof(double2);
  // the register-staged fused pass keeps one tile
  const size_t tiles = fused && !fft_regs(n) ? 2 * tile : tile;
  return fused ? tiles + (size_t)(n / 2) * sizeof(double2) + (size_t)n * sizeof(double)
               : tile + (size_t)(n / 2) * sizeof(double2);
}

// LDS a workgroup may hold on gfx950.
constexpr size_t kLdsMax = 163840;

// Threads the fused x pass may use: 512 on meshes of 512 and more (tiles
// of eight lines at 512), else kFftThreads; a launch takes 512 only when
// its tile needs them.
int xg_threads(int n) { return fft_regs(n) && n >= 512 ? 512 : kFftThreads; }

// Lines per workgroup.  Register-staged passes: 2048 elements per tile (one
// column of eight per thread; at most 16 lines); smaller meshes: 16 lines.
// At most n, and halved until the workgroup's LDS fits (and, for the fused
// x pass, its tile in eight elements per thread).  OG_FFT_LINES=k (a power
// of two, 1..16), read at each launch, replaces the width (still at most n
// and halved until it fits), so that the tests run every width and tile
// size the library can pick on small meshes.
int fft_lines(int n, bool fused) {
  const int per = 8 * (fused ? xg_threads(n) : kFftThreads);  // tile elements the workgroup holds in registers
  int tl = fft_regs(n) ? (per / n > 16 ? 16 : per / n) : 16;
  const char *e = getenv("OG_FFT_LINES");
  const int want = e ? atoi(e) : 0;
  if (want >= 1 && want <= 16 && (want & (want - 1)) == 0) tl = want;
  if (tl > n) tl = n;
  while (tl > 1 && (fft_lds_bytes(n, tl, fused) > kLdsMax || (fused && tl * n > per))) tl >>= 1;
  return tl;
}

// The forward z pass that reads the fixed-point sums (k_fft_z_density, all
// in LDS, lp layout; its loads gather the block halos, and it runs fastest
// with the narrower tiles that leave more workgroups per CU): 16, 8, 4, 4
// and 2 lines at n <= 64, 128, 256, 512 and 1024, or OG_FFT_LINES.
size_t fft_z_lds_bytes(int n, int tl) {
  return (size_t)lp_size(tl * n) * sizeof(double2) + (size_t)(n / 2) * sizeof(double2);
}
int fft_z_lines(int n) {
  int tl = n <= 64 ? 16 : (n <= 128 ? 8 : (n <= 512 ? 4 : 2));
  const char *e = getenv("OG_FFT_LINES");
  const int want = e ? atoi(e) : 0;
  if (want >= 1 && want <= 16 && (want & (want - 1)) == 0) tl = want;
  if (tl > n) tl = n;
  while (tl > 1 && fft_z_lds_bytes(n, tl) > kLdsMax) tl >>= 1;
  return tl;
}

namespace {
// Dynamic LDS beyond the default 64 KB is enabled once per process for the
// FFT kernels.
void allow_large_lds() {
  static const bool done = [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_axis<-1>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_axis<1>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_z_density),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_x_green),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft8_axis<-1>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft8_axis<1>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft8_x_green<kFftThreads>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft8_x_green<512>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
    return true;
  }();
  (void)done;
}

void launch_fft_pass(double2 *data, const PmTables &Tb, int n, int logn, int sign, int axis, hipStream_t s) {
  const int tl = fft_lines(n, false);
  const uint32_t blocks = (uint32_t)((uint64_t)n * n / tl);
  const size_t lds = fft_lds_bytes(n, tl, false);
  if (fft_regs(n)) {
    if (sign < 0) k_fft8_axis<-1><<<blocks, kFftThreads, lds, s>>>(data, Tb.twf, n, logn, axis, tl);
    else k_fft8_axis<1><<<blocks, kFftThreads, lds, s>>>(data, Tb.twi, n, logn, axis, tl);
  } else if (sign < 0) {
    k_fft_axis<-1><<<blocks, kFftThreads, lds, s>>>(data, Tb.twf, n, logn, axis, tl);
  } else {
    k_fft_axis<1><<<blocks, kFftThreads, lds, s>>>(data, Tb.twi, n, logn, axis, tl);
  }
}
}  // namespace

void launch_pm(const PmArgs &P, hipStream_t s) {
  const uint64_t cells = (uint64_t)P.n * P.n * P.n;
  const double d = P.L / P.n, inv_d = P.n / P.L;
  int logn = 0;
  while ((1 << logn) < P.n) ++logn;
  // the fixed-point mesh aliases A until the fused x pass writes A
  unsigned long long *fixed = reinterpret_cast<unsigned long long *>(P.A);
  const PartRef R{P.pos, P.mass, P.part};
  // Tree order: block workgroups (see k_deposit_blocks); the halo entries
  // live in the second half of A, which the fixed-point mesh leaves free.
  const bool blocks = P.part != nullptr && P.keys != nullptr && P.bstart != nullptr;
  BlockRef BR{nullptr, nullptr, 0, 0, 0.0};
  const uint32_t nblocks = (uint32_t)(cells / (kBlk * kBlk * kBlk));
  allow_large_lds();
  const PmTables Tb{P.tables, P.tables + P.n / 2, reinterpret_cast<double *>(P.tables + P.n)};
  k_pm_tables<<<blocks_for((uint64_t)P.n, kPmThreads, 64), kPmThreads, 0, s>>>(Tb, P.n, P.L, P.r_s);
  k_fill_u64<<<1, kPmThreads, 0, s>>>(P.mmax, 1);
  k_mass_max<<<blocks_for(P.N, kPmThreads, 1024), kPmThreads, 0, s>>>(R, P.N, P.mmax);
  const unsigned long long *halo = nullptr;
  if (blocks) {
    BR = BlockRef{P.keys, P.bstart, 3 * (kLevels - (logn - 3)), P.curve, P.tscale};
    unsigned long long *hb = fixed + cells;
    k_block_starts<<<blocks_for(nblocks + 1ull, kPmThreads, 1u << 30), kPmThreads, 0, s>>>(BR, P.N, nblocks,
                                                                                          P.bstart);
    k_deposit_blocks<<<nblocks, kPmThreads, 0, s>>>(P.part, BR, P.N, P.n, logn, inv_d, P.mmax, fixed, hb);
    // what blocks of more than kBlockChunk particles left: atomics onto
    // the stored mesh (the halo stays apart until the density is read)
    k_deposit_tiled<<<blocks_for(P.N, kPmThreads, 1u << 30), kPmThreads, 0, s>>>(R, P.N, P.n, inv_d, P.mmax,
                                                                                 fixed, BR);
    halo = hb;
  } else {
    // Caller order: direct atomics (neighbouring threads rarely share a node).
    k_fill_u64<<<blocks_for(cells, kPmThreads, 8192), kPmThreads, 0, s>>>(fixed, cells);
    k_deposit<<<blocks_for(P.N, kPmThreads, 1u << 30), kPmThreads, 0, s>>>(R, P.N, P.n, inv_d, P.mmax, fixed);
  }
  // forward transform: z (reading the density), y, then x fused with the
  // Green's function and the inverse x passes; then the inverse y and z
  // passes of both fields
  {
    const int tl = fft_z_lines(P.n);
    k_fft_z_density<<<(uint32_t)((uint64_t)P.n * P.n / tl), kFftThreads, fft_z_lds_bytes(P.n, tl), s>>>(
        fixed, halo, P.N, P.mmax, 1.0 / (d * d * d), Tb.twf, P.B, P.n, logn, tl);
  }
  launch_fft_pass(P.B, Tb, P.n, logn, -1, 1, s);
  {
    const int tl = fft_lines(P.n, true);
    const uint32_t blocks = (uint32_t)((uint64_t)P.n * P.n / tl);
    const size_t lds = fft_lds_bytes(P.n, tl, true);
    if (fft_regs(P.n) && tl * P.n > 8 * kFftThreads)  // one column of eight per thread
      k_fft8_x_green<512><<<blocks, 512, lds, s>>>(P.B, P.A, Tb, P.n, logn, tl, P.L, P.G);
    else if (fft_regs(P.n))
      k_fft8_x_green<kFftThreads><<<blocks, kFftThreads, lds, s>>>(P.B, P.A, Tb, P.n, logn, tl, P.L, P.G);
    else k_fft_x_green<<<blocks, kFftThreads, lds, s>>>(P.B, P.A, Tb, P.n, logn, tl, P.L, P.G);
  }
  for (double2 *f : {P.A, P.B}) {
    launch_fft_pass(f, Tb, P.n, logn, +1, 1, s);
    launch_fft_pass(f, Tb, P.n, logn, +1, 2, s);
  }
  const double self = P.G / (std::sqrt(M_PI) * P.r_s);
  if (blocks)
    k_interp_blocks<<<nblocks, kPmThreads, 0, s>>>(P.A, P.B, P.part, BR, P.perm, P.n, logn, inv_d,
                                                   1.0 / (double)cells, self, P.acc, P.pot, P.accumulate);
  k_interp<<<blocks_for(P.N, kPmThreads, 1u << 30), kPmThreads, 0, s>>>(
      P.A, P.B, R, P.part ? P.perm : nullptr, P.N, P.n, inv_d, 1.0 / (double)cells, self, P.acc, P.pot,
      P.accumulate, BR);
}

}  // namespace og
