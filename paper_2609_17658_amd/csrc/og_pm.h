// Particle-mesh launch interface (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace og {

struct PmArgs {
  const double *pos;   // caller [N][3] (when part is null)
  const double *mass;  // caller [N]
  const double4 *part; // or: a tree's particles in curve order, (x, y, z, m)
  const uint32_t *perm;  // with part: curve position -> caller index
  uint32_t N;
  int n;               // mesh points per axis, power of two, 8..1024
  double L, G, r_s;
  double2 *A, *B;      // n^3 complex each
  unsigned long long *mmax;
  double *acc;         // [N][3]
  double *pot;         // [N] or null
  int accumulate;      // 1: add to acc/pot
  // With part (a periodic tree whose root cube is the mesh box): the tree's
  // sorted keys and curve, its level-21 cell scale 2^21 / L, and room for
  // (n/8)^3 + 1 block starts (pm_block_words).
  const uint64_t *keys;
  int curve;
  double tscale;
  uint32_t *bstart;
  double2 *tables;     // 3n/2 double2: FFT twiddles and the deconvolution (pm_table_bytes)
};

// Bytes of the per-size tables: n/2 forward and n/2 inverse twiddles, n
// deconvolution factors.
inline size_t pm_table_bytes(int n) { return (size_t)n * 16 + (size_t)n * 8; }

// Words of block starts the tree-order path needs for an n^3 mesh.
inline size_t pm_block_words(int n) { return (size_t)(n / 8) * (n / 8) * (n / 8) + 1; }

void launch_pm(const PmArgs &P, hipStream_t s);
int fft_lines(int n, bool fused);
size_t fft_lds_bytes(int n, int tl, bool fused);

}  // namespace og
