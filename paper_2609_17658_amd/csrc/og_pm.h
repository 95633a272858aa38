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
};

void launch_pm(const PmArgs &P, hipStream_t s);
void launch_fft3(double2 *data, int n, int sign, hipStream_t s);
int fft_lines_per_block(int n);

}  // namespace og
