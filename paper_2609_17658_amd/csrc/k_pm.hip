// Particle-mesh long-range force for CDNA4 (gfx950).
//
// Paper, "Particle Mesh": the particles' mass is assigned to a periodic
// mesh, the density is Fourier transformed, multiplied by the Green's
// function of the Poisson equation with the Gaussian filter
// exp(-k^2 A_smth^2), and transformed back; the tree carries the erfc part
// of the split, the mesh the erf part.
//
// Layout: an n^3 mesh of complex FP64 values (double2), index (x*n + y)*n + z.
//   1. deposit: cloud-in-cell weights onto the nodes j*L/n, summed with
//      64-bit fixed-point atomics (a power-of-two scale fitted to N * max m),
//      so the mesh does not depend on the order of the atomic additions;
//   2. forward 3-D FFT of the density (three passes of length-n transforms
//      along z, y and x; each workgroup transforms a tile of neighbouring
//      lines in LDS, so every pass reads and writes whole cache lines);
//   3. per wave vector: phi_k = -4 pi G exp(-k^2 r_s^2) / k^2 / W(k)^2 rho_k,
//      W the CIC window, and a_k = -i k phi_k; the two inverse transforms
//      carry (a_x + i a_y) and (a_z + i phi), each a pair of real fields;
//   4. inverse FFTs, then CIC interpolation at the particles.
#include <climits>
#include <cmath>
#include <cstdlib>

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

__global__ __launch_bounds__(kPmThreads) void k_deposit_tiled(PartRef P, uint32_t N, int n, double inv_d,
                                                              const unsigned long long *mmax,
                                                              unsigned long long *acc_mesh) {
  __shared__ unsigned long long tile[kDepositTile];
  __shared__ int red[6][kPmThreads / 64];
  const uint32_t i = blockIdx.x * kPmThreads + threadIdx.x;
  const bool ok = i < N;
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

// Fixed point -> density (mass / cell volume), as the real part.
__global__ __launch_bounds__(kPmThreads) void k_density(const unsigned long long *acc_mesh, uint64_t cells,
                                                        uint32_t N, const unsigned long long *mmax,
                                                        double inv_vol, double2 *rho) {
  const double f = inv_vol / fixed_scale(mmax, N);
  for (uint64_t i = blockIdx.x * (uint64_t)kPmThreads + threadIdx.x; i < cells;
       i += (uint64_t)gridDim.x * kPmThreads)
    rho[i] = make_double2((double)acc_mesh[i] * f, 0.0);
}

// Length-n transforms along one axis, radix 2, decimation in time (input in
// bit-reversed order).  kSign = -1: forward e^{-2 pi i jk/n}; +1: inverse
// without the 1/n.  Lines: axis 2 (z, contiguous) takes `tl` consecutive
// lines; axes 1 and 0 take `tl` lines with consecutive z, so element j of
// the tile is `tl` contiguous values.
template <int kSign>
__global__ __launch_bounds__(kFftThreads) void k_fft_axis(double2 *data, int n, int logn, int axis, int tl) {
  extern __shared__ double2 sm[];
  double2 *buf = sm;
  double2 *tw = sm + (size_t)tl * n;
  const int tid = threadIdx.x;
  for (int k = tid; k < n / 2; k += kFftThreads) {
    double s, c;
    sincospi(2.0 * k / n, &s, &c);
    tw[k] = make_double2(c, kSign * s);
  }
  const uint32_t g = blockIdx.x;
  const uint32_t per = (uint32_t)(n / tl);
  const uint32_t a = g / per, z0 = (g % per) * tl;
  const uint64_t nn = (uint64_t)n;
  auto addr = [&](int t, int j) -> uint64_t {
    if (axis == 2) return ((uint64_t)g * tl + t) * nn + j;
    if (axis == 1) return ((uint64_t)a * nn + j) * nn + z0 + t;
    return ((uint64_t)j * nn + a) * nn + z0 + t;
  };
  const int total = tl * n;
  for (int idx = tid; idx < total; idx += kFftThreads) {
    int t, j;
    if (axis == 2) {
      t = idx >> logn;
      j = idx & (n - 1);
    } else {
      t = idx % tl;
      j = idx / tl;
    }
    const int jr = (int)(__brev((uint32_t)j) >> (32 - logn));
    buf[t * n + jr] = data[addr(t, j)];
  }
  __syncthreads();
  int s = 1;
  if (logn & 1) {
    // one radix-2 stage (len 2, twiddle 1) when log2 n is odd
    for (int b = tid; b < total / 2; b += kFftThreads) {
      const int i0 = 2 * b;
      const double2 u = buf[i0], v = buf[i0 + 1];
      buf[i0] = make_double2(u.x + v.x, u.y + v.y);
      buf[i0 + 1] = make_double2(u.x - v.x, u.y - v.y);
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
      const double2 w1 = tw[pos * step1], w2 = tw[pos * step2];
      // the second stage's twiddle for the odd pair is w2 exp(sign i pi/2)
      const double2 w3 = make_double2(-kSign * w2.y, kSign * w2.x);
      const double2 a = buf[i0], b0 = buf[i0 + h], c = buf[i0 + 2 * h], d0 = buf[i0 + 3 * h];
      const double2 vb = make_double2(b0.x * w1.x - b0.y * w1.y, b0.x * w1.y + b0.y * w1.x);
      const double2 vd = make_double2(d0.x * w1.x - d0.y * w1.y, d0.x * w1.y + d0.y * w1.x);
      const double2 a1 = make_double2(a.x + vb.x, a.y + vb.y), b1 = make_double2(a.x - vb.x, a.y - vb.y);
      const double2 c1 = make_double2(c.x + vd.x, c.y + vd.y), d1 = make_double2(c.x - vd.x, c.y - vd.y);
      const double2 vc = make_double2(c1.x * w2.x - c1.y * w2.y, c1.x * w2.y + c1.y * w2.x);
      const double2 ve = make_double2(d1.x * w3.x - d1.y * w3.y, d1.x * w3.y + d1.y * w3.x);
      buf[i0] = make_double2(a1.x + vc.x, a1.y + vc.y);
      buf[i0 + 2 * h] = make_double2(a1.x - vc.x, a1.y - vc.y);
      buf[i0 + h] = make_double2(b1.x + ve.x, b1.y + ve.y);
      buf[i0 + 3 * h] = make_double2(b1.x - ve.x, b1.y - ve.y);
    }
    __syncthreads();
  }
  for (int idx = tid; idx < total; idx += kFftThreads) {
    int t, j;
    if (axis == 2) {
      t = idx >> logn;
      j = idx & (n - 1);
    } else {
      t = idx % tl;
      j = idx / tl;
    }
    data[addr(t, j)] = buf[t * n + j];
  }
}

__device__ inline double sinc(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

// Green's function, CIC deconvolution and gradient, per wave vector:
// B holds rho_k on entry and (a_z + i phi)_k on exit, A gets (a_x + i a_y)_k.
// The deconvolution 1 / W^2 = prod over axes of sinc(pi m / n)^-4 is
// tabulated once per workgroup (n <= 1024 entries); n is a power of two,
// so the cell index splits by shifts.
__global__ __launch_bounds__(kPmThreads) void k_green(double2 *B, double2 *A, int n, double L, double G,
                                                      double r_s) {
  __shared__ double dec[1024];
  for (int j = threadIdx.x; j < n; j += kPmThreads) {
    const int m = j < n / 2 ? j : j - n;
    const double sj = sinc(M_PI * m / n), s2 = sj * sj;
    dec[j] = 1.0 / (s2 * s2);
  }
  __syncthreads();
  const int logn = __builtin_ctz((unsigned)n);
  const uint64_t cells = (uint64_t)n * n * n, mask = (uint64_t)(n - 1);
  const double kf = 2.0 * M_PI / L;
  for (uint64_t i = blockIdx.x * (uint64_t)kPmThreads + threadIdx.x; i < cells;
       i += (uint64_t)gridDim.x * kPmThreads) {
    const int iz = (int)(i & mask), iy = (int)((i >> logn) & mask), ix = (int)(i >> (2 * logn));
    const int mx = ix < n / 2 ? ix : ix - n, my = iy < n / 2 ? iy : iy - n, mz = iz < n / 2 ? iz : iz - n;
    const double kx = kf * mx, ky = kf * my, kz = kf * mz;
    const double k2 = kx * kx + ky * ky + kz * kz;
    if (k2 == 0.0) {
      A[i] = make_double2(0.0, 0.0);
      B[i] = make_double2(0.0, 0.0);
      continue;
    }
    const double g = -4.0 * M_PI * G * exp(-k2 * r_s * r_s) / k2 * (dec[ix] * dec[iy] * dec[iz]);
    const double2 rho = B[i];
    const double pr = g * rho.x, pi = g * rho.y;  // phi_k
    // derivative wavenumbers, the Nyquist one dropped
    const double dx = mx == -n / 2 ? 0.0 : kx, dy = my == -n / 2 ? 0.0 : ky, dz = mz == -n / 2 ? 0.0 : kz;
    // a_k = -i k phi_k = k (phi_i, -phi_r)
    const double axr = dx * pi, axi = -dx * pr;
    const double ayr = dy * pi, ayi = -dy * pr;
    const double azr = dz * pi, azi = -dz * pr;
    A[i] = make_double2(axr - ayi, axi + ayr);
    B[i] = make_double2(azr - pi, azi + pr);
  }
}

__global__ __launch_bounds__(kPmThreads) void k_interp(const double2 *A, const double2 *B, PartRef P,
                                                       const uint32_t *perm, uint32_t N, int n, double inv_d,
                                                       double norm, double self, double *acc, double *pot,
                                                       int accumulate) {
  const uint32_t t = blockIdx.x * kPmThreads + threadIdx.x;
  if (t >= N) return;
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

inline uint32_t blocks_for(uint64_t work, uint32_t threads, uint32_t cap) {
  const uint64_t b = (work + threads - 1) / threads;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(b, cap));
}

}  // namespace

// Lines per workgroup: up to 16, at most n, and a tile plus twiddles within
// 64 KB of LDS (16 up to n = 128, then 8, 4 and 2 at n = 256, 512 and
// 1024).  OG_FFT_LINES=k (a power of two, 1..16), read at each launch,
// caps it, so that the tests run every width the library can pick on small
// meshes.
int fft_lines_per_block(int n) {
  int tl = 16;
  while (tl > 1 && (tl > n || (size_t)tl * n * sizeof(double2) + (size_t)(n / 2) * sizeof(double2) > 65536)) tl >>= 1;
  const char *e = getenv("OG_FFT_LINES");
  const int cap = e ? atoi(e) : 0;
  if (cap >= 1 && cap <= 16 && (cap & (cap - 1)) == 0 && cap < tl) tl = cap;
  return tl;
}

void launch_fft3(double2 *data, int n, int sign, hipStream_t s) {
  int logn = 0;
  while ((1 << logn) < n) ++logn;
  const int tl = fft_lines_per_block(n);
  const uint32_t blocks = (uint32_t)((uint64_t)n * n / tl);
  const size_t lds = ((size_t)tl * n + n / 2) * sizeof(double2);
  for (int axis = 2; axis >= 0; --axis) {
    if (sign < 0) k_fft_axis<-1><<<blocks, kFftThreads, lds, s>>>(data, n, logn, axis, tl);
    else k_fft_axis<1><<<blocks, kFftThreads, lds, s>>>(data, n, logn, axis, tl);
  }
}

void launch_pm(const PmArgs &P, hipStream_t s) {
  const uint64_t cells = (uint64_t)P.n * P.n * P.n;
  const double d = P.L / P.n, inv_d = P.n / P.L;
  unsigned long long *fixed = reinterpret_cast<unsigned long long *>(P.A);  // aliases A until k_green
  k_fill_u64<<<blocks_for(cells, kPmThreads, 8192), kPmThreads, 0, s>>>(fixed, cells);
  k_fill_u64<<<1, kPmThreads, 0, s>>>(P.mmax, 1);
  // Caller order: direct atomics (neighbouring threads rarely share a node).
  // Curve order (a tree's particles): LDS tiles per workgroup.  Interpolation
  // in curve order shares the eight nodes of neighbouring threads in cache.
  const PartRef R{P.pos, P.mass, P.part};
  k_mass_max<<<blocks_for(P.N, kPmThreads, 1024), kPmThreads, 0, s>>>(R, P.N, P.mmax);
  if (P.part)
    k_deposit_tiled<<<blocks_for(P.N, kPmThreads, 1u << 30), kPmThreads, 0, s>>>(R, P.N, P.n, inv_d, P.mmax,
                                                                                 fixed);
  else
    k_deposit<<<blocks_for(P.N, kPmThreads, 1u << 30), kPmThreads, 0, s>>>(R, P.N, P.n, inv_d, P.mmax, fixed);
  k_density<<<blocks_for(cells, kPmThreads, 8192), kPmThreads, 0, s>>>(fixed, cells, P.N, P.mmax,
                                                                       1.0 / (d * d * d), P.B);
  launch_fft3(P.B, P.n, -1, s);
  k_green<<<blocks_for(cells, kPmThreads, 8192), kPmThreads, 0, s>>>(P.B, P.A, P.n, P.L, P.G, P.r_s);
  launch_fft3(P.A, P.n, +1, s);
  launch_fft3(P.B, P.n, +1, s);
  const double self = P.G / (std::sqrt(M_PI) * P.r_s);
  k_interp<<<blocks_for(P.N, kPmThreads, 1u << 30), kPmThreads, 0, s>>>(
      P.A, P.B, R, P.part ? P.perm : nullptr, P.N, P.n, inv_d, 1.0 / (double)cells, self, P.acc, P.pot,
      P.accumulate);
}

}  // namespace og
