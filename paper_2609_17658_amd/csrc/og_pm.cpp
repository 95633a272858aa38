// C ABI of the particle-mesh long-range force (og_pm_*), see include/og.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>

#include "og_forest.h"
#include "og_pm.h"

using namespace og;

struct og_pm {
  int n = 0;
  double L = 0, G = 0, r_s = 0;
  hipStream_t stream = nullptr;
  void *mem = nullptr;
  double2 *A = nullptr, *B = nullptr;
  unsigned long long *mmax = nullptr;
  double2 *tables = nullptr;
  uint32_t *bstart = nullptr;
};

namespace {

bool pow2_in_range(int32_t n) { return n >= 8 && n <= 1024 && (n & (n - 1)) == 0; }

size_t pm_bytes(int32_t n) {
  const size_t cells = (size_t)n * n * n;
  return 2 * cells * sizeof(double2) + 256 + ((pm_table_bytes(n) + 255) & ~(size_t)255) +
         ((pm_block_words(n) * 4 + 255) & ~(size_t)255);
}

}  // namespace

extern "C" {

size_t og_pm_workspace_bound(int32_t n_grid) {
  if (!pow2_in_range(n_grid)) return 0;
  return pm_bytes(n_grid);
}

int og_pm_create(int32_t n_grid, double box, double G, double r_s, void *stream, og_pm **out) {
  if (!out) return fail(OG_EINVAL, "out is NULL");
  if (!pow2_in_range(n_grid)) return fail(OG_EINVAL, "n_grid must be a power of two in 8..1024");
  if (!(box > 0.0) || !std::isfinite(box)) return fail(OG_EINVAL, "box must be > 0");
  if (!(r_s > 0.0) || !std::isfinite(r_s)) return fail(OG_EINVAL, "r_s must be > 0");
  if (!std::isfinite(G)) return fail(OG_EINVAL, "G must be finite");
  og_pm *p = new (std::nothrow) og_pm();
  if (!p) return fail(OG_ENOMEM, "host allocation");
  p->n = n_grid;
  p->L = box;
  p->G = G;
  p->r_s = r_s;
  p->stream = (hipStream_t)stream;
  if (fault_fires(kFaultAlloc)) {
    delete p;
    return fail(OG_ENOMEM, "forced failure of the mesh allocation (OG_FAULT_ALLOC)");
  }
  hipError_t e = hipMalloc(&p->mem, pm_bytes(n_grid));
  if (e != hipSuccess) {
    delete p;
    (void)hipGetLastError();
    return fail(OG_ENOMEM, "hipMalloc(%zu) for the mesh failed", pm_bytes(n_grid));
  }
  const size_t cells = (size_t)n_grid * n_grid * n_grid;
  p->A = static_cast<double2 *>(p->mem);
  p->B = p->A + cells;
  p->mmax = reinterpret_cast<unsigned long long *>(p->B + cells);
  p->tables = reinterpret_cast<double2 *>(reinterpret_cast<char *>(p->mmax) + 256);
  p->bstart = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(p->tables) +
                                           ((pm_table_bytes(n_grid) + 255) & ~(size_t)255));
  *out = p;
  return OG_OK;
}

int og_pm_force(og_pm *pm, const double *pos, const double *mass, int64_t N, double *acc, double *pot,
                int32_t accumulate) {
  const og::TraceRange trace_range("og_pm_force");
  if (!pm) return fail(OG_EINVAL, "pm is NULL");
  if (N < 1 || N > 0x7fffffffll) return fail(OG_EINVAL, "N = %lld outside [1, 2^31-1]", (long long)N);
  if (!is_device_ptr(pos) || !is_device_ptr(mass) || !is_device_ptr(acc) || (pot && !is_device_ptr(pot)))
    return fail(OG_EINVAL, "pos/mass/acc/pot must be device pointers");
  PmArgs P{};
  P.pos = pos;
  P.mass = mass;
  P.N = (uint32_t)N;
  P.n = pm->n;
  P.L = pm->L;
  P.G = pm->G;
  P.r_s = pm->r_s;
  P.A = pm->A;
  P.B = pm->B;
  P.mmax = pm->mmax;
  P.tables = pm->tables;
  P.acc = acc;
  P.pot = pot;
  P.accumulate = accumulate ? 1 : 0;
  launch_pm(P, pm->stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "particle-mesh launch");
  return OG_OK;
}

int og_pm_force_tree(og_pm *pm, const og_tree *tree, double *acc, double *pot, int32_t accumulate) {
  const og::TraceRange trace_range("og_pm_force_tree");
  if (!pm || !tree) return fail(OG_EINVAL, "pm or tree is NULL");
  const Forest &F = tree->F;
  const BoxDev &b = F.hboxes[0];
  if (!b.periodic || b.box != pm->L) return fail(OG_EINVAL, "the tree must be periodic with the mesh's box side");
  if (!is_device_ptr(acc) || (pot && !is_device_ptr(pot))) return fail(OG_EINVAL, "acc/pot must be device pointers");
  PmArgs P{};
  P.part = F.A.part64;
  P.perm = F.A.perm;
  P.keys = F.A.keys_a;
  P.curve = b.curve;
  P.tscale = b.scale;
  P.bstart = pm->bstart;
  P.N = F.N;
  P.n = pm->n;
  P.L = pm->L;
  P.G = pm->G;
  P.r_s = pm->r_s;
  P.A = pm->A;
  P.B = pm->B;
  P.mmax = pm->mmax;
  P.tables = pm->tables;
  P.acc = acc;
  P.pot = pot;
  P.accumulate = accumulate ? 1 : 0;
  // the tree's particles are ready once its stream has passed the build
  const int rc = order_after(pm->stream, F.stream);
  if (rc != OG_OK) return rc;
  launch_pm(P, pm->stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "particle-mesh launch");
  return OG_OK;
}

int og_pm_free(og_pm *pm) {
  if (!pm) return OG_OK;
  (void)hipStreamSynchronize(pm->stream);
  if (pm->mem) (void)hipFree(pm->mem);
  delete pm;
  return OG_OK;
}

}  // extern "C"
