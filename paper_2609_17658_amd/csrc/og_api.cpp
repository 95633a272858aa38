// C ABI of the tree force library: argument checks, device memory layout,
// tree/batch objects and stream-ordered launches.  No torch types; every
// array is a raw device pointer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/og.h"
#include "og_forest.h"

using namespace og;

// ------------------------------------------------------------ errors --
namespace og {
thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  (void)hipGetLastError();
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(OG_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(OG_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool is_device_ptr(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

bool trace_on() {
  static const bool on = [] {
    const char *e = std::getenv("OG_TRACE");
    return e && std::atoi(e) == 1;
  }();
  return on;
}
TraceRange::TraceRange(const char *name) : on(trace_on()) {
  if (on) roctxRangePushA(name);
}
TraceRange::~TraceRange() {
  if (on) roctxRangePop();
}

bool fault_fires(FaultKind k) {
  static std::mutex mu;
  static std::string seen[2];
  static long count[2] = {0, 0};
  const char *v = std::getenv(k == kFaultAlloc ? "OG_FAULT_ALLOC" : "OG_FAULT_LAUNCH");
  const std::string cur = v ? v : "";
  std::lock_guard<std::mutex> lk(mu);
  if (cur != seen[k]) {
    seen[k] = cur;
    count[k] = 0;
  }
  const long at = cur.empty() ? 0 : std::strtol(cur.c_str(), nullptr, 10);
  return at > 0 && ++count[k] == at;
}

// ---------------------------------------------------------- layout --
namespace {
struct Carver {
  size_t off = 0;
  char *base = nullptr;
  template <class T>
  T *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += sizeof(T) * (count ? count : 1);
    return p;
  }
};

void carve(Carver &c, BuildArrays &A, uint32_t n, uint32_t node_cap, int B, bool soft) {
  A.boxes = c.take<BoxDev>(B);
  A.minmax = c.take<uint64_t>(6ull * B);
  A.keys_a = c.take<uint64_t>(n);
  A.keys_b = c.take<uint64_t>(n);
  A.vals_a = c.take<uint32_t>(n);
  A.vals_b = c.take<uint32_t>(n);
  A.hist = c.take<uint32_t>(radix_hist_words(n));
  A.digit_tot = c.take<uint32_t>(256);
  A.perm = c.take<uint32_t>(n);
  A.inv = c.take<uint32_t>(n);
  A.part64 = c.take<double4>(n);
  A.part32 = c.take<float4>(n);
  A.lcp = c.take<int8_t>(n);
  A.depth = c.take<uint8_t>(n);
  A.nstart = c.take<uint32_t>(n);
  A.S = c.take<uint32_t>(n + 1ull);
  A.scan_partial = c.take<uint32_t>(std::max<size_t>(n, node_cap) / kScanTile + 4);
  A.topo = c.take<Topo>(node_cap);
  A.mom64 = c.take<Mom64>(node_cap);
  A.mom32 = c.take<Mom32>(node_cap);
  A.wnode = c.take<WNode>(node_cap);
  A.cen64 = c.take<double4>(node_cap);
  A.first = c.take<uint32_t>(node_cap);
  A.skip = c.take<uint32_t>(node_cap);
  A.parent = c.take<uint32_t>(node_cap);
  A.top_cap = top_node_bound(node_cap);
  A.top_cnt = c.take<uint32_t>(32);
  A.top_buf = c.take<uint32_t>(kTopWords * A.top_cap);
  A.top_id = c.take<uint32_t>(node_cap);
  A.scalars = c.take<uint32_t>(32);
  if (soft) {
    A.seps = c.take<double>(n);
    A.semax = c.take<double>(node_cap);
    A.semin = c.take<double>(node_cap);
  }
}
}  // namespace

uint64_t node_bound(uint64_t n, int leaf_max) { return n + 21ull * (n / (uint64_t)(leaf_max + 1)) + 1ull; }

size_t forest_bytes(uint32_t n, uint32_t node_cap, int B, bool soft) {
  Carver c;
  BuildArrays A{};
  carve(c, A, n, node_cap, B, soft);
  return c.off + 256;
}

// --------------------------------------------------------- params --
int check_params(const og_params *p, int64_t N, double box, bool need_stream_fields) {
  (void)need_stream_fields;
  if (!p) return fail(OG_EINVAL, "params is NULL");
  if (p->struct_size != sizeof(og_params))
    return fail(OG_EINVAL, "og_params.struct_size = %u, expected %zu", p->struct_size, sizeof(og_params));
  if (N < 1 || N > (int64_t)kCountMask) return fail(OG_EINVAL, "N = %lld outside [1, 2^27-1]", (long long)N);
  if (!(box > 0.0) || !std::isfinite(box)) return fail(OG_EINVAL, "box must be > 0");
  if (!(p->eps >= 0.0) || !std::isfinite(p->eps)) return fail(OG_EINVAL, "eps must be >= 0");
  if (!(p->theta >= 0.0) || !std::isfinite(p->theta)) return fail(OG_EINVAL, "theta must be >= 0");
  if (!std::isfinite(p->G)) return fail(OG_EINVAL, "G must be finite");
  if (p->leaf_max < 1 || p->leaf_max > 4096) return fail(OG_EINVAL, "leaf_max outside 1..4096");
  if (p->group_max < 0 || p->group_max > 64) return fail(OG_EINVAL, "group_max outside 0..64");
  if (p->walk_list_cap != 0 && p->walk_list_cap != 4 && p->walk_list_cap != 8 && p->walk_list_cap != 16 &&
      p->walk_list_cap != 32)
    return fail(OG_EINVAL, "walk_list_cap must be 0, 4, 8, 16 or 32");
  if (p->precision != OG_PREC_FP64 && p->precision != OG_PREC_MIXED)
    return fail(OG_EINVAL, "unknown precision %d", p->precision);
  if (p->softening != OG_SOFT_PLUMMER && p->softening != OG_SOFT_SPLINE)
    return fail(OG_EINVAL, "unknown softening %d", p->softening);
  if (p->softening == OG_SOFT_SPLINE && !(p->eps > 0.0) && !p->eps_particle)
    return fail(OG_EINVAL, "spline softening needs eps > 0");
  if (p->lists != OG_LISTS_TARGET && p->lists != OG_LISTS_GROUP)
    return fail(OG_EINVAL, "unknown lists mode %d", p->lists);
  if (p->eps_particle && !is_device_ptr(p->eps_particle))
    return fail(OG_EINVAL, "eps_particle must be a device pointer");
  if (p->eps_particle && p->lists == OG_LISTS_GROUP)
    return fail(OG_EUNSUPPORTED, "per-particle softening with group-shared lists is not available");
  if (p->curve != OG_CURVE_MORTON && p->curve != OG_CURVE_HILBERT)
    return fail(OG_EINVAL, "unknown curve %d", p->curve);
  if (p->criterion != OG_OPEN_BH && p->criterion != OG_OPEN_RELATIVE)
    return fail(OG_EINVAL, "unknown opening criterion %d", p->criterion);
  if (p->criterion == OG_OPEN_RELATIVE && !(p->alpha > 0.0 && std::isfinite(p->alpha)))
    return fail(OG_EINVAL, "the relative criterion needs alpha > 0");
  if (!std::isfinite(p->r_s) || !std::isfinite(p->r_cut) || p->r_cut < 0.0)
    return fail(OG_EINVAL, "r_s / r_cut invalid");
  const double rcut = p->r_cut > 0.0 ? p->r_cut : 4.5 * p->r_s;
  if (p->periodic) {
    if (!(p->r_s > 0.0)) return fail(OG_EINVAL, "periodic boxes need r_s > 0 (short-range force)");
    if (!(rcut < 0.5 * box)) return fail(OG_EINVAL, "r_cut must be < box/2 in a periodic box");
  } else if (p->r_s > 0.0 && !(rcut > 0.0)) {
    return fail(OG_EINVAL, "r_cut must be > 0");
  }
  return OG_OK;
}

void fill_box(BoxDev &b, const double *pos, const double *mass, int64_t N, double box, const og_params &p,
              uint32_t p_off) {
  std::memset(&b, 0, sizeof(b));
  b.pos = pos;
  b.mass = mass;
  b.box = box;
  b.periodic = p.periodic ? 1 : 0;
  b.cutoff = p.r_s > 0.0 ? 1 : 0;
  b.leaf_max = p.leaf_max;
  b.p_off = p_off;
  b.n = (uint32_t)N;
  b.G = p.G;
  b.eps2 = p.eps * p.eps;
  b.r_s = p.r_s;
  b.rcut = p.r_cut > 0.0 ? p.r_cut : 4.5 * p.r_s;
  b.rc2 = b.rcut * b.rcut;
  b.theta2 = p.theta * p.theta;
  b.Gf = (float)p.G;
  b.eps2f = (float)b.eps2;
  b.inv2rsf = b.cutoff ? (float)(1.0 / (2.0 * p.r_s)) : 0.0f;
  b.rcutf = (float)b.rcut;
  b.rc2f = (float)b.rc2;
  b.theta2f = (float)b.theta2;
  b.spline = p.softening == OG_SOFT_SPLINE ? 1 : 0;
  b.relative = p.criterion == OG_OPEN_RELATIVE ? 1 : 0;
  b.hs = 2.8 * p.eps;
  b.alpha = p.alpha;
  b.hsf = (float)b.hs;
  b.hinvf = b.spline ? (float)(1.0 / b.hs) : 0.0f;
  b.curve = p.curve == OG_CURVE_HILBERT ? 1 : 0;
  b.epsp = p.eps_particle;
  b.eps = p.eps;
  if (b.periodic) {
    b.lo[0] = b.lo[1] = b.lo[2] = 0.0;
    b.L = box;
  } else {  // set on the device from the bounding cube
    b.L = 1.0;
  }
  b.scale = 2097152.0 / b.L;
  b.Lf = (float)b.L;
  b.h22f = (float)(b.L * 0x1p-22);
}

// --------------------------------------------------------- forest --
int Forest::init(const std::vector<BoxDev> &boxes, uint64_t node_cap_, hipStream_t s, int prec, int gmax,
                 void *workspace, size_t ws_bytes) {
  B = (int)boxes.size();
  uint64_t ntot = 0;
  for (auto &b : boxes) ntot += b.n;
  if (ntot > kCountMask) return fail(OG_EINVAL, "total particle count %llu exceeds 2^27-1", (unsigned long long)ntot);
  // the walks tell a leaf's record from an internal node's by the sign bit
  // of the skip / tag word, so node indices stay below 2^31
  if (node_cap_ > 0x7fffffffull) return fail(OG_EINVAL, "node bound too large");
  N = (uint32_t)ntot;
  node_cap = (uint32_t)node_cap_;
  stream = s;
  precision = prec;
  group_max = gmax > 0 ? (uint32_t)gmax : 64u;
  hboxes = boxes;
  // walk groups: chunks of group_max consecutive sorted particles per box
  uint64_t gtot = 0;
  for (auto &b : hboxes) {
    b.g_off = (uint32_t)gtot;
    gtot += (b.n + group_max - 1) / group_max;
  }
  n_groups = (uint32_t)gtot;
  bool soft = false;
  for (auto &b : hboxes) soft |= b.epsp != nullptr;
  bytes = forest_bytes(N, node_cap, B, soft);
  if (workspace) {
    if (!is_device_ptr(workspace)) return fail(OG_EINVAL, "workspace is not device memory");
    if (ws_bytes < bytes) return fail(OG_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, bytes);
    mem = workspace;
    own = false;
  } else {
    if (fault_fires(kFaultAlloc)) return fail(OG_ENOMEM, "forced failure of the tree allocation (OG_FAULT_ALLOC)");
    hipError_t e = hipMalloc(&mem, bytes);
    if (e != hipSuccess) {
      mem = nullptr;
      return hip_fail(e, "hipMalloc(tree)");
    }
    own = true;
  }
  Carver c;
  c.base = static_cast<char *>(mem);
  carve(c, A, N, node_cap, B, soft);
  A.B = B;
  A.n = N;
  A.node_cap = node_cap;
  A.any_open = 0;
  A.leaf_max = 1;
  for (auto &b : hboxes) {
    A.any_open |= b.periodic ? 0 : 1;
    A.leaf_max = std::max(A.leaf_max, (int)b.leaf_max);
  }
  hipError_t e = hipMemcpyAsync(A.boxes, hboxes.data(), sizeof(BoxDev) * B, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(boxes)");
  return OG_OK;
}

int Forest::build() {
  if (fault_fires(kFaultLaunch)) return fail(OG_EDEVICE, "forced failure of the build launch (OG_FAULT_LAUNCH)");
  launch_build(A, stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "build launch");
  return OG_OK;
}

WalkArgs Forest::walk_args() const {
  WalkArgs W{};
  W.boxes = A.boxes;
  W.topo = A.topo;
  W.mom32 = A.mom32;
  W.wnode = A.wnode;
  W.cen64 = A.cen64;
  W.mom64 = A.mom64;
  W.part32 = A.part32;
  W.part64 = A.part64;
  W.perm = A.perm;
  W.skeys = A.keys_a;
  W.chunk = group_max;
  W.list_cap = list_cap;
  W.B = B;
  auto kind = [](const BoxDev &b) { return b.cutoff ? (b.periodic ? 2 : 1) : 3; };
  W.box_kind = kind(hboxes[0]);
  for (const auto &b : hboxes) {
    if (kind(b) != W.box_kind) W.box_kind = 0;
    if (b.spline || b.relative) W.ext = 1;
  }
  W.counter = &A.scalars[8];
  W.group_lists = group_lists;
  W.seps = A.seps;
  W.semax = A.semax;
  W.semin = A.semin;
  if (A.seps) W.ext = 1;
  W.wide_nodes = (uint64_t)node_cap * sizeof(WNode) > 0xffffffffull ? 1 : 0;
  // u = r / (2 r_s) < r_cut / (2 r_s) for every pair term (r < r_cut); a margin
  // covers the rounding of u
  for (const auto &b : hboxes)
    if (b.cutoff && !(b.rcut * (0.5 / b.r_s) < 2.99)) W.erfc_tail = 1;
  return W;
}

int Forest::walk_all(int prec, hipStream_t s, double *acc, double *pot, int pot_override, int64_t *nint,
                     const double *a_old) {
  if (fault_fires(kFaultLaunch)) return fail(OG_EDEVICE, "forced failure of the walk launch (OG_FAULT_LAUNCH)");
  WalkArgs W = walk_args();
  W.a_old = a_old;
  W.n_groups = n_groups;
  W.acc = acc;
  W.pot = pot;
  W.pot_override = pot_override;
  W.nint = nint;
  launch_walk(W, prec, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "walk launch");
  return OG_OK;
}

// Carve the scratch of a subset walk of M targets from `base` (null: only
// measure); returns its size in bytes.
size_t subset_plan(TargetArrays &T, uint32_t M, char *base) {
  Carver c;
  c.base = base;
  T.tkey_a = c.take<uint64_t>(M);
  T.tkey_b = c.take<uint64_t>(M);
  T.tval_a = c.take<uint32_t>(M);
  T.tval_b = c.take<uint32_t>(M);
  T.hist = c.take<uint32_t>(radix_hist_words(M));
  T.digit_tot = c.take<uint32_t>(256);
  T.scalars = c.take<uint32_t>(32);
  return c.off + 256;
}

int Forest::walk_subset_in(int prec, hipStream_t s, const int64_t *idx, uint32_t M, double *acc, double *pot,
                           int64_t *nint, const double *a_old, void *scratch) {
  TargetArrays T{};
  subset_plan(T, M, static_cast<char *>(scratch));
  T.idx = idx;
  T.M = M;
  launch_targets(A, T, s);
  WalkArgs W = walk_args();
  W.n_groups = (M + group_max - 1) / group_max;
  W.n_targets = M;
  W.counter = &T.scalars[8];
  W.tkey = T.tkey;
  W.tval = T.tval;
  W.acc = acc;
  W.pot = pot;
  W.pot_override = 1;
  W.nint = nint;
  W.a_old = a_old;
  launch_walk(W, prec, s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "walk launch (targets)");
  return OG_OK;
}

int Forest::walk_subset(int prec, hipStream_t s, const int64_t *idx, uint32_t M, double *acc, double *pot,
                        int64_t *nint, const double *a_old) {
  TargetArrays T{};
  const size_t bytes = subset_plan(T, M, nullptr);
  if (fault_fires(kFaultLaunch)) return fail(OG_EDEVICE, "forced failure of the walk launch (OG_FAULT_LAUNCH)");
  if (fault_fires(kFaultAlloc)) return fail(OG_ENOMEM, "forced failure of the target scratch (OG_FAULT_ALLOC)");
  void *tmp = nullptr;
  hipError_t e = hipMallocAsync(&tmp, bytes, s);
  if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(targets)");
  const int rc = walk_subset_in(prec, s, idx, M, acc, pot, nint, a_old, tmp);
  e = hipFreeAsync(tmp, s);
  if (rc != OG_OK) return rc;
  if (e != hipSuccess) return hip_fail(e, "hipFreeAsync(targets)");
  return OG_OK;
}

int Forest::walk_active(int prec, hipStream_t s, const int8_t *bin, int32_t level, double *acc, double *pot,
                        int64_t *nint, const double *a_old, int64_t *n_active) {
  ActiveArrays T{};
  auto plan = [&](Carver &cv) {
    T.flags = cv.take<uint32_t>(N);
    T.offs = cv.take<uint32_t>((size_t)N + 1);
    T.partial = cv.take<uint32_t>(scan_partial_words(N));
    T.tkey = cv.take<uint64_t>(N);
    T.tval = cv.take<uint32_t>(N);
    T.counts = cv.take<uint32_t>(32);
  };
  Carver c;
  plan(c);
  if (fault_fires(kFaultLaunch)) return fail(OG_EDEVICE, "forced failure of the walk launch (OG_FAULT_LAUNCH)");
  if (fault_fires(kFaultAlloc)) return fail(OG_ENOMEM, "forced failure of the active-set scratch (OG_FAULT_ALLOC)");
  void *tmp = nullptr;
  hipError_t e = hipMallocAsync(&tmp, c.off + 256, s);
  if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(active)");
  Carver c2;
  c2.base = static_cast<char *>(tmp);
  plan(c2);
  T.bin = bin;
  T.level = level;
  T.n_active = n_active;
  launch_active(A, T, group_max, s);
  WalkArgs W = walk_args();
  W.n_groups = (N + group_max - 1) / group_max;  // bound for the grid; the count is read on the device
  W.n_targets = N;
  W.dev_count = T.counts;
  W.counter = &T.counts[8];
  W.tkey = T.tkey;
  W.tval = T.tval;
  W.acc = acc;
  W.pot = pot;
  W.pot_override = 1;
  W.nint = nint;
  W.a_old = a_old;
  launch_walk(W, prec, s);
  e = hipGetLastError();
  hipError_t e2 = hipFreeAsync(tmp, s);
  if (e != hipSuccess) return hip_fail(e, "walk launch (active)");
  if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync(active)");
  return OG_OK;
}

int Forest::read_status(hipStream_t s) {
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  uint32_t st = 0;
  e = hipMemcpy(&st, &A.scalars[0], sizeof(st), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(status)");
  if (st & kStatusRange) return fail(OG_ERANGE, "a position lies outside [0, box) or is not finite");
  if (st & kStatusNodes) return fail(OG_EDEVICE, "node bound exceeded");
  if (st & kStatusTarget) return fail(OG_ERANGE, "a target index lies outside [0, N)");
  return OG_OK;
}

int order_after(hipStream_t waiter, hipStream_t producer) {
  if (waiter == producer) return OG_OK;
  hipEvent_t ev;
  hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  e = hipEventRecord(ev, producer);
  if (e == hipSuccess) e = hipStreamWaitEvent(waiter, ev, 0);
  (void)hipEventDestroy(ev);  // released once the wait is satisfied
  if (e != hipSuccess) return hip_fail(e, "stream ordering");
  return OG_OK;
}

// Release paths ignore HIP errors: there is nothing left to report them to.
void Forest::release() {
  if (gexec) {
    (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
  }
  if (own_stream) {
    (void)hipStreamDestroy(own_stream);
    own_stream = nullptr;
  }
  if (mem && own) (void)hipFree(mem);
  mem = nullptr;
}

}  // namespace og

// ------------------------------------------- allocation-free subset walk --
// og_tree_force_noalloc takes the target list's scratch (sorted keys and
// slots with their sort ping-pong, histograms, queue counters) from this
// array instead of a stream-ordered allocation.  Every buffer in it is
// written or reset by the kernels of each call before it is read.  Host
// code reaches the array only through the address hipGetSymbolAddress
// gives for the current device (its name stands for a host-side shadow).
namespace {
constexpr uint32_t kNoAllocTargets = OG_NOALLOC_MAX_TARGETS;
constexpr size_t noalloc_align(size_t x) { return (x + 255) & ~(size_t)255; }
// the sizes subset_plan carves for M targets, each 256-byte aligned
constexpr size_t noalloc_bytes(size_t M) {
  const size_t parts[7] = {8 * M, 8 * M, 4 * M, 4 * M, 4 * 256 * ((M + kSortTile - 1) / kSortTile), 4 * 256, 4 * 32};
  size_t off = 0;
  for (size_t p : parts) off = noalloc_align(off) + p;
  return off + 256;
}
constexpr size_t kNoAllocBytes = noalloc_bytes(kNoAllocTargets);
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// The device address of `scratch` on the current device, looked up on the
// first call there.
int scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(OG_EDEVICE, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    TargetArrays T{};
    if (subset_plan(T, kNoAllocTargets, nullptr) > kNoAllocBytes)
      return fail(OG_EDEVICE, "allocation-free scratch smaller than its plan");
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return OG_OK;
}
}  // namespace

// ================================================================= ABI ==
struct og_batch {
  Forest F;
  std::vector<og_box> boxes;
};

void og::tree_free_nosync(og_tree *t) {
  if (!t) return;
  t->F.release();
  delete t;
}

extern "C" {

void og_params_default(og_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(og_params);
  p->G = 1.0;
  p->theta = 0.5;
  p->periodic = 1;
  p->leaf_max = 8;
  p->precision = OG_PREC_MIXED;
}

size_t og_tree_workspace_bound(int64_t N, const og_params *p) {
  if (!p || p->struct_size != sizeof(og_params) || N < 1 || N > (int64_t)kCountMask || p->leaf_max < 1 ||
      p->leaf_max > 4096)
    return 0;
  return forest_bytes((uint32_t)N, (uint32_t)node_bound((uint64_t)N, p->leaf_max), 1, p->eps_particle != nullptr);
}

int og_tree_build(const double *pos, const double *mass, int64_t N, double box, const og_params *params,
                  og_tree **out) {
  const TraceRange trace_range("og_tree_build");
  if (!out) return fail(OG_EINVAL, "out is NULL");
  int rc = check_params(params, N, box, true);
  if (rc) return rc;
  if (!is_device_ptr(pos) || !is_device_ptr(mass)) return fail(OG_EINVAL, "pos/mass must be device pointers");
  og_tree *t = new (std::nothrow) og_tree();
  if (!t) return fail(OG_ENOMEM, "host allocation");
  std::vector<BoxDev> boxes(1);
  fill_box(boxes[0], pos, mass, N, box, *params, 0);
  t->F.list_cap = params->walk_list_cap;
  t->F.group_lists = params->lists == OG_LISTS_GROUP ? 1 : 0;
  rc = t->F.init(boxes, node_bound((uint64_t)N, params->leaf_max), (hipStream_t)params->stream,
                 params->precision, params->group_max, params->workspace, params->workspace_bytes);
  if (rc == OG_OK) rc = t->F.build();
  if (rc != OG_OK) {
    t->F.release();
    delete t;
    return rc;
  }
  *out = t;
  return OG_OK;
}

int og_tree_force_ex(const og_tree *tree, const og_targets *targets, const og_force_opts *opts, double *acc,
                     double *pot) {
  const TraceRange trace_range("og_tree_force");
  if (!tree) return fail(OG_EINVAL, "tree is NULL");
  og_tree *t = const_cast<og_tree *>(tree);
  Forest &F = t->F;
  int prec = F.precision;
  hipStream_t s = F.stream;
  int64_t *nint = nullptr;
  const double *a_old = nullptr;
  if (opts) {
    if (opts->struct_size != sizeof(og_force_opts)) return fail(OG_EINVAL, "og_force_opts.struct_size mismatch");
    if (opts->precision >= 0) {
      if (opts->precision != OG_PREC_FP64 && opts->precision != OG_PREC_MIXED)
        return fail(OG_EINVAL, "unknown precision %d", opts->precision);
      prec = opts->precision;
    }
    if (opts->stream) s = (hipStream_t)opts->stream;
    nint = opts->n_inter;
    if (nint && !is_device_ptr(nint)) return fail(OG_EINVAL, "n_inter must be a device pointer");
    a_old = opts->a_old;
  }
  if (F.hboxes[0].relative) {
    if (!a_old) return fail(OG_EINVAL, "the relative criterion needs a_old (og_force_opts)");
    if (!is_device_ptr(a_old)) return fail(OG_EINVAL, "a_old must be a device pointer");
  } else {
    a_old = nullptr;
  }
  if (!is_device_ptr(acc)) return fail(OG_EINVAL, "acc must be a device pointer");
  if (pot && !is_device_ptr(pot)) return fail(OG_EINVAL, "pot must be a device pointer");
  {
    const int rc = order_after(s, F.stream);  // after the build on the tree's stream
    if (rc != OG_OK) return rc;
  }
  if (!targets || !targets->idx) {
    if (targets && targets->M != (int64_t)F.N)
      return fail(OG_EINVAL, "targets->idx NULL requires M == N");
    return F.walk_all(prec, s, acc, pot, 1, nint, a_old);
  }
  if (targets->M < 1 || targets->M > (int64_t)kCountMask) return fail(OG_EINVAL, "targets->M out of range");
  if (!is_device_ptr(targets->idx)) return fail(OG_EINVAL, "targets->idx must be a device pointer");
  return F.walk_subset(prec, s, targets->idx, (uint32_t)targets->M, acc, pot, nint, a_old);
}

int og_tree_force(const og_tree *tree, const og_targets *targets, double *acc, double *pot) {
  return og_tree_force_ex(tree, targets, nullptr, acc, pot);
}

int og_tree_force_noalloc(const og_tree *tree, const og_targets *targets, double *acc, double *pot) {
  const TraceRange trace_range("og_tree_force_noalloc");
  if (!tree) return fail(OG_EINVAL, "tree is NULL");
  og_tree *t = const_cast<og_tree *>(tree);
  Forest &F = t->F;
  if (F.hboxes[0].relative) return fail(OG_EINVAL, "the relative criterion needs a_old (og_tree_force_ex)");
  if (!is_device_ptr(acc)) return fail(OG_EINVAL, "acc must be a device pointer");
  if (pot && !is_device_ptr(pot)) return fail(OG_EINVAL, "pot must be a device pointer");
  if (!targets || !targets->idx) {  // every particle: the tree's own workspace suffices
    if (targets && targets->M != (int64_t)F.N)
      return fail(OG_EINVAL, "targets->idx NULL requires M == N");
    return F.walk_all(F.precision, F.stream, acc, pot, 1, nullptr);
  }
  if (targets->M < 1) return fail(OG_EINVAL, "targets->M out of range");
  if (targets->M > (int64_t)kNoAllocTargets)
    return fail(OG_EINVAL, "targets->M = %lld exceeds the allocation-free limit of %u targets",
                (long long)targets->M, kNoAllocTargets);
  if (!is_device_ptr(targets->idx)) return fail(OG_EINVAL, "targets->idx must be a device pointer");
  void *scr = nullptr;
  const int rc = scratch_address(&scr);
  if (rc != OG_OK) return rc;
  return F.walk_subset_in(F.precision, F.stream, targets->idx, (uint32_t)targets->M, acc, pot, nullptr,
                          nullptr, scr);
}

int og_tree_force_active(const og_tree *tree, const int8_t *bin, int32_t level, const og_force_opts *opts,
                         double *acc, double *pot, int64_t *n_active) {
  const TraceRange trace_range("og_tree_force_active");
  if (!tree) return fail(OG_EINVAL, "tree is NULL");
  og_tree *t = const_cast<og_tree *>(tree);
  Forest &F = t->F;
  int prec = F.precision;
  hipStream_t s = F.stream;
  int64_t *nint = nullptr;
  const double *a_old = nullptr;
  if (opts) {
    if (opts->struct_size != sizeof(og_force_opts)) return fail(OG_EINVAL, "og_force_opts.struct_size mismatch");
    if (opts->precision >= 0) {
      if (opts->precision != OG_PREC_FP64 && opts->precision != OG_PREC_MIXED)
        return fail(OG_EINVAL, "unknown precision %d", opts->precision);
      prec = opts->precision;
    }
    if (opts->stream) s = (hipStream_t)opts->stream;
    nint = opts->n_inter;
    a_old = opts->a_old;
  }
  if (!is_device_ptr(bin)) return fail(OG_EINVAL, "bin must be a device pointer");
  if (!is_device_ptr(acc)) return fail(OG_EINVAL, "acc must be a device pointer");
  if (pot && !is_device_ptr(pot)) return fail(OG_EINVAL, "pot must be a device pointer");
  if (nint && !is_device_ptr(nint)) return fail(OG_EINVAL, "n_inter must be a device pointer");
  if (n_active && !is_device_ptr(n_active)) return fail(OG_EINVAL, "n_active must be a device pointer");
  if (F.hboxes[0].relative) {
    if (!a_old) return fail(OG_EINVAL, "the relative criterion needs a_old (og_force_opts)");
    if (!is_device_ptr(a_old)) return fail(OG_EINVAL, "a_old must be a device pointer");
  } else {
    a_old = nullptr;
  }
  {
    const int rc = order_after(s, F.stream);
    if (rc != OG_OK) return rc;
  }
  return F.walk_active(prec, s, bin, level, acc, pot, nint, a_old, n_active);
}

int og_tree_status(const og_tree *tree) {
  if (!tree) return fail(OG_EINVAL, "tree is NULL");
  return const_cast<og_tree *>(tree)->F.read_status(tree->F.stream);
}

int og_tree_stats(const og_tree *tree, int64_t *n_nodes, int32_t *depth, size_t *bytes) {
  if (!tree) return fail(OG_EINVAL, "tree is NULL");
  Forest &F = const_cast<og_tree *>(tree)->F;
  if (depth) launch_max_level(F.A, &F.A.scalars[5], F.stream);
  hipError_t e = hipStreamSynchronize(F.stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  uint32_t sc[8];
  e = hipMemcpy(sc, F.A.scalars, sizeof(sc), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(scalars)");
  if (n_nodes) *n_nodes = sc[3];
  if (depth) *depth = (int32_t)sc[5];
  if (bytes) *bytes = F.bytes;
  return OG_OK;
}

int og_tree_export(const og_tree *tree, uint64_t *keys, uint32_t *perm, uint32_t *first, uint32_t *count,
                   uint8_t *level, uint32_t *skip, uint32_t *parent, double *node_m_com) {
  if (!tree) return fail(OG_EINVAL, "tree is NULL");
  Forest &F = const_cast<og_tree *>(tree)->F;
  hipError_t e = hipStreamSynchronize(F.stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  uint32_t nn = 0;
  e = hipMemcpy(&nn, &F.A.scalars[3], sizeof(nn), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  const uint32_t N = F.N;
  auto cp = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
    if (!dst) return hipSuccess;
    return hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
  };
  if ((e = cp(keys, F.A.keys_a, 8ull * N)) != hipSuccess) return hip_fail(e, "export keys");
  if ((e = cp(perm, F.A.perm, 4ull * N)) != hipSuccess) return hip_fail(e, "export perm");
  if ((e = cp(first, F.A.first, 4ull * nn)) != hipSuccess) return hip_fail(e, "export first");
  if ((e = cp(skip, F.A.skip, 4ull * nn)) != hipSuccess) return hip_fail(e, "export skip");
  if ((e = cp(parent, F.A.parent, 4ull * nn)) != hipSuccess) return hip_fail(e, "export parent");
  if (count || level) {
    std::vector<Topo> tp(nn);
    if ((e = cp(tp.data(), F.A.topo, sizeof(Topo) * nn)) != hipSuccess) return hip_fail(e, "export topo");
    for (uint32_t r = 0; r < nn; ++r) {
      if (count) count[r] = tp[r].b & kCountMask;
      if (level) level[r] = (uint8_t)(tp[r].b >> kCountBits);
    }
  }
  if (node_m_com) {
    std::vector<Mom64> m(nn);
    if ((e = cp(m.data(), F.A.mom64, sizeof(Mom64) * nn)) != hipSuccess) return hip_fail(e, "export moments");
    for (uint32_t r = 0; r < nn; ++r) {
      node_m_com[4ull * r] = m[r].m;
      node_m_com[4ull * r + 1] = m[r].cx;
      node_m_com[4ull * r + 2] = m[r].cy;
      node_m_com[4ull * r + 3] = m[r].cz;
    }
  }
  return OG_OK;
}

int og_tree_free(og_tree *tree) {
  if (!tree) return OG_OK;
  (void)hipStreamSynchronize(tree->F.stream);
  tree->F.release();
  delete tree;
  return OG_OK;
}

// ---------------------------------------------------------------- batch --
int og_batch_build(const og_box *boxes, int32_t B, void *stream, og_batch **out) {
  const TraceRange trace_range("og_batch_build");
  if (!out || !boxes) return fail(OG_EINVAL, "NULL argument");
  if (B < 1 || B > 65536) return fail(OG_EINVAL, "B = %d outside 1..65536", B);
  std::vector<BoxDev> hb(B);
  uint64_t off = 0, cap = 0;
  for (int b = 0; b < B; ++b) {
    const og_box &x = boxes[b];
    int rc = check_params(&x.params, x.N, x.box, false);
    if (rc) return fail(rc, "box %d: %s", b, og_last_error());
    if (!is_device_ptr(x.pos) || !is_device_ptr(x.mass) || !is_device_ptr(x.acc) ||
        (x.pot && !is_device_ptr(x.pot)))
      return fail(OG_EINVAL, "box %d: pos/mass/acc/pot must be device pointers", b);
    if (x.params.criterion == OG_OPEN_RELATIVE)
      return fail(OG_EUNSUPPORTED, "box %d: the relative criterion needs a_old, not available in a batch", b);
    if (x.params.precision != boxes[0].params.precision || x.params.group_max != boxes[0].params.group_max ||
        x.params.walk_list_cap != boxes[0].params.walk_list_cap || x.params.lists != boxes[0].params.lists)
      return fail(OG_EINVAL, "box %d: precision, group_max, walk_list_cap and lists must match box 0", b);
    if (off + (uint64_t)x.N > kCountMask) return fail(OG_EINVAL, "batch exceeds 2^27-1 particles");
    fill_box(hb[b], x.pos, x.mass, x.N, x.box, x.params, (uint32_t)off);
    hb[b].acc = x.acc;
    hb[b].pot = x.pot;
    off += (uint64_t)x.N;
    cap += node_bound((uint64_t)x.N, x.params.leaf_max);
  }
  og_batch *bt = new (std::nothrow) og_batch();
  if (!bt) return fail(OG_ENOMEM, "host allocation");
  bt->boxes.assign(boxes, boxes + B);
  bt->F.list_cap = boxes[0].params.walk_list_cap;
  bt->F.group_lists = boxes[0].params.lists == OG_LISTS_GROUP ? 1 : 0;
  int rc = bt->F.init(hb, cap, (hipStream_t)stream, boxes[0].params.precision, boxes[0].params.group_max,
                      nullptr, 0);
  if (rc == OG_OK) rc = bt->F.build();
  if (rc != OG_OK) {
    bt->F.release();
    delete bt;
    return rc;
  }
  *out = bt;
  return OG_OK;
}

int og_batch_force(og_batch *b) {
  const TraceRange trace_range("og_batch_force");
  if (!b) return fail(OG_EINVAL, "batch is NULL");
  return b->F.walk_all(b->F.precision, b->F.stream, nullptr, nullptr, 0, nullptr);
}

int og_batch_graph_replay(og_batch *b) {
  const TraceRange trace_range("og_batch_graph_replay");
  if (!b) return fail(OG_EINVAL, "batch is NULL");
  Forest &F = b->F;
  hipStream_t cs = F.stream;
  hipError_t e;
  if (!cs) {
    if (!F.own_stream) {
      e = hipStreamCreateWithFlags(&F.own_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    }
    cs = F.own_stream;
  }
  if (!F.gexec) {
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipStream_t keep = F.stream;
    F.stream = cs;
    int rc1 = F.build();
    int rc2 = F.walk_all(F.precision, cs, nullptr, nullptr, 0, nullptr);
    F.stream = keep;
    e = hipStreamEndCapture(cs, &g);
    if (rc1 || rc2) {
      if (g) (void)hipGraphDestroy(g);
      return rc1 ? rc1 : rc2;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&F.gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      F.gexec = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
  }
  if (cs != F.stream) {  // order the private stream after the caller's stream and back
    int rc = order_after(cs, F.stream);
    if (rc != OG_OK) return rc;
    e = hipGraphLaunch(F.gexec, cs);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return order_after(F.stream, cs);
  }
  e = hipGraphLaunch(F.gexec, cs);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return OG_OK;
}

int og_batch_status(const og_batch *b) {
  if (!b) return fail(OG_EINVAL, "batch is NULL");
  Forest &F = const_cast<og_batch *>(b)->F;
  if (F.own_stream) {
    hipError_t e = hipStreamSynchronize(F.own_stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  }
  return F.read_status(F.stream);
}

int og_batch_free(og_batch *b) {
  if (!b) return OG_OK;
  (void)hipStreamSynchronize(b->F.stream);
  if (b->F.own_stream) (void)hipStreamSynchronize(b->F.own_stream);
  b->F.release();
  delete b;
  return OG_OK;
}

const char *og_strerror(int code) {
  switch (code) {
    case OG_OK: return "ok";
    case OG_EINVAL: return "invalid argument";
    case OG_ERANGE: return "position out of range";
    case OG_ENOMEM: return "out of device memory";
    case OG_EDEVICE: return "device error";
    case OG_EBUSY: return "busy";
    case OG_EUNSUPPORTED: return "unsupported";
    case OG_ENOTFOUND: return "not found";
    case OG_ECORRUPT: return "tree invariant violated";
    default: return "unknown error";
  }
}

const char *og_last_error(void) { return og::g_last_error.c_str(); }

}  // extern "C"
