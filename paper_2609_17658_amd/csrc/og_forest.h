// Host-side tree object shared by the single-tree, batch and server entry
// points: owns (or borrows) one device allocation carved into the arrays of
// BuildArrays, and launches build and walk on a stream.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/og.h"
#include "og_kernels.h"

namespace og {
struct Forest;
}

namespace og {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
// Make `waiter` wait for the work enqueued so far on `producer` (no-op when
// they are the same stream).  OG_OK or OG_EDEVICE.
int order_after(hipStream_t waiter, hipStream_t producer);
bool is_device_ptr(const void *p);
// Host-forced faults, for tests of the error paths; nothing is enqueued when
// one fires.  OG_FAULT_ALLOC=k makes the k-th device allocation of the
// library (tree workspace, server arena, a served request's admission,
// target and active-set scratch, mesh) fail with OG_ENOMEM; OG_FAULT_LAUNCH=k
// makes the k-th enqueue of a build or a walk fail with OG_EDEVICE.  The
// count restarts whenever the variable's value changes.  (og_tree_validate
// has its own knob, OG_FAULT_CORRUPT, which edits its host copy only.)
enum FaultKind { kFaultAlloc = 0, kFaultLaunch = 1 };
bool fault_fires(FaultKind k);
int check_params(const og_params *p, int64_t N, double box, bool need_stream_fields);
void fill_box(BoxDev &b, const double *pos, const double *mass, int64_t N, double box, const og_params &p,
              uint32_t p_off);
uint64_t node_bound(uint64_t n, int leaf_max);
size_t forest_bytes(uint32_t n, uint32_t node_cap, int B, bool soft);
// Scratch of a walk over M listed targets, carved from `base` (null: only
// measure); returns its size in bytes.
size_t subset_plan(TargetArrays &T, uint32_t M, char *base);

struct Forest {
  int B = 0;
  uint32_t N = 0;
  uint32_t node_cap = 0;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;  // private capture stream when `stream` is the null stream
  int precision = OG_PREC_MIXED;
  uint32_t group_max = 64;
  uint32_t n_groups = 0;
  int list_cap = 0;  // mixed walk list capacity (0 = default)
  int group_lists = 0;  // group-shared interaction lists
  void *mem = nullptr;
  size_t bytes = 0;
  bool own = false;
  std::vector<BoxDev> hboxes;
  BuildArrays A{};
  hipGraphExec_t gexec = nullptr;

  int init(const std::vector<BoxDev> &boxes, uint64_t node_cap, hipStream_t s, int prec, int gmax,
           void *workspace, size_t ws_bytes);
  int build();
  WalkArgs walk_args() const;
  int walk_all(int prec, hipStream_t s, double *acc, double *pot, int pot_override, int64_t *nint,
               const double *a_old = nullptr);
  int walk_subset(int prec, hipStream_t s, const int64_t *idx, uint32_t M, double *acc, double *pot,
                  int64_t *nint, const double *a_old = nullptr);
  // The same walk with its target scratch (subset_plan bytes) given.
  int walk_subset_in(int prec, hipStream_t s, const int64_t *idx, uint32_t M, double *acc, double *pot,
                     int64_t *nint, const double *a_old, void *scratch);
  int walk_active(int prec, hipStream_t s, const int8_t *bin, int32_t level, double *acc, double *pot,
                  int64_t *nint, const double *a_old, int64_t *n_active);
  int read_status(hipStream_t s);
  void release();
};

// Free a tree whose queued work is known to be complete (no stream sync).
void tree_free_nosync(og_tree *t);

}  // namespace og

// A single tree (og_tree_* entry points): one forest of one box.
struct og_tree {
  og::Forest F;
};
