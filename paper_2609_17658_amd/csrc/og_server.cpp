// Serving entry points (continuous batching over resident trees).
#include <hip/hip_runtime.h>

#include "og_forest.h"

using namespace og;

extern "C" {
int og_server_create(size_t, int32_t, og_server **) { return fail(OG_EUNSUPPORTED, "server not built"); }
int og_server_submit(og_server *, const og_box *, uint64_t *) { return fail(OG_EUNSUPPORTED, "server not built"); }
int og_server_progress(og_server *) { return fail(OG_EUNSUPPORTED, "server not built"); }
int og_server_poll(og_server *, uint64_t, int32_t *, double *, double *) {
  return fail(OG_EUNSUPPORTED, "server not built");
}
int og_server_wait(og_server *, uint64_t) { return fail(OG_EUNSUPPORTED, "server not built"); }
int og_server_release(og_server *, uint64_t) { return fail(OG_EUNSUPPORTED, "server not built"); }
int og_server_stats(const og_server *, size_t *, int32_t *, int32_t *) {
  return fail(OG_EUNSUPPORTED, "server not built");
}
int og_server_destroy(og_server *) { return OG_OK; }
}
