// server.cpp -- continuous-batching server (placeholder until implemented).
#include "dg_internal.h"
#include "solver_impl.h"

using namespace dg;

extern "C" {
dg_status dg_server_create(void *, size_t, size_t, int32_t, void *, void *, dg_server **out) {
  if (out) *out = nullptr;
  return fail(DG_EINVAL, "server not available in this build");
}
dg_status dg_server_submit(dg_server *, const dg_params *, const dg_mesh *, const double *, int32_t, double, double,
                           int64_t *) {
  return fail(DG_EINVAL, "server not available in this build");
}
dg_status dg_server_run(dg_server *, int32_t) { return fail(DG_EINVAL, "server not available in this build"); }
dg_status dg_server_poll(dg_server *, int64_t, int32_t *) { return fail(DG_EINVAL, "server not available"); }
dg_status dg_server_fetch(dg_server *, int64_t, double *, dg_timing *) { return fail(DG_EINVAL, "server not available"); }
void dg_server_destroy(dg_server *) {}
}
