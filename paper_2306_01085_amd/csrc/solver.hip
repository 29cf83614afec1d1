// Implicit DIRK stages solved by Newton-GMRES (sections 3.1, 3.2).
#include "internal.h"

namespace dg {

struct Workspace {};

void free_workspace(dg_mesh_s* m) {
  delete m->ws;
  m->ws = nullptr;
}

dg_status_t implicit_step(dg_mesh_s* m, double t, double dt, double* u, const dg_solver_opts_t& o,
                          dg_step_stats_t* st, hipStream_t s) {
  (void)m; (void)t; (void)dt; (void)u; (void)o; (void)st; (void)s;
  set_error("dg_implicit_step: not built yet");
  return DG_ERR_UNSUPPORTED;
}

}  // namespace dg
