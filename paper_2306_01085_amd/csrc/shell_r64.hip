// The element pass of the FP64 residual R(u) on the cubed-sphere shell (every launch
// configuration and extended-physics mode), in a translation unit of its own so that it
// can be compiled with its own code-generation options; the kernel is in shell_pass1.h.
#include "shell_pass1.h"

namespace dg {

void shell_pass1_f64(dg_mesh_s* m, const ShellDev& M, const PhysC& ph, const GllC& gc, double t, const double* u,
                     double* out, double* fn, hipStream_t s, int pid) {
  const double* none = nullptr;
  switch (m->p) {
    case 2: dispatch_p1<2, double>(m, M, ph, gc, t, u, none, out, fn, s, pid); break;
    case 3: dispatch_p1<3, double>(m, M, ph, gc, t, u, none, out, fn, s, pid); break;
    case 4: dispatch_p1<4, double>(m, M, ph, gc, t, u, none, out, fn, s, pid); break;
    default: break;   // the caller has rejected other degrees
  }
}

}  // namespace dg
