"""FP64 CPU oracle of the thermosphere DG hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, literal implementation of what the GPU library computes, written
from the paper (Vila-Perez, Nguyen, Peraire, "A high-order discontinuous Galerkin
approach for physics-based thermospheric modeling"):

* gll       -- Gauss-Lobatto-Legendre nodes, weights, differentiation (section 3.1 spaces)
* physics   -- pointwise fluxes and sources of eq. (fluxSWNondimensional) with the
               acceleration of section 2.5 and the transport laws of section 2.1.2
* mesh      -- 1D radial columns and the cubed-sphere shell of section 3.3
* dg        -- the LDG weak form eq. (DGformulation) with traces eq. (LDG2)
* jac       -- J(u)v by complex step and by finite differences (section 3.2)
* timeint   -- DIRK (Alexander) stages with Newton (eq. NewtonSolve) and GMRES
* mlp       -- the per-element warm-start network (forward, backward, Adam)

Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py may
import this package. It shares no code with the HIP library and never calls it.
"""
