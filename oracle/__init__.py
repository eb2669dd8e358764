"""Plain FP64 CPU oracle of the RIDG predictor/corrector (TEST INFRASTRUCTURE ONLY).

This package is the checker that the GPU library is compared against. It is
deliberately slow and direct: every element matrix is built by tensor
Gauss-Legendre quadrature, every region system is assembled as one dense
matrix and solved with LAPACK (partial pivoting), and the correction is the
flux-form update written out term by term.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it. It shares no code with the GPU library
(``paper_2101_01231_amd``): it has its own basis, its own quadrature, its own
assembly and its own solver call.

Paper passages followed (arXiv 2101.01231):
  * Sec. 2.1 (general setup): conservation law, orthonormal modal basis,
    the fully discrete one-step update.
  * Sec. 2.2 (RIDG prediction step), eq. (pred_full_system) and Fig. 1:
    the region of 3^d vertex neighbours, time term, internal flux term,
    surface flux term (upwind inside the region, interior trace on the
    region boundary), causal source; keep the centre only.
  * Sec. 2.3 (correction step): explicit flux-form update with the
    predicted space-time solution and Rusanov (= upwind for linear
    advection) fluxes.
  * Sec. 4 (terminology): eq. (l2relerror) and eq. (Mratio).
  * Sec. 3 (Newton on the region system, Jacobian by quadrature, by projection of F'(w) with
    precomputed triple products, and by perturbation) and eq. (burger2d): ``oracle.burgers``.
"""

from .basis import (  # noqa: F401
    spatial_indices,
    spacetime_indices,
    psi,
    dpsi,
    gauss,
)
from .scheme import Problem, step, predict, region_system, element_blocks  # noqa: F401
from .project import project, exact_translate, exact_rotation, l2rel_paper  # noqa: F401
