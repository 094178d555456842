"""Plain, slow, obviously-correct CPU oracle for the recursive sweeping preconditioner.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package.  The
product path (the HIP library under ``paper_1502_07266_amd``) never calls it, and the
two share no code: the oracle imports nothing from the product package and the product
imports nothing from here.  Both only consume the seeded synthetic inputs made by
``paper_1502_07266_amd.inputs`` (which holds none of the method's arithmetic).

Source: F. Liu and L. Ying, "Recursive Sweeping Preconditioner for the 3D Helmholtz
Equation" (Feb 2015).  Everything is complex128 / float64 (the paper does not fix a
precision).  Each function cites the section, equation or algorithm it follows:

* ``problem``   -- Sec. 2: PML profiles sigma, s and the 7-point system, eq. (3).
* ``partition`` -- Sec. 3 (first b layers as one block) and the implementation notes at
                   the end of Sec. 4.2 (several layers per auxiliary problem, thinner
                   auxiliary PML): groups, windows, moving-PML profiles.
* ``sweep``     -- Sec. 4: quasi-1D block LDU (Sec. 4.1), Algorithms 3/4 (inner sweep)
                   and 5/6 (outer sweep), and the adjoint of Algorithm 6.
* ``nested``    -- Sec. 6: 1D nested dissection of the line problems (the parallel
                   alternative to the block LDU; oracle only so far).
* ``krylov``    -- Sec. 5: GMRES as the outer solver (flexible, right preconditioned).
* ``gradient``  -- the adjoint-state misfit gradient (not in the paper; derived from
                   eq. (3), whose only dependence on c is the diagonal omega^2/c^2).
* ``reference`` -- test devices that pin the sweeps: the non-recursive Algorithm 2 with
                   exact sparse solves of the auxiliary problems, and the exact dense
                   block LDU of Sec. 3.

Parity status of each function is recorded in its module docstring.
"""

from .problem import (Problem, sigma, stretch, boundary_profile, axis_profile,
                      assemble_box, helmholtz_matrix)
from .partition import groups, groups_two_fronts, window, window_fronts
from .sweep import LineFactors, SlabSweep, RecursiveSweep, elimination_order
from .nested import NestedDissection
from .krylov import fgmres
from .gradient import misfit_and_gradient

__all__ = [
    "Problem", "sigma", "stretch", "boundary_profile", "axis_profile", "assemble_box",
    "helmholtz_matrix", "groups", "groups_two_fronts", "window", "window_fronts", "LineFactors", "SlabSweep", "RecursiveSweep", "elimination_order",
    "NestedDissection", "fgmres", "misfit_and_gradient",
]
