"""FP64 CPU oracle for PRISM's trajectory-projection QP.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The HIP library
never imports, links or calls it, and this package imports nothing from the HIP
library: the two share no code. Inputs come from the separate ``workloads``
package, which holds only seeded random draws.

Contents (each function cites the passage of the paper it follows):

* ``problem``     -- the per-joint derivative maps, the stacked G/h/A/b of the
                     compact QP, and the velocity-unit constraint rows used by
                     the headline solver;
* ``factor``      -- the KKT matrix M of the primal update, its one-time
                     factorization, and the reduced inverse (K, k);
* ``admm``        -- the headline ADMM iteration (scaled dual, velocity-unit
                     rows), the paper's printed Bregman iteration as a flag,
                     residuals, per-column early exit and warm start;
* ``exact``       -- independent exact-projection checkers: brute-force face
                     enumeration for tiny horizons, active-set polishing, and a
                     KKT certificate with non-negative least squares;
* ``feasibility`` -- physical-unit constraint violations of a trajectory;
* ``sigma_eff``   -- the single-joint sampling diagnostic (Sec. III-C).

Parity status: the exact projection is pinned by brute force, KKT certificates
and closed-form special cases; the ADMM iterates at a fixed count have no
printed values in the paper ("parity unpinned" against the paper) and are pinned
by per-step optimality conditions and by convergence to the exact projection.
"""

from . import problem, factor, admm, exact, feasibility  # noqa: F401
