"""FP64 CPU oracle for the distilled multi-time-step (DMTS) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or calls this
package; only the test suite, the smoke check and the benchmark's CPU-baseline leg do.
It shares no code, tables or constants with the HIP path.

What it computes, plainly and slowly, in float64 NumPy:

  * ``neighbors``   -- the pair set {(i, j): j != i, |minimage(x_j - x_i)| < r_c}, by brute
                       force (and a k-d tree for large periodic boxes), restricted to one
                       molecule when molecules are batched with open boundaries.
  * ``potentials``  -- energies and analytic forces of the two synthetic neural network
                       potentials that stand in for the paper's fast distilled model and
                       its expensive reference model (Methods: neural network
                       architectures; the fast model has one message-passing interaction
                       and a 3.5 A receptive field, the reference two interactions).
  * ``integrators`` -- the BAOAB-RESPA multi-time-step step of Algorithm 1 (force
                       splitting F_large - F_small applied at the outer level) and the
                       single-time-step BAOAB integrator used as the baseline (Experiments:
                       STS comparator), with the Langevin O-step optional.

Every function names the passage of the paper (or the reading of it) that it follows.
"""

from . import neighbors, potentials, integrators  # noqa: F401
