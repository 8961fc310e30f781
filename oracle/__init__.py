"""FP64 CPU oracle of the swap potential (Ciarella & Ellenbroek, arXiv 1912.08569).

TEST INFRASTRUCTURE ONLY.  Nothing in the engine (``paper_1912_08569_amd``)
imports, links or runs anything in this package; only the tests, the
``smoke()`` check and the CPU-baseline leg of the benchmark do.  The oracle
shares no code, header, table or constant generator with the HIP path.  Its
inputs come from the seeded generators in ``workloads`` (which hold none of
the method's arithmetic) or from hand-placed configurations.

What it computes (all in float64):

* ``swap_ref``  -- numpy evaluator of the total energy, per-particle energies,
  forces, configurational virial and bond count of the potential: the
  generalized-LJ pair term (Sec. 2, eq. 2b), the switching factor v-hat
  (eq. pot) and the three-body term lambda*eps*vhat_ij*vhat_ik (eq. 3bp),
  summed once per centre i and unordered partner pair {j, k}; the triplet
  virial of the pressure tensor (Sec. 2.1, eq. p3); one BAOAB Langevin step.
* ``literal``   -- the same energy by explicit triple loops, for a handful of
  particles (pins the triplet counting of ``swap_ref``).
* ``philox_ref`` -- the Philox4x32-10 counter-based generator (Salmon et al.,
  SC'11) and the Box-Muller map used for the thermostat noise.
* ``brute``     -- a plain C, OpenMP, O(N^2) brute-force evaluator of the same
  quantities (independent code, built with ``-ffp-contract=off``), used for
  large systems, sampled-particle checks and the CPU baseline timing.
* ``adjoint_ref`` -- analytic Hessian-vector products and parameter gradients
  of the total energy (the calculus of the same terms), pinned by central
  finite differences of ``swap_ref`` forces and energies; the force-parameter
  vector-Jacobian product by central differences of ``swap_ref`` forces.

Parity status of each function is listed in its module header.
"""
