"""Seeded synthetic inputs for the swap-potential engine.

This package only *generates inputs*: particle positions, types, velocities,
box lengths and the per-type-pair coefficient tables of the systems that the
engine and its tests run on.  It holds none of the method's arithmetic (no
potential, force, integrator or bond criterion); the FP64 oracle and the HIP
engine each consume these inputs on their own.

Recipes (all seeded with numpy PCG64):

* ``small_reactive``  -- N identical reactive particles, uniform random
  sequential addition with a minimum image distance, cubic periodic box.
* ``assembly_mixture`` -- 50/50 mixture of inert WCA colloids and small
  reactive sites (the 1M-particle self-assembly workload and its small
  versions).
* ``replica_set``     -- many independent replicas of uneven size, density,
  lambda and inert fraction.
* ``vitrimer_network`` -- bead-spring chains (FENE springs) with reactive
  sites and free two-bead crosslinkers, grown self-avoiding in the box.
* ``dumbbell_mixture`` -- the A/B bond-swap mixture (A:B = 3:2, n = 100,
  density 0.125) of the paper's swap test and performance figure.
* ``planar_reactive`` -- reactive particles in the plane z = 0 of the paper's
  2d square box (side 39.63), for the integrator's dim = 2 mode.
* ``patchy_mixture``  -- the 2d mixture of tri- and difunctional patchy disks
  (rigid bodies: centres plus rim patches) in the same box.
* ``cluster``         -- hand-placed few-particle configurations.
"""
from .systems import (  # noqa: F401
    KIND_NONE, KIND_SWAP, KIND_WCA, WCA_CUT_FACTOR,
    PairTable, System, fp32_box, wrap_fp32,
    swap_table_single, assembly_table,
    small_reactive, unequal_lambda_mixture, assembly_mixture, replica_set, cluster, vitrimer_network, vitrimer_table,
    dumbbell_mixture, dumbbell_table, planar_reactive, patchy_mixture, patchy_table,
    maxwell_velocities, rsa_positions,
)
