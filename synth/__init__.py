"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only *draws* inputs: atomic systems (water lattices, solvated
random-walk chains, serving replica mixes), model weight vectors laid out in
the documented manifest order, initial velocities and arrival times.  It holds
none of the method's arithmetic (no model, no integrator, no neighbour rule),
so that neither the CPU oracle nor the GPU path depends on the other through
it.
"""

from .systems import (  # noqa: F401
    SPECIES, SPECIES_INDEX, MASS_AMU, System,
    water_box, solvated_chain, replica_mix, maxwell_boltzmann,
    cluster_pair, water_config,
)
from .weights import (  # noqa: F401
    cons_manifest, nc_manifest, random_weights, manifest_size, ModelSpec,
    CONS_CFG0, CONS_CFG1, NC_CFG0, NC_CFG1,
)
