"""CPU oracle of (scalable) K-MMSE error concealment — TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding) never
calls it, and it shares no code with that path.

Everything is float64 NumPy written straight from the paper's definitions:

* ``skmmse``  — frame driver, BRL / IDL / HQL layers, profile gate (vectorised
  over candidates, one block at a time);
* ``brute``   — the same estimators in pure-Python loops for tiny frames, used
  to pin the vectorised code;
* ``cnn``     — float64 forward and hand-derived backward of the learned
  layer manager.
"""
from .skmmse import (  # noqa: F401
    Params, PROFILES, LAYER_BRL, LAYER_IDL, LAYER_HQL, LAYER_FILL,
    conceal, lost_cells, ring_offsets, block_context, candidate_set,
    block_distances, idl_radii, log_nu_by_radius, estimate_block, hql_estimate,
    UnsupportedLoss,
)
