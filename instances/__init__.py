"""Seeded synthetic Ising instances.

This package only draws numbers: it holds none of the method's arithmetic
(no energies, no enumeration, no selection).  Both the CPU oracle tests and
the GPU path read the arrays it returns, so that the two sides see the same
bytes.  Every generator is deterministic in its seed (NumPy PCG64).

Layout convention for every instance: ``J`` is a dense row-major ``N x N``
array of which only the strict upper triangle (i < j) carries couplings; the
diagonal and the lower triangle are zero.  ``h`` has length ``N``.  Spin ``i``
is bit ``i`` of a state mask, bit set meaning ``s_i = +1``.
"""

from .generators import (  # noqa: F401
    random_int_dense,
    random_f32_dense,
    chimera_edges,
    chimera_pm1,
    batched_f32_dense,
    logz_batch,
    ferromagnet,
    mattis,
    free_spins_pow2_fields,
    open_chain,
    listing1_dict,
    dict_to_dense,
    workload,
)
