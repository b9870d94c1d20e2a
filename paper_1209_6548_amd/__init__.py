"""MI355X (gfx950) lattice ES-BGK: one fused pull-stream + collide HIP kernel
per time step, behind a small C ABI (include/esbgk.h), with a thin ctypes
binding. Build the library with ``python -m paper_1209_6548_amd.build``."""

from .binding import (Batch, EsbgkError, Lattice, TVDLattice, lattice_info, lib, make_problem,  # noqa: F401
                      split_fields, tvd_velocity_set)
