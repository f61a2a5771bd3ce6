"""CPU oracle of the H/S build: TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and the benchmark's cpu_baseline leg may
import this package. The product path (paper_1611_00606_amd) never does; it
fails loudly when its HIP library is missing instead of falling back here.
"""

from .hs_oracle import (  # noqa: F401
    overlap,
    hamiltonian,
    overlap_entrywise,
    hamiltonian_entrywise,
    overlap_columns,
    hamiltonian_columns,
    bilinear,
    cholesky_lower,
    atom_products,
)
from .hsdla_host import algorithm1  # noqa: F401
from .gep import cholesky_full, gep_reduce  # noqa: F401,E402
