"""Seeded synthetic inputs for the H/S build.

This module is shared by the CPU oracle, the tests and the benchmark. It draws
random numbers and arranges them in the ABI layout; it holds none of the
arithmetic that builds H or S.

Layout (row-major, complex128 = interleaved re/im doubles):
  A, B        [K, N_G]        atoms stacked along rows, K = sum_a N_L(a)
  T_AA, T_AB, T_BB            packed 1-D, atom a's N_L(a) x N_L(a) block row-major,
                              blocks concatenated in atom order
  U           [K]             diagonal of each U_a, concatenated
  nl          int32 [N_A]     N_L of each atom
"""

from .gen import (  # noqa: F401
    Problem,
    CONFIGS,
    make_problem,
    make_config,
    SERVING,
    serving_requests,
    serving_arrivals,
    serving_atoms,
    serving_request_ab,
    cn,
)
