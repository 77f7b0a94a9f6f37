"""FP64 CPU oracle for the Adam-based inflation protocol (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It wraps `rcp_oracle.c` (plain C, -ffp-contract=off)
through ctypes and adds the schedule builder of Eq. (trigger).  It shares no
code with the HIP library.
"""
from .oracle import (build, lib, splitmix64, u01, pairs_brute, pairs_cells,
                     rows_pairs, energy_grad, rows_grad, shrink, phi, rsa,
                     run, Params, Schedule, n_trig, default_schedule,
                     time_iterations, set_threads, num_threads, RunState,
                     default_params, absolute_schedule, Result, set_list_check,
                     list_misses, rsa_rounds, set_frozen, phi_frozen, seat,
                     cascade, cascade_counts, set_dim, get_dim, release_schedule,
                     set_boundary, get_boundary)
from . import oracle

__all__ = [
    "build", "lib", "splitmix64", "u01", "pairs_brute", "pairs_cells",
    "rows_pairs", "energy_grad", "rows_grad", "shrink", "phi", "rsa", "run",
    "Params", "Schedule", "n_trig", "default_schedule", "time_iterations",
    "set_threads", "num_threads", "RunState", "set_list_check", "list_misses",
    "rsa_rounds", "set_frozen", "phi_frozen", "seat", "cascade", "cascade_counts",
    "set_dim", "get_dim", "release_schedule", "set_boundary", "get_boundary",
]
