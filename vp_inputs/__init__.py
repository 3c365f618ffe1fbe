"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the method: only workload descriptions
(domains, resolutions, time steps, initial-condition parameters) and seeded
random arrays.  Both the CPU oracle and the HIP library receive what is made
here; neither is imported from here.
"""

from .configs import CONFIGS, Workload, workload
from .random import random_field, random_shifts, edge_shifts, rng

__all__ = ["CONFIGS", "Workload", "workload", "random_field", "random_shifts",
           "edge_shifts", "rng"]
