"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package holds no arithmetic of the particle-mesh + neutrino step itself: it only
draws particle positions and growing-mode velocities (a Zel'dovich-displaced lattice with
a power-law spectrum) and builds smooth power-spectrum histories of the shape a simulation
would have stored.
Everything it returns is plain NumPy data that both the HIP library and the FP64 oracle
consume unchanged.
"""
from .ics import zeldovich_lattice, zeldovich_ics, batched_lattices, morton_codes, CONFIGS
from .history import synthetic_history, log_spaced_nodes, growth_history, free_streaming_ic

__all__ = ["zeldovich_lattice", "zeldovich_ics", "batched_lattices", "morton_codes",
           "synthetic_history", "log_spaced_nodes", "growth_history", "free_streaming_ic",
           "CONFIGS"]
