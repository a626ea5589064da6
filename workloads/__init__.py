"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package holds only input generation: closed, outward-oriented triangle
surface meshes with their port (source / sink) triangle sets, and seeded
random vectors.  It contains none of the method's arithmetic (no basis
functions, no integrals, no loop analysis), so the oracle and the GPU path
can both consume it without sharing any computation.
"""
from .geometry import (Structure, box_bar, prism, paper_bar_e1, bond_wires,
                       config1_bar, config2_wires, traces, config3_traces, pdn, config4_pdn)
from .vectors import complex_normal, real_normal

__all__ = ["Structure", "box_bar", "prism", "paper_bar_e1", "bond_wires",
           "config1_bar", "config2_wires", "traces", "config3_traces", "pdn", "config4_pdn",
           "complex_normal", "real_normal"]
