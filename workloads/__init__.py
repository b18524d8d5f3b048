"""Seeded synthetic inputs with the shapes of the paper's workloads.

This package only *generates inputs* (node coordinates of stretched grids,
cell resistivity models, source and receiver layouts, frequency lists).  It
contains none of the method's arithmetic and is the only code shared by the
CPU oracle and the HIP path.
"""
from .configs import (Workload, axis_nodes, c1_wholespace, c2_marine1d,
                      c3_blocks, c4_batched, c5_large, tiny, by_name,
                      with_vti, with_window)

__all__ = ["Workload", "axis_nodes", "c1_wholespace", "c2_marine1d",
           "c3_blocks", "c4_batched", "c5_large", "tiny", "by_name",
           "with_vti", "with_window"]
