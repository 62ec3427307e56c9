"""MI355X (gfx950) Wedge-Frontier pull engine.

Python face of libwedge.so (include/wedge.h): graphs, BFS, CC, SSSP, PageRank
and the frontier translation step. See _binding for the ctypes layer.
"""
from ._binding import (Graph, WedgeError, bfs, bfs_batch, bfs_multisource, cc, frontier_translate,
                       header_functions, lib, pagerank, sssp, tune_bfs, tune_lookup, u32, LIB_PATH)

__all__ = ["Graph", "WedgeError", "bfs", "bfs_batch", "bfs_multisource", "cc", "sssp",
           "pagerank", "frontier_translate", "tune_bfs", "tune_lookup", "lib", "u32",
           "header_functions", "LIB_PATH"]
