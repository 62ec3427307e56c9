"""MI355X (gfx950) Wedge-Frontier pull engine.

Python face of libwedge.so (include/wedge.h): graphs, BFS, CC, SSSP, PageRank
and the frontier translation step. See _binding for the ctypes layer.
"""
from ._binding import (Graph, Model, TraceSample, WedgeError, bfs, bfs_batch, bfs_multisource,
                       bfs_noalloc, cc, features, frontier_translate, header_functions, lib, pagerank,
                       samples_to_dicts, sssp, trace_counterfactual, tune_bfs, tune_lookup, u32,
                       LIB_PATH)

__all__ = ["Graph", "Model", "TraceSample", "WedgeError", "bfs", "bfs_batch", "bfs_multisource",
           "bfs_noalloc", "cc", "sssp", "pagerank", "frontier_translate", "features", "trace_counterfactual",
           "samples_to_dicts", "tune_bfs", "tune_lookup", "lib", "u32", "header_functions",
           "LIB_PATH"]
