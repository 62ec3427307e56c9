"""Shared test helpers (no arithmetic of the method)."""
import numpy as np


def relabel(ro, col, perm, w=None):
    """The graph with vertex v renamed perm[v]; rows sorted, parallel edges in input order."""
    n = len(ro) - 1
    deg = np.diff(ro.astype(np.int64))
    u = np.repeat(np.arange(n), deg)
    key = (perm[u].astype(np.uint64) << np.uint64(32)) | perm[col].astype(np.uint64)
    order = np.argsort(key, kind="stable")
    nro = np.zeros(n + 1, np.uint64)
    nro[1:] = np.cumsum(np.bincount(perm[u], minlength=n))
    return nro, perm[col][order].astype(np.uint32), (None if w is None else w[order])
