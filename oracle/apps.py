"""The paper's two applications of a stable integer sort (Section 6.2),
written from their definitions -- TEST INFRASTRUCTURE ONLY.

Graph transpose: a directed graph in compressed sparse row form (offsets of
length V + 1, targets of length E; the out-edges of u are
targets[offsets[u]:offsets[u+1]]) becomes the graph with every edge (u, v)
reversed to (v, u), again in compressed sparse row form.  Sorting the edges
stably by v keeps, within each v, the sources in the order the edges were
listed (u ascending), which is the order written out below.

Morton order: the z-value of a d-dimensional point interleaves the bits of
its coordinates (bit i of coordinate j becomes bit d*i + j of the code);
the points are then stably sorted by z-value.  With 32-bit codes each
coordinate contributes its low 32 // d bits.
"""
from __future__ import annotations

import numpy as np


def transpose_csr(offsets: np.ndarray, targets: np.ndarray, n_vertices: int):
    """Reversed graph in CSR: (t_offsets, t_targets), built vertex by vertex
    from the definition (in-lists in edge-list order)."""
    offsets = offsets.astype(np.int64)
    targets = targets.astype(np.int64)
    n_edges = int(offsets[-1])
    indeg = np.zeros(n_vertices, dtype=np.int64)
    np.add.at(indeg, targets, 1)
    t_offsets = np.zeros(n_vertices + 1, dtype=np.int64)
    t_offsets[1:] = np.cumsum(indeg)
    fill = t_offsets[:-1].copy()
    t_targets = np.zeros(n_edges, dtype=np.int64)
    sources = np.repeat(np.arange(n_vertices, dtype=np.int64), np.diff(offsets))
    for e in range(n_edges):  # edge-list order: u ascending, then position in u's list
        v = targets[e]
        t_targets[fill[v]] = sources[e]
        fill[v] += 1
    return t_offsets.astype(np.uint64), t_targets.astype(np.uint32)


def transpose_csr_fast(offsets: np.ndarray, targets: np.ndarray, n_vertices: int):
    """The same result through a library stable sort (for larger graphs)."""
    offsets = offsets.astype(np.int64)
    sources = np.repeat(np.arange(n_vertices, dtype=np.uint32), np.diff(offsets))
    o = np.argsort(targets, kind="stable")
    t_targets = sources[o]
    t_offsets = np.zeros(n_vertices + 1, dtype=np.uint64)
    t_offsets[1:] = np.cumsum(np.bincount(targets.astype(np.int64), minlength=n_vertices)).astype(np.uint64)
    return t_offsets, t_targets.astype(np.uint32)


def morton_code_u32(coords: np.ndarray) -> np.ndarray:
    """z-values of points given as coords[d][i] (d = 2 or 3), bit by bit."""
    d = coords.shape[0]
    per = 32 // d
    out = np.zeros(coords.shape[1], dtype=np.uint64)
    for i in range(per):
        for j in range(d):
            bit = (coords[j].astype(np.uint64) >> np.uint64(i)) & np.uint64(1)
            out |= bit << np.uint64(d * i + j)
    return out.astype(np.uint32)


def morton_sort(coords: np.ndarray):
    """(sorted z-values, point indices in Morton order; ties by index)."""
    z = morton_code_u32(coords)
    o = np.argsort(z, kind="stable")
    return z[o], o.astype(np.uint32)
