"""Seeded synthetic inputs: graphs in canonical CSR form and query pairs.

This module is shared by the HIP path, the tests and the benchmark.  It holds
no part of the estimator's arithmetic: it only builds undirected, unweighted,
connected graphs and draws (s, t) node pairs, all from explicit seeds.

Canonical CSR (the form both the library and the CPU checker take):
  * ``row_ptr`` int64[n+1] (converted to int32 at the library boundary),
    ``col_idx`` int32[nnz];
  * symmetric, no self-loops, no duplicate entries, every degree >= 1;
  * each row sorted ascending by node id.  The walk sampler picks the
    ``(draw mod d(u))``-th entry of row u, so this order is part of the
    walk definition.

Graph families (the paper evaluates on SNAP social/collaboration graphs of
mean degree 5-76 with power-law degree skew, Section 6 / dataset table; none
of those datasets is available here, so these synthetic families stand in):
  * ``erdos_renyi_path``: uniform random edges plus a spanning path over a
    seeded permutation, so the graph is connected;
  * ``chung_lu``: expected-degree power-law graph, largest component only;
  * ``rmat``: recursive-matrix (Graph500-style) graph, largest component.
"""

from __future__ import annotations

import dataclasses

import os

import numpy as np

__all__ = [
    "CSRGraph",
    "from_edges",
    "erdos_renyi_path",
    "chung_lu",
    "rmat",
    "complete_graph",
    "cycle_graph",
    "path_graph",
    "star_graph",
    "complete_bipartite",
    "lollipop_graph",
    "uniform_pairs",
    "degree_pairs",
    "edge_pairs",
]


@dataclasses.dataclass
class CSRGraph:
    """Undirected graph in canonical CSR form (see module docstring)."""

    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col_idx: np.ndarray  # int32[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        """Number of undirected edges."""
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def row_ptr32(self) -> np.ndarray:
        if self.nnz >= 2**31:
            raise ValueError("graph too large for int32 CSR offsets")
        return np.ascontiguousarray(self.row_ptr, dtype=np.int32)

    def edges(self) -> np.ndarray:
        """Undirected edge list (u < v), int64[m, 2]."""
        deg = self.degrees()
        src = np.repeat(np.arange(self.n, dtype=np.int64), deg)
        dst = self.col_idx.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep]], axis=1)


def from_edges(n: int, edges: np.ndarray, *, largest_component: bool = False,
               name: str = "") -> CSRGraph:
    """Canonical CSR from an (m, 2) integer edge array.

    Self-loops and duplicate edges are dropped; both directions are stored.
    With ``largest_component`` the graph is restricted to its largest
    connected component and relabelled compactly, keeping the relative order
    of the surviving node ids.
    """
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    key = np.unique(lo * n + hi)
    lo = key // n
    hi = key % n
    # both directions, sorted by (row, column) through one key sort
    key = np.concatenate([lo * n + hi, hi * n + lo])
    del lo, hi
    key.sort()
    src = key // n
    dst = key % n
    del key
    if largest_component:
        keep_nodes = _largest_component(n, src, dst)
        if keep_nodes.size < n:
            relabel = np.full(n, -1, dtype=np.int64)
            relabel[keep_nodes] = np.arange(keep_nodes.size, dtype=np.int64)
            ok = relabel[src] >= 0
            # the relabelling is increasing, so the (row, column) order survives
            src = relabel[src[ok]]
            dst = relabel[dst[ok]]
            n = int(keep_nodes.size)
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSRGraph(n=n, row_ptr=row_ptr, col_idx=dst.astype(np.int32), name=name)


def _largest_component(n: int, src: np.ndarray, dst: np.ndarray) -> np.ndarray:
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    # (src, dst) arrive sorted by row, so the CSR is built directly
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=indptr[1:])
    adj = sp.csr_matrix((np.ones(src.size, dtype=np.int8), dst, indptr), shape=(n, n))
    ncomp, labels = connected_components(adj, directed=False)
    sizes = np.bincount(labels, minlength=ncomp)
    # nodes of degree 0 form singleton components; never pick one of those
    big = int(np.argmax(sizes))
    return np.flatnonzero(labels == big).astype(np.int64)


# --------------------------------------------------------------------------
# Graph families
# --------------------------------------------------------------------------

def erdos_renyi_path(n: int, mean_degree: float, seed: int) -> CSRGraph:
    """Connected uniform random graph with exactly m = n * mean_degree / 2 edges.

    A spanning path over a seeded random permutation (n - 1 edges) makes the
    graph connected; the remaining edges are distinct uniform pairs that are
    not path edges.
    """
    rng = np.random.default_rng(seed)
    m_total = int(round(n * mean_degree / 2))
    if m_total < n - 1:
        raise ValueError("mean degree too small for a spanning path")
    perm = rng.permutation(n)
    path = np.stack([perm[:-1], perm[1:]], axis=1).astype(np.int64)
    have = set(np.minimum(path[:, 0], path[:, 1]) * n + np.maximum(path[:, 0], path[:, 1]))
    need = m_total - (n - 1)
    extra = []
    while need > 0:
        cand = rng.integers(0, n, size=(max(2 * need, 1024), 2), dtype=np.int64)
        cand = cand[cand[:, 0] != cand[:, 1]]
        keys = np.minimum(cand[:, 0], cand[:, 1]) * n + np.maximum(cand[:, 0], cand[:, 1])
        _, first = np.unique(keys, return_index=True)
        for idx in np.sort(first):
            k = int(keys[idx])
            if k in have:
                continue
            have.add(k)
            extra.append(k)
            need -= 1
            if need == 0:
                break
    extra = np.asarray(extra, dtype=np.int64)
    e = np.concatenate([path, np.stack([extra // n, extra % n], axis=1)])
    return from_edges(n, e, name=f"er_path(n={n},deg={mean_degree},seed={seed})")


def chung_lu(n: int, gamma: float, mean_degree: float, seed: int) -> CSRGraph:
    """Chung-Lu expected-degree graph, largest component only.

    Node i gets weight w_i proportional to (i + 1)^(-1/(gamma - 1)); weights
    are capped at sqrt(mean_degree * n) and rescaled to the requested mean.
    ``n * mean_degree / 2`` endpoint pairs are drawn independently with
    probability proportional to w; self-loops and duplicates are dropped.
    Node ids stay in descending-weight order after the component is taken.
    """
    rng = np.random.default_rng(seed)
    w = np.power(np.arange(1, n + 1, dtype=np.float64), -1.0 / (gamma - 1.0))
    cap = np.sqrt(mean_degree * n)
    for _ in range(50):
        w *= mean_degree / w.mean()
        if w.max() <= cap * (1 + 1e-12):
            break
        w = np.minimum(w, cap)
    p = w / w.sum()
    cdf = np.cumsum(p)
    cdf[-1] = 1.0
    m_samples = int(round(n * mean_degree / 2))
    e = np.empty((m_samples, 2), dtype=np.int64)
    chunk = 1 << 22
    for lo in range(0, m_samples, chunk):
        hi = min(m_samples, lo + chunk)
        u = rng.random((hi - lo, 2))
        e[lo:hi] = np.searchsorted(cdf, u, side="right")
    np.minimum(e, n - 1, out=e)
    return from_edges(n, e, largest_component=True,
                      name=f"chung_lu(n={n},gamma={gamma},deg={mean_degree},seed={seed})")


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
         progress=None) -> CSRGraph:
    """R-MAT graph with 2^scale nodes and edge_factor * 2^scale edge samples.

    Each sample descends ``scale`` levels of the adjacency matrix, choosing a
    quadrant with probabilities (a, b, c, 1 - a - b - c) from one uniform draw
    per level.  Samples come in chunks of 2^22, each with its own child of the
    seed's SeedSequence (so chunks can be drawn in parallel and the result does
    not depend on the thread count).  Node labels are then permuted by a seeded
    permutation (removing the generator's id locality), the result is
    symmetrised and deduplicated, and the largest component is kept.
    ``progress``, if given, is called with a short message after every 16
    chunks and before the CSR is built.
    """
    from concurrent.futures import ThreadPoolExecutor

    n = 1 << scale
    m_samples = edge_factor * n
    chunk = 1 << 22
    nchunks = (m_samples + chunk - 1) // chunk
    seqs = np.random.SeedSequence(seed).spawn(nchunks + 1)
    perm = np.random.default_rng(seqs[0]).permutation(n).astype(np.int64)
    t1, t2, t3 = np.float32(a), np.float32(a + b), np.float32(a + b + c)
    out = np.empty((m_samples, 2), dtype=np.int64)

    def draw(i):
        lo = i * chunk
        cnt = min(m_samples, lo + chunk) - lo
        rng = np.random.default_rng(seqs[i + 1])
        src = np.zeros(cnt, dtype=np.int64)
        dst = np.zeros(cnt, dtype=np.int64)
        for level in range(scale):
            u = rng.random(cnt, dtype=np.float32)
            # quadrant 0..3 = (row bit, column bit) with probabilities a, b, c, d
            q = (u >= t1).astype(np.int64) + (u >= t2) + (u >= t3)
            shift = scale - 1 - level
            src |= (q >> 1) << shift
            dst |= (q & 1) << shift
        out[lo:lo + cnt, 0] = perm[src]
        out[lo:lo + cnt, 1] = perm[dst]

    with ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1))) as ex:
        for i, _ in enumerate(ex.map(draw, range(nchunks))):
            if progress and ((i + 1) % 16 == 0 or i + 1 == nchunks):
                progress(f"rmat: {i + 1}/{nchunks} sample chunks")
    if progress:
        progress("rmat: building the CSR")
    return from_edges(n, out, largest_component=True,
                      name=f"rmat(scale={scale},ef={edge_factor},seed={seed})")


# Small deterministic graphs with closed-form answers ------------------------

def complete_graph(n: int) -> CSRGraph:
    iu = np.triu_indices(n, 1)
    return from_edges(n, np.stack(iu, axis=1), name=f"K{n}")


def cycle_graph(n: int) -> CSRGraph:
    i = np.arange(n)
    return from_edges(n, np.stack([i, (i + 1) % n], axis=1), name=f"C{n}")


def path_graph(n: int) -> CSRGraph:
    i = np.arange(n - 1)
    return from_edges(n, np.stack([i, i + 1], axis=1), name=f"P{n}")


def star_graph(leaves: int) -> CSRGraph:
    i = np.arange(1, leaves + 1)
    return from_edges(leaves + 1, np.stack([np.zeros_like(i), i], axis=1), name=f"S{leaves}")


def complete_bipartite(a: int, b: int) -> CSRGraph:
    u, v = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return from_edges(a + b, np.stack([u.ravel(), v.ravel()], axis=1), name=f"K{a},{b}")


def lollipop_graph(clique: int, tail: int) -> CSRGraph:
    """Complete graph on ``clique`` nodes with a path of ``tail`` extra nodes."""
    iu = np.stack(np.triu_indices(clique, 1), axis=1)
    chain = np.arange(clique - 1, clique + tail)
    tail_e = np.stack([chain[:-1], chain[1:]], axis=1)
    return from_edges(clique + tail, np.concatenate([iu, tail_e]),
                      name=f"lollipop({clique},{tail})")


def stochastic_block(blocks: int, size: int, p_in: float, p_out: float, seed: int) -> CSRGraph:
    """Planted partition: ``blocks`` groups of ``size`` nodes, each node pair an
    edge with probability ``p_in`` inside a group and ``p_out`` across
    (dense rows with slow mixing); largest component."""
    rng = np.random.default_rng(seed)
    n = blocks * size
    iu = np.triu_indices(n, 1)
    same = (iu[0] // size) == (iu[1] // size)
    keep = rng.random(iu[0].size) < np.where(same, p_in, p_out)
    return from_edges(n, np.stack([iu[0][keep], iu[1][keep]], axis=1), largest_component=True,
                      name=f"sbm({blocks}x{size},{p_in},{p_out})")


# --------------------------------------------------------------------------
# Query pairs
# --------------------------------------------------------------------------

def uniform_pairs(n: int, count: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """``count`` pairs (s, t), s != t, each endpoint uniform over the nodes."""
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, size=count, dtype=np.int64)
    off = rng.integers(1, n, size=count, dtype=np.int64)
    t = (s + off) % n
    return s.astype(np.int32), t.astype(np.int32)


def degree_pairs(g: CSRGraph, count: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Pairs whose endpoints are each drawn with probability proportional to degree."""
    rng = np.random.default_rng(seed)
    # a uniformly random CSR entry's column is a degree-proportional node
    s = g.col_idx[rng.integers(0, g.nnz, size=count)].astype(np.int64)
    t = g.col_idx[rng.integers(0, g.nnz, size=count)].astype(np.int64)
    clash = s == t
    while clash.any():
        t[clash] = g.col_idx[rng.integers(0, g.nnz, size=int(clash.sum()))]
        clash = s == t
    return s.astype(np.int32), t.astype(np.int32)


def edge_pairs(g: CSRGraph, count: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Pairs (s, t) that are edges of the graph, uniform over the undirected edges."""
    rng = np.random.default_rng(seed)
    e = g.edges()
    pick = rng.integers(0, e.shape[0], size=count)
    return e[pick, 0].astype(np.int32), e[pick, 1].astype(np.int32)
