"""Seeded synthetic graph generators (inputs only; no vertex-cover arithmetic).

Every workload the solver and its CPU checker are run on comes from here, so
that both sides read the very same CSR arrays.  The graphs stand in for the
paper's real sparse datasets (Network Data Repository, PACE 2019; Sec. V-A),
which are not available: the shapes follow the five workload descriptions
(Erdos-Renyi, component-splitting blocks with hubs, planted-cover Chung-Lu
power-law graphs, a mixed batch and a served request stream).

A graph is simple and undirected (Sec. II-A) and is stored as symmetric CSR:
``offsets`` (uint32, n+1 entries) and ``cols`` (uint16 when n <= 65536 and
the caller asks for it, else uint32), both directions of every edge present,
no self-loops, no duplicate edges, rows sorted ascending.  Vertex ids are
passed through a seeded random permutation so that planted or block structure
is not visible in the id order.

Randomness: ``numpy.random.Generator(PCG64(seed))``; per-instance seeds of a
batch are ``seed * 1_000_003 + i``.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Graph", "rng", "from_edges", "relabel", "disjoint_union", "sha256",
    "gnp", "path", "cycle", "complete", "complete_bipartite", "star",
    "petersen", "grid", "hypercube", "random_tree", "fig1_tree",
    "random_regular", "config1_gnp60", "config2_blocks_hubs",
    "config3_chung_lu", "config4_batch", "config5_stream", "planted_gnp",
    "chung_lu_planted", "pack_batch",
]


@dataclass
class Graph:
    n: int
    offsets: np.ndarray            # uint32[n+1]
    cols: np.ndarray               # uint16 or uint32 [nnz]
    name: str = ""
    planted: np.ndarray | None = None   # planted cover (vertex ids), if any
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.offsets[-1])

    @property
    def m(self) -> int:
        return self.nnz // 2

    @property
    def col_bytes(self) -> int:
        return int(self.cols.dtype.itemsize)

    def edges(self) -> tuple[np.ndarray, np.ndarray]:
        """Each undirected edge once, as (u, v) with u < v."""
        src = np.repeat(np.arange(self.n, dtype=np.int64),
                        np.diff(self.offsets.astype(np.int64)))
        dst = self.cols.astype(np.int64)
        keep = src < dst
        return src[keep], dst[keep]

    def with_cols(self, col_bytes: int) -> "Graph":
        dt = np.uint16 if col_bytes == 2 else np.uint32
        if col_bytes == 2 and self.n > 65536:
            raise ValueError("16-bit column ids need n <= 65536")
        return Graph(self.n, self.offsets, self.cols.astype(dt), self.name,
                     self.planted, dict(self.meta))


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _col_dtype(n: int, col_bytes: int | None):
    if col_bytes is None:
        col_bytes = 2 if n <= 65536 else 4
    if col_bytes == 2 and n > 65536:
        raise ValueError("16-bit column ids need n <= 65536")
    return np.uint16 if col_bytes == 2 else np.uint32


def from_edges(n: int, u, v, name: str = "", col_bytes: int | None = None,
               planted=None, meta=None) -> Graph:
    """Symmetric CSR from an undirected edge list (each edge once)."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if u.size:
        if np.any(u == v):
            raise ValueError("self-loop in edge list")
        if u.min() < 0 or v.min() < 0 or max(u.max(), v.max()) >= n:
            raise ValueError("vertex id out of range")
        a, b = np.minimum(u, v), np.maximum(u, v)
        key = a * n + b
        if np.unique(key).size != key.size:
            raise ValueError("duplicate edge in edge list")
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    counts = np.bincount(src, minlength=n) if src.size else np.zeros(n, np.int64)
    off = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(counts, out=off[1:])
    if off[-1] >= 2**32:
        raise ValueError("nnz does not fit 32-bit offsets")
    g = Graph(n, off.astype(np.uint32), dst.astype(_col_dtype(n, col_bytes)),
              name, None if planted is None else np.asarray(planted, np.int64),
              dict(meta or {}))
    return g


def relabel(g: Graph, seed: int, col_bytes: int | None = None) -> Graph:
    """Apply a seeded random permutation to the vertex ids."""
    perm = rng(seed).permutation(g.n)
    u, v = g.edges()
    planted = None if g.planted is None else np.sort(perm[g.planted])
    cb = g.col_bytes if col_bytes is None else col_bytes
    return from_edges(g.n, perm[u], perm[v], g.name, cb, planted, g.meta)


def disjoint_union(graphs, name: str = "union") -> Graph:
    us, vs, base = [], [], 0
    for g in graphs:
        u, v = g.edges()
        us.append(u + base)
        vs.append(v + base)
        base += g.n
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    return from_edges(base, u, v, name)


def sha256(g: Graph) -> str:
    h = hashlib.sha256()
    h.update(np.asarray([g.n, g.nnz, g.col_bytes], np.uint64).tobytes())
    h.update(np.ascontiguousarray(g.offsets).tobytes())
    h.update(np.ascontiguousarray(g.cols).tobytes())
    return h.hexdigest()


# ---------------------------------------------------------------- families

def gnp(n: int, p: float, seed: int, col_bytes: int | None = None,
        name: str = "") -> Graph:
    """Erdos-Renyi G(n, p): every one of the n(n-1)/2 pairs independently."""
    r = rng(seed)
    iu, ju = np.triu_indices(n, k=1)
    keep = r.random(iu.size) < p
    return from_edges(n, iu[keep], ju[keep], name or f"gnp({n},{p})", col_bytes)


def path(n: int) -> Graph:
    a = np.arange(max(n - 1, 0))
    return from_edges(n, a, a + 1, f"P{n}")


def cycle(n: int) -> Graph:
    if n < 3:
        raise ValueError("a simple cycle needs n >= 3")
    a = np.arange(n)
    return from_edges(n, a, (a + 1) % n, f"C{n}")


def complete(n: int) -> Graph:
    iu, ju = np.triu_indices(n, k=1)
    return from_edges(n, iu, ju, f"K{n}")


def complete_bipartite(a: int, b: int) -> Graph:
    u = np.repeat(np.arange(a), b)
    v = np.tile(np.arange(b), a) + a
    return from_edges(a + b, u, v, f"K{a},{b}")


def star(k: int) -> Graph:
    return from_edges(k + 1, np.zeros(k, np.int64), np.arange(1, k + 1), f"S{k}")


def petersen() -> Graph:
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    e = np.array(outer + spokes + inner)
    return from_edges(10, e[:, 0], e[:, 1], "petersen")


def grid(a: int, b: int) -> Graph:
    idx = np.arange(a * b).reshape(a, b)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return from_edges(a * b, u, v, f"grid{a}x{b}")


def hypercube(d: int) -> Graph:
    n = 1 << d
    us, vs = [], []
    for bit in range(d):
        x = np.arange(n)
        lo = x[(x >> bit) & 1 == 0]
        us.append(lo)
        vs.append(lo | (1 << bit))
    return from_edges(n, np.concatenate(us), np.concatenate(vs), f"Q{d}")


def random_tree(n: int, seed: int) -> Graph:
    """Uniform random recursive tree: vertex i attaches to a uniform earlier vertex."""
    r = rng(seed)
    if n <= 1:
        return from_edges(n, [], [], f"tree{n}")
    parent = np.array([r.integers(0, i) for i in range(1, n)], dtype=np.int64)
    return from_edges(n, np.arange(1, n), parent, f"tree{n}")


def fig1_tree() -> Graph:
    """The nine-vertex example of the search-tree figure (Sec. II-B).

    Vertices a..i are 0..8.  e (4) has maximum degree with N(e) = {b, d, f, h};
    removing e leaves the components {a, b, c} and {g, h, i}; the minimum
    cover is {b, e, h} of size three.
    """
    a, b, c, d, e, f, g, h, i = range(9)
    E = [(e, b), (e, d), (e, f), (e, h), (b, a), (b, c), (h, g), (h, i)]
    arr = np.array(E)
    return from_edges(9, arr[:, 0], arr[:, 1], "fig1")


def random_regular(n: int, d: int, r: np.random.Generator) -> tuple[np.ndarray, np.ndarray]:
    """Uniform simple d-regular graph by the pairing model with rejection."""
    if (n * d) % 2:
        raise ValueError("n*d must be even")
    pts = np.repeat(np.arange(n), d)
    while True:
        p = r.permutation(pts)
        u, v = p[0::2], p[1::2]
        if np.any(u == v):
            continue
        a, b = np.minimum(u, v), np.maximum(u, v)
        if np.unique(a * n + b).size != a.size:
            continue
        return a, b


def planted_gnp(n: int, s_size: int, mean_deg: float, r: np.random.Generator):
    """Random graph whose edges all touch a planted set S (|S| = s_size).

    Every pair with at least one endpoint in S is kept independently with
    probability mean_deg * n / (2 * P), P = C(n,2) - C(n - |S|, 2), so the
    expected mean degree is mean_deg.
    """
    S = r.choice(n, size=s_size, replace=False)
    inS = np.zeros(n, bool)
    inS[S] = True
    iu, ju = np.triu_indices(n, k=1)
    touch = inS[iu] | inS[ju]
    P = n * (n - 1) // 2 - (n - s_size) * (n - s_size - 1) // 2
    p = min(1.0, mean_deg * n / (2.0 * P)) if P else 0.0
    keep = touch & (r.random(iu.size) < p)
    return iu[keep], ju[keep], np.sort(S)


def _chung_lu_weights(n: int, gamma: float, i0: float) -> np.ndarray:
    i = np.arange(n, dtype=np.float64)
    return (i + i0) ** (-1.0 / (gamma - 1.0))


def chung_lu_planted(n: int, m: int, gamma: float, s_size: int, seed: int,
                     bipartite: bool = False, col_bytes: int | None = None,
                     name: str = "") -> Graph:
    """Power-law (Chung-Lu style) graph with a planted vertex cover S.

    Weights w_i = (i + i0)^(-1/(gamma-1)); S is the s_size heaviest vertices.
    Each edge draws u from S with probability proportional to w and v from V
    (from V \\ S when ``bipartite``) proportional to w; self-pairs and repeats
    are rejected until exactly m distinct edges exist, so every edge has an
    endpoint in S.  i0 is the smallest offset (found by bisection) for which
    the heaviest vertex's expected degree is at most sqrt(2m) (if no offset
    up to 1e9 meets that cap, i0 = that bound: nearly flat weights).  When three
    rounds of weighted draws in a row add under 1% of the missing edges (a
    small instance close to saturating S x V), the remaining edges are drawn
    uniformly from S x V.
    """
    r = rng(seed)
    cap = math.sqrt(2.0 * m)

    def maxdeg(i0):
        w = _chung_lu_weights(n, gamma, i0)
        ws = w[:s_size].sum()
        wv = (w[s_size:].sum() if bipartite else w.sum())
        return m * w[0] / ws + (0.0 if bipartite else m * w[0] / wv)

    lo, hi = 0.0, 1.0
    while maxdeg(hi) > cap and hi < 1e9:
        hi *= 2.0
    cap_met = maxdeg(hi) <= cap
    if cap_met:
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if maxdeg(mid) > cap:
                lo = mid
            else:
                hi = mid
    # (a small instance can need more than sqrt(2m) per vertex of S on
    # average; then the flattest weights tried, i0 = hi, are used)
    i0 = hi
    w = _chung_lu_weights(n, gamma, i0)
    cs = np.cumsum(w[:s_size])
    cs /= cs[-1]
    if bipartite:
        base = s_size
        cv = np.cumsum(w[s_size:])
    else:
        base = 0
        cv = np.cumsum(w)
    cv /= cv[-1]
    keys = np.zeros(0, np.int64)
    need = m
    pairs = s_size * (s_size - 1) // 2 + s_size * (n - s_size) if not bipartite \
        else s_size * (n - s_size)
    if m > pairs:
        raise ValueError(f"{m} edges cannot all touch {s_size} of {n} vertices")
    stalls = 0
    while True:
        batch = int(need * 1.25) + 1024
        if stalls < 3:
            u = np.searchsorted(cs, r.random(batch), side="right").astype(np.int64)
            v = (np.searchsorted(cv, r.random(batch), side="right") + base).astype(np.int64)
        else:
            # the weighted draws have stopped finding new pairs (a small,
            # dense instance): the rest of the edges are drawn uniformly
            # over S x V, which keeps S a cover
            u = r.integers(0, s_size, batch).astype(np.int64)
            v = r.integers(base, n, batch).astype(np.int64)
        np.minimum(u, s_size - 1, out=u)
        np.minimum(v, n - 1, out=v)
        ok = u != v
        a, b = np.minimum(u[ok], v[ok]), np.maximum(u[ok], v[ok])
        allk = np.concatenate([keys, a * n + b])
        _, first = np.unique(allk, return_index=True)
        first.sort()
        keys = allk[first]
        if keys.size >= m:
            keys = keys[:m]
            break
        stalls = stalls + 1 if (m - keys.size) > 0.99 * need else 0
        need = m - keys.size
    a, b = keys // n, keys % n
    perm = r.permutation(n)
    S = np.sort(perm[np.arange(s_size)])
    meta = {"gamma": gamma, "i0": i0, "planted_size": s_size, "bipartite": bipartite,
            "degree_cap_met": bool(cap_met), "uniform_fill": stalls >= 3}
    return from_edges(n, perm[a], perm[b], name or f"chung_lu(n={n},m={m})",
                      col_bytes, S, meta)


# ---------------------------------------------------------------- workloads

def config1_gnp60(seed: int = 1) -> Graph:
    """One G(60, 0.1) graph, CSR uint32 offsets + uint16 cols."""
    return gnp(60, 0.1, seed, col_bytes=2, name=f"gnp60_s{seed}")


def config2_blocks_hubs(seed: int = 2, nblocks: int = 20, bsize: int = 96,
                        nhubs: int = 8, per_block: int = 30,
                        col_bytes: int = 4) -> Graph:
    """Component-splitting graph: random 3-regular blocks joined by hubs.

    nblocks uniform random 3-regular graphs on bsize vertices, plus nhubs hub
    vertices, each joined to per_block distinct uniform vertices of every
    block (no hub-hub edges).  Removing the hubs splits the graph into the
    blocks.  Defaults: 20 x 96 + 8 = 1,928 vertices, 7,680 edges.
    """
    r = rng(seed)
    us, vs = [], []
    for blk in range(nblocks):
        a, b = random_regular(bsize, 3, r)
        us.append(a + blk * bsize)
        vs.append(b + blk * bsize)
    hub0 = nblocks * bsize
    for h in range(nhubs):
        for blk in range(nblocks):
            t = r.choice(bsize, size=per_block, replace=False) + blk * bsize
            us.append(np.full(per_block, hub0 + h))
            vs.append(t)
    n = hub0 + nhubs
    g = from_edges(n, np.concatenate(us), np.concatenate(vs),
                   f"blocks{nblocks}x{bsize}+hubs{nhubs}")
    return relabel(g, seed * 1_000_003, col_bytes)


def config3_chung_lu(seed: int = 3, n: int = 1_000_000, m: int = 5_000_000,
                     gamma: float = 2.1, s_size: int = 60_000,
                     bipartite: bool = False) -> Graph:
    return chung_lu_planted(n, m, gamma, s_size, seed, bipartite, col_bytes=4,
                            name=f"chung_lu_pvc(n={n},m={m},S={s_size})")


def config4_instance(i: int, seed: int = 4, n_lo: int = 50, n_hi: int = 800,
                     d_lo: float = 4.0, d_hi: float = 12.0,
                     planted_frac: float = 0.25) -> Graph:
    """Instance i of the uneven batch: G(n, d/(n-1)) or planted |S| = 0.3 n,
    from its own seed (seed * 1,000,003 + i)."""
    r = rng(seed * 1_000_003 + i)
    n = int(r.integers(n_lo, n_hi + 1))
    d = float(r.uniform(d_lo, d_hi))
    if r.random() < planted_frac:
        u, v, S = planted_gnp(n, int(round(0.3 * n)), d, r)
        return from_edges(n, u, v, f"b{i}_planted", 2, S, {"d": d})
    iu, ju = np.triu_indices(n, k=1)
    keep = r.random(iu.size) < d / (n - 1)
    return from_edges(n, iu[keep], ju[keep], f"b{i}_gnp", 2, None, {"d": d})


def config4_batch(seed: int = 4, count: int = 4096, n_lo: int = 50,
                  n_hi: int = 800, d_lo: float = 4.0, d_hi: float = 12.0,
                  planted_frac: float = 0.25) -> list[Graph]:
    """Batch of uneven graphs: G(n, d/(n-1)) or planted |S| = 0.3 n."""
    return [config4_instance(i, seed, n_lo, n_hi, d_lo, d_hi, planted_frac)
            for i in range(count)]


def pack_batch(graphs: list[Graph]):
    """Pack graphs into one offsets buffer and one 16-bit cols buffer.

    Returns (n[count] u32, nnz[count] u64, offs_base[count] u64,
    cols_base[count] u64, offsets u32[sum(n+1)], cols u16[sum(nnz)]).
    Graph i's offsets are offsets[offs_base[i] : offs_base[i] + n[i] + 1]
    (local, starting at 0) and its columns cols[cols_base[i] : ... + nnz[i]].
    """
    ns = np.array([g.n for g in graphs], np.uint32)
    nnz = np.array([g.nnz for g in graphs], np.uint64)
    ob = np.zeros(len(graphs), np.uint64)
    cb = np.zeros(len(graphs), np.uint64)
    if len(graphs) > 1:
        ob[1:] = np.cumsum(ns[:-1].astype(np.uint64) + 1)
        cb[1:] = np.cumsum(nnz[:-1])
    offsets = np.concatenate([g.offsets for g in graphs]).astype(np.uint32)
    cols = np.concatenate([g.cols.astype(np.uint16) for g in graphs])
    return ns, nnz, ob, cb, offsets, cols


def config5_request(i: int, seed: int = 5, n_lo: int = 100, n_hi: int = 100_000,
                    mean_deg: float = 8.0, gamma: float = 2.3, s_frac: float = 0.06,
                    mvc_frac: float = 0.7) -> dict:
    """Request i of the served stream, from its own seed (seed * 1,000,003 +
    i): a planted Chung-Lu graph of log-uniform size, an MVC request or a PVC
    request with k = |S| + 1 or |S| - 1 by a seeded coin."""
    r = rng(seed * 1_000_003 + i)
    n = int(round(math.exp(r.uniform(math.log(n_lo), math.log(n_hi)))))
    s = max(1, int(round(s_frac * n)))
    m = int(round(mean_deg * n / 2))
    g = chung_lu_planted(n, m, gamma, s, int(r.integers(1 << 62)),
                         col_bytes=None, name=f"req{i}")
    if r.random() < mvc_frac:
        return {"graph": g, "kind": "min", "k": 0}
    k = s + (1 if r.random() < 0.5 else -1)
    return {"graph": g, "kind": "param", "k": max(k, 0)}


def config5_stream(seed: int = 5, count: int = 2000, n_lo: int = 100,
                   n_hi: int = 100_000, mean_deg: float = 8.0,
                   gamma: float = 2.3, s_frac: float = 0.06,
                   mvc_frac: float = 0.7):
    """Served request stream: planted Chung-Lu graphs of log-uniform size.

    Returns a list of dicts {graph, kind ('min'|'param'), k} in arrival order;
    PVC requests use k = |S| + 1 or |S| - 1 by a seeded coin.  Arrival times
    are drawn by the server from its own rate.
    """
    return [config5_request(i, seed, n_lo, n_hi, mean_deg, gamma, s_frac, mvc_frac)
            for i in range(count)]
