"""Counter-based seeded generators for the synthetic workloads.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a counter-based
generator: draw ``i`` of a stream with key ``k`` is ``mix64(k + (i + 1) * G)``
with ``G = 0x9E3779B97F4A7C15``.  A stream key is derived from a seed and a
tag, so every array below is a pure function of its seed.

Graph convention (Section 4.2 of the paper): the adjacency matrix entry
``A[i, j]`` holds the weight of the edge ``j -> i``.  Generators return edge
lists ``(src, dst)``; callers fold them with rows = ``dst`` and
cols = ``src``.

Workload shapes follow the paper's synthetic inputs (independent-probability
sparsity, Section 6.1; random graphs, Section 6.3) and the R-MAT / stencil /
power-law families used for schedule training.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "GOLDEN", "mix64", "stream_key", "rand_u64", "uniform_f64", "uniform_f32",
    "randint", "permutation", "er_edges", "rmat_edges", "stencil27_edges",
    "powerlaw_edges", "bernoulli_keys", "pick_sources", "edge_values",
    "er_batch_params", "selector_matrix", "selector_panel_rows", "dense_graph", "FAMILIES", "SEED_CFG0", "SEED_CFG1", "SEED_CFG2", "SEED_CFG3",
    "SEED_CFG4",
]

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

SEED_CFG0 = 0x5EED0000
SEED_CFG1 = 0x5EED0001
SEED_CFG2 = 0x5EED0002
SEED_CFG3 = 0x5EED0003
SEED_CFG4 = 0x5EED0004


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied elementwise to uint64 values."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _chunked(fn, n: int, chunk: int = 1 << 20) -> None:
    """fn(e0, e1) over consecutive chunks of 0..n-1 on a few threads (numpy
    releases the interpreter lock in its array loops); the draws are
    counter-based, so the result does not depend on the split."""
    bounds = [(e, min(n, e + chunk)) for e in range(0, n, chunk)]
    if len(bounds) <= 1:
        for e0, e1 in bounds:
            fn(e0, e1)
        return
    import concurrent.futures
    import os
    workers = max(1, min(16, len(os.sched_getaffinity(0)), len(bounds)))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda b: fn(*b), bounds))


def stream_key(seed: int, tag: int) -> int:
    """Key of the stream ``tag`` under ``seed`` (a 64-bit integer)."""
    s = np.array([(seed * 0x100000001B3 + tag) & 0xFFFFFFFFFFFFFFFF],
                 dtype=np.uint64)
    return int(mix64(s)[0])


def rand_u64(key: int, n: int, offset: int = 0) -> np.ndarray:
    """Draws ``offset .. offset+n-1`` of stream ``key`` as uint64."""
    i = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + i * GOLDEN
    return mix64(z)


def uniform_f64(key: int, n: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1): top 53 bits times 2^-53."""
    if n > (1 << 22):
        out = np.empty(n, dtype=np.float64)

        def part(e0, e1):
            out[e0:e1] = uniform_f64(key, e1 - e0, offset + e0)

        _chunked(part, n)
        return out
    x = rand_u64(key, n, offset)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_f32(key: int, n: int, offset: int = 0) -> np.ndarray:
    """Uniform floats in [0, 1): top 24 bits times 2^-24 (exact in fp32)."""
    x = rand_u64(key, n, offset)
    return ((x >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)).astype(np.float32)


def randint(key: int, n: int, lo: int, hi: int) -> np.ndarray:
    """Uniform integers in [lo, hi] by rejection on the top 32 bits.

    A 32-bit draw ``u`` is accepted when ``u < 2^32 - (2^32 mod r)``
    (``r = hi - lo + 1``) and mapped to ``lo + u mod r``; rejected slots are
    redrawn from later counters of the same stream.
    """
    r = hi - lo + 1
    assert 1 <= r <= (1 << 32)
    limit = (1 << 32) - ((1 << 32) % r)
    out = np.empty(n, dtype=np.int64)
    todo = np.arange(n, dtype=np.int64)
    offset = 0
    while todo.size:
        u = (rand_u64(key, todo.size, offset) >> np.uint64(32)).astype(np.int64)
        offset += todo.size
        ok = u < limit
        out[todo[ok]] = lo + (u[ok] % r)
        todo = todo[~ok]
    return out


def permutation(key: int, n: int) -> np.ndarray:
    """A seeded random permutation of 0..n-1 (argsort of distinct draws)."""
    x = rand_u64(key, n)
    # ties are impossible in practice; a stable sort keeps it a bijection anyway
    return np.argsort(x, kind="stable").astype(np.int64)


def _geometric_positions(key: int, total: int, p: float) -> np.ndarray:
    """Positions of successes among ``total`` independent Bernoulli(p) slots.

    Gaps between successes are Geometric(p) (Batagelj and Brandes, 2005):
    ``gap = floor(log(U) / log(1 - p))`` with ``U`` uniform in (0, 1].
    """
    if p <= 0.0 or total <= 0:
        return np.zeros(0, dtype=np.int64)
    if p >= 1.0:
        return np.arange(total, dtype=np.int64)
    lq = math.log1p(-p)
    chunks = []
    pos = -1
    offset = 0
    batch = max(1024, int(total * p * 1.05) + 64)
    while True:
        u = 1.0 - uniform_f64(key, batch, offset)  # in (0, 1]
        offset += batch
        gaps = np.floor(np.log(u) / lq).astype(np.int64) + 1
        cs = pos + np.cumsum(gaps)
        keep = cs < total
        chunks.append(cs[keep])
        if not keep.all():
            break
        pos = int(cs[-1])
        batch = max(1024, int((total - pos) * p * 1.1) + 64)
    return np.concatenate(chunks)


def er_edges(n: int, d: float, seed: int, tag: int = 0):
    """Directed Erdos-Renyi G(n, p), p = d/(n-1), no self-loops.

    Every ordered pair (u, v), u != v, is an edge independently with
    probability p.  Returns int64 arrays (src, dst) in row-major slot order.
    """
    if n <= 1:
        z = np.zeros(0, dtype=np.int64)
        return z, z.copy()
    p = min(1.0, d / (n - 1))
    s = _geometric_positions(stream_key(seed, 100 + tag), n * (n - 1), p)
    src = s // (n - 1)
    r = s % (n - 1)
    dst = r + (r >= src)
    return src.astype(np.int64), dst.astype(np.int64)


def rmat_edges(scale: int, edge_factor: int, a: float, b: float, c: float,
               seed: int, relabel: bool = True, tag: int = 0):
    """R-MAT edge list (Chakrabarti, Zhan and Faloutsos, 2004).

    ``edge_factor * 2^scale`` edges; at each of ``scale`` levels the quadrant
    is drawn with probabilities (a, b, c, 1-a-b-c): (0,0), (0,1), (1,0), (1,1)
    for (src bit, dst bit).  No noise.  Self-loops and duplicate edges are
    kept (the fold combines duplicates).  With ``relabel`` the same seeded
    random permutation is applied to sources and destinations, as the paper
    suggests for load balance (Section 5.1).
    """
    m = edge_factor << scale
    key = stream_key(seed, 200 + tag)
    src = np.zeros(m, dtype=np.int64)
    dst = np.zeros(m, dtype=np.int64)
    ab, abc = a + b, a + b + c

    def edges(e0, e1):
        # edges e0 .. e1-1: draw lvl * m + e of the stream decides level lvl
        for lvl in range(scale):
            u = uniform_f64(key, e1 - e0, lvl * m + e0)
            sbit = (u >= ab).astype(np.int64)
            dbit = (((u >= a) & (u < ab)) | (u >= abc)).astype(np.int64)
            sh = scale - 1 - lvl
            src[e0:e1] |= sbit << sh
            dst[e0:e1] |= dbit << sh

    _chunked(edges, m)
    if relabel:
        perm = permutation(stream_key(seed, 300 + tag), 1 << scale)
        src = perm[src]
        dst = perm[dst]
    return src, dst


def stencil27_edges(g: int):
    """27-point stencil on a g^3 grid: (u, v) for all v within Chebyshev
    distance 1 of u (the centre included).  Vertex id = (x*g + y)*g + z."""
    idx = np.arange(g, dtype=np.int64)
    x, y, z = np.meshgrid(idx, idx, idx, indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    srcs, dsts = [], []
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                xx, yy, zz = x + dx, y + dy, z + dz
                ok = (xx >= 0) & (xx < g) & (yy >= 0) & (yy < g) & (zz >= 0) & (zz < g)
                srcs.append(((x * g + y) * g + z)[ok])
                dsts.append(((xx * g + yy) * g + zz)[ok])
    return np.concatenate(srcs), np.concatenate(dsts)


def powerlaw_edges(n: int, gamma: float, seed: int, tag: int = 0):
    """Rows with power-law nonzero counts: P(k) proportional to k^-gamma for
    k in 1..n; columns uniform (with replacement; duplicates are combined by
    the fold).  Returned as (src=column, dst=row) so that row ``dst`` of the
    folded matrix carries the drawn count."""
    k = np.arange(1, n + 1, dtype=np.float64)
    w = k ** (-gamma)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = uniform_f64(stream_key(seed, 400 + tag), n)
    deg = np.searchsorted(cdf, u, side="right").astype(np.int64) + 1
    deg = np.minimum(deg, n)
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    cols = randint(stream_key(seed, 500 + tag), rows.size, 0, n - 1)
    return cols, rows


def bernoulli_keys(dims, p: float, seed: int, tag: int = 0, shuffle: bool = True):
    """Linearized keys (last mode fastest) of a tensor whose entries are
    present independently with probability p; returned in shuffled order."""
    total = int(np.prod(np.asarray(dims, dtype=np.int64)))
    keys = _geometric_positions(stream_key(seed, 600 + tag), total, p)
    if shuffle and keys.size:
        keys = keys[permutation(stream_key(seed, 700 + tag), keys.size)]
    return keys


def pick_sources(n: int, src_of_edges: np.ndarray, count: int, seed: int, tag: int = 0):
    """``count`` distinct vertices drawn uniformly among those with
    out-degree >= 1 (fewer if not enough exist)."""
    eligible = np.unique(src_of_edges)
    if eligible.size == 0:
        return np.zeros(0, dtype=np.int64)
    perm = permutation(stream_key(seed, 800 + tag), eligible.size)
    return np.sort(eligible[perm[:count]]).astype(np.int64)


def edge_values(kind: str, m: int, seed: int, tag: int = 0, lo: int = 1, hi: int = 100):
    """Edge values: 'f64'/'f32' uniform [0,1); 'i32' uniform integers in
    [lo, hi]; 'bool' all ones (uint8)."""
    key = stream_key(seed, 900 + tag)
    if kind == "f64":
        return uniform_f64(key, m)
    if kind == "f32":
        return uniform_f32(key, m)
    if kind == "i32":
        return randint(key, m, lo, hi).astype(np.int32)
    if kind == "bool":
        return np.ones(m, dtype=np.uint8)
    raise ValueError(kind)


def selector_panel_rows(n: int, j: int, seed: int, lo: int = 10, hi: int = 14):
    """Row set of panel j of a wide-matrix family in the selector training
    set: 2^u rows (u uniform in [lo, hi]) drawn without replacement from
    0..n-1, sorted."""
    u = uniform_f64(stream_key(seed, 6000 + j), 1)[0]
    k = min(n, int(2 ** (lo + (hi - lo) * u)))
    return np.sort(permutation(stream_key(seed, 6100 + j), n)[:k]).astype(np.int64)


def dense_graph(n: int, seed: int, lo: int = 1, hi: int = None, tag: int = 0):
    """Complete directed graph on n vertices (every ordered pair u != v) with
    integer weights uniform in [lo, hi] (hi defaults to n^2): the dense APSP
    workload of the paper's path-doubling experiment (Section 6).  Returns
    int64 (src, dst) in row-major slot order and int32 weights."""
    if hi is None:
        hi = max(lo, n * n)
    if n <= 1:
        z = np.zeros(0, dtype=np.int64)
        return z, z.copy(), np.zeros(0, dtype=np.int32)
    s = np.arange(n * (n - 1), dtype=np.int64)
    src = s // (n - 1)
    r = s % (n - 1)
    dst = r + (r >= src)
    w = randint(stream_key(seed, 1100 + tag), s.size, lo, hi).astype(np.int32)
    return src, dst, w


def er_batch_params(count: int, seed: int, nmin: float = 1e3, nmax: float = 1e5,
                    dmin: float = 4.0, dmax: float = 32.0):
    """Per-instance (n, d) for a batch of ER graphs: n log-uniform in
    [nmin, nmax], d uniform in [dmin, dmax]."""
    u = uniform_f64(stream_key(seed, 1000), count)
    v = uniform_f64(stream_key(seed, 1001), count)
    n = np.floor(np.exp(np.log(nmin) + u * (np.log(nmax) - np.log(nmin)))).astype(np.int64)
    d = dmin + v * (dmax - dmin)
    return n, d


FAMILIES = ("er", "rmat", "stencil27", "powerlaw")


def selector_matrix(i: int, seed: int):
    """Matrix i of the schedule-selector training set: family i % 4 with
    seeded parameters.  Returns (family, n, src, dst, params).  Sizes:
    ER n log-uniform in [2^12, 2^16], degree uniform in [2, 24]; R-MAT
    scale 12-15, edge factor 4-16, a uniform in [0.45, 0.70] with
    b = c = 0.19 (1 - a) / 0.43; 27-point stencil on g^3, g in [16, 40];
    power-law rows, n log-uniform in [2^12, 2^15], exponent in [1.8, 2.6]."""
    fam = FAMILIES[i % 4]
    u = uniform_f64(stream_key(seed, 5000 + i), 4)
    if fam == "er":
        n = int(2 ** (12 + 4 * u[0]))
        d = 2.0 + 22.0 * u[1]
        src, dst = er_edges(n, d, seed, tag=5000 + i)
        return fam, n, src, dst, {"n": n, "d": d}
    if fam == "rmat":
        scale = 12 + int(u[0] * 4)
        ef = 4 + int(u[1] * 13)
        a = 0.45 + 0.25 * u[2]
        b = 0.19 * (1.0 - a) / 0.43
        src, dst = rmat_edges(scale, ef, a, b, b, seed, tag=5000 + i)
        return fam, 1 << scale, src, dst, {"scale": scale, "ef": ef, "a": a}
    if fam == "stencil27":
        g = 16 + int(u[0] * 25)
        src, dst = stencil27_edges(g)
        return fam, g ** 3, src, dst, {"g": g}
    n = int(2 ** (12 + 3 * u[0]))
    gamma = 1.8 + 0.8 * u[1]
    src, dst = powerlaw_edges(n, gamma, seed, tag=5000 + i)
    return fam, n, src, dst, {"n": n, "gamma": gamma}
