"""Seeded synthetic workloads for the D-iteration PageRank solver.

This module only *generates inputs*: graphs (source-ordered CSR), personalization
seed sets, random fluid states for single-round checks, and Poisson request
streams.  It holds none of the method's arithmetic, and both the CPU oracle
(tests / baseline timing) and the GPU library consume what it produces.

Graph recipes follow the workloads the D-iteration is evaluated on (Section 4:
power-law web-like graphs with many dangling nodes, and a 10^6-node web crawl):
out-degree drawn from a shifted Zipf law with exponent 2.1 (the shift is solved
so that the requested mean holds), a fixed fraction of dangling nodes, and
preferential-attachment targets; the "web" recipe adds host blocks of
consecutive ids with most links staying inside a block.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib_handle = None


def build(force: bool = True) -> str:
    """Compile the generator with g++ into workloads/libgraphgen.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.wl_zipf_shift.restype = ctypes.c_double
        lib.wl_zipf_shift.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double]
        lib.wl_outdeg.restype = ctypes.c_int64
        lib.wl_outdeg.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int, ctypes.c_double, ctypes.c_uint64,
                                  ctypes.c_void_p]
        lib.wl_targets.restype = ctypes.c_int
        lib.wl_targets.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_uint64]
        _lib_handle = lib
    return _lib_handle


@dataclasses.dataclass
class Graph:
    """Directed graph as source-ordered CSR: the out-links of node i are
    col_idx[row_ptr[i]:row_ptr[i+1]].  A node with no out-link is dangling."""
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col_idx: np.ndarray  # int32[m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def outdeg(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    @property
    def n_dangling(self) -> int:
        return int(np.count_nonzero(self.outdeg == 0))

    def edges(self):
        """(src, dst) arrays, one entry per edge."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.outdeg)
        return src, self.col_idx.astype(np.int64)


def from_edges(n: int, src, dst, name: str = "") -> Graph:
    """CSR from an edge list (self-loops and repeated edges kept as given)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int64)
    return Graph(n, row_ptr, dst.astype(np.int32), name)


def powerlaw(n: int, mean: float, dangling: float, kmax: int, seed: int,
             alpha: float = 2.1, block: int = 0, p_intra: float = 0.0,
             p_uniform: float = 0.1, name: str = "") -> Graph:
    """Power-law graph: shifted-Zipf(alpha) out-degrees on [1,kmax] with overall
    mean `mean` (dangling nodes included), `dangling` fraction of degree-0 nodes,
    growing-network preferential-attachment targets with a p_uniform share of
    uniform links; block>0 adds host blocks of `block` ids with a p_intra
    share of intra-block links."""
    lib = _lib()
    kmax = int(min(kmax, n - 1))
    target = mean / (1.0 - dangling)
    shift = lib.wl_zipf_shift(alpha, kmax, target)
    if shift < 0:
        raise ValueError("mean %.3f unreachable with kmax=%d" % (target, kmax))
    outdeg = np.empty(n, dtype=np.int32)
    m = lib.wl_outdeg(n, alpha, shift, kmax, dangling, seed, outdeg.ctypes.data)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(outdeg, out=row_ptr[1:])
    assert row_ptr[-1] == m
    col_idx = np.empty(m, dtype=np.int32)
    rc = lib.wl_targets(n, row_ptr.ctypes.data, col_idx.ctypes.data, block,
                        p_intra, p_uniform, seed)
    if rc != 0:
        raise ValueError("degree sequence not realisable")
    return Graph(n, row_ptr, col_idx, name or "powerlaw-n%d" % n)


# Named recipes.  Sizes, exponents and dangling fractions are those of the
# single-solve, web-shaped, batched and serving workloads; kmax=1000 for the
# larger graphs is a chosen cap.
RECIPES = {
    "pagerank-10k": dict(n=10_000, mean=8.0, dangling=0.10, kmax=200, seed=1),
    "powerlaw-1m": dict(n=1_000_000, mean=10.0, dangling=0.10, kmax=1000, seed=2),
    "web-20m": dict(n=20_000_000, mean=15.0, dangling=0.15, kmax=1000, seed=3,
                    block=1000, p_intra=0.8),
    "serve-100k": dict(n=100_000, mean=10.0, dangling=0.10, kmax=1000, seed=51),
    "serve-500k": dict(n=500_000, mean=10.0, dangling=0.10, kmax=1000, seed=52),
    "serve-1m": dict(n=1_000_000, mean=10.0, dangling=0.10, kmax=1000, seed=53),
    "serve-5m": dict(n=5_000_000, mean=10.0, dangling=0.10, kmax=1000, seed=54),
}


def recipe(name: str, **override) -> Graph:
    kw = dict(RECIPES[name])
    kw.update(override)
    return powerlaw(name=name, **kw)


# ---------------------------------------------------------------- small graphs

def cycle(n: int) -> Graph:
    s = np.arange(n)
    return from_edges(n, s, (s + 1) % n, "cycle%d" % n)


def in_star(k: int) -> Graph:
    """k leaves 1..k each linking to a dangling centre 0."""
    return from_edges(k + 1, np.arange(1, k + 1), np.zeros(k, np.int64), "instar%d" % k)


def out_star(k: int) -> Graph:
    """Centre 0 linking to k dangling leaves."""
    return from_edges(k + 1, np.zeros(k, np.int64), np.arange(1, k + 1), "outstar%d" % k)


def bi_star(k: int) -> Graph:
    """Centre 0 linked both ways with each of k leaves."""
    leaves = np.arange(1, k + 1)
    return from_edges(k + 1, np.concatenate([np.zeros(k, np.int64), leaves]),
                      np.concatenate([leaves, np.zeros(k, np.int64)]), "bistar%d" % k)


def random_small(n: int, m: int, seed: int, p_dangling: float = 0.2,
                 self_loops: bool = True, multi: bool = True) -> Graph:
    """Uniform random multigraph with a dangling share, for property tests.
    When m >= the number of non-dangling nodes each of them has an out-link."""
    rng = np.random.default_rng(seed)
    live = rng.random(n) >= p_dangling
    if not live.any():
        live[rng.integers(n)] = True
    srcs = np.flatnonzero(live)
    # every non-dangling node gets at least one out-link
    extra = rng.choice(srcs, size=max(m - len(srcs), 0))
    src = np.concatenate([srcs, extra]) if m >= len(srcs) else rng.choice(srcs, size=m)
    dst = rng.integers(0, n, size=len(src))
    if not self_loops:
        clash = src == dst
        dst[clash] = (dst[clash] + 1) % n
    if not multi:
        pairs = np.unique(np.stack([src, dst], 1), axis=0)
        src, dst = pairs[:, 0], pairs[:, 1]
    return from_edges(n, src, dst, "rand%d_%d_%d" % (n, m, seed))


# ------------------------------------------------------------ other inputs

def modify_graph(g: Graph, frac: float, seed: int) -> Graph:
    """A changed copy of g (a graph update): a fraction `frac` of the nodes,
    chosen uniformly, get a new out-link list -- degree changed by -2..+2
    (10% of them become dangling), targets uniform over the other nodes,
    without repeats.  The other rows are kept as they are."""
    rng = np.random.default_rng(seed)
    n = g.n
    deg = np.diff(g.row_ptr)
    chosen = np.zeros(n, dtype=bool)
    chosen[rng.choice(n, size=max(1, int(frac * n)), replace=False)] = True
    src_old = np.repeat(np.arange(n, dtype=np.int64), deg)
    keep = ~chosen[src_old]
    srcs, dsts = [src_old[keep]], [g.col_idx[keep].astype(np.int64)]
    for i in np.nonzero(chosen)[0]:
        k = 0 if rng.random() < 0.1 else int(np.clip(deg[i] + rng.integers(-2, 3), 1, n - 1))
        if k == 0:
            continue
        t = rng.choice(n - 1, size=k, replace=False)
        t = t + (t >= i)  # no self-link
        srcs.append(np.full(k, i, dtype=np.int64))
        dsts.append(t.astype(np.int64))
    return from_edges(n, np.concatenate(srcs), np.concatenate(dsts), g.name + "-mod")


# The six synthetic scenarios of the paper's simulation section (N, alpha, L);
# the dangling counts the paper's tables print for them are test fixtures.
PAPER_SCENARIOS = {
    "S1": (10_000, 2.0, 2172), "S2": (10_000, 2.0, 8081), "S3": (10_000, 2.0, 28507),
    "S1b": (10_000, 1.5, 12624), "S2b": (10_000, 1.5, 61189), "S3b": (10_000, 1.5, 265245),
}


def paper_scenario(name: str, seed: int = 1) -> Graph:
    """The paper's simulation graphs (simulation scenario of Section 4.1): the
    source and the destination of each link are drawn independently, node k
    with probability proportional to 1/k^alpha, each of the two laws carried
    to the nodes by N random transpositions of the rank order (so node order
    carries no bias).  Reading of what the text leaves open: links are drawn
    until L distinct ones exist, self-links are redrawn."""
    n, alpha, L = PAPER_SCENARIOS[name]
    rng = np.random.default_rng(seed)

    def law():
        p = 1.0 / np.arange(1, n + 1, dtype=np.float64) ** alpha
        p /= p.sum()
        perm = np.arange(n)
        for a, b in zip(rng.integers(0, n, n), rng.integers(0, n, n)):
            perm[a], perm[b] = perm[b], perm[a]
        q = np.empty(n)
        q[perm] = p
        return q

    ps, pd = law(), law()
    uniq = np.zeros(0, dtype=np.int64)  # distinct links so far, in order of first draw
    k = 2 * L + 1000
    while len(uniq) < L:
        s = rng.choice(n, k, p=ps)
        d = rng.choice(n, k, p=pd)
        keep = s != d
        codes = np.concatenate([uniq, s[keep].astype(np.int64) * n + d[keep]])
        _, first = np.unique(codes, return_index=True)
        uniq = codes[np.sort(first)]
        k *= 2
    chosen = uniq[:L]
    return from_edges(n, chosen // n, chosen % n, "paper-" + name)


def random_weights(g: Graph, seed: int) -> np.ndarray:
    """Link weights for g: positive, uniform in (0.05, 1], each non-empty row
    normalised to sum to one."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.05, 1.0, size=g.m)
    deg = np.diff(g.row_ptr)
    src = np.repeat(np.arange(g.n), deg)
    tot = np.bincount(src, weights=w, minlength=g.n)
    return w / tot[src]


def uniform_v(n: int) -> np.ndarray:
    return np.full(n, 1.0 / n)


def ppr_seed_sets(n: int, count: int, smax: int, seed: int):
    """`count` seed sets, sizes floor(exp(U(0, ln(smax+1)))) clipped to
    [1, smax] (log-uniform), members uniform without replacement.
    Returns (seed_ptr int64[count+1], seeds int32[...])."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(0.0, np.log(smax + 1), size=count)))
    sizes = np.clip(sizes, 1, min(smax, n)).astype(np.int64)
    sets = [np.sort(rng.choice(n, size=int(s), replace=False)) for s in sizes]
    ptr = np.zeros(count + 1, dtype=np.int64)
    np.cumsum(sizes, out=ptr[1:])
    seeds = np.concatenate(sets).astype(np.int32) if sets else np.zeros(0, np.int32)
    return ptr, seeds


def seed_vector(n: int, seeds) -> np.ndarray:
    """Personalization vector uniform over a seed set."""
    v = np.zeros(n)
    v[np.asarray(seeds)] = 1.0 / len(seeds)
    return v


def random_fluid(n: int, seed: int, nonzero: float = 0.6, scale: float = 1e-3):
    """A random non-negative FP32 fluid vector and FP64 history vector (one
    diffusion round's state), with exact zeros mixed in."""
    rng = np.random.default_rng(seed)
    f = (rng.exponential(scale / n, size=n) * (rng.random(n) < nonzero)).astype(np.float32)
    h = rng.exponential(1.0 / n, size=n)
    return f, h


def poisson_stream(rate: float, duration: float, n_graphs: int, smax: int,
                   tols, seed: int):
    """Open-loop Poisson request stream: arrival times, graph ids, seed-set
    sizes (log-uniform on [1,smax]) and per-request tolerances."""
    rng = np.random.default_rng(seed)
    count = rng.poisson(rate * duration)
    t = np.sort(rng.uniform(0.0, duration, size=count))
    gid = rng.integers(0, n_graphs, size=count)
    sizes = np.clip(np.floor(np.exp(rng.uniform(0, np.log(smax + 1), size=count))),
                    1, smax).astype(np.int64)
    tol = np.asarray(tols)[rng.integers(0, len(tols), size=count)]
    sub = rng.integers(0, 2**63 - 1, size=count, dtype=np.int64)
    return t, gid, sizes, tol, sub


def request_seeds(n: int, size: int, subseed: int) -> np.ndarray:
    rng = np.random.default_rng(int(subseed))
    return np.sort(rng.choice(n, size=min(size, n), replace=False)).astype(np.int32)
