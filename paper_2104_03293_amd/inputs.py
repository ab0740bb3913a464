"""Seeded synthetic inputs: Ising instances, parameter sets and scan grids.

This module only draws random numbers and builds arrays.  It holds none of the
simulation's arithmetic (no energies, phases, butterflies, schedules or
reductions), so that both the HIP path and the CPU oracle can consume the same
inputs without sharing any computation.

Instance layout (plain dict of numpy arrays):
  n  : number of qubits / Ising spins
  h  : float64[n]   local fields h_i           (Eq. HC, Sec. III.A.1)
  ei : int32[m]     first endpoint i of each coupling, i < j
  ej : int32[m]     second endpoint j
  J  : float64[m]   coupling J_ij              (Eq. HC)

The paper's own workload (exact-cover instances with F=472 clauses, Sec. III.A.3)
is not available; random Ising instances of the shapes below stand in for it.
"""
from __future__ import annotations

import math

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def regular3_edges(n: int, rng: np.random.Generator) -> np.ndarray:
    """Random 3-regular simple graph by the pairing (configuration) model.

    Shuffle 3n stubs, pair neighbours, reject on self-loops or repeated pairs.
    For odd n, 3n is odd and no 3-regular graph exists: one stub of a uniformly
    chosen vertex is dropped, leaving that vertex with degree 2 and (3n-1)/2 edges.
    Returns int64[m, 2] with i < j, rows sorted.
    """
    if n < 4:
        raise ValueError("3-regular graph needs n >= 4")
    stubs = np.repeat(np.arange(n), 3)
    if n % 2 == 1:
        drop = int(rng.integers(n))
        stubs = np.delete(stubs, 3 * drop)
    for _ in range(100000):
        perm = rng.permutation(stubs)
        pairs = np.sort(perm.reshape(-1, 2), axis=1)
        if np.any(pairs[:, 0] == pairs[:, 1]):
            continue
        key = pairs[:, 0] * n + pairs[:, 1]
        if len(np.unique(key)) != len(key):
            continue
        order = np.lexsort((pairs[:, 1], pairs[:, 0]))
        return pairs[order]
    raise RuntimeError("pairing model did not produce a simple graph")


def gnm_edges(n: int, m: int, rng: np.random.Generator) -> np.ndarray:
    """G(n, M): m distinct unordered pairs drawn uniformly without replacement."""
    npairs = n * (n - 1) // 2
    if m > npairs:
        raise ValueError("too many edges")
    idx = np.sort(rng.choice(npairs, size=m, replace=False))
    # decode pair index -> (i, j), i < j, row-major over the upper triangle
    out = np.empty((m, 2), dtype=np.int64)
    starts = np.array([i * n - i * (i + 1) // 2 for i in range(n)], dtype=np.int64)
    for k, t in enumerate(idx):
        i = int(np.searchsorted(starts, t, side="right") - 1)
        j = int(t - starts[i] + i + 1)
        out[k] = (i, j)
    return out


def make_instance(n: int, edges: np.ndarray, h: np.ndarray, J: np.ndarray) -> dict:
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return {
        "n": int(n),
        "h": np.ascontiguousarray(h, dtype=np.float64),
        "ei": np.ascontiguousarray(edges[:, 0], dtype=np.int32),
        "ej": np.ascontiguousarray(edges[:, 1], dtype=np.int32),
        "J": np.ascontiguousarray(J, dtype=np.float64),
    }


def regular3_pm1(n: int, seed: int) -> dict:
    """3-regular graph, J_ij uniform in {-1,+1}, h_i uniform in {-1,0,+1}."""
    rng = _rng(seed)
    e = regular3_edges(n, rng)
    J = rng.choice(np.array([-1.0, 1.0]), size=len(e))
    h = rng.integers(-1, 2, size=n).astype(np.float64)
    return make_instance(n, e, h, J)


def degree4_int2(n: int, seed: int) -> dict:
    """G(n, 2n) (average degree 4), J_ij uniform integers in [-2,2], h_i in {-1,0,1}.

    Couplings drawn as 0 are kept as edges (they are inert)."""
    rng = _rng(seed)
    e = gnm_edges(n, 2 * n, rng)
    J = rng.integers(-2, 3, size=len(e)).astype(np.float64)
    h = rng.integers(-1, 2, size=n).astype(np.float64)
    return make_instance(n, e, h, J)


def random_real(n: int, m: int, seed: int, hscale: float = 1.0, jscale: float = 1.0) -> dict:
    """G(n, m) with real-valued fields and couplings (uniform in [-scale, scale])."""
    rng = _rng(seed)
    e = gnm_edges(n, m, rng)
    J = rng.uniform(-jscale, jscale, size=len(e))
    h = rng.uniform(-hscale, hscale, size=n)
    return make_instance(n, e, h, J)


def ring(n: int, J: float = 1.0, h: float = 0.0) -> dict:
    e = np.array([(i, (i + 1) % n) for i in range(n)])
    e = np.sort(e, axis=1)
    return make_instance(n, e, np.full(n, h), np.full(n, J))


def fields_only(n: int, seed: int) -> dict:
    """No couplings (product-state Hamiltonian), h_i uniform in {-1,0,1}."""
    rng = _rng(seed)
    h = rng.integers(-1, 2, size=n).astype(np.float64)
    return make_instance(n, np.zeros((0, 2), dtype=np.int64), h, np.zeros(0))


def exact_cover_matrix(nrows: int, ncols: int, seed: int, nplanted: int | None = None) -> np.ndarray:
    """Boolean problem matrix a in {0,1}^{nrows x ncols} of an exact cover
    instance (Sec. III.A.3 shape: N rows = qubits, F columns) with a planted
    solution: `nplanted` rows (default nrows // 4) partition the columns (each
    column in exactly one of them), every other row covers a uniformly random
    column subset of the same expected size.  Only random draws; the Ising
    form of the instance is computed by the library and by the oracle."""
    rng = _rng(seed)
    k = nplanted if nplanted is not None else max(1, nrows // 4)
    a = np.zeros((nrows, ncols), dtype=np.uint8)
    rows = rng.permutation(nrows)
    planted = rows[:k]
    a[planted[rng.integers(0, k, size=ncols)], np.arange(ncols)] = 1
    for r in rows[k:]:
        a[r] = (rng.random(ncols) < 1.0 / k).astype(np.uint8)
    return a


# --- the benchmark workloads ----------------------------------------------------------

def small_regular3_instance() -> dict:
    """n=14, 3-regular, J in {-1,+1}, h in {-1,0,1}, seed 0."""
    return regular3_pm1(14, 0)


SMALL_GAMMA, SMALL_BETA = 0.4, 0.3


def aqa_degree4_instance(n: int = 26) -> dict:
    """n=26, G(26,52), integer J in [-2,2], h in {-1,0,1}, seed 1."""
    return degree4_int2(n, 1)


def grad_degree4_instance(n: int = 30) -> dict:
    return degree4_int2(n, 2)


def batch_instances(count: int = 2048, nmin: int = 10, nmax: int = 18, base_seed: int = 3000) -> list:
    """Batched scan: instance k has n ~ U{nmin..nmax} (drawn from seed base_seed+k)."""
    out = []
    for k in range(count):
        rng = _rng(base_seed + k)
        n = int(rng.integers(nmin, nmax + 1))
        out.append(regular3_pm1(n, base_seed + k))
    return out


def batch_grid(ng: int = 32, nb: int = 32):
    """Half-open grid gamma_a = a*pi/ng, beta_b = (pi/2)*b/nb (a, b = 0..ng-1, nb-1)."""
    g = np.arange(ng) * (math.pi / ng)
    b = np.arange(nb) * (0.5 * math.pi / nb)
    return g, b


def full_size_instance(n: int) -> dict:
    return degree4_int2(n, 4 + n)


def linear_ramp_params(p: int, tau: float = 0.5):
    """Parameter set used for the QAOA gradient workloads: gamma_k = tau*k/p,
    beta_k = -tau*(1 - k/p), k = 1..p (an annealing-like ramp)."""
    k = np.arange(1, p + 1, dtype=np.float64)
    return tau * k / p, -tau * (1.0 - k / p)


def uniform_params(p: int, seed: int, lo: float = -1.0, hi: float = 1.0):
    rng = _rng(seed)
    return rng.uniform(lo, hi, size=p), rng.uniform(lo, hi, size=p)


def block_instance(n: int, seed: int, block: int = 5) -> dict:
    """Ising instance whose coupling graph is a union of disjoint cliques: a seeded
    random permutation of the n qubits is cut into consecutive blocks of `block`
    qubits (the last one takes the remainder), every pair inside a block is
    coupled with J uniform integer in [-2, 2] (zeros kept), h_i uniform in
    {-1, 0, 1}.  The blocks scatter over all bit positions, so at full size every
    tile group holds qubits of coupled pairs.  Only random draws."""
    rng = _rng(seed)
    perm = rng.permutation(n)
    edges = []
    for b0 in range(0, n, block):
        qs = np.sort(perm[b0:b0 + block])
        for a in range(len(qs)):
            for c in range(a + 1, len(qs)):
                edges.append((int(qs[a]), int(qs[c])))
    edges = np.array(sorted(edges), dtype=np.int64).reshape(-1, 2)
    J = rng.integers(-2, 3, size=len(edges)).astype(np.float64)
    h = rng.integers(-1, 2, size=n).astype(np.float64)
    return make_instance(n, edges, h, J)
