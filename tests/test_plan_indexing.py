"""CPU replay of the tile-pass addressing for every plan the library builds.

For each tile group and layout it rebuilds, exactly as the kernel does, the
global index z = base(tile) | gmap(thread bits) | gmap(register bits) and the
LDS slot swizzle(thread part) ^ swizzle(register part), then checks that every
layout visits each basis state exactly once and stays inside the state and the
LDS tile.  This runs before any kernel ever touches a buffer.
"""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def sv():
    from paper_2104_03293_amd import sv as m

    return m


def swizzle(u, G):
    x = u >> G
    f = np.zeros_like(u)
    for _ in range(6):
        f ^= x
        x >>= G
    return u ^ (f & ((1 << G) - 1))


def replay(n, g, G):
    T, R, c, lo, gb = g["T"], g["R"], g["c"], g["lo"], g["g"]
    ntiles = g["ntiles"]
    phantom = g["phantom"]
    assert ntiles == (1 << (n - T) if n > T else 1)
    NT, NR = 1 << (T - R), 1 << R
    tiles = np.arange(ntiles, dtype=np.uint64)
    nlow = lo - c
    base = ((tiles & np.uint64((1 << nlow) - 1)) << np.uint64(c)) | ((tiles >> np.uint64(nlow)) << np.uint64(lo + gb))

    def gmap(u):
        u = u.astype(np.uint64)
        return (u & np.uint64((1 << c) - 1)) | ((u >> np.uint64(c)) << np.uint64(lo))

    for blk in g["blocks"]:
        rb = blk["bits"]
        assert len(rb) == R and all(0 <= b < T for b in rb) and len(set(rb)) == R
        tb = [l for l in range(T) if l not in rb]
        t = np.arange(NT, dtype=np.int64)
        thr_u = np.zeros(NT, dtype=np.int64)
        for j, l in enumerate(tb):
            thr_u |= ((t >> j) & 1) << l
        r = np.arange(NR, dtype=np.int64)
        reg_u = np.zeros(NR, dtype=np.int64)
        for k, l in enumerate(rb):
            reg_u |= ((r >> k) & 1) << l
        u = thr_u[:, None] | reg_u[None, :]
        assert np.array_equal(np.sort(u.ravel()), np.arange(1 << T))
        lds = swizzle(thr_u, G)[:, None] ^ swizzle(reg_u, G)[None, :]
        assert np.array_equal(np.sort(lds.ravel()), np.arange(1 << T)), "LDS slots must be a permutation"
        valid = (u & phantom) == 0
        zt = (gmap(thr_u)[:, None] | gmap(reg_u)[None, :])[valid]
        z = (base[:, None] | zt[None, :]).ravel()
        assert z.max() < (1 << n)
        assert len(z) == 1 << n
        assert np.array_equal(np.sort(z), np.arange(1 << n, dtype=np.uint64))


# LDS swizzle widths the library accepts (knob ldsswz): the default 4 at every
# size, 3 and 5 at sizes that cover one, two and three tile groups
BIJECTION_CASES = [(n, 4) for n in (1, 2, 4, 7, 9, 12, 13, 14, 15, 16, 19, 21, 24)] + [
    (n, G) for n in (7, 14, 16, 21) for G in (3, 5)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,G", BIJECTION_CASES)
def test_every_layout_is_a_bijection(sv, dtype, n, G):
    d = sv.describe(n, dtype)
    for key in ("nv1", "grad_nv1", "grad_nv2"):
        for g in d["plans"][key]:
            replay(n, g, G)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [26, 30, 32, 33, 34])
def test_large_plans_in_bounds(sv, dtype, n):
    """Full-size plans: check bounds on the first and last tiles only."""
    if dtype == "c128" and n > 33:
        pytest.skip("complex128 holds at most 33 qubits")
    d = sv.describe(n, dtype)
    for key in ("nv1", "grad_nv1", "grad_nv2"):
        for g in d["plans"][key]:
            T, c, lo, gb = g["T"], g["c"], g["lo"], g["g"]
            assert g["ntiles"] == 1 << (n - T)
            nlow = lo - c
            w = g["ntiles"] - 1
            base = ((w & ((1 << nlow) - 1)) << c) | ((w >> nlow) << (lo + gb))
            top = base | ((1 << c) - 1) | (((1 << gb) - 1) << lo)
            assert top == (1 << n) - 1


def bank_extra_cycles(g, G, lanes_per_cycle, pivot):
    """Extra LDS cycles of one exchange write/read over all registers of every
    layout, when `lanes_per_cycle` consecutive lanes are served together and a
    cycle covers that many consecutive element slots (modulo)."""
    T, R = g["T"], g["R"]
    extra = 0
    for blk in g["blocks"]:
        rb = blk["bits"]
        tb = [l for l in range(T) if l not in rb]
        regs = range(1 << (R - 1)) if pivot else range(1 << R)
        lane = np.arange(64)
        thr = np.zeros(64, dtype=np.int64)
        for j in range(6):
            thr |= ((lane >> j) & 1) << tb[j]
        for r in regs:
            ru = sum(((r >> k) & 1) << rb[k] for k in range(R))
            u = thr | ru
            if pivot:
                u &= (1 << (T - 1)) - 1
            slot = swizzle(u, G) % lanes_per_cycle
            for w0 in range(0, 64, lanes_per_cycle):
                extra += np.bincount(slot[w0:w0 + lanes_per_cycle], minlength=lanes_per_cycle).max() - 1
    return int(extra)


@pytest.mark.parametrize("n", [14, 20, 23, 26, 30, 32, 33])
def test_complex128_exchanges_conflict_free(sv, n):
    """Every complex128 exchange slot pattern is free of LDS bank conflicts
    whether 8 or 16 lanes of 16-B elements are served per cycle."""
    d = sv.describe(n, "c128")
    for key in ("nv1", "grad_nv1", "grad_nv2"):
        for g in d["plans"][key]:
            for lanes in (8, 16):
                assert bank_extra_cycles(g, 4, lanes, key != "grad_nv2") == 0, (key, g["c"], lanes)
