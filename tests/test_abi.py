"""CPU-side checks of the C-ABI library: it loads, exports every symbol that
include/sv.h declares, validates arguments before touching the GPU, and its
host-only logic (schedules, tile planning) is right.  No kernel runs here."""
import ctypes
import math
import re
from pathlib import Path

import numpy as np
import pytest

ROOT = Path(__file__).resolve().parents[1]


@pytest.fixture(scope="module")
def sv():
    from paper_2104_03293_amd import sv as m

    return m


def declared_symbols():
    text = (ROOT / "include" / "sv.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sv_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for need in ["sv_alloc", "sv_wrap", "sv_init_plus", "sv_cost_phase", "sv_mixer", "sv_qaoa_forward",
                 "sv_aqa_run", "sv_expect", "sv_grad", "sv_ground", "sv_batch_p1_scan"]:
        assert need in names


def test_library_exports_every_declared_symbol(sv):
    lib = ctypes.CDLL(str(sv.LIB_PATH))
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_version(sv):
    assert "gfx950" in sv.version()


# ----------------------------------------------------------------------------- schedules
@pytest.mark.parametrize("steps,tau", [(20, 0.5), (20, 1.0), (7, 0.3), (1, 0.9)])
def test_linear_schedule_matches_oracle(sv, orc, steps, tau):
    for sign in (True, False):
        g, b = sv.schedule_linear(steps, tau, paper_sign=sign)
        og, ob = orc.aqa_linear_schedule(steps, tau, paper_sign=sign)
        assert np.array_equal(g, og) and np.max(np.abs(b - ob)) < 1e-15


@pytest.mark.parametrize("p", [2, 3, 13, 51])
def test_second_order_schedule_matches_oracle(sv, orc, p):
    g, b = sv.schedule_second_order(p, 0.4)
    og, ob = orc.second_order_schedule(p, 0.4)
    assert np.max(np.abs(g - og)) < 1e-15 and np.max(np.abs(b - ob)) < 1e-15
    s = np.arange(p) / (p - 1)
    A = np.cos(s)
    B = s ** 2
    g, b = sv.schedule_second_order(p, 0.8, A, B)
    og, ob = orc.second_order_schedule(p, 0.8, A, B)
    assert np.max(np.abs(g - og)) < 1e-15 and np.max(np.abs(b - ob)) < 1e-15


def test_schedule_errors(sv):
    with pytest.raises(sv.SVError) as e:
        sv.schedule_second_order(1, 0.5)
    assert e.value.code == 1
    with pytest.raises(sv.SVError) as e:
        sv.schedule_linear(0, 0.5)
    assert e.value.code == 1
    with pytest.raises(sv.SVError) as e:
        sv.schedule_linear(3, float("nan"))
    assert e.value.code == 5


# ----------------------------------------------------------------------------- validation
def _create(sv, n, h, ei, ej, J):
    h = np.asarray(h, dtype=np.float64)
    ei = np.asarray(ei, dtype=np.int32)
    ej = np.asarray(ej, dtype=np.int32)
    J = np.asarray(J, dtype=np.float64)
    out = ctypes.c_void_p()
    rc = sv.lib.sv_ising_create(n, sv._dp(h), len(J), ei.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                ej.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), sv._dp(J), ctypes.byref(out))
    return rc


@pytest.mark.parametrize("case,code", [
    ((3, [0, 0, 0], [0], [0], [1.0]), 1),          # self coupling
    ((3, [0, 0, 0], [0], [3], [1.0]), 1),          # endpoint out of range
    ((3, [0, 0, 0], [0, 1], [1, 0], [1.0, 2.0]), 1),  # pair listed twice
    ((3, [0, float("inf"), 0], [0], [1], [1.0]), 5),  # non-finite field
    ((3, [0, 0, 0], [0], [1], [float("nan")]), 5),  # non-finite coupling
    ((0, [], [], [], []), 1),                       # n < 1
    ((35, [0] * 35, [], [], []), 1),                # n too large
])
def test_ising_validation(sv, case, code):
    assert _create(sv, *case) == code
    assert sv.last_error() != ""


def test_exact_cover_validation(sv):
    out = ctypes.c_void_p()
    c = ctypes.c_double()
    bad = np.array([[0, 1, 2], [1, 0, 0]], dtype=np.uint8)
    rc = sv.lib.sv_ising_exact_cover(2, 3, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ctypes.byref(c),
                                     ctypes.byref(out))
    assert rc == 1 and "not 0/1" in sv.last_error()
    ok = np.zeros((2, 3), dtype=np.uint8)
    assert sv.lib.sv_ising_exact_cover(0, 3, ok.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), None,
                                       ctypes.byref(out)) == 1
    assert sv.lib.sv_ising_exact_cover(2, 0, ok.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), None,
                                       ctypes.byref(out)) == 1


def test_state_validation(sv):
    out = ctypes.c_void_p()
    assert sv.lib.sv_wrap(10, 2, ctypes.c_void_p(0), 1 << 20, None, ctypes.byref(out)) == 1
    assert sv.lib.sv_wrap(10, 2, ctypes.c_void_p(4096), 100, None, ctypes.byref(out)) == 1  # too small
    assert sv.lib.sv_wrap(10, 3, ctypes.c_void_p(4096), 1 << 20, None, ctypes.byref(out)) == 1  # dtype
    assert sv.lib.sv_wrap(34, 2, ctypes.c_void_p(4096), 1 << 40, None, ctypes.byref(out)) == 1  # n > 33 c128
    assert sv.lib.sv_alloc(0, 1, None, ctypes.byref(out)) == 1
    # host-only handles: a wrapped state can be made and freed without touching the GPU
    assert sv.lib.sv_wrap(10, 1, ctypes.c_void_p(4096), 1 << 13, None, ctypes.byref(out)) == 0
    st = out
    assert sv.lib.sv_mixer(st, ctypes.c_double(float("nan"))) == 5
    assert sv.lib.sv_copy_to_host(st, ctypes.c_void_p(4096), 12) == 1  # byte count mismatch
    # general layers: argument checks come before any GPU work
    U = np.zeros(10 * 8)
    U[0] = np.inf
    dp = ctypes.POINTER(ctypes.c_double)
    assert sv.lib.sv_gate_layers(st, -1, U.ctypes.data_as(dp)) == 1
    assert sv.lib.sv_gate_layers(st, 1, None) == 1
    assert sv.lib.sv_gate_layers(st, 1, U.ctypes.data_as(dp)) == 5
    assert sv.lib.sv_gate_layers(st, 0, None) == 0
    assert sv.lib.sv_gate_layers(None, 1, U.ctypes.data_as(dp)) == 1
    assert sv.lib.sv_qsds_run(st, None, 1, ctypes.c_double(0.5), U.ctypes.data_as(dp), U.ctypes.data_as(dp), 1,
                              None, None, None) == 1
    assert sv.lib.sv_free(st) == 0


def test_knobs(sv):
    assert sv.tune_get("fuse") == 1
    with pytest.raises(sv.SVError):
        sv.tune_set("no_such_knob", 1)
    with pytest.raises(sv.SVError):
        sv.tune_set("fuse", 7)


# ----------------------------------------------------------------------------- planning
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 3, 5, 9, 12, 13, 14, 15, 18, 20, 24, 26, 30, 32, 33, 34])
def test_plan_covers_every_qubit_once(sv, dtype, n):
    if dtype == "c128" and n > 33:
        pytest.skip("complex128 holds at most 33 qubits")
    d = sv.describe(n, dtype)
    for key in ("nv1", "grad_nv1", "grad_nv2"):
        groups = d["plans"][key]
        covered = []
        for gi, g in enumerate(groups):
            T, R, c, lo, gb = g["T"], g["R"], g["c"], g["lo"], g["g"]
            if gi == 0:
                active = list(range(min(n, T)))
                assert gb == 0
            else:
                active = list(range(c, T))
                assert c >= (3 if dtype == "c128" else 4), "carrier run below 128 bytes"
                assert c + gb == T and lo >= c
            # tile bit -> global bit
            glob = [l if l < c else lo + (l - c) for l in active]
            covered += glob if gi > 0 else [l for l in active]
            # blocks: every active bit is butterflied exactly once in each direction,
            # either as a register slot or as a cross-lane pair (lane position 3 or 4)
            for direction in ("fwd", "bwd"):
                seen = []
                for blk in g["blocks"]:
                    m = blk[direction]
                    seen += [blk["bits"][k] for k in range(R) if m >> k & 1]
                    tb = [l for l in range(T) if l not in blk["bits"]]
                    assert blk["dpp"] in (0, 8, 16)
                    seen += [tb[q] for q in range(6) if blk["dpp"] >> q & 1]
                assert sorted(seen) == active
            # the first layout leaves tile bits 0..5 as lane bits (coalesced loads)
            if n >= T and len(g["blocks"]) > 1:
                assert min(g["blocks"][0]["bits"]) >= 6
        assert sorted(covered) == list(range(n))


def test_tune_cache_overrides_plan(sv, tmp_path):
    """A tuned (dtype, n) override changes the plan for that size only."""
    base = sv.describe(30, "c128")["plans"]["nv1"]
    f = tmp_path / "cache.txt"
    f.write_text("c128 30 cmin128 5\nc64 30 bogus 3\n")
    sv.tune_load(f)
    try:
        tuned = sv.describe(30, "c128")["plans"]["nv1"]
        other = sv.describe(29, "c128")["plans"]["nv1"]
    finally:
        sv.tune_load(None)
    assert all(g["c"] >= 5 for g in tuned[1:])
    assert [g["c"] for g in tuned] != [g["c"] for g in base]
    assert [g["c"] for g in other] == [g["c"] for g in sv.describe(29, "c128")["plans"]["nv1"]]
    with pytest.raises(sv.SVError):
        sv.tune_load(tmp_path / "missing.txt")
    sv.tune_load(None)
