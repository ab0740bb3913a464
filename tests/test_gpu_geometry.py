"""Parity at the tile geometries and depths of the full-size workloads, through
the C ABI, against the FP64 oracle.

* Element-wise at sizes with three tile groups (complex128 n = 24, 26, 28;
  complex64 n = 25, 26, 28), integer and real-valued instances, p = 3 and 4
  (both snake directions, the phase between two mixers of one group): the
  state of the fused energy evaluation, the adjoint gradient (p = 3) and the
  per-step observables of an annealing run.
* The same with the largest-first group split (knob split = 1), which puts
  group B at bits 13..22 with 3 carrier bits: the group-B tile geometry of the
  n = 32 complex128 workload.
* Depth p = 8 (the 16-parameter gradient workload): the adjoint against the
  oracle's forward-mode gradient at n = 12, 16, 20, and against central
  differences of the oracle energy at n = 20.
* Full size (n = 32 in both precisions, n = 33 complex128, n = 34 complex64)
  with couplings: instances whose coupling graph is a set of disjoint 5-qubit
  cliques scattered over all bit positions, so every tile group holds coupled
  qubits.  The QAOA state is then the tensor product of the cliques' states
  (oracle.block_states): sampled amplitudes, <H_C>, P_gs, the adjoint gradient
  and per-step annealing observables are compared with it.

Tolerances as in test_gpu_parity: amplitudes 1e-11 (complex128) / 2e-5
(complex64), at full size scaled by the typical amplitude 2^{-(n-20)/2};
energies 1e-6 * max(|E|, sum|h| + sum|J|); probabilities 1e-11 / 1e-6;
gradients GRAD_TOL * max(max|g|, sum|h| + sum|J|).  The achieved errors are
recorded (printed per case and summarised at the end of the run).
"""
import sys
from pathlib import Path

import numpy as np
import pytest

from paper_2104_03293_amd import inputs as I

pytestmark = pytest.mark.gpu

AMP_TOL = {"c128": 1e-11, "c64": 2e-5}
PROB_TOL = {"c128": 1e-11, "c64": 1e-6}
GRAD_TOL = {"c128": 1e-6, "c64": 5e-6}
GIB = 1 << 30


@pytest.fixture(scope="module")
def sv():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2104_03293_amd import sv as m

    return m


@pytest.fixture(autouse=True)
def _announce(request):
    import torch

    print(f"\n[gpu] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def need_free(nbytes):
    import torch

    free, _ = torch.cuda.mem_get_info()
    if free < nbytes + 2 * GIB:
        pytest.skip(f"needs {nbytes / GIB:.0f} GiB free device memory, {free / GIB:.0f} GiB available")


def energy_tol(orc, inst, ref):
    return 1e-6 * max(abs(ref), orc.coeff_scale(inst), 1.0)


def grad_scale(orc, inst, rg, rb):
    return max(float(np.max(np.abs(np.concatenate([rg, rb])))), orc.coeff_scale(inst))


def instance(n, kind, seed):
    if kind == "int":
        return I.degree4_int2(n, seed)
    return I.random_real(n, 2 * n, seed)


class Knob:
    """Set a plan knob for the duration of a block."""

    def __init__(self, sv, name, value):
        self.sv, self.name, self.value = sv, name, value

    def __enter__(self):
        self.old = self.sv.tune_get(self.name)
        self.sv.tune_set(self.name, self.value)

    def __exit__(self, *exc):
        self.sv.tune_set(self.name, self.old)


THREE_GROUP = [("c128", 24), ("c128", 26), ("c128", 28), ("c64", 25), ("c64", 26), ("c64", 28)]


# ----------------------------------------------------------------------------- three tile groups, element-wise
@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("dtype,n", THREE_GROUP)
def test_three_group_energy_evaluation(sv, orc, record_error, dtype, n, split):
    """Final state, <H_C>, P_gs and norm of the fused energy evaluation (p = 4
    on an integer instance, p = 3 on a real-valued one) element by element."""
    with Knob(sv, "split", split):
        plan = sv.describe(n, dtype)["plans"]["nv1"]
        assert len(plan) == 3, plan
        if split == 1 and dtype == "c128":
            assert (plan[1]["c"], plan[1]["lo"], plan[1]["g"]) == (3, 13, 10)
        for kind, p in (("int", 4), ("real", 3)):
            inst = instance(n, kind, 300 + n + 7 * split + (kind == "real"))
            H = sv.Ising.from_instance(inst)
            g, b = I.uniform_params(p, 310 + n + p, -1.1, 1.1)
            s = sv.State(n, dtype)
            e, pg, nrm = sv.qaoa_energy(s, H, g, b)
            E = orc.energies(inst)
            ref = orc.qaoa_state(inst, g, b, E=E)
            err = float(np.max(np.abs(s.to_numpy() - ref)))
            record_error(f"amp max-abs {dtype}", err)
            assert err <= AMP_TOL[dtype], (kind, err)
            _, ren, rpg = orc.observables(inst, ref, E=E)
            record_error(f"energy rel {dtype}", abs(e - ren) / max(abs(ren), 1.0))
            assert abs(e - ren) <= energy_tol(orc, inst, ren)
            assert abs(pg - rpg) <= PROB_TOL[dtype]
            assert abs(nrm - 1.0) <= (1e-12 if dtype == "c128" else 1e-5)
            del s, ref, E


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("dtype,n", [("c128", 24), ("c128", 26), ("c64", 25), ("c64", 26)])
def test_three_group_gradient(sv, orc, record_error, dtype, n, split):
    """Adjoint gradient (p = 3) against the oracle's forward-mode gradient."""
    p = 3
    with Knob(sv, "split", split):
        assert len(sv.describe(n, dtype)["plans"]["grad_nv2"]) == 3
        for kind in ("int", "real"):
            inst = instance(n, kind, 330 + n + 7 * split + (kind == "real"))
            H = sv.Ising.from_instance(inst)
            g, b = I.uniform_params(p, 340 + n, -1.0, 1.0)
            psi, lam = sv.State(n, dtype), sv.State(n, dtype)
            e, pg, dg, db = sv.grad(psi, lam, H, g, b, with_pgs=True)
            del psi, lam
            E = orc.energies(inst)
            f, rg, rb = orc.grad_tangent(inst, g, b, E=E)
            scale = grad_scale(orc, inst, rg, rb)
            gerr = max(np.max(np.abs(dg - rg)), np.max(np.abs(db - rb)))
            record_error(f"grad / scale {dtype}", gerr / scale)
            record_error(f"grad / max|g| {dtype}", gerr / max(np.max(np.abs(np.concatenate([rg, rb]))), 1e-300))
            assert abs(e - f) <= energy_tol(orc, inst, f)
            assert gerr <= GRAD_TOL[dtype] * scale, (kind, gerr, scale)


@pytest.mark.parametrize("dtype,n", [("c128", 24), ("c128", 26), ("c64", 25), ("c64", 26)])
def test_three_group_annealing_observables(sv, orc, record_error, dtype, n):
    """Per-step <H_C>, P_gs and <sigma^z_i> of a coarse annealing run (the sums
    ride in the pass that ends each step) and the final state."""
    inst = instance(n, "int", 360 + n)
    H = sv.Ising.from_instance(inst)
    steps = 5
    g, b = sv.schedule_linear(steps, 0.7)
    s = sv.State(n, dtype)
    pg, en, sz = sv.aqa_run_observe(s, H, g, b)
    E = orc.energies(inst)
    gs = orc.ground(inst, E)
    psi = orc.plus_state(n)
    for k in range(steps):
        psi = orc.qaoa_state(inst, [g[k]], [b[k]], psi0=psi, E=E)
        _, ren, rpg = orc.observables(inst, psi, E=E, gs=gs)
        assert abs(en[k] - ren) <= energy_tol(orc, inst, ren), k
        assert abs(pg[k] - rpg) <= PROB_TOL[dtype], k
        serr = float(np.max(np.abs(sz[k] - orc.spin_z(n, psi))))
        record_error(f"spin max-abs {dtype}", serr)
        assert serr <= PROB_TOL[dtype] * 10, (k, serr)
    err = float(np.max(np.abs(s.to_numpy() - psi)))
    record_error(f"amp max-abs {dtype}", err)
    assert err <= AMP_TOL[dtype]


# ----------------------------------------------------------------------------- p = 8 (the gradient workload depth)
@pytest.mark.parametrize("params", ["ramp", "uniform"])
@pytest.mark.parametrize("n", [12, 16, 20])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_grad_p8_vs_oracle(sv, orc, record_error, dtype, n, params):
    """16 parameters: energy, P_gs and the adjoint gradient against the oracle's
    forward-mode tangents, on the degree-4 integer workload family."""
    p = 8
    inst = I.degree4_int2(n, 2 + n)
    H = sv.Ising.from_instance(inst)
    g, b = I.linear_ramp_params(p) if params == "ramp" else I.uniform_params(p, 370 + n, -1.0, 1.0)
    psi, lam = sv.State(n, dtype), sv.State(n, dtype)
    e, pg, dg, db = sv.grad(psi, lam, H, g, b, with_pgs=True)
    E = orc.energies(inst)
    f, rg, rb = orc.grad_tangent(inst, g, b, E=E)
    _, _, rpg = orc.observables(inst, orc.qaoa_state(inst, g, b, E=E), E=E)
    scale = grad_scale(orc, inst, rg, rb)
    gerr = max(np.max(np.abs(dg - rg)), np.max(np.abs(db - rb)))
    record_error(f"grad / scale {dtype}", gerr / scale)
    record_error(f"grad / max|g| {dtype}", gerr / np.max(np.abs(np.concatenate([rg, rb]))))
    record_error(f"energy rel {dtype}", abs(e - f) / max(abs(f), 1.0))
    assert abs(e - f) <= energy_tol(orc, inst, f)
    assert abs(pg - rpg) <= PROB_TOL[dtype]
    assert gerr <= GRAD_TOL[dtype] * scale, (gerr, scale)


def test_grad_p8_n20_vs_oracle_central_differences(sv, orc, record_error):
    """n = 20, p = 8: the complex128 adjoint against central differences of the
    oracle energy (Richardson pair h = 1e-4, 5e-5), a reference that involves
    neither the GPU nor the oracle's tangents."""
    n, p = 20, 8
    inst = I.degree4_int2(n, 2 + n)
    H = sv.Ising.from_instance(inst)
    g, b = I.linear_ramp_params(p)
    psi, lam = sv.State(n, "c128"), sv.State(n, "c128")
    e, dg, db = sv.grad(psi, lam, H, g, b)
    E = orc.energies(inst)
    fg, fb = orc.grad_fd(inst, g, b, h=1e-4, E=E)
    scale = grad_scale(orc, inst, fg, fb)
    gerr = max(np.max(np.abs(dg - fg)), np.max(np.abs(db - fb)))
    record_error("grad vs FD / scale c128", gerr / scale)
    assert gerr <= GRAD_TOL["c128"] * scale


# ----------------------------------------------------------------------------- full size, coupled instances
FULL = [("c128", 32), ("c64", 32), ("c128", 33), ("c64", 34)]
TUNE_CACHE = Path(__file__).resolve().parents[1] / "paper_2104_03293_amd" / "tune_cache.txt"


@pytest.fixture
def bench_plan(sv):
    """The plan knobs the benchmark runs with: the committed autotuner cache
    (when present) on top of the built-in defaults."""
    if TUNE_CACHE.exists():
        sv.tune_load(str(TUNE_CACHE))
    yield
    sv.tune_load(None)


def sample_indices(n, count, seed):
    rng = np.random.default_rng(seed)
    z = rng.integers(0, 1 << n, size=count, dtype=np.uint64)
    return np.concatenate([np.array([0, (1 << n) - 1], dtype=np.uint64), z])


def gather(s, zs):
    import torch

    return s.tensor[torch.from_numpy(zs.astype(np.int64)).to(s.tensor.device)].cpu().numpy()


@pytest.mark.parametrize("dtype,n", FULL)
def test_block_instance_full_size_state(sv, orc, record_error, bench_plan, dtype, n):
    """p = 4 energy evaluation in the benchmark's tile geometry: 8192 sampled
    amplitudes, <H_C> and P_gs against the tensor product of the cliques' states."""
    elem = 16 if dtype == "c128" else 8
    need_free((1 << n) * elem)
    inst = I.block_instance(n, 40 + n)
    H = sv.Ising.from_instance(inst)
    g, b = I.linear_ramp_params(4)
    s = sv.State(n, dtype)
    e, pg, nrm = sv.qaoa_energy(s, H, g, b)
    blocks = orc.block_states(inst, g, b)
    zs = sample_indices(n, 8192, 50 + n)
    err = float(np.max(np.abs(gather(s, zs) - orc.block_amplitudes(blocks, zs))))
    tol = AMP_TOL[dtype] * 2.0 ** (-(n - 20) / 2)
    record_error(f"amp max-abs x 2^((n-20)/2) {dtype}", err * 2.0 ** ((n - 20) / 2))
    assert err <= tol, (err, tol)
    ren, rpg = orc.block_observables(inst, blocks)
    record_error(f"energy rel {dtype}", abs(e - ren) / max(abs(ren), 1.0))
    assert abs(e - ren) <= energy_tol(orc, inst, ren)
    assert abs(pg - rpg) <= PROB_TOL[dtype] * max(1.0, rpg)
    assert abs(nrm - 1.0) <= (1e-12 if dtype == "c128" else 1e-5)
    del s


@pytest.mark.parametrize("dtype,n", FULL)
def test_block_instance_full_size_gradient(sv, orc, record_error, bench_plan, dtype, n):
    """Adjoint gradient (p = 4, 8 parameters) at full size with couplings: the sum
    of the cliques' forward-mode gradients."""
    elem = 16 if dtype == "c128" else 8
    need_free(2 * (1 << n) * elem)
    inst = I.block_instance(n, 60 + n)
    H = sv.Ising.from_instance(inst)
    g, b = I.uniform_params(4, 70 + n, -0.9, 0.9)
    psi = sv.State(n, dtype, owner="lib")
    lam = sv.State(n, dtype, owner="lib")
    e, pg, dg, db = sv.grad(psi, lam, H, g, b, with_pgs=True)
    psi.close()
    lam.close()
    f, rg, rb = orc.block_grad(inst, g, b)
    _, rpg = orc.block_observables(inst, orc.block_states(inst, g, b))
    scale = grad_scale(orc, inst, rg, rb)
    gerr = max(np.max(np.abs(dg - rg)), np.max(np.abs(db - rb)))
    record_error(f"grad / scale {dtype}", gerr / scale)
    record_error(f"grad / max|g| {dtype}", gerr / np.max(np.abs(np.concatenate([rg, rb]))))
    assert abs(e - f) <= energy_tol(orc, inst, f)
    assert abs(pg - rpg) <= PROB_TOL[dtype] * max(1.0, rpg)
    assert gerr <= GRAD_TOL[dtype] * scale, (gerr, scale)


@pytest.mark.parametrize("dtype,n", FULL)
def test_block_instance_full_size_annealing(sv, orc, record_error, bench_plan, dtype, n):
    """Ten coarse annealing steps: per-step <H_C> and P_gs, and the final
    <sigma^z_i>, against the cliques' step-by-step states."""
    elem = 16 if dtype == "c128" else 8
    need_free((1 << n) * elem)
    inst = I.block_instance(n, 80 + n)
    H = sv.Ising.from_instance(inst)
    steps = 10
    g, b = sv.schedule_linear(steps, 0.5)
    s = sv.State(n, dtype, owner="lib")
    pg, en, sz = sv.aqa_run_observe(s, H, g, b)
    s.close()
    ren, rpg = orc.block_aqa_observables(inst, g, b)
    for k in range(steps):
        assert abs(en[k] - ren[k]) <= energy_tol(orc, inst, ren[k]), k
        assert abs(pg[k] - rpg[k]) <= PROB_TOL[dtype] * max(1.0, rpg[k]), k
    record_error(f"energy rel {dtype}", float(np.max(np.abs(en - ren) / np.maximum(np.abs(ren), 1.0))))
    # final spin expectations from the cliques' final states
    ref_sz = np.empty(n)
    for qs, psi in orc.block_states(inst, g, b):
        loc = orc.spin_z(len(qs), psi)
        for r, q in enumerate(qs):
            ref_sz[q] = loc[r]
    serr = float(np.max(np.abs(sz[-1] - ref_sz)))
    record_error(f"spin max-abs {dtype}", serr)
    assert serr <= PROB_TOL[dtype] * 10


# ----------------------------------------------------------------------------- XCD-aware tile orders
@pytest.mark.parametrize("dtype,n", [("c128", 26), ("c64", 26), ("c128", 15)])
def test_xcd_tile_orders_agree(sv, orc, record_error, dtype, n):
    """The XCD-aware tile orders only change which workgroup takes which tile;
    the per-tile partial sums are indexed by tile, so the state, the observables
    and the adjoint gradient are bit-identical for every order (knob xcd = 0 ..
    5, and the automatic choices -1 and -2; at n = 15 the tile count is below the
    stream count and the plain order is kept), and they match the oracle."""
    inst = I.degree4_int2(n, 640 + n)
    H = sv.Ising.from_instance(inst)
    g, b = I.uniform_params(3, 641 + n, -1.1, 1.1)
    out = {}
    for x in (-2, -1, 0, 1, 2, 3, 4, 5):
        with Knob(sv, "xcd", x):
            s = sv.State(n, dtype)
            lam = sv.State(n, dtype)
            e, pg, nrm = sv.qaoa_energy(s, H, g, b)
            psi = s.to_numpy()
            ge, dg, db = sv.grad(s, lam, H, g, b)
            out[x] = (e, pg, nrm, psi, ge, dg, db)
            del s, lam
    ref = out[0]
    for x, o in out.items():
        assert o[:3] == ref[:3], (x, o[:3], ref[:3])
        assert np.array_equal(o[3], ref[3]), x
        assert o[4] == ref[4] and np.array_equal(o[5], ref[5]) and np.array_equal(o[6], ref[6]), x
    E = orc.energies(inst)
    rpsi = orc.qaoa_state(inst, g, b, E=E)
    err = float(np.max(np.abs(ref[3] - rpsi)))
    record_error(f"amp max-abs {dtype}", err)
    assert err <= AMP_TOL[dtype]
    _, rg, rb = orc.grad_tangent(inst, g, b)
    scale = grad_scale(orc, inst, rg, rb)
    gerr = max(np.max(np.abs(ref[5] - rg)), np.max(np.abs(ref[6] - rb))) / scale
    record_error(f"grad / scale {dtype}", gerr)
    assert gerr <= GRAD_TOL[dtype]


@pytest.mark.parametrize("dtype,n", [("c128", 26), ("c64", 26)])
def test_lds_swizzle_and_nontemporal_agree(sv, orc, record_error, dtype, n):
    """The LDS slot swizzle width (knob ldsswz = 3, 4, 5) only moves where a
    tile's amplitudes sit in LDS during an exchange, and the nontemporal
    threshold (ntmin = 0: every pass, 64: none) only changes cache hints: the
    state, the observables and the adjoint gradient are bit-identical, and they
    match the oracle."""
    inst = I.degree4_int2(n, 680 + n)
    H = sv.Ising.from_instance(inst)
    g, b = I.uniform_params(3, 681 + n, -1.1, 1.1)
    out = {}
    for knob, vals in (("ldsswz", (3, 4, 5)), ("ntmin", (0, 4, 64))):
        for v in vals:
            with Knob(sv, knob, v):
                s = sv.State(n, dtype)
                lam = sv.State(n, dtype)
                e, pg, nrm = sv.qaoa_energy(s, H, g, b)
                psi = s.to_numpy()
                ge, dg, db = sv.grad(s, lam, H, g, b)
                out[(knob, v)] = (e, pg, nrm, psi, ge, dg, db)
                del s, lam
    ref = out[("ldsswz", 4)]
    for k, o in out.items():
        assert o[:3] == ref[:3], (k, o[:3], ref[:3])
        assert np.array_equal(o[3], ref[3]), k
        assert o[4] == ref[4] and np.array_equal(o[5], ref[5]) and np.array_equal(o[6], ref[6]), k
    rpsi = orc.qaoa_state(inst, g, b, E=orc.energies(inst))
    err = float(np.max(np.abs(ref[3] - rpsi)))
    record_error(f"amp max-abs {dtype}", err)
    assert err <= AMP_TOL[dtype]
    _, rg, rb = orc.grad_tangent(inst, g, b)
    scale = grad_scale(orc, inst, rg, rb)
    gerr = max(np.max(np.abs(ref[5] - rg)), np.max(np.abs(ref[6] - rb))) / scale
    record_error(f"grad / scale {dtype}", gerr)
    assert gerr <= GRAD_TOL[dtype]


@pytest.mark.parametrize("dtype,n", [("c128", 20), ("c64", 21), ("c128", 26)])
def test_stream_ceiling_leaves_state_unchanged(sv, dtype, n):
    """sv_stream_ceiling reads and writes every amplitude in place with each tile
    geometry of the plan: the state is bit-identical afterwards and a time is
    reported; geometries that do not fit the state are argument errors."""
    rng = np.random.default_rng(660 + n)
    psi0 = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    s = sv.State(n, dtype)
    s.from_numpy(psi0)
    before = s.to_numpy()
    for g in sv.describe(n, dtype)["plans"]["nv1"]:
        ms = sv.stream_ceiling(s, g["c"], g["lo"])
        assert ms > 0.0
        assert np.array_equal(s.to_numpy(), before), (g["c"], g["lo"])
    T = sv.describe(n, dtype)["plans"]["nv1"][0]["T"]
    with pytest.raises(sv.SVError) as e:
        sv.stream_ceiling(s, 3, n - 2)  # group bits beyond the state
    assert e.value.code == 1
    with pytest.raises(sv.SVError):
        sv.stream_ceiling(s, T + 1, 0)
