"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (stated once, used everywhere):
  complex128 amplitudes  max |psi_gpu - psi_oracle| <= 1e-11
  complex64  amplitudes  max |psi_gpu - psi_oracle| <= 2e-5
  energies / probabilities |x_gpu - x_ref| <= 1e-6 * max(|x_ref|, sum|h| + sum|J|)  (energies)
                           |p_gpu - p_ref| <= 1e-6 (complex128: 1e-11)              (probabilities)
  gradients  max |g_gpu - g_ref| <= GRAD_TOL[dtype] * max(max|g_ref|, sum|h| + sum|J|)
             (1e-6 for complex128; 5e-6 for complex64, whose forward and reverse
             passes each round the amplitudes to f32)
Sizes span n below the tile (phantom bits), exactly one tile, several tiles in
one and two groups, and several groups with ragged group widths.
"""
import math
import sys

import numpy as np
import pytest

from paper_2104_03293_amd import inputs as I

pytestmark = pytest.mark.gpu

AMP_TOL = {"c128": 1e-11, "c64": 2e-5}
PROB_TOL = {"c128": 1e-11, "c64": 1e-6}
GRAD_TOL = {"c128": 1e-6, "c64": 5e-6}


@pytest.fixture(scope="module")
def sv():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2104_03293_amd import sv as m

    return m


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


def rand_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


def energy_tol(orc, inst, ref):
    return 1e-6 * max(abs(ref), orc.coeff_scale(inst), 1.0)


def instance_for(n, kind, seed):
    if kind == "int" and n >= 4:
        return I.degree4_int2(n, seed)
    if kind == "pm1" and n >= 4:
        return I.regular3_pm1(n, seed)
    m = min(2 * n, n * (n - 1) // 2)
    return I.random_real(n, m, seed)


SIZES = [1, 2, 5, 9, 12, 13, 14, 15, 17, 20, 23]


# ----------------------------------------------------------------------------- primitives
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 4, 13, 14, 16, 21])
def test_init_plus(sv, dtype, n):
    s = sv.State(n, dtype)
    sv.init_plus(s)
    got = s.to_numpy()
    assert np.max(np.abs(got - 2.0 ** (-n / 2))) <= (1e-16 if dtype == "c128" else 1e-8)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", SIZES)
def test_mixer(sv, orc, dtype, n):
    psi0 = rand_state(n, 10 + n)
    s = sv.State(n, dtype)
    s.from_numpy(psi0)
    beta = 0.37 + 0.1 * n
    sv.mixer(s, beta)
    ref = orc.mixer(n, psi0, beta)
    assert np.max(np.abs(s.to_numpy() - ref)) <= AMP_TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kind", ["int", "real"])
def test_cost_phase(sv, orc, dtype, n, kind):
    inst = instance_for(n, kind, 20 + n)
    H = sv.Ising.from_instance(inst)
    psi0 = rand_state(n, 30 + n)
    s = sv.State(n, dtype)
    s.from_numpy(psi0)
    gamma = -0.83 + 0.05 * n
    sv.cost_phase(s, H, gamma)
    ref = orc.cost_phase(inst, psi0, gamma)
    assert np.max(np.abs(s.to_numpy() - ref)) <= AMP_TOL[dtype]


@pytest.mark.parametrize("n", [2, 8, 13, 14, 15, 19, 22])
@pytest.mark.parametrize("kind", ["int", "real", "pm1"])
def test_ground(sv, orc, n, kind):
    inst = instance_for(n, kind, 40 + n)
    H = sv.Ising.from_instance(inst)
    got = sv.ground(H)
    ref = orc.ground(inst)
    if kind == "real":
        assert abs(got[0] - ref[0]) <= 1e-12 * max(1.0, orc.coeff_scale(inst))
    else:
        assert got[0] == ref[0]
    assert got[1] == ref[1] and got[2] == ref[2]


def test_ground_degenerate(sv, orc):
    # no fields: every state and its complement share an energy (degeneracy >= 2)
    inst = I.regular3_pm1(16, 5)
    inst = dict(inst, h=np.zeros(16))
    got = sv.ground(sv.Ising.from_instance(inst))
    ref = orc.ground(inst)
    assert got == (ref[0], ref[1], ref[2]) and ref[1] >= 2


# ----------------------------------------------------------------------------- circuits
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("p", [1, 3])
def test_qaoa_forward_and_expect(sv, orc, dtype, n, p):
    inst = instance_for(n, "int" if n % 2 else "real", 50 + n)
    H = sv.Ising.from_instance(inst)
    g, b = I.uniform_params(p, 60 + n, -1.2, 1.2)
    s = sv.State(n, dtype)
    sv.qaoa_forward(s, H, g, b)
    E = orc.energies(inst)
    ref = orc.qaoa_state(inst, g, b, E=E)
    assert np.max(np.abs(s.to_numpy() - ref)) <= AMP_TOL[dtype]
    en, pgs, nrm = sv.expect(s, H)
    rn, ren, rpgs = orc.observables(inst, ref, E=E)
    assert abs(en - ren) <= energy_tol(orc, inst, ren)
    assert abs(pgs - rpgs) <= PROB_TOL[dtype]
    assert abs(nrm - 1.0) <= (1e-12 if dtype == "c128" else 1e-5)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [3, 13, 16, 21])
def test_qaoa_energy_fused(sv, orc, dtype, n):
    """Forward with the observables fused into the last pass equals forward,
    then expect, and the oracle; the stored state is the forward state."""
    p = 3
    inst = instance_for(n, "int" if n % 2 else "real", 160 + n)
    H = sv.Ising.from_instance(inst)
    g, b = I.uniform_params(p, 170 + n, -1.0, 1.0)
    E = orc.energies(inst)
    ref = orc.qaoa_state(inst, g, b, E=E)
    ro = orc.observables(inst, ref, E=E)
    s = sv.State(n, dtype)
    e, pg, nrm = sv.qaoa_energy(s, H, g, b)
    assert np.max(np.abs(s.to_numpy() - ref)) <= AMP_TOL[dtype]
    assert abs(e - ro[1]) <= energy_tol(orc, inst, ro[1])
    assert abs(pg - ro[2]) <= PROB_TOL[dtype]
    assert abs(nrm - 1.0) <= (1e-12 if dtype == "c128" else 1e-5)
    e2, pg2, nrm2 = sv.expect(s, H)
    assert abs(e - e2) <= energy_tol(orc, inst, ro[1]) and abs(pg - pg2) <= PROB_TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [6, 14, 18])
def test_qaoa_from_given_state(sv, orc, dtype, n):
    inst = instance_for(n, "int", 70 + n)
    H = sv.Ising.from_instance(inst)
    psi0 = rand_state(n, 71 + n)
    s = sv.State(n, dtype)
    s.from_numpy(psi0)
    g, b = [0.3, -0.9], [1.1, 0.4]
    sv.qaoa_forward(s, H, g, b, from_plus=False)
    ref = orc.qaoa_state(inst, g, b, psi0=psi0)
    assert np.max(np.abs(s.to_numpy() - ref)) <= AMP_TOL[dtype]


def test_small_regular3_p1(sv, orc):
    """n = 14, p = 1, gamma = 0.4, beta = 0.3, complex128, 3-regular +-1 instance."""
    inst = I.small_regular3_instance()
    H = sv.Ising.from_instance(inst)
    s = sv.State(14, "c128")
    sv.qaoa_forward(s, H, [I.SMALL_GAMMA], [I.SMALL_BETA])
    E = orc.energies(inst)
    ref = orc.qaoa_state(inst, [I.SMALL_GAMMA], [I.SMALL_BETA], E=E)
    assert np.max(np.abs(s.to_numpy() - ref)) <= 1e-11
    en, pgs, nrm = sv.expect(s, H)
    _, ren, rpgs = orc.observables(inst, ref, E=E)
    assert abs(en - ren) <= 1e-6 * max(abs(ren), orc.coeff_scale(inst))
    assert abs(pgs - rpgs) <= 1e-11
    assert sv.ground(H)[:2] == orc.ground(inst, E)[:2]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fusion_plans_agree(sv, orc, dtype):
    n = 22 if dtype == "c128" else 24
    inst = instance_for(n, "int", 80)
    H = sv.Ising.from_instance(inst)
    g, b = I.uniform_params(4, 81)
    a = sv.State(n, dtype)
    sv.qaoa_forward(a, H, g, b)
    sv.tune_set("fuse", 0)
    try:
        c = sv.State(n, dtype)
        sv.qaoa_forward(c, H, g, b)
    finally:
        sv.tune_set("fuse", 1)
    assert np.max(np.abs(a.to_numpy() - c.to_numpy())) <= AMP_TOL[dtype] / 10


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_group_orders_agree(sv, orc, dtype):
    """Three tile groups: index-order and middle-A snake schedules give the same
    state, energy and gradient (the mixer factors of one layer commute)."""
    n = 24 if dtype == "c128" else 26
    assert len(sv.describe(n, dtype)["plans"]["nv1"]) == 3
    inst = instance_for(n, "int", 82)
    H = sv.Ising.from_instance(inst)
    g, b = I.uniform_params(3, 83)
    out = {}
    for snake in (1, 0):
        sv.tune_set("snake", snake)
        try:
            a = sv.State(n, dtype)
            e = sv.qaoa_energy(a, H, g, b)
            lam = sv.State(n, dtype)
            psi = sv.State(n, dtype)
            gr = sv.grad(psi, lam, H, g, b)
            out[snake] = (a.to_numpy(), e, gr)
        finally:
            sv.tune_set("snake", 1)
    (a1, e1, g1), (a0, e0, g0) = out[1], out[0]
    assert np.max(np.abs(a1 - a0)) <= AMP_TOL[dtype] / 10
    assert abs(e1[0] - e0[0]) <= energy_tol(orc, inst, e0[0])
    scale = orc.coeff_scale(inst)
    assert np.max(np.abs(g1[1] - g0[1])) <= GRAD_TOL[dtype] * scale
    assert np.max(np.abs(g1[2] - g0[2])) <= GRAD_TOL[dtype] * scale


@pytest.mark.parametrize("dtype,n", [("c128", 23), ("c64", 24), ("c64", 10), ("c64", 16)])
def test_lane_butterfly_plans(sv, orc, dtype, n):
    """Plans that butterfly one qubit across lanes (instead of one more LDS
    layout) against the oracle, for the forward state, the fused energy and the
    adjoint gradient, and against the same run with that option off."""
    plans = sv.describe(n, dtype)["plans"]
    assert any(b["dpp"] for g in plans["nv1"] for b in g["blocks"])
    p = 2
    inst = instance_for(n, "int", 90 + n)
    H = sv.Ising.from_instance(inst)
    g, b = I.uniform_params(p, 91 + n, -1.0, 1.0)
    E = orc.energies(inst)
    ref = orc.qaoa_state(inst, g, b, E=E)
    ro = orc.observables(inst, ref, E=E)
    s = sv.State(n, dtype)
    e = sv.qaoa_energy(s, H, g, b)
    assert np.max(np.abs(s.to_numpy() - ref)) <= AMP_TOL[dtype]
    assert abs(e[0] - ro[1]) <= energy_tol(orc, inst, ro[1])
    psi, lam = sv.State(n, dtype), sv.State(n, dtype)
    f, dg, db = sv.grad(psi, lam, H, g, b)
    _, rg, rb = orc.grad_tangent(inst, g, b)
    scale = max(np.max(np.abs(np.concatenate([rg, rb]))), orc.coeff_scale(inst))
    assert np.max(np.abs(dg - rg)) <= GRAD_TOL[dtype] * scale
    assert np.max(np.abs(db - rb)) <= GRAD_TOL[dtype] * scale
    sv.tune_set("dpp", 0)
    try:
        assert not any(b["dpp"] for g in sv.describe(n, dtype)["plans"]["nv1"] for b in g["blocks"])
        s0 = sv.State(n, dtype)
        sv.qaoa_forward(s0, H, g, b)
    finally:
        sv.tune_set("dpp", 1)
    assert np.max(np.abs(s0.to_numpy() - s.to_numpy())) <= AMP_TOL[dtype]


@pytest.mark.parametrize("n", [24])
def test_complex64_lane_position_4_plans(sv, orc, n):
    """complex64 14-bit tiles planned with lane position 4 allowed (knob c64occ=0:
    the one-workgroup-per-CU kernel with both lane butterflies) against the
    oracle and against the default plan."""
    inst = instance_for(n, "int", 95 + n)
    H = sv.Ising.from_instance(inst)
    g, b = I.uniform_params(2, 96 + n, -1.0, 1.0)
    ref = orc.qaoa_state(inst, g, b)
    s1 = sv.State(n, "c64")
    sv.qaoa_forward(s1, H, g, b)
    sv.tune_set("c64occ", 0)
    try:
        used = [blk["dpp"] for grp in sv.describe(n, "c64")["plans"]["nv1"] for blk in grp["blocks"]]
        s0 = sv.State(n, "c64")
        sv.qaoa_forward(s0, H, g, b)
    finally:
        sv.tune_set("c64occ", 1)
    assert any(d & 16 for d in used), used
    assert np.max(np.abs(s0.to_numpy() - ref)) <= AMP_TOL["c64"]
    assert np.max(np.abs(s1.to_numpy() - ref)) <= AMP_TOL["c64"]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_zero_angles_identity(sv, dtype):
    n = 17
    inst = instance_for(n, "int", 90)
    H = sv.Ising.from_instance(inst)
    s = sv.State(n, dtype)
    sv.qaoa_forward(s, H, [0.0, 0.0, 0.0], [0.0, 0.0, 0.0])
    assert np.max(np.abs(s.to_numpy() - 2 ** (-n / 2))) <= (1e-16 if dtype == "c128" else 1e-8)


# ----------------------------------------------------------------------------- AQA
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [8, 14, 19])
def test_aqa_per_step(sv, orc, dtype, n):
    inst = instance_for(n, "int", 100 + n)
    H = sv.Ising.from_instance(inst)
    g, b = orc.aqa_linear_schedule(6, 0.5)
    s = sv.State(n, dtype)
    pg, en = sv.aqa_run(s, H, g, b, per_step=True)
    E = orc.energies(inst)
    gs = orc.ground(inst, E)
    psi = orc.plus_state(n)
    for k in range(6):
        psi = orc.qaoa_state(inst, g[k:k + 1], b[k:k + 1], psi0=psi, E=E)
        _, ren, rpg = orc.observables(inst, psi, E=E, gs=gs)
        assert abs(pg[k] - rpg) <= PROB_TOL[dtype]
        assert abs(en[k] - ren) <= energy_tol(orc, inst, ren)
    assert np.max(np.abs(s.to_numpy() - psi)) <= AMP_TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [3, 12, 14, 17, 23])
def test_spin_z(sv, orc, dtype, n):
    inst = instance_for(n, "int" if n % 2 else "real", 180 + n)
    H = sv.Ising.from_instance(inst)
    g, b = I.uniform_params(2, 181 + n, -1.0, 1.0)
    s = sv.State(n, dtype)
    sv.qaoa_forward(s, H, g, b)
    got = sv.spin_z(s)
    ref = orc.spin_z(n, orc.qaoa_state(inst, g, b))
    assert np.max(np.abs(got - ref)) <= PROB_TOL[dtype] * 10


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [8, 14, 19])
def test_aqa_per_step_spins(sv, orc, dtype, n):
    """Per-step <sigma^z_i>, P_gs and <H_C> of an AQA run (fused into the step
    passes) against the oracle, step by step."""
    inst = instance_for(n, "int", 190 + n)
    H = sv.Ising.from_instance(inst)
    steps = 6
    g, b = sv.schedule_linear(steps, 0.8)
    s = sv.State(n, dtype)
    pg, en, sz = sv.aqa_run_observe(s, H, g, b)
    E = orc.energies(inst)
    gs = orc.ground(inst, E)
    psi = orc.plus_state(n)
    for k in range(steps):
        psi = orc.qaoa_state(inst, [g[k]], [b[k]], psi0=psi, E=E)
        _, ren, rpg = orc.observables(inst, psi, E=E, gs=gs)
        assert abs(en[k] - ren) <= energy_tol(orc, inst, ren)
        assert abs(pg[k] - rpg) <= PROB_TOL[dtype]
        assert np.max(np.abs(sz[k] - orc.spin_z(n, psi))) <= PROB_TOL[dtype] * 10
    # same state as the plain AQA call
    pg2, en2 = sv.aqa_run(s, H, g, b, per_step=True)
    assert np.max(np.abs(en2 - en)) <= 1e-12 * max(1.0, np.max(np.abs(en)))


def test_aqa_equals_qaoa_call(sv, orc):
    """AQA with n steps is one QAOA call with p = n + 1 (Sec. III.B.2)."""
    n = 16
    inst = instance_for(n, "int", 110)
    H = sv.Ising.from_instance(inst)
    g, b = sv.schedule_second_order(11, 0.4)
    a = sv.State(n, "c128")
    sv.aqa_run(a, H, g, b)
    c = sv.State(n, "c128")
    sv.qaoa_forward(c, H, g, b)
    assert np.array_equal(a.to_numpy(), c.to_numpy())


# ----------------------------------------------------------------------------- adjoint
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [3, 9, 13, 14, 15, 18, 21])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_grad_vs_oracle(sv, orc, dtype, n, p):
    inst = instance_for(n, "int" if n % 2 else "real", 120 + n)
    H = sv.Ising.from_instance(inst)
    g, b = I.uniform_params(p, 130 + n + p, -1.0, 1.0)
    psi = sv.State(n, dtype)
    lam = sv.State(n, dtype)
    e, pg, dg, db = sv.grad(psi, lam, H, g, b, with_pgs=True)
    f, rg, rb = orc.grad_tangent(inst, g, b)
    _, _, rpg = orc.observables(inst, orc.qaoa_state(inst, g, b))
    scale = max(np.max(np.abs(np.concatenate([rg, rb]))), orc.coeff_scale(inst))
    assert abs(e - f) <= energy_tol(orc, inst, f)
    assert abs(pg - rpg) <= PROB_TOL[dtype]
    assert np.max(np.abs(dg - rg)) <= GRAD_TOL[dtype] * scale
    assert np.max(np.abs(db - rb)) <= GRAD_TOL[dtype] * scale


@pytest.mark.parametrize("zeta", [0, 1])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,kind", [(5, "real"), (14, "int"), (21, "real"), (26, "int")])
def test_grad_both_reverse_sweeps(sv, orc, record_error, dtype, n, kind, zeta):
    """Both adjoint schemes against the oracle's forward-mode gradient, from |+> and
    from a given forward state: one sweep of psi and lambda in two-vector passes
    (knob adjzeta = 0), and two one-vector sweeps of psi +- i t lambda whose
    quadratic forms differ by 4 t Im <lambda|A|psi> (adjzeta = 1); n = 26 has three
    tile groups, n = 5 is smaller than one tile."""
    p = 3
    inst = instance_for(n, kind, 700 + n)
    H = sv.Ising.from_instance(inst)
    g, b = I.uniform_params(p, 701 + n, -1.1, 1.1)
    f, rg, rb = orc.grad_tangent(inst, g, b)
    _, _, rpg = orc.observables(inst, orc.qaoa_state(inst, g, b))
    scale = max(np.max(np.abs(np.concatenate([rg, rb]))), orc.coeff_scale(inst))
    old = sv.tune_get("adjzeta")
    sv.tune_set("adjzeta", zeta)
    try:
        for from_state in (False, True):
            psi = sv.State(n, dtype)
            lam = sv.State(n, dtype)
            if from_state:
                sv.qaoa_forward(psi, H, g, b)
            e, pg, dg, db = sv.grad(psi, lam, H, g, b, psi_is_forward=from_state, with_pgs=True)
            err = max(np.max(np.abs(dg - rg)), np.max(np.abs(db - rb))) / scale
            record_error(f"grad / scale {dtype} adjzeta={zeta}", err)
            assert abs(e - f) <= energy_tol(orc, inst, f)
            assert abs(pg - rpg) <= PROB_TOL[dtype]
            assert err <= GRAD_TOL[dtype], (from_state, err)
            del psi, lam
    finally:
        sv.tune_set("adjzeta", old)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_grad_from_forward_state(sv, orc, dtype):
    n, p = 17, 3
    inst = instance_for(n, "int", 140)
    H = sv.Ising.from_instance(inst)
    g, b = I.linear_ramp_params(p)
    psi = sv.State(n, dtype)
    lam = sv.State(n, dtype)
    sv.qaoa_forward(psi, H, g, b)
    e, dg, db = sv.grad(psi, lam, H, g, b, psi_is_forward=True)
    f, rg, rb = orc.grad_tangent(inst, g, b)
    scale = max(np.max(np.abs(np.concatenate([rg, rb]))), orc.coeff_scale(inst))
    assert np.max(np.abs(dg - rg)) <= GRAD_TOL[dtype] * scale
    assert np.max(np.abs(db - rb)) <= GRAD_TOL[dtype] * scale


@pytest.mark.parametrize("first", ["c128", "c64"])
def test_one_instance_both_dtypes(sv, orc, first):
    """Regression: tile tables cached per instance must not be shared between
    amplitude types (complex128 forward passes and complex64 adjoint passes use
    the same tile shape but different LDS swizzles and byte strides)."""
    n, p = 16, 2
    inst = instance_for(n, "int", 150)
    H = sv.Ising.from_instance(inst)
    g, b = I.linear_ramp_params(p)
    f, rg, rb = orc.grad_tangent(inst, g, b)
    scale = max(np.max(np.abs(np.concatenate([rg, rb]))), orc.coeff_scale(inst))
    ref = orc.qaoa_state(inst, g, b)
    for dtype in ([first, "c64" if first == "c128" else "c128"] * 2):
        psi = sv.State(n, dtype)
        sv.qaoa_forward(psi, H, g, b)
        assert np.max(np.abs(psi.to_numpy() - ref)) <= AMP_TOL[dtype]
        lam = sv.State(n, dtype)
        e, dg, db = sv.grad(psi, lam, H, g, b)
        assert np.max(np.abs(dg - rg)) <= GRAD_TOL[dtype] * scale
        assert np.max(np.abs(db - rb)) <= GRAD_TOL[dtype] * scale


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [9, 14, 17])
def test_exact_cover_instances(sv, orc, dtype, n):
    """Dense exact cover instances (half-integer h, J; Eqs. HChi-HCC): the
    library's Ising form (ground energy -C, rescale factor), the QAOA state with
    rescaled angles gamma / r, the fused observables and the adjoint gradient
    against the oracle's independent construction."""
    a = I.exact_cover_matrix(n, 472, 700 + n)
    inst, C = orc.exact_cover_ising(a)
    H, C_lib = sv.Ising.exact_cover(a)
    assert C_lib == C
    emin, deg, _ = sv.ground(H)
    assert emin == -C and deg >= 1
    r = sv.rescale_factor(H)
    assert r == orc.rescale_factor(inst)
    g, b = I.linear_ramp_params(3)
    gr = g / r
    E = orc.energies(inst)
    ref = orc.qaoa_state(inst, gr, b, E=E)
    s = sv.State(n, dtype)
    e, pgs, nrm = sv.qaoa_energy(s, H, gr, b)
    assert np.max(np.abs(s.to_numpy() - ref)) <= AMP_TOL[dtype]
    _, ren, rpgs = orc.observables(inst, ref, E=E)
    assert abs(e - ren) <= energy_tol(orc, inst, ren)
    assert abs(pgs - rpgs) <= PROB_TOL[dtype]
    lam = sv.State(n, dtype)
    f, dg, db = sv.grad(s, lam, H, gr, b)
    _, rg, rb = orc.grad_tangent(inst, gr, b, E=E)
    scale = max(np.max(np.abs(np.concatenate([rg, rb]))), orc.coeff_scale(inst))
    assert np.max(np.abs(dg - rg)) <= GRAD_TOL[dtype] * scale
    assert np.max(np.abs(db - rb)) <= GRAD_TOL[dtype] * scale


def test_grad_errors(sv):
    H = sv.Ising.from_instance(instance_for(10, "int", 1))
    a = sv.State(10, "c128")
    b = sv.State(10, "c64")
    with pytest.raises(sv.SVError) as e:
        sv.grad(a, b, H, [0.1], [0.2])
    assert e.value.code == 1
    with pytest.raises(sv.SVError) as e:
        sv.grad(a, a, H, [0.1], [0.2])
    assert e.value.code == 1
    c = sv.State(11, "c128")
    with pytest.raises(sv.SVError):
        sv.qaoa_forward(c, H, [0.1], [0.2])


# ----------------------------------------------------------------------------- batch scan
def _batch_oracle(orc, inst, gam, bet):
    E = orc.energies(inst)
    gs = orc.ground(inst, E)
    en = np.empty((len(gam), len(bet)))
    pg = np.empty((len(gam), len(bet)))
    for a, g in enumerate(gam):
        for b, bb in enumerate(bet):
            psi = orc.qaoa_state(inst, [g], [bb], E=E)
            _, en[a, b], pg[a, b] = orc.observables(inst, psi, E=E, gs=gs)
    return en, pg


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_scan_vs_oracle(sv, orc, dtype):
    """Uneven n (tiny, LDS-resident and larger than one LDS slice), integer and
    real-valued instances, half-open grid with its gamma = 0 and beta = 0 edges."""
    ns = [1, 3, 4, 7, 10, 12, 13, 14, 15, 16, 18]
    insts = []
    for k, n in enumerate(ns):
        if n >= 4:
            insts.append(I.regular3_pm1(n, 500 + k))
        else:
            insts.append(instance_for(n, "real", 500 + k))
    insts.append(I.random_real(11, 20, 77))
    gam, bet = I.batch_grid(6, 5)
    Hs = [sv.Ising.from_instance(x) for x in insts]
    en, pg = sv.batch_p1_scan(Hs, gam, bet, dtype=dtype)
    for i, inst in enumerate(insts):
        ren, rpg = _batch_oracle(orc, inst, gam, bet)
        tol = 1e-6 * max(orc.coeff_scale(inst), 1.0)
        assert np.max(np.abs(en[i] - ren)) <= tol, (i, inst["n"])
        assert np.max(np.abs(pg[i] - rpg)) <= PROB_TOL[dtype], (i, inst["n"])


@pytest.mark.parametrize("dtype,knob,val", [("c64", "batchwide", 0), ("c64", "batchwide", 1),
                                            ("c64", "batchwide", 2), ("c128", "batch128", 0),
                                            ("c128", "batch128", 1), ("c64", "batchslab", 0),
                                            ("c64", "batchslab", 1), ("c128", "batchslab", 0),
                                            ("c128", "batchslab", 1)])
def test_batch_scan_variants(sv, orc, dtype, knob, val):
    """Every batch kernel variant (complex64: one workgroup per CU with 2^14 LDS
    states and four or eight waves, or two per CU with 2^13; complex128: four or
    eight waves) against the oracle.  States above the 2^13-amplitude LDS tile
    take the sliced path by default; batchslab = 0 sends them through the
    per-workgroup slots instead, and a 1 MiB slab makes launches of one or two
    states that split an instance's beta row."""
    ns = [3, 9, 12, 13, 14, 15, 17, 18]
    insts = [I.regular3_pm1(n, 520 + k) if n >= 4 else instance_for(n, "real", 520 + k) for k, n in enumerate(ns)]
    insts.append(I.random_real(14, 25, 78))
    gam, bet = I.batch_grid(4, 5)
    Hs = [sv.Ising.from_instance(x) for x in insts]
    old = sv.tune_get(knob)
    sv.tune_set(knob, val)
    try:
        en, pg = sv.batch_p1_scan(Hs, gam, bet, dtype=dtype)
    finally:
        sv.tune_set(knob, old)
    for i, inst in enumerate(insts):
        ren, rpg = _batch_oracle(orc, inst, gam, bet)
        tol = 1e-6 * max(orc.coeff_scale(inst), 1.0)
        assert np.max(np.abs(en[i] - ren)) <= tol, (i, inst["n"])
        assert np.max(np.abs(pg[i] - rpg)) <= PROB_TOL[dtype], (i, inst["n"])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_scan_any_beta(sv, orc, dtype):
    """Mixer angles off the half-open grid: negative, at and across +-pi/4 and
    +-pi/2 (where cos beta = 0), beyond pi, on states that fit one LDS slice and
    states that do not."""
    betas = np.array([0.0, -0.3, math.pi / 4, -math.pi / 4, 0.8, math.pi / 2, -math.pi / 2, 2.0, -2.6,
                      math.pi, 7.3, -11.0])
    gams = np.array([0.0, 0.37, -1.9])
    ns = [2, 6, 11, 13, 14, 15, 17]
    insts = [I.regular3_pm1(n, 590 + k) if n >= 4 else instance_for(n, "real", 590 + k) for k, n in enumerate(ns)]
    insts.append(I.random_real(16, 30, 591))
    Hs = [sv.Ising.from_instance(x) for x in insts]
    en, pg = sv.batch_p1_scan(Hs, gams, betas, dtype=dtype)
    for i, inst in enumerate(insts):
        ren, rpg = _batch_oracle(orc, inst, gams, betas)
        tol = 1e-6 * max(orc.coeff_scale(inst), 1.0)
        assert np.max(np.abs(en[i] - ren)) <= tol, (i, inst["n"])
        assert np.max(np.abs(pg[i] - rpg)) <= PROB_TOL[dtype], (i, inst["n"])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_scan_integer_range_beyond_table(sv, orc, dtype):
    """Integer-valued instances whose energy range exceeds the 1024-entry phase
    table take the FP64 energy-table path, in and above one LDS slice, next to
    instances that use the table."""
    insts = []
    for k, n in enumerate([9, 13, 16]):
        base = I.regular3_pm1(n, 610 + k)
        insts.append(dict(base, J=np.asarray(base["J"]) * 40.0, h=np.asarray(base["h"]) * 7.0))
        insts.append(I.regular3_pm1(n, 620 + k))
    for x in insts[::2]:
        assert 2 * (np.sum(np.abs(x["h"])) + np.sum(np.abs(x["J"]))) + 1 > 1024
    gam, bet = np.array([0.0, 0.013, -0.21]), np.array([0.1, 0.9, -1.4])
    Hs = [sv.Ising.from_instance(x) for x in insts]
    en, pg = sv.batch_p1_scan(Hs, gam, bet, dtype=dtype)
    for i, inst in enumerate(insts):
        ren, rpg = _batch_oracle(orc, inst, gam, bet)
        tol = 1e-6 * max(orc.coeff_scale(inst), 1.0)
        assert np.max(np.abs(en[i] - ren)) <= tol, (i, inst["n"])
        assert np.max(np.abs(pg[i] - rpg)) <= PROB_TOL[dtype], (i, inst["n"])


def test_batch_scan_closed_form_full_grid(sv, orc):
    """32 x 32 grid of the batched workload on 64 instances: <H_C> at every point
    against the depth-one closed form (test_oracle_pins.p1_closed_form_energy)."""
    from tests.test_oracle_pins import p1_closed_form_energy

    insts = I.batch_instances(64)
    gam, bet = I.batch_grid()
    Hs = [sv.Ising.from_instance(x) for x in insts]
    en, pg = sv.batch_p1_scan(Hs, gam, bet, dtype="c64")
    for i in range(0, 64, 7):
        inst = insts[i]
        for a in (0, 3, 17, 31):
            for b in (0, 5, 22, 31):
                ref = p1_closed_form_energy(inst, gam[a], bet[b])
                assert abs(en[i, a, b] - ref) <= 1e-6 * max(orc.coeff_scale(inst), 1.0)
    # gamma = 0 or beta = 0: P_gs = degeneracy / 2^n exactly (up to f32 rounding)
    for i in range(0, 64, 9):
        _, deg, _ = orc.ground(insts[i])
        assert abs(pg[i, 0, 7] - deg / 2 ** insts[i]["n"]) <= 1e-6
        assert abs(pg[i, 5, 0] - deg / 2 ** insts[i]["n"]) <= 1e-6


def test_batch_scan_errors(sv):
    H = sv.Ising.from_instance(I.regular3_pm1(20, 1))
    with pytest.raises(sv.SVError) as e:
        sv.batch_p1_scan([H], [0.1], [0.2], dtype="c128")
    assert e.value.code == 4


# ----------------------------------------------------------------------------- degenerate cases
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 7, 15, 20])
def test_zero_hamiltonian(sv, orc, dtype, n):
    """h = 0 and no couplings: every basis state is a ground state (E = 0), the cost
    phase is the identity, <H_C> = 0, P_gs = 1 and the gradient vanishes."""
    inst = {"n": n, "h": np.zeros(n), "ei": np.zeros(0, np.int32), "ej": np.zeros(0, np.int32), "J": np.zeros(0)}
    H = sv.Ising.from_instance(inst)
    emin, deg, arg = sv.ground(H)
    assert emin == 0.0 and deg == 2 ** n and arg == 0
    g, b = I.uniform_params(3, 400 + n, -2.0, 2.0)
    s = sv.State(n, dtype)
    e, pgs, nrm = sv.qaoa_energy(s, H, g, b)
    ref = orc.qaoa_state(inst, g, b)
    assert np.max(np.abs(s.to_numpy() - ref)) <= AMP_TOL[dtype]
    assert abs(e) <= 1e-12 and abs(pgs - 1.0) <= PROB_TOL[dtype] * 10 and abs(nrm - 1.0) <= PROB_TOL[dtype] * 10
    psi, lam = sv.State(n, dtype), sv.State(n, dtype)
    f, dg, db = sv.grad(psi, lam, H, g, b)
    assert abs(f) <= 1e-12 and np.max(np.abs(dg)) <= 1e-12 and np.max(np.abs(db)) <= 1e-12


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("beta", [0.0, math.pi / 4, math.pi / 2, -3 * math.pi / 4, math.pi, 7.3, -11.0])
def test_mixer_angle_reduction(sv, orc, dtype, beta):
    """Mixer angles at and beyond the reduction boundaries (multiples of pi/4, pi and
    large |beta|) on a random state spanning several tile groups."""
    n = 23
    psi0 = rand_state(n, 410)
    s = sv.State(n, dtype)
    s.from_numpy(psi0)
    sv.mixer(s, beta)
    assert np.max(np.abs(s.to_numpy() - orc.mixer(n, psi0, beta))) <= AMP_TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_identity_parameters_keep_plus_state(sv, dtype):
    """gamma = beta = 0 leaves |+>^n unchanged (every pass runs, nothing rotates)."""
    n = 22
    inst = instance_for(n, "int", 420)
    H = sv.Ising.from_instance(inst)
    s = sv.State(n, dtype)
    sv.qaoa_forward(s, H, [0.0, 0.0], [0.0, 0.0])
    assert np.max(np.abs(s.to_numpy() - 2.0 ** (-n / 2))) <= AMP_TOL[dtype] * 1e-2


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("n", [9, 15, 18, 21])
def test_complex64_adjoint_tile_sizes(sv, orc, mode, n):
    """The complex64 adjoint on 13-bit tiles (c64g14=0) and on 14-bit tiles with
    1024-thread two-vector passes (c64g14=1), against the oracle gradient."""
    p = 3
    inst = instance_for(n, "int" if n % 2 else "real", 430 + n)
    H = sv.Ising.from_instance(inst)
    g, b = I.uniform_params(p, 431 + n, -1.0, 1.0)
    sv.tune_set("c64g14", mode)
    try:
        psi, lam = sv.State(n, "c64"), sv.State(n, "c64")
        e, pg, dg, db = sv.grad(psi, lam, H, g, b, with_pgs=True)
    finally:
        sv.tune_set("c64g14", 2)
    f, rg, rb = orc.grad_tangent(inst, g, b)
    scale = max(np.max(np.abs(np.concatenate([rg, rb]))), orc.coeff_scale(inst))
    assert abs(e - f) <= energy_tol(orc, inst, f)
    assert np.max(np.abs(dg - rg)) <= GRAD_TOL["c64"] * scale
    assert np.max(np.abs(db - rb)) <= GRAD_TOL["c64"] * scale


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_autograd_function(sv, orc, dtype):
    """QAOAEnergy (torch.autograd.Function over the adjoint sweep): the energy and the
    gradients that reach gamma and beta through a downstream expression."""
    import torch

    n, p = 16, 3
    inst = instance_for(n, "int", 440)
    H = sv.Ising.from_instance(inst)
    g0, b0 = I.uniform_params(p, 441, -1.0, 1.0)
    g = torch.tensor(g0, dtype=torch.float64, requires_grad=True)
    b = torch.tensor(b0, dtype=torch.float64, requires_grad=True)
    psi, lam = sv.State(n, dtype), sv.State(n, dtype)
    e = sv.QAOAEnergy.apply(g, b, psi, lam, H)
    loss = 3.0 * e + e * e
    loss.backward()
    f, rg, rb = orc.grad_tangent(inst, g0, b0)
    assert abs(e.item() - f) <= energy_tol(orc, inst, f)
    scale = max(np.max(np.abs(np.concatenate([rg, rb]))), orc.coeff_scale(inst)) * abs(3.0 + 2.0 * f)
    assert np.max(np.abs(g.grad.numpy() - (3.0 + 2.0 * f) * rg)) <= GRAD_TOL[dtype] * scale
    assert np.max(np.abs(b.grad.numpy() - (3.0 + 2.0 * f) * rb)) <= GRAD_TOL[dtype] * scale



@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_autograd_function_forward_only(sv, orc, dtype):
    """Without a gradient to compute (inputs without requires_grad, or under
    torch.no_grad) QAOAEnergy runs only the energy evaluation: same energy as
    sv_qaoa_energy, and the adjoint vector lam keeps its contents."""
    import torch

    n, p = 14, 2
    inst = instance_for(n, "int", 450)
    H = sv.Ising.from_instance(inst)
    g0, b0 = I.uniform_params(p, 451, -1.0, 1.0)
    psi, lam = sv.State(n, dtype), sv.State(n, dtype)
    ref = sv.qaoa_energy(sv.State(n, dtype), H, g0, b0)[0]
    marker = np.full(1 << n, 0.25 - 0.5j)
    lam.from_numpy(marker)
    e1 = sv.QAOAEnergy.apply(torch.tensor(g0), torch.tensor(b0), psi, lam, H)
    g = torch.tensor(g0, requires_grad=True)
    b = torch.tensor(b0, requires_grad=True)
    with torch.no_grad():
        e2 = sv.QAOAEnergy.apply(g, b, psi, lam, H)
    assert e1.item() == ref and e2.item() == ref
    assert np.array_equal(lam.to_numpy(), marker.astype(lam.to_numpy().dtype))
    f = orc.energy_of(inst, g0, b0)
    assert abs(ref - f) <= energy_tol(orc, inst, f)

@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_mixer_tables_rebuilt_after_last_state_freed(sv, orc, dtype):
    """Mixer-only programs use instance-free geometry tables that the library
    frees with its last state; a state made afterwards rebuilds them."""
    import gc

    gc.collect()
    for n in (15, 21, 15):
        psi0 = rand_state(n, 700 + n)
        s = sv.State(n, dtype)
        s.from_numpy(psi0)
        sv.mixer(s, 0.61)
        assert np.max(np.abs(s.to_numpy() - orc.mixer(n, psi0, 0.61))) <= AMP_TOL[dtype]
        s.close()
        gc.collect()
