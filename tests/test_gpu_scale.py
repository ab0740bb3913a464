"""Full-size GPU checks (the largest single-GPU states and the n = 26 / n = 30
workloads), through the C ABI.

No full oracle state fits at n = 33 / 34, so these use what holds at any size:
  * J = 0 instances: sampled amplitudes and <H_C> against the factorised
    oracle state (oracle.product_amplitudes / product_energy);
  * AQA run with per-step observables == the QAOA call with the same schedule;
  * conjugation: (gamma, beta) -> (-gamma, -beta) keeps <H_C> and P_gs;
  * adjoint gradient == central finite differences of the complex128 energy
    (h = 1e-4 with the Richardson pair).
At n = 26 (AQA, 20 steps) and n = 30 (p = 8 gradient) the oracle or the
complex128 path supplies the reference.

Tolerances as in test_gpu_parity: amplitudes 1e-11 (complex128) / 2e-5
(complex64); energies 1e-6 * max(|E|, sum|h| + sum|J|); gradients
1e-6 (complex128) / 5e-6 (complex64) times max(|g|, sum|h| + sum|J|).
"""
import sys

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


def sample_indices(n, count, seed):
    rng = np.random.default_rng(seed)
    z = rng.integers(0, 1 << n, size=count, dtype=np.uint64)
    return np.concatenate([np.array([0, (1 << n) - 1], dtype=np.uint64), z])


@pytest.mark.parametrize("dtype,n", [("c128", 32), ("c64", 32), ("c128", 33), ("c64", 34)])
def test_product_state_full_size(sv, orc, dtype, n):
    import torch

    need_free((1 << n) * (16 if dtype == "c128" else 8))
    inst = I.fields_only(n, 40 + n)
    H = sv.Ising.from_instance(inst)
    g, b = I.linear_ramp_params(4)
    s = sv.State(n, dtype)
    e, pgs, nrm = sv.qaoa_energy(s, H, g, b)
    zs = sample_indices(n, 4096, 41 + n)
    got = s.tensor[torch.from_numpy(zs.astype(np.int64)).to(s.tensor.device)].cpu().numpy()
    ref = orc.product_amplitudes(inst["h"], g, b, zs)
    assert np.max(np.abs(got - ref)) <= AMP_TOL[dtype] * 2.0 ** (-(n - 20) / 2)  # amplitudes scale as 2^(-n/2)
    eref = orc.product_energy(inst["h"], g, b)
    assert abs(e - eref) <= energy_tol(orc, inst, eref)
    assert abs(nrm - 1.0) <= (1e-12 if dtype == "c128" else 1e-5)
    del s


@pytest.mark.parametrize("dtype,n", [("c128", 33), ("c64", 34)])
def test_hadamard_circuit_full_size(sv, dtype, n):
    """(H^{xN})^{11} on |+>^n gives |0...0> (the Hadamard benchmark circuit)."""
    import torch

    need_free((1 << n) * (16 if dtype == "c128" else 8))
    had = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
    s = sv.State(n, dtype)
    sv.init_plus(s)
    sv.gate_layers(s, np.broadcast_to(had, (11, n, 2, 2)))
    zs = sample_indices(n, 4096, 60 + n)
    got = s.tensor[torch.from_numpy(zs.astype(np.int64)).to(s.tensor.device)].cpu().numpy()
    tol = 1e-11 if dtype == "c128" else 2e-5
    assert abs(got[0] - 1.0) <= tol
    assert np.max(np.abs(got[1:])) <= tol * 2.0 ** (-(n - 20) / 2)
    assert abs(torch.linalg.vector_norm(s.tensor).item() - 1.0) <= tol
    del s


@pytest.mark.parametrize("dtype,n", [("c128", 33), ("c64", 34)])
def test_qsds_product_state_full_size(sv, orc, dtype, n):
    """Eq. AQA4 stepping of a J = 0 instance against the factorised oracle state."""
    import torch

    need_free((1 << n) * (16 if dtype == "c128" else 8))
    inst = I.fields_only(n, 70 + n)
    H = sv.Ising.from_instance(inst)
    A, B = np.array([0.9, 0.6, 0.35, 0.1]), np.array([0.1, 0.4, 0.65, 0.9])
    s = sv.State(n, dtype)
    en, pg, sz = sv.qsds_run(s, H, 0.55, A, B, observe=True)
    phi = orc.qsds_product_factors(inst["h"], 0.55, A, B)
    zs = sample_indices(n, 4096, 71 + n)
    got = s.tensor[torch.from_numpy(zs.astype(np.int64)).to(s.tensor.device)].cpu().numpy()
    ref = orc.factor_amplitudes(phi, zs)
    assert np.max(np.abs(got - ref)) <= AMP_TOL[dtype] * 2.0 ** (-(n - 20) / 2)
    eref = orc.factor_energy(inst["h"], phi)
    assert abs(en[-1] - eref) <= energy_tol(orc, inst, eref)
    szref = np.abs(phi[:, 1]) ** 2 - np.abs(phi[:, 0]) ** 2
    assert np.max(np.abs(sz[-1] - szref)) <= 10 * PROB_TOL[dtype]
    del s


@pytest.mark.parametrize("dtype,n", [("c128", 33), ("c64", 34)])
def test_aqa_equals_qaoa_full_size(sv, dtype, n):
    need_free((1 << n) * (16 if dtype == "c128" else 8))
    inst = I.full_size_instance(n)
    H = sv.Ising.from_instance(inst)
    g, b = sv.schedule_linear(10, 0.5)
    s = sv.State(n, dtype, owner="lib")
    pg, en = sv.aqa_run(s, H, g, b, per_step=True)
    e, pgs, nrm = sv.qaoa_energy(s, H, g, b)
    assert abs(en[-1] - e) <= 1e-9 * max(1.0, abs(e))
    assert abs(pg[-1] - pgs) <= 1e-9 * max(pgs, 1e-300) + 1e-15
    assert abs(nrm - 1.0) <= (1e-12 if dtype == "c128" else 1e-5)
    assert np.all(pg >= 0) and np.all(np.isfinite(en))
    # conjugation: (gamma, beta) -> (-gamma, -beta) conjugates the state
    e2, pgs2, _ = sv.qaoa_energy(s, H, -g, -b)
    assert abs(e2 - e) <= 1e-9 * max(1.0, abs(e)) and abs(pgs2 - pgs) <= 1e-9 * pgs + 1e-15
    s.close()


def test_grad_full_size_c128_n33(sv, orc):
    n, p = 33, 4
    need_free(2 * (1 << n) * 16)
    inst = I.full_size_instance(n)
    H = sv.Ising.from_instance(inst)
    g, b = I.linear_ramp_params(p)
    psi = sv.State(n, "c128", owner="lib")
    lam = sv.State(n, "c128", owner="lib")
    f, dg, db = sv.grad(psi, lam, H, g, b)
    lam.close()

    def energy(gg, bb):
        return sv.qaoa_energy(psi, H, gg, bb)[0]

    def central(k, is_gamma, h):
        g1, b1, g2, b2 = g.copy(), b.copy(), g.copy(), b.copy()
        if is_gamma:
            g1[k] += h
            g2[k] -= h
        else:
            b1[k] += h
            b2[k] -= h
        return (energy(g1, b1) - energy(g2, b2)) / (2 * h)

    fd_g = np.array([(4 * central(k, True, 5e-5) - central(k, True, 1e-4)) / 3 for k in range(p)])
    fd_b = np.array([(4 * central(k, False, 5e-5) - central(k, False, 1e-4)) / 3 for k in range(p)])
    scale = max(np.max(np.abs(np.concatenate([fd_g, fd_b]))), orc.coeff_scale(inst))
    assert abs(f - energy(g, b)) <= energy_tol(orc, inst, f)
    assert np.max(np.abs(dg - fd_g)) <= GRAD_TOL["c128"] * scale
    assert np.max(np.abs(db - fd_b)) <= GRAD_TOL["c128"] * scale
    psi.close()


def test_grad_c64_n30_p8(sv, orc):
    """n = 30, p = 8: complex64 adjoint (16 parameters) against the complex128
    adjoint and central differences of the complex128 energy."""
    n, p = 30, 8
    need_free(2 * (1 << n) * 16 + 2 * (1 << n) * 8)
    inst = I.grad_degree4_instance(n)
    H = sv.Ising.from_instance(inst)
    g, b = I.linear_ramp_params(p)
    psi, lam = sv.State(n, "c64"), sv.State(n, "c64")
    f64, dg64, db64 = sv.grad(psi, lam, H, g, b)
    del psi, lam
    psi, lam = sv.State(n, "c128"), sv.State(n, "c128")
    f, dg, db = sv.grad(psi, lam, H, g, b)
    del lam

    def energy(gg, bb):
        return sv.qaoa_energy(psi, H, gg, bb)[0]

    def central(k, is_gamma, h):
        g1, b1, g2, b2 = g.copy(), b.copy(), g.copy(), b.copy()
        if is_gamma:
            g1[k] += h
            g2[k] -= h
        else:
            b1[k] += h
            b2[k] -= h
        return (energy(g1, b1) - energy(g2, b2)) / (2 * h)

    fd_g = np.array([(4 * central(k, True, 5e-5) - central(k, True, 1e-4)) / 3 for k in range(p)])
    fd_b = np.array([(4 * central(k, False, 5e-5) - central(k, False, 1e-4)) / 3 for k in range(p)])
    scale = max(np.max(np.abs(np.concatenate([fd_g, fd_b]))), orc.coeff_scale(inst))
    assert np.max(np.abs(dg - fd_g)) <= GRAD_TOL["c128"] * scale
    assert np.max(np.abs(db - fd_b)) <= GRAD_TOL["c128"] * scale
    assert np.max(np.abs(dg64 - dg)) <= GRAD_TOL["c64"] * scale
    assert np.max(np.abs(db64 - db)) <= GRAD_TOL["c64"] * scale
    assert abs(f64 - f) <= energy_tol(orc, inst, f)


@pytest.fixture(scope="module")
def aqa26_reference(orc):
    """Oracle per-step (<H_C>, P_gs) of the n = 26 AQA run (20 steps, tau = 0.5)."""
    n = 26
    inst = I.aqa_degree4_instance(n)
    g, b = orc.aqa_linear_schedule(20, 0.5)
    E = orc.energies(inst)
    gs = orc.ground(inst, E)
    psi = orc.plus_state(n)
    out = []
    for k in range(20):
        psi = orc.qaoa_state(inst, [g[k]], [b[k]], psi0=psi, E=E)
        _, ren, rpg = orc.observables(inst, psi, E=E, gs=gs)
        out.append((ren, rpg))
    return inst, np.array(out)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_aqa_n26_20_steps(sv, orc, aqa26_reference, dtype):
    """n = 26, 20 coarse steps, tau = 0.5, paper sign: per-step P_gs and <H_C>
    against the oracle; tau = 1.0 with the literal sign against the paper sign
    on the negated problem (<H>_literal(H) = -<H>_paper(-H) at every step)."""
    n = 26
    inst, ref = aqa26_reference
    H = sv.Ising.from_instance(inst)
    g, b = sv.schedule_linear(20, 0.5)
    s = sv.State(n, dtype)
    pg, en = sv.aqa_run(s, H, g, b, per_step=True)
    for k in range(20):
        assert abs(en[k] - ref[k, 0]) <= energy_tol(orc, inst, ref[k, 0]), k
        assert abs(pg[k] - ref[k, 1]) <= PROB_TOL[dtype], k
    neg = dict(inst)
    neg["h"] = -np.asarray(inst["h"])
    neg["J"] = -np.asarray(inst["J"])
    Hn = sv.Ising.from_instance(neg)
    gl, bl = sv.schedule_linear(20, 1.0, paper_sign=False)
    gp, bp = sv.schedule_linear(20, 1.0, paper_sign=True)
    _, en_lit = sv.aqa_run(s, H, gl, bl, per_step=True)
    _, en_neg = sv.aqa_run(s, Hn, gp, bp, per_step=True)
    assert np.max(np.abs(en_lit + en_neg)) <= 1e-6 * orc.coeff_scale(inst)
