"""Python face of the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It loads ``oracle/liboracle.so`` (built
from ``oracle/oracle.c`` by ``oracle/build.py``) and adds:

  * the AQA / QAOA parameter schedules, written from Sec. III.B and Appendix A;
  * a dense-matrix cross-check (Kronecker products + ``scipy.linalg.expm``) for
    n <= 10, independent of the bit-loop code in ``oracle.c``;
  * central finite differences with a Richardson pair for gradients.

Nothing here imports the HIP library or the product package.

Parity status of each function is documented in its docstring; every function
below is pinned by a ``-m "not gpu"`` test (see tests/test_oracle_*.py).
"""
from __future__ import annotations

import ctypes
import math
import os
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_LIB = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


# another compiled copy of oracle.c (use_library, or $ORACLE_LIBRARY: the
# sanitized build of build.py), else oracle/liboracle.so
_LIB_PATH = Path(os.environ["ORACLE_LIBRARY"]).resolve() if os.environ.get("ORACLE_LIBRARY") else None


def use_library(path) -> None:
    """Load the C oracle from another compiled copy of oracle.c (the timing build
    of the CPU-baseline leg); the next call of lib() loads it."""
    global _LIB, _LIB_PATH
    _LIB, _LIB_PATH = None, Path(path)


def lib():
    global _LIB
    if _LIB is None:
        path = _LIB_PATH or (_HERE / "liboracle.so")
        if not path.exists():
            from . import build as _b  # noqa: F401  (oracle/build.py)

            _b.build()
        L = ctypes.CDLL(str(path))
        L.orc_energy.restype = ctypes.c_double
        L.orc_energy.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _ip, _ip, _dp, ctypes.c_uint64]
        L.orc_energies.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _ip, _ip, _dp, _dp]
        L.orc_ground.argtypes = [ctypes.c_int, _dp, ctypes.c_double, _dp, _u64p, _u64p]
        L.orc_init_plus.argtypes = [ctypes.c_int, _dp]
        L.orc_cost_phase.argtypes = [ctypes.c_int, _dp, ctypes.c_double, _dp]
        L.orc_rx.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp]
        L.orc_mixer.argtypes = [ctypes.c_int, ctypes.c_double, _dp]
        L.orc_gate_1q.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.orc_qaoa.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp]
        L.orc_observables.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                      _dp, _dp, _dp]
        L.orc_spin_z.argtypes = [ctypes.c_int, _dp, _dp]
        L.orc_grad_tangent.restype = ctypes.c_int
        L.orc_grad_tangent.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _LIB = L
    return _LIB


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(t: int) -> None:
    lib().orc_set_num_threads(int(t))


# ----------------------------------------------------------------------------- energies
def _inst(inst):
    n = int(inst["n"])
    h = np.ascontiguousarray(inst["h"], dtype=np.float64)
    ei = np.ascontiguousarray(inst["ei"], dtype=np.int32)
    ej = np.ascontiguousarray(inst["ej"], dtype=np.int32)
    J = np.ascontiguousarray(inst["J"], dtype=np.float64)
    return n, h, ei, ej, J


def energy(inst, z: int) -> float:
    """E(z) of Eq. HC with s_i = 2 b_i - 1 (|0> is the -1 eigenstate, Sec. III.A.3)."""
    n, h, ei, ej, J = _inst(inst)
    return lib().orc_energy(n, _d(h), len(J), _i(ei), _i(ej), _d(J), int(z))


def energies(inst) -> np.ndarray:
    """E(z) for all 2^n basis states (Eq. HC)."""
    n, h, ei, ej, J = _inst(inst)
    E = np.empty(1 << n, dtype=np.float64)
    lib().orc_energies(n, _d(h), len(J), _i(ei), _i(ej), _d(J), _d(E))
    return E


def coeff_scale(inst) -> float:
    """sum |h| + sum |J|: bound on |E(z)|, used to scale tolerances."""
    return float(np.sum(np.abs(inst["h"])) + np.sum(np.abs(inst["J"])))


def ground_tol(inst) -> float:
    """Energies within this distance of the minimum count as ground states.
    Integer-valued instances compare exactly (tolerance 0)."""
    vals = np.concatenate([np.asarray(inst["h"]), np.asarray(inst["J"])])
    if np.all(vals == np.round(vals)):
        return 0.0
    return 1e-9 * max(1.0, coeff_scale(inst))


def ground(inst, E=None):
    """Brute-force ground state: (E_min, degeneracy, smallest argmin)."""
    n = int(inst["n"])
    if E is None:
        E = energies(inst)
    emin = ctypes.c_double()
    deg = ctypes.c_uint64()
    am = ctypes.c_uint64()
    lib().orc_ground(n, _d(E), ground_tol(inst), ctypes.byref(emin), ctypes.byref(deg), ctypes.byref(am))
    return emin.value, int(deg.value), int(am.value)


# ----------------------------------------------------------------------------- states
def _c2i(psi: np.ndarray) -> np.ndarray:
    """complex128[N] -> float64[2N] interleaved view/copy."""
    return np.ascontiguousarray(psi, dtype=np.complex128).view(np.float64)


def plus_state(n: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().orc_init_plus(n, _d(psi.view(np.float64)))
    return psi


def cost_phase(inst, psi: np.ndarray, gamma: float, E=None) -> np.ndarray:
    """exp(-i gamma H_C) psi (returns a new array)."""
    if E is None:
        E = energies(inst)
    out = np.array(psi, dtype=np.complex128, copy=True)
    lib().orc_cost_phase(int(inst["n"]), _d(E), float(gamma), _d(out.view(np.float64)))
    return out


def rx(n: int, psi: np.ndarray, q: int, beta: float) -> np.ndarray:
    """exp(-i beta sigma^x_q) psi (Eq. twocomponentupdates)."""
    out = np.array(psi, dtype=np.complex128, copy=True)
    lib().orc_rx(n, int(q), float(beta), _d(out.view(np.float64)))
    return out


def mixer(n: int, psi: np.ndarray, beta: float) -> np.ndarray:
    """exp(-i beta H_D) psi, H_D = sum_i sigma^x_i."""
    out = np.array(psi, dtype=np.complex128, copy=True)
    lib().orc_mixer(n, float(beta), _d(out.view(np.float64)))
    return out


def gate_1q(n: int, psi: np.ndarray, q: int, U) -> np.ndarray:
    """A 2x2 complex matrix U on qubit q (new array)."""
    u = np.ascontiguousarray(np.asarray(U, dtype=np.complex128).reshape(2, 2)).view(np.float64).reshape(-1)
    out = np.array(psi, dtype=np.complex128, copy=True)
    lib().orc_gate_1q(n, int(q), _d(u), _d(out.view(np.float64)))
    return out


def gate_layers(n: int, psi: np.ndarray, U) -> np.ndarray:
    """Layers of single-qubit gates, U[k, q] (2x2) on qubit q in layer k; within a
    layer the qubits go 0..n-1 (they commute)."""
    U = np.asarray(U, dtype=np.complex128)
    out = np.array(psi, dtype=np.complex128, copy=True)
    for k in range(U.shape[0]):
        for q in range(n):
            out = gate_1q(n, out, q, U[k, q])
    return out


def qaoa_state(inst, gamma, beta, psi0=None, E=None) -> np.ndarray:
    """Eq. QAOA_state: prod_k exp(-i beta_k H_D) exp(-i gamma_k H_C) applied to
    |+>^n (or to psi0 when given)."""
    n = int(inst["n"])
    gamma = np.ascontiguousarray(np.atleast_1d(gamma), dtype=np.float64)
    beta = np.ascontiguousarray(np.atleast_1d(beta), dtype=np.float64)
    assert len(gamma) == len(beta)
    if E is None:
        E = energies(inst)
    if psi0 is None:
        psi = np.empty(1 << n, dtype=np.complex128)
        from_plus = 1
    else:
        psi = np.array(psi0, dtype=np.complex128, copy=True)
        from_plus = 0
    lib().orc_qaoa(n, _d(E), len(gamma), _d(gamma), _d(beta), from_plus, _d(psi.view(np.float64)))
    return psi


def observables(inst, psi, E=None, gs=None):
    """(norm, <H_C>, ground-state probability) of psi (Sec. III.B.1)."""
    n = int(inst["n"])
    if E is None:
        E = energies(inst)
    if gs is None:
        gs = ground(inst, E)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    norm = ctypes.c_double()
    en = ctypes.c_double()
    pgs = ctypes.c_double()
    lib().orc_observables(n, _d(E), _d(psi.view(np.float64)), gs[0], ground_tol(inst),
                          ctypes.byref(norm), ctypes.byref(en), ctypes.byref(pgs))
    return norm.value, en.value, pgs.value


def spin_z(n: int, psi) -> np.ndarray:
    """<sigma^z_i> for every qubit (spin expectations of Sec. III.B.2)."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.empty(n, dtype=np.float64)
    lib().orc_spin_z(n, _d(psi.view(np.float64)), _d(out))
    return out


def grad_tangent(inst, gamma, beta, E=None):
    """(f, df/dgamma, df/dbeta) for f = <beta,gamma|H_C|beta,gamma> by forward-mode
    tangents (one extra state vector per parameter)."""
    n = int(inst["n"])
    gamma = np.ascontiguousarray(np.atleast_1d(gamma), dtype=np.float64)
    beta = np.ascontiguousarray(np.atleast_1d(beta), dtype=np.float64)
    p = len(gamma)
    if E is None:
        E = energies(inst)
    dg = np.empty(p)
    db = np.empty(p)
    f = ctypes.c_double()
    rc = lib().orc_grad_tangent(n, _d(E), p, _d(gamma), _d(beta), ctypes.byref(f), _d(dg), _d(db))
    if rc != 0:
        raise MemoryError("oracle gradient: allocation failed")
    return f.value, dg, db


def energy_of(inst, gamma, beta, E=None) -> float:
    if E is None:
        E = energies(inst)
    psi = qaoa_state(inst, gamma, beta, E=E)
    return observables(inst, psi, E=E, gs=(0.0, 0, 0))[1]


def grad_fd(inst, gamma, beta, h=1e-4, E=None):
    """Central finite differences with the Richardson pair (h, h/2):
    g = (4 D(h/2) - D(h)) / 3, truncation O(h^4)."""
    if E is None:
        E = energies(inst)
    gamma = np.array(np.atleast_1d(gamma), dtype=np.float64)
    beta = np.array(np.atleast_1d(beta), dtype=np.float64)
    p = len(gamma)

    def central(vec_is_gamma, k, step):
        g1, b1 = gamma.copy(), beta.copy()
        g2, b2 = gamma.copy(), beta.copy()
        if vec_is_gamma:
            g1[k] += step
            g2[k] -= step
        else:
            b1[k] += step
            b2[k] -= step
        return (energy_of(inst, g1, b1, E) - energy_of(inst, g2, b2, E)) / (2 * step)

    dg = np.empty(p)
    db = np.empty(p)
    for k in range(p):
        dg[k] = (4 * central(True, k, h / 2) - central(True, k, h)) / 3
        db[k] = (4 * central(False, k, h / 2) - central(False, k, h)) / 3
    return dg, db


# ----------------------------------------------------------------------------- exact cover
def exact_cover_ising(a):
    """Ising form of the exact cover objective sum_f (sum_i a_if x_i - 1)^2 with
    x_i = (1 + s_i)/2 (Eqs. exactcover, xtosigma): h_i = sum_j (a a^T)_ij / 2
    - (a b)_i, J_ij = (a a^T)_ij / 2 for i < j (Eqs. HChi, HCJij) and
    C = b^T b + sum_{i<j} (a a^T)_ij / 2 + sum_i ((a a^T)_ii - 2 (a b)_i) / 2
    (Eq. HCC), b = ones(F).  Returns (instance dict with the nonzero J_ij, C)."""
    a = np.asarray(a, dtype=np.int64)
    nr, nc = a.shape
    A = a @ a.T
    ab = a.sum(axis=1)
    h = 0.5 * A.sum(axis=1) - ab
    iu, ju = np.triu_indices(nr, k=1)
    Jall = 0.5 * A[iu, ju]
    keep = Jall != 0
    C = float(nc) + 0.5 * float(A[iu, ju].sum()) + 0.5 * float(np.sum(np.diag(A) - 2 * ab))
    inst = {"n": int(nr), "h": h.astype(np.float64), "ei": iu[keep].astype(np.int32),
            "ej": ju[keep].astype(np.int32), "J": Jall[keep].astype(np.float64)}
    return inst, C


def exact_cover_objective(a, z: int) -> int:
    """sum_f (sum_i a_if x_i - 1)^2 for the assignment x_i = bit i of z."""
    a = np.asarray(a, dtype=np.int64)
    x = (int(z) >> np.arange(a.shape[0])) & 1
    return int(np.sum((x @ a - 1) ** 2))


def rescale_factor(inst, hmax=2.0, jmax=1.0) -> float:
    """r of Eq. rescale with h_max = -h_min = 2 and J_max = -J_min = 1."""
    h = np.asarray(inst["h"], dtype=np.float64)
    J = np.asarray(inst["J"], dtype=np.float64)
    cands = [max(h.max() / hmax, 0.0), max(h.min() / -hmax, 0.0)]
    if len(J):
        cands += [max(J.max() / jmax, 0.0), max(J.min() / -jmax, 0.0)]
    return float(max(cands))


# ----------------------------------------------------------------------------- product states
def product_state_factors(h, gamma, beta) -> np.ndarray:
    """Single-qubit factors of the QAOA state when all couplings vanish (Eq. HC
    with J = 0): H_C = sum_i h_i s_i separates, so every layer of Eq. QAOA_state
    acts on each qubit alone and the state is the tensor product of
    phi_i = prod_k exp(-i beta_k X) exp(-i gamma_k h_i s) |+>, s = -1 for bit 0
    and +1 for bit 1 (Sec. III.A.3).  Returns phi[i, b], shape (n, 2)."""
    h = np.asarray(h, dtype=np.float64)
    phi = np.full((len(h), 2), 1.0 / math.sqrt(2.0), dtype=np.complex128)
    for g, b in zip(np.atleast_1d(gamma), np.atleast_1d(beta)):
        phi[:, 0] *= np.exp(1j * g * h)    # s = -1: exp(-i g h (-1))
        phi[:, 1] *= np.exp(-1j * g * h)   # s = +1
        c, sn = math.cos(b), math.sin(b)
        a0, a1 = phi[:, 0].copy(), phi[:, 1].copy()
        phi[:, 0] = c * a0 - 1j * sn * a1  # exp(-i b X) = c - i s X
        phi[:, 1] = c * a1 - 1j * sn * a0
    return phi


def factor_amplitudes(phi, zs) -> np.ndarray:
    """Amplitudes psi(z) = prod_i phi_i[bit_i(z)] of a product state at the basis
    indices zs (any n, no state vector)."""
    zs = np.asarray(zs, dtype=np.uint64)
    out = np.ones(len(zs), dtype=np.complex128)
    for i in range(phi.shape[0]):
        bit = ((zs >> np.uint64(i)) & np.uint64(1)).astype(np.int64)
        out *= phi[i, bit]
    return out


def factor_energy(h, phi) -> float:
    """<H_C> = sum_i h_i (|phi_i[1]|^2 - |phi_i[0]|^2) of a product state (J = 0)."""
    pz = np.abs(phi[:, 1]) ** 2 - np.abs(phi[:, 0]) ** 2
    return float(np.sum(np.asarray(h, dtype=np.float64) * pz))


def product_amplitudes(h, gamma, beta, zs) -> np.ndarray:
    """Amplitudes of the J = 0 QAOA state at the basis indices zs."""
    return factor_amplitudes(product_state_factors(h, gamma, beta), zs)


def product_energy(h, gamma, beta) -> float:
    """<H_C> of the J = 0 QAOA state."""
    return factor_energy(h, product_state_factors(h, gamma, beta))


def qsds_product_factors(h, tau, A, B) -> np.ndarray:
    """Single-qubit factors of the Eq. AQA4 state when all couplings vanish: the
    zz exponential is the identity, so each step acts on qubit i alone as the
    outer factor exp(i tau/2 (A X - B h_i Z)) applied twice.  phi[i, b], shape (n, 2)."""
    h = np.asarray(h, dtype=np.float64)
    phi = np.full((len(h), 2), 1.0 / math.sqrt(2.0), dtype=np.complex128)
    for a, b in zip(np.atleast_1d(A), np.atleast_1d(B)):
        for i in range(len(h)):
            m = single_spin_exponential(tau / 2.0, a, -b * h[i])
            phi[i] = m @ (m @ phi[i])
    return phi


# ----------------------------------------------------------------------------- QSDS time stepping
_SX = np.array([[0.0, 1.0], [1.0, 0.0]], dtype=np.complex128)
_SZ = np.array([[-1.0, 0.0], [0.0, 1.0]], dtype=np.complex128)   # |0> is the -1 eigenstate


def single_spin_exponential(theta: float, hx: float, hz: float) -> np.ndarray:
    """exp(i theta (hx sigma^x + hz sigma^z)) as a 2x2 matrix (scipy expm)."""
    from scipy.linalg import expm
    return expm(1j * theta * (hx * _SX + hz * _SZ))


def coupling_phase(inst, psi: np.ndarray, angle: float) -> np.ndarray:
    """exp(i angle sum_{i<j} J_ij sigma^z_i sigma^z_j) psi: the cost phase of the
    instance with its fields removed, at gamma = -angle."""
    zero = dict(inst)
    zero["h"] = np.zeros(int(inst["n"]))
    return cost_phase(zero, psi, -angle)


def qsds_run(inst, tau: float, A, B, psi0=None, observe: bool = False):
    """Eq. AQA4 for the Hamiltonian of Eqs. AQA0-AQA3: step l applies
        exp(i tau/2 sum_i (hx sigma^x_i + hz_i sigma^z_i))
        exp(i tau sum_{i<j} Jz_ij sigma^z_i sigma^z_j)
        exp(i tau/2 sum_i (hx sigma^x_i + hz_i sigma^z_i))
    with hx = A[l], hz_i = -B[l] h_i, Jz_ij = -B[l] J_ij, starting from |+>^n (or
    psi0).  observe=True also returns per-step (<H_C>, P_gs, <sigma^z_i>)."""
    n = int(inst["n"])
    h = np.asarray(inst["h"], dtype=np.float64)
    psi = plus_state(n) if psi0 is None else np.array(psi0, dtype=np.complex128)
    E = energies(inst) if observe else None
    gs = ground(inst, E) if observe else None
    en, pg, sz = [], [], []
    for a, b in zip(np.atleast_1d(A), np.atleast_1d(B)):
        outer = [single_spin_exponential(tau / 2.0, a, -b * h[i]) for i in range(n)]
        for i in range(n):
            psi = gate_1q(n, psi, i, outer[i])
        psi = coupling_phase(inst, psi, -tau * b)
        for i in range(n):
            psi = gate_1q(n, psi, i, outer[i])
        if observe:
            _, e, p = observables(inst, psi, E=E, gs=gs)
            en.append(e)
            pg.append(p)
            sz.append(spin_z(n, psi))
    if observe:
        return psi, np.array(en), np.array(pg), np.array(sz)
    return psi


# ----------------------------------------------------------------------------- schedules
def aqa_linear_schedule(steps: int, tau: float, paper_sign: bool = True):
    """Coarse first-order annealing steps with A(s) = 1 - s, B(s) = s (a linear
    stand-in for the DW_2000Q_6 schedule of Fig. 4, whose data is not available).

    Step k = 1..steps applies exp(-i tau B(s_k) H_C) then exp(+i tau A(s_k) H_D)
    with s_k = k/steps: the annealing Hamiltonian H(s) = A(s) H_I + B(s) H_C with
    H_I = -H_D (Eq. HI, Eq. Hofs).  In QAOA variables that is gamma_k = tau s_k and
    beta_k = -tau (1 - s_k).  ``paper_sign=False`` returns beta_k = +tau (1 - s_k),
    i.e. evolution under +H_D, which anneals toward the maximum of H_C.
    """
    s = np.arange(1, steps + 1, dtype=np.float64) / steps
    gamma = tau * s
    beta = (-1.0 if paper_sign else 1.0) * tau * (1.0 - s)
    return gamma, beta


def second_order_schedule(p: int, tau: float, A=None, B=None):
    """Second-order Suzuki-Trotter parameters (Eqs. beta_k-gamma_k, Appendix A).

    Grid s_k = (k-1)/(p-1), k = 1..p (Sec. III.B.1); for AQA with n steps the same
    grid arises from s_k = k/n, k = 0..n with p = n + 1 (Sec. III.B.2).
      beta_k  = -tau (A(s_{k+1}) + A(s_k)) / 2,  k = 1..p-1
      beta_p  = -tau A(s_p) / 2
      gamma_k =  tau B(s_k),                       k = 1..p
    A, B: callables of s or arrays of length p sampled on the grid; default to
    the linear stand-in A = 1 - s, B = s.  p = 1 has no grid (0/0) and is rejected.
    """
    if p < 2:
        raise ValueError("second-order schedule needs p >= 2")
    s = np.arange(p, dtype=np.float64) / (p - 1)
    a = _sample(A, s, lambda x: 1.0 - x)
    b = _sample(B, s, lambda x: x)
    beta = np.empty(p)
    beta[:-1] = -tau * (a[1:] + a[:-1]) / 2.0
    beta[-1] = -tau * a[-1] / 2.0
    gamma = tau * b
    return gamma, beta


def _sample(f, s, default):
    if f is None:
        return default(s)
    if callable(f):
        return np.array([f(x) for x in s], dtype=np.float64)
    arr = np.asarray(f, dtype=np.float64)
    if arr.shape != s.shape:
        raise ValueError("schedule array must have one value per grid point")
    return arr


# ----------------------------------------------------------------------------- block-separable instances
def coupling_components(inst):
    """Qubit sets of the connected components of the coupling graph (every listed
    pair (i, j) joins its two qubits, whatever J_ij), each sorted ascending;
    the components are ordered by their smallest qubit."""
    n = int(inst["n"])
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for i, j in zip(np.asarray(inst["ei"]).tolist(), np.asarray(inst["ej"]).tolist()):
        ri, rj = find(int(i)), find(int(j))
        if ri != rj:
            parent[max(ri, rj)] = min(ri, rj)
    groups = {}
    for q in range(n):
        groups.setdefault(find(q), []).append(q)
    return [sorted(g) for _, g in sorted(groups.items())]


def sub_instance(inst, qubits):
    """The part of Eq. HC that acts on the given qubits (a coupling component),
    relabelled so that qubits[r] becomes local qubit r."""
    qubits = [int(q) for q in qubits]
    local = {q: r for r, q in enumerate(qubits)}
    h = np.asarray(inst["h"], dtype=np.float64)[qubits]
    ei, ej, J = [], [], []
    for i, j, v in zip(np.asarray(inst["ei"]).tolist(), np.asarray(inst["ej"]).tolist(),
                       np.asarray(inst["J"]).tolist()):
        if int(i) in local:
            ei.append(local[int(i)])
            ej.append(local[int(j)])
            J.append(v)
    return {"n": len(qubits), "h": h, "ei": np.array(ei, dtype=np.int32), "ej": np.array(ej, dtype=np.int32),
            "J": np.array(J, dtype=np.float64)}


def block_states(inst, gamma, beta):
    """QAOA state of an instance whose coupling graph splits into small components,
    as one oracle state per component.  H_C is then a sum of terms on disjoint
    qubit sets and H_D a sum of single-qubit terms, so every factor of Eq.
    QAOA_state is a product over the components and the state is the tensor
    product of the components' own QAOA states (same gamma, beta).
    Returns [(qubits, psi_b)], psi_b indexed by the component's local bits."""
    out = []
    for qs in coupling_components(inst):
        out.append((qs, qaoa_state(sub_instance(inst, qs), gamma, beta)))
    return out


def block_amplitudes(blocks, zs) -> np.ndarray:
    """psi(z) = prod_b psi_b(z restricted to the qubits of component b) at the
    basis indices zs (any n; no full state vector)."""
    zs = np.asarray(zs, dtype=np.uint64)
    out = np.ones(len(zs), dtype=np.complex128)
    for qs, psi in blocks:
        loc = np.zeros(len(zs), dtype=np.int64)
        for r, q in enumerate(qs):
            loc |= (((zs >> np.uint64(q)) & np.uint64(1)).astype(np.int64)) << r
        out *= psi[loc]
    return out


def block_observables(inst, blocks):
    """(<H_C>, ground-state probability) of a product over coupling components:
    <H_C> = sum_b <H_b> (each factor has unit norm), and since E(z) = sum_b E_b(z_b)
    with the z_b independent, the ground set is the product of the components'
    ground sets and P_gs = prod_b P_gs,b."""
    en, pg = 0.0, 1.0
    for qs, psi in blocks:
        sub = sub_instance(inst, qs)
        _, e, p = observables(sub, psi)
        en += e
        pg *= p
    return en, pg


def block_grad(inst, gamma, beta):
    """(f, df/dgamma, df/dbeta) of a component-separable instance: f = sum_b f_b with
    f_b the QAOA energy of component b at the same (gamma, beta), so the gradient
    is the sum of the components' forward-mode tangent gradients."""
    p = len(np.atleast_1d(gamma))
    f, dg, db = 0.0, np.zeros(p), np.zeros(p)
    for qs in coupling_components(inst):
        fb, gb, bb = grad_tangent(sub_instance(inst, qs), gamma, beta)
        f += fb
        dg += gb
        db += bb
    return f, dg, db


def block_aqa_observables(inst, gamma, beta):
    """Per-step (<H_C>[k], P_gs[k]) of the layer sequence (gamma_k, beta_k) on a
    component-separable instance, from the components' step-by-step states."""
    comps = [(qs, sub_instance(inst, qs)) for qs in coupling_components(inst)]
    states = [plus_state(len(qs)) for qs, _ in comps]
    gss = [ground(sub) for _, sub in comps]
    en, pg = [], []
    for g, b in zip(np.atleast_1d(gamma), np.atleast_1d(beta)):
        e_sum, p_prod = 0.0, 1.0
        for c, (qs, sub) in enumerate(comps):
            states[c] = qaoa_state(sub, [g], [b], psi0=states[c])
            _, e, p = observables(sub, states[c], gs=gss[c])
            e_sum += e
            p_prod *= p
        en.append(e_sum)
        pg.append(p_prod)
    return np.array(en), np.array(pg)
