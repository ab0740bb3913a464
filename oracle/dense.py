"""Dense-matrix cross-check for n <= 10 (TEST INFRASTRUCTURE ONLY).

Builds H_C and H_D as explicit 2^n x 2^n matrices from Kronecker products of
2x2 Pauli matrices, with qubit 0 as the LAST (rightmost) factor so that it is
bit 0 of the basis index (Sec. II.A tensor notation), and sigma^z = diag(-1, +1)
in the {|0>, |1>} basis because the paper labels the -1 eigenstate |0>
(Sec. III.A.3).  The exponentials are taken with scipy.linalg.expm: the exact
action of each matrix exponential on a state (Sec. III.B.2, remark after Eq. AQA4).

Shares no code with oracle.c: no bit loops, no butterflies.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

X = np.array([[0.0, 1.0], [1.0, 0.0]], dtype=np.complex128)
Z_PAPER = np.array([[-1.0, 0.0], [0.0, 1.0]], dtype=np.complex128)
I2 = np.eye(2, dtype=np.complex128)


def single(n: int, q: int, P: np.ndarray) -> np.ndarray:
    """P acting on qubit q: I x ... x P x ... x I with qubit 0 as the last factor."""
    M = np.ones((1, 1), dtype=np.complex128)
    for pos in range(n - 1, -1, -1):
        M = np.kron(M, P if pos == q else I2)
    return M


def h_cost(inst) -> np.ndarray:
    n = int(inst["n"])
    H = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    Zs = [single(n, q, Z_PAPER) for q in range(n)]
    for i in range(n):
        H += inst["h"][i] * Zs[i]
    for a, b, j in zip(inst["ei"], inst["ej"], inst["J"]):
        H += j * (Zs[int(a)] @ Zs[int(b)])
    return H


def h_driver(n: int) -> np.ndarray:
    H = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for q in range(n):
        H += single(n, q, X)
    return H


def plus(n: int) -> np.ndarray:
    v = np.ones(2, dtype=np.complex128) / np.sqrt(2.0)
    out = np.ones(1, dtype=np.complex128)
    for _ in range(n):
        out = np.kron(out, v)
    return out


def qaoa_state(inst, gamma, beta, psi0=None) -> np.ndarray:
    n = int(inst["n"])
    HC, HD = h_cost(inst), h_driver(n)
    psi = plus(n) if psi0 is None else np.array(psi0, dtype=np.complex128)
    for g, b in zip(np.atleast_1d(gamma), np.atleast_1d(beta)):
        psi = expm(-1j * g * HC) @ psi
        psi = expm(-1j * b * HD) @ psi
    return psi


def energy(inst, psi) -> float:
    return float(np.real(np.conj(psi) @ (h_cost(inst) @ psi)))
