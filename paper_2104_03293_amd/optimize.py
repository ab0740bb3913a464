"""Classical optimisation loop around the QAOA energy (Sec. III.B.1, Sec. III.C.1).

The variational parameters (gamma_1..p, beta_1..p) of the QAOA state are handed
to a scipy optimiser that minimises the energy <H_C>; every evaluation is one
call of the simulator, and the loop stops after a fixed number of calls even if
the optimiser has not converged (the paper caps it at 200).  The paper's four
optimisers are SLSQP, Nelder-Mead, L-BFGS-B and CG.  The gradient-based ones can
take their derivatives from the library's adjoint sweep (one call for all 2p
derivatives) instead of finite differences (2p extra energy calls each time);
the result records both counts so the two ways of paying for a gradient can be
compared.

Rescaling (Eq. rescale): with `scale=r` the optimiser sees the problem H_C / r,
i.e. the variables (r*gamma, beta) and the objective <H_C>/r; results and the
history are reported in the original units.

Initial parameters follow the paper's second-order Trotter initialisation
(Eqs. beta_k-gamma_k) via `second_order_init`.
"""
from __future__ import annotations

import json
import time
from dataclasses import asdict, dataclass, field
from typing import List, Optional, Sequence

import numpy as np

PAPER_METHODS = ("SLSQP", "Nelder-Mead", "L-BFGS-B", "CG")
GRADIENT_METHODS = ("SLSQP", "L-BFGS-B", "CG", "BFGS", "TNC")


class DeviceQAOA:
    """Energy, ground-state probability and adjoint gradient of the p-layer QAOA
    state of one instance, evaluated by the library on the GPU."""

    def __init__(self, H, dtype: str = "c128"):
        from . import sv
        self._sv = sv
        self.H = H
        self.dtype = dtype
        self.psi = sv.State(H.n, dtype)
        self.lam = None

    def energy(self, gamma, beta):
        e, pgs, _ = self._sv.qaoa_energy(self.psi, self.H, gamma, beta)
        return e, pgs

    def energy_grad(self, gamma, beta):
        if self.lam is None:
            self.lam = self._sv.State(self.H.n, self.dtype)
        return self._sv.grad(self.psi, self.lam, self.H, gamma, beta, with_pgs=True)

    def close(self):
        for s in (self.psi, self.lam):
            if s is not None:
                s.close()


def second_order_init(p: int, tau: float, A: Optional[Sequence[float]] = None,
                      B: Optional[Sequence[float]] = None):
    """(gamma, beta) of the second-order initialisation (Eqs. beta_k-gamma_k)."""
    from . import sv
    return sv.schedule_second_order(p, tau, A, B)


@dataclass
class Call:
    index: int
    kind: str                      # "energy" or "grad"
    gamma: List[float]
    beta: List[float]
    energy: float
    p_gs: float
    seconds: float
    dgamma: Optional[List[float]] = None
    dbeta: Optional[List[float]] = None


@dataclass
class OptResult:
    method: str
    p: int
    gamma: List[float]             # best point (lowest energy over all calls)
    beta: List[float]
    energy: float
    p_gs: float
    calls: int                     # simulator calls (energy + adjoint)
    energy_calls: int
    grad_calls: int
    fd_equivalent_calls: int       # energy calls a forward-difference gradient would need instead
    max_calls: int
    budget_hit: bool
    converged: bool
    message: str
    scale: float
    use_grad: bool
    history: List[Call] = field(default_factory=list)

    def to_json(self, path: Optional[str] = None) -> str:
        text = json.dumps(asdict(self), indent=1)
        if path is not None:
            with open(path, "w") as f:
                f.write(text)
        return text

    @staticmethod
    def from_json(text: str) -> "OptResult":
        d = json.loads(text)
        d["history"] = [Call(**c) for c in d["history"]]
        return OptResult(**d)


def time_to_energy(result: "OptResult", target: float) -> Optional[dict]:
    """Simulator seconds and calls until the run first reached <H_C> <= target
    (None if it never did): the fair comparison of two optimisers that stop at
    different energies."""
    t = 0.0
    for c in result.history:
        t += c.seconds
        if c.energy <= target:
            return {"seconds": t, "calls": c.index + 1}
    return None


class _Budget(Exception):
    pass


def optimize_qaoa(sim, gamma0, beta0, method: str = "SLSQP", max_calls: int = 200,
                  use_grad: Optional[bool] = None, scale: float = 1.0, tol: Optional[float] = None,
                  options: Optional[dict] = None) -> OptResult:
    """Minimise <H_C> over (gamma, beta) starting at (gamma0, beta0).

    sim: an object with energy(gamma, beta) -> (E, P_gs) and
         energy_grad(gamma, beta) -> (E, P_gs, dE/dgamma, dE/dbeta)
         (`DeviceQAOA` for the GPU).
    use_grad: take derivatives from energy_grad (default: True for the
         gradient-based methods); False lets scipy difference energy calls.
    max_calls: hard cap on simulator calls; the loop stops when it is reached.
    scale: the rescale factor r of Eq. rescale (1 = no rescaling).
    """
    from scipy.optimize import minimize

    g0 = np.asarray(gamma0, dtype=np.float64).reshape(-1)
    b0 = np.asarray(beta0, dtype=np.float64).reshape(-1)
    if len(g0) != len(b0) or len(g0) == 0:
        raise ValueError("gamma0 and beta0 must be non-empty and of equal length")
    if max_calls < 1:
        raise ValueError("max_calls must be >= 1")
    if not (np.isfinite(scale) and scale > 0):
        raise ValueError("scale must be a positive finite number")
    p = len(g0)
    if use_grad is None:
        use_grad = method in GRADIENT_METHODS
    if use_grad and method not in GRADIENT_METHODS:
        raise ValueError(f"method {method} does not use gradients")
    r = float(scale)
    hist: List[Call] = []

    def split(x):
        return x[:p] / r, x[p:].copy()

    def record(kind, g, b, e, pg, t0, dg=None, db=None):
        hist.append(Call(len(hist), kind, g.tolist(), b.tolist(), float(e), float(pg), time.perf_counter() - t0,
                         None if dg is None else np.asarray(dg).tolist(),
                         None if db is None else np.asarray(db).tolist()))

    def fun(x):
        if len(hist) >= max_calls:
            raise _Budget()
        g, b = split(x)
        t0 = time.perf_counter()
        e, pg = sim.energy(g, b)
        record("energy", g, b, e, pg, t0)
        return e / r

    def fun_grad(x):
        if len(hist) >= max_calls:
            raise _Budget()
        g, b = split(x)
        t0 = time.perf_counter()
        e, pg, dg, db = sim.energy_grad(g, b)
        record("grad", g, b, e, pg, t0, dg, db)
        # d(E/r)/d(r gamma) = dE/dgamma / r^2, d(E/r)/d beta = dE/dbeta / r
        return e / r, np.concatenate([np.asarray(dg) / (r * r), np.asarray(db) / r])

    x0 = np.concatenate([g0 * r, b0])
    budget_hit, converged, message = False, False, ""
    try:
        if use_grad:
            res = minimize(fun_grad, x0, jac=True, method=method, tol=tol, options=options)
        else:
            res = minimize(fun, x0, method=method, tol=tol, options=options)
        converged, message = bool(res.success), str(res.message)
    except _Budget:
        budget_hit, message = True, f"stopped after {max_calls} simulator calls"
    if not hist:
        raise RuntimeError("optimizer made no simulator call")
    best = min(hist, key=lambda c: c.energy)
    ne = sum(1 for c in hist if c.kind == "energy")
    ng = len(hist) - ne
    return OptResult(method=method, p=p, gamma=list(best.gamma), beta=list(best.beta), energy=best.energy,
                     p_gs=best.p_gs, calls=len(hist), energy_calls=ne, grad_calls=ng,
                     fd_equivalent_calls=ne + ng * (2 * p + 1), max_calls=int(max_calls), budget_hit=budget_hit,
                     converged=converged, message=message, scale=r, use_grad=bool(use_grad), history=hist)
