"""Thin ctypes binding of libsv.so (declared in include/sv.h).

Argument marshalling only: every step of the simulation runs in the library's
HIP kernels.  PyTorch supplies device memory and the stream.  If libsv.so is
missing the import fails; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import json
import os
from pathlib import Path
from typing import Optional, Sequence

import numpy as np

_HERE = Path(__file__).resolve().parent
# SV_LIBRARY names another build of the same sources (the sanitized host build
# libsv_san.so of build.py); default: the in-tree libsv.so
LIB_PATH = Path(os.environ["SV_LIBRARY"]).resolve() if os.environ.get("SV_LIBRARY") else _HERE / "libsv.so"

SV_C64, SV_C128 = 1, 2
_CODES = {0: "ok", 1: "bad argument", 2: "out of memory", 3: "HIP error", 4: "unsupported", 5: "non-finite value"}


class SVError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsv error {code} ({_CODES.get(code, '?')}): {msg}")
        self.code = code


def _load():
    if not LIB_PATH.exists():
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2104_03293_amd.build` "
            "(the HIP library is required; there is no fallback)")
    # torch ships its own HIP runtime under the same soname; loading torch first
    # makes libsv.so bind to that copy, so the process holds one runtime and
    # torch's streams and allocations are valid handles for the library
    import torch  # noqa: F401

    L = ctypes.CDLL(str(LIB_PATH))
    vp, dp, ip, u64p, i32p = (ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                              ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int32))
    sig = {
        "sv_last_error": (ctypes.c_char_p, []),
        "sv_version": (ctypes.c_char_p, []),
        "sv_alloc": (ip, [ip, ip, vp, ctypes.POINTER(vp)]),
        "sv_wrap": (ip, [ip, ip, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
        "sv_free": (ip, [vp]),
        "sv_set_stream": (ip, [vp, vp]),
        "sv_init_plus": (ip, [vp]),
        "sv_copy_to_host": (ip, [vp, vp, ctypes.c_size_t]),
        "sv_copy_from_host": (ip, [vp, vp, ctypes.c_size_t]),
        "sv_ising_create": (ip, [ip, dp, ip, i32p, i32p, dp, ctypes.POINTER(vp)]),
        "sv_ising_free": (ip, [vp]),
        "sv_ising_exact_cover": (ip, [ip, ip, ctypes.POINTER(ctypes.c_uint8), dp, ctypes.POINTER(vp)]),
        "sv_rescale_factor": (ip, [vp, dp]),
        "sv_ground": (ip, [vp, dp, u64p, u64p]),
        "sv_cost_phase": (ip, [vp, vp, ctypes.c_double]),
        "sv_mixer": (ip, [vp, ctypes.c_double]),
        "sv_qaoa_forward": (ip, [vp, vp, ip, dp, dp, ip]),
        "sv_qaoa_energy": (ip, [vp, vp, ip, dp, dp, ip, dp, dp, dp]),
        "sv_qaoa_energy_noalloc": (ip, [vp, vp, ip, dp, dp, ip, vp]),
        "sv_aqa_run": (ip, [vp, vp, ip, dp, dp, dp, dp]),
        "sv_aqa_run_observe": (ip, [vp, vp, ip, dp, dp, dp, dp, dp]),
        "sv_spin_z": (ip, [vp, dp]),
        "sv_expect": (ip, [vp, vp, dp, dp, dp]),
        "sv_gate_layers": (ip, [vp, ip, dp]),
        "sv_qsds_run": (ip, [vp, vp, ip, ctypes.c_double, dp, dp, ip, dp, dp, dp]),
        "sv_grad": (ip, [vp, vp, vp, ip, dp, dp, ip, dp, dp, dp, dp]),
        "sv_schedule_linear": (ip, [ip, ctypes.c_double, ip, dp, dp]),
        "sv_schedule_second_order": (ip, [ip, ctypes.c_double, dp, dp, dp, dp]),
        "sv_batch_p1_scan": (ip, [ip, ctypes.POINTER(vp), ip, dp, ip, dp, ip, vp, dp, dp]),
        "sv_tune_set": (ip, [ctypes.c_char_p, ip]),
        "sv_tune_get": (ip, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)]),
        "sv_tune_describe": (ip, [ip, ip, ctypes.c_char_p, ctypes.c_size_t]),
        "sv_tune_load": (ip, [ctypes.c_char_p]),
        "sv_profile_enable": (ip, [ip]),
        "sv_profile_report": (ip, [ctypes.c_char_p, ctypes.c_size_t]),
        "sv_stream_ceiling": (ip, [vp, ip, ip, dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()


def _check(rc: int) -> None:
    if rc != 0:
        raise SVError(rc, lib.sv_last_error().decode())


def last_error() -> str:
    return lib.sv_last_error().decode()


def version() -> str:
    return lib.sv_version().decode()


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.atleast_1d(np.asarray(x, dtype=np.float64)))


def _stream_handle(stream=None) -> int:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


# ----------------------------------------------------------------------------- instances
class Ising:
    """Ising instance of Eq. HC (h_i fields, couplings (i, j, J_ij)) on the device."""

    def __init__(self, n: int, h, ei, ej, J):
        h = _f64(h)
        ei = np.ascontiguousarray(np.asarray(ei, dtype=np.int32).reshape(-1))
        ej = np.ascontiguousarray(np.asarray(ej, dtype=np.int32).reshape(-1))
        J = _f64(J) if len(np.atleast_1d(J)) else np.zeros(0)
        if len(h) != n or not (len(ei) == len(ej) == len(J)):
            raise ValueError("Ising: inconsistent array lengths")
        self.n, self.m = int(n), len(J)
        self.h, self.ei, self.ej, self.J = h, ei, ej, J
        handle = ctypes.c_void_p()
        _check(lib.sv_ising_create(int(n), _dp(h), self.m, ei.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   ej.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(J),
                                   ctypes.byref(handle)))
        self._h = handle

    @classmethod
    def from_instance(cls, inst: dict) -> "Ising":
        return cls(inst["n"], inst["h"], inst["ei"], inst["ej"], inst["J"])

    @classmethod
    def exact_cover(cls, a):
        """Ising form of the exact cover matrix a (rows = qubits, Sec. III.A.3)
        built by the library: (instance, constant C), E(z) + C = objective."""
        a = np.ascontiguousarray(np.asarray(a, dtype=np.uint8))
        if a.ndim != 2:
            raise ValueError("exact cover matrix must be 2-D")
        obj = cls.__new__(cls)
        handle = ctypes.c_void_p()
        c = ctypes.c_double()
        _check(lib.sv_ising_exact_cover(a.shape[0], a.shape[1], a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                        ctypes.byref(c), ctypes.byref(handle)))
        obj._h = handle
        obj.n, obj.m = a.shape[0], -1
        return obj, c.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.sv_ising_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rescale_factor(H: Ising) -> float:
    """r of Eq. rescale (apply as gamma / r and <H_C> * r)."""
    r = ctypes.c_double()
    _check(lib.sv_rescale_factor(H.handle, ctypes.byref(r)))
    return r.value


def ground(H: Ising):
    """(E_min, degeneracy, smallest argmin) by full enumeration on the GPU."""
    e = ctypes.c_double()
    d = ctypes.c_uint64()
    a = ctypes.c_uint64()
    _check(lib.sv_ground(H.handle, ctypes.byref(e), ctypes.byref(d), ctypes.byref(a)))
    return e.value, int(d.value), int(a.value)


# ----------------------------------------------------------------------------- states
class State:
    """2^n amplitudes in device memory: a torch tensor (default) or a
    library-owned buffer (owner="lib", for states near the HBM capacity)."""

    def __init__(self, n: int, dtype: str = "c128", device: int = 0, owner: str = "torch", stream=None):
        import torch

        if dtype not in ("c64", "c128"):
            raise ValueError("dtype must be 'c64' or 'c128'")
        self.n, self.dtype = int(n), dtype
        self.code = SV_C128 if dtype == "c128" else SV_C64
        self.elem = 16 if dtype == "c128" else 8
        self.device = torch.device("cuda", device)
        self.stream = stream
        h = ctypes.c_void_p()
        sh = _stream_handle(stream)
        if owner == "torch":
            tdt = torch.complex128 if dtype == "c128" else torch.complex64
            with torch.cuda.device(self.device):
                self.tensor = torch.empty(1 << self.n, dtype=tdt, device=self.device)
            _check(lib.sv_wrap(self.n, self.code, ctypes.c_void_p(self.tensor.data_ptr()),
                               self.tensor.numel() * self.elem, ctypes.c_void_p(sh), ctypes.byref(h)))
        elif owner == "lib":
            self.tensor = None
            with torch.cuda.device(self.device):
                _check(lib.sv_alloc(self.n, self.code, ctypes.c_void_p(sh), ctypes.byref(h)))
        else:
            raise ValueError("owner must be 'torch' or 'lib'")
        self._h = h

    @property
    def handle(self):
        return self._h

    @property
    def nbytes(self) -> int:
        return (1 << self.n) * self.elem

    def to_numpy(self) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=np.complex128 if self.dtype == "c128" else np.complex64)
        _check(lib.sv_copy_to_host(self._h, ctypes.c_void_p(out.ctypes.data), out.nbytes))
        return out

    def from_numpy(self, a) -> None:
        a = np.ascontiguousarray(a, dtype=np.complex128 if self.dtype == "c128" else np.complex64)
        if a.size != 1 << self.n:
            raise ValueError("size mismatch")
        _check(lib.sv_copy_from_host(self._h, ctypes.c_void_p(a.ctypes.data), a.nbytes))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.sv_free(self._h)
            self._h = ctypes.c_void_p()
        self.tensor = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- operations
def init_plus(s: State) -> None:
    _check(lib.sv_init_plus(s.handle))


def cost_phase(s: State, H: Ising, gamma: float) -> None:
    _check(lib.sv_cost_phase(s.handle, H.handle, float(gamma)))


def mixer(s: State, beta: float) -> None:
    _check(lib.sv_mixer(s.handle, float(beta)))


def qaoa_forward(s: State, H: Ising, gamma, beta, from_plus: bool = True) -> None:
    g, b = _f64(gamma), _f64(beta)
    if len(g) != len(b):
        raise ValueError("gamma and beta must have equal length")
    _check(lib.sv_qaoa_forward(s.handle, H.handle, len(g), _dp(g), _dp(b), int(bool(from_plus))))


def qaoa_energy(s: State, H: Ising, gamma, beta, from_plus: bool = True):
    """QAOA forward with the observables fused into its last pass: (energy, p_gs, norm)."""
    g, b = _f64(gamma), _f64(beta)
    if len(g) != len(b):
        raise ValueError("gamma and beta must have equal length")
    e, p, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib.sv_qaoa_energy(s.handle, H.handle, len(g), _dp(g), _dp(b), int(bool(from_plus)), ctypes.byref(e),
                              ctypes.byref(p), ctypes.byref(n)))
    return e.value, p.value, n.value


def qaoa_energy_noalloc(s: State, H: Ising, gamma, beta, out, from_plus: bool = True) -> None:
    """sv_qaoa_energy without allocation: writes (norm, energy, p_gs) into the
    float64 CUDA tensor out (3 elements, on the state's device) on the state's
    stream and returns without synchronising."""
    import torch

    g, b = _f64(gamma), _f64(beta)
    if len(g) != len(b):
        raise ValueError("gamma and beta must have equal length")
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64 and out.numel() >= 3
            and out.is_contiguous()):
        raise ValueError("out must be a contiguous float64 CUDA tensor of at least 3 elements")
    _check(lib.sv_qaoa_energy_noalloc(s.handle, H.handle, len(g), _dp(g), _dp(b), int(bool(from_plus)),
                                      ctypes.c_void_p(out.data_ptr())))


def aqa_run(s: State, H: Ising, gamma, beta, per_step: bool = False):
    g, b = _f64(gamma), _f64(beta)
    if len(g) != len(b):
        raise ValueError("gamma and beta must have equal length")
    if per_step:
        pg = np.empty(len(g))
        en = np.empty(len(g))
        _check(lib.sv_aqa_run(s.handle, H.handle, len(g), _dp(g), _dp(b), _dp(pg), _dp(en)))
        return pg, en
    null = ctypes.POINTER(ctypes.c_double)()
    _check(lib.sv_aqa_run(s.handle, H.handle, len(g), _dp(g), _dp(b), null, null))
    return None


def aqa_run_observe(s: State, H: Ising, gamma, beta):
    """AQA run returning per-step (P_gs[steps], <H_C>[steps], <sigma^z>[steps, n])."""
    g, b = _f64(gamma), _f64(beta)
    if len(g) != len(b):
        raise ValueError("gamma and beta must have equal length")
    pg = np.empty(len(g))
    en = np.empty(len(g))
    sz = np.empty((len(g), s.n))
    _check(lib.sv_aqa_run_observe(s.handle, H.handle, len(g), _dp(g), _dp(b), _dp(pg), _dp(en), _dp(sz)))
    return pg, en, sz


def spin_z(s: State) -> np.ndarray:
    """<sigma^z_i> of the current state for every qubit i."""
    out = np.empty(s.n)
    _check(lib.sv_spin_z(s.handle, _dp(out)))
    return out


def gate_layers(s: State, U) -> None:
    """Apply single-qubit gate layers: U has shape (layers, n, 2, 2) complex
    (layer k applies U[k, q] to qubit q)."""
    U = np.asarray(U, dtype=np.complex128)
    if U.ndim != 4 or U.shape[1:] != (s.n, 2, 2):
        raise ValueError(f"U must have shape (layers, {s.n}, 2, 2)")
    flat = np.ascontiguousarray(U).view(np.float64).reshape(-1)
    _check(lib.sv_gate_layers(s.handle, U.shape[0], _dp(flat)))


def qsds_run(s: State, H: Ising, tau: float, A, B, from_plus: bool = True, observe: bool = False):
    """Eq. AQA4 time stepping with the annealing samples A[l], B[l]; with
    observe=True returns per-step (<H_C>[steps], P_gs[steps], <sigma^z>[steps, n])."""
    a, b = _f64(A), _f64(B)
    if len(a) != len(b):
        raise ValueError("A and B must have equal length")
    if observe:
        en = np.empty(len(a))
        pg = np.empty(len(a))
        sz = np.empty((len(a), s.n))
        _check(lib.sv_qsds_run(s.handle, H.handle, len(a), float(tau), _dp(a), _dp(b), int(bool(from_plus)),
                               _dp(en), _dp(pg), _dp(sz)))
        return en, pg, sz
    null = ctypes.POINTER(ctypes.c_double)()
    _check(lib.sv_qsds_run(s.handle, H.handle, len(a), float(tau), _dp(a), _dp(b), int(bool(from_plus)), null, null,
                           null))
    return None


def expect(s: State, H: Ising):
    """(energy <H_C>, ground-state probability, norm)."""
    e, p, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib.sv_expect(s.handle, H.handle, ctypes.byref(e), ctypes.byref(p), ctypes.byref(n)))
    return e.value, p.value, n.value


def grad(psi: State, lam: State, H: Ising, gamma, beta, psi_is_forward: bool = False, with_pgs: bool = False):
    """(energy, dE/dgamma[p], dE/dbeta[p]) by the adjoint reverse sweep;
    with_pgs=True: (energy, p_gs, dE/dgamma[p], dE/dbeta[p])."""
    g, b = _f64(gamma), _f64(beta)
    if len(g) != len(b):
        raise ValueError("gamma and beta must have equal length")
    e, pg = ctypes.c_double(), ctypes.c_double()
    dg = np.empty(len(g))
    db = np.empty(len(g))
    _check(lib.sv_grad(psi.handle, lam.handle, H.handle, len(g), _dp(g), _dp(b), int(bool(psi_is_forward)),
                       ctypes.byref(e), ctypes.byref(pg), _dp(dg), _dp(db)))
    if with_pgs:
        return e.value, pg.value, dg, db
    return e.value, dg, db


def schedule_linear(steps: int, tau: float, paper_sign: bool = True):
    g = np.empty(steps)
    b = np.empty(steps)
    _check(lib.sv_schedule_linear(int(steps), float(tau), int(bool(paper_sign)), _dp(g), _dp(b)))
    return g, b


def schedule_second_order(p: int, tau: float, A: Optional[Sequence[float]] = None,
                          B: Optional[Sequence[float]] = None):
    g = np.empty(p)
    b = np.empty(p)
    null = ctypes.POINTER(ctypes.c_double)()
    a_arr = _f64(A) if A is not None else None
    b_arr = _f64(B) if B is not None else None
    for arr in (a_arr, b_arr):
        if arr is not None and len(arr) != p:
            raise ValueError("schedule arrays must have length p")
    _check(lib.sv_schedule_second_order(int(p), float(tau), _dp(a_arr) if a_arr is not None else null,
                                        _dp(b_arr) if b_arr is not None else null, _dp(g), _dp(b)))
    return g, b


def batch_p1_scan(instances: Sequence[Ising], gammas, betas, dtype: str = "c64", stream=None):
    g, b = _f64(gammas), _f64(betas)
    n_inst = len(instances)
    arr = (ctypes.c_void_p * n_inst)(*[H.handle.value for H in instances])
    en = np.empty((n_inst, len(g), len(b)))
    pg = np.empty((n_inst, len(g), len(b)))
    code = SV_C128 if dtype == "c128" else SV_C64
    _check(lib.sv_batch_p1_scan(n_inst, arr, len(g), _dp(g), len(b), _dp(b), code,
                                ctypes.c_void_p(_stream_handle(stream)), _dp(en), _dp(pg)))
    return en, pg


def tune_set(name: str, value: int) -> None:
    _check(lib.sv_tune_set(name.encode(), int(value)))


def tune_get(name: str) -> int:
    v = ctypes.c_int()
    _check(lib.sv_tune_get(name.encode(), ctypes.byref(v)))
    return v.value


def tune_load(path=None) -> None:
    _check(lib.sv_tune_load(None if path is None else str(path).encode()))


def describe(n: int, dtype: str = "c128") -> dict:
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib.sv_tune_describe(int(n), SV_C128 if dtype == "c128" else SV_C64, buf, len(buf)))
    return json.loads(buf.value.decode())


def profile_enable(on: bool = True) -> None:
    _check(lib.sv_profile_enable(int(bool(on))))


def profile_report() -> dict:
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib.sv_profile_report(buf, len(buf)))
    return json.loads(buf.value.decode())


def stream_ceiling(s: State, c: int, lo: int = 0) -> float:
    """Kernel time (ms) of one in-place streaming read + write of the state with
    the tile passes' access pattern for carrier bits c and group start lo."""
    ms = ctypes.c_double()
    _check(lib.sv_stream_ceiling(s.handle, int(c), int(lo), ctypes.byref(ms)))
    return ms.value


# ----------------------------------------------------------------------------- autograd
class QAOAEnergy:
    """torch.autograd.Function wrapper: f(gamma, beta) = <beta,gamma|H_C|beta,gamma>.

    When gamma or beta needs a gradient, the forward call runs the library's
    adjoint sweep (forward circuit plus one reverse sweep) and keeps the 2p
    derivatives for backward; otherwise (no input requires grad, or grad mode
    is off) it runs only the energy evaluation, and lam is not touched.
    """

    @staticmethod
    def apply(gamma, beta, psi: State, lam: State, H: Ising):
        import torch

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(ctx, g, b):
                gn, bn = g.detach().cpu().numpy(), b.detach().cpu().numpy()
                e, dg, db = grad(psi, lam, H, gn, bn)
                ctx.save_for_backward(torch.from_numpy(dg).to(g), torch.from_numpy(db).to(b))
                return torch.tensor(e, dtype=g.dtype, device=g.device)

            @staticmethod
            def backward(ctx, go):
                dg, db = ctx.saved_tensors
                return go * dg, go * db

        if not torch.is_grad_enabled() or not (gamma.requires_grad or beta.requires_grad):
            e, _, _ = qaoa_energy(psi, H, gamma.detach().cpu().numpy(), beta.detach().cpu().numpy())
            return torch.tensor(e, dtype=gamma.dtype, device=gamma.device)
        return _F.apply(gamma, beta)
