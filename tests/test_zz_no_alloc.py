"""sv_qaoa_energy_noalloc against sv_qaoa_energy, through the C ABI.

The no-allocation entry point runs the same program and kernels as
sv_qaoa_energy with its reduction partials and phase tables in the library's
fixed device array; its results must equal those of sv_qaoa_energy (the
energies to the relative 1e-6 of the parity bar and the probabilities and
norms to 1e-11, and in fact bit for bit, since the reduction order is the
same), on consecutive calls whose second input is smaller than the first.
"""
import ctypes
import sys

import numpy as np
import pytest

from paper_2104_03293_amd import inputs as I

pytestmark = pytest.mark.gpu


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


def _reference(sv, H, n, dtype, g, b):
    s = sv.State(n, dtype)
    e, pg, nrm = sv.qaoa_energy(s, H, g, b)
    return (nrm, e, pg), s.to_numpy()


def _noalloc(sv, H, n, dtype, g, b, out):
    import torch

    s = sv.State(n, dtype)
    out.fill_(np.nan)
    sv.qaoa_energy_noalloc(s, H, g, b, out)
    torch.cuda.synchronize()
    return tuple(float(x) for x in out.cpu().numpy()), s.to_numpy()


def _same(got, ref, scale):
    nrm, e, pg = got
    rn, re, rp = ref
    assert abs(e - re) <= 1e-6 * max(abs(re), scale), (e, re)
    assert abs(pg - rp) <= 1e-11 and abs(nrm - rn) <= 1e-11, (got, ref)
    assert got == ref, (got, ref)  # same kernels, same reduction order


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noalloc_energy_matches_sv_qaoa_energy(sv, orc, dtype):
    """Two calls in a row, the second on a smaller state (n = 26: three tile
    groups, then n = 18), each against sv_qaoa_energy on the same seeded
    instance and angles; the final states are identical too."""
    import torch

    out = torch.empty(3, dtype=torch.float64, device="cuda")
    for n, p, seed in ((26, 4, 11), (18, 3, 12)):
        inst = I.degree4_int2(n, seed)
        H = sv.Ising.from_instance(inst)
        g, b = I.uniform_params(p, seed)
        ref, ref_psi = _reference(sv, H, n, dtype, g, b)
        got, psi = _noalloc(sv, H, n, dtype, g, b, out)
        _same(got, ref, orc.coeff_scale(inst))
        assert np.array_equal(psi, ref_psi)
        # a second evaluation of the same instance at other angles reuses the scratch
        g2, b2 = I.linear_ramp_params(p)
        ref2, _ = _reference(sv, H, n, dtype, g2, b2)
        got2, _ = _noalloc(sv, H, n, dtype, g2, b2, out)
        _same(got2, ref2, orc.coeff_scale(inst))
        H.close()


def test_noalloc_refuses_unprepared_instance_and_bad_output(sv):
    """An instance without device tables or ground-state cache for this n and
    dtype is refused (SV_ERR_UNSUPPORTED) and the output is left untouched; a
    NULL output pointer is SV_ERR_ARG."""
    import torch

    n = 16
    inst = I.degree4_int2(n, 5)
    H = sv.Ising.from_instance(inst)
    s = sv.State(n, "c128")
    out = torch.full((3,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(sv.SVError) as e:
        sv.qaoa_energy_noalloc(s, H, [0.3], [0.2], out)
    assert e.value.code == 4, e.value
    torch.cuda.synchronize()
    assert out.cpu().tolist() == [7.0, 7.0, 7.0]
    g = np.array([0.3])
    b = np.array([0.2])
    dp = ctypes.POINTER(ctypes.c_double)
    rc = sv.lib.sv_qaoa_energy_noalloc(s.handle, H.handle, 1, g.ctypes.data_as(dp), b.ctypes.data_as(dp), 1, None)
    assert rc == 1
    H.close()
