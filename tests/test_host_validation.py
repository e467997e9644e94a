"""Failure injection on the host side of the C ABI: every invalid or
non-finite descriptor is rejected by nlte_column_plan_bytes (the same checks
nlte_column_create runs before it touches the device) with the documented
status, and a valid one is sized.  No device is needed."""
import copy

import numpy as np
import pytest

from paper_2406_17234_amd import nlte
from paper_2406_17234_amd import synth as S


@pytest.fixture(scope="module")
def base():
    return S.chromo6(nz=24, nnu=160)


def _status(problem, precision=nlte.FP64):
    try:
        nlte.plan_bytes(problem, precision)
        return nlte.NLTE_OK
    except nlte.NLTEError as e:
        return e.status


def test_valid_problem_is_sized(base):
    b64 = nlte.plan_bytes(base, nlte.FP64)
    b32 = nlte.plan_bytes(base, nlte.FP32_FORM)
    d = base.dims
    # at least the [nz][nnu] tables and scratch of the formal solution
    assert b64 > 8 * d["nz"] * d["nnu"] * 8
    assert b32 > b64  # FP32 copies of the n-independent tables come on top


def test_optional_inputs_change_the_size(base):
    p = copy.deepcopy(base)
    p.atmos.eta_c = np.ones((p.atmos.nz, p.grid.nnu))
    assert nlte.plan_bytes(p) >= nlte.plan_bytes(base) + 8 * p.atmos.nz * p.grid.nnu
    q = copy.deepcopy(base)
    q.grid.w_nu = np.gradient(q.grid.nu)
    assert nlte.plan_bytes(q) >= nlte.plan_bytes(base)


def _set(path, fn):
    def mutate(p):
        obj = p
        parts = path.split(".")
        for a in parts[:-1]:
            obj = getattr(obj, a)
        setattr(obj, parts[-1], fn(getattr(obj, parts[-1]), p))
    return mutate


def _at(i, value):
    def f(x, p):
        x = np.array(x, dtype=np.asarray(x).dtype, copy=True)
        x.flat[i] = value
        return x
    return f


NONFINITE = {
    "T NaN": _set("atmos.T", _at(3, np.nan)),
    "ntot Inf": _set("atmos.ntot", _at(0, np.inf)),
    "z NaN": _set("atmos.z", _at(5, np.nan)),
    "ne NaN": _set("atmos.ne", _at(2, np.nan)),
    "chi_c Inf": _set("atmos.chi_c", _at(1, np.inf)),
    "chi_sca NaN": _set("atmos.chi_sca", _at(1, np.nan)),
    "nu NaN": _set("grid.nu", _at(10, np.nan)),
    "E NaN": _set("atom.E", _at(1, np.nan)),
    "C_up NaN": _set("C_up", _at(7, np.nan)),
    "eta_c NaN": lambda p: setattr(p.atmos, "eta_c", np.where(
        np.arange(p.atmos.nz * p.grid.nnu).reshape(p.atmos.nz, -1) == 9, np.nan, 1.0)),
    "w_nu Inf": lambda p: setattr(p.grid, "w_nu", np.where(np.arange(p.grid.nnu) == 4, np.inf, 1.0)),
    "vlos NaN": lambda p: setattr(p.atmos, "vlos", np.where(np.arange(p.atmos.nz) == 2, np.nan, 1e5)),
}

INVALID = {
    "ntot zero": _set("atmos.ntot", _at(4, 0.0)),
    "ntot negative": _set("atmos.ntot", _at(4, -1.0)),
    "T zero": _set("atmos.T", _at(0, 0.0)),
    "ne negative": _set("atmos.ne", _at(0, -5.0)),
    "z not increasing": _set("atmos.z", lambda z, p: np.concatenate([z[:3], z[2:3], z[4:]])),
    "nu not increasing": _set("grid.nu", lambda nu, p: nu[::-1].copy()),
    "mu zero": _set("grid.mu", _at(0, 0.0)),
    "mu one": _set("grid.mu", _at(0, 1.0)),
    "mu weights not normalised": _set("grid.w_mu", lambda w, p: 1.5 * w),
    "window outside grid": _set("grid.win_hi", _at(0, 10 ** 6)),
    "window too short": _set("grid.win_hi", lambda w, p: np.where(np.arange(len(w)) == 0,
                                                                   p.grid.win_lo[0] + 1, w)),
    "line levels reversed": _set("atom.line_up", lambda u, p: np.where(np.arange(len(u)) == 0,
                                                                       p.atom.line_lo[0], u)),
    "A_ul zero": _set("atom.A_ul", _at(0, 0.0)),
    "damping too large": _set("atom.a_damp", _at(0, 0.5)),
    "g zero": _set("atom.g", _at(2, 0.0)),
    "negative collision rate": _set("C_up", _at(3, -1.0)),
    "negative background opacity": _set("atmos.chi_c", _at(3, -1.0)),
    "negative eta_c": lambda p: setattr(p.atmos, "eta_c", -np.ones((p.atmos.nz, p.grid.nnu))),
    "zero frequency weight": lambda p: setattr(p.grid, "w_nu", np.zeros(p.grid.nnu)),
    "vlos beyond c/10": lambda p: setattr(p.atmos, "vlos", np.full(p.atmos.nz, 4e9)),
}


@pytest.mark.parametrize("name", sorted(NONFINITE))
def test_nonfinite_descriptor_rejected(base, name):
    p = copy.deepcopy(base)
    NONFINITE[name](p)
    assert _status(p) == nlte.NLTE_E_NONFINITE


@pytest.mark.parametrize("name", sorted(INVALID))
def test_invalid_descriptor_rejected(base, name):
    p = copy.deepcopy(base)
    INVALID[name](p)
    assert _status(p) == nlte.NLTE_E_INVALID


def test_structural_limits(base):
    """Sizes beyond the documented limits: fewer than 3 depths, more than 8
    angles, the depth-parallel variant beyond 256 depths, a bad precision."""
    assert _status(S.chromo6(nz=2, nnu=160)) == nlte.NLTE_E_INVALID
    assert _status(S.chromo6(nz=24, nnu=160, nmu=9)) == nlte.NLTE_E_INVALID
    big = S.chromo6(nz=300, nnu=160)
    assert _status(big) == nlte.NLTE_OK
    assert _status(big, nlte.FP32_FORM | nlte.DEPTH_SCAN) == nlte.NLTE_E_INVALID
    assert _status(base, 7) == nlte.NLTE_E_INVALID


def test_null_arguments_rejected():
    import ctypes
    L = nlte.lib()
    nb = ctypes.c_size_t()
    assert L.nlte_column_plan_bytes(None, None, None, None, 0, ctypes.byref(nb)) == nlte.NLTE_E_INVALID
    assert L.nlte_column_plan_bytes(None, None, None, None, 0, None) == nlte.NLTE_E_INVALID
    assert len(L.nlte_last_error()) > 0


def test_velocity_field_limits(base):
    """A velocity field is accepted with the sequential formal solution (FP64
    or the FP32 form) and sized with its per-ray tables; the depth-parallel
    variant rejects it."""
    p = copy.deepcopy(base)
    p.atmos.vlos = np.linspace(0.0, 3e5, p.atmos.nz)
    assert nlte.plan_bytes(p) > nlte.plan_bytes(base) + 2 * p.grid.nmu * p.atmos.nz * p.grid.nnu * 8
    assert _status(p, nlte.FP32_FORM) == nlte.NLTE_OK
    assert _status(p, nlte.FP64 | nlte.DEPTH_SCAN) == nlte.NLTE_E_INVALID
    assert _status(p, nlte.FP32_FORM | nlte.DEPTH_SCAN) == nlte.NLTE_E_INVALID
