"""C-ABI checks that need no GPU: the library loads, exports every function the header
declares, validates its inputs on the host, and builds the same moment matrix as the
oracle (Sec. II rows) with an accurate block inverse."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_1411_6697_amd import lbkm as L
from paper_1411_6697_amd import workloads as W
from oracle import dvm as odvm
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:lbkm_status|const char\*)\s+(lbkm_\w+)\s*\(", text, re.M))
    return names


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert set(L.SIGNATURES) | {"lbkm_last_error"} >= names


def _grid(nx=16, ny=4, dvm=W.DVM_SOD, dx=1e-3, dt=1e-5, bcx=1, bcy=0):
    return L.Grid(nx=nx, ny=ny, dx=dx, dy=dx, dt=dt, bc_x=bcx, bc_y=bcy, dvm=L.Dvm(*dvm))


def _create(g):
    lib = L.load()
    h = ctypes.c_void_p()
    st = lib.lbkm_create(ctypes.byref(g), None, ctypes.byref(h))
    msg = lib.lbkm_last_error(h).decode() if h.value else ""
    return st, h, msg


def _destroy(h):
    if h.value:
        assert L.load().lbkm_destroy(h) == 0


@pytest.mark.parametrize("kw,status", [({"nx": 0}, -1), ({"ny": -3}, -1), ({"dx": -1.0}, -1),
                                       ({"dt": 0.0}, -1), ({"bcx": 7}, -1),
                                       ({"dvm": (2.0, 2.0, 1.2, 1.0, 1.0, 0.5)}, -2),
                                       ({"dvm": (2.0, 1.0, 1.2, -1.0, 2.0, 0.5)}, -1),
                                       ({"nx": 4730, "ny": 4730}, -1), ({"nx": 4729, "ny": 4729}, 0),
                                       ({}, 0)])
def test_create_validates_grid(kw, status):
    st, h, msg = _create(_grid(**kw))
    try:
        assert st == status, msg
        if status:
            assert msg
    finally:
        _destroy(h)


def _set_params(h, S, gamma=1.4, Pr=0.0, Q=0.0, w=(0.0, 0.0), m=1.0, n=1.0, Tig=1.1):
    lib = L.load()
    arr = (ctypes.c_double * 24)(*S)
    r = L.Rates(omega1=w[0], omega2=w[1], m=m, n=n, T_ig=Tig)
    st = lib.lbkm_set_params(h, arr, gamma, Pr, Q, ctypes.byref(r))
    return st, lib.lbkm_last_error(h).decode()


@pytest.mark.parametrize("kw,status", [
    ({}, 0), ({"gamma": 1.0}, -1), ({"gamma": 2.0}, -1), ({"gamma": float("nan")}, -1),
    ({"S": [1e5] * 23 + [0.0]}, -1), ({"S": [1e5] * 4 + [2.5e5] + [1e5] * 19}, -1),
    ({"Pr": 2.0, "S": [1e5] * 4 + [1e4, 2e4] + [1e4] * 18}, -1), ({"Pr": 2.0, "S": [1e4] * 24}, 0),
    ({"w": (-1.0, 0.0)}, -1), ({"Tig": -0.5}, -1), ({"m": -1.0}, -1), ({"Q": float("inf")}, -1)])
def test_set_params_validates(kw, status):
    st, h, msg = _create(_grid())
    assert st == 0, msg
    try:
        S = kw.pop("S", [1e5] * 24)
        st, msg = _set_params(h, S, **kw)
        assert st == status, msg
    finally:
        _destroy(h)


@pytest.mark.parametrize("tau,status", [(1e-4, 0), (0.0, 0), (-1e-4, -1), (float("nan"), -1),
                                        (float("inf"), -1), (1e-5 / 2.5, -1), (1e-5 / 1.9, 0)])
def test_set_srt_validates(tau, status):
    """Single-relaxation-time switch (Eq. SRT): tau >= 0, finite, dt / tau < 2."""
    st, h, msg = _create(_grid())
    assert st == 0, msg
    try:
        st = L.load().lbkm_set_srt(h, tau)
        assert st == status, L.load().lbkm_last_error(h).decode()
    finally:
        _destroy(h)


@pytest.mark.parametrize("order,status", [(1, 0), (2, 0), (3, 0), (0, -1), (4, -1), (-2, -1)])
def test_set_time_scheme_validates(order, status):
    """Forward Euler (1) or the SSP Runge-Kutta schemes of order 2 and 3."""
    st, h, msg = _create(_grid())
    assert st == 0, msg
    try:
        assert L.load().lbkm_set_time_scheme(h, order) == status
    finally:
        _destroy(h)


@pytest.mark.parametrize("side,typ,state,status", [
    (0, 1, None, 0), (1, 2, (1.0, 0.5, 2.0, 0.0, 0.0), 0), (0, 3, (0.0, 1.0, 0.1, 0.0, 0.0), 0), (0, 0, None, 0),
    (4, 1, None, -1), (0, 4, None, -1), (2, 1, None, -1), (0, 2, None, -1),
    (0, 2, (0.0, 0.5, 2.0, 0.0, 0.0), -1), (0, 3, (1.0, 0.0, 0.1, 0.0, 0.0), -1),
    (1, 2, (1.0, float("nan"), 2.0, 0.0, 0.0), -1)])
def test_set_boundary_validates(side, typ, state, status):
    """Wall sides (Sec. IV C-D): side 0..3, type 0..3, walls only on an outflow axis (the
    grid here is outflow in x, periodic in y), Dirichlet needs rho, T > 0, the
    extrapolation wall T > 0, all finite."""
    st, h, msg = _create(_grid())
    assert st == 0, msg
    try:
        arr = None if state is None else (ctypes.c_double * 5)(*state)
        st = L.load().lbkm_set_boundary(h, side, typ, arr)
        assert st == status, L.load().lbkm_last_error(h).decode()
    finally:
        _destroy(h)


def test_bind_buffers_rejects_a_pitch_beyond_32_bit_plane_offsets():
    """The planes of one state are addressed with 32-bit byte offsets: 24 * ny * pitch
    doubles must stay within 4 GiB.  The check comes before any device work."""
    lib = L.load()
    st, h, msg = _create(_grid())
    try:
        assert st == 0, msg
        ny = _grid().ny
        pitch = (0xFFFFFFFF // (24 * 8 * ny)) + 1
        assert lib.lbkm_bind_buffers(h, 1, 2, 3, 4, ctypes.c_int64(pitch)) == -1
        assert "4 GiB" in lib.lbkm_last_error(h).decode()
        assert lib.lbkm_bind_buffers(h, 1, 2, 3, 4, ctypes.c_int64(3)) == -1   # pitch < nx
    finally:
        _destroy(h)


def test_walls_on_a_grid_too_long_for_the_ghost_layers_are_rejected():
    """27 planes x 4 sides x 2 layers x max(nx, ny) ghost doubles must stay within 4 GiB."""
    lib = L.load()
    st, h, msg = _create(_grid(nx=2_500_000, ny=1, bcx=1, bcy=1))
    try:
        assert st == 0, msg
        assert lib.lbkm_set_boundary(h, 0, 1, None) == -1
        assert "4 GiB" in lib.lbkm_last_error(h).decode()
    finally:
        _destroy(h)


def test_calls_out_of_order_are_rejected():
    lib = L.load()
    st, h, msg = _create(_grid())
    try:
        assert lib.lbkm_step(h, 1) == -5
        assert "bound" in lib.lbkm_last_error(h).decode()
        out = (ctypes.c_double * 8)()
        assert lib.lbkm_reduce(h, out) == -5
    finally:
        _destroy(h)


@pytest.mark.parametrize("d", [W.DVM_SOD, W.DVM_STEADY_DET, W.DVM_UNSTEADY_DET, (0.8, 1.2, 1.3, 1.0, 2.7, 0.8),
                               W.DVM_LAX, W.DVM_SJOGREN])
def test_library_moment_matrix_matches_oracle(d):
    """The library's M equals the oracle's correctly rounded M entry by entry, and its
    block inverse agrees with the oracle's exactly rounded M^-1 to a few ulp of the
    largest entry."""
    st, h, msg = _create(_grid(dvm=d))
    assert st == 0, msg
    try:
        M = (ctypes.c_double * 576)()
        Mi = (ctypes.c_double * 576)()
        cond = ctypes.c_double()
        assert L.load().lbkm_get_matrices(h, M, Mi, ctypes.byref(cond)) == 0
        M = np.array(M[:]).reshape(24, 24)
        Mi = np.array(Mi[:]).reshape(24, 24)
        Mo = odvm.moment_matrix(oracle.DVM(*d))
        Mio = odvm.inverse_moment_matrix(oracle.DVM(*d))
        assert np.max(np.abs(M - Mo)) <= 2e-16 * np.abs(Mo).max()
        assert np.max(np.abs(Mi - Mio)) <= 4e-16 * np.abs(Mio).max()
        assert 1.0 < cond.value < 1e7
    finally:
        _destroy(h)


def test_gamma_maps_to_integer_internal_dof():
    """gamma = 1.4 gives I = 3 exactly (snap), so f_hat^eq uses the paper's I."""
    st, h, msg = _create(_grid())
    try:
        assert _set_params(h, [1e5] * 24, gamma=1.4)[0] == 0
        assert _set_params(h, [1e5] * 24, gamma=1.5)[0] == 0
        assert _set_params(h, [1e5] * 24, gamma=1.0 + 2.0 / 7.0)[0] == 0   # I = 5
    finally:
        _destroy(h)


def _batch_create(nx, g=None):
    lib = L.load()
    h = ctypes.c_void_p()
    arr = (ctypes.c_int32 * max(len(nx), 1))(*nx)
    st = lib.lbkm_batch_create(len(nx), arr, ctypes.byref(g or _grid()), None, ctypes.byref(h))
    msg = lib.lbkm_last_error(h).decode() if h.value else ""
    return st, h, msg


@pytest.mark.parametrize("nx,g,status", [([], None, -1), ([5, 0, 7], None, -1), ([3, -2], None, -1),
                                         ([2 ** 27, 2 ** 27], None, -1),
                                         ([10], _grid(dvm=(2.0, 2.0, 1.2, 1.0, 1.0, 0.5)), -2),
                                         ([10], _grid(dt=-1.0), -1)])
def test_batch_create_validates_on_the_host(nx, g, status):
    st, h, msg = _batch_create(nx, g)
    try:
        assert st == status, msg
        if h.value:
            assert msg
            # a batched context refuses the single-grid calls
            lib = L.load()
            assert lib.lbkm_step(h, 1) == -5
            assert lib.lbkm_bind_buffers(h, 1, 2, 3, 4, 64) == -5
    finally:
        _destroy(h)
