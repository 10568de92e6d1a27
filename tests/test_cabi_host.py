"""Host-side contract of the C ABI (no GPU needed): the library loads, exports every
function include/wave.h declares, and rejects bad arguments before touching the
device."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1912_00695_amd import wave

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "wave.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wave_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = wave.lib()
    names = _declared()
    assert "wave_forward" in names and "wave_gradient" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(wave.SYMBOLS) <= set(names)


def test_status_strings():
    L = wave.lib()
    for s in (0, -1, -2, -3, -4, -5, -6, -7):
        assert L.wave_status_string(s)
    assert L.wave_version().startswith(b"wave")


@pytest.mark.parametrize("so", [2, 4, 8, 12, 16, 20, 24])
@pytest.mark.parametrize("h", [(10.0, 10.0, 10.0), (5.0, 12.0, 7.0)])
def test_cfl_matches_oracle(so, h):
    # independent implementations: closed form in the library, Fornberg in the oracle
    assert wave.cfl_dt_max(so, 3000.0, h) == pytest.approx(oracle.cfl_dt_max(so, 3000.0, h),
                                                           rel=1e-13)


def test_cfl_rejects_bad_args():
    for so in (0, 1, 3, 26):
        assert wave.cfl_dt_max(so, 1500.0, (10.0,) * 3) < 0
    assert wave.cfl_dt_max(4, 0.0, (10.0,) * 3) < 0


def _grid(**kw):
    d = dict(n=(32, 32, 32), h=(10.0,) * 3, so=8, nt=10, nbl=(0,) * 6, vmax=2000.0)
    d.update(kw)
    dt = d.pop("dt", 0.5 * wave.cfl_dt_max(d["so"], d["vmax"], d["h"]))
    return wave.make_grid(d["n"], d["h"], d["so"], dt, d["nt"], d["nbl"], d["vmax"],
                          d.get("storage", 0), d.get("path", 0), d.get("zchunk", 0))


def test_workspace_bytes():
    g = _grid()
    f = wave.workspace_bytes(g, 1, 10, wave.MODE_FORWARD)
    assert f >= 3 * 32 * 32 * 32 * 4
    gr = wave.workspace_bytes(g, 1, 10, wave.MODE_GRADIENT, 5)
    assert gr > f
    assert wave.workspace_bytes(_grid(so=5), 1, 1) == 0
    assert wave.workspace_bytes(g, -1, 1) == 0
    assert wave.checkpoint_bytes(g, 4) == 3 * 2 * 32 ** 3 * 4
    assert wave.checkpoint_bytes(g, 0) == 0


FAKE = ctypes.c_void_p(0x100000)  # never dereferenced: every call below fails validation


def _fwd(g, **kw):
    a = dict(vel=FAKE, wav=FAKE, src=None, ns=0, rec=None, nr=0, out=FAKE, ws=FAKE,
             wsb=1 << 40)
    a.update(kw)
    return wave.lib().wave_forward(ctypes.byref(g), a["vel"], a["wav"], a["src"], a["ns"],
                                   a["rec"], a["nr"], a["out"], None, None, None, None, 0,
                                   a["ws"], a["wsb"], None)


def test_forward_rejects_before_enqueue():
    g = _grid()
    assert _fwd(_grid(so=7)) == wave.EINVAL
    assert _fwd(_grid(so=26)) == wave.EINVAL
    assert _fwd(_grid(n=(0, 4, 4))) == wave.EINVAL
    assert _fwd(_grid(nbl=(20, 20, 0, 0, 0, 0))) == wave.EINVAL
    assert _fwd(_grid(storage=7)) == wave.EINVAL
    assert _fwd(_grid(storage=wave.STORE_DIFF)) == wave.EINVAL  # FP32 has no difference form
    dtm = wave.cfl_dt_max(8, 2000.0, (10.0,) * 3)
    assert _fwd(_grid(dt=1.01 * dtm)) == wave.ECFL
    assert _fwd(g, vel=None) == wave.EINVAL
    pts = np.array([[10.0, 10.0, 10.0]])
    off = np.array([[10.0, 10.0, 311.0]])  # beyond (nz-1) h
    p = pts.ctypes.data_as(ctypes.c_void_p)
    assert _fwd(g, src=off.ctypes.data_as(ctypes.c_void_p), ns=1) == wave.EINVAL
    assert _fwd(g, src=p, ns=1, wav=None) == wave.EINVAL
    assert _fwd(g, rec=p, nr=1, out=None) == wave.EINVAL
    assert _fwd(g, ws=ctypes.c_void_p(0x100004)) == wave.EINVAL  # misaligned workspace
    need = wave.workspace_bytes(g, 0, 0)
    assert _fwd(g, wsb=need - 1) == wave.ENOMEM


def test_reduced_storage_workspace_and_limits():
    f32 = wave.workspace_bytes(_grid(n=(64, 64, 64)), 1, 1)
    f16 = wave.workspace_bytes(_grid(n=(64, 64, 64), storage=wave.STORE_F16), 1, 1)
    f16d = wave.workspace_bytes(_grid(n=(64, 64, 64), storage=wave.STORE_F16 | wave.STORE_DIFF),
                                1, 1)
    # FP32 at radius <= 4 holds c2 and four levels (the two-step kernel's buffers);
    # 16-bit storage holds c2 and two (naive) or three (difference form) 2-byte arrays
    assert f16 < f16d < f32 and f32 >= 5 * 64 ** 3 * 4 and f16d < 64 ** 3 * (4 + 3 * 2) * 1.1
    f32_so16 = wave.workspace_bytes(_grid(n=(64, 64, 64), so=16), 1, 1)
    assert 3 * 64 ** 3 * 4 <= f32_so16 < 4 * 64 ** 3 * 4
    L = wave.lib()
    for st in (wave.STORE_F16, wave.STORE_BF16 | wave.STORE_DIFF):
        g = _grid(storage=st)
        # checkpoints, adjoint and gradient are FP32-storage only
        assert L.wave_forward(ctypes.byref(g), FAKE, None, None, 0, None, 0, None, None, None,
                              None, FAKE, 4, FAKE, 1 << 40, None) == wave.EINVAL
        assert L.wave_adjoint(ctypes.byref(g), FAKE, FAKE, None, 0, None, 0, FAKE, None, FAKE,
                              1 << 40, None) == wave.EINVAL
        assert L.wave_gradient(ctypes.byref(g), FAKE, FAKE, None, 0, None, 0, FAKE, None, 0,
                               FAKE, None, FAKE, 1 << 40, None) == wave.EINVAL


def test_adjoint_and_gradient_reject_before_enqueue():
    g = _grid()
    L = wave.lib()
    assert L.wave_adjoint(ctypes.byref(_grid(so=3)), FAKE, FAKE, None, 0, None, 0, FAKE, None,
                          FAKE, 1 << 40, None) == wave.EINVAL
    assert L.wave_adjoint(ctypes.byref(g), FAKE, FAKE, None, 0, None, 0, FAKE, None, FAKE, 16,
                          None) == wave.ENOMEM
    assert L.wave_gradient(ctypes.byref(g), FAKE, FAKE, None, 0, None, 0, FAKE, None, 0, None,
                           None, FAKE, 1 << 40, None) == wave.EINVAL  # no grad_vel
    assert L.wave_gradient(ctypes.byref(g), FAKE, FAKE, None, 0, None, 0, FAKE, FAKE, 0, FAKE,
                           None, FAKE, 1 << 40, None) == wave.EINVAL  # ckpt without interval


def test_path_flags_validated():
    """Execution-path flags and the z-chunk length are arguments (no environment
    variable changes a call): contradictory or unknown flags and chunk lengths out
    of 0..256 are rejected before anything is enqueued."""
    for bad in (wave.PATH_ONE_STEP | wave.PATH_TWO_STEP, wave.PATH_STREAM | wave.PATH_CACHED,
                wave.PATH_GRAPH | wave.PATH_DIRECT, wave.PATH_TILE16 | wave.PATH_TILE32, 512, -1):
        assert _fwd(_grid(path=bad)) == wave.EINVAL, bad
    for zc in (-1, 257):
        assert _fwd(_grid(zchunk=zc)) == wave.EINVAL, zc
    assert wave.workspace_bytes(_grid(zchunk=300), 0, 0) == 0
    # valid flags pass validation (the call then fails on the workspace size)
    for ok in (wave.PATH_ONE_STEP, wave.PATH_TWO_STEP | wave.PATH_STREAM | wave.PATH_LINEAR,
               wave.PATH_CACHED | wave.PATH_GRAPH, wave.PATH_DIRECT, wave.PATH_TILE16,
               wave.PATH_TILE32 | wave.PATH_ONE_STEP):
        g = _grid(path=ok, zchunk=7)
        assert _fwd(g, wsb=wave.workspace_bytes(g, 0, 0) - 1) == wave.ENOMEM


def test_unfactorised_rejects_other_orders_and_storage():
    L = wave.lib()
    for kw in (dict(so=4), dict(so=10), dict(storage=wave.STORE_F16)):
        g = _grid(**kw)
        assert L.wave_forward_unfactorised(ctypes.byref(g), FAKE, None, None, 0, None, 0, None,
                                           None, None, None, FAKE, 1 << 40, None) == wave.EINVAL


def test_no_environment_reads_in_the_library():
    """The library's sources read no environment variable (execution choices are
    call arguments)."""
    import glob
    for f in glob.glob(os.path.join(ROOT, "paper_1912_00695_amd", "csrc", "*")):
        assert "getenv" not in open(f).read(), f


def test_noalloc_limit_checked_before_any_device_call():
    """wave_forward_noalloc rejects a problem whose one-step layout exceeds its static
    device array (WAVE_ELIMIT) during validation, before any HIP call: this runs
    without a GPU."""
    L = wave.lib()
    assert L.wave_noalloc_limit_bytes() == 64 << 20
    big = _grid(n=(256, 256, 256))
    assert L.wave_forward_noalloc(ctypes.byref(big), FAKE, None, None, 0, None, 0, None, None,
                                  None, None, None) == wave.ELIMIT
    assert L.wave_forward_noalloc(ctypes.byref(_grid(so=7)), FAKE, None, None, 0, None, 0, None,
                                  None, None, None, None) == wave.EINVAL
    two = _grid(path=wave.PATH_TWO_STEP)
    assert L.wave_forward_noalloc(ctypes.byref(two), FAKE, None, None, 0, None, 0, None, None,
                                  None, None, None) == wave.EINVAL
