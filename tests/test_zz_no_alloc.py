"""wave_forward_noalloc (the library's static device array as workspace) against
wave_forward on the one-step path: two calls in a row on one device, the second on
a smaller grid (the array keeps the first call's contents), each bitwise equal to
wave_forward of the same problem; the second pair is also checked against the FP64
oracle. Also a storage format with the bookkeeping region (FP16 difference form)."""
import numpy as np
import pytest

from helpers import Case, ragged_case, rel_l2
from paper_1912_00695_amd import inputs

pytestmark = pytest.mark.gpu


def _pair(case, storage=0):
    import torch
    from paper_1912_00695_amd import wave
    dev = torch.device("cuda:0")
    t = lambda a: None if a is None else torch.from_numpy(
        np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    args = (t(case.vel), t(case.wavelet), case.src, case.rec)
    kw = dict(u0=t(case.u0), um1=t(case.um1), want_final=True)
    a = wave.forward_noalloc(case.wgrid(storage=storage), *args, **kw)
    b = wave.forward(case.wgrid(storage=storage, path=wave.PATH_ONE_STEP), *args, **kw)
    torch.cuda.synchronize()
    return ((a["rec"].cpu().numpy(), a["u_final"].cpu().numpy()),
            (b["rec"].cpu().numpy(), b["u_final"].cpu().numpy()))


def _small_case():
    n, h = (70, 21, 13), (10.0, 11.0, 9.0)
    vel = inputs.smooth_random_range(n, 1500.0, 2500.0, 5.0, seed=201)
    c = Case(n, h, 4, 37, vel, 2500.0, nbl=(3, 4, 2, 2, 1, 3))
    c.src = inputs.random_points(n, h, 2, 202, margin=1.0)
    c.wavelet = np.random.default_rng(203).standard_normal((c.nt, 2)).astype(np.float32)
    c.rec = inputs.random_points(n, h, 17, 204)
    c.u0 = inputs.random_field(vel.shape, 205) * 1e-2
    c.um1 = inputs.random_field(vel.shape, 206) * 1e-2
    return c


def test_noalloc_matches_forward_twice_in_a_row():
    first = ragged_case(8, nt=40, seed=200)
    second = _small_case()
    for k, case in enumerate((first, second)):
        print("noalloc call", k, case.n, "SO", case.so, flush=True)
        (ra, ua), (rb, ub) = _pair(case)
        assert np.abs(ua).max() > 0
        assert np.array_equal(ra, rb) and np.array_equal(ua, ub)
    for kk in ("u0", "um1"):
        setattr(second, kk, np.asarray(getattr(second, kk), dtype=np.float32))
    orec, ouf, _ = second.oracle_forward()
    e = (rel_l2(ua, ouf), rel_l2(ra, orec))
    print("second call vs oracle: field %.3e traces %.3e" % e, flush=True)
    assert e[0] <= 1e-5 and e[1] <= 1e-5


def test_noalloc_reduced_storage_and_limit():
    from paper_1912_00695_amd import wave
    case = ragged_case(4, nt=30, seed=210)
    print("noalloc FP16 difference form", flush=True)
    (ra, ua), (rb, ub) = _pair(case, storage=wave.STORE_F16 | wave.STORE_DIFF)
    assert np.array_equal(ra, rb) and np.array_equal(ua, ub)
    big = wave.make_grid((256, 256, 256), (10.0,) * 3, 8, 1e-4, 2, vmax=3000.0)
    import torch
    vel = torch.full((256, 256, 256), 1500.0, device="cuda:0")
    with pytest.raises(wave.WaveError) as ei:
        wave.forward_noalloc(big, vel)
    assert ei.value.status == wave.ELIMIT
