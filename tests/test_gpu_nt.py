"""Parity of the non-temporal kernel instantiations (the path the library takes
when one step's arrays exceed the 256 MiB Infinity Cache: streamed arrays carry
non-temporal hints and the xy-halo is loaded when its plane is staged instead of
through the halo ring), forced on small grids with WAVE_PATH_STREAM.

FP32 storage, every space order 2..24: traces and final field against the FP64
oracle, rel-L2 <= 1e-5 and element-wise |err| <= 1e-4 max|ref|. Each 16-bit form:
bitwise equal to the same solve on the cached path (the hints and the halo's load
point change where values come from, never the values), and its error against the
oracle stated, with the bounds of the storage formats (FP16 difference form <= 1e-2;
BF16 difference form <= 5e-2; the naive forms only finite: their error is stated).
"""
import numpy as np
import pytest

from helpers import ragged_case, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-5
SOS = [2, 4, 6, 8, 10, 12, 14, 16, 18, 20, 22, 24]


def _run(case, storage=0, path=0):
    import torch
    from paper_1912_00695_amd import wave
    dev = torch.device("cuda:0")
    t = lambda a: None if a is None else torch.from_numpy(
        np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    out = wave.forward(case.wgrid(storage=storage, path=path), t(case.vel), t(case.wavelet),
                       case.src, case.rec, u0=t(case.u0), um1=t(case.um1), want_final=True)
    torch.cuda.synchronize()
    return out["rec"].cpu().numpy(), out["u_final"].cpu().numpy()


def _oracle(case):
    for k in ("u0", "um1"):
        setattr(case, k, np.asarray(getattr(case, k), dtype=np.float32))
    return case.oracle_forward()


def max_rel(x, ref):
    return float(np.abs(np.asarray(x, np.float64) - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("so", SOS)
def test_stream_path_fp32_matches_oracle(so):
    from paper_1912_00695_amd import wave
    case = ragged_case(so, nt=50, seed=90 + so)
    print("stream path FP32 ragged SO", so, flush=True)
    orec, ouf, _ = _oracle(case)
    rec, uf = _run(case, path=wave.PATH_STREAM | wave.PATH_ONE_STEP)
    e = (rel_l2(uf, ouf), rel_l2(rec, orec), max_rel(uf, ouf), max_rel(rec, orec))
    print("  field %.3e traces %.3e | max field %.3e max traces %.3e" % e, flush=True)
    assert e[0] <= TOL and e[1] <= TOL and e[2] <= 1e-4 and e[3] <= 1e-4
    rc, uc = _run(case, path=wave.PATH_CACHED | wave.PATH_ONE_STEP)
    assert np.array_equal(rc, rec) and np.array_equal(uc, uf)
    if so in (2, 4, 6, 8, 16, 20):  # the 64 x 32 workgroup tiles of these orders: same bits
        rt, ut = _run(case, path=wave.PATH_STREAM | wave.PATH_ONE_STEP | wave.PATH_TILE32)
        assert np.array_equal(rt, rec) and np.array_equal(ut, uf)


FORMS = {"f16": 1, "bf16": 2, "f16_diff": 17, "bf16_diff": 18}
BOUND = {"f16_diff": 1e-2, "bf16_diff": 5e-2}


@pytest.mark.parametrize("so", SOS)
@pytest.mark.parametrize("form", sorted(FORMS))
def test_stream_path_16bit(form, so):
    from paper_1912_00695_amd import wave
    case = ragged_case(so, nt=50, seed=110 + so)
    print("stream path", form, "ragged SO", so, flush=True)
    rs, us = _run(case, FORMS[form], wave.PATH_STREAM)
    rc, uc = _run(case, FORMS[form], wave.PATH_CACHED)
    assert np.isfinite(us).all() and np.isfinite(rs).all()
    assert np.array_equal(rs, rc) and np.array_equal(us, uc)
    orec, ouf, _ = _oracle(case)
    eu, er = rel_l2(us, ouf), rel_l2(rs, orec)
    print("  vs oracle: field %.3e traces %.3e" % (eu, er), flush=True)
    if form in BOUND:
        assert eu <= BOUND[form] and er <= BOUND[form]
