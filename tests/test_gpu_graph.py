"""Graph replay of the time loop. A call's launches are recorded; a call whose
launches equal an earlier call's (same arguments, same buffers) is captured into a
HIP graph and replayed from the library's cache (WAVE_PATH_GRAPH: from the first
call; WAVE_PATH_DIRECT: never). A replay runs the same kernels with the same
arguments, so every result is bitwise that of direct launches. Each replay below
is preceded by eager torch work and a synchronisation, and checked on its own."""
import numpy as np
import pytest

from helpers import ragged_case, rel_l2

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return None if a is None else torch.from_numpy(
        np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def _eager_noise():
    import torch
    x = torch.randn(1 << 20, device="cuda:0")
    (x * 2.0 + 1.0).sum().item()
    torch.cuda.synchronize()


@pytest.mark.parametrize("form", ["f32", "f16_diff", "two_step", "ckpt"])
def test_forward_replays_are_bitwise_direct(form):
    import torch
    from paper_1912_00695_amd import wave
    case = ragged_case(4 if form == "two_step" else 8, nt=40, seed=300)
    storage = 17 if form == "f16_diff" else 0
    extra = wave.PATH_TWO_STEP if form == "two_step" else 0
    zc = 8 if form == "two_step" else 0
    ck = 7 if form == "ckpt" else 0
    vel, wav, u0, um1 = _dev(case.vel), _dev(case.wavelet), _dev(case.u0), _dev(case.um1)
    print("graph replay forward", form, flush=True)

    def run(path, bufs=None):
        g = case.wgrid(storage=storage, path=path | extra, zchunk=zc)
        kw = dict(u0=u0, um1=um1, want_final=True, ckpt_every=ck)
        if bufs is not None:
            kw.update(workspace=bufs[0], rec_out=bufs[1], u_final=bufs[2])
        o = wave.forward(g, vel, wav, case.src, case.rec, **kw)
        torch.cuda.synchronize()
        return o["rec"].cpu().numpy(), o["u_final"].cpu().numpy(), \
            (o["ckpt"].cpu().numpy() if o["ckpt"] is not None else None)

    ref = run(wave.PATH_DIRECT)
    g0 = case.wgrid(storage=storage, path=extra, zchunk=zc)
    bufs = (torch.empty(wave.workspace_bytes(g0, len(case.src), len(case.rec)),
                        dtype=torch.uint8, device="cuda:0"),
            torch.empty((case.nt, len(case.rec)), dtype=torch.float32, device="cuda:0"),
            torch.empty(tuple(reversed(case.n)), dtype=torch.float32, device="cuda:0"))
    # default policy on fixed buffers: direct, captured, replayed, replayed
    for k in range(4):
        _eager_noise()
        got = run(0, bufs)
        for a, b in zip(got, ref):
            assert (a is None and b is None) or np.array_equal(a, b), (form, k)
    # capture at the first call, fresh output buffers each time
    for k in range(2):
        _eager_noise()
        got = run(wave.PATH_GRAPH)
        for a, b in zip(got, ref):
            assert (a is None and b is None) or np.array_equal(a, b), (form, "graph", k)
    if form == "f32":
        for kk in ("u0", "um1"):
            setattr(case, kk, np.asarray(getattr(case, kk), dtype=np.float32))
        orec, ouf, _ = case.oracle_forward()
        assert rel_l2(ref[1], ouf) <= 1e-5 and rel_l2(ref[0], orec) <= 1e-5


def test_adjoint_gradient_rtm_replays_are_bitwise_direct():
    import torch
    from paper_1912_00695_amd import wave
    case = ragged_case(8, nt=30, seed=310)
    vel, wav = _dev(case.vel), _dev(case.wavelet)
    d = _dev(np.random.default_rng(311).standard_normal((case.nt, len(case.rec))))
    print("graph replay adjoint / gradient / rtm", flush=True)

    def all_three(path):
        g = case.wgrid(path=path)
        a = wave.adjoint(g, vel, d, case.rec, case.src, want_final=True)
        gr = wave.gradient(g, vel, wav, case.src, case.rec, d, ckpt_every=7)
        im = wave.rtm(g, vel, wav, case.src, case.rec, d, ckpt_every=7)
        torch.cuda.synchronize()
        return [a["src"].cpu().numpy(), a["lam_final"].cpu().numpy(),
                gr["grad_vel"].cpu().numpy(), gr["grad_wavelet"].cpu().numpy(), im.cpu().numpy()]

    ref = all_three(wave.PATH_DIRECT)
    assert np.abs(ref[2]).max() > 0
    for k in range(3):
        _eager_noise()
        got = all_three(wave.PATH_GRAPH)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), k
