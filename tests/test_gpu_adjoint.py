"""GPU adjoint and gradient (through the C ABI) against the FP64 oracle, the
dot-product test and finite differences.

Tolerances: adjoint traces and final level rel-L2 <= 1e-5 (FP32 vs FP64);
dot test <= 1e-5 (FP32 solves, FP64 inner products); gradient rel-L2 <= 1e-4
against the oracle's gradient (a sum over every time step of products of two
FP32 fields); finite differences <= 1e-2.
"""
import numpy as np
import pytest

import oracle
from helpers import ragged_case, rel_l2
from paper_1912_00695_amd import inputs

pytestmark = pytest.mark.gpu
TALL = (2, 4, 6, 8, 16, 20)  # orders with 64 x 32 workgroup tiles (WAVE_PATH_TILE32)


def _dev():
    import torch
    return torch.device("cuda:0")


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(_dev())


@pytest.mark.parametrize("so", [2, 4, 8, 16])
def test_adjoint_matches_oracle(so):
    from paper_1912_00695_amd import wave
    case = ragged_case(so, nt=45, seed=3)
    rng = np.random.default_rng(so)
    d = rng.standard_normal((case.nt, len(case.rec))).astype(np.float32)
    print("adjoint ragged SO", so, flush=True)
    out = wave.adjoint(case.wgrid(), _t(case.vel), _t(d), case.rec, case.src, want_final=True)
    src_o, lam_o = oracle.adjoint(case.ogrid(), case.vel, d, case.rec, case.src)
    e_s = rel_l2(out["src"].cpu().numpy(), src_o)
    e_l = rel_l2(out["lam_final"].cpu().numpy(), lam_o)
    print("SO", so, "src", e_s, "lambda0", e_l, flush=True)
    assert e_s <= 1e-5 and e_l <= 1e-5
    if so in TALL:  # 64 x 32 workgroup tiles (the default on large grids): same bits
        o2 = wave.adjoint(case.wgrid(path=wave.PATH_TILE32), _t(case.vel), _t(d), case.rec,
                          case.src, want_final=True)
        assert np.array_equal(o2["src"].cpu().numpy(), out["src"].cpu().numpy())
        assert np.array_equal(o2["lam_final"].cpu().numpy(), out["lam_final"].cpu().numpy())


def _dot(case, seed):
    from paper_1912_00695_amd import wave
    rng = np.random.default_rng(seed)
    s = rng.standard_normal((case.nt, len(case.src))).astype(np.float32)
    d = rng.standard_normal((case.nt, len(case.rec))).astype(np.float32)
    g = case.wgrid()
    Fs = wave.forward(g, _t(case.vel), _t(s), case.src, case.rec)["rec"].cpu().numpy()
    Ftd = wave.adjoint(g, _t(case.vel), _t(d), case.rec, case.src)["src"].cpu().numpy()
    a = np.vdot(Fs.astype(np.float64), d.astype(np.float64))
    b = np.vdot(s.astype(np.float64), Ftd.astype(np.float64))
    return a, b


@pytest.mark.parametrize("so", [4, 8, 16])
def test_dot_product_ragged(so):
    case = ragged_case(so, nt=60, seed=5)
    a, b = _dot(case, 7)
    print("dot SO", so, a, b, abs(a - b) / abs(a), flush=True)
    assert abs(a - b) <= 1e-5 * max(abs(a), abs(b))


def _c3(nt=800, n=(256, 256, 256), true_model=False):
    """256^3 SO8: two-layer background (or the perturbed true model), 10 Hz Ricker
    at (128,128,20), receivers on the whole plane z = 20, dt = 0.5 dt_max at the
    true model's maximum velocity, 40-cell sponge."""
    from helpers import Case
    h = (10.0, 10.0, 10.0)
    vtrue = inputs.perturbed_two_layer(n, 0.05, 20.0, seed=1)
    vmax = float(vtrue.max())
    vel = vtrue if true_model else inputs.two_layer(n, 1500.0, 3000.0, n[2] // 2)
    c = Case(n, h, 8, nt, vel, vmax, nbl=(40,) * 6)
    c.src = inputs.point((n[0] // 2, n[1] // 2, 20), h)
    c.wavelet = inputs.ricker(10.0, c.dt, nt)[:, None]
    c.rec = inputs.plane_z(n, h, 20)
    return c


def test_dot_product_full_size():
    """Full C3 geometry: 256^3, 800 steps, 65,536 receivers on a plane; seeded
    random s and d (seeds 2, 3)."""
    case = _c3()
    from paper_1912_00695_amd import wave
    rng_s, rng_d = np.random.default_rng(2), np.random.default_rng(3)
    s = rng_s.standard_normal((case.nt, 1)).astype(np.float32)
    d = rng_d.standard_normal((case.nt, len(case.rec))).astype(np.float32)
    g = case.wgrid()
    print("dot C3 full", flush=True)
    Fs = wave.forward(g, _t(case.vel), _t(s), case.src, case.rec)["rec"].cpu().numpy()
    Ftd = wave.adjoint(g, _t(case.vel), _t(d), case.rec, case.src)["src"].cpu().numpy()
    a = np.vdot(Fs.astype(np.float64), d.astype(np.float64))
    b = np.vdot(s.astype(np.float64), Ftd.astype(np.float64))
    print("dot C3", a, b, abs(a - b) / abs(a), flush=True)
    assert abs(a - b) <= 1e-5 * max(abs(a), abs(b))


@pytest.mark.parametrize("so,ckpt", [(4, 0), (8, 7), (16, 50)])
def test_gradient_matches_oracle(so, ckpt):
    from paper_1912_00695_amd import wave
    case = ragged_case(so, nt=40, seed=11)
    case.u0 = case.um1 = None
    vtrue = case.vel * (1.0 + 0.03 * inputs.smooth_random(case.n, 5.0, seed=12)).astype(np.float32)
    vtrue = np.minimum(vtrue, case.vmax).astype(np.float32)
    obs, _, _ = oracle.forward(case.ogrid(), vtrue, case.wavelet, case.src, case.rec)
    syn, _, _ = oracle.forward(case.ogrid(), case.vel, case.wavelet, case.src, case.rec)
    resid = (syn - obs).astype(np.float32)
    gm_o, gv_o, gw_o = oracle.gradient(case.ogrid(), case.vel, case.wavelet, case.src, case.rec,
                                       resid, ckpt_every=ckpt)
    g = case.wgrid()
    print("gradient ragged SO", so, "ckpt", ckpt, flush=True)
    ck = None
    if ckpt:
        ck = wave.forward(g, _t(case.vel), _t(case.wavelet), case.src, case.rec,
                          ckpt_every=ckpt)["ckpt"]
    out = wave.gradient(g, _t(case.vel), _t(case.wavelet), case.src, case.rec, _t(resid),
                        ckpt=ck, ckpt_every=ckpt)
    e_v = rel_l2(out["grad_vel"].cpu().numpy(), gv_o)
    e_w = rel_l2(out["grad_wavelet"].cpu().numpy(), gw_o)
    print("SO", so, "grad_vel", e_v, "grad_wavelet", e_w, flush=True)
    assert e_v <= 1e-4 and e_w <= 1e-4
    # the internal-forward path (ckpt=None) gives the same bits as the checkpoint path
    if ckpt:
        out2 = wave.gradient(g, _t(case.vel), _t(case.wavelet), case.src, case.rec, _t(resid),
                             ckpt=None, ckpt_every=ckpt)
        assert np.array_equal(out2["grad_vel"].cpu().numpy(), out["grad_vel"].cpu().numpy())
    if so in TALL:  # 64 x 32 workgroup tiles: same bits
        out3 = wave.gradient(case.wgrid(path=wave.PATH_TILE32), _t(case.vel), _t(case.wavelet),
                             case.src, case.rec, _t(resid), ckpt=ck, ckpt_every=ckpt)
        assert np.array_equal(out3["grad_vel"].cpu().numpy(), out["grad_vel"].cpu().numpy())
        assert np.array_equal(out3["grad_wavelet"].cpu().numpy(),
                              out["grad_wavelet"].cpu().numpy())


def test_gradient_finite_differences_c3():
    """C3: 256^3 SO8, 800 steps, 65,536 receivers, checkpoints every 50 steps, through
    the torch.autograd.Function. Central differences of J = 0.5||d - d_obs||^2 on
    five seeded smooth directions (seeds 10-14), |e dv| / |v| ~ 1e-3."""
    import torch
    from paper_1912_00695_amd import autograd, wave
    case = _c3()
    true = _c3(true_model=True)
    g = case.wgrid()
    dev = _dev()
    wav = _t(case.wavelet)
    obs = wave.forward(g, _t(true.vel), wav, case.src, case.rec)["rec"]
    v = _t(case.vel).requires_grad_(True)
    print("C3 gradient via autograd", flush=True)
    J = autograd.fwi_misfit(v, wav, g, case.src, case.rec, obs, ckpt_every=50)
    J.backward()
    grad = v.grad.detach().double()
    assert torch.isfinite(grad).all()

    def J_of(vel):
        d = wave.forward(g, vel, wav, case.src, case.rec)["rec"].double()
        return float(0.5 * torch.sum((d - obs.double()) ** 2))

    v0 = _t(case.vel)
    for seed in range(10, 15):
        p = torch.from_numpy(inputs.smooth_random(case.n, 20.0, seed=seed)).to(dev)
        dv = (p * v0.double() * 1e-3).float()
        if float((v0 + dv).max()) > case.vmax:
            dv = -dv.abs()
        fd = (J_of(v0 + dv) - J_of(v0 - dv)) / 2.0
        an = float(torch.sum(grad * dv.double()))
        print("direction", seed, "fd", fd, "adjoint", an, "rel", abs(fd - an) / abs(fd),
              flush=True)
        assert abs(fd - an) <= 1e-2 * abs(fd)


@pytest.mark.parametrize("so,ckpt", [(4, 0), (8, 9)])
def test_rtm_image_matches_oracle(so, ckpt):
    from paper_1912_00695_amd import wave
    case = ragged_case(so, nt=40, seed=17)
    rng = np.random.default_rng(so + 100)
    d = rng.standard_normal((case.nt, len(case.rec))).astype(np.float32)
    want = oracle.rtm_image(case.ogrid(), case.vel, case.wavelet, case.src, case.rec, d,
                            ckpt_every=ckpt)
    g = case.wgrid()
    ck = None
    if ckpt:
        ck = wave.forward(g, _t(case.vel), _t(case.wavelet), case.src, case.rec,
                          ckpt_every=ckpt)["ckpt"]
    img = wave.rtm(g, _t(case.vel), _t(case.wavelet), case.src, case.rec, _t(d), ckpt=ck,
                   ckpt_every=ckpt).cpu().numpy()
    e = rel_l2(img, want)
    print("rtm SO", so, "ckpt", ckpt, "rel-L2", e, flush=True)
    assert np.abs(want).max() > 0 and e <= 1e-4
