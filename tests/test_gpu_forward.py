"""GPU parity of the forward solve against the FP64 oracle (through the C ABI).

Tolerance: relative L2 <= 1e-5 for final wavefields and for traces, FP32
arithmetic against FP64, both on the same seeded inputs.
"""
import numpy as np
import pytest

from helpers import c1_case, c2_case, ragged_case, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _run(case, want_final=True, ckpt_every=0, path=0, zchunk=0):
    import torch
    from paper_1912_00695_amd import wave
    dev = torch.device("cuda:0")
    vel = torch.from_numpy(case.vel).to(dev)
    wav = torch.from_numpy(np.ascontiguousarray(case.wavelet, dtype=np.float32)).to(dev) \
        if case.wavelet is not None and len(case.src) else None
    u0 = torch.from_numpy(np.ascontiguousarray(case.u0, dtype=np.float32)).to(dev) \
        if case.u0 is not None else None
    um1 = torch.from_numpy(np.ascontiguousarray(case.um1, dtype=np.float32)).to(dev) \
        if case.um1 is not None else None
    out = wave.forward(case.wgrid(path=path, zchunk=zchunk), vel, wav, case.src, case.rec,
                       u0=u0, um1=um1, want_final=want_final, ckpt_every=ckpt_every)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    return res


def _oracle_inputs(case):
    # the GPU receives FP32 levels; give the oracle exactly the same values
    for k in ("u0", "um1"):
        v = getattr(case, k)
        if v is not None:
            setattr(case, k, np.asarray(v, dtype=np.float32))


def test_c1_plain_forward():
    case = c1_case()
    _oracle_inputs(case)
    print("case C1 64^3 SO4 nt=100", flush=True)
    g = _run(case)
    _, uf, _ = case.oracle_forward()
    err = rel_l2(g["u_final"], uf)
    print("C1 rel-L2", err)
    assert err <= TOL


@pytest.mark.parametrize("so", [2, 4, 6, 8, 10, 12, 14, 16, 18, 20, 22, 24])
def test_ragged_multitile(so):
    case = ragged_case(so)
    _oracle_inputs(case)
    print("case ragged", case.n, "SO", so, flush=True)
    g = _run(case)
    rec, uf, _ = case.oracle_forward()
    e_u, e_r = rel_l2(g["u_final"], uf), rel_l2(g["rec"], rec)
    print("SO", so, "field", e_u, "traces", e_r)
    assert e_u <= TOL and e_r <= TOL
    assert max_rel(g["u_final"], uf) <= 1e-4 and max_rel(g["rec"], rec) <= 1e-4
    if so in (2, 4, 6, 8, 16, 20):  # 64 x 32 workgroup tiles (two tiles along y, the last half
        from paper_1912_00695_amd import wave  # empty): the same bits as 64 x 16
        t = _run(case, path=wave.PATH_TILE32)
        assert np.array_equal(t["u_final"], g["u_final"]) and np.array_equal(t["rec"], g["rec"])


@pytest.mark.parametrize("so", [2, 4, 8, 12, 16, 24])
def test_c2_reduced_grid(so):
    case = c2_case(so, nt=120, n=(96, 80, 72))
    print("case C2-reduced", case.n, "SO", so, flush=True)
    g = _run(case)
    rec, uf, _ = case.oracle_forward()
    e_u, e_r = rel_l2(g["u_final"], uf), rel_l2(g["rec"], rec)
    print("SO", so, "field", e_u, "traces", e_r)
    assert e_u <= TOL and e_r <= TOL


def test_c2_full_size_so8_short():
    """Full 256^3 grid in the benchmark's launch configuration, 40 steps (the oracle
    finishes in seconds)."""
    from paper_1912_00695_amd import inputs
    case = c2_case(8, nt=40)
    case.wavelet = inputs.ricker(40.0, case.dt, case.nt)[:, None]  # peaks within 40 steps
    case.rec = np.concatenate([case.rec, inputs.line_x(case.n, case.h, 128, 131)])
    print("case C2 256^3 SO8 nt=40", flush=True)
    g = _run(case)
    rec, uf, _ = case.oracle_forward()
    e_u, e_r = rel_l2(g["u_final"], uf), rel_l2(g["rec"], rec)
    print("field", e_u, "traces", e_r)
    assert e_u <= TOL and e_r <= TOL


def max_rel(x, ref):
    """max |x - ref| / max |ref| (element-wise bound, FP64)."""
    return float(np.abs(np.asarray(x, np.float64) - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("so", [2, 4, 8, 12, 16, 24])
def test_c2_full_length(so):
    """The full benchmark problem (256^3, 500 steps, launch configuration of the
    benchmark) against the oracle; a second receiver line near the source gives
    the traces signal (the configured line at z = 20 is beyond the distance the
    wave travels in 500 steps). Besides rel-L2, every point: |err| <= 1e-4 max|ref|
    (a wrong value in a quiet region cannot hide under the norm)."""
    from paper_1912_00695_amd import inputs
    case = c2_case(so, nt=500)
    case.rec = np.concatenate([case.rec, inputs.line_x(case.n, case.h, 128, 150)])
    print("case C2 256^3 SO%d nt=500" % so, flush=True)
    g = _run(case)
    rec, uf, _ = case.oracle_forward()
    e_u, e_r = rel_l2(g["u_final"], uf), rel_l2(g["rec"], rec)
    m_u, m_r = max_rel(g["u_final"], uf), max_rel(g["rec"], rec)
    print("SO", so, "field", e_u, "traces", e_r, "max", m_u, m_r, flush=True)
    assert e_u <= TOL and e_r <= TOL
    assert m_u <= 1e-4 and m_r <= 1e-4
    if so in (8, 12, 16, 24):
        _unfactorised_full_length(case, rec, uf)


def _unfactorised_full_length(case, rec, uf):
    """The ablation's unfactorised update (wave_forward_unfactorised) on the same
    full-length problem against the same oracle result. That form rounds each of its
    6r + 5 terms separately at the magnitude of u and forms u^{n+1} directly from
    u^n and u^{n-1}, so a step's rounding acts like an error in the stored previous
    level, which leapfrog amplifies by 1/sin(theta) for a mode of phase theta per
    step (theta ~ 0.045 for the 10 Hz wavelet here). Per step ~(6r+5) 2^-24 |u|
    of rounding, random-walking over 500 steps and amplified ~1/theta, gives 1e-4
    to 2e-4; bound 5e-4 on field and traces."""
    import torch
    from paper_1912_00695_amd import wave
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    o = wave.forward(case.wgrid(), t(case.vel), t(case.wavelet), case.src, case.rec,
                     want_final=True, unfactorised=True)
    torch.cuda.synchronize()
    eb = (rel_l2(o["u_final"].cpu().numpy(), uf), rel_l2(o["rec"].cpu().numpy(), rec))
    print("  unfactorised SO%d: field %.3e traces %.3e" % ((case.so,) + eb), flush=True)
    assert eb[0] <= 5e-4 and eb[1] <= 5e-4


def test_c2_full_size_properties():
    """At the full benchmark size and length (256^3, SO8, 500 steps): linearity in
    the wavelet and source-receiver reciprocity, to FP32 roundoff. (Scaling by 2 is
    exact only until the first subnormal rounding differs; after that the two runs'
    rounding errors decorrelate, so the comparison measures roundoff, not bits.)"""
    from paper_1912_00695_amd import inputs
    case = c2_case(8, nt=500)
    case.rec = np.concatenate([case.rec, inputs.line_x(case.n, case.h, 128, 150)])
    print("case C2 256^3 SO8 nt=500 linearity", flush=True)
    a = _run(case, want_final=False)["rec"]
    case.wavelet = 2.0 * case.wavelet
    b = _run(case, want_final=False)["rec"]
    print("linearity rel", rel_l2(b, 2.0 * a), flush=True)
    assert np.abs(a).max() > 0
    assert rel_l2(b, 2.0 * a) <= TOL
    case.wavelet = case.wavelet / 2.0
    A = np.array([[1280.0, 1280.0, 1280.0]])
    B = np.array([[900.0, 1400.0, 1100.0]])
    case.src, case.rec = A, B
    ab = _run(case, want_final=False)["rec"]
    case.src, case.rec = B, A
    ba = _run(case, want_final=False)["rec"]
    print("reciprocity rel", rel_l2(ab, ba), "max", np.abs(ab).max(), flush=True)
    assert np.abs(ab).max() > 1e-6
    assert rel_l2(ab, ba) <= TOL


def test_edge_cases():
    import torch
    from paper_1912_00695_amd import wave
    # nt = 0: no work, final level is u0
    case = ragged_case(4, nt=0)
    _oracle_inputs(case)
    case.wavelet = np.zeros((0, 3), dtype=np.float32)
    g = _run(case)
    assert np.array_equal(g["u_final"], case.u0)
    assert g["rec"].shape == (0, len(case.rec))
    # degenerate thin grids (single plane / single row / single column)
    from helpers import Case
    from paper_1912_00695_amd import inputs
    for n in [(1, 1, 40), (40, 1, 1), (1, 30, 1), (5, 3, 2), (64, 16, 1)]:
        h = (10.0, 12.0, 9.0)
        vel = inputs.smooth_random_range(n, 1500.0, 2600.0, 6.0, seed=1)
        c = Case(n, h, 4, 12, vel, 2600.0)
        c.src = np.array([[0.0, 0.0, 0.0]])
        c.wavelet = inputs.random_field((12, 1), 5)
        c.rec = np.array([[0.0, 0.0, 0.0], [(n[0] - 1) * h[0], (n[1] - 1) * h[1],
                                            (n[2] - 1) * h[2]]])
        c.u0 = inputs.random_field(vel.shape, 6) * 1e-2
        c.um1 = inputs.random_field(vel.shape, 7) * 1e-2
        g = _run(c)
        rec, uf, _ = c.oracle_forward()
        print("thin grid", n, rel_l2(g["u_final"], uf), rel_l2(g["rec"], rec), flush=True)
        assert rel_l2(g["u_final"], uf) <= TOL and rel_l2(g["rec"], rec) <= TOL, n
    # the workspace is reusable: same call twice on one workspace, identical bits
    case = ragged_case(8, nt=20)
    dev = torch.device("cuda:0")
    grid = case.wgrid()
    ws = torch.empty(wave.workspace_bytes(grid, len(case.src), len(case.rec)), dtype=torch.uint8,
                     device=dev)
    vel = torch.from_numpy(case.vel).to(dev)
    wav = torch.from_numpy(case.wavelet).to(dev)
    r1 = wave.forward(grid, vel, wav, case.src, case.rec, workspace=ws)["rec"].cpu()
    r2 = wave.forward(grid, vel, wav, case.src, case.rec, workspace=ws)["rec"].cpu()
    assert torch.equal(r1, r2)


def test_checkpoints_are_levels():
    case = ragged_case(4, nt=23)
    _oracle_inputs(case)
    g = _run(case, ckpt_every=7)
    ck = g["ckpt"]
    assert ck.shape[0] == 4
    np.testing.assert_array_equal(ck[0, 0], case.u0)
    np.testing.assert_array_equal(ck[0, 1], case.um1)
    for k in range(1, 4):
        _, uf, umf = _with_nt(case, 7 * k).oracle_forward()
        assert rel_l2(ck[k, 0], uf) <= TOL and rel_l2(ck[k, 1], umf) <= TOL


def _with_nt(case, nt):
    import copy
    c = copy.copy(case)
    c.nt = nt
    c.wavelet = case.wavelet[:nt]
    return c


@pytest.mark.parametrize("so", [2, 4, 6, 8, 10, 12, 14, 16, 24])
def test_chunk_lengths_give_identical_results(so):
    """z-chunks of 2, 5, 8 and 23 planes (the whole grid) against the default
    chunking (1 plane on this 97 x 37 x 23 grid): every point's update reads the
    same values in the same order whatever the chunk (queue priming, the halo loads
    and the LDS ring that holds them only change when values are fetched), so traces
    and final field are bitwise equal; the default run is also checked against the
    oracle."""
    case = ragged_case(so, nt=30, seed=60 + so)
    _oracle_inputs(case)
    print("chunk lengths SO", so, flush=True)
    ref = _run(case)
    rec, uf, _ = case.oracle_forward()
    assert rel_l2(ref["u_final"], uf) <= TOL and rel_l2(ref["rec"], rec) <= TOL
    for zc in (2, 5, 8, 23):
        g = _run(case, zchunk=zc)
        print("  zchunk", zc, "field equal", np.array_equal(g["u_final"], ref["u_final"]),
              flush=True)
        assert np.array_equal(g["u_final"], ref["u_final"])
        assert np.array_equal(g["rec"], ref["rec"])


def test_concurrent_calls_on_two_streams():
    """Two different solves, each with its own workspace, enqueued alternately three
    times on two streams: every result is bitwise that of the same solve run alone
    (concurrent calls share only the library's pool of host staging buffers for
    their tables; the second case's 3,000 extra off-grid receivers make its tables
    large)."""
    import torch
    from paper_1912_00695_amd import inputs, wave
    dev = torch.device("cuda:0")
    cases = [ragged_case(8, nt=40, seed=80), ragged_case(4, nt=40, seed=81)]
    c1 = cases[1]
    c1.rec = np.concatenate([c1.rec, inputs.random_points(c1.n, c1.h, 3000, 82)])
    for c in cases:
        _oracle_inputs(c)
    alone = [_run(c) for c in cases]
    t = lambda a: None if a is None else torch.from_numpy(
        np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    dev_in = [(t(c.vel), t(c.wavelet), t(c.u0), t(c.um1)) for c in cases]
    streams = [torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)]
    wss, outs = [], []
    for c, s in zip(cases, streams):
        with torch.cuda.stream(s):
            wss.append(torch.empty(wave.workspace_bytes(c.wgrid(), len(c.src), len(c.rec)),
                                   dtype=torch.uint8, device=dev))
    torch.cuda.synchronize()
    print("two streams, 3 rounds", flush=True)
    for _ in range(3):
        for k, (c, s) in enumerate(zip(cases, streams)):
            vel, wav, u0, um1 = dev_in[k]
            with torch.cuda.stream(s):
                outs.append((k, wave.forward(c.wgrid(), vel, wav, c.src, c.rec, u0=u0, um1=um1,
                                             want_final=True, workspace=wss[k], stream=s)))
    torch.cuda.synchronize()
    for k, o in outs:
        assert np.array_equal(o["rec"].cpu().numpy(), alone[k]["rec"])
        assert np.array_equal(o["u_final"].cpu().numpy(), alone[k]["u_final"])


@pytest.mark.parametrize("so", [4, 8, 16, 20])
def test_tall_tiles_sources_on_tile_edges(so):
    """Sources and receivers on and next to the edges of one-step tiles (y = 15 / 16,
    47 / 48) and of the two-tile workgroup tiles of SO4, SO8, SO16 and SO20 (y = 31 / 32,
    63 / 64; forced with WAVE_PATH_TILE32, which the library takes by itself only on
    grids with 256 or more such workgroups), on x-tile edges (63 / 64) and z-chunk edges
    (8-plane chunks), on a grid whose last workgroup tile holds a single one-step tile
    (ny = 80): against the oracle; the 64 x 16 tiling and the same request through the
    serving engine (one-step tiles, the engine's own chunking) bitwise against it."""
    import torch
    from helpers import Case
    from paper_1912_00695_amd import inputs, serving, wave
    n, h = (130, 80, 40), (10.0, 10.0, 10.0)
    vel = inputs.smooth_random_range(n, 1500.0, 2500.0, 8.0, seed=70 + so)
    case = Case(n, h, so, 40, vel, 2500.0, nbl=(6,) * 6)
    pts = [(63, 15, 7), (64, 16, 8), (63.5, 31.5, 15.5), (10, 32, 16), (100, 47, 23),
           (64.25, 48, 24), (30, 63, 31.75), (31, 64, 20), (120.5, 79, 12), (5, 0.5, 33)]
    case.src = np.array([[p[0] * h[0], p[1] * h[1], p[2] * h[2]] for p in pts])
    case.wavelet = np.random.default_rng(71).standard_normal((case.nt, len(pts))).astype(np.float32)
    case.rec = np.concatenate([case.src, inputs.random_points(n, h, 40, 72)])
    print("tall tiles: SO", so, "edge sources", flush=True)
    g = _run(case, zchunk=8, path=wave.PATH_TILE32)
    rec, uf, _ = case.oracle_forward()
    e_u, e_r = rel_l2(g["u_final"], uf), rel_l2(g["rec"], rec)
    print("  field %.3e traces %.3e" % (e_u, e_r), flush=True)
    assert e_u <= TOL and e_r <= TOL
    s = _run(case, zchunk=8, path=wave.PATH_TILE16)
    assert np.array_equal(s["u_final"], g["u_final"]) and np.array_equal(s["rec"], g["rec"])
    dev = torch.device("cuda:0")
    grid = case.wgrid(path=wave.PATH_TILE32)
    f = wave.forward(grid, torch.from_numpy(case.vel).to(dev),
                     torch.from_numpy(case.wavelet).to(dev), case.src, case.rec)["rec"].cpu().numpy()
    with serving.Engine(4 << 30, 4) as eng:
        _, o = eng.submit(grid, case.vel, case.wavelet, case.src, case.rec)
        eng.drain(120)
    print("  engine equals wave_forward:", np.array_equal(o, f), flush=True)
    assert np.array_equal(o, f)
