"""Continuous-batching engine on the GPU: results alone vs in the mix (bitwise), against
wave_forward (bitwise: same tile function) and the FP64 oracle, admission under a
tight memory budget, and overlap of requests arriving while others run."""
import time

import numpy as np
import pytest

import oracle
from helpers import rel_l2
from paper_1912_00695_amd import inputs

pytestmark = pytest.mark.gpu


def _small_mix(seed=0, count=6):
    from paper_1912_00695_amd import serving
    rng = np.random.default_rng(seed)
    shapes = [(64, 64, 64), (96, 80, 72), (70, 50, 90), (128, 64, 48)]
    # sources at depth 24.5 cells, near the receiver line at z = 20
    return [serving.mixed_request(rng, shapes=shapes, nt_range=(60, 160), nbl=8, src_z=24.5)
            for _ in range(count)]


def _engine(budget=8 << 30, slots=32):
    from paper_1912_00695_amd import serving
    return serving.Engine(budget, slots)


def test_alone_equals_mix_equals_forward():
    import torch
    from paper_1912_00695_amd import wave
    reqs = _small_mix()
    with _engine() as eng:
        mix = [eng.submit(r["grid"], r["vel"], r["wavelet"], r["src"], r["rec"]) for r in reqs]
        eng.drain(120)
        st = eng.stats()
        print("mix stats", st, flush=True)
        assert st["completed"] == len(reqs) and st["max_resident"] >= 2
        alone = []
        for r in reqs:
            alone.append(eng.submit(r["grid"], r["vel"], r["wavelet"], r["src"], r["rec"]))
            eng.drain(120)
        for (i1, o1), (i2, o2) in zip(mix, alone):
            assert eng.poll(i1)[0] == 0 and eng.poll(i2)[0] == 0
            assert np.abs(o1).max() > 0
            assert np.array_equal(o1, o2)
    dev = torch.device("cuda:0")
    for r, (_, o) in zip(reqs, mix):
        f = wave.forward(r["grid"], torch.from_numpy(r["vel"]).to(dev),
                         torch.from_numpy(r["wavelet"]).to(dev), r["src"], r["rec"])["rec"]
        assert np.array_equal(f.cpu().numpy(), o)


def test_engine_matches_oracle():
    reqs = _small_mix(seed=3, count=2)
    with _engine() as eng:
        outs = [eng.submit(r["grid"], r["vel"], r["wavelet"], r["src"], r["rec"]) for r in reqs]
        eng.drain(120)
    for r, (_, o) in zip(reqs, outs):
        g = r["grid"]
        og = oracle.Grid((g.nx, g.ny, g.nz), (g.hx, g.hy, g.hz), g.so, g.dt, g.nt,
                         nbl=tuple(g.nbl), vmax=g.vmax)
        orec, _, _ = oracle.forward(og, r["vel"], r["wavelet"], r["src"], r["rec"])
        print("engine vs oracle traces", rel_l2(o, orec), flush=True)
        assert rel_l2(o, orec) <= 1e-5


def test_shots_finishing_at_different_steps():
    """Shots resident together whose step counts differ (long, short, long, short,
    long): the short ones finish while the others keep stepping in the same graph,
    and each shot's counter must still be its own. Every result bitwise equals
    wave_forward of the same request, and the engine drains (bounded wait)."""
    import torch
    from paper_1912_00695_amd import serving, wave
    rng = np.random.default_rng(41)
    reqs = []
    for nt in (240, 40, 200, 60, 160):
        reqs.append(serving.mixed_request(rng, shapes=[(64, 64, 64), (80, 48, 56)],
                                          nt_range=(nt, nt), nbl=8, src_z=24.5))
    print("engine: shots of 240/40/200/60/160 steps submitted together", flush=True)
    with _engine() as eng:
        outs = [eng.submit(r["grid"], r["vel"], r["wavelet"], r["src"], r["rec"])
                for r in reqs]
        eng.drain(60)
        st = eng.stats()
        assert all(eng.poll(i)[0] == 0 for i, _ in outs)
    print("  stats", st, flush=True)
    assert st["completed"] == len(reqs)
    dev = torch.device("cuda:0")
    for r, (_, o) in zip(reqs, outs):
        f = wave.forward(r["grid"], torch.from_numpy(r["vel"]).to(dev),
                         torch.from_numpy(r["wavelet"]).to(dev), r["src"], r["rec"])["rec"]
        assert np.abs(o).max() > 0
        assert np.array_equal(f.cpu().numpy(), o)


def test_engine_full_size_shot_matches_oracle():
    """One shot of the serving mix at full size (160 x 160 x 320, SO8, 20-cell sponge,
    layered model, 300 steps, source 20 cells below the receiver line), run on the
    engine beside two 96^3 shots: traces against the FP64 oracle (rel-L2 <= 1e-5,
    element-wise <= 1e-4 max|ref|) and bitwise against wave_forward."""
    import torch
    from paper_1912_00695_amd import serving, wave
    rng = np.random.default_rng(21)
    big = serving.mixed_request(rng, shapes=[(160, 160, 320)], sos=(8,), nt_range=(300, 300),
                                src_z=40.0)
    small = [serving.mixed_request(rng, shapes=[(96, 96, 96)], sos=(8,), nt_range=(150, 250),
                                   src_z=40.0) for _ in range(2)]
    print("engine full-size shot 160x160x320 SO8 nt=300", flush=True)
    with _engine(budget=16 << 30) as eng:
        outs = [eng.submit(r["grid"], r["vel"], r["wavelet"], r["src"], r["rec"])
                for r in [big] + small]
        eng.drain(300)
        assert all(eng.poll(i)[0] == 0 for i, _ in outs)
    got = outs[0][1]
    g = big["grid"]
    og = oracle.Grid((g.nx, g.ny, g.nz), (g.hx, g.hy, g.hz), g.so, g.dt, g.nt,
                     nbl=tuple(g.nbl), vmax=g.vmax)
    orec, _, _ = oracle.forward(og, big["vel"], big["wavelet"], big["src"], big["rec"])
    e, m = rel_l2(got, orec), float(np.abs(got - orec).max() / np.abs(orec).max())
    print("  traces vs oracle: rel-L2 %.3e max %.3e" % (e, m), flush=True)
    assert np.abs(orec).max() > 0 and e <= 1e-5 and m <= 1e-4
    dev = torch.device("cuda:0")
    f = wave.forward(g, torch.from_numpy(big["vel"]).to(dev),
                     torch.from_numpy(big["wavelet"]).to(dev), big["src"], big["rec"])["rec"]
    assert np.array_equal(f.cpu().numpy(), got)


def test_budget_pressure_and_rejection():
    from paper_1912_00695_amd import serving, wave
    reqs = _small_mix(seed=7, count=6)
    need = [serving.request_bytes(r["grid"], 1, len(r["rec"])) for r in reqs]
    budget = sorted(need)[-1] + sorted(need)[-2]  # at most about two resident at once
    with _engine(budget=budget, slots=8) as eng:
        outs = [eng.submit(r["grid"], r["vel"], r["wavelet"], r["src"], r["rec"]) for r in reqs]
        eng.drain(300)
        st = eng.stats()
        print("budget", budget, "stats", st, flush=True)
        assert st["completed"] == 6 and st["max_pool_bytes"] <= budget
        assert st["max_resident"] <= 3
        big = serving.mixed_request(np.random.default_rng(1), shapes=[(256, 256, 256)])
        with pytest.raises(wave.WaveError) as ei:
            eng.submit(big["grid"], big["vel"], big["wavelet"], big["src"], big["rec"])
        assert ei.value.status == wave.EBUSY
        assert eng.stats()["rejected"] == 1
    with _engine() as ref:
        routs = [ref.submit(r["grid"], r["vel"], r["wavelet"], r["src"], r["rec"]) for r in reqs]
        ref.drain(120)
    for (_, a), (_, b) in zip(outs, routs):
        assert np.array_equal(a, b)


def test_continuous_arrivals_overlap():
    """Requests arriving while others run are admitted and run concurrently."""
    from paper_1912_00695_amd import serving
    with _engine() as eng:
        rng = np.random.default_rng(11)
        make = lambda r: serving.mixed_request(r, shapes=[(96, 96, 96), (128, 128, 128)],
                                               nt_range=(200, 400), nbl=10)
        stats, recs = serving.run_poisson(eng, 24, 60.0, seed=5, make=make)
        print("poisson stats", stats, flush=True)
        assert all(r["status"] == 0 for r in recs)
        assert stats["completed"] == 24 and stats["max_resident"] >= 2
        # some request was admitted while an earlier one was still running
        recs.sort(key=lambda r: r["t_admit"])
        overlap = any(b["t_admit"] < a["t_done"] for a, b in zip(recs, recs[1:]))
        assert overlap
        assert 0 < stats["p50_latency_s"] <= stats["p99_latency_s"]


def test_cache_groups_give_identical_results():
    """With a 1 MB cache-group cap every resident shot is stepped in a group of its
    own (16 launches per group, group after group): the traces must be bitwise those
    of the default grouping, in which the whole small mix shares one group."""
    reqs = _small_mix(seed=7, count=5)
    outs = {}
    for cap in (None, "1"):
        with _engine() as eng:
            if cap is not None:
                eng.set_group_bytes(1 << 20)
            got = [eng.submit(r["grid"], r["vel"], r["wavelet"], r["src"], r["rec"])
                   for r in reqs]
            eng.drain(120)
            st = eng.stats()
            assert st["completed"] == len(reqs)
            outs[cap] = [o for _, o in got]
        print("group cap", cap, "max resident", st["max_resident"], flush=True)
    for a, b in zip(outs[None], outs["1"]):
        assert np.abs(a).max() > 0
        assert np.array_equal(a, b)


def _tall_request(seed, nt=90):
    """128^3 SO8 request whose cache group the engine steps in 64 x 32 workgroup tiles:
    sources on and next to one-step and two-tile edges (x 63 / 64, y 15 / 16 and 31 /
    32, z on 4- and 8-plane chunk edges), 700 receivers (two sampling workgroups of
    512 threads)."""
    from paper_1912_00695_amd import wave
    rng = np.random.default_rng(seed)
    n, h = (128, 128, 128), (10.0, 10.0, 10.0)
    vel = inputs.layered(n, 3, 1500.0, 3500.0, seed=seed)
    vmax = float(vel.max())
    dt = 0.5 * wave.cfl_dt_max(8, vmax, h)
    pts = [(63, 15, 32), (64, 16, 40), (63.5, 31.5, 47.5), (20.25, 32, 64),
           (100, 47, 71), (float(rng.uniform(20, 100)), float(rng.uniform(20, 100)), 56.5)]
    src = np.array([[p[0] * h[0], p[1] * h[1], p[2] * h[2]] for p in pts])
    wav = rng.standard_normal((nt, len(pts))).astype(np.float32)
    rec = np.concatenate([inputs.line_x(n, h, 64, 20), inputs.random_points(n, h, 572, seed + 1)])
    grid = wave.make_grid(n, h, 8, dt, nt, (10,) * 6, vmax=vmax)
    return {"grid": grid, "vel": vel, "wavelet": wav, "src": src, "rec": rec}


def test_engine_tall_tile_groups():
    """Cache groups whose 64 x 32 workgroups fill the 256 CUs evenly are stepped on
    those tiles: two 128^3 SO8 shots in one group (8-plane chunks, 2 x 128 tall
    workgroups, then both shots' sampling workgroups), then one alone (4-plane chunks,
    256). Each result bitwise equals wave_forward on 64 x 32 and on 64 x 16 tiles; one
    against the FP64 oracle (rel-L2 <= 1e-5)."""
    import torch
    from paper_1912_00695_amd import wave
    reqs = [_tall_request(s) for s in (81, 82, 83)]
    print("engine tall-tile groups: 2 x 128^3 SO8 together, then 1 alone", flush=True)
    with _engine() as eng:
        outs = [eng.submit(r["grid"], r["vel"], r["wavelet"], r["src"], r["rec"])
                for r in reqs[:2]]
        eng.drain(120)
        outs.append(eng.submit(reqs[2]["grid"], reqs[2]["vel"], reqs[2]["wavelet"],
                               reqs[2]["src"], reqs[2]["rec"]))
        eng.drain(120)
        assert all(eng.poll(i)[0] == 0 for i, _ in outs)
    dev = torch.device("cuda:0")
    for r, (_, o) in zip(reqs, outs):
        assert np.abs(o).max() > 0
        g = r["grid"]
        for tile in (wave.PATH_TILE32, wave.PATH_TILE16):
            g2 = wave.make_grid((g.nx, g.ny, g.nz), (g.hx, g.hy, g.hz), g.so, g.dt, g.nt,
                                tuple(g.nbl), vmax=g.vmax, path=tile)
            f = wave.forward(g2, torch.from_numpy(r["vel"]).to(dev),
                             torch.from_numpy(r["wavelet"]).to(dev), r["src"], r["rec"])["rec"]
            assert np.array_equal(f.cpu().numpy(), o), tile
    g, r = reqs[2]["grid"], reqs[2]
    og = oracle.Grid((g.nx, g.ny, g.nz), (g.hx, g.hy, g.hz), g.so, g.dt, g.nt,
                     nbl=tuple(g.nbl), vmax=g.vmax)
    orec, _, _ = oracle.forward(og, r["vel"], r["wavelet"], r["src"], r["rec"])
    e = rel_l2(outs[2][1], orec)
    print("  alone vs oracle: traces rel-L2 %.3e" % e, flush=True)
    assert e <= 1e-5
