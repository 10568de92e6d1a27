"""Benchmark: Gpt-updates/s and fraction of the HBM roofline of the forward solve.

One benchmark step = one complete forward solve of the workload below (every
time step: damped star-stencil update, source injection, receiver sampling), with
all inputs already resident in HBM:

  256^3 grid (sponge included), h = 10 m, SO8, two-layer 1500/3000 m/s with the
  interface at z = 128, 40-cell sponge on all faces, 10 Hz Ricker at the centre,
  dt = 0.5 dt_max(3000 m/s), 500 time steps, 256 receivers along x at z = 20.

value = 256^3 * 500 * steps / elapsed / 1e9 (grid points updated per second).

Printed on stdout: ONE JSON line. Progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
ALG_BYTES_PER_PT = 16          # read u^n, u^{n-1}, v^2 dt^2; write u^{n+1} (FP32)
METRIC = "Gpt-updates/s and % HBM roofline at 256^3 SO4-16; p50/p99 shot latency"
KERNEL_SOURCES = ["paper_1912_00695_amd/csrc/wave_kernels.hip",
                  "paper_1912_00695_amd/csrc/wave_device.h",
                  "paper_1912_00695_amd/csrc/wave_internal.h"]
COUNTERS_FILE = os.path.join(ROOT, "profiles", "step_kernel_256cube_so8_counters.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter summary,
    or None when it is missing or was taken on different kernel sources."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    txt = open(COUNTERS_FILE).read()
    m = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", txt)
    t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not t or m.group(1) != kernel_hash():
        return None
    return float(t.group(1))


def c2_problem(so, nt=500, n=(256, 256, 256), path=0, zchunk=0):
    import numpy as np
    from paper_1912_00695_amd import inputs, wave
    h = (10.0, 10.0, 10.0)
    vmax = 3000.0
    dt = 0.5 * wave.cfl_dt_max(so, vmax, h)
    vel = inputs.two_layer(n, 1500.0, 3000.0, n[2] // 2)
    src = inputs.point((n[0] // 2, n[1] // 2, n[2] // 2), h)
    rec = inputs.line_x(n, h, n[1] // 2, 20)
    wav = inputs.ricker(10.0, dt, nt)[:, None]
    grid = wave.make_grid(n, h, so, dt, nt, (40,) * 6, vmax=vmax, path=path, zchunk=zchunk)
    return dict(grid=grid, vel=vel, src=src, rec=rec, wav=wav, n=n, nt=nt, so=so, dt=dt,
                h=h, vmax=vmax, nbl=(40,) * 6, np=np)


class Solver:
    """Device-resident inputs, a reusable workspace and output buffer for repeated
    solves. With the library's default launch policy a repeated call is replayed
    from a captured graph; the constructor makes two untimed calls (the second one
    captures), so timed calls replay."""

    def __init__(self, P, dev, unfactorised=False):
        import torch
        from paper_1912_00695_amd import wave
        self.P, self.wave, self.torch = P, wave, torch
        self.vel = torch.from_numpy(P["vel"]).to(dev)
        self.wav = torch.from_numpy(P["wav"]).to(dev)
        self.rec_out = torch.empty((P["nt"], len(P["rec"])), dtype=torch.float32, device=dev)
        nbytes = wave.workspace_bytes(P["grid"], len(P["src"]), len(P["rec"]))
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.unfactorised = unfactorised
        for _ in range(2):
            self.run()

    def run(self):
        self.wave.forward(self.P["grid"], self.vel, self.wav, self.P["src"], self.P["rec"],
                          workspace=self.ws, rec_out=self.rec_out,
                          unfactorised=self.unfactorised)


def time_solves(solver, steps, warmup, per_solve=None):
    """Elapsed seconds of `steps` back-to-back solves (HIP events on the solves'
    stream) and the host wall time; per_solve, if a list, receives each solve's
    own event-timed seconds."""
    import torch
    for _ in range(warmup):
        solver.run()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        solver.run()
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if per_solve is not None:
        per_solve.extend(ev[k].elapsed_time(ev[k + 1]) / 1000.0 for k in range(steps))
    return ev[0].elapsed_time(ev[steps]) / 1000.0, wall


def small_grid_leg(dev, solves=20):
    """Launch-bound sizes: the plain case (64^3, h = 10 m, SO4, v = 1500 m/s, no
    sponge, Gaussian pulse of sigma = 3 cells at rest at the centre, 100 steps; the
    earlier level is the pulse itself, as timing does not depend on the start) and
    a 96^3 case of the serving mix (SO4, 20-cell sponge, two-layer 1500/3000 m/s,
    Ricker source, receiver line, 200 steps). Each solve timed with direct
    launches and with the graph replay of repeated calls, for the default z-chunks
    and for 1-plane chunks (the most workgroups)."""
    import torch
    from paper_1912_00695_amd import inputs, wave
    res = {}
    h = (10.0, 10.0, 10.0)
    n1 = (64, 64, 64)
    dt1 = 0.5 * wave.cfl_dt_max(4, 1500.0, h)
    v1 = torch.from_numpy(inputs.constant(n1, 1500.0)).to(dev)
    u0 = torch.from_numpy(inputs.gaussian_pulse(n1, (32, 32, 32), 3.0)).to(dev)
    n2 = (96, 96, 96)
    dt2 = 0.5 * wave.cfl_dt_max(4, 3000.0, h)
    v2 = torch.from_numpy(inputs.two_layer(n2, 1500.0, 3000.0, 48)).to(dev)
    w2 = torch.from_numpy(inputs.ricker(10.0, dt2, 200)[:, None]).to(dev)
    src2, rec2 = inputs.point((48, 48, 48), h), inputs.line_x(n2, h, 48, 20)
    for name, zc in (("auto_chunks", 0), ("1_plane_chunks", 1)):
        for mode, path in (("direct", wave.PATH_DIRECT), ("graph", wave.PATH_GRAPH)):
            g1 = wave.make_grid(n1, h, 4, dt1, 100, vmax=1500.0, path=path, zchunk=zc)
            ws1 = torch.empty(wave.workspace_bytes(g1, 0, 0), dtype=torch.uint8, device=dev)
            uf = torch.empty((64, 64, 64), dtype=torch.float32, device=dev)
            g2 = wave.make_grid(n2, h, 4, dt2, 200, (20,) * 6, vmax=3000.0, path=path, zchunk=zc)
            ws2 = torch.empty(wave.workspace_bytes(g2, 1, 96), dtype=torch.uint8, device=dev)
            r2 = torch.empty((200, 96), dtype=torch.float32, device=dev)
            cases = (("c1_64cube_so4", 64 ** 3, 100,
                      lambda: wave.forward(g1, v1, None, None, None, u0=u0, um1=u0,
                                           workspace=ws1, u_final=uf)),
                     ("96cube_so4", 96 ** 3, 200,
                      lambda: wave.forward(g2, v2, w2, src2, rec2, workspace=ws2, rec_out=r2)))
            for cname, npts, nsteps, fn in cases:
                upd = npts * nsteps
                for _ in range(3):
                    fn()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                t0 = time.perf_counter()
                e0.record()
                for _ in range(solves):
                    fn()
                e1.record()
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                el = e0.elapsed_time(e1) / 1000.0
                res.setdefault(cname, {})["%s_%s" % (name, mode)] = {
                    "gpts": round(upd * solves / el / 1e9, 2),
                    "us_per_step": round(el / solves / nsteps * 1e6, 3),
                    "host_wall_s": round(wall, 4)}
            del ws1, ws2
    log("small grids: %s" % res)
    return res


def c1_leg(dev, mode, solves=20):
    """The plain case alone (64^3 SO4, v = 1500 m/s, Gaussian pulse at rest, no
    sponge, 100 steps), `solves` repeated solves with direct launches (mode
    "direct") or graph replay ("graph"), for kernel traces of the launch gaps."""
    import torch
    from paper_1912_00695_amd import inputs, wave
    h, n = (10.0, 10.0, 10.0), (64, 64, 64)
    path = {"direct": wave.PATH_DIRECT, "graph": wave.PATH_GRAPH}[mode]
    g = wave.make_grid(n, h, 4, 0.5 * wave.cfl_dt_max(4, 1500.0, h), 100, vmax=1500.0,
                       path=path)
    v = torch.from_numpy(inputs.constant(n, 1500.0)).to(dev)
    u0 = torch.from_numpy(inputs.gaussian_pulse(n, (32, 32, 32), 3.0)).to(dev)
    ws = torch.empty(wave.workspace_bytes(g, 0, 0), dtype=torch.uint8, device=dev)
    uf = torch.empty((64, 64, 64), dtype=torch.float32, device=dev)
    fn = lambda: wave.forward(g, v, None, None, None, u0=u0, um1=u0, workspace=ws, u_final=uf)
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(solves):
        fn()
    e1.record()
    torch.cuda.synchronize()
    el = e0.elapsed_time(e1) / 1000.0
    res = {"mode": mode, "gpts": round(64 ** 3 * 100 * solves / el / 1e9, 2),
           "us_per_step": round(el / solves / 100 * 1e6, 3)}
    log("c1 %s: %s" % (mode, res))
    return res


_C4_VEL = {}


def _c4_velocity():
    """The 512^3 smoothed-random 1500-4500 m/s model (seed 4), generated once."""
    from paper_1912_00695_amd import inputs
    if "v" not in _C4_VEL:
        _C4_VEL["v"] = inputs.smooth_random_range((512, 512, 512), 1500.0, 4500.0, 20.0, seed=4)
    return _C4_VEL["v"]


def reduced_precision_leg(dev):
    """512^3 SO8, smoothed-random 1500-4500 m/s, 15 Hz Ricker at the centre, 1000 steps,
    40-cell sponge, receivers at every 4th point of two lines along x (10 cells below
    the source and at z = 20): throughput of each wavefield storage format, speedup
    over FP32 storage, rel-L2 of the final field and traces against the FP32 run and,
    when tests/golden/c4_reference.npz (the FP64 oracle's result of this workload) is
    present, against the oracle (field on its 64^3 sub-lattice sample)."""
    import numpy as np
    import torch
    from paper_1912_00695_amd import inputs, wave
    n, h, nt = (512, 512, 512), (10.0, 10.0, 10.0), 1000
    vmax = 4500.0
    dt = 0.5 * wave.cfl_dt_max(8, vmax, h)
    vel = torch.from_numpy(_c4_velocity()).to(dev)
    wav = torch.from_numpy(inputs.ricker(15.0, dt, nt)[:, None]).to(dev)
    src = inputs.point((256, 256, 256), h)
    rec = np.concatenate([inputs.line_x(n, h, 256, 266)[::4], inputs.line_x(n, h, 256, 20)[::4]])
    gold = os.path.join(ROOT, "tests", "golden", "c4_reference.npz")
    gold = np.load(gold, allow_pickle=False) if os.path.exists(gold) else None
    res, ref = {}, None
    for name, st in (("f32", 0), ("f16_diff", 17), ("bf16_diff", 18), ("f16", 1), ("bf16", 2)):
        # every format on the one-step kernel (the FP32 default here is the two-step
        # kernel, which has no 16-bit form)
        g = wave.make_grid(n, h, 8, dt, nt, (40,) * 6, vmax=vmax, storage=st,
                           path=wave.PATH_ONE_STEP)
        ws = torch.empty(wave.workspace_bytes(g, 1, len(rec)), dtype=torch.uint8, device=dev)
        recb = torch.empty((nt, len(rec)), dtype=torch.float32, device=dev)
        wave.forward(g, vel, wav, src, rec, workspace=ws, rec_out=recb)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        wave.forward(g, vel, wav, src, rec, workspace=ws, rec_out=recb)
        e1.record()
        torch.cuda.synchronize()
        el = e0.elapsed_time(e1) / 1000.0
        out = wave.forward(g, vel, wav, src, rec, workspace=ws, want_final=True)
        u = out["u_final"].double()
        r = out["rec"].double()
        gp = 512 ** 3 * nt / el / 1e9
        bpp = {0: 16, 1: 10, 2: 10, 17: 12, 18: 12}[st]
        item = {"gpts": round(gp, 2), "alg_bytes_per_pt": bpp,
                "hbm_frac": round(gp * bpp / HBM_PEAK_GBS, 4)}
        if gold is not None:
            smp = u[4::8, 4::8, 4::8].cpu().numpy()
            gs, gt = gold["sample"].astype(np.float64), gold["traces"].astype(np.float64)
            item["field_rel_l2_vs_oracle"] = float(np.linalg.norm(smp - gs) / np.linalg.norm(gs))
            item["traces_rel_l2_vs_oracle"] = float(np.linalg.norm(r.cpu().numpy() - gt) /
                                                    np.linalg.norm(gt))
        if ref is None:
            ref = (u, r, gp)
        else:
            item["speedup_vs_f32"] = round(gp / ref[2], 3)
            item["field_rel_l2_vs_f32"] = float(torch.linalg.norm(u - ref[0]) /
                                                torch.linalg.norm(ref[0]))
            item["traces_rel_l2_vs_f32"] = float(torch.linalg.norm(r - ref[1]) /
                                                 torch.linalg.norm(ref[1]))
        res[name] = item
        log("lowp %s: %s" % (name, item))
        del ws, out, u, r, recb
    return res


def two_step_leg(dev):
    """Temporal blocking: the forward solve with two fused leapfrog steps per launch
    (the library's z-chunks: 64 planes, 128 at SO8 where that still gives 512
    workgroups) against one step per launch, on the sweep's 256^3 workload and at
    512^3 (FP32; 20 algorithmic bytes per point per two-step launch)."""
    from paper_1912_00695_amd import wave
    res = {}
    for n, so, nt in ((256, 4, 500), (256, 8, 500), (512, 2, 100), (512, 4, 100), (512, 6, 100),
                      (512, 8, 100)):
        item = {}
        for name, path, zc in (("two_step", wave.PATH_TWO_STEP, 0),
                               ("one_step", wave.PATH_ONE_STEP, 0)):
            S = Solver(c2_problem(so, nt=nt, n=(n, n, n), path=path, zchunk=zc), dev)
            e, _ = time_solves(S, 2, 1)
            item[name + "_gpts"] = round(n ** 3 * nt * 2 / e / 1e9, 2)
            del S
        item["speedup"] = round(item["two_step_gpts"] / item["one_step_gpts"], 3)
        res["%d^3_so%d" % (n, so)] = item
        log("two-step %d^3 SO%d: %s" % (n, so, item))
    res["default"] = ("two-step kernel used by default for SO2 from 3e7, SO4 from 6e7 and SO6 "
                      "from 8e7 grid points; at SO8 only when asked (WAVE_PATH_TWO_STEP)")
    return res


def basic_leg(dev):
    """Ablation after the paper's basic/aggressive experiment (Tables 2-3): the
    forward solve at 256^3 (the sweep's workload) with the unfactorised update
    (every term divided by r0 separately) against the factorised kernel, SO 8-24;
    throughput and rel-L2 of the basic form's final field against the factorised one
    (the workload's receivers at z = 20 see no arrival within 500 steps)."""
    import numpy as np
    import torch
    from paper_1912_00695_amd import wave
    res = {}
    for so in (8, 12, 16, 24):
        item = {}
        fields = {}
        for name, basic in (("basic", True), ("factorised", False)):
            P = c2_problem(so)
            S = Solver(P, dev, unfactorised=basic)
            e, _ = time_solves(S, 2, 1)
            item[name + "_gpts"] = round(256 ** 3 * 500 * 2 / e / 1e9, 2)
            out = wave.forward(P["grid"], S.vel, S.wav, P["src"], P["rec"], want_final=True,
                               workspace=S.ws, unfactorised=basic)
            fields[name] = out["u_final"].double()
            del S, out
        item["speedup_factorised_over_basic"] = round(item["factorised_gpts"] / item["basic_gpts"], 3)
        item["basic_field_rel_l2_vs_factorised"] = float(
            torch.linalg.norm(fields["basic"] - fields["factorised"]) /
            torch.linalg.norm(fields["factorised"]))
        del fields
        res["so%d" % so] = item
        log("basic vs factorised SO%d: %s" % (so, item))
    return res


def adjoint_gradient_leg(dev):
    """The gradient workload: 256^3 SO8, two-layer background with 40-cell sponge,
    10 Hz Ricker at (128, 128, 20), 65,536 receivers on the plane z = 20, 800 steps,
    checkpoints every 50. Times the forward solve that writes the checkpoints, one
    adjoint solve, the gradient given the checkpoints (segment recompute + adjoint
    with accumulation) and the RTM image (same pass, imaging condition); seeded random
    data for the adjoint-driven passes. Algorithmic bytes per point and step: adjoint
    16; gradient / image 44 (recomputed forward step 16, adjoint step 16, stored level
    4, accumulator read and write 8)."""
    import numpy as np
    import torch
    from paper_1912_00695_amd import inputs, wave
    n, h, nt, C = (256, 256, 256), (10.0, 10.0, 10.0), 800, 50
    dt = 0.5 * wave.cfl_dt_max(8, 3000.0, h)
    g = wave.make_grid(n, h, 8, dt, nt, (40,) * 6, vmax=3000.0)
    vel = torch.from_numpy(inputs.two_layer(n, 1500.0, 3000.0, 128)).to(dev)
    wav = torch.from_numpy(inputs.ricker(10.0, dt, nt)[:, None]).to(dev)
    src = inputs.point((128, 128, 20), h)
    rec = inputs.plane_z(n, h, 20)
    d = torch.from_numpy(np.random.default_rng(3).standard_normal(
        (nt, len(rec))).astype(np.float32)).to(dev)
    npts = 256 ** 3
    res = {}

    def timed(fn, reps=2):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            out = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1000.0 / reps, out

    t, fw = timed(lambda: wave.forward(g, vel, wav, src, rec, ckpt_every=C))
    ck = fw["ckpt"]
    res["forward_with_checkpoints"] = {"gpts": round(npts * nt / t / 1e9, 2), "ms": round(t * 1e3, 2)}
    del fw
    t, _ = timed(lambda: wave.adjoint(g, vel, d, rec, src))
    res["adjoint"] = {"gpts": round(npts * nt / t / 1e9, 2), "ms": round(t * 1e3, 2),
                      "hbm_frac_16B": round(npts * nt * 16 / t / 8e12, 4)}
    t, _ = timed(lambda: wave.gradient(g, vel, wav, src, rec, d, ckpt=ck, ckpt_every=C))
    res["gradient_given_checkpoints"] = {"gpts": round(npts * nt / t / 1e9, 2),
                                         "ms": round(t * 1e3, 2),
                                         "hbm_frac_44B": round(npts * nt * 44 / t / 8e12, 4)}
    t, _ = timed(lambda: wave.rtm(g, vel, wav, src, rec, d, ckpt=ck, ckpt_every=C))
    res["rtm_given_checkpoints"] = {"gpts": round(npts * nt / t / 1e9, 2), "ms": round(t * 1e3, 2),
                                    "hbm_frac_44B": round(npts * nt * 44 / t / 8e12, 4)}
    del ck
    log("adjoint/gradient C3: %s" % res)
    return res


def serving_saturated_leg(dev, count=40, reps=3):
    """The first `count` requests of a seeded serving mix submitted at once (saturated
    engine), against the same shots solved one by one with wave_forward; `reps`
    interleaved runs of each (a run's throughput varies by several per cent with the
    host's timing of submissions and uploads), medians reported."""
    import numpy as np
    import torch
    from paper_1912_00695_amd import serving, wave

    def requests():
        rng = np.random.default_rng(6)
        return [serving.mixed_request(rng) for _ in range(count)]

    upd = sum(r["updates"] for r in requests())
    batched, plain, builds = [], [], []
    for _ in range(reps):
        reqs = requests()
        with serving.Engine(96 << 30, 64) as eng:
            t0 = time.perf_counter()
            for r in reqs:
                eng.submit(r["grid"], r["vel"], r["wavelet"], r["src"], r["rec"])
            eng.drain(900)
            batched.append(upd / (time.perf_counter() - t0) / 1e9)
            builds.append(eng.stats()["graph_builds"])
        reqs = requests()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in reqs:
            wave.forward(r["grid"], torch.from_numpy(r["vel"]).to(dev),
                         torch.from_numpy(r["wavelet"]).to(dev), r["src"], r["rec"])["rec"].cpu()
        torch.cuda.synchronize()
        plain.append(upd / (time.perf_counter() - t0) / 1e9)
    mb, mp = float(np.median(batched)), float(np.median(plain))
    res = {"requests": count, "runs": reps, "batched_gpts": round(mb, 2),
           "plain_sequential_gpts": round(mp, 2), "speedup": round(mb / mp, 3),
           "batched_runs_gpts": [round(v, 1) for v in batched],
           "plain_runs_gpts": [round(v, 1) for v in plain], "graph_builds": builds,
           "note": "medians of interleaved runs; same requests, bitwise-identical results; "
                   "both include host->device upload of each request's inputs"}
    log("serving saturated: %s" % res)
    return res


def serving_leg(dev, nreq):
    """The serving workload: Poisson arrivals at 20/s (seed 5) of forward shots drawn
    from {96^3, 128^3, 192^3, 256^3, 160x160x320} x SO {4, 8} x nt in [200, 1000],
    layered 1500-4500 m/s models, 20-cell sponge, receiver line at z = 20; then 40
    requests of the same mix (seed 6) submitted at once (saturated engine) and solved
    one by one with wave_forward, for the batched-vs-plain throughput."""
    from paper_1912_00695_amd import serving
    res = {}
    with serving.Engine(96 << 30, 64) as eng:
        st, recs = serving.run_poisson(eng, nreq, 20.0, seed=5, log=log)
    ok = sum(1 for r in recs if r["status"] == 0)
    upd = sum(r["updates"] for r in recs)
    res["poisson"] = {"requests": nreq, "rate_per_s": 20.0, "completed": ok,
                      "p50_latency_s": round(st["p50_latency_s"], 4),
                      "p99_latency_s": round(st["p99_latency_s"], 4),
                      "mean_latency_s": round(st["mean_latency_s"], 4),
                      "aggregate_gpts": round(upd / st["span_s"] / 1e9, 2),
                      "offered_gpts": round(upd / (nreq / 20.0) / 1e9, 2),
                      "busy_gpts": round(st["total_gpt"] / max(st["busy_s"], 1e-9), 2),
                      "max_resident": st["max_resident"], "graph_builds": st["graph_builds"]}
    log("serving poisson: %s" % res["poisson"])
    res["saturated_40"] = serving_saturated_leg(dev)
    return res


def _oracle_sample(P, target_s, est_steps=6):
    """Time the FP64 oracle on the first steps of workload P: a 2-step run (thread
    start-up, first touch), an est_steps run for the time per step, then as many
    steps as fit target_s. Returns (Gpt-updates/s, steps, seconds)."""
    import numpy as np
    import oracle
    og = oracle.Grid(P["n"], P["h"], P["so"], P["dt"], 2, nbl=P["nbl"], vmax=P["vmax"])
    oracle.forward(og, P["vel"], P["wav"][:2], P["src"], P["rec"])
    og = og.replace(nt=est_steps)
    t0 = time.perf_counter()
    oracle.forward(og, P["vel"], P["wav"][:est_steps], P["src"], P["rec"])
    per_step = (time.perf_counter() - t0) / est_steps
    nsteps = int(max(2, min(P["nt"], target_s / max(per_step, 1e-6))))
    og = og.replace(nt=nsteps)
    t0 = time.perf_counter()
    oracle.forward(og, P["vel"], P["wav"][:nsteps], P["src"], P["rec"])
    el = time.perf_counter() - t0
    return int(np.prod(P["n"])) * nsteps / el / 1e9, nsteps, el


def cpu_baseline(P, target_s=15.0):
    """The FP64 oracle on the host cores, on bounded samples (the first time steps)
    of the benchmark workload (256^3 SO8), of the same at SO4, and of the 512^3 SO8
    reduced-precision workload; and on one thread for the plain 64^3 case."""
    import oracle
    val, nsteps, el = _oracle_sample(P, target_s)
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    res = {"value": val, "unit": "Gpt-updates/s",
           "cores": oracle.num_threads(), "kind": "oracle", "cpu_model": cpu,
           "sample": "FP64 oracle, 256^3 SO8 two-layer + 40-cell sponge, source and 256 "
                     "receivers, first %d of the 500 time steps (%.1f s)" % (nsteps, el)}
    v4, n4, e4 = _oracle_sample(c2_problem(4), 8.0)
    res["c2_256cube_so4"] = {"value": round(v4, 4), "unit": "Gpt-updates/s",
                             "sample": "first %d of 500 steps (%.1f s)" % (n4, e4)}
    from paper_1912_00695_amd import inputs
    n5, h5 = (512, 512, 512), (10.0, 10.0, 10.0)
    dt5 = 0.5 * oracle.cfl_dt_max(8, 4500.0, h5)
    P5 = dict(n=n5, h=h5, so=8, dt=dt5, nt=1000, nbl=(40,) * 6, vmax=4500.0,
              vel=_c4_velocity(), wav=inputs.ricker(15.0, dt5, 1000)[:, None],
              src=inputs.point((256, 256, 256), h5), rec=inputs.line_x(n5, h5, 256, 266))
    v5, n5s, e5 = _oracle_sample(P5, 8.0, est_steps=2)
    res["c4_512cube_so8"] = {"value": round(v5, 4), "unit": "Gpt-updates/s",
                             "sample": "first %d of 1000 steps (%.1f s)" % (n5s, e5)}
    # one thread on the small plain case: 64^3 SO4, homogeneous 1500 m/s, Gaussian
    # pulse at rest at the centre, 100 steps
    n1, h1 = (64, 64, 64), (10.0, 10.0, 10.0)
    v1 = inputs.constant(n1, 1500.0)
    g1 = oracle.Grid(n1, h1, 4, 0.5 * oracle.cfl_dt_max(4, 1500.0, h1), 100, vmax=1500.0)
    u0 = inputs.gaussian_pulse(n1, (32, 32, 32), 3.0)
    um1 = oracle.taylor_start(g1, v1, u0)
    nthreads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.forward(g1, v1, None, None, None, u0=u0, um1=um1)
        el1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(nthreads)
    res["single_thread_64cube_so4"] = {"value": 64 ** 3 * 100 / el1 / 1e9,
                                       "unit": "Gpt-updates/s", "seconds": round(el1, 2)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--so", type=int, default=8)
    ap.add_argument("--n", type=int, default=256,
                    help="grid points per axis of the timed workload (profiling runs; the "
                         "benchmark line is quoted at 256)")
    ap.add_argument("--nt", type=int, default=500, help="time steps of the timed workload")
    ap.add_argument("--launch", default="default", choices=["default", "direct", "graph"],
                    help="launch policy of the timed solves (default: graph replay of "
                         "repeated calls)")
    ap.add_argument("--kernel", default="default", choices=["default", "one_step", "two_step"],
                    help="kernel family of the timed solve (default: the library's choice, "
                         "the one-step kernel at 256^3)")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="requests in the Poisson serving stream (rate 20/s)")
    ap.add_argument("--only-timed", action="store_true",
                    help="run only the timed solves (for profiler runs)")
    ap.add_argument("--leg", default="",
                    help="run only this leg after the timed solves and print its JSON "
                         "(small_grids, c1_direct, c1_graph, adjoint_gradient, "
                         "serving_saturated, serving)")
    ap.add_argument("--with-copy", action="store_true",
                    help="after the timed solves, run a plain 256 MiB device copy three times "
                         "(calibrates profiler byte counters against a known size)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: this solver has no multi-GPU path (shots shard "
              "across GPUs with no exchange; see the sharding notes). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1912_00695_amd import wave
    dev = torch.device("cuda:0")
    wave.lib()

    if (args.n != 256 or args.nt != 500) and not args.only_timed:
        print("--n/--nt change the workload: use them with --only-timed", file=sys.stderr)
        sys.exit(2)
    from paper_1912_00695_amd import wave as _w
    launch_path = {"default": 0, "direct": _w.PATH_DIRECT, "graph": _w.PATH_GRAPH}[args.launch]
    launch_path |= {"default": 0, "one_step": _w.PATH_ONE_STEP,
                    "two_step": _w.PATH_TWO_STEP}[args.kernel]
    P = c2_problem(args.so, nt=args.nt, n=(args.n,) * 3, path=launch_path)
    solver = Solver(P, dev)
    log("timing %d solves of %d^3 SO%d x %d steps (warmup %d)" % (args.steps, args.n, args.so,
                                                                  P["nt"], args.warmup))
    per_solve = []
    el, wall = time_solves(solver, args.steps, args.warmup, per_solve)
    npts = args.n ** 3
    gpts = npts * P["nt"] * args.steps / el / 1e9
    launch_s = el / (args.steps * P["nt"])
    achieved = ALG_BYTES_PER_PT * npts / launch_s / 1e9
    log("Gpt/s %.2f  per-step %.2f us  effective %.0f GB/s" % (gpts, launch_s * 1e6, achieved))
    out = {
        "metric": METRIC, "value": round(gpts, 3), "unit": "Gpt-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1000.0, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "forward solve %d^3 SO%d, two-layer 1500/3000 m/s, 40-cell "
                               "sponge, 10 Hz Ricker at centre, %d receivers, %d steps, "
                               "dt=0.5*CFL" % (args.n, args.so, args.n, P["nt"]),
                   "grid": [args.n] * 3, "so": args.so, "nt": P["nt"], "nsrc": 1,
                   "nrec": args.n, "storage": "f32"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     # the committed counters cover the 256^3 SO8 one-step kernel only
                     "traffic": measured_traffic() if (args.n, args.so, args.kernel) in
                     ((256, 8, "default"), (256, 8, "one_step")) else None,
                     "kernel": ("fused2_kernel<%d> (16 B/pt one-step equivalent)"
                                if args.kernel == "two_step" else "step_kernel<%d,false>")
                     % (args.so // 2),
                     "alg_bytes_per_launch": ALG_BYTES_PER_PT * npts,
                     "avg_launch_us": round(launch_s * 1e6, 3),
                     "kernel_source_hash": kernel_hash()},
        "wall_s_timed": round(wall, 4),
        "per_solve": {"median_gpts": round(npts * P["nt"] / sorted(per_solve)[len(per_solve) // 2]
                                           / 1e9, 2),
                      "max_gpts": round(npts * P["nt"] / min(per_solve) / 1e9, 2),
                      "solves": len(per_solve),
                      "note": "each timed solve on its own (the paper times 5 runs)"},
    }
    del solver
    if args.with_copy:
        x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * x.numel() * 4
        del x, y
    if args.leg == "small_grids":
        out["small_grids"] = small_grid_leg(dev)
    elif args.leg in ("c1_direct", "c1_graph"):
        out["c1"] = c1_leg(dev, args.leg[3:])
    elif args.leg == "adjoint_gradient":
        out["adjoint_gradient_c3"] = adjoint_gradient_leg(dev)
    elif args.leg == "serving_saturated":
        out["serving_saturated"] = serving_saturated_leg(dev)
    elif args.leg == "serving":
        out["serving"] = serving_leg(dev, args.serving_requests)
    if args.only_timed or args.leg:
        print(json.dumps(out), flush=True)
        return
    if not args.no_sweep:
        sweep = {}
        for so in (2, 4, 8, 12, 16, 24):
            S = Solver(c2_problem(so), dev)
            e, _ = time_solves(S, 3, 1)
            g = npts * 500 * 3 / e / 1e9
            sweep["so%d" % so] = {"gpts": round(g, 2),
                                  "hbm_frac": round(g * ALG_BYTES_PER_PT / HBM_PEAK_GBS, 4)}
            log("sweep SO%d: %.2f Gpt/s" % (so, g))
            del S
        out["so_sweep_256"] = sweep
        # cache-defeating control: the one-step kernel at 512^3 (4 fields x 537 MB per
        # step, far above the 256 MB Infinity Cache), the library's default path there;
        # the two-step kernel timed beside it
        from paper_1912_00695_amd import wave as _w5
        ctl = {}
        for key, path in (("gpts", _w5.PATH_ONE_STEP), ("two_step_gpts", _w5.PATH_TWO_STEP)):
            S = Solver(c2_problem(8, nt=500, n=(512, 512, 512), path=path), dev)
            e, _ = time_solves(S, 2, 0)
            ctl[key] = round(512 ** 3 * 500 * 2 / e / 1e9, 2)
            del S
        out["control_512_so8"] = {"gpts": ctl["gpts"],
                                  "kernel": "step_kernel<4,false> (one step, the default path)",
                                  "hbm_frac": round(ctl["gpts"] * ALG_BYTES_PER_PT / HBM_PEAK_GBS, 4),
                                  "nt": 500, "two_step_gpts": ctl["two_step_gpts"],
                                  "two_step": "two-step kernel, 128-plane chunks (forced)"}
        log("control 512^3 SO8: %s" % out["control_512_so8"])
    if not args.no_sweep:
        out["small_grids"] = small_grid_leg(dev)
        out["lowp_512_so8"] = reduced_precision_leg(dev)
        out["two_step_kernel"] = two_step_leg(dev)
        out["basic_vs_factorised_256"] = basic_leg(dev)
        out["adjoint_gradient_c3"] = adjoint_gradient_leg(dev)
    if not args.no_serving:
        out["serving"] = serving_leg(dev, args.serving_requests)
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(P)
        log("cpu baseline %.4f Gpt/s on %d threads" % (out["cpu_baseline"]["value"],
                                                       out["cpu_baseline"]["cores"]))
    out["paper_context"] = {"v100_so8_aggressive_gpts": 32.9, "v100_so8_alg_hbm_frac": 0.58,
                            "titanz_so8_aggressive_gpts": 3.71,
                            "note": "Gpt/s derived from the paper's Table 3 / Table 2 times at "
                                    "256^3 x 30000 steps; other hardware, context only"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
