"""Continuous-batching shot server: ctypes binding of the wave_engine_* C ABI and a
seeded Poisson request driver.

The engine (C++ worker thread inside libwave.so) owns the GPU work; this module only
marshals requests, keeps each request's host output buffer alive until it completes,
and generates synthetic request streams.
"""
import ctypes
import time

import numpy as np

from . import inputs, wave


class WaveRequest(ctypes.Structure):
    _fields_ = [("grid", wave.WaveGrid), ("vel_h", ctypes.c_void_p),
                ("wavelet_h", ctypes.c_void_p), ("src_xyz_h", ctypes.c_void_p),
                ("nsrc", ctypes.c_int32), ("rec_xyz_h", ctypes.c_void_p),
                ("nrec", ctypes.c_int32), ("rec_out_h", ctypes.c_void_p)]


class WaveResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class WaveStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("resident", ctypes.c_uint64),
                ("p50_latency_s", ctypes.c_double), ("p99_latency_s", ctypes.c_double),
                ("mean_latency_s", ctypes.c_double), ("max_latency_s", ctypes.c_double),
                ("total_gpt", ctypes.c_double), ("busy_s", ctypes.c_double),
                ("span_s", ctypes.c_double), ("graph_builds", ctypes.c_uint64),
                ("replays", ctypes.c_uint64), ("max_resident", ctypes.c_uint64),
                ("max_pool_bytes", ctypes.c_size_t)]


_bound = False


def _bind():
    global _bound
    L = wave.lib()
    if not _bound:
        vp = ctypes.c_void_p
        L.wave_engine_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(vp)]
        L.wave_engine_create.restype = ctypes.c_int
        L.wave_engine_submit.argtypes = [vp, ctypes.POINTER(WaveRequest),
                                         ctypes.POINTER(ctypes.c_uint64)]
        L.wave_engine_submit.restype = ctypes.c_int
        L.wave_engine_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(WaveResult)]
        L.wave_engine_poll.restype = ctypes.c_int
        L.wave_engine_stats.argtypes = [vp, ctypes.POINTER(WaveStats)]
        L.wave_engine_stats.restype = ctypes.c_int
        L.wave_engine_drain.argtypes = [vp, ctypes.c_double]
        L.wave_engine_drain.restype = ctypes.c_int
        L.wave_engine_destroy.argtypes = [vp]
        L.wave_engine_destroy.restype = None
        L.wave_engine_request_bytes.argtypes = [ctypes.POINTER(wave.WaveGrid), ctypes.c_int,
                                                ctypes.c_int]
        L.wave_engine_request_bytes.restype = ctypes.c_size_t
        L.wave_engine_set_group_bytes.argtypes = [vp, ctypes.c_size_t]
        L.wave_engine_set_group_bytes.restype = ctypes.c_int
        _bound = True
    return L


def request_bytes(grid, nsrc, nrec):
    return _bind().wave_engine_request_bytes(ctypes.byref(grid), int(nsrc), int(nrec))


class Engine:
    """One engine: a device pool of budget_bytes and up to max_slots resident shots."""

    def __init__(self, budget_bytes, max_slots=64):
        import torch
        torch.cuda.init()  # the engine allocates on the current device
        L = _bind()
        h = ctypes.c_void_p()
        st = L.wave_engine_create(int(budget_bytes), int(max_slots), ctypes.byref(h))
        if st != wave.OK:
            raise wave.WaveError(st, "wave_engine_create")
        self._h = h
        self._out = {}

    def submit(self, grid, vel, wavelet, src_xyz, rec_xyz):
        """Queue one forward shot (host numpy inputs, copied by the engine). Returns
        (id, traces array [nt][nrec] filled when the request completes)."""
        vel = np.ascontiguousarray(vel, dtype=np.float32)
        src = np.ascontiguousarray(np.asarray(src_xyz, dtype=np.float64).reshape(-1, 3))
        rec = np.ascontiguousarray(np.asarray(rec_xyz, dtype=np.float64).reshape(-1, 3))
        wav = np.ascontiguousarray(np.asarray(wavelet, dtype=np.float32).reshape(grid.nt, -1))
        out = np.zeros((grid.nt, rec.shape[0]), dtype=np.float32)
        r = WaveRequest()
        r.grid = grid
        r.vel_h = vel.ctypes.data
        r.wavelet_h = wav.ctypes.data if src.shape[0] else None
        r.src_xyz_h = src.ctypes.data if src.shape[0] else None
        r.nsrc = src.shape[0]
        r.rec_xyz_h = rec.ctypes.data if rec.shape[0] else None
        r.nrec = rec.shape[0]
        r.rec_out_h = out.ctypes.data if rec.shape[0] else None
        rid = ctypes.c_uint64()
        st = _bind().wave_engine_submit(self._h, ctypes.byref(r), ctypes.byref(rid))
        if st != wave.OK:
            raise wave.WaveError(st, "wave_engine_submit")
        self._out[rid.value] = out
        return rid.value, out

    def set_group_bytes(self, nbytes):
        """Per-step bytes of the shots stepped together in one cache group (0: default)."""
        st = _bind().wave_engine_set_group_bytes(self._h, int(nbytes))
        if st != wave.OK:
            raise wave.WaveError(st, "wave_engine_set_group_bytes")

    def poll(self, rid):
        res = WaveResult()
        st = _bind().wave_engine_poll(self._h, int(rid), ctypes.byref(res))
        return st, {"t_submit": res.t_submit, "t_admit": res.t_admit, "t_done": res.t_done}

    def stats(self):
        s = WaveStats()
        _bind().wave_engine_stats(self._h, ctypes.byref(s))
        return {k: getattr(s, k) for k, _ in WaveStats._fields_}

    def drain(self, timeout_s=600.0, log=None, every_s=5.0):
        """Wait until nothing is queued or resident; with log, report the engine's
        counters every every_s seconds while waiting."""
        t_end = time.perf_counter() + timeout_s
        while True:
            left = t_end - time.perf_counter()
            if left <= 0:
                raise TimeoutError("engine did not drain within %.0f s" % timeout_s)
            st = _bind().wave_engine_drain(self._h, float(min(left, every_s)))
            if st == wave.OK:
                return
            if log is not None:
                s = self.stats()
                log("draining: completed %d queued %d resident %d replays %d graph builds %d"
                    % (s["completed"], s["queued"], s["resident"], s["replays"],
                       s["graph_builds"]))

    def close(self):
        if self._h is not None:
            _bind().wave_engine_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# Shot mix of the serving workload: grid shapes (nx, ny, nz), space orders,
# step counts, layered models, 20-cell sponge, one receiver line at z = 20.
SHAPES = [(96, 96, 96), (128, 128, 128), (192, 192, 192), (256, 256, 256), (160, 160, 320)]


def mixed_request(rng, shapes=SHAPES, sos=(4, 8), nt_range=(200, 1000), nbl=20, h=10.0,
                  src_z=None):
    """One seeded request of the serving mix: shape, SO and nt drawn uniformly, a 2-5
    layer ascending model in [1500, 4500] m/s, a 10 Hz Ricker at a uniform position
    outside the sponge (depth src_z cells when given), a receiver line along x at
    (i, ny/2, 20)."""
    n = shapes[rng.integers(len(shapes))]
    so = int(sos[rng.integers(len(sos))])
    nt = int(rng.integers(nt_range[0], nt_range[1] + 1))
    vel = inputs.layered(n, int(rng.integers(2, 6)), 1500.0, 4500.0,
                         seed=int(rng.integers(1 << 31)))
    vmax = float(vel.max())
    hh = (h, h, h)
    dt = 0.5 * wave.cfl_dt_max(so, vmax, hh)
    pos = [float(rng.uniform(nbl, n[a] - 1 - nbl)) for a in range(3)]
    if src_z is not None:
        pos[2] = float(src_z)
    src = inputs.point(pos, hh)
    rec = inputs.line_x(n, hh, n[1] // 2, min(20, n[2] - 1))
    wav = inputs.ricker(10.0, dt, nt)[:, None]
    grid = wave.make_grid(n, hh, so, dt, nt, (nbl,) * 6, vmax=vmax)
    return {"grid": grid, "vel": vel, "wavelet": wav, "src": src, "rec": rec,
            "updates": n[0] * n[1] * n[2] * nt}


def run_poisson(engine, nreq, rate, seed, make=mixed_request, timeout_s=900.0, log=None):
    """Submit nreq seeded requests at Poisson arrival times (rate per second), wait for
    all, return (engine stats, per-request records)."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, nreq))
    reqs_rng = np.random.default_rng(seed + 1)
    t0 = time.perf_counter()
    ids = []
    nxt = make(reqs_rng)
    for k in range(nreq):
        wait = arrivals[k] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        rid, _ = engine.submit(nxt["grid"], nxt["vel"], nxt["wavelet"], nxt["src"], nxt["rec"])
        ids.append((rid, nxt["updates"]))
        if log and (k + 1) % 50 == 0:
            log("submitted %d/%d" % (k + 1, nreq))
        if k + 1 < nreq:
            nxt = make(reqs_rng)
    engine.drain(timeout_s, log=log)
    recs = []
    for rid, upd in ids:
        st, t = engine.poll(rid)
        recs.append(dict(id=rid, status=st, updates=upd, **t))
    return engine.stats(), recs
