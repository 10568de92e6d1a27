"""ctypes binding of libwave.so (include/wave.h).

Argument marshalling only: tensors are passed as device pointers, coordinates
as host float64 arrays, and every step of the solve runs in the HIP library on
the given stream (default: torch's current stream). PyTorch provides device
memory and streams.
If libwave.so has not been built, every entry point raises.
"""
import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwave.so")

OK, EINVAL, ECFL, ENOMEM, EDEVICE, EBUSY, EAGAIN, ELIMIT = 0, -1, -2, -3, -4, -5, -6, -7
STORE_F32, STORE_F16, STORE_BF16, STORE_DIFF = 0, 1, 2, 16
MODE_FORWARD, MODE_ADJOINT, MODE_GRADIENT = 0, 1, 2
# execution-path flags (kernels, launch shapes, cache hints; never the arithmetic)
PATH_ONE_STEP, PATH_TWO_STEP, PATH_STREAM, PATH_CACHED, PATH_LINEAR = 1, 2, 4, 8, 16
PATH_GRAPH, PATH_DIRECT, PATH_TILE16, PATH_TILE32 = 32, 64, 128, 256

# Entry points declared in include/wave.h.
SYMBOLS = ["wave_cfl_dt_max", "wave_workspace_bytes", "wave_checkpoint_bytes", "wave_forward",
           "wave_forward_unfactorised", "wave_forward_noalloc", "wave_noalloc_limit_bytes",
           "wave_adjoint", "wave_gradient", "wave_rtm", "wave_status_string", "wave_version"]


class WaveError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib().wave_status_string(status).decode() if _lib is not None else str(status)
        super().__init__("%s: %s (%d)" % (where, msg, status))


class WaveGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
                ("so", ctypes.c_int32), ("dt", ctypes.c_double), ("nt", ctypes.c_int32),
                ("nbl", ctypes.c_int32 * 6), ("vmax", ctypes.c_double),
                ("storage", ctypes.c_int32), ("path", ctypes.c_int32),
                ("zchunk", ctypes.c_int32)]

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


_lib = None


def lib():
    """Load libwave.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libwave.so is not built (run __graft_entry__.build()); "
                               "the solver has no non-HIP fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, fp, sz = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t
        gp = ctypes.POINTER(WaveGrid)
        i = ctypes.c_int
        L.wave_cfl_dt_max.argtypes = [i] + [ctypes.c_double] * 4
        L.wave_cfl_dt_max.restype = ctypes.c_double
        L.wave_workspace_bytes.argtypes = [gp, i, i, i, i]
        L.wave_workspace_bytes.restype = sz
        L.wave_checkpoint_bytes.argtypes = [gp, i]
        L.wave_checkpoint_bytes.restype = sz
        L.wave_forward.argtypes = [gp, fp, fp, dp, i, dp, i, fp, fp, fp, fp, fp, i, vp, sz, vp]
        L.wave_forward.restype = i
        L.wave_forward_unfactorised.argtypes = [gp, fp, fp, dp, i, dp, i, fp, fp, fp, fp, vp,
                                                sz, vp]
        L.wave_forward_unfactorised.restype = i
        L.wave_forward_noalloc.argtypes = [gp, fp, fp, dp, i, dp, i, fp, fp, fp, fp, vp]
        L.wave_forward_noalloc.restype = i
        L.wave_noalloc_limit_bytes.argtypes = []
        L.wave_noalloc_limit_bytes.restype = sz
        L.wave_adjoint.argtypes = [gp, fp, fp, dp, i, dp, i, fp, fp, vp, sz, vp]
        L.wave_adjoint.restype = i
        L.wave_gradient.argtypes = [gp, fp, fp, dp, i, dp, i, fp, fp, i, fp, fp, vp, sz, vp]
        L.wave_gradient.restype = i
        L.wave_rtm.argtypes = [gp, fp, fp, dp, i, dp, i, fp, fp, i, fp, vp, sz, vp]
        L.wave_rtm.restype = i
        L.wave_status_string.argtypes = [i]
        L.wave_status_string.restype = ctypes.c_char_p
        L.wave_version.argtypes = []
        L.wave_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def make_grid(n, h, so, dt, nt, nbl=(0,) * 6, vmax=None, storage=STORE_F32, path=0,
              zchunk=0):
    """n = (nx, ny, nz), h = (hx, hy, hz) metres, vmax = velocity bound (m/s); path
    (PATH_* flags) and zchunk choose the execution path (0: the library's choice)."""
    if vmax is None:
        raise ValueError("vmax (an upper bound of the velocity) is required")
    g = WaveGrid()
    g.nx, g.ny, g.nz = (int(v) for v in n)
    g.hx, g.hy, g.hz = (float(v) for v in h)
    g.so, g.dt, g.nt = int(so), float(dt), int(nt)
    for k, v in enumerate(nbl):
        g.nbl[k] = int(v)
    g.vmax = float(vmax)
    g.storage = int(storage)
    g.path = int(path)
    g.zchunk = int(zchunk)
    return g


def cfl_dt_max(so, vmax, h):
    return lib().wave_cfl_dt_max(int(so), float(vmax), *(float(v) for v in h))


def workspace_bytes(grid, nsrc, nrec, mode=MODE_FORWARD, ckpt_every=0):
    return lib().wave_workspace_bytes(ctypes.byref(grid), int(nsrc), int(nrec), int(mode),
                                      int(ckpt_every))


def checkpoint_bytes(grid, ckpt_every):
    return lib().wave_checkpoint_bytes(ctypes.byref(grid), int(ckpt_every))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _host_xyz(xyz):
    if xyz is None:
        return np.zeros((0, 3), dtype=np.float64)
    a = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
    return a


def _hptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a.shape[0] else None


def _dev_f32(t, shape, name):
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32):
        raise TypeError("%s must be a float32 CUDA tensor" % name)
    t = t.contiguous()
    if tuple(t.shape) != tuple(shape):
        t = t.reshape(shape)
    return t


def _workspace(nbytes, device, workspace):
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise WaveError(ENOMEM, "workspace")
        return workspace
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _device_of(vel):
    if not (isinstance(vel, torch.Tensor) and vel.is_cuda):
        raise TypeError("vel must be a float32 CUDA tensor")
    return vel.device


def _on(device, stream):
    """The stream a call runs on: `stream`, else torch's current stream of device.
    Every temporary, input copy, output and workspace of the call is allocated (and
    every copy made) while that stream is current, so torch's caching allocator
    orders their reuse after the call's work on it."""
    return stream if stream is not None else torch.cuda.current_stream(device)


def _sptr(s):
    return ctypes.c_void_p(s.cuda_stream)


def forward(grid, vel, wavelet=None, src_xyz=None, rec_xyz=None, u0=None, um1=None,
            want_final=False, ckpt_every=0, workspace=None, stream=None, rec_out=None,
            unfactorised=False, u_final=None):
    """Forward solve. Returns dict(rec=[nt][nrec], u_final=[nz][ny][nx] or None,
    ckpt=[nck][2][nz][ny][nx] or None). unfactorised=True runs the ablation entry
    point wave_forward_unfactorised (no checkpoints). rec_out and u_final may be
    passed in (reused output buffers), which also implies want_final."""
    s = _on(_device_of(vel), stream)
    with torch.cuda.stream(s):
        return _forward(grid, vel, wavelet, src_xyz, rec_xyz, u0, um1, want_final, ckpt_every,
                        workspace, s, rec_out, unfactorised, u_final)


def _forward(grid, vel, wavelet, src_xyz, rec_xyz, u0, um1, want_final, ckpt_every, workspace,
             s, rec_out, unfactorised, u_final):
    vel = _dev_f32(vel, grid.shape, "vel")
    dev = vel.device
    src = _host_xyz(src_xyz)
    rec = _host_xyz(rec_xyz)
    ns, nr, nt = src.shape[0], rec.shape[0], grid.nt
    wav = _dev_f32(wavelet, (nt, ns), "wavelet") if ns else None
    if rec_out is None:
        rec_out = torch.empty((nt, nr), dtype=torch.float32, device=dev)
    u0 = _dev_f32(u0, grid.shape, "u0")
    um1 = _dev_f32(um1, grid.shape, "um1")
    uf = u_final if u_final is not None else (
        torch.empty(grid.shape, dtype=torch.float32, device=dev) if want_final else None)
    ck = None
    if ckpt_every > 0:
        nck = (nt + ckpt_every - 1) // ckpt_every
        ck = torch.empty((nck, 2) + tuple(grid.shape), dtype=torch.float32, device=dev)
    nbytes = workspace_bytes(grid, ns, nr, MODE_FORWARD)
    if nbytes == 0:
        raise WaveError(EINVAL, "wave_workspace_bytes")
    ws = _workspace(nbytes, dev, workspace)
    if unfactorised:
        if ck is not None:
            raise WaveError(EINVAL, "wave_forward_unfactorised: no checkpoints")
        st = lib().wave_forward_unfactorised(
            ctypes.byref(grid), _ptr(vel), _ptr(wav), _hptr(src), ns, _hptr(rec), nr,
            _ptr(rec_out) if nr else None, _ptr(u0), _ptr(um1), _ptr(uf), _ptr(ws), ws.numel(),
            _sptr(s))
        if st != OK:
            raise WaveError(st, "wave_forward_unfactorised")
    else:
        st = lib().wave_forward(ctypes.byref(grid), _ptr(vel), _ptr(wav), _hptr(src), ns,
                                _hptr(rec), nr, _ptr(rec_out) if nr else None, _ptr(u0),
                                _ptr(um1), _ptr(uf), _ptr(ck), int(ckpt_every), _ptr(ws),
                                ws.numel(), _sptr(s))
        if st != OK:
            raise WaveError(st, "wave_forward")
    return {"rec": rec_out, "u_final": uf, "ckpt": ck}


def forward_noalloc(grid, vel, wavelet=None, src_xyz=None, rec_xyz=None, u0=None, um1=None,
                    want_final=False, stream=None, rec_out=None, u_final=None):
    """Forward solve through wave_forward_noalloc: the library's static device array
    is the workspace (no device allocation inside the call). Outputs (rec_out
    [nt][nrec], u_final [nz][ny][nx]) may be passed in; otherwise they are
    allocated here, before the call. Returns dict(rec, u_final)."""
    s = _on(_device_of(vel), stream)
    with torch.cuda.stream(s):
        vel = _dev_f32(vel, grid.shape, "vel")
        dev = vel.device
        src = _host_xyz(src_xyz)
        rec = _host_xyz(rec_xyz)
        ns, nr, nt = src.shape[0], rec.shape[0], grid.nt
        wav = _dev_f32(wavelet, (nt, ns), "wavelet") if ns else None
        if rec_out is None:
            rec_out = torch.empty((nt, nr), dtype=torch.float32, device=dev)
        if u_final is None and want_final:
            u_final = torch.empty(grid.shape, dtype=torch.float32, device=dev)
        u0 = _dev_f32(u0, grid.shape, "u0")
        um1 = _dev_f32(um1, grid.shape, "um1")
        st = lib().wave_forward_noalloc(ctypes.byref(grid), _ptr(vel), _ptr(wav), _hptr(src), ns,
                                        _hptr(rec), nr, _ptr(rec_out) if nr else None, _ptr(u0),
                                        _ptr(um1), _ptr(u_final), _sptr(s))
        if st != OK:
            raise WaveError(st, "wave_forward_noalloc")
        return {"rec": rec_out, "u_final": u_final}


def noalloc_limit_bytes():
    return lib().wave_noalloc_limit_bytes()


def adjoint(grid, vel, rec_data, rec_xyz, src_xyz, want_final=False, workspace=None,
            stream=None):
    """Backward solve (transpose of forward). Returns dict(src=[nt][nsrc], lam_final)."""
    s = _on(_device_of(vel), stream)
    with torch.cuda.stream(s):
        return _adjoint(grid, vel, rec_data, rec_xyz, src_xyz, want_final, workspace, s)


def _adjoint(grid, vel, rec_data, rec_xyz, src_xyz, want_final, workspace, s):
    vel = _dev_f32(vel, grid.shape, "vel")
    dev = vel.device
    src = _host_xyz(src_xyz)
    rec = _host_xyz(rec_xyz)
    ns, nr, nt = src.shape[0], rec.shape[0], grid.nt
    d = _dev_f32(rec_data, (nt, nr), "rec_data") if nr else None
    out = torch.empty((nt, ns), dtype=torch.float32, device=dev)
    lf = torch.empty(grid.shape, dtype=torch.float32, device=dev) if want_final else None
    nbytes = workspace_bytes(grid, ns, nr, MODE_ADJOINT)
    if nbytes == 0:
        raise WaveError(EINVAL, "wave_workspace_bytes")
    ws = _workspace(nbytes, dev, workspace)
    st = lib().wave_adjoint(ctypes.byref(grid), _ptr(vel), _ptr(d), _hptr(rec), nr, _hptr(src), ns,
                            _ptr(out) if ns else None, _ptr(lf), _ptr(ws), ws.numel(),
                            _sptr(s))
    if st != OK:
        raise WaveError(st, "wave_adjoint")
    return {"src": out, "lam_final": lf}


def gradient(grid, vel, wavelet, src_xyz, rec_xyz, rec_grad, ckpt=None, ckpt_every=0,
             want_wavelet_grad=True, workspace=None, stream=None):
    """Gradient of L(d) given dL/dd. Returns dict(grad_vel, grad_wavelet)."""
    s = _on(_device_of(vel), stream)
    with torch.cuda.stream(s):
        return _gradient(grid, vel, wavelet, src_xyz, rec_xyz, rec_grad, ckpt, ckpt_every,
                         want_wavelet_grad, workspace, s)


def _gradient(grid, vel, wavelet, src_xyz, rec_xyz, rec_grad, ckpt, ckpt_every,
              want_wavelet_grad, workspace, s):
    vel = _dev_f32(vel, grid.shape, "vel")
    dev = vel.device
    src = _host_xyz(src_xyz)
    rec = _host_xyz(rec_xyz)
    ns, nr, nt = src.shape[0], rec.shape[0], grid.nt
    wav = _dev_f32(wavelet, (nt, ns), "wavelet") if ns else None
    rg = _dev_f32(rec_grad, (nt, nr), "rec_grad") if nr else None
    if ckpt is not None:
        ckpt = ckpt.contiguous()
        if ckpt_every <= 0:
            raise WaveError(EINVAL, "wave_gradient: ckpt needs ckpt_every")
    gv = torch.empty(grid.shape, dtype=torch.float32, device=dev)
    gw = torch.empty((nt, ns), dtype=torch.float32, device=dev) if (want_wavelet_grad and ns) \
        else None
    nbytes = workspace_bytes(grid, ns, nr, MODE_GRADIENT, ckpt_every)
    if nbytes == 0:
        raise WaveError(EINVAL, "wave_workspace_bytes")
    ws = _workspace(nbytes, dev, workspace)
    st = lib().wave_gradient(ctypes.byref(grid), _ptr(vel), _ptr(wav), _hptr(src), ns, _hptr(rec),
                             nr, _ptr(rg), _ptr(ckpt), int(ckpt_every), _ptr(gv), _ptr(gw),
                             _ptr(ws), ws.numel(), _sptr(s))
    if st != OK:
        raise WaveError(st, "wave_gradient")
    return {"grad_vel": gv, "grad_wavelet": gw}


def rtm(grid, vel, wavelet, src_xyz, rec_xyz, rec_data, ckpt=None, ckpt_every=0, workspace=None,
        stream=None):
    """Zero-lag cross-correlation image sum_n u^n lambda^n of the forward field with the
    backward field driven by rec_data. Returns the image [nz][ny][nx]."""
    s = _on(_device_of(vel), stream)
    with torch.cuda.stream(s):
        return _rtm(grid, vel, wavelet, src_xyz, rec_xyz, rec_data, ckpt, ckpt_every, workspace,
                    s)


def _rtm(grid, vel, wavelet, src_xyz, rec_xyz, rec_data, ckpt, ckpt_every, workspace, s):
    vel = _dev_f32(vel, grid.shape, "vel")
    dev = vel.device
    src = _host_xyz(src_xyz)
    rec = _host_xyz(rec_xyz)
    ns, nr, nt = src.shape[0], rec.shape[0], grid.nt
    wav = _dev_f32(wavelet, (nt, ns), "wavelet") if ns else None
    rd = _dev_f32(rec_data, (nt, nr), "rec_data") if nr else None
    if ckpt is not None:
        ckpt = ckpt.contiguous()
    img = torch.empty(grid.shape, dtype=torch.float32, device=dev)
    nbytes = workspace_bytes(grid, ns, nr, MODE_GRADIENT, ckpt_every)
    if nbytes == 0:
        raise WaveError(EINVAL, "wave_workspace_bytes")
    ws = _workspace(nbytes, dev, workspace)
    st = lib().wave_rtm(ctypes.byref(grid), _ptr(vel), _ptr(wav), _hptr(src), ns, _hptr(rec), nr,
                        _ptr(rd), _ptr(ckpt), int(ckpt_every), _ptr(img), _ptr(ws), ws.numel(),
                        _sptr(s))
    if st != OK:
        raise WaveError(st, "wave_rtm")
    return img
