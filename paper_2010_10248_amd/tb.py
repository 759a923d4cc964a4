"""ctypes binding of the C ABI in ``include/tb.h`` (libtbwave.so).

Argument marshalling only: every step of the propagators runs in the HIP
library. Device memory and streams come from PyTorch. The functions keep the
C names without the ``tb_`` prefix; ``Acoustic`` bundles a model, its sparse
operators and a workspace for convenience.

A missing library is an error: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtbwave.so")

OK, EINVAL, EUNSUPPORTED, EUNSTABLE, ERANGE, ENOMEM, EHIP, EWORKSPACE = 0, -1, -2, -3, -4, -5, -6, -7
ACOUSTIC, TTI, ELASTIC = 0, 1, 2
SCHED_SB, SCHED_TB = 0, 1
OP_FORWARD, OP_ADJOINT, OP_GRADIENT = 0, 1, 2

_STATUS_NAMES = {OK: "TB_OK", EINVAL: "TB_EINVAL", EUNSUPPORTED: "TB_EUNSUPPORTED",
                 EUNSTABLE: "TB_EUNSTABLE", ERANGE: "TB_ERANGE", ENOMEM: "TB_ENOMEM",
                 EHIP: "TB_EHIP", EWORKSPACE: "TB_EWORKSPACE"}


class TbError(RuntimeError):
    def __init__(self, status: int, what: str, msg: str):
        super().__init__(f"{what}: {_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ModelDesc(ctypes.Structure):
    _fields_ = [("physics", ctypes.c_int32), ("shape", ctypes.c_int32 * 3),
                ("spacing", ctypes.c_double * 3), ("origin", ctypes.c_double * 3),
                ("space_order", ctypes.c_int32), ("nbl", ctypes.c_int32),
                ("dt", ctypes.c_double), ("nt", ctypes.c_int32), ("damp_vmax", ctypes.c_double),
                ("vp", ctypes.c_void_p), ("epsilon", ctypes.c_void_p), ("delta", ctypes.c_void_p),
                ("theta", ctypes.c_void_p), ("phi", ctypes.c_void_p), ("vs", ctypes.c_void_p),
                ("rho", ctypes.c_void_p), ("slowness2", ctypes.c_void_p)]


class Schedule(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("time_tile", ctypes.c_int32),
                ("tile_y", ctypes.c_int32), ("chunk_x", ctypes.c_int32)]

    def __repr__(self):
        return (f"Schedule(mode={'SB' if self.mode == SCHED_SB else 'TB'}, T={self.time_tile}, "
                f"tile_y={self.tile_y}, chunk_x={self.chunk_x})")


def schedule(mode: str = "tb", T: int = 2, tile_y: int = 32, chunk_x: int = 0) -> Schedule:
    if mode.lower() == "sb":
        return Schedule(SCHED_SB, 1, tile_y, chunk_x)
    return Schedule(SCHED_TB, T, tile_y, chunk_x)


class Request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("model", ctypes.c_void_p), ("sparse", ctypes.c_void_p),
                ("sched", ctypes.POINTER(Schedule)), ("d_obs", ctypes.c_void_p),
                ("rec_out", ctypes.c_void_p), ("grad_out", ctypes.c_void_p),
                ("checkpoint_every", ctypes.c_int32)]


SERVE_GRAPHS = 1

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_ip = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p

# Every entry point of include/tb.h with its ctypes signature.
_SIGNATURES = {
    "tb_create_model": (ctypes.c_int32, [ctypes.POINTER(ModelDesc), ctypes.POINTER(_vp)]),
    "tb_destroy_model": (None, [_vp]),
    "tb_inspect_sparse": (ctypes.c_int32, [_vp, ctypes.c_int32, _dp, _dp, ctypes.c_int32, _dp,
                                           ctypes.POINTER(_vp)]),
    "tb_destroy_sparse": (None, [_vp]),
    "tb_sparse_counts": (ctypes.c_int32, [_vp, _ip, _ip]),
    "tb_inspect_host": (ctypes.c_int32, [_ip, _dp, _dp, ctypes.c_double, ctypes.c_int32, _fp,
                                         ctypes.c_int32, _dp, _dp, _ip, _ip, _fp]),
    "tb_schedule_segments_host": (ctypes.c_int32, [_ip, ctypes.c_int32, ctypes.POINTER(Schedule),
                                                   ctypes.c_int32, _ip, _ip, _ip]),
    "tb_workspace_size": (ctypes.c_int32, [_vp, _vp, ctypes.POINTER(Schedule), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_size_t)]),
    "tb_forward": (ctypes.c_int32, [_vp, _vp, ctypes.POINTER(Schedule), _vp, ctypes.c_size_t,
                                    _vp, _vp, _vp, _vp]),
    "tb_forward_noalloc": (ctypes.c_int32, [_vp, _vp, ctypes.POINTER(Schedule), _vp, _vp, _vp,
                                            _vp]),
    "tb_adjoint": (ctypes.c_int32, [_vp, _vp, ctypes.POINTER(Schedule), _vp, ctypes.c_size_t,
                                    _vp, _vp, _vp]),
    "tb_gradient": (ctypes.c_int32, [_vp, _vp, ctypes.POINTER(Schedule), _vp, ctypes.c_size_t,
                                     _vp, _vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                     _vp]),
    "tb_gradient_workspace_size": (ctypes.c_int32, [_vp, _vp, ctypes.POINTER(Schedule),
                                                    ctypes.c_int32,
                                                    ctypes.POINTER(ctypes.c_size_t)]),
    "tb_autotune": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, _vp, ctypes.POINTER(Schedule),
                                     ctypes.POINTER(ctypes.c_double)]),
    "tb_autotune_clear": (ctypes.c_int32, []),
    "tb_server_create": (ctypes.c_int32, [ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(_vp)]),
    "tb_server_submit": (ctypes.c_int32, [_vp, ctypes.POINTER(Request),
                                          ctypes.POINTER(ctypes.c_int64)]),
    "tb_server_step": (ctypes.c_int32, [_vp, _ip, _ip]),
    "tb_server_poll": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_double), _ip]),
    "tb_server_stats": (ctypes.c_int32, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]),
    "tb_server_destroy": (None, [_vp]),
    "tb_kernel_timing": (ctypes.c_int32, [ctypes.c_int32]),
    "tb_kernel_timing_read": (ctypes.c_int32, [_ip, ctypes.POINTER(ctypes.c_double)]),
    "tb_last_error": (ctypes.c_char_p, []),
    "tb_version": (ctypes.c_char_p, []),
}


def lib():
    """Open libtbwave.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run "
                               "__graft_entry__.build() or paper_2010_10248_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().tb_last_error().decode()


def version() -> str:
    return lib().tb_version().decode()


def kernel_timing(enable: bool):
    _check(lib().tb_kernel_timing(1 if enable else 0), "tb_kernel_timing")


def kernel_timing_read():
    """(launches, total device ms) of the propagation kernels since enable."""
    n = ctypes.c_int32()
    ms = ctypes.c_double()
    _check(lib().tb_kernel_timing_read(ctypes.byref(n), ctypes.byref(ms)), "tb_kernel_timing_read")
    return n.value, ms.value


def _check(st: int, what: str):
    if st != OK:
        raise TbError(st, what, last_error())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _tptr(t) -> Optional[int]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> Optional[int]:
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def create_model(shape, spacing, origin, space_order, nbl, dt, nt, vp, damp_vmax=0.0,
                 physics=ACOUSTIC, epsilon=None, delta=None, theta=None, phi=None, vs=None,
                 rho=None, slowness2=None):
    """vp (and the physics' other parameters): float32 CUDA tensors
    [nx][ny][nz]; acoustic models may give the squared slowness ``slowness2``
    instead of vp (vp None). Returns an opaque handle."""
    d = ModelDesc()
    d.physics = physics
    d.shape[:] = [int(v) for v in shape]
    d.spacing[:] = [float(v) for v in spacing]
    d.origin[:] = [float(v) for v in origin]
    d.space_order = int(space_order)
    d.nbl = int(nbl)
    d.dt = float(dt)
    d.nt = int(nt)
    d.damp_vmax = float(damp_vmax)
    d.vp = None if vp is None else vp.data_ptr()
    for name, t in (("epsilon", epsilon), ("delta", delta), ("theta", theta), ("phi", phi),
                    ("vs", vs), ("rho", rho), ("slowness2", slowness2)):
        setattr(d, name, None if t is None else t.data_ptr())
    h = _vp()
    _check(lib().tb_create_model(ctypes.byref(d), ctypes.byref(h)), "tb_create_model")
    return h


def destroy_model(h):
    if h:
        lib().tb_destroy_model(h)


def inspect_sparse(model, src_xyz, src_wavelet, rec_xyz):
    sx = np.ascontiguousarray(src_xyz, dtype=np.float64).reshape(-1, 3)
    sw = np.ascontiguousarray(src_wavelet, dtype=np.float64)
    rx = np.ascontiguousarray(rec_xyz, dtype=np.float64).reshape(-1, 3)
    h = _vp()
    _check(lib().tb_inspect_sparse(model, sx.shape[0], _dptr(sx), _dptr(sw), rx.shape[0],
                                   _dptr(rx), ctypes.byref(h)), "tb_inspect_sparse")
    return h


def destroy_sparse(h):
    if h:
        lib().tb_destroy_sparse(h)


def sparse_counts(s):
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().tb_sparse_counts(s, ctypes.byref(a), ctypes.byref(b)), "tb_sparse_counts")
    return a.value, b.value


def inspect_host(shape, spacing, origin, dt, nt, vp_host, src_xyz, src_wavelet):
    """Host-only inspector: (nodes[npts][3], dcmp[nt][npts]) of the sources."""
    shp = np.asarray(shape, dtype=np.int32)
    sp = np.asarray(spacing, dtype=np.float64)
    og = np.asarray(origin, dtype=np.float64)
    vp = np.ascontiguousarray(vp_host, dtype=np.float32)
    sx = np.ascontiguousarray(src_xyz, dtype=np.float64).reshape(-1, 3)
    sw = np.ascontiguousarray(src_wavelet, dtype=np.float64)
    cap = 8 * max(sx.shape[0], 1)
    nodes = np.zeros((cap, 3), dtype=np.int32)
    dcmp = np.zeros((max(nt, 1), cap), dtype=np.float32)
    n = ctypes.c_int32(cap)
    _check(lib().tb_inspect_host(shp.ctypes.data_as(_ip), _dptr(sp), _dptr(og), float(dt),
                                 int(nt), vp.ctypes.data_as(_fp), sx.shape[0], _dptr(sx),
                                 _dptr(sw), ctypes.byref(n), nodes.ctypes.data_as(_ip),
                                 dcmp.ctypes.data_as(_fp)), "tb_inspect_host")
    k = n.value
    return nodes[:k].copy(), dcmp[:nt, :k].copy()


def schedule_segments(shape, space_order: int, sched: Schedule, wgs: int):
    """Host-only work decomposition of an acoustic schedule: (tile, segs) with
    tile = (rows, z width, owned rows, owned z) and segs[k] = (workgroup,
    tile y index, tile z index, xs, xe) in launch order."""
    shp = np.asarray(shape, dtype=np.int32)
    tile = np.zeros(4, dtype=np.int32)
    n = ctypes.c_int32(0)
    st = lib().tb_schedule_segments_host(shp.ctypes.data_as(_ip), int(space_order),
                                         ctypes.byref(sched), int(wgs), tile.ctypes.data_as(_ip),
                                         ctypes.byref(n), None)
    if st not in (0, EWORKSPACE):
        _check(st, "tb_schedule_segments_host")
    segs = np.zeros((max(n.value, 1), 5), dtype=np.int32)
    cap = ctypes.c_int32(segs.shape[0])
    _check(lib().tb_schedule_segments_host(shp.ctypes.data_as(_ip), int(space_order),
                                           ctypes.byref(sched), int(wgs), tile.ctypes.data_as(_ip),
                                           ctypes.byref(cap), segs.ctypes.data_as(_ip)),
           "tb_schedule_segments_host")
    return tuple(int(v) for v in tile), segs[:cap.value].copy()


def workspace_size(model, sparse, sched: Optional[Schedule], op: int = OP_FORWARD) -> int:
    b = ctypes.c_size_t()
    _check(lib().tb_workspace_size(model, sparse, None if sched is None else ctypes.byref(sched),
                                   op, ctypes.byref(b)), "tb_workspace_size")
    return b.value


def forward(model, sparse, sched, ws, rec_out=None, field_out=None, field_prev_out=None,
            stream=None):
    _check(lib().tb_forward(model, sparse, None if sched is None else ctypes.byref(sched),
                            _tptr(ws), ws.numel() * ws.element_size(), _tptr(rec_out),
                            _tptr(field_out), _tptr(field_prev_out), _stream(stream)),
           "tb_forward")


def forward_noalloc(model, sparse, sched, rec_out=None, field_out=None, field_prev_out=None,
                    stream=None):
    """tb_forward with the library's fixed device workspace (no allocation)."""
    _check(lib().tb_forward_noalloc(model, sparse, None if sched is None else ctypes.byref(sched),
                                    _tptr(rec_out), _tptr(field_out), _tptr(field_prev_out),
                                    _stream(stream)), "tb_forward_noalloc")


def adjoint(model, sparse, sched, ws, rec_in, src_out, stream=None):
    _check(lib().tb_adjoint(model, sparse, None if sched is None else ctypes.byref(sched),
                            _tptr(ws), ws.numel() * ws.element_size(), _tptr(rec_in),
                            _tptr(src_out), _stream(stream)), "tb_adjoint")


def gradient_workspace_size(model, sparse, sched: Optional[Schedule], checkpoint_every=0) -> int:
    b = ctypes.c_size_t()
    _check(lib().tb_gradient_workspace_size(model, sparse,
                                            None if sched is None else ctypes.byref(sched),
                                            int(checkpoint_every), ctypes.byref(b)),
           "tb_gradient_workspace_size")
    return b.value


def gradient(model, sparse, sched, ws, d_obs, grad_m, checkpoint_every=0, stream=None):
    """dJ/dm into grad_m; returns J (synchronises the stream)."""
    loss = ctypes.c_double()
    _check(lib().tb_gradient(model, sparse, None if sched is None else ctypes.byref(sched),
                             _tptr(ws), ws.numel() * ws.element_size(), _tptr(d_obs),
                             _tptr(grad_m), ctypes.byref(loss), int(checkpoint_every),
                             _stream(stream)), "tb_gradient")
    return loss.value


def autotune(model, sparse, steps=8, stream=None):
    """Time every valid schedule on the device; cache and return the best
    (Schedule, ms per step)."""
    best = Schedule()
    ms = ctypes.c_double()
    _check(lib().tb_autotune(model, sparse, int(steps), _stream(stream), ctypes.byref(best),
                             ctypes.byref(ms)), "tb_autotune")
    return best, ms.value


def autotune_clear():
    _check(lib().tb_autotune_clear(), "tb_autotune_clear")


class Server:
    """Continuous-batching server (tb_server_*). Requests reference models and
    sparse sets (and output tensors) that must stay alive until completion."""

    STAT_NAMES = ("epochs", "rounds", "launches", "passes_batched", "graph_captures",
                  "graph_replays", "actions", "completed")

    def __init__(self, arena_bytes: int, max_active: int, graphs: bool = True):
        h = _vp()
        _check(lib().tb_server_create(int(arena_bytes), int(max_active),
                                      SERVE_GRAPHS if graphs else 0, ctypes.byref(h)),
               "tb_server_create")
        self.h = h
        self._keep = {}

    def _submit(self, rq, keep):
        rid = ctypes.c_int64()
        _check(lib().tb_server_submit(self.h, ctypes.byref(rq), ctypes.byref(rid)),
               "tb_server_submit")
        self._keep[rid.value] = keep
        return rid.value

    def submit_forward(self, prop, rec_out, sched=None):
        rq = Request(OP_FORWARD, prop.model, prop.sparse,
                     None if sched is None else ctypes.pointer(sched), None,
                     rec_out.data_ptr(), None, 0)
        return self._submit(rq, (prop, rec_out))

    def submit_gradient(self, prop, d_obs, grad_out, sched=None, checkpoint_every=0):
        rq = Request(OP_GRADIENT, prop.model, prop.sparse,
                     None if sched is None else ctypes.pointer(sched), d_obs.data_ptr(), None,
                     grad_out.data_ptr(), int(checkpoint_every))
        return self._submit(rq, (prop, d_obs, grad_out))

    def step(self):
        a, q = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().tb_server_step(self.h, ctypes.byref(a), ctypes.byref(q)), "tb_server_step")
        return a.value, q.value

    def poll(self, cap=256):
        ids = (ctypes.c_int64 * cap)()
        losses = (ctypes.c_double * cap)()
        n = ctypes.c_int32()
        _check(lib().tb_server_poll(self.h, cap, ids, losses, ctypes.byref(n)), "tb_server_poll")
        out = [(ids[i], losses[i]) for i in range(n.value)]
        for rid, _ in out:
            self._keep.pop(rid, None)
        return out

    def stats(self):
        v = (ctypes.c_int64 * 8)()
        _check(lib().tb_server_stats(self.h, v, 8), "tb_server_stats")
        return dict(zip(self.STAT_NAMES, list(v)))

    def close(self):
        if self.h:
            lib().tb_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Propagator:
    """A model (acoustic or TTI, from the shot's physics) plus its sparse
    operators on the current CUDA device."""

    def __init__(self, shot, vp=None, src_wav=None, device="cuda", damp_vmax: float = 0.0,
                 slowness2=None):
        import torch

        self.shot = shot
        self.device = torch.device(device)

        def dev(a):
            if isinstance(a, torch.Tensor):
                return a.to(device=self.device, dtype=torch.float32).contiguous()
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=self.device)

        # An acoustic model may be given by its squared slowness instead of vp.
        self.slowness2 = None if slowness2 is None else dev(slowness2)
        self.vp = None if slowness2 is not None else dev(shot.vp if vp is None else vp)
        physics = getattr(shot, "physics", ACOUSTIC)
        self.physics = physics
        extra = {}
        names = {TTI: ("epsilon", "delta", "theta", "phi"), ELASTIC: ("vs", "rho")}
        if physics in names:
            for name in names[physics]:
                extra[name] = torch.as_tensor(
                    np.ascontiguousarray(getattr(shot, name), dtype=np.float32),
                    device=self.device)
        self._params = extra
        self.model = create_model(shot.shape, shot.spacing, shot.origin, shot.space_order,
                                  shot.nbl, shot.dt, shot.nt, self.vp, damp_vmax=damp_vmax,
                                  physics=physics, slowness2=self.slowness2, **extra)
        wav = shot.src_wav if src_wav is None else src_wav
        self.sparse = inspect_sparse(self.model, shot.src_xyz, wav, shot.rec_xyz)
        self.nsrc = shot.src_xyz.shape[0]
        self.nrec = shot.rec_xyz.shape[0]
        self._ws = {}

    def close(self):
        destroy_sparse(self.sparse)
        destroy_model(self.model)
        self.sparse = self.model = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, sched=None, op=OP_FORWARD):
        import torch

        nb = workspace_size(self.model, self.sparse, sched, op)
        key = op
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nb:
            ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def forward(self, sched=None, want_fields=True, stream=None):
        """Traces and the last two levels. Elastic: traces [2][nt][nrec]
        (vz, then pressure), u_last = vz^{nt-1/2}, u_prev = tzz^{nt}."""
        import torch

        ws = self.workspace(sched, OP_FORWARD)
        nt = self.shot.nt
        shape = ((2, nt, self.nrec) if getattr(self.shot, "physics", ACOUSTIC) == ELASTIC
                 else (nt, self.nrec))
        rec = torch.empty(shape, dtype=torch.float32, device=self.device)
        u = torch.empty(self.shot.shape, dtype=torch.float32, device=self.device) if want_fields else None
        up = torch.empty(self.shot.shape, dtype=torch.float32, device=self.device) if want_fields else None
        forward(self.model, self.sparse, sched, ws, rec, u, up, stream)
        return dict(traces=rec, u_last=u, u_prev=up)

    def adjoint(self, rec_in, sched=None, stream=None):
        import torch

        ws = self.workspace(sched, OP_ADJOINT)
        out = torch.empty((self.shot.nt, self.nsrc), dtype=torch.float32, device=self.device)
        adjoint(self.model, self.sparse, sched, ws, rec_in.contiguous(), out, stream)
        return out

    def gradient(self, d_obs, sched=None, checkpoint_every=0, stream=None):
        """(J, dJ/dm) for observed traces d_obs [nt][nrec] (CUDA float32)."""
        import torch

        nb = gradient_workspace_size(self.model, self.sparse, sched, checkpoint_every)
        key = ("grad", nb)
        ws = self._ws.get(key)
        if ws is None:
            self._ws = {k: v for k, v in self._ws.items() if not (isinstance(k, tuple))}
            ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        shape = tuple(self.shot.shape)
        if self.physics == ELASTIC:
            shape = (3,) + shape  # d/dlambda, d/dmu, d/db
        g = torch.empty(shape, dtype=torch.float32, device=self.device)
        J = gradient(self.model, self.sparse, sched, ws, d_obs.contiguous(), g, checkpoint_every,
                     stream)
        return J, g


Acoustic = Propagator
