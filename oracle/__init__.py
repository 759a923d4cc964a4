"""FP64 CPU oracle (ctypes wrapper around ``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline leg may use it; the product package never imports it. It shares no
code with the GPU library. See ``oracle.c`` for what each routine computes and
which passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP)."""
    srcs = [os.path.join(_HERE, f) for f in ("oracle.c", "oracle_tti.c", "oracle_elastic.c")
            if os.path.exists(os.path.join(_HERE, f))]
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", *srcs, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        srcs = [os.path.join(_HERE, f) for f in ("oracle.c", "oracle_tti.c", "oracle_elastic.c")]
        if not os.path.exists(_LIB_PATH) or any(
                os.path.getmtime(f) > os.path.getmtime(_LIB_PATH) for f in srcs if os.path.exists(f)):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        c_int, c_double = ctypes.c_int, ctypes.c_double
        vp = ctypes.c_void_p
        L.or_fornberg.argtypes = [c_int, c_int, _dp, c_double, _dp]
        L.or_weights_d2.argtypes = [c_int, _dp]
        L.or_weights_d1.argtypes = [c_int, _dp]
        L.or_weights_d1_staggered.argtypes = [c_int, _dp]
        L.or_trilinear.argtypes = [_dp, _dp, _dp, _ip, _ip, _dp]
        L.or_damping.argtypes = [_ip, _dp, c_int, c_double, _dp]
        L.or_damping.restype = None
        L.or_laplacian.argtypes = [_ip, _dp, c_int, _dp, _dp]
        L.or_acoustic_forward.argtypes = [_ip, _dp, _dp, c_int, c_int, c_double, c_int, _dp,
                                          c_double, c_int, _dp, _dp, c_int, _dp,
                                          vp, vp, vp, vp, vp, vp]
        L.or_acoustic_inject_increment.argtypes = [_ip, _dp, _dp, c_int, c_double, _dp, c_int,
                                                   _dp, _dp, c_int, _dp]
        L.or_acoustic_adjoint.argtypes = [_ip, _dp, _dp, c_int, c_int, c_double, c_int, _dp,
                                          c_double, c_int, _dp, _dp, c_int, _dp, _dp,
                                          vp, vp, vp, vp]
        L.or_misfit.argtypes = [c_int, c_int, _dp, _dp, vp]
        L.or_misfit.restype = c_double
        L.or_num_threads.restype = c_int
        if hasattr(L, "or_tti_forward"):
            L.or_tti_forward.argtypes = [_ip, _dp, _dp, c_int, c_int, c_double, c_int,
                                         _dp, _dp, _dp, _dp, _dp, c_double,
                                         c_int, _dp, _dp, c_int, _dp, vp, vp, vp, vp, vp,
                                         vp, vp]
        if hasattr(L, "or_tti_adjoint"):
            L.or_tti_adjoint.argtypes = [_ip, _dp, _dp, c_int, c_int, c_double, c_int,
                                         _dp, _dp, _dp, _dp, _dp, c_double,
                                         c_int, _dp, vp, c_int, _dp, _dp, vp, vp, vp, vp]
        if hasattr(L, "or_tti_operators"):
            L.or_tti_operators.argtypes = [_ip, _dp, c_int, _dp, _dp, _dp, vp, vp]
        if hasattr(L, "or_elastic_adjoint"):
            L.or_elastic_adjoint.argtypes = [_ip, _dp, _dp, c_int, c_int, c_double, c_int,
                                             _dp, _dp, _dp, c_double, c_int, _dp, c_int, _dp,
                                             _dp, vp, vp, vp]
        if hasattr(L, "or_elastic_passes"):
            L.or_elastic_passes.argtypes = [_ip, _dp, c_int, c_int, c_double, _dp, _dp, _dp,
                                            c_double, c_int, _dp]
        if hasattr(L, "or_elastic_forward"):
            L.or_elastic_forward.argtypes = [_ip, _dp, _dp, c_int, c_int, c_double, c_int,
                                             _dp, _dp, _dp, c_double,
                                             c_int, _dp, _dp, c_int, _dp, vp, vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(st: int, what: str):
    if st < 0:
        raise RuntimeError(f"oracle {what} failed with status {st}")


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().or_num_threads())


def fornberg(m: int, x, x0: float) -> np.ndarray:
    x = _f64(x)
    out = np.zeros(len(x))
    _check(lib().or_fornberg(m, len(x), x, float(x0), out), "fornberg")
    return out


def weights_d2(so: int) -> np.ndarray:
    out = np.zeros(so // 2 + 1)
    _check(lib().or_weights_d2(so, out), "weights_d2")
    return out


def weights_d1(so: int) -> np.ndarray:
    out = np.zeros(so // 2)
    _check(lib().or_weights_d1(so, out), "weights_d1")
    return out


def weights_d1_staggered(so: int) -> np.ndarray:
    out = np.zeros(so // 2)
    _check(lib().or_weights_d1_staggered(so, out), "weights_d1_staggered")
    return out


def trilinear(p, o, h, n):
    """Return (nodes[k][3], weights[k]) of the non-zero trilinear corners."""
    nodes = np.zeros((8, 3), dtype=np.int32)
    w = np.zeros(8)
    cnt = lib().or_trilinear(_f64(p), _f64(o), _f64(h), np.asarray(n, dtype=np.int32),
                             nodes, w)
    if cnt < 0:
        raise ValueError("point outside the grid")
    return nodes[:cnt].copy(), w[:cnt].copy()


def damping(shape, spacing, nbl: int, vmax: float) -> np.ndarray:
    out = np.zeros(shape)
    lib().or_damping(np.asarray(shape, dtype=np.int32), _f64(spacing), int(nbl), float(vmax),
                     out)
    return out


def laplacian(u: np.ndarray, spacing, so: int) -> np.ndarray:
    u = _f64(u)
    out = np.zeros_like(u)
    _check(lib().or_laplacian(np.asarray(u.shape, dtype=np.int32), _f64(spacing), so, u, out),
           "laplacian")
    return out


def acoustic_forward(shot, vp: Optional[np.ndarray] = None, src_wav=None, vmax_damp: float = 0.0,
                     u0=None, u1=None, want_history: bool = False, nbl: Optional[int] = None,
                     src_xyz=None, rec_xyz=None, nt: Optional[int] = None):
    """Run the FP64 acoustic forward of a ``workloads.Shot``.

    Returns dict(traces[nt][nrec], u_last, u_prev, history (optional)).
    """
    n = np.asarray(shot.shape, dtype=np.int32)
    vp = _f64(shot.vp if vp is None else vp)
    wav = _f64(shot.src_wav if src_wav is None else src_wav)
    sx = _f64(shot.src_xyz if src_xyz is None else src_xyz)
    rx = _f64(shot.rec_xyz if rec_xyz is None else rec_xyz)
    nt = shot.nt if nt is None else nt
    nsrc = sx.shape[0]
    nrec = rx.shape[0]
    traces = np.zeros((nt, nrec))
    u_last = np.zeros(shot.shape)
    u_prev = np.zeros(shot.shape)
    hist = np.zeros((nt + 1,) + tuple(shot.shape)) if want_history else None
    u0 = None if u0 is None else _f64(u0)
    u1 = None if u1 is None else _f64(u1)
    st = lib().or_acoustic_forward(n, _f64(shot.spacing), _f64(shot.origin), shot.space_order,
                                   shot.nbl if nbl is None else nbl, float(shot.dt), nt, vp,
                                   float(vmax_damp), nsrc, sx, wav, nrec, rx,
                                   _ptr(u0), _ptr(u1), _ptr(traces), _ptr(u_last),
                                   _ptr(u_prev), _ptr(hist))
    _check(st, "acoustic_forward")
    out = dict(traces=traces, u_last=u_last, u_prev=u_prev)
    if want_history:
        out["history"] = hist
    return out


def acoustic_inject_increment(shot, t: int, vp=None) -> np.ndarray:
    out = np.zeros(shot.shape)
    _check(lib().or_acoustic_inject_increment(
        np.asarray(shot.shape, dtype=np.int32), _f64(shot.spacing), _f64(shot.origin),
        shot.space_order, float(shot.dt), _f64(shot.vp if vp is None else vp),
        shot.src_xyz.shape[0], _f64(shot.src_xyz), _f64(shot.src_wav), int(t), out),
        "inject_increment")
    return out


def acoustic_adjoint(shot, res: np.ndarray, vp=None, vmax_damp: float = 0.0,
                     u_hist: Optional[np.ndarray] = None, want_grad: bool = False,
                     want_qhat: bool = True, nbl: Optional[int] = None):
    """Adjoint run driven by data-space vector ``res[nt][nrec]``.

    Returns dict(qhat[nt][nsrc], grad (if want_grad, needs u_hist), nu1).
    """
    n = np.asarray(shot.shape, dtype=np.int32)
    vp = _f64(shot.vp if vp is None else vp)
    nsrc = shot.src_xyz.shape[0]
    nrec = shot.rec_xyz.shape[0]
    res = _f64(res)
    qhat = np.zeros((shot.nt, nsrc)) if want_qhat else None
    grad = np.zeros(shot.shape) if want_grad else None
    nu1 = np.zeros(shot.shape)
    if want_grad:
        if u_hist is None:
            raise ValueError("gradient needs the forward history")
        u_hist = _f64(u_hist)
    st = lib().or_acoustic_adjoint(n, _f64(shot.spacing), _f64(shot.origin), shot.space_order,
                                   shot.nbl if nbl is None else nbl, float(shot.dt), shot.nt, vp,
                                   float(vmax_damp), nsrc, _f64(shot.src_xyz),
                                   _f64(shot.src_wav), nrec, _f64(shot.rec_xyz), res,
                                   _ptr(u_hist), _ptr(grad), _ptr(qhat), _ptr(nu1))
    _check(st, "acoustic_adjoint")
    return dict(qhat=qhat, grad=grad, nu1=nu1)


def acoustic_gradient(shot, dobs: np.ndarray, vp=None, vmax_damp: float = 0.0):
    """J(m) and dJ/dm (m = 1/vp^2) for J = 1/2 sum |P_r u^k - dobs^k|^2."""
    fw = acoustic_forward(shot, vp=vp, vmax_damp=vmax_damp, want_history=True)
    res = np.zeros_like(fw["traces"])
    J = lib().or_misfit(shot.nt, shot.rec_xyz.shape[0], _f64(fw["traces"]), _f64(dobs),
                        _ptr(res))
    adj = acoustic_adjoint(shot, res, vp=vp, vmax_damp=vmax_damp,
                           u_hist=fw["history"][:shot.nt], want_grad=True, want_qhat=False)
    return float(J), adj["grad"], fw


def tti_forward(shot, vp=None, vmax_damp: float = 0.0, src_wav=None, epsilon=None, delta=None,
                theta=None, phi=None, want_history: bool = False):
    """FP64 pseudo-acoustic TTI forward of a ``workloads.Shot`` (zero initial
    state). Returns dict(traces[nt][nrec] of p, p_last, p_prev, r_last, r_prev
    and, with want_history, p_hist, r_hist [nt][N] (levels 0..nt-1))."""
    n = np.asarray(shot.shape, dtype=np.int32)
    f = lambda a, b: _f64(b if a is None else a)
    vp = f(vp, shot.vp)
    eps, dl, th, ph = (f(epsilon, shot.epsilon), f(delta, shot.delta), f(theta, shot.theta),
                       f(phi, shot.phi))
    wav = f(src_wav, shot.src_wav)
    sx = _f64(shot.src_xyz)
    rx = _f64(shot.rec_xyz)
    out = dict(traces=np.zeros((shot.nt, rx.shape[0])))
    for k in ("p_last", "p_prev", "r_last", "r_prev"):
        out[k] = np.zeros(shot.shape)
    ph_, rh_ = None, None
    if want_history:
        ph_ = out["p_hist"] = np.zeros((shot.nt,) + tuple(shot.shape))
        rh_ = out["r_hist"] = np.zeros((shot.nt,) + tuple(shot.shape))
    st = lib().or_tti_forward(n, _f64(shot.spacing), _f64(shot.origin), shot.space_order,
                              shot.nbl, float(shot.dt), shot.nt, vp, eps, dl, th, ph,
                              float(vmax_damp), sx.shape[0], sx, wav, rx.shape[0], rx,
                              _ptr(out["traces"]), _ptr(out["p_last"]), _ptr(out["p_prev"]),
                              _ptr(out["r_last"]), _ptr(out["r_prev"]), _ptr(ph_), _ptr(rh_))
    _check(st, "tti_forward")
    return out


def tti_adjoint(shot, res: np.ndarray, vmax_damp: float = 0.0, vp=None, hist=None):
    """Adjoint of the TTI map q -> d driven by ``res[nt][nrec]``; returns
    qhat[nt][nsrc], or (qhat, grad) when ``hist`` = (p_hist, r_hist) of the
    forward is given (grad of 1/2 |P_r p - dobs|^2 w.r.t. m = 1/vp^2 for
    res = P_r p - dobs)."""
    n = np.asarray(shot.shape, dtype=np.int32)
    sx = _f64(shot.src_xyz)
    rx = _f64(shot.rec_xyz)
    qhat = np.zeros((shot.nt, sx.shape[0]))
    grad = np.zeros(shot.shape) if hist is not None else None
    ph_, rh_ = (None, None) if hist is None else (_f64(hist[0]), _f64(hist[1]))
    st = lib().or_tti_adjoint(n, _f64(shot.spacing), _f64(shot.origin), shot.space_order,
                              shot.nbl, float(shot.dt), shot.nt, _f64(shot.vp if vp is None else vp),
                              _f64(shot.epsilon), _f64(shot.delta), _f64(shot.theta),
                              _f64(shot.phi), float(vmax_damp), sx.shape[0], sx,
                              _ptr(_f64(shot.src_wav)), rx.shape[0], rx, _f64(res), _ptr(ph_),
                              _ptr(rh_), _ptr(grad), _ptr(qhat))
    _check(st, "tti_adjoint")
    return qhat if hist is None else (qhat, grad)


def tti_gradient(shot, dobs: np.ndarray, vp=None, vmax_damp: float = 0.0):
    """J(m) and dJ/dm (m = 1/vp^2) of the TTI propagator for
    J = 1/2 sum_k |P_r p^k - dobs^k|^2."""
    fw = tti_forward(shot, vp=vp, vmax_damp=vmax_damp, want_history=True)
    res = fw["traces"] - _f64(dobs)
    J = 0.5 * float(np.sum(res * res))
    _, g = tti_adjoint(shot, res, vmax_damp=vmax_damp, vp=vp, hist=(fw["p_hist"], fw["r_hist"]))
    return J, g


def tti_operators(u, spacing, so: int, theta, phi):
    """(L u, Hz u) of the TTI oracle for a field u with per-node angles."""
    u = _f64(u)
    n = np.asarray(u.shape, dtype=np.int32)
    lap_out = np.zeros(u.shape)
    hz = np.zeros(u.shape)
    _check(lib().or_tti_operators(n, _f64(spacing), so, _f64(np.broadcast_to(theta, u.shape)),
                                  _f64(np.broadcast_to(phi, u.shape)), u, _ptr(lap_out),
                                  _ptr(hz)), "tti_operators")
    return lap_out, hz


ELASTIC_FIELDS = ("vx", "vy", "vz", "txx", "tyy", "tzz", "txy", "txz", "tyz")


def elastic_adjoint(shot, res: np.ndarray, vmax_damp: float = 0.0, vp=None, vs=None, rho=None,
                    hist=None):
    """Adjoint of the elastic map q -> (vz, P) traces driven by
    ``res[2][nt][nrec]`` (vz block, then P); returns qhat[nt][nsrc], or
    (qhat, grad[3][...]) w.r.t. (lambda, mu, b = 1/rho) when the forward
    history ``hist`` is given and res = traces - dobs."""
    n = np.asarray(shot.shape, dtype=np.int32)
    f = lambda a, b: _f64(b if a is None else a)
    sx = _f64(shot.src_xyz)
    rx = _f64(shot.rec_xyz)
    qhat = np.zeros((shot.nt, sx.shape[0]))
    grad = np.zeros((3,) + tuple(shot.shape)) if hist is not None else None
    st = lib().or_elastic_adjoint(n, _f64(shot.spacing), _f64(shot.origin), shot.space_order,
                                  shot.nbl, float(shot.dt), shot.nt, f(vp, shot.vp),
                                  f(vs, shot.vs), f(rho, shot.rho), float(vmax_damp),
                                  sx.shape[0], sx, rx.shape[0], rx, _f64(res),
                                  _ptr(None if hist is None else _f64(hist)), _ptr(grad),
                                  _ptr(qhat))
    _check(st, "elastic_adjoint")
    return qhat if hist is None else (qhat, grad)


def elastic_gradient(shot, dobs: np.ndarray, vmax_damp: float = 0.0, vp=None, vs=None, rho=None):
    """J and dJ/d(lambda, mu, b) [3][...] of J = 1/2 |traces - dobs|^2 for
    the elastic propagator (traces [2][nt][nrec]: vz, then P)."""
    fw = elastic_forward(shot, vmax_damp=vmax_damp, vp=vp, vs=vs, rho=rho, want_history=True)
    res = np.stack([fw["vz"], fw["p"]]) - _f64(dobs)
    J = 0.5 * float(np.sum(res * res))
    _, g = elastic_adjoint(shot, res, vmax_damp=vmax_damp, vp=vp, vs=vs, rho=rho,
                           hist=fw["hist"])
    return J, g


def elastic_forward(shot, vmax_damp: float = 0.0, src_wav=None, vp=None, vs=None, rho=None,
                    want_energy: bool = False, want_history: bool = False):
    """FP64 elastic velocity-stress forward of a ``workloads.Shot`` (zero
    initial state). Returns dict(vz[nt][nrec], p[nt][nrec] traces, the nine
    final fields by name (vz as "vz_field"), energy[nt] if asked)."""
    n = np.asarray(shot.shape, dtype=np.int32)
    f = lambda a, b: _f64(b if a is None else a)
    vp, vs, rho = f(vp, shot.vp), f(vs, shot.vs), f(rho, shot.rho)
    wav = f(src_wav, shot.src_wav)
    sx = _f64(shot.src_xyz)
    rx = _f64(shot.rec_xyz)
    nrec = rx.shape[0]
    traces = np.zeros((2, shot.nt, nrec))
    state = np.zeros((9,) + tuple(shot.shape))
    energy = np.zeros(shot.nt) if want_energy else None
    hist = np.zeros((shot.nt, 9) + tuple(shot.shape)) if want_history else None
    st = lib().or_elastic_forward(n, _f64(shot.spacing), _f64(shot.origin), shot.space_order,
                                  shot.nbl, float(shot.dt), shot.nt, vp, vs, rho,
                                  float(vmax_damp), sx.shape[0], sx, wav, nrec, rx,
                                  _ptr(traces), _ptr(state), _ptr(energy), _ptr(hist))
    _check(st, "elastic_forward")
    out = {k if k != "vz" else "vz_field": state[i] for i, k in enumerate(ELASTIC_FIELDS)}
    out.update(vz=traces[0], p=traces[1])
    if want_energy:
        out["energy"] = energy
    if want_history:
        out["hist"] = hist
    return out


def elastic_passes(state, spacing, so: int, dt: float, vp, vs, rho, which: int = 3,
                   nbl: int = 0, vmax_damp: float = 0.0) -> np.ndarray:
    """Apply one velocity pass (which & 1) and/or one stress pass (which & 2)
    of the elastic oracle to ``state[9][...]`` (vx vy vz txx tyy tzz txy txz
    tyz); returns the new state."""
    F = np.array(state, dtype=np.float64, order="C", copy=True)
    shape = F.shape[1:]
    b = lambda a: _f64(np.broadcast_to(a, shape))
    _check(lib().or_elastic_passes(np.asarray(shape, dtype=np.int32), _f64(spacing), so, int(nbl),
                                   float(dt), b(vp), b(vs), b(rho), float(vmax_damp), int(which),
                                   F), "elastic_passes")
    return F


def misfit(d, dobs) -> float:
    d = _f64(d)
    dobs = _f64(dobs)
    return float(lib().or_misfit(d.shape[0], d.shape[1], d, dobs, None))
