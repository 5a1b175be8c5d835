"""ctypes declarations of include/treepm.h and the argument marshalling for each call."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtreepm.so")

TREEPM_OK, TREEPM_PENDING = 0, 1
TREEPM_FP32, TREEPM_FP64 = 0, 1
TREEPM_HOST, TREEPM_DEVICE = 0, 1
TREEPM_OPEN_FIXED, TREEPM_OPEN_DISTANCE = 0, 1
TREEPM_WALK_AUTO, TREEPM_WALK_ONE_PASS, TREEPM_WALK_TWO_PASS = 0, 1, 2

ERROR_NAMES = {
    -1: "TREEPM_ERR_ARG", -2: "TREEPM_ERR_RANGE", -3: "TREEPM_ERR_OOM",
    -4: "TREEPM_ERR_DEVICE", -5: "TREEPM_ERR_STATE", -6: "TREEPM_ERR_QUEUE_FULL",
    -7: "TREEPM_ERR_OVERFLOW",
}


class TreePMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class treepm_params(C.Structure):
    _fields_ = [("L", C.c_double), ("mesh", C.c_double), ("r_cut", C.c_double),
                ("eps", C.c_double), ("theta", C.c_double), ("n_leaf", C.c_int32),
                ("n_crit", C.c_int32), ("precision", C.c_int32), ("opening", C.c_int32),
                ("theta_max", C.c_double), ("quadrupole", C.c_int32)]


class treepm_stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_nodes", C.c_int64), ("n_groups", C.c_int64),
                ("n_cell_entries", C.c_int64), ("n_part_entries", C.c_int64),
                ("interactions", C.c_int64), ("max_level", C.c_int32),
                ("max_group", C.c_int32), ("t_ms", C.c_double * 4), ("evaluated", C.c_int64),
                ("latency_ms", C.c_double), ("queue_ms", C.c_double),
                ("stage_ms", C.c_double * 3), ("batch_boxes", C.c_int32), ("reserved_", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_
             if k not in ("t_ms", "stage_ms", "reserved_")}
        d["t_ms"] = list(self.t_ms)
        d["stage_ms"] = list(self.stage_ms)
        return d


_lib = None
_p = C.c_void_p
_i = C.c_int
_i64 = C.c_int64

_SIGS = {
    "treepm_version": (C.c_char_p, []),
    "treepm_create": (_i, [C.POINTER(treepm_params), _i, C.POINTER(_p)]),
    "treepm_destroy": (_i, [_p]),
    "treepm_release_cached": (_i, [_i]),
    "treepm_set_params": (_i, [_p, C.POINTER(treepm_params)]),
    "treepm_set_timing": (_i, [_p, _i]),
    "treepm_set_walk_passes": (_i, [_p, _i]),
    "treepm_build": (_i, [_p, _i64, _p, _p, _p, _p, _i, _p]),
    "treepm_walk": (_i, [_p, _p, C.POINTER(treepm_stats)]),
    "treepm_force_short": (_i, [_p, _p, _p, _p, _i, _i, _p]),
    "treepm_force_short_batch": (_i, [_p, _i, _p, _p, _p, _i, _p]),
    "treepm_force_long": (_i, [_p, _p, _p, _p, _i, _i, _i, _p]),
    "treepm_eps_of_z": (C.c_double, [C.c_double, C.c_double, C.c_double]),
    "treepm_timestep": (_i, [_p, _i64, _p, _p, _p, _p, _p, _p, _i, C.c_double, C.c_double, _p,
                             C.POINTER(C.c_double)]),
    "treepm_timestep_noalloc": (_i, [_p, _i64, _p, _p, _p, _p, _p, _p, _i, C.c_double,
                                     C.c_double, _p, C.POINTER(C.c_double)]),
    "treepm_kick_short": (_i, [_p, _p, _p, _p, C.c_double, _p]),
    "treepm_kick_drift": (_i, [_p, _i64, _p, _p, _p, _p, _p, _p, _p, _p, _p, _i, C.c_double,
                               C.c_double, _p]),
    "treepm_get_stats": (_i, [_p, C.POINTER(treepm_stats)]),
    "treepm_export_sorted": (_i, [_p, _p, _p]),
    "treepm_export_nodes": (_i, [_p, _i64, _p, _p, _p, _p, _p, _p]),
    "treepm_export_groups": (_i, [_p, _i64, _p, _p, _p, _p, _p, _p]),
    "treepm_export_lists": (_i, [_p, _i64, _i64, _p, _p, _p]),
    "treepm_last_error": (C.c_char_p, [_p]),
    "treepm_pairwise_f32": (_i, [C.POINTER(treepm_params), _i, _i64, _p, _i64, _p, _p, _p, _p]),
    "treepm_autotune": (_i, [_p, _i64, _p, _p, _p, _p, _i, _p, _p, C.c_int32, _p, _p]),
    "treepm_ens_create": (_i, [_i, C.c_size_t, _i, C.POINTER(_p)]),
    "treepm_ens_destroy": (_i, [_p]),
    "treepm_ens_set_batching": (_i, [_p, _i]),
    "treepm_ensemble_submit": (_i, [_p, C.c_uint64, C.POINTER(treepm_params), _i64, _p, _p, _p,
                                    _p, C.POINTER(C.c_uint64)]),
    "treepm_ensemble_poll": (_i, [_p, C.c_uint64, _p, _p, _p, C.POINTER(treepm_stats)]),
    "treepm_ens_info": (_i, [_p, _p, _p, _p, _p]),
}


def lib():
    """Load libtreepm.so (built by paper_0910_0121_amd/build.py); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -m paper_0910_0121_amd.build` "
                "(the tree force has no non-HIP implementation)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def treepm_version() -> str:
    return lib().treepm_version().decode()


def treepm_last_error(ctx) -> str:
    return lib().treepm_last_error(ctx).decode()


def _check(rc: int, ctx=None):
    if rc < 0:
        msg = treepm_last_error(ctx) if ctx else ""
        raise TreePMError(rc, msg)
    return rc


def make_params(L=1.0, mesh=None, r_cut=None, eps=0.0, theta=0.5, n_leaf=10, n_crit=0,
                precision=TREEPM_FP32, opening=TREEPM_OPEN_FIXED,
                theta_max=0.0, quadrupole=0) -> treepm_params:
    """opening=TREEPM_OPEN_DISTANCE selects theta(d) of eq. (12): theta is then theta_0 and
    theta_max its cap.  quadrupole=1 adds the cells' second-order terms."""
    if mesh is None and r_cut is None:
        raise ValueError("give mesh or r_cut")
    if mesh is None:
        mesh = r_cut / 3.0
    if r_cut is None:
        r_cut = 3.0 * mesh
    return treepm_params(L, mesh, r_cut, eps, theta, n_leaf, n_crit, precision, opening,
                         theta_max, quadrupole)


# ----------------------------------------------------------------------------- buffers

def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _buf(a, dtype_name):
    """(pointer, mem_kind, keepalive) for a torch tensor or numpy array."""
    if _is_torch(a):
        if not a.is_contiguous():
            raise ValueError("buffers must be contiguous")
        if str(a.dtype) != "torch." + dtype_name:
            raise TypeError(f"expected torch.{dtype_name}, got {a.dtype}")
        kind = TREEPM_DEVICE if a.is_cuda else TREEPM_HOST
        return a.data_ptr(), kind, a
    arr = np.asarray(a)
    if arr.dtype != np.dtype(dtype_name) or not arr.flags.c_contiguous:
        raise TypeError(f"expected a contiguous numpy {dtype_name} array")
    return arr.ctypes.data, TREEPM_HOST, arr


def _stream(stream, kind):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    if kind == TREEPM_DEVICE:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return 0


# ----------------------------------------------------------------------------- entry points

def treepm_create(params: treepm_params, device: int = 0):
    h = C.c_void_p()
    _check(lib().treepm_create(C.byref(params), device, C.byref(h)))
    return h.value


def treepm_destroy(ctx) -> None:
    _check(lib().treepm_destroy(ctx))


def treepm_release_cached(device: int = 0) -> None:
    _check(lib().treepm_release_cached(device))


def treepm_set_params(ctx, params: treepm_params) -> None:
    _check(lib().treepm_set_params(ctx, C.byref(params)), ctx)


def treepm_set_timing(ctx, enable: bool) -> None:
    _check(lib().treepm_set_timing(ctx, int(bool(enable))), ctx)


def treepm_set_walk_passes(ctx, mode: int) -> None:
    _check(lib().treepm_set_walk_passes(ctx, int(mode)), ctx)


def treepm_build(ctx, x, y, z, m, stream=None) -> None:
    bufs = [_buf(a, "float64") for a in (x, y, z, m)]
    kinds = {b[1] for b in bufs}
    if len(kinds) != 1:
        raise ValueError("x, y, z, m must all be host or all be device buffers")
    kind = kinds.pop()
    n = len(bufs[0][2])
    _check(lib().treepm_build(ctx, n, bufs[0][0], bufs[1][0], bufs[2][0], bufs[3][0], kind,
                              _stream(stream, kind)), ctx)


def treepm_walk(ctx, stream=None) -> treepm_stats:
    st = treepm_stats()
    _check(lib().treepm_walk(ctx, _stream(stream, TREEPM_DEVICE), C.byref(st)), ctx)
    return st


def treepm_force_short(ctx, ax, ay, az, stream=None) -> None:
    dt = "float64" if (str(getattr(ax, "dtype", "")) in ("torch.float64", "float64")) else "float32"
    bufs = [_buf(a, dt) for a in (ax, ay, az)]
    kinds = {b[1] for b in bufs}
    if len(kinds) != 1:
        raise ValueError("ax, ay, az must all be host or all be device buffers")
    kind = kinds.pop()
    prec = TREEPM_FP64 if dt == "float64" else TREEPM_FP32
    _check(lib().treepm_force_short(ctx, bufs[0][0], bufs[1][0], bufs[2][0], prec, kind,
                                    _stream(stream, kind)), ctx)


def treepm_force_short_batch(ctxs, outs, stream=None) -> None:
    """Walk and FP32 short-range force of several built boxes with shared launches.  outs[b]
    is box b's (ax, ay, az), float32, all host or all device buffers."""
    nb = len(ctxs)
    if nb != len(outs):
        raise ValueError("one (ax, ay, az) per box")
    bufs = [[_buf(a, "float32") for a in o] for o in outs]
    kinds = {b[1] for bb in bufs for b in bb}
    if len(kinds) != 1:
        raise ValueError("all outputs must be host or all device buffers")
    kind = kinds.pop()
    arr = C.c_void_p * max(nb, 1)
    cs = arr(*ctxs)
    ax, ay, az = (arr(*[bb[a][0] for bb in bufs]) for a in range(3))
    rc = lib().treepm_force_short_batch(cs, nb, ax, ay, az, kind, _stream(stream, kind))
    if rc < 0:
        msgs = [treepm_last_error(c) for c in ctxs if c]
        named = [m for m in msgs if m and m != "another box of the batch failed"]
        raise TreePMError(rc, named[0] if named else (msgs[0] if msgs else ""))


def treepm_force_long(ctx, ax, ay, az, accumulate=False, stream=None) -> None:
    dt = "float64" if (str(getattr(ax, "dtype", "")) in ("torch.float64", "float64")) else "float32"
    bufs = [_buf(a, dt) for a in (ax, ay, az)]
    kinds = {b[1] for b in bufs}
    if len(kinds) != 1:
        raise ValueError("ax, ay, az must all be host or all be device buffers")
    kind = kinds.pop()
    prec = TREEPM_FP64 if dt == "float64" else TREEPM_FP32
    _check(lib().treepm_force_long(ctx, bufs[0][0], bufs[1][0], bufs[2][0], prec, kind,
                                   1 if accumulate else 0, _stream(stream, kind)), ctx)


def treepm_eps_of_z(z, eps_fin, z_crit) -> float:
    return float(lib().treepm_eps_of_z(z, eps_fin, z_crit))


def _dev_ptrs(arrs, dtypes):
    out = []
    for a, dt in zip(arrs, dtypes):
        p, kind, _ = _buf(a, dt)
        if kind != TREEPM_DEVICE:
            raise ValueError("time-stepping calls take device tensors")
        out.append(p)
    return out


def treepm_timestep(ctx, vx, vy, vz, ax, ay, az, eps, zeta, stream=None) -> float:
    """Shared step of eq. (7) from device velocities (float64) and accelerations."""
    adt = "float64" if str(ax.dtype) == "torch.float64" else "float32"
    ptr = _dev_ptrs((vx, vy, vz, ax, ay, az), ("float64",) * 3 + (adt,) * 3)
    dt = C.c_double()
    _check(lib().treepm_timestep(ctx, vx.shape[0], *ptr,
                                 TREEPM_FP64 if adt == "float64" else TREEPM_FP32, eps, zeta,
                                 _stream(stream, TREEPM_DEVICE), C.byref(dt)), ctx)
    return dt.value


def treepm_timestep_noalloc(ctx, vx, vy, vz, ax, ay, az, eps, zeta, stream=None) -> float:
    """treepm_timestep without any device allocation (static scratch in the library)."""
    adt = "float64" if str(ax.dtype) == "torch.float64" else "float32"
    ptr = _dev_ptrs((vx, vy, vz, ax, ay, az), ("float64",) * 3 + (adt,) * 3)
    dt = C.c_double()
    _check(lib().treepm_timestep_noalloc(ctx, vx.shape[0], *ptr,
                                         TREEPM_FP64 if adt == "float64" else TREEPM_FP32, eps,
                                         zeta, _stream(stream, TREEPM_DEVICE), C.byref(dt)), ctx)
    return dt.value


def treepm_kick_short(ctx, vx, vy, vz, dt, stream=None) -> None:
    """In place on device float64 tensors: v += dt a_short (the kick fused with the force)."""
    ptr = _dev_ptrs((vx, vy, vz), ("float64",) * 3)
    _check(lib().treepm_kick_short(ctx, *ptr, dt, _stream(stream, TREEPM_DEVICE)), ctx)


def treepm_kick_drift(ctx, x, y, z, vx, vy, vz, ax, ay, az, dt_kick, dt_drift,
                      stream=None) -> None:
    """In place on device tensors: v += a dt_kick, x += v dt_drift (wrapped into [0, L))."""
    adt = "float64" if str(ax.dtype) == "torch.float64" else "float32"
    ptr = _dev_ptrs((x, y, z, vx, vy, vz, ax, ay, az), ("float64",) * 6 + (adt,) * 3)
    _check(lib().treepm_kick_drift(ctx, x.shape[0], *ptr,
                                   TREEPM_FP64 if adt == "float64" else TREEPM_FP32, dt_kick,
                                   dt_drift, _stream(stream, TREEPM_DEVICE)), ctx)


def treepm_autotune(ctx, x, y, z, m, candidates, stream=None):
    """Returns (best n_crit, its build+walk+force time in ms); the context keeps the winner."""
    bufs = [_buf(a, "float64") for a in (x, y, z, m)]
    kinds = {b[1] for b in bufs}
    if len(kinds) != 1:
        raise ValueError("x, y, z, m must all be host or all be device buffers")
    kind = kinds.pop()
    cand = np.ascontiguousarray(candidates, dtype=np.int32)
    best = C.c_int32()
    ms = C.c_double()
    _check(lib().treepm_autotune(ctx, len(bufs[0][2]), bufs[0][0], bufs[1][0], bufs[2][0],
                                 bufs[3][0], kind, _stream(stream, kind), cand.ctypes.data,
                                 cand.size, C.byref(best), C.byref(ms)), ctx)
    return best.value, ms.value


def treepm_get_stats(ctx) -> treepm_stats:
    st = treepm_stats()
    _check(lib().treepm_get_stats(ctx, C.byref(st)), ctx)
    return st


def treepm_export_sorted(ctx):
    n = treepm_get_stats(ctx).n
    keys = np.zeros(n, dtype=np.uint64)
    idx = np.zeros(n, dtype=np.int64)
    _check(lib().treepm_export_sorted(ctx, keys.ctypes.data, idx.ctypes.data), ctx)
    return keys, idx


def treepm_export_nodes(ctx):
    nn = treepm_get_stats(ctx).n_nodes
    code = np.zeros(nn, dtype=np.uint64)
    first = np.zeros(nn, dtype=np.int64)
    count = np.zeros(nn, dtype=np.int64)
    nchild = np.zeros(nn, dtype=np.int32)
    mass = np.zeros(nn)
    com = np.zeros((nn, 3))
    _check(lib().treepm_export_nodes(ctx, nn, code.ctypes.data, first.ctypes.data,
                                     count.ctypes.data, nchild.ctypes.data, mass.ctypes.data,
                                     com.ctypes.data), ctx)
    return dict(code=code, first=first, count=count, nchild=nchild, mass=mass, com=com)


def treepm_export_groups(ctx):
    ng = treepm_get_stats(ctx).n_groups
    code = np.zeros(ng, dtype=np.uint64)
    first = np.zeros(ng, dtype=np.int64)
    count = np.zeros(ng, dtype=np.int64)
    lo, hi, xg = (np.zeros((ng, 3)) for _ in range(3))
    _check(lib().treepm_export_groups(ctx, ng, code.ctypes.data, first.ctypes.data,
                                      count.ctypes.data, lo.ctypes.data, hi.ctypes.data,
                                      xg.ctypes.data), ctx)
    return dict(code=code, first=first, count=count, lo=lo, hi=hi, xg=xg)


def treepm_export_lists(ctx):
    st = treepm_get_stats(ctx)
    ne = st.n_cell_entries + st.n_part_entries
    off = np.zeros(st.n_groups + 1, dtype=np.int64)
    isc = np.zeros(max(ne, 1), dtype=np.uint8)
    val = np.zeros(max(ne, 1), dtype=np.uint64)
    _check(lib().treepm_export_lists(ctx, st.n_groups + 1, max(ne, 1), off.ctypes.data,
                                     isc.ctypes.data, val.ctypes.data), ctx)
    return off, isc[:ne], val[:ne]


def treepm_pairwise_f32(params: treepm_params, xi, xj, mj, xg, device: int = 0):
    """Per-pair FP32 accelerations, shape (n_i, n_j, 3)."""
    xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1, 3)
    xj = np.ascontiguousarray(xj, dtype=np.float64).reshape(-1, 3)
    mj = np.ascontiguousarray(mj, dtype=np.float64).reshape(-1)
    xg = np.ascontiguousarray(xg, dtype=np.float64).reshape(3)
    out = np.zeros((xi.shape[0], xj.shape[0], 3))
    _check(lib().treepm_pairwise_f32(C.byref(params), device, xi.shape[0], xi.ctypes.data,
                                     xj.shape[0], xj.ctypes.data, mj.ctypes.data, xg.ctypes.data,
                                     out.ctypes.data))
    return out


# ----------------------------------------------------------------------------- ensemble

def treepm_ens_create(device: int = 0, hbm_budget: int = 8 << 30, max_inflight: int = 4):
    h = C.c_void_p()
    _check(lib().treepm_ens_create(device, hbm_budget, max_inflight, C.byref(h)))
    return h.value


def treepm_ens_destroy(ens) -> None:
    _check(lib().treepm_ens_destroy(ens))


def treepm_ensemble_submit(ens, box_id: int, params: treepm_params, x, y, z, m) -> int:
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, z, m)]
    t = C.c_uint64()
    _check(lib().treepm_ensemble_submit(ens, box_id, C.byref(params), arrs[0].size,
                                        *(a.ctypes.data for a in arrs), C.byref(t)))
    return t.value


def treepm_ensemble_poll(ens, ticket: int, ax=None, ay=None, az=None):
    """(TREEPM_OK, stats) when done (results copied into the given float32 arrays),
    (TREEPM_PENDING, None) while queued or running; raises on an error."""
    st = treepm_stats()
    ptr = [None if a is None else a.ctypes.data for a in (ax, ay, az)]
    for a in (ax, ay, az):
        if a is not None and (a.dtype != np.float32 or not a.flags.c_contiguous):
            raise TypeError("poll outputs must be contiguous float32 arrays")
    rc = lib().treepm_ensemble_poll(ens, ticket, *ptr, C.byref(st))
    if rc == TREEPM_PENDING:
        return rc, None
    _check(rc)
    return rc, st


def treepm_ens_set_batching(ens, enable: bool) -> None:
    _check(lib().treepm_ens_set_batching(ens, 1 if enable else 0))


def treepm_ens_info(ens):
    v = [C.c_int64() for _ in range(4)]
    _check(lib().treepm_ens_info(ens, *(C.byref(x) for x in v)))
    return dict(queued=v[0].value, inflight=v[1].value, resident_bytes=v[2].value,
                resident_boxes=v[3].value)
