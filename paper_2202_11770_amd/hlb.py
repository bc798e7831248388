"""Python binding of the C ABI in include/hlb.h (argument marshalling only).

Every function here has the name of the C entry point it calls and does no
computation of its own: the update, the boundary rules, the macroscopic
fields and the reductions all run in libhlb.so's gfx950 kernels.  If the
library has not been built this module raises on first use; there is no
fallback.

Arrays are numpy (host) or anything exposing a device pointer (an integer,
or an object with ``data_ptr()`` such as a torch tensor on the GPU).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libhlb.so")

HLB_OK, HLB_EINVAL, HLB_ENOMEM, HLB_EDEVICE, HLB_ESTATE, HLB_ENUMERIC = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "HLB_OK", -1: "HLB_EINVAL", -2: "HLB_ENOMEM", -3: "HLB_EDEVICE", -4: "HLB_ESTATE",
                -5: "HLB_ENUMERIC"}
HLB_F64, HLB_F32_SHIFTED, HLB_F16_SHIFTED = 0, 1, 2
STORAGE = {"f64": HLB_F64, "f32": HLB_F32_SHIFTED, "f16": HLB_F16_SHIFTED}
HLB_ORDER_INPUT, HLB_ORDER_LEX, HLB_ORDER_MORTON, HLB_ORDER_BRICK, HLB_ORDER_BANDS, HLB_ORDER_COLUMNS = range(6)
HLB_IOLET_VELOCITY, HLB_IOLET_PRESSURE = 0, 1
HLB_SCHEME_PULL, HLB_SCHEME_PUSH = 0, 1
HLB_LINK_WALL = -1
SCHEME = {"pull": HLB_SCHEME_PULL, "push": HLB_SCHEME_PUSH}
ORDER = {"input": 0, "lex": 1, "morton": 2, "brick": 3, "bands": 4, "columns": 5}
Q = 19


class HLBError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class hlb_iolet(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("role", ctypes.c_int32), ("centre", ctypes.c_double * 3),
                ("normal", ctypes.c_double * 3), ("radius", ctypes.c_double), ("vdir", ctypes.c_double * 3)]


class hlb_options(ctypes.Structure):
    _fields_ = [("storage", ctypes.c_int32), ("order", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("adjoint", ctypes.c_int32), ("rho0", ctypes.c_double), ("max_device_bytes", ctypes.c_int64),
                ("scheme", ctypes.c_int32), ("sites_per_thread", ctypes.c_int32),
                ("graph_steps", ctypes.c_int32), ("order_block", ctypes.c_int32), ("ladd_rho_local", ctypes.c_int32)]


class hlb_windkessel(ctypes.Structure):
    _fields_ = [("rho_ref", ctypes.c_double), ("R1", ctypes.c_double), ("C", ctypes.c_double),
                ("R2", ctypes.c_double), ("X0", ctypes.c_double)]


class hlb_info_t(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int64), ("n_padded", ctypes.c_int64), ("group_sites", ctypes.c_int64 * 6),
                ("storage", ctypes.c_int32), ("order", ctypes.c_int32), ("bytes_per_lup", ctypes.c_double),
                ("device_bytes", ctypes.c_int64), ("table_bytes_per_site", ctypes.c_double),
                ("n_segments", ctypes.c_int64), ("n_iolets", ctypes.c_int64), ("adjoint", ctypes.c_int32),
                ("porous", ctypes.c_int32), ("scheme", ctypes.c_int32), ("sites_per_thread", ctypes.c_int32),
                ("graph_steps", ctypes.c_int32), ("xcd_remap", ctypes.c_int32)]


class hlb_stats_t(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("kernel_ms", ctypes.c_double), ("step_ms", ctypes.c_double),
                ("adj_steps", ctypes.c_int64), ("adj_ms", ctypes.c_double), ("mlups", ctypes.c_double),
                ("alg_gbs", ctypes.c_double)]


_P = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_d = ctypes.c_double
_PP = ctypes.POINTER(ctypes.c_void_p)

# name -> argtypes (restype is the int status unless noted)
_SIGS = {
    "hlb_default_options": [ctypes.POINTER(hlb_options)],
    "hlb_create": [_i64, _P, _P, _P, _d, _P, _i32, ctypes.POINTER(hlb_options), _PP],
    "hlb_destroy": [_P],
    "hlb_set_stream": [_P, _P],
    "hlb_set_iolet_table": [_P, _i32, _P, _i64],
    "hlb_set_porosity": [_P, _P],
    "hlb_set_iolet_table_device": [_P, _i32, _P, _i64],
    "hlb_set_porosity_device": [_P, _P],
    "hlb_init_equilibrium": [_P, _P, _P, _i64],
    "hlb_step": [_P, _i64],
    "hlb_macros": [_P, _P, _P, _P],
    "hlb_macros_device": [_P, _P, _P, _P],
    "hlb_get_state": [_P, _P],
    "hlb_set_state": [_P, _P, _i64],
    "hlb_mass_balance": [_P, _P, _P],
    "hlb_mass_balance_noalloc": [_P, _P],
    "hlb_time": [_P, ctypes.POINTER(_i64)],
    "hlb_info": [_P, ctypes.POINTER(hlb_info_t)],
    "hlb_set_timing": [_P, _i32],
    "hlb_stats": [_P, ctypes.POINTER(hlb_stats_t)],
    "hlb_snapshot_alloc": [_P, _i32],
    "hlb_snapshot_save": [_P, _i32],
    "hlb_snapshot_restore": [_P, _i32],
    "hlb_state_bytes": [_P, ctypes.POINTER(_i64)],
    "hlb_state_save": [_P, _P],
    "hlb_state_load": [_P, _P],
    "hlb_sync": [_P],
    "hlb_copy_bandwidth": [_i64, _i32, ctypes.POINTER(_d)],
    "hlb_set_objective": [_P, _i32, _P],
    "hlb_set_windkessel": [_P, _i32, ctypes.POINTER(hlb_windkessel)],
    "hlb_windkessel_state": [_P, _i32, _P, _P, _P],
    "hlb_create_part": [_i64, _P, _P, _P, _d, _P, _i32, ctypes.POINTER(hlb_options), _P, _PP],
    "hlb_halo_set": [_P, _i64, _P, _P, _P, _i64, _P, _P, _P],
    "hlb_halo_pack": [_P],
    "hlb_halo_ghost_slots": [_P, _i64, _P, _P, _P, _P],
    "hlb_halo_add_peer": [_P, _i64, _P, _P, _P, _P, _P],
    "hlb_halo_clear_peers": [_P],
    "hlb_halo_unpack": [_P],
    "hlb_step_edge": [_P],
    "hlb_step_mid": [_P],
    "hlb_set_mid_stream": [_P, _P],
    "hlb_adjoint_run": [_P, _i64, _i64, _i64, _i32, _P, _P, _P, ctypes.POINTER(_i64)],
    "hlb_adjoint_run_device": [_P, _i64, _i64, _i64, _i32, _P, _P, _P, ctypes.POINTER(_i64)],
    "hlb_revolve_forward_steps": [_i64, _i32, ctypes.POINTER(_i64)],
    "hlb_last_error": [],
}
EXPORTED = tuple(_SIGS)

_lib = None


def _bind_torch_runtime():
    """One HIP runtime per process: torch ships its own libamdhip64.so.7, so
    load it (by importing torch) before libhlb.so, whose dependency of the same
    soname then resolves to it.  Device pointers and streams from torch are
    then valid in the library."""
    try:
        import torch  # noqa: F401
    except ImportError:
        return


def load():
    """Load libhlb.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    _bind_torch_runtime()
    if not os.path.exists(LIBPATH):
        raise RuntimeError(f"{LIBPATH} is missing: build it with __graft_entry__.build() "
                           "(python -m paper_2202_11770_amd.build)")
    lib = ctypes.CDLL(LIBPATH)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.hlb_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def hlb_last_error() -> str:
    return load().hlb_last_error().decode()


def _check(status: int, where: str):
    if status != HLB_OK:
        raise HLBError(status, where, hlb_last_error())


def _host(a, dtype, shape=None):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=dtype)
    if shape is not None and arr.shape != shape:
        arr = arr.reshape(shape)
    return arr, arr.ctypes.data_as(_P)


def _devptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return _P(x)
    return _P(int(x.data_ptr()))


def make_iolets(iolets):
    arr = (hlb_iolet * max(1, len(iolets)))()
    for k, io in enumerate(iolets):
        arr[k].kind = int(io.kind)
        arr[k].role = int(io.role)
        arr[k].centre[:] = [float(v) for v in io.centre]
        arr[k].normal[:] = [float(v) for v in io.normal]
        arr[k].radius = float(io.radius)
        vd = getattr(io, "vdir", None) or (0.0, 0.0, 0.0)
        arr[k].vdir[:] = [float(v) for v in vd]
    return arr


def hlb_default_options() -> hlb_options:
    o = hlb_options()
    _check(load().hlb_default_options(ctypes.byref(o)), "hlb_default_options")
    return o


def hlb_create(coords, site_type, nbr, tau: float, iolets=(), options: hlb_options | None = None):
    """Returns an opaque context handle (ctypes.c_void_p)."""
    c, cp = _host(coords, np.int32)
    t, tp = _host(site_type, np.uint8)
    nb, nbp = _host(nbr, np.int32)
    n = int(t.shape[0])
    if c.shape != (n, 3) or nb.shape != (n, Q):
        raise ValueError("coords must be (n,3) and nbr (n,19)")
    io = make_iolets(list(iolets))
    out = ctypes.c_void_p()
    opt = ctypes.byref(options) if options is not None else None
    _check(load().hlb_create(n, cp, tp, nbp, float(tau), ctypes.cast(io, _P), len(iolets), opt, ctypes.byref(out)),
           "hlb_create")
    return out


def hlb_set_windkessel(ctx, k: int, model=None):
    """model: (rho_ref, R1, C, R2, X0), or None to turn the model off."""
    w = None if model is None else ctypes.byref(hlb_windkessel(*[float(v) for v in model]))
    _check(load().hlb_set_windkessel(ctx, int(k), w), "hlb_set_windkessel")


def hlb_windkessel_state(ctx, k: int):
    """(rho the next update uses, X, outflow of the last update)."""
    r, x, q = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(load().hlb_windkessel_state(ctx, int(k), ctypes.byref(r), ctypes.byref(x), ctypes.byref(q)),
           "hlb_windkessel_state")
    return r.value, x.value, q.value


HLB_PART_MID, HLB_PART_EDGE, HLB_PART_GHOST = 0, 1, 2


def hlb_create_part(coords, site_type, nbr, tau: float, iolets, role, options: hlb_options | None = None):
    """hlb_create for one partition of a split domain; role [n] uint8 (HLB_PART_*)."""
    c, cp = _host(coords, np.int32)
    t, tp = _host(site_type, np.uint8)
    nb, nbp = _host(nbr, np.int32)
    r, rp = _host(role, np.uint8)
    n = int(t.shape[0])
    if c.shape != (n, 3) or nb.shape != (n, Q) or r.shape != (n,):
        raise ValueError("coords must be (n,3), nbr (n,19), role (n,)")
    io = make_iolets(list(iolets))
    out = ctypes.c_void_p()
    opt = ctypes.byref(options) if options is not None else None
    _check(load().hlb_create_part(n, cp, tp, nbp, float(tau), ctypes.cast(io, _P), len(iolets), opt, rp,
                                  ctypes.byref(out)), "hlb_create_part")
    return out


def hlb_halo_set(ctx, send_site, send_dir, send_buf, recv_site, recv_dir, recv_buf):
    """Halo lists (caller ids, directions) and the caller's device buffers
    (torch tensors or raw device addresses) of the storage type."""
    ss, ssp = _host(send_site, np.int32)
    sd, sdp = _host(send_dir, np.int32)
    rs, rsp = _host(recv_site, np.int32)
    rd, rdp = _host(recv_dir, np.int32)
    _check(load().hlb_halo_set(ctx, ss.size, ssp, sdp, _devptr(send_buf), rs.size, rsp, rdp, _devptr(recv_buf)),
           "hlb_halo_set")


def hlb_halo_ghost_slots(ctx, site, dirs):
    """Element index of each (ghost site, direction) slot in the partition's
    population buffers, and the two buffers' device addresses."""
    sp, spp = _host(site, np.int32)
    dp, dpp = _host(dirs, np.int32)
    elem = np.empty(sp.size, dtype=np.int64)
    bufs = (ctypes.c_void_p * 2)()
    _check(load().hlb_halo_ghost_slots(ctx, sp.size, spp, dpp, elem.ctypes.data_as(_P), bufs),
           "hlb_halo_ghost_slots")
    return elem, (bufs[0], bufs[1])


def hlb_halo_add_peer(ctx, site, dirs, peer_buf0, peer_buf1, peer_elem):
    sp, spp = _host(site, np.int32)
    dp, dpp = _host(dirs, np.int32)
    ep, epp = _host(peer_elem, np.int64)
    _check(load().hlb_halo_add_peer(ctx, sp.size, spp, dpp, _P(peer_buf0), _P(peer_buf1), epp), "hlb_halo_add_peer")


def hlb_halo_clear_peers(ctx):
    _check(load().hlb_halo_clear_peers(ctx), "hlb_halo_clear_peers")


def hlb_halo_pack(ctx):
    _check(load().hlb_halo_pack(ctx), "hlb_halo_pack")


def hlb_halo_unpack(ctx):
    _check(load().hlb_halo_unpack(ctx), "hlb_halo_unpack")


def hlb_step_edge(ctx):
    _check(load().hlb_step_edge(ctx), "hlb_step_edge")


def hlb_step_mid(ctx):
    _check(load().hlb_step_mid(ctx), "hlb_step_mid")


def hlb_set_mid_stream(ctx, stream):
    """stream: a hipStream_t as an int, or None (hlb_step_mid on the context's stream)."""
    _check(load().hlb_set_mid_stream(ctx, _P(int(stream)) if stream else None), "hlb_set_mid_stream")


def hlb_destroy(ctx):
    _check(load().hlb_destroy(ctx), "hlb_destroy")


def hlb_set_stream(ctx, stream):
    """stream: a hipStream_t as an int (e.g. torch.cuda.current_stream().cuda_stream) or None."""
    _check(load().hlb_set_stream(ctx, _P(int(stream)) if stream else None), "hlb_set_stream")


def hlb_set_iolet_table(ctx, k: int, values):
    v, vp = _host(values, np.float64)
    v = v.reshape(-1)
    _check(load().hlb_set_iolet_table(ctx, int(k), vp, v.size), "hlb_set_iolet_table")


def hlb_set_porosity(ctx, phi):
    p, pp = _host(phi, np.float64)
    _check(load().hlb_set_porosity(ctx, pp), "hlb_set_porosity")


def _dev_f64(x, n, what):
    """A contiguous FP64 CUDA tensor of n elements (checked, not converted)."""
    if not (x.is_cuda and x.dtype.is_floating_point and x.element_size() == 8 and x.is_contiguous()
            and x.numel() == n):
        raise ValueError(f"{what}: need a contiguous float64 CUDA tensor of {n} elements")
    return _P(int(x.data_ptr()))


def hlb_set_iolet_table_device(ctx, k: int, values):
    """values: contiguous float64 CUDA tensor (the table of iolet k)."""
    _check(load().hlb_set_iolet_table_device(ctx, int(k), _dev_f64(values, values.numel(), "table"),
                                             int(values.numel())), "hlb_set_iolet_table_device")


def hlb_set_porosity_device(ctx, phi):
    """phi: contiguous float64 CUDA tensor [n_sites] in caller order, or None."""
    pp = None if phi is None else _dev_f64(phi, hlb_info(ctx)["n_sites"], "porosity")
    _check(load().hlb_set_porosity_device(ctx, pp), "hlb_set_porosity_device")


def hlb_init_equilibrium(ctx, rho=None, u=None, t0: int = 0):
    r, rp = _host(rho, np.float64)
    v, vp = _host(u, np.float64)
    _check(load().hlb_init_equilibrium(ctx, rp, vp, int(t0)), "hlb_init_equilibrium")


def hlb_step(ctx, n: int):
    _check(load().hlb_step(ctx, int(n)), "hlb_step")


def hlb_info(ctx) -> dict:
    i = hlb_info_t()
    _check(load().hlb_info(ctx, ctypes.byref(i)), "hlb_info")
    return dict(n_sites=i.n_sites, n_padded=i.n_padded, group_sites=list(i.group_sites), storage=i.storage,
                order=i.order, bytes_per_lup=i.bytes_per_lup, device_bytes=i.device_bytes,
                table_bytes_per_site=i.table_bytes_per_site, n_segments=i.n_segments, n_iolets=i.n_iolets,
                adjoint=i.adjoint, porous=i.porous, scheme=i.scheme, sites_per_thread=i.sites_per_thread,
                graph_steps=i.graph_steps, xcd_remap=i.xcd_remap)


def hlb_macros(ctx, want=("rho", "u", "wss")):
    n = hlb_info(ctx)["n_sites"]
    rho = np.empty(n) if "rho" in want else None
    u = np.empty((n, 3)) if "u" in want else None
    wss = np.empty(n) if "wss" in want else None
    P = lambda a: a.ctypes.data_as(_P) if a is not None else None
    _check(load().hlb_macros(ctx, P(rho), P(u), P(wss)), "hlb_macros")
    return rho, u, wss


def hlb_macros_device(ctx, rho=None, u=None, wss=None):
    _check(load().hlb_macros_device(ctx, _devptr(rho), _devptr(u), _devptr(wss)), "hlb_macros_device")


def hlb_get_state(ctx) -> np.ndarray:
    n = hlb_info(ctx)["n_sites"]
    f = np.empty((n, Q))
    _check(load().hlb_get_state(ctx, f.ctypes.data_as(_P)), "hlb_get_state")
    return f


def hlb_set_state(ctx, f, t: int):
    a, ap = _host(f, np.float64)
    _check(load().hlb_set_state(ctx, ap, int(t)), "hlb_set_state")


def hlb_mass_balance(ctx):
    m = ctypes.c_double()
    r = ctypes.c_double()
    _check(load().hlb_mass_balance(ctx, ctypes.byref(m), ctypes.byref(r)), "hlb_mass_balance")
    return m.value, r.value


def hlb_time(ctx) -> int:
    t = ctypes.c_int64()
    _check(load().hlb_time(ctx, ctypes.byref(t)), "hlb_time")
    return t.value


def hlb_mass_balance_noalloc(ctx, out):
    """out: a contiguous float64 CUDA tensor of 2 elements, caller-allocated;
    receives (M(t), R(t)) asynchronously on the context stream.  Nothing is
    allocated by this call or by the library."""
    _check(load().hlb_mass_balance_noalloc(ctx, _dev_f64(out, 2, "out")), "hlb_mass_balance_noalloc")


def hlb_set_timing(ctx, enable: bool):
    _check(load().hlb_set_timing(ctx, 1 if enable else 0), "hlb_set_timing")


def hlb_stats(ctx) -> dict:
    s = hlb_stats_t()
    _check(load().hlb_stats(ctx, ctypes.byref(s)), "hlb_stats")
    return dict(steps=s.steps, kernel_ms=s.kernel_ms, step_ms=s.step_ms, adj_steps=s.adj_steps, adj_ms=s.adj_ms,
                mlups=s.mlups, alg_gbs=s.alg_gbs)


def hlb_snapshot_alloc(ctx, n_slots: int):
    _check(load().hlb_snapshot_alloc(ctx, int(n_slots)), "hlb_snapshot_alloc")


def hlb_snapshot_save(ctx, slot: int):
    _check(load().hlb_snapshot_save(ctx, int(slot)), "hlb_snapshot_save")


def hlb_snapshot_restore(ctx, slot: int):
    _check(load().hlb_snapshot_restore(ctx, int(slot)), "hlb_snapshot_restore")


def hlb_state_bytes(ctx) -> int:
    b = ctypes.c_int64()
    _check(load().hlb_state_bytes(ctx, ctypes.byref(b)), "hlb_state_bytes")
    return b.value


def hlb_state_save(ctx) -> bytearray:
    buf = bytearray(hlb_state_bytes(ctx))
    cbuf = (ctypes.c_char * len(buf)).from_buffer(buf)
    _check(load().hlb_state_save(ctx, ctypes.cast(cbuf, _P)), "hlb_state_save")
    return buf


def hlb_state_load(ctx, buf):
    b = bytearray(buf)
    cbuf = (ctypes.c_char * len(b)).from_buffer(b)
    _check(load().hlb_state_load(ctx, ctypes.cast(cbuf, _P)), "hlb_state_load")


def hlb_sync(ctx):
    _check(load().hlb_sync(ctx), "hlb_sync")


HLB_OBJ_WSS = 0
HLB_OBJ_IOLET_FLUX = 1


def hlb_set_objective(ctx, kind: int, weights=None):
    """Objective of hlb_adjoint_run: HLB_OBJ_WSS, or HLB_OBJ_IOLET_FLUX with
    per-iolet weights [n_iolets]."""
    w, wp = (None, None) if weights is None else _host(weights, np.float64)
    _check(load().hlb_set_objective(ctx, int(kind), wp), "hlb_set_objective")


def hlb_revolve_forward_steps(n: int, n_snap: int) -> int:
    """Forward steps hlb_adjoint_run takes for n steps with n_snap snapshots."""
    v = ctypes.c_int64()
    _check(load().hlb_revolve_forward_steps(int(n), int(n_snap), ctypes.byref(v)), "hlb_revolve_forward_steps")
    return int(v.value)


def hlb_adjoint_run(ctx, n: int, obj_t0: int, obj_t1: int, n_snap: int, want_dA=True, want_dphi=True):
    """Returns (J, dJ_dA [n_iolets][n] or None, dJ_dphi [n_sites] or None, forward_steps).
    Row k of dJ_dA: the amplitude (velocity iolet) or ghost density (pressure
    iolet) iolet k uses in each of the n updates."""
    info = hlb_info(ctx)
    nio = info["n_iolets"]
    J = np.zeros(1)
    dA = np.zeros((max(nio, 1), n)) if want_dA else None
    dphi = np.zeros(info["n_sites"]) if want_dphi else None
    fw = ctypes.c_int64()
    P = lambda a: a.ctypes.data_as(_P) if a is not None else None
    _check(load().hlb_adjoint_run(ctx, int(n), int(obj_t0), int(obj_t1), int(n_snap), P(J), P(dA), P(dphi),
                                  ctypes.byref(fw)), "hlb_adjoint_run")
    if dA is not None:
        dA = dA[:nio]
    return float(J[0]), dA, dphi, fw.value


def hlb_adjoint_run_device(ctx, n: int, obj_t0: int, obj_t1: int, n_snap: int, J, dJ_dA=None, dJ_dphi=None) -> int:
    """Device outputs (contiguous float64 CUDA tensors): J [1], dJ_dA
    [n_iolets, n] or None, dJ_dphi [n_sites] or None, written asynchronously
    on the context stream.  Returns the forward steps taken."""
    info = hlb_info(ctx)
    fw = ctypes.c_int64()
    pJ = _dev_f64(J, 1, "J")
    pA = None if dJ_dA is None or info["n_iolets"] == 0 else _dev_f64(dJ_dA, info["n_iolets"] * int(n), "dJ_dA")
    pphi = None if dJ_dphi is None else _dev_f64(dJ_dphi, info["n_sites"], "dJ_dphi")
    _check(load().hlb_adjoint_run_device(ctx, int(n), int(obj_t0), int(obj_t1), int(n_snap), pJ, pA, pphi,
                                         ctypes.byref(fw)), "hlb_adjoint_run_device")
    return fw.value


def hlb_copy_bandwidth(nbytes: int = 4 << 30, reps: int = 20) -> float:
    g = ctypes.c_double()
    _check(load().hlb_copy_bandwidth(int(nbytes), int(reps), ctypes.byref(g)), "hlb_copy_bandwidth")
    return g.value


# ---------------------------------------------------------------------------

@dataclass
class Simulation:
    """Owning wrapper of one context built from a geometry-like object
    (``coords``, ``types``, ``nbr``, ``iolets`` with optional ``table``)."""

    ctx: ctypes.c_void_p
    n: int
    iolet_kinds: list = None

    @classmethod
    def create(cls, geom, tau: float, storage: str = "f64", order: str | None = None, xcd_remap: int = -1,
               rho0: float = 1.0, max_device_bytes: int = 0, tables=None, adjoint: bool = False,
               scheme: str = "pull", sites_per_thread: int = 0, graph_steps: int = 0, order_block: int = 0,
               ladd_rho_local: bool = False):
        """order: the site order (None: the library's default); order_block:
        log2 of the band / column width of the "bands" and "columns" orders
        (0: the library's default)."""
        opt = hlb_default_options()
        if order_block:
            opt.order_block = int(order_block)
        opt.ladd_rho_local = 1 if ladd_rho_local else 0
        opt.scheme = SCHEME[scheme]
        opt.sites_per_thread = int(sites_per_thread)
        opt.graph_steps = int(graph_steps)
        opt.storage = STORAGE[storage]
        if order is not None:
            opt.order = ORDER[order]
        opt.xcd_remap = int(xcd_remap)
        opt.rho0 = float(rho0)
        opt.max_device_bytes = int(max_device_bytes)
        opt.adjoint = 1 if adjoint else 0
        ctx = hlb_create(geom.coords, geom.types, geom.nbr, tau, geom.iolets, opt)
        sim = cls(ctx, int(geom.types.shape[0]))
        sim.iolet_kinds = [int(io.kind) for io in geom.iolets]
        for k, io in enumerate(geom.iolets):
            tab = tables[k] if tables is not None and tables[k] is not None else getattr(io, "table", None)
            if tab is not None:
                hlb_set_iolet_table(ctx, k, tab)
        return sim

    def close(self):
        if self.ctx:
            hlb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        hlb_step(self.ctx, n)

    def macros(self):
        return hlb_macros(self.ctx)

    def state(self):
        return hlb_get_state(self.ctx)

    @property
    def t(self) -> int:
        return hlb_time(self.ctx)

    def info(self) -> dict:
        return hlb_info(self.ctx)
