"""ctypes binding of libsfrom (include/sfrom.h), function for function.

Argument marshalling only: numpy arrays become host pointers, torch tensors
on the GPU become device pointers; every computation happens in the
library's HIP kernels. Importing this module raises if the library has not
been built (``python -m paper_1604_06750_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SFROM_LIBRARY selects another build of the same library (the host-
# sanitized one of build.build_sanitized, for instance)
LIB_PATH = os.environ.get("SFROM_LIBRARY") or os.path.join(_HERE, "libsfrom.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_1604_06750_amd.build`")
_lib = C.CDLL(LIB_PATH)

SFROM_F64, SFROM_F32, SFROM_BF16 = 0, 1, 2
CELL_VARIANTS = 6          # cell-phase kernel variants 0..5 (4: the scalar kernel)

STATUS = {
    0: "OK", -1: "EINVAL", -2: "ENOTSYM", -3: "ENOTNSD", -4: "EBPOS", -5: "ESUPPORT",
    -6: "EBREAKDOWN", -7: "ENOTSPD", -8: "ECFL", -9: "ENONFINITE", -10: "EDEVICE",
    -11: "ESTATE", -12: "ENOMEM", -13: "ESPLIT",
}


class SfromError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class sfrom_build_opts(C.Structure):
    _fields_ = [("m", C.c_int32), ("m_per_cell", C.POINTER(C.c_int32)), ("shift", C.c_double),
                ("online_prec", C.c_int32), ("cells_per_batch", C.c_int32)]


class sfrom_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("n_cells", C.c_int32), ("n_pieces", C.c_int32),
                ("n_piece_dofs", C.c_int64), ("n_hidden_dofs", C.c_int64), ("max_b", C.c_int32),
                ("max_m", C.c_int32), ("n_sources", C.c_int32), ("n_receivers", C.c_int32),
                ("built", C.c_int32), ("online_prec", C.c_int32), ("block_bytes", C.c_int64),
                ("build_ms", C.c_double), ("cell_variant", C.c_int32), ("steps_done", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = C.c_void_p
_SIGS = {
    "sfrom_create": [C.POINTER(_P), C.c_int, _P],
    "sfrom_destroy": [_P],
    "sfrom_last_error": [_P],
    "sfrom_set_pencil": [_P, C.c_int64, _P, _P, _P, _P],
    "sfrom_add_cell": [_P, C.c_int32, C.c_int32, _P, _P, _P, _P, _P],
    "sfrom_add_piece": [_P, C.c_int32, C.c_int32, _P, C.c_int32, _P],
    "sfrom_setup_voxel_acoustic": [_P, _P, _P, _P, _P, _P, C.c_int32, C.c_int32],
    "sfrom_setup_voxel_elastic": [_P, _P, _P, _P, _P, _P, C.c_int32, C.c_int32],
    "sfrom_setup_voxel_acoustic_rules": [_P, _P, _P, _P, _P, _P, C.c_int32, _P, _P, C.c_int32],
    "sfrom_partition_graph": [_P, C.c_int32, C.c_double, C.c_double],
    "sfrom_set_breakdown_policy": [_P, C.c_int32],
    "sfrom_gramian_bases": [_P, C.c_double, C.c_double, C.c_int32, C.c_int32],
    "sfrom_gramian_bases_zolotarev": [_P, C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_int32, C.c_double],
    "sfrom_remove_corner_set": [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int64)],
    "sfrom_corner_map": [_P, _P, _P, _P, _P, _P],
    "sfrom_set_corner_correction": [_P, C.c_int32],
    "sfrom_set_persistent": [_P, C.c_int32],
    "sfrom_build": [_P, C.POINTER(sfrom_build_opts)],
    "sfrom_import_rom": [_P, C.c_int32, C.c_int32, C.c_int32, _P, _P],
    "sfrom_export_rom": [_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), _P, _P],
    "sfrom_set_sources": [_P, C.c_int32, _P, _P, _P, C.c_int32],
    "sfrom_set_receivers": [_P, C.c_int32, _P, _P, _P, C.c_int32],
    "sfrom_point_columns": [_P, C.c_int32, _P, _P, _P, _P],
    "sfrom_reset": [_P],
    "sfrom_save": [_P, C.c_char_p],
    "sfrom_load": [_P, C.c_char_p],
    "sfrom_run": [_P, C.c_int64, C.c_double, _P, C.c_int32, _P, C.c_int32],
    "sfrom_run_noalloc": [_P, C.c_int64, C.c_double, _P, _P],
    "sfrom_fine_reset": [_P],
    "sfrom_fine_run": [_P, C.c_int64, C.c_double, _P, C.c_int32, _P, C.c_int32, C.c_int32],
    "sfrom_fine_lambda_max": [_P, C.POINTER(C.c_double)],
    "sfrom_rom_lambda_max": [_P, C.POINTER(C.c_double)],
    "sfrom_get_info": [_P, C.POINTER(sfrom_info)],
    "sfrom_set_graph": [_P, C.c_int32],
    "sfrom_set_cell_variant": [_P, C.c_int32],
    "sfrom_set_build_path": [_P, C.c_int32],
    "sfrom_profile": [_P, C.c_int32],
    "sfrom_profile_read": [_P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)],
    "sfrom_export_pencil": [_P, _P, _P, _P, _P],
    "sfrom_export_cell": [_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                          _P, _P, _P, _P, _P],
    "sfrom_export_piece": [_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), _P, _P],
    "sfrom_surrogate_create": [C.POINTER(_P), C.c_int32, _P, C.c_int32, C.c_int32, C.c_int32],
    "sfrom_surrogate_destroy": [_P],
    "sfrom_surrogate_last_error": [_P],
    "sfrom_surrogate_param_count": [_P, C.POINTER(C.c_int64)],
    "sfrom_surrogate_set_params": [_P, _P],
    "sfrom_surrogate_get_params": [_P, _P],
    "sfrom_surrogate_set_scale": [_P, _P, _P],
    "sfrom_surrogate_gradients": [_P, _P, _P, C.c_int32, C.POINTER(C.c_float), _P],
    "sfrom_surrogate_train_step": [_P, _P, _P, C.c_int32, C.c_float, C.POINTER(C.c_float)],
    "sfrom_surrogate_forward": [_P, _P, C.c_int32, C.c_int32, _P],
    "sfrom_surrogate_targets": [_P, C.c_int32, _P, _P],
    "sfrom_build_learned": [_P, C.POINTER(sfrom_build_opts), _P, C.c_int32, _P, _P, C.c_double, C.c_double,
                            _P, _P],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.sfrom_destroy.restype = None
_lib.sfrom_last_error.restype = C.c_char_p
_lib.sfrom_surrogate_destroy.restype = None
_lib.sfrom_surrogate_last_error.restype = C.c_char_p

EXPORTED = tuple(_SIGS)


def _ptr(a, dtype=None):
    """Host pointer of a contiguous numpy array (kept alive by the caller)."""
    if a is None:
        return None
    return a.ctypes.data_as(_P)


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _dev(t):
    """Device pointer of a torch tensor."""
    return _P(t.data_ptr())


def _check(h, rc):
    if rc != 0:
        msg = _lib.sfrom_last_error(h).decode() if h else ""
        raise SfromError(rc, msg)


# ---------------------------------------------------------------------------
# one wrapper per C function
# ---------------------------------------------------------------------------

def sfrom_create(device: int = 0, stream: int = 0):
    h = _P()
    rc = _lib.sfrom_create(C.byref(h), device, _P(stream) if stream else None)
    if rc != 0:
        raise SfromError(rc, "sfrom_create failed: " + _lib.sfrom_last_error(None).decode())
    return h


def sfrom_destroy(h):
    _lib.sfrom_destroy(h)


def sfrom_last_error(h) -> str:
    return _lib.sfrom_last_error(h).decode()


def sfrom_set_pencil(h, rowptr, col, a, b):
    rowptr = _host(rowptr, np.int64); col = _host(col, np.int32)
    a = _host(a, np.float64); b = _host(b, np.float64)
    _check(h, _lib.sfrom_set_pencil(h, len(b), _ptr(rowptr), _ptr(col), _ptr(a), _ptr(b)))


def sfrom_add_cell(h, cell, global_node, rowptr, col, a, b):
    g = _host(global_node, np.int64); rp = _host(rowptr, np.int32); cl = _host(col, np.int32)
    av = _host(a, np.float64); bv = _host(b, np.float64)
    _check(h, _lib.sfrom_add_cell(h, cell, len(g), _ptr(g), _ptr(rp), _ptr(cl), _ptr(av), _ptr(bv)))


def sfrom_add_piece(h, piece, global_node, S):
    g = _host(global_node, np.int64)
    S = np.asfortranarray(np.asarray(S, dtype=np.float64))
    kp, bp = S.shape
    Sf = S.ravel(order="F")
    _check(h, _lib.sfrom_add_piece(h, piece, kp, _ptr(g), bp, _ptr(Sf)))


def sfrom_setup_voxel_acoustic(h, sigma, rho, cuts, modes_face, modes_edge):
    """sigma, rho: arrays indexed [x, y, z]; cuts: three sequences of plane
    coordinates."""
    sigma = np.asarray(sigma, dtype=np.float64)
    nvox = np.array(sigma.shape, dtype=np.int32)
    s = np.ascontiguousarray(sigma.transpose(2, 1, 0)).ravel()       # x fastest
    r = np.ascontiguousarray(np.asarray(rho, dtype=np.float64).transpose(2, 1, 0)).ravel()
    ncut = np.array([len(c) for c in cuts], dtype=np.int32)
    cc = np.concatenate([np.asarray(c, dtype=np.int32) for c in cuts]) if ncut.sum() else np.zeros(1, np.int32)
    _check(h, _lib.sfrom_setup_voxel_acoustic(h, _ptr(nvox), _ptr(s), _ptr(r), _ptr(ncut), _ptr(cc),
                                              modes_face, modes_edge))


def sfrom_setup_voxel_acoustic_rules(h, sigma, rho, cuts, face_area_max, face_modes, modes_edge):
    """As sfrom_setup_voxel_acoustic with face-mode counts by face area."""
    sigma = np.asarray(sigma, dtype=np.float64)
    nvox = np.array(sigma.shape, dtype=np.int32)
    s = np.ascontiguousarray(sigma.transpose(2, 1, 0)).ravel()
    r = np.ascontiguousarray(np.asarray(rho, dtype=np.float64).transpose(2, 1, 0)).ravel()
    ncut = np.array([len(c) for c in cuts], dtype=np.int32)
    cc = np.concatenate([np.asarray(c, dtype=np.int32) for c in cuts]) if ncut.sum() else np.zeros(1, np.int32)
    am = np.ascontiguousarray(face_area_max, dtype=np.int32)
    fm = np.ascontiguousarray(face_modes, dtype=np.int32)
    _check(h, _lib.sfrom_setup_voxel_acoustic_rules(h, _ptr(nvox), _ptr(s), _ptr(r), _ptr(ncut), _ptr(cc),
                                                    len(am), _ptr(am), _ptr(fm), modes_edge))


def sfrom_setup_voxel_elastic(h, c21, rho, cuts, modes_face, modes_edge):
    """c21: (nx, ny, nz, 21) upper-triangle Voigt stiffness per voxel, rho:
    (nx, ny, nz); arrays indexed [x, y, z] (x fastest in memory order F)."""
    rho = np.asarray(rho, np.float64)
    nvox = np.array(rho.shape, np.int32)
    r = np.ascontiguousarray(rho.transpose(2, 1, 0))
    c = np.ascontiguousarray(np.asarray(c21, np.float64).transpose(2, 1, 0, 3))
    ncut = np.array([len(x) for x in cuts], np.int32)
    cc = np.ascontiguousarray(np.concatenate([np.asarray(x, np.int32) for x in cuts]) if ncut.sum() else np.zeros(1, np.int32))
    _check(h, _lib.sfrom_setup_voxel_elastic(h, _ptr(nvox), _ptr(c), _ptr(r), _ptr(ncut), _ptr(cc),
                                             int(modes_face), int(modes_edge)))


def sfrom_partition_graph(h, n_cells, alpha=0.5, beta=0.5):
    _check(h, _lib.sfrom_partition_graph(h, int(n_cells), float(alpha), float(beta)))


def sfrom_set_breakdown_policy(h, reduce_m):
    _check(h, _lib.sfrom_set_breakdown_policy(h, int(bool(reduce_m))))


def sfrom_gramian_bases(h, omega_max, eps, max_modes, depth):
    _check(h, _lib.sfrom_gramian_bases(h, float(omega_max), float(eps), int(max_modes), int(depth)))


def sfrom_gramian_bases_zolotarev(h, omega_max, eps, max_modes, depth, n_poles, gamma):
    _check(h, _lib.sfrom_gramian_bases_zolotarev(h, float(omega_max), float(eps), int(max_modes), int(depth),
                                                 int(n_poles), float(gamma)))


def sfrom_remove_corner_set(h):
    """Returns (n_new, n_corner, n_hanging)."""
    n1 = C.c_int64(); nk = C.c_int32(); nh = C.c_int64()
    _check(h, _lib.sfrom_remove_corner_set(h, C.byref(n1), C.byref(nk), C.byref(nh)))
    return n1.value, nk.value, nh.value


def sfrom_corner_map(h, n_old, n_corner, n_hanging):
    """Returns (new_of_old, corner, hang_ptr, hang_node, hang_weight)."""
    new_of_old = np.empty(n_old, np.int64)
    corner = np.empty(n_corner, np.int64)
    ptr = np.empty(n_corner + 1, np.int64)
    node = np.empty(n_hanging, np.int64)
    wt = np.empty(n_hanging, np.float64)
    _check(h, _lib.sfrom_corner_map(h, new_of_old.ctypes.data, corner.ctypes.data, ptr.ctypes.data,
                                    node.ctypes.data, wt.ctypes.data))
    return new_of_old, corner, ptr, node, wt


def sfrom_set_persistent(h, enable):
    _check(h, _lib.sfrom_set_persistent(h, int(enable)))


def sfrom_set_corner_correction(h, enable):
    _check(h, _lib.sfrom_set_corner_correction(h, int(enable)))


def sfrom_build(h, m, shift, online_prec=SFROM_F32, m_per_cell=None, cells_per_batch=0):
    o = sfrom_build_opts()
    o.m = m
    keep = None
    if m_per_cell is not None:
        keep = _host(m_per_cell, np.int32)
        o.m_per_cell = keep.ctypes.data_as(C.POINTER(C.c_int32))
    o.shift = shift
    o.online_prec = online_prec
    o.cells_per_batch = cells_per_batch
    _check(h, _lib.sfrom_build(h, C.byref(o)))
    del keep


def sfrom_import_rom(h, cell, Ghat, G):
    Ghat = np.asarray(Ghat, dtype=np.float64); G = np.asarray(G, dtype=np.float64)
    m, b, _ = Ghat.shape
    gh = np.ascontiguousarray(Ghat.transpose(0, 2, 1)).ravel()   # column-major blocks
    g = np.ascontiguousarray(G.transpose(0, 2, 1)).ravel()
    _check(h, _lib.sfrom_import_rom(h, cell, m, b, _ptr(gh), _ptr(g)))


def sfrom_export_rom(h, cell):
    m = C.c_int32(); b = C.c_int32()
    _check(h, _lib.sfrom_export_rom(h, cell, C.byref(m), C.byref(b), None, None))
    gh = np.empty(m.value * b.value * b.value); g = np.empty_like(gh)
    _check(h, _lib.sfrom_export_rom(h, cell, C.byref(m), C.byref(b), _ptr(gh), _ptr(g)))
    shp = (m.value, b.value, b.value)
    return gh.reshape(shp).transpose(0, 2, 1).copy(), g.reshape(shp).transpose(0, 2, 1).copy()


def _csc(cols, n_cols):
    colptr, row, val = cols
    return _host(colptr, np.int64), _host(row, np.int64), _host(val, np.float64)


def sfrom_set_sources(h, colptr, row, val, project=True):
    cp, rw, vl = _csc((colptr, row, val), None)
    _check(h, _lib.sfrom_set_sources(h, len(cp) - 1, _ptr(cp), _ptr(rw), _ptr(vl), int(project)))


def sfrom_set_receivers(h, colptr, row, val, project=True):
    cp, rw, vl = _csc((colptr, row, val), None)
    _check(h, _lib.sfrom_set_receivers(h, len(cp) - 1, _ptr(cp), _ptr(rw), _ptr(vl), int(project)))


def sfrom_point_columns(h, nodes, max_piece_nodes):
    nodes = _host(nodes, np.int64)
    cp = np.empty(len(nodes) + 1, np.int64)
    rw = np.empty(max(1, len(nodes) * max_piece_nodes), np.int64)
    vl = np.empty(max(1, len(nodes) * max_piece_nodes), np.float64)
    _check(h, _lib.sfrom_point_columns(h, len(nodes), _ptr(nodes), _ptr(cp), _ptr(rw), _ptr(vl)))
    return cp, rw[:cp[-1]].copy(), vl[:cp[-1]].copy()


def sfrom_reset(h):
    _check(h, _lib.sfrom_reset(h))


def sfrom_save(h, path):
    _check(h, _lib.sfrom_save(h, os.fsencode(path)))


def sfrom_load(h, path):
    _check(h, _lib.sfrom_load(h, os.fsencode(path)))


def _device_tensor(t, what):
    """A torch tensor handed to the library as a device pointer: it must live
    in GPU memory (the kernels dereference it) and be contiguous."""
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{what}: a torch tensor must be on the GPU (got device {t.device}); "
                         "pass a numpy array for host memory")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return _dev(t)


def _wave_arg(w):
    if hasattr(w, "data_ptr"):
        return _device_tensor(w, "wavelet"), 1, None
    w = _host(w, np.float64)
    return _ptr(w), 0, w


def _trace_arg(traces):
    if hasattr(traces, "data_ptr"):
        return _device_tensor(traces, "traces"), 1
    if not isinstance(traces, np.ndarray):
        raise ValueError("traces must be a numpy array or a GPU torch tensor")
    if not (traces.flags.c_contiguous and traces.flags.writeable):
        raise ValueError("traces must be a C-contiguous, writeable numpy array")
    return _ptr(traces), 0


def _check_buffers(h, n_steps, w, traces, prec):
    """The library cannot see buffer sizes: refuse a trace buffer of the
    wrong element type or too few elements, and a short wavelet, before any
    kernel writes to them."""
    info = sfrom_get_info(h)
    need = int(n_steps) * info["n_receivers"] * info["n_sources"]
    itemsize = 8 if prec == SFROM_F64 else 4
    t_item = traces.element_size() if hasattr(traces, "element_size") else np.asarray(traces).itemsize
    t_count = traces.numel() if hasattr(traces, "numel") else np.asarray(traces).size
    if n_steps > 0:
        if t_item != itemsize:
            raise ValueError(f"traces must hold {itemsize}-byte values for this precision (got {t_item})")
        if t_count < need:
            raise ValueError(f"traces hold {t_count} values, the run writes {need}")
        if hasattr(traces, "is_contiguous") and not traces.is_contiguous():
            raise ValueError("traces must be contiguous")
        w_count = w.numel() if hasattr(w, "numel") else np.asarray(w).size
        w_item = w.element_size() if hasattr(w, "element_size") else 8
        if w_count < n_steps or w_item != 8:
            raise ValueError("the wavelet needs n_steps float64 samples")


def sfrom_run(h, n_steps, dt, w, traces):
    """w: numpy float64 (host) or torch float64 CUDA tensor; traces: numpy
    or torch array of n_steps x n_r x n_s in the on-line precision (float64
    for F64, float32 otherwise)."""
    _check_buffers(h, n_steps, w, traces, sfrom_get_info(h)["online_prec"])
    wp, wdev, keep = _wave_arg(w)
    tp, tdev = _trace_arg(traces)
    _check(h, _lib.sfrom_run(h, n_steps, dt, wp, wdev, tp, tdev))


def sfrom_run_noalloc(h, n_steps, dt, w, traces):
    """sfrom_run without device allocation: w (float64) and traces (on-line
    precision, n_steps x n_r x n_s) must be contiguous GPU torch tensors."""
    _check_buffers(h, n_steps, w, traces, sfrom_get_info(h)["online_prec"])
    wp = _device_tensor(w, "wavelet")
    tp = _device_tensor(traces, "traces")
    _check(h, _lib.sfrom_run_noalloc(h, n_steps, dt, wp, tp))


def sfrom_fine_reset(h):
    _check(h, _lib.sfrom_fine_reset(h))


def sfrom_fine_run(h, n_steps, dt, w, traces, prec=SFROM_F32):
    _check_buffers(h, n_steps, w, traces, prec)
    wp, wdev, keep = _wave_arg(w)
    tp, tdev = _trace_arg(traces)
    _check(h, _lib.sfrom_fine_run(h, n_steps, dt, wp, wdev, tp, tdev, prec))


def sfrom_fine_lambda_max(h) -> float:
    v = C.c_double()
    _check(h, _lib.sfrom_fine_lambda_max(h, C.byref(v)))
    return v.value


def sfrom_rom_lambda_max(h) -> float:
    v = C.c_double()
    _check(h, _lib.sfrom_rom_lambda_max(h, C.byref(v)))
    return v.value


def sfrom_set_graph(h, enable=True):
    _check(h, _lib.sfrom_set_graph(h, int(enable)))


def sfrom_set_build_path(h, mode=0):
    """0 automatic, 1 blocked wide-band kernels, 2 one workgroup per cell."""
    _check(h, _lib.sfrom_set_build_path(h, mode))


def sfrom_set_cell_variant(h, variant=-1):
    _check(h, _lib.sfrom_set_cell_variant(h, int(variant)))


def sfrom_profile(h, enable=True):
    """enable: False/0 off, True/1 every step, N > 1 one step in N."""
    _check(h, _lib.sfrom_profile(h, int(enable)))


KERNEL_CELL, KERNEL_PIECE, KERNEL_RECEIVERS, KERNEL_FINE = 0, 1, 2, 3


def sfrom_profile_read(h, kernel):
    """(total_ms, launches) of kernel id since the last read."""
    ms = C.c_double(); n = C.c_int64()
    _check(h, _lib.sfrom_profile_read(h, kernel, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def sfrom_get_info(h) -> dict:
    i = sfrom_info()
    _check(h, _lib.sfrom_get_info(h, C.byref(i)))
    return i.as_dict()


def sfrom_export_pencil(h):
    info = sfrom_get_info(h)
    rp = np.empty(info["n"] + 1, np.int64); cl = np.empty(info["nnz"], np.int32)
    a = np.empty(info["nnz"]); b = np.empty(info["n"])
    _check(h, _lib.sfrom_export_pencil(h, _ptr(rp), _ptr(cl), _ptr(a), _ptr(b)))
    return rp, cl, a, b


def sfrom_export_cell(h, cell):
    n = C.c_int32(); nnz = C.c_int32(); bd = C.c_int32()
    _check(h, _lib.sfrom_export_cell(h, cell, C.byref(n), C.byref(nnz), C.byref(bd), None, None, None, None, None))
    g = np.empty(n.value, np.int64); rp = np.empty(n.value + 1, np.int32); cl = np.empty(nnz.value, np.int32)
    a = np.empty(nnz.value); b = np.empty(n.value)
    _check(h, _lib.sfrom_export_cell(h, cell, C.byref(n), C.byref(nnz), C.byref(bd), _ptr(g), _ptr(rp), _ptr(cl),
                                     _ptr(a), _ptr(b)))
    return {"global_node": g, "rowptr": rp, "col": cl, "a": a, "b": b, "b_dim": bd.value}


def sfrom_export_piece(h, piece):
    k = C.c_int32(); bp = C.c_int32()
    _check(h, _lib.sfrom_export_piece(h, piece, C.byref(k), C.byref(bp), None, None))
    g = np.empty(k.value, np.int64); S = np.empty(k.value * bp.value)
    _check(h, _lib.sfrom_export_piece(h, piece, C.byref(k), C.byref(bp), _ptr(g), _ptr(S)))
    return g, S.reshape(bp.value, k.value).T.copy()


# ---------------------------------------------------------------------------
# learned off-line stage
# ---------------------------------------------------------------------------

def _scheck(s, rc):
    if rc != 0:
        msg = _lib.sfrom_surrogate_last_error(s).decode() if s else ""
        raise SfromError(rc, msg)


def sfrom_surrogate_create(device: int, stream: int, conv_ch: int, hidden: int, n_out: int):
    s = _P()
    rc = _lib.sfrom_surrogate_create(C.byref(s), device, _P(stream) if stream else None, conv_ch, hidden, n_out)
    if rc != 0:
        raise SfromError(rc, "sfrom_surrogate_create failed")
    return s


def sfrom_surrogate_destroy(s):
    _lib.sfrom_surrogate_destroy(s)


def sfrom_surrogate_last_error(s) -> str:
    return _lib.sfrom_surrogate_last_error(s).decode()


def sfrom_surrogate_param_count(s) -> int:
    n = C.c_int64()
    _scheck(s, _lib.sfrom_surrogate_param_count(s, C.byref(n)))
    return n.value


def sfrom_surrogate_set_params(s, theta):
    theta = _host(theta, np.float32)
    _scheck(s, _lib.sfrom_surrogate_set_params(s, _ptr(theta)))


def sfrom_surrogate_get_params(s):
    out = np.empty(sfrom_surrogate_param_count(s), np.float32)
    _scheck(s, _lib.sfrom_surrogate_get_params(s, _ptr(out)))
    return out


def sfrom_surrogate_set_scale(s, mu, sd):
    mu = _host(mu, np.float32); sd = _host(sd, np.float32)
    _scheck(s, _lib.sfrom_surrogate_set_scale(s, _ptr(mu), _ptr(sd)))


def sfrom_surrogate_gradients(s, x, t):
    """x, t: float32 CUDA tensors (n x 1024, n x n_out). Returns (loss, grad)."""
    loss = C.c_float()
    g = np.empty(sfrom_surrogate_param_count(s), np.float32)
    _scheck(s, _lib.sfrom_surrogate_gradients(s, _dev(x), _dev(t), x.shape[0], C.byref(loss), _ptr(g)))
    return float(loss.value), g


def sfrom_surrogate_train_step(s, x, t, lr):
    loss = C.c_float()
    _scheck(s, _lib.sfrom_surrogate_train_step(s, _dev(x), _dev(t), x.shape[0], lr, C.byref(loss)))
    return float(loss.value)


def sfrom_surrogate_forward(s, x, y, bf16=True):
    _scheck(s, _lib.sfrom_surrogate_forward(s, _dev(x), x.shape[0], 1 if bf16 else 0, _dev(y)))


def sfrom_surrogate_targets(h, cells, t):
    """cells: host int32 ids; t: float32 CUDA tensor (n x n_out)."""
    cells = _host(cells, np.int32)
    _check(h, _lib.sfrom_surrogate_targets(h, len(cells), _ptr(cells), _dev(t)))


def sfrom_build_learned(h, m, shift, prec, s, cells, x, omega_max, tol, m_per_cell=None, cells_per_batch=0):
    """Returns (accepted int32 array, mismatch float64 array) per candidate."""
    cells = _host(cells, np.int32)
    o = sfrom_build_opts()
    o.m = m
    keep = None
    if m_per_cell is not None:
        keep = _host(m_per_cell, np.int32)
        o.m_per_cell = keep.ctypes.data_as(C.POINTER(C.c_int32))
    o.shift = shift
    o.online_prec = prec
    o.cells_per_batch = cells_per_batch
    acc = np.zeros(len(cells), np.int32)
    mis = np.zeros(len(cells), np.float64)
    _check(h, _lib.sfrom_build_learned(h, C.byref(o), s, len(cells), _ptr(cells), _dev(x) if len(cells) else None,
                                       omega_max, tol, _ptr(acc), _ptr(mis)))
    return acc, mis
