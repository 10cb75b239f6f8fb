"""ctypes binding of libapril.so (include/april.h), same names as the C ABI.

Argument marshalling only: every step of the filter runs in the library's
HIP kernels.  Device arrays are torch tensors on a HIP device (their
data_ptr() is passed through); streams are torch.cuda streams.  The binding
raises if the library has not been built -- there is no fallback path.
"""

from __future__ import annotations

import atexit
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapril.so")

OK, PENDING = 0, 1
E_INVALID, E_GRID, E_NOMEM, E_HIP, E_CORRUPT, E_NODEV, E_IO = -1, -2, -3, -4, -5, -6, -7
TN, TH, INDECISIVE, BAD_PAIR = 0, 1, 2, 255
STRICT = 1
GRID_PARTITIONED = 1
CODEC_RAW, CODEC_VBYTE = 0, 1
SCHED_PLAIN, SCHED_BATCHED = 0, 1
VALIDATE = 1
WS_DECODE_CACHE = 2
WAVE_TIMES = 4
WAVE_TIMES_OFFSET = 24448

_ERRNAMES = {E_INVALID: "APRIL_E_INVALID", E_GRID: "APRIL_E_GRID", E_NOMEM: "APRIL_E_NOMEM",
             E_HIP: "APRIL_E_HIP", E_CORRUPT: "APRIL_E_CORRUPT", E_NODEV: "APRIL_E_NODEV",
             E_IO: "APRIL_E_IO"}


class AprilError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class april_grid_t(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("side", C.c_double),
                ("order", C.c_uint32), ("flags", C.c_uint32)]


class april_lists_info_t(C.Structure):
    _fields_ = [("n_objects", C.c_uint64), ("n_a", C.c_uint64), ("n_f", C.c_uint64),
                ("device_bytes", C.c_uint64), ("on_device", C.c_int32), ("codec", C.c_uint32)]


class april_filter_opts_t(C.Structure):
    _fields_ = [("schedule", C.c_uint32), ("flags", C.c_uint32), ("waves", C.c_uint32),
                ("tile", C.c_uint32), ("chunk", C.c_uint32), ("thread_max", C.c_uint32),
                ("search_min", C.c_uint32), ("wg_min", C.c_uint32),
                ("d_workspace", C.c_void_p), ("workspace_bytes", C.c_uint64)]


class april_device_info_t(C.Structure):
    _fields_ = [("device", C.c_int32), ("compute_units", C.c_int32),
                ("wavefront_size", C.c_int32), ("reserved", C.c_int32),
                ("hbm_bytes", C.c_uint64), ("arch", C.c_char * 64), ("name", C.c_char * 128)]


class april_serve_opts_t(C.Structure):
    _fields_ = [("mbr_grid", C.c_uint32), ("slots", C.c_uint32), ("mem_budget", C.c_uint64),
                ("max_batch", C.c_uint32), ("host_threads", C.c_uint32),
                ("gpu_build_cells", C.c_uint32), ("reserved", C.c_uint32),
                ("filter", april_filter_opts_t)]


class april_result_t(C.Structure):
    _fields_ = [("status", C.c_int32), ("reserved", C.c_uint32), ("n_pairs", C.c_uint64),
                ("s_ids", C.POINTER(C.c_uint32)), ("verdict", C.POINTER(C.c_uint8)),
                ("counts", C.c_uint64 * 3), ("t_submit", C.c_double), ("t_built", C.c_double),
                ("t_done", C.c_double)]


class april_serve_stats_t(C.Structure):
    _fields_ = [("slots", C.c_uint32), ("slots_busy", C.c_uint32), ("queued", C.c_uint64),
                ("ready", C.c_uint64), ("cap_pairs", C.c_uint64), ("cap_intervals", C.c_uint64),
                ("cap_queries", C.c_uint64)]


_lib = None
_exiting = False


@atexit.register
def _mark_exit():
    global _exiting
    _exiting = True


def lib():
    """Load libapril.so; raise (never fall back) when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                          "or python paper_2307_01716_amd/_build.py")
    L = C.CDLL(LIB_PATH)
    P, u64, u32, i32 = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int
    L.april_build_lists.argtypes = [C.POINTER(april_grid_t), P, P, u64, u32, C.POINTER(P)]
    L.april_build_lists_partitioned.argtypes = [P, u32, P, P, P, u64, u32, C.POINTER(P)]
    L.april_build_lists_gpu.argtypes = [C.POINTER(april_grid_t), P, P, u64, u32, P, C.POINTER(P)]
    L.april_lists_from_arrays.argtypes = [C.POINTER(april_grid_t), u64, P, P, P, P, P, P, i32,
                                          C.POINTER(P)]
    L.april_lists_info.argtypes = [P, C.POINTER(april_lists_info_t)]
    L.april_lists_export.argtypes = [P] * 7
    L.april_lists_to_device.argtypes = [P, u32, P, C.POINTER(P)]
    L.april_lists_download.argtypes = [P, P, C.POINTER(P)]
    L.april_lists_free.argtypes = [P]
    L.april_lists_save.argtypes = [P, C.c_char_p]
    L.april_lists_load.argtypes = [C.c_char_p, i32, C.POINTER(P)]
    L.april_lists_free.restype = None
    L.april_filter_pairs.argtypes = [P, P, P, P, u64, P, P, C.POINTER(april_filter_opts_t), P]
    L.april_filter_pairs_static.argtypes = [P, P, P, P, u64, P, P, C.POINTER(april_filter_opts_t), P]
    L.april_alg2_bytes.argtypes = [P, P, P, P, u64, P, P]
    L.april_filter_workspace_size.argtypes = [u64, C.POINTER(april_filter_opts_t), C.POINTER(u64)]
    L.april_mbr_join.argtypes = [P, u64, P, u64, P, P, u64, C.POINTER(u64)]
    L.april_device_info.argtypes = [C.POINTER(april_device_info_t)]
    L.april_serve_create.argtypes = [P, P, C.POINTER(april_serve_opts_t), C.POINTER(P)]
    L.april_serve_submit.argtypes = [P, P, u64, C.POINTER(u64)]
    L.april_serve_poll.argtypes = [P, u64, C.POINTER(april_result_t)]
    L.april_serve_wait.argtypes = [P, u64, C.c_double, C.POINTER(april_result_t)]
    L.april_serve_release.argtypes = [P, u64]
    L.april_serve_cancel.argtypes = [P, u64]
    L.april_serve_stats.argtypes = [P, C.POINTER(april_serve_stats_t)]
    L.april_serve_destroy.argtypes = [P]
    L.april_serve_destroy.restype = None
    L.april_polys_to_device.argtypes = [P, P, u64, u32, P, C.POINTER(P)]
    L.april_polys_free.argtypes = [P]
    L.april_polys_free.restype = None
    L.april_refine_pairs.argtypes = [P, P, P, P, u64, P, P, P, P]
    L.april_build_cells.argtypes = [C.POINTER(april_grid_t), P, P, u64, u32, C.POINTER(P)]
    L.april_cells_to_device.argtypes = [P, P, C.POINTER(P)]
    L.april_cells_info.argtypes = [P, C.POINTER(u64), C.POINTER(u64)]
    L.april_cells_export.argtypes = [P, P, P]
    L.april_cells_free.argtypes = [P]
    L.april_cells_free.restype = None
    for name in ("april_filter_within", "april_filter_linestrings", "april_filter_mixed"):
        getattr(L, name).argtypes = [P, P, P, P, u64, P, P, P]
        getattr(L, name).restype = C.c_int
    for name in ("april_build_cells", "april_cells_to_device", "april_cells_info", "april_cells_export"):
        getattr(L, name).restype = C.c_int
    L.april_last_error.restype = C.c_char_p
    for name in ("april_build_lists", "april_build_lists_partitioned", "april_build_lists_gpu", "april_lists_from_arrays", "april_lists_info",
                 "april_lists_export", "april_lists_to_device", "april_lists_download",
                 "april_filter_pairs", "april_filter_pairs_static",
                 "april_alg2_bytes", "april_filter_workspace_size",
                 "april_mbr_join", "april_device_info", "april_serve_create",
                 "april_serve_submit", "april_serve_poll", "april_serve_wait", "april_serve_release",
                 "april_serve_cancel", "april_serve_stats", "april_polys_to_device",
                 "april_refine_pairs"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def april_last_error() -> str:
    return lib().april_last_error().decode()


def _check(rc):
    if rc < 0:
        raise AprilError(rc, april_last_error())
    return rc


def _np(a):
    return a.ctypes.data_as(C.c_void_p)


def _grid(grid) -> april_grid_t:
    x0, y0, side, order = grid.as_tuple() if hasattr(grid, "as_tuple") else grid
    return april_grid_t(float(x0), float(y0), float(side), int(order), 0)


def _dptr(t):
    """Device pointer of a torch tensor (or an int address, or None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("device array expected (a torch tensor on a HIP device)")
    if not t.is_contiguous():
        raise ValueError("device array must be contiguous")
    return t.data_ptr()


def _counts_ptr(t):
    """Address of a counts array: a device tensor, or a pinned host tensor
    (which the filter's last kernel writes through its device mapping)."""
    if t is not None and not isinstance(t, int) and not t.is_cuda:
        if not t.is_pinned():
            raise ValueError("counts must be a device tensor or a pinned host tensor")
        if not t.is_contiguous():
            raise ValueError("counts must be contiguous")
        return t.data_ptr()
    return _dptr(t)


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Lists:
    """Owning handle of an april_lists_t (host- or device-resident)."""

    def __init__(self, handle: int, keep=None):
        self._h = handle
        self._keep = keep      # host lists a pending upload still reads

    @property
    def handle(self):
        if not self._h:
            raise ValueError("lists were freed")
        return self._h

    def info(self) -> april_lists_info_t:
        inf = april_lists_info_t()
        _check(lib().april_lists_info(self.handle, C.byref(inf)))
        return inf

    def __len__(self):
        return int(self.info().n_objects)

    def export(self):
        """(offA, sA, eA, offF, sF, eF) numpy arrays of host lists."""
        inf = self.info()
        n, na, nf = int(inf.n_objects), int(inf.n_a), int(inf.n_f)
        out = (np.empty(n + 1, np.uint64), np.empty(na, np.uint32), np.empty(na, np.uint32),
               np.empty(n + 1, np.uint64), np.empty(nf, np.uint32), np.empty(nf, np.uint32))
        _check(lib().april_lists_export(self.handle, *[_np(a) for a in out]))
        return out

    def free(self):
        if self._h and not _exiting:
            lib().april_lists_free(self._h)
        self._h = None
        self._keep = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def april_build_lists(grid, xy: np.ndarray, vtx_off: np.ndarray, flags: int = 0) -> Lists:
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    vo = np.ascontiguousarray(vtx_off, dtype=np.uint64)
    g = _grid(grid)
    h = C.c_void_p()
    _check(lib().april_build_lists(C.byref(g), _np(xy), _np(vo), len(vo) - 1, flags, C.byref(h)))
    return Lists(h.value)


def april_build_lists_gpu(grid, xy: np.ndarray, vtx_off: np.ndarray, flags: int = 0, stream=None) -> Lists:
    """The lists of april_build_lists, built on the current GPU; device lists."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    vo = np.ascontiguousarray(vtx_off, dtype=np.uint64)
    g = _grid(grid)
    h = C.c_void_p()
    _check(lib().april_build_lists_gpu(C.byref(g), _np(xy), _np(vo), len(vo) - 1, flags, _stream(stream),
                                       C.byref(h)))
    return Lists(h.value)


def april_lists_from_arrays(grid, offA, sA, eA, offF, sF, eF, validate: bool = True) -> Lists:
    arrs = [np.ascontiguousarray(offA, np.uint64), np.ascontiguousarray(sA, np.uint32),
            np.ascontiguousarray(eA, np.uint32), np.ascontiguousarray(offF, np.uint64),
            np.ascontiguousarray(sF, np.uint32), np.ascontiguousarray(eF, np.uint32)]
    g = _grid(grid)
    h = C.c_void_p()
    _check(lib().april_lists_from_arrays(C.byref(g), len(arrs[0]) - 1, *[_np(a) for a in arrs],
                                         int(validate), C.byref(h)))
    return Lists(h.value)


def april_lists_to_device(host: Lists, codec: int = CODEC_RAW, stream=None) -> Lists:
    h = C.c_void_p()
    _check(lib().april_lists_to_device(host.handle, codec, _stream(stream), C.byref(h)))
    return Lists(h.value, keep=host)


def _opts(schedule=SCHED_PLAIN, flags=0, waves=0, tile=0, chunk=0, thread_max=0, search_min=0,
          wg_min=0, workspace=None):
    ws = _dptr(workspace) if workspace is not None else None
    nbytes = int(workspace.numel() * workspace.element_size()) if hasattr(workspace, "numel") else 0
    return april_filter_opts_t(schedule, flags, waves, tile, chunk, thread_max, search_min,
                               wg_min, ws, nbytes)


def april_filter_workspace_size(n_pairs: int, schedule=SCHED_BATCHED, flags=0) -> int:
    o = _opts(schedule, flags)
    out = C.c_uint64()
    _check(lib().april_filter_workspace_size(n_pairs, C.byref(o), C.byref(out)))
    return out.value


def april_lists_save(host: Lists, path) -> None:
    """Write host lists to a versioned list file sealed with its SHA-256."""
    _check(lib().april_lists_save(host.handle, os.fsencode(path)))


def april_lists_load(path, validate: bool = True) -> Lists:
    """Host lists read back from a list file (digest checked; with validate,
    the lists too)."""
    h = C.c_void_p()
    _check(lib().april_lists_load(os.fsencode(path), int(validate), C.byref(h)))
    return Lists(h.value)


def april_lists_download(dev: Lists, stream=None) -> Lists:
    """Device lists back to host lists (compressed ones decoded on the device)."""
    h = C.c_void_p()
    _check(lib().april_lists_download(dev.handle, _stream(stream), C.byref(h)))
    return Lists(h.value)


def april_filter_pairs(R: Lists, S: Lists, r, s, verdict, counts=None, schedule=SCHED_PLAIN,
                       flags=0, waves=0, stream=None, **tuning) -> int:
    """r, s: int32/uint32 device tensors [P]; verdict: uint8 device tensor [P];
    counts: int64 tensor [3] on the device or in pinned host memory, or
    None.  `tuning` keys: tile, chunk,
    thread_max, search_min, workspace (a device tensor)."""
    n = int(r.numel()) if hasattr(r, "numel") else (0 if isinstance(r, int) else int(len(r)))
    opts = _opts(schedule, flags, waves, **tuning)
    return _check(lib().april_filter_pairs(R.handle, S.handle, _dptr(r), _dptr(s), n,
                                           _dptr(verdict), _counts_ptr(counts), C.byref(opts),
                                           _stream(stream)))


def april_filter_pairs_static(R: Lists, S: Lists, r, s, verdict, counts=None, schedule=SCHED_PLAIN,
                              flags=0, waves=0, stream=None, **tuning) -> int:
    """april_filter_pairs on the library's static scratch: allocates nothing
    (raw lists; no workspace)."""
    n = int(r.numel()) if hasattr(r, "numel") else (0 if isinstance(r, int) else int(len(r)))
    opts = _opts(schedule, flags, waves, **tuning)
    return _check(lib().april_filter_pairs_static(R.handle, S.handle, _dptr(r), _dptr(s), n,
                                                  _dptr(verdict), _counts_ptr(counts), C.byref(opts),
                                                  _stream(stream)))


def april_alg2_bytes(R: Lists, S: Lists, r, s, bytes_out, stream=None) -> int:
    """Per-pair bytes Alg. 2 moves (device uint64 tensor [P], here int64)."""
    n = int(r.numel())
    return _check(lib().april_alg2_bytes(R.handle, S.handle, _dptr(r), _dptr(s), n,
                                         _dptr(bytes_out), _stream(stream)))


class Cells:
    """Owning handle of linestring cell lists (host- or device-resident)."""

    def __init__(self, handle: int, keep=None):
        self._h = handle
        self._keep = keep

    @property
    def handle(self):
        if not self._h:
            raise ValueError("cells were freed")
        return self._h

    def info(self):
        n, m = C.c_uint64(), C.c_uint64()
        _check(lib().april_cells_info(self.handle, C.byref(n), C.byref(m)))
        return int(n.value), int(m.value)

    def __len__(self):
        return self.info()[0]

    def export(self):
        """(off, ids) numpy arrays of host cells."""
        n, m = self.info()
        off, ids = np.empty(n + 1, np.uint64), np.empty(m, np.uint32)
        _check(lib().april_cells_export(self.handle, _np(off), _np(ids)))
        return off, ids

    def free(self):
        if self._h and not _exiting:
            lib().april_cells_free(self._h)
        self._h = None
        self._keep = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def april_build_cells(grid, xy: np.ndarray, vtx_off: np.ndarray, flags: int = 0) -> Cells:
    """Cell lists of linestrings (open chains) on `grid`; host cells."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    vo = np.ascontiguousarray(vtx_off, dtype=np.uint64)
    g = _grid(grid)
    h = C.c_void_p()
    _check(lib().april_build_cells(C.byref(g), _np(xy), _np(vo), len(vo) - 1, flags, C.byref(h)))
    return Cells(h.value)


def april_cells_to_device(host: Cells, stream=None) -> Cells:
    h = C.c_void_p()
    _check(lib().april_cells_to_device(host.handle, _stream(stream), C.byref(h)))
    return Cells(h.value, keep=host)


def _variant(fn, A, B, a, b, verdict, counts, stream):
    n = int(a.numel())
    return _check(fn(A.handle, B.handle, _dptr(a), _dptr(b), n, _dptr(verdict), _dptr(counts), _stream(stream)))


def april_filter_within(R: Lists, S: Lists, r, s, verdict, counts=None, stream=None) -> int:
    """Within-join filter: is R[r[i]] within S[s[i]]? (device tensors)"""
    return _variant(lib().april_filter_within, R, S, r, s, verdict, counts, stream)


def april_filter_linestrings(P: Lists, L: Cells, p, l, verdict, counts=None, stream=None) -> int:
    """Polygon-linestring filter on device lists and device cells."""
    return _variant(lib().april_filter_linestrings, P, L, p, l, verdict, counts, stream)


def april_filter_mixed(R: Lists, S: Lists, r, s, verdict, counts=None, stream=None) -> int:
    """Alg. 2 across grid orders (same data space)."""
    return _variant(lib().april_filter_mixed, R, S, r, s, verdict, counts, stream)


class Polys:
    """Owning handle of a device polygon collection (april_polys_t)."""

    def __init__(self, handle: int):
        self._h = handle

    @property
    def handle(self):
        if not self._h:
            raise ValueError("polygons were freed")
        return self._h

    def free(self):
        if self._h and not _exiting:
            lib().april_polys_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def april_polys_to_device(xy: np.ndarray, vtx_off: np.ndarray, flags: int = 0, stream=None) -> Polys:
    """Polygons (CSR form, as for april_build_lists) to the current device."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    vo = np.ascontiguousarray(vtx_off, dtype=np.uint64)
    h = C.c_void_p()
    _check(lib().april_polys_to_device(_np(xy), _np(vo), len(vo) - 1, flags, _stream(stream), C.byref(h)))
    return Polys(h.value)


def april_refine_pairs(R: Polys, S: Polys, r, s, out, verdict=None, counts=None, stream=None) -> int:
    """Exact test of pairs (r[i], s[i]): out[i] = 1 if the polygons share a
    point, else 0.  r, s: int32/uint32 device tensors [P]; out: uint8 device
    tensor [P]; verdict: the filter's uint8 verdicts (TN/TH answered without
    geometry) or None; counts: int64 device tensor [2] or None."""
    n = int(r.numel())
    return _check(lib().april_refine_pairs(R.handle, S.handle, _dptr(r), _dptr(s), n, _dptr(verdict),
                                           _dptr(out), _dptr(counts), _stream(stream)))


def april_mbr_join(boxes_r: np.ndarray, boxes_s: np.ndarray):
    """Candidate pairs (r, s) of intersecting closed MBRs, grouped by r with the
    r objects in the Z-order of their MBR centres (s ascending within r)."""
    br = np.ascontiguousarray(boxes_r, np.float64)
    bs = np.ascontiguousarray(boxes_s, np.float64)
    need = C.c_uint64()
    L = lib()
    rc = L.april_mbr_join(_np(br), len(br), _np(bs), len(bs), None, None, 0, C.byref(need))
    if rc != E_NOMEM:
        _check(rc)
    r = np.empty(need.value, np.uint32)
    s = np.empty(need.value, np.uint32)
    _check(L.april_mbr_join(_np(br), len(br), _np(bs), len(bs), _np(r), _np(s), need.value,
                            C.byref(need)))
    return r, s


def april_device_info() -> dict:
    inf = april_device_info_t()
    _check(lib().april_device_info(C.byref(inf)))
    return {"device": inf.device, "compute_units": inf.compute_units,
            "wavefront_size": inf.wavefront_size, "hbm_bytes": inf.hbm_bytes,
            "arch": inf.arch.decode(), "name": inf.name.decode()}


class Result:
    """A finished request: S ids (ascending) with their verdicts, copied out."""

    def __init__(self, r: april_result_t):
        self.status = r.status
        n = int(r.n_pairs)
        self.s_ids = np.ctypeslib.as_array(r.s_ids, shape=(n,)).copy() if n else np.zeros(0, np.uint32)
        self.verdict = np.ctypeslib.as_array(r.verdict, shape=(n,)).copy() if n else np.zeros(0, np.uint8)
        self.counts = [int(c) for c in r.counts]
        self.t_submit, self.t_built, self.t_done = r.t_submit, r.t_built, r.t_done

    @property
    def latency(self):
        return self.t_done - self.t_submit


class Server:
    """april_serve_* on a device-resident collection S (see include/april.h)."""

    def __init__(self, S_dev: Lists, s_boxes: np.ndarray, mbr_grid=0, slots=0, mem_budget=0,
                 max_batch=0, host_threads=0, gpu_build_cells=0, **tuning):
        self._S = S_dev
        boxes = np.ascontiguousarray(s_boxes, np.float64)
        o = april_serve_opts_t(mbr_grid, slots, mem_budget, max_batch, host_threads, gpu_build_cells, 0,
                               _opts(SCHED_BATCHED, **tuning))
        h = C.c_void_p()
        _check(lib().april_serve_create(S_dev.handle, _np(boxes), C.byref(o), C.byref(h)))
        self._h = h.value

    def submit(self, xy: np.ndarray) -> int:
        xy = np.ascontiguousarray(xy, np.float64)
        t = C.c_uint64()
        _check(lib().april_serve_submit(self._h, _np(xy), len(xy), C.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """None while pending; a Result (status OK) when done; raises on failure."""
        r = april_result_t()
        rc = lib().april_serve_poll(self._h, ticket, C.byref(r))
        if rc == PENDING:
            return None
        _check(rc)
        return Result(r)

    def wait(self, ticket: int, timeout: float = 60.0):
        r = april_result_t()
        rc = lib().april_serve_wait(self._h, ticket, timeout, C.byref(r))
        if rc == PENDING:
            raise TimeoutError(f"ticket {ticket} still pending after {timeout}s")
        _check(rc)
        return Result(r)

    def release(self, ticket: int):
        _check(lib().april_serve_release(self._h, ticket))

    def cancel(self, ticket: int):
        _check(lib().april_serve_cancel(self._h, ticket))

    def stats(self) -> dict:
        st = april_serve_stats_t()
        _check(lib().april_serve_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in april_serve_stats_t._fields_}

    def close(self):
        if self._h and not _exiting:
            lib().april_serve_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
