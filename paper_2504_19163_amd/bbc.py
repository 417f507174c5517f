"""Python binding of libbbc.so (include/bbc.h): argument marshalling only.

Device memory and streams come from PyTorch (ROCm); every step of the method
runs in the library's HIP kernels.  Importing this module does not need a GPU;
calling into the library does, and fails loudly if libbbc.so was not built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbbc.so")

OK, EINVAL, ENOMEM, EBUDGET, EDEVICE, EUNSUPPORTED, EQUEUE = 0, -1, -2, -3, -4, -5, -6
CHAIN = {"R": 0, "T": 1, "RR": 2}
MEM_HOST, MEM_DEVICE = 0, 1
FLAG_FIXED_DEPTH, FLAG_NO_REMAINDER, FLAG_IMPLICIT_IRR, FLAG_DEGREE_REDUCTION = 1, 2, 4, 8
QUERY_FUSED, QUERY_STAGED, QUERY_EXHAUSTIVE = 0, 1, 16
QUERY_UNIFORM, QUERY_ONE_SAMPLE, QUERY_BINS = 32, 64, 96

EXPORTS = [
    "bbc_build_bounds", "bbc_rebuild_bounds", "bbc_free_bounds", "bbc_bounds_info", "bbc_bounds_save",
    "bbc_bounds_load", "bbc_export_leaves",
    "bbc_export_grid", "bbc_query_irradiance", "bbc_query_irradiance_ex", "bbc_set_tuning", "bbc_get_tuning",
    "bbc_query_kernel_ms", "bbc_last_error", "bbc_server_create", "bbc_server_submit", "bbc_server_poll",
    "bbc_server_wait", "bbc_server_resume", "bbc_server_stats", "bbc_server_destroy",
    "bbc_query_irradiance_noalloc", "bbc_build_kernel_ms", "bbc_export_tuples",
]
SERVER_PAUSED, SERVER_GRAPH = 1, 2
TUNE_QUERY_WAVES, TUNE_QUERY_GRID, TUNE_BUILD_GRID_PER_CU, TUNE_QUERY_TILE, TUNE_TIMING = 1, 2, 3, 4, 5
TUNE_NEWTON_STEPS, TUNE_NEWTON_RESULTS, TUNE_STAGED_PAIRS, TUNE_GRAPH, TUNE_RR_OUTLINED = 6, 7, 8, 9, 10
TUNE_NEWTON_GRID_PER_CU, TUNE_BUILD_GRAPH, TUNE_SUBDIV_SPLIT = 11, 12, 13


class BBCError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where} failed with status {status}: {last_error()}")


class Scene(C.Structure):
    _fields_ = [
        ("chain", C.c_int32), ("memory", C.c_int32), ("n_tri", C.c_int64), ("pos", C.c_void_p), ("nrm", C.c_void_p),
        ("n_tri2", C.c_int64), ("pos2", C.c_void_p), ("nrm2", C.c_void_p), ("eta", C.c_float),
        ("q0", C.c_float * 3), ("f1", C.c_float * 3), ("f2", C.c_float * 3),
    ]


class Emitters(C.Structure):
    _fields_ = [("memory", C.c_int32), ("n", C.c_int64), ("pos", C.c_void_p), ("I0", C.c_void_p),
                ("edges", C.c_void_p)]


class SubdivParams(C.Structure):
    _fields_ = [
        ("max_depth", C.c_int32), ("sigma", C.c_float), ("alpha", C.c_float), ("grid_res", C.c_int32),
        ("init_pieces", C.c_int32), ("init_levels", C.c_int32), ("flags", C.c_int32), ("cover_frac", C.c_float),
    ]


class BoundsInfo(C.Structure):
    _fields_ = [
        ("n_tuples", C.c_int64), ("n_live_tuples", C.c_int64), ("n_boxes", C.c_int64), ("n_leaves", C.c_int64),
        ("n_grid_entries", C.c_int64), ("n_inf_leaves", C.c_int64), ("n_fp64_boxes", C.c_int64),
        ("device_bytes", C.c_int64), ("grid_res", C.c_int32), ("max_depth_reached", C.c_int32),
        ("n_cover_tuples", C.c_int64),
    ]


class QueryStats(C.Structure):
    _fields_ = [
        ("n_points", C.c_int64), ("sum_U", C.c_int64), ("sum_S", C.c_int64), ("n_roots", C.c_int64),
        ("n_newton", C.c_int64), ("sum_varbound", C.c_double), ("n_pairs", C.c_int64), ("n_iter_fp32", C.c_int64),
        ("n_iter_fp64", C.c_int64),
    ]


class ServerConfig(C.Structure):
    _fields_ = [
        ("hbm_budget_bytes", C.c_int64), ("max_inflight", C.c_int32), ("max_batch_points", C.c_int32),
        ("max_batch_requests", C.c_int32), ("queue_capacity", C.c_int32), ("mode", C.c_int32), ("flags", C.c_int32),
    ]


class Request(C.Structure):
    _fields_ = [
        ("memory", C.c_int32), ("scene", C.c_int32), ("n", C.c_int64), ("points", C.c_void_p), ("out", C.c_void_p),
        ("spp", C.c_int32), ("seed", C.c_uint64), ("point_index_base", C.c_int64),
    ]


class ServerCounters(C.Structure):
    _fields_ = [
        ("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64), ("batches", C.c_int64),
        ("points", C.c_int64), ("mean_batch_points", C.c_double), ("mean_batch_requests", C.c_double),
        ("latency_p50_ms", C.c_double), ("latency_p99_ms", C.c_double), ("latency_max_ms", C.c_double),
        ("batch_gpu_ms", C.c_double), ("arena_bytes", C.c_int64), ("arena_peak_bytes", C.c_int64),
        ("inflight_peak", C.c_int32), ("queue_peak", C.c_int32),
    ]


_lib = None


def lib():
    """Load libbbc.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2504_19163_amd.build_lib.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, u64 = C.c_void_p, C.c_int64, C.c_int32, C.c_uint64
        sig = {
            "bbc_build_bounds": [vp, vp, vp, vp, vp],
            "bbc_rebuild_bounds": [vp, vp, vp, vp, vp],
            "bbc_free_bounds": [vp],
            "bbc_bounds_info": [vp, vp],
            "bbc_bounds_save": [vp, C.c_char_p],
            "bbc_bounds_load": [C.c_char_p, vp, vp],
            "bbc_export_leaves": [vp, vp, vp, vp, vp, vp],
            "bbc_export_grid": [vp, vp, vp, vp],
            "bbc_export_tuples": [vp, vp, i64, vp],
            "bbc_query_irradiance": [vp, vp, i64, i32, u64, vp, vp, vp],
            "bbc_query_irradiance_ex": [vp, vp, i64, i32, u64, i64, i32, vp, vp, vp, vp],
            "bbc_query_irradiance_noalloc": [vp, vp, i64, i32, u64, i64, i32, vp, vp, vp],
            "bbc_set_tuning": [vp, i32, i64],
            "bbc_get_tuning": [vp, i32, vp],
            "bbc_query_kernel_ms": [vp, vp],
            "bbc_build_kernel_ms": [vp, vp, vp],
            "bbc_server_create": [vp, i32, vp, vp],
            "bbc_server_submit": [vp, vp, vp],
            "bbc_server_poll": [vp, u64, vp],
            "bbc_server_wait": [vp, u64, vp],
            "bbc_server_resume": [vp],
            "bbc_server_stats": [vp, vp, i32],
            "bbc_server_destroy": [vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int32
        L.bbc_last_error.argtypes = []
        L.bbc_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def last_error():
    if _lib is None:
        return ""
    return _lib.bbc_last_error().decode()


def _check(st, where):
    if st != OK:
        raise BBCError(st, where)


def default_params(max_depth=8, sigma=1e-4, alpha=2.0, grid_res=512, init_pieces=100, init_levels=4, flags=0,
                   cover_frac=0.5):
    return dict(max_depth=max_depth, sigma=sigma, alpha=alpha, grid_res=grid_res, init_pieces=init_pieces,
                init_levels=init_levels, flags=flags, cover_frac=cover_frac)


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class DeviceScene:
    """Scene arrays resident in device memory (torch tensors) and the C structs
    that point at them."""

    def __init__(self, scene, device="cuda"):
        import torch
        self.src = scene
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=device)
        self.pos = t(scene["pos"])
        self.nrm = t(scene["nrm"])
        self.epos = t(scene["epos"])
        self.eI = t(scene["eI"])
        s = Scene()
        s.chain = CHAIN[scene["chain"]]
        s.memory = MEM_DEVICE
        s.n_tri = self.pos.shape[1]
        s.pos = self.pos.data_ptr()
        s.nrm = self.nrm.data_ptr()
        s.n_tri2 = 0
        if "pos2" in scene:
            self.pos2 = t(scene["pos2"])
            self.nrm2 = t(scene["nrm2"])
            s.n_tri2 = self.pos2.shape[1]
            s.pos2 = self.pos2.data_ptr()
            s.nrm2 = self.nrm2.data_ptr()
        s.eta = float(scene["eta"])
        for k in ("q0", "f1", "f2"):
            getattr(s, k)[:] = [float(x) for x in scene[k]]
        e = Emitters()
        e.memory = MEM_DEVICE
        e.n = self.eI.shape[0]
        e.pos = self.epos.data_ptr()
        e.I0 = self.eI.data_ptr()
        if scene.get("eedge") is not None:  # area lights
            self.eedge = t(scene["eedge"])
            e.edges = self.eedge.data_ptr()
        self.c_scene = s
        self.c_emit = e
        self.n_tuples = s.n_tri * e.n * (s.n_tri2 if s.n_tri2 else 1)


class Bounds:
    """A device-resident bound hierarchy and receiver grid (bbc_build_bounds)."""

    def __init__(self, dscene, params=None, stream=None):
        self.dscene = dscene
        self.params = dict(default_params(), **(params or {}))
        self._p = SubdivParams(**self.params)
        h = C.c_void_p()
        _check(lib().bbc_build_bounds(C.byref(dscene.c_scene), C.byref(dscene.c_emit), C.byref(self._p),
                                      _stream_handle(stream), C.byref(h)), "bbc_build_bounds")
        self.h = h

    def save(self, path):
        """Write the hierarchy to a file (bbc_bounds_save)."""
        _check(lib().bbc_bounds_save(self.h, os.fsencode(path)), "bbc_bounds_save")

    @classmethod
    def load(cls, path, dscene=None, params=None, stream=None):
        """Read a file written by save() into a new handle on the current
        device (bbc_bounds_load).  `dscene` and `params` (optional) are what
        rebuild() will use; the loaded hierarchy itself carries its own."""
        self = cls.__new__(cls)
        self.dscene = dscene
        self.params = dict(default_params(), **(params or {}))
        self._p = SubdivParams(**self.params)
        h = C.c_void_p()
        _check(lib().bbc_bounds_load(os.fsencode(path), _stream_handle(stream), C.byref(h)), "bbc_bounds_load")
        self.h = h
        return self

    def rebuild(self, stream=None):
        _check(lib().bbc_rebuild_bounds(self.h, C.byref(self.dscene.c_scene), C.byref(self.dscene.c_emit),
                                        C.byref(self._p), _stream_handle(stream)), "bbc_rebuild_bounds")

    def free(self):
        if getattr(self, "h", None):
            lib().bbc_free_bounds(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def set_tuning(self, knob, value):
        _check(lib().bbc_set_tuning(self.h, int(knob), int(value)), "bbc_set_tuning")

    def get_tuning(self, knob):
        v = C.c_int64()
        _check(lib().bbc_get_tuning(self.h, int(knob), C.byref(v)), "bbc_get_tuning")
        return v.value

    def kernel_ms(self):
        v = C.c_float()
        _check(lib().bbc_query_kernel_ms(self.h, C.byref(v)), "bbc_query_kernel_ms")
        return v.value

    def build_kernel_ms(self):
        """(ms, launches) of the subdivision kernels of the last build."""
        v = C.c_float()
        n = C.c_int32()
        _check(lib().bbc_build_kernel_ms(self.h, C.byref(v), C.byref(n)), "bbc_build_kernel_ms")
        return v.value, n.value

    def info(self):
        i = BoundsInfo()
        _check(lib().bbc_bounds_info(self.h, C.byref(i)), "bbc_bounds_info")
        return {k: getattr(i, k) for k, _ in BoundsInfo._fields_}

    def leaves(self):
        n = self.info()["n_leaves"]
        t = np.zeros(n, np.uint32)
        c = np.zeros(n, np.uint32)
        box = np.zeros((n, 4), np.float32)
        uk = np.zeros((n, 4), np.float32)
        E = np.zeros((n, 2), np.float32)
        _check(lib().bbc_export_leaves(self.h, t.ctypes.data, c.ctypes.data, box.ctypes.data, uk.ctypes.data,
                                       E.ctypes.data), "bbc_export_leaves")
        depth = (c >> 28).astype(np.int32)
        iu = ((c >> 14) & 0x3FFF).astype(np.int32)
        iv = (c & 0x3FFF).astype(np.int32)
        return dict(tuple=t.astype(np.int64), code=np.stack([depth, iu, iv], 1), box=box, uk=uk, E=E)

    def tuples(self):
        """The tuple numbers the build works on (constructed pairs for two
        reflections), ascending."""
        n = C.c_int64()
        _check(lib().bbc_export_tuples(self.h, None, 0, C.byref(n)), "bbc_export_tuples")
        out = np.zeros(max(n.value, 1), np.uint32)
        _check(lib().bbc_export_tuples(self.h, out.ctypes.data, n.value, C.byref(n)), "bbc_export_tuples")
        return out[:n.value].astype(np.int64)

    def grid(self):
        """(offsets [G*G + 2], tuples, E~): slices 0 .. G*G - 1 are the cells,
        slice G*G the cover-all list."""
        info = self.info()
        G = info["grid_res"]
        off = np.zeros(G * G + 2, np.uint32)
        t = np.zeros(max(info["n_grid_entries"], 1), np.uint32)
        e = np.zeros(max(info["n_grid_entries"], 1), np.float32)
        _check(lib().bbc_export_grid(self.h, off.ctypes.data, t.ctypes.data, e.ctypes.data), "bbc_export_grid")
        n = info["n_grid_entries"]
        return off, t[:n], e[:n]

    def query(self, points, spp, seed, mode=QUERY_FUSED, out=None, stats=False, point_index_base=0, stream=None,
              host_stats=False):
        """points: torch float32 [3, n] on the GPU.  Returns (E [n], stats [n,4] or None)."""
        import torch
        assert points.is_cuda and points.dtype == torch.float32 and points.dim() == 2 and points.shape[0] == 3
        points = points.contiguous()
        n = points.shape[1]
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=points.device)
        st = torch.zeros((n, 4), dtype=torch.float32, device=points.device) if stats else None
        hs = QueryStats() if host_stats else None
        _check(lib().bbc_query_irradiance_ex(self.h, points.data_ptr(), n, int(spp), int(seed),
                                             int(point_index_base), int(mode), out.data_ptr(),
                                             st.data_ptr() if st is not None else None,
                                             C.byref(hs) if hs is not None else None, _stream_handle(stream)),
               "bbc_query_irradiance_ex")
        if host_stats:
            return out, st, {k: getattr(hs, k) for k, _ in QueryStats._fields_}
        return out, st


    def query_noalloc(self, points, spp, seed, mode=QUERY_STAGED, out=None, stats=False, point_index_base=0,
                      stream=None):
        """The staged query over the library's own device work space
        (bbc_query_irradiance_noalloc); `out` and the stats array are
        allocated here when not given."""
        import torch
        assert points.is_cuda and points.dtype == torch.float32 and points.dim() == 2 and points.shape[0] == 3
        points = points.contiguous()
        n = points.shape[1]
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=points.device)
        st = torch.zeros((n, 4), dtype=torch.float32, device=points.device) if stats else None
        _check(lib().bbc_query_irradiance_noalloc(self.h, points.data_ptr(), n, int(spp), int(seed),
                                                  int(point_index_base), int(mode), out.data_ptr(),
                                                  st.data_ptr() if st is not None else None, _stream_handle(stream)),
               "bbc_query_irradiance_noalloc")
        return out, st


class Server:
    """Continuous-batching server over resident bounds (bbc_server_*).

    submit() takes points as a numpy [3, n] float32 array (host request) or a
    torch CUDA tensor (device request) and returns a ticket; the output array
    is allocated here and kept alive until wait() returns it."""

    def __init__(self, bounds, hbm_budget_bytes=8 << 30, max_inflight=4, max_batch_points=262144,
                 max_batch_requests=4096, queue_capacity=4096, mode=0, paused=False, graph=False):
        self.bounds = list(bounds)  # keeps the handles alive
        arr = (C.c_void_p * len(self.bounds))(*[b.h.value for b in self.bounds])
        cfg = ServerConfig(int(hbm_budget_bytes), int(max_inflight), int(max_batch_points), int(max_batch_requests),
                           int(queue_capacity), int(mode),
                           (SERVER_PAUSED if paused else 0) | (SERVER_GRAPH if graph else 0))
        h = C.c_void_p()
        _check(lib().bbc_server_create(arr, len(self.bounds), C.byref(cfg), C.byref(h)), "bbc_server_create")
        self.h = h
        self._live = {}

    def submit(self, scene, points, spp, seed, point_index_base=0, sync_inputs=True):
        """Queue a request; returns its ticket.  Raises BBCError (status
        EBUDGET / EQUEUE / EINVAL) when it is not accepted.  Device points must
        be complete before the server's streams read them: sync_inputs=True
        synchronises torch's current stream first."""
        r = Request()
        r.scene = int(scene)
        r.spp = int(spp)
        r.seed = int(seed)
        r.point_index_base = int(point_index_base)
        if isinstance(points, np.ndarray):
            pts = np.ascontiguousarray(points, dtype=np.float32)
            assert pts.ndim == 2 and pts.shape[0] == 3
            out = np.zeros(pts.shape[1], np.float32)
            r.memory = MEM_HOST
            r.points = pts.ctypes.data
            r.out = out.ctypes.data
        else:
            import torch
            pts = points.contiguous()
            assert pts.is_cuda and pts.dtype == torch.float32 and pts.dim() == 2 and pts.shape[0] == 3
            out = torch.empty(pts.shape[1], dtype=torch.float32, device=pts.device)
            if sync_inputs:
                torch.cuda.current_stream().synchronize()
            r.memory = MEM_DEVICE
            r.points = pts.data_ptr()
            r.out = out.data_ptr()
        r.n = pts.shape[1]
        t = C.c_uint64()
        _check(lib().bbc_server_submit(self.h, C.byref(r), C.byref(t)), "bbc_server_submit")
        self._live[t.value] = (pts, out)
        return t.value

    def poll(self, ticket):
        """(done, out or None)."""
        d = C.c_int32()
        st = lib().bbc_server_poll(self.h, C.c_uint64(ticket), C.byref(d))
        if d.value:
            pts, out = self._live.pop(ticket)
            _check(st, "bbc_server_poll")
            return True, out
        _check(st, "bbc_server_poll")
        return False, None

    def wait(self, ticket):
        """Block until the request is complete; returns (out, latency_ms)."""
        lat = C.c_double()
        st = lib().bbc_server_wait(self.h, C.c_uint64(ticket), C.byref(lat))
        pts, out = self._live.pop(ticket)
        _check(st, "bbc_server_wait")
        return out, lat.value

    def resume(self):
        _check(lib().bbc_server_resume(self.h), "bbc_server_resume")

    def stats(self, reset=False):
        c = ServerCounters()
        _check(lib().bbc_server_stats(self.h, C.byref(c), 1 if reset else 0), "bbc_server_stats")
        return {k: getattr(c, k) for k, _ in ServerCounters._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().bbc_server_destroy(self.h)
            self.h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


TUNING_FILE = os.path.join(HERE, "tuning.json")


def tuned_value(workload_key, knob, default, path=TUNING_FILE):
    """One recorded choice for this device (see apply_tuning), or default."""
    import json
    if not os.path.exists(path):
        return default
    import torch
    dev = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    with open(path) as f:
        return json.load(f).get(dev, {}).get(workload_key, {}).get(knob, default)


def apply_tuning(bounds, workload_key, path=TUNING_FILE):
    """Apply launch-shape choices recorded for this device and workload in a
    JSON table ({arch: {workload: {knob: value}}}, tuning.json beside this
    module, written by autotune.py on the GPU); returns the chosen entry, or {}
    when none was recorded.  Results never depend on these knobs."""
    import json
    if not os.path.exists(path):
        return {}
    import torch
    dev = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    table = json.load(open(path))
    entry = table.get(dev, {}).get(workload_key, {})
    knobs = {"query_waves": TUNE_QUERY_WAVES, "query_tile": TUNE_QUERY_TILE, "query_grid": TUNE_QUERY_GRID,
             "build_grid_per_cu": TUNE_BUILD_GRID_PER_CU, "newton_steps": TUNE_NEWTON_STEPS, "graph": TUNE_GRAPH,
             "newton_grid_per_cu": TUNE_NEWTON_GRID_PER_CU, "build_graph": TUNE_BUILD_GRAPH,
             "subdiv_split": TUNE_SUBDIV_SPLIT}
    for k, knob in knobs.items():
        if k in entry:
            bounds.set_tuning(knob, entry[k])
    return entry
