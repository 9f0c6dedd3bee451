"""Python binding of libmxr.so (include/mxr.h): argument marshalling only.

Every step of the tracing runs in the library's HIP kernels; this module
turns instrument dicts (see ``workloads``) into ``mxr_component_desc``
structs, hands device pointers of torch tensors and the current HIP stream
to the C ABI, and raises ``MxrError`` on a negative status.  torch provides
device memory and streams only.  If the library is missing the import fails:
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmxr.so")

MXR_ABI_VERSION = 1
MAX_COMPONENTS = 16

TYPE_CODES = {
    "source_rect_cone": 0,
    "source_cone_beam": 1,
    "source_gaussian": 2,
    "slit": 3,
    "box": 4,
    "phantom": 5,
    "mirror_elliptic": 6,
    "dcm": 7,
    "powder": 8,
    "detector": 9,
}
STATUS_EXITED = 1
STATUS_ABSORBED = 2


class MxrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mxr status {status}: {msg}")
        self.status = status


class mxr_component_desc(ctypes.Structure):
    _fields_ = [
        ("type", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("pos", ctypes.c_double * 3),
        ("rot", ctypes.c_double * 9),
        ("par", ctypes.c_double * 16),
        ("data", ctypes.c_void_p * 2),
        ("data_len", ctypes.c_uint64 * 2),
        ("dims", ctypes.c_uint32 * 4),
    ]


class mxr_instrument_desc(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32),
        ("n_components", ctypes.c_uint32),
        ("components", ctypes.POINTER(mxr_component_desc)),
    ]


class mxr_tally(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_void_p),
        ("sum_w", ctypes.c_void_p),
        ("sum_w2", ctypes.c_void_p),
        ("n_bins", ctypes.c_uint64),
    ]


class mxr_ray_soa(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("x", "y", "z", "dx", "dy", "dz", "E", "w", "status", "dead_at", "bin")]


MAX_DETECTORS = 4


class mxr_batch_job(ctypes.Structure):
    _fields_ = [
        ("instrument", ctypes.c_void_p),
        ("n_rays", ctypes.c_uint64),
        ("seed", ctypes.c_uint64),
        ("job", ctypes.c_uint32),
        ("tallies", mxr_tally * MAX_DETECTORS),
    ]


class mxr_batch_schedule(ctypes.Structure):
    _fields_ = [("groups_per_cu", ctypes.c_uint32), ("tile_rays", ctypes.c_uint32)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2410_08747_amd/build.py (or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    lib.mxr_abi_version.restype = ctypes.c_uint32
    lib.mxr_last_error.restype = ctypes.c_char_p
    lib.mxr_instrument_create.argtypes = [ctypes.POINTER(mxr_instrument_desc), ctypes.POINTER(ctypes.c_void_p)]
    lib.mxr_instrument_create.restype = ctypes.c_int
    lib.mxr_instrument_destroy.argtypes = [ctypes.c_void_p]
    lib.mxr_instrument_destroy.restype = None
    lib.mxr_run.argtypes = [
        ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
        ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(mxr_tally), ctypes.c_uint32, ctypes.c_void_p,
        ctypes.c_void_p,
    ]
    lib.mxr_run.restype = ctypes.c_int
    lib.mxr_trace_rays.argtypes = [
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
        ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(mxr_ray_soa), ctypes.c_void_p,
    ]
    lib.mxr_trace_rays.restype = ctypes.c_int
    lib.mxr_batch_create.argtypes = [ctypes.POINTER(mxr_batch_job), ctypes.c_uint32,
                                     ctypes.POINTER(mxr_batch_schedule), ctypes.POINTER(ctypes.c_void_p)]
    lib.mxr_batch_create.restype = ctypes.c_int
    lib.mxr_batch_run.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.mxr_batch_run.restype = ctypes.c_int
    lib.mxr_batch_get_schedule.argtypes = [ctypes.c_void_p, ctypes.POINTER(mxr_batch_schedule)]
    lib.mxr_batch_get_schedule.restype = ctypes.c_int
    lib.mxr_batch_set_schedule.argtypes = [ctypes.c_void_p, ctypes.POINTER(mxr_batch_schedule)]
    lib.mxr_batch_set_schedule.restype = ctypes.c_int
    lib.mxr_batch_destroy.argtypes = [ctypes.c_void_p]
    lib.mxr_batch_destroy.restype = None
    lib.mxr_batch_autotune.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_char_p,
                                       ctypes.POINTER(mxr_batch_schedule)]
    lib.mxr_batch_autotune.restype = ctypes.c_int
    if lib.mxr_abi_version() != MXR_ABI_VERSION:
        raise ImportError(f"libmxr ABI {lib.mxr_abi_version()} != binding {MXR_ABI_VERSION}")
    return lib


lib = _load()


def _check(status: int) -> None:
    if status < 0:
        raise MxrError(status, lib.mxr_last_error().decode())


def _stream_handle(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


# ------------------------------------------------------- C ABI, same names --

def mxr_abi_version() -> int:
    return int(lib.mxr_abi_version())


def mxr_last_error() -> str:
    return lib.mxr_last_error().decode()


def mxr_instrument_create(desc: mxr_instrument_desc) -> int:
    h = ctypes.c_void_p()
    _check(lib.mxr_instrument_create(ctypes.byref(desc), ctypes.byref(h)))
    return h.value


def mxr_instrument_destroy(handle: int) -> None:
    lib.mxr_instrument_destroy(handle)


def mxr_run(handle: int, first_ray: int, n_rays: int, n_total: int, seed: int, purpose: int, job: int,
            tallies: Sequence[mxr_tally], ledger_ptr: Optional[int] = None, stream=None) -> None:
    arr = (mxr_tally * max(1, len(tallies)))(*tallies)
    _check(lib.mxr_run(handle, first_ray, n_rays, n_total, seed, purpose, job, arr, len(tallies),
                       ledger_ptr, _stream_handle(stream)))


def mxr_trace_rays(handle: int, ids_ptr: int, n: int, n_total: int, seed: int, purpose: int, job: int,
                   out: mxr_ray_soa, stream=None) -> None:
    _check(lib.mxr_trace_rays(handle, ids_ptr, n, n_total, seed, purpose, job, ctypes.byref(out),
                              _stream_handle(stream)))


def mxr_batch_create(jobs: Sequence[mxr_batch_job], schedule: Optional[mxr_batch_schedule] = None) -> int:
    arr = (mxr_batch_job * max(1, len(jobs)))(*jobs)
    h = ctypes.c_void_p()
    _check(lib.mxr_batch_create(arr, len(jobs), ctypes.byref(schedule) if schedule is not None else None,
                                ctypes.byref(h)))
    return h.value


def mxr_batch_run(handle: int, stream=None) -> None:
    _check(lib.mxr_batch_run(handle, _stream_handle(stream)))


def mxr_batch_get_schedule(handle: int) -> mxr_batch_schedule:
    out = mxr_batch_schedule()
    _check(lib.mxr_batch_get_schedule(handle, ctypes.byref(out)))
    return out


def mxr_batch_set_schedule(handle: int, schedule: mxr_batch_schedule) -> None:
    _check(lib.mxr_batch_set_schedule(handle, ctypes.byref(schedule)))


def mxr_batch_destroy(handle: int) -> None:
    lib.mxr_batch_destroy(handle)


def mxr_batch_autotune(handle: int, rays_fraction: float, cache_path: Optional[str] = None) -> mxr_batch_schedule:
    out = mxr_batch_schedule()
    _check(lib.mxr_batch_autotune(handle, rays_fraction, cache_path.encode() if cache_path else None,
                                  ctypes.byref(out)))
    return out


# ------------------------------------------------------------ marshalling --

def _params(c: Dict, s: mxr_component_desc, upload) -> None:
    t = c["type"]
    p = s.par
    if t == "source_rect_cone":
        p[0], p[1], p[2], p[3], p[4] = c["wx"], c["wy"], c["half_angle"], c["emin"], c["emax"]
    elif t == "source_cone_beam":
        vals = [c["half_angle"], c["emin"], c["emax"], c["e0"], c["f_cont"], c["e_line1"], c["f_line1"],
                c["e_line2"], c["f_line2"], c["line_sigma"]]
        for i, v in enumerate(vals):
            p[i] = v
        s.dims[0] = int(c.get("strata", 1))
    elif t == "source_gaussian":
        vals = [c["sigma_x"], c["sigma_y"], c["sigma_xp"], c["sigma_yp"], c["e0"], c["rel_halfwidth"]]
        for i, v in enumerate(vals):
            p[i] = v
    elif t == "slit":
        if c.get("circular", False):
            s.flags = 1
            p[2] = c["radius"]
        else:
            p[0], p[1] = c["w"], c["h"]
    elif t == "box":
        p[0], p[1], p[2], p[3], p[4] = c["hx"], c["hy"], c["hz"], c["mu_a"], c["mu_b"]
    elif t == "phantom":
        vol = c["volume"]
        nz, ny, nx = vol.shape
        mu = np.asarray(c["mu_table"], dtype=np.float64)
        s.data[0], s.data_len[0] = upload(vol, np.uint8)
        s.data[1], s.data_len[1] = upload(mu, np.float64)
        s.dims[0], s.dims[1], s.dims[2], s.dims[3] = nx, ny, nz, mu.shape[0]
        p[0], p[1], p[2] = c["voxel"], c["table_emin"], c["table_emax"]
    elif t == "mirror_elliptic":
        s.data[0], s.data_len[0] = upload(c["reflectivity"], np.float64)
        p[0], p[1], p[2], p[3], p[4], p[5] = c["p"], c["q"], c["theta0"], c["length"], c["width"], c["theta_max"]
    elif t == "dcm":
        p[0], p[1], p[2], p[3] = c["d_spacing"], c["theta_c"], c["darwin_width"], c["gap"]
    elif t == "powder":
        s.data[0], s.data_len[0] = upload(c["d_spacings"], np.float64)
        p[0], p[1] = c["w"], c["h"]
    elif t == "detector":
        p[0], p[1], p[2], p[3], p[4], p[5] = c["xmin"], c["xmax"], c["ymin"], c["ymax"], c["emin"], c["emax"]
        s.dims[0], s.dims[1], s.dims[2] = c["nx"], c["ny"], c["ne"]
        s.flags = 1 if c.get("wavelength", False) else 0
    else:
        raise ValueError(f"unknown component type {t}")


class Instrument:
    """An instrument on the current device: uploads the dict's arrays once
    (torch tensors own them) and holds the library handle."""

    def __init__(self, instr: Dict, device=None, shared: Optional[Dict] = None):
        """``shared``: a dict reused across instruments so that the same
        numpy array (e.g. one phantom seen at many angles) is uploaded once."""
        import torch
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self._tensors: List = []
        comps = instr["components"]
        self.n_components = len(comps)
        descs = (mxr_component_desc * len(comps))()
        self.detectors: List[Dict] = []

        def upload(arr, dtype):
            key = (id(arr), np.dtype(dtype).str)
            if shared is not None and key in shared:
                t = shared[key][1]
            else:
                a = np.ascontiguousarray(np.asarray(arr, dtype=dtype))
                t = torch.from_numpy(a.reshape(-1)).to(self.device)
                if shared is not None:
                    shared[key] = (arr, t)  # holding arr keeps its id unique
            self._tensors.append(t)
            return t.data_ptr(), t.numel()

        for k, c in enumerate(comps):
            s = descs[k]
            s.type = TYPE_CODES[c["type"]]
            pos = c.get("pos", (0.0, 0.0, 0.0))
            rot = np.asarray(c.get("rot", np.eye(3)), dtype=np.float64).reshape(9)
            for i in range(3):
                s.pos[i] = float(pos[i])
            for i in range(9):
                s.rot[i] = float(rot[i])
            _params(c, s, upload)
            if c["type"] == "detector":
                self.detectors.append(c)
        desc = mxr_instrument_desc(MXR_ABI_VERSION, len(comps), descs)
        with torch.cuda.device(self.device):
            self.handle = mxr_instrument_create(desc)

    def close(self) -> None:
        """Free the library handle (also done on garbage collection)."""
        h = getattr(self, "handle", None)
        if h and lib is not None:
            lib.mxr_instrument_destroy(h)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass  # interpreter shutdown: module globals may already be gone

    def new_tallies(self):
        """Zeroed histograms (count, sum_w, sum_w2) for every monitor."""
        import torch
        out = []
        for d in self.detectors:
            nb = int(d["nx"]) * int(d["ny"]) * int(d["ne"])
            out.append({
                "count": torch.zeros(nb, dtype=torch.int64, device=self.device),
                "sum_w": torch.zeros(nb, dtype=torch.float64, device=self.device),
                "sum_w2": torch.zeros(nb, dtype=torch.float64, device=self.device),
            })
        return out

    @staticmethod
    def tally_structs(tallies) -> List[mxr_tally]:
        return [mxr_tally(t["count"].data_ptr(), t["sum_w"].data_ptr(), t["sum_w2"].data_ptr(), t["count"].numel())
                for t in tallies]

    def run(self, n_rays: int, seed: int, first_ray: int = 0, n_total: Optional[int] = None, purpose: int = 0,
            job: int = 0, tallies=None, ledger=None, stream=None):
        """Trace rays [first_ray, first_ray + n_rays) of an n_total-ray run,
        adding into ``tallies`` (new zeroed ones if None).  Asynchronous."""
        n_total = n_rays if n_total is None else n_total
        if tallies is None:
            tallies = self.new_tallies()
        mxr_run(self.handle, first_ray, n_rays, n_total, seed, purpose, job, self.tally_structs(tallies),
                ledger.data_ptr() if ledger is not None else None, stream)
        return tallies

    def new_ledger(self):
        import torch
        return torch.zeros(4 * self.n_components + 1, dtype=torch.float64, device=self.device)

    def trace_rays(self, ids, seed: int, n_total: int, purpose: int = 0, job: int = 0, stream=None):
        """Final state of each listed ray (device tensors)."""
        import torch
        ids = torch.as_tensor(np.asarray(ids, dtype=np.uint64).view(np.int64)).to(self.device)
        n = ids.numel()
        f64 = lambda: torch.empty(n, dtype=torch.float64, device=self.device)
        out = {k: f64() for k in ("x", "y", "z", "dx", "dy", "dz", "E", "w")}
        out["status"] = torch.empty(n, dtype=torch.int32, device=self.device)
        out["dead_at"] = torch.empty(n, dtype=torch.int32, device=self.device)
        out["bin"] = torch.empty(n, dtype=torch.int64, device=self.device)
        soa = mxr_ray_soa(*[out[k].data_ptr() for k in ("x", "y", "z", "dx", "dy", "dz", "E", "w", "status",
                                                         "dead_at", "bin")])
        mxr_trace_rays(self.handle, ids.data_ptr(), n, n_total, seed, purpose, job, soa, stream)
        return out


class Batch:
    """Many runs of instruments with one component chain (e.g. every angle
    of every phantom of a CT acquisition) traced by one captured launch.

    ``jobs`` is a list of (Instrument, n_rays, seed, job, tallies); the
    instruments and tallies must stay alive as long as the batch."""

    def __init__(self, jobs, schedule=None):
        self._keep = [(j[0], j[4]) for j in jobs]
        structs = []
        for instr, n_rays, seed, job, tallies in jobs:
            ts = Instrument.tally_structs(tallies)
            js = mxr_batch_job(instr.handle, n_rays, seed, job)
            for i, t in enumerate(ts):
                js.tallies[i] = t
            structs.append(js)
        sched = None if schedule is None else mxr_batch_schedule(*schedule)
        self.handle = mxr_batch_create(structs, sched)

    def run(self, stream=None) -> None:
        """Trace every job once, adding into its tallies.  Asynchronous."""
        mxr_batch_run(self.handle, stream)

    @property
    def schedule(self):
        s = mxr_batch_get_schedule(self.handle)
        return (s.groups_per_cu, s.tile_rays)

    @schedule.setter
    def schedule(self, value) -> None:
        mxr_batch_set_schedule(self.handle, mxr_batch_schedule(*value))

    def autotune(self, rays_fraction: float, cache_path: Optional[str] = None):
        """Pick the fastest launch shape (timing runs add into the tallies)."""
        s = mxr_batch_autotune(self.handle, rays_fraction, cache_path)
        return (s.groups_per_cu, s.tile_rays)

    def close(self) -> None:
        h = getattr(self, "handle", None)
        if h and lib is not None:
            lib.mxr_batch_destroy(h)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
