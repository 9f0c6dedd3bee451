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

MXR_ABI_VERSION = 2
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
    "lens_crl": 10,
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


BATCH_GRID, BATCH_PERSISTENT, BATCH_LAUNCHES = 0, 1, 2


class mxr_batch_schedule(ctypes.Structure):
    _fields_ = [("form", ctypes.c_uint32), ("groups_per_cu", ctypes.c_uint32), ("tile_rays", ctypes.c_uint32),
                ("branches", ctypes.c_uint32)]


MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS = 6, 128, 56, 24632
MLP_NOALLOC_ROWS = 4096
WS_REGIONS = ("X", "Z1", "H1", "Z2", "H2", "O", "DO", "DOH", "DZ2", "DZ2H", "DZ1", "DZ1H", "PARTIAL", "Y", "W",
              "ROWLOSS", "SCALARS", "WT", "COLS")


class mxr_launch_shape(ctypes.Structure):
    _fields_ = [("occupancy", ctypes.c_uint32), ("compact", ctypes.c_uint32), ("rounds", ctypes.c_uint32),
                ("xcd_order", ctypes.c_uint32)]


class mxr_train_cfg(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("batch", ctypes.c_uint32), ("epochs", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("first_step", ctypes.c_uint32)]


class mxr_train_rows(ctypes.Structure):
    _fields_ = [
        ("ctx", ctypes.c_void_p),
        ("y", ctypes.c_void_p),
        ("w", ctypes.c_void_p),
        ("bin", ctypes.c_void_p),
        ("n_rows", ctypes.c_uint64),
        ("n_runs", ctypes.c_uint32),
        ("run_first", ctypes.POINTER(ctypes.c_uint64)),
        ("run_image", ctypes.POINTER(ctypes.c_void_p)),
        ("n_bins", ctypes.c_uint64),
        ("floor_frac", ctypes.c_double),
    ]


class mxr_hits(ctypes.Structure):
    _fields_ = [
        ("ctx", ctypes.c_void_p),
        ("y", ctypes.c_void_p),
        ("w", ctypes.c_void_p),
        ("bin", ctypes.c_void_p),
        ("capacity", ctypes.c_uint64),
        ("count", ctypes.c_void_p),
        ("context", ctypes.c_float * 6),
    ]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2410_08747_amd/build.py (or __graft_entry__.build())")
    # torch ships its own HIP and HSA runtimes under the same sonames as the
    # system ROCm libraries this library links.  Loading torch first makes
    # libmxr.so bind to the runtime torch already uses; loading libmxr.so
    # first would put two HIP runtimes on one HSA runtime in the process, and
    # one of them then finds no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    lib.mxr_peak_launch.argtypes = [ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
    lib.mxr_peak_launch.restype = ctypes.c_int
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
    lib.mxr_proposal_set.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double]
    lib.mxr_proposal_set.restype = ctypes.c_int
    lib.mxr_collect.argtypes = [
        ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
        ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(mxr_tally), ctypes.c_uint32, ctypes.POINTER(mxr_hits),
        ctypes.c_void_p,
    ]
    lib.mxr_collect.restype = ctypes.c_int
    P, U64, D3 = ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)
    lib.mxr_mlp_workspace_bytes.argtypes = [U64]
    lib.mxr_mlp_workspace_bytes.restype = U64
    lib.mxr_mlp_workspace_layout.argtypes = [U64, P]
    lib.mxr_mlp_workspace_layout.restype = ctypes.c_int
    lib.mxr_mlp_to_bf16.argtypes = [P, U64, P, P]
    lib.mxr_mlp_to_bf16.restype = ctypes.c_int
    lib.mxr_mlp_forward.argtypes = [P, P, U64, P, P, U64, P]
    lib.mxr_mlp_forward.restype = ctypes.c_int
    lib.mxr_mlp_forward_noalloc.argtypes = [P, P, U64, P, P]
    lib.mxr_mlp_forward_noalloc.restype = ctypes.c_int
    lib.mxr_mlp_mixture.argtypes = [P, U64, D3, D3, P, P]
    lib.mxr_mlp_mixture.restype = ctypes.c_int
    lib.mxr_mlp_loss_grad.argtypes = [P, P, P, P, U64, D3, D3, P, P, P, U64, P]
    lib.mxr_mlp_loss_grad.restype = ctypes.c_int
    lib.mxr_adam_step.argtypes = [P, P, P, P, P, U64, ctypes.c_uint32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_float, P]
    lib.mxr_adam_step.restype = ctypes.c_int
    lib.mxr_train_weights.argtypes = [P, P, U64, P, U64, ctypes.c_double, P, P, P]
    lib.mxr_train_weights.restype = ctypes.c_int
    lib.mxr_mlp_train.argtypes = [P, P, P, U64, ctypes.POINTER(mxr_train_cfg), D3, D3, P, P, P, P, P, P, U64, P, P]
    lib.mxr_mlp_train.restype = ctypes.c_int
    lib.mxr_get_launch_shape.argtypes = [P, ctypes.POINTER(mxr_launch_shape)]
    lib.mxr_get_launch_shape.restype = ctypes.c_int
    lib.mxr_set_launch_shape.argtypes = [P, ctypes.POINTER(mxr_launch_shape)]
    lib.mxr_set_launch_shape.restype = ctypes.c_int
    lib.mxr_autotune_instrument.argtypes = [P, U64, ctypes.c_double, ctypes.POINTER(mxr_tally), ctypes.c_uint32,
                                            ctypes.c_char_p, ctypes.POINTER(mxr_launch_shape)]
    lib.mxr_autotune_instrument.restype = ctypes.c_int
    lib.mxr_proposal_box.argtypes = [P, D3, D3]
    lib.mxr_proposal_box.restype = ctypes.c_int
    lib.mxr_proposal_train.argtypes = [P, ctypes.POINTER(mxr_train_rows), ctypes.POINTER(mxr_train_cfg), P, P, P, P,
                                       P, P, P, U64, P, P]
    lib.mxr_proposal_train.restype = ctypes.c_int
    lib.mxr_proposal_apply.argtypes = [P, P, ctypes.POINTER(ctypes.c_float), ctypes.c_double, P, U64, P]
    lib.mxr_proposal_apply.restype = ctypes.c_int
    lib.mxr_batch_means.argtypes = [P, ctypes.c_uint32, U64, U64, P, P, P]
    lib.mxr_batch_means.restype = ctypes.c_int
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


def mxr_proposal_set(handle: int, gmm_ptr: Optional[int], alpha: float) -> None:
    _check(lib.mxr_proposal_set(handle, gmm_ptr, alpha))


def mxr_collect(handle: int, first_ray: int, n_rays: int, n_total: int, seed: int, purpose: int, job: int,
                tallies: Sequence[mxr_tally], hits: mxr_hits, stream=None) -> None:
    arr = (mxr_tally * max(1, len(tallies)))(*tallies)
    _check(lib.mxr_collect(handle, first_ray, n_rays, n_total, seed, purpose, job, arr, len(tallies),
                           ctypes.byref(hits), _stream_handle(stream)))


def _d3(v):
    return (ctypes.c_double * 3)(*[float(x) for x in v])


def mxr_mlp_workspace_bytes(batch: int) -> int:
    return int(lib.mxr_mlp_workspace_bytes(batch))


def mxr_mlp_workspace_layout(batch: int) -> List[int]:
    off = (ctypes.c_uint64 * len(WS_REGIONS))()
    _check(lib.mxr_mlp_workspace_layout(batch, off))
    return [int(x) for x in off]


def mxr_mlp_to_bf16(x_ptr: int, n: int, y_ptr: int, stream=None) -> None:
    _check(lib.mxr_mlp_to_bf16(x_ptr, n, y_ptr, _stream_handle(stream)))


def mxr_mlp_forward(w_ptr, ctx_ptr, n, out_ptr, ws_ptr, ws_bytes, stream=None) -> None:
    _check(lib.mxr_mlp_forward(w_ptr, ctx_ptr, n, out_ptr, ws_ptr, ws_bytes, _stream_handle(stream)))


def mxr_mlp_forward_noalloc(w_ptr, ctx_ptr, n, out_ptr, stream=None) -> None:
    _check(lib.mxr_mlp_forward_noalloc(w_ptr, ctx_ptr, n, out_ptr, _stream_handle(stream)))


def mxr_mlp_mixture(out_ptr, n, lo, hi, gmm_ptr, stream=None) -> None:
    _check(lib.mxr_mlp_mixture(out_ptr, n, _d3(lo), _d3(hi), gmm_ptr, _stream_handle(stream)))


def mxr_mlp_loss_grad(w_ptr, ctx_ptr, y_ptr, omega_ptr, n, lo, hi, grad_ptr, loss_ptr, ws_ptr, ws_bytes,
                      stream=None) -> None:
    _check(lib.mxr_mlp_loss_grad(w_ptr, ctx_ptr, y_ptr, omega_ptr, n, _d3(lo), _d3(hi), grad_ptr, loss_ptr, ws_ptr,
                                 ws_bytes, _stream_handle(stream)))


def mxr_adam_step(master, w, grad, m, v, n_params, step, lr, beta1, beta2, eps, stream=None) -> None:
    _check(lib.mxr_adam_step(master, w, grad, m, v, n_params, step, lr, beta1, beta2, eps, _stream_handle(stream)))


def mxr_train_weights(w, bin_, n, sum_w, n_bins, floor_frac, omega, scratch, stream=None) -> None:
    _check(lib.mxr_train_weights(w, bin_, n, sum_w, n_bins, floor_frac, omega, scratch, _stream_handle(stream)))


def mxr_mlp_train(ctx, y, omega, n_rows, cfg: mxr_train_cfg, lo, hi, master, w, m, v, grad, ws, ws_bytes, loss_log,
                  stream=None) -> None:
    _check(lib.mxr_mlp_train(ctx, y, omega, n_rows, ctypes.byref(cfg), _d3(lo), _d3(hi), master, w, m, v, grad, ws,
                             ws_bytes, loss_log, _stream_handle(stream)))


def mxr_get_launch_shape(handle: int) -> mxr_launch_shape:
    out = mxr_launch_shape()
    _check(lib.mxr_get_launch_shape(handle, ctypes.byref(out)))
    return out


def mxr_set_launch_shape(handle: int, shape: mxr_launch_shape) -> None:
    _check(lib.mxr_set_launch_shape(handle, ctypes.byref(shape)))


def mxr_autotune_instrument(handle: int, n_total: int, rays_fraction: float, tallies: Sequence[mxr_tally],
                            cache_path: Optional[str] = None) -> mxr_launch_shape:
    arr = (mxr_tally * max(1, len(tallies)))(*tallies)
    out = mxr_launch_shape()
    _check(lib.mxr_autotune_instrument(handle, n_total, rays_fraction, arr, len(tallies),
                                       cache_path.encode() if cache_path else None, ctypes.byref(out)))
    return out


def mxr_proposal_box(handle: int):
    lo, hi = (ctypes.c_double * 3)(), (ctypes.c_double * 3)()
    _check(lib.mxr_proposal_box(handle, lo, hi))
    return tuple(lo), tuple(hi)


def mxr_proposal_train(handle: int, rows: mxr_train_rows, cfg: mxr_train_cfg, master, w, m, v, grad, omega, ws,
                       ws_bytes, loss_log, stream=None) -> None:
    _check(lib.mxr_proposal_train(handle, ctypes.byref(rows), ctypes.byref(cfg), master, w, m, v, grad, omega, ws,
                                  ws_bytes, loss_log, _stream_handle(stream)))


def mxr_proposal_apply(handle: int, w, context, alpha: float, ws, ws_bytes, stream=None) -> None:
    c = (ctypes.c_float * 6)(*[float(x) for x in context])
    _check(lib.mxr_proposal_apply(handle, w, c, alpha, ws, ws_bytes, _stream_handle(stream)))


def mxr_batch_means(sums_ptr, R, n_bins, rays_per_replica, mean_ptr, rel_ptr, stream=None) -> None:
    _check(lib.mxr_batch_means(sums_ptr, R, n_bins, rays_per_replica, mean_ptr, rel_ptr, _stream_handle(stream)))


def batch_means(sums, rays_per_replica: int, stream=None):
    """(mean, rel) per bin of an (R, n_bins) float64 device tensor of replica sums."""
    import torch
    R, nb = sums.shape
    mean = torch.empty(nb, dtype=torch.float64, device=sums.device)
    rel = torch.empty(nb, dtype=torch.float64, device=sums.device)
    mxr_batch_means(sums.contiguous().data_ptr(), R, nb, rays_per_replica, mean.data_ptr(), rel.data_ptr(), stream)
    return mean, rel


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


PEAK_KINDS = {"fp64_fma": 0, "u32_mulhi": 1, "fp64_exp": 2, "read": 3, "atomic_f64": 4}


def mxr_peak_launch(kind: str, buf_ptr: int, nbytes: int, spread: int, iters: int, groups: int, stream=None) -> float:
    """Launch one micro-benchmark kernel; returns the operations (bytes for
    the read) it performs."""
    work = ctypes.c_double(0.0)
    _check(lib.mxr_peak_launch(PEAK_KINDS[kind], ctypes.c_void_p(buf_ptr), nbytes, spread, iters, groups,
                               ctypes.byref(work), _stream_handle(stream)))
    return work.value


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
        # a scattering phantom's table has three channels: (3, n_mat, n_ebin)
        s.dims[0], s.dims[1], s.dims[2], s.dims[3] = nx, ny, nz, mu.shape[1] if mu.ndim == 3 else mu.shape[0]
        p[0], p[1], p[2] = c["voxel"], c["table_emin"], c["table_emax"]
        if c.get("step") is not None:
            s.flags |= 1
            p[3] = c["step"]
        if c.get("scatter_order") is not None:
            s.flags |= 2
            p[4] = c["scatter_order"]
            if c.get("scatter_target") is not None:
                s.flags |= 4
                for i, v in enumerate(np.asarray(c["scatter_target"], dtype=np.float64).reshape(9)):
                    p[5 + i] = v
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
    elif t == "lens_crl":
        vals = [c["R"], c["n_lenses"], c["web"], c["pitch"], c["aperture"], c["delta_ref"], c["e_ref"],
                c["mu_a"], c["mu_b"]]
        for i, v in enumerate(vals):
            p[i] = v
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

    def set_proposal(self, gmm=None, alpha: float = 0.1) -> None:
        """Draw the cone-beam source from the proposal mixture ``gmm`` (a
        device tensor of 56 float64: 8 x (pi, mu_u, mu_v, mu_E, sigma_u,
        sigma_v, sigma_E)), or switch it off with None."""
        if gmm is None:
            mxr_proposal_set(self.handle, None, alpha)
            return
        assert gmm.dtype.is_floating_point and gmm.numel() == 56 and gmm.is_cuda
        g = gmm.reshape(56).to(dtype=__import__("torch").float64).contiguous()
        mxr_proposal_set(self.handle, g.data_ptr(), alpha)

    @property
    def launch_shape(self):
        """(occupancy, compact, rounds, xcd_order) of plain runs."""
        s = mxr_get_launch_shape(self.handle)
        return (s.occupancy, s.compact, s.rounds, s.xcd_order)

    @launch_shape.setter
    def launch_shape(self, value) -> None:
        mxr_set_launch_shape(self.handle, mxr_launch_shape(*[int(v) for v in value]))

    def autotune(self, n_total: int, rays_fraction: float, tallies=None, cache_path: Optional[str] = None):
        """mxr_autotune_instrument; timing runs add into ``tallies`` (new ones
        if None).  Returns the chosen shape."""
        if tallies is None:
            tallies = self.new_tallies()
        s = mxr_autotune_instrument(self.handle, n_total, rays_fraction, self.tally_structs(tallies), cache_path)
        return (s.occupancy, s.compact, s.rounds, s.xcd_order)

    def proposal_box(self):
        """(lo, hi) of the cone-beam source's proposal coordinates (u, v, E)."""
        return mxr_proposal_box(self.handle)

    def apply_proposal(self, net, context, alpha: float = 0.1, stream=None) -> None:
        """Draw the cone-beam source from the network ``net``'s mixture at
        ``context`` (one forward, the library's own box)."""
        mxr_proposal_apply(self.handle, net.w.data_ptr(), context, alpha, net.ws.data_ptr(), net.ws_bytes, stream)

    def new_hits(self, capacity: int):
        """Device buffers for ``capacity`` collected rows and a zeroed counter."""
        import torch
        dev = self.device
        return {"ctx": torch.empty(capacity, 6, dtype=torch.float32, device=dev),
                "y": torch.empty(capacity, 3, dtype=torch.float64, device=dev),
                "w": torch.empty(capacity, dtype=torch.float64, device=dev),
                "bin": torch.empty(capacity, dtype=torch.int64, device=dev),
                "count": torch.zeros(1, dtype=torch.int64, device=dev),
                "capacity": capacity}

    def collect(self, n_rays: int, seed: int, context, hits, first_ray: int = 0, n_total: Optional[int] = None,
                purpose: int = 0, job: int = 0, tallies=None, stream=None):
        """mxr_run that appends every detected ray to ``hits`` (see new_hits)."""
        n_total = n_rays if n_total is None else n_total
        if tallies is None:
            tallies = self.new_tallies()
        h = mxr_hits(hits["ctx"].data_ptr(), hits["y"].data_ptr(), hits["w"].data_ptr(), hits["bin"].data_ptr(),
                     hits["capacity"], hits["count"].data_ptr())
        for i in range(6):
            h.context[i] = float(context[i])
        mxr_collect(self.handle, first_ray, n_rays, n_total, seed, purpose, job, self.tally_structs(tallies), h,
                    stream)
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
    instruments and tallies must stay alive as long as the batch.  A
    schedule is (form, groups_per_cu, tile_rays, branches)."""

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
        return (s.form, s.groups_per_cu, s.tile_rays, s.branches)

    @schedule.setter
    def schedule(self, value) -> None:
        mxr_batch_set_schedule(self.handle, mxr_batch_schedule(*value))

    def autotune(self, rays_fraction: float, cache_path: Optional[str] = None):
        """Pick the fastest launch shape (timing runs add into the tallies)."""
        s = mxr_batch_autotune(self.handle, rays_fraction, cache_path)
        return (s.form, s.groups_per_cu, s.tile_rays, s.branches)

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


class ProposalNet:
    """The proposal network's device state: float32 master parameters, their
    bfloat16 working copy, Adam moments, a gradient buffer and a workspace
    for batches of up to ``batch`` rows (torch tensors own the memory; every
    computation is a library call)."""

    def __init__(self, params, batch: int, device=None):
        import torch
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        p = torch.as_tensor(np.asarray(params, dtype=np.float32)).to(self.device)
        assert p.numel() == MLP_PARAMS
        self.master = p.contiguous()
        self.w = torch.empty(MLP_PARAMS, dtype=torch.bfloat16, device=self.device)
        self.m = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=self.device)
        self.grad = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=self.device)
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.batch = batch
        # the network's workspace, with room for mxr_proposal_apply's tail
        self.ws_bytes = max(mxr_mlp_workspace_bytes(batch), mxr_mlp_workspace_bytes(1) + 1024)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.step = 0
        mxr_mlp_to_bf16(self.master.data_ptr(), MLP_PARAMS, self.w.data_ptr())

    def region(self, name: str, n: int, dtype, width: int):
        """View of workspace region ``name`` as an (n, width) tensor, laid out
        for a batch of n rows."""
        import torch
        off = mxr_mlp_workspace_layout(n)[WS_REGIONS.index(name)]
        item = torch.empty(0, dtype=dtype).element_size()
        return self.ws[off:off + n * width * item].view(dtype).view(n, width)

    def forward(self, ctx, stream=None):
        import torch
        n = ctx.shape[0]
        assert n <= self.batch
        out = torch.empty(n, MLP_OUT, dtype=torch.float32, device=self.device)
        mxr_mlp_forward(self.w.data_ptr(), ctx.contiguous().data_ptr(), n, out.data_ptr(), self.ws.data_ptr(),
                        self.ws_bytes, stream)
        return out

    def mixture(self, out, lo, hi, stream=None):
        import torch
        g = torch.empty(out.shape[0], MLP_OUT, dtype=torch.float64, device=self.device)
        mxr_mlp_mixture(out.contiguous().data_ptr(), out.shape[0], lo, hi, g.data_ptr(), stream)
        return g

    def loss_grad(self, ctx, y, omega, lo, hi, stream=None):
        n = ctx.shape[0]
        assert n <= self.batch
        mxr_mlp_loss_grad(self.w.data_ptr(), ctx.contiguous().data_ptr(), y.contiguous().data_ptr(),
                          omega.contiguous().data_ptr(), n, lo, hi, self.grad.data_ptr(), self.loss.data_ptr(),
                          self.ws.data_ptr(), self.ws_bytes, stream)
        return self.loss, self.grad

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step += 1
        mxr_adam_step(self.master.data_ptr(), self.w.data_ptr(), self.grad.data_ptr(), self.m.data_ptr(),
                      self.v.data_ptr(), MLP_PARAMS, self.step, lr, beta1, beta2, eps, stream)

    def train(self, ctx, y, omega, lo, hi, epochs: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed: int = 1,
              loss_log=None, stream=None):
        n = ctx.shape[0]
        cfg = mxr_train_cfg(lr, beta1, beta2, eps, self.batch, epochs, seed, self.step)
        mxr_mlp_train(ctx.contiguous().data_ptr(), y.contiguous().data_ptr(), omega.contiguous().data_ptr(), n, cfg,
                      lo, hi, self.master.data_ptr(), self.w.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                      self.grad.data_ptr(), self.ws.data_ptr(), self.ws_bytes,
                      loss_log.data_ptr() if loss_log is not None else None, stream)
        self.step += epochs * ((n + min(self.batch, n) - 1) // min(self.batch, n))


    def train_from_runs(self, ins, hits, run_first, run_images, epochs: int, lr=1e-3, beta1=0.9, beta2=0.999,
                        eps=1e-8, seed: int = 1, floor_frac: float = 1e-3, loss_log=None, stream=None):
        """mxr_proposal_train: the training weights of the collected rows
        ``hits`` (rows [run_first[r], run_first[r + 1]) from the run whose
        monitor image is run_images[r]) and Adam training in the box of the
        instrument ``ins``'s source.  Returns the weights (device tensor)."""
        import torch
        n = int(run_first[-1])
        omega = torch.empty(n, dtype=torch.float64, device=self.device)
        first = (ctypes.c_uint64 * len(run_first))(*[int(x) for x in run_first])
        images = (ctypes.c_void_p * len(run_images))(*[t.data_ptr() for t in run_images])
        rows = mxr_train_rows(hits["ctx"].data_ptr(), hits["y"].data_ptr(), hits["w"].data_ptr(),
                              hits["bin"].data_ptr(), n, len(run_images), first, images, run_images[0].numel(),
                              floor_frac)
        cfg = mxr_train_cfg(lr, beta1, beta2, eps, self.batch, epochs, seed, self.step)
        mxr_proposal_train(ins.handle, rows, cfg, self.master.data_ptr(), self.w.data_ptr(), self.m.data_ptr(),
                           self.v.data_ptr(), self.grad.data_ptr(), omega.data_ptr(), self.ws.data_ptr(),
                           self.ws_bytes, loss_log.data_ptr() if loss_log is not None else None, stream)
        self.step += epochs * ((n + min(self.batch, n) - 1) // min(self.batch, n))
        return omega


def train_weights(hits, count: int, sum_w, floor_frac: float = 1e-3, stream=None):
    """omega of the first ``count`` collected rows (see mxr_train_weights)."""
    import torch
    dev = sum_w.device
    omega = torch.empty(count, dtype=torch.float64, device=dev)
    scratch = torch.empty(2 * 256 + 1, dtype=torch.float64, device=dev)
    mxr_train_weights(hits["w"].data_ptr(), hits["bin"].data_ptr(), count, sum_w.data_ptr(), sum_w.numel(),
                      floor_frac, omega.data_ptr(), scratch.data_ptr(), stream)
    return omega
