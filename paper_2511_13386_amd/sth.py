"""Thin ctypes binding of libsth.so (C-ABI in include/sth.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  Names follow the C entry points.  The binding raises if the library
is missing; there is no CPU fallback.

Device memory can come from PyTorch: pass ``arena`` as a CUDA/HIP tensor (its
data pointer and byte size are handed to ``sth_create``) and ``stream`` as a
``torch.cuda.Stream`` (its ``cuda_stream`` handle is the hipStream_t).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsth.so")

STH_OK, STH_EINVAL, STH_ENOMEM, STH_EHIP, STH_ENONFINITE, STH_ESTATE = 0, -1, -2, -3, -4, -5
HYBRID, FIELD, LITERAL_R, LITERAL_FLUX, COARSE_EXPLICIT = 1, 2, 4, 8, 16
FP64, FP32_BULK = 0, 1
START_LIFT, START_CARRY = 0, 1

EXPORTS = (
    "sth_footprint_bytes", "sth_create", "sth_coarse_sweep", "sth_fine_sweep_batched",
    "sth_parareal_correct", "sth_moments_criteria", "sth_get_rho", "sth_get_g", "sth_get_info",
    "sth_fine_run", "sth_destroy", "sth_last_error", "sth_parareal_correct_batched", "sth_get_errors",
    "sth_graph_create", "sth_graph_launch", "sth_graph_wait", "sth_graph_destroy",
    "sth_fine_config_candidates", "sth_set_fine_config", "sth_get_fine_config",
    "sth_coarse_sweep_batched", "sth_fine_sweep_chunk", "sth_fine_run_masks", "sth_fine_run_noalloc",
)


class StHError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sth error {code}: {msg}")
        self.code = code


class ProblemDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("nv", ctypes.c_int),
        ("Lx", ctypes.c_double), ("vstar", ctypes.c_double),
        ("eps_iface", ctypes.POINTER(ctypes.c_double)),
        ("eps_cell", ctypes.POINTER(ctypes.c_double)),
        ("rho0", ctypes.POINTER(ctypes.c_double)),
        ("g0", ctypes.POINTER(ctypes.c_double)),
        ("T", ctypes.c_double), ("n_slices", ctypes.c_int), ("k_max", ctypes.c_int),
        ("tol", ctypes.c_double), ("eta0", ctypes.c_double), ("delta0", ctypes.c_double),
        ("lift_order", ctypes.c_int), ("start_mode", ctypes.c_int),
        ("cfl_theta", ctypes.c_double), ("flags", ctypes.c_int), ("precision", ctypes.c_int),
        ("steps_override", ctypes.c_longlong),
        ("nv_y", ctypes.c_int), ("nv_z", ctypes.c_int),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("dx", ctypes.c_double), ("dv", ctypes.c_double), ("dt", ctypes.c_double),
        ("dtG", ctypes.c_double), ("m2", ctypes.c_double), ("rhobar", ctypes.c_double),
        ("steps_per_slice", ctypes.c_longlong), ("k_done", ctypes.c_int),
        ("n_slices", ctypes.c_int), ("kinetic_iface_steps", ctypes.c_double),
        ("last_err", ctypes.c_double), ("footprint_bytes", ctypes.c_size_t),
        ("fine_resident", ctypes.c_int), ("fine_block", ctypes.c_int),
        ("coarse_steps", ctypes.c_longlong),
        ("norm_scale", ctypes.c_double),
    ]


class FineConfig(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("resident", ctypes.c_int)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_VP = ctypes.c_void_p


def lib() -> ctypes.CDLL:
    """Load libsth.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime under the same soname as the
        # system one; loading it first makes libsth.so bind to it, so device
        # pointers and streams from torch are valid in the library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              f"`python -m paper_2511_13386_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.sth_footprint_bytes.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.POINTER(ctypes.c_size_t)]
        L.sth_create.argtypes = [ctypes.POINTER(ProblemDesc), _VP, ctypes.c_size_t, ctypes.POINTER(_VP)]
        L.sth_coarse_sweep.argtypes = [_VP, _VP]
        L.sth_fine_sweep_batched.argtypes = [ctypes.POINTER(_VP), ctypes.c_int, _VP]
        L.sth_coarse_sweep_batched.argtypes = [ctypes.POINTER(_VP), ctypes.c_int, _VP]
        L.sth_fine_sweep_chunk.argtypes = [ctypes.POINTER(_VP), ctypes.c_int, ctypes.c_longlong,
                                           ctypes.POINTER(ctypes.c_int), _VP]
        L.sth_parareal_correct.argtypes = [_VP, _D, ctypes.POINTER(ctypes.c_int), _VP]
        L.sth_moments_criteria.argtypes = [_VP, ctypes.c_int, _D, _D, _D, _D, _D,
                                           ctypes.POINTER(ctypes.c_int), _VP]
        L.sth_get_rho.argtypes = [_VP, _D]
        L.sth_get_g.argtypes = [_VP, ctypes.c_int, _D]
        L.sth_get_info.argtypes = [_VP, ctypes.POINTER(Info)]
        L.sth_fine_run.argtypes = [_VP, _D, _D, ctypes.c_longlong, _D, _D,
                                   ctypes.POINTER(ctypes.c_int), _D, _VP]
        L.sth_fine_run_masks.argtypes = [_VP, _D, _D, ctypes.c_longlong, _VP, _VP, ctypes.c_longlong, _D, _D,
                                         ctypes.POINTER(ctypes.c_int), _D, _VP]
        L.sth_fine_run_noalloc.argtypes = [_VP, _D, _D, ctypes.c_longlong, _D, _D,
                                           ctypes.POINTER(ctypes.c_int), _D, _VP]
        L.sth_parareal_correct_batched.argtypes = [ctypes.POINTER(_VP), ctypes.c_int, _D, _VP]
        L.sth_get_errors.argtypes = [_VP, _D]
        L.sth_graph_create.argtypes = [ctypes.POINTER(_VP), ctypes.c_int, ctypes.POINTER(_VP)]
        L.sth_graph_launch.argtypes = [_VP, _VP]
        L.sth_graph_wait.argtypes = [_VP, _VP, ctypes.POINTER(ctypes.c_int), _D]
        L.sth_graph_destroy.argtypes = [_VP]
        L.sth_graph_destroy.restype = None
        L.sth_fine_config_candidates.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                 ctypes.POINTER(FineConfig), ctypes.c_int,
                                                 ctypes.POINTER(ctypes.c_int)]
        L.sth_set_fine_config.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(FineConfig)]
        L.sth_get_fine_config.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(FineConfig)]
        L.sth_destroy.argtypes = [_VP]
        L.sth_destroy.restype = None
        L.sth_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != STH_OK:
        raise StHError(rc, lib().sth_last_error().decode())


def _d(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_D)


def _stream(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(getattr(stream, "cuda_stream"))


@dataclass
class Desc:
    """Problem description mirroring sth_problem_desc."""
    nx: int
    nv: int
    eps_iface: np.ndarray
    eps_cell: np.ndarray
    rho0: np.ndarray
    T: float
    n_slices: int
    k_max: int = 8
    tol: float = 0.0
    eta0: float = 1e-3
    delta0: float = 1e-3
    lift_order: int = 3
    start_mode: int = START_LIFT
    cfl_theta: float = 1.0
    flags: int = FIELD
    precision: int = FP64
    g0: Optional[np.ndarray] = None
    Lx: float = 1.0
    vstar: float = 8.0
    steps_override: int = 0
    nv_y: int = 0                    # 1D3V (separable form) when nv_y, nv_z > 0
    nv_z: int = 0

    def to_c(self):
        keep = [np.ascontiguousarray(self.eps_iface, dtype=np.float64),
                np.ascontiguousarray(self.eps_cell, dtype=np.float64),
                np.ascontiguousarray(self.rho0, dtype=np.float64)]
        g0 = None if self.g0 is None else np.ascontiguousarray(self.g0, dtype=np.float64)
        keep.append(g0)
        c = ProblemDesc(int(self.nx), int(self.nv), float(self.Lx), float(self.vstar),
                        _d(keep[0]), _d(keep[1]), _d(keep[2]), _d(g0), float(self.T),
                        int(self.n_slices), int(self.k_max), float(self.tol), float(self.eta0),
                        float(self.delta0), int(self.lift_order), int(self.start_mode),
                        float(self.cfl_theta), int(self.flags), int(self.precision),
                        int(self.steps_override), int(self.nv_y), int(self.nv_z))
        return c, keep


def sth_footprint_bytes(desc: Desc) -> int:
    c, keep = desc.to_c()
    out = ctypes.c_size_t()
    _check(lib().sth_footprint_bytes(ctypes.byref(c), ctypes.byref(out)))
    return int(out.value)


class Problem:
    """Owning handle of an sth_problem."""

    def __init__(self, desc: Desc, arena=None):
        self.desc = desc
        c, keep = desc.to_c()
        h = _VP()
        ptr, nbytes = None, 0
        self._arena = arena
        if arena is not None:
            ptr = int(arena.data_ptr())
            nbytes = int(arena.numel() * arena.element_size())
        _check(lib().sth_create(ctypes.byref(c), ptr, nbytes, ctypes.byref(h)))
        self.h = h
        self.nx, self.nv, self.N = desc.nx, desc.nv, desc.n_slices

    def close(self):
        if getattr(self, "h", None):
            lib().sth_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> Info:
        out = Info()
        _check(lib().sth_get_info(self.h, ctypes.byref(out)))
        return out


def sth_create(desc: Desc, arena=None) -> Problem:
    return Problem(desc, arena)


def sth_coarse_sweep(p: Problem, stream=None) -> None:
    _check(lib().sth_coarse_sweep(p.h, _stream(stream)))


def sth_coarse_sweep_batched(problems: Sequence[Problem], stream=None) -> None:
    arr = (_VP * len(problems))(*[q.h for q in problems])
    _check(lib().sth_coarse_sweep_batched(arr, len(problems), _stream(stream)))


def sth_fine_sweep_batched(problems: Sequence[Problem], stream=None) -> None:
    arr = (_VP * len(problems))(*[q.h for q in problems])
    _check(lib().sth_fine_sweep_batched(arr, len(problems), _stream(stream)))


def sth_fine_sweep_chunk(problems: Sequence[Problem], max_steps: int, stream=None) -> list:
    """Advance the fine sweeps by at most max_steps steps per slice; returns,
    per problem, whether its sweep has ended (and awaits its correction)."""
    n = len(problems)
    arr = (_VP * n)(*[q.h for q in problems])
    done = (ctypes.c_int * max(n, 1))()
    _check(lib().sth_fine_sweep_chunk(arr, n, int(max_steps), done, _stream(stream)))
    return [bool(done[i]) for i in range(n)]


def sth_parareal_correct(p: Problem, want_err: bool = True, stream=None):
    err = ctypes.c_double(-1.0)
    k = ctypes.c_int(0)
    _check(lib().sth_parareal_correct(p.h, ctypes.byref(err) if want_err else None,
                                      ctypes.byref(k), _stream(stream)))
    return (err.value if want_err else None), k.value


def sth_parareal_correct_batched(problems: Sequence[Problem], want_err: bool = True, stream=None,
                                 nonfinite_ok: bool = False):
    """Corrections of several problems in one launch; returns their errors
    (None when want_err is False).  A non-finite error raises StHError
    (STH_ENONFINITE) unless nonfinite_ok, which returns it in the list."""
    arr = (_VP * len(problems))(*[q.h for q in problems])
    errs = np.zeros(len(problems)) if want_err else None
    rc = lib().sth_parareal_correct_batched(arr, len(problems), _d(errs), _stream(stream))
    if not (nonfinite_ok and rc == STH_ENONFINITE):
        _check(rc)
    return None if errs is None else errs.tolist()


def sth_get_errors(p: Problem) -> list:
    """Successive errors of the iterations done so far."""
    k = p.info().k_done
    out = np.zeros(max(k, 1))
    _check(lib().sth_get_errors(p.h, _d(out)))
    return out[:k].tolist()


class Graph:
    """Owning handle of an sth_graph: a whole parareal solve of the given
    problems recorded once and replayed by one launch."""

    def __init__(self, problems: Sequence[Problem]):
        self.problems = list(problems)
        arr = (_VP * len(self.problems))(*[q.h for q in self.problems])
        h = _VP()
        _check(lib().sth_graph_create(arr, len(self.problems), ctypes.byref(h)))
        self.h = h

    def launch(self, stream=None) -> None:
        _check(lib().sth_graph_launch(self.h, _stream(stream)))

    def wait(self, stream=None):
        """Returns (iterations done, last error) per problem."""
        n = len(self.problems)
        iters = (ctypes.c_int * n)()
        errs = np.zeros(n)
        _check(lib().sth_graph_wait(self.h, _stream(stream), iters, _d(errs)))
        return list(iters), errs.tolist()

    def close(self):
        if getattr(self, "h", None):
            lib().sth_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sth_fine_config_candidates(precision: int, nx: int, nv: int) -> list:
    """[(block, resident)] supported for the class of (precision, nx, nv)."""
    n = ctypes.c_int()
    buf = (FineConfig * 16)()
    _check(lib().sth_fine_config_candidates(int(precision), int(nx), int(nv), buf, 16, ctypes.byref(n)))
    return [(buf[i].block, buf[i].resident) for i in range(min(n.value, 16))]


def sth_set_fine_config(precision: int, nx: int, nv: int, config=None) -> None:
    """Set (block, resident) for the class, or None for the default rule."""
    if config is None:
        _check(lib().sth_set_fine_config(int(precision), int(nx), int(nv), None))
    else:
        c = FineConfig(int(config[0]), int(config[1]))
        _check(lib().sth_set_fine_config(int(precision), int(nx), int(nv), ctypes.byref(c)))


def sth_get_fine_config(precision: int, nx: int, nv: int) -> tuple:
    c = FineConfig()
    _check(lib().sth_get_fine_config(int(precision), int(nx), int(nv), ctypes.byref(c)))
    return (c.block, c.resident)


def sth_moments_criteria(p: Problem, slice_: int, stream=None) -> dict:
    out = {k: np.zeros(p.nx) for k in ("E", "J", "Phi", "N", "R")}
    mask = np.zeros(p.nx, dtype=np.int32)
    _check(lib().sth_moments_criteria(p.h, int(slice_), _d(out["E"]), _d(out["J"]), _d(out["Phi"]),
                                      _d(out["N"]), _d(out["R"]),
                                      mask.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                      _stream(stream)))
    out["mask"] = mask
    return out


def sth_get_rho(p: Problem) -> np.ndarray:
    out = np.zeros((p.N + 1, p.nx))
    _check(lib().sth_get_rho(p.h, _d(out)))
    return out


def sth_get_g(p: Problem, slice_: int) -> np.ndarray:
    out = np.zeros((p.nx, p.nv))
    _check(lib().sth_get_g(p.h, int(slice_), _d(out)))
    return out


def sth_get_info(p: Problem) -> Info:
    return p.info()


def sth_fine_run(p: Problem, rho_in, g_in, nsteps: int, stream=None):
    rho_in = np.ascontiguousarray(rho_in, dtype=np.float64)
    g_arr = None if g_in is None else np.ascontiguousarray(g_in, dtype=np.float64)
    rho = np.zeros(p.nx)
    g = np.zeros((p.nx, p.nv))
    mask = np.zeros(p.nx, dtype=np.int32)
    kin = ctypes.c_double()
    _check(lib().sth_fine_run(p.h, _d(rho_in), _d(g_arr), int(nsteps), _d(rho), _d(g),
                              mask.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ctypes.byref(kin),
                              _stream(stream)))
    return rho, g, mask, kin.value


def sth_fine_run_noalloc(p: Problem, rho_in, g_in, nsteps: int, stream=None, want_g=True):
    """sth_fine_run through the allocation-free entry point (static device
    workspace); want_g=False passes no g_out."""
    rho_in = np.ascontiguousarray(rho_in, dtype=np.float64)
    g_arr = None if g_in is None else np.ascontiguousarray(g_in, dtype=np.float64)
    rho = np.zeros(p.nx)
    g = np.zeros((p.nx, p.nv)) if want_g else None
    mask = np.zeros(p.nx, dtype=np.int32)
    kin = ctypes.c_double()
    _check(lib().sth_fine_run_noalloc(p.h, _d(rho_in), _d(g_arr), int(nsteps), _d(rho), _d(g),
                                      mask.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ctypes.byref(kin),
                                      _stream(stream)))
    return rho, g, mask, kin.value


def sth_fine_run_masks(p: Problem, rho_in, g_in, nsteps: int, replay=None, stream=None):
    """sth_fine_run with the cell status of every step: returns (rho, g,
    cell_mask, kin, hist), hist[n, i] = 1 if cell i is kinetic at step n
    (n = 0..nsteps).  replay ([nsteps + 1, nx], nonzero = kinetic) imposes
    those statuses instead of the rule.  The bit rows live in torch device
    tensors for the call."""
    import torch
    nsteps = int(nsteps)
    rho_in = np.ascontiguousarray(rho_in, dtype=np.float64)
    g_arr = None if g_in is None else np.ascontiguousarray(g_in, dtype=np.float64)
    mw = (p.nx + 63) // 64
    rows = nsteps + 1

    def pack(m):
        m = np.asarray(m) != 0
        if m.shape != (rows, p.nx):
            raise ValueError("replay must have shape (nsteps + 1, nx)")
        bits = np.zeros((rows, mw * 64), dtype=np.uint8)
        bits[:, :p.nx] = m
        # little-endian words: bit i of a row is bit (i mod 64) of word i / 64
        return np.packbits(bits, axis=-1, bitorder="little").view("<u8")

    dev = torch.device("cuda", torch.cuda.current_device())
    d_rep = None
    if replay is not None:
        d_rep = torch.from_numpy(pack(replay).view(np.int64)).to(dev)
    d_hist = torch.zeros((rows, mw), dtype=torch.int64, device=dev)
    rho = np.zeros(p.nx)
    g = np.zeros((p.nx, p.nv))
    mask = np.zeros(p.nx, dtype=np.int32)
    kin = ctypes.c_double()
    torch.cuda.synchronize(dev)
    _check(lib().sth_fine_run_masks(p.h, _d(rho_in), _d(g_arr), nsteps,
                                    None if d_rep is None else d_rep.data_ptr(), d_hist.data_ptr(),
                                    rows * mw,
                                    _d(rho), _d(g), mask.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                    ctypes.byref(kin), _stream(stream)))
    words = np.ascontiguousarray(d_hist.cpu().numpy()).view("<u8")
    bits = np.unpackbits(words.view(np.uint8), axis=-1, bitorder="little")
    hist = bits[:, :p.nx].astype(np.uint8)
    return rho, g, mask, kin.value, hist


def sth_destroy(p: Problem) -> None:
    p.close()


def sth_last_error() -> str:
    return lib().sth_last_error().decode()


def parareal_solve(p: Problem, K: Optional[int] = None, tol: float = 0.0, stream=None,
                   fixed_iterations: bool = False):
    """Coarse guess, then fine sweep + correction until err < tol or K
    iterations.  Returns the list of successive errors."""
    K = p.desc.k_max if K is None else K
    sth_coarse_sweep(p, stream)
    errs = []
    for _ in range(min(K, p.N)):
        sth_fine_sweep_batched([p], stream)
        e, k = sth_parareal_correct(p, want_err=True, stream=stream)
        errs.append(e)
        if not fixed_iterations and e < tol:
            break
    return errs
