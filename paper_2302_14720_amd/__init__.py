"""Python binding of libswmi.so -- Swendsen-Wang dynamics on one MI355X
(Protzman & Giedt, Sec. 2): the 2D Ising model, the q-state Potts model
(``q=2..8``) and the simple cubic lattice (``dims=3``); batched replicas
(``Batch``) and a job server (``Server``).

The binding only marshals arguments: every step of a sweep runs in the HIP
kernels of ``csrc/``.  Function names match the C ABI in ``include/swmi.h``;
``Sim`` is a thin object wrapper whose device workspace is a torch uint8
tensor and whose stream is a torch stream (torch provides memory and
streams, nothing else).  If the library has not been built the first call
raises -- there is no fallback implementation.

    sim = Sim(1024, 0.4406868, seed=1)           # 2D Ising, hot start
    sim.sweep(100); rec = sim.observables()      # energy, magnetisation, clusters
    potts = Sim(1024, 1.0050525, q=3)            # 2D q = 3 Potts at ln(1 + sqrt 3)
    cube = Sim(128, 0.2216544, dims=3)           # 3D Ising on 128^3 sites
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswmi.so")

SW_OK, SW_EINVAL, SW_ERANGE, SW_ENOMEM, SW_EHIP, SW_ESTATE = 0, -1, -2, -3, -4, -5
SW_INIT_HOT, SW_INIT_COLD = 0, 1
SW_FLAG_LABELS, SW_FLAG_DENSE_HIST, SW_FLAG_LABEL_EQUIV = 1, 2, 4

# Layout of ``sw_obs`` (swmi.h).
OBS_DTYPE = np.dtype(
    [
        ("sweep", "<u8"),
        ("e_sum", "<i8"),
        ("energy", "<f8"),
        ("m_sum", "<i8"),
        ("n_clusters", "<u8"),
        ("max_cluster", "<u8"),
        ("sum_sq_sizes", "<u8"),
        ("hist_log2", "<u8", (33,)),
    ]
)
assert OBS_DTYPE.itemsize == 320


class sw_config(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("init", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("beta", ctypes.c_double),
        ("J", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("ring", ctypes.c_int64),
        ("q", ctypes.c_int32),
        ("dims", ctypes.c_int32),
    ]


SW_JOB_QUEUED, SW_JOB_ACTIVE, SW_JOB_DONE = 0, 1, 2


class sw_job_info(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int64),
        ("state", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("sweeps_done", ctypes.c_int64),
        ("sweeps_total", ctypes.c_int64),
        ("bytes", ctypes.c_uint64),
    ]


class SwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"swmi error {code}: {msg}")
        self.code = code


# Every symbol swmi.h declares, with (restype, argtypes).
_P = ctypes.c_void_p
_SIGNATURES = {
    "sw_config_init": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64]),
    "sw_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "sw_workspace_bytes_ex": (ctypes.c_size_t, [_P]),
    "sw_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, _P]),
    "sw_create_in": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                    _P, ctypes.c_size_t, _P, _P]),
    "sw_create_ex": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P, _P]),
    "sw_reset": (ctypes.c_int, [_P, ctypes.c_int]),
    "sw_sweep": (ctypes.c_int, [_P, ctypes.c_int64]),
    "sw_sync": (ctypes.c_int, [_P]),
    "sw_profile": (ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.c_int32]),
    "sw_observables": (ctypes.c_int, [_P, _P]),
    "sw_series": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _P]),
    "sw_cluster_hist": (ctypes.c_int, [_P, _P, ctypes.c_int64]),
    "sw_get_spins": (ctypes.c_int, [_P, _P, ctypes.c_int64]),
    "sw_set_spins": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_uint64]),
    "sw_get_labels": (ctypes.c_int, [_P, _P, ctypes.c_int64]),
    "sw_threshold": (ctypes.c_uint32, [_P]),
    "sw_label_passes": (ctypes.c_int32, [_P]),
    "sw_next_sweep": (ctypes.c_int64, [_P]),
    "sw_lattice": (ctypes.c_int32, [_P]),
    "sw_tile": (ctypes.c_int32, [_P]),
    "sw_sites": (ctypes.c_int64, [_P]),
    "sw_destroy": (None, [_P]),
    "sw_last_error": (ctypes.c_char_p, []),
    "sw_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, _P, ctypes.c_int64, ctypes.c_int32]),
    "sw_batch_create": (ctypes.c_int, [ctypes.c_int32, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_int32, _P, ctypes.c_size_t, _P, _P]),
    "sw_batch_workspace_bytes_potts": (ctypes.c_size_t, [ctypes.c_int32, _P, _P, ctypes.c_int64, ctypes.c_int32]),
    "sw_batch_create_potts": (ctypes.c_int, [ctypes.c_int32, _P, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_int64,
                                             ctypes.c_int32, _P, ctypes.c_size_t, _P, _P]),
    "sw_batch_reset": (ctypes.c_int, [_P, ctypes.c_int32]),
    "sw_batch_sweep": (ctypes.c_int, [_P, ctypes.c_int64]),
    "sw_batch_sync": (ctypes.c_int, [_P]),
    "sw_batch_observables": (ctypes.c_int, [_P, _P]),
    "sw_batch_series": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _P]),
    "sw_batch_get_spins": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int64]),
    "sw_batch_size": (ctypes.c_int32, [_P]),
    "sw_batch_next_sweep": (ctypes.c_int64, [_P]),
    "sw_batch_lattice": (ctypes.c_int32, [_P, ctypes.c_int32]),
    "sw_batch_threshold": (ctypes.c_uint32, [_P, ctypes.c_int32]),
    "sw_batch_tile": (ctypes.c_int32, [_P]),
    "sw_batch_replica_tile": (ctypes.c_int32, [_P, ctypes.c_int32]),
    "sw_batch_replica_merge": (ctypes.c_int32, [_P, ctypes.c_int32]),
    "sw_batch_workspace_bytes_ex": (ctypes.c_size_t, [ctypes.c_int32, _P, _P, _P, _P, ctypes.c_int64]),
    "sw_batch_create_ex": (ctypes.c_int, [ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, ctypes.c_int32,
                                          ctypes.c_int64, _P, ctypes.c_size_t, _P, _P]),
    "sw_batch_destroy": (None, [_P]),
    "sw_server_job_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int64]),
    "sw_server_job_bytes_potts": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64]),
    "sw_server_create": (ctypes.c_int, [_P, ctypes.c_size_t, ctypes.c_int32, _P, _P]),
    "sw_server_submit": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                        ctypes.c_int32, ctypes.c_int64, _P]),
    "sw_server_submit_potts": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _P]),
    "sw_server_step": (ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.c_int32, _P]),
    "sw_server_job_info": (ctypes.c_int, [_P, ctypes.c_int64, _P]),
    "sw_server_job_series": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _P]),
    "sw_server_job_spins": (ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.c_int64]),
    "sw_server_release": (ctypes.c_int, [_P, ctypes.c_int64]),
    "sw_server_status": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "sw_server_destroy": (None, [_P]),
    "sw_phi4_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int64]),
    "sw_phi4_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, ctypes.c_int32,
                                      ctypes.c_int64, _P, ctypes.c_size_t, _P, _P]),
    "sw_phi4_reset": (ctypes.c_int, [_P, ctypes.c_int32]),
    "sw_phi4_sweep": (ctypes.c_int, [_P, ctypes.c_int64]),
    "sw_phi4_sync": (ctypes.c_int, [_P]),
    "sw_phi4_profile": (ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.c_int32]),
    "sw_phi4_series": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _P]),
    "sw_phi4_get_field": (ctypes.c_int, [_P, _P, ctypes.c_int64]),
    "sw_phi4_set_field": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_uint64]),
    "sw_phi4_get_labels": (ctypes.c_int, [_P, _P, ctypes.c_int64]),
    "sw_phi4_sites": (ctypes.c_int64, [_P]),
    "sw_phi4_next_sweep": (ctypes.c_int64, [_P]),
    "sw_phi4_destroy": (None, [_P]),
    "sw_sweep_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                        ctypes.c_uint64, _P, _P, _P]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libswmi.so; raises if it has not been built.

    torch is imported first: its HIP and HSA runtime libraries carry the
    sonames libswmi.so links against, so the library binds to the runtime
    that owns torch's pointers and streams.  Loaded before torch it would
    bring in a second HIP/HSA runtime, which finds no device once the first
    has opened it, and to which torch's streams mean nothing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        import torch  # noqa: F401  (one HIP runtime per process, torch's)

        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


def _check(rc: int) -> None:
    if rc != SW_OK:
        raise SwError(rc, lib().sw_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ------------------------------------------------------------- C-named calls
def sw_config_init(L: int, beta: float, J: float = 1.0, seed: int = 0, *, init: int = SW_INIT_HOT,
                   tile: int = 0, flags: int = 0, ring: int = 0, q: int = 0, dims: int = 0) -> sw_config:
    cfg = sw_config()
    _check(lib().sw_config_init(ctypes.byref(cfg), L, beta, J, seed))
    cfg.init, cfg.tile, cfg.flags, cfg.ring, cfg.q, cfg.dims = init, tile, flags, ring, q, dims
    return cfg


def sw_workspace_bytes(L: int) -> int:
    return int(lib().sw_workspace_bytes(L))


def sw_workspace_bytes_ex(cfg: sw_config) -> int:
    return int(lib().sw_workspace_bytes_ex(ctypes.byref(cfg)))


def sw_create_ex(cfg: sw_config, ws_ptr: int = 0, ws_bytes: int = 0, stream_ptr: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(lib().sw_create_ex(ctypes.byref(cfg), ws_ptr or None, ws_bytes, stream_ptr or None,
                              ctypes.byref(h)))
    return h.value


def sw_create(L: int, beta: float, J: float, seed: int) -> int:
    h = ctypes.c_void_p()
    _check(lib().sw_create(L, beta, J, seed, ctypes.byref(h)))
    return h.value


def sw_create_in(L: int, beta: float, J: float, seed: int, ws_ptr: int, ws_bytes: int,
                 stream_ptr: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(lib().sw_create_in(L, beta, J, seed, ws_ptr, ws_bytes, stream_ptr or None, ctypes.byref(h)))
    return h.value


def sw_reset(h: int, init_mode: int = SW_INIT_HOT) -> None:
    _check(lib().sw_reset(h, init_mode))


def sw_sweep(h: int, n: int) -> None:
    _check(lib().sw_sweep(h, n))


def sw_sync(h: int) -> None:
    _check(lib().sw_sync(h))


PROFILE_STAGES = ("tile", "union", "flatten", "roots", "record", "resolve")


def sw_profile(h: int, n: int) -> dict:
    ms = np.zeros(len(PROFILE_STAGES), dtype=np.float64)
    _check(lib().sw_profile(h, n, _ptr(ms), ms.size))
    return dict(zip(PROFILE_STAGES, ms.tolist()))


def sw_observables(h: int) -> np.void:
    out = np.zeros(1, dtype=OBS_DTYPE)
    _check(lib().sw_observables(h, _ptr(out)))
    return out[0]


def sw_series(h: int, first: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=OBS_DTYPE)
    _check(lib().sw_series(h, first, count, _ptr(out)))
    return out


def sw_cluster_hist(h: int, n_sites: int) -> np.ndarray:
    out = np.zeros(n_sites + 1, dtype=np.uint64)
    _check(lib().sw_cluster_hist(h, _ptr(out), out.size))
    return out


def sw_get_spins(h: int, n_sites: int) -> np.ndarray:
    out = np.empty(n_sites, dtype=np.int8)
    _check(lib().sw_get_spins(h, _ptr(out), n_sites))
    return out


def sw_set_spins(h: int, spins: np.ndarray, next_sweep: int) -> None:
    s = np.ascontiguousarray(spins, dtype=np.int8)
    _check(lib().sw_set_spins(h, _ptr(s), s.size, next_sweep))


def sw_get_labels(h: int, n_sites: int) -> np.ndarray:
    out = np.empty(n_sites, dtype=np.uint32)
    _check(lib().sw_get_labels(h, _ptr(out), n_sites))
    return out


def sw_threshold(h: int) -> int:
    return int(lib().sw_threshold(h))


def sw_next_sweep(h: int) -> int:
    return int(lib().sw_next_sweep(h))


def sw_destroy(h: int) -> None:
    if h:
        lib().sw_destroy(h)


def sw_last_error() -> str:
    return lib().sw_last_error().decode()


def sw_sweep_noalloc(L: int, beta: float, J: float, seed: int, t: int, spins_ptr: int, rec_ptr: int,
                     stream_ptr: int = 0) -> None:
    """Sweep t of the lattice whose int8 spins sit at device address
    spins_ptr (overwritten in place); record t to the sw_obs at rec_ptr.
    Allocates nothing (the library's static scratch holds every other
    buffer); returns without waiting for the stream."""
    _check(lib().sw_sweep_noalloc(L, beta, J, seed, t, spins_ptr or None, rec_ptr or None, stream_ptr or None))


# ------------------------------------------------------------- batch calls
def _replica_arrays(L, beta, J, seed):
    n = len(L)
    La = np.ascontiguousarray(L, dtype=np.int32)
    ba = np.ascontiguousarray(np.broadcast_to(np.asarray(beta, dtype=np.float64), (n,)))
    Ja = np.ascontiguousarray(np.broadcast_to(np.asarray(J, dtype=np.float64), (n,)))
    sa = np.ascontiguousarray(np.broadcast_to(np.asarray(seed, dtype=np.uint64), (n,)))
    return n, La, ba, Ja, sa


SW_MERGE_AUTO, SW_MERGE_LDS, SW_MERGE_GLOBAL = 0, 1, 2


def _per_replica(v, n):
    return None if v is None else np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.int32), (n,)))


def sw_batch_workspace_bytes(L, ring: int = 0, tile: int = 0, q=None, tiles=None, merge=None) -> int:
    La = np.ascontiguousarray(L, dtype=np.int32)
    if tiles is not None or merge is not None:
        qa, ta, ma = _per_replica(q, La.size), _per_replica(tiles, La.size), _per_replica(merge, La.size)
        return int(lib().sw_batch_workspace_bytes_ex(La.size, _ptr(La), None if qa is None else _ptr(qa),
                                                     None if ta is None else _ptr(ta),
                                                     None if ma is None else _ptr(ma), ring))
    if q is not None:
        qa = _per_replica(q, La.size)
        return int(lib().sw_batch_workspace_bytes_potts(La.size, _ptr(La), _ptr(qa), ring, tile))
    return int(lib().sw_batch_workspace_bytes(La.size, _ptr(La), ring, tile))


def sw_batch_create(L, beta, J, seed, init: int = SW_INIT_HOT, ring: int = 0, tile: int = 0, ws_ptr: int = 0,
                    ws_bytes: int = 0, stream_ptr: int = 0, q=None, tiles=None, merge=None) -> int:
    """q: None for Ising replicas (sw_batch_create), else the Potts q of every
    replica (sw_batch_create_potts); tiles / merge: per-replica tile widths
    and merges (sw_batch_create_ex, where q may mix 0 = Ising and Potts)."""
    n, La, ba, Ja, sa = _replica_arrays(L, beta, J, seed)
    h = ctypes.c_void_p()
    if tiles is not None or merge is not None:
        qa, ta, ma = _per_replica(q, n), _per_replica(tiles, n), _per_replica(merge, n)
        _check(lib().sw_batch_create_ex(n, _ptr(La), _ptr(ba), _ptr(Ja), _ptr(sa),
                                        None if qa is None else _ptr(qa), None if ta is None else _ptr(ta),
                                        None if ma is None else _ptr(ma), init, ring, ws_ptr or None, ws_bytes,
                                        stream_ptr or None, ctypes.byref(h)))
    elif q is not None:
        qa = _per_replica(q, n)
        _check(lib().sw_batch_create_potts(n, _ptr(La), _ptr(ba), _ptr(Ja), _ptr(sa), _ptr(qa), init, ring, tile,
                                           ws_ptr or None, ws_bytes, stream_ptr or None, ctypes.byref(h)))
    else:
        _check(lib().sw_batch_create(n, _ptr(La), _ptr(ba), _ptr(Ja), _ptr(sa), init, ring, tile, ws_ptr or None,
                                     ws_bytes, stream_ptr or None, ctypes.byref(h)))
    return h.value


def sw_batch_reset(h: int, init_mode: int = SW_INIT_HOT) -> None:
    _check(lib().sw_batch_reset(h, init_mode))


def sw_batch_sweep(h: int, n: int) -> None:
    _check(lib().sw_batch_sweep(h, n))


def sw_batch_sync(h: int) -> None:
    _check(lib().sw_batch_sync(h))


def sw_batch_observables(h: int) -> np.ndarray:
    out = np.zeros(int(lib().sw_batch_size(h)), dtype=OBS_DTYPE)
    _check(lib().sw_batch_observables(h, _ptr(out)))
    return out


def sw_batch_series(h: int, r: int, first: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=OBS_DTYPE)
    _check(lib().sw_batch_series(h, r, first, count, _ptr(out)))
    return out


def sw_batch_get_spins(h: int, r: int) -> np.ndarray:
    L = int(lib().sw_batch_lattice(h, r))
    if L == 0:
        raise SwError(SW_ERANGE, "replica index out of range")
    out = np.empty(L * L, dtype=np.int8)
    _check(lib().sw_batch_get_spins(h, r, _ptr(out), out.size))
    return out


def sw_batch_destroy(h: int) -> None:
    if h:
        lib().sw_batch_destroy(h)


# ------------------------------------------------------------------- wrapper
class Sim:
    """One lattice on the current GPU; workspace and stream come from torch."""

    def __init__(self, L: int, beta: float, J: float = 1.0, seed: int = 0, *, init: int = SW_INIT_HOT,
                 tile: int = 0, flags: int = 0, ring: int = 0, q: int = 0, dims: int = 2, device=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("Sim needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.L, self.N = L, L ** (3 if dims == 3 else 2)
        self.cfg = sw_config_init(L, beta, J, seed, init=init, tile=tile, flags=flags, ring=ring, q=q,
                                  dims=dims)
        nbytes = sw_workspace_bytes_ex(self.cfg)
        if nbytes == 0:
            # same validation as create, for the error message
            self.handle = sw_create_ex(self.cfg)
        dev = torch.device("cuda" if device is None else device)
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        # a stream of our own (default priority): the legacy null stream
        # cannot be captured into a graph
        self._stream = torch.cuda.Stream(device=dev)
        torch.cuda.current_stream(dev).synchronize()
        self.handle = sw_create_ex(self.cfg, self._ws.data_ptr(), nbytes, self._stream.cuda_stream)

    def sweep(self, n: int) -> None:
        sw_sweep(self.handle, n)

    def sync(self) -> None:
        sw_sync(self.handle)

    def reset(self, init: int = SW_INIT_HOT) -> None:
        sw_reset(self.handle, init)

    def observables(self):
        return sw_observables(self.handle)

    def profile(self, n: int) -> dict:
        return sw_profile(self.handle, n)

    def series(self, first: int, count: int) -> np.ndarray:
        return sw_series(self.handle, first, count)

    def spins(self) -> np.ndarray:
        return sw_get_spins(self.handle, self.N)

    def set_spins(self, spins: np.ndarray, next_sweep: int) -> None:
        sw_set_spins(self.handle, spins, next_sweep)

    def labels(self) -> np.ndarray:
        return sw_get_labels(self.handle, self.N)

    def cluster_hist(self) -> np.ndarray:
        return sw_cluster_hist(self.handle, self.N)

    @property
    def threshold(self) -> int:
        return sw_threshold(self.handle)

    @property
    def label_passes(self) -> int:
        """Scan/analysis passes of the last sweep (label-equivalence sims)."""
        return int(lib().sw_label_passes(self.handle))

    @property
    def next_sweep(self) -> int:
        return sw_next_sweep(self.handle)

    @property
    def tile(self) -> int:
        return int(lib().sw_tile(self.handle))

    def close(self) -> None:
        h, self.handle = getattr(self, "handle", None), None
        if h:
            sw_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Independent replicas swept together (one launch per kernel of a sweep
    for the whole batch); workspace and stream come from torch.  L is a
    sequence of lattice sides; beta, J and seed are scalars or sequences of
    the same length."""

    def __init__(self, L, beta, J=1.0, seed=0, *, init: int = SW_INIT_HOT, ring: int = 0, tile: int = 0,
                 q=None, tiles=None, merge=None, device=None):
        """q: None for Ising replicas, else the Potts q of every replica
        (a scalar or a sequence; with tiles or merge given, 0 marks an Ising
        replica); tiles / merge: per-replica tile widths (0, 32, 64) and
        merges (SW_MERGE_*), scalars or sequences."""
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("Batch needs a ROCm GPU (torch.cuda.is_available() is False)")
        n, La, ba, Ja, sa = _replica_arrays(L, beta, J, seed)
        self.L = La.tolist()
        self.q = q
        nbytes = sw_batch_workspace_bytes(La, ring, tile, q=q, tiles=tiles, merge=merge)
        if nbytes == 0:  # raises with the reason
            self.handle = sw_batch_create(La, ba, Ja, sa, init, ring, tile, q=q, tiles=tiles, merge=merge)
        dev = torch.device("cuda" if device is None else device)
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self._stream = torch.cuda.Stream(device=dev)
        torch.cuda.current_stream(dev).synchronize()
        self.handle = sw_batch_create(La, ba, Ja, sa, init, ring, tile, self._ws.data_ptr(), nbytes,
                                      self._stream.cuda_stream, q=q, tiles=tiles, merge=merge)

    def __len__(self) -> int:
        return len(self.L)

    def sweep(self, n: int) -> None:
        sw_batch_sweep(self.handle, n)

    def sync(self) -> None:
        sw_batch_sync(self.handle)

    def reset(self, init: int = SW_INIT_HOT) -> None:
        sw_batch_reset(self.handle, init)

    def observables(self) -> np.ndarray:
        return sw_batch_observables(self.handle)

    def series(self, r: int, first: int, count: int) -> np.ndarray:
        return sw_batch_series(self.handle, r, first, count)

    def spins(self, r: int) -> np.ndarray:
        return sw_batch_get_spins(self.handle, r)

    def threshold(self, r: int) -> int:
        return int(lib().sw_batch_threshold(self.handle, r))

    @property
    def next_sweep(self) -> int:
        return int(lib().sw_batch_next_sweep(self.handle))

    @property
    def tile(self) -> int:
        """The tile width every replica uses (0 if they differ)."""
        return int(lib().sw_batch_tile(self.handle))

    def replica_tile(self, r: int) -> int:
        return int(lib().sw_batch_replica_tile(self.handle, r))

    def replica_merge(self, r: int) -> int:
        return int(lib().sw_batch_replica_merge(self.handle, r))

    def close(self) -> None:
        h, self.handle = getattr(self, "handle", None), None
        if h:
            sw_batch_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# Layout of ``sw_phi4_obs`` (swmi.h).
PHI4_OBS_DTYPE = np.dtype(
    [
        ("sweep", "<u8"),
        ("e_fix", "<i8"),
        ("action", "<f8"),
        ("m_fix", "<i8", (4,)),
        ("m_abs", "<f8"),
        ("n_clusters", "<u8"),
        ("max_cluster", "<u8"),
        ("sum_sq_sizes", "<u8"),
        ("hist_log2", "<u8", (33,)),
    ]
)
PHI4_KERNELS = ("proj", "bond_union", "flatten", "reflect", "record")


class Phi4:
    """The O(4) phi^4 theory with unit fields on the L^4 periodic lattice,
    one multicluster Wolff-embedding update per sweep (paper Sec. 3);
    workspace and stream come from torch.  Fields are an (L^4, 4) float64
    array."""

    def __init__(self, L: int, kappa: float, seed: int = 0, *, init: int = SW_INIT_HOT, ring: int = 0,
                 device=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("Phi4 needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.L, self.N = L, L ** 4
        nbytes = int(lib().sw_phi4_workspace_bytes(L, ring))
        h = ctypes.c_void_p()
        if nbytes == 0:  # same validation as create, for the error message
            _check(lib().sw_phi4_create(L, kappa, seed, init, ring, None, 0, None, ctypes.byref(h)))
        dev = torch.device("cuda" if device is None else device)
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self._stream = torch.cuda.Stream(device=dev)
        torch.cuda.current_stream(dev).synchronize()
        _check(lib().sw_phi4_create(L, kappa, seed, init, ring, self._ws.data_ptr(), nbytes,
                                    self._stream.cuda_stream, ctypes.byref(h)))
        self.handle = h.value

    def sweep(self, n: int) -> None:
        _check(lib().sw_phi4_sweep(self.handle, n))

    def sync(self) -> None:
        _check(lib().sw_phi4_sync(self.handle))

    def reset(self, init: int = SW_INIT_HOT) -> None:
        _check(lib().sw_phi4_reset(self.handle, init))

    def profile(self, n: int) -> dict:
        ms = np.zeros(len(PHI4_KERNELS), dtype=np.float64)
        _check(lib().sw_phi4_profile(self.handle, n, _ptr(ms), ms.size))
        return dict(zip(PHI4_KERNELS, ms.tolist()))

    def series(self, first: int, count: int) -> np.ndarray:
        out = np.zeros(count, dtype=PHI4_OBS_DTYPE)
        _check(lib().sw_phi4_series(self.handle, first, count, _ptr(out)))
        return out

    def field(self) -> np.ndarray:
        out = np.empty((self.N, 4), dtype=np.float64)
        _check(lib().sw_phi4_get_field(self.handle, _ptr(out), out.size))
        return out

    def set_field(self, phi: np.ndarray, next_sweep: int) -> None:
        f = np.ascontiguousarray(phi, dtype=np.float64)
        _check(lib().sw_phi4_set_field(self.handle, _ptr(f), f.size, next_sweep))

    def labels(self) -> np.ndarray:
        out = np.empty(self.N, dtype=np.uint32)
        _check(lib().sw_phi4_get_labels(self.handle, _ptr(out), out.size))
        return out

    @property
    def next_sweep(self) -> int:
        return int(lib().sw_phi4_next_sweep(self.handle))

    def close(self) -> None:
        h, self.handle = getattr(self, "handle", None), None
        if h:
            lib().sw_phi4_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """Serving runtime: jobs (L, beta, J, seed, sweeps) queue for room in a
    device memory pool (a torch uint8 tensor of pool_bytes) and are advanced
    together by the batched kernels; each job's results are those of a plain
    sim run alone."""

    def __init__(self, pool_bytes: int, max_jobs: int = 256, device=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("Server needs a ROCm GPU (torch.cuda.is_available() is False)")
        dev = torch.device("cuda" if device is None else device)
        self._pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=dev)
        self._stream = torch.cuda.Stream(device=dev)
        torch.cuda.current_stream(dev).synchronize()
        h = ctypes.c_void_p()
        _check(lib().sw_server_create(self._pool.data_ptr(), int(pool_bytes), max_jobs, self._stream.cuda_stream,
                                      ctypes.byref(h)))
        self.handle = h.value
        self._done_buf = np.zeros(4096, dtype=np.int64)

    @staticmethod
    def job_bytes(L: int, sweeps: int, q: int = 0) -> int:
        if q:
            return int(lib().sw_server_job_bytes_potts(L, q, sweeps))
        return int(lib().sw_server_job_bytes(L, sweeps))

    def submit(self, L: int, beta: float, J: float = 1.0, seed: int = 0, sweeps: int = 100,
               init: int = SW_INIT_HOT, q: int = 0) -> int:
        """q = 0: an Ising job; q = 2..8: a q-state Potts job."""
        jid = ctypes.c_int64()
        if q:
            _check(lib().sw_server_submit_potts(self.handle, L, beta, J, seed, q, init, sweeps, ctypes.byref(jid)))
        else:
            _check(lib().sw_server_submit(self.handle, L, beta, J, seed, init, sweeps, ctypes.byref(jid)))
        return jid.value

    def step(self, n: int) -> list:
        nd = ctypes.c_int32()
        _check(lib().sw_server_step(self.handle, n, _ptr(self._done_buf), self._done_buf.size, ctypes.byref(nd)))
        return self._done_buf[: min(nd.value, self._done_buf.size)].tolist()

    def info(self, job: int) -> dict:
        i = sw_job_info()
        _check(lib().sw_server_job_info(self.handle, job, ctypes.byref(i)))
        return {"id": i.id, "state": i.state, "L": i.L, "sweeps_done": i.sweeps_done,
                "sweeps_total": i.sweeps_total, "bytes": i.bytes}

    def series(self, job: int, first: int, count: int) -> np.ndarray:
        out = np.zeros(count, dtype=OBS_DTYPE)
        _check(lib().sw_server_job_series(self.handle, job, first, count, _ptr(out)))
        return out

    def spins(self, job: int) -> np.ndarray:
        L = self.info(job)["L"]
        out = np.empty(L * L, dtype=np.int8)
        _check(lib().sw_server_job_spins(self.handle, job, _ptr(out), out.size))
        return out

    def release(self, job: int) -> None:
        _check(lib().sw_server_release(self.handle, job))

    def status(self) -> dict:
        q, a = ctypes.c_int32(), ctypes.c_int32()
        used, su = ctypes.c_size_t(), ctypes.c_uint64()
        _check(lib().sw_server_status(self.handle, ctypes.byref(q), ctypes.byref(a), ctypes.byref(used),
                                      ctypes.byref(su)))
        return {"queued": q.value, "active": a.value, "bytes_used": used.value, "site_updates": su.value}

    def close(self) -> None:
        h, self.handle = getattr(self, "handle", None), None
        if h:
            lib().sw_server_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
