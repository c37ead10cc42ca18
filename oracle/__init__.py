"""CPU oracle for the Swendsen-Wang sweep (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  It wraps ``sw_oracle.c`` -- a plain
sequential C implementation written from the paper's Sec. 2 (bond formation,
cluster formation, assignment of new spins, measurement) -- through ctypes.
It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Record layout of ``orc_obs`` (sw_oracle.h).
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


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc -O2 (plain C, one thread)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
             "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _bind(l: ctypes.CDLL) -> ctypes.CDLL:
    P = ctypes.c_void_p
    i32, u32, u64, i64, f64 = (ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64,
                               ctypes.c_int64, ctypes.c_double)
    l.orc_philox4x32_10.argtypes = [P, P, P]
    l.orc_philox4x32_10.restype = None
    l.orc_threshold.argtypes = [f64, f64]
    l.orc_threshold.restype = u32
    l.orc_init.argtypes = [i32, u64, i32, P]
    l.orc_init.restype = None
    l.orc_bonds.argtypes = [i32, u32, u64, u32, P, P]
    l.orc_bonds.restype = None
    l.orc_label.argtypes = [i32, P, P]
    l.orc_label.restype = None
    l.orc_flip_spin.argtypes = [u64, u32, u32]
    l.orc_flip_spin.restype = i32
    l.orc_assign.argtypes = [i32, u64, u32, P, P]
    l.orc_assign.restype = None
    l.orc_observe.argtypes = [i32, f64, u64, P, P, P, P]
    l.orc_observe.restype = None
    l.orc_sweep.argtypes = [i32, f64, u32, u64, u32, P, P, P, P, P]
    l.orc_sweep.restype = ctypes.c_int
    l.orc_run.argtypes = [i32, f64, u32, u64, u32, i64, P, P]
    l.orc_run.restype = ctypes.c_int
    l.orc_chains.argtypes = [i32, f64, u32, u64, i64, i32, P, P]
    l.orc_chains.restype = ctypes.c_int
    l.orc_one_step_codes.argtypes = [i32, u32, u64, i64, u32, P, P]
    l.orc_one_step_codes.restype = ctypes.c_int
    l.orc_potts_threshold.argtypes = [f64, f64]
    l.orc_potts_threshold.restype = u32
    l.orc_potts_init.argtypes = [i32, u64, i32, i32, P]
    l.orc_potts_init.restype = None
    l.orc_potts_spin.argtypes = [u64, u32, u32, i32]
    l.orc_potts_spin.restype = i32
    l.orc_potts_sweep.argtypes = [i32, f64, u32, i32, u64, u32, P, P, P]
    l.orc_potts_sweep.restype = ctypes.c_int
    l.orc_potts_run.argtypes = [i32, f64, u32, i32, u64, u32, i64, P, P]
    l.orc_potts_run.restype = ctypes.c_int
    l.orc_potts_chains.argtypes = [i32, f64, u32, i32, u64, i64, i32, P, P]
    l.orc_potts_chains.restype = ctypes.c_int
    l.orc_cubic_init.argtypes = [i32, u64, i32, i32, P]
    l.orc_cubic_init.restype = None
    l.orc_cubic_bonds.argtypes = [i32, u32, u64, u32, P, P]
    l.orc_cubic_bonds.restype = None
    l.orc_cubic_label.argtypes = [i32, P, P]
    l.orc_cubic_label.restype = None
    l.orc_cubic_observe.argtypes = [i32, f64, i32, u64, P, P, P, P]
    l.orc_cubic_observe.restype = None
    l.orc_cubic_sweep.argtypes = [i32, f64, u32, i32, u64, u32, P, P, P, P, P]
    l.orc_cubic_sweep.restype = ctypes.c_int
    l.orc_cubic_run.argtypes = [i32, f64, u32, i32, u64, u32, i64, P, P]
    l.orc_cubic_run.restype = ctypes.c_int
    l.orc_cubic_chains.argtypes = [i32, f64, u32, i32, u64, i64, i32, P, P]
    l.orc_cubic_chains.restype = ctypes.c_int
    l.orc_phi4_direction.argtypes = [u64, u32, P, P]
    l.orc_phi4_direction.restype = None
    l.orc_phi4_expm.argtypes = [f64]
    l.orc_phi4_expm.restype = f64
    l.orc_phi4_init.argtypes = [i32, i32, u64, i32, P]
    l.orc_phi4_init.restype = None
    l.orc_phi4_bonds.argtypes = [i32, i32, f64, u64, u32, P, P]
    l.orc_phi4_bonds.restype = None
    l.orc_phi4_label.argtypes = [i32, i32, P, P]
    l.orc_phi4_label.restype = None
    l.orc_phi4_flip.argtypes = [u64, u32, u32]
    l.orc_phi4_flip.restype = i32
    l.orc_phi4_reflect.argtypes = [i32, i32, u64, u32, P, P]
    l.orc_phi4_reflect.restype = None
    l.orc_phi4_observe.argtypes = [i32, i32, f64, u64, P, P, P]
    l.orc_phi4_observe.restype = None
    l.orc_phi4_sweep.argtypes = [i32, i32, f64, u64, u32, P, P, P, P]
    l.orc_phi4_sweep.restype = ctypes.c_int
    l.orc_phi4_run.argtypes = [i32, i32, f64, u64, u32, i64, P, P]
    l.orc_phi4_run.restype = ctypes.c_int
    return l


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


class using:
    """Context manager that routes every call of this module to another
    build of the oracle (used by the tests that plant mistakes in a copy of
    sw_oracle.c and check that the pins catch them)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = _bind(ctypes.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved


def build_variant(source: str, out_dir: str, name: str) -> str:
    """Compiles C source text (a modified copy of sw_oracle.c) to a shared
    library in out_dir and returns its path."""
    src = os.path.join(out_dir, name + ".c")
    with open(src, "w") as f:
        f.write(source)
    so = os.path.join(out_dir, name + ".so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-I" + _HERE,
                           "-o", so, src, "-lm"])
    return so


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def threshold(beta: float, J: float = 1.0) -> int:
    return int(lib().orc_threshold(beta, J))


def init(L: int, seed: int, cold: bool = False) -> np.ndarray:
    s = np.empty(L * L, dtype=np.int8)
    lib().orc_init(L, seed, 1 if cold else 0, _p(s))
    return s


def bonds(L: int, T: int, seed: int, t: int, spins: np.ndarray) -> np.ndarray:
    sp = np.ascontiguousarray(spins, dtype=np.int8)
    b = np.empty(L * L, dtype=np.uint8)
    lib().orc_bonds(L, T, seed, t, _p(sp), _p(b))
    return b


def label(L: int, bond_mask: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(bond_mask, dtype=np.uint8)
    lab = np.empty(L * L, dtype=np.uint32)
    lib().orc_label(L, _p(b), _p(lab))
    return lab


def flip_spin(seed: int, t: int, root: int) -> int:
    return int(lib().orc_flip_spin(seed, t, root))


def assign(L: int, seed: int, t: int, labels: np.ndarray) -> np.ndarray:
    lab = np.ascontiguousarray(labels, dtype=np.uint32)
    s = np.empty(L * L, dtype=np.int8)
    lib().orc_assign(L, seed, t, _p(lab), _p(s))
    return s


def observe(L: int, J: float, sweep: int, spins: np.ndarray, labels=None,
            dense: bool = False):
    sp = np.ascontiguousarray(spins, dtype=np.int8)
    lab = None if labels is None else np.ascontiguousarray(labels, dtype=np.uint32)
    rec = np.zeros(1, dtype=OBS_DTYPE)
    d = np.zeros(L * L + 1, dtype=np.uint64) if dense else None
    lib().orc_observe(L, J, sweep, _p(sp), _p(lab), _p(rec), _p(d))
    return (rec[0], d) if dense else rec[0]


def sweep(L: int, J: float, T: int, seed: int, t: int, spins: np.ndarray,
          dense: bool = False):
    """One sweep in place on ``spins``; returns (record, labels, bonds[, dense])."""
    assert spins.dtype == np.int8 and spins.flags.c_contiguous and spins.size == L * L
    lab = np.empty(L * L, dtype=np.uint32)
    b = np.empty(L * L, dtype=np.uint8)
    rec = np.zeros(1, dtype=OBS_DTYPE)
    d = np.zeros(L * L + 1, dtype=np.uint64) if dense else None
    rc = lib().orc_sweep(L, J, T, seed, t, _p(spins), _p(lab), _p(b), _p(rec), _p(d))
    if rc != 0:
        raise MemoryError("oracle sweep: allocation failed")
    if dense:
        return rec[0], lab, b, d
    return rec[0], lab, b


def run(L: int, J: float, T: int, seed: int, t0: int, count: int,
        spins: np.ndarray) -> np.ndarray:
    """``count`` sweeps in place on ``spins``; returns their records."""
    assert spins.dtype == np.int8 and spins.flags.c_contiguous and spins.size == L * L
    recs = np.zeros(count, dtype=OBS_DTYPE)
    rc = lib().orc_run(L, J, T, seed, t0, count, _p(spins), _p(recs))
    if rc != 0:
        raise MemoryError("oracle run: allocation failed")
    return recs


def chains(L: int, J: float, T: int, seed0: int, nchains: int, nsweeps: int):
    e = np.zeros(nchains, dtype=np.int64)
    m = np.zeros(nchains, dtype=np.int64)
    rc = lib().orc_chains(L, J, T, seed0, nchains, nsweeps, _p(e), _p(m))
    if rc != 0:
        raise MemoryError("oracle chains: allocation failed")
    return e, m


def one_step_codes(L: int, T: int, seed0: int, nseeds: int, t: int,
                   start: np.ndarray) -> np.ndarray:
    st = np.ascontiguousarray(start, dtype=np.int8)
    codes = np.zeros(nseeds, dtype=np.uint64)
    rc = lib().orc_one_step_codes(L, T, seed0, nseeds, t, _p(st), _p(codes))
    if rc != 0:
        raise ValueError("oracle one_step_codes: lattice too large")
    return codes


# ------------------------------------------------------------ q-state Potts
def potts_threshold(beta: float, J: float = 1.0) -> int:
    return int(lib().orc_potts_threshold(beta, J))


def potts_init(L: int, seed: int, q: int, cold: bool = False) -> np.ndarray:
    s = np.empty(L * L, dtype=np.int8)
    lib().orc_potts_init(L, seed, q, 1 if cold else 0, _p(s))
    return s


def potts_spin(seed: int, t: int, root: int, q: int) -> int:
    return int(lib().orc_potts_spin(seed, t, root, q))


def potts_sweep(L: int, J: float, T: int, q: int, seed: int, t: int, spins: np.ndarray):
    """One Potts sweep in place on ``spins``; returns (record, labels)."""
    assert spins.dtype == np.int8 and spins.flags.c_contiguous and spins.size == L * L
    lab = np.empty(L * L, dtype=np.uint32)
    rec = np.zeros(1, dtype=OBS_DTYPE)
    if lib().orc_potts_sweep(L, J, T, q, seed, t, _p(spins), _p(lab), _p(rec)) != 0:
        raise MemoryError("oracle potts sweep: allocation failed")
    return rec[0], lab


def potts_run(L: int, J: float, T: int, q: int, seed: int, t0: int, count: int,
              spins: np.ndarray) -> np.ndarray:
    assert spins.dtype == np.int8 and spins.flags.c_contiguous and spins.size == L * L
    recs = np.zeros(count, dtype=OBS_DTYPE)
    if lib().orc_potts_run(L, J, T, q, seed, t0, count, _p(spins), _p(recs)) != 0:
        raise MemoryError("oracle potts run: allocation failed")
    return recs


def potts_chains(L: int, J: float, T: int, q: int, seed0: int, nchains: int, nsweeps: int):
    e = np.zeros(nchains, dtype=np.int64)
    n0 = np.zeros(nchains, dtype=np.int64)
    if lib().orc_potts_chains(L, J, T, q, seed0, nchains, nsweeps, _p(e), _p(n0)) != 0:
        raise MemoryError("oracle potts chains: allocation failed")
    return e, n0


# ------------------------------------------------------- simple cubic lattice
# L x L x L sites, s = (z*L + y)*L + x; q = 0 is the Ising model (threshold
# ``threshold``), q = 2..8 the Potts model (threshold ``potts_threshold``).
def cubic_init(L: int, seed: int, q: int = 0, cold: bool = False) -> np.ndarray:
    s = np.empty(L ** 3, dtype=np.int8)
    lib().orc_cubic_init(L, seed, q, 1 if cold else 0, _p(s))
    return s


def cubic_bonds(L: int, T: int, seed: int, t: int, spins: np.ndarray) -> np.ndarray:
    sp = np.ascontiguousarray(spins, dtype=np.int8)
    assert sp.size == L ** 3
    b = np.empty(L ** 3, dtype=np.uint8)
    lib().orc_cubic_bonds(L, T, seed, t, _p(sp), _p(b))
    return b


def cubic_label(L: int, bond_mask: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(bond_mask, dtype=np.uint8)
    assert b.size == L ** 3
    lab = np.empty(L ** 3, dtype=np.uint32)
    lib().orc_cubic_label(L, _p(b), _p(lab))
    return lab


def cubic_observe(L: int, J: float, q: int, sweep: int, spins: np.ndarray, labels=None,
                  dense: bool = False):
    sp = np.ascontiguousarray(spins, dtype=np.int8)
    lab = None if labels is None else np.ascontiguousarray(labels, dtype=np.uint32)
    rec = np.zeros(1, dtype=OBS_DTYPE)
    d = np.zeros(L ** 3 + 1, dtype=np.uint64) if dense else None
    lib().orc_cubic_observe(L, J, q, sweep, _p(sp), _p(lab), _p(rec), _p(d))
    return (rec[0], d) if dense else rec[0]


def cubic_sweep(L: int, J: float, T: int, q: int, seed: int, t: int, spins: np.ndarray,
                dense: bool = False):
    """One sweep in place on ``spins``; returns (record, labels, bonds[, dense])."""
    n = L ** 3
    assert spins.dtype == np.int8 and spins.flags.c_contiguous and spins.size == n
    lab = np.empty(n, dtype=np.uint32)
    b = np.empty(n, dtype=np.uint8)
    rec = np.zeros(1, dtype=OBS_DTYPE)
    d = np.zeros(n + 1, dtype=np.uint64) if dense else None
    if lib().orc_cubic_sweep(L, J, T, q, seed, t, _p(spins), _p(lab), _p(b), _p(rec), _p(d)) != 0:
        raise MemoryError("oracle cubic sweep: allocation failed")
    if dense:
        return rec[0], lab, b, d
    return rec[0], lab, b


def cubic_run(L: int, J: float, T: int, q: int, seed: int, t0: int, count: int,
              spins: np.ndarray) -> np.ndarray:
    assert spins.dtype == np.int8 and spins.flags.c_contiguous and spins.size == L ** 3
    recs = np.zeros(count, dtype=OBS_DTYPE)
    if lib().orc_cubic_run(L, J, T, q, seed, t0, count, _p(spins), _p(recs)) != 0:
        raise MemoryError("oracle cubic run: allocation failed")
    return recs


def cubic_chains(L: int, J: float, T: int, q: int, seed0: int, nchains: int, nsweeps: int):
    """Final e_sum and m_sum (Ising) or count of value 0 (Potts) of
    independent hot-start chains."""
    e = np.zeros(nchains, dtype=np.int64)
    m = np.zeros(nchains, dtype=np.int64)
    if lib().orc_cubic_chains(L, J, T, q, seed0, nchains, nsweeps, _p(e), _p(m)) != 0:
        raise MemoryError("oracle cubic chains: allocation failed")
    return e, m


# ------------------------------------------------- O(4) model (phi^4, unit fields)
# D-dimensional periodic hypercube of side L, s = sum_mu x_mu L^mu, fields as
# an (N, 4) float64 array; one multicluster Wolff-embedding update per sweep.
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


def phi4_direction(seed: int, t: int):
    """(r, rr): the unnormalised random direction of sweep t and r . r."""
    r = np.zeros(4, dtype=np.float64)
    rr = np.zeros(1, dtype=np.float64)
    lib().orc_phi4_direction(seed, t, _p(r), _p(rr))
    return r, float(rr[0])


def phi4_expm(a: float) -> float:
    return float(lib().orc_phi4_expm(a))


def phi4_init(D: int, L: int, seed: int, cold: bool = False) -> np.ndarray:
    f = np.empty((L ** D, 4), dtype=np.float64)
    lib().orc_phi4_init(D, L, seed, 1 if cold else 0, _p(f))
    return f


def _phi(phi: np.ndarray, n: int) -> np.ndarray:
    assert phi.dtype == np.float64 and phi.flags.c_contiguous and phi.shape == (n, 4)
    return phi


def phi4_bonds(D: int, L: int, kappa: float, seed: int, t: int, phi: np.ndarray) -> np.ndarray:
    f = _phi(phi, L ** D)
    b = np.empty(L ** D, dtype=np.uint8)
    lib().orc_phi4_bonds(D, L, kappa, seed, t, _p(f), _p(b))
    return b


def phi4_label(D: int, L: int, bond_mask: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(bond_mask, dtype=np.uint8)
    assert b.size == L ** D
    lab = np.empty(L ** D, dtype=np.uint32)
    lib().orc_phi4_label(D, L, _p(b), _p(lab))
    return lab


def phi4_flip(seed: int, t: int, root: int) -> int:
    return int(lib().orc_phi4_flip(seed, t, root))


def phi4_reflect(D: int, L: int, seed: int, t: int, labels: np.ndarray, phi: np.ndarray) -> None:
    """Reflects, in place, the sites of the clusters drawn for reflection."""
    lab = np.ascontiguousarray(labels, dtype=np.uint32)
    lib().orc_phi4_reflect(D, L, seed, t, _p(lab), _p(_phi(phi, L ** D)))


def phi4_observe(D: int, L: int, kappa: float, sweep: int, phi: np.ndarray, labels=None):
    lab = None if labels is None else np.ascontiguousarray(labels, dtype=np.uint32)
    rec = np.zeros(1, dtype=PHI4_OBS_DTYPE)
    lib().orc_phi4_observe(D, L, kappa, sweep, _p(_phi(phi, L ** D)), _p(lab), _p(rec))
    return rec[0]


def phi4_sweep(D: int, L: int, kappa: float, seed: int, t: int, phi: np.ndarray):
    """One multicluster update in place on ``phi``; returns (record, labels, bonds)."""
    n = L ** D
    lab = np.empty(n, dtype=np.uint32)
    b = np.empty(n, dtype=np.uint8)
    rec = np.zeros(1, dtype=PHI4_OBS_DTYPE)
    if lib().orc_phi4_sweep(D, L, kappa, seed, t, _p(_phi(phi, n)), _p(lab), _p(b), _p(rec)) != 0:
        raise MemoryError("oracle phi4 sweep: allocation failed")
    return rec[0], lab, b


def phi4_run(D: int, L: int, kappa: float, seed: int, t0: int, count: int, phi: np.ndarray) -> np.ndarray:
    """``count`` updates in place on ``phi``; returns their records."""
    recs = np.zeros(count, dtype=PHI4_OBS_DTYPE)
    if lib().orc_phi4_run(D, L, kappa, seed, t0, count, _p(_phi(phi, L ** D)), _p(recs)) != 0:
        raise MemoryError("oracle phi4 run: allocation failed")
    return recs
