"""FP64 CPU oracle (ctypes wrapper around md_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the package smoke check and by the
benchmark's CPU-baseline leg.  The product path never imports this package.

Each wrapper returns NumPy arrays; inputs are the same NumPy arrays the seeded input
generator produces.  Functions and the passages they follow are documented in
md_oracle.c.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "md_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

N_OBS = 16
OBS_NAMES = ["e_embed", "e_pair", "e_morse", "e_kin", "w_xx", "w_yy", "w_zz", "w_xy", "w_xz",
             "w_yz", "find_x", "find_y", "find_z", "ind_z", "nbuilds", "unused"]


def build() -> str:
    """Compile md_oracle.c with gcc (FP contraction off, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Box(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("len", C.c_double * 3),
                ("periodic", C.c_int32 * 3), ("pad", C.c_int32)]


class _Eam(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("A", "c", "d", "c0", "c1", "c2")]


class _Morse(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("D", "alpha", "r0", "rc")]


PAPER_KEYS = ("Fo", "n", "rho_e", "alpha", "P_e", "fe", "re", "beta", "a0", "a1", "a2", "a3", "d", "rc")


class _Paper(C.Structure):
    _fields_ = [(k, C.c_double) for k in PAPER_KEYS]


class _Params(C.Structure):
    _fields_ = [("box", _Box), ("eam", _Eam), ("morse", _Morse), ("mass", C.c_double),
                ("dt", C.c_double), ("v_ind", C.c_double), ("skin", C.c_double),
                ("use_lists", C.c_int32), ("cap", C.c_int32), ("potential", C.c_int32),
                ("pad", C.c_int32), ("paper", _Paper)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64 = C.c_int64
        d = C.c_double
        L.orc_wrap.argtypes = [P, i64, P]
        L.orc_neighbors.argtypes = [P, d, i64, P, i64, P, i64, P, P]
        L.orc_neighbors.restype = i64
        L.orc_cross_neighbors.argtypes = [P, d, i64, P, i64, P, d, i64, P, i64, P, P]
        L.orc_cross_neighbors.restype = i64
        L.orc_neighbors_cells.argtypes = [P, d, i64, P, i64, P, P]
        L.orc_neighbors_cells.restype = i64
        L.orc_cross_neighbors_cells.argtypes = [P, d, i64, P, i64, P, d, i64, P, P]
        L.orc_cross_neighbors_cells.restype = i64
        L.orc_density.argtypes = [P, P, i64, P, P, P, i64, P, P]
        L.orc_eam_forces.argtypes = [P, P, i64, P, P, P, i64, P, P, P, P]
        L.orc_morse_forces.argtypes = [P, P, i64, P, i64, P, d, P, P, i64, P, P]
        L.orc_sample_forces.argtypes = [P, P, P, i64, P, i64, P, d, i64, P, P, P, P, P]
        L.orc_md_run.argtypes = [P, i64, P, P, P, P, i64, P, P, i64, P]
        L.orc_md_run.restype = i64
        L.orc_evaluate.argtypes = [P, i64, P, P, P, P, i64, P, d, P, P, P, P]
        L.orc_paper_values.argtypes = [P, d, d, d, P]
        L.orc_sample_forces_paper.argtypes = [P, P, P, i64, P, i64, P, d, i64, P, P, P, P]
        L.orc_density_paper.argtypes = [P, P, i64, P, P, P, i64, P, P, P, P]
        L.orc_eam_forces_paper.argtypes = [P, P, i64, P, P, P, i64, P, P, P, P, P]
        L.orc_potential_values.argtypes = [P, P, d, P]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of the oracle's parallel loops."""
    lib().orc_set_num_threads(int(n))


def make_box(lo, length, periodic) -> _Box:
    b = _Box()
    for a in range(3):
        b.lo[a] = float(lo[a])
        b.len[a] = float(length[a])
        b.periodic[a] = int(bool(periodic[a]))
    return b


def make_eam(p: dict) -> _Eam:
    return _Eam(**{k: float(p[k]) for k in ("A", "c", "d", "c0", "c1", "c2")})


def make_morse(p: dict) -> _Morse:
    return _Morse(**{k: float(p[k]) for k in ("D", "alpha", "r0", "rc")})


def box_of(s) -> _Box:
    return make_box(s.box_lo, s.box_len, s.periodic)


def wrap(s, x=None) -> np.ndarray:
    x = _f64(s.x if x is None else x).copy()
    b = box_of(s)
    lib().orc_wrap(C.byref(b), x.shape[0], _p(x))
    return x


def neighbors(s, r: float, x=None, rows=None, cap: int = 128):
    """Brute-force neighbour sets {j != i : |x_j - x_i|^2 < r^2} (ascending j).
    Returns (cnt, idx[rows, cap]); raises if a set exceeds cap."""
    x = _f64(s.x if x is None else x)
    n = x.shape[0]
    rr = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    m = n if rr is None else rr.shape[0]
    cnt = np.zeros(max(m, 1), np.int32)
    idx = np.full((max(m, 1), cap), -1, np.int32)
    b = box_of(s)
    mx = lib().orc_neighbors(C.byref(b), float(r), n, _p(x), m, _p(rr), cap, _p(cnt), _p(idx))
    if mx > cap:
        raise ValueError(f"neighbour set of {mx} exceeds cap {cap}")
    return cnt[:m], idx[:m]


def cross_neighbors(s, r: float, x=None, ind_z: float = 0.0, rows=None, cap: int = 128):
    x = _f64(s.x if x is None else x)
    xc = _f64(s.xc).reshape(-1, 3)
    n = x.shape[0]
    rr = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    m = n if rr is None else rr.shape[0]
    cnt = np.zeros(max(m, 1), np.int32)
    idx = np.full((max(m, 1), cap), -1, np.int32)
    b = box_of(s)
    mx = lib().orc_cross_neighbors(C.byref(b), float(r), n, _p(x), xc.shape[0], _p(xc),
                                   float(ind_z), m, _p(rr), cap, _p(cnt), _p(idx))
    if mx > cap:
        raise ValueError(f"cross set of {mx} exceeds cap {cap}")
    return cnt[:m], idx[:m]


def neighbors_cells(s, r: float, x=None, cap: int = 128):
    """The sets of `neighbors` for every atom, found through a cell grid (large systems)."""
    x = _f64(s.x if x is None else x)
    n = x.shape[0]
    cnt = np.zeros(max(n, 1), np.int32)
    idx = np.full((max(n, 1), cap), -1, np.int32)
    b = box_of(s)
    mx = lib().orc_neighbors_cells(C.byref(b), float(r), n, _p(x), cap, _p(cnt), _p(idx))
    if mx > cap:
        raise ValueError(f"neighbour set of {mx} exceeds cap {cap}")
    return cnt[:n], idx[:n]


def cross_neighbors_cells(s, r: float, x=None, ind_z: float = 0.0, cap: int = 128):
    """The sets of `cross_neighbors` for every atom, found through a cell grid of the carbons."""
    x = _f64(s.x if x is None else x)
    xc = _f64(s.xc).reshape(-1, 3)
    n = x.shape[0]
    cnt = np.zeros(max(n, 1), np.int32)
    idx = np.full((max(n, 1), cap), -1, np.int32)
    b = box_of(s)
    mx = lib().orc_cross_neighbors_cells(C.byref(b), float(r), n, _p(x), xc.shape[0], _p(xc),
                                         float(ind_z), cap, _p(cnt), _p(idx))
    if mx > cap:
        raise ValueError(f"cross set of {mx} exceeds cap {cap}")
    return cnt[:n], idx[:n]


def neighbor_sets(cnt, idx):
    return [idx[t, :cnt[t]].tolist() for t in range(cnt.shape[0])]


def density(s, x=None, lists=None):
    """rho_i and F'(rho_i) (all pairs, or over a (cnt, idx) list)."""
    x = _f64(s.x if x is None else x)
    n = x.shape[0]
    rho = np.zeros(max(n, 1))
    dF = np.zeros(max(n, 1))
    b, e = box_of(s), make_eam(s.eam)
    cnt, idx = (None, None) if lists is None else lists
    cap = 0 if lists is None else idx.shape[1]
    lib().orc_density(C.byref(b), C.byref(e), n, _p(x), _p(cnt), _p(idx), cap, _p(rho), _p(dF))
    return rho[:n], dF[:n]


def eam_forces(s, dF, x=None, lists=None):
    """Eq. (1) forces, per-atom half pair energy and per-atom half virial (6 comps)."""
    x = _f64(s.x if x is None else x)
    n = x.shape[0]
    f = np.zeros((max(n, 1), 3))
    ep = np.zeros(max(n, 1))
    vir = np.zeros((max(n, 1), 6))
    b, e = box_of(s), make_eam(s.eam)
    cnt, idx = (None, None) if lists is None else lists
    cap = 0 if lists is None else idx.shape[1]
    dF = _f64(dF)
    lib().orc_eam_forces(C.byref(b), C.byref(e), n, _p(x), _p(cnt), _p(idx), cap, _p(dF),
                         _p(f), _p(ep), _p(vir))
    return f[:n], ep[:n], vir[:n]


def morse_forces(s, x=None, ind_z: float = 0.0, lists=None):
    """Per-Cr-atom Morse force and per-atom shifted Morse energy."""
    x = _f64(s.x if x is None else x)
    xc = _f64(s.xc).reshape(-1, 3)
    n = x.shape[0]
    fm = np.zeros((max(n, 1), 3))
    em = np.zeros(max(n, 1))
    b, m = box_of(s), make_morse(s.morse)
    cnt, idx = (None, None) if lists is None else lists
    cap = 0 if lists is None else idx.shape[1]
    lib().orc_morse_forces(C.byref(b), C.byref(m), n, _p(x), xc.shape[0], _p(xc), float(ind_z),
                           _p(cnt), _p(idx), cap, _p(fm), _p(em))
    return fm[:n], em[:n]


def sample_forces(s, sample, x=None, ind_z: float = 0.0):
    """Total force, rho, F'(rho) and Morse force of the sampled atoms, each from all-atom
    loops (for systems too large for whole-system all-pairs evaluation)."""
    x = _f64(s.x if x is None else x)
    xc = _f64(s.xc).reshape(-1, 3)
    smp = np.ascontiguousarray(sample, dtype=np.int64)
    ns = smp.shape[0]
    f = np.zeros((max(ns, 1), 3))
    rho = np.zeros(max(ns, 1))
    dF = np.zeros(max(ns, 1))
    fm = np.zeros((max(ns, 1), 3))
    b, e, m = box_of(s), make_eam(s.eam), make_morse(s.morse)
    lib().orc_sample_forces(C.byref(b), C.byref(e), C.byref(m), x.shape[0], _p(x), xc.shape[0],
                            _p(xc), float(ind_z), ns, _p(smp), _p(f), _p(rho), _p(dF), _p(fm))
    return f[:ns], rho[:ns], dF[:ns], fm[:ns]


def sample_forces_paper(s, sample, x=None, ind_z: float = 0.0):
    """sample_forces for a system with the paper's form: (force, rho, F'(rho)) of the sampled
    atoms from all-atom loops."""
    x = _f64(s.x if x is None else x)
    xc = _f64(s.xc).reshape(-1, 3)
    smp = np.ascontiguousarray(sample, dtype=np.int64)
    ns = smp.shape[0]
    f = np.zeros((max(ns, 1), 3))
    rho = np.zeros(max(ns, 1))
    dF = np.zeros(max(ns, 1))
    b, pp, m = box_of(s), make_paper(s.paper), make_morse(s.morse)
    lib().orc_sample_forces_paper(C.byref(b), C.byref(pp), C.byref(m), x.shape[0], _p(x), xc.shape[0],
                                  _p(xc), float(ind_z), ns, _p(smp), _p(f), _p(rho), _p(dF))
    return f[:ns], rho[:ns], dF[:ns]


def params_of(s, use_lists=False, cap: int = 96) -> _Params:
    """use_lists: False (all pairs), True (Verlet lists by brute force) or "cells" (the same
    lists through a cell grid)."""
    P = _Params()
    P.box = box_of(s)
    P.eam = make_eam(s.eam)
    P.morse = make_morse(s.morse)
    P.mass = float(s.mass)
    P.dt = float(s.dt)
    P.v_ind = float(s.v_ind)
    P.skin = float(s.skin)
    P.use_lists = 2 if use_lists == "cells" else int(bool(use_lists))
    P.cap = int(cap)
    P.potential = 1 if getattr(s, "potential", "fs") == "paper" else 0
    P.paper = make_paper(getattr(s, "paper", None) or {k: 0.0 for k in PAPER_KEYS})
    return P


def make_paper(p: dict) -> _Paper:
    return _Paper(**{k: float(p[k]) for k in PAPER_KEYS})


def paper_values(s, r: float, rho: float = 1.0, P: float = 1.0) -> dict:
    """f, f', Phi, Phi' at r, F, F' at rho and M, M' at P of the paper's form."""
    out = np.zeros(8)
    pp = make_paper(s.paper)
    lib().orc_paper_values(C.byref(pp), float(r), float(rho), float(P), _p(out))
    return dict(f=out[0], df=out[1], phi=out[2], dphi=out[3], F=out[4], dF=out[5], M=out[6], dM=out[7])


def evaluate(s, x=None, ind_z: float = 0.0):
    """Forces (EAM + Morse), rho, F'(rho), Morse force and the observables vector of one
    configuration, all pairs (with the paper's form also P and M'(P); obs[e_embed] then
    holds sum F(rho) + M(P)).  obs[e_kin], obs[ind_z], obs[nbuilds] are not filled."""
    x = _f64(s.x if x is None else x)
    n = x.shape[0]
    xc = _f64(s.xc).reshape(-1, 3)
    f = np.zeros((max(n, 1), 3))
    rho = np.zeros(max(n, 1))
    dF = np.zeros(max(n, 1))
    fm = np.zeros((max(n, 1), 3))
    obs = np.zeros(N_OBS)
    Pd = np.zeros(max(n, 1))
    dM = np.zeros(max(n, 1))
    P = params_of(s)
    lib().orc_evaluate(C.byref(P), n, _p(x), _p(f), _p(rho), _p(dF), xc.shape[0], _p(xc),
                       float(ind_z), _p(fm), _p(obs), _p(Pd), _p(dM))
    return dict(f=f[:n], rho=rho[:n], dF=dF[:n], fm=fm[:n], obs=obs, P=Pd[:n], dM=dM[:n])


def md_run(s, nsteps: int, use_lists=False, cap: int = 96, ind_z: float = 0.0):
    """Velocity-Verlet trajectory (Tasks 1-5); use_lists as in params_of.  Returns dict with the final x, v, f,
    indenter displacement and the (nsteps+1, N_OBS) observables table."""
    x = _f64(s.x).copy()
    v = _f64(s.v).copy()
    n = x.shape[0]
    f = np.zeros((max(n, 1), 3))
    fixed = np.ascontiguousarray(s.fixed, dtype=np.uint8)
    xc = _f64(s.xc).reshape(-1, 3)
    obs = np.zeros((nsteps + 1, N_OBS))
    iz = C.c_double(float(ind_z))
    P = params_of(s, use_lists, cap)
    ovf = lib().orc_md_run(C.byref(P), n, _p(x), _p(v), _p(f), _p(fixed), xc.shape[0], _p(xc),
                           C.byref(iz), int(nsteps), _p(obs))
    if ovf:
        raise ValueError(f"oracle list overflow: needs cap {ovf}")
    return dict(x=x, v=v, f=f[:n], ind_z=iz.value, obs=obs)


def potential_values(s, r: float) -> dict:
    out = np.zeros(8)
    e, m = make_eam(s.eam), make_morse(s.morse)
    lib().orc_potential_values(C.byref(e), C.byref(m), float(r), _p(out))
    return dict(phi=out[0], dphi=out[1], f=out[2], df=out[3], F=out[4], dF=out[5],
                phiM=out[6], dphiM=out[7])


def total_energy(obs_row) -> float:
    return float(obs_row[0] + obs_row[1] + obs_row[2] + obs_row[3])


class use_library:
    """Temporarily route every wrapper through another build of md_oracle.c (used by the
    mutation tests, which compile deliberately broken copies)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self._saved = lib()
        _lib = None
        saved_path = globals()["_LIB"]
        globals()["_LIB"] = self.path
        try:
            lib()
        finally:
            globals()["_LIB"] = saved_path
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False
