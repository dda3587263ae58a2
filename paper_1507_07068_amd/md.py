"""Python binding of the C ABI in include/md.h (ctypes; argument marshalling only).

Device memory and streams come from PyTorch-ROCm; every step of the MD path runs in the
HIP kernels of libmd.so.  There is no CPU fallback: if the library or a GPU is missing,
constructing a ``Simulation`` raises.

Function names follow the C ABI: md_build_neighbors, md_eam_forces, md_morse_forces,
md_verlet_step, md_energy (plus md_check and set-up calls).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmd.so")

# constants of md.h
MD_OK, MD_ERR_ARG, MD_ERR_HIP, MD_ERR_STATE = 0, 1, 2, 3
MD_TILE = 256
MD_FP64, MD_MIXED = 0, 1
MD_PHASE_KICK_DRIFT, MD_PHASE_KICK = 1, 2
MD_F_DENSITY, MD_F_FORCE, MD_F_MORSE, MD_F_KICK, MD_F_ENERGY, MD_F_MIXED = 1, 2, 4, 8, 16, 32
MD_B_FORCE = 1
MD_NOBS = 16
MD_E_EMBED, MD_E_PAIR, MD_E_MORSE, MD_E_KIN, MD_W_XX, MD_F_IND_X, MD_IND_Z, MD_NBUILDS = 0, 1, 2, 3, 4, 10, 13, 14
MD_SCRATCH_BYTES = 16 << 20
OBS = ["e_embed", "e_pair", "e_morse", "e_kin", "w_xx", "w_yy", "w_zz", "w_xy", "w_xz", "w_yz",
       "find_x", "find_y", "find_z", "ind_z", "nbuilds", "unused"]

API = ["md_system_create", "md_system_destroy", "md_system_atoms", "md_system_carbons",
       "md_replica_offset", "md_workspace_bytes", "md_workspace_bind", "md_workspace_bind_static",
       "md_build_neighbors",
       "md_eam_forces", "md_morse_forces", "md_verlet_step", "md_energy", "md_run",
       "md_graph_create", "md_graph_launch", "md_graph_destroy", "md_set_indenter_velocity",
       "md_check", "md_clear_flags", "md_strerror"]


class EamParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("A", "c", "d", "c0", "c1", "c2")]


class MorseParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("D", "alpha", "r0", "rc")]


PAPER_KEYS = ("Fo", "n", "rho_e", "alpha", "P_e", "fe", "re", "beta", "a0", "a1", "a2", "a3", "d", "rc")
MD_POT_FS, MD_POT_PAPER = 0, 1


class PaperParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in PAPER_KEYS]


class Params(C.Structure):
    _fields_ = [("eam", EamParams), ("morse", MorseParams), ("mass", C.c_double),
                ("dt", C.c_double), ("v_ind", C.c_double), ("skin", C.c_double),
                ("cap", C.c_int32), ("xcap", C.c_int32), ("tpa", C.c_int32), ("shadow", C.c_int32),
                ("potential", C.c_int32), ("icap", C.c_int32), ("paper", PaperParams),
                ("list_tgt", C.c_int32), ("pad", C.c_int32)]


class ReplicaDesc(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("len", C.c_double * 3), ("periodic", C.c_int32 * 3),
                ("n", C.c_int32), ("n_c", C.c_int32), ("pad", C.c_int32)]


class Atoms(C.Structure):
    _fields_ = [("q", C.c_void_p), ("v", C.c_void_p), ("f", C.c_void_p), ("fixed", C.c_void_p),
                ("id", C.c_void_p), ("xc", C.c_void_p)]


class Lists(C.Structure):
    _fields_ = [("idx", C.c_void_p), ("cnt", C.c_void_p), ("xidx", C.c_void_p),
                ("xcnt", C.c_void_p), ("iidx", C.c_void_p), ("icnt", C.c_void_p)]


class Status(C.Structure):
    _fields_ = [("overflow", C.c_int32), ("xoverflow", C.c_int32), ("nonfinite", C.c_int32),
                ("nbuilds", C.c_int32), ("sync_timeout", C.c_int32), ("nnear", C.c_int32),
                ("ioverflow", C.c_int32), ("pad", C.c_int32)]


MD_TRACE_EVENTS = 8


class Trace(C.Structure):
    _fields_ = [("events", C.c_void_p), ("builds", C.c_void_p)]


# A Cr-Cr list entry keeps the neighbour's slot in its low 27 bits (the bits above give the
# neighbour's cell relative to the atom's cell at the build).
LIST_IDX_MASK = (1 << 27) - 1


class MDError(RuntimeError):
    pass


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmd.so (built in-tree by __graft_entry__.build()).  Raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise MDError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(path)
    P, i32, u32, i64, sz = C.c_void_p, C.c_int32, C.c_uint32, C.c_int64, C.c_size_t
    L.md_system_create.argtypes = [P, i32, P, C.POINTER(P)]
    L.md_system_create.restype = C.c_int
    L.md_system_destroy.argtypes = [P]
    L.md_system_destroy.restype = None
    L.md_system_atoms.argtypes = [P]
    L.md_system_atoms.restype = i64
    L.md_system_carbons.argtypes = [P]
    L.md_system_carbons.restype = i64
    L.md_replica_offset.argtypes = [P, i32]
    L.md_replica_offset.restype = i64
    L.md_workspace_bytes.argtypes = [P]
    L.md_workspace_bytes.restype = sz
    L.md_workspace_bind.argtypes = [P, P, sz, P]
    L.md_workspace_bind_static.argtypes = [P, P]
    L.md_build_neighbors.argtypes = [P, P, P, u32, P]
    L.md_eam_forces.argtypes = [P, P, P, u32, P, P]
    L.md_morse_forces.argtypes = [P, P, P, u32, P]
    L.md_verlet_step.argtypes = [P, i32, P, P]
    L.md_energy.argtypes = [P, P, P, P]
    L.md_run.argtypes = [P, P, P, i32, u32, i32, P, P, P]
    L.md_graph_create.argtypes = [P, P, P, i32, u32, i32, P, P, C.POINTER(P)]
    L.md_graph_launch.argtypes = [P, P]
    L.md_graph_destroy.argtypes = [P]
    L.md_set_indenter_velocity.argtypes = [P, C.c_double]
    L.md_check.argtypes = [P, P, P]
    L.md_clear_flags.argtypes = [P, P]
    L.md_strerror.argtypes = [C.c_int]
    L.md_strerror.restype = C.c_char_p
    for name in ("md_workspace_bind", "md_workspace_bind_static", "md_build_neighbors", "md_eam_forces", "md_morse_forces",
                 "md_verlet_step", "md_energy", "md_run", "md_graph_create", "md_graph_launch",
                 "md_graph_destroy", "md_set_indenter_velocity", "md_check", "md_clear_flags"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _ok(code: int, what: str):
    if code != MD_OK:
        msg = load_library().md_strerror(code).decode()
        raise MDError(f"{what}: {msg} ({code})")


def make_params(s, cap: int = 64, xcap: int = 64, tpa: int = 1, shadow: bool = False, icap: int = 0,
                list_tgt: int = 0) -> Params:
    p = Params()
    p.eam = EamParams(**{k: float(s.eam[k]) for k in ("A", "c", "d", "c0", "c1", "c2")})
    p.morse = MorseParams(**{k: float(s.morse[k]) for k in ("D", "alpha", "r0", "rc")})
    p.mass = float(s.mass)
    p.dt = float(s.dt)
    p.v_ind = float(s.v_ind)
    p.skin = float(s.skin)
    p.cap = int(cap)
    p.xcap = int(xcap)
    p.tpa = int(tpa)
    p.shadow = int(bool(shadow))
    p.icap = int(icap)
    p.list_tgt = int(list_tgt)
    if getattr(s, "potential", "fs") == "paper":
        p.potential = MD_POT_PAPER
        p.paper = PaperParams(**{k: float(s.paper[k]) for k in PAPER_KEYS})
    return p


def make_replica_desc(s) -> ReplicaDesc:
    d = ReplicaDesc()
    for a in range(3):
        d.lo[a] = float(s.box_lo[a])
        d.len[a] = float(s.box_len[a])
        d.periodic[a] = int(bool(s.periodic[a]))
    d.n = int(s.n)
    d.n_c = int(s.n_c)
    return d


class Simulation:
    """One or more replicas (``inputs.System``) resident on one GPU.

    All replicas share potential parameters, mass, dt, v_ind and skin (taken from the
    first).  ``precision`` is "fp64" or "mixed".
    """

    def __init__(self, systems, precision: str = "fp64", cap: int | None = None, xcap: int = 160,
                 tpa: int = 1, device: str = "cuda:0", shadow: bool | None = None,
                 static_workspace: bool = False, icap: int = 0, list_tgt: int = 0):
        """cap: Cr-Cr list capacity per atom (a multiple of tpa).  shadow: keep the FP32
        cell-local positions for the FP32-mixed passes (default: when precision is mixed).
        icap: two-tier lists (Section 2.6) with this inner-list capacity per atom; the
        Cr-Cr list of capacity cap is then the outer list (give the system the outer skin).
        list_tgt: atoms a list-build work item aims at (0: the library's default).
        static_workspace: bind the library's static device scratch (md_workspace_bind_static)
        instead of a workspace tensor."""
        import torch
        if cap is None:
            cap = 64
        if not torch.cuda.is_available():
            raise MDError("no GPU visible: the MD path runs only on the GPU")
        self.torch = torch
        self.lib = load_library()
        self.systems = list(systems) if isinstance(systems, (list, tuple)) else [systems]
        self.nrep = len(self.systems)
        self.precision = precision
        self.mixed = precision == "mixed"
        self.device = torch.device(device)
        s0 = self.systems[0]
        # the FP32 cell-local shadow serves the FP32-mixed passes only
        self.params = make_params(s0, cap, xcap, tpa,
                                  shadow=(precision == "mixed") if shadow is None else shadow, icap=icap,
                                  list_tgt=list_tgt)
        self.tpa = tpa
        descs = (ReplicaDesc * self.nrep)(*[make_replica_desc(s) for s in self.systems])
        h = C.c_void_p()
        _ok(self.lib.md_system_create(C.cast(descs, C.c_void_p), self.nrep, C.byref(self.params),
                                      C.byref(h)), "md_system_create")
        self.handle = h
        self.ntot = int(self.lib.md_system_atoms(h))
        self.ctot = int(self.lib.md_system_carbons(h))
        self.offsets = [int(self.lib.md_replica_offset(h, r)) for r in range(self.nrep)]
        self.cap, self.xcap, self.icap = cap, xcap, icap
        self._atoms_c = self._lists_c = None
        self.graphs = []
        dev = self.device
        with torch.cuda.device(dev):
            n, nc = self.ntot, self.ctot
            self.q = torch.zeros((n, 4), dtype=torch.float64, device=dev)
            self.v = torch.zeros((n, 3), dtype=torch.float64, device=dev)
            self.f = torch.zeros((n, 3), dtype=torch.float64, device=dev)
            self.fixed = torch.ones(n, dtype=torch.uint8, device=dev)
            self.id = torch.full((n,), -1, dtype=torch.int32, device=dev)
            self.xc = torch.zeros((max(nc, 1), 3), dtype=torch.float64, device=dev)
            self.idx = torch.zeros(cap * n, dtype=torch.int32, device=dev)
            self.cnt = torch.zeros(n, dtype=torch.int32, device=dev)
            self.xidx = torch.zeros((n, xcap), dtype=torch.int32, device=dev)
            self.xcnt = torch.zeros(n, dtype=torch.int32, device=dev)
            self.iidx = torch.zeros(icap * n, dtype=torch.int32, device=dev) if icap else None
            self.icnt = torch.zeros(n, dtype=torch.int32, device=dev) if icap else None
            self.rho = torch.zeros(n, dtype=torch.float64, device=dev)
            self.obs_dev = torch.zeros((self.nrep, MD_NOBS), dtype=torch.float64, device=dev)
            self.static_workspace = static_workspace
            wsb = int(self.lib.md_workspace_bytes(h))
            self.ws = None if static_workspace else torch.empty(wsb + 256, dtype=torch.uint8, device=dev)
            self.load([s.x for s in self.systems], [s.v for s in self.systems])
            self._bind()

    # -- marshalling ---------------------------------------------------------------------
    @property
    def stream(self) -> C.c_void_p:
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _ptr(self, t) -> C.c_void_p:
        return C.c_void_p(t.data_ptr())

    def _atoms(self) -> Atoms:
        if self._atoms_c is None:
            self._atoms_c = Atoms(self.q.data_ptr(), self.v.data_ptr(), self.f.data_ptr(),
                                  self.fixed.data_ptr(), self.id.data_ptr(),
                                  self.xc.data_ptr() if self.ctot else None)
        return self._atoms_c

    def _lists(self) -> Lists:
        if self._lists_c is None:
            self._lists_c = Lists(self.idx.data_ptr(), self.cnt.data_ptr(), self.xidx.data_ptr(),
                                  self.xcnt.data_ptr(), self.iidx.data_ptr() if self.icap else None,
                                  self.icnt.data_ptr() if self.icap else None)
        return self._lists_c

    def _bind(self):
        if self.static_workspace:
            _ok(self.lib.md_workspace_bind_static(self.handle, self.stream), "md_workspace_bind_static")
            return
        base = self.ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.ws_ptr = aligned
        _ok(self.lib.md_workspace_bind(self.handle, C.c_void_p(aligned),
                                       int(self.lib.md_workspace_bytes(self.handle)), self.stream),
            "md_workspace_bind")

    def bind(self):
        """Bind the workspace again (after another system took over the static scratch)."""
        self._bind()

    def load(self, xs: Sequence[np.ndarray], vs: Sequence[np.ndarray]):
        """Copy positions / velocities (and fixed flags, ids, carbons) of every replica in."""
        torch = self.torch
        q = np.zeros((self.ntot, 4))
        v = np.zeros((self.ntot, 3))
        fixed = np.ones(self.ntot, np.uint8)
        ids = np.full(self.ntot, -1, np.int32)
        xc = np.zeros((max(self.ctot, 1), 3))
        c0 = 0
        for r, s in enumerate(self.systems):
            a0 = self.offsets[r]
            q[a0:a0 + s.n, :3] = xs[r]
            v[a0:a0 + s.n] = vs[r]
            fixed[a0:a0 + s.n] = s.fixed
            ids[a0:a0 + s.n] = s.ids
            xc[c0:c0 + s.n_c] = s.xc
            c0 += s.n_c
        self.q.copy_(torch.from_numpy(q))
        self.v.copy_(torch.from_numpy(v))
        self.fixed.copy_(torch.from_numpy(fixed))
        self.id.copy_(torch.from_numpy(ids))
        self.xc.copy_(torch.from_numpy(xc))
        self.f.zero_()

    def close(self):
        for g in getattr(self, "graphs", []):
            self.lib.md_graph_destroy(g)
        self.graphs = []
        if getattr(self, "handle", None):
            self.lib.md_system_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the C ABI, one call each ----------------------------------------------------------
    def md_build_neighbors(self, force: bool = False):
        _ok(self.lib.md_build_neighbors(self.handle, C.byref(self._atoms()), C.byref(self._lists()),
                                        MD_B_FORCE if force else 0, self.stream), "md_build_neighbors")

    def md_eam_forces(self, flags: int, rho: bool = False):
        if self.mixed:
            flags |= MD_F_MIXED
        _ok(self.lib.md_eam_forces(self.handle, C.byref(self._atoms()), C.byref(self._lists()), flags,
                                   self._ptr(self.rho) if rho else None, self.stream), "md_eam_forces")

    def md_morse_forces(self, flags: int = 0):
        if self.mixed:
            flags |= MD_F_MIXED
        _ok(self.lib.md_morse_forces(self.handle, C.byref(self._atoms()), C.byref(self._lists()),
                                     flags, self.stream), "md_morse_forces")

    def md_verlet_step(self, phase: int):
        _ok(self.lib.md_verlet_step(self.handle, phase, C.byref(self._atoms()), self.stream),
            "md_verlet_step")

    def md_energy(self) -> np.ndarray:
        _ok(self.lib.md_energy(self.handle, C.byref(self._atoms()), self._ptr(self.obs_dev),
                               self.stream), "md_energy")
        return self.obs_dev.cpu().numpy().copy()

    def md_check(self) -> dict:
        st = Status()
        _ok(self.lib.md_check(self.handle, C.byref(st), self.stream), "md_check")
        return dict(overflow=st.overflow, xoverflow=st.xoverflow, nonfinite=st.nonfinite,
                    nbuilds=st.nbuilds, sync_timeout=st.sync_timeout, nnear=st.nnear,
                    ioverflow=st.ioverflow)

    def md_set_indenter_velocity(self, v_ind: float):
        _ok(self.lib.md_set_indenter_velocity(self.handle, float(v_ind)), "md_set_indenter_velocity")

    def md_clear_flags(self):
        _ok(self.lib.md_clear_flags(self.handle, self.stream), "md_clear_flags")

    def md_run(self, nsteps: int, energy_every: int = 0, obs=None, events=None, builds=None):
        """Enqueue nsteps whole steps in C.  obs: device float64 tensor with room for
        nsteps // energy_every rows of (nrep, MD_NOBS).  For measurement (md_trace): events, a
        list of MD_TRACE_EVENTS * nsteps events or None entries (objects whose ``cuda_event``
        is a HIP event handle), per step two around the EAM force kernel, two around the Cr-Cr
        list kernel and two around the density kernel; builds, a device int32 tensor of
        (nsteps, nrep) receiving each replica's list-build count after every step."""
        flags = MD_F_MIXED if self.mixed else 0
        tr = None
        if events is not None or builds is not None:
            tr = Trace()
            if events is not None:
                if len(events) != MD_TRACE_EVENTS * nsteps:
                    raise MDError(f"md_run: give {MD_TRACE_EVENTS} timing events (or None) per step")
                handles = [None if e is None else e.cuda_event for e in events]
                if not all(h is None or h for h in handles):
                    raise MDError("md_run: record each timing event once before passing it")
                self._trace_events = (C.c_void_p * len(events))(*handles)
                tr.events = C.cast(self._trace_events, C.c_void_p)
            if builds is not None:
                if builds.dtype != self.torch.int32 or builds.numel() < nsteps * self.nrep or not builds.is_cuda:
                    raise MDError("md_run: builds must be a device int32 tensor of nsteps x nrep")
                tr.builds = builds.data_ptr()
        _ok(self.lib.md_run(self.handle, C.byref(self._atoms()), C.byref(self._lists()), int(nsteps),
                            flags, int(energy_every), self._ptr(obs) if obs is not None else None,
                            C.byref(tr) if tr is not None else None, self.stream), "md_run")

    def md_graph_create(self, nsteps: int, energy_every: int = 0, obs=None):
        """Capture nsteps whole steps into a HIP graph; returns an opaque handle."""
        flags = MD_F_MIXED if self.mixed else 0
        g = C.c_void_p()
        _ok(self.lib.md_graph_create(self.handle, C.byref(self._atoms()), C.byref(self._lists()),
                                     int(nsteps), flags, int(energy_every),
                                     self._ptr(obs) if obs is not None else None, self.stream,
                                     C.byref(g)), "md_graph_create")
        self.graphs.append(g)
        return g

    def md_graph_launch(self, g):
        _ok(self.lib.md_graph_launch(g, self.stream), "md_graph_launch")

    # -- the time step (Table 1 order) ---------------------------------------------------------
    def initial_forces(self, energy: bool = True):
        """List build and forces at t = 0 (before the first step)."""
        self.md_build_neighbors(force=True)
        self.md_eam_forces(MD_F_DENSITY | MD_F_FORCE | MD_F_MORSE | (MD_F_ENERGY if energy else 0))

    def step(self, energy: bool = False):
        """Tasks 2+3, 1, 4 and 5 of one time step (Task 5 fused into the force pass)."""
        self.md_verlet_step(MD_PHASE_KICK_DRIFT)
        self.md_build_neighbors()
        self.md_eam_forces(MD_F_DENSITY | MD_F_FORCE | MD_F_MORSE | MD_F_KICK |
                           (MD_F_ENERGY if energy else 0))

    def step_unfused(self, energy: bool = False):
        """Same step with Task 4c and Task 5 as separate calls."""
        self.md_verlet_step(MD_PHASE_KICK_DRIFT)
        self.md_build_neighbors()
        e = MD_F_ENERGY if energy else 0
        self.md_eam_forces(MD_F_DENSITY | MD_F_FORCE | e)
        self.md_morse_forces(e)
        self.md_verlet_step(MD_PHASE_KICK)

    def run(self, nsteps: int, energy_every: int = 0) -> list:
        """nsteps steps; observables every energy_every steps (list of (step, obs))."""
        out = []
        for k in range(1, nsteps + 1):
            e = energy_every > 0 and k % energy_every == 0
            self.step(energy=e)
            if e:
                out.append((k, self.md_energy()))
        return out

    # -- read back -------------------------------------------------------------------------
    def state(self) -> list:
        """Per replica: dict of x, v, f, dF (F'(rho)), rho (last density pass with rho=True),
        each ordered by atom id, plus the slot of each id."""
        q = self.q.cpu().numpy()
        v = self.v.cpu().numpy()
        f = self.f.cpu().numpy()
        ids = self.id.cpu().numpy()
        rho = self.rho.cpu().numpy()
        out = []
        for r, s in enumerate(self.systems):
            a0 = self.offsets[r]
            sl = slice(a0, a0 + s.n)
            order = np.argsort(ids[sl], kind="stable")
            slots = a0 + order
            out.append(dict(x=q[slots, :3], dF=q[slots, 3], v=v[slots], f=f[slots], rho=rho[slots],
                            ids=ids[slots], slots=slots))
        return out

    def neighbor_sets(self, r: int = 0, cross: bool = False, only=None, inner: bool = False) -> list:
        """Neighbour sets of replica r in id space: [sorted ids of neighbours of id 0, ...]
        (entries for the ids in `only` alone when given, None for the others).  inner: the
        inner list of two-tier lists."""
        ids = self.id.cpu().numpy()
        cnt = (self.xcnt if cross else self.cnt).cpu().numpy()
        s = self.systems[r]
        a0 = self.offsets[r]
        sets = [None] * s.n
        slots = np.arange(a0, a0 + s.n)
        if only is not None:
            want = np.zeros(s.n, bool)
            want[np.asarray(only, dtype=np.int64)] = True
            slots = slots[want[ids[a0:a0 + s.n]]]
        if cross:
            xidx = self.xidx.cpu().numpy()
            c0 = sum(t.n_c for t in self.systems[:r])
            for p in slots:
                sets[ids[p]] = sorted((xidx[p, :cnt[p]] - c0).tolist())
            return sets
        lists = self.list_rows(slots, inner=inner)
        for p, row in zip(slots, lists):
            sets[ids[p]] = sorted(ids[row].tolist())
        return sets

    def list_rows(self, slots=None, inner: bool = False) -> list:
        """Cr-Cr list of every atom slot, or of the given slots (slots of the neighbours, in
        list order); inner: the inner list of two-tier lists."""
        T, n = self.tpa, self.ntot
        idx = (self.iidx if inner else self.idx).cpu().numpy()
        cnt = (self.icnt if inner else self.cnt).cpu().numpy()
        k = np.arange(self.icap if inner else self.cap)
        rows = []
        for p in (range(n) if slots is None else slots):
            kk = k[:cnt[p]]
            rows.append(idx[(kk // T) * n * T + p * T + kk % T] & LIST_IDX_MASK)
        return rows

    def list_counts(self) -> np.ndarray:
        """Cr-Cr list length of every atom slot."""
        return self.cnt.cpu().numpy()
