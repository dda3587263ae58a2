"""Seeded synthetic workloads for the short-range MD step.

Builds BCC Cr films, rigid diamond-lattice carbon hemispheres and Maxwell-Boltzmann
velocities (the set-up of the paper's Section 2.5, with the synthetic potential and
film sizes used here).  This module places atoms and draws random numbers only: it
holds no force, density, energy or integrator arithmetic, so that the CPU oracle and
the HIP path can both take their inputs from it without sharing any of the method.

Units: eV, Angstrom, fs, atomic mass unit (u).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

# Lattice and mass constants of the workloads.
A_CR = 2.885          # BCC Cr lattice constant (Angstrom)
A_C = 3.567           # diamond lattice constant (Angstrom)
M_CR = 52.0           # Cr mass (u)
KB_EV = 8.617333262e-5  # Boltzmann constant (eV/K), CODATA 2018
# (eV/u) -> (Angstrom/fs)^2, used only to draw thermal velocities:
# 1 eV / 1 u = 1.602176634e-19 J / 1.66053906660e-27 kg, and 1 m^2/s^2 = 1e-10 A^2/fs^2.
EV_PER_U_TO_A2_FS2 = 1.602176634e-19 / 1.66053906660e-27 * 1e-10

# Synthetic Finnis-Sinclair-form EAM for Cr-Cr and shifted Morse for Cr-C.
EAM = dict(A=1.45, c=3.9, d=3.6, c0=29.14, c1=-23.37, c2=4.77)
MORSE = dict(D=0.8, alpha=1.7, r0=2.0, rc=5.0)
# The paper's own EAM form (Appendix, Eqs. A1-A4) with synthetic parameter values (the paper
# prints none): r_e, r* = 3 r_e and the pair cutoff x < d are the paper's; rho_e and P_e are
# rho and P of the perfect BCC lattice (a = 2.885 A, f cut at r*), so that F' and M' vanish
# there; the Pasianot coefficients give a repulsive core, a shallow well and zero pair pressure
# on that lattice.  Energies in eV, lengths in Angstrom.
PAPER_EAM = dict(Fo=3.0, n=0.5, rho_e=21.69, alpha=0.05, P_e=29.32, fe=1.0, re=2.754, beta=6.0,
                 a0=69.50, a1=-195.07, a2=178.68, a3=-53.50, d=1.65, rc=8.262)
SKIN = 0.3
DT = 1.0               # fs
V_IND = -0.001         # indenter velocity along z (Angstrom/fs): -0.1 A per 100 steps
TEMPERATURE = 300.0    # K

# Diamond-cubic basis (fractions of the cubic cell): FCC sites plus the (1/4,1/4,1/4) copy.
_FCC = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
_DIAMOND = np.concatenate([_FCC, _FCC + 0.25])


@dataclass
class System:
    """One MD system: Cr film (+ optional rigid C indenter) in a box.

    Arrays are NumPy, positions in Angstrom.  ``box_len`` is the periodic length on
    periodic axes and the extent of the cell grid on open axes (atoms outside it are
    still handled; the extent only shapes the binning).
    """
    name: str
    x: np.ndarray            # (n, 3) float64 Cr positions
    v: np.ndarray            # (n, 3) float64 Cr velocities (A/fs)
    fixed: np.ndarray        # (n,) uint8, 1 = held fixed
    ids: np.ndarray          # (n,) int32 global ids 0..n-1
    xc: np.ndarray           # (n_c, 3) float64 carbon positions at indenter displacement 0
    box_lo: np.ndarray       # (3,)
    box_len: np.ndarray      # (3,)
    periodic: np.ndarray     # (3,) bool
    steps: int = 100
    dt: float = DT
    v_ind: float = 0.0       # indenter velocity along z (A/fs)
    mass: float = M_CR
    skin: float = SKIN
    eam: dict = field(default_factory=lambda: dict(EAM))
    morse: dict = field(default_factory=lambda: dict(MORSE))
    precision: str = "fp64"
    potential: str = "fs"    # "fs": the synthetic potential `eam`; "paper": the paper's form `paper`
    paper: dict = field(default_factory=lambda: dict(PAPER_EAM))
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_c(self) -> int:
        return int(self.xc.shape[0])

    @property
    def cutoff(self) -> float:
        """Largest Cr-Cr cutoff of the potential."""
        if self.potential == "paper":
            return max(self.paper["rc"], self.paper["d"] * self.paper["re"])
        return self.eam["c"]

    @property
    def r_list(self) -> float:
        return self.cutoff + self.skin

    @property
    def r_list_cross(self) -> float:
        return self.morse["rc"] + self.skin

    def copy(self) -> "System":
        return dataclasses.replace(
            self, x=self.x.copy(), v=self.v.copy(), fixed=self.fixed.copy(),
            ids=self.ids.copy(), xc=self.xc.copy(), box_lo=self.box_lo.copy(),
            box_len=self.box_len.copy(), periodic=self.periodic.copy(),
            eam=dict(self.eam), morse=dict(self.morse), paper=dict(self.paper), meta=dict(self.meta))


# ----------------------------------------------------------------------------------------
# Lattices
# ----------------------------------------------------------------------------------------
def bcc_sites(nx: int, ny: int, nz: int, a: float = A_CR) -> np.ndarray:
    """Sites (i,j,k)a and (i+1/2,j+1/2,k+1/2)a for i<nx, j<ny, k<nz (periodic block).

    Ordered by k, then j, then i, then the two basis sites, so that storage order is
    already spatially coherent.  2*nx*ny*nz sites.
    """
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    base = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    pts = np.empty((base.shape[0], 2, 3))
    pts[:, 0] = base
    pts[:, 1] = base + 0.5
    return pts.reshape(-1, 3) * a


def paper_open_block(nx: int, ny: int, nz: int, a: float = A_CR) -> np.ndarray:
    """The paper's open BCC block (Section 2.5): every cube corner of an nx x ny x nz
    block of unit cells plus every body centre, (nx+1)(ny+1)(nz+1) + nx*ny*nz sites."""
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    corners = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    centres = bcc_sites(nx, ny, nz, 1.0).reshape(-1, 2, 3)[:, 1]
    return np.concatenate([corners, centres]) * a


def diamond_hemisphere(radius: float, a: float = A_C) -> np.ndarray:
    """Diamond-cubic sites p (cubic axes = box axes, a lattice site at the origin)
    with |p| <= radius and p_z <= 0: the lower half of a sphere, as offsets from its centre."""
    m = int(np.ceil(radius / a)) + 1
    g = np.arange(-m, m + 1)
    k, j, i = np.meshgrid(g, g, g, indexing="ij")
    cells = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    p = (cells[:, None, :] + _DIAMOND[None, :, :]).reshape(-1, 3) * a
    r2 = np.einsum("ij,ij->i", p, p)
    keep = (r2 <= radius * radius * (1.0 + 1e-12)) & (p[:, 2] <= 1e-12)
    p = p[keep]
    # deterministic order: by z, then y, then x
    order = np.lexsort((p[:, 0], p[:, 1], p[:, 2]))
    return np.ascontiguousarray(p[order])


def thermal_velocities(rng: np.random.Generator, mobile: np.ndarray, temperature: float,
                       mass: float) -> np.ndarray:
    """Per-component N(0, kB*T/m) for mobile atoms, minus the centre-of-mass velocity of the
    mobile set (Section 2.5: Gaussian sampling, then the COM velocity is removed)."""
    n = mobile.shape[0]
    v = np.zeros((n, 3))
    nm = int(mobile.sum())
    if nm == 0 or temperature <= 0.0:
        return v
    sigma = np.sqrt(KB_EV * temperature / mass * EV_PER_U_TO_A2_FS2)
    vm = rng.normal(0.0, sigma, size=(nm, 3))
    vm -= vm.mean(axis=0)
    v[mobile.astype(bool)] = vm
    return v


# ----------------------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------------------
def bulk(n_cells: int = 10, seed: int = 0, noise: float = 0.02, temperature: float = TEMPERATURE,
         steps: int = 100, a: float = A_CR, name: str = "bulk") -> System:
    """Fully periodic BCC block, lattice + N(0, noise^2) per component, no indenter."""
    x = bcc_sites(n_cells, n_cells, n_cells, a)
    n = x.shape[0]
    rng = np.random.default_rng(seed)
    if noise > 0:
        x = x + rng.normal(0.0, noise, size=x.shape)
    fixed = np.zeros(n, np.uint8)
    v = thermal_velocities(rng, 1 - fixed, temperature, M_CR)
    L = n_cells * a
    return System(name=name, x=x, v=v, fixed=fixed, ids=np.arange(n, dtype=np.int32),
                  xc=np.zeros((0, 3)), box_lo=np.zeros(3), box_len=np.full(3, L),
                  periodic=np.array([True, True, True]), steps=steps, v_ind=0.0,
                  meta=dict(n_cells=n_cells, seed=seed, noise=noise))


def film(nx: int, ny: int, nz: int, radius: float, gap: float, seed: int, *,
         noise: float = 0.0, temperature: float = TEMPERATURE, steps: int = 2000,
         preindent: float | None = None, v_ind: float = V_IND, a: float = A_CR,
         name: str = "film", rng: np.random.Generator | None = None) -> System:
    """Cr film periodic in x,y with a free top surface, bottom two atomic planes fixed,
    and a rigid diamond carbon hemisphere above the film centre.

    ``gap``: height of the lowest carbon atom above the top Cr plane.  ``preindent``:
    if given, the lowest carbon atom is placed that far *below* the top plane instead,
    and Cr atoms within radius + r0 of the sphere centre are removed.
    ``radius <= 0`` means no indenter.
    """
    x = bcc_sites(nx, ny, nz, a)
    Lx, Ly = nx * a, ny * a
    z_top = (nz - 0.5) * a
    fixed = (x[:, 2] < 0.75 * a).astype(np.uint8)          # planes z=0 and z=a/2
    if radius > 0:
        p = diamond_hemisphere(radius)
        pz_min = p[:, 2].min()
        z_low = z_top - preindent if preindent is not None else z_top + gap
        centre = np.array([0.5 * Lx, 0.5 * Ly, z_low - pz_min])
        xc = p + centre
        if preindent is not None:
            d = x - centre
            d[:, 0] -= Lx * np.round(d[:, 0] / Lx)
            d[:, 1] -= Ly * np.round(d[:, 1] / Ly)
            keep = np.einsum("ij,ij->i", d, d) >= (radius + MORSE["r0"]) ** 2
            x, fixed = x[keep], fixed[keep]
    else:
        xc = np.zeros((0, 3))
        centre = np.array([0.5 * Lx, 0.5 * Ly, z_top])
    n = x.shape[0]
    rng = np.random.default_rng(seed) if rng is None else rng
    if noise > 0:
        x = x + rng.normal(0.0, noise, size=x.shape) * (1 - fixed)[:, None]
    v = thermal_velocities(rng, 1 - fixed, temperature, M_CR)
    # Cell-grid extent along the open z axis: below the film to above the indenter.
    z_hi = max(z_top, xc[:, 2].max() if xc.shape[0] else z_top)
    lo = np.array([0.0, 0.0, -2.0 * a])
    length = np.array([Lx, Ly, z_hi + 2.0 * a - lo[2]])
    return System(name=name, x=x, v=v, fixed=fixed, ids=np.arange(n, dtype=np.int32),
                  xc=np.ascontiguousarray(xc), box_lo=lo, box_len=length,
                  periodic=np.array([True, True, False]), steps=steps,
                  v_ind=v_ind if xc.shape[0] else 0.0,
                  meta=dict(nx=nx, ny=ny, nz=nz, radius=radius, gap=gap, seed=seed,
                            preindent=preindent, z_top=z_top, centre=centre.tolist()))


def replica_draws(r: int) -> dict:
    """Sizes of ensemble replica r: nx, ny ~ U{10..30}, nz ~ U{8..20}, radius ~ U[5, 20] A,
    gap ~ U[0, 5] A, drawn from default_rng(3000 + r) before the replica's own state."""
    rng = np.random.default_rng(3000 + r)
    nx = int(rng.integers(10, 31))
    ny = int(rng.integers(10, 31))
    nz = int(rng.integers(8, 21))
    radius = float(rng.uniform(5.0, 20.0))
    gap = float(rng.uniform(0.0, 5.0))
    return dict(nx=nx, ny=ny, nz=nz, radius=radius, gap=gap, rng=rng)


def replica(r: int, steps: int = 1000) -> System:
    d = replica_draws(r)
    rng = d.pop("rng")
    s = film(d["nx"], d["ny"], d["nz"], d["radius"], d["gap"], 3000 + r, steps=steps,
             name=f"replica{r}", rng=rng)
    s.precision = "mixed"
    return s


# Section 2.6's two-tier lists: the outer list reaches 1.7 r*, a skin of 0.7 r* beyond the
# inner list's radius r* (the paper's cutoff).
OUTER_SKIN_FACTOR = 0.7


def two_tier(s: System) -> System:
    """`s` with the paper's form and the two-tier lists' outer skin (0.7 r*)."""
    s.potential = "paper"
    s.skin = OUTER_SKIN_FACTOR * s.cutoff
    return s


def config(index: int) -> System | list:
    """The five benchmark workloads (c0..c4).  c3 returns a list of 64 replicas."""
    if index == 0:
        return bulk(10, seed=0, noise=0.02, steps=100, name="c0_bulk_2k_fp64")
    if index == 1:
        return film(60, 60, 30, 20.0, 3.0, 1, steps=2000, name="c1_film_216k_fp64")
    if index == 2:
        s = film(100, 100, 50, 30.0, 3.0, 2, steps=2000, name="c2_film_1m")
        s.precision = "mixed"
        return s
    if index == 3:
        return [replica(r) for r in range(64)]
    if index == 4:
        s = film(200, 200, 100, 50.0, 0.0, 4, steps=500, preindent=20.0,
                 name="c4_film_8m")
        s.precision = "mixed"
        return s
    raise ValueError(f"no workload {index}")


def small_film(nx=8, ny=8, nz=6, radius=6.0, gap=1.0, seed=11, noise=0.02, steps=50) -> System:
    """A film small enough for all-pairs oracle trajectories, with an indenter."""
    return film(nx, ny, nz, radius, gap, seed, noise=noise, steps=steps, name="small_film")


def random_gas(n: int, box: float, seed: int, periodic=(True, True, True), lengths=None) -> System:
    """Uniform random atoms in a cube of edge `box`, or a box of the given `lengths`
    (list-build edge cases: irregular counts, close pairs, atoms slightly outside the box on
    periodic axes, long and crowded cell rows)."""
    rng = np.random.default_rng(seed)
    L = np.full(3, float(box)) if lengths is None else np.asarray(lengths, float)
    x = rng.uniform(-0.1 * L, 1.1 * L, size=(n, 3))
    per = np.array(periodic, bool)
    for ax in range(3):
        if not per[ax]:
            x[:, ax] = np.clip(x[:, ax], 0.0, L[ax])
    v = np.zeros((n, 3))
    return System(name="gas", x=x, v=v, fixed=np.zeros(n, np.uint8),
                  ids=np.arange(n, dtype=np.int32), xc=np.zeros((0, 3)),
                  box_lo=np.zeros(3), box_len=L, periodic=per, steps=0)
