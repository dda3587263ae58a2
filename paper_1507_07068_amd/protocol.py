"""The full nano-indentation protocol (Section 2.5; Section 4.3, Figure 14) on one GPU through
the C ABI: the film relaxes with the indenter at rest, the indenter moves in at constant speed
until its lowest atom is a given depth below the initial free surface, then it is withdrawn at
the same speed to where it started.  The load (sum of the z forces on the indenter) and the depth
(of the indenter's lowest atom below the initial free surface) are recorded along the way, and
the unloading curve is analysed for the contact modulus and hardness the way Section 4.3 does
(Oliver and Pharr).

Host-side orchestration only: every step runs in md_run; the analysis is post-processing of
the recorded series.
"""
from __future__ import annotations

import dataclasses

import numpy as np

# 1 eV / Angstrom^3 in GPa (1.602176634e-19 J / 1e-30 m^3 = 1.602176634e11 Pa)
EV_PER_A3_GPA = 160.2176634


@dataclasses.dataclass
class Protocol:
    relax_steps: int = 10000      # Section 4.3: 10,000 time steps of relaxation
    speed: float = 1e-4           # Angstrom / fs, in and out (10 m/s)
    depth: float = 3.08           # Angstrom below the initial free surface
    record_every: int = 100       # observables every so many steps

    def phases(self, system) -> list:
        """(name, steps, indenter velocity) of the three phases for `system`: the load phase
        takes the lowest carbon from its start to `depth`, the unload phase back."""
        d0 = start_depth(system)
        n = int(round((self.depth - d0) / (self.speed * system.dt)))
        if n <= 0:
            raise ValueError(f"the indenter starts at depth {d0:.3f} A, at or beyond {self.depth} A")
        return [("relax", self.relax_steps, 0.0), ("load", n, -self.speed), ("unload", n, self.speed)]


def surface_z(system) -> float:
    """Height of the initial free surface: the top atomic plane of the film."""
    return float(system.meta["z_top"])


def start_depth(system) -> float:
    """Depth of the indenter's lowest atom below the initial free surface at zero displacement
    (negative while it is above the surface)."""
    return surface_z(system) - float(system.xc[:, 2].min())


def run(sim, system, proto: Protocol, replica: int = 0) -> dict:
    """Run the protocol on `sim` (a Simulation holding `system` as replica `replica`, forces
    evaluated at the start).  Returns the recorded series: step, phase (0 relax, 1 load,
    2 unload), depth and load (Angstrom, eV/Angstrom), total energy (eV), and the observables."""
    import torch

    from . import md
    rows, phase_of, steps_of = [], [], []
    step = 0
    nrep = sim.nrep
    for k, (name, n, v) in enumerate(proto.phases(system)):
        sim.md_set_indenter_velocity(v)
        ee = proto.record_every
        nobs = n // ee
        obs = torch.zeros((max(nobs, 1), nrep, md.MD_NOBS), dtype=torch.float64, device=sim.device)
        sim.md_run(n, energy_every=ee, obs=obs)
        o = obs.cpu().numpy()[:nobs, replica]
        rows.append(o)
        phase_of += [k] * nobs
        steps_of += list(step + ee * np.arange(1, nobs + 1))
        step += n
    sim.md_set_indenter_velocity(system.v_ind)
    o = np.concatenate(rows, axis=0)
    depth = start_depth(system) - o[:, md.MD_IND_Z]
    return dict(step=np.array(steps_of), phase=np.array(phase_of), depth=depth, load=o[:, md.MD_F_IND_X + 2],
                e_tot=o[:, 0:4].sum(axis=1), obs=o)


def unloading_slope(depth, load, phase, frac: float = 0.25) -> float:
    """dP/dh at the start of unloading: least-squares slope of load against depth over the
    unloading records whose depth lies within `frac` of the unloading depth range from its
    start."""
    d, p = depth[phase == 2], load[phase == 2]
    if d.size < 3:
        raise ValueError("too few unloading records")
    top = d.max()
    sel = d >= top - frac * (top - d.min())
    if sel.sum() < 3:
        sel = np.argsort(-d)[:3]
    return float(np.polyfit(d[sel], p[sel], 1)[0])


def contact_analysis(p_max: float, h_max: float, slope: float, radius: float, h_c: float | None = None,
                     nu: float = 0.21, e_ind: float = 1141.0, nu_ind: float = 0.07) -> dict:
    """Section 4.3's analysis of an indentation by a sphere of `radius` (Oliver and Pharr):
    contact radius a = sqrt(2 R h_c - h_c^2) at contact depth h_c (the maximum depth, as the
    paper takes it, unless given), projected area A = pi a^2, contact modulus
    E* = (sqrt(pi) / 2) S / sqrt(A), hardness H = P_max / A, and the film's Young's modulus from
    1/E* = (1 - nu^2)/E + (1 - nu_ind^2)/E_ind (the paper prints neither Poisson ratio nor the
    indenter's modulus: nu = 0.21 for Cr and diamond's 1141 GPa, 0.07 are assumed).
    Lengths in Angstrom, loads in eV/Angstrom; moduli in GPa."""
    hc = h_max if h_c is None else h_c
    a = float(np.sqrt(2.0 * radius * hc - hc * hc))
    area = np.pi * a * a
    e_star = np.sqrt(np.pi) / 2.0 * slope / np.sqrt(area) * EV_PER_A3_GPA
    hard = p_max / area * EV_PER_A3_GPA
    e_film = (1.0 - nu * nu) / (1.0 / e_star - (1.0 - nu_ind * nu_ind) / e_ind)
    return dict(contact_radius=a, area=float(area), e_star_gpa=float(e_star), hardness_gpa=float(hard),
                e_film_gpa=float(e_film), contact_depth=hc)


def analyse(rec: dict, radius: float) -> dict:
    """Maximum load and depth, initial unloading slope and the contact analysis of a record."""
    i = int(np.argmax(rec["depth"]))
    p_max, h_max = float(rec["load"][i]), float(rec["depth"][i])
    s = unloading_slope(rec["depth"], rec["load"], rec["phase"])
    out = dict(p_max=p_max, h_max=h_max, unloading_slope=s)
    if s > 0 and p_max > 0:
        out.update(contact_analysis(p_max, h_max, s, radius))
    return out
