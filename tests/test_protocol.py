"""The indentation protocol's host-side parts (Section 2.5, Section 4.3): the phase plan from
the geometry, and the contact analysis against the paper's printed worked example and against
an elastic Hertzian contact with a known modulus.  CPU only."""
import json
import os

import numpy as np
import pytest

from paper_1507_07068_amd import inputs as I
from paper_1507_07068_amd import protocol as P

HERE = os.path.dirname(os.path.abspath(__file__))


def test_paper_worked_example():
    g = json.load(open(os.path.join(HERE, "golden", "paper_indentation_analysis.json")))
    i, pr = g["inputs"], g["printed"]
    out = P.contact_analysis(i["max_load_eV_per_A"], i["depth_A"], i["unloading_slope_eV_per_A2"],
                             i["indenter_radius_A"])
    assert abs(out["contact_radius"] - pr["contact_radius_A"]) < 0.05
    assert abs(out["hardness_gpa"] - pr["hardness_GPa"]) < 0.1
    assert abs(out["e_film_gpa"] - pr["film_modulus_GPa"]) < 2.0
    assert abs(out["e_star_gpa"] - 260.0) < 1.0      # the printed 265.7 is inconsistent (see golden)


@pytest.mark.parametrize("e_star_gpa,R", [(150.0, 2000.0), (300.0, 5000.0)])
def test_recovers_hertzian_modulus(e_star_gpa, R):
    """Elastic sphere: P = (4/3) E* sqrt(R) h^(3/2) both ways.  With the Oliver-Pharr contact
    depth h_c = h - 0.75 P / S = h / 2, the analysis returns E* to within the h / (8 R) of the
    paraboloid approximation."""
    e = e_star_gpa / P.EV_PER_A3_GPA
    h = np.concatenate([np.linspace(0.0, 3.0, 301)[1:], np.linspace(3.0, 0.0, 301)[1:]])
    phase = np.array([1] * 300 + [2] * 300)
    load = 4.0 / 3.0 * e * np.sqrt(R) * h ** 1.5
    s = P.unloading_slope(h, load, phase, frac=0.01)
    assert abs(s - 2 * e * np.sqrt(R * 3.0)) < 5e-3 * s   # a line through the top 1% of unloading
    out = P.contact_analysis(load.max(), 3.0, s, R, h_c=3.0 - 0.75 * load.max() / s)
    assert abs(out["contact_depth"] - 1.5) < 1e-2
    assert abs(out["e_star_gpa"] / e_star_gpa - 1.0) < 3.0 / (8 * R) + 6e-3


def test_phase_plan_from_geometry():
    s = I.config(1)      # lowest carbon 3 A above the surface
    pr = P.Protocol()
    assert abs(P.start_depth(s) + 3.0) < 1e-9
    ph = pr.phases(s)
    assert [p[0] for p in ph] == ["relax", "load", "unload"]
    assert ph[0][1] == 10000 and ph[0][2] == 0.0
    assert ph[1][1] == ph[2][1] == 60800 and ph[1][2] == -1e-4 and ph[2][2] == 1e-4
