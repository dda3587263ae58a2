"""Pins of the oracle's evaluation of the paper's own EAM form (Appendix, Eqs. A1-A4) against
facts that do not come from the oracle: the paper's printed force terms T1-T4 (Eqs. A6-A9),
closed-form lattice sums and the dimer, finite differences of the energy, conservation laws,
and the strain derivative of the energy.  CPU only."""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_1507_07068_amd import inputs as I

PP = I.PAPER_EAM


def paper_bulk(n_cells, seed=0, noise=0.0, a=I.A_CR, temperature=0.0):
    s = I.bulk(n_cells, seed=seed, noise=noise, temperature=temperature, a=a, name="paper_bulk")
    s.potential = "paper"
    return s


def f_cf(r):
    return np.where(r < PP["rc"], PP["fe"] * (PP["re"] / r) ** PP["beta"], 0.0)


def phi_cf(r):
    x = r / PP["re"]
    return np.where(x < PP["d"], (x - PP["d"]) ** 2 * (PP["a3"] * x ** 3 + PP["a2"] * x ** 2 + PP["a1"] * x
                                                      + PP["a0"]), 0.0)


def F_cf(rho):
    t = rho / PP["rho_e"]
    return -PP["Fo"] * (1 - np.log(t ** PP["n"])) * t ** PP["n"]


def M_cf(P):
    u = P / PP["P_e"] - 1
    return PP["alpha"] * u * u * np.exp(-u * u)


def shells(a, rmax):
    """(count, distance) of the BCC shells within rmax: sites are (a/2)(X, Y, Z) with X, Y, Z
    all even or all odd, so a shell is an integer N = X^2 + Y^2 + Z^2 at distance (a/2) sqrt(N)."""
    m = int(2 * rmax / a) + 2
    count = {}
    for X, Y, Z in itertools.product(range(-m, m + 1), repeat=3):
        if (X % 2 == Y % 2 == Z % 2) and (X, Y, Z) != (0, 0, 0):
            N = X * X + Y * Y + Z * Z
            if 0.5 * a * np.sqrt(N) < rmax:
                count[N] = count.get(N, 0) + 1
    return [(c, 0.5 * a * np.sqrt(N)) for N, c in sorted(count.items())]


# --------------------------------------------------------------------------------------
# The paper's printed force terms (Eqs. A6-A9)
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("r", [2.3, 2.5, 2.9, 3.6, 4.2, 5.5, 7.9])
@pytest.mark.parametrize("rho", [4.0, 18.0, 21.69, 30.0])
def test_T1_embedding_term(r, rho):
    """A6: T1 = -(n^2 Fo beta fe / (r rho)) (re/r)^beta (rho/rho_e)^n ln(rho/rho_e) is the
    derivative of atom i's embedding energy with respect to r_ij, F'(rho_i) f'(r)."""
    s = paper_bulk(6)
    v = O.paper_values(s, r, rho=rho)
    n, Fo, beta, fe, re, rho_e = PP["n"], PP["Fo"], PP["beta"], PP["fe"], PP["re"], PP["rho_e"]
    T1 = -(n * n * Fo * beta * fe / (r * rho)) * (re / r) ** beta * (rho / rho_e) ** n * np.log(rho / rho_e)
    assert abs(v["dF"] * v["df"] - T1) <= 1e-13 * max(abs(T1), 1e-12)


@pytest.mark.parametrize("r", [2.3, 2.5, 2.9, 3.6, 5.5, 7.9])
@pytest.mark.parametrize("P", [5.0, 25.0, 29.32, 40.0, 60.0])
def test_T2_cauchy_term(r, P):
    """A7: T2 = -(4 alpha beta fe^2 P / (P_e^2 r)) (re/r)^(2 beta) (2 - P/P_e) (P/P_e - 1)
    exp(-(P/P_e - 1)^2) is M'(P_i) d(f^2)/dr."""
    s = paper_bulk(6)
    v = O.paper_values(s, r, P=P)
    al, beta, fe, re, Pe = PP["alpha"], PP["beta"], PP["fe"], PP["re"], PP["P_e"]
    T2 = (-(4 * al * beta * fe * fe * P / (Pe * Pe * r)) * (re / r) ** (2 * beta) * (2 - P / Pe) * (P / Pe - 1)
          * np.exp(-(P / Pe - 1) ** 2))
    assert abs(v["dM"] * 2 * v["f"] * v["df"] - T2) <= 1e-13 * max(abs(T2), 1e-15)


@pytest.mark.parametrize("r", [2.0, 2.4, 2.7, 3.1, 3.8, 4.4, 4.54])
def test_T3_pair_term(r):
    """A8: T3 = -((x - d)/re) (5 a3 x^3 + (4 a2 - 3 a3 d) x^2 + (3 a1 - 2 a2 d) x + (2 a0 - a1 d))
    is minus the derivative of the Pasianot pair Phi(x), x = r/re."""
    s = paper_bulk(6)
    v = O.paper_values(s, r)
    x, d, re = r / PP["re"], PP["d"], PP["re"]
    a0, a1, a2, a3 = PP["a0"], PP["a1"], PP["a2"], PP["a3"]
    T3 = -((x - d) / re) * (5 * a3 * x ** 3 + (4 * a2 - 3 * a3 * d) * x ** 2 + (3 * a1 - 2 * a2 * d) * x
                            + (2 * a0 - a1 * d))
    assert abs(v["dphi"] + T3) <= 1e-12 * max(abs(T3), 1.0)
    assert abs(v["phi"] - phi_cf(r)) <= 1e-13 * max(abs(v["phi"]), 1.0)


@pytest.mark.parametrize("y", [1.6, 2.0, 2.6, 3.5, 4.9])
def test_T4_morse_term(y):
    """A9 with alpha_x = 2 alpha r0, y_eq = r0, D_o = D (the Morse form used here):
    T4 = (D_o alpha_x / y_eq) [exp(-alpha_x (y/y_eq - 1)) - exp(-(alpha_x/2) (y/y_eq - 1))]
    is minus the derivative of the Cr-C pair."""
    s = paper_bulk(6)
    pv = O.potential_values(s, y)
    D, al, r0 = I.MORSE["D"], I.MORSE["alpha"], I.MORSE["r0"]
    ax, yeq = 2 * al * r0, r0
    T4 = (D * ax / yeq) * (np.exp(-ax * (y / yeq - 1)) - np.exp(-(ax / 2) * (y / yeq - 1)))
    assert abs(pv["dphiM"] + T4) <= 1e-13 * max(abs(T4), 1.0)


# --------------------------------------------------------------------------------------
# Closed forms
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("a", [2.80, 2.885, 2.95])
def test_perfect_lattice_closed_form(a):
    """Periodic BCC: rho and P are the shell sums of f and f^2 within r*, the energy per atom
    F(rho) + M(P) + 1/2 sum Phi (A1), and the forces vanish by inversion symmetry."""
    s = paper_bulk(7, a=a)
    r = O.evaluate(s)
    sh = shells(a, PP["rc"] + 1.0)
    rho = sum(c * f_cf(d) for c, d in sh)
    P = sum(c * f_cf(d) ** 2 for c, d in sh)
    e = F_cf(rho) + M_cf(P) + 0.5 * sum(c * phi_cf(d) for c, d in sh)
    assert np.allclose(r["rho"], rho, rtol=1e-12, atol=0)
    assert np.allclose(r["P"], P, rtol=1e-12, atol=0)
    assert abs((r["obs"][0] + r["obs"][1]) / s.n - e) < 1e-11 * max(1.0, abs(e))
    assert np.abs(r["f"]).max() < 1e-10
    if a == 2.885:   # rho_e and P_e are these lattice sums, rounded: F' and M' nearly vanish
        assert abs(rho - PP["rho_e"]) < 5e-3 and abs(P - PP["P_e"]) < 5e-3
        assert sum(c for c, d in sh if d < PP["rc"]) == 180


@pytest.mark.parametrize("r", [2.2, 2.6, 3.3, 4.3, 6.0])
def test_dimer_energy_and_force(r):
    """Two atoms: rho = f(r), P = f(r)^2 on each, E = 2 F(f) + 2 M(f^2) + Phi(r); the force on
    each is minus dE/dr along the bond (derivative of the closed form by differences)."""
    from tests.test_oracle import two_atoms
    s = two_atoms(r, box=60.0)
    s.potential = "paper"
    ev = O.evaluate(s)

    def E(rr):
        fr = f_cf(rr)
        return 2 * F_cf(fr) + 2 * M_cf(fr * fr) + phi_cf(rr)
    assert abs(ev["obs"][0] + ev["obs"][1] - E(r)) < 1e-12 * max(1.0, abs(E(r)))
    h = 1e-6
    dEdr = (E(r + h) - E(r - h)) / (2 * h)
    u = (s.x[1] - s.x[0]) / r
    assert np.allclose(ev["f"][1], -dEdr * u, rtol=1e-7, atol=1e-9)
    assert np.allclose(ev["f"][0], dEdr * u, rtol=1e-7, atol=1e-9)


# --------------------------------------------------------------------------------------
# Forces are minus the gradient of the energy; invariants
# --------------------------------------------------------------------------------------
def _total_E(s, x=None):
    obs = O.evaluate(s, x)["obs"]
    return obs[0] + obs[1] + obs[2]


def test_force_is_minus_energy_gradient():
    """Central differences on a noisy bulk (no pair within h of a cutoff in this draw)."""
    s = paper_bulk(6, seed=3, noise=0.08)
    ev = O.evaluate(s)
    fscale = np.sqrt(np.mean(np.sum(ev["f"] ** 2, axis=1)))
    assert fscale > 0.05
    h = 1e-5
    for i in (0, 31, 200, 401):
        for a in range(3):
            xp = s.x.copy(); xp[i, a] += h
            xm = s.x.copy(); xm[i, a] -= h
            g = (_total_E(s, xp) - _total_E(s, xm)) / (2 * h)
            assert abs(-g - ev["f"][i, a]) < 2e-7 * fscale + 1e-9, (i, a, -g, ev["f"][i, a])


def test_zero_net_force_and_translation():
    s = paper_bulk(6, seed=4, noise=0.1)
    ev = O.evaluate(s)
    assert np.abs(ev["f"].sum(0)).max() < 1e-11 * s.n
    ev2 = O.evaluate(s, s.x + np.array([0.3, -1.2, 2.9]))
    assert np.allclose(ev2["f"], ev["f"], rtol=0, atol=1e-10)


def test_virial_matches_strain_derivative():
    s = paper_bulk(6, seed=1, noise=0.05)
    ev = O.evaluate(s)
    tr = ev["obs"][4] + ev["obs"][5] + ev["obs"][6]
    eps = 1e-6

    def e_scaled(k):
        t = s.copy()
        t.x = s.x * k
        t.box_len = s.box_len * k
        return _total_E(t)
    dE = (e_scaled(1 + eps) - e_scaled(1 - eps)) / (2 * eps)
    assert abs(tr + dE) < 1e-6 * abs(dE)


def test_film_with_indenter_balance_and_list_mode():
    """On a film with the indenter: the EAM forces sum to zero, the Cr total balances the load,
    and Verlet-list trajectories equal all-pairs ones bitwise."""
    s = I.small_film(nx=7, ny=7, nz=5, radius=6.0, gap=-0.5, seed=27, noise=0.03)
    s.potential = "paper"
    ev = O.evaluate(s)
    assert np.abs((ev["f"] - ev["fm"]).sum(0)).max() < 1e-11 * s.n
    assert np.allclose(ev["f"].sum(0), -ev["obs"][10:13], atol=1e-11)
    a = O.md_run(s, 12, use_lists=False)
    b = O.md_run(s, 12, use_lists=True, cap=256)
    for k in ("x", "v", "f", "obs"):
        assert np.array_equal(a[k], b[k]), k


def test_sampled_forces_equal_whole_system():
    s = I.small_film(nx=7, ny=7, nz=4, radius=6.0, gap=-0.5, seed=33, noise=0.04)
    s.potential = "paper"
    ev = O.evaluate(s)
    smp = np.array([0, 9, s.n // 2, s.n - 1] + list(np.nonzero(np.abs(ev["fm"]).sum(1))[0][:3]))
    f, rho, dF = O.sample_forces_paper(s, smp)
    assert np.allclose(f, ev["f"][smp], rtol=0, atol=1e-11)
    assert np.allclose(rho, ev["rho"][smp], rtol=1e-14)
    assert np.allclose(dF, ev["dF"][smp], rtol=1e-13)
