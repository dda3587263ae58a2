"""Plant plausible mistakes in copies of the oracle (on the CPU) and check that the pins
in test_oracle.py catch every one.  Shows the pins are sensitive to a dropped term, a
wrong sign, a wrong factor and a transposed operand."""
import os
import subprocess

import pytest

import oracle as O
import tests.test_oracle as T
import tests.test_oracle_paper as TP

SRC = os.path.join(os.path.dirname(O.__file__), "md_oracle.c")

MUTATIONS = [
    # (name, original text, replacement, pin that must fail)
    ("drop F'(rho_j) term of Eq. 1", "g += (dF[i] + dF[j]) * dens_df(p, r);",
     "g += (dF[i] + dF[i]) * dens_df(p, r);", T.test_force_is_minus_energy_gradient_bulk),
    ("wrong sign of the minimum-image shift", "            d -= b->len[a];\n        else if (d < -half)",
     "            d += b->len[a];\n        else if (d < -half)",
     lambda: T.test_neighbor_sets_vs_kdtree(300, 12.0, (1, 1, 1))),
    ("pair energy not halved", "e += 0.5 * pair_phi(p, r);", "e += pair_phi(p, r);",
     T.test_perfect_bcc_lattice_closed_form),
    ("Verlet drift without the 1/2", "v[3 * i + a] * dt + 0.5 * ai * dt * dt;",
     "v[3 * i + a] * dt + ai * dt * dt;", T.test_morse_oscillator_matches_ode_solution),
    ("Morse force direction transposed", "for (int a = 0; a < 3; ++a) fi[a] += -g * (-s[a]) / r;\n                e += morse_phi",
     "for (int a = 0; a < 3; ++a) fi[a] += -g * (s[a]) / r;\n                e += morse_phi",
     T.test_force_is_minus_energy_gradient_film_with_indenter),
    ("density cutoff uses the pair cutoff", "if (r < p->d) acc += dens_f(p, r);\n        });",
     "if (r < p->c) acc += dens_f(p, r);\n        });",
     T.test_lattice_energy_vs_lattice_constant_is_smooth_and_consistent),
    ("rebuild test at full skin", "double lim = 0.5 * P->skin;", "double lim = P->skin;",
     T.test_half_skin_rule_catches_approaching_pair),
    ("carbon position ignores the indenter displacement", "p[2] = xc[3 * k + 2] + ind_z;",
     "p[2] = xc[3 * k + 2];", lambda: T.test_morse_pair_at_indenter_displacement(2.0, 0.75)),
    ("indenter displacement with the wrong sign", "p[2] = xc[3 * k + 2] + ind_z;",
     "p[2] = xc[3 * k + 2] - ind_z;", lambda: T.test_morse_pair_at_indenter_displacement(3.1, -1.3)),
    ("rebuild rule without the indenter term", "if (fabs(S->ind_z - S->ind_z_ref) > lim) return 1;",
     "if (0 && fabs(S->ind_z - S->ind_z_ref) > lim) return 1;", T.test_rebuild_rule_indenter_term),
    ("indenter reference not reset at a build", "S->ind_z_ref = S->ind_z;\n    S->nbuilds++;",
     "S->nbuilds++;", T.test_rebuild_rule_indenter_term),
    # the paper's EAM form
    ("paper form: M'(P_j) term dropped", "(dM[i] + dM[j]) * 2.0 * fr * dfr", "(dM[i] + dM[i]) * 2.0 * fr * dfr",
     TP.test_force_is_minus_energy_gradient),
    ("paper form: F'(rho_j) term dropped", "(dF[i] + dF[j]) * dfr", "(dF[i] + dF[i]) * dfr",
     TP.test_force_is_minus_energy_gradient),
    ("paper form: f' with the wrong power", "pow(p->re / r, p->beta - 1.0)", "pow(p->re / r, p->beta)",
     lambda: TP.test_T1_embedding_term(2.9, 18.0)),
    ("paper form: P sums f, not f^2", "                accp += fr * fr;", "                accp += fr;",
     lambda: TP.test_perfect_lattice_closed_form(2.80)),
    ("paper form: sign of M' cubic term", "exp(-u * u) * (-2.0 * u)", "exp(-u * u) * (2.0 * u)",
     lambda: TP.test_T2_cauchy_term(2.5, 40.0)),
    ("paper form: Phi' without dx/dr", "u * u * dpoly) / p->re;", "u * u * dpoly);",
     lambda: TP.test_T3_pair_term(3.1)),
    ("paper form: M(P) left out of the energy", "            sum_add(&e_emb, paper_M(&P->paper, S->Pd[i]));\n",
     "", lambda: TP.test_perfect_lattice_closed_form(2.80)),
]


@pytest.mark.parametrize("name,old,new,pin", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_planted_mistake(tmp_path, name, old, new, pin):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique: {name}"
    mutated = tmp_path / "md_oracle_mut.c"
    mutated.write_text(src.replace(old, new))
    so = tmp_path / "liborc_mut.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-o", str(so), str(mutated), "-lm"], check=True)
    pin()  # the pin passes on the real oracle
    with O.use_library(str(so)):
        with pytest.raises((AssertionError, ValueError)):
            pin()
