"""Planted mistakes: each plausible slip in the oracle, compiled into a copy of
it on the CPU, must be rejected by at least one of the law pins. This shows the
pins have the power to catch what they are meant to catch."""
import os
import subprocess

import pytest

from oracle import build as oracle_build
from oracle import oracle as O

from . import laws

SRC = open(oracle_build.SRC).read()

MUTATIONS = {
    # infection no longer proportional to phi
    "phi_ignored": ([("if (p->uses_phi[k]) v = v * phi;", "if (p->uses_phi[k]) v = v * 1.0;")],
                    laws.check_two_node),
    # the literal Algorithm 1 loop: a draw past the window end is still applied
    "overshoot_applied": ([("if (!(s + tau < 1.0)) break;", "if (!(s < 1.0)) break;")],
                          laws.check_sis_decay),
    # waiting time uniform instead of exponential
    "missing_log": ([("oracle_neglog(oracle_u53(o[0], o[1]))", "(1.0 - oracle_u53(o[0], o[1]))")],
                    laws.check_sis_decay),
    # transition column taken in reverse order
    "wrong_column": ([("x[c] += p->S[(size_t)c * p->Nt + j];", "x[c] += p->S[(size_t)c * p->Nt + (p->Nt - 1 - j)];")],
                     laws.check_flip_state),
    # rate constant of the other transition
    "wrong_rate": ([("double v = p->coef[(size_t)r * p->Nt + k];",
                     "double v = p->coef[(size_t)r * p->Nt + (p->Nt - 1 - k)];")],
                   laws.check_sis_decay),
    # season boundary off by one day
    "season_boundary": ([("if (doy <= 91) return 0;", "if (doy < 91) return 0;")],
                        laws.check_phi_closed_form),
    # sign of the decay term
    "decay_sign": ([("double a = 1.0 - p->beta", "double a = 1.0 + p->beta")],
                   laws.check_phi_closed_form),
    # sampling with replacement
    "with_replacement": ([("rem[chosen] -= 1;", "(void)0;")], laws.check_hypergeometric),
    # compartments walked without skipping unselected ones
    "mask_ignored": ([("if (!(mask & (1u << c))) continue;\n            if (pick",
                       "if (0) continue;\n            if (pick")], laws.check_multivariate_walk),
    # moved animals dropped instead of added at the destination
    "lost_move": ([("xt[to] += m[c];", "(void)to;")], laws.check_conservation),
    # an external transfer lands its animals unshifted (the shift applied to internal ones only)
    "external_shift_ignored": ([("int32_t to = c + (sh >= 0 ? p->Nsh",
                                 "int32_t to = c + (sh >= 0 && kind == EV_INTERNAL ? p->Nsh")],
                               laws.check_two_node_shifted),
    # the same slip seen by the class totals of a farm network with shifted moves
    "external_shift_ignored_totals": ([("int32_t to = c + (sh >= 0 ? p->Nsh",
                                        "int32_t to = c + (sh >= 0 && kind == EV_INTERNAL ? p->Nsh")],
                                      laws.check_conservation),
    # the day's longest chain taken from one node instead of the maximum over nodes
    "max_transitions_one_node": ([("if (ntr[i] > most) most = ntr[i];", "if (i == 0) most = ntr[i];")],
                                 laws.check_max_transitions),
    # prevalence counting nodes by their size instead of their infected
    "prevalence_counts_size": ([("if (p->phi_I_mask & (1u << c)) I += ur[(size_t)i * Nc + c];",
                                 "if (p->phi_N_mask & (1u << c)) I += ur[(size_t)i * Nc + c];")],
                               laws.check_prevalence_law),
    # phi fed by the state before the events (the other reading of eq:numstep5)
    "phi_before_events": ([("if (!p->phi_pre_events) {", "if (0) {"),
                           ("ntr[i] = ssa_node(p, r, i, d, ur + (size_t)i * Nc, vr[i]);",
                            "{ ntr[i] = ssa_node(p, r, i, d, ur + (size_t)i * Nc, vr[i]);"
                            " vr[i] = phi_update(p, r, d, ur + (size_t)i * Nc, vr[i]); }")],
                          laws.check_two_node),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    edits, check = MUTATIONS[name]
    src = SRC
    for old, new in edits:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    c = tmp_path / "mutant.c"
    c.write_text(src)
    so = str(tmp_path / f"lib_{name}.so")
    subprocess.run(["gcc", *oracle_build.CFLAGS, str(c), "-o", so, "-lm"], check=True,
                   capture_output=True)
    try:
        ok, stat = check(lib_path=so)
    except O.OracleError as e:        # the mutant reached an impossible state: caught as well
        ok, stat = False, str(e)
    assert not ok, (name, stat)


def test_unmutated_copy_passes(tmp_path):
    c = tmp_path / "same.c"
    c.write_text(SRC)
    so = str(tmp_path / "lib_same.so")
    subprocess.run(["gcc", *oracle_build.CFLAGS, str(c), "-o", so, "-lm"], check=True)
    for check in {m[1] for m in MUTATIONS.values()}:
        ok, stat = check(lib_path=so)
        assert ok, (check.__name__, stat)
