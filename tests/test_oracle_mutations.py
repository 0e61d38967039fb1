"""Planted mistakes in the oracle must fail its pins.

Each case copies the oracle's C source, turns one line into a plausible
mistake, builds it on the CPU and runs the pin tests that should notice
against that build (a subprocess with SMCX_ORACLE_LIB naming it).  The same
pins pass on the unmodified oracle (the other test files), so a failing run
here means the pins see the mistake.
"""
import os
import subprocess
import sys

import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))

MUTANTS = [
    ("a-b bond counted", "if (ja != b) na[s][occ[ja]] += 1;", "na[s][occ[ja]] += 1;",
     ["test_oracle_mc.py::test_delta_e_matches_recomputation"]),
    ("dE sign", "double dv = V[((size_t)s * K + q) * K + t] - V[((size_t)s * K + p) * K + t];",
     "double dv = V[((size_t)s * K + p) * K + t] - V[((size_t)s * K + q) * K + t];",
     ["test_oracle_mc.py::test_delta_e_matches_recomputation"]),
    ("Boltzmann factor sign", "double P = exp(-x);", "double P = exp(x);",
     ["test_oracle_mc.py::test_exact_canonical_mean_energy"]),
    ("uniform from the wrong bits", "<< 21) | (uint64_t)(w[2] >> 11)", "<< 20) | (uint64_t)(w[2] >> 12)",
     ["test_oracle_mc.py::test_exact_canonical_mean_energy", "test_oracle_mc.py::test_energy_histogram_matches_boltzmann"]),
    ("energy without the 1/2", "return 0.5 * acc;", "return acc;",
     ["test_oracle_counts.py::test_energy_vs_brute_force"]),
    ("SRO without Z_s", "(((double)Z[s] * (double)Nk[k]) * (double)Nk[l])", "((double)Nk[k] * (double)Nk[l])",
     ["test_oracle_counts.py::test_sro_of_b2_order", "test_oracle_mc.py::test_sro_vanishes_at_infinite_temperature"]),
    ("Philox multiplier", "M0 = 0xD2511F53u", "M0 = 0xD2511F57u",
     ["test_oracle_rng.py::test_known_answer_vectors"]),
    ("a shell skipped", "for (int target = 1; nr < S && target < 64; ++target)",
     "for (int target = 1; nr < S && target < 64; target += 2)",
     ["test_oracle_geometry.py::test_textbook_coordination"]),
    ("link-cell rule one short", "while (!(2 * ell > 1 + reach)) ++ell;", "while (!(2 * ell > reach)) ++ell;",
     ["test_oracle_geometry.py::test_link_cell_rule_reproduces_paper", "test_oracle_geometry.py::test_link_cell_rule_is_tight"]),
    ("exchange energy difference reversed", "double x = (beta_slot[i] - beta_slot[i + 1]) * (E[a] - E[b]);",
     "double x = (beta_slot[i] - beta_slot[i + 1]) * (E[b] - E[a]);",
     ["test_oracle_tempering.py::test_exchange_acceptance_frequency",
      "test_oracle_tempering.py::test_tempering_slots_sample_their_temperature"]),
    ("exchange factor inverted", "double P = exp(x);", "double P = exp(-x);",
     ["test_oracle_tempering.py::test_exchange_acceptance_frequency"]),
    ("exchange ignores the round parity", "for (int i = (int)(round & 1u); i + 1 < R; i += 2)",
     "for (int i = 0; i + 1 < R; i += 2)",
     ["test_oracle_tempering.py::test_exchange_special_cases"]),
    ("heat capacity without beta^2", "return beta * beta * v / (double)N;", "return v / (double)N;",
     ["test_oracle_anneal.py::test_heat_capacity_closed_forms",
      "test_oracle_anneal.py::test_heat_capacity_exact_sixteen_site_cell"]),
    ("heat capacity from the sample variance", "v = v / (double)n;", "v = v / (double)(n - 1);",
     ["test_oracle_anneal.py::test_heat_capacity_closed_forms"]),
    ("local energy without the 1/2", "return acc * 0.5;", "return acc;",
     ["test_oracle_clusters.py::test_local_energy_brute_force"]),
    ("cluster labelled by the site that reached it", "label[j] = (int32_t)i;", "label[j] = (int32_t)a;",
     ["test_oracle_clusters.py::test_clusters_against_connected_components"]),
    ("strict cluster threshold", "if (e[j] <= threshold && label[j] < 0) {", "if (e[j] < threshold && label[j] < 0) {",
     ["test_oracle_clusters.py::test_clusters_against_connected_components"]),
    ("qSRO quadratic term not squared", "acc = acc + W[(size_t)s * K + p] * (f * f);", "acc = acc + W[(size_t)s * K + p] * f;",
     ["test_oracle_qsro.py::test_closed_form_one_impurity"]),
    ("qSRO affected set without the partner's neighbours",
     "            for (int a = 0; a < 3; ++a) cand[n][a] = ab[a] + sy->d[s][j][a];\n            ++n;\n", "",
     ["test_oracle_qsro.py::test_delta_e_is_the_total_energy_difference"]),
    ("qSRO affected set with duplicates", "dup = v[j][0] == cand[i][0] && v[j][1] == cand[i][1] && v[j][2] == cand[i][2];",
     "dup = 0;", ["test_oracle_qsro.py::test_delta_e_is_the_total_energy_difference"]),
    ("replay keyed on the site only",
     "if (rp->replay[i].replica == r && rp->replay[i].sweep == t && rp->replay[i].site == a) {",
     "if (rp->replay[i].site == a) {",
     ["test_oracle_ties.py::test_replay_under_other_keys_is_ignored",
      "test_oracle_ties.py::test_replay_keyed_by_replica_and_sweep"]),
    ("replay keyed without the sweep",
     "if (rp->replay[i].replica == r && rp->replay[i].sweep == t && rp->replay[i].site == a) {",
     "if (rp->replay[i].replica == r && rp->replay[i].site == a) {",
     ["test_oracle_ties.py::test_replay_keyed_by_replica_and_sweep"]),
    ("replayed decision ignored", "if (rp && replay_lookup(rp, (int32_t)r, t, a, &dec)) accept = dec;",
     "if (rp && replay_lookup(rp, (int32_t)r, t, a, &dec)) accept = accept;",
     ["test_oracle_ties.py::test_replay_flips_exactly_the_tied_swap"]),
    ("trial near-tie never detected", "accept = u < P;\n            if (fabs(u - P) < 1e-12) {\n                flags |= TR_TIE;",
     "accept = u < P;\n            if (fabs(u - P) < 0.0) {\n                flags |= TR_TIE;",
     ["test_oracle_ties.py::test_forced_trial_tie_is_logged"]),
    ("exchange replay keyed on the replica", "if (replay_lookup(&rp, -1, round, i, &dec)) accept = dec;",
     "if (replay_lookup(&rp, -1, round, a, &dec)) accept = dec;",
     ["test_oracle_ties.py::test_exchange_replay_flips_the_tied_pair"]),
]


@pytest.mark.parametrize("name,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, old, new, pins, tmp_path):
    src = open(O.SRC).read()
    assert src.count(old) == 1, f"mutation site not found: {old}"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = O.compile_source(str(mut), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, SMCX_ORACLE_LIB=lib)
    args = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
    args += [os.path.join(HERE, p) for p in pins]
    r = subprocess.run(args, cwd=os.path.dirname(HERE), env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins {pins} did not notice '{name}':\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout or "error" in r.stdout.lower(), r.stdout[-2000:]


def test_unmodified_source_passes_the_same_pins(tmp_path):
    """Control: the same procedure on the unmodified source passes, so the
    failures above come from the planted mistakes."""
    lib = O.compile_source(O.SRC, str(tmp_path / "libcontrol.so"))
    env = dict(os.environ, SMCX_ORACLE_LIB=lib)
    pins = sorted({p for m in MUTANTS for p in m[3]})
    args = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
    args += [os.path.join(HERE, p) for p in pins]
    r = subprocess.run(args, cwd=os.path.dirname(HERE), env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:]
