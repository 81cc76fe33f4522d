"""Plant plausible mistakes in a copy of the oracle and check that the pins
catch every one of them (CPU only).  Each mutant is the oracle source with
one textual change; at least one fast pin must fail on it."""
import os
import shutil

import pytest

import oracle_pins as P
from oracle.oracle import build_oracle

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "sx_oracle.c")

MUTANTS = {
    "recombination_sign": ("+ hb * (x * x);", "- hb * (x * x);"),
    "ionisation_uses_transmission": ("- ha * ion + hb", "- ha * (1.0 - ion) + hb"),
    "rate_missing_dt": ("double a = n_in / (dt * nHV);", "double a = n_in / nHV;"),
    "substep_length": ("double h = dt / (double)n_sub;", "double h = dt;"),
    "transmission_ignores_ionisation": ("tr_sum += exp(-y * tau);", "tr_sum += exp(-tau);"),
    "perpendicular_admitted": ("if (!(c > g->cos_min)) continue;", "if (!(c >= g->cos_min)) continue;"),
    "tie_to_higher_id": ("(c == cb && g->nbr[b + s] < g->nbr[b + best])",
                         "(c == cb && g->nbr[b + s] > g->nbr[b + best])"),
    "edge_bin_tie_to_higher": ("if (c > cb) { cb = c; best = k; }", "if (c >= cb) { cb = c; best = k; }"),
    "cosine_drops_z": ("return (a + b) + c;", "return (a + b);"),
    "only_two_per_bin": ("for (int r = 0; r < g->mpb; r++) {", "for (int r = 0; r < g->mpb - 1; r++) {"),
    "transport_wrong_bin": ("g->I[(int64_t)s[t] * K + k] += v;", "g->I[(int64_t)s[t] * K + (k + 1) % K] += v;"),
    "transport_transposed_bins": ("\n            double v = g->O[i * K + k];",
                                  "\n            double v = g->O[i * K + (K - 1 - k)];"),
    "no_split_over_neighbours": ("{\n                g->O[j * K + k] = out / (double)mm;",
                                 "{\n                g->O[j * K + k] = out;"),
    "source_not_split": ("double share = E / (double)deg;", "double share = E;"),
    "path_length_sum_not_mean": ("kappa * (sum / (double)deg)", "kappa * sum"),
    "optical_depth_without_sigma": ("g->tau[i] = (g->nH[i] * sigma) * g->dL[i];",
                                    "g->tau[i] = g->nH[i] * g->dL[i];"),
    "escape_lost": ("g->escaped += out;\n                g->O[j * K + k] = 0.0;",
                    "g->escaped += 0.0 * out;\n                g->O[j * K + k] = 0.0;"),
    "ballistic_not_reversed": ("double u[3] = {-g->edir[3 * e + 0], -g->edir[3 * e + 1],",
                               "double u[3] = {g->edir[3 * e + 0], g->edir[3 * e + 1],"),
    "mode_ignores_neutral_fraction": ("(g->y[j] * g->tau[j] >= g->tau_switch)",
                                      "(g->tau[j] >= g->tau_switch)"),
    "mode_from_previous_layout": ("    if (g->mode[j] == 0)\n        g->I[",
                                  "    if (g->layout[j] == 0)\n        g->I["),
    "ballistic_conversion_first_bin": ("deliver(g, e, g->ebin[e], v);", "deliver(g, e, 0, v);"),
    "ballistic_not_split": ("if (g->bm[e] > 0) g->Oe[e] = out / (double)g->bm[e];",
                            "if (g->bm[e] > 0) g->Oe[e] = out;"),
    "ballistic_escape_lost": ("g->Oe[e] = out / (double)g->bm[e];\n                else g->escaped += out;",
                              "g->Oe[e] = out / (double)g->bm[e];\n                else g->escaped += 0.0 * out;"),
    "filed_at_sender_slot": ("g->Ie[g->ptr[j] + g->rev[e]] += v;", "g->Ie[e] += v;"),
    "in_flight_skips_edges": ("f += g->Oe[e] * (double)g->bm[e];", "f += 0.0 * g->Oe[e];"),
    "edge_reference_unused": ("if (best >= 0) c = select_slots(g, i, &g->edir[3 * (b + best)], slots);",
                              "if (best >= 0) c = select_slots(g, i, ref, slots);"),
    "edge_reference_admits_backward": ("double cb = g->cos_min;\n                for (int64_t s = 0;",
                                       "double cb = -2.0;\n                for (int64_t s = 0;"),
    "diffuse_not_split": ("double share = Di / (double)deg;", "double share = Di;"),
    "diffuse_chemistry_case_b": ("return g->alpha_A > 0.0 ? g->alpha_A : g->alpha_B;",
                                 "return g->alpha_B;"),
    "diffuse_all_recombinations": ("* ((g->alpha_A - g->alpha_B) / g->alpha_A);", "* 1.0;"),
    "diffuse_not_counted": ("    g->emitted += Dj;\n", "\n"),
    "diffuse_sent_late": ("    diffuse_send(g);\n\n    /* Interaction and chemistry at every vertex",
                          "\n    /* Interaction and chemistry at every vertex"),
    "beam_filed_in_edge_bin": ("g->I[(int64_t)g->nbr[e] * K + kb] += share;",
                               "g->I[(int64_t)g->nbr[e] * K + g->ebin[e]] += share;"),
    "beam_combined_filed_in_edge_bin": ("deliver(g, b + slots[t], kb, share);",
                                        "deliver(g, b + slots[t], g->ebin[b + slots[t]], share);"),
    "rotation_keeps_bin_index": ("to[k] = nearest_bin(g, &b_old[3 * k]);", "to[k] = (int32_t)k;"),
    "rotation_maps_from_given_bins": ("to[k] = nearest_bin(g, &b_old[3 * k]);",
                                      "to[k] = nearest_bin(g, &g->bins0[3 * k]);"),
    "rotation_keeps_last_merged_bin": ("if (to[k] == kn) held += O_old",
                                       "if (to[k] == kn) held = O_old"),
    "rotation_escape_not_tallied": ("g->escaped += held;\n                g->in_flight -= held;",
                                    "g->in_flight -= held;"),
    "multihop_emission_not_split": ("if (H > 1) E = E / (double)H;", "if (H > 1) E = E;"),
    "multihop_no_atom_cap": ("            if (a > cap) {\n                a = cap;",
                             "            if (a > 2.0 * cap + 1e300) {\n                a = cap;"),
    "multihop_chemistry_every_hop": ("            if (hop == H - 1) {\n                double hb",
                                     "            if (hop >= 0) {\n                double hb"),
    "nin_skips_first_bin": ("\n        for (int64_t k = 0; k < K; k++) nin += g->I[j * K + k];",
                            "\n        for (int64_t k = 1; k < K; k++) nin += g->I[j * K + k];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    txt = open(SRC).read()
    assert txt.count(old) == 1, f"mutation site for {name} not unique/found"
    src = tmp_path / "sx_oracle.c"
    src.write_text(txt.replace(old, new))
    shutil.copy(os.path.join(os.path.dirname(SRC), "sx_oracle.h"), tmp_path / "sx_oracle.h")
    lib = build_oracle(force=True, src=str(src), out=str(tmp_path / f"lib_{name}.so"))
    caught = []
    for pin in P.FAST_PINS:
        try:
            pin(lib)
        except Exception as e:  # noqa: BLE001 - any failure counts as caught
            caught.append((pin.__name__, type(e).__name__))
            break
    assert caught, f"no pin caught mutant {name}"
