"""Planted mistakes in copies of the oracle must each fail at least one pin.

Every mutant is a textual edit of ``oracle/bpsf_oracle.c`` compiled into a
temporary directory on the CPU; the real oracle is never modified. A mutant
that survives every pin would mean the pins leave that part of the method
unchecked.
"""
import os
import tempfile

import pytest

from oracle import build as obuild
from oracle.oracle import OracleLib
from tests import pins

# (name, text in the oracle, replacement)
MUTANTS = [
    ("v2c_drops_channel_llr", "                real acc = L[v];\n                for (int b",
     "                real acc = 0;\n                for (int b"),
    ("v2c_includes_own_edge", "if (e2 != e) acc = acc + w->c2v[e2];", "acc = acc + w->c2v[e2];"),
    ("c2v_ignores_syndrome", "    int arg = -1;\n    int par = s[c] & 1;",
     "    int arg = -1;\n    int par = 0;"),
    ("c2v_min_includes_own_edge", "real mag = (e == arg) ? min2 : min1;", "real mag = min1;"),
    ("c2v_no_second_min_update", "else if (a < min2) { min2 = a; }", "else { }"),
    ("c2v_no_normalization", "real val = alpha * mag;", "real val = mag;"),
    ("c2v_sign_includes_own_edge", "int neg = par ^ (w->v2c[e] < 0);", "int neg = par;"),
    ("adaptive_alpha_off_by_one", "1.0 - ldexp(1.0, -iter)", "1.0 - ldexp(1.0, -iter - 1)"),
    ("marginal_drops_channel_llr",
     "            real acc = L[v];\n            for (int a = g->var_ptr[v]; a < g->var_ptr[v + 1]; a++) acc",
     "            real acc = 0;\n            for (int a = g->var_ptr[v]; a < g->var_ptr[v + 1]; a++) acc"),
    ("hard_decision_tie_to_zero", "w->hard[v] = (acc > 0) ? 0 : 1;", "w->hard[v] = (acc >= 0) ? 0 : 1;"),
    ("oscillation_counts_ones", "w->flips[v] += (w->hard[v] ^ w->prev[v]);", "w->flips[v] += w->hard[v];"),
    ("oscillation_never_updates_prev", "            w->prev[v] = w->hard[v];\n", "\n"),
    ("stop_test_ignores_syndrome",
     "            int par = s[c] & 1;\n            for (int e = g->row_ptr[c]; e < g->row_ptr[c + 1]; e++) par ^= w->hard",
     "            int par = 0;\n            for (int e = g->row_ptr[c]; e < g->row_ptr[c + 1]; e++) par ^= w->hard"),
    ("top_k_ascending", "w->flips[v] > w->flips[bi]", "w->flips[v] < w->flips[bi]"),
    ("top_k_ties_to_high_index", "w->flips[v] > w->flips[bi]", "w->flips[v] >= w->flips[bi]"),
    ("trial_syndrome_not_flipped", "par ^= t[g->col_idx[e]];", "(void)t;"),
    ("trial_messages_not_reset", "for (int e = 0; e < E; e++) w->c2v[e] = (real)0;",
     "if (track) for (int e = 0; e < E; e++) w->c2v[e] = (real)0;"),
    ("trial_output_not_undone", "for (int v = 0; v < N; v++) w->hard[v] ^= t[v];", "(void)t;"),
    ("selection_keeps_heaviest", "wt < best_w", "wt > best_w"),
    ("layered_posterior_not_written", "w->lout[g->col_idx[e]] = w->v2c[e] + w->c2v[e];", "(void)0;"),
    ("layered_no_subtraction", "w->v2c[e] = w->lout[g->col_idx[e]] - w->c2v[e];",
     "w->v2c[e] = w->lout[g->col_idx[e]];"),
    ("layered_reverse_order", "const int c = g->order[i];", "const int c = g->order[g->M - 1 - i];"),
    ("layers_ignore_shared_bits", "if (c2 < c) used[layer[c2]] = 1;", "(void)c2;"),
    ("trial_masks_skip_last", "for (int64_t i = 0; i < n; i++) masks[i] = (uint64_t)i;",
     "for (int64_t i = 0; i < n; i++) masks[i] = (uint64_t)(i ? i - 1 : 0);"),
    ("wide_mask_bits_truncated", "if ((mask >> j) & 1ull) t[phi[j]] = 1;",
     "if (((uint32_t)mask >> (j & 31)) & 1u) t[phi[j]] = 1;"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new):
    src = open(obuild.SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mutant.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new, 1))
        libs = obuild.build(src=path, out_dir=d, variants=("f64",))
        O = OracleLib(paths=libs)
        caught = []
        for pin in pins.PINS:
            try:
                pin(O)
            except (AssertionError, ValueError, IndexError) as exc:   # a failing pin
                caught.append((pin.__name__, type(exc).__name__))
                break
        assert caught, f"mutant {name} passed every pin"
