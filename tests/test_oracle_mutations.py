"""The oracle's pins catch plausible mistakes.

Each case copies the oracle, the input generator and the tests into a
temporary directory, plants one mistake in the copy of ``oracle/oracle.c``
(CPU only; the repository's oracle is never touched), rebuilds it and runs
``tests/test_oracle.py`` there, which must fail.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, text in oracle.c, replacement): a dropped or flipped comparison, a wrong
# operand, an off-by-one, a missing reset, each a mistake a reader could miss.
MUTATIONS = [
    ("mass_prefix_ge_to_gt", "if (run >= thr) break;", "if (run > thr) break;"),
    ("magnitude_sort_ascending", "if (p->a > q->a) return -1;", "if (p->a > q->a) return 1;"),
    ("magnitude_tie_higher_id", "return (p->id > q->id) - (p->id < q->id);",
     "return (p->id < q->id) - (p->id > q->id);"),
    ("alpha_complement", "double thr = alpha * mass;", "double thr = (1.0 - alpha) * mass;"),
    ("window_index", "out_ptr[(int64_t)idx[e] * sigma + i / window + 1]++;",
     "out_ptr[(int64_t)idx[e] * sigma + i % sigma + 1]++;"),
    ("heap_tie_higher_id", "return sa > sb || (sa == sb && ia < ib);",
     "return sa > sb || (sa == sb && ia > ib);"),
    ("rerank_with_pruned_query",
     "double d = dot_rows(didx + dptr[i], dval + dptr[i], dptr[i + 1] - dptr[i], qi, qv, n);",
     "double d = dot_rows(didx + dptr[i], dval + dptr[i], dptr[i + 1] - dptr[i], pi, pv, np);"),
    ("coarse_with_full_query",
     "precise_search_one(nd, window, sigma, iptr, idoc, ival, pi, pv, np, gamma, A, &h);",
     "precise_search_one(nd, window, sigma, iptr, idoc, ival, qi, qv, n, gamma, A, &h);"),
    ("gradient_operand", "if (gx) gx[e] += g * (double)qval[a];",
     "if (gx) gx[e] += g * (double)dval[e];"),
    ("dot_drops_last_term", "while (a < na && b < nb) {", "while (a + 1 < na && b < nb) {"),
    ("last_window_full_length",
     "int64_t wlen = nd - w * window < window ? nd - w * window : window;",
     "int64_t wlen = window;"),
    ("distance_array_not_reset", "            A[m] = 0.0;\n        }", "        }"),
    ("top_k_tie_dropped",
     "if (r->len == r->cap && !ranks_before(s, id, r->s[r->len - 1], r->id[r->len - 1])) return;",
     "if (r->len == r->cap && s <= r->s[r->len - 1] && id < 0) return;"),
    ("vnp_keeps_one_fewer", "for (int64_t t = 0; t < n && t < vn; ++t) keep[tmp[t].pos] = 1;",
     "for (int64_t t = 0; t + 1 < n && t < vn; ++t) keep[tmp[t].pos] = 1;"),
    ("lp_tie_higher_doc", "return (p->doc > q->doc) - (p->doc < q->doc);",
     "return (p->doc < q->doc) - (p->doc > q->doc);"),
]


def _run_pins(tmp_path, text=None, repl=None):
    for d in ("oracle", "synth", "tests"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d,
                        ignore=shutil.ignore_patterns("liboracle.so", "__pycache__", "*.tmp"))
    if text is not None:
        src = tmp_path / "oracle" / "oracle.c"
        code = src.read_text()
        assert code.count(text) >= 1, "the text to replace is not in oracle.c"
        src.write_text(code.replace(text, repl, 1))
    return subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle.py", "-x", "-q",
                           "-p", "no:cacheprovider"], cwd=tmp_path, capture_output=True,
                          text=True, timeout=600)


@pytest.mark.slow
def test_unchanged_copy_passes(tmp_path):
    """Control: the copied oracle, unchanged, passes its pins in the temporary directory."""
    r = _run_pins(tmp_path)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]


@pytest.mark.slow
@pytest.mark.parametrize("name,text,repl", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, text, repl):
    r = _run_pins(tmp_path, text, repl)
    assert r.returncode != 0, f"{name}: the planted mistake passed every pin\n{r.stdout[-2000:]}"
